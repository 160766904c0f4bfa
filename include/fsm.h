/*
 * fsm.h -- C ABI of libfsm, the MI355X (gfx950) library for milled 3D surface topography by
 * the forward solution method (FSM).
 *
 * Problem statement (Sec. 2 and 3 of the paper): tool geometry + cutting parameters +
 * workpiece grid -> per-cell minimum height map (Z-map) + areal / profile roughness.
 * The library discretises the cutting edges (Eq. (1), (6)), moves every edge point through the
 * cutting-edge -> tool -> spindle -> workpiece transformations (Eq. (2)-(5)) at every time
 * step, bins it into the sampling boundary of a grid node (Eq. (7)), keeps the lowest height
 * per node (Sec. 2.3), and reduces the Z-map to the ISO 25178-2 amplitude parameters and the
 * profile Ra along the feed and pick-feed directions (Sec. 4.1, 4.2).
 *
 * Conventions
 *   - Lengths in mm, angles in rad.  Feed runs along +X, parallel passes step along +Y, Z is
 *     the workpiece normal.  The spindle turns counter-clockwise seen from +Z (the sign of
 *     omega*t in Eq. (3)); tooth K trails tooth 0 by theta_K.
 *   - Every call returns FSM_OK (0) or a negative FSM_E* code.  No exception, abort or
 *     exit crosses the ABI.  Points that fall outside the grid are not errors; they are
 *     dropped (not clamped) and counted.
 *   - Parameter structs are plain host memory, borrowed for the duration of the call.
 *   - Device pointers are caller-owned device memory (for instance a torch tensor's
 *     data_ptr()); the library never frees them.
 *   - A context is used by one host thread at a time.  Calls on one context are
 *     stream-ordered on the stream passed in (a hipStream_t; NULL = the null stream).
 *
 * Z-map layout: row-major [ny][nx]; cell (i, j) is the sampling boundary of node
 * (x0 + i*dd, y0 + j*dd), half-open [x_i - dd/2, x_i + dd/2) x [y_j - dd/2, y_j + dd/2).
 * Element type double (FSM_F64) or float (FSM_F32).  Cells no point reached hold +inf.
 */
#ifndef FSM_H
#define FSM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FSM_ABI_VERSION 2
#define FSM_MAX_TEETH 8
#define FSM_MAX_EDGE 4096

/* status codes */
#define FSM_OK 0
#define FSM_EINVAL (-1)   /* invalid argument or parameter */
#define FSM_ENOMEM (-2)   /* host or device allocation failed */
#define FSM_EDEVICE (-3)  /* HIP runtime error (message kept in the context) */
#define FSM_EAGAIN (-4)   /* batch admission refused: memory budget or slots exhausted */
#define FSM_ENOTSUP (-5)  /* reserved for valid requests the library cannot serve; ABI
                             version 1 reports its limits (edge points, window width) as
                             FSM_EINVAL */

/* precision of the Z-map and of the edge-point arithmetic */
#define FSM_F64 0  /* every operation in double precision; binning bit-exact with the plain
                      double-precision definition */
#define FSM_F32 1  /* rotation and tilt of tool-local coordinates in single precision;
                      tool-centre path, binning and roughness moments in double precision;
                      Z-map stored as float */

/* tool kinds */
#define FSM_TOOL_ROUND 0  /* round cutting edge: circular insert / corner-radius profile of
                             radius R_edge whose lowest point lies at radius D/2 (Eq. (1)) */
#define FSM_TOOL_BALL 1   /* ball end: sphere of radius D/2 centred on the tool axis */

/* result flags */
#define FSM_FLAG_SQ_ZERO 1u       /* Sq == 0: Ssk and Sku are NaN */
#define FSM_FLAG_NO_HIT 2u        /* no cell was reached: every parameter is NaN */
#define FSM_FLAG_LOW_COVERAGE 4u  /* fewer than 99 % of the cells were reached */

typedef struct fsm_tool {
    int32_t kind;            /* FSM_TOOL_ROUND or FSM_TOOL_BALL */
    int32_t n_teeth;         /* z_n, 1..FSM_MAX_TEETH */
    int32_t n_edge;          /* N, points per cutting edge, 1..FSM_MAX_EDGE (Eq. (6)) */
    int32_t uniform_pitch;   /* nonzero: tooth K at 2*pi*K/z_n (Eq. (3)); zero: theta[K] */
    double D;                /* cutting diameter through the edges' lowest points (Eq. (2)) */
    double R_edge;           /* edge profile radius R (round edge; ignored for a ball) */
    double helix;            /* helix angle beta: a point at profile height z trails the
                                lowest point by z*tan(beta)/(D/2) about the tool axis */
    double rake_radial;      /* gamma_f of Eq. (2) */
    double rake_axial;       /* gamma_p of Eq. (2) */
    double theta[FSM_MAX_TEETH];   /* angular position of each tooth (variable pitch) */
    double runout_ecc;       /* eccentric runout: offset e of the cutter body from the
                                spindle axis */
    double runout_phase;     /* its direction lambda in the cutter body */
    double eps_r[FSM_MAX_TEETH];   /* radial offset of each insert, added to D/2 in Eq. (2)
                                      (the paper's (K-1)*eps_r, given per tooth) */
    double eps_a[FSM_MAX_TEETH];   /* axial offset of each insert in Eq. (2) (the paper's
                                      (K-1)*eps_a, given per tooth) */
    double tilt_lead;        /* tool tilt about the workpiece Y axis; positive lowers the
                                leading (+X) side */
    double tilt_side;        /* tool tilt about the workpiece X axis; positive raises +Y */
} fsm_tool;

typedef struct fsm_cut {
    double f_z;              /* feed per tooth, >= 0 */
    double a_p;              /* axial depth of cut, > 0 (sets the engaged edge length; a round
                                edge's chord is capped at R_edge, so a_p >= R_edge engages
                                the whole half profile) */
    double a_e;              /* stepover between parallel passes; <= 0: one pass */
    double phi0;             /* initial phase angle phi of Eq. (3) */
    int32_t steps_per_rev;   /* S, time steps per spindle revolution, >= 1 (FSM_TIME_PER_REV) */
    int32_t n_passes;        /* parallel passes; 0: enough to cover the grid */
    int64_t n_steps;         /* time steps per pass; 0: whole revolutions covering the grid */
    double x_start;          /* tool-centre x at step 0; NaN: a full reach before the grid */
    double y_first;          /* tool-centre y of pass 0; NaN: a full reach below the grid
                                (or the grid centre line for a single pass) */
    int32_t time_mode;       /* FSM_TIME_PER_REV: steps_per_rev steps per revolution;
                                FSM_TIME_FIXED_DT: the paper's fixed time step dt at cutting
                                speed v_c (Sec. 4.3), spindle speed 1000 v_c / (pi D) */
    int32_t reserved;
    double v_c;              /* cutting speed, m/min (FSM_TIME_FIXED_DT) */
    double dt;               /* time step, s (FSM_TIME_FIXED_DT) */
    double x_end;            /* end of the travel the automatic step count covers; NaN: a full
                                reach past the grid */
} fsm_cut;

#define FSM_TIME_PER_REV 0
#define FSM_TIME_FIXED_DT 1

typedef struct fsm_grid {
    double x0, y0;           /* position of node (0, 0) */
    double dd;               /* sampling interval (Sec. 2.2), > 0 */
    int64_t nx, ny;          /* nodes along X (feed) and Y (pick feed), >= 1 */
} fsm_grid;

typedef struct fsm_plan_info {
    double r_reach;          /* bound on any edge point's horizontal distance from the axis */
    double x_start;          /* resolved tool-centre start */
    double y_first;          /* resolved first pass */
    int64_t n_passes;
    int64_t n_steps;         /* per pass */
    int64_t n_evals;         /* passes * steps * teeth * edge points */
    int64_t n_cells;         /* nx * ny */
    int64_t zmap_bytes;      /* bytes of the caller's Z-map at this precision */
    int64_t workspace_bytes; /* device bytes the library needs for this simulation */
    int32_t zmap_path;       /* FSM_PATH_* a fresh context's launch parameters take */
    int32_t n_slices;        /* slices of its binned Z-map with those parameters */
} fsm_plan_info;

typedef struct fsm_rough {
    double Sa, Sq, Sp, Sv, Sz, Ssk, Sku;   /* areal parameters over the reached cells */
    double Ra_feed;          /* profile Ra along row ny/2 (feed direction) */
    double Ra_pick;          /* profile Ra along column nx/2 (pick-feed direction) */
    double mean;             /* mean height of the reached cells (reference plane) */
    double pos_err;          /* FSM_F32: bound on the single-precision error of every evaluated
                                position along x and y (mm), 2^-20 times the largest distance of
                                an edge point from the tool origin (at most 13 roundings per
                                coordinate, each below 2^-24 times that distance); heights err
                                by no more.  0 in FSM_F64 */
    int64_t n_hit;           /* reached cells */
    int64_t n_evals;         /* edge-point evaluations */
    int64_t n_binned;        /* evaluations that fell inside the grid */
    int64_t n_feed, n_pick;  /* reached cells on the two profiles */
    int64_t n_near;          /* FSM_F32: in-grid evaluations that lay within pos_err of a cell
                                boundary: the only binning decisions that may differ from
                                double precision (a cell's height differs from the double-
                                precision map by more than pos_err only where one of them
                                decided its minimum).  0 in FSM_F64 */
    uint32_t flags;          /* FSM_FLAG_* */
    uint32_t reserved;
} fsm_rough;

/* Per-kernel device times of the last fsm_simulate / fsm_simulate_batch / fsm_roughness call
 * on a context with profiling on, measured with HIP events on the stream the library launches
 * on (milliseconds).  Per-stage times need eager launches: with FSM_OPT_GRAPHS on, only
 * total_ms is reported (the other fields are zero). */
typedef struct fsm_timings {
    float upload_ms;         /* plan tables host -> device */
    float fill_ms;           /* Z-map initialisation */
    float scatter_ms;        /* kinematics + binning + per-cell minimum (all slices) */
    float rough_ms;          /* roughness passes (or the decode pass) */
    float total_ms;          /* first event to last event */
    /* stages of the binned Z-map, summed over its slices (0 for the scatter strategy) */
    float count_ms;          /* kinematics + binning, points counted per tile */
    float index_ms;          /* scans of the counts into bucket offsets */
    float write_ms;          /* kinematics + binning again, points written to their buckets */
    float reduce_ms;         /* per-tile minimum in LDS (+ first roughness pass) */
    int32_t n_slices;        /* slices of the binned Z-map */
    int32_t valid;           /* 1 once a profiled call has completed */
    int32_t zmap_path;       /* FSM_PATH_* the Z-map took */
    int32_t reserved;
} fsm_timings;

/* Z-map paths (fsm_timings.zmap_path, fsm_plan_info.zmap_path).  The binned strategy counts
 * the points of a row of binning items per tile in LDS when a simulation's tiles fit one
 * histogram (histogram mode), per super-tile of up to 64 tiles with a split pass into the
 * tiles otherwise (super mode), and with global atomics per tile when even its super-tiles do
 * not fit or the row matrix would exceed FSM_OPT_HIST_BYTES (run mode).  Every path gives the
 * same Z-map; FSM_PATH_SCATTER is the scatter strategy. */
#define FSM_PATH_SCATTER 0
#define FSM_PATH_RUN 1
#define FSM_PATH_HIST 2
#define FSM_PATH_SUPER 3

typedef struct fsm_ctx fsm_ctx;

/* ABI version (FSM_ABI_VERSION). */
int fsm_version(void);

/* Static description of a status code; never NULL. */
const char *fsm_strerror(int code);

/* Host only.  Validates the parameters and resolves the automatic path (Sec. 2.2: travel,
 * passes and steps), reporting sizes and the memory footprint.  FSM_EINVAL on bad input. */
int fsm_plan(const fsm_tool *tool, const fsm_cut *cut, const fsm_grid *grid, int precision,
             fsm_plan_info *out);

/* Host only.  The discretised edge of every tooth in the tool frame (Eq. (1), (6), (2) plus
 * helix lag and eccentric runout): out is caller-owned host memory of n_teeth*n_edge*3
 * doubles, [tooth][point][x,y,z]. */
int fsm_edge_points(const fsm_tool *tool, const fsm_cut *cut, double *out);

/* Host only.  Coverage-complete planning: the smallest edge-point count and time step at
 * which consecutive samples of the swept edge lie at most `spacing` apart -- neighbouring edge
 * points in space, and each edge point between consecutive time steps (its turn about the axis
 * plus the feed) -- so that with spacing <= half the grid interval no cell the edge sweeps is
 * left without a point (the paper refines the time step for the same reason, Sec. 2.2-2.3).
 * Writes copies of the tool and cut with n_edge raised, and steps_per_rev raised (per-
 * revolution mode) or dt lowered (fixed-step mode); never coarser than the input; n_steps is
 * cleared so the path is planned again.  FSM_EINVAL for bad parameters, a spacing <= 0, or a
 * refinement beyond 4096 edge points or 2^24 steps per revolution. */
int fsm_refine(const fsm_tool *tool, const fsm_cut *cut, const fsm_grid *grid, double spacing,
               fsm_tool *tool_out, fsm_cut *cut_out);

/* Create a context on HIP device `device`.  The context owns the device workspace (edge and
 * angle tables, reduction partials, counters), the slots of asynchronous batches and pinned
 * host staging; they grow on demand and are freed by fsm_ctx_destroy (which first waits for
 * batches still in flight).  FSM_EDEVICE if the device cannot be used. */
int fsm_ctx_create(fsm_ctx **out, int device);
void fsm_ctx_destroy(fsm_ctx *ctx);

/* Copy the last error message of the context (NUL-terminated, truncated to n). */
int fsm_last_error(const fsm_ctx *ctx, char *buf, size_t n);

/* context options (fsm_ctx_set_option) */
#define FSM_OPT_ZMAP_STRATEGY 1   /* how points reach the Z-map:
                                       FSM_ZMAP_BINNED (default): bucket the points by cell
                                       tile (FSM_OPT_TILE_SHAPE), then min-reduce each tile in
                                       LDS and store it once; FSM_ZMAP_SCATTER: one global
                                       atomic min per point */
#define FSM_OPT_BUCKET_BYTES 2    /* device bytes the binned strategy may use for its point
                                       buckets (default 16 GiB); larger simulations run in
                                       slices of the evaluation range */
#define FSM_OPT_GRAPHS 3           /* nonzero: capture the launch sequences of fsm_simulate and
                                       fsm_simulate_batch into HIP graphs (on a stream of the
                                       context, ordered after the caller's) and replay them for
                                       later calls of the same shape */
#define FSM_OPT_TILE_SHAPE 4      /* cell tile of the binned Z-map and of the roughness partials:
                                       16 * log2(width) + log2(height), both 16..256 cells and the
                                       tile's keys within the device's LDS per workgroup (160
                                       KiB on gfx950); 0 (default): 64 x 64 cells in
                                       double precision, 128 x 64 in single */
#define FSM_OPT_TARGET_ROWS 5     /* binning rows (one workgroup each) per launch of the
                                       histogram mode, 256..65536; 0 (default): 4096 */
#define FSM_OPT_AUTOTUNED 6       /* nonzero (default): a call whose workload class fsm_autotune
                                       has measured uses the parameters it kept; zero: the
                                       context's own options */
#define FSM_OPT_ASYNC_SLOTS 7      /* asynchronous batches in flight at once, 1..16 (default 2);
                                       FSM_EAGAIN while any is in flight */
#define FSM_OPT_HBM_BUDGET 8       /* device bytes the workspaces of the asynchronous slots may
                                       hold together; 0 (default): no limit */
#define FSM_OPT_HIST_BYTES 9       /* device bytes the binned strategy's row matrix may take
                                       (histogram and super modes; default 1 GiB); a launch
                                       whose matrix would be larger runs in run mode, and 0
                                       makes every binned launch do so */
#define FSM_ZMAP_BINNED 0
#define FSM_ZMAP_SCATTER 1

/* Set a context option.  FSM_EINVAL for an unknown option or value. */
int fsm_ctx_set_option(fsm_ctx *ctx, int option, int64_t value);

/* Turn per-kernel event timing on (nonzero) or off for later calls on the context.  Costs
 * a few event records per call; off by default. */
int fsm_ctx_set_profiling(fsm_ctx *ctx, int on);

/* Timings of the last profiled call (valid == 0 if there is none). */
int fsm_last_timings(const fsm_ctx *ctx, fsm_timings *out);

/* One simulation: the forward solution of Sec. 2.3 -- every edge point of Eq. (6) at every time
 * step moved into the workpiece frame by Eq. (2)-(5), binned into the sampling boundary of a
 * grid node by Eq. (7) and kept as that node's lowest height -- then the roughness of the map
 * (Sec. 4.1: ISO 25178-2 amplitude parameters, profile Ra).
 * zmap_dev: caller-owned device memory of nx*ny doubles (FSM_F64) or floats
 * (FSM_F32), overwritten with the Z-map.  out: host memory for the roughness, or NULL to
 * compute the Z-map only.  The work is queued on `stream`; the call returns after it has
 * finished.  FSM_EINVAL on bad parameters, FSM_EDEVICE on a HIP error. */
int fsm_simulate(fsm_ctx *ctx, const fsm_tool *tool, const fsm_cut *cut, const fsm_grid *grid,
                 int precision, void *zmap_dev, fsm_rough *out, void *stream);

/* For callers that cannot allocate memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): fsm_simulate without any device or pinned-host
 * allocation.  The scratch it needs (reduction partials, counters, the binned Z-map's row
 * matrix and buckets, the plan image) is a fixed device array of FSM_NOALLOC_SCRATCH_BYTES
 * inside the library, one per GPU, held until the process ends; the binned Z-map runs in as
 * many slices as that size requires (the row matrix gets at most a quarter of it).  The caller
 * passes the Z-map and the result record as for fsm_simulate, and gets the same Z-map and
 * roughness.  The plan is built in ordinary host memory.  FSM_EINVAL, with a message, when
 * the simulation cannot run within the array (its tile partials, row matrix and one slice of
 * buckets exceed it), besides fsm_simulate's errors.  Every call on a GPU uses that GPU's one
 * array: calls that overlap in time on one GPU (from any context or thread) race and must be
 * serialised by the caller. */
#define FSM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int fsm_simulate_noalloc(fsm_ctx *ctx, const fsm_tool *tool, const fsm_cut *cut,
                         const fsm_grid *grid, int precision, void *zmap_dev, fsm_rough *out,
                         void *stream);

/* The trajectory module (Sec. 3.2): for every pass q, time step s and tooth K, the
 * workpiece-frame position of the lowest point (least z) of the tooth's discretised edge,
 * the first such point on a tie.  traj_dev: caller-owned device memory of
 * n_passes * n_steps * n_teeth * 3 doubles (FSM_F64) or floats (FSM_F32), [q][s][K][x, y, z];
 * index_dev (nullable): as many int32 edge-point indices.  Sizes from fsm_plan.  The work is
 * queued on `stream`; the call returns after it has finished. */
int fsm_trajectory(fsm_ctx *ctx, const fsm_tool *tool, const fsm_cut *cut, const fsm_grid *grid,
                   int precision, void *traj_dev, int32_t *index_dev, void *stream);

/* One simulation of a batch.  Every pointer is borrowed for the duration of the call. */
typedef struct fsm_job {
    const fsm_tool *tool;
    const fsm_cut *cut;
    const fsm_grid *grid;
    void *zmap_dev;          /* caller-owned device Z-map of this job (precision of the batch) */
} fsm_job;

/* Many simulations of different shapes in one launch sequence (the dataset generation of
 * Sec. 4.3, which calls the method for many parameter sets): all their work items and
 * tiles are numbered consecutively and every kernel of the pipeline covers the whole batch
 * at once, so small and large simulations share the device (the batched form of the method,
 * used for dataset generation).  out: n host records.  With FSM_OPT_GRAPHS on, the launch
 * sequence is captured into a HIP graph keyed by its shape and replayed when a batch of the
 * same shape comes again.  Returns after the work has finished.  FSM_EINVAL, naming two jobs,
 * when their Z-maps share a byte (checked before anything is queued). */
int fsm_simulate_batch(fsm_ctx *ctx, int n, const fsm_job *jobs, int precision,
                       fsm_rough *out, void *stream);

/* Asynchronous batches.  fsm_batch_submit plans the jobs (on the host, before it returns),
 * takes a free slot of the context (its own stream and workspace), and queues the batch's
 * upload, kernels and result copy on the slot's stream behind the work already queued on
 * `stream`; later work on `stream` is ordered after the batch.  The host returns at once with
 * *batch_id, so the next batch can be planned while this one runs.  The Z-maps stay borrowed
 * until fsm_batch_wait returns; the tool, cut and grid records only for the call.
 * FSM_EAGAIN (nothing queued) when every slot holds a batch not yet waited for, or when the
 * slot's workspace would take the slots' workspaces beyond FSM_OPT_HBM_BUDGET; FSM_EINVAL for
 * bad jobs and overlapping Z-maps as fsm_simulate_batch.  Batches in flight at the same time
 * must not share Z-maps either (not checked). */
int fsm_batch_submit(fsm_ctx *ctx, int n, const fsm_job *jobs, int precision, void *stream,
                     uint64_t *batch_id);

/* *done = 1 if the batch has finished on the device, else 0.  FSM_EINVAL for an unknown (or
 * already waited for) batch. */
int fsm_batch_poll(fsm_ctx *ctx, uint64_t batch_id, int *done);

/* Wait for the batch, write its n result records to out (host memory, nullable) and free its
 * slot; the id is then no longer valid.  FSM_EINVAL for an unknown batch. */
int fsm_batch_wait(fsm_ctx *ctx, uint64_t batch_id, fsm_rough *out);

/* Launch parameters chosen by fsm_autotune. */
typedef struct fsm_tune_result {
    int32_t strategy;        /* FSM_ZMAP_BINNED or FSM_ZMAP_SCATTER */
    int32_t tile_shape;      /* FSM_OPT_TILE_SHAPE encoding */
    int32_t target_rows;     /* FSM_OPT_TARGET_ROWS value */
    int32_t n_tried;         /* candidates timed */
    float best_ms;           /* time of one launch sequence with the kept parameters */
    float default_ms;        /* the same with the default parameters */
} fsm_tune_result;

/* The project's autotuner for the batched launch.  Times candidate launch parameters (Z-map
 * strategy, cell tile shape, histogram rows per launch) on the n jobs run as one batch, by
 * coordinate search from the defaults, each candidate the fastest of at least three timed
 * runs (and of as many as fill 20 ms, at most 64) after one untimed one, and keeps the
 * fastest for the jobs' workload class (precision, number of
 * simulations, and the binary orders of magnitude of their total cells and edge-point
 * evaluations).  Later fsm_simulate / fsm_simulate_batch / fsm_serve_run calls of the same
 * class use them while FSM_OPT_AUTOTUNED is on.  Parameters change only the launch, not the
 * Z-maps; roughness sums may differ in the last bits with the tile shape.  The jobs' Z-maps
 * are overwritten (FSM_EINVAL when two of them overlap, as fsm_simulate_batch).  out: the kept
 * parameters and timings. */
int fsm_autotune(fsm_ctx *ctx, int n, const fsm_job *jobs, int precision, fsm_tune_result *out,
                 void *stream);

/* One entry of a context's tuning table: the workload class (as fsm_autotune forms it) and
 * the launch parameters kept for it. */
typedef struct fsm_tune_entry {
    char key[64];            /* workload class, NUL-terminated */
    int32_t strategy;        /* FSM_ZMAP_BINNED or FSM_ZMAP_SCATTER */
    int32_t tile_shape;      /* FSM_OPT_TILE_SHAPE encoding (0: default) */
    int32_t target_rows;     /* FSM_OPT_TARGET_ROWS value */
    int32_t reserved;
} fsm_tune_entry;

/* Copy the context's tuning table into out[0..cap) (sorted by key); *n receives the number of
 * entries (which may exceed cap).  Lets a caller save what fsm_autotune measured. */
int fsm_tune_get(const fsm_ctx *ctx, fsm_tune_entry *out, int cap, int *n);

/* Add (or replace) n entries of the context's tuning table, e.g. from a saved table of the same
 * device type.  FSM_EINVAL for a bad strategy, tile shape or row count. */
int fsm_tune_set(fsm_ctx *ctx, const fsm_tune_entry *entries, int n);

/* Roughness of an existing Z-map in device memory (+inf = empty cell), same estimator as
 * fsm_simulate: the ISO 25178-2 amplitude parameters of Sec. 4.1 about the mean plane of the
 * reached cells, and the profile Ra of Sec. 4.1 along row ny/2 and column nx/2.  n_evals and
 * n_binned of the result are zero. */
int fsm_roughness(fsm_ctx *ctx, const fsm_grid *grid, int precision, const void *zmap_dev,
                  fsm_rough *out, void *stream);

/* ---- surface texture of a Z-map ---------------------------------------------------------------
 *
 * The paper's measured topographies pass an S-filter (10 um) and an L-filter (0.8 mm) before
 * their roughness is taken (Sec. 4.1.1).  These calls apply the same operators to a predicted
 * Z-map in device memory, so that predictions and measurements are evaluated alike and a
 * dataset of maps (Sec. 4.3) carries measurement-like roughness.  Empty cells (+inf) take no
 * part and stay empty.  zmap_in and zmap_out may be the same map; otherwise an output shares
 * no byte with any map of the call (inputs may share bytes), else FSM_EINVAL before anything
 * is queued.  Each call waits for its work on `stream` before it returns.  Scratch: 16 bytes
 * per cell (filter) from the context's workspace, which grows on demand. */

/* F-operator: subtract the least-squares plane z = plane[0] + plane[1] x + plane[2] y (x, y
 * the cells' node coordinates, mm) fitted over the hit cells.  plane may be NULL.
 * FSM_EINVAL for a bad grid, pointer or precision, and when fewer than three cells are hit or
 * all hit cells lie on one line (zmap_out then holds the input values). */
int fsm_level(fsm_ctx *ctx, const fsm_grid *grid, int precision, const void *zmap_in,
              void *zmap_out, double plane[3], void *stream);

#define FSM_FILTER_SMOOTH 0   /* the weighted mean: the S-filter's output */
#define FSM_FILTER_ROUGH 1    /* the input minus the weighted mean: the L-filter's output */

/* Areal Gaussian filter of cut-off wavelength `cutoff` (mm): weights
 * exp(-pi (r / (alpha cutoff))^2), alpha = sqrt(ln 2 / pi), whose transmission is 50 % at the
 * cut-off wavelength, over the square window of half-width R = floor(trunc cutoff / dd + 1e-9)
 * cells, normalised over the hit cells inside it (so the map's border and holes need no
 * padding).  mode FSM_FILTER_SMOOTH or FSM_FILTER_ROUGH.  FSM_EINVAL for cutoff <= 0, trunc
 * outside (0, 4], a half-width above 3072 cells, or a bad grid, pointer, precision or mode. */
int fsm_filter(fsm_ctx *ctx, const fsm_grid *grid, int precision, const void *zmap_in,
               void *zmap_out, double cutoff, double trunc, int mode, void *stream);

typedef struct fsm_texture_spec {
    double lambda_s;   /* S-filter cut-off (mm), 0: none (the paper's instrument: 0.010) */
    double lambda_c;   /* L-filter cut-off (mm), 0: none (the paper's instrument: 0.8) */
    double trunc;      /* window half-width in cut-offs, both filters (0 < trunc <= 4) */
    int32_t level;     /* nonzero: remove the least-squares plane between the two filters */
    int32_t reserved;
} fsm_texture_spec;

/* The chain S-filter -> F-operator -> L-filter, then the roughness of the result (as
 * fsm_roughness).  plane (nullable) receives the removed plane (zeros without levelling).
 * Errors as the single operators. */
int fsm_texture(fsm_ctx *ctx, const fsm_grid *grid, int precision, const void *zmap_in,
                void *zmap_out, const fsm_texture_spec *spec, fsm_rough *out, double plane[3],
                void *stream);

/* fsm_texture over n maps of one grid in one launch sequence (a dataset of predicted maps,
 * Sec. 4.3): zmaps_in[m] -> zmaps_out[m] (device pointers; a map may be its own output),
 * out[m] its roughness, planes[3m .. 3m + 2] its removed plane (planes nullable).  The maps
 * are processed in groups whose filter scratch (16 bytes per cell and map) stays within
 * 4 GiB (a larger map forms a group of its own).  Errors as fsm_texture; a degenerate map is
 * named in the message. */
int fsm_texture_batch(fsm_ctx *ctx, int n, const fsm_grid *grid, int precision,
                      const void *const *zmaps_in, void *const *zmaps_out,
                      const fsm_texture_spec *spec, fsm_rough *out, double *planes, void *stream);

/* ---- serving loop --------------------------------------------------------------------------
 *
 * Simulations of different sizes and parameters arriving over time, the way a surrogate-model
 * dataset generator calls the method (Sec. 4.3 names dataset generation as the use of the
 * speed-up).  The caller's thread runs the loop: requests arrive at their stated times, are
 * admitted first come, first served as soon as their Z-map fits the device arena, and are
 * gathered into batches that run on n_slots streams at once, each with its own workspace, so
 * requests that arrive while others are on the device join it as soon as a slot frees up
 * (continuous batching).  Every batch is one fsm_simulate_batch launch sequence, so each
 * result equals the same simulation run alone. */

typedef struct fsm_request {
    const fsm_tool *tool;
    const fsm_cut *cut;
    const fsm_grid *grid;
    double arrival_s;        /* arrival time, seconds after the start of the run */
    void *zmap_dev;          /* caller-owned device Z-map (kept), or NULL: the server holds the
                                map in its arena while the request is in flight and returns
                                only the roughness.  The caller-owned maps of one run share no
                                byte (FSM_EINVAL from fsm_serve_run otherwise) */
} fsm_request;

typedef struct fsm_request_result {
    fsm_rough rough;
    double admit_s;          /* seconds after the start: admitted (arena range taken) */
    double start_s;          /* its batch was queued on the device */
    double done_s;           /* its batch was seen finished by the loop */
    int32_t status;          /* FSM_OK, FSM_EINVAL (bad parameters) or FSM_ENOMEM (larger
                                than the arena or than one slot's workspace) */
    int32_t batch;           /* index of its batch, -1 if it never ran */
    int32_t slot;            /* slot (stream) its batch ran on, -1 if it never ran */
    int32_t pad;
} fsm_request_result;

typedef struct fsm_serve_config {
    int32_t precision;       /* FSM_F64 or FSM_F32, for every request */
    int32_t n_slots;         /* batches in flight at once, 1..16 */
    int32_t max_batch;       /* simulations per batch, >= 1 */
    int32_t realtime;        /* 1: requests arrive at arrival_s on the wall clock; 0: all at 0,
                                queued in the order of arrival_s (ties: request order) */
    int64_t arena_bytes;     /* device bytes for server-held Z-maps (allocated once per run) */
    int64_t slot_bytes;      /* device workspace per slot (allocated once per run); batches are
                                sized, and their buckets sliced, to fit it */
} fsm_serve_config;

/* Serve n requests to completion on ctx's device.  out: n records, written for every request
 * (a rejected request carries its status; the call still returns FSM_OK).  The call allocates
 * the arena and the slot workspaces once at the start and frees them at the end; no device
 * memory is allocated while requests are served (each slot's pinned host staging grows to the
 * largest batch image it has carried).  Returns FSM_EINVAL for a bad configuration or
 * overlapping caller-owned Z-maps (before anything runs), FSM_ENOMEM if the arena or
 * workspaces cannot be allocated, FSM_EDEVICE on a HIP error. */
int fsm_serve_run(fsm_ctx *ctx, const fsm_serve_config *cfg, int n, const fsm_request *req,
                  fsm_request_result *out);

/* Device model of the dry run: a batch occupies its slot for launch_s plus, for every
 * simulation, per_eval_s per edge-point evaluation and per_cell_s per Z-map cell. */
typedef struct fsm_serve_model {
    double launch_s;
    double per_eval_s;
    double per_cell_s;
} fsm_serve_model;

/* Host only: the same scheduler as fsm_serve_run (arrivals, admission, batching, the slot
 * workspace rule) against a simulated clock and the device model; zmap_dev is ignored except
 * for NULL (server-held) versus non-NULL (caller-owned).  The roughness records are zero.
 * arena_peak (nullable) receives the most arena bytes held at once. */
int fsm_serve_dry_run(const fsm_serve_config *cfg, const fsm_serve_model *model, int n,
                      const fsm_request *req, fsm_request_result *out, int64_t *arena_peak);

#ifdef __cplusplus
}
#endif
#endif /* FSM_H */
