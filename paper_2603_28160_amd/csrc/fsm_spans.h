// fsm_spans.h -- whether byte ranges of caller-owned device memory conflict.
//
// Maps of one call are read and written by the same launches, so a map that is written must
// share no byte with any other map of the call; maps that are only read may share bytes with
// each other.  The calls that take several maps check their ranges with this before queueing
// anything.  Host-only and free of HIP, so that it is tested on its own.
#pragma once

#include <algorithm>
#include <cstdint>
#include <utility>
#include <vector>

namespace fsm {

struct Span {
    uintptr_t begin, end;   // [begin, end) in bytes; empty when end <= begin
    int owner;              // the caller's index of the map (job or map number)
    bool read_only;         // only read by the call
};

// The owners of two spans that share a byte while at least one of them is written, or
// {-1, -1} when there are none.  Empty spans share nothing.  After sorting by start, a span
// conflicts with an earlier one exactly when it starts before the furthest end among the
// earlier written spans, or, being written itself, before the furthest end among the earlier
// read-only ones; one sweep keeps both ends.
inline std::pair<int, int> first_conflict(std::vector<Span> s)
{
    s.erase(std::remove_if(s.begin(), s.end(), [](const Span &r) { return r.end <= r.begin; }), s.end());
    std::sort(s.begin(), s.end(), [](const Span &a, const Span &b) {
        return a.begin != b.begin ? a.begin < b.begin : a.end < b.end;
    });
    const Span none = {0, 0, -1, true};
    Span wr = none, rd = none;   // furthest-reaching written and read-only spans so far
    for (const Span &k : s) {
        if (k.begin < wr.end) return {wr.owner, k.owner};
        if (!k.read_only && k.begin < rd.end) return {rd.owner, k.owner};
        Span &m = k.read_only ? rd : wr;
        if (k.end > m.end) m = k;
    }
    return {-1, -1};
}

}  // namespace fsm
