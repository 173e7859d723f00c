// rr_host.h -- host-side logic of librr.so that involves no device code:
// the time index of a registered series, the serving arena's first-fit
// allocator and the serving loop's tick planner.
//
// Plain C++17 with no HIP types, so that the host tests build it on its own
// (with AddressSanitizer and UndefinedBehaviorSanitizer) and check it
// against brute-force models; the library includes the same code.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <iterator>
#include <map>
#include <vector>

namespace rr {

// One light curve of a registered series whose exposures are the contiguous
// run [start, end) of the arrays with non-decreasing times t_first ..
// t_last.  Its index (nb + 1 entries at boff of the series' bucket array):
// entry b < nb is the first exposure with t >= t_first + b * bw
// (bw = (t_last - t_first)/nb, inv_bw = 1/bw, or 0 when all times are
// equal), entry nb is end.
struct SeriesLc {
    int32_t start, end, boff, nb;
    double t_first, t_last, inv_bw;
};

// The time index of a series (npt exposures, light-curve ids lcids[npt] in
// [0, nlc) or NULL for one light curve).  Returns whether every light curve
// is one contiguous run of finite, non-decreasing times ("indexed"); only
// then are lcs[nlc] and buckets filled (nb = the run's length, one bucket
// per exposure on average; an empty light curve gets nb = 0 and a single
// entry, one whose times are all equal nb = 1).  *all_zero tells whether
// every id is 0 (always true without ids).  Ids outside [0, nlc) or a
// non-finite time make the series not indexed; nothing is read beyond
// times[npt], lcids[npt].
inline bool build_series_index(const double* times, const int32_t* lcids, int32_t npt,
                               int32_t nlc, std::vector<SeriesLc>* lcs_out,
                               std::vector<int32_t>* buckets_out, bool* all_zero) {
    std::vector<SeriesLc> lcs(size_t(nlc), SeriesLc{0, 0, 0, 0, 0.0, 0.0, 0.0});
    std::vector<char> seen(size_t(nlc), 0);
    bool indexed = true;
    bool zero = true;
    int32_t prev = 0;
    for (int32_t i = 0; i < npt; ++i) {
        const int32_t l = lcids ? lcids[i] : 0;
        if (l < 0 || l >= nlc || !std::isfinite(times[i])) { indexed = false; break; }
        zero = zero && l == 0;
        if (i == 0 || l != prev) {
            if (seen[size_t(l)]) { indexed = false; break; }    // a second run of l
            seen[size_t(l)] = 1;
            lcs[size_t(l)].start = i;
        } else if (!(times[i] >= times[i - 1])) {
            indexed = false;
            break;
        }
        lcs[size_t(l)].end = i + 1;
        prev = l;
    }
    *all_zero = lcids ? zero : true;
    lcs_out->clear();
    buckets_out->clear();
    if (!indexed) return false;
    std::vector<int32_t>& buckets = *buckets_out;
    for (int32_t l = 0; l < nlc; ++l) {
        SeriesLc& sl = lcs[size_t(l)];
        const int32_t n = sl.end - sl.start;
        sl.boff = int32_t(buckets.size());
        if (n <= 0) {
            sl.start = sl.end = 0;
            sl.nb = 0;
            buckets.push_back(0);
            continue;
        }
        sl.t_first = times[sl.start];
        sl.t_last = times[sl.end - 1];
        if (!(sl.t_last > sl.t_first)) {
            sl.nb = 1;
            sl.inv_bw = 0.0;
            buckets.push_back(sl.start);
            buckets.push_back(sl.end);
            continue;
        }
        sl.nb = n;
        const double bw = (sl.t_last - sl.t_first) / n;
        sl.inv_bw = 1.0 / bw;
        int32_t i = sl.start;
        for (int32_t b = 0; b < n; ++b) {
            const double edge = sl.t_first + b * bw;
            while (i < sl.end && times[i] < edge) ++i;
            buckets.push_back(i);
        }
        buckets.push_back(sl.end);
    }
    *lcs_out = std::move(lcs);
    return true;
}

// First-fit allocator over [0, size) in 256-byte granules: an allocation
// takes the lowest-addressed free block that is large enough, and a release
// merges with both neighbours, so free blocks are always maximal.
class Arena {
  public:
    static constexpr size_t kGranule = 256;
    static size_t round(size_t bytes) { return (bytes + kGranule - 1) / kGranule * kGranule; }

    void init(size_t size) {
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(size_t bytes, size_t* off) {
        bytes = round(bytes);
        if (bytes == 0) bytes = kGranule;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, o = it->first + bytes;
                free_.erase(it);
                if (rest) free_[o] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = round(bytes);
        if (bytes == 0) bytes = kGranule;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    const std::map<size_t, size_t>& free_blocks() const { return free_; }

  private:
    std::map<size_t, size_t> free_;   // offset -> length
};

// Admission in arrival order: while fewer than max_jobs were admitted in
// this round, the oldest pending request (pending.front()) is given
// bytes_of(request) from the arena (first fit) and passed with its offset
// to on_admit; the first one that does not fit stops the round, so no
// request overtakes an older one and a large request is not starved by a
// stream of small ones.  Returns the number admitted.
template <class Queue, class BytesOf, class OnAdmit>
int admit_in_order(Queue& pending, Arena& arena, int max_jobs, BytesOf bytes_of,
                   OnAdmit on_admit) {
    int n = 0;
    while (!pending.empty() && n < max_jobs) {
        auto r = pending.front();
        size_t off = 0;
        if (!arena.alloc(bytes_of(r), &off)) break;
        pending.pop_front();
        on_admit(r, off);
        ++n;
    }
    return n;
}

// One active request as the tick planner sees it: rows not yet launched,
// workgroups per row (the series' time tiles) and its precision slot (0 or
// 1: one grouped launch per precision).
struct TickReq {
    int32_t remaining, ntiles, slot;
};
struct TickPart {
    int32_t req, rows;     // index into the active list, rows this tick
};

// One tick: at most max_blocks workgroups and max_jobs parts per slot.  A
// first pass gives every request, in order, up to its fair share
// (max_blocks / #active workgroups, whole rows); a second pass fills what
// is left in the same order.  A single row larger than the whole tick is
// launched alone (the first request's row when nothing else fits).  Parts
// come out in launch order; a request may appear once per pass.
inline std::vector<TickPart> plan_tick(const std::vector<TickReq>& active, int32_t max_blocks,
                                       int32_t max_jobs) {
    std::vector<TickPart> parts;
    if (active.empty() || max_blocks < 1) return parts;
    std::vector<int32_t> left_rows(active.size());
    for (size_t i = 0; i < active.size(); ++i) left_rows[i] = std::max(0, active[i].remaining);
    int32_t jobs[2] = {0, 0};
    int32_t left = max_blocks;
    const int32_t share = std::max<int32_t>(1, max_blocks / int32_t(active.size()));
    for (int pass = 0; pass < 2 && left > 0; ++pass) {
        for (size_t i = 0; i < active.size(); ++i) {
            if (left <= 0) break;
            const TickReq& r = active[i];
            const int p = r.slot ? 1 : 0;
            if (jobs[p] >= max_jobs) continue;
            if (left_rows[i] <= 0 || r.ntiles < 1) continue;
            const int32_t cap = pass == 0 ? std::min(share, left) : left;
            int32_t rows = std::min(left_rows[i], cap / r.ntiles);
            if (rows == 0 && pass == 0 && parts.empty()) rows = 1;   // one row > tick
            if (rows == 0) continue;
            jobs[p] += 1;
            left -= rows * r.ntiles;
            left_rows[i] -= rows;
            parts.push_back(TickPart{int32_t(i), rows});
        }
    }
    return parts;
}

}  // namespace rr
