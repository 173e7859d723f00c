// Host checks of rr_host.h (the series time index, the serving arena, the
// admission rule and the tick planner) against brute-force models, built
// with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_host_sanitized.py.  Prints one line per check and exits
// non-zero on the first violation.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <random>
#include <vector>

#include "rr_host.h"

using namespace rr;

static int g_fail = 0;
#define CHECK(cond, ...)                                              \
    do {                                                              \
        if (!(cond)) {                                                \
            std::fprintf(stderr, "FAIL %s:%d: %s: ", __FILE__, __LINE__, #cond); \
            std::fprintf(stderr, __VA_ARGS__);                        \
            std::fprintf(stderr, "\n");                               \
            std::exit(1);                                             \
        }                                                             \
    } while (0)

// ---------------------------------------------------------------- index
static void check_index_of(const std::vector<double>& t, const std::vector<int32_t>& ids,
                           int nlc, bool expect_indexed) {
    std::vector<SeriesLc> lcs;
    std::vector<int32_t> bk;
    bool all_zero = false;
    const int npt = int(t.size());
    const bool ix = build_series_index(t.data(), ids.empty() ? nullptr : ids.data(), npt, nlc,
                                       &lcs, &bk, &all_zero);
    CHECK(ix == expect_indexed, "indexed %d expected %d (npt %d nlc %d)", ix, expect_indexed,
          npt, nlc);
    bool z = true;
    for (int32_t v : ids) z = z && v == 0;
    if (ix) CHECK(all_zero == z, "all_zero");
    if (!ix) {
        CHECK(lcs.empty() && bk.empty(), "not indexed but index filled");
        return;
    }
    CHECK(int(lcs.size()) == nlc, "lcs size");
    std::vector<int> covered(static_cast<size_t>(npt), 0);
    for (int l = 0; l < nlc; ++l) {
        const SeriesLc& s = lcs[size_t(l)];
        CHECK(s.boff >= 0 && s.boff + s.nb < int(bk.size()), "boff out of range");
        // the run: exactly the exposures with id l
        int n = 0;
        for (int i = 0; i < npt; ++i) {
            const int li = ids.empty() ? 0 : ids[size_t(i)];
            if (li == l) {
                CHECK(i >= s.start && i < s.end, "exposure %d of lc %d outside its run", i, l);
                ++n;
            }
        }
        CHECK(n == s.end - s.start, "run length");
        if (n == 0) {
            CHECK(s.nb == 0 && bk[size_t(s.boff)] == 0, "empty light curve");
            continue;
        }
        for (int i = s.start; i < s.end; ++i) covered[size_t(i)] += 1;
        CHECK(s.t_first == t[size_t(s.start)] && s.t_last == t[size_t(s.end - 1)], "ends");
        CHECK(bk[size_t(s.boff)] == s.start || s.nb == 1, "first bucket");
        CHECK(bk[size_t(s.boff + s.nb)] == s.end, "last entry");
        if (!(s.t_last > s.t_first)) {
            CHECK(s.nb == 1 && s.inv_bw == 0.0 && bk[size_t(s.boff)] == s.start, "constant run");
            continue;
        }
        CHECK(s.nb == n, "nb");
        const double bw = (s.t_last - s.t_first) / n;
        CHECK(s.inv_bw == 1.0 / bw, "inv_bw");
        for (int b = 0; b < s.nb; ++b) {
            const int lo = bk[size_t(s.boff + b)], hi = bk[size_t(s.boff + b + 1)];
            CHECK(lo <= hi && lo >= s.start && hi <= s.end, "bucket %d order", b);
            const double edge = s.t_first + b * bw;
            // entry b is the first exposure at or after its edge
            for (int i = s.start; i < lo; ++i) CHECK(t[size_t(i)] < edge, "before edge");
            if (lo < s.end) CHECK(t[size_t(lo)] >= edge, "at edge");
        }
    }
    for (int i = 0; i < npt; ++i) CHECK(covered[size_t(i)] == 1, "exposure %d covered", i);
}

static void check_index(std::mt19937_64& rng) {
    std::uniform_real_distribution<double> U(0.0, 1.0);
    int cases = 0;
    for (int it = 0; it < 600; ++it) {
        const int nlc = 1 + int(rng() % 6);
        std::vector<std::vector<double>> runs(static_cast<size_t>(nlc));
        for (auto& r : runs) {
            const int kind = int(rng() % 6);
            const int n = kind == 0 ? 0 : 1 + int(rng() % 300);
            double x = 2.46e6 + 100 * U(rng);
            for (int i = 0; i < n; ++i) {
                if (kind == 1) { r.push_back(x); continue; }               // constant
                const double gap = kind == 2 ? (U(rng) < 0.3 ? 0.0 : U(rng))  // repeats
                                 : kind == 3 ? (U(rng) < 0.05 ? 3.0 : 0.01)  // gaps
                                             : 0.001388 * (0.5 + U(rng));
                x += gap;
                r.push_back(x);
            }
        }
        // runs in a random order of light curves
        std::vector<int> order(static_cast<size_t>(nlc));
        for (int l = 0; l < nlc; ++l) order[size_t(l)] = l;
        std::shuffle(order.begin(), order.end(), rng);
        std::vector<double> t;
        std::vector<int32_t> ids;
        for (int l : order)
            for (double v : runs[size_t(l)]) { t.push_back(v); ids.push_back(l); }
        check_index_of(t, ids, nlc, true);
        if (nlc == 1) check_index_of(t, {}, 1, true);
        ++cases;
        if (t.size() < 3) continue;
        // broken variants: each must come out not indexed
        {
            std::vector<double> b = t;                      // a NaN time
            b[size_t(rng() % b.size())] = std::nan("");
            check_index_of(b, ids, nlc, false);
        }
        {
            std::vector<int32_t> b = ids;                   // an id out of range
            b[size_t(rng() % b.size())] = (rng() & 1) ? nlc : -1;
            check_index_of(t, b, nlc, false);
        }
        for (size_t i = 1; i < t.size(); ++i) {            // a decreasing step
            if (ids[i] == ids[i - 1] && t[i] > t[i - 1]) {
                std::vector<double> b = t;
                std::swap(b[i], b[i - 1]);
                check_index_of(b, ids, nlc, false);
                break;
            }
        }
        if (nlc >= 2 && ids.front() != ids.back()) {       // a second run of one id
            std::vector<int32_t> b = ids;
            std::vector<double> bt = t;
            b.push_back(ids.front());
            bt.push_back(t.back() + 1.0);
            check_index_of(bt, b, nlc, false);
        }
    }
    check_index_of({}, {}, 1, true);                          // no exposures
    check_index_of({}, {}, 3, true);
    std::printf("index: %d random series and their broken variants\n", cases);
}

// ---------------------------------------------------------------- arena
struct Model {      // granule bitmap, first fit over maximal free runs
    std::vector<char> used;
    explicit Model(size_t n) : used(n, 0) {}
    bool alloc(size_t g, size_t* off) {
        size_t i = 0;
        while (i < used.size()) {
            if (used[i]) { ++i; continue; }
            size_t j = i;
            while (j < used.size() && !used[j]) ++j;
            if (j - i >= g) {
                for (size_t k = i; k < i + g; ++k) used[k] = 1;
                *off = i;
                return true;
            }
            i = j;
        }
        return false;
    }
    void release(size_t off, size_t g) {
        for (size_t k = off; k < off + g; ++k) used[k] = 0;
    }
    std::vector<std::pair<size_t, size_t>> runs() const {
        std::vector<std::pair<size_t, size_t>> r;
        size_t i = 0;
        while (i < used.size()) {
            if (used[i]) { ++i; continue; }
            size_t j = i;
            while (j < used.size() && !used[j]) ++j;
            r.emplace_back(i, j - i);
            i = j;
        }
        return r;
    }
};

static void check_arena(std::mt19937_64& rng) {
    const size_t G = Arena::kGranule;
    long ops = 0;
    for (int it = 0; it < 200; ++it) {
        const size_t ngran = 1 + rng() % 400;
        Arena a;
        a.init(ngran * G);
        Model m(ngran);
        std::vector<std::pair<size_t, size_t>> live;   // offset, bytes asked
        for (int step = 0; step < 400; ++step, ++ops) {
            if (live.empty() || rng() % 3) {
                const size_t bytes = 1 + rng() % (40 * G);
                size_t off = 0, moff = 0;
                const bool ok = a.alloc(bytes, &off);
                const bool mok = m.alloc(Arena::round(bytes) / G, &moff);
                CHECK(ok == mok, "alloc success differs (bytes %zu)", bytes);
                if (ok) {
                    CHECK(off == moff * G, "first fit: %zu vs %zu", off, moff * G);
                    CHECK(off % G == 0 && off + Arena::round(bytes) <= ngran * G, "bounds");
                    live.emplace_back(off, bytes);
                }
            } else {
                const size_t k = rng() % live.size();
                a.release(live[k].first, live[k].second);
                m.release(live[k].first / G, Arena::round(live[k].second) / G);
                live[k] = live.back();
                live.pop_back();
            }
            // free blocks are exactly the model's maximal runs
            const auto runs = m.runs();
            const auto& fb = a.free_blocks();
            CHECK(fb.size() == runs.size(), "free block count %zu vs %zu", fb.size(), runs.size());
            size_t i = 0;
            for (const auto& kv : fb) {
                CHECK(kv.first == runs[i].first * G && kv.second == runs[i].second * G,
                      "free block %zu", i);
                ++i;
            }
        }
        for (auto& l : live) a.release(l.first, l.second);
        CHECK(a.free_blocks().size() == 1 && a.free_blocks().begin()->second == ngran * G,
              "arena not whole after releasing everything");
    }
    std::printf("arena: %ld operations against the bitmap model\n", ops);
}

// ------------------------------------------------------------ admission
static void check_admission(std::mt19937_64& rng) {
    const size_t G = Arena::kGranule;
    long admitted_total = 0;
    for (int it = 0; it < 200; ++it) {
        const size_t budget = (8 + rng() % 200) * G;
        Arena a;
        a.init(budget);
        struct Req { int id; size_t bytes, off; int life; };
        std::deque<Req*> pending;
        std::vector<Req*> running;
        std::vector<Req> all(static_cast<size_t>(50 + rng() % 200));
        for (size_t i = 0; i < all.size(); ++i)
            all[i] = Req{int(i), 1 + rng() % budget, 0, 1 + int(rng() % 5)};   // each fits alone
        size_t next = 0;
        int last_admitted = -1, rounds = 0;
        const int max_jobs = 1 + int(rng() % 24);
        while (next < all.size() || !pending.empty() || !running.empty()) {
            CHECK(++rounds < 100000, "admission does not drain");
            for (int k = int(rng() % 4); k > 0 && next < all.size(); --k)
                pending.push_back(&all[next++]);
            const size_t before = pending.size();
            std::vector<Req*> got;
            const int n = admit_in_order(
                pending, a, max_jobs, [](Req* r) { return r->bytes; },
                [&](Req* r, size_t off) { r->off = off; got.push_back(r); });
            CHECK(n == int(got.size()) && n <= max_jobs && before - pending.size() == size_t(n),
                  "admitted count");
            for (Req* r : got) {
                CHECK(r->id == last_admitted + 1, "admitted out of order");
                last_admitted = r->id;
                running.push_back(r);
            }
            if (n < max_jobs && !pending.empty()) {
                size_t off = 0;                       // the head really does not fit
                CHECK(!a.alloc(pending.front()->bytes, &off), "head fits but was not admitted");
            }
            // live allocations never overlap
            std::vector<std::pair<size_t, size_t>> iv;
            for (Req* r : running) iv.emplace_back(r->off, Arena::round(r->bytes));
            std::sort(iv.begin(), iv.end());
            for (size_t i = 1; i < iv.size(); ++i)
                CHECK(iv[i - 1].first + iv[i - 1].second <= iv[i].first, "overlap");
            for (size_t i = 0; i < running.size();) {
                if (--running[i]->life <= 0) {
                    a.release(running[i]->off, running[i]->bytes);
                    running[i] = running.back();
                    running.pop_back();
                } else {
                    ++i;
                }
            }
        }
        CHECK(last_admitted == int(all.size()) - 1, "not every request admitted");
        CHECK(a.free_blocks().size() == 1 && a.free_blocks().begin()->second == budget, "arena");
        admitted_total += long(all.size());
    }
    std::printf("admission: %ld requests admitted in arrival order\n", admitted_total);
}

// -------------------------------------------------------------- ticks
static void check_ticks(std::mt19937_64& rng) {
    long ticks = 0;
    for (int it = 0; it < 200; ++it) {
        const int nreq = 1 + int(rng() % 40);
        const int32_t max_blocks = (it % 10 == 0 ? 1 : 64) + int32_t(rng() % 4096);
        const int32_t max_jobs = 1 + int32_t(rng() % 24);
        std::vector<TickReq> req(static_cast<size_t>(nreq));
        std::vector<int32_t> npv(static_cast<size_t>(nreq)), done(static_cast<size_t>(nreq), 0);
        for (int i = 0; i < nreq; ++i) {
            npv[size_t(i)] = 1 + int32_t(rng() % (it % 10 == 0 ? 64 : 2048));
            req[size_t(i)] = TickReq{npv[size_t(i)], 1 + int32_t(rng() % 400), int32_t(rng() % 2)};
        }
        int guard = 0;
        while (true) {
            std::vector<TickReq> act;
            std::vector<int> map;
            for (int i = 0; i < nreq; ++i)
                if (req[size_t(i)].remaining > 0) { act.push_back(req[size_t(i)]); map.push_back(i); }
            if (act.empty()) break;
            CHECK(++guard < 1000000, "ticks do not drain");
            const auto parts = plan_tick(act, max_blocks, max_jobs);
            CHECK(!parts.empty(), "no progress with %zu active", act.size());
            int64_t blocks = 0;
            int jobs[2] = {0, 0};
            std::vector<int> seen(act.size(), 0);
            for (const TickPart& p : parts) {
                CHECK(p.req >= 0 && p.req < int(act.size()) && p.rows >= 1, "part");
                seen[size_t(p.req)] += 1;
                CHECK(seen[size_t(p.req)] <= 2, "request more than once per pass");
                blocks += int64_t(p.rows) * act[size_t(p.req)].ntiles;
                jobs[act[size_t(p.req)].slot] += 1;
                TickReq& r = req[size_t(map[size_t(p.req)])];
                r.remaining -= p.rows;
                CHECK(r.remaining >= 0, "more rows than remain");
                done[size_t(map[size_t(p.req)])] += p.rows;
            }
            CHECK(jobs[0] <= max_jobs && jobs[1] <= max_jobs, "jobs per slot");
            const bool lone = parts.size() == 1 && parts[0].rows == 1;
            CHECK(blocks <= max_blocks || lone, "tick of %lld > %d blocks", (long long)blocks,
                  max_blocks);
            if (lone && blocks > max_blocks)
                CHECK(act[size_t(parts[0].req)].ntiles > max_blocks, "lone row that fits");
            // fair share: with job slots free, the first pass gives each request
            // min(rows left, share / ntiles) rows or more, in order, until the tick fills
            const int32_t share = std::max<int32_t>(1, max_blocks / int32_t(act.size()));
            int32_t left = max_blocks;
            int js[2] = {0, 0};
            bool first = true;
            for (size_t i = 0; i < act.size() && left > 0; ++i) {
                const int p = act[i].slot;
                if (js[p] >= max_jobs) continue;
                int32_t want = std::min(act[i].remaining, std::min(share, left) / act[i].ntiles);
                if (want == 0 && first) want = 1;        // a row larger than the tick
                if (want > 0) first = false;
                int32_t got = 0;
                for (const TickPart& q : parts)
                    if (q.req == int(i)) got += q.rows;
                if (want > 0) {
                    CHECK(got >= want, "request %zu got %d < fair %d", i, got, want);
                    js[p] += 1;
                    left -= want * act[i].ntiles;
                }
            }
            ++ticks;
        }
        for (int i = 0; i < nreq; ++i) CHECK(done[size_t(i)] == npv[size_t(i)], "rows launched");
    }
    std::printf("ticks: %ld planned, every row launched once\n", ticks);
}

int main() {
    std::mt19937_64 rng(2009085000ull);
    check_index(rng);
    check_arena(rng);
    check_admission(rng);
    check_ticks(rng);
    std::printf("OK\n");
    return g_fail;
}
