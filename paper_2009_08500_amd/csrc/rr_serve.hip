// rr_serve.hip -- continuous-batching request loop over resident tables.
//
// Time series are registered once and stay on the device with the LD
// tables.  A request is a population of parameter rows against one series;
// its footprint (rows, per-row constants, and the output unless the caller
// gives a device buffer for it) is carved from a device arena sized at
// creation, and requests are admitted in arrival order as arena space
// frees up.  A worker thread cuts every admitted request into
// (row x time-tile) workgroups and packs workgroups of all admitted requests
// into "ticks": one grouped forward launch per precision, at most
// max_tick_blocks workgroups, each active request first getting a fair
// share so that small requests are not queued behind large ones.  Ticks
// alternate over two streams, so a tick's kernels overlap the next one's
// and requests that arrive while others run join the next tick.  When all
// rows of a request are done its output is copied to the caller's host
// buffer (host-output requests) or is already in the caller's device
// buffer (device-output requests), and its arena space is released;
// latency is completion minus submission, on the host's steady clock.
// A request keeps its own copy of its series' description, taken at
// submission under the lock, so the worker never reads the series list
// that rr_server_add_series may grow concurrently.
//
// Every request runs the same forward_block() code as rr_evaluate, so its
// results do not depend on what it was batched with.
#include <algorithm>
#include <cmath>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "rr_internal.h"
#include "rr_serve.h"

namespace rr {
namespace {

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Series {
    double* times = nullptr;
    int32_t* lcids = nullptr;
    LcInfo* lc = nullptr;
    int32_t npt = 0, ntiles = 0;
    int64_t nsub = 0;          // subsamples per parameter row
    int32_t max_nss = 1;       // largest nss of its light curves
};

enum ReqState { kQueued = 0, kRunning = 1, kDone = 2 };

struct Request {
    int64_t id = 0;
    int32_t series = 0, npv = 0, npar = 0, precision = 0;
    Series se;                 // the series' description, copied at submission
    std::vector<double> pv;
    void* out_host = nullptr;  // host output, or
    void* out_user = nullptr;  // the caller's device output buffer
    size_t out_bytes = 0, off = 0, bytes = 0;
    double* pv_dev = nullptr;
    PvConst* pvc_dev = nullptr;
    void* out_dev = nullptr;
    int32_t next_row = 0, rows_done = 0;
    int state = kQueued;
    bool copying = false;
    hipEvent_t done_ev = nullptr;
    double t_submit = 0, t_done = 0;
    std::atomic<int> err{RR_OK};
};

// A grouped launch and the request rows it covers.  ev == nullptr marks a
// tick whose launch failed: its stream was synchronised instead, so it
// counts as complete (its requests carry RR_EDEVICE).
struct Tick {
    hipEvent_t ev = nullptr;
    std::vector<std::pair<Request*, int32_t>> parts;
};

}  // namespace
}  // namespace rr

using namespace rr;

struct rr_server {
    const rr_tables* t = nullptr;
    int device = 0;
    size_t budget = 0;
    char* arena_base = nullptr;
    Arena arena;
    int32_t max_tick_blocks = 0;
    hipStream_t streams[2] = {nullptr, nullptr};
    hipStream_t setup_stream = nullptr, copy_stream = nullptr;
    hipEvent_t setup_ev = nullptr;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> incoming;                      // guarded by mu
    std::unordered_map<int64_t, Request*> reqs;         // guarded by mu
    std::vector<Series> series;                         // guarded by mu
    int64_t next_id = 1;
    bool stop = false;
    std::thread worker;
    // worker-only state
    std::deque<Request*> pending;
    std::vector<Request*> active;
    std::vector<Request*> copying;
    std::deque<Tick> ticks;
    std::vector<hipEvent_t> tick_events;   // completed ticks' events, for reuse
    int tick_stream = 0;
    std::atomic<int> fail_next_tick{0};   // test hook: fail the next tick's launch
    // statistics (guarded by mu)
    int64_t completed = 0, points = 0, nticks = 0;
    int last_error = RR_OK;

    size_t footprint(int32_t npv, int32_t npar, int32_t npt, int32_t precision,
                     bool device_out) const {
        const size_t elt = precision == RR_FP64 ? 8 : 4;
        auto r = [](size_t b) { return (b + 255) / 256 * 256; };
        return r(size_t(npv) * npar * 8) + r(size_t(npv) * sizeof(PvConst)) +
               (device_out ? 0 : r(size_t(npv) * npt * elt));
    }

    void run();
    bool step();
    void finish(Request* r);
};

// Release a request's arena space and mark it done (worker thread).
void rr_server::finish(Request* r) {
    const double t = now_s();
    arena.release(r->off, r->bytes);
    {
        std::lock_guard<std::mutex> lk(mu);
        r->t_done = t;
        r->state = kDone;
        completed += 1;
        points += int64_t(r->npv) * r->se.nsub;
    }
    cv_done.notify_all();
}

bool rr_server::step() {
    bool did = false;
    {
        std::lock_guard<std::mutex> lk(mu);
        while (!incoming.empty()) {
            pending.push_back(incoming.front());
            incoming.pop_front();
        }
    }
    // 1. completed ticks (in order)
    while (!ticks.empty() &&
           (!ticks.front().ev || hipEventQuery(ticks.front().ev) == hipSuccess)) {
        Tick& tk = ticks.front();
        for (auto& pr : tk.parts) {
            Request* r = pr.first;
            r->rows_done += pr.second;
            if (r->rows_done == r->npv && !r->copying) {
                r->copying = true;
                if (r->out_user || r->err != RR_OK) {
                    // the rows are in the caller's device buffer (or failed)
                    finish(r);
                    continue;
                }
                hipError_t e = hipMemcpyAsync(r->out_host, r->out_dev, r->out_bytes,
                                              hipMemcpyDeviceToHost, copy_stream);
                if (e == hipSuccess) e = hipEventRecord(r->done_ev, copy_stream);
                if (e != hipSuccess) {
                    (void)hipStreamSynchronize(copy_stream);
                    r->err = RR_EDEVICE;
                }
                copying.push_back(r);
            }
        }
        if (tk.ev) tick_events.push_back(tk.ev);
        ticks.pop_front();
        did = true;
    }
    // 2. finished copies
    for (size_t i = 0; i < copying.size();) {
        Request* r = copying[i];
        if (r->err != RR_OK || hipEventQuery(r->done_ev) == hipSuccess) {
            finish(r);
            copying[i] = copying.back();
            copying.pop_back();
            did = true;
        } else {
            ++i;
        }
    }
    // 3. admission in arrival order while the arena has room
    SetupTable st;
    st.njobs = 0;
    int32_t nthreads = 0;
    const int nadm = admit_in_order(
        pending, arena, kMaxJobs, [](Request* r) { return r->bytes; },
        [&](Request* r, size_t off) {
            r->off = off;
            char* base = arena_base + off;
            const size_t pvb = Arena::round(size_t(r->npv) * r->npar * 8);
            const size_t pcb = Arena::round(size_t(r->npv) * sizeof(PvConst));
            r->pv_dev = reinterpret_cast<double*>(base);
            r->pvc_dev = reinterpret_cast<PvConst*>(base + pvb);
            r->out_dev = r->out_user ? r->out_user : base + pvb + pcb;
            hipError_t e = hipMemcpyAsync(r->pv_dev, r->pv.data(),
                                          size_t(r->npv) * r->npar * 8,
                                          hipMemcpyHostToDevice, setup_stream);
            if (e != hipSuccess) r->err = RR_EDEVICE;
            SetupJob& sj = st.j[st.njobs++];
            sj.pv = r->pv_dev;
            sj.pvc = r->pvc_dev;
            sj.npv = r->npv;
            sj.npar = r->npar;
            sj.thread0 = nthreads;
            sj.f32 = r->precision == RR_FP64 ? 0 : 1;
            nthreads += r->npv;
            {
                std::lock_guard<std::mutex> lk(mu);
                r->state = kRunning;
            }
            active.push_back(r);
        });
    if (nadm) did = true;
    if (st.njobs) {
        if (launch_pv_setup_jobs(t, st, nthreads, setup_stream) != hipSuccess ||
            hipEventRecord(setup_ev, setup_stream) != hipSuccess)
            last_error = RR_EDEVICE;
    }
    // 4. one tick if fewer than two are in flight
    if (!active.empty() && ticks.size() < 2) {
        std::vector<TickReq> want(active.size());
        for (size_t i = 0; i < active.size(); ++i)
            want[i] = TickReq{active[i]->npv - active[i]->next_row, active[i]->se.ntiles,
                              active[i]->precision == RR_FP64 ? 0 : 1};
        JobTable jt[2];
        int32_t nb[2] = {0, 0};
        jt[0].njobs = jt[1].njobs = 0;
        Tick tk;
        for (const TickPart& part : plan_tick(want, max_tick_blocks, kMaxJobs)) {
            Request* r = active[size_t(part.req)];
            const int p = want[size_t(part.req)].slot;
            const Series& se = r->se;
            FwdJob& j = jt[p].j[jt[p].njobs++];
            j.times = se.times; j.lcids = se.lcids; j.lc = se.lc; j.pv = r->pv_dev;
            j.pvc = r->pvc_dev; j.out = r->out_dev; j.npt = se.npt; j.npar = r->npar;
            j.pv0 = r->next_row; j.npv = part.rows; j.ntiles = se.ntiles; j.block0 = nb[p];
            j.max_nss = se.max_nss;
            j.ldw_pv = nullptr; j.inv_istar_pv = nullptr; j.ldw_exact_k = 0; j.spread = 1;
            nb[p] += part.rows * se.ntiles;
            r->next_row += part.rows;
            tk.parts.emplace_back(r, part.rows);
        }
        if (!tk.parts.empty()) {
            hipStream_t s = streams[tick_stream];
            tick_stream ^= 1;
            hipError_t e = hipStreamWaitEvent(s, setup_ev, 0);
            if (e == hipSuccess && fail_next_tick.exchange(0)) e = hipErrorLaunchFailure;
            for (int p = 0; p < 2 && e == hipSuccess; ++p)
                e = launch_forward_jobs(t, jt[p], nb[p], p == 0 ? RR_FP64 : RR_MIXED, s);
            if (e == hipSuccess) {
                if (!tick_events.empty()) {
                    tk.ev = tick_events.back();
                    tick_events.pop_back();
                } else {
                    e = hipEventCreateWithFlags(&tk.ev, hipEventDisableTiming);
                }
            }
            if (e == hipSuccess) e = hipEventRecord(tk.ev, s);
            if (e != hipSuccess) {
                // whatever did launch finishes before the tick counts as
                // complete, so no arena space is released under a kernel
                if (tk.ev) (void)hipEventDestroy(tk.ev);
                tk.ev = nullptr;
                (void)hipStreamSynchronize(s);
                last_error = RR_EDEVICE;
                for (auto& pr : tk.parts) pr.first->err = RR_EDEVICE;
            }
            ticks.push_back(std::move(tk));
            std::lock_guard<std::mutex> lk(mu);
            nticks += 1;
            did = true;
        }
        // A request leaves `active` as soon as its last rows are launched,
        // before any tick of it can complete: once finish() has marked it
        // done, the caller may release (delete) it at any moment, so no
        // list of the worker may still hold it then.
        active.erase(std::remove_if(active.begin(), active.end(),
                                    [](Request* r) { return r->next_row >= r->npv; }),
                     active.end());
    }
    return did;
}

void rr_server::run() {
    (void)hipSetDevice(device);
    while (true) {
        const bool did = step();
        hipEvent_t oldest = nullptr;
        bool poll = false;
        {
            std::unique_lock<std::mutex> lk(mu);
            const bool idle = incoming.empty() && pending.empty() && active.empty() &&
                              ticks.empty() && copying.empty();
            if (stop && idle) break;
            if (did) continue;
            if (idle) {
                cv_work.wait_for(lk, std::chrono::milliseconds(2));
                continue;
            }
            // A timed sleep lasts tens of us, longer than a short tick, so
            // while ticks are in flight the worker does not sleep: with both
            // tick slots busy and nothing else to watch it waits on the
            // oldest tick's event (nothing else can happen first); with a
            // slot free it polls that event for a while, taking a new
            // request or a finished copy at the next step.
            if (incoming.empty() && copying.empty() && ticks.size() >= 2 && ticks.front().ev)
                oldest = ticks.front().ev;
            else if (!ticks.empty() && ticks.front().ev)
                poll = true;
            else
                cv_work.wait_for(lk, std::chrono::microseconds(20));
        }
        if (oldest) {
            (void)hipEventSynchronize(oldest);
        } else if (poll) {
            const auto until = std::chrono::steady_clock::now() + std::chrono::microseconds(50);
            while (hipEventQuery(ticks.front().ev) == hipErrorNotReady &&
                   std::chrono::steady_clock::now() < until) {
                std::this_thread::yield();
                std::lock_guard<std::mutex> lk(mu);
                if (!incoming.empty()) break;
            }
        }
    }
}

extern "C" {

RR_API int rr_server_create(const rr_tables* t, int64_t budget_bytes, int32_t max_tick_blocks,
                            rr_server** out) {
    if (!out) { set_error("out is NULL"); return RR_EINVAL; }
    *out = nullptr;
    if (!t) { set_error("tables handle is NULL"); return RR_EINVAL; }
    if (budget_bytes < (1 << 20)) { set_error("budget must be >= 1 MiB"); return RR_EINVAL; }
    if (max_tick_blocks < 1) { set_error("max_tick_blocks must be >= 1"); return RR_EINVAL; }
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (cur != t->device) { set_error("tables live on another device"); return RR_EINVAL; }
    rr_server* s = new (std::nothrow) rr_server();
    if (!s) return RR_ENOMEM;
    s->t = t;
    s->device = cur;
    s->budget = size_t(budget_bytes);
    s->max_tick_blocks = max_tick_blocks;
    e = hipMalloc((void**)&s->arena_base, s->budget);
    if (e != hipSuccess) {
        delete s;
        set_error("arena allocation failed");
        return e == hipErrorOutOfMemory ? RR_ENOMEM : RR_EDEVICE;
    }
    s->arena.init(s->budget);
    bool ok = true;
    for (auto& st : s->streams) ok = ok && hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&s->setup_stream, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&s->setup_ev, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventRecord(s->setup_ev, s->setup_stream) == hipSuccess;
    if (!ok) {
        set_error("stream/event creation failed");
        rr_server_destroy(s);
        return RR_EDEVICE;
    }
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return RR_OK;
}

RR_API int rr_server_add_series(rr_server* s, const double* times, const int32_t* lcids,
                                int32_t npt, const int32_t* pbids, const int32_t* nss,
                                const double* exptimes, int32_t nlc, int32_t* series_id) {
    if (!s || !series_id) { set_error("server or series_id is NULL"); return RR_EINVAL; }
    if (npt < 1 || !times) { set_error("times must hold npt >= 1 values"); return RR_EINVAL; }
    if (nlc < 1 || !pbids || !nss || !exptimes) { set_error("light-curve arrays required"); return RR_EINVAL; }
    if (nlc > RR_MAX_LC) { set_error("nlc exceeds RR_MAX_LC"); return RR_ELIMIT; }
    if (!lcids && nlc != 1) { set_error("lcids may be NULL only when nlc == 1"); return RR_EINVAL; }
    LcInfo lc = {};
    lc.nlc = nlc;
    for (int i = 0; i < RR_MAX_LC; ++i) {
        if (i < nlc) {
            if (pbids[i] < 0 || pbids[i] >= s->t->npb) { set_error("pbids entry outside [0, npb)"); return RR_EINVAL; }
            if (nss[i] < 1) { set_error("nss entries must be >= 1"); return RR_EINVAL; }
            if (nss[i] > RR_MAX_NSS) { set_error("nss entry exceeds RR_MAX_NSS"); return RR_ELIMIT; }
            if (!(exptimes[i] >= 0.0) || !std::isfinite(exptimes[i])) { set_error("exptimes must be finite and >= 0"); return RR_EINVAL; }
            lc.pb[i] = pbids[i]; lc.nss[i] = nss[i]; lc.exptime[i] = exptimes[i];
        } else {
            lc.pb[i] = 0; lc.nss[i] = 1; lc.exptime[i] = 0.0;
        }
    }
    Series se;
    se.npt = npt;
    for (int32_t i = 0; i < npt; ++i) {
        const int32_t l = lcids ? lcids[i] : 0;
        se.nsub += (l >= 0 && l < nlc) ? lc.nss[l] : 0;
    }
    se.ntiles = (npt + kFwdTile - 1) / kFwdTile;
    for (int32_t i = 0; i < nlc; ++i) se.max_nss = std::max(se.max_nss, lc.nss[i]);
    hipError_t e = hipMalloc((void**)&se.times, sizeof(double) * npt);
    if (e == hipSuccess && lcids) e = hipMalloc((void**)&se.lcids, sizeof(int32_t) * npt);
    if (e == hipSuccess) e = hipMalloc((void**)&se.lc, sizeof(LcInfo));
    if (e == hipSuccess) e = hipMemcpy(se.times, times, sizeof(double) * npt, hipMemcpyHostToDevice);
    if (e == hipSuccess && lcids) e = hipMemcpy(se.lcids, lcids, sizeof(int32_t) * npt, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(se.lc, &lc, sizeof(LcInfo), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (se.times) (void)hipFree(se.times);
        if (se.lcids) (void)hipFree(se.lcids);
        if (se.lc) (void)hipFree(se.lc);
        return hip_fail(e, "series upload");
    }
    std::lock_guard<std::mutex> lk(s->mu);
    s->series.push_back(se);
    *series_id = int32_t(s->series.size() - 1);
    return RR_OK;
}

static int submit_impl(rr_server* s, int32_t series_id, const double* pv, int32_t npv,
                       int32_t npar, int32_t precision, void* out_host, void* out_dev,
                       int64_t* request_id) {
    if (!s || !request_id) { set_error("server or request_id is NULL"); return RR_EINVAL; }
    if (!pv || (!out_host && !out_dev)) { set_error("pv and out are required"); return RR_EINVAL; }
    if (npv < 1) { set_error("npv must be >= 1"); return RR_EINVAL; }
    if (npar != 6 + s->t->npb) { set_error("npar must equal 6 + npb of the tables"); return RR_EINVAL; }
    if (precision != RR_FP64 && precision != RR_MIXED) { set_error("bad precision"); return RR_EINVAL; }
    Request* r = new (std::nothrow) Request();
    if (!r) return RR_ENOMEM;
    int32_t npt = 0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (series_id < 0 || size_t(series_id) >= s->series.size()) {
            delete r;
            set_error("unknown series id");
            return RR_EINVAL;
        }
        r->se = s->series[series_id];
        npt = r->se.npt;
    }
    r->out_user = out_dev;
    r->bytes = s->footprint(npv, npar, npt, precision, out_dev != nullptr);
    if (r->bytes > s->budget) {
        delete r;
        set_error("request footprint exceeds the server's memory budget");
        return RR_ELIMIT;
    }
    // the copy-completion event serves host outputs only
    if (!out_dev && hipEventCreateWithFlags(&r->done_ev, hipEventDisableTiming) != hipSuccess) {
        delete r;
        return hip_fail(hipErrorUnknown, "hipEventCreate");
    }
    r->series = series_id;
    r->npv = npv;
    r->npar = npar;
    r->precision = precision;
    r->pv.assign(pv, pv + size_t(npv) * npar);
    r->out_host = out_host;
    r->out_bytes = size_t(npv) * npt * (precision == RR_FP64 ? 8 : 4);
    r->t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        r->id = s->next_id++;
        s->reqs[r->id] = r;
        s->incoming.push_back(r);
    }
    s->cv_work.notify_one();
    *request_id = r->id;
    return RR_OK;
}

RR_API int rr_server_submit(rr_server* s, int32_t series_id, const double* pv, int32_t npv,
                            int32_t npar, int32_t precision, void* out_host,
                            int64_t* request_id) {
    if (!out_host) { set_error("out is required"); return RR_EINVAL; }
    return submit_impl(s, series_id, pv, npv, npar, precision, out_host, nullptr, request_id);
}

RR_API int rr_server_submit_device(rr_server* s, int32_t series_id, const double* pv,
                                   int32_t npv, int32_t npar, int32_t precision, void* out_dev,
                                   int64_t* request_id) {
    if (!out_dev) { set_error("out is required"); return RR_EINVAL; }
    return submit_impl(s, series_id, pv, npv, npar, precision, nullptr, out_dev, request_id);
}

RR_API int rr_server_fail_next_tick(rr_server* s) {
    if (!s) { set_error("server is NULL"); return RR_EINVAL; }
    s->fail_next_tick.store(1);
    return RR_OK;
}

RR_API int rr_server_poll(rr_server* s, int64_t request_id, int32_t* status, double* latency_s) {
    if (!s) { set_error("server is NULL"); return RR_EINVAL; }
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(request_id);
    if (it == s->reqs.end()) return RR_ENOTFOUND;
    Request* r = it->second;
    const int err = r->err.load();
    if (status) *status = (err != RR_OK && r->state == kDone) ? err : r->state;
    if (latency_s) *latency_s = r->state == kDone ? r->t_done - r->t_submit : -1.0;
    return RR_OK;
}

RR_API int rr_server_wait(rr_server* s, int64_t request_id, double timeout_s, double* latency_s) {
    if (!s) { set_error("server is NULL"); return RR_EINVAL; }
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(request_id);
    if (it == s->reqs.end()) return RR_ENOTFOUND;
    Request* r = it->second;
    const bool done = s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s),
                                          [r] { return r->state == kDone; });
    if (!done) return RR_EBUSY;
    if (latency_s) *latency_s = r->t_done - r->t_submit;
    return r->err.load();
}

RR_API int rr_server_release(rr_server* s, int64_t request_id) {
    if (!s) { set_error("server is NULL"); return RR_EINVAL; }
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(request_id);
    if (it == s->reqs.end()) return RR_ENOTFOUND;
    if (it->second->state != kDone) { set_error("request still in flight"); return RR_EBUSY; }
    if (it->second->done_ev) (void)hipEventDestroy(it->second->done_ev);
    delete it->second;
    s->reqs.erase(it);
    return RR_OK;
}

RR_API int rr_server_stats(rr_server* s, int64_t* stats) {
    if (!s || !stats) { set_error("server or stats is NULL"); return RR_EINVAL; }
    std::lock_guard<std::mutex> lk(s->mu);
    stats[0] = s->completed;
    stats[1] = s->points;
    stats[2] = s->nticks;
    stats[3] = int64_t(s->incoming.size());
    stats[4] = s->last_error;
    return RR_OK;
}

RR_API void rr_server_destroy(rr_server* s) {
    if (!s) return;
    if (s->worker.joinable()) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stop = true;
        }
        s->cv_work.notify_all();
        s->worker.join();
    }
    for (auto& st : s->streams)
        if (st) (void)hipStreamDestroy(st);
    if (s->setup_stream) (void)hipStreamDestroy(s->setup_stream);
    if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
    if (s->setup_ev) (void)hipEventDestroy(s->setup_ev);
    for (hipEvent_t ev : s->tick_events) (void)hipEventDestroy(ev);
    for (auto& se : s->series) {
        if (se.times) (void)hipFree(se.times);
        if (se.lcids) (void)hipFree(se.lcids);
        if (se.lc) (void)hipFree(se.lc);
    }
    for (auto& kv : s->reqs) {
        if (kv.second->done_ev) (void)hipEventDestroy(kv.second->done_ev);
        delete kv.second;
    }
    if (s->arena_base) (void)hipFree(s->arena_base);
    delete s;
}

}  // extern "C"
