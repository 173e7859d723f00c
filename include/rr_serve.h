/*
 * rr_serve.h -- continuous-batching serving loop of librr.so.
 *
 * Serves many population light-curve evaluations (Sect. 3.4.4: populations
 * of parameter vectors as in MCMC sampling; Sect. 4.2: heterogeneous time
 * series) against LD tables and time series that stay resident on the
 * device.  Requests are admitted by device-memory footprint as arena space
 * frees up and their work is packed, together with that of every other
 * admitted request, into grouped launches, so requests that arrive while
 * others run overlap with them on the GPU.  Each request runs the same
 * kernel code as rr_evaluate; its result does not depend on what it was
 * batched with.  All functions are thread-safe.
 */
#ifndef RR_SERVE_H
#define RR_SERVE_H

#include "rr.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rr_server rr_server;   /* opaque, owned by the library */

/* Request status values of rr_server_poll (negative values are RR_E*). */
#define RR_REQ_QUEUED  0
#define RR_REQ_RUNNING 1
#define RR_REQ_DONE    2

/* Start a server on the current device over tables `t` (which must outlive
 * it).  budget_bytes (>= 1 MiB) of device memory are allocated once as the
 * request arena; a request needs about npv (8 npar + 160 + npt * 4 or 8)
 * bytes of it while in flight.  max_tick_blocks (>= 1) bounds the
 * workgroups (one wave64 over 512 times each) of one grouped launch;
 * smaller values favour
 * latency of small requests, larger ones throughput.  Starts a worker
 * thread. */
RR_API int rr_server_create(const rr_tables* t, int64_t budget_bytes,
                            int32_t max_tick_blocks, rr_server** out);

/* Register a time series (host arrays, same meaning and limits as the
 * time-series arguments of rr_evaluate, npt >= 1); it is copied to the
 * device now and stays resident until rr_server_destroy.  Synchronous. */
RR_API int rr_server_add_series(rr_server* s, const double* times,
                                const int32_t* lcids, int32_t npt,
                                const int32_t* pbids, const int32_t* nss,
                                const double* exptimes, int32_t nlc,
                                int32_t* series_id);

/* Queue a request: npv >= 1 parameter rows pv[npv][npar] (host, copied
 * before returning; npar == 6 + npb) against a registered series, in
 * RR_FP64 or RR_MIXED.  Fluxes are written to out_host[npv][npt] (double
 * or float), which must stay valid until the request is done; page-locked
 * memory makes the copy asynchronous.  RR_ELIMIT if the footprint exceeds
 * the whole budget.  The submission time starts the request's latency. */
RR_API int rr_server_submit(rr_server* s, int32_t series_id, const double* pv,
                            int32_t npv, int32_t npar, int32_t precision,
                            void* out_host, int64_t* request_id);

/* The same with the output written straight to out_dev[npv][npt] (double
 * or float by precision), a device buffer of the server's device that the
 * caller owns and must not read or free until the request is done; the
 * request's arena footprint then excludes the output (about npv (8 npar +
 * 160) bytes).  Done means the kernels that wrote out_dev have completed,
 * so any stream may read it afterwards.  This form measures the GPU side of
 * serving without the device-to-host copy of every result. */
RR_API int rr_server_submit_device(rr_server* s, int32_t series_id,
                                   const double* pv, int32_t npv, int32_t npar,
                                   int32_t precision, void* out_dev,
                                   int64_t* request_id);

/* Status (RR_REQ_*, or a negative error) and, once done, the latency in
 * seconds (submission to the output being in out_host, or to the kernels
 * that wrote out_dev having completed); -1 before. */
RR_API int rr_server_poll(rr_server* s, int64_t request_id, int32_t* status,
                          double* latency_s);

/* Block until the request is done or timeout_s passes (RR_EBUSY). */
RR_API int rr_server_wait(rr_server* s, int64_t request_id, double timeout_s,
                          double* latency_s);

/* Forget a finished request (its id becomes unknown); RR_EBUSY while it is
 * still in flight.  Safe from any thread as soon as the request is done: the
 * server keeps no reference to a request once its last rows have launched
 * beyond the completion that marks it done. */
RR_API int rr_server_release(rr_server* s, int64_t request_id);

/* stats[0..4] = completed requests, completed light-curve points
 * (npv x sum over times of nss), grouped launches issued, requests not yet
 * seen by the worker, last device error (0 if none). */
RR_API int rr_server_stats(rr_server* s, int64_t* stats);

/* Test instrumentation of the failure path: the next grouped launch is
 * not made and is treated as failed on the host (no kernel is involved);
 * the requests it covered finish with RR_EDEVICE and the server keeps
 * serving the others. */
RR_API int rr_server_fail_next_tick(rr_server* s);

/* Finish all queued and running requests, then free the server. */
RR_API void rr_server_destroy(rr_server* s);

#ifdef __cplusplus
}
#endif

#endif /* RR_SERVE_H */
