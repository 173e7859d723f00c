#!/usr/bin/env python3
"""Throughput benchmark of the RoadRunner light-curve path on one MI355X.

Workload: the population evaluation: 512 parameter vectors drawn from a
fixed seed (k ~ U(0.05, 0.2), a ~ U(5, 20), b ~ U(0, 0.9), e ~ U(0, 0.3),
w ~ U(0, 2 pi), P ~ U(1, 10) d, t0 ~ U(0, P)) over 20 000 times at 2-min
cadence (27.8 d), one power-2 limb-darkening profile tabulated at 200 mu,
no supersampling, default table grid.  One step is one rr_evaluate call
(per-vector setup kernel + forward kernel) over the whole population with
inputs and tables resident in HBM.  The mixed-precision path (FP64 time
reduction, FP32 bulk) gives the headline value; the FP64 path is timed the
same way and reported beside it.

Prints one JSON line.  --gpus above 1 exits with a message: this benchmark
measures one GPU.
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "light-curve points/s (npv×npt×nss) FP32 vs FP64 at 1 ppm; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
PVCONST_BYTES = 144


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="budget of the CPU-oracle baseline leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--serving-burst", type=int, default=300)
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the heterogeneous-series and log-likelihood legs")
    ap.add_argument("--legs", default="heterogeneous,per_vector_ld,direct,small_planet,"
                                      "variants,loglik",
                    help="comma-separated extra legs to run (unless --no-extra)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy --steps times "
                         "(the reference kernel for scaling HBM byte counters)")
    return ap.parse_args()


def source_hash():
    h = hashlib.sha256()
    for f in ("rr_forward.hip", "rr_device.h", "rr_internal.h"):
        with open(os.path.join(ROOT, "paper_2009_08500_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


VALU_LANE_SLOTS = 256 * 4 * 16 * 2.4e9   # CUs x SIMDs x lanes x clock: wave64 takes 4 cycles


def profile_counters(kernel):
    """Per-launch counters of `kernel` from the committed PMC summary, if it
    was taken on the current kernel sources; otherwise None."""
    path = os.path.join(ROOT, "profiles", "forward_population_counters.json")
    try:
        with open(path) as fh:
            prof = json.load(fh)
    except (OSError, ValueError):
        return None
    if prof.get("source_hash") != source_hash():
        return None
    return prof.get("kernels", {}).get(kernel)


def valu_view(kernel, kernel_ms):
    """Issued VALU lane-slots per launch (SQ_INSTS_VALU x 64) against the
    chip's VALU issue rate over the event-timed kernel duration."""
    k = profile_counters(kernel)
    if not k or "SQ_INSTS_VALU" not in k:
        return None
    slots = 64.0 * k["SQ_INSTS_VALU"]
    v = dict(valu_instrs_per_launch=k["SQ_INSTS_VALU"], lane_slots_per_launch=slots,
             peak_lane_slots_per_s=VALU_LANE_SLOTS,
             issue_frac=slots / (kernel_ms * 1e-3) / VALU_LANE_SLOTS)
    if "fp32_flop_per_launch" in k:
        # upper bounds (all 64 lanes counted); peaks: unpacked FP32 and FP64 vector
        v["fp32_tflops"] = k["fp32_flop_per_launch"] / (kernel_ms * 1e-3) / 1e12
        v["fp64_tflops"] = k["fp64_flop_per_launch"] / (kernel_ms * 1e-3) / 1e12
        v["fp32_peak_tflops"] = 78.6
        v["fp64_peak_tflops"] = 78.6
    return v


def time_path(rr, tab, series, pv, prec, steps, warmup, lib):
    """Throughput: `steps` back-to-back evaluations between two
    synchronisations (no per-step instrumentation), first as eager calls
    from Python, then as replays of one call captured in a HIP graph
    (Evaluator.capture: the same setup and forward kernels, without the
    host's per-call launch work).  Then the same number of eager calls again
    with HIP events around each call, for latency percentiles, and, through
    rr_set_kernel_events, as the forward kernel launch's own start and stop
    events, for the kernel time.  Returns (eager wall, graph wall, step ms,
    kernel ms, output)."""
    import torch
    ev_fn = rr.Evaluator(tab, series, pv.shape[0], prec)
    for _ in range(warmup):
        ev_fn(pv)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ev_fn(pv)
    torch.cuda.synchronize()
    wall_eager = time.perf_counter() - t0
    ev_g = rr.Evaluator(tab, series, pv.shape[0], prec)
    ev_g.capture(pv)
    for _ in range(warmup):
        ev_g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ev_g.replay()
    torch.cuda.synchronize()
    wall_graph = time.perf_counter() - t0
    if not torch.equal(ev_g.out, ev_fn.out):
        raise RuntimeError("graph replay and eager call disagree")
    step_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(steps)]
    kern_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(steps)]
    for a, b in kern_ev:          # materialise the event handles
        a.record()
        b.record()
    torch.cuda.synchronize()
    for i in range(steps):
        step_ev[i][0].record()
        lib.rr_set_kernel_events(kern_ev[i][0].cuda_event, kern_ev[i][1].cuda_event)
        ev_fn(pv)
        step_ev[i][1].record()
    torch.cuda.synchronize()
    lib.rr_set_kernel_events(None, None)
    step_ms = [a.elapsed_time(b) for a, b in step_ev]
    kern_ms = [a.elapsed_time(b) for a, b in kern_ev]
    return wall_eager, wall_graph, step_ms, kern_ms, ev_fn.out


def pct(x, q):
    import numpy as np
    return float(np.percentile(np.asarray(x), q))


_POOL_STATE = {}


def _pool_rows(args):
    """Worker of the N-core oracle leg: the oracle on one chunk of rows,
    single-threaded (the tables come with the forked process)."""
    from threadpoolctl import threadpool_limits
    from oracle import roadrunner as orr
    r0, r1 = args
    st = _POOL_STATE
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        orr.evaluate(st["otab"], st["times"], st["pv"][r0:r1])
        return r1 - r0, time.perf_counter() - t0


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, grid, budget_s, gpu_out64, gpu_out32):
    """The FP64 oracle, untuned, on the host: whole population passes over
    parameter-row chunks until the time budget is used, first on one core,
    then on N cores (a pool of N forked worker processes over row chunks,
    N = the host cores given to this GPU, at most 16).  Tables are built
    outside the timed region, as on the GPU side."""
    import multiprocessing as mp
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import roadrunner as orr
    otab = orr.Tables(w["mu_s"], w["I_s"], **grid)
    npv = w["pv"].shape[0]
    chunk = 32
    done_rows = 0
    t_used = 0.0
    d64, d32, intr = [], [], []           # |GPU - oracle| per point, first pass
    with threadpool_limits(limits=1):
        while t_used < budget_s:
            r0 = done_rows % npv
            rows = slice(r0, min(npv, r0 + chunk))
            t0 = time.perf_counter()
            ref = orr.evaluate(otab, w["times"], w["pv"][rows])
            t_used += time.perf_counter() - t0
            done_rows += ref.shape[0]
            if done_rows <= npv:
                d64.append(np.abs(gpu_out64[rows] - ref).ravel())
                d32.append(np.abs(gpu_out32[rows] - ref).ravel())
                intr.append((ref < 1.0).ravel())
    pts = done_rows * w["times"].size
    single = dict(value=pts / t_used, unit="points/s", cores=1,
                  sample=f"{done_rows} rows x {w['times'].size} times, {t_used:.1f} s")
    # N cores: fork (no exec) after the tables are built; workers use no GPU
    ncores = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
                        else (os.cpu_count() or 1)))
    _POOL_STATE.update(otab=otab, times=w["times"], pv=w["pv"])
    jobs = [(r0, min(npv, r0 + 8)) for r0 in range(0, npv, 8)]
    ctx = mp.get_context("fork")
    rows_done, t_wall = 0, 0.0
    with ctx.Pool(ncores) as pool:
        while t_wall < budget_s:
            t0 = time.perf_counter()
            for n, _ in pool.imap_unordered(_pool_rows, jobs):
                rows_done += n
            t_wall += time.perf_counter() - t0
    pts_n = rows_done * w["times"].size
    sample = (f"{rows_done} parameter rows of the same population (chunks of 8 rows over "
              f"{ncores} forked single-threaded workers, whole passes over all {npv} rows) x "
              f"{w['times'].size} times, {t_wall:.1f} s wall; one core: {single['sample']}")
    d64, d32, intr = np.concatenate(d64), np.concatenate(d32), np.concatenate(intr)

    def stats(d, scale):
        out = {}
        for name, m in (("in_transit", intr), ("out_of_transit", ~intr)):
            x = d[m] * scale
            out[name] = (dict(points=int(m.sum()), max=float(x.max()), p99=float(np.percentile(x, 99)),
                              mean=float(x.mean())) if m.any() else dict(points=0))
        return out

    acc = dict(rows_checked=min(done_rows, npv), max_abs_err_fp64=float(d64.max()),
               max_abs_err_mixed_ppm=float(d32.max()) * 1e6,
               fp64_abs=stats(d64, 1.0), mixed_ppm=stats(d32, 1e6))
    return dict(value=pts_n / t_wall, unit="points/s", cores=ncores, kind="oracle",
                sample=sample, cpu_model=cpu_model(), single_core=single), acc


def heterogeneous_leg(rr, wl, steps, warmup, lib):
    """Four passbands with their own profiles and chromatic k, two 30-min
    light curves with nss = 10 and two 2-min ones with nss = 1 over 27 d,
    256 rows: subsamples/s for both precisions, and the error of every
    output against the oracle (same grid)."""
    import numpy as np
    import torch
    from oracle import roadrunner as orr
    w = wl.heterogeneous(npv=256)
    grid = wl.DEFAULT_GRID
    tab = rr.Tables(w["mu_s"], w["I_s"], grid)
    ser = rr.TimeSeries(w["times"], w["lcids"], w["pbids"], w["nss"], w["exptimes"])
    pv = torch.as_tensor(w["pv"], device="cuda")
    npv = pv.shape[0]
    subs = npv * int(np.sum(w["nss"][w["lcids"]]))
    res = dict(workload="heterogeneous: 256 rows, 4 passbands, 2 x 30-min LCs (nss 10) + "
                        "2 x 2-min LCs (nss 1) over 27 d", npv=npv, npt=int(w["times"].size),
               subsamples_per_call=subs)
    outs = {}
    for prec in ("mixed", "fp64"):
        wall, wall_graph, step_ms, kern_ms, out = time_path(rr, tab, ser, pv, prec, steps,
                                                            warmup, lib)
        ms = 1e3 * wall / steps
        res[prec] = dict(subsamples_per_s=subs / (ms / 1e3), ms_per_step=ms,
                         graph_replay_ms_per_step=1e3 * wall_graph / steps,
                         kernel_ms=float(np.mean(kern_ms)),
                         latency_ms=dict(p50=pct(step_ms, 50), p99=pct(step_ms, 99)))
        outs[prec] = out.cpu().numpy().astype(np.float64)
    otab = orr.Tables(w["mu_s"], w["I_s"], **grid)
    ref = orr.evaluate(otab, w["times"], w["pv"], lcids=w["lcids"], pbids=w["pbids"],
                       nss=w["nss"], exptimes=w["exptimes"])
    res["accuracy_vs_oracle"] = dict(rows_checked=npv,
                                     max_abs_err_fp64=float(np.abs(outs["fp64"] - ref).max()),
                                     max_abs_err_mixed_ppm=float(np.abs(outs["mixed"] - ref).max()) * 1e6)
    return res


def per_vector_ld_leg(rr, wl, steps, warmup, lib):
    """The population (512 x 20 000, nss 1) with a power-2 LD profile of its
    own for every row (rr_evaluate_ld): points/s and per-call latency for
    both precisions, the forward kernel's own time (launch events), and the
    error of eight sampled rows against the oracle."""
    import numpy as np
    import torch
    from oracle import roadrunner as orr
    w = wl.population_ld()
    grid = wl.DEFAULT_GRID
    tab = rr.Tables(w["mu_s"], w["I_s"], grid)
    ser = rr.TimeSeries(w["times"])
    pv = torch.as_tensor(w["pv"], device="cuda")
    prof = torch.as_tensor(w["prof_pv"], device="cuda")
    npv, npt = pv.shape[0], int(w["times"].size)
    res = dict(workload=f"population with per-vector power-2 LD: npv={npv} npt={npt} nss=1, "
                        "profiles at 200 mu", npv=npv, npt=npt)
    outs = {}
    for prec in ("mixed", "fp64"):
        dtype = torch.float64 if prec == "fp64" else torch.float32
        out = torch.empty((npv, npt), dtype=dtype, device="cuda")
        for _ in range(warmup):
            rr.evaluate_ld(tab, ser, pv, prof, prec, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            rr.evaluate_ld(tab, ser, pv, prof, prec, out=out)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        step_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                   for _ in range(steps)]
        kern_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                   for _ in range(steps)]
        for a, b in kern_ev:
            a.record()
            b.record()
        torch.cuda.synchronize()
        for i in range(steps):
            step_ev[i][0].record()
            lib.rr_set_kernel_events(kern_ev[i][0].cuda_event, kern_ev[i][1].cuda_event)
            rr.evaluate_ld(tab, ser, pv, prof, prec, out=out)
            step_ev[i][1].record()
        torch.cuda.synchronize()
        lib.rr_set_kernel_events(None, None)
        step_ms = [a.elapsed_time(b) for a, b in step_ev]
        kern_ms = [a.elapsed_time(b) for a, b in kern_ev]
        res[prec] = dict(points_per_s=npv * npt / (ms / 1e3), ms_per_step=ms,
                         forward_kernel_ms=float(np.mean(kern_ms)),
                         latency_ms=dict(p50=pct(step_ms, 50), p99=pct(step_ms, 99)))
        outs[prec] = out.cpu().numpy().astype(np.float64)
    rows = np.random.default_rng(9).choice(npv, 8, replace=False)
    otab = orr.Tables(w["mu_s"], w["I_s"], **grid)
    ref = orr.evaluate_ld(otab, w["times"], w["pv"][rows], w["prof_pv"][rows])
    res["accuracy_vs_oracle"] = dict(
        rows_checked=len(rows),
        max_abs_err_fp64=float(np.abs(outs["fp64"][rows] - ref).max()),
        max_abs_err_mixed_ppm=float(np.abs(outs["mixed"][rows] - ref).max()) * 1e6)
    return res


def direct_leg(rr, wl, steps, warmup):
    """The population (512 x 20 000, nss 1) through the direct model
    (rr_evaluate_direct: weights for each row's own k): points/s and
    per-call latency for both precisions, and the error of eight sampled
    rows against the oracle's direct model."""
    import numpy as np
    import torch
    from oracle import roadrunner as orr
    w = wl.population()
    grid = wl.DEFAULT_GRID
    tab = rr.Tables(w["mu_s"], w["I_s"], grid)
    ser = rr.TimeSeries(w["times"])
    pv = torch.as_tensor(w["pv"], device="cuda")
    npv, npt = pv.shape[0], int(w["times"].size)
    res = dict(workload=f"population through the direct model: npv={npv} npt={npt} nss=1",
               npv=npv, npt=npt)
    outs = {}
    for prec in ("mixed", "fp64"):
        dtype = torch.float64 if prec == "fp64" else torch.float32
        out = torch.empty((npv, npt), dtype=dtype, device="cuda")
        for _ in range(warmup):
            rr.evaluate_direct(tab, ser, pv, prec, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            rr.evaluate_direct(tab, ser, pv, prec, out=out)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        res[prec] = dict(points_per_s=npv * npt / (ms / 1e3), ms_per_step=ms)
        outs[prec] = out.cpu().numpy().astype(np.float64)
    rows = np.random.default_rng(10).choice(npv, 8, replace=False)
    otab = orr.Tables(w["mu_s"], w["I_s"], **grid)
    ref = orr.evaluate_direct(otab, w["times"], w["pv"][rows])
    res["accuracy_vs_oracle"] = dict(
        rows_checked=len(rows),
        max_abs_err_fp64=float(np.abs(outs["fp64"][rows] - ref).max()),
        max_abs_err_mixed_ppm=float(np.abs(outs["mixed"][rows] - ref).max()) * 1e6)
    return res


def small_planet_leg(rr, wl, steps, warmup):
    """Small planets (512 x 20 000, nss 1, k ~ logU(0.003, 0.03)) through
    the small-planet approximation with threshold 0.01
    (rr_evaluate_small_planet): points/s and per-call latency for both
    precisions, the same population through the interpolated model for
    comparison (rows below the tables' k0 are NaN there, so it is timed with
    k raised to 0.01), the log-likelihood with its parameter gradient
    (rr_loglik_grad_small_planet), and the error of eight sampled rows
    against the oracle."""
    import numpy as np
    import torch
    from oracle import roadrunner as orr
    w = wl.population_small()
    grid = wl.DEFAULT_GRID
    tab = rr.Tables(w["mu_s"], w["I_s"], grid)
    ser = rr.TimeSeries(w["times"])
    pv = torch.as_tensor(w["pv"], device="cuda")
    pv_tab = pv.clone()
    pv_tab[:, 6] = pv_tab[:, 6].clamp(min=grid["k0"])
    npv, npt = pv.shape[0], int(w["times"].size)
    nsmall = int((w["pv"][:, 6] < 0.01).sum())
    res = dict(workload=f"small planets: npv={npv} npt={npt} nss=1, k ~ logU(0.003, 0.03), "
                        f"threshold 0.01 ({nsmall} vectors below)", npv=npv, npt=npt)

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / steps

    outs = {}
    for prec in ("mixed", "fp64"):
        dtype = torch.float64 if prec == "fp64" else torch.float32
        out = torch.empty((npv, npt), dtype=dtype, device="cuda")
        ms = timed(lambda: rr.evaluate_small_planet(tab, ser, pv, 0.01, prec, out=out))
        outs[prec] = out.cpu().numpy().astype(np.float64)
        ms_tab = timed(lambda: rr.evaluate(tab, ser, pv_tab, prec, out=out))
        # log-likelihood and parameter gradient of the same rows against the
        # first row's light curve plus 200 ppm of seeded noise
        noise = torch.as_tensor(np.random.default_rng(12).normal(0.0, 2e-4, npt), device="cuda")
        obs = (torch.as_tensor(outs[prec][0], device="cuda") + noise).to(out.dtype)
        ms_ll = timed(lambda: rr.loglik_grad_small_planet(tab, ser, pv, obs, 2e-4, 0.01, prec))
        res[prec] = dict(points_per_s=npv * npt / (ms / 1e3), ms_per_step=ms,
                         interpolated_model_ms=ms_tab, loglik_grad_ms=ms_ll)
    rows = np.random.default_rng(11).choice(npv, 8, replace=False)
    otab = orr.Tables(w["mu_s"], w["I_s"], **grid)
    ref = orr.evaluate_small_planet(otab, w["times"], w["pv"][rows], 0.01)
    res["accuracy_vs_oracle"] = dict(
        rows_checked=len(rows),
        max_abs_err_fp64=float(np.abs(outs["fp64"][rows] - ref).max()),
        max_abs_err_mixed_ppm=float(np.abs(outs["mixed"][rows] - ref).max()) * 1e6)
    return res


def variant_leg(rr, wl):
    """Trial-run selection of the forward-kernel variant (rr_select_variant)
    on three workloads: the population, a small problem (32 x 2000) and the
    heterogeneous four-passband series; the mean time per forward launch of
    each variant (4/8/16 exposures per lane; subsamples spread or one lane
    per exposure) and the one chosen."""
    import torch
    res = {}
    w = wl.population()
    cases = [("population 512 x 20000", w, rr.TimeSeries(w["times"]), w["pv"]),
             ("small 32 x 2000", w, rr.TimeSeries(w["times"][:2000]), w["pv"][:32])]
    wh = wl.heterogeneous()
    cases.append(("heterogeneous 256 x 41472 (nss 10/1)", wh,
                  rr.TimeSeries(wh["times"], wh["lcids"], wh["pbids"], wh["nss"],
                                wh["exptimes"]), wh["pv"]))
    for name, wk, ser, pv in cases:
        tab = rr.Tables(wk["mu_s"], wk["I_s"], wl.DEFAULT_GRID)
        pvd = torch.as_tensor(pv, device="cuda")
        res[name] = {}
        for prec in ("mixed", "fp64"):
            best, ms = rr.select_variant(tab, ser, pvd, prec, reps=20)
            res[name][prec] = dict(best=best, us_per_variant=[round(1e3 * m, 2) for m in ms])
    return res


def loglik_leg(rr, wl, steps, warmup):
    """Gaussian log-likelihood and its adjoint for 1024 walkers around a truth
    vector, 50 000 times at 2-min cadence with nss = 5 (data = the oracle's
    light curve at the truth + seeded 200 ppm noise): subsamples/s of
    rr_loglik_grad (logL and the parameter gradients) for both precisions,
    the time of a full autograd step through the power-2 LD coefficients,
    and the errors of 16 walkers against the oracle's analytic gradient."""
    import numpy as np
    import torch
    from oracle import gradient as ogr
    from oracle import roadrunner as orr
    w = wl.loglik_walkers()
    grid = wl.DEFAULT_GRID
    otab = orr.Tables(w["mu_s"], w["I_s"], **grid)
    obs = orr.evaluate(otab, w["times"], w["truth"][None, :], nss=w["nss"],
                       exptimes=w["exptimes"])[0] + w["noise"]
    tab = rr.Tables(w["mu_s"], w["I_s"], grid)
    ser = rr.TimeSeries(w["times"], nss=w["nss"], exptimes=w["exptimes"])
    pv = torch.as_tensor(w["pv"], device="cuda")
    npv = pv.shape[0]
    subs = npv * int(w["times"].size) * int(w["nss"][0])
    res = dict(workload="log-likelihood + gradient: 1024 walkers, 50 000 times at 2 min, nss 5",
               npv=npv, npt=int(w["times"].size), nss=int(w["nss"][0]),
               subsamples_per_call=subs)
    nchk = 16
    for prec in ("mixed", "fp64"):
        obs_d = torch.as_tensor(obs, device="cuda",
                                dtype=torch.float64 if prec == "fp64" else torch.float32)
        for _ in range(warmup):
            rr.loglik_grad(tab, ser, pv, obs_d, w["sigma"], prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ll, g, _ = rr.loglik_grad(tab, ser, pv, obs_d, w["sigma"], prec)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        ll, g = ll.cpu().numpy(), g.cpu().numpy()
        obs_in = obs if prec == "fp64" else obs.astype(np.float32).astype(np.float64)
        oll, og, _ = ogr.loglik_grad(otab, w["times"], w["pv"][:nchk], obs_in, w["sigma"],
                                     nss=w["nss"], exptimes=w["exptimes"], want_profile=False)
        scale = np.abs(og).max(axis=1, keepdims=True)
        res[prec] = dict(subsamples_per_s=subs / (ms / 1e3), ms_per_step=ms,
                         walkers_checked=nchk,
                         max_rel_err_logl=float(np.max(np.abs(ll[:nchk] - oll) / np.abs(oll))),
                         max_rel_err_grad=float(np.max(np.abs(g[:nchk] - og) / scale)))
    # one autograd step: profile from (c, alpha) in torch -> logL -> backward
    mu = torch.as_tensor(w["mu_s"], device="cuda")
    pos = mu > 0
    logmu = torch.log(torch.where(pos, mu, torch.ones_like(mu)))
    c = torch.tensor(w["ld_c"], device="cuda", dtype=torch.float64, requires_grad=True)
    al = torch.tensor(w["ld_alpha"], device="cuda", dtype=torch.float64, requires_grad=True)
    pvg = pv.clone().requires_grad_(True)
    obs_d = torch.as_tensor(obs, device="cuda", dtype=torch.float32)

    def step():
        mu_al = torch.where(pos, torch.exp(al * logmu), torch.zeros_like(mu))
        prof = (1.0 - c * (1.0 - mu_al))[None, :]
        ll = rr.RRLogLik.apply(pvg, prof, tab, ser, obs_d, w["sigma"], "mixed")
        ll.sum().backward()

    for _ in range(2):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(max(2, steps // 2)):
        step()
    torch.cuda.synchronize()
    res["autograd_step_ms_mixed"] = 1e3 * (time.perf_counter() - t0) / max(2, steps // 2)
    # the same walkers with a power-2 profile each (rr_loglik_grad_ld), with
    # the gradient with respect to every walker's profile
    rng = np.random.default_rng(31)
    cw = w["ld_c"] * (1.0 + 0.01 * rng.standard_normal(npv))
    aw = w["ld_alpha"] * (1.0 + 0.01 * rng.standard_normal(npv))
    prof_pv = torch.as_tensor(
        (1.0 - cw[:, None] * (1.0 - w["mu_s"][None, :] ** aw[:, None]))[:, None, :],
        device="cuda")
    per_row = {}
    for prec in ("mixed", "fp64"):
        obs_d = torch.as_tensor(obs, device="cuda",
                                dtype=torch.float64 if prec == "fp64" else torch.float32)
        for _ in range(warmup):
            rr.loglik_grad_ld(tab, ser, pv, prof_pv, obs_d, w["sigma"], prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            rr.loglik_grad_ld(tab, ser, pv, prof_pv, obs_d, w["sigma"], prec)
        torch.cuda.synchronize()
        per_row[prec] = dict(ms_per_step=1e3 * (time.perf_counter() - t0) / steps)
    res["per_walker_ld_with_profile_gradients"] = per_row
    return res


class _Ring:
    """First-in, first-out allocator over one preallocated byte buffer (page-
    locked host or device memory), so that the serving protocol allocates
    nothing per request: requests take their outputs from it in submission
    order and give them back in the same order once done."""

    def __init__(self, nbytes, device):
        import threading
        import torch
        self.size = int(nbytes)
        self.buf = (torch.empty(self.size, dtype=torch.uint8, device="cuda") if device
                    else torch.empty(self.size, dtype=torch.uint8, pin_memory=True))
        self.live = []            # (start, end) in allocation order
        self.head = 0
        self.lock = threading.Lock()

    def alloc(self, nbytes):
        n = (int(nbytes) + 255) // 256 * 256
        with self.lock:
            if not self.live:
                self.head = 0
            tail = self.live[0][0] if self.live else 0
            if not self.live or self.head > tail:
                if self.head + n <= self.size:
                    start = self.head
                elif n <= tail:
                    start = 0
                else:
                    return None
            else:
                if self.head + n <= tail:
                    start = self.head
                else:
                    return None
            self.live.append((start, start + n))
            self.head = start + n
            return start

    def free_oldest(self):
        with self.lock:
            self.live.pop(0)

    def view(self, start, npv, npt, dtype):
        import torch
        nb = npv * npt * (8 if dtype is torch.float64 else 4)
        return self.buf[start:start + nb].view(dtype).view(npv, npt)


def serving_leg(rr, wl, nreq, nburst):
    """Serving protocol: requests each with their own resident time series
    (npt ~ logU(1e3, 1e5), nss in {1, 5, 10}, 1-4 passbands split evenly
    into 2-min light curves) and npv ~ logU(1, 2048) rows, against resident
    tables of four passbands.  For each precision and output mode (device
    buffer; page-locked host buffer) a burst of `nburst` requests submitted
    at once gives the saturated request rate, then the same `nreq` requests
    arrive as a Poisson stream at 0.5 and at 0.9 times that rate.  Outputs
    come from preallocated ring buffers, so nothing is allocated per
    request.  Latency is the server's (submission to the kernels that wrote
    the output having completed, or to the output being in host memory);
    `submit_lag` is how late the submitting thread was against the drawn
    arrival times."""
    import queue
    import threading
    import numpy as np
    import torch
    het = wl.heterogeneous(npv=1)
    tab = rr.Tables(het["mu_s"], het["I_s"], wl.DEFAULT_GRID)
    series, reqs = wl.serving_stream(nreq)
    srv = rr.Server(tab, budget_bytes=16 << 30, max_tick_blocks=32768)
    t_reg = time.perf_counter()
    sids = [srv.add_series(se["times"], se["lcids"], se["pbids"], se["nss"], se["exptimes"])
            for se in series]
    t_reg = time.perf_counter() - t_reg
    nsub = [int(np.sum(se["nss"][se["lcids"]])) for se in series]
    npts = [int(se["times"].size) for se in series]
    work = np.array([r["pv"].shape[0] * nsub[r["series"]] for r in reqs], dtype=np.float64)
    rings = {True: _Ring(8 << 30, True), False: _Ring(8 << 30, False)}
    res = dict(
        workload="Poisson streams of requests, each with its own series: npv~logU(1,2048), "
                 "npt~logU(1e3,1e5), nss in {1,5,10}, 1-4 passbands; resident tables and series",
        requests_per_stream=nreq, burst_requests=nburst, series_registered=len(series),
        series_registration_s=t_reg, mean_points_per_request=float(np.mean(work)),
        max_points_per_request=float(np.max(work)))

    def run(prec, device, idx, gaps):
        """Submit requests `idx` (after the given gaps, or all at once) and
        wait for them in order on a second thread.  Returns (elapsed s,
        latencies s, submit lags s, ring stalls)."""
        dtype = torch.float64 if prec == "fp64" else torch.float32
        ring = rings[device]
        q = queue.Queue()
        lat = []

        def waiter():
            while True:
                h = q.get()
                if h is None:
                    return
                srv.wait(h, timeout=300.0)
                lat.append(h.latency)
                srv.release(h)
                h.out = None
                ring.free_oldest()

        th = threading.Thread(target=waiter)
        th.start()
        lags, stalls = [], 0
        t0 = time.perf_counter()
        due = t0
        for k, i in enumerate(idx):
            r = reqs[i]
            npv, npt = r["pv"].shape[0], npts[r["series"]]
            if gaps is not None:
                due += gaps[k]
                d = due - time.perf_counter()
                if d > 0:
                    time.sleep(d)
            while True:
                off = ring.alloc(npv * npt * (8 if prec == "fp64" else 4))
                if off is not None:
                    break
                stalls += 1
                time.sleep(50e-6)
            out = ring.view(off, npv, npt, dtype)
            if gaps is not None:
                lags.append(time.perf_counter() - due)
            q.put(srv.submit(sids[r["series"]], r["pv"], prec, device_out=device, out=out))
        q.put(None)
        th.join()
        return time.perf_counter() - t0, lat, lags, stalls

    rng = np.random.default_rng(2009085004)
    unit = rng.exponential(1.0, nreq)                  # the same arrival pattern, scaled
    # The submitting and the waiting thread share the interpreter lock; with
    # the default 5 ms switch interval one of them can hold it through many
    # requests while the other waits, which made the burst's rate swing
    # between runs.  A short interval keeps the two alternating.
    switch = sys.getswitchinterval()
    sys.setswitchinterval(1e-4)
    for prec in ("mixed", "fp64"):
        for device in (True, False):
            key = f"{prec}_{'device' if device else 'host'}_output"
            # untimed warm-up over the same requests: the first pass grows the
            # server's and the rings' memory, which the timed burst must not see
            run(prec, device, range(nburst), None)
            el, _, _, _ = run(prec, device, range(nburst), None)
            sat = nburst / el
            entry = dict(saturated_requests_per_s=sat,
                         saturated_points_per_s=float(np.sum(work[:nburst])) / el)
            for frac in (0.5, 0.9):
                rate = frac * sat
                el, lat, lags, stalls = run(prec, device, range(nreq), unit / rate)
                entry[f"rate_{frac}"] = dict(
                    arrival_rate_per_s=rate, points_per_s=float(np.sum(work[:nreq])) / el,
                    latency_ms=dict(p50=1e3 * float(np.percentile(lat, 50)),
                                    p99=1e3 * float(np.percentile(lat, 99)),
                                    max=1e3 * float(np.max(lat))),
                    submit_lag_ms_p99=1e3 * float(np.percentile(lags, 99)),
                    ring_stalls=stalls)
            res[key] = entry
            print(f"serving {key}: " + json.dumps(entry), file=sys.stderr, flush=True)
    sys.setswitchinterval(switch)
    st = srv.stats()
    res["grouped_launches"] = st["ticks"]
    res["device_errors"] = st["last_error"]
    srv.close()
    tab.close()
    return res


def single_lc_leg(rr, wl, steps, warmup):
    """One light curve, the smallest call (npv 1, 1000 times, circular orbit,
    quadratic LD at 100 mu, no supersampling): microseconds per call, as
    throughput of back-to-back calls and as per-call latency percentiles
    (HIP events around each call); latency-bound, not a throughput figure."""
    import numpy as np
    import torch
    w = wl.single_light_curve()
    tab = rr.Tables(w["mu_s"], w["I_s"], wl.DEFAULT_GRID)
    ser = rr.TimeSeries(w["times"])
    pv = torch.as_tensor(w["pv"], device="cuda")
    res = dict(workload="single light curve: npv 1, npt 1000, circular, quadratic LD, nss 1")
    for prec in ("fp64", "mixed"):
        ev = rr.Evaluator(tab, ser, 1, prec)
        for _ in range(warmup):
            ev(pv)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ev(pv)
        torch.cuda.synchronize()
        us = 1e6 * (time.perf_counter() - t0) / steps
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(steps)]
        for a, b in evs:
            a.record()
            ev(pv)
            b.record()
        torch.cuda.synchronize()
        lat = [1e3 * a.elapsed_time(b) for a, b in evs]
        res[prec] = dict(us_per_call=us, latency_us=dict(p50=pct(lat, 50), p99=pct(lat, 99)))
    return res


def note(msg):
    """A progress line on stderr (stdout carries only the result line)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: every run here has a single MI355X; "
              "the path would shard over parameter vectors (one slice per GPU, "
              "tables replicated; only gradients with respect to the shared profile "
              "would be summed across GPUs).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2009_08500_amd as rr
    import workloads as wl

    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps(dict(copy_bytes_read=src.numel() * 4, copy_bytes_written=dst.numel() * 4,
                              launches=args.steps)), flush=True)
        return
    lib = rr.lib()
    note("library loaded; population workload")
    w = wl.population()
    grid = wl.DEFAULT_GRID
    npv, npt = w["pv"].shape[0], w["times"].size
    nss = 1
    tab = rr.Tables(w["mu_s"], w["I_s"], grid)
    series = rr.TimeSeries(w["times"])
    pv = torch.as_tensor(w["pv"], device="cuda")

    res = {}
    outs = {}
    for prec in ("mixed", "fp64"):
        wall, wall_graph, step_ms, kern_ms, out = time_path(rr, tab, series, pv, prec,
                                                            args.steps, args.warmup, lib)
        res[prec] = dict(wall=wall, wall_graph=wall_graph, step_ms=step_ms, kern_ms=kern_ms)
        outs[prec] = out
        note(f"population {prec} timed")
    out32, out64 = outs["mixed"], outs["fp64"]
    points = npv * npt * nss

    def summary(prec, out_bytes):
        r = res[prec]
        ms = 1e3 * r["wall"] / args.steps
        kern = float(np.mean(r["kern_ms"]))
        # outputs, times and parameter rows, plus the per-row setup's output
        # where the kernel reads it (every launch but the fused split one)
        fused = series.kernel(tab, npv, prec) == "split_fused"
        traffic_alg = (npv * npt * out_bytes + npt * 8 +
                       npv * (8 * pv.shape[1] + (0 if fused else PVCONST_BYTES)))
        ms_graph = 1e3 * r["wall_graph"] / args.steps
        return dict(value=points / (ms / 1e3), ms_per_step=ms,
                    graph_replay=dict(value=points / (ms_graph / 1e3), ms_per_step=ms_graph),
                    latency_ms=dict(p50=pct(r["step_ms"], 50), p99=pct(r["step_ms"], 99)),
                    kernel_ms=dict(mean=kern, p50=pct(r["kern_ms"], 50), p99=pct(r["kern_ms"], 99)),
                    alg_bytes=traffic_alg)

    m = summary("mixed", 4)
    d = summary("fp64", 8)
    # the forward kernel the library launches on this series (rr_series_kernel)
    kform = {"split": "k_forward_split<%s, false>", "split_fused": "k_forward_split<%s, true>",
             "tiles": "k_forward<%s, false, 8>"}
    kname = {p: kform[series.kernel(tab, npv, p)] % t
             for p, t in (("mixed", "float"), ("fp64", "double"))}
    achieved = m["alg_bytes"] / (m["kernel_ms"]["mean"] / 1e3) / 1e9
    kc = profile_counters(kname["mixed"])
    traffic = kc.get("hbm_bytes_per_launch") if kc else None
    roof = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                frac=achieved / HBM_PEAK_GBS, traffic=traffic,
                kernel=kname["mixed"], alg_bytes_per_launch=m["alg_bytes"],
                kernel_ms=m["kernel_ms"]["mean"],
                valu=valu_view(kname["mixed"], m["kernel_ms"]["mean"]))
    achieved64 = d["alg_bytes"] / (d["kernel_ms"]["mean"] / 1e3) / 1e9

    line = dict(
        metric=METRIC, value=m["value"], unit="points/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=m["ms_per_step"], higher_is_better=True,
        scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
        config=dict(workload=f"population evaluation npv={npv} npt={npt} nss={nss}, "
                             "2-min cadence, power-2 LD tabulated at 200 mu",
                    npv=npv, npt=npt, nss=nss, precision="mixed (FP64 time reduction, FP32 bulk)",
                    grid=grid,
                    launch="one rr_evaluate_series call per step from Python (%sforward "
                           "kernel '%s'); 'graph_replay' = the same call captured as a HIP "
                           "graph and replayed" % (
                               "" if kname["mixed"].endswith("true>") else "per-row setup + ",
                               kname["mixed"])),
        graph_replay=m["graph_replay"],
        latency_ms=m["latency_ms"],
        fp64=dict(value=d["value"], ms_per_step=d["ms_per_step"], graph_replay=d["graph_replay"],
                  latency_ms=d["latency_ms"],
                  dtype="f64", roofline=dict(bound="hbm", achieved=achieved64,
                                             peak=HBM_PEAK_GBS, unit="GB/s",
                                             frac=achieved64 / HBM_PEAK_GBS,
                                             kernel=kname["fp64"],
                                             kernel_ms=d["kernel_ms"]["mean"],
                                             valu=valu_view(kname["fp64"],
                                                            d["kernel_ms"]["mean"]))),
        roofline=roof,
        in_transit_fraction=None,
        source_hash=source_hash(),
    )
    o32 = out32.cpu().numpy().astype(np.float64)
    o64 = out64.cpu().numpy()
    line["in_transit_fraction"] = float(np.mean(o64 < 1.0))
    if not args.no_serving:
        line["serving"] = serving_leg(rr, wl, args.serving_requests, args.serving_burst)
        note("serving leg done")
    if not args.no_serving:
        line["single_light_curve"] = single_lc_leg(rr, wl, min(args.steps, 200), 20)
        note("single light curve leg done")
    legs = set() if args.no_extra else set(args.legs.split(","))
    if "heterogeneous" in legs:
        line["heterogeneous"] = heterogeneous_leg(rr, wl, min(args.steps, 50), 5, lib)
        note("heterogeneous leg done")
    if "per_vector_ld" in legs:
        line["per_vector_ld"] = per_vector_ld_leg(rr, wl, min(args.steps, 50), 5, lib)
        note("per-vector LD leg done")
    if "direct" in legs:
        line["direct_model"] = direct_leg(rr, wl, min(args.steps, 20), 2)
        note("direct model leg done")
    if "small_planet" in legs:
        line["small_planet"] = small_planet_leg(rr, wl, min(args.steps, 20), 2)
        note("small-planet leg done")
    if "variants" in legs:
        line["variant_selection"] = variant_leg(rr, wl)
        note("variant leg done")
    if "loglik" in legs:
        line["loglik_grad"] = loglik_leg(rr, wl, 10, 2)
        note("log-likelihood leg done")
    if not args.no_cpu_baseline:
        note("oracle baseline on the host")
        cb, acc = cpu_baseline(w, grid, args.cpu_seconds, o64, o32)
        line["cpu_baseline"] = cb
        line["accuracy_vs_oracle"] = acc
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
