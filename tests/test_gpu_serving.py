"""The continuous-batching server on the GPU: results are the same alone and
in a mix (the same kernel code as rr_evaluate, independent of batching),
match the oracle, and the arena admits requests as memory frees up."""

import numpy as np
import pytest

import workloads as wl
from oracle import roadrunner as orr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_08500_amd as rr
    het = wl.heterogeneous(npv=1)
    grid = wl.TEST_GRID
    tab = rr.Tables(het["mu_s"], het["I_s"], grid)
    otab = orr.Tables(het["mu_s"], het["I_s"], **grid)
    series, reqs = wl.serving_mix(40, nseries=6, max_npv=256, max_npt=20000, seed_extra=1)
    return rr, tab, otab, series, reqs


def evaluate_direct(rr, tab, se, pv, prec):
    """rr_evaluate on the same series: the per-tile kernel the server's
    grouped launches share, so its values are the server's bit for bit."""
    ser = rr.TimeSeries(se["times"], se["lcids"], se["pbids"], se["nss"], se["exptimes"])
    return rr.evaluate_unregistered(tab, ser, pv, prec).cpu().numpy()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_alone_equals_in_mix(env, prec):
    rr, tab, otab, series, reqs = env
    srv = rr.Server(tab, budget_bytes=1 << 30, max_tick_blocks=512)
    sids = [srv.add_series(s["times"], s["lcids"], s["pbids"], s["nss"], s["exptimes"])
            for s in series]
    probe = reqs[0]
    a = srv.submit(sids[probe["series"]], probe["pv"], prec)
    alone = srv.wait(a).numpy().copy()
    handles = []
    for i, r in enumerate(reqs):
        handles.append(srv.submit(sids[r["series"]], r["pv"], prec))
        if i == len(reqs) // 2:
            mid = srv.submit(sids[probe["series"]], probe["pv"], prec)
    outs = [srv.wait(h).numpy().copy() for h in handles]
    in_mix = srv.wait(mid).numpy()
    assert np.abs(in_mix.astype(np.float64) - alone).max() <= 1e-6
    assert np.array_equal(in_mix, alone)          # bitwise: batching changes nothing
    for r, o in zip(reqs, outs):
        direct = evaluate_direct(rr, tab, series[r["series"]], r["pv"], prec)
        assert np.array_equal(o, direct)
    st = srv.stats()
    assert st["completed"] == len(reqs) + 2 and st["last_error"] == 0
    lat = np.array([h.latency for h in handles])
    assert np.all(lat > 0)
    print(f"serving {prec}: {len(reqs)} requests, {st['ticks']} ticks, "
          f"p50 {np.percentile(lat, 50) * 1e3:.2f} ms p99 {np.percentile(lat, 99) * 1e3:.2f} ms")
    srv.close()


def test_served_results_match_oracle(env):
    rr, tab, otab, series, reqs = env
    srv = rr.Server(tab, budget_bytes=1 << 30)
    sids = [srv.add_series(s["times"], s["lcids"], s["pbids"], s["nss"], s["exptimes"])
            for s in series]
    for r in reqs[:4]:
        se = series[r["series"]]
        pv = r["pv"][:3]
        h64 = srv.submit(sids[r["series"]], pv, "fp64")
        h32 = srv.submit(sids[r["series"]], pv, "mixed")
        f64, f32 = srv.wait(h64).numpy(), srv.wait(h32).numpy().astype(np.float64)
        ref = orr.evaluate(otab, se["times"], pv, lcids=se["lcids"], pbids=se["pbids"],
                           nss=se["nss"], exptimes=se["exptimes"])
        assert np.abs(f64 - ref).max() <= 1e-9
        assert np.abs(f32 - ref).max() <= 1e-6
    srv.close()


def test_admission_by_footprint(env):
    """A 4 MiB arena: requests whose combined footprint is many times the
    budget all complete (admitted as memory frees up); one larger than the
    whole budget is refused at submission."""
    rr, tab, otab, series, reqs = env
    srv = rr.Server(tab, budget_bytes=4 << 20, max_tick_blocks=64)
    se = series[0]
    sid = srv.add_series(se["times"], se["lcids"], se["pbids"], se["nss"], se["exptimes"])
    npt = se["times"].size
    rows_fit = max(1, int((3 << 20) / (npt * 4 + 300)))
    pv = wl.draw_orbits(np.random.default_rng(0), rows_fit, npb=4, chromatic=0.05)
    hs = [srv.submit(sid, pv, "mixed") for _ in range(12)]
    direct = evaluate_direct(rr, tab, se, pv, "mixed")
    for h in hs:
        assert np.array_equal(srv.wait(h).numpy(), direct)
    big = wl.draw_orbits(np.random.default_rng(1), 4 * rows_fit + 64, npb=4, chromatic=0.05)
    with pytest.raises(rr.RRError) as e:
        srv.submit(sid, big, "mixed")
    assert e.value.code == -4
    with pytest.raises(rr.RRError):
        srv.submit(sid + 99, pv, "mixed")                 # unknown series
    with pytest.raises(rr.RRError):
        srv.submit(sid, pv[:, :7], "mixed")               # npar mismatch
    srv.close()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_device_output_equals_host_output(env, prec):
    """rr_server_submit_device: the kernels write the caller's device buffer
    (no host copy); its values equal the host-output form and rr_evaluate
    bitwise, mixed with host-output requests in the same ticks."""
    import torch
    rr, tab, otab, series, reqs = env
    srv = rr.Server(tab, budget_bytes=1 << 30, max_tick_blocks=512)
    sids = [srv.add_series(s["times"], s["lcids"], s["pbids"], s["nss"], s["exptimes"])
            for s in series]
    hd, hh = [], []
    for r in reqs[:16]:
        hd.append(srv.submit(sids[r["series"]], r["pv"], prec, device_out=True))
        hh.append(srv.submit(sids[r["series"]], r["pv"], prec))
    for r, a, b in zip(reqs[:16], hd, hh):
        srv.wait(a)
        srv.wait(b)
        assert a.out.is_cuda and a.latency > 0
        dev = a.out.cpu().numpy()
        assert np.array_equal(dev, b.out.numpy())
        assert np.array_equal(dev, evaluate_direct(rr, tab, series[r["series"]], r["pv"], prec))
    # footprint without the output: a request whose output alone exceeds the
    # arena is admitted in device-output form
    small = rr.Server(tab, budget_bytes=1 << 20, max_tick_blocks=256)
    se = series[0]
    sid = small.add_series(se["times"], se["lcids"], se["pbids"], se["nss"], se["exptimes"])
    npt = se["times"].size
    nrow = (2 << 20) // (npt * 4) + 1                     # > 2 MiB of float output
    pv = wl.draw_orbits(np.random.default_rng(5), nrow, npb=4, chromatic=0.05)
    with pytest.raises(rr.RRError):
        small.submit(sid, pv, "mixed")
    out = torch.empty((nrow, npt), dtype=torch.float32, device="cuda")
    h = small.submit(sid, pv, "mixed", device_out=True, out=out)
    small.wait(h)
    assert np.array_equal(out.cpu().numpy(), evaluate_direct(rr, tab, se, pv, "mixed"))
    small.close()
    srv.close()


def test_series_added_while_requests_run(env):
    """Series registered from another thread while requests are queued and
    running: every request completes with the values of rr_evaluate (each
    request works from its own copy of its series' description)."""
    import threading
    rr, tab, otab, series, reqs = env
    srv = rr.Server(tab, budget_bytes=1 << 30, max_tick_blocks=256)
    sids = [srv.add_series(s["times"], s["lcids"], s["pbids"], s["nss"], s["exptimes"])
            for s in series[:2]]
    extra = []
    stop = threading.Event()

    def add_many():
        k = 0
        while not stop.is_set() and k < 200:
            se = series[k % len(series)]
            extra.append(srv.add_series(se["times"], se["lcids"], se["pbids"], se["nss"],
                                        se["exptimes"]))
            k += 1

    th = threading.Thread(target=add_many)
    th.start()
    hs = [(r, srv.submit(sids[r["series"] % 2], r["pv"][:32], "mixed")) for r in reqs[:24]]
    th.join()
    stop.set()
    for r, h in hs:
        srv.wait(h)
        ref = evaluate_direct(rr, tab, series[r["series"] % 2], r["pv"][:32], "mixed")
        assert np.array_equal(h.out.numpy(), ref)
    assert len(extra) == 200
    h = srv.submit(extra[-1], reqs[0]["pv"][:4], "mixed")       # a series added last
    srv.wait(h)
    assert np.array_equal(h.out.numpy(),
                          evaluate_direct(rr, tab, series[199 % len(series)], reqs[0]["pv"][:4],
                                          "mixed"))
    srv.close()


def test_failed_launch_completes_requests_with_error(env):
    """A grouped launch that fails (forced on the host: no kernel runs) ends
    its requests with RR_EDEVICE instead of leaving them pending; later
    requests are served and the server shuts down."""
    rr, tab, otab, series, reqs = env
    srv = rr.Server(tab, budget_bytes=1 << 30, max_tick_blocks=1 << 20)
    se = series[0]
    sid = srv.add_series(se["times"], se["lcids"], se["pbids"], se["nss"], se["exptimes"])
    pv = reqs[0]["pv"][:8]
    ok = srv.submit(sid, pv, "mixed")
    srv.wait(ok)
    srv.fail_next_tick()
    bad = srv.submit(sid, pv, "mixed")
    with pytest.raises(rr.RRError) as e:
        srv.wait(bad)
    assert e.value.code == -3                              # RR_EDEVICE
    assert srv.stats()["last_error"] == -3
    again = srv.submit(sid, pv, "mixed")
    srv.wait(again)
    assert np.array_equal(again.out.numpy(), ok.out.numpy())
    srv.close()


def test_release_as_soon_as_done(env):
    """A waiting thread releases every request the moment it completes while
    the submitting thread keeps queueing more: every request completes (the
    wait's time limit turns a lost request into a failure, not a hang), with
    its values, and the server's count matches.  Guards the rule that the
    worker holds no reference to a request once it can complete."""
    import queue
    import threading
    import torch
    rr, tab, otab, series, reqs = env
    srv = rr.Server(tab, budget_bytes=1 << 28, max_tick_blocks=64)
    combos = []
    for k in range(4):
        se = series[k]
        sid = srv.add_series(se["times"], se["lcids"], se["pbids"], se["nss"], se["exptimes"])
        pv = reqs[k]["pv"][:3]
        combos.append((sid, pv, evaluate_direct(rr, tab, se, pv, "mixed")))
    n = 400
    q = queue.Queue()
    bad = []

    def waiter():
        for _ in range(n):
            i, h = q.get()
            try:
                out = srv.wait(h, timeout=30.0)
                torch.cuda.synchronize()
                if not np.array_equal(out.cpu().numpy(), combos[i % 4][2]):
                    bad.append(i)
                srv.release(h)
            except Exception as e:          # noqa: BLE001 -- reported below
                bad.append((i, repr(e)))

    th = threading.Thread(target=waiter)
    th.start()
    for i in range(n):
        sid, pv, _ = combos[i % 4]
        q.put((i, srv.submit(sid, pv, "mixed", device_out=True)))
    th.join(timeout=90.0)
    assert not th.is_alive()
    assert bad == []
    assert srv.stats()["completed"] == n
    srv.close()
