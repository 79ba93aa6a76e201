"""Serving (elbm_server_*): each request's result is the same in the mix as
alone (bitwise: the batched step computes every site exactly as the single
step does), admission under a pool that holds one request at a time, kept
states, and isolation of a request that goes non-finite."""
import time

import numpy as np
import pytest
import torch

from paper_1904_00866_amd import serving
from paper_1904_00866_amd import workloads as Wk

pytestmark = pytest.mark.gpu


def _dim(D):
    return 3 if D == 19 else D  # lattice code 19: D3Q19


def _fields(D, shape, seed):
    N = int(np.prod(shape))
    if D == 2 and shape[0] == shape[1]:
        rho, u = Wk.shear_layer(shape[0])
        return rho.reshape(-1), u.reshape(2, -1)
    rho, u = Wk.random_velocity_field(_dim(D), N, 0.05, seed=seed)
    return rho, u


def _alone(gpu, D, shape, rho, u, steps, **kw):
    with gpu.Simulation(D, *shape, rho0=rho, u0=u, **kw) as s:
        s.step(steps)
        r, v = s.moments()
        torch.cuda.synchronize()
        return r.cpu().numpy(), v.cpu().numpy(), s.populations().cpu().numpy()


MIX = [  # (D, shape, steps, kwargs)
    (2, (64, 64, 1), 120, dict(storage="f32", beta=0.99)),
    (2, (37, 23, 1), 75, dict(storage="f16dev", beta=0.97)),
    (2, (128, 128, 1), 200, dict(storage="f32", beta=0.995)),
    (2, (48, 40, 1), 0, dict(storage="f32", beta=0.99)),
    (3, (16, 12, 9), 60, dict(storage="f32", beta=0.98)),
    (2, (64, 64, 1), 90, dict(storage="f32", beta=0.99, mode="bgk")),
    (2, (96, 96, 1), 150, dict(storage="f16dev", beta=0.99)),
    (2, (33, 65, 1), 41, dict(storage="f64", beta=0.9)),
    (2, (256, 256, 1), 64, dict(storage="f32", beta=0.999)),
    (3, (20, 20, 20), 30, dict(storage="f16dev", beta=0.99)),
    (2, (64, 64, 1), 120, dict(storage="f32", beta=0.99)),
    (2, (50, 50, 1), 333, dict(storage="f32", beta=0.96, mode="secant")),
    (19, (14, 10, 9), 50, dict(storage="f32", beta=0.98)),
    (19, (16, 16, 16), 80, dict(storage="f16dev", beta=0.99)),
    (2, (64, 48, 1), 100, dict(storage="f16dev", beta=0.99, fp64="mixed")),
    (3, (16, 16, 8), 40, dict(storage="f32dev", beta=0.98, fp64="mixed")),
]


def test_server_mix_equals_alone(gpu):
    """Sixteen requests of mixed lattices, sizes, storages, alpha modes, site
    arithmetic and step counts, arriving while earlier ones run (5 slots,
    37-step rounds): the final rho, u of each equal those of the same
    simulation advanced alone."""
    dev = torch.device("cuda")
    stream = torch.cuda.Stream()
    fields = [_fields(D, shp, 100 + k) for k, (D, shp, _, _) in enumerate(MIX)]
    outs, ids = [], []
    with gpu.Server(256 << 20, max_active=5, round_steps=37, stream=stream) as srv:
        for k, ((D, shp, steps, kw), (rho, u)) in enumerate(zip(MIX, fields)):
            N = int(np.prod(shp))
            with torch.cuda.stream(stream):
                o = (torch.empty(N, dtype=torch.float64, device=dev),
                     torch.empty(_dim(D), N, dtype=torch.float64, device=dev))
            outs.append(o)
            ids.append(srv.submit(D, *shp, rho0=rho, u0=u, nsteps=steps, out_rho=o[0],
                                  out_u=o[1], **kw))
            if k % 3 == 2:
                time.sleep(0.005)
        for i in ids:
            srv.wait(i, 60.0)
        st = srv.stats()
        infos = [srv.poll(i) for i in ids]
    torch.cuda.synchronize()
    assert st["completed"] == len(MIX) and st["failed"] == 0
    assert 1 < st["max_resident"] <= 5
    assert st["site_updates"] == sum(int(np.prod(s)) * n for _, s, n, _ in MIX)
    for k, ((D, shp, steps, kw), (rho, u), inf) in enumerate(zip(MIX, fields, infos)):
        assert inf["state"] == "done" and inf["steps_done"] == steps
        assert inf["t_submit"] <= inf["t_admit"] <= inf["t_done"]
        r0, u0, _ = _alone(gpu, D, shp, rho, u, steps, **kw)
        assert np.array_equal(outs[k][0].cpu().numpy(), r0), k
        assert np.array_equal(outs[k][1].cpu().numpy(), u0), k


def elbm_state(gpu, r):
    cfg = gpu.make_config("d2q9", r["n"], r["n"], 1, storage=r["storage"], beta=r["beta"])
    return (gpu.state_bytes(cfg) + 255) // 256 * 256


def test_server_admission_small_pool(gpu):
    """A pool that fits one request at a time: requests run one after
    another in arrival order; one that can never fit is rejected."""
    reqs = [dict(k=k, n=n, steps=s, storage="f32", beta=0.99, arrival=0.0)
            for k, (n, s) in enumerate([(128, 40), (120, 30), (128, 20), (112, 50)])]
    pool = max(serving.footprint(r) for r in reqs) + 4096
    # no request fits beside the resident state of another
    state = {r["n"]: elbm_state(gpu, r) for r in reqs}
    assert all(state[a["n"]] + serving.footprint(b) > pool for a in reqs for b in reqs)
    stream = torch.cuda.Stream()
    with gpu.Server(pool, max_active=8, round_steps=16, stream=stream) as srv:
        big = Wk.shear_layer(512)
        with pytest.raises(gpu.ElbmError) as e:
            srv.submit("d2q9", 512, 512, 1, rho0=big[0], u0=big[1], nsteps=1)
        assert e.value.status == -3
        ids = []
        for r in reqs:
            rho, u = Wk.shear_layer(r["n"])
            ids.append(srv.submit("d2q9", r["n"], r["n"], 1, rho0=rho, u0=u,
                                  nsteps=r["steps"], beta=r["beta"]))
        for i in ids:
            srv.wait(i, 60.0)
        infos = [srv.poll(i) for i in ids]
        st = srv.stats()
    assert st["completed"] == 4 and st["max_resident"] == 1
    for a, b in zip(infos, infos[1:]):
        assert b["t_admit"] >= a["t_done"]
    assert all(inf["footprint"] == serving.footprint(r) for inf, r in zip(infos, reqs))


def test_server_keep_state_and_release(gpu):
    """A kept simulation continues outside the server exactly as an
    uninterrupted run; releasing it frees its pool block for the next
    request."""
    n, s1, s2 = 64, 70, 30
    rho, u = Wk.shear_layer(n)
    req = dict(n=n, storage="f32", beta=0.99)
    pool = serving.footprint(req) + 4096
    stream = torch.cuda.Stream()
    _, _, ref = _alone(gpu, 2, (n, n, 1), rho, u, s1 + s2, storage="f32", beta=0.99)
    with gpu.Server(pool, max_active=4, round_steps=25, stream=stream) as srv:
        i = srv.submit("d2q9", n, n, 1, rho0=rho, u0=u, nsteps=s1, keep_state=True,
                       storage="f32", beta=0.99)
        srv.wait(i, 60.0)
        sim = srv.simulation(i)
        assert sim.t == s1
        with torch.cuda.stream(stream):
            sim.step(s2)
            f = sim.populations()
        stream.synchronize()
        assert np.array_equal(f.cpu().numpy(), ref)
        j = srv.submit("d2q9", n, n, 1, rho0=rho, u0=u, nsteps=5, storage="f32", beta=0.99)
        time.sleep(0.2)
        assert srv.poll(j)["state"] == "queued"  # the kept state holds the pool
        sim.close()  # elbm_server_release
        srv.wait(j, 60.0)
        assert srv.poll(j)["state"] == "done"
        with pytest.raises(gpu.ElbmError):
            srv.simulation(j)  # not a keep_state request


def test_server_isolates_a_diverging_request(gpu):
    """An LBGK request that diverges (a sharp shear layer at nu ~ 1e-6) in
    the same batched launches as two stable LBGK requests: the stable ones
    still equal their alone runs.  Invalid requests are rejected at
    submission without disturbing the others."""
    n = 48
    bad = Wk.shear_layer(n, u0=0.3, kappa=200.0)
    good = [Wk.shear_layer(64), Wk.shear_layer(n)]
    dev = torch.device("cuda")
    stream = torch.cuda.Stream()
    outs = []
    with gpu.Server(64 << 20, max_active=4, round_steps=50, stream=stream) as srv:
        with torch.cuda.stream(stream):
            for m in (64, n, n):
                outs.append((torch.empty(m * m, dtype=torch.float64, device=dev),
                             torch.empty(2, m * m, dtype=torch.float64, device=dev)))
        ids = [srv.submit("d2q9", 64, 64, 1, rho0=good[0][0], u0=good[0][1], nsteps=400,
                          out_rho=outs[0][0], out_u=outs[0][1], mode="bgk", beta=0.95),
               srv.submit("d2q9", n, n, 1, rho0=bad[0], u0=bad[1], nsteps=400,
                          out_rho=outs[2][0], out_u=outs[2][1], mode="bgk", beta=0.99999),
               srv.submit("d2q9", n, n, 1, rho0=good[1][0], u0=good[1][1], nsteps=300,
                          out_rho=outs[1][0], out_u=outs[1][1], mode="bgk", beta=0.95)]
        rho_bad = np.ones(n * n)
        rho_bad[7] = np.nan
        for r, u in [(rho_bad, good[1][1]), (-good[1][0], good[1][1]),
                     (good[1][0], good[1][1] * 30.0)]:
            with pytest.raises(gpu.ElbmError) as e:
                srv.submit("d2q9", n, n, 1, rho0=r, u0=u, nsteps=10, mode="bgk")
            assert e.value.status == -1
        for i in ids:
            srv.wait(i, 60.0)
        st = srv.stats()
    torch.cuda.synchronize()
    assert st["completed"] == 3 and st["failed"] == 0 and st["submitted"] == 3
    for (m, steps, (rho, u)), o in zip([(64, 400, good[0]), (n, 300, good[1])], outs):
        r0, u0, _ = _alone(gpu, 2, (m, m, 1), rho, u, steps, mode="bgk", beta=0.95,
                           storage="f32")
        assert np.array_equal(o[0].cpu().numpy(), r0)
        assert np.array_equal(o[1].cpu().numpy(), u0)
    ub = outs[2][1].cpu().numpy()
    assert not np.all(np.isfinite(ub)) or np.abs(ub).max() > 1.0


def test_serving_stream_small(gpu):
    """A short seeded stream through the Python driver: every request
    completes, latencies are positive, and two sampled requests equal their
    alone runs."""
    reqs = Wk.serving_stream(10, rate=50.0, seed=7, sizes=(64, 128, 256),
                             steps_range=(50, 400))
    res = serving.run_stream(reqs, max_active=4, round_steps=40, keep=(0, 5))
    assert res["completed"] == 10 and res["failed"] == 0
    assert 0 < res["p50_s"] <= res["p99_s"]
    for k in (0, 5):
        r0, u0 = serving.run_alone(reqs[k])
        torch.cuda.synchronize()
        assert torch.equal(res["outputs"][k][0], r0)
        assert torch.equal(res["outputs"][k][1], u0)


LONG = (2, (128, 128, 1), 20000, dict(storage="f16dev", beta=0.99))
SHORT = [(2, (64, 64, 1), 60, dict(storage="f32", beta=0.99)),
         (3, (16, 12, 9), 40, dict(storage="f32dev", beta=0.98)),
         (19, (14, 10, 9), 60, dict(storage="f32", beta=0.98))]
# for a pool with room for LONG only: each needs more than LONG's state leaves
SHORT_POOL = [(2, (88, 88, 1), 60, dict(storage="f32", beta=0.99)),
              (3, (16, 12, 9), 40, dict(storage="f32dev", beta=0.98)),
              (2, (80, 96, 1), 60, dict(storage="f32", beta=0.99))]


def _footprint(gpu, D, shape, kw):
    lat = {1: "d1q3", 2: "d2q9", 3: "d3q27", 19: "d3q19"}[D]
    cfg = gpu.make_config(lat, *shape, **kw)
    N = int(np.prod(shape))
    up = lambda b: (b + 255) // 256 * 256
    return up(gpu.state_bytes(cfg)) + up(N * (1 + _dim(D)) * 8)


def _run_long_then_short(gpu, pool, max_active, preempt_rounds, short=SHORT):
    """Submit LONG, wait until it runs, then the short requests; return the
    requests, fields, outputs, request infos (LONG first) and server stats."""
    dev = torch.device("cuda")
    stream = torch.cuda.Stream()
    reqs = [LONG] + short
    fields = [_fields(D, shp, 300 + k) for k, (D, shp, _, _) in enumerate(reqs)]
    outs, ids = [], []
    with gpu.Server(pool, max_active=max_active, round_steps=20, preempt_rounds=preempt_rounds,
                    stream=stream) as srv:
        for k, ((D, shp, steps, kw), (rho, u)) in enumerate(zip(reqs, fields)):
            N = int(np.prod(shp))
            with torch.cuda.stream(stream):
                o = (torch.empty(N, dtype=torch.float64, device=dev),
                     torch.empty(_dim(D), N, dtype=torch.float64, device=dev))
            outs.append(o)
            ids.append(srv.submit(D, *shp, rho0=rho, u0=u, nsteps=steps, out_rho=o[0],
                                  out_u=o[1], **kw))
            if k == 0:
                t0 = time.time()
                while srv.poll(ids[0])["state"] != "running" and time.time() - t0 < 10:
                    time.sleep(0.0005)
                assert srv.poll(ids[0])["state"] == "running"
        for i in ids:
            srv.wait(i, 120.0)
        infos = [srv.poll(i) for i in ids]
        st = srv.stats()
    torch.cuda.synchronize()
    return reqs, fields, outs, infos, st


@pytest.mark.parametrize("limit", ["slots", "pool"])
def test_server_preemption_is_exact_and_lets_short_requests_through(gpu, limit):
    """With preemption, a long request resident when short ones arrive is
    moved out to host memory (its checkpoint) and resumed later: the short
    requests finish first, and every result, the preempted one included,
    equals its run alone bitwise.  The head of the queue is blocked either by
    the slot limit (one slot) or by the pool (room for one request)."""
    if limit == "slots":
        pool, slots, short = 64 << 20, 1, SHORT
    else:
        D, shp, _, kw = LONG
        lat = {2: "d2q9"}[D]
        pool = _footprint(gpu, D, shp, kw) + 4096
        left = pool - (gpu.state_bytes(gpu.make_config(lat, *shp, **kw)) + 255) // 256 * 256
        slots, short = 8, SHORT_POOL
        assert all(_footprint(gpu, d, sh, k) > left for d, sh, _, k in short)
        assert all(_footprint(gpu, d, sh, k) <= pool for d, sh, _, k in short)
    reqs, fields, outs, infos, st = _run_long_then_short(gpu, pool, slots, preempt_rounds=2,
                                                         short=short)
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["preemptions"] >= 1 and infos[0]["preemptions"] >= 1
    assert all(inf["t_done"] < infos[0]["t_done"] for inf in infos[1:])
    for k, ((D, shp, steps, kw), (rho, u), inf) in enumerate(zip(reqs, fields, infos)):
        assert inf["state"] == "done" and inf["steps_done"] == steps
        r0, u0, _ = _alone(gpu, D, shp, rho, u, steps, **kw)
        assert np.array_equal(outs[k][0].cpu().numpy(), r0), k
        assert np.array_equal(outs[k][1].cpu().numpy(), u0), k


def test_server_without_preemption_keeps_arrival_order(gpu):
    """preempt_rounds = 0: the long request keeps its slot to the end."""
    reqs, fields, outs, infos, st = _run_long_then_short(gpu, 64 << 20, 1, preempt_rounds=0)
    assert st["completed"] == len(reqs) and st["preemptions"] == 0
    assert all(inf["t_done"] > infos[0]["t_done"] for inf in infos[1:])
    assert all(inf["preemptions"] == 0 for inf in infos)


def test_server_cancel(gpu):
    """Cancellation: with a pool that holds the long request only, a queued
    request is dropped without running and the running long request ends
    between rounds, freeing its block for the request waiting behind it,
    which then completes with the same result as alone.  Neither cancelled
    request writes its outputs; a finished request cannot be cancelled."""
    dev = torch.device("cuda")
    stream = torch.cuda.Stream()
    D, shp, _, kw = LONG
    pool = _footprint(gpu, D, shp, kw) + 4096
    reqs = [LONG, SHORT_POOL[0], SHORT_POOL[2]]
    fields = [_fields(d, sh, 500 + k) for k, (d, sh, _, _) in enumerate(reqs)]
    outs, ids = [], []
    with gpu.Server(pool, max_active=8, round_steps=20, stream=stream) as srv:
        for k, ((d, sh, steps, kw_), (rho, u)) in enumerate(zip(reqs, fields)):
            N = int(np.prod(sh))
            with torch.cuda.stream(stream):
                o = (torch.full((N,), float("nan"), dtype=torch.float64, device=dev),
                     torch.full((_dim(d), N), float("nan"), dtype=torch.float64, device=dev))
            outs.append(o)
            ids.append(srv.submit(d, *sh, rho0=rho, u0=u, nsteps=steps, out_rho=o[0],
                                  out_u=o[1], **kw_))
            if k == 0:
                t0 = time.time()
                while srv.poll(ids[0])["state"] != "running" and time.time() - t0 < 10:
                    time.sleep(0.0005)
        assert srv.poll(ids[0])["state"] == "running"
        assert srv.poll(ids[2])["state"] == "queued"
        srv.cancel(ids[2])
        srv.cancel(ids[0])
        for i in (ids[0], ids[2]):
            with pytest.raises(gpu.ElbmError, match="cancelled"):
                srv.wait(i, 60.0)
        srv.wait(ids[1], 60.0)
        infos = [srv.poll(i) for i in ids]
        with pytest.raises(gpu.ElbmError, match="ESTATE"):
            srv.cancel(ids[1])
        with pytest.raises(gpu.ElbmError, match="ESTATE"):
            srv.cancel(ids[0])
        st = srv.stats()
    torch.cuda.synchronize()
    assert [inf["state"] for inf in infos] == ["cancelled", "done", "cancelled"]
    assert infos[0]["steps_done"] < LONG[2] and infos[2]["t_admit"] == 0
    assert st["cancelled"] == 2 and st["completed"] == 1 and st["failed"] == 0
    for k in (0, 2):
        assert torch.isnan(outs[k][0]).all() and torch.isnan(outs[k][1]).all()
    d, sh, steps, kw_ = reqs[1]
    r0, u0, _ = _alone(gpu, d, sh, *fields[1], steps, **kw_)
    assert np.array_equal(outs[1][0].cpu().numpy(), r0)
    assert np.array_equal(outs[1][1].cpu().numpy(), u0)
