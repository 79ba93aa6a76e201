"""Request-stream driver for the ELBM server (elbm_server_* of libelbm.so).

Submits a seeded stream of D2Q9 shear-layer requests at their arrival times
from the calling thread, while the library's scheduler thread admits them by
pool footprint and free slots and advances every resident simulation with
batched launches.  Reports per-request latency (scheduled arrival to
completion observed on the host), p50/p99, and aggregate throughput.
"""
from __future__ import annotations

import time
from typing import Optional

import numpy as np
import torch

from . import elbm
from . import workloads as Wk


def footprint(req: dict) -> int:
    """Pool bytes one request holds while resident: state + staging copy."""
    cfg = elbm.make_config("d2q9", req["n"], req["n"], 1, storage=req["storage"],
                           beta=req["beta"])
    stage = req["n"] * req["n"] * 3 * 8
    a = 256
    return (elbm.state_bytes(cfg) + a - 1) // a * a + (stage + a - 1) // a * a


def run_stream(reqs, *, pool_bytes: Optional[int] = None, max_active: int = 64,
               round_steps: int = 50, preempt_rounds: int = 0, keep: tuple = (),
               realtime: bool = True, device: str = "cuda", log=None) -> dict:
    """Serve `reqs` (workloads.serving_stream) and return the measurements.

    keep: request indices whose final rho/u are returned (for comparisons
    with alone runs).  pool_bytes defaults to twice the largest footprint
    times max_active, capped at 64 GiB.  preempt_rounds: the server's
    preemption setting (0: first come, first served)."""
    dev = torch.device(device)
    fields = {n: Wk.shear_layer(n) for n in sorted({r["n"] for r in reqs})}
    fields = {n: (np.ascontiguousarray(rho.reshape(-1)), np.ascontiguousarray(u.reshape(2, -1)))
              for n, (rho, u) in fields.items()}
    if pool_bytes is None:
        pool_bytes = min(max(footprint(r) for r in reqs) * max_active * 2, 64 << 30)
    stream = torch.cuda.Stream(device=dev)
    keep = set(keep)
    outs = {}
    lag = np.zeros(len(reqs))
    ids = []
    with elbm.Server(pool_bytes, max_active=max_active, round_steps=round_steps,
                     preempt_rounds=preempt_rounds, device=dev, stream=stream) as srv:
        t0 = time.perf_counter()
        for r in reqs:
            if realtime:
                dt = t0 + r["arrival"] - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
            n = r["n"]
            rho, u = fields[n]
            orho = ou = None
            if r["k"] in keep:
                with torch.cuda.stream(stream):
                    orho = torch.empty(n * n, dtype=torch.float64, device=dev)
                    ou = torch.empty(2, n * n, dtype=torch.float64, device=dev)
                outs[r["k"]] = (orho, ou)
            lag[r["k"]] = time.perf_counter() - t0 - (r["arrival"] if realtime else 0.0)
            ids.append(srv.submit("d2q9", n, n, 1, rho0=rho, u0=u, nsteps=r["steps"],
                                  out_rho=orho, out_u=ou, storage=r["storage"],
                                  beta=r["beta"]))
        if log:
            log(f"serving: {len(reqs)} requests submitted in "
                f"{time.perf_counter() - t0:.2f} s")
        for i in ids:
            srv.wait(i)
        infos = [srv.poll(i) for i in ids]
        st = srv.stats()
    torch.cuda.synchronize(dev)
    lat = np.array([inf["t_done"] - inf["t_submit"] for inf in infos]) + np.maximum(lag, 0.0)
    qwait = np.array([inf["t_admit"] - inf["t_submit"] for inf in infos])
    updates = sum(r["n"] * r["n"] * r["steps"] for r in reqs)
    span = st["t_last_done"] - st["t_first_submit"]
    return dict(
        n_req=len(reqs), completed=st["completed"], failed=st["failed"],
        p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
        mean_s=float(lat.mean()), max_s=float(lat.max()),
        queue_p50_s=float(np.percentile(qwait, 50)), queue_p99_s=float(np.percentile(qwait, 99)),
        submit_lag_max_s=float(lag.max()),
        mlups=updates / span / 1e6 if span > 0 else None, span_s=span,
        site_updates=updates, rounds=st["rounds"], launches=st["launches"],
        max_resident=st["max_resident"], pool_bytes=int(pool_bytes),
        max_active=max_active, round_steps=round_steps, preempt_rounds=preempt_rounds,
        preemptions=st["preemptions"],
        latency_s=lat.tolist(), outputs=outs)


def run_alone(req: dict, device: str = "cuda"):
    """One request advanced alone (elbm_step, no server); returns rho, u."""
    n = req["n"]
    rho, u = Wk.shear_layer(n)
    with elbm.Simulation("d2q9", n, n, 1, rho0=rho, u0=u, device=device,
                         storage=req["storage"], beta=req["beta"]) as sim:
        sim.step(req["steps"])
        return sim.moments()
