#!/usr/bin/env python3
"""Measurements of the ELBM hot path beyond the headline benchmark, on one
MI355X, through the C ABI only (the FP64 GPU path is the reference where one
is needed; its parity with the CPU oracle is established by the GPU tests).

    python experiments.py w1     D2Q9 64^2 Taylor-Green, FP64, 1000 steps, every
                                 alpha mode: us/step, decay rate vs Eq. (2), drift
    python experiments.py w2     D2Q9 1024^2 shear layer, FP32, 20000 steps:
                                 fraction of sites with alpha < 2, alpha range,
                                 alpha vs vorticity, MLUPS
    python experiments.py e2     D2Q9 128^2 shear layer, nu = 1e-5, 3200 steps:
                                 proportion of sites accepting alpha = 2
    python experiments.py w4     D3Q27 256^3 Taylor-Green, 2000 steps, storage
                                 FP64 / FP32 / FP32-dev / FP16-dev under FP64,
                                 mixed and FP32 site arithmetic: per-site H
                                 increases, errors against the FP64-storage
                                 run; with --w4-out DIR the fields on a
                                 sub-lattice and the kinetic-energy curve
    python experiments.py w4cmp --w4-ref REF.npz --w4-out DIR
                                 those fields against the FP64 oracle's
                                 reference run (stored arrays only, no GPU)
    python experiments.py w5p    the serving stream (64 requests at 20/s) through
                                 a server with 8 slots, first come first served
                                 and with preemption: latency percentiles, MLUPS
    python experiments.py f3     D3Q19 beside D3Q27: 512^3 step time and HBM
                                 roofline fraction of the closed form, LBGK and
                                 (256^3) Newton; 128^3 Re = 1600 Taylor-Green:
                                 kinetic-energy decay and the share of sites
                                 with alpha < 2 on both lattices (FP32 storage
                                 and FP64 arithmetic unless --f3-storage and
                                 --f3-arith say otherwise)
    python experiments.py f3burg Burg's entropy beside the Boltzmann entropy
                                 (closed form, FP32 storage): step time and HBM
                                 fraction at D3Q27 512^3 and D2Q9 2048^2, Newton
                                 at 256^3; 128^3 Re = 1600 Taylor-Green: kinetic
                                 energy and the share of sites with alpha < 2
Each prints one JSON object per experiment on stdout.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

from paper_1904_00866_amd import elbm
from paper_1904_00866_amd import workloads as Wk


def log(msg):
    print(f"[exp {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def _kinetic(rho, u):
    return 0.5 * float((rho * (u * u).sum(0)).sum())


def _timed_steps(sim, n):
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(sim.stream):
        ev0.record(sim.stream)
        sim.step(n)
        ev1.record(sim.stream)
    ev1.synchronize()
    return ev0.elapsed_time(ev1) / n


# --------------------------------------------------------------------- W1 --
def w1():
    n, T, beta = 64, 1000, 0.95
    rho, u = Wk.taylor_green_2d(n)
    nu = (1.0 / beta - 1.0) / 6.0
    k2 = 2.0 * (2.0 * math.pi / n) ** 2
    out = {"experiment": "w1", "workload": "D2Q9 Taylor-Green 64^2, u0 = 0.05, beta = 0.95, "
           "FP64 storage, 1000 steps", "nu_eq2": nu, "modes": {}}
    for mode in ("closed", "secant", "newton", "bisect", "bgk"):
        with elbm.Simulation("d2q9", n, n, 1, rho0=rho, u0=u, storage="f64", beta=beta,
                             mode=mode, diag=elbm.DIAG_COUNTS | elbm.DIAG_SUMS) as sim:
            ts, kes, m0 = [], [], None
            ms_total = 0.0
            for t in range(0, T + 1, 100):
                if t:
                    ms_total += _timed_steps(sim, 100) * 100
                r, v = sim.moments()
                torch.cuda.synchronize()
                ts.append(t)
                kes.append(_kinetic(r, v))
                if m0 is None:
                    m0 = float(r.sum())
                mass = float(r.sum())
            st = sim.stats()
        slope = np.polyfit(ts, np.log(kes), 1)[0]
        nu_fit = -slope / (2.0 * k2)
        out["modes"][mode] = {"us_per_step": round(ms_total / T * 1e3, 2),
                              "nu_fit": nu_fit, "nu_rel_err": (nu_fit - nu) / nu,
                              "ke_ratio_1000": kes[-1] / kes[0],
                              "mass_drift_rel": (mass - m0) / m0,
                              "iters_per_site_last_step": st["total_iters"] / (n * n)}
        log(f"w1 {mode}: {out['modes'][mode]}")
    out["ke_ratio_eq2"] = math.exp(-2.0 * nu * k2 * T)
    return out


# --------------------------------------------------------------------- W2 --
def _vorticity(u, n):
    ux, uy = u[0].reshape(n, n), u[1].reshape(n, n)  # [y, x]
    dvy_dx = (torch.roll(uy, -1, 1) - torch.roll(uy, 1, 1)) * 0.5
    dux_dy = (torch.roll(ux, -1, 0) - torch.roll(ux, 1, 0)) * 0.5
    return (dvy_dx - dux_dy).reshape(-1)


def w2(steps=20000, every=100, snap_every=1000):
    n = 1024
    beta = Wk.shear_beta(n)
    rho, u = Wk.shear_layer(n)
    out = {"experiment": "w2", "workload": f"D2Q9 shear layer {n}^2, u0 = 0.04, kappa = 80, "
           f"delta = 0.05, Re = 3e4 (beta = {beta:.6f}), FP32 storage, {steps} steps",
           "beta": beta}
    with elbm.Simulation("d2q9", n, n, 1, rho0=rho, u0=u, storage="f32", beta=beta) as sim:
        sim.step(20)
        ms = _timed_steps(sim, 2000)
    out["ms_per_step"] = ms
    out["mlups"] = n * n / ms / 1e3
    out["gbs_algorithmic"] = 2 * 9 * 4 * n * n / ms / 1e6
    curve, snaps = [], []
    diag = elbm.DIAG_ALPHA | elbm.DIAG_COUNTS | elbm.DIAG_SUMS
    with elbm.Simulation("d2q9", n, n, 1, rho0=rho, u0=u, storage="f32", beta=beta,
                         diag=diag) as sim:
        H0 = None
        for t in range(every, steps + 1, every):
            sim.step(every)
            st = sim.stats()
            if H0 is None:
                H0 = st["sum_H"]
            curve.append([t, st["n_alpha_lt2"] / (n * n), st["n_accept2"] / (n * n),
                          st["alpha_min"], st["sum_H"]])
            if t % snap_every == 0:
                a = sim.alpha_field()
                r, v = sim.moments()
                w = _vorticity(v, n).abs()
                dev = 2.0 - a
                c = torch.corrcoef(torch.stack([dev, w]))[0, 1].item()
                snaps.append({"t": t, "alpha_min": a.min().item(),
                              "frac_alpha_lt2": (a < 2.0).double().mean().item(),
                              "corr_2_minus_alpha_abs_vorticity": c,
                              "kinetic_energy": _kinetic(r, v)})
                log(f"w2 t={t}: {snaps[-1]}")
    fr = np.array([c[1] for c in curve])
    Hs = np.array([c[4] for c in curve])
    out.update({"fraction_alpha_lt2": {"mean": float(fr.mean()), "min": float(fr.min()),
                                       "max": float(fr.max()), "last": float(fr[-1])},
                "sum_H_increases": int((np.diff(Hs) > 0).sum()),
                "sum_H_checks": int(len(Hs) - 1),
                "curve_every_1000": [c for c in curve if c[0] % 1000 == 0],
                "snapshots": snaps})
    return out


# --------------------------------------------------------------------- E2 --
def e2():
    n, T, nu = 128, 3200, 1e-5
    beta = Wk.beta_from_nu(nu)
    rho, u = Wk.shear_layer(n)
    out = {"experiment": "e2", "workload": f"D2Q9 shear layer {n}^2, nu = 1e-5 "
           f"(beta = {beta:.8f}), FP64 storage, {T} steps (t = 1)"}
    p = []
    with elbm.Simulation("d2q9", n, n, 1, rho0=rho, u0=u, storage="f64", beta=beta,
                         diag=elbm.DIAG_COUNTS) as sim:
        for t in range(1, T + 1):
            sim.step(1)
            p.append(sim.stats()["n_accept2"] / (n * n))
    p = np.array(p)
    tt = np.arange(1, T + 1) / T
    late = p[tt >= 0.25]
    out.update({"proportion_mean_t_ge_0.25": float(late.mean()),
                "proportion_min_t_ge_0.25": float(late.min()),
                "proportion_max_t_ge_0.25": float(late.max()),
                "proportion_at": {f"{x:.2f}": float(p[int(x * T) - 1])
                                  for x in (0.1, 0.25, 0.5, 0.75, 1.0)},
                "paper": "around 0.5 for most of the time (Fig. 5 discussion)"})
    return out


# --------------------------------------------------------------------- W4 --
def _H_site(f, W):
    return (f * torch.log(f / W[:, None])).sum(0)


W4_SUB = (4, 4, 8)  # sub-lattice strides in x, y, z of the saved fields


def w4_sub_index(n: int) -> np.ndarray:
    """Site indices s = x + n (y + n z) of the sub-lattice x, y = 0, 4, 8, ...,
    z = 0, 8, 16, ... (x fastest): where the precision sweep saves its fields
    for the comparison with the FP64 oracle's reference run."""
    z, y, x = np.meshgrid(np.arange(0, n, W4_SUB[2]), np.arange(0, n, W4_SUB[1]),
                          np.arange(0, n, W4_SUB[0]), indexing="ij")
    return (x + n * (y + n * z)).reshape(-1).astype(np.int64)


def w4(n=256, T=2000, out_dir=None):
    beta = Wk.tgv3d_beta(n)
    rho, u = Wk.taylor_green_3d(n)
    N = n ** 3
    L = [(a, b, c) for c in (0, 1, -1) for b in (0, 1, -1) for a in (0, 1, -1)]
    wa = {0: 2.0 / 3.0, 1: 1.0 / 6.0, -1: 1.0 / 6.0}
    W = torch.tensor([wa[a] * wa[b] * wa[c] for a, b, c in L], dtype=torch.float64,
                     device="cuda")
    ulp = {"f64": 2.0 ** -53, "f32": 2.0 ** -24, "f32dev": 2.0 ** -24, "f16dev": 2.0 ** -11}
    # (storage, site arithmetic): FP64 throughout; mixed (FP32 moments,
    # equilibrium and collision, FP64 alpha evaluation); FP32 throughout
    cases = [("f64", "fp64"), ("f32", "fp64"), ("f32dev", "fp64"), ("f16dev", "fp64"),
             ("f32", "mixed"), ("f32dev", "mixed"), ("f16dev", "mixed"),
             ("f32", "fp32"), ("f16dev", "fp32")]
    out = {"experiment": "w4", "workload": f"D3Q27 Taylor-Green {n}^3, u0 = 0.05, Re = 1600 "
           f"(beta = {beta:.6f}), {T} steps, closed-form alpha", "cases": {}}
    ref = None
    sites = torch.arange(N, dtype=torch.int64, device="cuda")
    sub = torch.as_tensor(w4_sub_index(n), device="cuda")
    if out_dir:
        os.makedirs(out_dir, exist_ok=True)
    for storage, arith in cases:
        name = f"{storage}/{arith}-arith"
        diag = elbm.DIAG_COUNTS | elbm.DIAG_SUMS | (elbm.DIAG_ALPHA if arith == "mixed" else 0)
        with elbm.Simulation("d3q27", n, n, n, rho0=rho, u0=u, storage=storage, fp64=arith,
                             beta=beta, diag=diag) as sim:
            Hsum, neg, kes = [], 0, []
            r, v = sim.moments()
            kes.append([0, _kinetic(r, v)])
            for t in range(0, T, 100):
                sim.step(100)
                st = sim.stats()
                Hsum.append(st["sum_H"])
                neg = max(neg, st["n_negative"])
                r, v = sim.moments()
                kes.append([t + 100, _kinetic(r, v)])
            ke = kes[-1][1]
            if out_dir:
                np.savez(os.path.join(out_dir, f"w4_{storage}_{arith}.npz"), n=n, steps=T,
                         sub_strides=np.array(W4_SUB), rho_sub=r[sub].cpu().numpy(),
                         u_sub=v[:, sub].cpu().numpy(), kinetic_energy=ke,
                         ke_curve=np.array(kes), sum_rho=float(r.sum()))
            # per-site H balance of one more step: pre-collision f(x,T) vs the
            # stored post-collision value written at x
            f0 = sim.populations()
            sim.step(1)
            f1 = sim.gather(sites, 1)
            torch.cuda.synchronize()
            dH = _H_site(f1, W) - _H_site(f0, W)
            tauH = 8 * 2.0 ** -52 * r * torch.clamp(
                (f0 / r * torch.log(f0 / W[:, None]).abs()).sum(0), min=1.0)
            lw = (torch.log(f1 / W[:, None]) + 1.0).abs()
            # change of H from rounding each stored value to the storage format
            if storage.endswith("dev"):
                # s = f/W - rho_ref is rounded: |df| <= W ulp(|s|) / 2, with
                # FP16's subnormal spacing as the floor
                s = (f1 / W[:, None] - 1.0).abs()
                df = W[:, None] * torch.clamp(s, min=2.0 ** -14) * ulp[storage]
            else:
                df = f1.abs() * ulp[storage]
            tauS = (lw * df).sum(0)
            inc_fp64 = int((dH > tauH).sum())
            inc_round = int((dH > tauH + tauS).sum())
            res = {"kinetic_energy": ke, "negative_population_sites_max": neg,
                   "sum_H_increases_per_100_steps": int((np.diff(Hsum) > 0).sum()),
                   "site_H_increase_beyond_fp64_tol": inc_fp64,
                   "site_H_increase_beyond_storage_rounding": inc_round}
            if arith == "mixed":
                # the FP32 rounding of the mixed collision s~ = s + alpha beta
                # (s^eq - s), relative to its operands (s^eq recovered from the
                # step's own alpha: s^eq - s = (s~ - s) / (alpha beta)) and to
                # the FP32 moments that form s^eq
                a = sim.alpha_field()
                s0 = f0 / W[:, None] - 1.0
                s1 = f1 / W[:, None] - 1.0
                d = (s1 - s0) / (a * beta)
                seq = s0 + d
                ws = (W[:, None] * s0.abs()).sum(0)
                ra = W[:, None] * 2.0 ** -24 * (s1.abs() + 2 * d.abs() + 8 * seq.abs() + 8 * ws)
                res["site_H_increase_beyond_storage_and_fp32_arith"] = int(
                    (dH > tauH + tauS + (lw * ra).sum(0)).sum())
                del a, s0, s1, d, seq, ra
            del f0, f1, dH, tauH, tauS, df, lw
            if ref is None:
                ref = (r.clone(), v.clone(), ke)
            else:
                du = (v - ref[1]).abs()
                umax = ref[1].abs().max().item()
                res.update({"u_linf_rel_vs_fp64_gpu": du.max().item() / umax,
                            "u_l2_rel_vs_fp64_gpu": (du.pow(2).sum().sqrt() /
                                                     ref[1].pow(2).sum().sqrt()).item(),
                            "ke_rel_err_vs_fp64_gpu": (ke - ref[2]) / ref[2],
                            "rho_linf_vs_fp64_gpu": (r - ref[0]).abs().max().item()})
            del r, v
            torch.cuda.empty_cache()
        out["cases"][name] = res
        log(f"w4 {name}: {res}")
    return out


def w4cmp(ref_path, run_dir):
    """The precision sweep's fields against the FP64 oracle's reference run
    (an .npz written by the oracle's reference script): velocity L-inf and L2
    errors relative to the largest velocity and to the velocity norm on the
    saved sub-lattice, density L-inf there, kinetic-energy error over the
    whole box, and the kinetic-energy curve.  Reads stored arrays only."""
    refz = np.load(ref_path)
    n = int(refz["n"])
    assert np.array_equal(refz["sub_index"], w4_sub_index(n)), "sub-lattices differ"
    uref, rref, keref = refz["u_sub"], refz["rho_sub"], float(refz["kinetic_energy"])
    curve_ref = refz["ke_curve"]
    out = {"experiment": "w4cmp", "reference": os.path.basename(ref_path),
           "reference_sites_compared": int(uref.shape[1]), "cases": {}}
    for fn in sorted(os.listdir(run_dir)):
        if not (fn.startswith("w4_") and fn.endswith(".npz")):
            continue
        z = np.load(os.path.join(run_dir, fn))
        du = np.abs(z["u_sub"] - uref)
        cur = z["ke_curve"]
        assert np.array_equal(cur[:, 0], curve_ref[:, 0])
        out["cases"][fn[3:-4]] = {
            "u_linf_rel": float(du.max() / np.abs(uref).max()),
            "u_l2_rel": float(np.sqrt((du ** 2).sum() / (uref ** 2).sum())),
            "rho_linf": float(np.abs(z["rho_sub"] - rref).max()),
            "ke_rel_err": float((float(z["kinetic_energy"]) - keref) / keref),
            "ke_curve_max_rel_err": float(np.max(np.abs(cur[:, 1] - curve_ref[:, 1]) /
                                                 curve_ref[:, 1]))}
    return out


# --------------------------------------------------------------------- F3 --
HBM_PEAK_GBS = 8000.0
ELEM_BYTES = {"f64": 8, "f32": 4, "f32dev": 4, "f16dev": 2}


def f3(n=512, newton_n=256, steps=20, tgv_n=128, tgv_steps=2000, copy_mib=0,
       modes=("closed", "bgk", "newton"), lattices=("d3q19", "d3q27"), storage="f32",
       arith="fp64", late_t=0):
    out = {"experiment": "f3", "workload": f"3-D Taylor-Green (u0 = 0.05, Re = 1600), {storage} "
           f"storage, {arith} site arithmetic: step timing at {n}^3 (Newton {newton_n}^3), "
           f"{steps} timed steps after 3 warm-up; limiter statistics at {tgv_n}^3 over "
           f"{tgv_steps} steps", "timing": {}, "tgv": {}}
    if copy_mib:
        # a plain copy of known size, for scaling the HBM counters of a
        # profiler run of this command
        a = torch.empty(copy_mib << 18, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    fields = {}
    for lat in lattices:
        Q = 19 if lat == "d3q19" else 27
        for mode in modes:
            m = newton_n if mode == "newton" else n
            N = m ** 3
            if m not in fields:
                fields[m] = Wk.taylor_green_3d(m)
            rho, u = fields[m]
            with elbm.Simulation(lat, m, m, m, rho0=rho, u0=u, storage=storage, mode=mode,
                                 fp64=arith, beta=Wk.tgv3d_beta(m)) as sim:
                sim.step(3)
                k = steps if mode != "newton" else 3
                ms = _timed_steps(sim, k)
                ms_late = None
                if late_t > 3 + 2 * k and mode != "newton":
                    # the developed flow: as many steps timed again, ending at
                    # t = late_t
                    sim.step(late_t - 3 - 2 * k)
                    ms_late = _timed_steps(sim, k)
            b = ELEM_BYTES[storage]
            gbs = 2.0 * Q * b * N / (ms * 1e-3) / 1e9
            out["timing"][f"{lat}_{mode}"] = {
                "n": m, "ms_per_step": round(ms, 4), "mlups": round(N / (ms * 1e-3) / 1e6, 1),
                "algorithmic_gb_per_step": round(2.0 * Q * b * N / 1e9, 4),
                "hbm_gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
            if ms_late is not None:
                out["timing"][f"{lat}_{mode}"]["late"] = {"t": late_t,
                                                         "ms_per_step": round(ms_late, 4)}
            log(f"f3 {lat} {mode} {m}^3: {out['timing'][f'{lat}_{mode}']}")
            torch.cuda.empty_cache()
    fields.clear()
    for lat in lattices if tgv_steps > 0 else ():
        m = tgv_n
        rho, u = Wk.taylor_green_3d(m)
        rec = []
        with elbm.Simulation(lat, m, m, m, rho0=rho, u0=u, storage=storage, fp64=arith,
                             beta=Wk.tgv3d_beta(m), diag=elbm.DIAG_COUNTS) as sim:
            r, v = sim.moments()
            ke0 = _kinetic(r, v)
            for t in range(250, tgv_steps + 1, 250):
                sim.step(249)
                sim.step(1)
                st = sim.stats()
                r, v = sim.moments()
                torch.cuda.synchronize()
                rec.append({"t": t, "ke_ratio": _kinetic(r, v) / ke0,
                            "alpha_lt2_frac": st["n_alpha_lt2"] / st["n_sites"],
                            "alpha_min": st["alpha_min"],
                            "alphastar_lt2": st["n_alphastar_lt2"]})
        out["tgv"][lat] = rec
        log(f"f3 tgv {lat}: {rec[-1]}")
    if len(out["tgv"]) == 2:
        a19, a27 = out["tgv"]["d3q19"], out["tgv"]["d3q27"]
        out["tgv_ke_ratio_diff_max"] = max(abs(x["ke_ratio"] - y["ke_ratio"])
                                           for x, y in zip(a19, a27))
    T = out["timing"]
    if "d3q19_closed" in T and "d3q27_closed" in T:
        out["q19_closed_over_q27_closed_mlups"] = round(
            T["d3q19_closed"]["mlups"] / T["d3q27_closed"]["mlups"], 3)
    if "d3q19_closed" in T and "d3q19_newton" in T:
        out["q19_closed_over_newton"] = round(
            T["d3q19_closed"]["mlups"] / T["d3q19_newton"]["mlups"], 1)
    return out


def f3burg(n3=512, n2=2048, newton_n=256, steps=20, tgv_n=128, tgv_steps=2000,
           copy_mib=0, cases=None):
    out = {"experiment": "f3burg", "workload": f"Taylor-Green (u0 = 0.05, Re = 1600), FP32 "
           f"storage, FP64 site arithmetic, closed-form alpha unless noted: D3Q27 {n3}^3, "
           f"D2Q9 {n2}^2, Newton at {newton_n}^3; {steps} timed steps after 3 warm-up; "
           f"Taylor-Green {tgv_n}^3 over {tgv_steps} steps", "timing": {}, "tgv": {}}
    if copy_mib:
        a = torch.empty(copy_mib << 18, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    all_cases = [("d3q27", n3, "closed", "burg"), ("d3q27", n3, "closed", "boltzmann"),
                 ("d2q9", n2, "closed", "burg"), ("d2q9", n2, "closed", "boltzmann"),
                 ("d3q27", newton_n, "newton", "burg")]
    for lat, m, mode, ent in all_cases:
        if cases and f"{lat}_{mode}_{ent}" not in cases:
            continue
        Q = 27 if lat == "d3q27" else 9
        if lat == "d3q27":
            rho, u = Wk.taylor_green_3d(m)
            shape, beta = (m, m, m), Wk.tgv3d_beta(m)
        else:
            rho, u = Wk.taylor_green_2d(m)
            shape, beta = (m, m, 1), Wk.beta_from_nu(0.05 * m / (2.0 * math.pi) / 1600.0)
        N = int(np.prod(shape))
        with elbm.Simulation(lat, *shape, rho0=rho, u0=u, storage="f32", mode=mode, beta=beta,
                             entropy=ent) as sim:
            del rho, u
            sim.step(3)
            ms = _timed_steps(sim, steps if mode != "newton" else 3)
        gbs = 2.0 * Q * 4 * N / (ms * 1e-3) / 1e9
        key = f"{lat}_{mode}_{ent}"
        out["timing"][key] = {"n": m, "ms_per_step": round(ms, 4),
                              "mlups": round(N / (ms * 1e-3) / 1e6, 1),
                              "hbm_gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
        log(f"f3burg {key}: {out['timing'][key]}")
        torch.cuda.empty_cache()
    for ent in ("burg", "boltzmann") if tgv_steps > 0 else ():
        m = tgv_n
        rho, u = Wk.taylor_green_3d(m)
        rec = []
        with elbm.Simulation("d3q27", m, m, m, rho0=rho, u0=u, storage="f32",
                             beta=Wk.tgv3d_beta(m), diag=elbm.DIAG_COUNTS, entropy=ent) as sim:
            r, v = sim.moments()
            ke0 = _kinetic(r, v)
            for t in range(250, tgv_steps + 1, 250):
                sim.step(249)
                sim.step(1)
                st = sim.stats()
                r, v = sim.moments()
                torch.cuda.synchronize()
                rec.append({"t": t, "ke_ratio": _kinetic(r, v) / ke0,
                            "alpha_lt2_frac": st["n_alpha_lt2"] / st["n_sites"],
                            "alpha_min": st["alpha_min"],
                            "alphastar_lt2": st["n_alphastar_lt2"]})
        out["tgv"][ent] = rec
        log(f"f3burg tgv {ent}: {rec[-1]}")
    T = out["timing"]
    for lat in ("d3q27", "d2q9"):
        a, b = T.get(f"{lat}_closed_burg"), T.get(f"{lat}_closed_boltzmann")
        if a and b:
            out[f"{lat}_burg_over_boltzmann_time"] = round(a["ms_per_step"] / b["ms_per_step"], 3)
    if "d3q27_closed_burg" in T and "d3q27_newton_burg" in T:
        out["burg_closed_over_newton"] = round(
            T["d3q27_closed_burg"]["mlups"] / T["d3q27_newton_burg"]["mlups"], 1)
    return out


# -------------------------------------------------------------------- W5p --
def w5p(n_req=64, rate=20.0, max_active=8, round_steps=50, preempt_rounds=20):
    """The W5 stream through a server whose slots are the bottleneck, once
    first come first served and once with preemption (long residents moved
    out to host memory so that queued requests get in)."""
    from paper_1904_00866_amd import serving
    reqs = Wk.serving_stream(n_req, rate=rate)
    out = {"experiment": "w5p",
           "workload": f"{n_req} D2Q9 shear-layer requests at {rate}/s (seed 20250101), "
                       f"{max_active} slots, rounds of {round_steps} steps", "runs": {}}
    for name, pr in (("fcfs", 0), (f"preempt_{preempt_rounds}", preempt_rounds)):
        res = serving.run_stream(reqs, max_active=max_active, round_steps=round_steps,
                                 preempt_rounds=pr, log=log)
        lat = np.array(res["latency_s"])
        work = np.array([r["n"] * r["n"] * r["steps"] for r in reqs], dtype=float)
        small = work <= np.median(work)
        out["runs"][name] = {
            "p50_s": res["p50_s"], "p99_s": res["p99_s"], "mean_s": res["mean_s"],
            "max_s": res["max_s"], "queue_p50_s": res["queue_p50_s"],
            "queue_p99_s": res["queue_p99_s"], "mlups": res["mlups"], "span_s": res["span_s"],
            "preemptions": res["preemptions"], "completed": res["completed"],
            "failed": res["failed"],
            "p50_smaller_half_s": float(np.percentile(lat[small], 50)),
            "p50_larger_half_s": float(np.percentile(lat[~small], 50))}
        log(f"w5p {name}: {out['runs'][name]}")
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("which", nargs="+",
                    choices=["w1", "w2", "e2", "w4", "w4cmp", "w5p", "f3", "f3burg"])
    ap.add_argument("--w4-out", default=None,
                    help="w4: directory for the fields on the comparison sub-lattice")
    ap.add_argument("--w4-ref", default=None,
                    help="w4cmp: the FP64 oracle reference (.npz of the reference script)")
    ap.add_argument("--w2-steps", type=int, default=20000)
    ap.add_argument("--f3-n", type=int, default=512)
    ap.add_argument("--f3-steps", type=int, default=20)
    ap.add_argument("--f3-tgv-steps", type=int, default=2000)
    ap.add_argument("--f3-modes", default="closed,bgk,newton")
    ap.add_argument("--f3-lattices", default="d3q19,d3q27")
    ap.add_argument("--f3-storage", default="f32", choices=sorted(ELEM_BYTES))
    ap.add_argument("--f3-arith", default="fp64", choices=["fp64", "fp32", "mixed"])
    ap.add_argument("--f3-late-t", type=int, default=0,
                    help="also time the steps that end at this t (0: no)")
    ap.add_argument("--f3burg-cases", default="",
                    help="comma list of lattice_mode_entropy cases (default: all)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one torch copy of this many MiB first (HBM counter scale)")
    args = ap.parse_args()
    if args.which == ["w4cmp"]:
        # reads stored arrays only (no GPU)
        print(json.dumps(w4cmp(args.w4_ref, args.w4_out)), flush=True)
        return 0
    if not torch.cuda.is_available():
        print("experiments.py needs a GPU", file=sys.stderr)
        return 1
    elbm.lib()
    for w in args.which:
        t0 = time.time()
        res = {"w1": w1, "e2": e2, "w4": lambda: w4(out_dir=args.w4_out), "w5p": w5p,
               "f3burg": lambda: f3burg(n3=args.f3_n, steps=args.f3_steps,
                                        tgv_steps=args.f3_tgv_steps, copy_mib=args.copy_probe_mib,
                                        cases=[c for c in args.f3burg_cases.split(",") if c]),
               "f3": lambda: f3(n=args.f3_n, steps=args.f3_steps,
                                tgv_steps=args.f3_tgv_steps, copy_mib=args.copy_probe_mib,
                                modes=tuple(args.f3_modes.split(",")),
                                lattices=tuple(args.f3_lattices.split(",")),
                                storage=args.f3_storage, arith=args.f3_arith,
                                late_t=args.f3_late_t)
               }.get(w, lambda: w2(args.w2_steps))()
        res["wall_s"] = round(time.time() - t0, 1)
        print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
