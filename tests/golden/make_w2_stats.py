"""Statistics of the FP64 oracle on the 1024^2 doubly periodic shear layer
(u0 = 0.04, kappa = 80, delta = 0.05, Re = 3e4), closed-form alpha
(Eqs. (8)-(9)), over its first 2000 steps: every 100 steps, of the
pre-collision state f(x, t),
  - the share of sites with alpha < 2 and with alpha_* = 2 accepted (the
    quantity of the Fig. 5 discussion),
  - the smallest alpha,
  - the kinetic energy 1/2 sum_x rho |u|^2.

    python tests/golden/make_w2_stats.py [--threads 8]

Calls only the CPU oracle; writes tests/golden/w2_shear_1024_stats.json
(2.1e9 site updates: a few minutes on eight cores).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1904_00866_amd import workloads as Wk  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--every", type=int, default=100)
    ap.add_argument("--threads", type=int, default=8)
    ap.add_argument("--out", default=os.path.join(HERE, "w2_shear_1024_stats.json"))
    a = ap.parse_args()
    n = a.n
    beta = Wk.shear_beta(n)
    rho0, u0 = Wk.shear_layer(n)
    cfg = oracle.Config(D=2, nx=n, ny=n, beta=beta, mode="closed", nthreads=a.threads)
    f = oracle.init(cfg, rho0, u0)
    rows = []
    t0 = time.time()
    t = 0
    while t <= a.steps - 1:
        want = t % a.every == 0
        if want:
            r, u = oracle.moments(cfg, f)
            ke = 0.5 * float((r * (u * u).sum(0)).sum())
            fn, _, d = oracle.step(cfg, f, want_diag=True)
            rows.append({"t": t, "frac_alpha_lt2": d["n_alpha_lt2"] / n ** 2,
                         "frac_accept2": d["n_accept2"] / n ** 2,
                         "alpha_min": d["alpha_min"], "kinetic_energy": ke})
            print(f"[w2 stats] {rows[-1]} ({time.time() - t0:.0f} s)", flush=True)
        else:
            fn, _, _ = oracle.step(cfg, f)
        f = fn
        t += 1
    out = {"_comment": "FP64 oracle statistics of the pre-collision state f(x, t) of the "
                       "1024^2 doubly periodic shear layer (u0 = 0.04, kappa = 80, "
                       "delta = 0.05, Re = 3e4, beta from nu = u0 n / Re), closed-form "
                       "alpha; written by tests/golden/make_w2_stats.py",
           "n": n, "beta": beta, "every": a.every, "rows": rows}
    with open(a.out, "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"[w2 stats] wrote {a.out} in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
