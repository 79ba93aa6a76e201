"""FP64 oracle reference of the precision sweep: the D3Q27 Taylor-Green vortex
at 256^3, Re = 1600, closed-form alpha (Eqs. (8)-(9)), 2000 steps.

    python tests/golden/make_w4_reference.py [--n 256] [--steps 2000]
           [--threads 6] [--out tests/golden/w4_reference_256.npz]

It calls only the CPU oracle (FP64, OpenMP over sites).  The output is large
and stays out of version control; it holds, for the state f(x, T):
  * rho and u on the sub-lattice x, y = 0, 4, 8, ..., z = 0, 8, 16, ...
    (every 4th site in x and y, every 8th in z; site order x fastest);
  * over the whole box: kinetic energy 1/2 sum rho |u|^2, sum rho, max |u|,
    and the kinetic energy every 100 steps;
  * the oracle's domain diagnostics of the last step.
At 256^3 this is 3.4e10 site updates: about two hours on six cores.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1904_00866_amd import workloads as Wk  # noqa: E402

SUB = (4, 4, 8)  # sub-lattice strides in x, y, z


def sub_index(n: int) -> np.ndarray:
    """Site indices s = x + n (y + n z) of the sub-lattice, x fastest."""
    z, y, x = np.meshgrid(np.arange(0, n, SUB[2]), np.arange(0, n, SUB[1]),
                          np.arange(0, n, SUB[0]), indexing="ij")
    return (x + n * (y + n * z)).reshape(-1).astype(np.int64)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--every", type=int, default=100)
    ap.add_argument("--threads", type=int, default=6)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                  "w4_reference_256.npz"))
    a = ap.parse_args()
    n, T = a.n, a.steps
    beta = Wk.tgv3d_beta(n)
    rho0, u0 = Wk.taylor_green_3d(n)
    cfg = oracle.Config(D=3, nx=n, ny=n, nz=n, beta=beta, mode="closed", nthreads=a.threads)
    f = oracle.init(cfg, rho0, u0)
    del rho0, u0

    ke_curve = []

    def ke_of(ff):
        r, u = oracle.moments(cfg, ff)
        return 0.5 * float((r * (u * u).sum(0)).sum()), r, u

    ke_curve.append((0, ke_of(f)[0]))
    t0 = time.time()

    def cb(t, ff):
        if t % a.every == 0:
            ke_curve.append((t, ke_of(ff)[0]))
            print(f"[w4 ref] t={t} ke={ke_curve[-1][1]:.12e} "
                  f"elapsed {time.time() - t0:.0f} s", flush=True)

    # the last step with diagnostics (pre-collision state of step T-1)
    f, _, _ = oracle.run(cfg, f, T - 1, callback=cb)
    fT, _, dg = oracle.step(cfg, f, want_diag=True)
    del f
    cb(T, fT)
    ke, r, u = ke_of(fT)
    idx = sub_index(n)
    np.savez(a.out, n=n, steps=T, beta=beta, sub_strides=np.array(SUB), sub_index=idx,
             rho_sub=r[idx], u_sub=u[:, idx], kinetic_energy=ke,
             sum_rho=float(r.sum()), u_max=float(np.abs(u).max()),
             ke_curve=np.array(ke_curve),
             diag_last_step=np.array([dg["n_accept2"], dg["n_alphastar_lt2"],
                                      dg["n_alpha_lt2"], dg["n_negative"]]),
             sum_H_last_step=dg["sum_H"], wall_seconds=time.time() - t0,
             threads=a.threads)
    print(f"[w4 ref] wrote {a.out}: ke {ke:.12e}, {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
