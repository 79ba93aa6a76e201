"""Test-side reference material written independently of the oracle and of
the HIP library: textbook lattice tables, a Lagrange-multiplier minimisation
of the entropy, and high-precision (mpmath) entropies."""
from __future__ import annotations

import itertools

import mpmath as mp
import numpy as np

# Direction order of the C ABI: i = d(cx) + 3 d(cy) + 9 d(cz), d(0)=0, d(1)=1, d(-1)=2.
_DIGIT = {0: 0, 1: 1, 2: -1}


def dim(lat: int) -> int:
    """Dimension of a lattice code: 1, 2, 3 (D1Q3, D2Q9, D3Q27) or 19 (D3Q19)."""
    return 3 if lat == 19 else lat


def abi_velocities(D: int) -> np.ndarray:
    if D == 19:
        # D3Q19: the D3Q27 directions without the 8 corners, in D3Q27 order
        c27 = abi_velocities(3)
        return c27[np.count_nonzero(c27, axis=1) <= 2]
    Q = 3 ** D
    c = np.zeros((Q, 3), dtype=np.int64)
    for i in range(Q):
        rem = i
        for a in range(D):
            c[i, a] = _DIGIT[rem % 3]
            rem //= 3
    return c


# Textbook weights: D1Q3 (2/3, 1/6, 1/6); D2Q9 rest 4/9, axis 1/9, diagonal 1/36;
# D3Q27 rest 8/27, face 2/27, edge 1/54, corner 1/216.  Indexed by the number
# of non-zero velocity components.
TEXTBOOK_W = {1: {0: (2, 3), 1: (1, 6)},
              2: {0: (4, 9), 1: (1, 9), 2: (1, 36)},
              3: {0: (8, 27), 1: (2, 27), 2: (1, 54), 3: (1, 216)},
              19: {0: (1, 3), 1: (1, 18), 2: (1, 36)}}  # D3Q19 rest, face, edge


def textbook_weights(D: int) -> np.ndarray:
    c = abi_velocities(D)
    return np.array([TEXTBOOK_W[D][int(np.count_nonzero(ci))][0] /
                     TEXTBOOK_W[D][int(np.count_nonzero(ci))][1] for ci in c])


def lagrange_equilibrium(D: int, rho: float, u, iters: int = 60) -> np.ndarray:
    """Minimise H(g) = sum g ln(g/W) subject to sum g = rho, sum c g = rho u by
    Newton's method on the Lagrange multipliers: g_i = W_i exp(l0 + l.c_i).
    D is a lattice code (19: D3Q19)."""
    lat, D = D, dim(D)
    c = abi_velocities(lat)[:, :D].astype(np.float64)
    W = textbook_weights(lat)
    A = np.hstack([np.ones((c.shape[0], 1)), c])  # [Q, D+1]
    target = np.concatenate([[rho], rho * np.asarray(u[:D], dtype=np.float64)])
    lam = np.zeros(D + 1)
    lam[0] = np.log(rho)
    for _ in range(iters):
        g = W * np.exp(A @ lam)
        r = A.T @ g - target
        J = A.T @ (g[:, None] * A)
        step = np.linalg.solve(J, r)
        lam -= step
        if np.max(np.abs(step)) < 1e-17:
            break
    return W * np.exp(A @ lam)


def mp_lagrange_equilibrium(D: int, rho, u, dps: int = 50):
    """Same minimisation in mpmath arithmetic (returns a list of mpf)."""
    lat, D = D, dim(D)
    with mp.workdps(dps):
        c = abi_velocities(lat)[:, :D]
        W = mp_weights(lat)
        rho = mp.mpf(rho)
        uu = [mp.mpf(x) for x in u[:D]]
        lam = [mp.log(rho)] + [mp.mpf(0)] * D
        Q = len(c)
        for _ in range(200):
            g = [W[i] * mp.exp(lam[0] + sum(lam[a + 1] * int(c[i, a]) for a in range(D)))
                 for i in range(Q)]
            rows = [[mp.mpf(1)] + [mp.mpf(int(c[i, a])) for a in range(D)] for i in range(Q)]
            r = [sum(g) - rho] + [sum(g[i] * rows[i][a + 1] for i in range(Q)) - rho * uu[a]
                                  for a in range(D)]
            J = mp.matrix(D + 1, D + 1)
            for p in range(D + 1):
                for q in range(D + 1):
                    J[p, q] = sum(g[i] * rows[i][p] * rows[i][q] for i in range(Q))
            step = mp.lu_solve(J, mp.matrix(r))
            lam = [lam[k] - step[k] for k in range(D + 1)]
            if max(abs(step[k]) for k in range(D + 1)) < mp.mpf(10) ** (-dps + 5):
                break
        return [W[i] * mp.exp(lam[0] + sum(lam[a + 1] * int(c[i, a]) for a in range(D)))
                for i in range(Q)]


def mp_weights(D: int):
    c = abi_velocities(D)
    out = []
    for ci in c:
        num, den = TEXTBOOK_W[D][int(np.count_nonzero(ci))]
        out.append(mp.mpf(num) / mp.mpf(den))
    return out


def mp_H(f, W) -> mp.mpf:
    """Eq. (3) in mpmath: sum f ln(f/W), 0 ln 0 = 0."""
    h = mp.mpf(0)
    for fi, wi in zip(f, W):
        fi = mp.mpf(fi)
        if fi < 0:
            raise ValueError("negative population")
        if fi > 0:
            h += fi * mp.log(fi / wi)
    return h


def mp_G(D: int, f, alpha, dps: int = 50) -> mp.mpf:
    """H(f + alpha (f^eq - f)) - H(f) with everything in mpmath: the
    equilibrium from the multiplier minimisation, f taken exactly as given."""
    with mp.workdps(dps):
        fm = [mp.mpf(float(v)) for v in f]
        rho = sum(fm)
        c = abi_velocities(D)
        u = [sum(fm[i] * int(c[i, a]) for i in range(len(fm))) / rho for a in range(dim(D))]
        feq = mp_lagrange_equilibrium(D, rho, u, dps)
        W = mp_weights(D)
        a = mp.mpf(float(alpha))
        fs = [fm[i] + a * (feq[i] - fm[i]) for i in range(len(fm))]
        # the component that defines alpha_max is zero up to the rounding of
        # the double-precision alpha: read values of that size as zero
        floor = -mp.mpf(1e-13) * max(fm)
        fs = [max(v, mp.mpf(0)) if v > floor else v for v in fs]
        return mp_H(fs, W) - mp_H(fm, W)


def mp_alpha_closed(D: int, f, dps: int = 60, full: bool = False):
    """The closed-form alpha in mpmath: alpha_* = min(2, alpha_max)
    (Eq. (8), alpha_max = 1 + 1 / max_i x_i over x_i > 0), accepted when
    H(f*(alpha_*)) <= H(f), else Eq. (9) clipped to [1, alpha_*]; the
    equilibrium from the multiplier minimisation, f taken exactly as given.
    full=True returns (alpha_*, alpha, H(f*(alpha_*)) - H(f),
    H(f*(alpha_*)) - H(f^eq)), each entropy from Eq. (3) literally."""
    with mp.workdps(dps):
        fm = [mp.mpf(float(v)) for v in f]
        rho = sum(fm)
        c = abi_velocities(D)
        u = [sum(fm[i] * int(c[i, a]) for i in range(len(fm))) / rho for a in range(dim(D))]
        feq = mp_lagrange_equilibrium(D, rho, u, dps)
        W = mp_weights(D)
        xmax = max(fm[i] / feq[i] - 1 for i in range(len(fm)))
        astar = mp.mpf(2) if xmax <= 1 else 1 + 1 / xmax
        fs = [fm[i] + astar * (feq[i] - fm[i]) for i in range(len(fm))]
        # at alpha_* = alpha_max one component of f*(alpha_*) is zero, up to
        # the working precision's rounding: read it as zero
        floor = -mp.mpf(10) ** (-dps + 10) * max(fm)
        fs = [max(v, mp.mpf(0)) if v > floor else v for v in fs]
        Hs, H0, He = mp_H(fs, W), mp_H(fm, W), mp_H(feq, W)
        Gs, Ds = Hs - H0, Hs - He
        if Gs <= 0:
            alpha = astar
        else:
            alpha = min(max(astar + Gs / Ds * (1 - astar), mp.mpf(1)), astar)
        return (astar, alpha, Gs, Ds) if full else alpha


def mp_root(D: int, f, lo, hi, dps: int = 40, iters: int = 80):
    """Nontrivial root of G on [lo, hi] by mpmath bisection (G(lo) <= 0 < G(hi))."""
    with mp.workdps(dps):
        fm = [mp.mpf(float(v)) for v in f]
        rho = sum(fm)
        c = abi_velocities(D)
        u = [sum(fm[i] * int(c[i, a]) for i in range(len(fm))) / rho for a in range(dim(D))]
        feq = mp_lagrange_equilibrium(D, rho, u, dps)
        W = mp_weights(D)
        H0 = mp_H(fm, W)

        def G(a):
            fs = [fm[i] + a * (feq[i] - fm[i]) for i in range(len(fm))]
            fs = [max(v, mp.mpf(0)) for v in fs]
            return mp_H(fs, W) - H0

        lo, hi = mp.mpf(lo), mp.mpf(hi)
        for _ in range(iters):
            mid = (lo + hi) / 2
            if G(mid) > 0:
                hi = mid
            else:
                lo = mid
        return lo


def near_equilibrium_state(D: int, rho: float, u, eps: float, rng, feq_fn) -> np.ndarray:
    """f = f^eq (1 + eps xi) with xi projected so that f keeps the moments of
    f^eq (feq_fn supplies the equilibrium; the projection uses only 1 and c)."""
    c = abi_velocities(D)[:, :dim(D)].astype(np.float64)
    feq = feq_fn(D, rho, u)
    A = np.hstack([np.ones((c.shape[0], 1)), c])
    xi = rng.standard_normal(c.shape[0])
    # remove the part of feq*xi that changes the moments: solve A^T (feq xi - feq A m) = 0
    M = A.T @ (feq[:, None] * A)
    m = np.linalg.solve(M, A.T @ (feq * xi))
    xi = xi - A @ m
    xi /= np.max(np.abs(xi))
    return feq * (1.0 + eps * xi)


# ---- Burg's entropy H(f) = -sum_i W_i ln(f_i / W_i) ----------------------
def burg_equilibrium(D: int, rho: float, u, iters: int = 100) -> np.ndarray:
    """Minimise Burg's entropy under the mass and momentum constraints by
    Newton's method on the multipliers of g_i = W_i / (mu . (1, c_i)), with
    step halving that keeps every mu . (1, c_i) positive (float64).  D is a
    lattice code."""
    lat, D = D, dim(D)
    c = abi_velocities(lat)[:, :D].astype(np.float64)
    W = textbook_weights(lat)
    A = np.hstack([np.ones((c.shape[0], 1)), c])
    b = np.concatenate([[rho], rho * np.asarray(u[:D], dtype=np.float64)])
    mu = np.zeros(D + 1)
    mu[0] = 1.0 / rho
    for _ in range(iters):
        d = A @ mu
        r = A.T @ (W / d) - b
        J = -(A.T @ ((W / d ** 2)[:, None] * A))
        step = np.linalg.solve(J, r)
        t = 1.0
        while np.any(A @ (mu - t * step) <= 0):
            t *= 0.5
        mu = mu - t * step
        if np.max(np.abs(t * step)) < 1e-17:
            break
    return W / (A @ mu)


def mp_burg_equilibrium(D: int, rho, u, dps: int = 50):
    """The same minimisation in mpmath arithmetic (list of mpf)."""
    lat, D = D, dim(D)
    with mp.workdps(dps):
        c = abi_velocities(lat)[:, :D]
        W = mp_weights(lat)
        Q = len(c)
        rho = mp.mpf(rho)
        b = [rho] + [rho * mp.mpf(x) for x in u[:D]]
        rows = [[mp.mpf(1)] + [mp.mpf(int(c[i, a])) for a in range(D)] for i in range(Q)]
        mu = [1 / rho] + [mp.mpf(0)] * D
        for _ in range(200):
            d = [sum(mu[k] * rows[i][k] for k in range(D + 1)) for i in range(Q)]
            r = [sum(W[i] * rows[i][k] / d[i] for i in range(Q)) - b[k] for k in range(D + 1)]
            J = mp.matrix(D + 1, D + 1)
            for p in range(D + 1):
                for q in range(D + 1):
                    J[p, q] = -sum(W[i] * rows[i][p] * rows[i][q] / d[i] ** 2 for i in range(Q))
            step = mp.lu_solve(J, mp.matrix(r))
            t = mp.mpf(1)
            while any(sum((mu[k] - t * step[k]) * rows[i][k] for k in range(D + 1)) <= 0
                      for i in range(Q)):
                t /= 2
            mu = [mu[k] - t * step[k] for k in range(D + 1)]
            if max(abs(step[k]) for k in range(D + 1)) < mp.mpf(10) ** (-dps + 5):
                break
        return [W[i] / sum(mu[k] * rows[i][k] for k in range(D + 1)) for i in range(Q)]


def mp_H_burg(f, W) -> mp.mpf:
    """Burg's entropy in mpmath: -sum W ln(f/W); +inf at a zero population."""
    h = mp.mpf(0)
    for fi, wi in zip(f, W):
        fi = mp.mpf(fi)
        if fi < 0:
            raise ValueError("negative population")
        if fi == 0:
            return mp.inf
        h -= wi * mp.log(fi / wi)
    return h


def _mp_state_burg(D, f, dps):
    fm = [mp.mpf(float(v)) for v in f]
    rho = sum(fm)
    c = abi_velocities(D)
    u = [sum(fm[i] * int(c[i, a]) for i in range(len(fm))) / rho for a in range(dim(D))]
    return fm, mp_burg_equilibrium(D, rho, u, dps), mp_weights(D)


def mp_G_burg(D: int, f, alpha, dps: int = 50) -> mp.mpf:
    """H(f + alpha (f^eq - f)) - H(f) for Burg's entropy, all in mpmath."""
    with mp.workdps(dps):
        fm, feq, W = _mp_state_burg(D, f, dps)
        a = mp.mpf(float(alpha))
        fs = [fm[i] + a * (feq[i] - fm[i]) for i in range(len(fm))]
        return mp_H_burg(fs, W) - mp_H_burg(fm, W)


def mp_root_burg(D: int, f, lo, hi, dps: int = 40, iters: int = 80):
    """Nontrivial root of Burg's G on [lo, hi] by mpmath bisection."""
    with mp.workdps(dps):
        fm, feq, W = _mp_state_burg(D, f, dps)
        H0 = mp_H_burg(fm, W)

        def G(a):
            fs = [fm[i] + a * (feq[i] - fm[i]) for i in range(len(fm))]
            if min(fs) <= 0:
                return mp.inf
            return mp_H_burg(fs, W) - H0

        lo, hi = mp.mpf(lo), mp.mpf(hi)
        for _ in range(iters):
            mid = (lo + hi) / 2
            if G(mid) > 0:
                hi = mid
            else:
                lo = mid
        return lo


def check_collision_invariants(orc, lat, f0, f1, ag, W, rng_seed):
    """Per-site invariants of one collision f0 -> f1 at alpha = ag (FP64,
    recomputed on the CPU): positive populations; mass and momentum to
    1e-14 rho; the discrete H-theorem H(f1) <= H(f0) up to 8 eps rho
    max(1, sum_i (f_i / rho) |ln(f_i / W_i)|) of rounding; and, where ag is
    given, Eq. (7) G(ag) = H(f*(ag)) - H(f0) <= 1e-14 rho on 200 sampled
    sites, G evaluated by the oracle."""
    assert np.all(f1 > 0)
    c, _ = orc.lattice(lat)
    rho = f0.sum(0)
    assert np.all(np.abs(f1.sum(0) - rho) <= 1e-14 * rho)
    for a in range(c.shape[1]):
        assert np.all(np.abs(c[:, a] @ f1 - c[:, a] @ f0) <= 1e-14 * rho)
    if ag is not None:
        N = f0.shape[1]
        for s in np.random.default_rng(rng_seed).choice(N, min(N, 200), replace=False):
            assert orc.G(lat, f0[:, s], ag[s]) <= 1e-14 * rho[s]
    Hs = lambda f: (f * np.log(f / W)).sum(0)
    tau = 8 * 2.0 ** -52 * rho * np.maximum(1.0, (f0 / rho * np.abs(np.log(f0 / W))).sum(0))
    assert np.all(Hs(f1) - Hs(f0) <= tau)


def entropy_scale(f, W) -> float:
    """sum_x sum_i |f_i ln(f_i / W_i)|: the size of the terms whose sum is
    sum_x H(f(x)) (Eq. (3) summed as in Eq. (6)); that sum cancels between
    sites with rho above and below 1, so its rounding is relative to this
    scale, not to the sum itself."""
    W = np.asarray(W, dtype=np.float64).reshape(-1, 1)
    return float(np.sum(np.abs(f * np.log(f / W))))
