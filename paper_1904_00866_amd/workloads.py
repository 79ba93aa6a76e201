"""Seeded synthetic inputs: analytic initial fields and random states.

This module holds the workload definitions shared by the tests, the
benchmark and the oracle's checks.  It contains none of the method's
arithmetic (no equilibrium, entropy or alpha): it only produces density and
velocity fields, or arbitrary positive population arrays, for each side to
start from.  Sites are ordered s = x + nx*(y + ny*z); fields are numpy
float64, rho[N] and u[D, N].
"""
from __future__ import annotations

import math

import numpy as np


def beta_from_nu(nu: float) -> float:
    """Eq. (2) in lattice units (delta_t = 1, c_s^2 = 1/3)."""
    return (1.0 / 3.0) / (2.0 * nu + 1.0 / 3.0)


def _grid(nx, ny=1, nz=1):
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.reshape(-1).astype(np.float64), y.reshape(-1).astype(np.float64), \
        z.reshape(-1).astype(np.float64)


def taylor_green_2d(n: int, u0: float = 0.05, rho0: float = 1.0):
    """D2Q9 Taylor-Green vortex on an n x n periodic box, wavenumber 2 pi/n:
    u_x = -u0 cos(kx) sin(ky), u_y = u0 sin(kx) cos(ky), and the density
    carrying the incompressible pressure, rho = rho0 - (3/4) rho0 u0^2
    (cos 2kx + cos 2ky)."""
    x, y, _ = _grid(n, n)
    k = 2.0 * math.pi / n
    ux = -u0 * np.cos(k * x) * np.sin(k * y)
    uy = u0 * np.sin(k * x) * np.cos(k * y)
    rho = rho0 - 0.75 * rho0 * u0 * u0 * (np.cos(2 * k * x) + np.cos(2 * k * y))
    return rho, np.stack([ux, uy])


def taylor_green_3d(n: int, u0: float = 0.05, rho0: float = 1.0):
    """D3Q27 Taylor-Green vortex on an n^3 periodic box, k = 2 pi/n:
    u = u0 (sin kx cos ky cos kz, -cos kx sin ky cos kz, 0),
    rho = rho0 + (3 u0^2/16)(cos 2kx + cos 2ky)(cos 2kz + 2)."""
    x, y, z = _grid(n, n, n)
    k = 2.0 * math.pi / n
    ux = u0 * np.sin(k * x) * np.cos(k * y) * np.cos(k * z)
    uy = -u0 * np.cos(k * x) * np.sin(k * y) * np.cos(k * z)
    uz = np.zeros_like(ux)
    rho = rho0 + rho0 * (3.0 * u0 * u0 / 16.0) * (np.cos(2 * k * x) + np.cos(2 * k * y)) \
        * (np.cos(2 * k * z) + 2.0)
    return rho, np.stack([ux, uy, uz])


def tgv3d_beta(n: int, u0: float = 0.05, re: float = 1600.0) -> float:
    """beta of the 3-D Taylor-Green vortex at Reynolds number re with length
    scale L = n / (2 pi): nu = u0 L / re."""
    return beta_from_nu(u0 * (n / (2.0 * math.pi)) / re)


def shear_layer(n: int, u0: float = 0.04, kappa: float = 80.0, delta: float = 0.05):
    """Doubly periodic shear layer on the unit square sampled at x = i/n,
    y = j/n: u_x = u0 tanh(kappa (y - 1/4)) for y <= 1/2 and
    u0 tanh(kappa (3/4 - y)) above, u_y = delta u0 sin(2 pi (x + 1/4)),
    rho = 1 (the double shear flow of the paper's second test)."""
    x, y, _ = _grid(n, n)
    X, Y = x / n, y / n
    ux = np.where(Y <= 0.5, u0 * np.tanh(kappa * (Y - 0.25)), u0 * np.tanh(kappa * (0.75 - Y)))
    uy = delta * u0 * np.sin(2.0 * math.pi * (X + 0.25))
    return np.ones_like(X), np.stack([ux, uy])


def shear_beta(n: int, u0: float = 0.04, re: float = 3e4) -> float:
    """beta for the shear layer with nu = u0 n / re."""
    return beta_from_nu(u0 * n / re)


def shock_tube(n: int = 800, rho_left: float = 1.5, rho_right: float = 0.75):
    """1-D shock tube: rho = rho_left on sites x <= n/2, rho_right above, u = 0."""
    x, _, _ = _grid(n)
    rho = np.where(x <= n // 2, rho_left, rho_right)
    return rho, np.zeros((1, n))


def random_velocity_field(D: int, N: int, umax: float, seed: int, rho_spread: float = 0.05):
    """rho in [1 - spread, 1 + spread], each u_a uniform in [-umax, umax]."""
    rng = np.random.default_rng(seed)
    rho = 1.0 + rho_spread * (2.0 * rng.random(N) - 1.0)
    u = umax * (2.0 * rng.random((D, N)) - 1.0)
    return rho, u


def random_populations(weights, N: int, eps: float, seed: int, tilt: float = 0.1,
                       log_uniform_eps: bool = False):
    """Positive, non-equilibrium populations for N sites:
        f[i, s] = w_i rho_s (1 + e_s xi_is) (1 + t_s tau_i),
    with the weight profile w given by the caller, rho_s uniform in
    [0.9, 1.1], xi_is uniform in [-1, 1], tau_i = -1 ... 1 evenly over the Q
    directions (so t_s uniform in [-tilt, tilt] adds momentum), and e_s = eps,
    or log-uniform in [eps/1000, eps] with log_uniform_eps."""
    rng = np.random.default_rng(seed)
    w = np.asarray(weights, dtype=np.float64)
    Q = w.size
    rho = 1.0 + 0.1 * (2.0 * rng.random(N) - 1.0)
    e = eps * 10.0 ** (-3.0 * rng.random(N)) if log_uniform_eps else np.full(N, eps)
    xi = 2.0 * rng.random((Q, N)) - 1.0
    t = tilt * (2.0 * rng.random(N) - 1.0)
    tau = np.linspace(-1.0, 1.0, Q)
    f = w[:, None] * rho[None, :] * (1.0 + e[None, :] * xi) * (1.0 + t[None, :] * tau[:, None])
    return np.ascontiguousarray(f)


SERVING_SIZES = (128, 256, 512, 1024, 2048)


def serving_stream(n_req: int, rate: float = 20.0, seed: int = 20250101,
                   sizes=SERVING_SIZES, re_range=(1e3, 1e5), steps_range=(1000, 20000),
                   storages=("f32", "f16dev")):
    """Seeded request stream of D2Q9 doubly periodic shear-layer solves:
    Poisson arrivals at `rate` per second (exponential gaps), box edge
    uniform over `sizes`, Reynolds number log-uniform over `re_range`, step
    count uniform over the integers of `steps_range`, storage uniform over
    `storages`.  Each request gets beta from nu = 0.04 n / Re (shear_beta)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(n_req):
        t += rng.exponential(1.0 / rate)
        n = int(sizes[rng.integers(0, len(sizes))])
        re = float(np.exp(rng.uniform(math.log(re_range[0]), math.log(re_range[1]))))
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        storage = storages[int(rng.integers(0, len(storages)))]
        out.append(dict(k=k, arrival=t, n=n, re=re, steps=steps, storage=storage,
                        beta=shear_beta(n, re=re)))
    return out
