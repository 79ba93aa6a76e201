"""ctypes binding of the FP64 CPU oracle (test infrastructure only).

The oracle stores the paper's f(x, t) (pre-collision populations) as
SoA float64 arrays f[i, s], s = x + nx*(y + ny*z), and advances them by
collide (Eq. (1)) then periodic push-streaming (Eq. (5b)).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle_elbm.so")

CLOSED, NEWTON, BISECT, BGK, SECANT = 0, 1, 2, 3, 4
MODES = {"closed": CLOSED, "newton": NEWTON, "bisect": BISECT, "bgk": BGK,
         "secant": SECANT}


class Params(C.Structure):
    _fields_ = [("lattice", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
                ("nz", C.c_int32), ("beta", C.c_double), ("mode", C.c_int32),
                ("secant_iters", C.c_int32), ("root_tol", C.c_double),
                ("root_max_iter", C.c_int32), ("nthreads", C.c_int32),
                ("entropy", C.c_int32)]


class SiteInfo(C.Structure):
    _fields_ = [("rho", C.c_double), ("u", C.c_double * 3),
                ("alpha", C.c_double), ("alpha_max", C.c_double),
                ("alpha_star", C.c_double), ("G_star", C.c_double),
                ("D", C.c_double), ("accepted2", C.c_int32),
                ("guard", C.c_int32), ("iters", C.c_int32)]


class Diag(C.Structure):
    _fields_ = [("n_sites", C.c_int64), ("n_accept2", C.c_int64),
                ("n_alphastar_lt2", C.c_int64), ("n_alpha_lt2", C.c_int64),
                ("n_guard", C.c_int64), ("n_negative", C.c_int64),
                ("total_iters", C.c_int64), ("alpha_min", C.c_double),
                ("alpha_max", C.c_double), ("sum_rho", C.c_double),
                ("sum_j", C.c_double * 3), ("sum_H", C.c_double)]


_lib = None


def lib():
    """Load liboracle_elbm.so, building it with gcc if it is absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from .build_oracle import build
            build()
        L = C.CDLL(_LIB_PATH)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        L.orc_lattice.argtypes = [C.c_int32, ip, ip, dp]
        L.orc_equilibrium.argtypes = [C.c_int32, C.c_double, dp, dp]
        L.orc_equilibrium_minimiser.argtypes = [C.c_int32, C.c_double, dp, dp, ip]
        L.orc_equilibrium_poly.argtypes = [C.c_int32, C.c_double, dp, dp]
        L.orc_moments_site.argtypes = [C.c_int32, dp, dp, dp]
        L.orc_entropy.argtypes = [C.c_int32, dp]
        L.orc_entropy.restype = C.c_double
        L.orc_entropy_rel.argtypes = [C.c_int32, dp, dp]
        L.orc_entropy_rel.restype = C.c_double
        L.orc_alpha_max.argtypes = [C.c_int32, dp, dp]
        L.orc_alpha_max.restype = C.c_double
        L.orc_G.argtypes = [C.c_int32, dp, C.c_double]
        L.orc_G.restype = C.c_double
        L.orc_alpha.argtypes = [C.POINTER(Params), dp, C.POINTER(SiteInfo)]
        L.orc_collide_site.argtypes = [C.POINTER(Params), dp, dp,
                                       C.POINTER(SiteInfo)]
        L.orc_init.argtypes = [C.POINTER(Params), dp, dp, dp]
        L.orc_moments.argtypes = [C.POINTER(Params), dp, dp, dp]
        L.orc_step.argtypes = [C.POINTER(Params), dp, dp, dp, C.POINTER(Diag)]
        _lib = L
    return _lib


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


# ---------------------------------------------------------------- lattice ---
# Lattice codes: 1, 2, 3 for the tensor-product lattices D1Q3, D2Q9, D3Q27;
# 19 for D3Q19.  Single-state functions take a model code: the lattice code
# + 256 x entropy (0: the Boltzmann entropy of Eq. (3), 1: Burg's entropy).
D3Q19 = 19
ENTROPIES = {"boltzmann": 0, "burg": 1}


def model(lat: int, entropy: str = "boltzmann") -> int:
    return lat + 256 * ENTROPIES[entropy]


def lattice_Q(lat: int) -> int:
    lat &= 255
    return 19 if lat == D3Q19 else 3 ** lat


def lattice_D(lat: int) -> int:
    lat &= 255
    return 3 if lat == D3Q19 else lat


def lattice(lat: int):
    """(c[Q,3] int, W[Q] float64) in the library's direction order."""
    Q = lattice_Q(lat)
    c = np.zeros((Q, 3), np.int32)
    W = np.zeros(Q, np.float64)
    q = C.c_int32()
    rc = lib().orc_lattice(lat, C.byref(q), c.ctypes.data_as(C.POINTER(C.c_int32)),
                           _dp(W))
    if rc:
        raise ValueError(f"bad lattice code {lat}")
    return c, W


def equilibrium(lat, rho, u, poly=False):
    u3 = _f64(list(u) + [0.0] * (3 - len(u)))
    out = np.zeros(lattice_Q(lat))
    fn = lib().orc_equilibrium_poly if poly else lib().orc_equilibrium
    if fn(lat, float(rho), _dp(u3), _dp(out)):
        raise ValueError("equilibrium undefined (rho <= 0 or u outside the velocities' hull)")
    return out


def equilibrium_minimiser(lat, rho, u):
    """f^eq by Newton's method on the Lagrange multipliers (any lattice);
    returns (feq, Newton iterations)."""
    u3 = _f64(list(u) + [0.0] * (3 - len(u)))
    out = np.zeros(lattice_Q(lat))
    it = C.c_int32()
    if lib().orc_equilibrium_minimiser(lat, float(rho), _dp(u3), _dp(out), C.byref(it)):
        raise ValueError("no minimiser (rho <= 0, u outside the hull, or no convergence)")
    return out, it.value


def moments_site(lat, f):
    f = _f64(f)
    r = C.c_double()
    u = np.zeros(3)
    lib().orc_moments_site(lat, _dp(f), C.byref(r), _dp(u))
    return r.value, u[:lattice_D(lat)]


def entropy(lat, f):
    return lib().orc_entropy(lat, _dp(_f64(f)))


def entropy_rel(lat, g, feq):
    return lib().orc_entropy_rel(lat, _dp(_f64(g)), _dp(_f64(feq)))


def alpha_max(lat, f, feq):
    return lib().orc_alpha_max(lat, _dp(_f64(f)), _dp(_f64(feq)))


def G(lat, f, alpha):
    """H(f*(alpha)) - H(f) with f^eq computed from f's moments."""
    return lib().orc_G(lat, _dp(_f64(f)), float(alpha))


# ------------------------------------------------------------ parameters ---
@dataclass
class Config:
    D: int
    nx: int
    ny: int = 1
    nz: int = 1
    beta: float = 0.95
    mode: str = "closed"
    secant_iters: int = 3
    root_tol: float = 1e-13
    root_max_iter: int = 200
    nthreads: int = 1
    q: int = 0            # 0: the tensor-product lattice 3^D; 19: D3Q19 (D = 3)
    entropy: str = "boltzmann"  # or "burg"

    @property
    def lattice(self) -> int:
        if self.q not in (0, 19) or (self.q == 19 and self.D != 3):
            raise ValueError(f"no lattice D{self.D}Q{self.q}")
        return D3Q19 if self.q == 19 else self.D

    def params(self) -> Params:
        return Params(self.lattice, self.nx, self.ny, self.nz, self.beta,
                      MODES[self.mode], self.secant_iters, self.root_tol,
                      self.root_max_iter, self.nthreads, ENTROPIES[self.entropy])

    @property
    def model(self) -> int:
        return model(self.lattice, self.entropy)

    @property
    def N(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def Q(self) -> int:
        return lattice_Q(self.lattice)


def _info_dict(si: SiteInfo) -> dict:
    return dict(rho=si.rho, u=np.array(si.u[:]), alpha=si.alpha,
                alpha_max=si.alpha_max, alpha_star=si.alpha_star,
                G_star=si.G_star, D=si.D, accepted2=bool(si.accepted2),
                guard=bool(si.guard), iters=si.iters)


def alpha_site(cfg: Config, f) -> dict:
    si = SiteInfo()
    p = cfg.params()
    if lib().orc_alpha(C.byref(p), _dp(_f64(f)), C.byref(si)):
        raise ValueError("invalid parameters")
    return _info_dict(si)


def collide_site(cfg: Config, f):
    """Post-collision f~ (Eq. (1)) of one site and the alpha record."""
    f = _f64(f)
    out = np.zeros_like(f)
    si = SiteInfo()
    p = cfg.params()
    if lib().orc_collide_site(C.byref(p), _dp(f), _dp(out), C.byref(si)):
        raise ValueError("invalid parameters")
    return out, _info_dict(si)


def init(cfg: Config, rho0, u0):
    """f(x, 0) = f^eq(rho0(x), u0(x)); rho0[N], u0[D, N] (SoA)."""
    rho0 = _f64(rho0).reshape(-1)
    u0 = _f64(u0).reshape(cfg.D, -1)
    f = np.zeros((cfg.Q, cfg.N))
    p = cfg.params()
    rc = lib().orc_init(C.byref(p), _dp(rho0), _dp(u0), _dp(f))
    if rc:
        raise ValueError(f"orc_init failed ({rc})")
    return f


def moments(cfg: Config, f):
    f = _f64(f)
    rho = np.zeros(cfg.N)
    u = np.zeros((cfg.D, cfg.N))
    p = cfg.params()
    lib().orc_moments(C.byref(p), _dp(f), _dp(rho), _dp(u))
    return rho, u


def diag_dict(d: Diag) -> dict:
    return dict(n_sites=d.n_sites, n_accept2=d.n_accept2,
                n_alphastar_lt2=d.n_alphastar_lt2, n_alpha_lt2=d.n_alpha_lt2,
                n_guard=d.n_guard, n_negative=d.n_negative,
                total_iters=d.total_iters, alpha_min=d.alpha_min,
                alpha_max=d.alpha_max, sum_rho=d.sum_rho,
                sum_j=np.array(d.sum_j[:]), sum_H=d.sum_H)


def step(cfg: Config, f, want_alpha=False, want_diag=False):
    """One collide + stream step. Returns (f_next, alpha or None, diag or None)."""
    f = _f64(f)
    fn = np.empty_like(f)
    alpha = np.empty(cfg.N) if want_alpha else None
    d = Diag() if want_diag else None
    p = cfg.params()
    rc = lib().orc_step(C.byref(p), _dp(f), _dp(fn), _dp(alpha),
                        C.byref(d) if d is not None else None)
    if rc:
        raise ValueError(f"orc_step failed ({rc})")
    return fn, alpha, (diag_dict(d) if d is not None else None)


def run(cfg: Config, f, nsteps, want_alpha=False, diag_every=0, callback=None):
    """nsteps steps; diag_every > 0 collects the diagnostics every k steps.

    Returns (f, alpha_of_last_step or None, list of (step, diag))."""
    f = _f64(f).copy()
    fn = np.empty_like(f)
    p = cfg.params()
    L = lib()
    d = Diag()
    diags = []
    alpha = np.empty(cfg.N) if want_alpha else None
    for t in range(nsteps):
        want = diag_every > 0 and (t % diag_every == 0)
        last = t == nsteps - 1
        rc = L.orc_step(C.byref(p), _dp(f), _dp(fn),
                        _dp(alpha) if (want_alpha and last) else None,
                        C.byref(d) if want else None)
        if rc:
            raise ValueError(f"orc_step failed ({rc})")
        if want:
            diags.append((t, diag_dict(d)))
        f, fn = fn, f
        if callback is not None:
            callback(t + 1, f)
    return f, alpha, diags
