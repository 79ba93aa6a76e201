"""ctypes binding of libelbm.so (include/elbm.h).

Argument marshalling only: every step of the method runs in the HIP
kernels of libelbm.so.  PyTorch provides the device memory (the caller-owned
state buffer and the input/output arrays) and the HIP stream.  If the
library has not been built this module raises on first use; there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libelbm.so")

D1Q3, D2Q9, D3Q27, D3Q19 = 1, 2, 3, 19
LATTICES = {"d1q3": D1Q3, "d2q9": D2Q9, "d3q27": D3Q27, "d3q19": D3Q19}


def lattice_dq(code: int):
    """(D, Q) of a lattice code."""
    return (3, 19) if code == D3Q19 else (code, 3 ** code)
MODES = {"closed": 0, "newton": 1, "bisect": 2, "bgk": 3, "secant": 4}
STORAGES = {"f64": 0, "f32": 1, "f32dev": 2, "f16dev": 3}
DIAG_ALPHA, DIAG_COUNTS, DIAG_SUMS = 1, 2, 4
ENTROPIES = {"boltzmann": 0, "burg": 1}
ARITH = {"fp32": 0, "fp64": 1, "mixed": 2}
STATUS = {0: "ELBM_OK", -1: "ELBM_EINVAL", -2: "ELBM_EDEVICE", -3: "ELBM_ENOMEM",
          -4: "ELBM_ESTATE", -5: "ELBM_EUNSUPPORTED"}
EXPORTS = ["elbm_config_default", "elbm_state_bytes", "elbm_init", "elbm_set_populations",
           "elbm_step", "elbm_moments", "elbm_populations", "elbm_gather",
           "elbm_alpha_field", "elbm_stats", "elbm_time", "elbm_destroy",
           "elbm_last_error", "elbm_step_batch", "elbm_server_create", "elbm_server_submit",
           "elbm_server_poll", "elbm_server_wait", "elbm_server_sim", "elbm_server_release",
           "elbm_server_cancel",
           "elbm_server_get_stats", "elbm_server_destroy", "elbm_checkpoint_bytes",
           "elbm_export", "elbm_import", "elbm_step_noalloc"]
REQ_STATES = {0: "queued", 1: "running", 2: "done", 3: "failed", 4: "cancelled"}


class ElbmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Config(C.Structure):
    _fields_ = [("lattice", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
                ("nz", C.c_int32), ("beta", C.c_double), ("alpha_mode", C.c_int32),
                ("storage", C.c_int32), ("alpha_fp64", C.c_int32),
                ("secant_iters", C.c_int32), ("rho_ref", C.c_double),
                ("root_tol", C.c_double), ("root_max_iter", C.c_int32),
                ("diag", C.c_uint32), ("entropy", C.c_int32), ("reserved", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("step", C.c_int64), ("n_sites", C.c_int64), ("n_accept2", C.c_int64),
                ("n_alphastar_lt2", C.c_int64), ("n_alpha_lt2", C.c_int64),
                ("n_guard", C.c_int64), ("n_fallback", C.c_int64),
                ("n_negative", C.c_int64), ("n_nonfinite", C.c_int64),
                ("total_iters", C.c_int64), ("alpha_min", C.c_double),
                ("alpha_max", C.c_double), ("sum_rho", C.c_double),
                ("sum_j", C.c_double * 3), ("sum_H", C.c_double)]


class ServerConfig(C.Structure):
    _fields_ = [("pool", C.c_void_p), ("pool_bytes", C.c_size_t), ("hip_stream", C.c_void_p),
                ("max_active", C.c_int32), ("round_steps", C.c_int32),
                ("preempt_rounds", C.c_int32), ("reserved", C.c_int32)]


class Request(C.Structure):
    _fields_ = [("cfg", Config), ("rho0", C.c_void_p), ("u0", C.c_void_p),
                ("nsteps", C.c_int64), ("out_rho", C.c_void_p), ("out_u", C.c_void_p),
                ("keep_state", C.c_int32), ("reserved", C.c_int32)]


class RequestInfo(C.Structure):
    _fields_ = [("state", C.c_int32), ("preemptions", C.c_int32), ("steps_done", C.c_int64),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double),
                ("footprint", C.c_size_t)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
                ("rounds", C.c_int64), ("launches", C.c_int64), ("site_updates", C.c_int64),
                ("max_resident", C.c_int64), ("t_first_submit", C.c_double),
                ("t_last_done", C.c_double), ("preemptions", C.c_int64),
                ("cancelled", C.c_int64)]


_lib = None


def lib():
    """Load libelbm.so; raise if it is missing (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run "
                               "`python -m paper_1904_00866_amd.build` first")
        L = C.CDLL(LIB_PATH)
        vp, cfgp = C.c_void_p, C.POINTER(Config)
        L.elbm_config_default.argtypes = [cfgp, C.c_int32, C.c_int32, C.c_int32, C.c_int32]
        L.elbm_state_bytes.argtypes = [cfgp]
        L.elbm_state_bytes.restype = C.c_size_t
        L.elbm_init.argtypes = [cfgp, vp, vp, vp, C.c_size_t, vp, C.POINTER(vp)]
        L.elbm_set_populations.argtypes = [vp, vp]
        L.elbm_step.argtypes = [vp, C.c_int64]
        L.elbm_moments.argtypes = [vp, vp, vp]
        L.elbm_populations.argtypes = [vp, vp]
        L.elbm_gather.argtypes = [vp, vp, C.c_int64, C.c_int32, vp]
        L.elbm_alpha_field.argtypes = [vp, vp]
        L.elbm_stats.argtypes = [vp, C.POINTER(Stats)]
        L.elbm_time.argtypes = [vp]
        L.elbm_time.restype = C.c_int64
        L.elbm_destroy.argtypes = [vp]
        L.elbm_last_error.argtypes = []
        L.elbm_last_error.restype = C.c_char_p
        L.elbm_step_batch.argtypes = [C.POINTER(vp), C.POINTER(C.c_int64), C.c_int32]
        L.elbm_server_create.argtypes = [C.POINTER(ServerConfig), C.POINTER(vp)]
        L.elbm_server_submit.argtypes = [vp, C.POINTER(Request), C.POINTER(C.c_int64)]
        L.elbm_server_poll.argtypes = [vp, C.c_int64, C.POINTER(RequestInfo)]
        L.elbm_server_wait.argtypes = [vp, C.c_int64, C.c_double]
        L.elbm_server_sim.argtypes = [vp, C.c_int64, C.POINTER(vp)]
        L.elbm_server_release.argtypes = [vp, C.c_int64]
        L.elbm_server_cancel.argtypes = [vp, C.c_int64]
        L.elbm_server_get_stats.argtypes = [vp, C.POINTER(ServerStats)]
        L.elbm_server_destroy.argtypes = [vp]
        L.elbm_checkpoint_bytes.argtypes = [vp]
        L.elbm_checkpoint_bytes.restype = C.c_size_t
        L.elbm_export.argtypes = [vp, vp, C.c_size_t, C.POINTER(C.c_int64)]
        L.elbm_import.argtypes = [vp, vp, C.c_size_t, C.c_int64]
        L.elbm_step_noalloc.argtypes = [vp, C.c_int64, C.c_uint32, vp]
        for name in EXPORTS:
            getattr(L, name).restype = getattr(L, name).restype or C.c_int
        L.elbm_state_bytes.restype = C.c_size_t
        L.elbm_time.restype = C.c_int64
        L.elbm_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise ElbmError(rc, lib().elbm_last_error().decode())


def make_config(lattice, nx, ny=1, nz=1, *, beta=0.95, mode="closed", storage="f32",
                fp64=True, secant_iters=3, rho_ref=1.0, root_tol=1e-13,
                root_max_iter=200, diag=0, entropy="boltzmann") -> Config:
    cfg = Config()
    lat = LATTICES[lattice] if isinstance(lattice, str) else int(lattice)
    _check(lib().elbm_config_default(C.byref(cfg), lat, nx, ny, nz))
    cfg.beta = float(beta)
    cfg.alpha_mode = MODES[mode] if isinstance(mode, str) else int(mode)
    cfg.storage = STORAGES[storage] if isinstance(storage, str) else int(storage)
    # fp64: True / False, or an ARITH name ("fp64", "fp32", "mixed")
    cfg.alpha_fp64 = ARITH[fp64] if isinstance(fp64, str) else (1 if fp64 else 0)
    cfg.secant_iters = int(secant_iters)
    cfg.rho_ref = float(rho_ref)
    cfg.root_tol = float(root_tol)
    cfg.root_max_iter = int(root_max_iter)
    cfg.diag = int(diag)
    cfg.entropy = ENTROPIES[entropy] if isinstance(entropy, str) else int(entropy)
    return cfg


def state_bytes(cfg: Config) -> int:
    n = lib().elbm_state_bytes(C.byref(cfg))
    if n == 0:
        _check(-1)
    return n


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev_f64(a, shape, device) -> torch.Tensor:
    t = torch.as_tensor(a, dtype=torch.float64).to(device).contiguous()
    return t.reshape(shape)


class Simulation:
    """One periodic ELBM simulation resident in a caller-owned device buffer.

    rho0: [N] and u0: [D, N] (or any shape with those sizes), SoA with the site
    index s = x + nx*(y + ny*z).  All methods enqueue on `stream` (default:
    torch's current stream on `device`)."""

    def __init__(self, lattice, nx, ny=1, nz=1, *, rho0, u0, device="cuda",
                 stream: Optional[torch.cuda.Stream] = None, **kw):
        self.cfg = make_config(lattice, nx, ny, nz, **kw)
        self.D, self.Q = lattice_dq(self.cfg.lattice)
        self.N = nx * ny * nz
        self.device = torch.device(device)
        self.stream = stream or torch.cuda.current_stream(self.device)
        self.nbytes = state_bytes(self.cfg)
        with torch.cuda.device(self.device), torch.cuda.stream(self.stream):
            self.state = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
            r = _dev_f64(rho0, (self.N,), self.device)
            u = _dev_f64(u0, (self.D, self.N), self.device)
            h = C.c_void_p()
            _check(lib().elbm_init(C.byref(self.cfg), _ptr(r), _ptr(u), _ptr(self.state),
                                   self.nbytes, C.c_void_p(self.stream.cuda_stream),
                                   C.byref(h)))
        self.handle = h

    # -- lifecycle -------------------------------------------------------
    def close(self):
        if getattr(self, "handle", None):
            _check(lib().elbm_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- calls -----------------------------------------------------------
    @property
    def t(self) -> int:
        return lib().elbm_time(self.handle)

    def step(self, n: int = 1):
        _check(lib().elbm_step(self.handle, int(n)))

    def set_populations(self, f):
        ft = _dev_f64(f, (self.Q, self.N), self.device)
        with torch.cuda.stream(self.stream):
            _check(lib().elbm_set_populations(self.handle, _ptr(ft)))
            self.stream.synchronize()

    def moments(self):
        rho = torch.empty(self.N, dtype=torch.float64, device=self.device)
        u = torch.empty(self.D, self.N, dtype=torch.float64, device=self.device)
        _check(lib().elbm_moments(self.handle, _ptr(rho), _ptr(u)))
        return rho, u

    def populations(self) -> torch.Tensor:
        f = torch.empty(self.Q, self.N, dtype=torch.float64, device=self.device)
        _check(lib().elbm_populations(self.handle, _ptr(f)))
        return f

    def gather(self, sites, which: int = 0) -> torch.Tensor:
        st = torch.as_tensor(sites, dtype=torch.int64).to(self.device).contiguous()
        out = torch.empty(self.Q, st.numel(), dtype=torch.float64, device=self.device)
        _check(lib().elbm_gather(self.handle, _ptr(st), st.numel(), int(which), _ptr(out)))
        self.stream.synchronize()
        return out

    def alpha_field(self) -> torch.Tensor:
        a = torch.empty(self.N, dtype=torch.float64, device=self.device)
        _check(lib().elbm_alpha_field(self.handle, _ptr(a)))
        return a

    def export(self):
        """Checkpoint: (device uint8 tensor of the stored populations, t)."""
        n = lib().elbm_checkpoint_bytes(self.handle)
        with torch.cuda.stream(self.stream):
            blob = torch.empty(n, dtype=torch.uint8, device=self.device)
        t = C.c_int64()
        _check(lib().elbm_export(self.handle, _ptr(blob), n, C.byref(t)))
        return blob, t.value

    def import_(self, blob: torch.Tensor, t: int):
        """Resume from a checkpoint of a simulation with the same lattice,
        box and storage."""
        _check(lib().elbm_import(self.handle, _ptr(blob), blob.numel(), int(t)))

    def stats(self) -> dict:
        s = Stats()
        _check(lib().elbm_stats(self.handle, C.byref(s)))
        return stats_dict(s)

    def step_noalloc(self, n: int, diag: int, dev_stats: torch.Tensor):
        """elbm_step_noalloc: n steps, the last step's diagnostics into
        dev_stats (a device tensor of STATS_BYTES bytes) on the stream."""
        assert dev_stats.device.type == "cuda" and dev_stats.nbytes >= STATS_BYTES
        _check(lib().elbm_step_noalloc(self.handle, int(n), int(diag), _ptr(dev_stats)))


STATS_BYTES = C.sizeof(Stats)


def stats_dict(s: Stats) -> dict:
    return dict(step=s.step, n_sites=s.n_sites, n_accept2=s.n_accept2,
                n_alphastar_lt2=s.n_alphastar_lt2, n_alpha_lt2=s.n_alpha_lt2,
                n_guard=s.n_guard, n_fallback=s.n_fallback, n_negative=s.n_negative,
                n_nonfinite=s.n_nonfinite, total_iters=s.total_iters,
                alpha_min=s.alpha_min, alpha_max=s.alpha_max, sum_rho=s.sum_rho,
                sum_j=list(s.sum_j), sum_H=s.sum_H)


def stats_from_bytes(raw) -> dict:
    """An elbm_stats_t copied out of device memory (bytes or a uint8 array)."""
    return stats_dict(Stats.from_buffer_copy(bytes(raw)[:STATS_BYTES]))


def step_batch(sims, nsteps):
    """Advance several simulations (same stream, lattice, storage, mode) with
    one kernel launch per step."""
    n = len(sims)
    hs = (C.c_void_p * n)(*[s.handle for s in sims])
    ns = (C.c_int64 * n)(*[int(k) for k in nsteps])
    _check(lib().elbm_step_batch(hs, ns, n))


class KeptSimulation(Simulation):
    """A simulation kept resident by a server (keep_state=1): the handle and
    its state belong to the server; close() releases them back to the pool."""

    def __init__(self, server: "Server", rid: int, cfg: Config, handle):
        self.cfg = cfg
        self.D, self.Q = lattice_dq(cfg.lattice)
        self.N = cfg.nx * cfg.ny * cfg.nz
        self.device = server.device
        self.stream = server.stream
        self.handle = handle
        self._server, self._rid = server, rid

    def close(self):
        if getattr(self, "handle", None):
            self.handle = None
            if self._server.handle:  # a destroyed server has freed it already
                _check(lib().elbm_server_release(self._server.handle, self._rid))


class Server:
    """Continuous-batching server over one device memory pool.

    pool_bytes of device memory are allocated here (torch) and handed to the
    library, which sub-allocates the states of admitted requests.  All server
    work runs on `stream`."""

    def __init__(self, pool_bytes: int, *, max_active: int = 64, round_steps: int = 50,
                 preempt_rounds: int = 0, device="cuda",
                 stream: Optional[torch.cuda.Stream] = None):
        self.device = torch.device(device)
        self.stream = stream or torch.cuda.current_stream(self.device)
        with torch.cuda.device(self.device):
            self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device=self.device)
            torch.cuda.synchronize(self.device)
            sc = ServerConfig(C.c_void_p(self.pool.data_ptr()), int(pool_bytes),
                              C.c_void_p(self.stream.cuda_stream), int(max_active),
                              int(round_steps), int(preempt_rounds), 0)
            h = C.c_void_p()
            _check(lib().elbm_server_create(C.byref(sc), C.byref(h)))
        self.handle = h
        self._cfgs = {}
        self._keep = {}

    def submit(self, lattice, nx, ny=1, nz=1, *, rho0, u0, nsteps: int, out_rho=None,
               out_u=None, keep_state: bool = False, **kw) -> int:
        """Queue a request; rho0 [N] and u0 [D, N] are host arrays (copied
        here).  out_rho [N] / out_u [D, N] float64 device tensors, or None."""
        import numpy as np
        cfg = make_config(lattice, nx, ny, nz, **kw)
        r = np.ascontiguousarray(np.asarray(rho0, dtype=np.float64).reshape(-1))
        u = np.ascontiguousarray(np.asarray(u0, dtype=np.float64).reshape(-1))
        q = Request(cfg, C.c_void_p(r.ctypes.data), C.c_void_p(u.ctypes.data), int(nsteps),
                    _ptr(out_rho), _ptr(out_u), 1 if keep_state else 0, 0)
        rid = C.c_int64()
        _check(lib().elbm_server_submit(self.handle, C.byref(q), C.byref(rid)))
        self._cfgs[rid.value] = cfg
        return rid.value

    def poll(self, rid: int) -> dict:
        i = RequestInfo()
        _check(lib().elbm_server_poll(self.handle, int(rid), C.byref(i)))
        return dict(state=REQ_STATES[i.state], steps_done=i.steps_done, t_submit=i.t_submit,
                    t_admit=i.t_admit, t_done=i.t_done, footprint=i.footprint,
                    preemptions=i.preemptions)

    def wait(self, rid: int, timeout: float = -1.0):
        _check(lib().elbm_server_wait(self.handle, int(rid), float(timeout)))

    def cancel(self, rid: int):
        _check(lib().elbm_server_cancel(self.handle, int(rid)))

    def simulation(self, rid: int) -> KeptSimulation:
        h = C.c_void_p()
        _check(lib().elbm_server_sim(self.handle, int(rid), C.byref(h)))
        return KeptSimulation(self, int(rid), self._cfgs[int(rid)], h)

    def stats(self) -> dict:
        s = ServerStats()
        _check(lib().elbm_server_get_stats(self.handle, C.byref(s)))
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "handle", None):
            h, self.handle = self.handle, None
            _check(lib().elbm_server_destroy(h))

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
