"""elbm_step_noalloc (the step whose diagnostics scratch is the library's
static device array) against elbm_step + elbm_stats on the same state: the
same populations, alpha field and statistics, bit for bit, on two calls in a
row with different simulations, the second smaller than the first; and the
size limit of the scratch, rejected before any device work."""
import numpy as np
import pytest
import torch

import helpers as H
from paper_1904_00866_amd import workloads as Wk

pytestmark = pytest.mark.gpu


def _state(D, N, seed):
    """Populations mixing near- and far-from-equilibrium sites (alpha_* < 2
    at some), so that every count of the statistics is exercised."""
    W = H.textbook_weights(D)
    far = Wk.random_populations(W, N, 0.7, seed, tilt=0.2)
    near = Wk.random_populations(W, N, 0.05, seed + 1, tilt=0.1, log_uniform_eps=True)
    pick = np.random.default_rng(seed + 2).random(N) < 0.3
    return np.ascontiguousarray(np.where(pick[None, :], far, near))


def _compare(gpu, D, shape, nsteps, seed, mode, dev_stats, storage="f64", arith=True):
    nx, ny, nz = shape
    N = nx * ny * nz
    f0 = _state(D, N, seed)
    rho, u = np.ones(N), np.zeros((D, N))
    kw = dict(storage=storage, beta=0.97, mode=mode, fp64=arith)
    a = gpu.Simulation(D, nx, ny, nz, rho0=rho, u0=u,
                       diag=gpu.DIAG_ALPHA | gpu.DIAG_COUNTS | gpu.DIAG_SUMS, **kw)
    b = gpu.Simulation(D, nx, ny, nz, rho0=rho, u0=u, diag=gpu.DIAG_ALPHA, **kw)
    a.set_populations(f0)
    b.set_populations(f0)
    a.step(nsteps)
    sa = a.stats()
    with torch.cuda.stream(b.stream):
        b.step_noalloc(nsteps, gpu.DIAG_COUNTS | gpu.DIAG_SUMS, dev_stats)
        raw = dev_stats.cpu().numpy()
    sb = gpu.stats_from_bytes(raw.tobytes())
    assert sa == sb, (sa, sb)
    assert sb["n_sites"] == N and sb["step"] == nsteps
    assert sb["n_alphastar_lt2"] > 0
    assert torch.equal(a.populations(), b.populations())
    assert torch.equal(a.alpha_field(), b.alpha_field())
    # the handle's own records were not written by the no-allocation steps
    with pytest.raises(gpu.ElbmError):
        b.stats()
    a.close()
    b.close()


def test_step_noalloc_matches_step_and_stats(gpu):
    dev_stats = torch.zeros(gpu.STATS_BYTES, dtype=torch.uint8, device="cuda")
    # two calls in a row, the second on a smaller box (the scratch keeps the
    # first call's records beyond the second's workgroups)
    _compare(gpu, 3, (40, 36, 30), 3, 9100, "closed", dev_stats)
    _compare(gpu, 2, (37, 23, 1), 2, 9200, "closed", dev_stats)
    _compare(gpu, 2, (64, 12, 1), 2, 9300, "newton", dev_stats)


def test_step_noalloc_four_tile_kernels(gpu):
    """The kernels that update four tiles per workgroup (D2Q9 with 4- and
    2-byte storage: one record per four tiles), on general and grouped-row
    boxes, FP64 and mixed site arithmetic, each against elbm_step bit for
    bit, in a row on one scratch."""
    dev_stats = torch.zeros(gpu.STATS_BYTES, dtype=torch.uint8, device="cuda")
    _compare(gpu, 2, (1024, 6, 1), 2, 9400, "closed", dev_stats, storage="f16dev", arith="mixed")
    _compare(gpu, 2, (37, 23, 1), 2, 9500, "closed", dev_stats, storage="f32")
    _compare(gpu, 2, (1024, 2, 1), 3, 9600, "secant", dev_stats, storage="f16dev")


def test_step_noalloc_rejects_boxes_beyond_the_scratch(gpu):
    """A box of more than 65536 workgroup records is refused with
    ELBM_EINVAL before any launch; the limit itself is accepted.  D3Q27
    workgroups hold 256 sites, so the limit is 2^24 sites (256^3)."""
    dev_stats = torch.zeros(gpu.STATS_BYTES, dtype=torch.uint8, device="cuda")
    n = 256
    for nz, ok in ((n + 1, False), (n, True)):
        N = n * n * nz
        rho, u = np.ones(N), np.zeros((3, N))
        with gpu.Simulation("d3q27", n, n, nz, rho0=rho, u0=u, storage="f16dev") as s:
            if not ok:
                with pytest.raises(gpu.ElbmError) as e:
                    s.step_noalloc(1, gpu.DIAG_COUNTS, dev_stats)
                assert "scratch" in str(e.value) and s.t == 0
            else:
                s.step_noalloc(1, gpu.DIAG_COUNTS, dev_stats)
                st = gpu.stats_from_bytes(dev_stats.cpu().numpy().tobytes())
                assert st["n_sites"] == N and st["step"] == 1
                # f = f^eq everywhere: the guard accepts alpha = 2
                assert st["n_accept2"] == N
