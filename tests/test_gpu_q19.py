"""GPU parity on the D3Q19 lattice: the HIP path (through the C ABI)
against the FP64 oracle on identical seeded inputs.

D3Q19's weights do not factorise, so the equilibrium is the minimiser of
Eq. (3) found per site by Newton's method on the Lagrange multipliers, on
the GPU (in X_a = exp(l_a), from the per-axis D1Q3 solution) and in the
oracle (in l, from l = 0, with step halving): two independent solvers of the
same minimisation.  Tolerances as for the tensor-product lattices: FP64
storage 1e-13 per population for one step and 1e-11 over a run; reduced
storage one rounding of the output; FP32 laminar velocity 1e-5.
"""
import numpy as np
import pytest
import torch

import helpers as H
from paper_1904_00866_amd import workloads as Wk

pytestmark = pytest.mark.gpu

RAGGED = (11, 9, 7)   # N = 693: two full tiles and a ragged one
ROWS = (64, 5, 3)     # nx % 64 == 0: row-descriptor loads, ragged N
W19 = H.textbook_weights(19)[:, None]


def _sim(gpu, shape, f=None, rho=None, u=None, **kw):
    nx, ny, nz = shape
    N = nx * ny * nz
    if rho is None:
        rho, u = np.ones(N), np.zeros((3, N))
    sim = gpu.Simulation("d3q19", nx, ny, nz, rho0=rho, u0=u, **kw)
    if f is not None:
        sim.set_populations(f)
    return sim


def _ocfg(orc, shape, **kw):
    nx, ny, nz = shape
    return orc.Config(D=3, nx=nx, ny=ny, nz=nz, q=19, **kw)


def _state(N, seed, eps=0.05, tilt=0.1, log_uniform=True):
    return Wk.random_populations(H.textbook_weights(19), N, eps, seed, tilt=tilt,
                                 log_uniform_eps=log_uniform)


def _tol(storage, fo):
    if storage == "f64":
        return 1e-13 * np.abs(fo)
    if storage == "f32":
        return 2.0 ** -24 * np.abs(fo) * 1.01 + 1e-300
    if storage == "f32dev":
        return W19 * (2.0 ** -24 * np.abs(fo / W19 - 1.0) * 1.01 + 1e-12)
    return W19 * (2.0 ** -11 * np.abs(fo / W19 - 1.0) * 1.01 + 2.0 ** -24)


def test_q19_init_places_the_oracle_equilibrium(gpu, orc):
    """elbm_init writes f^eq(rho0, u0): the GPU's Newton minimiser against
    the oracle's, for velocities up to 0.3 per component."""
    shape = (13, 11, 6)
    N = int(np.prod(shape))
    rho, u = Wk.random_velocity_field(3, N, 0.3, seed=41, rho_spread=0.3)
    sim = _sim(gpu, shape, rho=rho, u=u, storage="f64")
    fg = sim.populations().cpu().numpy()
    fo = orc.init(_ocfg(orc, shape), rho, u)
    assert np.max(np.abs(fg - fo) / fo) <= 4e-15
    r, v = sim.moments()
    assert np.max(np.abs(r.cpu().numpy() - rho)) <= 4e-15
    assert np.max(np.abs(v.cpu().numpy() - u)) <= 4e-15
    sim.close()


@pytest.mark.parametrize("mode", ["closed", "secant", "newton", "bgk"])
def test_q19_one_step_fp64(gpu, orc, mode):
    N = int(np.prod(RAGGED))
    f0 = _state(N, seed=1900 + len(mode))
    sim = _sim(gpu, RAGGED, f0, storage="f64", beta=0.97, mode=mode,
               diag=gpu.DIAG_ALPHA | gpu.DIAG_COUNTS | gpu.DIAG_SUMS)
    assert np.array_equal(sim.populations().cpu().numpy(), f0)
    sim.step(1)
    fg = sim.populations().cpu().numpy()
    ag = sim.alpha_field().cpu().numpy()
    cfg = _ocfg(orc, RAGGED, beta=0.97, mode=mode, root_max_iter=200)
    fo, ao, d = orc.step(cfg, f0, want_alpha=True, want_diag=True)
    assert np.max(np.abs(fg - fo) / np.abs(fo)) <= 1e-13
    st = sim.stats()
    assert st["n_sites"] == N and st["step"] == 1
    if mode != "bgk":
        assert np.max(np.abs(ag - ao)) <= 1e-12
        assert abs(st["n_accept2"] - d["n_accept2"]) <= 2
        assert st["n_alphastar_lt2"] == d["n_alphastar_lt2"]
        assert 0 < st["n_alpha_lt2"] < N
        # H(f) summed over the box (Eq. (6)) from the GPU's H(f^eq) + D
        assert abs(st["sum_H"] - d["sum_H"]) <= 1e-12 * abs(d["sum_H"])
    assert abs(st["sum_rho"] - d["sum_rho"]) <= 1e-13 * d["sum_rho"]
    np.testing.assert_allclose(st["sum_j"], d["sum_j"], rtol=0, atol=1e-12 * d["sum_rho"])
    sim.close()


def test_q19_one_step_fp64_bisection(gpu, orc):
    """Compared through the stop window, as on the other lattices."""
    N = int(np.prod(RAGGED))
    f0 = _state(N, seed=1977)
    sim = _sim(gpu, RAGGED, f0, storage="f64", beta=0.97, mode="bisect", diag=gpu.DIAG_ALPHA)
    sim.step(1)
    ag = sim.alpha_field().cpu().numpy()
    _, ao, _ = orc.step(_ocfg(orc, RAGGED, beta=0.97, mode="bisect"), f0, want_alpha=True)
    same = np.abs(ag - ao) <= 1e-12
    assert same.mean() > 0.99
    for s in np.nonzero(~same)[0][:20]:
        g = orc.G(19, f0[:, s], ag[s])
        assert -1e-13 - 1e-16 <= g <= 1e-16
    sim.close()


@pytest.mark.parametrize("shape", [RAGGED, ROWS])
@pytest.mark.parametrize("storage", ["f64", "f32", "f32dev", "f16dev"])
@pytest.mark.parametrize("mode", ["closed", "bgk"])
def test_q19_one_step_storages(gpu, orc, shape, storage, mode):
    """From the decoded stored state, one GPU step equals one oracle step up
    to one rounding of the output to the storage format (general and
    row-descriptor loads)."""
    N = int(np.prod(shape))
    f0 = _state(N, seed=1950 + len(storage) + 3 * len(mode) + shape[0], eps=0.02, tilt=0.05)
    sim = _sim(gpu, shape, f0, storage=storage, beta=0.97, mode=mode)
    fq = sim.populations().cpu().numpy()
    sim.step(1)
    fg = sim.populations().cpu().numpy()
    fo, _, _ = orc.step(_ocfg(orc, shape, beta=0.97, mode=mode), fq)
    assert np.all(np.abs(fg - fo) <= _tol(storage, fo))
    sim.close()


@pytest.mark.parametrize("eps,log_uniform", [(0.05, True), (0.7, False)])
@pytest.mark.parametrize("mode", ["closed", "secant", "newton"])
def test_q19_per_site_invariants(gpu, orc, eps, log_uniform, mode):
    """One collision on the kernel's own output (FP64 storage, f~ read back
    where the step wrote it), recomputed on the CPU: positivity, mass and
    momentum to 1e-14 rho, the per-site H-theorem up to rounding, and Eq. (7)
    at the kernel's alpha for the solvers that bound the root from below."""
    N = int(np.prod(RAGGED))
    f0 = _state(N, seed=1990 + len(mode), eps=eps, log_uniform=log_uniform)
    sim = _sim(gpu, RAGGED, f0, storage="f64", beta=0.98, mode=mode, diag=gpu.DIAG_ALPHA)
    sim.step(1)
    f1 = sim.gather(np.arange(N), 1).cpu().numpy()
    ag = sim.alpha_field().cpu().numpy()
    sim.close()
    H.check_collision_invariants(orc, 19, f0, f1, None if mode == "newton" else ag, W19, 19)


def test_q19_rare_tier_states(gpu, orc):
    """States far from equilibrium (alpha_* < 2 on many sites): the deferred
    rare path (long series, log1p forms) against the oracle, FP64."""
    N = int(np.prod(RAGGED))
    f0 = _state(N, seed=1999, eps=0.7, tilt=0.2, log_uniform=False)
    sim = _sim(gpu, RAGGED, f0, storage="f64", beta=0.9,
               diag=gpu.DIAG_ALPHA | gpu.DIAG_COUNTS)
    sim.step(1)
    fg = sim.populations().cpu().numpy()
    fo, ao, d = orc.step(_ocfg(orc, RAGGED, beta=0.9), f0, want_alpha=True, want_diag=True)
    assert d["n_alphastar_lt2"] > N // 10
    assert np.max(np.abs(fg - fo) / np.abs(fo)) <= 1e-12
    assert np.max(np.abs(sim.alpha_field().cpu().numpy() - ao)) <= 1e-11
    assert sim.stats()["n_alphastar_lt2"] == d["n_alphastar_lt2"]
    sim.close()


def test_q19_fp32_arithmetic(gpu, orc):
    """All-FP32 site arithmetic (closed form, FP32 Newton for f^eq): one
    step within 2e-6 relative."""
    N = int(np.prod(RAGGED))
    f0 = _state(N, seed=1905, eps=0.02)
    sim = _sim(gpu, RAGGED, f0, storage="f32", beta=0.97, fp64=False)
    fq = sim.populations().cpu().numpy()
    sim.step(1)
    fg = sim.populations().cpu().numpy()
    fo, _, _ = orc.step(_ocfg(orc, RAGGED, beta=0.97), fq)
    assert np.max(np.abs(fg - fo) / np.abs(fo)) <= 2e-6
    sim.close()


def test_q19_taylor_green_multistep_fp64(gpu, orc):
    """3-D Taylor-Green, Re = 1600, 24^3, 300 steps, FP64 storage: max
    relative population error <= 1e-11; sum_x H non-increasing."""
    n, steps = 24, 300
    beta = Wk.tgv3d_beta(n)
    rho, u = Wk.taylor_green_3d(n)
    sim = _sim(gpu, (n, n, n), rho=rho, u=u, storage="f64", beta=beta,
               diag=gpu.DIAG_COUNTS | gpu.DIAG_SUMS)
    Hs = []
    for _ in range(6):
        sim.step(steps // 6)
        Hs.append(sim.stats()["sum_H"])
    fg = sim.populations().cpu().numpy()
    cfg = _ocfg(orc, (n, n, n), beta=beta, nthreads=16)
    fo, _, _ = orc.run(cfg, orc.init(cfg, rho, u), steps)
    assert np.max(np.abs(fg - fo) / np.abs(fo)) <= 1e-11
    assert np.all(np.diff(Hs) <= 1e-12 * abs(Hs[0]))
    sim.close()


@pytest.mark.parametrize("storage", ["f32", "f32dev"])
def test_q19_taylor_green_fp32_velocity(gpu, orc, storage):
    """FP32 storage, 3-D Taylor-Green at Re = 1600, 48^3 over the laminar
    horizon (458 steps): velocity within 1e-5 of the FP64 oracle, relative
    to the velocity scale."""
    n = 48
    steps = int(round(3.0 * n / (2.0 * np.pi) / 0.05))
    beta = Wk.tgv3d_beta(n)
    rho, u = Wk.taylor_green_3d(n)
    sim = _sim(gpu, (n, n, n), rho=rho, u=u, storage=storage, beta=beta)
    sim.step(steps)
    _, ug = sim.moments()
    cfg = _ocfg(orc, (n, n, n), beta=beta, nthreads=16)
    fo, _, _ = orc.run(cfg, orc.init(cfg, rho, u), steps)
    _, uo = orc.moments(cfg, fo)
    assert np.max(np.abs(ug.cpu().numpy() - uo)) / np.max(np.abs(uo)) <= 1e-5
    sim.close()


def test_q19_batch_equals_alone(gpu):
    """elbm_step_batch over D3Q19 simulations of different boxes equals
    stepping each alone, bitwise."""
    shapes = [(16, 12, 9), (64, 4, 3), (7, 5, 3)]
    fields = [Wk.random_velocity_field(3, int(np.prod(s)), 0.08, seed=60 + k)
              for k, s in enumerate(shapes)]
    steps = [7, 4, 9]
    alone = []
    for s, (rho, u), n in zip(shapes, fields, steps):
        with _sim(gpu, s, rho=rho, u=u, beta=0.98) as sim:
            sim.step(n)
            alone.append(sim.populations().cpu().numpy())
    sims = [_sim(gpu, s, rho=rho, u=u, beta=0.98) for s, (rho, u) in zip(shapes, fields)]
    gpu.step_batch(sims, steps)
    for sim, ref in zip(sims, alone):
        assert np.array_equal(sim.populations().cpu().numpy(), ref)
        sim.close()


def test_q19_checkpoint_resume_is_bitwise(gpu):
    shape = (20, 12, 9)
    rho, u = Wk.random_velocity_field(3, int(np.prod(shape)), 0.06, seed=93)
    with _sim(gpu, shape, rho=rho, u=u, storage="f16dev", beta=0.99) as a:
        a.step(12)
        ck, t = a.export()
        a.step(8)
        ref = a.populations().cpu().numpy()
    with _sim(gpu, shape, rho=np.ones(int(np.prod(shape))), u=np.zeros((3, int(np.prod(shape)))),
              storage="f16dev", beta=0.99) as b:
        b.import_(ck, t)
        b.step(8)
        assert b.t == 20
        assert np.array_equal(b.populations().cpu().numpy(), ref)


def test_q19_init_rejects_outside_the_hull(gpu):
    """|u_x| + |u_y| + |u_z| >= 2 is outside D3Q19's hull (valid on D3Q27)."""
    N = 8
    rho = np.ones(N)
    u = np.zeros((3, N))
    u[:, 3] = [0.9, 0.8, 0.4]
    with pytest.raises(gpu.ElbmError) as e:
        _sim(gpu, (2, 2, 2), rho=rho, u=u)
    assert e.value.status == -1
    gpu.Simulation("d3q27", 2, 2, 2, rho0=rho, u0=u).close()
    u[:, 3] = [0.7, 0.6, 0.5]
    with _sim(gpu, (2, 2, 2), rho=rho, u=u, storage="f64") as s:
        np.testing.assert_allclose(s.moments()[1].cpu().numpy()[:, 3], [0.7, 0.6, 0.5],
                                   rtol=0, atol=1e-14)


def test_q19_edge_boxes(gpu, orc):
    """Single-site and thin periodic boxes, FP64, 3 steps."""
    for shape in [(1, 1, 1), (1, 1, 5), (3, 1, 1), (2, 2, 2), (1, 70, 1)]:
        N = int(np.prod(shape))
        f0 = _state(N, seed=sum(shape), eps=0.05)
        sim = _sim(gpu, shape, f0, storage="f64", beta=0.95)
        sim.step(3)
        fo = f0
        for _ in range(3):
            fo, _, _ = orc.step(_ocfg(orc, shape, beta=0.95), fo)
        assert np.max(np.abs(sim.populations().cpu().numpy() - fo) / fo) <= 1e-13, shape
        sim.close()


@pytest.mark.parametrize("n,storage", [(512, "f32"), (256, "f16dev")])
def test_q19_full_size_sampled(gpu, orc, n, storage):
    """The 512^3 Taylor-Green box of the D3Q19 timing (FP32 storage), and
    256^3 with FP16 deviation storage (the closed form's first-term tier on
    the stored deviations): one step after three, checked against the
    oracle's collision of the GPU's decoded pre-state at 2048 sampled sites
    (row ends and the last site included); one rounding into the storage
    format."""
    b = Wk.tgv3d_beta(n)
    rho, u = Wk.taylor_green_3d(n)
    sim = _sim(gpu, (n, n, n), rho=rho, u=u, storage=storage, beta=b)
    del rho, u
    sim.step(3)
    rng = np.random.default_rng(519)
    sites = np.unique(np.concatenate([rng.integers(0, n ** 3, 2040),
                                      [0, n - 1, n * n - 1, n ** 3 - n, n ** 3 - 1]]))
    pre = sim.gather(sites, 0).cpu().numpy()
    sim.step(1)
    post = sim.gather(sites, 1).cpu().numpy()
    sim.close()
    cfg = orc.Config(D=3, nx=1, q=19, beta=b)
    for k in range(sites.size):
        ft, _ = orc.collide_site(cfg, pre[:, k])
        tol = _tol(storage, ft[:, None])[:, 0]
        assert np.all(np.abs(post[:, k] - ft) <= tol), (sites[k], post[:, k], ft)
    torch.cuda.empty_cache()
