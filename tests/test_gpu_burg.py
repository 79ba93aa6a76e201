"""GPU parity with Burg's entropy H(f) = -sum W ln(f/W): the HIP path
(through the C ABI) against the FP64 oracle on identical seeded inputs, on
every lattice.

The equilibrium (f^eq_i = W_i / (m0 + m.c_i)) is found per site by Newton's
method on the multipliers on both sides, by independent solvers (GPU: from
the third-order solution kept inside d > 0, Armijo steps only for long
steps; oracle: from the rest state, Armijo steps throughout).  Tolerances as
for the Boltzmann entropy: FP64 storage 1e-13 per population for one step,
1e-11 over a run; FP32 storage one rounding of the output.
"""
import numpy as np
import pytest
import torch

import helpers as H
from paper_1904_00866_amd import workloads as Wk

pytestmark = pytest.mark.gpu

SHAPES = {1: (300, 1, 1), 2: (37, 23, 1), 3: (11, 9, 7), 19: (11, 9, 7)}
ROWS = {1: (192, 1, 1), 2: (128, 6, 1), 3: (64, 5, 3), 19: (64, 5, 3)}
NAMES = {1: "d1q3", 2: "d2q9", 3: "d3q27", 19: "d3q19"}


def _sim(gpu, lat, shape, f=None, rho=None, u=None, **kw):
    N = int(np.prod(shape))
    if rho is None:
        rho, u = np.ones(N), np.zeros((H.dim(lat), N))
    sim = gpu.Simulation(NAMES[lat], *shape, rho0=rho, u0=u, entropy="burg", **kw)
    if f is not None:
        sim.set_populations(f)
    return sim


def _ocfg(orc, lat, shape, **kw):
    nx, ny, nz = shape
    return orc.Config(D=H.dim(lat), nx=nx, ny=ny, nz=nz, q=19 if lat == 19 else 0,
                      entropy="burg", **kw)


def _state(lat, N, seed, eps=0.05, tilt=0.1, log_uniform=True):
    return Wk.random_populations(H.textbook_weights(lat), N, eps, seed, tilt=tilt,
                                 log_uniform_eps=log_uniform)


@pytest.mark.parametrize("lat", [1, 2, 3, 19])
def test_burg_init_places_the_oracle_equilibrium(gpu, orc, lat):
    shape = SHAPES[lat]
    N = int(np.prod(shape))
    rho, u = Wk.random_velocity_field(H.dim(lat), N, 0.25, seed=70 + lat, rho_spread=0.3)
    sim = _sim(gpu, lat, shape, rho=rho, u=u, storage="f64")
    fg = sim.populations().cpu().numpy()
    fo = orc.init(_ocfg(orc, lat, shape), rho, u)
    # two independent Newton solvers, each converged to rounding, |u_a| <= 0.25
    assert np.max(np.abs(fg - fo) / fo) <= 1e-14
    sim.close()


@pytest.mark.parametrize("lat", [1, 2, 3, 19])
@pytest.mark.parametrize("mode", ["closed", "secant", "newton"])
def test_burg_one_step_fp64(gpu, orc, lat, mode):
    shape = SHAPES[lat]
    N = int(np.prod(shape))
    f0 = _state(lat, N, seed=2100 + 10 * lat + len(mode))
    sim = _sim(gpu, lat, shape, f0, storage="f64", beta=0.97, mode=mode,
               diag=gpu.DIAG_ALPHA | gpu.DIAG_COUNTS | gpu.DIAG_SUMS)
    assert np.array_equal(sim.populations().cpu().numpy(), f0)
    sim.step(1)
    fg = sim.populations().cpu().numpy()
    ag = sim.alpha_field().cpu().numpy()
    fo, ao, d = orc.step(_ocfg(orc, lat, shape, beta=0.97, mode=mode, root_max_iter=200), f0,
                         want_alpha=True, want_diag=True)
    assert np.max(np.abs(fg - fo) / np.abs(fo)) <= 1e-13
    assert np.max(np.abs(ag - ao)) <= 1e-12
    st = sim.stats()
    assert abs(st["n_accept2"] - d["n_accept2"]) <= 2
    assert st["n_alphastar_lt2"] == d["n_alphastar_lt2"]
    assert 0 < st["n_alpha_lt2"] < N
    # sum_x H(f(x,t)) with Burg's entropy (Eq. (6)), from H(f^eq) + D per site
    assert abs(st["sum_H"] - d["sum_H"]) <= 1e-12 * max(1.0, abs(d["sum_H"]))
    assert abs(st["sum_rho"] - d["sum_rho"]) <= 1e-13 * d["sum_rho"]
    sim.close()


@pytest.mark.parametrize("lat", [2, 3])
def test_burg_one_step_fp64_bisection(gpu, orc, lat):
    shape = SHAPES[lat]
    N = int(np.prod(shape))
    f0 = _state(lat, N, seed=2177 + lat)
    sim = _sim(gpu, lat, shape, f0, storage="f64", beta=0.97, mode="bisect", diag=gpu.DIAG_ALPHA)
    sim.step(1)
    ag = sim.alpha_field().cpu().numpy()
    _, ao, _ = orc.step(_ocfg(orc, lat, shape, beta=0.97, mode="bisect"), f0, want_alpha=True)
    same = np.abs(ag - ao) <= 1e-12
    assert same.mean() > 0.9
    for s in np.nonzero(~same)[0][:20]:
        g = orc.G(lat + 256, f0[:, s], ag[s])
        assert -1e-13 - 1e-16 <= g <= 1e-16
    sim.close()


@pytest.mark.parametrize("lat", [2, 3, 19])
def test_burg_far_from_equilibrium(gpu, orc, lat):
    """alpha_* < 2 on many sites (alpha = 1 there, the limit of Eq. (9)) and
    the log1p path: one FP64 step against the oracle."""
    shape = SHAPES[lat]
    N = int(np.prod(shape))
    f0 = _state(lat, N, seed=2199 + lat, eps=0.7, tilt=0.2, log_uniform=False)
    sim = _sim(gpu, lat, shape, f0, storage="f64", beta=0.9, diag=gpu.DIAG_ALPHA | gpu.DIAG_COUNTS)
    sim.step(1)
    fg = sim.populations().cpu().numpy()
    fo, ao, d = orc.step(_ocfg(orc, lat, shape, beta=0.9), f0, want_alpha=True, want_diag=True)
    assert d["n_alphastar_lt2"] > N // 20
    assert np.max(np.abs(fg - fo) / np.abs(fo)) <= 1e-12
    ag = sim.alpha_field().cpu().numpy()
    assert np.max(np.abs(ag - ao)) <= 1e-11
    assert np.sum(ag == 1.0) >= d["n_alphastar_lt2"] - 2
    st = sim.stats()
    assert st["n_alphastar_lt2"] == d["n_alphastar_lt2"]
    sim.close()


@pytest.mark.parametrize("lat", [1, 2, 3, 19])
@pytest.mark.parametrize("rows", [False, True])
def test_burg_one_step_fp32_storage(gpu, orc, lat, rows):
    shape = (ROWS if rows else SHAPES)[lat]
    N = int(np.prod(shape))
    f0 = _state(lat, N, seed=2300 + lat + 7 * rows, eps=0.02, tilt=0.05)
    sim = _sim(gpu, lat, shape, f0, storage="f32", beta=0.97)
    fq = sim.populations().cpu().numpy()
    sim.step(1)
    fg = sim.populations().cpu().numpy()
    fo, _, _ = orc.step(_ocfg(orc, lat, shape, beta=0.97), fq)
    assert np.all(np.abs(fg - fo) <= 2.0 ** -24 * np.abs(fo) * 1.01 + 1e-300)
    sim.close()


def test_burg_taylor_green_multistep_fp64(gpu, orc):
    """2-D Taylor-Green 64^2, 300 steps, and 3-D 16^3, 60 steps, FP64
    storage: max relative population error <= 1e-11."""
    n = 64
    rho, u = Wk.taylor_green_2d(n)
    sim = _sim(gpu, 2, (n, n, 1), rho=rho, u=u, storage="f64", beta=0.95)
    sim.step(300)
    fg = sim.populations().cpu().numpy()
    cfg = _ocfg(orc, 2, (n, n, 1), beta=0.95, nthreads=16)
    fo, _, _ = orc.run(cfg, orc.init(cfg, rho, u), 300)
    assert np.max(np.abs(fg - fo) / np.abs(fo)) <= 1e-11
    sim.close()
    n3 = 16
    rho3, u3 = Wk.taylor_green_3d(n3)
    b3 = Wk.tgv3d_beta(n3)
    for lat in (3, 19):
        sim = _sim(gpu, lat, (n3, n3, n3), rho=rho3, u=u3, storage="f64", beta=b3)
        sim.step(60)
        fg = sim.populations().cpu().numpy()
        cfg = _ocfg(orc, lat, (n3, n3, n3), beta=b3, nthreads=16)
        fo, _, _ = orc.run(cfg, orc.init(cfg, rho3, u3), 60)
        assert np.max(np.abs(fg - fo) / np.abs(fo)) <= 1e-11, lat
        sim.close()


def test_burg_batch_rules(gpu):
    """A batch shares one kernel: Burg and Boltzmann simulations cannot be
    stepped together; Burg simulations batched equal alone, bitwise."""
    n = 32
    rho, u = Wk.taylor_green_2d(n)
    a = _sim(gpu, 2, (n, n, 1), rho=rho, u=u, beta=0.97)
    b = gpu.Simulation("d2q9", n, n, 1, rho0=rho, u0=u, beta=0.97)
    with pytest.raises(gpu.ElbmError, match="entropy"):
        gpu.step_batch([a, b], [1, 1])
    b.close()
    c = _sim(gpu, 2, (48, 40, 1), rho=np.ones(48 * 40),
             u=0.05 * np.ones((2, 48 * 40)), beta=0.97)
    gpu.step_batch([a, c], [5, 3])
    ra, rc = a.populations().cpu().numpy(), c.populations().cpu().numpy()
    with _sim(gpu, 2, (n, n, 1), rho=rho, u=u, beta=0.97) as a1:
        a1.step(5)
        assert np.array_equal(a1.populations().cpu().numpy(), ra)
    with _sim(gpu, 2, (48, 40, 1), rho=np.ones(48 * 40), u=0.05 * np.ones((2, 48 * 40)),
              beta=0.97) as c1:
        c1.step(3)
        assert np.array_equal(c1.populations().cpu().numpy(), rc)
    a.close()
    c.close()


def test_burg_full_size_sampled(gpu, orc):
    """The 512^3 D3Q27 Taylor-Green box of the Burg-entropy timing (FP32
    storage, closed form): one step after three, checked against the
    oracle's collision of the GPU's decoded pre-state at 2048 sampled sites
    (row ends and the last site included); one FP32 rounding of the output."""
    n = 512
    b = Wk.tgv3d_beta(n)
    rho, u = Wk.taylor_green_3d(n)
    sim = _sim(gpu, 3, (n, n, n), rho=rho, u=u, storage="f32", beta=b)
    del rho, u
    sim.step(3)
    rng = np.random.default_rng(533)
    sites = np.unique(np.concatenate([rng.integers(0, n ** 3, 2040),
                                      [0, n - 1, n * n - 1, n ** 3 - n, n ** 3 - 1]]))
    pre = sim.gather(sites, 0).cpu().numpy()
    sim.step(1)
    post = sim.gather(sites, 1).cpu().numpy()
    sim.close()
    cfg = orc.Config(D=3, nx=1, beta=b, entropy="burg")
    for k in range(sites.size):
        ft, _ = orc.collide_site(cfg, pre[:, k])
        assert np.all(np.abs(post[:, k] - ft) <= 2.0 ** -24 * np.abs(ft) * 1.01), sites[k]
    torch.cuda.empty_cache()
