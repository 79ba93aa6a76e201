"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/elbm.h declares, its structs have the header's
layout, and configuration errors are reported before any device work."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_1904_00866_amd import elbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "elbm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(elbm_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    L = elbm.lib()
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(elbm.EXPORTS)


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(f'''#include <stdio.h>
#include <stddef.h>
#include "{HEADER}"
int main(void) {{
  printf("%zu %zu %zu %zu %zu\\n", sizeof(elbm_config), offsetof(elbm_config, beta),
         offsetof(elbm_config, rho_ref), offsetof(elbm_config, diag), sizeof(elbm_stats_t));
  printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(elbm_server_config), sizeof(elbm_request),
         offsetof(elbm_request, nsteps), offsetof(elbm_request, keep_state),
         sizeof(elbm_request_info), offsetof(elbm_request_info, footprint),
         sizeof(elbm_server_stats));
  return 0;
}}''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-o", str(exe), str(src)], check=True)
    got = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    want = [C.sizeof(elbm.Config), elbm.Config.beta.offset, elbm.Config.rho_ref.offset,
            elbm.Config.diag.offset, C.sizeof(elbm.Stats),
            C.sizeof(elbm.ServerConfig), C.sizeof(elbm.Request), elbm.Request.nsteps.offset,
            elbm.Request.keep_state.offset, C.sizeof(elbm.RequestInfo),
            elbm.RequestInfo.footprint.offset, C.sizeof(elbm.ServerStats)]
    assert [int(v) for v in got] == want


def test_default_config_and_state_bytes():
    cfg = elbm.make_config("d3q27", 64, 64, 64)
    assert cfg.alpha_mode == 0 and cfg.storage == 1 and cfg.alpha_fp64 == 1
    assert abs(cfg.beta - 0.95) < 1e-15 and cfg.root_tol == 1e-13
    nb = elbm.state_bytes(cfg)
    assert nb >= 2 * 27 * 64 ** 3 * 4
    assert nb < 2 * 27 * (64 ** 3 + 1024) * 4 + 65536
    cfg16 = elbm.make_config("d3q27", 64, 64, 64, storage="f16dev")
    assert elbm.state_bytes(cfg16) < nb
    cfgd = elbm.make_config("d3q27", 64, 64, 64, diag=elbm.DIAG_ALPHA | elbm.DIAG_COUNTS)
    assert elbm.state_bytes(cfgd) >= nb + 8 * 64 ** 3


def test_d3q19_config_and_state_bytes():
    """D3Q19 (lattice code 19) is a three-dimensional lattice of 19
    directions: two buffers of 19 populations per (padded) site; the codes
    4..18 are no lattice."""
    cfg = elbm.make_config("d3q19", 64, 64, 64)
    assert cfg.lattice == 19 and elbm.lattice_dq(19) == (3, 19)
    nb = elbm.state_bytes(cfg)
    assert 2 * 19 * 64 ** 3 * 4 <= nb < 2 * 19 * (64 ** 3 + 2048) * 4 + 65536
    assert elbm.state_bytes(elbm.make_config("d3q19", 64, 64, 64, storage="f64")) > nb
    for mode in ("closed", "newton", "bisect", "bgk", "secant"):
        assert elbm.state_bytes(elbm.make_config("d3q19", 8, 8, 8, mode=mode)) > 0
    assert elbm.state_bytes(elbm.make_config("d3q19", 8, 8, 8, fp64=False)) > 0
    for bad in (4, 9, 18, 27):
        c = elbm.make_config("d3q27", 8, 8, 8)
        c.lattice = bad
        assert elbm.lib().elbm_state_bytes(C.byref(c)) == 0
        with pytest.raises(elbm.ElbmError, match="unknown lattice"):
            elbm.state_bytes(c)


def test_burg_entropy_configs():
    """Burg's entropy is built for the entropic alpha modes with FP64
    arithmetic and FP64 / FP32 storage on every lattice; LBGK (no entropy),
    deviation storage and FP32 arithmetic are refused, unknown entropies are
    invalid."""
    for lat in ("d1q3", "d2q9", "d3q27", "d3q19"):
        shape = {"d1q3": (64, 1, 1), "d2q9": (16, 16, 1)}.get(lat, (8, 8, 8))
        for mode in ("closed", "newton", "bisect", "secant"):
            for storage in ("f64", "f32"):
                cfg = elbm.make_config(lat, *shape, mode=mode, storage=storage, entropy="burg")
                assert elbm.state_bytes(cfg) > 0
    # elbm_state_bytes returns 0 and sets the message (the status of the
    # configuration check is in the message's wording)
    for kw, msg in [(dict(mode="bgk"), "LBGK uses no entropy"), (dict(storage="f16dev"), "no kernel"),
                    (dict(storage="f32dev"), "no kernel"), (dict(fp64=False), "no kernel"),
                    (dict(entropy=2), "unknown entropy")]:
        args = dict(entropy="burg")
        args.update(kw)
        with pytest.raises(elbm.ElbmError, match=msg):
            elbm.state_bytes(elbm.make_config("d2q9", 16, 16, **args))
    c = elbm.make_config("d2q9", 16, 16)
    c.reserved = 1
    with pytest.raises(elbm.ElbmError, match="reserved"):
        elbm.state_bytes(c)


def test_mixed_arithmetic_configs():
    """ELBM_ARITH_MIXED (FP32 site arithmetic, FP64 alpha evaluation) is
    built for the closed form on the tensor-product lattices with FP32 and
    deviation storage and the Boltzmann entropy; other combinations report
    that no kernel exists, and unknown codes are rejected."""
    for lat, shape in (("d1q3", (64, 1, 1)), ("d2q9", (16, 16, 1)), ("d3q27", (8, 8, 8))):
        for storage in ("f32", "f32dev", "f16dev"):
            cfg = elbm.make_config(lat, *shape, storage=storage, fp64="mixed")
            assert cfg.alpha_fp64 == 2
            assert elbm.state_bytes(cfg) > 0
    for kw in (dict(lattice="d3q19"), dict(entropy="burg")):
        args = dict(lattice="d2q9", fp64="mixed")
        args.update(kw)
        lat = args.pop("lattice")
        with pytest.raises(elbm.ElbmError, match="no kernel"):
            elbm.state_bytes(elbm.make_config(lat, 8, 8, 8 if lat == "d3q19" else 1, **args))
    c = elbm.make_config("d2q9", 16, 16)
    c.alpha_fp64 = 3
    with pytest.raises(elbm.ElbmError, match="alpha_fp64"):
        elbm.state_bytes(c)


def test_large_boxes_fit_the_layout():
    """A 1024^3 FP32 D3Q27 state (232 GB with both buffers) is a valid
    configuration: the blocked layout has no per-buffer size limit."""
    cfg = elbm.make_config("d3q27", 1024, 1024, 1024)
    nb = elbm.state_bytes(cfg)
    assert 2 * 27 * 4 * 1024 ** 3 <= nb < 2 * 27 * 4 * 1024 ** 3 + (1 << 24)


@pytest.mark.parametrize("kw,msg", [
    (dict(beta=1.0), "beta"),
    (dict(beta=0.0), "beta"),
    (dict(mode="newton", fp64=False), "closed-form alpha only"),
    (dict(mode="bgk", fp64="mixed"), "closed-form alpha only"),
    (dict(storage="f64", fp64=False), "FP64 storage"),
    (dict(storage="f64", fp64="mixed"), "FP64 storage"),
    (dict(diag=elbm.DIAG_SUMS), "SUMS"),
    (dict(diag=64), "diagnostics"),
    (dict(storage="f16dev", rho_ref=0.0), "rho_ref"),
    (dict(mode="secant", secant_iters=0), "secant"),
])
def test_invalid_configs_are_rejected(kw, msg):
    cfg = elbm.make_config("d2q9", 32, 32, 1, **kw)
    assert elbm.lib().elbm_state_bytes(C.byref(cfg)) == 0
    assert msg in elbm.lib().elbm_last_error().decode()


@pytest.mark.parametrize("dims,msg", [
    (("d2q9", 32, 32, 2), "nz = 1"),
    (("d1q3", 32, 2, 1), "ny = nz = 1"),
    (("d3q27", 0, 4, 4), ">= 1"),
    (("d3q27", 2 ** 20, 4, 4), "extent"),
    (("d3q27", 2048, 2048, 1024), "sites exceed"),
])
def test_invalid_boxes_are_rejected(dims, msg):
    cfg = elbm.make_config(*dims)
    assert elbm.lib().elbm_state_bytes(C.byref(cfg)) == 0
    assert msg in elbm.lib().elbm_last_error().decode()


def test_init_argument_errors_before_device_work():
    L = elbm.lib()
    cfg = elbm.make_config("d2q9", 8, 8, 1)
    h = C.c_void_p()
    assert L.elbm_init(C.byref(cfg), None, None, None, 0, None, C.byref(h)) == -1
    assert b"dev_state" in L.elbm_last_error()
    assert L.elbm_init(C.byref(cfg), None, None, C.c_void_p(256), 10, None, C.byref(h)) == -3
    assert L.elbm_init(C.byref(cfg), None, None, C.c_void_p(255), 1 << 30, None,
                       C.byref(h)) == -1
    assert b"aligned" in L.elbm_last_error()
    assert L.elbm_init(C.byref(cfg), None, None, C.c_void_p(256), 1 << 30, None, None) == -1
    assert L.elbm_step(None, 1) == -1
    assert L.elbm_destroy(None) == 0
    assert L.elbm_time(None) == -1
    assert L.elbm_checkpoint_bytes(None) == 0
    t = C.c_int64()
    assert L.elbm_export(None, None, 0, C.byref(t)) == -1
    assert L.elbm_import(None, None, 0, 0) == -1
    assert L.elbm_step_noalloc(None, 1, elbm.DIAG_COUNTS, None) == -1


def test_batch_argument_errors():
    L = elbm.lib()
    assert L.elbm_step_batch(None, None, 0) == 0
    assert L.elbm_step_batch(None, None, -1) == -1
    assert L.elbm_step_batch(None, None, 2) == -1


def test_server_argument_errors_before_device_work():
    L = elbm.lib()
    h = C.c_void_p()
    sc = elbm.ServerConfig(None, 1 << 20, None, 4, 10)
    assert L.elbm_server_create(C.byref(sc), C.byref(h)) == -1
    assert b"pool" in L.elbm_last_error()
    sc = elbm.ServerConfig(C.c_void_p(4096 + 8), 1 << 20, None, 4, 10)
    assert L.elbm_server_create(C.byref(sc), C.byref(h)) == -1
    assert b"aligned" in L.elbm_last_error()
    sc = elbm.ServerConfig(C.c_void_p(4096), 1 << 20, None, 0, 10)
    assert L.elbm_server_create(C.byref(sc), C.byref(h)) == -1
    sc = elbm.ServerConfig(C.c_void_p(4096), 1 << 20, None, 4, 0)
    assert L.elbm_server_create(C.byref(sc), C.byref(h)) == -1
    sc = elbm.ServerConfig(C.c_void_p(4096), 1 << 20, None, 4, 10, -1, 0)
    assert L.elbm_server_create(C.byref(sc), C.byref(h)) == -1
    assert b"preempt_rounds" in L.elbm_last_error()
    sc = elbm.ServerConfig(C.c_void_p(4096), 1 << 20, None, 4, 10, 0, 1)
    assert L.elbm_server_create(C.byref(sc), C.byref(h)) == -1
    assert L.elbm_server_create(None, C.byref(h)) == -1
    assert L.elbm_server_submit(None, None, None) == -1
    assert L.elbm_server_poll(None, 1, None) == -1
    assert L.elbm_server_wait(None, 1, 0.0) == -1
    assert L.elbm_server_release(None, 1) == -1
    assert L.elbm_server_cancel(None, 1) == -1
    assert L.elbm_server_destroy(None) == 0
