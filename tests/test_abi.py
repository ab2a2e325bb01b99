"""CPU-side checks of the C ABI: the library loads, exports every entry point that
include/lmfr.h declares, and rejects invalid arguments before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1903_06304_amd import lmfr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lmfr.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fr_[a-z0-9_]+)\s*\(", src)))


def _lib():
    if not os.path.exists(lmfr.LIB_PATH):
        pytest.skip("liblmfr.so not built")
    return lmfr.load_library()


def test_header_declares_expected_entry_points():
    decl = _declared()
    for name in ["fr_create", "fr_set_geometry", "fr_residual", "fr_jvp", "fr_vjp",
                 "fr_block_jacobi_factor", "fr_block_jacobi_apply", "fr_bdf2_step", "fr_last_error",
                 "fr_destroy"]:
        assert name in decl
    assert sorted(lmfr.EXPORTS) == decl


def test_library_exports_every_declared_symbol():
    L = _lib()
    for name in _declared():
        assert hasattr(L, name), name


def _params(order=2, E=4):
    return lmfr.fr_params(order, order, E, 1, 0, 1.4, 0.1, 100.0, 0.72, 1.0, 1.0, 0.1)


def _table(nx=2, ny=2):
    from paper_1903_06304_amd import inputs as I
    m = I.Mesh(nx, ny, 1)
    return m.connectivity()


def _create(prm, nbr, nbf):
    L = _lib()
    h = ctypes.c_void_p()
    st = L.fr_create(ctypes.byref(prm), nbr.ctypes.data_as(ctypes.c_void_p),
                     nbf.ctypes.data_as(ctypes.c_void_p), None, ctypes.byref(h))
    return st, h


def test_create_rejects_unsupported_order():
    nbr, nbf, _ = _table()
    st, h = _create(_params(order=5), nbr, nbf)
    assert st == lmfr.FR_EUNSUPPORTED and not h.value
    assert b"order" in _lib().fr_last_error()
    st, _ = _create(_params(order=0), nbr, nbf)
    assert st == lmfr.FR_EUNSUPPORTED


def test_create_rejects_bad_tables_and_parameters():
    nbr, nbf, _ = _table()
    bad = nbr.copy(); bad[0, 0] = 99
    st, _ = _create(_params(), bad, nbf)
    assert st == lmfr.FR_EINVAL
    nbr3, nbf3, _ = _table(3, 3)
    asym = nbr3.copy(); asym[0, 1] = asym[0, 0]
    st, _ = _create(_params(E=9), asym, nbf3)
    assert st == lmfr.FR_EINVAL
    prm = _params(); prm.mach_ref = -1.0
    st, _ = _create(prm, nbr, nbf)
    assert st == lmfr.FR_EINVAL
    unknown = nbr.copy(); unknown[0, 0] = -4     # boundary codes are -1..-3
    st, _ = _create(_params(), unknown, nbf)
    assert st == lmfr.FR_EINVAL and b"boundary" in _lib().fr_last_error()
    prm = _params(); prm.n_elem = 0
    st, _ = _create(prm, nbr, nbf)
    assert st == lmfr.FR_EINVAL


def test_null_arguments_rejected():
    L = _lib()
    assert L.fr_create(None, None, None, None, None) == lmfr.FR_EINVAL
    assert L.fr_residual(None, None, None, None) == lmfr.FR_EINVAL
    assert L.fr_jvp(None, None, None, None, None, None) == lmfr.FR_EINVAL
    assert L.fr_vjp(None, None, None, None, None) == lmfr.FR_EINVAL
    assert L.fr_bdf2_step(None, None, None, None, None, None) == lmfr.FR_EINVAL
    assert L.fr_block_jacobi_apply(None, None, None, None) == lmfr.FR_EINVAL
    L.fr_destroy(None)


def test_binding_refuses_without_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("device present")
    from paper_1903_06304_amd import inputs as I
    c = I.config_c1(nx=2)
    nbr, nbf, flip = c.connectivity()
    with pytest.raises(RuntimeError):
        lmfr.Context(c.prm, nbr, nbf, flip)


def test_null_arguments_rejected_everywhere():
    """Every entry point validates its handles and pointers before any device work."""
    L = _lib()
    vp = None
    assert L.fr_set_geometry(vp, vp, vp, vp) == lmfr.FR_EINVAL
    assert L.fr_bdf_operator(vp, vp, vp, 1.0, 0.0, vp, vp) == lmfr.FR_EINVAL
    assert L.fr_block_jacobi_factor(vp, vp, 1.0, 0.0, 0, vp) == lmfr.FR_EINVAL
    assert L.fr_get_blocks(vp, vp, vp) == lmfr.FR_EINVAL
    assert L.fr_affine_elements(vp, vp, vp) == lmfr.FR_EINVAL
    assert L.fr_set_farfield(vp, vp) == lmfr.FR_EINVAL
    assert L.fr_steady_solve(vp, vp, vp, vp, vp) == lmfr.FR_EINVAL
    assert L.fr_batch_steady_solve(vp, vp, vp, vp, vp) == lmfr.FR_EINVAL
    assert L.fr_set_option(vp, b"graph", 1) == lmfr.FR_EINVAL
    assert L.fr_autotune(vp, None, vp) == lmfr.FR_EINVAL
    assert L.fr_batch_create(vp, 0, vp) == lmfr.FR_EINVAL
    n = ctypes.c_int64()
    assert L.fr_batch_layout(vp, ctypes.byref(n), vp) == lmfr.FR_EINVAL
    assert L.fr_batch_residual(vp, vp, vp, vp) == lmfr.FR_EINVAL
    assert L.fr_batch_jvp(vp, vp, vp, vp, vp) == lmfr.FR_EINVAL
    assert L.fr_batch_bdf2_step(vp, vp, vp, vp, vp, vp) == lmfr.FR_EINVAL
    assert L.fr_batch_set_option(vp, b"graph", 1) == lmfr.FR_EINVAL
    assert L.fr_batch_autotune(vp, None, vp) == lmfr.FR_EINVAL
    L.fr_batch_destroy(vp)
    arr = (ctypes.c_void_p * 2)(None, None)
    assert L.fr_batch_create(arr, 2, ctypes.byref(ctypes.c_void_p())) == lmfr.FR_EINVAL


def test_create_rejects_sizes_beyond_32_bit_offsets():
    # 4 E (p+1)^2 >= 2^31 would overflow the kernels' 32-bit state offsets
    nbr, nbf, _ = _table()
    prm = _params(order=4, E=(1 << 31) // 100 + 1)
    st, h = _create(prm, nbr, nbf)
    assert st == lmfr.FR_EINVAL and not h.value
    assert b"2^31" in _lib().fr_last_error()
    # p = 1: 4 flux points per face pair outnumber the 4 solution points; 8 E * 8 >= 2^32 bytes
    # per flux-point field would overflow the fused kernels' 32-bit byte offsets (the check
    # comes before the tables are read, so the small table is never indexed past its end)
    prm = _params(order=1, E=1 << 26)
    st, h = _create(prm, nbr, nbf)
    assert st == lmfr.FR_EINVAL and not h.value
    assert b"2^32" in _lib().fr_last_error()


def test_library_marks_solver_phases_with_roctx_ranges():
    """The solver phases (BDF2 step, Newton iteration, GMRES solve, refresh, steady solve,
    autotuner) push named roctx ranges: the library imports the range calls from ROCm's
    roctx library, so rocprofv3 --marker-trace shows them."""
    import shutil
    import subprocess
    if not os.path.exists(lmfr.LIB_PATH):
        pytest.skip("liblmfr.so not built")
    if shutil.which("readelf") is None:
        pytest.skip("readelf missing")
    dyn = subprocess.run(["readelf", "-d", lmfr.LIB_PATH], capture_output=True, text=True).stdout
    assert "librocprofiler-sdk-roctx" in dyn
    syms = subprocess.run(["readelf", "--dyn-syms", "-W", lmfr.LIB_PATH], capture_output=True, text=True).stdout
    undefined = {ln.split()[-1].split("@")[0] for ln in syms.splitlines() if " UND " in ln}
    assert {"roctxRangePushA", "roctxRangePop"} <= undefined
    strings = open(lmfr.LIB_PATH, "rb").read()
    for name in (b"lmfr: BDF2 step (Newton loop)", b"lmfr: Newton iteration", b"lmfr: GMRES solve",
                 b"lmfr: steady solve", b"lmfr: autotune"):
        assert name in strings
