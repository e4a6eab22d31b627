"""CPU checks of the C ABI: the library loads, exports every declared
symbol, and rejects bad arguments before touching a device."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(pmp\w+)\s*\(", text, re.M))
    return names


def test_header_declares_boundary_calls():
    d = _declared()
    for name in ("pmp_setup", "pmp_iterate", "pmp_solve", "pmp_residuals"):
        assert name in d


def test_library_exports_every_declared_symbol():
    from paper_2509_10722_amd import pmp
    pmp.load_library()
    out = subprocess.run(["nm", "-D", "--defined-only", pmp.LIB_PATH],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\b(pmp_\w+)\b", out))
    missing = _declared() - exported
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_2509_10722_amd import pmp
    assert _declared() <= set(pmp.exported_symbols())


def test_defaults_follow_the_paper():
    from paper_2509_10722_amd import pmp
    p = pmp.params_default()
    assert (p.rho0, p.alpha, p.mu, p.gamma, p.adapt_every) == (1.0, 1.6, 2.0, 1.1, 50)
    assert p.check_every == 10 and abs(p.eps_abs - 1e-4) < 1e-18 and p.eps_rel == 0.0


def test_workspace_size_and_shape_errors():
    from paper_2509_10722_amd import pmp
    lib = pmp.load_library()
    prob = pmp.pmp_problem(m=10, n=20, nnz=50, dtype=pmp.PMP_F32)
    prm = pmp.params_default()
    b = ctypes.c_size_t()
    assert lib.pmp_workspace_size(ctypes.byref(prob), ctypes.byref(prm), ctypes.byref(b)) == 0
    assert b.value > 0 and b.value % 256 == 0
    prob.nnz = 1 << 31
    assert lib.pmp_workspace_size(ctypes.byref(prob), ctypes.byref(prm),
                                  ctypes.byref(b)) == pmp.PMP_ERR_SHAPE


def test_binned_layout_size_limits():
    from paper_2509_10722_amd import pmp
    lib = pmp.load_library()
    b = ctypes.c_size_t()
    prm = pmp.params_default()
    # a billion links and streams, few nonzeros: far too many tiles for the
    # binned layout, which is refused when asked for and not chosen by AUTO
    prob = pmp.pmp_problem(m=1 << 30, n=1 << 30, nnz=1 << 22, dtype=pmp.PMP_F32)
    prm.layout = pmp.PMP_LAYOUT_BINNED
    assert lib.pmp_workspace_size(ctypes.byref(prob), ctypes.byref(prm),
                                  ctypes.byref(b)) == pmp.PMP_ERR_SHAPE
    assert b"tiles" in lib.pmp_last_error()
    prm.layout = pmp.PMP_LAYOUT_AUTO
    assert lib.pmp_workspace_size(ctypes.byref(prob), ctypes.byref(prm), ctypes.byref(b)) == 0
    gather = b.value
    prm.layout = pmp.PMP_LAYOUT_GATHER
    assert lib.pmp_workspace_size(ctypes.byref(prob), ctypes.byref(prm), ctypes.byref(b)) == 0
    assert b.value == gather


@pytest.mark.parametrize("field,value,status", [
    ("rho0", 0.0, 1), ("alpha", 2.5, 1), ("mu", 1.0, 1), ("gamma", 0.5, 1),
    ("eps_rel", -1e-4, 1), ("eps_rel", float("nan"), 1),
    ("check_every", 0, 1), ("adapt_every", 15, 1),
])
def test_setup_rejects_bad_params_without_device_work(field, value, status):
    from paper_2509_10722_amd import pmp
    lib = pmp.load_library()
    rp = np.array([0, 1], np.int32)
    ci = np.array([0], np.int32)
    c = np.ones(1, np.float32)
    w = np.ones(1, np.float32)
    u = np.zeros(1, np.uint8)
    prob = pmp.pmp_problem(1, 1, 1, rp.ctypes.data, ci.ctypes.data, c.ctypes.data,
                           w.ctypes.data, u.ctypes.data, 0.0, 10.0, pmp.PMP_F32, pmp.PMP_MEM_HOST)
    prm = pmp.params_default(**{field: value})
    h = ctypes.c_void_p()
    st = lib.pmp_setup(ctypes.byref(prob), ctypes.byref(prm), None, 0, None, ctypes.byref(h))
    assert st == status
    assert lib.pmp_last_error().decode()


@pytest.mark.parametrize("lo,hi,m", [(-1.0, 1.0, 1), (2.0, 1.0, 1), (0.0, 1.0, 0)])
def test_setup_rejects_bad_box_or_shape(lo, hi, m):
    from paper_2509_10722_amd import pmp
    lib = pmp.load_library()
    prob = pmp.pmp_problem(m=m, n=0, nnz=0, lo=lo, hi=hi, dtype=pmp.PMP_F32,
                           memory=pmp.PMP_MEM_HOST)
    prm = pmp.params_default()
    h = ctypes.c_void_p()
    st = lib.pmp_setup(ctypes.byref(prob), ctypes.byref(prm), None, 0, None, ctypes.byref(h))
    assert st in (pmp.PMP_ERR_INVALID, pmp.PMP_ERR_SHAPE)


def test_status_strings():
    from paper_2509_10722_amd import pmp
    lib = pmp.load_library()
    assert lib.pmp_status_string(0) == b"ok"
    assert lib.pmp_status_string(6) == b"not converged"


def test_null_handles_are_rejected():
    from paper_2509_10722_amd import pmp
    lib = pmp.load_library()
    b = ctypes.c_size_t()
    sizes = (ctypes.c_int64 * 3)()
    assert lib.pmp_get_path_prices(None, None) == pmp.PMP_ERR_INVALID
    assert lib.pmp_prune_workspace_size(None, ctypes.byref(b)) == pmp.PMP_ERR_INVALID
    assert lib.pmp_prune(None, None, None, 0, None, None, None, None, None, None, None, None,
                         sizes) == pmp.PMP_ERR_INVALID
    assert lib.pmp_state_size(None, ctypes.byref(b)) == pmp.PMP_ERR_INVALID
    assert lib.pmp_last_error().decode()


@pytest.mark.parametrize("chunk,status", [(0, 0), (1024, 0), (8192, 0), (1 << 20, 0),
                                          (1023, 1), (-5, 1), ((1 << 20) + 1, 1)])
def test_batch_options_heavy_chunk_range(chunk, status):
    """pmp_batch_options: defaults, and heavy_chunk accepted as 0 or within
    [1024, 2^20] by pmp_batch_workspace_size (host-only call)."""
    from paper_2509_10722_amd import pmp
    lib = pmp.load_library()
    o = pmp.batch_options_default()
    assert (list(o.tile_cap), o.wg_per_cu, o.heavy_chunk) == ([8192] * 3, 4, 8192)
    o.heavy_chunk = chunk
    prob = pmp.pmp_problem(m=10, n=20, nnz=50, dtype=pmp.PMP_F32)
    prm = pmp.params_default()
    b = ctypes.c_size_t()
    st = lib.pmp_batch_workspace_size(1, ctypes.byref(prob), ctypes.byref(prm), ctypes.byref(o),
                                      ctypes.byref(b))
    assert st == (pmp.PMP_ERR_INVALID if status else 0)
    if not status:
        assert b.value > 0 and b.value % 256 == 0


@pytest.mark.parametrize("k,ok", [(0, True), (1, True), (24, True), (30, True), (-1, False),
                                  (31, False)])
def test_batch_options_wait_bound_range(k, ok):
    """pmp_batch_options.wait_log2 (the bound of a grid barrier wait, 2^k
    polls): default 24, accepted in [0, 30]."""
    from paper_2509_10722_amd import pmp
    lib = pmp.load_library()
    o = pmp.batch_options_default()
    assert o.wait_log2 == 24
    o.wait_log2 = k
    prob = pmp.pmp_problem(m=10, n=20, nnz=50, dtype=pmp.PMP_F32)
    prm = pmp.params_default()
    b = ctypes.c_size_t()
    st = lib.pmp_batch_workspace_size(1, ctypes.byref(prob), ctypes.byref(prm), ctypes.byref(o),
                                      ctypes.byref(b))
    assert st == (0 if ok else pmp.PMP_ERR_INVALID)
