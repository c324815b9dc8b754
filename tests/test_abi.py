"""CPU-side checks of the C ABI: the library loads, exports every function
declared in include/polyaipm.h, and rejects invalid input before any device
call (no compute call is made here)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "polyaipm.h")


def _lib():
    from paper_1411_3769_amd import polyaipm
    if not os.path.exists(polyaipm.LIB_PATH):
        pytest.skip("libpolyaipm.so not built")
    return polyaipm


def declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(psdp_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_expected_entry_points():
    names = declared()
    for must in ("psdp_polya_setup", "psdp_ipm_solve", "psdp_ipm_solve_batched", "psdp_query",
                 "psdp_get_polya", "psdp_free", "psdp_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    P = _lib()
    lib = C.CDLL(P.LIB_PATH)
    for name in declared():
        assert hasattr(lib, name), name
    assert set(P.EXPORTS) <= set(declared())


def test_version_and_defaults():
    P = _lib()
    assert "gfx950" in P.version()
    o = P.make_opts(stream=None)
    assert o.gap_tol == 1e-8 and o.max_iter == 100 and abs(o.sigma - 1 / 3) < 1e-15
    assert o.ladder_rho == 0.9 and o.step_frac == 0.95 and o.ladder_len == 300


@pytest.mark.parametrize("args,code,frag", [
    (dict(n=0), -1, "n must be"),
    (dict(n=129), -1, "n must be"),
    (dict(l=0), -1, "l must be"),
    (dict(dp=-1), -1, "negative degree"),
    (dict(d=20), -2, "above 20"),
    (dict(nan=True), -1, "non-finite"),
])
def test_setup_validation(args, code, frag):
    P = _lib()
    n, l, dp, d = args.get("n", 3), args.get("l", 2), args.get("dp", 1), args.get("d", 1)
    A = np.zeros((max(l, 1), max(n, 1), max(n, 1)))
    if args.get("nan"):
        A[0, 0, 0] = np.nan
    with pytest.raises(P.PsdpError) as ei:
        P.polya_setup(A, n, l, dp, d)
    assert ei.value.code == code
    assert frag in str(ei.value)


def test_null_arguments_rejected():
    P = _lib()
    lib = P.load()
    h = C.c_void_p()
    assert lib.psdp_polya_setup(None, 3, 2, 1, 1, None, C.byref(h)) == -1
    assert b"NULL" in lib.psdp_last_error()
    assert lib.psdp_query(None, None) == -1
    assert lib.psdp_ipm_solve(None, None, None) == -1
    assert lib.psdp_ipm_solve_batched(None, 0, None, None) == -1
    lib.psdp_free(None)   # ignored


def test_batched_setup_validation():
    P = _lib()
    lib = P.load()
    out = (C.c_void_p * 2)()
    assert lib.psdp_polya_setup_batched(-1, None, None, None, None, None, None, out) == -1
    assert lib.psdp_polya_setup_batched(2, None, None, None, None, None, None, out) == -1
    assert b"NULL" in lib.psdp_last_error()
    assert lib.psdp_polya_setup_batched(0, None, None, None, None, None, None, None) == 0
    A = np.zeros((2, 3, 3))
    A[0, 0, 0] = np.nan
    with pytest.raises(P.PsdpError) as ei:
        P.polya_setup_batched([(A, 3, 2, 1, 1), (np.zeros((2, 3, 3)), 3, 2, 1, 1)])
    assert ei.value.code == -1
    assert "system 0" in str(ei.value) and "non-finite" in str(ei.value)


def test_product_path_has_no_cpu_fallback(tmp_path):
    from paper_1411_3769_amd import polyaipm as P
    saved = P._lib
    try:
        P._lib = None
        with pytest.raises(ImportError):
            P.load(str(tmp_path / "missing.so"))
    finally:
        P._lib = saved


@pytest.mark.parametrize("dims,prec,batch,frag", [
    ((4, 3, 3, 2), 0, 8, "precision"),
    ((4, 3, 3, 2), 1, 0, "max_batch"),
    ((0, 3, 3, 2), 1, 8, "width"),
])
def test_mlp_create_validation(dims, prec, batch, frag):
    P = _lib()
    lib = P.load()
    h = C.c_void_p()
    d = (C.c_int * 4)(*dims)
    rc = lib.psdp_mlp_create(C.cast(d, C.c_void_p), prec, batch, C.byref(h))
    assert rc == -1 and frag in lib.psdp_last_error().decode()
    assert not h.value


def test_warm_start_option_validation():
    P = _lib()
    o = P.make_opts(stream=None)
    assert o.warm_margin == 1e-6 and o.warm_center == 1 and o.warm_iter_cap == 0
    assert not o.warm_y and not o.warm_logx and o.label_gap == 0.0



def test_result_buffers_of_a_batch():
    """ipm_solve_batched's caller buffers: one host allocation, per system the
    views P [L0][n][n], y [K], logx / label_logx [L+M], label_y [K], each C
    result pointing at its own views and no two views overlapping."""
    import types
    P = _lib()
    shapes = [types.SimpleNamespace(L0=10, n=10, K=550, L=35, M=56),
              types.SimpleNamespace(L0=4, n=3, K=24, L=10, M=20),
              types.SimpleNamespace(L0=1, n=1, K=1, L=1, M=1)]
    sdps = shapes * 3
    arr = (P.CResult * len(sdps))()
    views = P._prep_batch(sdps, 0, arr)
    spans = []
    for s, r, (Pm, y, (lx, ly, llx), hist) in zip(sdps, arr, views):
        assert Pm.shape == (s.L0, s.n, s.n) and y.shape == (s.K,) and ly.shape == (s.K,)
        assert lx.shape == (s.L + s.M,) and llx.shape == (s.L + s.M,) and hist is None
        got = (r.P, r.y, r.logx, r.label_y, r.label_logx)
        assert got == tuple(a.ctypes.data for a in (Pm, y, lx, ly, llx))
        assert r.history_cap == 0
        spans += [(a.ctypes.data, a.ctypes.data + a.nbytes) for a in (Pm, y, lx, ly, llx)]
    spans.sort()
    assert all(a[1] <= b[0] for a, b in zip(spans, spans[1:]))
    # history records when asked for
    arr2 = (P.CResult * 2)()
    views2 = P._prep_batch(shapes[:2], 7, arr2)
    assert all(v[3] is not None and len(v[3]) == 7 for v in views2)
    assert arr2[0].history_cap == 7
