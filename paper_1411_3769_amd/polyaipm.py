"""Python binding of libpolyaipm.so (argument marshalling only).

Every step of the set-up and of the solver runs in the HIP library; this
module converts arrays, fills the C option structs and unpacks results.  It
raises if the shared library has not been built (there is no CPU fallback).

Functions mirror the C ABI in include/polyaipm.h:
    polya_setup(A, n, l, dp, d, ...)      -> SDP handle (psdp_polya_setup)
    SDP.dims / SDP.get_polya() / SDP.basis()
    ipm_solve(sdp, **opts)               -> Result (psdp_ipm_solve)
    ipm_solve_batched([sdp, ...], **opts) -> [Result] (psdp_ipm_solve_batched)
    eval_newton(sdp, X, Z, y)            -> dict (psdp_eval_newton)
    eval_ladder(sdp, V, dV, **opts)      -> (step, kstar) (psdp_eval_ladder)
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpolyaipm.so")

FEASIBLE, INFEASIBLE, UNKNOWN = 0, 1, 2
VERDICTS = {0: "FEASIBLE", 1: "INFEASIBLE", 2: "UNKNOWN"}
REASONS = ["converged", "farkas", "stall", "max_iter", "ladder_fail", "chol_fail", "nonfinite"]
VERDICT_MODES = {"paper_then_phase1": 0, "paper_only": 1, "phase1_only": 2}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2}
STOP_RULES = {"relative": 0, "absolute": 1}
SIGMA_RULES = {"fixed": 0, "mehrotra": 1}
ERRORS = {-1: "EINVAL", -2: "EOVERFLOW", -3: "ENOMEM", -4: "EDEVICE", -5: "ENUMERIC"}
NPROF = 16
PROF_CLASSES = ["cholinv", "BT", "B", "pre", "assemble", "chol_panel", "chol_update", "trsv",
                "gemm", "ladder", "misc", "cert", "phase1"]


def new_prof() -> np.ndarray:
    """Array for psdp_opts.prof: [NPROF][2] = (device ms, launches) per class."""
    return np.zeros((NPROF, 2))

DP = C.POINTER(C.c_double)


class SetupOpts(C.Structure):
    _fields_ = [("da", C.c_int), ("d1", C.c_int), ("d2", C.c_int), ("delta", C.c_double),
                ("eps", C.c_double), ("paper_literal", C.c_int), ("a_on_device", C.c_int),
                ("form", C.c_int)]


class Dims(C.Structure):
    _fields_ = [(k, C.c_int) for k in ("n", "l", "da", "dp", "d1", "d2", "L0", "L", "M", "Na", "Nt")] + \
               [("K", C.c_int64), ("Kpad", C.c_int64), ("device_bytes", C.c_int64), ("form", C.c_int),
                ("bo", C.c_int)]


class Opts(C.Structure):
    _fields_ = [("gap_tol", C.c_double), ("feas_tol", C.c_double), ("max_iter", C.c_int),
                ("sigma", C.c_double), ("step_frac", C.c_double), ("ladder_rho", C.c_double),
                ("ladder_len", C.c_int), ("verdict_mode", C.c_int), ("precision", C.c_int),
                ("ir_max", C.c_int), ("stream", C.c_void_p), ("record_history", C.c_int), ("prof", DP),
                ("warm_y", C.POINTER(DP)), ("warm_logx", C.POINTER(DP)), ("warm_iter_cap", C.c_int),
                ("warm_margin", C.c_double), ("warm_center", C.c_int), ("asm_path", C.c_int),
                ("solve_path", C.c_int), ("use_graph", C.c_int),
                ("label_gap", C.c_double), ("chol_shift_max", C.c_double),
                ("chol_shift_force", C.c_double), ("stop_rule", C.c_int), ("sigma_rule", C.c_int),
                ("chol_panels", C.c_int), ("chol_subpanels", C.c_int)]


class IterRec(C.Structure):
    _fields_ = [("iter", C.c_int)] + [(k, C.c_double) for k in
                                      ("phi", "psi", "gap_rel", "pinf", "dinf", "mu", "tp", "td")]


class CResult(C.Structure):
    # caller buffers (double *) are declared as plain addresses: same ABI,
    # and integer addresses assign without building pointer objects
    _fields_ = [("verdict", C.c_int), ("reason", C.c_int), ("P", C.c_void_p), ("y", C.c_void_p),
                ("phi", C.c_double), ("psi", C.c_double), ("gap_abs", C.c_double),
                ("gap_rel", C.c_double), ("pinf", C.c_double), ("dinf", C.c_double),
                ("margin", C.c_double), ("margin_P", C.c_double), ("margin_D", C.c_double),
                ("iterations", C.c_int), ("phase1_used", C.c_int), ("phase1_iterations", C.c_int),
                ("t_star", C.c_double), ("time_solve_s", C.c_double), ("iters_lowprec", C.c_int),
                ("ir_steps", C.c_int), ("ir_eta_max", C.c_double),
                ("warm_used", C.c_int), ("warm_fallback", C.c_int), ("warm_iterations", C.c_int),
                ("logx", C.c_void_p), ("label_y", C.c_void_p), ("label_logx", C.c_void_p),
                ("label_iter", C.c_int),
                ("asm_path", C.c_int), ("solve_path", C.c_int),
                ("history", C.POINTER(IterRec)), ("history_cap", C.c_int), ("history_len", C.c_int),
                ("chol_shifts", C.c_int), ("graph_replays", C.c_int), ("phase1_reason", C.c_int),
                ("chol_panels", C.c_int), ("chol_subpanels", C.c_int),
                ("time_prepare_s", C.c_double), ("time_warm_s", C.c_double),
                ("time_paper_s", C.c_double), ("time_phase1_s", C.c_double), ("time_cert_s", C.c_double)]


class BisectRec(C.Structure):
    _fields_ = [("t", C.c_double), ("verdict", C.c_int), ("iterations", C.c_int), ("margin", C.c_double)]


class PsdpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


_lib = None

EXPORTS = ["psdp_setup_opts_default", "psdp_opts_default", "psdp_polya_setup", "psdp_polya_setup_batched",
           "psdp_query",
           "psdp_get_polya", "psdp_ipm_solve", "psdp_ipm_solve_batched", "psdp_ipm_solve_noalloc",
           "psdp_eval_newton", "psdp_eval_schur", "psdp_poly_on_simplex", "psdp_bisect_simplex",
           "psdp_eval_ladder", "psdp_basis", "psdp_free", "psdp_last_error", "psdp_version",
           "psdp_fp64_mfma_rate",
           "psdp_mlp_create", "psdp_mlp_param_count", "psdp_mlp_set_params", "psdp_mlp_get_params",
           "psdp_mlp_forward", "psdp_mlp_loss_grad", "psdp_mlp_adam", "psdp_mlp_free"]


def load(path: str = LIB_PATH):
    """Loads the HIP library; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1411_3769_amd.build`")
    # torch carries its own HIP runtime; it must take the device before this
    # library's runtime does, or torch finds no GPU afterwards
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()
    except ImportError:
        pass
    lib = C.CDLL(path)
    vp = C.c_void_p
    lib.psdp_setup_opts_default.argtypes = [C.POINTER(SetupOpts)]
    lib.psdp_setup_opts_default.restype = None
    lib.psdp_opts_default.argtypes = [C.POINTER(Opts)]
    lib.psdp_opts_default.restype = None
    lib.psdp_polya_setup.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int,
                                     C.POINTER(SetupOpts), C.POINTER(vp)]
    lib.psdp_polya_setup_batched.argtypes = [C.c_int, C.POINTER(vp), C.POINTER(C.c_int), C.POINTER(C.c_int),
                                             C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(SetupOpts),
                                             C.POINTER(vp)]
    lib.psdp_query.argtypes = [vp, C.POINTER(Dims)]
    lib.psdp_get_polya.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.psdp_ipm_solve.argtypes = [vp, C.POINTER(Opts), C.POINTER(CResult)]
    lib.psdp_ipm_solve_batched.argtypes = [C.POINTER(vp), C.c_int, C.POINTER(Opts), C.POINTER(CResult)]
    lib.psdp_ipm_solve_noalloc.argtypes = [vp, C.POINTER(Opts), C.POINTER(CResult)]
    lib.psdp_poly_on_simplex.argtypes = [C.c_int, C.c_int, C.c_int, vp, vp, C.c_int, vp, C.c_int, vp]
    lib.psdp_bisect_simplex.argtypes = [C.c_int, C.c_int, C.c_int, vp, vp, C.c_int, vp, vp, C.c_int, C.c_int,
                                        C.c_double, C.c_double, C.c_double, C.c_int, C.POINTER(SetupOpts),
                                        C.POINTER(Opts), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                        C.POINTER(BisectRec), C.c_int, C.POINTER(C.c_int)]
    lib.psdp_eval_newton.argtypes = [vp] * 10 + [C.c_int, C.c_int, vp]
    lib.psdp_eval_schur.argtypes = [vp, vp, vp, C.c_int, vp, vp]
    lib.psdp_eval_ladder.argtypes = [vp, vp, vp, C.POINTER(Opts), C.POINTER(C.c_double),
                                     C.POINTER(C.c_int)]
    lib.psdp_basis.argtypes = [vp, vp]
    lib.psdp_free.argtypes = [vp]
    lib.psdp_free.restype = None
    lib.psdp_last_error.restype = C.c_char_p
    lib.psdp_version.restype = C.c_char_p
    lib.psdp_fp64_mfma_rate.argtypes = [C.POINTER(C.c_double), vp]
    lib.psdp_mlp_create.argtypes = [vp, C.c_int, C.c_int, C.POINTER(vp)]
    lib.psdp_mlp_param_count.argtypes = [vp]
    lib.psdp_mlp_param_count.restype = C.c_int64
    lib.psdp_mlp_set_params.argtypes = [vp, vp]
    lib.psdp_mlp_get_params.argtypes = [vp, vp, vp]
    lib.psdp_mlp_forward.argtypes = [vp, vp, C.c_int, vp, vp]
    lib.psdp_mlp_loss_grad.argtypes = [vp, vp, vp, C.c_int, C.POINTER(C.c_double), vp]
    lib.psdp_mlp_adam.argtypes = [vp, C.c_float, C.c_float, C.c_float, C.c_float, vp]
    lib.psdp_mlp_free.argtypes = [vp]
    lib.psdp_mlp_free.restype = None
    for name in ("psdp_polya_setup", "psdp_query", "psdp_get_polya", "psdp_ipm_solve",
                 "psdp_ipm_solve_batched", "psdp_ipm_solve_noalloc", "psdp_poly_on_simplex", "psdp_eval_schur",
                 "psdp_bisect_simplex", "psdp_eval_newton", "psdp_eval_ladder", "psdp_basis",
                 "psdp_mlp_create", "psdp_mlp_set_params", "psdp_mlp_get_params", "psdp_mlp_forward",
                 "psdp_mlp_loss_grad", "psdp_mlp_adam"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _check(rc: int):
    if rc != 0:
        raise PsdpError(rc, load().psdp_last_error().decode())


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _current_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return None


class SDP:
    """Handle of one structured SDP (psdp_polya_setup)."""

    def __init__(self, handle: int, dims: Dims):
        self._h = C.c_void_p(handle)
        d = dims
        self.n, self.l, self.da, self.dp, self.d1, self.d2 = d.n, d.l, d.da, d.dp, d.d1, d.d2
        self.L0, self.L, self.M, self.Na, self.Nt = d.L0, d.L, d.M, d.Na, d.Nt
        self.K, self.Kpad, self.device_bytes = int(d.K), int(d.Kpad), int(d.device_bytes)
        self.form = "discrete" if d.form == 1 else "continuous"
        self.bo = d.bo          # order of every block of the SDP

    @property
    def nb(self):
        return self.L + self.M

    @property
    def handle(self):
        return self._h

    def get_polya(self):
        beta = np.zeros((self.L0, self.L), np.int64)
        coef = np.zeros((self.L0, self.M, self.Na), np.int64)
        H = np.zeros((self.M, self.L0, self.n, self.n))
        scale = np.zeros(self.nb)
        cdiag = np.zeros(self.nb)
        _check(load().psdp_get_polya(self._h, _ptr(beta), _ptr(coef), _ptr(H), _ptr(scale), _ptr(cdiag)))
        return dict(beta=beta, coef=coef, H=H, scale=scale, cdiag=cdiag)

    def basis(self) -> np.ndarray:
        pairs = np.zeros((self.Nt, 2), np.int32)
        _check(load().psdp_basis(self._h, _ptr(pairs)))
        return pairs

    def close(self):
        if self._h is not None and self._h.value:
            load().psdp_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


FORMS = {"continuous": 0, "discrete": 1}


def polya_setup(A, n: int, l: int, dp: int, d: int, *, da: int = 1, d1: Optional[int] = None,
                d2: Optional[int] = None, delta: float = 1e-3, eps: float = 1e-3,
                paper_literal: bool = False, form: str = "continuous") -> SDP:
    """psdp_polya_setup.  A: [Na][n][n] FP64 host array, or a torch CUDA tensor
    (then read on the device).  form: "continuous" (x' = A x) or "discrete"
    (x+ = A x)."""
    lib = load()
    o = SetupOpts()
    lib.psdp_setup_opts_default(C.byref(o))
    o.da = da
    o.form = FORMS[form]
    o.d1 = -1 if d1 is None else d1
    o.d2 = -1 if d2 is None else d2
    o.delta, o.eps, o.paper_literal = delta, eps, int(paper_literal)
    keep = None
    if hasattr(A, "is_cuda") and A.is_cuda:
        import torch
        keep = A.to(torch.float64).contiguous()
        o.a_on_device = 1
        aptr = C.c_void_p(keep.data_ptr())
    else:
        keep = np.ascontiguousarray(A, dtype=np.float64)
        aptr = _ptr(keep)
    h = C.c_void_p()
    _check(lib.psdp_polya_setup(aptr, n, l, dp, d, C.byref(o), C.byref(h)))
    dims = Dims()
    _check(lib.psdp_query(h, C.byref(dims)))
    return SDP(h.value, dims)


def polya_setup_batched(systems, *, da: int = 1, delta: float = 1e-3, eps: float = 1e-3,
                        paper_literal: bool = False, form: str = "continuous") -> list:
    """psdp_polya_setup_batched.  systems: sequence of (A, n, l, dp, d), every A
    a host array or every A a torch CUDA tensor.  Returns one SDP per system."""
    lib = load()
    systems = list(systems)
    cnt = len(systems)
    o = SetupOpts()
    lib.psdp_setup_opts_default(C.byref(o))
    o.da = da
    o.form = FORMS[form]
    o.delta, o.eps, o.paper_literal = delta, eps, int(paper_literal)
    keep, ptrs = [], (C.c_void_p * max(cnt, 1))()
    dev = [hasattr(s[0], "is_cuda") and s[0].is_cuda for s in systems]
    if any(dev) and not all(dev):
        raise ValueError("polya_setup_batched: vertices must be all on the host or all on the device")
    o.a_on_device = int(bool(dev) and all(dev))
    if o.a_on_device:
        import torch
    for i, (A, *_rest) in enumerate(systems):
        if o.a_on_device:
            t = A if A.dtype == torch.float64 and A.is_contiguous() else A.to(torch.float64).contiguous()
            keep.append(t)
            ptrs[i] = t.data_ptr()
        else:
            a = np.ascontiguousarray(A, dtype=np.float64)
            keep.append(a)
            ptrs[i] = a.ctypes.data
    ints = [(C.c_int * max(cnt, 1))(*[int(s[k]) for s in systems]) for k in (1, 2, 3, 4)]
    out = (C.c_void_p * max(cnt, 1))()
    _check(lib.psdp_polya_setup_batched(cnt, ptrs, ints[0], ints[1], ints[2], ints[3], C.byref(o), out))
    # the sizes depend only on the shape (the options are common to the call)
    res, dims_of = [], {}
    for i, sy in enumerate(systems):
        key = tuple(int(v) for v in sy[1:5])
        dims = dims_of.get(key)
        if dims is None:
            dims = Dims()
            _check(lib.psdp_query(out[i], C.byref(dims)))
            dims_of[key] = dims
        res.append(SDP(out[i], dims))
    return res


def make_opts(**kw) -> Opts:
    lib = load()
    o = Opts()
    lib.psdp_opts_default(C.byref(o))
    for k, v in kw.items():
        if k == "verdict_mode" and isinstance(v, str):
            v = VERDICT_MODES[v]
        if k == "precision" and isinstance(v, str):
            v = PRECISIONS[v]
        if k == "stop_rule" and isinstance(v, str):
            v = STOP_RULES[v]
        if k == "sigma_rule" and isinstance(v, str):
            v = SIGMA_RULES[v]
        if k == "stream":
            v = C.c_void_p(v) if isinstance(v, int) else v
        if k == "prof":
            v = v.ctypes.data_as(DP) if v is not None else DP()
        setattr(o, k, v)
    if "stream" not in kw:
        o.stream = _current_stream()
    return o


@dataclass
class Result:
    verdict: int
    reason: int
    P: np.ndarray
    y: np.ndarray
    phi: float
    psi: float
    gap_abs: float
    gap_rel: float
    pinf: float
    dinf: float
    margin: float
    margin_P: float
    margin_D: float
    iterations: int
    phase1_used: bool
    phase1_iterations: int
    t_star: float
    time_solve_s: float
    iters_lowprec: int = 0
    ir_steps: int = 0
    ir_eta_max: float = float("nan")
    warm_used: bool = False
    warm_fallback: bool = False
    warm_iterations: int = 0
    logx: np.ndarray = None
    label_y: np.ndarray = None
    label_logx: np.ndarray = None
    label_iter: int = -1
    asm_path: int = -1
    solve_path: int = -1
    history: list = field(default_factory=list)
    chol_shifts: int = 0
    graph_replays: int = 0
    phase1_reason: int = -1
    chol_panels: int = 0
    chol_subpanels: int = 0
    phase_times: dict = field(default_factory=dict)   # wall seconds per phase of the call

    @property
    def verdict_name(self):
        return VERDICTS[self.verdict]

    @property
    def reason_name(self):
        return REASONS[self.reason] if 0 <= self.reason < len(REASONS) else str(self.reason)


def _prep_batch(sdps, cap: int, arr):
    """Caller buffers of every system's result in one host allocation; the
    entries of arr (CResult) point into it.  Returns per system (P, y,
    (logx, label_y, label_logx), history)."""
    sizes = [(s.L0 * s.n * s.n, s.K, s.L + s.M) for s in sdps]
    total = sum(p + 2 * k + 2 * b for p, k, b in sizes)
    buf = np.zeros(max(total, 1))
    base, item = buf.ctypes.data, buf.itemsize
    out, o = [], 0
    for i, (s, (p, k, b)) in enumerate(zip(sdps, sizes)):
        offs = (o, o + p, o + p + k, o + p + k + b, o + p + 2 * k + b)
        o += p + 2 * k + 2 * b
        P = buf[offs[0]:offs[1]].reshape(s.L0, s.n, s.n)
        y, lx = buf[offs[1]:offs[2]], buf[offs[2]:offs[3]]
        ly, llx = buf[offs[3]:offs[4]], buf[offs[4]:o]
        r = arr[i]
        r.P, r.y, r.logx, r.label_y, r.label_logx = (base + item * q for q in offs)
        hist = None
        if cap:
            hist = (IterRec * cap)()
            r.history = C.cast(hist, C.POINTER(IterRec))
        r.history_cap = cap
        out.append((P, y, (lx, ly, llx), hist))
    return out


def _warm_arrays(sdps, warm_y, warm_logx):
    """Host pointer arrays for the warm start (entries may be None)."""
    keep, ptrs = [], []
    for vals, size in ((warm_y, lambda s: s.K), (warm_logx, lambda s: s.L + s.M)):
        if vals is None:
            ptrs.append(C.POINTER(DP)())
            continue
        if len(vals) != len(sdps):
            raise ValueError("one warm-start entry per system")
        arr = (DP * len(sdps))()
        for i, (v, s) in enumerate(zip(vals, sdps)):
            if v is None:
                continue
            v = np.ascontiguousarray(v, dtype=np.float64)
            if v.shape != (size(s),):
                raise ValueError(f"warm-start entry {i} has shape {v.shape}, wants ({size(s)},)")
            keep.append(v)
            arr[i] = v.ctypes.data_as(DP)
        keep.append(arr)
        ptrs.append(C.cast(arr, C.POINTER(DP)))
    return ptrs, keep


def _unpack(r: CResult, P, y, lx, hist) -> Result:
    h = []
    if hist is not None:
        for i in range(r.history_len):
            e = hist[i]
            h.append(dict(iter=e.iter, phi=e.phi, psi=e.psi, gap_rel=e.gap_rel, pinf=e.pinf,
                          dinf=e.dinf, mu=e.mu, tp=e.tp, td=e.td))
    return Result(r.verdict, r.reason, P, y, r.phi, r.psi, r.gap_abs, r.gap_rel, r.pinf, r.dinf,
                  r.margin, r.margin_P, r.margin_D, r.iterations, bool(r.phase1_used),
                  r.phase1_iterations, r.t_star, r.time_solve_s, r.iters_lowprec,
                  r.ir_steps, r.ir_eta_max, bool(r.warm_used), bool(r.warm_fallback),
                  r.warm_iterations, lx[0], lx[1] if r.label_iter >= 0 else None,
                  lx[2] if r.label_iter >= 0 else None, r.label_iter, r.asm_path, r.solve_path, h,
                  r.chol_shifts, r.graph_replays, r.phase1_reason, r.chol_panels, r.chol_subpanels,
                  {"prepare": r.time_prepare_s, "warm": r.time_warm_s, "paper": r.time_paper_s,
                   "phase1": r.time_phase1_s, "cert": r.time_cert_s})


def ipm_solve(sdp: SDP, warm_y=None, warm_logx=None, **opts) -> Result:
    """Alg. 2 for one SDP.  warm_y (K values in the library's dual order) and
    warm_logx (L+M log block scales of X) give an optional warm start."""
    o = make_opts(**opts)
    cap = 512 if o.record_history else 0
    arr = (CResult * 1)()
    (P, y, lx, hist), = _prep_batch([sdp], cap, arr)
    (wy, wl), wkeep = _warm_arrays([sdp], None if warm_y is None else [warm_y],
                                   None if warm_logx is None else [warm_logx])
    o.warm_y, o.warm_logx = wy, wl
    _check(load().psdp_ipm_solve(sdp.handle, C.byref(o), arr))
    del wkeep
    return _unpack(arr[0], P, y, lx, hist)


def ipm_solve_noalloc(sdp: SDP, **opts) -> Result:
    """psdp_ipm_solve_noalloc: Alg. 2 for one SDP with every device buffer in
    the library's static scratch (no device allocation; eager launches on the
    caller's stream)."""
    o = make_opts(**opts)
    cap = 512 if o.record_history else 0
    arr = (CResult * 1)()
    (P, y, lx, hist), = _prep_batch([sdp], cap, arr)
    _check(load().psdp_ipm_solve_noalloc(sdp.handle, C.byref(o), arr))
    return _unpack(arr[0], P, y, lx, hist)


def ipm_solve_batched(sdps: Sequence[SDP], warm_y=None, warm_logx=None, **opts) -> List[Result]:
    o = make_opts(**opts)
    cap = 512 if o.record_history else 0
    n = len(sdps)
    arr = (CResult * n)()
    keep = _prep_batch(sdps, cap, arr)
    (wy, wl), wkeep = _warm_arrays(sdps, warm_y, warm_logx)
    o.warm_y, o.warm_logx = wy, wl
    hs = (C.c_void_p * n)(*[s.handle.value for s in sdps])
    _check(load().psdp_ipm_solve_batched(hs, n, C.byref(o), arr))
    del wkeep
    return [_unpack(arr[i], *keep[i]) for i in range(n)]


def eval_newton(sdp: SDP, X: np.ndarray, Z: np.ndarray, y: np.ndarray, chol_panels=0,
                chol_subpanels=0, stream=None, schur=True) -> dict:
    """psdp_eval_newton; schur=False leaves out the K x K matrices Lam and LamL
    (NULL in the call)."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    nb, n, K = sdp.nb, sdp.bo, sdp.K
    out = dict(Zi=np.zeros((nb, n, n)), BTy=np.zeros((nb, n, n)), BX=np.zeros(K), sol=np.zeros(K))
    if schur:
        out["Lam"], out["LamL"] = np.zeros((K, K)), np.zeros((K, K))
    st = stream if stream is not None else _current_stream()
    _check(load().psdp_eval_newton(sdp.handle, _ptr(X), _ptr(Z), _ptr(y), _ptr(out["Zi"]),
                                   _ptr(out["BTy"]), _ptr(out["BX"]),
                                   _ptr(out["Lam"]) if schur else None,
                                   _ptr(out["LamL"]) if schur else None, _ptr(out["sol"]),
                                   int(chol_panels), int(chol_subpanels), st))
    return out


def eval_schur(sdp: SDP, X: np.ndarray, Z: np.ndarray, precision="fp64", stream=None) -> np.ndarray:
    """psdp_eval_schur: the Schur complement [K][K] at (X, Z) in a precision form."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    out = np.zeros((sdp.K, sdp.K))
    st = stream if stream is not None else _current_stream()
    _check(load().psdp_eval_schur(sdp.handle, _ptr(X), _ptr(Z), prec, _ptr(out), st))
    return out


def eval_ladder(sdp: SDP, V: np.ndarray, dV: np.ndarray, **opts):
    V = np.ascontiguousarray(V, dtype=np.float64)
    dV = np.ascontiguousarray(dV, dtype=np.float64)
    o = make_opts(**opts)
    step = C.c_double()
    k = C.c_int()
    _check(load().psdp_eval_ladder(sdp.handle, _ptr(V), _ptr(dV), C.byref(o), C.byref(step), C.byref(k)))
    return step.value, k.value


def _terms(exps, mats):
    exps = np.ascontiguousarray(exps, dtype=np.int32)
    mats = np.ascontiguousarray(mats, dtype=np.float64)
    if exps.ndim != 2 or mats.ndim != 3 or mats.shape[0] != exps.shape[0] or mats.shape[1] != mats.shape[2]:
        raise ValueError("exps [count][lx] and mats [count][n][n] expected")
    return exps, mats


def poly_on_simplex(exps, mats, G, l: int, da: int) -> np.ndarray:
    """psdp_poly_on_simplex: coefficients [f(l, da)][n][n] of the homogeneous
    B(alpha) equal to A(G alpha) on the simplex (G = None: identity)."""
    from math import comb
    exps, mats = _terms(exps, mats)
    count, lx = exps.shape
    n = mats.shape[1]
    Gm = None if G is None else np.ascontiguousarray(G, dtype=np.float64)
    if Gm is not None and Gm.shape != (lx, l):
        raise ValueError(f"G must be [{lx}][{l}]")
    out = np.zeros((comb(l + da - 1, l - 1), n, n))
    _check(load().psdp_poly_on_simplex(n, lx, count, _ptr(exps), _ptr(mats), l, _ptr(Gm), da, _ptr(out)))
    return out


@dataclass
class BisectResult:
    t_cert: float
    t_other: float
    trials: list


def bisect_simplex(exps, mats, G0, G1, l: int, dp: int, d: int, t_feas: float, t_infeas: float,
                   tol: float, width: int = 1, delta: float = 1e-3, eps: float = 1e-3, **opts) -> BisectResult:
    """psdp_bisect_simplex: certified end of the bracket over regions
    x = (G0 + t G1) alpha; trials as (t, verdict, iterations, margin)."""
    exps, mats = _terms(exps, mats)
    count, lx = exps.shape
    n = mats.shape[1]
    G0 = np.ascontiguousarray(G0, dtype=np.float64)
    G1 = np.ascontiguousarray(G1, dtype=np.float64)
    lib = load()
    so = SetupOpts()
    lib.psdp_setup_opts_default(C.byref(so))
    so.delta, so.eps = delta, eps
    o = make_opts(**opts)
    cap = 1024
    recs = (BisectRec * cap)()
    tc, to, nr = C.c_double(), C.c_double(), C.c_int()
    _check(lib.psdp_bisect_simplex(n, lx, count, _ptr(exps), _ptr(mats), l, _ptr(G0), _ptr(G1), dp, d,
                                   t_feas, t_infeas, tol, width, C.byref(so), C.byref(o), C.byref(tc),
                                   C.byref(to), recs, cap, C.byref(nr)))
    trials = [(recs[i].t, recs[i].verdict, recs[i].iterations, recs[i].margin) for i in range(nr.value)]
    return BisectResult(tc.value, to.value, trials)


def version() -> str:
    return load().psdp_version().decode()


def fp64_mfma_rate(stream=None) -> float:
    """psdp_fp64_mfma_rate: attainable FP64 matrix-core TFLOP/s of the device."""
    v = C.c_double(0.0)
    _check(load().psdp_fp64_mfma_rate(C.byref(v), stream if stream is not None else _current_stream()))
    return v.value


class MLP:
    """The warm-start network on the device (psdp_mlp_*).  Inputs and
    targets are CUDA float32 tensors [batch x width]."""

    def __init__(self, dims, precision="bf16", max_batch=256):
        self.dims = tuple(int(d) for d in dims)
        self.max_batch = int(max_batch)
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        h = C.c_void_p()
        d = (C.c_int * 4)(*self.dims)
        _check(load().psdp_mlp_create(C.cast(d, C.c_void_p), prec, self.max_batch, C.byref(h)))
        self._h = h
        self.nparam = int(load().psdp_mlp_param_count(h))

    def set_params(self, flat: np.ndarray):
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        if flat.shape != (self.nparam,):
            raise ValueError(f"expected {self.nparam} parameters, got {flat.shape}")
        _check(load().psdp_mlp_set_params(self._h, _ptr(flat)))

    def get_params(self) -> np.ndarray:
        out = np.empty(self.nparam, np.float32)
        _check(load().psdp_mlp_get_params(self._h, _ptr(out), None))
        return out

    def get_grad(self) -> np.ndarray:
        out = np.empty(self.nparam, np.float32)
        _check(load().psdp_mlp_get_params(self._h, None, _ptr(out)))
        return out

    @staticmethod
    def _dev(t, width):
        import torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32):
            raise TypeError("expected a CUDA float32 tensor")
        if t.dim() != 2 or t.shape[1] != width or not t.is_contiguous():
            raise ValueError(f"expected a contiguous [batch x {width}] tensor")
        return C.c_void_p(t.data_ptr())

    def forward(self, x):
        import torch
        out = torch.empty((x.shape[0], self.dims[3]), device=x.device, dtype=torch.float32)
        _check(load().psdp_mlp_forward(self._h, self._dev(x, self.dims[0]), int(x.shape[0]),
                                       C.c_void_p(out.data_ptr()), _current_stream()))
        return out

    def loss_grad(self, x, t) -> float:
        loss = C.c_double()
        _check(load().psdp_mlp_loss_grad(self._h, self._dev(x, self.dims[0]), self._dev(t, self.dims[3]),
                                         int(x.shape[0]), C.byref(loss), _current_stream()))
        return loss.value

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        _check(load().psdp_mlp_adam(self._h, lr, b1, b2, eps, _current_stream()))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().psdp_mlp_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

