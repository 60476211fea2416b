"""ctypes binding of libwdirac.so (the C ABI in include/wdirac.h).

Argument marshalling only: torch tensors provide device memory and the current HIP stream;
every step of the computation runs in the library's HIP kernels. The binding fails loudly when
the library is missing; there is no CPU fallback.

Functions keep the C names: wd_gauge_create, wd_gauge_destroy, wd_apply, wd_apply_dag,
bicgstab_solve, bicgstab_m_solve, wd_multimass_solve, wd_batch_solve, wd_gauge_grad.
Fields are complex128 CUDA tensors: fermions [T, Z, Y, X, 3, 4], links [4, T, Z, Y, X, 3, 3].
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "libwdirac.so")

WD_OK, WD_ERR_ARG, WD_ERR_HIP, WD_ERR_OOM, WD_ERR_NOCONV, WD_ERR_BREAKDOWN, WD_ERR_NAN, WD_ERR_UNSUPPORTED = range(8)
WD_F64, WD_F32, WD_F16, WD_BF16 = range(4)
WD_METHOD_SEQUENTIAL, WD_METHOD_MULTISHIFT, WD_METHOD_BATCHED = 0, 1, 2
WD_GUESS_NONE, WD_GUESS_POLY, WD_GUESS_MINRES = 0, 1, 2
WD_MIXED_RELIABLE, WD_MIXED_DEFECT = 0, 1
PREC = {"f64": WD_F64, "f32": WD_F32, "f16": WD_F16, "bf16": WD_BF16}


class Geom(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int * 4), ("antiperiodic_t", ctypes.c_int)]


class SolverParams(ctypes.Structure):
    _fields_ = [
        ("tol", ctypes.c_double),
        ("max_iter", ctypes.c_int),
        ("mixed", ctypes.c_int),
        ("spinor_store", ctypes.c_int),
        ("link_store", ctypes.c_int),
        ("recon", ctypes.c_int),
        ("eo", ctypes.c_int),
        ("delta_reliable", ctypes.c_double),
        ("use_x0", ctypes.c_int),
        ("dagger", ctypes.c_int),
        ("mixed_mode", ctypes.c_int),
        ("guess_order", ctypes.c_int),
        ("temporal_gauge", ctypes.c_int),
        ("gamma_basis", ctypes.c_int),
    ]


class SolverStats(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int),
        ("reliable_updates", ctypes.c_int),
        ("status", ctypes.c_int),
        ("true_rel_res", ctypes.c_double),
        ("seconds", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class OpVariant(ctypes.Structure):
    _fields_ = [
        ("red", ctypes.c_int),
        ("stage", ctypes.c_int),
        ("nontemporal", ctypes.c_int),
        ("tile", ctypes.c_int),
        ("copies", ctypes.c_int),
        ("rhs_per_thread", ctypes.c_int),
        ("dagger", ctypes.c_int),
    ]


WD_RED_NONE, WD_RED_ZDOT, WD_RED_OUTX, WD_RED_NORM = range(4)
RED = {"none": WD_RED_NONE, "zdot": WD_RED_ZDOT, "outx": WD_RED_OUTX, "norm": WD_RED_NORM}


class System(ctypes.Structure):
    _fields_ = [("gauge", ctypes.c_void_p), ("kappa", ctypes.c_double), ("b", ctypes.c_void_p),
                ("x", ctypes.c_void_p)]


EXPORTED = [
    "wd_params_default", "wd_gauge_create", "wd_gauge_destroy", "wd_apply", "wd_apply_dag", "bicgstab_solve",
    "bicgstab_m_solve", "wd_multimass_solve", "wd_batch_solve", "wd_normal_solve", "wd_gauge_grad",
    "wd_status_str", "wd_last_error", "wd_timing_enable", "wd_timing_reset", "wd_timing_get", "wd_gauge_device_bytes",
    "wd_set_graphs", "wd_op_variant_default", "wd_apply_prec", "wd_apply_noalloc",
]

_lib = None


class WdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{status_name(code)}: {msg}")
        self.code = code


def load(path: str = LIBPATH):
    """Load libwdirac.so (no compute); raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build() (hipcc, gfx950)")
    L = ctypes.CDLL(path)
    vp, d, i = ctypes.c_void_p, ctypes.c_double, ctypes.c_int
    L.wd_params_default.argtypes = [ctypes.POINTER(SolverParams)]
    L.wd_params_default.restype = None
    L.wd_gauge_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Geom), vp, ctypes.POINTER(SolverParams), vp]
    L.wd_gauge_destroy.argtypes = [vp]
    for f in (L.wd_apply, L.wd_apply_dag):
        f.argtypes = [vp, d, vp, vp, vp]
    L.wd_apply_noalloc.argtypes = [vp, d, vp, vp, i, vp]
    L.bicgstab_solve.argtypes = [vp, d, vp, vp, ctypes.POINTER(SolverParams), ctypes.POINTER(SolverStats), vp]
    L.bicgstab_m_solve.argtypes = [vp, i, ctypes.POINTER(d), ctypes.POINTER(vp), vp, ctypes.POINTER(SolverParams),
                                   ctypes.POINTER(SolverStats), vp]
    L.wd_multimass_solve.argtypes = [vp, i, ctypes.POINTER(d), ctypes.POINTER(vp), vp, i, i,
                                     ctypes.POINTER(SolverParams), ctypes.POINTER(SolverStats), vp]
    L.wd_batch_solve.argtypes = [i, ctypes.POINTER(System), ctypes.POINTER(SolverParams),
                                 ctypes.POINTER(SolverStats), vp]
    L.wd_normal_solve.argtypes = [vp, d, i, ctypes.POINTER(d), ctypes.POINTER(vp), vp, i, i,
                                  ctypes.POINTER(SolverParams), ctypes.POINTER(SolverStats), vp]
    L.wd_gauge_grad.argtypes = [vp, vp, vp, vp, i, vp]
    L.wd_op_variant_default.argtypes = [ctypes.POINTER(OpVariant)]
    L.wd_op_variant_default.restype = None
    L.wd_apply_prec.argtypes = [vp, d, vp, vp, ctypes.POINTER(SolverParams), ctypes.POINTER(OpVariant),
                                ctypes.POINTER(d), vp]
    L.wd_status_str.argtypes = [i]
    L.wd_status_str.restype = ctypes.c_char_p
    L.wd_last_error.argtypes = [ctypes.c_char_p, ctypes.c_size_t]
    L.wd_timing_enable.argtypes = [i]
    L.wd_timing_enable.restype = None
    L.wd_timing_reset.argtypes = []
    L.wd_timing_reset.restype = None
    L.wd_timing_get.argtypes = [i, ctypes.POINTER(d), ctypes.POINTER(ctypes.c_long), ctypes.POINTER(d)]
    L.wd_set_graphs.argtypes = [i]
    L.wd_set_graphs.restype = None
    L.wd_gauge_device_bytes.argtypes = [vp]
    L.wd_gauge_device_bytes.restype = ctypes.c_size_t
    for name in ("wd_gauge_create", "wd_gauge_destroy", "wd_apply", "wd_apply_dag", "bicgstab_solve",
                 "bicgstab_m_solve", "wd_multimass_solve", "wd_batch_solve", "wd_normal_solve", "wd_gauge_grad",
                 "wd_last_error", "wd_timing_get", "wd_apply_prec", "wd_apply_noalloc"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def status_name(code: int) -> str:
    try:
        return load().wd_status_str(int(code)).decode()
    except Exception:
        return f"status {code}"


def last_error() -> str:
    buf = ctypes.create_string_buffer(1024)
    load().wd_last_error(buf, 1024)
    return buf.value.decode()


def _check(code: int, allow=(WD_OK,)):
    if code not in allow:
        raise WdError(code, last_error())
    return code


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor, name: str, shape=None):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous complex128 CUDA tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


def params(tol=1e-8, max_iter=5000, mixed=True, spinor="f32", links="f16", recon=12, eo=True, delta=0.1,
           use_x0=False, dagger=False, defect_correction=False, guess_order=0,
           temporal_gauge=False, nonchiral=False) -> SolverParams:
    p = SolverParams()
    load().wd_params_default(ctypes.byref(p))
    p.tol, p.max_iter, p.mixed = float(tol), int(max_iter), int(bool(mixed))
    p.spinor_store, p.link_store, p.recon = PREC[spinor], PREC[links], int(recon)
    p.eo, p.delta_reliable, p.use_x0, p.dagger = int(bool(eo)), float(delta), int(bool(use_x0)), int(bool(dagger))
    p.mixed_mode = WD_MIXED_DEFECT if defect_correction else WD_MIXED_RELIABLE
    p.guess_order = int(guess_order)
    p.temporal_gauge = int(bool(temporal_gauge))
    p.gamma_basis = int(bool(nonchiral))
    return p


@dataclass
class Gauge:
    """A wd_gauge handle: one lattice with its links, packed into the library's layout."""

    handle: ctypes.c_void_p
    dims: tuple
    antiperiodic: bool

    @property
    def field_shape(self):
        X, Y, Z, T = self.dims
        return (T, Z, Y, X, 3, 4)

    @property
    def link_shape(self):
        X, Y, Z, T = self.dims
        return (4, T, Z, Y, X, 3, 3)

    def close(self):
        if self.handle:
            load().wd_gauge_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def device_bytes(self) -> int:
        return int(load().wd_gauge_device_bytes(self.handle))


def wd_gauge_create(U: torch.Tensor, antiperiodic: bool = True, hint: SolverParams | None = None) -> Gauge:
    if U.ndim != 7 or U.shape[0] != 4 or tuple(U.shape[-2:]) != (3, 3):
        raise ValueError("U must have shape [4, T, Z, Y, X, 3, 3]")
    T, Z, Y, X = (int(v) for v in U.shape[1:5])
    g = Geom()
    g.dims[:] = [X, Y, Z, T]
    g.antiperiodic_t = int(bool(antiperiodic))
    h = ctypes.c_void_p()
    _check(load().wd_gauge_create(ctypes.byref(h), ctypes.byref(g), _ptr(U, "U"),
                                  ctypes.byref(hint) if hint is not None else None, _stream()))
    return Gauge(h, (X, Y, Z, T), bool(antiperiodic))


def wd_gauge_destroy(g: Gauge) -> None:
    g.close()


def wd_apply(g: Gauge, kappa: float, psi: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    out = torch.empty_like(psi) if out is None else out
    _check(load().wd_apply(g.handle, float(kappa), _ptr(out, "out", g.field_shape), _ptr(psi, "in", g.field_shape),
                           _stream()))
    return out


def wd_apply_dag(g: Gauge, kappa: float, psi: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    out = torch.empty_like(psi) if out is None else out
    _check(load().wd_apply_dag(g.handle, float(kappa), _ptr(out, "out", g.field_shape),
                               _ptr(psi, "in", g.field_shape), _stream()))
    return out


def op_variant(red="none", stage=-1, nontemporal=-1, tile=-1, copies=1, rhs_per_thread=-1,
               dagger=False) -> OpVariant:
    v = OpVariant()
    load().wd_op_variant_default(ctypes.byref(v))
    v.red = RED[red] if isinstance(red, str) else int(red)
    v.stage, v.nontemporal, v.tile = int(stage), int(nontemporal), int(tile)
    v.copies, v.rhs_per_thread, v.dagger = int(copies), int(rhs_per_thread), int(bool(dagger))
    return v


def wd_apply_prec(g: Gauge, kappa: float, psi: torch.Tensor, p: SolverParams | None = None,
                  v: OpVariant | None = None, out: torch.Tensor | None = None):
    """The solvers' even-odd operator in their storage formats: returns (out, dots) with
    out_e = M_prec in_e, out_o = D_oe in_e (adjoint hops with v.dagger). psi: one field
    [T, Z, Y, X, 3, 4], or [copies, T, Z, Y, X, 3, 4] for v.copies systems in one launch.
    dots: numpy array [copies, 3] of the fused sums of v.red."""
    import numpy as np

    p = params() if p is None else p
    v = op_variant() if v is None else v
    shape = tuple(psi.shape)
    want = (v.copies, *g.field_shape) if v.copies > 1 or len(shape) == 7 else g.field_shape
    out = torch.empty_like(psi) if out is None else out
    _ptr(psi, "in", want)
    _ptr(out, "out", want)
    dots = (ctypes.c_double * (3 * v.copies))()
    _check(load().wd_apply_prec(g.handle, float(kappa), _ptr(out, "out"), _ptr(psi, "in"), ctypes.byref(p),
                                ctypes.byref(v), dots, _stream()))
    return out, np.array(dots[:], dtype=np.float64).reshape(v.copies, 3)


def wd_apply_noalloc(g: Gauge, kappa: float, psi: torch.Tensor, out: torch.Tensor, dagger: bool = False) -> torch.Tensor:
    """out = M(kappa) psi (or M^dag psi) with no device allocation by the library; out must be
    given (a caller that cannot allocate owns it)."""
    _check(load().wd_apply_noalloc(g.handle, float(kappa), _ptr(out, "out", g.field_shape),
                                   _ptr(psi, "in", g.field_shape), int(bool(dagger)), _stream()))
    return out


NONFATAL = (WD_OK, WD_ERR_NOCONV, WD_ERR_BREAKDOWN, WD_ERR_NAN)


def bicgstab_solve(g: Gauge, kappa: float, b: torch.Tensor, x: torch.Tensor | None = None,
                   p: SolverParams | None = None, raise_on_fail: bool = True):
    """Solve M(kappa) x = b; returns (x, stats dict). With p.use_x0, x holds the start vector."""
    p = params() if p is None else p
    x = torch.zeros_like(b) if x is None else x
    st = SolverStats()
    code = load().bicgstab_solve(g.handle, float(kappa), _ptr(x, "x", g.field_shape), _ptr(b, "b", g.field_shape),
                                 ctypes.byref(p), ctypes.byref(st), _stream())
    _check(code, (WD_OK,) if raise_on_fail else NONFATAL)
    return x, st.as_dict()


def _xs(g, xs, n, like):
    if xs is None:
        xs = [torch.zeros_like(like) for _ in range(n)]
    arr = (ctypes.c_void_p * n)(*[_ptr(t, "x[i]", g.field_shape).value for t in xs])
    return xs, arr


def bicgstab_m_solve(g: Gauge, kappas, b: torch.Tensor, xs=None, p: SolverParams | None = None,
                     raise_on_fail: bool = True):
    """BiCGstab-M for all kappas at once; returns (list of x, list of stats dicts)."""
    p = params(mixed=False, eo=False) if p is None else p
    n = len(kappas)
    k = (ctypes.c_double * n)(*[float(v) for v in kappas])
    xs, arr = _xs(g, xs, n, b)
    st = (SolverStats * n)()
    code = load().bicgstab_m_solve(g.handle, n, k, arr, _ptr(b, "b", g.field_shape), ctypes.byref(p), st, _stream())
    _check(code, (WD_OK,) if raise_on_fail else NONFATAL)
    return xs, [s.as_dict() for s in st]


def wd_multimass_solve(g: Gauge, kappas, b: torch.Tensor, method: int = WD_METHOD_SEQUENTIAL,
                       guess: int = WD_GUESS_POLY, xs=None, p: SolverParams | None = None,
                       raise_on_fail: bool = True):
    p = params() if p is None else p
    n = len(kappas)
    k = (ctypes.c_double * n)(*[float(v) for v in kappas])
    xs, arr = _xs(g, xs, n, b)
    st = (SolverStats * n)()
    code = load().wd_multimass_solve(g.handle, n, k, arr, _ptr(b, "b", g.field_shape), int(method), int(guess),
                                     ctypes.byref(p), st, _stream())
    _check(code, (WD_OK,) if raise_on_fail else NONFATAL)
    return xs, [s.as_dict() for s in st]


def wd_batch_solve(systems, p: SolverParams | None = None, raise_on_fail: bool = True):
    """systems: list of (Gauge, kappa, b, x); all iterate together. Returns the list of stats dicts."""
    p = params() if p is None else p
    n = len(systems)
    arr = (System * n)()
    for i, (g, kappa, b, x) in enumerate(systems):
        arr[i].gauge = g.handle
        arr[i].kappa = float(kappa)
        arr[i].b = _ptr(b, "b", g.field_shape).value
        arr[i].x = _ptr(x, "x", g.field_shape).value
    st = (SolverStats * n)()
    code = load().wd_batch_solve(n, arr, ctypes.byref(p), st, _stream())
    _check(code, (WD_OK,) if raise_on_fail else NONFATAL)
    return [s.as_dict() for s in st]


def wd_normal_solve(g: Gauge, kappa: float, sigmas, b: torch.Tensor, method: int = WD_METHOD_SEQUENTIAL,
                    guess: int = WD_GUESS_POLY, xs=None, p: SolverParams | None = None,
                    raise_on_fail: bool = True):
    """(M_prec^dag M_prec + sigma_i) x_i = b_e on the even sites (odd sites of b ignored, of x_i
    zero): CG per shift (sequential or batched) or CG-M (method WD_METHOD_MULTISHIFT)."""
    p = params() if p is None else p
    n = len(sigmas)
    s = (ctypes.c_double * n)(*[float(v) for v in sigmas])
    xs, arr = _xs(g, xs, n, b)
    st = (SolverStats * n)()
    code = load().wd_normal_solve(g.handle, float(kappa), n, s, arr, _ptr(b, "b", g.field_shape), int(method),
                                  int(guess), ctypes.byref(p), st, _stream())
    _check(code, (WD_OK,) if raise_on_fail else NONFATAL)
    return xs, [q.as_dict() for q in st]


def wd_gauge_grad(g: Gauge, x: torch.Tensor, lam: torch.Tensor, project: bool = False,
                  out: torch.Tensor | None = None) -> torch.Tensor:
    out = torch.empty(g.link_shape, dtype=torch.complex128, device=x.device) if out is None else out
    _check(load().wd_gauge_grad(g.handle, _ptr(x, "x", g.field_shape), _ptr(lam, "lam", g.field_shape),
                                _ptr(out, "dU", g.link_shape), int(bool(project)), _stream()))
    return out


def set_graphs(on: bool = True):
    """Replay solver iteration chunks from captured HIP graphs, or launch eagerly (default)."""
    load().wd_set_graphs(int(bool(on)))


def timing_enable(on: bool = True):
    load().wd_timing_enable(int(bool(on)))


def timing_reset():
    load().wd_timing_reset()


def timing_get(cls: int):
    ms, n, by = ctypes.c_double(), ctypes.c_long(), ctypes.c_double()
    _check(load().wd_timing_get(int(cls), ctypes.byref(ms), ctypes.byref(n), ctypes.byref(by)))
    return ms.value, n.value, by.value
