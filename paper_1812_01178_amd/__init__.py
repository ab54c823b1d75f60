"""Python binding of libtri, the MI355X (gfx950) library of batched
partitioned tridiagonal solves (PDD / PPT, Sec. 3.2 of arXiv:1812.01178).

Argument marshalling only: every solve runs in the HIP kernels of
``libtri.so`` behind the C ABI declared in ``include/tri.h``; this module
converts Python arguments to that ABI and raises on a non-zero status.  The
function names are the C names.  Device memory and streams come from
PyTorch (``tensor.data_ptr()``, ``torch.cuda.current_stream().cuda_stream``)
or any other HIP allocator.

There is no CPU fallback: if ``libtri.so`` has not been built, the first call
raises ``TriError``.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime libtri binds to)

__all__ = [
    "TriError", "lib", "tri_create", "tri_destroy", "tri_set_stream", "tri_set_pdd_tolerance", "tri_sync_status",
    "tri_status_string", "tri_last_error", "tri_pdd_solve", "tri_ppt_solve", "adi_sweep",
    "poisson_wavenumber_solve", "tri_plan_create", "tri_plan_execute", "tri_plan_capture",
    "tri_plan_graph_launch", "tri_plan_item_partitions", "tri_plan_item_describe", "tri_plan_launch_count",
    "tri_plan_destroy", "TriLines", "TriCoef", "TriInfo", "TriItem", "EXPORTED",
    "TRI_F64", "TRI_F32_REFINE", "TRI_REAL", "TRI_COMPLEX", "TRI_PDD", "TRI_PPT",
    "TRI_DIR_X", "TRI_DIR_Y", "TRI_DIR_Z", "TRI_ITEM_ADI_X", "TRI_ITEM_ADI_Y",
    "TRI_ITEM_ADI_Z", "TRI_ITEM_POISSON", "TRI_MAX_PARTITIONS", "tri_stream_copy", "tri_reserve",
    "spanwise_rfft", "spanwise_irfft", "projection_divergence_rfft", "projection_correct", "projection_step",
    "poisson_shifted_solve", "streamwise_dct", "streamwise_idct", "projection3d_divergence_rfft",
    "projection3d_correct", "projection3d_step", "tri_ppt_pivots", "adi_sweep_noalloc",
    "TriNsConfig", "ns_create", "ns_step", "ns_destroy",
]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libtri.so")

TRI_OK, TRI_E_ARG, TRI_E_SHAPE, TRI_E_ZERO_PIVOT = 0, 1, 2, 3
TRI_E_PDD_UNSAFE, TRI_E_NOT_CONVERGED, TRI_E_HIP, TRI_E_NOMEM, TRI_E_UNSUPPORTED = 4, 5, 6, 7, 8
TRI_F64, TRI_F32_REFINE = 0, 1
TRI_REAL, TRI_COMPLEX = 0, 1
TRI_PDD, TRI_PPT = 0, 1
TRI_DIR_X, TRI_DIR_Y, TRI_DIR_Z = 0, 1, 2
TRI_ITEM_ADI_X, TRI_ITEM_ADI_Y, TRI_ITEM_ADI_Z, TRI_ITEM_POISSON = 0, 1, 2, 3
TRI_MAX_PARTITIONS = 16
TRI_NOALLOC_SCRATCH_BYTES = 1 << 20

# every symbol include/tri.h declares
EXPORTED = [
    "tri_create", "tri_destroy", "tri_set_stream", "tri_set_pdd_tolerance", "tri_sync_status", "tri_status_string",
    "tri_last_error", "tri_pdd_solve", "tri_ppt_solve", "adi_sweep", "poisson_wavenumber_solve",
    "tri_plan_create", "tri_plan_execute", "tri_plan_capture", "tri_plan_graph_launch",
    "tri_plan_item_partitions", "tri_plan_item_describe", "tri_plan_launch_count", "tri_plan_destroy",
    "tri_stream_copy", "tri_reserve",
    "spanwise_rfft", "spanwise_irfft", "projection_divergence_rfft", "projection_correct", "projection_step",
    "poisson_shifted_solve", "streamwise_dct", "streamwise_idct", "projection3d_divergence_rfft",
    "projection3d_correct", "projection3d_step", "tri_ppt_pivots", "adi_sweep_noalloc",
    "ns_create", "ns_step", "ns_destroy",
]


class TriError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        msg = f"{where}: {tri_status_string(status) if _lib else status}"
        if detail:
            msg += f" ({detail})"
        super().__init__(msg)
        self.status = status


class TriLines(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("n", "nb0", "nb1", "s_j", "s_b0", "s_b1")]


class TriCoef(ctypes.Structure):
    _fields_ = [("a", ctypes.c_void_p), ("b", ctypes.c_void_p), ("c", ctypes.c_void_p),
                ("cs_j", ctypes.c_int64), ("cs_b0", ctypes.c_int64), ("cs_b1", ctypes.c_int64)]


class TriInfo(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int), ("pdd_drop_max", ctypes.c_double),
                ("resid_max", ctypes.c_double)]


class TriItem(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("field", ctypes.c_void_p),
                ("Nx", ctypes.c_int64), ("Ny", ctypes.c_int64), ("Nz", ctypes.c_int64),
                ("a", ctypes.c_void_p), ("b", ctypes.c_void_p), ("c", ctypes.c_void_p),
                ("lam", ctypes.c_void_p), ("P", ctypes.c_int), ("periodic", ctypes.c_int),
                ("method", ctypes.c_int)]


class TriNsConfig(ctypes.Structure):
    _fields_ = [("Nx", ctypes.c_int64), ("Ny", ctypes.c_int64), ("Nz", ctypes.c_int64),
                ("dx", ctypes.c_double), ("dz", ctypes.c_double), ("dy", ctypes.POINTER(ctypes.c_double)),
                ("dt", ctypes.c_double), ("nu", ctypes.c_double), ("P_adi", ctypes.c_int * 3),
                ("P_poisson", ctypes.c_int)]


_lib = None
_V = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64


def lib():
    """Load libtri.so (raises TriError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise TriError(TRI_E_UNSUPPORTED, "libtri",
                       f"{LIB_PATH} missing: build it with python -m paper_1812_01178_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "tri_create": (_I, [ctypes.POINTER(_V), _I, _V]),
        "tri_destroy": (_I, [_V]),
        "tri_set_stream": (_I, [_V, _V]),
        "tri_set_pdd_tolerance": (_I, [_V, ctypes.c_double]),
        "tri_sync_status": (_I, [_V]),
        "tri_status_string": (ctypes.c_char_p, [_I]),
        "tri_last_error": (ctypes.c_char_p, [_V]),
        "tri_pdd_solve": (_I, [_V, ctypes.POINTER(TriCoef), ctypes.POINTER(TriLines), _I, _V, _I, _I,
                               _I, ctypes.POINTER(TriInfo)]),
        "tri_ppt_solve": (_I, [_V, ctypes.POINTER(TriCoef), ctypes.POINTER(TriLines), _I, _V, _I, _I,
                               _I, ctypes.POINTER(TriInfo)]),
        "tri_ppt_pivots": (_I, [_V, ctypes.POINTER(TriCoef), ctypes.POINTER(TriLines), _V, _I, _I, _V]),
        "ns_create": (_I, [_V, ctypes.POINTER(TriNsConfig), ctypes.POINTER(_V)]),
        "ns_step": (_I, [_V, _V, _V, _V, _V]),
        "ns_destroy": (_I, [_V]),
        "adi_sweep_noalloc": (_I, [_V, _I, _V, _I64, _I64, _I64, _V, _V, _V, _I, _I, _I, _I]),
        "adi_sweep": (_I, [_V, _I, _V, _I64, _I64, _I64, _V, _V, _V, _I, _I, _I, _I,
                           ctypes.POINTER(TriInfo)]),
        "poisson_wavenumber_solve": (_I, [_V, _V, _I64, _I64, _I64, _V, _V, _V, _I, _I, _I,
                                          ctypes.POINTER(TriInfo)]),
        "tri_plan_create": (_I, [_V, ctypes.POINTER(TriItem), _I, _I, ctypes.POINTER(_V)]),
        "tri_plan_execute": (_I, [_V]),
        "tri_plan_capture": (_I, [_V, ctypes.POINTER(_V)]),
        "tri_plan_graph_launch": (_I, [_V]),
        "tri_plan_item_partitions": (_I, [_V, _I]),
        "tri_plan_item_describe": (_I, [_V, _I, ctypes.c_char_p, _I]),
        "tri_plan_launch_count": (_I, [_V]),
        "tri_plan_destroy": (_I, [_V]),
        "tri_stream_copy": (_I, [_V, _V, _V, _I64]),
        "tri_reserve": (_I, [_V, _I64, _I, _I64]),
        "poisson_shifted_solve": (_I, [_V, _V, _I64, _I64, _I64, _V, _V, _V, _V, _I, _I]),
        "streamwise_dct": (_I, [_V, _V, _I64, _I64]),
        "streamwise_idct": (_I, [_V, _V, _I64, _I64]),
        "projection3d_divergence_rfft": (_I, [_V, _V, _V, _V, ctypes.c_double, _V, ctypes.c_double, _V,
                                              _I64, _I64, _I64]),
        "projection3d_correct": (_I, [_V, _V, _V, _V, _V, _V, ctypes.c_double, _V, ctypes.c_double,
                                      _I64, _I64, _I64]),
        "projection3d_step": (_I, [_V, _V, _V, _V, ctypes.c_double, _V, ctypes.c_double, _V, _V, _V, _V, _V, _V,
                                   _I64, _I64, _I64, _I]),
        "spanwise_rfft": (_I, [_V, _V, _V, _I64, _I64]),
        "spanwise_irfft": (_I, [_V, _V, _V, _I64, _I64]),
        "projection_divergence_rfft": (_I, [_V, _V, _V, _V, ctypes.c_double, _V, _I64, _I64, _I64]),
        "projection_correct": (_I, [_V, _V, _V, _V, _V, _V, ctypes.c_double, _I64, _I64, _I64]),
        "projection_step": (_I, [_V, _V, _V, _V, ctypes.c_double, _V, _V, _V, _V, _V, _I64, _I64, _I64, _I]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def tri_status_string(status: int) -> str:
    return lib().tri_status_string(int(status)).decode()


def tri_last_error(ctx) -> str:
    return lib().tri_last_error(ctx).decode()


def _check(st: int, where: str, ctx=None):
    if st != TRI_OK:
        raise TriError(st, where, tri_last_error(ctx) if ctx else "")


def _ptr(x) -> int | None:
    """Device address of a torch tensor (or an int address, or None)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if not x.is_cuda:
        raise TriError(TRI_E_ARG, "argument", "tensors passed to libtri must be on the GPU")
    return x.data_ptr()


def _info(want: bool):
    return TriInfo() if want else None


def _info_dict(info):
    if info is None:
        return None
    return {"sweeps": info.sweeps, "pdd_drop_max": info.pdd_drop_max, "resid_max": info.resid_max}


def tri_create(device: int = 0, stream: int | None = None):
    """Returns an opaque context handle (c_void_p)."""
    h = _V()
    st = lib().tri_create(ctypes.byref(h), int(device), stream)
    _check(st, "tri_create")
    return h


def tri_destroy(ctx) -> None:
    _check(lib().tri_destroy(ctx), "tri_destroy")


def tri_set_stream(ctx, stream: int | None) -> None:
    _check(lib().tri_set_stream(ctx, stream), "tri_set_stream", ctx)


def tri_reserve(ctx, n: int, P: int, matrices: int) -> None:
    """Grow the context workspace for one-shot solves with up to `matrices`
    shared matrices of n rows at P partitions (waits for the stream)."""
    _check(lib().tri_reserve(ctx, int(n), int(P), int(matrices)), "tri_reserve", ctx)


def tri_set_pdd_tolerance(ctx, tol: float) -> None:
    """Strict PDD: later PDD solves whose dropped entries exceed tol (> 0) make
    tri_sync_status raise TRI_E_PDD_UNSAFE; 0 turns the check off."""
    _check(lib().tri_set_pdd_tolerance(ctx, float(tol)), "tri_set_pdd_tolerance", ctx)


def tri_sync_status(ctx) -> int:
    """Waits for the context stream; raises on a device-side status."""
    st = lib().tri_sync_status(ctx)
    _check(st, "tri_sync_status", ctx)
    return st


def _lines(n, nb0, nb1, s_j, s_b0, s_b1):
    return TriLines(int(n), int(nb0), int(nb1), int(s_j), int(s_b0), int(s_b1))


def _solve(fn, name, ctx, a, b, c, d, lines, coef_strides=(1, 0, 0), complex_field=False,
           P=1, periodic=False, prec=TRI_F64, info=False):
    coef = TriCoef(_ptr(a), _ptr(b), _ptr(c), *[int(s) for s in coef_strides])
    ln = _lines(*lines)
    inf = _info(info)
    st = fn(ctx, ctypes.byref(coef), ctypes.byref(ln), TRI_COMPLEX if complex_field else TRI_REAL,
            _ptr(d), int(P), int(bool(periodic)), int(prec), ctypes.byref(inf) if inf else None)
    _check(st, name, ctx)
    return _info_dict(inf)


def tri_pdd_solve(ctx, a, b, c, d, lines, coef_strides=(1, 0, 0), complex_field=False, P=1,
                  periodic=False, prec=TRI_F64, info=False):
    """lines = (n, nb0, nb1, s_j, s_b0, s_b1); coef_strides = (cs_j, cs_b0, cs_b1)."""
    return _solve(lib().tri_pdd_solve, "tri_pdd_solve", ctx, a, b, c, d, lines, coef_strides,
                  complex_field, P, periodic, prec, info)


def tri_ppt_solve(ctx, a, b, c, d, lines, coef_strides=(1, 0, 0), complex_field=False, P=1,
                  periodic=False, prec=TRI_F64, info=False):
    return _solve(lib().tri_ppt_solve, "tri_ppt_solve", ctx, a, b, c, d, lines, coef_strides,
                  complex_field, P, periodic, prec, info)


def tri_ppt_pivots(ctx, a, b, c, d, lines, coef_strides, piv, P=1, periodic=False) -> None:
    """Per-line PPT (real, FP64) that also writes every row's pivot kind into
    the uint8 device tensor piv (nb0*nb1*n bytes; 1, 2 = first row of a 2x2
    pivot, 0 = its second row)."""
    coef = TriCoef(_ptr(a), _ptr(b), _ptr(c), *[int(s) for s in coef_strides])
    ln = _lines(*lines)
    st = lib().tri_ppt_pivots(ctx, ctypes.byref(coef), ctypes.byref(ln), _ptr(d), int(P), int(bool(periodic)),
                              _ptr(piv))
    _check(st, "tri_ppt_pivots", ctx)


def adi_sweep(ctx, direction: int, u, a, b, c, P: int, periodic=False, method=TRI_PDD,
              prec=TRI_F64, info=False, shape=None):
    """In-place sweep of u[Nz][Ny][Nx] (x fastest) along direction 0/1/2."""
    Nz, Ny, Nx = shape if shape is not None else tuple(u.shape)
    inf = _info(info)
    st = lib().adi_sweep(ctx, int(direction), _ptr(u), Nx, Ny, Nz, _ptr(a), _ptr(b), _ptr(c),
                         int(P), int(bool(periodic)), int(method), int(prec),
                         ctypes.byref(inf) if inf else None)
    _check(st, "adi_sweep", ctx)
    return _info_dict(inf)


def adi_sweep_noalloc(ctx, direction: int, u, a, b, c, P: int, periodic=False, method=TRI_PDD,
                      prec=TRI_F64, shape=None) -> None:
    """adi_sweep with the factor tables in the library's static device scratch:
    no allocation, no synchronisation (calls on one GPU must not overlap)."""
    Nz, Ny, Nx = shape if shape is not None else tuple(u.shape)
    st = lib().adi_sweep_noalloc(ctx, int(direction), _ptr(u), Nx, Ny, Nz, _ptr(a), _ptr(b), _ptr(c), int(P),
                                 int(bool(periodic)), int(method), int(prec))
    _check(st, "adi_sweep_noalloc", ctx)


def ns_create(ctx, Nx: int, Ny: int, Nz: int, dx: float, dz: float, dy, dt: float, nu: float,
              P_adi=(8, 4, 16), P_poisson: int = 8):
    """Set up the fractional-step time step on an Nx x Ny x Nz grid; dy is a host
    (numpy) array of Ny cell widths.  Returns an opaque handle."""
    import numpy as np
    dyh = np.ascontiguousarray(dy, dtype=np.float64)
    cfg = TriNsConfig(int(Nx), int(Ny), int(Nz), float(dx), float(dz),
                      dyh.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(dt), float(nu),
                      (ctypes.c_int * 3)(*[int(p) for p in P_adi]), int(P_poisson))
    h = _V()
    _check(lib().ns_create(ctx, ctypes.byref(cfg), ctypes.byref(h)), "ns_create", ctx)
    return h


def ns_step(ns, u, v, w, p, ctx=None) -> None:
    """One time step in place on u[Nz][Ny][Nx+1], v[Nz][Ny+1][Nx], w[Nz][Ny][Nx], p[Nz][Ny][Nx]."""
    _check(lib().ns_step(ns, _ptr(u), _ptr(v), _ptr(w), _ptr(p)), "ns_step", ctx)


def ns_destroy(ns) -> None:
    _check(lib().ns_destroy(ns), "ns_destroy")


def poisson_wavenumber_solve(ctx, phihat, ay, cy, lam, P: int = 4, prec=TRI_F64,
                             fp64_kmax: int = 2, info=False, shape=None):
    """In-place wall-normal solves of phihat[Nk][Ny][Nx] complex128."""
    Nk, Ny, Nx = shape if shape is not None else tuple(phihat.shape)
    inf = _info(info)
    st = lib().poisson_wavenumber_solve(ctx, _ptr(phihat), Nx, Ny, Nk, _ptr(ay), _ptr(cy),
                                        _ptr(lam), int(P), int(prec), int(fp64_kmax),
                                        ctypes.byref(inf) if inf else None)
    _check(st, "poisson_wavenumber_solve", ctx)
    return _info_dict(inf)


def poisson_shifted_solve(ctx, phihat, ay, cy, lamz, lamx, P: int = 8, method=TRI_PPT) -> None:
    """In-place wall-normal solves of phihat[Nk][Ny][Nx] complex128 with the shift lamz_k + lamx_i."""
    Nk, Ny, Nx = phihat.shape
    _check(lib().poisson_shifted_solve(ctx, _ptr(phihat), Nx, Ny, Nk, _ptr(ay), _ptr(cy), _ptr(lamz), _ptr(lamx),
                                       int(P), int(method)), "poisson_shifted_solve", ctx)


def streamwise_dct(ctx, xhat) -> None:
    """In-place cosine transform along the last axis of a complex128 tensor."""
    Nx = xhat.shape[-1]
    _check(lib().streamwise_dct(ctx, _ptr(xhat), Nx, xhat.numel() // Nx), "streamwise_dct", ctx)


def streamwise_idct(ctx, xhat) -> None:
    """In-place inverse of streamwise_dct."""
    Nx = xhat.shape[-1]
    _check(lib().streamwise_idct(ctx, _ptr(xhat), Nx, xhat.numel() // Nx), "streamwise_idct", ctx)


def projection3d_divergence_rfft(ctx, u, v, w, dx: float, dy, dz: float, dhat) -> None:
    """dhat = spanwise FFT of div(u, v, w); u[Nz][Ny][Nx+1], v[Nz][Ny+1][Nx], w[Nz][Ny][Nx]."""
    Nz, Ny, Nx = w.shape
    _check(lib().projection3d_divergence_rfft(ctx, _ptr(u), _ptr(v), _ptr(w), float(dx), _ptr(dy), float(dz),
                                              _ptr(dhat), Nx, Ny, Nz), "projection3d_divergence_rfft", ctx)


def projection3d_correct(ctx, phihat, phi, u, v, w, dx: float, dy, dz: float) -> None:
    """phi = inverse spanwise FFT of phihat; u, v, w corrected in place by grad phi."""
    Nz, Ny, Nx = w.shape
    _check(lib().projection3d_correct(ctx, _ptr(phihat), _ptr(phi), _ptr(u), _ptr(v), _ptr(w), float(dx), _ptr(dy),
                                      float(dz), Nx, Ny, Nz), "projection3d_correct", ctx)


def projection3d_step(ctx, u, v, w, dx: float, dy, dz: float, ay, cy, lamz, lamx, phihat, phi, P: int = 8) -> None:
    """Divergence + spanwise FFT, streamwise cosine transform, shifted Poisson solves (PPT),
    inverse transforms, gradient correction of u, v, w."""
    Nz, Ny, Nx = w.shape
    _check(lib().projection3d_step(ctx, _ptr(u), _ptr(v), _ptr(w), float(dx), _ptr(dy), float(dz), _ptr(ay),
                                   _ptr(cy), _ptr(lamz), _ptr(lamx), _ptr(phihat), _ptr(phi), Nx, Ny, Nz, int(P)),
           "projection3d_step", ctx)


def spanwise_rfft(ctx, x, xhat) -> None:
    """xhat[Nz/2+1][...] (complex128) = real FFT along axis 0 of x[Nz][...] (float64)."""
    Nz = x.shape[0]
    lines = x.numel() // Nz
    _check(lib().spanwise_rfft(ctx, _ptr(x), _ptr(xhat), lines, Nz), "spanwise_rfft", ctx)


def spanwise_irfft(ctx, xhat, x) -> None:
    """x[Nz][...] (float64) = inverse real FFT along axis 0 of xhat[Nz/2+1][...]."""
    Nz = x.shape[0]
    lines = x.numel() // Nz
    _check(lib().spanwise_irfft(ctx, _ptr(xhat), _ptr(x), lines, Nz), "spanwise_irfft", ctx)


def projection_divergence_rfft(ctx, v, w, dy, dz: float, dhat) -> None:
    """dhat[Nz/2+1][Ny][Nx] = spanwise FFT of div(v, w); v[Nz][Ny+1][Nx], w[Nz][Ny][Nx]."""
    Nz, Ny, Nx = w.shape
    _check(lib().projection_divergence_rfft(ctx, _ptr(v), _ptr(w), _ptr(dy), float(dz), _ptr(dhat),
                                            Nx, Ny, Nz), "projection_divergence_rfft", ctx)


def projection_correct(ctx, phihat, phi, v, w, dy, dz: float) -> None:
    """phi = inverse spanwise FFT of phihat; v, w corrected in place by grad phi."""
    Nz, Ny, Nx = w.shape
    _check(lib().projection_correct(ctx, _ptr(phihat), _ptr(phi), _ptr(v), _ptr(w), _ptr(dy), float(dz),
                                    Nx, Ny, Nz), "projection_correct", ctx)


def projection_step(ctx, v, w, dy, dz: float, ay, cy, lam, phihat, phi, P: int = 4) -> None:
    """Divergence + FFT, Poisson wavenumber solves (PPT), inverse FFT + correction."""
    Nz, Ny, Nx = w.shape
    _check(lib().projection_step(ctx, _ptr(v), _ptr(w), _ptr(dy), float(dz), _ptr(ay), _ptr(cy), _ptr(lam),
                                 _ptr(phihat), _ptr(phi), Nx, Ny, Nz, int(P)), "projection_step", ctx)


def tri_plan_create(ctx, items, prec=TRI_F64):
    """items: list of dicts with keys kind, field, Nx, Ny, Nz, a, b, c, lam, P, periodic, method."""
    arr = (TriItem * max(1, len(items)))()
    for i, it in enumerate(items):
        arr[i] = TriItem(int(it["kind"]), _ptr(it["field"]), int(it["Nx"]), int(it["Ny"]),
                         int(it["Nz"]), _ptr(it.get("a")), _ptr(it.get("b")), _ptr(it.get("c")),
                         _ptr(it.get("lam")), int(it.get("P", 0)), int(bool(it.get("periodic", 0))),
                         int(it.get("method", TRI_PPT)))
    h = _V()
    st = lib().tri_plan_create(ctx, arr, len(items), int(prec), ctypes.byref(h))
    _check(st, "tri_plan_create", ctx)
    return h


def tri_plan_execute(plan) -> None:
    _check(lib().tri_plan_execute(plan), "tri_plan_execute")


def tri_plan_capture(plan) -> int:
    g = _V()
    _check(lib().tri_plan_capture(plan, ctypes.byref(g)), "tri_plan_capture")
    return g.value


def tri_plan_graph_launch(plan) -> None:
    _check(lib().tri_plan_graph_launch(plan), "tri_plan_graph_launch")


def tri_plan_item_partitions(plan, i: int) -> int:
    return int(lib().tri_plan_item_partitions(plan, int(i)))


def tri_plan_item_describe(plan, i: int) -> str:
    buf = ctypes.create_string_buffer(256)
    if lib().tri_plan_item_describe(plan, int(i), buf, 256) < 0:
        raise TriError(TRI_E_ARG, "tri_plan_item_describe")
    return buf.value.decode()


def tri_plan_launch_count(plan) -> int:
    return int(lib().tri_plan_launch_count(plan))


def tri_plan_destroy(plan) -> None:
    _check(lib().tri_plan_destroy(plan), "tri_plan_destroy")


def tri_stream_copy(ctx, dst, src, n: int | None = None) -> None:
    """Reference copy of n doubles (default: all of src) from src to dst on
    the context stream (measurement aid for bandwidth fractions)."""
    if n is None:
        n = src.numel() * (2 if src.is_complex() else 1)
    _check(lib().tri_stream_copy(ctx, _ptr(dst), _ptr(src), int(n)), "tri_stream_copy", ctx)
