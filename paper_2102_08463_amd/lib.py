"""ctypes binding of libmnufft (include/mnufft.h): argument marshalling only.

Every step of the transform runs in the library's HIP kernels (the FFT in
rocFFT).  PyTorch provides device memory and the stream; torch is imported
before the library is loaded so that both share one HIP runtime.  There is
no CPU fallback: if the library is missing, loading raises.
"""
import ctypes
import itertools
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmnufft.so")

OK = 0
WARN_EPS_CLAMPED = 1
ERR_ARG, ERR_ALLOC, ERR_HIP, ERR_FFT, ERR_STATE, ERR_PTS, ERR_UNSUPPORTED = -1, -2, -3, -4, -5, -6, -7
F32, F64 = 0, 1
METHOD_AUTO, METHOD_GM, METHOD_GMSORT, METHOD_SM = 0, 1, 2, 3
METHODS = {"auto": METHOD_AUTO, "gm": METHOD_GM, "gmsort": METHOD_GMSORT, "sm": METHOD_SM}

# Every symbol the public header declares.
EXPORTS = (
    "mnufft_default_opts", "mnufft_makeplan", "mnufft_setpts", "mnufft_setpts3", "mnufft_execute",
    "mnufft_execute_sorted",
    "mnufft_execute_adjoint", "mnufft_interp_grad", "mnufft_spread", "mnufft_interp",
    "mnufft_get_sort",
    "mnufft_get_subproblems", "mnufft_get_info", "mnufft_destroy", "mnufft_strerror",
    "mnufft_choose_params", "mnufft_choose_params_sigma", "mnufft_correction_factors",
    "mnufft_type3_grid",
    "mnufft_set_timing", "mnufft_get_timing", "mnufft_set_stream",
    "mnufft_batch_makeplan", "mnufft_batch_setpts", "mnufft_batch_execute",
    "mnufft_batch_set_timing", "mnufft_batch_get_timing", "mnufft_batch_get_totals",
    "mnufft_batch_destroy", "mnufft_tune_candidates", "mnufft_tune_time",
    "mnufft_density_features", "mnufft_density_features_batch",
    "mnufft_density_features_batch_noalloc", "mnufft_mlp_nparams", "mnufft_mlp_forward",
    "mnufft_mlp_loss_grad", "mnufft_mlp_backward", "mnufft_mlp_adam",
    "mnufft_selector_load", "mnufft_selector_clear", "mnufft_select", "mnufft_batch_select",
)
TUNE_OFF, TUNE_AUTOTUNE, TUNE_LEARNED = 0, 1, 2
TUNES = {"off": TUNE_OFF, "autotune": TUNE_AUTOTUNE, "learned": TUNE_LEARNED}
DENSITY_WORK_BYTES = 512 * 256 * 4
DENSITY_BATCH_WORK_BYTES = 32 * 256 * 4  # per point set
DENSITY_NOALLOC_MAX_SETS = 64


STAGES = ("setpts", "zero", "spread", "fft", "deconv", "precorrect", "interp", "addback", "scale")


class Opts(ctypes.Structure):
    _fields_ = [
        ("method", ctypes.c_int),
        ("binsize", ctypes.c_int * 3),
        ("msub", ctypes.c_int),
        ("validate_pts", ctypes.c_int),
        ("device", ctypes.c_int),
        ("stream", ctypes.c_void_p),
        ("upsampfac", ctypes.c_double),
        ("tune", ctypes.c_int),
        ("reserved", ctypes.c_int * 5),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("type", ctypes.c_int), ("dim", ctypes.c_int), ("prec", ctypes.c_int),
        ("iflag", ctypes.c_int),
        ("nmodes", ctypes.c_int64 * 3), ("nfine", ctypes.c_int64 * 3),
        ("ntransf", ctypes.c_int64), ("M", ctypes.c_int64),
        ("w", ctypes.c_int), ("beta", ctypes.c_double),
        ("method", ctypes.c_int), ("binsize", ctypes.c_int * 3), ("msub", ctypes.c_int),
        ("nbins", ctypes.c_int64), ("nsub_max", ctypes.c_int64),
        ("device_bytes", ctypes.c_int64), ("upsampfac", ctypes.c_double),
        ("ntargets", ctypes.c_int64),
    ]

    def as_dict(self):
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if hasattr(v, "__len__") else v
        return out


class MnufftError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})")


_lib = None


def load():
    """Load libmnufft.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    L.mnufft_default_opts.argtypes = [ctypes.POINTER(Opts)]
    L.mnufft_makeplan.argtypes = [ci, ci, ctypes.POINTER(i64), ci, i64, ctypes.c_double, ci,
                                  ctypes.POINTER(Opts), ctypes.POINTER(vp)]
    L.mnufft_setpts.argtypes = [vp, i64, vp, vp, vp]
    L.mnufft_setpts3.argtypes = [vp, i64, vp, vp, vp, i64, vp, vp, vp]
    L.mnufft_execute.argtypes = [vp, vp, vp]
    L.mnufft_execute_sorted.argtypes = [vp, vp, vp]
    L.mnufft_execute_adjoint.argtypes = [vp, vp, vp]
    L.mnufft_interp_grad.argtypes = [vp, vp, vp, vp, vp, vp]
    L.mnufft_spread.argtypes = [vp, vp, vp]
    L.mnufft_interp.argtypes = [vp, vp, vp]
    L.mnufft_get_sort.argtypes = [vp, vp, vp]
    L.mnufft_get_subproblems.argtypes = [vp, vp, vp]
    L.mnufft_get_info.argtypes = [vp, ctypes.POINTER(Info)]
    L.mnufft_destroy.argtypes = [vp]
    L.mnufft_strerror.argtypes = [ci]
    L.mnufft_strerror.restype = ctypes.c_char_p
    L.mnufft_choose_params.argtypes = [ctypes.c_double, ci, i64, ctypes.POINTER(ci),
                                       ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
    L.mnufft_choose_params_sigma.argtypes = [ctypes.c_double, ci, i64, ctypes.c_double,
                                             ctypes.POINTER(ci), ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(i64)]
    L.mnufft_correction_factors.argtypes = [i64, i64, ci, ctypes.c_double,
                                            ctypes.POINTER(ctypes.c_double)]
    L.mnufft_type3_grid.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, ci,
                                    ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double)]
    L.mnufft_set_timing.argtypes = [vp, ci]
    L.mnufft_set_stream.argtypes = [vp, vp]
    L.mnufft_get_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(i64), ci]
    i32p = ctypes.POINTER(ctypes.c_int32)
    L.mnufft_batch_makeplan.argtypes = [ci, ci, ci, ctypes.POINTER(i64), ctypes.POINTER(i64), ci,
                                        ctypes.c_double, ci, i32p, i32p, ctypes.POINTER(Opts),
                                        ctypes.POINTER(vp)]
    L.mnufft_batch_setpts.argtypes = [vp, vp, vp, vp]
    L.mnufft_batch_execute.argtypes = [vp, vp, vp]
    L.mnufft_batch_set_timing.argtypes = [vp, ci]
    L.mnufft_batch_get_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(i64), ci]
    L.mnufft_batch_get_totals.argtypes = [vp, ctypes.POINTER(i64)]
    L.mnufft_batch_destroy.argtypes = [vp]
    L.mnufft_tune_candidates.argtypes = [ci, ci, ctypes.c_double, ctypes.POINTER(Opts), ci]
    L.mnufft_tune_time.argtypes = [ci, ci, ctypes.POINTER(i64), ci, ctypes.c_double, ci, i64, vp, vp,
                                   vp, vp, vp, ctypes.POINTER(Opts), ci, ci, ctypes.c_double,
                                   ctypes.POINTER(ctypes.c_double)]
    fp = ctypes.POINTER(ctypes.c_float)
    L.mnufft_density_features.argtypes = [ci, i64, vp, vp, vp, vp, vp]
    L.mnufft_density_features_batch.argtypes = [ci, ci, vp, vp, vp, vp, ci, vp, vp]
    L.mnufft_density_features_batch_noalloc.argtypes = [ci, ci, vp, vp, vp, vp, ci, vp]
    L.mnufft_mlp_nparams.argtypes = [ci, ci, ci]
    L.mnufft_mlp_forward.argtypes = [ci, ci, ci, vp, ci, vp, vp, vp, vp, vp]
    L.mnufft_mlp_loss_grad.argtypes = [ci, ci, vp, vp, vp, vp, vp, vp]
    L.mnufft_mlp_backward.argtypes = [ci, ci, ci, vp, ci, vp, vp, vp, vp, vp, vp, vp]
    L.mnufft_mlp_adam.argtypes = [i64, vp, vp, vp, vp, ctypes.c_float, ctypes.c_float,
                                  ctypes.c_float, ctypes.c_float, ci, vp]
    L.mnufft_selector_load.argtypes = [ctypes.c_char_p]
    L.mnufft_selector_clear.argtypes = []
    L.mnufft_select.argtypes = [ci, ci, ctypes.POINTER(i64), ci, ctypes.c_double, ci, i64, vp, vp,
                                vp, ci, ctypes.POINTER(Opts), ctypes.POINTER(Opts),
                                ctypes.POINTER(ci)]
    # (raw addresses for the arrays: batch_select passes numpy buffers)
    L.mnufft_batch_select.argtypes = [ci, ci, ci, vp, vp, vp, vp, vp, ctypes.c_double, ci, ci,
                                      ctypes.POINTER(Opts), vp, vp, vp]
    for name in EXPORTS:
        getattr(L, name).restype = ctypes.c_char_p if name == "mnufft_strerror" else ci
    L.mnufft_mlp_nparams.restype = ctypes.c_int64
    _lib = L
    return L


def strerror(code):
    try:
        return load().mnufft_strerror(int(code)).decode()
    except Exception:  # pragma: no cover
        return "status %d" % code


def check(code, what):
    if code < 0:
        raise MnufftError(code, what)
    return code


def default_opts():
    o = Opts()
    check(load().mnufft_default_opts(ctypes.byref(o)), "mnufft_default_opts")
    return o


def choose_params(eps, prec, N, sigma=2.0):
    """(w, beta, n, status) as the library picks them for one dimension and
    upsampling factor sigma (host only)."""
    w, beta, n = ctypes.c_int(), ctypes.c_double(), ctypes.c_int64()
    rc = check(load().mnufft_choose_params_sigma(float(eps), int(prec), int(N), float(sigma),
                                                 ctypes.byref(w), ctypes.byref(beta),
                                                 ctypes.byref(n)),
               "mnufft_choose_params_sigma")
    return w.value, beta.value, n.value, rc


def correction_factors(N, n, w, beta):
    """The library's per-dimension correction factors (host only), as a list."""
    out = (ctypes.c_double * int(N))()
    check(load().mnufft_correction_factors(int(N), int(n), int(w), float(beta), out),
          "mnufft_correction_factors")
    return list(out)


def tune_candidates(dim, prec, eps):
    """The autotuner's candidate options (list of Opts), in the library's order."""
    n = check(load().mnufft_tune_candidates(int(dim), int(prec), float(eps), None, 0),
              "mnufft_tune_candidates")
    arr = (Opts * max(n, 1))()
    check(load().mnufft_tune_candidates(int(dim), int(prec), float(eps), arr, n),
          "mnufft_tune_candidates")
    return [arr[i] for i in range(n)]


def selector_load(path):
    """Register a learned selector file with the library (mnufft_selector_load)."""
    check(load().mnufft_selector_load(str(path).encode()), "mnufft_selector_load")


def select(nufft_type, n_modes, points, eps, mode="learned", isign=None, upsampfac=0.0):
    """(Opts chosen by mnufft_select, source: 0 learned / 1 autotuner) for one
    problem on its points (torch device tensors of the run precision)."""
    import torch
    dim = len(n_modes)
    prec = F32 if points[0].dtype == torch.float32 else F64
    nm = (ctypes.c_int64 * 3)(*(list(n_modes) + [1] * (3 - dim)))
    base = default_opts()
    base.stream = torch.cuda.current_stream().cuda_stream
    base.upsampfac = float(upsampfac)
    out, src = Opts(), ctypes.c_int(-1)
    ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)
    pts = list(points) + [None] * (3 - dim)
    isign = isign if isign is not None else (-1 if nufft_type == 1 else 1)
    check(load().mnufft_select(int(nufft_type), dim, nm, int(isign), float(eps), prec,
                               points[0].numel(), ptr(pts[0]), ptr(pts[1]), ptr(pts[2]),
                               TUNES[mode], ctypes.byref(base), ctypes.byref(out),
                               ctypes.byref(src)), "mnufft_select")
    return out, src.value


def batch_select(nufft_type, n_modes_list, npts, x, y, eps, z=None, mode="learned"):
    """Per-transform (binsize list, msub list, source list) from
    mnufft_batch_select for point sets stored back to back in x, y (, z)."""
    import numpy as np
    import torch
    T = len(npts)
    dim = len(n_modes_list[0])
    prec = F32 if x.dtype == torch.float32 else F64
    # (raw addresses: numpy's ctypes.data_as and ctypes.cast cost microseconds
    # each, and this call sits on the selection's critical path)
    nm = np.ones((T, 3), np.int64)
    nm[:, :dim] = np.fromiter(itertools.chain.from_iterable(n_modes_list), np.int64,
                              T * dim).reshape(T, dim)
    npa = np.fromiter(npts, np.int64, T)
    out = np.zeros(5 * T, np.int32)  # binsize (3 T), msub (T), source (T)
    base = _base_opts()
    base.stream = torch.cuda.current_stream().cuda_stream
    o = out.ctypes.data
    check(load().mnufft_batch_select(int(nufft_type), dim, T, nm.ctypes.data, npa.ctypes.data,
                                     x.data_ptr(), y.data_ptr(),
                                     z.data_ptr() if z is not None else None, float(eps), prec,
                                     TUNES[mode], ctypes.byref(base), o, o + 12 * T, o + 16 * T),
          "mnufft_batch_select")
    bins = out[:3 * T].reshape(T, 3)[:, :dim].tolist()
    return [tuple(b) for b in bins], out[3 * T:4 * T].tolist(), out[4 * T:].tolist()


_BASE = None


def _base_opts():
    """A fresh copy of the library's default options (read once)."""
    global _BASE
    if _BASE is None:
        _BASE = default_opts()
    o = Opts()
    ctypes.pointer(o)[0] = _BASE
    return o


def describe(o):
    """Short text form of a candidate's method / bins / msub."""
    name = {METHOD_AUTO: "auto", METHOD_GM: "gm", METHOD_GMSORT: "gmsort", METHOD_SM: "sm"}[o.method]
    return f"{name}:{'x'.join(str(b) for b in o.binsize if b)}:{o.msub}"
