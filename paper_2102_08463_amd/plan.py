"""Plan object over the C ABI: plan / set points / execute / destroy (Sec. I-A).

Tensors are torch device tensors; their pointers and torch's current stream
are handed to libmnufft.  This module only checks shapes and dtypes and
allocates outputs; all computation happens in the library.
"""
import ctypes

import torch

from . import lib as L

_REAL = {torch.complex64: torch.float32, torch.complex128: torch.float64}
_PREC = {torch.complex64: L.F32, torch.complex128: L.F64}


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _need(t, dtype, device, what):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what} must be a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{what} must have dtype {dtype}, got {t.dtype}")
    if t.device != device:
        raise ValueError(f"{what} must be on {device}, got {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")


class Plan:
    """A 1D, 2D or 3D type 1, 2 or 3 NUFFT plan on one GPU.

    nufft_type   1 (nonuniform -> modes), 2 (modes -> nonuniform) or
                 3 (nonuniform points -> nonuniform frequencies)
    n_modes      (N1,), (N1, N2) or (N1, N2, N3); arrays of modes have shape
                 (..., N3, N2, N1), i.e. k1 fastest, modes ascending from -N/2.
                 For type 3 the dimension (1, 2 or 3) instead
    n_trans      number of vectors sharing one set of points
    eps          requested relative l2 tolerance
    isign        sign of the exponent; default -1 for types 1 and 3, +1 for type 2
    dtype        torch.complex64 (fp32) or torch.complex128 (fp64)
    method       "auto", "gm", "gmsort" or "sm"
    binsize      bin extents m_i (None = library default), msub: points per subproblem
    upsampfac    fine-grid upsampling factor sigma (0 = 2; 1.25 .. 2 allowed)
    tune         "off", "autotune" or "learned": every setpts lets the library
                 choose method, bins and msub for the points (mnufft_select)
    """

    def __init__(self, nufft_type, n_modes, n_trans=1, eps=1e-6, isign=None,
                 dtype=torch.complex64, method="auto", binsize=None, msub=0,
                 device=None, validate_pts=False, upsampfac=0.0, tune="off"):
        self._lib = L.load()
        self._h = ctypes.c_void_p(0)
        if dtype not in _PREC:
            raise TypeError("dtype must be torch.complex64 or torch.complex128")
        self.type = int(nufft_type)
        if self.type == 3:
            self.dim = int(n_modes) if isinstance(n_modes, int) else len(n_modes)
            self.n_modes = None
        else:
            self.n_modes = tuple(int(n) for n in n_modes)
            self.dim = len(self.n_modes)
        self.n_trans = int(n_trans)
        self.eps = float(eps)
        self.isign = int(isign if isign is not None else (1 if self.type == 2 else -1))
        self.dtype = dtype
        self.rdtype = _REAL[dtype]
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        o = L.default_opts()
        o.method = L.METHODS[method] if isinstance(method, str) else int(method)
        if binsize is not None:
            for d, m in enumerate(binsize):
                o.binsize[d] = int(m)
        o.msub = int(msub)
        o.validate_pts = int(bool(validate_pts))
        o.upsampfac = float(upsampfac)
        o.tune = L.TUNES[tune] if isinstance(tune, str) else int(tune)
        o.device = self.device.index if self.device.index is not None else -1
        o.stream = torch.cuda.current_stream(self.device).cuda_stream
        self._stream = torch.cuda.current_stream(self.device)
        nm = None if self.type == 3 else \
            (ctypes.c_int64 * 3)(*(list(self.n_modes) + [1] * (3 - self.dim)))
        rc = self._lib.mnufft_makeplan(self.type, self.dim, nm, self.isign, self.n_trans,
                                       self.eps, _PREC[dtype], ctypes.byref(o),
                                       ctypes.byref(self._h))
        L.check(rc, "mnufft_makeplan")
        self.status = rc
        self.M = None
        self.K = None
        self._pts = None

    # -- lifetime ------------------------------------------------------------
    def destroy(self):
        if self._h and self._h.value:
            L.check(self._lib.mnufft_destroy(self._h), "mnufft_destroy")
        self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.destroy()

    # -- info ----------------------------------------------------------------
    def info(self):
        inf = L.Info()
        L.check(self._lib.mnufft_get_info(self._h, ctypes.byref(inf)), "mnufft_get_info")
        return inf.as_dict()

    @property
    def fine_shape(self):
        """Fine grid (n_d, ..., n_1) as a tensor shape (first coordinate fastest)."""
        n = self.info()["nfine"][: self.dim]
        return tuple(n[::-1])

    @property
    def mode_shape(self):
        return tuple(self.n_modes[::-1])

    def set_stream(self, stream):
        """Order the plan's later work on `stream` (a torch.cuda.Stream); after
        one eager call of each direction, execute / execute_adjoint can be
        captured into a CUDA/HIP graph on that stream."""
        L.check(self._lib.mnufft_set_stream(self._h, ctypes.c_void_p(stream.cuda_stream)),
                "mnufft_set_stream")
        self._stream = stream

    def set_timing(self, enable=True):
        """Turn the library's per-stage HIP-event timers on or off."""
        L.check(self._lib.mnufft_set_timing(self._h, int(bool(enable))), "mnufft_set_timing")

    def timing(self, reset=True):
        """{stage: (total ms, intervals)} since the last reset (synchronises)."""
        ms = (ctypes.c_double * len(L.STAGES))()
        cnt = (ctypes.c_int64 * len(L.STAGES))()
        L.check(self._lib.mnufft_get_timing(self._h, ms, cnt, int(bool(reset))),
                "mnufft_get_timing")
        return {name: (ms[i], cnt[i]) for i, name in enumerate(L.STAGES)}

    # -- points --------------------------------------------------------------
    def setpts(self, x, y=None, z=None, s=None, t=None, u=None):
        """Set the points (x[, y[, z]]); for type 3 also the frequencies (s[, t[, u]])."""
        if self.type == 3:
            return self._setpts3((x, y, z), (s, t, u))
        M = x.shape[0]
        given = (x, y, z)
        for d, nm in enumerate("xyz"):
            a = given[d]
            if d >= self.dim:
                if a is not None:
                    raise ValueError(f"{nm} given for a {self.dim}D plan")
                continue
            _need(a, self.rdtype, self.device, nm)
            if a.ndim != 1 or a.shape[0] != M:
                raise ValueError("the coordinate arrays must be 1-D of equal length")
        ptrs = [_ptr(a) if d < self.dim else None for d, a in enumerate(given)]
        rc = self._lib.mnufft_setpts(self._h, M, *ptrs)
        L.check(rc, "mnufft_setpts")
        self.M = M
        return self

    def _setpts3(self, pts, freqs):
        if any(a is not None for a in pts[self.dim:] + freqs[self.dim:]):
            raise ValueError(f"coordinates given for an absent dimension of a {self.dim}D plan")
        pts, freqs = pts[: self.dim], freqs[: self.dim]
        if any(a is None for a in pts + freqs):
            raise ValueError(f"type 3 needs {self.dim} point and {self.dim} frequency arrays")
        M, K = pts[0].shape[0], freqs[0].shape[0]
        for arrs, n, nm in ((pts, M, "points"), (freqs, K, "frequencies")):
            for a in arrs:
                _need(a, self.rdtype, self.device, nm)
                if a.ndim != 1 or a.shape[0] != n:
                    raise ValueError(f"{nm} must be 1-D arrays of equal length")
        pp = [_ptr(a) for a in pts] + [None] * (3 - self.dim)
        ff = [_ptr(a) for a in freqs] + [None] * (3 - self.dim)
        L.check(self._lib.mnufft_setpts3(self._h, M, *pp, K, *ff), "mnufft_setpts3")
        self.M, self.K = M, K
        return self

    # -- execution -------------------------------------------------------------
    def _c_shape(self):
        return (self.n_trans, self.M) if self.n_trans > 1 else (self.M,)

    def _f_shape(self):
        return ((self.n_trans,) if self.n_trans > 1 else ()) + self.mode_shape

    def _run(self, fn, c_in, f_in, what):
        if self.M is None:
            raise RuntimeError("setpts must be called before execute")
        if c_in is not None:
            _need(c_in, self.dtype, self.device, "c")
            if c_in.numel() != self.n_trans * self.M:
                raise ValueError(f"c must hold {self.n_trans} x {self.M} values")
            f = torch.empty(self._f_shape(), dtype=self.dtype, device=self.device)
            L.check(fn(self._h, _ptr(c_in), _ptr(f)), what)
            return f
        _need(f_in, self.dtype, self.device, "f")
        if f_in.numel() != self.n_trans * int(torch.tensor(self.n_modes).prod()):
            raise ValueError(f"f must hold {self.n_trans} x {self.n_modes} values")
        c = torch.empty(self._c_shape(), dtype=self.dtype, device=self.device)
        L.check(fn(self._h, _ptr(c), _ptr(f_in)), what)
        return c

    def execute(self, data):
        """Type 1: data = strengths c -> modes f.  Type 2: data = modes f -> values c.
        Type 3: data = strengths c (M,) or (n_trans, M) -> f (K,) or (n_trans, K)."""
        if self.type == 3:
            if self.M is None:
                raise RuntimeError("setpts must be called before execute")
            _need(data, self.dtype, self.device, "c")
            if data.numel() != self.n_trans * self.M:
                raise ValueError(f"c must hold {self.n_trans} x {self.M} values")
            f = torch.empty((self.n_trans, self.K) if self.n_trans > 1 else (self.K,),
                            dtype=self.dtype, device=self.device)
            L.check(self._lib.mnufft_execute(self._h, _ptr(data), _ptr(f)), "mnufft_execute")
            return f
        if self.type == 1:
            return self._run(self._lib.mnufft_execute, data, None, "mnufft_execute")
        return self._run(self._lib.mnufft_execute, None, data, "mnufft_execute")

    def execute_sorted(self, data):
        """As execute, with the point-indexed side (c) in bin-sorted order:
        c[..., i] belongs to input point perm[i] of get_sort()."""
        if self.type == 1:
            return self._run(self._lib.mnufft_execute_sorted, data, None, "mnufft_execute_sorted")
        return self._run(self._lib.mnufft_execute_sorted, None, data, "mnufft_execute_sorted")

    def execute_adjoint(self, data):
        """Adjoint operator on the same points (other type, opposite sign)."""
        if self.type == 1:
            return self._run(self._lib.mnufft_execute_adjoint, None, data, "mnufft_execute_adjoint")
        return self._run(self._lib.mnufft_execute_adjoint, data, None, "mnufft_execute_adjoint")

    def interp_grad(self, modes, wts):
        """Position gradients: for each dimension i, the M reals
        sum_t Re(conj(wts[t, j]) d v_t(x_j)/dx_i), v_t the type 2 sum of modes[t]
        in the plan's type 2 direction.  Returns a tuple of dim tensors."""
        _need(modes, self.dtype, self.device, "modes")
        _need(wts, self.dtype, self.device, "wts")
        if modes.numel() != self.n_trans * int(torch.tensor(self.n_modes).prod()):
            raise ValueError("modes has the wrong size")
        if wts.numel() != self.n_trans * self.M:
            raise ValueError("wts has the wrong size")
        outs = [torch.empty((self.M,), dtype=self.rdtype, device=self.device)
                for _ in range(self.dim)]
        ptrs = [_ptr(o) for o in outs] + [ctypes.c_void_p(0)] * (3 - self.dim)
        L.check(self._lib.mnufft_interp_grad(self._h, _ptr(modes), _ptr(wts), *ptrs),
                "mnufft_interp_grad")
        return tuple(outs)

    def spread(self, c):
        """Step 1 of type 1 alone for one vector c (M,) -> fine grid."""
        _need(c, self.dtype, self.device, "c")
        grid = torch.empty(self.fine_shape, dtype=self.dtype, device=self.device)
        L.check(self._lib.mnufft_spread(self._h, _ptr(c), _ptr(grid)), "mnufft_spread")
        return grid

    def interp(self, grid):
        """Step 3 of type 2 alone: fine grid -> values at the points (M,)."""
        _need(grid, self.dtype, self.device, "grid")
        if tuple(grid.shape) != self.fine_shape:
            raise ValueError(f"grid must have shape {self.fine_shape}")
        c = torch.empty((self.M,), dtype=self.dtype, device=self.device)
        L.check(self._lib.mnufft_interp(self._h, _ptr(grid), _ptr(c)), "mnufft_interp")
        return c

    def get_sort(self):
        """(perm, binstart) int32 device tensors from the last setpts."""
        inf = self.info()
        perm = torch.empty((max(self.M, 0),), dtype=torch.int32, device=self.device)
        bs = torch.empty((inf["nbins"] + 1,), dtype=torch.int32, device=self.device)
        L.check(self._lib.mnufft_get_sort(self._h, _ptr(perm), _ptr(bs)), "mnufft_get_sort")
        return perm, bs

    def get_subproblems(self):
        """(records (nsub, 4) int32, nsub) from the last setpts."""
        inf = self.info()
        cap = max(int(inf["nsub_max"]), 1)
        sub = torch.zeros((cap, 4), dtype=torch.int32, device=self.device)
        n = torch.zeros((1,), dtype=torch.int32, device=self.device)
        L.check(self._lib.mnufft_get_subproblems(self._h, _ptr(sub), _ptr(n)),
                "mnufft_get_subproblems")
        k = int(n.item())
        return sub[:k], k


def nufft_type1(points, c, n_modes, eps=1e-6, isign=-1, **kw):
    """One-shot type 1: points = (x[, y[, z]]) real tensors, c complex (M,) or (T, M)."""
    T = c.shape[0] if c.ndim == 2 else 1
    with Plan(1, n_modes, T, eps, isign, dtype=c.dtype, **kw) as p:
        p.setpts(*points)
        return p.execute(c.contiguous())


def nufft_type2(points, f, eps=1e-6, isign=+1, **kw):
    """One-shot type 2: f complex (..., N2, N1) or with a leading transform axis."""
    dim = len(points)
    n_modes = tuple(f.shape[-dim:][::-1])
    T = f.shape[0] if f.ndim == dim + 1 else 1
    with Plan(2, n_modes, T, eps, isign, dtype=f.dtype, **kw) as p:
        p.setpts(*points)
        return p.execute(f.contiguous())


def nufft_type3(points, c, freqs, eps=1e-6, isign=-1, **kw):
    """One-shot type 3: points = (x, y[, z]) and freqs = (s, t[, u]) real tensors,
    c complex (M,) or (T, M); returns f complex (K,) or (T, K)."""
    T = c.shape[0] if c.ndim == 2 else 1
    dim = len(points)
    with Plan(3, dim, T, eps, isign, dtype=c.dtype, **kw) as p:
        p.setpts(*points, *([None] * (3 - dim)), *freqs)
        return p.execute(c.contiguous())
