"""Batches of transforms of uneven size in one launch per stage (C ABI mnufft_batch_*).

Points, strengths and modes are concatenated in transform order; this
module only builds the descriptor arrays, checks sizes and allocates
outputs.
"""
import ctypes

import torch

from . import lib as L
from .plan import _PREC, _REAL, _need, _ptr


class Batch:
    """ntr transforms of one type / dimension / sign / eps / precision.

    n_modes   list of (N1, N2[, N3]) per transform
    n_points  list of M per transform
    binsize   optional list of per-transform bin extents; msub: optional list
    upsampfac fine-grid upsampling factor sigma (0 = 2; 1.25 .. 2 allowed)
    """

    def __init__(self, nufft_type, n_modes, n_points, eps=1e-6, isign=None,
                 dtype=torch.complex64, binsize=None, msub=None, device=None, upsampfac=0.0):
        self._lib = L.load()
        self._h = ctypes.c_void_p(0)
        self.type = int(nufft_type)
        self.n_modes = [tuple(int(v) for v in nm) for nm in n_modes]
        self.dim = len(self.n_modes[0])
        self.n_points = [int(m) for m in n_points]
        self.T = len(self.n_modes)
        if len(self.n_points) != self.T:
            raise ValueError("n_modes and n_points differ in length")
        self.isign = int(isign if isign is not None else (-1 if self.type == 1 else 1))
        self.dtype = dtype
        self.rdtype = _REAL[dtype]
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        nm = (ctypes.c_int64 * (3 * self.T))()
        for t, m in enumerate(self.n_modes):
            for d in range(3):
                nm[3 * t + d] = m[d] if d < self.dim else 1
        npts = (ctypes.c_int64 * self.T)(*self.n_points)
        bs = None
        if binsize is not None:
            bs = (ctypes.c_int32 * (3 * self.T))()
            for t, b in enumerate(binsize):
                for d in range(len(b)):
                    bs[3 * t + d] = int(b[d])
        ms = (ctypes.c_int32 * self.T)(*[int(v) for v in msub]) if msub is not None else None
        o = L.default_opts()
        o.device = self.device.index if self.device.index is not None else -1
        o.stream = torch.cuda.current_stream(self.device).cuda_stream
        o.upsampfac = float(upsampfac)
        rc = self._lib.mnufft_batch_makeplan(self.type, self.dim, self.T, nm, npts, self.isign,
                                             float(eps), _PREC[dtype], bs, ms, ctypes.byref(o),
                                             ctypes.byref(self._h))
        L.check(rc, "mnufft_batch_makeplan")
        self.mode_counts = [int(torch.tensor(m).prod()) for m in self.n_modes]
        self.Mtot = sum(self.n_points)
        self.Ktot = sum(self.mode_counts)

    def destroy(self):
        if self._h and self._h.value:
            L.check(self._lib.mnufft_batch_destroy(self._h), "mnufft_batch_destroy")
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

    def setpts(self, x, y, z=None):
        for t, name in ((x, "x"), (y, "y")) + (((z, "z"),) if self.dim == 3 else ()):
            _need(t, self.rdtype, self.device, name)
            if t.numel() != self.Mtot:
                raise ValueError(f"{name} must hold {self.Mtot} points")
        L.check(self._lib.mnufft_batch_setpts(self._h, _ptr(x), _ptr(y),
                                              _ptr(z) if self.dim == 3 else None),
                "mnufft_batch_setpts")
        return self

    def execute(self, data):
        """Type 1: data = concatenated strengths -> concatenated modes;
        type 2: the reverse."""
        _need(data, self.dtype, self.device, "data")
        if self.type == 1:
            if data.numel() != self.Mtot:
                raise ValueError("c has the wrong size")
            f = torch.empty((self.Ktot,), dtype=self.dtype, device=self.device)
            L.check(self._lib.mnufft_batch_execute(self._h, _ptr(data), _ptr(f)), "mnufft_batch_execute")
            return f
        if data.numel() != self.Ktot:
            raise ValueError("f has the wrong size")
        c = torch.empty((self.Mtot,), dtype=self.dtype, device=self.device)
        L.check(self._lib.mnufft_batch_execute(self._h, _ptr(c), _ptr(data)), "mnufft_batch_execute")
        return c

    def split_modes(self, f):
        """List of per-transform mode arrays shaped (.., N2, N1)."""
        out, k = [], 0
        for nm, cnt in zip(self.n_modes, self.mode_counts):
            out.append(f[k:k + cnt].reshape(nm[::-1]))
            k += cnt
        return out

    def set_timing(self, enable=True):
        L.check(self._lib.mnufft_batch_set_timing(self._h, int(bool(enable))), "mnufft_batch_set_timing")

    def timing(self, reset=True):
        ms = (ctypes.c_double * len(L.STAGES))()
        cnt = (ctypes.c_int64 * len(L.STAGES))()
        L.check(self._lib.mnufft_batch_get_timing(self._h, ms, cnt, int(bool(reset))),
                "mnufft_batch_get_timing")
        return {name: (ms[i], cnt[i]) for i, name in enumerate(L.STAGES)}

    def totals(self):
        t = (ctypes.c_int64 * 6)()
        L.check(self._lib.mnufft_batch_get_totals(self._h, t), "mnufft_batch_get_totals")
        return dict(zip(("points", "modes", "cells", "bins", "nsub_max", "device_bytes"), list(t)))
