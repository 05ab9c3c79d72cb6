"""The three-step type 1 / type 2 algorithm of Sec. II in plain FP64.

Part of the oracle (test infrastructure; see ``oracle/__init__.py``).

Type 1 (Sec. II-A): spread onto the fine grid, FFT, truncate to the central
modes and multiply by the correction factors.  Type 2 (Sec. II-B): the same
steps transposed: precorrect and zero-pad, FFT of the opposite role,
interpolate.  The sign of the exponent (iflag) is a free parameter; the FFT
carries that sign and no 1/n normalisation is applied anywhere.
"""
import numpy as np

from . import direct, params

try:
    import scipy.fft as _sfft
except ImportError:  # pragma: no cover
    _sfft = None


class Params:
    """w, beta and the fine grid of Sec. II for given modes and tolerance."""

    def __init__(self, Ns, eps, wmax=16, sigma=params.SIGMA):
        self.Ns = tuple(int(N) for N in Ns)
        self.dim = len(self.Ns)
        self.eps = float(eps)
        self.sigma = sigma
        self.w = params.kernel_width(eps, wmax=wmax, sigma=sigma)
        self.beta = params.kernel_beta(self.w, sigma=sigma)
        self.ns = tuple(params.fine_grid_size(N, self.w, sigma=sigma) for N in self.Ns)

    def factors(self):
        return [params.correction_factors(N, n, self.w, self.beta)
                for N, n in zip(self.Ns, self.ns)]


def _fft_signed(b, iflag, workers):
    """sum_l b_l exp(iflag 2 pi i l.k / n) over all axes, unnormalised."""
    kw = {} if _sfft is None else {"workers": workers}
    if iflag < 0:
        return (_sfft.fftn(b, **kw) if _sfft else np.fft.fftn(b))
    out = _sfft.ifftn(b, **kw) if _sfft else np.fft.ifftn(b)
    return out * float(np.prod(b.shape))


def _fold_index(N, n):
    """Fine-grid index k mod n of each mode k in I_N."""
    return params.mode_indices(N) % n


def _outer_factors(fs):
    """Tensor product of per-dimension factors, shaped (..., K2, K1)."""
    out = fs[0]
    for p in fs[1:]:
        out = np.multiply.outer(p, out)
    return out


def type1(pts, c, Ns, eps, iflag=-1, workers=None, sigma=params.SIGMA):
    """Approximate f_k = sum_j c_j exp(iflag i k.x_j) for k in I_N (Sec. II-A).

    Returns complex of shape (N2, N1) or (N3, N2, N1), k1 fastest."""
    P = Params(Ns, eps, sigma=sigma)
    workers = workers or direct.num_threads()
    b = direct.spread(pts, c, P.ns, P.w, P.beta)           # step 1
    bhat = _fft_signed(b, iflag, workers)                  # step 2
    idx = [_fold_index(N, n) for N, n in zip(P.Ns, P.ns)]  # step 3
    sub = bhat[np.ix_(*idx[::-1])]
    return _outer_factors(P.factors()) * sub


def type2(pts, f, eps, iflag=+1, workers=None, sigma=params.SIGMA):
    """Approximate c_j = sum_k f_k exp(iflag i k.x_j) (Sec. II-B).

    f: complex (N2, N1) or (N3, N2, N1), k1 fastest.  Returns complex (M,)."""
    f = np.asarray(f, dtype=np.complex128)
    Ns = f.shape[::-1]
    P = Params(Ns, eps, sigma=sigma)
    workers = workers or direct.num_threads()
    bhat = np.zeros(P.ns[::-1], dtype=np.complex128)       # step 1: precorrect
    idx = [_fold_index(N, n) for N, n in zip(P.Ns, P.ns)]  # and zero-pad
    bhat[np.ix_(*idx[::-1])] = _outer_factors(P.factors()) * f
    b = _fft_signed(bhat, iflag, workers)                  # step 2
    return direct.interp(pts, b, P.w, P.beta)              # step 3


def rel_l2(approx, exact):
    """Relative l2 error ||approx - exact|| / ||exact|| over all entries."""
    approx = np.asarray(approx).ravel()
    exact = np.asarray(exact).ravel()
    return float(np.linalg.norm(approx - exact) / np.linalg.norm(exact))
