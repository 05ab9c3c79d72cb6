"""The three-step type 1 / type 2 algorithm of Sec. II in plain FP64, and
type 3 built from it.

Part of the oracle (test infrastructure; see ``oracle/__init__.py``).

Type 1 (Sec. II-A): spread onto the fine grid, FFT, truncate to the central
modes and multiply by the correction factors.  Type 2 (Sec. II-B): the same
steps transposed: precorrect and zero-pad, FFT of the opposite role,
interpolate.  The sign of the exponent (iflag) is a free parameter; the FFT
carries that sign and no 1/n normalisation is applied anywhere.

Type 3 (nonuniform points to nonuniform frequencies) is only named in
Sec. I-B and Sec. VI as beyond the paper; ``type3`` follows the published
type 3 method of the FINUFFT paper (Barnett, Magland, af Klinteberg, SIAM J.
Sci. Comput. 2019): shift and rescale, spread onto a grid with no
upsampling of its own, a type 2 at the rescaled frequencies, divide by the
kernel's Fourier transform.  The readings it takes are listed in
``type3_params``.
"""
import math

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


def _smooth_even(n):
    """Smallest even 2^q 3^p 5^r >= n."""
    n = max(int(n), 2)
    n += n % 2
    while not params.is_5smooth(n):
        n += 2
    return n


def type3_params(pts, freqs, w, sigma=params.SIGMA):
    """Per dimension (C, D, gamma, h, nf) of the type 3 reduction.

    C, X: centre and half-width of the points; D, S: the same of the
    frequencies.  With x' = x - C and s' = s - D, the points are rescaled to
    x'/gamma and spread onto nf cells of spacing h = 2 pi / nf; the type 2
    then needs the frequencies h gamma s'.  gamma = nf / (2 sigma S) puts the
    largest |gamma s'| at nf / (2 sigma), the role N/2 plays in type 1, so the
    kernel's aliasing error is that of type 1 with the same w and beta.  The
    points must keep all w taps inside the grid without wrapping, which holds
    when nf >= 2 sigma S X / pi + w; one cell more is taken for rounding.

    Readings (the paper gives none of this): nf is the smallest even
    5-smooth integer >= max(ceil(2 sigma S X / pi) + w + 1, 2w); when S = 0
    (all frequencies equal in a dimension) S is replaced by 1/X (by 1 when X
    is 0 too), which leaves that dimension's result to the phase factors."""
    out = []
    for x, s in zip(pts, freqs):
        x = np.asarray(x, dtype=np.float64)
        s = np.asarray(s, dtype=np.float64)
        xl, xh = (float(x.min()), float(x.max())) if x.size else (0.0, 0.0)
        sl, sh = (float(s.min()), float(s.max())) if s.size else (0.0, 0.0)
        C, X = 0.5 * (xh + xl), 0.5 * (xh - xl)
        D, S = 0.5 * (sh + sl), 0.5 * (sh - sl)
        if S == 0.0:
            S = 1.0 / X if X > 0.0 else 1.0
        nf = _smooth_even(max(math.ceil(2.0 * sigma * S * X / math.pi) + w + 1, 2 * w))
        gamma = nf / (2.0 * sigma * S)
        out.append((C, D, gamma, 2.0 * math.pi / nf, nf))
    return out


def type3(pts, c, freqs, eps, iflag=-1, sigma=params.SIGMA, workers=None):
    """Approximate f_k = sum_j c_j exp(iflag i s_k.x_j) at real frequencies s_k.

    Steps: (1) pre-phase c'_j = c_j exp(iflag i D.(x_j - C)); (2) spread c'
    at the points (x_j - C)/gamma onto nf^d cells (Sec. II-A step 1 with no
    upsampling: the grid itself is what the type 2 upsamples); (3) type 2
    (Sec. II-B) of the grid, as modes -nf/2 .. nf/2 - 1, at the frequencies
    t_k = h gamma (s_k - D); (4) multiply by exp(iflag i s_k.C) and, per
    dimension, (2/w) / phi_hat(w t_k / 2) (the spacing h over the transform
    of the kernel phi(t / alpha), alpha = w h / 2).  Returns complex (K,)."""
    dim = len(pts)
    w = params.kernel_width(eps, sigma=sigma)
    beta = params.kernel_beta(w, sigma=sigma)
    tp = type3_params(pts, freqs, w, sigma)
    x = [np.asarray(a, dtype=np.float64) for a in pts]
    s = [np.asarray(a, dtype=np.float64) for a in freqs]
    pre = sum(D * (xd - C) for (C, D, _, _, _), xd in zip(tp, x))
    c1 = np.asarray(c, dtype=np.complex128) * np.exp(1j * iflag * pre)       # step 1
    xr = tuple((xd - C) / g for (C, _, g, _, _), xd in zip(tp, x))
    b = direct.spread(xr, c1, [nf for *_, nf in tp], w, beta)                 # step 2
    tt = tuple(h * g * (sd - D) for (_, D, g, h, _), sd in zip(tp, s))
    inner = type2(tt, b, eps, iflag=iflag, workers=workers, sigma=sigma)      # step 3
    post = np.exp(1j * iflag * sum(C * sd for (C, *_), sd in zip(tp, s)))    # step 4
    for td in tt:
        post = post * ((2.0 / w) / params.es_fourier(0.5 * w * td, beta))
    return post * inner


def rel_l2(approx, exact):
    """Relative l2 error ||approx - exact|| / ||exact|| over all entries."""
    approx = np.asarray(approx).ravel()
    exact = np.asarray(exact).ravel()
    return float(np.linalg.norm(approx - exact) / np.linalg.norm(exact))
