"""Parameter choices and kernel transforms of the method (Sec. II), in FP64.

Part of the oracle (test infrastructure; see ``oracle/__init__.py``).
"""
import math

import numpy as np

SIGMA = 2  # upsampling factor, fixed to 2 in Sec. II


def kernel_width(eps, wmax=16, sigma=SIGMA):
    """Kernel width w = ceil(log10(1/eps)) + 1 (Sec. II, upsampling 2).

    Reading: 1e-9 is subtracted before the ceiling so that decade tolerances
    (whose logarithm is not exactly an integer in floating point) give the
    intended width; w is clamped to [2, wmax].
    Upsampling sigma < 2 is only named as future work (Sec. VI); for it the
    published rule of the FINUFFT paper (Barnett, Magland, af Klinteberg,
    SISC 2019) is read in: w = ceil(ln(1/eps) / (pi sqrt(1 - 1/sigma))).
    """
    if not (0.0 < eps < 1.0):
        raise ValueError("eps must lie in (0, 1)")
    if sigma == SIGMA:
        w = int(math.ceil(math.log10(1.0 / eps) - 1e-9)) + 1
    else:
        w = int(math.ceil(math.log(1.0 / eps) / (math.pi * math.sqrt(1.0 - 1.0 / sigma)) - 1e-9))
    return max(2, min(wmax, w))


def kernel_beta(w, sigma=SIGMA):
    """Shape parameter beta = 2.30 w of the ES kernel (Sec. II); for sigma < 2
    the same paper's beta = 0.97 pi w (1 - 1/(2 sigma))."""
    if sigma == SIGMA:
        return 2.30 * w
    return 0.97 * math.pi * w * (1.0 - 0.5 / sigma)


def is_5smooth(n):
    """True when n = 2^q 3^p 5^r."""
    if n < 1:
        return False
    for p in (2, 3, 5):
        while n % p == 0:
            n //= p
    return n == 1


def fine_grid_size(N, w, sigma=SIGMA):
    """Smallest 2^q 3^p 5^r that is >= max(sigma N, 2w) (Sec. II; sigma N
    rounded up)."""
    n = max(int(math.ceil(sigma * int(N) - 1e-9)), 2 * int(w))
    while not is_5smooth(n):
        n += 1
    return n


def es_kernel(z, beta):
    """ES kernel phi_beta(z) = exp(beta (sqrt(1 - z^2) - 1)) on |z| <= 1 (eq. es)."""
    z = np.asarray(z, dtype=np.float64)
    out = np.zeros_like(z)
    m = np.abs(z) <= 1.0
    out[m] = np.exp(beta * (np.sqrt(1.0 - z[m] ** 2) - 1.0))
    return out


_GL_CACHE = {}


def _gauss_legendre(q):
    if q not in _GL_CACHE:
        _GL_CACHE[q] = np.polynomial.legendre.leggauss(q)
    return _GL_CACHE[q]


def es_fourier(xi, beta, nodes=200):
    """phi_hat(xi) = int_{-1}^{1} phi_beta(z) exp(-i xi z) dz (the transform
    convention of Sec. II).  phi_beta is even, so this is
    2 int_0^1 phi(z) cos(xi z) dz; the substitution z = sin(theta) removes the
    square-root endpoint behaviour of phi, leaving the smooth integrand
    2 exp(beta (cos theta - 1)) cos(xi sin theta) cos theta on [0, pi/2],
    integrated by a `nodes`-point Gauss-Legendre rule."""
    t, wq = _gauss_legendre(nodes)
    th = (t + 1.0) * (np.pi / 4.0)
    wq = wq * (np.pi / 4.0)
    base = wq * np.exp(beta * (np.cos(th) - 1.0)) * np.cos(th)
    xi = np.asarray(xi, dtype=np.float64)
    return 2.0 * (base * np.cos(np.multiply.outer(xi, np.sin(th)))).sum(axis=-1)


def mode_indices(N):
    """The frequency set I_N = {k integer : -N/2 <= k < N/2} in ascending order (eq. I)."""
    return np.arange(-(N // 2), N - N // 2, dtype=np.int64)


def correction_factors(N, n, w, beta):
    """Per-dimension factors of Sec. II-A step 3, including the lattice phase.

    p_k = (2/w) / phi_hat(alpha k) with alpha = w pi / n, for k in I_N; the
    product over dimensions is the paper's p_{k1,k2}.  Because this oracle puts
    fine-grid point l at l h - pi (the lattice used for binning in Sec. III-A)
    rather than at l h, each factor also carries exp(-s i k pi) = (-1)^k, which
    does not depend on the sign s.
    """
    k = mode_indices(N)
    alpha = w * math.pi / n
    p = (2.0 / w) / es_fourier(alpha * k, beta)
    return p * np.where(k % 2 == 0, 1.0, -1.0)


def density(M, Ns, sigma=SIGMA):
    """Problem density rho = M / (sigma^d prod N_i) (eq. den)."""
    return M / float(np.prod([sigma * int(N) for N in Ns]))


def sm_tile_bytes(m, w, bytes_per_cell=16):
    """Shared-memory bytes of a padded bin bounded as bytes_per_cell * prod(m_i + w)
    (second remark of Sec. III-A) and the bin-to-padded-bin volume ratio."""
    vol = 1
    padded = 1
    for mi in m:
        vol *= mi
        padded *= mi + w
    return bytes_per_cell * padded, vol / padded
