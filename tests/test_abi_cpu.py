"""Host-side checks of the C ABI that need no GPU: the library loads and
exports every symbol the header declares, arguments are rejected before any
device call, and the host math (parameters, correction factors) agrees with
the oracle."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from oracle import params as oparams
from paper_2102_08463_amd import lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    txt = open(os.path.join(ROOT, "include", "mnufft.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+char\s*\*\s*|int\s+|int64_t\s+)(mnufft_\w+)\s*\(", txt, re.M)))


def test_exports_match_header():
    lib = L.load()
    names = _header_functions()
    assert set(names) == set(L.EXPORTS), names
    for n in names:
        assert hasattr(lib, n), n


def test_struct_layouts():
    # mnufft_opts: 7 ints + pointer + double + 6 reserved ints, natural alignment
    assert ctypes.sizeof(L.Opts) == 72
    assert L.Opts.stream.offset == 32
    assert L.Opts.upsampfac.offset == 40
    assert L.Opts.tune.offset == 48
    # mnufft_info ends with upsampfac (double) and ntargets (int64)
    assert L.Info.ntargets.offset == L.Info.upsampfac.offset + 8
    assert ctypes.sizeof(L.Info) == L.Info.ntargets.offset + 8


def test_default_opts_and_strerror():
    o = L.default_opts()
    assert o.method == L.METHOD_AUTO and o.device == -1 and o.msub == 0
    assert list(o.binsize) == [0, 0, 0] and not o.stream
    assert L.load().mnufft_default_opts(None) == L.ERR_ARG
    for code in (0, 1, -1, -2, -3, -4, -5, -6, -7, 99):
        assert isinstance(L.strerror(code), str)


def _makeplan(type_=1, dim=2, nm=(16, 16, 1), iflag=-1, ntr=1, eps=1e-6, prec=0, opts=None):
    h = ctypes.c_void_p(0)
    arr = (ctypes.c_int64 * 3)(*nm)
    rc = L.load().mnufft_makeplan(type_, dim, arr, iflag, ntr, eps, prec,
                                  ctypes.byref(opts) if opts is not None else None,
                                  ctypes.byref(h))
    return rc, h


@pytest.mark.parametrize("kw", [
    dict(type_=4), dict(type_=0), dict(type_=3, dim=4), dict(type_=3, eps=0.0),
    dict(type_=3, iflag=0), dict(type_=3, ntr=0), dict(dim=0), dict(type_=3, dim=0), dict(dim=4), dict(iflag=0), dict(iflag=2),
    dict(ntr=0), dict(eps=0.0), dict(eps=1.0), dict(eps=-1e-3), dict(eps=float("nan")),
    dict(prec=2), dict(nm=(0, 16, 1)), dict(nm=(16, -1, 1)), dict(dim=3, nm=(8, 8, 0)),
    dict(dim=1, nm=((1 << 24) + 1, 1, 1)),
])
def test_makeplan_rejects_bad_arguments(kw):
    rc, h = _makeplan(**kw)
    assert rc == L.ERR_ARG and not h.value


def test_makeplan_rejects_bad_opts():
    for field, val in (("method", 7), ("method", -1), ("msub", -5), ("device", -3)):
        o = L.default_opts()
        setattr(o, field, val)
        rc, h = _makeplan(opts=o)
        assert rc == L.ERR_ARG and not h.value, field
    o = L.default_opts()
    o.reserved[3] = 1
    assert _makeplan(opts=o)[0] == L.ERR_ARG
    o = L.default_opts()
    o.binsize[1] = -2
    assert _makeplan(opts=o)[0] == L.ERR_ARG
    # an explicit SM request whose padded bin cannot fit in LDS
    o = L.default_opts()
    o.method = L.METHOD_SM
    o.binsize[0], o.binsize[1], o.binsize[2] = 64, 64, 64
    assert _makeplan(dim=3, nm=(64, 64, 64), prec=1, opts=o)[0] == L.ERR_ARG


def test_null_plan_calls():
    lib = L.load()
    nul = ctypes.c_void_p(0)
    assert lib.mnufft_setpts(nul, 10, None, None, None) == L.ERR_ARG
    assert lib.mnufft_setpts3(nul, 10, None, None, None, 5, None, None, None) == L.ERR_ARG
    assert lib.mnufft_execute(nul, None, None) == L.ERR_ARG
    assert lib.mnufft_execute_adjoint(nul, None, None) == L.ERR_ARG
    assert lib.mnufft_spread(nul, None, None) == L.ERR_ARG
    assert lib.mnufft_interp(nul, None, None) == L.ERR_ARG
    assert lib.mnufft_get_sort(nul, None, None) == L.ERR_ARG
    assert lib.mnufft_get_subproblems(nul, None, None) == L.ERR_ARG
    assert lib.mnufft_get_info(nul, ctypes.byref(L.Info())) == L.ERR_ARG
    assert lib.mnufft_destroy(nul) == L.OK
    h = ctypes.c_void_p(0)
    assert lib.mnufft_makeplan(1, 2, None, -1, 1, 1e-6, 0, None, ctypes.byref(h)) == L.ERR_ARG
    arr = (ctypes.c_int64 * 3)(8, 8, 1)
    assert lib.mnufft_makeplan(1, 2, arr, -1, 1, 1e-6, 0, None, None) == L.ERR_ARG


@pytest.mark.parametrize("eps", [1e-1, 1e-2, 1e-5, 1e-6, 1e-7, 1e-9, 1e-12, 1e-15, 3e-4])
@pytest.mark.parametrize("N", [1, 7, 41, 64, 333, 1024])
def test_choose_params_match_oracle(eps, N):
    w, beta, n, rc = L.choose_params(eps, L.F64, N)
    assert w == oparams.kernel_width(eps)
    assert math.isclose(beta, oparams.kernel_beta(w))
    assert n == oparams.fine_grid_size(N, w)
    assert rc == L.OK
    w32, _, n32, rc32 = L.choose_params(eps, L.F32, N)
    assert w32 == min(w, 8)
    assert rc32 == (L.WARN_EPS_CLAMPED if w > 8 else L.OK)
    assert n32 == oparams.fine_grid_size(N, w32)


def test_choose_params_rejects():
    for args in ((0.0, 0, 8), (1.0, 0, 8), (1e-3, 2, 8), (1e-3, 0, 0), (1e-3, 0, 8, 1.2),
                 (1e-3, 0, 8, 2.5)):
        with pytest.raises(L.MnufftError):
            L.choose_params(*args)


@pytest.mark.parametrize("sigma", [1.25, 1.5, 2.0])
@pytest.mark.parametrize("eps", [1e-2, 1e-4, 1e-6, 1e-9, 1e-12])
@pytest.mark.parametrize("N", [1, 41, 64, 333])
def test_choose_params_sigma_match_oracle(sigma, eps, N):
    w, beta, n, rc = L.choose_params(eps, L.F64, N, sigma)
    wr = oparams.kernel_width(eps, sigma=sigma)
    assert w == wr
    assert math.isclose(beta, oparams.kernel_beta(w, sigma=sigma), rel_tol=1e-15)
    assert n == oparams.fine_grid_size(N, w, sigma=sigma)
    uncapped = oparams.kernel_width(eps, wmax=99, sigma=sigma)
    assert rc == (L.WARN_EPS_CLAMPED if uncapped > 16 else L.OK)
    w32, _, _, rc32 = L.choose_params(eps, L.F32, N, sigma)
    assert w32 == oparams.kernel_width(max(eps, 1e-7), sigma=sigma)
    assert rc32 == (L.WARN_EPS_CLAMPED if eps < 1e-7 or
                    oparams.kernel_width(max(eps, 1e-7), wmax=99, sigma=sigma) > 16 else L.OK)


@pytest.mark.parametrize("w", [2, 3, 6, 7, 9, 13, 16])
@pytest.mark.parametrize("N,n", [(64, 128), (41, 90), (333, 675), (1, 32)])
def test_correction_factors_match_oracle(w, N, n):
    """The library's tanh-sinh factors against the oracle's Gauss-Legendre ones."""
    beta = oparams.kernel_beta(w)
    got = np.array(L.correction_factors(N, n, w, beta))
    ref = oparams.correction_factors(N, n, w, beta)
    assert np.allclose(got, ref, rtol=1e-12, atol=0)


def test_correction_factors_reject():
    for args in ((0, 8, 6, 13.8), (8, 8, 6, 13.8), (8, 16, 1, 13.8), (8, 16, 17, 13.8),
                 (8, 16, 6, 0.0)):
        with pytest.raises(L.MnufftError):
            L.correction_factors(*args)


def test_batch_makeplan_rejects_bad_arguments():
    lib = L.load()

    def mk(type_=1, dim=2, ntr=2, nm=(8, 8, 1, 9, 7, 1), npts=(10, 20), iflag=-1, eps=1e-5,
           prec=0, bs=None, ms=None, opts=None):
        h = ctypes.c_void_p(0)
        nma = (ctypes.c_int64 * len(nm))(*nm)
        npa = (ctypes.c_int64 * len(npts))(*npts)
        bsa = (ctypes.c_int32 * len(bs))(*bs) if bs else None
        msa = (ctypes.c_int32 * len(ms))(*ms) if ms else None
        rc = lib.mnufft_batch_makeplan(type_, dim, ntr, nma, npa, iflag, eps, prec, bsa, msa,
                                       ctypes.byref(opts) if opts else None, ctypes.byref(h))
        return rc, h

    for kw in (dict(type_=3), dict(dim=1), dict(ntr=0), dict(iflag=0), dict(eps=1.5),
               dict(prec=7), dict(nm=(0, 8, 1, 9, 7, 1)), dict(npts=(-1, 5)),
               dict(bs=(8, -8, 1, 8, 8, 1)), dict(ms=(10, -1))):
        rc, h = mk(**kw)
        assert rc == L.ERR_ARG and not h.value, kw
    o = L.default_opts()
    o.method = L.METHOD_GMSORT
    assert mk(opts=o)[0] == L.ERR_UNSUPPORTED
    assert lib.mnufft_batch_destroy(ctypes.c_void_p(0)) == L.OK
    assert lib.mnufft_batch_setpts(ctypes.c_void_p(0), None, None, None) == L.ERR_ARG
    assert lib.mnufft_batch_execute(ctypes.c_void_p(0), None, None) == L.ERR_ARG


def test_type3_grid_matches_oracle():
    """The library's type 3 grid rule (host helper used by mnufft_setpts3)
    against the oracle's type3_params on the same half-widths."""
    from oracle import nufft as onufft
    lib = L.load()
    R = np.random.default_rng(5)
    nf = ctypes.c_int64(0)
    gam = ctypes.c_double(0.0)
    cases = [(math.pi, 512.0), (0.0, 3.0), (2.5, 0.0), (0.0, 0.0), (40.0, 1.5), (1e-3, 7e4)]
    cases += [(float(R.uniform(0, 50)), float(R.uniform(0, 300))) for _ in range(40)]
    for X, S in cases:
        for sigma in (2.0, 1.5, 1.25):
            for w in (2, 6, 13, 16):
                assert lib.mnufft_type3_grid(X, S, sigma, w, ctypes.byref(nf), ctypes.byref(gam)) == L.OK
                # one dimension with points on [C - X, C + X], frequencies on [D - S, D + S]
                pts, frq = (np.array([1.0 - X, 1.0 + X]),), (np.array([-2.0 - S, -2.0 + S]),)
                C, D, g, h, n = onufft.type3_params(pts, frq, w, sigma)[0]
                assert nf.value == n, (X, S, sigma, w)
                assert gam.value == pytest.approx(g, rel=1e-15)


def test_type3_grid_rejects():
    lib = L.load()
    nf = ctypes.c_int64(0)
    gam = ctypes.c_double(0.0)
    for args in ((-1.0, 1.0, 2.0, 6), (1.0, -1.0, 2.0, 6), (float("nan"), 1.0, 2.0, 6),
                 (1.0, 1.0, 1.0, 6), (1.0, 1.0, 2.0, 1), (1.0, 1.0, 2.0, 17), (1e6, 1e6, 2.0, 6)):
        assert lib.mnufft_type3_grid(*args, ctypes.byref(nf), ctypes.byref(gam)) == L.ERR_ARG, args


@pytest.mark.parametrize("dim,prec,eps", [(2, 0, 1e-6), (2, 1, 1e-12), (3, 0, 1e-5), (3, 1, 1e-9)])
def test_tune_candidates_fixed_order_and_lds_fit(dim, prec, eps):
    """The autotuner's candidate list (host only): SM bin shapes x msub in a
    fixed order, each within the 160 KB of LDS per workgroup, then GM-sort
    and GM; msub values from {256, 1024, 4096, 16384}."""
    lib = L.load()
    cands = L.tune_candidates(dim, prec, eps)
    assert len(cands) == lib.mnufft_tune_candidates(dim, prec, eps, None, 0)
    methods = [o.method for o in cands]
    assert methods[-2:] == [L.METHOD_GMSORT, L.METHOD_GM]
    assert all(m == L.METHOD_SM for m in methods[:-2]) and len(methods) > 2
    w = oparams.kernel_width(eps, wmax=8 if prec == 0 else 16)
    P = (w + 1) // 2
    seen = set()
    for o in cands[:-2]:
        m = [o.binsize[d] for d in range(dim)]
        assert o.msub in (256, 1024, 4096, 16384)
        cells = int(np.prod([mi + 2 * P for mi in m]))
        rs = 4 if prec == 0 else 8
        # interpolation stages the padded bin as complex values; spreading needs at most
        # two 64-bit words per cell plus (single precision) a staging area of strengths
        assert cells * 2 * rs <= 160 * 1024
        key = (tuple(m), o.msub)
        assert key not in seen
        seen.add(key)
    # the same list on every call
    assert [L.describe(o) for o in L.tune_candidates(dim, prec, eps)] == \
        [L.describe(o) for o in cands]


@pytest.mark.parametrize("field", ["binsize", "msub", "method", "type3", "dim1", "bad"])
def test_makeplan_rejects_tune_with_fixed_parameters(field):
    """opts.tune picks method, bins and msub itself (types 1 / 2, 2D / 3D):
    combined with fixed ones, or out of range, makeplan refuses before any
    device call."""
    lib = L.load()
    o = L.default_opts()
    o.tune = L.TUNE_LEARNED
    typ, dim = 1, 2
    if field == "binsize":
        o.binsize[0] = 32
    elif field == "msub":
        o.msub = 1024
    elif field == "method":
        o.method = L.METHOD_SM
    elif field == "type3":
        typ = 3
    elif field == "dim1":
        dim = 1
    else:
        o.tune = 7
    nm = (ctypes.c_int64 * 3)(64, 64, 1)
    h = ctypes.c_void_p(0)
    assert lib.mnufft_makeplan(typ, dim, nm, -1, 1, 1e-6, L.F32, ctypes.byref(o),
                               ctypes.byref(h)) == L.ERR_ARG
    assert not h.value


def _selector_file(path, dim=2, prec=0, eps=1e-6, H=8, margin=0.0, recs=None, extra=b""):
    cands = L.tune_candidates(dim, prec, eps)
    K = len(cands)
    if recs is None:
        recs = [[o.method, o.binsize[0], o.binsize[1], o.binsize[2], o.msub] for o in cands]
    n = int(L.load().mnufft_mlp_nparams(262, H, K))
    with open(path, "wb") as fh:
        fh.write(b"MNSEL001" + np.array([dim, prec], np.int32).tobytes() +
                 np.array([eps], np.float64).tobytes() + np.array([262, H, K], np.int32).tobytes() +
                 np.array([margin], np.float64).tobytes() + np.array(recs, np.int32).tobytes() +
                 np.zeros(n, np.float32).tobytes() + extra)


def test_selector_load_format(tmp_path):
    """mnufft_selector_load (host only) takes a well-formed file and refuses a
    missing file, a wrong magic, a candidate list that is not the
    autotuner's, and trailing bytes."""
    lib = L.load()
    good = tmp_path / "good.bin"
    _selector_file(good)
    assert lib.mnufft_selector_load(str(good).encode()) == L.OK
    assert lib.mnufft_selector_load(str(tmp_path / "missing.bin").encode()) == L.ERR_ARG
    bad = tmp_path / "magic.bin"
    bad.write_bytes(b"MNSELxxx" + good.read_bytes()[8:])
    assert lib.mnufft_selector_load(str(bad).encode()) == L.ERR_ARG
    cands = L.tune_candidates(2, 0, 1e-6)
    recs = [[o.method, o.binsize[0], o.binsize[1], o.binsize[2], o.msub] for o in cands][::-1]
    _selector_file(tmp_path / "order.bin", recs=recs)
    assert lib.mnufft_selector_load(str(tmp_path / "order.bin").encode()) == L.ERR_ARG
    _selector_file(tmp_path / "extra.bin", extra=b"\0")
    assert lib.mnufft_selector_load(str(tmp_path / "extra.bin").encode()) == L.ERR_ARG
    assert lib.mnufft_selector_clear() == L.OK
