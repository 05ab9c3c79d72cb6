// Host side of libmnufft: plan construction, parameter choice, correction
// factors, the rocFFT fine-grid transform and the C ABI declared in
// include/mnufft.h.  The stages follow the paper's plan / setup / execute /
// destroy interface (Sec. I-A) and three-step algorithm (Sec. II); every
// step on the device runs in the kernels of kernels_*.hip except the FFT.
#include "../../include/mnufft.h"
#include "host_common.h"
#include "internal.h"

#include <rocfft/rocfft.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

namespace {

constexpr double kPi = mn::host::kPi;
constexpr size_t kLdsMax = 160 * 1024;  // LDS per workgroup on gfx950
constexpr int kMergeGroup = 32;         // tiles summed per leader in heavy bins

using mn::host::bits_for;
using mn::host::correction;
using mn::host::fine_size;
using mn::host::width_for_eps;
using mn::host::StageTimer;

std::once_flag g_fft_once;
rocfft_status g_fft_setup = rocfft_status_success;

}  // namespace

struct mnufft_plan_s {
    int type = 1, dim = 2, prec = 0, iflag = -1;
    int64_t N[3] = {1, 1, 1};
    int64_t ntransf = 1;
    double eps = 1e-6;
    double sigma = 2.0;  // upsampling factor
    mn::Geom g{};
    int method = MNUFFT_METHOD_SM;
    int msub = 1024;
    int device = -1;
    int validate = 0;
    hipStream_t stream = nullptr;
    size_t rsz = 4;             // bytes per real of the plan precision
    size_t grid_elems = 0;      // complex cells per transform
    void *grid = nullptr;       // ntransf fine grids
    void *pfac[3] = {nullptr, nullptr, nullptr};
    // points
    int64_t M = -1;
    int64_t Mcap = -1;
    void *su[3] = {nullptr, nullptr, nullptr};
    void *su_in[3] = {nullptr, nullptr, nullptr};
    void *su_tmp[3] = {nullptr, nullptr, nullptr};
    uint32_t *keyA = nullptr, *valA = nullptr, *keyB = nullptr, *valB = nullptr;
    uint32_t *key_in = nullptr;
    uint32_t *skey = nullptr;   // alias of keyA/keyB after the sort
    int32_t *perm = nullptr;    // alias of valA/valB after the sort
    // method SM: the sorted points in the kernels' processing order (see
    // k_balance): coordinates, permutation and sorted position
    void *su_proc[3] = {nullptr, nullptr, nullptr};
    int32_t *perm_proc = nullptr, *spos_proc = nullptr;
    uint16_t *hslot_proc = nullptr;
    int32_t *binstart = nullptr, *subcount = nullptr, *sub = nullptr, *nsub = nullptr;
    int nsub_max = 0, nsub_cap = 0;
    uint32_t *hist = nullptr, *partials = nullptr;
    size_t hist_cap = 0, partials_cap = 0;
    int *flag = nullptr;
    // SM spreading: tile slots, merge list and cover tables
    void *scratch = nullptr;
    size_t scratch_bytes = 0;
    int ts2 = 0;
    int32_t *mergelist = nullptr, *nmerge = nullptr;
    int2 *cov[3] = {nullptr, nullptr, nullptr};
    void *cmax = nullptr;
    size_t cov_bytes[3] = {0, 0, 0};
    int kmax[3] = {1, 1, 1};
    // FFT
    rocfft_plan fft[2] = {nullptr, nullptr};  // [0]: exponent sign -1, [1]: +1
    rocfft_execution_info fftinfo = nullptr;
    void *fftwork = nullptr;
    size_t fftwork_bytes = 0;
    int64_t devbytes = 0;
    mn::host::Timers tm;  // stage timers
    // type 3: a spreading plan on the rescaled points (grid = the inner
    // transform's modes) and a type 2 plan at the rescaled frequencies
    mnufft_opts opts{};
    mnufft_plan t3spr = nullptr, t3inner = nullptr;
    int64_t K = -1;                    // frequencies of the last setpts
    int64_t t3Mcap = -1, t3Kcap = -1;
    void *t3pre = nullptr, *t3post = nullptr, *t3cp = nullptr;
    mn::PtMap ptmap{};                 // map applied before binning (type 3 sub-plans)
    double *t3part = nullptr;          // bounds partials, 2 x 1024 blocks x 3 dims x 3
    double *t3quad = nullptr;          // ximax and the Chebyshev terms of log phi_hat
    int t3nq = 0;
    double C[3] = {0, 0, 0}, D[3] = {0, 0, 0}, gam[3] = {1, 1, 1}, hstep[3] = {1, 1, 1};
    int64_t nf3[3] = {1, 1, 1};
};

namespace {

#define MN_HIP(call)                                                  \
    do {                                                              \
        hipError_t e_ = (call);                                       \
        if (e_ != hipSuccess) return e_ == hipErrorOutOfMemory ? MNUFFT_ERR_ALLOC : MNUFFT_ERR_HIP; \
    } while (0)

int dalloc(mnufft_plan p, void **ptr, size_t bytes)
{
    *ptr = nullptr;
    if (bytes == 0) return MNUFFT_OK;
    hipError_t e = hipMalloc(ptr, bytes);
    if (e != hipSuccess) {
        *ptr = nullptr;
        (void)hipGetLastError();
        return e == hipErrorOutOfMemory ? MNUFFT_ERR_ALLOC : MNUFFT_ERR_HIP;
    }
    p->devbytes += (int64_t)bytes;
    return MNUFFT_OK;
}

void dfree(mnufft_plan p, void **ptr, size_t bytes)
{
    if (*ptr) {
        (void)hipFree(*ptr);
        p->devbytes -= (int64_t)bytes;
    }
    *ptr = nullptr;
}

int use_device(mnufft_plan p)
{
    if (p->device >= 0) MN_HIP(hipSetDevice(p->device));
    return MNUFFT_OK;
}

void free_points(mnufft_plan p)
{
    if (p->Mcap < 0) return;
    const size_t M = (size_t)std::max<int64_t>(p->Mcap, 1);
    for (int d = 0; d < 3; ++d) {
        dfree(p, &p->su[d], M * p->rsz);
        dfree(p, &p->su_in[d], M * p->rsz);
        dfree(p, &p->su_tmp[d], M * p->rsz);
    }
    dfree(p, (void **)&p->keyA, M * 4);
    dfree(p, (void **)&p->valA, M * 4);
    dfree(p, (void **)&p->keyB, M * 4);
    dfree(p, (void **)&p->valB, M * 4);
    dfree(p, (void **)&p->key_in, M * 4);
    for (int d = 0; d < 3; ++d) dfree(p, &p->su_proc[d], M * p->rsz);
    dfree(p, (void **)&p->perm_proc, M * 4);
    dfree(p, (void **)&p->spos_proc, M * 4);
    dfree(p, (void **)&p->hslot_proc, M * 2);
    dfree(p, (void **)&p->sub, (size_t)p->nsub_cap * 16);
    dfree(p, (void **)&p->hist, p->hist_cap * 4);
    dfree(p, (void **)&p->partials, p->partials_cap * 4);
    dfree(p, &p->scratch, p->scratch_bytes);
    dfree(p, (void **)&p->mergelist, (size_t)p->nsub_cap * 4);
    p->scratch_bytes = 0;
    p->Mcap = -1;
    p->nsub_cap = 0;
    p->hist_cap = 0;
    p->partials_cap = 0;
}

// SM plans in 2D and 3D process each subproblem's points in the bank-
// balanced order of k_balance (kept in the *_proc arrays); 1D tiles are a
// single row, where the sorted order does as well.
bool balanced(const mnufft_plan_s *p) { return p->method == MNUFFT_METHOD_SM && p->dim >= 2; }

int alloc_points(mnufft_plan p, int64_t M)
{
    free_points(p);
    const size_t Ma = (size_t)std::max<int64_t>(M, 1);
    int rc;
    for (int d = 0; d < p->dim; ++d) {
        if ((rc = dalloc(p, &p->su[d], Ma * p->rsz))) return rc;
        if ((rc = dalloc(p, &p->su_tmp[d], Ma * p->rsz))) return rc;
        if (p->method == MNUFFT_METHOD_GM && (rc = dalloc(p, &p->su_in[d], Ma * p->rsz))) return rc;
    }
    if ((rc = dalloc(p, (void **)&p->keyA, Ma * 4))) return rc;
    if ((rc = dalloc(p, (void **)&p->valA, Ma * 4))) return rc;
    if ((rc = dalloc(p, (void **)&p->keyB, Ma * 4))) return rc;
    if ((rc = dalloc(p, (void **)&p->valB, Ma * 4))) return rc;
    if (p->method == MNUFFT_METHOD_GM && (rc = dalloc(p, (void **)&p->key_in, Ma * 4))) return rc;
    p->nsub_cap = (int)(p->g.nbins + (M + p->msub - 1) / p->msub);
    if ((rc = dalloc(p, (void **)&p->sub, (size_t)std::max(p->nsub_cap, 1) * 16))) return rc;
    if (p->method == MNUFFT_METHOD_SM) {
        // (spos_proc: each processed point's sorted position, the identity
        // without balancing, for execute_sorted)
        if ((rc = dalloc(p, (void **)&p->spos_proc, Ma * 4))) return rc;
        if (balanced(p)) {
            for (int d = 0; d < p->dim; ++d)
                if ((rc = dalloc(p, &p->su_proc[d], Ma * p->rsz))) return rc;
            if ((rc = dalloc(p, (void **)&p->perm_proc, Ma * 4))) return rc;
            if ((rc = dalloc(p, (void **)&p->hslot_proc, Ma * 2))) return rc;
        }
        p->scratch_bytes = (size_t)std::max(p->nsub_cap, 1) * p->ts2 * p->rsz;
        if ((rc = dalloc(p, &p->scratch, p->scratch_bytes))) return rc;
        if ((rc = dalloc(p, (void **)&p->mergelist, (size_t)std::max(p->nsub_cap, 1) * 4)))
            return rc;
    }
    p->hist_cap = mn::radix_hist_elems((int)M);
    if ((rc = dalloc(p, (void **)&p->hist, p->hist_cap * 4))) return rc;
    p->partials_cap = std::max(mn::scan_partial_elems(p->hist_cap),
                               mn::scan_partial_elems((size_t)p->g.nbins + 1));
    if ((rc = dalloc(p, (void **)&p->partials, p->partials_cap * 4))) return rc;
    p->Mcap = M;
    return MNUFFT_OK;
}

int make_fft(mnufft_plan p, int which)
{
    if (p->fft[which]) return MNUFFT_OK;
    size_t len[3];
    for (int d = 0; d < p->dim; ++d) len[d] = (size_t)p->g.n[d];  // first dimension fastest
    rocfft_status st = rocfft_plan_create(
        &p->fft[which], rocfft_placement_inplace,
        which == 0 ? rocfft_transform_type_complex_forward : rocfft_transform_type_complex_inverse,
        p->prec == MNUFFT_F32 ? rocfft_precision_single : rocfft_precision_double,
        (size_t)p->dim, len, (size_t)p->ntransf, nullptr);
    if (st != rocfft_status_success) {
        p->fft[which] = nullptr;
        return MNUFFT_ERR_FFT;
    }
    size_t wb = 0;
    if (rocfft_plan_get_work_buffer_size(p->fft[which], &wb) != rocfft_status_success)
        return MNUFFT_ERR_FFT;
    if (wb > p->fftwork_bytes) {
        dfree(p, &p->fftwork, p->fftwork_bytes);
        p->fftwork_bytes = 0;
        int rc = dalloc(p, &p->fftwork, wb);
        if (rc) return rc;
        p->fftwork_bytes = wb;
    }
    return MNUFFT_OK;
}

// In-place unnormalised FFT of all ntransf grids with exponent sign `sign`.
int run_fft(mnufft_plan p, int sign)
{
    const int which = sign < 0 ? 0 : 1;
    int rc = make_fft(p, which);
    if (rc) return rc;
    if (rocfft_execution_info_set_stream(p->fftinfo, p->stream) != rocfft_status_success)
        return MNUFFT_ERR_FFT;
    if (p->fftwork_bytes &&
        rocfft_execution_info_set_work_buffer(p->fftinfo, p->fftwork, p->fftwork_bytes) !=
            rocfft_status_success)
        return MNUFFT_ERR_FFT;
    void *buf[1] = {p->grid};
    if (rocfft_execute(p->fft[which], buf, nullptr, p->fftinfo) != rocfft_status_success)
        return MNUFFT_ERR_FFT;
    return MNUFFT_OK;
}

mn::Pts points_of(mnufft_plan p)
{
    mn::Pts P{};
    P.M = (int)p->M;
    for (int d = 0; d < 3; ++d) {
        P.u[d] = p->su[d];
        P.u_in[d] = p->su_in[d];
    }
    P.key = p->skey;
    P.perm = p->perm;
    P.spos = nullptr;
    P.binstart = p->binstart;
    P.sub = p->sub;
    P.nsub = p->nsub;
    P.nsub_max = p->nsub_max;
    P.key_in = p->key_in;
    P.suboff = p->subcount;
    P.scratch = p->scratch;
    P.ts2 = p->ts2;
    P.G = kMergeGroup;
    P.mergelist = p->mergelist;
    P.nmerge = p->nmerge;
    // the heavy-bin list of the add-back follows the nbins + 1 subproblem offsets
    P.heavy = p->method == MNUFFT_METHOD_SM ? p->subcount + p->g.nbins + 1 : nullptr;
    P.cmax = p->cmax;
    P.msub = p->msub;
    P.tg = nullptr;
    P.T = 1;
    P.ncells = (long long)p->grid_elems;
    for (int d = 0; d < 3; ++d) {
        P.cov[d] = p->cov[d];
        P.kmax[d] = p->kmax[d];
    }
    return P;
}

// The points as the SM spreading / interpolation kernels take them: in their
// processing order (k_balance); other methods use the sorted order.  With
// `sorted`, the vectors are in bin-sorted order and are reached through the
// points' sorted positions.
mn::Pts kernel_points(mnufft_plan p, bool sorted)
{
    mn::Pts P = points_of(p);
    if (balanced(p)) {
        for (int d = 0; d < 3; ++d) P.u[d] = p->su_proc[d];
        P.perm = p->perm_proc;
        P.hslot = p->hslot_proc;
    }
    if (sorted && p->method == MNUFFT_METHOD_SM) P.spos = p->spos_proc;
    if (sorted) P.perm = nullptr;
    return P;
}

size_t grid_bytes(mnufft_plan p) { return p->grid_elems * 2 * p->rsz; }

// SM spreading with the two-word accumulator (double precision, and single
// precision in 1D) needs max |c| before the tile kernel.
bool needs_cmax(mnufft_plan p) { return p->prec == MNUFFT_F64 || p->dim == 1; }

// Step 1 of type 1 for all ntransf vectors: c (ntransf x M) -> p->grid; c in
// bin-sorted order when `sorted`.
int spread_all(mnufft_plan p, const void *c, bool sorted = false)
{
    mn::Pts P = kernel_points(p, sorted);
    if (p->method != MNUFFT_METHOD_SM) {  // SM writes every cell itself
        StageTimer tm(p->tm, MNUFFT_STAGE_ZERO, p->stream);
        MN_HIP(mn::launch_zero(p->grid, grid_bytes(p) * p->ntransf, p->stream));
    }
    for (int64_t t = 0; t < p->ntransf; ++t) {
        const char *ct = (const char *)c + (size_t)t * p->M * 2 * p->rsz;
        char *gt = (char *)p->grid + (size_t)t * grid_bytes(p);
        if (p->method == MNUFFT_METHOD_SM && needs_cmax(p)) {
            // max |c| for the two-word fixed-point scale (2D / 3D single
            // precision scales each subproblem inside the spreading kernel)
            StageTimer tm(p->tm, MNUFFT_STAGE_SCALE, p->stream);
            MN_HIP(mn::launch_zero(p->cmax, 1024 * 8, p->stream));
            MN_HIP(mn::launch_spread(p->g, p->prec, p->method, P, ct, gt, p->stream, 4));
        }
        {
            StageTimer tm(p->tm, MNUFFT_STAGE_SPREAD, p->stream);
            MN_HIP(mn::launch_spread(p->g, p->prec, p->method, P, ct, gt, p->stream, 1));
        }
        if (p->method == MNUFFT_METHOD_SM) {
            StageTimer tm(p->tm, MNUFFT_STAGE_ADDBACK, p->stream);
            MN_HIP(mn::launch_spread(p->g, p->prec, p->method, P, ct, gt, p->stream, 2));
        }
    }
    return MNUFFT_OK;
}

// Type 1 with exponent sign `sign`: c (ntransf x M) -> f (ntransf x N).
int exec_type1(mnufft_plan p, int sign, const void *c, void *f, bool sorted = false)
{
    int rc = spread_all(p, c, sorted);
    if (rc) return rc;
    {
        StageTimer tm(p->tm, MNUFFT_STAGE_FFT, p->stream);
        rc = run_fft(p, sign);
    }
    if (rc) return rc;
    StageTimer tm(p->tm, MNUFFT_STAGE_DECONV, p->stream);
    MN_HIP(mn::launch_deconv(p->dim, p->N, p->g.n, p->prec, (int)p->ntransf, p->grid,
                             p->pfac, f, p->stream));
    return MNUFFT_OK;
}

// Type 2 with exponent sign `sign`: f (ntransf x N) -> c (ntransf x M); c in
// bin-sorted order when `sorted`.
int exec_type2(mnufft_plan p, int sign, const void *f, void *c, bool sorted = false)
{
    mn::Pts P = kernel_points(p, sorted);
    {
        StageTimer tm(p->tm, MNUFFT_STAGE_PRECORRECT, p->stream);
        MN_HIP(mn::launch_precorrect(p->dim, p->N, p->g.n, p->prec, (int)p->ntransf, f,
                                     p->pfac, p->grid, p->stream));
    }
    int rc;
    {
        StageTimer tm(p->tm, MNUFFT_STAGE_FFT, p->stream);
        rc = run_fft(p, sign);
    }
    if (rc) return rc;
    for (int64_t t = 0; t < p->ntransf; ++t) {
        char *ct = (char *)c + (size_t)t * p->M * 2 * p->rsz;
        const char *gt = (const char *)p->grid + (size_t)t * grid_bytes(p);
        StageTimer tm(p->tm, MNUFFT_STAGE_INTERP, p->stream);
        MN_HIP(mn::launch_interp(p->g, p->prec, p->method, P, gt, ct, p->stream));
    }
    return MNUFFT_OK;
}

// Per-dimension cover table of the SM add-back: for every grid index l, the
// (bin, offset in its padded tile) pairs whose tile lands on l after periodic
// wrapping; rows padded to the largest count with bin -1.
int build_cover(mnufft_plan p, int d)
{
    const mn::Geom &g = p->g;
    std::vector<int2> tab;
    mn::host::cover_table(g.n[d], g.m[d], g.B[d], g.pad, tab, p->kmax[d]);
    p->cov_bytes[d] = tab.size() * sizeof(int2);
    int rc = dalloc(p, (void **)&p->cov[d], p->cov_bytes[d]);
    if (rc) return rc;
    if (hipMemcpy(p->cov[d], tab.data(), p->cov_bytes[d], hipMemcpyHostToDevice) != hipSuccess)
        return MNUFFT_ERR_HIP;
    return MNUFFT_OK;
}

// Bin-sort of Sec. III-A: keys, stable permutation, bin starts, subproblems
// and the sorted bin-relative coordinates, all enqueued on the plan stream.
int enqueue_setpts(mnufft_plan p, int64_t M, const void *x, const void *y, const void *z)
{
    const mn::Geom &g = p->g;
    hipStream_t s = p->stream;
    p->nsub_max = (int)(g.nbins + (M + p->msub - 1) / p->msub);
    if (p->validate) MN_HIP(mn::launch_zero(p->flag, 16, s));
    // The bin-relative coordinates ride along with the keys through the radix
    // passes and must end in su.  Going backwards from the last pass the
    // destinations alternate su, su_tmp, su, ...; binkey writes the start
    // buffer (su_in for GM, which keeps an input-order copy).
    const int passes = mn::radix_passes(bits_for(g.nbins));
    std::vector<void *const *> bufs(passes + 1);
    for (int k = 0; k <= passes; ++k) bufs[passes - k] = (k % 2 == 0) ? p->su : p->su_tmp;
    if (p->method == MNUFFT_METHOD_GM) bufs[0] = p->su_in;
    std::vector<mn::Payload> pays(passes);
    for (int q = 0; q < passes; ++q)
        for (int d = 0; d < 3; ++d) {
            pays[q].in[d] = bufs[q][d];
            pays[q].out[d] = bufs[q + 1][d];
        }
    // GM keeps input-order copies of the keys and coordinates (k_binkey);
    // otherwise the sort's first pass computes them from the points itself
    const bool gm = p->method == MNUFFT_METHOD_GM;
    if (gm) {
        void *u0[3] = {bufs[0][0], bufs[0][1], bufs[0][2]};
        MN_HIP(mn::launch_binkey(g, p->prec, (int)M, x, y, z, p->keyA, u0, p->flag, s, nullptr,
                                 1, p->ptmap.on ? &p->ptmap : nullptr));
        if (M > 0)
            MN_HIP(hipMemcpyAsync(p->key_in, p->keyA, (size_t)M * 4, hipMemcpyDeviceToDevice, s));
    }
    const mn::KeySrc ks{g, x, y, z, p->flag, nullptr, 1, p->ptmap};
    uint32_t *sk = nullptr, *sv = nullptr;
    MN_HIP(mn::radix_sort((int)M, bits_for(g.nbins), p->prec, p->dim, p->keyA, p->valA, p->keyB,
                          p->valB, pays.data(), p->hist, p->partials, &sk, &sv, s,
                          gm ? nullptr : &ks));
    p->skey = sk;
    p->perm = reinterpret_cast<int32_t *>(sv);
    MN_HIP(mn::launch_binstart((int)M, g.nbins, p->skey, p->binstart, s));
    MN_HIP(mn::launch_subproblems(g.nbins, p->msub, p->nsub_max, p->binstart, p->subcount,
                                  p->partials, p->sub, p->nsub, s));
    if (p->method == MNUFFT_METHOD_SM) {
        MN_HIP(mn::launch_zero(p->nmerge, 4, s));
        MN_HIP(mn::launch_merge_list(p->nsub_max, p->nsub, p->sub, p->subcount, kMergeGroup,
                                     p->mergelist, p->nmerge, s));
    }
    if (p->method == MNUFFT_METHOD_SM && !balanced(p))
        MN_HIP(mn::launch_iota(p->spos_proc, (int)M, s));
    if (balanced(p)) {
        const void *su[3] = {p->su[0], p->su[1], p->su[2]};
        MN_HIP(mn::launch_balance(g, p->prec, p->nsub_max, p->sub, p->nsub, su, p->perm,
                                  p->su_proc, p->perm_proc, p->spos_proc, p->hslot_proc, s));
    }
    return MNUFFT_OK;
}

int plan_geometry(mnufft_plan p, const int64_t nf[3], int w, double beta, const mnufft_opts &o);
int plan_bins_device(mnufft_plan p);

// New method, bins and msub for a type 1 / 2 plan (the fine grid, the FFT
// and the correction factors stay): drops the point storage and the bin
// tables and makes them again for the new bins.
int replan(mnufft_plan p, const mnufft_opts &c)
{
    free_points(p);
    dfree(p, (void **)&p->binstart, ((size_t)p->g.nbins + 1) * 4);
    dfree(p, (void **)&p->subcount, (2 * (size_t)p->g.nbins + 1) * 4);
    for (int d = 0; d < 3; ++d) {
        dfree(p, (void **)&p->cov[d], p->cov_bytes[d]);
        p->cov_bytes[d] = 0;
        p->kmax[d] = 1;
    }
    p->M = -1;
    mnufft_opts o = p->opts;
    o.method = c.method;
    for (int d = 0; d < 3; ++d) o.binsize[d] = c.binsize[d];
    o.msub = c.msub;
    o.tune = MNUFFT_TUNE_OFF;
    p->msub = o.msub > 0 ? o.msub : 4096;
    int64_t nf[3] = {p->g.n[0], p->g.n[1], p->g.n[2]};
    int rc = plan_geometry(p, nf, p->g.w, p->g.beta, o);
    if (!rc) rc = plan_bins_device(p);
    return rc;
}

}  // namespace

int mn::host::plan_set_params(mnufft_plan p, const mnufft_opts &c)
{
    if (!p || p->type == 3) return MNUFFT_ERR_ARG;
    int rc = use_device(p);
    if (!rc) rc = replan(p, c);
    return rc;
}

namespace {

// Parameter selection at setpts for plans with opts.tune set: pick method,
// bins and msub for these points and re-plan when they change.
int tune_for_points(mnufft_plan p, int64_t M, const void *x, const void *y, const void *z)
{
    mnufft_opts c;
    int rc = mnufft_select(p->type, p->dim, p->N, p->iflag, p->eps, p->prec, M, x, y, z,
                           p->opts.tune, &p->opts, &c, nullptr);
    if (rc < 0) return rc;
    bool same = c.method == p->method && c.msub == p->msub;
    for (int d = 0; d < p->dim; ++d) same = same && std::min(c.binsize[d], p->g.n[d]) == p->g.m[d];
    if (same) return MNUFFT_OK;
    return replan(p, c);
}

int check_ready(mnufft_plan p)
{
    if (!p) return MNUFFT_ERR_ARG;
    if (p->M < 0) return MNUFFT_ERR_STATE;
    return MNUFFT_OK;
}

mnufft_plan new_plan(int type, int dim, const int64_t *nmodes, int iflag, int64_t ntransf,
                     double eps, int prec, const mnufft_opts &o, double sigma)
{
    mnufft_plan p = new (std::nothrow) mnufft_plan_s();
    if (!p) return nullptr;
    p->type = type;
    p->dim = dim;
    p->prec = prec;
    p->iflag = iflag;
    p->ntransf = ntransf;
    p->eps = eps;
    p->rsz = prec == MNUFFT_F32 ? 4 : 8;
    p->device = o.device;
    p->validate = o.validate_pts;
    p->stream = (hipStream_t)o.stream;
    p->msub = o.msub > 0 ? o.msub : 4096;
    p->sigma = sigma;
    p->opts = o;
    for (int d = 0; d < 3; ++d) p->N[d] = (nmodes && d < dim) ? nmodes[d] : 1;
    return p;
}

// Fine grid nf, kernel (w, beta), bins and method of a type 1 / 2 plan (host
// only).  ERR_ARG when the grid or the bin count is too large or method SM
// was asked for with padded bins that do not fit in LDS.
int plan_geometry(mnufft_plan p, const int64_t nf[3], int w, double beta, const mnufft_opts &o)
{
    const int dim = p->dim;
    int64_t cells = 1;
    for (int d = 0; d < dim; ++d) {
        if (nf[d] > (int64_t)1 << 30) return MNUFFT_ERR_ARG;
        cells *= nf[d];
    }
    if (cells > ((int64_t)1 << 40) / p->ntransf) return MNUFFT_ERR_ARG;
    mn::Geom &g = p->g;
    g.dim = dim;
    g.w = w;
    g.beta = beta;
    g.pad = (w + 1) / 2;
    // 1D bins stay short: sorted points carry their coordinate relative to the
    // bin start in the plan precision, and in single precision a 1024-cell bin
    // would leave those coordinates only about 6e-5 cells of resolution
    int defm[3];
    mn::host::default_bins(dim, nf, defm);
    bool user_bins = false;
    for (int d = 0; d < 3; ++d) {
        g.n[d] = d < dim ? (int)nf[d] : 1;
        int m = d < dim ? (o.binsize[d] > 0 ? o.binsize[d] : defm[d]) : 1;
        user_bins = user_bins || (d < dim && o.binsize[d] > 0);
        g.m[d] = std::min(m, g.n[d]);
        g.S[d] = (double)g.n[d] / (2.0 * kPi);
    }
    auto lds_of = [&]() {
        return std::max(mn::sm_lds_bytes(g, p->prec, false, p->msub),
                        mn::sm_lds_bytes(g, p->prec, true, p->msub));
    };
    // Default bins whose padded tiles do not fit in LDS (wide kernels, double
    // precision) are halved along their longest side until they do.
    while (!user_bins && lds_of() > kLdsMax) {
        int dl = 0;
        for (int d = 1; d < dim; ++d)
            if (g.m[d] > g.m[dl]) dl = d;
        if (g.m[dl] <= 1) break;
        g.m[dl] = (g.m[dl] + 1) / 2;
    }
    int64_t nbins = 1;
    for (int d = 0; d < 3; ++d) {
        g.B[d] = (g.n[d] + g.m[d] - 1) / g.m[d];
        nbins *= g.B[d];
    }
    if (nbins > ((int64_t)1 << 30)) return MNUFFT_ERR_ARG;
    g.nbins = (int)nbins;
    p->grid_elems = (size_t)cells;
    const size_t lds = lds_of();
    p->ts2 = mn::sm_tile_stride(g);
    if (o.method == MNUFFT_METHOD_AUTO)
        p->method = lds <= kLdsMax ? MNUFFT_METHOD_SM : MNUFFT_METHOD_GMSORT;
    else
        p->method = o.method;
    if (p->method == MNUFFT_METHOD_SM && lds > kLdsMax) return MNUFFT_ERR_ARG;
    return MNUFFT_OK;
}

// The device state that depends on the bins: bin starts, per-bin subproblem
// offsets and, for method SM, the merge counter, the max |c| partials and
// the cover tables of the add-back.
int plan_bins_device(mnufft_plan p)
{
    const mn::Geom &g = p->g;
    int rc = dalloc(p, (void **)&p->binstart, ((size_t)g.nbins + 1) * 4);
    // subproblem offsets (nbins + 1), then the add-back's list of bins (nbins)
    if (!rc) rc = dalloc(p, (void **)&p->subcount, (2 * (size_t)g.nbins + 1) * 4);
    if (!rc && p->method == MNUFFT_METHOD_SM) {
        if (!p->nmerge) rc = dalloc(p, (void **)&p->nmerge, 16);
        if (!rc && !p->cmax) rc = dalloc(p, &p->cmax, 1024 * 8);  // partial maxima, see k_maxabs
        for (int d = 0; d < p->dim && !rc; ++d) rc = build_cover(p, d);
    }
    return rc;
}

// Device state of a plan after plan_geometry: fine grids, bin tables, cover
// tables and, with_fft, the correction factors and the rocFFT plan (a type 3
// plan's spreading plan has neither).
int plan_device(mnufft_plan p, bool with_fft)
{
    const int dim = p->dim;
    const mn::Geom &g = p->g;
    std::call_once(g_fft_once, [] { g_fft_setup = rocfft_setup(); });
    int rc = MNUFFT_OK;
    if (g_fft_setup != rocfft_status_success) rc = MNUFFT_ERR_FFT;
    if (!rc) rc = use_device(p);
    if (!rc) rc = dalloc(p, &p->grid, p->grid_elems * 2 * p->rsz * p->ntransf);
    for (int d = 0; d < 3 && !rc && with_fft; ++d) {
        std::vector<double> fac;
        if (d < dim) correction(p->N[d], g.n[d], g.w, g.beta, fac);
        else fac.assign(1, 1.0);
        rc = dalloc(p, &p->pfac[d], fac.size() * p->rsz);
        if (rc) break;
        if (p->prec == MNUFFT_F32) {
            std::vector<float> ff(fac.begin(), fac.end());
            if (hipMemcpy(p->pfac[d], ff.data(), ff.size() * 4, hipMemcpyHostToDevice))
                rc = MNUFFT_ERR_HIP;
        } else if (hipMemcpy(p->pfac[d], fac.data(), fac.size() * 8, hipMemcpyHostToDevice)) {
            rc = MNUFFT_ERR_HIP;
        }
    }
    if (!rc) rc = dalloc(p, (void **)&p->nsub, 16);
    if (!rc) rc = dalloc(p, (void **)&p->flag, 16);
    if (!rc) rc = plan_bins_device(p);
    if (with_fft) {
        if (!rc && rocfft_execution_info_create(&p->fftinfo) != rocfft_status_success)
            rc = MNUFFT_ERR_FFT;
        if (!rc) rc = make_fft(p, p->iflag < 0 ? 0 : 1);
    }
    return rc;
}

// ---- type 3 ---------------------------------------------------------------
// The type 3 deconvolution needs phi_hat at w t / 2 for every frequency, with
// |t| <= pi / sigma.  log phi_hat is smooth and even there, so it is
// expanded once per plan in Chebyshev polynomials of u = 2 (xi / ximax)^2 - 1
// on [0, ximax], ximax = 1.01 w pi / (2 sigma): 20 terms fit it to about
// 1e-14 relative for every w <= 16 and sigma in [1.25, 2], and a frequency
// then costs 20 fused multiply-adds instead of a quadrature.
constexpr int kT3Cheb = 20;

void t3_cheb(int w, double beta, double sigma, std::vector<double> &out)
{
    const double ximax = 1.01 * w * kPi / (2.0 * sigma);
    std::vector<double> xi(kT3Cheb), ph;
    for (int j = 0; j < kT3Cheb; ++j) {
        const double u = std::cos(kPi * (j + 0.5) / kT3Cheb);
        xi[j] = ximax * std::sqrt(0.5 * (u + 1.0));
    }
    mn::host::es_fourier(beta, xi, ph);
    out.assign(kT3Cheb + 1, 0.0);
    out[0] = ximax;
    for (int k = 0; k < kT3Cheb; ++k) {
        double a = 0.0;
        for (int j = 0; j < kT3Cheb; ++j) a += std::log(ph[j]) * std::cos(kPi * k * (j + 0.5) / kT3Cheb);
        out[1 + k] = (k == 0 ? 1.0 : 2.0) * a / kT3Cheb;
    }
}

int make_type3(int dim, int iflag, int64_t ntransf, double eps, int prec, const mnufft_opts &o,
               double sigma, mnufft_plan *out)
{
    int w = 0;
    double beta = 0;
    int64_t n1 = 0;
    const int warn = mnufft_choose_params_sigma(eps, prec, 1, sigma, &w, &beta, &n1);
    if (warn < 0) return warn;
    mnufft_plan p = new_plan(3, dim, nullptr, iflag, ntransf, eps, prec, o, sigma);
    if (!p) return MNUFFT_ERR_ALLOC;
    p->g.dim = dim;
    p->g.w = w;
    p->g.beta = beta;
    p->method = o.method == MNUFFT_METHOD_AUTO ? MNUFFT_METHOD_SM : o.method;
    std::vector<double> zz;
    t3_cheb(w, beta, sigma, zz);
    p->t3nq = kT3Cheb;
    int rc = use_device(p);
    if (!rc) rc = dalloc(p, (void **)&p->t3quad, zz.size() * 8);
    if (!rc && hipMemcpy(p->t3quad, zz.data(), zz.size() * 8, hipMemcpyHostToDevice))
        rc = MNUFFT_ERR_HIP;
    if (!rc) rc = dalloc(p, (void **)&p->t3part, 2 * 1024 * 3 * 3 * 8);
    if (rc) {
        mnufft_destroy(p);
        return rc;
    }
    *out = p;
    return warn;
}

// Smallest even 2^a 3^b 5^c >= n.
int64_t smooth_even(int64_t n)
{
    n = std::max<int64_t>(n, 2);
    n += n & 1;
    for (;; n += 2) {
        int64_t r = n;
        for (int64_t f : {2, 3, 5})
            while (r % f == 0) r /= f;
        if (r == 1) return n;
    }
}

// (min, max) per dimension of n values from the partials of launch_t3_bounds;
// false if a value is non-finite.  n = 0 gives (0, 0).
bool reduce_bounds(const double *part, int nb, int dim, int n, double lo[3], double hi[3])
{
    bool ok = true;
    for (int d = 0; d < dim; ++d) {
        lo[d] = INFINITY;
        hi[d] = -INFINITY;
        for (int b = 0; b < nb; ++b) {
            const double *q = part + 3 * ((size_t)b * dim + d);
            lo[d] = std::min(lo[d], q[0]);
            hi[d] = std::max(hi[d], q[1]);
            if (q[2] != 0.0) ok = false;
        }
        if (n == 0) lo[d] = hi[d] = 0.0;
    }
    return ok;
}

void free_t3_points(mnufft_plan p)
{
    const size_t cz = 2 * p->rsz;
    if (p->t3Mcap >= 0) {
        const size_t M = (size_t)std::max<int64_t>(p->t3Mcap, 1);
        dfree(p, &p->t3pre, M * cz);
        dfree(p, &p->t3cp, M * cz * p->ntransf);
    }
    if (p->t3Kcap >= 0) {
        const size_t K = (size_t)std::max<int64_t>(p->t3Kcap, 1);
        dfree(p, &p->t3post, K * cz);
    }
    p->t3Mcap = p->t3Kcap = -1;
}

void destroy_t3_plans(mnufft_plan p)
{
    if (p->t3spr) mnufft_destroy(p->t3spr);
    if (p->t3inner) mnufft_destroy(p->t3inner);
    p->t3spr = p->t3inner = nullptr;
}

// Spreading plan (grid nf, no FFT) and inner type 2 plan (modes nf) of a
// type 3 plan, made anew when nf changes.
int make_t3_plans(mnufft_plan p, const int64_t nf[3])
{
    bool same = p->t3spr && p->t3inner;
    for (int d = 0; d < p->dim && same; ++d) same = p->nf3[d] == nf[d];
    if (same) return MNUFFT_OK;
    destroy_t3_plans(p);
    mnufft_opts o = p->opts;
    o.validate_pts = 0;  // the rescaled coordinates lie in [-pi, pi) by construction
    mnufft_plan s = new_plan(1, p->dim, nf, p->iflag, p->ntransf, p->eps, p->prec, o, p->sigma);
    if (!s) return MNUFFT_ERR_ALLOC;
    int rc = plan_geometry(s, nf, p->g.w, p->g.beta, o);
    if (rc) {
        delete s;
        return rc;
    }
    rc = plan_device(s, false);
    if (rc) {
        mnufft_destroy(s);
        return rc;
    }
    s->tm.on = p->tm.on;
    p->t3spr = s;
    rc = mnufft_makeplan(2, p->dim, nf, p->iflag, p->ntransf, p->eps, p->prec, &o, &p->t3inner);
    if (rc < 0) {
        p->t3inner = nullptr;
        destroy_t3_plans(p);
        return rc;
    }
    p->t3inner->tm.on = p->tm.on;
    for (int d = 0; d < 3; ++d) p->nf3[d] = d < p->dim ? nf[d] : 1;
    return MNUFFT_OK;
}

// Type 3 with the plan's sign: c (ntransf x M) -> f (ntransf x K).
int exec_type3(mnufft_plan p, const void *c, void *f)
{
    {
        StageTimer tm(p->tm, MNUFFT_STAGE_DECONV, p->stream);
        MN_HIP(mn::launch_cmul(p->prec, p->M, (int)p->ntransf, c, p->t3pre, p->t3cp, p->stream));
    }
    int rc = spread_all(p->t3spr, p->t3cp);
    if (rc) return rc;
    if ((rc = exec_type2(p->t3inner, p->iflag, p->t3spr->grid, f))) return rc;
    StageTimer tm(p->tm, MNUFFT_STAGE_DECONV, p->stream);
    MN_HIP(mn::launch_cmul(p->prec, p->K, (int)p->ntransf, f, p->t3post, f, p->stream));
    return MNUFFT_OK;
}

}  // namespace

extern "C" {

const char *mnufft_strerror(int s)
{
    switch (s) {
    case MNUFFT_OK: return "ok";
    case MNUFFT_WARN_EPS_CLAMPED: return "eps below the precision floor; kernel width capped";
    case MNUFFT_ERR_ARG: return "invalid argument";
    case MNUFFT_ERR_ALLOC: return "allocation failed";
    case MNUFFT_ERR_HIP: return "HIP runtime error";
    case MNUFFT_ERR_FFT: return "rocFFT error";
    case MNUFFT_ERR_STATE: return "call out of order (points not set)";
    case MNUFFT_ERR_PTS: return "point coordinate non-finite or outside [-3pi, 3pi)";
    case MNUFFT_ERR_UNSUPPORTED: return "unsupported request";
    }
    return "unknown status";
}

int mnufft_default_opts(mnufft_opts *o)
{
    if (!o) return MNUFFT_ERR_ARG;
    std::memset(o, 0, sizeof(*o));
    o->method = MNUFFT_METHOD_AUTO;
    o->device = -1;
    return MNUFFT_OK;
}

int mnufft_choose_params_sigma(double eps, int prec, int64_t N, double sigma, int *w,
                               double *beta, int64_t *n)
{
    if (!(eps > 0.0 && eps < 1.0) || (prec != MNUFFT_F32 && prec != MNUFFT_F64) || N < 1 ||
        !(sigma >= 1.25 && sigma <= 2.0) || !w || !beta || !n)
        return MNUFFT_ERR_ARG;
    int rc = MNUFFT_OK;
    // single precision: tolerances below 1e-7 (w = 8 at sigma = 2) are not reachable
    if (prec == MNUFFT_F32 && eps < 1e-7) {
        eps = 1e-7;
        rc = MNUFFT_WARN_EPS_CLAMPED;
    }
    int ww = std::max(2, mn::host::width_for_eps_sigma(eps, sigma));
    if (ww > 16) {
        ww = 16;
        rc = MNUFFT_WARN_EPS_CLAMPED;
    }
    *w = ww;
    *beta = mn::host::beta_for(ww, sigma);
    *n = fine_size(N, ww, sigma);
    return rc;
}

int mnufft_choose_params(double eps, int prec, int64_t N, int *w, double *beta, int64_t *n)
{
    return mnufft_choose_params_sigma(eps, prec, N, 2.0, w, beta, n);
}

int mnufft_type3_grid(double X, double S, double sigma, int w, int64_t *nf, double *gamma)
{
    if (!(X >= 0.0) || !(S >= 0.0) || !(sigma >= 1.25 && sigma <= 2.0) || w < 2 || w > 16 ||
        !nf || !gamma)
        return MNUFFT_ERR_ARG;
    if (S == 0.0) S = X > 0.0 ? 1.0 / X : 1.0;
    const double need = std::ceil(2.0 * sigma * S * X / kPi) + w + 1;
    if (!(need <= (double)(1 << 24))) return MNUFFT_ERR_ARG;
    *nf = smooth_even(std::max<int64_t>((int64_t)need, 2 * (int64_t)w));
    *gamma = (double)*nf / (2.0 * sigma * S);
    return MNUFFT_OK;
}

int mnufft_correction_factors(int64_t N, int64_t n, int w, double beta, double *out)
{
    if (N < 1 || n <= N || w < 2 || w > 16 || !(beta > 0.0) || !out) return MNUFFT_ERR_ARG;
    std::vector<double> p;
    correction(N, n, w, beta, p);
    std::copy(p.begin(), p.end(), out);
    return MNUFFT_OK;
}

int mnufft_makeplan(int type, int dim, const int64_t *nmodes, int iflag, int64_t ntransf,
                    double eps, int prec, const mnufft_opts *opts, mnufft_plan *out)
{
    if (!out) return MNUFFT_ERR_ARG;
    *out = nullptr;
    // ---- validate everything before touching the device ----
    if ((type != 1 && type != 2 && type != 3) || dim < 1 || dim > 3 ||
        (!nmodes && type != 3) || (iflag != 1 && iflag != -1) || ntransf < 1 ||
        !(eps > 0.0 && eps < 1.0) || (prec != MNUFFT_F32 && prec != MNUFFT_F64))
        return MNUFFT_ERR_ARG;
    mnufft_opts o;
    mnufft_default_opts(&o);
    if (opts) o = *opts;
    if (o.method < MNUFFT_METHOD_AUTO || o.method > MNUFFT_METHOD_SM || o.msub < 0 ||
        o.device < -1)
        return MNUFFT_ERR_ARG;
    for (int i = 0; i < 5; ++i)
        if (o.reserved[i]) return MNUFFT_ERR_ARG;
    if (o.tune < MNUFFT_TUNE_OFF || o.tune > MNUFFT_TUNE_LEARNED) return MNUFFT_ERR_ARG;
    // parameter selection covers types 1 and 2 in 2D / 3D and picks method,
    // bins and msub itself
    if (o.tune != MNUFFT_TUNE_OFF &&
        (type == 3 || dim == 1 || o.method != MNUFFT_METHOD_AUTO || o.msub != 0 ||
         o.binsize[0] || o.binsize[1] || o.binsize[2]))
        return MNUFFT_ERR_ARG;
    const double sigma = o.upsampfac == 0.0 ? 2.0 : o.upsampfac;
    if (!(sigma >= 1.25 && sigma <= 2.0)) return MNUFFT_ERR_ARG;
    for (int d = 0; d < dim; ++d)
        if ((type != 3 && (nmodes[d] < 1 || nmodes[d] > (1 << 24))) || o.binsize[d] < 0)
            return MNUFFT_ERR_ARG;
    if (type == 3) return make_type3(dim, iflag, ntransf, eps, prec, o, sigma, out);

    int w = 0;
    double beta = 0;
    int64_t nf[3] = {1, 1, 1};
    int warn = MNUFFT_OK;
    for (int d = 0; d < dim; ++d) {
        int rc = mnufft_choose_params_sigma(eps, prec, nmodes[d], sigma, &w, &beta, &nf[d]);
        if (rc < 0) return rc;
        if (rc > 0) warn = rc;
    }
    mnufft_plan p = new_plan(type, dim, nmodes, iflag, ntransf, eps, prec, o, sigma);
    if (!p) return MNUFFT_ERR_ALLOC;
    int rc = plan_geometry(p, nf, w, beta, o);
    if (rc) {
        delete p;
        return rc;
    }
    rc = plan_device(p, true);
    if (rc) {
        mnufft_destroy(p);
        return rc;
    }
    *out = p;
    return warn;
}

int mnufft_setpts(mnufft_plan p, int64_t M, const void *x, const void *y, const void *z)
{
    if (!p || p->type == 3 || M < 0 || M > 2147483647LL) return MNUFFT_ERR_ARG;
    if (p->dim == 1 && (y || z)) return MNUFFT_ERR_ARG;
    if (M > 0 && (!x || (p->dim >= 2 && !y))) return MNUFFT_ERR_ARG;
    if (M > 0 && p->dim >= 2 && ((p->dim == 3) != (z != nullptr))) return MNUFFT_ERR_ARG;
    int rc = use_device(p);
    if (rc) return rc;
    if (p->opts.tune != MNUFFT_TUNE_OFF && (rc = tune_for_points(p, M, x, y, z)) < 0) return rc;
    if (p->g.nbins + (M + p->msub - 1) / p->msub > 2147483647LL) return MNUFFT_ERR_ARG;
    p->M = -1;  // invalid until the whole setup has been enqueued
    if (M > p->Mcap && (rc = alloc_points(p, M))) {
        free_points(p);
        return rc;
    }
    {
        StageTimer tm(p->tm, MNUFFT_STAGE_SETPTS, p->stream);
        rc = enqueue_setpts(p, M, x, y, z);
    }
    if (rc) return rc;
    if (p->validate) {
        int h = 0;
        MN_HIP(hipMemcpyAsync(&h, p->flag, sizeof(int), hipMemcpyDeviceToHost, p->stream));
        MN_HIP(hipStreamSynchronize(p->stream));
        if (h) return MNUFFT_ERR_PTS;
    }
    p->M = M;
    return MNUFFT_OK;
}

int mnufft_setpts3(mnufft_plan p, int64_t M, const void *x, const void *y, const void *z,
                   int64_t K, const void *s, const void *t, const void *u)
{
    if (!p || p->type != 3 || M < 0 || M > 2147483647LL || K < 0 || K > 2147483647LL)
        return MNUFFT_ERR_ARG;
    const int dim = p->dim;
    const void *xs[3] = {x, dim >= 2 ? y : nullptr, dim == 3 ? z : nullptr};
    const void *ss[3] = {s, dim >= 2 ? t : nullptr, dim == 3 ? u : nullptr};
    if ((dim < 3 && (z || u)) || (dim < 2 && (y || t))) return MNUFFT_ERR_ARG;
    for (int d = 0; d < dim; ++d)
        if ((M > 0 && !xs[d]) || (K > 0 && !ss[d])) return MNUFFT_ERR_ARG;
    int rc = use_device(p);
    if (rc) return rc;
    p->M = p->K = -1;  // invalid until the whole setup has been enqueued
    hipStream_t st = p->stream;
    StageTimer tmr(p->tm, MNUFFT_STAGE_SETPTS, st);
    // centres and half-widths of the points and the frequencies
    const int nbx = mn::t3_bounds_blocks((int)M), nbs = mn::t3_bounds_blocks((int)K);
    double *partx = p->t3part, *parts = p->t3part + 1024 * 3 * 3;
    MN_HIP(mn::launch_t3_bounds(p->prec, (int)M, dim, xs, partx, st));
    MN_HIP(mn::launch_t3_bounds(p->prec, (int)K, dim, ss, parts, st));
    std::vector<double> hp(2 * 1024 * 3 * 3);
    MN_HIP(hipMemcpyAsync(hp.data(), p->t3part, hp.size() * 8, hipMemcpyDeviceToHost, st));
    MN_HIP(hipStreamSynchronize(st));
    double xl[3], xh[3], sl[3], sh[3];
    const bool okx = reduce_bounds(hp.data(), nbx, dim, (int)M, xl, xh);
    const bool oks = reduce_bounds(hp.data() + 1024 * 3 * 3, nbs, dim, (int)K, sl, sh);
    if (!okx || !oks) return MNUFFT_ERR_PTS;
    // rescaling: gamma = nf / (2 sigma S) puts the rescaled frequencies within
    // pi / sigma, and nf >= 2 sigma S X / pi + w + 1 keeps every point's taps
    // inside the grid without wrapping
    const int w = p->g.w;
    int64_t nf[3] = {1, 1, 1};
    for (int d = 0; d < dim; ++d) {
        p->C[d] = 0.5 * (xh[d] + xl[d]);
        p->D[d] = 0.5 * (sh[d] + sl[d]);
        rc = mnufft_type3_grid(0.5 * (xh[d] - xl[d]), 0.5 * (sh[d] - sl[d]), p->sigma, w, &nf[d],
                               &p->gam[d]);
        if (rc) return rc;  // space-bandwidth product too large
        p->hstep[d] = 2.0 * kPi / (double)nf[d];
    }
    if ((rc = make_t3_plans(p, nf))) return rc;
    // per-point and per-frequency buffers
    const size_t cz = 2 * p->rsz;
    if (M > p->t3Mcap || K > p->t3Kcap) {
        free_t3_points(p);
        const size_t Ma = (size_t)std::max<int64_t>(M, 1), Ka = (size_t)std::max<int64_t>(K, 1);
        rc = dalloc(p, &p->t3pre, Ma * cz);
        if (!rc) rc = dalloc(p, &p->t3cp, Ma * cz * p->ntransf);
        if (!rc) rc = dalloc(p, &p->t3post, Ka * cz);
        p->t3Mcap = M;
        p->t3Kcap = K;
        if (rc) {
            free_t3_points(p);
            return rc;
        }
    }
    mn::T3Affine ax{}, as{};
    mn::PtMap mx{}, ms{};
    mx.on = ms.on = 1;
    for (int d = 0; d < dim; ++d) {
        ax.off[d] = mx.off[d] = p->C[d];
        ax.scale[d] = mx.mul[d] = 1.0 / p->gam[d];  // points: (x - C) / gamma
        ax.mul[d] = p->D[d];
        as.off[d] = ms.off[d] = p->D[d];
        as.scale[d] = ms.mul[d] = p->hstep[d] * p->gam[d];  // frequencies: h gamma (s - D)
        as.mul[d] = p->C[d];
    }
    MN_HIP(mn::launch_t3_prephase(p->prec, (int)M, dim, xs, ax, p->iflag, p->t3pre, st));
    MN_HIP(mn::launch_t3_postfac(p->prec, (int)K, dim, ss, as, p->iflag, w, p->t3quad, p->t3nq,
                                 p->t3post, st));
    // both sets are binned straight from the caller's coordinates through the maps
    p->t3spr->ptmap = mx;
    p->t3inner->ptmap = ms;
    if ((rc = mnufft_setpts(p->t3spr, M, xs[0], xs[1], xs[2]))) return rc;
    if ((rc = mnufft_setpts(p->t3inner, K, ss[0], ss[1], ss[2]))) return rc;
    p->M = M;
    p->K = K;
    return MNUFFT_OK;
}

int mnufft_execute(mnufft_plan p, void *c, void *f)
{
    int rc = check_ready(p);
    if (rc) return rc;
    if (p->type == 3) {
        if ((p->K > 0 && !f) || (p->M > 0 && !c)) return MNUFFT_ERR_ARG;
        if ((rc = use_device(p))) return rc;
        return exec_type3(p, c, f);
    }
    if (!f || (p->M > 0 && !c)) return MNUFFT_ERR_ARG;
    if ((rc = use_device(p))) return rc;
    return p->type == 1 ? exec_type1(p, p->iflag, c, f) : exec_type2(p, p->iflag, f, c);
}

int mnufft_execute_sorted(mnufft_plan p, void *c, void *f)
{
    int rc = check_ready(p);
    if (rc) return rc;
    if (p->type == 3 || p->method == MNUFFT_METHOD_GM) return MNUFFT_ERR_UNSUPPORTED;
    if (!f || (p->M > 0 && !c)) return MNUFFT_ERR_ARG;
    if ((rc = use_device(p))) return rc;
    return p->type == 1 ? exec_type1(p, p->iflag, c, f, true)
                        : exec_type2(p, p->iflag, f, c, true);
}

int mnufft_execute_adjoint(mnufft_plan p, void *c, void *f)
{
    int rc = check_ready(p);
    if (rc) return rc;
    if (p->type == 3) return MNUFFT_ERR_UNSUPPORTED;
    if (!f || (p->M > 0 && !c)) return MNUFFT_ERR_ARG;
    if ((rc = use_device(p))) return rc;
    return p->type == 1 ? exec_type2(p, -p->iflag, f, c) : exec_type1(p, -p->iflag, c, f);
}

int mnufft_spread(mnufft_plan p, const void *c, void *grid)
{
    int rc = check_ready(p);
    if (rc) return rc;
    if (p->type == 3) return MNUFFT_ERR_UNSUPPORTED;
    if (!grid || (p->M > 0 && !c)) return MNUFFT_ERR_ARG;
    if ((rc = use_device(p))) return rc;
    if (p->method != MNUFFT_METHOD_SM) MN_HIP(mn::launch_zero(grid, grid_bytes(p), p->stream));
    else if (needs_cmax(p)) MN_HIP(mn::launch_zero(p->cmax, 1024 * 8, p->stream));
    MN_HIP(mn::launch_spread(p->g, p->prec, p->method, kernel_points(p, false), c, grid, p->stream));
    return MNUFFT_OK;
}

int mnufft_interp(mnufft_plan p, const void *grid, void *c)
{
    int rc = check_ready(p);
    if (rc) return rc;
    if (p->type == 3) return MNUFFT_ERR_UNSUPPORTED;
    if (!grid || (p->M > 0 && !c)) return MNUFFT_ERR_ARG;
    if ((rc = use_device(p))) return rc;
    MN_HIP(mn::launch_interp(p->g, p->prec, p->method, kernel_points(p, false), grid, c, p->stream));
    return MNUFFT_OK;
}

int mnufft_interp_grad(mnufft_plan p, const void *modes, const void *wts, void *gx, void *gy,
                       void *gz)
{
    int rc = check_ready(p);
    if (rc) return rc;
    if (p->type == 3) return MNUFFT_ERR_UNSUPPORTED;
    if (!modes || (p->M > 0 && (!wts || !gx || (p->dim >= 2 && !gy) || (p->dim == 3 && !gz))))
        return MNUFFT_ERR_ARG;
    if ((rc = use_device(p))) return rc;
    // field = type 2 of `modes` with the sign of the plan's type 2 direction
    const int sign = p->type == 2 ? p->iflag : -p->iflag;
    MN_HIP(mn::launch_precorrect(p->dim, p->N, p->g.n, p->prec, (int)p->ntransf, modes,
                                 p->pfac, p->grid, p->stream));
    if ((rc = run_fft(p, sign))) return rc;
    void *out[3] = {gx, p->dim >= 2 ? gy : nullptr, p->dim == 3 ? gz : nullptr};
    MN_HIP(mn::launch_interp_grad(p->g, p->prec, points_of(p), (int)p->ntransf, p->grid, wts,
                                  out, p->stream));
    return MNUFFT_OK;
}

int mnufft_get_sort(mnufft_plan p, int32_t *perm, int32_t *binstart)
{
    int rc = check_ready(p);
    if (rc) return rc;
    if (p->type == 3) return MNUFFT_ERR_UNSUPPORTED;
    if ((rc = use_device(p))) return rc;
    if (perm && p->M > 0)
        MN_HIP(hipMemcpyAsync(perm, p->perm, (size_t)p->M * 4, hipMemcpyDeviceToDevice, p->stream));
    if (binstart)
        MN_HIP(hipMemcpyAsync(binstart, p->binstart, ((size_t)p->g.nbins + 1) * 4,
                              hipMemcpyDeviceToDevice, p->stream));
    return MNUFFT_OK;
}

int mnufft_get_subproblems(mnufft_plan p, int32_t *sub, int32_t *nsub)
{
    int rc = check_ready(p);
    if (rc) return rc;
    if (p->type == 3) return MNUFFT_ERR_UNSUPPORTED;
    if ((rc = use_device(p))) return rc;
    if (sub && p->nsub_max > 0)
        MN_HIP(hipMemcpyAsync(sub, p->sub, (size_t)p->nsub_max * 16, hipMemcpyDeviceToDevice,
                              p->stream));
    if (nsub)
        MN_HIP(hipMemcpyAsync(nsub, p->nsub, 4, hipMemcpyDeviceToDevice, p->stream));
    return MNUFFT_OK;
}

int mnufft_set_stream(mnufft_plan p, void *stream)
{
    if (!p) return MNUFFT_ERR_ARG;
    int rc = use_device(p);
    if (rc) return rc;
    // both FFT directions exist from here on, so execute / execute_adjoint
    // allocate nothing and can be captured into a graph
    for (mnufft_plan q : {p, p->t3inner}) {
        if (!q || !q->fftinfo) continue;
        if ((rc = make_fft(q, 0)) || (rc = make_fft(q, 1))) return rc;
    }
    for (mnufft_plan q : {p, p->t3spr, p->t3inner}) {
        if (!q) continue;
        q->stream = (hipStream_t)stream;
        q->opts.stream = stream;
    }
    return MNUFFT_OK;
}

int mnufft_set_timing(mnufft_plan p, int enable)
{
    if (!p) return MNUFFT_ERR_ARG;
    p->tm.on = enable != 0;
    if (p->t3spr) p->t3spr->tm.on = p->tm.on;
    if (p->t3inner) p->t3inner->tm.on = p->tm.on;
    return MNUFFT_OK;
}

int mnufft_get_timing(mnufft_plan p, double *ms, int64_t *count, int reset)
{
    if (!p || !ms) return MNUFFT_ERR_ARG;
    int rc = use_device(p);
    if (rc) return rc;
    if ((rc = p->tm.read(p->stream, ms, count, reset))) return rc;
    // a type 3 plan adds the stages of its spreading and type 2 plans
    for (mnufft_plan q : {p->t3spr, p->t3inner}) {
        if (!q) continue;
        double qm[MNUFFT_NSTAGES];
        int64_t qc[MNUFFT_NSTAGES];
        if ((rc = q->tm.read(q->stream, qm, qc, reset))) return rc;
        for (int st = 0; st < MNUFFT_NSTAGES; ++st) {
            if (st == MNUFFT_STAGE_SETPTS) continue;  // inside the type 3 plan's own interval
            ms[st] += qm[st];
            if (count) count[st] += qc[st];
        }
    }
    return MNUFFT_OK;
}

int mnufft_get_info(mnufft_plan p, mnufft_info *info)
{
    if (!p || !info) return MNUFFT_ERR_ARG;
    std::memset(info, 0, sizeof(*info));
    info->type = p->type;
    info->dim = p->dim;
    info->prec = p->prec;
    info->iflag = p->iflag;
    for (int d = 0; d < 3; ++d) {
        info->nmodes[d] = p->N[d];
        info->nfine[d] = p->g.n[d];
        info->binsize[d] = p->g.m[d];
    }
    info->ntransf = p->ntransf;
    info->M = p->M;
    info->w = p->g.w;
    info->beta = p->g.beta;
    info->method = p->method;
    info->msub = p->msub;
    info->nbins = p->g.nbins;
    info->nsub_max = p->M >= 0 ? p->nsub_max : 0;
    info->device_bytes = p->devbytes;
    info->upsampfac = p->sigma;
    info->ntargets = p->type == 3 ? p->K : 0;
    if (p->type == 3) {
        // modes and fine grid of the inner type 2; bins of the spreading plan
        for (mnufft_plan q : {p->t3spr, p->t3inner})
            if (q) info->device_bytes += q->devbytes;
        for (int d = 0; d < 3; ++d) {
            info->nmodes[d] = p->nf3[d];
            info->nfine[d] = p->t3inner ? p->t3inner->g.n[d] : 1;
            info->binsize[d] = p->t3spr ? p->t3spr->g.m[d] : 0;
        }
        info->nbins = p->t3spr ? p->t3spr->g.nbins : 0;
        info->nsub_max = p->t3spr && p->M >= 0 ? p->t3spr->nsub_max : 0;
        if (p->t3spr) info->method = p->t3spr->method;
    }
    return MNUFFT_OK;
}

int mnufft_destroy(mnufft_plan p)
{
    if (!p) return MNUFFT_OK;
    int rc = MNUFFT_OK;
    if (p->device >= 0 && hipSetDevice(p->device) != hipSuccess) rc = MNUFFT_ERR_HIP;
    if (hipStreamSynchronize(p->stream) != hipSuccess) rc = MNUFFT_ERR_HIP;
    for (int k = 0; k < 2; ++k)
        if (p->fft[k]) rocfft_plan_destroy(p->fft[k]);
    if (p->fftinfo) rocfft_execution_info_destroy(p->fftinfo);
    p->tm.destroy();
    destroy_t3_plans(p);
    free_t3_points(p);
    dfree(p, (void **)&p->t3part, 0);
    dfree(p, (void **)&p->t3quad, 0);
    free_points(p);
    dfree(p, &p->fftwork, p->fftwork_bytes);
    dfree(p, &p->grid, p->grid_elems * 2 * p->rsz * p->ntransf);
    for (int d = 0; d < 3; ++d) dfree(p, &p->pfac[d], 0);
    dfree(p, (void **)&p->binstart, 0);
    dfree(p, (void **)&p->subcount, 0);
    dfree(p, (void **)&p->nsub, 0);
    dfree(p, (void **)&p->flag, 0);
    dfree(p, (void **)&p->nmerge, 0);
    dfree(p, &p->cmax, 0);
    for (int d = 0; d < 3; ++d) dfree(p, (void **)&p->cov[d], p->cov_bytes[d]);
    delete p;
    return rc;
}

}  // extern "C"
