// Batches of transforms of uneven sizes run as one: all transforms' bins
// share a global numbering (bin_off per transform), their points, fine grids
// and modes are concatenated, so the bin-sort is one sort, the subproblem list
// is one list, and the add-back and the corrections are one persistent launch
// each, whose work items look up their transform in a device table.
// Transforms with the same bins and msub form a class, numbered in class
// order, so each class's subproblems are one range of the list; spreading
// and interpolation run one launch per class (each with exactly the LDS its
// tiles need, on parallel streams), so that a few transforms with large
// bins do not lower the occupancy of all the others.  Only the fine-grid
// FFTs run per transform (rocFFT plans cached by size).  The method is SM
// for every transform.
#include "../../include/mnufft.h"
#include "host_common.h"
#include "internal.h"

#include <rocfft/rocfft.h>

#include <algorithm>
#include <array>
#include <cstring>
#include <map>
#include <new>
#include <vector>

using mn::host::StageTimer;

namespace {
constexpr size_t kLdsMax = 160 * 1024;
constexpr int kMergeGroup = 32;
}  // namespace

struct mnufft_batch_s {
    int type = 1, dim = 2, prec = 0, iflag = -1, T = 0;
    double eps = 1e-6;
    int device = -1;
    hipStream_t stream = nullptr;
    size_t rsz = 4;
    mn::Geom g{};  // shared fields; m holds the largest bin extents of the batch
    std::vector<mn::TGeom> geo;
    mn::TGeom *d_geo = nullptr;
    int64_t Mtot = 0, cells = 0, modes = 0;
    int nbins = 0, nsub_max = 0, msub_max = 1, ts2 = 0;
    // classes of transforms with equal bins and msub: bins [b0, b1) of the
    // global numbering, at most nsub_max subproblems
    struct Cls {
        int m[3];
        int msub;
        int b0, b1;
        int nsub_max;
    };
    std::vector<Cls> cls;
    int32_t *bin_t = nullptr;  // transform of every bin (device)
    void *grid = nullptr;
    void *pfac[3] = {nullptr, nullptr, nullptr};
    int2 *cov[3] = {nullptr, nullptr, nullptr};
    void *su[3] = {nullptr, nullptr, nullptr}, *su_tmp[3] = {nullptr, nullptr, nullptr};
    uint32_t *keyA = nullptr, *valA = nullptr, *keyB = nullptr, *valB = nullptr;
    uint32_t *skey = nullptr;
    int32_t *perm = nullptr;
    int32_t *binstart = nullptr, *subcount = nullptr, *sub = nullptr, *nsub = nullptr;
    int32_t *mergelist = nullptr, *nmerge = nullptr;
    uint32_t *hist = nullptr, *partials = nullptr;
    void *scratch = nullptr, *cmax = nullptr;
    int *flag = nullptr;
    std::map<std::array<int, 3>, rocfft_plan> fft;
    // The transforms' FFTs are independent and mostly small: they run spread
    // over kFftStreams streams (default priority), forked from and joined
    // back to the batch's stream with events.
    static constexpr int kFftStreams = 8;
    hipStream_t fstream[kFftStreams] = {};
    hipEvent_t fork = nullptr, join[kFftStreams] = {};
    rocfft_execution_info info[kFftStreams] = {};
    void *fftwork = nullptr;  // kFftStreams slices of fftwork_bytes
    size_t fftwork_bytes = 0;
    std::vector<int> fft_order;  // transforms by decreasing grid size
    bool pts_set = false;
    mn::host::Timers tm;
    std::vector<void *> allocs;
    int64_t devbytes = 0;
};

namespace {

int balloc(mnufft_batch b, void **p, size_t bytes)
{
    *p = nullptr;
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return e == hipErrorOutOfMemory ? MNUFFT_ERR_ALLOC : MNUFFT_ERR_HIP;
    }
    b->allocs.push_back(*p);
    b->devbytes += (int64_t)bytes;
    return MNUFFT_OK;
}

int upload(void *dst, const void *src, size_t bytes)
{
    return hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess ? MNUFFT_OK
                                                                             : MNUFFT_ERR_HIP;
}

mn::Pts batch_points(mnufft_batch b)
{
    mn::Pts P{};
    P.M = (int)b->Mtot;
    for (int d = 0; d < 3; ++d) {
        P.u[d] = b->su[d];
        P.cov[d] = b->cov[d];
        P.kmax[d] = 1;
        for (const mn::TGeom &t : b->geo) P.kmax[d] = std::max(P.kmax[d], t.kmax[d]);
    }
    P.key = b->skey;
    P.perm = b->perm;
    P.binstart = b->binstart;
    P.sub = b->sub;
    P.nsub = b->nsub;
    P.nsub_max = b->nsub_max;
    P.suboff = b->subcount;
    P.scratch = b->scratch;
    P.ts2 = b->ts2;
    P.G = kMergeGroup;
    P.mergelist = b->mergelist;
    P.nmerge = b->nmerge;
    P.heavy = nullptr;  // the batched add-back gathers per cell
    P.cmax = b->cmax;
    P.spos = nullptr;
    P.msub = b->msub_max;
    P.tg = b->d_geo;
    P.T = b->T;
    P.ncells = b->cells;
    P.bin_t = b->bin_t;
    return P;
}

// Spreading (interp false) or interpolation of every class: one launch per
// class with its own bins and msub over its range of the subproblem list,
// forked over the side streams when there are several classes.
int sm_classes(mnufft_batch b, const mn::Pts &P, bool interp, const void *in, void *out)
{
    const int nc = (int)b->cls.size();
    const bool fork = nc > 1;
    if (fork && hipEventRecord(b->fork, b->stream) != hipSuccess) return MNUFFT_ERR_HIP;
    const int ns = std::min(nc, (int)mnufft_batch_s::kFftStreams);
    for (int k = 0; fork && k < ns; ++k)
        if (hipStreamWaitEvent(b->fstream[k], b->fork, 0) != hipSuccess) return MNUFFT_ERR_HIP;
    for (int c = 0; c < nc; ++c) {
        const mnufft_batch_s::Cls &k = b->cls[c];
        mn::Geom g = b->g;
        for (int d = 0; d < 3; ++d) g.m[d] = k.m[d];
        mn::Pts Pc = P;
        Pc.q0 = P.suboff + k.b0;
        Pc.nsub = P.suboff + k.b1;
        Pc.nsub_max = std::max(k.nsub_max, 1);
        Pc.msub = k.msub;
        hipStream_t st = fork ? b->fstream[c % ns] : b->stream;
        const hipError_t e =
            interp ? mn::launch_interp(g, b->prec, MNUFFT_METHOD_SM, Pc, in, out, st)
                   : mn::launch_spread(g, b->prec, MNUFFT_METHOD_SM, Pc, in, out, st, 1);
        if (e != hipSuccess) return MNUFFT_ERR_HIP;
    }
    for (int k = 0; fork && k < ns; ++k)
        if (hipEventRecord(b->join[k], b->fstream[k]) != hipSuccess ||
            hipStreamWaitEvent(b->stream, b->join[k], 0) != hipSuccess)
            return MNUFFT_ERR_HIP;
    return MNUFFT_OK;
}

int run_ffts(mnufft_batch b, int sign)
{
    (void)sign;  // plans were made for the batch's single direction
    if (hipEventRecord(b->fork, b->stream) != hipSuccess) return MNUFFT_ERR_HIP;
    for (int k = 0; k < mnufft_batch_s::kFftStreams; ++k) {
        if (hipStreamWaitEvent(b->fstream[k], b->fork, 0) != hipSuccess) return MNUFFT_ERR_HIP;
        if (rocfft_execution_info_set_stream(b->info[k], b->fstream[k]) != rocfft_status_success)
            return MNUFFT_ERR_FFT;
        if (b->fftwork_bytes &&
            rocfft_execution_info_set_work_buffer(b->info[k],
                                                  (char *)b->fftwork + k * b->fftwork_bytes,
                                                  b->fftwork_bytes) != rocfft_status_success)
            return MNUFFT_ERR_FFT;
    }
    // largest grids first, each to the stream with the least work so far
    double load[mnufft_batch_s::kFftStreams] = {};
    for (int t : b->fft_order) {
        const mn::TGeom &g = b->geo[t];
        int k = 0;
        for (int j = 1; j < mnufft_batch_s::kFftStreams; ++j)
            if (load[j] < load[k]) k = j;
        load[k] += (double)g.n[0] * g.n[1] * g.n[2];
        const std::array<int, 3> key = {g.n[0], g.n[1], g.n[2]};
        void *buf[1] = {(char *)b->grid + (size_t)g.grid_off * 2 * b->rsz};
        if (rocfft_execute(b->fft[key], buf, nullptr, b->info[k]) != rocfft_status_success)
            return MNUFFT_ERR_FFT;
    }
    for (int k = 0; k < mnufft_batch_s::kFftStreams; ++k) {
        if (hipEventRecord(b->join[k], b->fstream[k]) != hipSuccess) return MNUFFT_ERR_HIP;
        if (hipStreamWaitEvent(b->stream, b->join[k], 0) != hipSuccess) return MNUFFT_ERR_HIP;
    }
    return MNUFFT_OK;
}

}  // namespace

extern "C" {

int mnufft_batch_destroy(mnufft_batch b)
{
    if (!b) return MNUFFT_OK;
    int rc = MNUFFT_OK;
    if (b->device >= 0 && hipSetDevice(b->device) != hipSuccess) rc = MNUFFT_ERR_HIP;
    if (hipStreamSynchronize(b->stream) != hipSuccess) rc = MNUFFT_ERR_HIP;
    for (int k = 0; k < mnufft_batch_s::kFftStreams; ++k)
        if (b->fstream[k] && hipStreamSynchronize(b->fstream[k]) != hipSuccess) rc = MNUFFT_ERR_HIP;
    for (auto &kv : b->fft) rocfft_plan_destroy(kv.second);
    for (int k = 0; k < mnufft_batch_s::kFftStreams; ++k) {
        if (b->info[k]) rocfft_execution_info_destroy(b->info[k]);
        if (b->join[k]) (void)hipEventDestroy(b->join[k]);
        if (b->fstream[k]) (void)hipStreamDestroy(b->fstream[k]);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    b->tm.destroy();
    for (void *p : b->allocs) (void)hipFree(p);
    delete b;
    return rc;
}

int mnufft_batch_makeplan(int type, int dim, int ntr, const int64_t *nmodes, const int64_t *npts,
                          int iflag, double eps, int prec, const int32_t *binsize,
                          const int32_t *msub, const mnufft_opts *opts, mnufft_batch *out)
{
    if (!out) return MNUFFT_ERR_ARG;
    *out = nullptr;
    if ((type != 1 && type != 2) || (dim != 2 && dim != 3) || ntr < 1 || !nmodes || !npts ||
        (iflag != 1 && iflag != -1) || !(eps > 0.0 && eps < 1.0) ||
        (prec != MNUFFT_F32 && prec != MNUFFT_F64))
        return MNUFFT_ERR_ARG;
    mnufft_opts o;
    mnufft_default_opts(&o);
    if (opts) o = *opts;
    if (o.msub < 0 || o.device < -1) return MNUFFT_ERR_ARG;
    const double sigma = o.upsampfac == 0.0 ? 2.0 : o.upsampfac;
    if (!(sigma >= 1.25 && sigma <= 2.0)) return MNUFFT_ERR_ARG;
    if (o.method != MNUFFT_METHOD_AUTO && o.method != MNUFFT_METHOD_SM) return MNUFFT_ERR_UNSUPPORTED;
    int64_t Mtot = 0;
    for (int t = 0; t < ntr; ++t) {
        if (npts[t] < 0) return MNUFFT_ERR_ARG;
        Mtot += npts[t];
        for (int d = 0; d < dim; ++d)
            if (nmodes[3 * t + d] < 1 || nmodes[3 * t + d] > (1 << 24)) return MNUFFT_ERR_ARG;
        for (int d = 0; d < 3 && binsize; ++d)
            if (binsize[3 * t + d] < 0) return MNUFFT_ERR_ARG;
        if (msub && msub[t] < 0) return MNUFFT_ERR_ARG;
    }
    if (Mtot > 2147483647LL) return MNUFFT_ERR_ARG;
    int w = 0;
    double beta = 0;
    int64_t ntmp = 0;
    int warn = mnufft_choose_params_sigma(eps, prec, 1, sigma, &w, &beta, &ntmp);
    if (warn < 0) return warn;

    mnufft_batch b = new (std::nothrow) mnufft_batch_s();
    if (!b) return MNUFFT_ERR_ALLOC;
    b->type = type;
    b->dim = dim;
    b->prec = prec;
    b->iflag = iflag;
    b->T = ntr;
    b->eps = eps;
    b->rsz = prec == MNUFFT_F32 ? 4 : 8;
    b->device = o.device;
    b->stream = (hipStream_t)o.stream;
    b->g.dim = dim;
    b->g.w = w;
    b->g.beta = beta;
    b->g.pad = (w + 1) / 2;
    const int P = b->g.pad;
    b->geo.resize(ntr);
    std::vector<double> pf[3];
    std::vector<int2> cv[3];
    int64_t bin_off = 0, pt_off = 0, grid_off = 0, mode_off = 0, nsub_max = 0;
    int mmax[3] = {1, 1, 1};
    for (int t = 0; t < ntr; ++t) {
        mn::TGeom &tg = b->geo[t];
        std::memset(&tg, 0, sizeof(tg));
        int64_t cells = 1, nm = 1, nb = 1;
        int64_t nf[3];
        for (int d = 0; d < 3; ++d)
            nf[d] = d < dim ? mn::host::fine_size(nmodes[3 * t + d], w, sigma) : 1;
        int defm[3];
        mn::host::default_bins(dim, nf, defm);
        for (int d = 0; d < 3; ++d) {
            const int64_t N = d < dim ? nmodes[3 * t + d] : 1;
            const int64_t n = nf[d];
            int m = d < dim ? (binsize && binsize[3 * t + d] > 0
                                   ? binsize[3 * t + d]
                                   : (o.binsize[d] > 0 ? o.binsize[d] : defm[d]))
                            : 1;
            m = (int)std::min<int64_t>(m, n);
            tg.N[d] = (int)N;
            tg.n[d] = (int)n;
            tg.m[d] = m;
            tg.B[d] = (int)((n + m - 1) / m);
            tg.S[d] = (double)n / (2.0 * mn::host::kPi);
            cells *= n;
            nm *= N;
            nb *= tg.B[d];
            mmax[d] = std::max(mmax[d], m);
            // correction factors (third dimension of a 2D batch: a single 1)
            std::vector<double> fac;
            if (d < dim) mn::host::correction(N, n, w, beta, fac);
            else fac.assign(1, 1.0);
            tg.p_off[d] = (int)pf[d].size();
            pf[d].insert(pf[d].end(), fac.begin(), fac.end());
            std::vector<int2> tab;
            int km = 1;
            if (d < dim) mn::host::cover_table((int)n, m, tg.B[d], P, tab, km);
            else tab.assign(1, make_int2(0, 0));
            tg.cov_off[d] = (int)cv[d].size();
            tg.kmax[d] = km;
            cv[d].insert(cv[d].end(), tab.begin(), tab.end());
        }
        tg.nbins = (int)nb;
        tg.pt_off = (int)pt_off;
        tg.M = (int)npts[t];
        tg.msub = msub && msub[t] > 0 ? msub[t] : (o.msub > 0 ? o.msub : 4096);
        tg.grid_off = grid_off;
        tg.mode_off = mode_off;
        b->msub_max = std::max(b->msub_max, tg.msub);
        bin_off += nb;  // total so far (the offsets are assigned per class below)
        pt_off += npts[t];
        grid_off += cells;
        mode_off += nm;
        nsub_max += nb + (npts[t] + tg.msub - 1) / tg.msub;
    }
    if (bin_off > (1LL << 30) || nsub_max > 2147483647LL || grid_off > (1LL << 40)) {
        delete b;
        return MNUFFT_ERR_ARG;
    }
    // classes of equal bins and msub, in order of first appearance; bins are
    // numbered class by class (transforms in input order within a class)
    std::vector<int> cls_of(ntr);
    for (int t = 0; t < ntr; ++t) {
        const mn::TGeom &tg = b->geo[t];
        int c = 0;
        for (; c < (int)b->cls.size(); ++c) {
            const mnufft_batch_s::Cls &k = b->cls[c];
            if (k.m[0] == tg.m[0] && k.m[1] == tg.m[1] && k.m[2] == tg.m[2] && k.msub == tg.msub)
                break;
        }
        if (c == (int)b->cls.size())
            b->cls.push_back({{tg.m[0], tg.m[1], tg.m[2]}, tg.msub, 0, 0, 0});
        cls_of[t] = c;
    }
    {
        int64_t next = 0;
        for (int c = 0; c < (int)b->cls.size(); ++c) {
            mnufft_batch_s::Cls &k = b->cls[c];
            k.b0 = (int)next;
            int64_t ns = 0;
            for (int t = 0; t < ntr; ++t) {
                if (cls_of[t] != c) continue;
                mn::TGeom &tg = b->geo[t];
                tg.bin_off = (int)next;
                next += tg.nbins;
                ns += tg.nbins + (npts[t] + tg.msub - 1) / tg.msub;
            }
            k.b1 = (int)next;
            k.nsub_max = (int)std::min<int64_t>(ns, 2147483647LL);
        }
    }
    b->Mtot = Mtot;
    b->cells = grid_off;
    b->modes = mode_off;
    b->nbins = (int)bin_off;
    b->nsub_max = (int)nsub_max;
    for (int d = 0; d < 3; ++d) b->g.m[d] = mmax[d];
    b->g.nbins = b->nbins;
    b->ts2 = mn::sm_tile_stride(b->g);
    for (const mnufft_batch_s::Cls &k : b->cls) {
        mn::Geom g = b->g;
        for (int d = 0; d < 3; ++d) g.m[d] = k.m[d];
        if (mn::sm_lds_bytes(g, prec, false, k.msub) > kLdsMax ||
            mn::sm_lds_bytes(g, prec, true, k.msub) > kLdsMax) {
            delete b;
            return MNUFFT_ERR_ARG;
        }
    }

    // ---- device state ----
    int rc = MNUFFT_OK;
    if (rocfft_setup() != rocfft_status_success) rc = MNUFFT_ERR_FFT;
    if (!rc && b->device >= 0 && hipSetDevice(b->device) != hipSuccess) rc = MNUFFT_ERR_HIP;
    if (!rc) rc = balloc(b, (void **)&b->d_geo, sizeof(mn::TGeom) * ntr);
    if (!rc) rc = upload(b->d_geo, b->geo.data(), sizeof(mn::TGeom) * ntr);
    if (!rc) {
        std::vector<int32_t> bt((size_t)std::max(b->nbins, 1), 0);
        for (int t = 0; t < ntr; ++t)
            for (int k = 0; k < b->geo[t].nbins; ++k) bt[(size_t)b->geo[t].bin_off + k] = t;
        rc = balloc(b, (void **)&b->bin_t, bt.size() * 4);
        if (!rc) rc = upload(b->bin_t, bt.data(), bt.size() * 4);
    }
    if (!rc) rc = balloc(b, &b->grid, (size_t)b->cells * 2 * b->rsz);
    for (int d = 0; d < 3 && !rc; ++d) {
        rc = balloc(b, &b->pfac[d], pf[d].size() * b->rsz);
        if (rc) break;
        if (prec == MNUFFT_F32) {
            std::vector<float> ff(pf[d].begin(), pf[d].end());
            rc = upload(b->pfac[d], ff.data(), ff.size() * 4);
        } else {
            rc = upload(b->pfac[d], pf[d].data(), pf[d].size() * 8);
        }
        if (!rc) rc = balloc(b, (void **)&b->cov[d], cv[d].size() * sizeof(int2));
        if (!rc) rc = upload(b->cov[d], cv[d].data(), cv[d].size() * sizeof(int2));
    }
    const size_t Ma = (size_t)std::max<int64_t>(Mtot, 1);
    for (int d = 0; d < dim && !rc; ++d) {
        rc = balloc(b, &b->su[d], Ma * b->rsz);
        if (!rc) rc = balloc(b, &b->su_tmp[d], Ma * b->rsz);
    }
    if (!rc) rc = balloc(b, (void **)&b->keyA, Ma * 4);
    if (!rc) rc = balloc(b, (void **)&b->valA, Ma * 4);
    if (!rc) rc = balloc(b, (void **)&b->keyB, Ma * 4);
    if (!rc) rc = balloc(b, (void **)&b->valB, Ma * 4);
    const size_t hist = mn::radix_hist_elems((int)Mtot);
    if (!rc) rc = balloc(b, (void **)&b->hist, hist * 4);
    if (!rc)
        rc = balloc(b, (void **)&b->partials,
                    4 * std::max(mn::scan_partial_elems(hist),
                                 mn::scan_partial_elems((size_t)b->nbins + 1)));
    if (!rc) rc = balloc(b, (void **)&b->binstart, ((size_t)b->nbins + 1) * 4);
    if (!rc) rc = balloc(b, (void **)&b->subcount, ((size_t)b->nbins + 1) * 4);
    if (!rc) rc = balloc(b, (void **)&b->sub, (size_t)std::max(b->nsub_max, 1) * 16);
    if (!rc) rc = balloc(b, (void **)&b->nsub, 16);
    if (!rc) rc = balloc(b, (void **)&b->mergelist, (size_t)std::max(b->nsub_max, 1) * 4);
    if (!rc) rc = balloc(b, (void **)&b->nmerge, 16);
    if (!rc) rc = balloc(b, &b->scratch, (size_t)std::max(b->nsub_max, 1) * b->ts2 * b->rsz);
    if (!rc) rc = balloc(b, &b->cmax, 1024 * 8);
    if (!rc) rc = balloc(b, (void **)&b->flag, 16);
    if (!rc && hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess)
        rc = MNUFFT_ERR_HIP;
    for (int k = 0; k < mnufft_batch_s::kFftStreams && !rc; ++k) {
        if (rocfft_execution_info_create(&b->info[k]) != rocfft_status_success) rc = MNUFFT_ERR_FFT;
        else if (hipStreamCreateWithFlags(&b->fstream[k], hipStreamNonBlocking) != hipSuccess ||
                 hipEventCreateWithFlags(&b->join[k], hipEventDisableTiming) != hipSuccess)
            rc = MNUFFT_ERR_HIP;
    }
    b->fft_order.resize(ntr);
    for (int t = 0; t < ntr; ++t) b->fft_order[t] = t;
    std::stable_sort(b->fft_order.begin(), b->fft_order.end(), [&](int a, int c) {
        const mn::TGeom &ga = b->geo[a], &gc = b->geo[c];
        return (int64_t)ga.n[0] * ga.n[1] * ga.n[2] > (int64_t)gc.n[0] * gc.n[1] * gc.n[2];
    });
    size_t work = 0;
    for (int t = 0; t < ntr && !rc; ++t) {
        const mn::TGeom &tg = b->geo[t];
        const std::array<int, 3> key = {tg.n[0], tg.n[1], tg.n[2]};
        if (b->fft.count(key)) continue;
        void *pl = nullptr;
        size_t wb = 0;
        rc = mn::host::make_rocfft(prec, dim, tg.n, 1, iflag, &pl, &wb);
        if (rc) break;
        b->fft[key] = (rocfft_plan)pl;
        work = std::max(work, wb);
    }
    if (!rc && work) {
        work = (work + 255) / 256 * 256;
        rc = balloc(b, &b->fftwork, work * mnufft_batch_s::kFftStreams);
        b->fftwork_bytes = work;
    }
    if (rc) {
        mnufft_batch_destroy(b);
        return rc;
    }
    *out = b;
    return warn;
}

int mnufft_batch_setpts(mnufft_batch b, const void *x, const void *y, const void *z)
{
    if (!b) return MNUFFT_ERR_ARG;
    if (b->Mtot > 0 && (!x || !y || ((b->dim == 3) != (z != nullptr)))) return MNUFFT_ERR_ARG;
    if (b->device >= 0 && hipSetDevice(b->device) != hipSuccess) return MNUFFT_ERR_HIP;
    b->pts_set = false;
    hipStream_t s = b->stream;
    const int M = (int)b->Mtot;
    {
        StageTimer tm(b->tm, MNUFFT_STAGE_SETPTS, s);
        const int passes = mn::radix_passes(mn::host::bits_for(b->nbins));
        std::vector<void *const *> bufs(passes + 1);
        for (int k = 0; k <= passes; ++k) bufs[passes - k] = (k % 2 == 0) ? b->su : b->su_tmp;
        std::vector<mn::Payload> pays(passes);
        for (int q = 0; q < passes; ++q)
            for (int d = 0; d < 3; ++d) {
                pays[q].in[d] = bufs[q][d];
                pays[q].out[d] = bufs[q + 1][d];
            }
        // the sort's first pass computes keys and coordinates from the points
        const mn::KeySrc ks{b->g, x, y, z, b->flag, b->d_geo, b->T, mn::PtMap{}};
        uint32_t *sk = nullptr, *sv = nullptr;
        if (mn::radix_sort(M, mn::host::bits_for(b->nbins), b->prec, b->dim, b->keyA, b->valA,
                           b->keyB, b->valB, pays.data(), b->hist, b->partials, &sk, &sv, s, &ks))
            return MNUFFT_ERR_HIP;
        b->skey = sk;
        b->perm = reinterpret_cast<int32_t *>(sv);
        if (mn::launch_binstart(M, b->nbins, b->skey, b->binstart, s)) return MNUFFT_ERR_HIP;
        if (mn::launch_subproblems(b->nbins, b->msub_max, b->nsub_max, b->binstart, b->subcount,
                                   b->partials, b->sub, b->nsub, s, b->d_geo, b->T, b->bin_t))
            return MNUFFT_ERR_HIP;
        if (mn::launch_zero(b->nmerge, 4, s)) return MNUFFT_ERR_HIP;
        if (mn::launch_merge_list(b->nsub_max, b->nsub, b->sub, b->subcount, kMergeGroup,
                                  b->mergelist, b->nmerge, s))
            return MNUFFT_ERR_HIP;
    }
    b->pts_set = true;
    return MNUFFT_OK;
}

int mnufft_batch_execute(mnufft_batch b, void *c, void *f)
{
    if (!b) return MNUFFT_ERR_ARG;
    if (!b->pts_set) return MNUFFT_ERR_STATE;
    if (!f || (b->Mtot > 0 && !c)) return MNUFFT_ERR_ARG;
    if (b->device >= 0 && hipSetDevice(b->device) != hipSuccess) return MNUFFT_ERR_HIP;
    hipStream_t s = b->stream;
    const mn::Pts P = batch_points(b);
    int rc;
    if (b->type == 1) {
        if (b->prec == MNUFFT_F64) {  // max |c| for the double-precision fixed-point scale
            StageTimer tm(b->tm, MNUFFT_STAGE_SCALE, s);
            if (mn::launch_zero(b->cmax, 1024 * 8, s)) return MNUFFT_ERR_HIP;
            if (mn::launch_spread(b->g, b->prec, MNUFFT_METHOD_SM, P, c, b->grid, s, 4))
                return MNUFFT_ERR_HIP;
        }
        {
            StageTimer tm(b->tm, MNUFFT_STAGE_SPREAD, s);
            rc = sm_classes(b, P, false, c, b->grid);
            if (rc) return rc;
        }
        {
            StageTimer tm(b->tm, MNUFFT_STAGE_ADDBACK, s);
            if (mn::launch_spread(b->g, b->prec, MNUFFT_METHOD_SM, P, c, b->grid, s, 2))
                return MNUFFT_ERR_HIP;
        }
        {
            StageTimer tm(b->tm, MNUFFT_STAGE_FFT, s);
            rc = run_ffts(b, b->iflag);
        }
        if (rc) return rc;
        StageTimer tm(b->tm, MNUFFT_STAGE_DECONV, s);
        if (mn::launch_deconv_batch(b->d_geo, b->T, b->modes, b->prec, b->grid, b->pfac, f, s))
            return MNUFFT_ERR_HIP;
        return MNUFFT_OK;
    }
    {
        StageTimer tm(b->tm, MNUFFT_STAGE_PRECORRECT, s);
        if (mn::launch_precorrect_batch(b->d_geo, b->T, b->cells, b->prec, f, b->pfac, b->grid, s))
            return MNUFFT_ERR_HIP;
    }
    {
        StageTimer tm(b->tm, MNUFFT_STAGE_FFT, s);
        rc = run_ffts(b, b->iflag);
    }
    if (rc) return rc;
    StageTimer tm(b->tm, MNUFFT_STAGE_INTERP, s);
    return sm_classes(b, P, true, b->grid, c);
}

int mnufft_batch_set_timing(mnufft_batch b, int enable)
{
    if (!b) return MNUFFT_ERR_ARG;
    b->tm.on = enable != 0;
    return MNUFFT_OK;
}

int mnufft_batch_get_timing(mnufft_batch b, double *ms, int64_t *count, int reset)
{
    if (!b || !ms) return MNUFFT_ERR_ARG;
    if (b->device >= 0 && hipSetDevice(b->device) != hipSuccess) return MNUFFT_ERR_HIP;
    return b->tm.read(b->stream, ms, count, reset);
}

int mnufft_batch_get_totals(mnufft_batch b, int64_t *totals)
{
    if (!b || !totals) return MNUFFT_ERR_ARG;
    totals[0] = b->Mtot;
    totals[1] = b->modes;
    totals[2] = b->cells;
    totals[3] = b->nbins;
    totals[4] = b->nsub_max;
    totals[5] = b->devbytes;
    return MNUFFT_OK;
}

}  // extern "C"
