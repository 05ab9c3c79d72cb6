// Parameter selection for plans and batches: the exhaustive autotuner
// (timing every candidate of mnufft_tune_candidates on the caller's points,
// cached per problem class) and the learned selector (density features ->
// MLP -> predicted log run time per candidate -> argmin), with the autotuner
// as the selector's fallback.  The paper tuned bins and the subproblem size
// by hand on its GPU (Sec. III-A, first remark); these choose them per
// problem.  Selection changes which parameters run, never the result beyond
// rounding.
#include "../../include/mnufft.h"
#include "host_common.h"
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

namespace {

constexpr int kHist = 256;     // density features
constexpr int kScal = 6;       // scalar features
constexpr int kF = kHist + kScal;
constexpr int kMaxK = 128;     // candidates a selector may score (two mask words)

struct Selector {
    int dim = 0, prec = 0;
    double eps = 0, margin = 0;
    int F = 0, H = 0, K = 0;
    std::vector<mnufft_opts> cands;
    std::vector<float> params;
    std::map<int, float *> dev;  // device copy of params, per device
};

std::mutex g_mu;                          // guards everything below
std::vector<Selector> g_sel;
std::map<std::string, mnufft_opts> g_tuned;  // autotuner choices per problem class
// per-device workspace of the selection calls and its pinned host staging
// buffer (both grow, never shrink)
struct Work {
    void *ptr = nullptr;
    size_t bytes = 0;
    void *host = nullptr;
    size_t hbytes = 0;
    int clean_sets = 0;  // leading partial-histogram rows (sets) known to be zero
};
std::map<int, Work> g_work;

bool same_eps(double a, double b) { return std::fabs(a - b) <= 1e-12 * std::max(a, b); }

Selector *find_selector(int dim, int prec, double eps)
{
    for (auto &s : g_sel)
        if (s.dim == dim && s.prec == prec && same_eps(s.eps, eps)) return &s;
    return nullptr;
}

int current_device()
{
    int d = 0;
    return hipGetDevice(&d) == hipSuccess ? d : -1;
}

// Device workspace of at least `bytes` on the current device (g_mu held).
void *workspace(size_t bytes)
{
    Work &w = g_work[current_device()];
    if (w.bytes < bytes) {
        if (w.ptr) (void)hipFree(w.ptr);
        w.ptr = nullptr;
        w.bytes = 0;
        w.clean_sets = 0;
        if (hipMalloc(&w.ptr, bytes) != hipSuccess) {
            (void)hipGetLastError();
            w.ptr = nullptr;
            return nullptr;
        }
        w.bytes = bytes;
    }
    return w.ptr;
}

// Pinned host staging of at least `bytes` for the current device (g_mu held).
void *host_stage(size_t bytes)
{
    Work &w = g_work[current_device()];
    if (w.hbytes < bytes) {
        if (w.host) (void)hipHostFree(w.host);
        w.host = nullptr;
        w.hbytes = 0;
        if (hipHostMalloc(&w.host, bytes, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            w.host = nullptr;
            return nullptr;
        }
        w.hbytes = bytes;
    }
    return w.host;
}

float *device_params(Selector &s)
{
    const int d = current_device();
    auto it = s.dev.find(d);
    if (it != s.dev.end()) return it->second;
    float *p = nullptr;
    if (hipMalloc(&p, s.params.size() * 4) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (hipMemcpy(p, s.params.data(), s.params.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(p);
        return nullptr;
    }
    s.dev[d] = p;
    return p;
}

// The scalar features of one problem (the same as the training side's):
// log2 M / 24, log2 n_i / 12 for the three dimensions (0 when absent), w / 16
// and the type (0 for type 1, 1 for type 2), with n_i and w the sigma = 2
// parameters of the tolerance.
void scalar_features(int type, int dim, const int64_t *nmodes, int64_t M, double eps, int prec,
                     float *out)
{
    int w = 0;
    double beta = 0;
    int64_t n = 0;
    mnufft_choose_params(eps, prec, 1, &w, &beta, &n);
    out[0] = (float)(std::log2((double)std::max<int64_t>(M, 1)) / 24.0);
    for (int d = 0; d < 3; ++d) {
        int64_t nf = 1;
        if (d < dim) mnufft_choose_params(eps, prec, nmodes[d], &w, &beta, &nf);
        out[1 + d] = nf > 1 ? (float)(std::log2((double)nf) / 12.0) : 0.0f;
    }
    out[4] = (float)(w / 16.0);
    out[5] = (float)(type - 1);
}

// The selector's candidates that a problem may use: all of them for a plan,
// the SM ones for a batch.
void allowed_mask(const Selector &s, bool sm_only, unsigned long long mask[2])
{
    mask[0] = mask[1] = 0;
    for (int k = 0; k < s.K; ++k)
        if (!sm_only || s.cands[k].method == MNUFFT_METHOD_SM) mask[k / 64] |= 1ull << (k % 64);
}

// Problem class of the autotuner's cache: type, dimension, precision,
// tolerance, rounded log2 of the mode counts and of M, and the clustering
// level (twice the largest density feature, rounded).
std::string tune_key(int type, int dim, const int64_t *nmodes, int prec, double eps, int64_t M,
                     float maxfeat, bool sm_only)
{
    char buf[256];
    auto lg = [](int64_t v) { return (int)std::lround(std::log2((double)std::max<int64_t>(v, 1))); };
    std::snprintf(buf, sizeof(buf), "t%d-d%d-p%d-e%.3g-N%d.%d.%d-M%d-c%d-%s", type, dim, prec, eps,
                  lg(nmodes[0]), dim >= 2 ? lg(nmodes[1]) : 0, dim == 3 ? lg(nmodes[2]) : 0,
                  lg(M), (int)std::lround(2.0 * maxfeat), sm_only ? "sm" : "any");
    return buf;
}

// Density features of one point set into feat[0..255] (device), on stream s.
int density(int prec, int64_t M, const void *x, const void *y, float *feat, void *work,
            hipStream_t s)
{
    return mnufft_density_features(prec, M, x, y, feat, work, s);
}

// Exhaustive autotuning of one problem on its points (g_mu not held).
int autotune(int type, int dim, const int64_t *nmodes, int iflag, double eps, int prec, int64_t M,
             const void *x, const void *y, const void *z, const mnufft_opts &base, bool sm_only,
             mnufft_opts *out)
{
    const int n = mnufft_tune_candidates(dim, prec, eps, nullptr, 0);
    if (n <= 0) return n < 0 ? n : MNUFFT_ERR_ARG;
    std::vector<mnufft_opts> cands(n);
    mnufft_tune_candidates(dim, prec, eps, cands.data(), n);
    std::vector<mnufft_opts> use;
    for (auto c : cands) {
        if (sm_only && c.method != MNUFFT_METHOD_SM) continue;
        c.stream = base.stream;
        c.device = base.device;
        c.upsampfac = base.upsampfac;
        use.push_back(c);
    }
    int64_t K = 1;
    for (int d = 0; d < dim; ++d) K *= nmodes[d];
    const size_t rsz = prec == MNUFFT_F32 ? 8 : 16;  // one complex
    void *c = nullptr, *f = nullptr;
    if (hipMalloc(&c, (size_t)std::max<int64_t>(M, 1) * rsz) != hipSuccess ||
        hipMalloc(&f, (size_t)K * rsz) != hipSuccess) {
        (void)hipGetLastError();
        if (c) (void)hipFree(c);
        return MNUFFT_ERR_ALLOC;
    }
    hipStream_t s = (hipStream_t)base.stream;
    // the run time of the kernels does not depend on the values
    int rc = MNUFFT_OK;
    if (mn::launch_zero(c, (size_t)std::max<int64_t>(M, 1) * rsz, s) != hipSuccess ||
        mn::launch_zero(f, (size_t)K * rsz, s) != hipSuccess)
        rc = MNUFFT_ERR_HIP;
    std::vector<double> ms(use.size(), -1.0);
    if (!rc)
        rc = mnufft_tune_time(type, dim, nmodes, iflag, eps, prec, M, x, y, z, c, f, use.data(),
                              (int)use.size(), 3, 4.0, ms.data());
    (void)hipStreamSynchronize(s);
    (void)hipFree(c);
    (void)hipFree(f);
    if (rc < 0) return rc;
    int best = -1;
    for (size_t k = 0; k < use.size(); ++k)
        if (ms[k] > 0 && (best < 0 || ms[k] < ms[best])) best = (int)k;
    if (best < 0) return MNUFFT_ERR_ARG;
    *out = use[best];
    return MNUFFT_OK;
}

bool valid_mode(int mode) { return mode == MNUFFT_TUNE_AUTOTUNE || mode == MNUFFT_TUNE_LEARNED; }

}  // namespace

extern "C" {

int mnufft_selector_load(const char *path)
{
    if (!path) return MNUFFT_ERR_ARG;
    FILE *fh = std::fopen(path, "rb");
    if (!fh) return MNUFFT_ERR_ARG;
    Selector s;
    char magic[8];
    int32_t hdr[5];
    double eps = 0, margin = 0;
    bool ok = std::fread(magic, 1, 8, fh) == 8 && std::memcmp(magic, "MNSEL001", 8) == 0 &&
              std::fread(hdr, 4, 2, fh) == 2 && std::fread(&eps, 8, 1, fh) == 1 &&
              std::fread(hdr + 2, 4, 3, fh) == 3 && std::fread(&margin, 8, 1, fh) == 1;
    if (ok) {
        s.dim = hdr[0];
        s.prec = hdr[1];
        s.eps = eps;
        s.F = hdr[2];
        s.H = hdr[3];
        s.K = hdr[4];
        s.margin = margin;
        ok = (s.dim == 2 || s.dim == 3) && (s.prec == MNUFFT_F32 || s.prec == MNUFFT_F64) &&
             eps > 0 && eps < 1 && s.F == kF && s.H >= 1 && s.H <= 256 && s.K >= 1 &&
             s.K <= kMaxK && margin >= 0;
    }
    if (ok) {
        // the candidate list must be the autotuner's for this class, in order
        const int n = mnufft_tune_candidates(s.dim, s.prec, s.eps, nullptr, 0);
        std::vector<mnufft_opts> ref(std::max(n, 0));
        if (n > 0) mnufft_tune_candidates(s.dim, s.prec, s.eps, ref.data(), n);
        ok = n == s.K;
        for (int k = 0; k < s.K && ok; ++k) {
            int32_t r[5];
            ok = std::fread(r, 4, 5, fh) == 5 && r[0] == ref[k].method &&
                 r[1] == ref[k].binsize[0] && r[2] == ref[k].binsize[1] &&
                 r[3] == ref[k].binsize[2] && r[4] == ref[k].msub;
        }
        s.cands = ref;
    }
    if (ok) {
        const int64_t np = mnufft_mlp_nparams(s.F, s.H, s.K);
        s.params.resize((size_t)np);
        ok = np > 0 && std::fread(s.params.data(), 4, (size_t)np, fh) == (size_t)np;
        char extra;
        ok = ok && std::fread(&extra, 1, 1, fh) == 0;  // nothing after the parameters
    }
    std::fclose(fh);
    if (!ok) return MNUFFT_ERR_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    Selector *old = find_selector(s.dim, s.prec, s.eps);
    if (old) {
        for (auto &kv : old->dev) (void)hipFree(kv.second);
        *old = std::move(s);
    } else {
        g_sel.push_back(std::move(s));
    }
    return MNUFFT_OK;
}

int mnufft_selector_clear(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &s : g_sel)
        for (auto &kv : s.dev) (void)hipFree(kv.second);
    g_sel.clear();
    g_tuned.clear();
    return MNUFFT_OK;
}

int mnufft_select(int type, int dim, const int64_t *nmodes, int iflag, double eps, int prec,
                  int64_t M, const void *x, const void *y, const void *z, int mode,
                  const mnufft_opts *base, mnufft_opts *out, int *source)
{
    if ((type != 1 && type != 2) || (dim != 2 && dim != 3) || !nmodes ||
        (iflag != 1 && iflag != -1) || !(eps > 0.0 && eps < 1.0) ||
        (prec != MNUFFT_F32 && prec != MNUFFT_F64) || M < 0 || M > 2147483647LL ||
        !valid_mode(mode) || !out || (M > 0 && (!x || !y || ((dim == 3) != (z != nullptr)))))
        return MNUFFT_ERR_ARG;
    for (int d = 0; d < dim; ++d)
        if (nmodes[d] < 1 || nmodes[d] > (1 << 24)) return MNUFFT_ERR_ARG;
    mnufft_opts b;
    mnufft_default_opts(&b);
    if (base) {
        b.stream = base->stream;
        b.device = base->device;
        b.upsampfac = base->upsampfac;
    }
    if (b.device >= 0 && hipSetDevice(b.device) != hipSuccess) return MNUFFT_ERR_HIP;
    hipStream_t s = (hipStream_t)b.stream;
    // density features (and the learned prediction) under the lock: the
    // workspace is shared by all selection calls on a device
    float host_feat[kF];
    std::string key;
    int pick = -1;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        Selector *sel = mode == MNUFFT_TUNE_LEARNED ? find_selector(dim, prec, eps) : nullptr;
        const int K = sel ? sel->K : 0, H = sel ? sel->H : 0;
        const size_t need = (size_t)MNUFFT_DENSITY_WORK_BYTES + 4 * ((size_t)kF + 2);
        char *ws = (char *)workspace(need);
        if (!ws) return MNUFFT_ERR_ALLOC;
        float *feat = (float *)(ws + MNUFFT_DENSITY_WORK_BYTES);
        int rc = density(prec, M, x, y, feat, ws, s);
        if (rc < 0) return rc;
        scalar_features(type, dim, nmodes, M, eps, prec, host_feat + kHist);
        if (hipMemcpyAsync(feat + kHist, host_feat + kHist, kScal * 4, hipMemcpyHostToDevice, s) !=
            hipSuccess)
            return MNUFFT_ERR_HIP;
        float *params = sel ? device_params(*sel) : nullptr;
        if (sel && !params) return MNUFFT_ERR_ALLOC;
        // the network and the argmin over all candidates in one launch; the
        // pick is trusted when the runner-up is at least the selector's
        // margin behind (in predicted log time)
        int *idx = (int *)(feat + kF);
        float *gap = (float *)(idx + 1);
        int hidx = -1;
        float hgap = 0.f;
        if (sel) {
            unsigned long long mask[2];
            allowed_mask(*sel, false, mask);
            if (mn::launch_mlp_argmin(kF, H, K, params, 1, feat, kF, mask, idx, gap, s) !=
                    hipSuccess ||
                hipMemcpyAsync(&hidx, idx, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipMemcpyAsync(&hgap, gap, 4, hipMemcpyDeviceToHost, s) != hipSuccess)
                return MNUFFT_ERR_HIP;
        }
        if (hipMemcpyAsync(host_feat, feat, kHist * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return MNUFFT_ERR_HIP;
        if (sel) {
            const int best = hidx;
            if (best >= 0 && (double)hgap >= sel->margin) pick = best;
            if (pick >= 0) {
                *out = sel->cands[pick];
                out->stream = b.stream;
                out->device = b.device;
                out->upsampfac = b.upsampfac;
                if (source) *source = 0;
                return MNUFFT_OK;
            }
        }
        const float mx = *std::max_element(host_feat, host_feat + kHist);
        key = tune_key(type, dim, nmodes, prec, eps, M, mx, false);
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) {
            *out = it->second;
            out->stream = b.stream;
            out->device = b.device;
            out->upsampfac = b.upsampfac;
            if (source) *source = 1;
            return MNUFFT_OK;
        }
    }
    mnufft_opts best;
    const int rc = autotune(type, dim, nmodes, iflag, eps, prec, M, x, y, z, b, false, &best);
    if (rc < 0) return rc;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_tuned[key] = best;
    }
    *out = best;
    if (source) *source = 1;
    return MNUFFT_OK;
}

int mnufft_batch_select(int type, int dim, int ntr, const int64_t *nmodes, const int64_t *npts,
                        const void *x, const void *y, const void *z, double eps, int prec,
                        int mode, const mnufft_opts *base, int32_t *binsize, int32_t *msub,
                        int32_t *source)
{
    if ((type != 1 && type != 2) || (dim != 2 && dim != 3) || ntr < 1 || ntr > 65535 ||
        !nmodes || !npts || !(eps > 0.0 && eps < 1.0) ||
        (prec != MNUFFT_F32 && prec != MNUFFT_F64) || !valid_mode(mode) || !binsize || !msub ||
        !x || !y || ((dim == 3) != (z != nullptr)))
        return MNUFFT_ERR_ARG;
    int64_t tot = 0;
    for (int t = 0; t < ntr; ++t) {
        if (npts[t] < 0) return MNUFFT_ERR_ARG;
        for (int d = 0; d < dim; ++d)
            if (nmodes[3 * t + d] < 1 || nmodes[3 * t + d] > (1 << 24)) return MNUFFT_ERR_ARG;
        tot += npts[t];
    }
    if (tot > 2147483647LL) return MNUFFT_ERR_ARG;
    mnufft_opts b;
    mnufft_default_opts(&b);
    if (base) {
        b.stream = base->stream;
        b.device = base->device;
        b.upsampfac = base->upsampfac;
    }
    if (b.device >= 0 && hipSetDevice(b.device) != hipSuccess) return MNUFFT_ERR_HIP;
    hipStream_t s = (hipStream_t)b.stream;
    const size_t rsz = prec == MNUFFT_F32 ? 4 : 8;
    std::vector<int> need_tune;  // transforms left to the autotuner
    {
        std::lock_guard<std::mutex> lk(g_mu);
        Selector *sel = mode == MNUFFT_TUNE_LEARNED ? find_selector(dim, prec, eps) : nullptr;
        if (!sel) {
            for (int t = 0; t < ntr; ++t) need_tune.push_back(t);
        } else {
            // one upload (set offsets and scalar features), the batched
            // histogram counts, one launch for the features, the network and
            // the argmin of every transform, and one download (picks and
            // gaps), through pinned staging
            const int K = sel->K, H = sel->H;
            const size_t hist = (size_t)ntr * MNUFFT_DENSITY_BATCH_WORK_BYTES;
            const size_t offb = ((size_t)ntr + 1) * 8, scb = (size_t)ntr * kScal * 4;
            const size_t outb = (size_t)ntr * 8;
            char *ws = (char *)workspace(hist + offb + scb + outb);
            char *hs = (char *)host_stage(offb + scb + outb);
            float *params = device_params(*sel);
            if (!ws || !hs || !params) return MNUFFT_ERR_ALLOC;
            int64_t *off = (int64_t *)(ws + hist);
            float *scal = (float *)(ws + hist + offb);
            int *idx = (int *)(ws + hist + offb + scb);
            float *gap = (float *)(idx + ntr);
            int64_t *hoff = (int64_t *)hs;
            float *hscal = (float *)(hs + offb);
            const int *hidx = (const int *)(hs + offb + scb);
            const float *hgap = (const float *)(hidx + ntr);
            hoff[0] = 0;
            for (int t = 0; t < ntr; ++t) {
                hoff[t + 1] = hoff[t] + npts[t];
                scalar_features(type, dim, nmodes + 3 * t, npts[t], eps, prec,
                                hscal + (size_t)t * kScal);
            }
            // The partial rows are cleared only when they may hold something:
            // the selection kernel returns the rows it reads to zero, and the
            // rows past this call's sets may be overwritten by its other data.
            Work &wk = g_work[current_device()];
            uint32_t *part = (uint32_t *)ws;
            const bool need_clear = wk.clean_sets < ntr;
            wk.clean_sets = 0;
            unsigned long long mask[2];
            allowed_mask(*sel, true, mask);
            if (hipMemcpyAsync(off, hoff, offb + scb, hipMemcpyHostToDevice, s) != hipSuccess ||
                (need_clear && mn::launch_hist_clear(ntr, part, s) != hipSuccess) ||
                mn::launch_hist_count(prec, ntr, off, x, y, part, s) != hipSuccess ||
                mn::launch_select_rows(ntr, off, part, scal, kScal, kF, H, K, params, mask, idx,
                                       gap, s) != hipSuccess ||
                hipMemcpyAsync((void *)hidx, idx, outb, hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                return MNUFFT_ERR_HIP;
            wk.clean_sets = ntr;
            for (int t = 0; t < ntr; ++t) {
                if (hidx[t] < 0 || (double)hgap[t] < sel->margin) {
                    need_tune.push_back(t);
                    continue;
                }
                const mnufft_opts &c = sel->cands[hidx[t]];
                for (int d = 0; d < 3; ++d) binsize[3 * t + d] = d < dim ? c.binsize[d] : 0;
                msub[t] = c.msub;
                if (source) source[t] = 0;
            }
        }
    }
    int64_t o = 0;
    std::vector<int64_t> offs(ntr + 1, 0);
    for (int t = 0; t < ntr; ++t) offs[t + 1] = offs[t] + npts[t];
    for (int t : need_tune) {
        o = offs[t];
        const char *xs = (const char *)x + o * rsz, *ys = (const char *)y + o * rsz;
        const char *zs = z ? (const char *)z + o * rsz : nullptr;
        mnufft_opts best;
        const int rc = autotune(type, dim, nmodes + 3 * t, type == 1 ? -1 : 1, eps, prec, npts[t],
                                xs, ys, zs, b, true, &best);
        if (rc < 0) return rc;
        for (int d = 0; d < 3; ++d) binsize[3 * t + d] = d < dim ? best.binsize[d] : 0;
        msub[t] = best.msub;
        if (source) source[t] = 1;
    }
    return MNUFFT_OK;
}

}  // extern "C"
