// Autotuner: the candidate parameter sets (method x bin extents x msub) and
// their measured cost on a given problem.  The paper hand-tuned its bins and
// subproblem size on its GPU (Sec. III-A, first remark); here the choice is
// measured per problem class instead.
#include "../../include/mnufft.h"
#include "host_common.h"
#include "internal.h"

#include <algorithm>
#include <cstring>
#include <vector>

namespace {
constexpr size_t kLdsMax = 160 * 1024;

// LDS bytes of the SM kernels for bins m (both directions use the larger).
size_t sm_lds(int dim, int prec, int w, const int *m, int msub)
{
    mn::Geom g{};
    g.dim = dim;
    g.w = w;
    for (int d = 0; d < 3; ++d) g.m[d] = d < dim ? m[d] : 1;
    return std::max(mn::sm_lds_bytes(g, prec, false, msub), mn::sm_lds_bytes(g, prec, true, msub));
}
}  // namespace

extern "C" {

int mnufft_tune_candidates(int dim, int prec, double eps, mnufft_opts *list, int cap)
{
    if ((dim != 2 && dim != 3) || (prec != MNUFFT_F32 && prec != MNUFFT_F64) ||
        !(eps > 0.0 && eps < 1.0) || cap < 0 || (cap > 0 && !list))
        return MNUFFT_ERR_ARG;
    int w = 0;
    double beta = 0;
    int64_t n = 0;
    if (mnufft_choose_params(eps, prec, 1, &w, &beta, &n) < 0) return MNUFFT_ERR_ARG;
    // 2D: bin extents from {8, 16, 32, 64, 128} in each dimension, the
    // first at least the second (the transposed shapes behave alike);
    // 3D: shapes around the default 16 x 8 x 8 and the paper's 16 x 16 x 2
    static const int bins2[][3] = {{8, 8, 1},    {16, 8, 1},   {16, 16, 1},  {32, 8, 1},
                                   {32, 16, 1},  {32, 32, 1},  {64, 8, 1},   {64, 16, 1},
                                   {64, 32, 1},  {64, 64, 1},  {128, 8, 1},  {128, 16, 1},
                                   {128, 32, 1}, {128, 64, 1}, {128, 128, 1}};
    static const int bins3[][3] = {{8, 8, 8}, {16, 16, 2}, {16, 16, 4}, {16, 16, 8}, {32, 16, 4}, {16, 8, 8}};
    static const int msubs2[] = {1024, 4096};
    static const int msubs3[] = {256, 1024, 4096, 16384};
    int cnt = 0;
    auto push = [&](int method, const int *m, int msub) {
        if (cnt < cap) {
            mnufft_default_opts(&list[cnt]);
            list[cnt].method = method;
            for (int d = 0; d < 3; ++d) list[cnt].binsize[d] = d < dim ? m[d] : 0;
            list[cnt].msub = msub;
        }
        ++cnt;
    };
    const int nb = dim == 2 ? 15 : 6;
    const int *msubs = dim == 2 ? msubs2 : msubs3;
    const int nm = dim == 2 ? 2 : 4;
    for (int i = 0; i < nb; ++i) {
        const int *m = dim == 2 ? bins2[i] : bins3[i];
        for (int k = 0; k < nm; ++k)
            if (sm_lds(dim, prec, w, m, msubs[k]) <= kLdsMax) push(MNUFFT_METHOD_SM, m, msubs[k]);
    }
    const int *mdef = dim == 2 ? bins2[5] : bins3[1];
    push(MNUFFT_METHOD_GMSORT, mdef, 1024);
    push(MNUFFT_METHOD_GM, mdef, 1024);
    return cnt;
}

int mnufft_tune_time(int type, int dim, const int64_t *nmodes, int iflag, double eps, int prec,
                     int64_t M, const void *x, const void *y, const void *z, void *c, void *f,
                     const mnufft_opts *cands, int ncand, int reps, double cutoff, double *ms)
{
    if (!cands || !ms || ncand < 0 || reps < 1 || !(cutoff > 1.0)) return MNUFFT_ERR_ARG;
    for (int k = 0; k < ncand; ++k) ms[k] = -1.0;
    if (ncand == 0) return MNUFFT_OK;
    // one plan (fine grid, FFT and correction factors are the same for every
    // candidate), given each candidate's method, bins and msub in turn
    mnufft_opts base;
    mnufft_default_opts(&base);
    base.stream = cands[0].stream;
    base.device = cands[0].device;
    base.upsampfac = cands[0].upsampfac;
    mnufft_plan p = nullptr;
    if (mnufft_makeplan(type, dim, nmodes, iflag, 1, eps, prec, &base, &p) < 0) return MNUFFT_ERR_ARG;
    hipStream_t s = (hipStream_t)base.stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        mnufft_destroy(p);
        return MNUFFT_ERR_HIP;
    }
    double best = 1e300;
    for (int k = 0; k < ncand; ++k) {
        int rc = mn::host::plan_set_params(p, cands[k]);
        if (rc == MNUFFT_ERR_ARG) continue;  // candidate not valid for this problem: left at -1
        if (rc < 0) break;
        std::vector<double> t;
        for (int r = 0; r < reps + 1 && rc >= 0; ++r) {
            (void)hipEventRecord(e0, s);
            rc = mnufft_setpts(p, M, x, y, z);
            if (rc >= 0) rc = mnufft_execute(p, c, f);
            (void)hipEventRecord(e1, s);
            if (hipEventSynchronize(e1) != hipSuccess) rc = MNUFFT_ERR_HIP;
            float el = 0.f;
            (void)hipEventElapsedTime(&el, e0, e1);
            if (r > 0) t.push_back(el);           // the first run warms up
            if (r == 0 && el > cutoff * best) {   // far slower than the best: one sample suffices
                t.push_back(el);
                break;
            }
        }
        if (rc < 0 || t.empty()) {
            if (rc == MNUFFT_ERR_HIP) {
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
                mnufft_destroy(p);
                return rc;
            }
            continue;
        }
        std::sort(t.begin(), t.end());
        ms[k] = t[t.size() / 2];
        best = std::min(best, ms[k]);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    mnufft_destroy(p);
    return MNUFFT_OK;
}

}  // extern "C"
