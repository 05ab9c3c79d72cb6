// Dispatch of spreading / interpolation to the instantiated kernel slices.
#include "internal.h"

#include <algorithm>

namespace mn {
namespace detail {
template <typename T, int DIM>
hipError_t spread_dim(const Geom &g, int method, const Pts &P, const void *c, void *grid,
                      hipStream_t s, size_t lds, int part);
template <typename T, int DIM>
hipError_t interp_dim(const Geom &g, int method, const Pts &P, const void *grid, void *c,
                      hipStream_t s, size_t lds);
#define MN_EXTERN(TT, DD)                                                                  \
    extern template hipError_t spread_dim<TT, DD>(const Geom &, int, const Pts &, const void *, \
                                                  void *, hipStream_t, size_t, int);          \
    extern template hipError_t interp_dim<TT, DD>(const Geom &, int, const Pts &, const void *, \
                                                  void *, hipStream_t, size_t);               \
    extern template hipError_t grad_dim<TT, DD>(const Geom &, const Pts &, int, const void *,   \
                                                const void *, void *const[3], hipStream_t);
template <typename T, int DIM>
hipError_t grad_dim(const Geom &g, const Pts &P, int ntransf, const void *grid, const void *wts,
                    void *const out[3], hipStream_t s);
MN_EXTERN(float, 1) MN_EXTERN(float, 2) MN_EXTERN(float, 3)
MN_EXTERN(double, 1) MN_EXTERN(double, 2) MN_EXTERN(double, 3)
#undef MN_EXTERN
}  // namespace detail

hipError_t launch_interp_grad(const Geom &g, int prec, const Pts &P, int ntransf,
                              const void *grid, const void *wts, void *const out[3],
                              hipStream_t s)
{
    if (P.M == 0) return hipSuccess;
#define MN_GRAD(TT)                                                                          \
    (g.dim == 1   ? detail::grad_dim<TT, 1>(g, P, ntransf, grid, wts, out, s)                \
     : g.dim == 2 ? detail::grad_dim<TT, 2>(g, P, ntransf, grid, wts, out, s)                \
                  : detail::grad_dim<TT, 3>(g, P, ntransf, grid, wts, out, s))
    const hipError_t e = prec == 0 ? MN_GRAD(float) : MN_GRAD(double);
#undef MN_GRAD
    return e;
}

int sm_tile_stride(const Geom &g)
{
    const int P = (g.w + 1) / 2;
    size_t cells = 1;
    for (int d = 0; d < g.dim; ++d) cells *= (size_t)(g.m[d] + 2 * P);
    return (int)((2 * cells + 7) / 8 * 8);
}

size_t sm_lds_bytes(const Geom &g, int prec, bool interp, int msub)
{
    const size_t rsz = prec == 0 ? sizeof(float) : sizeof(double);
    // The spreading kernels build a start-cell histogram of
    // (m_2 + 2) (m_1 + w + 1) words (m_1 + w + 1 in 1D) in the tile's LDS
    // before clearing the tile; it always fits in the ts2 words of a
    // single-precision tile and its slots fit 16 bits, which this check
    // confirms.
    if (!interp) {
        size_t hist = (size_t)g.m[0] + g.w + 1;
        if (g.dim >= 2) hist *= (size_t)g.m[1] + 2;
        if (hist > (size_t)sm_tile_stride(g) || hist > 65535) return ~(size_t)0;
    }
    // 64-bit fixed-point accumulators: one word per cell in single precision,
    // one per part in double precision
    // (single precision also stages smp_stage strengths, 8 bytes each, and
    // their 16-bit histogram slots, rounded up to 16 bytes)
    // (1D single precision uses the two-word accumulator of double precision)
    // (the two-word kernel stages sm2_stage strengths of 2 rsz bytes each)
    if (!interp)
        return prec == 0 && g.dim >= 2
                   ? (size_t)sm_tile_stride(g) * 4 + (size_t)8 * smp_stage(g.dim, msub) +
                         ((size_t)2 * smp_stage(g.dim, msub) + 15) / 16 * 16
                   : (size_t)sm_tile_stride(g) * 8 + (size_t)sm2_stage(g.dim, prec, msub) * 2 * rsz;
    const int P = (g.w + 1) / 2;
    size_t cells = 1;
    for (int d = 0; d < g.dim; ++d) cells *= (size_t)(g.m[d] + 2 * P);
    return cells * 2 * rsz;
}

namespace {
__global__ void k_merge_list(int nsub_max, const int32_t *__restrict__ nsubp,
                             const int32_t *__restrict__ sub, const int32_t *__restrict__ suboff,
                             int G, int32_t *__restrict__ mergelist, int32_t *__restrict__ nmerge)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nsub_max || q >= *nsubp) return;
    const int b = reinterpret_cast<const int4 *>(sub)[q].x;
    const int first = suboff[b], k = suboff[b + 1] - first;
    if (k > G && (q - first) % G == 0) mergelist[atomicAdd(nmerge, 1)] = q;
}
}  // namespace

hipError_t launch_merge_list(int nsub_max, const int32_t *nsub, const int32_t *sub,
                             const int32_t *suboff, int G, int32_t *mergelist, int32_t *nmerge,
                             hipStream_t s)
{
    if (nsub_max <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_merge_list, dim3((nsub_max + 255) / 256), dim3(256), 0, s, nsub_max,
                       nsub, sub, suboff, G, mergelist, nmerge);
    return hipGetLastError();
}

hipError_t launch_spread(const Geom &g, int prec, int method, const Pts &P, const void *c,
                         void *grid, hipStream_t s, int part)
{
    if (P.M == 0) {
        // nothing to accumulate; the SM add-back alone owns writing the grid
        if (method != 3 || !(part & 2)) return hipSuccess;
        return launch_zero(grid, (size_t)P.ncells * 2 * (prec == 0 ? sizeof(float) : sizeof(double)),
                           s);
    }
    // the SM kernels reach every strength through an index array
    if (method == 3 && !P.perm && !P.spos) return hipErrorInvalidValue;
    const size_t lds = method == 3 ? sm_lds_bytes(g, prec, false, P.msub) : 0;
#define MN_SPREAD(TT)                                                                        \
    (g.dim == 1   ? detail::spread_dim<TT, 1>(g, method, P, c, grid, s, lds, part)           \
     : g.dim == 2 ? detail::spread_dim<TT, 2>(g, method, P, c, grid, s, lds, part)           \
                  : detail::spread_dim<TT, 3>(g, method, P, c, grid, s, lds, part))
    const hipError_t e = prec == 0 ? MN_SPREAD(float) : MN_SPREAD(double);
#undef MN_SPREAD
    return e;
}

hipError_t launch_interp(const Geom &g, int prec, int method, const Pts &P, const void *grid,
                         void *c, hipStream_t s)
{
    if (P.M == 0) return hipSuccess;
    if (method == 3 && !P.perm && !P.spos) return hipErrorInvalidValue;
    const size_t lds = method == 3 ? sm_lds_bytes(g, prec, true, P.msub) : 0;
#define MN_INTERP(TT)                                                                        \
    (g.dim == 1   ? detail::interp_dim<TT, 1>(g, method, P, grid, c, s, lds)                 \
     : g.dim == 2 ? detail::interp_dim<TT, 2>(g, method, P, grid, c, s, lds)                 \
                  : detail::interp_dim<TT, 3>(g, method, P, grid, c, s, lds))
    const hipError_t e = prec == 0 ? MN_INTERP(float) : MN_INTERP(double);
#undef MN_INTERP
    return e;
}

}  // namespace mn
