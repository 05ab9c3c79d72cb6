// Kernel templates for spreading / interpolation; included by the
// per-(precision, dimension) instantiation units.  See spread_inst.hip.
#pragma once
#include "internal.h"

// Spreading (type 1 step 1, Sec. II-A) and interpolation (type 2 step 3,
// Sec. II-B) with the exponential-of-semicircle kernel
//   phi_beta(z) = exp(beta (sqrt(1 - z^2) - 1)),  |z| <= 1   (eq. es)
// rescaled to w fine-grid cells.  A point with grid coordinate g (grid point
// l sits at l h - pi) touches, per dimension, the w cells l0 .. l0 + w - 1
// with l0 = ceil(g - w/2) and weights phi(2 (l - g) / w).
//
// Methods (Sec. III-A / III-B):
//   GM      one thread per point in input order, global atomics
//   GMSORT  one thread per point in bin-sorted order, global atomics
//   SM      one workgroup per subproblem (<= msub sorted points of one bin):
//           type 1 accumulates into an LDS copy of the padded bin with LDS
//           atomics, then adds the nonzero cells to the grid with wrapped
//           global atomics (eq. addtoglobal); type 2 stages the padded bin
//           in LDS and every point reads its w^d values from there.
//
// Sorted points carry bin-relative coordinates u = g - binstart computed in
// double and rounded once, so single-precision runs keep full accuracy even
// on large grids.  Kernels are instantiated per width w (2..16) so that the
// tap loops unroll into registers.


#include <algorithm>

namespace mn {
namespace detail {

constexpr int kThreads = 256;

template <typename T> struct Cplx;
template <> struct Cplx<float> { using type = float2; };
template <> struct Cplx<double> { using type = double2; };

// Kernel value at z (|z| <= 1 up to rounding).  `bk` is beta*log2(e) in
// single precision (the exponential is evaluated as a power of two) and
// beta in double precision.
__device__ __forceinline__ float es_val(float z, float bk)
{
    const float t = fmaxf(1.0f - z * z, 0.0f);
    return __builtin_amdgcn_exp2f(bk * (__builtin_amdgcn_sqrtf(t) - 1.0f));
}
__device__ __forceinline__ double es_val(double z, double bk)
{
    const double t = fmax(1.0 - z * z, 0.0);
    return exp(bk * (sqrt(t) - 1.0));
}

// First tap index (as an integer) and the W kernel weights of a point at
// coordinate v on a lattice of unit spacing.
template <typename T, int W>
__device__ __forceinline__ int taps(T v, T bk, T (&k)[W])
{
    const T s = ceil(v - (T)(0.5 * W));
    const T z0 = (s - v) * (T)(2.0 / W);
#pragma unroll
    for (int a = 0; a < W; ++a) k[a] = es_val(z0 + (T)a * (T)(2.0 / W), bk);
    return (int)s;
}

// First tap of a point at v, with z0 = 2 (first tap - v) / W; the weight of
// tap a is es_val(z0 + 2a/W).  Used for the outermost dimension, whose taps
// are produced inside a rolled loop.
template <typename T, int W>
__device__ __forceinline__ int tap_start(T v, T &z0)
{
    const T s = ceil(v - (T)(0.5 * W));
    z0 = (s - v) * (T)(2.0 / W);
    return (int)s;
}

__device__ __forceinline__ int wrap1(int l, int n)  // l in [-n, 2n)
{
    return l < 0 ? l + n : (l >= n ? l - n : l);
}

__device__ __forceinline__ int wrapmod(int l, int n)
{
    l %= n;
    return l < 0 ? l + n : l;
}

template <typename T>
__device__ __forceinline__ void gadd(T *p, T v) { unsafeAtomicAdd(p, v); }

// ----------------------------------------------------------------------------
// GM / GM-sort spreading: thread i handles point i of the given order.
// perm == nullptr means input order (GM).
template <typename T, int DIM, int W>
__global__ void __launch_bounds__(kThreads)
k_spread_gm(Geom g, int M, const uint32_t *__restrict__ key, const T *__restrict__ u0,
            const T *__restrict__ u1, const T *__restrict__ u2,
            const int32_t *__restrict__ perm, const typename Cplx<T>::type *__restrict__ c,
            typename Cplx<T>::type *__restrict__ grid, T bk)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    uint32_t b = key[i];
    const int bx = b % g.B[0]; b /= g.B[0];
    const int by = b % g.B[1]; b /= g.B[1];
    const int bz = b;
    T kx[W], ky[W];
    const int sx = taps<T, W>(u0[i], bk, kx) + bx * g.m[0];
    const int sy = taps<T, W>(u1[i], bk, ky) + by * g.m[1];
    const auto cv = c[perm ? perm[i] : i];
    int lx[W];
#pragma unroll
    for (int a = 0; a < W; ++a) lx[a] = wrap1(sx + a, g.n[0]);
    if constexpr (DIM == 2) {
#pragma unroll
        for (int a2 = 0; a2 < W; ++a2) {
            const T wr = cv.x * ky[a2], wi = cv.y * ky[a2];
            T *row = reinterpret_cast<T *>(grid) + 2 * (size_t)wrap1(sy + a2, g.n[1]) * g.n[0];
#pragma unroll
            for (int a1 = 0; a1 < W; ++a1) {
                gadd(row + 2 * lx[a1], wr * kx[a1]);
                gadd(row + 2 * lx[a1] + 1, wi * kx[a1]);
            }
        }
    } else {
        T z0;
        const int sz = tap_start<T, W>(u2[i], z0) + bz * g.m[2];
#pragma unroll 1
        for (int a3 = 0; a3 < W; ++a3) {
            const T kz = es_val(z0 + (T)a3 * (T)(2.0 / W), bk);
            const T cr = cv.x * kz, ci = cv.y * kz;
            const size_t plane = (size_t)wrap1(sz + a3, g.n[2]) * g.n[1];
#pragma unroll
            for (int a2 = 0; a2 < W; ++a2) {
                const T wr = cr * ky[a2], wi = ci * ky[a2];
                T *row = reinterpret_cast<T *>(grid) +
                         2 * (plane + (size_t)wrap1(sy + a2, g.n[1])) * g.n[0];
#pragma unroll
                for (int a1 = 0; a1 < W; ++a1) {
                    gadd(row + 2 * lx[a1], wr * kx[a1]);
                    gadd(row + 2 * lx[a1] + 1, wi * kx[a1]);
                }
            }
        }
    }
}

// GM / GM-sort interpolation.
template <typename T, int DIM, int W>
__global__ void __launch_bounds__(kThreads)
k_interp_gm(Geom g, int M, const uint32_t *__restrict__ key, const T *__restrict__ u0,
            const T *__restrict__ u1, const T *__restrict__ u2,
            const int32_t *__restrict__ perm, const typename Cplx<T>::type *__restrict__ grid,
            typename Cplx<T>::type *__restrict__ c, T bk)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    uint32_t b = key[i];
    const int bx = b % g.B[0]; b /= g.B[0];
    const int by = b % g.B[1]; b /= g.B[1];
    const int bz = b;
    T kx[W], ky[W];
    const int sx = taps<T, W>(u0[i], bk, kx) + bx * g.m[0];
    const int sy = taps<T, W>(u1[i], bk, ky) + by * g.m[1];
    int lx[W];
#pragma unroll
    for (int a = 0; a < W; ++a) lx[a] = wrap1(sx + a, g.n[0]);
    T ar = 0, ai = 0;
    if constexpr (DIM == 2) {
#pragma unroll
        for (int a2 = 0; a2 < W; ++a2) {
            const auto *row = grid + (size_t)wrap1(sy + a2, g.n[1]) * g.n[0];
            T rr = 0, ri = 0;
#pragma unroll
            for (int a1 = 0; a1 < W; ++a1) {
                const auto v = row[lx[a1]];
                rr += v.x * kx[a1];
                ri += v.y * kx[a1];
            }
            ar += rr * ky[a2];
            ai += ri * ky[a2];
        }
    } else {
        T z0;
        const int sz = tap_start<T, W>(u2[i], z0) + bz * g.m[2];
#pragma unroll 1
        for (int a3 = 0; a3 < W; ++a3) {
            const T kz = es_val(z0 + (T)a3 * (T)(2.0 / W), bk);
            const size_t plane = (size_t)wrap1(sz + a3, g.n[2]) * g.n[1];
            T pr = 0, pi = 0;
#pragma unroll
            for (int a2 = 0; a2 < W; ++a2) {
                const auto *row = grid + (plane + (size_t)wrap1(sy + a2, g.n[1])) * g.n[0];
                T rr = 0, ri = 0;
#pragma unroll
                for (int a1 = 0; a1 < W; ++a1) {
                    const auto v = row[lx[a1]];
                    rr += v.x * kx[a1];
                    ri += v.y * kx[a1];
                }
                pr += rr * ky[a2];
                pi += ri * ky[a2];
            }
            ar += pr * kz;
            ai += pi * kz;
        }
    }
    typename Cplx<T>::type out;
    out.x = ar;
    out.y = ai;
    c[perm ? perm[i] : i] = out;
}

// ----------------------------------------------------------------------------
// SM spreading.  Grid-stride loop over the subproblem list; the padded bin
// (p_i = m_i + 2 ceil(w/2), offset binstart - ceil(w/2)) lives in dynamic LDS
// as interleaved (re, im).
template <typename T, int DIM, int W>
__global__ void __launch_bounds__(kThreads)
k_spread_sm(Geom g, const int32_t *__restrict__ sub, const int32_t *__restrict__ nsubp,
            const T *__restrict__ u0, const T *__restrict__ u1, const T *__restrict__ u2,
            const int32_t *__restrict__ perm, const typename Cplx<T>::type *__restrict__ c,
            typename Cplx<T>::type *__restrict__ grid, T bk)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *tile = reinterpret_cast<T *>(smem_raw);
    constexpr int P = (W + 1) / 2;
    const int p1 = g.m[0] + 2 * P, p2 = g.m[1] + 2 * P;
    const int p3 = DIM == 3 ? g.m[2] + 2 * P : 1;
    const int tsize = p1 * p2 * p3;
    const int nsub = *nsubp;
    for (int q = blockIdx.x; q < nsub; q += gridDim.x) {
        const int4 rec = reinterpret_cast<const int4 *>(sub)[q];
        int b = rec.x;
        const int bx = b % g.B[0]; b /= g.B[0];
        const int by = b % g.B[1]; b /= g.B[1];
        const int bz = b;
        for (int e = threadIdx.x; e < tsize; e += blockDim.x) {
            tile[2 * e] = 0;
            tile[2 * e + 1] = 0;
        }
        __syncthreads();
        const int end = rec.y + rec.z;
        for (int i = rec.y + threadIdx.x; i < end; i += blockDim.x) {
            T kx[W], ky[W];
            const int sx = taps<T, W>(u0[i] + (T)P, bk, kx);
            const int sy = taps<T, W>(u1[i] + (T)P, bk, ky);
            const auto cv = c[perm[i]];
            if constexpr (DIM == 2) {
#pragma unroll
                for (int a2 = 0; a2 < W; ++a2) {
                    const T wr = cv.x * ky[a2], wi = cv.y * ky[a2];
                    T *row = tile + 2 * ((sy + a2) * p1 + sx);
#pragma unroll
                    for (int a1 = 0; a1 < W; ++a1) {
                        atomicAdd(row + 2 * a1, wr * kx[a1]);
                        atomicAdd(row + 2 * a1 + 1, wi * kx[a1]);
                    }
                }
            } else {
                T z0;
                const int sz = tap_start<T, W>(u2[i] + (T)P, z0);
#pragma unroll 1
                for (int a3 = 0; a3 < W; ++a3) {
                    const T kz = es_val(z0 + (T)a3 * (T)(2.0 / W), bk);
                    const T cr = cv.x * kz, ci = cv.y * kz;
#pragma unroll
                    for (int a2 = 0; a2 < W; ++a2) {
                        const T wr = cr * ky[a2], wi = ci * ky[a2];
                        T *row = tile + 2 * (((sz + a3) * p2 + sy + a2) * p1 + sx);
#pragma unroll
                        for (int a1 = 0; a1 < W; ++a1) {
                            atomicAdd(row + 2 * a1, wr * kx[a1]);
                            atomicAdd(row + 2 * a1 + 1, wi * kx[a1]);
                        }
                    }
                }
            }
        }
        __syncthreads();
        const int o1 = bx * g.m[0] - P, o2 = by * g.m[1] - P, o3 = DIM == 3 ? bz * g.m[2] - P : 0;
        for (int e = threadIdx.x; e < tsize; e += blockDim.x) {
            const T re = tile[2 * e], im = tile[2 * e + 1];
            if (re == (T)0 && im == (T)0) continue;
            const int s1 = e % p1, r = e / p1;
            const int s2 = r % p2, s3 = r / p2;
            const int l1 = wrapmod(o1 + s1, g.n[0]);
            const int l2 = wrapmod(o2 + s2, g.n[1]);
            const int l3 = DIM == 3 ? wrapmod(o3 + s3, g.n[2]) : 0;
            T *dst = reinterpret_cast<T *>(grid) +
                     2 * (((size_t)l3 * g.n[1] + l2) * g.n[0] + l1);
            gadd(dst, re);
            gadd(dst + 1, im);
        }
        __syncthreads();
    }
}

// SM interpolation: stage the padded bin in LDS, then every point of the
// subproblem reads its w^d values there.
template <typename T, int DIM, int W>
__global__ void __launch_bounds__(kThreads)
k_interp_sm(Geom g, const int32_t *__restrict__ sub, const int32_t *__restrict__ nsubp,
            const T *__restrict__ u0, const T *__restrict__ u1, const T *__restrict__ u2,
            const int32_t *__restrict__ perm, const typename Cplx<T>::type *__restrict__ grid,
            typename Cplx<T>::type *__restrict__ c, T bk)
{
    using C = typename Cplx<T>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *tile = reinterpret_cast<C *>(smem_raw);
    constexpr int P = (W + 1) / 2;
    const int p1 = g.m[0] + 2 * P, p2 = g.m[1] + 2 * P;
    const int p3 = DIM == 3 ? g.m[2] + 2 * P : 1;
    const int tsize = p1 * p2 * p3;
    const int nsub = *nsubp;
    for (int q = blockIdx.x; q < nsub; q += gridDim.x) {
        const int4 rec = reinterpret_cast<const int4 *>(sub)[q];
        int b = rec.x;
        const int bx = b % g.B[0]; b /= g.B[0];
        const int by = b % g.B[1]; b /= g.B[1];
        const int bz = b;
        const int o1 = bx * g.m[0] - P, o2 = by * g.m[1] - P, o3 = DIM == 3 ? bz * g.m[2] - P : 0;
        for (int e = threadIdx.x; e < tsize; e += blockDim.x) {
            const int s1 = e % p1, r = e / p1;
            const int s2 = r % p2, s3 = r / p2;
            const int l1 = wrapmod(o1 + s1, g.n[0]);
            const int l2 = wrapmod(o2 + s2, g.n[1]);
            const int l3 = DIM == 3 ? wrapmod(o3 + s3, g.n[2]) : 0;
            tile[e] = grid[((size_t)l3 * g.n[1] + l2) * g.n[0] + l1];
        }
        __syncthreads();
        const int end = rec.y + rec.z;
        for (int i = rec.y + threadIdx.x; i < end; i += blockDim.x) {
            T kx[W], ky[W];
            const int sx = taps<T, W>(u0[i] + (T)P, bk, kx);
            const int sy = taps<T, W>(u1[i] + (T)P, bk, ky);
            T ar = 0, ai = 0;
            if constexpr (DIM == 2) {
#pragma unroll
                for (int a2 = 0; a2 < W; ++a2) {
                    const C *row = tile + (sy + a2) * p1 + sx;
                    T rr = 0, ri = 0;
#pragma unroll
                    for (int a1 = 0; a1 < W; ++a1) {
                        const C v = row[a1];
                        rr += v.x * kx[a1];
                        ri += v.y * kx[a1];
                    }
                    ar += rr * ky[a2];
                    ai += ri * ky[a2];
                }
            } else {
                T z0;
                const int sz = tap_start<T, W>(u2[i] + (T)P, z0);
#pragma unroll 1
                for (int a3 = 0; a3 < W; ++a3) {
                    const T kz = es_val(z0 + (T)a3 * (T)(2.0 / W), bk);
                    T pr = 0, pi = 0;
#pragma unroll
                    for (int a2 = 0; a2 < W; ++a2) {
                        const C *row = tile + ((sz + a3) * p2 + sy + a2) * p1 + sx;
                        T rr = 0, ri = 0;
#pragma unroll
                        for (int a1 = 0; a1 < W; ++a1) {
                            const C v = row[a1];
                            rr += v.x * kx[a1];
                            ri += v.y * kx[a1];
                        }
                        pr += rr * ky[a2];
                        pi += ri * ky[a2];
                    }
                    ar += pr * kz;
                    ai += pi * kz;
                }
            }
            C out;
            out.x = ar;
            out.y = ai;
            c[perm[i]] = out;
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------------------
// Dispatch over (precision, dimension, width).
inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

template <typename T> T kernel_param(double beta);
template <> inline float kernel_param<float>(double beta) { return (float)(beta * 1.4426950408889634); }
template <> inline double kernel_param<double>(double beta) { return beta; }

// Persistent grid size for the subproblem loops.
inline int sm_grid(const Pts &P) { return std::max(1, std::min(P.nsub_max, 256 * 16)); }

template <typename T, int DIM, int W>
hipError_t spread_w(const Geom &g, int method, const Pts &P, const void *c, void *grid,
                    hipStream_t s, size_t lds)
{
    using C = typename Cplx<T>::type;
    const T bk = kernel_param<T>(g.beta);
    if (method == 3) {
        auto kern = k_spread_sm<T, DIM, W>;
        if (lds > 65536)
            (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds);
        hipLaunchKernelGGL(kern, dim3(sm_grid(P)), dim3(kThreads), lds, s, g, P.sub, P.nsub,
                           (const T *)P.u[0], (const T *)P.u[1], (const T *)P.u[2], P.perm,
                           (const C *)c, (C *)grid, bk);
    } else {
        const bool gm = method == 1;
        hipLaunchKernelGGL((k_spread_gm<T, DIM, W>), dim3(cdiv(P.M, kThreads)), dim3(kThreads),
                           0, s, g, P.M, gm ? P.key_in : P.key,
                           (const T *)(gm ? P.u_in[0] : P.u[0]),
                           (const T *)(gm ? P.u_in[1] : P.u[1]),
                           (const T *)(gm ? P.u_in[2] : P.u[2]), gm ? nullptr : P.perm,
                           (const C *)c, (C *)grid, bk);
    }
    return hipGetLastError();
}

template <typename T, int DIM, int W>
hipError_t interp_w(const Geom &g, int method, const Pts &P, const void *grid, void *c,
                    hipStream_t s, size_t lds)
{
    using C = typename Cplx<T>::type;
    const T bk = kernel_param<T>(g.beta);
    if (method == 3) {
        auto kern = k_interp_sm<T, DIM, W>;
        if (lds > 65536)
            (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds);
        hipLaunchKernelGGL(kern, dim3(sm_grid(P)), dim3(kThreads), lds, s, g, P.sub, P.nsub,
                           (const T *)P.u[0], (const T *)P.u[1], (const T *)P.u[2], P.perm,
                           (const C *)grid, (C *)c, bk);
    } else {
        const bool gm = method == 1;
        hipLaunchKernelGGL((k_interp_gm<T, DIM, W>), dim3(cdiv(P.M, kThreads)), dim3(kThreads),
                           0, s, g, P.M, gm ? P.key_in : P.key,
                           (const T *)(gm ? P.u_in[0] : P.u[0]),
                           (const T *)(gm ? P.u_in[1] : P.u[1]),
                           (const T *)(gm ? P.u_in[2] : P.u[2]), gm ? nullptr : P.perm,
                           (const C *)grid, (C *)c, bk);
    }
    return hipGetLastError();
}

template <typename T, int DIM>
hipError_t spread_dim(const Geom &g, int method, const Pts &P, const void *c, void *grid,
                      hipStream_t s, size_t lds)
{
    switch (g.w) {
#define MN_CASE(WW) case WW: return spread_w<T, DIM, WW>(g, method, P, c, grid, s, lds);
        MN_CASE(2) MN_CASE(3) MN_CASE(4) MN_CASE(5) MN_CASE(6) MN_CASE(7) MN_CASE(8)
        MN_CASE(9) MN_CASE(10) MN_CASE(11) MN_CASE(12) MN_CASE(13) MN_CASE(14)
        MN_CASE(15) MN_CASE(16)
#undef MN_CASE
    }
    return hipErrorInvalidValue;
}

template <typename T, int DIM>
hipError_t interp_dim(const Geom &g, int method, const Pts &P, const void *grid, void *c,
                      hipStream_t s, size_t lds)
{
    switch (g.w) {
#define MN_CASE(WW) case WW: return interp_w<T, DIM, WW>(g, method, P, grid, c, s, lds);
        MN_CASE(2) MN_CASE(3) MN_CASE(4) MN_CASE(5) MN_CASE(6) MN_CASE(7) MN_CASE(8)
        MN_CASE(9) MN_CASE(10) MN_CASE(11) MN_CASE(12) MN_CASE(13) MN_CASE(14)
        MN_CASE(15) MN_CASE(16)
#undef MN_CASE
    }
    return hipErrorInvalidValue;
}

}  // namespace detail
}  // namespace mn
