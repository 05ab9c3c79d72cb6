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
// Strengths (spreading) and results (interpolation) are in the caller's point
// order, reached through the sort permutation; with a null permutation they
// are in bin-sorted order instead (mnufft_execute_sorted).  The SM kernels
// take one index array for this: the input index of each point they
// process, or its sorted position.
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
#include <type_traits>

namespace mn {
namespace detail {

constexpr int kThreads = 256;

template <typename T> struct Cplx;
template <> struct Cplx<float> { using type = float2; };
template <> struct Cplx<double> { using type = double2; };

// 16-byte vector of T, for tile copies.
template <typename T> struct Vec16;
template <> struct Vec16<float> { using type = float4; };
template <> struct Vec16<double> { using type = double2; };
__device__ __forceinline__ void vadd(float4 &a, const float4 &b)
{
    a.x += b.x; a.y += b.y; a.z += b.z; a.w += b.w;
}
__device__ __forceinline__ void vadd(double2 &a, const double2 &b)
{
    a.x += b.x; a.y += b.y;
}

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
// c is read at perm[i]; perm == nullptr reads c[i], i.e. c in the order of
// the coordinate arrays given (input order for GM, sorted order otherwise).
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
    int sy = 0;
    if constexpr (DIM >= 2) sy = taps<T, W>(u1[i], bk, ky) + by * g.m[1];
    const auto cv = c[perm ? perm[i] : i];
    int lx[W];
#pragma unroll
    for (int a = 0; a < W; ++a) lx[a] = wrap1(sx + a, g.n[0]);
    if constexpr (DIM == 1) {
        T *row = reinterpret_cast<T *>(grid);
#pragma unroll
        for (int a1 = 0; a1 < W; ++a1) {
            gadd(row + 2 * lx[a1], cv.x * kx[a1]);
            gadd(row + 2 * lx[a1] + 1, cv.y * kx[a1]);
        }
    } else if constexpr (DIM == 2) {
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
    int sy = 0;
    if constexpr (DIM >= 2) sy = taps<T, W>(u1[i], bk, ky) + by * g.m[1];
    int lx[W];
#pragma unroll
    for (int a = 0; a < W; ++a) lx[a] = wrap1(sx + a, g.n[0]);
    T ar = 0, ai = 0;
    if constexpr (DIM == 1) {
#pragma unroll
        for (int a1 = 0; a1 < W; ++a1) {
            const auto v = grid[lx[a1]];
            ar += v.x * kx[a1];
            ai += v.y * kx[a1];
        }
    } else if constexpr (DIM == 2) {
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

// Partial maxima of max(|Re c_j|, |Im c_j|) for the fixed-point scale of
// k_spread_sm: block b writes out[b]; the consumer takes the max over the
// kMaxParts entries (blocks beyond the launch leave theirs at zero).
constexpr int kMaxParts = 1024;

template <typename T>
__global__ void __launch_bounds__(kThreads)
k_maxabs(const typename Cplx<T>::type *__restrict__ c, int M, T *__restrict__ out)
{
    T m = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < M; i += gridDim.x * blockDim.x) {
        const auto v = c[i];
        m = fmax(m, fmax(fabs(v.x), fabs(v.y)));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    __shared__ T wm[kThreads / 64];
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < kThreads / 64; ++k) m = fmax(m, wm[k]);
        out[blockIdx.x] = m;
    }
}

// max over the kMaxParts partial maxima, by one workgroup of NT threads.
template <typename T, int NT = kThreads>
__device__ __forceinline__ T block_cmax(const T *__restrict__ parts)
{
    __shared__ T red[NT / 64];
    T m = 0;
    for (int k = threadIdx.x; k < kMaxParts; k += NT) m = fmax(m, parts[k]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    m = red[0];
    for (int k = 1; k < NT / 64; ++k) m = fmax(m, red[k]);
    __syncthreads();
    return m;
}

// ----------------------------------------------------------------------------
// Rounding of a scaled contribution to the fixed-point word.
__device__ __forceinline__ long long to_fixed(float v) { return __float2ll_rn(v); }
__device__ __forceinline__ long long to_fixed(double v) { return __double2ll_rn(v); }

// SM spreading, step 2 of Sec. III-A: each subproblem accumulates its points
// into an LDS copy of its padded bin (p_i = m_i + 2 ceil(w/2), offset
// binstart - ceil(w/2)), then stores the tile to its own scratch slot.
// Adding the tiles into the grid (SM step 3) is done without atomics by
// k_tile_merge / k_tile_gather below.
//
// The LDS accumulators are 64-bit fixed point: on gfx950 integer LDS atomics
// (ds_add_u64) sustain roughly ten times the rate of floating-point ones.
// A contribution v = c_j phi phi (phi) becomes round(v S); integer addition
// is exact and associative, so a tile is the same whatever order its atomics
// land in, and only the final cell values have to fit the word.
//
// The scale S of a subproblem comes from a bound on its cells.  A point
// whose first tap (in padded-tile coordinates) is s covers the cells
// s .. s + w - 1 per dimension with weights at most one, so
//   |Re b_l|, |Im b_l| <= sum over points with s in (l - w, l] of a_j,
//   a_j = max(|Re c_j|, |Im c_j|).
// Each subproblem histograms ceil(a_j / u) (u a power of two) over the start
// cells in LDS, takes box sums of width w along x and y and their maximum
// B; B u bounds every cell of the tile.  (In 3D the histogram sums over
// the z start, which bounds each cell too and keeps the sums 2D.)  This is tighter than the
// subproblem's whole strength sum by roughly the ratio of the bin to the
// kernel footprint (about 20x for 32 x 32 bins and w = 6), and it follows
// the strengths where they are: large strengths elsewhere in the input do
// not coarsen this subproblem's quantum.  The histogram and its box sums use
// the tile's own LDS before the tile is cleared.

// Words of a tile with padded extents p1 x p2 (x p3): two per cell,
// rounded up to a multiple of 8 (the layout sm_tile_stride gives a plan).
template <int DIM>
__device__ __forceinline__ int tile_words(int p1, int p2, int p3)
{
    const int cells = DIM == 1 ? p1 : (DIM == 2 ? p1 * p2 : p1 * p2 * p3);
    return (2 * cells + 7) / 8 * 8;
}

// Start cell (first tap in padded-tile coordinates) of a point at
// bin-relative coordinate u: the expression taps() evaluates for u + P
// (start_cell_rt in internal.h, which setpts uses for the same slots).
template <typename T, int W>
__device__ __forceinline__ int start_cell(T u)
{
    return start_cell_rt<T>(u, W);
}

__device__ __forceinline__ int ceil_log2(unsigned v) { return v <= 1u ? 0 : 32 - __clz(v - 1u); }

template <int DIM, int W>
__device__ __forceinline__ StartHist start_hist(int m1, int m2, int m3)
{
    return start_hist_rt(DIM, W, m1, m2, m3);
}

template <int DIM>
__device__ __forceinline__ int hist_slot(const StartHist &h, int s1, int s2, int s3)
{
    return hist_slot_rt(h, DIM >= 2 ? s2 : 0, DIM == 3 ? s3 : 0, s1);
}

// Box sums of width W along a line of `len` slots (stride st) in place, by
// one thread: after the call slot k holds the sum of the original slots
// (k - W, k].
__device__ __forceinline__ void box_in_place(unsigned *H, int len, int st, int W)
{
    unsigned acc = 0;
    for (int k = 0; k < len; ++k) {
        acc += H[k * st];
        H[k * st] = acc;
    }
    for (int k = len - 1; k >= W; --k) H[k * st] -= H[(k - W) * st];
}

// Largest box sum of width W along a line holding `cnt` values (stride st),
// over all cnt + W - 1 window positions, by one thread.
__device__ __forceinline__ unsigned box_max(const unsigned *H, int cnt, int st, int W)
{
    unsigned acc = 0, mx = 0;
    for (int k = 0; k < cnt + W - 1; ++k) {
        if (k < cnt) acc += H[k * st];
        if (k >= W) acc -= H[(k - W) * st];
        mx = max(mx, acc);
    }
    return mx;
}

// The same with one wave per line (window positions <= 64): lane k holds
// position k and adds the W - 1 positions below it by lane shuffles.  Lines
// are line(l) + k st for l < nl, k < cnt (the positions up to npos are zero
// beyond cnt).  In place (box sums written back) or, with mx, the largest
// box sum is folded into *mx instead.
template <typename Line>
__device__ __forceinline__ void box_lines(unsigned *H, int nl, int cnt, int npos, int st, int W,
                                          Line line, unsigned *mx)
{
    const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    for (int l = threadIdx.x >> 6; l < nl; l += nw) {
        unsigned *p = H + line(l);
        const unsigned v = lane < cnt ? p[lane * st] : 0u;
        unsigned sum = v;
        for (int j = 1; j < W; ++j) {
            const unsigned t = (unsigned)__shfl_up((int)v, j, 64);
            if (lane >= j) sum += t;
        }
        if (lane >= npos) sum = 0u;
        if (mx) *mx = max(*mx, sum);
        else if (lane < npos) p[lane * st] = sum;
    }
}

// Largest w-box sum of the start histogram over every cell of the tile
// (all threads of the block call this; it ends with a barrier).  Lines of
// up to 64 window positions are summed one wave per line, longer ones one
// thread per line.  (The histogram is two-dimensional in 3D; see StartHist.)
template <int DIM, int W>
__device__ unsigned tile_bound(unsigned *H, const StartHist &h, unsigned *red)
{
    const int tid = threadIdx.x, NT = blockDim.x;
    unsigned mx = 0;
    if constexpr (DIM == 1) {
        if (h.c[0] + W - 1 <= 64)
            box_lines(H, 1, h.c[0], h.c[0] + W - 1, 1, W, [](int) { return 0; }, &mx);
        else if (tid == 0)
            mx = box_max(H, h.c[0], 1, W);
    } else {
        // along x, in place, then the largest box sum along y
        if (h.lx <= 64)
            box_lines(H, h.c[1], h.c[0], h.lx, 1, W, [&](int r) { return r * h.lx; }, nullptr);
        else
            for (int r = tid; r < h.c[1]; r += NT) box_in_place(H + r * h.lx, h.lx, 1, W);
        __syncthreads();
        if (h.c[1] + W - 1 <= 64)
            box_lines(H, h.lx, h.c[1], h.c[1] + W - 1, h.lx, W, [](int x) { return x; }, &mx);
        else
            for (int x = tid; x < h.lx; x += NT) mx = max(mx, box_max(H + x, h.c[1], h.lx, W));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = max(mx, (unsigned)__shfl_xor((int)mx, o, 64));
    if ((tid & 63) == 0) red[tid >> 6] = mx;
    __syncthreads();
    mx = red[0];
    for (int k = 1; k < NT / 64; ++k) mx = max(mx, red[k]);
    __syncthreads();
    return mx;
}

// SM spreading with two 64-bit words per cell (one per part): double
// precision, and single precision in 1D.  The histogram unit is
// u = 2^(e + ceil(log2 n_q) - 31) with cmax < 2^e the largest part of any
// strength of the vector (k_maxabs) and n_q the subproblem's point count, so
// the histogram's total stays below 2^32; with the box bound B u < 2^E the
// scale is S = 2^(61 - E) and every cell stays below 2^62 in magnitude.
// Grid-stride loop over the subproblem list; the tile is interleaved
// (re, im) with ts2 >= 2 p1 p2 p3 entries per slot (a multiple of 8).
template <typename T, int DIM, int W, bool BATCH>
__global__ void __launch_bounds__(kThreads)
k_spread_sm(Geom g, const int32_t *__restrict__ sub, const int32_t *__restrict__ nsubp,
            const T *__restrict__ u0, const T *__restrict__ u1, const T *__restrict__ u2,
            const int32_t *__restrict__ idx, const uint16_t *__restrict__ hslot,
            const typename Cplx<T>::type *__restrict__ c,
            const T *__restrict__ cmaxp, T *__restrict__ scratch, int ts2, int lts, T bk,
            int stage_cap, const TGeom *__restrict__ tg, const int32_t *__restrict__ bin_t,
            const int32_t *__restrict__ q0p)
{
    using V = typename Vec16<T>::type;
    using C = typename Cplx<T>::type;
    constexpr int NV = 16 / sizeof(T);
    // LDS: the tile (lts words, the launch's largest), then the first
    // stage_cap strengths of the subproblem, gathered once by the histogram
    // pass and read again by the accumulation pass
    extern __shared__ __align__(16) unsigned char smem_raw[];
    unsigned long long *tile = reinterpret_cast<unsigned long long *>(smem_raw);
    unsigned *H = reinterpret_cast<unsigned *>(smem_raw);  // start histogram, before the tile
    C *cs = reinterpret_cast<C *>(tile + lts);
    __shared__ unsigned red[kThreads / 64];
    constexpr int P = (W + 1) / 2;
    const int nsub = *nsubp;
    const int q0 = q0p ? *q0p : 0;
    int ecm;
    frexp(block_cmax(cmaxp), &ecm);  // cmax < 2^ecm
    for (int q = q0 + (int)blockIdx.x; q < nsub; q += gridDim.x) {
        const int4 rec = reinterpret_cast<const int4 *>(sub)[q];
        int m1 = g.m[0], m2 = g.m[1], m3 = g.m[2];
        if constexpr (BATCH) {
            const TGeom &tt =
                tg[bin_t[rec.x]];
            m1 = tt.m[0];
            m2 = tt.m[1];
            m3 = tt.m[2];
        }
        const int p1 = m1 + 2 * P, p2 = m2 + 2 * P;
        // this tile's own words (a batch's ts2 fits its largest bins)
        const int tsz = BATCH ? tile_words<DIM>(p1, p2, m3 + 2 * P) : ts2;
        const StartHist hg = start_hist<DIM, W>(m1, m2, m3);
        const int end = rec.y + rec.z;
        int sh;  // S = 2^sh
        if constexpr (std::is_same<T, float>::value) {
            // single precision (1D): the subproblem's count times the largest
            // part bounds every cell, and 2^-61 of that is far below a float's
            // own rounding, so no box bound (nor its pass over the points)
            sh = 61 - ceil_log2((unsigned)rec.z) - ecm;
        } else {
        // histogram of ceil(a_j / u) over the start cells
        const int hu = 31 - ceil_log2((unsigned)rec.z) - ecm;  // a_j 2^hu < 2^(31 - lg n_q)
        for (int e = threadIdx.x; e < hg.size; e += blockDim.x) H[e] = 0u;
        __syncthreads();
        for (int i = rec.y + threadIdx.x; i < end; i += blockDim.x) {
            const C cv = c[idx[i]];
            if (i - rec.y < stage_cap) cs[i - rec.y] = cv;
            int hs;
            if (hslot) {
                hs = hslot[i];
            } else {
                const int s1 = start_cell<T, W>(u0[i]);
                const int s2 = DIM >= 2 ? start_cell<T, W>(u1[i]) : 0;
                const int s3 = DIM == 3 ? start_cell<T, W>(u2[i]) : 0;
                hs = hist_slot<DIM>(hg, s1, s2, s3);
            }
            const unsigned hv = (unsigned)ceil(ldexp(fmax(fabs(cv.x), fabs(cv.y)), hu));
            atomicAdd(H + hs, hv);
        }
        __syncthreads();
        const unsigned B = tile_bound<DIM, W>(H, hg, red);
        sh = 61 - (ceil_log2(B) - hu);
        }
        for (int e = threadIdx.x; e < tsz; e += blockDim.x) tile[e] = 0ull;
        __syncthreads();
        for (int i = rec.y + threadIdx.x; i < end; i += blockDim.x) {
            T kx[W], ky[W];
            const int sx = taps<T, W>(u0[i] + (T)P, bk, kx);
            int sy = 0;
            if constexpr (DIM >= 2) sy = taps<T, W>(u1[i] + (T)P, bk, ky);
            const C cv = i - rec.y < stage_cap ? cs[i - rec.y] : c[idx[i]];
            const T cr0 = ldexp(cv.x, sh), ci0 = ldexp(cv.y, sh);
            if constexpr (DIM == 1) {
                unsigned long long *row = tile + 2 * sx;
#pragma unroll
                for (int a1 = 0; a1 < W; ++a1) {
                    atomicAdd(row + 2 * a1,
                              (unsigned long long)to_fixed(cr0 * kx[a1]));
                    atomicAdd(row + 2 * a1 + 1,
                              (unsigned long long)to_fixed(ci0 * kx[a1]));
                }
            } else if constexpr (DIM == 2) {
#pragma unroll
                for (int a2 = 0; a2 < W; ++a2) {
                    const T wr = cr0 * ky[a2], wi = ci0 * ky[a2];
                    unsigned long long *row = tile + 2 * ((sy + a2) * p1 + sx);
#pragma unroll
                    for (int a1 = 0; a1 < W; ++a1) {
                        atomicAdd(row + 2 * a1,
                                  (unsigned long long)to_fixed(wr * kx[a1]));
                        atomicAdd(row + 2 * a1 + 1,
                                  (unsigned long long)to_fixed(wi * kx[a1]));
                    }
                }
            } else {
                T z0;
                const int sz = tap_start<T, W>(u2[i] + (T)P, z0);
#pragma unroll 1
                for (int a3 = 0; a3 < W; ++a3) {
                    const T kz = es_val(z0 + (T)a3 * (T)(2.0 / W), bk);
                    const T cr = cr0 * kz, ci = ci0 * kz;
#pragma unroll
                    for (int a2 = 0; a2 < W; ++a2) {
                        const T wr = cr * ky[a2], wi = ci * ky[a2];
                        unsigned long long *row = tile + 2 * (((sz + a3) * p2 + sy + a2) * p1 + sx);
#pragma unroll
                        for (int a1 = 0; a1 < W; ++a1) {
                            atomicAdd(row + 2 * a1,
                                      (unsigned long long)to_fixed(wr * kx[a1]));
                            atomicAdd(row + 2 * a1 + 1,
                                      (unsigned long long)to_fixed(wi * kx[a1]));
                        }
                    }
                }
            }
        }
        __syncthreads();
        V *dst = reinterpret_cast<V *>(scratch + (size_t)q * ts2);
        for (int e = threadIdx.x; e < tsz / NV; e += blockDim.x) {
            T vals[NV];
#pragma unroll
            for (int k = 0; k < NV; ++k)
                vals[k] = (T)ldexp((double)(long long)tile[e * NV + k], -sh);
            V out;
            __builtin_memcpy(&out, vals, sizeof(V));
            dst[e] = out;
        }
        __syncthreads();
    }
}

// SM spreading in single precision with one LDS atomic per tap (2D / 3D).
//
// Same input and output as k_spread_sm<float>, but both parts of a cell share
// one 64-bit LDS word: a contribution (a, b) becomes the integers
// r = round(a S), i = round(b S) and the word is incremented by i 2^32 + r
// (modulo 2^64).  Integer addition is exact, so the word holds
// (sum i) 2^32 + (sum r) as long as both sums stay within int32, and the two
// sums are read back from its low (signed) and high halves.  The histogram
// unit is u = 2^(ea + ceil(log2 n_q) - 31) with 2^ea above every part of the
// subproblem's strengths (a maximum, which unlike a floating-point sum does
// not depend on the order the points are visited in), so the histogram's
// total stays below 2^32; with the box bound B u < 2^E the scale is
// S = 2^(30 - E), which keeps every cell's parts below 2^30 plus at most
// n_q / 2 of rounding.  This halves the
// atomics of the two-word tile, which bound 3D spreading, and halves its LDS.
// The strengths gathered for the scale (up to stage_cap of them) stay in LDS
// for the histogram and the accumulation: the random gather through the
// permutation moves a whole cache line per point and is the kernel's main
// HBM traffic, so it is done once.  The same pass loads the coordinates and
// keeps each point's histogram slot (16 bits) in LDS, so the histogram pass
// reads LDS only.
// (LDS use, the tile plus the staged strengths, allows about three
// workgroups per CU, i.e. three waves per SIMD; the register budget follows.)
template <typename T, int DIM, int W, bool BATCH>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3)))
k_spread_smp(Geom g, const int32_t *__restrict__ sub, const int32_t *__restrict__ nsubp,
             const float *__restrict__ u0, const float *__restrict__ u1,
             const float *__restrict__ u2, const int32_t *__restrict__ idx,
             const uint16_t *__restrict__ hslot, const float2 *__restrict__ c,
             float *__restrict__ scratch, int ts2, int lts, float bk, int stage_cap,
             const TGeom *__restrict__ tg, const int32_t *__restrict__ bin_t,
             const int32_t *__restrict__ q0p)
{
    static_assert(std::is_same<T, float>::value && DIM >= 2, "2D / 3D single precision only");
    constexpr int P = (W + 1) / 2;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    // LDS: the tile (lts / 2 cells, the launch's largest), then the staged
    // strengths; tiles in scratch are ts2 floats apart
    unsigned long long *tile = reinterpret_cast<unsigned long long *>(smem_raw);
    unsigned *H = reinterpret_cast<unsigned *>(smem_raw);  // start histogram, before the tile
    float2 *cs = reinterpret_cast<float2 *>(tile + lts / 2);  // first stage_cap strengths
    unsigned short *slot = reinterpret_cast<unsigned short *>(cs + stage_cap);  // their slots
    __shared__ float red[kThreads / 64];
    __shared__ unsigned redu[kThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int nsub = *nsubp;
    const int q0 = q0p ? *q0p : 0;
    for (int q = q0 + (int)blockIdx.x; q < nsub; q += gridDim.x) {
        const int4 rec = reinterpret_cast<const int4 *>(sub)[q];
        int m1 = g.m[0], m2 = g.m[1], m3 = g.m[2];
        if constexpr (BATCH) {
            const TGeom &tt =
                tg[bin_t[rec.x]];
            m1 = tt.m[0];
            m2 = tt.m[1];
            m3 = tt.m[2];
        }
        const int p1 = m1 + 2 * P, p2 = m2 + 2 * P;
        // this tile's own words (a batch's ts2 fits its largest bins)
        const int tsz = BATCH ? tile_words<DIM>(p1, p2, m3 + 2 * P) : ts2;
        const StartHist hg = start_hist<DIM, W>(m1, m2, m3);
        const int end = rec.y + rec.z;
        // the largest part of any strength and the histogram slots of the
        // staged points (the loads are issued kPre at a time so that their
        // latencies overlap)
        constexpr int kPre = 8;
        float am = 0.f;
        for (int i0 = rec.y + tid; i0 < end; i0 += kPre * kThreads) {
            int pj[kPre], hs[kPre];
#pragma unroll
            for (int k = 0; k < kPre; ++k) {
                const int i = i0 + k * kThreads;
                const bool in = i < end;
                pj[k] = in ? idx[i] : -1;
                const bool st = in && i - rec.y < stage_cap;
                if (hslot) {
                    hs[k] = st ? (int)hslot[i] : 0;
                } else if (st) {
                    hs[k] = hist_slot<DIM>(hg, start_cell<float, W>(u0[i]),
                                           start_cell<float, W>(u1[i]),
                                           DIM == 3 ? start_cell<float, W>(u2[i]) : 0);
                } else {
                    hs[k] = 0;
                }
            }
#pragma unroll
            for (int k = 0; k < kPre; ++k) {
                if (pj[k] >= 0) {
                    const float2 cv = c[pj[k]];
                    am = fmaxf(am, fmaxf(fabsf(cv.x), fabsf(cv.y)));
                    const int j = i0 + k * kThreads - rec.y;
                    if (j < stage_cap) {
                        cs[j] = cv;
                        slot[j] = (unsigned short)hs[k];
                    }
                }
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) am = fmaxf(am, __shfl_xor(am, o, 64));
        if (lane == 0) red[wv] = am;
        for (int e = tid; e < hg.size; e += kThreads) H[e] = 0u;
        __syncthreads();
        float A = 0.f;
        for (int k = 0; k < kThreads / 64; ++k) A = fmaxf(A, red[k]);
        int ea;
        frexpf(A, &ea);  // every part of every strength is below 2^ea
        // histogram unit 2^-hu: each entry is below 2^(31 - lg n_q), so the
        // histogram's total stays below 2^32
        const int hu = 31 - ceil_log2((unsigned)rec.z) - ea;
        // strengths past the staged ones are gathered again
        auto strength = [&](int ii) {
            return ii - rec.y < stage_cap ? cs[ii - rec.y] : c[idx[ii]];
        };
        // histogram of ceil(a_j 2^hu) over the start cells
        for (int i = rec.y + tid; i < end; i += kThreads) {
            const int j = i - rec.y;
            int hs;
            float2 cv;
            if (j < stage_cap) {
                hs = slot[j];
                cv = cs[j];
            } else {
                hs = hslot ? (int)hslot[i]
                           : hist_slot<DIM>(hg, start_cell<float, W>(u0[i]),
                                            start_cell<float, W>(u1[i]),
                                            DIM == 3 ? start_cell<float, W>(u2[i]) : 0);
                cv = c[idx[i]];
            }
            const unsigned hv = (unsigned)ceilf(ldexpf(fmaxf(fabsf(cv.x), fabsf(cv.y)), hu));
            atomicAdd(H + hs, hv);
        }
        __syncthreads();
        const unsigned B = tile_bound<DIM, W>(H, hg, redu);
        // S = 2^sh keeps the cells below 2^30.  A term below 2^22 is rounded
        // to an integer by adding 1.5 2^23 inside the FMA that forms it (the
        // sum's float bits are then that integer plus a constant, removed in
        // the 64-bit word): one instruction instead of a multiply and a
        // two-instruction conversion.  Every term is below 2^22 when
        // S <= 2^(22 - ea).  That scale is taken when it is no coarser than
        // the cells' (dense cells), and for kernels of width 6 or less
        // (tolerances of 1e-5 and looser) when it is at most 8x coarser: the
        // quantum stays below 2^-21 of the largest strength, far below the
        // tolerance.  Otherwise (tight tolerances, or a few strengths far
        // above the rest) the terms are converted.
        constexpr int kCoarser = W <= 6 ? 3 : 0;
        const int sh_cell = 30 - (ceil_log2(B) - hu);
        const bool magic = 22 - ea >= sh_cell - kCoarser;
        const int sh = magic ? min(sh_cell, 22 - ea) : sh_cell;
        for (int e = tid; e < tsz / 2; e += kThreads) tile[e] = 0ull;
        __syncthreads();
        // points of this thread, with the next one's loads issued ahead
        int i = rec.y + tid;
        float nu0 = 0.f, nu1 = 0.f, nu2 = 0.f;
        float2 ncv = make_float2(0.f, 0.f);
        if (i < end) {
            nu0 = u0[i];
            if constexpr (DIM >= 2) nu1 = u1[i];
            if constexpr (DIM == 3) nu2 = u2[i];
            ncv = strength(i);
        }
        for (; i < end; i += kThreads) {
            const float x0 = nu0, x1 = nu1, x2 = nu2;
            const float2 cv = ncv;
            if (i + kThreads < end) {
                nu0 = u0[i + kThreads];
                if constexpr (DIM >= 2) nu1 = u1[i + kThreads];
                if constexpr (DIM == 3) nu2 = u2[i + kThreads];
                ncv = strength(i + kThreads);
            }
            float kx[W], ky[W];
            const int sx = taps<float, W>(x0 + (float)P, bk, kx);
            int sy = 0;
            if constexpr (DIM >= 2) sy = taps<float, W>(x1 + (float)P, bk, ky);
            const float cr0 = ldexpf(cv.x, sh), ci0 = ldexpf(cv.y, sh);
            // contributions are rounded to nearest (ties to even): truncation,
            // or ties away from zero, would bias the terms, and ties are
            // common (a float between 2^22 and 2^23 is a multiple of 1/2)
            auto row_add = [&](unsigned long long *row, float wr, float wi) {
                if (magic) {
                    constexpr float kMagic = 12582912.0f;  // 1.5 2^23
                    constexpr unsigned long long kMagicPair = 0x4B4000004B400000ull;
#pragma unroll
                    for (int a1 = 0; a1 < W; ++a1) {
                        const unsigned lo = __float_as_uint(fmaf(wr, kx[a1], kMagic));
                        const unsigned hi = __float_as_uint(fmaf(wi, kx[a1], kMagic));
                        atomicAdd(row + a1,
                                  (((unsigned long long)hi << 32) | lo) - kMagicPair);
                    }
                } else {
#pragma unroll
                    for (int a1 = 0; a1 < W; ++a1) {
                        const int r = __float2int_rn(wr * kx[a1]);
                        const int im = __float2int_rn(wi * kx[a1]);
                        atomicAdd(row + a1, ((unsigned long long)(unsigned)im << 32) +
                                                (unsigned long long)(long long)r);
                    }
                }
            };
            if constexpr (DIM == 2) {
#pragma unroll
                for (int a2 = 0; a2 < W; ++a2)
                    row_add(tile + (sy + a2) * p1 + sx, cr0 * ky[a2], ci0 * ky[a2]);
            } else {
                float z0;
                const int sz = tap_start<float, W>(x2 + (float)P, z0);
#pragma unroll 1
                for (int a3 = 0; a3 < W; ++a3) {
                    const float kz = es_val(z0 + (float)a3 * (float)(2.0 / W), bk);
                    const float cr = cr0 * kz, ci = ci0 * kz;
#pragma unroll
                    for (int a2 = 0; a2 < W; ++a2)
                        row_add(tile + ((sz + a3) * p2 + sy + a2) * p1 + sx, cr * ky[a2],
                                ci * ky[a2]);
                }
            }
        }
        __syncthreads();
        float4 *dst = reinterpret_cast<float4 *>(scratch + (size_t)q * ts2);
        for (int e = tid; e < tsz / 4; e += kThreads) {
            float v[4];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const long long word = (long long)tile[2 * e + h];
                const int r = (int)(unsigned)(word & 0xffffffffll);
                const long long im = (word - (long long)r) >> 32;
                v[2 * h] = ldexpf((float)r, -sh);
                v[2 * h + 1] = ldexpf((float)im, -sh);
            }
            dst[e] = make_float4(v[0], v[1], v[2], v[3]);
        }
        __syncthreads();
    }
}

// Merge of the tiles of heavily loaded bins: for each leader q (every G-th
// subproblem of a bin holding more than G of them), tiles q .. q+G-1 are
// summed into tile q.  Work items are (leader, chunk of 256 vectors).
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_tile_merge(int32_t *__restrict__ nmergep, const int32_t *__restrict__ mergelist,
             const int32_t *__restrict__ sub, const int32_t *__restrict__ suboff,
             T *__restrict__ scratch, int ts2, int G)
{
    // (nmergep[1] counts the bins the bin-wise add-back lists after this launch)
    if (blockIdx.x == 0 && threadIdx.x == 0) nmergep[1] = 0;
    using V = typename Vec16<T>::type;
    constexpr int NV = 16 / sizeof(T);
    const int nvec = ts2 / NV;
    const int nchunk = (nvec + kThreads - 1) / kThreads;
    const int total = *nmergep * nchunk;
    for (int wi = blockIdx.x; wi < total; wi += gridDim.x) {
        const int q0 = mergelist[wi / nchunk];
        const int v = (wi % nchunk) * kThreads + threadIdx.x;
        if (v >= nvec) continue;
        const int b = reinterpret_cast<const int4 *>(sub)[q0].x;
        const int last = suboff[b + 1];
        const int cnt = min(G, last - q0);
        V *base = reinterpret_cast<V *>(scratch);
        V acc = base[(size_t)q0 * nvec + v];
        for (int j = 1; j < cnt; ++j) vadd(acc, base[(size_t)(q0 + j) * nvec + v]);
        base[(size_t)q0 * nvec + v] = acc;
    }
}

// Each fine-grid cell is the sum of the tile cells that cover it (the wrapped
// add-back of eq. addtoglobal, computed as a gather): per dimension, cov_i
// lists for grid index l the pairs (bin index, offset in that bin's padded
// tile) that land on l, up to kmax_i of them (unused entries have bin -1).
// Bins with more than G tiles are read through their merged leaders.
template <typename T, int DIM, bool BATCH>
__global__ void __launch_bounds__(kThreads)
k_tile_gather(Geom g, const int32_t *__restrict__ suboff, const T *__restrict__ scratch,
              int ts2, int G, const int2 *__restrict__ cov0_, const int2 *__restrict__ cov1_,
              const int2 *__restrict__ cov2_, int k0_, int k1_, int k2_, int P,
              typename Cplx<T>::type *__restrict__ grid, long long ncell_all,
              const TGeom *__restrict__ tg, int T_)
{
    __shared__ long long soff[BATCH ? kTCache : 1];
    const auto fld = [](const TGeom &a) { return a.grid_off; };
    bool cached = false;
    if constexpr (BATCH) cached = cache_offsets(soff, tg, T_, fld);
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < ncell_all;
         e += (long long)gridDim.x * blockDim.x) {
        Geom gg = g;
        const int2 *cov0 = cov0_, *cov1 = cov1_, *cov2 = cov2_;
        int k0 = k0_, k1 = k1_, k2 = k2_, boff = 0;
        long long el = e;
        if constexpr (BATCH) {
            const TGeom &tt =
                tg[cached ? find_cached(soff, T_, e) : find_transform(tg, T_, e, fld)];
            gg = geom_of(g, tt);
            cov0 = cov0_ + tt.cov_off[0];
            cov1 = cov1_ + tt.cov_off[1];
            cov2 = DIM == 3 ? cov2_ + tt.cov_off[2] : cov2_;
            k0 = tt.kmax[0];
            k1 = tt.kmax[1];
            k2 = tt.kmax[2];
            boff = tt.bin_off;
            el = e - tt.grid_off;
        }
        const int p1 = gg.m[0] + 2 * P, p2 = gg.m[1] + 2 * P;
        const int l1 = (int)(el % gg.n[0]);
        const long long r = el / gg.n[0];
        const int l2 = (int)(r % gg.n[1]);
        const int l3 = DIM == 3 ? (int)(r / gg.n[1]) : 0;
        if constexpr (DIM == 1) k1 = 1;  // one row: the single entry (bin 0, offset 0)
        T ar = 0, ai = 0;
        for (int j3 = 0; j3 < (DIM == 3 ? k2 : 1); ++j3) {
            int nb3 = 0, s3 = 0;
            if constexpr (DIM == 3) {
                const int2 c3 = cov2[(size_t)l3 * k2 + j3];
                if (c3.x < 0) break;
                nb3 = c3.x;
                s3 = c3.y;
            }
            for (int j2 = 0; j2 < k1; ++j2) {
                const int2 c2 = DIM >= 2 ? cov1[(size_t)l2 * k1 + j2] : make_int2(0, 0);
                if (c2.x < 0) break;
                for (int j1 = 0; j1 < k0; ++j1) {
                    const int2 c1 = cov0[(size_t)l1 * k0 + j1];
                    if (c1.x < 0) break;
                    const int b = boff + c1.x + gg.B[0] * (c2.x + gg.B[1] * nb3);
                    const int first = suboff[b], k = suboff[b + 1] - first;
                    const int step = k > G ? G : 1;
                    const size_t off = 2 * ((size_t)c1.y + (size_t)p1 * (c2.y + (size_t)p2 * s3));
                    for (int q = first; q < first + k; q += step) {
                        const T *t = scratch + (size_t)q * ts2 + off;
                        ar += t[0];
                        ai += t[1];
                    }
                }
            }
        }
        typename Cplx<T>::type out;
        out.x = ar;
        out.y = ai;
        grid[e] = out;
    }
}

// Fast path of k_tile_gather when every cover table holds at most two
// entries per grid index (bins at least as wide as the halo, the usual case):
// every cell's cover entries, the first tile of each covering bin and those
// tiles' values are loaded in three rounds of independent loads, not one
// dependent chain per covering bin.  The sum is taken in the same order.
template <typename T, int DIM, bool BATCH>
__global__ void __launch_bounds__(kThreads)
k_tile_gather2(Geom g, const int32_t *__restrict__ suboff, const T *__restrict__ scratch,
               int ts2, int G, const int2 *__restrict__ cov0_, const int2 *__restrict__ cov1_,
               const int2 *__restrict__ cov2_, int k0_, int k1_, int k2_, int P,
               typename Cplx<T>::type *__restrict__ grid, long long ncell,
               const TGeom *__restrict__ tg, int T_)
{
    constexpr int NY = DIM >= 2 ? 2 : 1, NZ = DIM == 3 ? 2 : 1, NC = 2 * NY * NZ;
    __shared__ long long soff[BATCH ? kTCache : 1];
    const auto fld = [](const TGeom &a) { return a.grid_off; };
    bool cached = false;
    if constexpr (BATCH) cached = cache_offsets(soff, tg, T_, fld);
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < ncell;
         e += (long long)gridDim.x * blockDim.x) {
        Geom gg = g;
        const int2 *cov0 = cov0_, *cov1 = cov1_, *cov2 = cov2_;
        int k0 = k0_, k1 = k1_, k2 = k2_, boff = 0;
        long long el = e;
        if constexpr (BATCH) {
            const TGeom &tt =
                tg[cached ? find_cached(soff, T_, e) : find_transform(tg, T_, e, fld)];
            gg = geom_of(g, tt);
            cov0 = cov0_ + tt.cov_off[0];
            cov1 = cov1_ + tt.cov_off[1];
            cov2 = DIM == 3 ? cov2_ + tt.cov_off[2] : cov2_;
            k0 = tt.kmax[0];
            k1 = tt.kmax[1];
            k2 = tt.kmax[2];
            boff = tt.bin_off;
            el = e - tt.grid_off;
        }
        const int p1 = gg.m[0] + 2 * P, p2 = gg.m[1] + 2 * P;
        const int l1 = (int)(el % gg.n[0]);
        const long long r = el / gg.n[0];
        const int l2 = (int)(r % gg.n[1]);
        const int l3 = DIM == 3 ? (int)(r / gg.n[1]) : 0;
        int2 c1[2], c2[2], c3[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            c1[j] = j < k0 ? cov0[(size_t)l1 * k0 + j] : make_int2(-1, 0);
            c2[j] = DIM >= 2 ? (j < k1 ? cov1[(size_t)l2 * k1 + j] : make_int2(-1, 0))
                             : make_int2(j == 0 ? 0 : -1, 0);
            c3[j] = (DIM == 3 && j < k2) ? cov2[(size_t)l3 * k2 + j] : make_int2(j == 0 ? 0 : -1, 0);
        }
        int bin[NC];
        size_t off[NC];
#pragma unroll
        for (int j3 = 0; j3 < NZ; ++j3)
#pragma unroll
            for (int j2 = 0; j2 < NY; ++j2)
#pragma unroll
                for (int j1 = 0; j1 < 2; ++j1) {
                    const int v = (j3 * NY + j2) * 2 + j1;
                    const bool ok = c1[j1].x >= 0 && c2[j2].x >= 0 && c3[j3].x >= 0;
                    bin[v] = ok ? boff + c1[j1].x + gg.B[0] * (c2[j2].x + gg.B[1] * c3[j3].x) : -1;
                    off[v] = 2 * ((size_t)c1[j1].y +
                                  (size_t)p1 * (c2[j2].y + (size_t)p2 * c3[j3].y));
                }
        int first[NC], cnt[NC];
#pragma unroll
        for (int v = 0; v < NC; ++v) {
            first[v] = bin[v] >= 0 ? suboff[bin[v]] : 0;
            cnt[v] = bin[v] >= 0 ? suboff[bin[v] + 1] - first[v] : 0;
        }
        T ar = 0, ai = 0;
#pragma unroll
        for (int v = 0; v < NC; ++v) {
            if (cnt[v] > 0) {
                const T *t = scratch + (size_t)first[v] * ts2 + off[v];
                ar += t[0];
                ai += t[1];
            }
            const int step = cnt[v] > G ? G : 1;
            for (int q = first[v] + step; q < first[v] + cnt[v]; q += step) {
                const T *t = scratch + (size_t)q * ts2 + off[v];
                ar += t[0];
                ai += t[1];
            }
        }
        typename Cplx<T>::type out;
        out.x = ar;
        out.y = ai;
        grid[e] = out;
    }
}

// Bin-oriented add-back, for grids whose bins (the last one of a dimension
// possibly narrower, n_i - (B_i - 1) m_i) are all at least two halos wide:
// a workgroup writes the cells of one bin.  Per dimension a cell at
// bin-relative r of a bin of width mb is covered by its own bin's tile (at
// r + P) and, within P of an edge, by one neighbour's, periodically: at
// r + mp + P in the previous bin (width mp) if r < P, at r - mb + P in the
// next if r >= mb - P.  With the tile lists of the 3^d neighbouring bins read
// once per workgroup every tile value is one independent load.  A cell's
// tiles are summed own tile first in each dimension (x fastest), then in
// list order, each bin's tiles in subproblem order.
//
// Two passes.  HEAVY = false takes every bin whose neighbourhood holds at
// most one tile per bin (CPT cells per thread loaded before any is summed;
// neighbouring bins read pieces of the same tile rows, so each XCD takes a
// contiguous range of bins: 3D 0.244 -> 0.222 ms at n = 256^3) and appends
// the other bins to `heavy` (count in cnt[1], cleared by k_tile_merge).
// HEAVY = true splits each listed bin over kSlices workgroups, one cell per
// thread, the further tiles of a bin loaded kBurst at a time: a bin of
// clustered points may hold dozens of tiles, and one workgroup summing them
// alone would hold up the whole launch.
constexpr int kSlices = 4;
template <typename T, int DIM, bool HEAVY>
__global__ void __launch_bounds__(kThreads)
k_tile_sum(Geom g, const int32_t *__restrict__ suboff, const T *__restrict__ scratch, int ts2,
           int G, int P, typename Cplx<T>::type *__restrict__ grid, int32_t *__restrict__ heavy,
           int32_t *__restrict__ cnt)
{
    using C = typename Cplx<T>::type;
    constexpr int NB = DIM == 3 ? 27 : 9;
    constexpr int NC = DIM == 3 ? 8 : 4;   // tile combinations per cell, at most
    constexpr int CPT = HEAVY ? 1 : (sizeof(T) == 4 ? 2 : 1);
    constexpr int kBurst = 8;
    __shared__ int sfirst[NB], scnt[NB];
    const int p1 = g.m[0] + 2 * P, p2 = g.m[1] + 2 * P;
    const int nwork = HEAVY ? cnt[1] * kSlices : g.nbins;
    for (int w = xcd_block(blockIdx.x, gridDim.x); w < nwork; w += gridDim.x) {
        const int b = HEAVY ? heavy[w / kSlices] : w;
        const int slice = HEAVY ? w % kSlices : 0;
        const int b1 = b % g.B[0], b23 = b / g.B[0];
        const int b2 = b23 % g.B[1], b3 = DIM == 3 ? b23 / g.B[1] : 0;
        const int bb[3] = {b1, b2, b3};
        int mb[3], mp[3];  // width of this bin and of the previous one, per dimension
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int last = d < DIM ? g.n[d] - (g.B[d] - 1) * g.m[d] : 1;
            const int m = d < DIM ? g.m[d] : 1;
            mb[d] = bb[d] == g.B[d] - 1 ? last : m;
            mp[d] = bb[d] == 0 ? last : m;
        }
        const int m1 = mb[0], m2 = mb[1], m3 = mb[2];
        const int ncb = m1 * m2 * m3;
        __syncthreads();  // the previous bin's lists are no longer read
        if (threadIdx.x < NB) {
            const int j1 = threadIdx.x % 3, j2 = (threadIdx.x / 3) % 3, j3 = threadIdx.x / 9;
            const int n1 = (b1 + j1 - 1 + g.B[0]) % g.B[0];
            const int n2 = (b2 + j2 - 1 + g.B[1]) % g.B[1];
            const int n3 = DIM == 3 ? (b3 + j3 - 1 + g.B[2]) % g.B[2] : 0;
            const int nb = n1 + g.B[0] * (n2 + g.B[1] * n3);
            const int f = suboff[nb];
            sfirst[threadIdx.x] = f;
            scnt[threadIdx.x] = suboff[nb + 1] - f;
        }
        __syncthreads();
        if constexpr (!HEAVY) {
            bool several = false;
#pragma unroll
            for (int l = 0; l < NB; ++l) several = several || scnt[l] > 1;
            if (several) {  // the same for the whole workgroup
                if (threadIdx.x == 0) heavy[atomicAdd(&cnt[1], 1)] = b;
                continue;
            }
        }
        const int cstep = (HEAVY ? kSlices : CPT) * kThreads;
        for (int c0 = slice * kThreads + threadIdx.x; c0 < ncb; c0 += cstep) {
            int lst[CPT][NC];      // neighbour list of each combination (-1: none)
            int off[CPT][NC];      // offset of the cell in that neighbour's tiles (reals)
            T vr[CPT][NC], vi[CPT][NC];
#pragma unroll
            for (int k = 0; k < CPT; ++k) {
                const int c = c0 + k * kThreads;
                const int r1 = c % m1, r12 = c / m1;
                const int r2 = r12 % m2, r3 = DIM == 3 ? r12 / m2 : 0;
                // per dimension: [0] own tile, [1] the neighbour's (j = -1 when none)
                int j[3][2], s[3][2];
                const int rr[3] = {r1, r2, r3};
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    j[d][0] = 1;
                    s[d][0] = rr[d] + P;
                    j[d][1] = -1;
                    s[d][1] = 0;
                    if (d < DIM) {
                        if (rr[d] < P) {
                            j[d][1] = 0;
                            s[d][1] = rr[d] + mp[d] + P;
                        } else if (rr[d] >= mb[d] - P) {
                            j[d][1] = 2;
                            s[d][1] = rr[d] - mb[d] + P;
                        }
                    } else {
                        j[d][0] = 0;
                        s[d][0] = 0;
                    }
                }
#pragma unroll
                for (int v = 0; v < NC; ++v) {
                    const int a1 = v & 1, a2 = (v >> 1) & 1, a3 = DIM == 3 ? (v >> 2) & 1 : 0;
                    const bool ok = c < ncb && j[0][a1] >= 0 && j[1][a2] >= 0 && j[2][a3] >= 0;
                    lst[k][v] = ok ? (j[2][a3] * 3 + j[1][a2]) * 3 + j[0][a1] : -1;
                    off[k][v] = 2 * (s[0][a1] + p1 * (s[1][a2] + p2 * s[2][a3]));
                }
            }
            // first tile of every combination, all loads in flight together
#pragma unroll
            for (int k = 0; k < CPT; ++k)
#pragma unroll
                for (int v = 0; v < NC; ++v) {
                    vr[k][v] = 0;
                    vi[k][v] = 0;
                    const int l = lst[k][v];
                    if (l >= 0 && scnt[l] > 0) {
                        const C t = *reinterpret_cast<const C *>(
                            scratch + (size_t)sfirst[l] * ts2 + off[k][v]);
                        vr[k][v] = t.x;
                        vi[k][v] = t.y;
                    }
                }
#pragma unroll
            for (int k = 0; k < CPT; ++k) {
                const int c = c0 + k * kThreads;
                if (c >= ncb) break;
                T ar = 0, ai = 0;
#pragma unroll
                for (int v = 0; v < NC; ++v) {
                    const int l = lst[k][v];
                    if (l < 0) continue;
                    ar += vr[k][v];
                    ai += vi[k][v];
                    if constexpr (HEAVY) {
                        const int first = sfirst[l], end = first + scnt[l];
                        const int step = scnt[l] > G ? G : 1;
                        for (int q = first + step; q < end; q += kBurst * step) {
                            T tr[kBurst], ti[kBurst];
#pragma unroll
                            for (int u = 0; u < kBurst; ++u) {
                                tr[u] = 0;
                                ti[u] = 0;
                                if (q + u * step < end) {
                                    const C t = *reinterpret_cast<const C *>(
                                        scratch + (size_t)(q + u * step) * ts2 + off[k][v]);
                                    tr[u] = t.x;
                                    ti[u] = t.y;
                                }
                            }
#pragma unroll
                            for (int u = 0; u < kBurst; ++u) {
                                ar += tr[u];
                                ai += ti[u];
                            }
                        }
                    }
                }
                const int r1 = c % m1, r12 = c / m1;
                const int r2 = r12 % m2, r3 = DIM == 3 ? r12 / m2 : 0;
                const size_t e = (size_t)(b1 * g.m[0] + r1) +
                                 (size_t)g.n[0] * ((size_t)(b2 * g.m[1] + r2) +
                                                   (size_t)g.n[1] * (size_t)(b3 * g.m[2] + r3));
                C o;
                o.x = ar;
                o.y = ai;
                grid[e] = o;
            }
        }
    }
}

// SM interpolation: stage the padded bin in LDS, then every point of the
// subproblem reads its w^d values there.
template <typename T, int DIM, int W, bool BATCH>
__global__ void __launch_bounds__(kThreads)
k_interp_sm(Geom g, const int32_t *__restrict__ sub, const int32_t *__restrict__ nsubp,
            const T *__restrict__ u0, const T *__restrict__ u1, const T *__restrict__ u2,
            const int32_t *__restrict__ idx, const typename Cplx<T>::type *__restrict__ grid_,
            typename Cplx<T>::type *__restrict__ c, T bk, const TGeom *__restrict__ tg,
            const int32_t *__restrict__ bin_t, const int32_t *__restrict__ q0p)
{
    using C = typename Cplx<T>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *tile = reinterpret_cast<C *>(smem_raw);
    constexpr int P = (W + 1) / 2;
    const int nsub = *nsubp;
    const int q0 = q0p ? *q0p : 0;
    for (int q = q0 + (int)blockIdx.x; q < nsub; q += gridDim.x) {
        const int4 rec = reinterpret_cast<const int4 *>(sub)[q];
        int b = rec.x;
        Geom gg = g;
        const C *grid = grid_;
        if constexpr (BATCH) {
            const TGeom &tt =
                tg[bin_t[rec.x]];
            gg = geom_of(g, tt);
            grid = grid_ + tt.grid_off;
            b -= tt.bin_off;
        }
        const int p1 = gg.m[0] + 2 * P, p2 = DIM >= 2 ? gg.m[1] + 2 * P : 1;
        const int p3 = DIM == 3 ? gg.m[2] + 2 * P : 1;
        const int tsize = p1 * p2 * p3;
        const int bx = b % gg.B[0]; b /= gg.B[0];
        const int by = b % gg.B[1]; b /= gg.B[1];
        const int bz = b;
        const int o1 = bx * gg.m[0] - P, o2 = DIM >= 2 ? by * gg.m[1] - P : 0;
        const int o3 = DIM == 3 ? bz * gg.m[2] - P : 0;
        // The results of the previous subproblem may still be in flight; on
        // this GPU one counter tracks vector loads and stores together, so a
        // wait for a load also waits for the stores issued before it.  Loads
        // are therefore issued kStage at a time here, and one point ahead in
        // the loop below, so that each wait covers several of them.
        constexpr int kStage = 4;
        for (int e0 = threadIdx.x; e0 < tsize; e0 += kStage * blockDim.x) {
            C v[kStage];
#pragma unroll
            for (int k = 0; k < kStage; ++k) {
                const int e = e0 + k * blockDim.x;
                if (e < tsize) {
                    const int s1 = e % p1, r = e / p1;
                    const int s2 = r % p2, s3 = r / p2;
                    const int l1 = wrapmod(o1 + s1, gg.n[0]);
                    const int l2 = DIM >= 2 ? wrapmod(o2 + s2, gg.n[1]) : 0;
                    const int l3 = DIM == 3 ? wrapmod(o3 + s3, gg.n[2]) : 0;
                    v[k] = grid[((size_t)l3 * gg.n[1] + l2) * gg.n[0] + l1];
                }
            }
#pragma unroll
            for (int k = 0; k < kStage; ++k)
                if (e0 + k * (int)blockDim.x < tsize) tile[e0 + k * blockDim.x] = v[k];
        }
        __syncthreads();
        const int end = rec.y + rec.z;
        const int NT = blockDim.x;
        // Round r of the subproblem's points is thread t's point rec.y + t + r NT.
        // Its loads are issued kAhead rounds before its use: one counter tracks
        // vector loads and stores together, so waiting for a load also waits
        // for every store issued before it, and the scattered result stores
        // are slow to complete.  Every load is unconditional (lanes past the
        // last point take the last point again and store the same value to
        // the same place), so the compiler can wait for exactly the loads it
        // needs.  The deeper the ring, the older the stores a wait covers:
        // 16 rounds in 2D single precision (2D default workload 0.234 ->
        // 0.173 ms against 4), 4 elsewhere: 3D's 216-tap reads need the
        // registers (6 rounds: 0.76 -> 0.80 ms), and 1D got slower with 16
        // (0.231 -> 0.256 ms).
        constexpr int kAhead = (DIM == 2 && sizeof(T) == 4) ? 16 : 4;
        const int nr = (rec.z + NT - 1) / NT;  // rounds, the same for every thread
        T a0[kAhead], a1[kAhead], a2[kAhead];
        int ap[kAhead];
        auto load_round = [&](int r, int k) {
            const int ii = min(rec.y + (int)threadIdx.x + r * NT, end - 1);
            a0[k] = u0[ii];
            a1[k] = DIM >= 2 ? u1[ii] : (T)0;
            a2[k] = DIM == 3 ? u2[ii] : (T)0;
            ap[k] = idx[ii];
        };
#pragma unroll
        for (int k = 0; k < kAhead; ++k) load_round(k, k);
        for (int r0 = 0; r0 < nr; r0 += kAhead) {
#pragma unroll
        for (int k = 0; k < kAhead; ++k) {
            if (r0 + k >= nr) continue;
            const T x0 = a0[k], x1 = a1[k], x2 = a2[k];
            const int pj = ap[k];
            load_round(r0 + k + kAhead, k);
            T kx[W], ky[W];
            const int sx = taps<T, W>(x0 + (T)P, bk, kx);
            int sy = 0;
            if constexpr (DIM >= 2) sy = taps<T, W>(x1 + (T)P, bk, ky);
            T ar = 0, ai = 0;
            if constexpr (DIM == 1) {
                const C *row = tile + sx;
#pragma unroll
                for (int a1 = 0; a1 < W; ++a1) {
                    const C v = row[a1];
                    ar += v.x * kx[a1];
                    ai += v.y * kx[a1];
                }
            } else if constexpr (DIM == 2) {
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
                const int sz = tap_start<T, W>(x2 + (T)P, z0);
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
            c[pj] = out;
        }
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

// Index array of the SM kernels: the input index of each processed point
// (strength / result in the caller's order), or for vectors kept in
// bin-sorted order its sorted position.
inline const int32_t *sm_index(const Pts &P) { return P.perm ? P.perm : P.spos; }

// Persistent grid size for the subproblem loops.
inline int sm_grid(const Pts &P) { return std::max(1, std::min(P.nsub_max, 256 * 16)); }

// ----------------------------------------------------------------------------
// Position gradient by ES-derivative interpolation.  For a field b on the
// fine grid and weights v_j (one complex per point), with
//   c_j = sum_l b_l prod_i phi(z_i),  z_i = 2 (l_i - g_i) / w,  g_i = (x_i + pi) n_i / (2 pi),
// the kernel returns out_i[j] = sum_t Re(conj(v_tj) dc_tj / dx_i) with
//   dc_j / dx_i = -(n_i / (pi w)) sum_l b_l phi'(z_i) prod_{i' != i} phi(z_i'),
//   phi'(z) = -beta z / sqrt(1 - z^2) phi(z)   (0 where 1 - z^2 <= 0).
// Reads the grid straight from memory in bin-sorted order.
template <typename T>
__device__ __forceinline__ void es_val_der(T z, T bk, T beta, T &v, T &dv)
{
    const T t = (T)1 - z * z;
    if (t <= (T)0) {
        v = es_val(z, bk);
        dv = 0;
        return;
    }
    const T r = sqrt(t);
    v = es_val(z, bk);
    dv = -beta * z / r * v;
}

template <typename T, int W>
__device__ __forceinline__ int taps_der(T u, T bk, T beta, T (&k)[W], T (&dk)[W])
{
    const T s = ceil(u - (T)(0.5 * W));
    const T z0 = (s - u) * (T)(2.0 / W);
#pragma unroll
    for (int a = 0; a < W; ++a) es_val_der(z0 + (T)a * (T)(2.0 / W), bk, beta, k[a], dk[a]);
    return (int)s;
}

template <typename T, int DIM, int W>
__global__ void __launch_bounds__(kThreads)
k_interp_grad(Geom g, int M, int ntransf, const uint32_t *__restrict__ key,
              const T *__restrict__ u0, const T *__restrict__ u1, const T *__restrict__ u2,
              const int32_t *__restrict__ perm, const typename Cplx<T>::type *__restrict__ grid,
              const typename Cplx<T>::type *__restrict__ wts, T *__restrict__ o0,
              T *__restrict__ o1, T *__restrict__ o2, T bk, T beta)
{
    using C = typename Cplx<T>::type;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    uint32_t b = key[i];
    const int bx = b % g.B[0]; b /= g.B[0];
    const int by = b % g.B[1]; b /= g.B[1];
    const int bz = b;
    T kx[W], ky[W], dkx[W], dky[W];
    const int sx = taps_der<T, W>(u0[i], bk, beta, kx, dkx) + bx * g.m[0];
    int sy = 0;
    if constexpr (DIM >= 2) {
        sy = taps_der<T, W>(u1[i], bk, beta, ky, dky) + by * g.m[1];
    } else {
        ky[0] = 1;  // one row, weight one
        dky[0] = 0;
    }
    T kz[W], dkz[W];
    int sz = 0;
    if constexpr (DIM == 3) sz = taps_der<T, W>(u2[i], bk, beta, kz, dkz) + bz * g.m[2];
    int lx[W];
#pragma unroll
    for (int a = 0; a < W; ++a) lx[a] = wrap1(sx + a, g.n[0]);
    const size_t ncell = (size_t)g.n[0] * (DIM >= 2 ? g.n[1] : 1) * (DIM == 3 ? g.n[2] : 1);
    const int j = perm[i];
    T acc[3] = {0, 0, 0};
    for (int t = 0; t < ntransf; ++t) {
        const C *gt = grid + (size_t)t * ncell;
        // D_i = sum over taps of b * (derivative in dimension i) as complex
        T dr[3] = {0, 0, 0}, di[3] = {0, 0, 0};
        for (int a3 = 0; a3 < (DIM == 3 ? W : 1); ++a3) {
            T wz = 1, dwz = 0;
            size_t plane = 0;
            if constexpr (DIM == 3) {
                wz = kz[a3];
                dwz = dkz[a3];
                plane = (size_t)wrap1(sz + a3, g.n[2]) * g.n[1];
            }
#pragma unroll
            for (int a2 = 0; a2 < (DIM >= 2 ? W : 1); ++a2) {
                const C *row = gt + (plane + (DIM >= 2 ? (size_t)wrap1(sy + a2, g.n[1]) : 0)) * g.n[0];
                T sr = 0, si = 0, xr = 0, xi = 0;  // sum b kx, sum b dkx along the row
#pragma unroll
                for (int a1 = 0; a1 < W; ++a1) {
                    const C v = row[lx[a1]];
                    sr += v.x * kx[a1];
                    si += v.y * kx[a1];
                    xr += v.x * dkx[a1];
                    xi += v.y * dkx[a1];
                }
                dr[0] += xr * ky[a2] * wz;
                di[0] += xi * ky[a2] * wz;
                if constexpr (DIM >= 2) {
                    dr[1] += sr * dky[a2] * wz;
                    di[1] += si * dky[a2] * wz;
                }
                if constexpr (DIM == 3) {
                    dr[2] += sr * ky[a2] * dwz;
                    di[2] += si * ky[a2] * dwz;
                }
            }
        }
        const C v = wts[(size_t)t * M + j];
#pragma unroll
        for (int d = 0; d < DIM; ++d) acc[d] += v.x * dr[d] + v.y * di[d];  // Re(conj(v) D)
    }
    T *outs[3] = {o0, o1, o2};
#pragma unroll
    for (int d = 0; d < DIM; ++d) outs[d][j] = acc[d] * (-(T)g.n[d] / ((T)3.141592653589793 * (T)W));
}

template <typename T, int DIM, int W>
hipError_t grad_w(const Geom &g, const Pts &P, int ntransf, const void *grid, const void *wts,
                  void *const out[3], hipStream_t s)
{
    using C = typename Cplx<T>::type;
    hipLaunchKernelGGL((k_interp_grad<T, DIM, W>), dim3(cdiv(P.M, kThreads)), dim3(kThreads), 0,
                       s, g, P.M, ntransf, P.key, (const T *)P.u[0], (const T *)P.u[1],
                       (const T *)P.u[2], P.perm, (const C *)grid, (const C *)wts, (T *)out[0],
                       (T *)out[1], (T *)out[2], kernel_param<T>(g.beta), (T)g.beta);
    return hipGetLastError();
}

template <typename T, int DIM>
hipError_t grad_dim(const Geom &g, const Pts &P, int ntransf, const void *grid, const void *wts,
                    void *const out[3], hipStream_t s)
{
    switch (g.w) {
#define MN_CASE(WW) case WW: return grad_w<T, DIM, WW>(g, P, ntransf, grid, wts, out, s);
        MN_CASE(2) MN_CASE(3) MN_CASE(4) MN_CASE(5) MN_CASE(6) MN_CASE(7) MN_CASE(8)
        MN_CASE(9) MN_CASE(10) MN_CASE(11) MN_CASE(12) MN_CASE(13) MN_CASE(14)
        MN_CASE(15) MN_CASE(16)
#undef MN_CASE
    }
    return hipErrorInvalidValue;
}

// part: bit 0 = accumulate (all methods), bit 1 = SM add-back (merge + gather),
// bit 2 = SM max|c| pre-pass.  P.tg != nullptr selects the batched kernels.
template <typename T, int DIM, int W, bool BATCH>
hipError_t spread_wb(const Geom &g, int method, const Pts &P, const void *c, void *grid,
                     hipStream_t s, size_t lds, int part)
{
    using C = typename Cplx<T>::type;
    const T bk = kernel_param<T>(g.beta);
    if (method == 3) {
        // the packed single-precision kernel (2D / 3D) scales per subproblem
        // and needs no max|c|
        constexpr bool packed = std::is_same<T, float>::value && DIM >= 2;
        if ((part & 4) && !packed) {
            hipLaunchKernelGGL(k_maxabs<T>, dim3(std::max(1, std::min(cdiv(P.M, kThreads), kMaxParts))),
                               dim3(kThreads), 0, s, (const C *)c, P.M, (T *)P.cmax);
        }
        if (part & 1) {
            if constexpr (packed) {
                auto pk = k_spread_smp<T, DIM, W, BATCH>;
                if (lds > 65536)
                    (void)hipFuncSetAttribute((const void *)pk,
                                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
                hipLaunchKernelGGL(pk, dim3(sm_grid(P)), dim3(kThreads), lds, s, g, P.sub,
                                   P.nsub, (const float *)P.u[0], (const float *)P.u[1],
                                   (const float *)P.u[2], sm_index(P), P.hslot, (const float2 *)c,
                                   (float *)P.scratch, P.ts2, sm_tile_stride(g), (float)bk,
                                   smp_stage(DIM, P.msub), P.tg, P.bin_t, P.q0);
            } else {
                auto kern = k_spread_sm<T, DIM, W, BATCH>;
                if (lds > 65536)
                    (void)hipFuncSetAttribute((const void *)kern,
                                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
                hipLaunchKernelGGL(kern, dim3(sm_grid(P)), dim3(kThreads), lds, s, g, P.sub,
                                   P.nsub, (const T *)P.u[0], (const T *)P.u[1], (const T *)P.u[2],
                                   sm_index(P), P.hslot, (const C *)c, (const T *)P.cmax,
                                   (T *)P.scratch, P.ts2, sm_tile_stride(g), bk,
                                   sm2_stage(DIM, sizeof(T) == 4 ? 0 : 1, P.msub), P.tg,
                                   P.bin_t, P.q0);
            }
        }
        if (!(part & 2)) return hipGetLastError();
        const int nvec = P.ts2 / (16 / (int)sizeof(T));
        const int nchunk = (nvec + kThreads - 1) / kThreads;
        const int mgrid = std::max(1, std::min(P.nsub_max / std::max(P.G, 1) * nchunk + nchunk, 8192));
        hipLaunchKernelGGL(k_tile_merge<T>, dim3(mgrid), dim3(kThreads), 0, s, P.nmerge,
                           P.mergelist, P.sub, P.suboff, (T *)P.scratch, P.ts2, P.G);
        if constexpr (!BATCH && DIM >= 2) {
            bool wide = true;  // every bin, the last one included, two halos wide
            for (int d = 0; d < DIM; ++d) {
                const int last = g.n[d] - (g.B[d] - 1) * g.m[d];
                wide = wide && std::min(g.m[d], last) >= 2 * ((W + 1) / 2);
            }
            if (wide && P.heavy) {
                // bins of one tile per neighbourhood, then the listed others
                hipLaunchKernelGGL((k_tile_sum<T, DIM, false>), dim3(std::min(g.nbins, 1 << 20)),
                                   dim3(kThreads), 0, s, g, P.suboff, (const T *)P.scratch,
                                   P.ts2, P.G, (W + 1) / 2, (C *)grid, P.heavy, P.nmerge);
                hipLaunchKernelGGL((k_tile_sum<T, DIM, true>),
                                   dim3(std::min(g.nbins * kSlices, 2048)), dim3(kThreads), 0, s,
                                   g, P.suboff, (const T *)P.scratch, P.ts2, P.G, (W + 1) / 2,
                                   (C *)grid, P.heavy, P.nmerge);
                return hipGetLastError();
            }
        }
        const long long ncell = P.ncells;
        const int ggrid = (int)std::min<long long>((ncell + kThreads - 1) / kThreads, 16384);
        // (for a batch, P.kmax holds the largest table width over its transforms)
        if (P.kmax[0] <= 2 && (DIM == 1 || P.kmax[1] <= 2) && (DIM <= 2 || P.kmax[2] <= 2)) {
            hipLaunchKernelGGL((k_tile_gather2<T, DIM, BATCH>), dim3(std::max(ggrid, 1)),
                               dim3(kThreads), 0, s, g, P.suboff, (const T *)P.scratch, P.ts2,
                               P.G, P.cov[0], P.cov[1], P.cov[2], P.kmax[0], P.kmax[1],
                               P.kmax[2], (W + 1) / 2, (C *)grid, ncell, P.tg, P.T);
            return hipGetLastError();
        }
        hipLaunchKernelGGL((k_tile_gather<T, DIM, BATCH>), dim3(std::max(ggrid, 1)), dim3(kThreads),
                           0, s, g, P.suboff, (const T *)P.scratch, P.ts2, P.G, P.cov[0], P.cov[1],
                           P.cov[2], P.kmax[0], P.kmax[1], P.kmax[2], (W + 1) / 2, (C *)grid, ncell,
                           P.tg, P.T);
    } else if (part & 1) {
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
hipError_t spread_w(const Geom &g, int method, const Pts &P, const void *c, void *grid,
                    hipStream_t s, size_t lds, int part)
{
    if (P.tg) return spread_wb<T, DIM, W, true>(g, method, P, c, grid, s, lds, part);
    return spread_wb<T, DIM, W, false>(g, method, P, c, grid, s, lds, part);
}

template <typename T, int DIM, int W, bool BATCH>
hipError_t interp_wb(const Geom &g, int method, const Pts &P, const void *grid, void *c,
                     hipStream_t s, size_t lds)
{
    using C = typename Cplx<T>::type;
    const T bk = kernel_param<T>(g.beta);
    if (method == 3) {
        auto kern = k_interp_sm<T, DIM, W, BATCH>;
        if (lds > 65536)
            (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)lds);
        hipLaunchKernelGGL(kern, dim3(sm_grid(P)), dim3(kThreads), lds, s, g, P.sub, P.nsub,
                           (const T *)P.u[0], (const T *)P.u[1], (const T *)P.u[2], sm_index(P),
                           (const C *)grid, (C *)c, bk, P.tg, P.bin_t, P.q0);
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

template <typename T, int DIM, int W>
hipError_t interp_w(const Geom &g, int method, const Pts &P, const void *grid, void *c,
                    hipStream_t s, size_t lds)
{
    if (P.tg) return interp_wb<T, DIM, W, true>(g, method, P, grid, c, s, lds);
    return interp_wb<T, DIM, W, false>(g, method, P, grid, c, s, lds);
}

template <typename T, int DIM>
hipError_t spread_dim(const Geom &g, int method, const Pts &P, const void *c, void *grid,
                      hipStream_t s, size_t lds, int part)
{
    switch (g.w) {
#define MN_CASE(WW) case WW: return spread_w<T, DIM, WW>(g, method, P, c, grid, s, lds, part);
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
