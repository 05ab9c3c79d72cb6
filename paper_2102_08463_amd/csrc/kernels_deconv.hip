// Correction steps around the fine-grid FFT (Sec. II-A step 3 and Sec. II-B
// step 1): one thread per output element, per the embarrassingly parallel
// scheme of Sec. III.
//
// Mode k in I_N (ascending from -floor(N/2)) lives at fine-grid index k mod n.
// The factors p_i[k] = (2/w) / phi_hat(alpha_i k) are separable; the library
// stores them with the lattice phase (-1)^k folded in (grid point l sits at
// l h - pi), so both corrections are a plain product.
#include "internal.h"

#include <algorithm>

namespace mn {
namespace {

constexpr int kThreads = 256;

template <typename T> struct Cplx;
template <> struct Cplx<float> { using type = float2; };
template <> struct Cplx<double> { using type = double2; };

// Type 1: f[t][i3][i2][i1] = p1[i1] p2[i2] p3[i3] bhat[t][k3 mod n3][k2 mod n2][k1 mod n1].
// One block row per (t, i3, i2); blockIdx.x = row * chunks + chunk.
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_deconv(int N1, int N2, int N3, int n1, int n2, int n3, int chunks,
         const typename Cplx<T>::type *__restrict__ grid, const T *__restrict__ p1,
         const T *__restrict__ p2, const T *__restrict__ p3,
         typename Cplx<T>::type *__restrict__ f)
{
    const int64_t row = blockIdx.x / chunks;
    const int i1 = (int)(blockIdx.x % chunks) * kThreads + threadIdx.x;
    if (i1 >= N1) return;
    const int i2 = (int)(row % N2);
    const int64_t r3 = row / N2;
    const int i3 = (int)(r3 % N3);
    const int64_t t = r3 / N3;
    const int k1 = i1 - N1 / 2, k2 = i2 - N2 / 2, k3 = i3 - N3 / 2;
    const int l1 = k1 < 0 ? k1 + n1 : k1;
    const int l2 = k2 < 0 ? k2 + n2 : k2;
    const int l3 = k3 < 0 ? k3 + n3 : k3;
    const size_t src = (((size_t)t * n3 + l3) * n2 + l2) * n1 + l1;
    const T s = p1[i1] * p2[i2] * p3[i3];
    auto v = grid[src];
    v.x *= s;
    v.y *= s;
    f[(((size_t)t * N3 + i3) * N2 + i2) * N1 + i1] = v;
}

// Type 2: grid[t][l] = p1 p2 p3 f[t][k] where l = k mod n for k in I_N, else 0.
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_precorrect(int N1, int N2, int N3, int n1, int n2, int n3, int chunks, int64_t nwork,
             const typename Cplx<T>::type *__restrict__ f, const T *__restrict__ p1,
             const T *__restrict__ p2, const T *__restrict__ p3,
             typename Cplx<T>::type *__restrict__ grid)
{
    // frequency held by index l: k = l for l <= kmax, k = l - n for l >= n + kmin
    auto idx = [](int l, int N, int n) -> int {
        const int kmin = -(N / 2), kmax = N - 1 - N / 2;
        if (l <= kmax) return l - kmin;
        if (l >= n + kmin) return l - n - kmin;
        return -1;
    };
    // work item = (row, chunk of kThreads cells); a persistent grid, so that
    // each wave writes several rows, not one 512 B piece
    for (int64_t w = blockIdx.x; w < nwork; w += gridDim.x) {
        const int64_t row = w / chunks;
        const int l1 = (int)(w % chunks) * kThreads + threadIdx.x;
        if (l1 >= n1) continue;
        const int l2 = (int)(row % n2);
        const int64_t r3 = row / n2;
        const int l3 = (int)(r3 % n3);
        const int64_t t = r3 / n3;
        const int i1 = idx(l1, N1, n1), i2 = idx(l2, N2, n2), i3 = idx(l3, N3, n3);
        typename Cplx<T>::type v;
        v.x = 0;
        v.y = 0;
        if (i1 >= 0 && i2 >= 0 && i3 >= 0) {
            const T s = p1[i1] * p2[i2] * p3[i3];
            v = f[(((size_t)t * N3 + i3) * N2 + i2) * N1 + i1];
            v.x *= s;
            v.y *= s;
        }
        grid[(((size_t)t * n3 + l3) * n2 + l2) * n1 + l1] = v;
    }
}

// Batched forms: one launch over the concatenated modes (deconvolution) or
// fine cells (precorrection) of all transforms; element e belongs to the
// transform whose mode_off / grid_off range holds it.  Correction factors
// are concatenated per dimension at p_off.
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_deconv_batch(const TGeom *__restrict__ tg, int T_, long long nmodes,
               const typename Cplx<T>::type *__restrict__ grid, const T *__restrict__ p1,
               const T *__restrict__ p2, const T *__restrict__ p3,
               typename Cplx<T>::type *__restrict__ f)
{
    __shared__ long long soff[kTCache];
    const auto fld = [](const TGeom &a) { return a.mode_off; };
    const bool cached = cache_offsets(soff, tg, T_, fld);
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nmodes;
         e += (long long)gridDim.x * blockDim.x) {
        const TGeom &t = tg[cached ? find_cached(soff, T_, e) : find_transform(tg, T_, e, fld)];
        const long long el = e - t.mode_off;
        const int i1 = (int)(el % t.N[0]);
        const long long r = el / t.N[0];
        const int i2 = (int)(r % t.N[1]);
        const int i3 = (int)(r / t.N[1]);
        const int k1 = i1 - t.N[0] / 2, k2 = i2 - t.N[1] / 2, k3 = i3 - t.N[2] / 2;
        const int l1 = k1 < 0 ? k1 + t.n[0] : k1;
        const int l2 = k2 < 0 ? k2 + t.n[1] : k2;
        const int l3 = k3 < 0 ? k3 + t.n[2] : k3;
        const T sc = p1[t.p_off[0] + i1] * p2[t.p_off[1] + i2] * p3[t.p_off[2] + i3];
        auto v = grid[t.grid_off + ((long long)l3 * t.n[1] + l2) * t.n[0] + l1];
        v.x *= sc;
        v.y *= sc;
        f[e] = v;
    }
}

template <typename T>
__global__ void __launch_bounds__(kThreads)
k_precorrect_batch(const TGeom *__restrict__ tg, int T_, long long ncells,
                   const typename Cplx<T>::type *__restrict__ f, const T *__restrict__ p1,
                   const T *__restrict__ p2, const T *__restrict__ p3,
                   typename Cplx<T>::type *__restrict__ grid)
{
    auto idx = [](int l, int N, int n) -> int {
        const int kmin = -(N / 2), kmax = N - 1 - N / 2;
        if (l <= kmax) return l - kmin;
        if (l >= n + kmin) return l - n - kmin;
        return -1;
    };
    __shared__ long long soff[kTCache];
    const auto fld = [](const TGeom &a) { return a.grid_off; };
    const bool cached = cache_offsets(soff, tg, T_, fld);
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < ncells;
         e += (long long)gridDim.x * blockDim.x) {
        const TGeom &t = tg[cached ? find_cached(soff, T_, e) : find_transform(tg, T_, e, fld)];
        const long long el = e - t.grid_off;
        const int l1 = (int)(el % t.n[0]);
        const long long r = el / t.n[0];
        const int l2 = (int)(r % t.n[1]);
        const int l3 = (int)(r / t.n[1]);
        const int i1 = idx(l1, t.N[0], t.n[0]), i2 = idx(l2, t.N[1], t.n[1]);
        const int i3 = idx(l3, t.N[2], t.n[2]);
        typename Cplx<T>::type v;
        v.x = 0;
        v.y = 0;
        if (i1 >= 0 && i2 >= 0 && i3 >= 0) {
            const T sc = p1[t.p_off[0] + i1] * p2[t.p_off[1] + i2] * p3[t.p_off[2] + i3];
            v = f[t.mode_off + ((long long)i3 * t.N[1] + i2) * t.N[0] + i1];
            v.x *= sc;
            v.y *= sc;
        }
        grid[e] = v;
    }
}

template <typename V>
__global__ void k_zero(V *__restrict__ p, size_t nv, unsigned char *__restrict__ tail, int ntail)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t e = i; e < nv; e += stride) p[e] = V{};
    if (i < (size_t)ntail) tail[i] = 0;
}

}  // namespace

hipError_t launch_deconv(int dim, const int64_t N[3], const int n[3], int prec, int ntransf,
                         const void *grid, const void *const p[3], void *f, hipStream_t s)
{
    const int N1 = (int)N[0], N2 = (int)N[1], N3 = dim == 3 ? (int)N[2] : 1;
    const int n3 = dim == 3 ? n[2] : 1;
    const int chunks = (N1 + kThreads - 1) / kThreads;
    const int64_t rows = (int64_t)N2 * N3 * ntransf;
    const dim3 grd((unsigned)(rows * chunks)), blk(kThreads);
    if (prec == 0)
        hipLaunchKernelGGL(k_deconv<float>, grd, blk, 0, s, N1, N2, N3, n[0], n[1], n3, chunks,
                           (const float2 *)grid, (const float *)p[0], (const float *)p[1],
                           (const float *)p[2], (float2 *)f);
    else
        hipLaunchKernelGGL(k_deconv<double>, grd, blk, 0, s, N1, N2, N3, n[0], n[1], n3, chunks,
                           (const double2 *)grid, (const double *)p[0], (const double *)p[1],
                           (const double *)p[2], (double2 *)f);
    return hipGetLastError();
}

hipError_t launch_precorrect(int dim, const int64_t N[3], const int n[3], int prec,
                             int ntransf, const void *f, const void *const p[3], void *grid,
                             hipStream_t s)
{
    const int N1 = (int)N[0], N2 = (int)N[1], N3 = dim == 3 ? (int)N[2] : 1;
    const int n3 = dim == 3 ? n[2] : 1;
    const int chunks = (n[0] + kThreads - 1) / kThreads;
    const int64_t rows = (int64_t)n[1] * n3 * ntransf;
    const int64_t nwork = rows * chunks;
    const dim3 grd((unsigned)std::min<int64_t>(nwork, 8192)), blk(kThreads);
    if (prec == 0)
        hipLaunchKernelGGL(k_precorrect<float>, grd, blk, 0, s, N1, N2, N3, n[0], n[1], n3,
                           chunks, nwork, (const float2 *)f, (const float *)p[0],
                           (const float *)p[1], (const float *)p[2], (float2 *)grid);
    else
        hipLaunchKernelGGL(k_precorrect<double>, grd, blk, 0, s, N1, N2, N3, n[0], n[1], n3,
                           chunks, nwork, (const double2 *)f, (const double *)p[0],
                           (const double *)p[1], (const double *)p[2], (double2 *)grid);
    return hipGetLastError();
}

hipError_t launch_deconv_batch(const TGeom *tg, int T, long long nmodes, int prec,
                               const void *grid, const void *const p[3], void *f, hipStream_t s)
{
    if (nmodes == 0) return hipSuccess;
    const unsigned blocks = (unsigned)std::min<long long>((nmodes + kThreads - 1) / kThreads, 16384);
    if (prec == 0)
        hipLaunchKernelGGL(k_deconv_batch<float>, dim3(blocks), dim3(kThreads), 0, s, tg, T, nmodes,
                           (const float2 *)grid, (const float *)p[0], (const float *)p[1],
                           (const float *)p[2], (float2 *)f);
    else
        hipLaunchKernelGGL(k_deconv_batch<double>, dim3(blocks), dim3(kThreads), 0, s, tg, T, nmodes,
                           (const double2 *)grid, (const double *)p[0], (const double *)p[1],
                           (const double *)p[2], (double2 *)f);
    return hipGetLastError();
}

hipError_t launch_precorrect_batch(const TGeom *tg, int T, long long ncells, int prec,
                                   const void *f, const void *const p[3], void *grid,
                                   hipStream_t s)
{
    if (ncells == 0) return hipSuccess;
    const unsigned blocks = (unsigned)std::min<long long>((ncells + kThreads - 1) / kThreads, 16384);
    if (prec == 0)
        hipLaunchKernelGGL(k_precorrect_batch<float>, dim3(blocks), dim3(kThreads), 0, s, tg, T,
                           ncells, (const float2 *)f, (const float *)p[0], (const float *)p[1],
                           (const float *)p[2], (float2 *)grid);
    else
        hipLaunchKernelGGL(k_precorrect_batch<double>, dim3(blocks), dim3(kThreads), 0, s, tg, T,
                           ncells, (const double2 *)f, (const double *)p[0], (const double *)p[1],
                           (const double *)p[2], (double2 *)grid);
    return hipGetLastError();
}

hipError_t launch_zero(void *ptr, size_t bytes, hipStream_t s)
{
    if (bytes == 0) return hipSuccess;
    // 16-byte stores when the pointer allows (library buffers come from
    // hipMalloc); otherwise bytes one at a time (caller buffers of odd offset).
    const bool a16 = ((uintptr_t)ptr % 16) == 0;
    const size_t unit = a16 ? 16 : 1;
    const size_t nv = bytes / unit;
    const int ntail = (int)(bytes % unit);
    const size_t want = (nv + 255) / 256;
    const unsigned blocks = (unsigned)(want < 8192 ? (want ? want : 1) : 8192);
    if (a16)
        hipLaunchKernelGGL(k_zero<uint4>, dim3(blocks), dim3(256), 0, s, (uint4 *)ptr, nv,
                           (unsigned char *)ptr + nv * 16, ntail);
    else
        hipLaunchKernelGGL(k_zero<unsigned char>, dim3(blocks), dim3(256), 0, s,
                           (unsigned char *)ptr, nv, (unsigned char *)ptr + nv, 0);
    return hipGetLastError();
}

}  // namespace mn
