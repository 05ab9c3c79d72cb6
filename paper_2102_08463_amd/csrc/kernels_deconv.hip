// Correction steps around the fine-grid FFT (Sec. II-A step 3 and Sec. II-B
// step 1): one thread per output element, per the embarrassingly parallel
// scheme of Sec. III.
//
// Mode k in I_N (ascending from -floor(N/2)) lives at fine-grid index k mod n.
// The factors p_i[k] = (2/w) / phi_hat(alpha_i k) are separable; the library
// stores them with the lattice phase (-1)^k folded in (grid point l sits at
// l h - pi), so both corrections are a plain product.
#include "internal.h"

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
k_precorrect(int N1, int N2, int N3, int n1, int n2, int n3, int chunks,
             const typename Cplx<T>::type *__restrict__ f, const T *__restrict__ p1,
             const T *__restrict__ p2, const T *__restrict__ p3,
             typename Cplx<T>::type *__restrict__ grid)
{
    const int64_t row = blockIdx.x / chunks;
    const int l1 = (int)(blockIdx.x % chunks) * kThreads + threadIdx.x;
    if (l1 >= n1) return;
    const int l2 = (int)(row % n2);
    const int64_t r3 = row / n2;
    const int l3 = (int)(r3 % n3);
    const int64_t t = r3 / n3;
    // frequency held by index l: k = l for l <= kmax, k = l - n for l >= n + kmin
    auto idx = [](int l, int N, int n) -> int {
        const int kmin = -(N / 2), kmax = N - 1 - N / 2;
        if (l <= kmax) return l - kmin;
        if (l >= n + kmin) return l - n - kmin;
        return -1;
    };
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
    const dim3 grd((unsigned)(rows * chunks)), blk(kThreads);
    if (prec == 0)
        hipLaunchKernelGGL(k_precorrect<float>, grd, blk, 0, s, N1, N2, N3, n[0], n[1], n3,
                           chunks, (const float2 *)f, (const float *)p[0], (const float *)p[1],
                           (const float *)p[2], (float2 *)grid);
    else
        hipLaunchKernelGGL(k_precorrect<double>, grd, blk, 0, s, N1, N2, N3, n[0], n[1], n3,
                           chunks, (const double2 *)f, (const double *)p[0],
                           (const double *)p[1], (const double *)p[2], (double2 *)grid);
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
