// Kernels of the type 3 transform (nonuniform points to nonuniform
// frequencies), which the paper names as beyond its scope (Sec. I-B,
// Sec. VI).  The reduction to a spread plus a type 2 follows the published
// type 3 method of the FINUFFT paper (Barnett, Magland, af Klinteberg, SIAM
// J. Sci. Comput. 2019):
//   f_k = e^{i sg s_k.C} prod_d (2/w) / phi_hat(w t_kd / 2)
//         * sum_l b_l e^{i sg l.t_k},   t_kd = h_d gamma_d (s_kd - D_d),
//   b   = spread of c_j e^{i sg D.(x_j - C)} at (x_j - C) / gamma,
// with C, D the centres of the points and frequencies, sg the exponent sign.
// These kernels do the elementwise parts: bounds and the two phase /
// deconvolution factors.  All phase arguments are formed in double from the
// caller's coordinates, whatever the plan precision; the rescaled points and
// frequencies are binned from the caller's coordinates too (launch_binkey's
// PtMap), so no rescaled value is ever rounded to single precision.
#include "internal.h"

#include <math.h>

#include <type_traits>

namespace mn {
namespace {

constexpr int kT3Threads = 256;

template <typename T> struct C2;
template <> struct C2<float> { using type = float2; };
template <> struct C2<double> { using type = double2; };

struct Planes {
    const void *p[3];
};

// (cos ph, sin ph) for a phase formed in double.  Double precision plans
// evaluate it in double; single precision plans reduce ph by whole turns in
// double (exact to about 1e-16 ph) and take the single-precision sine and
// cosine of the remainder in [-pi, pi], which is all a float result keeps.
template <typename T>
__device__ __forceinline__ void unit_phase(double ph, double &sn, double &cs)
{
    if constexpr (std::is_same<T, double>::value) {
        sincos(ph, &sn, &cs);
    } else {
        const double turns = rint(ph * 0.15915494309189535);  // ph / (2 pi), rounded
        const float r = (float)fma(-turns, 6.283185307179586, ph);
        float s, c;
        sincosf(r, &s, &c);
        sn = s;
        cs = c;
    }
}

// Per block and dimension: (min, max, 1 if a value is non-finite else 0).
template <typename T>
__global__ void __launch_bounds__(kT3Threads)
k_t3_bounds(int n, int dim, Planes a, double *__restrict__ part)
{
    __shared__ double red[3][3][kT3Threads / 64];
    for (int d = 0; d < dim; ++d) {
        const T *v = static_cast<const T *>(a.p[d]);
        double lo = INFINITY, hi = -INFINITY, bad = 0.0;
        // four independent loads in flight per thread and step
        constexpr int U = 4;
        const int stride = gridDim.x * blockDim.x;
        for (int i0 = blockIdx.x * blockDim.x + threadIdx.x; i0 < n; i0 += U * stride) {
            T x[U];
#pragma unroll
            for (int u = 0; u < U; ++u) x[u] = i0 + u * stride < n ? v[i0 + u * stride] : v[i0];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const double xv = (double)x[u];
                if (!isfinite(xv)) bad = 1.0;
                else { lo = fmin(lo, xv); hi = fmax(hi, xv); }
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            lo = fmin(lo, __shfl_xor(lo, o, 64));
            hi = fmax(hi, __shfl_xor(hi, o, 64));
            bad = fmax(bad, __shfl_xor(bad, o, 64));
        }
        if ((threadIdx.x & 63) == 0) {
            red[d][0][threadIdx.x >> 6] = lo;
            red[d][1][threadIdx.x >> 6] = hi;
            red[d][2][threadIdx.x >> 6] = bad;
        }
    }
    __syncthreads();
    if (threadIdx.x < dim) {
        const int d = threadIdx.x;
        double lo = red[d][0][0], hi = red[d][1][0], bad = red[d][2][0];
        for (int k = 1; k < kT3Threads / 64; ++k) {
            lo = fmin(lo, red[d][0][k]);
            hi = fmax(hi, red[d][1][k]);
            bad = fmax(bad, red[d][2][k]);
        }
        double *o = part + 3 * ((size_t)blockIdx.x * dim + d);
        o[0] = lo;
        o[1] = hi;
        o[2] = bad;
    }
}

// pre[j] = exp(i sg sum_d D_d (x_jd - C_d)).
template <typename T>
__global__ void __launch_bounds__(kT3Threads)
k_t3_prephase(int n, int dim, Planes x, T3Affine af, int sg,
              typename C2<T>::type *__restrict__ pre)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double ph = 0.0;
    for (int d = 0; d < dim; ++d)
        ph += af.mul[d] * ((double)static_cast<const T *>(x.p[d])[i] - af.off[d]);
    double sn, cs;
    unit_phase<T>((double)sg * ph, sn, cs);
    typename C2<T>::type v;
    v.x = (T)cs;
    v.y = (T)sn;
    pre[i] = v;
}

// post[k] = exp(i sg sum_d s_kd C_d) prod_d (2/w) / phi_hat(w t_kd / 2) with
// t_kd = scale_d (s_kd - off_d).  log phi_hat(xi) comes from its Chebyshev
// expansion in u = 2 (xi / ximax)^2 - 1: cheb = (ximax, c_0 .. c_{nc-1}),
// summed by Clenshaw's recurrence.
template <typename T>
__global__ void __launch_bounds__(kT3Threads)
k_t3_postfac(int n, int dim, Planes s, T3Affine af, int sg, int w,
             const double *__restrict__ cheb, int nc, typename C2<T>::type *__restrict__ post)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double ximax = cheb[0];
    double ph = 0.0, lsum = 0.0;
    for (int d = 0; d < dim; ++d) {
        const double sv = (double)static_cast<const T *>(s.p[d])[i];
        ph += sv * af.mul[d];
        const double r = 0.5 * (double)w * (af.scale[d] * (sv - af.off[d])) / ximax;
        const double u = 2.0 * r * r - 1.0;
        double b1 = 0.0, b2 = 0.0;
        for (int k = nc - 1; k >= 1; --k) {
            const double b0 = cheb[1 + k] + 2.0 * u * b1 - b2;
            b2 = b1;
            b1 = b0;
        }
        lsum += cheb[1] + u * b1 - b2;
    }
    double fac = exp(-lsum);
    for (int d = 0; d < dim; ++d) fac *= 2.0 / (double)w;
    double sn, cs;
    unit_phase<T>((double)sg * ph, sn, cs);
    typename C2<T>::type v;
    v.x = (T)(fac * cs);
    v.y = (T)(fac * sn);
    post[i] = v;
}

// out[t][i] = in[t][i] * fac[i] for ntransf stacked vectors (in may be out).
template <typename T>
__global__ void __launch_bounds__(kT3Threads)
k_cmul(long long n, int ntransf, const typename C2<T>::type *in,
       const typename C2<T>::type *__restrict__ fac, typename C2<T>::type *out)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const auto f = fac[i];
    for (int t = 0; t < ntransf; ++t) {
        const auto a = in[(size_t)t * n + i];
        typename C2<T>::type r;
        r.x = a.x * f.x - a.y * f.y;
        r.y = a.x * f.y + a.y * f.x;
        out[(size_t)t * n + i] = r;
    }
}

inline unsigned blocks_for(long long n) { return (unsigned)((n + kT3Threads - 1) / kT3Threads); }

Planes planes(const void *const a[3])
{
    Planes p;
    for (int d = 0; d < 3; ++d) p.p[d] = a[d];
    return p;
}

}  // namespace

int t3_bounds_blocks(int n)
{
    const long long b = (n + kT3Threads - 1) / kT3Threads;
    return (int)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

hipError_t launch_t3_bounds(int prec, int n, int dim, const void *const a[3], double *part,
                            hipStream_t s)
{
    const int nb = t3_bounds_blocks(n);
    if (prec == 0)
        hipLaunchKernelGGL(k_t3_bounds<float>, dim3(nb), dim3(kT3Threads), 0, s, n, dim,
                           planes(a), part);
    else
        hipLaunchKernelGGL(k_t3_bounds<double>, dim3(nb), dim3(kT3Threads), 0, s, n, dim,
                           planes(a), part);
    return hipGetLastError();
}

hipError_t launch_t3_prephase(int prec, int n, int dim, const void *const x[3],
                              const T3Affine &af, int sg, void *pre, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (prec == 0)
        hipLaunchKernelGGL(k_t3_prephase<float>, dim3(blocks_for(n)), dim3(kT3Threads), 0, s, n,
                           dim, planes(x), af, sg, static_cast<float2 *>(pre));
    else
        hipLaunchKernelGGL(k_t3_prephase<double>, dim3(blocks_for(n)), dim3(kT3Threads), 0, s,
                           n, dim, planes(x), af, sg, static_cast<double2 *>(pre));
    return hipGetLastError();
}

hipError_t launch_t3_postfac(int prec, int n, int dim, const void *const sf[3],
                             const T3Affine &af, int sg, int w, const double *cheb, int nc,
                             void *post, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (prec == 0)
        hipLaunchKernelGGL(k_t3_postfac<float>, dim3(blocks_for(n)), dim3(kT3Threads), 0, s, n,
                           dim, planes(sf), af, sg, w, cheb, nc, static_cast<float2 *>(post));
    else
        hipLaunchKernelGGL(k_t3_postfac<double>, dim3(blocks_for(n)), dim3(kT3Threads), 0, s, n,
                           dim, planes(sf), af, sg, w, cheb, nc, static_cast<double2 *>(post));
    return hipGetLastError();
}

hipError_t launch_cmul(int prec, long long n, int ntransf, const void *in, const void *fac,
                       void *out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (prec == 0)
        hipLaunchKernelGGL(k_cmul<float>, dim3(blocks_for(n)), dim3(kT3Threads), 0, s, n,
                           ntransf, static_cast<const float2 *>(in),
                           static_cast<const float2 *>(fac), static_cast<float2 *>(out));
    else
        hipLaunchKernelGGL(k_cmul<double>, dim3(blocks_for(n)), dim3(kT3Threads), 0, s, n,
                           ntransf, static_cast<const double2 *>(in),
                           static_cast<const double2 *>(fac), static_cast<double2 *>(out));
    return hipGetLastError();
}

}  // namespace mn
