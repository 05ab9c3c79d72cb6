// Learned parameter selector: point-density features and a small MLP
// (F -> H -> H -> K, ReLU) with forward, masked mean-squared-error gradient,
// backward and Adam kernels.  The network predicts the log run time of each
// autotuner candidate from the features; the selector takes the argmin.
//
// Parameter layout (one flat float array): W1 (F x H, row i = input i), b1 (H),
// W2 (H x H), b2 (H), W3 (H x K), b3 (K).
#include "../../include/mnufft.h"
#include "internal.h"

#include <algorithm>
#include <mutex>

namespace {

constexpr int kThreads = 256;
constexpr int kHistBlocks = 512;  // partial histograms; see MNUFFT_DENSITY_WORK_BYTES
constexpr double kPi = 3.141592653589793;

// Y[b][o] = act(bias[o] + sum_i X[b][i] W[i][o]); act = ReLU or identity.
__global__ void k_dense(int B, int In, int Out, const float *__restrict__ X,
                        const float *__restrict__ W, const float *__restrict__ bias,
                        float *__restrict__ Y, int relu)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= B * Out) return;
    const int b = e / Out, o = e % Out;
    float acc = bias[o];
    const float *x = X + (size_t)b * In;
    for (int i = 0; i < In; ++i) acc = fmaf(x[i], W[(size_t)i * Out + o], acc);
    Y[e] = relu ? fmaxf(acc, 0.0f) : acc;
}

// dW[i][o] = sum_b A[b][i] D[b][o]  (A: B x In, D: B x Out)
__global__ void k_outer_sum(int B, int In, int Out, const float *__restrict__ A,
                            const float *__restrict__ D, float *__restrict__ dW)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= In * Out) return;
    const int i = e / Out, o = e % Out;
    float acc = 0.0f;
    for (int b = 0; b < B; ++b) acc = fmaf(A[(size_t)b * In + i], D[(size_t)b * Out + o], acc);
    dW[e] = acc;
}

// db[o] = sum_b D[b][o]
__global__ void k_colsum(int B, int Out, const float *__restrict__ D, float *__restrict__ db)
{
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= Out) return;
    float acc = 0.0f;
    for (int b = 0; b < B; ++b) acc += D[(size_t)b * Out + o];
    db[o] = acc;
}

// dA[b][i] = (sum_o D[b][o] W[i][o]) * (A[b][i] > 0): back through W and the ReLU.
__global__ void k_back_relu(int B, int In, int Out, const float *__restrict__ D,
                            const float *__restrict__ W, const float *__restrict__ A,
                            float *__restrict__ dA)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= B * In) return;
    const int b = e / In, i = e % In;
    float acc = 0.0f;
    for (int o = 0; o < Out; ++o) acc = fmaf(D[(size_t)b * Out + o], W[(size_t)i * Out + o], acc);
    dA[e] = A[e] > 0.0f ? acc : 0.0f;
}

// Masked MSE: loss = sum m (y - t)^2 / sum m; dY = 2 m (y - t) / sum m.  One block.
__global__ void k_mse(int n, const float *__restrict__ Y, const float *__restrict__ T,
                      const float *__restrict__ mask, float *__restrict__ dY,
                      float *__restrict__ loss)
{
    __shared__ float sm[kThreads], sl[kThreads];
    float m = 0.0f, l = 0.0f;
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
        const float r = Y[e] - T[e];
        m += mask[e];
        l += mask[e] * r * r;
    }
    sm[threadIdx.x] = m;
    sl[threadIdx.x] = l;
    __syncthreads();
    for (int o = kThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            sm[threadIdx.x] += sm[threadIdx.x + o];
            sl[threadIdx.x] += sl[threadIdx.x + o];
        }
        __syncthreads();
    }
    const float msum = fmaxf(sm[0], 1.0f);
    if (threadIdx.x == 0) *loss = sl[0] / msum;
    for (int e = threadIdx.x; e < n; e += blockDim.x)
        dY[e] = 2.0f * mask[e] * (Y[e] - T[e]) / msum;
}

__global__ void k_adam(long long n, float *__restrict__ p, const float *__restrict__ g,
                       float *__restrict__ m, float *__restrict__ v, float lr, float b1, float b2,
                       float eps, float c1, float c2)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const float gi = g[e];
    const float mi = b1 * m[e] + (1.0f - b1) * gi;
    const float vi = b2 * v[e] + (1.0f - b2) * gi * gi;
    m[e] = mi;
    v[e] = vi;
    p[e] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// 16 x 16 cell of a point: the same folded grid coordinate as the bin-sort,
// on a 16-cell grid per dimension.
__device__ __forceinline__ int cell16(double x)
{
    const double S = 16.0 / (2.0 * kPi);
    double g = __dmul_rn(__dadd_rn(x, kPi), S);
    if (g < 0.0) g = __dadd_rn(g, 16.0);
    if (g >= 16.0) g = __dsub_rn(g, 16.0);
    if (!(g >= 0.0 && g < 16.0)) {
        g = __dsub_rn(g, __dmul_rn(floor(__ddiv_rn(g, 16.0)), 16.0));
        if (!(g >= 0.0 && g < 16.0)) g = 0.0;
    }
    return (int)g;
}

template <typename T>
__global__ void __launch_bounds__(kThreads)
k_hist_partial(long long M, const T *__restrict__ x, const T *__restrict__ y,
               uint32_t *__restrict__ part)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    for (long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x; j < M;
         j += (long long)gridDim.x * blockDim.x)
        atomicAdd(&h[cell16((double)x[j]) + 16 * cell16((double)y[j])], 1u);
    __syncthreads();
    part[(size_t)blockIdx.x * 256 + threadIdx.x] = h[threadIdx.x];
}

// feature[c] = log(1 + 256 count[c] / M): the density relative to uniform.
__global__ void k_hist_final(long long M, int nblk, const uint32_t *__restrict__ part,
                             float *__restrict__ feat)
{
    const int c = threadIdx.x;
    unsigned long long s = 0;
    for (int b = 0; b < nblk; ++b) s += part[(size_t)b * 256 + c];
    feat[c] = M > 0 ? log1pf(256.0f * (float)((double)s / (double)M)) : 0.0f;
}

// Batched histograms, balanced over points rather than sets (a few large
// sets would otherwise keep a few blocks busy long after the rest): the
// concatenated points are cut into chunks of kHistChunk, block b takes
// chunks b, b + gridDim.x, ..., and for each set a chunk overlaps it counts
// that set's part in LDS (one histogram per wave) and adds the counts to the
// set's partial row (chunk index mod kBatchChunks).  The rows must start at
// zero (k_hist_clear).
constexpr int kBatchChunks = 32;  // partial rows per set; see MNUFFT_DENSITY_BATCH_WORK_BYTES
constexpr int kHistChunk = 8192;
constexpr int kHistBatchBlocks = 2048;
constexpr int kHistUnroll = 8;
constexpr int kHistOffCache = 1024;  // set offsets kept in LDS (sets below this count)

__global__ void k_hist_clear(size_t n, uint32_t *__restrict__ part)
{
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (size_t)gridDim.x * blockDim.x)
        part[e] = 0u;
}

template <typename T>
__global__ void __launch_bounds__(kThreads)
k_hist_batch(int nset, const int64_t *__restrict__ off, const T *__restrict__ x,
             const T *__restrict__ y, uint32_t *__restrict__ part)
{
    constexpr int kWaves = kThreads / 64;
    __shared__ uint32_t h[kWaves][256];
    __shared__ long long soff[kHistOffCache];
    __shared__ int first;
    // the set offsets, from LDS when they fit (the searches below touch them
    // for every chunk)
    const bool cached = nset < kHistOffCache;
    if (cached)
        for (int k = threadIdx.x; k <= nset; k += kThreads) soff[k] = off[k];
    __syncthreads();
    const auto O = [&](int k) { return cached ? soff[k] : (long long)off[k]; };
    const long long Mtot = O(nset);
    const int wave = threadIdx.x >> 6;
    for (long long a = (long long)blockIdx.x * kHistChunk; a < Mtot;
         a += (long long)gridDim.x * kHistChunk) {
        const long long e = min(a + (long long)kHistChunk, Mtot);
        if (threadIdx.x == 0) {  // the first set whose points reach past a
            int lo = 0, hi = nset - 1;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (O(mid + 1) > a) hi = mid;
                else lo = mid + 1;
            }
            first = lo;
        }
        __syncthreads();
        const int t0 = first;
        __syncthreads();
        const int row = (int)((a / kHistChunk) % kBatchChunks);
        // the bounds below are the same for every thread, so is the control flow
        for (int t = t0; t < nset && O(t) < e; ++t) {
            const long long s0 = max(a, O(t)), s1 = min(e, O(t + 1));
            if (s0 >= s1) continue;
            for (int k = threadIdx.x; k < kWaves * 256; k += kThreads) (&h[0][0])[k] = 0u;
            __syncthreads();
            for (long long j = s0 + threadIdx.x; j < s1; j += kHistUnroll * kThreads) {
                T xv[kHistUnroll], yv[kHistUnroll];
#pragma unroll
                for (int u = 0; u < kHistUnroll; ++u) {
                    const long long jj = min(j + (long long)u * kThreads, s1 - 1);
                    xv[u] = x[jj];
                    yv[u] = y[jj];
                }
#pragma unroll
                for (int u = 0; u < kHistUnroll; ++u)
                    if (j + (long long)u * kThreads < s1)
                        atomicAdd(&h[wave][cell16((double)xv[u]) + 16 * cell16((double)yv[u])], 1u);
            }
            __syncthreads();
            for (int c = threadIdx.x; c < 256; c += kThreads) {
                uint32_t v = 0;
#pragma unroll
                for (int w = 0; w < kWaves; ++w) v += h[w][c];
                if (v) atomicAdd(&part[((size_t)t * kBatchChunks + row) * 256 + c], v);
            }
            __syncthreads();
        }
    }
}

// Features of set t from its partial rows; with scal, also copies the set's
// nscal extra features (scal + t * nscal) after the 256 density features.
__global__ void k_hist_batch_final(const int64_t *__restrict__ off,
                                   const uint32_t *__restrict__ part, float *__restrict__ feat,
                                   int ldf, const float *__restrict__ scal, int nscal)
{
    const int t = blockIdx.x, c = threadIdx.x;
    const long long M = off[t + 1] - off[t];
    unsigned long long s = 0;
    for (int b = 0; b < kBatchChunks; ++b) s += part[((size_t)t * kBatchChunks + b) * 256 + c];
    feat[(size_t)t * ldf + c] = M > 0 ? log1pf(256.0f * (float)((double)s / (double)M)) : 0.0f;
    if (scal && c < nscal) feat[(size_t)t * ldf + 256 + c] = scal[(size_t)t * nscal + c];
}

// One layer of the network inside a block: out = act(bias + W^T in), with
// the In-sum of each output split over the block's blockDim / Out thread
// groups (few terms per thread, so the weight loads are all in flight at
// once) and the group sums added in LDS.  Out <= 256.  Ends with a barrier.
__device__ void block_dense(int In, int Out, const float *in, const float *__restrict__ W,
                            const float *__restrict__ bias, float *out, float *red, bool relu)
{
    const int G = max(1, (int)blockDim.x / Out);
    const int o = threadIdx.x % Out, grp = threadIdx.x / Out;
    if (grp < G) {
        float acc = 0.0f;
#pragma unroll 8
        for (int i = grp; i < In; i += G) acc = fmaf(in[i], W[(size_t)i * Out + o], acc);
        red[grp * Out + o] = acc;
    }
    __syncthreads();
    if ((int)threadIdx.x < Out) {
        float v = bias[threadIdx.x];
        for (int q = 0; q < G; ++q) v += red[q * Out + threadIdx.x];
        out[threadIdx.x] = relu ? fmaxf(v, 0.0f) : v;
    }
    __syncthreads();
}

// The selector's whole pass for one row per block: the three layers of the
// network on the row's features, then the allowed output of smallest value
// and its gap to the runner-up (infinity with one allowed output, index -1
// with none).
constexpr int kFusedMaxF = 512, kFusedMaxH = 256, kFusedMaxK = 128, kFusedThreads = 1024;
__global__ void __launch_bounds__(kFusedThreads)
k_mlp_argmin(int F, int H, int K, const float *__restrict__ params, const float *__restrict__ X,
             int ldx, unsigned long long m0, unsigned long long m1, int *__restrict__ idx,
             float *__restrict__ gap)
{
    __shared__ float xs[kFusedMaxF], h1[kFusedMaxH], h2[kFusedMaxH], ys[kFusedMaxK];
    __shared__ float red[kFusedThreads];
    const int b = blockIdx.x;
    const float *W1 = params, *b1 = W1 + (size_t)F * H, *W2 = b1 + H, *b2 = W2 + (size_t)H * H;
    const float *W3 = b2 + H, *b3 = W3 + (size_t)H * K;
    for (int i = threadIdx.x; i < F; i += blockDim.x) xs[i] = X[(size_t)b * ldx + i];
    __syncthreads();
    block_dense(F, H, xs, W1, b1, h1, red, true);
    block_dense(H, H, h1, W2, b2, h2, red, true);
    block_dense(H, K, h2, W3, b3, ys, red, false);
    if (threadIdx.x == 0) {
        int best = -1;
        float v0 = INFINITY, v1 = INFINITY;
        for (int k = 0; k < K; ++k) {
            const unsigned long long m = k < 64 ? m0 : m1;
            if (!((m >> (k & 63)) & 1ull)) continue;
            const float v = ys[k];
            if (v < v0) {
                v1 = v0;
                v0 = v;
                best = k;
            } else if (v < v1) {
                v1 = v;
            }
        }
        idx[b] = best;
        gap[b] = v1 - v0;
    }
}

// The selector's whole pass for set t = blockIdx.x from the partial
// histogram rows: the set's features (the 256 density features as
// k_hist_batch_final computes them, then its nscal scalars), which also
// returns the set's rows to zero for the next count, the network, and the
// argmin of k_mlp_argmin.
__global__ void __launch_bounds__(kFusedThreads)
k_select_rows(const int64_t *__restrict__ off, uint32_t *__restrict__ part,
              const float *__restrict__ scal, int nscal, int H, int K,
              const float *__restrict__ params, unsigned long long m0, unsigned long long m1,
              int *__restrict__ idx, float *__restrict__ gap)
{
    __shared__ float xs[kFusedMaxF], h1[kFusedMaxH], h2[kFusedMaxH], ys[kFusedMaxK];
    __shared__ float red[kFusedThreads];
    __shared__ unsigned long long cnt[4][256];
    const int t = blockIdx.x, tid = threadIdx.x;
    const int F = 256 + nscal;
    {
        // four groups of 256 threads sum eight partial rows each
        const int c = tid & 255, grp = tid >> 8;
        unsigned long long sum = 0;
        for (int b = grp; b < kBatchChunks; b += 4) {
            uint32_t *r = part + ((size_t)t * kBatchChunks + b) * 256 + c;
            sum += *r;
            *r = 0u;
        }
        cnt[grp][c] = sum;
    }
    __syncthreads();
    if (tid < 256) {
        const long long M = off[t + 1] - off[t];
        const unsigned long long sum = cnt[0][tid] + cnt[1][tid] + cnt[2][tid] + cnt[3][tid];
        xs[tid] = M > 0 ? log1pf(256.0f * (float)((double)sum / (double)M)) : 0.0f;
    } else if (tid < 256 + nscal) {
        xs[tid] = scal[(size_t)t * nscal + tid - 256];
    }
    __syncthreads();
    const float *W1 = params, *b1 = W1 + (size_t)F * H, *W2 = b1 + H, *b2 = W2 + (size_t)H * H;
    const float *W3 = b2 + H, *b3 = W3 + (size_t)H * K;
    block_dense(F, H, xs, W1, b1, h1, red, true);
    block_dense(H, H, h1, W2, b2, h2, red, true);
    block_dense(H, K, h2, W3, b3, ys, red, false);
    if (tid == 0) {
        int best = -1;
        float v0 = INFINITY, v1 = INFINITY;
        for (int k = 0; k < K; ++k) {
            const unsigned long long m = k < 64 ? m0 : m1;
            if (!((m >> (k & 63)) & 1ull)) continue;
            const float v = ys[k];
            if (v < v0) {
                v1 = v0;
                v0 = v;
                best = k;
            } else if (v < v1) {
                v1 = v;
            }
        }
        idx[t] = best;
        gap[t] = v1 - v0;
    }
}

inline int blocks_for(long long n) { return (int)std::max<long long>(1, (n + kThreads - 1) / kThreads); }


// Workspace of mnufft_density_features_batch_noalloc: the partial histograms
// of up to kNoAllocSets point sets (2 MiB), one copy per GPU for the life of
// the process.  In host code `scratch` names a host-side stand-in; the device
// address of each GPU's copy comes from hipGetSymbolAddress, taken once per
// device and kept in g_scratch.
constexpr int kNoAllocSets = 64;
static __device__ __align__(256) uint32_t scratch[kNoAllocSets * kBatchChunks * 256];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};

// Device address of the current device's workspace (looked up on its first use).
int scratch_of_current_device(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return MNUFFT_ERR_HIP;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return MNUFFT_ERR_HIP;
        }
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return MNUFFT_OK;
}

int density_batch(int prec, int T, const int64_t *off, const void *x, const void *y, float *feat,
                  int ldf, void *work, hipStream_t s, const float *scal = nullptr, int nscal = 0)
{
    uint32_t *part = (uint32_t *)work;
    const size_t nrow = (size_t)T * kBatchChunks * 256;
    hipLaunchKernelGGL(k_hist_clear, dim3((unsigned)std::min<size_t>(1024, (nrow + 255) / 256)),
                       dim3(256), 0, s, nrow, part);
    if (prec == MNUFFT_F32)
        hipLaunchKernelGGL(k_hist_batch<float>, dim3(kHistBatchBlocks), dim3(kThreads), 0, s, T,
                           off, (const float *)x, (const float *)y, part);
    else
        hipLaunchKernelGGL(k_hist_batch<double>, dim3(kHistBatchBlocks), dim3(kThreads), 0, s, T,
                           off, (const double *)x, (const double *)y, part);
    hipLaunchKernelGGL(k_hist_batch_final, dim3(T), dim3(256), 0, s, off,
                       (const uint32_t *)part, feat, ldf, scal, nscal);
    return hipGetLastError() == hipSuccess ? MNUFFT_OK : MNUFFT_ERR_HIP;
}

}  // namespace

namespace mn {

hipError_t launch_select_rows(int T, const int64_t *off, uint32_t *part, const float *scal,
                              int nscal, int F, int H, int K, const float *params,
                              const unsigned long long mask[2], int *idx, float *gap,
                              hipStream_t s)
{
    if (nscal < 0 || F != 256 + nscal || F > kFusedMaxF || H < 1 || H > kFusedMaxH || K < 1 ||
        K > kFusedMaxK)
        return hipErrorInvalidValue;
    if (T <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_select_rows, dim3(T), dim3(kFusedThreads), 0, s, off, part, scal, nscal,
                       H, K, params, mask[0], mask[1], idx, gap);
    return hipGetLastError();
}

hipError_t launch_hist_clear(int T, uint32_t *part, hipStream_t s)
{
    const size_t nrow = (size_t)T * kBatchChunks * 256;
    if (T <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_hist_clear, dim3((unsigned)std::min<size_t>(1024, (nrow + 255) / 256)),
                       dim3(256), 0, s, nrow, part);
    return hipGetLastError();
}

hipError_t launch_hist_count(int prec, int T, const int64_t *off, const void *x, const void *y,
                             uint32_t *part, hipStream_t s)
{
    if (prec == MNUFFT_F32)
        hipLaunchKernelGGL(k_hist_batch<float>, dim3(kHistBatchBlocks), dim3(kThreads), 0, s, T,
                           off, (const float *)x, (const float *)y, part);
    else
        hipLaunchKernelGGL(k_hist_batch<double>, dim3(kHistBatchBlocks), dim3(kThreads), 0, s, T,
                           off, (const double *)x, (const double *)y, part);
    return hipGetLastError();
}


hipError_t launch_mlp_argmin(int F, int H, int K, const float *params, int T, const float *X,
                             int ldx, const unsigned long long mask[2], int *idx, float *gap,
                             hipStream_t s)
{
    if (F < 1 || F > kFusedMaxF || H < 1 || H > kFusedMaxH || K < 1 || K > kFusedMaxK ||
        ldx < F)
        return hipErrorInvalidValue;
    if (T <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_argmin, dim3(T), dim3(kFusedThreads), 0, s, F, H, K, params, X, ldx,
                       mask[0], mask[1], idx, gap);
    return hipGetLastError();
}
}  // namespace mn

extern "C" {

int64_t mnufft_mlp_nparams(int F, int H, int K)
{
    if (F < 1 || H < 1 || K < 1) return MNUFFT_ERR_ARG;
    return (int64_t)F * H + H + (int64_t)H * H + H + (int64_t)H * K + K;
}

int mnufft_mlp_forward(int F, int H, int K, const float *params, int B, const float *X, float *H1,
                       float *H2, float *Y, void *stream)
{
    if (F < 1 || H < 1 || K < 1 || B < 0 || !params || (B > 0 && (!X || !H1 || !H2 || !Y)))
        return MNUFFT_ERR_ARG;
    if (B == 0) return MNUFFT_OK;
    hipStream_t s = (hipStream_t)stream;
    const float *W1 = params, *b1 = W1 + (size_t)F * H, *W2 = b1 + H, *b2 = W2 + (size_t)H * H;
    const float *W3 = b2 + H, *b3 = W3 + (size_t)H * K;
    hipLaunchKernelGGL(k_dense, dim3(blocks_for((long long)B * H)), dim3(kThreads), 0, s, B, F, H,
                       X, W1, b1, H1, 1);
    hipLaunchKernelGGL(k_dense, dim3(blocks_for((long long)B * H)), dim3(kThreads), 0, s, B, H, H,
                       (const float *)H1, W2, b2, H2, 1);
    hipLaunchKernelGGL(k_dense, dim3(blocks_for((long long)B * K)), dim3(kThreads), 0, s, B, H, K,
                       (const float *)H2, W3, b3, Y, 0);
    return hipGetLastError() == hipSuccess ? MNUFFT_OK : MNUFFT_ERR_HIP;
}

int mnufft_mlp_loss_grad(int K, int B, const float *Y, const float *T, const float *mask, float *dY,
                         float *loss, void *stream)
{
    if (K < 1 || B < 1 || !Y || !T || !mask || !dY || !loss) return MNUFFT_ERR_ARG;
    hipLaunchKernelGGL(k_mse, dim3(1), dim3(kThreads), 0, (hipStream_t)stream, B * K, Y, T, mask,
                       dY, loss);
    return hipGetLastError() == hipSuccess ? MNUFFT_OK : MNUFFT_ERR_HIP;
}

int mnufft_mlp_backward(int F, int H, int K, const float *params, int B, const float *X,
                        const float *H1, const float *H2, const float *dY, float *work,
                        float *grads, void *stream)
{
    if (F < 1 || H < 1 || K < 1 || B < 1 || !params || !X || !H1 || !H2 || !dY || !work || !grads)
        return MNUFFT_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    const float *W2 = params + (size_t)F * H + H, *W3 = W2 + (size_t)H * H + H;
    float *dW1 = grads, *db1 = dW1 + (size_t)F * H, *dW2 = db1 + H, *db2 = dW2 + (size_t)H * H;
    float *dW3 = db2 + H, *db3 = dW3 + (size_t)H * K;
    float *dH2 = work, *dH1 = work + (size_t)B * H;
    hipLaunchKernelGGL(k_outer_sum, dim3(blocks_for((long long)H * K)), dim3(kThreads), 0, s, B, H,
                       K, H2, dY, dW3);
    hipLaunchKernelGGL(k_colsum, dim3(blocks_for(K)), dim3(kThreads), 0, s, B, K, dY, db3);
    hipLaunchKernelGGL(k_back_relu, dim3(blocks_for((long long)B * H)), dim3(kThreads), 0, s, B, H,
                       K, dY, W3, H2, dH2);
    hipLaunchKernelGGL(k_outer_sum, dim3(blocks_for((long long)H * H)), dim3(kThreads), 0, s, B, H,
                       H, H1, (const float *)dH2, dW2);
    hipLaunchKernelGGL(k_colsum, dim3(blocks_for(H)), dim3(kThreads), 0, s, B, H,
                       (const float *)dH2, db2);
    hipLaunchKernelGGL(k_back_relu, dim3(blocks_for((long long)B * H)), dim3(kThreads), 0, s, B, H,
                       H, (const float *)dH2, W2, H1, dH1);
    hipLaunchKernelGGL(k_outer_sum, dim3(blocks_for((long long)F * H)), dim3(kThreads), 0, s, B, F,
                       H, X, (const float *)dH1, dW1);
    hipLaunchKernelGGL(k_colsum, dim3(blocks_for(H)), dim3(kThreads), 0, s, B, H,
                       (const float *)dH1, db1);
    return hipGetLastError() == hipSuccess ? MNUFFT_OK : MNUFFT_ERR_HIP;
}

int mnufft_mlp_adam(int64_t n, float *params, const float *grads, float *m, float *v, float lr,
                    float beta1, float beta2, float eps, int step, void *stream)
{
    if (n < 0 || step < 1 || !params || !grads || !m || !v) return MNUFFT_ERR_ARG;
    if (n == 0) return MNUFFT_OK;
    const float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(n)), dim3(kThreads), 0, (hipStream_t)stream, n,
                       params, grads, m, v, lr, beta1, beta2, eps, c1, c2);
    return hipGetLastError() == hipSuccess ? MNUFFT_OK : MNUFFT_ERR_HIP;
}

int mnufft_density_features(int prec, int64_t M, const void *x, const void *y, float *feat,
                            void *work, void *stream)
{
    if ((prec != MNUFFT_F32 && prec != MNUFFT_F64) || M < 0 || !feat || !work ||
        (M > 0 && (!x || !y)))
        return MNUFFT_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    uint32_t *part = (uint32_t *)work;
    const int nblk = (int)std::min<long long>(kHistBlocks, std::max<long long>(1, (M + kThreads - 1) / kThreads));
    if (prec == MNUFFT_F32)
        hipLaunchKernelGGL(k_hist_partial<float>, dim3(nblk), dim3(kThreads), 0, s, (long long)M,
                           (const float *)x, (const float *)y, part);
    else
        hipLaunchKernelGGL(k_hist_partial<double>, dim3(nblk), dim3(kThreads), 0, s, (long long)M,
                           (const double *)x, (const double *)y, part);
    hipLaunchKernelGGL(k_hist_final, dim3(1), dim3(256), 0, s, (long long)M, nblk,
                       (const uint32_t *)part, feat);
    return hipGetLastError() == hipSuccess ? MNUFFT_OK : MNUFFT_ERR_HIP;
}

int mnufft_density_features_batch(int prec, int T, const int64_t *off, const void *x,
                                  const void *y, float *feat, int ldf, void *work, void *stream)
{
    if ((prec != MNUFFT_F32 && prec != MNUFFT_F64) || T < 1 || T > 65535 || !off || !x || !y ||
        !feat || !work || ldf < 256)
        return MNUFFT_ERR_ARG;
    return density_batch(prec, T, off, x, y, feat, ldf, work, (hipStream_t)stream);
}

int mnufft_density_features_batch_noalloc(int prec, int T, const int64_t *off, const void *x,
                                          const void *y, float *feat, int ldf, void *stream)
{
    if ((prec != MNUFFT_F32 && prec != MNUFFT_F64) || T < 1 || T > kNoAllocSets || !off || !x ||
        !y || !feat || ldf < 256)
        return MNUFFT_ERR_ARG;
    void *ws = nullptr;
    const int rc = scratch_of_current_device(&ws);
    if (rc) return rc;
    // density_batch clears the partial rows it uses (with a kernel) before
    // counting, so nothing is left over from an earlier call
    return density_batch(prec, T, off, x, y, feat, ldf, ws, (hipStream_t)stream);
}

}  // extern "C"
