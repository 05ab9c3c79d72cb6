// Microbenchmarks behind the design of the SM kernels (not part of the
// library): LDS atomic / read throughput for the access patterns of
// spreading and interpolation, and the cost of scattering or gathering
// 8-byte items through a random permutation in HBM.
//
//   paper_2102_08463_amd/microbench        (built by build.py)
//
// LDS: 2048 workgroups x 256 threads, each lane walks an address stream in a
// 32 KB LDS array (consecutive lanes on consecutive words; random words;
// sorted runs where about 2.4 lanes share a word, like points sorted by cell;
// or groups of 8 lanes on 8 consecutive words at a random base per group,
// all 8 or only 6 of them active, like one row of taps per point),
// 8 operations per step, 512 steps; the rate is lane-operations per clock per
// CU at 2.4 GHz and 256 CUs.  Every address is masked into the array.
// HBM: 1e7 items, a random permutation p and its inverse q; out[p[i]] = in[i]
// versus out[i] = in[q[i]] versus a plain copy.  Every index is in [0, 1e7).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

namespace {
constexpr int kWords = 4096;
constexpr int kSteps = 512;

__device__ __forceinline__ uint32_t mix(uint32_t x)
{
    x ^= x >> 16; x *= 0x7feb352du; x ^= x >> 15; x *= 0x846ca68bu; x ^= x >> 16;
    return x;
}

// MODE 0 f32 atomic, 1 u32 atomic, 2 u64 atomic, 3 u32 read, 4 u64 read,
// 5 128-bit read (two adjacent u64 words at an even word address).
// PAT 0 consecutive, 1 random, 2 sorted runs with repeats, 3 random groups of
// 8 consecutive words, 4 the same with lanes 6 and 7 of each group idle.
template <int MODE, int PAT>
__global__ void __launch_bounds__(256) k_lds(float *out, int salt)
{
    __shared__ unsigned long long lu[kWords];
    unsigned *l32 = reinterpret_cast<unsigned *>(lu);
    float *lf = reinterpret_cast<float *>(lu);
    for (int i = threadIdx.x; i < kWords; i += 256) lu[i] = 0;
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    constexpr bool grouped = PAT >= 3;
    const uint32_t who = grouped ? threadIdx.x >> 3 : threadIdx.x;
    const uint32_t r = mix(who * 7919u + salt), st = (mix(who + 99u * salt) | 1u) & 1023u;
    const uint32_t off = PAT == 0 ? lane + wv * 1024
                         : (PAT == 1 ? r : (grouped ? r + (lane & 7) : (lane * 27u) / 64u + wv * 1024));
    const bool active = PAT != 4 || (lane & 7) < 6;
    unsigned long long acc = 0;
#pragma unroll 1
    for (int it = 0; it < kSteps; ++it) {
        const uint32_t base = (PAT == 1 || grouped) ? off + it * st : off + it * 97u;
        if (!active) continue;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t a = (base + u * ((PAT == 1 || grouped) ? 613u : 38u)) & (kWords - 1);
            if (MODE == 0) atomicAdd(&lf[a], 1.0f);
            else if (MODE == 1) atomicAdd(&l32[a], 1u);
            else if (MODE == 2) atomicAdd(&lu[a], 1ull);
            else if (MODE == 3) acc += l32[a];
            else if (MODE == 4) acc += lu[a];
            else {
                const ulonglong2 v = *reinterpret_cast<const ulonglong2 *>(&lu[a & ~1u]);
                acc += v.x + v.y;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = (float)(lu[salt & (kWords - 1)] + acc);
}

template <int MODE, int PAT>
void run_lds(float *d, const char *name)
{
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    const int blocks = 2048;
    hipLaunchKernelGGL((k_lds<MODE, PAT>), dim3(blocks), dim3(256), 0, 0, d, 1);
    (void)hipDeviceSynchronize();
    (void)hipEventRecord(e0);
    for (int r = 0; r < 5; ++r) hipLaunchKernelGGL((k_lds<MODE, PAT>), dim3(blocks), dim3(256), 0, 0, d, r);
    (void)hipEventRecord(e1);
    (void)hipEventSynchronize(e1);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    const double ops = 5.0 * blocks * 256.0 * kSteps * 8 * (PAT == 4 ? 0.75 : 1.0);
    printf("lds  %-26s %6.2f lane-ops/clk/CU\n", name, ops / (ms * 1e-3) / 256.0 / 2.4e9);
}

__global__ void k_scatter(int n, const float2 *__restrict__ in, const int *__restrict__ p,
                          float2 *__restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[p[i]] = in[i];
}
__global__ void k_gather(int n, const float2 *__restrict__ in, const int *__restrict__ q,
                         float2 *__restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[q[i]];
}
__global__ void k_copy(int n, const float2 *__restrict__ in, float2 *__restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[i];
}
}  // namespace

int main()
{
    float *d = nullptr;
    if (hipMalloc(&d, 2048 * sizeof(float)) != hipSuccess) return 1;
    run_lds<1, 0>(d, "u32 atomic consecutive"); run_lds<1, 1>(d, "u32 atomic random");
    run_lds<1, 2>(d, "u32 atomic sorted runs");
    run_lds<2, 0>(d, "u64 atomic consecutive"); run_lds<2, 1>(d, "u64 atomic random");
    run_lds<2, 2>(d, "u64 atomic sorted runs");
    run_lds<2, 3>(d, "u64 atomic 8-word groups"); run_lds<2, 4>(d, "u64 atomic 6-of-8 groups");
    run_lds<0, 0>(d, "f32 atomic consecutive"); run_lds<0, 1>(d, "f32 atomic random");
    run_lds<3, 0>(d, "u32 read consecutive"); run_lds<3, 1>(d, "u32 read random");
    run_lds<4, 0>(d, "u64 read consecutive"); run_lds<4, 1>(d, "u64 read random");
    run_lds<4, 2>(d, "u64 read sorted runs");
    run_lds<4, 3>(d, "u64 read 8-word groups"); run_lds<4, 4>(d, "u64 read 6-of-8 groups");
    run_lds<5, 0>(d, "u128 read consecutive"); run_lds<5, 1>(d, "u128 read random");
    (void)hipFree(d);

    const int n = 10000000;
    std::vector<int> p(n), q(n);
    for (int i = 0; i < n; ++i) p[i] = i;
    std::mt19937 g(1);
    std::shuffle(p.begin(), p.end(), g);
    for (int i = 0; i < n; ++i) q[p[i]] = i;
    float2 *a = nullptr, *b = nullptr;
    int *dp = nullptr, *dq = nullptr;
    if (hipMalloc(&a, (size_t)n * 8) != hipSuccess || hipMalloc(&b, (size_t)n * 8) != hipSuccess ||
        hipMalloc(&dp, (size_t)n * 4) != hipSuccess || hipMalloc(&dq, (size_t)n * 4) != hipSuccess)
        return 1;
    (void)hipMemset(a, 0, (size_t)n * 8);
    (void)hipMemcpy(dp, p.data(), (size_t)n * 4, hipMemcpyHostToDevice);
    (void)hipMemcpy(dq, q.data(), (size_t)n * 4, hipMemcpyHostToDevice);
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    const int blocks = (n + 255) / 256;
    for (int k = 0; k < 3; ++k) {
        float ms = 0;
        for (int rep = 0; rep < 2; ++rep) {
            (void)hipEventRecord(e0);
            for (int r = 0; r < 10; ++r) {
                if (k == 0) hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, 0, n, a, b);
                else if (k == 1) hipLaunchKernelGGL(k_scatter, dim3(blocks), dim3(256), 0, 0, n, a, dp, b);
                else hipLaunchKernelGGL(k_gather, dim3(blocks), dim3(256), 0, 0, n, a, dq, b);
            }
            (void)hipEventRecord(e1);
            (void)hipEventSynchronize(e1);
            (void)hipEventElapsedTime(&ms, e0, e1);
        }
        printf("hbm  %-26s %.4f ms per 1e7 x 8 B\n", k == 0 ? "copy" : (k == 1 ? "scatter out[p[i]]" : "gather in[q[i]]"), ms / 10);
    }
    return 0;
}
