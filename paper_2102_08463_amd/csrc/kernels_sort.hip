// Bin-sort of the nonuniform points (Sec. III-A, GM-sort and SM step 1).
//
// A point lies in the bin that holds its integer fine-grid coordinates
// l_i = floor((x_i + pi) / h_i).  The permutation t lists bin 0's points
// first, then bin 1's, ...; inside a bin the input order is kept, which makes
// t unique and reproducible.  It is built as a stable LSD radix sort of
// (bin key, input index) pairs with 8-bit digits: per pass a digit histogram
// per 4096-key tile, one exclusive scan over the (digit, tile) counts, and a
// scatter whose in-tile ranks come from wavefront ballots (all lanes holding
// the same digit are found with eight 64-bit ballots, so no lane order has to
// be assumed of LDS atomics).
//
// The grid coordinate is evaluated with a fixed sequence of correctly rounded
// double operations and no contraction: g = (x + pi) * S with S = n / (2 pi)
// rounded once on the host; then one whole-period correction.  That makes
// the keys, and hence t, reproducible bit for bit on any IEEE machine.
#include "internal.h"

#include <algorithm>

namespace mn {
namespace {

constexpr double kPi = 3.141592653589793;
constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr int kTile = kThreads * kItems;  // keys per radix block

// Folded grid coordinate in [0, n).  `bad` is set when one period shift does
// not bring the value into range (non-finite or beyond about [-3pi, 3pi)).
__device__ __forceinline__ double grid_coord(double x, double S, int n, int &bad)
{
    const double nd = (double)n;
    double g = __dmul_rn(__dadd_rn(x, kPi), S);
    if (g < 0.0) g = __dadd_rn(g, nd);
    if (g >= nd) g = __dsub_rn(g, nd);
    if (!(g >= 0.0 && g < nd)) {
        bad = 1;
        const double q = floor(__ddiv_rn(g, nd));
        g = __dsub_rn(g, __dmul_rn(q, nd));
        if (g >= nd) g = __dsub_rn(g, nd);
        if (!(g >= 0.0 && g < nd)) g = 0.0;
    }
    return g;
}

// Bin key of point j and its bin-relative coordinates u[0..dim-1]; bad is
// set when a coordinate needed a fallback fold.  For a batch (BATCH), the
// point's transform is found among the pt_off values (soff: an LDS copy when
// cached, else the table itself).
// (xv: the point's coordinates, already loaded; unused dimensions ignored)
template <typename T, bool BATCH>
__device__ __forceinline__ uint32_t point_key_of(const Geom &g, const T xc[3], const PtMap &map,
                                                 const TGeom *tg, int T_, const long long *soff,
                                                 bool cached, int j, T u[3], int &bad)
{
    uint32_t k = 0, stride = 1;
    Geom gg = g;
    if constexpr (BATCH) {
        const auto fld = [](const TGeom &a) { return a.pt_off; };
        const int t = cached ? find_cached(soff, T_, j) : find_transform(tg, T_, j, fld);
        gg = geom_of(g, tg[t]);
        k = (uint32_t)tg[t].bin_off;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        u[d] = (T)0;
        if (d >= gg.dim) continue;
        double xv = (double)xc[d];
        if (map.on) xv = __dmul_rn(__dsub_rn(xv, map.off[d]), map.mul[d]);
        const double gc = grid_coord(xv, gg.S[d], gg.n[d], bad);
        const int l = (int)gc;  // gc >= 0, so truncation is floor; l <= n - 1
        const int b = l / gg.m[d];
        k += (uint32_t)b * stride;
        stride *= (uint32_t)gg.B[d];
        u[d] = (T)(gc - (double)b * (double)gg.m[d]);
    }
    return k;
}

template <typename T, bool BATCH>
__device__ __forceinline__ uint32_t point_key(const Geom &g, const T *x, const T *y, const T *z,
                                              const PtMap &map, const TGeom *tg, int T_,
                                              const long long *soff, bool cached, int j, T u[3],
                                              int &bad)
{
    const T xc[3] = {x[j], g.dim >= 2 ? y[j] : (T)0, g.dim == 3 ? z[j] : (T)0};
    return point_key_of<T, BATCH>(g, xc, map, tg, T_, soff, cached, j, u, bad);
}

template <typename T, bool BATCH>
__global__ void __launch_bounds__(kThreads)
k_binkey(Geom g, int M, const T *__restrict__ x, const T *__restrict__ y,
         const T *__restrict__ z, uint32_t *__restrict__ key, T *__restrict__ u0,
         T *__restrict__ u1, T *__restrict__ u2, int *__restrict__ flag,
         const TGeom *__restrict__ tg, int T_, PtMap map)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    __shared__ long long soff[BATCH ? kTCache : 1];
    bool cached = false;
    if constexpr (BATCH) cached = cache_offsets(soff, tg, T_, [](const TGeom &a) { return a.pt_off; });
    if (j >= M) return;
    int bad = 0;
    T u[3];
    const uint32_t k = point_key<T, BATCH>(g, x, y, z, map, tg, T_, soff, cached, j, u, bad);
    T *us[3] = {u0, u1, u2};
#pragma unroll
    for (int d = 0; d < 3; ++d)
        if (d < g.dim) us[d][j] = u[d];
    key[j] = k;
    if (bad) atomicOr(flag, 1);
}

// Digit histogram of the first radix pass straight from the points (keys
// computed as point_key does; the validation flag set as k_binkey sets it).
// (1024 threads, kTile / 1024 points each: the key arithmetic is long, so
// more points are in flight per tile than with k_radix_hist's layout)
constexpr int kSrcThreads = 1024;
constexpr int kSrcItems = kTile / kSrcThreads;
template <typename T, bool BATCH>
__global__ void __launch_bounds__(kSrcThreads)
k_radix_hist_src(KeySrc src, int M, int shift, uint32_t dmask, int nblk,
                 uint32_t *__restrict__ hist)
{
    __shared__ uint32_t h[256];
    __shared__ long long soff[BATCH ? kTCache : 1];
    const int tid = threadIdx.x;
    if (tid < 256) h[tid] = 0;
    bool cached = false;
    if constexpr (BATCH)
        cached = cache_offsets(soff, src.tg, src.T, [](const TGeom &a) { return a.pt_off; });
    else
        __syncthreads();
    const T *x = (const T *)src.x, *y = (const T *)src.y, *z = (const T *)src.z;
    const int dim = src.g.dim;
    const int64_t base = (int64_t)blockIdx.x * kTile;
    int bad = 0;
    // every coordinate load first, so that their latencies overlap
    T xc[kSrcItems][3];
#pragma unroll
    for (int r = 0; r < kSrcItems; ++r) {
        const int64_t jc =
            std::min<int64_t>(base + (int64_t)r * kSrcThreads + tid, (int64_t)M - 1);
        xc[r][0] = x[jc];
        xc[r][1] = dim >= 2 ? y[jc] : (T)0;
        xc[r][2] = dim == 3 ? z[jc] : (T)0;
    }
#pragma unroll
    for (int r = 0; r < kSrcItems; ++r) {
        const int64_t idx = base + (int64_t)r * kSrcThreads + tid;
        const bool valid = idx < M;
        uint32_t d = 0;
        if (valid) {
            T u[3];
            d = (point_key_of<T, BATCH>(src.g, xc[r], src.map, src.tg, src.T, soff, cached,
                                        (int)idx, u, bad) >> shift) & dmask;
        }
        const uint32_t d0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)d);
        const bool same = !valid || d == d0;
        if (__all(same)) {
            const uint64_t vm = __ballot(valid);
            if ((threadIdx.x & 63) == 0 && vm) atomicAdd(&h[d0], (uint32_t)__popcll(vm));
        } else if (valid) {
            atomicAdd(&h[d], 1u);
        }
    }
    if (bad) atomicOr(src.flag, 1);
    __syncthreads();
    if (tid < 256) hist[(int64_t)tid * nblk + blockIdx.x] = h[tid];
}

// Per-tile digit histogram, stored digit-major: hist[d * nblk + blk]; the
// digit is (key >> shift) & dmask with dmask + 1 <= 256.
__global__ void __launch_bounds__(kThreads)
k_radix_hist(const uint32_t *__restrict__ keys, int M, int shift, uint32_t dmask, int nblk,
             uint32_t *__restrict__ hist)
{
    __shared__ uint32_t h[256];
    const int tid = threadIdx.x;
    h[tid] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
    // every key load first, so that their latencies overlap
    uint32_t kv[kItems];
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int64_t idx = base + (int64_t)r * kThreads + tid;
        kv[r] = idx < M ? keys[idx] : 0u;
    }
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int64_t idx = base + (int64_t)r * kThreads + tid;
        const bool valid = idx < M;
        const uint32_t d = valid ? (kv[r] >> shift) & dmask : 0u;
        // Lanes are contiguous in idx, so lane 0 is valid whenever any lane is.
        const uint32_t d0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)d);
        const bool same = !valid || d == d0;
        if (__all(same)) {
            const uint64_t vm = __ballot(valid);
            if ((threadIdx.x & 63) == 0 && vm) atomicAdd(&h[d0], (uint32_t)__popcll(vm));
        } else if (valid) {
            atomicAdd(&h[d], 1u);
        }
    }
    __syncthreads();
    hist[(int64_t)tid * nblk + blockIdx.x] = h[tid];
}

// Stable scatter of one radix pass over a tile of kTile keys, with NT
// threads: wave w owns keys [blk*kTile + w*items*64, +items*64), items =
// kTile / NT, and walks them in rounds of 64 consecutive keys, so ranks grow
// with the input index.  The tile is first rearranged in LDS into digit order
// (key, value and ND payload planes of T, the bin-relative coordinates), then
// each digit's run is written to its global range with consecutive threads
// on consecutive addresses.  When the staged tile takes more than 64 KB of
// LDS (3D, or double precision) one workgroup fills a CU, and 1024 threads
// hide its memory latency better than 512 (measured: 3D setpts 0.93 ->
// 0.74 ms at M = 2^24).
template <typename T, int ND>
constexpr int scatter_threads()
{
    return kTile * (8 + ND * (int)sizeof(T)) > 65536 ? 1024 : 512;
}

// SRC: 0 reads keys and payload; 1 computes them from the points (src, a
// plain plan); 2 the same for a batch (transform by binary search of pt_off).
template <typename T, int ND, int SRC = 0, int NT = scatter_threads<T, ND>()>
__global__ void __launch_bounds__(NT)
k_radix_scatter(const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin, int M,
                int shift, int dbits, int nblk, const uint32_t *__restrict__ offs,
                uint32_t *__restrict__ kout, uint32_t *__restrict__ vout, Payload pl, KeySrc src)
{
    constexpr int kSWaves = NT / 64, kSItems = kTile / NT;
    __shared__ uint32_t cnt[kSWaves][256];   // running per-wave digit counts, then prefixes
    __shared__ uint32_t tstart[256];         // tile-local start of each digit run
    __shared__ uint32_t gbase[256];          // global start of each digit run
    extern __shared__ __align__(16) unsigned char stage_raw[];
    uint32_t *skey = reinterpret_cast<uint32_t *>(stage_raw);
    uint32_t *sval = skey + kTile;
    T *spay = reinterpret_cast<T *>(sval + kTile);

    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    for (int e = tid; e < kSWaves * 256; e += NT) (&cnt[0][0])[e] = 0;
    __syncthreads();

    const int64_t tbase = (int64_t)blockIdx.x * kTile;
    const int64_t base = tbase + (int64_t)wave * (64 * kSItems);
    const int tcount = (int)std::min<int64_t>(kTile, (int64_t)M - tbase);
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const uint32_t dmask = (1u << dbits) - 1u;
    uint32_t kk[kSItems], vv[kSItems], rk[kSItems];
    T pu[SRC ? kSItems : 1][ND];  // payload computed from the points (SRC)
    if constexpr (SRC) {
        // every coordinate load first, so that their latencies overlap
        const T *cs[3] = {(const T *)src.x, (const T *)src.y, (const T *)src.z};
#pragma unroll
        for (int r = 0; r < kSItems; ++r) {
            const int64_t jc = std::min<int64_t>(base + r * 64 + lane, (int64_t)M - 1);
#pragma unroll
            for (int q = 0; q < ND; ++q) pu[r][q] = cs[q][jc];
        }
    }
#pragma unroll
    for (int r = 0; r < kSItems; ++r) {
        const int64_t idx = base + r * 64 + lane;
        const bool valid = idx < M;
        uint32_t key = 0u;
        if constexpr (SRC) {
            if (valid) {
                T xc[3] = {pu[r][0], ND >= 2 ? pu[r][ND >= 2 ? 1 : 0] : (T)0,
                           ND == 3 ? pu[r][ND == 3 ? 2 : 0] : (T)0};
                T u[3];
                int bad = 0;
                key = point_key_of<T, SRC == 2>(src.g, xc, src.map, src.tg, src.T, nullptr,
                                                false, (int)idx, u, bad);
#pragma unroll
                for (int q = 0; q < ND; ++q) pu[r][q] = u[q];
            }
        } else {
            key = valid ? kin[idx] : 0u;
        }
        const uint32_t val = valid ? (vin ? vin[idx] : (uint32_t)idx) : 0u;
        const uint32_t d = (key >> shift) & dmask;
        uint64_t mask = __ballot(valid);
        for (int b = 0; b < dbits; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            mask &= bit ? bb : ~bb;
        }
        const uint32_t rank = (uint32_t)__popcll(mask & lt);
        uint32_t old = 0;
        if (valid) {
            old = cnt[wave][d];
            if (rank == 0) cnt[wave][d] = old + (uint32_t)__popcll(mask);
        }
        kk[r] = key;
        vv[r] = val;
        rk[r] = old + rank;
    }
    __syncthreads();
    if (tid < 256) {
        // per digit: prefix over waves, then an exclusive scan over digits
        const int d = tid;
        uint32_t run = 0;
        for (int w = 0; w < kSWaves; ++w) {
            const uint32_t c = cnt[w][d];
            cnt[w][d] = run;
            run += c;
        }
        tstart[d] = run;  // digit total, scanned below
        gbase[d] = offs[(int64_t)d * nblk + blockIdx.x];
    }
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        uint32_t v = 0;
        if (tid < 256 && tid >= o) v = tstart[tid - o];
        __syncthreads();
        if (tid < 256) tstart[tid] += v;
        __syncthreads();
    }
    // tstart[d] now holds the inclusive sum of the digit totals, so digit d's
    // run in the tile starts at tstart[d - 1] (0 for d = 0).
#pragma unroll
    for (int r = 0; r < kSItems; ++r) {
        const int64_t idx = base + r * 64 + lane;
        if (idx < M) {
            const uint32_t d = (kk[r] >> shift) & dmask;
            const uint32_t start = d == 0 ? 0u : tstart[d - 1];
            const uint32_t lpos = start + cnt[wave][d] + rk[r];
            if (lpos >= (uint32_t)kTile) continue;  // cannot happen when the counts agree
            skey[lpos] = kk[r];
            sval[lpos] = vv[r];
#pragma unroll
            for (int q = 0; q < ND; ++q) {
                if constexpr (SRC) spay[q * kTile + lpos] = pu[r][q];
                else spay[q * kTile + lpos] = static_cast<const T *>(pl.in[q])[idx];
            }
        }
    }
    __syncthreads();
    for (int e = tid; e < tcount; e += NT) {
        const uint32_t key = skey[e];
        const uint32_t d = (key >> shift) & dmask;
        const uint32_t start = d == 0 ? 0u : tstart[d - 1];
        const uint32_t gpos = gbase[d] + (uint32_t)e - start;
        if (gpos >= (uint32_t)M) continue;  // cannot happen when the counts agree
        kout[gpos] = key;
        vout[gpos] = sval[e];
#pragma unroll
        for (int q = 0; q < ND; ++q) static_cast<T *>(pl.out[q])[gpos] = spay[q * kTile + e];
    }
}

// ---- generic exclusive scan (chunk totals; down-sweep adds earlier ones) ----
constexpr int kScanChunk = kThreads * kItems;

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane)
{
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// Exclusive scan of one value per thread over the block; returns the block total.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t &excl)
{
    __shared__ uint32_t wsum[kThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t inc = wave_incl_scan(v, lane);
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    uint32_t before = 0, total = 0;
    for (int w = 0; w < kThreads / 64; ++w) {
        if (w < wave) before += wsum[w];
        total += wsum[w];
    }
    __syncthreads();
    excl = before + inc - v;
    return total;
}

__global__ void __launch_bounds__(kThreads)
k_scan_reduce(const uint32_t *__restrict__ in, size_t n, uint32_t *__restrict__ partials)
{
    const size_t base = (size_t)blockIdx.x * kScanChunk;
    uint32_t s = 0;
    for (int r = 0; r < kItems; ++r) {
        const size_t i = base + (size_t)r * kThreads + threadIdx.x;
        if (i < n) s += in[i];
    }
    uint32_t ex;
    const uint32_t tot = block_excl_scan(s, ex);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kThreads)
k_scan_down(const uint32_t *__restrict__ in, uint32_t *__restrict__ out, size_t n,
            const uint32_t *__restrict__ partials)
{
    __shared__ uint32_t buf[kScanChunk + kScanChunk / 32];
    const size_t base = (size_t)blockIdx.x * kScanChunk;
    auto sk = [](int e) { return e + (e >> 5); };  // skew against bank conflicts
    for (int r = 0; r < kItems; ++r) {
        const int e = r * kThreads + threadIdx.x;
        const size_t i = base + e;
        buf[sk(e)] = (i < n) ? in[i] : 0u;
    }
    __syncthreads();
    // this chunk's offset: the sum of the earlier chunks' totals
    uint32_t before = 0;
    for (int k = threadIdx.x; k < (int)blockIdx.x; k += kThreads) before += partials[k];
    uint32_t ex0;
    before = block_excl_scan(before, ex0);
    uint32_t s = 0;
    for (int q = 0; q < kItems; ++q) s += buf[sk(threadIdx.x * kItems + q)];
    uint32_t ex;
    block_excl_scan(s, ex);
    uint32_t run = ex + before;
    for (int q = 0; q < kItems; ++q) {
        const int e = threadIdx.x * kItems + q;
        const uint32_t v = buf[sk(e)];
        buf[sk(e)] = run;
        run += v;
    }
    __syncthreads();
    for (int r = 0; r < kItems; ++r) {
        const int e = r * kThreads + threadIdx.x;
        const size_t i = base + e;
        if (i < n) out[i] = buf[sk(e)];
    }
}

__global__ void k_binstart(int M, int nbins, const uint32_t *__restrict__ skey,
                           int32_t *__restrict__ binstart)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b > nbins) return;
    int lo = 0, hi = M;  // first position with skey >= b
    while (lo < hi) {
        const int mid = lo + ((hi - lo) >> 1);
        if (skey[mid] < (uint32_t)b) lo = mid + 1; else hi = mid;
    }
    binstart[b] = lo;
}

// msub of bin b: the plan's, or in a batch that of the bin's transform.
__device__ __forceinline__ int msub_of(int b, int msub, const TGeom *tg, const int32_t *bin_t)
{
    return tg ? tg[bin_t[b]].msub : msub;
}

__global__ void k_subcount(int nbins, int msub, const int32_t *__restrict__ binstart,
                           uint32_t *__restrict__ cnt, const TGeom *__restrict__ tg,
                           const int32_t *__restrict__ bin_t)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b > nbins) return;
    if (b == nbins) { cnt[b] = 0; return; }
    const int c = binstart[b + 1] - binstart[b];
    const int ms = msub_of(b, msub, tg, bin_t);
    cnt[b] = (uint32_t)((c + ms - 1) / ms);
}

__global__ void k_subfill(int nbins, int msub, int nsub_max, const int32_t *__restrict__ binstart,
                          const uint32_t *__restrict__ off, int32_t *__restrict__ sub,
                          int32_t *__restrict__ nsub, const TGeom *__restrict__ tg,
                          const int32_t *__restrict__ bin_t)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    // the count is clamped to the list's capacity so that no consumer can
    // read past it, whatever the counts held
    const int total = std::min((int)off[nbins], nsub_max);
    if (q == 0) *nsub = total;
    if (q >= total || q >= nsub_max) return;
    int lo = 0, hi = nbins - 1;  // last bin b with off[b] <= q
    while (lo < hi) {
        const int mid = lo + ((hi - lo + 1) >> 1);
        if (off[mid] <= (uint32_t)q) lo = mid; else hi = mid - 1;
    }
    const int b = lo;
    const int ms = msub_of(b, msub, tg, bin_t);
    const int s = q - (int)off[b];
    const int start = binstart[b] + s * ms;
    const int len = std::min(ms, binstart[b + 1] - start);
    int4 rec;
    rec.x = b; rec.y = start; rec.z = len; rec.w = 0;
    reinterpret_cast<int4 *>(sub)[q] = rec;
}

inline int nblocks(int64_t n, int t) { return (int)((n + t - 1) / t); }

}  // namespace

size_t radix_hist_elems(int M) { return (size_t)256 * std::max(1, nblocks(M, kTile)); }

size_t scan_partial_elems(size_t n) { return (n + kScanChunk - 1) / kScanChunk + 1; }

hipError_t scan_exclusive(const uint32_t *in, uint32_t *out, size_t n, uint32_t *partials,
                          hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const int np = (int)((n + kScanChunk - 1) / kScanChunk);
    // chunk totals, then each chunk adds the totals before it (one chunk:
    // nothing before it, so the first kernel is skipped)
    if (np > 1)
        hipLaunchKernelGGL(k_scan_reduce, dim3(np), dim3(kThreads), 0, s, in, n, partials);
    hipLaunchKernelGGL(k_scan_down, dim3(np), dim3(kThreads), 0, s, in, out, n,
                       (const uint32_t *)partials);
    return hipGetLastError();
}

hipError_t launch_binkey(const Geom &g, int prec, int M, const void *x, const void *y,
                         const void *z, uint32_t *key, void *const u_in[3], int *flag,
                         hipStream_t s, const TGeom *tg, int T, const PtMap *map)
{
    if (M == 0) return hipSuccess;
    const dim3 grid(nblocks(M, kThreads)), blk(kThreads);
    PtMap pm{};
    if (map) pm = *map;
#define MN_BK(TT, BB)                                                                        \
    hipLaunchKernelGGL((k_binkey<TT, BB>), grid, blk, 0, s, g, M, (const TT *)x, (const TT *)y, \
                       (const TT *)z, key, (TT *)u_in[0], (TT *)u_in[1], (TT *)u_in[2], flag, tg, T, \
                       pm)
    if (prec == 0) {
        if (tg) MN_BK(float, true); else MN_BK(float, false);
    } else {
        if (tg) MN_BK(double, true); else MN_BK(double, false);
    }
#undef MN_BK
    return hipGetLastError();
}

int radix_passes(int bits) { return std::max(1, (bits + 7) / 8); }

hipError_t radix_sort(int M, int bits, int prec, int dim, uint32_t *keysA, uint32_t *valsA,
                      uint32_t *keysB, uint32_t *valsB, const Payload *pays, uint32_t *hist,
                      uint32_t *partials, uint32_t **keys_out, uint32_t **vals_out, hipStream_t s,
                      const KeySrc *src)
{
    // Keys start in keysA with implicit values 0..M-1; each pass moves the
    // pairs to the other buffer.  Pass p moves the payload as pays[p] says.
    // Digits of equal width dbits <= 8 over the passes: fewer digits per pass
    // mean longer runs of each digit per tile, hence more coalesced writes.
    const int passes = radix_passes(bits);
    const int dbits = std::max(1, (bits + passes - 1) / passes);
    const uint32_t dmask = (1u << dbits) - 1u;
    const int nblk = std::max(1, nblocks(M, kTile));
    uint32_t *kb[2] = {keysA, keysB}, *vb[2] = {valsA, valsB};
    int cur = 0;
    for (int p = 0; p < passes; ++p) {
        if (M > 0) {
            const int shift = dbits * p;
            // pass 0 from the points themselves when a source is given
            const int from = (p == 0 && src) ? (src->tg ? 2 : 1) : 0;
            const KeySrc ks = src ? *src : KeySrc{};
            if (from) {
#define MN_HSRC(TT)                                                                           \
    do {                                                                                      \
        if (from == 2)                                                                        \
            hipLaunchKernelGGL((k_radix_hist_src<TT, true>), dim3(nblk), dim3(kSrcThreads), 0, \
                               s, ks, M, shift, dmask, nblk, hist);                           \
        else                                                                                  \
            hipLaunchKernelGGL((k_radix_hist_src<TT, false>), dim3(nblk), dim3(kSrcThreads),   \
                               0, s, ks, M, shift, dmask, nblk, hist);                        \
    } while (0)
                if (prec == 0) MN_HSRC(float);
                else MN_HSRC(double);
#undef MN_HSRC
            } else {
                hipLaunchKernelGGL(k_radix_hist, dim3(nblk), dim3(kThreads), 0, s,
                                   (const uint32_t *)kb[cur], M, shift, dmask, nblk, hist);
            }
            // digits above dmask are empty: only the first dmask + 1 rows are scanned
            hipError_t e = scan_exclusive(hist, hist, (size_t)(dmask + 1) * nblk, partials, s);
            if (e != hipSuccess) return e;
            const uint32_t *vin = p == 0 ? nullptr : (const uint32_t *)vb[cur];
#define MN_SCATTER1(TT, DD, SS)                                                             \
    do {                                                                                    \
        const size_t lds = (size_t)kTile * (8 + DD * sizeof(TT));                           \
        if (lds > 65536)                                                                    \
            (void)hipFuncSetAttribute((const void *)k_radix_scatter<TT, DD, SS>,            \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
        hipLaunchKernelGGL((k_radix_scatter<TT, DD, SS>), dim3(nblk),                       \
                           dim3(scatter_threads<TT, DD>()), lds, s,                        \
                           (const uint32_t *)kb[cur], vin, M, shift, dbits, nblk,           \
                           (const uint32_t *)hist, kb[1 - cur], vb[1 - cur], pays[p], ks); \
    } while (0)
#define MN_SCATTER(TT, DD)                                                                  \
    do {                                                                                    \
        if (from == 2) MN_SCATTER1(TT, DD, 2);                                              \
        else if (from == 1) MN_SCATTER1(TT, DD, 1);                                         \
        else MN_SCATTER1(TT, DD, 0);                                                        \
    } while (0)
            if (prec == 0) {
                if (dim == 1) MN_SCATTER(float, 1);
                else if (dim == 2) MN_SCATTER(float, 2);
                else MN_SCATTER(float, 3);
            } else {
                if (dim == 1) MN_SCATTER(double, 1);
                else if (dim == 2) MN_SCATTER(double, 2);
                else MN_SCATTER(double, 3);
            }
#undef MN_SCATTER
#undef MN_SCATTER1
        }
        cur = 1 - cur;
    }
    *keys_out = kb[cur];
    *vals_out = vb[cur];
    return hipGetLastError();
}

hipError_t launch_binstart(int M, int nbins, const uint32_t *skey, int32_t *binstart,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_binstart, dim3(nblocks(nbins + 1, 256)), dim3(256), 0, s, M, nbins,
                       skey, binstart);
    return hipGetLastError();
}

// ---- processing order of the SM kernels -----------------------------------
// The SM kernels give each lane of a wave one point and have all lanes touch
// the same tap of their points at once, so a wave's LDS addresses are the
// points' tile start cells plus a common offset.  The LDS serves 64-bit
// accesses sixteen lanes at a time and stalls when two of them hit the same
// bank; the banks follow the cell index modulo 16 (two or four banks per
// cell), so sixteen points whose start-cell indices differ modulo 16 are
// served without conflict whatever the tap.  This kernel orders each
// subproblem's points round-robin over their start-cell index modulo 16:
// every point of rank k in its residue class comes before every point of
// rank k + 1, residues ascending within a rank, i.e. point (r, k) goes to
//   pos = sum_t min(c_t, k) + #{t < r : c_t > k}     (c_t = class sizes).
// The sorted coordinates, the permutation, each point's sorted position and
// its slot in the spreading kernels' start-cell histogram are written in
// that order.  Subproblems above kBalCap points keep their sorted order.
// A block loads a subproblem's points once (coalesced, kBalItems per
// thread), ranks them in their classes with LDS atomics, then writes each
// output array through an LDS stage so that the global stores are
// contiguous too.  The ranks come from LDS atomics, so the order within a
// class may differ between runs; the SM kernels' results do not depend on
// the order (integer tile sums, per-point interpolation).
constexpr int kBalCap = 4096;
constexpr int kBalThreads = 256;
// Two instantiations share the subproblems: ITEMS = 8 takes those of up to
// 2048 points (3D bins, typically), ITEMS = 16 the rest, so small
// subproblems neither load unused rounds nor hold the larger one's registers.
template <typename T, int DIM, int ITEMS>
__global__ void __launch_bounds__(kBalThreads)
k_balance(Geom g, const int32_t *__restrict__ sub, const int32_t *__restrict__ nsubp,
          const T *__restrict__ u0, const T *__restrict__ u1, const T *__restrict__ u2,
          const int32_t *__restrict__ perm, T *__restrict__ v0, T *__restrict__ v1,
          T *__restrict__ v2, int32_t *__restrict__ vperm, int32_t *__restrict__ spos,
          uint16_t *__restrict__ hslot)
{
    constexpr int kBalItems = ITEMS;
    constexpr int kLo = ITEMS == 8 ? 0 : 8 * kBalThreads;         // sizes n with kLo < n
    constexpr int kHi = ITEMS == 8 ? 8 * kBalThreads : 1 << 30;   // and n <= kHi
    __shared__ unsigned cnt[16];
    __shared__ __align__(16) unsigned char stage_raw[kBalItems * kBalThreads * sizeof(T)];
    T *sT = reinterpret_cast<T *>(stage_raw);
    int32_t *sI = reinterpret_cast<int32_t *>(stage_raw);
    uint16_t *sH = reinterpret_cast<uint16_t *>(stage_raw);
    const int tid = threadIdx.x;
    const int P = (g.w + 1) / 2;
    const int p1 = g.m[0] + 2 * P, p2 = g.m[1] + 2 * P;
    const T lead = (T)P - (T)(0.5 * g.w);
    const StartHist hg = start_hist_rt(DIM, g.w, g.m[0], g.m[1], g.m[2]);
    // the spreading kernels' start-cell histogram slot (same expressions)
    const auto slot = [&](T a, T b, T c) {
        return (uint16_t)hist_slot_rt(hg, DIM >= 2 ? start_cell_rt<T>(b, g.w) : 0,
                                      DIM == 3 ? start_cell_rt<T>(c, g.w) : 0,
                                      start_cell_rt<T>(a, g.w));
    };
    const int nsub = *nsubp;
    for (int q = blockIdx.x; q < nsub; q += gridDim.x) {
        const int4 rec = reinterpret_cast<const int4 *>(sub)[q];
        const int n = rec.z;
        if (n <= kLo || n > kHi) continue;  // the other instantiation's subproblem
        if (n > kBalCap) {  // the same for the whole block: keep the sorted order
            for (int j = tid; j < n; j += kBalThreads) {
                const int i = rec.y + j;
                const T a = u0[i], b = DIM >= 2 ? u1[i] : (T)0, c = DIM == 3 ? u2[i] : (T)0;
                v0[i] = a;
                if (DIM >= 2) v1[i] = b;
                if (DIM == 3) v2[i] = c;
                vperm[i] = perm[i];
                spos[i] = i;
                hslot[i] = slot(a, b, c);
            }
            continue;
        }
        if (tid < 16) cnt[tid] = 0u;
        __syncthreads();
        T a[kBalItems], b[kBalItems], c[kBalItems];
        int pm[kBalItems], pos[kBalItems];
#pragma unroll
        for (int it = 0; it < kBalItems; ++it) {
            const int j = tid + it * kBalThreads;
            const int i = rec.y + min(j, n - 1);
            a[it] = u0[i];
            b[it] = DIM >= 2 ? u1[i] : (T)0;
            c[it] = DIM == 3 ? u2[i] : (T)0;
            pm[it] = perm[i];
        }
#pragma unroll
        for (int it = 0; it < kBalItems; ++it) {
            const int j = tid + it * kBalThreads;
            pos[it] = 0;
            if (j < n) {
                int base = (int)ceil(a[it] + lead);
                if (DIM >= 2) base += p1 * (int)ceil(b[it] + lead);
                if (DIM == 3) base += p1 * p2 * (int)ceil(c[it] + lead);
                const unsigned r = (unsigned)base & 15u;
                pos[it] = (int)(r | (atomicAdd(&cnt[r], 1u) << 4));
            }
        }
        __syncthreads();
        unsigned cc[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) cc[t] = cnt[t];
#pragma unroll
        for (int it = 0; it < kBalItems; ++it) {
            const unsigned r = (unsigned)pos[it] & 15u, k = (unsigned)pos[it] >> 4;
            int o = 0;
#pragma unroll
            for (int t = 0; t < 16; ++t) o += (int)min(cc[t], k) + ((t < (int)r && cc[t] > k) ? 1 : 0);
            pos[it] = o;
        }
        // each output through the stage: scattered LDS writes, contiguous stores
        const auto emit = [&](auto *stage, auto *dst, auto value) {
#pragma unroll
            for (int it = 0; it < kBalItems; ++it)
                if (tid + it * kBalThreads < n) stage[pos[it]] = value(it);
            __syncthreads();
            for (int j = tid; j < n; j += kBalThreads) dst[rec.y + j] = stage[j];
            __syncthreads();
        };
        emit(sT, v0, [&](int it) { return a[it]; });
        if constexpr (DIM >= 2) emit(sT, v1, [&](int it) { return b[it]; });
        if constexpr (DIM == 3) emit(sT, v2, [&](int it) { return c[it]; });
        emit(sI, vperm, [&](int it) { return pm[it]; });
        emit(sI, spos, [&](int it) { return rec.y + tid + it * kBalThreads; });
        emit(sH, hslot, [&](int it) { return slot(a[it], b[it], c[it]); });
    }
}

namespace {
__global__ void k_iota(int n, int32_t *__restrict__ out)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        out[i] = i;
}
}  // namespace

hipError_t launch_iota(int32_t *out, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_iota, dim3(std::min(nblocks(n, 256), 4096)), dim3(256), 0, s, n, out);
    return hipGetLastError();
}

hipError_t launch_balance(const Geom &g, int prec, int nsub_max, const int32_t *sub,
                          const int32_t *nsub, const void *const u[3], const int32_t *perm,
                          void *const v[3], int32_t *vperm, int32_t *spos, uint16_t *hslot,
                          hipStream_t s)
{
    if (nsub_max <= 0) return hipSuccess;
    const dim3 grid(std::max(1, std::min(nsub_max, 256 * 8)));
#define MN_BAL1(TT, DD, II)                                                                    \
    hipLaunchKernelGGL((k_balance<TT, DD, II>), grid, dim3(kBalThreads), 0, s, g, sub, nsub,   \
                       (const TT *)u[0], (const TT *)u[1], (const TT *)u[2], perm, (TT *)v[0],  \
                       (TT *)v[1], (TT *)v[2], vperm, spos, hslot)
#define MN_BAL(TT, DD)                                                                         \
    do {                                                                                       \
        MN_BAL1(TT, DD, 8);                                                                    \
        MN_BAL1(TT, DD, 16);                                                                   \
    } while (0)
    if (prec == 0) {
        if (g.dim == 1) MN_BAL(float, 1);
        else if (g.dim == 2) MN_BAL(float, 2);
        else MN_BAL(float, 3);
    } else {
        if (g.dim == 1) MN_BAL(double, 1);
        else if (g.dim == 2) MN_BAL(double, 2);
        else MN_BAL(double, 3);
    }
#undef MN_BAL
#undef MN_BAL1
    return hipGetLastError();
}

hipError_t launch_subproblems(int nbins, int msub, int nsub_max, const int32_t *binstart,
                              int32_t *subcount, uint32_t *partials, int32_t *sub,
                              int32_t *nsub, hipStream_t s, const TGeom *tg, int T,
                              const int32_t *bin_t)
{
    if (tg && !bin_t) return hipErrorInvalidValue;
    (void)T;
    uint32_t *cnt = reinterpret_cast<uint32_t *>(subcount);
    hipLaunchKernelGGL(k_subcount, dim3(nblocks(nbins + 1, 256)), dim3(256), 0, s, nbins, msub,
                       binstart, cnt, tg, bin_t);
    hipError_t e = scan_exclusive(cnt, cnt, (size_t)nbins + 1, partials, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_subfill, dim3(nblocks(std::max(nsub_max, 1), 256)), dim3(256), 0, s,
                       nbins, msub, nsub_max, binstart, (const uint32_t *)cnt, sub, nsub, tg,
                       bin_t);
    return hipGetLastError();
}

}  // namespace mn
