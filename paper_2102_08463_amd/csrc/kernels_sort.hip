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

template <typename T, bool BATCH>
__global__ void __launch_bounds__(kThreads)
k_binkey(Geom g, int M, const T *__restrict__ x, const T *__restrict__ y,
         const T *__restrict__ z, uint32_t *__restrict__ key, T *__restrict__ u0,
         T *__restrict__ u1, T *__restrict__ u2, int *__restrict__ flag,
         const TGeom *__restrict__ tg, int T_)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    int bad = 0;
    uint32_t k = 0, stride = 1;
    Geom gg = g;
    if constexpr (BATCH) {
        const int t = find_transform(tg, T_, j, [](const TGeom &a) { return a.pt_off; });
        gg = geom_of(g, tg[t]);
        k = (uint32_t)tg[t].bin_off;
    }
    const T *xs[3] = {x, y, z};
    T *us[3] = {u0, u1, u2};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (d >= gg.dim) break;
        const double gc = grid_coord((double)xs[d][j], gg.S[d], gg.n[d], bad);
        const int l = (int)gc;  // gc >= 0, so truncation is floor; l <= n - 1
        const int b = l / gg.m[d];
        k += (uint32_t)b * stride;
        stride *= (uint32_t)gg.B[d];
        us[d][j] = (T)(gc - (double)b * (double)gg.m[d]);
    }
    key[j] = k;
    if (bad) atomicOr(flag, 1);
}

// Per-tile digit histogram, stored digit-major: hist[d * nblk + blk].
__global__ void __launch_bounds__(kThreads)
k_radix_hist(const uint32_t *__restrict__ keys, int M, int shift, int nblk,
             uint32_t *__restrict__ hist)
{
    __shared__ uint32_t h[256];
    const int tid = threadIdx.x;
    h[tid] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int r = 0; r < kItems; ++r) {
        const int64_t idx = base + (int64_t)r * kThreads + tid;
        const bool valid = idx < M;
        const uint32_t d = valid ? (keys[idx] >> shift) & 255u : 0u;
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

// Stable scatter of one radix pass over a tile of kTile keys, with kSThreads
// threads: wave w owns keys [blk*kTile + w*kSItems*64, +kSItems*64) and walks
// them in kSItems rounds of 64 consecutive keys, so ranks grow with the
// input index.  The tile is first rearranged in LDS into digit order (key,
// value and ND payload planes of T, the bin-relative coordinates), then each
// digit's run is written to its global range with consecutive threads on
// consecutive addresses.
constexpr int kSThreads = 512;
constexpr int kSWaves = kSThreads / 64;
constexpr int kSItems = kTile / kSThreads;

template <typename T, int ND>
__global__ void __launch_bounds__(kSThreads)
k_radix_scatter(const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin, int M,
                int shift, int nblk, const uint32_t *__restrict__ offs,
                uint32_t *__restrict__ kout, uint32_t *__restrict__ vout, Payload pl)
{
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
    for (int e = tid; e < kSWaves * 256; e += kSThreads) (&cnt[0][0])[e] = 0;
    __syncthreads();

    const int64_t tbase = (int64_t)blockIdx.x * kTile;
    const int64_t base = tbase + (int64_t)wave * (64 * kSItems);
    const int tcount = (int)std::min<int64_t>(kTile, (int64_t)M - tbase);
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t kk[kSItems], vv[kSItems], rk[kSItems];
#pragma unroll
    for (int r = 0; r < kSItems; ++r) {
        const int64_t idx = base + r * 64 + lane;
        const bool valid = idx < M;
        const uint32_t key = valid ? kin[idx] : 0u;
        const uint32_t val = valid ? (vin ? vin[idx] : (uint32_t)idx) : 0u;
        const uint32_t d = (key >> shift) & 255u;
        uint64_t mask = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
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
            const uint32_t d = (kk[r] >> shift) & 255u;
            const uint32_t start = d == 0 ? 0u : tstart[d - 1];
            const uint32_t lpos = start + cnt[wave][d] + rk[r];
            if (lpos >= (uint32_t)kTile) continue;  // cannot happen when the counts agree
            skey[lpos] = kk[r];
            sval[lpos] = vv[r];
#pragma unroll
            for (int q = 0; q < ND; ++q)
                spay[q * kTile + lpos] = static_cast<const T *>(pl.in[q])[idx];
        }
    }
    __syncthreads();
    for (int e = tid; e < tcount; e += kSThreads) {
        const uint32_t key = skey[e];
        const uint32_t d = (key >> shift) & 255u;
        const uint32_t start = d == 0 ? 0u : tstart[d - 1];
        const uint32_t gpos = gbase[d] + (uint32_t)e - start;
        if (gpos >= (uint32_t)M) continue;  // cannot happen when the counts agree
        kout[gpos] = key;
        vout[gpos] = sval[e];
#pragma unroll
        for (int q = 0; q < ND; ++q) static_cast<T *>(pl.out[q])[gpos] = spay[q * kTile + e];
    }
}

// ---- generic exclusive scan (reduce, scan partials, down-sweep) ----------
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

__global__ void __launch_bounds__(1024) k_scan_partials(uint32_t *__restrict__ partials, int np)
{
    // One block: thread t scans a contiguous run of the partials serially.
    __shared__ uint32_t sums[1024];
    const int t = threadIdx.x;
    const int per = (np + 1023) / 1024;
    const int lo = std::min(np, t * per), hi = std::min(np, lo + per);
    uint32_t s = 0;
    for (int i = lo; i < hi; ++i) s += partials[i];
    sums[t] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const uint32_t v = (t >= o) ? sums[t - o] : 0u;
        __syncthreads();
        sums[t] += v;
        __syncthreads();
    }
    uint32_t run = sums[t] - s;
    for (int i = lo; i < hi; ++i) {
        const uint32_t v = partials[i];
        partials[i] = run;
        run += v;
    }
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
    uint32_t s = 0;
    for (int q = 0; q < kItems; ++q) s += buf[sk(threadIdx.x * kItems + q)];
    uint32_t ex;
    block_excl_scan(s, ex);
    uint32_t run = ex + partials[blockIdx.x];
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
__device__ __forceinline__ int msub_of(int b, int msub, const TGeom *tg, int T)
{
    if (!tg) return msub;
    return tg[find_transform(tg, T, b, [](const TGeom &a) { return a.bin_off; })].msub;
}

__global__ void k_subcount(int nbins, int msub, const int32_t *__restrict__ binstart,
                           uint32_t *__restrict__ cnt, const TGeom *__restrict__ tg, int T)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b > nbins) return;
    if (b == nbins) { cnt[b] = 0; return; }
    const int c = binstart[b + 1] - binstart[b];
    const int ms = msub_of(b, msub, tg, T);
    cnt[b] = (uint32_t)((c + ms - 1) / ms);
}

__global__ void k_subfill(int nbins, int msub, int nsub_max, const int32_t *__restrict__ binstart,
                          const uint32_t *__restrict__ off, int32_t *__restrict__ sub,
                          int32_t *__restrict__ nsub, const TGeom *__restrict__ tg, int T)
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
    const int ms = msub_of(b, msub, tg, T);
    const int s = q - (int)off[b];
    const int start = binstart[b] + s * ms;
    const int len = std::min(ms, binstart[b + 1] - start);
    int4 rec;
    rec.x = b; rec.y = start; rec.z = len; rec.w = 0;
    reinterpret_cast<int4 *>(sub)[q] = rec;
}

// Order inside each subproblem by first tap cell.  A subproblem's points are
// rearranged so that their first tap cells (s_1, s_2) in the padded bin
// (s_i = ceil(u_i + P - w/2), P = ceil(w/2)) ascend in row-major order, equal
// cells keeping the bin-sorted order.  One workgroup of kCellWaves wavefronts
// per chunk of up to kCellChunk points of a subproblem (chunks are ordered
// independently); wavefront v owns the v-th quarter of the chunk:
//   A. keys into LDS and per-wavefront counts per cell (LDS integer atomics:
//      counts do not depend on their order);
//   B. one exclusive scan over cells of the summed counts, and per cell the
//      running sum over wavefronts: each wavefront's first slot in each cell;
//   C. every wavefront sweeps its quarter 64 points at a time in order: lanes
//      holding equal keys are found with one ballot per key bit, each point
//      gets its wavefront's slot plus its rank among equal keys before it,
//      and the lowest of them advances the slot (no atomics, so the result
//      does not depend on any order of LDS operations);
//   D. every new position reads its point (the inverse order is kept in LDS,
//      so the stores are coalesced and only the loads scatter, within the
//      chunk's few kilobytes).
// The result is deterministic and stays within the chunk's own range.
constexpr int kCellChunk = 4096;
constexpr int kCellWaves = 4;
constexpr int kCellThreads = 64 * kCellWaves;

__device__ __forceinline__ unsigned long long peers_of(int key, int bits, bool ok)
{
    unsigned long long m = __ballot(ok);
    for (int b = 0; b < bits; ++b) {
        const bool on = (key >> b) & 1;
        const unsigned long long v = __ballot(on);
        m &= on ? v : ~v;
    }
    return m;
}

template <typename T, bool BATCH>
__global__ void __launch_bounds__(kCellThreads)
k_cellsort(Geom g, int W, const int32_t *__restrict__ sub, const int32_t *__restrict__ nsubp,
           const T *__restrict__ ui0, const T *__restrict__ ui1, const int32_t *__restrict__ pin,
           T *__restrict__ uo0, T *__restrict__ uo1, int32_t *__restrict__ pout,
           const TGeom *__restrict__ tg, int T_)
{
    // kCellWaves x ncap counters (ncap >= p1 p2), then 2 x kCellChunk 16-bit slots
    extern __shared__ uint32_t lds[];
    __shared__ uint32_t wsum[kCellWaves];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const unsigned long long below = (1ull << lane) - 1ull;
    const int P = (W + 1) / 2;
    const T hw = (T)(0.5 * W);
    const int nsub = *nsubp;
    int ncap = (g.m[0] + 2 * P) * (g.m[1] + 2 * P);  // the largest padded bin
    uint16_t *kp = reinterpret_cast<uint16_t *>(lds + kCellWaves * ncap);  // key of point j
    uint16_t *src = kp + kCellChunk;                                      // point at position o
    for (int q = blockIdx.x; q < nsub; q += gridDim.x) {
        const int4 rec = reinterpret_cast<const int4 *>(sub)[q];
        int m0 = g.m[0], m1 = g.m[1];
        if constexpr (BATCH) {
            const TGeom &tt =
                tg[find_transform(tg, T_, rec.x, [](const TGeom &a) { return a.bin_off; })];
            m0 = tt.m[0];
            m1 = tt.m[1];
        }
        const int p1 = m0 + 2 * P, p2 = m1 + 2 * P, nh = p1 * p2;
        const int bits = nh > 1 ? 32 - __clz(nh - 1) : 0;
        uint32_t *cw = lds + wv * ncap;  // this wavefront's counters
        for (int c0 = rec.y; c0 < rec.y + rec.z; c0 += kCellChunk) {
            const int n = min(kCellChunk, rec.y + rec.z - c0);
            const int lo = n * wv / kCellWaves, hi = n * (wv + 1) / kCellWaves;
            for (int e = tid; e < kCellWaves * ncap; e += kCellThreads) lds[e] = 0u;
            __syncthreads();
            // A. keys (the same rounding as the spreading kernels' first tap) and counts
            for (int j = lo + lane; j < hi; j += 64) {
                const int sx = min(max((int)ceil((ui0[c0 + j] + (T)P) - hw), 0), p1 - 1);
                const int sy = min(max((int)ceil((ui1[c0 + j] + (T)P) - hw), 0), p2 - 1);
                const int key = sy * p1 + sx;
                kp[j] = (uint16_t)key;
                atomicAdd(&cw[key], 1u);
            }
            __syncthreads();
            // B. first slot of each wavefront in each cell
            {
                const int per = (nh + kCellThreads - 1) / kCellThreads;
                const int elo = min(tid * per, nh), ehi = min(elo + per, nh);
                uint32_t sum = 0;
                for (int e = elo; e < ehi; ++e)
                    for (int v = 0; v < kCellWaves; ++v) sum += lds[v * ncap + e];
                uint32_t x = sum;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const uint32_t y = __shfl_up(x, o, 64);
                    if (lane >= o) x += y;
                }
                if (lane == 63) wsum[wv] = x;
                __syncthreads();
                uint32_t run = x - sum;
                for (int v = 0; v < wv; ++v) run += wsum[v];
                for (int e = elo; e < ehi; ++e)
                    for (int v = 0; v < kCellWaves; ++v) {
                        const uint32_t c = lds[v * ncap + e];
                        lds[v * ncap + e] = run;
                        run += c;
                    }
            }
            __syncthreads();
            // C. positions, in order within each wavefront's quarter (a
            //    wavefront's LDS operations complete in program order)
            for (int j0 = lo; j0 < hi; j0 += 64) {
                const bool ok = j0 + lane < hi;
                const int key = ok ? (int)kp[j0 + lane] : 0;
                const unsigned long long pe = peers_of(key, bits, ok);
                const int pos = ok ? (int)cw[key] + __popcll(pe & below) : 0;
                __builtin_amdgcn_wave_barrier();
                if (ok && (pe & below) == 0ull) cw[key] += (uint32_t)__popcll(pe);
                if (ok) src[pos] = (uint16_t)(j0 + lane);
                __builtin_amdgcn_wave_barrier();
            }
            __syncthreads();
            // D. move
            for (int o = tid; o < n; o += kCellThreads) {
                const int j = c0 + (int)src[o];
                uo0[c0 + o] = ui0[j];
                uo1[c0 + o] = ui1[j];
                pout[c0 + o] = pin[j];
            }
            __syncthreads();
        }
    }
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
    hipLaunchKernelGGL(k_scan_reduce, dim3(np), dim3(kThreads), 0, s, in, n, partials);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, s, partials, np);
    hipLaunchKernelGGL(k_scan_down, dim3(np), dim3(kThreads), 0, s, in, out, n,
                       (const uint32_t *)partials);
    return hipGetLastError();
}

hipError_t launch_binkey(const Geom &g, int prec, int M, const void *x, const void *y,
                         const void *z, uint32_t *key, void *const u_in[3], int *flag,
                         hipStream_t s, const TGeom *tg, int T)
{
    if (M == 0) return hipSuccess;
    const dim3 grid(nblocks(M, kThreads)), blk(kThreads);
#define MN_BK(TT, BB)                                                                        \
    hipLaunchKernelGGL((k_binkey<TT, BB>), grid, blk, 0, s, g, M, (const TT *)x, (const TT *)y, \
                       (const TT *)z, key, (TT *)u_in[0], (TT *)u_in[1], (TT *)u_in[2], flag, tg, T)
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
                      uint32_t *partials, uint32_t **keys_out, uint32_t **vals_out, hipStream_t s)
{
    // Keys start in keysA with implicit values 0..M-1; each pass moves the
    // pairs to the other buffer.  Pass p moves the payload as pays[p] says.
    const int passes = radix_passes(bits);
    const int nblk = std::max(1, nblocks(M, kTile));
    uint32_t *kb[2] = {keysA, keysB}, *vb[2] = {valsA, valsB};
    int cur = 0;
    for (int p = 0; p < passes; ++p) {
        if (M > 0) {
            const int shift = 8 * p;
            hipLaunchKernelGGL(k_radix_hist, dim3(nblk), dim3(kThreads), 0, s,
                               (const uint32_t *)kb[cur], M, shift, nblk, hist);
            hipError_t e = scan_exclusive(hist, hist, (size_t)256 * nblk, partials, s);
            if (e != hipSuccess) return e;
            const uint32_t *vin = p == 0 ? nullptr : (const uint32_t *)vb[cur];
#define MN_SCATTER(TT, DD)                                                                  \
    do {                                                                                    \
        const size_t lds = (size_t)kTile * (8 + DD * sizeof(TT));                           \
        if (lds > 65536)                                                                    \
            (void)hipFuncSetAttribute((const void *)k_radix_scatter<TT, DD>,                \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
        hipLaunchKernelGGL((k_radix_scatter<TT, DD>), dim3(nblk), dim3(kSThreads), lds, s,   \
                           (const uint32_t *)kb[cur], vin, M, shift, nblk,                  \
                           (const uint32_t *)hist, kb[1 - cur], vb[1 - cur], pays[p]);      \
    } while (0)
            if (prec == 0) {
                if (dim == 2) MN_SCATTER(float, 2); else MN_SCATTER(float, 3);
            } else {
                if (dim == 2) MN_SCATTER(double, 2); else MN_SCATTER(double, 3);
            }
#undef MN_SCATTER
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

hipError_t launch_subproblems(int nbins, int msub, int nsub_max, const int32_t *binstart,
                              int32_t *subcount, uint32_t *partials, int32_t *sub,
                              int32_t *nsub, hipStream_t s, const TGeom *tg, int T)
{
    uint32_t *cnt = reinterpret_cast<uint32_t *>(subcount);
    hipLaunchKernelGGL(k_subcount, dim3(nblocks(nbins + 1, 256)), dim3(256), 0, s, nbins, msub,
                       binstart, cnt, tg, T);
    hipError_t e = scan_exclusive(cnt, cnt, (size_t)nbins + 1, partials, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_subfill, dim3(nblocks(std::max(nsub_max, 1), 256)), dim3(256), 0, s,
                       nbins, msub, nsub_max, binstart, (const uint32_t *)cnt, sub, nsub, tg, T);
    return hipGetLastError();
}

hipError_t launch_cellsort(const Geom &g, int prec, int nsub_max, const int32_t *sub,
                           const int32_t *nsub, const void *const u_in[3], const int32_t *perm_in,
                           void *const u_out[3], int32_t *perm_out, int ts2, hipStream_t s,
                           const TGeom *tg, int T)
{
    (void)ts2;
    if (nsub_max <= 0) return hipSuccess;
    const int P = (g.w + 1) / 2;
    const int64_t ncap = (int64_t)(g.m[0] + 2 * P) * (g.m[1] + 2 * P);
    if (g.dim != 2 || ncap > 65535) return hipErrorInvalidValue;  // cell keys are 16-bit
    const size_t lds = (size_t)kCellWaves * ncap * 4 + (size_t)kCellChunk * 4;
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    const dim3 grid(std::min(nsub_max, 16384)), block(kCellThreads);
#define MN_CELLSORT(TT, BB)                                                                   \
    do {                                                                                      \
        auto k = k_cellsort<TT, BB>;                                                          \
        if (lds > 65536)                                                                      \
            (void)hipFuncSetAttribute((const void *)k,                                       \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);   \
        hipLaunchKernelGGL(k, grid, block, lds, s, g, g.w, sub, nsub, (const TT *)u_in[0],   \
                           (const TT *)u_in[1], perm_in, (TT *)u_out[0], (TT *)u_out[1],      \
                           perm_out, tg, T);                                                  \
    } while (0)
    if (prec == 0) {
        if (tg) MN_CELLSORT(float, true); else MN_CELLSORT(float, false);
    } else {
        if (tg) MN_CELLSORT(double, true); else MN_CELLSORT(double, false);
    }
#undef MN_CELLSORT
    return hipGetLastError();
}

}  // namespace mn
