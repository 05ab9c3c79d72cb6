// Internal declarations shared by the host plan code and the kernel
// translation units of libmnufft.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mn {

// Geometry of the fine grid and its bins, as the kernels see it.
struct Geom {
    int dim;
    int n[3];        // fine grid n_i (1 for unused dimensions)
    int m[3];        // bin extents m_i
    int B[3];        // bins per dimension ceil(n_i / m_i)
    int nbins;
    double S[3];     // n_i / (2 pi), rounded once in double
    int w;           // kernel width
    double beta;     // ES shape parameter
    int pad;         // ceil(w / 2): halo of a padded bin (Sec. III-A, SM step 2)
};

// Per-transform geometry of a batch, kept in a device table.  A batch puts
// all transforms' bins in one global numbering (bin_off), their points,
// fine grids and modes back to back (pt_off, grid_off, mode_off), so that one
// sort, one subproblem list and one launch per stage cover every transform.
struct TGeom {
    int n[3], m[3], B[3];
    int N[3];
    int bin_off, nbins;
    int pt_off, M;
    int msub;
    int p_off[3];    // offsets into the concatenated correction factors, per dimension
    int cov_off[3];  // offsets (entries) into the concatenated cover tables, per dimension
    int kmax[3];
    long long grid_off;
    long long mode_off;
    double S[3];
};

// Index t of the last table entry whose `field` is <= v (entries sorted by field).
template <typename F>
__device__ __forceinline__ int find_transform(const TGeom *tg, int T, long long v, F field)
{
    int lo = 0, hi = T - 1;
    while (lo < hi) {
        const int mid = lo + ((hi - lo + 1) >> 1);
        if ((long long)field(tg[mid]) <= v) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Per-element lookups in a batch go through an LDS copy of one offset field
// of the table when it is short enough: a binary search in global memory is a
// chain of dependent loads per element, in LDS it is a few cycles per step.
constexpr int kTCache = 1024;
template <typename F>
__device__ __forceinline__ bool cache_offsets(long long *s, const TGeom *tg, int T, F field)
{
    const bool ok = T <= kTCache;
    if (ok)
        for (int t = threadIdx.x; t < T; t += blockDim.x) s[t] = (long long)field(tg[t]);
    __syncthreads();
    return ok;
}
// Index of the last cached offset <= v.
__device__ __forceinline__ int find_cached(const long long *s, int T, long long v)
{
    int lo = 0, hi = T - 1;
    while (lo < hi) {
        const int mid = lo + ((hi - lo + 1) >> 1);
        if (s[mid] <= v) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Workgroups of a launch are dispatched to the eight XCDs in turn (block b to
// XCD b mod 8), and each XCD has its own L2.  Kernels whose neighbouring
// blocks read neighbouring data renumber their blocks with this map, so that
// each XCD takes one contiguous range of the logical block indices and the
// shared cache lines meet in one L2.
__device__ __forceinline__ int xcd_block(int b, int nb)
{
    constexpr int kXcd = 8;
    const int q = nb / kXcd, r = nb % kXcd, x = b % kXcd;
    return x * q + min(x, r) + b / kXcd;
}

// Geometry of transform t as a Geom (shared fields from g).
__device__ __forceinline__ Geom geom_of(const Geom &g, const TGeom &t)
{
    Geom r = g;
    for (int d = 0; d < 3; ++d) {
        r.n[d] = t.n[d];
        r.m[d] = t.m[d];
        r.B[d] = t.B[d];
        r.S[d] = t.S[d];
    }
    r.nbins = t.nbins;
    return r;
}

// ---- start-cell histogram of the SM spreading scale ------------------------
// Start cell (first tap in padded-tile coordinates, halo P = ceil(w/2)) of a
// point at bin-relative coordinate u: ceil(u + P - w/2), evaluated the same
// way by the spreading kernels and by setpts.
template <typename T>
__host__ __device__ inline int start_cell_rt(T u, int w)
{
    const T v = u + (T)((w + 1) / 2);
    return (int)ceil(v - (T)(0.5 * w));
}

// Layout of the start-cell histogram of a tile with bin extents m: start
// cells s_d in [0, m_d + 1] (c_d of them) in the first two dimensions, x
// rows of pitch lx = c_1 + w - 1 (room for the box sums along x in place).
// In 3D the third start coordinate is not kept: summing a cell's column
// over every z start still bounds it, at a cost of about (m_3 + 2) / w in
// tightness, and the box sums stay two-dimensional and cheap.
struct StartHist {
    int c[3];
    int lx, ly;
    int size;
};

__host__ __device__ inline StartHist start_hist_rt(int dim, int w, int m1, int m2, int m3)
{
    (void)m3;
    StartHist h;
    h.c[0] = m1 + 2;
    h.c[1] = dim >= 2 ? m2 + 2 : 1;
    h.c[2] = 1;
    h.lx = h.c[0] + w - 1;
    h.ly = h.c[1];
    h.size = h.ly * h.lx;
    return h;
}

// Histogram slot of start cell (s1, s2, s3), clamped into the histogram (the
// start of a point inside its bin is always in range); s2 = s3 = 0 for
// absent dimensions.
__host__ __device__ inline int hist_slot_rt(const StartHist &h, int s2, int s3, int s1)
{
    s1 = s1 < 0 ? 0 : (s1 > h.c[0] - 1 ? h.c[0] - 1 : s1);
    s2 = s2 < 0 ? 0 : (s2 > h.c[1] - 1 ? h.c[1] - 1 : s2);
    s3 = s3 < 0 ? 0 : (s3 > h.c[2] - 1 ? h.c[2] - 1 : s3);
    return (s3 * h.ly + s2) * h.lx + s1;
}

// Sorted-point storage produced by setpts.
struct Pts {
    int M;
    const void *u[3];        // bin-relative coordinates g_i - binstart_i (plan precision), sorted
    const uint32_t *key;     // bin index per sorted point
    const int32_t *perm;     // sorted position -> input index; null: c in sorted order
    const int32_t *spos;     // with perm null: sorted position of each processed point
                             // (null: the position itself)
    const uint16_t *hslot;   // SM spreading: start-cell histogram slot of each processed
                             // point (null: computed from the coordinates)
    const int32_t *binstart; // nbins + 1
    const int32_t *sub;      // subproblem records (bin, start, len, 0)
    const int32_t *nsub;     // device count of records
    int nsub_max;
    // unsorted (input order) copies for the GM method
    const void *u_in[3];
    const uint32_t *key_in;
    // SM spreading: per-subproblem tile slots and their reduction
    const int32_t *suboff;    // nbins + 1: first subproblem of each bin
    void *scratch;            // nsub_max slots of ts2 reals
    int ts2;                  // reals per slot (>= 2 * padded-bin cells, multiple of 8)
    int G;                    // tiles merged per leader in heavily loaded bins
    const int32_t *mergelist; // leaders (subproblem indices)
    int32_t *nmerge;          // device: [0] count of leaders, [1] count of listed bins
    int32_t *heavy;           // bin-wise add-back: bins whose neighbourhood holds a bin of
                              // several tiles (nbins entries; null: the add-back gathers)
    const int2 *cov[3];       // per-dimension cover tables (see k_tile_gather)
    int kmax[3];
    void *cmax;               // 1024 partial maxima of |Re c|, |Im c| of the vector being spread
    int msub;                 // maximum points per subproblem
    // batches: per-transform geometry (device) and count; nullptr / 1 for a plain plan
    const TGeom *tg;
    int T;
    long long ncells;         // fine-grid cells over all transforms
    const int32_t *bin_t;     // batches: transform of every bin (nbins entries)
    const int32_t *q0;        // SM kernels: first subproblem to process (device; null: 0),
                              // with *nsub the end of the range
};

// ---- bin sort (kernels_sort.hip) ------------------------------------------
// Scratch needed by the radix sort for M keys.
size_t radix_hist_elems(int M);
size_t scan_partial_elems(size_t n);

// Planes of per-point reals carried along by a radix pass.
struct Payload {
    const void *in[3];
    void *out[3];
};

// Optional affine map applied to the coordinates before binning, in double:
// x -> (x - off) * mul (used by type 3, whose rescaled points are never
// rounded to the plan precision before their bin-relative coordinate is).
struct PtMap {
    int on;
    double off[3];
    double mul[3];
};

// key[j] and u_in[d][j]: bin index and bin-relative coordinates of every
// point in input order; flag |= 1 if a coordinate is non-finite or outside
// [-3pi, 3pi).
// With a batch table tg (T entries), point j belongs to the transform whose
// pt_off range holds j and gets the global key bin_off + local key.
hipError_t launch_binkey(const Geom &g, int prec, int M, const void *x, const void *y,
                         const void *z, uint32_t *key, void *const u_in[3], int *flag,
                         hipStream_t s, const TGeom *tg = nullptr, int T = 1,
                         const PtMap *map = nullptr);

// The caller's points as the source of a bin-sort's keys: with one, the
// sort's first pass computes every point's bin key and bin-relative
// coordinates itself (the expressions of k_binkey) instead of reading keys
// and payload that launch_binkey wrote, and sets *flag like launch_binkey.
struct KeySrc {
    Geom g;
    const void *x, *y, *z;
    int *flag;
    const TGeom *tg;  // batches: per-transform table (T entries), else null
    int T;
    PtMap map;
};

// Number of 8-bit passes for keys of `bits` bits (at least one).
int radix_passes(int bits);

// Stable LSD radix sort of (key, index) pairs on the low `bits` bits, with
// dim payload planes of the plan precision; pass p reads pays[p].in and
// writes pays[p].out.  Returns in *keys_out / *vals_out the buffers (among
// the two ping-pong pairs) that hold the sorted keys and the permutation.
// With src, pass 0 takes keys and payload from the points (keysA and
// pays[0].in are not read).
hipError_t radix_sort(int M, int bits, int prec, int dim, uint32_t *keysA, uint32_t *valsA,
                      uint32_t *keysB, uint32_t *valsB, const Payload *pays, uint32_t *hist,
                      uint32_t *partials, uint32_t **keys_out, uint32_t **vals_out, hipStream_t s,
                      const KeySrc *src = nullptr);

// binstart[b] = first sorted position with key >= b, b = 0..nbins.
hipError_t launch_binstart(int M, int nbins, const uint32_t *skey, int32_t *binstart,
                           hipStream_t s);

// Subproblem list from bin starts; nsub_max = nbins + ceil(M / msub).
// With a batch table, each bin uses its transform's msub.
hipError_t launch_subproblems(int nbins, int msub, int nsub_max, const int32_t *binstart,
                              int32_t *subcount, uint32_t *partials, int32_t *sub,
                              int32_t *nsub, hipStream_t s, const TGeom *tg = nullptr, int T = 1,
                              const int32_t *bin_t = nullptr);

// Processing order of the SM kernels within each subproblem (see k_balance):
// v[d] / vperm / spos / hslot receive the sorted coordinates, the
// permutation, the sorted position and the start-cell histogram slot of the
// point processed at each position.
// out[i] = i for i < n.
hipError_t launch_iota(int32_t *out, int n, hipStream_t s);
hipError_t launch_balance(const Geom &g, int prec, int nsub_max, const int32_t *sub,
                          const int32_t *nsub, const void *const u[3], const int32_t *perm,
                          void *const v[3], int32_t *vperm, int32_t *spos, uint16_t *hslot,
                          hipStream_t s);

// Exclusive prefix sum of n uint32 values (in and out may alias).
hipError_t scan_exclusive(const uint32_t *in, uint32_t *out, size_t n, uint32_t *partials,
                          hipStream_t s);

// ---- spreading / interpolation (kernels_spread.hip) -----------------------
// Spreading of c (one vector) with the given method.  part bit 0 runs the
// accumulation (GM / GMSORT: atomics into a zeroed grid; SM: per-subproblem
// tiles), bit 1 the SM add-back that writes every grid cell, bit 2 the SM
// pre-pass computing partial maxima of |c| into P.cmax (zeroed before it).
hipError_t launch_spread(const Geom &g, int prec, int method, const Pts &P, const void *c,
                         void *grid, hipStream_t s, int part = 7);
// c = interpolation of grid (one vector) with the given method.
hipError_t launch_interp(const Geom &g, int prec, int method, const Pts &P, const void *grid,
                         void *c, hipStream_t s);
// out_i[j] = sum_t Re(conj(wts[t][j]) d/dx_i (interpolation of grid t at x_j)),
// for ntransf grids (one complex per cell each) and weights (ntransf x M,
// input order); out planes are M reals in input order.
hipError_t launch_interp_grad(const Geom &g, int prec, const Pts &P, int ntransf,
                              const void *grid, const void *wts, void *const out[3],
                              hipStream_t s);
// Dynamic LDS bytes the SM kernels need for these bins and subproblem size.
size_t sm_lds_bytes(const Geom &g, int prec, bool interp, int msub);
// Single-precision SM spreading keeps up to this many gathered strengths of
// a subproblem in LDS, so the strengths are read from HBM once (fewer in 3D,
// where bins hold fewer points and LDS occupancy matters more).
// (2D: 2816 keeps the default 32 x 32 tile plus the stage within 40 KB, four
// workgroups per CU; a uniform 2D bin of the default workload holds about
// 2440 points, and the few strengths past the stage are gathered again:
// measured 2D spread 0.265 -> 0.250 ms uniform, 0.188 -> 0.165 ms clustered)
inline int smp_stage(int dim, int msub)
{
    const int cap = dim <= 2 ? 2816 : 1024;
    return msub < cap ? msub : cap;
}
// Strengths the two-word SM spreading kernel stages in LDS per subproblem
// for its second pass over them (1D double precision only: single precision
// makes one pass, and in 2D / 3D double precision the tiles leave no room).
inline int sm2_stage(int dim, int prec, int msub)
{
    const int cap = dim == 1 && prec != 0 ? 2048 : 0;
    return msub < cap ? msub : cap;
}
// Reals per scratch tile slot of SM spreading.
int sm_tile_stride(const Geom &g);
// Leaders of tile groups to merge: subproblems q with (q - suboff[bin]) % G == 0
// in bins with more than G subproblems (*nmerge must be zero on entry).
hipError_t launch_merge_list(int nsub_max, const int32_t *nsub, const int32_t *sub,
                             const int32_t *suboff, int G, int32_t *mergelist, int32_t *nmerge,
                             hipStream_t s);

// ---- correction (kernels_deconv.hip) --------------------------------------
// f[t] = p1 p2 p3 * grid[t][k mod n] over the modes, for ntransf transforms.
hipError_t launch_deconv(int dim, const int64_t N[3], const int n[3], int prec, int ntransf,
                         const void *grid, const void *const p[3], void *f, hipStream_t s);
// grid[t] = zero-padded p1 p2 p3 * f[t] (Sec. II-B step 1).
hipError_t launch_precorrect(int dim, const int64_t N[3], const int n[3], int prec,
                             int ntransf, const void *f, const void *const p[3], void *grid,
                             hipStream_t s);
// Batched correction over all transforms of a batch (concatenated layout).
hipError_t launch_deconv_batch(const TGeom *tg, int T, long long nmodes, int prec,
                               const void *grid, const void *const p[3], void *f, hipStream_t s);
hipError_t launch_precorrect_batch(const TGeom *tg, int T, long long ncells, int prec,
                                   const void *f, const void *const p[3], void *grid,
                                   hipStream_t s);
// ---- type 3 (kernels_type3.hip) -------------------------------------------
// Per-dimension constants of the type 3 factors (see kernels_type3.hip): the
// rescaled value of v is (v - off) * scale; the phases use mul.
struct T3Affine {
    double off[3];
    double scale[3];
    double mul[3];
};
// Blocks (<= 1024) that launch_t3_bounds uses for n values; part needs
// 3 * dim doubles per block: (min, max, non-finite flag) per dimension.
int t3_bounds_blocks(int n);
hipError_t launch_t3_bounds(int prec, int n, int dim, const void *const a[3], double *part,
                            hipStream_t s);
// pre[j] = exp(i sg sum_d mul_d (x_jd - off_d)), complex of the plan precision.
hipError_t launch_t3_prephase(int prec, int n, int dim, const void *const x[3],
                              const T3Affine &af, int sg, void *pre, hipStream_t s);
// post[k] = exp(i sg sum_d mul_d s_kd) prod_d (2/w) / phi_hat(w scale_d (s_kd - off_d) / 2),
// log phi_hat from cheb = (ximax, nc Chebyshev terms in 2 (xi/ximax)^2 - 1) (device, double).
hipError_t launch_t3_postfac(int prec, int n, int dim, const void *const sf[3],
                             const T3Affine &af, int sg, int w, const double *cheb, int nc,
                             void *post, hipStream_t s);
// out[t][i] = in[t][i] * fac[i] over ntransf stacked complex vectors of n entries.
hipError_t launch_cmul(int prec, long long n, int ntransf, const void *in, const void *fac,
                       void *out, hipStream_t s);

// ---- learned selector (kernels_mlp.hip) -----------------------------------
// The batched density histograms (mnufft_density_features_batch) in parts,
// for callers that keep the partial rows (T * MNUFFT_DENSITY_BATCH_WORK_BYTES
// at part) between calls: clearing them, and counting into them (they must
// be zero before).
hipError_t launch_hist_clear(int T, uint32_t *part, hipStream_t s);
hipError_t launch_hist_count(int prec, int T, const int64_t *off, const void *x, const void *y,
                             uint32_t *part, hipStream_t s);
// The selector's pass over T counted sets in one launch: features from the
// partial rows (returned to zero) and the nscal scalars per set (scal, T x
// nscal), the network (F = 256 + nscal inputs) and the argmin as
// launch_mlp_argmin gives it.
hipError_t launch_select_rows(int T, const int64_t *off, uint32_t *part, const float *scal,
                              int nscal, int F, int H, int K, const float *params,
                              const unsigned long long mask[2], int *idx, float *gap,
                              hipStream_t s);
// The network (F -> H -> H -> K, mnufft_mlp_forward's parameter layout) and
// an argmin fused, one block per row of X (T rows of stride ldx): idx[t] is
// the column of smallest output among those whose bit is set in mask
// (column k: bit k % 64 of mask[k / 64], K <= 128), -1 when none is allowed,
// and gap[t] its distance to the runner-up (infinity with one allowed).
// F <= 512, H <= 256, K <= 128, else hipErrorInvalidValue.
hipError_t launch_mlp_argmin(int F, int H, int K, const float *params, int T, const float *X,
                             int ldx, const unsigned long long mask[2], int *idx, float *gap,
                             hipStream_t s);

// Fill n bytes of device memory with zero by a kernel.
hipError_t launch_zero(void *ptr, size_t bytes, hipStream_t s);

}  // namespace mn
