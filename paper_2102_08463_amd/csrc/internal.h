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

// Sorted-point storage produced by setpts.
struct Pts {
    int M;
    const void *u[3];        // bin-relative coordinates g_i - binstart_i (plan precision), sorted
    const uint32_t *key;     // bin index per sorted point
    const int32_t *perm;     // sorted position -> input index
    const int32_t *binstart; // nbins + 1
    const int32_t *sub;      // subproblem records (bin, start, len, 0)
    const int32_t *nsub;     // device count of records
    int nsub_max;
    // unsorted (input order) copies for the GM method
    const void *u_in[3];
    const uint32_t *key_in;
};

// ---- bin sort (kernels_sort.hip) ------------------------------------------
// Scratch needed by the radix sort for M keys.
size_t radix_hist_elems(int M);
size_t scan_partial_elems(size_t n);

// key[j] and (optionally, for GM) u_in: bin index and bin-relative
// coordinates of every point in input order; flag |= 1 if a coordinate is
// non-finite or outside [-3pi, 3pi).
hipError_t launch_binkey(const Geom &g, int prec, int M, const void *x, const void *y,
                         const void *z, uint32_t *key, void *const u_in[3], int *flag,
                         hipStream_t s);

// Stable LSD radix sort of (key, index) pairs on the low `bits` bits.
// Returns in *keys_out / *vals_out the buffers (among the two ping-pong
// pairs) that hold the sorted keys and the permutation.
hipError_t radix_sort(int M, int bits, uint32_t *keysA, uint32_t *valsA, uint32_t *keysB,
                      uint32_t *valsB, uint32_t *hist, uint32_t *partials,
                      uint32_t **keys_out, uint32_t **vals_out, hipStream_t s);

// binstart[b] = first sorted position with key >= b, b = 0..nbins.
hipError_t launch_binstart(int M, int nbins, const uint32_t *skey, int32_t *binstart,
                           hipStream_t s);

// Subproblem list from bin starts; nsub_max = nbins + ceil(M / msub).
hipError_t launch_subproblems(int nbins, int msub, int nsub_max, const int32_t *binstart,
                              int32_t *subcount, uint32_t *partials, int32_t *sub,
                              int32_t *nsub, hipStream_t s);

// Sorted bin-relative coordinates: u[i] = g(x[perm[i]]) - binstart(key[i]).
hipError_t launch_gather_coords(const Geom &g, int prec, int M, const void *x, const void *y,
                                const void *z, const int32_t *perm, const uint32_t *skey,
                                void *const u[3], hipStream_t s);

// Exclusive prefix sum of n uint32 values (in and out may alias).
hipError_t scan_exclusive(const uint32_t *in, uint32_t *out, size_t n, uint32_t *partials,
                          hipStream_t s);

// ---- spreading / interpolation (kernels_spread.hip) -----------------------
// grid += spread of c (one vector) with the given method.
hipError_t launch_spread(const Geom &g, int prec, int method, const Pts &P, const void *c,
                         void *grid, hipStream_t s);
// c = interpolation of grid (one vector) with the given method.
hipError_t launch_interp(const Geom &g, int prec, int method, const Pts &P, const void *grid,
                         void *c, hipStream_t s);
// Dynamic LDS bytes the SM kernels need for these bins, and whether it fits.
size_t sm_lds_bytes(const Geom &g, int prec, bool interp);

// ---- correction (kernels_deconv.hip) --------------------------------------
// f[t] = p1 p2 p3 * grid[t][k mod n] over the modes, for ntransf transforms.
hipError_t launch_deconv(int dim, const int64_t N[3], const int n[3], int prec, int ntransf,
                         const void *grid, const void *const p[3], void *f, hipStream_t s);
// grid[t] = zero-padded p1 p2 p3 * f[t] (Sec. II-B step 1).
hipError_t launch_precorrect(int dim, const int64_t N[3], const int n[3], int prec,
                             int ntransf, const void *f, const void *const p[3], void *grid,
                             hipStream_t s);
// Fill n bytes of device memory with zero by a kernel.
hipError_t launch_zero(void *ptr, size_t bytes, hipStream_t s);

}  // namespace mn
