// Host-side helpers shared by plans and batches of libmnufft (not public).
#pragma once

#include "../../include/mnufft.h"
#include "internal.h"

#include <stdint.h>
#include <utility>
#include <vector>

namespace mn {
namespace host {

constexpr double kPi = 3.141592653589793;

// Kernel width w = ceil(log10(1/eps)) + 1 (Sec. II); a guard of 1e-9 keeps
// decade tolerances (whose logarithm is not exactly an integer in floating
// point) on the intended side.
int width_for_eps(double eps);

// Smallest 2^a 3^b 5^c >= max(2N, 2w) (Sec. II).
// General upsampling factor sigma (sigma = 2: the rule above, exactly).
int width_for_eps_sigma(double eps, double sigma);
double beta_for(int w, double sigma);
int64_t fine_size(int64_t N, int w, double sigma = 2.0);

// p_k = (2/w) / phi_hat(alpha k) * (-1)^k for k in I_N, alpha = w pi / n
// (Sec. II-A step 3; the sign is the lattice phase of grid point l at l h - pi).
void correction(int64_t N, int64_t n, int w, double beta, std::vector<double> &p);

// phi_hat(xi) = int_{-1}^{1} phi_beta(z) cos(xi z) dz at every xi (tanh-sinh
// quadrature, 513 nodes).
void es_fourier(double beta, const std::vector<double> &xi, std::vector<double> &out);

// Default bin extents for a fine grid n (dim dimensions): 64 cells in 1D,
// 32 x 32 in 2D and 16 x 8 x 8 in 3D (measured on gfx950; the paper's V100
// choice was 32 x 32 and 16 x 16 x 2, Sec. III-A, first remark), each at most
// the grid, then halved along the longest side while the grid holds fewer
// than kMinBins bins and that side is above kMinSide: a small grid cut into
// few bins leaves most of the GPU's compute units idle.
constexpr int64_t kMinBins = 1024;
constexpr int kMinSide = 8;
void default_bins(int dim, const int64_t n[3], int m[3]);

// Give a type 1 / 2 plan another method, bins and msub (c.method, binsize,
// msub; the rest of c is ignored), keeping its fine grid, FFT and correction
// factors; the points must be set again.  Used by the autotuner to time
// candidates on one plan.  Errors: ERR_ARG (bins that do not fit LDS for
// method SM, a type 3 plan), ERR_ALLOC, ERR_HIP.
int plan_set_params(mnufft_plan p, const mnufft_opts &c);

// Bits needed to hold bin indices 0 .. nbins - 1.
int bits_for(int64_t nbins);

// Cover table of the SM add-back for one dimension: for every grid index l,
// the (bin, offset in its padded tile) pairs whose tile lands on l after
// periodic wrapping; rows padded to the largest count kmax with bin -1.
void cover_table(int n, int m, int B, int P, std::vector<int2> &tab, int &kmax);

// Per-stage HIP-event timers on one stream.
struct Timers {
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[MNUFFT_NSTAGES];
    size_t used[MNUFFT_NSTAGES] = {};
    // Sum of recorded durations per stage (synchronises s); optionally clears.
    int read(hipStream_t s, double *ms, int64_t *count, int reset);
    void destroy();
};

// Brackets one stage with an event pair when the timers are on.
struct StageTimer {
    Timers &t;
    int stage;
    hipStream_t s;
    bool on;
    StageTimer(Timers &tt, int st, hipStream_t ss);
    ~StageTimer();
};

// In-place C2C rocFFT plan of the given lengths (first fastest); `sign` is
// the exponent sign.  Returns MNUFFT_OK or MNUFFT_ERR_FFT; *work receives the
// work-buffer size.
int make_rocfft(int prec, int dim, const int *n, size_t batch, int sign, void **plan,
                size_t *work);

}  // namespace host
}  // namespace mn
