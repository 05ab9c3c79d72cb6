// Host-side helpers shared by plans and batches of libmnufft.
#include "host_common.h"

#include <rocfft/rocfft.h>

#include <algorithm>
#include <cmath>

namespace mn {
namespace host {

int width_for_eps(double eps) { return (int)std::ceil(std::log10(1.0 / eps) - 1e-9) + 1; }

static bool smooth235(int64_t n)
{
    for (int64_t p : {2, 3, 5})
        while (n % p == 0) n /= p;
    return n == 1;
}

int width_for_eps_sigma(double eps, double sigma)
{
    if (sigma == 2.0) return width_for_eps(eps);
    return (int)std::ceil(std::log(1.0 / eps) / (kPi * std::sqrt(1.0 - 1.0 / sigma)) - 1e-9);
}

double beta_for(int w, double sigma)
{
    return sigma == 2.0 ? 2.30 * w : 0.97 * kPi * w * (1.0 - 0.5 / sigma);
}

int64_t fine_size(int64_t N, int w, double sigma)
{
    const int64_t sn = sigma == 2.0 ? 2 * N : (int64_t)std::ceil(sigma * (double)N - 1e-9);
    int64_t n = std::max<int64_t>(sn, 2 * (int64_t)w);
    while (!smooth235(n)) ++n;
    return n;
}

// phi_hat(xi) = int_{-1}^{1} phi_beta(z) exp(-i xi z) dz = 2 int_0^1 phi(z) cos(xi z) dz
// by the tanh-sinh rule z = (1 + tanh u)/2, u = (pi/2) sinh t, which is
// insensitive to the square-root behaviour of phi at z = 1.  Step h, nodes
// t = k h for |k| <= K; ww carries the kernel value and the Jacobian.
static void es_quadrature(double beta, double h, int K, std::vector<double> &zz,
                          std::vector<double> &ww)
{
    zz.clear();
    ww.clear();
    zz.reserve(2 * K + 1);
    ww.reserve(2 * K + 1);
    for (int k = -K; k <= K; ++k) {
        const double t = k * h;
        const double u = 0.5 * kPi * std::sinh(t);
        const double one_minus_z = 1.0 / (1.0 + std::exp(2.0 * u));
        const double z = 1.0 - one_minus_z;
        const double ch = std::cosh(u);
        const double dz = 0.25 * kPi * std::cosh(t) / (ch * ch);
        const double s = one_minus_z * (1.0 + z);  // 1 - z^2 without cancellation
        const double phi = std::exp(beta * (std::sqrt(std::max(s, 0.0)) - 1.0));
        zz.push_back(z);
        ww.push_back(h * dz * phi);
    }
}

void es_fourier(double beta, const std::vector<double> &xi, std::vector<double> &out)
{
    std::vector<double> zz, ww;
    es_quadrature(beta, 1.0 / 64.0, 4 * 64, zz, ww);  // t in [-4, 4]: weights beyond < 1e-20
    out.assign(xi.size(), 0.0);
    for (size_t i = 0; i < xi.size(); ++i) {
        double acc = 0.0;
        for (size_t q = 0; q < zz.size(); ++q) acc += ww[q] * std::cos(xi[i] * zz[q]);
        out[i] = 2.0 * acc;
    }
}

void correction(int64_t N, int64_t n, int w, double beta, std::vector<double> &p)
{
    std::vector<double> xi(N), ph;
    const double alpha = w * kPi / (double)n;
    for (int64_t i = 0; i < N; ++i) xi[i] = alpha * (double)(i - N / 2);
    es_fourier(beta, xi, ph);
    p.resize(N);
    for (int64_t i = 0; i < N; ++i) {
        const int64_t k = i - N / 2;
        p[i] = (2.0 / w) / ph[i] * ((k % 2 == 0) ? 1.0 : -1.0);
    }
}

void default_bins(int dim, const int64_t n[3], int m[3])
{
    static const int defm[3][3] = {{64, 1, 1}, {32, 32, 1}, {16, 8, 8}};
    for (int d = 0; d < 3; ++d)
        m[d] = d < dim ? (int)std::min<int64_t>(defm[dim - 1][d], n[d]) : 1;
    for (;;) {
        int64_t nb = 1;
        int dl = 0;
        for (int d = 0; d < dim; ++d) {
            nb *= (n[d] + m[d] - 1) / m[d];
            if (m[d] > m[dl]) dl = d;
        }
        if (nb >= kMinBins || m[dl] <= kMinSide) break;
        m[dl] = (m[dl] + 1) / 2;
    }
}

int bits_for(int64_t nbins)
{
    int b = 0;
    while (((int64_t)1 << b) < nbins) ++b;
    return b;
}

void cover_table(int n, int m, int B, int P, std::vector<int2> &tab, int &kmax)
{
    const int pt = m + 2 * P;
    std::vector<std::vector<int2>> lists((size_t)n);
    for (int nb = 0; nb < B; ++nb)
        for (int s = 0; s < pt; ++s) {
            int l = (nb * m - P + s) % n;
            if (l < 0) l += n;
            lists[(size_t)l].push_back(make_int2(nb, s));
        }
    kmax = 1;
    for (auto &v : lists) kmax = std::max(kmax, (int)v.size());
    tab.assign((size_t)n * kmax, make_int2(-1, 0));
    for (int l = 0; l < n; ++l)
        for (size_t j = 0; j < lists[(size_t)l].size(); ++j)
            tab[(size_t)l * kmax + j] = lists[(size_t)l][j];
}

int Timers::read(hipStream_t s, double *ms, int64_t *count, int reset)
{
    if (hipStreamSynchronize(s) != hipSuccess) return MNUFFT_ERR_HIP;
    for (int st = 0; st < MNUFFT_NSTAGES; ++st) {
        double tot = 0.0;
        for (size_t i = 0; i < used[st]; ++i) {
            float e = 0.f;
            if (hipEventElapsedTime(&e, ev[st][i].first, ev[st][i].second) != hipSuccess)
                return MNUFFT_ERR_HIP;
            tot += e;
        }
        ms[st] = tot;
        if (count) count[st] = (int64_t)used[st];
        if (reset) used[st] = 0;
    }
    return MNUFFT_OK;
}

void Timers::destroy()
{
    for (int st = 0; st < MNUFFT_NSTAGES; ++st) {
        for (auto &e : ev[st]) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        ev[st].clear();
        used[st] = 0;
    }
}

StageTimer::StageTimer(Timers &tt, int st, hipStream_t ss) : t(tt), stage(st), s(ss), on(tt.on)
{
    if (!on) return;
    auto &v = t.ev[stage];
    if (t.used[stage] == v.size()) {
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess) { on = false; return; }
        if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); on = false; return; }
        v.emplace_back(a, b);
    }
    (void)hipEventRecord(v[t.used[stage]].first, s);
}

StageTimer::~StageTimer()
{
    if (!on) return;
    (void)hipEventRecord(t.ev[stage][t.used[stage]].second, s);
    ++t.used[stage];
}

int make_rocfft(int prec, int dim, const int *n, size_t batch, int sign, void **plan, size_t *work)
{
    size_t len[3];
    for (int d = 0; d < dim; ++d) len[d] = (size_t)n[d];
    rocfft_plan pl = nullptr;
    rocfft_status st = rocfft_plan_create(
        &pl, rocfft_placement_inplace,
        sign < 0 ? rocfft_transform_type_complex_forward : rocfft_transform_type_complex_inverse,
        prec == MNUFFT_F32 ? rocfft_precision_single : rocfft_precision_double, (size_t)dim, len,
        batch, nullptr);
    if (st != rocfft_status_success) return MNUFFT_ERR_FFT;
    size_t wb = 0;
    if (rocfft_plan_get_work_buffer_size(pl, &wb) != rocfft_status_success) {
        rocfft_plan_destroy(pl);
        return MNUFFT_ERR_FFT;
    }
    *plan = pl;
    *work = wb;
    return MNUFFT_OK;
}

}  // namespace host
}  // namespace mn
