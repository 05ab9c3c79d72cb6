// Dispatch of spreading / interpolation to the instantiated kernel slices.
#include "internal.h"

namespace mn {
namespace detail {
template <typename T, int DIM>
hipError_t spread_dim(const Geom &g, int method, const Pts &P, const void *c, void *grid,
                      hipStream_t s, size_t lds);
template <typename T, int DIM>
hipError_t interp_dim(const Geom &g, int method, const Pts &P, const void *grid, void *c,
                      hipStream_t s, size_t lds);
extern template hipError_t spread_dim<float, 2>(const Geom &, int, const Pts &, const void *,
                                                void *, hipStream_t, size_t);
extern template hipError_t spread_dim<float, 3>(const Geom &, int, const Pts &, const void *,
                                                void *, hipStream_t, size_t);
extern template hipError_t spread_dim<double, 2>(const Geom &, int, const Pts &, const void *,
                                                 void *, hipStream_t, size_t);
extern template hipError_t spread_dim<double, 3>(const Geom &, int, const Pts &, const void *,
                                                 void *, hipStream_t, size_t);
extern template hipError_t interp_dim<float, 2>(const Geom &, int, const Pts &, const void *,
                                                void *, hipStream_t, size_t);
extern template hipError_t interp_dim<float, 3>(const Geom &, int, const Pts &, const void *,
                                                void *, hipStream_t, size_t);
extern template hipError_t interp_dim<double, 2>(const Geom &, int, const Pts &, const void *,
                                                 void *, hipStream_t, size_t);
extern template hipError_t interp_dim<double, 3>(const Geom &, int, const Pts &, const void *,
                                                 void *, hipStream_t, size_t);
}  // namespace detail
size_t sm_lds_bytes(const Geom &g, int prec, bool /*interp*/)
{
    const int P = (g.w + 1) / 2;
    size_t cells = 1;
    for (int d = 0; d < g.dim; ++d) cells *= (size_t)(g.m[d] + 2 * P);
    return cells * 2 * (prec == 0 ? sizeof(float) : sizeof(double));
}

hipError_t launch_spread(const Geom &g, int prec, int method, const Pts &P, const void *c,
                         void *grid, hipStream_t s)
{
    if (P.M == 0) return hipSuccess;
    const size_t lds = method == 3 ? sm_lds_bytes(g, prec, false) : 0;
    if (prec == 0)
        return g.dim == 2 ? detail::spread_dim<float, 2>(g, method, P, c, grid, s, lds)
                          : detail::spread_dim<float, 3>(g, method, P, c, grid, s, lds);
    return g.dim == 2 ? detail::spread_dim<double, 2>(g, method, P, c, grid, s, lds)
                      : detail::spread_dim<double, 3>(g, method, P, c, grid, s, lds);
}

hipError_t launch_interp(const Geom &g, int prec, int method, const Pts &P, const void *grid,
                         void *c, hipStream_t s)
{
    if (P.M == 0) return hipSuccess;
    const size_t lds = method == 3 ? sm_lds_bytes(g, prec, true) : 0;
    if (prec == 0)
        return g.dim == 2 ? detail::interp_dim<float, 2>(g, method, P, grid, c, s, lds)
                          : detail::interp_dim<float, 3>(g, method, P, grid, c, s, lds);
    return g.dim == 2 ? detail::interp_dim<double, 2>(g, method, P, grid, c, s, lds)
                      : detail::interp_dim<double, 3>(g, method, P, grid, c, s, lds);
}

}  // namespace mn
