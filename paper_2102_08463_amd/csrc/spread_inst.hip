// One (precision, dimension) slice of the spreading / interpolation kernels,
// selected by MN_T (float or double) and MN_D (1, 2 or 3) on the compiler
// command line, so that the 6 slices compile in parallel.
#include "spread_kernels.h"

#if !defined(MN_T) || !defined(MN_D)
#error "compile with -DMN_T=float|double -DMN_D=1|2|3"
#endif

namespace mn {
namespace detail {
template hipError_t spread_dim<MN_T, MN_D>(const Geom &, int, const Pts &, const void *, void *,
                                          hipStream_t, size_t, int);
template hipError_t interp_dim<MN_T, MN_D>(const Geom &, int, const Pts &, const void *, void *,
                                          hipStream_t, size_t);
template hipError_t grad_dim<MN_T, MN_D>(const Geom &, const Pts &, int, const void *, const void *,
                                        void *const[3], hipStream_t);
}  // namespace detail
}  // namespace mn
