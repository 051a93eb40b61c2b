// kernels_n6.hip -- the DGSEM kernels at polynomial degree 6 (templates in kernels.h).
#include "kernels.h"

namespace dg {
template hipError_t launch_n<6, double>(Kernel, int, const View<double> *, const int *, int, int,
                                        const View<double> &, hipStream_t);
template hipError_t launch_n<6, float>(Kernel, int, const View<float> *, const int *, int, int,
                                       const View<float> &, hipStream_t);
}  // namespace dg
