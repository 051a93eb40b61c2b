// kernels_n2.hip -- the DGSEM kernels at polynomial degree 2 (templates in kernels.h).
#include "kernels.h"

namespace dg {
template hipError_t launch_n<2, double>(Kernel, int, const View<double> *, const int *, int, int,
                                        const View<double> &, hipStream_t);
template hipError_t launch_n<2, float>(Kernel, int, const View<float> *, const int *, int, int,
                                       const View<float> &, hipStream_t);
}  // namespace dg
