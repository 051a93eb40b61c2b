// kernels_n5.hip -- the DGSEM kernels at polynomial degree 5 (templates in kernels.h).
#include "kernels.h"

namespace dg {
template hipError_t launch_n<5, double>(Kernel, int, const View<double> *, const int *, int, int,
                                        const View<double> &, hipStream_t);
template hipError_t launch_n<5, float>(Kernel, int, const View<float> *, const int *, int, int,
                                       const View<float> &, hipStream_t);
}  // namespace dg
