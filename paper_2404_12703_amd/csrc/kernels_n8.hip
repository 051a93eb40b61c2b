// kernels_n8.hip -- the DGSEM kernels at polynomial degree 8 (templates in kernels.h).
#include "kernels.h"

namespace dg {
template hipError_t launch_n<8, double>(Kernel, int, const View<double> *, const int *, int, int,
                                        const View<double> &, hipStream_t);
template hipError_t launch_n<8, float>(Kernel, int, const View<float> *, const int *, int, int,
                                       const View<float> &, hipStream_t);
}  // namespace dg
