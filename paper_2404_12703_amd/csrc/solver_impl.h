// solver_impl.h -- the solver object behind the opaque dg_solver handle.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "dg_internal.h"

namespace dg {

constexpr int kRedBlocks = 1024;  // blocks of the reduction kernels

// byte offsets of every array inside the caller's workspace (SIZE_MAX: absent)
struct Layout {
  size_t U, dU, Ja, invJ, NS, Utr0, Utr1, Hv, Vol, conn, Xs, basis, alpha, alpha_raw, alpha_in, scratch, total;
};

Layout make_layout(const dg_params &p, int64_t E);
dg_status check_params(const dg_params *p);
// kernels index one row of a volume or face array with 32-bit lane offsets
inline bool elems_in_range(int N, int64_t E) {
  const int64_t n = N + 1;
  return E >= 1 && E * n * n * n < INT32_MAX && E * 6 * n * n < INT32_MAX;
}
dg_status fail(dg_status code, const std::string &msg);

extern const double RK_A[5], RK_B[5], RK_C[5];

// host staging buffers of a set-up upload
struct Staging {
  std::vector<std::vector<double>> d;
  std::vector<std::vector<float>> f;
  std::vector<int2> c;
};

template <typename real>
void fill_view(View<real> &v, void *base, const Layout &L, const dg_params &p, int64_t E);
dg_status setup_upload(const dg_params &p, const dg_mesh &m, void *base, const Layout &L, hipStream_t st,
                       Staging &stg);
dg_status device_error(dg_solver *s, hipError_t e, const char *what);

struct ProfEvent {
  int kernel;
  hipEvent_t a, b;
};

}  // namespace dg

struct dg_solver {
  dg_params p{};
  int64_t E = 0;
  void *ws = nullptr;
  size_t ws_bytes = 0;
  dg::Layout L{};
  hipStream_t st = nullptr;
  bool mixed = false;
  bool broken = false;
  dg::View<double> vd{};
  dg::View<float> vf{};
  double t = 0.0;
  int cur = 0;
  bool traces_valid = false;
  bool prof_on = false;
  std::vector<dg::ProfEvent> prof_events;
};
