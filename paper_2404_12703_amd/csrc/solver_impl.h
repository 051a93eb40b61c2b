// solver_impl.h -- the solver object behind the opaque dg_solver handle.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "dg_internal.h"

namespace dg {

constexpr int kRedBlocks = 1024;  // blocks of the reduction kernels
// elements the allocation-free dissipation call takes (its static device
// array holds 3 doubles per element: 6 MiB)
constexpr int64_t kStaticElems = int64_t(1) << 18;

// byte offsets of every array inside the caller's workspace (SIZE_MAX: absent)
struct Layout {
  size_t U, dU, Ja, invJ, NS, Utr0, Utr1, Hv, Vol, diag, conn, Xs, basis, alpha, alpha_raw, alpha_in, blend, scratch,
      total;
};

// part 0: every array of one solve; 1: the per-solve state and temporaries
// only; 2: the read-only geometry only (metrics, normals, connectivity, node
// positions, operator block), which solves of one mesh can share.  Arrays of
// the other part are SIZE_MAX.
enum LayoutPart { LAYOUT_ALL = 0, LAYOUT_STATE = 1, LAYOUT_GEOMETRY = 2 };
Layout make_layout(const dg_params &p, int64_t E, int part = LAYOUT_ALL);
dg_status check_params(const dg_params *p);
// kernels index one row of a volume or face array with 32-bit lane offsets
inline bool elems_in_range(int N, int64_t E) {
  const int64_t n = N + 1;
  return E >= 1 && E * n * n * n < INT32_MAX && E * 6 * n * n < INT32_MAX;
}
dg_status fail(dg_status code, const std::string &msg);

extern const double RK_A[5], RK_B[5], RK_C[5];

// Host half of a solve's set-up: bases, geometry and metrics in the solve's
// arithmetic type, ready to upload.  Makes no HIP call, so it may run on any
// thread.
struct HostSetup {
  std::vector<double> Ja, invJ, NS, basis, Xs;  // FP64 form
  std::vector<float> fJa, finvJ, fNS, fbasis;   // mixed form
  std::vector<int2> conn;
  size_t bytes() const {
    return 8 * (Ja.size() + invJ.size() + NS.size() + basis.size() + Xs.size()) +
           4 * (fJa.size() + finvJ.size() + fNS.size() + fbasis.size()) + sizeof(int2) * conn.size();
  }
};

template <typename real>
void fill_view(View<real> &v, void *base, const Layout &L, const dg_params &p, int64_t E);
// DG_EMESH with err on a mesh that fails the geometric checks
dg_status setup_host(const dg_params &p, const dg_mesh &m, HostSetup &hs, std::string &err);
// the step of dg_stable_dt with CFL = DFL = cfl on the state U0 [5][E][n3],
// in FP64 from the set-up's metrics (in the solve's arithmetic type, as on
// the device)
double host_stable_dt(const dg_params &p, int64_t E, const HostSetup &hs, const double *U0, double cfl);
// zero the workspace and copy the set-up in on st (L from LAYOUT_ALL); hs must
// stay alive until the copies have completed
hipError_t setup_device(const dg_params &p, const HostSetup &hs, void *base, const Layout &L, hipStream_t st);
// the geometry part alone (L from LAYOUT_GEOMETRY): uploads only, no clearing
hipError_t upload_geometry(const dg_params &p, const HostSetup &hs, void *base, const Layout &L, hipStream_t st);
// point a view's geometry arrays at a geometry block (L from LAYOUT_GEOMETRY)
template <typename real>
void attach_geometry(View<real> &v, void *base, const Layout &L);
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
  int bpar = 0;  // alternates over surface sweeps (blend-pass list counts)
  bool traces_valid = false;
  bool prof_on = false;
  std::vector<dg::ProfEvent> prof_events;
};
