// solver.cpp -- the C ABI of one solve: workspace layout, set-up upload, the
// RK stage driver and the small reductions.  Every step of the time
// derivative runs in the HIP kernels of kernels.hip.
//
// Paper (GALAEXI, arXiv 2404.12703): the time-stepping loop of Sec. 2.2
// ("Time integration": Carpenter-Kennedy five-stage or Niegemann et al.
// fourteen-stage fourth-order 2N-storage schemes) around the DG operator of
// Eq. dgsem; all of it on the device with no host transfers during time
// stepping (Sec. 3, design principles).  The dissipation rates of Sec. 5.2
// come from one volume sweep with per-element sums switched on.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "dg_internal.h"
#include "physics.h"
#include "solver_impl.h"

namespace dg {

thread_local std::string g_last_error;

dg_status fail(dg_status code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

// Carpenter-Kennedy (1994) five-stage fourth-order 2N-storage coefficients
const double RK_A[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                        -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
const double RK_B[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                        1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                        2277821191437.0 / 14882151754819.0};
const double RK_C[5] = {0.0, 1432997174477.0 / 9575080441755.0, 2526269341429.0 / 6820363962896.0,
                        2006345519317.0 / 3224310063776.0, 2802321613138.0 / 2924317926251.0};

// Niegemann, Diehl and Busch (2012): fourteen-stage fourth-order 2N-storage
// scheme with a stability region stretched along the imaginary axis (the
// scheme of the paper's application runs); published coefficients
const double RK14_A[14] = {0.0, -0.7188012108672410, -0.7785331173421570, -0.0053282796654044,
                           -0.8552979934029281, -3.9564138245774565, -1.5780575380587385,
                           -2.0837094552574054, -0.7483334182761610, -0.7032861106563359,
                           0.0013917096117681, -0.0932075369637460, -0.9514200470875948,
                           -7.1151571693922548};
const double RK14_B[14] = {0.0367762454319673, 0.3136296607553959, 0.1531848691869027, 0.0030097086818182,
                           0.3326293790646110, 0.2440251405350864, 0.3718879239592277, 0.6204126221582444,
                           0.1524043173028741, 0.0760894927419266, 0.0077604214040978, 0.0024647284755382,
                           0.0780348340049386, 5.5059777270269628};
const double RK14_C[14] = {0.0, 0.0367762454319673, 0.1249685262725025, 0.2446177702277698,
                           0.2476149531070420, 0.2969311120382472, 0.3978149645802642, 0.5270854589440328,
                           0.6981269994175695, 0.8190890835352128, 0.8527059887098624, 0.8604711817462826,
                           0.8627060376969976, 0.8734213127600976};

int rk_scheme(int scheme, const double **A, const double **B, const double **C) {
  if (scheme == 1) {
    *A = RK14_A;
    *B = RK14_B;
    *C = RK14_C;
    return 14;
  }
  *A = RK_A;
  *B = RK_B;
  *C = RK_C;
  return 5;
}

dg_status check_params(const dg_params *p) {
  if (!p) return fail(DG_EINVAL, "params is NULL");
  if (p->abi_version != DG_ABI_VERSION) return fail(DG_EINVAL, "abi_version mismatch");
  if (p->N < 1 || p->N > N_MAX) return fail(DG_EINVAL, "N must be in 1..9");
  if (p->nodes != 0 && p->nodes != 1) return fail(DG_EINVAL, "nodes must be 0 (Gauss) or 1 (Lobatto)");
  if (p->riemann != 0 && p->riemann != 1) return fail(DG_EINVAL, "riemann must be 0 (LLF) or 1 (Roe)");
  if (p->precision != 0 && p->precision != 1) return fail(DG_EINVAL, "precision must be 0 or 1");
  if (p->shock_capturing && (p->nodes != 1 || p->N < 2 || p->N > 7))
    return fail(DG_EINVAL, "shock capturing needs Gauss-Lobatto nodes and 2 <= N <= 7");
  if (!(p->gamma > 1.0) || !(p->R > 0.0) || !(p->Pr > 0.0) || !(p->mu >= 0.0) || !std::isfinite(p->gamma) ||
      !std::isfinite(p->R) || !std::isfinite(p->Pr) || !std::isfinite(p->mu))
    return fail(DG_EINVAL, "need finite gamma > 1, R > 0, Pr > 0, mu >= 0");
  if (p->shock_capturing &&
      !(p->alpha_max >= 0.0 && p->alpha_max <= 1.0 && p->alpha_min >= 0.0 && p->alpha_min < 0.5 && p->ind_a > 0.0 &&
        std::isfinite(p->ind_a) && std::isfinite(p->ind_c) && p->ind_s > 0.0 && std::isfinite(p->ind_s)))
    return fail(DG_EINVAL, "bad indicator parameters (need 0 <= alpha_min < 0.5, 0 <= alpha_max <= 1, finite a, c and s, "
                           "a > 0, s > 0)");
  if (p->volume_flux != 0 && p->volume_flux != 1) return fail(DG_EINVAL, "volume_flux must be 0 or 1");
  if (p->volume_flux == 1 && p->nodes != 1) return fail(DG_EINVAL, "the split form needs Gauss-Lobatto nodes");
  if (p->viscosity_law != 0 && p->viscosity_law != 1) return fail(DG_EINVAL, "viscosity_law must be 0 or 1");
  if (p->viscosity_law == 1 && !(p->T_ref > 0.0 && std::isfinite(p->T_ref) && p->mu > 0.0))
    return fail(DG_EINVAL, "Sutherland's law needs a finite T_ref > 0 and mu > 0");
  if (p->time_scheme != 0 && p->time_scheme != 1) return fail(DG_EINVAL, "time_scheme must be 0 or 1");
  if (p->alpha_smooth != 0 && p->alpha_smooth != 1) return fail(DG_EINVAL, "alpha_smooth must be 0 or 1");
  if (!std::isfinite(p->p_ref) || p->p_ref < 0.0) return fail(DG_EINVAL, "p_ref must be finite and >= 0");
  if (p->p_ref > 0.0 && p->volume_flux == 1)
    return fail(DG_EINVAL, "p_ref applies to the standard form (the split form's fluxes use the full pressure)");
  return DG_OK;
}

namespace {
size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
}  // namespace

Layout make_layout(const dg_params &p, int64_t E, int part) {
  Layout L;
  const int n = p.N + 1;
  const int64_t n3 = (int64_t)n * n * n, n2 = (int64_t)n * n;
  const size_t rs = p.precision ? sizeof(float) : sizeof(double);
  size_t o = 0;
  const bool st = part != LAYOUT_GEOMETRY, geo = part != LAYOUT_STATE;
  auto take = [&](bool in_part, size_t bytes) {
    if (!in_part) return SIZE_MAX;
    size_t at = o;
    o += align256(bytes);
    return at;
  };
  L.U = take(st, 5 * E * n3 * 8);
  L.dU = take(st, 5 * E * n3 * 8);
  L.Ja = take(geo, 9 * E * n3 * rs);
  L.invJ = take(geo, E * n3 * rs);
  L.NS = take(geo, 3 * E * 6 * n2 * rs);
  L.Utr0 = take(st, 5 * E * 6 * n2 * rs);
  L.Utr1 = take(st, 5 * E * 6 * n2 * rs);
  // the two sweeps exchange each side's viscous face flux (4 values per face
  // node, viscous only) and the volume integral (5 per node)
  L.Hv = take(st && p.viscous, 4 * E * 6 * n2 * rs);
  L.Vol = take(st && (p.viscous || p.shock_capturing || p.volume_flux), 5 * E * n3 * rs);
  // per-element dissipation sums of dg_dissipation (viscous only)
  L.diag = take(st && p.viscous, 3 * E * sizeof(double));
  L.conn = take(geo, 6 * E * sizeof(int2));
  L.Xs = take(geo && p.source, 3 * E * n3 * 8);
  L.basis = take(geo, BasisOffsets(n).total * rs);
  L.alpha = take(st, E * rs);
  L.alpha_raw = take(st, E * rs);
  L.alpha_in = take(st, E * rs);
  // shock capturing: the workgroups left to the blend pass (two counts,
  // used by alternate surface sweeps, and at most one entry per element)
  L.blend = take(st && p.shock_capturing, (2 + E) * sizeof(int));
  L.scratch = take(st, kRedBlocks * 8 * sizeof(double));
  L.total = o;
  return L;
}

template <typename real>
void fill_view(View<real> &v, void *base, const Layout &L, const dg_params &p, int64_t E) {
  char *ws = (char *)base;
  auto at = [&](size_t off) -> char * { return off == SIZE_MAX ? nullptr : ws + off; };
  v.E = E;
  v.U = (double *)at(L.U);
  v.dU = (double *)at(L.dU);
  v.R = nullptr;
  v.Ja = (const real *)at(L.Ja);
  v.invJ = (const real *)at(L.invJ);
  v.NS = (const real *)at(L.NS);
  v.Utr0 = (real *)at(L.Utr0);
  v.Utr1 = (real *)at(L.Utr1);
  v.Hv = (real *)at(L.Hv);
  v.Vol = (real *)at(L.Vol);
  v.conn = (const int2 *)at(L.conn);
  v.Xs = (const double *)at(L.Xs);
  v.basis = (const real *)at(L.basis);
  v.alpha = (real *)at(L.alpha);
  v.alpha_raw = (real *)at(L.alpha_raw);
  v.alpha_in = nullptr;
  v.bcnt = (int *)at(L.blend);
  v.blist = v.bcnt ? v.bcnt + 2 : nullptr;
  v.diag = nullptr;  // [E][3] sums, set for one sweep by dg_dissipation
  v.base = nullptr;
  v.gamma = (real)p.gamma;
  v.Rgas = (real)p.R;
  v.rRgas = (real)(1.0 / p.R);
  v.mu = (real)p.mu;
  v.lambda = (real)(p.gamma * p.R * p.mu / ((p.gamma - 1.0) * p.Pr));
  v.Pr = p.Pr;
  // the mixed form's background pressure (FP64 keeps the state as it is)
  const double pref = sizeof(real) == 4 ? p.p_ref : 0.0;
  v.bg_p = (real)pref;
  v.bg_H = (real)(p.gamma * pref / (p.gamma - 1.0));
  v.e_ref = pref / (p.gamma - 1.0);
  v.rTref = (real)(p.viscosity_law ? 1.0 / p.T_ref : 1.0);
  v.kappa = (real)(p.gamma * p.R / ((p.gamma - 1.0) * p.Pr));
  v.cpR = (real)(p.gamma * p.R / (p.gamma - 1.0));
  v.Rgas4 = real(4) * (real)p.R;
  v.cpR2 = real(2) * v.cpR;
  v.split = p.volume_flux;
  v.visc_law = p.viscosity_law;
  v.alpha_smooth = p.alpha_smooth;
  v.t = 0.0;
  v.dt = 0.0;
  v.rkA = 0.0;
  v.rkB = 0.0;
  v.cur = 0;
  v.viscous = p.viscous;
  v.riemann = p.riemann;
  v.source = p.source;
  v.shock = p.shock_capturing;
  v.lgl = p.nodes == 1;
  {
    const char *env = std::getenv("DG_XCD_REMAP");
    v.remap = env ? std::atoi(env) : 0;
  }
  v.nt = L.total >= kStreamBytes;
  v.ind_a = (real)p.ind_a;
  v.ind_c = (real)p.ind_c;
  v.ind_s = (real)p.ind_s;
  v.alpha_min = (real)p.alpha_min;
  v.alpha_max = (real)p.alpha_max;
  v.ind_T = (real)(p.ind_a * std::pow(10.0, -p.ind_c * std::pow(p.N + 1.0, 0.25)));
}
template void fill_view<double>(View<double> &, void *, const Layout &, const dg_params &, int64_t);
template void fill_view<float>(View<float> &, void *, const Layout &, const dg_params &, int64_t);

// Host set-up of one solve (no HIP calls), then its upload.
dg_status setup_host(const dg_params &p, const dg_mesh &m, HostSetup &hs, std::string &err) {
  Basis b = make_basis(p.N, p.nodes);
  Geometry g;
  dg_status rc = build_geometry(b, m, g, err);
  if (rc) return rc;
  std::vector<double> invJ(g.J.size());
  for (size_t i = 0; i < g.J.size(); ++i) invJ[i] = 1.0 / g.J[i];
  std::vector<double> blk = basis_block(b);
  if (p.precision == 1) {
    auto to_f = [](const std::vector<double> &x) {
      std::vector<float> f(x.size());
      for (size_t i = 0; i < x.size(); ++i) f[i] = (float)x[i];
      return f;
    };
    hs.fJa = to_f(g.Ja);
    hs.finvJ = to_f(invJ);
    hs.fNS = to_f(g.NS);
    hs.fbasis = to_f(blk);
  } else {
    hs.Ja = std::move(g.Ja);
    hs.invJ = std::move(invJ);
    hs.NS = std::move(g.NS);
    hs.basis = std::move(blk);
  }
  hs.conn = std::move(g.conn);
  if (p.source) hs.Xs = std::move(g.Xs);
  return DG_OK;
}

double host_stable_dt(const dg_params &p, int64_t E, const HostSetup &hs, const double *U0, double cfl) {
  // the time-step estimate of dg_stable_dt (App. A.5): convective
  // 2/((2N+1) sum_i lambda_i) and, with viscosity, 4/((N+1)^4 nu sum_i (|Ja^i|/J)^2)
  const int n = p.N + 1, n3 = n * n * n;
  const bool mixed = p.precision == 1;
  auto ja = [&](size_t i) { return mixed ? (double)hs.fJa[i] : hs.Ja[i]; };
  auto ij = [&](size_t i) { return mixed ? (double)hs.finvJ[i] : hs.invJ[i]; };
  const double gam = p.gamma, nfac = std::pow((double)n, 4.0);
  double dta = 1e300, dtv = 1e300;
  for (int64_t e = 0; e < E; ++e)
    for (int a = 0; a < n3; ++a) {
      double U[5];
      for (int c = 0; c < 5; ++c) U[c] = U0[((size_t)c * E + e) * n3 + a];
      const double rho = U[0], ir = 1.0 / rho, u = U[1] * ir, v = U[2] * ir, w = U[3] * ir;
      const double pr = (gam - 1.0) * (U[4] - 0.5 * rho * (u * u + v * v + w * w));
      const double c = std::sqrt(gam * pr / rho), iJ = ij((size_t)e * n3 + a);
      double lamsum = 0.0, vis = 0.0;
      for (int ci = 0; ci < 3; ++ci) {
        const double j0 = ja(((size_t)(3 * ci) * E + e) * n3 + a), j1 = ja(((size_t)(3 * ci + 1) * E + e) * n3 + a),
                     j2 = ja(((size_t)(3 * ci + 2) * E + e) * n3 + a);
        const double nj = std::sqrt(j0 * j0 + j1 * j1 + j2 * j2);
        lamsum += (std::fabs(u * j0 + v * j1 + w * j2) + c * nj) * iJ;
        vis += (nj * iJ) * (nj * iJ);
      }
      dta = std::min(dta, 2.0 / ((2.0 * p.N + 1.0) * lamsum));
      if (p.viscous && p.mu > 0) {
        // with Sutherland's law the viscosity at this node's temperature, as on the device
        const double mu = p.viscosity_law ? sutherland<double>(pr / (rho * p.R), p.mu, 1.0 / p.T_ref) : p.mu;
        const double nu = std::max(4.0 / 3.0, gam / p.Pr) * mu / rho;
        dtv = std::min(dtv, 4.0 / (nfac * nu * vis));
      }
    }
  return std::min(cfl * dta, cfl * dtv);
}

hipError_t upload_geometry(const dg_params &p, const HostSetup &hs, void *base, const Layout &L, hipStream_t st) {
  char *ws = (char *)base;
  const bool mixed = p.precision == 1;
  auto put = [&](size_t off, const std::vector<double> &d, const std::vector<float> &f) -> hipError_t {
    return mixed ? hipMemcpyAsync(ws + off, f.data(), f.size() * 4, hipMemcpyHostToDevice, st)
                 : hipMemcpyAsync(ws + off, d.data(), d.size() * 8, hipMemcpyHostToDevice, st);
  };
  hipError_t e = put(L.Ja, hs.Ja, hs.fJa);
  if (e == hipSuccess) e = put(L.invJ, hs.invJ, hs.finvJ);
  if (e == hipSuccess) e = put(L.NS, hs.NS, hs.fNS);
  if (e == hipSuccess) e = put(L.basis, hs.basis, hs.fbasis);
  if (e == hipSuccess) e = hipMemcpyAsync(ws + L.conn, hs.conn.data(), hs.conn.size() * sizeof(int2), hipMemcpyHostToDevice, st);
  if (e == hipSuccess && p.source) e = hipMemcpyAsync(ws + L.Xs, hs.Xs.data(), hs.Xs.size() * 8, hipMemcpyHostToDevice, st);
  return e;
}

template <typename real>
void attach_geometry(View<real> &v, void *base, const Layout &L) {
  char *g = (char *)base;
  v.Ja = (const real *)(g + L.Ja);
  v.invJ = (const real *)(g + L.invJ);
  v.NS = (const real *)(g + L.NS);
  v.conn = (const int2 *)(g + L.conn);
  v.Xs = L.Xs == SIZE_MAX ? nullptr : (const double *)(g + L.Xs);
  v.basis = (const real *)(g + L.basis);
}
template void attach_geometry<double>(View<double> &, void *, const Layout &);
template void attach_geometry<float>(View<float> &, void *, const Layout &);

hipError_t setup_device(const dg_params &p, const HostSetup &hs, void *base, const Layout &L, hipStream_t st) {
  hipError_t e = hipMemsetAsync(base, 0, L.total, st);
  if (e == hipSuccess) e = upload_geometry(p, hs, base, L, st);
  return e;
}

// upload a host FP64 array into device memory of the solve's arithmetic type
static hipError_t upload_real(dg_solver *s, size_t off, const std::vector<double> &h) {
  char *dst = (char *)s->ws + off;
  if (!s->mixed) return hipMemcpyAsync(dst, h.data(), h.size() * 8, hipMemcpyHostToDevice, s->st);
  std::vector<float> f(h.size());
  for (size_t i = 0; i < h.size(); ++i) f[i] = (float)h[i];
  hipError_t e = hipMemcpyAsync(dst, f.data(), f.size() * 4, hipMemcpyHostToDevice, s->st);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);  // f goes out of scope
  return e;
}

dg_status device_error(dg_solver *s, hipError_t e, const char *what) {
  if (s) s->broken = true;
  return fail(DG_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// enqueue one kernel for this solve (records profiling events when enabled)
template <typename real>
static hipError_t run_kernel(dg_solver *s, Kernel k, int mode, const View<real> &v) {
  int blocks = blocks_per_elements(s->p.N, s->E);
  if (s->prof_on) {
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    (void)hipEventRecord(a, s->st);
    hipError_t e = launch<real>(k, s->p.N, mode, nullptr, nullptr, 0, blocks, v, s->st);
    (void)hipEventRecord(b, s->st);
    s->prof_events.push_back({(int)k, a, b});
    return e;
  }
  return launch<real>(k, s->p.N, mode, nullptr, nullptr, 0, blocks, v, s->st);
}

template <typename real>
static View<real> &view_of(dg_solver *s);
template <>
View<double> &view_of<double>(dg_solver *s) {
  return s->vd;
}
template <>
View<float> &view_of<float>(dg_solver *s) {
  return s->vf;
}

// one evaluation of the operator: traces (if stale), lifting, time derivative.
// mode 0: stage update with (t, dt, A, B); mode 1: write R to Rout.
template <typename real>
static hipError_t stage(dg_solver *s, int mode, double t, double dt, double A, double B, double *Rout) {
  View<real> &v = view_of<real>(s);
  v.t = t;
  v.dt = dt;
  v.rkA = A;
  v.rkB = B;
  v.cur = s->cur;
  v.bpar = s->bpar;
  v.R = Rout;
  hipError_t e = hipSuccess;
  if (!s->traces_valid) {
    e = run_kernel<real>(s, K_TRACE, 0, v);
    if (e != hipSuccess) return e;
    s->traces_valid = true;
  }
  if (s->p.viscous || s->p.shock_capturing || s->p.volume_flux) {  // lifting, indicator, split form
    e = run_kernel<real>(s, K_LIFT, 0, v);
    if (e != hipSuccess) return e;
  }
  e = run_kernel<real>(s, K_RHS, mode, v);
  if (e != hipSuccess) return e;
  s->bpar ^= 1;
  if (mode == 0) s->cur ^= 1;
  return hipSuccess;
}

template <typename real>
static hipError_t advance_impl(dg_solver *s, int nsteps, double dt) {
  const double *A, *B, *C;
  const int ns = rk_scheme(s->p.time_scheme, &A, &B, &C);
  for (int st = 0; st < nsteps; ++st) {
    const double t0 = s->t;
    for (int k = 0; k < ns; ++k) {
      hipError_t e = stage<real>(s, 0, t0 + C[k] * dt, dt, A[k], B[k], nullptr);
      if (e != hipSuccess) return e;
    }
    s->t = t0 + dt;
  }
  return hipSuccess;
}

hipError_t solver_advance(dg_solver *s, int nsteps, double dt) {
  return s->mixed ? advance_impl<float>(s, nsteps, dt) : advance_impl<double>(s, nsteps, dt);
}

// One volume sweep of the current state with the dissipation sums on (stage
// temporaries only: the volume integral and the viscous face fluxes), the
// per-element sums into diag[E][3], their fixed-order total into sums[3],
// and the two rates of Sec. 5.2 on the host.
hipError_t dissipation_sweep(dg_solver *s, double *diag, double *sums, double out[2]) {
  hipError_t e = hipSuccess;
  auto sweep = [&](auto &v) {
    using real = typename std::remove_reference<decltype(v)>::type::value_type;
    v.t = s->t;
    v.cur = s->cur;
    v.bpar = s->bpar;
    v.R = nullptr;
    if (!s->traces_valid) {
      e = run_kernel<real>(s, K_TRACE, 0, v);
      if (e != hipSuccess) return;
      s->traces_valid = true;
    }
    v.diag = diag;
    e = run_kernel<real>(s, K_DIAG, 0, v);
    v.diag = nullptr;
  };
  if (s->mixed) sweep(s->vf);
  else sweep(s->vd);
  double h[3] = {0.0, 0.0, 0.0};
  if (e == hipSuccess) e = launch_sum3(diag, s->E, sums, s->st);
  if (e == hipSuccess) e = hipMemcpyAsync(h, sums, sizeof h, hipMemcpyDeviceToHost, s->st);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  if (e != hipSuccess) return e;
  out[0] = h[0] / h[2];
  out[1] = 4.0 / 3.0 * h[1] / h[2];
  return hipSuccess;
}

// The allocation-free dissipation entry point's device memory: a file-scope
// array on every GPU the library runs on, held until the process ends.  Host
// code never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol): it takes the array's device address from
// hipGetSymbolAddress, once per device with that device current, and uses
// that address everywhere.  Calls that overlap on one GPU share the array and
// race.
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[3 * kStaticElems + 8];
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kMaxDevices] = {};

hipError_t static_scratch(int dev, double **ptr) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = (double *)p;
  }
  *ptr = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace dg

using namespace dg;

extern "C" {

int32_t dg_abi_version(void) { return DG_ABI_VERSION; }

const char *dg_last_error(void) { return g_last_error.c_str(); }

dg_status dg_workspace_bytes(const dg_params *p, int64_t n_elems, size_t *bytes) {
  dg_status rc = check_params(p);
  if (rc) return rc;
  if (!elems_in_range(p->N, n_elems)) return fail(DG_EINVAL, "n_elems out of range");
  if (!bytes) return fail(DG_EINVAL, "bytes is NULL");
  *bytes = make_layout(*p, n_elems).total;
  return DG_OK;
}

dg_status dg_create(const dg_params *p, const dg_mesh *m, void *d_workspace, size_t ws_bytes, void *hip_stream,
                    dg_solver **out) {
  g_last_error.clear();
  if (!out) return fail(DG_EINVAL, "out is NULL");
  *out = nullptr;
  dg_status rc = check_params(p);
  if (rc) return rc;
  if (!m || !m->x_geo || !m->nbr_elem || !m->nbr_face || !m->nbr_orient) return fail(DG_EINVAL, "mesh arrays missing");
  if (!elems_in_range(p->N, m->n_elems)) return fail(DG_EINVAL, "n_elems out of range");
  if (m->n_geo < 1 || m->n_geo > p->N) return fail(DG_EINVAL, "n_geo must be in 1..N");
  if (!d_workspace) return fail(DG_EINVAL, "workspace is NULL");
  if ((uintptr_t)d_workspace % 256) return fail(DG_EINVAL, "workspace must be 256-byte aligned");
  Layout L = make_layout(*p, m->n_elems);
  if (ws_bytes < L.total)
    return fail(DG_ENOMEM, "workspace too small: need " + std::to_string(L.total) + " bytes");

  std::unique_ptr<dg_solver> s(new (std::nothrow) dg_solver());
  if (!s) return fail(DG_ENOMEM, "host allocation failed");
  s->p = *p;
  s->E = m->n_elems;
  s->ws = d_workspace;
  s->ws_bytes = ws_bytes;
  s->L = L;
  s->st = (hipStream_t)hip_stream;
  s->mixed = p->precision == 1;

  fill_view(s->vd, s->ws, L, *p, s->E);
  fill_view(s->vf, s->ws, L, *p, s->E);
  HostSetup hs;
  std::string err;
  rc = setup_host(*p, *m, hs, err);
  if (rc) return fail(rc, err);
  hipError_t e = setup_device(*p, hs, s->ws, L, s->st);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);  // the host buffers go out of scope
  if (e != hipSuccess) return device_error(nullptr, e, "dg_create upload");
  s->t = 0.0;
  s->cur = 0;
  s->traces_valid = false;
  *out = s.release();
  return DG_OK;
}

void dg_destroy(dg_solver *s) {
  if (!s) return;
  for (auto &pe : s->prof_events) {
    (void)hipEventDestroy(pe.a);
    (void)hipEventDestroy(pe.b);
  }
  delete s;
}

#define CHECK_SOLVER(s)                                                         \
  do {                                                                          \
    if (!(s)) return fail(DG_EINVAL, "solver is NULL");                         \
    if ((s)->broken) return fail(DG_ESTATE, "solver unusable after a device error"); \
  } while (0)

dg_status dg_set_state(dg_solver *s, const double *U, int32_t on_device, double t) {
  CHECK_SOLVER(s);
  if (!U) return fail(DG_EINVAL, "U is NULL");
  if (!std::isfinite(t)) return fail(DG_EINVAL, "t must be finite");
  size_t bytes = (size_t)5 * s->E * (s->p.N + 1) * (s->p.N + 1) * (s->p.N + 1) * 8;
  hipError_t e = hipMemcpyAsync((char *)s->ws + s->L.U, U, bytes,
                                on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s->st);
  if (e == hipSuccess && !on_device) e = hipStreamSynchronize(s->st);
  if (e != hipSuccess) return device_error(s, e, "dg_set_state");
  s->t = t;
  s->traces_valid = false;
  return DG_OK;
}

dg_status dg_get_state(dg_solver *s, double *U, int32_t on_device, double *t) {
  CHECK_SOLVER(s);
  if (!U) return fail(DG_EINVAL, "U is NULL");
  size_t bytes = (size_t)5 * s->E * (s->p.N + 1) * (s->p.N + 1) * (s->p.N + 1) * 8;
  hipError_t e = hipMemcpyAsync(U, (char *)s->ws + s->L.U, bytes,
                                on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s->st);
  if (e == hipSuccess && !on_device) e = hipStreamSynchronize(s->st);
  if (e != hipSuccess) return device_error(s, e, "dg_get_state");
  if (t) *t = s->t;
  return DG_OK;
}

dg_status dg_advance(dg_solver *s, int32_t n_steps, double dt) {
  CHECK_SOLVER(s);
  if (n_steps < 0 || !(dt > 0.0) || !std::isfinite(dt)) return fail(DG_EINVAL, "need n_steps >= 0 and dt > 0");
  if (!s->p.check_finite) {
    hipError_t e = solver_advance(s, n_steps, dt);
    if (e != hipSuccess) return device_error(s, e, "dg_advance");
    return DG_OK;
  }
  // checked stepping: one step, a finiteness flag on the device, its read-back
  int *flag = (int *)((char *)s->ws + s->L.scratch);
  const size_t count = (size_t)5 * s->E * (s->p.N + 1) * (s->p.N + 1) * (s->p.N + 1);
  for (int st = 0; st < n_steps; ++st) {
    hipError_t e = solver_advance(s, 1, dt);
    if (e == hipSuccess) e = launch_zero_int(flag, 1, s->st);
    if (e == hipSuccess) e = launch_finite((const double *)((char *)s->ws + s->L.U), (int64_t)count, flag, s->st);
    int h = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s->st);
    if (e == hipSuccess) e = hipStreamSynchronize(s->st);
    if (e != hipSuccess) return device_error(s, e, "dg_advance finiteness check");
    if (h)
      return fail(DG_ENONFINITE, "state not finite after step " + std::to_string(st + 1) + " of " +
                                     std::to_string(n_steps) + " (t = " + std::to_string(s->t) + ")");
  }
  return DG_OK;
}

dg_status dg_rhs(dg_solver *s, double t, double *Ut, int32_t on_device) {
  CHECK_SOLVER(s);
  if (!Ut) return fail(DG_EINVAL, "Ut is NULL");
  if (!std::isfinite(t)) return fail(DG_EINVAL, "t must be finite");
  // a host destination is staged through the RK register, which carries no
  // information between steps (A_1 = 0 restarts it)
  double *dst = on_device ? Ut : (double *)((char *)s->ws + s->L.dU);
  hipError_t e = s->mixed ? stage<float>(s, 1, t, 0.0, 0.0, 0.0, dst) : stage<double>(s, 1, t, 0.0, 0.0, 0.0, dst);
  if (e == hipSuccess && !on_device) {
    size_t bytes = (size_t)5 * s->E * (s->p.N + 1) * (s->p.N + 1) * (s->p.N + 1) * 8;
    e = hipMemcpyAsync(Ut, dst, bytes, hipMemcpyDeviceToHost, s->st);
    if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  }
  if (e != hipSuccess) return device_error(s, e, "dg_rhs");
  return DG_OK;
}

dg_status dg_stable_dt(dg_solver *s, double cfl, double dfl, double *dt) {
  CHECK_SOLVER(s);
  if (!dt || !(cfl > 0) || !(dfl > 0) || !std::isfinite(cfl) || !std::isfinite(dfl))
    return fail(DG_EINVAL, "need dt and finite cfl, dfl > 0");
  double *scr = (double *)((char *)s->ws + s->L.scratch);
  hipError_t e = s->mixed ? launch_dt<float>(s->p.N, s->vf, scr, kRedBlocks, s->st)
                          : launch_dt<double>(s->p.N, s->vd, scr, kRedBlocks, s->st);
  std::vector<double> h(2 * kRedBlocks);
  if (e == hipSuccess) e = hipMemcpyAsync(h.data(), scr, h.size() * 8, hipMemcpyDeviceToHost, s->st);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  if (e != hipSuccess) return device_error(s, e, "dg_stable_dt");
  double a = 1e300, v = 1e300;
  for (int b = 0; b < kRedBlocks; ++b) {
    a = std::min(a, h[2 * b]);
    v = std::min(v, h[2 * b + 1]);
  }
  if (!(a < 1e299)) return fail(DG_ENONFINITE, "no finite time step (state not finite?)");
  *dt = std::min(cfl * a, dfl * v);
  return DG_OK;
}

dg_status dg_integrals(dg_solver *s, double out[7]) {
  CHECK_SOLVER(s);
  if (!out) return fail(DG_EINVAL, "out is NULL");
  double *scr = (double *)((char *)s->ws + s->L.scratch);
  hipError_t e = s->mixed ? launch_integrals<float>(s->p.N, s->vf, scr, kRedBlocks, s->st)
                          : launch_integrals<double>(s->p.N, s->vd, scr, kRedBlocks, s->st);
  std::vector<double> h(7 * kRedBlocks);
  if (e == hipSuccess) e = hipMemcpyAsync(h.data(), scr, h.size() * 8, hipMemcpyDeviceToHost, s->st);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  if (e != hipSuccess) return device_error(s, e, "dg_integrals");
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int b = 0; b < kRedBlocks; ++b)
    for (int c = 0; c < 7; ++c) acc[c] += h[7 * b + c];
  for (int c = 0; c < 5; ++c) out[c] = acc[c];
  out[5] = acc[5] / acc[6];
  out[6] = acc[6];
  return DG_OK;
}

dg_status dg_dissipation(dg_solver *s, double out[2]) {
  CHECK_SOLVER(s);
  if (!out) return fail(DG_EINVAL, "out is NULL");
  if (!s->p.viscous) return fail(DG_EINVAL, "the dissipation rates need the viscous operator");
  double *d = (double *)((char *)s->ws + s->L.diag);
  double *sums = (double *)((char *)s->ws + s->L.scratch);
  hipError_t e = dissipation_sweep(s, d, sums, out);
  if (e != hipSuccess) return device_error(s, e, "dg_dissipation");
  return DG_OK;
}

dg_status dg_dissipation_noalloc(dg_solver *s, double out[2]) {
  CHECK_SOLVER(s);
  if (!out) return fail(DG_EINVAL, "out is NULL");
  if (!s->p.viscous) return fail(DG_EINVAL, "the dissipation rates need the viscous operator");
  if (s->E > kStaticElems)
    return fail(DG_EINVAL, "dg_dissipation_noalloc takes at most " + std::to_string(kStaticElems) +
                               " elements (its static device array); this solve has " + std::to_string(s->E));
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_error(nullptr, e, "dg_dissipation_noalloc");
  hipPointerAttribute_t at;
  e = hipPointerGetAttributes(&at, s->ws);
  if (e != hipSuccess) return device_error(nullptr, e, "dg_dissipation_noalloc workspace attributes");
  if (at.device != dev)
    return fail(DG_EINVAL, "dg_dissipation_noalloc: the solver's workspace is on device " + std::to_string(at.device) +
                               ", the current device is " + std::to_string(dev));
  double *base = nullptr;
  e = static_scratch(dev, &base);
  if (e != hipSuccess) return device_error(nullptr, e, "dg_dissipation_noalloc scratch address");
  e = dissipation_sweep(s, base, base + 3 * kStaticElems, out);
  if (e != hipSuccess) return device_error(s, e, "dg_dissipation_noalloc");
  return DG_OK;
}

dg_status dg_alpha(dg_solver *s, double *alpha_host) {
  CHECK_SOLVER(s);
  if (!alpha_host) return fail(DG_EINVAL, "alpha is NULL");
  const size_t E = s->E;
  hipError_t e;
  if (s->mixed) {
    std::vector<float> f(E);
    e = hipMemcpyAsync(f.data(), (char *)s->ws + s->L.alpha, E * 4, hipMemcpyDeviceToHost, s->st);
    if (e == hipSuccess) e = hipStreamSynchronize(s->st);
    for (size_t i = 0; i < E; ++i) alpha_host[i] = f[i];
  } else {
    e = hipMemcpyAsync(alpha_host, (char *)s->ws + s->L.alpha, E * 8, hipMemcpyDeviceToHost, s->st);
    if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  }
  if (e != hipSuccess) return device_error(s, e, "dg_alpha");
  return DG_OK;
}

dg_status dg_set_alpha(dg_solver *s, const double *alpha_host) {
  CHECK_SOLVER(s);
  if (!alpha_host) {
    s->vd.alpha_in = nullptr;
    s->vf.alpha_in = nullptr;
    return DG_OK;
  }
  std::vector<double> a(alpha_host, alpha_host + s->E);
  for (double x : a)
    if (!(x >= 0.0 && x <= 1.0)) return fail(DG_EINVAL, "alpha must lie in [0, 1]");
  hipError_t e = upload_real(s, s->L.alpha_in, a);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  if (e != hipSuccess) return device_error(s, e, "dg_set_alpha");
  s->vd.alpha_in = (const double *)((char *)s->ws + s->L.alpha_in);
  s->vf.alpha_in = (const float *)((char *)s->ws + s->L.alpha_in);
  return DG_OK;
}

dg_status dg_synchronize(dg_solver *s) {
  CHECK_SOLVER(s);
  hipError_t e = hipStreamSynchronize(s->st);
  if (e != hipSuccess) return device_error(s, e, "dg_synchronize");
  return DG_OK;
}

dg_status dg_profile_enable(dg_solver *s, int32_t on) {
  CHECK_SOLVER(s);
  s->prof_on = on != 0;
  for (auto &pe : s->prof_events) {
    (void)hipEventDestroy(pe.a);
    (void)hipEventDestroy(pe.b);
  }
  s->prof_events.clear();
  return DG_OK;
}

dg_status dg_profile_read(dg_solver *s, int32_t n, double *ms, int64_t *launches) {
  CHECK_SOLVER(s);
  if (n < 0 || (n > 0 && (!ms || !launches))) return fail(DG_EINVAL, "bad arguments");
  hipError_t e = hipStreamSynchronize(s->st);
  if (e != hipSuccess) return device_error(s, e, "dg_profile_read");
  for (int k = 0; k < n; ++k) {
    ms[k] = 0.0;
    launches[k] = 0;
  }
  for (auto &pe : s->prof_events) {
    float t = 0.f;
    (void)hipEventElapsedTime(&t, pe.a, pe.b);
    if (pe.kernel < n) {
      ms[pe.kernel] += t;
      launches[pe.kernel] += 1;
    }
    (void)hipEventDestroy(pe.a);
    (void)hipEventDestroy(pe.b);
  }
  s->prof_events.clear();
  return DG_OK;
}

}  // extern "C"
