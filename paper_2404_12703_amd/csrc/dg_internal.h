// dg_internal.h -- internal types shared by the host setup, the stage driver,
// the server and the HIP kernels of the DGSEM library.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dgsem.h"

namespace dg {

constexpr int NV = 5;   // conservative variables
constexpr int NLIFT = 4; // lifted primitives u, v, w, T
constexpr int NG = 12;  // lifted gradient components: 3 directions x 4 variables
constexpr int N_MAX = 9;
constexpr int MAX_STAGES = 14;  // low-storage RK stages of the longest scheme

// Device view of one solve: every pointer and scalar a kernel needs for one
// RK stage.  `real` is the arithmetic type of the time derivative (double
// for FP64, float for the mixed form); state and RK register stay double.
template <typename real>
struct View {
  using value_type = real;
  int64_t E;        // elements
  double *U;        // [5][E][n3]
  double *dU;       // [5][E][n3]   low-storage RK register
  double *R;        // [5][E][n3]   output of the time derivative (rhs mode), else null
  const real *Ja;   // [9][E][n3]   Ja[3*i + d]: computational direction i, Cartesian d
  const real *invJ; // [E][n3]
  const real *NS;   // [3][E*6][n2] outward n*shat of the face flux at this node
  real *Utr0;       // [5][E*6][n2] conservative traces, ping
  real *Utr1;       // [5][E*6][n2] conservative traces, pong
  real *Hv;         // [4][E*6][n2] own-side viscous normal flux F_v(prim, g).n of the face flux (momentum, energy)
  real *Vol;        // [5][E][n3]  volume integral sum_i D-hat (Ja^i . (F_adv - F_v))
  const int2 *conn; // [E][6]: x = 6*nbr_elem + nbr_face, y = orient | primary << 3
  const double *Xs; // [3][E][n3] node positions (manufactured source only)
  const real *basis; // operator block, see BasisOffsets
  real *alpha;      // [E] blending factors
  real *alpha_raw;  // [E] indicator values of the elements (before the optional smoothing)
  const real *alpha_in; // [E] frozen blending factors or null
  int *bcnt;        // shock capturing: [2] entries of blist, used by alternate surface sweeps
  int *blist;       // shock capturing: [E] workgroups with a blended element, this sweep
  double *diag;     // [E][3] per-element sums of the volume sweep: w J mu |curl u|^2, w J mu (div u)^2, w J; or null
  char *base;       // batched launches, in the argument view: the arena that the
                    // descriptors' pointer fields are byte offsets into
  real gamma, Rgas, rRgas, mu, lambda; // perfect gas (rRgas = 1/R); mu, lambda at T_ref under Sutherland's law
  real bg_p, bg_H;  // mixed form: background pressure p_ref and gamma p_ref/(gamma-1) (zero in FP64)
  double e_ref;     // mixed form: p_ref/(gamma-1), taken off the energy where the FP64 state becomes FP32
  real rTref;       // 1/T_ref (Sutherland)
  real kappa;       // lambda/mu = gamma R/((gamma - 1) Pr)
  real cpR;         // gamma R/(gamma - 1): specific total enthalpy H = cpR T + |u|^2/2
  real Rgas4, cpR2; // 4 R and 2 cpR (the split form's two-point sums)
  double Pr;        // Prandtl number (time-step estimate only)
  double t, dt, rkA, rkB;       // stage time, step, LSERK coefficients
  int cur;          // trace buffer read this stage (0: Utr0, 1: Utr1)
  int bpar;         // entry of bcnt this surface sweep counts in; it clears the other
  int viscous, riemann, source, shock;
  int split;        // split-form volume integral with Pirozzoli's two-point flux (Gauss-Lobatto)
  int visc_law;     // 0 constant viscosity, 1 Sutherland's law
  int alpha_smooth; // 1: raise alpha to half the largest face neighbour's indicator value
  int lgl;          // Gauss-Lobatto nodes: l(-1), l(+1) are unit vectors, l-hat vanishes off the end nodes
  int remap;        // XCD-contiguous block order (single solve)
  int nt;           // streaming (non-temporal) loads and stores in the two sweeps: set when the
                    // working set exceeds what the on-die caches could keep (kStreamBytes)
  real ind_a, ind_c, ind_s, alpha_min, alpha_max, ind_T; // indicator (ind_T precomputed threshold)
};

// workspace bytes above which the sweeps stream their single-use data past the
// caches: MI355X's 256 MB Infinity Cache keeps smaller working sets between
// sweeps, and plain accesses serve those better
constexpr size_t kStreamBytes = size_t(384) << 20;

// offsets (in elements of `real`) inside the basis block, for n = N+1
struct BasisOffsets {
  int Dhat, D, Vinv, lm, lp, lhm, lhp, w, x, xhalf, total;
  __host__ __device__ explicit BasisOffsets(int n) {
    int o = 0;
    Dhat = o; o += n * n;
    D = o; o += n * n;
    Vinv = o; o += n * n;
    lm = o; o += n;
    lp = o; o += n;
    lhm = o; o += n;
    lhp = o; o += n;
    w = o; o += n;
    x = o; o += n;
    xhalf = o; o += n + 1;
    total = o;
  }
};

// host-side 1-D operators in FP64
struct Basis {
  int N = 0, n = 0, nodes = 0;
  std::vector<double> x, w, D, Dhat, lm, lp, lhm, lhp, Vinv, xhalf;
};

Basis make_basis(int N, int nodes);
// Gauss-Lobatto nodes and weights of degree N
void lobatto(int N, std::vector<double> &x, std::vector<double> &w);
// fill the basis block (n = N+1) in the layout of BasisOffsets
std::vector<double> basis_block(const Basis &b);

// host geometry of a mesh on the solution nodes (FP64, SoA layouts of View)
struct Geometry {
  std::vector<double> Ja;   // [9][E][n3]
  std::vector<double> J;    // [E][n3]
  std::vector<double> NS;   // [3][E*6][n2]   (already oriented per View::NS)
  std::vector<double> Xs;   // [3][E][n3]
  std::vector<int2> conn;   // [E][6]
};

// builds metrics, face normals and connectivity; returns DG_OK or DG_EMESH
// with a message in err.
int build_geometry(const Basis &b, const dg_mesh &m, Geometry &g, std::string &err);

// orientation code map (p,q) -> neighbour face coordinates
__host__ __device__ inline void orient_map(int code, int p, int q, int N, int &pp, int &qq) {
  int a = (code & 1) ? q : p;
  int c = (code & 1) ? p : q;
  pp = (code & 2) ? N - a : a;
  qq = (code & 4) ? N - c : c;
}

// ---------------------------------------------------------------------------
// kernel launchers (kernels.hip).  `views` is a device array of nreq views;
// blk_start[r] is the first block of request r (prefix sums, nreq+1 entries,
// device).  A single solve passes nreq = 0 and its view in v0.
// ---------------------------------------------------------------------------
// K_DIAG: the volume sweep with the per-element dissipation sums (View::diag)
enum Kernel { K_TRACE = 0, K_LIFT = 1, K_RHS = 2, K_DIAG = 3 };

// workgroup shape of an element block at degree N
template <int N>
struct Sz {
  static constexpr int n = N + 1, n2 = n * n, n3 = n2 * n, nf = 6 * n2;
  static constexpr int epb = (256 / n3) > 1 ? 256 / n3 : 1;  // elements per workgroup
  static constexpr int threads = ((epb * n3 + 63) / 64) * 64;
  // waves per SIMD to plan registers for (128 VGPRs): two 512-thread or four
  // 256-thread workgroups per CU
  static constexpr int minw = (threads == 512 || threads == 256) ? 4 : 1;
};

// the kernels of one degree (kernels_n<N>.hip); the dispatch over N is launch()
template <int N, typename real>
hipError_t launch_n(Kernel k, int mode, const View<real> *views, const int *blk_start, int nreq, int blocks,
                    const View<real> &v0, hipStream_t st);

// the low-storage RK scheme of dg_params::time_scheme: stage count and
// pointers to its A, B, c coefficients
int rk_scheme(int scheme, const double **A, const double **B, const double **C);

int blocks_per_elements(int N, int64_t E);  // number of blocks covering E elements
int block_threads(int N);

template <typename real>
hipError_t launch(Kernel k, int N, int mode, const View<real> *views_dev, const int *blk_start_dev,
                  int nreq, int total_blocks, const View<real> &v0, hipStream_t st);

// reductions: per-block partial results into scratch, returns blocks used
template <typename real>
hipError_t launch_dt(int N, const View<real> &v, double *scratch, int nblk, hipStream_t st);
template <typename real>
hipError_t launch_integrals(int N, const View<real> &v, double *scratch, int nblk, hipStream_t st);
// sets *flag to 1 if U[0..count) holds a NaN or Inf (leaves it otherwise)
hipError_t launch_finite(const double *U, int64_t count, int *flag, hipStream_t st);
hipError_t launch_zero_int(int *p, int count, hipStream_t st);
// out[c] = sum over e < E of in[3 e + c], c = 0..2, in a fixed order
hipError_t launch_sum3(const double *in, int64_t E, double *out, hipStream_t st);
hipError_t launch_cast(const double *src, float *dst, int64_t count, hipStream_t st);

}  // namespace dg
