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

// Device view of one solve: every pointer and scalar a kernel needs for one
// RK stage.  `real` is the arithmetic type of the time derivative (double
// for FP64, float for the mixed form); state and RK register stay double.
template <typename real>
struct View {
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
  real *alpha_raw;  // [E] indicator values before neighbour propagation
  const real *alpha_in; // [E] frozen blending factors or null
  int *bcnt;        // shock capturing: [2] entries of blist, used by alternate surface sweeps
  int *blist;       // shock capturing: [E] workgroups with a blended element, this sweep
  char *base;       // batched launches, in the argument view: the arena that the
                    // descriptors' pointer fields are byte offsets into
  real gamma, Rgas, rRgas, mu, lambda; // perfect gas (rRgas = 1/R), constant viscosity and conductivity
  double Pr;        // Prandtl number (time-step estimate only)
  double t, dt, rkA, rkB;       // stage time, step, LSERK coefficients
  int cur;          // trace buffer read this stage (0: Utr0, 1: Utr1)
  int bpar;         // entry of bcnt this surface sweep counts in; it clears the other
  int viscous, riemann, source, shock;
  int lgl;          // Gauss-Lobatto nodes: l(-1), l(+1) are unit vectors, l-hat vanishes off the end nodes
  int remap;        // XCD-contiguous block order (single solve)
  real ind_a, ind_c, ind_s, alpha_min, alpha_max, ind_T; // indicator (ind_T precomputed threshold)
};

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
enum Kernel { K_TRACE = 0, K_LIFT = 1, K_RHS = 2, K_COUNT = 3 };

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
hipError_t launch_finite(const double *U, int64_t count, int *flag, hipStream_t st);
hipError_t launch_cast(const double *src, float *dst, int64_t count, hipStream_t st);

}  // namespace dg
