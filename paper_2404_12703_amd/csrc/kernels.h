// kernels.h -- HIP kernels of the DGSEM time derivative and the low-storage
// RK update for gfx950 (CDNA4, wave64), as templates over the polynomial
// degree.  Each degree is instantiated in a translation unit of its own
// (kernels_n<N>.hip), so the degrees compile in parallel; kernels.hip holds
// the reductions and the dispatch over N.
//
// Paper (GALAEXI, arXiv 2404.12703) routines, Table tab:dg_routines and App. A:
//   ConsToPrim, ProlongToFace, FillFlux, VolInt, SurfInt, ApplyJac and the
//   Lift_* copies of BR1 (Sec. 2.2 "Second-Order Equations").
//
// Design: one workgroup slot per element, one thread per volume node.  Per
// RK stage with viscosity or shock capturing, two sweeps (BR1 needs every
// neighbour's lifted gradient before any viscous face flux can be formed):
//   k_volume : (shock capturing) the a-priori indicator value of the element;
//              BR1 lifting with g kept on chip; each own face node's viscous
//              normal flux; the whole volume integral.
//   k_surface: (shock capturing) the blending factor from the neighbours'
//              indicator values; the face fluxes (Riemann + BR1 viscous
//              mean) of the six faces, computed by both neighbours from the
//              same operands in the same order so both hold the same bits
//              and nothing is stored; the per-DOF SurfInt gather (one writer
//              per entry, as the paper's GPU SurfInt); ApplyJac; the LSERK
//              stage update; and the next stage's U traces (ProlongToFace).
//   k_blend  : (shock capturing) the same for the workgroups holding an
//              element with a positive blending factor, which k_surface lists
//              and skips, plus the FV subcell operator.
// Euler without shock capturing takes one sweep, k_rhs.
// Traces are ping-ponged between stages because the last sweep reads the
// neighbours' traces of the old state while writing those of the new one.
// Layouts are structure-of-arrays with one contiguous (N+1)^3 block per
// element and variable, so every global access of a workgroup is contiguous.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>

#include "dg_internal.h"
#include "physics.h"

namespace dg {

// loads and stores of single-use streams: non-temporal when NT (the working
// set exceeds the on-die caches), plain otherwise
template <bool NT, typename T>
__device__ __forceinline__ T ld(const T *p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT, typename T>
__device__ __forceinline__ void st(T x, T *p) {
  if constexpr (NT) __builtin_nontemporal_store(x, p);
  else *p = x;
}

__device__ __forceinline__ int vnode(int n, int i, int j, int k) { return i + n * (j + n * k); }

template <int n>
__device__ __forceinline__ int lnode(int d, int l, int p, int q) {
  return d == 0 ? l + n * (p + n * q) : (d == 1 ? p + n * (l + n * q) : p + n * (q + n * l));
}

// Buffers that are read along face lines hold the volume nodes with padded
// strides: row (fixed j, k) n + 1 values, plane (fixed k) n (n + 1).  A wave
// prolongs one face; unpadded, the lanes of a xi face read n apart, which for
// n = 8 puts eight distinct doubles on each LDS bank pair.
template <int n>
struct Pad {
  static constexpr int row = n + 1, plane = n * (n + 1), size = n * n * (n + 1);
  static __device__ __forceinline__ int at(int i, int j, int k) { return i + row * j + plane * k; }
  // the line normal to face f through face node pq, in padded coordinates
  static __device__ __forceinline__ void face_line(int f, int pq, int &base, int &stride) {
    const int d = f >> 1, p = pq % n, q = pq / n;
    base = d == 0 ? row * p + plane * q : (d == 1 ? p + plane * q : p + row * q);
    stride = d == 0 ? 1 : (d == 1 ? row : plane);
  }
};

// a state value (FP64) in the arithmetic type; the mixed form's energy carries
// the background shift (rho e - p_ref/(gamma - 1))
template <typename real>
__device__ __forceinline__ real to_real(double u, int c, const View<real> &v) {
  if constexpr (sizeof(real) == 4) return (real)(c == 4 ? u - v.e_ref : u);
  else return u;
}

// ProlongToFace of the five conservative variables at one face node from a
// padded LDS copy of the element's state (rows of Pad<n>::size values).
// Explicit multiply-adds in a fixed order: an element that recomputes its own
// trace gets the bits its neighbours read from the stored one.
template <int n, typename real>
__device__ __forceinline__ void prolong_state(const real *rows, const real *lv, int base, int stride, real *out) {
  real s[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int l = 0; l < n; ++l) {
    const real lw = lv[l];
#pragma unroll
    for (int c = 0; c < 5; ++c) s[c] = fma(lw, rows[c * Pad<n>::size + base + l * stride], s[c]);
  }
#pragma unroll
  for (int c = 0; c < 5; ++c) out[c] = s[c];
}

// The conservative state at one face node: with Gauss-Lobatto nodes the end
// node of the line (l(-1), l(+1) are unit vectors), else ProlongToFace.
template <int n, bool LGL, typename real>
__device__ __forceinline__ void face_state(const real *rows, const real *lv, int base, int stride, bool plus,
                                           real *out) {
  if constexpr (LGL) {
    const int at = base + (plus ? (n - 1) * stride : 0);
#pragma unroll
    for (int c = 0; c < 5; ++c) out[c] = rows[c * Pad<n>::size + at];
  } else {
    prolong_state<n>(rows, lv, base, stride, out);
  }
}

// which view and which element block this workgroup works on: a single
// solve (nreq = 0) takes its view from the kernel arguments; a batch of solves
// looks its request up in the block prefix sums and loads that request's view.
// One instantiation serves both, so a request computes the same bits alone and
// in any batch.
// The hardware hands consecutive workgroups to the eight XCDs in turn; with
// `remap` each XCD instead receives one contiguous range of element blocks, so
// face neighbours (adjacent element indices) share that XCD's L2.  A bijection
// of [0, gridDim.x).
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int q = nb >> 3, r = nb & 7, x = b & 7, idx = b >> 3;
  const int start = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
  return start + idx;
}

// the descriptors of a batch hold byte offsets into the arena; rebuilding the
// pointers from the argument's arena pointer keeps every access a global-memory
// one (pointers read from memory would be addressed as generic pointers)
template <typename real>
__device__ __forceinline__ View<real> rebase(View<real> v, char *const base) {
  auto at = [base](auto p) { return (decltype(p))(base + (intptr_t)p); };
  auto at_or_null = [base](auto p) { return p ? (decltype(p))(base + (intptr_t)p) : p; };
  v.U = at(v.U);
  v.dU = at(v.dU);
  v.R = at_or_null(v.R);
  v.Ja = at(v.Ja);
  v.invJ = at(v.invJ);
  v.NS = at(v.NS);
  v.Utr0 = at(v.Utr0);
  v.Utr1 = at(v.Utr1);
  v.Hv = at_or_null(v.Hv);
  v.Vol = at_or_null(v.Vol);
  v.conn = at(v.conn);
  v.Xs = at_or_null(v.Xs);
  v.basis = at(v.basis);
  v.alpha = at(v.alpha);
  v.alpha_raw = at(v.alpha_raw);
  v.alpha_in = at_or_null(v.alpha_in);
  v.bcnt = at_or_null(v.bcnt);
  v.blist = at_or_null(v.blist);
  v.diag = at_or_null(v.diag);
  return v;
}

template <typename real>
__device__ __forceinline__ View<real> select_view(const View<real> *views, const int *blk_start, int nreq,
                                                  const View<real> &single, int &lblk) {
  if (nreq == 0) {
    lblk = single.remap ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
    return single;
  }
  const int b = blockIdx.x;
  int r = 0;
  while (r + 1 < nreq && b >= blk_start[r + 1]) ++r;
  lblk = b - blk_start[r];
  return rebase(views[r], single.base);
}

template <int N, typename real>
struct Smem {
  using S = Sz<N>;
  real Dh[S::n * (S::n + 1)];  // rows padded to n + 1: lanes reading different rows hit different banks
  real lm[S::n], lp[S::n], lhm[S::n], lhp[S::n];
};

template <int N, typename real>
__device__ __forceinline__ void load_basis(Smem<N, real> &sb, const real *basis) {
  using S = Sz<N>;
  constexpr int n = S::n;
  BasisOffsets o(n);
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) sb.Dh[(t / n) * (n + 1) + t % n] = basis[o.Dhat + t];
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    sb.lm[t] = basis[o.lm + t];
    sb.lp[t] = basis[o.lp + t];
    sb.lhm[t] = basis[o.lhm + t];
    sb.lhp[t] = basis[o.lhp + t];
  }
}

// ---------------------------------------------------------------------------
// ProlongToFace of the state into the current trace buffer
// ---------------------------------------------------------------------------
template <int N, typename real, bool LGL>
__global__ void __launch_bounds__(Sz<N>::threads) k_trace(const View<real> *views, const int *blk_start, int nreq,
                                                         View<real> single) {
  using S = Sz<N>;
  constexpr int n = S::n, n2 = S::n2, n3 = S::n3, nf = S::nf, epb = S::epb;
  int lblk;
  const View<real> v = select_view(views, blk_start, nreq, single, lblk);
  __shared__ Smem<N, real> sb;
  __shared__ real sU[epb][5 * Pad<n>::size];
  load_basis<N, real>(sb, v.basis);
  const int le = threadIdx.x / n3, a = threadIdx.x - le * n3;
  const int64_t e = (int64_t)lblk * epb + le;
  const bool active = le < epb && e < v.E;
  const int64_t Ev = v.E * n3, Ef = v.E * 6 * n2;
  const uint32_t vi = (uint32_t)(e * n3 + a), fb = (uint32_t)(e * 6 * n2);
  const int i = a % n, j = (a / n) % n, k = a / n2;
  real *const su = sU[le < epb ? le : 0];
  if (active) {
#pragma unroll
    for (int c = 0; c < 5; ++c) su[c * Pad<n>::size + Pad<n>::at(i, j, k)] = to_real((v.U + c * Ev)[vi], c, v);
  }
  __syncthreads();
  if (active) {
    real *tr = v.cur ? v.Utr1 : v.Utr0;
    for (int fn = a; fn < nf; fn += n3) {
      const int f = fn / n2, pq = fn - f * n2;
      int base, stride;
      Pad<n>::face_line(f, pq, base, stride);
      real t[5];
      face_state<n, LGL>(su, (f & 1) ? sb.lp : sb.lm, base, stride, f & 1, t);
#pragma unroll
      for (int c = 0; c < 5; ++c) (tr + c * Ef)[fb + fn] = t[c];
    }
  }
}

// ---------------------------------------------------------------------------
// a-priori indicator (Sec. 2.3): modal energy of eps = rho p.  m = (V^-1 (x)
// V^-1 (x) V^-1) eps by three line transforms through LDS rows r0..r2 (V^-1
// staged in vs), then fixed-order sums of the energies (no atomics, so the
// value is reproducible): within each wave by lane exchanges and over the
// waves of the element through r3..r6 where elements and waves align, else a
// tree through r3..r6.  The energy fractions of the top two shells (modes
// whose largest degree is N, and N - 1) are summed directly rather than formed
// as differences of nearly equal totals: the same quantity, but its rounding
// is relative to itself, which in FP32 keeps the logistic's steep part from
// amplifying the cancellation.  Every thread of the block must call it.
// Returns the clipped logistic value on thread a == 0 of each element.
// ---------------------------------------------------------------------------
template <int N, typename real>
__device__ __forceinline__ real indicator_raw(const View<real> &v, const real *Vinv, real *r0, real *r1, real *r2,
                                              real *r3, real *r4, real *r5, real *r6, real *vs, bool active, int a,
                                              real eps) {
  constexpr int n = N + 1, n2 = n * n, n3 = n2 * n;
  const int i = a % n, j = (a / n) % n, k = a / n2;
  if (active) {
    for (int t = a; t < n2; t += n3) vs[t] = Vinv[t];
    r0[a] = eps;
  }
  __syncthreads();
  if (active) {
    real t = real(0);
#pragma unroll
    for (int r = 0; r < n; ++r) t += vs[i * n + r] * r0[vnode(n, r, j, k)];
    r1[a] = t;
  }
  __syncthreads();
  if (active) {
    real t = real(0);
#pragma unroll
    for (int r = 0; r < n; ++r) t += vs[j * n + r] * r1[vnode(n, i, r, k)];
    r2[a] = t;
  }
  __syncthreads();
  // energies: all modes, largest degree <= N - 1, largest degree N, largest degree N - 1
  real e0 = real(0), e1 = real(0), h1 = real(0), h2 = real(0);
  if (active) {
    real m = real(0);
#pragma unroll
    for (int r = 0; r < n; ++r) m += vs[k * n + r] * r2[vnode(n, i, j, r)];
    e0 = m * m;
    const int top = max(i, max(j, k));
    e1 = top < N ? e0 : real(0);
    h1 = top == N ? e0 : real(0);
    h2 = top == N - 1 ? e0 : real(0);
  }
  // each element's nodes fill whole waves (or the element is alone in the
  // workgroup): reduce within waves, then over the element's waves
  constexpr bool wave_sums = (n3 % 64 == 0) || Sz<N>::epb == 1;
  real tot = real(0), c1 = real(0), t1 = real(0), t2 = real(0);
  if constexpr (wave_sums) {
    // every lane takes part; lanes without a node add zeros
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      e0 += __shfl_xor(e0, off, 64);
      e1 += __shfl_xor(e1, off, 64);
      h1 += __shfl_xor(h1, off, 64);
      h2 += __shfl_xor(h2, off, 64);
    }
    constexpr int W = (n3 + 63) / 64;
    if (active && (a & 63) == 0) {
      r3[a >> 6] = e0;
      r4[a >> 6] = e1;
      r5[a >> 6] = h1;
      r6[a >> 6] = h2;
    }
    __syncthreads();
    if (active && a == 0) {
#pragma unroll
      for (int w = 0; w < W; ++w) {
        tot += r3[w];
        c1 += r4[w];
        t1 += r5[w];
        t2 += r6[w];
      }
    }
  } else {
    if (active) {
      r3[a] = e0;
      r4[a] = e1;
      r5[a] = h1;
      r6[a] = h2;
    }
    __syncthreads();
    constexpr int P2 = n3 <= 8 ? 8 : (n3 <= 16 ? 16 : (n3 <= 32 ? 32 : (n3 <= 64 ? 64 : (n3 <= 128 ? 128 : (n3 <= 256 ? 256 : (n3 <= 512 ? 512 : 1024))))));
#pragma unroll
    for (int st = P2 / 2; st > 0; st >>= 1) {
      if (active && a < st && a + st < n3) {
        r3[a] += r3[a + st];
        r4[a] += r4[a + st];
        r5[a] += r5[a + st];
        r6[a] += r6[a + st];
      }
      __syncthreads();
    }
    if (active && a == 0) {
      tot = r3[0];
      c1 = r4[0];
      t1 = r5[0];
      t2 = r6[0];
    }
  }
  real alpha = real(0);
  if (active && a == 0) {
    const real E1 = tot > real(0) ? t1 / tot : real(0);
    const real E2 = c1 > real(0) ? t2 / c1 : real(0);
    const real Ev = fmax(E1, E2);
    const real T = v.ind_T;
    alpha = real(1) / (real(1) + exp(-(v.ind_s / T) * (Ev - T)));
    if (alpha < v.alpha_min) alpha = real(0);
    else if (alpha > real(1) - v.alpha_min) alpha = real(1);
    alpha = fmin(alpha, v.alpha_max);
  }
  return alpha;
}

// reconstruction helpers of the FV subcells
template <typename real>
__device__ __forceinline__ real minmod2(real a, real b) {
  if (a * b <= real(0)) return real(0);
  return (a > real(0) ? real(1) : real(-1)) * fmin(fabs(a), fabs(b));
}

template <typename real>
__device__ __forceinline__ void prim2cons(const real *q, real gamma, real *U) {
  U[0] = q[0];
  U[1] = q[0] * q[1];
  U[2] = q[0] * q[2];
  U[3] = q[0] * q[3];
  U[4] = q[4] / (gamma - real(1)) + real(0.5) * q[0] * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
}

// ---------------------------------------------------------------------------
// Euler without shock capturing: one sweep per stage.  FillFlux (Riemann
// flux of both sides' stored U traces), VolInt of F_adv through LDS one
// direction at a time, the SurfInt gather, ApplyJac, the stage update and the
// next U traces.  mode 0: du = A du + dt R, U += B du; mode 1: write R only.
// ---------------------------------------------------------------------------
template <int N, typename real>
__global__ void __launch_bounds__(Sz<N>::threads, Sz<N>::minw) k_rhs(const View<real> *views, const int *blk_start,
                                                                      int nreq, View<real> single, int mode) {
  using S = Sz<N>;
  constexpr int n = S::n, n2 = S::n2, n3 = S::n3, nf = S::nf, epb = S::epb;
  int lblk;
  const View<real> v = select_view(views, blk_start, nreq, single, lblk);
  __shared__ Smem<N, real> sb;
  // contravariant fluxes of one direction (rows of n3), later the updated
  // state (padded rows) for the next traces
  __shared__ real sB[epb][5 * Pad<n>::size];
  __shared__ real sS[epb][5][nf];
  load_basis<N, real>(sb, v.basis);
  const int le = threadIdx.x / n3, a = threadIdx.x - le * n3;
  const int64_t e = (int64_t)lblk * epb + le;
  const bool active = le < epb && e < v.E;
  real *const sm = sB[le < epb ? le : 0];
  const int64_t Ev = v.E * n3, Ef = v.E * 6 * n2;
  const uint32_t vi = (uint32_t)(e * n3 + a), fb = (uint32_t)(e * 6 * n2);
  const real gam = v.gamma, rR = v.rRgas;
  const Bg<real> bg{v.bg_p, v.bg_H};
  const real *tr = v.cur ? v.Utr1 : v.Utr0;
  const int i = a % n, j = (a / n) % n, k = a / n2;
  if (active) {
    // FillFlux for the six faces of this element (face nodes spread over the threads)
    for (int fn = a; fn < nf; fn += n3) {
      const int f = fn / n2, pq = fn - f * n2, p = pq % n, q = pq / n;
      const int2 c = v.conn[e * 6 + f];
      const bool primary = (c.y >> 3) & 1;
      int pp, qq;
      orient_map(c.y & 7, p, q, N, pp, qq);
      const uint32_t io = fb + fn, in = (uint32_t)c.x * n2 + pp + n * qq;
      const uint32_t im = primary ? io : in, is = primary ? in : io;
      real Um[5], Us[5], Pm[6], Ps[6];
#pragma unroll
      for (int s = 0; s < 5; ++s) {
        Um[s] = (tr + s * Ef)[im];
        Us[s] = (tr + s * Ef)[is];
      }
      cons2prim(Um, gam, rR, Pm, bg);
      cons2prim(Us, gam, rR, Ps, bg);
      real nsv[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const real ns = (v.NS + d * Ef)[io];
        nsv[d] = primary ? ns : -ns;
      }
      const real sh = sqrt(nsv[0] * nsv[0] + nsv[1] * nsv[1] + nsv[2] * nsv[2]);
      const real ish = real(1) / sh;
      const real nv[3] = {nsv[0] * ish, nsv[1] * ish, nsv[2] * ish};
      real Fs[5];
      if (v.riemann == 1) riemann_roe(Um, Pm, Us, Ps, nv, gam, Fs, bg);
      else riemann_llf(Um, Pm, Us, Ps, nv, gam, Fs, bg);
#pragma unroll
      for (int s = 0; s < 5; ++s) sS[le][s][fn] = primary ? Fs[s] * sh : -(Fs[s] * sh);
    }
  }
  real Ja[9], Fx[5], Fy[5], Fz[5];
  double Uold[5] = {0, 0, 0, 0, 0};
  if (active) {
    real U[5], P[6];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      Uold[c] = (v.U + c * Ev)[vi];
      U[c] = to_real(Uold[c], c, v);
    }
    cons2prim(U, gam, rR, P, bg);
    flux_adv<0>(U, P, Fx, bg);
    flux_adv<1>(U, P, Fy, bg);
    flux_adv<2>(U, P, Fz, bg);
#pragma unroll
    for (int c = 0; c < 9; ++c) Ja[c] = (v.Ja + c * Ev)[vi];
  }
  // VolInt: one computational direction at a time through LDS
  real V[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int ci = 0; ci < 3; ++ci) {
    if (active) {
#pragma unroll
      for (int c = 0; c < 5; ++c) sm[c * n3 + a] = Ja[3 * ci + 0] * Fx[c] + Ja[3 * ci + 1] * Fy[c] + Ja[3 * ci + 2] * Fz[c];
    }
    __syncthreads();
    if (active) {
      const int idx = ci == 0 ? i : (ci == 1 ? j : k);
#pragma unroll
      for (int alp = 0; alp < n; ++alp) {
        const int src = ci == 0 ? vnode(n, alp, j, k) : (ci == 1 ? vnode(n, i, alp, k) : vnode(n, i, j, alp));
        const real dh = sb.Dh[idx * (n + 1) + alp];
#pragma unroll
        for (int c = 0; c < 5; ++c) V[c] += dh * sm[c * n3 + src];
      }
    }
    __syncthreads();
  }
  double Unew[5] = {0, 0, 0, 0, 0};
  if (active) {
    // 1/J and the RK register, loaded before the gather: their latency
    // overlaps it, and the register's five loads precede its five stores
    // (which the compiler could not move them across)
    const real iJ = v.invJ[vi];
    double dUo[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) dUo[c] = (mode == 0 && v.rkA != 0.0) ? (v.dU + c * Ev)[vi] : 0.0;
    // SurfInt gather (one writer per entry) and ApplyJac
    const int pqf[3] = {j + n * k, i + n * k, i + n * j};
    const int lf[3] = {i, j, k};
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      const int d = f >> 1;
      const real lh = (f & 1) ? sb.lhp[lf[d]] : sb.lhm[lf[d]];
#pragma unroll
      for (int c = 0; c < 5; ++c) V[c] += sS[le][c][f * n2 + pqf[d]] * lh;
    }
    double R[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) R[c] = (double)(-(V[c] * iJ));
    if (v.source == 1) {
      const double x = v.Xs[vi], y = (v.Xs + Ev)[vi], z = (v.Xs + 2 * Ev)[vi];
      const double cs = 0.1 * M_PI * cos(M_PI * (x + y + z - v.t));
      const double gg = (double)gam;
      R[0] += 2.0 * cs;
      R[1] += 3.0 * cs;
      R[2] += 3.0 * cs;
      R[3] += 3.0 * cs;
      R[4] += 2.0 * (3.0 * gg - 2.0) / (gg - 1.0) * cs;
    }
    if (mode == 1) {
#pragma unroll
      for (int c = 0; c < 5; ++c) (v.R + c * Ev)[vi] = R[c];
    } else {
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        double *dUc = v.dU + c * Ev;
        // the first stage (A = 0) does not read the register: whatever it
        // holds (a restored state, an aborted step) cannot leak into the step
        const double du = (v.rkA != 0.0 ? v.rkA * dUo[c] : 0.0) + v.dt * R[c];
        dUc[vi] = du;
        Unew[c] = Uold[c] + v.rkB * du;
        (v.U + c * Ev)[vi] = Unew[c];
      }
    }
  }
  if (mode == 0) {
    // ProlongToFace of the updated state for the next stage (the last
    // barrier of the volume integral precedes these writes)
    if (active) {
#pragma unroll
      for (int c = 0; c < 5; ++c) sm[c * Pad<n>::size + Pad<n>::at(i, j, k)] = to_real(Unew[c], c, v);
    }
    __syncthreads();
    if (active) {
      real *trn = v.cur ? v.Utr0 : v.Utr1;
      for (int fn = a; fn < nf; fn += n3) {
        const int f = fn / n2, pq = fn - f * n2;
        int base, stride;
        Pad<n>::face_line(f, pq, base, stride);
        real t[5];
        prolong_state<n>(sm, (f & 1) ? sb.lp : sb.lm, base, stride, t);
#pragma unroll
        for (int c = 0; c < 5; ++c) (trn + c * Ef)[fb + fn] = t[c];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// FV subcell volume term of one element (Sec. 2.3).  Subcells sit on the
// Lobatto nodes with interfaces at the cumulative weights; the interface
// metric accumulates w_m (D Ja)_m along each line from the element face;
// primitives are reconstructed with minmod slopes (zero in the two boundary
// subcells) and joined by the LLF flux.  `rows` are 16 LDS rows of n3 values
// of this element: 0-4 primitives, 5-7 the metric of one direction, 8-10
// w_l (D Ja)_l, 11-15 interface fluxes.  sFV holds D, w, x, xhalf.  Every
// thread of the workgroup calls it: it holds barriers.  Adds the subcell
// term at this node to Vfv (the sign convention of the DG volume integral).
// ---------------------------------------------------------------------------
template <int N, typename real>
__device__ __forceinline__ void fv_subcells(real *rows, const real *sFV, bool active, int a, int i, int j, int k,
                                            const real *P, const real *Ja, real gam, real rR, Bg<real> bg,
                                            real *Vfv) {
  constexpr int n = N + 1, n3 = n * n * n;
  const real *Dm = sFV;
  const real *wq = sFV + n * n;
  const real *xq = sFV + n * n + n;
  const real *xh = sFV + n * n + 2 * n;
  if (active) {
#pragma unroll
    for (int c = 0; c < 5; ++c) rows[c * n3 + a] = P[c];
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int l = d == 0 ? i : (d == 1 ? j : k);
    const int pp = d == 0 ? j : i, qq = d == 2 ? j : k;
    if (active) {
#pragma unroll
      for (int c = 0; c < 3; ++c) rows[(5 + c) * n3 + a] = Ja[3 * d + c];
    }
    __syncthreads();
    if (active) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        real s = real(0);
#pragma unroll
        for (int m = 0; m < n; ++m) s += Dm[l * n + m] * rows[(5 + c) * n3 + lnode<n>(d, m, pp, qq)];
        rows[(8 + c) * n3 + a] = wq[l] * s;
      }
    }
    __syncthreads();
    if (active && l < N) {
      real Jh[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        real acc = rows[(5 + c) * n3 + lnode<n>(d, 0, pp, qq)];
        for (int m = 0; m <= l; ++m) acc += rows[(8 + c) * n3 + lnode<n>(d, m, pp, qq)];
        Jh[c] = acc;
      }
      const real sh = sqrt(Jh[0] * Jh[0] + Jh[1] * Jh[1] + Jh[2] * Jh[2]);
      const real nv[3] = {Jh[0] / sh, Jh[1] / sh, Jh[2] / sh};
      real qL[5], qR[5];
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        const real q0 = rows[c * n3 + lnode<n>(d, l, pp, qq)];
        const real q1 = rows[c * n3 + lnode<n>(d, l + 1, pp, qq)];
        real s0 = real(0), s1 = real(0);
        if (l >= 1) {
          const real qm = rows[c * n3 + lnode<n>(d, l - 1, pp, qq)];
          s0 = minmod2((q0 - qm) / (xq[l] - xq[l - 1]), (q1 - q0) / (xq[l + 1] - xq[l]));
        }
        if (l + 1 <= N - 1) {
          const real q2 = rows[c * n3 + lnode<n>(d, l + 2, pp, qq)];
          s1 = minmod2((q1 - q0) / (xq[l + 1] - xq[l]), (q2 - q1) / (xq[l + 2] - xq[l + 1]));
        }
        qL[c] = q0 + s0 * (xh[l + 1] - xq[l]);
        qR[c] = q1 - s1 * (xq[l + 1] - xh[l + 1]);
      }
      real UL[5], UR[5], PL[6], PR[6], F[5];
      prim2cons(qL, gam, UL);
      prim2cons(qR, gam, UR);
      cons2prim(UL, gam, rR, PL, bg);
      cons2prim(UR, gam, rR, PR, bg);
      riemann_llf(UL, PL, UR, PR, nv, gam, F, bg);
#pragma unroll
      for (int c = 0; c < 5; ++c) rows[(11 + c) * n3 + a] = F[c] * sh;
    }
    __syncthreads();
    if (active) {
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        real r = real(0);
        if (l < N) r += rows[(11 + c) * n3 + a];
        if (l > 0) r -= rows[(11 + c) * n3 + lnode<n>(d, l - 1, pp, qq)];
        Vfv[c] += r / wq[l];
      }
    }
    __syncthreads();
  }
}

// Face work unit t of an element: the direction d and first side s0 of its
// face nodes and their face index pq.  fpu = 2: both sides of line pq; fpu = 1:
// face node t.  With plane waves each wave's units share one face direction.
template <int n, int fpu, bool plane_waves>
__device__ __forceinline__ void face_unit(int t, int &d, int &s0, int &pq) {
  constexpr int n2 = n * n;
  int g = t / n2;  // d (fpu = 2) or the face (fpu = 1)
  if constexpr (plane_waves) g = __builtin_amdgcn_readfirstlane(g);
  pq = t - g * n2;
  d = fpu == 2 ? g : g >> 1;
  s0 = fpu == 2 ? 0 : g & 1;
}

template <int N, typename real, bool SHOCK, bool SPLIT>
struct VolLds {
  using S = Sz<N>;
  static constexpr int n3 = S::n3, nf = S::nf;
  // per-element offsets.  Lifting: primitives u, v, w, T (4 rows of n3), the
  // nine metric rows Ja^i_d (9 x n3), with the split form the density (1 x
  // n3), BR1 face averages (4 x nf) and own outward n shat (3 x nf).  g (12
  // padded rows) then covers the first blocks, and the 15 rows of
  // contravariant fluxes the whole area.
  static constexpr int V = 0, J = 4 * n3, Rho = 13 * n3, Avg = (SPLIT ? 14 : 13) * n3, Ns = Avg + 4 * nf, G = 0,
                       F = 0;
  static constexpr int gsz = Pad<S::n>::size;  // one padded row of g
  static constexpr int rows = (Ns + 3 * nf) > 15 * n3 ? (Ns + 3 * nf) : 15 * n3;
  // Face work units: with fpu = 2 a thread takes the two face nodes at the
  // ends of one line of nodes, so the line of g is read once for both; with
  // fpu = 1 one face node.  Two per unit halves the LDS reads of
  // Lift_ProlongToFace but also the threads that share them.  Measured per
  // degree on ~7M-DOF meshes, one per unit is faster at N = 6, and at N = 5
  // in FP64; two elsewhere (8% less volume-sweep time at N = 3, 3% at N = 7).
  // The FP64 sweeps at N = 9 and with shock capturing or the split form at
  // N = 7 take one: two would spill registers.
  static constexpr bool f64 = sizeof(real) == 8;
  static constexpr int fpu = (N == 6 || (f64 && (N == 5 || N >= 9 || (N == 7 && (SHOCK || SPLIT))))) ? 1 : 2;
  // Nodes per thread: at N = 7 (and N = 5 in the mixed form; one element
  // per workgroup, even n) a thread of the standard form without shock
  // capturing takes the two nodes k and k + n/2 of one column.  They share
  // the reads along zeta, the D-hat rows along xi and eta and the zeta faces
  // of Lift_SurfInt; the workgroup has half the threads, each with twice the
  // registers.  That took 7% off the mixed sweep at both degrees and 2 to 3%
  // off the FP64 sweep at N = 7, where the lifting contraction is unrolled by
  // 2 instead of n: fully unrolled, its loads in flight spilled past 256 VGPRs
  // (by 4: 216 VGPRs and slower than by 2, 176 VGPRs; not unrolled: slower
  // again).
  static constexpr bool plane_waves = S::n2 == 64 && S::epb == 1;
  static constexpr int npt = ((N == 7 && !SHOCK && !SPLIT) || (N == 5 && !SHOCK && !SPLIT && !f64)) ? 2 : 1;
  // The split form's loop also carries the two-point flux: not unrolled, it
  // fits the register budget of two 512-thread workgroups per CU at N = 7
  // (128 VGPRs, one spill; unrolled by 2 it needed 148, which left one
  // workgroup per CU and took 1.04 ms instead of 0.68 ms on the 24^3
  // supersonic TGV; 0.79 against 0.68 ms at N = 5).
  static constexpr int lift_unroll = SPLIT ? 1 : ((npt == 2 && f64) ? 2 : S::n);
  static constexpr int tpe = n3 / npt;  // threads per element
  static constexpr int threads = npt == 1 ? S::threads : tpe;
  static constexpr int minw = npt == 1 ? S::minw : 2;
  // FP64 at N = 7 (a wave is one k-plane): the xi and eta contractions of the
  // volume integral on the matrix cores (4x4x4, four blocks), results in the
  // lanes that own them (see k_volume)
  static constexpr bool mfma = f64 && N == 7;
  static constexpr int units = nf / fpu;
  static constexpr int upt = (units + tpe - 1) / tpe;  // units per thread
  static_assert(12 * gsz <= Ns, "g must not cover n shat");
  static_assert(npt == 1 || (S::n % 2 == 0 && S::epb == 1), "column pairs need an even n and one element");
};

// ---------------------------------------------------------------------------
// Volume sweep.  From the lifted gradient, which never leaves the chip, it
// forms (a) at each own face node this side's viscous normal flux
// H = F_v(prim, g).n, with n in the primary side's orientation, and (b) the
// complete volume integral of F_adv - F_v.  Writes H (4 values per face node:
// the mass component is zero) and the volume integral (5 per node); with
// shock capturing also the element's indicator value; with DIAG the
// element's dissipation sums (View::diag).  SUTH: Sutherland's law for the
// viscosity (a template flag: its divisions would cost the constant-viscosity
// sweeps registers).
// Split form (SPLIT, Gauss-Lobatto nodes; Sec. 2.2 "Nonlinear Stability"):
// the advective part of the volume integral becomes
//   sum_alpha (D + D-hat)_{i alpha} F#(U_ijk, U_alpha jk; mean Ja^1) + ...
// with Pirozzoli's two-point flux F#.  On Gauss-Lobatto nodes D + D-hat =
// 2 D - W^-1 B (summation by parts), so this is the strong split form with
// the boundary values of its surface correction folded in, and the weak
// form's surface integral of f* completes it.  The two-point fluxes take
// their operands from the rows the lifting contraction reads anyway (the
// metric rows, u, v, w, T) plus one density row; pressure and enthalpy
// follow from them: p = rho R T, H = gamma R T/(gamma - 1) + |u|^2/2.
// The viscous part keeps the weak form.
// ---------------------------------------------------------------------------
template <int N, typename real, bool SHOCK, bool LGL, bool SPLIT, bool SUTH, bool DIAG = false, bool NT = false>
__global__ void __launch_bounds__((VolLds<N, real, SHOCK, SPLIT>::threads), (VolLds<N, real, SHOCK, SPLIT>::minw))
    k_volume(const View<real> *views, const int *blk_start, int nreq, View<real> single) {
  using S = Sz<N>;
  using L = VolLds<N, real, SHOCK, SPLIT>;
  constexpr int n = S::n, n2 = S::n2, n3 = S::n3, nf = S::nf, epb = S::epb;
  constexpr int npt = L::npt, tpe = L::tpe, kstep = n / npt;
  static_assert(!SPLIT || LGL, "the split form needs Gauss-Lobatto nodes");
  int lblk;
  const View<real> v = select_view(views, blk_start, nreq, single, lblk);
  __shared__ Smem<N, real> sb;
  __shared__ __align__(16) real sA[epb][L::rows];
  // (D + D-hat)/16, rows padded to n + 1: the weights of the two-point sums
  // (two_point_kep_sums), exact scaling by a power of two
  __shared__ real sDs[SPLIT ? n * (n + 1) : 1];
  load_basis<N, real>(sb, v.basis);
  if constexpr (SPLIT) {
    const BasisOffsets o(n);
    for (int t = threadIdx.x; t < n * n; t += blockDim.x)
      sDs[(t / n) * (n + 1) + t % n] = (v.basis[o.D + t] + v.basis[o.Dhat + t]) * real(0.0625);
  }
  // thread a of an element holds its nodes a + m tpe, m < npt: the same i and
  // j, and k = k0 + m kstep
  const int le = threadIdx.x / tpe, a = threadIdx.x - le * tpe;
  const int64_t e = (int64_t)lblk * epb + le;
  const bool active = le < epb && e < v.E;
  real *const sm = sA[le < epb ? le : 0];
  // row strides of the volume and face arrays; per-lane indices are 32-bit
  // (the host keeps every row below 2^31 entries)
  const int64_t Ev = v.E * n3, Ef = v.E * 6 * n2;
  const uint32_t vi = (uint32_t)(e * n3 + a), fb = (uint32_t)(e * 6 * n2);
  const real gam = v.gamma, rR = v.rRgas, mu = v.mu, lam = v.lambda;
  const Bg<real> bg{v.bg_p, v.bg_H};
  const bool visc = v.viscous != 0;  // the same for the whole grid
  constexpr bool suth = SUTH;
  const real *tr = v.cur ? v.Utr1 : v.Utr0;
  const int i = a % n, j = (a / n) % n, k0 = a / n2;
  // when a wave is one k-plane of one element (n^2 = 64), the k rows of D-hat
  // and the face of a face node are the same on every lane: scalar loads
  // instead of LDS reads
  constexpr bool plane_waves = L::plane_waves;
  real dk[npt][n];
  if constexpr (plane_waves) {
    const int ku = __builtin_amdgcn_readfirstlane(k0);
    const BasisOffsets o(n);
#pragma unroll
    for (int m = 0; m < npt; ++m)
#pragma unroll
      for (int al = 0; al < n; ++al) dk[m][al] = v.basis[o.Dhat + (ku + m * kstep) * n + al];
  }
  real U[npt][5];
  real pf[L::upt][L::fpu][4];  // own face velocity and viscosity at this thread's face nodes
  real mun[npt];               // viscosity at this thread's nodes (Sutherland: mu(T), computed early,
                               // where few registers are live)
  if (active) {
#pragma unroll
    for (int m = 0; m < npt; ++m)
#pragma unroll
      for (int c = 0; c < 5; ++c) U[m][c] = to_real(ld<NT>(v.U + c * Ev + vi + m * tpe), c, v);
  }
  // 1/J at this thread's nodes, fetched beside the state: its first use comes
  // after the lifting sums, and a load issued there would stall the wave
  real iJe[npt];
  if (active && visc) {
#pragma unroll
    for (int m = 0; m < npt; ++m) iJe[m] = v.invJ[vi + m * tpe];
  }
  // Lift_FillFlux operands: both sides' U traces and this side's n shat at
  // the thread's face nodes.  With one node per thread they are fetched here,
  // beside the state, which hides their latency behind the metric loads (the
  // split-form sweep 3.9% faster at N = 7); the column-pair sweep fetches
  // them where it uses them (1% faster so).
  real tUo[L::upt][L::fpu][5], tUn[L::upt][L::fpu][5], tNs[L::upt][L::fpu][3];
  bool prim[L::upt][L::fpu];  // this side is the face's primary side (read with the traces)
  auto fetch_face = [&](int r, int u, int f, int fn, int pq) {
    const int2 c = v.conn[e * 6 + f];
    prim[r][u] = (c.y >> 3) & 1;
    int pp, qq;
    orient_map(c.y & 7, pq % n, pq / n, N, pp, qq);
    const uint32_t io = fb + fn, in = (uint32_t)c.x * n2 + pp + n * qq;
#pragma unroll
    for (int s = 0; s < 5; ++s) {
      tUo[r][u][s] = (tr + s * Ef)[io];
      tUn[r][u][s] = (tr + s * Ef)[in];
    }
#pragma unroll
    for (int dd = 0; dd < 3; ++dd) tNs[r][u][dd] = (v.NS + dd * Ef)[io];
  };
  if (npt == 1 && active && visc) {
#pragma unroll
    for (int r = 0; r < L::upt; ++r) {
      const int t = a + r * tpe;
      if (t < L::units) {
        int d, s0, pq;
        face_unit<n, L::fpu, plane_waves>(t, d, s0, pq);
#pragma unroll
        for (int u = 0; u < L::fpu; ++u) fetch_face(r, u, 2 * d + s0 + u, (2 * d + s0 + u) * n2 + pq, pq);
      }
    }
  }
  if constexpr (SHOCK) {
    static_assert(npt == 1, "the indicator takes one node per thread");
    // a-priori indicator of this element (Sec. 2.3) on epsilon = rho p, in the
    // metric rows before they are filled
    real eps = real(0);
    if (active) {
      real P[6];
      cons2prim(U[0], gam, rR, P, bg);
      eps = P[0] * full_p(P[4], bg);
    }
    const BasisOffsets o(n);
    real *r = sm + L::J;
    const real al = indicator_raw<N, real>(v, v.basis + o.Vinv, r, r + n3, r + 2 * n3, r + 3 * n3, r + 4 * n3,
                                           r + 5 * n3, r + 6 * n3, r + 7 * n3, active, a, eps);
    if (active && a == 0) v.alpha_raw[e] = al;
    __syncthreads();
  }
  if (active) {
#pragma unroll
    for (int m = 0; m < npt; ++m) {
      const int am = a + m * tpe;
#pragma unroll
      for (int c = 0; c < 9; ++c) sm[L::J + c * n3 + am] = ld<NT>(v.Ja + c * Ev + vi + m * tpe);
      real P[6];
      cons2prim(U[m], gam, rR, P, bg);
      sm[L::V + 0 * n3 + am] = P[1];
      sm[L::V + 1 * n3 + am] = P[2];
      sm[L::V + 2 * n3 + am] = P[3];
      sm[L::V + 3 * n3 + am] = P[5];
      if constexpr (SPLIT) sm[L::Rho + am] = P[0];
      mun[m] = suth ? sutherland(P[5], mu, v.rTref) : mu;
    }
  }
  if (active && visc) {
    // Lift_FillFlux: the BR1 average of both sides' traces, and this side's
    // outward n shat, face velocity and temperature for its viscous flux later on
#pragma unroll
    for (int r = 0; r < L::upt; ++r) {
      const int t = a + r * tpe;
      if (t < L::units) {
        int d, s0, pq;
        face_unit<n, L::fpu, plane_waves>(t, d, s0, pq);
#pragma unroll
        for (int u = 0; u < L::fpu; ++u) {
          const int f = 2 * d + s0 + u, fn = f * n2 + pq;
          if constexpr (npt != 1) fetch_face(r, u, f, fn, pq);
          real Po[6], Pn[6];
          cons2prim(tUo[r][u], gam, rR, Po, bg);
          cons2prim(tUn[r][u], gam, rR, Pn, bg);
          const real vo[4] = {Po[1], Po[2], Po[3], Po[5]}, vn[4] = {Pn[1], Pn[2], Pn[3], Pn[5]};
#pragma unroll
          for (int s = 0; s < 4; ++s) sm[L::Avg + s * nf + fn] = real(0.5) * (vo[s] + vn[s]);
#pragma unroll
          for (int dd = 0; dd < 3; ++dd) {
            sm[L::Ns + dd * nf + fn] = tNs[r][u][dd];
            pf[r][u][dd] = Po[1 + dd];
          }
          pf[r][u][3] = suth ? sutherland(Po[5], mu, v.rTref) : mu;
        }
      }
    }
  }
  __syncthreads();
  real Fc[npt][15];  // contravariant fluxes Ja^i . (F_adv - F_v), i = 0..2 (split form: -F_v only)
  real g[npt][12];
  real Vs[npt][5];   // split form: the advective volume integral of the two-point fluxes
#pragma unroll
  for (int m = 0; m < npt; ++m) {
#pragma unroll
    for (int c = 0; c < 12; ++c) g[m][c] = real(0);
#pragma unroll
    for (int c = 0; c < 5; ++c) Vs[m][c] = real(0);
  }
  if (active && (visc || SPLIT)) {
    // Lift_VolInt along the three computational directions.  Along xi and eta
    // a thread's nodes share the D-hat row; along zeta they share the line.
    // The split form's two-point fluxes ride on the same reads.
    real JG[npt][12];
#pragma unroll
    for (int m = 0; m < npt; ++m)
#pragma unroll
      for (int c = 0; c < 12; ++c) JG[m][c] = real(0);
    // own operands of the two-point flux (split form): rho, u, v, w, 4 p and 2 H
    real orho[npt], ou[npt], ov[npt], ow[npt], op4[npt], oH2[npt];
    const real R4 = v.Rgas4, cp2R = v.cpR2;
    if constexpr (SPLIT) {
#pragma unroll
      for (int m = 0; m < npt; ++m) {
        const int am = a + m * tpe;
        orho[m] = sm[L::Rho + am];
        ou[m] = sm[L::V + am];
        ov[m] = sm[L::V + n3 + am];
        ow[m] = sm[L::V + 2 * n3 + am];
        const real T = sm[L::V + 3 * n3 + am];
        op4[m] = orho[m] * (R4 * T);
        oH2[m] = cp2R * T + (ou[m] * ou[m] + ov[m] * ov[m] + ow[m] * ow[m]);
      }
    }
#pragma unroll
    for (int ci = 0; ci < 3; ++ci) {
      const real *Jr = sm + L::J + 3 * ci * n3;
      real oJ[npt][3];  // own metric vector Ja^ci (split form)
      if constexpr (SPLIT) {
#pragma unroll
        for (int m = 0; m < npt; ++m)
#pragma unroll
          for (int d = 0; d < 3; ++d) oJ[m][d] = Jr[d * n3 + a + m * tpe];
      }
      if constexpr (!SPLIT) {
#pragma unroll L::lift_unroll
      for (int al = 0; al < n; ++al) {
        if (ci < 2) {
          const real dh = sb.Dh[(ci == 0 ? i : j) * (n + 1) + al];
#pragma unroll
          for (int m = 0; m < npt; ++m) {
            const int km = k0 + m * kstep;
            const int src = ci == 0 ? vnode(n, al, j, km) : vnode(n, i, al, km);
            const real dj[3] = {dh * Jr[src], dh * Jr[n3 + src], dh * Jr[2 * n3 + src]};
            const real vv[4] = {sm[L::V + src], sm[L::V + n3 + src], sm[L::V + 2 * n3 + src],
                                sm[L::V + 3 * n3 + src]};
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
              for (int s = 0; s < 4; ++s) JG[m][d * 4 + s] += dj[d] * vv[s];
          }
        } else {
          const int src = vnode(n, i, j, al);
          const real jr[3] = {Jr[src], Jr[n3 + src], Jr[2 * n3 + src]};
          const real vv[4] = {sm[L::V + src], sm[L::V + n3 + src], sm[L::V + 2 * n3 + src], sm[L::V + 3 * n3 + src]};
#pragma unroll
          for (int m = 0; m < npt; ++m) {
            const real dh = plane_waves ? dk[m][al] : sb.Dh[(k0 + m * kstep) * (n + 1) + al];
            const real dj[3] = {dh * jr[0], dh * jr[1], dh * jr[2]};
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
              for (int s = 0; s < 4; ++s) JG[m][d * 4 + s] += dj[d] * vv[s];
          }
        }
      }
      } else {
      // one source node of node m's line: lifting sums and the split form's two-point flux
      auto take = [&](int m, int idx, int al, int src, const real *jr, const real *vv, real dh) {
        if (visc) {
          // D-hat times the metric first: 3 products and 12 multiply-adds per source node
          const real dj[3] = {dh * jr[0], dh * jr[1], dh * jr[2]};
#pragma unroll
          for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int s = 0; s < 4; ++s) JG[m][d * 4 + s] += dj[d] * vv[s];
        }
        if constexpr (SPLIT) {
          const real rs = sm[L::Rho + src];
          const real ps4 = rs * (R4 * vv[3]);
          const real Hs2 = cp2R * vv[3] + (vv[0] * vv[0] + vv[1] * vv[1] + vv[2] * vv[2]);
          real G[5];
          two_point_kep_sums(orho[m] + rs, ou[m] + vv[0], ov[m] + vv[1], ow[m] + vv[2], op4[m] + ps4, oH2[m] + Hs2,
                             oJ[m][0] + jr[0], oJ[m][1] + jr[1], oJ[m][2] + jr[2], G);
          const real ds = sDs[idx * (n + 1) + al];  // (D + D-hat)/16
#pragma unroll
          for (int c = 0; c < 5; ++c) Vs[m][c] += ds * G[c];
        }
      };
#pragma unroll L::lift_unroll
      for (int al = 0; al < n; ++al) {
        if (ci < 2) {
          const real dh = sb.Dh[(ci == 0 ? i : j) * (n + 1) + al];
#pragma unroll
          for (int m = 0; m < npt; ++m) {
            const int km = k0 + m * kstep;
            const int src = ci == 0 ? vnode(n, al, j, km) : vnode(n, i, al, km);
            const real jr[3] = {Jr[src], Jr[n3 + src], Jr[2 * n3 + src]};
            const real vv[4] = {sm[L::V + src], sm[L::V + n3 + src], sm[L::V + 2 * n3 + src],
                                sm[L::V + 3 * n3 + src]};
            take(m, ci == 0 ? i : j, al, src, jr, vv, dh);
          }
        } else {
          const int src = vnode(n, i, j, al);
          const real jr[3] = {Jr[src], Jr[n3 + src], Jr[2 * n3 + src]};
          const real vv[4] = {sm[L::V + src], sm[L::V + n3 + src], sm[L::V + 2 * n3 + src], sm[L::V + 3 * n3 + src]};
#pragma unroll
          for (int m = 0; m < npt; ++m) {
            const int km = k0 + m * kstep;
            const real dh = plane_waves ? dk[m][al] : sb.Dh[km * (n + 1) + al];
            take(m, km, al, src, jr, vv, dh);
          }
        }
      }
      }
    }
    if (visc) {
      // Lift_SurfInt: the face average times n shat, through l-hat
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        const int d = f >> 1;
        const int end = (f & 1) ? n - 1 : 0;  // the only node with nonzero l-hat at Gauss-Lobatto nodes
        if (d < 2) {
          if (LGL && (d == 0 ? i : j) != end) continue;
          const real lh = (f & 1) ? sb.lhp[d == 0 ? i : j] : sb.lhm[d == 0 ? i : j];
#pragma unroll
          for (int m = 0; m < npt; ++m) {
            const int km = k0 + m * kstep;
            const int fn = f * n2 + (d == 0 ? j : i) + n * km;
            const real av[4] = {sm[L::Avg + fn], sm[L::Avg + nf + fn], sm[L::Avg + 2 * nf + fn],
                                sm[L::Avg + 3 * nf + fn]};
#pragma unroll
            for (int dd = 0; dd < 3; ++dd) {
              const real nl = sm[L::Ns + dd * nf + fn] * lh;
#pragma unroll
              for (int s = 0; s < 4; ++s) JG[m][dd * 4 + s] += av[s] * nl;
            }
          }
        } else {
          const int fn = f * n2 + i + n * j;
          const real av[4] = {sm[L::Avg + fn], sm[L::Avg + nf + fn], sm[L::Avg + 2 * nf + fn], sm[L::Avg + 3 * nf + fn]};
          const real ns[3] = {sm[L::Ns + fn], sm[L::Ns + nf + fn], sm[L::Ns + 2 * nf + fn]};
#pragma unroll
          for (int m = 0; m < npt; ++m) {
            const int km = k0 + m * kstep;
            if (LGL && km != end) continue;
            const real lh = (f & 1) ? sb.lhp[km] : sb.lhm[km];
#pragma unroll
            for (int dd = 0; dd < 3; ++dd) {
              const real nl = ns[dd] * lh;
#pragma unroll
              for (int s = 0; s < 4; ++s) JG[m][dd * 4 + s] += av[s] * nl;
            }
          }
        }
      }
#pragma unroll
      for (int m = 0; m < npt; ++m) {
#pragma unroll
        for (int c = 0; c < 12; ++c) g[m][c] = JG[m][c] * iJe[m];
      }
    }
  }
  // dissipation sums of Sec. 5.2 at this thread's nodes: w J mu |curl u|^2 and w J mu (div u)^2
  double dS = 0.0, dD = 0.0, dW = 0.0;
  if (DIAG && active && visc) {
    const BasisOffsets o(n);
    const real *wq = v.basis + o.w;
#pragma unroll
    for (int m = 0; m < npt; ++m) {
      const real *gm = g[m];
      const double T = (double)sm[L::V + 3 * n3 + a + m * tpe];
      const double mud = v.visc_law ? sutherland<double>(T, (double)mu, (double)v.rTref) : (double)mu;
      const double wJ = (double)wq[i] * (double)wq[j] * (double)wq[k0 + m * kstep] / (double)v.invJ[vi + m * tpe];
      const double wx = (double)gm[1 * 4 + 2] - (double)gm[2 * 4 + 1];
      const double wy = (double)gm[2 * 4 + 0] - (double)gm[0 * 4 + 2];
      const double wz = (double)gm[0 * 4 + 1] - (double)gm[1 * 4 + 0];
      const double dv = (double)gm[0] + (double)gm[5] + (double)gm[10];
      dS += wJ * mud * (wx * wx + wy * wy + wz * wz);
      dD += wJ * mud * dv * dv;
      dW += wJ;
    }
  }
  if (active) {
    // volume fluxes at each node, projected on the three contravariant directions
#pragma unroll
    for (int m = 0; m < npt; ++m) {
      const int am = a + m * tpe;
      real P[6];
      cons2prim(U[m], gam, rR, P, bg);
      real Fx[5], Fy[5], Fz[5];
      if constexpr (SPLIT) {
#pragma unroll
        for (int c = 0; c < 5; ++c) Fx[c] = Fy[c] = Fz[c] = real(0);
      } else {
        flux_adv<0>(U[m], P, Fx, bg);
        flux_adv<1>(U[m], P, Fy, bg);
        flux_adv<2>(U[m], P, Fz, bg);
      }
      if (visc) {
        const real lamn = suth ? mun[m] * v.kappa : lam;
        real Vx[5], Vy[5], Vz[5];
        flux_visc<0>(P, g[m], mun[m], lamn, Vx);
        flux_visc<1>(P, g[m], mun[m], lamn, Vy);
        flux_visc<2>(P, g[m], mun[m], lamn, Vz);
#pragma unroll
        for (int c = 0; c < 5; ++c) {
          Fx[c] -= Vx[c];
          Fy[c] -= Vy[c];
          Fz[c] -= Vz[c];
        }
      }
#pragma unroll
      for (int ci = 0; ci < 3; ++ci) {
        const real j0 = sm[L::J + (3 * ci) * n3 + am], j1 = sm[L::J + (3 * ci + 1) * n3 + am],
                   j2 = sm[L::J + (3 * ci + 2) * n3 + am];
#pragma unroll
        for (int c = 0; c < 5; ++c) Fc[m][5 * ci + c] = j0 * Fx[c] + j1 * Fy[c] + j2 * Fz[c];
      }
    }
  }
  __syncthreads();  // the rows read above are covered by g below
  if (active && visc) {
#pragma unroll
    for (int m = 0; m < npt; ++m) {
      const int pa = Pad<n>::at(i, j, k0 + m * kstep);
#pragma unroll
      for (int c = 0; c < 12; ++c) sm[L::G + c * L::gsz + pa] = g[m][c];
    }
  }
  __syncthreads();
  if (active && visc) {
    // Lift_ProlongToFace of g, then this side's viscous normal flux
#pragma unroll
    for (int r = 0; r < L::upt; ++r) {
      const int t = a + r * tpe;
      if (t < L::units) {
        int d, s0, pq;
        face_unit<n, L::fpu, plane_waves>(t, d, s0, pq);
        int base, stride;
        Pad<n>::face_line(2 * d, pq, base, stride);
        // l(-1) and l(+1) weights: scalar loads where the face is the same on
        // every lane
        const BasisOffsets o(n);
        const real *lw[L::fpu];
#pragma unroll
        for (int u = 0; u < L::fpu; ++u) {
          const bool plus = (s0 + u) != 0;
          lw[u] = plane_waves ? v.basis + (plus ? o.lp : o.lm) : (plus ? sb.lp : sb.lm);
        }
        real gt[L::fpu][12];
#pragma unroll
        for (int u = 0; u < L::fpu; ++u)
#pragma unroll
          for (int s = 0; s < 12; ++s) gt[u][s] = real(0);
        if constexpr (LGL) {
          // Gauss-Lobatto: the trace is the end node of the line
#pragma unroll
          for (int u = 0; u < L::fpu; ++u) {
            const real *row = sm + L::G + base + ((s0 + u) != 0 ? (n - 1) * stride : 0);
#pragma unroll
            for (int s = 0; s < 12; ++s) gt[u][s] = row[s * L::gsz];
          }
        } else {
#pragma unroll
          for (int l = 0; l < n; ++l) {
            real w[L::fpu];
#pragma unroll
            for (int u = 0; u < L::fpu; ++u) w[u] = lw[u][l];
            const real *row = sm + L::G + base + l * stride;
#pragma unroll
            for (int s = 0; s < 12; ++s) {
              const real gv = row[s * L::gsz];
#pragma unroll
              for (int u = 0; u < L::fpu; ++u) gt[u][s] += w[u] * gv;
            }
          }
        }
#pragma unroll
        for (int u = 0; u < L::fpu; ++u) {
          const int f = 2 * d + s0 + u, fn = f * n2 + pq;
          const bool primary = prim[r][u];
          real nsv[3];
#pragma unroll
          for (int dd = 0; dd < 3; ++dd) {
            const real ns = sm[L::Ns + dd * nf + fn];
            nsv[dd] = primary ? ns : -ns;
          }
          const real ish = real(1) / sqrt(nsv[0] * nsv[0] + nsv[1] * nsv[1] + nsv[2] * nsv[2]);
          const real nv[3] = {nsv[0] * ish, nsv[1] * ish, nsv[2] * ish};
          const real Pf[6] = {real(0), pf[r][u][0], pf[r][u][1], pf[r][u][2], real(0), real(0)};
          const real muf = pf[r][u][3];
          const real lamf = suth ? muf * v.kappa : lam;
          real H[5] = {0, 0, 0, 0, 0}, tmp[5];
          flux_visc<0>(Pf, gt[u], muf, lamf, tmp);
#pragma unroll
          for (int s = 0; s < 5; ++s) H[s] += tmp[s] * nv[0];
          flux_visc<1>(Pf, gt[u], muf, lamf, tmp);
#pragma unroll
          for (int s = 0; s < 5; ++s) H[s] += tmp[s] * nv[1];
          flux_visc<2>(Pf, gt[u], muf, lamf, tmp);
#pragma unroll
          for (int s = 0; s < 5; ++s) H[s] += tmp[s] * nv[2];
#pragma unroll
          for (int s = 1; s < 5; ++s) st<NT>(H[s], v.Hv + (s - 1) * Ef + fb + fn);
        }
      }
    }
  }
  __syncthreads();  // g and n shat are read above; the flux rows below cover them
  // VolInt: the fluxes of all three directions at once (split form: the
  // viscous fluxes; without viscosity there is nothing left to contract)
  const bool contract = !SPLIT || visc;
  // the viscous fluxes have no mass component: the split form contracts four
  constexpr int c0 = SPLIT ? 1 : 0;
  if (active && contract) {
#pragma unroll
    for (int m = 0; m < npt; ++m)
#pragma unroll
      for (int c = 0; c < 15; ++c)
        if (c % 5 >= c0) sm[L::F + c * n3 + a + m * tpe] = Fc[m][c];
  }
  __syncthreads();
  if (active) {
    real Vi[npt][5];
#pragma unroll
    for (int m = 0; m < npt; ++m)
#pragma unroll
      for (int c = 0; c < 5; ++c) Vi[m][c] = real(0);
    if (contract && L::mfma) {
      // xi and eta on the FP64 4x4x4 four-block matrix instruction.  Its
      // operands sit at A[m][k]: lane 16k + 4b + m, B[k][n]: lane 16k + 4b + n,
      // and its result at D[m][n]: lane 16m + 4b + n.  A wave holds one
      // k-plane (with column pairs also the plane n/2 above) with node (i, j)
      // on lane i + 8j, so taking i = n + 4 (b & 1) and
      // j = (b >> 1) + 2m as the output indices puts every result in the lane
      // that owns the node.  xi: A = fluxes (row j, source l), B = D-hat^T;
      // eta: A = D-hat (row j), B = fluxes (column i, source l); sources in
      // two halves of four.  Each lane reads each flux value it feeds once.
      const int lane = threadIdx.x & 63, lk = lane >> 4;
      const int ix = lane & 7, jx = ((lane >> 3) & 1) + 2 * (lane & 3);
      double bx[2], ay[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        bx[h] = sb.Dh[ix * (n + 1) + 4 * h + lk];
        ay[h] = sb.Dh[jx * (n + 1) + 4 * h + lk];
      }
#pragma unroll
      for (int m = 0; m < npt; ++m) {
        const int km = k0 + m * kstep;
#pragma unroll
        for (int c = c0; c < 5; ++c) {
          double acc = 0.0;
#pragma unroll
          for (int h = 0; h < 2; ++h)
            acc = __builtin_amdgcn_mfma_f64_4x4x4f64(sm[L::F + c * n3 + vnode(n, 4 * h + lk, jx, km)], bx[h], acc, 0,
                                                     0, 0);
#pragma unroll
          for (int h = 0; h < 2; ++h)
            acc = __builtin_amdgcn_mfma_f64_4x4x4f64(ay[h], sm[L::F + (5 + c) * n3 + vnode(n, ix, 4 * h + lk, km)],
                                                     acc, 0, 0, 0);
          Vi[m][c] = acc;
        }
      }
      // zeta along the thread's own column
#pragma unroll
      for (int alp = 0; alp < n; ++alp) {
        const int src = vnode(n, i, j, alp);
        real fz[5];
#pragma unroll
        for (int c = c0; c < 5; ++c) fz[c] = sm[L::F + (10 + c) * n3 + src];
#pragma unroll
        for (int m = 0; m < npt; ++m) {
          const real dh = plane_waves ? dk[m][alp] : sb.Dh[(k0 + m * kstep) * (n + 1) + alp];
#pragma unroll
          for (int c = c0; c < 5; ++c) Vi[m][c] += dh * fz[c];
        }
      }
    } else if (contract) {
#pragma unroll
      for (int ci = 0; ci < 3; ++ci) {
#pragma unroll
        for (int alp = 0; alp < n; ++alp) {
          if (ci < 2) {
            const real dh = sb.Dh[(ci == 0 ? i : j) * (n + 1) + alp];
#pragma unroll
            for (int m = 0; m < npt; ++m) {
              const int km = k0 + m * kstep;
              const int src = ci == 0 ? vnode(n, alp, j, km) : vnode(n, i, alp, km);
#pragma unroll
              for (int c = c0; c < 5; ++c) Vi[m][c] += dh * sm[L::F + (5 * ci + c) * n3 + src];
            }
          } else {
            const int src = vnode(n, i, j, alp);
            real fz[5];
#pragma unroll
            for (int c = c0; c < 5; ++c) fz[c] = sm[L::F + (10 + c) * n3 + src];
#pragma unroll
            for (int m = 0; m < npt; ++m) {
              const real dh = plane_waves ? dk[m][alp] : sb.Dh[(k0 + m * kstep) * (n + 1) + alp];
#pragma unroll
              for (int c = c0; c < 5; ++c) Vi[m][c] += dh * fz[c];
            }
          }
        }
      }
    }
    if constexpr (SPLIT) {
      // the two-point sums carry 8 F_0, 16 F_1..3 and 32 F_4 against weights /16
#pragma unroll
      for (int m = 0; m < npt; ++m) {
        Vs[m][0] *= real(2);
        Vs[m][4] *= real(0.5);
      }
    }
#pragma unroll
    for (int m = 0; m < npt; ++m)
#pragma unroll
      for (int c = 0; c < 5; ++c)
        st<NT>(SPLIT ? Vs[m][c] + Vi[m][c] : Vi[m][c], v.Vol + c * Ev + vi + m * tpe);
  }
  if constexpr (DIAG) {
    // the element's dissipation sums in a fixed order (reproducible, no atomics)
    __syncthreads();
    // 3 tpe doubles per element fit its rows at every degree and precision
    double *sd = (double *)&sA[0][0] + (le < epb ? le : 0) * 3 * tpe;
    if (active) {
      sd[a] = dS;
      sd[tpe + a] = dD;
      sd[2 * tpe + a] = dW;
    }
    __syncthreads();
    if (active && a == 0) {
      double s0 = 0.0, s1 = 0.0, s2 = 0.0;
      for (int t = 0; t < tpe; ++t) {
        s0 += sd[t];
        s1 += sd[tpe + t];
        s2 += sd[2 * tpe + t];
      }
      v.diag[3 * e] = s0;
      v.diag[3 * e + 1] = s1;
      v.diag[3 * e + 2] = s2;
    }
  }
}

// ---------------------------------------------------------------------------
// Surface sweep of one workgroup of elements: FillFlux from this side's
// recomputed U trace, the neighbour's stored one and the mean of both sides'
// H; SurfInt gather, ApplyJac, the stage update (mode 0) or R (mode 1), and
// the next U traces.  SH = 1 (shock capturing, first pass) also forms the
// blending factors and hands a workgroup with a blended element to the blend
// pass; SH = 2 (the blend pass) adds the FV subcell operator, and with SPLIT
// takes the split form's advective volume integral for the blend.
// ---------------------------------------------------------------------------
template <int N, typename real, int SH, bool LGL, bool SPLIT = false, bool NT = false>
__device__ __forceinline__ void surface_body(const View<real> &v, const int lblk, const int mode) {
  using S = Sz<N>;
  constexpr int n = S::n, n2 = S::n2, n3 = S::n3, nf = S::nf, epb = S::epb;
  constexpr bool SHOCK = SH != 0, FV = SH == 2;
  __shared__ Smem<N, real> sb;
  __shared__ real sB[epb][5][Pad<n>::size];
  __shared__ real sS[epb][5][nf];
  // the blend pass: 16 rows per element for the subcell operator and the
  // advective volume integral, the 1-D operators of the subcells
  __shared__ real sX[FV ? epb * 16 * n3 : 1];
  __shared__ real sFV[FV ? (n * n + 3 * n + 1) : 1];  // D, w, x, xhalf
  __shared__ real sAl[epb];
  load_basis<N, real>(sb, v.basis);
  // the first pass clears the count of the next sweep (which alternates
  // entries, so no pass reads a count that another pass clears)
  if (SH == 1 && lblk == 0 && threadIdx.x == 0) v.bcnt[1 - v.bpar] = 0;
  if constexpr (FV) {
    const BasisOffsets o(n);
    for (int t = threadIdx.x; t < n * n; t += blockDim.x) sFV[t] = v.basis[o.D + t];
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
      sFV[n * n + t] = v.basis[o.w + t];
      sFV[n * n + n + t] = v.basis[o.x + t];
    }
    for (int t = threadIdx.x; t < n + 1; t += blockDim.x) sFV[n * n + 2 * n + t] = v.basis[o.xhalf + t];
  }
  const int le = threadIdx.x / n3, a = threadIdx.x - le * n3;
  const int64_t e = (int64_t)lblk * epb + le;
  const bool active = le < epb && e < v.E;
  const int64_t Ev = v.E * n3, Ef = v.E * 6 * n2;
  const uint32_t vi = (uint32_t)(e * n3 + a), fb = (uint32_t)(e * 6 * n2);
  const real gam = v.gamma, rR = v.rRgas;
  const Bg<real> bg{v.bg_p, v.bg_H};
  const bool visc = v.viscous != 0;  // the same for the whole grid
  const real *tr = v.cur ? v.Utr1 : v.Utr0;
  const int i = a % n, j = (a / n) % n, k = a / n2;
  constexpr bool plane_waves = n2 == 64 && epb == 1;  // a wave is one face of one element
  real *const su = &sB[le < epb ? le : 0][0][0];
  const int pa = Pad<n>::at(i, j, k);
  // the state, in LDS for this element's own traces and for the update.  The
  // FP64 copy is exact, so it is read back after the face phase instead of
  // being held in registers through it (they would spill); the mixed form
  // keeps the FP64 values, and so does the blend pass, whose occupancy its
  // LDS sets.
  constexpr bool exact_lds = sizeof(real) == sizeof(double) && !FV;
  double Uold[5] = {0, 0, 0, 0, 0};
  if (active) {
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      Uold[c] = ld<NT>(v.U + c * Ev + vi);
      su[c * Pad<n>::size + pa] = to_real(Uold[c], c, v);
    }
  }
  if (SHOCK && le < epb && a == 0) {
    // blending factor: frozen, or the element's own indicator value, an
    // operator local to the element (Sec. 2.3); with alpha_smooth raised to
    // half of its face neighbours' values, then clipped again.  Zero past the
    // last element.
    real a0 = real(0);
    if (active) {
      if (v.alpha_in) {
        a0 = v.alpha_in[e];
      } else {
        a0 = v.alpha_raw[e];
        if (v.alpha_smooth) {
#pragma unroll
          for (int f = 0; f < 6; ++f) a0 = fmax(a0, real(0.5) * v.alpha_raw[v.conn[e * 6 + f].x / 6]);
          if (a0 < v.alpha_min) a0 = real(0);
          a0 = fmin(a0, v.alpha_max);
        }
      }
    }
    sAl[le] = a0;
  }
  __syncthreads();
  real al = real(0);
  bool any = false;  // some element of the workgroup is blended
  if constexpr (SHOCK) {
#pragma unroll
    for (int q = 0; q < epb; ++q) any = any || sAl[q] > real(0);
    if (active) {
      al = sAl[le];
      if (a == 0) v.alpha[e] = al;
    }
    if constexpr (SH == 1) {
      // a workgroup with a blended element is left to the blend pass
      if (any) {
        if (threadIdx.x == 0) v.blist[atomicAdd(v.bcnt + v.bpar, 1)] = lblk;
        return;
      }
    }
  }
  if (active) {
    // FillFlux: Riemann flux of the U traces minus the mean of both sides' H.
    // This side's trace is recomputed from the state (the same bits as the
    // stored one); the neighbour's is read.
    for (int fn = a; fn < nf; fn += n3) {
      int f = fn / n2;
      if constexpr (plane_waves) f = __builtin_amdgcn_readfirstlane(f);
      const int pq = fn - f * n2, p = pq % n, q = pq / n;
      const int2 c = v.conn[e * 6 + f];
      const bool primary = (c.y >> 3) & 1;
      int pp, qq;
      orient_map(c.y & 7, p, q, N, pp, qq);
      const uint32_t io = fb + fn, in = (uint32_t)c.x * n2 + pp + n * qq;
      const uint32_t im = primary ? io : in, is = primary ? in : io;
      real Uo[5], Un[5];
      {
        int base, stride;
        Pad<n>::face_line(f, pq, base, stride);
        face_state<n, LGL>(su, (f & 1) ? sb.lp : sb.lm, base, stride, f & 1, Uo);
      }
#pragma unroll
      for (int s = 0; s < 5; ++s) Un[s] = (tr + s * Ef)[in];
      real Um[5], Us[5], Pm[6], Ps[6];
#pragma unroll
      for (int s = 0; s < 5; ++s) {
        Um[s] = primary ? Uo[s] : Un[s];
        Us[s] = primary ? Un[s] : Uo[s];
      }
      cons2prim(Um, gam, rR, Pm, bg);
      cons2prim(Us, gam, rR, Ps, bg);
      real nsv[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const real ns = (v.NS + d * Ef)[io];
        nsv[d] = primary ? ns : -ns;
      }
      const real sh = sqrt(nsv[0] * nsv[0] + nsv[1] * nsv[1] + nsv[2] * nsv[2]);
      const real nv[3] = {nsv[0] / sh, nsv[1] / sh, nsv[2] / sh};
      real Fs[5];
      if (v.riemann == 1) riemann_roe(Um, Pm, Us, Ps, nv, gam, Fs, bg);
      else riemann_llf(Um, Pm, Us, Ps, nv, gam, Fs, bg);
      if (visc) {
#pragma unroll
        for (int s = 1; s < 5; ++s) Fs[s] -= real(0.5) * ((v.Hv + (s - 1) * Ef)[im] + (v.Hv + (s - 1) * Ef)[is]);
      }
#pragma unroll
      for (int s = 0; s < 5; ++s) sS[le][s][fn] = primary ? Fs[s] * sh : -(Fs[s] * sh);
    }
  }
  __syncthreads();
  if constexpr (exact_lds) {
    if (active) {
#pragma unroll
      for (int c = 0; c < 5; ++c) Uold[c] = su[c * Pad<n>::size + pa];
    }
  }
  // blended elements: alpha (V_FV - V_adv) joins the stored volume integral,
  // i.e. (1 - alpha) V_adv + alpha V_FV + V_visc
  real Vb[5] = {0, 0, 0, 0, 0};
  if constexpr (FV) {
    if (any) {  // the same on every thread of the workgroup
      real *rows = sX + (le < epb ? le : 0) * 16 * n3;
      real U[5], P[6], Ja[9];
      if (active) {
#pragma unroll
        for (int c = 0; c < 5; ++c) U[c] = to_real(Uold[c], c, v);
        cons2prim(U, gam, rR, P, bg);
#pragma unroll
        for (int c = 0; c < 9; ++c) Ja[c] = (v.Ja + c * Ev)[vi];
      }
      real Vfv[5] = {0, 0, 0, 0, 0};
      fv_subcells<N, real>(rows, sFV, active, a, i, j, k, P, Ja, gam, rR, bg, Vfv);
      if constexpr (SPLIT) {
        // the split form's advective volume integral: two-point fluxes of
        // the primitives (rows 0-4, still those of the subcell pass), the
        // metric rows (5-13) and the specific total enthalpy (14)
        if (active) {
#pragma unroll
          for (int c = 0; c < 9; ++c) rows[(5 + c) * n3 + a] = Ja[c];
          rows[14 * n3 + a] = (U[4] + P[4]) / P[0];
        }
        __syncthreads();
      } else {
        // the advective DG volume integral, the three directions at once
        if (active) {
          real Fx[5], Fy[5], Fz[5];
          flux_adv<0>(U, P, Fx, bg);
          flux_adv<1>(U, P, Fy, bg);
          flux_adv<2>(U, P, Fz, bg);
#pragma unroll
          for (int ci = 0; ci < 3; ++ci)
#pragma unroll
            for (int c = 0; c < 5; ++c)
              rows[(5 * ci + c) * n3 + a] = Ja[3 * ci + 0] * Fx[c] + Ja[3 * ci + 1] * Fy[c] + Ja[3 * ci + 2] * Fz[c];
        }
        __syncthreads();
      }
      if (active && al > real(0)) {
        real Va[5] = {0, 0, 0, 0, 0};
        const real Hn = SPLIT ? rows[14 * n3 + a] : real(0);
#pragma unroll
        for (int ci = 0; ci < 3; ++ci) {
          const int idx = ci == 0 ? i : (ci == 1 ? j : k);
#pragma unroll
          for (int alp = 0; alp < n; ++alp) {
            const int src = ci == 0 ? vnode(n, alp, j, k) : (ci == 1 ? vnode(n, i, alp, k) : vnode(n, i, j, alp));
            const real dh = sb.Dh[idx * (n + 1) + alp];
            if constexpr (SPLIT) {
              const real ds = sFV[idx * n + alp] + dh;  // D + D-hat
              real F[5];
              two_point_kep(P[0], P[1], P[2], P[3], P[4], Hn, rows[src], rows[n3 + src], rows[2 * n3 + src],
                            rows[3 * n3 + src], rows[4 * n3 + src], rows[14 * n3 + src],
                            real(0.5) * (Ja[3 * ci + 0] + rows[(5 + 3 * ci) * n3 + src]),
                            real(0.5) * (Ja[3 * ci + 1] + rows[(6 + 3 * ci) * n3 + src]),
                            real(0.5) * (Ja[3 * ci + 2] + rows[(7 + 3 * ci) * n3 + src]), F);
#pragma unroll
              for (int c = 0; c < 5; ++c) Va[c] += ds * F[c];
            } else {
#pragma unroll
              for (int c = 0; c < 5; ++c) Va[c] += dh * rows[(5 * ci + c) * n3 + src];
            }
          }
        }
#pragma unroll
        for (int c = 0; c < 5; ++c) Vb[c] = al * (Vfv[c] - Va[c]);
      }
    }
  }
  double Unew[5] = {0, 0, 0, 0, 0};
  if (active) {
    real V[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) V[c] = ld<NT>(v.Vol + c * Ev + vi) + Vb[c];
    // 1/J and the RK register, loaded with the volume integral: their latency
    // overlaps the gather, and the register's five loads precede its five
    // stores (which the compiler could not move them across)
    const real iJ = v.invJ[vi];
    double dUo[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) dUo[c] = (mode == 0 && v.rkA != 0.0) ? ld<NT>(v.dU + c * Ev + vi) : 0.0;
    // SurfInt gather (one writer per entry) and ApplyJac
    const int pqf[3] = {j + n * k, i + n * k, i + n * j};
    const int lf[3] = {i, j, k};
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      const int d = f >> 1;
      // at Gauss-Lobatto nodes l-hat vanishes off the end node of the line
      const real lh = (f & 1) ? sb.lhp[lf[d]] : sb.lhm[lf[d]];
#pragma unroll
      for (int c = 0; c < 5; ++c) V[c] += sS[le][c][f * n2 + pqf[d]] * lh;
    }
    double R[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) R[c] = (double)(-(V[c] * iJ));
    if (v.source == 1) {
      const double x = v.Xs[vi], y = (v.Xs + Ev)[vi], z = (v.Xs + 2 * Ev)[vi];
      const double cs = 0.1 * M_PI * cos(M_PI * (x + y + z - v.t));
      const double gg = (double)gam;
      R[0] += 2.0 * cs;
      R[1] += 3.0 * cs;
      R[2] += 3.0 * cs;
      R[3] += 3.0 * cs;
      R[4] += 2.0 * (3.0 * gg - 2.0) / (gg - 1.0) * cs;
    }
    if (mode == 1) {
#pragma unroll
      for (int c = 0; c < 5; ++c) (v.R + c * Ev)[vi] = R[c];
    } else {
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        double *dUc = v.dU + c * Ev;
        // the first stage (A = 0) does not read the register: whatever it
        // holds (a restored state, an aborted step) cannot leak into the step
        const double du = (v.rkA != 0.0 ? v.rkA * dUo[c] : 0.0) + v.dt * R[c];
        st<NT>(du, dUc + vi);
        Unew[c] = Uold[c] + v.rkB * du;
        st<NT>(Unew[c], v.U + c * Ev + vi);
      }
    }
  }
  if (mode == 0) {
    // ProlongToFace of the updated state for the next stage
    // (every face-phase read of the old state is behind the barrier above)
    if (active) {
#pragma unroll
      for (int c = 0; c < 5; ++c) su[c * Pad<n>::size + pa] = to_real(Unew[c], c, v);
    }
    __syncthreads();
    if (active) {
      real *trn = v.cur ? v.Utr0 : v.Utr1;
      for (int fn = a; fn < nf; fn += n3) {
        int f = fn / n2;
        if constexpr (plane_waves) f = __builtin_amdgcn_readfirstlane(f);
        const int pq = fn - f * n2;
        int base, stride;
        Pad<n>::face_line(f, pq, base, stride);
        real t[5];
        face_state<n, LGL>(su, (f & 1) ? sb.lp : sb.lm, base, stride, f & 1, t);
#pragma unroll
        for (int c = 0; c < 5; ++c) st<NT>(t[c], trn + c * Ef + fb + fn);
      }
    }
  }
}


// Surface sweep: SH = 0 without shock capturing; SH = 1 with it, for the
// workgroups without a blended element (the others are listed for k_blend).
template <int N, typename real, int SH, bool LGL, bool NT>
__global__ void __launch_bounds__(Sz<N>::threads, Sz<N>::minw) k_surface(const View<real> *views, const int *blk_start,
                                                                          int nreq, View<real> single, int mode) {
  int lblk;
  const View<real> v = select_view(views, blk_start, nreq, single, lblk);
  surface_body<N, real, SH, LGL, false, NT>(v, lblk, mode);
}

// Blend pass: the surface sweep with the FV subcell blend, for the workgroups
// that k_surface<SH = 1> listed, request by request; a fixed grid strides over
// each list.  The compiler hoists the body's invariant work out of the loop
// and takes up to 256 VGPRs (one workgroup per SIMD); an out-of-line body
// needs half, but its call stack made every launch, empty ones included,
// 8 us slower, and the pass rarely has more than a few workgroups.
template <int N, typename real, bool LGL, bool SPLIT>
__global__ void __launch_bounds__(Sz<N>::threads, Sz<N>::minw) k_blend(const View<real> *views, int nreq,
                                                                        View<real> single, int mode) {
  const int nr = nreq == 0 ? 1 : nreq;
  for (int r = 0; r < nr; ++r) {
    const View<real> v = nreq == 0 ? single : rebase(views[r], single.base);
    const int cnt = v.bcnt[v.bpar];
    for (int idx = blockIdx.x; idx < cnt; idx += gridDim.x) {
      surface_body<N, real, 2, LGL, SPLIT>(v, v.blist[idx], mode);
      __syncthreads();  // LDS is reused by the next listed workgroup
    }
  }
}

// workgroups of the blend pass: one per CU
constexpr int kBlendBlocks = 256;

// the volume sweep with the viscosity law of the view (a template flag)
template <int N, typename real, bool SHOCK, bool LGL, bool SPLIT>
static void volume_sweep(dim3 grid, const View<real> *views, const int *blk_start, int nreq, const View<real> &v0,
                         hipStream_t st) {
  constexpr int threads = VolLds<N, real, SHOCK, SPLIT>::threads;
  if (v0.nt) {
    if (v0.visc_law)
      k_volume<N, real, SHOCK, LGL, SPLIT, true, false, true><<<grid, threads, 0, st>>>(views, blk_start, nreq, v0);
    else
      k_volume<N, real, SHOCK, LGL, SPLIT, false, false, true><<<grid, threads, 0, st>>>(views, blk_start, nreq, v0);
  } else {
    if (v0.visc_law)
      k_volume<N, real, SHOCK, LGL, SPLIT, true><<<grid, threads, 0, st>>>(views, blk_start, nreq, v0);
    else
      k_volume<N, real, SHOCK, LGL, SPLIT, false><<<grid, threads, 0, st>>>(views, blk_start, nreq, v0);
  }
}

template <int N, typename real, bool LGL>
static hipError_t launch_nl(Kernel k, int mode, const View<real> *views, const int *blk_start, int nreq, int blocks,
                           const View<real> &v0, hipStream_t st) {
  dim3 grid(blocks), block(Sz<N>::threads);
  switch (k) {
    case K_TRACE:
      k_trace<N, real, LGL><<<grid, block, 0, st>>>(views, blk_start, nreq, v0);
      break;
    case K_LIFT:
      // volume sweep: indicator (shock capturing), lifting (viscous), VolInt
      // (standard or split form)
      if (v0.split) {
        if constexpr (LGL) {  // the split form takes Gauss-Lobatto nodes only
          if (v0.shock) {
            if constexpr (N >= 2 && N <= 7) {  // the degrees shock capturing accepts
              volume_sweep<N, real, true, true, true>(grid, views, blk_start, nreq, v0, st);
            } else {
              return hipErrorInvalidValue;
            }
          } else {
            volume_sweep<N, real, false, true, true>(grid, views, blk_start, nreq, v0, st);
          }
        } else {
          return hipErrorInvalidValue;
        }
      } else if (v0.shock) {
        if constexpr (N >= 2 && N <= 7) {
          volume_sweep<N, real, true, LGL, false>(grid, views, blk_start, nreq, v0, st);
        } else {
          return hipErrorInvalidValue;
        }
      } else {
        volume_sweep<N, real, false, LGL, false>(grid, views, blk_start, nreq, v0, st);
      }
      break;
    case K_DIAG:
      // the lifting of the volume sweep with the dissipation sums; the
      // volume integral it also writes is a stage temporary
      k_volume<N, real, false, LGL, false, false, true>
          <<<grid, (VolLds<N, real, false, false>::threads), 0, st>>>(views, blk_start, nreq, v0);
      break;
    case K_RHS:
      // surface sweep (after a volume sweep), or the one-sweep Euler operator
      if (v0.shock) {
        if constexpr (N >= 2 && N <= 7) {  // the degrees shock capturing accepts
          if (v0.nt)
            k_surface<N, real, 1, LGL, true><<<grid, block, 0, st>>>(views, blk_start, nreq, v0, mode);
          else
            k_surface<N, real, 1, LGL, false><<<grid, block, 0, st>>>(views, blk_start, nreq, v0, mode);
          if (v0.split) {
            if constexpr (LGL) {
              k_blend<N, real, LGL, true><<<std::min(blocks, kBlendBlocks), block, 0, st>>>(views, nreq, v0, mode);
            } else {
              return hipErrorInvalidValue;
            }
          } else {
            k_blend<N, real, LGL, false><<<std::min(blocks, kBlendBlocks), block, 0, st>>>(views, nreq, v0, mode);
          }
        } else {
          return hipErrorInvalidValue;
        }
      } else if (v0.viscous || v0.split) {
        if (v0.nt)
          k_surface<N, real, 0, LGL, true><<<grid, block, 0, st>>>(views, blk_start, nreq, v0, mode);
        else
          k_surface<N, real, 0, LGL, false><<<grid, block, 0, st>>>(views, blk_start, nreq, v0, mode);
      } else {
        k_rhs<N, real><<<grid, block, 0, st>>>(views, blk_start, nreq, v0, mode);
      }
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Gauss-Lobatto nodes take their own instantiations (face values are end nodes)
template <int N, typename real>
hipError_t launch_n(Kernel k, int mode, const View<real> *views, const int *blk_start, int nreq, int blocks,
                           const View<real> &v0, hipStream_t st) {
  return v0.lgl ? launch_nl<N, real, true>(k, mode, views, blk_start, nreq, blocks, v0, st)
                : launch_nl<N, real, false>(k, mode, views, blk_start, nreq, blocks, v0, st);
}

}  // namespace dg
