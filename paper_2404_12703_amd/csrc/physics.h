// physics.h -- pointwise physics of the compressible Navier-Stokes equations
// for the HIP kernels: ConsToPrim, advective and viscous fluxes, Riemann
// solvers.  Paper (GALAEXI, arXiv 2404.12703): Sec. 2.1 Eqs. nse, eos_p, eos_T;
// Table tab:dg_routines (ConsToPrim, FillFlux); App. A (FillFlux).
#pragma once

#include <hip/hip_runtime.h>

namespace dg {

// The background pressure p_ref the mixed form takes out of its FP32
// arithmetic: the FP32 state carries rho e - p_ref/(gamma - 1), so ConsToPrim
// yields p - p_ref, which the momentum fluxes use as is (a constant pressure
// adds nothing to the discrete divergence: freestream preservation); the
// temperature, the sound speed and the enthalpy add it back.  p = bg.p,
// H = gamma p_ref/(gamma - 1) (the energy plus pressure of the background).
// FP64 ignores it.
template <typename real>
struct Bg {
  real p = real(0), H = real(0);
};
template <typename real>
__device__ __forceinline__ real full_p(real p, Bg<real> bg) {
  if constexpr (sizeof(real) == 4) return p + bg.p;
  else return p;
}
template <typename real>
__device__ __forceinline__ real full_E(real E, Bg<real> bg) {  // rho e + p with the background
  if constexpr (sizeof(real) == 4) return E + bg.H;
  else return E;
}

// prim = (rho, u, v, w, p, T) from U = (rho, rho u, rho v, rho w, rho e);
// rRgas = 1/R.  One reciprocal of rho replaces four divisions.  (Mixed form
// with a background: P[4] = p - p_ref, T from p.)
template <typename real>
__device__ __forceinline__ void cons2prim(const real *U, real gamma, real rRgas, real *P, Bg<real> bg = {}) {
  const real rho = U[0];
  const real ir = real(1) / rho;
  const real u = U[1] * ir, v = U[2] * ir, w = U[3] * ir;
  const real p = (gamma - real(1)) * (U[4] - real(0.5) * rho * (u * u + v * v + w * w));
  P[0] = rho;
  P[1] = u;
  P[2] = v;
  P[3] = w;
  P[4] = p;
  P[5] = full_p(p, bg) * (ir * rRgas);
}

// advective flux in Cartesian direction d (compile-time)
template <int d, typename real>
__device__ __forceinline__ void flux_adv(const real *U, const real *P, real *F, Bg<real> bg = {}) {
  const real ud = P[1 + d];
  F[0] = U[1 + d];
  F[1] = U[1] * ud;
  F[2] = U[2] * ud;
  F[3] = U[3] * ud;
  F[1 + d] += P[4];
  F[4] = full_E(U[4] + P[4], bg) * ud;
}

// viscous flux in direction d from primitives and lifted gradients
// g[dd*4 + var], var = (u, v, w, T): tau = mu (grad u + grad u^T - 2/3 div u I),
// energy: tau.u + lambda dT/dx_d.  Enters the total flux as F_adv - F_visc.
template <int d, typename real>
__device__ __forceinline__ void flux_visc(const real *P, const real *g, real mu, real lambda, real *F) {
  const real divu = g[0] + g[5] + g[10];
  real tau[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    tau[a] = mu * (g[d * 4 + a] + g[a * 4 + d]);
    if (a == d) tau[a] -= real(2.0 / 3.0) * mu * divu;
  }
  F[0] = real(0);
  F[1] = tau[0];
  F[2] = tau[1];
  F[3] = tau[2];
  F[4] = tau[0] * P[1] + tau[1] * P[2] + tau[2] * P[3] + lambda * g[d * 4 + 3];
}

// Sec. 2.1 Eq. sutherland: the viscosity at temperature T, normalised by the
// reference temperature: mu(T) = mu_ref 1.4042 th^(3/2) / (th + 0.4042), th = T/T_ref
template <typename real>
__host__ __device__ __forceinline__ real sutherland(real T, real mu_ref, real rTref) {
  const real th = T * rTref;
  return mu_ref * real(1.4042) * th * sqrt(th) / (th + real(0.4042));
}

// Sec. 2.2 "Nonlinear Stability": Pirozzoli's kinetic-energy-preserving
// two-point flux of the split form along the unnormalised direction m (the
// mean of the two nodes' metric vectors).  Arithmetic means of density,
// velocity, pressure and specific total enthalpy; the mass flux carries
// momentum and enthalpy.  Consistent (F#(U, U) = F(U).m) and symmetric.
template <typename real>
__device__ __forceinline__ void two_point_kep(real rL, real uL, real vL, real wL, real pL, real HL, real rR, real uR,
                                              real vR, real wR, real pR, real HR, real m0, real m1, real m2,
                                              real *F) {
  const real rho = real(0.5) * (rL + rR);
  const real u = real(0.5) * (uL + uR), v = real(0.5) * (vL + vR), w = real(0.5) * (wL + wR);
  const real p = real(0.5) * (pL + pR), H = real(0.5) * (HL + HR);
  const real mf = rho * (u * m0 + v * m1 + w * m2);
  F[0] = mf;
  F[1] = mf * u + p * m0;
  F[2] = mf * v + p * m1;
  F[3] = mf * w + p * m2;
  F[4] = mf * H;
}

// The same flux from sums instead of means, for the volume sweep's inner
// loop: with S_x = x_L + x_R, S_p4 = 4 (p_L + p_R), S_H2 = 2 (H_L + H_R) and
// s = Ja_L + Ja_R it returns G = (8 F_0, 16 F_1, 16 F_2, 16 F_3, 32 F_4).  Each
// halving of the means is a power of two, so G is F scaled exactly; the
// caller folds the factors into its weights.
template <typename real>
__device__ __forceinline__ void two_point_kep_sums(real Sr, real Su, real Sv, real Sw, real Sp4, real SH2, real s0,
                                                   real s1, real s2, real *G) {
  const real X = Sr * (Su * s0 + Sv * s1 + Sw * s2);
  G[0] = X;
  G[1] = X * Su + Sp4 * s0;
  G[2] = X * Sv + Sp4 * s1;
  G[3] = X * Sw + Sp4 * s2;
  G[4] = X * SH2;
}

template <typename real>
__device__ __forceinline__ void flux_normal(const real *U, const real *P, const real *nv, real *F, Bg<real> bg = {}) {
  real f[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) F[v] = real(0);
  flux_adv<0>(U, P, f, bg);
#pragma unroll
  for (int v = 0; v < 5; ++v) F[v] += f[v] * nv[0];
  flux_adv<1>(U, P, f, bg);
#pragma unroll
  for (int v = 0; v < 5; ++v) F[v] += f[v] * nv[1];
  flux_adv<2>(U, P, f, bg);
#pragma unroll
  for (int v = 0; v < 5; ++v) F[v] += f[v] * nv[2];
}

// local Lax-Friedrichs: 1/2 (F_L + F_R).n - 1/2 max(|u.n| + c) (U_R - U_L)
template <typename real>
__device__ __forceinline__ void riemann_llf(const real *UL, const real *PL, const real *UR, const real *PR,
                                            const real *nv, real gamma, real *F, Bg<real> bg = {}) {
  real FL[5], FR[5];
  flux_normal(UL, PL, nv, FL, bg);
  flux_normal(UR, PR, nv, FR, bg);
  const real cL = sqrt(gamma * full_p(PL[4], bg) / PL[0]), cR = sqrt(gamma * full_p(PR[4], bg) / PR[0]);
  const real unL = PL[1] * nv[0] + PL[2] * nv[1] + PL[3] * nv[2];
  const real unR = PR[1] * nv[0] + PR[2] * nv[1] + PR[3] * nv[2];
  const real lmax = fmax(fabs(unL) + cL, fabs(unR) + cR);
#pragma unroll
  for (int v = 0; v < 5; ++v) F[v] = real(0.5) * (FL[v] + FR[v]) - real(0.5) * lmax * (UR[v] - UL[v]);
}

// Roe's approximate Riemann solver without entropy fix: central flux minus
// half the sum over the five characteristic waves |lambda_k| a_k r_k at the
// Roe-averaged state.
template <typename real>
__device__ __forceinline__ void riemann_roe(const real *UL, const real *PL, const real *UR, const real *PR,
                                            const real *nv, real gamma, real *F, Bg<real> bg = {}) {
  real FL[5], FR[5];
  flux_normal(UL, PL, nv, FL, bg);
  flux_normal(UR, PR, nv, FR, bg);
  const real sL = sqrt(PL[0]), sR = sqrt(PR[0]);
  const real inv = real(1) / (sL + sR);
  const real HL = full_E(UL[4] + PL[4], bg) / PL[0], HR = full_E(UR[4] + PR[4], bg) / PR[0];
  real ut[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) ut[d] = (sL * PL[1 + d] + sR * PR[1 + d]) * inv;
  const real Ht = (sL * HL + sR * HR) * inv;
  const real q2 = ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2];
  const real c2 = (gamma - real(1)) * (Ht - real(0.5) * q2);
  const real ct = sqrt(c2);
  const real rt = sL * sR;
  const real un = ut[0] * nv[0] + ut[1] * nv[1] + ut[2] * nv[2];
  real du[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) du[d] = PR[1 + d] - PL[1 + d];
  const real dun = du[0] * nv[0] + du[1] * nv[1] + du[2] * nv[2];
  const real drho = PR[0] - PL[0], dp = PR[4] - PL[4];
  const real a1 = (dp - rt * ct * dun) / (real(2) * c2);
  const real a2 = drho - dp / c2;
  const real a3 = (dp + rt * ct * dun) / (real(2) * c2);
  const real l1 = fabs(un - ct) * a1, l2 = fabs(un) * a2, l3 = fabs(un + ct) * a3;
  const real ls = fabs(un) * rt;
  real dut[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) dut[d] = du[d] - dun * nv[d];
  const real udut = ut[0] * dut[0] + ut[1] * dut[1] + ut[2] * dut[2];
  real Dis[5];
  Dis[0] = l1 + l2 + l3;
#pragma unroll
  for (int d = 0; d < 3; ++d)
    Dis[1 + d] = l1 * (ut[d] - ct * nv[d]) + l2 * ut[d] + ls * dut[d] + l3 * (ut[d] + ct * nv[d]);
  Dis[4] = l1 * (Ht - un * ct) + l2 * real(0.5) * q2 + ls * udut + l3 * (Ht + un * ct);
#pragma unroll
  for (int v = 0; v < 5; ++v) F[v] = real(0.5) * (FL[v] + FR[v]) - real(0.5) * Dis[v];
}

}  // namespace dg
