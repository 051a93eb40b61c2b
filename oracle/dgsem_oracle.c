/*
 * dgsem_oracle.c -- plain, slow, FP64 CPU reference of the DGSEM time
 * derivative for the compressible Navier-Stokes equations and of the
 * low-storage Runge-Kutta update.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header, table or constant
 * generator with the HIP library; the two meet only through the seeded inputs.
 *
 * Paper: Kurz, Kempf et al., "GALAEXI: Solving complex compressible flows with
 * high-order discontinuous Galerkin methods on accelerator-based systems"
 * (arXiv 2404.12703).  Every routine below cites the passage it follows.
 *
 * Style: the operations are written in the order the paper lists them
 * (Sec. 2.2, Table "tab:dg_routines", App. A): ConsToPrim, ProlongToFace,
 * the Lift_* copies, FillFlux, VolInt, SurfInt (as the loop over faces of
 * Alg. "SurfInt (CPU)", primary side +f*, replica side -f*), ApplyJac.
 * No blocking, fusion or reordering.  Face-node correspondence is found
 * geometrically (coincident physical coordinates modulo the periodic box);
 * the orientation codes of the mesh are never read.
 *
 * Internal layout: arrays of structures, [elem][node][var], node index
 * i + n*(j + n*k) with i fastest.  The public state layout is [var][elem][node].
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* The basis and the metric terms are computed in extended precision (x87
 * long double) and rounded once to double. */
typedef long double xr;
#define XPI 3.141592653589793238462643383279502884L

#define NV 5  /* rho, rho u, rho v, rho w, rho e */
#define NL 4  /* lifted primitives u, v, w, T    */
/* position of lifted variable v in prim = (rho, u, v, w, p, T) */
static const int LIFT_IDX[NL] = {1, 2, 3, 5};

typedef struct orc {
  int N, n, n2, n3, node_type, ngeo;
  long E;
  double period[3];
  /* 1-D operators on the solution nodes (Sec. 2.2, Eq. dgsem) */
  double *x, *w, *D, *Dhat, *lm, *lp, *lhm, *lhp;
  xr *xL, *xgL, *DgL, *Mg2sL;  /* extended-precision copies for the set-up */
  /* geometry */
  double *XL;  /* [E][n3][3]  positions on LGL(N)                        */
  double *Xs;  /* [E][n3][3]  positions at the solution nodes             */
  double *Ja;  /* [E][n3][3][3]  Ja[..][i][d]: computational i, Cartesian d */
  double *J;   /* [E][n3] */
  double *nS;  /* [E][6][n2][3]  outward normal times surface element      */
  long *nbr;   /* [E][6] */
  int *nbrf;   /* [E][6] */
  int *fmap;   /* [E][6][n2]  node on the neighbour face coincident with (p,q) */
  /* parameters */
  double gamma, R, Pr, mu;
  int riemann, viscous, source, shock;
  double alpha_max, alpha_min, ind_a, ind_c, ind_s;
  int alpha_smooth;     /* 1: raise alpha to half the largest face neighbour's value */
  int volume_flux;      /* 0 standard weak form; 1 split form, Pirozzoli's two-point flux;
                           2 split form with the mean of the two fluxes (a pin only) */
  int visc_law;         /* 0 constant mu; 1 Sutherland's law, mu = mu(T_ref) */
  int rk_scheme;        /* 0 five-stage, 1 fourteen-stage low-storage RK */
  double T_ref;         /* Sutherland reference temperature */
  double *alpha;        /* [E] last blending factors */
  int alpha_frozen;     /* 1: use alpha[] as given instead of the indicator */
  double *Vinv;         /* [n][n] inverse orthonormal-Legendre Vandermonde */
  double *xhalf;        /* [n+1] subcell interface positions */
  /* work arrays sized at create time */
  double *Ui, *prim, *Uf, *primf, *G, *Gf, *V, *faceF, *liftF;
  double *Vadv, *Vvis, *Vfv;
  char err[256];
} orc;

/* ------------------------------------------------------------------------ */
/* Sec. 2.2 "Solution Representation": Legendre polynomials, Gauss and      */
/* Gauss-Lobatto nodes, Lagrange basis.                                     */
/* ------------------------------------------------------------------------ */


/* Legendre P_m(x) and P_m'(x) by the three-term recurrence. */
static void legendre(int m, xr x, xr *P, xr *dP) {
  xr p0 = 1.0L, p1 = x, d0 = 0.0L, d1 = 1.0L;
  if (m == 0) { *P = 1.0L; *dP = 0.0L; return; }
  for (int k = 2; k <= m; ++k) {
    xr p2 = ((2.0L * k - 1.0L) * x * p1 - (k - 1.0L) * p0) / k;
    xr d2 = d0 + (2.0L * k - 1.0L) * p1;
    p0 = p1; p1 = p2; d0 = d1; d1 = d2;
  }
  *P = p1; *dP = d1;
}

/* Legendre-Gauss nodes: roots of P_{N+1}; weights 2/((1-x^2) P'_{N+1}^2). */
static void gauss_nodes(int N, xr *x, xr *w) {
  int n = N + 1;
  for (int k = 0; k < n; ++k) {
    xr xk = -cosl((2.0L * k + 1.0L) * XPI / (2.0L * N + 2.0L));
    for (int it = 0; it < 100; ++it) {
      xr P, dP;
      legendre(n, xk, &P, &dP);
      xr dx = P / dP;
      xk -= dx;
      if (fabsl(dx) < 1e-19L) break;
    }
    xr P, dP;
    legendre(n, xk, &P, &dP);
    x[k] = xk;
    w[k] = 2.0L / ((1.0L - xk * xk) * dP * dP);
  }
}

/* Legendre-Gauss-Lobatto nodes: -1, roots of P_N', +1;
 * weights 2/(N(N+1) P_N^2).  P_N'' from the Legendre equation. */
static void lobatto_nodes(int N, xr *x, xr *w) {
  x[0] = -1.0L; x[N] = 1.0L;
  for (int k = 1; k < N; ++k) {
    xr xk = -cosl(XPI * k / N);
    for (int it = 0; it < 100; ++it) {
      xr P, dP;
      legendre(N, xk, &P, &dP);
      xr d2P = (2.0L * xk * dP - N * (N + 1.0L) * P) / (1.0L - xk * xk);
      xr dx = dP / d2P;
      xk -= dx;
      if (fabsl(dx) < 1e-19L) break;
    }
    x[k] = xk;
  }
  for (int k = 0; k <= N; ++k) {
    xr P, dP;
    legendre(N, x[k], &P, &dP);
    w[k] = 2.0L / (N * (N + 1.0L) * P * P);
  }
}

/* Lagrange polynomial l_j(s) = prod_{i != j} (s - x_i)/(x_j - x_i). */
static xr lagrange(int n, const xr *xn, int j, xr s) {
  xr r = 1.0L;
  for (int i = 0; i < n; ++i)
    if (i != j) r *= (s - xn[i]) / (xn[j] - xn[i]);
  return r;
}

/* D_ij = l_j'(x_i): for i != j from the derivative of the product formula
 * evaluated at a node, D_ii = -sum_{j != i} D_ij (exact for constants). */
static void diff_matrix(int n, const xr *xn, xr *D) {
  for (int i = 0; i < n; ++i) {
    xr s = 0.0L;
    for (int j = 0; j < n; ++j) {
      if (i == j) continue;
      /* l_j'(x_i) = prod_{k != j, k != i}(x_i - x_k) / prod_{k != j}(x_j - x_k) */
      xr num = 1.0L, den = 1.0L;
      for (int k = 0; k < n; ++k) {
        if (k != j && k != i) num *= (xn[i] - xn[k]);
        if (k != j) den *= (xn[j] - xn[k]);
      }
      D[i * n + j] = num / den;
      s += D[i * n + j];
    }
    D[i * n + i] = -s;
  }
}

/* M[b][a] = l_a(to_b): interpolation from nodes `from` to points `to`. */
static void interp_matrix(int n, const xr *from, int m, const xr *to, xr *M) {
  for (int b = 0; b < m; ++b)
    for (int a = 0; a < n; ++a) M[b * n + a] = lagrange(n, from, a, to[b]);
}

/* ------------------------------------------------------------------------ */
/* Tensor-product helpers on an n^3 block with c interleaved components.     */
/* ------------------------------------------------------------------------ */
static inline int nidx(int n, int i, int j, int k) { return i + n * (j + n * k); }

/* node index of the point with index l along direction d and face
 * coordinates (p,q) along the two other directions in increasing order */
static inline int line_node(int n, int d, int l, int p, int q) {
  if (d == 0) return nidx(n, l, p, q);
  if (d == 1) return nidx(n, p, l, q);
  return nidx(n, p, q, l);
}

/* out = (M (x) M (x) M) in : n^3 -> m^3 points, c components */
static void interp3(int n, int m, const double *M, const double *in, double *out, int c) {
  double *t1 = (double *)calloc((size_t)m * n * n * c, sizeof(double));
  double *t2 = (double *)calloc((size_t)m * m * n * c, sizeof(double));
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int a = 0; a < m; ++a)
        for (int v = 0; v < c; ++v) {
          double s = 0.0;
          for (int i = 0; i < n; ++i) s += M[a * n + i] * in[(i + n * (j + n * k)) * c + v];
          t1[(a + m * (j + n * k)) * c + v] = s;
        }
  for (int k = 0; k < n; ++k)
    for (int b = 0; b < m; ++b)
      for (int a = 0; a < m; ++a)
        for (int v = 0; v < c; ++v) {
          double s = 0.0;
          for (int j = 0; j < n; ++j) s += M[b * n + j] * t1[(a + m * (j + n * k)) * c + v];
          t2[(a + m * (b + m * k)) * c + v] = s;
        }
  for (int g = 0; g < m; ++g)
    for (int b = 0; b < m; ++b)
      for (int a = 0; a < m; ++a)
        for (int v = 0; v < c; ++v) {
          double s = 0.0;
          for (int k = 0; k < n; ++k) s += M[g * n + k] * t2[(a + m * (b + m * k)) * c + v];
          out[(a + m * (b + m * g)) * c + v] = s;
        }
  free(t1);
  free(t2);
}

/* derivative of scalar field f along computational direction d: (D f)_line */
static void deriv_dir(int n, const double *D, int d, const double *f, int fs, double *out, int os) {
  for (int q = 0; q < n; ++q)
    for (int p = 0; p < n; ++p)
      for (int l = 0; l < n; ++l) {
        double s = 0.0;
        for (int a = 0; a < n; ++a) s += D[l * n + a] * f[line_node(n, d, a, p, q) * fs];
        out[line_node(n, d, l, p, q) * os] = s;
      }
}

/* the same two helpers in extended precision, for the set-up */
static void interp3x(int n, int m, const xr *M, const xr *in, xr *out, int c) {
  xr *t1 = (xr *)calloc((size_t)m * n * n * c, sizeof(xr));
  xr *t2 = (xr *)calloc((size_t)m * m * n * c, sizeof(xr));
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int a = 0; a < m; ++a)
        for (int v = 0; v < c; ++v) {
          xr s = 0.0L;
          for (int i = 0; i < n; ++i) s += M[a * n + i] * in[(i + n * (j + n * k)) * c + v];
          t1[(a + m * (j + n * k)) * c + v] = s;
        }
  for (int k = 0; k < n; ++k)
    for (int b = 0; b < m; ++b)
      for (int a = 0; a < m; ++a)
        for (int v = 0; v < c; ++v) {
          xr s = 0.0L;
          for (int j = 0; j < n; ++j) s += M[b * n + j] * t1[(a + m * (j + n * k)) * c + v];
          t2[(a + m * (b + m * k)) * c + v] = s;
        }
  for (int g = 0; g < m; ++g)
    for (int b = 0; b < m; ++b)
      for (int a = 0; a < m; ++a)
        for (int v = 0; v < c; ++v) {
          xr s = 0.0L;
          for (int k = 0; k < n; ++k) s += M[g * n + k] * t2[(a + m * (b + m * k)) * c + v];
          out[(a + m * (b + m * g)) * c + v] = s;
        }
  free(t1);
  free(t2);
}

static void deriv_dirx(int n, const xr *D, int d, const xr *f, int fs, xr *out, int os) {
  for (int q = 0; q < n; ++q)
    for (int p = 0; p < n; ++p)
      for (int l = 0; l < n; ++l) {
        xr s = 0.0L;
        for (int a = 0; a < n; ++a) s += D[l * n + a] * f[line_node(n, d, a, p, q) * fs];
        out[line_node(n, d, l, p, q) * os] = s;
      }
}

/* ------------------------------------------------------------------------ */
/* Sec. 2.1: ConsToPrim (Eqs. eos_p, eos_T).  prim = (rho,u,v,w,p,T).       */
/* ------------------------------------------------------------------------ */
static void cons_to_prim(const orc *o, const double *U, double *P) {
  double rho = U[0];
  double u = U[1] / rho, v = U[2] / rho, w = U[3] / rho;
  double p = (o->gamma - 1.0) * (U[4] - 0.5 * rho * (u * u + v * v + w * w));
  P[0] = rho; P[1] = u; P[2] = v; P[3] = w; P[4] = p; P[5] = p / (rho * o->R);
}

static void prim_to_cons(const orc *o, const double *q /* rho,u,v,w,p */, double *U) {
  U[0] = q[0];
  U[1] = q[0] * q[1];
  U[2] = q[0] * q[2];
  U[3] = q[0] * q[3];
  U[4] = q[4] / (o->gamma - 1.0) + 0.5 * q[0] * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
}

/* Sec. 2.1 Eq. nse: advective flux in Cartesian direction d */
static void flux_adv(const double *U, const double *P, int d, double *F) {
  double ud = P[1 + d];
  F[0] = U[1 + d];
  F[1] = U[1] * ud;
  F[2] = U[2] * ud;
  F[3] = U[3] * ud;
  F[1 + d] += P[4];
  F[4] = (U[4] + P[4]) * ud;
}

/* Sec. 2.1, Eq. sutherland: the dynamic viscosity at temperature T.  The
 * paper writes Sutherland's law normalised by the reference temperature,
 * mu = mu_ref 1.4042 (T/T_ref)^(3/2) / (T/T_ref + 0.4042); without it the
 * viscosity is the constant mu. */
static double viscosity(const orc *o, double T) {
  if (o->visc_law == 0) return o->mu;
  double th = T / o->T_ref;
  return o->mu * 1.4042 * th * sqrt(th) / (th + 0.4042);
}

/* Sec. 2.1: viscous flux in direction d from the primitives and the lifted
 * gradients g[dd][var] (var: u,v,w,T).  tau = mu(grad u + grad u^T - 2/3 div u I),
 * q = -lambda grad T, lambda = gamma R mu / ((gamma-1) Pr), mu = mu(T).
 * Enters as F - Fv. */
static void flux_visc(const orc *o, const double *P, const double *g, int d, double *F) {
  double mu = viscosity(o, P[5]);
  double lam = o->gamma * o->R * mu / ((o->gamma - 1.0) * o->Pr);
  double divu = g[0 * NL + 0] + g[1 * NL + 1] + g[2 * NL + 2];
  double tau[3];
  for (int a = 0; a < 3; ++a) {
    /* tau_{a d} = mu (du_a/dx_d + du_d/dx_a) - 2/3 mu div u delta_ad */
    tau[a] = mu * (g[d * NL + a] + g[a * NL + d]);
    if (a == d) tau[a] -= 2.0 / 3.0 * mu * divu;
  }
  F[0] = 0.0;
  F[1] = tau[0];
  F[2] = tau[1];
  F[3] = tau[2];
  F[4] = tau[0] * P[1] + tau[1] * P[2] + tau[2] * P[3] + lam * g[d * NL + 3];
}

/* ------------------------------------------------------------------------ */
/* Riemann solvers f*(U_L, U_R; n) (Eq. weak_form, FillFlux in App. A).      */
/* The paper does not name the solver; local Lax-Friedrichs and Roe.         */
/* ------------------------------------------------------------------------ */
static void flux_normal(const double *U, const double *P, const double *nv, double *F) {
  double f[NV];
  for (int v = 0; v < NV; ++v) F[v] = 0.0;
  for (int d = 0; d < 3; ++d) {
    flux_adv(U, P, d, f);
    for (int v = 0; v < NV; ++v) F[v] += f[v] * nv[d];
  }
}

static void riemann_llf(const orc *o, const double *UL, const double *PL, const double *UR,
                        const double *PR, const double *nv, double *F) {
  double FL[NV], FR[NV];
  flux_normal(UL, PL, nv, FL);
  flux_normal(UR, PR, nv, FR);
  double cL = sqrt(o->gamma * PL[4] / PL[0]), cR = sqrt(o->gamma * PR[4] / PR[0]);
  double unL = PL[1] * nv[0] + PL[2] * nv[1] + PL[3] * nv[2];
  double unR = PR[1] * nv[0] + PR[2] * nv[1] + PR[3] * nv[2];
  double lmax = fmax(fabs(unL) + cL, fabs(unR) + cR);
  for (int v = 0; v < NV; ++v) F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * lmax * (UR[v] - UL[v]);
}

/* Roe's approximate Riemann solver (Roe 1981), no entropy fix:
 * f* = 1/2 (F_L + F_R).n - 1/2 sum_k |lambda_k| a_k r_k with Roe averages. */
static void riemann_roe(const orc *o, const double *UL, const double *PL, const double *UR,
                        const double *PR, const double *nv, double *F) {
  double FL[NV], FR[NV];
  flux_normal(UL, PL, nv, FL);
  flux_normal(UR, PR, nv, FR);
  double g1 = o->gamma - 1.0;
  double sL = sqrt(PL[0]), sR = sqrt(PR[0]);
  double HL = (UL[4] + PL[4]) / PL[0], HR = (UR[4] + PR[4]) / PR[0];
  double ut[3];
  for (int d = 0; d < 3; ++d) ut[d] = (sL * PL[1 + d] + sR * PR[1 + d]) / (sL + sR);
  double Ht = (sL * HL + sR * HR) / (sL + sR);
  double q2 = ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2];
  double ct = sqrt(g1 * (Ht - 0.5 * q2));
  double rt = sL * sR;
  double unt = ut[0] * nv[0] + ut[1] * nv[1] + ut[2] * nv[2];
  double drho = PR[0] - PL[0], dp = PR[4] - PL[4];
  double du[3];
  for (int d = 0; d < 3; ++d) du[d] = PR[1 + d] - PL[1 + d];
  double dun = du[0] * nv[0] + du[1] * nv[1] + du[2] * nv[2];
  double a1 = (dp - rt * ct * dun) / (2.0 * ct * ct);
  double a2 = drho - dp / (ct * ct);
  double a3 = (dp + rt * ct * dun) / (2.0 * ct * ct);
  double l1 = fabs(unt - ct), l2 = fabs(unt), l3 = fabs(unt + ct);
  double dut[3];
  for (int d = 0; d < 3; ++d) dut[d] = du[d] - dun * nv[d];
  double udut = ut[0] * dut[0] + ut[1] * dut[1] + ut[2] * dut[2];
  double Dis[NV];
  /* acoustic wave u-c */
  Dis[0] = l1 * a1;
  for (int d = 0; d < 3; ++d) Dis[1 + d] = l1 * a1 * (ut[d] - ct * nv[d]);
  Dis[4] = l1 * a1 * (Ht - unt * ct);
  /* entropy wave */
  Dis[0] += l2 * a2;
  for (int d = 0; d < 3; ++d) Dis[1 + d] += l2 * a2 * ut[d];
  Dis[4] += l2 * a2 * 0.5 * q2;
  /* shear waves */
  for (int d = 0; d < 3; ++d) Dis[1 + d] += l2 * rt * dut[d];
  Dis[4] += l2 * rt * udut;
  /* acoustic wave u+c */
  Dis[0] += l3 * a3;
  for (int d = 0; d < 3; ++d) Dis[1 + d] += l3 * a3 * (ut[d] + ct * nv[d]);
  Dis[4] += l3 * a3 * (Ht + unt * ct);
  for (int v = 0; v < NV; ++v) F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * Dis[v];
}

static void riemann(const orc *o, int which, const double *UL, const double *PL, const double *UR,
                    const double *PR, const double *nv, double *F) {
  if (which == 1) riemann_roe(o, UL, PL, UR, PR, nv, F);
  else riemann_llf(o, UL, PL, UR, PR, nv, F);
}

/* ------------------------------------------------------------------------ */
/* Sec. 2.2 "Nonlinear Stability": two-point volume fluxes of the split      */
/* form along an unnormalised direction m (in the volume integral, the mean  */
/* of the two nodes' contravariant metric vectors).  Both are consistent:    */
/* F#(U, U; m) = F(U).m, and symmetric in their two states.                  */
/* ------------------------------------------------------------------------ */

/* Pirozzoli's kinetic-energy-preserving flux: arithmetic means of density,
 * velocity, pressure and specific total enthalpy H = (rho e + p)/rho; the
 * mass flux is mean(rho) mean(u).m, momentum and energy are carried by it. */
static void two_point_kep(const double *UL, const double *PL, const double *UR, const double *PR,
                          const double *m, double *F) {
  double rho = 0.5 * (PL[0] + PR[0]);
  double u[3];
  for (int d = 0; d < 3; ++d) u[d] = 0.5 * (PL[1 + d] + PR[1 + d]);
  double p = 0.5 * (PL[4] + PR[4]);
  double H = 0.5 * ((UL[4] + PL[4]) / PL[0] + (UR[4] + PR[4]) / PR[0]);
  double mf = rho * (u[0] * m[0] + u[1] * m[1] + u[2] * m[2]);
  F[0] = mf;
  for (int d = 0; d < 3; ++d) F[1 + d] = mf * u[d] + p * m[d];
  F[4] = mf * H;
}

/* the mean of the two states' fluxes along m; with it the split form is the
 * standard DG operator on meshes with constant metric terms */
static void two_point_mean(const double *UL, const double *PL, const double *UR, const double *PR,
                           const double *m, double *F) {
  double FL[NV], FR[NV];
  flux_normal(UL, PL, m, FL);
  flux_normal(UR, PR, m, FR);
  for (int v = 0; v < NV; ++v) F[v] = 0.5 * (FL[v] + FR[v]);
}

static void two_point(const orc *o, const double *UL, const double *PL, const double *UR,
                      const double *PR, const double *m, double *F) {
  if (o->volume_flux == 2) two_point_mean(UL, PL, UR, PR, m, F);
  else two_point_kep(UL, PL, UR, PR, m, F);
}

/* ------------------------------------------------------------------------ */
/* Setup: nodes, operators, curl-form metrics (Sec. 2.2 "Mapping the        */
/* Equations"), face metrics and geometric face matching.                    */
/* ------------------------------------------------------------------------ */
static void *xalloc(size_t n) {
  void *p = calloc(n ? n : 1, 1);
  if (!p) { fprintf(stderr, "oracle: out of memory\n"); abort(); }
  return p;
}
#define ALLOC(T, cnt) ((T *)xalloc(sizeof(T) * (size_t)(cnt)))

void orc_destroy(orc *o);

/* Basis of Sec. 2.2: D-hat_ij = -(w_j/w_i) l_i'(x_j) (Kopriva's definition;
 * the printed weight ratio is inverted) and l-hat^pm_i = l_i(+-1)/w_i. */
static void build_basis(orc *o) {
  int n = o->n;
  o->x = ALLOC(double, n); o->w = ALLOC(double, n);
  o->D = ALLOC(double, n * n); o->Dhat = ALLOC(double, n * n);
  o->lm = ALLOC(double, n); o->lp = ALLOC(double, n);
  o->lhm = ALLOC(double, n); o->lhp = ALLOC(double, n);
  o->xL = ALLOC(xr, n); o->xgL = ALLOC(xr, n); o->DgL = ALLOC(xr, n * n); o->Mg2sL = ALLOC(xr, n * n);
  xr *wL = ALLOC(xr, n), *wgL = ALLOC(xr, n), *DL = ALLOC(xr, n * n);
  if (o->node_type == 0) gauss_nodes(o->N, o->xL, wL);
  else lobatto_nodes(o->N, o->xL, wL);
  lobatto_nodes(o->N, o->xgL, wgL);
  diff_matrix(n, o->xL, DL);
  diff_matrix(n, o->xgL, o->DgL);
  for (int i = 0; i < n; ++i) {
    o->x[i] = (double)o->xL[i];
    o->w[i] = (double)wL[i];
  }
  for (int i = 0; i < n * n; ++i) o->D[i] = (double)DL[i];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) o->Dhat[i * n + j] = (double)(-(wL[j] / wL[i]) * DL[j * n + i]);
  for (int i = 0; i < n; ++i) {
    xr lm = lagrange(n, o->xL, i, -1.0L), lp = lagrange(n, o->xL, i, 1.0L);
    o->lm[i] = (double)lm;
    o->lp[i] = (double)lp;
    o->lhm[i] = (double)(lm / wL[i]);
    o->lhp[i] = (double)(lp / wL[i]);
  }
  interp_matrix(n, o->xgL, n, o->xL, o->Mg2sL);
  /* FV subcell interfaces: xi_{-1/2} = -1, xi_{m+1/2} = -1 + sum_{k<=m} w_k */
  o->xhalf = ALLOC(double, n + 1);
  o->xhalf[0] = -1.0;
  for (int m = 0; m < n; ++m) o->xhalf[m + 1] = o->xhalf[m] + o->w[m];
  /* orthonormal Legendre Vandermonde V_ia = sqrt((2a+1)/2) P_a(x_i), inverted by
   * Gauss-Jordan elimination with partial pivoting */
  xr *V = ALLOC(xr, n * n), *I = ALLOC(xr, n * n);
  for (int i = 0; i < n; ++i)
    for (int a = 0; a < n; ++a) {
      xr P, dP;
      legendre(a, o->xL[i], &P, &dP);
      V[i * n + a] = sqrtl((2.0L * a + 1.0L) / 2.0L) * P;
      I[i * n + a] = (i == a);
    }
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (fabsl(V[r * n + c]) > fabsl(V[piv * n + c])) piv = r;
    for (int k = 0; k < n; ++k) {
      xr t = V[c * n + k]; V[c * n + k] = V[piv * n + k]; V[piv * n + k] = t;
      t = I[c * n + k]; I[c * n + k] = I[piv * n + k]; I[piv * n + k] = t;
    }
    xr d = V[c * n + c];
    for (int k = 0; k < n; ++k) { V[c * n + k] /= d; I[c * n + k] /= d; }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      xr f = V[r * n + c];
      for (int k = 0; k < n; ++k) { V[r * n + k] -= f * V[c * n + k]; I[r * n + k] -= f * I[c * n + k]; }
    }
  }
  o->Vinv = ALLOC(double, n * n);
  for (int i = 0; i < n * n; ++i) o->Vinv[i] = (double)I[i];
  free(V); free(I); free(wL); free(wgL); free(DL);
}

/* Curl form of Sec. 2.2: Ja^i_n = -e_i . curl_xi (x_l grad_xi x_m), (n,m,l)
 * cyclic, e_i the i-th computational unit vector, evaluated on LGL(N) with the
 * LGL differentiation matrix and interpolated to the solution nodes. */
static void build_metrics(orc *o, const double *x_geo) {
  int n = o->n, n3 = o->n3, ng = o->ngeo + 1, ng3 = ng * ng * ng;
  long E = o->E;
  o->XL = ALLOC(double, E * n3 * 3);
  o->Xs = ALLOC(double, E * n3 * 3);
  o->Ja = ALLOC(double, E * n3 * 9);
  o->J = ALLOC(double, E * n3);
  o->nS = ALLOC(double, E * 6 * o->n2 * 3);
  xr *xgeo_nodes = ALLOC(xr, ng), *wgeo = ALLOC(xr, ng);
  lobatto_nodes(o->ngeo, xgeo_nodes, wgeo);
  xr *Mgeo = ALLOC(xr, n * ng);
  interp_matrix(ng, xgeo_nodes, n, o->xgL, Mgeo);
#pragma omp parallel for schedule(static)
  for (long e = 0; e < E; ++e) {
    xr *in = ALLOC(xr, ng3 * 3);
    for (int a = 0; a < ng3; ++a)
      for (int c = 0; c < 3; ++c) in[a * 3 + c] = x_geo[(e * 3 + c) * ng3 + a];
    xr *XL = ALLOC(xr, n3 * 3);
    interp3x(ng, n, Mgeo, in, XL, 3);
    free(in);
    for (int a = 0; a < n3 * 3; ++a) o->XL[e * n3 * 3 + a] = (double)XL[a];
    /* dX[j][m] = d x_m / d xi_j on LGL(N) */
    xr *dX = ALLOC(xr, n3 * 9);
    for (int j = 0; j < 3; ++j)
      for (int m = 0; m < 3; ++m) deriv_dirx(n, o->DgL, j, XL + m, 3, dX + j * 3 + m, 9);
    xr *JaL = ALLOC(xr, n3 * 9);
    xr *Vv = ALLOC(xr, n3 * 3), *dV = ALLOC(xr, n3);
    /* The curl form is unchanged by a constant shift of x (the discrete curl
     * of a discrete gradient vanishes, D_b D_c = D_c D_b); positions are taken
     * relative to the element's first geometry node to avoid cancellation. */
    xr x0[3] = {XL[0], XL[1], XL[2]};
    for (int nn = 0; nn < 3; ++nn) {
      int m = (nn + 1) % 3, l = (nn + 2) % 3;
      /* V_j = x_l d_j x_m, pointwise on the LGL grid */
      for (int a = 0; a < n3; ++a)
        for (int j = 0; j < 3; ++j) Vv[a * 3 + j] = (XL[a * 3 + l] - x0[l]) * dX[a * 9 + j * 3 + m];
      /* (curl V)_0 = d1 V2 - d2 V1, (curl V)_1 = d2 V0 - d0 V2, (curl V)_2 = d0 V1 - d1 V0 */
      for (int i = 0; i < 3; ++i) {
        int b = (i + 1) % 3, c = (i + 2) % 3;
        for (int a = 0; a < n3; ++a) JaL[a * 9 + i * 3 + nn] = 0.0L;
        deriv_dirx(n, o->DgL, b, Vv + c, 3, dV, 1);
        for (int a = 0; a < n3; ++a) JaL[a * 9 + i * 3 + nn] -= dV[a];
        deriv_dirx(n, o->DgL, c, Vv + b, 3, dV, 1);
        for (int a = 0; a < n3; ++a) JaL[a * 9 + i * 3 + nn] += dV[a];
      }
    }
    free(Vv); free(dV);
    /* to the solution nodes */
    xr *tmp = ALLOC(xr, n3 * 9);
    interp3x(n, n, o->Mg2sL, JaL, tmp, 9);
    for (int a = 0; a < n3 * 9; ++a) o->Ja[e * n3 * 9 + a] = (double)tmp[a];
    interp3x(n, n, o->Mg2sL, XL, tmp, 3);
    for (int a = 0; a < n3 * 3; ++a) o->Xs[e * n3 * 3 + a] = (double)tmp[a];
    interp3x(n, n, o->Mg2sL, dX, tmp, 9);
    for (int a = 0; a < n3; ++a) {
      const xr *A = tmp + a * 9; /* A[j*3+m] = d x_m / d xi_j */
      o->J[e * n3 + a] = (double)(A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                                  A[2] * (A[3] * A[7] - A[4] * A[6]));
    }
    free(tmp);
    /* face metrics: Ja^d on the LGL face slice, 2-D interpolated to the
     * solution face nodes; outward n*shat = +-Ja^d */
    for (int f = 0; f < 6; ++f) {
      int d = f / 2, side = f % 2;
      int l = side ? n - 1 : 0;
      xr sgn = side ? 1.0L : -1.0L;
      for (int q = 0; q < n; ++q)
        for (int p = 0; p < n; ++p) {
          xr a[3] = {0, 0, 0};
          for (int qq = 0; qq < n; ++qq)
            for (int pp = 0; pp < n; ++pp) {
              xr wgt = o->Mg2sL[p * n + pp] * o->Mg2sL[q * n + qq];
              int a_node = line_node(n, d, l, pp, qq);
              for (int c = 0; c < 3; ++c) a[c] += wgt * JaL[a_node * 9 + d * 3 + c];
            }
          double *ns = o->nS + ((e * 6 + f) * o->n2 + p + n * q) * 3;
          for (int c = 0; c < 3; ++c) ns[c] = (double)(sgn * a[c]);
        }
    }
    free(JaL); free(dX); free(XL);
  }
  free(xgeo_nodes); free(wgeo); free(Mgeo);
}

/* Unstructured connectivity (Sec. 2.2, last paragraph; App. A ProlongToFace):
 * the node correspondence on each face is recovered from coincident physical
 * positions of the LGL(N) face nodes, modulo the periodic box.  Two faces are
 * related by a relative rotation or reflection of the face frame, i.e. one of
 * the eight symmetries of the square grid.  A face that touches its own
 * periodic image (one element across the box) has edge nodes that coincide
 * with several neighbour nodes modulo the period, so the correspondence is
 * the unique symmetry under which every node lands on a coincident node. */
static void square_map(int code, int n, int p, int q, int *pp, int *qq) {
  int a = (code & 1) ? q : p, b = (code & 1) ? p : q;
  *pp = (code & 2) ? n - 1 - a : a;
  *qq = (code & 4) ? n - 1 - b : b;
}

static int match_faces(orc *o, const long *nbr_elem, const int8_t *nbr_face) {
  int n = o->n, n2 = o->n2;
  long E = o->E;
  o->nbr = ALLOC(long, E * 6);
  o->nbrf = ALLOC(int, E * 6);
  o->fmap = ALLOC(int, E * 6 * n2);
  int bad = 0;
  long bad_e = -1; int bad_f = -1;
#pragma omp parallel for schedule(static)
  for (long e = 0; e < E; ++e) {
    char *coin = (char *)xalloc((size_t)n2 * n2);
    for (int f = 0; f < 6; ++f) {
      long e2 = nbr_elem[e * 6 + f];
      int f2 = nbr_face[e * 6 + f];
      o->nbr[e * 6 + f] = e2;
      o->nbrf[e * 6 + f] = f2;
      if (e2 < 0 || e2 >= E || f2 < 0 || f2 > 5) {
#pragma omp critical
        { bad = 1; bad_e = e; bad_f = f; }
        continue;
      }
      int d = f / 2, l = (f % 2) ? n - 1 : 0;
      int d2 = f2 / 2, l2 = (f2 % 2) ? n - 1 : 0;
      const double *X1 = o->XL + e * o->n3 * 3, *X2 = o->XL + e2 * o->n3 * 3;
      /* length scale: face diagonal */
      const double *c0 = X1 + line_node(n, d, l, 0, 0) * 3;
      const double *c1 = X1 + line_node(n, d, l, n - 1, n - 1) * 3;
      double hs = sqrt((c1[0] - c0[0]) * (c1[0] - c0[0]) + (c1[1] - c0[1]) * (c1[1] - c0[1]) +
                       (c1[2] - c0[2]) * (c1[2] - c0[2]));
      double tol = 1e-8 * hs;
      /* coin[a][b]: own node a coincides with neighbour node b (mod period) */
      for (int a = 0; a < n2; ++a)
        for (int b = 0; b < n2; ++b) {
          const double *xa = X1 + line_node(n, d, l, a % n, a / n) * 3;
          const double *xb = X2 + line_node(n, d2, l2, b % n, b / n) * 3;
          double dist2 = 0.0;
          for (int c = 0; c < 3; ++c) {
            double dd = xa[c] - xb[c];
            if (o->period[c] > 0.0) dd -= o->period[c] * nearbyint(dd / o->period[c]);
            dist2 += dd * dd;
          }
          coin[a * n2 + b] = sqrt(dist2) <= tol;
        }
      int found = -1, count = 0;
      for (int code = 0; code < 8; ++code) {
        int ok = 1;
        for (int a = 0; a < n2 && ok; ++a) {
          int pp, qq;
          square_map(code, n, a % n, a / n, &pp, &qq);
          ok = coin[a * n2 + pp + n * qq];
        }
        if (ok) { found = code; ++count; }
      }
      if (count != 1) {
#pragma omp critical
        { bad = 1; bad_e = e; bad_f = f; }
        continue;
      }
      for (int a = 0; a < n2; ++a) {
        int pp, qq;
        square_map(found, n, a % n, a / n, &pp, &qq);
        o->fmap[(e * 6 + f) * n2 + a] = pp + n * qq;
      }
    }
    free(coin);
  }
  if (bad) {
    snprintf(o->err, sizeof o->err, "faces do not coincide (or not uniquely): element %ld face %d", bad_e, bad_f);
    return -2;
  }
  return 0;
}

static inline int is_master(const orc *o, long e, int f) {
  long e2 = o->nbr[e * 6 + f];
  int f2 = o->nbrf[e * 6 + f];
  return (e * 6 + f) < (e2 * 6 + f2);
}

orc *orc_create(int N, int node_type, int ngeo, long E, const double *x_geo, const long *nbr_elem,
                const int8_t *nbr_face, const double *period, char *errbuf, int errlen) {
  orc *o = (orc *)xalloc(sizeof(orc));
  o->N = N; o->n = N + 1; o->n2 = o->n * o->n; o->n3 = o->n2 * o->n;
  o->node_type = node_type; o->ngeo = ngeo; o->E = E;
  for (int c = 0; c < 3; ++c) o->period[c] = period ? period[c] : 0.0;
  o->gamma = 1.4; o->R = 1.0; o->Pr = 0.72; o->mu = 0.0;
  o->riemann = 0; o->viscous = 0; o->source = 0; o->shock = 0;
  o->alpha_max = 1.0; o->alpha_min = 0.001; o->ind_a = 0.5; o->ind_c = 1.8; o->ind_s = log(9999.0);
  o->alpha_smooth = 0; o->volume_flux = 0; o->visc_law = 0; o->T_ref = 1.0; o->rk_scheme = 0;
  build_basis(o);
  build_metrics(o, x_geo);
  int rc = match_faces(o, nbr_elem, nbr_face);
  if (rc) {
    if (errbuf) snprintf(errbuf, errlen, "%s", o->err);
    orc_destroy(o);
    return NULL;
  }
  size_t n3 = o->n3, n2 = o->n2;
  o->alpha = ALLOC(double, E);
  o->Ui = ALLOC(double, E * n3 * NV);
  o->prim = ALLOC(double, E * n3 * 6);
  o->Uf = ALLOC(double, E * 6 * n2 * NV);
  o->primf = ALLOC(double, E * 6 * n2 * 6);
  o->G = ALLOC(double, E * n3 * 3 * NL);
  o->Gf = ALLOC(double, E * 6 * n2 * 3 * NL);
  o->V = ALLOC(double, E * n3 * NV);
  o->faceF = ALLOC(double, E * 6 * n2 * NV);
  o->liftF = ALLOC(double, E * 6 * n2 * 3 * NL);
  o->Vadv = ALLOC(double, E * n3 * NV);
  o->Vvis = ALLOC(double, E * n3 * NV);
  o->Vfv = ALLOC(double, E * n3 * NV);
  return o;
}

void orc_destroy(orc *o) {
  if (!o) return;
  void *ptrs[] = {o->x, o->w, o->D, o->Dhat, o->lm, o->lp, o->lhm, o->lhp, o->xL, o->xgL, o->DgL,
                  o->Mg2sL, o->XL, o->Xs, o->Ja, o->J, o->nS, o->nbr, o->nbrf, o->fmap, o->alpha,
                  o->Vinv, o->xhalf, o->Ui, o->prim, o->Uf, o->primf, o->G, o->Gf, o->V,
                  o->faceF, o->liftF, o->Vadv, o->Vvis, o->Vfv};
  for (size_t i = 0; i < sizeof ptrs / sizeof ptrs[0]; ++i) free(ptrs[i]);
  free(o);
}

/* the switches added to the standard scheme: alpha smoothing, split-form
 * volume flux, Sutherland's law (reference temperature T_ref), RK scheme */
void orc_set_params2(orc *o, int alpha_smooth, int volume_flux, int visc_law, double T_ref, int rk_scheme) {
  o->alpha_smooth = alpha_smooth;
  o->volume_flux = volume_flux;
  o->visc_law = visc_law;
  o->T_ref = T_ref;
  o->rk_scheme = rk_scheme;
}

void orc_set_params(orc *o, double gamma, double R, double Pr, double mu, int riemann, int viscous,
                    int source, int shock, double alpha_max, double alpha_min, double ind_a,
                    double ind_c, double ind_s) {
  o->gamma = gamma; o->R = R; o->Pr = Pr; o->mu = mu;
  o->riemann = riemann; o->viscous = viscous; o->source = source; o->shock = shock;
  o->alpha_max = alpha_max; o->alpha_min = alpha_min;
  o->ind_a = ind_a; o->ind_c = ind_c; o->ind_s = ind_s;
}

/* ------------------------------------------------------------------------ */
/* Shock capturing (Sec. 2.3): a-priori modal indicator -> alpha.            */
/* ------------------------------------------------------------------------ */
static double indicator_alpha(const orc *o, long e) {
  int n = o->n, n3 = o->n3, N = o->N;
  double *eps = ALLOC(double, n3), *m = ALLOC(double, n3);
  for (int a = 0; a < n3; ++a) {
    const double *P = o->prim + (e * n3 + a) * 6;
    eps[a] = P[0] * P[4];
  }
  interp3(n, n, o->Vinv, eps, m, 1); /* modal coefficients (V^-1 (x) V^-1 (x) V^-1) eps */
  double tot = 0.0, c1 = 0.0, c2 = 0.0;
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        double m2 = m[nidx(n, i, j, k)] * m[nidx(n, i, j, k)];
        tot += m2;
        if (i <= N - 1 && j <= N - 1 && k <= N - 1) c1 += m2;
        if (i <= N - 2 && j <= N - 2 && k <= N - 2) c2 += m2;
      }
  free(eps); free(m);
  double E1 = (tot > 0.0) ? (tot - c1) / tot : 0.0;
  double E2 = (c1 > 0.0) ? (c1 - c2) / c1 : 0.0;
  double Ev = fmax(E1, E2);
  double T = o->ind_a * pow(10.0, -o->ind_c * pow(N + 1.0, 0.25));
  double alpha = 1.0 / (1.0 + exp(-(o->ind_s / T) * (Ev - T)));
  if (alpha < o->alpha_min) alpha = 0.0;
  else if (alpha > 1.0 - o->alpha_min) alpha = 1.0;
  alpha = fmin(alpha, o->alpha_max);
  return alpha;
}

static inline double minmod(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  return (a > 0.0 ? 1.0 : -1.0) * fmin(fabs(a), fabs(b));
}

/* FV subcell operator of Sec. 2.3 on the LGL subcells of element e: the
 * interface metrics are accumulated along each line from the LGL
 * differentiation of Ja, primitives are reconstructed with minmod slopes,
 * and the interfaces are closed with the local Lax-Friedrichs flux.  Only
 * interfaces inside the element; the element faces stay with SurfInt. */
static void fv_volume(const orc *o, long e, double *Vfv) {
  int n = o->n, n3 = o->n3, N = o->N;
  const double *xw = o->x, *ww = o->w;
  for (int a = 0; a < n3 * NV; ++a) Vfv[a] = 0.0;
  double Jah[32][3];
  double q[32][5], sl[32][5];
  for (int d = 0; d < 3; ++d)
    for (int qq = 0; qq < n; ++qq)
      for (int pp = 0; pp < n; ++pp) {
        /* interface metric (Ja^d)_{m+1/2}, m = -1..N */
        for (int c = 0; c < 3; ++c) Jah[0][c] = o->Ja[(e * n3 + line_node(n, d, 0, pp, qq)) * 9 + d * 3 + c];
        for (int m = 0; m < n; ++m)
          for (int c = 0; c < 3; ++c) {
            double s = 0.0;
            for (int l = 0; l < n; ++l)
              s += o->D[m * n + l] * o->Ja[(e * n3 + line_node(n, d, l, pp, qq)) * 9 + d * 3 + c];
            Jah[m + 1][c] = Jah[m][c] + ww[m] * s;
          }
        for (int l = 0; l < n; ++l) {
          const double *P = o->prim + (e * n3 + line_node(n, d, l, pp, qq)) * 6;
          for (int v = 0; v < 5; ++v) q[l][v] = P[v];
        }
        for (int v = 0; v < 5; ++v) { sl[0][v] = 0.0; sl[N][v] = 0.0; }
        for (int l = 1; l < N; ++l)
          for (int v = 0; v < 5; ++v)
            sl[l][v] = minmod((q[l][v] - q[l - 1][v]) / (xw[l] - xw[l - 1]),
                              (q[l + 1][v] - q[l][v]) / (xw[l + 1] - xw[l]));
        double fh[32][NV];
        for (int m = 0; m < N; ++m) {
          double xh = o->xhalf[m + 1];
          double qL[5], qR[5], UL[NV], UR[NV], PL[6], PR[6];
          for (int v = 0; v < 5; ++v) {
            qL[v] = q[m][v] + sl[m][v] * (xh - xw[m]);
            qR[v] = q[m + 1][v] - sl[m + 1][v] * (xw[m + 1] - xh);
          }
          prim_to_cons(o, qL, UL);
          prim_to_cons(o, qR, UR);
          cons_to_prim(o, UL, PL);
          cons_to_prim(o, UR, PR);
          const double *a = Jah[m + 1];
          double sh = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
          double nv[3] = {a[0] / sh, a[1] / sh, a[2] / sh};
          double F[NV];
          riemann_llf(o, UL, PL, UR, PR, nv, F);
          for (int v = 0; v < NV; ++v) fh[m][v] = F[v] * sh;
        }
        for (int l = 0; l < n; ++l) {
          double *out = Vfv + line_node(n, d, l, pp, qq) * NV;
          for (int v = 0; v < NV; ++v) {
            double r = 0.0;
            if (l < N) r += fh[l][v];
            if (l > 0) r -= fh[l - 1][v];
            out[v] += r / ww[l];
          }
        }
      }
}

/* ------------------------------------------------------------------------ */
/* The DG operator, Eq. dgsem, with BR1 lifting (Sec. 2.2 "Second-Order      */
/* Equations") and FV blending (Sec. 2.3).  Ut = R(U, t).                     */
/* ------------------------------------------------------------------------ */
int orc_rhs(orc *o, const double *Usoa, double t, double *Utsoa) {
  int n = o->n, n2 = o->n2, n3 = o->n3;
  long E = o->E;
  /* state to [elem][node][var] */
#pragma omp parallel for schedule(static)
  for (long e = 0; e < E; ++e)
    for (int a = 0; a < n3; ++a)
      for (int v = 0; v < NV; ++v) o->Ui[(e * n3 + a) * NV + v] = Usoa[((long)v * E + e) * n3 + a];

  /* ConsToPrim (volume) */
#pragma omp parallel for schedule(static)
  for (long e = 0; e < E; ++e)
    for (int a = 0; a < n3; ++a) cons_to_prim(o, o->Ui + (e * n3 + a) * NV, o->prim + (e * n3 + a) * 6);

  /* ProlongToFace: U~(p,q) = sum_l l_l(+-1) U_l along the face-normal line;
   * then ConsToPrim (surface) */
#pragma omp parallel for schedule(static)
  for (long e = 0; e < E; ++e)
    for (int f = 0; f < 6; ++f) {
      int d = f / 2;
      const double *lv = (f % 2) ? o->lp : o->lm;
      for (int q = 0; q < n; ++q)
        for (int p = 0; p < n; ++p) {
          double *uf = o->Uf + ((e * 6 + f) * n2 + p + n * q) * NV;
          for (int v = 0; v < NV; ++v) {
            double s = 0.0;
            for (int l = 0; l < n; ++l) s += lv[l] * o->Ui[(e * n3 + line_node(n, d, l, p, q)) * NV + v];
            uf[v] = s;
          }
          cons_to_prim(o, uf, o->primf + ((e * 6 + f) * n2 + p + n * q) * 6);
        }
    }

  if (o->viscous) {
    /* Lift_FillFlux: on each face, v* = (v_primary + v_replica)/2 for v = u,v,w,T,
     * times the primary side's n*shat; the replica receives it negated. */
#pragma omp parallel for schedule(static)
    for (long e = 0; e < E; ++e)
      for (int f = 0; f < 6; ++f) {
        long e2 = o->nbr[e * 6 + f];
        int f2 = o->nbrf[e * 6 + f];
        int prim_side = is_master(o, e, f);
        for (int pq = 0; pq < n2; ++pq) {
          /* the primary face node and its replica */
          long em, es; int fm, fs, pqm, pqs;
          if (prim_side) { em = e; fm = f; pqm = pq; es = e2; fs = f2; pqs = o->fmap[(e * 6 + f) * n2 + pq]; }
          else { es = e; fs = f; pqs = pq; em = e2; fm = f2; pqm = o->fmap[(e * 6 + f) * n2 + pq]; }
          const double *Pm = o->primf + ((em * 6 + fm) * n2 + pqm) * 6;
          const double *Ps = o->primf + ((es * 6 + fs) * n2 + pqs) * 6;
          const double *ns = o->nS + ((em * 6 + fm) * n2 + pqm) * 3;
          double sgn = prim_side ? 1.0 : -1.0;
          double *out = o->liftF + ((e * 6 + f) * n2 + pq) * 3 * NL;
          for (int d = 0; d < 3; ++d)
            for (int v = 0; v < NL; ++v) {
              double vs = 0.5 * (Pm[LIFT_IDX[v]] + Ps[LIFT_IDX[v]]);
              out[d * NL + v] = sgn * vs * ns[d];
            }
        }
      }
    /* Lift_VolInt: J g_{d,v} = sum_i sum_alpha D-hat (Ja^i_d v)_alpha along line i;
     * Lift_SurfInt: + sum_faces (v* n_d shat) l-hat^pm; ApplyJac: g = (J g)/J */
#pragma omp parallel for schedule(static)
    for (long e = 0; e < E; ++e) {
      double *G = o->G + e * n3 * 3 * NL;
      for (int a = 0; a < n3 * 3 * NL; ++a) G[a] = 0.0;
      for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
          for (int i = 0; i < n; ++i) {
            int node = nidx(n, i, j, k);
            int ijk[3] = {i, j, k};
            for (int ci = 0; ci < 3; ++ci)
              for (int al = 0; al < n; ++al) {
                int src;
                if (ci == 0) src = nidx(n, al, j, k);
                else if (ci == 1) src = nidx(n, i, al, k);
                else src = nidx(n, i, j, al);
                double Dh = o->Dhat[ijk[ci] * n + al];
                const double *P = o->prim + (e * n3 + src) * 6;
                const double *Ja = o->Ja + (e * n3 + src) * 9 + ci * 3;
                for (int d = 0; d < 3; ++d)
                  for (int v = 0; v < NL; ++v) G[node * 3 * NL + d * NL + v] += Dh * (Ja[d] * P[LIFT_IDX[v]]);
              }
          }
      for (int f = 0; f < 6; ++f) {
        int d0 = f / 2;
        const double *lh = (f % 2) ? o->lhp : o->lhm;
        for (int q = 0; q < n; ++q)
          for (int p = 0; p < n; ++p) {
            const double *lf = o->liftF + ((e * 6 + f) * n2 + p + n * q) * 3 * NL;
            for (int l = 0; l < n; ++l) {
              int node = line_node(n, d0, l, p, q);
              for (int c = 0; c < 3 * NL; ++c) G[node * 3 * NL + c] += lf[c] * lh[l];
            }
          }
      }
      for (int a = 0; a < n3; ++a)
        for (int c = 0; c < 3 * NL; ++c) G[a * 3 * NL + c] = G[a * 3 * NL + c] / o->J[e * n3 + a];
      /* Lift_ProlongToFace */
      for (int f = 0; f < 6; ++f) {
        int d0 = f / 2;
        const double *lv = (f % 2) ? o->lp : o->lm;
        for (int q = 0; q < n; ++q)
          for (int p = 0; p < n; ++p) {
            double *gf = o->Gf + ((e * 6 + f) * n2 + p + n * q) * 3 * NL;
            for (int c = 0; c < 3 * NL; ++c) {
              double s = 0.0;
              for (int l = 0; l < n; ++l) s += lv[l] * G[line_node(n, d0, l, p, q) * 3 * NL + c];
              gf[c] = s;
            }
          }
      }
    }
  }

  /* FillFlux: f* = [F*_adv(U_primary, U_replica; n) - (Fv(primary) + Fv(replica))/2 . n] shat,
   * with the primary side's normal; stored per element face with the sign of
   * its own outward normal (replica: -f*). */
#pragma omp parallel for schedule(static)
  for (long e = 0; e < E; ++e)
    for (int f = 0; f < 6; ++f) {
      long e2 = o->nbr[e * 6 + f];
      int f2 = o->nbrf[e * 6 + f];
      int prim_side = is_master(o, e, f);
      for (int pq = 0; pq < n2; ++pq) {
        long em, es; int fm, fs, pqm, pqs;
        if (prim_side) { em = e; fm = f; pqm = pq; es = e2; fs = f2; pqs = o->fmap[(e * 6 + f) * n2 + pq]; }
        else { es = e; fs = f; pqs = pq; em = e2; fm = f2; pqm = o->fmap[(e * 6 + f) * n2 + pq]; }
        long im = (em * 6 + fm) * n2 + pqm, is = (es * 6 + fs) * n2 + pqs;
        const double *ns = o->nS + im * 3;
        double sh = sqrt(ns[0] * ns[0] + ns[1] * ns[1] + ns[2] * ns[2]);
        double nv[3] = {ns[0] / sh, ns[1] / sh, ns[2] / sh};
        double F[NV];
        riemann(o, o->riemann, o->Uf + im * NV, o->primf + im * 6, o->Uf + is * NV, o->primf + is * 6, nv, F);
        if (o->viscous) {
          double fvm[NV], fvs[NV], tmp[NV];
          for (int v = 0; v < NV; ++v) { fvm[v] = 0.0; fvs[v] = 0.0; }
          for (int d = 0; d < 3; ++d) {
            flux_visc(o, o->primf + im * 6, o->Gf + im * 3 * NL, d, tmp);
            for (int v = 0; v < NV; ++v) fvm[v] += tmp[v] * nv[d];
            flux_visc(o, o->primf + is * 6, o->Gf + is * 3 * NL, d, tmp);
            for (int v = 0; v < NV; ++v) fvs[v] += tmp[v] * nv[d];
          }
          for (int v = 0; v < NV; ++v) F[v] -= 0.5 * (fvm[v] + fvs[v]);
        }
        double sgn = prim_side ? 1.0 : -1.0;
        double *out = o->faceF + ((e * 6 + f) * n2 + pq) * NV;
        for (int v = 0; v < NV; ++v) out[v] = sgn * F[v] * sh;
      }
    }

  /* blending factors (Sec. 2.3), one per element: the indicator value of the
   * element, an operator local to the element.  With alpha_smooth (outside
   * the paper: Hennemann's neighbour smoothing) the value is raised to half
   * the largest value among its face neighbours, so that elements about to
   * be reached by a shock are already blended; values below alpha_min then
   * drop to zero and alpha_max caps the result. */
  if (o->shock && !o->alpha_frozen) {
    double *raw = ALLOC(double, E);
#pragma omp parallel for schedule(static)
    for (long e = 0; e < E; ++e) raw[e] = indicator_alpha(o, e);
#pragma omp parallel for schedule(static)
    for (long e = 0; e < E; ++e) {
      double a = raw[e];
      if (o->alpha_smooth) {
        for (int f = 0; f < 6; ++f) a = fmax(a, 0.5 * raw[o->nbr[e * 6 + f]]);
        if (a < o->alpha_min) a = 0.0;
        a = fmin(a, o->alpha_max);
      }
      o->alpha[e] = a;
    }
    free(raw);
  }

  /* VolInt: contravariant fluxes F^i = Ja^i . (F_adv - F_v) at every node, then
   * sum_alpha F^1_{alpha jk} D-hat_{i alpha} + ... (Eq. dgsem).
   * Split form (Sec. 2.2 "Nonlinear Stability", Gauss-Lobatto nodes): the
   * advective part becomes sum_alpha (2 D - W^-1 B)_{i alpha} F#^1(U_ijk, U_alpha jk)
   * + ..., the strong-form two-point volume term with the boundary values of
   * the strong form's surface correction folded in, so that the weak form's
   * surface integral of f* below completes it.  On these nodes the summation-
   * by-parts property W D + D^T W = B gives 2 D - W^-1 B = D + D-hat.  F#^1 is
   * taken along the mean of the two nodes' metric vectors Ja^1.  The viscous
   * part keeps the weak form. */
#pragma omp parallel for schedule(static)
  for (long e = 0; e < E; ++e) {
    int blend = o->shock && o->alpha[e] > 0.0;
    int split = o->volume_flux != 0;
    double *Vt = o->V + e * n3 * NV;
    double *Va = o->Vadv + e * n3 * NV, *Vv = o->Vvis + e * n3 * NV;
    for (int a = 0; a < n3 * NV; ++a) { Vt[a] = 0.0; Va[a] = 0.0; Vv[a] = 0.0; }
    /* contravariant fluxes at every node: Fc[node][i][v] (total), and the
     * advective / viscous parts when blending */
    double *Fc = ALLOC(double, n3 * 3 * NV), *Fa = ALLOC(double, n3 * 3 * NV), *Fv = ALLOC(double, n3 * 3 * NV);
    for (int a = 0; a < n3; ++a) {
      const double *U = o->Ui + (e * n3 + a) * NV;
      const double *P = o->prim + (e * n3 + a) * 6;
      const double *g = o->G + (e * n3 + a) * 3 * NL;
      double Fd[3][NV], Gd[3][NV];
      for (int d = 0; d < 3; ++d) {
        flux_adv(U, P, d, Fd[d]);
        if (o->viscous) flux_visc(o, P, g, d, Gd[d]);
        else for (int v = 0; v < NV; ++v) Gd[d][v] = 0.0;
      }
      const double *Ja = o->Ja + (e * n3 + a) * 9;
      for (int i = 0; i < 3; ++i)
        for (int v = 0; v < NV; ++v) {
          double sa = 0.0, sv = 0.0, st = 0.0;
          for (int d = 0; d < 3; ++d) {
            st += Ja[i * 3 + d] * (Fd[d][v] - Gd[d][v]);
            sa += Ja[i * 3 + d] * Fd[d][v];
            sv += Ja[i * 3 + d] * Gd[d][v];
          }
          Fc[(a * 3 + i) * NV + v] = st;
          Fa[(a * 3 + i) * NV + v] = sa;
          Fv[(a * 3 + i) * NV + v] = sv;
        }
    }
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
          int node = nidx(n, i, j, k);
          int ijk[3] = {i, j, k};
          for (int ci = 0; ci < 3; ++ci)
            for (int al = 0; al < n; ++al) {
              int src;
              if (ci == 0) src = nidx(n, al, j, k);
              else if (ci == 1) src = nidx(n, i, al, k);
              else src = nidx(n, i, j, al);
              double Dh = o->Dhat[ijk[ci] * n + al];
              for (int v = 0; v < NV; ++v) {
                if (!blend && !split) Vt[node * NV + v] += Dh * Fc[(src * 3 + ci) * NV + v];
                else {
                  if (!split) Va[node * NV + v] += Dh * Fa[(src * 3 + ci) * NV + v];
                  Vv[node * NV + v] -= Dh * Fv[(src * 3 + ci) * NV + v];
                }
              }
              if (split) {
                double Ds = o->D[ijk[ci] * n + al] + Dh;
                const double *J1 = o->Ja + (e * n3 + node) * 9 + ci * 3;
                const double *J2 = o->Ja + (e * n3 + src) * 9 + ci * 3;
                double m[3] = {0.5 * (J1[0] + J2[0]), 0.5 * (J1[1] + J2[1]), 0.5 * (J1[2] + J2[2])};
                double Fs[NV];
                two_point(o, o->Ui + (e * n3 + node) * NV, o->prim + (e * n3 + node) * 6,
                          o->Ui + (e * n3 + src) * NV, o->prim + (e * n3 + src) * 6, m, Fs);
                for (int v = 0; v < NV; ++v) Va[node * NV + v] += Ds * Fs[v];
              }
            }
        }
    free(Fc); free(Fa); free(Fv);
    if (split && !blend)
      for (int a = 0; a < n3 * NV; ++a) Vt[a] = Va[a] + Vv[a];
    if (blend) {
      /* (1 - alpha) V_DG,adv + alpha V_FV + V_DG,visc */
      double al = o->alpha[e];
      double *Vf = o->Vfv + e * n3 * NV;
      fv_volume(o, e, Vf);
      for (int a = 0; a < n3 * NV; ++a) Vt[a] = (1.0 - al) * Va[a] + al * Vf[a] + Vv[a];
    }
  }

  /* SurfInt: the loop over faces of the CPU algorithm; every element face
   * holds +f* (primary) or -f* (replica) at its own node, added with
   * l-hat^pm along the face-normal line. */
#pragma omp parallel for schedule(static)
  for (long e = 0; e < E; ++e)
    for (int f = 0; f < 6; ++f) {
      int d0 = f / 2;
      const double *lh = (f % 2) ? o->lhp : o->lhm;
      double *Vt = o->V + e * n3 * NV;
      for (int q = 0; q < n; ++q)
        for (int p = 0; p < n; ++p) {
          const double *ff = o->faceF + ((e * 6 + f) * n2 + p + n * q) * NV;
          for (int l = 0; l < n; ++l) {
            int node = line_node(n, d0, l, p, q);
            for (int v = 0; v < NV; ++v) Vt[node * NV + v] += ff[v] * lh[l];
          }
        }
    }

  /* ApplyJac: Ut = -Ut / J, plus the manufactured-solution source */
  double g = o->gamma;
#pragma omp parallel for schedule(static)
  for (long e = 0; e < E; ++e)
    for (int a = 0; a < n3; ++a) {
      double Jv = o->J[e * n3 + a];
      double src[NV] = {0, 0, 0, 0, 0};
      if (o->source == 1) {
        /* rho = 2 + 0.1 sin(pi(x+y+z-t)), u = v = w = 1, p = rho: source
         * 0.1 pi cos(.) (2, 3, 3, 3, 2(3 gamma - 2)/(gamma - 1)) */
        const double *X = o->Xs + (e * n3 + a) * 3;
        double c = 0.1 * M_PI * cos(M_PI * (X[0] + X[1] + X[2] - t));
        src[0] = 2.0 * c; src[1] = 3.0 * c; src[2] = 3.0 * c; src[3] = 3.0 * c;
        src[4] = 2.0 * (3.0 * g - 2.0) / (g - 1.0) * c;
      }
      for (int v = 0; v < NV; ++v)
        Utsoa[((long)v * E + e) * n3 + a] = -o->V[(e * n3 + a) * NV + v] / Jv + src[v];
    }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Sec. 2.2 "Time integration": the five-stage fourth-order low-storage      */
/* Runge-Kutta scheme of Carpenter and Kennedy (2N storage).                 */
/* ------------------------------------------------------------------------ */
static const double RK_A[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                               -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
static const double RK_B[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                               1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                               2277821191437.0 / 14882151754819.0};
static const double RK_C[5] = {0.0, 1432997174477.0 / 9575080441755.0, 2526269341429.0 / 6820363962896.0,
                               2006345519317.0 / 3224310063776.0, 2802321613138.0 / 2924317926251.0};

/* The fourteen-stage fourth-order 2N-storage scheme of Niegemann, Diehl and
 * Busch (2012), the paper's choice for its application runs (Sec. 2.2 "Time
 * integration"): its stability region is stretched along the imaginary axis
 * for convection-dominated problems.  Published 16-digit coefficients. */
static const double RK14_A[14] = {0.0, -0.7188012108672410, -0.7785331173421570, -0.0053282796654044,
                                  -0.8552979934029281, -3.9564138245774565, -1.5780575380587385,
                                  -2.0837094552574054, -0.7483334182761610, -0.7032861106563359,
                                  0.0013917096117681, -0.0932075369637460, -0.9514200470875948,
                                  -7.1151571693922548};
static const double RK14_B[14] = {0.0367762454319673, 0.3136296607553959, 0.1531848691869027, 0.0030097086818182,
                                  0.3326293790646110, 0.2440251405350864, 0.3718879239592277, 0.6204126221582444,
                                  0.1524043173028741, 0.0760894927419266, 0.0077604214040978, 0.0024647284755382,
                                  0.0780348340049386, 5.5059777270269628};
static const double RK14_C[14] = {0.0, 0.0367762454319673, 0.1249685262725025, 0.2446177702277698,
                                  0.2476149531070420, 0.2969311120382472, 0.3978149645802642, 0.5270854589440328,
                                  0.6981269994175695, 0.8190890835352128, 0.8527059887098624, 0.8604711817462826,
                                  0.8627060376969976, 0.8734213127600976};

void orc_rk_coefficients(double *A, double *B, double *C) {
  for (int s = 0; s < 5; ++s) { A[s] = RK_A[s]; B[s] = RK_B[s]; C[s] = RK_C[s]; }
}

/* coefficients of scheme 0 (five stages) or 1 (fourteen); returns the stage count */
int orc_rk_scheme(int scheme, double *A, double *B, double *C) {
  int ns = scheme == 1 ? 14 : 5;
  for (int s = 0; s < ns; ++s) {
    A[s] = scheme == 1 ? RK14_A[s] : RK_A[s];
    B[s] = scheme == 1 ? RK14_B[s] : RK_B[s];
    C[s] = scheme == 1 ? RK14_C[s] : RK_C[s];
  }
  return ns;
}

/* advance U (state layout [var][elem][node]) by nsteps steps of size dt with
 * the low-storage scheme the parameters select: per stage s,
 * du = A_s du + dt R(U, t + c_s dt), U = U + B_s du (A_1 = 0) */
int orc_advance(orc *o, double *U, double t0, double dt, int nsteps) {
  long tot = (long)NV * o->E * o->n3;
  double *du = ALLOC(double, tot), *R = ALLOC(double, tot);
  double A[14], B[14], Cc[14];
  int ns = orc_rk_scheme(o->rk_scheme, A, B, Cc);
  double t = t0;
  for (int st = 0; st < nsteps; ++st) {
    for (int s = 0; s < ns; ++s) {
      orc_rhs(o, U, t + Cc[s] * dt, R);
#pragma omp parallel for schedule(static)
      for (long a = 0; a < tot; ++a) {
        du[a] = A[s] * du[a] + dt * R[a];
        U[a] = U[a] + B[s] * du[a];
      }
    }
    t = t0 + (st + 1) * dt;
  }
  free(du); free(R);
  return 0;
}

/* blending factors of the last RHS evaluation, or freeze them */
void orc_get_alpha(const orc *o, double *alpha) { memcpy(alpha, o->alpha, sizeof(double) * o->E); }
void orc_set_alpha(orc *o, const double *alpha) {
  if (alpha) { memcpy(o->alpha, alpha, sizeof(double) * o->E); o->alpha_frozen = 1; }
  else o->alpha_frozen = 0;
}

/* Integrals by the collocated quadrature: mass, momentum (3), energy, kinetic
 * energy (Sec. 5.2, normalised by the domain volume, rho0 = U0 = 1) and |Omega|. */
void orc_integrals(const orc *o, const double *U, double *out) {
  int n = o->n, n3 = o->n3;
  long E = o->E;
  double s[7] = {0, 0, 0, 0, 0, 0, 0};
  for (long e = 0; e < E; ++e)
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
          int a = nidx(n, i, j, k);
          double wJ = o->w[i] * o->w[j] * o->w[k] * o->J[e * n3 + a];
          double u[NV];
          for (int v = 0; v < NV; ++v) u[v] = U[((long)v * E + e) * n3 + a];
          for (int v = 0; v < NV; ++v) s[v] += wJ * u[v];
          s[5] += wJ * 0.5 * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) / u[0];
          s[6] += wJ;
        }
  for (int v = 0; v < 5; ++v) out[v] = s[v];
  out[5] = s[5] / s[6];
  out[6] = s[6];
}

/* Time step from the advective and viscous spectral estimates (the paper does
 * not give one): dt = min(CFL * 2/((2N+1) sum_i lambda_i), DFL * 4/((N+1)^4 nu sum_i (|Ja^i|/J)^2)). */
double orc_stable_dt(const orc *o, const double *U, double cfl, double dfl) {
  int n3 = o->n3, N = o->N;
  long E = o->E;
  double dta = 1e300, dtv = 1e300;
  double g = o->gamma;
  for (long e = 0; e < E; ++e)
    for (int a = 0; a < n3; ++a) {
      double Uv[NV], P[6];
      for (int v = 0; v < NV; ++v) Uv[v] = U[((long)v * E + e) * n3 + a];
      cons_to_prim(o, Uv, P);
      double c = sqrt(g * P[4] / P[0]);
      const double *Ja = o->Ja + (e * n3 + a) * 9;
      double Jv = o->J[e * n3 + a];
      double lam = 0.0, vis = 0.0;
      for (int i = 0; i < 3; ++i) {
        double un = P[1] * Ja[i * 3] + P[2] * Ja[i * 3 + 1] + P[3] * Ja[i * 3 + 2];
        double nj = sqrt(Ja[i * 3] * Ja[i * 3] + Ja[i * 3 + 1] * Ja[i * 3 + 1] + Ja[i * 3 + 2] * Ja[i * 3 + 2]);
        lam += (fabs(un) + c * nj) / Jv;
        vis += (nj / Jv) * (nj / Jv);
      }
      double t1 = cfl * 2.0 / ((2.0 * N + 1.0) * lam);
      if (t1 < dta) dta = t1;
      if (o->viscous && o->mu > 0.0) {
        double nu = fmax(4.0 / 3.0, g / o->Pr) * viscosity(o, P[5]) / P[0];
        double t2 = dfl * 4.0 / (pow(N + 1.0, 4) * nu * vis);
        if (t2 < dtv) dtv = t2;
      }
    }
  return fmin(dta, dtv);
}

/* ---- accessors for the pins ---- */
int orc_n(const orc *o) { return o->n; }
void orc_basis(const orc *o, double *x, double *w, double *D, double *Dhat, double *lhm, double *lhp,
               double *lm, double *lp) {
  int n = o->n;
  memcpy(x, o->x, sizeof(double) * n);
  memcpy(w, o->w, sizeof(double) * n);
  memcpy(D, o->D, sizeof(double) * n * n);
  memcpy(Dhat, o->Dhat, sizeof(double) * n * n);
  memcpy(lhm, o->lhm, sizeof(double) * n);
  memcpy(lhp, o->lhp, sizeof(double) * n);
  memcpy(lm, o->lm, sizeof(double) * n);
  memcpy(lp, o->lp, sizeof(double) * n);
}
/* Ja [E][n3][3][3], J [E][n3], nS [E][6][n2][3], Xs [E][n3][3], fmap [E][6][n2] */
void orc_geometry(const orc *o, double *Ja, double *J, double *nS, double *Xs, int *fmap) {
  long E = o->E;
  if (Ja) memcpy(Ja, o->Ja, sizeof(double) * E * o->n3 * 9);
  if (J) memcpy(J, o->J, sizeof(double) * E * o->n3);
  if (nS) memcpy(nS, o->nS, sizeof(double) * E * 6 * o->n2 * 3);
  if (Xs) memcpy(Xs, o->Xs, sizeof(double) * E * o->n3 * 3);
  if (fmap) memcpy(fmap, o->fmap, sizeof(int) * E * 6 * o->n2);
}
/* metric identity sum_i d/dxi^i (Ja^i_d) at the solution nodes, [E][n3][3] */
void orc_metric_identity(const orc *o, double *out) {
  int n = o->n, n3 = o->n3;
  for (long e = 0; e < o->E; ++e) {
    double *tmp = ALLOC(double, n3);
    for (int a = 0; a < n3 * 3; ++a) out[e * n3 * 3 + a] = 0.0;
    for (int i = 0; i < 3; ++i)
      for (int d = 0; d < 3; ++d) {
        deriv_dir(n, o->D, i, o->Ja + e * n3 * 9 + i * 3 + d, 9, tmp, 1);
        for (int a = 0; a < n3; ++a) out[(e * n3 + a) * 3 + d] += tmp[a];
      }
    free(tmp);
  }
}
/* single-point Riemann solver, for the pins */
void orc_riemann(orc *o, int which, const double *UL, const double *UR, const double *nv, double *F) {
  double PL[6], PR[6];
  cons_to_prim(o, UL, PL);
  cons_to_prim(o, UR, PR);
  riemann(o, which, UL, PL, UR, PR, nv, F);
}
/* the FV subcell volume term alone for element e on state U, [n3][5] */
void orc_fv_volume(orc *o, const double *Usoa, long e, double *out) {
  int n3 = o->n3;
  long E = o->E;
  for (int a = 0; a < n3; ++a) {
    double Uv[NV];
    for (int v = 0; v < NV; ++v) Uv[v] = Usoa[((long)v * E + e) * n3 + a];
    cons_to_prim(o, Uv, o->prim + (e * n3 + a) * 6);
  }
  fv_volume(o, e, out);
}
/* indicator value alpha of element e for state U */
double orc_indicator(orc *o, const double *Usoa, long e) {
  int n3 = o->n3;
  long E = o->E;
  for (int a = 0; a < n3; ++a) {
    double Uv[NV];
    for (int v = 0; v < NV; ++v) Uv[v] = Usoa[((long)v * E + e) * n3 + a];
    cons_to_prim(o, Uv, o->prim + (e * n3 + a) * 6);
  }
  return indicator_alpha(o, e);
}

/* Sec. 5.2 dissipation rates from the lifted gradients g of an evaluation of
 * the operator on U: out[0] = (1/|Omega|) sum w J mu(T) omega.omega and
 * out[1] = (4/(3 |Omega|)) sum w J mu(T) (div u)^2, omega = curl u.  With
 * rho0 = U0 = L = 1 these are the paper's solenoidal and dilatational rates
 * (its mu(T)/(mu0 Re) is mu(T)).  Needs the viscous operator (returns -1
 * otherwise). */
int orc_dissipation(orc *o, const double *Usoa, double *out) {
  if (!o->viscous) return -1;
  int n = o->n, n3 = o->n3;
  long E = o->E, tot = (long)NV * E * n3;
  double *R = ALLOC(double, tot);
  orc_rhs(o, Usoa, 0.0, R);
  free(R);
  double sS = 0.0, sD = 0.0, vol = 0.0;
  for (long e = 0; e < E; ++e)
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
          int a = nidx(n, i, j, k);
          double wJ = o->w[i] * o->w[j] * o->w[k] * o->J[e * n3 + a];
          const double *g = o->G + (e * n3 + a) * 3 * NL; /* g[d*NL + v] = d(prim v)/dx_d */
          double mu = viscosity(o, o->prim[(e * n3 + a) * 6 + 5]);
          double wx = g[1 * NL + 2] - g[2 * NL + 1];  /* dw/dy - dv/dz */
          double wy = g[2 * NL + 0] - g[0 * NL + 2];  /* du/dz - dw/dx */
          double wz = g[0 * NL + 1] - g[1 * NL + 0];  /* dv/dx - du/dy */
          double dv = g[0 * NL + 0] + g[1 * NL + 1] + g[2 * NL + 2];
          sS += wJ * mu * (wx * wx + wy * wy + wz * wz);
          sD += wJ * mu * dv * dv;
          vol += wJ;
        }
  out[0] = sS / vol;
  out[1] = 4.0 / 3.0 * sD / vol;
  return 0;
}

/* single-point two-point volume flux along m, for the pins */
void orc_two_point(orc *o, int which, const double *UL, const double *UR, const double *m, double *F) {
  double PL[6], PR[6];
  cons_to_prim(o, UL, PL);
  cons_to_prim(o, UR, PR);
  if (which == 2) two_point_mean(UL, PL, UR, PR, m, F);
  else two_point_kep(UL, PL, UR, PR, m, F);
}

/* viscosity at temperature T under the current law, for the pins */
double orc_viscosity(const orc *o, double T) { return viscosity(o, T); }
