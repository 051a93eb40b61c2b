// setup.cpp -- host-side set-up of the DGSEM operator in FP64: nodes and
// weights, the 1-D operators of the semi-discrete form, the curl-form metric
// terms and face normals, and the face connectivity with its checks.
//
// Paper (GALAEXI, arXiv 2404.12703):
//   Sec. 2.2 "Solution Representation": Lagrange basis on Gauss or Gauss-Lobatto nodes.
//   Sec. 2.2 Eq. dgsem: D-hat_ij = -(w_j/w_i) l_i'(x_j) (the weight ratio as in
//     Kopriva's book; the printed ratio is inverted), l-hat^pm_i = l_i(+-1)/w_i.
//   Sec. 2.2 "Mapping the Equations": Ja^i_n = -e_i . curl_xi(x_l grad_xi x_m).
//   Sec. 2.3: subcell interfaces at the cumulative Lobatto weights.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <thread>

#include "dg_internal.h"

namespace dg {

namespace {

// Legendre P_k and P_k' at s (Bonnet recurrence)
void legendre_pair(int k, double s, double &P, double &dP) {
  double pm1 = 1.0, p = s;
  if (k == 0) {
    P = 1.0;
    dP = 0.0;
    return;
  }
  for (int m = 1; m < k; ++m) {
    double pn = ((2 * m + 1) * s * p - m * pm1) / (m + 1);
    pm1 = p;
    p = pn;
  }
  P = p;
  // P_k' = k (s P_k - P_{k-1}) / (s^2 - 1), away from the end points
  dP = (std::fabs(std::fabs(s) - 1.0) < 1e-14) ? 0.5 * k * (k + 1) * std::pow(s, k + 1) : k * (s * p - pm1) / (s * s - 1.0);
}

void gauss(int N, std::vector<double> &x, std::vector<double> &w) {
  int n = N + 1;
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int k = 0; k < (n + 1) / 2; ++k) {
    // Tricomi-type initial guess for the k-th largest root of P_n
    double s = std::cos(M_PI * (k + 0.75) / (n + 0.5));
    for (int it = 0; it < 60; ++it) {
      double P, dP;
      legendre_pair(n, s, P, dP);
      double ds = P / dP;
      s -= ds;
      if (std::fabs(ds) < 1e-17) break;
    }
    double P, dP;
    legendre_pair(n, s, P, dP);
    double wk = 2.0 / ((1.0 - s * s) * dP * dP);
    x[n - 1 - k] = s;
    x[k] = -s;
    w[n - 1 - k] = wk;
    w[k] = wk;
  }
  if (n % 2) x[n / 2] = 0.0;
}

}  // namespace

void lobatto(int N, std::vector<double> &x, std::vector<double> &w) {
  int n = N + 1;
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  x[0] = -1.0;
  x[N] = 1.0;
  // interior nodes: roots of q = P_{N+1} - P_{N-1} = (2N+1)/(N(N+1)) (x^2-1) P_N',
  // with q' = (2N+1) P_N
  for (int k = 1; k <= N / 2; ++k) {
    double s = std::cos(M_PI * k / N);
    for (int it = 0; it < 60; ++it) {
      double Pa, dPa, Pb, dPb, Pn, dPn;
      legendre_pair(N + 1, s, Pa, dPa);
      legendre_pair(N - 1, s, Pb, dPb);
      legendre_pair(N, s, Pn, dPn);
      double ds = (Pa - Pb) / ((2.0 * N + 1.0) * Pn);
      s -= ds;
      if (std::fabs(ds) < 1e-17) break;
    }
    x[N - k] = s;
    x[k] = -s;
  }
  if (n % 2) x[N / 2] = 0.0;
  for (int k = 0; k < n; ++k) {
    double P, dP;
    legendre_pair(N, x[k], P, dP);
    w[k] = 2.0 / (N * (N + 1.0) * P * P);
  }
}

namespace {

// barycentric weights lambda_j = 1 / prod_{k != j} (x_j - x_k)
std::vector<double> bary(const std::vector<double> &x) {
  int n = (int)x.size();
  std::vector<double> lam(n, 1.0);
  for (int j = 0; j < n; ++j)
    for (int k = 0; k < n; ++k)
      if (k != j) lam[j] /= (x[j] - x[k]);
  return lam;
}

// values l_j(s) of all basis polynomials at s, barycentric form
void lagrange_values(const std::vector<double> &x, const std::vector<double> &lam, double s,
                     std::vector<double> &out) {
  int n = (int)x.size();
  out.assign(n, 0.0);
  for (int j = 0; j < n; ++j)
    if (s == x[j]) {
      out[j] = 1.0;
      return;
    }
  double den = 0.0;
  for (int j = 0; j < n; ++j) den += lam[j] / (s - x[j]);
  for (int j = 0; j < n; ++j) out[j] = lam[j] / (s - x[j]) / den;
}

// M[b][a] = l_a(t_b)
std::vector<double> interp(const std::vector<double> &from, const std::vector<double> &to) {
  std::vector<double> lam = bary(from), row;
  std::vector<double> M(to.size() * from.size());
  for (size_t b = 0; b < to.size(); ++b) {
    lagrange_values(from, lam, to[b], row);
    for (size_t a = 0; a < from.size(); ++a) M[b * from.size() + a] = row[a];
  }
  return M;
}

// D_ij = l_j'(x_i) = (lam_j / lam_i) / (x_i - x_j), D_ii = -sum_{j != i} D_ij
std::vector<double> diffmat(const std::vector<double> &x) {
  int n = (int)x.size();
  std::vector<double> lam = bary(x), D(n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      D[i * n + j] = (lam[j] / lam[i]) / (x[i] - x[j]);
      s += D[i * n + j];
    }
    D[i * n + i] = -s;
  }
  return D;
}

}  // namespace

Basis make_basis(int N, int nodes) {
  Basis b;
  b.N = N;
  b.n = N + 1;
  b.nodes = nodes;
  int n = b.n;
  if (nodes == 0) gauss(N, b.x, b.w);
  else lobatto(N, b.x, b.w);
  b.D = diffmat(b.x);
  b.Dhat.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) b.Dhat[i * n + j] = -(b.w[j] / b.w[i]) * b.D[j * n + i];
  std::vector<double> lam = bary(b.x);
  lagrange_values(b.x, lam, -1.0, b.lm);
  lagrange_values(b.x, lam, 1.0, b.lp);
  b.lhm.resize(n);
  b.lhp.resize(n);
  for (int i = 0; i < n; ++i) {
    b.lhm[i] = b.lm[i] / b.w[i];
    b.lhp[i] = b.lp[i] / b.w[i];
  }
  b.xhalf.assign(n + 1, -1.0);
  for (int m = 0; m < n; ++m) b.xhalf[m + 1] = b.xhalf[m] + b.w[m];
  // inverse of V_ia = sqrt((2a+1)/2) P_a(x_i): by discrete orthogonality of the
  // Legendre polynomials under the nodal quadrature, (V^-1)_ai = w_i sqrt((2a+1)/2) P_a(x_i) / gamma_a,
  // with gamma_a = sum_i w_i ((2a+1)/2) P_a(x_i)^2 (= 1 except the top Lobatto mode).
  b.Vinv.assign(n * n, 0.0);
  for (int a = 0; a < n; ++a) {
    double ga = 0.0;
    std::vector<double> phi(n);
    for (int i = 0; i < n; ++i) {
      double P, dP;
      legendre_pair(a, b.x[i], P, dP);
      phi[i] = std::sqrt((2.0 * a + 1.0) / 2.0) * P;
      ga += b.w[i] * phi[i] * phi[i];
    }
    for (int i = 0; i < n; ++i) b.Vinv[a * n + i] = b.w[i] * phi[i] / ga;
  }
  return b;
}

std::vector<double> basis_block(const Basis &b) {
  int n = b.n;
  BasisOffsets o(n);
  std::vector<double> blk(o.total, 0.0);
  std::copy(b.Dhat.begin(), b.Dhat.end(), blk.begin() + o.Dhat);
  std::copy(b.D.begin(), b.D.end(), blk.begin() + o.D);
  std::copy(b.Vinv.begin(), b.Vinv.end(), blk.begin() + o.Vinv);
  std::copy(b.lm.begin(), b.lm.end(), blk.begin() + o.lm);
  std::copy(b.lp.begin(), b.lp.end(), blk.begin() + o.lp);
  std::copy(b.lhm.begin(), b.lhm.end(), blk.begin() + o.lhm);
  std::copy(b.lhp.begin(), b.lhp.end(), blk.begin() + o.lhp);
  std::copy(b.w.begin(), b.w.end(), blk.begin() + o.w);
  std::copy(b.x.begin(), b.x.end(), blk.begin() + o.x);
  std::copy(b.xhalf.begin(), b.xhalf.end(), blk.begin() + o.xhalf);
  return blk;
}

namespace {

template <class F>
void parallel_for(int64_t count, F &&fn) {
  unsigned nt = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
  if (count < 64) nt = 1;
  std::vector<std::thread> th;
  int64_t chunk = (count + nt - 1) / nt;
  for (unsigned t = 0; t < nt; ++t) {
    int64_t b = t * chunk, e = std::min<int64_t>(count, b + chunk);
    if (b >= e) break;
    th.emplace_back([=, &fn] {
      for (int64_t i = b; i < e; ++i) fn(i);
    });
  }
  for (auto &x : th) x.join();
}

inline int vid(int n, int i, int j, int k) { return i + n * (j + n * k); }

// node of index l along direction d and face coordinates (p,q)
inline int lnode(int n, int d, int l, int p, int q) {
  return d == 0 ? vid(n, l, p, q) : (d == 1 ? vid(n, p, l, q) : vid(n, p, q, l));
}

// y = (A along direction d) x on an n^3 block (A is n x n, row-major)
void apply_dir(int n, const double *A, int d, const double *x, double *y) {
  for (int q = 0; q < n; ++q)
    for (int p = 0; p < n; ++p)
      for (int l = 0; l < n; ++l) {
        double s = 0.0;
        for (int a = 0; a < n; ++a) s += A[l * n + a] * x[lnode(n, d, a, p, q)];
        y[lnode(n, d, l, p, q)] = s;
      }
}

// tensor interpolation of a scalar field from an m^3 to an n^3 grid (M is n x m)
void tensor_interp(int m, int n, const double *M, const double *x, double *y) {
  std::vector<double> a((size_t)n * m * m), b((size_t)n * n * m);
  for (int k = 0; k < m; ++k)
    for (int j = 0; j < m; ++j)
      for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int r = 0; r < m; ++r) s += M[i * m + r] * x[r + m * (j + m * k)];
        a[i + n * (j + m * k)] = s;
      }
  for (int k = 0; k < m; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int r = 0; r < m; ++r) s += M[j * m + r] * a[i + n * (r + m * k)];
        b[i + n * (j + n * k)] = s;
      }
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int r = 0; r < m; ++r) s += M[k * m + r] * b[i + n * (j + n * r)];
        y[i + n * (j + n * k)] = s;
      }
}

}  // namespace

int build_geometry(const Basis &b, const dg_mesh &m, Geometry &g, std::string &err) {
  const int N = b.N, n = b.n, n2 = n * n, n3 = n2 * n;
  const int64_t E = m.n_elems;
  const int ng = m.n_geo + 1, ng3 = ng * ng * ng;
  std::vector<double> xl, wl, xgeo, wgeo;
  lobatto(N, xl, wl);
  lobatto(m.n_geo, xgeo, wgeo);
  const std::vector<double> Mgeo = interp(xgeo, xl);  // LGL(n_geo) -> LGL(N)
  const std::vector<double> Ml2s = interp(xl, b.x);   // LGL(N) -> solution nodes
  const std::vector<double> DL = diffmat(xl);
  g.Ja.assign((size_t)9 * E * n3, 0.0);
  g.J.assign((size_t)E * n3, 0.0);
  g.Xs.assign((size_t)3 * E * n3, 0.0);
  std::vector<double> nsRaw((size_t)3 * E * 6 * n2, 0.0);  // own outward n*shat per face node

  parallel_for(E, [&](int64_t e) {
    // geometry on LGL(N), element-local origin for the curl form
    double X[3][1000], dX[3][3][1000];  // X[m][node], dX[j][m][node] = d x_m / d xi_j
    double Xsh[3][1000], tmp[1000], V[1000], dV[1000];
    for (int c = 0; c < 3; ++c) tensor_interp(ng, n, Mgeo.data(), m.x_geo + ((size_t)e * 3 + c) * ng3, X[c]);
    for (int c = 0; c < 3; ++c)
      for (int a = 0; a < n3; ++a) Xsh[c][a] = X[c][a] - X[c][0];
    for (int j = 0; j < 3; ++j)
      for (int c = 0; c < 3; ++c) apply_dir(n, DL.data(), j, X[c], dX[j][c]);
    // Ja^i_nn on LGL(N):  -(curl_xi (x_l grad x_m))_i,  (nn, m, l) cyclic
    double JaL[3][3][1000];  // [i][nn][node]
    for (int nn = 0; nn < 3; ++nn) {
      int mm = (nn + 1) % 3, ll = (nn + 2) % 3;
      for (int i = 0; i < 3; ++i) {
        int bb = (i + 1) % 3, cc = (i + 2) % 3;
        // (curl W)_i = d_bb W_cc - d_cc W_bb,  W_j = x_ll d_j x_mm
        for (int a = 0; a < n3; ++a) V[a] = Xsh[ll][a] * dX[cc][mm][a];
        apply_dir(n, DL.data(), bb, V, dV);
        for (int a = 0; a < n3; ++a) JaL[i][nn][a] = -dV[a];
        for (int a = 0; a < n3; ++a) V[a] = Xsh[ll][a] * dX[bb][mm][a];
        apply_dir(n, DL.data(), cc, V, dV);
        for (int a = 0; a < n3; ++a) JaL[i][nn][a] += dV[a];
      }
    }
    // to the solution nodes
    for (int i = 0; i < 3; ++i)
      for (int d = 0; d < 3; ++d) {
        tensor_interp(n, n, Ml2s.data(), JaL[i][d], tmp);
        for (int a = 0; a < n3; ++a) g.Ja[((size_t)(3 * i + d) * E + e) * n3 + a] = tmp[a];
      }
    for (int c = 0; c < 3; ++c) {
      tensor_interp(n, n, Ml2s.data(), X[c], tmp);
      for (int a = 0; a < n3; ++a) g.Xs[((size_t)c * E + e) * n3 + a] = tmp[a];
    }
    double A[3][3][1000];
    for (int j = 0; j < 3; ++j)
      for (int c = 0; c < 3; ++c) tensor_interp(n, n, Ml2s.data(), dX[j][c], A[j][c]);
    for (int a = 0; a < n3; ++a) {
      double det = A[0][0][a] * (A[1][1][a] * A[2][2][a] - A[1][2][a] * A[2][1][a]) -
                   A[0][1][a] * (A[1][0][a] * A[2][2][a] - A[1][2][a] * A[2][0][a]) +
                   A[0][2][a] * (A[1][0][a] * A[2][1][a] - A[1][1][a] * A[2][0][a]);
      g.J[(size_t)e * n3 + a] = det;
    }
    // face metrics: slice of Ja^d on the LGL face, interpolated in 2-D
    for (int f = 0; f < 6; ++f) {
      int d = f / 2;
      int l = (f & 1) ? n - 1 : 0;
      double sg = (f & 1) ? 1.0 : -1.0;
      for (int c = 0; c < 3; ++c) {
        double slice[100], half[100];
        for (int q = 0; q < n; ++q)
          for (int p = 0; p < n; ++p) slice[p + n * q] = JaL[d][c][lnode(n, d, l, p, q)];
        for (int q = 0; q < n; ++q)
          for (int p = 0; p < n; ++p) {
            double s = 0.0;
            for (int r = 0; r < n; ++r) s += Ml2s[p * n + r] * slice[r + n * q];
            half[p + n * q] = s;
          }
        for (int q = 0; q < n; ++q)
          for (int p = 0; p < n; ++p) {
            double s = 0.0;
            for (int r = 0; r < n; ++r) s += Ml2s[q * n + r] * half[p + n * r];
            nsRaw[((size_t)c * E * 6 + e * 6 + f) * n2 + p + n * q] = sg * s;
          }
      }
    }
  });

  // checks: Jacobian, symmetric connectivity, watertight faces
  for (int64_t e = 0; e < E; ++e)
    for (int a = 0; a < n3; ++a)
      if (!(g.J[(size_t)e * n3 + a] > 0.0)) {
        err = "element " + std::to_string(e) + ": Jacobian not positive at node " + std::to_string(a);
        return DG_EMESH;
      }
  g.conn.assign((size_t)E * 6, int2{0, 0});
  g.NS.assign((size_t)3 * E * 6 * n2, 0.0);
  for (int64_t e = 0; e < E; ++e)
    for (int f = 0; f < 6; ++f) {
      int64_t e2 = m.nbr_elem[e * 6 + f];
      int f2 = m.nbr_face[e * 6 + f], code = m.nbr_orient[e * 6 + f];
      char where[96];
      std::snprintf(where, sizeof where, "element %lld face %d: ", (long long)e, f);
      if (e2 < 0 || e2 >= E || f2 < 0 || f2 > 5 || code < 0 || code > 7) {
        err = std::string(where) + "neighbour out of range";
        return DG_EMESH;
      }
      if (m.nbr_elem[e2 * 6 + f2] != e || m.nbr_face[e2 * 6 + f2] != f) {
        err = std::string(where) + "neighbour table not symmetric";
        return DG_EMESH;
      }
      int back = m.nbr_orient[e2 * 6 + f2];
      for (int q = 0; q < n; ++q)
        for (int p = 0; p < n; ++p) {
          int pp, qq, p3, q3;
          orient_map(code, p, q, N, pp, qq);
          orient_map(back, pp, qq, N, p3, q3);
          if (p3 != p || q3 != q) {
            err = std::string(where) + "orientation codes of the two sides are not inverse";
            return DG_EMESH;
          }
        }
      bool primary = (e * 6 + f) < (e2 * 6 + f2);
      g.conn[e * 6 + f] = int2{(int)(e2 * 6 + f2), code | (primary ? 8 : 0)};
      double scale = 0.0, worst = 0.0;
      for (int q = 0; q < n; ++q)
        for (int p = 0; p < n; ++p) {
          int pp, qq;
          orient_map(code, p, q, N, pp, qq);
          for (int c = 0; c < 3; ++c) {
            double own = nsRaw[((size_t)c * E * 6 + e * 6 + f) * n2 + p + n * q];
            double oth = nsRaw[((size_t)c * E * 6 + e2 * 6 + f2) * n2 + pp + n * qq];
            scale = std::max(scale, std::fabs(own));
            worst = std::max(worst, std::fabs(own + oth));
            // the face flux uses the primary side's normal; the replica stores it negated
            g.NS[((size_t)c * E * 6 + e * 6 + f) * n2 + p + n * q] = primary ? own : -oth;
          }
        }
      if (worst > 1e-9 * scale) {
        err = std::string(where) + "faces not watertight (normals differ)";
        return DG_EMESH;
      }
    }
  return DG_OK;
}

}  // namespace dg
