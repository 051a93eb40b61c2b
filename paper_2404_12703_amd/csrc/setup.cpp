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

// Set-up arithmetic runs in x87 extended precision (T = long double) and is
// rounded once to double, so every stored set-up quantity is accurate to the
// last bit of its double value.
using xr = long double;

// Legendre P_k and P_k' at s (Bonnet recurrence)
template <class T>
void legendre_pair(int k, T s, T &P, T &dP) {
  T pm1 = 1.0, p = s;
  if (k == 0) {
    P = 1.0;
    dP = 0.0;
    return;
  }
  for (int m = 1; m < k; ++m) {
    T pn = ((2 * m + 1) * s * p - m * pm1) / (m + 1);
    pm1 = p;
    p = pn;
  }
  P = p;
  // P_k' = k (s P_k - P_{k-1}) / (s^2 - 1), away from the end points
  dP = (std::fabs(std::fabs(s) - T(1)) < T(1e-14)) ? T(0.5) * k * (k + 1) * std::pow(s, T(k + 1))
                                                   : k * (s * p - pm1) / (s * s - T(1));
}

const xr kPi = 3.141592653589793238462643383279502884L;

template <class T>
void gauss(int N, std::vector<T> &x, std::vector<T> &w) {
  int n = N + 1;
  x.assign(n, T(0));
  w.assign(n, T(0));
  for (int k = 0; k < (n + 1) / 2; ++k) {
    // Tricomi-type initial guess for the k-th largest root of P_n
    T s = std::cos(T(kPi) * (k + T(0.75)) / (n + T(0.5)));
    for (int it = 0; it < 60; ++it) {
      T P, dP;
      legendre_pair<T>(n, s, P, dP);
      T ds = P / dP;
      s -= ds;
      if (std::fabs(ds) < T(1e-19)) break;
    }
    T P, dP;
    legendre_pair<T>(n, s, P, dP);
    T wk = T(2) / ((T(1) - s * s) * dP * dP);
    x[n - 1 - k] = s;
    x[k] = -s;
    w[n - 1 - k] = wk;
    w[k] = wk;
  }
  if (n % 2) x[n / 2] = T(0);
}

template <class T>
void lobatto_t(int N, std::vector<T> &x, std::vector<T> &w) {
  int n = N + 1;
  x.assign(n, T(0));
  w.assign(n, T(0));
  x[0] = T(-1);
  x[N] = T(1);
  // interior nodes: roots of q = P_{N+1} - P_{N-1} = (2N+1)/(N(N+1)) (x^2-1) P_N',
  // with q' = (2N+1) P_N
  for (int k = 1; k <= N / 2; ++k) {
    T s = std::cos(T(kPi) * k / N);
    for (int it = 0; it < 60; ++it) {
      T Pa, dPa, Pb, dPb, Pn, dPn;
      legendre_pair<T>(N + 1, s, Pa, dPa);
      legendre_pair<T>(N - 1, s, Pb, dPb);
      legendre_pair<T>(N, s, Pn, dPn);
      T ds = (Pa - Pb) / ((T(2) * N + T(1)) * Pn);
      s -= ds;
      if (std::fabs(ds) < T(1e-19)) break;
    }
    x[N - k] = s;
    x[k] = -s;
  }
  if (n % 2) x[N / 2] = T(0);
  for (int k = 0; k < n; ++k) {
    T P, dP;
    legendre_pair<T>(N, x[k], P, dP);
    w[k] = T(2) / (N * (N + T(1)) * P * P);
  }
}

}  // namespace

void lobatto(int N, std::vector<double> &x, std::vector<double> &w) {
  std::vector<xr> xl, wl;
  lobatto_t<xr>(N, xl, wl);
  x.assign(xl.begin(), xl.end());
  w.assign(wl.begin(), wl.end());
}

namespace {

// barycentric weights lambda_j = 1 / prod_{k != j} (x_j - x_k)
template <class T>
std::vector<T> bary(const std::vector<T> &x) {
  int n = (int)x.size();
  std::vector<T> lam(n, T(1));
  for (int j = 0; j < n; ++j)
    for (int k = 0; k < n; ++k)
      if (k != j) lam[j] /= (x[j] - x[k]);
  return lam;
}

// values l_j(s) of all basis polynomials at s, barycentric form
template <class T>
void lagrange_values(const std::vector<T> &x, const std::vector<T> &lam, T s, std::vector<T> &out) {
  int n = (int)x.size();
  out.assign(n, T(0));
  for (int j = 0; j < n; ++j)
    if (s == x[j]) {
      out[j] = T(1);
      return;
    }
  T den = T(0);
  for (int j = 0; j < n; ++j) den += lam[j] / (s - x[j]);
  for (int j = 0; j < n; ++j) out[j] = lam[j] / (s - x[j]) / den;
}

// M[b][a] = l_a(t_b)
template <class T>
std::vector<T> interp(const std::vector<T> &from, const std::vector<T> &to) {
  std::vector<T> lam = bary(from), row;
  std::vector<T> M(to.size() * from.size());
  for (size_t b = 0; b < to.size(); ++b) {
    lagrange_values(from, lam, to[b], row);
    for (size_t a = 0; a < from.size(); ++a) M[b * from.size() + a] = row[a];
  }
  return M;
}

// D_ij = l_j'(x_i) = (lam_j / lam_i) / (x_i - x_j), D_ii = -sum_{j != i} D_ij
template <class T>
std::vector<T> diffmat(const std::vector<T> &x) {
  int n = (int)x.size();
  std::vector<T> lam = bary(x), D(n * n, T(0));
  for (int i = 0; i < n; ++i) {
    T s = T(0);
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
  std::vector<xr> x, w;
  if (nodes == 0) gauss<xr>(N, x, w);
  else lobatto_t<xr>(N, x, w);
  std::vector<xr> D = diffmat(x);
  auto rd = [](const std::vector<xr> &v) { return std::vector<double>(v.begin(), v.end()); };
  b.x = rd(x);
  b.w = rd(w);
  b.D = rd(D);
  b.Dhat.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) b.Dhat[i * n + j] = (double)(-(w[j] / w[i]) * D[j * n + i]);
  std::vector<xr> lam = bary(x), lm, lp;
  lagrange_values<xr>(x, lam, xr(-1), lm);
  lagrange_values<xr>(x, lam, xr(1), lp);
  b.lm = rd(lm);
  b.lp = rd(lp);
  b.lhm.resize(n);
  b.lhp.resize(n);
  for (int i = 0; i < n; ++i) {
    b.lhm[i] = (double)(lm[i] / w[i]);
    b.lhp[i] = (double)(lp[i] / w[i]);
  }
  b.xhalf.assign(n + 1, -1.0);
  for (int m = 0; m < n; ++m) b.xhalf[m + 1] = b.xhalf[m] + b.w[m];
  // inverse of V_ia = sqrt((2a+1)/2) P_a(x_i): by discrete orthogonality of the
  // Legendre polynomials under the nodal quadrature, (V^-1)_ai = w_i sqrt((2a+1)/2) P_a(x_i) / gamma_a,
  // with gamma_a = sum_i w_i ((2a+1)/2) P_a(x_i)^2 (= 1 except the top Lobatto mode).
  b.Vinv.assign(n * n, 0.0);
  for (int a = 0; a < n; ++a) {
    xr ga = 0.0;
    std::vector<xr> phi(n);
    for (int i = 0; i < n; ++i) {
      xr P, dP;
      legendre_pair<xr>(a, x[i], P, dP);
      phi[i] = std::sqrt((xr(2) * a + 1) / 2) * P;
      ga += w[i] * phi[i] * phi[i];
    }
    for (int i = 0; i < n; ++i) b.Vinv[a * n + i] = (double)(w[i] * phi[i] / ga);
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
template <class T>
void apply_dir(int n, const T *A, int d, const T *x, T *y) {
  for (int q = 0; q < n; ++q)
    for (int p = 0; p < n; ++p)
      for (int l = 0; l < n; ++l) {
        T s = T(0);
        for (int a = 0; a < n; ++a) s += A[l * n + a] * x[lnode(n, d, a, p, q)];
        y[lnode(n, d, l, p, q)] = s;
      }
}

// tensor interpolation of a scalar field from an m^3 to an n^3 grid (M is n x m)
template <class T, class S>
void tensor_interp(int m, int n, const T *M, const S *x, T *y) {
  std::vector<T> a((size_t)n * m * m), b((size_t)n * n * m);
  for (int k = 0; k < m; ++k)
    for (int j = 0; j < m; ++j)
      for (int i = 0; i < n; ++i) {
        T s = T(0);
        for (int r = 0; r < m; ++r) s += M[i * m + r] * T(x[r + m * (j + m * k)]);
        a[i + n * (j + m * k)] = s;
      }
  for (int k = 0; k < m; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        T s = T(0);
        for (int r = 0; r < m; ++r) s += M[j * m + r] * a[i + n * (r + m * k)];
        b[i + n * (j + n * k)] = s;
      }
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        T s = T(0);
        for (int r = 0; r < m; ++r) s += M[k * m + r] * b[i + n * (j + n * r)];
        y[i + n * (j + n * k)] = s;
      }
}

}  // namespace

int build_geometry(const Basis &b, const dg_mesh &m, Geometry &g, std::string &err) {
  const int N = b.N, n = b.n, n2 = n * n, n3 = n2 * n;
  const int64_t E = m.n_elems;
  const int ng = m.n_geo + 1, ng3 = ng * ng * ng;
  std::vector<xr> xl, wl, xgeo, wgeo, xs, ws;
  lobatto_t<xr>(N, xl, wl);
  lobatto_t<xr>(m.n_geo, xgeo, wgeo);
  if (b.nodes == 0) gauss<xr>(N, xs, ws);
  else lobatto_t<xr>(N, xs, ws);
  const std::vector<xr> Mgeo = interp(xgeo, xl);  // LGL(n_geo) -> LGL(N)
  const std::vector<xr> Ml2s = interp(xl, xs);    // LGL(N) -> solution nodes
  const std::vector<xr> DL = diffmat(xl);
  g.Ja.assign((size_t)9 * E * n3, 0.0);
  g.J.assign((size_t)E * n3, 0.0);
  g.Xs.assign((size_t)3 * E * n3, 0.0);
  std::vector<double> nsRaw((size_t)3 * E * 6 * n2, 0.0);  // own outward n*shat per face node

  parallel_for(E, [&](int64_t e) {
    // geometry on LGL(N), element-local origin for the curl form (a constant
    // shift leaves the curl form unchanged: the discrete curl of a discrete
    // gradient vanishes because the line derivatives commute)
    std::vector<xr> buf((size_t)(3 + 9 + 3 + 3 + 9 + 9) * n3 + 2 * n3);
    xr *X = buf.data(), *dX = X + 3 * n3, *Xsh = dX + 9 * n3, *tmp = Xsh + 3 * n3;
    xr *JaL = tmp + 3 * n3, *A = JaL + 9 * n3, *V = A + 9 * n3, *dV = V + n3;
    auto x_ = [&](int c) { return X + c * n3; };
    auto dx_ = [&](int j, int c) { return dX + (j * 3 + c) * n3; };
    auto ja_ = [&](int i, int c) { return JaL + (i * 3 + c) * n3; };
    for (int c = 0; c < 3; ++c) tensor_interp(ng, n, Mgeo.data(), m.x_geo + ((size_t)e * 3 + c) * ng3, x_(c));
    for (int c = 0; c < 3; ++c)
      for (int a = 0; a < n3; ++a) Xsh[c * n3 + a] = x_(c)[a] - x_(c)[0];
    for (int j = 0; j < 3; ++j)
      for (int c = 0; c < 3; ++c) apply_dir(n, DL.data(), j, x_(c), dx_(j, c));
    // Ja^i_nn on LGL(N):  -(curl_xi (x_l grad x_m))_i,  (nn, m, l) cyclic
    for (int nn = 0; nn < 3; ++nn) {
      int mm = (nn + 1) % 3, ll = (nn + 2) % 3;
      for (int i = 0; i < 3; ++i) {
        int bb = (i + 1) % 3, cc = (i + 2) % 3;
        // (curl W)_i = d_bb W_cc - d_cc W_bb,  W_j = x_ll d_j x_mm
        for (int a = 0; a < n3; ++a) V[a] = Xsh[ll * n3 + a] * dx_(cc, mm)[a];
        apply_dir(n, DL.data(), bb, V, dV);
        for (int a = 0; a < n3; ++a) ja_(i, nn)[a] = -dV[a];
        for (int a = 0; a < n3; ++a) V[a] = Xsh[ll * n3 + a] * dx_(bb, mm)[a];
        apply_dir(n, DL.data(), cc, V, dV);
        for (int a = 0; a < n3; ++a) ja_(i, nn)[a] += dV[a];
      }
    }
    // to the solution nodes
    for (int i = 0; i < 3; ++i)
      for (int d = 0; d < 3; ++d) {
        tensor_interp(n, n, Ml2s.data(), ja_(i, d), tmp);
        for (int a = 0; a < n3; ++a) g.Ja[((size_t)(3 * i + d) * E + e) * n3 + a] = (double)tmp[a];
      }
    for (int c = 0; c < 3; ++c) {
      tensor_interp(n, n, Ml2s.data(), x_(c), tmp);
      for (int a = 0; a < n3; ++a) g.Xs[((size_t)c * E + e) * n3 + a] = (double)tmp[a];
    }
    for (int j = 0; j < 3; ++j)
      for (int c = 0; c < 3; ++c) tensor_interp(n, n, Ml2s.data(), dx_(j, c), A + (j * 3 + c) * n3);
    auto A_ = [&](int j, int c, int a) { return A[(j * 3 + c) * n3 + a]; };
    for (int a = 0; a < n3; ++a) {
      xr det = A_(0, 0, a) * (A_(1, 1, a) * A_(2, 2, a) - A_(1, 2, a) * A_(2, 1, a)) -
               A_(0, 1, a) * (A_(1, 0, a) * A_(2, 2, a) - A_(1, 2, a) * A_(2, 0, a)) +
               A_(0, 2, a) * (A_(1, 0, a) * A_(2, 1, a) - A_(1, 1, a) * A_(2, 0, a));
      g.J[(size_t)e * n3 + a] = (double)det;
    }
    // face metrics: slice of Ja^d on the LGL face, interpolated in 2-D
    for (int f = 0; f < 6; ++f) {
      int d = f / 2;
      int l = (f & 1) ? n - 1 : 0;
      xr sg = (f & 1) ? 1.0L : -1.0L;
      for (int c = 0; c < 3; ++c) {
        xr slice[100], half[100];
        for (int q = 0; q < n; ++q)
          for (int p = 0; p < n; ++p) slice[p + n * q] = ja_(d, c)[lnode(n, d, l, p, q)];
        for (int q = 0; q < n; ++q)
          for (int p = 0; p < n; ++p) {
            xr sum = 0.0L;
            for (int r = 0; r < n; ++r) sum += Ml2s[p * n + r] * slice[r + n * q];
            half[p + n * q] = sum;
          }
        for (int q = 0; q < n; ++q)
          for (int p = 0; p < n; ++p) {
            xr sum = 0.0L;
            for (int r = 0; r < n; ++r) sum += Ml2s[q * n + r] * half[p + n * r];
            nsRaw[((size_t)c * E * 6 + e * 6 + f) * n2 + p + n * q] = (double)(sg * sum);
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
