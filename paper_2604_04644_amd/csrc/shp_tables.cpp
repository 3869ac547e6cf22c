// Host construction of the reference tables of libshp: 1D quadrature rules,
// modal basis functions and derivatives at the points, collocation
// differentiation matrices and the sum-factorisation column table.
//
// Quadrature (Sec. 2.1): Gauss-Jacobi zeros by Newton iteration on the Jacobi
// polynomial with deflation of the zeros already found, weights from the
// Christoffel closed form; Gauss-Lobatto-Legendre as the end points plus the
// Gauss-Jacobi(1,1) zeros, weights 2 / (Q (Q-1) P_{Q-1}(x)^2); Gauss-Radau-
// Jacobi as -1 plus the Gauss-Jacobi(a, b+1) zeros.
// Collocation derivative (Sec. 2.2, eq. dphitodh): barycentric form of the
// derivative of the Lagrange interpolant, D_ij = (l_j / l_i) / (x_i - x_j),
// D_ii = -sum_{j != i} D_ij.
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/shp.h"
#include "shp_internal.hpp"

namespace shp {

static double jac_p(int n, double a, double b, double x) {
  if (n == 0) return 1.0;
  double p0 = 1.0, p1 = 0.5 * (a - b + (a + b + 2.0) * x);
  for (int k = 2; k <= n; ++k) {
    const double c = 2.0 * k + a + b;
    const double a1 = 2.0 * k * (k + a + b) * (c - 2.0);
    const double a2 = (c - 1.0) * (a * a - b * b);
    const double a3 = (c - 2.0) * (c - 1.0) * c;
    const double a4 = 2.0 * (k + a - 1.0) * (k + b - 1.0) * c;
    const double p2 = ((a2 + a3 * x) * p1 - a4 * p0) / a1;
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

static double jac_dp(int n, double a, double b, double x) {
  if (n == 0) return 0.0;
  return 0.5 * (n + a + b + 1.0) * jac_p(n - 1, a + 1.0, b + 1.0, x);
}

void gauss_jacobi(int Q, double a, double b, double* x, double* w) {
  const double pi = 3.14159265358979323846;
  for (int k = 0; k < Q; ++k) {
    double r = -std::cos((2.0 * k + 1.0) * pi / (2.0 * Q));
    if (k > 0) r = 0.5 * (r + x[k - 1]);
    for (int it = 0; it < 100; ++it) {
      double defl = 0.0;
      for (int j = 0; j < k; ++j) defl += 1.0 / (r - x[j]);
      const double f = jac_p(Q, a, b, r);
      const double df = jac_dp(Q, a, b, r);
      const double step = f / (df - defl * f);
      r -= step;
      if (std::fabs(step) < 1e-17) break;
    }
    x[k] = r;
  }
  // sort ascending (Newton from ascending guesses normally keeps order)
  for (int i = 1; i < Q; ++i)
    for (int j = i; j > 0 && x[j] < x[j - 1]; --j) std::swap(x[j], x[j - 1]);
  const double lc = (a + b + 1.0) * std::log(2.0) + std::lgamma(Q + a + 1.0) + std::lgamma(Q + b + 1.0) -
                    std::lgamma(Q + a + b + 1.0) - std::lgamma(Q + 1.0);
  const double C = std::exp(lc);
  for (int i = 0; i < Q; ++i) {
    const double d = jac_dp(Q, a, b, x[i]);
    w[i] = C / ((1.0 - x[i] * x[i]) * d * d);
  }
}

void gauss_lobatto(int Q, double* x, double* w) {
  x[0] = -1.0;
  x[Q - 1] = 1.0;
  if (Q > 2) {
    std::vector<double> xi(Q - 2), wi(Q - 2);
    gauss_jacobi(Q - 2, 1.0, 1.0, xi.data(), wi.data());
    for (int i = 0; i < Q - 2; ++i) x[i + 1] = xi[i];
  }
  for (int i = 0; i < Q; ++i) {
    const double pl = jac_p(Q - 1, 0.0, 0.0, x[i]);
    w[i] = 2.0 / (Q * (Q - 1.0) * pl * pl);
  }
}

// Gauss-Radau-Jacobi with the node -1: for f of degree <= 2Q-2 write
// f(x) = f(-1) + (1 + x) g(x); g is integrated exactly under the weight
// (1-x)^a (1+x)^(b+1) by the (Q-1)-point Gauss-Jacobi(a, b+1) rule, so the other
// nodes are its zeros with weights w_i / (1 + x_i), and the weight of -1 is the
// closed form 2^(a+b+1) (b+1) G(b+1)^2 G(Q) G(Q+a) / (G(Q+b+1) G(Q+a+b+1)).
void gauss_radau_jacobi(int Q, double a, double b, double* x, double* w) {
  x[0] = -1.0;
  const double l0 = (a + b + 1.0) * std::log(2.0) + std::log(b + 1.0) + 2.0 * std::lgamma(b + 1.0) +
                    std::lgamma((double)Q) + std::lgamma(Q + a) - std::lgamma(Q + b + 1.0) - std::lgamma(Q + a + b + 1.0);
  w[0] = std::exp(l0);
  if (Q > 1) {
    gauss_jacobi(Q - 1, a, b + 1.0, x + 1, w + 1);
    for (int i = 1; i < Q; ++i) w[i] /= (1.0 + x[i]);
  }
}

void rule_1d(int Q, int alpha, int pts, double* x, double* w) {
  if (alpha == 0)
    gauss_lobatto(Q, x, w);
  else if (pts == SHP_PTS_RADAU)
    gauss_radau_jacobi(Q, (double)alpha, 0.0, x, w);
  else
    gauss_jacobi(Q, (double)alpha, 0.0, x, w);
}

// modified basis in one direction
static double fA(int p, double z) {
  if (p == 0) return 0.5 * (1.0 - z);
  if (p == 1) return 0.5 * (1.0 + z);
  return 0.25 * (1.0 - z) * (1.0 + z) * jac_p(p - 2, 1.0, 1.0, z);
}
static double fdA(int p, double z) {
  if (p == 0) return -0.5;
  if (p == 1) return 0.5;
  return -0.5 * z * jac_p(p - 2, 1.0, 1.0, z) + 0.25 * (1.0 - z) * (1.0 + z) * jac_dp(p - 2, 1.0, 1.0, z);
}
static double fC(int k, int r, double z) {
  if (k == 0) return fA(r, z);
  const double v0 = 0.5 * (1.0 - z);
  const double v0k = std::pow(v0, k);
  if (r == 0) return v0k;
  return v0k * 0.5 * (1.0 + z) * jac_p(r - 1, 2.0 * k - 1.0, 1.0, z);
}
static double fdC(int k, int r, double z) {
  if (k == 0) return fdA(r, z);
  const double v0 = 0.5 * (1.0 - z), v1 = 0.5 * (1.0 + z);
  const double v0km1 = std::pow(v0, k - 1);
  if (r == 0) return -0.5 * k * v0km1;
  const double J = jac_p(r - 1, 2.0 * k - 1.0, 1.0, z);
  const double dJ = jac_dp(r - 1, 2.0 * k - 1.0, 1.0, z);
  return -0.5 * k * v0km1 * v1 * J + v0km1 * v0 * (0.5 * J + v1 * dJ);
}

static void colloc_deriv(int Q, const double* x, double* D) {
  std::vector<double> l(Q);
  for (int j = 0; j < Q; ++j) {
    double p = 1.0;
    for (int k = 0; k < Q; ++k)
      if (k != j) p *= (x[j] - x[k]);
    l[j] = 1.0 / p;
  }
  for (int i = 0; i < Q; ++i) {
    double s = 0.0;
    for (int j = 0; j < Q; ++j) {
      if (j == i) continue;
      const double v = (l[j] / l[i]) / (x[i] - x[j]);
      D[i * Q + j] = v;
      s += v;
    }
    D[i * Q + i] = -s;
  }
}

void build_tables(int sh, int P, int pts, std::vector<double>& tab, std::vector<int>& itab) {
  const TabLayout L = tab_layout(sh, P);
  const int Q = L.Q, n = L.n;
  tab.assign(L.total, 0.0);
  double* z = tab.data() + L.z;
  double* w = tab.data() + L.w;
  for (int d = 0; d < 3; ++d) rule_1d(Q, alpha_dir(sh, d), pts, z + d * Q, w + d * Q);
  const double* z1 = z;
  const double* z2 = z + Q;
  const double* z3 = z + 2 * Q;
  for (int p = 0; p < n; ++p)
    for (int i = 0; i < Q; ++i) {
      tab[L.A1 + p * Q + i] = fA(p, z1[i]);
      tab[L.dA1 + p * Q + i] = fdA(p, z1[i]);
    }
  if (sh == TET) {
    for (int p = 0; p <= P; ++p)
      for (int q = 0; q <= P - p; ++q)
        for (int j = 0; j < Q; ++j) {
          tab[L.B2 + fam_index(P, p, q) * Q + j] = fC(p, q, z2[j]);
          tab[L.dB2 + fam_index(P, p, q) * Q + j] = fdC(p, q, z2[j]);
        }
  } else {
    for (int q = 0; q <= P; ++q)
      for (int j = 0; j < Q; ++j) {
        tab[L.B2 + q * Q + j] = fA(q, z2[j]);
        tab[L.dB2 + q * Q + j] = fdA(q, z2[j]);
      }
  }
  const int kmax = (sh == HEX) ? 0 : P;
  for (int k = 0; k <= kmax; ++k)
    for (int r = 0; r <= P - k; ++r)
      for (int kk = 0; kk < Q; ++kk) {
        tab[L.C3 + fam_index(P, k, r) * Q + kk] = fC(k, r, z3[kk]);
        tab[L.dC3 + fam_index(P, k, r) * Q + kk] = fdC(k, r, z3[kk]);
      }
  for (int d = 0; d < 3; ++d) colloc_deriv(Q, z + d * Q, tab.data() + L.D + d * Q * Q);

  // column table, p-major, q, with the running mode offset; then the columns
  // grouped by eta3 family kappa: family starts [P + 2] and the column order [NC]
  const int NC = num_cols(sh, P);
  itab.assign(NC * ICOL + (P + 2) + NC, 0);
  int c = 0, off = 0;
  for (int p = 0; p <= P; ++p)
    for (int q = 0; q < nq_of(sh, P, p); ++q) {
      int* ct = itab.data() + c * ICOL;
      ct[0] = p;
      ct[1] = q;
      ct[2] = off;
      ct[3] = col_len(sh, P, p, q);
      ct[4] = fam_index(P, kappa3(sh, p, q), 0);
      off += ct[3];
      ++c;
    }
  int* fst = itab.data() + NC * ICOL;
  int* perm = fst + (P + 2);
  int k = 0;
  for (int kap = 0; kap <= P; ++kap) {
    fst[kap] = k;
    for (int cc = 0; cc < NC; ++cc) {
      const int* ct = itab.data() + cc * ICOL;
      if (kappa3(sh, ct[0], ct[1]) == kap) perm[k++] = cc;
    }
  }
  fst[P + 1] = k;
}

// Dense reference matrices [B; d_1 B; d_2 B; d_3 B] at the quadrature points
// for the local-matrix strategy: row d*Q3p + q, column m; rows padded to a
// multiple of 16, columns to a multiple of 16 (zeros).  Each mode is a product
// of 1D functions of eta (the collapsed-vertex modes drop the factors of the
// collapsed coordinates), differentiated factor by factor.
// 1D factors of mode (p, q, r): every mode is a product a(eta1) b(eta2)
// c(eta3) of 1D functions; the collapsed-vertex modes drop the factors of the
// collapsed coordinates (constant 1).  Kinds: 0 = constant 1, 1 = A_a,
// 2 = C_{a,b}, 3 = v1.
struct Factor {
  int kind, a, b;
  bool operator==(const Factor& o) const { return kind == o.kind && a == o.a && b == o.b; }
};

static void mode_factors(int sh, int p, int q, int r, Factor f[3]) {
  if (sh == HEX) {
    f[0] = {1, p, 0}; f[1] = {1, q, 0}; f[2] = {1, r, 0};
  } else if (sh == PRISM) {
    if (p == 0 && r == 1) { f[0] = {0, 0, 0}; f[1] = {1, q, 0}; f[2] = {3, 0, 0}; }
    else { f[0] = {1, p, 0}; f[1] = {1, q, 0}; f[2] = {2, p, r}; }
  } else if (sh == PYR) {
    if (p == 0 && q == 0 && r == 1) { f[0] = {0, 0, 0}; f[1] = {0, 0, 0}; f[2] = {3, 0, 0}; }
    else { f[0] = {1, p, 0}; f[1] = {1, q, 0}; f[2] = {2, imax(p, q), r}; }
  } else {
    if (p == 0 && q == 0 && r == 1) { f[0] = {0, 0, 0}; f[1] = {0, 0, 0}; f[2] = {3, 0, 0}; }
    else if (p == 0 && q == 1) { f[0] = {0, 0, 0}; f[1] = {3, 0, 0}; f[2] = {2, 1, r}; }
    else { f[0] = {1, p, 0}; f[1] = {2, p, q}; f[2] = {2, p + q, r}; }
  }
}

static double factor_value(const Factor& f, double x, bool der) {
  switch (f.kind) {
    case 0: return der ? 0.0 : 1.0;
    case 1: return der ? fdA(f.a, x) : fA(f.a, x);
    case 2: return der ? fdC(f.a, f.b, x) : fC(f.a, f.b, x);
    default: return der ? 0.5 : 0.5 * (1.0 + x);
  }
}

// Dense reference matrices [B; d_1 B; d_2 B; d_3 B] at the quadrature points
// for the local-matrix strategy: row d*Q3p + q, column m; rows padded to a
// multiple of 16, columns to a multiple of 16 (zeros).  Each mode's 1D factors
// are differentiated factor by factor.
void build_dense_deriv(int sh, int P, int pts, std::vector<double>& dm, int& Q3p) {
  std::vector<double> tab;
  std::vector<int> itab;
  build_tables(sh, P, pts, tab, itab);
  const TabLayout L = tab_layout(sh, P);
  const int Q = P + 2, Q3 = Q * Q * Q;
  Q3p = (Q3 + 15) / 16 * 16;
  dm.assign((size_t)3 * Q3p * Q3p, 0.0);
  // point (i0, i1, i2) at (i0 Q + i1) Q + i2; D_d couples points that differ
  // in index d only, with the 1D entry D^(d)[i_d][j_d]
  for (int p0 = 0; p0 < Q3; ++p0) {
    const int i[3] = {p0 / (Q * Q), (p0 / Q) % Q, p0 % Q};
    for (int d = 0; d < 3; ++d)
      for (int j = 0; j < Q; ++j) {
        int k[3] = {i[0], i[1], i[2]};
        k[d] = j;
        const int p1 = (k[0] * Q + k[1]) * Q + k[2];
        dm[((size_t)d * Q3p + p0) * Q3p + p1] = tab[L.D + d * Q * Q + i[d] * Q + j];
      }
  }
}

void build_localmat(int sh, int P, int pts, std::vector<double>& bcat, int& Q3p, int& Kp) {
  const int Q = P + 2, Q3 = Q * Q * Q, NP = num_modes(sh, P);
  Q3p = (Q3 + 15) / 16 * 16;
  Kp = (NP + 15) / 16 * 16;
  bcat.assign((size_t)4 * Q3p * Kp, 0.0);
  std::vector<double> z(3 * Q), w(3 * Q);
  for (int d = 0; d < 3; ++d) rule_1d(Q, alpha_dir(sh, d), pts, z.data() + d * Q, w.data() + d * Q);
  int m = 0;
  for (int p = 0; p <= P; ++p)
    for (int q = 0; q < nq_of(sh, P, p); ++q)
      for (int r = 0; r < col_len(sh, P, p, q); ++r, ++m) {
        Factor f[3];
        mode_factors(sh, p, q, r, f);
        for (int i = 0; i < Q; ++i)
          for (int j = 0; j < Q; ++j)
            for (int k = 0; k < Q; ++k) {
              const int pt = (i * Q + j) * Q + k;
              const double x[3] = {z[i], z[Q + j], z[2 * Q + k]};
              double v[3], dv[3];
              for (int d = 0; d < 3; ++d) {
                v[d] = factor_value(f[d], x[d], false);
                dv[d] = factor_value(f[d], x[d], true);
              }
              bcat[(size_t)(0 * Q3p + pt) * Kp + m] = v[0] * v[1] * v[2];
              bcat[(size_t)(1 * Q3p + pt) * Kp + m] = dv[0] * v[1] * v[2];
              bcat[(size_t)(2 * Q3p + pt) * Kp + m] = v[0] * dv[1] * v[2];
              bcat[(size_t)(3 * Q3p + pt) * Kp + m] = v[0] * v[1] * dv[2];
            }
      }
}

// Tables of the sum-factorised Helmholtz diagonal.  The distinct eta1 factors
// (rows), the distinct (eta1 row, eta2 factor) pairs and every mode's eta3
// factor, each as values and derivatives at the direction's points:
//   doubles: U1[n1][Q] W1[n1][Q] U2[n12][Q] W2[n12][Q] U3[NP][Q] W3[NP][Q]
//   ints:    row of pair [n12], pair of mode [NP]
void build_diag_tables(int sh, int P, int pts, std::vector<double>& dt, std::vector<int>& di, int& n1, int& n12) {
  const int Q = P + 2, NP = num_modes(sh, P);
  std::vector<double> z(3 * Q), w(3 * Q);
  for (int d = 0; d < 3; ++d) rule_1d(Q, alpha_dir(sh, d), pts, z.data() + d * Q, w.data() + d * Q);
  std::vector<Factor> rows;
  std::vector<std::pair<int, Factor>> pairs;
  std::vector<int> mode_pair;
  std::vector<Factor> mode_c;
  for (int p = 0; p <= P; ++p)
    for (int q = 0; q < nq_of(sh, P, p); ++q)
      for (int r = 0; r < col_len(sh, P, p, q); ++r) {
        Factor f[3];
        mode_factors(sh, p, q, r, f);
        int ir = 0;
        while (ir < (int)rows.size() && !(rows[ir] == f[0])) ++ir;
        if (ir == (int)rows.size()) rows.push_back(f[0]);
        int ip = 0;
        while (ip < (int)pairs.size() && !(pairs[ip].first == ir && pairs[ip].second == f[1])) ++ip;
        if (ip == (int)pairs.size()) pairs.push_back({ir, f[1]});
        mode_pair.push_back(ip);
        mode_c.push_back(f[2]);
      }
  n1 = (int)rows.size();
  n12 = (int)pairs.size();
  dt.assign((size_t)2 * Q * (n1 + n12 + NP), 0.0);
  double* U1 = dt.data();
  double* W1 = U1 + n1 * Q;
  double* U2 = W1 + n1 * Q;
  double* W2 = U2 + n12 * Q;
  double* U3 = W2 + n12 * Q;
  double* W3 = U3 + NP * Q;
  for (int a = 0; a < n1; ++a)
    for (int i = 0; i < Q; ++i) {
      U1[a * Q + i] = factor_value(rows[a], z[i], false);
      W1[a * Q + i] = factor_value(rows[a], z[i], true);
    }
  for (int b = 0; b < n12; ++b)
    for (int j = 0; j < Q; ++j) {
      U2[b * Q + j] = factor_value(pairs[b].second, z[Q + j], false);
      W2[b * Q + j] = factor_value(pairs[b].second, z[Q + j], true);
    }
  for (int m = 0; m < NP; ++m)
    for (int k = 0; k < Q; ++k) {
      U3[m * Q + k] = factor_value(mode_c[m], z[2 * Q + k], false);
      W3[m * Q + k] = factor_value(mode_c[m], z[2 * Q + k], true);
    }
  di.assign(n12 + NP, 0);
  for (int b = 0; b < n12; ++b) di[b] = pairs[b].first;
  for (int m = 0; m < NP; ++m) di[n12 + m] = mode_pair[m];
}

// d eta / d xi of the collapse at (e1, e2, e3), rows eta_d, columns xi_a, and
// the factor 2^{-sum alpha} that the Jacobi weights leave out (Sec. 2.3)
static void collapse_deriv(int sh, double e1, double e2, double e3, double G[9], double* scale) {
  for (int c = 0; c < 9; ++c) G[c] = (c % 4 == 0) ? 1.0 : 0.0;
  *scale = 1.0;
  if (sh == PRISM) {
    G[0] = 2.0 / (1.0 - e3);
    G[2] = (1.0 + e1) / (1.0 - e3);
    *scale = 0.5;
  } else if (sh == PYR) {
    G[0] = 2.0 / (1.0 - e3);
    G[2] = (1.0 + e1) / (1.0 - e3);
    G[4] = 2.0 / (1.0 - e3);
    G[5] = (1.0 + e2) / (1.0 - e3);
    *scale = 0.25;
  } else if (sh == TET) {
    const double s = (1.0 - e2) * (1.0 - e3);
    G[0] = 4.0 / s;
    G[1] = 2.0 * (1.0 + e1) / s;
    G[2] = 2.0 * (1.0 + e1) / s;
    G[4] = 2.0 / (1.0 - e3);
    G[5] = (1.0 + e2) / (1.0 - e3);
    *scale = 0.125;
  }
}

// the 7 reference matrices of an affine element, row-major
// Acat[m][k Kp + n] (Kp = N_P padded to 16)
static void affine_mats_rows(int sh, int P, int pts, std::vector<double>& acat, int& Kp) {
  std::vector<double> bcat;
  int Q3p = 0;
  build_localmat(sh, P, pts, bcat, Q3p, Kp);
  const int Q = P + 2, Q3 = Q * Q * Q, NP = num_modes(sh, P);
  std::vector<double> z(3 * Q), w(3 * Q);
  for (int d = 0; d < 3; ++d) rule_1d(Q, alpha_dir(sh, d), pts, z.data() + d * Q, w.data() + d * Q);
  // reference weights and xi-derivatives of the modes at the points
  std::vector<double> wr(Q3), dx((size_t)3 * Q3 * NP);
  for (int i = 0; i < Q; ++i)
    for (int j = 0; j < Q; ++j)
      for (int k = 0; k < Q; ++k) {
        const int pt = (i * Q + j) * Q + k;
        double G[9], scale;
        collapse_deriv(sh, z[i], z[Q + j], z[2 * Q + k], G, &scale);
        wr[pt] = w[i] * w[Q + j] * w[2 * Q + k] * scale;
        for (int m = 0; m < NP; ++m)
          for (int a = 0; a < 3; ++a) {
            double v = 0.0;
            for (int d = 0; d < 3; ++d) v += G[d * 3 + a] * bcat[(size_t)((1 + d) * Q3p + pt) * Kp + m];
            dx[((size_t)a * Q3 + pt) * NP + m] = v;
          }
      }
  // Acat[m][k Kp + n]: A_0 = B^T W B, then S_00, S_01 + S_10, S_02 + S_20,
  // S_11, S_12 + S_21, S_22 with S_ab = (d_a B)^T W (d_b B) in xi
  const int NK = 7, W7 = NK * Kp;
  acat.assign((size_t)Kp * W7, 0.0);
  const int pa[6] = {0, 0, 0, 1, 1, 2}, pb[6] = {0, 1, 2, 1, 2, 2};
  for (int m = 0; m < NP; ++m)
    for (int n = 0; n < NP; ++n) {
      double mass = 0.0, S[3][3] = {};
      for (int pt = 0; pt < Q3; ++pt) {
        const double ww = wr[pt];
        mass += ww * bcat[(size_t)pt * Kp + m] * bcat[(size_t)pt * Kp + n];
        for (int a = 0; a < 3; ++a) {
          const double da = ww * dx[((size_t)a * Q3 + pt) * NP + m];
          for (int b = 0; b < 3; ++b) S[a][b] += da * dx[((size_t)b * Q3 + pt) * NP + n];
        }
      }
      double* row = acat.data() + (size_t)m * W7;
      row[0 * Kp + n] = mass;
      for (int c = 0; c < 6; ++c) {
        const int a = pa[c], b = pb[c];
        row[(1 + c) * Kp + n] = (a == b) ? S[a][a] : S[a][b] + S[b][a];
      }
    }
}

void build_affine_mats(int sh, int P, int pts, std::vector<double>& acat, int& Kp) {
  affine_mats_rows(sh, P, pts, acat, Kp);
  const int NK = NAFF, W7 = NK * Kp;
  // MFMA fragment order: A operand of v_mfma_f64_16x16x4f64, lane l holding
  // row 16 mb + l%16 and column 4 kb + l/16 of A_k
  const int MB = Kp / 16;
  std::vector<double> frag(acat.size());
  for (int kb = 0; kb < Kp / 4; ++kb)
    for (int k = 0; k < NK; ++k)
      for (int mb = 0; mb < MB; ++mb)
        for (int l = 0; l < 64; ++l)
          frag[(((size_t)kb * NK + k) * MB + mb) * 64 + l] =
              acat[(size_t)(mb * 16 + l % 16) * W7 + k * Kp + 4 * kb + l / 16];
  acat.swap(frag);
}

// bfloat16 bits of a float, rounded to nearest even (finite values)
static uint16_t bf16_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

static double bf16_value(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

void build_affine_mats_bf16(int sh, int P, int pts, std::vector<uint16_t>& frag, int& NPp, int& KS, int& MB) {
  std::vector<double> acat;
  int Kp = 0;
  affine_mats_rows(sh, P, pts, acat, Kp);
  const int NP = num_modes(sh, P), W7 = NAFF * Kp;
  NPp = (NP + 7) / 8 * 8;
  KS = (NAFF * NPp + 31) / 32;
  MB = (NP + 15) / 16;
  frag.assign((size_t)KS * MB * BF16_PARTS * 64 * 8, 0);
  for (int kb = 0; kb < KS; ++kb)
    for (int mb = 0; mb < MB; ++mb)
      for (int l = 0; l < 64; ++l)
        for (int j = 0; j < 8; ++j) {
          const int m = 16 * mb + l % 16, kap = 32 * kb + 8 * (l / 16) + j;
          const int k = kap / NPp, n = kap - k * NPp;
          if (m >= NP || k >= NAFF || n >= NP) continue;
          double rest = acat[(size_t)m * W7 + k * Kp + n];
          for (int part = 0; part < BF16_PARTS; ++part) {
            const uint16_t h = bf16_bits((float)rest);
            frag[((((size_t)kb * MB + mb) * BF16_PARTS + part) * 64 + l) * 8 + j] = h;
            rest -= bf16_value(h);
          }
        }
}

void reference_points(int sh, int Q, int pts, double* xi, double* wout) {
  std::vector<double> z(3 * Q), w(3 * Q);
  for (int d = 0; d < 3; ++d) rule_1d(Q, alpha_dir(sh, d), pts, z.data() + d * Q, w.data() + d * Q);
  const int Q3 = Q * Q * Q;
  for (int i = 0; i < Q; ++i)
    for (int j = 0; j < Q; ++j)
      for (int k = 0; k < Q; ++k) {
        const int pt = (i * Q + j) * Q + k;
        const double e1 = z[i], e2 = z[Q + j], e3 = z[2 * Q + k];
        double x1 = e1, x2 = e2, x3 = e3;
        if (sh == PRISM) {
          x1 = 0.5 * (1.0 + e1) * (1.0 - e3) - 1.0;
        } else if (sh == PYR) {
          x1 = 0.5 * (1.0 + e1) * (1.0 - e3) - 1.0;
          x2 = 0.5 * (1.0 + e2) * (1.0 - e3) - 1.0;
        } else if (sh == TET) {
          x1 = 0.25 * (1.0 + e1) * (1.0 - e2) * (1.0 - e3) - 1.0;
          x2 = 0.5 * (1.0 + e2) * (1.0 - e3) - 1.0;
        }
        xi[0 * Q3 + pt] = x1;
        xi[1 * Q3 + pt] = x2;
        xi[2 * Q3 + pt] = x3;
        if (wout) wout[pt] = w[i] * w[Q + j] * w[2 * Q + k];
      }
}

}  // namespace shp

namespace shp {

// Reference weights of the tensor points: the product of the three 1D weights
// divided by prod (1 - eta_d)^alpha_d, the Jacobi weight that the rule of a
// collapsed direction carries (Sec. 2.3), so that jw = wref |det d x/d eta|.
void build_ref_weights(int sh, int P, int pts, std::vector<double>& wref) {
  const int Q = P + 2;
  std::vector<double> z(3 * Q), w(3 * Q);
  for (int d = 0; d < 3; ++d) rule_1d(Q, alpha_dir(sh, d), pts, z.data() + d * Q, w.data() + d * Q);
  wref.assign((size_t)Q * Q * Q, 0.0);
  for (int i = 0; i < Q; ++i)
    for (int j = 0; j < Q; ++j)
      for (int k = 0; k < Q; ++k) {
        double v = w[i] * w[Q + j] * w[2 * Q + k];
        v /= std::pow(1.0 - z[i], alpha_dir(sh, 0)) * std::pow(1.0 - z[Q + j], alpha_dir(sh, 1)) *
             std::pow(1.0 - z[2 * Q + k], alpha_dir(sh, 2));
        wref[(size_t)(i * Q + j) * Q + k] = v;
      }
}

}  // namespace shp

namespace shp {

// Reference tables of a 2D shape (quadrilateral, triangle) at order P in the
// layout of tab_layout2d: points and weights per direction (GLL in eta1 and in
// the quadrilateral's eta2; Gauss-Jacobi(1,0) or Gauss-Radau-Jacobi(1,0) in
// the triangle's collapsed eta2), A_p and derivatives in eta1, the eta2
// functions (A_q, or C_{p,q} at row fam_index(P, p, q)) and derivatives, and
// the collocation derivative of each direction.
void build_tables2d(int sh, int P, int pts, std::vector<double>& tab) {
  const int Q = P + 2, n = P + 1;
  const int nb2 = (sh == TRI) ? (P + 1) * (P + 2) / 2 : n;
  const int oz = 0, ow = 2 * Q, oA = 4 * Q, odA = oA + n * Q, oB = odA + n * Q, odB = oB + nb2 * Q, oD = odB + nb2 * Q;
  tab.assign(oD + 2 * Q * Q, 0.0);
  double* z = tab.data() + oz;
  double* w = tab.data() + ow;
  rule_1d(Q, 0, pts, z, w);
  rule_1d(Q, sh == TRI ? 1 : 0, pts, z + Q, w + Q);
  for (int p = 0; p < n; ++p)
    for (int i = 0; i < Q; ++i) {
      tab[oA + p * Q + i] = fA(p, z[i]);
      tab[odA + p * Q + i] = fdA(p, z[i]);
    }
  if (sh == TRI) {
    for (int p = 0; p <= P; ++p)
      for (int q = 0; q <= P - p; ++q)
        for (int j = 0; j < Q; ++j) {
          tab[oB + fam_index(P, p, q) * Q + j] = fC(p, q, z[Q + j]);
          tab[odB + fam_index(P, p, q) * Q + j] = fdC(p, q, z[Q + j]);
        }
  } else {
    for (int q = 0; q < n; ++q)
      for (int j = 0; j < Q; ++j) {
        tab[oB + q * Q + j] = fA(q, z[Q + j]);
        tab[odB + q * Q + j] = fdA(q, z[Q + j]);
      }
  }
  for (int d = 0; d < 2; ++d) colloc_deriv(Q, z + d * Q, tab.data() + oD + d * Q * Q);
}

// Quadrature points of a 2D shape in reference coordinates (xi [2][Q^2],
// component slowest; the triangle's collapse xi1 = (1 + eta1)(1 - eta2)/2 - 1)
// and the products of the 1D weights.
void reference_points2d(int sh, int Q, int pts, double* xi, double* wout) {
  std::vector<double> z(2 * Q), w(2 * Q);
  rule_1d(Q, 0, pts, z.data(), w.data());
  rule_1d(Q, sh == TRI ? 1 : 0, pts, z.data() + Q, w.data() + Q);
  const int Q2 = Q * Q;
  for (int i = 0; i < Q; ++i)
    for (int j = 0; j < Q; ++j) {
      const int pt = i * Q + j;
      const double e1 = z[i], e2 = z[Q + j];
      xi[pt] = (sh == TRI) ? 0.5 * (1.0 + e1) * (1.0 - e2) - 1.0 : e1;
      xi[Q2 + pt] = e2;
      if (wout) wout[pt] = w[i] * w[Q + j];
    }
}

}  // namespace shp
