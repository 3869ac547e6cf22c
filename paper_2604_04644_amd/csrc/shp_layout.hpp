// Compile-time shape traits and reference-table layout shared by the host
// library and the HIP kernels of libshp.
//
// Collapsed-coordinate tensor structure (Sec. 2.3): every mode is a product
// a(eta1) b(eta2) c(eta3) of 1D functions.  Sum-factorisation contracts eta3
// first (the innermost, ragged index r), then eta2 (q), then eta1 (p); the
// "columns" of the first stage are the (p,q) pairs that own a run of r.
#pragma once
#include <cstdint>

namespace shp {

enum : int { HEX = 0, PRISM = 1, PYR = 2, TET = 3, QUAD = 4, TRI = 5 };

constexpr int imax(int a, int b) { return a > b ? a : b; }

// number of modes N_P
constexpr int num_modes(int sh, int P) {
  return sh == HEX ? (P + 1) * (P + 1) * (P + 1)
       : sh == PRISM ? (P + 1) * (P + 1) * (P + 2) / 2
       : sh == PYR ? (P + 1) * (P + 2) * (2 * P + 3) / 6
                   : (P + 1) * (P + 2) * (P + 3) / 6;
}
// number of modes of the 2D shapes: quadrilateral (P+1)^2, triangle (P+1)(P+2)/2
constexpr int num_modes2(int sh, int P) { return sh == QUAD ? (P + 1) * (P + 1) : (P + 1) * (P + 2) / 2; }
constexpr bool is_2d(int sh) { return sh == QUAD || sh == TRI; }
// number of (p,q) columns
constexpr int num_cols(int sh, int P) { return sh == TET ? (P + 1) * (P + 2) / 2 : (P + 1) * (P + 1); }
// run length of r in column (p,q)
constexpr int col_len(int sh, int P, int p, int q) {
  return sh == HEX ? P + 1 : sh == PRISM ? P + 1 - p : sh == PYR ? P + 1 - imax(p, q) : P + 1 - p - q;
}
// number of q values for a given p
constexpr int nq_of(int sh, int P, int p) { return sh == TET ? P + 1 - p : P + 1; }
// first column of p (columns are p-major)
constexpr int col_base(int sh, int P, int p) {
  return sh == TET ? p * (P + 1) - p * (p - 1) / 2 : p * (P + 1);
}
// index of the eta3 function family C_{kappa,.} used by column (p,q)
constexpr int kappa3(int sh, int p, int q) {
  return sh == HEX ? 0 : sh == PRISM ? p : sh == PYR ? imax(p, q) : p + q;
}
// columns (p, q) of the eta3 family kappa, and the first of them in the
// family-major column order (prism: kappa = p; pyramid: max(p, q); tet: p + q)
constexpr int fam_ncols(int sh, int P, int kappa) {
  return sh == PRISM ? P + 1 : sh == PYR ? 2 * kappa + 1 : sh == TET ? kappa + 1 : (P + 1) * (P + 1);
}
constexpr int fam_start(int sh, int P, int kappa) {
  int s = 0;
  for (int k = 0; k < kappa; ++k) s += fam_ncols(sh, P, k);
  return s;
}
// Jacobi exponent of the rule in direction d (0: GLL)
constexpr int alpha_dir(int sh, int d) {
  return d == 0 ? 0 : d == 1 ? (sh == TET ? 1 : 0) : (sh == HEX ? 0 : sh == PRISM ? 1 : 2);
}
// innermost stride of point buffers in LDS.  FP64 LDS accesses are served 32
// lanes at a time by 32 double-wide banks; the line stages walk i-, j- and
// k-lines from consecutive task indices.  Over all stage patterns a model of
// the bank conflicts favours padding to Q+1 only for Q = 4 and 8 (unpadded
// strides of 4 and 8 put 4-8 k-line lanes on one bank); Q = 6, 10 and 12 do
// better unpadded, and odd Q need no padding.
constexpr int qpad(int Q) { return (Q == 4 || Q == 8) ? Q + 1 : Q; }

// Reference tables of one (shape, P), Q = P + 2, laid out in one FP64 array:
//   z[3][Q]          points per direction
//   w[3][Q]          1D weights per direction
//   A1[n][Q],  dA1   A_p(z1_i) and derivative
//   B2[nb2][Q], dB2  eta2 functions: A_q (kappa 0 only) or C_{p,q} (tet)
//   C3[nc3][Q], dC3  eta3 functions C_{kappa,r}; kappa 0 is A_r
//   D[3][Q][Q]       collocation derivative on each direction's points
// The family index of (kappa, r) with r <= P - kappa (kappa = 0: r <= P) is
// kappa*(P+1) - kappa*(kappa-1)/2 + r.
struct TabLayout {
  int P, Q, n, nb2, nc3;
  int z, w, A1, dA1, B2, dB2, C3, dC3, D, total;
};

constexpr int fam_index(int P, int kappa, int r) { return kappa * (P + 1) - kappa * (kappa - 1) / 2 + r; }

constexpr TabLayout tab_layout(int sh, int P) {
  TabLayout t{};
  t.P = P;
  t.Q = P + 2;
  t.n = P + 1;
  const int tri = (P + 1) * (P + 2) / 2;
  t.nb2 = (sh == TET) ? tri : t.n;
  t.nc3 = (sh == HEX) ? t.n : tri;
  int o = 0;
  t.z = o;   o += 3 * t.Q;
  t.w = o;   o += 3 * t.Q;
  t.A1 = o;  o += t.n * t.Q;
  t.dA1 = o; o += t.n * t.Q;
  t.B2 = o;  o += t.nb2 * t.Q;
  t.dB2 = o; o += t.nb2 * t.Q;
  t.C3 = o;  o += t.nc3 * t.Q;
  t.dC3 = o; o += t.nc3 * t.Q;
  t.D = o;   o += 3 * t.Q * t.Q;
  t.total = o;
  return t;
}

// Per-column integer table: (p, q, mode offset, run length, eta3 family base)
constexpr int ICOL = 5;

// Geometric factors per curved element: FAC channels [jw, g00, g01, g02, g11,
// g12, g22] then DXI channels d eta_d / d x_i at d*3+i, each [N_Q].
constexpr int NFAC = 7;
constexpr int NDXI = 9;

}  // namespace shp
