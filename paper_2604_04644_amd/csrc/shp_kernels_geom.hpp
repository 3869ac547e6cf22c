// HIP kernel of libshp for gfx950: FP64 geometric factors of a block from
// d x/d xi at the quadrature points.
#pragma once
#include "shp_kernels.hpp"

namespace shp {

// ---------------------------------------------------------------------------
// geometric factors (FP64): from d x/d xi at the points to jw, g and d eta/d x
// ---------------------------------------------------------------------------

struct GeomArgs {
  const double* tab;
  const double* jac;  // curved [n][9][Q3], affine [n][9]
  double* fac;        // [n][NFAC][Q3]
  double* dxi;        // [n][NDXI][Q3]
  int* status;        // set to 1 when a det <= 0 or a non-finite value is met
  long long n_elem;
  int affine;
};

template <int SH, int P>
__global__ void __launch_bounds__(256) k_geometry(GeomArgs g) {
  using D = Dims<SH, P>;
  constexpr int Q = D::Q, Q3 = D::Q3;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.n_elem * Q3) return;
  const long long e = t / Q3;
  const int pt = (int)(t - e * Q3);
  const int i = pt / (Q * Q), j = (pt / Q) % Q, k = pt % Q;
  const double* z = g.tab + D::L.z;
  const double* w = g.tab + D::L.w;
  const double e1 = z[0 * Q + i], e2 = z[1 * Q + j], e3 = z[2 * Q + k];
  const double wq = w[0 * Q + i] * w[1 * Q + j] * w[2 * Q + k];
  double J[9];
  if (g.affine) {
#pragma unroll
    for (int c = 0; c < 9; ++c) J[c] = g.jac[e * 9 + c];
  } else {
#pragma unroll
    for (int c = 0; c < 9; ++c) J[c] = g.jac[(e * 9 + c) * Q3 + pt];
  }
  // inverse of d x/d xi by cofactors
  const double c00 = J[4] * J[8] - J[5] * J[7];
  const double c01 = J[5] * J[6] - J[3] * J[8];
  const double c02 = J[3] * J[7] - J[4] * J[6];
  const double det = J[0] * c00 + J[1] * c01 + J[2] * c02;
  bool bad = !(det > 0.0) || !isfinite(det);
  const double id = 1.0 / det;
  double X[9];  // d xi_a / d x_i at a*3+i
  X[0] = c00 * id;
  X[1] = (J[2] * J[7] - J[1] * J[8]) * id;
  X[2] = (J[1] * J[5] - J[2] * J[4]) * id;
  X[3] = c01 * id;
  X[4] = (J[0] * J[8] - J[2] * J[6]) * id;
  X[5] = (J[2] * J[3] - J[0] * J[5]) * id;
  X[6] = c02 * id;
  X[7] = (J[1] * J[6] - J[0] * J[7]) * id;
  X[8] = (J[0] * J[4] - J[1] * J[3]) * id;
  // d eta / d xi of the collapse (rows eta_d, columns xi_a)
  double Gc[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  double scale = 1.0;  // 2^{-sum alpha}
  if (SH == PRISM) {
    Gc[0] = 2.0 / (1.0 - e3);
    Gc[2] = (1.0 + e1) / (1.0 - e3);
    scale = 0.5;
  } else if (SH == PYR) {
    Gc[0] = 2.0 / (1.0 - e3);
    Gc[2] = (1.0 + e1) / (1.0 - e3);
    Gc[4] = 2.0 / (1.0 - e3);
    Gc[5] = (1.0 + e2) / (1.0 - e3);
    scale = 0.25;
  } else if (SH == TET) {
    const double s = (1.0 - e2) * (1.0 - e3);
    Gc[0] = 4.0 / s;
    Gc[1] = 2.0 * (1.0 + e1) / s;
    Gc[2] = 2.0 * (1.0 + e1) / s;
    Gc[4] = 2.0 / (1.0 - e3);
    Gc[5] = (1.0 + e2) / (1.0 - e3);
    scale = 0.125;
  }
  double M[9];  // d eta_d / d x_i
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int ii = 0; ii < 3; ++ii)
      M[d * 3 + ii] = Gc[d * 3 + 0] * X[0 * 3 + ii] + Gc[d * 3 + 1] * X[1 * 3 + ii] + Gc[d * 3 + 2] * X[2 * 3 + ii];
  const double jw = wq * scale * det;
  double gm[6];
  gm[0] = jw * (M[0] * M[0] + M[1] * M[1] + M[2] * M[2]);
  gm[1] = jw * (M[0] * M[3] + M[1] * M[4] + M[2] * M[5]);
  gm[2] = jw * (M[0] * M[6] + M[1] * M[7] + M[2] * M[8]);
  gm[3] = jw * (M[3] * M[3] + M[4] * M[4] + M[5] * M[5]);
  gm[4] = jw * (M[3] * M[6] + M[4] * M[7] + M[5] * M[8]);
  gm[5] = jw * (M[6] * M[6] + M[7] * M[7] + M[8] * M[8]);
  double* f = g.fac + e * (NFAC * Q3) + pt;
  f[0] = jw;
#pragma unroll
  for (int c = 0; c < 6; ++c) f[(c + 1) * Q3] = gm[c];
  double* m = g.dxi + e * (NDXI * Q3) + pt;
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    m[c * Q3] = M[c];
    bad = bad || !isfinite(M[c]);
  }
  if (bad) atomicOr(g.status, 1);
}

}  // namespace shp
