// Diagonal of the elemental Helmholtz operator H = lambda M + L, sum-factorised.
//
// With the collocated form (Sec. 2.2.1, eq. helm1) the derivatives of a mode
// at the points are those of its 1D factors, so for mode m = a(eta1) b(eta2)
// c(eta3)
//   H_mm = sum_q lambda jw phi_m^2 + sum_{d,e} g_de (d_d phi_m)(d_e phi_m),
// and every term is a point field f in {jw, g00, g01, g02, g11, g12, g22}
// contracted with one product of 1D values per direction: u^2, u w or w^2
// (u the factor, w its derivative).  Per field: contract eta1 over the
// distinct eta1 factors, eta2 over the distinct (eta1, eta2) factor pairs,
// eta3 per mode -- the three stages of a sum-factorised inner product
// (Sec. 3.3.2), about the work of one operator action.
#include <hip/hip_runtime.h>

#include "shp_internal.hpp"

namespace shp {
namespace {

// product type of field f (jw, g00, g01, g02, g11, g12, g22) in direction d:
// 0 = u u, 1 = u w, 2 = w w (the derivative factor sits in the directions
// the metric entry pairs)
__device__ __forceinline__ int ptype(int f, int d) {
  const int dd[NFAC][2] = {{-1, -1}, {0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
  return (dd[f][0] == d) + (dd[f][1] == d);
}

__device__ __forceinline__ double prod(const double* __restrict__ U, const double* __restrict__ Wd, int idx,
                                       int type) {
  const double u = U[idx], w = Wd[idx];
  return type == 0 ? u * u : type == 1 ? u * w : w * w;
}

__global__ void __launch_bounds__(256) k_helm_diag(const double* __restrict__ fac, const double* __restrict__ dt,
                                                   const int* __restrict__ di, int Q, int n1, int n12, int NP,
                                                   double lambda, double* __restrict__ diag, long long e_base) {
  extern __shared__ double sm[];
  const int Q2 = Q * Q, Q3 = Q2 * Q;
  double* F = sm;                 // one field [Q^3]
  double* S1 = F + Q3;            // [n1][Q^2]
  double* S2 = S1 + n1 * Q2;      // [n12][Q]
  double* acc = S2 + n12 * Q;     // [NP]
  const double* U1 = dt;
  const double* W1 = U1 + n1 * Q;
  const double* U2 = W1 + n1 * Q;
  const double* W2 = U2 + n12 * Q;
  const double* U3 = W2 + n12 * Q;
  const double* W3 = U3 + NP * Q;
  const int* row_of = di;
  const int* pair_of = di + n12;
  const long long e = e_base + blockIdx.x;
  const double* fe = fac + e * (long long)(NFAC * Q3);
  for (int m = threadIdx.x; m < NP; m += blockDim.x) acc[m] = 0.0;
  for (int f = 0; f < NFAC; ++f) {
    __syncthreads();
    for (int t = threadIdx.x; t < Q3; t += blockDim.x) F[t] = fe[f * Q3 + t];
    __syncthreads();
    const int t1 = ptype(f, 0), t2 = ptype(f, 1), t3 = ptype(f, 2);
    // eta1: S1[a][j][k] = sum_i (a a)(z_i) F[i][j][k]
    for (int t = threadIdx.x; t < n1 * Q2; t += blockDim.x) {
      const int a = t / Q2, jk = t - a * Q2;
      double s = 0.0;
      for (int i = 0; i < Q; ++i) s = fma(prod(U1, W1, a * Q + i, t1), F[i * Q2 + jk], s);
      S1[t] = s;
    }
    __syncthreads();
    // eta2: S2[b][k] = sum_j (b b)(z_j) S1[row(b)][j][k]
    for (int t = threadIdx.x; t < n12 * Q; t += blockDim.x) {
      const int b = t / Q, k = t - b * Q;
      const double* s1 = S1 + row_of[b] * Q2 + k;
      double s = 0.0;
      for (int j = 0; j < Q; ++j) s = fma(prod(U2, W2, b * Q + j, t2), s1[j * Q], s);
      S2[t] = s;
    }
    __syncthreads();
    // eta3 per mode, weighted into the diagonal
    // the off-diagonal metric entries count twice (g is symmetric)
    const double wt = f == 0 ? lambda : (f == 2 || f == 3 || f == 5) ? 2.0 : 1.0;
    for (int m = threadIdx.x; m < NP; m += blockDim.x) {
      const double* s2 = S2 + pair_of[m] * Q;
      double s = 0.0;
      for (int k = 0; k < Q; ++k) s = fma(prod(U3, W3, m * Q + k, t3), s2[k], s);
      acc[m] = fma(wt, s, acc[m]);
    }
  }
  __syncthreads();
  for (int m = threadIdx.x; m < NP; m += blockDim.x) diag[e * NP + m] = acc[m];
}

}  // namespace

hipError_t launch_helm_diag(const double* fac, const double* dt, const int* di, int Q, int n1, int n12, int NP,
                            long long n_elem, double lambda, double* diag, hipStream_t s) {
  if (n_elem <= 0) return hipSuccess;
  const size_t lds = sizeof(double) * ((size_t)Q * Q * Q + (size_t)n1 * Q * Q + (size_t)n12 * Q + NP);
  // at most 2^22 work-groups per launch (grid x times threads stays below 2^32)
  for (long long e0 = 0; e0 < n_elem; e0 += (1LL << 22)) {
    const long long ne = n_elem - e0 < (1LL << 22) ? n_elem - e0 : (1LL << 22);
    hipLaunchKernelGGL(k_helm_diag, dim3((unsigned)ne), dim3(256), lds, s, fac, dt, di, Q, n1, n12, NP, lambda, diag,
                       e0);
    if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace shp
