// Dispatch from runtime (shape, P, operator) to the templated launchers: the
// per-shape block launchers (shp_k_<shape>.hip) and the whole-mesh launchers
// of each order (shp_k_mixed_p<P>.hip); plus the device max-difference check.
#include <algorithm>

#include "shp_kernels.hpp"
#include "shp_kernels_lm.hpp"

namespace shp {

hipError_t launch_block_hex(int P, int opk, const OpArgs& a, int threads, int persist, hipStream_t s);
hipError_t launch_block_prism(int P, int opk, const OpArgs& a, int threads, int persist, hipStream_t s);
hipError_t launch_block_pyr(int P, int opk, const OpArgs& a, int threads, int persist, hipStream_t s);
hipError_t launch_block_tet(int P, int opk, const OpArgs& a, int threads, int persist, hipStream_t s);
hipError_t launch_geometry_hex(int P, const GeomArgs& g, hipStream_t s);
hipError_t launch_geometry_prism(int P, const GeomArgs& g, hipStream_t s);
hipError_t launch_geometry_pyr(int P, const GeomArgs& g, hipStream_t s);
hipError_t launch_geometry_tet(int P, const GeomArgs& g, hipStream_t s);
hipError_t launch_localmat_hex(int P, int opk, const LocalMatArgs& a, hipStream_t s);
hipError_t launch_localmat_prism(int P, int opk, const LocalMatArgs& a, hipStream_t s);
hipError_t launch_localmat_pyr(int P, int opk, const LocalMatArgs& a, hipStream_t s);
hipError_t launch_localmat_tet(int P, int opk, const LocalMatArgs& a, hipStream_t s);

hipError_t launch_localmat_affine_hex(int P, int opk, const AffineMatArgs& a, hipStream_t s);
hipError_t launch_localmat_affine_prism(int P, int opk, const AffineMatArgs& a, hipStream_t s);
hipError_t launch_localmat_affine_pyr(int P, int opk, const AffineMatArgs& a, hipStream_t s);
hipError_t launch_localmat_affine_tet(int P, int opk, const AffineMatArgs& a, hipStream_t s);

hipError_t launch_localmat_xform_hex(int P, int opk, const LocalXformArgs& a, hipStream_t s);
hipError_t launch_localmat_xform_prism(int P, int opk, const LocalXformArgs& a, hipStream_t s);
hipError_t launch_localmat_xform_pyr(int P, int opk, const LocalXformArgs& a, hipStream_t s);
hipError_t launch_localmat_xform_tet(int P, int opk, const LocalXformArgs& a, hipStream_t s);

hipError_t launch_localmat_xform(int sh, int P, int opk, const LocalXformArgs& a, hipStream_t s) {
  switch (sh) {
    case HEX: return launch_localmat_xform_hex(P, opk, a, s);
    case PRISM: return launch_localmat_xform_prism(P, opk, a, s);
    case PYR: return launch_localmat_xform_pyr(P, opk, a, s);
    case TET: return launch_localmat_xform_tet(P, opk, a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_localmat_affine_f32_hex(int P, int opk, const AffineMatArgs32& a, hipStream_t s);
hipError_t launch_localmat_affine_f32_prism(int P, int opk, const AffineMatArgs32& a, hipStream_t s);
hipError_t launch_localmat_affine_f32_pyr(int P, int opk, const AffineMatArgs32& a, hipStream_t s);
hipError_t launch_localmat_affine_f32_tet(int P, int opk, const AffineMatArgs32& a, hipStream_t s);

hipError_t launch_localmat_affine_f32(int sh, int P, int opk, const float* afrag, const double* coef, const float* in,
                                      float* out, long long n_elem, double lambda, hipStream_t s) {
  AffineMatArgs32 a;
  a.afrag = afrag;
  a.coef = coef;
  a.in = in;
  a.out = out;
  a.n_elem = n_elem;
  a.lambda = lambda;
  switch (sh) {
    case HEX: return launch_localmat_affine_f32_hex(P, opk, a, s);
    case PRISM: return launch_localmat_affine_f32_prism(P, opk, a, s);
    case PYR: return launch_localmat_affine_f32_pyr(P, opk, a, s);
    case TET: return launch_localmat_affine_f32_tet(P, opk, a, s);
  }
  return hipErrorInvalidValue;
}

template <int P>
static long long aff_waves(int sh, long long n) {
  switch (sh) {
    case HEX: return lm_waves<HEX, P>(n, lm_tiles_per_wave<HEX, P>(), lm_rows_per_wave<HEX, P>());
    case PRISM: return lm_waves<PRISM, P>(n, lm_tiles_per_wave<PRISM, P>(), lm_rows_per_wave<PRISM, P>());
    case PYR: return lm_waves<PYR, P>(n, lm_tiles_per_wave<PYR, P>(), lm_rows_per_wave<PYR, P>());
    default: return lm_waves<TET, P>(n, lm_tiles_per_wave<TET, P>(), lm_rows_per_wave<TET, P>());
  }
}

template <int P>
static hipError_t launch_aff_mesh_p(int opk, AffineMatMesh& m, hipStream_t s) {
  long long g = 0;
  for (int b = 0; b < m.nblk; ++b) {
    m.wg0[b] = g;
    g += (aff_waves<P>(m.shape[b], m.blk[b].n_elem) + 3) / 4;
  }
  m.wg0[m.nblk] = g;
  if (g <= 0) return hipSuccess;
  switch (opk) {
    case OPK_MASS_LM: hipLaunchKernelGGL((k_localmat_affine_mesh<P, OPK_MASS>), dim3((unsigned)g), dim3(256), 0, s, m); break;
    case OPK_LAP_LM: hipLaunchKernelGGL((k_localmat_affine_mesh<P, OPK_LAP>), dim3((unsigned)g), dim3(256), 0, s, m); break;
    case OPK_HELM_LM: hipLaunchKernelGGL((k_localmat_affine_mesh<P, OPK_HELM>), dim3((unsigned)g), dim3(256), 0, s, m); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_localmat_affine_mesh(int P, int opk, int nblk, const int* shape, const AffineMatArgs* blk,
                                       hipStream_t s) {
  if (nblk < 1 || nblk > AFF_MESH_MAX) return hipErrorInvalidValue;
  AffineMatMesh m;
  m.nblk = nblk;
  for (int b = 0; b < nblk; ++b) {
    m.blk[b] = blk[b];
    m.shape[b] = shape[b];
  }
  switch (P) {
    case 1: return launch_aff_mesh_p<1>(opk, m, s);
    case 2: return launch_aff_mesh_p<2>(opk, m, s);
    case 3: return launch_aff_mesh_p<3>(opk, m, s);
    case 4: return launch_aff_mesh_p<4>(opk, m, s);
  }
  return hipErrorInvalidValue;
}

template <int P>
static long long aff32_waves(int sh, long long n) {
  switch (sh) {
    case HEX: return lm_waves<HEX, P>(n, lm32_tiles_per_wave<HEX, P>(), lm32_rows_per_wave<HEX, P>());
    case PRISM: return lm_waves<PRISM, P>(n, lm32_tiles_per_wave<PRISM, P>(), lm32_rows_per_wave<PRISM, P>());
    case PYR: return lm_waves<PYR, P>(n, lm32_tiles_per_wave<PYR, P>(), lm32_rows_per_wave<PYR, P>());
    default: return lm_waves<TET, P>(n, lm32_tiles_per_wave<TET, P>(), lm32_rows_per_wave<TET, P>());
  }
}

template <int P>
static hipError_t launch_aff32_mesh_p(int opk, AffineMatMesh32& m, hipStream_t s) {
  long long g = 0;
  for (int b = 0; b < m.nblk; ++b) {
    m.wg0[b] = g;
    g += (aff32_waves<P>(m.shape[b], m.blk[b].n_elem) + 3) / 4;
  }
  m.wg0[m.nblk] = g;
  if (g <= 0) return hipSuccess;
  switch (opk) {
    case OPK_MASS_LM: hipLaunchKernelGGL((k_localmat_affine_f32_mesh<P, OPK_MASS>), dim3((unsigned)g), dim3(256), 0, s, m); break;
    case OPK_LAP_LM: hipLaunchKernelGGL((k_localmat_affine_f32_mesh<P, OPK_LAP>), dim3((unsigned)g), dim3(256), 0, s, m); break;
    case OPK_HELM_LM: hipLaunchKernelGGL((k_localmat_affine_f32_mesh<P, OPK_HELM>), dim3((unsigned)g), dim3(256), 0, s, m); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_localmat_affine_f32_mesh(int P, int opk, int nblk, const int* shape, const AffineMatArgs32* blk,
                                           hipStream_t s) {
  if (nblk < 1 || nblk > AFF_MESH_MAX) return hipErrorInvalidValue;
  AffineMatMesh32 m;
  m.nblk = nblk;
  for (int b = 0; b < nblk; ++b) {
    m.blk[b] = blk[b];
    m.shape[b] = shape[b];
  }
  switch (P) {
    case 1: return launch_aff32_mesh_p<1>(opk, m, s);
    case 2: return launch_aff32_mesh_p<2>(opk, m, s);
    case 3: return launch_aff32_mesh_p<3>(opk, m, s);
    case 4: return launch_aff32_mesh_p<4>(opk, m, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_localmat_affine(int sh, int P, int opk, const AffineMatArgs& a, hipStream_t s) {
  switch (sh) {
    case HEX: return launch_localmat_affine_hex(P, opk, a, s);
    case PRISM: return launch_localmat_affine_prism(P, opk, a, s);
    case PYR: return launch_localmat_affine_pyr(P, opk, a, s);
    case TET: return launch_localmat_affine_tet(P, opk, a, s);
  }
  return hipErrorInvalidValue;
}

// per-element coefficients of an affine element's local matrices from its
// constant d x_i/d xi_j (jac [n][9], i*3+j): |J| and |J| (J^-1 J^-T)_ab
__global__ void __launch_bounds__(256) k_affine_coef(const double* __restrict__ jac, double* __restrict__ coef,
                                                     long long n, int* __restrict__ status) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double J[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) J[c] = jac[e * 9 + c];
  const double c00 = J[4] * J[8] - J[5] * J[7];
  const double c01 = J[5] * J[6] - J[3] * J[8];
  const double c02 = J[3] * J[7] - J[4] * J[6];
  const double det = J[0] * c00 + J[1] * c01 + J[2] * c02;
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
  const int pa[6] = {0, 0, 0, 1, 1, 2}, pb[6] = {0, 1, 2, 1, 2, 2};
  double* out = coef + e * NAFF;
  out[0] = det;
  bool bad = !(det > 0.0) || !isfinite(det);
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const int ra = pa[c] * 3, rb = pb[c] * 3;
    out[1 + c] = det * (X[ra] * X[rb] + X[ra + 1] * X[rb + 1] + X[ra + 2] * X[rb + 2]);
    bad = bad || !isfinite(out[1 + c]);
  }
  if (bad) atomicOr(status, 1);
}

hipError_t launch_affine_coef(const double* jac, double* coef, long long n, int* status, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_affine_coef, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, jac, coef, n, status);
  return hipGetLastError();
}

hipError_t launch_localmat(int sh, int P, int opk, const LocalMatArgs& a, hipStream_t s) {
  switch (sh) {
    case HEX: return launch_localmat_hex(P, opk, a, s);
    case PRISM: return launch_localmat_prism(P, opk, a, s);
    case PYR: return launch_localmat_pyr(P, opk, a, s);
    default: return launch_localmat_tet(P, opk, a, s);
  }
}

size_t lds_bytes_f32_hex(int P, int E);
size_t lds_bytes_f32_prism(int P, int E);
size_t lds_bytes_f32_pyr(int P, int E);
size_t lds_bytes_f32_tet(int P, int E);

size_t lds_bytes_f32(int sh, int P, int E) {
  switch (sh) {
    case HEX: return lds_bytes_f32_hex(P, E);
    case PRISM: return lds_bytes_f32_prism(P, E);
    case PYR: return lds_bytes_f32_pyr(P, E);
    default: return lds_bytes_f32_tet(P, E);
  }
}

size_t lds_bytes_hex(int P, int E, int nbuf);
size_t lds_bytes_prism(int P, int E, int nbuf);
size_t lds_bytes_pyr(int P, int E, int nbuf);
size_t lds_bytes_tet(int P, int E, int nbuf);

size_t op_lds_bytes(int sh, int P, int opk, int E, int variant) {
  // nbuf 0: the Laplacian / Helmholtz tile of the prefetch launches (variants
  // 1 and 2, advection-diffusion-reaction, iso-parametric), whose LDS head
  // holds only the tables it reads per lane
  const bool helm = opk == OPK_HELM || opk == OPK_LAP || opk == OPK_ADR;
  const int nbuf = (opk == OPK_HELM_NC || opk == OPK_LAP_NC) ? 5
                   : (variant >= 3 && helm) ? 3
                   : (helm && (variant == 1 || variant == 2)) ? 0 : 4;
  switch (sh) {
    case HEX: return lds_bytes_hex(P, E, nbuf);
    case PRISM: return lds_bytes_prism(P, E, nbuf);
    case PYR: return lds_bytes_pyr(P, E, nbuf);
    default: return lds_bytes_tet(P, E, nbuf);
  }
}

hipError_t launch_block(int sh, int P, int opk, const OpArgs& a, int threads, int persist, hipStream_t s) {
  switch (sh) {
    case HEX: return launch_block_hex(P, opk, a, threads, persist, s);
    case PRISM: return launch_block_prism(P, opk, a, threads, persist, s);
    case PYR: return launch_block_pyr(P, opk, a, threads, persist, s);
    default: return launch_block_tet(P, opk, a, threads, persist, s);
  }
}

int num_cus() {
  static int cus[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  if (cus[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1) n = 256;
    cus[dev] = n;
  }
  return cus[dev];
}

long long persistent_grid(const void* kernel, int threads, size_t lds) {
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, threads, lds) != hipSuccess || occ < 1) occ = 1;
  return (long long)occ * num_cus();
}

int points_per_thread(long long points, int threads) {
  const long long need = (points + threads - 1) / threads;
  return need <= 2 ? 2 : need <= 4 ? 4 : need <= 8 ? 8 : 0;
}

hipError_t launch_geometry(int sh, int P, const GeomArgs& g, hipStream_t s) {
  switch (sh) {
    case HEX: return launch_geometry_hex(P, g, s);
    case PRISM: return launch_geometry_prism(P, g, s);
    case PYR: return launch_geometry_pyr(P, g, s);
    default: return launch_geometry_tet(P, g, s);
  }
}

#define D_(p)                                                                                                      \
  hipError_t launch_mixed_P##p(int opk, const BlockStatic* blocks, const Tile* tiles, int ntiles, const double* in, \
                               double* out, long long in_cs, long long out_cs, double lambda, int threads,          \
                               size_t lds, int E, int persist, hipStream_t s);                                      \
  hipError_t launch_mixed_f32_P##p(int opk, const BlockStatic* blocks, const Tile* tiles, int ntiles,               \
                                   const float* in, float* out, double lambda, int threads, size_t lds, int E,       \
                                   bool fac32, hipStream_t s);                                                       \
  hipError_t launch_adr_P##p(const BlockStatic* blocks, const Tile* tiles, int ntiles, const double* in,            \
                             double* out, const double* adv, double lambda, int threads, size_t lds, int E,          \
                             hipStream_t s);                                                                         \
  hipError_t launch_iso_P##p(int opk, const BlockStatic* blocks, const Tile* tiles, int ntiles, const double* in,   \
                             double* out, double lambda, int threads, size_t lds, int E, int blk_only, long long nwg, \
                             hipStream_t s);                                                                         \
  hipError_t launch_iso_check_P##p(const BlockStatic* blocks, int blk, int E, long long nwg, int threads, size_t lds, \
                                   int* status, hipStream_t s);
D_(1) D_(2) D_(3) D_(4) D_(5) D_(6) D_(7) D_(8) D_(9) D_(10)
#undef D_

hipError_t launch_mixed_f32(int P, int opk, const BlockStatic* blocks, const Tile* tiles, int ntiles, const float* in,
                            float* out, double lambda, int threads, size_t lds, int E, bool fac32, hipStream_t s) {
  switch (P) {
#define C_(p) \
  case p: return launch_mixed_f32_P##p(opk, blocks, tiles, ntiles, in, out, lambda, threads, lds, E, fac32, s);
    C_(1) C_(2) C_(3) C_(4) C_(5) C_(6) C_(7) C_(8) C_(9) C_(10)
#undef C_
  }
  return hipErrorInvalidValue;
}

hipError_t launch_adr(int P, const BlockStatic* blocks, const Tile* tiles, int ntiles, const double* in, double* out,
                      const double* adv, double lambda, int threads, size_t lds, int E, hipStream_t s) {
  switch (P) {
#define C_(p) \
  case p: return launch_adr_P##p(blocks, tiles, ntiles, in, out, adv, lambda, threads, lds, E, s);
    C_(1) C_(2) C_(3) C_(4) C_(5) C_(6) C_(7) C_(8) C_(9) C_(10)
#undef C_
  }
  return hipErrorInvalidValue;
}

hipError_t launch_iso(int P, int opk, const BlockStatic* blocks, const Tile* tiles, int ntiles, const double* in,
                      double* out, double lambda, int threads, size_t lds, int E, int blk_only, long long nwg,
                      hipStream_t s) {
  switch (P) {
#define C_(p) \
  case p: return launch_iso_P##p(opk, blocks, tiles, ntiles, in, out, lambda, threads, lds, E, blk_only, nwg, s);
    C_(1) C_(2) C_(3) C_(4) C_(5) C_(6) C_(7) C_(8) C_(9) C_(10)
#undef C_
  }
  return hipErrorInvalidValue;
}

hipError_t launch_iso_check(int P, const BlockStatic* blocks, int blk, int E, long long nwg, int threads, size_t lds,
                            int* status, hipStream_t s) {
  switch (P) {
#define C_(p) \
  case p: return launch_iso_check_P##p(blocks, blk, E, nwg, threads, lds, status, s);
    C_(1) C_(2) C_(3) C_(4) C_(5) C_(6) C_(7) C_(8) C_(9) C_(10)
#undef C_
  }
  return hipErrorInvalidValue;
}

#define D2_(lo)                                                                                                    \
  hipError_t dispatch2d_P##lo(int which, int sh, int p, int opk, const OpArgs* a, int threads,                     \
                              const BlockStatic* blocks, const Tile* tiles, int ntiles, const double* in,          \
                              double* out, long long in_cs, long long out_cs, double lambda, size_t lds,           \
                              const double* tab, const double* jac, double* fac, double* dxi, long long n_elem,    \
                              int affine, int* status, size_t* bytes, int E, hipStream_t s);
D2_(1) D2_(6)
#undef D2_

static hipError_t dispatch2d(int which, int sh, int P, int opk, const OpArgs* a, int threads,
                             const BlockStatic* blocks, const Tile* tiles, int ntiles, const double* in, double* out,
                             long long in_cs, long long out_cs, double lambda, size_t lds, const double* tab,
                             const double* jac, double* fac, double* dxi, long long n_elem, int affine, int* status,
                             size_t* bytes, int E, hipStream_t s) {
  if (P >= 1 && P <= 5)
    return dispatch2d_P1(which, sh, P, opk, a, threads, blocks, tiles, ntiles, in, out, in_cs, out_cs, lambda, lds,
                         tab, jac, fac, dxi, n_elem, affine, status, bytes, E, s);
  if (P >= 6 && P <= 10)
    return dispatch2d_P6(which, sh, P, opk, a, threads, blocks, tiles, ntiles, in, out, in_cs, out_cs, lambda, lds,
                         tab, jac, fac, dxi, n_elem, affine, status, bytes, E, s);
  return hipErrorInvalidValue;
}

hipError_t launch_block2d(int sh, int P, int opk, const OpArgs& a, int threads, hipStream_t s) {
  return dispatch2d(0, sh, P, opk, &a, threads, nullptr, nullptr, 0, nullptr, nullptr, 0, 0, 0.0, 0, nullptr, nullptr,
                    nullptr, nullptr, 0, 0, nullptr, nullptr, a.E, s);
}

hipError_t launch_mixed2d(int P, int opk, const BlockStatic* blocks, const Tile* tiles, int ntiles, const double* in,
                          double* out, long long in_cs, long long out_cs, double lambda, int threads, size_t lds,
                          int E, hipStream_t s) {
  return dispatch2d(1, QUAD, P, opk, nullptr, threads, blocks, tiles, ntiles, in, out, in_cs, out_cs, lambda, lds,
                    nullptr, nullptr, nullptr, nullptr, 0, 0, nullptr, nullptr, E, s);
}

hipError_t launch_geometry2d(int sh, int P, const double* tab, const double* jac, double* fac, double* dxi,
                             long long n_elem, int affine, int* status, hipStream_t s) {
  return dispatch2d(2, sh, P, 0, nullptr, 0, nullptr, nullptr, 0, nullptr, nullptr, 0, 0, 0.0, 0, tab, jac, fac, dxi,
                    n_elem, affine, status, nullptr, 0, s);
}

size_t lds_bytes_2d(int sh, int P, int E, int opk, int threads) {
  size_t b = 0;
  dispatch2d(3, sh, P, opk, nullptr, threads, nullptr, nullptr, 0, nullptr, nullptr, 0, 0, 0.0, 0, nullptr, nullptr,
             nullptr, nullptr, 0, 0, nullptr, &b, E, nullptr);
  return b;
}

// Advection factors of one block: a_d = jw sum_i b_i d eta_d / d x_i at every
// point, from the block's factors (jw first of NFAC per point) and d eta/d x
// (NDXI = 9 per point, row eta_d, column x_i); vel is [3][vstride] with the
// block's points first, adv [n][3][Q^3].
__global__ void __launch_bounds__(256) k_adv_factors(const double* __restrict__ fac, const double* __restrict__ dxi,
                                                     const double* __restrict__ vel, long long vstride,
                                                     double* __restrict__ adv, long long n_elem, int Q3) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_elem * Q3) return;
  const long long e = t / Q3;
  const int pt = (int)(t - e * Q3);
  const double jw = fac[e * (NFAC * (long long)Q3) + pt];
  const double* m = dxi + e * (NDXI * (long long)Q3) + pt;
  const double b0 = vel[t], b1 = vel[vstride + t], b2 = vel[2 * vstride + t];
  double* o = adv + e * (3LL * Q3) + pt;
#pragma unroll
  for (int d = 0; d < 3; ++d)
    o[d * Q3] = jw * (b0 * m[(d * 3 + 0) * Q3] + b1 * m[(d * 3 + 1) * Q3] + b2 * m[(d * 3 + 2) * Q3]);
}

hipError_t launch_adv_factors(const double* fac, const double* dxi, const double* vel, long long vstride, double* adv,
                              long long n_elem, int Q3, hipStream_t s) {
  const long long n = n_elem * Q3;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adv_factors, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, fac, dxi, vel, vstride, adv,
                     n_elem, Q3);
  return hipGetLastError();
}

hipError_t launch_mixed(int P, int opk, const BlockStatic* blocks, const Tile* tiles, int ntiles, const double* in,
                        double* out, long long in_cs, long long out_cs, double lambda, int threads, size_t lds, int E,
                        int persist, hipStream_t s) {
  switch (P) {
#define C_(p)                                                                                                   \
  case p:                                                                                                       \
    return launch_mixed_P##p(opk, blocks, tiles, ntiles, in, out, in_cs, out_cs, lambda, threads, lds, E, persist, \
                             s);
    C_(1) C_(2) C_(3) C_(4) C_(5) C_(6) C_(7) C_(8) C_(9) C_(10)
#undef C_
  }
  return hipErrorInvalidValue;
}

}  // namespace shp

namespace shp {

// max |a - b| and max |b| over n values, as the bit patterns of non-negative
// doubles (which order like unsigned integers; a NaN difference orders above
// every finite value).
__global__ void __launch_bounds__(256) k_maxdiff(const double* __restrict__ a, const double* __restrict__ b,
                                                 long long n, unsigned long long* out) {
  double dm = 0.0, bm = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double d = fabs(a[i] - b[i]);
    dm = (d > dm || d != d) ? d : dm;
    bm = fmax(bm, fabs(b[i]));
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double od = __shfl_down(dm, off);
    const double ob = __shfl_down(bm, off);
    dm = (od > dm || od != od) ? od : dm;
    bm = fmax(bm, ob);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(out + 0, (unsigned long long)__double_as_longlong(dm));
    atomicMax(out + 1, (unsigned long long)__double_as_longlong(bm));
  }
}

hipError_t launch_maxdiff(const double* a, const double* b, long long n, unsigned long long* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const long long nb = std::min<long long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_maxdiff, dim3((unsigned)nb), dim3(256), 0, s, a, b, n, out);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_round_f32(const double* __restrict__ a, float* __restrict__ b, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    b[i] = (float)a[i];
}

hipError_t launch_round_f32(const double* a, float* b, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const long long nb = std::min<long long>((n + 255) / 256, 16384);
  hipLaunchKernelGGL(k_round_f32, dim3((unsigned)nb), dim3(256), 0, s, a, b, n);
  return hipGetLastError();
}

}  // namespace shp
