// Launchers of the split-BF16 affine local-matrix kernels: every shape,
// P = 1..4, mass / Laplacian / Helmholtz, two or three parts.
#include "shp_internal.hpp"
#include "shp_kernels_bf16.hpp"

namespace shp {

template <int SH, int P, int OP, int NPART>
static hipError_t launch_bf16_op(const AffineBf16Args& a, hipStream_t s) {
  const long long nwave = bf16_waves<SH, P>((a.n_elem + 15) / 16);
  if (nwave <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_localmat_affine_bf16<SH, P, OP, NPART>), dim3((unsigned)((nwave + 3) / 4)), dim3(256), 0, s,
                     a);
  return hipGetLastError();
}

template <int P>
static long long block_waves(int sh, long long ntile) {
  switch (sh) {
    case HEX: return bf16_waves<HEX, P>(ntile);
    case PRISM: return bf16_waves<PRISM, P>(ntile);
    case PYR: return bf16_waves<PYR, P>(ntile);
    default: return bf16_waves<TET, P>(ntile);
  }
}

template <int P, int NPART>
static hipError_t launch_bf16_mesh_pn(int opk, AffineBf16Mesh& m, hipStream_t s) {
  long long g = 0;
  for (int b = 0; b < m.nblk; ++b) {
    m.wg0[b] = g;
    g += (block_waves<P>(m.shape[b], (m.blk[b].n_elem + 15) / 16) + 3) / 4;
  }
  m.wg0[m.nblk] = g;
  if (g <= 0) return hipSuccess;
  switch (opk) {
    case OPK_MASS_LM: hipLaunchKernelGGL((k_localmat_affine_bf16_mesh<P, OPK_MASS, NPART>), dim3((unsigned)g), dim3(256), 0, s, m); break;
    case OPK_LAP_LM: hipLaunchKernelGGL((k_localmat_affine_bf16_mesh<P, OPK_LAP, NPART>), dim3((unsigned)g), dim3(256), 0, s, m); break;
    case OPK_HELM_LM: hipLaunchKernelGGL((k_localmat_affine_bf16_mesh<P, OPK_HELM, NPART>), dim3((unsigned)g), dim3(256), 0, s, m); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int SH, int P>
static hipError_t launch_bf16_sp(int opk, int nparts, const AffineBf16Args& a, hipStream_t s) {
  const bool three = nparts == 3;
  switch (opk) {
    case OPK_MASS_LM:
      return three ? launch_bf16_op<SH, P, OPK_MASS, 3>(a, s) : launch_bf16_op<SH, P, OPK_MASS, 2>(a, s);
    case OPK_LAP_LM:
      return three ? launch_bf16_op<SH, P, OPK_LAP, 3>(a, s) : launch_bf16_op<SH, P, OPK_LAP, 2>(a, s);
    case OPK_HELM_LM:
      return three ? launch_bf16_op<SH, P, OPK_HELM, 3>(a, s) : launch_bf16_op<SH, P, OPK_HELM, 2>(a, s);
  }
  return hipErrorInvalidValue;
}

template <int SH>
static hipError_t launch_bf16_s(int P, int opk, int nparts, const AffineBf16Args& a, hipStream_t s) {
  switch (P) {
    case 1: return launch_bf16_sp<SH, 1>(opk, nparts, a, s);
    case 2: return launch_bf16_sp<SH, 2>(opk, nparts, a, s);
    case 3: return launch_bf16_sp<SH, 3>(opk, nparts, a, s);
    case 4: return launch_bf16_sp<SH, 4>(opk, nparts, a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_localmat_affine_bf16(int sh, int P, int opk, int nparts, const bf16_frag* afrag, const double* coef,
                                       const float* in, float* out, long long n_elem, double lambda, hipStream_t s) {
  if (nparts != 2 && nparts != 3) return hipErrorInvalidValue;
  AffineBf16Args a;
  a.afrag = reinterpret_cast<const bf16x8*>(afrag);
  a.coef = coef;
  a.in = in;
  a.out = out;
  a.n_elem = n_elem;
  a.lambda = lambda;
  switch (sh) {
    case HEX: return launch_bf16_s<HEX>(P, opk, nparts, a, s);
    case PRISM: return launch_bf16_s<PRISM>(P, opk, nparts, a, s);
    case PYR: return launch_bf16_s<PYR>(P, opk, nparts, a, s);
    case TET: return launch_bf16_s<TET>(P, opk, nparts, a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_localmat_affine_bf16_mesh(int P, int opk, int nparts, int nblk, const int* shape,
                                            const bf16_frag* const* afrag, const double* const* coef,
                                            const float* const* in, float* const* out, const long long* n_elem,
                                            double lambda, hipStream_t s) {
  if ((nparts != 2 && nparts != 3) || nblk < 1 || nblk > BF16_MAX_BLOCKS) return hipErrorInvalidValue;
  AffineBf16Mesh m{};
  m.nblk = nblk;
  for (int b = 0; b < nblk; ++b) {
    m.shape[b] = shape[b];
    m.blk[b].afrag = reinterpret_cast<const bf16x8*>(afrag[b]);
    m.blk[b].coef = coef[b];
    m.blk[b].in = in[b];
    m.blk[b].out = out[b];
    m.blk[b].n_elem = n_elem[b];
    m.blk[b].lambda = lambda;
  }
  const bool three = nparts == 3;
  switch (P) {
    case 1: return three ? launch_bf16_mesh_pn<1, 3>(opk, m, s) : launch_bf16_mesh_pn<1, 2>(opk, m, s);
    case 2: return three ? launch_bf16_mesh_pn<2, 3>(opk, m, s) : launch_bf16_mesh_pn<2, 2>(opk, m, s);
    case 3: return three ? launch_bf16_mesh_pn<3, 3>(opk, m, s) : launch_bf16_mesh_pn<3, 2>(opk, m, s);
    case 4: return three ? launch_bf16_mesh_pn<4, 3>(opk, m, s) : launch_bf16_mesh_pn<4, 2>(opk, m, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace shp
