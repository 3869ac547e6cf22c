// Launchers of the split-BF16 affine local-matrix kernels: every shape,
// P = 1..4, mass / Laplacian / Helmholtz, two or three parts.
#include "shp_internal.hpp"
#include "shp_kernels_bf16.hpp"

namespace shp {

// output row blocks per wave: at most 4, so that a tile's rows spread over
// several waves (a block of a few thousand elements still fills the chip)
// while a K step's MFMA work (MBW x 3 or 6) keeps up with forming its split B
// operand (about 70 VALU instructions per step)
template <int SH, int P>
constexpr int bf16_mbw() {
  constexpr int MB = (num_modes(SH, P) + 15) / 16;
  return MB < 4 ? MB : 4;
}

template <int SH, int P, int OP, int NPART>
static hipError_t launch_bf16_op(const AffineBf16Args& a, hipStream_t s) {
  constexpr int MBW = bf16_mbw<SH, P>();
  constexpr int MB = (num_modes(SH, P) + 15) / 16;
  constexpr int NMW = (MB + MBW - 1) / MBW;
  const long long nwave = (a.n_elem + 15) / 16 * NMW;
  if (nwave <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_localmat_affine_bf16<SH, P, OP, NPART, MBW>), dim3((unsigned)((nwave + 3) / 4)), dim3(256), 0,
                     s, a);
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

}  // namespace shp
