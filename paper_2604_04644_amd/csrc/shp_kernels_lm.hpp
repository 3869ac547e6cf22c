// HIP kernels of libshp for gfx950: the local-matrix strategy on FP64 MFMA,
// curved blocks ([B; d_d B] with the per-point metric) and affine blocks (7
// reference matrices, 7 coefficients per element).
#pragma once
#include "shp_kernels.hpp"

namespace shp {

// ---------------------------------------------------------------------------
// Local-matrix strategy on FP64 MFMA (Sec. 3.3.1 StdMat, Alg. 1; the
// non-collocated form the paper prescribes for it, Sec. 3.3.4)
// ---------------------------------------------------------------------------
// A work-group of 4 waves takes 16 elements (the N = 16 columns of the MFMA
// tiles).  Bcat = [B; d_1 B; d_2 B; d_3 B] (rows: points, padded to 16;
// columns: modes, padded to 16) is shared by all elements.  Each wave walks
// blocks of 16 points:
//   U_d = Bcat_d[block] X        (v_mfma_f64_16x16x4f64, K = modes)
//   metric on U_d in registers   (lane l, register i: point 4i + l/16, element l%16)
//   Y  += Bcat_d[block]^T U'_d   (the accumulator registers are the B operand)
// and the waves' partial Y are summed in LDS in a fixed order.
// MFMA operand layouts: A lane l = A[l%16][l/16]; B lane l = B[l/16][l%16];
// D lane l register i = D[4i + l/16][l%16].

typedef double dbl4 __attribute__((ext_vector_type(4)));

struct LocalMatArgs {
  const double* bcat;  // [4*Q3p][Kp]
  const double* bt;    // the same transposed, [Kp][4*Q3p]
  const double* fac;   // [n][NFAC][Q3]
  const double* in;    // [n][NP]
  double* out;         // [n][NP]
  long long n_elem;
  double lambda;
};

template <int SH, int P, int OP>
__device__ void localmat_tile(const LocalMatArgs& a, long long e0, int ne, double* smem) {
  constexpr int Q = P + 2, Q3 = Q * Q * Q;
  constexpr int Q3p = (Q3 + 15) / 16 * 16;
  constexpr int NP = num_modes(SH, P);
  constexpr int Kp = (NP + 15) / 16 * 16;
  constexpr int MB = Kp / 16;               // 16-row blocks of Y
  constexpr int ND = (OP == OPK_MASS) ? 1 : 4;
  constexpr int D0 = (OP == OPK_LAP) ? 1 : 0;  // the Laplacian has no mass term
  double* X = smem;            // [Kp][16]
  double* R = smem + Kp * 16;  // [Kp][16] reduction
  const int tidx = threadIdx.x, lane = tidx & 63, wave = tidx >> 6;
  const int col = lane & 15, kq = lane >> 4;
  // x tile transposed into LDS, zero padded
  for (int t = tidx; t < Kp * 16; t += blockDim.x) {
    const int m = t / 16, e = t - m * 16;
    X[t] = (m < NP && e < ne) ? a.in[(e0 + e) * NP + m] : 0.0;
  }
  __syncthreads();
  const gptr_t B = as_global(a.bcat);
  const gptr_t Bt = as_global(a.bt);
  const gptr_t G = as_global(a.fac) + e0 * (long long)(NFAC * Q3);
  const bool live = col < ne;
  dbl4 y[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) y[mb] = dbl4{0.0, 0.0, 0.0, 0.0};
  for (int qb = wave; qb < Q3p / 16; qb += (int)(blockDim.x >> 6)) {
    dbl4 u[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) u[d] = dbl4{0.0, 0.0, 0.0, 0.0};
    // U_d = Bcat_d[qb] X (a step's fragments loaded together, from the
    // transposed copy: the point index runs across lanes)
    for (int kb = 0; kb < Kp / 4; ++kb) {
      const double b = X[(4 * kb + kq) * 16 + col];
      double av[ND];
#pragma unroll
      for (int d = 0; d < ND; ++d) av[d] = Bt[(long long)(4 * kb + kq) * (4 * Q3p) + d * Q3p + qb * 16 + col];
#pragma unroll
      for (int d = 0; d < ND; ++d) u[d] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[d], b, u[d], 0, 0, 0);
    }
    // metric at the lane's 4 points of this element: loads from clamped
    // indices without branches, dead lanes and padding points zeroed after
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int pt = qb * 16 + 4 * i + kq;
      const bool on = live && pt < Q3;
      const gptr_t g = G + (live ? col : 0) * (NFAC * Q3) + (pt < Q3 ? pt : Q3 - 1);
      const double jw = g[0];
      if (OP == OPK_MASS) {
        u[0][i] = on ? jw * u[0][i] : 0.0;
      } else {
        const double g00 = g[1 * Q3], g01 = g[2 * Q3], g02 = g[3 * Q3];
        const double g11 = g[4 * Q3], g12 = g[5 * Q3], g22 = g[6 * Q3];
        const double d0 = u[1][i], d1 = u[2][i], d2 = u[3][i];
        u[1][i] = on ? g00 * d0 + g01 * d1 + g02 * d2 : 0.0;
        u[2][i] = on ? g01 * d0 + g11 * d1 + g12 * d2 : 0.0;
        u[3][i] = on ? g02 * d0 + g12 * d1 + g22 * d2 : 0.0;
        u[0][i] = (OP == OPK_HELM && on) ? a.lambda * jw * u[0][i] : 0.0;
      }
    }
    // Y += Bcat_d[qb]^T U'_d; the K-slab kb of this block is register kb
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      double av[ND][4];
#pragma unroll
      for (int d = D0; d < ND; ++d)
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) av[d][kb] = B[(long long)(d * Q3p + qb * 16 + 4 * kb + kq) * Kp + mb * 16 + col];
#pragma unroll
      for (int d = D0; d < ND; ++d)
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) y[mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[d][kb], u[d][kb], y[mb], 0, 0, 0);
    }
  }
  // sum the waves' partial results in a fixed order
  const int nw = (int)(blockDim.x >> 6);
  for (int w = 0; w < nw; ++w) {
    if (wave == w) {
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int m = mb * 16 + 4 * i + kq;
          R[m * 16 + col] = (w == 0 ? 0.0 : R[m * 16 + col]) + y[mb][i];
        }
    }
    __syncthreads();
  }
  for (int t = tidx; t < ne * NP; t += blockDim.x) {
    const int e = t / NP, m = t - e * NP;
    a.out[(e0 + e) * NP + m] = R[m * 16 + e];
  }
}

template <int SH, int P, int OP>
__global__ void __launch_bounds__(256) k_localmat(LocalMatArgs a) {
  extern __shared__ double smem[];
  const long long e0 = (long long)blockIdx.x * 16;
  const long long rem = a.n_elem - e0;
  const int ne = rem < 16 ? (int)rem : 16;
  if (ne <= 0) return;
  localmat_tile<SH, P, OP>(a, e0, ne, smem);
}

// ---------------------------------------------------------------------------
// Local matrices of affine elements (FP64 MFMA)
// ---------------------------------------------------------------------------
// With constant d xi/d x the elemental operator is a combination of 7 shared
// reference matrices, H_e = lambda |J| A_0 + sum_{k=1..6} c_{e,k} A_k (mass and
// the xi-space stiffness blocks, built from the same quadrature), so
//   Y = [A_0 ... A_6] [c_0 X; ...; c_6 X]
// is one dense FP64 contraction with K = 7 N_P per 16-element tile.  A
// tile's B operand is its coefficients scaled by the element's c_k, and the A
// fragments stream from a fragment-ordered copy of the matrices (64
// consecutive doubles per fragment, one per lane):
//   afrag[((kb * 7 + k) * MB + mb) * 64 + lane] = A_k[16 mb + lane%16][4 kb + lane/16].

// Work per wave of the affine kernels: G 16-element tiles that share every A
// fragment the wave loads (G MFMAs per fragment load), and MBW of the tile's
// row blocks (the tile's rows are split among MB / MBW waves).  Every MFMA
// takes its own A fragment, so a row split repeats only the cheap B operand;
// it gives a mesh block of a few thousand elements enough waves to hide the
// fragment loads from L2.  Measured on every shape at P = 3 and 4, at the
// mesh blocks' sizes and at 4M DOF: one row block and two tiles per wave is
// fastest in FP64 at every order (hex P = 4, 8192 elements: 95 -> 47 us;
// 32000: 172 -> 157 us), except on tetrahedra, whose few row blocks stay in
// one wave (and at P = 4 one tile per wave).  Uneven splits (a last wave
// with fewer row blocks) measured far slower and are not offered.
template <int SH, int P>
__host__ __device__ constexpr int lm_row_blocks() {
  return (num_modes(SH, P) + 15) / 16;
}
template <int SH, int P>
__host__ __device__ constexpr int lm_rows_per_wave() {
  return SH == TET ? lm_row_blocks<SH, P>() : 1;
}
template <int SH, int P>
__host__ __device__ constexpr int lm_tiles_per_wave() {
  return (SH == TET && P == 4) ? 1 : 2;
}
// The FP32 kernel (half the fragment bytes) gains from the split and the
// shared fragments at P = 4 only (and hex P = 3 from two tiles per wave);
// below, one tile and all its row blocks per wave measured fastest.
template <int SH, int P>
__host__ __device__ constexpr int lm32_rows_per_wave() {
  return (P == 4 && SH != TET) ? 1 : lm_row_blocks<SH, P>();
}
template <int SH, int P>
__host__ __device__ constexpr int lm32_tiles_per_wave() {
  return ((P == 4 && SH != TET) || (P == 3 && SH == HEX)) ? 2 : 1;
}
// waves of a launch over n_elem elements with G tiles and MBW row blocks per wave
template <int SH, int P>
__host__ __device__ constexpr long long lm_waves(long long n_elem, int G, int MBW) {
  return ((n_elem + 15) / 16 + G - 1) / G * (lm_row_blocks<SH, P>() / MBW);
}

struct AffineMatArgs {
  const double* afrag;  // fragment-ordered reference matrices
  const double* coef;   // [n][7]
  const double* in;     // [n][NP]
  double* out;          // [n][NP]
  long long n_elem;
  double lambda;
};

// wave gw of one affine block
template <int SH, int P, int OP, int G, int MBW>
__device__ __forceinline__ void lma_wave(const AffineMatArgs& a, long long gw) {
  constexpr int NP = num_modes(SH, P);
  constexpr int MB = lm_row_blocks<SH, P>();
  static_assert(MB % MBW == 0, "a tile's row blocks split evenly among its waves");
  constexpr int W = MB / MBW;
  constexpr int K0 = (OP == OPK_LAP) ? 1 : 0;     // the Laplacian has no mass term
  constexpr int K1 = (OP == OPK_MASS) ? 1 : NAFF;  // the mass has only A_0
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, kq = lane >> 4;
  const long long e0 = gw / W * (16 * G);  // the wave's first element
  const int mb0 = (int)(gw % W) * MBW;     // and first row block
  if (e0 >= a.n_elem) return;  // whole waves only: no barriers below
  bool live[G];
  long long ec[G];
  double c[G][NAFF];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    live[g] = e0 + 16 * g + col < a.n_elem;
    // dead lanes read a live element: no branches around the loads, so that
    // a step's loads are in flight together
    ec[g] = live[g] ? e0 + 16 * g + col : e0;
#pragma unroll
    for (int k = 0; k < NAFF; ++k) c[g][k] = live[g] ? a.coef[ec[g] * NAFF + k] : 0.0;
    if (OP == OPK_HELM) c[g][0] *= a.lambda;
  }
  dbl4 acc[G][MBW];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int j = 0; j < MBW; ++j) acc[g][j] = dbl4{0.0, 0.0, 0.0, 0.0};
  const gptr_t Af = as_global(a.afrag) + (long long)mb0 * 64 + lane;
  const gptr_t X = as_global(a.in);
  // K steps of 4 up to N_P only: the columns of A_k past N_P are zero padding
  // (at N_P = 4 that is one step of the four a 16-wide padding would take)
  double xn[G];
#pragma unroll
  for (int g = 0; g < G; ++g) xn[g] = X[ec[g] * NP + (kq < NP ? kq : NP - 1)];
  for (int kb = 0; kb < (NP + 3) / 4; ++kb) {
    const int n = 4 * kb + kq;
    const int nn = n + 4 < NP ? n + 4 : NP - 1;
    double xb[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      xb[g] = (live[g] && n < NP) ? xn[g] : 0.0;
      xn[g] = X[ec[g] * NP + nn];  // the next step's value, in flight during this one
    }
#pragma unroll
    for (int k = K0; k < K1; ++k) {
      double av[MBW];  // the step's fragments of A_k, loaded together
#pragma unroll
      for (int j = 0; j < MBW; ++j) av[j] = Af[(long long)((kb * NAFF + k) * MB + j) * 64];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const double b = xb[g] * c[g][k];
#pragma unroll
        for (int j = 0; j < MBW; ++j) acc[g][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[j], b, acc[g][j], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int g = 0; g < G; ++g) {
    double* Y = a.out + (e0 + 16 * g + col) * NP;
#pragma unroll
    for (int j = 0; j < MBW; ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = (mb0 + j) * 16 + 4 * i + kq;
        if (live[g] && m < NP) Y[m] = acc[g][j][i];
      }
  }
}

template <int SH, int P, int OP, int G = lm_tiles_per_wave<SH, P>(), int MBW = lm_rows_per_wave<SH, P>()>
__global__ void __launch_bounds__(256) k_localmat_affine(AffineMatArgs a) {
  lma_wave<SH, P, OP, G, MBW>(a, (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
}

// Every affine block of one order in one launch: block b owns the
// work-groups from wg0[b] (its waves rounded up to whole work-groups), so
// the blocks run side by side instead of one launch after another.
constexpr int AFF_MESH_MAX = 8;
struct AffineMatMesh {
  AffineMatArgs blk[AFF_MESH_MAX];
  long long wg0[AFF_MESH_MAX + 1];
  int shape[AFF_MESH_MAX];
  int nblk;
};

template <int P, int OP>
__global__ void __launch_bounds__(256) k_localmat_affine_mesh(AffineMatMesh m) {
  const long long g = blockIdx.x;
  int b = 0;
  while (b + 1 < m.nblk && g >= m.wg0[b + 1]) ++b;
  const long long w = (g - m.wg0[b]) * (blockDim.x >> 6) + (threadIdx.x >> 6);
  switch (m.shape[b]) {
    case HEX: lma_wave<HEX, P, OP, lm_tiles_per_wave<HEX, P>(), lm_rows_per_wave<HEX, P>()>(m.blk[b], w); break;
    case PRISM: lma_wave<PRISM, P, OP, lm_tiles_per_wave<PRISM, P>(), lm_rows_per_wave<PRISM, P>()>(m.blk[b], w); break;
    case PYR: lma_wave<PYR, P, OP, lm_tiles_per_wave<PYR, P>(), lm_rows_per_wave<PYR, P>()>(m.blk[b], w); break;
    default: lma_wave<TET, P, OP, lm_tiles_per_wave<TET, P>(), lm_rows_per_wave<TET, P>()>(m.blk[b], w); break;
  }
}

// ---------------------------------------------------------------------------
// Local-matrix forms of the transforms (Sec. 3.3.1, Alg. 1: the backward
// transform as one GEMM over all elements, no element-wise scaling)
// ---------------------------------------------------------------------------
// One wave owns a 16-element tile (the N = 16 columns), 4 waves per
// work-group, no LDS.  With Bcat = [B; d_1 B; d_2 B; d_3 B] (rows: points
// padded to Q3p, columns: modes padded to Kp) and per point jw and
// d eta_d / d x_i:
//   BwdTrans       U = B X                          (M = points, K = modes)
//   IProduct       Y = B^T (jw F)                   (M = modes, K = points)
//   IProductDeriv  Y = sum_d (d_d B)^T (jw sum_i d eta_d/d x_i F_i)
//   PhysDeriv      dU/dx_i = sum_d d eta_d/d x_i (D_d U), D_d the dense
//                  collocation derivative matrices (Q3p x Q3p) of the tensor
//                  points, since PhysDeriv acts on values at the points.
// Loads sit outside branches (clamped indices, values masked after), so that
// a step's fragments are in flight together.

struct LocalXformArgs {
  const double* bcat;  // [4 Q3p][Kp]
  const double* dmat;  // [3][Q3p][Q3p] (PhysDeriv), each D_d transposed: [in][out]
  const double* bt;    // [Kp][4 Q3p] Bcat transposed (BwdTrans reads its B part)
  const double* fac;   // [n][NFAC][Q3]
  const double* dxi;   // [n][NDXI][Q3]
  const double* in;
  double* out;
  long long n_elem;
  long long in_cs, out_cs;  // component strides of vector fields at the points
  int wpt;                  // waves per tile (BwdTrans, PhysDeriv: they share the point row blocks)
};

template <int SH, int P, int OP>
__global__ void __launch_bounds__(256) k_localmat_xform(LocalXformArgs a) {
  constexpr int Q = P + 2, Q3 = Q * Q * Q;
  constexpr int Q3p = (Q3 + 15) / 16 * 16;
  constexpr int NP = num_modes(SH, P);
  constexpr int Kp = (NP + 15) / 16 * 16;
  constexpr int MB = Kp / 16, QB = Q3p / 16;
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, kq = lane >> 4;
  // a tile's point row blocks qb = w0, w0 + wpt, ... go to its wpt waves
  const long long gw = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const long long e0 = gw / a.wpt * 16;
  const int w0 = (int)(gw % a.wpt);
  if (e0 >= a.n_elem) return;  // whole waves only
  const long long e = e0 + col;
  const bool live = e < a.n_elem;
  const long long ec = live ? e : e0;
  const gptr_t Bc = as_global(a.bcat);
  if constexpr (OP == OPK_BWD) {
    const gptr_t Bt = as_global(a.bt);
    // the tile's coefficients in registers: xr[kb] = x_e[4 kb + kq]
    constexpr int KS = Kp / 4;
    double xr[KS];
#pragma unroll
    for (int kb = 0; kb < KS; ++kb) {
      const int n = 4 * kb + kq;
      const double v = a.in[ec * NP + (n < NP ? n : NP - 1)];
      xr[kb] = (live && n < NP) ? v : 0.0;
    }
    for (int qb = w0; qb < QB; qb += a.wpt) {
      dbl4 acc = dbl4{0.0, 0.0, 0.0, 0.0};
      double av[KS];
#pragma unroll
      for (int kb = 0; kb < KS; ++kb) av[kb] = Bt[(long long)(4 * kb + kq) * (4 * Q3p) + qb * 16 + col];
#pragma unroll
      for (int kb = 0; kb < KS; ++kb) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[kb], xr[kb], acc, 0, 0, 0);
      if (live)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int pt = qb * 16 + 4 * i + kq;
          if (pt < Q3) a.out[e * Q3 + pt] = acc[i];
        }
    }
  } else if constexpr (OP == OPK_IPR || OP == OPK_IPRD) {
    constexpr int ND = (OP == OPK_IPR) ? 1 : 3;
    constexpr int D0 = (OP == OPK_IPR) ? 0 : 1;  // Bcat row block of the first table
    dbl4 acc[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) acc[mb] = dbl4{0.0, 0.0, 0.0, 0.0};
    const double* fac = a.fac + ec * (long long)(NFAC * Q3);
    const double* dxi = a.dxi + ec * (long long)(NDXI * Q3);
    for (int kb = 0; kb < Q3p / 4; ++kb) {
      const int pt = 4 * kb + kq;
      const int pc = pt < Q3 ? pt : Q3 - 1;
      const bool on = live && pt < Q3;
      const double jw = fac[pc];
      double g[ND];
      if constexpr (OP == OPK_IPR) {
        g[0] = on ? jw * a.in[ec * Q3 + pc] : 0.0;
      } else {
        const double f0 = a.in[0 * a.in_cs + ec * Q3 + pc];
        const double f1 = a.in[1 * a.in_cs + ec * Q3 + pc];
        const double f2 = a.in[2 * a.in_cs + ec * Q3 + pc];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const double v = dxi[(d * 3 + 0) * Q3 + pc] * f0 + dxi[(d * 3 + 1) * Q3 + pc] * f1 +
                           dxi[(d * 3 + 2) * Q3 + pc] * f2;
          g[d] = on ? jw * v : 0.0;
        }
      }
      double av[ND][MB];
#pragma unroll
      for (int d = 0; d < ND; ++d)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) av[d][mb] = Bc[(long long)((D0 + d) * Q3p + pt) * Kp + mb * 16 + col];
#pragma unroll
      for (int d = 0; d < ND; ++d)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) acc[mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[d][mb], g[d], acc[mb], 0, 0, 0);
    }
    if (live)
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int m = mb * 16 + 4 * i + kq;
          if (m < NP) a.out[e * NP + m] = acc[mb][i];
        }
  } else {
    static_assert(OP == OPK_DERIV, "local-matrix transform");
    const gptr_t Dm = as_global(a.dmat);
    const double* dxi = a.dxi + ec * (long long)(NDXI * Q3);
    for (int qb = w0; qb < QB; qb += a.wpt) {
      dbl4 acc[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) acc[d] = dbl4{0.0, 0.0, 0.0, 0.0};
      for (int kb = 0; kb < Q3p / 4; ++kb) {
        const int pin = 4 * kb + kq;
        const double u = a.in[ec * Q3 + (pin < Q3 ? pin : Q3 - 1)];
        const double ub = (live && pin < Q3) ? u : 0.0;
        double av[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) av[d] = Dm[((long long)d * Q3p + 4 * kb + kq) * Q3p + qb * 16 + col];
#pragma unroll
        for (int d = 0; d < 3; ++d) acc[d] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[d], ub, acc[d], 0, 0, 0);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int pt = qb * 16 + 4 * i + kq;
        const int pc = pt < Q3 ? pt : Q3 - 1;
        double m[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) m[c] = dxi[c * Q3 + pc];
        if (live && pt < Q3)
#pragma unroll
          for (int x = 0; x < 3; ++x)
            a.out[x * a.out_cs + e * Q3 + pt] = m[0 * 3 + x] * acc[0][i] + m[1 * 3 + x] * acc[1][i] + m[2 * 3 + x] * acc[2][i];
      }
    }
  }
}

// The same contraction in FP32 on v_mfma_f32_16x16x4f32 (FP32 vectors, the
// fragment-ordered matrices rounded to FP32, coefficients rounded to FP32):
// the operand layouts are those of the FP64 instruction, the accumulator's
// register i holds row 4 (l/16) + i.
typedef float flt4_ __attribute__((ext_vector_type(4)));

struct AffineMatArgs32 {
  const float* afrag;  // the FP64 fragments rounded to FP32, same order
  const double* coef;  // [n][7]
  const float* in;     // [n][NP]
  float* out;          // [n][NP]
  long long n_elem;
  double lambda;
};

template <int SH, int P, int OP, int G, int MBW>
__device__ __forceinline__ void lma32_wave(const AffineMatArgs32& a, long long gw) {
  constexpr int NP = num_modes(SH, P);
  constexpr int MB = lm_row_blocks<SH, P>();
  static_assert(MB % MBW == 0, "a tile's row blocks split evenly among its waves");
  constexpr int W = MB / MBW;
  constexpr int K0 = (OP == OPK_LAP) ? 1 : 0;
  constexpr int K1 = (OP == OPK_MASS) ? 1 : NAFF;
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, kq = lane >> 4;
  const long long e0 = gw / W * (16 * G);
  const int mb0 = (int)(gw % W) * MBW;
  if (e0 >= a.n_elem) return;
  bool live[G];
  long long ec[G];
  float c[G][NAFF];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    live[g] = e0 + 16 * g + col < a.n_elem;
    ec[g] = live[g] ? e0 + 16 * g + col : e0;
#pragma unroll
    for (int k = 0; k < NAFF; ++k) {
      double cd = a.coef[ec[g] * NAFF + k];
      if (OP == OPK_HELM && k == 0) cd *= a.lambda;
      c[g][k] = live[g] ? (float)cd : 0.0f;
    }
  }
  flt4_ acc[G][MBW];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int j = 0; j < MBW; ++j) acc[g][j] = flt4_{0.0f, 0.0f, 0.0f, 0.0f};
  const float* Af = a.afrag + (long long)mb0 * 64 + lane;
  const float* X = a.in;
  float xn[G];
#pragma unroll
  for (int g = 0; g < G; ++g) xn[g] = X[ec[g] * NP + (kq < NP ? kq : NP - 1)];
  for (int kb = 0; kb < (NP + 3) / 4; ++kb) {
    const int n = 4 * kb + kq;
    const int nn = n + 4 < NP ? n + 4 : NP - 1;
    float xb[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      xb[g] = (live[g] && n < NP) ? xn[g] : 0.0f;
      xn[g] = X[ec[g] * NP + nn];
    }
#pragma unroll
    for (int k = K0; k < K1; ++k) {
      float av[MBW];
#pragma unroll
      for (int j = 0; j < MBW; ++j) av[j] = Af[(long long)((kb * NAFF + k) * MB + j) * 64];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const float b = xb[g] * c[g][k];
#pragma unroll
        for (int j = 0; j < MBW; ++j) acc[g][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[j], b, acc[g][j], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int g = 0; g < G; ++g) {
    if (!live[g]) continue;
    float* Y = a.out + (e0 + 16 * g + col) * NP;
#pragma unroll
    for (int j = 0; j < MBW; ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = (mb0 + j) * 16 + 4 * kq + i;
        if (m < NP) Y[m] = acc[g][j][i];
      }
  }
}

template <int SH, int P, int OP, int G = lm32_tiles_per_wave<SH, P>(), int MBW = lm32_rows_per_wave<SH, P>()>
__global__ void __launch_bounds__(256) k_localmat_affine_f32(AffineMatArgs32 a) {
  lma32_wave<SH, P, OP, G, MBW>(a, (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
}

// every FP32 affine block of one order in one launch (as the FP64 one)
struct AffineMatMesh32 {
  AffineMatArgs32 blk[AFF_MESH_MAX];
  long long wg0[AFF_MESH_MAX + 1];
  int shape[AFF_MESH_MAX];
  int nblk;
};

template <int P, int OP>
__global__ void __launch_bounds__(256) k_localmat_affine_f32_mesh(AffineMatMesh32 m) {
  const long long g = blockIdx.x;
  int b = 0;
  while (b + 1 < m.nblk && g >= m.wg0[b + 1]) ++b;
  const long long w = (g - m.wg0[b]) * (blockDim.x >> 6) + (threadIdx.x >> 6);
  switch (m.shape[b]) {
    case HEX: lma32_wave<HEX, P, OP, lm32_tiles_per_wave<HEX, P>(), lm32_rows_per_wave<HEX, P>()>(m.blk[b], w); break;
    case PRISM: lma32_wave<PRISM, P, OP, lm32_tiles_per_wave<PRISM, P>(), lm32_rows_per_wave<PRISM, P>()>(m.blk[b], w); break;
    case PYR: lma32_wave<PYR, P, OP, lm32_tiles_per_wave<PYR, P>(), lm32_rows_per_wave<PYR, P>()>(m.blk[b], w); break;
    default: lma32_wave<TET, P, OP, lm32_tiles_per_wave<TET, P>(), lm32_rows_per_wave<TET, P>()>(m.blk[b], w); break;
  }
}

template <int SH, int P>
constexpr size_t lds_bytes_localmat() {
  constexpr int Kp = (num_modes(SH, P) + 15) / 16 * 16;
  return sizeof(double) * 2 * Kp * 16;
}

}  // namespace shp
