// HIP kernels of libshp for gfx950: the affine local-matrix action with
// split-BF16 operands on the BF16 matrix cores (v_mfma_f32_16x16x32_bf16),
// FP32 accumulation.
//
// An affine element's operator is H_e = sum_k c_{e,k} A_k over 7 shared
// reference matrices (the local-matrix form, Sec. 3.3.1), so a tile of 16
// elements is one dense contraction
//   Y[m][e] = sum_kappa A[m][kappa] B[kappa][e],  kappa = k NPp + n,
//   B[k NPp + n][e] = c_{e,k} x_e[n]
// with K = 7 NPp (N_P padded to a multiple of 8, so that the 8 values a lane
// holds belong to one matrix).  Each operand is a sum of bfloat16 parts, each
// the bfloat16 part of what the previous parts leave (A: rounded to nearest on
// the host; B: truncated, see below); a product of two split operands keeps
// the part products of order below NPART:
//   NPART = 2: a0 b0 + a0 b1 + a1 b0            (3 MFMAs, about 2^-16)
//   NPART = 3: ... + a0 b2 + a1 b1 + a2 b0      (6 MFMAs, about 2^-24)
// relative to |a||b| per product, accumulated in FP32.
//
// MFMA operand layouts of v_mfma_f32_16x16x32_bf16: A lane l holds row l%16
// and 8 consecutive K values from 8 (l/16); B lane l holds column l%16 and the
// same K values; D lane l register i holds row 4 (l/16) + i, column l%16.
// Only the row and column maps matter for the result: A and B share one K
// order.
#pragma once
#include "shp_kernels.hpp"

namespace shp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

struct AffineBf16Args {
  const bf16x8* afrag;  // [KS][MB][3 parts][64 lanes] fragments of the reference matrices
  const double* coef;   // [n][7]: |J| and |J| (J^-1 J^-T)_ab
  const float* in;      // [n][NP]
  float* out;           // [n][NP]
  long long n_elem;
  double lambda;
};

// One wave owns a 16-element tile and MBW of its MB blocks of 16 output rows
// (the tile's MB / MBW waves each form the tile's B operand and stream their
// rows' A fragments); 4 waves per work-group, no LDS and no barriers.  The B
// parts are truncations, so three parts hold an FP32 value exactly:
// v = h0 + h1 + h2 with h the top 16 bits of what is left; two parts leave
// at most 2^-16 of it.
// output row blocks per wave: at most 4, so that a tile's rows spread over
// several waves (a block of a few thousand elements still fills the chip)
// while a K step's MFMA work (MBW x 3 or 6) keeps up with forming its split B
// operand (about 70 VALU instructions per step); the rows shared evenly
// among the tile's waves.  Measured exception: the prism at P = 4 (5 row
// blocks) keeps them in one wave, as a 3 + 2 split ran up to 1.6x slower.
template <int SH, int P>
constexpr int bf16_mbw() {
  constexpr int MB = (num_modes(SH, P) + 15) / 16;
  constexpr int NW = (MB + 3) / 4;
  return (SH == PRISM && P == 4) ? MB : (MB + NW - 1) / NW;
}

// tiles of 16 elements per wave: each A fragment a wave loads serves G
// tiles' MFMAs; 2, and 4 for the prism and the tetrahedron at P = 4 (their
// waves then form 4 tiles' split operands per A fragment; measured 1.2-1.6x
// faster on both the mixed mesh's blocks and 4M-DOF blocks)
template <int SH, int P>
constexpr int bf16_g() {
  return ((SH == PRISM || SH == TET) && P == 4) ? 4 : 2;
}

// waves of a block of ntile 16-element tiles: (MB / MBW) per group of G
template <int SH, int P>
constexpr int bf16_waves_per_tile() {
  constexpr int MB = (num_modes(SH, P) + 15) / 16;
  return (MB + bf16_mbw<SH, P>() - 1) / bf16_mbw<SH, P>();
}

template <int SH, int P>
constexpr long long bf16_waves(long long ntile) {
  return (ntile + bf16_g<SH, P>() - 1) / bf16_g<SH, P>() * bf16_waves_per_tile<SH, P>();
}

// wave w of one block
template <int SH, int P, int OP, int NPART, int MBW = bf16_mbw<SH, P>(), int G = bf16_g<SH, P>()>
__device__ __forceinline__ void bf16_wave(const AffineBf16Args& a, long long w) {
  constexpr int NP = num_modes(SH, P);
  constexpr int NPp = (NP + 7) / 8 * 8;
  constexpr int MB = (NP + 15) / 16;
  constexpr int NMW = (MB + MBW - 1) / MBW;  // waves per tile
  constexpr int K0 = (OP == OPK_LAP) ? NPp : 0;           // the Laplacian has no mass term
  constexpr int K1 = (OP == OPK_MASS) ? NPp : NAFF * NPp;  // the mass has only A_0
  constexpr int KB0 = K0 / 32, KB1 = (K1 + 31) / 32;
  const int lane = threadIdx.x & 63;
  const long long eg = (w / NMW) * (16 * G);  // first element of the wave's tiles
  const int mb0 = (int)(w % NMW) * MBW;
  if (eg >= a.n_elem) return;  // whole waves only
  const int col = lane & 15, kq = lane >> 4;
  bool live[G];
  long long ee[G];
  float c[G][NAFF];
  const float* X[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    ee[g] = eg + 16 * g + col;
    live[g] = ee[g] < a.n_elem;
    const long long ec = live[g] ? ee[g] : eg;  // dead lanes read a live element (no branches around loads)
#pragma unroll
    for (int k = 0; k < NAFF; ++k) {
      double cd = a.coef[ec * NAFF + k];
      if (OP == OPK_HELM && k == 0) cd *= a.lambda;
      c[g][k] = live[g] ? (float)cd : 0.0f;
    }
    X[g] = a.in + ec * NP;
  }
  flt4 acc[G][MBW];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int i = 0; i < MBW; ++i) acc[g][i] = flt4{0.0f, 0.0f, 0.0f, 0.0f};
  // this lane's 8 K values of step kb: matrix k = kappa / NPp, modes n0 .. n0
  // + 7; loads from clamped (in-bounds) indices without branches, so that a
  // step's loads are in flight together and the next step's during this one
  auto load = [&](int kb, float (*v)[8]) {
    const int kap0 = 32 * kb + 8 * kq;
    const int n0 = kap0 - (kap0 / NPp) * NPp;
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int j = 0; j < 8; ++j) v[g][j] = X[g][n0 + j < NP ? n0 + j : NP - 1];
  };
  float xv[G][8];
  load(KB0, xv);
  for (int kb = KB0; kb < KB1; ++kb) {
    float xn[G][8];
    load(kb + 1 < KB1 ? kb + 1 : kb, xn);
    const int kap0 = 32 * kb + 8 * kq;
    const int k = kap0 / NPp, n0 = kap0 - k * NPp;
    const bool kin = kap0 >= K0 && kap0 < K1;
    u32x4 bw[G][NPART];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      float ck = c[g][0];
#pragma unroll
      for (int kk = 1; kk < NAFF; ++kk) ck = (k == kk) ? c[g][kk] : ck;
      const bool on = kin && live[g];
#pragma unroll
      for (int j2 = 0; j2 < 4; ++j2) {
        float v0 = (on && n0 + 2 * j2 < NP) ? ck * xv[g][2 * j2] : 0.0f;
        float v1 = (on && n0 + 2 * j2 + 1 < NP) ? ck * xv[g][2 * j2 + 1] : 0.0f;
#pragma unroll
        for (int pt = 0; pt < NPART; ++pt) {
          const unsigned u0 = __float_as_uint(v0) & 0xFFFF0000u, u1 = __float_as_uint(v1) & 0xFFFF0000u;
          bw[g][pt][j2] = (u0 >> 16) | u1;  // K value 2 j2 in the low half, 2 j2 + 1 in the high half
          v0 -= __uint_as_float(u0);
          v1 -= __uint_as_float(u1);
        }
      }
    }
    const bf16x8* Af = a.afrag + ((long long)kb * MB + mb0) * (BF16_PARTS * 64) + lane;
#pragma unroll
    for (int i = 0; i < MBW; ++i) {
      if (mb0 + i >= MB) break;
#pragma unroll
      for (int pa = 0; pa < NPART; ++pa) {
        const bf16x8 av = Af[(i * BF16_PARTS + pa) * 64];
#pragma unroll
        for (int pb = 0; pb + pa < NPART; ++pb)
#pragma unroll
          for (int g = 0; g < G; ++g)
            acc[g][i] =
                __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, __builtin_bit_cast(bf16x8, bw[g][pb]), acc[g][i], 0, 0, 0);
      }
    }
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int j = 0; j < 8; ++j) xv[g][j] = xn[g][j];
  }
#pragma unroll
  for (int g = 0; g < G; ++g) {
    if (!live[g]) continue;
    float* Y = a.out + ee[g] * NP;
#pragma unroll
    for (int i = 0; i < MBW; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = (mb0 + i) * 16 + 4 * kq + r;
        if (mb0 + i < MB && m < NP) Y[m] = acc[g][i][r];
      }
  }
}

template <int SH, int P, int OP, int NPART>
__global__ void __launch_bounds__(256) k_localmat_affine_bf16(AffineBf16Args a) {
  bf16_wave<SH, P, OP, NPART>(a, (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
}

// Every block of one order in one launch: block b owns the work-groups from
// wg0[b] (each block's waves rounded up to whole work-groups, so that a
// work-group's shape is uniform and the blocks' launches overlap).
constexpr int BF16_MAX_BLOCKS = 8;
struct AffineBf16Mesh {
  AffineBf16Args blk[BF16_MAX_BLOCKS];
  long long wg0[BF16_MAX_BLOCKS + 1];
  int shape[BF16_MAX_BLOCKS];
  int nblk;
};

template <int P, int OP, int NPART>
__global__ void __launch_bounds__(256) k_localmat_affine_bf16_mesh(AffineBf16Mesh m) {
  const long long g = blockIdx.x;
  int b = 0;
  while (b + 1 < m.nblk && g >= m.wg0[b + 1]) ++b;
  const long long w = (g - m.wg0[b]) * (blockDim.x >> 6) + (threadIdx.x >> 6);
  switch (m.shape[b]) {
    case HEX: bf16_wave<HEX, P, OP, NPART>(m.blk[b], w); break;
    case PRISM: bf16_wave<PRISM, P, OP, NPART>(m.blk[b], w); break;
    case PYR: bf16_wave<PYR, P, OP, NPART>(m.blk[b], w); break;
    default: bf16_wave<TET, P, OP, NPART>(m.blk[b], w); break;
  }
}

}  // namespace shp
