// HIP kernels of libshp for gfx950: Laplacian / Helmholtz actions of
// iso-parametric elements with the geometry recomputed in every launch.
//
// An iso-parametric element's map is a polynomial of the solution's degree in
// the element's own basis, x_c = sum_m X_cm phi_m (Sec. 2.1: J is then a
// polynomial; Sec. 4: curvilinear elements with iso-parametric mappings).
// Instead of streaming 7 precomputed FP64 factors per point (56 Q^3 bytes per
// element), a tile reads its 3 N_P coordinate coefficients (24 N_P bytes) and
// rebuilds them in FP64: each coordinate goes through the backward transform
// and the collocated derivatives (the stages of the Helmholtz tile), which
// give d x_c/d eta_d at the points; then per point the determinant, the
// inverse d eta/d x, jw = w |det| / prod (1 - eta_d)^alpha_d (the reference
// weight table wref) and g = jw (d eta/d x)(d eta/d x)^T.
#pragma once
#include "shp_kernels.hpp"

namespace shp {

// d x/d eta at the tile's points -> the 7 factors of each point a thread owns
// (slots as in the geometry prefetch); returns false when a determinant is not
// positive or a factor not finite.  Ends with a barrier (LDS free again).
template <int SH, int P, int PPT>
__device__ __forceinline__ bool iso_geometry(const double* __restrict__ xco, const double* __restrict__ wref, long long e0, int ne,
                             const Tile_<SH, P, double>& T, GeoRegs<PPT>& g) {
  using D = Dims<SH, P>;
  constexpr int Q3 = D::Q3, NP = D::NP;
  double J[PPT][9];  // d x_c / d eta_d at c*3 + d
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    for (int t = tid(); t < ne * NP; t += nthr()) {
      const int e = t / NP, m = t - e * NP;
      T.G(e, 0)[m] = xco[((e0 + e) * 3 + c) * NP + m];
    }
    __syncthreads();
    bwd_r<SH, P, false>(T, ne, 0, 1);
    __syncthreads();
    bwd_q<SH, P, false>(T, ne, 1, 2);
    __syncthreads();
    bwd_p_grad0<SH, P>(T, ne);  // U = x_c, G0 = d x_c / d eta_1
    __syncthreads();
    grad12<SH, P, false>(T, ne);  // G1, G2 = d x_c / d eta_2, d eta_3
    __syncthreads();
#pragma unroll
    for (int it = 0; it < PPT; ++it) {
      const int t = tid() + it * nthr();
      if (t < ne * Q3) {
        const int e = t / Q3, pt = t - e * Q3;
        const int lp = lds_pt<SH, P>(pt);
        J[it][c * 3 + 0] = T.G(e, 0)[lp];
        J[it][c * 3 + 1] = T.G(e, 1)[lp];
        J[it][c * 3 + 2] = T.G(e, 2)[lp];
      }
    }
    __syncthreads();
  }
  bool ok = true;
#pragma unroll
  for (int it = 0; it < PPT; ++it) {
    const int t = tid() + it * nthr();
    if (t < ne * Q3) {
      const int pt = t - (t / Q3) * Q3;
      const double* A = J[it];
      // cofactors: inverse[d][i] = d eta_d / d x_i = cof[i][d] / det
      const double c00 = A[4] * A[8] - A[5] * A[7];
      const double c01 = A[5] * A[6] - A[3] * A[8];
      const double c02 = A[3] * A[7] - A[4] * A[6];
      const double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
      const double id = 1.0 / det;
      double M[9];  // d eta_d / d x_i at d*3 + i
      M[0] = c00 * id;
      M[1] = (A[2] * A[7] - A[1] * A[8]) * id;
      M[2] = (A[1] * A[5] - A[2] * A[4]) * id;
      M[3] = c01 * id;
      M[4] = (A[0] * A[8] - A[2] * A[6]) * id;
      M[5] = (A[2] * A[3] - A[0] * A[5]) * id;
      M[6] = c02 * id;
      M[7] = (A[1] * A[6] - A[0] * A[7]) * id;
      M[8] = (A[0] * A[4] - A[1] * A[3]) * id;
      const double jw = wref[pt] * det;
      double* f = g.v[it];
      f[0] = jw;
      f[1] = jw * (M[0] * M[0] + M[1] * M[1] + M[2] * M[2]);
      f[2] = jw * (M[0] * M[3] + M[1] * M[4] + M[2] * M[5]);
      f[3] = jw * (M[0] * M[6] + M[1] * M[7] + M[2] * M[8]);
      f[4] = jw * (M[3] * M[3] + M[4] * M[4] + M[5] * M[5]);
      f[5] = jw * (M[3] * M[6] + M[4] * M[7] + M[5] * M[8]);
      f[6] = jw * (M[6] * M[6] + M[7] * M[7] + M[8] * M[8]);
      bool good = det > 0.0 && isfinite(det);
#pragma unroll
      for (int c = 1; c < NFAC; ++c) good = good && isfinite(f[c]);
      ok = ok && good;
    }
  }
  return ok;
}

// The tile of work-group blockIdx.x: from the tile list, or, with
// blk_only >= 0, the tiles of E_only elements of that block in order.
__device__ __forceinline__ bool iso_tile(const BlockStatic* __restrict__ blocks, const Tile* __restrict__ tiles,
                                         int ntiles, int blk_only, int E_only, Tile& tl) {
  if (blk_only >= 0) {
    tl.blk = blk_only;
    tl.e0 = (long long)blockIdx.x * E_only;
    const long long rem = blocks[blk_only].n_elem - tl.e0;
    if (rem <= 0) return false;
    tl.ne = rem < E_only ? (int)rem : E_only;
    return true;
  }
  if ((int)blockIdx.x >= ntiles) return false;
  tl = tiles[blockIdx.x];
  return true;
}

template <int SH, int P, int OP, int PPT>
__device__ __forceinline__ void iso_helm(const BlockStatic& b, const Tile& tl, const double* in, double* out, double lambda,
                         double* smem) {
  OpArgs a;
  a.tab = b.tab;
  a.itab = b.itab;
  a.fac = nullptr;
  a.dxi = nullptr;
  a.n_elem = b.n_elem;
  a.in = in;
  a.out = out;
  a.in_cs = 0;
  a.out_cs = 0;
  a.lambda = lambda;
  a.E = 0;
  a.pad_ = 0;
  const Tile_<SH, P> T = make_tile_h<SH, P, double>(smem, b.tab);
  load_tables_helm<SH, P>(a, T);
  GeoRegs<PPT> g;
  iso_geometry<SH, P, PPT>(b.xco, b.wref, tl.e0, tl.ne, T, g);
  helm_tile<SH, P, OP, PPT>(a, tl.e0, tl.ne, T, g, false, []() {});
}

// Laplacian (OP = OPK_LAP) or Helmholtz (OPK_HELM) action of iso-parametric
// blocks of order P, one tile per work-group; in/out are whole-mesh buffers,
// or one block's buffers when blk_only >= 0.
template <int P, int OP, int PPT>
__global__ void __launch_bounds__(512) k_helm_mixed_iso(const BlockStatic* __restrict__ blocks,
                                                        const Tile* __restrict__ tiles, int ntiles, const double* in,
                                                        double* out, double lambda, int blk_only, int E_only) {
  extern __shared__ double smem[];
  Tile tl;
  if (!iso_tile(blocks, tiles, ntiles, blk_only, E_only, tl)) return;
  const BlockStatic b = blocks[tl.blk];
  const double* bin = in + (blk_only >= 0 ? 0 : b.coeff_off);
  double* bout = out + (blk_only >= 0 ? 0 : b.coeff_off);
  switch (b.shape) {
    case HEX: iso_helm<HEX, P, OP, PPT>(b, tl, bin, bout, lambda, smem); break;
    case PRISM: iso_helm<PRISM, P, OP, PPT>(b, tl, bin, bout, lambda, smem); break;
    case PYR: iso_helm<PYR, P, OP, PPT>(b, tl, bin, bout, lambda, smem); break;
    default: iso_helm<TET, P, OP, PPT>(b, tl, bin, bout, lambda, smem); break;
  }
}

template <int SH, int P, int PPT>
__device__ __forceinline__ void iso_check_tile(const BlockStatic& b, const Tile& tl, double* smem, int* status) {
  OpArgs a;
  a.tab = b.tab;
  a.itab = b.itab;
  const Tile_<SH, P> T = make_tile_h<SH, P, double>(smem, b.tab);
  load_tables_helm<SH, P>(a, T);
  GeoRegs<PPT> g;
  if (!iso_geometry<SH, P, PPT>(b.xco, b.wref, tl.e0, tl.ne, T, g)) atomicOr(status, 1);
}

// The geometry of block blk's tiles only: status set to 1 when some point has
// a non-positive determinant or a non-finite factor.
template <int P, int PPT>
__global__ void __launch_bounds__(512) k_iso_check(const BlockStatic* __restrict__ blocks, int blk, int E,
                                                   int* __restrict__ status) {
  extern __shared__ double smem[];
  Tile tl;
  if (!iso_tile(blocks, nullptr, 0, blk, E, tl)) return;
  const BlockStatic b = blocks[blk];
  switch (b.shape) {
    case HEX: iso_check_tile<HEX, P, PPT>(b, tl, smem, status); break;
    case PRISM: iso_check_tile<PRISM, P, PPT>(b, tl, smem, status); break;
    case PYR: iso_check_tile<PYR, P, PPT>(b, tl, smem, status); break;
    default: iso_check_tile<TET, P, PPT>(b, tl, smem, status); break;
  }
}

}  // namespace shp
