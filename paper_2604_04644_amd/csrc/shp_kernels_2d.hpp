// HIP kernels of libshp for gfx950: the elemental operators of quadrilaterals
// and triangles (Sec. 2.2, the two-dimensional formulation; Sec. 2.3, the
// triangle as a collapsed square).
//
// Modes (p, q), q fastest: quadrilateral A_p(eta1) A_q(eta2), 0 <= p, q <= P;
// triangle A_p(eta1) C_{p,q}(eta2), p + q <= P, whose collapsed-vertex mode
// (0,1) is v1(eta2) = C_{0,1}(eta2) on both the p = 0 and p = 1 columns
// (A_0 + A_1 = 1).  Points (i, j) at i*Q + j, eta2 fastest.
//
// A work-group holds E elements in LDS: the modes, and three point buffers U,
// G0, G1 of Q^2 values each.  Stages (each a set of independent 1D line tasks
// strided over the threads, separated by barriers):
//   bwd_q : modes -> F[p][j]     contract q with the eta2 table of column p
//   bwd_p : F     -> U[i][j]     contract p with A_p(z1_i)
//   grad  : U     -> G0, G1      collocation derivatives (eq. dphitodh)
//   metric: (G0, G1) <- g (G0, G1), U <- lambda jw U
//   the transposed stages back to modes (B^T, D^T), as in eq. helm1.
#pragma once
#include "shp_kernels.hpp"

namespace shp {

// Reference tables of one 2D (shape, P), Q = P + 2, in one FP64 array:
//   z[2][Q], w[2][Q], A1[n][Q], dA1[n][Q], B2[nb2][Q], dB2[nb2][Q], D[2][Q][Q]
// B2 holds A_q (quadrilateral, nb2 = n) or C_{p,q} at row fam_index(P, p, q)
// (triangle, nb2 = (P+1)(P+2)/2).
struct TabLayout2D {
  int Q, n, nb2, z, w, A1, dA1, B2, dB2, D, total;
};

constexpr TabLayout2D tab_layout2d(int sh, int P) {
  TabLayout2D t{};
  t.Q = P + 2;
  t.n = P + 1;
  t.nb2 = (sh == TRI) ? (P + 1) * (P + 2) / 2 : P + 1;
  int o = 0;
  t.z = o;   o += 2 * t.Q;
  t.w = o;   o += 2 * t.Q;
  t.A1 = o;  o += t.n * t.Q;
  t.dA1 = o; o += t.n * t.Q;
  t.B2 = o;  o += t.nb2 * t.Q;
  t.dB2 = o; o += t.nb2 * t.Q;
  t.D = o;   o += 2 * t.Q * t.Q;
  t.total = o;
  return t;
}

// 2D geometric factors per point: (jw, g00, g01, g11) and d eta_d/d x_i at d*2 + i
constexpr int NFAC2 = 4;
constexpr int NDXI2 = 4;

template <int SH, int P>
struct Dims2 {
  static constexpr int n = P + 1;
  static constexpr int Q = P + 2;
  static constexpr int Q2 = Q * Q;
  static constexpr int NP = num_modes2(SH, P);
  static constexpr TabLayout2D L = tab_layout2d(SH, P);
  // per element in LDS: modes (padded to even) and three point buffers
  static constexpr int MP = (NP + 1) / 2 * 2;
  static constexpr int PER = MP + 3 * Q2;
};

// first mode of column p and its number of q values
template <int SH, int P>
__device__ __forceinline__ int col2_base(int p) {
  return SH == TRI ? p * (P + 1) - p * (p - 1) / 2 : p * (P + 1);
}
template <int SH, int P>
__device__ __forceinline__ int col2_len(int p) {
  return SH == TRI ? P + 1 - p : P + 1;
}

template <int SH, int P>
struct Tile2 {
  using D = Dims2<SH, P>;
  double* tab;  // tables in LDS
  double* el;
  __device__ double* X(int e) const { return el + e * D::PER; }
  __device__ double* U(int e) const { return el + e * D::PER + D::MP; }
  __device__ double* G(int e, int d) const { return el + e * D::PER + D::MP + (d + 1) * D::Q2; }
};

template <int SH, int P>
__device__ Tile2<SH, P> make_tile2(double* smem) {
  Tile2<SH, P> T;
  T.tab = smem;
  T.el = smem + (Dims2<SH, P>::L.total + 1) / 2 * 2;
  return T;
}

template <int SH, int P>
constexpr size_t lds_bytes2(int E) {
  return sizeof(double) * ((size_t)(Dims2<SH, P>::L.total + 1) / 2 * 2 + (size_t)E * Dims2<SH, P>::PER);
}

// modes of column p (buffer X) -> F[p][j] (buffer G0, row p of Q values)
template <int SH, int P, bool DER>
__device__ void bwd2_q(const Tile2<SH, P>& T, int ne) {
  using D = Dims2<SH, P>;
  constexpr int Q = D::Q, n = D::n;
  const double* B2 = T.tab + (DER ? D::L.dB2 : D::L.B2);
  for (int t = threadIdx.x; t < ne * n; t += blockDim.x) {
    const int e = t / n, p = t - e * n;
    const double* x = T.X(e) + col2_base<SH, P>(p);
    const int nq = col2_len<SH, P>(p);
    const int row0 = SH == TRI ? fam_index(P, p, 0) : 0;
    double acc[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) acc[j] = 0.0;
#pragma unroll
    for (int q = 0; q < n; ++q) {
      if (q < nq) {
        const double xv = x[q];
        const double* b = B2 + (row0 + q) * Q;
#pragma unroll
        for (int j = 0; j < Q; ++j) acc[j] = fma(b[j], xv, acc[j]);
      }
    }
    if (SH == TRI && p == 1) {
      // the collapsed-vertex mode (0,1): v1(eta2) = C_{0,1} on the p = 1 column too
      const double xv = T.X(e)[1];
      const double* b = B2 + fam_index(P, 0, 1) * Q;
#pragma unroll
      for (int j = 0; j < Q; ++j) acc[j] = fma(b[j], xv, acc[j]);
    }
    double* F = T.G(e, 0) + p * Q;
#pragma unroll
    for (int j = 0; j < Q; ++j) F[j] = acc[j];
  }
}

// F[p][j] (G0) -> U[i][j] with A_p (or dA_p) in eta1
template <int SH, int P, bool DER>
__device__ void bwd2_p(const Tile2<SH, P>& T, int ne) {
  using D = Dims2<SH, P>;
  constexpr int Q = D::Q, n = D::n;
  const double* A1 = T.tab + (DER ? D::L.dA1 : D::L.A1);
  for (int t = threadIdx.x; t < ne * Q; t += blockDim.x) {
    const int e = t / Q, j = t - e * Q;
    const double* F = T.G(e, 0) + j;
    double f[n];
#pragma unroll
    for (int p = 0; p < n; ++p) f[p] = F[p * Q];
    double* u = T.U(e) + j;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      double s = 0.0;
#pragma unroll
      for (int p = 0; p < n; ++p) s = fma(A1[p * Q + i], f[p], s);
      u[i * Q] = s;
    }
  }
}

// point values s[i][j] (U) -> Fp[p][j] = sum_i A_p(z1_i) s[i][j] into G1
template <int SH, int P>
__device__ void ipr2_p(const Tile2<SH, P>& T, int ne) {
  using D = Dims2<SH, P>;
  constexpr int Q = D::Q, n = D::n;
  const double* A1 = T.tab + D::L.A1;
  for (int t = threadIdx.x; t < ne * Q; t += blockDim.x) {
    const int e = t / Q, j = t - e * Q;
    const double* sp = T.U(e) + j;
    double v[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) v[i] = sp[i * Q];
    double out[n];
#pragma unroll
    for (int p = 0; p < n; ++p) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < Q; ++i) s = fma(A1[p * Q + i], v[i], s);
      out[p] = s;
    }
    double* F = T.G(e, 1) + j;
#pragma unroll
    for (int p = 0; p < n; ++p) F[p * Q] = out[p];
  }
}

// Fp[p][j] (G1) -> modes y[p,q] = sum_j C_{p,q}(z2_j) Fp[p][j] into buffer X
template <int SH, int P>
__device__ void ipr2_q(const Tile2<SH, P>& T, int ne) {
  using D = Dims2<SH, P>;
  constexpr int Q = D::Q, n = D::n;
  const double* B2 = T.tab + D::L.B2;
  for (int t = threadIdx.x; t < ne * n; t += blockDim.x) {
    const int e = t / n, p = t - e * n;
    const double* F = T.G(e, 1) + p * Q;
    double f[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) f[j] = F[j];
    const int nq = col2_len<SH, P>(p);
    const int row0 = SH == TRI ? fam_index(P, p, 0) : 0;
    double* y = T.X(e) + col2_base<SH, P>(p);
#pragma unroll
    for (int q = 0; q < n; ++q) {
      if (q < nq) {
        const double* b = B2 + (row0 + q) * Q;
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < Q; ++j) s = fma(b[j], f[j], s);
        y[q] = s;
      }
    }
  }
}

// the adjoint of the collapsed-vertex term: y[(0,1)] += sum_j v1(z2_j) Fp[1][j]
// (after ipr2_q has written every mode; one task per element)
template <int SH, int P>
__device__ void ipr2_vertex(const Tile2<SH, P>& T, int ne) {
  using D = Dims2<SH, P>;
  constexpr int Q = D::Q;
  if (SH != TRI) return;
  const double* v1 = T.tab + D::L.B2 + fam_index(P, 0, 1) * Q;
  for (int e = threadIdx.x; e < ne; e += blockDim.x) {
    const double* F = T.G(e, 1) + 1 * Q;
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < Q; ++j) s = fma(v1[j], F[j], s);
    T.X(e)[1] += s;
  }
}

// collocation derivative along eta_{DIR+1}: G_DIR = D_DIR U (TRANS: G_DIR <- D^T G_DIR)
template <int SH, int P, int DIR, bool TRANS>
__device__ void grad2(const Tile2<SH, P>& T, int ne) {
  using D = Dims2<SH, P>;
  constexpr int Q = D::Q;
  constexpr int stride = DIR == 0 ? Q : 1;
  const double* Dm = T.tab + D::L.D + DIR * Q * Q;
  for (int t = threadIdx.x; t < ne * Q; t += blockDim.x) {
    const int e = t / Q, a = t - e * Q;
    const int base = DIR == 0 ? a : a * Q;
    const double* src = (TRANS ? T.G(e, DIR) : T.U(e)) + base;
    double v[Q];
#pragma unroll
    for (int l = 0; l < Q; ++l) v[l] = src[l * stride];
    double* g = T.G(e, DIR) + base;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < Q; ++l) s = fma(TRANS ? Dm[l * Q + i] : Dm[i * Q + l], v[l], s);
      g[i * stride] = s;
    }
  }
}

// One tile of operator OP (OPK_BWD .. OPK_HELM) for elements e0 .. e0+ne-1 of
// a 2D block: in/out in the block's layouts (vector fields [2][n][Q^2] with
// component strides in_cs / out_cs).
template <int SH, int P, int OP>
__device__ void tile2d(const OpArgs& a, long long e0, int ne, const Tile2<SH, P>& T) {
  using D = Dims2<SH, P>;
  constexpr int Q2 = D::Q2, NP = D::NP;
  for (int t = threadIdx.x; t < D::L.total; t += blockDim.x) T.tab[t] = a.tab[t];
  constexpr bool in_modes = (OP == OPK_BWD || OP == OPK_MASS || OP == OPK_LAP || OP == OPK_HELM);
  if (in_modes) {
    const double* src = a.in + e0 * NP;
    for (int t = threadIdx.x; t < ne * NP; t += blockDim.x) {
      const int e = t / NP, m = t - e * NP;
      T.X(e)[m] = src[t];
    }
  } else if (OP == OPK_IPRD) {
    // sum_i d eta_d / d x_i jw f_i into G_d, d = 0, 1
    for (int t = threadIdx.x; t < ne * Q2; t += blockDim.x) {
      const int e = t / Q2, pt = t - e * Q2;
      const long long ge = e0 + e;
      const double* dx = a.dxi + ge * (NDXI2 * Q2) + pt;
      const double jw = a.fac[ge * (NFAC2 * Q2) + pt];
      const double f0 = a.in[ge * Q2 + pt], f1 = a.in[a.in_cs + ge * Q2 + pt];
      T.G(e, 0)[pt] = jw * (dx[0 * Q2] * f0 + dx[1 * Q2] * f1);
      T.G(e, 1)[pt] = jw * (dx[2 * Q2] * f0 + dx[3 * Q2] * f1);
    }
  } else {
    // point values into U (IProduct weighs them by jw; PhysDeriv takes them as they are)
    for (int t = threadIdx.x; t < ne * Q2; t += blockDim.x) {
      const int e = t / Q2, pt = t - e * Q2;
      const long long ge = e0 + e;
      const double v = a.in[ge * Q2 + pt];
      T.U(e)[pt] = (OP == OPK_IPR) ? a.fac[ge * (NFAC2 * Q2) + pt] * v : v;
    }
  }
  __syncthreads();
  if (in_modes) {
    bwd2_q<SH, P, false>(T, ne);
    __syncthreads();
    bwd2_p<SH, P, false>(T, ne);
    __syncthreads();
  }
  if (OP == OPK_BWD) {
    for (int t = threadIdx.x; t < ne * Q2; t += blockDim.x) {
      const int e = t / Q2, pt = t - e * Q2;
      a.out[(e0 + e) * Q2 + pt] = T.U(e)[pt];
    }
    return;
  }
  if (OP == OPK_DERIV || OP == OPK_LAP || OP == OPK_HELM) {
    grad2<SH, P, 0, false>(T, ne);
    grad2<SH, P, 1, false>(T, ne);
    __syncthreads();
  }
  if (OP == OPK_DERIV) {
    // d u / d x_i = sum_d (d eta_d / d x_i) (D_d u)
    for (int t = threadIdx.x; t < ne * Q2; t += blockDim.x) {
      const int e = t / Q2, pt = t - e * Q2;
      const long long ge = e0 + e;
      const double* dx = a.dxi + ge * (NDXI2 * Q2) + pt;
      const double d0 = T.G(e, 0)[pt], d1 = T.G(e, 1)[pt];
      a.out[ge * Q2 + pt] = dx[0 * Q2] * d0 + dx[2 * Q2] * d1;
      a.out[a.out_cs + ge * Q2 + pt] = dx[1 * Q2] * d0 + dx[3 * Q2] * d1;
    }
    return;
  }
  if (OP == OPK_MASS || OP == OPK_LAP || OP == OPK_HELM) {
    for (int t = threadIdx.x; t < ne * Q2; t += blockDim.x) {
      const int e = t / Q2, pt = t - e * Q2;
      const double* f = a.fac + (e0 + e) * (NFAC2 * Q2) + pt;
      if (OP == OPK_MASS) {
        T.U(e)[pt] *= f[0];
      } else {
        const double d0 = T.G(e, 0)[pt], d1 = T.G(e, 1)[pt];
        T.G(e, 0)[pt] = f[1 * Q2] * d0 + f[2 * Q2] * d1;
        T.G(e, 1)[pt] = f[2 * Q2] * d0 + f[3 * Q2] * d1;
        if (OP == OPK_HELM) T.U(e)[pt] = a.lambda * f[0] * T.U(e)[pt];
      }
    }
    __syncthreads();
  }
  if (OP == OPK_LAP || OP == OPK_HELM || OP == OPK_IPRD) {
    grad2<SH, P, 0, true>(T, ne);
    grad2<SH, P, 1, true>(T, ne);
    __syncthreads();
    // sum of the point buffers into U: D_0^T v0 + D_1^T v1 (+ lambda jw u)
    for (int t = threadIdx.x; t < ne * Q2; t += blockDim.x) {
      const int e = t / Q2, pt = t - e * Q2;
      double s = (OP == OPK_HELM) ? T.U(e)[pt] : 0.0;
      s += T.G(e, 0)[pt];
      s += T.G(e, 1)[pt];
      T.U(e)[pt] = s;
    }
    __syncthreads();
  }
  // points (U) -> modes: p^T into G1, q^T into X
  ipr2_p<SH, P>(T, ne);
  __syncthreads();
  ipr2_q<SH, P>(T, ne);
  __syncthreads();
  ipr2_vertex<SH, P>(T, ne);
  __syncthreads();
  double* dst = a.out + e0 * NP;
  for (int t = threadIdx.x; t < ne * NP; t += blockDim.x) {
    const int e = t / NP, m = t - e * NP;
    dst[t] = T.X(e)[m];
  }
}

// one tile of E elements per work-group, one block
template <int SH, int P, int OP>
__global__ void __launch_bounds__(512) k_block2d(OpArgs a) {
  extern __shared__ double smem[];
  const long long e0 = (long long)blockIdx.x * a.E;
  const long long rem = a.n_elem - e0;
  const int ne = rem < a.E ? (int)rem : a.E;
  if (ne <= 0) return;
  tile2d<SH, P, OP>(a, e0, ne, make_tile2<SH, P>(smem));
}

// whole-mesh launch over 2D blocks of one P, tiles from a list
template <int P, int OP>
__global__ void __launch_bounds__(512) k_mixed2d(const BlockStatic* __restrict__ blocks, const Tile* __restrict__ tiles,
                                                 int ntiles, const double* in, double* out, long long in_cs,
                                                 long long out_cs, double lambda) {
  extern __shared__ double smem[];
  if ((int)blockIdx.x >= ntiles) return;
  const Tile tl = tiles[blockIdx.x];
  const BlockStatic b = blocks[tl.blk];
  constexpr bool in_modes = (OP == OPK_BWD || OP == OPK_MASS || OP == OPK_LAP || OP == OPK_HELM);
  constexpr bool out_modes = !(OP == OPK_BWD || OP == OPK_DERIV);
  OpArgs a;
  a.tab = b.tab;
  a.itab = b.itab;
  a.fac = b.fac;
  a.dxi = b.dxi;
  a.n_elem = b.n_elem;
  a.in = in + (in_modes ? b.coeff_off : b.phys_off);
  a.out = out + (out_modes ? b.coeff_off : b.phys_off);
  a.in_cs = in_cs;
  a.out_cs = out_cs;
  a.lambda = lambda;
  a.E = 0;
  a.pad_ = 0;
  if (b.shape == QUAD)
    tile2d<QUAD, P, OP>(a, tl.e0, tl.ne, make_tile2<QUAD, P>(smem));
  else
    tile2d<TRI, P, OP>(a, tl.e0, tl.ne, make_tile2<TRI, P>(smem));
}

// ---------------------------------------------------------------------------
// Collocated Laplacian / Helmholtz tile (eq. helm1 in two dimensions)
// ---------------------------------------------------------------------------
// The 2D counterpart of the 3D helm_tile: the tile's 4 factors per point are
// issued into registers (PPT points per thread) right after its modes reach
// LDS, so their HBM latency overlaps the backward transform and gradients;
// tables read at wave-uniform indices (A_p, the collocation derivatives, the
// quadrilateral's A_q) are scalar loads; only the triangle's eta2 table,
// whose row depends on the lane's column p, sits in LDS (the compact head).
// Stages, 7 barriers:
//   q:   modes -> F[p][j]                    (G0 rows)
//   p:   F -> U[i][j], and G0 = D_1 U from the same column in registers
//   j:   G1 = D_2 U                          (rows of U)
//   metric (registers): (G0, G1) <- g (G0, G1), U <- lambda jw U
//   jT:  G1 <- D_2^T G1                      (rows)
//   pT:  per column j, v = U + G1 + D_1^T G0, then A_p^T v -> G1 rows
//   qT:  G1 rows -> modes, with the triangle's collapsed-vertex adjoint

template <int PPT>
struct GeoRegs2 {
  double v[PPT][NFAC2];
};

// compact LDS head (doubles): the triangle's eta2 table only
template <int SH, int P>
constexpr int head2h() {
  return SH == TRI ? Dims2<SH, P>::L.nb2 * Dims2<SH, P>::Q : 0;
}

template <int SH, int P>
constexpr size_t lds_bytes2h(int E) {
  return sizeof(double) * ((size_t)head2h<SH, P>() + (size_t)E * Dims2<SH, P>::PER);
}

template <int SH, int P>
__device__ Tile2<SH, P> make_tile2h(double* smem) {
  Tile2<SH, P> T;
  T.tab = smem;  // the triangle's eta2 table (row fam_index(P, p, q))
  T.el = smem + head2h<SH, P>();
  return T;
}

template <int P, int PPT>
__device__ __forceinline__ void prefetch_geo2(const double* __restrict__ fac, long long e0, int ne, GeoRegs2<PPT>& g) {
  constexpr int Q2 = (P + 2) * (P + 2);
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(fac + e0 * (long long)(NFAC2 * Q2)), (short)0, ne * (NFAC2 * Q2 * 8), 0x00020000);
  const int n = ne * Q2;
#pragma unroll
  for (int it = 0; it < PPT; ++it) {
    const int t = threadIdx.x + it * blockDim.x;
    const int e = t / Q2, pt = t - e * Q2;
    // out of range past the tile: the load returns zero without a memory access
    const int off = t < n ? (e * (NFAC2 * Q2) + pt) * 8 : ne * (NFAC2 * Q2 * 8);
#pragma unroll
    for (int c = 0; c < NFAC2; ++c)
      g.v[it][c] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, off + c * Q2 * 8, 0, 2));
  }
}

// eta2 row of mode (p, q): wave-uniform table for the quadrilateral, the
// lane's own LDS row for the triangle
template <int SH, int P>
struct Eta2Rows {
  ctab_t ct;
  const double* lds;
};

template <int SH, int P, int OP, int PPT>
__device__ void helm2d_tile(const OpArgs& a, long long e0, int ne, const Tile2<SH, P>& T) {
  using D = Dims2<SH, P>;
  constexpr int Q = D::Q, Q2 = D::Q2, n = D::n, NP = D::NP;
  const ctab_t ct = as_const(a.tab);
  if (SH == TRI)
    for (int t = threadIdx.x; t < D::L.nb2 * Q; t += blockDim.x) T.tab[t] = a.tab[D::L.B2 + t];
  {
    const double* src = a.in + e0 * NP;
    for (int t = threadIdx.x; t < ne * NP; t += blockDim.x) {
      const int e = t / NP, m = t - e * NP;
      T.X(e)[m] = src[t];
    }
  }
  GeoRegs2<PPT> g;
  prefetch_geo2<P, PPT>(a.fac, e0, ne, g);
  __syncthreads();
  // q: modes of column p -> F[p][j] in G0
  for (int t = threadIdx.x; t < ne * n; t += blockDim.x) {
    const int e = t / n, p = t - e * n;
    const double* x = T.X(e) + col2_base<SH, P>(p);
    const int nq = col2_len<SH, P>(p);
    double acc[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) acc[j] = 0.0;
#pragma unroll
    for (int q = 0; q < n; ++q) {
      if (q < nq) {
        const double xv = x[q];
        if (SH == QUAD) {
          const ctab_t b = launder(ct) + D::L.B2 + q * Q;
#pragma unroll
          for (int j = 0; j < Q; ++j) acc[j] = fma(b[j], xv, acc[j]);
        } else {
          const double* b = T.tab + fam_index(P, p, q) * Q;
#pragma unroll
          for (int j = 0; j < Q; ++j) acc[j] = fma(b[j], xv, acc[j]);
        }
      }
    }
    if (SH == TRI && p == 1) {
      // the collapsed-vertex mode (0,1): v1(eta2) = C_{0,1} on the p = 1 column too
      const double xv = T.X(e)[1];
      const ctab_t b = launder(ct) + D::L.B2 + fam_index(P, 0, 1) * Q;
#pragma unroll
      for (int j = 0; j < Q; ++j) acc[j] = fma(b[j], xv, acc[j]);
    }
    double* F = T.G(e, 0) + p * Q;
#pragma unroll
    for (int j = 0; j < Q; ++j) F[j] = acc[j];
  }
  __syncthreads();
  // p: column j of F -> U[.][j], and D_1 of that column into G0[.][j]
  for (int t = threadIdx.x; t < ne * Q; t += blockDim.x) {
    const int e = t / Q, j = t - e * Q;
    double* G0 = T.G(e, 0) + j;
    double f[n];
#pragma unroll
    for (int p = 0; p < n; ++p) f[p] = G0[p * Q];
    double u[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const ctab_t A1 = launder(ct) + D::L.A1;
      double s = 0.0;
#pragma unroll
      for (int p = 0; p < n; ++p) s = fma(A1[p * Q + i], f[p], s);
      u[i] = s;
    }
    double* U = T.U(e) + j;
#pragma unroll
    for (int i = 0; i < Q; ++i) U[i * Q] = u[i];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const ctab_t Dm = launder(ct) + D::L.D;
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < Q; ++l) s = fma(Dm[i * Q + l], u[l], s);
      G0[i * Q] = s;
    }
  }
  __syncthreads();
  // j: G1 = D_2 U along the rows
  for (int t = threadIdx.x; t < ne * Q; t += blockDim.x) {
    const int e = t / Q, i = t - e * Q;
    const double* U = T.U(e) + i * Q;
    double v[Q];
#pragma unroll
    for (int l = 0; l < Q; ++l) v[l] = U[l];
    double* G1 = T.G(e, 1) + i * Q;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const ctab_t Dm = launder(ct) + D::L.D + Q * Q;
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < Q; ++l) s = fma(Dm[j * Q + l], v[l], s);
      G1[j] = s;
    }
  }
  __syncthreads();
  // metric from the registers
  const double lam = (OP == OPK_HELM) ? a.lambda : 0.0;
#pragma unroll
  for (int it = 0; it < PPT; ++it) {
    const int t = threadIdx.x + it * blockDim.x;
    if (t < ne * Q2) {
      const int e = t / Q2, pt = t - e * Q2;
      const double* f = g.v[it];
      double* p0 = T.G(e, 0) + pt;
      double* p1 = T.G(e, 1) + pt;
      const double d0 = *p0, d1 = *p1;
      *p0 = f[1] * d0 + f[2] * d1;
      *p1 = f[2] * d0 + f[3] * d1;
      if (OP == OPK_HELM) {
        double* u = T.U(e) + pt;
        *u = lam * f[0] * (*u);
      }
    }
  }
  __syncthreads();
  // jT: G1 <- D_2^T G1 along the rows
  for (int t = threadIdx.x; t < ne * Q; t += blockDim.x) {
    const int e = t / Q, i = t - e * Q;
    double* G1 = T.G(e, 1) + i * Q;
    double w[Q];
#pragma unroll
    for (int l = 0; l < Q; ++l) w[l] = G1[l];
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const ctab_t Dm = launder(ct) + D::L.D + Q * Q;
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < Q; ++l) s = fma(Dm[l * Q + j], w[l], s);
      G1[j] = s;
    }
  }
  __syncthreads();
  // pT: per column j, v = U + G1 + D_1^T G0, then F[p][j] = sum_i A_p(z_i) v_i into G1
  for (int t = threadIdx.x; t < ne * Q; t += blockDim.x) {
    const int e = t / Q, j = t - e * Q;
    const double* G0 = T.G(e, 0) + j;
    double* G1 = T.G(e, 1) + j;
    const double* U = T.U(e) + j;
    double w[Q], v[Q];
#pragma unroll
    for (int l = 0; l < Q; ++l) w[l] = G0[l * Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const ctab_t Dm = launder(ct) + D::L.D;
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < Q; ++l) s = fma(Dm[l * Q + i], w[l], s);
      v[i] = (OP == OPK_HELM ? U[i * Q] : 0.0) + G1[i * Q] + s;
    }
#pragma unroll
    for (int p = 0; p < n; ++p) {
      const ctab_t A1 = launder(ct) + D::L.A1;
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < Q; ++i) s = fma(A1[p * Q + i], v[i], s);
      G1[p * Q] = s;
    }
  }
  __syncthreads();
  // qT: G1 rows -> modes in X (the triangle's column 0 also takes the adjoint
  // of the collapsed-vertex term from row 1)
  for (int t = threadIdx.x; t < ne * n; t += blockDim.x) {
    const int e = t / n, p = t - e * n;
    const double* F = T.G(e, 1) + p * Q;
    double f[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) f[j] = F[j];
    const int nq = col2_len<SH, P>(p);
    double* y = T.X(e) + col2_base<SH, P>(p);
#pragma unroll
    for (int q = 0; q < n; ++q) {
      if (q < nq) {
        double s = 0.0;
        if (SH == QUAD) {
          const ctab_t b = launder(ct) + D::L.B2 + q * Q;
#pragma unroll
          for (int j = 0; j < Q; ++j) s = fma(b[j], f[j], s);
        } else {
          const double* b = T.tab + fam_index(P, p, q) * Q;
#pragma unroll
          for (int j = 0; j < Q; ++j) s = fma(b[j], f[j], s);
        }
        y[q] = s;
      }
    }
    if (SH == TRI && p == 0) {
      const double* F1 = T.G(e, 1) + 1 * Q;
      const ctab_t v1 = launder(ct) + D::L.B2 + fam_index(P, 0, 1) * Q;
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < Q; ++j) s = fma(v1[j], F1[j], s);
      y[1] += s;
    }
  }
  __syncthreads();
  double* dst = a.out + e0 * NP;
  for (int t = threadIdx.x; t < ne * NP; t += blockDim.x) {
    const int e = t / NP, m = t - e * NP;
    dst[t] = T.X(e)[m];
  }
}

template <int SH, int P, int OP, int PPT>
__global__ void __launch_bounds__(512) k_helm_block2d(OpArgs a) {
  extern __shared__ double smem[];
  const long long e0 = (long long)blockIdx.x * a.E;
  const long long rem = a.n_elem - e0;
  const int ne = rem < a.E ? (int)rem : a.E;
  if (ne <= 0) return;
  helm2d_tile<SH, P, OP, PPT>(a, e0, ne, make_tile2h<SH, P>(smem));
}

template <int P, int OP, int PPT>
__global__ void __launch_bounds__(512) k_helm_mixed2d(const BlockStatic* __restrict__ blocks,
                                                      const Tile* __restrict__ tiles, int ntiles, const double* in,
                                                      double* out, double lambda) {
  extern __shared__ double smem[];
  if ((int)blockIdx.x >= ntiles) return;
  const Tile tl = tiles[blockIdx.x];
  const BlockStatic b = blocks[tl.blk];
  OpArgs a;
  a.tab = b.tab;
  a.itab = b.itab;
  a.fac = b.fac;
  a.dxi = b.dxi;
  a.n_elem = b.n_elem;
  a.in = in + b.coeff_off;
  a.out = out + b.coeff_off;
  a.in_cs = 0;
  a.out_cs = 0;
  a.lambda = lambda;
  a.E = 0;
  a.pad_ = 0;
  if (b.shape == QUAD)
    helm2d_tile<QUAD, P, OP, PPT>(a, tl.e0, tl.ne, make_tile2h<QUAD, P>(smem));
  else
    helm2d_tile<TRI, P, OP, PPT>(a, tl.e0, tl.ne, make_tile2h<TRI, P>(smem));
}

// 2D geometric factors from d x_i/d xi_j (curved [n][4][Q^2], affine [n][4])
template <int SH, int P>
__global__ void __launch_bounds__(256) k_geometry2d(const double* __restrict__ tab, const double* __restrict__ jac,
                                                    double* __restrict__ fac, double* __restrict__ dxi, long long n_elem,
                                                    int affine, int* __restrict__ status) {
  using D = Dims2<SH, P>;
  constexpr int Q = D::Q, Q2 = D::Q2;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_elem * Q2) return;
  const long long e = t / Q2;
  const int pt = (int)(t - e * Q2);
  const int i = pt / Q, j = pt - i * Q;
  const double e1 = tab[D::L.z + i], e2 = tab[D::L.z + Q + j];
  const double wq = tab[D::L.w + i] * tab[D::L.w + Q + j];
  double J[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) J[c] = affine ? jac[e * 4 + c] : jac[(e * 4 + c) * Q2 + pt];
  const double det = J[0] * J[3] - J[1] * J[2];
  bool bad = !(det > 0.0) || !isfinite(det);
  const double id = 1.0 / det;
  // d xi_a / d x_i at a*2 + i
  const double X[4] = {J[3] * id, -J[1] * id, -J[2] * id, J[0] * id};
  // d eta / d xi of the collapse (rows eta_d, columns xi_a): the triangle's
  // eta1 = 2 (1 + xi1)/(1 - xi2) - 1 gives 2/(1 - eta2) and (1 + eta1)/(1 - eta2)
  double Gc[4] = {1.0, 0.0, 0.0, 1.0};
  double scale = 1.0;
  if (SH == TRI) {
    Gc[0] = 2.0 / (1.0 - e2);
    Gc[1] = (1.0 + e1) / (1.0 - e2);
    scale = 0.5;
  }
  double M[4];  // d eta_d / d x_i at d*2 + i
#pragma unroll
  for (int d = 0; d < 2; ++d)
#pragma unroll
    for (int ii = 0; ii < 2; ++ii) M[d * 2 + ii] = Gc[d * 2 + 0] * X[0 * 2 + ii] + Gc[d * 2 + 1] * X[1 * 2 + ii];
  const double jw = wq * scale * det;
  double* f = fac + e * (NFAC2 * Q2) + pt;
  f[0] = jw;
  f[1 * Q2] = jw * (M[0] * M[0] + M[1] * M[1]);
  f[2 * Q2] = jw * (M[0] * M[2] + M[1] * M[3]);
  f[3 * Q2] = jw * (M[2] * M[2] + M[3] * M[3]);
  double* m = dxi + e * (NDXI2 * Q2) + pt;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    m[c * Q2] = M[c];
    bad = bad || !isfinite(M[c]);
  }
  if (bad) atomicOr(status, 1);
}

}  // namespace shp
