// HIP kernels of libshp for gfx950: LDS-staged sum-factorisation over tiles of
// elements, one work-group per tile.
//
// Work decomposition.  A work-group holds E elements in LDS.  Every stage of an
// operator is a set of independent "line" tasks (a 1D contraction producing Q or
// n outputs from one line of its input), strided over the work-group's threads;
// a barrier separates stages.  1D tables (basis functions and collocation
// derivatives at the quadrature points of each direction) sit in LDS.
//
// Stages (Sec. 3.3.2 sum-factorisation; Sec. 2.3 collapsed tensor structure):
//   bwd_r : x (modes)      -> F[col][k]   contract r with C_{kappa,r}(z3_k)
//   bwd_q : F              -> G[p][j][k]  contract q with B2_{p,q}(z2_j)
//   bwd_p : G              -> U[i][j][k]  contract p with A_p(z1_i)
//   ipr_p, ipr_q, ipr_r    the transposed contractions (B^T)
//   grad  : U              -> G0,G1,G2    collocation derivatives D_d (eq. dphitodh)
//   gradT : V_d            -> D_d^T V_d   in place
// The collapsed-vertex modes (functions independent of a collapsed coordinate)
// are split with A_0 + A_1 = 1 into the p = 0 and p = 1 (and q = 0, 1) columns;
// each stage adds the extra terms, and the transposed stages add their adjoints.
//
// The collocated Helmholtz action (Sec. 2.2.1 eq. helm1, Alg. 6) is
//   y = B^T [ sum_d D_d^T ( sum_e g_de D_e u ) + lambda jw u ],  u = B x,
// with g = jw (d eta/d x)(d eta/d x)^T and jw the quadrature weight times |J|.
#pragma once
#include <hip/hip_runtime.h>

#include "shp_internal.hpp"
#include "shp_layout.hpp"

namespace shp {

enum : int {
  OPK_BWD = 0,
  OPK_IPR = 1,
  OPK_DERIV = 2,
  OPK_IPRD = 3,
  OPK_MASS = 4,
  OPK_LAP = 5,
  OPK_HELM = 6,
  OPK_HELM_NC = 7,  // non-collocated Helmholtz (Alg. 5)
  OPK_LAP_NC = 8,   // non-collocated Laplacian
  OPK_MASS_LM = 9,  // local-matrix strategy (FP64 MFMA): mass
  OPK_LAP_LM = 10,  //   Laplacian
  OPK_HELM_LM = 11, //   Helmholtz
  OPK_ADR = 12,     // advection-diffusion-reaction: Helmholtz plus b . grad u tested with the basis
  OPK_HELM_ISO = 13,  // iso-parametric blocks, geometry recomputed in the launch: Helmholtz
  OPK_LAP_ISO = 14,   //   Laplacian
  OPK_BWD_LM = 15,    // local-matrix strategy (FP64 MFMA): backward transform
  OPK_IPR_LM = 16,    //   inner product
  OPK_DERIV_LM = 17,  //   physical derivative
  OPK_IPRD_LM = 18,   //   inner product with the derivatives
  OPK_COUNT = 19
};

// Arguments of one block for one operator call.
struct OpArgs {
  const double* tab;  // reference tables (tab_layout)
  const int* itab;    // column table [NC][ICOL]
  const double* fac;  // [n_elem][NFAC][Q^3]
  const double* dxi;  // [n_elem][NDXI][Q^3]
  const double* in;
  double* out;
  long long n_elem;
  long long in_cs;   // component stride of a vector-field input (points)
  long long out_cs;  // component stride of a vector-field output (points)
  double lambda;
  int E;             // elements per tile
  int pad_;
};

// A tile of a mixed launch: block index, first element, element count.
struct Tile {
  int blk;
  int ne;
  long long e0;
};

template <int SH, int P_>
struct Dims {
  static constexpr int P = P_;
  static constexpr int n = P + 1;
  static constexpr int Q = P + 2;
  static constexpr int Q2 = Q * Q;
  static constexpr int Q3 = Q * Q * Q;
  static constexpr int QP = qpad(Q);
  static constexpr int S3 = Q * Q * QP;  // one padded point buffer in LDS
  static constexpr int NP = num_modes(SH, P);
  static constexpr int NC = num_cols(SH, P);
  static constexpr TabLayout L = tab_layout(SH, P);
  static constexpr int NTAB = L.total;
  static constexpr int NITAB = NC * ICOL + (P + 2) + NC;  // columns, family starts, family order
  // LDS words (doubles) before the per-element region
  static constexpr int HEAD = NTAB + (NITAB + 1) / 2;
  static constexpr int PER_ELEM = 4 * S3;
  __device__ __host__ static constexpr int pidx(int i, int j, int k) { return (i * Q + j) * QP + k; }
};

// Pointers for tables that every lane reads at the same index: loads through
// the constant address space become scalar loads into SGPRs, which feed the
// FP64 FMAs directly and take no LDS bandwidth.  Streamed data is read through
// the global address space.
template <typename R>
using ctab = const __attribute__((address_space(4))) R*;
typedef ctab<double> ctab_t;
typedef const __attribute__((address_space(1))) double* gptr_t;
__device__ __forceinline__ ctab_t as_const(const double* p) { return (ctab_t)(p); }
// Re-derive a table pointer inside a loop so the scalar loads stay in the loop
// body (hoisting every table value out of the loop spills SGPRs).
template <typename R>
__device__ __forceinline__ ctab<R> launder(ctab<R> p) {
  unsigned long long v = (unsigned long long)p;
  asm volatile("" : "+s"(v));
  return (ctab<R>)v;
}
__device__ __forceinline__ gptr_t as_global(const double* p) { return (gptr_t)(p); }

// LDS view of one tile.
// R is the type of the contractions and of the field data in LDS (double, or
// float for the mixed-precision path); geometric factors stay double.
template <int SH, int P, typename R = double>
struct Tile_ {
  using D = Dims<SH, P>;
  R* tab;
  int* itab;
  R* b2;       // the tet's eta2 table B2 in LDS (inside tab, or alone in the compact head)
  ctab<R> ct;  // the same tables in global memory, for lane-uniform reads
  R* el;       // E * per
  int per;     // values per element: 4 buffers (U, G0, G1, G2), 3 fused, 5 non-collocated
  __device__ R* U(int e) const { return el + e * per; }
  __device__ R* G(int e, int d) const { return el + e * per + (d + 1) * D::S3; }
};

__device__ __forceinline__ int tid() { return threadIdx.x; }
__device__ __forceinline__ int nthr() { return blockDim.x; }

template <int SH, int P, typename R>
__device__ void load_tables(const OpArgs& a, const Tile_<SH, P, R>& T) {
  using D = Dims<SH, P>;
  for (int t = tid(); t < D::NTAB; t += nthr()) T.tab[t] = (R)a.tab[t];
  for (int t = tid(); t < D::NITAB; t += nthr()) T.itab[t] = a.itab[t];
}

// The part of the tables the collocated Laplacian / Helmholtz tile reads from
// LDS: the collapsed shapes' column table and the tet's eta2 table B2 (tables
// read at wave-uniform indices go through the constant path).
template <int SH, int P, typename R>
__device__ void load_tables_helm(const OpArgs& a, const Tile_<SH, P, R>& T) {
  using D = Dims<SH, P>;
  if (SH == HEX) return;
  if (SH == TET)
    for (int t = tid(); t < D::L.nb2 * D::Q; t += nthr()) T.b2[t] = (R)a.tab[D::L.B2 + t];
  for (int t = tid(); t < D::NITAB; t += nthr()) T.itab[t] = a.itab[t];
}

// ---------------------------------------------------------------------------
// modes -> points
// ---------------------------------------------------------------------------

// one eta3 family of a collapsed shape's stage r (see bwd_r), lanes ln of a wave
template <int SH, int P, bool DER, typename R, int KAP>
__device__ __forceinline__ void bwd_r_fam(const Tile_<SH, P, R>& T, int ne, int xbuf, int fbuf, int ln) {
  using D = Dims<SH, P>;
  constexpr int Q = D::Q, RL = P + 1 - KAP;
  constexpr int ncol = fam_ncols(SH, P, KAP), c0 = fam_start(SH, P, KAP);
  const int* perm = T.itab + D::NC * ICOL + (P + 2);
  for (int t = ln; t < ne * ncol; t += 64) {
    const ctab<R> C3 = launder(T.ct) + (DER ? D::L.dC3 : D::L.C3);
    const ctab<R> cf = C3 + fam_index(P, KAP, 0) * Q;
    const ctab<R> V1 = C3 + 1 * Q;  // family (0,1): v1 or its derivative 1/2
    const int e = t / ncol;
    const int c = perm[c0 + t - e * ncol];
    const int* ct = T.itab + c * ICOL;
    const int p = ct[0], q = ct[1], off = ct[2];
    const R* x = (xbuf < 0 ? T.U(e) : T.G(e, xbuf));
    R acc[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) acc[k] = 0.0;
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      const R xr = x[off + r];
#pragma unroll
      for (int k = 0; k < Q; ++k) acc[k] = fma(cf[r * Q + k], xr, acc[k]);
    }
    // collapsed-vertex modes: extra eta3 term v1 in columns p = 1 (and q = 1)
    R xe = 0.0;
    bool extra = false;
    if (SH == PRISM) {
      if (p == 1) { xe = x[q * (P + 1) + 1]; extra = true; }
    } else if (SH == PYR) {
      if ((p == 1 && q <= 1) || (p == 0 && q == 1)) { xe = x[1]; extra = true; }
    } else if (SH == TET) {
      if ((p == 1 && q == 0) || (p == 0 && q == 1)) { xe = x[1]; extra = true; }
    }
    if (extra) {
#pragma unroll
      for (int k = 0; k < Q; ++k) acc[k] = fma(V1[k], xe, acc[k]);
    }
    R* f = T.G(e, fbuf) + c * D::QP;
#pragma unroll
    for (int k = 0; k < Q; ++k) f[k] = acc[k];
  }
}

template <int SH, int P, bool DER, typename R, int KAP>
__device__ __forceinline__ void bwd_r_fams(const Tile_<SH, P, R>& T, int ne, int xbuf, int fbuf, int wv, int nw,
                                           int ln) {
  if constexpr (KAP <= P) {
    if (KAP % nw == wv) bwd_r_fam<SH, P, DER, R, KAP>(T, ne, xbuf, fbuf, ln);
    bwd_r_fams<SH, P, DER, R, KAP + 1>(T, ne, xbuf, fbuf, wv, nw, ln);
  }
}

// stage r: X (modes of element e) -> F[c][k] at c*QP + k
template <int SH, int P, bool DER, typename R>
__device__ void bwd_r(const Tile_<SH, P, R>& T, int ne, int xbuf, int fbuf) {
  using D = Dims<SH, P>;
  constexpr int Q = D::Q, n = D::n;
  if (SH == HEX) {
    // every column runs r over 0..P with the same table: lane-uniform reads
    for (int t = tid(); t < ne * D::NC; t += nthr()) {
      const ctab<R> C3 = launder(T.ct) + (DER ? D::L.dC3 : D::L.C3);
      const int e = t / D::NC, c = t - e * D::NC;
      const R* x = (xbuf < 0 ? T.U(e) : T.G(e, xbuf)) + c * n;
      R xr[n];
#pragma unroll
      for (int r = 0; r < n; ++r) xr[r] = x[r];
      R* f = T.G(e, fbuf) + c * D::QP;
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        R a = 0.0;
#pragma unroll
        for (int r = 0; r < n; ++r) a = fma(C3[r * Q + k], xr[r], a);
        f[k] = a;
      }
    }
    return;
  }
  // collapsed shapes: the columns grouped by eta3 family kappa share their
  // table rows and their run length P+1-kappa.  Each wave takes whole
  // families (kappa = wave, wave + waves, ...; a wave-uniform branch per
  // family), so the table rows are read through uniform pointers (scalar
  // loads) and the run length, column count and offsets are constants.
  const int nw = nthr() >> 6, ln = tid() & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid() >> 6);
  bwd_r_fams<SH, P, DER, R, 0>(T, ne, xbuf, fbuf, wv, nw, ln);
}

// stage q: F[c][k] -> G[p][j][k] (p*Q*QP + j*QP + k)
template <int SH, int P, bool DER, typename R>
__device__ void bwd_q(const Tile_<SH, P, R>& T, int ne, int fbuf, int gbuf) {
  using D = Dims<SH, P>;
  constexpr int Q = D::Q, n = D::n, QP = D::QP;
  if (SH != TET) {
    // eta2 functions A_q for every p: lane-uniform table
    for (int t = tid(); t < ne * n * Q; t += nthr()) {
      const ctab<R> B2 = launder(T.ct) + (DER ? D::L.dB2 : D::L.B2);
      const int e = t / (n * Q);
      const int rem = t - e * (n * Q);
      const int p = rem / Q, k = rem - p * Q;
      const R* F = T.G(e, fbuf) + (p * n) * QP + k;
      R fv[n];
#pragma unroll
      for (int q = 0; q < n; ++q) fv[q] = F[q * QP];
      R* G = T.G(e, gbuf) + p * Q * QP + k;
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        R a = 0.0;
#pragma unroll
        for (int q = 0; q < n; ++q) a = fma(B2[q * Q + j], fv[q], a);
        G[j * QP] = a;
      }
    }
    return;
  }
  const R* B2 = DER ? T.tab + D::L.dB2 : T.b2;
  // v1 in eta2 (or its derivative) is the family (0,1) row of the tet's table
  const R* V1 = B2 + 1 * Q;
  for (int t = tid(); t < ne * n * Q; t += nthr()) {
    const int e = t / (n * Q);
    const int rem = t - e * (n * Q);
    const int p = rem / Q, k = rem - p * Q;
    const R* F = T.G(e, fbuf);
    const int nq = nq_of(SH, P, p), cb = col_base(SH, P, p);
    const int bfam = fam_index(P, p, 0);
    R acc[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) acc[j] = 0.0;
#pragma unroll
    for (int q = 0; q < n; ++q) {
      if (q < nq) {
        const R fv = F[(cb + q) * QP + k];
        const R* b = B2 + (bfam + q) * Q;
#pragma unroll
        for (int j = 0; j < Q; ++j) acc[j] = fma(b[j], fv, acc[j]);
      }
    }
    if (p == 1) {
      const R fv = F[1 * QP + k];  // column (0,1)
#pragma unroll
      for (int j = 0; j < Q; ++j) acc[j] = fma(V1[j], fv, acc[j]);
    }
    R* G = T.G(e, gbuf) + p * Q * QP + k;
#pragma unroll
    for (int j = 0; j < Q; ++j) G[j * QP] = acc[j];
  }
}

// stage p: G[p][j][k] -> U[i][j][k] (U buffer index ubuf: -1 = U, else G(ubuf))
template <int SH, int P, bool DER, typename R>
__device__ void bwd_p(const Tile_<SH, P, R>& T, int ne, int gbuf, int ubuf) {
  using D = Dims<SH, P>;
  constexpr int Q = D::Q, n = D::n, QP = D::QP;
  for (int t = tid(); t < ne * Q * Q; t += nthr()) {
    const ctab<R> A1 = launder(T.ct) + (DER ? D::L.dA1 : D::L.A1);
    const int e = t / (Q * Q);
    const int rem = t - e * (Q * Q);
    const int j = rem / Q, k = rem - j * Q;
    const R* G = T.G(e, gbuf) + j * QP + k;
    R g[n];
#pragma unroll
    for (int p = 0; p < n; ++p) g[p] = G[p * Q * QP];
    R* U = (ubuf < 0 ? T.U(e) : T.G(e, ubuf)) + j * QP + k;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      R s = 0.0;
#pragma unroll
      for (int p = 0; p < n; ++p) s = fma(A1[p * Q + i], g[p], s);
      U[i * Q * QP] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// points -> modes (transposed stages)
// ---------------------------------------------------------------------------

// stage p^T: s(i,j,k) = sum over the buffers in mask (bit0: U, bit1..3: G0..G2)
// -> Gp[p][j][k], written in place into buffer dst (-1 = U) at (p, j, k).
template <int SH, int P, bool DER, typename R>
__device__ void ipr_p(const Tile_<SH, P, R>& T, int ne, int mask, int dst) {
  using D = Dims<SH, P>;
  constexpr int Q = D::Q, n = D::n, QP = D::QP;
  for (int t = tid(); t < ne * Q * Q; t += nthr()) {
    const ctab<R> A1 = launder(T.ct) + (DER ? D::L.dA1 : D::L.A1);
    const int e = t / (Q * Q);
    const int rem = t - e * (Q * Q);
    const int j = rem / Q, k = rem - j * Q;
    const int o = j * QP + k;
    R s[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) s[i] = 0.0;
    if (mask & 1) {
      const R* b = T.U(e) + o;
#pragma unroll
      for (int i = 0; i < Q; ++i) s[i] += b[i * Q * QP];
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (mask & (2 << d)) {
        const R* b = T.G(e, d) + o;
#pragma unroll
        for (int i = 0; i < Q; ++i) s[i] += b[i * Q * QP];
      }
    }
    R* G = (dst < 0 ? T.U(e) : T.G(e, dst)) + o;
#pragma unroll
    for (int p = 0; p < n; ++p) {
      R a = 0.0;
#pragma unroll
      for (int i = 0; i < Q; ++i) a = fma(A1[p * Q + i], s[i], a);
      G[p * Q * QP] = a;
    }
  }
}

// stage q^T: Gp[p][j][k] (buffer gbuf) -> F[c][k] (buffer fbuf)
template <int SH, int P, bool DER, typename R>
__device__ void ipr_q(const Tile_<SH, P, R>& T, int ne, int gbuf, int fbuf) {
  using D = Dims<SH, P>;
  constexpr int Q = D::Q, n = D::n, QP = D::QP;
  if (SH != TET) {
    for (int t = tid(); t < ne * n * Q; t += nthr()) {
      const ctab<R> B2 = launder(T.ct) + (DER ? D::L.dB2 : D::L.B2);
      const int e = t / (n * Q);
      const int rem = t - e * (n * Q);
      const int p = rem / Q, k = rem - p * Q;
      const R* G = (gbuf < 0 ? T.U(e) : T.G(e, gbuf)) + p * Q * QP + k;
      R g[Q];
#pragma unroll
      for (int j = 0; j < Q; ++j) g[j] = G[j * QP];
      R* F = T.G(e, fbuf) + (p * n) * QP + k;
#pragma unroll
      for (int q = 0; q < n; ++q) {
        R a = 0.0;
#pragma unroll
        for (int j = 0; j < Q; ++j) a = fma(B2[q * Q + j], g[j], a);
        F[q * QP] = a;
      }
    }
    return;
  }
  const R* B2 = DER ? T.tab + D::L.dB2 : T.b2;
  const R* V1 = B2 + 1 * Q;
  for (int t = tid(); t < ne * n * Q; t += nthr()) {
    const int e = t / (n * Q);
    const int rem = t - e * (n * Q);
    const int p = rem / Q, k = rem - p * Q;
    const R* G = (gbuf < 0 ? T.U(e) : T.G(e, gbuf)) + p * Q * QP + k;
    R g[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) g[j] = G[j * QP];
    const int nq = nq_of(SH, P, p), cb = col_base(SH, P, p);
    const int bfam = fam_index(P, p, 0);
    R* F = T.G(e, fbuf);
#pragma unroll
    for (int q = 0; q < n; ++q) {
      if (q >= nq) continue;
      const R* b = B2 + (bfam + q) * Q;
      R a = 0.0;
#pragma unroll
      for (int j = 0; j < Q; ++j) a = fma(b[j], g[j], a);
      if (p == 0 && q == 1) {
        // adjoint of the tet's extra eta2 term: column (0,1) also collects v1 * Gp[1]
        const R* G1 = G + 1 * Q * QP;
#pragma unroll
        for (int j = 0; j < Q; ++j) a = fma(V1[j], G1[j * QP], a);
      }
      F[(cb + q) * QP + k] = a;
    }
  }
}

// one eta3 family of a collapsed shape's stage r^T (see ipr_r), lanes ln of a wave
template <int SH, int P, bool DER, typename R, int KAP>
__device__ __forceinline__ void ipr_r_fam(const Tile_<SH, P, R>& T, int ne, int fbuf, int ybuf, bool accumulate,
                                          int ln) {
  using D = Dims<SH, P>;
  constexpr int Q = D::Q, QP = D::QP, RL = P + 1 - KAP;
  constexpr int ncol = fam_ncols(SH, P, KAP), c0 = fam_start(SH, P, KAP);
  const int* perm = T.itab + D::NC * ICOL + (P + 2);
  for (int t = ln; t < ne * ncol; t += 64) {
    const ctab<R> C3 = launder(T.ct) + (DER ? D::L.dC3 : D::L.C3);
    const ctab<R> cf = C3 + fam_index(P, KAP, 0) * Q;
    const ctab<R> V1 = C3 + 1 * Q;
    const int e = t / ncol;
    const int c = perm[c0 + t - e * ncol];
    const int* ct = T.itab + c * ICOL;
    const int p = ct[0], q = ct[1], off = ct[2];
    const R* F = T.G(e, fbuf);
    R f[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) f[k] = F[c * QP + k];
    R* y = (ybuf < 0 ? T.U(e) : T.G(e, ybuf)) + off;
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      R a = 0.0;
#pragma unroll
      for (int k = 0; k < Q; ++k) a = fma(cf[r * Q + k], f[k], a);
      // adjoints of the collapsed-vertex splits
      const bool vx = (r == 1) && ((SH == PRISM && p == 0) || ((SH == PYR || SH == TET) && p == 0 && q == 0));
      if (vx) {
        R s[Q];
#pragma unroll
        for (int k = 0; k < Q; ++k) s[k] = 0.0;
        if (SH == PRISM) {
          const R* Fe = F + ((P + 1) + q) * QP;  // column (1,q)
#pragma unroll
          for (int k = 0; k < Q; ++k) s[k] = Fe[k];
        } else if (SH == PYR) {
          const R* Fa = F + (P + 1) * QP;  // (1,0)
          const R* Fb = F + 1 * QP;        // (0,1)
          const R* Fc = F + (P + 2) * QP;  // (1,1)
#pragma unroll
          for (int k = 0; k < Q; ++k) s[k] = Fa[k] + Fb[k] + Fc[k];
        } else {
          const R* Fa = F + 1 * QP;        // (0,1)
          const R* Fb = F + (P + 1) * QP;  // (1,0)
#pragma unroll
          for (int k = 0; k < Q; ++k) s[k] = Fa[k] + Fb[k];
        }
#pragma unroll
        for (int k = 0; k < Q; ++k) a = fma(V1[k], s[k], a);
      }
      if (accumulate)
        y[r] += a;
      else
        y[r] = a;
    }
  }
}

template <int SH, int P, bool DER, typename R, int KAP>
__device__ __forceinline__ void ipr_r_fams(const Tile_<SH, P, R>& T, int ne, int fbuf, int ybuf, bool accumulate,
                                           int wv, int nw, int ln) {
  if constexpr (KAP <= P) {
    if (KAP % nw == wv) ipr_r_fam<SH, P, DER, R, KAP>(T, ne, fbuf, ybuf, accumulate, ln);
    ipr_r_fams<SH, P, DER, R, KAP + 1>(T, ne, fbuf, ybuf, accumulate, wv, nw, ln);
  }
}

// stage r^T: F[c][k] (buffer fbuf) -> y modes into buffer ybuf (-1 = U), [NP]
template <int SH, int P, bool DER, typename R>
__device__ void ipr_r(const Tile_<SH, P, R>& T, int ne, int fbuf, int ybuf, bool accumulate) {
  using D = Dims<SH, P>;
  constexpr int Q = D::Q, QP = D::QP, n = D::n;
  if (SH == HEX) {
    for (int t = tid(); t < ne * D::NC; t += nthr()) {
      const ctab<R> C3u = launder(T.ct) + (DER ? D::L.dC3 : D::L.C3);
      const int e = t / D::NC, c = t - e * D::NC;
      const R* F = T.G(e, fbuf) + c * QP;
      R f[Q];
#pragma unroll
      for (int k = 0; k < Q; ++k) f[k] = F[k];
      R* y = (ybuf < 0 ? T.U(e) : T.G(e, ybuf)) + c * n;
#pragma unroll
      for (int r = 0; r < n; ++r) {
        R a = 0.0;
#pragma unroll
        for (int k = 0; k < Q; ++k) a = fma(C3u[r * Q + k], f[k], a);
        if (accumulate)
          y[r] += a;
        else
          y[r] = a;
      }
    }
    return;
  }
  // columns grouped by eta3 family, whole families per wave (as in bwd_r)
  const int nw = nthr() >> 6, ln = tid() & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid() >> 6);
  ipr_r_fams<SH, P, DER, R, 0>(T, ne, fbuf, ybuf, accumulate, wv, nw, ln);
}

// ---------------------------------------------------------------------------
// collocation derivatives
// ---------------------------------------------------------------------------

// one direction of the collocation derivative: lines along eta_{d+1}
template <int SH, int P, int DIR, bool TRANS, typename R>
__device__ __forceinline__ void grad_dir(const Tile_<SH, P, R>& T, int ne) {
  using D = Dims<SH, P>;
  constexpr int Q = D::Q, QP = D::QP;
  constexpr int stride = DIR == 0 ? Q * QP : DIR == 1 ? QP : 1;
  for (int t = tid(); t < ne * Q * Q; t += nthr()) {
    const ctab<R> Dm = launder(T.ct) + D::L.D + DIR * Q * Q;
    const int e = t / (Q * Q);
    const int r2 = t - e * (Q * Q);
    const int a = r2 / Q, b = r2 - a * Q;
    const int base = DIR == 0 ? a * QP + b : DIR == 1 ? a * Q * QP + b : (a * Q + b) * QP;
    const R* src = (TRANS ? T.G(e, DIR) : T.U(e)) + base;
    R v[Q];
#pragma unroll
    for (int l = 0; l < Q; ++l) v[l] = src[l * stride];
    R* g = T.G(e, DIR) + base;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      R s = 0.0;
#pragma unroll
      for (int l = 0; l < Q; ++l) s = fma(TRANS ? Dm[l * Q + i] : Dm[i * Q + l], v[l], s);
      g[i * stride] = s;
    }
  }
}

// G_d = D_d U for d = 0,1,2
template <int SH, int P, typename R>
__device__ void grad3(const Tile_<SH, P, R>& T, int ne) {
  grad_dir<SH, P, 0, false>(T, ne);
  grad_dir<SH, P, 1, false>(T, ne);
  grad_dir<SH, P, 2, false>(T, ne);
}

// G_d <- D_d^T G_d in place, d = 0,1,2
template <int SH, int P, typename R>
__device__ void grad3T(const Tile_<SH, P, R>& T, int ne) {
  grad_dir<SH, P, 0, true>(T, ne);
  grad_dir<SH, P, 1, true>(T, ne);
  grad_dir<SH, P, 2, true>(T, ne);
}

// ---------------------------------------------------------------------------
// merged and fused line stages of the Laplacian / Helmholtz tile
// ---------------------------------------------------------------------------
// The stages below do the same arithmetic per output as bwd_p, grad_dir and
// ipr_p (same operands, same order), so their results are bitwise those of the
// separate stages; they decompose each task index once and keep several lines
// of LDS reads in flight.

// bwd_p (G2 -> U) and, from the U line still in registers, the eta1
// derivative G0 = D_0 U: one task per (e, j, k)
template <int SH, int P, typename R>
__device__ void bwd_p_grad0(const Tile_<SH, P, R>& T, int ne) {
  using D = Dims<SH, P>;
  constexpr int Q = D::Q, n = D::n, QP = D::QP;
  for (int t = tid(); t < ne * Q * Q; t += nthr()) {
    const ctab<R> A1 = launder(T.ct) + D::L.A1;
    const int e = t / (Q * Q);
    const int rem = t - e * (Q * Q);
    const int j = rem / Q, k = rem - j * Q;
    const int o = j * QP + k;
    const R* G = T.G(e, 2) + o;
    R g[n];
#pragma unroll
    for (int p = 0; p < n; ++p) g[p] = G[p * Q * QP];
    R u[Q];
    R* U = T.U(e) + o;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      R s = 0.0;
#pragma unroll
      for (int p = 0; p < n; ++p) s = fma(A1[p * Q + i], g[p], s);
      u[i] = s;
      U[i * Q * QP] = s;
    }
    const ctab<R> Dm = launder(T.ct) + D::L.D;
    R* g0 = T.G(e, 0) + o;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      R s = 0.0;
#pragma unroll
      for (int l = 0; l < Q; ++l) s = fma(Dm[i * Q + l], u[l], s);
      g0[i * Q * QP] = s;
    }
  }
}

// eta2 and eta3 collocation derivatives in one task loop: G_d = D_d U
// (TRANS = false) or G_d <- D_d^T G_d in place (TRANS = true), d = 1, 2;
// task (e, a, b) is the j-line at (i, k) = (a, b) and the k-line at
// (i, j) = (a, b)
template <int SH, int P, bool TRANS, typename R>
__device__ void grad12(const Tile_<SH, P, R>& T, int ne) {
  using D = Dims<SH, P>;
  constexpr int Q = D::Q, QP = D::QP;
  for (int t = tid(); t < ne * Q * Q; t += nthr()) {
    const int e = t / (Q * Q);
    const int r2 = t - e * (Q * Q);
    const int a = r2 / Q, b = r2 - a * Q;
    const int o1 = a * Q * QP + b, o2 = (a * Q + b) * QP;
    const R* s1 = (TRANS ? T.G(e, 1) : T.U(e)) + o1;
    const R* s2 = (TRANS ? T.G(e, 2) : T.U(e)) + o2;
    R v1[Q], v2[Q];
#pragma unroll
    for (int l = 0; l < Q; ++l) {
      v1[l] = s1[l * QP];
      v2[l] = s2[l];
    }
    {
      const ctab<R> Dm = launder(T.ct) + D::L.D + 1 * Q * Q;
      R* g = T.G(e, 1) + o1;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        R s = 0.0;
#pragma unroll
        for (int l = 0; l < Q; ++l) s = fma(TRANS ? Dm[l * Q + i] : Dm[i * Q + l], v1[l], s);
        g[i * QP] = s;
      }
    }
    {
      const ctab<R> Dm = launder(T.ct) + D::L.D + 2 * Q * Q;
      R* g = T.G(e, 2) + o2;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        R s = 0.0;
#pragma unroll
        for (int l = 0; l < Q; ++l) s = fma(TRANS ? Dm[l * Q + i] : Dm[i * Q + l], v2[l], s);
        g[i] = s;
      }
    }
  }
}

// the eta1 transposed derivative D_0^T G0 kept in registers and summed with
// U (mask bit 0), G1 and G2 in ipr_p's order, then stage p^T into U
template <int SH, int P, typename R>
__device__ void grad0T_ipr_p(const Tile_<SH, P, R>& T, int ne, bool with_u) {
  using D = Dims<SH, P>;
  constexpr int Q = D::Q, n = D::n, QP = D::QP;
  for (int t = tid(); t < ne * Q * Q; t += nthr()) {
    const int e = t / (Q * Q);
    const int rem = t - e * (Q * Q);
    const int j = rem / Q, k = rem - j * Q;
    const int o = j * QP + k;
    // The eta1 line of G0 is held in registers. Up to Q = 8 the U, G1 and G2
    // lines are too; above that they are read per output, since holding all
    // four lines spills registers there. The sums are the same either way.
    constexpr bool hold = Q <= 8;
    R v[Q], u[hold ? Q : 1], w1[hold ? Q : 1], w2[hold ? Q : 1];
    const R* g0 = T.G(e, 0) + o;
    const R* pu = T.U(e) + o;
    const R* g1 = T.G(e, 1) + o;
    const R* g2 = T.G(e, 2) + o;
#pragma unroll
    for (int l = 0; l < Q; ++l) {
      v[l] = g0[l * Q * QP];
      if constexpr (hold) {
        if (with_u) u[l] = pu[l * Q * QP];
        w1[l] = g1[l * Q * QP];
        w2[l] = g2[l * Q * QP];
      }
    }
    R s[Q];
    const ctab<R> Dm0 = hold ? launder(T.ct) + D::L.D : T.ct + D::L.D;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      // above Q = 8 re-derived per output, so only one column of D is live
      // in SGPRs (the whole table does not fit)
      ctab<R> Dm = Dm0;
      if constexpr (!hold) Dm = launder(T.ct) + D::L.D;
      R d0 = 0.0;
#pragma unroll
      for (int l = 0; l < Q; ++l) d0 = fma(Dm[l * Q + i], v[l], d0);
      R a = 0.0;
      if (with_u) a += hold ? u[hold ? i : 0] : pu[i * Q * QP];
      a += d0;
      a += hold ? w1[hold ? i : 0] : g1[i * Q * QP];
      a += hold ? w2[hold ? i : 0] : g2[i * Q * QP];
      s[i] = a;
    }
    const ctab<R> A10 = hold ? launder(T.ct) + D::L.A1 : T.ct + D::L.A1;
    R* G = T.U(e) + o;
#pragma unroll
    for (int p = 0; p < n; ++p) {
      ctab<R> A1 = A10;
      if constexpr (!hold) A1 = launder(T.ct) + D::L.A1;
      R a = 0.0;
#pragma unroll
      for (int i = 0; i < Q; ++i) a = fma(A1[p * Q + i], s[i], a);
      G[p * Q * QP] = a;
    }
  }
}

// ---------------------------------------------------------------------------
// global <-> LDS
// ---------------------------------------------------------------------------

template <int SH, int P, typename R>
__device__ void load_modes(const Tile_<SH, P, R>& T, const R* __restrict__ in, long long e0, int ne, int buf) {
  using D = Dims<SH, P>;
  const R* src = in + e0 * D::NP;
  for (int t = tid(); t < ne * D::NP; t += nthr()) {
    const int e = t / D::NP, m = t - e * D::NP;
    (buf < 0 ? T.U(e) : T.G(e, buf))[m] = src[t];
  }
}

template <int SH, int P, typename R>
__device__ void store_modes(const Tile_<SH, P, R>& T, R* __restrict__ out, long long e0, int ne, int buf) {
  using D = Dims<SH, P>;
  R* dst = out + e0 * D::NP;
  for (int t = tid(); t < ne * D::NP; t += nthr()) {
    const int e = t / D::NP, m = t - e * D::NP;
    dst[t] = (buf < 0 ? T.U(e) : T.G(e, buf))[m];
  }
}

template <int SH, int P>
__device__ __forceinline__ int lds_pt(int pt) {
  using D = Dims<SH, P>;
  const int i = pt / D::Q2;
  const int r = pt - i * D::Q2;
  const int j = r / D::Q, k = r - j * D::Q;
  return D::pidx(i, j, k);
}

// ---------------------------------------------------------------------------
// tile bodies, one per operator
// ---------------------------------------------------------------------------

template <int SH, int P, typename R>
__device__ void bwd_chain(const Tile_<SH, P, R>& T, int ne) {
  // modes in G0 -> F in G1 -> G in G2 -> U
  bwd_r<SH, P, false>(T, ne, 0, 1);
  __syncthreads();
  bwd_q<SH, P, false>(T, ne, 1, 2);
  __syncthreads();
  bwd_p<SH, P, false>(T, ne, 2, -1);
  __syncthreads();
}

// points summed over mask -> modes in buffer G1; returns after a barrier
template <int SH, int P, typename R>
__device__ void ipr_chain(const Tile_<SH, P, R>& T, int ne, int mask) {
  ipr_p<SH, P, false>(T, ne, mask, -1);
  __syncthreads();
  ipr_q<SH, P, false>(T, ne, -1, 0);
  __syncthreads();
  ipr_r<SH, P, false>(T, ne, 0, 1, false);
  __syncthreads();
}

// The tile of every collocated operator: the stages read their tables through
// the constant path except the tet's eta2 table and the column table, which
// are all the (compact) LDS head holds.
template <int SH, int P, int OP, typename R>
__device__ void tile_body(const OpArgs& a, long long e0, int ne, const Tile_<SH, P, R>& T) {
  using D = Dims<SH, P>;
  constexpr int Q3 = D::Q3;
  load_tables_helm<SH, P>(a, T);
  // the mass's jw at a thread's first PF points, loaded at the start so that
  // the loads overlap the line stages (points past PF nthr() are read where
  // they are used; prefetching the 9 d eta/d x of the physical derivative the
  // same way costs it occupancy and time)
  constexpr int PF = 4;
  double gpf[PF];
  if constexpr (OP == OPK_MASS) {
    const double* g = a.fac + e0 * (long long)(NFAC * Q3);
#pragma unroll
    for (int it = 0; it < PF; ++it) {
      const int t = tid() + it * nthr();
      const int tc = t < ne * Q3 ? t : 0;  // in bounds; unused when t is past the tile
      const int e = tc / Q3, pt = tc - e * Q3;
      gpf[it] = g[e * (NFAC * Q3) + pt];
    }
  }
  if (OP == OPK_BWD || OP == OPK_MASS || OP == OPK_LAP || OP == OPK_HELM) {
    load_modes<SH, P>(T, reinterpret_cast<const R*>(a.in), e0, ne, 0);
    __syncthreads();
    bwd_chain<SH, P>(T, ne);
  } else {
    __syncthreads();
  }

  if (OP == OPK_BWD) {
    R* dst = reinterpret_cast<R*>(a.out) + e0 * Q3;
    for (int t = tid(); t < ne * Q3; t += nthr()) {
      const int e = t / Q3, pt = t - e * Q3;
      dst[t] = T.U(e)[lds_pt<SH, P>(pt)];
    }
    return;
  }

  if (OP == OPK_IPR || OP == OPK_MASS) {
    const double* fac = a.fac + e0 * (long long)(NFAC * Q3);
    const R* src = reinterpret_cast<const R*>(a.in) + e0 * Q3;
    int it = 0;
    for (int t = tid(); t < ne * Q3; t += nthr(), ++it) {
      const int e = t / Q3, pt = t - e * Q3;
      double jw;
      if constexpr (OP == OPK_MASS)
        jw = it < PF ? gpf[it < PF ? it : 0] : fac[e * (NFAC * Q3) + pt];
      else
        jw = fac[e * (NFAC * Q3) + pt];
      R* u = T.U(e) + lds_pt<SH, P>(pt);
      const double f = (OP == OPK_IPR) ? src[t] : *u;
      *u = jw * f;
    }
    __syncthreads();
    ipr_chain<SH, P>(T, ne, 1);
    store_modes<SH, P>(T, reinterpret_cast<R*>(a.out), e0, ne, 1);
    return;
  }

  if (OP == OPK_DERIV) {
    const R* src = reinterpret_cast<const R*>(a.in) + e0 * Q3;
    for (int t = tid(); t < ne * Q3; t += nthr()) {
      const int e = t / Q3, pt = t - e * Q3;
      T.U(e)[lds_pt<SH, P>(pt)] = src[t];
    }
    __syncthreads();
    grad3<SH, P>(T, ne);
    __syncthreads();
    const double* dxi = a.dxi + e0 * (long long)(NDXI * Q3);
    for (int t = tid(); t < ne * Q3; t += nthr()) {
      const int e = t / Q3, pt = t - e * Q3;
      const int lp = lds_pt<SH, P>(pt);
      const double g0 = T.G(e, 0)[lp], g1 = T.G(e, 1)[lp], g2 = T.G(e, 2)[lp];
      const double* m = dxi + e * (NDXI * Q3) + pt;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double v = m[(0 * 3 + i) * Q3] * g0 + m[(1 * 3 + i) * Q3] * g1 + m[(2 * 3 + i) * Q3] * g2;
        reinterpret_cast<R*>(a.out)[i * a.out_cs + e0 * Q3 + t] = (R)v;
      }
    }
    return;
  }

  if (OP == OPK_IPRD) {
    const double* dxi = a.dxi + e0 * (long long)(NDXI * Q3);
    const double* fac = a.fac + e0 * (long long)(NFAC * Q3);
    for (int t = tid(); t < ne * Q3; t += nthr()) {
      const int e = t / Q3, pt = t - e * Q3;
      const int lp = lds_pt<SH, P>(pt);
      const R* fin = reinterpret_cast<const R*>(a.in);
      const double f0 = fin[0 * a.in_cs + e0 * Q3 + t];
      const double f1 = fin[1 * a.in_cs + e0 * Q3 + t];
      const double f2 = fin[2 * a.in_cs + e0 * Q3 + t];
      const double jw = fac[e * (NFAC * Q3) + pt];
      const double* m = dxi + e * (NDXI * Q3) + pt;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double v = m[(d * 3 + 0) * Q3] * f0 + m[(d * 3 + 1) * Q3] * f1 + m[(d * 3 + 2) * Q3] * f2;
        T.G(e, d)[lp] = jw * v;
      }
    }
    __syncthreads();
    grad3T<SH, P>(T, ne);
    __syncthreads();
    ipr_chain<SH, P>(T, ne, 2 | 4 | 8);
    store_modes<SH, P>(T, reinterpret_cast<R*>(a.out), e0, ne, 1);
    return;
  }

  if (OP == OPK_LAP || OP == OPK_HELM) {
    grad3<SH, P>(T, ne);
    __syncthreads();
    const double* fac = a.fac + e0 * (long long)(NFAC * Q3);
    const double lam = (OP == OPK_HELM) ? a.lambda : 0.0;
    for (int t = tid(); t < ne * Q3; t += nthr()) {
      const int e = t / Q3, pt = t - e * Q3;
      const int lp = lds_pt<SH, P>(pt);
      const double* g = fac + e * (NFAC * Q3) + pt;
      const double jw = g[0];
      const double g00 = g[1 * Q3], g01 = g[2 * Q3], g02 = g[3 * Q3];
      const double g11 = g[4 * Q3], g12 = g[5 * Q3], g22 = g[6 * Q3];
      R* u = T.U(e) + lp;
      R* p0 = T.G(e, 0) + lp;
      R* p1 = T.G(e, 1) + lp;
      R* p2 = T.G(e, 2) + lp;
      const double d0 = *p0, d1 = *p1, d2 = *p2;
      *p0 = g00 * d0 + g01 * d1 + g02 * d2;
      *p1 = g01 * d0 + g11 * d1 + g12 * d2;
      *p2 = g02 * d0 + g12 * d1 + g22 * d2;
      if (OP == OPK_HELM) *u = lam * jw * (*u);
    }
    __syncthreads();
    grad3T<SH, P>(T, ne);
    __syncthreads();
    ipr_chain<SH, P>(T, ne, (OP == OPK_HELM ? 1 : 0) | 2 | 4 | 8);
    store_modes<SH, P>(T, reinterpret_cast<R*>(a.out), e0, ne, 1);
    return;
  }
}

template <int SH, int P>
__device__ Tile_<SH, P> make_tile(double* smem, const double* gtab) {
  using D = Dims<SH, P>;
  Tile_<SH, P> T;
  T.tab = smem;
  T.itab = reinterpret_cast<int*>(smem + D::NTAB);
  T.b2 = smem + D::L.B2;
  T.ct = as_const(gtab);
  T.el = smem + D::HEAD;
  T.per = D::PER_ELEM;
  return T;
}

// LDS head (tables and column table) in units of R
template <int SH, int P, typename R>
constexpr int head_r() {
  using D = Dims<SH, P>;
  return D::NTAB + (int)((D::NITAB * sizeof(int) + sizeof(R) - 1) / sizeof(R));
}

template <int SH, int P, typename R>
__device__ Tile_<SH, P, R> make_tile_r(void* smem, const R* gtab) {
  using D = Dims<SH, P>;
  Tile_<SH, P, R> T;
  T.tab = reinterpret_cast<R*>(smem);
  T.itab = reinterpret_cast<int*>(T.tab + D::NTAB);
  T.b2 = T.tab + D::L.B2;
  T.ct = (ctab<R>)(gtab);
  T.el = T.tab + head_r<SH, P, R>();
  T.per = D::PER_ELEM;
  return T;
}

template <int SH, int P, typename R>
constexpr size_t lds_bytes_r(int E) {
  return sizeof(R) * (size_t)(head_r<SH, P, R>() + E * Dims<SH, P>::PER_ELEM);
}

// Compact LDS head of the Laplacian / Helmholtz tile (helm_tile), in units of
// R: only the tables that tile reads per lane, the tet's eta2 table B2 and the
// collapsed shapes' column table (every other table is read at wave-uniform
// indices through the constant path).  At P = 10 it takes the tet's tile from
// 88 to 63 KB of LDS, so two work-groups fit a CU's 160 KB instead of one.
template <int SH, int P, typename R>
constexpr int head_h() {
  using D = Dims<SH, P>;
  constexpr int b2 = SH == TET ? D::L.nb2 * D::Q : 0;
  constexpr int it = SH == HEX ? 0 : (int)((D::NITAB * sizeof(int) + sizeof(R) - 1) / sizeof(R));
  return b2 + it;
}

template <int SH, int P, typename R>
__device__ Tile_<SH, P, R> make_tile_h(void* smem, const R* gtab) {
  using D = Dims<SH, P>;
  Tile_<SH, P, R> T;
  T.tab = reinterpret_cast<R*>(smem);  // no full table: only b2 and itab are read
  T.b2 = T.tab;
  T.itab = reinterpret_cast<int*>(T.tab + (SH == TET ? D::L.nb2 * D::Q : 0));
  T.ct = (ctab<R>)(gtab);
  T.el = T.tab + head_h<SH, P, R>();
  T.per = D::PER_ELEM;
  return T;
}

template <int SH, int P, typename R>
constexpr size_t lds_bytes_h(int E) {
  return sizeof(R) * (size_t)(head_h<SH, P, R>() + E * Dims<SH, P>::PER_ELEM);
}

template <int SH, int P>
__device__ Tile_<SH, P> make_tile3(double* smem, const double* gtab) {
  Tile_<SH, P> T = make_tile<SH, P>(smem, gtab);
  T.per = 3 * Dims<SH, P>::S3;
  return T;
}

// one tile per work-group, tiles of one block
template <int SH, int P, int OP>
__global__ void __launch_bounds__(512) k_block(OpArgs a) {
  extern __shared__ double smem[];
  const long long e0 = (long long)blockIdx.x * a.E;
  const long long rem = a.n_elem - e0;
  const int ne = rem < a.E ? (int)rem : a.E;
  if (ne <= 0) return;
  const Tile_<SH, P> T = make_tile_h<SH, P, double>(smem, a.tab);
  tile_body<SH, P, OP>(a, e0, ne, T);
}

// Mixed-shape launch: one tile per work-group from a tile list that spans every
// block (all blocks share P).  Block b's part of the whole-mesh buffers starts
// at its coefficient or point offset.
template <int P, int OP>
__global__ void __launch_bounds__(512) k_mixed(const BlockStatic* __restrict__ blocks, const Tile* __restrict__ tiles,
                                               int ntiles, const double* in, double* out, long long in_cs,
                                               long long out_cs, double lambda) {
  extern __shared__ double smem[];
  const int ti = blockIdx.x;
  if (ti >= ntiles) return;
  const Tile tl = tiles[ti];
  const BlockStatic b = blocks[tl.blk];
  constexpr bool in_modes = (OP == OPK_BWD || OP == OPK_MASS || OP == OPK_LAP || OP == OPK_HELM || OP == OPK_HELM_NC ||
                             OP == OPK_LAP_NC);
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
  a.E = b.E;
  a.pad_ = 0;
  switch (b.shape) {
    case HEX: tile_body<HEX, P, OP>(a, tl.e0, tl.ne, make_tile_h<HEX, P, double>(smem, a.tab)); break;
    case PRISM: tile_body<PRISM, P, OP>(a, tl.e0, tl.ne, make_tile_h<PRISM, P, double>(smem, a.tab)); break;
    case PYR: tile_body<PYR, P, OP>(a, tl.e0, tl.ne, make_tile_h<PYR, P, double>(smem, a.tab)); break;
    default: tile_body<TET, P, OP>(a, tl.e0, tl.ne, make_tile_h<TET, P, double>(smem, a.tab)); break;
  }
}

// ---------------------------------------------------------------------------
// Pipelined Laplacian / Helmholtz: persistent work-groups, geometry in registers
// ---------------------------------------------------------------------------
// Each work-group walks the tile list with a stride of the grid size.  The 7
// geometric factors of the points a thread owns in the metric stage are loaded
// into registers before they are needed: for the first tile at kernel start,
// for every later tile right after the previous tile's metric stage, so the
// HBM latency of the dominant byte stream overlaps the sum-factorisation stages.
// PPT is the number of points a thread owns in the metric stage.

// G: the type the factors are stored in (double, or float for the FP32
// actions of a plan with an FP32 copy of its factors)
template <int PPT, typename G = double>
struct GeoRegs {
  G v[PPT][NFAC];
};

// Every slot issues its loads, so the number of loads in flight is a
// compile-time constant: a wait for data loaded before the prefetch then
// counts past these loads instead of draining them.  The loads go through a
// buffer resource that spans the tile's factors: a slot past the tile's last
// point reads out of range, which returns zero without touching memory.
template <int P, int PPT, typename G>
__device__ __forceinline__ void prefetch_geo(const G* __restrict__ fac, long long e0, int ne, GeoRegs<PPT, G>& g) {
  constexpr int Q3 = (P + 2) * (P + 2) * (P + 2);
  constexpr int W = (int)sizeof(G);
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(fac + e0 * (long long)(NFAC * Q3)), (short)0, ne * (NFAC * Q3 * W), 0x00020000);
  const int n = ne * Q3;
#pragma unroll
  for (int it = 0; it < PPT; ++it) {
    const int t = tid() + it * nthr();
    const int e = t / Q3, pt = t - e * Q3;
    // byte offset of factor 0 of this point; out of range past the tile
    const int off = t < n ? (e * (NFAC * Q3) + pt) * W : ne * (NFAC * Q3 * W);
#pragma unroll
    for (int c = 0; c < NFAC; ++c) {
      if constexpr (W == 8)
        g.v[it][c] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, off + c * Q3 * 8, 0, 2));
      else
        g.v[it][c] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, off + c * Q3 * 4, 0, 2));
    }
  }
}

// register slots per thread for a tile's modes when its points fill at most
// PPT slots per thread (E N_P / threads <= PPT N_P / Q^3)
template <int SH, int P, int PPT>
constexpr int mode_slots() {
  constexpr int Q3 = (P + 2) * (P + 2) * (P + 2);
  return (PPT * num_modes(SH, P) + Q3 - 1) / Q3;
}

struct NoPrefetch {
  __device__ void operator()() const {}
};

// OP = OPK_ADR adds the advection term sum_d a_d D_d u at the points to the
// reaction term, with a_d = jw sum_i b_i d eta_d / d x_i read from adv
// ([n_elem][3][Q^3] of the tile's block).
// pre() runs after the tile's modes are requested and before they are written
// to LDS: the one-tile-per-work-group launches issue the tile's geometry
// prefetch there, so the first stages run while the geometry streams in.
template <int SH, int P, int OP, int PPT, typename Next, typename R, typename G, typename Pre = NoPrefetch>
__device__ void helm_tile(const OpArgs& a, long long e0, int ne, const Tile_<SH, P, R>& T, GeoRegs<PPT, G>& g,
                          bool tables, Next next, const double* __restrict__ adv = nullptr, Pre pre = Pre{}) {
  using D = Dims<SH, P>;
  constexpr int Q3 = D::Q3;
  if (tables) load_tables_helm<SH, P>(a, T);
  {
    // modes into registers (every slot loads; slots past the tile re-read
    // its last mode), then the prefetch, then the LDS writes
    constexpr int MS = mode_slots<SH, P, PPT>();
    const int nm = ne * D::NP;
    const R* src = reinterpret_cast<const R*>(a.in) + e0 * D::NP;
    R mv[MS];
#pragma unroll
    for (int s = 0; s < MS; ++s) {
      const int t = tid() + s * nthr();
      mv[s] = src[t < nm ? t : nm - 1];
    }
    pre();
    // slots past the tile write their (re-read) last mode to its own place,
    // so every slot's load has a use on every path and stays ahead of pre()
#pragma unroll
    for (int s = 0; s < MS; ++s) {
      const int t0 = tid() + s * nthr();
      const int t = t0 < nm ? t0 : nm - 1;
      const int e = t / D::NP, m = t - e * D::NP;
      T.G(e, 0)[m] = mv[s];
    }
    for (int t = tid() + MS * nthr(); t < nm; t += nthr()) {
      const int e = t / D::NP, m = t - e * D::NP;
      T.G(e, 0)[m] = src[t];
    }
  }
  __syncthreads();
  // modes in G0 -> F in G1 -> G in G2 -> U, with G0 = D_0 U from the same task
  bwd_r<SH, P, false>(T, ne, 0, 1);
  __syncthreads();
  bwd_q<SH, P, false>(T, ne, 1, 2);
  __syncthreads();
  bwd_p_grad0<SH, P>(T, ne);
  __syncthreads();
  grad12<SH, P, false>(T, ne);
  __syncthreads();
  // the metric in FP64, or in FP32 when the factors are stored in FP32
  using MT = G;
  const MT lam = (OP == OPK_HELM || OP == OPK_ADR) ? (MT)a.lambda : (MT)0;
#pragma unroll
  for (int it = 0; it < PPT; ++it) {
    const int t = tid() + it * nthr();
    if (t < ne * Q3) {
      const int e = t / Q3, pt = t - e * Q3;
      const int lp = lds_pt<SH, P>(pt);
      const MT* gg = g.v[it];
      R* p0 = T.G(e, 0) + lp;
      R* p1 = T.G(e, 1) + lp;
      R* p2 = T.G(e, 2) + lp;
      const MT d0 = *p0, d1 = *p1, d2 = *p2;
      *p0 = gg[1] * d0 + gg[2] * d1 + gg[3] * d2;
      *p1 = gg[2] * d0 + gg[4] * d1 + gg[5] * d2;
      *p2 = gg[3] * d0 + gg[5] * d1 + gg[6] * d2;
      if (OP == OPK_HELM) {
        R* u = T.U(e) + lp;
        *u = lam * gg[0] * (*u);
      }
      if constexpr (OP == OPK_ADR) {
        const gptr_t av = as_global(adv) + (e0 + e) * (3LL * Q3) + pt;
        R* u = T.U(e) + lp;
        *u = lam * gg[0] * (*u) + (av[0] * d0 + av[Q3] * d1 + av[2 * Q3] * d2);
      }
    }
  }
  next();  // registers of this tile's geometry are dead: start the next tile's loads
  __syncthreads();
  grad12<SH, P, true>(T, ne);
  __syncthreads();
  // points -> modes: stage p^T (with D_0^T) into U, q^T into G0, r^T into G1
  grad0T_ipr_p<SH, P>(T, ne, OP == OPK_HELM || OP == OPK_ADR);
  __syncthreads();
  ipr_q<SH, P, false>(T, ne, -1, 0);
  __syncthreads();
  ipr_r<SH, P, false>(T, ne, 0, 1, false);
  __syncthreads();
  store_modes<SH, P>(T, reinterpret_cast<R*>(a.out), e0, ne, 1);
}

template <int SH, int P, int OP, int PPT>
__global__ void __launch_bounds__(512) k_helm_persist(OpArgs a, int ntiles) {
  extern __shared__ double smem[];
  int ti = blockIdx.x;
  if (ti >= ntiles) return;
  const Tile_<SH, P> T = make_tile_h<SH, P, double>(smem, a.tab);
  auto ne_of = [&](int i) {
    const long long r = a.n_elem - (long long)i * a.E;
    return (int)(r < a.E ? r : a.E);
  };
  GeoRegs<PPT> g;
  prefetch_geo<P, PPT>(a.fac, (long long)ti * a.E, ne_of(ti), g);
  bool first = true;
  while (true) {
    const int nx = ti + (int)gridDim.x;
    __syncthreads();
    helm_tile<SH, P, OP, PPT>(a, (long long)ti * a.E, ne_of(ti), T, g, first, [&]() {
      if (nx < ntiles) prefetch_geo<P, PPT>(a.fac, (long long)nx * a.E, ne_of(nx), g);
    });
    first = false;
    if (nx >= ntiles) break;
    ti = nx;
  }
}

template <int P, int OP, int PPT>
__global__ void __launch_bounds__(512) k_helm_mixed_persist(const BlockStatic* __restrict__ blocks,
                                                            const Tile* __restrict__ tiles, int ntiles,
                                                            const double* in, double* out, double lambda) {
  extern __shared__ double smem[];
  int ti = blockIdx.x;
  if (ti >= ntiles) return;
  Tile tl = tiles[ti];
  GeoRegs<PPT> g;
  prefetch_geo<P, PPT>(blocks[tl.blk].fac, tl.e0, tl.ne, g);
  int prev = -1;
  while (true) {
    const int nx = ti + (int)gridDim.x;
    Tile tn = tl;
    if (nx < ntiles) tn = tiles[nx];
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
    const bool tables = (tl.blk != prev);
    auto next = [&]() {
      if (nx < ntiles) prefetch_geo<P, PPT>(blocks[tn.blk].fac, tn.e0, tn.ne, g);
    };
    __syncthreads();
    switch (b.shape) {
      case HEX: helm_tile<HEX, P, OP, PPT>(a, tl.e0, tl.ne, make_tile_h<HEX, P, double>(smem, a.tab), g, tables, next); break;
      case PRISM: helm_tile<PRISM, P, OP, PPT>(a, tl.e0, tl.ne, make_tile_h<PRISM, P, double>(smem, a.tab), g, tables, next); break;
      case PYR: helm_tile<PYR, P, OP, PPT>(a, tl.e0, tl.ne, make_tile_h<PYR, P, double>(smem, a.tab), g, tables, next); break;
      default: helm_tile<TET, P, OP, PPT>(a, tl.e0, tl.ne, make_tile_h<TET, P, double>(smem, a.tab), g, tables, next); break;
    }
    prev = tl.blk;
    if (nx >= ntiles) break;
    ti = nx;
    tl = tn;
  }
}

// One tile per work-group, with the tile's geometric factors loaded into
// registers at kernel start (they arrive during the sum-factorisation stages).
template <int SH, int P, int OP, int PPT>
__global__ void __launch_bounds__(512) k_helm_block_pf(OpArgs a) {
  extern __shared__ double smem[];
  const long long e0 = (long long)blockIdx.x * a.E;
  const long long rem = a.n_elem - e0;
  const int ne = rem < a.E ? (int)rem : a.E;
  if (ne <= 0) return;
  GeoRegs<PPT> g;
  helm_tile<SH, P, OP, PPT>(a, e0, ne, make_tile_h<SH, P, double>(smem, a.tab), g, true, []() {}, nullptr,
                            [&]() { prefetch_geo<P, PPT>(a.fac, e0, ne, g); });
}

// G = float reads the plan's FP32 copy of the factors (BlockStatic::fac32)
template <int P, int OP, int PPT, typename R = double, typename G = double>
__global__ void __launch_bounds__(512) k_helm_mixed_pf(const BlockStatic* __restrict__ blocks,
                                                       const Tile* __restrict__ tiles, int ntiles, const double* in,
                                                       double* out, double lambda) {
  extern __shared__ double smem[];
  const int ti = blockIdx.x;
  if (ti >= ntiles) return;
  const Tile tl = tiles[ti];
  const BlockStatic b = blocks[tl.blk];
  GeoRegs<PPT, G> g;
  OpArgs a;
  a.tab = b.tab;
  a.itab = b.itab;
  a.fac = b.fac;
  a.dxi = b.dxi;
  a.n_elem = b.n_elem;
  // in/out hold values of type R; the offsets count values
  a.in = reinterpret_cast<const double*>(reinterpret_cast<const R*>(in) + b.coeff_off);
  a.out = reinterpret_cast<double*>(reinterpret_cast<R*>(out) + b.coeff_off);
  a.in_cs = 0;
  a.out_cs = 0;
  a.lambda = lambda;
  a.E = 0;
  a.pad_ = 0;
  const R* gt = sizeof(R) == sizeof(double) ? reinterpret_cast<const R*>(b.tab) : reinterpret_cast<const R*>(b.tabf);
  const G* gf;
  if constexpr (sizeof(G) == sizeof(double))
    gf = b.fac;
  else
    gf = b.fac32;
  auto none = []() {};
  auto pf = [&]() { prefetch_geo<P, PPT>(gf, tl.e0, tl.ne, g); };
  switch (b.shape) {
    case HEX:
      helm_tile<HEX, P, OP, PPT>(a, tl.e0, tl.ne, make_tile_h<HEX, P, R>(smem, gt), g, true, none, nullptr, pf);
      break;
    case PRISM:
      helm_tile<PRISM, P, OP, PPT>(a, tl.e0, tl.ne, make_tile_h<PRISM, P, R>(smem, gt), g, true, none, nullptr, pf);
      break;
    case PYR:
      helm_tile<PYR, P, OP, PPT>(a, tl.e0, tl.ne, make_tile_h<PYR, P, R>(smem, gt), g, true, none, nullptr, pf);
      break;
    default:
      helm_tile<TET, P, OP, PPT>(a, tl.e0, tl.ne, make_tile_h<TET, P, R>(smem, gt), g, true, none, nullptr, pf);
      break;
  }
}

// Whole-mesh advection-diffusion-reaction action (FP64): k_helm_mixed_pf with
// the advection factors adv ([3][Q^3] per element, blocks concatenated like the
// point buffers).
template <int P, int PPT>
__global__ void __launch_bounds__(512) k_adr_mixed_pf(const BlockStatic* __restrict__ blocks,
                                                      const Tile* __restrict__ tiles, int ntiles, const double* in,
                                                      double* out, double lambda, const double* __restrict__ adv) {
  extern __shared__ double smem[];
  const int ti = blockIdx.x;
  if (ti >= ntiles) return;
  const Tile tl = tiles[ti];
  const BlockStatic b = blocks[tl.blk];
  GeoRegs<PPT> g;
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
  const double* ab = adv + 3 * b.phys_off;
  auto none = []() {};
  auto pf = [&]() { prefetch_geo<P, PPT>(b.fac, tl.e0, tl.ne, g); };
  switch (b.shape) {
    case HEX: helm_tile<HEX, P, OPK_ADR, PPT>(a, tl.e0, tl.ne, make_tile_h<HEX, P, double>(smem, b.tab), g, true, none, ab, pf); break;
    case PRISM:
      helm_tile<PRISM, P, OPK_ADR, PPT>(a, tl.e0, tl.ne, make_tile_h<PRISM, P, double>(smem, b.tab), g, true, none, ab, pf);
      break;
    case PYR: helm_tile<PYR, P, OPK_ADR, PPT>(a, tl.e0, tl.ne, make_tile_h<PYR, P, double>(smem, b.tab), g, true, none, ab, pf); break;
    default: helm_tile<TET, P, OPK_ADR, PPT>(a, tl.e0, tl.ne, make_tile_h<TET, P, double>(smem, b.tab), g, true, none, ab, pf); break;
  }
}

// ---------------------------------------------------------------------------
// Fused collocated Laplacian / Helmholtz (three LDS buffers per element)
// ---------------------------------------------------------------------------
// The stages are grouped by line orientation so that each thread keeps a line
// in registers across several operations:
//   i-lines: stage p of B fused with D_1          (U <- u, G0 <- D_1 u)
//   j-lines: D_2                                  (G1 <- D_2 u)
//   k-lines: D_3, the metric, D_3^T and lambda jw u in registers
//            (U <- D_3^T v_3 + lambda jw u, G0 <- v_1, G1 <- v_2)
//   j-lines: D_2^T in place on G1
//   i-lines: D_1^T fused with stage p of B^T      (U <- sum_i A_p(z_i) (...))
// A k-line's 7 Q geometric factors are contiguous in HBM, so a thread reads
// them with wide loads, either in the k-line stage or (PF) at the start of the
// tile into registers.

template <int Q>
struct GeoLine {
  double v[NFAC][Q];
};

template <int P>
__device__ __forceinline__ void load_geo_line(gptr_t fac_tile, int e, int i, int j, GeoLine<P + 2>& g) {
  constexpr int Q = P + 2, Q3 = Q * Q * Q;
  const gptr_t f = fac_tile + e * (NFAC * Q3) + (i * Q + j) * Q;
#pragma unroll
  for (int c = 0; c < NFAC; ++c)
#pragma unroll
    for (int k = 0; k < Q; ++k) g.v[c][k] = __builtin_nontemporal_load(f + c * Q3 + k);
}

// i-lines: Gq (in U, p rows) -> U = u and G0 = D_1 u
template <int SH, int P>
__device__ void bwd_p_d1(const Tile_<SH, P>& T, int ne) {
  using D = Dims<SH, P>;
  constexpr int Q = D::Q, n = D::n, QP = D::QP;
  for (int t = tid(); t < ne * Q * Q; t += nthr()) {
    const ctab_t A1 = launder(T.ct) + D::L.A1;
    const ctab_t D1 = launder(T.ct) + D::L.D;
    const int e = t / (Q * Q);
    const int rem = t - e * (Q * Q);
    const int j = rem / Q, k = rem - j * Q;
    double* U = T.U(e) + j * QP + k;
    double* G0 = T.G(e, 0) + j * QP + k;
    double g[n];
#pragma unroll
    for (int p = 0; p < n; ++p) g[p] = U[p * Q * QP];
    double u[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      double s = 0.0;
#pragma unroll
      for (int p = 0; p < n; ++p) s = fma(A1[p * Q + i], g[p], s);
      u[i] = s;
      U[i * Q * QP] = s;
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < Q; ++l) s = fma(D1[i * Q + l], u[l], s);
      G0[i * Q * QP] = s;
    }
  }
}

// j-lines: G1 = D_2 U (TRANS: G1 <- D_2^T G1)
template <int SH, int P, bool TRANS>
__device__ void d2_lines(const Tile_<SH, P>& T, int ne) {
  using D = Dims<SH, P>;
  constexpr int Q = D::Q, QP = D::QP;
  for (int t = tid(); t < ne * Q * Q; t += nthr()) {
    const ctab_t Dm = launder(T.ct) + D::L.D + 1 * Q * Q;
    const int e = t / (Q * Q);
    const int rem = t - e * (Q * Q);
    const int i = rem / Q, k = rem - i * Q;
    const int base = i * Q * QP + k;
    const double* src = (TRANS ? T.G(e, 1) : T.U(e)) + base;
    double v[Q];
#pragma unroll
    for (int l = 0; l < Q; ++l) v[l] = src[l * QP];
    double* g = T.G(e, 1) + base;
#pragma unroll
    for (int jj = 0; jj < Q; ++jj) {
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < Q; ++l) s = fma(TRANS ? Dm[l * Q + jj] : Dm[jj * Q + l], v[l], s);
      g[jj * QP] = s;
    }
  }
}

// k-lines: the metric stage with D_3 and D_3^T in registers
template <int SH, int P, int OP, bool PF>
__device__ void kline_metric(const Tile_<SH, P>& T, int ne, gptr_t fac_tile, double lam, GeoLine<P + 2>& gpf) {
  using D = Dims<SH, P>;
  constexpr int Q = D::Q, QP = D::QP;
  for (int t = tid(); t < ne * Q * Q; t += nthr()) {
    const ctab_t D3 = launder(T.ct) + D::L.D + 2 * Q * Q;
    const int e = t / (Q * Q);
    const int rem = t - e * (Q * Q);
    const int i = rem / Q, j = rem - i * Q;
    GeoLine<Q> gl;
    if (!PF) load_geo_line<P>(fac_tile, e, i, j, gl);
    const GeoLine<Q>& g = PF ? gpf : gl;
    const int base = (i * Q + j) * QP;
    double* U = T.U(e) + base;
    double* G0 = T.G(e, 0) + base;
    double* G1 = T.G(e, 1) + base;
    double u[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) u[k] = U[k];
    double v2[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      double d2 = 0.0;
#pragma unroll
      for (int l = 0; l < Q; ++l) d2 = fma(D3[k * Q + l], u[l], d2);
      const double d0 = G0[k], d1 = G1[k];
      G0[k] = g.v[1][k] * d0 + g.v[2][k] * d1 + g.v[3][k] * d2;
      G1[k] = g.v[2][k] * d0 + g.v[4][k] * d1 + g.v[5][k] * d2;
      v2[k] = g.v[3][k] * d0 + g.v[5][k] * d1 + g.v[6][k] * d2;
    }
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      double o = (OP == OPK_HELM) ? lam * g.v[0][k] * u[k] : 0.0;
#pragma unroll
      for (int m = 0; m < Q; ++m) o = fma(D3[m * Q + k], v2[m], o);
      U[k] = o;
    }
  }
}

// i-lines: D_1^T on G0 plus U + G1, then stage p of B^T -> Gp in U
template <int SH, int P>
__device__ void ipr_p_d1t(const Tile_<SH, P>& T, int ne) {
  using D = Dims<SH, P>;
  constexpr int Q = D::Q, n = D::n, QP = D::QP;
  for (int t = tid(); t < ne * Q * Q; t += nthr()) {
    const ctab_t A1 = launder(T.ct) + D::L.A1;
    const ctab_t D1 = launder(T.ct) + D::L.D;
    const int e = t / (Q * Q);
    const int rem = t - e * (Q * Q);
    const int j = rem / Q, k = rem - j * Q;
    const int o = j * QP + k;
    const double* G0 = T.G(e, 0) + o;
    const double* G1 = T.G(e, 1) + o;
    double* U = T.U(e) + o;
    double g0[Q];
#pragma unroll
    for (int l = 0; l < Q; ++l) g0[l] = G0[l * Q * QP];
    double sv[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      double s = U[i * Q * QP] + G1[i * Q * QP];
#pragma unroll
      for (int l = 0; l < Q; ++l) s = fma(D1[l * Q + i], g0[l], s);
      sv[i] = s;
    }
#pragma unroll
    for (int p = 0; p < n; ++p) {
      double a = 0.0;
#pragma unroll
      for (int i = 0; i < Q; ++i) a = fma(A1[p * Q + i], sv[i], a);
      U[p * Q * QP] = a;
    }
  }
}

template <int SH, int P, int OP, bool PF>
__device__ void helm_fused_tile(const OpArgs& a, long long e0, int ne, const Tile_<SH, P>& T, bool tables) {
  using D = Dims<SH, P>;
  constexpr int Q = D::Q, Q3 = D::Q3;
  const gptr_t fac_tile = as_global(a.fac) + e0 * (long long)(NFAC * Q3);
  GeoLine<Q> gpf;
  if (PF) {
    const int t = tid();
    if (t < ne * Q * Q) {
      const int e = t / (Q * Q);
      const int rem = t - e * (Q * Q);
      load_geo_line<P>(fac_tile, e, rem / Q, rem - (rem / Q) * Q, gpf);
    }
  }
  if (tables) load_tables<SH, P>(a, T);
  load_modes<SH, P>(T, a.in, e0, ne, 0);
  __syncthreads();
  bwd_r<SH, P, false>(T, ne, 0, 1);  // modes in G0 -> F in G1
  __syncthreads();
  bwd_q<SH, P, false>(T, ne, 1, -1);  // F -> Gq in U
  __syncthreads();
  bwd_p_d1<SH, P>(T, ne);
  __syncthreads();
  d2_lines<SH, P, false>(T, ne);
  __syncthreads();
  kline_metric<SH, P, OP, PF>(T, ne, fac_tile, (OP == OPK_HELM) ? a.lambda : 0.0, gpf);
  __syncthreads();
  d2_lines<SH, P, true>(T, ne);
  __syncthreads();
  ipr_p_d1t<SH, P>(T, ne);
  __syncthreads();
  ipr_q<SH, P, false>(T, ne, -1, 0);  // Gp in U -> F in G0
  __syncthreads();
  ipr_r<SH, P, false>(T, ne, 0, 1, false);  // -> modes in G1
  __syncthreads();
  store_modes<SH, P>(T, a.out, e0, ne, 1);
}

template <int SH, int P, int OP, bool PF>
__global__ void __launch_bounds__(512) k_helm_fused(OpArgs a) {
  extern __shared__ double smem[];
  const long long e0 = (long long)blockIdx.x * a.E;
  const long long rem = a.n_elem - e0;
  const int ne = rem < a.E ? (int)rem : a.E;
  if (ne <= 0) return;
  helm_fused_tile<SH, P, OP, PF>(a, e0, ne, make_tile3<SH, P>(smem, a.tab), true);
}

template <int P, int OP, bool PF>
__global__ void __launch_bounds__(512) k_helm_fused_mixed(const BlockStatic* __restrict__ blocks,
                                                          const Tile* __restrict__ tiles, int ntiles,
                                                          const double* in, double* out, double lambda) {
  extern __shared__ double smem[];
  const int ti = blockIdx.x;
  if (ti >= ntiles) return;
  const Tile tl = tiles[ti];
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
  switch (b.shape) {
    case HEX: helm_fused_tile<HEX, P, OP, PF>(a, tl.e0, tl.ne, make_tile3<HEX, P>(smem, a.tab), true); break;
    case PRISM: helm_fused_tile<PRISM, P, OP, PF>(a, tl.e0, tl.ne, make_tile3<PRISM, P>(smem, a.tab), true); break;
    case PYR: helm_fused_tile<PYR, P, OP, PF>(a, tl.e0, tl.ne, make_tile3<PYR, P>(smem, a.tab), true); break;
    default: helm_fused_tile<TET, P, OP, PF>(a, tl.e0, tl.ne, make_tile3<TET, P>(smem, a.tab), true); break;
  }
}

template <int SH, int P>
constexpr size_t lds_bytes3(int E) {
  using D = Dims<SH, P>;
  return sizeof(double) * (size_t)(D::HEAD + E * 3 * D::S3);
}

// ---------------------------------------------------------------------------
// Non-collocated Laplacian / Helmholtz (Alg. 5): sum-factorised B and d_d B
// ---------------------------------------------------------------------------
// u = B x and v_d = (d_d B) x share a tree of 1D stages (tables A/dA in eta1,
// B2/dB2 in eta2, C3/dC3 in eta3); after the metric the transposed tree sums
// the table pairs:  y = C3^T[B2^T(A^T(lam W u) + dA^T v_1') + dB2^T A^T v_2']
//                     + dC3^T B2^T A^T v_3'.
// Five LDS buffers per element (U = B0, G(0..3) = B1..B4).

template <int SH, int P>
__device__ Tile_<SH, P> make_tile5(double* smem, const double* gtab) {
  Tile_<SH, P> T = make_tile<SH, P>(smem, gtab);
  T.per = 5 * Dims<SH, P>::S3;
  return T;
}

__device__ __forceinline__ int bufidx(int b) { return b - 1; }  // B0 -> -1 (U), Bk -> G(k-1)

// stage p of B: Gu (p rows, in buffer src) -> u in place and v_1 = dA rows into dst1
template <int SH, int P>
__device__ void nc_bwd_p_uv(const Tile_<SH, P>& T, int ne, int src, int dst1) {
  using D = Dims<SH, P>;
  constexpr int Q = D::Q, n = D::n, QP = D::QP;
  for (int t = tid(); t < ne * Q * Q; t += nthr()) {
    const ctab_t A1 = launder(T.ct) + D::L.A1;
    const ctab_t dA1 = launder(T.ct) + D::L.dA1;
    const int e = t / (Q * Q);
    const int rem = t - e * (Q * Q);
    const int j = rem / Q, k = rem - j * Q;
    double* S = (src < 0 ? T.U(e) : T.G(e, src)) + j * QP + k;
    double* V = T.G(e, dst1) + j * QP + k;
    double g[n];
#pragma unroll
    for (int p = 0; p < n; ++p) g[p] = S[p * Q * QP];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      double a = 0.0, b = 0.0;
#pragma unroll
      for (int p = 0; p < n; ++p) {
        a = fma(A1[p * Q + i], g[p], a);
        b = fma(dA1[p * Q + i], g[p], b);
      }
      S[i * Q * QP] = a;
      V[i * Q * QP] = b;
    }
  }
}

// stage p of B^T with two inputs: dst <- A^T(a) (+ dA^T(b) when b >= -1); in place over a
template <int SH, int P, bool TWO>
__device__ void nc_ipr_p(const Tile_<SH, P>& T, int ne, int a_buf, int b_buf) {
  using D = Dims<SH, P>;
  constexpr int Q = D::Q, n = D::n, QP = D::QP;
  for (int t = tid(); t < ne * Q * Q; t += nthr()) {
    const ctab_t A1 = launder(T.ct) + D::L.A1;
    const ctab_t dA1 = launder(T.ct) + D::L.dA1;
    const int e = t / (Q * Q);
    const int rem = t - e * (Q * Q);
    const int j = rem / Q, k = rem - j * Q;
    double* Ab = (a_buf < 0 ? T.U(e) : T.G(e, a_buf)) + j * QP + k;
    double sa[Q], sb[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) sa[i] = Ab[i * Q * QP];
    if (TWO) {
      const double* Bb = (b_buf < 0 ? T.U(e) : T.G(e, b_buf)) + j * QP + k;
#pragma unroll
      for (int i = 0; i < Q; ++i) sb[i] = Bb[i * Q * QP];
    }
#pragma unroll
    for (int p = 0; p < n; ++p) {
      double acc = 0.0;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        acc = fma(A1[p * Q + i], sa[i], acc);
        if (TWO) acc = fma(dA1[p * Q + i], sb[i], acc);
      }
      Ab[p * Q * QP] = acc;
    }
  }
}

// stage q of B^T with up to two inputs: F (dst) <- B2^T(a) [+ dB2^T(b)]
template <int SH, int P, bool TWO>
__device__ void nc_ipr_q(const Tile_<SH, P>& T, int ne, int a_buf, int b_buf, int dst) {
  using D = Dims<SH, P>;
  constexpr int Q = D::Q, n = D::n, QP = D::QP;
  for (int t = tid(); t < ne * n * Q; t += nthr()) {
    const int e = t / (n * Q);
    const int rem = t - e * (n * Q);
    const int p = rem / Q, k = rem - p * Q;
    const double* GA = (a_buf < 0 ? T.U(e) : T.G(e, a_buf)) + p * Q * QP + k;
    const double* GB = (b_buf < 0 ? T.U(e) : T.G(e, b_buf)) + p * Q * QP + k;
    double ga[Q], gb[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) ga[j] = GA[j * QP];
    if (TWO) {
#pragma unroll
      for (int j = 0; j < Q; ++j) gb[j] = GB[j * QP];
    }
    double* F = T.G(e, dst);
    const int nq = nq_of(SH, P, p), cb = col_base(SH, P, p);
    const int bfam = (SH == TET) ? fam_index(P, p, 0) : 0;
    const double* B2 = T.tab + D::L.B2;
    const double* dB2 = T.tab + D::L.dB2;
    for (int q = 0; q < nq; ++q) {
      double acc = 0.0;
      const double* b = B2 + (bfam + q) * Q;
      const double* db = dB2 + (bfam + q) * Q;
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        acc = fma(b[j], ga[j], acc);
        if (TWO) acc = fma(db[j], gb[j], acc);
      }
      if (SH == TET && p == 0 && q == 1) {
        // adjoints of the tet's extra eta2 term, one per (table, input) pair
        const double* GA1 = GA + 1 * Q * QP;
        const double* GB1 = GB + 1 * Q * QP;
#pragma unroll
        for (int j = 0; j < Q; ++j) {
          acc = fma(B2[1 * Q + j], GA1[j * QP], acc);
          if (TWO) acc = fma(dB2[1 * Q + j], GB1[j * QP], acc);
        }
      }
      F[(cb + q) * QP + k] = acc;
    }
  }
}

// stage r of B^T with two inputs: y (dst) <- C3^T(Fa) + dC3^T(Fb)
template <int SH, int P>
__device__ void nc_ipr_r(const Tile_<SH, P>& T, int ne, int fa, int fb_buf, int dst) {
  using D = Dims<SH, P>;
  constexpr int Q = D::Q, QP = D::QP;
  const double* C3 = T.tab + D::L.C3;
  const double* dC3 = T.tab + D::L.dC3;
  for (int t = tid(); t < ne * D::NC; t += nthr()) {
    const int e = t / D::NC, c = t - e * D::NC;
    const int* ct = T.itab + c * ICOL;
    const int p = ct[0], q = ct[1], off = ct[2], RL = ct[3], fam = ct[4];
    const double* FA = T.G(e, fa);
    const double* FB = T.G(e, fb_buf);
    double f[Q], g[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      f[k] = FA[c * QP + k];
      g[k] = FB[c * QP + k];
    }
    double* y = (dst < 0 ? T.U(e) : T.G(e, dst)) + off;
    for (int r = 0; r < RL; ++r) {
      const double* cf = C3 + (fam + r) * Q;
      const double* dcf = dC3 + (fam + r) * Q;
      double a = 0.0;
#pragma unroll
      for (int k = 0; k < Q; ++k) a = fma(cf[k], f[k], fma(dcf[k], g[k], a));
      const bool vx = (r == 1) && ((SH == PRISM && p == 0) || ((SH == PYR || SH == TET) && p == 0 && q == 0));
      if (vx) {
        // the collapsed-vertex splits, adjoint per (table, input) pair
        int cols[3];
        int nc = 0;
        if (SH == PRISM) {
          cols[nc++] = (P + 1) + q;
        } else if (SH == PYR) {
          cols[nc++] = P + 1;
          cols[nc++] = 1;
          cols[nc++] = P + 2;
        } else {
          cols[nc++] = 1;
          cols[nc++] = P + 1;
        }
        for (int u = 0; u < nc; ++u) {
#pragma unroll
          for (int k = 0; k < Q; ++k)
            a = fma(C3[1 * Q + k], FA[cols[u] * QP + k], fma(dC3[1 * Q + k], FB[cols[u] * QP + k], a));
        }
      }
      y[r] = a;
    }
  }
}

template <int SH, int P, int OP>
__device__ void helm_nc_tile(const OpArgs& a, long long e0, int ne, const Tile_<SH, P>& T) {
  using D = Dims<SH, P>;
  constexpr int Q3 = D::Q3;
  load_tables<SH, P>(a, T);
  load_modes<SH, P>(T, a.in, e0, ne, 3);  // x in B4
  __syncthreads();
  bwd_r<SH, P, false>(T, ne, 3, 0);  // F  (C3)  -> B1
  bwd_r<SH, P, true>(T, ne, 3, 1);   // F' (dC3) -> B2
  __syncthreads();
  bwd_q<SH, P, false>(T, ne, 0, -1);  // Gu  = B2 F   -> B0
  bwd_q<SH, P, true>(T, ne, 0, 2);    // G2' = dB2 F  -> B3
  bwd_q<SH, P, false>(T, ne, 1, 3);   // G3' = B2 F'  -> B4
  __syncthreads();
  nc_bwd_p_uv<SH, P>(T, ne, -1, 0);   // u -> B0, v_1 -> B1
  bwd_p<SH, P, false>(T, ne, 2, 2);   // v_2 -> B3 (in place)
  bwd_p<SH, P, false>(T, ne, 3, 3);   // v_3 -> B4 (in place)
  __syncthreads();
  const gptr_t fac = as_global(a.fac) + e0 * (long long)(NFAC * Q3);
  const double lam = (OP == OPK_HELM) ? a.lambda : 0.0;
  for (int t = tid(); t < ne * Q3; t += nthr()) {
    const int e = t / Q3, pt = t - e * Q3;
    const int lp = lds_pt<SH, P>(pt);
    const gptr_t g = fac + e * (NFAC * Q3) + pt;
    double* u = T.U(e) + lp;
    double* p1 = T.G(e, 0) + lp;
    double* p2 = T.G(e, 2) + lp;
    double* p3 = T.G(e, 3) + lp;
    const double d0 = *p1, d1 = *p2, d2 = *p3;
    const double jw = g[0];
    const double g00 = g[1 * Q3], g01 = g[2 * Q3], g02 = g[3 * Q3];
    const double g11 = g[4 * Q3], g12 = g[5 * Q3], g22 = g[6 * Q3];
    *p1 = g00 * d0 + g01 * d1 + g02 * d2;
    *p2 = g01 * d0 + g11 * d1 + g12 * d2;
    *p3 = g02 * d0 + g12 * d1 + g22 * d2;
    *u = lam * jw * (*u);
  }
  __syncthreads();
  nc_ipr_p<SH, P, true>(T, ne, -1, 0);  // Hu = A^T(lam W u) + dA^T v_1' -> B0
  nc_ipr_p<SH, P, false>(T, ne, 2, 0);  // H2 = A^T v_2' -> B3
  nc_ipr_p<SH, P, false>(T, ne, 3, 0);  // H3 = A^T v_3' -> B4
  __syncthreads();
  nc_ipr_q<SH, P, true>(T, ne, -1, 2, 0);  // K  = B2^T Hu + dB2^T H2 -> B1
  nc_ipr_q<SH, P, false>(T, ne, 3, 3, 1);  // K3 = B2^T H3           -> B2
  __syncthreads();
  nc_ipr_r<SH, P>(T, ne, 0, 1, -1);  // y = C3^T K + dC3^T K3 -> B0
  __syncthreads();
  store_modes<SH, P>(T, a.out, e0, ne, -1);
}

template <int SH, int P, int OP>
__global__ void __launch_bounds__(512) k_helm_nc(OpArgs a) {
  extern __shared__ double smem[];
  const long long e0 = (long long)blockIdx.x * a.E;
  const long long rem = a.n_elem - e0;
  const int ne = rem < a.E ? (int)rem : a.E;
  if (ne <= 0) return;
  helm_nc_tile<SH, P, OP>(a, e0, ne, make_tile5<SH, P>(smem, a.tab));
}

template <int P, int OP>
__global__ void __launch_bounds__(512) k_helm_nc_mixed(const BlockStatic* __restrict__ blocks,
                                                       const Tile* __restrict__ tiles, int ntiles, const double* in,
                                                       double* out, double lambda) {
  extern __shared__ double smem[];
  const int ti = blockIdx.x;
  if (ti >= ntiles) return;
  const Tile tl = tiles[ti];
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
  switch (b.shape) {
    case HEX: helm_nc_tile<HEX, P, OP>(a, tl.e0, tl.ne, make_tile5<HEX, P>(smem, a.tab)); break;
    case PRISM: helm_nc_tile<PRISM, P, OP>(a, tl.e0, tl.ne, make_tile5<PRISM, P>(smem, a.tab)); break;
    case PYR: helm_nc_tile<PYR, P, OP>(a, tl.e0, tl.ne, make_tile5<PYR, P>(smem, a.tab)); break;
    default: helm_nc_tile<TET, P, OP>(a, tl.e0, tl.ne, make_tile5<TET, P>(smem, a.tab)); break;
  }
}

template <int SH, int P>
constexpr size_t lds_bytes5(int E) {
  using D = Dims<SH, P>;
  return sizeof(double) * (size_t)(D::HEAD + E * 5 * D::S3);
}

// LDS bytes of a tile of E elements
template <int SH, int P>
constexpr size_t lds_bytes(int E) {
  using D = Dims<SH, P>;
  return sizeof(double) * (size_t)(D::HEAD + E * D::PER_ELEM);
}

}  // namespace shp
