// C ABI of libshp (declared in include/shp.h): plans, workspace layout,
// validation, geometry setup and operator dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/shp.h"
#include "shp_kernels.hpp"
#include "shp_kernels_geom.hpp"
#include "shp_kernels_lm.hpp"
#include "shp_kernels_iso.hpp"
#include "shp_kernels_2d.hpp"

using namespace shp;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int dev_fail(hipError_t e, const char* what) {
  return fail(SHP_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

constexpr size_t ALIGN = 256;
constexpr int MLP_NIN = 11;           // cost-model features (shp_mlp_* in shp_mlp.hip)
constexpr int MODEL_MAX_MEMBERS = 4;  // networks averaged by a loaded cost model
size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

struct Tiling {
  int E = 0;
  int NT = 0;
  int persist = 2;  // Laplacian/Helmholtz launch variant: 0 plain, 1 persistent + prefetch, 2 prefetch per tile
};

struct Block {
  shp_block_desc d{};
  int NP = 0, NQ = 0;
  std::vector<double> tab;
  std::vector<int> itab;
  size_t off_tab = 0, off_itab = 0, off_fac = 0, off_dxi = 0, off_lm = 0, off_tabf = 0;
  std::vector<double> lm;  // [B; d_d B] for the local-matrix strategy (P <= 4)
  std::vector<double> dm;  // dense collocation derivatives, each transposed: [3][Q3p in][Q3p out] (local-matrix PhysDeriv)
  size_t off_dm = 0;
  std::vector<double> bt;  // [B; d_d B] transposed, [Kp][4 Q3p] (local-matrix U = B X products)
  size_t off_bt = 0;
  std::vector<double> am;  // affine blocks: 7 reference matrices, MFMA fragment order
  size_t off_am = 0, off_coef = 0;
  std::vector<uint16_t> am16;  // the same as BF16 parts, BF16 MFMA fragment order
  size_t off_am16 = 0;
  std::vector<float> am32;     // the FP64 fragments rounded to FP32 (FP32 MFMA)
  size_t off_am32 = 0;
  std::vector<float> tabf; // the reference tables rounded to FP32
  std::vector<double> dtab; // sum-factorised Helmholtz diagonal: 1D factor tables
  std::vector<int> ditab;   //   and their pair and mode indices
  int dn1 = 0, dn12 = 0;
  size_t off_dtab = 0, off_ditab = 0;
  std::vector<double> wref; // iso-parametric blocks: reference weights [Q^3]
  size_t off_xco = 0, off_wref = 0;
  bool iso() const { return d.geom == SHP_ISOPARAM; }
  long long coeff_off = 0, phys_off = 0;
  bool geom_ok = false;
  Tiling tiling[OPK_COUNT];
  int auto_strategy[7] = {2, 2, 2, 2, 2, 2, 2};  // per public operator, used by SHP_AUTO
  int auto_src[7] = {};  // where auto_strategy came from: 0 default, 1 tuned or set, 2 cost model
  struct Tuned {
    bool valid = false;
    int strategy = 2, E = 0, NT = 0, variant = 0;
    double ms = 0.0;
  } tuned[7];
};

}  // namespace

struct shp_plan_s {
  std::vector<Block> blocks;
  size_t ws_bytes = 0;
  char* ws = nullptr;
  float* fac32 = nullptr;  // caller's FP32 copy of the factors for the FP32 actions, or null
  size_t off_status = 0, off_bstat = 0, off_tiles = 0;
  long long total_elem = 0, total_coeff = 0, total_phys = 0;
  long long max_tiles = 0;  // tile slots reserved per operator
  Tiling mixed[OPK_COUNT];
  int mixed_ntiles[OPK_COUNT] = {};
  bool mixed_dirty[OPK_COUNT] = {};
  bool uniform_P = true;
  int auto_mixed[7] = {2, 2, 2, 2, 2, 2, 2};
  int auto_mixed_src[7] = {};  // 0 default, 1 tuned or set
  Block::Tuned tuned_mixed[7];
  // cost model in the workspace: parameters [MODEL_MAX_MEMBERS][nparam], then
  // features [3][nin], per-sample work [3][work floats], predictions [members][3]
  size_t off_model = 0;
  int model_members = 0;
  double model_mu = 0.0, model_sigma = 1.0;  // prediction = exp(mu + sigma * score) seconds per DOF
  int mlp_nparam = 0;
  long long mlp_work = 0;
};

namespace {

bool valid_shape(int s) { return s >= SHP_HEX && s <= SHP_TRI; }

int opk_of(int op, int strategy, int* opk) {
  if (strategy < SHP_AUTO || strategy > SHP_LOCALMAT) return fail(SHP_ERR_INVALID_ARG, "bad strategy %d", strategy);
  if (strategy == SHP_LOCALMAT) {
    switch (op) {
      case SHP_OP_BWDTRANS: *opk = OPK_BWD_LM; return SHP_OK;
      case SHP_OP_IPRODUCT: *opk = OPK_IPR_LM; return SHP_OK;
      case SHP_OP_PHYSDERIV: *opk = OPK_DERIV_LM; return SHP_OK;
      case SHP_OP_IPRODUCT_DERIV: *opk = OPK_IPRD_LM; return SHP_OK;
      case SHP_OP_MASS: *opk = OPK_MASS_LM; return SHP_OK;
      case SHP_OP_LAPLACIAN: *opk = OPK_LAP_LM; return SHP_OK;
      case SHP_OP_HELMHOLTZ: *opk = OPK_HELM_LM; return SHP_OK;
    }
    return fail(SHP_ERR_INVALID_ARG, "bad operator %d", op);
  }
  switch (op) {
    case SHP_OP_BWDTRANS: *opk = OPK_BWD; return SHP_OK;
    case SHP_OP_IPRODUCT: *opk = OPK_IPR; return SHP_OK;
    case SHP_OP_PHYSDERIV: *opk = OPK_DERIV; return SHP_OK;
    case SHP_OP_IPRODUCT_DERIV: *opk = OPK_IPRD; return SHP_OK;
    case SHP_OP_MASS: *opk = OPK_MASS; return SHP_OK;
    case SHP_OP_LAPLACIAN:
    case SHP_OP_HELMHOLTZ:
      if (strategy == SHP_SUMFAC)
        *opk = (op == SHP_OP_LAPLACIAN) ? OPK_LAP_NC : OPK_HELM_NC;
      else
        *opk = (op == SHP_OP_LAPLACIAN) ? OPK_LAP : OPK_HELM;
      return SHP_OK;
  }
  return fail(SHP_ERR_INVALID_ARG, "bad operator %d", op);
}

bool is_xform_lm(int opk) { return opk >= OPK_BWD_LM && opk <= OPK_IPRD_LM; }
bool is_localmat(int opk) { return (opk >= OPK_MASS_LM && opk <= OPK_HELM_LM) || is_xform_lm(opk); }
bool in_is_modes(int opk) {
  return opk == OPK_BWD || opk == OPK_MASS || opk == OPK_LAP || opk == OPK_HELM || opk == OPK_HELM_NC ||
         opk == OPK_LAP_NC || (opk >= OPK_MASS_LM && opk <= OPK_HELM_LM) || opk == OPK_BWD_LM;
}
bool out_is_modes(int opk) { return !(opk == OPK_BWD || opk == OPK_DERIV || opk == OPK_BWD_LM || opk == OPK_DERIV_LM); }

// Default launch shape: as many elements per work-group as fit an LDS budget
// (at most 16; several work-groups share a CU), 256 threads, and for the
// Laplacian and Helmholtz actions the geometry-prefetch launch with at most 4
// points per thread (8 register slots of 7 factors cost occupancy).  The
// budget is 40 KiB; the whole-mesh Laplacian and Helmholtz launch raises it to
// 64 KiB where 40 KiB leaves at most 2 points per thread, which happens at
// P = 6 (8^3 points): two elements per work-group there take 0.95 ms per FP64
// action on the 32^3-cell mixed mesh against 1.21 ms for one.
// From P = 7 on (729 or more points per element) the Laplacian / Helmholtz
// launches take the shapes the tuner measured fastest on the 32^3-cell mixed
// mesh's blocks (FP64, HIP events after a cache flush): mostly 512 threads, so
// that 4 geometry slots per thread hold the tile's points, and two elements
// per work-group at P = 7 and 8.  Per shape (hex, prism, pyramid, tet) and
// P = 7..10: elements per work-group, threads.
constexpr int HI_E[4][4] = {{1, 2, 1, 1}, {2, 2, 1, 1}, {2, 2, 1, 1}, {2, 1, 1, 1}};
constexpr int HI_NT[4][4] = {{256, 512, 512, 512}, {512, 512, 512, 512}, {512, 512, 512, 512}, {512, 256, 512, 512}};
// the whole-mesh launch at P = 7..10 (one launch shape for every block)
constexpr int HI_MESH_E[4] = {2, 1, 1, 1};
constexpr int HI_MESH_NT[4] = {512, 256, 512, 512};

Tiling default_tiling(int sh, int P, int opk, size_t lds_budget = 40 * 1024) {
  Tiling t;
  t.NT = 256;
  const bool helm = (opk == OPK_HELM || opk == OPK_LAP || opk == OPK_ADR);
  const long long Q3 = (long long)(P + 2) * (P + 2) * (P + 2);
  if (is_2d(sh)) {
    const int Q = P + 2;
    int E = 1;
    if (opk == OPK_HELM || opk == OPK_LAP) {
      // the fused tile: the tile's points in at most 8 register slots per
      // thread and at most 32 KiB of LDS (a sweep of elements x threads on
      // the 2D mesh at P = 2, 4, 8 puts this within 3 % of the fastest shape)
      while (E < 64 && (E + 1) * Q * Q <= 8 * t.NT && lds_bytes_2d(sh, P, E + 1, opk, t.NT) <= 32 * 1024) ++E;
    } else {
      // enough elements that a stage has about two line tasks per thread
      while (E < 64 && lds_bytes_2d(sh, P, E + 1) <= 48 * 1024 && (E + 1) * Q <= 2 * t.NT) ++E;
    }
    t.E = E;
    t.persist = 0;
    return t;
  }
  if (opk == OPK_BWD || opk == OPK_IPR || opk == OPK_DERIV || opk == OPK_IPRD || opk == OPK_MASS) {
    // the plain collocated tile is bound by the latency of its staged line
    // stages: about 1500 points per work-group, 512 threads from 768 points
    // (the tuner's choices for these operators on the 32^3-cell mixed mesh
    // at P = 2, 4, 6 were 640-960, 1512 and 2048 points)
    int E = std::max(1, std::min(12, (int)((1536 + Q3 / 2) / Q3)));
    while (E > 1 && op_lds_bytes(sh, P, opk, E, 2) > 64 * 1024) --E;
    t.E = E;
    t.NT = E * Q3 > 768 ? 512 : 256;
    t.persist = 0;
    return t;
  }
  if (helm && P >= 7) {
    t.E = HI_E[sh][P - 7];
    t.NT = HI_NT[sh][P - 7];
    t.persist = points_per_thread((long long)t.E * Q3, t.NT) > 0 ? 2 : 0;
    return t;
  }
  int E = 1;
  while (E < 16 && op_lds_bytes(sh, P, opk, E + 1, 2) <= lds_budget && (!helm || (E + 1) * Q3 <= 4LL * t.NT)) ++E;
  t.E = E;
  t.persist = points_per_thread((long long)E * (P + 2) * (P + 2) * (P + 2), t.NT) > 0 ? 2 : 0;
  return t;
}

// Iso-parametric launches keep 9 FP64 derivatives per owned point in
// registers while they rebuild the geometry, so they own at most 2 points per
// thread (4 from P = 9, where one element has more than 1024 points): as many
// elements as fill 512 points on 256 threads, else one element on 512.
Tiling iso_tiling(int P) {
  const int Q3 = (P + 2) * (P + 2) * (P + 2);
  Tiling t;
  t.E = std::max(1, std::min(16, 512 / Q3));
  t.NT = (t.E * Q3 <= 512) ? 256 : 512;
  t.persist = 2;
  return t;
}

Tiling effective(const Tiling& set, int sh, int P, int opk) {
  if (opk == OPK_HELM_ISO || opk == OPK_LAP_ISO) return iso_tiling(P);
  return (set.E > 0 && set.NT > 0) ? set : default_tiling(sh, P, opk);
}

int check_plan(shp_plan p) {
  if (!p) return fail(SHP_ERR_INVALID_ARG, "null plan");
  return SHP_OK;
}

}  // namespace

extern "C" {

const char* shp_last_error(void) { return g_err.c_str(); }

int shp_num_modes(int shape, int P, int* n) {
  if (!n) return fail(SHP_ERR_INVALID_ARG, "null output");
  if (!valid_shape(shape)) return fail(SHP_ERR_INVALID_ARG, "bad shape %d", shape);
  if (P < 1 || P > MAX_P) return fail(SHP_ERR_UNSUPPORTED, "P=%d outside [1,%d]", P, MAX_P);
  *n = is_2d(shape) ? num_modes2(shape, P) : num_modes(shape, P);
  return SHP_OK;
}

int shp_num_points(int shape, int Q, int* n) {
  if (!n) return fail(SHP_ERR_INVALID_ARG, "null output");
  if (!valid_shape(shape)) return fail(SHP_ERR_INVALID_ARG, "bad shape %d", shape);
  if (Q < 3 || Q > MAX_P + 2) return fail(SHP_ERR_UNSUPPORTED, "Q=%d outside [3,%d]", Q, MAX_P + 2);
  *n = is_2d(shape) ? Q * Q : Q * Q * Q;
  return SHP_OK;
}

int shp_vertex_modes(int shape, int P, int* idx, double* xi, int* n_vertices) {
  if (!idx || !xi || !n_vertices) return fail(SHP_ERR_INVALID_ARG, "null output");
  if (!valid_shape(shape) || is_2d(shape)) return fail(SHP_ERR_INVALID_ARG, "bad shape %d", shape);
  if (P < 1 || P > MAX_P) return fail(SHP_ERR_UNSUPPORTED, "P=%d outside [1,%d]", P, MAX_P);
  // (p, q, r) of each vertex mode and the reference vertex where it is one
  struct V {
    int p, q, r;
    double x, y, z;
  };
  std::vector<V> vs;
  if (shape == SHP_HEX) {
    for (int p = 0; p < 2; ++p)
      for (int q = 0; q < 2; ++q)
        for (int r = 0; r < 2; ++r) vs.push_back({p, q, r, 2.0 * p - 1, 2.0 * q - 1, 2.0 * r - 1});
  } else if (shape == SHP_TET) {
    vs = {{0, 0, 0, -1, -1, -1}, {1, 0, 0, 1, -1, -1}, {0, 1, 0, -1, 1, -1}, {0, 0, 1, -1, -1, 1}};
  } else {
    for (int p = 0; p < 2; ++p)
      for (int q = 0; q < 2; ++q) vs.push_back({p, q, 0, 2.0 * p - 1, 2.0 * q - 1, -1});
    vs.push_back({0, 0, 1, -1, -1, 1});
    if (shape == SHP_PRISM) vs.push_back({0, 1, 1, -1, 1, 1});
  }
  for (size_t v = 0; v < vs.size(); ++v) {
    int off = 0;  // modes before column (p, q): columns are p-major, then q
    for (int p = 0; p < vs[v].p; ++p)
      for (int q = 0; q < nq_of(shape, P, p); ++q) off += col_len(shape, P, p, q);
    for (int q = 0; q < vs[v].q; ++q) off += col_len(shape, P, vs[v].p, q);
    idx[v] = off + vs[v].r;
    xi[3 * v + 0] = vs[v].x;
    xi[3 * v + 1] = vs[v].y;
    xi[3 * v + 2] = vs[v].z;
  }
  *n_vertices = (int)vs.size();
  return SHP_OK;
}

int shp_quadrature(int shape, int Q, int pts, double* xi, double* w) {
  if (!xi) return fail(SHP_ERR_INVALID_ARG, "null xi");
  if (!valid_shape(shape)) return fail(SHP_ERR_INVALID_ARG, "bad shape %d", shape);
  if (pts != SHP_PTS_GJ && pts != SHP_PTS_RADAU) return fail(SHP_ERR_INVALID_ARG, "bad point set %d", pts);
  if (Q < 3 || Q > MAX_P + 2) return fail(SHP_ERR_UNSUPPORTED, "Q=%d outside [3,%d]", Q, MAX_P + 2);
  if (is_2d(shape))
    reference_points2d(shape, Q, pts, xi, w);
  else
    reference_points(shape, Q, pts, xi, w);
  return SHP_OK;
}

int shp_plan_create(shp_plan* out, const shp_block_desc* blk, int nblk) {
  if (!out || !blk) return fail(SHP_ERR_INVALID_ARG, "null argument");
  if (nblk < 1 || nblk > 64) return fail(SHP_ERR_INVALID_ARG, "nblk=%d outside [1,64]", nblk);
  for (int b = 0; b < nblk; ++b) {
    const shp_block_desc& d = blk[b];
    if (!valid_shape(d.shape)) return fail(SHP_ERR_INVALID_ARG, "block %d: bad shape %d", b, d.shape);
    if (d.P < 1 || d.P > MAX_P) return fail(SHP_ERR_UNSUPPORTED, "block %d: P=%d outside [1,%d]", b, d.P, MAX_P);
    if (d.Q != d.P + 2) return fail(SHP_ERR_UNSUPPORTED, "block %d: Q=%d, only Q=P+2 is built", b, d.Q);
    if (d.n_elem < 0 || d.n_elem > (1LL << 31)) return fail(SHP_ERR_INVALID_ARG, "block %d: n_elem=%lld", b, (long long)d.n_elem);
    if (d.geom != SHP_AFFINE && d.geom != SHP_CURVED && d.geom != SHP_ISOPARAM)
      return fail(SHP_ERR_INVALID_ARG, "block %d: bad geom %d", b, d.geom);
    if (d.pts != SHP_PTS_GJ && d.pts != SHP_PTS_RADAU) return fail(SHP_ERR_INVALID_ARG, "block %d: bad point set %d", b, d.pts);
  }
  for (int b = 1; b < nblk; ++b)
    if (is_2d(blk[b].shape) != is_2d(blk[0].shape))
      return fail(SHP_ERR_INVALID_ARG, "block %d: a plan holds 2D or 3D shapes, not both", b);
  for (int b = 0; b < nblk; ++b)
    if (is_2d(blk[b].shape) && blk[b].geom == SHP_ISOPARAM)
      return fail(SHP_ERR_UNSUPPORTED, "block %d: iso-parametric 2D blocks are not built", b);
  shp_plan p = new (std::nothrow) shp_plan_s;
  if (!p) return fail(SHP_ERR_INVALID_ARG, "out of host memory");
  p->blocks.resize(nblk);
  size_t off = 0;
  p->off_status = off;
  off = align_up(off + 256);
  p->off_bstat = off;
  off = align_up(off + sizeof(BlockStatic) * nblk);
  long long cofs = 0, pofs = 0;
  for (int b = 0; b < nblk; ++b) {
    Block& B = p->blocks[b];
    B.d = blk[b];
    if (is_2d(B.d.shape)) {
      // 2D: the tables only (the solve, tuning and local matrices are 3D)
      B.NP = num_modes2(B.d.shape, B.d.P);
      B.NQ = B.d.Q * B.d.Q;
      build_tables2d(B.d.shape, B.d.P, B.d.pts, B.tab);
      B.coeff_off = cofs;
      B.phys_off = pofs;
      cofs += B.d.n_elem * B.NP;
      pofs += B.d.n_elem * B.NQ;
      p->total_elem += B.d.n_elem;
      if (B.d.P != blk[0].P) p->uniform_P = false;
      continue;
    }
    B.NP = num_modes(B.d.shape, B.d.P);
    B.NQ = B.d.Q * B.d.Q * B.d.Q;
    build_tables(B.d.shape, B.d.P, B.d.pts, B.tab, B.itab);
    build_diag_tables(B.d.shape, B.d.P, B.d.pts, B.dtab, B.ditab, B.dn1, B.dn12);
    if (B.iso()) build_ref_weights(B.d.shape, B.d.P, B.d.pts, B.wref);
    if (B.d.P <= LOCALMAT_MAX_P && !B.iso()) {
      int q3p, kp;
      build_localmat(B.d.shape, B.d.P, B.d.pts, B.lm, q3p, kp);
      build_dense_deriv(B.d.shape, B.d.P, B.d.pts, B.dm, q3p);
      // the products U = B X (BwdTrans, the curved local matrices) and
      // PhysDeriv read their matrices with the output point fastest across
      // lanes: store [B; d_d B] and each D_d transposed as well
      B.bt.assign((size_t)kp * 4 * q3p, 0.0);
      for (int r = 0; r < 4 * q3p; ++r)
        for (int m = 0; m < kp; ++m) B.bt[(size_t)m * 4 * q3p + r] = B.lm[(size_t)r * kp + m];
      for (int d = 0; d < 3; ++d) {
        double* D = B.dm.data() + (size_t)d * q3p * q3p;
        for (int i = 0; i < q3p; ++i)
          for (int j = i + 1; j < q3p; ++j) std::swap(D[(size_t)i * q3p + j], D[(size_t)j * q3p + i]);
      }
      if (B.d.geom == SHP_AFFINE) {
        build_affine_mats(B.d.shape, B.d.P, B.d.pts, B.am, kp);
        B.am32.assign(B.am.begin(), B.am.end());
        int npp, ks, mb;
        build_affine_mats_bf16(B.d.shape, B.d.P, B.d.pts, B.am16, npp, ks, mb);
      }
    }
    B.coeff_off = cofs;
    B.phys_off = pofs;
    cofs += B.d.n_elem * B.NP;
    pofs += B.d.n_elem * B.NQ;
    p->total_elem += B.d.n_elem;
    if (B.d.P != blk[0].P) p->uniform_P = false;
  }
  p->total_coeff = cofs;
  p->total_phys = pofs;
  shp_mlp_num_params(&p->mlp_nparam);
  shp_mlp_work_floats(3, &p->mlp_work);
  p->off_model = off;
  off = align_up(off + sizeof(float) * ((size_t)MODEL_MAX_MEMBERS * p->mlp_nparam + 3 * MLP_NIN + p->mlp_work +
                                        3 * MODEL_MAX_MEMBERS));
  p->max_tiles = std::max<long long>(1, p->total_elem);
  p->off_tiles = off;
  off = align_up(off + sizeof(Tile) * (size_t)p->max_tiles * OPK_COUNT);
  for (auto& B : p->blocks) {
    B.off_tab = off;
    off = align_up(off + sizeof(double) * B.tab.size());
    B.off_itab = off;
    off = align_up(off + sizeof(int) * B.itab.size());
    B.off_lm = off;
    off = align_up(off + sizeof(double) * B.lm.size());
    B.off_dm = off;
    off = align_up(off + sizeof(double) * B.dm.size());
    B.off_bt = off;
    off = align_up(off + sizeof(double) * B.bt.size());
    B.off_tabf = off;
    off = align_up(off + sizeof(float) * B.tab.size());
    B.off_am = off;
    off = align_up(off + sizeof(double) * B.am.size());
    B.off_am16 = off;
    off = align_up(off + sizeof(uint16_t) * B.am16.size());
    B.off_am32 = off;
    off = align_up(off + sizeof(float) * B.am32.size());
    B.off_dtab = off;
    off = align_up(off + sizeof(double) * B.dtab.size());
    B.off_ditab = off;
    off = align_up(off + sizeof(int) * B.ditab.size());
  }
  for (auto& B : p->blocks) {
    if (B.iso()) {
      // coordinate coefficients instead of the per-point factors
      B.off_xco = off;
      off = align_up(off + sizeof(double) * (size_t)B.d.n_elem * 3 * B.NP);
      B.off_wref = off;
      off = align_up(off + sizeof(double) * B.wref.size());
      B.off_fac = B.off_dxi = 0;
      continue;
    }
    const int nfac = is_2d(B.d.shape) ? NFAC2 : NFAC, ndxi = is_2d(B.d.shape) ? NDXI2 : NDXI;
    B.off_fac = off;
    off = align_up(off + sizeof(double) * (size_t)B.d.n_elem * nfac * B.NQ);
    B.off_dxi = off;
    off = align_up(off + sizeof(double) * (size_t)B.d.n_elem * ndxi * B.NQ);
    if (!B.am.empty()) {
      B.off_coef = off;
      off = align_up(off + sizeof(double) * (size_t)B.d.n_elem * NAFF);
    }
  }
  p->ws_bytes = off;
  for (int k = 0; k < OPK_COUNT; ++k) p->mixed_dirty[k] = true;
  *out = p;
  return SHP_OK;
}

int shp_plan_destroy(shp_plan p) {
  if (!p) return fail(SHP_ERR_INVALID_ARG, "null plan");
  delete p;
  return SHP_OK;
}

int shp_plan_workspace_bytes(shp_plan p, size_t* bytes) {
  if (int r = check_plan(p)) return r;
  if (!bytes) return fail(SHP_ERR_INVALID_ARG, "null output");
  *bytes = p->ws_bytes;
  return SHP_OK;
}

// Forget the cost model and the choices it made (the workspace changed or a
// new model is loaded).
static void drop_model(shp_plan p) {
  p->model_members = 0;
  for (auto& B : p->blocks)
    for (int op = 0; op < 7; ++op)
      if (B.auto_src[op] == 2) {
        B.auto_src[op] = 0;
        B.auto_strategy[op] = SHP_SUMFAC_COLL;
      }
}

static int upload_static(shp_plan p, hipStream_t s) {
  std::vector<BlockStatic> bs(p->blocks.size());
  for (size_t b = 0; b < p->blocks.size(); ++b) {
    const Block& B = p->blocks[b];
    bs[b].tab = reinterpret_cast<const double*>(p->ws + B.off_tab);
    bs[b].itab = reinterpret_cast<const int*>(p->ws + B.off_itab);
    bs[b].fac = reinterpret_cast<const double*>(p->ws + B.off_fac);
    bs[b].dxi = reinterpret_cast<const double*>(p->ws + B.off_dxi);
    bs[b].tabf = reinterpret_cast<const float*>(p->ws + B.off_tabf);
    bs[b].xco = B.iso() ? reinterpret_cast<const double*>(p->ws + B.off_xco) : nullptr;
    bs[b].wref = B.iso() ? reinterpret_cast<const double*>(p->ws + B.off_wref) : nullptr;
    bs[b].fac32 = (p->fac32 && !B.iso() && !is_2d(B.d.shape)) ? p->fac32 + B.phys_off * NFAC : nullptr;
    bs[b].n_elem = B.d.n_elem;
    bs[b].coeff_off = B.coeff_off;
    bs[b].phys_off = B.phys_off;
    bs[b].shape = B.d.shape;
    bs[b].E = 0;
  }
  hipError_t e = hipMemcpyAsync(p->ws + p->off_bstat, bs.data(), sizeof(BlockStatic) * bs.size(),
                                hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return dev_fail(e, "hipMemcpyAsync(block table)");
  return hipStreamSynchronize(s) == hipSuccess ? SHP_OK : dev_fail(hipGetLastError(), "hipStreamSynchronize");
}

int shp_plan_bind_workspace(shp_plan p, void* ws, size_t ws_bytes, void* stream) {
  if (int r = check_plan(p)) return r;
  if (!ws) return fail(SHP_ERR_WORKSPACE, "null workspace");
  if (reinterpret_cast<uintptr_t>(ws) % ALIGN) return fail(SHP_ERR_WORKSPACE, "workspace not %zu-byte aligned", ALIGN);
  if (ws_bytes < p->ws_bytes) return fail(SHP_ERR_WORKSPACE, "workspace %zu bytes < required %zu", ws_bytes, p->ws_bytes);
  hipStream_t s = static_cast<hipStream_t>(stream);
  p->ws = static_cast<char*>(ws);
  for (auto& B : p->blocks) {
    B.geom_ok = false;
    hipError_t e = hipMemcpyAsync(p->ws + B.off_tab, B.tab.data(), sizeof(double) * B.tab.size(),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !B.itab.empty())
      e = hipMemcpyAsync(p->ws + B.off_itab, B.itab.data(), sizeof(int) * B.itab.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !B.lm.empty())
      e = hipMemcpyAsync(p->ws + B.off_lm, B.lm.data(), sizeof(double) * B.lm.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !B.dm.empty())
      e = hipMemcpyAsync(p->ws + B.off_dm, B.dm.data(), sizeof(double) * B.dm.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !B.bt.empty())
      e = hipMemcpyAsync(p->ws + B.off_bt, B.bt.data(), sizeof(double) * B.bt.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !B.am.empty())
      e = hipMemcpyAsync(p->ws + B.off_am, B.am.data(), sizeof(double) * B.am.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !B.am32.empty())
      e = hipMemcpyAsync(p->ws + B.off_am32, B.am32.data(), sizeof(float) * B.am32.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !B.am16.empty())
      e = hipMemcpyAsync(p->ws + B.off_am16, B.am16.data(), sizeof(uint16_t) * B.am16.size(), hipMemcpyHostToDevice,
                         s);
    if (e == hipSuccess && B.iso())
      e = hipMemcpyAsync(p->ws + B.off_wref, B.wref.data(), sizeof(double) * B.wref.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !B.dtab.empty())
      e = hipMemcpyAsync(p->ws + B.off_dtab, B.dtab.data(), sizeof(double) * B.dtab.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !B.ditab.empty())
      e = hipMemcpyAsync(p->ws + B.off_ditab, B.ditab.data(), sizeof(int) * B.ditab.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
      B.tabf.assign(B.tab.begin(), B.tab.end());
      e = hipMemcpyAsync(p->ws + B.off_tabf, B.tabf.data(), sizeof(float) * B.tabf.size(), hipMemcpyHostToDevice, s);
    }
    if (e != hipSuccess) return dev_fail(e, "hipMemcpyAsync(tables)");
  }
  for (int k = 0; k < OPK_COUNT; ++k) p->mixed_dirty[k] = true;
  drop_model(p);
  return upload_static(p, s);
}

int shp_plan_set_geometry(shp_plan p, int blk, const double* jac, void* stream) {
  if (int r = check_plan(p)) return r;
  if (blk < 0 || blk >= (int)p->blocks.size()) return fail(SHP_ERR_INVALID_ARG, "bad block %d", blk);
  if (!p->ws) return fail(SHP_ERR_STATE, "no workspace bound");
  Block& B = p->blocks[blk];
  if (B.d.n_elem == 0) {
    B.geom_ok = true;
    return SHP_OK;
  }
  if (!jac) return fail(SHP_ERR_INVALID_ARG, "null jac");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int* status = reinterpret_cast<int*>(p->ws + p->off_status);
  hipError_t e = hipMemsetAsync(status, 0, sizeof(int), s);
  if (e != hipSuccess) return dev_fail(e, "hipMemsetAsync(status)");
  if (is_2d(B.d.shape)) {
    e = launch_geometry2d(B.d.shape, B.d.P, reinterpret_cast<const double*>(p->ws + B.off_tab), jac,
                          reinterpret_cast<double*>(p->ws + B.off_fac), reinterpret_cast<double*>(p->ws + B.off_dxi),
                          B.d.n_elem, B.d.geom == SHP_AFFINE, status, s);
    if (e != hipSuccess) return dev_fail(e, "2D geometry kernel launch");
  } else if (B.iso()) {
    // keep the coordinate coefficients; check the geometry they give at
    // every point with the launches' own FP64 reconstruction
    e = hipMemcpyAsync(p->ws + B.off_xco, jac, sizeof(double) * (size_t)B.d.n_elem * 3 * B.NP,
                       hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return dev_fail(e, "coordinate copy");
    const Tiling t = iso_tiling(B.d.P);
    e = launch_iso_check(B.d.P, reinterpret_cast<const BlockStatic*>(p->ws + p->off_bstat), blk, t.E,
                         (B.d.n_elem + t.E - 1) / t.E, t.NT, op_lds_bytes(B.d.shape, B.d.P, OPK_HELM, t.E, 2),
                         status, s);
    if (e != hipSuccess) return dev_fail(e, "iso-parametric geometry check launch");
  } else {
  GeomArgs g;
  g.tab = reinterpret_cast<const double*>(p->ws + B.off_tab);
  g.jac = jac;
  g.fac = reinterpret_cast<double*>(p->ws + B.off_fac);
  g.dxi = reinterpret_cast<double*>(p->ws + B.off_dxi);
  g.status = status;
  g.n_elem = B.d.n_elem;
  g.affine = (B.d.geom == SHP_AFFINE);
  e = launch_geometry(B.d.shape, B.d.P, g, s);
  if (e != hipSuccess) return dev_fail(e, "geometry kernel launch");
  if (!B.am.empty()) {
    e = launch_affine_coef(jac, reinterpret_cast<double*>(p->ws + B.off_coef), B.d.n_elem, status, s);
    if (e != hipSuccess) return dev_fail(e, "affine coefficient kernel launch");
  }
  }
  int h = 0;
  e = hipMemcpyAsync(&h, status, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return dev_fail(e, "geometry status readback");
  if (h) {
    B.geom_ok = false;
    return fail(SHP_ERR_BAD_GEOMETRY, "block %d: det(dx/dxi) <= 0 or non-finite factor", blk);
  }
  B.geom_ok = true;
  if (p->fac32 && !B.iso() && !is_2d(B.d.shape)) {
    // keep the FP32 copy of the factors current
    e = launch_round_f32(reinterpret_cast<const double*>(p->ws + B.off_fac), p->fac32 + B.phys_off * NFAC,
                         B.d.n_elem * NFAC * (long long)B.NQ, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return dev_fail(e, "FP32 factor copy");
  }
  return SHP_OK;
}

int shp_plan_set_fp32_factors(shp_plan p, float* fac32, void* stream) {
  if (int r = check_plan(p)) return r;
  if (!p->ws) return fail(SHP_ERR_STATE, "no workspace bound");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!fac32) {
    p->fac32 = nullptr;
    return upload_static(p, s);
  }
  if (reinterpret_cast<uintptr_t>(fac32) % 4) return fail(SHP_ERR_INVALID_ARG, "fac32 not 4-byte aligned");
  for (size_t b = 0; b < p->blocks.size(); ++b) {
    const Block& B = p->blocks[b];
    if (B.iso() || is_2d(B.d.shape))
      return fail(SHP_ERR_UNSUPPORTED, "block %zu: FP32 factors need 3D blocks with precomputed factors", b);
    if (!B.geom_ok) return fail(SHP_ERR_STATE, "block %zu: geometry not set", b);
  }
  for (const Block& B : p->blocks) {
    const hipError_t e = launch_round_f32(reinterpret_cast<const double*>(p->ws + B.off_fac),
                                          fac32 + B.phys_off * NFAC, B.d.n_elem * NFAC * (long long)B.NQ, s);
    if (e != hipSuccess) return dev_fail(e, "FP32 factor copy");
  }
  p->fac32 = fac32;
  return upload_static(p, s);
}

}  // extern "C"

namespace shp {

long long plan_total_coeff(const shp_plan_s* p) { return p ? p->total_coeff : 0; }

int plan_helm_diag(shp_plan_s* p, double lambda, double* diag, hipStream_t s) {
  for (const Block& B : p->blocks) {
    const hipError_t e = launch_helm_diag(reinterpret_cast<const double*>(p->ws + B.off_fac),
                                          reinterpret_cast<const double*>(p->ws + B.off_dtab),
                                          reinterpret_cast<const int*>(p->ws + B.off_ditab), B.d.Q, B.dn1, B.dn12,
                                          B.NP, B.d.n_elem, lambda, diag + B.coeff_off, s);
    if (e != hipSuccess) return dev_fail(e, "Helmholtz diagonal");
  }
  return SHP_OK;
}

int plan_check_solve(shp_plan_s* p, int inner_prec) {
  if (int r = check_plan(p)) return r;
  if (!p->ws) return fail(SHP_ERR_STATE, "no workspace bound");
  for (const auto& B : p->blocks) {
    if (B.iso()) return fail(SHP_ERR_UNSUPPORTED, "the solve and its diagonal need precomputed factors, not iso-parametric blocks");
    if (is_2d(B.d.shape)) return fail(SHP_ERR_UNSUPPORTED, "the solve covers the 3D shapes");
  }
  for (size_t b = 0; b < p->blocks.size(); ++b)
    if (!p->blocks[b].geom_ok) return fail(SHP_ERR_STATE, "block %zu: geometry not set", b);
  if (inner_prec == SHP_FP32 && !p->uniform_P)
    return fail(SHP_ERR_UNSUPPORTED, "FP32 whole-mesh launch needs one P for all blocks");
  if (inner_prec == SHP_BF16 || inner_prec == SHP_BF16X3)
    for (size_t b = 0; b < p->blocks.size(); ++b)
      if (p->blocks[b].am16.empty())
        return fail(SHP_ERR_UNSUPPORTED, "block %zu: BF16 inner actions need affine blocks with P <= %d", b,
                    LOCALMAT_MAX_P);
  return SHP_OK;
}

int set_error(int code, const char* msg) { return fail(code, "%s", msg); }

}  // namespace shp

extern "C" {

int shp_block_offsets(shp_plan p, int blk, int64_t* coeff_off, int64_t* phys_off) {
  if (int r = check_plan(p)) return r;
  if (blk < 0 || blk >= (int)p->blocks.size()) return fail(SHP_ERR_INVALID_ARG, "bad block %d", blk);
  if (coeff_off) *coeff_off = p->blocks[blk].coeff_off;
  if (phys_off) *phys_off = p->blocks[blk].phys_off;
  return SHP_OK;
}

int shp_set_tiling(shp_plan p, int blk, int op, int strategy, int E, int NT, int persistent) {
  if (int r = check_plan(p)) return r;
  const bool dim2 = is_2d(p->blocks[0].d.shape);
  int opk;
  if (int r = opk_of(op, strategy, &opk)) return r;
  if (dim2 && opk > OPK_HELM)
    return fail(SHP_ERR_UNSUPPORTED, "2D blocks run the collocated sum-factorisation (SHP_SUMFAC_COLL)");
  if (blk < -1 || blk >= (int)p->blocks.size()) return fail(SHP_ERR_INVALID_ARG, "bad block %d", blk);
  if (!(E == 0 && NT == 0)) {
    if (E < 1 || E > 64) return fail(SHP_ERR_INVALID_ARG, "elements per work-group %d outside [1,64]", E);
    if (NT < 64 || NT > 512 || NT % 64) return fail(SHP_ERR_INVALID_ARG, "threads %d: multiple of 64 in [64,512]", NT);
    // a prefetch variant whose points do not fit 8 register slots per thread
    // runs the plain tile, with every table in LDS
    auto variant_of = [&](const Block& B) {
      const long long Q3 = (long long)B.d.Q * B.d.Q * B.d.Q;
      return ((persistent == 1 || persistent == 2) && points_per_thread(E * Q3, NT) == 0) ? 0 : persistent;
    };
    // 2D launches have no variants: the fused Laplacian / Helmholtz tile
    // whenever the tile's points fit its register slots
    auto lds_of = [&](const Block& B) {
      return dim2 ? lds_bytes_2d(B.d.shape, B.d.P, E, opk, NT) : op_lds_bytes(B.d.shape, B.d.P, opk, E, variant_of(B));
    };
    if (blk >= 0) {
      const Block& B = p->blocks[blk];
      if (lds_of(B) > LDS_LIMIT)
        return fail(SHP_ERR_UNSUPPORTED, "%d elements exceed the LDS of a work-group", E);
    } else {
      for (const auto& B : p->blocks)
        if (lds_of(B) > LDS_LIMIT)
          return fail(SHP_ERR_UNSUPPORTED, "%d elements exceed the LDS of a work-group", E);
    }
  }
  if (persistent < 0 || persistent > 4) return fail(SHP_ERR_INVALID_ARG, "launch variant must be in [0,4]");
  Tiling t;
  t.E = E;
  t.NT = NT;
  t.persist = persistent;
  if (blk >= 0)
    p->blocks[blk].tiling[opk] = t;
  else {
    p->mixed[opk] = t;
    p->mixed_dirty[opk] = true;
  }
  return SHP_OK;
}

static Tiling mixed_tiling(shp_plan p, int opk);

int shp_get_tiling(shp_plan p, int blk, int op, int strategy, int* E, int* NT, int* persistent) {
  if (int r = check_plan(p)) return r;
  int opk;
  if (int r = opk_of(op, strategy, &opk)) return r;
  if (blk < -1 || blk >= (int)p->blocks.size()) return fail(SHP_ERR_INVALID_ARG, "bad block %d", blk);
  if (!E || !NT || !persistent) return fail(SHP_ERR_INVALID_ARG, "null output");
  Tiling t;
  if (blk >= 0) {
    const Block& B = p->blocks[blk];
    t = effective(B.tiling[opk], B.d.shape, B.d.P, opk);
  } else {
    t = mixed_tiling(p, opk);
  }
  *E = t.E;
  *NT = t.NT;
  *persistent = t.persist;
  return SHP_OK;
}

// Build and upload the whole-mesh tile list of one operator: tiles of E
// elements from every block, heaviest first (longest-processing-time order).
static Tiling mixed_tiling(shp_plan p, int opk) {
  Tiling t = p->mixed[opk];
  if (t.E > 0 && t.NT > 0) return t;
  if (opk == OPK_HELM_ISO || opk == OPK_LAP_ISO) return iso_tiling(p->blocks[0].d.P);
  const int P0 = p->blocks[0].d.P;
  const bool dim2 = is_2d(p->blocks[0].d.shape);
  if ((opk == OPK_HELM || opk == OPK_LAP || opk == OPK_ADR) && p->uniform_P && P0 >= 7 && !dim2) {
    t.E = HI_MESH_E[P0 - 7];
    t.NT = HI_MESH_NT[P0 - 7];
    t.persist = 2;
    return t;
  }
  t = Tiling{64, 512, 2};
  for (const auto& B : p->blocks) {
    Tiling d = default_tiling(B.d.shape, B.d.P, opk);
    const long long Q3 = (long long)B.d.Q * B.d.Q * B.d.Q;
    if ((opk == OPK_HELM || opk == OPK_LAP || opk == OPK_ADR) && !dim2 && d.E * Q3 <= 2LL * d.NT)
      d = default_tiling(B.d.shape, B.d.P, opk, 64 * 1024);
    t.E = std::min(t.E, d.E);
    t.NT = std::min(t.NT, d.NT);
    t.persist = std::min(t.persist, d.persist);
  }
  return t;
}

// Relative cost of one element by shape (hex, prism, pyramid, tet) and
// P = 1..10: the FP64 collocated Helmholtz launch time per element of the
// largest curved batch of each shape in the MI355X order sweep (about 4M DOF,
// default launch shape), divided by the hexahedron's at the same P.
constexpr double LPT_WEIGHT[4][10] = {
    {1.00, 1.00, 1.00, 1.00, 1.00, 1.00, 1.00, 1.00, 1.00, 1.00},
    {1.03, 1.11, 1.08, 1.02, 1.06, 1.04, 1.13, 1.07, 1.30, 1.70},
    {1.03, 1.08, 1.04, 0.99, 1.03, 1.03, 1.08, 1.05, 1.28, 1.65},
    {1.23, 1.11, 1.06, 1.07, 1.07, 1.14, 1.15, 1.58, 1.44, 1.75}};

static int build_tiles(shp_plan p, int opk, hipStream_t s) {
  const int E = mixed_tiling(p, opk).E;
  struct T2 {
    Tile t;
    double cost;
  };
  std::vector<T2> tl;
  for (int b = 0; b < (int)p->blocks.size(); ++b) {
    const Block& B = p->blocks[b];
    // per-element cost weight: the measured Helmholtz launch time per element
    // of the shape relative to the hexahedron at the same P
    const double w = is_2d(B.d.shape) ? 1.0 : LPT_WEIGHT[B.d.shape][B.d.P - 1];
    for (long long e0 = 0; e0 < B.d.n_elem; e0 += E) {
      T2 x;
      x.t.blk = b;
      x.t.e0 = e0;
      x.t.ne = (int)std::min<long long>(E, B.d.n_elem - e0);
      x.cost = w * x.t.ne;
      tl.push_back(x);
    }
  }
  std::stable_sort(tl.begin(), tl.end(), [](const T2& a, const T2& b) { return a.cost > b.cost; });
  if ((long long)tl.size() > p->max_tiles) return fail(SHP_ERR_WORKSPACE, "tile list overflow");
  std::vector<Tile> host(tl.size());
  for (size_t i = 0; i < tl.size(); ++i) host[i] = tl[i].t;
  Tile* dst = reinterpret_cast<Tile*>(p->ws + p->off_tiles) + (size_t)opk * p->max_tiles;
  hipError_t e = hipSuccess;
  if (!host.empty()) e = hipMemcpyAsync(dst, host.data(), sizeof(Tile) * host.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return dev_fail(e, "tile list upload");
  p->mixed_ntiles[opk] = (int)host.size();
  p->mixed_dirty[opk] = false;
  return SHP_OK;
}

// ---------------------------------------------------------------------------
// Learned strategy choice: the cost model's predictions for a block
// ---------------------------------------------------------------------------

// Strategies in the order of the model's strategy one-hot features.
constexpr int MODEL_STRATS[3] = {SHP_LOCALMAT, SHP_SUMFAC, SHP_SUMFAC_COLL};

static bool model_op(int op) { return op == SHP_OP_LAPLACIAN || op == SHP_OP_HELMHOLTZ; }

static bool strategy_available(const Block& B, int op, int st) {
  if (st == SHP_LOCALMAT) return (model_op(op) || op == SHP_OP_MASS) && B.d.P <= LOCALMAT_MAX_P;
  if (st == SHP_SUMFAC) return model_op(op);
  return st == SHP_SUMFAC_COLL;
}

// Standardised predictions (mean over the model's networks) for the three
// strategies of block blk; synchronises the stream to read them.
static int model_predict(shp_plan p, int blk, float pred[3], hipStream_t s) {
  const Block& B = p->blocks[blk];
  float X[3][MLP_NIN] = {};
  for (int j = 0; j < 3; ++j) {
    X[j][B.d.shape] = 1.f;
    X[j][4] = B.d.P / 10.f;
    X[j][5] = B.d.Q / 12.f;
    X[j][6] = (float)(std::log2((double)B.d.n_elem) / 22.0);
    X[j][7] = B.d.geom == SHP_CURVED ? 1.f : 0.f;
    X[j][8 + j] = 1.f;
  }
  float* prm = reinterpret_cast<float*>(p->ws + p->off_model);
  float* dX = prm + (size_t)MODEL_MAX_MEMBERS * p->mlp_nparam;
  float* work = dX + 3 * MLP_NIN;
  float* dy = work + p->mlp_work;
  hipError_t e = hipMemcpyAsync(dX, X, sizeof X, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return dev_fail(e, "cost model features");
  for (int m = 0; m < p->model_members; ++m)
    if (shp_mlp_forward(prm + (size_t)m * p->mlp_nparam, dX, 3, dy + 3 * m, work, s) != SHP_OK)
      return dev_fail(hipGetLastError(), "cost model forward");
  float y[MODEL_MAX_MEMBERS * 3];
  e = hipMemcpyAsync(y, dy, sizeof(float) * 3 * p->model_members, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return dev_fail(e, "cost model prediction");
  for (int j = 0; j < 3; ++j) {
    float acc = 0.f;
    for (int m = 0; m < p->model_members; ++m) acc += y[3 * m + j];
    pred[j] = acc / p->model_members;
  }
  return SHP_OK;
}

// The strategy SHP_AUTO runs for (blk, op): a tuned or set choice; else the
// cost model's argmin over the block's available strategies (Laplacian and
// Helmholtz, when a model is loaded; remembered for later calls); else the
// collocated sum-factorisation.
static int resolve_auto(shp_plan p, int blk, int op, hipStream_t s, int* strategy) {
  Block& B = p->blocks[blk];
  if (B.auto_src[op] == 0 && p->model_members > 0 && model_op(op) && B.d.n_elem > 0 && !B.iso() &&
      !is_2d(B.d.shape)) {
    float pred[3];
    if (int r = model_predict(p, blk, pred, s)) return r;
    int best = SHP_SUMFAC_COLL;
    float bv = 0.f;
    bool have = false;
    for (int j = 0; j < 3; ++j)
      if (strategy_available(B, op, MODEL_STRATS[j]) && std::isfinite(pred[j]) && (!have || pred[j] < bv)) {
        best = MODEL_STRATS[j];
        bv = pred[j];
        have = true;
      }
    B.auto_strategy[op] = best;
    B.auto_src[op] = 2;
  }
  *strategy = B.auto_strategy[op];
  return SHP_OK;
}

int shp_apply(shp_plan p, int blk, int op, int strategy, const double* in, double* out, double lambda, void* stream) {
  if (int r = check_plan(p)) return r;
  if (strategy == SHP_AUTO && op >= 0 && op <= SHP_OP_HELMHOLTZ && blk >= -1 && blk < (int)p->blocks.size()) {
    if (!in || !out) return fail(SHP_ERR_INVALID_ARG, "null in/out");
    if (!std::isfinite(lambda)) return fail(SHP_ERR_INVALID_ARG, "lambda not finite");
    if (!p->ws) return fail(SHP_ERR_STATE, "no workspace bound");
    hipStream_t s0 = static_cast<hipStream_t>(stream);
    if (blk >= 0) {
      if (int r = resolve_auto(p, blk, op, s0, &strategy)) return r;
    } else if (p->auto_mixed_src[op] == 0 && p->model_members > 0 && model_op(op)) {
      // every block's own choice: one whole-mesh collocated launch when all
      // blocks pick it, else one launch per block
      bool one_launch = p->uniform_P;
      for (int b = 0; b < (int)p->blocks.size(); ++b) {
        if (!p->blocks[b].geom_ok) return fail(SHP_ERR_STATE, "block %d: geometry not set", b);
        int st;
        if (int r = resolve_auto(p, b, op, s0, &st)) return r;
        if (st != SHP_SUMFAC_COLL) one_launch = false;
      }
      if (!one_launch) {
        for (int b = 0; b < (int)p->blocks.size(); ++b) {
          const Block& B = p->blocks[b];
          if (int r = shp_apply(p, b, op, B.auto_strategy[op], in + B.coeff_off, out + B.coeff_off, lambda, stream))
            return r;
        }
        return SHP_OK;
      }
      strategy = SHP_SUMFAC_COLL;
    } else {
      strategy = p->auto_mixed[op];
    }
  }
  int opk;
  if (int r = opk_of(op, strategy, &opk)) return r;
  if (blk < -1 || blk >= (int)p->blocks.size()) return fail(SHP_ERR_INVALID_ARG, "bad block %d", blk);
  if (!in || !out) return fail(SHP_ERR_INVALID_ARG, "null in/out");
  if (!std::isfinite(lambda)) return fail(SHP_ERR_INVALID_ARG, "lambda not finite");
  if (!p->ws) return fail(SHP_ERR_STATE, "no workspace bound");
  const bool needs_geom = !(opk == OPK_BWD || opk == OPK_BWD_LM);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (is_2d(p->blocks[0].d.shape)) {
    // quadrilaterals and triangles: the collocated sum-factorisation
    if (opk > OPK_HELM)
      return fail(SHP_ERR_UNSUPPORTED, "2D blocks run the collocated sum-factorisation (SHP_SUMFAC_COLL)");
    const int b0 = blk >= 0 ? blk : 0, b1 = blk >= 0 ? blk + 1 : (int)p->blocks.size();
    for (int b = b0; b < b1; ++b)
      if (needs_geom && !p->blocks[b].geom_ok) return fail(SHP_ERR_STATE, "block %d: geometry not set", b);
    hipError_t e = hipSuccess;
    if (blk >= 0 || !p->uniform_P) {
      for (int b = b0; b < b1 && e == hipSuccess; ++b) {
        const Block& B = p->blocks[b];
        const Tiling t = effective(B.tiling[opk], B.d.shape, B.d.P, opk);
        OpArgs a{};
        a.tab = reinterpret_cast<const double*>(p->ws + B.off_tab);
        a.fac = reinterpret_cast<const double*>(p->ws + B.off_fac);
        a.dxi = reinterpret_cast<const double*>(p->ws + B.off_dxi);
        a.in = in + (blk >= 0 ? 0 : (in_is_modes(opk) ? B.coeff_off : B.phys_off));
        a.out = out + (blk >= 0 ? 0 : (out_is_modes(opk) ? B.coeff_off : B.phys_off));
        a.n_elem = B.d.n_elem;
        a.in_cs = a.out_cs = (blk >= 0) ? B.d.n_elem * (long long)B.NQ : p->total_phys;
        a.lambda = lambda;
        a.E = t.E;
        e = launch_block2d(B.d.shape, B.d.P, opk, a, t.NT, s);
      }
    } else {
      if (p->mixed_dirty[opk])
        if (int r = build_tiles(p, opk, s)) return r;
      const Tiling mt = mixed_tiling(p, opk);
      size_t lds = 0;
      for (const auto& B : p->blocks) lds = std::max(lds, lds_bytes_2d(B.d.shape, B.d.P, mt.E, opk, mt.NT));
      const Tile* tiles = reinterpret_cast<const Tile*>(p->ws + p->off_tiles) + (size_t)opk * p->max_tiles;
      e = launch_mixed2d(p->blocks[0].d.P, opk, reinterpret_cast<const BlockStatic*>(p->ws + p->off_bstat), tiles,
                         p->mixed_ntiles[opk], in, out, p->total_phys, p->total_phys, lambda, mt.NT, lds, mt.E, s);
    }
    if (e != hipSuccess) return dev_fail(e, "2D launch");
    return SHP_OK;
  }
  {
    // iso-parametric blocks: the backward transform as for any block, and the
    // collocated Laplacian / Helmholtz with the geometry rebuilt in the launch
    const int b0 = blk >= 0 ? blk : 0, b1 = blk >= 0 ? blk + 1 : (int)p->blocks.size();
    int niso = 0;
    for (int b = b0; b < b1; ++b) niso += p->blocks[b].iso() ? 1 : 0;
    if (niso > 0 && opk != OPK_BWD) {
      if (opk != OPK_HELM && opk != OPK_LAP)
        return fail(SHP_ERR_UNSUPPORTED, "iso-parametric blocks support the backward transform and the collocated "
                                         "Laplacian and Helmholtz actions");
      if (niso != b1 - b0)
        return fail(SHP_ERR_UNSUPPORTED, "a whole-mesh launch takes iso-parametric blocks only with each other");
      if (blk < 0 && !p->uniform_P) return fail(SHP_ERR_UNSUPPORTED, "the whole-mesh launch needs one P for all blocks");
      for (int b = b0; b < b1; ++b)
        if (!p->blocks[b].geom_ok) return fail(SHP_ERR_STATE, "block %d: geometry not set", b);
      const int iopk = (opk == OPK_HELM) ? OPK_HELM_ISO : OPK_LAP_ISO;
      const BlockStatic* bst = reinterpret_cast<const BlockStatic*>(p->ws + p->off_bstat);
      hipError_t e;
      if (blk >= 0) {
        const Block& B = p->blocks[blk];
        const Tiling t = iso_tiling(B.d.P);
        e = launch_iso(B.d.P, iopk, bst, nullptr, 0, in, out, lambda, t.NT,
                       op_lds_bytes(B.d.shape, B.d.P, OPK_HELM, t.E, 2), t.E, blk, (B.d.n_elem + t.E - 1) / t.E, s);
      } else {
        if (p->mixed_dirty[iopk])
          if (int r = build_tiles(p, iopk, s)) return r;
        const Tiling t = mixed_tiling(p, iopk);
        size_t lds = 0;
        for (const auto& B : p->blocks) lds = std::max(lds, op_lds_bytes(B.d.shape, B.d.P, OPK_HELM, t.E, 2));
        const Tile* tiles = reinterpret_cast<const Tile*>(p->ws + p->off_tiles) + (size_t)iopk * p->max_tiles;
        e = launch_iso(p->blocks[0].d.P, iopk, bst, tiles, p->mixed_ntiles[iopk], in, out, lambda, t.NT, lds, t.E, -1,
                       p->mixed_ntiles[iopk], s);
      }
      if (e != hipSuccess) return dev_fail(e, "iso-parametric launch");
      return SHP_OK;
    }
  }
  if (is_localmat(opk)) {
    const int b0 = blk >= 0 ? blk : 0, b1 = blk >= 0 ? blk + 1 : (int)p->blocks.size();
    for (int b = b0; b < b1; ++b) {
      const Block& B = p->blocks[b];
      if (B.d.P > LOCALMAT_MAX_P) return fail(SHP_ERR_UNSUPPORTED, "local-matrix strategy needs P <= %d", LOCALMAT_MAX_P);
      if (needs_geom && !B.geom_ok) return fail(SHP_ERR_STATE, "block %d: geometry not set", b);
    }
    if (blk < 0 && !is_xform_lm(opk) && p->uniform_P && b1 - b0 >= 1 && b1 - b0 <= 8) {
      // every block affine: one launch over all of them
      bool all = true;
      for (int b = b0; b < b1; ++b) all = all && !p->blocks[b].am.empty();
      if (all) {
        AffineMatArgs arr[8];
        int shp_of[8];
        for (int b = b0; b < b1; ++b) {
          const Block& B = p->blocks[b];
          AffineMatArgs& aa = arr[b - b0];
          aa.afrag = reinterpret_cast<const double*>(p->ws + B.off_am);
          aa.coef = reinterpret_cast<const double*>(p->ws + B.off_coef);
          aa.in = in + B.coeff_off;
          aa.out = out + B.coeff_off;
          aa.n_elem = B.d.n_elem;
          aa.lambda = lambda;
          shp_of[b - b0] = B.d.shape;
        }
        hipError_t e = launch_localmat_affine_mesh(p->blocks[b0].d.P, opk, b1 - b0, shp_of, arr, s);
        if (e != hipSuccess) return dev_fail(e, "affine local-matrix mesh launch");
        return SHP_OK;
      }
    }
    for (int b = b0; b < b1; ++b) {
      const Block& B = p->blocks[b];
      if (is_xform_lm(opk)) {
        // the transforms: [B; d_d B] (or the dense collocation derivatives)
        // with the per-point factors, for affine and curved blocks alike
        LocalXformArgs xa;
        xa.bcat = reinterpret_cast<const double*>(p->ws + B.off_lm);
        xa.dmat = reinterpret_cast<const double*>(p->ws + B.off_dm);
        xa.bt = reinterpret_cast<const double*>(p->ws + B.off_bt);
        xa.fac = reinterpret_cast<const double*>(p->ws + B.off_fac);
        xa.dxi = reinterpret_cast<const double*>(p->ws + B.off_dxi);
        xa.in = in + (blk >= 0 ? 0 : (in_is_modes(opk) ? B.coeff_off : B.phys_off));
        xa.out = out + (blk >= 0 ? 0 : (out_is_modes(opk) ? B.coeff_off : B.phys_off));
        xa.n_elem = B.d.n_elem;
        xa.in_cs = xa.out_cs = (blk >= 0) ? B.d.n_elem * (long long)B.NQ : p->total_phys;
        xa.wpt = 1;  // the launcher chooses the waves per tile
        hipError_t e = launch_localmat_xform(B.d.shape, B.d.P, opk, xa, s);
        if (e != hipSuccess) return dev_fail(e, "local-matrix transform launch");
        continue;
      }
      if (!B.am.empty()) {
        // affine block: 7 reference matrices and 7 coefficients per element
        AffineMatArgs aa;
        aa.afrag = reinterpret_cast<const double*>(p->ws + B.off_am);
        aa.coef = reinterpret_cast<const double*>(p->ws + B.off_coef);
        aa.in = in + (blk >= 0 ? 0 : B.coeff_off);
        aa.out = out + (blk >= 0 ? 0 : B.coeff_off);
        aa.n_elem = B.d.n_elem;
        aa.lambda = lambda;
        hipError_t e = launch_localmat_affine(B.d.shape, B.d.P, opk, aa, s);
        if (e != hipSuccess) return dev_fail(e, "affine local-matrix launch");
        continue;
      }
      LocalMatArgs la;
      la.bcat = reinterpret_cast<const double*>(p->ws + B.off_lm);
      la.bt = reinterpret_cast<const double*>(p->ws + B.off_bt);
      la.fac = reinterpret_cast<const double*>(p->ws + B.off_fac);
      la.in = in + (blk >= 0 ? 0 : B.coeff_off);
      la.out = out + (blk >= 0 ? 0 : B.coeff_off);
      la.n_elem = B.d.n_elem;
      la.lambda = lambda;
      hipError_t e = launch_localmat(B.d.shape, B.d.P, opk, la, s);
      if (e != hipSuccess) return dev_fail(e, "local-matrix launch");
    }
    return SHP_OK;
  }
  if (blk >= 0) {
    Block& B = p->blocks[blk];
    if (needs_geom && !B.geom_ok) return fail(SHP_ERR_STATE, "block %d: geometry not set", blk);
    const Tiling t = effective(B.tiling[opk], B.d.shape, B.d.P, opk);
    OpArgs a{};
    a.tab = reinterpret_cast<const double*>(p->ws + B.off_tab);
    a.itab = reinterpret_cast<const int*>(p->ws + B.off_itab);
    a.fac = reinterpret_cast<const double*>(p->ws + B.off_fac);
    a.dxi = reinterpret_cast<const double*>(p->ws + B.off_dxi);
    a.in = in;
    a.out = out;
    a.n_elem = B.d.n_elem;
    a.in_cs = B.d.n_elem * (long long)B.NQ;
    a.out_cs = a.in_cs;
    a.lambda = lambda;
    a.E = t.E;
    hipError_t e = launch_block(B.d.shape, B.d.P, opk, a, t.NT, t.persist, s);
    if (e != hipSuccess) return dev_fail(e, "operator launch");
    return SHP_OK;
  }
  // whole mesh
  for (size_t b = 0; b < p->blocks.size(); ++b)
    if (needs_geom && !p->blocks[b].geom_ok) return fail(SHP_ERR_STATE, "block %zu: geometry not set", b);
  if (!p->uniform_P) {
    // blocks of different order: one launch per block on the stream
    for (size_t b = 0; b < p->blocks.size(); ++b) {
      Block& B = p->blocks[b];
      const double* bin = in + (in_is_modes(opk) ? B.coeff_off : B.phys_off);
      double* bout = out + (out_is_modes(opk) ? B.coeff_off : B.phys_off);
      const Tiling t = effective(B.tiling[opk], B.d.shape, B.d.P, opk);
      OpArgs a{};
      a.tab = reinterpret_cast<const double*>(p->ws + B.off_tab);
      a.itab = reinterpret_cast<const int*>(p->ws + B.off_itab);
      a.fac = reinterpret_cast<const double*>(p->ws + B.off_fac);
      a.dxi = reinterpret_cast<const double*>(p->ws + B.off_dxi);
      a.in = bin;
      a.out = bout;
      a.n_elem = B.d.n_elem;
      a.in_cs = p->total_phys;
      a.out_cs = p->total_phys;
      a.lambda = lambda;
      a.E = t.E;
      hipError_t e = launch_block(B.d.shape, B.d.P, opk, a, t.NT, t.persist, s);
      if (e != hipSuccess) return dev_fail(e, "operator launch");
    }
    return SHP_OK;
  }
  if (p->mixed_dirty[opk])
    if (int r = build_tiles(p, opk, s)) return r;
  const Tiling mt = mixed_tiling(p, opk);
  const int E = mt.E, NT = mt.NT;
  size_t lds = 0;
  for (const auto& B : p->blocks) lds = std::max(lds, op_lds_bytes(B.d.shape, B.d.P, opk, E, mt.persist));
  const Tile* tiles = reinterpret_cast<const Tile*>(p->ws + p->off_tiles) + (size_t)opk * p->max_tiles;
  hipError_t e = launch_mixed(p->blocks[0].d.P, opk, reinterpret_cast<const BlockStatic*>(p->ws + p->off_bstat), tiles,
                              p->mixed_ntiles[opk], in, out, p->total_phys, p->total_phys, lambda, NT, lds, E, mt.persist, s);
  if (e != hipSuccess) return dev_fail(e, "mixed launch");
  return SHP_OK;
}


// affine local-matrix actions in split BF16 (SHP_BF16, SHP_BF16X3) or in FP32
// on the FP32 matrix cores (SHP_FP32), of one block or of every block
static int apply_bf16(shp_plan p, int blk, int op, int strategy, int prec, const void* in, void* out, double lambda,
                      void* stream) {
  if (op != SHP_OP_MASS && op != SHP_OP_LAPLACIAN && op != SHP_OP_HELMHOLTZ)
    return fail(SHP_ERR_UNSUPPORTED, "local-matrix contractions below FP64 cover the mass, Laplacian and Helmholtz actions");
  if (strategy != SHP_AUTO && strategy != SHP_LOCALMAT)
    return fail(SHP_ERR_UNSUPPORTED, "BF16 contractions use the affine local matrices (SHP_LOCALMAT)");
  const bool f32 = prec == SHP_FP32;
  if (blk < -1 || blk >= (int)p->blocks.size()) return fail(SHP_ERR_INVALID_ARG, "bad block %d", blk);
  if (!in || !out) return fail(SHP_ERR_INVALID_ARG, "null in/out");
  if (!std::isfinite(lambda)) return fail(SHP_ERR_INVALID_ARG, "lambda not finite");
  const int b0 = blk >= 0 ? blk : 0, b1 = blk >= 0 ? blk + 1 : (int)p->blocks.size();
  for (int b = b0; b < b1; ++b)
    if (p->blocks[b].am16.empty())
      return fail(SHP_ERR_UNSUPPORTED, "block %d: BF16 and FP32 local-matrix contractions need an affine 3D block with P <= %d", b,
                  LOCALMAT_MAX_P);
  if (!p->ws) return fail(SHP_ERR_STATE, "no workspace bound");
  for (int b = b0; b < b1; ++b)
    if (!p->blocks[b].geom_ok) return fail(SHP_ERR_STATE, "block %d: geometry not set", b);
  const int opk = op == SHP_OP_MASS ? OPK_MASS_LM : op == SHP_OP_LAPLACIAN ? OPK_LAP_LM : OPK_HELM_LM;
  const int nparts = prec == SHP_BF16 ? 3 : 2;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (f32) {
    if (blk < 0 && p->uniform_P && b1 - b0 >= 1 && b1 - b0 <= 8) {
      // every block in one launch
      AffineMatArgs32 arr[8];
      int shp_of[8];
      for (int b = b0; b < b1; ++b) {
        const Block& B = p->blocks[b];
        AffineMatArgs32& aa = arr[b - b0];
        aa.afrag = reinterpret_cast<const float*>(p->ws + B.off_am32);
        aa.coef = reinterpret_cast<const double*>(p->ws + B.off_coef);
        aa.in = static_cast<const float*>(in) + B.coeff_off;
        aa.out = static_cast<float*>(out) + B.coeff_off;
        aa.n_elem = B.d.n_elem;
        aa.lambda = lambda;
        shp_of[b - b0] = B.d.shape;
      }
      hipError_t e = launch_localmat_affine_f32_mesh(p->blocks[b0].d.P, opk, b1 - b0, shp_of, arr, s);
      if (e != hipSuccess) return dev_fail(e, "FP32 local-matrix mesh launch");
      return SHP_OK;
    }
    for (int b = b0; b < b1; ++b) {
      const Block& B = p->blocks[b];
      const long long off = blk >= 0 ? 0 : B.coeff_off;
      hipError_t e = launch_localmat_affine_f32(
          B.d.shape, B.d.P, opk, reinterpret_cast<const float*>(p->ws + B.off_am32),
          reinterpret_cast<const double*>(p->ws + B.off_coef), static_cast<const float*>(in) + off,
          static_cast<float*>(out) + off, B.d.n_elem, lambda, s);
      if (e != hipSuccess) return dev_fail(e, "FP32 local-matrix launch");
    }
    return SHP_OK;
  }
  bool one_p = b1 - b0 <= 8;
  for (int b = b0; b < b1; ++b) one_p = one_p && p->blocks[b].d.P == p->blocks[b0].d.P;
  if (blk < 0 && one_p) {
    // every block in one launch (their work overlaps on the chip)
    int shape[8];
    const bf16_frag* af[8];
    const double* cf[8];
    const float* xi[8];
    float* yo[8];
    long long ne[8];
    for (int b = b0; b < b1; ++b) {
      const Block& B = p->blocks[b];
      shape[b] = B.d.shape;
      af[b] = reinterpret_cast<const bf16_frag*>(p->ws + B.off_am16);
      cf[b] = reinterpret_cast<const double*>(p->ws + B.off_coef);
      xi[b] = static_cast<const float*>(in) + B.coeff_off;
      yo[b] = static_cast<float*>(out) + B.coeff_off;
      ne[b] = B.d.n_elem;
    }
    hipError_t e = launch_localmat_affine_bf16_mesh(p->blocks[b0].d.P, opk, nparts, b1 - b0, shape, af, cf, xi, yo, ne,
                                                    lambda, s);
    if (e != hipSuccess) return dev_fail(e, "BF16 local-matrix launch");
    return SHP_OK;
  }
  for (int b = b0; b < b1; ++b) {
    const Block& B = p->blocks[b];
    const long long off = blk >= 0 ? 0 : B.coeff_off;
    hipError_t e = launch_localmat_affine_bf16(
        B.d.shape, B.d.P, opk, nparts, reinterpret_cast<const bf16_frag*>(p->ws + B.off_am16),
        reinterpret_cast<const double*>(p->ws + B.off_coef), static_cast<const float*>(in) + off,
        static_cast<float*>(out) + off, B.d.n_elem, lambda, s);
    if (e != hipSuccess) return dev_fail(e, "BF16 local-matrix launch");
  }
  return SHP_OK;
}

int shp_apply_prec(shp_plan p, int blk, int op, int strategy, int prec, const void* in, void* out, double lambda,
                   void* stream) {
  if (int r = check_plan(p)) return r;
  if (prec == SHP_FP64)
    return shp_apply(p, blk, op, strategy, static_cast<const double*>(in), static_cast<double*>(out), lambda, stream);
  if (prec == SHP_BF16 || prec == SHP_BF16X3) return apply_bf16(p, blk, op, strategy, prec, in, out, lambda, stream);
  if (prec != SHP_FP32) return fail(SHP_ERR_INVALID_ARG, "bad precision %d", prec);
  if (strategy == SHP_LOCALMAT) return apply_bf16(p, blk, op, strategy, prec, in, out, lambda, stream);
  if (strategy == SHP_AUTO && blk == -1 && op >= 0 && op <= SHP_OP_HELMHOLTZ && p->auto_mixed[op] == SHP_LOCALMAT) {
    // the plan's whole-mesh choice is the local matrices: FP32 on the matrix
    // cores when every block has them (affine, P <= 4)
    bool all = !p->blocks.empty();
    for (const auto& B : p->blocks) all = all && !B.am32.empty();
    if (all) return apply_bf16(p, blk, op, SHP_LOCALMAT, prec, in, out, lambda, stream);
  }
  if (op != SHP_OP_HELMHOLTZ && op != SHP_OP_LAPLACIAN)
    return fail(SHP_ERR_UNSUPPORTED, "FP32 contractions cover the Laplacian and Helmholtz actions");
  if (strategy != SHP_AUTO && strategy != SHP_SUMFAC_COLL)
    return fail(SHP_ERR_UNSUPPORTED, "FP32 contractions use the collocated sum-factorisation");
  if (blk != -1) return fail(SHP_ERR_UNSUPPORTED, "FP32 contractions run as a whole-mesh launch (blk = -1)");
  if (!in || !out) return fail(SHP_ERR_INVALID_ARG, "null in/out");
  if (!std::isfinite(lambda)) return fail(SHP_ERR_INVALID_ARG, "lambda not finite");
  if (!p->ws) return fail(SHP_ERR_STATE, "no workspace bound");
  if (!p->uniform_P) return fail(SHP_ERR_UNSUPPORTED, "FP32 whole-mesh launch needs one P for all blocks");
  for (size_t b = 0; b < p->blocks.size(); ++b) {
    if (!p->blocks[b].geom_ok) return fail(SHP_ERR_STATE, "block %zu: geometry not set", b);
    if (p->blocks[b].iso()) return fail(SHP_ERR_UNSUPPORTED, "FP32 contractions need precomputed factors");
    if (is_2d(p->blocks[b].d.shape)) return fail(SHP_ERR_UNSUPPORTED, "FP32 contractions cover the 3D shapes");
  }
  const int opk = (op == SHP_OP_HELMHOLTZ) ? OPK_HELM : OPK_LAP;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (p->mixed_dirty[opk])
    if (int r = build_tiles(p, opk, s)) return r;
  const Tiling mt = mixed_tiling(p, opk);
  size_t lds = 0;
  for (const auto& B : p->blocks) lds = std::max(lds, lds_bytes_f32(B.d.shape, B.d.P, mt.E));
  if (points_per_thread((long long)mt.E * (p->blocks[0].d.Q) * p->blocks[0].d.Q * p->blocks[0].d.Q, mt.NT) == 0)
    return fail(SHP_ERR_UNSUPPORTED, "launch shape too large for the FP32 kernel's register slots");
  const Tile* tiles = reinterpret_cast<const Tile*>(p->ws + p->off_tiles) + (size_t)opk * p->max_tiles;
  hipError_t e = launch_mixed_f32(p->blocks[0].d.P, opk, reinterpret_cast<const BlockStatic*>(p->ws + p->off_bstat),
                                  tiles, p->mixed_ntiles[opk], static_cast<const float*>(in), static_cast<float*>(out),
                                  lambda, mt.NT, lds, mt.E, p->fac32 != nullptr, s);
  if (e != hipSuccess) return dev_fail(e, "FP32 launch");
  return SHP_OK;
}

int shp_advection_factors(shp_plan p, const double* vel, double* adv, void* stream) {
  if (int r = check_plan(p)) return r;
  if (!vel || !adv) return fail(SHP_ERR_INVALID_ARG, "null vel/adv");
  if (!p->ws) return fail(SHP_ERR_STATE, "no workspace bound");
  for (size_t b = 0; b < p->blocks.size(); ++b) {
    if (!p->blocks[b].geom_ok) return fail(SHP_ERR_STATE, "block %zu: geometry not set", b);
    if (p->blocks[b].iso() || is_2d(p->blocks[b].d.shape))
      return fail(SHP_ERR_UNSUPPORTED, "advection factors need 3D blocks with precomputed factors");
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (const Block& B : p->blocks) {
    const hipError_t e = launch_adv_factors(reinterpret_cast<const double*>(p->ws + B.off_fac),
                                            reinterpret_cast<const double*>(p->ws + B.off_dxi), vel + B.phys_off,
                                            p->total_phys, adv + 3 * B.phys_off, B.d.n_elem, B.NQ, s);
    if (e != hipSuccess) return dev_fail(e, "advection factors");
  }
  return SHP_OK;
}

int shp_apply_adr(shp_plan p, const double* adv, const double* in, double* out, double lambda, void* stream) {
  if (int r = check_plan(p)) return r;
  if (!adv || !in || !out) return fail(SHP_ERR_INVALID_ARG, "null adv/in/out");
  if (!std::isfinite(lambda)) return fail(SHP_ERR_INVALID_ARG, "lambda not finite");
  if (!p->ws) return fail(SHP_ERR_STATE, "no workspace bound");
  if (!p->uniform_P) return fail(SHP_ERR_UNSUPPORTED, "the whole-mesh launch needs one P for all blocks");
  for (size_t b = 0; b < p->blocks.size(); ++b) {
    if (!p->blocks[b].geom_ok) return fail(SHP_ERR_STATE, "block %zu: geometry not set", b);
    if (p->blocks[b].iso() || is_2d(p->blocks[b].d.shape))
      return fail(SHP_ERR_UNSUPPORTED, "the advection-diffusion-reaction action needs 3D blocks with precomputed factors");
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (p->mixed_dirty[OPK_ADR])
    if (int r = build_tiles(p, OPK_ADR, s)) return r;
  const Tiling mt = mixed_tiling(p, OPK_ADR);
  const int Q = p->blocks[0].d.Q;
  if (points_per_thread((long long)mt.E * Q * Q * Q, mt.NT) == 0)
    return fail(SHP_ERR_UNSUPPORTED, "launch shape too large for the advection-diffusion-reaction kernel");
  size_t lds = 0;
  for (const auto& B : p->blocks) lds = std::max(lds, op_lds_bytes(B.d.shape, B.d.P, OPK_ADR, mt.E, 2));
  const Tile* tiles = reinterpret_cast<const Tile*>(p->ws + p->off_tiles) + (size_t)OPK_ADR * p->max_tiles;
  const hipError_t e = launch_adr(p->blocks[0].d.P, reinterpret_cast<const BlockStatic*>(p->ws + p->off_bstat), tiles,
                                  p->mixed_ntiles[OPK_ADR], in, out, adv, lambda, mt.NT, lds, mt.E, s);
  if (e != hipSuccess) return dev_fail(e, "advection-diffusion-reaction launch");
  return SHP_OK;
}

// ---------------------------------------------------------------------------
// Autotuning
// ---------------------------------------------------------------------------

static long long out_count(shp_plan p, int blk, int op) {
  long long modes = 0, pts = 0;
  if (blk >= 0) {
    const Block& B = p->blocks[blk];
    modes = B.d.n_elem * B.NP;
    pts = B.d.n_elem * B.NQ;
  } else {
    modes = p->total_coeff;
    pts = p->total_phys;
  }
  if (op == SHP_OP_BWDTRANS) return pts;
  if (op == SHP_OP_PHYSDERIV) return 3 * pts;
  return modes;
}

static void set_tiling_raw(shp_plan p, int blk, int opk, const Tiling& t) {
  if (blk >= 0)
    p->blocks[blk].tiling[opk] = t;
  else {
    p->mixed[opk] = t;
    p->mixed_dirty[opk] = true;
  }
}

static Tiling get_tiling_raw(shp_plan p, int blk, int opk) {
  return blk >= 0 ? p->blocks[blk].tiling[opk] : p->mixed[opk];
}

int shp_tune(shp_plan p, int blk, int op, const double* in, double* out, double* ref, double lambda, int reps,
             int quick, shp_tune_result* res, shp_tune_record* records, int max_records, int* n_records,
             void* stream) {
  if (int r = check_plan(p)) return r;
  if (blk < -1 || blk >= (int)p->blocks.size()) return fail(SHP_ERR_INVALID_ARG, "bad block %d", blk);
  if (op < 0 || op > SHP_OP_HELMHOLTZ) return fail(SHP_ERR_INVALID_ARG, "bad operator %d", op);
  if (!in || !out || !ref || !res) return fail(SHP_ERR_INVALID_ARG, "null argument");
  if (reps < 1 || reps > 1000) return fail(SHP_ERR_INVALID_ARG, "reps=%d outside [1,1000]", reps);
  if (is_2d(p->blocks[0].d.shape)) return fail(SHP_ERR_UNSUPPORTED, "tuning covers the 3D shapes");
  if (max_records > 0 && !records) return fail(SHP_ERR_INVALID_ARG, "null records");
  if (!p->ws) return fail(SHP_ERR_STATE, "no workspace bound");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool helm = (op == SHP_OP_HELMHOLTZ || op == SHP_OP_LAPLACIAN);
  bool lm_ok = true;  // every operator has a local-matrix form up to LOCALMAT_MAX_P
  if (blk >= 0)
    lm_ok = lm_ok && p->blocks[blk].d.P <= LOCALMAT_MAX_P;
  else
    for (const auto& B : p->blocks) lm_ok = lm_ok && B.d.P <= LOCALMAT_MAX_P;
  int strategies[3] = {SHP_SUMFAC_COLL, SHP_SUMFAC, SHP_LOCALMAT};
  int nstrat = helm ? 2 : 1;
  if (lm_ok) strategies[nstrat++] = SHP_LOCALMAT;
  int opks[3];
  for (int i = 0; i < nstrat; ++i)
    if (int r = opk_of(op, strategies[i], &opks[i])) return r;
  // keep the caller's launch shapes to restore the loser's afterwards
  Tiling saved[3];
  for (int i = 0; i < nstrat; ++i) saved[i] = get_tiling_raw(p, blk, opks[i]);
  const long long nout = out_count(p, blk, op);
  unsigned long long* dd = reinterpret_cast<unsigned long long*>(p->ws + p->off_status + 64);
  // reference: the default launch of the collocated strategy
  set_tiling_raw(p, blk, opks[0], Tiling{0, 0, 2});
  if (int r = shp_apply(p, blk, op, SHP_SUMFAC_COLL, in, ref, lambda, stream)) {
    for (int i = 0; i < nstrat; ++i) set_tiling_raw(p, blk, opks[i], saved[i]);
    return r;
  }
  hipEvent_t ev[2 * 64];
  const int nev = std::min(reps, 64);
  for (int i = 0; i < 2 * nev; ++i)
    if (hipEventCreate(&ev[i]) != hipSuccess) {
      for (int j = 0; j < i; ++j) hipEventDestroy(ev[j]);
      for (int k = 0; k < nstrat; ++k) set_tiling_raw(p, blk, opks[k], saved[k]);
      return dev_fail(hipGetLastError(), "hipEventCreate");
    }
  // smallest P of the blocks involved, for the launch-shape limits
  int P = MAX_P;
  if (blk >= 0)
    P = p->blocks[blk].d.P;
  else
    for (const auto& B : p->blocks) P = std::min(P, B.d.P);
  const int Q = P + 2;
  // candidate list: (strategy, launch shape); blocks of different P under one
  // whole-mesh call run one launch per block with the blocks' own shapes, so
  // only the strategy is a candidate there
  struct Cand {
    int si, E, NT, V;
  };
  std::vector<Cand> cands;
  std::vector<int> Es, NTs;
  if (quick) {
    Es = {1, 2, 4, 8};
    NTs = {128, 256};
  } else {
    for (int E = 1; E <= 16; ++E) Es.push_back(E);
    NTs = {64, 128, 192, 256, 320, 384, 512};
  }
  const bool shapes_apply = (blk >= 0 || p->uniform_P);
  for (int si = 0; si < nstrat; ++si) {
    const int st = strategies[si], opk = opks[si];
    if (!shapes_apply) {
      cands.push_back(Cand{si, 0, 0, 0});
      continue;
    }
    std::vector<int> Vs = {0};
    if (helm && st == SHP_SUMFAC_COLL) Vs = quick ? std::vector<int>{0, 2, 3} : std::vector<int>{0, 1, 2, 3, 4};
    const bool lm = (st == SHP_LOCALMAT);  // one launch shape: 16 elements, 4 waves
    for (int E : (lm ? std::vector<int>{16} : Es))
      for (int NT : (lm ? std::vector<int>{256} : NTs))
        for (int V : Vs) {
          if ((V == 1 || V == 2) && (long long)E * Q * Q * Q > 8LL * NT) continue;
          if (V == 4 && E * Q * Q > NT) continue;
          if (!lm && NT > 64 && NT > 2 * E * Q * Q * Q) continue;  // most threads would idle
          bool fits = true;
          if (blk >= 0)
            fits = op_lds_bytes(p->blocks[blk].d.shape, p->blocks[blk].d.P, opk, E, V) <= 64 * 1024 * 2;
          else
            for (const auto& B : p->blocks) fits = fits && op_lds_bytes(B.d.shape, B.d.P, opk, E, V) <= 64 * 1024 * 2;
          if (lm) fits = true;
          if (fits) cands.push_back(Cand{si, E, NT, V});
        }
  }
  // the Infinity Cache (MALL, 256 MiB) is flushed before every timed launch by
  // writing a 1 GiB buffer outside the timing events, so small batches are
  // timed against HBM as large ones are
  const size_t flush_bytes = size_t(1) << 30;
  void* flush = nullptr;
  if (hipMalloc(&flush, flush_bytes) != hipSuccess) {
    for (int i = 0; i < 2 * nev; ++i) hipEventDestroy(ev[i]);
    for (int i = 0; i < nstrat; ++i) set_tiling_raw(p, blk, opks[i], saved[i]);
    return dev_fail(hipGetLastError(), "hipMalloc of the 1 GiB cache-flush buffer");
  }
  int ncand = 0, nrej = 0, nrec = 0;
  Block::Tuned best;
  best.ms = 1e300;
  int rc = SHP_OK;
  for (const Cand& c : cands) {
    const int st = strategies[c.si], opk = opks[c.si];
    set_tiling_raw(p, blk, opk, Tiling{c.E, c.NT, c.V});
    ++ncand;
    bool pass = false;
    double med = -1.0;
    const int ra = shp_apply(p, blk, op, st, in, out, lambda, stream);
    if (ra == SHP_ERR_DEVICE) {
      rc = ra;
      break;
    }
    if (ra == SHP_OK) {
      hipError_t e = hipMemsetAsync(dd, 0, 2 * sizeof(unsigned long long), s);
      if (e == hipSuccess) e = launch_maxdiff(out, ref, nout, dd, s);
      unsigned long long h[2] = {0, 0};
      if (e == hipSuccess) e = hipMemcpyAsync(h, dd, sizeof h, hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) {
        rc = dev_fail(e, "tuning parity check");
        break;
      }
      double dmax, bmax;
      std::memcpy(&dmax, &h[0], sizeof dmax);
      std::memcpy(&bmax, &h[1], sizeof bmax);
      pass = std::isfinite(dmax) && dmax <= 1e-12 * std::max(bmax, 1e-300);
    }
    if (pass) {
      for (int r = 0; r < nev && rc == SHP_OK; ++r) {
        if (hipMemsetAsync(flush, r & 0xff, flush_bytes, s) != hipSuccess) {
          rc = dev_fail(hipGetLastError(), "cache flush");
          break;
        }
        hipEventRecord(ev[2 * r], s);
        rc = shp_apply(p, blk, op, st, in, out, lambda, stream);
        hipEventRecord(ev[2 * r + 1], s);
      }
      if (rc) break;
      if (hipError_t e = hipStreamSynchronize(s); e != hipSuccess) {
        rc = dev_fail(e, "tuning timing");
        break;
      }
      std::vector<float> t(nev);
      for (int r = 0; r < nev; ++r) hipEventElapsedTime(&t[r], ev[2 * r], ev[2 * r + 1]);
      std::sort(t.begin(), t.end());
      med = t[nev / 2];
      if (med < best.ms) {
        best.valid = true;
        best.ms = med;
        best.strategy = st;
        best.E = c.E;
        best.NT = c.NT;
        best.variant = c.V;
      }
    } else {
      ++nrej;  // failed the parity gate, or a launch shape the operator rejects
    }
    if (records && nrec < max_records) {
      shp_tune_record& R = records[nrec++];
      R.strategy = st;
      R.elems_per_wg = c.E;
      R.threads = c.NT;
      R.variant = c.V;
      R.ms = med;
      R.passed = pass ? 1 : 0;
    }
  }
  hipFree(flush);
  for (int i = 0; i < 2 * nev; ++i) hipEventDestroy(ev[i]);
  for (int i = 0; i < nstrat; ++i) set_tiling_raw(p, blk, opks[i], saved[i]);
  if (rc) return rc;
  if (n_records) *n_records = nrec;
  if (!best.valid) return fail(SHP_ERR_NOT_CONVERGED, "no candidate passed the parity gate");
  int bopk;
  opk_of(op, best.strategy, &bopk);
  set_tiling_raw(p, blk, bopk, Tiling{best.E, best.NT, best.variant});
  if (blk >= 0) {
    p->blocks[blk].auto_strategy[op] = best.strategy;
    p->blocks[blk].auto_src[op] = 1;
    p->blocks[blk].tuned[op] = best;
  } else {
    p->auto_mixed[op] = best.strategy;
    p->auto_mixed_src[op] = 1;
    p->tuned_mixed[op] = best;
  }
  res->strategy = best.strategy;
  res->elems_per_wg = best.E;
  res->threads = best.NT;
  res->variant = best.variant;
  res->ms = best.ms;
  res->n_candidates = ncand;
  res->n_rejected = nrej;
  return SHP_OK;
}

int shp_set_auto_strategy(shp_plan p, int blk, int op, int strategy) {
  if (int r = check_plan(p)) return r;
  if (blk < -1 || blk >= (int)p->blocks.size()) return fail(SHP_ERR_INVALID_ARG, "bad block %d", blk);
  if (op < 0 || op > SHP_OP_HELMHOLTZ) return fail(SHP_ERR_INVALID_ARG, "bad operator %d", op);
  if (strategy < SHP_SUMFAC || strategy > SHP_LOCALMAT) return fail(SHP_ERR_INVALID_ARG, "bad strategy");
  if (blk >= 0) {
    p->blocks[blk].auto_strategy[op] = strategy;
    p->blocks[blk].auto_src[op] = 1;
  } else {
    p->auto_mixed[op] = strategy;
    p->auto_mixed_src[op] = 1;
  }
  return SHP_OK;
}


// ---- cost model ------------------------------------------------------------

int shp_plan_set_model(shp_plan p, const float* params, int n_members, double mu, double sigma, void* stream) {
  if (int r = check_plan(p)) return r;
  if (!params) return fail(SHP_ERR_INVALID_ARG, "null params");
  if (n_members < 1 || n_members > MODEL_MAX_MEMBERS)
    return fail(SHP_ERR_INVALID_ARG, "n_members=%d outside [1,%d]", n_members, MODEL_MAX_MEMBERS);
  if (!std::isfinite(mu) || !(sigma > 0.0) || !std::isfinite(sigma))
    return fail(SHP_ERR_INVALID_ARG, "mu, sigma must be finite with sigma > 0");
  if (!p->ws) return fail(SHP_ERR_STATE, "no workspace bound");
  hipStream_t s = static_cast<hipStream_t>(stream);
  drop_model(p);
  hipError_t e = hipMemcpyAsync(p->ws + p->off_model, params, sizeof(float) * (size_t)n_members * p->mlp_nparam,
                                hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return dev_fail(e, "cost model upload");
  p->model_members = n_members;
  p->model_mu = mu;
  p->model_sigma = sigma;
  return SHP_OK;
}

// value of "key": <number> in a one-line JSON header, or NAN
static double json_number(const std::string& h, const char* key) {
  const std::string k = std::string("\"") + key + "\"";
  size_t i = h.find(k);
  if (i == std::string::npos) return NAN;
  i += k.size();
  while (i < h.size() && (h[i] == ' ' || h[i] == ':')) ++i;
  char* end = nullptr;
  const double v = std::strtod(h.c_str() + i, &end);
  return end == h.c_str() + i ? NAN : v;
}

int shp_plan_load_model(shp_plan p, const char* path, void* stream) {
  if (int r = check_plan(p)) return r;
  if (!path) path = std::getenv("SHP_MODEL_PATH");
  if (!path || !*path) return fail(SHP_ERR_INVALID_ARG, "no model path (argument NULL and SHP_MODEL_PATH unset)");
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(SHP_ERR_INVALID_ARG, "cannot open model file %s", path);
  std::string head;
  int c;
  while ((c = std::fgetc(f)) != EOF && c != '\n' && head.size() < 4096) head.push_back((char)c);
  std::vector<float> prm;
  bool ok = (c == '\n') && head.find("\"shp-mlp\"") != std::string::npos;
  const double nin = json_number(head, "nin"), nh = json_number(head, "nh"), np = json_number(head, "n_params");
  const double nm = json_number(head, "members"), mu = json_number(head, "mu"), sg = json_number(head, "sigma");
  ok = ok && nin == MLP_NIN && nh == 64 && np == p->mlp_nparam && nm >= 1 && nm <= MODEL_MAX_MEMBERS &&
       nm == std::floor(nm) && std::isfinite(mu) && sg > 0.0 && std::isfinite(sg);
  if (ok) {
    prm.resize((size_t)nm * p->mlp_nparam);
    ok = std::fread(prm.data(), sizeof(float), prm.size(), f) == prm.size() && std::fgetc(f) == EOF;
    for (float v : prm) ok = ok && std::isfinite(v);
  }
  std::fclose(f);
  if (!ok)
    return fail(SHP_ERR_INVALID_ARG, "%s is not a cost model file (one JSON header line with format \"shp-mlp\", "
                "nin 11, nh 64, n_params %d, members 1..%d, mu, sigma > 0; then members x n_params finite FP32 values)",
                path, p->mlp_nparam, MODEL_MAX_MEMBERS);
  if (!p->ws) return fail(SHP_ERR_STATE, "no workspace bound");
  hipStream_t s = static_cast<hipStream_t>(stream);
  drop_model(p);
  hipError_t e = hipMemcpyAsync(p->ws + p->off_model, prm.data(), sizeof(float) * prm.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return dev_fail(e, "cost model upload");
  p->model_members = (int)nm;
  p->model_mu = mu;
  p->model_sigma = sg;
  return SHP_OK;
}

int shp_model_choose(shp_plan p, int blk, int op, int* strategy, double* pred_ms, void* stream) {
  if (int r = check_plan(p)) return r;
  if (blk < 0 || blk >= (int)p->blocks.size()) return fail(SHP_ERR_INVALID_ARG, "bad block %d", blk);
  if (op < 0 || op > SHP_OP_HELMHOLTZ) return fail(SHP_ERR_INVALID_ARG, "bad operator %d", op);
  if (!strategy) return fail(SHP_ERR_INVALID_ARG, "null strategy");
  if (!model_op(op)) return fail(SHP_ERR_UNSUPPORTED, "the cost model predicts Laplacian and Helmholtz launches");
  if (!p->ws) return fail(SHP_ERR_STATE, "no workspace bound");
  if (p->model_members == 0) return fail(SHP_ERR_STATE, "no cost model loaded");
  const Block& B = p->blocks[blk];
  if (B.d.n_elem == 0) return fail(SHP_ERR_INVALID_ARG, "block %d is empty", blk);
  if (is_2d(B.d.shape)) return fail(SHP_ERR_UNSUPPORTED, "the cost model covers the 3D shapes");
  float pred[3];
  if (int r = model_predict(p, blk, pred, static_cast<hipStream_t>(stream))) return r;
  int best = SHP_SUMFAC_COLL;
  double bv = INFINITY;
  const double dof = (double)B.d.n_elem * B.NP;
  for (int j = 0; j < 3; ++j) {
    const bool av = strategy_available(B, op, MODEL_STRATS[j]) && std::isfinite(pred[j]);
    const double ms = av ? std::exp(p->model_mu + p->model_sigma * pred[j]) * dof * 1e3 : INFINITY;
    if (pred_ms) pred_ms[j] = ms;
    if (ms < bv) {
      bv = ms;
      best = MODEL_STRATS[j];
    }
  }
  *strategy = best;
  return SHP_OK;
}

// --- persisted tuning cache: one JSON object per line -----------------------

static std::string device_name() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string n = prop.gcnArchName;
  for (auto& c : n)
    if (c == '"' || c == '\\') c = '_';
  return n;
}

static int nbucket(long long n) {
  int b = 0;
  while (n > 1) {
    n >>= 1;
    ++b;
  }
  return b;
}

static std::string mixed_signature(shp_plan p) {
  std::string sig;
  for (const auto& B : p->blocks) {
    char buf[64];
    std::snprintf(buf, sizeof buf, "%s%d:%d:%d:%d", sig.empty() ? "" : ",", B.d.shape, B.d.P, nbucket(B.d.n_elem),
                  B.d.geom);
    sig += buf;
  }
  return sig;
}

static bool json_int(const std::string& l, const char* key, long long* v) {
  const std::string k = std::string("\"") + key + "\":";
  const size_t i = l.find(k);
  if (i == std::string::npos) return false;
  *v = std::strtoll(l.c_str() + i + k.size(), nullptr, 10);
  return true;
}

static bool json_str(const std::string& l, const char* key, std::string* v) {
  const std::string k = std::string("\"") + key + "\":\"";
  const size_t i = l.find(k);
  if (i == std::string::npos) return false;
  const size_t j = l.find('"', i + k.size());
  if (j == std::string::npos) return false;
  *v = l.substr(i + k.size(), j - i - k.size());
  return true;
}

int shp_tune_cache_save(shp_plan p, const char* path) {
  if (int r = check_plan(p)) return r;
  if (!path) return fail(SHP_ERR_INVALID_ARG, "null path");
  FILE* f = std::fopen(path, "a");
  if (!f) return fail(SHP_ERR_INVALID_ARG, "cannot open %s", path);
  const std::string dev = device_name();
  for (const auto& B : p->blocks)
    for (int op = 0; op < 7; ++op) {
      const auto& t = B.tuned[op];
      if (!t.valid) continue;
      std::fprintf(f,
                   "{\"kind\":\"block\",\"device\":\"%s\",\"prec\":\"fp64\",\"op\":%d,\"shape\":%d,\"P\":%d,\"Q\":%d,"
                   "\"nbucket\":%d,\"geom\":%d,\"strategy\":%d,\"E\":%d,\"NT\":%d,\"variant\":%d,\"us\":%lld}\n",
                   dev.c_str(), op, B.d.shape, B.d.P, B.d.Q, nbucket(B.d.n_elem), B.d.geom, t.strategy, t.E, t.NT,
                   t.variant, (long long)(t.ms * 1e3));
    }
  for (int op = 0; op < 7; ++op) {
    const auto& t = p->tuned_mixed[op];
    if (!t.valid) continue;
    std::fprintf(f,
                 "{\"kind\":\"mixed\",\"device\":\"%s\",\"prec\":\"fp64\",\"op\":%d,\"blocks\":\"%s\",\"strategy\":%d,"
                 "\"E\":%d,\"NT\":%d,\"variant\":%d,\"us\":%lld}\n",
                 dev.c_str(), op, mixed_signature(p).c_str(), t.strategy, t.E, t.NT, t.variant, (long long)(t.ms * 1e3));
  }
  std::fclose(f);
  return SHP_OK;
}

int shp_tune_cache_load(shp_plan p, const char* path, int* n_applied) {
  if (int r = check_plan(p)) return r;
  if (!path) return fail(SHP_ERR_INVALID_ARG, "null path");
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(SHP_ERR_INVALID_ARG, "cannot open %s", path);
  const std::string dev = device_name();
  int applied = 0;
  char line[1024];
  while (std::fgets(line, sizeof line, f)) {
    const std::string l(line);
    std::string kind, d, prec;
    long long op, st, E, NT, V;
    if (!json_str(l, "kind", &kind) || !json_str(l, "device", &d) || !json_str(l, "prec", &prec)) continue;
    if (d != dev || prec != "fp64") continue;
    if (!json_int(l, "op", &op) || !json_int(l, "strategy", &st) || !json_int(l, "E", &E) || !json_int(l, "NT", &NT) ||
        !json_int(l, "variant", &V))
      continue;
    if (op < 0 || op > 6 || st < SHP_SUMFAC || st > SHP_LOCALMAT || E < 1 || E > 64 || NT < 64 || NT > 512 ||
        NT % 64 || V < 0 || V > 4)
      continue;  // a corrupt entry is skipped
    int opk;
    if (opk_of((int)op, (int)st, &opk)) continue;
    if (kind == "block") {
      long long sh, P, Q, nb, geom;
      if (!json_int(l, "shape", &sh) || !json_int(l, "P", &P) || !json_int(l, "Q", &Q) || !json_int(l, "nbucket", &nb) ||
          !json_int(l, "geom", &geom))
        continue;
      for (auto& B : p->blocks) {
        if (B.d.shape != sh || B.d.P != P || B.d.Q != Q || nbucket(B.d.n_elem) != nb || B.d.geom != geom) continue;
        if (op_lds_bytes(B.d.shape, B.d.P, opk, (int)E, (int)V) > LDS_LIMIT) continue;
        B.tiling[opk] = Tiling{(int)E, (int)NT, (int)V};
        B.auto_strategy[op] = (int)st;
        B.auto_src[op] = 1;
        ++applied;
      }
    } else if (kind == "mixed") {
      std::string sig;
      if (!json_str(l, "blocks", &sig) || sig != mixed_signature(p)) continue;
      p->mixed[opk] = Tiling{(int)E, (int)NT, (int)V};
      p->mixed_dirty[opk] = true;
      p->auto_mixed[op] = (int)st;
      p->auto_mixed_src[op] = 1;
      ++applied;
    }
  }
  std::fclose(f);
  if (n_applied) *n_applied = applied;
  return SHP_OK;
}

}  // extern "C"
