// Internal declarations of libshp shared by the host API and the kernel
// launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "shp_layout.hpp"

struct shp_plan_s;

namespace shp {

struct OpArgs;
struct Tile;
struct GeomArgs;
struct LocalMatArgs;
struct AffineMatArgs;
struct LocalXformArgs;

// Static per-block data of a mixed launch (device copy in the workspace).
struct BlockStatic {
  const double* tab;
  const int* itab;
  const double* fac;
  const double* dxi;
  const float* tabf;    // the reference tables rounded to FP32
  const double* xco;    // iso-parametric blocks: coordinate coefficients [n_elem][3][N_P]
  const double* wref;   // iso-parametric blocks: w / prod (1 - eta_d)^alpha_d per point [Q^3]
  const float* fac32;   // FP32 copy of fac for the FP32 actions, or null
  long long n_elem;
  long long coeff_off;  // element offset * N_P of the block in whole-mesh coefficient buffers
  long long phys_off;   // element offset * N_Q in whole-mesh point buffers
  int shape;
  int E;
};

// host tables (shp_tables.cpp)
void gauss_jacobi(int Q, double a, double b, double* x, double* w);
void gauss_lobatto(int Q, double* x, double* w);
void gauss_radau_jacobi(int Q, double a, double b, double* x, double* w);
void rule_1d(int Q, int alpha, int pts, double* x, double* w);
void build_tables(int sh, int P, int pts, std::vector<double>& tab, std::vector<int>& itab);
void reference_points(int sh, int Q, int pts, double* xi, double* w);
void build_localmat(int sh, int P, int pts, std::vector<double>& bcat, int& Q3p, int& Kp);
// dense collocation derivative matrices of the tensor points, [3][Q3p][Q3p]
// (d/d eta_d of the Lagrange interpolant; zero padding past Q^3)
void build_dense_deriv(int sh, int P, int pts, std::vector<double>& dm, int& Q3p);
// tables of the sum-factorised Helmholtz diagonal (see shp_tables.cpp)
void build_diag_tables(int sh, int P, int pts, std::vector<double>& dt, std::vector<int>& di, int& n1, int& n12);
// diag(lambda M + L) of n_elem elements of one block from its factors
// fac [n_elem][NFAC][Q^3]: one work-group per element; diag [n_elem][NP]
hipError_t launch_helm_diag(const double* fac, const double* dt, const int* di, int Q, int n1, int n12, int NP,
                            long long n_elem, double lambda, double* diag, hipStream_t s);
constexpr int LOCALMAT_MAX_P = 4;  // dense reference matrices only at low order
// affine blocks: the 7 reference matrices of H = sum_k c_{e,k} A_k in MFMA
// fragment order (Kp = modes padded to 16, 7 Kp^2 values); coefficients per element
// (|J|, |J| K00, |J| K01, |J| K02, |J| K11, |J| K12, |J| K22), K = J^-1 J^-T
void build_affine_mats(int sh, int P, int pts, std::vector<double>& acat, int& Kp);
constexpr int NAFF = 7;
// the same matrices as sums of BF16_PARTS bfloat16 parts (each the rounding of
// what the previous parts leave) for the split-BF16 MFMA kernels: columns
// kappa = k NPp + n (N_P padded to NPp, a multiple of 8), KS steps of 32,
// rows in MB blocks of 16; A operand of v_mfma_f32_16x16x32_bf16 with lane l
// holding row 16 mb + l%16 and columns 32 kb + 8 (l/16) + j, j = 0..7:
//   frag[(((kb MB + mb) BF16_PARTS + part) 64 + l) 8 + j]
constexpr int BF16_PARTS = 3;
void build_affine_mats_bf16(int sh, int P, int pts, std::vector<uint16_t>& frag, int& NPp, int& KS, int& MB);
// the affine local-matrix action (opk = OPK_MASS_LM, OPK_LAP_LM, OPK_HELM_LM)
// of one block in split-BF16 with nparts = 2 or 3 parts, FP32 in/out; afrag
// from build_affine_mats_bf16 (16-byte fragments), coef [n][7]
struct bf16_frag {
  uint16_t h[8];
};
hipError_t launch_localmat_affine_bf16(int sh, int P, int opk, int nparts, const bf16_frag* afrag, const double* coef,
                                       const float* in, float* out, long long n_elem, double lambda, hipStream_t s);
// the same for nblk <= 8 blocks of one order P in one launch (per-block
// arrays of shapes, fragments, coefficients, in/out pointers and sizes)
hipError_t launch_localmat_affine_bf16_mesh(int P, int opk, int nparts, int nblk, const int* shape,
                                            const bf16_frag* const* afrag, const double* const* coef,
                                            const float* const* in, float* const* out, const long long* n_elem,
                                            double lambda, hipStream_t s);

// launchers (shp_k_*.hip); return hipSuccess or the launch error
size_t op_lds_bytes(int sh, int P, int opk, int E, int variant);
hipError_t launch_block(int sh, int P, int opk, const OpArgs& a, int threads, int persist, hipStream_t s);
hipError_t launch_geometry(int sh, int P, const GeomArgs& g, hipStream_t s);
hipError_t launch_localmat(int sh, int P, int opk, const LocalMatArgs& a, hipStream_t s);
hipError_t launch_localmat_affine(int sh, int P, int opk, const AffineMatArgs& a, hipStream_t s);
// every affine block of one order in one launch (nblk <= 8, blocks' args in order)
hipError_t launch_localmat_affine_mesh(int P, int opk, int nblk, const int* shape, const AffineMatArgs* blk,
                                       hipStream_t s);
struct AffineMatArgs32;
hipError_t launch_localmat_affine_f32_mesh(int P, int opk, int nblk, const int* shape, const AffineMatArgs32* blk,
                                           hipStream_t s);
// the affine local-matrix action in FP32 on the FP32 matrix cores: afrag the
// FP64 fragments rounded to FP32 (same order), FP32 in/out
hipError_t launch_localmat_affine_f32(int sh, int P, int opk, const float* afrag, const double* coef, const float* in,
                                      float* out, long long n_elem, double lambda, hipStream_t s);
// local-matrix BwdTrans, IProduct, PhysDeriv, IProductDeriv (opk OPK_*_LM)
hipError_t launch_localmat_xform(int sh, int P, int opk, const LocalXformArgs& a, hipStream_t s);
hipError_t launch_affine_coef(const double* jac, double* coef, long long n, int* status, hipStream_t s);
// whole-mesh advection-diffusion-reaction action (FP64, geometry-prefetch launch)
// and the advection factors of one block
hipError_t launch_adr(int P, const BlockStatic* blocks, const Tile* tiles, int ntiles, const double* in, double* out,
                      const double* adv, double lambda, int threads, size_t lds, int E, hipStream_t s);
hipError_t launch_adv_factors(const double* fac, const double* dxi, const double* vel, long long vstride, double* adv,
                              long long n_elem, int Q3, hipStream_t s);
hipError_t launch_mixed(int P, int opk, const BlockStatic* blocks, const Tile* tiles, int ntiles, const double* in,
                        double* out, long long in_cs, long long out_cs, double lambda, int threads, size_t lds, int E,
                        int persist, hipStream_t s);
// iso-parametric blocks of one order P: Laplacian/Helmholtz action with the
// geometry recomputed from coordinates (tile list, or one block's tiles of E
// elements when blk_only >= 0), and the geometry check of one block
hipError_t launch_iso(int P, int opk, const BlockStatic* blocks, const Tile* tiles, int ntiles, const double* in,
                      double* out, double lambda, int threads, size_t lds, int E, int blk_only, long long nwg,
                      hipStream_t s);
hipError_t launch_iso_check(int P, const BlockStatic* blocks, int blk, int E, long long nwg, int threads, size_t lds,
                            int* status, hipStream_t s);
// 2D shapes (quadrilateral, triangle): tables, points, and the launchers
// (shp_k_2d_*.hip): block launch, whole-mesh launch, geometry, LDS bytes
void build_tables2d(int sh, int P, int pts, std::vector<double>& tab);
void reference_points2d(int sh, int Q, int pts, double* xi, double* w);
hipError_t launch_block2d(int sh, int P, int opk, const OpArgs& a, int threads, hipStream_t s);
hipError_t launch_mixed2d(int P, int opk, const BlockStatic* blocks, const Tile* tiles, int ntiles, const double* in,
                          double* out, long long in_cs, long long out_cs, double lambda, int threads, size_t lds,
                          int E, hipStream_t s);
hipError_t launch_geometry2d(int sh, int P, const double* tab, const double* jac, double* fac, double* dxi,
                             long long n_elem, int affine, int* status, hipStream_t s);
// LDS of the 2D launch of operator opk with E elements on threads threads
// (the fused Laplacian / Helmholtz tile when its points fit the registers)
size_t lds_bytes_2d(int sh, int P, int E, int opk = 0 /* the backward transform */, int threads = 256);
// reference weights w / prod (1 - eta_d)^alpha_d of the tensor points [Q^3]
void build_ref_weights(int sh, int P, int pts, std::vector<double>& wref);
// FP32 contractions (whole-mesh collocated Laplacian/Helmholtz, prefetch variant)
size_t lds_bytes_f32(int sh, int P, int E);
hipError_t launch_mixed_f32(int P, int opk, const BlockStatic* blocks, const Tile* tiles, int ntiles, const float* in,
                            float* out, double lambda, int threads, size_t lds, int E, bool fac32, hipStream_t s);
// round n FP64 values to FP32
hipError_t launch_round_f32(const double* a, float* b, long long n, hipStream_t s);
// persistent launches: CUs of the current device, grid = occupancy * CUs, and
// the register slots per thread of the metric stage (2, 4, 8; 0 = too many)
int num_cus();
long long persistent_grid(const void* kernel, int threads, size_t lds);
int points_per_thread(long long points, int threads);
// max |a-b| and max |b| into out[0], out[1] (bit patterns of non-negative doubles)
hipError_t launch_maxdiff(const double* a, const double* b, long long n, unsigned long long* out, hipStream_t s);

constexpr int MAX_P = 10;
constexpr size_t LDS_LIMIT = 160 * 1024;

// Plan queries for the solver (shp_api.cpp): the mesh's coefficient count,
// the Helmholtz diagonal, and the error text reported by shp_last_error.
long long plan_total_coeff(const shp_plan_s* p);
// diag(lambda M + L) of every element, whole-mesh layout (sum-factorised, FP64)
int plan_helm_diag(shp_plan_s* p, double lambda, double* diag, hipStream_t s);
int plan_check_solve(shp_plan_s* p, int inner_prec);  // workspace, geometry, FP32 needs one P
int set_error(int code, const char* msg);

}  // namespace shp
