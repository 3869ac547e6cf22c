/*
 * shp.h - C ABI of libshp, matrix-free elemental spectral/hp operators on one
 * AMD MI355X (gfx950).
 *
 * The operators are those of the Helmholtz problem's elemental Galerkin system
 * H^e u = f (Sec. 2.1): the backward transform u = B x, the inner product with
 * the basis B^T W f, the inner product with the basis derivatives, the physical
 * derivative, and the mass, Laplacian and Helmholtz actions y = (lambda M + L) x
 * with M = B^T W B (Sec. 2.2, eq. mass) and L the weak Laplacian (Sec. 2.2,
 * eq. Lap).  Elements are hexahedra, prisms, pyramids and tetrahedra with the
 * collapsed-coordinate (Duffy) tensorial modal basis (Sec. 2.3).  A "block" is
 * a batch of elements of one shape, order P, quadrature Q and mapping type,
 * stored with a constant stride (Sec. 3.3, blocks; App. A.2 Field/Block).
 *
 * Conventions
 * -----------
 * - Device pointers point to HIP device memory owned by the caller.  Host
 *   pointers are marked "host".  The library never frees caller memory.
 * - stream is a hipStream_t passed as void*; NULL means the default stream.
 *   Work is enqueued on it; calls return before the work completes unless
 *   stated otherwise.
 * - Layouts (Sec. App. A.2, default layout: points or modes fastest, then
 *   elements, then components):
 *     coefficients  [n_elem][N_P]      modes (p,q,r) lexicographic, r fastest
 *     point values  [n_elem][N_Q]      N_Q = Q^3, point (i,j,k) at (i*Q+j)*Q+k
 *     vector field  [3][n_elem][N_Q]   component slowest
 *   A whole-mesh call (blk = -1) uses block-concatenated buffers: block b
 *   starts at the element offset given by shp_block_offsets; vector fields are
 *   [3][total points].
 * - Mode sets (modified C0 basis; A_p, C_{k,r} built on Jacobi polynomials):
 *     hex   A_p A_q A_r, 0<=p,q,r<=P
 *     prism A_p A_q C_{p,r}, r<=P-p
 *     pyr   A_p A_q C_{max(p,q),r}, r<=P-max(p,q)
 *     tet   A_p C_{p,q} C_{p+q,r}, p+q+r<=P
 *   with the collapsed-vertex modes prism (0,q,1), pyramid (0,0,1), tet (0,0,1)
 *   and (0,1,r) independent of the collapsed coordinate(s).
 * - Quadrature: Q points per direction; Gauss-Lobatto-Legendre in directions
 *   that are not collapsed, and in a direction collapsed alpha times (prism
 *   eta3: 1, pyramid eta3: 2, tet eta2: 1, eta3: 2) Gauss-Jacobi(alpha,0)
 *   (SHP_PTS_GJ, the default) or Gauss-Radau-Jacobi(alpha,0) with the node
 *   eta = -1 (SHP_PTS_RADAU).  Hexahedra have no collapsed direction, so the
 *   choice does not change them.
 *   This build supports 1 <= P <= 10 and Q = P + 2 (Sec. 2.1: at least P+2
 *   points per direction).
 *
 * Errors: every call returns SHP_OK (0) or a negative code; no C++ exception
 * crosses the ABI.  shp_last_error() returns a thread-local message describing
 * the last failure of the calling thread.  Arguments are validated before any
 * HIP call, so validation errors leave device state untouched.
 */
#ifndef SHP_H
#define SHP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SHP_OK 0
#define SHP_ERR_INVALID_ARG (-1)   /* null pointer, out-of-range enum or index */
#define SHP_ERR_UNSUPPORTED (-2)   /* P outside [1,10], Q != P+2, mixed P in one launch */
#define SHP_ERR_BAD_GEOMETRY (-3)  /* det(d x/d xi) <= 0 or non-finite at some point */
#define SHP_ERR_WORKSPACE (-4)     /* workspace missing, misaligned or too small */
#define SHP_ERR_STATE (-5)         /* call out of order (e.g. apply before geometry) */
#define SHP_ERR_DEVICE (-6)        /* a HIP runtime call failed (message included) */
#define SHP_ERR_NOT_CONVERGED (-7) /* an iterative solve did not reach its tolerance */

/* Shapes.  The 2D shapes follow the two-dimensional formulation (Sec. 2.2)
 * and the triangle as a collapsed square (Sec. 2.3): modes (p,q), q fastest,
 * quadrilateral A_p(eta1) A_q(eta2) with 0 <= p,q <= P (N_P = (P+1)^2),
 * triangle A_p(eta1) C_{p,q}(eta2) with p+q <= P (N_P = (P+1)(P+2)/2) and the
 * collapsed-vertex mode (0,1) = v1(eta2); Q^2 points (i,j) at i*Q + j, GLL
 * in eta1 and in the quadrilateral's eta2, Gauss-Jacobi(1,0) (or Radau) in the
 * triangle's eta2.  Geometry d x_i/d xi_j at component i*2 + j: curved
 * [n_elem][4][Q^2], affine [n_elem][4]; vector fields [2][n][Q^2].  A plan
 * holds 2D or 3D blocks, not both.  2D blocks run every operator with the
 * collocated sum-factorisation (SHP_AUTO or SHP_SUMFAC_COLL, per block or as
 * one whole-mesh launch); tuning, launch shapes, the cost model, FP32
 * contractions, the solve, iso-parametric maps and the
 * advection-diffusion-reaction action cover the 3D shapes only
 * (SHP_ERR_UNSUPPORTED). */
typedef enum { SHP_HEX = 0, SHP_PRISM = 1, SHP_PYR = 2, SHP_TET = 3, SHP_QUAD = 4, SHP_TRI = 5 } shp_shape;
/* Mapping of a block's elements.  SHP_AFFINE and SHP_CURVED take d x/d xi
 * and keep 7 FP64 geometric factors per point in the workspace (Sec. 4:
 * precomputed factors).  SHP_ISOPARAM takes the map as a polynomial of the
 * solution's degree in the block's own basis (Sec. 2.1: J is then polynomial;
 * Sec. 4: iso-parametric curvilinear elements), 3 N_P FP64 coordinate
 * coefficients per element, and the collocated Laplacian and Helmholtz
 * actions rebuild J and the factors in FP64 at every point in every launch:
 * 24 N_P bytes per element in place of 56 Q^3.  Iso-parametric blocks support
 * the backward transform and those two actions (FP64, SHP_SUMFAC_COLL or
 * SHP_AUTO; a whole-mesh launch only over iso-parametric blocks of one P);
 * other operators, precisions, the solve and the advection-diffusion-reaction
 * action return SHP_ERR_UNSUPPORTED for them. */
typedef enum { SHP_AFFINE = 0, SHP_CURVED = 1, SHP_ISOPARAM = 2 } shp_geom;
typedef enum { SHP_PTS_GJ = 0, SHP_PTS_RADAU = 1 } shp_points;
typedef enum {
  SHP_OP_BWDTRANS = 0,       /* [n][N_P] -> [n][N_Q]   u = B x                      */
  SHP_OP_IPRODUCT = 1,       /* [n][N_Q] -> [n][N_P]   y = B^T W f                  */
  SHP_OP_PHYSDERIV = 2,      /* [n][N_Q] -> [3][n][N_Q] d u/d x_i of the interpolant */
  SHP_OP_IPRODUCT_DERIV = 3, /* [3][n][N_Q] -> [n][N_P] y = sum_i (d_i B)^T W f_i   */
  SHP_OP_MASS = 4,           /* [n][N_P] -> [n][N_P]   y = M x                      */
  SHP_OP_LAPLACIAN = 5,      /* [n][N_P] -> [n][N_P]   y = L x                      */
  SHP_OP_HELMHOLTZ = 6       /* [n][N_P] -> [n][N_P]   y = (lambda M + L) x         */
} shp_op;
typedef enum {
  SHP_AUTO = 0,        /* tuned or set choice, else the cost model's (when one is
                          loaded, Laplacian and Helmholtz), else SHP_SUMFAC_COLL */
  SHP_SUMFAC = 1,      /* sum-factorisation, non-collocated derivatives (Alg. 5)  */
  SHP_SUMFAC_COLL = 2, /* sum-factorisation, collocated derivatives (Alg. 6)      */
  SHP_LOCALMAT = 3     /* local matrices on FP64 MFMA (Alg. 1, StdMat), P <= 4
                          (higher orders: SHP_ERR_UNSUPPORTED).  BwdTrans is one
                          GEMM U = B X over the block; IProduct B^T (jw F);
                          IProductDeriv sum_d (d_d B)^T (jw sum_i d eta_d/d x_i
                          F_i); PhysDeriv applies the dense collocation
                          derivative matrices of the tensor points (its input is
                          values at the points) and the metric d eta/d x.  Mass,
                          Laplacian and Helmholtz: curved blocks apply
                          [B; d_d B] with the per-point metric (the
                          non-collocated form); affine blocks apply
                          H_e = lambda |J| A_0 + sum_k c_{e,k} A_k with 7 shared
                          reference matrices (mass and the xi-space stiffness
                          blocks) and 7 coefficients per element */
} shp_strategy;

typedef struct {
  int shape;       /* shp_shape */
  int P;           /* polynomial order, 1..10 */
  int Q;           /* points per direction, P + 2 */
  int64_t n_elem;  /* elements in the block, >= 0 */
  int geom;        /* shp_geom: SHP_CURVED takes d x/d xi per point, SHP_AFFINE per element,
                      SHP_ISOPARAM coordinate coefficients per element */
  int pts;         /* shp_points of the collapsed directions; 0 (SHP_PTS_GJ) by default */
} shp_block_desc;

typedef struct shp_plan_s* shp_plan;

/* Number of modes N_P of a shape at order P (Sec. 2.1, N_P; the mode sets above). */
int shp_num_modes(int shape, int P, int* n_modes /* host out */);

/* Number of quadrature points N_Q = Q^3 (Q^2 for the 2D shapes): every
 * shape takes the tensor product of Q points per direction (Sec. 2.1, tensor
 * quadrature; the collapsed shapes keep the full tensor grid in eta, Sec. 2.3). */
int shp_num_points(int shape, int Q, int* n_points /* host out */);

/* The block's quadrature points in reference coordinates and their weights
 * (Sec. 2.1 tensor quadrature; Sec. 2.3 collapse) for point set pts
 * (shp_points).  xi: host [3][Q^3], component slowest ([2][Q^2] for the 2D
 * shapes); w: host [Q^3] (or [Q^2]) = product of the 1D weights, may be NULL.  The mesh's Jacobian d x/d xi is
 * expected at exactly these points. */
int shp_quadrature(int shape, int Q, int pts, double* xi /* host out */, double* w /* host out or NULL */);

/* The vertex modes of a shape at order P (Sec. 2.3: the collapsed-vertex
 * construction; each is one at its vertex and zero at the others): idx (host
 * out, at most 8) the mode index of each, xi (host out [8][3]) the reference
 * coordinates of that vertex, n_vertices (host out) their number (hex 8,
 * prism 6, pyramid 5, tet 4).  Iso-parametric coordinates of straight-sided
 * elements are the vertex positions on these modes and zero elsewhere. */
int shp_vertex_modes(int shape, int P, int* idx /* host out */, double* xi /* host out */,
                     int* n_vertices /* host out */);

/* Create a plan for nblk blocks (host metadata only; copies blk). */
int shp_plan_create(shp_plan* plan /* host out */, const shp_block_desc* blk /* host [nblk] */,
                    int nblk);

/* Device workspace the plan needs: reference tables, geometric factors and
 * launch metadata.  The caller allocates it (256-byte aligned). */
int shp_plan_workspace_bytes(shp_plan plan, size_t* bytes /* host out */);

/* Attach a caller-owned workspace and upload the reference tables into it
 * (enqueued on stream).  The workspace must stay allocated while the plan is
 * used.  Re-binding invalidates the geometry of every block. */
int shp_plan_bind_workspace(shp_plan plan, void* ws, size_t ws_bytes, void* stream);

/* Geometric factors of block blk (Sec. 4 precomputed geometric factors; the
 * chain rule of Sec. 2.1 and the collapse Jacobian of Sec. 2.3), computed in
 * FP64 on the device from jac = d x_i/d xi_j:
 *   SHP_CURVED: jac [n_elem][9][Q^3], component i*3+j, at shp_quadrature points;
 *   SHP_AFFINE: jac [n_elem][9], constant per element (also the 7 coefficients
 *               |J| and |J| (J^-1 J^-T)_ab per element of the local-matrix
 *               strategy, for P <= 4);
 *   SHP_ISOPARAM: jac [n_elem][3][N_P], the coordinate coefficients X of
 *               x_c = sum_m X[e][c][m] phi_m, copied into the workspace; the
 *               geometry they give is checked at every point with the FP64
 *               reconstruction the actions use.
 * Synchronises stream to report SHP_ERR_BAD_GEOMETRY when det <= 0 or a value
 * is not finite.  Not safe to call concurrently with applies of the plan. */
int shp_plan_set_geometry(shp_plan plan, int blk, const double* jac /* device */, void* stream);

/* Element offset of block blk in whole-mesh coefficient and point buffers:
 * coefficients of block blk start at element coeff_off (in units of doubles:
 * sum over earlier blocks of n_elem*N_P), points at phys_off (sum of n_elem*N_Q). */
int shp_block_offsets(shp_plan plan, int blk, int64_t* coeff_off /* host out */,
                      int64_t* phys_off /* host out */);

/* Apply operator op to block blk, or to the whole mesh with blk = -1 (one
 * launch over all blocks when they share P and Q; tiles of all blocks are
 * ordered longest first).  in/out are FP64 device buffers in the layouts
 * above; in and out must not overlap.  lambda is used by SHP_OP_HELMHOLTZ.
 * The first whole-mesh apply of an operator after the workspace is bound (and
 * the first after its tiling changes) writes that operator's tile list into the
 * workspace and synchronises the stream; otherwise the call is read-only on
 * the workspace and applies on different streams may run concurrently.  Make
 * one whole-mesh apply of each operator first before applying concurrently. */
int shp_apply(shp_plan plan, int blk, int op, int strategy, const double* in /* device */,
              double* out /* device */, double lambda, void* stream);

/* Contraction precision: SHP_FP64, or SHP_FP32 (FP32 data, tables and
 * accumulation in the sum-factorisation stages; the FP64 geometric factors are
 * applied in FP64 and the results rounded, or, once shp_plan_set_fp32_factors
 * has attached an FP32 copy of the factors, that copy is read and the metric
 * applied in FP32), or split BF16 on the BF16 matrix cores with FP32
 * accumulation (the paper's fields take float or double, App. A.2; BF16 is
 * this library's addition): every operand is a sum of bfloat16 parts, each
 * the bfloat16 rounding of what the previous parts leave, and a product keeps
 * the part products of order below the part count:
 *   SHP_BF16    three parts, six products per product (about 2^-24 of |a||b|);
 *   SHP_BF16X3  two parts, three products (about 2^-16 of |a||b|). */
typedef enum { SHP_FP64 = 0, SHP_FP32 = 1, SHP_BF16 = 2, SHP_BF16X3 = 3 } shp_prec;

/* shp_apply with a contraction precision: in/out are device arrays of doubles
 * (SHP_FP64) or floats (the others) in the same layouts.  SHP_FP32 with
 * strategy SHP_AUTO or SHP_SUMFAC_COLL covers the collocated Laplacian and
 * Helmholtz actions as a whole-mesh launch (blk = -1, one P for all blocks);
 * with SHP_AUTO and blk = -1 it takes the FP32 local matrices below instead
 * when the plan's whole-mesh choice for the operator is SHP_LOCALMAT and
 * every block is affine with P <= 4.
 * SHP_BF16 and SHP_BF16X3 (strategy SHP_AUTO or SHP_LOCALMAT), and SHP_FP32
 * with strategy SHP_LOCALMAT (on v_mfma_f32_16x16x4f32, the matrices rounded to
 * FP32), cover the mass, Laplacian and Helmholtz actions of affine 3D blocks
 * with P <= 4 in the local-matrix form (Sec. 3.3.1): y_e = sum_k c_{e,k} A_k x_e
 * as one contraction over the 7 reference matrices, with B operand c_{e,k} x_e
 * rounded to FP32 (before the split for BF16); one block (blk >= 0, its own
 * buffers) or every block (blk = -1, whole-mesh buffers; the BF16 kernels take
 * every block of one order in one launch).  Other combinations return
 * SHP_ERR_UNSUPPORTED. */
int shp_apply_prec(shp_plan plan, int blk, int op, int strategy, int prec, const void* in /* device */,
                   void* out /* device */, double lambda, void* stream);

/* FP32 copy of the geometric factors for the FP32 actions (the data type of
 * the paper's fields is a template parameter, float or double; here the
 * factors of the FP32 inner operator may be float too).  The FP32 action
 * streams 8 N_P + 56 Q^3 bytes per element with FP64 factors, 8 N_P + 28 Q^3
 * with this copy.  fac32: device floats [sum over blocks of n_elem 7 Q^3],
 * blocks concatenated like point buffers, each element's 7 factors as in the
 * plan ([7][Q^3]); owned by the caller, 4-byte aligned, kept unchanged and
 * alive while attached.  The call rounds the plan's FP64 factors into it
 * (every block's geometry must be set; 3D blocks with precomputed factors
 * only), and shp_plan_set_geometry refreshes its block's part while attached.
 * From then on SHP_FP32 actions, and so the FP32 inner iterations of
 * shp_helmholtz_solve, read it; the FP64 actions and residuals are
 * unchanged.  fac32 = NULL detaches it.  Synchronises stream. */
int shp_plan_set_fp32_factors(shp_plan plan, float* fac32 /* device */, void* stream);

/* ---- Advection-diffusion-reaction action --------------------------------
 * The collocated form of the Helmholtz action carries over to any operator
 * tested against the basis or its derivatives (Sec. 2.2.1, after eq. helm1);
 * here the linear advection-diffusion-reaction operator
 *   y_m = sum_e integral phi_m (lambda u + b . grad u) + grad phi_m . grad u,
 * u = sum_n x_n phi_n, with a velocity field b given at the quadrature points.
 * At the points the advection term adds sum_d a_d D_d u to the reaction term
 * lambda jw u before the restriction B^T, with the advection factors
 * a_d = jw sum_i b_i d eta_d / d x_i (FP64, three per point). */

/* Advection factors of every block from the velocity b at the points.
 * vel: device FP64 [3][total points] (component slowest, blocks concatenated
 * as in shp_block_offsets); adv: device FP64 [3 * total points], block b's
 * factors from 3 * (its point offset), [n_elem][3][N_Q] within the block.
 * Needs every block's geometry.  Enqueued on stream. */
int shp_advection_factors(shp_plan plan, const double* vel /* device */, double* adv /* device */, void* stream);

/* Whole-mesh advection-diffusion-reaction action in FP64 with the collocated
 * sum-factorisation (one launch; every block of one P): in/out are whole-mesh
 * coefficient buffers, adv the factors from shp_advection_factors.  With adv
 * all zero the result equals the Helmholtz action.  The first call writes the
 * operator's tile list into the workspace as shp_apply does. */
int shp_apply_adr(shp_plan plan, const double* adv /* device */, const double* in /* device */,
                  double* out /* device */, double lambda, void* stream);

/* ---- Helmholtz solve with mixed precision ------------------------------
 * Solves H x = b for the elemental (unassembled, block-diagonal) Helmholtz
 * operator H = lambda M + L of every element of the plan (Sec. 2, the
 * Helmholtz problem; each H_e is symmetric positive definite for lambda > 0).
 * Both calls below use a device scratch buffer ws, 256-byte aligned, of at
 * least shp_solve_workspace_bytes, owned by the caller and not kept after
 * return; both synchronise stream. */
int shp_solve_workspace_bytes(shp_plan plan, size_t* bytes /* host out */);

/* Jacobi preconditioner: diag[i] = H_e[m][m] for the coefficient i = mode m of
 * element e, in the whole-mesh layout (device FP64 out, [total coefficients]).
 * Sum-factorised in FP64 from the geometric factors: with the collocated
 * derivatives (Sec. 2.2.1, eq. helm1) each mode's values and derivatives at
 * the points are products of its 1D factors, so H_mm is each of the 7 factor
 * fields contracted direction by direction with squared 1D values (about one
 * operator action of work).  ws is validated as for the solve but not used. */
int shp_helmholtz_diag(shp_plan plan, double lambda, double* diag /* device out */, void* ws /* device */,
                       size_t ws_bytes, void* stream);

/* Mixed-precision solve: a Jacobi-preconditioned conjugate-gradient iteration
 * whose operator actions, vectors and updates run in inner_prec (SHP_FP64;
 * SHP_FP32 through shp_apply_prec's SHP_AUTO action; SHP_BF16 or SHP_BF16X3
 * through its split-BF16 affine local matrices, FP32 vectors) with FP64 dot
 * products, refined in FP64
 * by reliable updates: whenever the recursive residual has fallen by the factor
 * inner_tol since the last update (or predicts the tolerance), the correction
 * accumulated in inner_prec is added to x in FP64 and the residual is replaced
 * by r = b - H x from the FP64 action; the iteration then continues from it
 * with its search direction kept, or restarts the direction when the true
 * residual exceeds the recursive one twice over (rounding near the floor of
 * the FP64 residual).  The FP64 actions follow the plan's SHP_AUTO choice for
 * the whole mesh (tuned, set with shp_set_auto_strategy, or a loaded cost
 * model's; by default the collocated sum-factorisation).  The residual enters the inner precision scaled by
 * 1/max|r_0|.  An update that does not lower the FP64 residual is undone
 * (the direction restarts from the previous x); five in a row end the solve,
 * as do max_outer updates or max_inner iterations, and x then holds the
 * iterate with the smallest FP64 residual.  Updates come at least every 2000
 * iterations.
 *
 * diag: from shp_helmholtz_diag with the same lambda.  b, x: device FP64
 * arrays [total coefficients] in the whole-mesh layout; x holds the initial
 * guess on entry and the solution on return.  Stops when ||b - H x||_2 <= tol
 * ||b||_2 for the FP64 residual (checked on entry and at every update), after
 * max_outer updates or max_inner iterations in all (convergence is tested
 * every 10 iterations), or on error.  Returns SHP_ERR_NOT_CONVERGED (stats
 * filled in) when the tolerance is not reached, SHP_ERR_INVALID_ARG for b = 0,
 * SHP_ERR_UNSUPPORTED for an FP32 request on a plan with more than one P or a
 * BF16 request on a plan with a block that is not affine with P <= 4. */
typedef struct {
  int outer_iters;     /* reliable updates (FP64 residual replacements) taken */
  int inner_iters;     /* CG iterations in all */
  int converged;       /* 1 when ||b - H x|| <= tol ||b|| */
  double rel_residual; /* final ||b - H x||_2 / ||b||_2, FP64 action */
} shp_solve_stats;

int shp_helmholtz_solve(shp_plan plan, double lambda, const double* diag /* device */, const double* b /* device */,
                        double* x /* device, in/out */, int inner_prec, double tol, int max_outer, int max_inner,
                        double inner_tol, void* ws /* device */, size_t ws_bytes,
                        shp_solve_stats* stats /* host out */, void* stream);

/* Fix the launch shape used for (blk, op, strategy), blk = -1 for the
 * whole-mesh launch: elements per work-group (1..64, within the 160 KiB LDS of
 * a work-group), threads per work-group (multiple of 64 in [64,512]) and, for
 * the Laplacian and Helmholtz actions, the launch variant:
 *   0  one tile per work-group, geometric factors loaded in the metric stage;
 *   1  persistent work-groups; each tile's factors are loaded into registers
 *      during the previous tile;
 *   2  one tile per work-group, the tile's factors loaded into registers at
 *      the start of the tile.
 * Variants 1 and 2 are used when elems_per_wg * Q^3 <= 8 * threads, else
 * variant 0 runs.  (0, 0, 0) restores the default.  Used by tuning.  2D
 * blocks take elements per work-group and threads only (the variant is
 * ignored): their Laplacian and Helmholtz run the fused tile with the
 * factors in registers when elems_per_wg * Q^2 <= 8 * threads. */
int shp_set_tiling(shp_plan plan, int blk, int op, int strategy, int elems_per_wg, int threads, int variant);

/* Current launch shape for (blk, op, strategy). */
int shp_get_tiling(shp_plan plan, int blk, int op, int strategy, int* elems_per_wg /* host out */,
                   int* threads /* host out */, int* variant /* host out */);

/* Result of tuning one (block, operator). */
typedef struct {
  int strategy;      /* fastest strategy */
  int elems_per_wg;  /* its launch shape */
  int threads;
  int variant;
  double ms;         /* median launch time of the choice */
  int n_candidates;  /* candidates run */
  int n_rejected;    /* candidates that failed the parity gate */
} shp_tune_result;

/* One timed candidate. ms < 0 when the candidate failed the parity gate. */
typedef struct {
  int strategy, elems_per_wg, threads, variant;
  double ms;
  int passed;
} shp_tune_record;

/* Exhaustive tuning of operator op on block blk (-1: the whole-mesh launch):
 * "different implementation choices may be made per block" (Sec. 3.3).  Every
 * strategy and launch shape that fits (quick = 1: a reduced set) runs on the
 * caller's representative input in; its output must match the default
 * collocated launch's output (written to ref) to 1e-12 in the max norm
 * relative to max |ref| or it is rejected; accepted candidates are timed as the
 * median of reps launches (at most 64) with HIP events on stream, each launch
 * preceded, outside the events, by a write of a 1 GiB buffer that the call
 * allocates and frees, so that the 256 MiB Infinity Cache does not serve the
 * inputs of small batches.  The fastest becomes the launch shape of its
 * strategy and the choice SHP_AUTO makes for (blk, op).  With blk = -1 on a
 * plan whose blocks differ in P the whole-mesh call runs one launch per block
 * with each block's own launch shape, so only the strategies are candidates.
 * A candidate whose launch the library rejects counts as rejected; a HIP
 * error ends the call with SHP_ERR_DEVICE.
 * out and ref are caller device buffers of the operator's output size.
 * records (host, may be NULL) receives up to max_records candidate timings.
 * Synchronises stream.  Returns SHP_ERR_NOT_CONVERGED if no candidate passes. */
int shp_tune(shp_plan plan, int blk, int op, const double* in /* device */, double* out /* device */,
             double* ref /* device */, double lambda, int reps, int quick, shp_tune_result* result /* host out */,
             shp_tune_record* records /* host out or NULL */, int max_records, int* n_records /* host out or NULL */,
             void* stream);

/* Fix the strategy SHP_AUTO uses for (blk, op) without tuning (used by a cost
 * model that predicts the fastest strategy). */
int shp_set_auto_strategy(shp_plan plan, int blk, int op, int strategy);

/* ---- Learned strategy choice ---------------------------------------------
 * Different implementation choices may be made per block (Sec. 3.3); besides
 * exhaustive tuning (shp_tune) a plan can carry a cost model, the MLP of the
 * shp_mlp_* calls below (or an ensemble of up to 4 such networks whose
 * predictions are averaged), trained on measured launch times.  For a block it
 * predicts the standardised log launch time per DOF of each strategy from the
 * features (shape one-hot, P/10, Q/12, log2(n_elem)/22, curved, strategy
 * one-hot: local matrix, sum-factorisation, collocated); its choice is the
 * argmin over the strategies the block supports.
 *
 * With a model loaded, SHP_AUTO for the Laplacian and Helmholtz actions of a
 * block that has no tuned or set choice runs the model once (the first such
 * apply synchronises the stream to read the prediction) and keeps its choice;
 * a whole-mesh SHP_AUTO call without a tuned or set whole-mesh choice takes
 * every block's choice: one whole-mesh collocated launch when all blocks pick
 * the collocated strategy, else one launch per block with its own choice.
 * Re-binding the workspace drops the model and the choices it made. */

/* Copy a model into the plan's workspace: params device FP32
 * [n_members][shp_mlp_num_params] (1 <= n_members <= 4), standardisation
 * mu, sigma > 0 of the training targets (predicted seconds per DOF =
 * exp(mu + sigma * output)).  Enqueued on stream. */
int shp_plan_set_model(shp_plan plan, const float* params /* device */, int n_members, double mu, double sigma,
                       void* stream);

/* Load a model file into the plan: path (host string) or, when NULL, the
 * environment variable SHP_MODEL_PATH.  The file is one JSON header line,
 *   {"format": "shp-mlp", "nin": 11, "nh": 64, "n_params": N, "members": M,
 *    "mu": mu, "sigma": sigma, ...}
 * then M * N little-endian FP32 parameters (the layout of shp_mlp_forward)
 * and nothing else.  A missing or malformed file returns SHP_ERR_INVALID_ARG
 * before any HIP call; synchronises stream. */
int shp_plan_load_model(shp_plan plan, const char* path /* host or NULL */, void* stream);

/* The model's choice for operator op (SHP_OP_LAPLACIAN or SHP_OP_HELMHOLTZ)
 * on block blk (non-empty): strategy (host out) and, when pred_ms is not NULL,
 * the predicted launch time in ms of the local-matrix, sum-factorisation and
 * collocated strategies (host out [3], +inf where the block does not support
 * one).  Does not change what SHP_AUTO runs.  Synchronises stream.
 * SHP_ERR_STATE when no model is loaded. */
int shp_model_choose(shp_plan plan, int blk, int op, int* strategy /* host out */, double* pred_ms /* host out or NULL */,
                     void* stream);

/* Append the plan's tuned choices to a JSON-lines cache file, keyed by device,
 * precision, operator, shape, P, Q, log2 of the block size and mapping type. */
int shp_tune_cache_save(shp_plan plan, const char* path /* host */);

/* Apply the entries of a cache file that match this plan's blocks (same keys)
 * and device; malformed or out-of-range entries are skipped.  n_applied may be
 * NULL. */
int shp_tune_cache_load(shp_plan plan, const char* path /* host */, int* n_applied /* host out or NULL */);

/* ---- C0 assembly on a structured hexahedral grid ------------------------
 * The elemental systems joined into the global Helmholtz problem of Sec. 2.1
 * (H^e assembled by a local-to-global map A: the global operator is A^T H A)
 * on a grid of n0 x n1 x n2 hexahedra, element e = (i0 n1 + i1) n2 + i2,
 * whose reference axes xi_1, xi_2, xi_3 follow the grid directions: a face or
 * edge shared by several elements then carries the same modified-basis
 * functions in each, so the map needs no sign changes.  Homogeneous Dirichlet
 * data on the grid boundary: the boundary DOFs are dropped.  Per direction the
 * interior DOFs are the n P - 1 interior vertices and cell bubbles in line
 * order (vertex v at v P - 1, bubble b of cell c at c P + b); a global index is
 * (g0 m1 + g1) m2 + g2 with m_d = n_d P - 1.
 *
 * The plan must hold these elements as its only block (shape SHP_HEX, order
 * P, affine or curved, element order as above); coefficients in the plan's
 * [n_elem][N_P] layout are the local vectors.  Geometry continuous across
 * faces (a global mesh map) is the caller's responsibility. */
int shp_c0_hex_sizes(int n0, int n1, int n2, int P, int64_t* n_global /* host out */,
                     int64_t* n_local /* host out: n_elem N_P */, int64_t* n_entries /* host out */);
/* l2g: host [n_local], global index of each local coefficient or -1 on the
 * Dirichlet boundary; row_ptr: host [n_global + 1] and col: host [n_entries],
 * the local copies of each global DOF in ascending local order (CSR). */
int shp_c0_hex_map(int n0, int n1, int n2, int P, int64_t* l2g, int64_t* row_ptr, int64_t* col);

/* ---- C0 assembly on a conforming tetrahedral mesh ------------------------
 * The same global problem (Sec. 2.1) on tetrahedra that meet face to face.
 * verts: host [n_elem][4], the global vertex ids of each tet in its local
 * order (the reference vertices (-1,-1,-1), (1,-1,-1), (-1,1,-1),
 * (-1,-1,1)).  Local order rule: vertex 3 has the largest id of the four and
 * vertex 2 the second largest (then each face's collapse vertex is its
 * largest id in every element that holds it); vertices 0 and 1 in either
 * order, e.g. the one that makes the element positively oriented.  A shared
 * edge or face whose direction differs between two elements gets a sign
 * change on its odd modes (A_k(-t) = (-1)^k A_k(t)).
 *
 * Global numbering: vertices by increasing id; edges by (lower, higher) id,
 * then mode k = 2..P (the trace A_k running from the lower to the higher id);
 * faces by their sorted ids, then mode (p, q), p >= 2, q >= 1, p + q <= P,
 * lexicographic (trace A_p(a) C_{p,q}(b) in the face's collapsed coordinates:
 * collapse vertex the largest id, a from the smallest to the middle one); then
 * the element interiors, element by element in local mode order.  Homogeneous
 * Dirichlet data on the boundary faces (faces of one element): their vertex,
 * edge and face DOFs are dropped.  A face shared by more than two elements, a
 * repeated or negative id, or a local order against the rule is
 * SHP_ERR_INVALID_ARG.
 *
 * l2g: host [n_elem N_P]: g for a copy with sign +1, -2 - g for a copy with
 * sign -1, -1 for a dropped DOF.  row_ptr: host [n_global + 1], col: host
 * [n_entries]: the copies of each global DOF in ascending local order, col =
 * i, or -1 - i for a copy with sign -1.  The plan for shp_c0_apply and
 * shp_c0_helmholtz_solve holds these elements as its only block (shape
 * SHP_TET, order P, element order as in verts), with geometry continuous
 * across faces (a global mesh map). */
int shp_c0_tet_sizes(int64_t n_elem, const int64_t* verts /* host */, int P, int64_t* n_global /* host out */,
                     int64_t* n_local /* host out */, int64_t* n_entries /* host out */);
int shp_c0_tet_map(int64_t n_elem, const int64_t* verts /* host */, int P, int64_t* l2g, int64_t* row_ptr,
                   int64_t* col);

/* Assembled FP64 Helmholtz action yg = A^T H A xg (gather, whole-mesh
 * collocated action, scatter-sum in the fixed CSR order).  l2g, row_ptr, col,
 * xg, yg: device, from either map (signs as encoded there); work: device FP64
 * scratch of 2 n_local values. */
int shp_c0_apply(shp_plan plan, const int64_t* l2g, const int64_t* row_ptr, const int64_t* col, int64_t n_global,
                 const double* xg /* device */, double* yg /* device */, double lambda, double* work /* device */,
                 void* stream);

/* Assembled vector vg = A^T vl (each global DOF the sum of its local copies,
 * with their signs, in the fixed CSR order), e.g. a right-hand side from
 * shp_apply's inner products.  All arrays device; vl [n_local], vg [n_global]. */
int shp_c0_assemble(const int64_t* row_ptr, const int64_t* col, int64_t n_global, const double* vl /* device */,
                    double* vg /* device */, void* stream);

/* Local copies xl = A xg of a global vector (with their signs; 0 for dropped
 * DOFs): the element coefficients of an assembled solution, for shp_apply.
 * All arrays device; l2g, xl [n_local]. */
int shp_c0_gather(const int64_t* l2g, int64_t n_local, const double* xg /* device */, double* xl /* device */,
                  void* stream);

/* Solve A^T H A x = b with the mixed-precision PCG of shp_helmholtz_solve
 * (inner_prec, tol, max_outer, max_inner, inner_tol and the stats as there);
 * the Jacobi diagonal is the elemental diagonals summed per global DOF,
 * formed inside the call.  b, x: device FP64 [n_global].  ws: device,
 * 256-byte aligned, at least shp_c0_solve_workspace_bytes.  Synchronises
 * stream. */
int shp_c0_solve_workspace_bytes(shp_plan plan, int64_t n_global, size_t* bytes /* host out */);
int shp_c0_helmholtz_solve(shp_plan plan, const int64_t* l2g, const int64_t* row_ptr, const int64_t* col,
                           int64_t n_global, double lambda, const double* b /* device */, double* x /* device */,
                           int inner_prec, double tol, int max_outer, int max_inner, double inner_tol,
                           void* ws /* device */, size_t ws_bytes, shp_solve_stats* stats /* host out */,
                           void* stream);

/* ---- MLP cost model (11 -> 64 -> 64 -> 1, ReLU, FP32), trained on the GPU ----
 * Inputs per sample: shape one-hot (4), P/10, Q/12, log2(n_elem)/22, curved,
 * strategy one-hot (local matrix, sum-factorisation, collocated); output: a
 * standardised log launch time per DOF.  All pointers are device FP32 buffers
 * owned by the caller; work holds per-sample activations (shp_mlp_work_floats).
 * Parameters: W1 [64][11], b1 [64], W2 [64][64], b2 [64], W3 [1][64], b3 [1]. */
int shp_mlp_num_params(int* n /* host out */);
int shp_mlp_work_floats(int n_samples, long long* n /* host out */);
/* y [n] = network(X [n][11]). */
int shp_mlp_forward(const float* params, const float* X, int n, float* y, float* work, void* stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops): shp_mlp_forward without the work argument.
 * Its per-sample work lives in a static device array of the library, one per
 * device, sized for n <= 4096 samples (6.3 MB), held until the process ends;
 * larger n returns SHP_ERR_INVALID_ARG.  Runs on the current device (stream
 * must belong to it) and allocates nothing.  All calls on one device share
 * that array: calls that overlap on one device (different streams or host
 * threads without ordering) race and must be serialised by the caller. */
int shp_mlp_forward_noalloc(const float* params, const float* X, int n, float* y, void* stream);
/* Mean squared error of the network against target [n] (loss [1]) and its
 * gradient with respect to the parameters (grad [num_params]). */
int shp_mlp_loss_grad(const float* params, const float* X, const float* target, int n, float* grad, float* loss,
                      float* work, void* stream);
/* One Adam step (step counts from 1) on params with moments m, v. */
int shp_mlp_adam(float* params, const float* grad, float* m, float* v, int step, float lr, float beta1, float beta2,
                 float eps, void* stream);

/* Destroy a plan (host metadata only; the workspace stays the caller's). */
int shp_plan_destroy(shp_plan plan);

/* Thread-local message of the last failed call on this thread ("" if none). */
const char* shp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SHP_H */
