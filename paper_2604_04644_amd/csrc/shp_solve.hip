// Mixed-precision Helmholtz solve on the broken (elemental) space: a
// Jacobi-preconditioned CG whose actions and vectors are FP32 (or FP64), with
// FP64 reliable updates.
//
//   r = b - H x0 (FP64), scaled by 1/max|r| into the inner precision
//   CG on H d = r in the inner precision (FP64 dot products); whenever the
//   recursive residual has fallen by inner_tol since the last update:
//       x += d (FP64);  r = b - H x (FP64 action)  -- residual replacement
//       keep the search direction, or restart it when the true residual
//       exceeds the recursive one twice over; undo an update that does not
//       lower the FP64 residual
//   stop when ||b - H x|| <= tol ||b||
//
// The system is block diagonal (one SPD H_e per element, lambda > 0).  CG
// scalars stay on the device (dot products write them, the update kernels read
// them); the host reads a residual norm every few iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <vector>

#include "../../include/shp.h"
#include "shp_internal.hpp"

namespace {

constexpr int NB = 1024;  // blocks of the dot-product reduction
enum Slot { RZ = 0, PQ, RZN, RR, RR0, BB, RMAX, NSLOT };

template <typename T>
__global__ void k_dot(const T* __restrict__ a, const T* __restrict__ b, long long n, double* __restrict__ part) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    acc = fma((double)a[i], (double)b[i], acc);
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// slot[dst] = sum of the partials; when dst == RZN also keep beta = RZN / RZ in
// slot RMAX+1 and move RZN into RZ
__global__ void k_dot_final(const double* __restrict__ part, int np, double* __restrict__ slot, int dst) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) acc += part[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    slot[dst] = sh[0];
    if (dst == RZN) {
      slot[NSLOT] = slot[RZ] > 0.0 ? sh[0] / slot[RZ] : 0.0;
      slot[RZ] = sh[0];
    }
  }
}

// max |a| as the bit pattern of a non-negative double (ordered like an
// unsigned integer): reduced within the work-group, one atomic per group
__global__ void k_absmax(const double* __restrict__ a, long long n, unsigned long long* __restrict__ out) {
  __shared__ double sh[256];
  double m = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    m = fmax(m, fabs(a[i]));
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(out, (unsigned long long)__double_as_longlong(sh[0]));
}

// r = b - y (FP64); rs = s r in the inner precision, s = 1 / max|r| from slot RMAX
template <typename T>
__global__ void k_resid(const double* __restrict__ b, const double* __restrict__ y, double* __restrict__ r,
                        T* __restrict__ rs, const unsigned long long* __restrict__ rmax, long long n, int scale) {
  double s = 1.0;
  if (scale) {
    double m;
    const unsigned long long bits = *rmax;
    std::memcpy(&m, &bits, sizeof m);
    s = m > 0.0 ? 1.0 / m : 1.0;
  }
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double v = scale ? r[i] : b[i] - y[i];
    if (!scale) r[i] = v;
    rs[i] = (T)(v * s);
  }
}

// x += d / s (FP64 update of the outer solution)
template <typename T>
__global__ void k_update_x(double* __restrict__ x, const T* __restrict__ d, const unsigned long long* __restrict__ rmax,
                           long long n) {
  double m;
  const unsigned long long bits = *rmax;
  std::memcpy(&m, &bits, sizeof m);
  const double inv = m > 0.0 ? m : 1.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    x[i] += (double)d[i] * inv;
}

// z = r / diag
template <typename T>
__global__ void k_jacobi(const T* __restrict__ r, const T* __restrict__ dg, T* __restrict__ z, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    z[i] = r[i] / dg[i];
}

template <typename T>
__global__ void k_copy(const T* __restrict__ a, T* __restrict__ b, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    b[i] = a[i];
}

template <typename T>
__global__ void k_zero(T* __restrict__ a, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    a[i] = (T)0;
}

// One pass for the vector work of a CG step: alpha = RZ / PQ, d += alpha p,
// r -= alpha q, and the per-block partials of r^T z with z = r / diag (not
// stored).  Launched on NB blocks of 256 threads, so element i goes to the same
// thread, in the same order, as in k_dot: the partials equal k_dot's on (r, z).
template <typename T>
__global__ void k_cg1_rz(T* __restrict__ d, T* __restrict__ r, const T* __restrict__ p, const T* __restrict__ q,
                         const T* __restrict__ dg, const double* __restrict__ slot, long long n,
                         double* __restrict__ part) {
  __shared__ double sh[256];
  const T alpha = slot[PQ] > 0.0 ? (T)(slot[RZ] / slot[PQ]) : (T)0;  // 0 on breakdown, caught by the host check
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    d[i] += alpha * p[i];
    const T ri = r[i] - alpha * q[i];
    r[i] = ri;
    const T zi = ri / dg[i];
    acc = fma((double)ri, (double)zi, acc);
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// p = z + beta p (beta in slot NSLOT) with z = r / diag recomputed, rounded as
// in k_jacobi
template <typename T>
__global__ void k_cg2_r(T* __restrict__ p, const T* __restrict__ r, const T* __restrict__ dg,
                        const double* __restrict__ slot, long long n) {
  const T beta = (T)slot[NSLOT];
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = r[i] / dg[i] + beta * p[i];
}

__global__ void k_to_float(const double* __restrict__ a, float* __restrict__ b, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    b[i] = (float)a[i];
}

// assembled (C0) operator: local copies of global values and the sum of the
// local copies of each global DOF in a fixed (ascending local) order.  A copy
// may carry a sign change (an odd edge or face mode traversed against the
// global orientation): l2g holds g, -2 - g for a negated copy, or -1 for a
// dropped (Dirichlet) DOF; col holds i, or -1 - i for a negated copy.
template <typename T>
__global__ void k_c0_gather(const int64_t* __restrict__ l2g, long long n_local, const T* __restrict__ xg,
                            T* __restrict__ xl) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n_local;
       i += (long long)gridDim.x * blockDim.x) {
    const int64_t g = l2g[i];
    xl[i] = g >= 0 ? xg[g] : g <= -2 ? -xg[-2 - g] : (T)0;
  }
}
// SIGNED = false sums the copies without their signs (for the diagonal of
// A^T H A, where each sign appears squared)
template <typename T, bool SIGNED = true>
__global__ void k_c0_scatter(const int64_t* __restrict__ row_ptr, const int64_t* __restrict__ col, long long n_global,
                             const T* __restrict__ yl, T* __restrict__ yg) {
  for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g < n_global;
       g += (long long)gridDim.x * blockDim.x) {
    T acc = 0;
    for (int64_t j = row_ptr[g]; j < row_ptr[g + 1]; ++j) {
      const int64_t c = col[j];
      if (c >= 0)
        acc += yl[c];
      else
        acc += SIGNED ? -yl[-1 - c] : yl[-1 - c];
    }
    yg[g] = acc;
  }
}

inline dim3 grid_for(long long n) { return dim3((unsigned)std::min<long long>((n + 255) / 256, 8192)); }

int sfail(int code, const char* msg) { return shp::set_error(code, msg); }

struct SolveWs {
  double *r, *y, *xb, *slot, *part, *part_rz;  // part_rz: r^T z partials of k_cg1_rz
  float* diagf;
  void* vec;  // inner vectors: rs, z, p, q, d (5 n of the inner type)
  unsigned long long* rmax;
};

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

size_t carve(void* base, long long n, SolveWs* w) {
  char* p = static_cast<char*>(base);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    char* q = p ? p + o : nullptr;
    o = align256(o + bytes);
    return q;
  };
  SolveWs s{};
  s.r = reinterpret_cast<double*>(take(sizeof(double) * n));
  s.y = reinterpret_cast<double*>(take(sizeof(double) * n));
  s.xb = reinterpret_cast<double*>(take(sizeof(double) * n));
  s.diagf = reinterpret_cast<float*>(take(sizeof(float) * n));
  s.vec = take(sizeof(double) * 5 * n);
  s.slot = reinterpret_cast<double*>(take(sizeof(double) * 16));
  s.part = reinterpret_cast<double*>(take(sizeof(double) * NB));
  s.part_rz = reinterpret_cast<double*>(take(sizeof(double) * NB));
  s.rmax = reinterpret_cast<unsigned long long*>(take(sizeof(unsigned long long) * 2));
  if (w) *w = s;
  return o;
}

template <typename T>
int dot(const T* a, const T* b, long long n, SolveWs& w, int slot, hipStream_t s) {
  hipLaunchKernelGGL(k_dot<T>, dim3(NB), dim3(256), 0, s, a, b, n, w.part);
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(256), 0, s, w.part, NB, w.slot, slot);
  return hipGetLastError() == hipSuccess ? SHP_OK : SHP_ERR_DEVICE;
}

// inner precisions whose vectors are FP32: the FP32 sum-factorisation and the
// split-BF16 affine local matrices
bool f32_vectors(int prec) { return prec == SHP_FP32 || prec == SHP_BF16 || prec == SHP_BF16X3; }

template <typename T>
int apply_inner(shp_plan plan, const T* in, T* out, double lambda, int prec, hipStream_t s) {
  if constexpr (sizeof(T) == sizeof(float)) {
    if (prec == SHP_BF16 || prec == SHP_BF16X3)
      return shp_apply_prec(plan, -1, SHP_OP_HELMHOLTZ, SHP_LOCALMAT, prec, in, out, lambda, s);
    return shp_apply_prec(plan, -1, SHP_OP_HELMHOLTZ, SHP_AUTO, SHP_FP32, in, out, lambda, s);
  } else {
    return shp_apply_prec(plan, -1, SHP_OP_HELMHOLTZ, SHP_AUTO, SHP_FP64, in, out, lambda, s);
  }
}

// The operators of the solve: the FP64 action apply64 and the action in the
// inner type.  The FP64 actions take the plan's SHP_AUTO choice for the whole
// mesh (tuned or set, or a loaded cost model's; by default the collocated
// sum-factorisation), e.g. the local matrices of an affine mesh; the FP32
// inner actions take the FP32 local matrices when that choice is the local
// matrices and every block has them, else the FP32 sum-factorisation.  ElemOp is the block-diagonal elemental H; C0Op the assembled
// operator A^T H A of a local-to-global map A (gather, elemental action,
// scatter-sum).
struct ElemOp {
  shp_plan plan;
  double lambda;
  int prec;  // inner precision
  int apply64(const double* x, double* y, hipStream_t s) const {
    return shp_apply(plan, -1, SHP_OP_HELMHOLTZ, SHP_AUTO, x, y, lambda, s);
  }
  template <typename T>
  int apply(const T* x, T* y, hipStream_t s) const {
    return apply_inner<T>(plan, x, y, lambda, prec, s);
  }
};

struct C0Op {
  shp_plan plan;
  double lambda;
  int prec;  // inner precision
  const int64_t *l2g, *row_ptr, *col;
  long long n_local, n_global;
  double *xl, *yl;
  float *xlf, *ylf;
  template <typename T>
  int run(const T* x, T* y, T* xl_, T* yl_, hipStream_t s) const {
    hipLaunchKernelGGL(k_c0_gather<T>, grid_for(n_local), dim3(256), 0, s, l2g, n_local, x, xl_);
    if (int r = apply_inner<T>(plan, xl_, yl_, lambda, prec, s)) return r;
    hipLaunchKernelGGL(k_c0_scatter<T>, grid_for(n_global), dim3(256), 0, s, row_ptr, col, n_global, yl_, y);
    return hipGetLastError() == hipSuccess ? SHP_OK : SHP_ERR_DEVICE;
  }
  int apply64(const double* x, double* y, hipStream_t s) const { return run<double>(x, y, xl, yl, s); }
  template <typename T>
  int apply(const T* x, T* y, hipStream_t s) const {
    if constexpr (sizeof(T) == sizeof(float))
      return run<float>(x, y, xlf, ylf, s);
    else
      return run<double>(x, y, xl, yl, s);
  }
};

// FP64 true residual r = b - H x of the current x, its squared norm into slot
// RR, and (when T is the inner type) the scaled copy rs = r / rmax in T
template <typename T, typename Op>
int true_residual(const Op& op, const double* b, const double* x, long long n, SolveWs& w, bool scaled,
                  hipStream_t s) {
  const dim3 g = grid_for(n), bl(256);
  if (int r = op.apply64(x, w.y, s)) return r;
  hipLaunchKernelGGL(k_resid<T>, g, bl, 0, s, b, w.y, w.r, static_cast<T*>(w.vec), w.rmax, n, 0);
  if (scaled) hipLaunchKernelGGL(k_resid<T>, g, bl, 0, s, b, w.y, w.r, static_cast<T*>(w.vec), w.rmax, n, 1);
  return dot(w.r, w.r, n, w, RR, s);
}

// Jacobi-preconditioned CG whose actions, vectors and updates run in T, with
// reliable updates: every time the recursive residual has fallen by the factor
// delta since the last update (checked every 10 iterations), the correction
// accumulated in T is added to x in FP64, the residual is recomputed as
// b - H x with the FP64 action, and the CG recursion continues from it with
// its search direction kept.  Convergence is decided on that FP64 residual.
template <typename T, typename Op>
int pcg_reliable(const Op& op, const double* b, double* x, long long n, SolveWs& w, const T* dg, double tol,
                 int max_updates, int max_iter, double delta, double bnorm2, shp_solve_stats* st, hipStream_t s) {
  T* rs = static_cast<T*>(w.vec);
  T* z = rs + n;
  T* p = z + n;
  T* q = p + n;
  T* d = q + n;
  const dim3 g = grid_for(n), bl(256);
  double h[NSLOT + 1];
  auto readback = [&]() {
    return hipMemcpyAsync(h, w.slot, sizeof h, hipMemcpyDeviceToHost, s) == hipSuccess &&
           hipStreamSynchronize(s) == hipSuccess;
  };
  // the scale 1/max|r0| is fixed for the whole solve (w.rmax)
  if (hipMemsetAsync(w.rmax, 0, sizeof(unsigned long long), s) != hipSuccess)
    return sfail(SHP_ERR_DEVICE, "solver memset");
  hipLaunchKernelGGL(k_absmax, dim3(NB), bl, 0, s, w.r, n, w.rmax);
  hipLaunchKernelGGL(k_resid<T>, g, bl, 0, s, b, w.y, w.r, rs, w.rmax, n, 1);
  hipLaunchKernelGGL(k_zero<T>, g, bl, 0, s, d, n);
  hipLaunchKernelGGL(k_jacobi<T>, g, bl, 0, s, rs, dg, z, n);
  hipLaunchKernelGGL(k_copy<T>, g, bl, 0, s, z, p, n);
  if (int r = dot(rs, z, n, w, RZ, s)) return r;
  if (int r = dot(rs, rs, n, w, RR0, s)) return r;
  if (!readback()) return sfail(SHP_ERR_DEVICE, "solver readback");
  double rr_ref = h[RR0];
  // the scale, to turn the recursive residual into an estimate of ||b - H x||
  unsigned long long rbits = 0;
  if (hipMemcpyAsync(&rbits, w.rmax, sizeof rbits, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return sfail(SHP_ERR_DEVICE, "solver readback");
  double rmax;
  std::memcpy(&rmax, &rbits, sizeof rmax);
  const double rr_goal = (tol / rmax) * (tol / rmax) * bnorm2;  // ||rs||^2 at the tolerance
  double best = st->rel_residual;
  int stalls = 0, last = 0;
  constexpr int MAX_GAP = 2000;  // iterations between updates at most
  for (int it = 1; it <= max_iter; ++it) {
    if (int r = op.template apply<T>(p, q, s)) return r;
    if (int r = dot(p, q, n, w, PQ, s)) return r;
    hipLaunchKernelGGL(k_cg1_rz<T>, dim3(NB), bl, 0, s, d, rs, p, q, dg, w.slot, n, w.part_rz);
    st->inner_iters = it;
    bool fresh_rz = true;  // part_rz holds r^T z of the current rs
    if (it % 10 == 0 || it == max_iter) {
      if (int r = dot(rs, rs, n, w, RR, s)) return r;
      if (!readback()) return sfail(SHP_ERR_DEVICE, "solver readback");
      if (!(h[PQ] > 0.0) || !std::isfinite(h[RR])) return sfail(SHP_ERR_NOT_CONVERGED, "CG breakdown (p^T H p <= 0)");
      if (h[RR] <= delta * delta * rr_ref || h[RR] <= rr_goal || it == max_iter || it - last >= MAX_GAP) {
        // reliable update: x += d in FP64 (the previous x kept), true residual
        const double rr_rec = h[RR];
        last = it;
        fresh_rz = false;
        hipLaunchKernelGGL(k_copy<double>, g, bl, 0, s, x, w.xb, n);
        hipLaunchKernelGGL(k_update_x<T>, g, bl, 0, s, x, d, w.rmax, n);
        hipLaunchKernelGGL(k_zero<T>, g, bl, 0, s, d, n);
        if (int r = true_residual<T>(op, b, x, n, w, true, s)) return r;
        if (!readback()) return sfail(SHP_ERR_DEVICE, "solver readback");
        st->outer_iters += 1;
        const double rel = std::sqrt(h[RR] / bnorm2);
        bool restart = false;
        if (rel < best) {
          best = rel;
          stalls = 0;
          st->rel_residual = rel;
          if (rel <= tol) {
            st->converged = 1;
            return SHP_OK;
          }
          if (int r = dot(rs, rs, n, w, RR, s)) return r;
          if (!readback()) return sfail(SHP_ERR_DEVICE, "solver readback");
          rr_ref = h[RR];
          // a true residual well above the recursive one (rounding near the
          // floor) would make the next beta inconsistent: restart the direction
          restart = rr_ref > 4.0 * rr_rec;
        } else {
          // no progress: return to the previous x and its residual, restart
          hipLaunchKernelGGL(k_copy<double>, g, bl, 0, s, w.xb, x, n);
          if (int r = true_residual<T>(op, b, x, n, w, true, s)) return r;
          if (int r = dot(rs, rs, n, w, RR, s)) return r;
          if (!readback()) return sfail(SHP_ERR_DEVICE, "solver readback");
          rr_ref = h[RR];
          restart = true;
          if (++stalls >= 5) break;  // the residual floor of the FP64 action
        }
        if (st->outer_iters >= max_updates) break;
        if (restart) {
          hipLaunchKernelGGL(k_jacobi<T>, g, bl, 0, s, rs, dg, z, n);
          hipLaunchKernelGGL(k_copy<T>, g, bl, 0, s, z, p, n);
          if (int r = dot(rs, z, n, w, RZ, s)) return r;
          continue;
        }
      }
    }
    if (fresh_rz) {
      hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(256), 0, s, w.part_rz, NB, w.slot, (int)RZN);
    } else {
      hipLaunchKernelGGL(k_jacobi<T>, g, bl, 0, s, rs, dg, z, n);
      if (int r = dot(rs, z, n, w, RZN, s)) return r;
    }
    hipLaunchKernelGGL(k_cg2_r<T>, g, bl, 0, s, p, rs, dg, w.slot, n);
  }
  return sfail(SHP_ERR_NOT_CONVERGED, "the residual did not reach the tolerance (x is the best iterate)");
}

int check_solve_args(double lambda, double tol, double inner_tol, int max_outer, int max_inner, int inner_prec) {
  if (!(lambda > 0.0) || !(tol > 0.0) || !(inner_tol > 0.0) || max_outer < 1 || max_inner < 1)
    return sfail(SHP_ERR_INVALID_ARG, "lambda, tolerances and iteration limits must be positive");
  if (inner_prec != SHP_FP64 && !f32_vectors(inner_prec)) return sfail(SHP_ERR_INVALID_ARG, "bad inner precision");
  return SHP_OK;
}

// the solve of op x = b (n unknowns, Jacobi diagonal diag in FP64) on the
// carved workspace w
template <typename Op>
int solve_with(const Op& op, long long n, SolveWs& w, const double* diag, const double* b, double* x, int inner_prec,
               double tol, int max_outer, int max_inner, double inner_tol, shp_solve_stats* st, hipStream_t s) {
  const dim3 g = grid_for(n), bl(256);
  std::memset(st, 0, sizeof *st);
  if (f32_vectors(inner_prec)) hipLaunchKernelGGL(k_to_float, g, bl, 0, s, diag, w.diagf, n);
  // ||b|| and the initial FP64 residual
  if (int r = dot(b, b, n, w, BB, s)) return r;
  if (int r = (f32_vectors(inner_prec) ? true_residual<float>(op, b, x, n, w, false, s)
                                      : true_residual<double>(op, b, x, n, w, false, s)))
    return r;
  double hs[NSLOT + 1];
  if (hipMemcpyAsync(hs, w.slot, sizeof hs, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return sfail(SHP_ERR_DEVICE, "solver readback");
  if (!(hs[BB] > 0.0) || !std::isfinite(hs[BB]))
    return sfail(SHP_ERR_INVALID_ARG, "b is zero or not finite (relative residual undefined)");
  st->rel_residual = std::sqrt(hs[RR] / hs[BB]);
  if (st->rel_residual <= tol) {
    st->converged = 1;
    return SHP_OK;
  }
  if (f32_vectors(inner_prec))
    return pcg_reliable<float>(op, b, x, n, w, w.diagf, tol, max_outer, max_inner, inner_tol, hs[BB], st, s);
  return pcg_reliable<double>(op, b, x, n, w, diag, tol, max_outer, max_inner, inner_tol, hs[BB], st, s);
}

// workspace of the assembled solve: the PCG on n_global unknowns, the
// elemental diagonal's scratch, local copies (FP64 and FP32) and the global
// diagonal
struct C0Ws {
  SolveWs w;
  void* elem_ws;
  size_t elem_bytes;
  double *xl, *yl, *diag;
  float *xlf, *ylf;
};

size_t c0_carve(void* base, long long n_local, long long n_global, C0Ws* c) {
  char* p = static_cast<char*>(base);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    char* q = p ? p + o : nullptr;
    o = align256(o + bytes);
    return q;
  };
  C0Ws t{};
  const size_t pcg = carve(nullptr, n_global, nullptr);
  char* pc = take(pcg);
  t.elem_bytes = carve(nullptr, n_local, nullptr);
  t.elem_ws = take(t.elem_bytes);
  t.xl = reinterpret_cast<double*>(take(sizeof(double) * n_local));
  t.yl = reinterpret_cast<double*>(take(sizeof(double) * n_local));
  t.xlf = reinterpret_cast<float*>(take(sizeof(float) * n_local));
  t.ylf = reinterpret_cast<float*>(take(sizeof(float) * n_local));
  t.diag = reinterpret_cast<double*>(take(sizeof(double) * n_global));
  if (c) {
    carve(pc, n_global, &t.w);
    *c = t;
  }
  return o;
}

}  // namespace

extern "C" {

int shp_solve_workspace_bytes(shp_plan plan, size_t* bytes) {
  if (!plan || !bytes) return sfail(SHP_ERR_INVALID_ARG, "null argument");
  *bytes = carve(nullptr, shp::plan_total_coeff(plan), nullptr);
  return SHP_OK;
}

int shp_helmholtz_diag(shp_plan plan, double lambda, double* diag, void* ws, size_t ws_bytes, void* stream) {
  if (!plan || !diag || !ws) return sfail(SHP_ERR_INVALID_ARG, "null argument");
  const long long n = shp::plan_total_coeff(plan);
  if (n < 1) return sfail(SHP_ERR_INVALID_ARG, "empty mesh");
  if (!std::isfinite(lambda)) return sfail(SHP_ERR_INVALID_ARG, "lambda not finite");
  if (reinterpret_cast<uintptr_t>(ws) % 256 || ws_bytes < carve(nullptr, n, nullptr))
    return sfail(SHP_ERR_WORKSPACE, "solver workspace missing, misaligned or too small");
  if (int r = shp::plan_check_solve(plan, SHP_FP64)) return r;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // sum-factorised: every mode's 1D factors contracted with the 7 factors
  if (int r = shp::plan_helm_diag(plan, lambda, diag, s)) return r;
  if (hipStreamSynchronize(s) != hipSuccess) return sfail(SHP_ERR_DEVICE, "diagonal");
  return SHP_OK;
}

int shp_helmholtz_solve(shp_plan plan, double lambda, const double* diag, const double* b, double* x, int inner_prec,
                        double tol, int max_outer, int max_inner, double inner_tol, void* ws, size_t ws_bytes,
                        shp_solve_stats* st, void* stream) {
  if (!plan || !diag || !b || !x || !ws || !st) return sfail(SHP_ERR_INVALID_ARG, "null argument");
  const long long n_dof = shp::plan_total_coeff(plan);
  if (n_dof < 1) return sfail(SHP_ERR_INVALID_ARG, "empty mesh");
  if (int r = check_solve_args(lambda, tol, inner_tol, max_outer, max_inner, inner_prec)) return r;
  if (reinterpret_cast<uintptr_t>(ws) % 256 || ws_bytes < carve(nullptr, n_dof, nullptr))
    return sfail(SHP_ERR_WORKSPACE, "solver workspace missing, misaligned or too small");
  if (int r = shp::plan_check_solve(plan, inner_prec)) return r;
  SolveWs w;
  carve(ws, n_dof, &w);
  return solve_with(ElemOp{plan, lambda, inner_prec}, n_dof, w, diag, b, x, inner_prec, tol, max_outer, max_inner, inner_tol, st,
                    static_cast<hipStream_t>(stream));
}

// ---- C0 (assembled) operator -------------------------------------------

int shp_c0_apply(shp_plan plan, const int64_t* l2g, const int64_t* row_ptr, const int64_t* col, int64_t n_global,
                 const double* xg, double* yg, double lambda, double* work, void* stream) {
  if (!plan || !l2g || !row_ptr || !col || !xg || !yg || !work || n_global < 1)
    return sfail(SHP_ERR_INVALID_ARG, "null argument");
  const long long n_local = shp::plan_total_coeff(plan);
  if (n_local < 1) return sfail(SHP_ERR_INVALID_ARG, "empty mesh");
  if (int r = shp::plan_check_solve(plan, SHP_FP64)) return r;
  C0Op op{plan, lambda, SHP_FP64, l2g, row_ptr, col, n_local, n_global, work, work + n_local, nullptr, nullptr};
  return op.apply64(xg, yg, static_cast<hipStream_t>(stream));
}

int shp_c0_assemble(const int64_t* row_ptr, const int64_t* col, int64_t n_global, const double* vl, double* vg,
                    void* stream) {
  if (!row_ptr || !col || !vl || !vg || n_global < 1) return sfail(SHP_ERR_INVALID_ARG, "null argument");
  hipLaunchKernelGGL(k_c0_scatter<double>, grid_for(n_global), dim3(256), 0, static_cast<hipStream_t>(stream),
                     row_ptr, col, (long long)n_global, vl, vg);
  return hipGetLastError() == hipSuccess ? SHP_OK : sfail(SHP_ERR_DEVICE, "assembly launch");
}

int shp_c0_gather(const int64_t* l2g, int64_t n_local, const double* xg, double* xl, void* stream) {
  if (!l2g || !xg || !xl || n_local < 1) return sfail(SHP_ERR_INVALID_ARG, "null argument");
  hipLaunchKernelGGL(k_c0_gather<double>, grid_for(n_local), dim3(256), 0, static_cast<hipStream_t>(stream), l2g,
                     (long long)n_local, xg, xl);
  return hipGetLastError() == hipSuccess ? SHP_OK : sfail(SHP_ERR_DEVICE, "gather launch");
}

int shp_c0_solve_workspace_bytes(shp_plan plan, int64_t n_global, size_t* bytes) {
  if (!plan || !bytes || n_global < 1) return sfail(SHP_ERR_INVALID_ARG, "null argument");
  *bytes = c0_carve(nullptr, shp::plan_total_coeff(plan), n_global, nullptr);
  return SHP_OK;
}

int shp_c0_helmholtz_solve(shp_plan plan, const int64_t* l2g, const int64_t* row_ptr, const int64_t* col,
                           int64_t n_global, double lambda, const double* b, double* x, int inner_prec, double tol,
                           int max_outer, int max_inner, double inner_tol, void* ws, size_t ws_bytes,
                           shp_solve_stats* st, void* stream) {
  if (!plan || !l2g || !row_ptr || !col || !b || !x || !ws || !st || n_global < 1)
    return sfail(SHP_ERR_INVALID_ARG, "null argument");
  const long long n_local = shp::plan_total_coeff(plan);
  if (n_local < 1) return sfail(SHP_ERR_INVALID_ARG, "empty mesh");
  if (int r = check_solve_args(lambda, tol, inner_tol, max_outer, max_inner, inner_prec)) return r;
  if (reinterpret_cast<uintptr_t>(ws) % 256 || ws_bytes < c0_carve(nullptr, n_local, n_global, nullptr))
    return sfail(SHP_ERR_WORKSPACE, "solver workspace missing, misaligned or too small");
  if (int r = shp::plan_check_solve(plan, inner_prec)) return r;
  hipStream_t s = static_cast<hipStream_t>(stream);
  C0Ws c;
  c0_carve(ws, n_local, n_global, &c);
  // Jacobi diagonal of A^T H A: the elemental diagonals summed over the local
  // copies of each global DOF
  if (int r = shp_helmholtz_diag(plan, lambda, c.xl, c.elem_ws, c.elem_bytes, s)) return r;
  hipLaunchKernelGGL((k_c0_scatter<double, false>), grid_for(n_global), dim3(256), 0, s, row_ptr, col,
                     (long long)n_global, c.xl, c.diag);
  C0Op op{plan, lambda, inner_prec, l2g, row_ptr, col, n_local, n_global, c.xl, c.yl, c.xlf, c.ylf};
  return solve_with(op, n_global, c.w, c.diag, b, x, inner_prec, tol, max_outer, max_inner, inner_tol, st, s);
}

}  // extern "C"
