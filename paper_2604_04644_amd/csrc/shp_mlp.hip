// A small MLP cost model trained and evaluated on the GPU with hand-written
// kernels: 11 inputs -> 64 -> 64 -> 1, ReLU, FP32, mean squared error, Adam.
// It predicts the log launch time per DOF of a (shape, P, Q, batch size,
// mapping, strategy) configuration; the strategy with the smallest prediction
// is the model's choice.
//
// Parameter vector (FP32), in order: W1 [64][11], b1 [64], W2 [64][64],
// b2 [64], W3 [1][64], b3 [1].  Work buffer per sample: Z1, H1, Z2, H2, dZ2,
// dZ1 (64 each) and y, dy (1 each).  Every reduction runs in a fixed order,
// so results are deterministic.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "../../include/shp.h"
#include "shp_internal.hpp"

// Work buffer of the allocation-free forward pass (shp_mlp_forward_noalloc):
// 4096 samples of 6 * 64 + 2 floats.
constexpr int NOALLOC_MAX_SAMPLES = 4096;
static __device__ __align__(256) float scratch[(size_t)NOALLOC_MAX_SAMPLES * (6 * 64 + 2)];

namespace {

constexpr int NIN = 11, NH = 64;
constexpr int OW1 = 0, OB1 = OW1 + NH * NIN, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH, OB3 = OW3 + NH;
constexpr int NPARAM = OB3 + 1;
constexpr int WS = 6 * NH + 2;  // work floats per sample
static_assert(WS == 6 * 64 + 2, "scratch is sized for 6 * 64 + 2 work floats per sample");
// work layout per sample s: Z1 H1 Z2 H2 dZ2 dZ1 at s*WS + k*NH, y at s*WS + 6NH, dy at +1

// Z = W x + b, H = relu(Z); one thread per (sample, output)
__global__ void k_dense(const float* __restrict__ in, int in_stride, int nin, const float* __restrict__ W,
                        const float* __restrict__ b, float* __restrict__ work, int zoff, int n, int nout) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * nout) return;
  const int s = t / nout, o = t - s * nout;
  const float* x = in + (long long)s * in_stride;
  float z = b[o];
  for (int i = 0; i < nin; ++i) z = fmaf(W[o * nin + i], x[i], z);
  float* w = work + (long long)s * WS;
  if (zoff == 6 * NH) {  // output layer: y only
    w[zoff] = z;
  } else {
    w[zoff + o] = z;
    w[zoff + NH + o] = z > 0.f ? z : 0.f;
  }
}

// dy = 2 (y - t) / n and the loss, one block, fixed reduction order
__global__ void __launch_bounds__(256) k_loss(const float* __restrict__ target, float* __restrict__ work, int n,
                                              float* __restrict__ loss) {
  __shared__ float part[256];
  float acc = 0.f;
  for (int s = threadIdx.x; s < n; s += blockDim.x) {
    float* w = work + (long long)s * WS;
    const float r = w[6 * NH] - target[s];
    w[6 * NH + 1] = 2.f * r / (float)n;
    acc = fmaf(r, r, acc);
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) part[threadIdx.x] += part[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = part[0] / (float)n;
}

// dZ_prev[s][i] = relu'(Z_prev) * sum_o dZ[s][o] W[o][i]; one thread per (sample, i)
__global__ void k_back_act(const float* __restrict__ W, float* __restrict__ work, int dz_off, int nout,
                           int zprev_off, int dprev_off, int n) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * NH) return;
  const int s = t / NH, i = t - s * NH;
  float* w = work + (long long)s * WS;
  float g = 0.f;
  for (int o = 0; o < nout; ++o) g = fmaf(w[dz_off + o], W[o * NH + i], g);
  w[dprev_off + i] = w[zprev_off + i] > 0.f ? g : 0.f;
}

// dW[o][i] = sum_s dZ[s][o] x[s][i], db[o] = sum_s dZ[s][o]; one thread per parameter
__global__ void k_back_w(const float* __restrict__ in, int in_stride, int in_off, int nin,
                         const float* __restrict__ work, int dz_off, int nout, int n, float* __restrict__ gW,
                         float* __restrict__ gb) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nout * (nin + 1)) return;
  const int o = t / (nin + 1), i = t - o * (nin + 1);
  float acc = 0.f;
  for (int s = 0; s < n; ++s) {
    const float dz = work[(long long)s * WS + dz_off + o];
    const float xv = (i == nin) ? 1.f : in[(long long)s * in_stride + in_off + i];
    acc = fmaf(dz, xv, acc);
  }
  if (i == nin)
    gb[o] = acc;
  else
    gW[o * nin + i] = acc;
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int np, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= np) return;
  const float gi = g[t];
  const float mi = b1 * m[t] + (1.f - b1) * gi;
  const float vi = b2 * v[t] + (1.f - b2) * gi * gi;
  m[t] = mi;
  v[t] = vi;
  p[t] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

inline unsigned nblk(long long n, int b) { return (unsigned)((n + b - 1) / b); }

// Work buffer of the allocation-free forward pass: one array per device for at
// most NOALLOC_MAX_SAMPLES samples (6.3 MB), held until the process ends.  Host
// code never passes the array's name to a kernel (on the host it is a stand-in
// symbol, not a device address): each device's address comes from
// hipGetSymbolAddress on the first call with that device current.

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[MAX_DEVICES] = {};

// the current device's address of scratch, or nullptr with the error set
float* scratch_on_current_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
    shp::set_error(SHP_ERR_DEVICE, "shp_mlp_forward_noalloc: no current HIP device");
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      shp::set_error(SHP_ERR_DEVICE, "shp_mlp_forward_noalloc: hipGetSymbolAddress(scratch) failed");
      return nullptr;
    }
    g_scratch_ptr[dev] = static_cast<float*>(ptr);
  }
  return g_scratch_ptr[dev];
}

int forward(const float* prm, const float* X, int n, float* work, hipStream_t s) {
  hipLaunchKernelGGL(k_dense, dim3(nblk((long long)n * NH, 256)), dim3(256), 0, s, X, NIN, NIN, prm + OW1,
                     prm + OB1, work, 0, n, NH);
  hipLaunchKernelGGL(k_dense, dim3(nblk((long long)n * NH, 256)), dim3(256), 0, s, work + NH, WS, NH, prm + OW2,
                     prm + OB2, work, 2 * NH, n, NH);
  hipLaunchKernelGGL(k_dense, dim3(nblk(n, 256)), dim3(256), 0, s, work + 3 * NH, WS, NH, prm + OW3, prm + OB3,
                     work, 6 * NH, n, 1);
  return hipGetLastError() == hipSuccess ? SHP_OK : SHP_ERR_DEVICE;
}

}  // namespace

extern "C" {

int shp_mlp_num_params(int* n) {
  if (!n) return SHP_ERR_INVALID_ARG;
  *n = NPARAM;
  return SHP_OK;
}

int shp_mlp_work_floats(int n_samples, long long* n) {
  if (!n || n_samples < 0) return SHP_ERR_INVALID_ARG;
  *n = (long long)n_samples * WS;
  return SHP_OK;
}

int shp_mlp_forward(const float* params, const float* X, int n, float* y, float* work, void* stream) {
  if (!params || !X || !y || !work || n < 1) return SHP_ERR_INVALID_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (int r = forward(params, X, n, work, s)) return r;
  // gather y (strided in the work buffer) with a device copy
  if (hipMemcpy2DAsync(y, sizeof(float), work + 6 * NH, WS * sizeof(float), sizeof(float), n,
                       hipMemcpyDeviceToDevice, s) != hipSuccess)
    return SHP_ERR_DEVICE;
  return SHP_OK;
}

int shp_mlp_forward_noalloc(const float* params, const float* X, int n, float* y, void* stream) {
  if (!params || !X || !y) return shp::set_error(SHP_ERR_INVALID_ARG, "shp_mlp_forward_noalloc: null argument");
  if (n < 1 || n > NOALLOC_MAX_SAMPLES)
    return shp::set_error(SHP_ERR_INVALID_ARG,
                          "shp_mlp_forward_noalloc: n must be in [1, 4096] (the size of its static work buffer)");
  float* work = scratch_on_current_device();
  if (!work) return SHP_ERR_DEVICE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (int r = forward(params, X, n, work, s)) return r;
  if (hipMemcpy2DAsync(y, sizeof(float), work + 6 * NH, WS * sizeof(float), sizeof(float), n,
                       hipMemcpyDeviceToDevice, s) != hipSuccess)
    return SHP_ERR_DEVICE;
  return SHP_OK;
}

int shp_mlp_loss_grad(const float* params, const float* X, const float* target, int n, float* grad, float* loss,
                      float* work, void* stream) {
  if (!params || !X || !target || !grad || !loss || !work || n < 1) return SHP_ERR_INVALID_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (int r = forward(params, X, n, work, s)) return r;
  hipLaunchKernelGGL(k_loss, dim3(1), dim3(256), 0, s, target, work, n, loss);
  // output layer: dZ3 = dy (work offset 6NH+1), input H2 (offset 3NH)
  hipLaunchKernelGGL(k_back_w, dim3(nblk(NH + 1, 256)), dim3(256), 0, s, work, WS, 3 * NH, NH, work, 6 * NH + 1, 1, n,
                     grad + OW3, grad + OB3);
  // dZ2 = relu'(Z2) * W3^T dy
  hipLaunchKernelGGL(k_back_act, dim3(nblk((long long)n * NH, 256)), dim3(256), 0, s, params + OW3, work, 6 * NH + 1,
                     1, 2 * NH, 4 * NH, n);
  hipLaunchKernelGGL(k_back_w, dim3(nblk(NH * (NH + 1), 256)), dim3(256), 0, s, work, WS, NH, NH, work, 4 * NH, NH,
                     n, grad + OW2, grad + OB2);
  // dZ1 = relu'(Z1) * W2^T dZ2
  hipLaunchKernelGGL(k_back_act, dim3(nblk((long long)n * NH, 256)), dim3(256), 0, s, params + OW2, work, 4 * NH, NH,
                     0, 5 * NH, n);
  hipLaunchKernelGGL(k_back_w, dim3(nblk(NH * (NIN + 1), 256)), dim3(256), 0, s, X, NIN, 0, NIN, work, 5 * NH, NH, n,
                     grad + OW1, grad + OB1);
  return hipGetLastError() == hipSuccess ? SHP_OK : SHP_ERR_DEVICE;
}

int shp_mlp_adam(float* params, const float* grad, float* m, float* v, int step, float lr, float beta1, float beta2,
                 float eps, void* stream) {
  if (!params || !grad || !m || !v || step < 1 || !(lr > 0.f)) return SHP_ERR_INVALID_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const float c1 = 1.f - std::pow(beta1, (float)step), c2 = 1.f - std::pow(beta2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(nblk(NPARAM, 256)), dim3(256), 0, s, params, grad, m, v, NPARAM, lr, beta1, beta2,
                     eps, c1, c2);
  return hipGetLastError() == hipSuccess ? SHP_OK : SHP_ERR_DEVICE;
}

}  // extern "C"
