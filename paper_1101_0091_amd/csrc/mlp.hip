// Kernel-variant selector network: 16 -> 64 -> 64 -> 7, ReLU, float32.
//
// Forward, backward (mean-squared error) and Adam update kernels. Training
// runs on the GPU through these kernels; the trained weights live in a
// per-device global array that plan creation reads. All reductions have a
// fixed order (no atomics), so training is reproducible.
//
// Flat parameter layout: W1[64,16] b1[64] W2[64,64] b2[64] W3[7,64] b3[7].
#include <cmath>

#include "common.hpp"

namespace spmv {
namespace {

constexpr int NI = 16, H1 = 64, H2 = 64, NO = 7;
constexpr int oW1 = 0, oB1 = oW1 + H1 * NI, oW2 = oB1 + H1, oB2 = oW2 + H2 * H1,
              oW3 = oB2 + H2, oB3 = oW3 + NO * H2, NPAR = oB3 + NO;
static_assert(NPAR == SPMV_MLP_PARAMS, "parameter layout");

__device__ float g_theta[SPMV_MLP_PARAMS];

__global__ __launch_bounds__(64) void k_mlp_fwd(const float* __restrict__ th,
                                                const float* __restrict__ X, int nb,
                                                float* __restrict__ Y, float* __restrict__ Z1,
                                                float* __restrict__ Z2) {
  __shared__ float x[NI], h1[H1], h2[H2];
  const int b = blockIdx.x, j = threadIdx.x;
  if (b >= nb) return;
  if (j < NI) x[j] = X[(int64_t)b * NI + j];
  __syncthreads();
  float z = th[oB1 + j];
  for (int k = 0; k < NI; ++k) z = fmaf(th[oW1 + j * NI + k], x[k], z);
  Z1[(int64_t)b * H1 + j] = z;
  h1[j] = z > 0.0f ? z : 0.0f;
  __syncthreads();
  z = th[oB2 + j];
  for (int k = 0; k < H1; ++k) z = fmaf(th[oW2 + j * H1 + k], h1[k], z);
  Z2[(int64_t)b * H2 + j] = z;
  h2[j] = z > 0.0f ? z : 0.0f;
  __syncthreads();
  if (j < NO) {
    float y = th[oB3 + j];
    for (int k = 0; k < H2; ++k) y = fmaf(th[oW3 + j * H2 + k], h2[k], y);
    Y[(int64_t)b * NO + j] = y;
  }
}

// Per-sample deltas: dY = 2 (Y - T) / (nb * 7), 0 where the target is NaN (no
// time for that variant); dZ2, dZ1 (ReLU'(0) = 0).
__global__ __launch_bounds__(64) void k_mlp_bwd_sample(
    const float* __restrict__ th, const float* __restrict__ Z1, const float* __restrict__ Z2,
    const float* __restrict__ Y, const float* __restrict__ T, int nb, float* __restrict__ dY,
    float* __restrict__ dZ2, float* __restrict__ dZ1) {
  __shared__ float dy[NO], dz2[H2];
  const int b = blockIdx.x, j = threadIdx.x;
  if (b >= nb) return;
  if (j < NO) {
    const float t = T[(int64_t)b * NO + j];
    const float d = t == t ? 2.0f * (Y[(int64_t)b * NO + j] - t) / (float)(nb * NO) : 0.0f;
    dy[j] = d;
    dY[(int64_t)b * NO + j] = d;
  }
  __syncthreads();
  float g = 0.0f;
  for (int o = 0; o < NO; ++o) g = fmaf(th[oW3 + o * H2 + j], dy[o], g);
  g = Z2[(int64_t)b * H2 + j] > 0.0f ? g : 0.0f;
  dz2[j] = g;
  dZ2[(int64_t)b * H2 + j] = g;
  __syncthreads();
  g = 0.0f;
  for (int k = 0; k < H2; ++k) g = fmaf(th[oW2 + k * H1 + j], dz2[k], g);
  dZ1[(int64_t)b * H1 + j] = Z1[(int64_t)b * H1 + j] > 0.0f ? g : 0.0f;
}

// Parameter gradients: one lane per parameter, batch summed in order.
__global__ __launch_bounds__(256) void k_mlp_bwd_params(
    const float* __restrict__ X, const float* __restrict__ Z1, const float* __restrict__ Z2,
    int nb, const float* __restrict__ dY, const float* __restrict__ dZ2,
    const float* __restrict__ dZ1, float* __restrict__ grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPAR) return;
  float g = 0.0f;
  if (p < oB1) {
    const int o = p / NI, i = p % NI;
    for (int b = 0; b < nb; ++b) g = fmaf(dZ1[(int64_t)b * H1 + o], X[(int64_t)b * NI + i], g);
  } else if (p < oW2) {
    const int o = p - oB1;
    for (int b = 0; b < nb; ++b) g += dZ1[(int64_t)b * H1 + o];
  } else if (p < oB2) {
    const int q = p - oW2, o = q / H1, i = q % H1;
    for (int b = 0; b < nb; ++b) {
      const float h = Z1[(int64_t)b * H1 + i];
      g = fmaf(dZ2[(int64_t)b * H2 + o], h > 0.0f ? h : 0.0f, g);
    }
  } else if (p < oW3) {
    const int o = p - oB2;
    for (int b = 0; b < nb; ++b) g += dZ2[(int64_t)b * H2 + o];
  } else if (p < oB3) {
    const int q = p - oW3, o = q / H2, i = q % H2;
    for (int b = 0; b < nb; ++b) {
      const float h = Z2[(int64_t)b * H2 + i];
      g = fmaf(dY[(int64_t)b * NO + o], h > 0.0f ? h : 0.0f, g);
    }
  } else {
    const int o = p - oB3;
    for (int b = 0; b < nb; ++b) g += dY[(int64_t)b * NO + o];
  }
  grad[p] = g;
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ th, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v,
                                              float lr, float b1, float b2, float eps,
                                              float bc1, float bc2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPAR) return;
  const float gp = g[p];
  const float mp = b1 * m[p] + (1.0f - b1) * gp;
  const float vp = b2 * v[p] + (1.0f - b2) * gp * gp;
  m[p] = mp;
  v[p] = vp;
  const float mh = mp / bc1, vh = vp / bc2;
  th[p] = th[p] - lr * mh / (sqrtf(vh) + eps);
}

constexpr int kMaxDev = 64;
const float* g_theta_ptr[kMaxDev] = {};

}  // namespace

int launch_mlp_forward(const float* theta, const float* X, int nb, float* Y, float* Z1,
                       float* Z2, hipStream_t s) {
  if (nb <= 0) return SPMV_OK;
  k_mlp_fwd<<<nb, 64, 0, s>>>(theta, X, nb, Y, Z1, Z2);
  SPMV_HIP(hipGetLastError());
  return SPMV_OK;
}

int launch_mlp_backward(const float* theta, const float* X, const float* Z1, const float* Z2,
                        const float* Y, const float* T, int nb, float* scratch, float* grad,
                        hipStream_t s) {
  if (nb <= 0) return SPMV_OK;
  float* dY = scratch;
  float* dZ2 = dY + (int64_t)nb * NO;
  float* dZ1 = dZ2 + (int64_t)nb * H2;
  k_mlp_bwd_sample<<<nb, 64, 0, s>>>(theta, Z1, Z2, Y, T, nb, dY, dZ2, dZ1);
  SPMV_HIP(hipGetLastError());
  k_mlp_bwd_params<<<(NPAR + 255) / 256, 256, 0, s>>>(X, Z1, Z2, nb, dY, dZ2, dZ1, grad);
  SPMV_HIP(hipGetLastError());
  return SPMV_OK;
}

int launch_mlp_adam(float* theta, const float* grad, float* m, float* v, int t, float lr,
                    float b1, float b2, float eps, hipStream_t s) {
  const float bc1 = (float)(1.0 - std::pow((double)b1, (double)t));
  const float bc2 = (float)(1.0 - std::pow((double)b2, (double)t));
  k_adam<<<(NPAR + 255) / 256, 256, 0, s>>>(theta, grad, m, v, lr, b1, b2, eps, bc1, bc2);
  SPMV_HIP(hipGetLastError());
  return SPMV_OK;
}

int selector_upload(const float* params) {
  int dev = 0;
  SPMV_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDev) return fail(SPMV_ERR_UNSUPPORTED, "device index too large");
  void* ptr = nullptr;
  SPMV_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(g_theta)));
  SPMV_HIP(hipMemcpy(ptr, params, sizeof(float) * NPAR, hipMemcpyHostToDevice));
  g_theta_ptr[dev] = static_cast<const float*>(ptr);
  return SPMV_OK;
}

const float* selector_theta_device() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) return nullptr;
  return g_theta_ptr[dev];
}

}  // namespace spmv
