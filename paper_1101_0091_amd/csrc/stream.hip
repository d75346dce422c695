// STREAM-style kernels: the practical bandwidth ceiling the paper sets its
// spMVM bandwidth against (Sect. 2), and a plain copy used to calibrate the
// memory-traffic counters. 16-byte vector accesses, grid-stride.
#include "common.hpp"

namespace spmv {
namespace {

typedef double f64x2 __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(256) void k_triad(double* __restrict__ a,
                                               const double* __restrict__ b,
                                               const double* __restrict__ c, double s,
                                               int64_t n) {
  const int64_t n2 = n / 2;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  f64x2* a2 = reinterpret_cast<f64x2*>(a);
  const f64x2* b2 = reinterpret_cast<const f64x2*>(b);
  const f64x2* c2 = reinterpret_cast<const f64x2*>(c);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += stride) {
    const f64x2 x = __builtin_nontemporal_load(b2 + i);
    const f64x2 y = __builtin_nontemporal_load(c2 + i);
    f64x2 r;
    r.x = fma(s, y.x, x.x);
    r.y = fma(s, y.y, x.y);
    __builtin_nontemporal_store(r, a2 + i);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && (n & 1)) a[n - 1] = fma(s, c[n - 1], b[n - 1]);
}

__global__ __launch_bounds__(256) void k_copy(double* __restrict__ d, const double* __restrict__ src,
                                              int64_t n) {
  const int64_t n2 = n / 2;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  f64x2* d2 = reinterpret_cast<f64x2*>(d);
  const f64x2* s2 = reinterpret_cast<const f64x2*>(src);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += stride)
    __builtin_nontemporal_store(__builtin_nontemporal_load(s2 + i), d2 + i);
  if (blockIdx.x == 0 && threadIdx.x == 0 && (n & 1)) d[n - 1] = src[n - 1];
}

unsigned stream_grid(int64_t n) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  const int64_t want = (n / 2 + 255) / 256;
  const int64_t cap = (int64_t)cus * 16;
  return (unsigned)std::max<int64_t>(1, std::min(want, cap));
}

}  // namespace

int launch_triad(double* a, const double* b, const double* c, double s, int64_t n,
                 hipStream_t st) {
  if (n <= 0) return SPMV_OK;
  k_triad<<<stream_grid(n), 256, 0, st>>>(a, b, c, s, n);
  SPMV_HIP(hipGetLastError());
  return SPMV_OK;
}

int launch_copy(double* dst, const double* src, int64_t n, hipStream_t st) {
  if (n <= 0) return SPMV_OK;
  k_copy<<<stream_grid(n), 256, 0, st>>>(dst, src, n);
  SPMV_HIP(hipGetLastError());
  return SPMV_OK;
}

}  // namespace spmv
