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
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n / 2) {
    const f64x2 x = __builtin_nontemporal_load(reinterpret_cast<const f64x2*>(b) + i);
    const f64x2 y = __builtin_nontemporal_load(reinterpret_cast<const f64x2*>(c) + i);
    f64x2 r;
    r.x = fma(s, y.x, x.x);
    r.y = fma(s, y.y, x.y);
    __builtin_nontemporal_store(r, reinterpret_cast<f64x2*>(a) + i);
  }
  if (i == 0 && (n & 1)) a[n - 1] = fma(s, c[n - 1], b[n - 1]);
}

__global__ __launch_bounds__(256) void k_copy(double* __restrict__ d, const double* __restrict__ src,
                                              int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n / 2)
    __builtin_nontemporal_store(
        __builtin_nontemporal_load(reinterpret_cast<const f64x2*>(src) + i),
        reinterpret_cast<f64x2*>(d) + i);
  if (i == 0 && (n & 1)) d[n - 1] = src[n - 1];
}

// one 16-byte vector per lane (no grid-stride loop): the fastest shape measured
unsigned stream_grid(int64_t n) {
  return (unsigned)std::max<int64_t>(1, (n / 2 + 255) / 256);
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
