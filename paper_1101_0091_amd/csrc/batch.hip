// Uneven batch of small CRS matrices in one persistent launch.
//
// At creation every matrix is cut into the same nnz-balanced row blocks as
// the single-matrix LDS variant, and a (matrix, first row, end row) tile
// list is written to the workspace. The apply kernel runs a fixed grid of
// workgroups sized to the device; workgroup w owns one contiguous range of
// tiles, so no counters or atomics are needed and the launch is graph-safe.
#include "common.hpp"
#include "device.hpp"

namespace spmv {
namespace {

// CRS checks for every matrix of the batch; err[0] gets violation bits and
// err[1] the lowest bad matrix index (err[1] starts at INT32_MAX).
__global__ __launch_bounds__(kWG) void k_batch_validate(
    int32_t count, const int64_t* __restrict__ nr, const int64_t* __restrict__ nc,
    const int64_t* __restrict__ nz, const int32_t* const* __restrict__ rps,
    const int32_t* const* __restrict__ cis, int32_t* err) {
  const int32_t m = blockIdx.x;
  if (m >= count) return;
  const int64_t n = nr[m], ncol = nc[m], nnz = nz[m];
  const int32_t* rp = rps[m];
  const int32_t* ci = cis[m];
  int bad = 0;
  for (int64_t i = threadIdx.x; i < n; i += kWG)
    if (rp[i + 1] < rp[i]) bad |= 1;
  for (int64_t j = threadIdx.x; j < nnz; j += kWG)
    if (ci[j] < 0 || (int64_t)ci[j] >= ncol) bad |= 2;
  if (threadIdx.x == 0) {
    if (rp[0] != 0) bad |= 4;
    if ((int64_t)rp[n] != nnz) bad |= 8;
  }
  if (bad) {
    atomicOr(&err[0], bad);
    atomicMin(&err[1], m);
  }
}

__device__ __forceinline__ int32_t first_row_at(const int32_t* __restrict__ rp, int64_t n,
                                                int64_t target) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)rp[mid] + mid >= target)
      hi = mid;
    else
      lo = mid + 1;
  }
  return (int32_t)lo;
}

__global__ __launch_bounds__(kWG) void k_batch_tiles(int32_t count,
                                                     const int64_t* __restrict__ nr,
                                                     const int64_t* __restrict__ toff,
                                                     const int32_t* const* __restrict__ rps,
                                                     int32_t* __restrict__ tiles) {
  const int32_t m = blockIdx.x;
  if (m >= count) return;
  const int64_t n = nr[m];
  const int64_t nb = toff[m + 1] - toff[m];
  const int32_t* rp = rps[m];
  for (int64_t b = threadIdx.x; b < nb; b += kWG) {
    const int32_t r0 = first_row_at(rp, n, b * kBlockBudget);
    const int32_t r1 = (b + 1 == nb) ? (int32_t)n : first_row_at(rp, n, (b + 1) * kBlockBudget);
    int32_t* t = tiles + 6 * (toff[m] + b);
    t[0] = m;
    t[1] = r0;
    t[2] = r1;
    t[3] = rp[r0];
    t[4] = rp[r1];
    t[5] = 0;
  }
}

template <typename VT, typename BT>
__global__ __launch_bounds__(kWG) void k_batch_apply(
    int64_t t0, int64_t t1, const int32_t* __restrict__ tiles,
    const int32_t* const* __restrict__ rps, const int32_t* const* __restrict__ cis,
    const void* const* __restrict__ vals, const void* const* __restrict__ Bs,
    double* const* __restrict__ Cs, const BT* __restrict__ B1, double* __restrict__ C1) {
  __shared__ dev::BlockLds L;
  const int64_t w = dev::xcd_remap(blockIdx.x, gridDim.x);
  const int64_t n = t1 - t0, g = gridDim.x;
  const int64_t lo = t0 + (n * w) / g, hi = t0 + (n * (w + 1)) / g;
  for (int64_t t = lo; t < hi; ++t) {
    const int32_t* tl = tiles + 6 * t;
    const int32_t m = tl[0], r0 = tl[1], r1 = tl[2], S = tl[3], E = tl[4];
    if (r0 >= r1) continue;
    const BT* B = Bs ? static_cast<const BT*>(Bs[m]) : B1;
    double* C = Cs ? Cs[m] : C1;
    __syncthreads();  // LDS of the previous tile is no longer read
    dev::lds_block<VT, BT>(L, rps[m], cis[m], static_cast<const VT*>(vals[m]), B, C, r0, r1, S,
                           E);
  }
}

}  // namespace

int batch_grid(int device) {
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
      cus <= 0)
    cus = 256;
  return cus * 8;  // 8 resident 256-lane workgroups per CU (16 KB LDS each)
}

int launch_batch_build(Batch& b, const int64_t* toff, const int64_t* nr, const int64_t* nc,
                       const int64_t* nz, hipStream_t s) {
  k_batch_validate<<<b.count, kWG, 0, s>>>(b.count, nr, nc, nz, b.row_ptrs, b.col_idxs, b.err);
  SPMV_HIP(hipGetLastError());
  k_batch_tiles<<<b.count, kWG, 0, s>>>(b.count, nr, toff, b.row_ptrs, b.tiles);
  SPMV_HIP(hipGetLastError());
  return SPMV_OK;
}

int launch_batch_apply(const Batch& b, int64_t t0, int64_t t1, const void* const* Bs,
                       double* const* Cs, const void* B1, double* C1, hipStream_t s) {
  if (t1 <= t0) return SPMV_OK;
  int64_t grid = std::min<int64_t>(b.grid, t1 - t0);
  if (b.vdt == SPMV_F64)
    k_batch_apply<double, double><<<(unsigned)grid, kWG, 0, s>>>(
        t0, t1, b.tiles, b.row_ptrs, b.col_idxs, b.vals, Bs, Cs,
        static_cast<const double*>(B1), C1);
  else
    k_batch_apply<float, float><<<(unsigned)grid, kWG, 0, s>>>(
        t0, t1, b.tiles, b.row_ptrs, b.col_idxs, b.vals, Bs, Cs, static_cast<const float*>(B1),
        C1);
  SPMV_HIP(hipGetLastError());
  return SPMV_OK;
}

}  // namespace spmv
