// Uneven batch of small CRS matrices in one launch.
//
// At creation every matrix is cut into the same nnz-balanced row blocks as
// the single-matrix LDS variant, and a (matrix, rows, nonzero range) tile
// list is written to the workspace. The apply is a single kernel over that
// list: one workgroup per tile by default, or a persistent grid sized to the
// device that walks the list statically or claims tiles from a
// self-resetting counter. Every mode is graph-safe (no memset nodes).
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
  const int32_t* rp = dev::global_ptr_at(rps, m);
  const int32_t* ci = dev::global_ptr_at(cis, m);
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
  const int32_t* rp = dev::global_ptr_at(rps, m);
  for (int64_t b = threadIdx.x; b < nb; b += kWG) {
    const int32_t r0 = first_row_at(rp, n, b * kBlockBudget);
    const int32_t r1 = (b + 1 == nb) ? (int32_t)n : first_row_at(rp, n, (b + 1) * kBlockBudget);
    int32_t* t = tiles + kTileInts * (toff[m] + b);
    t[0] = m;
    t[1] = r0;
    t[2] = r1;
    t[3] = rp[r0];
    t[4] = rp[r1];
    t[5] = 0;
    t[6] = -1;
    t[7] = 0;
    t[8] = 0;
    t[9] = 0;
  }
}

// Staging range of every tile (one workgroup per tile): the column bounds of
// its chunk [S, min(E, S + budget)) when they span at most the LDS array, else
// the budget-wide window of columns centred on the tile's rows (clamped to
// the matrix's columns). The chunk's columns are also stored as deltas from
// their smallest value, in 8 bits when they span at most 0xFF columns, else
// in 16 bits when they span at most 0xFFFF (tile fields 7 and 8: bits and
// base; 0 bits keeps the 4-byte columns); the product then reads 1 or 2
// bytes per column instead of 4. S and E are clamped to [0, nnz] so an
// invalid pattern (reported by validation in the same pass) reads nothing
// out of bounds.
__global__ __launch_bounds__(kWG) void k_batch_spans(int64_t ntiles,
                                                     const int64_t* __restrict__ nz,
                                                     const int64_t* __restrict__ nc,
                                                     const int32_t* const* __restrict__ cis,
                                                     int32_t* __restrict__ tiles,
                                                     uint8_t* __restrict__ deltas) {
  __shared__ int32_t lo[kWG / 64], hi[kWG / 64];
  const int64_t t = blockIdx.x;
  if (t >= ntiles) return;
  int32_t* tl = tiles + kTileInts * t;
  const int32_t m = tl[0];
  const int64_t nnz = nz[m];
  int64_t S = tl[3], E = tl[4];
  S = S < 0 ? 0 : S > nnz ? nnz : S;
  E = E < S ? S : E > nnz ? nnz : E;
  if (E - S > kBlockBudget) E = S + kBlockBudget;
  const int32_t* ci = dev::global_ptr_at(cis, m);
  int32_t a = INT32_MAX, z = INT32_MIN;
  for (int64_t j = S + threadIdx.x; j < E; j += kWG) {
    const int32_t c = ci[j];
    a = c < a ? c : a;
    z = c > z ? c : z;
  }
  for (int o = 32; o >= 1; o >>= 1) {
    const int32_t x = __shfl_xor(a, o), y = __shfl_xor(z, o);
    a = x < a ? x : a;
    z = y > z ? y : z;
  }
  if (threadIdx.x % 64 == 0) {
    lo[threadIdx.x / 64] = a;
    hi[threadIdx.x / 64] = z;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kWG / 64; ++w) {
      a = lo[w] < a ? lo[w] : a;
      z = hi[w] > z ? hi[w] : z;
    }
    a = lo[0] < a ? lo[0] : a;
    z = hi[0] > z ? hi[0] : z;
    lo[0] = a;  // block-wide bounds for the delta pass
    hi[0] = z;
    if (a > z) {  // empty chunk: nothing staged
      tl[5] = 0;
      tl[6] = -1;
    } else if ((int64_t)z - a < kBlockBudget) {
      tl[5] = a;
      tl[6] = z;
    } else {
      const int64_t ncol = nc[m];
      const int64_t mid = ((int64_t)tl[1] + tl[2]) / 2;
      int64_t w0 = mid - kBlockBudget / 2;
      w0 = w0 < 0 ? 0 : w0;
      const int64_t w1 = w0 + kBlockBudget < ncol ? w0 + kBlockBudget : ncol;
      w0 = w1 - kBlockBudget > 0 ? w1 - kBlockBudget : 0;
      tl[5] = w0 < w1 ? (int32_t)w0 : 0;
      tl[6] = w0 < w1 ? (int32_t)(w1 - 1) : -1;
    }
  }
  __syncthreads();
  a = lo[0];
  z = hi[0];
  const int64_t span = (int64_t)z - a;
  const int bits = a > z ? 0 : span <= 0xFF ? 8 : span <= 0xFFFF ? 16 : 0;
  uint8_t* d = deltas + (int64_t)2 * kBlockBudget * t;
  for (int64_t j = S + threadIdx.x; j < E; j += kWG) {
    const uint32_t x = (uint32_t)(ci[j] - a);
    if (bits == 8) d[j - S] = (uint8_t)x;
    if (bits == 16) reinterpret_cast<uint16_t*>(d)[j - S] = (uint16_t)x;
  }
  if (threadIdx.x == 0) {
    tl[7] = bits;
    tl[8] = bits ? a : 0;
  }
}

// B is staged in the LDS product array itself (2048 doubles): a 4096-entry
// staging area measured faster on uniform-random tiles but, at twice the LDS,
// cost more on banded ones through lost occupancy.
template <typename VT, typename BT>
__device__ __forceinline__ void batch_tile(dev::BlockLds& L, const int32_t* __restrict__ tiles,
                                           int64_t t, const int32_t* const* __restrict__ rps,
                                           const int32_t* const* __restrict__ cis,
                                           const void* const* __restrict__ vals,
                                           const void* const* __restrict__ Bs,
                                           double* const* __restrict__ Cs,
                                           const BT* __restrict__ B1, double* __restrict__ C1,
                                           const uint8_t* __restrict__ deltas) {
  const int32_t* tl = tiles + kTileInts * t;
  const int32_t m = tl[0], r0 = tl[1], r1 = tl[2], S = tl[3], E = tl[4], cmin = tl[5],
                cmax = tl[6], dbits = tl[7], dbase = tl[8];
  if (r0 >= r1) return;
  const BT* B = static_cast<const BT*>(dev::global_ptr_or(Bs, m, static_cast<const void*>(B1)));
  double* C = dev::global_ptr_or(Cs, m, C1);
  dev::lds_block<VT, BT, false, true, true>(
      L, dev::global_ptr_at(rps, m), dev::global_ptr_at(cis, m),
      static_cast<const VT*>(dev::global_ptr_at(vals, m)), B, C, r0, r1, S, E, cmin, cmax,
      L.prod, kBlockBudget, dbits, dbase, deltas + (int64_t)2 * kBlockBudget * t);
}

// Persistent, static: workgroup w owns one contiguous range of tiles.
template <typename VT, typename BT>
__global__ __launch_bounds__(kWG) void k_batch_static(
    int64_t t0, int64_t t1, const int32_t* __restrict__ tiles,
    const int32_t* const* __restrict__ rps, const int32_t* const* __restrict__ cis,
    const void* const* __restrict__ vals, const void* const* __restrict__ Bs,
    double* const* __restrict__ Cs, const BT* __restrict__ B1, double* __restrict__ C1,
    const uint8_t* __restrict__ deltas) {
  __shared__ dev::BlockLds L;
  const int64_t w = dev::xcd_remap(blockIdx.x, gridDim.x);
  const int64_t n = t1 - t0, g = gridDim.x;
  const int64_t lo = t0 + (n * w) / g, hi = t0 + (n * (w + 1)) / g;
  for (int64_t t = lo; t < hi; ++t) {
    __syncthreads();  // LDS of the previous tile is no longer read
    batch_tile<VT, BT>(L, tiles, t, rps, cis, vals, Bs, Cs, B1, C1, deltas);
  }
}

// Persistent, dynamic: workgroups claim the next kClaim consecutive tiles
// from a counter (one atomic per claim). The last workgroup to finish returns
// both counters to zero, so consecutive launches (and graph replays) need no
// clearing step.
constexpr int kClaim = 4;
template <typename VT, typename BT>
__global__ __launch_bounds__(kWG) void k_batch_dynamic(
    int64_t t0, int64_t t1, const int32_t* __restrict__ tiles,
    const int32_t* const* __restrict__ rps, const int32_t* const* __restrict__ cis,
    const void* const* __restrict__ vals, const void* const* __restrict__ Bs,
    double* const* __restrict__ Cs, const BT* __restrict__ B1, double* __restrict__ C1,
    const uint8_t* __restrict__ deltas, unsigned int* __restrict__ counters) {
  __shared__ dev::BlockLds L;
  __shared__ int64_t claim;
  for (;;) {
    __syncthreads();  // previous tile done with LDS and with `claim`
    if (threadIdx.x == 0) claim = t0 + kClaim * (int64_t)atomicAdd(&counters[0], 1u);
    __syncthreads();
    const int64_t c = claim;
    if (c >= t1) break;
    const int64_t ce = c + kClaim < t1 ? c + kClaim : t1;
    for (int64_t t = c; t < ce; ++t) {  // same trip count in every lane
      if (t > c) __syncthreads();       // previous tile done with LDS
      batch_tile<VT, BT>(L, tiles, t, rps, cis, vals, Bs, Cs, B1, C1, deltas);
    }
  }
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(&counters[1], 1u) == gridDim.x - 1) {
      atomicExch(&counters[0], 0u);
      atomicExch(&counters[1], 0u);
    }
  }
}

// One workgroup per tile (no persistence; the hardware dispatcher balances).
template <typename VT, typename BT>
__global__ __launch_bounds__(kWG) void k_batch_tilegrid(
    int64_t t0, int64_t t1, const int32_t* __restrict__ tiles,
    const int32_t* const* __restrict__ rps, const int32_t* const* __restrict__ cis,
    const void* const* __restrict__ vals, const void* const* __restrict__ Bs,
    double* const* __restrict__ Cs, const BT* __restrict__ B1, double* __restrict__ C1,
    const uint8_t* __restrict__ deltas) {
  __shared__ dev::BlockLds L;
  const int64_t t = t0 + dev::xcd_remap(blockIdx.x, t1 - t0);
  batch_tile<VT, BT>(L, tiles, t, rps, cis, vals, Bs, Cs, B1, C1, deltas);
}

template <typename VT, typename BT>
int batch_launch(const Batch& b, int64_t t0, int64_t t1, const void* const* Bs,
                 double* const* Cs, const void* B1v, double* C1, hipStream_t s) {
  const BT* B1 = static_cast<const BT*>(B1v);
  const int64_t n = t1 - t0;
  const int64_t pgrid = std::min<int64_t>(b.grid, n);
  switch (b.mode) {
    case SPMV_BATCH_STATIC:
      k_batch_static<VT, BT><<<(unsigned)pgrid, kWG, 0, s>>>(
          t0, t1, b.tiles, b.row_ptrs, b.col_idxs, b.vals, Bs, Cs, B1, C1, b.deltas);
      break;
    case SPMV_BATCH_TILE_GRID:
      k_batch_tilegrid<VT, BT><<<(unsigned)n, kWG, 0, s>>>(
          t0, t1, b.tiles, b.row_ptrs, b.col_idxs, b.vals, Bs, Cs, B1, C1, b.deltas);
      break;
    default:
      k_batch_dynamic<VT, BT><<<(unsigned)pgrid, kWG, 0, s>>>(
          t0, t1, b.tiles, b.row_ptrs, b.col_idxs, b.vals, Bs, Cs, B1, C1, b.deltas, b.counters);
  }
  SPMV_HIP(hipGetLastError());
  return SPMV_OK;
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
  if (b.ntiles > 0) {
    k_batch_spans<<<(unsigned)b.ntiles, kWG, 0, s>>>(b.ntiles, nz, nc, b.col_idxs, b.tiles,
                                                     b.deltas);
    SPMV_HIP(hipGetLastError());
  }
  return SPMV_OK;
}

int launch_batch_apply(const Batch& b, int64_t t0, int64_t t1, const void* const* Bs,
                       double* const* Cs, const void* B1, double* C1, hipStream_t s) {
  if (t1 <= t0) return SPMV_OK;
  if (b.vdt == SPMV_F64) return batch_launch<double, double>(b, t0, t1, Bs, Cs, B1, C1, s);
  return batch_launch<float, float>(b, t0, t1, Bs, Cs, B1, C1, s);
}

__global__ void k_counters_init(unsigned int* c) {
  c[0] = 0u;
  c[1] = 0u;
}

int launch_counters_init(unsigned int* c, hipStream_t s) {
  k_counters_init<<<1, 1, 0, s>>>(c);
  SPMV_HIP(hipGetLastError());
  return SPMV_OK;
}

}  // namespace spmv
