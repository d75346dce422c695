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

// Persistent, static: the tiles form kBatchQueues contiguous ranges, one per
// XCD; the g workgroups on an XCD (dispatched to the XCDs in turn) take its
// range's tiles in turn, l, l + g, l + 2 g, ... At any moment the tiles in
// flight on an XCD are neighbours, as in the one-workgroup-per-tile launch
// (contiguous ranges per workgroup put the workgroups' tiles far apart and
// ran 1.1x slower on the 4096-matrix batch). 8 wavefronts per SIMD, as many
// workgroups per CU as the one-per-tile launch.
template <typename VT, typename BT>
__global__ __launch_bounds__(kWG, 8) void k_batch_static(
    int64_t t0, int64_t t1, const int32_t* __restrict__ tiles,
    const int32_t* const* __restrict__ rps, const int32_t* const* __restrict__ cis,
    const void* const* __restrict__ vals, const void* const* __restrict__ Bs,
    double* const* __restrict__ Cs, const BT* __restrict__ B1, double* __restrict__ C1,
    const uint8_t* __restrict__ deltas) {
  __shared__ dev::BlockLds L;
  const int64_t n = t1 - t0, G = gridDim.x;
  const int64_t Q = G < kBatchQueues ? G : kBatchQueues;  // ranges (each with a workgroup)
  const int64_t x = blockIdx.x % Q, l = blockIdx.x / Q;
  const int64_t g = (G - x + Q - 1) / Q;  // workgroups on range x
  const int64_t lo = t0 + n * x / Q, hi = t0 + n * (x + 1) / Q;
#pragma unroll 1
  for (int64_t t = lo + l; t < hi; t += g) {
    dev::lds_sync();  // LDS of the previous tile is no longer read
    batch_tile<VT, BT>(L, tiles, t, rps, cis, vals, Bs, Cs, B1, C1, deltas);
  }
}

// Persistent, dynamic: the tiles form kBatchQueues contiguous ranges, one
// per XCD, each with its own claim counter, so that claims on different XCDs
// go to different addresses (atomics on one address serialise in memory).
// A workgroup claims kClaim consecutive tiles at a time from the queue of its
// XCD (workgroups are dispatched to the XCDs in turn), then from the others in
// order; a queue seen exhausted by a plain read is skipped without an atomic.
// One tile per claim measured fastest (4 and 16 lengthened the tail: the last
// claims run alone).
// The atomic for the next claim is issued as soon as a claim is taken, and its
// result is read after the claim's first tile, whose loads it overlapped; a
// claim once made is always processed. The last workgroup to finish returns
// every counter to zero, so consecutive launches (and graph replays) need no
// clearing step.
constexpr int kClaim = 1;

struct ClaimState {  // thread 0's: queue (x + i) % kBatchQueues, a claim issued ahead
  int i = 0;
  bool has_pend = false;
  unsigned pend = 0;
};

// The next claim [c, ce) (c == ce: no tiles left anywhere), on thread 0.
__device__ __forceinline__ void next_claim(ClaimState& S, int x, int64_t t0, int64_t n,
                                           unsigned int* counters, int64_t* out) {
  int64_t c = t0 + n, ce = t0 + n;
  while (S.i < kBatchQueues) {
    const int q = (x + S.i) % kBatchQueues;
    unsigned int* ctr = counters + q * kBatchCounterStride;
    const int64_t qlo = t0 + n * q / kBatchQueues, qhi = t0 + n * (q + 1) / kBatchQueues;
    if (!S.has_pend) {
      const unsigned seen = __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (qlo + kClaim * (int64_t)seen >= qhi) {
        ++S.i;
        continue;
      }
      S.pend = atomicAdd(ctr, 1u);
    }
    S.has_pend = false;
    const int64_t cc = qlo + kClaim * (int64_t)S.pend;
    if (cc >= qhi) {
      ++S.i;
      continue;
    }
    c = cc;
    ce = cc + kClaim < qhi ? cc + kClaim : qhi;
    if (ce < qhi) {  // more left on this queue: issue the next claim now
      S.pend = atomicAdd(ctr, 1u);
      S.has_pend = true;
    }
    break;
  }
  out[0] = c;
  out[1] = ce;
}

template <typename VT, typename BT>
__global__ __launch_bounds__(kWG, 8) void k_batch_dynamic(
    int64_t t0, int64_t t1, const int32_t* __restrict__ tiles,
    const int32_t* const* __restrict__ rps, const int32_t* const* __restrict__ cis,
    const void* const* __restrict__ vals, const void* const* __restrict__ Bs,
    double* const* __restrict__ Cs, const BT* __restrict__ B1, double* __restrict__ C1,
    const uint8_t* __restrict__ deltas, unsigned int* __restrict__ counters) {
  __shared__ dev::BlockLds L;
  __shared__ int64_t claim[2][2];  // double-buffered [first tile, end)
  const int64_t n = t1 - t0;
  const int x = blockIdx.x % kBatchQueues;
  ClaimState S;
  if (threadIdx.x == 0) next_claim(S, x, t0, n, counters, claim[0]);
  for (int k = 0;; k ^= 1) {
    dev::lds_sync();  // claim[k] written; the previous tile is done with LDS
    const int64_t c = claim[k][0], ce = claim[k][1];
    if (c >= ce) break;
#pragma unroll 1
    for (int64_t t = c; t < ce; ++t) {  // same trip count in every lane
      if (t > c) dev::lds_sync();       // previous tile done with LDS
      batch_tile<VT, BT>(L, tiles, t, rps, cis, vals, Bs, Cs, B1, C1, deltas);
      // after the first tile (which waited for its loads, the claim atomic
      // among them): the following claim, into the other buffer
      if (t == c && threadIdx.x == 0) next_claim(S, x, t0, n, counters, claim[k ^ 1]);
    }
  }
  if (threadIdx.x == 0) {
    __threadfence();
    unsigned int* done = counters + kBatchQueues * kBatchCounterStride;
    if (atomicAdd(done, 1u) == gridDim.x - 1) {
      for (int q = 0; q < kBatchQueues; ++q) atomicExch(counters + q * kBatchCounterStride, 0u);
      atomicExch(done, 0u);
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
  switch (b.mode) {
    case SPMV_BATCH_STATIC:
      k_batch_static<VT, BT><<<(unsigned)std::min<int64_t>(b.grid_static, n), kWG, 0, s>>>(
          t0, t1, b.tiles, b.row_ptrs, b.col_idxs, b.vals, Bs, Cs, B1, C1, b.deltas);
      break;
    case SPMV_BATCH_TILE_GRID:
      k_batch_tilegrid<VT, BT><<<(unsigned)n, kWG, 0, s>>>(
          t0, t1, b.tiles, b.row_ptrs, b.col_idxs, b.vals, Bs, Cs, B1, C1, b.deltas);
      break;
    default:
      k_batch_dynamic<VT, BT><<<(unsigned)std::min<int64_t>(b.grid_dynamic, n), kWG, 0, s>>>(
          t0, t1, b.tiles, b.row_ptrs, b.col_idxs, b.vals, Bs, Cs, B1, C1, b.deltas, b.counters);
  }
  SPMV_HIP(hipGetLastError());
  return SPMV_OK;
}

}  // namespace

template <typename VT>
int batch_grids_typed(int cus, int* g_static, int* g_dynamic) {
  int a = 0, b = 0;
  SPMV_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_batch_static<VT, VT>, kWG, 0));
  SPMV_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_batch_dynamic<VT, VT>, kWG, 0));
  *g_static = cus * std::max(a, 1);
  *g_dynamic = cus * std::max(b, 1);
  return SPMV_OK;
}

int batch_grids(int device, int vdt, int* g_static, int* g_dynamic) {
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
      cus <= 0)
    cus = 256;
  // a persistent grid larger than what is resident would run its surplus
  // workgroups as a second round after the first finished its share
  return vdt == SPMV_F64 ? batch_grids_typed<double>(cus, g_static, g_dynamic)
                         : batch_grids_typed<float>(cus, g_static, g_dynamic);
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
  for (int i = threadIdx.x; i < kBatchCounterWords; i += blockDim.x) c[i] = 0u;
}

int launch_counters_init(unsigned int* c, hipStream_t s) {
  k_counters_init<<<1, 64, 0, s>>>(c);
  SPMV_HIP(hipGetLastError());
  return SPMV_OK;
}

}  // namespace spmv
