// Analysis of a CRS pattern at plan creation: validation, row statistics
// (the selector's 16 features), row-length bins, and the nnz-balanced row
// blocks. Done once per pattern and reused by every product, as the paper
// does for its communication bookkeeping (Sect. 3.1).
#include <cmath>

#include "common.hpp"
#include "device.hpp"

namespace spmv {
namespace {

__device__ __forceinline__ int feature_bin(int64_t l) {
  return l == 0 ? 0 : l <= 4 ? 1 : l <= 16 ? 2 : l <= 64 ? 3 : l <= 1024 ? 4 : 5;
}

__device__ __forceinline__ int variant_bin(int64_t l) {
  return l <= 4 ? 0 : l <= 16 ? 1 : l <= 64 ? 2 : l <= 1024 ? 3 : 4;
}

__global__ void k_zero_header(WsHeader* h) {
  // cleared with a kernel (not a memset) so the sequence stays graph-safe
  int* p = reinterpret_cast<int*>(h);
  for (size_t i = threadIdx.x; i < sizeof(WsHeader) / sizeof(int); i += blockDim.x) p[i] = 0;
  __syncthreads();
  if (threadIdx.x == 0) h->cnt[C_LMIN] = ~0ull;
}

// CRS definition: row_ptr[0] = 0, nondecreasing, row_ptr[n] = nnz, 0 <= col < n_cols.
__global__ void k_validate(int64_t n, int64_t n_cols, int64_t nnz,
                           const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                           int32_t* err) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int bad = 0;
  for (int64_t i = t0; i < n; i += stride)
    if (rp[i + 1] < rp[i]) bad |= 1;
  for (int64_t j = t0; j < nnz; j += stride) {
    const int32_t c = ci[j];
    if (c < 0 || (int64_t)c >= n_cols) bad |= 2;
  }
  if (t0 == 0) {
    if (rp[0] != 0) bad |= 4;
    if ((int64_t)rp[n] != nnz) bad |= 8;
  }
  if (bad) atomicOr(err, bad);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

// Row statistics. Every row range is clamped to [0, nnz] so that an invalid
// pattern (reported by k_validate in the same pass) never reads out of bounds.
__global__ __launch_bounds__(kWG) void k_stats(int64_t n, int64_t nnz,
                                               const int32_t* __restrict__ rp,
                                               const int32_t* __restrict__ ci, WsHeader* h) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  unsigned long long sumsq = 0, bins[6] = {0, 0, 0, 0, 0, 0}, longnnz = 0, distlog = 0,
                     near = 0, total = 0;
  unsigned long long lmax = 0, lmin = ~0ull;
  unsigned long long vb[kNumBins] = {0, 0, 0, 0, 0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    int64_t s = rp[i], e = rp[i + 1];
    s = s < 0 ? 0 : s > nnz ? nnz : s;
    e = e < s ? s : e > nnz ? nnz : e;
    const int64_t l = e - s;
    const unsigned long long ul = (unsigned long long)l;
    total += ul;
    sumsq += ul * ul;
    lmax = ul > lmax ? ul : lmax;
    lmin = ul < lmin ? ul : lmin;
    bins[feature_bin(l)] += 1;
    vb[variant_bin(l)] += 1;
    if (l > 64) longnnz += ul;
    for (int64_t j = s; j < e; ++j) {
      int64_t d = (int64_t)ci[j] - i;
      d = d < 0 ? -d : d;
      distlog += (unsigned long long)(63 - __clzll((unsigned long long)d + 1));
      near += d <= 64;
    }
  }
  // one atomic per wave per counter
  sumsq = wave_sum(sumsq);
  longnnz = wave_sum(longnnz);
  distlog = wave_sum(distlog);
  near = wave_sum(near);
  total = wave_sum(total);
  for (int b = 0; b < 6; ++b) bins[b] = wave_sum(bins[b]);
  for (int b = 0; b < kNumBins; ++b) vb[b] = wave_sum(vb[b]);
  for (int o = 32; o >= 1; o >>= 1) {
    unsigned long long a = __shfl_xor(lmax, o), c = __shfl_xor(lmin, o);
    lmax = a > lmax ? a : lmax;
    lmin = c < lmin ? c : lmin;
  }
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&h->cnt[C_SUMSQ], sumsq);
    atomicAdd(&h->cnt[C_LONGNNZ], longnnz);
    atomicAdd(&h->cnt[C_DISTLOG], distlog);
    atomicAdd(&h->cnt[C_NEAR], near);
    atomicAdd(&h->cnt[C_NNZ], total);
    for (int b = 0; b < 6; ++b) atomicAdd(&h->cnt[C_BIN0 + b], bins[b]);
    atomicMax(&h->cnt[C_LMAX], lmax);
    atomicMin(&h->cnt[C_LMIN], lmin);
    for (int b = 0; b < kNumBins; ++b) atomicAdd(&h->bin_count[b], (int32_t)vb[b]);
  }
}

struct Standardize {
  float mu[SPMV_NUM_FEATURES];
  float sigma[SPMV_NUM_FEATURES];
};

// Features from the integer counters (the divisions in float64), the
// standardised selector input, and the bin offsets for the row lists.
__global__ void k_finalize(int64_t n, WsHeader* h, Standardize st) {
  if (threadIdx.x != 0) return;
  double f[SPMV_NUM_FEATURES];
  for (int q = 0; q < SPMV_NUM_FEATURES; ++q) f[q] = 0.0;
  if (n > 0) {
    const double N = (double)n, Z = (double)h->cnt[C_NNZ];
    const double mean = Z / N;
    const double var = (double)h->cnt[C_SUMSQ] / N - mean * mean;
    f[0] = log2(N);
    f[1] = log2(Z > 1.0 ? Z : 1.0);
    f[2] = mean;
    f[3] = var > 0.0 ? sqrt(var) : 0.0;
    f[4] = log2((double)h->cnt[C_LMAX] + 1.0);
    f[5] = (double)h->cnt[C_LMIN];
    for (int b = 0; b < 6; ++b) f[6 + b] = (double)h->cnt[C_BIN0 + b] / N;
    if (h->cnt[C_NNZ] > 0) {
      f[12] = (double)h->cnt[C_LONGNNZ] / Z;
      f[13] = (double)h->cnt[C_DISTLOG] / Z;
      f[14] = (double)h->cnt[C_NEAR] / Z;
      f[15] = (double)h->cnt[C_LMAX] / mean;
    }
  }
  for (int q = 0; q < SPMV_NUM_FEATURES; ++q) {
    h->features[q] = f[q];
    h->x_std[q] = ((float)f[q] - st.mu[q]) / st.sigma[q];
  }
  int32_t acc = 0;
  for (int b = 0; b < kNumBins; ++b) {
    h->bin_offset[b] = acc;
    h->bin_cursor[b] = 0;
    acc += h->bin_count[b];
  }
}

// Row lists per bin. Wave-aggregated atomics keep lane order inside a wave.
__global__ __launch_bounds__(kWG) void k_scatter_bins(int64_t n, int64_t nnz,
                                                      const int32_t* __restrict__ rp,
                                                      WsHeader* h, int32_t* __restrict__ rows) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t base = (int64_t)blockIdx.x * blockDim.x;
  // every lane of a wave runs the same number of iterations (stride is a multiple of 64)
  for (int64_t i0 = base; i0 < n; i0 += stride) {
    const int64_t i = i0 + threadIdx.x;
    int mybin = -1;
    if (i < n) {
      int64_t s = rp[i], e = rp[i + 1];
      s = s < 0 ? 0 : s > nnz ? nnz : s;
      e = e < s ? s : e > nnz ? nnz : e;
      mybin = variant_bin(e - s);
    }
    const uint64_t lt = __lanemask_lt();
    for (int b = 0; b < kNumBins; ++b) {
      const uint64_t m = __ballot(mybin == b);
      if (m == 0) continue;
      const int leader = __ffsll((unsigned long long)m) - 1;
      int32_t pos = 0;
      if ((int)__lane_id() == leader) pos = atomicAdd(&h->bin_cursor[b], __popcll(m));
      pos = __shfl(pos, leader);
      if (mybin == b) rows[h->bin_offset[b] + pos + __popcll(m & lt)] = (int32_t)i;
    }
  }
}

// Row blocks: R_b = first row r with row_ptr[r] + r >= b * budget. The key
// row_ptr[r] + r grows strictly with r, so every block holds at most `budget`
// rows, and all its rows except the last lie in one budget-sized chunk.
// Each entry also carries row_ptr[R_b], the start of the block's nonzeros.
__global__ void k_blocks(int64_t n, int64_t nblocks, const int32_t* __restrict__ rp,
                         int2* __restrict__ blocks) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b > nblocks) return;
  if (b == nblocks) {
    blocks[b] = make_int2((int32_t)n, rp[n]);
    return;
  }
  const int64_t target = b * (int64_t)kBlockBudget;
  int64_t lo = 0, hi = n;  // answer in [0, n]
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)rp[mid] + mid >= target)
      hi = mid;
    else
      lo = mid + 1;
  }
  blocks[b] = make_int2((int32_t)lo, rp[lo]);
}

inline unsigned grid_cap(int64_t threads, unsigned cap) {
  int64_t g = (threads + kWG - 1) / kWG;
  if (g < 1) g = 1;
  return (unsigned)(g < cap ? g : cap);
}

}  // namespace

int launch_validate(const Plan& p, hipStream_t s) {
  const int64_t work = std::max<int64_t>(p.n_rows, p.nnz);
  k_validate<<<grid_cap(work, 8192), kWG, 0, s>>>(p.n_rows, p.n_cols, p.nnz, p.row_ptr,
                                                  p.col_idx, &p.hdr->err);
  SPMV_HIP(hipGetLastError());
  return SPMV_OK;
}

int launch_analysis(Plan& p, const float* mu, const float* sigma, hipStream_t s) {
  Standardize st;
  for (int q = 0; q < SPMV_NUM_FEATURES; ++q) {
    st.mu[q] = mu ? mu[q] : 0.0f;
    st.sigma[q] = sigma ? sigma[q] : 1.0f;
  }
  if (p.n_rows > 0) {
    k_stats<<<grid_cap(p.n_rows, 8192), kWG, 0, s>>>(p.n_rows, p.nnz, p.row_ptr, p.col_idx,
                                                     p.hdr);
    SPMV_HIP(hipGetLastError());
  }
  k_finalize<<<1, 64, 0, s>>>(p.n_rows, p.hdr, st);
  SPMV_HIP(hipGetLastError());
  if (p.n_rows > 0) {
    k_scatter_bins<<<grid_cap(p.n_rows, 8192), kWG, 0, s>>>(p.n_rows, p.nnz, p.row_ptr, p.hdr,
                                                            p.bin_rows);
    SPMV_HIP(hipGetLastError());
    k_blocks<<<grid_cap(p.nblocks + 1, 1u << 30), kWG, 0, s>>>(p.n_rows, p.nblocks, p.row_ptr,
                                                               p.blocks);
    SPMV_HIP(hipGetLastError());
  }
  return SPMV_OK;
}

int launch_zero_header(WsHeader* h, hipStream_t s) {
  k_zero_header<<<1, kWG, 0, s>>>(h);
  SPMV_HIP(hipGetLastError());
  return SPMV_OK;
}

}  // namespace spmv
