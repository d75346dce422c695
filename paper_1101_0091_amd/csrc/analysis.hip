// Analysis of a CRS pattern at plan creation: validation, row statistics
// (the selector's 16 features), row-length bins, and the nnz-balanced row
// blocks. Done once per pattern and reused by every product, as the paper
// does for its communication bookkeeping (Sect. 3.1).
#include <algorithm>
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

// Partial-counter slots of one statistics workgroup.
enum : int {
  P_SUMSQ = 0, P_LMAX = 1, P_LMIN = 2, P_BIN0 = 3,  // feature bins P_BIN0..P_BIN0+5
  P_LONGNNZ = 9, P_DISTLOG = 10, P_NEAR = 11, P_NNZ = 12, P_VB0 = 13  // variant bins ..+4
};
static_assert(P_VB0 + kNumBins == kPartSlots, "partial slots");

// Workgroup w of a g-workgroup pass owns rows [w*R, min(n, (w+1)*R)), R = ceil(n/g).
__device__ __forceinline__ void row_range_of(int64_t n, int64_t w, int64_t g, int64_t& r0,
                                             int64_t& r1) {
  const int64_t R = (n + g - 1) / g;
  r0 = w * R < n ? w * R : n;
  r1 = r0 + R < n ? r0 + R : n;
}

// Row statistics. Each workgroup reduces its rows in registers and LDS and
// writes one record of partial counters (no atomics; k_finalize combines the
// records in a fixed order). Every row range is clamped to [0, nnz] so that
// an invalid pattern (reported by k_validate in the same pass) never reads
// out of bounds.
__global__ __launch_bounds__(kWG) void k_stats(int64_t n, int64_t nnz,
                                               const int32_t* __restrict__ rp,
                                               const int32_t* __restrict__ ci,
                                               unsigned long long* __restrict__ part) {
  __shared__ unsigned long long red[kWG / 64][kPartSlots];
  unsigned long long v[kPartSlots];
  for (int q = 0; q < kPartSlots; ++q) v[q] = 0;
  v[P_LMIN] = ~0ull;
  int64_t r0, r1;
  row_range_of(n, blockIdx.x, gridDim.x, r0, r1);
  for (int64_t i = r0 + threadIdx.x; i < r1; i += kWG) {
    int64_t s = rp[i], e = rp[i + 1];
    s = s < 0 ? 0 : s > nnz ? nnz : s;
    e = e < s ? s : e > nnz ? nnz : e;
    const int64_t l = e - s;
    const unsigned long long ul = (unsigned long long)l;
    v[P_NNZ] += ul;
    v[P_SUMSQ] += ul * ul;
    v[P_LMAX] = ul > v[P_LMAX] ? ul : v[P_LMAX];
    v[P_LMIN] = ul < v[P_LMIN] ? ul : v[P_LMIN];
    v[P_BIN0 + feature_bin(l)] += 1;
    v[P_VB0 + variant_bin(l)] += 1;
    if (l > 64) v[P_LONGNNZ] += ul;
    unsigned long long dl = 0, nr = 0;
    // eight columns loaded before any is used (integer sums: order-free); one
    // load at a time left every lane waiting on each load of its row
    constexpr int kU = 8;
    for (int64_t j0 = s; j0 < e; j0 += kU) {
      int32_t c[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) c[u] = j0 + u < e ? ci[j0 + u] : (int32_t)i;
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        int64_t d = (int64_t)c[u] - i;
        d = d < 0 ? -d : d;
        if (j0 + u < e) {
          dl += (unsigned long long)(63 - __clzll((unsigned long long)d + 1));
          nr += d <= 64;
        }
      }
    }
    v[P_DISTLOG] += dl;
    v[P_NEAR] += nr;
  }
  for (int q = 0; q < kPartSlots; ++q) {
    if (q == P_LMAX || q == P_LMIN) {
      for (int o = 32; o >= 1; o >>= 1) {
        const unsigned long long x = __shfl_xor(v[q], o);
        v[q] = q == P_LMAX ? (x > v[q] ? x : v[q]) : (x < v[q] ? x : v[q]);
      }
    } else {
      v[q] = wave_sum(v[q]);
    }
  }
  const int wv = threadIdx.x / 64;
  if (threadIdx.x % 64 == 0)
    for (int q = 0; q < kPartSlots; ++q) red[wv][q] = v[q];
  __syncthreads();
  if (threadIdx.x < kPartSlots) {
    const int q = threadIdx.x;
    unsigned long long a = red[0][q];
    for (int w = 1; w < kWG / 64; ++w) {
      const unsigned long long x = red[w][q];
      a = q == P_LMAX ? (x > a ? x : a) : q == P_LMIN ? (x < a ? x : a) : a + x;
    }
    part[(int64_t)blockIdx.x * kPartSlots + q] = a;
  }
}

struct Standardize {
  float mu[SPMV_NUM_FEATURES];
  float sigma[SPMV_NUM_FEATURES];
};

// Combines the g partial records into the header counters (integer sums,
// minima and maxima, so the order does not matter), then computes the
// features (divisions in float64), the standardised selector input, the bin
// offsets, and for every statistics workgroup its first slot inside each bin
// (an exclusive scan over workgroups). One thread per record, all records
// loaded at once: a loop over the records in 18 threads spent 100 us on
// memory latency.
constexpr int kFinWG = kStatsGrid;
__global__ __launch_bounds__(kFinWG) void k_finalize(int64_t n, int g,
                                                     const unsigned long long* __restrict__ part,
                                                     int32_t* __restrict__ bin_base, WsHeader* h,
                                                     Standardize st) {
  constexpr int kWaves = kFinWG / 64;
  __shared__ unsigned long long red[kWaves][kPartSlots];
  __shared__ unsigned long long tot[kPartSlots];
  __shared__ int32_t wave_bins[kWaves][kNumBins];
  const int t = threadIdx.x, wv = t / 64, ln = t % 64;
  unsigned long long v[kPartSlots];
  for (int q = 0; q < kPartSlots; ++q)
    v[q] = t < g ? part[(int64_t)t * kPartSlots + q] : q == P_LMIN ? ~0ull : 0ull;
  // inclusive scan of this record's variant-bin counts over the wavefront
  int32_t inc[kNumBins], own[kNumBins];
  for (int b = 0; b < kNumBins; ++b) {
    int32_t x = own[b] = (int32_t)v[P_VB0 + b];
    for (int o = 1; o < 64; o <<= 1) {
      const int32_t y = __shfl_up(x, o);
      if (ln >= o) x += y;
    }
    inc[b] = x;
    if (ln == 63) wave_bins[wv][b] = x;
  }
  for (int q = 0; q < kPartSlots; ++q) {
    if (q == P_LMAX || q == P_LMIN) {
      for (int o = 32; o >= 1; o >>= 1) {
        const unsigned long long x = __shfl_xor(v[q], o);
        v[q] = q == P_LMAX ? (x > v[q] ? x : v[q]) : (x < v[q] ? x : v[q]);
      }
    } else {
      v[q] = wave_sum(v[q]);
    }
  }
  if (ln == 0)
    for (int q = 0; q < kPartSlots; ++q) red[wv][q] = v[q];
  __syncthreads();
  if (t < g) {
    for (int b = 0; b < kNumBins; ++b) {
      int32_t off = 0;
      for (int w = 0; w < wv; ++w) off += wave_bins[w][b];
      bin_base[(int64_t)t * kNumBins + b] = off + inc[b] - own[b];
    }
  }
  if (t < kPartSlots) {
    unsigned long long a = red[0][t];
    for (int w = 1; w < kWaves; ++w) {
      const unsigned long long x = red[w][t];
      a = t == P_LMAX ? (x > a ? x : a) : t == P_LMIN ? (x < a ? x : a) : a + x;
    }
    tot[t] = a;
  }
  __syncthreads();
  if (t != 0) return;
  for (int q = 0; q < kPartSlots; ++q) {
    if (q < P_VB0) {
      const int c = q == P_SUMSQ ? C_SUMSQ : q == P_LMAX ? C_LMAX : q == P_LMIN ? C_LMIN
                  : q < P_LONGNNZ ? C_BIN0 + (q - P_BIN0) : q == P_LONGNNZ ? C_LONGNNZ
                  : q == P_DISTLOG ? C_DISTLOG : q == P_NEAR ? C_NEAR : C_NNZ;
      h->cnt[c] = tot[q];
    } else {
      h->bin_count[q - P_VB0] = (int32_t)tot[q];
    }
  }
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
    acc += h->bin_count[b];
  }
}

// Row lists per bin, each sorted by row: workgroup w walks its rows (the same
// ranges as k_stats) 256 at a time; a row's slot is the bin offset + the
// workgroup's base in that bin + the rows of that bin already placed by the
// workgroup + those of lower lanes in this round (ballot prefix counts).
__global__ __launch_bounds__(kWG) void k_scatter_bins(int64_t n, int64_t nnz,
                                                      const int32_t* __restrict__ rp,
                                                      const WsHeader* __restrict__ h,
                                                      const int32_t* __restrict__ bin_base,
                                                      int32_t* __restrict__ rows) {
  __shared__ int32_t wave_cnt[kWG / 64][kNumBins];
  __shared__ int32_t placed[kNumBins];
  int64_t r0, r1;
  row_range_of(n, blockIdx.x, gridDim.x, r0, r1);
  const int wv = threadIdx.x / 64;
  if (threadIdx.x < kNumBins) placed[threadIdx.x] = 0;
  int32_t base[kNumBins];
  for (int b = 0; b < kNumBins; ++b)
    base[b] = h->bin_offset[b] + bin_base[(int64_t)blockIdx.x * kNumBins + b];
  const uint64_t lt = __lanemask_lt();
  // every lane of the workgroup runs the same rounds
  for (int64_t c = r0; c < r1; c += kWG) {
    const int64_t i = c + threadIdx.x;
    int mybin = -1;
    if (i < r1) {
      int64_t s = rp[i], e = rp[i + 1];
      s = s < 0 ? 0 : s > nnz ? nnz : s;
      e = e < s ? s : e > nnz ? nnz : e;
      mybin = variant_bin(e - s);
    }
    int32_t lane_pos = 0;
    for (int b = 0; b < kNumBins; ++b) {
      const uint64_t m = __ballot(mybin == b);
      if (mybin == b) lane_pos = __popcll(m & lt);
      if (threadIdx.x % 64 == 0) wave_cnt[wv][b] = __popcll(m);
    }
    __syncthreads();
    if (mybin >= 0) {
      int32_t before = placed[mybin];
      for (int w = 0; w < wv; ++w) before += wave_cnt[w][mybin];
      rows[base[mybin] + before + lane_pos] = (int32_t)i;
    }
    __syncthreads();
    if (threadIdx.x < kNumBins) {
      int32_t add = 0;
      for (int w = 0; w < kWG / 64; ++w) add += wave_cnt[w][threadIdx.x];
      placed[threadIdx.x] += add;
    }
    __syncthreads();
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

// Staging range of every row block (one workgroup per block): the exact
// column bounds of its chunk [S, min(E, S + budget)) when they span at most
// W, the B entries the LDS array holds (counted in staged_blocks), else a
// W-wide window of columns: of kWinCand windows starting at the one centred on the block's
// rows shifted by multiples of kWinStep columns (clamped to [0, n_cols)), the
// one holding most of the chunk's entries (ties to the least shift). S and E
// are clamped to [0, nnz] so an invalid pattern (reported by validation in
// the same pass) reads nothing out of bounds.
constexpr int kWinCand = 9;     // candidate windows per block
constexpr int kWinStep = 256;   // shift between candidates, in columns
__global__ __launch_bounds__(kWG) void k_block_spans(int64_t nblocks, int64_t nnz, int64_t n_cols,
                                                     const int2* __restrict__ blocks,
                                                     const int32_t* __restrict__ ci,
                                                     int2* __restrict__ spans, WsHeader* h,
                                                     int32_t W) {
  __shared__ int32_t lo[kWG / 64], hi[kWG / 64];
  const int64_t b = blockIdx.x;
  if (b >= nblocks) return;
  int64_t S = blocks[b].y, E = blocks[b + 1].y;
  S = S < 0 ? 0 : S > nnz ? nnz : S;
  E = E < S ? S : E > nnz ? nnz : E;
  if (E - S > kBlockBudget) E = S + kBlockBudget;
  // the chunk's <= kBlockBudget columns, kPer per lane, loaded at once and
  // kept for the window count below
  constexpr int kPer = kBlockBudget / kWG;
  int32_t cc[kPer];
  int32_t a = INT32_MAX, z = INT32_MIN;
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int64_t j = S + threadIdx.x + (int64_t)u * kWG;
    cc[u] = j < E ? ci[j] : -1;
  }
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    if (S + threadIdx.x + (int64_t)u * kWG < E) {
      a = cc[u] < a ? cc[u] : a;
      z = cc[u] > z ? cc[u] : z;
    }
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
    lo[0] = a;  // the block-wide bounds, read by every lane after the barrier
    hi[0] = z;
    if (a > z) {
      spans[b] = make_int2(0, -1);  // empty chunk: nothing staged
    } else if ((int64_t)z - a < W) {
      spans[b] = make_int2(a, z);
      atomicAdd(&h->staged_blocks, 1);
    }
  }
  // wide chunk: every lane counts its entries inside each candidate window
  __syncthreads();
  const int32_t a0 = lo[0], z0 = hi[0];
  if (!(a0 <= z0) || (int64_t)z0 - a0 < W) return;  // block-uniform
  const int64_t mid = ((int64_t)blocks[b].x + blocks[b + 1].x) / 2;
  int64_t w0c[kWinCand];
  int32_t cnt[kWinCand];
  for (int q = 0; q < kWinCand; ++q) {
    int64_t w0 = mid - W / 2 + (int64_t)(q - kWinCand / 2) * kWinStep;
    w0 = w0 + W > n_cols ? n_cols - W : w0;
    w0c[q] = w0 < 0 ? 0 : w0;
    cnt[q] = 0;
  }
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    if (S + threadIdx.x + (int64_t)u * kWG < E) {
      const int64_t c = cc[u];
      for (int q = 0; q < kWinCand; ++q) cnt[q] += c >= w0c[q] && c < w0c[q] + W;
    }
  }
  __shared__ int32_t wc[kWG / 64][kWinCand];
  for (int q = 0; q < kWinCand; ++q) {
    int32_t x = cnt[q];
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
    if (threadIdx.x % 64 == 0) wc[threadIdx.x / 64][q] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int best = kWinCand / 2, best_n = -1;
    for (int k = 0; k < kWinCand; ++k) {
      // candidates in order of increasing shift: centre, -1, +1, -2, +2, ...
      const int q = kWinCand / 2 + ((k & 1) ? -(k + 1) / 2 : k / 2);
      int32_t n = 0;
      for (int w = 0; w < kWG / 64; ++w) n += wc[w][q];
      if (n > best_n) {
        best_n = n;
        best = q;
      }
    }
    const int64_t w1 = w0c[best] + W < n_cols ? w0c[best] + W : n_cols;
    spans[b] = w0c[best] < w1 ? make_int2((int32_t)w0c[best], (int32_t)(w1 - 1))
                              : make_int2(0, -1);
  }
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
  // one statistics workgroup per 256 rows, at most kStatsGrid
  const int g = (int)std::max<int64_t>(1, std::min<int64_t>(kStatsGrid, (p.n_rows + kWG - 1) / kWG));
  if (p.n_rows > 0) {
    k_stats<<<g, kWG, 0, s>>>(p.n_rows, p.nnz, p.row_ptr, p.col_idx, p.stats_part);
    SPMV_HIP(hipGetLastError());
  }
  k_finalize<<<1, kFinWG, 0, s>>>(p.n_rows, p.n_rows > 0 ? g : 0, p.stats_part, p.bin_base, p.hdr,
                              st);
  SPMV_HIP(hipGetLastError());
  if (p.n_rows > 0) {
    k_scatter_bins<<<g, kWG, 0, s>>>(p.n_rows, p.nnz, p.row_ptr, p.hdr, p.bin_base,
                                     p.bin_rows);
    SPMV_HIP(hipGetLastError());
    k_blocks<<<grid_cap(p.nblocks + 1, 1u << 30), kWG, 0, s>>>(p.n_rows, p.nblocks, p.row_ptr,
                                                               p.blocks);
    SPMV_HIP(hipGetLastError());
    if (p.nblocks > 0) {
      // W: the B entries a block stages (twice as many for float32 values)
      k_block_spans<<<(unsigned)p.nblocks, kWG, 0, s>>>(
          p.nblocks, p.nnz, p.n_cols, p.blocks, p.col_idx, p.spans, p.hdr,
          p.vdt == SPMV_F64 ? kStageEntries<double> : kStageEntries<float>);
      SPMV_HIP(hipGetLastError());
    }
  }
  return SPMV_OK;
}

int launch_zero_header(WsHeader* h, hipStream_t s) {
  k_zero_header<<<1, kWG, 0, s>>>(h);
  SPMV_HIP(hipGetLastError());
  return SPMV_OK;
}

}  // namespace spmv
