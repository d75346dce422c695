// Variant V6: the CRS product of Sect. 1.2 computed from a chunked copy of
// the matrix. Rows are cut into chunks of 64 consecutive rows (one chunk per
// wavefront, no reordering); a chunk is stored column by column with the
// width of its longest row, so slot (j, lane) of chunk k holds the j-th
// nonzero of row 64 k + lane. Shorter rows are padded with col = -1, val = 0.
// This is a sliced ELLPACK layout with slice height 64 (the SELL-C-sigma
// family with C = 64, sigma = 1). Every load of val and col_idx is then one
// contiguous 512- or 256-byte access per wavefront, no LDS or barrier is
// needed, and each row is still summed in CRS order by one lane.
//
// The copy is built on the device at plan creation in three passes: chunk
// widths, an exclusive scan of the widths, and the fill. Its capacity is
// reserved in the plan workspace; a pattern whose padded size does not fit
// is reported back and V6 is then unavailable for that plan.
#include "common.hpp"
#include "device.hpp"

namespace spmv {
namespace {

constexpr int kChunk = 64;  // rows per chunk = lanes per wavefront
constexpr int kSellU = 16;  // slots of one row loaded before the first is used

// Clamped row range: an invalid pattern (reported by validation, which runs
// earlier in the same stream) never makes these kernels read out of bounds.
__device__ __forceinline__ void row_range(int64_t r, int64_t n, int64_t nnz,
                                          const int32_t* __restrict__ rp, int64_t& s,
                                          int64_t& e) {
  s = 0;
  e = 0;
  if (r < n) {
    s = rp[r];
    e = rp[r + 1];
    s = s < 0 ? 0 : s > nnz ? nnz : s;
    e = e < s ? s : e > nnz ? nnz : e;
  }
}

// Width of every chunk = longest row in it (one wavefront per chunk).
__global__ __launch_bounds__(kWG) void k_sell_width(int64_t n, int64_t nnz,
                                                    const int32_t* __restrict__ rp,
                                                    int64_t nch, int32_t* __restrict__ width) {
  const int64_t chunk = ((int64_t)blockIdx.x * kWG + threadIdx.x) / kChunk;
  if (chunk >= nch) return;
  int64_t s, e;
  row_range(chunk * kChunk + (threadIdx.x % kChunk), n, nnz, rp, s, e);
  int64_t w = e - s;
  for (int o = 32; o >= 1; o >>= 1) {
    const int64_t x = __shfl_xor(w, o);
    w = x > w ? x : w;
  }
  if (threadIdx.x % kChunk == 0) width[chunk] = (int32_t)w;
}

// Fill the chunked copy. off = exclusive scan of the widths (nch + 1
// entries, in units of 64 slots). Nothing is written unless every chunk's
// slot range lies inside the reserved capacity.
template <typename VT>
__global__ __launch_bounds__(kWG) void k_sell_fill(
    int64_t n, int64_t nnz, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
    const VT* __restrict__ val, int64_t nch, const int32_t* __restrict__ off, int64_t cap64,
    int32_t* __restrict__ sci, VT* __restrict__ sval, int64_t* __restrict__ total_out) {
  const int64_t total = off[nch];
  if (blockIdx.x == 0 && threadIdx.x == 0) *total_out = total;
  const int64_t chunk = ((int64_t)blockIdx.x * kWG + threadIdx.x) / kChunk;
  if (chunk >= nch || total < 0 || total > cap64) return;
  const int64_t a = off[chunk], b = off[chunk + 1];
  if (a < 0 || b < a || b > total) return;
  const int lane = threadIdx.x % kChunk;
  int64_t s, e;
  row_range(chunk * kChunk + lane, n, nnz, rp, s, e);
  const int64_t len = e - s;
  int32_t* dc = sci + a * kChunk + lane;
  VT* dv = sval + a * kChunk + lane;
  for (int64_t j = 0; j < b - a; ++j) {
    if (j < len) {
      dc[j * kChunk] = ci[s + j];
      dv[j * kChunk] = val[s + j];
    } else {
      dc[j * kChunk] = -1;
      dv[j * kChunk] = (VT)0;
    }
  }
}

// C = A*B from the chunked copy: lane l of the wavefront of chunk k owns row
// 64 k + l and sums its slots in order. The width is uniform over the
// wavefront, so the loop and its masked last round are uniform branches.
template <typename VT, typename BT>
__global__ __launch_bounds__(kWG) void k_sell(int64_t nch, int64_t n,
                                              const int32_t* __restrict__ off,
                                              const int32_t* __restrict__ sci,
                                              const VT* __restrict__ sval,
                                              const BT* __restrict__ B, double* __restrict__ C) {
  const int64_t chunk = ((int64_t)blockIdx.x * kWG + threadIdx.x) / kChunk;
  if (chunk >= nch) return;
  const int lane = threadIdx.x % kChunk;
  const int64_t a = off[chunk];
  const int32_t w = (int32_t)(off[chunk + 1] - a);
  const VT* vp = sval + a * kChunk + lane;
  const int32_t* cp = sci + a * kChunk + lane;
  double acc = 0.0;
  for (int32_t j = 0; j < w; j += kSellU) {
    VT v[kSellU];
    int32_t c[kSellU];
    double x[kSellU];
#pragma unroll
    for (int u = 0; u < kSellU; ++u) {
      if (j + u < w) {
        v[u] = dev::ld_stream(vp + (int64_t)(j + u) * kChunk);
        c[u] = dev::ld_stream(cp + (int64_t)(j + u) * kChunk);
      } else {
        v[u] = (VT)0;
        c[u] = -1;
      }
    }
#pragma unroll
    for (int u = 0; u < kSellU; ++u) x[u] = c[u] >= 0 ? (double)B[c[u]] : 0.0;
    // padded and masked slots contribute fma(0, 0, acc) = acc exactly: acc
    // starts at +0, and a round-to-nearest sum with a +0 operand is never -0,
    // so acc is never -0
#pragma unroll
    for (int u = 0; u < kSellU; ++u) acc = fma(dev::widen(v[u]), x[u], acc);
  }
  const int64_t row = chunk * kChunk + lane;
  if (row < n) C[row] = acc;
}

inline unsigned grid_chunks(int64_t nch) {
  return (unsigned)((nch * kChunk + kWG - 1) / kWG);
}

}  // namespace

int64_t sell_chunks(int64_t n_rows) { return (n_rows + kChunk - 1) / kChunk; }

int64_t sell_capacity(int64_t nnz) {
  const int64_t slots = nnz + nnz / 2 + 4096;
  return (slots + kChunk - 1) / kChunk * kChunk;
}

int launch_sell_build(Plan& p, hipStream_t s) {
  const int64_t nch = p.sell_nch;
  if (nch == 0) return SPMV_OK;
  k_sell_width<<<grid_chunks(nch), kWG, 0, s>>>(p.n_rows, p.nnz, p.row_ptr, nch, p.sell_width);
  SPMV_HIP(hipGetLastError());
  int st = launch_exclusive_scan(p.sell_width, p.sell_off, nch, p.sell_partials, s);
  if (st) return st;
  const int64_t cap64 = p.sell_cap / kChunk;
  if (p.vdt == SPMV_F64)
    k_sell_fill<double><<<grid_chunks(nch), kWG, 0, s>>>(
        p.n_rows, p.nnz, p.row_ptr, p.col_idx, static_cast<const double*>(p.val), nch,
        p.sell_off, cap64, p.sell_ci, static_cast<double*>(p.sell_val), &p.hdr->sell_total);
  else
    k_sell_fill<float><<<grid_chunks(nch), kWG, 0, s>>>(
        p.n_rows, p.nnz, p.row_ptr, p.col_idx, static_cast<const float*>(p.val), nch,
        p.sell_off, cap64, p.sell_ci, static_cast<float*>(p.sell_val), &p.hdr->sell_total);
  SPMV_HIP(hipGetLastError());
  return SPMV_OK;
}

int launch_sell(const Plan& p, const void* B, double* C, hipStream_t s) {
  if (!p.sell_ok) return fail(SPMV_ERR_STATE, "V6 is not built for this plan");
  if (p.sell_nch == 0) return SPMV_OK;
  if (p.vdt == SPMV_F64)
    k_sell<double, double><<<grid_chunks(p.sell_nch), kWG, 0, s>>>(
        p.sell_nch, p.n_rows, p.sell_off, p.sell_ci, static_cast<const double*>(p.sell_val),
        static_cast<const double*>(B), C);
  else
    k_sell<float, float><<<grid_chunks(p.sell_nch), kWG, 0, s>>>(
        p.sell_nch, p.n_rows, p.sell_off, p.sell_ci, static_cast<const float*>(p.sell_val),
        static_cast<const float*>(B), C);
  SPMV_HIP(hipGetLastError());
  return SPMV_OK;
}

}  // namespace spmv
