// Local/remote split of a CRS matrix (the paper's Sect. 3.1 overlap kernel
// structure): entries whose column lies in [col_lo, col_hi) form the local
// part, the others the remote part. Both parts keep the original column
// indices and the original order of entries inside each row.
#include "common.hpp"

namespace spmv {
namespace {

__global__ __launch_bounds__(kWG) void k_split_count(int64_t n, const int32_t* __restrict__ rp,
                                                     const int32_t* __restrict__ ci,
                                                     int64_t lo, int64_t hi,
                                                     int32_t* __restrict__ len_loc,
                                                     int32_t* __restrict__ len_rem) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    int32_t a = 0, b = 0;
    for (int32_t j = rp[i]; j < rp[i + 1]; ++j) {
      const int64_t c = ci[j];
      if (c >= lo && c < hi)
        ++a;
      else
        ++b;
    }
    len_loc[i] = a;
    len_rem[i] = b;
  }
}

// Exclusive scan in three launches: per-block scan (kScanBlock entries per
// workgroup, totals to `partials`), scan of the totals by one workgroup,
// then the block offsets added. out has n+1 entries (out[n] = total).
constexpr int kScanBlock = 1024;

__device__ __forceinline__ int32_t block_exclusive_scan(int32_t x, int32_t* sh, int32_t* total) {
  // Hillis-Steele over kScanBlock lanes in LDS
  const int t = threadIdx.x;
  sh[t] = x;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    const int32_t y = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += y;
    __syncthreads();
  }
  const int32_t incl = sh[t];
  if (t == kScanBlock - 1) *total = incl;
  return incl - x;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_blocks(const int32_t* __restrict__ in,
                                                            int32_t* __restrict__ out, int64_t n,
                                                            int32_t* __restrict__ partials) {
  __shared__ int32_t sh[kScanBlock];
  __shared__ int32_t total;
  const int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
  const int32_t x = i < n ? in[i] : 0;
  const int32_t ex = block_exclusive_scan(x, sh, &total);
  if (i < n) out[i] = ex;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_partials(int32_t* __restrict__ partials,
                                                              int64_t np,
                                                              int32_t* __restrict__ grand) {
  __shared__ int32_t sh[kScanBlock];
  __shared__ int32_t total;
  int32_t carry = 0;
  for (int64_t base = 0; base < np; base += kScanBlock) {
    const int64_t i = base + threadIdx.x;
    const int32_t x = i < np ? partials[i] : 0;
    const int32_t ex = block_exclusive_scan(x, sh, &total);
    if (i < np) partials[i] = carry + ex;
    __syncthreads();
    carry += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) *grand = carry;
}

__global__ __launch_bounds__(kWG) void k_scan_add(int32_t* __restrict__ out, int64_t n,
                                                  const int32_t* __restrict__ partials,
                                                  const int32_t* __restrict__ grand) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += stride)
    out[i] = i < n ? out[i] + partials[i / kScanBlock] : *grand;
}

template <typename VT>
__global__ __launch_bounds__(kWG) void k_split_fill(
    int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
    const VT* __restrict__ val, int64_t lo, int64_t hi, const int32_t* __restrict__ rp_loc,
    const int32_t* __restrict__ rp_rem, int32_t* __restrict__ ci_loc, VT* __restrict__ val_loc,
    int32_t* __restrict__ ci_rem, VT* __restrict__ val_rem) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    int32_t a = rp_loc[i], b = rp_rem[i];
    for (int32_t j = rp[i]; j < rp[i + 1]; ++j) {
      const int32_t c = ci[j];
      if ((int64_t)c >= lo && (int64_t)c < hi) {
        ci_loc[a] = c;
        val_loc[a++] = val[j];
      } else {
        ci_rem[b] = c;
        val_rem[b++] = val[j];
      }
    }
  }
}

unsigned gs(int64_t n) {
  int64_t g = (n + kWG - 1) / kWG;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 8192));
}

}  // namespace

int scan_partials_count(int64_t n) { return (int)((n + kScanBlock - 1) / kScanBlock) + 1; }

int launch_split_count(int64_t n, const int32_t* rp, const int32_t* ci, int64_t col_lo,
                       int64_t col_hi, int32_t* len_loc, int32_t* len_rem, hipStream_t s) {
  if (n <= 0) return SPMV_OK;
  k_split_count<<<gs(n), kWG, 0, s>>>(n, rp, ci, col_lo, col_hi, len_loc, len_rem);
  SPMV_HIP(hipGetLastError());
  return SPMV_OK;
}

int launch_exclusive_scan(const int32_t* in, int32_t* out, int64_t n, int32_t* partials,
                          hipStream_t s) {
  const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  int32_t* grand = partials + nb;  // partials holds nb + 1 entries
  if (nb > 0) {
    k_scan_blocks<<<(unsigned)nb, kScanBlock, 0, s>>>(in, out, n, partials);
    SPMV_HIP(hipGetLastError());
  }
  k_scan_partials<<<1, kScanBlock, 0, s>>>(partials, nb, grand);
  SPMV_HIP(hipGetLastError());
  k_scan_add<<<gs(n + 1), kWG, 0, s>>>(out, n, partials, grand);
  SPMV_HIP(hipGetLastError());
  return SPMV_OK;
}

int launch_split_fill(int64_t n, const int32_t* rp, const int32_t* ci, const void* val, int vdt,
                      int64_t col_lo, int64_t col_hi, const int32_t* rp_loc,
                      const int32_t* rp_rem, int32_t* ci_loc, void* val_loc, int32_t* ci_rem,
                      void* val_rem, hipStream_t s) {
  if (n <= 0) return SPMV_OK;
  if (vdt == SPMV_F64)
    k_split_fill<double><<<gs(n), kWG, 0, s>>>(
        n, rp, ci, static_cast<const double*>(val), col_lo, col_hi, rp_loc, rp_rem, ci_loc,
        static_cast<double*>(val_loc), ci_rem, static_cast<double*>(val_rem));
  else
    k_split_fill<float><<<gs(n), kWG, 0, s>>>(
        n, rp, ci, static_cast<const float*>(val), col_lo, col_hi, rp_loc, rp_rem, ci_loc,
        static_cast<float*>(val_loc), ci_rem, static_cast<float*>(val_rem));
  SPMV_HIP(hipGetLastError());
  return SPMV_OK;
}

}  // namespace spmv
