// CRS product kernels: variants V0..V5 (V4 in its plain and its B-staging
// form; its window form is in window.hip) and the multi-RHS form; V6, which
// reads a chunked copy of the matrix, is in sell.hip.
//
// All compute C(i) = sum_j val(j) * B(col_idx(j)) (the paper's Sect. 1.2
// loop) with float64 accumulation; they differ only in how rows and nonzeros
// are mapped onto lanes. Each output element is reduced by one lane group in
// an order fixed by the matrix structure, so results are reproducible.
#include <type_traits>

#include "common.hpp"
#include "device.hpp"

namespace spmv {
namespace {

using dev::group_sum;
using dev::ld_stream;
using dev::widen;

// ---------------------------------------------------------------- V0
// One lane per row. LIST: rows come from a row list (binned variant).
template <typename VT, typename BT, bool LIST>
__global__ __launch_bounds__(kWG) void k_thread_row(int32_t nrows, const int32_t* __restrict__ list,
                                                    const int32_t* __restrict__ rp,
                                                    const int32_t* __restrict__ ci,
                                                    const VT* __restrict__ val,
                                                    const BT* __restrict__ B,
                                                    double* __restrict__ C) {
  for (int64_t t = (int64_t)blockIdx.x * kWG + threadIdx.x; t < nrows;
       t += (int64_t)gridDim.x * kWG) {
    const int32_t r = LIST ? list[t] : (int32_t)t;
    const int32_t s = rp[r], e = rp[r + 1];
    double acc = 0.0;
    int32_t j = s;
    for (; j + 4 <= e; j += 4) {
      VT v0 = ld_stream(val + j), v1 = ld_stream(val + j + 1), v2 = ld_stream(val + j + 2),
         v3 = ld_stream(val + j + 3);
      int32_t c0 = ld_stream(ci + j), c1 = ld_stream(ci + j + 1), c2 = ld_stream(ci + j + 2),
              c3 = ld_stream(ci + j + 3);
      BT b0 = B[c0], b1 = B[c1], b2 = B[c2], b3 = B[c3];
      acc = fma(widen(v0), widen(b0), acc);
      acc = fma(widen(v1), widen(b1), acc);
      acc = fma(widen(v2), widen(b2), acc);
      acc = fma(widen(v3), widen(b3), acc);
    }
    for (; j < e; ++j) acc = fma(widen(ld_stream(val + j)), widen(B[ld_stream(ci + j)]), acc);
    C[r] = acc;
  }
}

// ---------------------------------------------------------------- V1/V2/V3
// G lanes per row (4, 16 or 64): lane l takes nonzeros s+l, s+l+G, ...;
// coalesced segments of the val/col_idx streams; DPP reduction.
template <typename VT, typename BT, int G, bool LIST>
__global__ __launch_bounds__(kWG) void k_group_row(int32_t nrows, const int32_t* __restrict__ list,
                                                   const int32_t* __restrict__ rp,
                                                   const int32_t* __restrict__ ci,
                                                   const VT* __restrict__ val,
                                                   const BT* __restrict__ B,
                                                   double* __restrict__ C) {
  const int lane = threadIdx.x & (G - 1);
  // grid-stride over groups: the grid is capped (rows x G lanes can exceed
  // what one dispatch holds); whole groups leave together
  const int64_t stride = (int64_t)gridDim.x * (kWG / G);
  for (int64_t g = ((int64_t)blockIdx.x * kWG + threadIdx.x) / G; g < nrows; g += stride) {
    const int32_t r = LIST ? list[g] : (int32_t)g;
    const int32_t s = rp[r], e = rp[r + 1];
    double part = 0.0;
    int32_t j = s + lane;
    for (; j + G < e; j += 2 * G) {
      VT v0 = ld_stream(val + j), v1 = ld_stream(val + j + G);
      int32_t c0 = ld_stream(ci + j), c1 = ld_stream(ci + j + G);
      BT b0 = B[c0], b1 = B[c1];
      part = fma(widen(v0), widen(b0), part);
      part = fma(widen(v1), widen(b1), part);
    }
    if (j < e) part = fma(widen(ld_stream(val + j)), widen(B[ld_stream(ci + j)]), part);
    const double sum = group_sum<G>(part);
    if (lane == 0) C[r] = sum;
  }
}

// Whole workgroup per row (very long rows of the binned variant).
template <typename VT, typename BT>
__global__ __launch_bounds__(kWG) void k_block_row(int32_t nrows, const int32_t* __restrict__ list,
                                                   const int32_t* __restrict__ rp,
                                                   const int32_t* __restrict__ ci,
                                                   const VT* __restrict__ val,
                                                   const BT* __restrict__ B,
                                                   double* __restrict__ C) {
  __shared__ double wsum[kWG / 64];
  const int32_t r = list[blockIdx.x];
  const int32_t s = rp[r], e = rp[r + 1];
  const double part = group_sum<64>(dev::stream_row_part<VT, BT>(val, ci, B, s, e));
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = part;
  __syncthreads();
  if (threadIdx.x == 0) C[r] = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
  (void)nrows;
}

// ---------------------------------------------------------------- V4
template <typename VT, typename BT, bool ACC>
__global__ __launch_bounds__(kWG) void k_lds_block(int64_t nblocks, const int2* __restrict__ blocks,
                                                   const int32_t* __restrict__ rp,
                                                   const int32_t* __restrict__ ci,
                                                   const VT* __restrict__ val,
                                                   const BT* __restrict__ B,
                                                   double* __restrict__ C) {
  __shared__ dev::BlockLds L;
  const int64_t b = dev::xcd_remap(blockIdx.x, nblocks);
  const int2 m0 = blocks[b], m1 = blocks[b + 1];
  if (m0.x >= m1.x) return;
  dev::lds_block<VT, BT, ACC>(L, rp, ci, val, B, C, m0.x, m1.x, m0.y, m1.y);
}

// The same with B staging: each block copies its staging range of B (the
// exact column span when it fits the LDS product array, else a window around
// the block's rows) into LDS and gathers from it where it can. The staging
// path costs registers and changes the compiler's load schedule, so it is a
// kernel of its own; a plan uses it when at least a quarter of its blocks fit
// exactly, or when autotune measured it faster.
template <typename VT, typename BT, bool ACC>
__global__ __launch_bounds__(kWG) void k_lds_block_staged(int64_t nblocks,
                                                          const int2* __restrict__ blocks,
                                                          const int2* __restrict__ spans,
                                                          const int32_t* __restrict__ rp,
                                                          const int32_t* __restrict__ ci,
                                                          const VT* __restrict__ val,
                                                          const BT* __restrict__ B,
                                                          double* __restrict__ C) {
  __shared__ dev::BlockLds L;
  const int64_t b = dev::xcd_remap(blockIdx.x, nblocks);
  const int2 m0 = blocks[b], m1 = blocks[b + 1], sp = spans[b];
  if (m0.x >= m1.x) return;
  // float32 B: twice the entries in the same LDS (the spans were chosen for it)
  dev::lds_block<VT, BT, ACC, true>(L, rp, ci, val, B, C, m0.x, m1.x, m0.y, m1.y, sp.x, sp.y,
                                    L.prod, kStageEntries<BT>);
}

template <typename VT, typename BT, bool ACC>
void launch_lds_block(const Plan& p, const VT* val, const BT* B, double* C, hipStream_t s) {
  if (p.nblocks <= 0) return;
  if (!ACC && p.v4_form == kV4Window) {
    launch_win(p, B, C, s);
    return;
  }
  if (p.v4_form == kV4Staged)
    k_lds_block_staged<VT, BT, ACC><<<(unsigned)p.nblocks, kWG, 0, s>>>(
        p.nblocks, p.blocks, p.spans, p.row_ptr, p.col_idx, val, B, C);
  else
    k_lds_block<VT, BT, ACC><<<(unsigned)p.nblocks, kWG, 0, s>>>(p.nblocks, p.blocks, p.row_ptr,
                                                                 p.col_idx, val, B, C);
}

// ---------------------------------------------------------------- SpMM
// LPR lanes per row; lane l owns columns [c0, c0+CPL) with c0 = l*CPL + t*LPR*CPL.
// Each gathered B row segment is loaded as 16-byte vectors (CPL = 4 in
// float64 is two of them). A row is processed kSpmmU entries per round: all
// val/col loads of the round first, then all B segments, then the FMAs, so a
// short row costs three dependent round trips instead of one per entry pair.
constexpr int kSpmmU = 8;

template <typename T, int N>
struct Vec;
template <>
struct Vec<double, 1> { using type = double; };
template <>
struct Vec<double, 2> { using type = double2; };
template <>
struct Vec<float, 1> { using type = float; };
template <>
struct Vec<float, 2> { using type = float2; };
template <>
struct Vec<float, 4> { using type = float4; };

template <typename BT, int CPL>
__device__ __forceinline__ void load_vec(const BT* p, double* out) {
  if constexpr (std::is_same<BT, double>::value && CPL == 4) {
    load_vec<double, 2>(p, out);
    load_vec<double, 2>(p + 2, out + 2);
  } else {
    using V = typename Vec<BT, CPL>::type;
    V x = *reinterpret_cast<const V*>(p);
    if constexpr (CPL == 1) {
      out[0] = (double)x;
    } else if constexpr (CPL == 2) {
      out[0] = (double)x.x; out[1] = (double)x.y;
    } else {
      out[0] = (double)x.x; out[1] = (double)x.y; out[2] = (double)x.z; out[3] = (double)x.w;
    }
  }
}

template <int CPL>
__device__ __forceinline__ void store_vec(double* p, const double* x) {
  if constexpr (CPL == 1) {
    p[0] = x[0];
  } else {
#pragma unroll
    for (int t = 0; t < CPL; t += 2) *reinterpret_cast<double2*>(p + t) = double2{x[t], x[t + 1]};
  }
}

// VST: C rows are 16-byte aligned (vector stores of full column groups).
// SB: B rows are not aligned for vector loads (odd ldb, or an offset B):
// every column group takes the scalar-load path.
template <typename VT, typename BT, int LPR, int CPL, bool VST, bool SB>
__global__ __launch_bounds__(kWG) void k_spmm(int32_t nrows, int32_t k,
                                              const int32_t* __restrict__ rp,
                                              const int32_t* __restrict__ ci,
                                              const VT* __restrict__ val,
                                              const BT* __restrict__ B, int64_t ldb,
                                              double* __restrict__ C, int64_t ldc) {
  const int lane = threadIdx.x & (LPR - 1);
  // grid-stride over rows (the grid is capped: rows x LPR lanes can exceed
  // what one dispatch holds); the lanes of a row leave together
  const int64_t row_stride = (int64_t)gridDim.x * (kWG / LPR);
  for (int64_t row = ((int64_t)blockIdx.x * kWG + threadIdx.x) / LPR; row < nrows;
       row += row_stride) {
  const int32_t s = rp[row], e = rp[row + 1];
  for (int32_t c0 = lane * CPL; c0 < k; c0 += LPR * CPL) {
    double acc[CPL];
#pragma unroll
    for (int t = 0; t < CPL; ++t) acc[t] = 0.0;
    double* out = C + row * ldc + c0;
    if (!SB && c0 + CPL <= k) {
      // full column group: vector loads of B, masked entries read nothing
      if constexpr (!std::is_same<VT, double>::value || !std::is_same<BT, double>::value) {
        // narrower types: loaded in their own type and widened only after
        // every load of the round is issued (the empty asm pins keep each
        // widening from being moved next to its load, where it would wait)
        using V = typename Vec<BT, CPL>::type;
        for (int32_t j = s; j < e; j += kSpmmU) {
          VT vr[kSpmmU];
          int32_t c[kSpmmU];
#pragma unroll
          for (int u = 0; u < kSpmmU; ++u) {
            const bool in = j + u < e;
            vr[u] = in ? val[j + u] : (VT)0;
            c[u] = in ? ci[j + u] : -1;
          }
          BT b[kSpmmU][CPL];
#pragma unroll
          for (int u = 0; u < kSpmmU; ++u) {
            V x{};
            if (c[u] >= 0) x = *reinterpret_cast<const V*>(B + (int64_t)c[u] * ldb + c0);
            static_assert(CPL == 1 || CPL == 2 || CPL == 4,
                          "float column groups are 1, 2 or 4 wide");
            if constexpr (CPL == 1) {
              b[u][0] = x;
            } else if constexpr (CPL == 2) {
              b[u][0] = x.x;
              b[u][1] = x.y;
            } else {
              b[u][0] = x.x;
              b[u][1] = x.y;
              b[u][2] = x.z;
              b[u][3] = x.w;
            }
          }
#pragma unroll
          for (int u = 0; u < kSpmmU; ++u) {
            asm volatile("" : "+v"(vr[u]));
#pragma unroll
            for (int t = 0; t < CPL; ++t) asm volatile("" : "+v"(b[u][t]));
          }
#pragma unroll
          for (int u = 0; u < kSpmmU; ++u)
#pragma unroll
            for (int t = 0; t < CPL; ++t)
              acc[t] = fma(widen(vr[u]), (double)b[u][t], acc[t]);
        }
      } else
      for (int32_t j = s; j < e; j += kSpmmU) {
        double v[kSpmmU];
        int32_t c[kSpmmU];
#pragma unroll
        for (int u = 0; u < kSpmmU; ++u) {
          const bool in = j + u < e;
          v[u] = in ? widen(val[j + u]) : 0.0;
          c[u] = in ? ci[j + u] : -1;
        }
        double b[kSpmmU][CPL];
#pragma unroll
        for (int u = 0; u < kSpmmU; ++u) {
          if (c[u] >= 0) {
            load_vec<BT, CPL>(B + (int64_t)c[u] * ldb + c0, b[u]);
          } else {
#pragma unroll
            for (int t = 0; t < CPL; ++t) b[u][t] = 0.0;
          }
        }
        // masked entries add fma(0, 0, acc) = acc exactly (acc is never -0)
#pragma unroll
        for (int u = 0; u < kSpmmU; ++u)
#pragma unroll
          for (int t = 0; t < CPL; ++t) acc[t] = fma(v[u], b[u][t], acc[t]);
      }
      if constexpr (VST) {
        store_vec<CPL>(out, acc);
      } else {
#pragma unroll
        for (int t = 0; t < CPL; ++t) out[t] = acc[t];
      }
    } else {
      // last, partial column group (k not a multiple of CPL), or any group of
      // an unaligned B: the same rounds of kSpmmU entries with the B elements
      // loaded one by one (an entry at a time made each entry's loads wait
      // for the previous entry's FMAs: k = 6 took twice as long as k = 8)
      const int32_t kc = k - c0;
      for (int32_t j = s; j < e; j += kSpmmU) {
        VT vr[kSpmmU];
        int32_t c[kSpmmU];
#pragma unroll
        for (int u = 0; u < kSpmmU; ++u) {
          const bool in = j + u < e;
          vr[u] = in ? val[j + u] : (VT)0;
          c[u] = in ? ci[j + u] : -1;
        }
        BT b[kSpmmU][CPL];
#pragma unroll
        for (int u = 0; u < kSpmmU; ++u) {
          const BT* bq = B + (int64_t)(c[u] >= 0 ? c[u] : 0) * ldb + c0;
#pragma unroll
          for (int t = 0; t < CPL; ++t) b[u][t] = (c[u] >= 0 && t < kc) ? bq[t] : (BT)0;
        }
        if constexpr (!std::is_same<VT, double>::value || !std::is_same<BT, double>::value) {
#pragma unroll
          for (int u = 0; u < kSpmmU; ++u) {
            asm volatile("" : "+v"(vr[u]));
#pragma unroll
            for (int t = 0; t < CPL; ++t) asm volatile("" : "+v"(b[u][t]));
          }
        }
        // masked entries add fma(0, 0, acc) = acc exactly (acc is never -0)
#pragma unroll
        for (int u = 0; u < kSpmmU; ++u)
#pragma unroll
          for (int t = 0; t < CPL; ++t)
            acc[t] = fma(widen(vr[u]), (double)b[u][t], acc[t]);
      }
#pragma unroll
      for (int t = 0; t < CPL; ++t)
        if (t < kc) out[t] = acc[t];
    }
  }
  }
}

// ---------------------------------------------------------------- fill
template <typename T>
__global__ void k_fill(T* p, int64_t n, T v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Workgroups for `threads` lanes of a grid-stride kernel, at most kMaxGrid
// (n_rows x 64 lanes can pass the 2^32 work-items of one dispatch).
constexpr int64_t kMaxGrid = 1 << 20;
inline unsigned grid_for(int64_t threads) {
  const int64_t g = (threads + kWG - 1) / kWG;
  return (unsigned)(g < kMaxGrid ? g : kMaxGrid);
}

template <typename VT, typename BT>
int spmv_typed(const Plan& p, int variant, const BT* B, double* C, hipStream_t s) {
  const VT* val = static_cast<const VT*>(p.val);
  const int32_t n = (int32_t)p.n_rows;
  if (n == 0) return SPMV_OK;
  switch (variant) {
    case SPMV_V0_THREAD_ROW:
      k_thread_row<VT, BT, false><<<grid_for(n), kWG, 0, s>>>(n, nullptr, p.row_ptr, p.col_idx,
                                                              val, B, C);
      break;
    case SPMV_V1_LANES4:
      k_group_row<VT, BT, 4, false><<<grid_for((int64_t)n * 4), kWG, 0, s>>>(
          n, nullptr, p.row_ptr, p.col_idx, val, B, C);
      break;
    case SPMV_V2_LANES16:
      k_group_row<VT, BT, 16, false><<<grid_for((int64_t)n * 16), kWG, 0, s>>>(
          n, nullptr, p.row_ptr, p.col_idx, val, B, C);
      break;
    case SPMV_V3_WAVE_ROW:
      k_group_row<VT, BT, 64, false><<<grid_for((int64_t)n * 64), kWG, 0, s>>>(
          n, nullptr, p.row_ptr, p.col_idx, val, B, C);
      break;
    case SPMV_V4_LDS_BLOCK:
      launch_lds_block<VT, BT, false>(p, val, B, C, s);
      break;
    case SPMV_V5_BINNED: {
      const int32_t* L = p.bin_rows;
      const int32_t* o = p.bin_offset;
      const int32_t* c = p.bin_count;
      if (c[0])
        k_thread_row<VT, BT, true><<<grid_for(c[0]), kWG, 0, s>>>(c[0], L + o[0], p.row_ptr,
                                                                  p.col_idx, val, B, C);
      if (c[1])
        k_group_row<VT, BT, 4, true><<<grid_for((int64_t)c[1] * 4), kWG, 0, s>>>(
            c[1], L + o[1], p.row_ptr, p.col_idx, val, B, C);
      if (c[2])
        k_group_row<VT, BT, 16, true><<<grid_for((int64_t)c[2] * 16), kWG, 0, s>>>(
            c[2], L + o[2], p.row_ptr, p.col_idx, val, B, C);
      if (c[3])
        k_group_row<VT, BT, 64, true><<<grid_for((int64_t)c[3] * 64), kWG, 0, s>>>(
            c[3], L + o[3], p.row_ptr, p.col_idx, val, B, C);
      if (c[4])
        k_block_row<VT, BT><<<(unsigned)c[4], kWG, 0, s>>>(c[4], L + o[4], p.row_ptr,
                                                           p.col_idx, val, B, C);
      break;
    }
    case SPMV_V6_SELL64:
      return launch_sell(p, B, C, s);
    default:
      return fail(SPMV_ERR_INVALID_ARG, "unknown variant");
  }
  SPMV_HIP(hipGetLastError());
  return SPMV_OK;
}

template <typename VT, typename BT, int CPL, bool VST, bool SB>
int spmm_lpr(const Plan& p, int k, const BT* B, int64_t ldb, double* C, int64_t ldc,
             hipStream_t s) {
  const VT* val = static_cast<const VT*>(p.val);
  const int32_t n = (int32_t)p.n_rows;
  int need = (k + CPL - 1) / CPL;
  int lpr = 1;
  while (lpr < need && lpr < 64) lpr *= 2;
#define SPMM_CASE(L)                                                                        \
  case L:                                                                                   \
    k_spmm<VT, BT, L, CPL, VST, SB><<<grid_for((int64_t)n * L), kWG, 0, s>>>(               \
        n, k, p.row_ptr, p.col_idx, val, B, ldb, C, ldc);                                   \
    break;
  switch (lpr) {
    SPMM_CASE(1)
    SPMM_CASE(2)
    SPMM_CASE(4)
    SPMM_CASE(8)
    SPMM_CASE(16)
    SPMM_CASE(32)
    SPMM_CASE(64)
  }
#undef SPMM_CASE
  SPMV_HIP(hipGetLastError());
  return SPMV_OK;
}

template <typename VT, typename BT, int CPL, bool SB = false>
int spmm_store(const Plan& p, int k, const BT* B, int64_t ldb, double* C, int64_t ldc,
               hipStream_t s) {
  const bool vst = CPL > 1 && reinterpret_cast<uintptr_t>(C) % 16 == 0 && ldc % 2 == 0;
  return vst ? spmm_lpr<VT, BT, CPL, (CPL > 1), SB>(p, k, B, ldb, C, ldc, s)
             : spmm_lpr<VT, BT, CPL, false, SB>(p, k, B, ldb, C, ldc, s);
}

template <typename VT, typename BT>
int spmv_accumulate_typed(const Plan& p, const BT* B, double* C, hipStream_t s) {
  launch_lds_block<VT, BT, true>(p, static_cast<const VT*>(p.val), B, C, s);
  SPMV_HIP(hipGetLastError());
  return SPMV_OK;
}

}  // namespace

int launch_spmv_accumulate(const Plan& p, const void* B, double* C, hipStream_t s) {
  if (p.vdt == SPMV_F64)
    return spmv_accumulate_typed<double, double>(p, static_cast<const double*>(B), C, s);
  return spmv_accumulate_typed<float, float>(p, static_cast<const float*>(B), C, s);
}

int launch_spmv(const Plan& p, int variant, const void* B, double* C, hipStream_t s) {
  if (p.vdt == SPMV_F64)
    return spmv_typed<double, double>(p, variant, static_cast<const double*>(B), C, s);
  return spmv_typed<float, float>(p, variant, static_cast<const float*>(B), C, s);
}

int launch_spmm(const Plan& p, int k, const void* B, int64_t ldb, double* C, int64_t ldc,
                hipStream_t s) {
  if (p.n_rows == 0) return SPMV_OK;
  const uintptr_t a = reinterpret_cast<uintptr_t>(B);
  // column groups of 4 unless k = 2 mod 4, where groups of 2 leave no
  // partial group (k = 6 and 10 took twice as long with a partial group of 2)
  if (p.vdt == SPMV_F64) {
    const double* b = static_cast<const double*>(B);
    if (k >= 4 && k % 4 != 2 && a % 16 == 0 && ldb % 2 == 0)
      return spmm_store<double, double, 4>(p, k, b, ldb, C, ldc, s);
    if (k >= 2 && a % 16 == 0 && ldb % 2 == 0)
      return spmm_store<double, double, 2>(p, k, b, ldb, C, ldc, s);
    // B rows not aligned for vector loads (odd ldb): from k = 5 on, groups
    // of 4 columns with scalar loads (one column per lane re-reads every
    // row's entries in each of up to 16 lanes: k = 9 took 1.5x as long on a
    // 3M-row matrix; for k = 3 one column per lane was 14% faster)
    if (k >= 5) return spmm_store<double, double, 4, true>(p, k, b, ldb, C, ldc, s);
    return spmm_store<double, double, 1>(p, k, b, ldb, C, ldc, s);
  }
  const float* b = static_cast<const float*>(B);
  if (k >= 4 && k % 4 != 2 && a % 16 == 0 && ldb % 4 == 0)
    return spmm_store<float, float, 4>(p, k, b, ldb, C, ldc, s);
  if (k >= 2 && a % 8 == 0 && ldb % 2 == 0)
    return spmm_store<float, float, 2>(p, k, b, ldb, C, ldc, s);
  // unaligned float32 rows: scalar groups of 4 from k = 9 on (k = 5 and 7
  // ran 15-18% faster with one column per lane)
  if (k >= 9) return spmm_store<float, float, 4, true>(p, k, b, ldb, C, ldc, s);
  return spmm_store<float, float, 1>(p, k, b, ldb, C, ldc, s);
}

int launch_fill(void* dst, int dtype, int64_t n, double value, hipStream_t s) {
  if (n <= 0) return SPMV_OK;
  const unsigned g = (unsigned)std::min<int64_t>((n + kWG - 1) / kWG, 4096);
  if (dtype == SPMV_F64)
    k_fill<double><<<g, kWG, 0, s>>>(static_cast<double*>(dst), n, value);
  else
    k_fill<float><<<g, kWG, 0, s>>>(static_cast<float*>(dst), n, (float)value);
  SPMV_HIP(hipGetLastError());
  return SPMV_OK;
}

}  // namespace spmv
