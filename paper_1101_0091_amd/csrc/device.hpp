// Device-side building blocks: lane-group reductions with DPP, the XCD-aware
// workgroup remap, streaming loads, and the LDS row-block product that both
// the single-matrix and the batched kernels use.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "common.hpp"

namespace spmv {
namespace dev {

// ------------------------------------------------------------ reductions
// DPP controls of the GCN/CDNA data-parallel-primitive word (gfx9 family).
constexpr int kQuadXor1 = 0xB1;     // quad_perm [1,0,3,2]
constexpr int kQuadXor2 = 0x4E;     // quad_perm [2,3,0,1]
constexpr int kRowHalfMirror = 0x141;
constexpr int kRowMirror = 0x140;

template <int CTRL>
__device__ __forceinline__ double dpp(double x) {
  uint64_t u = __builtin_bit_cast(uint64_t, x);
  int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xF, 0xF, false);
  int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ __forceinline__ double swz_xor16(double x) {
  // ds_swizzle bit-mask mode inside 32-lane halves: and 0x1F, or 0, xor 0x10
  uint64_t u = __builtin_bit_cast(uint64_t, x);
  int lo = __builtin_amdgcn_ds_swizzle((int)(uint32_t)u, 0x401F);
  int hi = __builtin_amdgcn_ds_swizzle((int)(uint32_t)(u >> 32), 0x401F);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ __forceinline__ double perm_xor32(double x) {
  int addr = (int)((__lane_id() ^ 32u) << 2);
  uint64_t u = __builtin_bit_cast(uint64_t, x);
  int lo = __builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)u);
  int hi = __builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)(u >> 32));
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Sum over an aligned group of G lanes (G a power of two <= 64). Each step
// adds the value of the partner lane l^s; IEEE addition is commutative, so
// every lane of the group ends with the same bits (deterministic).
template <int G>
__device__ __forceinline__ double group_sum(double x) {
  if constexpr (G >= 2) x += dpp<kQuadXor1>(x);
  if constexpr (G >= 4) x += dpp<kQuadXor2>(x);
  if constexpr (G >= 8) x += dpp<kRowHalfMirror>(x);
  if constexpr (G >= 16) x += dpp<kRowMirror>(x);
  if constexpr (G >= 32) x += swz_xor16(x);
  if constexpr (G >= 64) x += perm_xor32(x);
  return x;
}

// ------------------------------------------------------------ loads
// A pointer read from device memory (the batch's arrays of matrix and vector
// pointers) is generic to the compiler, and generic (flat) loads also count
// against the LDS wait counter, so every LDS wait would wait for the streams
// too. All such pointers address global memory: reading the element through
// a global-pointer view of the array lets the compiler emit global loads and
// stores for everything derived from it.
template <typename T>
__device__ __forceinline__ T* global_ptr_at(T* const* arr, int64_t i) {
  using GP = __attribute__((address_space(1))) T*;
  return (T*)reinterpret_cast<const GP*>(arr)[i];
}

// arr ? arr[i] : alt, chosen between global pointers (a select of generic
// pointers would be generic again).
template <typename T>
__device__ __forceinline__ T* global_ptr_or(T* const* arr, int64_t i, T* alt) {
  using GP = __attribute__((address_space(1))) T*;
  const GP g = arr ? reinterpret_cast<const GP*>(arr)[i] : (GP)alt;
  return (T*)g;
}

template <typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
  return __builtin_nontemporal_load(p);
}

template <typename T>
__device__ __forceinline__ double widen(T x) {
  return (double)x;
}

// Workgroup barrier that orders LDS accesses only. __syncthreads also waits
// for every outstanding global access of the wave (on CDNA one counter covers
// loads and stores), so a persistent workgroup would sit out the write latency
// of one tile's results before loading the next tile; this barrier lets those
// stores drain while the next loads are in flight.
__device__ __forceinline__ void lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ------------------------------------------------------------ XCD remap
// Workgroups are dispatched round-robin over the 8 XCDs (w -> XCD w % 8).
// Map them so that each XCD walks one contiguous range of tiles, which keeps
// the B entries a tile range gathers inside one L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t w, int64_t n) {
  int64_t x = w % kNumXCD, k = w / kNumXCD;
  int64_t q = n / kNumXCD, r = n % kNumXCD;
  return x * q + (x < r ? x : r) + k;
}

// ------------------------------------------------------------ LDS row block
// One workgroup multiplies rows [r0, r1) of a CRS matrix. The rows were cut
// so that (rows + nonzeros) of the block stay within kBlockBudget, hence all
// rows but the last lie inside the chunk [S, S + kBlockBudget) of the
// val/col_idx streams, S = row_ptr[r0]. Phase 1 streams that chunk with
// coalesced loads and stores the products in LDS; phase 2 reduces each row
// with a lane group whose width G adapts to the rows per block; phase 3
// streams the remainder of the last row (a row longer than the budget) with
// the whole workgroup.
// Strided partial sum over [j0, E) by the lanes of one workgroup: lane t takes
// j0 + t, j0 + t + kWG, ... in ascending order. Eight positions per lane are
// loaded before any is used, so a long row costs about E/(8 kWG) round trips.
template <typename VT, typename BT>
__device__ __forceinline__ double stream_row_part(const VT* __restrict__ val,
                                                  const int32_t* __restrict__ ci,
                                                  const BT* __restrict__ B, int32_t j0,
                                                  int32_t E) {
  constexpr int kU = 8;
  double part = 0.0;
  for (int32_t jb = j0 + (int32_t)threadIdx.x; jb < E; jb += kU * kWG) {
    VT v[kU];
    int32_t c[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int32_t j = jb + u * kWG;
      if (j < E) {
        v[u] = ld_stream(val + j);
        c[u] = ld_stream(ci + j);
      }
    }
    BT b[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u)
      if (jb + u * kWG < E) b[u] = B[c[u]];
#pragma unroll
    for (int u = 0; u < kU; ++u)
      if (jb + u * kWG < E) part = fma(widen(v[u]), widen(b[u]), part);
  }
  return part;
}

// The lane's index within the workgroup, hidden from loop-invariant code
// motion: in a workgroup that runs the row-block code tile after tile, the
// compiler otherwise computes every index and LDS address derived from it
// once before the loop and keeps them all live across it (82 instead of 56
// registers for the persistent batch kernel, 5 instead of 8 wavefronts per
// SIMD). Without a loop it costs one register move.
__device__ __forceinline__ int opaque_tid() {
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  return tid;
}

struct BlockLds {
  double prod[kBlockBudget];
  double wsum[kWG / 64];
  double last_part;
};

// Sum of L.prod[k] for k = k0, k0 + STEP, ... < z with four independent
// accumulators (LDS reads overlap instead of forming one latency chain),
// combined in a fixed order.
template <int STEP>
__device__ __forceinline__ double lds_strided_sum(const BlockLds& L, int32_t k0, int32_t z) {
  double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
  int32_t k = k0;
  for (; k + 3 * STEP < z; k += 4 * STEP) {
    p0 += L.prod[k];
    p1 += L.prod[k + STEP];
    p2 += L.prod[k + 2 * STEP];
    p3 += L.prod[k + 3 * STEP];
  }
  for (; k < z; k += STEP) p0 += L.prod[k];
  return (p0 + p1) + (p2 + p3);
}

// Phase 2 of the row block: rows [r0, r1) reduced from LDS. Groups of G
// lanes take one row each; every lane of a wavefront runs the same number of
// rounds, so the cross-lane steps see all lanes active. A row with more than
// 32 G products in the chunk would make its G lanes the wavefront's
// straggler (power-law rows next to hundreds of short ones); such rows are
// collected with a ballot and summed one after another by the whole
// wavefront. The tail row's in-chunk sum goes to *last_part.
// ACC: add to C instead of overwriting it (second pass of a split product).
template <int G, bool ACC>
__device__ __forceinline__ void block_rows(const BlockLds& L, const int32_t* __restrict__ rp,
                                           int32_t r0, int32_t r1, int32_t S, int32_t cend,
                                           bool tail, double* __restrict__ C,
                                           double* last_part) {
  const int tid = opaque_tid();
  const int wl = tid & 63;
  const int lane = tid & (G - 1);
  constexpr int ngroups = kWG / G;
  constexpr int32_t kLong = 32 * G;
  for (int32_t rw = r0 + (tid & ~63) / G; rw < r1; rw += ngroups) {
    const int32_t r = rw + wl / G;
    const bool valid = r < r1;
    int32_t a = 0, z = 0;
    if (valid) {
      a = rp[r] - S;
      const int32_t e = rp[r + 1];
      z = (e < cend ? e : cend) - S;
    }
    const bool lng = valid && z - a > kLong;
    const double part = (valid && !lng) ? lds_strided_sum<G>(L, a + lane, z) : 0.0;
    const double sum = group_sum<G>(part);
    if (valid && !lng && lane == 0) {
      if (tail && r == r1 - 1)
        *last_part = sum;
      else
        C[r] = ACC ? C[r] + sum : sum;
    }
    for (uint64_t m = __ballot(lng && lane == 0); m; m &= m - 1) {
      const int src = __ffsll((unsigned long long)m) - 1;
      const int32_t ra = __shfl(a, src), rz = __shfl(z, src), rr = __shfl(r, src);
      const double s = group_sum<64>(lds_strided_sum<64>(L, ra + wl, rz));
      if (wl == 0) {
        if (tail && rr == r1 - 1)
          *last_part = s;
        else
          C[rr] = ACC ? C[rr] + s : s;
      }
    }
  }
}

// S = row_ptr[r0] and E = row_ptr[r1] come from the block table, so the
// workgroup's first dependent round trip already yields the stream bounds.
// When cmin <= cmax and the range fits the staging array `stage` (stage_cap
// doubles of LDS that may overlap L), B[cmin..cmax] is first copied into it
// with coalesced loads; gathers of columns inside the range read LDS, the
// others B; the products then overwrite the array. The range is either the
// exact column span of the chunk [S, min(E, S + budget)) or, for blocks whose
// span is wider, a window around the block's rows.
// STAGE = false compiles the path out (callers without a range).
// DELTA: the chunk's columns may come from dptr as dbits-bit deltas from
// dbase (8 or 16; 0 reads ci).
template <typename VT, typename BT, bool ACC = false, bool STAGE = false, bool DELTA = false>
__device__ __forceinline__ void lds_block(BlockLds& L, const int32_t* __restrict__ rp,
                                          const int32_t* __restrict__ ci,
                                          const VT* __restrict__ val, const BT* __restrict__ B,
                                          double* __restrict__ C, int32_t r0, int32_t r1,
                                          int32_t S, int32_t E, int32_t cmin = 0,
                                          int32_t cmax = -1, double* stage = nullptr,
                                          int32_t stage_cap = 0, int32_t dbits = 0,
                                          int32_t dbase = 0,
                                          const uint8_t* __restrict__ dptr = nullptr) {
  const int tid = opaque_tid();
  const int32_t cend = (E - S > kBlockBudget) ? S + kBlockBudget : E;
  const int32_t nin = cend - S;
  const bool tail = E > cend;
  const int32_t span = cmax - cmin + 1;
  // float32 B is staged as float32 (stage_cap up to 2 kBlockBudget entries
  // in the same LDS); the batch's unrolled staging holds kBlockBudget
  constexpr bool kStageF = std::is_same<BT, float>::value && !DELTA;
  const bool staged = STAGE && stage && cmin <= cmax && span <= stage_cap &&
                      span <= (kStageF ? 2 : 1) * kBlockBudget;

  // phase 1: products of the chunk into LDS; all loads issued before use
  constexpr int kPer = kBlockBudget / kWG;
  VT v[kPer];
  int32_t c[kPer];
  if (DELTA && dbits != 0) {
    // raw deltas held as 32-bit words and the base added after every load
    // is issued
    uint32_t d[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int k = tid + u * kWG;
      d[u] = 0;
      if (k < nin) {
        v[u] = ld_stream(val + S + k);
        d[u] = dbits == 8 ? (uint32_t)ld_stream(dptr + k)
                          : (uint32_t)ld_stream(reinterpret_cast<const uint16_t*>(dptr) + k);
      }
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) asm volatile("" : "+v"(d[u]));
#pragma unroll
    for (int u = 0; u < kPer; ++u) c[u] = dbase + (int32_t)d[u];
  } else {
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int k = tid + u * kWG;
      if (k < nin) {
        v[u] = ld_stream(val + S + k);
        c[u] = ld_stream(ci + S + k);
      }
    }
  }
  double b[kPer];
  if constexpr (STAGE) {
    if (staged) {
      if constexpr (kStageF) {
        float* sf = reinterpret_cast<float*>(stage);
        for (int32_t k = tid; k < span; k += kWG) sf[k] = B[cmin + k];
      } else if constexpr (!DELTA) {
        for (int32_t k = tid; k < span; k += kWG) stage[k] = widen(B[cmin + k]);
      } else {
        // the batch's tiles: span <= stage_cap <= kPer * kWG, every load
        // issued before the first LDS write (the loop above waits for each
        // load before its write; unrolled, it costs the single-matrix kernel
        // more through registers than it saves)
        BT sv[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
          const int k = tid + u * kWG;
          sv[u] = (BT)0;
          if (k < span) sv[u] = B[cmin + k];
        }
        if constexpr (!std::is_same<BT, double>::value) {
#pragma unroll
          for (int u = 0; u < kPer; ++u) asm volatile("" : "+v"(sv[u]));
        }
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
          const int k = tid + u * kWG;
          if (k < span) stage[k] = widen(sv[u]);
        }
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int k = tid + u * kWG;
        if (k < nin) {
          // the LDS read is unconditional (clamped index) and its value is
          // pinned by an empty register barrier, so that the compiler cannot
          // fold it and the global load into one flat load from a selected
          // address (flat loads also wait on the LDS counter)
          const bool in = c[u] >= cmin && c[u] <= cmax;
          double xs;
          if constexpr (kStageF) {
            float xf = reinterpret_cast<const float*>(stage)[in ? c[u] - cmin : 0];
            asm volatile("" : "+v"(xf));
            xs = (double)xf;
          } else {
            xs = stage[in ? c[u] - cmin : 0];
            asm volatile("" : "+v"(xs));
          }
          double xg = 0.0;
          if (!in) xg = widen(B[c[u]]);
          b[u] = in ? xs : xg;
        }
      }
      __syncthreads();  // every staged entry read before the products overwrite them
    }
  }
  if (!staged) {
    // (the staging kernel keeps the plain gather for its unstaged blocks: the
    // deferred widening below made its float32 form 5% slower on the
    // permuted mesh through the schedule of the whole kernel)
    if constexpr (std::is_same<BT, double>::value || STAGE) {
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int k = tid + u * kWG;
        if (k < nin) b[u] = widen(B[c[u]]);
      }
    } else {
      // narrower B: gathered in its own type and widened after every gather
      // is issued (the pin keeps each widening out of its masked gather,
      // where it would wait for that load before the next is issued)
      BT xg[kPer];
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int k = tid + u * kWG;
        xg[u] = (BT)0;
        if (k < nin) xg[u] = B[c[u]];
      }
#pragma unroll
      for (int u = 0; u < kPer; ++u) asm volatile("" : "+v"(xg[u]));
#pragma unroll
      for (int u = 0; u < kPer; ++u) b[u] = widen(xg[u]);
    }
  }
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int k = tid + u * kWG;
    if (k < nin) L.prod[k] = widen(v[u]) * b[u];
  }
  __syncthreads();

  // phase 2: lane groups of width G reduce rows from LDS
  const int32_t nrows = r1 - r0;
  if (nrows * 64 <= kWG)
    block_rows<64, ACC>(L, rp, r0, r1, S, cend, tail, C, &L.last_part);
  else if (nrows * 32 <= kWG)
    block_rows<32, ACC>(L, rp, r0, r1, S, cend, tail, C, &L.last_part);
  else if (nrows * 16 <= kWG)
    block_rows<16, ACC>(L, rp, r0, r1, S, cend, tail, C, &L.last_part);
  else if (nrows * 8 <= kWG)
    block_rows<8, ACC>(L, rp, r0, r1, S, cend, tail, C, &L.last_part);
  else if (nrows * 4 <= kWG)
    block_rows<4, ACC>(L, rp, r0, r1, S, cend, tail, C, &L.last_part);
  else if (nrows * 2 <= kWG)
    block_rows<2, ACC>(L, rp, r0, r1, S, cend, tail, C, &L.last_part);
  else
    block_rows<1, ACC>(L, rp, r0, r1, S, cend, tail, C, &L.last_part);

  // phase 3: remainder of a long last row, streamed by the whole workgroup
  if (tail) {
    const double part = group_sum<64>(stream_row_part<VT, BT>(val, ci, B, cend, E));
    if ((tid & 63) == 0) L.wsum[tid >> 6] = part;
    __syncthreads();
    if (tid == 0) {
      const double s = L.last_part + ((L.wsum[0] + L.wsum[1]) + (L.wsum[2] + L.wsum[3]));
      C[r1 - 1] = ACC ? C[r1 - 1] + s : s;
    }
  }
}

}  // namespace dev
}  // namespace spmv
