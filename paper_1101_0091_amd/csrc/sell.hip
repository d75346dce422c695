// Variant V6: the CRS product of Sect. 1.2 computed from a chunked copy of
// the matrix. Rows are cut into chunks of 64 consecutive rows (one chunk per
// wavefront, no reordering); chunk k has the width w of its longest row and
// 64 w slots; slot (j, lane) holds the j-th nonzero of row 64 k + lane.
// Shorter rows are padded with col = -1, val = 0. This is a sliced ELLPACK
// layout with slice height 64 (the SELL-C-sigma family with C = 64,
// sigma = 1). Inside a chunk the slots are stored in lane-interleaved groups
// of G (G = 2 for float64 values, 4 for float32): with Q = floor(w / G), slot
// j < G Q of lane l sits at G (64 floor(j / G) + l) + j mod G, and each of the
// w - G Q tail slots t at 64 G Q + 64 t + l. A lane then loads G slots of its
// row per instruction (16-byte val loads), every load is one contiguous
// access per wavefront, no LDS or barrier is needed, and each row is summed by
// one lane.
//
// Column deltas: within a chunk, slot j of the 64 rows often points at 64
// nearby columns (a band, a diagonal, a stencil). Each slot j then gets a
// 4-byte base (the smallest of its columns) and every entry a delta from it
// of 8 bits when every slot of the chunk spans at most 0xFE columns, else of
// 16 bits when every slot spans at most 0xFFFE (the all-ones delta marks
// padding): 9 or 10 instead of 12 bytes per float64 slot (5 or 6 instead of
// 8 for float32). Other chunks read the 4-byte columns. The column, and hence
// every product and the order of the sum, is the same either way.
//
// The copy is built on the device at plan creation in four passes: chunk
// widths, an exclusive scan of the widths, the fill, and the deltas. Its
// capacity is reserved in the plan workspace; a pattern whose padded size
// does not fit is reported back and V6 is then unavailable for that plan.
#include <type_traits>

#include "common.hpp"
#include "device.hpp"

namespace spmv {
namespace {

constexpr int kChunk = 64;  // rows per chunk = lanes per wavefront
constexpr int kSellUP = 8;  // slot pairs of one row loaded before the first is used

typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef int32_t i32x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// Delta bits of a chunk (its flag): 0 = 4-byte columns, 8 or 16.
template <int DB> constexpr uint32_t kPad = (1u << DB) - 1;  // delta of a padding slot

// Slots per lane-interleaved group for a value type (see the layout above).
template <typename VT> constexpr int kGroup = sizeof(VT) == 8 ? 2 : 4;

// Offset of slot j of `lane` inside a chunk of width w with groups of G.
template <int G>
__device__ __forceinline__ int64_t slot_offset(int64_t j, int lane, int64_t w) {
  const int64_t Q = w / G;
  return j < G * Q ? G * ((j / G) * kChunk + lane) + j % G
                   : G * Q * kChunk + (j - G * Q) * kChunk + lane;
}

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
  const int64_t len = e - s, w = b - a;
  int32_t* dc = sci + a * kChunk;
  VT* dv = sval + a * kChunk;
  constexpr int kU = 8;  // entries of the row loaded before any is stored
  for (int64_t j0 = 0; j0 < w; j0 += kU) {
    int32_t c[kU];
    VT v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t j = j0 + u;
      c[u] = j < len ? ci[s + j] : -1;
      v[u] = j < len ? val[s + j] : (VT)0;
    }
    // a whole group of G slots of the row goes out as one vector store of
    // columns and one of values (the group is G-aligned: kU and j0 are
    // multiples of G); the tail slots one at a time
    constexpr int G = kGroup<VT>;
    const int64_t GQ = G * (w / G);
#pragma unroll
    for (int u = 0; u < kU; u += G) {
      const int64_t j = j0 + u;
      if (j + G <= GQ) {
        const int64_t o = slot_offset<G>(j, lane, w);
        if constexpr (G == 2) {
          *reinterpret_cast<i32x2*>(dc + o) = i32x2{c[u], c[u + 1]};
          *reinterpret_cast<f64x2*>(dv + o) = f64x2{(double)v[u], (double)v[u + 1]};
        } else {
          *reinterpret_cast<i32x4*>(dc + o) = i32x4{c[u], c[u + 1], c[u + 2], c[u + 3]};
          *reinterpret_cast<f32x4*>(dv + o) = f32x4{(float)v[u], (float)v[u + 1],
                                                    (float)v[u + 2], (float)v[u + 3]};
        }
      } else {
#pragma unroll
        for (int t = 0; t < G; ++t) {
          if (j + t < w) {
            const int64_t o = slot_offset<G>(j + t, lane, w);
            dc[o] = c[u + t];
            dv[o] = v[u + t];
          }
        }
      }
    }
  }
}

// Column deltas of the filled copy (one wavefront per chunk): for each slot j
// the smallest column over the chunk's rows becomes base[off + j]; the largest
// span over the slots picks the chunk's delta width (flag[k] = 8, 16, or 0 when
// some slot spans more than 0xFFFE columns), and every entry stores its column
// minus the slot's base in that width (all ones for padding). 8-bit deltas fill
// the first half of the chunk's 16-bit delta region, at the same slot
// positions. Nothing is written unless the copy fit its reserve.
// One step of the wavefront min/max: combine with the partner lane that
// STEP (a DPP pattern inside rows, then the 16- and 32-lane swaps) names.
template <int STEP>
__device__ __forceinline__ int32_t partner(int32_t x) {
  if constexpr (STEP == 0) return __builtin_amdgcn_update_dpp(0, x, dev::kQuadXor1, 0xF, 0xF, false);
  if constexpr (STEP == 1) return __builtin_amdgcn_update_dpp(0, x, dev::kQuadXor2, 0xF, 0xF, false);
  if constexpr (STEP == 2)
    return __builtin_amdgcn_update_dpp(0, x, dev::kRowHalfMirror, 0xF, 0xF, false);
  if constexpr (STEP == 3) return __builtin_amdgcn_update_dpp(0, x, dev::kRowMirror, 0xF, 0xF, false);
  if constexpr (STEP == 4) return __builtin_amdgcn_ds_swizzle(x, 0x401F);  // lane ^ 16
  return __builtin_amdgcn_ds_bpermute((int)((__lane_id() ^ 32u) << 2), x);
}

template <int STEP>
__device__ __forceinline__ void min_max_step(int32_t& mn, int32_t& mx) {
  const int32_t x = partner<STEP>(mn), y = partner<STEP>(mx);
  mn = x < mn ? x : mn;
  mx = y > mx ? y : mx;
}

// Smallest and largest real column of a slot over the wavefront's 64 lanes
// (every lane of the wavefront is active here).
__device__ __forceinline__ void slot_min_max(int32_t c, int32_t& mn, int32_t& mx) {
  mn = c >= 0 ? c : INT32_MAX;  // padding: c = -1
  mx = c;
  min_max_step<0>(mn, mx);
  min_max_step<1>(mn, mx);
  min_max_step<2>(mn, mx);
  min_max_step<3>(mn, mx);
  min_max_step<4>(mn, mx);
  min_max_step<5>(mn, mx);
}

template <int G>
__global__ __launch_bounds__(kWG) void k_sell_narrow(int64_t nch, const int32_t* __restrict__ off,
                                                     int64_t cap64,
                                                     const int32_t* __restrict__ sci,
                                                     int32_t* __restrict__ sbase,
                                                     uint16_t* __restrict__ sdl,
                                                     int32_t* __restrict__ flag) {
  const int64_t total = off[nch];
  const int64_t chunk = ((int64_t)blockIdx.x * kWG + threadIdx.x) / kChunk;
  if (chunk >= nch || total < 0 || total > cap64) return;
  const int64_t a = off[chunk], b = off[chunk + 1];
  if (a < 0 || b < a || b > total) return;
  const int lane = threadIdx.x % kChunk;
  const int64_t w = b - a;
  int64_t span = 0;  // largest over the slots; uniform over the wavefront
  constexpr int kU = 8;  // slots loaded before any is reduced
  for (int64_t j0 = 0; j0 < w; j0 += kU) {
    int32_t c[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u)
      c[u] = j0 + u < w ? sci[a * kChunk + slot_offset<G>(j0 + u, lane, w)] : -1;
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if (j0 + u < w) {  // uniform
        int32_t mn, mx;
        slot_min_max(c[u], mn, mx);
        // slot j < w of the chunk's longest row is a real entry, so mn <= mx
        span = (int64_t)mx - mn > span ? (int64_t)mx - mn : span;
        if (lane == 0) sbase[a + j0 + u] = mn;
      }
    }
  }
  const int db = span < (int64_t)kPad<8> ? 8 : span < (int64_t)kPad<16> ? 16 : 0;
  if (db != 0) {
    uint8_t* d8 = reinterpret_cast<uint8_t*>(sdl + a * kChunk);
    for (int64_t j = 0; j < w; ++j) {
      const int64_t o = slot_offset<G>(j, lane, w);
      const int32_t c = sci[a * kChunk + o];
      int32_t mn, mx;
      slot_min_max(c, mn, mx);
      const uint32_t d = c >= 0 ? (uint32_t)(c - mn) : 0xFFFFFFFFu;
      if (db == 8)
        d8[o] = (uint8_t)d;
      else
        sdl[a * kChunk + o] = (uint16_t)d;
    }
  }
  if (lane == 0) flag[chunk] = db;
}

// Column of a slot read through its delta (-1 for padding).
template <int DB>
__device__ __forceinline__ int32_t delta_col(uint32_t d, int32_t base) {
  return d != kPad<DB> ? base + (int32_t)d : -1;
}

// Field i of a lane's delta word (G deltas of DB bits, the first in the low bits).
template <int DB, typename W>
__device__ __forceinline__ uint32_t delta_field(W d, int i) {
  if constexpr (std::is_same<W, u32x2>::value)  // four 16-bit deltas
    return ((i < 2 ? d.x : d.y) >> (DB * (i & 1))) & kPad<DB>;
  else
    return ((uint32_t)d >> (DB * i)) & kPad<DB>;
}

// C = A*B from the chunked copy with float64 values: lane l of the wavefront
// of chunk k owns row 64 k + l and sums its slots in order, kSellUP pairs per
// round, the odd last slot after the rounds. The width is uniform over the
// wavefront, so the loop and its masked last round are uniform branches.
// DB > 0 reads the columns as base + DB-bit delta (a lane's pair of deltas
// per 4- or 2-byte load, the bases as wavefront-uniform loads).
template <int DB>
__device__ __forceinline__ double sell_pairs_row(int64_t a, int32_t w, int lane,
                                                 const int32_t* __restrict__ sci,
                                                 const uint16_t* __restrict__ sdl,
                                                 const int32_t* __restrict__ sbase,
                                                 const double* __restrict__ sval,
                                                 const double* __restrict__ B) {
  using VT = double;
  using V2 = f64x2;
  const int32_t P = w >> 1;
  const V2* vp = reinterpret_cast<const V2*>(sval + a * kChunk) + lane;
  const i32x2* cp = reinterpret_cast<const i32x2*>(sci + a * kChunk) + lane;
  using DW = typename std::conditional<DB == 16, uint32_t, uint16_t>::type;  // 2 deltas
  using DT = typename std::conditional<DB == 16, uint16_t, uint8_t>::type;   // 1 delta
  const DW* dp = reinterpret_cast<const DW*>(sdl + a * kChunk) + lane;
  const int32_t* bp = sbase + a;
  double acc = 0.0;
  // padded and masked slots contribute fma(0, 0, acc) = acc exactly: acc
  // starts at +0, and a round-to-nearest sum with a +0 operand is never -0,
  // so acc is never -0
  for (int32_t p = 0; p < P; p += kSellUP) {
    V2 v[kSellUP];
    i32x2 c[kSellUP];
    double x0[kSellUP], x1[kSellUP];
    if constexpr (DB > 0) {
      // every load of the round is issued before any delta is decoded (each
      // word widened to 32 bits: two 8-bit pairs packed into one register
      // made every load wait for its predecessor)
      uint32_t d[kSellUP];
      i32x2 b[kSellUP];
#pragma unroll
      for (int u = 0; u < kSellUP; ++u) {
        if (p + u < P) {
          v[u] = dev::ld_stream(vp + (int64_t)(p + u) * kChunk);
          d[u] = dev::ld_stream(dp + (int64_t)(p + u) * kChunk);
          // two 4-byte loads: a chunk's bases start at an offset that can
          // be odd, so the pair is only 4-byte aligned
          b[u] = i32x2{bp[2 * (p + u)], bp[2 * (p + u) + 1]};
        } else {
          v[u] = V2{(VT)0, (VT)0};
          d[u] = 0xFFFFFFFFu;
          b[u] = i32x2{0, 0};
        }
      }
      if constexpr (DB == 8) {
#pragma unroll
        for (int u = 0; u < kSellUP; ++u) asm volatile("" : "+v"(d[u]));
      }
#pragma unroll
      for (int u = 0; u < kSellUP; ++u)
        c[u] = i32x2{delta_col<DB>(delta_field<DB>(d[u], 0), b[u].x),
                     delta_col<DB>(delta_field<DB>(d[u], 1), b[u].y)};
    } else {
#pragma unroll
      for (int u = 0; u < kSellUP; ++u) {
        if (p + u < P) {
          v[u] = dev::ld_stream(vp + (int64_t)(p + u) * kChunk);
          c[u] = dev::ld_stream(cp + (int64_t)(p + u) * kChunk);
        } else {
          v[u] = V2{(VT)0, (VT)0};
          c[u] = i32x2{-1, -1};
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kSellUP; ++u) {
      x0[u] = c[u].x >= 0 ? (double)B[c[u].x] : 0.0;
      x1[u] = c[u].y >= 0 ? (double)B[c[u].y] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kSellUP; ++u) {
      acc = fma(dev::widen(v[u].x), x0[u], acc);
      acc = fma(dev::widen(v[u].y), x1[u], acc);
    }
  }
  if (w & 1) {
    const int64_t o = a * kChunk + 2 * (int64_t)P * kChunk + lane;
    int32_t c;
    if constexpr (DB > 0)
      c = delta_col<DB>(dev::ld_stream(reinterpret_cast<const DT*>(sdl + a * kChunk) +
                                       2 * (int64_t)P * kChunk + lane),
                        bp[2 * P]);
    else
      c = dev::ld_stream(sci + o);
    if (c >= 0) acc = fma(dev::widen(dev::ld_stream(sval + o)), (double)B[c], acc);
  }
  return acc;
}

// Wavefront-uniform chunk index (one chunk per wavefront).
__device__ __forceinline__ int64_t chunk_of_wave() {
  return __builtin_amdgcn_readfirstlane((int32_t)(((int64_t)blockIdx.x * kWG + threadIdx.x) /
                                                  kChunk));
}

// flag is null when the plan keeps 4-byte columns only.
__global__ __launch_bounds__(kWG) void k_sell_pairs(int64_t nch, int64_t n,
                                                    const int32_t* __restrict__ off,
                                                    const int32_t* __restrict__ sci,
                                                    const int32_t* __restrict__ flag,
                                                    const int32_t* __restrict__ sbase,
                                                    const uint16_t* __restrict__ sdl,
                                                    const double* __restrict__ sval,
                                                    const double* __restrict__ B,
                                                    double* __restrict__ C) {
  const int64_t chunk = chunk_of_wave();
  if (chunk >= nch) return;
  const int lane = threadIdx.x % kChunk;
  const int64_t a = off[chunk];
  const int32_t w = (int32_t)(off[chunk + 1] - a);
  const int db = flag ? flag[chunk] : 0;
  const double acc = db == 8    ? sell_pairs_row<8>(a, w, lane, sci, sdl, sbase, sval, B)
                     : db == 16 ? sell_pairs_row<16>(a, w, lane, sci, sdl, sbase, sval, B)
                                : sell_pairs_row<0>(a, w, lane, sci, sdl, sbase, sval, B);
  const int64_t row = chunk * kChunk + lane;
  // nontemporal: C is written once and not read again in this launch
  // (1.6% faster on a 6M-row product; the float32 kernel lost 0.6% with it)
  if (row < n) __builtin_nontemporal_store(acc, C + row);
}

// float32 values: groups of four slots, kSellUQ groups per round; the up to
// three tail slots are loaded before the first round and summed in it.
// Three groups (62 VGPRs, 8 waves per SIMD) put a row of up to 15 entries in
// one round: 4.9% faster than two groups on a 6M-row matrix of width 15,
// four groups (66 VGPRs, 7 waves) 4%.
constexpr int kSellUQ = 3;

// DB > 0 reads the columns as base + DB-bit delta (a lane's four deltas per
// 8- or 4-byte load).
template <int DB, typename BT>
__device__ __forceinline__ double sell_quads_row(int64_t a, int32_t w, int lane,
                                                 const int32_t* __restrict__ sci,
                                                 const uint16_t* __restrict__ sdl,
                                                 const int32_t* __restrict__ sbase,
                                                 const float* __restrict__ sval,
                                                 const BT* __restrict__ B) {
  const int32_t Q = w >> 2, T = w & 3;
  const f32x4* vp = reinterpret_cast<const f32x4*>(sval + a * kChunk) + lane;
  const i32x4* cp = reinterpret_cast<const i32x4*>(sci + a * kChunk) + lane;
  using DW = typename std::conditional<DB == 16, u32x2, uint32_t>::type;   // 4 deltas
  using DT = typename std::conditional<DB == 16, uint16_t, uint8_t>::type;  // 1 delta
  const DW* dp = reinterpret_cast<const DW*>(sdl + a * kChunk) + lane;
  const int32_t* bp = sbase + a;
  // tail slots: raw column words now, decoded at their gather in the first
  // round, so no tail load is waited for before the round's loads are issued
  float tv[3];
  uint32_t tr[3];
  int32_t tb[3];
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    tb[t] = 0;
    if (t < T) {
      const int64_t o = a * kChunk + 4 * (int64_t)Q * kChunk + t * kChunk + lane;
      tv[t] = dev::ld_stream(sval + o);
      if constexpr (DB > 0) {
        tr[t] = dev::ld_stream(reinterpret_cast<const DT*>(sdl + a * kChunk) +
                               4 * (int64_t)Q * kChunk + t * kChunk + lane);
        tb[t] = bp[4 * Q + t];
      } else {
        tr[t] = (uint32_t)dev::ld_stream(sci + o);
      }
    } else {
      tv[t] = 0.0f;
      tr[t] = DB > 0 ? kPad<DB> : 0xFFFFFFFFu;
    }
  }
  double acc = 0.0;
  // padded and masked slots contribute fma(0, 0, acc) = acc exactly
  int32_t q = 0;
  bool first = true;
  do {
    f32x4 v[kSellUQ];
    i32x4 c[kSellUQ];
    if constexpr (DB > 0) {
      // every load of the round is issued before any delta is decoded
      DW d[kSellUQ];
      i32x4 b[kSellUQ];
#pragma unroll
      for (int u = 0; u < kSellUQ; ++u) {
        if (q + u < Q) {
          v[u] = dev::ld_stream(vp + (int64_t)(q + u) * kChunk);
          d[u] = dev::ld_stream(dp + (int64_t)(q + u) * kChunk);
          // four 4-byte loads: a chunk's bases are only 4-byte aligned
          b[u] = i32x4{bp[4 * (q + u)], bp[4 * (q + u) + 1], bp[4 * (q + u) + 2],
                       bp[4 * (q + u) + 3]};
        } else {
          v[u] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
          if constexpr (DB == 16)
            d[u] = u32x2{0xFFFFFFFFu, 0xFFFFFFFFu};
          else
            d[u] = 0xFFFFFFFFu;
          b[u] = i32x4{0, 0, 0, 0};
        }
      }
#pragma unroll
      for (int u = 0; u < kSellUQ; ++u)
        c[u] = i32x4{delta_col<DB>(delta_field<DB>(d[u], 0), b[u].x),
                     delta_col<DB>(delta_field<DB>(d[u], 1), b[u].y),
                     delta_col<DB>(delta_field<DB>(d[u], 2), b[u].z),
                     delta_col<DB>(delta_field<DB>(d[u], 3), b[u].w)};
    } else {
#pragma unroll
      for (int u = 0; u < kSellUQ; ++u) {
        if (q + u < Q) {
          v[u] = dev::ld_stream(vp + (int64_t)(q + u) * kChunk);
          c[u] = dev::ld_stream(cp + (int64_t)(q + u) * kChunk);
        } else {
          v[u] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
          c[u] = i32x4{-1, -1, -1, -1};
        }
      }
    }
    // gathered in B's own type and widened at the multiply, after every
    // gather of the round is issued (the empty asm keeps the compiler from
    // moving the widening into the masked gather, where each gather then
    // waited for its own load)
    BT tx[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      int32_t tc;
      if constexpr (DB > 0)
        tc = delta_col<DB>(tr[t], tb[t]);
      else
        tc = (int32_t)tr[t];
      tx[t] = (first && tc >= 0) ? B[tc] : (BT)0;
    }
    BT x[kSellUQ][4];
#pragma unroll
    for (int u = 0; u < kSellUQ; ++u) {
      x[u][0] = c[u].x >= 0 ? B[c[u].x] : (BT)0;
      x[u][1] = c[u].y >= 0 ? B[c[u].y] : (BT)0;
      x[u][2] = c[u].z >= 0 ? B[c[u].z] : (BT)0;
      x[u][3] = c[u].w >= 0 ? B[c[u].w] : (BT)0;
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) asm volatile("" : "+v"(tx[t]), "+v"(tv[t]));
#pragma unroll
    for (int u = 0; u < kSellUQ; ++u)
#pragma unroll
      for (int k = 0; k < 4; ++k) asm volatile("" : "+v"(x[u][k]));
#pragma unroll
    for (int u = 0; u < kSellUQ; ++u) {
      acc = fma((double)v[u].x, (double)x[u][0], acc);
      acc = fma((double)v[u].y, (double)x[u][1], acc);
      acc = fma((double)v[u].z, (double)x[u][2], acc);
      acc = fma((double)v[u].w, (double)x[u][3], acc);
    }
    if (first) {
#pragma unroll
      for (int t = 0; t < 3; ++t) acc = fma((double)tv[t], (double)tx[t], acc);
    }
    first = false;
    q += kSellUQ;
  } while (q < Q);
  return acc;
}

template <typename BT>
__global__ __launch_bounds__(kWG) void k_sell_quads(int64_t nch, int64_t n,
                                                    const int32_t* __restrict__ off,
                                                    const int32_t* __restrict__ sci,
                                                    const int32_t* __restrict__ flag,
                                                    const int32_t* __restrict__ sbase,
                                                    const uint16_t* __restrict__ sdl,
                                                    const float* __restrict__ sval,
                                                    const BT* __restrict__ B,
                                                    double* __restrict__ C) {
  const int64_t chunk = chunk_of_wave();
  if (chunk >= nch) return;
  const int lane = threadIdx.x % kChunk;
  const int64_t a = off[chunk];
  const int32_t w = (int32_t)(off[chunk + 1] - a);
  const int db = flag ? flag[chunk] : 0;
  const double acc = db == 8    ? sell_quads_row<8, BT>(a, w, lane, sci, sdl, sbase, sval, B)
                     : db == 16 ? sell_quads_row<16, BT>(a, w, lane, sci, sdl, sbase, sval, B)
                                : sell_quads_row<0, BT>(a, w, lane, sci, sdl, sbase, sval, B);
  const int64_t row = chunk * kChunk + lane;
  if (row < n) C[row] = acc;
}

// Multi-RHS form from the chunked copy: C[i, c0 + t] = sum_j val(j) B[col(j), c0 + t]
// for t < kc = min(KB, k - c0). Lane l of chunk k owns row 64 k + l and keeps
// KB accumulators; every slot gathers the row segment B[col, c0 .. c0 + KB).
// VEC = 1: vector loads of a full segment (16-byte for float64 pairs and
// float32 quads, 8-byte for float32 pairs); VEC = 2: a partial segment
// (kc < KB) in pairs with its odd last column alone; VEC = 0: scalar loads.
// Both vector forms need rows and segments aligned to the load. Slots per
// round shrink with KB to bound the registers in flight (16 up to KB = 4, 8
// for KB = 8, so a row of up to 16 or 8 entries is one round of loads).
// DB > 0 reads the columns through the chunk's DB-bit deltas.
template <typename VT, typename BT, int KB, int VEC, int DB>
__device__ __forceinline__ void sell_spmm_rows(int64_t a, int32_t w, int lane, int32_t kc,
                                               int32_t c0, const int32_t* __restrict__ sci,
                                               const uint16_t* __restrict__ sdl,
                                               const int32_t* __restrict__ sbase,
                                               const VT* __restrict__ sval,
                                               const BT* __restrict__ B, int64_t ldb,
                                               double* acc) {
  constexpr int G = kGroup<VT>;
  constexpr int U = KB <= 4 ? 16 : 8;
  using DT = typename std::conditional<DB == 16, uint16_t, uint8_t>::type;
  const DT* dp = reinterpret_cast<const DT*>(sdl + a * kChunk);
  const int32_t* bp = sbase + a;
  // narrower value or B types are loaded and gathered in their own type and
  // widened only after every load of the round is issued (empty asm pins
  // keep the compiler from moving a widening next to its load, which then
  // waits for that load before the next one is issued)
  constexpr bool kPinV = !std::is_same<VT, double>::value;
  constexpr bool kPinB = !std::is_same<BT, double>::value;
  // a lane's G slots of a full group are contiguous (values, columns and
  // deltas): one vector load each, as in the single-vector kernels
  // (Hamiltonian-like matrix, 6M rows, against one load per slot: float64
  // k = 2/3 241/353 -> 213/308 us, float32 storage k = 2/3/4 209/302/280 ->
  // 126/230/196 us)
  using VG = typename std::conditional<G == 2, f64x2, f32x4>::type;
  using CG = typename std::conditional<G == 2, i32x2, i32x4>::type;
  using DG = typename std::conditional<
      G == 2, typename std::conditional<DB == 16, uint32_t, uint16_t>::type,
      typename std::conditional<DB == 16, u32x2, uint32_t>::type>::type;
  const int32_t GQ = w - w % G;
  for (int32_t j = 0; j < w; j += U) {
    VT vr[U];
    int32_t c[U];
    if constexpr (DB > 0) {
      // deltas held as loaded and decoded after every load is issued
      DG dg[U / G];
      uint32_t d[U];
      int32_t b[U];
#pragma unroll
      for (int u = 0; u < U; u += G) {
        const int32_t j0 = j + u;
        if (j0 + G <= GQ) {
          const int64_t o = G * ((int64_t)(j0 / G) * kChunk + lane);
          const VG q = dev::ld_stream(reinterpret_cast<const VG*>(sval + a * kChunk + o));
          dg[u / G] = dev::ld_stream(reinterpret_cast<const DG*>(dp + o));
#pragma unroll
          for (int t = 0; t < G; ++t) {
            vr[u + t] = q[t];
            d[u + t] = 0xFFFFFFFFu;  // taken from dg below
            b[u + t] = bp[j0 + t];
          }
        } else {
          dg[u / G] = DG{};
#pragma unroll
          for (int t = 0; t < G; ++t) {
            if (j0 + t < w) {
              const int64_t o = slot_offset<G>(j0 + t, lane, w);
              vr[u + t] = dev::ld_stream(sval + a * kChunk + o);
              d[u + t] = dev::ld_stream(dp + o);
              b[u + t] = bp[j0 + t];
            } else {
              vr[u + t] = (VT)0;
              d[u + t] = kPad<DB>;
              b[u + t] = 0;
            }
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U / G; ++u) asm volatile("" : "+v"(dg[u]));
#pragma unroll
      for (int u = 0; u < U; ++u) asm volatile("" : "+v"(d[u]));
#pragma unroll
      for (int u = 0; u < U; u += G) {
        const bool full = j + u + G <= GQ;
#pragma unroll
        for (int t = 0; t < G; ++t)
          c[u + t] = delta_col<DB>(full ? delta_field<DB>(dg[u / G], t) : d[u + t], b[u + t]);
      }
    } else {
#pragma unroll
      for (int u = 0; u < U; u += G) {
        const int32_t j0 = j + u;
        if (j0 + G <= GQ) {
          const int64_t o = a * kChunk + G * ((int64_t)(j0 / G) * kChunk + lane);
          const VG q = dev::ld_stream(reinterpret_cast<const VG*>(sval + o));
          const CG cq = dev::ld_stream(reinterpret_cast<const CG*>(sci + o));
#pragma unroll
          for (int t = 0; t < G; ++t) {
            vr[u + t] = q[t];
            c[u + t] = cq[t];
          }
        } else {
#pragma unroll
          for (int t = 0; t < G; ++t) {
            if (j0 + t < w) {
              const int64_t o = a * kChunk + slot_offset<G>(j0 + t, lane, w);
              vr[u + t] = dev::ld_stream(sval + o);
              c[u + t] = dev::ld_stream(sci + o);
            } else {
              vr[u + t] = (VT)0;
              c[u + t] = -1;
            }
          }
        }
      }
    }
    if constexpr (kPinB) {
      BT xb[U][KB];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const BT* bq = B + (int64_t)(c[u] >= 0 ? c[u] : 0) * ldb + c0;
        if constexpr (VEC == 1 && KB >= 2) {
          // one 8-byte (KB = 2) or 16-byte load per 4 columns of the segment
          if (c[u] >= 0) {
            if constexpr (KB == 2) {
              const f32x2 q = *reinterpret_cast<const f32x2*>(bq);
              xb[u][0] = q.x;
              xb[u][1] = q.y;
            } else {
#pragma unroll
              for (int t = 0; t < KB; t += 4) {
                const f32x4 q = *reinterpret_cast<const f32x4*>(bq + t);
                xb[u][t] = q.x;
                xb[u][t + 1] = q.y;
                xb[u][t + 2] = q.z;
                xb[u][t + 3] = q.w;
              }
            }
          } else {
#pragma unroll
            for (int t = 0; t < KB; ++t) xb[u][t] = (BT)0;
          }
        } else if constexpr (VEC == 2) {
          // partial block: 8-byte pairs of the kc columns, the odd last one alone
#pragma unroll
          for (int t = 0; t < KB; t += 2) {
            if (c[u] >= 0 && t + 1 < kc) {
              const f32x2 q = *reinterpret_cast<const f32x2*>(bq + t);
              xb[u][t] = q.x;
              xb[u][t + 1] = q.y;
            } else {
              xb[u][t] = (c[u] >= 0 && t < kc) ? bq[t] : (BT)0;
              xb[u][t + 1] = (BT)0;
            }
          }
        } else {
#pragma unroll
          for (int t = 0; t < KB; ++t) xb[u][t] = (c[u] >= 0 && t < kc) ? bq[t] : (BT)0;
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if constexpr (kPinV) asm volatile("" : "+v"(vr[u]));
#pragma unroll
        for (int t = 0; t < KB; ++t) asm volatile("" : "+v"(xb[u][t]));
      }
      // masked slots add fma(0, 0, acc) = acc exactly (acc is never -0)
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int t = 0; t < KB; ++t)
          acc[t] = fma(dev::widen(vr[u]), (double)xb[u][t], acc[t]);
      continue;
    }
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = dev::widen(vr[u]);
    double x[U][KB];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const BT* bq = B + (int64_t)(c[u] >= 0 ? c[u] : 0) * ldb + c0;
      if constexpr (VEC == 1 && KB >= 2 && std::is_same<BT, double>::value) {
        if (c[u] >= 0) {
#pragma unroll
          for (int t = 0; t < KB; t += 2) {
            const f64x2 q = *reinterpret_cast<const f64x2*>(bq + t);
            x[u][t] = q.x;
            x[u][t + 1] = q.y;
          }
        } else {
#pragma unroll
          for (int t = 0; t < KB; ++t) x[u][t] = 0.0;
        }
      } else if constexpr (VEC == 2) {
        // partial block: 16-byte pairs of the kc columns, the odd last one alone
#pragma unroll
        for (int t = 0; t < KB; t += 2) {
          if (c[u] >= 0 && t + 1 < kc) {
            const f64x2 q = *reinterpret_cast<const f64x2*>(bq + t);
            x[u][t] = q.x;
            x[u][t + 1] = q.y;
          } else {
            x[u][t] = (c[u] >= 0 && t < kc) ? (double)bq[t] : 0.0;
            x[u][t + 1] = 0.0;
          }
        }
      } else {
#pragma unroll
        for (int t = 0; t < KB; ++t) x[u][t] = (c[u] >= 0 && t < kc) ? (double)bq[t] : 0.0;
      }
    }
    // masked slots add fma(0, 0, acc) = acc exactly (acc is never -0)
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int t = 0; t < KB; ++t) acc[t] = fma(v[u], x[u][t], acc[t]);
  }
}

// flag is null when the plan keeps 4-byte columns only.
template <typename VT, typename BT, int KB, int VEC>
__global__ __launch_bounds__(kWG) void k_sell_spmm(int64_t nch, int64_t n,
                                                   const int32_t* __restrict__ off,
                                                   const int32_t* __restrict__ sci,
                                                   const int32_t* __restrict__ flag,
                                                   const int32_t* __restrict__ sbase,
                                                   const uint16_t* __restrict__ sdl,
                                                   const VT* __restrict__ sval,
                                                   const BT* __restrict__ B, int64_t ldb,
                                                   double* __restrict__ C, int64_t ldc,
                                                   int32_t k, int32_t c0) {
  const int64_t chunk = chunk_of_wave();
  if (chunk >= nch) return;
  const int lane = threadIdx.x % kChunk;
  const int64_t a = off[chunk];
  const int32_t w = (int32_t)(off[chunk + 1] - a);
  const int32_t kc = k - c0 < KB ? k - c0 : KB;
  double acc[KB];
#pragma unroll
  for (int t = 0; t < KB; ++t) acc[t] = 0.0;
  const int db = flag ? flag[chunk] : 0;
  if (db == 8)
    sell_spmm_rows<VT, BT, KB, VEC, 8>(a, w, lane, kc, c0, sci, sdl, sbase, sval, B, ldb, acc);
  else if (db == 16)
    sell_spmm_rows<VT, BT, KB, VEC, 16>(a, w, lane, kc, c0, sci, sdl, sbase, sval, B, ldb, acc);
  else
    sell_spmm_rows<VT, BT, KB, VEC, 0>(a, w, lane, kc, c0, sci, sdl, sbase, sval, B, ldb, acc);
  const int64_t row = chunk * kChunk + lane;
  if (row < n) {
    double* out = C + row * ldc + c0;
#pragma unroll
    for (int t = 0; t < KB; ++t)
      if (t < kc) out[t] = acc[t];
  }
}

// Multi-RHS from the chunked copy with LPR lanes per row: lane g of a row
// owns the VPL CPL columns c0 + g VPL CPL .. (VPL 16-byte vectors of B of
// CPL = 2 float64 or 4 float32 each), so the LPR lanes of a row read its B
// row segment as one contiguous piece, and the 64 / LPR rows of a
// wavefront (consecutive rows of one chunk) read consecutive segments where
// their columns are consecutive. Wavefront w takes part w % LPR of chunk
// w / LPR. A row's entries are taken kSpmmLU per round, all their loads
// issued before the first is used; the lanes of a row load the same value
// and column (one memory access). Needs B, C, ldb and ldc aligned to the
// vector (checked by the caller) and c0 + LPR VPL CPL <= k. With remap set,
// each XCD takes a contiguous range of chunks (instead of every eighth
// workgroup), so that B rows shared by rows a few thousand apart (offset
// diagonals) can meet again in that XCD's L2.
constexpr int kSpmmLU = 16;

template <typename VT, typename BT, int LPR, int DB, int VPL>
__device__ __forceinline__ void sell_spmm_lanes_rows(int64_t a, int32_t w, int row, int g,
                                                     int32_t c0,
                                                     const int32_t* __restrict__ sci,
                                                     const uint16_t* __restrict__ sdl,
                                                     const int32_t* __restrict__ sbase,
                                                     const VT* __restrict__ sval,
                                                     const BT* __restrict__ B, int64_t ldb,
                                                     double* acc) {
  constexpr int G = kGroup<VT>;
  constexpr int CPL = 16 / sizeof(BT);
  using V = typename std::conditional<sizeof(BT) == 8, f64x2, f32x4>::type;
  using DT = typename std::conditional<DB == 16, uint16_t, uint8_t>::type;
  const DT* dp = reinterpret_cast<const DT*>(sdl + a * kChunk);
  const int32_t* bp = sbase + a;
  // a row's G slots of a full group are contiguous: one vector load each
  // (Hamiltonian-like matrix, 6M rows, against one load per slot: float32
  // k = 8/16/32 434/724/1420 -> 366/697/1383 us, float64 k = 8 653 -> 651;
  // float64 with 8 or 16 lanes per row 1243/2682 -> 1284/2713 at k = 16/32,
  // so those keep one load per slot)
  constexpr bool kVec = G == 4 || LPR <= 4;
  using VG = typename std::conditional<G == 2, f64x2, f32x4>::type;
  using CG = typename std::conditional<G == 2, i32x2, i32x4>::type;
  using DG = typename std::conditional<
      G == 2, typename std::conditional<DB == 16, uint32_t, uint16_t>::type,
      typename std::conditional<DB == 16, u32x2, uint32_t>::type>::type;
  const int32_t GQ = w - w % G;
  for (int32_t j = 0; j < w; j += kSpmmLU) {
    VT vr[kSpmmLU];
    int32_t c[kSpmmLU];
    if constexpr (DB > 0) {
      DG dg[kSpmmLU / G];
      uint32_t d[kSpmmLU];
      int32_t b[kSpmmLU];
#pragma unroll
      for (int u = 0; u < kSpmmLU; u += G) {
        const int32_t j0 = j + u;
        if (kVec && j0 + G <= GQ) {
          const int64_t o = G * ((int64_t)(j0 / G) * kChunk + row);
          const VG q = dev::ld_stream(reinterpret_cast<const VG*>(sval + a * kChunk + o));
          dg[u / G] = dev::ld_stream(reinterpret_cast<const DG*>(dp + o));
#pragma unroll
          for (int t = 0; t < G; ++t) {
            vr[u + t] = q[t];
            d[u + t] = 0xFFFFFFFFu;  // taken from dg below
            b[u + t] = bp[j0 + t];
          }
        } else {
          dg[u / G] = DG{};
#pragma unroll
          for (int t = 0; t < G; ++t) {
            if (j0 + t < w) {
              const int64_t o = slot_offset<G>(j0 + t, row, w);
              vr[u + t] = dev::ld_stream(sval + a * kChunk + o);
              d[u + t] = dev::ld_stream(dp + o);
              b[u + t] = bp[j0 + t];
            } else {
              vr[u + t] = (VT)0;
              d[u + t] = kPad<DB>;
              b[u + t] = 0;
            }
          }
        }
      }
#pragma unroll
      for (int u = 0; u < kSpmmLU / G; ++u) asm volatile("" : "+v"(dg[u]));
#pragma unroll
      for (int u = 0; u < kSpmmLU; ++u) asm volatile("" : "+v"(d[u]));
#pragma unroll
      for (int u = 0; u < kSpmmLU; u += G) {
        const bool full = kVec && j + u + G <= GQ;
#pragma unroll
        for (int t = 0; t < G; ++t)
          c[u + t] = delta_col<DB>(full ? delta_field<DB>(dg[u / G], t) : d[u + t], b[u + t]);
      }
    } else {
#pragma unroll
      for (int u = 0; u < kSpmmLU; u += G) {
        const int32_t j0 = j + u;
        if (kVec && j0 + G <= GQ) {
          const int64_t o = a * kChunk + G * ((int64_t)(j0 / G) * kChunk + row);
          const VG q = dev::ld_stream(reinterpret_cast<const VG*>(sval + o));
          const CG cq = dev::ld_stream(reinterpret_cast<const CG*>(sci + o));
#pragma unroll
          for (int t = 0; t < G; ++t) {
            vr[u + t] = q[t];
            c[u + t] = cq[t];
          }
        } else {
#pragma unroll
          for (int t = 0; t < G; ++t) {
            if (j0 + t < w) {
              const int64_t o = a * kChunk + slot_offset<G>(j0 + t, row, w);
              vr[u + t] = dev::ld_stream(sval + o);
              c[u + t] = dev::ld_stream(sci + o);
            } else {
              vr[u + t] = (VT)0;
              c[u + t] = -1;
            }
          }
        }
      }
    }
    V x[kSpmmLU][VPL];
#pragma unroll
    for (int u = 0; u < kSpmmLU; ++u) {
#pragma unroll
      for (int q = 0; q < VPL; ++q) {
        x[u][q] = V{};
        if (c[u] >= 0)
          x[u][q] = *reinterpret_cast<const V*>(B + (int64_t)c[u] * ldb + c0 +
                                                (g * VPL + q) * CPL);
      }
    }
    // the values and segments in their own types until every load is issued
#pragma unroll
    for (int u = 0; u < kSpmmLU; ++u) {
      asm volatile("" : "+v"(vr[u]));
#pragma unroll
      for (int q = 0; q < VPL; ++q) asm volatile("" : "+v"(x[u][q]));
    }
    // masked slots add fma(0, 0, acc) = acc exactly (acc is never -0)
#pragma unroll
    for (int u = 0; u < kSpmmLU; ++u) {
      const double v = dev::widen(vr[u]);
#pragma unroll
      for (int q = 0; q < VPL; ++q) {
        double* aq = acc + q * CPL;
        aq[0] = fma(v, (double)x[u][q][0], aq[0]);
        aq[1] = fma(v, (double)x[u][q][1], aq[1]);
        if constexpr (CPL == 4) {
          aq[2] = fma(v, (double)x[u][q][2], aq[2]);
          aq[3] = fma(v, (double)x[u][q][3], aq[3]);
        }
      }
    }
  }
}

template <typename VT, typename BT, int LPR, int VPL>
__global__ __launch_bounds__(kWG) void k_sell_spmm_lanes(
    int64_t nch, int64_t n, const int32_t* __restrict__ off, const int32_t* __restrict__ sci,
    const int32_t* __restrict__ flag, const int32_t* __restrict__ sbase,
    const uint16_t* __restrict__ sdl, const VT* __restrict__ sval, const BT* __restrict__ B,
    int64_t ldb, double* __restrict__ C, int64_t ldc, int32_t c0, int remap) {
  constexpr int CPL = 16 / sizeof(BT);
  const int64_t blk = remap ? dev::xcd_remap(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
  const int64_t wv = __builtin_amdgcn_readfirstlane(
      (int32_t)((blk * kWG + threadIdx.x) / kChunk));
  const int64_t chunk = wv / LPR;
  if (chunk >= nch) return;
  const int lane = threadIdx.x % kChunk;
  const int row = (int)(wv % LPR) * (kChunk / LPR) + lane / LPR;  // row inside the chunk
  const int g = lane % LPR;
  const int64_t a = off[chunk];
  const int32_t w = (int32_t)(off[chunk + 1] - a);
  double acc[CPL * VPL];
#pragma unroll
  for (int t = 0; t < CPL * VPL; ++t) acc[t] = 0.0;
  const int db = flag ? flag[chunk] : 0;
  if (db == 8)
    sell_spmm_lanes_rows<VT, BT, LPR, 8, VPL>(a, w, row, g, c0, sci, sdl, sbase, sval, B, ldb,
                                              acc);
  else if (db == 16)
    sell_spmm_lanes_rows<VT, BT, LPR, 16, VPL>(a, w, row, g, c0, sci, sdl, sbase, sval, B, ldb,
                                               acc);
  else
    sell_spmm_lanes_rows<VT, BT, LPR, 0, VPL>(a, w, row, g, c0, sci, sdl, sbase, sval, B, ldb,
                                              acc);
  const int64_t r = chunk * kChunk + row;
  if (r < n) {
    double* out = C + r * ldc + c0 + g * CPL * VPL;
#pragma unroll
    for (int t = 0; t < CPL * VPL; t += 2)
      *reinterpret_cast<f64x2*>(out + t) = f64x2{acc[t], acc[t + 1]};
  }
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
  if (!p.sell_wide) {
    if (p.vdt == SPMV_F64)
      k_sell_narrow<kGroup<double>><<<grid_chunks(nch), kWG, 0, s>>>(
          nch, p.sell_off, cap64, p.sell_ci, p.sell_base, p.sell_dl, p.sell_flag);
    else
      k_sell_narrow<kGroup<float>><<<grid_chunks(nch), kWG, 0, s>>>(
          nch, p.sell_off, cap64, p.sell_ci, p.sell_base, p.sell_dl, p.sell_flag);
    SPMV_HIP(hipGetLastError());
  }
  return SPMV_OK;
}

namespace {
template <typename VT, typename BT, int KB, int VEC>
int sell_spmm_pass(const Plan& p, int k, int c0, const BT* B, int64_t ldb, double* C, int64_t ldc,
                   hipStream_t s) {
  k_sell_spmm<VT, BT, KB, VEC><<<grid_chunks(p.sell_nch), kWG, 0, s>>>(
      p.sell_nch, p.n_rows, p.sell_off, p.sell_ci, p.sell_wide ? nullptr : p.sell_flag,
      p.sell_base, p.sell_dl, static_cast<const VT*>(p.sell_val), B, ldb, C, ldc, k, c0);
  SPMV_HIP(hipGetLastError());
  return SPMV_OK;
}

template <typename VT, typename BT, int LPR, int VPL = 1>
int sell_spmm_lanes_pass(const Plan& p, int c0, const BT* B, int64_t ldb, double* C,
                         int64_t ldc, hipStream_t s) {
  const int64_t threads = p.sell_nch * LPR * kChunk;
  // contiguous chunk ranges per XCD once B outgrows the 256 MB last-level
  // cache (measured on the Hamiltonian-like matrix: 12% faster at 768 MB of
  // B, 3% slower at 384 MB)
  const int remap = (double)p.n_cols * (LPR * VPL * 16) > 512.0 * (1 << 20);
  k_sell_spmm_lanes<VT, BT, LPR, VPL><<<(unsigned)((threads + kWG - 1) / kWG), kWG, 0, s>>>(
      p.sell_nch, p.n_rows, p.sell_off, p.sell_ci, p.sell_wide ? nullptr : p.sell_flag,
      p.sell_base, p.sell_dl, static_cast<const VT*>(p.sell_val), B, ldb, C, ldc, c0, remap);
  SPMV_HIP(hipGetLastError());
  return SPMV_OK;
}

template <typename VT, typename BT>
int sell_spmm_typed(const Plan& p, int k, const BT* B, int64_t ldb, double* C, int64_t ldc,
                    hipStream_t s) {
  // lane groups: k a multiple of the vector width, at most 16 lanes per row
  // in one pass, B and C aligned to 16-byte vectors; float64 from 4 lanes per
  // row (k = 8) on: at k = 4 one lane per row with two 16-byte B loads per
  // slot is faster (Hamiltonian-like matrix, 6M rows: 315 against 361 us;
  // float32 at 2 lanes per row, k = 8, the other way: 361 against 427 us)
  constexpr int CPL = 16 / sizeof(BT);
  constexpr int kMinLanes = std::is_same<BT, double>::value ? 4 : 2;
  const bool lanes_ok = k % CPL == 0 && k >= kMinLanes * CPL && k <= 16 * CPL &&
                        (double)p.sell_nch * (k / CPL) * kChunk < 4294967295.0 &&
                        reinterpret_cast<uintptr_t>(B) % 16 == 0 && ldb % CPL == 0 &&
                        reinterpret_cast<uintptr_t>(C) % 16 == 0 && ldc % 2 == 0;
  // float64: two B vectors (4 columns) per lane, half the lanes per row
  // (Hamiltonian-like matrix, 6M rows, k = 8/16/32: 653/1251/2671 -> 593/
  // 1216/2591 us; float32 with two quads per lane 5-11% slower at k = 16..64)
  if (lanes_ok && std::is_same<BT, double>::value) {
    switch (k / CPL) {
      case 4: return sell_spmm_lanes_pass<VT, BT, 2, 2>(p, 0, B, ldb, C, ldc, s);
      case 8: return sell_spmm_lanes_pass<VT, BT, 4, 2>(p, 0, B, ldb, C, ldc, s);
      case 16: return sell_spmm_lanes_pass<VT, BT, 8, 2>(p, 0, B, ldb, C, ldc, s);
      default: break;
    }
  }
  if (lanes_ok) {
    switch (k / CPL) {
      case 2: return sell_spmm_lanes_pass<VT, BT, 2>(p, 0, B, ldb, C, ldc, s);
      case 4: return sell_spmm_lanes_pass<VT, BT, 4>(p, 0, B, ldb, C, ldc, s);
      case 8: return sell_spmm_lanes_pass<VT, BT, 8>(p, 0, B, ldb, C, ldc, s);
      case 16: return sell_spmm_lanes_pass<VT, BT, 16>(p, 0, B, ldb, C, ldc, s);
      default: break;  // other widths: column blocks below
    }
  }
  // columns in blocks of KB = the smallest of 1, 2, 4, 8 covering min(k, 8)
  const int KB = k >= 5 ? 8 : k >= 3 ? 4 : k == 2 ? 2 : 1;
  // vector loads of B row segments need them aligned to the load width:
  // 16 bytes for float64 pairs and float32 quads, 8 for float32 pairs
  // (c0 is a multiple of KB)
  const uintptr_t ba = reinterpret_cast<uintptr_t>(B);
  const bool vec = KB >= 2 && (std::is_same<BT, double>::value ? ba % 16 == 0 && ldb % 2 == 0
                               : KB == 2 ? ba % 8 == 0 && ldb % 2 == 0
                                         : ba % 16 == 0 && ldb % 4 == 0);
  // a partial block (k = 3, 5..7) loads pairs where rows are aligned to them
  const bool pairs = std::is_same<BT, double>::value ? ba % 16 == 0 && ldb % 2 == 0
                                                     : ba % 8 == 0 && ldb % 2 == 0;
  for (int c0 = 0; c0 < k; c0 += KB) {
    // a full-width block takes the vector path; a partial last block pairs
    // and a scalar last column (scalar loads where rows are not aligned)
    const bool full = c0 + KB <= k;
    int st = SPMV_OK;
    switch (KB) {
      case 1: st = sell_spmm_pass<VT, BT, 1, 0>(p, k, c0, B, ldb, C, ldc, s); break;
      case 2:
        st = vec && full ? sell_spmm_pass<VT, BT, 2, 1>(p, k, c0, B, ldb, C, ldc, s)
                         : sell_spmm_pass<VT, BT, 2, 0>(p, k, c0, B, ldb, C, ldc, s);
        break;
      case 4:
        st = vec && full    ? sell_spmm_pass<VT, BT, 4, 1>(p, k, c0, B, ldb, C, ldc, s)
             : pairs && !full ? sell_spmm_pass<VT, BT, 4, 2>(p, k, c0, B, ldb, C, ldc, s)
                              : sell_spmm_pass<VT, BT, 4, 0>(p, k, c0, B, ldb, C, ldc, s);
        break;
      default:
        st = vec && full    ? sell_spmm_pass<VT, BT, 8, 1>(p, k, c0, B, ldb, C, ldc, s)
             : pairs && !full ? sell_spmm_pass<VT, BT, 8, 2>(p, k, c0, B, ldb, C, ldc, s)
                              : sell_spmm_pass<VT, BT, 8, 0>(p, k, c0, B, ldb, C, ldc, s);
    }
    if (st) return st;
  }
  return SPMV_OK;
}
}  // namespace

bool sell_spmm_lanes_fit(const Plan& p, int k, const void* B, int64_t ldb, const double* C,
                         int64_t ldc) {
  const int cpl = p.vdt == SPMV_F64 ? 2 : 4;
  const int lpr = k % cpl == 0 ? k / cpl : 0;
  return (lpr == 2 || lpr == 4 || lpr == 8 || lpr == 16) &&
         (double)p.sell_nch * lpr * kChunk < 4294967295.0 &&
         reinterpret_cast<uintptr_t>(B) % 16 == 0 && ldb % cpl == 0 &&
         reinterpret_cast<uintptr_t>(C) % 16 == 0 && ldc % 2 == 0;
}

int launch_sell_spmm(const Plan& p, int k, const void* B, int64_t ldb, double* C, int64_t ldc,
                     hipStream_t s) {
  if (!p.sell_ok) return fail(SPMV_ERR_STATE, "V6 is not built for this plan");
  if (p.sell_nch == 0) return SPMV_OK;
  if (p.vdt == SPMV_F64)
    return sell_spmm_typed<double, double>(p, k, static_cast<const double*>(B), ldb, C, ldc, s);
  return sell_spmm_typed<float, float>(p, k, static_cast<const float*>(B), ldb, C, ldc, s);
}

int launch_sell(const Plan& p, const void* B, double* C, hipStream_t s) {
  if (!p.sell_ok) return fail(SPMV_ERR_STATE, "V6 is not built for this plan");
  if (p.sell_nch == 0) return SPMV_OK;
  if (p.vdt == SPMV_F64)
    k_sell_pairs<<<grid_chunks(p.sell_nch), kWG, 0, s>>>(
        p.sell_nch, p.n_rows, p.sell_off, p.sell_ci, p.sell_wide ? nullptr : p.sell_flag,
        p.sell_base, p.sell_dl, static_cast<const double*>(p.sell_val),
        static_cast<const double*>(B), C);
  else
    k_sell_quads<float><<<grid_chunks(p.sell_nch), kWG, 0, s>>>(
        p.sell_nch, p.n_rows, p.sell_off, p.sell_ci, p.sell_wide ? nullptr : p.sell_flag,
        p.sell_base, p.sell_dl, static_cast<const float*>(p.sell_val),
        static_cast<const float*>(B), C);
  SPMV_HIP(hipGetLastError());
  return SPMV_OK;
}

}  // namespace spmv
