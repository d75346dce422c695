// V4 in its window form: row super-blocks that stage a few aligned windows of
// B in LDS, with every wavefront streaming its own row range.
//
// A super-block is kSbRows consecutive rows, one workgroup. At create, the
// columns of each super-block are counted per aligned bin of kWinSize columns
// and the WinCount<BT> most populated bins become its windows. At apply, the
// workgroup copies those windows of B into LDS with coalesced loads (the one
// barrier of the kernel); then each wavefront walks its share of the rows on
// its own: it streams their nonzeros in chunks (the loads of later chunks in
// flight while a chunk is summed), gathers B from LDS when the column lies in
// a window and from global memory otherwise, writes the products to its
// private LDS chunk, and adds them up row by row.
//
// A lane owns one row of a 64-row group and adds that row's products in CRS
// order, acc = acc + val(j) * B(col_idx(j)) with the product rounded before
// the sum: the Sect. 1.2 loop exactly, so every row reproduces the plain
// sequential loop bit for bit, whatever its length.
//
// The form suits matrices whose rows gather from a few column regions that
// are each dense in B but scattered inside: a stencil whose rows and columns
// were permuted within blocks is the case in point (the windows hold the
// diagonal block and the blocks one grid plane away).
#include <type_traits>

#include "common.hpp"
#include "device.hpp"

namespace spmv {
namespace {

using dev::group_sum;
using dev::ld_stream;
using dev::widen;

constexpr int kRowStep = 8;                 // products a lane adds per pass over its row

// Launch shape per element type (measured on the permuted 3D stencil, 21.95M
// rows: float64 two windows, 8 wavefronts, 256-entry chunks, two chunks in
// flight -- 80 KB of LDS, two workgroups per CU; 745-750 us against 765-810
// us for three windows and 16 wavefronts, 1024-lane workgroups or 512-entry
// chunks; float32 three windows, 8 wavefronts, 256-entry chunks, three chunks
// in flight -- 64 KB, 583 us against 595-645 us)
template <typename BT>
constexpr int WinCount = sizeof(BT) == 8 ? 2 : 3;
template <typename BT>
constexpr int WinWaves = 8;
template <typename BT>
constexpr int WinChunk = 256;
template <typename BT>
constexpr int WinDepth = sizeof(BT) == 8 ? 2 : 3;
static_assert(WinCount<float> <= kWinMax && WinCount<double> <= kWinMax, "window table");

// Raw buffer resources (gfx9 family: word 3 = 0x00020000, 32-bit data, no
// swizzle): a load at a byte offset at or past the resource's size returns
// zero and touches no memory, which bounds the loads of a chunk without a
// branch per lane.
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;
constexpr int kCpolNT = 2;  // nontemporal

__device__ __forceinline__ rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                           kRsrcWord3);
}

template <typename T, int CPOL>
__device__ __forceinline__ T buf_load(rsrc_t r, uint32_t off) {
  if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, CPOL));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, CPOL));
}

__device__ __forceinline__ void wave_sync() {
  // LDS written by one lane and read by another of the same wavefront: the
  // LDS unit serves a wavefront's instructions in order, so the compiler
  // only has to keep the accesses on their side of this point
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The val/col_idx stream of nonzeros [c0, min(c0 + kChunk, E)) through
// buffer resources: load u of a lane reads entry c0 + 64 u + lane from a
// resource based at c0 + 64 u and sized to the entries left there, so lanes
// past E read zeros (no memory traffic, no branch: every wait count before a
// use stays exact and the loads of later chunks stay in flight). The column
// loads go first, as the gathers wait for them.
template <typename VT, int PL>
__device__ __forceinline__ void load_chunk(const VT* __restrict__ val,
                                           const int32_t* __restrict__ ci, int32_t c0, int32_t E,
                                           uint32_t lane, VT (&v)[PL], int32_t (&c)[PL]) {
  // uniform; readfirstlane keeps the bounds (and the resources) scalar
  c0 = __builtin_amdgcn_readfirstlane(c0);
  const int32_t left = __builtin_amdgcn_readfirstlane(E - c0);
#pragma unroll
  for (int u = 0; u < PL; ++u) {
    const int32_t n = left - 64 * u;
    const uint32_t cnt =
        __builtin_amdgcn_readfirstlane(n <= 0 ? 0u : (n < 64 ? (uint32_t)n : 64u));
    c[u] = buf_load<int32_t, kCpolNT>(make_rsrc(ci + c0 + 64 * u, cnt * 4u), lane * 4u);
  }
#pragma unroll
  for (int u = 0; u < PL; ++u) {
    const int32_t n = left - 64 * u;
    const uint32_t cnt =
        __builtin_amdgcn_readfirstlane(n <= 0 ? 0u : (n < 64 ? (uint32_t)n : 64u));
    v[u] = buf_load<VT, kCpolNT>(make_rsrc(val + c0 + 64 * u, cnt * (uint32_t)sizeof(VT)),
                                 lane * (uint32_t)sizeof(VT));
  }
}

// The chunk's B values, gathered with no branch: an LDS read at the window
// slot (clamped to slot 0 when no window holds the column) and a global read
// that only lanes outside every window perform. BUFB: the global read goes
// through a buffer resource and lanes inside a window read at an offset past
// its end, which yields +0.0; xs is zeroed for lanes outside, so the value is
// xs + xg (adding +0.0 can only turn a -0.0 into +0.0, and the product of
// a zero B value adds a zero to a row sum that is never -0.0, so no result
// changes). Else xg of a lane inside a window reads the first entry of its
// window (a line shared by such lanes) and xs carries the selection.
template <typename BT, int NW, bool BUFB, int PL>
__device__ __forceinline__ void gather_chunk(const BT* __restrict__ B, rsrc_t rB, const BT* wB,
                                             const int32_t (&wbin)[NW > 0 ? NW : 1],
                                             const int32_t (&c)[PL], BT (&xs)[PL],
                                             BT (&xg)[PL], uint64_t (&inw)[PL]) {
#pragma unroll
  for (int u = 0; u < PL; ++u) {
    const int32_t col = c[u];
    const int32_t bin = col >> kWinLog;
    bool in = false;
    int32_t base = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      const bool h = bin == wbin[w];
      in = in || h;
      base = h ? w * kWinSize : base;
    }
    BT x = (BT)0;
    if constexpr (NW > 0) x = wB[base + (col & (kWinSize - 1))];
    if constexpr (BUFB) {
      xs[u] = in ? x : (BT)0;
      xg[u] = buf_load<BT, 0>(rB, in ? 0xFFFFFFFFu : (uint32_t)col * (uint32_t)sizeof(BT));
    } else {
      xs[u] = x;
      inw[u] = __ballot(in);
      xg[u] = B[in ? (col & ~(kWinSize - 1)) : col];
    }
  }
}

template <typename BT, bool BUFB>
__device__ __forceinline__ BT gather_pick(BT xs, BT xg, uint64_t inw, int lane) {
  if constexpr (BUFB)
    return xs + xg;
  else
    return ((inw >> lane) & 1) ? xs : xg;
}

// row_ptr of the lane's row in a 64-row group (cur) and the end of that row:
// the next lane's value, or for lane 63 lane 0 of the next group (nxt)
__device__ __forceinline__ int32_t row_end(int32_t cur, int32_t nxt, int lane) {
  const int32_t up = __shfl_down(cur, 1);
  const int32_t first_next = __shfl(nxt, 0);
  return lane < 63 ? up : first_next;
}

// BUFB: B is read through a buffer resource (n_cols * sizeof(BT) < 2^32).
// NW windows, WAVES wavefronts per workgroup, CHUNK nonzeros per wavefront
// chunk (the LDS holds NW * kWinSize entries of B and WAVES * CHUNK products).
template <typename VT, typename BT, bool BUFB, int NW = WinCount<BT>, int WAVES = WinWaves<BT>,
          int CHUNK = WinChunk<BT>, int DEPTH = WinDepth<BT>>
__global__ __launch_bounds__(WAVES * 64) void k_win_rows(int64_t n_rows, int64_t n_cols,
                                                        int64_t nsb,
                                                        const int32_t* __restrict__ win,
                                                        const int32_t* __restrict__ rp,
                                                        const int32_t* __restrict__ ci,
                                                        const VT* __restrict__ val,
                                                        const BT* __restrict__ B,
                                                        double* __restrict__ C) {
  constexpr int kPerLane = CHUNK / 64;
  constexpr int kRowsPerWave = kSbRows / WAVES;
  constexpr int kGroups = kRowsPerWave / 64;
  constexpr int kThreads = WAVES * 64;
  constexpr int kChunk = CHUNK;
  __shared__ BT wB[NW > 0 ? NW * kWinSize : 1];
  __shared__ double prod[WAVES * CHUNK];
  const int64_t q = dev::xcd_remap(blockIdx.x, nsb);
  // wave-uniform (readfirstlane tells the compiler, so that everything
  // derived from it -- row range, stream bounds, buffer resources -- lives in
  // scalar registers)
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t ra64 = q * kSbRows + (int64_t)wave * kRowsPerWave;
  const int32_t ra = (int32_t)(ra64 < n_rows ? ra64 : n_rows);
  const int32_t rb = (int32_t)(ra64 + kRowsPerWave < n_rows ? ra64 + kRowsPerWave : n_rows);
  int32_t wbin[NW > 0 ? NW : 1] = {-1};
#pragma unroll
  for (int w = 0; w < NW; ++w) wbin[w] = win[q * kWinMax + w];
  const rsrc_t rB = make_rsrc(B, BUFB ? (uint32_t)(n_cols * (int64_t)sizeof(BT)) : 0u);
  // row_ptr of all the wavefront's rows, one per lane and group (rows past
  // rb read row_ptr[rb]: empty rows, never stored); R[kGroups] = E
  int32_t R[kGroups + 1];
#pragma unroll
  for (int k = 0; k < kGroups; ++k) {
    const int32_t rr = ra + 64 * k + lane;
    R[k] = rp[rr < rb ? rr : rb];
  }
  const int32_t S = rp[ra], E = rp[rb];
  R[kGroups] = E;

  // the first chunk's stream is in flight while the windows are staged
  VT v[kPerLane];
  int32_t c[kPerLane];
  load_chunk(val, ci, S, E, lane, v, c);
  {
    // window u / kPerWin, offset threadIdx.x + (u % kPerWin) * kThreads
    constexpr int kPerWin = kWinSize / kThreads;
    constexpr int kSt = NW * kPerWin;
    BT st[kSt > 0 ? kSt : 1];
#pragma unroll
    for (int u = 0; u < kSt; ++u) {
      const int32_t bin = wbin[u / kPerWin];
      const int64_t col = ((int64_t)bin << kWinLog) + threadIdx.x + (u % kPerWin) * kThreads;
      st[u] = (bin >= 0 && col < n_cols) ? B[col] : (BT)0;
    }
#pragma unroll
    for (int u = 0; u < kSt; ++u) wB[threadIdx.x + u * kThreads] = st[u];
  }
  __syncthreads();

  int32_t rg = ra;
  int32_t r = rg + lane;
  bool valid = r < rb;
  int32_t s = R[0], e = row_end(R[0], R[1], lane);
  double acc = 0.0;
  int32_t c0 = S;
  double* P = prod + wave * kChunk;

  // Row sums of the chunk [c0, c1) whose products are in P; returns true when
  // the wavefront's rows are done.
  auto rows = [&](int32_t c1) __attribute__((always_inline)) -> bool {
    for (;;) {
      // the lane adds its row's products of this chunk in ascending order,
      // kRowStep per pass; the wavefront makes as many passes as its
      // longest row needs here (a masked slot adds +0.0, which leaves acc
      // unchanged: acc starts at +0.0 and a sum of finite values is -0.0
      // only when both terms are)
      const int32_t lo = s > c0 ? s : c0;
      const int32_t hi = e < c1 ? e : c1;
      for (int32_t k = lo; k < hi; k += kRowStep) {
        const double* pk = P + (k - c0);
        double p[kRowStep];
#pragma unroll
        for (int t = 0; t < kRowStep; ++t) p[t] = k + t < hi ? pk[t] : 0.0;
#pragma unroll
        for (int t = 0; t < kRowStep; ++t) acc += p[t];
      }
      if (!__all(!valid || e <= c1)) return false;  // a row of the group goes on
      if (valid) C[r] = acc;
      rg += 64;
      if (rg >= rb) return true;
      r = rg + lane;
      valid = r < rb;
#pragma unroll
      for (int k = 0; k < kGroups; ++k) R[k] = R[k + 1];
      s = R[0];
      e = row_end(R[0], R[1], lane);
      acc = 0.0;
    }
  };

  if constexpr (DEPTH == 2) {
    // While the products of chunk i are summed from LDS, the gathers of
    // chunk i+1 and the stream of chunk i+2 are in flight; once the sums are
    // done, chunk i+1's products replace chunk i's. The two stream buffers
    // swap roles every chunk; the loop is unrolled twice so that no register
    // a load is still filling is ever copied (a copy would wait for the load).
    VT vb[kPerLane];
    int32_t cb[kPerLane];
    {
      BT xs[kPerLane], xg[kPerLane];
      uint64_t inw[kPerLane];
      gather_chunk<BT, NW, BUFB, kPerLane>(B, rB, wB, wbin, c, xs, xg, inw);
      load_chunk(val, ci, S + kChunk, E, lane, vb, cb);
#pragma unroll
      for (int u = 0; u < kPerLane; ++u)
        P[lane + 64 * u] = widen(v[u]) * widen(gather_pick<BT, BUFB>(xs[u], xg[u], inw[u], lane));
      wave_sync();
    }
    auto step = [&](VT(&vN)[kPerLane], const int32_t(&cN)[kPerLane], VT(&vF)[kPerLane],
                    int32_t(&cF)[kPerLane]) __attribute__((always_inline)) -> bool {
      const int32_t c1 = c0 + kChunk < E ? c0 + kChunk : E;
      BT xs[kPerLane], xg[kPerLane];
      uint64_t inw[kPerLane];
      gather_chunk<BT, NW, BUFB, kPerLane>(B, rB, wB, wbin, cN, xs, xg, inw);
      load_chunk(val, ci, c1 + kChunk, E, lane, vF, cF);
      if (rows(c1)) return true;
      // (c1 == E with rows unfinished only happens for a row_ptr that is not
      // nondecreasing, possible with SPMV_FLAG_SKIP_VALIDATE: leave, do not spin)
      if (c1 >= E) return true;
      wave_sync();  // every read of this chunk's products before the next writes
#pragma unroll
      for (int u = 0; u < kPerLane; ++u)
        P[lane + 64 * u] =
            widen(vN[u]) * widen(gather_pick<BT, BUFB>(xs[u], xg[u], inw[u], lane));
      wave_sync();
      c0 = c1;
      return false;
    };
    VT va[kPerLane];
    int32_t ca[kPerLane];
    for (;;) {
      if (step(vb, cb, va, ca)) break;
      if (step(va, ca, vb, cb)) break;
    }
  } else {
    // Three chunks ahead: while chunk i is summed, the gathers of chunk i+1
    // (issued a chunk earlier) complete, those of chunk i+2 and the stream
    // of chunk i+3 are in flight; then chunk i+1's products replace chunk
    // i's. Three register sets rotate roles (the loop is unrolled three times).
    struct Set {
      VT v[kPerLane];
      int32_t c[kPerLane];
      BT xs[kPerLane], xg[kPerLane];
      uint64_t inw[kPerLane];
    };
    Set S0, S1, S2;
#pragma unroll
    for (int u = 0; u < kPerLane; ++u) {
      S0.v[u] = v[u];
      S0.c[u] = c[u];
    }
    load_chunk(val, ci, S + kChunk, E, lane, S1.v, S1.c);
    gather_chunk<BT, NW, BUFB, kPerLane>(B, rB, wB, wbin, S0.c, S0.xs, S0.xg, S0.inw);
#pragma unroll
    for (int u = 0; u < kPerLane; ++u)
      P[lane + 64 * u] =
          widen(S0.v[u]) * widen(gather_pick<BT, BUFB>(S0.xs[u], S0.xg[u], S0.inw[u], lane));
    wave_sync();
    load_chunk(val, ci, S + 2 * kChunk, E, lane, S2.v, S2.c);
    gather_chunk<BT, NW, BUFB, kPerLane>(B, rB, wB, wbin, S1.c, S1.xs, S1.xg, S1.inw);
    // Sa: chunk i+1 (gathered), Sb: chunk i+2 (to gather), Sc: receives chunk i+3
    auto step = [&](Set& Sa, Set& Sb, Set& Sc) __attribute__((always_inline)) -> bool {
      const int32_t c1 = c0 + kChunk < E ? c0 + kChunk : E;
      gather_chunk<BT, NW, BUFB, kPerLane>(B, rB, wB, wbin, Sb.c, Sb.xs, Sb.xg, Sb.inw);
      load_chunk(val, ci, c0 + 3 * kChunk, E, lane, Sc.v, Sc.c);
      if (rows(c1)) return true;
      if (c1 >= E) return true;  // (see above)
      wave_sync();
#pragma unroll
      for (int u = 0; u < kPerLane; ++u)
        P[lane + 64 * u] =
            widen(Sa.v[u]) * widen(gather_pick<BT, BUFB>(Sa.xs[u], Sa.xg[u], Sa.inw[u], lane));
      wave_sync();
      c0 = c1;
      return false;
    };
    for (;;) {
      if (step(S1, S2, S0)) break;
      if (step(S2, S0, S1)) break;
      if (step(S0, S1, S2)) break;
    }
  }
}

// Windows of every super-block: its columns counted per aligned bin of
// kWinSize columns in an LDS hash table (open addressing, at most kProbe
// probes; a bin that finds no slot is not counted, which can only cost
// coverage, never correctness), then the `nw` bins with the largest counts,
// ties to the smaller bin. Unused entries are -1. The entries the chosen
// windows hold are added to h->win_covered.
// 4096 slots (32 KB of LDS with the counts, four workgroups per CU): the
// permuted mesh's super-blocks hold ~2,700 distinct bins, most of them single
// random extras; 8192 slots took 1.8 ms longer there (two workgroups per CU),
// 2048 slots overflowed and probed long
constexpr int kHash = 4096;
constexpr int kHashLog = 12;
static_assert(kHash == 1 << kHashLog, "hash size");
constexpr int kProbe = 32;
constexpr int kSelWG = 512;  // 8 wavefronts: 3.1 against 4.0 ms with 4 for config 3

__global__ __launch_bounds__(kSelWG) void k_sb_windows(int64_t n_rows, int64_t nnz, int64_t nsb,
                                                       int nw, const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ ci,
                                                       int32_t* __restrict__ win, WsHeader* h) {
  __shared__ int32_t key[kHash];
  __shared__ int32_t cnt[kHash];
  __shared__ int32_t redc[kSelWG / 64], redk[kSelWG / 64], redi[kSelWG / 64];
  const int64_t q = blockIdx.x;
  if (q >= nsb) return;
  const int64_t r0 = q * kSbRows;
  const int64_t r1 = r0 + kSbRows < n_rows ? r0 + kSbRows : n_rows;
  int64_t S = rp[r0], E = rp[r1];
  S = S < 0 ? 0 : S > nnz ? nnz : S;
  E = E < S ? S : E > nnz ? nnz : E;
  for (int i = threadIdx.x; i < kHash; i += kSelWG) {
    key[i] = -1;
    cnt[i] = 0;
  }
  __syncthreads();
  // each wavefront first groups its 64 columns by bin (one ballot per
  // distinct bin), so one lane per bin touches the table: the bins of a
  // row block repeat, and per-entry atomics on a few hot slots serialised
  const int lane = threadIdx.x & 63;
  for (int64_t j0 = S + (threadIdx.x & ~63); j0 < E; j0 += kSelWG) {
    const int64_t j = j0 + lane;
    const bool act = j < E;
    const int32_t bin = act ? ci[j] >> kWinLog : 0;
    uint64_t todo = __ballot(act);
    while (todo) {
      const int leader = __ffsll((unsigned long long)todo) - 1;
      const int32_t lb = __shfl(bin, leader);
      const uint64_t same = __ballot(act && bin == lb);
      if (lane == leader) {
        uint32_t slot = ((uint32_t)lb * 2654435761u) >> (32 - kHashLog);
        for (int t = 0; t < kProbe; ++t) {
          const int32_t old = atomicCAS(&key[slot], -1, lb);
          if (old == -1 || old == lb) {
            atomicAdd(&cnt[slot], (int32_t)__popcll(same));
            break;
          }
          slot = (slot + 1) & (kHash - 1);
        }
      }
      todo &= ~same;
    }
  }
  __syncthreads();
  unsigned long long covered = 0;
  for (int w = 0; w < kWinMax; ++w) {
    int32_t bc = 0, bk = INT32_MAX, bi = -1;
    if (w < nw) {
      for (int i = threadIdx.x; i < kHash; i += kSelWG) {
        const int32_t n = cnt[i], k = key[i];
        if (n > bc || (n == bc && n > 0 && k < bk)) {
          bc = n;
          bk = k;
          bi = i;
        }
      }
      for (int o = 32; o >= 1; o >>= 1) {
        const int32_t oc = __shfl_xor(bc, o), ok = __shfl_xor(bk, o), oi = __shfl_xor(bi, o);
        if (oc > bc || (oc == bc && oc > 0 && ok < bk)) {
          bc = oc;
          bk = ok;
          bi = oi;
        }
      }
      if ((threadIdx.x & 63) == 0) {
        redc[threadIdx.x >> 6] = bc;
        redk[threadIdx.x >> 6] = bk;
        redi[threadIdx.x >> 6] = bi;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int32_t c = 0, k = -1, i = -1;
      if (w < nw) {
        c = redc[0], k = redk[0], i = redi[0];
        for (int x = 1; x < kSelWG / 64; ++x)
          if (redc[x] > c || (redc[x] == c && c > 0 && redk[x] < k)) {
            c = redc[x];
            k = redk[x];
            i = redi[x];
          }
      }
      win[q * kWinMax + w] = c > 0 ? k : -1;
      if (c > 0) {
        covered += (unsigned long long)c;
        cnt[i] = 0;  // taken
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && covered) atomicAdd(&h->win_covered, covered);
}

template <typename VT, typename BT>
int launch_win_typed(const Plan& p, const void* B, double* C, hipStream_t s) {
  const bool bufb = p.n_cols * (int64_t)sizeof(BT) < (int64_t)0xFFFFFFFF;
  constexpr unsigned kThreads = 64 * WinWaves<BT>;
  if (bufb)
    k_win_rows<VT, BT, true><<<(unsigned)p.nsb, kThreads, 0, s>>>(
        p.n_rows, p.n_cols, p.nsb, p.win, p.row_ptr, p.col_idx, static_cast<const VT*>(p.val),
        static_cast<const BT*>(B), C);
  else
    k_win_rows<VT, BT, false><<<(unsigned)p.nsb, kThreads, 0, s>>>(
        p.n_rows, p.n_cols, p.nsb, p.win, p.row_ptr, p.col_idx, static_cast<const VT*>(p.val),
        static_cast<const BT*>(B), C);
  SPMV_HIP(hipGetLastError());
  return SPMV_OK;
}

}  // namespace

int win_count(int vdt) { return vdt == SPMV_F64 ? WinCount<double> : WinCount<float>; }

int launch_win_build(Plan& p, hipStream_t s) {
  if (p.nsb <= 0) return SPMV_OK;
  k_sb_windows<<<(unsigned)p.nsb, kSelWG, 0, s>>>(p.n_rows, p.nnz, p.nsb, win_count(p.vdt),
                                                 p.row_ptr, p.col_idx, p.win, p.hdr);
  SPMV_HIP(hipGetLastError());
  return SPMV_OK;
}

int launch_win(const Plan& p, const void* B, double* C, hipStream_t s) {
  if (p.nsb <= 0) return SPMV_OK;
  // every row is empty: the kernel's loads need at least one nonzero
  if (p.nnz == 0) return launch_fill(C, SPMV_F64, p.n_rows, 0.0, s);
  if (p.vdt == SPMV_F64) return launch_win_typed<double, double>(p, B, C, s);
  return launch_win_typed<float, float>(p, B, C, s);
}

}  // namespace spmv
