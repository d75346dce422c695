// C ABI of libspmv (declared in include/spmv.h).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"

namespace spmv {

namespace {
thread_local std::string g_err;

struct SelectorHost {
  float mu[SPMV_NUM_FEATURES];
  float sigma[SPMV_NUM_FEATURES];
  float lo[SPMV_NUM_FEATURES];
  float hi[SPMV_NUM_FEATURES];
  float margin = 0.0f;
  bool have_norm = false;
};
SelectorHost g_sel;

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

int dtype_bytes(int dt) { return dt == SPMV_F64 ? 8 : 4; }
bool dtype_ok(int dt) { return dt == SPMV_F64 || dt == SPMV_F32; }

struct PlanLayout {
  size_t header = 0, blocks = 0, spans = 0, win = 0, bins = 0, stats = 0, bin_base = 0, at_B = 0, at_C = 0;
  size_t sell_width = 0, sell_off = 0, sell_partials = 0, sell_ci = 0, sell_val = 0;
  size_t sell_base = 0, sell_dl = 0, sell_flag = 0;
  size_t total = 0;
};

PlanLayout plan_layout(int64_t n_rows, int64_t n_cols, int64_t nnz, uint32_t flags) {
  PlanLayout L;
  const int64_t nb = lds_block_count(n_rows, nnz);
  size_t o = 0;
  L.header = o;
  o += kHeaderBytes;
  L.blocks = o;
  o += align256(sizeof(int2) * (size_t)(nb + 1));
  L.spans = o;
  o += align256(sizeof(int2) * (size_t)std::max<int64_t>(nb, 1));
  L.win = o;
  o += align256(sizeof(int32_t) * kWinMax * (size_t)std::max<int64_t>(super_block_count(n_rows), 1));
  L.bins = o;
  o += align256(sizeof(int32_t) * (size_t)std::max<int64_t>(n_rows, 1));
  L.stats = o;
  o += align256(8 * (size_t)kStatsGrid * kPartSlots);
  L.bin_base = o;
  o += align256(4 * (size_t)kStatsGrid * kNumBins);
  const uint32_t mode = flags & 0xFFu;
  // timing scratch: autotune and the MLP selector's fallback to it
  if (mode == SPMV_SELECT_MLP || mode == SPMV_SELECT_AUTOTUNE) {
    L.at_B = o;
    o += align256(8 * (size_t)std::max<int64_t>(n_cols, 1));
    L.at_C = o;
    o += align256(8 * (size_t)std::max<int64_t>(n_rows, 1));
  }
  if (flags & SPMV_FLAG_SELL) {
    const int64_t nch = sell_chunks(n_rows), cap = sell_capacity(nnz);
    L.sell_width = o;
    o += align256(4 * (size_t)std::max<int64_t>(nch, 1));
    L.sell_off = o;
    o += align256(4 * (size_t)(nch + 1));
    L.sell_partials = o;
    o += align256(4 * (size_t)scan_partials_count(nch));
    L.sell_ci = o;
    o += align256(4 * (size_t)cap);
    L.sell_val = o;
    o += align256(8 * (size_t)cap);
    L.sell_base = o;
    o += align256(4 * (size_t)(cap / 64));
    L.sell_dl = o;
    o += align256(2 * (size_t)cap);
    L.sell_flag = o;
    o += align256(4 * (size_t)std::max<int64_t>(nch, 1));
  }
  L.total = o;
  return L;
}

int check_shape(int64_t n_rows, int64_t n_cols, int64_t nnz) {
  if (n_rows < 0 || n_cols < 0 || nnz < 0) return fail(SPMV_ERR_INVALID_ARG, "negative size");
  if (nnz > kMaxDim || n_rows > kMaxDim || n_cols > kMaxDim)
    return fail(SPMV_ERR_UNSUPPORTED, "n_rows, n_cols and nnz must each be at most 2^31 - 4097");
  return SPMV_OK;
}

// Times every variant the plan has on a B of ones: one warm-up and one timed
// launch each; a variant within 1.5x of the best time so far gets four more
// and is scored by the median of its five. The fastest is kept.
int autotune(Plan& p, hipStream_t s) {
  if (!p.at_B || !p.at_C)
    return fail(SPMV_ERR_WORKSPACE, "autotune needs the workspace size of an autotune/MLP plan");
  int st = launch_fill(p.at_B, p.vdt, p.n_cols, 1.0, s);
  if (st) return st;
  hipEvent_t e0, e1;
  SPMV_HIP(hipEventCreate(&e0));
  SPMV_HIP(hipEventCreate(&e1));
  constexpr int kReps = 5;
  float best = INFINITY;
  auto timed = [&](int v, float* ms) {
    hipEventRecord(e0, s);
    int r = launch_spmv(p, v, p.at_B, p.at_C, s);
    hipEventRecord(e1, s);
    if (!r && hipEventSynchronize(e1) != hipSuccess) r = fail(SPMV_ERR_HIP, "event sync");
    if (!r) hipEventElapsedTime(ms, e0, e1);
    return r;
  };
  for (int v = 0; v < SPMV_NUM_VARIANTS && !st; ++v) {
    if (v == SPMV_V6_SELL64 && !p.sell_ok) {
      p.at_us[v] = INFINITY;
      continue;
    }
    // V4 is timed in its three forms (plain, B staged per row block, B windows
    // per super-block); the fastest stays
    const int forms = v == SPMV_V4_LDS_BLOCK && p.nblocks > 0 && !p.v4_form_forced ? 3 : 1;
    const int form0 = p.v4_form;
    float form_med[3] = {INFINITY, INFINITY, INFINITY};
    for (int f = 0; f < forms && !st; ++f) {
      if (forms == 3) p.v4_form = f;
      st = launch_spmv(p, v, p.at_B, p.at_C, s);
      if (st) break;
      float ms[kReps];
      st = timed(v, &ms[0]);
      if (st) break;
      int reps = 1;
      if (ms[0] <= 1.5f * best) {
        for (; reps < kReps && !st; ++reps) st = timed(v, &ms[reps]);
        if (st) break;
      }
      std::sort(ms, ms + reps);
      form_med[f] = ms[reps / 2];
      best = std::min(best, form_med[f]);
    }
    if (st) break;
    p.v4_form = forms == 3 ? (int)(std::min_element(form_med, form_med + 3) - form_med) : form0;
    p.at_us[v] = 1000.0 * *std::min_element(form_med, form_med + 3);
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st) return st;
  p.have_autotune = true;
  p.variant = (int)(std::min_element(p.at_us, p.at_us + SPMV_NUM_VARIANTS) - p.at_us);
  return SPMV_OK;
}

// The selector's V6 output counts only for a plan with the V6 copy.
bool selector_output_usable(const Plan& p, int v) { return v != SPMV_V6_SELL64 || p.sell_ok; }

bool selector_confident(const Plan& p) {
  float best = INFINITY, second = INFINITY;
  for (int v = 0; v < SPMV_NUM_SELECTOR_OUTPUTS; ++v) {
    if (!selector_output_usable(p, v)) continue;
    if (p.pred[v] < best) {
      second = best;
      best = p.pred[v];
    } else if (p.pred[v] < second) {
      second = p.pred[v];
    }
  }
  if (second - best < g_sel.margin) return false;
  for (int q = 0; q < SPMV_NUM_FEATURES; ++q)
    if (p.features[q] < g_sel.lo[q] || p.features[q] > g_sel.hi[q]) return false;
  return true;
}

// The selector's pick: the smallest predicted time among the usable outputs
// (the first such output on ties).
int selector_pick(const Plan& p) {
  int b = -1;
  for (int v = 0; v < SPMV_NUM_SELECTOR_OUTPUTS; ++v)
    if (selector_output_usable(p, v) && (b < 0 || p.pred[v] < p.pred[b])) b = v;
  return b;
}

}  // namespace

void set_error(const std::string& msg) { g_err = msg; }
int fail(int status, const std::string& msg) {
  g_err = msg;
  return status;
}
int hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return SPMV_ERR_HIP;
}

}  // namespace spmv

using namespace spmv;

struct spmv_plan {
  Plan p;
};
struct spmv_batch {
  Batch b;
};
struct spmv_graph {
  hipGraphExec_t exec = nullptr;
};
struct spmv_split {
  Plan loc, rem;
};

extern "C" {

const char* spmv_version(void) { return "1.0.0"; }

const char* spmv_status_string(int status) {
  switch (status) {
    case SPMV_OK: return "ok";
    case SPMV_ERR_INVALID_ARG: return "invalid argument";
    case SPMV_ERR_BAD_CRS: return "malformed CRS arrays";
    case SPMV_ERR_UNSUPPORTED: return "unsupported size or dtype";
    case SPMV_ERR_WORKSPACE: return "workspace missing, too small or misaligned";
    case SPMV_ERR_HIP: return "HIP runtime error";
    case SPMV_ERR_STATE: return "invalid state";
    default: return "unknown status";
  }
}

const char* spmv_last_error(void) { return g_err.c_str(); }

int spmv_workspace_size(int64_t n_rows, int64_t n_cols, int64_t nnz, uint32_t flags,
                        size_t* bytes) {
  if (!bytes) return fail(SPMV_ERR_INVALID_ARG, "bytes is null");
  int st = check_shape(n_rows, n_cols, nnz);
  if (st) return st;
  *bytes = plan_layout(n_rows, n_cols, nnz, flags).total;
  return SPMV_OK;
}

namespace {
// Analyse a CRS matrix into `p` (the body of spmv_create; also used for the
// two parts of a split plan).
int plan_build(Plan& p, int64_t n_rows, int64_t n_cols, int64_t nnz, const int32_t* row_ptr,
               const int32_t* col_idx, const void* val, int val_dtype, void* workspace,
               size_t ws_bytes, uint32_t flags, hipStream_t s) {
  int st = check_shape(n_rows, n_cols, nnz);
  if (st) return st;
  if (!dtype_ok(val_dtype)) return fail(SPMV_ERR_INVALID_ARG, "val_dtype must be SPMV_F64 or SPMV_F32");
  if (!row_ptr) return fail(SPMV_ERR_INVALID_ARG, "row_ptr is null");
  if (nnz > 0 && (!col_idx || !val)) return fail(SPMV_ERR_INVALID_ARG, "col_idx or val is null");
  const uint32_t mode = flags & 0xFFu;
  const int fixed = (int)((flags >> 8) & 0xFu);
  if (mode > SPMV_SELECT_FIXED) return fail(SPMV_ERR_INVALID_ARG, "unknown selection mode");
  if (mode == SPMV_SELECT_FIXED && fixed >= SPMV_NUM_VARIANTS)
    return fail(SPMV_ERR_INVALID_ARG, "variant out of range");
  if (flags & ~(0xFFFu | SPMV_FLAG_SKIP_VALIDATE | SPMV_FLAG_SELL | SPMV_FLAG_V4_STAGE_ON |
                SPMV_FLAG_V4_STAGE_OFF | SPMV_FLAG_SELL_WIDE | SPMV_FLAG_V4_WINDOWS))
    return fail(SPMV_ERR_INVALID_ARG, "unknown flag bits");
  if ((flags & SPMV_FLAG_SELL_WIDE) && !(flags & SPMV_FLAG_SELL))
    return fail(SPMV_ERR_INVALID_ARG, "SPMV_FLAG_SELL_WIDE needs SPMV_FLAG_SELL");
  {
    const uint32_t fm = flags & (SPMV_FLAG_V4_STAGE_ON | SPMV_FLAG_V4_STAGE_OFF | SPMV_FLAG_V4_WINDOWS);
    if (fm & (fm - 1))
      return fail(SPMV_ERR_INVALID_ARG,
                  "at most one of SPMV_FLAG_V4_STAGE_ON, _STAGE_OFF and _WINDOWS");
  }
  if (mode == SPMV_SELECT_FIXED && fixed == SPMV_V6_SELL64 && !(flags & SPMV_FLAG_SELL))
    return fail(SPMV_ERR_INVALID_ARG, "variant V6 needs SPMV_FLAG_SELL");
  const PlanLayout L = plan_layout(n_rows, n_cols, nnz, flags);
  if (!workspace) return fail(SPMV_ERR_WORKSPACE, "workspace is null");
  if (reinterpret_cast<uintptr_t>(workspace) % 256)
    return fail(SPMV_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < L.total)
    return fail(SPMV_ERR_WORKSPACE, "workspace too small: need " + std::to_string(L.total) +
                                        " bytes, got " + std::to_string(ws_bytes));
  p.n_rows = n_rows;
  p.n_cols = n_cols;
  p.nnz = nnz;
  p.row_ptr = row_ptr;
  p.col_idx = col_idx;
  p.val = val;
  p.vdt = val_dtype;
  p.ws = static_cast<char*>(workspace);
  p.ws_bytes = ws_bytes;
  p.hdr = reinterpret_cast<WsHeader*>(p.ws + L.header);
  p.blocks = reinterpret_cast<int2*>(p.ws + L.blocks);
  p.spans = reinterpret_cast<int2*>(p.ws + L.spans);
  p.win = reinterpret_cast<int32_t*>(p.ws + L.win);
  p.nsb = super_block_count(n_rows);
  p.nblocks = lds_block_count(n_rows, nnz);
  p.bin_rows = reinterpret_cast<int32_t*>(p.ws + L.bins);
  p.stats_part = reinterpret_cast<unsigned long long*>(p.ws + L.stats);
  p.bin_base = reinterpret_cast<int32_t*>(p.ws + L.bin_base);
  if (L.at_B) {
    p.at_B = p.ws + L.at_B;
    p.at_C = reinterpret_cast<double*>(p.ws + L.at_C);
  }
  if (flags & SPMV_FLAG_SELL) {
    p.sell_reserved = true;
    p.sell_nch = sell_chunks(n_rows);
    p.sell_cap = sell_capacity(nnz);
    p.sell_width = reinterpret_cast<int32_t*>(p.ws + L.sell_width);
    p.sell_off = reinterpret_cast<int32_t*>(p.ws + L.sell_off);
    p.sell_partials = reinterpret_cast<int32_t*>(p.ws + L.sell_partials);
    p.sell_ci = reinterpret_cast<int32_t*>(p.ws + L.sell_ci);
    p.sell_val = p.ws + L.sell_val;
    p.sell_base = reinterpret_cast<int32_t*>(p.ws + L.sell_base);
    p.sell_dl = reinterpret_cast<uint16_t*>(p.ws + L.sell_dl);
    p.sell_flag = reinterpret_cast<int32_t*>(p.ws + L.sell_flag);
    p.sell_wide = (flags & SPMV_FLAG_SELL_WIDE) != 0;
  }
  hipGetDevice(&p.device);

  const float* theta = selector_theta_device();
  const bool run_mlp =
      theta && (mode == SPMV_SELECT_MLP || mode == SPMV_SELECT_DEFAULT) && g_sel.have_norm;
  WsHeader hh;
  st = launch_zero_header(p.hdr, s);
  if (!st && !(flags & SPMV_FLAG_SKIP_VALIDATE)) st = launch_validate(p, s);
  if (!st) st = launch_analysis(p, run_mlp ? g_sel.mu : nullptr, run_mlp ? g_sel.sigma : nullptr, s);
  if (!st) st = launch_win_build(p, s);
  if (!st && run_mlp)
    st = launch_mlp_forward(theta, p.hdr->x_std, 1, p.hdr->pred, p.hdr->z1, p.hdr->z2, s);
  if (!st && p.sell_reserved) st = launch_sell_build(p, s);
  if (!st) {
    hipError_t e = hipMemcpyAsync(&hh, p.hdr, sizeof(WsHeader), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) st = hip_fail(e, "analysis readback");
  }
  if (!st && hh.err) {
    std::string why;
    if (hh.err & 4) why += " row_ptr[0]!=0;";
    if (hh.err & 1) why += " row_ptr decreases;";
    if (hh.err & 8) why += " row_ptr[n_rows]!=nnz;";
    if (hh.err & 2) why += " col_idx out of [0,n_cols);";
    st = fail(SPMV_ERR_BAD_CRS, "invalid CRS:" + why);
  }
  if (st) return st;
  std::memcpy(p.features, hh.features, sizeof(p.features));
  p.staged_blocks = hh.staged_blocks;
  p.win_covered = (int64_t)hh.win_covered;
  p.v4_form_forced =
      (flags & (SPMV_FLAG_V4_STAGE_ON | SPMV_FLAG_V4_STAGE_OFF | SPMV_FLAG_V4_WINDOWS)) != 0;
  // without a flag: staging when a quarter of the row blocks fit exactly, else
  // windows when they hold at least 65% of the nonzeros and there are enough
  // super-blocks to fill the chip (permuted 3D stencil, 21.95M rows: 74%
  // through two windows in float64, 85% through three in float32, both
  // faster than the other forms; a 6M-row matrix of 7 diagonal pairs with
  // 54-60% stays faster plain; below 512 super-blocks the grid leaves CUs idle)
  p.v4_form = (flags & SPMV_FLAG_V4_STAGE_ON)    ? kV4Staged
              : (flags & SPMV_FLAG_V4_STAGE_OFF) ? kV4Plain
              : (flags & SPMV_FLAG_V4_WINDOWS)   ? kV4Window
              : p.staged_blocks * 4 >= p.nblocks ? kV4Staged
              : p.win_covered * 20 >= 13 * p.nnz && p.nnz > 0 && p.nsb >= 512 ? kV4Window
                                                                              : kV4Plain;
  for (int b = 0; b < kNumBins; ++b) {
    p.bin_count[b] = hh.bin_count[b];
    p.bin_offset[b] = hh.bin_offset[b];
  }
  if (run_mlp) {
    std::memcpy(p.pred, hh.pred, sizeof(p.pred));
    p.have_pred = true;
  }
  if (p.sell_reserved) {
    // the fill kernel reports the padded width sum even when it does not fit
    p.sell_slots = p.sell_nch > 0 ? 64 * hh.sell_total : 0;
    p.sell_ok = p.sell_slots >= 0 && p.sell_slots <= p.sell_cap;
    if (!p.sell_ok && mode == SPMV_SELECT_FIXED && fixed == SPMV_V6_SELL64)
      return fail(SPMV_ERR_UNSUPPORTED, "V6 copy needs " + std::to_string(p.sell_slots) +
                                            " slots, reserve is " + std::to_string(p.sell_cap));
  }
  if (mode == SPMV_SELECT_FIXED) {
    p.variant = fixed;
  } else if (mode == SPMV_SELECT_AUTOTUNE) {
    st = autotune(p, s);
  } else if (mode == SPMV_SELECT_MLP) {
    if (p.have_pred && selector_confident(p))
      p.variant = selector_pick(p);
    else
      st = autotune(p, s);
  } else {  // default
    // structure measured at create decides first: windows that hold most of
    // the nonzeros (a pattern scattered inside a few dense column regions,
    // of which the selector's label collection has no example: its network
    // ranks V2 first on the permuted 3D stencil, 2.1x slower there than the
    // window form) take V4 in that form, and a chunked copy that fits takes
    // V6 (the best variant on most label matrices that have one); the
    // network ranks the rest, V4 without weights
    if (p.v4_form == kV4Window)
      p.variant = SPMV_V4_LDS_BLOCK;
    else if (p.sell_ok)
      p.variant = SPMV_V6_SELL64;
    else
      p.variant = p.have_pred ? selector_pick(p) : SPMV_V4_LDS_BLOCK;
  }
  return st;
}
}  // namespace

int spmv_create(spmv_handle* h, int64_t n_rows, int64_t n_cols, int64_t nnz,
                const int32_t* row_ptr, const int32_t* col_idx, const void* val, int val_dtype,
                void* workspace, size_t ws_bytes, uint32_t flags, void* stream) {
  if (!h) return fail(SPMV_ERR_INVALID_ARG, "handle pointer is null");
  *h = nullptr;
  auto* H = new (std::nothrow) spmv_plan;
  if (!H) return fail(SPMV_ERR_INVALID_ARG, "host allocation failed");
  const int st = plan_build(H->p, n_rows, n_cols, nnz, row_ptr, col_idx, val, val_dtype,
                            workspace, ws_bytes, flags, as_stream(stream));
  if (st) {
    delete H;
    return st;
  }
  *h = H;
  return SPMV_OK;
}

int spmv_apply(spmv_handle h, const void* B, int b_dtype, double* C, void* stream) {
  if (!h) return fail(SPMV_ERR_INVALID_ARG, "handle is null");
  const Plan& p = h->p;
  if (b_dtype != p.vdt) return fail(SPMV_ERR_UNSUPPORTED, "b_dtype must equal the plan's val_dtype");
  if ((!B && p.n_cols > 0 && p.nnz > 0) || (!C && p.n_rows > 0))
    return fail(SPMV_ERR_INVALID_ARG, "B or C is null");
  return launch_spmv(p, p.variant, B, C, as_stream(stream));
}

int spmm_apply(spmv_handle h, int32_t k, const void* B, int64_t ldb, int b_dtype, double* C,
               int64_t ldc, void* stream) {
  if (!h) return fail(SPMV_ERR_INVALID_ARG, "handle is null");
  const Plan& p = h->p;
  if (k < 1) return fail(SPMV_ERR_INVALID_ARG, "k must be >= 1");
  if (ldb < k || ldc < k) return fail(SPMV_ERR_INVALID_ARG, "ldb and ldc must be >= k");
  if (b_dtype != p.vdt) return fail(SPMV_ERR_UNSUPPORTED, "b_dtype must equal the plan's val_dtype");
  if ((!B && p.n_cols > 0 && p.nnz > 0) || (!C && p.n_rows > 0))
    return fail(SPMV_ERR_INVALID_ARG, "B or C is null");
  if ((int64_t)p.n_rows * ldc > INT64_MAX / 2) return fail(SPMV_ERR_UNSUPPORTED, "C too large");
  // one contiguous right-hand side is the single product, in the plan's own
  // variant and form (Hamiltonian-like matrix, 6M rows, from the V6 copy:
  // 160 us against 216 us through the one-column block kernel), except on a
  // V6 plan with short rows, where the row-group kernel below is faster
  // (256x256 Laplacian, graph-replayed: 2.40 against 2.80 us)
  const bool short_v6 = p.variant == SPMV_V6_SELL64 && p.nnz < 8 * p.n_rows;
  if (k == 1 && ldb == 1 && ldc == 1 && !short_v6)
    return launch_spmv(p, p.variant, B, C, as_stream(stream));
  // a plan running V6 multiplies up to 8 right-hand sides from its chunked copy
  // (one pass over it) when its rows average at least 8 entries; wider blocks
  // use the row-group kernel, which reads the matrix once for any k, and so
  // do short rows, where its lane groups keep more rows in flight than one
  // lane per row (5-point Laplacians, 262k and 1M rows: the copy took 1.1-1.3x
  // as long at k = 4 and 1.5-1.8x at k = 8; a 15-entry-per-row matrix ran
  // 1.1-2x faster from the copy)
  // (lane groups per row, one 16-byte B vector per lane: k = 8, 16, 32
  // in float64, 8 .. 64 in float32, aligned operands)
  if (p.variant == SPMV_V6_SELL64 && p.sell_ok && p.nnz >= 8 * p.n_rows &&
      (k <= 8 || sell_spmm_lanes_fit(p, k, B, ldb, C, ldc)))
    return launch_sell_spmm(p, k, B, ldb, C, ldc, as_stream(stream));
  return launch_spmm(p, k, B, ldb, C, ldc, as_stream(stream));
}

int spmv_get_variant(spmv_handle h, int* variant) {
  if (!h || !variant) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  *variant = h->p.variant;
  return SPMV_OK;
}

int spmv_set_variant(spmv_handle h, int variant) {
  if (!h) return fail(SPMV_ERR_INVALID_ARG, "handle is null");
  if (variant < 0 || variant >= SPMV_NUM_VARIANTS) return fail(SPMV_ERR_INVALID_ARG, "variant out of range");
  if (variant == SPMV_V6_SELL64 && !h->p.sell_ok)
    return fail(SPMV_ERR_STATE, "this plan has no V6 copy");
  h->p.variant = variant;
  return SPMV_OK;
}

int spmv_get_features(spmv_handle h, double* f) {
  if (!h || !f) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  std::memcpy(f, h->p.features, sizeof(h->p.features));
  return SPMV_OK;
}

int spmv_get_predictions(spmv_handle h, float* pred) {
  if (!h || !pred) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  if (!h->p.have_pred) return fail(SPMV_ERR_STATE, "the selector did not run for this plan");
  std::memcpy(pred, h->p.pred, sizeof(h->p.pred));
  return SPMV_OK;
}

int spmv_get_autotune_times(spmv_handle h, double* us) {
  if (!h || !us) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  if (!h->p.have_autotune) return fail(SPMV_ERR_STATE, "autotune did not run for this plan");
  std::memcpy(us, h->p.at_us, sizeof(h->p.at_us));
  return SPMV_OK;
}

int spmv_get_v4_staged(spmv_handle h, int* staged) {
  if (!h || !staged) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  *staged = h->p.v4_form == kV4Staged ? 1 : 0;
  return SPMV_OK;
}

int spmv_get_v4_form(spmv_handle h, int* form, int64_t* win_covered) {
  if (!h || !form) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  *form = h->p.v4_form;
  if (win_covered) *win_covered = h->p.win_covered;
  return SPMV_OK;
}

int spmv_set_v4_form(spmv_handle h, int form) {
  if (!h) return fail(SPMV_ERR_INVALID_ARG, "handle is null");
  if (form < SPMV_V4_PLAIN || form > SPMV_V4_WINDOWS)
    return fail(SPMV_ERR_INVALID_ARG, "unknown V4 form");
  h->p.v4_form = form;
  return SPMV_OK;
}

int spmv_get_sell_slots(spmv_handle h, int64_t* slots) {
  if (!h || !slots) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  if (!h->p.sell_ok) return fail(SPMV_ERR_STATE, "this plan has no V6 copy");
  *slots = h->p.sell_slots;
  return SPMV_OK;
}

int spmv_get_sell_stream_bytes(spmv_handle h, int64_t* bytes) {
  if (!h || !bytes) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  const Plan& p = h->p;
  if (!p.sell_ok) return fail(SPMV_ERR_STATE, "this plan has no V6 copy");
  const int64_t nch = p.sell_nch;
  const int64_t sv = p.vdt == SPMV_F64 ? 8 : 4;
  int64_t total = 0;
  if (nch > 0) {
    std::vector<int32_t> w((size_t)nch), f((size_t)nch, 0);
    SPMV_HIP(hipMemcpy(w.data(), p.sell_width, sizeof(int32_t) * (size_t)nch,
                       hipMemcpyDeviceToHost));
    if (!p.sell_wide)
      SPMV_HIP(hipMemcpy(f.data(), p.sell_flag, sizeof(int32_t) * (size_t)nch,
                         hipMemcpyDeviceToHost));
    for (int64_t k = 0; k < nch; ++k) {
      const int64_t slots = 64 * (int64_t)w[k];
      const int64_t col = f[k] == 8 ? 1 : f[k] == 16 ? 2 : 4;
      // chunk offset and delta flag, the slot bases (delta chunks), then per
      // slot its value and its column (delta or index)
      total += 8 + (f[k] ? 4 * (int64_t)w[k] : 0) + slots * (sv + col);
    }
  }
  *bytes = total;
  return SPMV_OK;
}

int spmv_get_sell_deltas(spmv_handle h, int64_t* chunks8, int64_t* chunks16, int64_t* chunks) {
  if (!h || !chunks8 || !chunks16 || !chunks) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  if (!h->p.sell_ok) return fail(SPMV_ERR_STATE, "this plan has no V6 copy");
  const int64_t nch = h->p.sell_nch;
  int64_t n8 = 0, n16 = 0;
  if (nch > 0 && !h->p.sell_wide) {
    std::vector<int32_t> f((size_t)nch);
    SPMV_HIP(hipMemcpy(f.data(), h->p.sell_flag, sizeof(int32_t) * (size_t)nch,
                       hipMemcpyDeviceToHost));
    for (int32_t x : f) {
      n8 += x == 8;
      n16 += x == 16;
    }
  }
  *chunks8 = n8;
  *chunks16 = n16;
  *chunks = nch;
  return SPMV_OK;
}

int spmv_get_num_blocks(spmv_handle h, int64_t* nblocks) {
  if (!h || !nblocks) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  *nblocks = h->p.nblocks;
  return SPMV_OK;
}

int spmv_destroy(spmv_handle h) {
  delete h;
  return SPMV_OK;
}

// ------------------------------------------------------------------ batch

namespace {
struct BatchLayout {
  size_t err = 0, tiles = 0, deltas = 0, toff = 0, nr = 0, nc = 0, nz = 0, total = 0;
};
BatchLayout batch_layout(int32_t count, int64_t max_tiles) {
  BatchLayout L;
  size_t o = 0;
  L.err = o;
  o += 256 + align256(sizeof(unsigned int) * kBatchCounterWords);  // err[2], then the counters
  L.tiles = o;
  o += align256(sizeof(int32_t) * kTileInts * (size_t)std::max<int64_t>(max_tiles, 1));
  L.deltas = o;
  o += align256((size_t)2 * kBlockBudget * (size_t)std::max<int64_t>(max_tiles, 1));
  L.toff = o;
  o += align256(sizeof(int64_t) * (size_t)(count + 1));
  L.nr = o;
  o += align256(sizeof(int64_t) * (size_t)count);
  L.nc = o;
  o += align256(sizeof(int64_t) * (size_t)count);
  L.nz = o;
  o += align256(sizeof(int64_t) * (size_t)count);
  L.total = o;
  return L;
}
__global__ void k_batch_err_init(int32_t* e) {
  e[0] = 0;
  e[1] = INT32_MAX;
}
}  // namespace

int spmv_batch_workspace_size(int32_t count, int64_t total_rows, int64_t total_nnz,
                              size_t* bytes) {
  if (!bytes) return fail(SPMV_ERR_INVALID_ARG, "bytes is null");
  if (count < 1 || total_rows < 0 || total_nnz < 0)
    return fail(SPMV_ERR_INVALID_ARG, "count must be >= 1 and totals >= 0");
  const int64_t max_tiles = (total_nnz + total_rows) / kBlockBudget + count;
  *bytes = batch_layout(count, max_tiles).total;
  return SPMV_OK;
}

int spmv_batch_create(spmv_batch_handle* h, int32_t count, const int64_t* n_rows,
                      const int64_t* n_cols, const int64_t* nnz, const int32_t* const* row_ptrs,
                      const int32_t* const* col_idxs, const void* const* vals, int val_dtype,
                      void* workspace, size_t ws_bytes, void* stream) {
  if (!h) return fail(SPMV_ERR_INVALID_ARG, "handle pointer is null");
  *h = nullptr;
  if (count < 1 || !n_rows || !n_cols || !nnz || !row_ptrs || !col_idxs || !vals)
    return fail(SPMV_ERR_INVALID_ARG, "null array or count < 1");
  if (!dtype_ok(val_dtype)) return fail(SPMV_ERR_INVALID_ARG, "bad val_dtype");
  std::vector<int64_t> toff((size_t)count + 1, 0);
  for (int32_t m = 0; m < count; ++m) {
    int st = check_shape(n_rows[m], n_cols[m], nnz[m]);
    if (st) return fail(st, "matrix " + std::to_string(m) + ": " + spmv_last_error());
    toff[m + 1] = toff[m] + lds_block_count(n_rows[m], nnz[m]);
  }
  const int64_t ntiles = toff[count];
  if (ntiles > INT32_MAX) return fail(SPMV_ERR_UNSUPPORTED, "too many tiles");
  const BatchLayout L = batch_layout(count, ntiles);
  if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 256)
    return fail(SPMV_ERR_WORKSPACE, "workspace null or not 256-byte aligned");
  if (ws_bytes < L.total)
    return fail(SPMV_ERR_WORKSPACE, "workspace too small: need " + std::to_string(L.total));
  hipStream_t s = as_stream(stream);
  char* ws = static_cast<char*>(workspace);
  auto* H = new (std::nothrow) spmv_batch;
  if (!H) return fail(SPMV_ERR_INVALID_ARG, "host allocation failed");
  Batch& b = H->b;
  b.count = count;
  b.vdt = val_dtype;
  b.row_ptrs = row_ptrs;
  b.col_idxs = col_idxs;
  b.vals = vals;
  b.tiles = reinterpret_cast<int32_t*>(ws + L.tiles);
  b.deltas = reinterpret_cast<uint8_t*>(ws + L.deltas);
  b.ntiles = ntiles;
  b.err = reinterpret_cast<int32_t*>(ws + L.err);
  b.counters = reinterpret_cast<unsigned int*>(ws + L.err + 256);
  int dev = 0;
  hipGetDevice(&dev);
  if (int st0 = batch_grids(dev, val_dtype, &b.grid_static, &b.grid_dynamic)) {
    delete H;
    return st0;
  }
  b.tile_offset_host = new int64_t[(size_t)count + 1];
  std::memcpy(b.tile_offset_host, toff.data(), sizeof(int64_t) * ((size_t)count + 1));
  b.rp_host = new const int32_t*[(size_t)count];
  b.ci_host = new const int32_t*[(size_t)count];
  b.val_host = new const void*[(size_t)count];
  int64_t* d_toff = reinterpret_cast<int64_t*>(ws + L.toff);
  int64_t* d_nr = reinterpret_cast<int64_t*>(ws + L.nr);
  int64_t* d_nc = reinterpret_cast<int64_t*>(ws + L.nc);
  int64_t* d_nz = reinterpret_cast<int64_t*>(ws + L.nz);
  int st = SPMV_OK;
  hipError_t e = hipMemcpyAsync(d_toff, toff.data(), sizeof(int64_t) * (count + 1),
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_nr, n_rows, sizeof(int64_t) * count, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_nc, n_cols, sizeof(int64_t) * count, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_nz, nnz, sizeof(int64_t) * count, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) st = hip_fail(e, "batch upload");
  if (!st) {
    k_batch_err_init<<<1, 1, 0, s>>>(b.err);
    e = hipGetLastError();
    if (e != hipSuccess) st = hip_fail(e, "batch init");
  }
  if (!st) st = launch_batch_build(b, d_toff, d_nr, d_nc, d_nz, s);
  if (!st) st = launch_counters_init(b.counters, s);
  int32_t herr[2] = {0, 0};
  if (!st) {
    e = hipMemcpyAsync(herr, b.err, sizeof(herr), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(b.rp_host, row_ptrs, sizeof(void*) * count, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(b.ci_host, col_idxs, sizeof(void*) * count, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(b.val_host, vals, sizeof(void*) * count, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) st = hip_fail(e, "batch readback");
  }
  if (!st && herr[0])
    st = fail(SPMV_ERR_BAD_CRS, "invalid CRS in batch matrix " + std::to_string(herr[1]));
  if (st) {
    spmv_batch_destroy(H);
    return st;
  }
  *h = H;
  return SPMV_OK;
}

int spmv_batch_apply(spmv_batch_handle h, const void* const* Bs, double* const* Cs,
                     int b_dtype, void* stream) {
  if (!h || !Bs || !Cs) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  if (b_dtype != h->b.vdt) return fail(SPMV_ERR_UNSUPPORTED, "b_dtype must equal val_dtype");
  return launch_batch_apply(h->b, 0, h->b.ntiles, Bs, Cs, nullptr, nullptr, as_stream(stream));
}

int spmv_batch_apply_each(spmv_batch_handle h, const void* const* Bs_host,
                          double* const* Cs_host, int b_dtype, void* stream) {
  if (!h || !Bs_host || !Cs_host) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  const Batch& b = h->b;
  if (b_dtype != b.vdt) return fail(SPMV_ERR_UNSUPPORTED, "b_dtype must equal val_dtype");
  for (int32_t m = 0; m < b.count; ++m) {
    int st = launch_batch_apply(b, b.tile_offset_host[m], b.tile_offset_host[m + 1], nullptr,
                                nullptr, Bs_host[m], Cs_host[m], as_stream(stream));
    if (st) return st;
  }
  return SPMV_OK;
}

int spmv_batch_set_mode(spmv_batch_handle h, int mode) {
  if (!h) return fail(SPMV_ERR_INVALID_ARG, "handle is null");
  if (mode < SPMV_BATCH_DYNAMIC || mode > SPMV_BATCH_TILE_GRID)
    return fail(SPMV_ERR_INVALID_ARG, "unknown batch mode");
  h->b.mode = mode;
  return SPMV_OK;
}

int spmv_batch_get_num_tiles(spmv_batch_handle h, int64_t* ntiles) {
  if (!h || !ntiles) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  *ntiles = h->b.ntiles;
  return SPMV_OK;
}

int spmv_batch_get_stream_bytes(spmv_batch_handle h, int64_t* bytes) {
  if (!h || !bytes) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  const Batch& b = h->b;
  const int64_t sv = b.vdt == SPMV_F64 ? 8 : 4;
  int64_t total = 0;
  if (b.ntiles > 0) {
    std::vector<int32_t> t((size_t)(kTileInts * b.ntiles));
    SPMV_HIP(hipMemcpy(t.data(), b.tiles, sizeof(int32_t) * t.size(), hipMemcpyDeviceToHost));
    for (int64_t k = 0; k < b.ntiles; ++k) {
      const int32_t* tl = t.data() + kTileInts * k;
      const int64_t n = (int64_t)tl[4] - tl[3];
      if (tl[2] <= tl[1] || n < 0) continue;
      const int64_t in = n < kBlockBudget ? n : kBlockBudget;
      const int64_t col = tl[7] == 8 ? 1 : tl[7] == 16 ? 2 : 4;
      // the tile record, the values, the chunk's columns (as deltas where the
      // tile has them) and a long last row's columns past the chunk
      total += 4 * kTileInts + n * sv + in * col + (n - in) * 4;
    }
  }
  *bytes = total;
  return SPMV_OK;
}

int spmv_batch_destroy(spmv_batch_handle h) {
  if (!h) return SPMV_OK;
  delete[] h->b.tile_offset_host;
  delete[] h->b.rp_host;
  delete[] h->b.ci_host;
  delete[] h->b.val_host;
  delete h;
  return SPMV_OK;
}

// ---------------------------------------------------------------- solvers

int spmv_cg_workspace_size(int64_t n, size_t* bytes) {
  if (!bytes || n < 0) return fail(SPMV_ERR_INVALID_ARG, "bad argument");
  *bytes = cg_workspace_bytes(n);
  return SPMV_OK;
}

int spmv_cg_solve(spmv_handle h, const double* b, double* x, double tol, int32_t maxit,
                  int32_t check_every, int32_t use_graph, void* workspace, size_t ws_bytes,
                  int32_t* iters, double* relres, void* stream) {
  if (!h || !iters || !relres) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  const Plan& P = h->p;
  if (P.n_rows != P.n_cols) return fail(SPMV_ERR_INVALID_ARG, "CG needs a square matrix");
  if (P.n_rows > 0 && (!b || !x)) return fail(SPMV_ERR_INVALID_ARG, "b or x is null");
  if (!(tol >= 0.0) || maxit < 0) return fail(SPMV_ERR_INVALID_ARG, "tol >= 0 and maxit >= 0");
  if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 256 ||
      ws_bytes < cg_workspace_bytes(P.n_rows))
    return fail(SPMV_ERR_WORKSPACE, "solver workspace missing, misaligned or too small");
  int it = 0;
  double rr = 0.0;
  const int st = run_cg(P, b, x, tol, maxit, check_every, use_graph != 0, workspace, &it, &rr,
                        as_stream(stream));
  *iters = it;
  *relres = rr;
  return st;
}

}  // extern "C"

// ---- CG with library-held scratch, for callers that cannot allocate
//
// `scratch` is one file-scope device array; every GPU the library runs on
// holds its own copy (at its own address) until the process ends. In host
// code the array's name is a host-side stand-in, not a device address: its
// device address is looked up once per device, with that device current,
// and only that pointer is handed to kernels.
namespace {
constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
int scratch_device_ptr(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices)
    return fail(SPMV_ERR_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(SPMV_ERR_HIP, "hipGetSymbolAddress(scratch) returned null");
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return SPMV_OK;
}
}  // namespace

extern "C" {

int spmv_cg_solve_noalloc(spmv_handle h, const double* b, double* x, double tol, int32_t maxit,
                          int32_t check_every, int32_t* iters, double* relres, void* stream) {
  if (!h || !iters || !relres) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  const Plan& P = h->p;
  if (P.n_rows != P.n_cols) return fail(SPMV_ERR_INVALID_ARG, "CG needs a square matrix");
  if (P.n_rows > 0 && (!b || !x)) return fail(SPMV_ERR_INVALID_ARG, "b or x is null");
  if (!(tol >= 0.0) || maxit < 0) return fail(SPMV_ERR_INVALID_ARG, "tol >= 0 and maxit >= 0");
  const size_t need = cg_workspace_bytes(P.n_rows);
  if (need > kNoAllocScratchBytes)
    return fail(SPMV_ERR_UNSUPPORTED,
                "n = " + std::to_string(P.n_rows) + " needs " + std::to_string(need) +
                    " bytes of solver scratch; the library holds " +
                    std::to_string(kNoAllocScratchBytes) + " (n <= 931680)");
  int dev = 0;
  SPMV_HIP(hipGetDevice(&dev));
  if (dev != P.device) return fail(SPMV_ERR_STATE, "the plan's device must be current");
  void* ws = nullptr;
  int st = scratch_device_ptr(dev, &ws);
  if (st) return st;
  int it = 0;
  double rr = 0.0;
  st = run_cg(P, b, x, tol, maxit, check_every, false, ws, &it, &rr, as_stream(stream));
  *iters = it;
  *relres = rr;
  return st;
}

int spmv_lanczos_workspace_size(int64_t n, int32_t k, size_t* bytes) {
  if (!bytes || n < 0 || k < 1) return fail(SPMV_ERR_INVALID_ARG, "bad argument");
  *bytes = lanczos_workspace_bytes(n, k);
  return SPMV_OK;
}

int spmv_lanczos(spmv_handle h, const double* v0, int32_t k, double* alpha, double* beta,
                 void* workspace, size_t ws_bytes, void* stream) {
  if (!h || !v0 || !alpha || !beta) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  const Plan& P = h->p;
  if (P.n_rows != P.n_cols || P.n_rows < 1)
    return fail(SPMV_ERR_INVALID_ARG, "Lanczos needs a non-empty square matrix");
  if (k < 1) return fail(SPMV_ERR_INVALID_ARG, "k >= 1");
  if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 256 ||
      ws_bytes < lanczos_workspace_bytes(P.n_rows, k))
    return fail(SPMV_ERR_WORKSPACE, "solver workspace missing, misaligned or too small");
  return run_lanczos(P, v0, k, alpha, beta, workspace, as_stream(stream));
}

// ------------------------------------------------------------------ split

namespace {
struct SplitLayout {
  size_t len_loc = 0, len_rem = 0, rp_loc = 0, rp_rem = 0, partials = 0, ci = 0, val = 0,
         ws_loc = 0, ws_rem = 0, total = 0;
  size_t plan_bytes = 0;
};
SplitLayout split_layout(int64_t n, int64_t n_cols, int64_t nnz) {
  SplitLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align256(bytes);
    return at;
  };
  const size_t n1 = (size_t)std::max<int64_t>(n, 1);
  L.len_loc = take(4 * n1);
  L.len_rem = take(4 * n1);
  L.rp_loc = take(4 * (n1 + 1));
  L.rp_rem = take(4 * (n1 + 1));
  L.partials = take(4 * (size_t)scan_partials_count(n + 1));
  L.ci = take(4 * (size_t)std::max<int64_t>(nnz, 1));
  L.val = take(8 * (size_t)std::max<int64_t>(nnz, 1));
  L.plan_bytes = plan_layout(n, n_cols, nnz, SPMV_FLAG_VARIANT(SPMV_V4_LDS_BLOCK)).total;
  L.ws_loc = take(L.plan_bytes);
  L.ws_rem = take(L.plan_bytes);
  L.total = o;
  return L;
}
}  // namespace

int spmv_split_workspace_size(int64_t n_rows, int64_t n_cols, int64_t nnz, size_t* bytes) {
  if (!bytes) return fail(SPMV_ERR_INVALID_ARG, "bytes is null");
  int st = check_shape(n_rows, n_cols, nnz);
  if (st) return st;
  *bytes = split_layout(n_rows, n_cols, nnz).total;
  return SPMV_OK;
}

int spmv_split_create(spmv_split_handle* h, int64_t n_rows, int64_t n_cols, int64_t nnz,
                      const int32_t* row_ptr, const int32_t* col_idx, const void* val,
                      int val_dtype, int64_t col_lo, int64_t col_hi, void* workspace,
                      size_t ws_bytes, void* stream) {
  if (!h) return fail(SPMV_ERR_INVALID_ARG, "handle pointer is null");
  *h = nullptr;
  int st = check_shape(n_rows, n_cols, nnz);
  if (st) return st;
  if (!dtype_ok(val_dtype)) return fail(SPMV_ERR_INVALID_ARG, "bad val_dtype");
  if (!row_ptr || (nnz > 0 && (!col_idx || !val)))
    return fail(SPMV_ERR_INVALID_ARG, "null CRS array");
  if (col_lo < 0 || col_hi < col_lo || col_hi > n_cols)
    return fail(SPMV_ERR_INVALID_ARG, "need 0 <= col_lo <= col_hi <= n_cols");
  const SplitLayout L = split_layout(n_rows, n_cols, nnz);
  if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 256)
    return fail(SPMV_ERR_WORKSPACE, "workspace null or not 256-byte aligned");
  if (ws_bytes < L.total)
    return fail(SPMV_ERR_WORKSPACE, "workspace too small: need " + std::to_string(L.total));
  hipStream_t s = as_stream(stream);
  char* ws = static_cast<char*>(workspace);
  auto* H = new (std::nothrow) spmv_split;
  if (!H) return fail(SPMV_ERR_INVALID_ARG, "host allocation failed");
  // validate the input once, through the local plan's header
  Plan& v = H->loc;
  v.n_rows = n_rows;
  v.n_cols = n_cols;
  v.nnz = nnz;
  v.row_ptr = row_ptr;
  v.col_idx = col_idx;
  v.hdr = reinterpret_cast<WsHeader*>(ws + L.ws_loc);
  int32_t herr = 0;
  st = launch_zero_header(v.hdr, s);
  if (!st) st = launch_validate(v, s);
  if (!st) {
    hipError_t e = hipMemcpyAsync(&herr, &v.hdr->err, sizeof(herr), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) st = hip_fail(e, "split validation readback");
  }
  if (!st && herr) st = fail(SPMV_ERR_BAD_CRS, "invalid CRS");
  int32_t* len_loc = reinterpret_cast<int32_t*>(ws + L.len_loc);
  int32_t* len_rem = reinterpret_cast<int32_t*>(ws + L.len_rem);
  int32_t* rp_loc = reinterpret_cast<int32_t*>(ws + L.rp_loc);
  int32_t* rp_rem = reinterpret_cast<int32_t*>(ws + L.rp_rem);
  int32_t* partials = reinterpret_cast<int32_t*>(ws + L.partials);
  int32_t tot[2] = {0, 0};
  if (!st) st = launch_split_count(n_rows, row_ptr, col_idx, col_lo, col_hi, len_loc, len_rem, s);
  if (!st) st = launch_exclusive_scan(len_loc, rp_loc, n_rows, partials, s);
  if (!st) st = launch_exclusive_scan(len_rem, rp_rem, n_rows, partials, s);
  if (!st) {
    hipError_t e = hipMemcpyAsync(&tot[0], rp_loc + n_rows, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&tot[1], rp_rem + n_rows, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) st = hip_fail(e, "split size readback");
  }
  if (!st && (int64_t)tot[0] + tot[1] != nnz) st = fail(SPMV_ERR_BAD_CRS, "split sizes disagree");
  const int vb = dtype_bytes(val_dtype);
  int32_t* ci_loc = reinterpret_cast<int32_t*>(ws + L.ci);
  int32_t* ci_rem = ci_loc + tot[0];
  char* val_loc = ws + L.val;
  char* val_rem = val_loc + (size_t)vb * tot[0];
  if (!st)
    st = launch_split_fill(n_rows, row_ptr, col_idx, val, val_dtype, col_lo, col_hi, rp_loc,
                           rp_rem, ci_loc, val_loc, ci_rem, val_rem, s);
  const uint32_t fl = SPMV_FLAG_VARIANT(SPMV_V4_LDS_BLOCK) | SPMV_FLAG_SKIP_VALIDATE;
  if (!st)
    st = plan_build(H->loc, n_rows, n_cols, tot[0], rp_loc, ci_loc, val_loc, val_dtype,
                    ws + L.ws_loc, L.plan_bytes, fl, s);
  if (!st)
    st = plan_build(H->rem, n_rows, n_cols, tot[1], rp_rem, ci_rem, val_rem, val_dtype,
                    ws + L.ws_rem, L.plan_bytes, fl, s);
  if (st) {
    delete H;
    return st;
  }
  *h = H;
  return SPMV_OK;
}

int spmv_split_apply(spmv_split_handle h, int pass, const void* B, int b_dtype, double* C,
                     void* stream) {
  if (!h) return fail(SPMV_ERR_INVALID_ARG, "handle is null");
  if (pass < -1 || pass > 1) return fail(SPMV_ERR_INVALID_ARG, "pass must be -1, 0 or 1");
  if (b_dtype != h->loc.vdt) return fail(SPMV_ERR_UNSUPPORTED, "b_dtype must equal val_dtype");
  if ((!B && h->loc.n_cols > 0) || (!C && h->loc.n_rows > 0))
    return fail(SPMV_ERR_INVALID_ARG, "B or C is null");
  hipStream_t s = as_stream(stream);
  int st = SPMV_OK;
  if (pass <= 0) st = launch_spmv(h->loc, SPMV_V4_LDS_BLOCK, B, C, s);
  if (!st && pass != 0) st = launch_spmv_accumulate(h->rem, B, C, s);
  return st;
}

int spmv_split_get_nnz(spmv_split_handle h, int64_t* nnz_local, int64_t* nnz_remote) {
  if (!h || !nnz_local || !nnz_remote) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  *nnz_local = h->loc.nnz;
  *nnz_remote = h->rem.nnz;
  return SPMV_OK;
}

int spmv_split_destroy(spmv_split_handle h) {
  delete h;
  return SPMV_OK;
}

// ------------------------------------------------------------------ graphs

int spmv_graph_begin(void* stream) {
  if (!stream) return fail(SPMV_ERR_INVALID_ARG, "graph capture needs a non-null stream");
  SPMV_HIP(hipStreamBeginCapture(as_stream(stream), hipStreamCaptureModeThreadLocal));
  return SPMV_OK;
}

int spmv_graph_end(void* stream, spmv_graph_handle* g) {
  if (!stream || !g) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  *g = nullptr;
  hipGraph_t graph = nullptr;
  SPMV_HIP(hipStreamEndCapture(as_stream(stream), &graph));
  hipGraphExec_t exec = nullptr;
  hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  auto* G = new (std::nothrow) spmv_graph;
  if (!G) {
    hipGraphExecDestroy(exec);
    return fail(SPMV_ERR_INVALID_ARG, "host allocation failed");
  }
  G->exec = exec;
  *g = G;
  return SPMV_OK;
}

int spmv_graph_launch(spmv_graph_handle g, void* stream) {
  if (!g) return fail(SPMV_ERR_INVALID_ARG, "graph is null");
  SPMV_HIP(hipGraphLaunch(g->exec, as_stream(stream)));
  return SPMV_OK;
}

int spmv_graph_destroy(spmv_graph_handle g) {
  if (!g) return SPMV_OK;
  hipGraphExecDestroy(g->exec);
  delete g;
  return SPMV_OK;
}

// ---------------------------------------------------------------- selector

int spmv_selector_load(const float* params, const float* mu, const float* sigma,
                       const float* lo, const float* hi, float margin) {
  if (!params || !mu || !sigma || !lo || !hi) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  for (int q = 0; q < SPMV_NUM_FEATURES; ++q)
    if (!(sigma[q] > 0.0f) || !std::isfinite(mu[q]) || lo[q] > hi[q])
      return fail(SPMV_ERR_INVALID_ARG, "bad standardisation or range");
  for (int i = 0; i < SPMV_MLP_PARAMS; ++i)
    if (!std::isfinite(params[i])) return fail(SPMV_ERR_INVALID_ARG, "non-finite weight");
  int st = selector_upload(params);
  if (st) return st;
  std::memcpy(g_sel.mu, mu, sizeof(g_sel.mu));
  std::memcpy(g_sel.sigma, sigma, sizeof(g_sel.sigma));
  std::memcpy(g_sel.lo, lo, sizeof(g_sel.lo));
  std::memcpy(g_sel.hi, hi, sizeof(g_sel.hi));
  g_sel.margin = margin;
  g_sel.have_norm = true;
  return SPMV_OK;
}

int spmv_selector_load_file(const char* path) {
  if (!path) return fail(SPMV_ERR_INVALID_ARG, "path is null");
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(SPMV_ERR_INVALID_ARG, std::string("cannot open ") + path);
  constexpr size_t kFloats = SPMV_MLP_PARAMS + 4 * SPMV_NUM_FEATURES + 1;
  char magic[8];
  std::vector<float> buf(kFloats + 1);
  const size_t m = std::fread(magic, 1, 8, f);
  const size_t n = std::fread(buf.data(), sizeof(float), kFloats + 1, f);
  std::fclose(f);
  if (m != 8 || std::memcmp(magic, "SPMVSEL2", 8) != 0 || n != kFloats)
    return fail(SPMV_ERR_INVALID_ARG, std::string("malformed selector file ") + path);
  const float* p = buf.data();
  const float* mu = p + SPMV_MLP_PARAMS;
  const float* sd = mu + SPMV_NUM_FEATURES;
  const float* lo = sd + SPMV_NUM_FEATURES;
  const float* hi = lo + SPMV_NUM_FEATURES;
  return spmv_selector_load(p, mu, sd, lo, hi, hi[SPMV_NUM_FEATURES]);
}

int spmv_selector_loaded(int* loaded) {
  if (!loaded) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  *loaded = (selector_theta_device() != nullptr && g_sel.have_norm) ? 1 : 0;
  return SPMV_OK;
}

int spmv_mlp_forward(const float* theta, const float* X, int32_t nb, float* Y, float* Z1,
                     float* Z2, void* stream) {
  if (nb < 0) return fail(SPMV_ERR_INVALID_ARG, "nb < 0");
  if (nb > 0 && (!theta || !X || !Y || !Z1 || !Z2)) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  return launch_mlp_forward(theta, X, nb, Y, Z1, Z2, as_stream(stream));
}

int spmv_mlp_backward(const float* theta, const float* X, const float* Z1, const float* Z2,
                      const float* Y, const float* T, int32_t nb, float* dz_scratch,
                      float* grad, void* stream) {
  if (nb < 0) return fail(SPMV_ERR_INVALID_ARG, "nb < 0");
  if (nb > 0 && (!theta || !X || !Z1 || !Z2 || !Y || !T || !dz_scratch || !grad))
    return fail(SPMV_ERR_INVALID_ARG, "null argument");
  return launch_mlp_backward(theta, X, Z1, Z2, Y, T, nb, dz_scratch, grad, as_stream(stream));
}

int spmv_mlp_adam(float* theta, const float* grad, float* m, float* v, int32_t t, float lr,
                  float beta1, float beta2, float eps, void* stream) {
  if (!theta || !grad || !m || !v) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  if (t < 1) return fail(SPMV_ERR_INVALID_ARG, "t must be >= 1");
  return launch_mlp_adam(theta, grad, m, v, t, lr, beta1, beta2, eps, as_stream(stream));
}

// ------------------------------------------------------------- measurement

int spmv_stream_triad(double* a, const double* b, const double* c, double s, int64_t n,
                      void* stream) {
  if (n < 0) return fail(SPMV_ERR_INVALID_ARG, "n < 0");
  if (n > 0 && (!a || !b || !c)) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  if ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b) |
       reinterpret_cast<uintptr_t>(c)) % 16)
    return fail(SPMV_ERR_INVALID_ARG, "arrays must be 16-byte aligned");
  return launch_triad(a, b, c, s, n, as_stream(stream));
}

int spmv_stream_copy(double* dst, const double* src, int64_t n, void* stream) {
  if (n < 0) return fail(SPMV_ERR_INVALID_ARG, "n < 0");
  if (n > 0 && (!dst || !src)) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  if ((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) % 16)
    return fail(SPMV_ERR_INVALID_ARG, "arrays must be 16-byte aligned");
  return launch_copy(dst, src, n, as_stream(stream));
}

}  // extern "C"
