// Internal declarations shared by the translation units of libspmv.
// gfx950 (CDNA4) only: 64-lane wavefronts, DPP row operations on 16-lane rows.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/spmv.h"

namespace spmv {

// ---------------------------------------------------------------- constants

constexpr int kWG = 256;          // threads per workgroup for the streaming kernels
constexpr int kBlockBudget = 2048;  // rows + in-chunk nonzeros of one LDS row block
// B entries a V4 row block stages in its kBlockBudget doubles of LDS: float32
// B is staged as float32, so twice as many.
template <typename BT>
constexpr int kStageEntries = sizeof(BT) == 4 ? 2 * kBlockBudget : kBlockBudget;
// V4 window form: a super-block of kSbRows rows per workgroup; windows of B
// are kWinSize aligned columns, at most kWinMax per super-block
constexpr int kSbRows = 4096;
constexpr int kWinLog = 12;
constexpr int kWinSize = 1 << kWinLog;
constexpr int kWinMax = 6;
constexpr int kNumXCD = 8;        // MI355X: 8 accelerator complex dies, one L2 each
constexpr int kNumBins = 5;       // row-length bins of the binned variant
// batch tile record: matrix, r0, r1, S, E, staging cmin, cmax, column-delta bits (0, 8 or 16),
// delta base, pad
constexpr int kTileInts = 10;
// Largest n_rows, n_cols and nnz: every int32 row, nonzero and column index
// plus a kernel's stride (at most 4096) stays below 2^31.
constexpr int64_t kMaxDim = 2147483647LL - 4096;
constexpr int kCounters = 32;     // u64 analysis counters in the workspace header
constexpr int kStatsGrid = 1024;  // most workgroups of the row-statistics pass
constexpr int kPartSlots = 18;    // u64 partial counters per statistics workgroup

// Workspace header (first kHeaderBytes of every plan workspace).
struct alignas(256) WsHeader {
  int32_t err;                 // CRS violation bits (validate)
  int32_t pad0[15];
  unsigned long long cnt[kCounters];  // analysis counters (stats)
  double features[SPMV_NUM_FEATURES];
  float x_std[SPMV_NUM_FEATURES];      // standardised selector input
  float pred[8];                       // selector output (6 used)
  float z1[64], z2[64];                // selector forward scratch
  int32_t bin_count[8];
  int32_t bin_offset[8];
  int64_t sell_total;  // padded width sum of the V6 copy, in units of 64 slots
  int32_t staged_blocks;  // row blocks whose chunk's columns fit the LDS staging array
  int32_t pad1;
  unsigned long long win_covered;  // nonzeros inside the windows of their super-block
};
constexpr size_t kHeaderBytes = (sizeof(WsHeader) + 255) / 256 * 256;

// Counter slots inside WsHeader::cnt
enum : int {
  C_SUMSQ = 0, C_LMAX = 1, C_LMIN = 2, C_BIN0 = 3,  // feature bins C_BIN0..C_BIN0+5
  C_LONGNNZ = 9, C_DISTLOG = 10, C_NEAR = 11, C_NNZ = 12
};

// ---------------------------------------------------------------- plan

// the three forms of V4 (the same rows and products, different B access)
enum : int { kV4Plain = 0, kV4Staged = 1, kV4Window = 2 };

struct Plan {
  int64_t n_rows = 0, n_cols = 0, nnz = 0;
  const int32_t* row_ptr = nullptr;
  const int32_t* col_idx = nullptr;
  const void* val = nullptr;
  int vdt = SPMV_F64;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  WsHeader* hdr = nullptr;        // device
  int2* blocks = nullptr;         // device [nblocks+1]: (first row, row_ptr[first row])
  int2* spans = nullptr;          // device [nblocks]: (smallest, largest) column of the block's chunk
  int64_t staged_blocks = 0;      // blocks with a span that fits the LDS staging array
  int v4_form = 0;                // V4 form: kV4Plain, kV4Staged or kV4Window
  bool v4_form_forced = false;    // the form was fixed by a plan flag
  int64_t nsb = 0;                // super-blocks of the window form
  int32_t* win = nullptr;         // device int32[nsb][kWinMax]: window bins, -1 unused
  int64_t win_covered = 0;        // nonzeros whose column lies in their super-block's windows
  int64_t nblocks = 0;
  int32_t* bin_rows = nullptr;    // device int32[n_rows]
  unsigned long long* stats_part = nullptr;  // device [kStatsGrid][kPartSlots]
  int32_t* bin_base = nullptr;    // device [kStatsGrid][kNumBins]: a workgroup's first slot per bin
  int32_t bin_count[kNumBins] = {0, 0, 0, 0, 0};
  int32_t bin_offset[kNumBins] = {0, 0, 0, 0, 0};
  void* at_B = nullptr;           // autotune scratch (device) or null
  double* at_C = nullptr;
  int variant = SPMV_V4_LDS_BLOCK;
  double features[SPMV_NUM_FEATURES] = {};
  float pred[SPMV_NUM_SELECTOR_OUTPUTS] = {};
  bool have_pred = false;
  double at_us[SPMV_NUM_VARIANTS] = {};
  bool have_autotune = false;
  int device = 0;
  // V6 chunked copy (present only with SPMV_FLAG_SELL)
  int64_t sell_nch = 0;           // chunks of 64 rows
  int64_t sell_cap = 0;           // reserved slots
  int64_t sell_slots = 0;         // slots in use (64 * sum of chunk widths)
  int32_t* sell_width = nullptr;  // device int32[nch]
  int32_t* sell_off = nullptr;    // device int32[nch + 1], in units of 64 slots
  int32_t* sell_partials = nullptr;
  int32_t* sell_ci = nullptr;     // device int32[cap]
  void* sell_val = nullptr;       // device val_dtype[cap]
  // column deltas: for chunk k (slots a = off[k] .. off[k+1] per lane),
  // base[a + j] is the smallest column of slot j and dl the column minus that
  // base in flag[k] = 8 or 16 bits (all ones for padding; 8-bit deltas in the
  // first half of the chunk's region), flag[k] = 0 for 4-byte columns
  int32_t* sell_base = nullptr;   // device int32[cap / 64]
  uint16_t* sell_dl = nullptr;    // device uint16[cap]
  int32_t* sell_flag = nullptr;   // device int32[nch]
  bool sell_wide = false;         // 32-bit columns in every chunk (no deltas built)
  bool sell_reserved = false;
  bool sell_ok = false;
};

struct Batch {
  int32_t count = 0;
  int vdt = SPMV_F64;
  const int32_t* const* row_ptrs = nullptr;  // device arrays of device pointers
  const int32_t* const* col_idxs = nullptr;
  const void* const* vals = nullptr;
  int32_t* tiles = nullptr;   // device int32[kTileInts * ntiles]
  uint8_t* deltas = nullptr;  // device [ntiles][2 * kBlockBudget]: column deltas per tile chunk
  int64_t ntiles = 0;
  int32_t* err = nullptr;     // device
  // device: kBatchQueues claim counters, then the finished-workgroup counter,
  // kBatchCounterStride words apart
  unsigned int* counters = nullptr;
  int mode = SPMV_BATCH_TILE_GRID;
  int64_t* tile_offset_host = nullptr;  // host [count+1]
  const int32_t** rp_host = nullptr;    // host copies of the device pointer arrays
  const int32_t** ci_host = nullptr;
  const void** val_host = nullptr;
  int grid_static = 0;   // resident workgroups of the persistent kernels
  int grid_dynamic = 0;  // (CUs x workgroups per CU at their occupancy)
};

// ---------------------------------------------------------------- errors

void set_error(const std::string& msg);
int fail(int status, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define SPMV_HIP(call)                                  \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return spmv::hip_fail(e_, #call); \
  } while (0)

inline size_t align256(size_t x) { return (x + 255) / 256 * 256; }

inline int64_t super_block_count(int64_t n_rows) { return (n_rows + kSbRows - 1) / kSbRows; }

inline int64_t lds_block_count(int64_t n_rows, int64_t nnz) {
  if (n_rows <= 0) return 0;
  return (nnz + n_rows + kBlockBudget - 1) / kBlockBudget;
}

// ---------------------------------------------------------------- launchers
// analysis.hip
int launch_zero_header(WsHeader* h, hipStream_t s);
int launch_validate(const Plan& p, hipStream_t s);
int launch_analysis(Plan& p, const float* mu, const float* sigma, hipStream_t s);
// spmv_kernels.hip
int launch_spmv(const Plan& p, int variant, const void* B, double* C, hipStream_t s);
int launch_spmm(const Plan& p, int k, const void* B, int64_t ldb, double* C, int64_t ldc,
                hipStream_t s);
int launch_fill(void* dst, int dtype, int64_t n, double value, hipStream_t s);
// C += A*B with the LDS-block kernel (second pass of a split product)
int launch_spmv_accumulate(const Plan& p, const void* B, double* C, hipStream_t s);
// split.hip
int launch_split_count(int64_t n, const int32_t* rp, const int32_t* ci, int64_t col_lo,
                       int64_t col_hi, int32_t* len_loc, int32_t* len_rem, hipStream_t s);
int launch_exclusive_scan(const int32_t* in, int32_t* out, int64_t n, int32_t* partials,
                          hipStream_t s);
int scan_partials_count(int64_t n);
int launch_split_fill(int64_t n, const int32_t* rp, const int32_t* ci, const void* val, int vdt,
                      int64_t col_lo, int64_t col_hi, const int32_t* rp_loc,
                      const int32_t* rp_rem, int32_t* ci_loc, void* val_loc, int32_t* ci_rem,
                      void* val_rem, hipStream_t s);
// batch.hip
int launch_batch_build(Batch& b, const int64_t* tile_offset_dev, const int64_t* n_rows_dev,
                       const int64_t* n_cols_dev, const int64_t* nnz_dev, hipStream_t s);
int launch_batch_apply(const Batch& b, int64_t t0, int64_t t1, const void* const* Bs,
                       double* const* Cs, const void* B1, double* C1, hipStream_t s);
constexpr int kBatchQueues = kNumXCD;   // claim queues of the dynamic batch kernel
constexpr int kBatchCounterStride = 32;  // 128 bytes between counters
constexpr int kBatchCounterWords = (kBatchQueues + 1) * kBatchCounterStride;
// workgroups of the static and dynamic persistent kernels that fit on the
// device at once, for value type vdt
int batch_grids(int device, int vdt, int* g_static, int* g_dynamic);
int launch_counters_init(unsigned int* c, hipStream_t s);
// mlp.hip
int launch_mlp_forward(const float* theta, const float* X, int nb, float* Y, float* Z1,
                       float* Z2, hipStream_t s);
int launch_mlp_backward(const float* theta, const float* X, const float* Z1, const float* Z2,
                        const float* Y, const float* T, int nb, float* scratch, float* grad,
                        hipStream_t s);
int launch_mlp_adam(float* theta, const float* grad, float* m, float* v, int t, float lr,
                    float b1, float b2, float eps, hipStream_t s);
int selector_upload(const float* params);
const float* selector_theta_device();  // null if not loaded on the current device
// solver.hip
size_t cg_workspace_bytes(int64_t n);
size_t lanczos_workspace_bytes(int64_t n, int k);
int run_cg(const Plan& P, const double* b, double* x, double tol, int maxit, int check_every,
           bool use_graph, void* ws, int* iters, double* relres, hipStream_t s);
int run_lanczos(const Plan& P, const double* v0, int k, double* alpha, double* beta, void* ws,
                hipStream_t s);
// sell.hip
int64_t sell_chunks(int64_t n_rows);
int64_t sell_capacity(int64_t nnz);
int launch_sell_build(Plan& p, hipStream_t s);
int launch_sell(const Plan& p, const void* B, double* C, hipStream_t s);
// whether the lane-group multi-RHS kernel of the chunked copy takes this k
// and these operands (k / vector width in {2, 4, 8, 16}, 16-byte alignment)
bool sell_spmm_lanes_fit(const Plan& p, int k, const void* B, int64_t ldb, const double* C,
                         int64_t ldc);
int launch_sell_spmm(const Plan& p, int k, const void* B, int64_t ldb, double* C, int64_t ldc,
                     hipStream_t s);
// window.hip
int win_count(int vdt);
int launch_win_build(Plan& p, hipStream_t s);
int launch_win(const Plan& p, const void* B, double* C, hipStream_t s);
// stream.hip
int launch_triad(double* a, const double* b, const double* c, double s, int64_t n,
                 hipStream_t st);
int launch_copy(double* dst, const double* src, int64_t n, hipStream_t st);

}  // namespace spmv
