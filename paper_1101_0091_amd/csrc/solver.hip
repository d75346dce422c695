// Iterative solvers on top of the CRS product: conjugate gradients and
// Lanczos, the kind of eigen- and linear solvers whose run time the paper's
// spMVM dominates (Sect. 1). Every vector operation is a kernel here; the
// scalars (alpha, beta, norms) stay in device memory, so an iteration is a
// fixed launch sequence that can be captured into a HIP graph. Dot products
// use a fixed grid and a fixed summation order: results are bitwise
// reproducible. The workgroup that finishes a reduction last (one counter
// atomic per workgroup) sums the partials and updates the scalars in the same
// launch, so an iteration is four launches: the product, the fused p.Ap
// reduction, the fused x/r update with r.r, and the p update. For plans whose
// product runs a lane per row or four lanes per row, the p update, the
// product and the p.Ap reduction are one launch (k_cg_step), so an iteration
// is two; a Lanczos step likewise (k_lz_step, then k_lz_b).
#include <cmath>
#include <vector>

#include "common.hpp"
#include "device.hpp"

namespace spmv {
namespace {

constexpr int kRed = 1024;  // workgroups of every reduction (fixed: deterministic order)
// Arrival counters of a reduction: kGroups group counters of kRed / kGroups
// workgroups each, one 128-byte line apart, then a top counter. A single
// counter hit by all 1024 workgroups serialises their atomics (a CG iteration
// took 43 us against 22 us with a separate finishing launch).
constexpr int kGroups = 32;
constexpr int kLine = 32;  // unsigned words per 128-byte line
constexpr int kCountWords = kLine * (kGroups + 1);
static_assert(kRed % kGroups == 0 && kGroups < 64, "group counters");
// scalar block: 64 double slots, then the counters
constexpr size_t kScBlock = ((sizeof(double) * 64 + sizeof(unsigned) * kCountWords) + 255) &
                            ~size_t(255);

// scalar slots in the solver workspace
enum : int { S_RR = 0, S_PAP = 1, S_ALPHA = 2, S_BETA = 3, S_BB = 4, S_TMP = 5 };

__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = dev::group_sum<64>(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  const double s = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return s;
}

// What the last workgroup of a reduction does with its result: the scalar
// update op (0: sc[dst] = sum; 1: sc[dst] = sqrt(sum); 2: alpha = rr / sum;
// 3: beta = sum / rr, rr = sum) and an optional copy into a history array.
struct Finish {
  double* sc;
  unsigned* count;  // kCountWords arrival counters, zero between launches
  double* hist;
  int op;
  int dst;
};

// Called by every workgroup of a kRed-workgroup reduction with its partial
// sum in thread 0. Thread 0 stores the partial as a device-scope atomic (a
// store that is coherent across the XCDs' L2 caches) and, once the store is
// acknowledged, counts the arrival in its group's counter; the workgroup that
// completes a group counts the group in the top counter, and the workgroup
// that completes the top counter has every partial behind it: it reads them
// with device-scope atomic loads in index order, applies the op and clears the
// counters for the next launch. No cache writeback or invalidation is needed
// (a __threadfence in each of the 1024 workgroups made a CG iteration three
// times slower), and no workgroup waits for another, so nothing can stall.
__device__ __forceinline__ void finish_if_last(double* __restrict__ partials, double part,
                                               const Finish& f, double* sh) {
  __shared__ unsigned last;
  if (threadIdx.x == 0) {
    __hip_atomic_store(partials + blockIdx.x, part, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // the arrival is counted only once the store is acknowledged
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    const unsigned grp = blockIdx.x / (kRed / kGroups);
    unsigned l = 0;
    if (atomicAdd(f.count + kLine * (1 + grp), 1u) == (unsigned)(kRed / kGroups - 1))
      l = atomicAdd(f.count, 1u) == (unsigned)(kGroups - 1);
    last = l;
  }
  __syncthreads();
  if (!last) return;
  // all loads issued before the first add; the sum keeps index order
  static_assert(kRed == 4 * kWG, "four partials per thread");
  double v[4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
    v[u] = __hip_atomic_load(partials + threadIdx.x + u * kWG, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < 4; ++u) s += v[u];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) {
    double* sc = f.sc;
    if (f.op == 0) sc[f.dst] = s;
    if (f.op == 1) sc[f.dst] = sqrt(s);
    if (f.op == 2) sc[S_ALPHA] = sc[S_RR] / s;
    if (f.op == 3) {
      sc[S_BETA] = s / sc[S_RR];
      sc[S_RR] = s;
    }
    if (f.hist) *f.hist = f.op == 1 ? sqrt(s) : s;
  }
  if (threadIdx.x <= kGroups)
    __hip_atomic_store(f.count + kLine * threadIdx.x, 0u, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// sum of x*y over all n, then the Finish op
__global__ __launch_bounds__(kWG) void k_dot(const double* __restrict__ x,
                                             const double* __restrict__ y, int64_t n,
                                             double* __restrict__ partials, Finish f) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += (int64_t)kRed * kWG)
    s = fma(x[i], y[i], s);
  s = block_sum(s, sh);
  finish_if_last(partials, s, f, sh);
}

__global__ __launch_bounds__(64) void k_clear_count(unsigned* count) {
  if (threadIdx.x <= kGroups)
    __hip_atomic_store(count + kLine * threadIdx.x, 0u, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// r = b - Ap ; p = r (and its float32 copy for FP32-storage plans)
__global__ __launch_bounds__(kWG) void k_cg_init(const double* __restrict__ b,
                                                 const double* __restrict__ Ap,
                                                 double* __restrict__ r, double* __restrict__ p,
                                                 float* __restrict__ p32, int64_t n,
                                                 double* __restrict__ sc) {
  // beta of the first step: k_cg_step forms p = r + 0 p
  if (blockIdx.x == 0 && threadIdx.x == 0) sc[S_BETA] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kWG) {
    const double v = b[i] - Ap[i];
    r[i] = v;
    p[i] = v;
    if (p32) p32[i] = (float)v;
  }
}

// x += alpha p ; r -= alpha Ap ; r.r, then beta = r.r / rr, rr = r.r
__global__ __launch_bounds__(kWG) void k_cg_xr(double* __restrict__ x, double* __restrict__ r,
                                               const double* __restrict__ p,
                                               const double* __restrict__ Ap, int64_t n,
                                               double* __restrict__ partials, Finish f) {
  __shared__ double sh[4];
  const double a = f.sc[S_ALPHA];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += (int64_t)kRed * kWG) {
    x[i] = fma(a, p[i], x[i]);
    const double ri = fma(-a, Ap[i], r[i]);
    r[i] = ri;
    s = fma(ri, ri, s);
  }
  s = block_sum(s, sh);
  finish_if_last(partials, s, f, sh);
}

// p = r + beta p (and its float32 copy for FP32-storage plans)
__global__ __launch_bounds__(kWG) void k_cg_p(double* __restrict__ p, float* __restrict__ p32,
                                              const double* __restrict__ r,
                                              const double* __restrict__ sc, int64_t n) {
  const double be = sc[S_BETA];
  for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kWG) {
    const double v = fma(be, p[i], r[i]);
    p[i] = v;
    if (p32) p32[i] = (float)v;
  }
}

// One CG step in one launch, for plans whose product runs a lane per row
// or four lanes per row: p = r + beta p is formed where it is used (at each
// gathered column from r and the previous p, for the thread's own row into
// pn), Ap = A p with a lane per row adding its products in CRS order (V0's
// order), and p.Ap reduced over the same element partition and in the same
// order as k_dot, then alpha = rr / p.Ap set by the last workgroup. With a
// V0 plan every value equals the four-launch iteration's bit for bit.
template <typename VT, typename BT>
__global__ __launch_bounds__(kWG) void k_cg_step(const int32_t* __restrict__ rp,
                                                 const int32_t* __restrict__ ci,
                                                 const VT* __restrict__ val, int64_t n,
                                                 const double* __restrict__ r,
                                                 const double* __restrict__ p,
                                                 double* __restrict__ pn, double* __restrict__ Ap,
                                                 double* __restrict__ partials, Finish f) {
  __shared__ double sh[4];
  const double be = f.sc[S_BETA];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += (int64_t)kRed * kWG) {
    const int32_t a = rp[i], e = rp[i + 1];
    double acc = 0.0;
    int32_t j = a;
    // four entries at a time, every load issued before the first use (the
    // products are still added one by one in CRS order)
    for (; j + 4 <= e; j += 4) {
      int32_t c[4];
      VT v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        c[u] = ci[j + u];
        v[u] = val[j + u];
      }
      double pv[4], rv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        pv[u] = p[c[u]];
        rv[u] = r[c[u]];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        acc = fma(dev::widen(v[u]), dev::widen((BT)fma(be, pv[u], rv[u])), acc);
    }
    for (; j < e; ++j) {
      const int32_t c = ci[j];
      acc = fma(dev::widen(val[j]), dev::widen((BT)fma(be, p[c], r[c])), acc);
    }
    const double pi = fma(be, p[i], r[i]);
    pn[i] = pi;
    Ap[i] = acc;
    s = fma(pi, acc, s);
  }
  s = block_sum(s, sh);
  finish_if_last(partials, s, f, sh);
}

// After k_cg_step: x += alpha pn ; r -= alpha Ap ; p = pn ; r.r, then
// beta = r.r / rr, rr = r.r
__global__ __launch_bounds__(kWG) void k_cg_xr_pn(double* __restrict__ x, double* __restrict__ r,
                                                  double* __restrict__ p,
                                                  const double* __restrict__ pn,
                                                  const double* __restrict__ Ap, int64_t n,
                                                  double* __restrict__ partials, Finish f) {
  __shared__ double sh[4];
  const double a = f.sc[S_ALPHA];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += (int64_t)kRed * kWG) {
    const double pi = pn[i];
    x[i] = fma(a, pi, x[i]);
    const double ri = fma(-a, Ap[i], r[i]);
    r[i] = ri;
    p[i] = pi;
    s = fma(ri, ri, s);
  }
  s = block_sum(s, sh);
  finish_if_last(partials, s, f, sh);
}

__global__ __launch_bounds__(kWG) void k_to_f32(float* __restrict__ d, const double* __restrict__ s,
                                                int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kWG)
    d[i] = (float)s[i];
}

// Lanczos: w -= beta_j v_prev (beta from the history array), then
// alpha_j = w.v into the history
__global__ __launch_bounds__(kWG) void k_lz_a(double* __restrict__ w,
                                              const double* __restrict__ v,
                                              const double* __restrict__ vprev,
                                              const double* __restrict__ beta_j, int64_t n,
                                              double* __restrict__ partials, Finish f) {
  __shared__ double sh[4];
  const double be = *beta_j;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += (int64_t)kRed * kWG) {
    const double wi = fma(-be, vprev[i], w[i]);
    w[i] = wi;
    s = fma(wi, v[i], s);
  }
  s = block_sum(s, sh);
  finish_if_last(partials, s, f, sh);
}

// w -= alpha_j v, then beta_{j+1} = ||w|| into the history
__global__ __launch_bounds__(kWG) void k_lz_b(double* __restrict__ w,
                                              const double* __restrict__ v,
                                              const double* __restrict__ alpha_j, int64_t n,
                                              double* __restrict__ partials, Finish f) {
  __shared__ double sh[4];
  const double al = *alpha_j;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += (int64_t)kRed * kWG) {
    const double wi = fma(-al, v[i], w[i]);
    w[i] = wi;
    s = fma(wi, wi, s);
  }
  s = block_sum(s, sh);
  finish_if_last(partials, s, f, sh);
}

// The first half of a Lanczos step in one launch, for plans whose product
// runs a lane per row or four lanes per row: v_j = w / beta_j formed where it
// is used (at each gathered column, and for the own row into vout) unless vin
// already holds v_j (the first step), w = A v_j - beta_j v_{j-1} with a lane
// per row adding its products in CRS order, and alpha_j = w.v_j over
// k_lz_a's element partition and order. With a V0 plan every value equals the
// four-launch step's (product, k_lz_a, k_lz_b, k_scale) bit for bit.
template <typename VT, typename BT>
__global__ __launch_bounds__(kWG) void k_lz_step(const int32_t* __restrict__ rp,
                                                 const int32_t* __restrict__ ci,
                                                 const VT* __restrict__ val, int64_t n,
                                                 const double* __restrict__ win,
                                                 const double* __restrict__ vin,
                                                 const double* __restrict__ beta_j,
                                                 double* __restrict__ vout,
                                                 const double* __restrict__ vprev,
                                                 double* __restrict__ wout,
                                                 double* __restrict__ partials, Finish f) {
  __shared__ double sh[4];
  const double bj = *beta_j;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += (int64_t)kRed * kWG) {
    const int32_t a = rp[i], e = rp[i + 1];
    double acc = 0.0;
    int32_t j = a;
    for (; j + 4 <= e; j += 4) {
      int32_t c[4];
      VT v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        c[u] = ci[j + u];
        v[u] = val[j + u];
      }
      double x[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) x[u] = vin ? vin[c[u]] : win[c[u]] / bj;
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = fma(dev::widen(v[u]), dev::widen((BT)x[u]), acc);
    }
    for (; j < e; ++j) {
      const int32_t c = ci[j];
      acc = fma(dev::widen(val[j]), dev::widen((BT)(vin ? vin[c] : win[c] / bj)), acc);
    }
    const double vi = vin ? vin[i] : win[i] / bj;
    if (!vin) vout[i] = vi;
    const double wi = fma(-bj, vprev[i], acc);
    wout[i] = wi;
    s = fma(wi, vi, s);
  }
  s = block_sum(s, sh);
  finish_if_last(partials, s, f, sh);
}

// v_out = w / beta (beta = norm stored at *beta_next), with its float32 copy
// for FP32-storage plans
__global__ __launch_bounds__(kWG) void k_scale(double* __restrict__ out, float* __restrict__ out32,
                                               const double* __restrict__ in,
                                               const double* __restrict__ denom, int64_t n) {
  const double d = *denom;
  for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kWG) {
    const double v = in[i] / d;
    out[i] = v;
    if (out32) out32[i] = (float)v;
  }
}

unsigned vgrid(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + kWG - 1) / kWG, 8192));
}

struct SolverWs {
  double* sc;
  unsigned* count;  // the reductions' arrival counters, in the scalar block
  double* partials;
  double* r;
  double* p;
  double* Ap;
  double* pn;  // the next search direction of the one-launch CG step
  float* p32;
};

size_t solver_ws_bytes(int64_t n, int64_t hist) {
  const size_t n1 = (size_t)std::max<int64_t>(n, 1);
  return kScBlock + align256(sizeof(double) * kRed) +
         4 * align256(sizeof(double) * n1) + align256(sizeof(float) * n1) +
         align256(sizeof(double) * (size_t)std::max<int64_t>(hist, 1));
}

SolverWs carve(void* ws, int64_t n) {
  char* c = static_cast<char*>(ws);
  const size_t n1 = (size_t)std::max<int64_t>(n, 1);
  SolverWs w;
  w.sc = reinterpret_cast<double*>(c);
  w.count = reinterpret_cast<unsigned*>(c + sizeof(double) * 64);
  c += kScBlock;
  w.partials = reinterpret_cast<double*>(c);
  c += align256(sizeof(double) * kRed);
  w.r = reinterpret_cast<double*>(c);
  c += align256(sizeof(double) * n1);
  w.p = reinterpret_cast<double*>(c);
  c += align256(sizeof(double) * n1);
  w.Ap = reinterpret_cast<double*>(c);
  c += align256(sizeof(double) * n1);
  w.pn = reinterpret_cast<double*>(c);
  c += align256(sizeof(double) * n1);
  w.p32 = reinterpret_cast<float*>(c);
  return w;
}

double* history(void* ws, int64_t n) {
  char* c = static_cast<char*>(ws);
  const size_t n1 = (size_t)std::max<int64_t>(n, 1);
  return reinterpret_cast<double*>(c + kScBlock +
                                   align256(sizeof(double) * kRed) +
                                   4 * align256(sizeof(double) * n1) +
                                   align256(sizeof(float) * n1));
}

// y = A x for a plan of either storage type (x float64; cast for FP32 plans)
int plan_apply(const Plan& p, const double* x, float* x32, double* y, hipStream_t s) {
  if (p.vdt == SPMV_F64) return launch_spmv(p, p.variant, x, y, s);
  k_to_f32<<<vgrid(p.n_cols), kWG, 0, s>>>(x32, x, p.n_cols);
  SPMV_HIP(hipGetLastError());
  return launch_spmv(p, p.variant, x32, y, s);
}

// y = A x where x already has its float32 copy x32 for FP32 plans
int plan_apply_cast(const Plan& p, const double* x, const float* x32, double* y,
                    hipStream_t s) {
  if (p.vdt == SPMV_F64) return launch_spmv(p, p.variant, x, y, s);
  return launch_spmv(p, p.variant, x32, y, s);
}

Finish fin(const SolverWs& w, int op, int dst, double* hist) {
  return Finish{w.sc, w.count, hist, op, dst};
}

int dot(const double* x, const double* y, int64_t n, SolverWs& w, int op, int dst,
        double* hist, hipStream_t s) {
  k_dot<<<kRed, kWG, 0, s>>>(x, y, n, w.partials, fin(w, op, dst, hist));
  SPMV_HIP(hipGetLastError());
  return SPMV_OK;
}

// plans whose product runs a lane per row or four lanes per row take the
// one-launch CG and Lanczos steps (their products go a lane per row)
bool one_launch_step(const Plan& P) {
  return P.variant == SPMV_V0_THREAD_ROW || P.variant == SPMV_V1_LANES4;
}

// one CG iteration: Ap = A p; alpha = rr/(p.Ap); x += alpha p; r -= alpha Ap;
// beta = r.r/rr; rr = r.r; p = r + beta p
int cg_iteration(const Plan& P, double* x, SolverWs& w, int64_t n, hipStream_t s) {
  if (one_launch_step(P)) {
    if (P.vdt == SPMV_F64)
      k_cg_step<double, double><<<kRed, kWG, 0, s>>>(
          P.row_ptr, P.col_idx, static_cast<const double*>(P.val), n, w.r, w.p, w.pn, w.Ap,
          w.partials, fin(w, 2, 0, nullptr));
    else
      k_cg_step<float, float><<<kRed, kWG, 0, s>>>(
          P.row_ptr, P.col_idx, static_cast<const float*>(P.val), n, w.r, w.p, w.pn, w.Ap,
          w.partials, fin(w, 2, 0, nullptr));
    SPMV_HIP(hipGetLastError());
    k_cg_xr_pn<<<kRed, kWG, 0, s>>>(x, w.r, w.p, w.pn, w.Ap, n, w.partials,
                                    fin(w, 3, 0, nullptr));
    SPMV_HIP(hipGetLastError());
    return SPMV_OK;
  }
  int st = plan_apply_cast(P, w.p, w.p32, w.Ap, s);
  if (!st) st = dot(w.p, w.Ap, n, w, 2, 0, nullptr, s);
  if (st) return st;
  k_cg_xr<<<kRed, kWG, 0, s>>>(x, w.r, w.p, w.Ap, n, w.partials, fin(w, 3, 0, nullptr));
  SPMV_HIP(hipGetLastError());
  k_cg_p<<<vgrid(n), kWG, 0, s>>>(w.p, P.vdt == SPMV_F64 ? nullptr : w.p32, w.r, w.sc, n);
  SPMV_HIP(hipGetLastError());
  return SPMV_OK;
}

}  // namespace

size_t cg_workspace_bytes(int64_t n) { return solver_ws_bytes(n, 1); }
size_t lanczos_workspace_bytes(int64_t n, int k) {
  // solver block plus history (alpha[k], beta[k+1]) plus three Lanczos vectors
  return solver_ws_bytes(n, 2 * (int64_t)k + 2) +
         3 * align256(sizeof(double) * (size_t)std::max<int64_t>(n, 1));
}

int run_cg(const Plan& P, const double* b, double* x, double tol, int maxit, int check_every,
           bool use_graph, void* ws, int* iters, double* relres, hipStream_t s) {
  const int64_t n = P.n_rows;
  SolverWs w = carve(ws, n);
  k_clear_count<<<1, 64, 0, s>>>(w.count);
  SPMV_HIP(hipGetLastError());
  // ||b||^2 and the initial residual
  int st = dot(b, b, n, w, 0, S_BB, nullptr, s);
  if (!st) st = plan_apply(P, x, w.p32, w.Ap, s);
  if (st) return st;
  k_cg_init<<<vgrid(n), kWG, 0, s>>>(b, w.Ap, w.r, w.p, P.vdt == SPMV_F64 ? nullptr : w.p32, n,
                                     w.sc);
  SPMV_HIP(hipGetLastError());
  st = dot(w.r, w.r, n, w, 0, S_RR, nullptr, s);
  if (st) return st;
  double h[6];
  SPMV_HIP(hipMemcpyAsync(h, w.sc, sizeof(h), hipMemcpyDeviceToHost, s));
  SPMV_HIP(hipStreamSynchronize(s));
  const double bn = h[S_BB] > 0.0 ? std::sqrt(h[S_BB]) : 1.0;
  double rr = h[S_RR];
  int it = 0;
  *relres = std::sqrt(rr) / bn;
  if (*relres <= tol || maxit <= 0) {
    *iters = 0;
    return SPMV_OK;
  }
  const int every = check_every > 0 ? check_every : 1;
  // a graph holds the iterations between two residual checks (at most 64:
  // the largest divisor of check_every up to 64), so one graph launch
  // replaces that many iterations' launches
  int per_graph = 1;
  for (int d = std::min(every, 64); d >= 1; --d)
    if (every % d == 0) {
      per_graph = d;
      break;
    }
  hipGraphExec_t exec = nullptr;
  if (use_graph) {
    if (!s) return fail(SPMV_ERR_INVALID_ARG, "graph mode needs a non-null stream");
    hipGraph_t g = nullptr;
    SPMV_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < per_graph && !st; ++k) st = cg_iteration(P, x, w, n, s);
    hipError_t e = hipStreamEndCapture(s, &g);
    if (st) {
      if (g) hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return hip_fail(e, "capture of a CG iteration");
    e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  }
  while (it < maxit) {
    if (exec && it + per_graph <= maxit) {
      hipError_t e = hipGraphLaunch(exec, s);
      if (e != hipSuccess) {
        hipGraphExecDestroy(exec);
        return hip_fail(e, "hipGraphLaunch");
      }
      it += per_graph;
    } else {
      st = cg_iteration(P, x, w, n, s);
      if (st) {
        if (exec) hipGraphExecDestroy(exec);
        return st;
      }
      ++it;
    }
    if (it % every == 0 || it == maxit) {
      hipError_t e = hipMemcpyAsync(&rr, w.sc + S_RR, sizeof(double), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) {
        if (exec) hipGraphExecDestroy(exec);
        return hip_fail(e, "residual readback");
      }
      *relres = std::sqrt(rr) / bn;
      if (*relres <= tol) break;
    }
  }
  if (exec) hipGraphExecDestroy(exec);
  *iters = it;
  return SPMV_OK;
}

int run_lanczos(const Plan& P, const double* v0, int k, double* alpha, double* beta, void* ws,
                hipStream_t s) {
  const int64_t n = P.n_rows;
  SolverWs w = carve(ws, n);
  double* hist = history(ws, n);  // alpha[k] then beta[k+1]
  double* ha = hist;
  double* hb = hist + k;
  char* vec = reinterpret_cast<char*>(hist) + align256(sizeof(double) * (2 * (size_t)k + 2));
  const size_t vb = align256(sizeof(double) * (size_t)std::max<int64_t>(n, 1));
  double* V[3] = {reinterpret_cast<double*>(vec), reinterpret_cast<double*>(vec + vb),
                  reinterpret_cast<double*>(vec + 2 * vb)};
  double* wv = w.Ap;
  float* v32 = P.vdt == SPMV_F64 ? nullptr : w.p32;  // float32 copy of the current vector
  k_clear_count<<<1, 64, 0, s>>>(w.count);
  SPMV_HIP(hipGetLastError());
  // beta_0 = 0, v_prev = 0, v = v0 / ||v0||
  int st = dot(v0, v0, n, w, 1, S_TMP, hb, s);
  if (st) return st;
  k_scale<<<vgrid(n), kWG, 0, s>>>(V[1], v32, v0, hb, n);
  SPMV_HIP(hipGetLastError());
  // any finite vector; it is scaled by beta_0 = 0
  k_scale<<<vgrid(n), kWG, 0, s>>>(V[0], nullptr, v0, hb, n);
  SPMV_HIP(hipGetLastError());
  static const double zero = 0.0;
  SPMV_HIP(hipMemcpyAsync(hb, &zero, sizeof(double), hipMemcpyHostToDevice, s));
  int prev = 0, cur = 1, nxt = 2;
  if (one_launch_step(P)) {
    // two launches per step; w alternates between two buffers, since a
    // step forms v_j from the previous w while it writes the new one
    double* wb[2] = {w.Ap, w.pn};
    for (int j = 0; j < k; ++j) {
      double* wo = wb[j & 1];
      const double* wi = j == 0 ? nullptr : wb[(j & 1) ^ 1];
      const double* vi = j == 0 ? V[cur] : nullptr;
      if (P.vdt == SPMV_F64)
        k_lz_step<double, double><<<kRed, kWG, 0, s>>>(
            P.row_ptr, P.col_idx, static_cast<const double*>(P.val), n, wi, vi, hb + j, V[cur],
            V[prev], wo, w.partials, fin(w, 0, S_TMP, ha + j));
      else
        k_lz_step<float, float><<<kRed, kWG, 0, s>>>(
            P.row_ptr, P.col_idx, static_cast<const float*>(P.val), n, wi, vi, hb + j, V[cur],
            V[prev], wo, w.partials, fin(w, 0, S_TMP, ha + j));
      SPMV_HIP(hipGetLastError());
      k_lz_b<<<kRed, kWG, 0, s>>>(wo, V[cur], ha + j, n, w.partials,
                                  fin(w, 1, S_TMP, hb + j + 1));
      SPMV_HIP(hipGetLastError());
      const int t = prev;
      prev = cur;
      cur = nxt;
      nxt = t;
    }
  } else {
    for (int j = 0; j < k; ++j) {
      st = plan_apply_cast(P, V[cur], v32, wv, s);
      if (st) return st;
      k_lz_a<<<kRed, kWG, 0, s>>>(wv, V[cur], V[prev], hb + j, n, w.partials,
                                  fin(w, 0, S_TMP, ha + j));
      SPMV_HIP(hipGetLastError());
      k_lz_b<<<kRed, kWG, 0, s>>>(wv, V[cur], ha + j, n, w.partials,
                                  fin(w, 1, S_TMP, hb + j + 1));
      SPMV_HIP(hipGetLastError());
      k_scale<<<vgrid(n), kWG, 0, s>>>(V[nxt], v32, wv, hb + j + 1, n);
      SPMV_HIP(hipGetLastError());
      const int t = prev;
      prev = cur;
      cur = nxt;
      nxt = t;
    }
  }
  std::vector<double> hh(2 * (size_t)k + 1);
  SPMV_HIP(hipMemcpyAsync(hh.data(), hist, sizeof(double) * hh.size(), hipMemcpyDeviceToHost, s));
  SPMV_HIP(hipStreamSynchronize(s));
  for (int j = 0; j < k; ++j) {
    alpha[j] = hh[j];
    beta[j] = hh[k + j + 1];
  }
  return SPMV_OK;
}

}  // namespace spmv
