/*
 * crsgen: seeded synthetic CRS matrices and dense vectors.
 *
 * This module only *builds inputs*. It holds none of the sparse
 * matrix-vector arithmetic; both the CPU oracle and the GPU library are
 * fed from it. Every random number comes from the counter-based
 * Philox4x32-10 generator (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11), keyed by (seed, purpose) and
 * counted by (row / element, matrix, slot, draw). The output therefore
 * does not depend on the number of OpenMP threads.
 *
 * Matrix shapes follow the paper's workloads: the Hamiltonian-like matrix
 * stands in for the Holstein-Hubbard matrix (dimension 6.2e6, about 15
 * nonzeros per row; Sect. 1.3.1) and the permuted 3D stencil with random
 * extras stands in for the sAMG Poisson matrix (dimension 2.2e7, about 7
 * nonzeros per row; Sect. 1.3.1). Both real matrices are not available.
 *
 * Layout conventions: 0-based int32 row_ptr (n_rows+1) and col_idx, float64
 * values, columns sorted ascending and distinct inside every row.
 * Row lengths are produced by a *_rowlens call; the caller prefix-sums them
 * into row_ptr and calls the matching *_fill.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------- Philox4x32-10 ---------------- */

#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

static inline void philox(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1,
                          uint32_t c2, uint32_t c3, uint32_t out[4]) {
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    uint64_t p0 = (uint64_t)PHILOX_M0 * c0;
    uint64_t p1 = (uint64_t)PHILOX_M1 * c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Exported for known-answer tests of the generator itself. */
void crsgen_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  philox(key[0], key[1], ctr[0], ctr[1], ctr[2], ctr[3], out);
}

/* 53-bit uniform in [0,1) from two 32-bit words. */
static inline double u01(uint32_t a, uint32_t b) {
  return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

/* Box-Muller standard normal from four words (uses the first pair for the
 * radius and the second for the angle). */
static inline double normal4(const uint32_t r[4]) {
  double u1 = 1.0 - u01(r[0], r[1]); /* (0,1] */
  double u2 = u01(r[2], r[3]);
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

/* Integer in [0, n) by 32x32->64 multiply-shift (bias < n/2^32). */
static inline uint32_t below(uint32_t x, uint32_t n) {
  return (uint32_t)(((uint64_t)x * (uint64_t)n) >> 32);
}

/* Purposes (second key word). */
enum {
  P_VEC = 1, P_HAM_OFF = 2, P_HAM_VAL = 3, P_MESH_VAL = 4, P_MESH_EXTRA = 5,
  P_MESH_PERM = 6, P_FAM_PARAM = 7, P_FAM_LEN = 8, P_FAM_COL = 9, P_FAM_VAL = 10
};

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/* Sort (col, val) pairs of one row by column (insertion sort; rows are short
 * or already nearly sorted). */
static void sort_pairs(int32_t* c, double* v, int64_t n) {
  for (int64_t i = 1; i < n; ++i) {
    int32_t ci = c[i];
    double vi = v[i];
    int64_t j = i - 1;
    while (j >= 0 && c[j] > ci) {
      c[j + 1] = c[j];
      v[j + 1] = v[j];
      --j;
    }
    c[j + 1] = ci;
    v[j + 1] = vi;
  }
}

/* ---------------- dense vectors ---------------- */

/* out[i] = U[-1,1) keyed (seed, P_VEC), counter (i_lo, i_hi, stream, 0). */
void crsgen_uniform_vec(uint32_t seed, uint32_t stream, int64_t n, double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    uint32_t r[4];
    philox(seed, P_VEC, (uint32_t)i, (uint32_t)((uint64_t)i >> 32), stream, 0, r);
    out[i] = 2.0 * u01(r[0], r[1]) - 1.0;
  }
}

/* out[i] = integer in [lo, hi] (as double), for exactness tests. */
void crsgen_int_vec(uint32_t seed, uint32_t stream, int64_t n, int32_t lo, int32_t hi,
                    double* out) {
  uint32_t span = (uint32_t)(hi - lo + 1);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    uint32_t r[4];
    philox(seed, P_VEC, (uint32_t)i, (uint32_t)((uint64_t)i >> 32), stream, 1, r);
    out[i] = (double)(lo + (int32_t)below(r[0], span));
  }
}

/* ---------------- config 1: 2D 5-point Laplacian ---------------- */

/* m x m grid, natural (x fastest) order, diag 4, neighbours -1. */
void crsgen_laplace2d(int32_t m, int32_t* row_ptr, int32_t* col, double* val) {
  int64_t n = (int64_t)m * m, p = 0;
  row_ptr[0] = 0;
  for (int64_t i = 0; i < n; ++i) {
    int32_t x = (int32_t)(i % m), y = (int32_t)(i / m);
    if (y > 0) { col[p] = (int32_t)(i - m); val[p++] = -1.0; }
    if (x > 0) { col[p] = (int32_t)(i - 1); val[p++] = -1.0; }
    col[p] = (int32_t)i; val[p++] = 4.0;
    if (x < m - 1) { col[p] = (int32_t)(i + 1); val[p++] = -1.0; }
    if (y < m - 1) { col[p] = (int32_t)(i + m); val[p++] = -1.0; }
    row_ptr[i + 1] = (int32_t)p;
  }
}

/* 1D tridiag(-1, 2, -1) of size n. */
void crsgen_laplace1d(int32_t n, int32_t* row_ptr, int32_t* col, double* val) {
  int64_t p = 0;
  row_ptr[0] = 0;
  for (int32_t i = 0; i < n; ++i) {
    if (i > 0) { col[p] = i - 1; val[p++] = -1.0; }
    col[p] = i; val[p++] = 2.0;
    if (i < n - 1) { col[p] = i + 1; val[p++] = -1.0; }
    row_ptr[i + 1] = (int32_t)p;
  }
}

/* ---------------- config 2: Hamiltonian-like symmetric matrix ----------------
 * Diagonal plus 7 symmetric offset pairs +-d_k. Stratified log-uniform
 * offsets: d_k = round(exp((k + U_k)/7 * ln(N/2))), redrawn until all seven
 * are distinct, then sorted ascending. */
void crsgen_ham_offsets(uint32_t seed, int64_t n, int32_t d[7]) {
  double lmax = log((double)n / 2.0);
  for (int k = 0; k < 7; ++k) d[k] = 0;
  for (int k = 0; k < 7; ++k) {
    for (uint32_t attempt = 0;; ++attempt) {
      uint32_t r[4];
      philox(seed, P_HAM_OFF, (uint32_t)k, attempt, 0, 0, r);
      double u = u01(r[0], r[1]);
      double dv = floor(exp(((double)k + u) / 7.0 * lmax) + 0.5);
      if (dv < 1.0) dv = 1.0;
      if (dv > (double)(n / 2)) dv = (double)(n / 2);
      int32_t cand = (int32_t)dv;
      int dup = 0;
      for (int q = 0; q < k; ++q) dup |= (d[q] == cand);
      if (!dup) { d[k] = cand; break; }
    }
  }
  qsort(d, 7, sizeof(int32_t), cmp_i32);
}

void crsgen_ham_rowlens(int64_t n, const int32_t d[7], int32_t* lens) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    int32_t c = 1;
    for (int k = 0; k < 7; ++k) c += (i - d[k] >= 0) + (i + d[k] < n);
    lens[i] = c;
  }
}

/* a(i, i+d_k) = a(i+d_k, i) = N(0,1) keyed by the lower index i and k;
 * a(i,i) = N(0,1) keyed (i, 7). */
void crsgen_ham_fill(uint32_t seed, int64_t n, const int32_t d[7], const int32_t* row_ptr,
                     int32_t* col, double* val) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    int64_t p = row_ptr[i];
    uint32_t r[4];
    for (int k = 6; k >= 0; --k) {
      int64_t j = i - d[k];
      if (j >= 0) {
        philox(seed, P_HAM_VAL, (uint32_t)j, (uint32_t)k, 0, 0, r);
        col[p] = (int32_t)j; val[p++] = normal4(r);
      }
    }
    philox(seed, P_HAM_VAL, (uint32_t)i, 7u, 0, 0, r);
    col[p] = (int32_t)i; val[p++] = normal4(r);
    for (int k = 0; k < 7; ++k) {
      int64_t j = i + d[k];
      if (j < n) {
        philox(seed, P_HAM_VAL, (uint32_t)i, (uint32_t)k, 0, 0, r);
        col[p] = (int32_t)j; val[p++] = normal4(r);
      }
    }
  }
}

/* ---------------- config 3: permuted 3D 7-point stencil + random extras ----
 * Unpermuted row i (grid m^3, x fastest): stencil neighbours i+-1, i+-m,
 * i+-m^2 inside the grid with N(0,1) values; with probability `extra_ppm`/1e6
 * the row gains c ~ U{1..max_extra} extra entries at distinct uniformly random
 * columns that are not stencil columns, N(0,1) values; the diagonal is
 * 1 + sum |off-diagonal| of the row (dominant). Then rows and columns are
 * permuted symmetrically by a seeded permutation inside each block of `blk`
 * consecutive indices (last block shorter). */

static int mesh_stencil(int64_t i, int32_t m, int64_t* cols /*7*/, int* slots /*7*/) {
  int64_t mm = (int64_t)m * m;
  int32_t x = (int32_t)(i % m), y = (int32_t)((i / m) % m), z = (int32_t)(i / mm);
  int c = 0;
  if (z > 0) { cols[c] = i - mm; slots[c++] = 0; }
  if (y > 0) { cols[c] = i - m; slots[c++] = 1; }
  if (x > 0) { cols[c] = i - 1; slots[c++] = 2; }
  cols[c] = i; slots[c++] = 3;
  if (x < m - 1) { cols[c] = i + 1; slots[c++] = 4; }
  if (y < m - 1) { cols[c] = i + m; slots[c++] = 5; }
  if (z < m - 1) { cols[c] = i + mm; slots[c++] = 6; }
  return c;
}

static int mesh_extra_count(uint32_t seed, int64_t i, uint32_t extra_ppm, int32_t max_extra) {
  uint32_t r[4];
  philox(seed, P_MESH_EXTRA, (uint32_t)i, 0xFFFFFFFFu, 0, 0, r);
  if (below(r[0], 1000000u) >= extra_ppm) return 0;
  return 1 + (int)below(r[1], (uint32_t)max_extra);
}

/* p[new] = old, within blocks of blk (Fisher-Yates, keyed by block). */
void crsgen_block_perm(uint32_t seed, int64_t n, int32_t blk, int32_t* p) {
  int64_t nb = (n + blk - 1) / blk;
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < nb; ++b) {
    int64_t s = b * blk, e = s + blk < n ? s + blk : n, len = e - s;
    for (int64_t t = 0; t < len; ++t) p[s + t] = (int32_t)(s + t);
    for (int64_t t = len - 1; t > 0; --t) {
      uint32_t r[4];
      philox(seed, P_MESH_PERM, (uint32_t)b, (uint32_t)t, 0, 0, r);
      int64_t j = below(r[0], (uint32_t)(t + 1));
      int32_t tmp = p[s + t]; p[s + t] = p[s + j]; p[s + j] = tmp;
    }
  }
}

/* lens[new] for the permuted matrix (p from crsgen_block_perm, or NULL for
 * the unpermuted one). */
void crsgen_mesh_rowlens(uint32_t seed, int32_t m, uint32_t extra_ppm, int32_t max_extra,
                         const int32_t* p, int32_t* lens) {
  int64_t n = (int64_t)m * m * m;
#pragma omp parallel for schedule(static)
  for (int64_t ni = 0; ni < n; ++ni) {
    int64_t i = p ? p[ni] : ni;
    int64_t cols[7]; int slots[7];
    lens[ni] = mesh_stencil(i, m, cols, slots) + mesh_extra_count(seed, i, extra_ppm, max_extra);
  }
}

/* q[old] = new (inverse of p), or NULL for identity. */
void crsgen_mesh_fill(uint32_t seed, int32_t m, uint32_t extra_ppm, int32_t max_extra,
                      const int32_t* p, const int32_t* q, const int32_t* row_ptr,
                      int32_t* col, double* val) {
  int64_t n = (int64_t)m * m * m;
#pragma omp parallel for schedule(static)
  for (int64_t ni = 0; ni < n; ++ni) {
    int64_t i = p ? p[ni] : ni;
    int64_t sc[7]; int sl[7];
    int ns = mesh_stencil(i, m, sc, sl);
    int ne = mesh_extra_count(seed, i, extra_ppm, max_extra);
    int64_t base = row_ptr[ni];
    int32_t* c = col + base;
    double* v = val + base;
    uint32_t r[4];
    double offsum = 0.0;
    int dpos = -1, w = 0;
    for (int s = 0; s < ns; ++s) {
      c[w] = (int32_t)(q ? q[sc[s]] : sc[s]);
      if (sc[s] == i) { dpos = w; v[w++] = 0.0; continue; }
      philox(seed, P_MESH_VAL, (uint32_t)i, (uint32_t)sl[s], 0, 0, r);
      v[w] = normal4(r);
      offsum += fabs(v[w]);
      ++w;
    }
    /* extras: distinct uniform columns in [0,n), not stencil columns */
    uint32_t draw = 0;
    for (int e = 0; e < ne; ++e) {
      int64_t cand;
      for (;;) {
        philox(seed, P_MESH_EXTRA, (uint32_t)i, (uint32_t)e, draw++, 1, r);
        cand = (int64_t)(((uint64_t)r[0] << 32 | r[1]) % (uint64_t)n);
        int clash = 0;
        for (int s = 0; s < ns; ++s) clash |= (sc[s] == cand);
        for (int t = 0; t < e; ++t) {
          int64_t prev = p ? (int64_t)p[c[ns + t]] : (int64_t)c[ns + t];
          clash |= (prev == cand);
        }
        if (!clash) break;
      }
      c[w] = (int32_t)(q ? q[cand] : cand);
      philox(seed, P_MESH_VAL, (uint32_t)i, (uint32_t)(7 + e), 0, 0, r);
      v[w] = normal4(r);
      offsum += fabs(v[w]);
      ++w;
    }
    v[dpos] = 1.0 + offsum;
    sort_pairs(c, v, w);
  }
}

/* ---------------- config 5: matrix families ----------------
 * Matrix `id` of a seeded collection: N log-uniform in [nlo, nhi]; family
 * 0 = row lengths uniform{1..30}, 1 = power law P(l) ~ l^-2.1 on 1..5000,
 * 2 = banded with total width w in [3,64]. Uniform and power-law rows take
 * distinct uniformly random columns; banded rows take the contiguous window
 * [i - floor((w-1)/2), i + ceil((w-1)/2)] clipped to [0, N). */

#define PL_MAX 5000
static double pl_cdf[PL_MAX];
static int pl_ready = 0;

static void pl_init(void) {
  if (pl_ready) return;
  double s = 0.0;
  for (int l = 1; l <= PL_MAX; ++l) s += pow((double)l, -2.1);
  double acc = 0.0;
  for (int l = 1; l <= PL_MAX; ++l) {
    acc += pow((double)l, -2.1) / s;
    pl_cdf[l - 1] = acc;
  }
  pl_cdf[PL_MAX - 1] = 1.0;
  pl_ready = 1;
}

/* Exported for a statistics test: P(l <= L) for the power-law family. */
double crsgen_powerlaw_cdf(int32_t l) {
  pl_init();
  if (l < 1) return 0.0;
  if (l > PL_MAX) return 1.0;
  return pl_cdf[l - 1];
}

static int32_t pl_draw(double u) {
  int lo = 0, hi = PL_MAX - 1;
  while (lo < hi) {
    int mid = (lo + hi) / 2;
    if (pl_cdf[mid] > u) hi = mid; else lo = mid + 1;
  }
  return lo + 1;
}

/* params: out[0]=N, out[1]=family, out[2]=band width */
void crsgen_family_params(uint32_t seed, uint32_t id, double nlo, double nhi, int64_t out[3]) {
  uint32_t r[4], r2[4];
  philox(seed, P_FAM_PARAM, id, 0, 0, 0, r);
  philox(seed, P_FAM_PARAM, id, 1, 0, 0, r2);
  double u = u01(r[0], r[1]);
  double nv = floor(exp(log(nlo) + u * (log(nhi) - log(nlo))) + 0.5);
  out[0] = (int64_t)nv;
  out[1] = (int64_t)below(r[2], 3u);
  out[2] = 3 + (int64_t)below(r2[0], 62u);
}

static int32_t fam_len(uint32_t seed, uint32_t id, int64_t n, int family, int32_t w, int64_t i) {
  if (family == 2) {
    int64_t lo = i - (w - 1) / 2, hi = i + w / 2;
    if (lo < 0) lo = 0;
    if (hi > n - 1) hi = n - 1;
    return (int32_t)(hi - lo + 1);
  }
  uint32_t r[4];
  philox(seed, P_FAM_LEN, (uint32_t)i, id, 0, 0, r);
  int32_t l = family == 0 ? 1 + (int32_t)below(r[0], 30u) : pl_draw(u01(r[0], r[1]));
  return l > n ? (int32_t)n : l;
}

void crsgen_family_rowlens(uint32_t seed, uint32_t id, int64_t n, int32_t family, int32_t w,
                           int32_t* lens) {
  pl_init();
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) lens[i] = fam_len(seed, id, n, family, w, i);
}

void crsgen_family_fill(uint32_t seed, uint32_t id, int64_t n, int32_t family, int32_t w,
                        const int32_t* row_ptr, int32_t* col, double* val) {
  pl_init();
#pragma omp parallel
  {
    /* open-addressing set for Floyd's sampling; capacity >= 2 * 5000 */
    int32_t* set = (int32_t*)malloc(sizeof(int32_t) * 16384);
#pragma omp for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
      int64_t base = row_ptr[i];
      int32_t l = row_ptr[i + 1] - row_ptr[i];
      int32_t* c = col + base;
      double* v = val + base;
      uint32_t r[4];
      if (family == 2) {
        int64_t lo = i - (w - 1) / 2;
        if (lo < 0) lo = 0;
        for (int32_t t = 0; t < l; ++t) c[t] = (int32_t)(lo + t);
      } else {
        /* Floyd: l distinct values from [0, n) */
        uint32_t cap = 16;
        while (cap < 2u * (uint32_t)l) cap <<= 1;
        for (uint32_t s = 0; s < cap; ++s) set[s] = -1;
        int32_t cnt = 0;
        for (int64_t j = n - l; j < n; ++j) {
          philox(seed, P_FAM_COL, (uint32_t)i, id, (uint32_t)(j - (n - l)), 0, r);
          int32_t t = (int32_t)below(r[0], (uint32_t)(j + 1));
          /* insert t, or j if t present */
          uint32_t h = ((uint32_t)t * 2654435761u) & (cap - 1);
          int present = 0;
          while (set[h] != -1) {
            if (set[h] == t) { present = 1; break; }
            h = (h + 1) & (cap - 1);
          }
          int32_t ins = present ? (int32_t)j : t;
          h = ((uint32_t)ins * 2654435761u) & (cap - 1);
          while (set[h] != -1) h = (h + 1) & (cap - 1);
          set[h] = ins;
          c[cnt++] = ins;
        }
        qsort(c, (size_t)l, sizeof(int32_t), cmp_i32);
      }
      for (int32_t t = 0; t < l; ++t) {
        philox(seed, P_FAM_VAL, (uint32_t)i, id, (uint32_t)t, 0, r);
        v[t] = normal4(r);
      }
    }
    free(set);
  }
}

/* Number of OpenMP threads the generator uses; set_threads(0) keeps the
 * runtime default. Output never depends on it. */
int crsgen_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void crsgen_set_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}
