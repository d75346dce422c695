/*
 * CPU oracle for CRS sparse matrix-vector multiplication.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library calls, links or
 * includes this file; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load it. It shares no code with the GPU path.
 *
 * Built with -O1 -ffp-contract=off: every product is rounded, then every
 * sum is rounded, in the order the loops below state. Single-threaded.
 *
 * Index base: 0 (the paper's listing is 1-based Fortran); row_ptr and
 * col_idx are int32 (the paper's 4-byte index), values float64 (8 bytes).
 */
#include <math.h>
#include <stdint.h>

/* Status codes, numerically equal to the library's documented ones. */
#define ORC_OK 0
#define ORC_BAD_CRS (-2)

/*
 * Structural validity of a CRS triple (Sect. 1.2: val/col_idx hold the
 * nonzeros row by row, row_ptr the start offset of every row):
 * row_ptr[0] = 0, row_ptr nondecreasing, row_ptr[n_rows] = nnz, and
 * 0 <= col_idx[j] < n_cols for every stored entry.
 */
int oracle_check_crs(int64_t n_rows, int64_t n_cols, int64_t nnz, const int32_t* row_ptr,
                     const int32_t* col_idx) {
  if (row_ptr[0] != 0) return ORC_BAD_CRS;
  for (int64_t i = 0; i < n_rows; ++i)
    if (row_ptr[i + 1] < row_ptr[i]) return ORC_BAD_CRS;
  if ((int64_t)row_ptr[n_rows] != nnz) return ORC_BAD_CRS;
  for (int64_t j = 0; j < nnz; ++j)
    if (col_idx[j] < 0 || (int64_t)col_idx[j] >= n_cols) return ORC_BAD_CRS;
  return ORC_OK;
}

/*
 * C = A*B, the loop of Sect. 1.2 with C starting from zero:
 *   for each row i:  for j in [row_ptr[i], row_ptr[i+1]):
 *                       C(i) = C(i) + val(j) * B(col_idx(j))
 * S[i] = sum_j |val(j) * B(col_idx(j))|, the magnitude sum that scales the
 * rounding-error bound of the row (may be NULL).
 */
void oracle_spmv(int64_t n_rows, const int32_t* row_ptr, const int32_t* col_idx,
                 const double* val, const double* B, double* C, double* S) {
  for (int64_t i = 0; i < n_rows; ++i) {
    double acc = 0.0, mag = 0.0;
    for (int64_t j = row_ptr[i]; j < row_ptr[i + 1]; ++j) {
      double prod = val[j] * B[col_idx[j]];
      acc = acc + prod;
      mag = mag + fabs(prod);
    }
    C[i] = acc;
    if (S) S[i] = mag;
  }
}

/*
 * Multi-RHS form: the same loop for every column c < k of a row-major
 * right-hand-side block, C[i*ldc + c] = sum_j val(j) * B[col_idx(j)*ldb + c].
 * S has the layout of C with leading dimension k (may be NULL).
 */
void oracle_spmm(int64_t n_rows, int32_t k, const int32_t* row_ptr, const int32_t* col_idx,
                 const double* val, const double* B, int64_t ldb, double* C, int64_t ldc,
                 double* S) {
  for (int32_t c = 0; c < k; ++c) {
    for (int64_t i = 0; i < n_rows; ++i) {
      double acc = 0.0, mag = 0.0;
      for (int64_t j = row_ptr[i]; j < row_ptr[i + 1]; ++j) {
        double prod = val[j] * B[(int64_t)col_idx[j] * ldb + c];
        acc = acc + prod;
        mag = mag + fabs(prod);
      }
      C[i * ldc + c] = acc;
      if (S) S[i * (int64_t)k + c] = mag;
    }
  }
}

/*
 * Row-statistics features of a CRS pattern, as defined for the kernel-variant
 * selector (no counterpart in the paper; the average row length N_nzr is the
 * paper's Sect. 1.2 quantity). With l_i = row length, N = n_rows:
 *  f0  log2(max(N,1))          f1  log2(max(nnz,1))
 *  f2  mean l = nnz/N          f3  population std of l
 *  f4  log2(max l + 1)         f5  min l
 *  f6  frac rows l == 0        f7  frac rows 1 <= l <= 4
 *  f8  frac rows 5..16         f9  frac rows 17..64
 *  f10 frac rows 65..1024      f11 frac rows > 1024
 *  f12 frac of nnz in rows with l > 64
 *  f13 mean over nnz of floor(log2(1 + |col - row|))
 *  f14 frac of nnz with |col - row| <= 64
 *  f15 max l / mean l (0 when nnz == 0)
 * All sums are exact integers; the final divisions are done in double.
 * N == 0 gives all zeros.
 */
void oracle_row_features(int64_t n_rows, const int32_t* row_ptr, const int32_t* col_idx,
                         double* f) {
  for (int q = 0; q < 16; ++q) f[q] = 0.0;
  if (n_rows <= 0) return;
  uint64_t nnz = 0, sum_sq = 0, bins[6] = {0, 0, 0, 0, 0, 0}, long_nnz = 0;
  uint64_t dist_log_sum = 0, near = 0;
  int64_t lmax = 0, lmin = INT64_MAX;
  for (int64_t i = 0; i < n_rows; ++i) {
    int64_t l = (int64_t)row_ptr[i + 1] - row_ptr[i];
    nnz += (uint64_t)l;
    sum_sq += (uint64_t)l * (uint64_t)l;
    if (l > lmax) lmax = l;
    if (l < lmin) lmin = l;
    int b = l == 0 ? 0 : l <= 4 ? 1 : l <= 16 ? 2 : l <= 64 ? 3 : l <= 1024 ? 4 : 5;
    bins[b] += 1;
    if (l > 64) long_nnz += (uint64_t)l;
    for (int64_t j = row_ptr[i]; j < row_ptr[i + 1]; ++j) {
      int64_t d = (int64_t)col_idx[j] - i;
      if (d < 0) d = -d;
      /* floor(log2(1 + d)) by repeated halving */
      uint64_t v = (uint64_t)d + 1;
      int lg = 0;
      while (v > 1) { v >>= 1; ++lg; }
      dist_log_sum += (uint64_t)lg;
      if (d <= 64) near += 1;
    }
  }
  double N = (double)n_rows, Z = (double)nnz;
  double mean = Z / N;
  double var = (double)sum_sq / N - mean * mean;
  f[0] = log2(N);
  f[1] = log2(Z > 1.0 ? Z : 1.0);
  f[2] = mean;
  f[3] = var > 0.0 ? sqrt(var) : 0.0;
  f[4] = log2((double)lmax + 1.0);
  f[5] = (double)lmin;
  for (int b = 0; b < 6; ++b) f[6 + b] = (double)bins[b] / N;
  if (nnz > 0) {
    f[12] = (double)long_nnz / Z;
    f[13] = (double)dist_log_sum / Z;
    f[14] = (double)near / Z;
    f[15] = (double)lmax / mean;
  }
}
