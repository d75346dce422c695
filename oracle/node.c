/*
 * Host baseline for the benchmark: the paper's node-level scheme for the CRS
 * product (Sect. 2), on all cores of the host that drives the GPU.
 *
 * TEST AND BENCHMARK INFRASTRUCTURE ONLY, like the oracle beside it: the
 * product library never calls, links or includes this file. It shares no
 * code with the GPU path.
 *
 * Scheme (Sect. 2): OpenMP threads share the row loop with a static
 * schedule, and every array is first written by the thread that later reads
 * it (a parallel copy with the same schedule), so that its pages are placed
 * in that thread's memory locality domain. B, read by every thread, is
 * placed by a static schedule over its own index. Each row is summed in the
 * order of the Sect. 1.2 loop, product rounded then sum rounded (built with
 * -ffp-contract=off), so C equals the single-threaded oracle bit for bit.
 *
 * Also a STREAM-style triad a = b + s c over float64 with the same placement,
 * the practical bandwidth ceiling the paper measures against (Sect. 2).
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

static double now_s(void) {
  struct timespec t;
  clock_gettime(CLOCK_MONOTONIC, &t);
  return (double)t.tv_sec + 1e-9 * (double)t.tv_nsec;
}

int node_threads(void) { return omp_get_max_threads(); }

/*
 * Copies the CRS triple and B into first-touched buffers, runs the product
 * until min_seconds have passed (at least one and at most max_reps times),
 * and copies the last C out. Host arrays; C has n_rows entries.
 * Returns 0, or -1 if an allocation failed. *reps and *seconds report the
 * timed products and their total time (the placement copy is not timed).
 */
int node_spmv_bench(int64_t n_rows, int64_t n_cols, const int32_t* row_ptr,
                    const int32_t* col_idx, const double* val, const double* B, double* C,
                    double min_seconds, int32_t max_reps, int32_t* reps, double* seconds) {
  const int64_t nnz = row_ptr[n_rows];
  int32_t* rp = aligned_alloc(64, (size_t)((n_rows + 1) * 4 + 64) / 64 * 64);
  int32_t* ci = aligned_alloc(64, (size_t)(nnz * 4 + 64) / 64 * 64);
  double* va = aligned_alloc(64, (size_t)(nnz * 8 + 64) / 64 * 64);
  double* b = aligned_alloc(64, (size_t)(n_cols * 8 + 64) / 64 * 64);
  double* c = aligned_alloc(64, (size_t)(n_rows * 8 + 64) / 64 * 64);
  if (!rp || !ci || !va || !b || !c) {
    free(rp), free(ci), free(va), free(b), free(c);
    return -1;
  }
  /* first touch: the rows (and their nonzeros) by the schedule of the product */
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n_rows; ++i) {
    rp[i] = row_ptr[i];
    c[i] = 0.0;
    for (int64_t j = row_ptr[i]; j < row_ptr[i + 1]; ++j) {
      ci[j] = col_idx[j];
      va[j] = val[j];
    }
  }
  rp[n_rows] = row_ptr[n_rows];
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < n_cols; ++j) b[j] = B[j];

  int32_t r = 0;
  double t = 0.0;
  do {
    const double t0 = now_s();
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_rows; ++i) {
      double acc = 0.0;
      for (int32_t j = rp[i]; j < rp[i + 1]; ++j) acc = acc + va[j] * b[ci[j]];
      c[i] = acc;
    }
    t += now_s() - t0;
    ++r;
  } while (t < min_seconds && r < max_reps);
  memcpy(C, c, (size_t)n_rows * 8);
  *reps = r;
  *seconds = t;
  free(rp), free(ci), free(va), free(b), free(c);
  return 0;
}

/*
 * Triad a[i] = b[i] + s c[i] over n float64, first-touched with the static
 * schedule; best of `reps` timed passes. *gbs = 24 n / best time (bytes read
 * and written, no write-allocate counted). Returns 0, -1 on allocation failure.
 */
int node_triad(int64_t n, int32_t reps, double* gbs) {
  double* a = aligned_alloc(64, (size_t)(n * 8 + 64) / 64 * 64);
  double* b = aligned_alloc(64, (size_t)(n * 8 + 64) / 64 * 64);
  double* c = aligned_alloc(64, (size_t)(n * 8 + 64) / 64 * 64);
  if (!a || !b || !c) {
    free(a), free(b), free(c);
    return -1;
  }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    a[i] = 0.0;
    b[i] = 1.0;
    c[i] = 2.0;
  }
  double best = 1e30;
  for (int32_t r = 0; r < reps; ++r) {
    const double t0 = now_s();
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) a[i] = b[i] + 3.0 * c[i];
    const double dt = now_s() - t0;
    if (dt < best) best = dt;
  }
  *gbs = 24.0 * (double)n / best / 1e9;
  free(a), free(b), free(c);
  return 0;
}
