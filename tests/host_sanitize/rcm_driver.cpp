// Host checks of the library's RCM ordering and symmetric permutation
// (spmv_rcm_order, spmv_permute_crs), meant to be built together with the
// library's reorder source under AddressSanitizer and UndefinedBehaviorSanitizer
// on the host code. Every call's status and output is checked; the program
// prints "rcm driver OK" and returns 0 when all checks hold.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <numeric>
#include <random>
#include <string>
#include <vector>

#include "spmv.h"

// The library's error recorder lives in its API source, which this driver
// does not link; the reorder code only needs the status passed through.
namespace spmv {
int fail(int status, const std::string&) { return status; }
}  // namespace spmv

namespace {

int g_bad = 0;

void expect(bool ok, const char* what) {
  if (!ok) {
    std::printf("FAILED: %s\n", what);
    ++g_bad;
  }
}

struct Crs {
  int64_t n = 0;
  std::vector<int32_t> rp{0}, ci;
  std::vector<double> va;
};

Crs grid(int mx, int my) {  // 5-point pattern of an mx x my grid
  Crs A;
  A.n = (int64_t)mx * my;
  for (int y = 0; y < my; ++y)
    for (int x = 0; x < mx; ++x) {
      const int i = y * mx + x;
      const int nb[5] = {i - mx, i - 1, i, i + 1, i + mx};
      const bool ok[5] = {y > 0, x > 0, true, x + 1 < mx, y + 1 < my};
      for (int k = 0; k < 5; ++k)
        if (ok[k]) {
          A.ci.push_back(nb[k]);
          A.va.push_back(k == 2 ? 4.0 : -1.0);
        }
      A.rp.push_back((int32_t)A.ci.size());
    }
  return A;
}

// Random pattern with empty rows, self loops, repeated and unsorted columns,
// and (with `wild`) columns out of range.
Crs random_crs(int64_t n, int maxlen, double empty_frac, bool wild, uint32_t seed) {
  std::mt19937 g(seed);
  std::uniform_real_distribution<double> u(0.0, 1.0);
  Crs A;
  A.n = n;
  for (int64_t i = 0; i < n; ++i) {
    const int len = u(g) < empty_frac ? 0 : (int)(g() % (maxlen + 1));
    for (int k = 0; k < len; ++k) {
      int64_t c = (int64_t)(g() % (uint32_t)n);
      if (k == 0 && u(g) < 0.2) c = i;  // self loop
      if (wild && u(g) < 0.05) c = (g() & 1) ? -1 - (int64_t)(g() % 5) : n + (g() % 5);
      A.ci.push_back((int32_t)c);
      A.va.push_back(u(g) - 0.5);
      if (u(g) < 0.1) {  // repeat the entry
        A.ci.push_back((int32_t)c);
        A.va.push_back(u(g));
      }
    }
    A.rp.push_back((int32_t)A.ci.size());
  }
  return A;
}

bool is_perm(const std::vector<int32_t>& p) {
  std::vector<char> seen(p.size(), 0);
  for (int32_t v : p) {
    if (v < 0 || (size_t)v >= p.size() || seen[v]) return false;
    seen[v] = 1;
  }
  return true;
}

// P A P^T against its definition: new row r is old row perm[r] with every
// column c mapped to inv[c], entries sorted by new column (stable).
void check_permute(const Crs& A, const std::vector<int32_t>& perm, const char* name) {
  const int64_t n = A.n, nnz = A.rp[n];
  std::vector<int32_t> rp(n + 1), ci(nnz);
  std::vector<double> va(nnz);
  std::vector<float> va32(nnz), in32(A.va.begin(), A.va.end());
  int st = spmv_permute_crs(n, A.rp.data(), A.ci.data(), A.va.data(), SPMV_F64, perm.data(),
                            rp.data(), ci.data(), va.data());
  expect(st == SPMV_OK, name);
  std::vector<int32_t> rp2(n + 1), ci2(nnz);
  st = spmv_permute_crs(n, A.rp.data(), A.ci.data(), in32.data(), SPMV_F32, perm.data(),
                        rp2.data(), ci2.data(), va32.data());
  expect(st == SPMV_OK && rp2 == rp && ci2 == ci, name);
  std::vector<int32_t> inv(n);
  for (int64_t r = 0; r < n; ++r) inv[perm[r]] = (int32_t)r;
  int64_t w = 0;
  for (int64_t r = 0; r < n; ++r) {
    const int32_t o = perm[r];
    std::vector<std::pair<int32_t, double>> e;
    for (int32_t j = A.rp[o]; j < A.rp[o + 1]; ++j) e.push_back({inv[A.ci[j]], A.va[j]});
    std::stable_sort(e.begin(), e.end(),
                     [](const auto& a, const auto& b) { return a.first < b.first; });
    expect(rp[r] == w, name);
    for (const auto& x : e) {
      expect(ci[w] == x.first && va[w] == x.second && va32[w] == (float)x.second, name);
      ++w;
    }
  }
  expect(rp[n] == nnz, name);
}

void rcm_case(const Crs& A, const char* name) {
  for (int sym = 0; sym < 2; ++sym) {
    std::vector<int32_t> perm(A.n, -7);
    const int st = spmv_rcm_order(A.n, A.rp.data(), A.ci.data(), sym, perm.data());
    expect(st == SPMV_OK, name);
    expect(is_perm(perm), name);
    if (st == SPMV_OK && is_perm(perm)) {
      bool in_range = true;
      for (int32_t c : A.ci) in_range = in_range && c >= 0 && c < A.n;
      if (in_range) check_permute(A, perm, name);
    }
  }
}

}  // namespace

int main() {
  rcm_case(grid(37, 23), "grid 37x23");
  rcm_case(grid(1, 50), "grid 1x50");
  rcm_case(random_crs(3000, 12, 0.2, false, 1), "random 3000");
  rcm_case(random_crs(20000, 6, 0.5, false, 2), "random 20000, half empty");
  rcm_case(random_crs(500, 40, 0.0, false, 3), "random 500, long rows");
  rcm_case(random_crs(800, 8, 0.1, true, 4), "columns out of range");  // RCM skips them
  Crs iso;  // isolated vertices only
  iso.n = 64;
  iso.rp.assign(65, 0);
  rcm_case(iso, "64 isolated vertices");
  Crs one;
  one.n = 1;
  one.rp = {0, 1};
  one.ci = {0};
  one.va = {2.0};
  rcm_case(one, "one row");

  // n = 0 succeeds and touches nothing
  expect(spmv_rcm_order(0, one.rp.data(), nullptr, 0, nullptr) == SPMV_OK, "n = 0");
  // errors
  std::vector<int32_t> perm(4);
  const int32_t bad_rp[5] = {0, 2, 1, 3, 3};
  const int32_t ci4[3] = {0, 1, 2};
  expect(spmv_rcm_order(-1, bad_rp, ci4, 0, perm.data()) == SPMV_ERR_INVALID_ARG, "n < 0");
  expect(spmv_rcm_order(4, bad_rp, ci4, 0, perm.data()) == SPMV_ERR_BAD_CRS, "row_ptr decreases");
  expect(spmv_rcm_order(4, nullptr, ci4, 0, perm.data()) == SPMV_ERR_INVALID_ARG, "null row_ptr");
  const Crs g = grid(3, 3);
  std::vector<int32_t> p9(9), rp(10), ci(g.ci.size());
  std::vector<double> va(g.ci.size());
  std::iota(p9.begin(), p9.end(), 0);
  p9[4] = 3;  // not a permutation
  expect(spmv_permute_crs(9, g.rp.data(), g.ci.data(), g.va.data(), SPMV_F64, p9.data(),
                          rp.data(), ci.data(), va.data()) == SPMV_ERR_INVALID_ARG,
         "perm not a permutation");
  std::iota(p9.begin(), p9.end(), 0);
  expect(spmv_permute_crs(9, g.rp.data(), g.ci.data(), g.va.data(), 7, p9.data(), rp.data(),
                          ci.data(), va.data()) == SPMV_ERR_INVALID_ARG,
         "bad dtype");
  Crs w = g;
  w.ci[5] = 9;  // column out of range
  expect(spmv_permute_crs(9, w.rp.data(), w.ci.data(), w.va.data(), SPMV_F64, p9.data(),
                          rp.data(), ci.data(), va.data()) == SPMV_ERR_BAD_CRS,
         "column out of range");
  if (g_bad) {
    std::printf("%d checks failed\n", g_bad);
    return 1;
  }
  std::printf("rcm driver OK\n");
  return 0;
}
