// Reverse Cuthill-McKee ordering (Cuthill & McKee 1969, reversed as proposed
// by George 1971) of the symmetrised sparsity pattern of a CRS matrix. The
// paper applies RCM to its Hamiltonian matrix to improve the locality of the
// B accesses (Sect. 1.3.1); here it is a host-side analysis step whose
// permutation the caller applies as P A P^T, P B, P^T C.
//
// Per connected component: start from a pseudo-peripheral vertex (George &
// Liu: repeat "BFS from the current vertex, move to a minimum-degree vertex
// of the last level" while the level count grows), then breadth-first search
// visiting the neighbours of each vertex in increasing degree order (ties by
// index). The concatenated order is reversed at the end.
#include <algorithm>
#include <cstdint>
#include <vector>

#include "common.hpp"

namespace spmv {
namespace {

struct Graph {
  std::vector<int64_t> ptr;
  std::vector<int32_t> adj;
  int64_t deg(int32_t v) const { return ptr[v + 1] - ptr[v]; }
};

// Pattern of A + A^T (or, with `both`, of the entries present in A and in
// A^T) without self loops and without duplicate edges.
Graph symmetrise(int64_t n, const int32_t* rp, const int32_t* ci, bool both) {
  // rows of A with self loops, out-of-range and repeated columns removed
  std::vector<int64_t> up(n + 1, 0);
  std::vector<int32_t> uc;
  uc.reserve(rp[n]);
  for (int64_t i = 0; i < n; ++i) {
    const size_t b = uc.size();
    for (int64_t j = rp[i]; j < rp[i + 1]; ++j)
      if (ci[j] != i && ci[j] >= 0 && ci[j] < n) uc.push_back(ci[j]);
    std::sort(uc.begin() + b, uc.end());
    uc.erase(std::unique(uc.begin() + b, uc.end()), uc.end());
    up[i + 1] = (int64_t)uc.size();
  }
  // every edge listed from both ends
  std::vector<int64_t> cnt(n + 1, 0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = up[i]; j < up[i + 1]; ++j) {
      ++cnt[i + 1];
      ++cnt[uc[j] + 1];
    }
  for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
  std::vector<int32_t> adj(cnt[n]);
  std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = up[i]; j < up[i + 1]; ++j) {
      adj[fill[i]++] = uc[j];
      adj[fill[uc[j]]++] = (int32_t)i;
    }
  // A + A^T: keep each neighbour once; A and A^T: keep neighbours listed twice
  Graph g;
  g.ptr.assign(n + 1, 0);
  int64_t w = 0;
  for (int64_t i = 0; i < n; ++i) {
    auto b = adj.begin() + cnt[i], e = adj.begin() + cnt[i + 1];
    std::sort(b, e);
    for (auto it = b; it != e;) {
      auto run = it;
      while (run != e && *run == *it) ++run;
      if (!both || run - it >= 2) adj[w++] = *it;
      it = run;
    }
    g.ptr[i + 1] = w;
  }
  adj.resize(w);
  g.adj.swap(adj);
  return g;
}

// BFS levels from `root` restricted to its component; returns the number of
// levels and fills `last_level` with the vertices of the deepest level.
int bfs_levels(const Graph& g, int32_t root, std::vector<int32_t>& mark, int32_t stamp,
               std::vector<int32_t>& queue, std::vector<int32_t>& last_level) {
  queue.clear();
  queue.push_back(root);
  mark[root] = stamp;
  size_t head = 0;
  int levels = 0;
  while (head < queue.size()) {
    const size_t end = queue.size();
    last_level.assign(queue.begin() + head, queue.begin() + end);
    ++levels;
    for (; head < end; ++head) {
      const int32_t v = queue[head];
      for (int64_t k = g.ptr[v]; k < g.ptr[v + 1]; ++k) {
        const int32_t u = g.adj[k];
        if (mark[u] != stamp) {
          mark[u] = stamp;
          queue.push_back(u);
        }
      }
    }
  }
  return levels;
}

}  // namespace
}  // namespace spmv

using namespace spmv;

extern "C" int spmv_rcm_order(int64_t n, const int32_t* row_ptr, const int32_t* col_idx,
                              int symmetric_part, int32_t* perm) {
  if (n < 0) return fail(SPMV_ERR_INVALID_ARG, "n < 0");
  if (n == 0) return SPMV_OK;
  if (!row_ptr || !perm || (row_ptr[n] > 0 && !col_idx))
    return fail(SPMV_ERR_INVALID_ARG, "null argument");
  if (n > INT32_MAX - 1) return fail(SPMV_ERR_UNSUPPORTED, "n too large");
  for (int64_t i = 0; i < n; ++i)
    if (row_ptr[i + 1] < row_ptr[i] || row_ptr[0] != 0)
      return fail(SPMV_ERR_BAD_CRS, "row_ptr must start at 0 and not decrease");
  const Graph g = symmetrise(n, row_ptr, col_idx, symmetric_part != 0);
  std::vector<int32_t> mark(n, -1), queue, last, order;
  std::vector<char> placed(n, 0);
  order.reserve(n);
  std::vector<int32_t> nbr;
  int32_t stamp = 0;
  for (int32_t seed = 0; seed < n; ++seed) {
    if (placed[seed]) continue;
    // pseudo-peripheral start vertex in this component
    int32_t root = seed;
    int levels = bfs_levels(g, root, mark, stamp++, queue, last);
    for (int it = 0; it < 3; ++it) {
      int32_t cand = last[0];
      for (int32_t v : last)
        if (g.deg(v) < g.deg(cand) || (g.deg(v) == g.deg(cand) && v < cand)) cand = v;
      const int lv = bfs_levels(g, cand, mark, stamp++, queue, last);
      if (lv <= levels) break;
      levels = lv;
      root = cand;
    }
    // Cuthill-McKee BFS from root, neighbours by increasing degree
    const size_t begin = order.size();
    order.push_back(root);
    placed[root] = 1;
    for (size_t head = begin; head < order.size(); ++head) {
      const int32_t v = order[head];
      nbr.clear();
      for (int64_t k = g.ptr[v]; k < g.ptr[v + 1]; ++k)
        if (!placed[g.adj[k]]) nbr.push_back(g.adj[k]);
      std::sort(nbr.begin(), nbr.end(), [&](int32_t a, int32_t b) {
        return g.deg(a) != g.deg(b) ? g.deg(a) < g.deg(b) : a < b;
      });
      for (int32_t u : nbr) {
        placed[u] = 1;
        order.push_back(u);
      }
    }
  }
  for (int64_t i = 0; i < n; ++i) perm[i] = order[n - 1 - i];
  return SPMV_OK;
}

namespace {
template <typename VT>
void permute_rows(int64_t n, const int32_t* rp, const int32_t* ci, const VT* val,
                  const int32_t* perm, const std::vector<int32_t>& inv, int32_t* rp_out,
                  int32_t* ci_out, VT* val_out) {
  rp_out[0] = 0;
  for (int64_t i = 0; i < n; ++i)
    rp_out[i + 1] = rp_out[i] + (rp[perm[i] + 1] - rp[perm[i]]);
  std::vector<std::pair<int32_t, VT>> tmp;
  for (int64_t i = 0; i < n; ++i) {
    const int32_t o = perm[i];
    tmp.clear();
    for (int32_t j = rp[o]; j < rp[o + 1]; ++j) tmp.emplace_back(inv[ci[j]], val[j]);
    std::stable_sort(tmp.begin(), tmp.end(),
                     [](const auto& a, const auto& b) { return a.first < b.first; });
    int32_t w = rp_out[i];
    for (const auto& t : tmp) {
      ci_out[w] = t.first;
      val_out[w++] = t.second;
    }
  }
}
}  // namespace

extern "C" int spmv_permute_crs(int64_t n, const int32_t* row_ptr, const int32_t* col_idx,
                                const void* val, int val_dtype, const int32_t* perm,
                                int32_t* row_ptr_out, int32_t* col_idx_out, void* val_out) {
  if (n < 0) return fail(SPMV_ERR_INVALID_ARG, "n < 0");
  if (!row_ptr || !perm || !row_ptr_out) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  if (val_dtype != SPMV_F64 && val_dtype != SPMV_F32) return fail(SPMV_ERR_INVALID_ARG, "bad dtype");
  const int64_t nnz = row_ptr[n];
  if (nnz > 0 && (!col_idx || !val || !col_idx_out || !val_out))
    return fail(SPMV_ERR_INVALID_ARG, "null argument");
  std::vector<int32_t> inv(n, -1);
  for (int64_t i = 0; i < n; ++i) {
    if (perm[i] < 0 || perm[i] >= n || inv[perm[i]] != -1)
      return fail(SPMV_ERR_INVALID_ARG, "perm is not a permutation");
    inv[perm[i]] = (int32_t)i;
  }
  for (int64_t j = 0; j < nnz; ++j)
    if (col_idx[j] < 0 || col_idx[j] >= n) return fail(SPMV_ERR_BAD_CRS, "column out of range");
  if (val_dtype == SPMV_F64)
    permute_rows(n, row_ptr, col_idx, static_cast<const double*>(val), perm, inv, row_ptr_out,
                 col_idx_out, static_cast<double*>(val_out));
  else
    permute_rows(n, row_ptr, col_idx, static_cast<const float*>(val), perm, inv, row_ptr_out,
                 col_idx_out, static_cast<float*>(val_out));
  return SPMV_OK;
}
