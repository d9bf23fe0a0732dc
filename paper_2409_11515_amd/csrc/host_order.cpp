// Fill-reducing column order for the LU of Algorithm 2: nested dissection of
// the symmetric pattern of A + A^T by recursive level-structure bisection.
//
// A piece of the graph is split by a breadth-first level structure grown
// from a pseudo-peripheral vertex: one level near the middle (the smallest
// level in the central band) is the separator, the levels before and after
// it are the two halves. Halves are ordered first, the separator last, so
// the fill of the factors stays inside the halves and the dense separator
// blocks. Separator vertices without a neighbour in the later half move to
// the earlier half (they separate nothing). Disconnected pieces are ordered
// one after another with no separator. Small pieces keep their natural order.

#include <algorithm>
#include <vector>

#include "internal.hpp"

namespace condest {

namespace {

struct Graph {
  int32_t n = 0;
  std::vector<int64_t> ptr;
  std::vector<int32_t> adj;
};

Graph symmetric_pattern(const HostCsr& a, const HostCsr& at) {
  Graph g;
  g.n = a.n;
  g.ptr.assign(a.n + 1, 0);
  g.adj.reserve(a.nnz() * 2);
  std::vector<int32_t> row;
  for (int32_t i = 0; i < a.n; ++i) {
    row.clear();
    for (int64_t p = a.rowptr[i]; p < a.rowptr[i + 1]; ++p)
      if (a.col[p] != i) row.push_back(a.col[p]);
    for (int64_t p = at.rowptr[i]; p < at.rowptr[i + 1]; ++p)
      if (at.col[p] != i) row.push_back(at.col[p]);
    std::sort(row.begin(), row.end());
    row.erase(std::unique(row.begin(), row.end()), row.end());
    g.adj.insert(g.adj.end(), row.begin(), row.end());
    g.ptr[i + 1] = static_cast<int64_t>(g.adj.size());
  }
  return g;
}

struct Piece {
  std::vector<int32_t> verts;
  int32_t lo;  // first output position of this piece
};

constexpr int32_t kLeaf = 96;

}  // namespace

void nested_dissection(const HostCsr& a, const HostCsr& at, std::vector<int32_t>& perm) {
  const int32_t n = a.n;
  Graph g = symmetric_pattern(a, at);
  perm.assign(n, -1);
  std::vector<int32_t> stamp(n, -1), level(n, -1);
  std::vector<int32_t> queue;
  queue.reserve(n);
  int32_t next_stamp = 0;

  // BFS restricted to vertices with stamp == s, from root; returns the number
  // reached and leaves the BFS order in queue, levels in level[].
  auto bfs = [&](int32_t s, int32_t root) {
    queue.clear();
    queue.push_back(root);
    level[root] = 0;
    size_t head = 0;
    const int32_t mark = -2 - s;  // visited marker distinct from any stamp
    stamp[root] = mark;
    while (head < queue.size()) {
      int32_t v = queue[head++];
      for (int64_t p = g.ptr[v]; p < g.ptr[v + 1]; ++p) {
        int32_t w = g.adj[p];
        if (stamp[w] == s) {
          stamp[w] = mark;
          level[w] = level[v] + 1;
          queue.push_back(w);
        }
      }
    }
    for (int32_t v : queue) stamp[v] = s;  // restore membership
    return queue.size();
  };
  auto degree_in = [&](int32_t v, int32_t s) {
    int32_t d = 0;
    for (int64_t p = g.ptr[v]; p < g.ptr[v + 1]; ++p) d += (stamp[g.adj[p]] == s);
    return d;
  };

  std::vector<Piece> stack;
  {
    Piece all;
    all.verts.resize(n);
    for (int32_t i = 0; i < n; ++i) all.verts[i] = i;
    all.lo = 0;
    stack.push_back(std::move(all));
  }
  while (!stack.empty()) {
    Piece pc = std::move(stack.back());
    stack.pop_back();
    const int32_t m = static_cast<int32_t>(pc.verts.size());
    if (m <= kLeaf) {
      std::sort(pc.verts.begin(), pc.verts.end());
      for (int32_t k = 0; k < m; ++k) perm[pc.lo + k] = pc.verts[k];
      continue;
    }
    const int32_t s = next_stamp++;
    for (int32_t v : pc.verts) stamp[v] = s;
    // pseudo-peripheral root: repeat BFS from a minimum-degree vertex of the last level
    int32_t root = pc.verts[0];
    size_t reached = bfs(s, root);
    int32_t ecc = level[queue.back()];
    for (int it = 0; it < 6 && reached == static_cast<size_t>(m); ++it) {
      int32_t last = level[queue.back()];
      int32_t best = queue.back(), bestd = 1 << 30;
      for (size_t k = queue.size(); k-- > 0 && level[queue[k]] == last;) {
        int32_t d = degree_in(queue[k], s);
        if (d < bestd || (d == bestd && queue[k] < best)) bestd = d, best = queue[k];
      }
      reached = bfs(s, best);
      int32_t e = level[queue.back()];
      if (e <= ecc) {
        if (e < ecc) reached = bfs(s, root);  // keep the deeper structure
        break;
      }
      ecc = e;
      root = best;
    }
    if (reached < static_cast<size_t>(m)) {
      // disconnected: the reached component first, the rest after it
      std::vector<int32_t> comp(queue.begin(), queue.end());
      for (int32_t v : comp) stamp[v] = -1;
      std::vector<int32_t> rest;
      rest.reserve(m - comp.size());
      for (int32_t v : pc.verts)
        if (stamp[v] == s) rest.push_back(v);
      for (int32_t v : pc.verts) stamp[v] = -1;
      Piece a1{std::move(comp), pc.lo};
      Piece a2{std::move(rest), pc.lo + static_cast<int32_t>(a1.verts.size())};
      stack.push_back(std::move(a2));
      stack.push_back(std::move(a1));
      continue;
    }
    const int32_t h = level[queue.back()];
    if (h < 2) {
      std::sort(pc.verts.begin(), pc.verts.end());
      for (int32_t k = 0; k < m; ++k) perm[pc.lo + k] = pc.verts[k];
      for (int32_t v : pc.verts) stamp[v] = -1;
      continue;
    }
    std::vector<int32_t> cnt(h + 1, 0);
    for (int32_t v : queue) cnt[level[v]]++;
    // separator level: smallest level whose preceding count lies in [0.3m, 0.7m]
    int32_t sep = -1, cum = 0;
    int64_t best_size = 1LL << 40;
    int32_t mid = -1;
    for (int32_t l = 0; l <= h; ++l) {
      if (mid < 0 && cum + cnt[l] >= m / 2) mid = l;
      if (l > 0 && l < h && cum >= (3 * static_cast<int64_t>(m)) / 10 &&
          cum <= (7 * static_cast<int64_t>(m)) / 10 && cnt[l] < best_size) {
        best_size = cnt[l];
        sep = l;
      }
      cum += cnt[l];
    }
    if (sep < 0) sep = std::min(std::max(mid, 1), h - 1);
    std::vector<int32_t> v1, v2, sv;
    for (int32_t v : queue) {
      int32_t l = level[v];
      if (l < sep) {
        v1.push_back(v);
      } else if (l > sep) {
        v2.push_back(v);
      } else {
        bool touches_later = false;
        for (int64_t p = g.ptr[v]; p < g.ptr[v + 1] && !touches_later; ++p) {
          int32_t w = g.adj[p];
          touches_later = (stamp[w] == s && level[w] == sep + 1);
        }
        (touches_later ? sv : v1).push_back(v);
      }
    }
    for (int32_t v : pc.verts) stamp[v] = -1;
    std::sort(sv.begin(), sv.end());
    const int32_t n1 = static_cast<int32_t>(v1.size()), n2 = static_cast<int32_t>(v2.size());
    for (size_t k = 0; k < sv.size(); ++k) perm[pc.lo + n1 + n2 + k] = sv[k];
    if (n2) stack.push_back(Piece{std::move(v2), pc.lo + n1});
    if (n1) stack.push_back(Piece{std::move(v1), pc.lo});
  }
}

}  // namespace condest

using namespace condest;

extern "C" int cond_order_nd(const cond_csr_t* A, int32_t* perm) {
  if (!perm) return fail(COND_EINVAL, "null perm");
  HostCsr a, at;
  int st = canonical_copy(A, a);
  if (st) return st;
  transpose(a, at);
  std::vector<int32_t> p;
  nested_dissection(a, at, p);
  std::copy(p.begin(), p.end(), perm);
  return COND_OK;
}
