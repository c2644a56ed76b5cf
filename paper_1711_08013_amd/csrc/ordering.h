// Host side of the band path: a bandwidth-reducing ordering of the reduced
// matrix P + sigma I + A'RA (the symbolic step of its factorisation; Section
// 3.1 orders the KKT matrix to limit fill before its LDL' factorisation).
//
// The pattern of P + A'A is the graph whose vertices are the variables and
// whose edges join two variables that share an entry of P or a row of A.
// Reverse Cuthill-McKee (Cuthill and McKee, 1969; George and Liu, 1981)
// numbers each connected component by breadth-first levels from a
// pseudo-peripheral start vertex (George-Liu search), neighbours by
// increasing degree, then reverses the numbering.  The half-bandwidth under
// the ordering decides whether the block-tridiagonal factor applies.
#pragma once

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <vector>

#include "osqp_mi.h"

namespace osqpmi {

// Adjacency (CSR, no self loops, no duplicates) of the pattern of P + A'A:
// the neighbours of variable j are the other columns of P's row j and of
// every row of A that holds j.  Returns false when some row of A has more
// than max_row entries (its clique alone would exceed the band the caller
// accepts).
inline bool reduced_pattern(const osqp_problem &p, int max_row, std::vector<int> &ptr,
                            std::vector<int> &adj) {
  const int n = p.n, m = p.m;
  for (int r = 0; r < m; ++r)
    if (p.A.indptr[r + 1] - p.A.indptr[r] > max_row) return false;
  // rows of A by column (the rows that hold each variable), and P's full
  // rows as neighbour lists
  std::vector<int> cptr(n + 1, 0), crow(p.A.nnz);
  for (int e = 0; e < p.A.nnz; ++e) cptr[p.A.indices[e] + 1]++;
  for (int j = 0; j < n; ++j) cptr[j + 1] += cptr[j];
  {
    std::vector<int> nx(cptr.begin(), cptr.end() - 1);
    for (int r = 0; r < m; ++r)
      for (int e = p.A.indptr[r]; e < p.A.indptr[r + 1]; ++e) crow[nx[p.A.indices[e]]++] = r;
  }
  std::vector<int> pptr(n + 1, 0), pcol;
  for (int i = 0; i < n; ++i)
    for (int e = p.P_upper.indptr[i]; e < p.P_upper.indptr[i + 1]; ++e) {
      const int j = p.P_upper.indices[e];
      if (j != i) { pptr[i + 1]++; pptr[j + 1]++; }
    }
  for (int j = 0; j < n; ++j) pptr[j + 1] += pptr[j];
  pcol.resize(pptr[n]);
  {
    std::vector<int> nx(pptr.begin(), pptr.end() - 1);
    for (int i = 0; i < n; ++i)
      for (int e = p.P_upper.indptr[i]; e < p.P_upper.indptr[i + 1]; ++e) {
        const int j = p.P_upper.indices[e];
        if (j != i) { pcol[nx[i]++] = j; pcol[nx[j]++] = i; }
      }
  }
  std::vector<int> mark(n, -1);
  ptr.assign(n + 1, 0);
  adj.clear();
  for (int j = 0; j < n; ++j) {
    mark[j] = j;
    for (int k = pptr[j]; k < pptr[j + 1]; ++k)
      if (mark[pcol[k]] != j) { mark[pcol[k]] = j; adj.push_back(pcol[k]); }
    for (int k = cptr[j]; k < cptr[j + 1]; ++k) {
      const int r = crow[k];
      for (int e = p.A.indptr[r]; e < p.A.indptr[r + 1]; ++e) {
        const int c = p.A.indices[e];
        if (mark[c] != j) { mark[c] = j; adj.push_back(c); }
      }
    }
    ptr[j + 1] = (int)adj.size();
  }
  return true;
}

// Breadth-first levels from `root` over the vertices not yet numbered;
// returns the eccentricity and leaves the last level in `last`.
inline int bfs_levels(int root, const std::vector<int> &ptr, const std::vector<int> &adj,
                      const std::vector<char> &numbered, std::vector<int> &level,
                      std::vector<int> &last) {
  std::vector<int> cur{root}, next;
  std::fill(level.begin(), level.end(), -1);
  level[root] = 0;
  int depth = 0;
  last = cur;
  while (!cur.empty()) {
    next.clear();
    for (int u : cur)
      for (int k = ptr[u]; k < ptr[u + 1]; ++k) {
        const int w = adj[k];
        if (!numbered[w] && level[w] < 0) { level[w] = depth + 1; next.push_back(w); }
      }
    if (next.empty()) break;
    ++depth;
    last = next;
    cur.swap(next);
  }
  return depth;
}

// perm[new position] = variable; returns the half-bandwidth of P + A'A under
// it (max |pos(u) - pos(v)| over the edges), or -1 if the pattern was
// refused (a row of A longer than max_row).
inline int rcm_ordering(const osqp_problem &p, int max_row, std::vector<int> &perm) {
  const int n = p.n;
  std::vector<int> ptr, adj;
  if (!reduced_pattern(p, max_row, ptr, adj)) return -1;
  auto deg = [&](int u) { return ptr[u + 1] - ptr[u]; };
  std::vector<char> numbered(n, 0);
  std::vector<int> level(n, -1), last, order;
  order.reserve(n);
  for (;;) {
    // start of the next component: an unnumbered vertex of least degree
    int root = -1;
    for (int u = 0; u < n; ++u)
      if (!numbered[u] && (root < 0 || deg(u) < deg(root))) root = u;
    if (root < 0) break;
    // pseudo-peripheral vertex: move to a least-degree vertex of the last
    // level while that increases the eccentricity
    int ecc = bfs_levels(root, ptr, adj, numbered, level, last);
    for (;;) {
      int cand = last[0];
      for (int u : last)
        if (deg(u) < deg(cand)) cand = u;
      std::vector<int> last2;
      const int e2 = bfs_levels(cand, ptr, adj, numbered, level, last2);
      if (e2 <= ecc) break;
      root = cand;
      ecc = e2;
      last.swap(last2);
    }
    // Cuthill-McKee numbering of this component from root
    size_t head = order.size();
    order.push_back(root);
    numbered[root] = 1;
    std::vector<int> nbrs;
    while (head < order.size()) {
      const int u = order[head++];
      nbrs.clear();
      for (int k = ptr[u]; k < ptr[u + 1]; ++k)
        if (!numbered[adj[k]]) nbrs.push_back(adj[k]);
      std::stable_sort(nbrs.begin(), nbrs.end(), [&](int a, int b) { return deg(a) < deg(b); });
      for (int w : nbrs) {
        numbered[w] = 1;
        order.push_back(w);
      }
    }
  }
  perm.assign(order.rbegin(), order.rend());
  std::vector<int> pos(n);
  for (int i = 0; i < n; ++i) pos[perm[i]] = i;
  int bw = 0;
  for (int u = 0; u < n; ++u)
    for (int k = ptr[u]; k < ptr[u + 1]; ++k) bw = std::max(bw, std::abs(pos[u] - pos[adj[k]]));
  return bw;
}

}  // namespace osqpmi
