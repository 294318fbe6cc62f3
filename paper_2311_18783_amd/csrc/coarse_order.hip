// Order of the coarse columns for the coarse Cholesky factor: nested
// dissection of the subdomain coupling graph (host code).
//
// Columns of subdomains i and j meet in E = Z^T A Z only if some free edge
// of Omega_i is coupled through A to some free edge of Omega_j; subdomains
// with no such pair never produce fill against each other until a common
// separator is eliminated.  Ordering each half of a bisection before the
// subdomains that separate the halves keeps the two halves' factor blocks
// independent: the block rows of the factor form a tree instead of a chain,
// so the sync-free triangular solves (which run every block row whose
// dependencies are done) and the factorisation work through independent
// branches at the same time.
#include <array>
#include <functional>
#include <numeric>

#include "precond.h"

namespace geneo {

std::vector<std::vector<int32_t>> subdomain_graph(const geneo_system* s, const geneo_decomp* dec) {
  const int N = dec->N;
  const int64_t n = s->n;
  // subdomains holding each free edge (CSR)
  std::vector<int64_t> sp(n + 1, 0);
  for (int i = 0; i < N; ++i)
    for (int64_t r = dec->dofs_ptr[i]; r < dec->dofs_ptr[i + 1]; ++r) sp[dec->dofs[r] + 1]++;
  for (int64_t e = 0; e < n; ++e) sp[e + 1] += sp[e];
  std::vector<int32_t> subs(sp[n]);
  {
    std::vector<int64_t> f(sp.begin(), sp.end() - 1);
    for (int i = 0; i < N; ++i)
      for (int64_t r = dec->dofs_ptr[i]; r < dec->dofs_ptr[i + 1]; ++r) subs[f[dec->dofs[r]]++] = i;
  }
  std::vector<std::vector<int32_t>> adj(N);
  parallel_for(N, [&](int j) {
    std::vector<uint8_t> seen(N, 0);
    seen[j] = 1;
    for (int64_t r = dec->dofs_ptr[j]; r < dec->dofs_ptr[j + 1]; ++r) {
      const int32_t e = dec->dofs[r];
      for (int32_t k = s->rowptr[e]; k < s->rowptr[e + 1]; ++k) {
        const int32_t f = s->colind[k];
        for (int64_t t = sp[f]; t < sp[f + 1]; ++t) {
          const int32_t i = subs[t];
          if (!seen[i]) {
            seen[i] = 1;
            adj[j].push_back(i);
          }
        }
      }
    }
    std::sort(adj[j].begin(), adj[j].end());
  });
  return adj;
}

// Minimum vertex separator between the two halves of a bisection: a minimum
// vertex cover of the bipartite graph of the edges that cross (Konig's
// theorem: from a maximum matching, the unmatched left vertices and what
// alternating paths reach from them; the cover is the unreached left
// vertices plus the reached right ones).
static std::vector<int32_t> min_separator(const std::vector<std::vector<int32_t>>& adj, const std::vector<int32_t>& A,
                                          std::vector<int8_t>& side) {
  std::vector<int32_t> L;                       // left vertices with a crossing edge
  std::vector<std::vector<int32_t>> nb;
  for (int32_t v : A) {
    std::vector<int32_t> x;
    for (int32_t u : adj[v])
      if (side[u] == 1) x.push_back(u);
    if (!x.empty()) {
      L.push_back(v);
      nb.push_back(std::move(x));
    }
  }
  const int nl = (int)L.size();
  const int N = (int)adj.size();
  std::vector<int32_t> match_r(N, -1), match_l(nl, -1);
  std::vector<int32_t> seen(N, -1);
  std::function<bool(int, int)> aug = [&](int li, int stamp) -> bool {
    for (int32_t u : nb[li]) {
      if (seen[u] == stamp) continue;
      seen[u] = stamp;
      if (match_r[u] < 0 || aug(match_r[u], stamp)) {
        match_r[u] = li;
        match_l[li] = u;
        return true;
      }
    }
    return false;
  };
  for (int li = 0; li < nl; ++li) aug(li, li);
  std::vector<uint8_t> vis_l(nl, 0), vis_r(N, 0);
  std::vector<int> stack;
  for (int li = 0; li < nl; ++li)
    if (match_l[li] < 0) {
      vis_l[li] = 1;
      stack.push_back(li);
    }
  while (!stack.empty()) {
    const int li = stack.back();
    stack.pop_back();
    for (int32_t u : nb[li]) {
      if (vis_r[u]) continue;
      vis_r[u] = 1;
      const int w = match_r[u];
      if (w >= 0 && !vis_l[w]) {
        vis_l[w] = 1;
        stack.push_back(w);
      }
    }
  }
  std::vector<int32_t> cover;
  for (int li = 0; li < nl; ++li)
    if (!vis_l[li]) cover.push_back(L[li]);
  for (int32_t u = 0; u < N; ++u)
    if (vis_r[u]) cover.push_back(u);
  return cover;
}

// Nested dissection: recursive coordinate bisection of the subdomains by
// their centroids, each bisection separated by a minimum vertex separator.
// Returns the groups in elimination order (the two halves' groups, then the
// separator): leaves of at most `leaf` subdomains and separators.
std::vector<std::vector<int32_t>> nested_dissection(const std::vector<std::vector<int32_t>>& adj,
                                                    const std::vector<std::array<double, 3>>& ctr, int leaf,
                                                    int* levels) {
  const int N = (int)adj.size();
  std::vector<std::vector<int32_t>> groups;
  std::vector<int8_t> side(N, -1);
  int depth_max = 0;
  std::function<void(std::vector<int32_t>, int)> rec = [&](std::vector<int32_t> S, int depth) {
    depth_max = std::max(depth_max, depth);
    if ((int)S.size() <= leaf) {
      std::sort(S.begin(), S.end());
      groups.push_back(std::move(S));
      return;
    }
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int32_t v : S)
      for (int a = 0; a < 3; ++a) {
        lo[a] = std::min(lo[a], ctr[v][a]);
        hi[a] = std::max(hi[a], ctr[v][a]);
      }
    int ax = 0;
    for (int a = 1; a < 3; ++a)
      if (hi[a] - lo[a] > hi[ax] - lo[ax]) ax = a;
    std::stable_sort(S.begin(), S.end(), [&](int32_t a, int32_t b) { return ctr[a][ax] < ctr[b][ax]; });
    const size_t h = S.size() / 2;
    std::vector<int32_t> A(S.begin(), S.begin() + h), B(S.begin() + h, S.end());
    for (int32_t v : A) side[v] = 0;
    for (int32_t v : B) side[v] = 1;
    std::vector<int32_t> sep = min_separator(adj, A, side);
    for (int32_t v : S) side[v] = -1;
    std::vector<uint8_t> in_sep(N, 0);
    for (int32_t v : sep) in_sep[v] = 1;
    auto drop = [&](std::vector<int32_t>& X) {
      X.erase(std::remove_if(X.begin(), X.end(), [&](int32_t v) { return in_sep[v] != 0; }), X.end());
    };
    drop(A);
    drop(B);
    if (A.empty() || B.empty()) {   // nothing separates: keep the part whole
      std::sort(S.begin(), S.end());
      groups.push_back(std::move(S));
      return;
    }
    rec(std::move(A), depth + 1);
    rec(std::move(B), depth + 1);
    std::sort(sep.begin(), sep.end());
    groups.push_back(std::move(sep));
  };
  std::vector<int32_t> all(N);
  std::iota(all.begin(), all.end(), 0);
  rec(all, 0);
  if (levels) *levels = depth_max;
  return groups;
}

std::vector<std::vector<int32_t>> subdomain_elimination_order(const geneo_system* s, const geneo_decomp* dec,
                                                              int* levels, std::vector<std::vector<int32_t>>* adj_out) {
  const int N = dec->N;
  std::vector<std::array<double, 3>> ctr(N, std::array<double, 3>{0.0, 0.0, 0.0});
  for (int i = 0; i < N; ++i) {
    const int64_t b = dec->dofs_ptr[i], e = dec->dofs_ptr[i + 1];
    for (int64_t r = b; r < e; ++r) {
      const int32_t g = s->free_edges[dec->dofs[r]];
      for (int q = 0; q < 2; ++q) {
        const int32_t v = s->edges[2 * (int64_t)g + q];
        for (int a = 0; a < 3; ++a) ctr[i][a] += s->xyz[3 * (int64_t)v + a];
      }
    }
    const double w = e > b ? 1.0 / (2.0 * (double)(e - b)) : 0.0;
    for (int a = 0; a < 3; ++a) ctr[i][a] *= w;
  }
  std::vector<std::vector<int32_t>> adj = subdomain_graph(s, dec);
  auto groups = nested_dissection(adj, ctr, 2, levels);
  if (adj_out) *adj_out = std::move(adj);
  return groups;
}

// Longest chain of dependent 128-column block rows in the triangular solves
// of E, predicted from the subdomains of its columns: pos_sub[p] = the
// subdomain of the column at factor position p (-1: a pad).  Block rows I > J
// couple if some column of I and some column of J belong to the same or to
// adjacent subdomains (E's entries between other columns are zero); the
// symbolic fill of that pattern gives the factor's block structure.
int predicted_solve_depth(const std::vector<int32_t>& pos_sub, const std::vector<std::vector<int32_t>>& adj) {
  const int64_t npos = (int64_t)pos_sub.size();
  const int nb = (int)((npos + NB - 1) / NB);
  const int N = (int)adj.size();
  std::vector<std::vector<int32_t>> tile_sub(nb);
  for (int64_t p = 0; p < npos; ++p) {
    const int32_t i = pos_sub[p];
    auto& t = tile_sub[p / NB];
    if (i >= 0 && (t.empty() || t.back() != i)) t.push_back(i);
  }
  std::vector<uint8_t> pat((size_t)nb * nb, 0);
  std::vector<int32_t> mark(N, -1);
  for (int I = 0; I < nb; ++I) {
    for (int32_t a : tile_sub[I]) {
      mark[a] = I;
      for (int32_t b : adj[a]) mark[b] = I;
    }
    for (int J = 0; J <= I; ++J)
      for (int32_t b : tile_sub[J])
        if (mark[b] == I) {
          pat[(size_t)I * nb + J] = 1;
          break;
        }
  }
  symbolic_fill(nb, pat);
  std::vector<int32_t> depth(nb, 1);
  int dmax = nb ? 1 : 0;
  for (int I = 0; I < nb; ++I) {
    for (int J = 0; J < I; ++J)
      if (pat[(size_t)I * nb + J]) depth[I] = std::max(depth[I], depth[J] + 1);
    dmax = std::max(dmax, depth[I]);
  }
  return dmax;
}

}  // namespace geneo
