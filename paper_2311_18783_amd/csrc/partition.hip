// Overlapping decomposition (host integer work): non-overlapping cell
// partition (boxes, recursive coordinate bisection or given), growth by
// layers of vertex-adjacent cells, subdomain dof sets N_i, the partition of
// unity D_i, and the local gradient columns G_i with floating components
// detected.
#include <algorithm>
#include <cmath>
#include <functional>
#include <numeric>

#include "internal.h"

namespace geneo {

static std::vector<double> cell_centroids(const geneo_system* s) {
  std::vector<double> c(3 * s->n_cells, 0.0);
  std::vector<int64_t> cnt(s->n_cells, 0);
  for (int64_t t = 0; t < s->n_tets; ++t) {
    int32_t cl = s->cell_of_tet[t];
    for (int d = 0; d < 3; ++d) {
      double m = 0;
      for (int k = 0; k < 4; ++k) m += s->xyz[3 * (int64_t)s->tets[4 * t + k] + d];
      c[3 * cl + d] += m / 4.0;
    }
    cnt[cl]++;
  }
  for (int64_t cl = 0; cl < s->n_cells; ++cl)
    for (int d = 0; d < 3; ++d) c[3 * cl + d] /= (double)cnt[cl];
  return c;
}

static std::vector<int32_t> box_partition(const geneo_system* s, const int32_t p[3]) {
  for (int a = 0; a < 3; ++a)
    if (p[a] < 1) throw Error(GENEO_EINVAL, "box partition counts must be >= 1");
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t v = 0; v < s->n_nodes; ++v)
    for (int d = 0; d < 3; ++d) {
      lo[d] = std::min(lo[d], s->xyz[3 * v + d]);
      hi[d] = std::max(hi[d], s->xyz[3 * v + d]);
    }
  auto c = cell_centroids(s);
  std::vector<int32_t> part(s->n_cells);
  for (int64_t cl = 0; cl < s->n_cells; ++cl) {
    int64_t idx[3];
    for (int a = 0; a < 3; ++a) {
      double f = std::floor((c[3 * cl + a] - lo[a]) / (hi[a] - lo[a]) * p[a]);
      idx[a] = std::min<int64_t>(std::max<int64_t>((int64_t)f, 0), p[a] - 1);
    }
    part[cl] = (int32_t)(idx[0] + p[0] * (idx[1] + p[1] * idx[2]));
  }
  return part;
}

// Recursive coordinate bisection: split along the axis of largest centroid
// extent (lowest axis on ties), cells ordered by (coordinate, id); the left
// child gets floor(k/2) parts and clip(round(n*floor(k/2)/k*(1+jitter)),
// floor(k/2), n-ceil(k/2)) cells; one jitter value per split in preorder.
static std::vector<int32_t> rcb_partition(const geneo_system* s, int32_t nparts, const double* jitter) {
  if (nparts < 1 || nparts > s->n_cells) throw Error(GENEO_EINVAL, "RCB part count out of range");
  auto c = cell_centroids(s);
  std::vector<int32_t> part(s->n_cells, -1);
  int32_t next = 0, jidx = 0;
  std::function<void(std::vector<int32_t>&, int32_t)> rec = [&](std::vector<int32_t>& cells, int32_t k) {
    if (k == 1) {
      for (auto cl : cells) part[cl] = next;
      ++next;
      return;
    }
    double d = jitter ? jitter[jidx] : 0.0;
    ++jidx;
    double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
    for (auto cl : cells)
      for (int a = 0; a < 3; ++a) {
        mn[a] = std::min(mn[a], c[3 * cl + a]);
        mx[a] = std::max(mx[a], c[3 * cl + a]);
      }
    int axis = 0;
    for (int a = 1; a < 3; ++a)
      if (mx[a] - mn[a] > mx[axis] - mn[axis]) axis = a;
    std::sort(cells.begin(), cells.end(), [&](int32_t x, int32_t y) {
      double cx = c[3 * x + axis], cy = c[3 * y + axis];
      return cx < cy || (cx == cy && x < y);
    });
    int32_t kl = k / 2, kr = k - k / 2;
    int64_t n = (int64_t)cells.size();
    int64_t nl = (int64_t)std::floor((double)n * kl / k * (1.0 + d) + 0.5);
    nl = std::min<int64_t>(std::max<int64_t>(nl, kl), n - kr);
    std::vector<int32_t> L(cells.begin(), cells.begin() + nl), R(cells.begin() + nl, cells.end());
    rec(L, kl);
    rec(R, kr);
  };
  std::vector<int32_t> all(s->n_cells);
  std::iota(all.begin(), all.end(), 0);
  rec(all, nparts);
  return part;
}

static int32_t find_root(std::vector<int32_t>& uf, int32_t x) {
  while (uf[x] != x) {
    uf[x] = uf[uf[x]];
    x = uf[x];
  }
  return x;
}

void build_decomposition(const geneo_system* s, const geneo_partition_opts* o, geneo_decomp* dec) {
  std::vector<int32_t> part;
  if (o->kind == GENEO_PART_BOX) {
    part = box_partition(s, o->box);
  } else if (o->kind == GENEO_PART_RCB) {
    part = rcb_partition(s, o->nparts, o->rcb_jitter);
  } else if (o->kind == GENEO_PART_EXPLICIT) {
    if (!o->part_of_cell) throw Error(GENEO_EINVAL, "explicit partition needs part_of_cell");
    part.assign(o->part_of_cell, o->part_of_cell + s->n_cells);
  } else {
    throw Error(GENEO_EINVAL, "unknown partition kind");
  }
  if (o->overlap < 0) throw Error(GENEO_EINVAL, "overlap must be >= 0");
  int32_t N = 0;
  for (auto p : part) {
    if (p < 0) throw Error(GENEO_EINVAL, "negative part id");
    N = std::max(N, p + 1);
  }
  std::vector<int64_t> sz(N, 0);
  for (auto p : part) sz[p]++;
  for (int32_t i = 0; i < N; ++i)
    if (sz[i] == 0) throw Error(GENEO_EINVAL, "empty part " + std::to_string(i));
  dec->N = N;
  dec->overlap = o->overlap;
  dec->part_of_cell = part;

  const int64_t H = s->n_cells, V = s->n_nodes, T = s->n_tets;
  // cell -> tets, cell -> nodes, node -> cells (CSR)
  std::vector<int64_t> ct_ptr(H + 1, 0);
  for (int64_t t = 0; t < T; ++t) ct_ptr[s->cell_of_tet[t] + 1]++;
  for (int64_t c = 0; c < H; ++c) ct_ptr[c + 1] += ct_ptr[c];
  std::vector<int32_t> ct(T);
  {
    std::vector<int64_t> f(ct_ptr.begin(), ct_ptr.end() - 1);
    for (int64_t t = 0; t < T; ++t) ct[f[s->cell_of_tet[t]]++] = (int32_t)t;
  }
  std::vector<int64_t> cn_ptr(H + 1, 0);
  std::vector<int32_t> cn;
  for (int64_t c = 0; c < H; ++c) {
    std::vector<int32_t> nodes;
    for (int64_t k = ct_ptr[c]; k < ct_ptr[c + 1]; ++k)
      for (int q = 0; q < 4; ++q) nodes.push_back(s->tets[4 * (int64_t)ct[k] + q]);
    std::sort(nodes.begin(), nodes.end());
    nodes.erase(std::unique(nodes.begin(), nodes.end()), nodes.end());
    cn.insert(cn.end(), nodes.begin(), nodes.end());
    cn_ptr[c + 1] = (int64_t)cn.size();
  }
  std::vector<int64_t> nc_ptr(V + 1, 0);
  for (auto v : cn) nc_ptr[v + 1]++;
  for (int64_t v = 0; v < V; ++v) nc_ptr[v + 1] += nc_ptr[v];
  std::vector<int32_t> nc(cn.size());
  {
    std::vector<int64_t> f(nc_ptr.begin(), nc_ptr.end() - 1);
    for (int64_t c = 0; c < H; ++c)
      for (int64_t k = cn_ptr[c]; k < cn_ptr[c + 1]; ++k) nc[f[cn[k]]++] = (int32_t)c;
  }

  const int ell = o->overlap;
  std::vector<int32_t> level(H, -1);   // reset per subdomain via touched lists
  std::vector<int32_t> node_level(V, INT32_MAX);
  std::vector<int32_t> f2l(s->n, -1);
  std::vector<std::vector<double>> chi(N);
  dec->dofs_ptr.assign(1, 0);
  dec->cells_ptr.assign(1, 0);
  dec->gn_ptr.assign(1, 0);
  dec->n_dropped.assign(N, 0);
  dec->p_all.assign(N, 0);
  std::vector<int32_t> members(N);
  std::vector<std::vector<int32_t>> cells_of(N);
  for (int64_t c = 0; c < H; ++c) cells_of[part[c]].push_back((int32_t)c);

  for (int32_t i = 0; i < N; ++i) {
    std::vector<int32_t> cur = cells_of[i];
    for (auto c : cur) level[c] = 0;
    std::vector<int32_t> all = cur;
    for (int d = 1; d <= ell; ++d) {
      std::vector<int32_t> nxt;
      for (auto c : cur)
        for (int64_t k = cn_ptr[c]; k < cn_ptr[c + 1]; ++k) {
          int32_t v = cn[k];
          for (int64_t q = nc_ptr[v]; q < nc_ptr[v + 1]; ++q) {
            int32_t c2 = nc[q];
            if (level[c2] < 0) {
              level[c2] = d;
              nxt.push_back(c2);
            }
          }
        }
      // a cell adjacent to any cell of the grown set: the frontier above only
      // expands from the previous layer, which reaches the same cells because
      // cells deeper inside share no vertex with new cells
      all.insert(all.end(), nxt.begin(), nxt.end());
      cur.swap(nxt);
    }
    std::sort(all.begin(), all.end());
    // tets, dofs, nodal levels
    std::vector<int32_t> dofs;
    std::vector<int32_t> touched_nodes;
    for (auto c : all) {
      for (int64_t k = ct_ptr[c]; k < ct_ptr[c + 1]; ++k) {
        int64_t t = ct[k];
        for (int p = 0; p < 6; ++p) {
          int32_t fe = s->edge_to_free[s->tet_edges[6 * t + p]];
          if (fe >= 0) dofs.push_back(fe);
        }
      }
      for (int64_t k = cn_ptr[c]; k < cn_ptr[c + 1]; ++k) {
        int32_t v = cn[k];
        if (node_level[v] == INT32_MAX) touched_nodes.push_back(v);
        node_level[v] = std::min(node_level[v], level[c]);
      }
    }
    std::sort(dofs.begin(), dofs.end());
    dofs.erase(std::unique(dofs.begin(), dofs.end()), dofs.end());
    chi[i].resize(dofs.size());
    for (size_t r = 0; r < dofs.size(); ++r) {
      int32_t e = s->free_edges[dofs[r]];
      int32_t a = s->edges[2 * (int64_t)e], b = s->edges[2 * (int64_t)e + 1];
      double ca = ell ? 1.0 - (double)node_level[a] / ell : 1.0;
      double cb = ell ? 1.0 - (double)node_level[b] / ell : 1.0;
      chi[i][r] = 0.5 * (ca + cb);
    }
    // local free-node columns of G_i: free nodes touched by N_i, ascending
    std::vector<int32_t> gn;
    for (auto fe : dofs) {
      int32_t e = s->free_edges[fe];
      for (int q = 0; q < 2; ++q) {
        int32_t fn = s->node_to_free[s->edges[2 * (int64_t)e + q]];
        if (fn >= 0) gn.push_back(fn);
      }
    }
    std::sort(gn.begin(), gn.end());
    gn.erase(std::unique(gn.begin(), gn.end()), gn.end());
    dec->p_all[i] = (int64_t)gn.size();
    // floating components: union-find over edges with two free ends
    std::vector<int32_t> uf(gn.size());
    std::iota(uf.begin(), uf.end(), 0);
    std::vector<char> anchored(gn.size(), 0);
    auto lidx = [&](int32_t fn) { return (int32_t)(std::lower_bound(gn.begin(), gn.end(), fn) - gn.begin()); };
    for (auto fe : dofs) {
      int32_t e = s->free_edges[fe];
      int32_t fa = s->node_to_free[s->edges[2 * (int64_t)e]], fb = s->node_to_free[s->edges[2 * (int64_t)e + 1]];
      if (fa >= 0 && fb >= 0) {
        int32_t ra = find_root(uf, lidx(fa)), rb = find_root(uf, lidx(fb));
        if (ra != rb) uf[std::max(ra, rb)] = std::min(ra, rb);
      }
    }
    for (auto fe : dofs) {
      int32_t e = s->free_edges[fe];
      int32_t fa = s->node_to_free[s->edges[2 * (int64_t)e]], fb = s->node_to_free[s->edges[2 * (int64_t)e + 1]];
      if ((fa >= 0) != (fb >= 0)) anchored[find_root(uf, lidx(fa >= 0 ? fa : fb))] = 1;
    }
    std::vector<char> drop(gn.size(), 0);
    std::vector<char> seen(gn.size(), 0);
    for (size_t k = 0; k < gn.size(); ++k) {
      int32_t r = find_root(uf, (int32_t)k);
      if (!anchored[r] && !seen[r]) {  // first (lowest) member of a floating component
        seen[r] = 1;
        drop[k] = 1;
        dec->n_dropped[i]++;
      }
    }
    for (size_t k = 0; k < gn.size(); ++k)
      if (!drop[k]) dec->gnodes.push_back(gn[k]);
    dec->gn_ptr.push_back((int64_t)dec->gnodes.size());
    dec->dofs.insert(dec->dofs.end(), dofs.begin(), dofs.end());
    dec->dofs_ptr.push_back((int64_t)dec->dofs.size());
    dec->cells.insert(dec->cells.end(), all.begin(), all.end());
    dec->cells_ptr.push_back((int64_t)dec->cells.size());
    for (auto c : all) level[c] = -1;
    for (auto v : touched_nodes) node_level[v] = INT32_MAX;
  }
  // partition of unity D_i = chi_i / sum_j chi_j
  std::vector<double> tot(s->n, 0.0);
  for (int32_t i = 0; i < N; ++i)
    for (int64_t r = dec->dofs_ptr[i]; r < dec->dofs_ptr[i + 1]; ++r) tot[dec->dofs[r]] += chi[i][r - dec->dofs_ptr[i]];
  dec->pou.resize(dec->dofs.size());
  for (int32_t i = 0; i < N; ++i)
    for (int64_t r = dec->dofs_ptr[i]; r < dec->dofs_ptr[i + 1]; ++r) {
      double t = tot[dec->dofs[r]];
      if (!(t > 0)) throw Error(GENEO_EINVAL, "partition of unity undefined on an edge");
      dec->pou[r] = chi[i][r - dec->dofs_ptr[i]] / t;
    }
  (void)members;
  (void)f2l;
}

}  // namespace geneo
