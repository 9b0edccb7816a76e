// Mesh ingest on the host: validation, ordering and the SELL-64 layout.
//
// The paper leaves the ILU(0) ordering unstated (section "Solution Update": L and U
// take the pattern of A).  Here the ordering is a colouring (independent sets, taken in
// ascending colour), which is what lets every cell of one colour be processed in
// parallel on the GPU:
//   AUTO       two colours when the cell graph is bipartite (every hex passage), else
//              GREEDY;
//   BIPARTITE  breadth-first two-colouring from the lowest uncoloured id (error if the
//              graph has an odd cycle);
//   GREEDY     first-fit colouring visiting cells in reverse Cuthill-McKee order;
//   USER       the caller's colours (must be a proper colouring).
// Internally cells are renumbered colour-major, and inside each colour by their reverse
// Cuthill-McKee position, so the 64 rows of a tile are neighbours in the mesh and the
// neighbour gathers of a tile touch a narrow window of the vectors.
#include "layout.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <queue>
#include <sstream>

namespace fnlh {

namespace {

struct Csr {
  std::vector<int64_t> ptr;
  std::vector<int32_t> nbr;
  std::vector<int64_t> eid;  // directed coupling id: 2e (a->b) or 2e+1 (b->a)
};

Csr adjacency(int64_t N, int64_t E, const int32_t* edges) {
  Csr g;
  g.ptr.assign(N + 1, 0);
  for (int64_t e = 0; e < E; ++e) {
    g.ptr[edges[2 * e] + 1]++;
    g.ptr[edges[2 * e + 1] + 1]++;
  }
  for (int64_t i = 0; i < N; ++i) g.ptr[i + 1] += g.ptr[i];
  g.nbr.resize(2 * E);
  g.eid.resize(2 * E);
  std::vector<int64_t> fill(g.ptr.begin(), g.ptr.end() - 1);
  for (int64_t e = 0; e < E; ++e) {
    int32_t a = edges[2 * e], b = edges[2 * e + 1];
    g.nbr[fill[a]] = b;
    g.eid[fill[a]++] = 2 * e;
    g.nbr[fill[b]] = a;
    g.eid[fill[b]++] = 2 * e + 1;
  }
  // neighbour lists sorted by neighbour id (deterministic regardless of edge order)
  for (int64_t i = 0; i < N; ++i) {
    int64_t s = g.ptr[i], t = g.ptr[i + 1];
    std::vector<std::pair<int32_t, int64_t>> v;
    v.reserve(t - s);
    for (int64_t p = s; p < t; ++p) v.emplace_back(g.nbr[p], g.eid[p]);
    std::sort(v.begin(), v.end());
    for (int64_t p = s; p < t; ++p) {
      g.nbr[p] = v[p - s].first;
      g.eid[p] = v[p - s].second;
    }
  }
  return g;
}

// Reverse Cuthill-McKee over every connected component.  Each component starts from a
// pseudo-peripheral cell (two BFS sweeps from its minimum-degree cell); neighbours are
// visited by ascending degree, ties by id.
std::vector<int32_t> rcm_order(int64_t N, const Csr& g) {
  std::vector<int32_t> order;
  order.reserve(N);
  std::vector<char> seen(N, 0);
  std::vector<int32_t> deg(N);
  for (int64_t i = 0; i < N; ++i) deg[i] = (int32_t)(g.ptr[i + 1] - g.ptr[i]);
  std::vector<int32_t> level(N, -1);
  auto bfs_last = [&](int32_t s, std::vector<int32_t>& comp) {
    comp.clear();
    std::queue<int32_t> q;
    q.push(s);
    level[s] = 0;
    comp.push_back(s);
    int32_t last = s;
    while (!q.empty()) {
      int32_t i = q.front();
      q.pop();
      last = i;
      for (int64_t p = g.ptr[i]; p < g.ptr[i + 1]; ++p) {
        int32_t k = g.nbr[p];
        if (level[k] < 0) {
          level[k] = level[i] + 1;
          q.push(k);
          comp.push_back(k);
        }
      }
    }
    // farthest cell of minimum degree on the last level
    int32_t best = last;
    for (int32_t c : comp)
      if (level[c] == level[last] && (deg[c] < deg[best] || (deg[c] == deg[best] && c < best))) best = c;
    for (int32_t c : comp) level[c] = -1;
    return best;
  };
  std::vector<int32_t> comp;
  for (int64_t s0 = 0; s0 < N; ++s0) {
    if (seen[s0]) continue;
    // component of s0: find its min-degree cell
    bfs_last((int32_t)s0, comp);
    int32_t start = comp[0];
    for (int32_t c : comp)
      if (deg[c] < deg[start] || (deg[c] == deg[start] && c < start)) start = c;
    start = bfs_last(start, comp);
    start = bfs_last(start, comp);
    // Cuthill-McKee from start
    size_t head = order.size();
    order.push_back(start);
    seen[start] = 1;
    std::vector<int32_t> nb;
    while (head < order.size()) {
      int32_t i = order[head++];
      nb.clear();
      for (int64_t p = g.ptr[i]; p < g.ptr[i + 1]; ++p)
        if (!seen[g.nbr[p]]) nb.push_back(g.nbr[p]);
      std::sort(nb.begin(), nb.end(), [&](int32_t x, int32_t y) {
        return deg[x] < deg[y] || (deg[x] == deg[y] && x < y);
      });
      for (int32_t k : nb) {
        seen[k] = 1;
        order.push_back(k);
      }
    }
  }
  std::reverse(order.begin(), order.end());
  return order;
}

bool bipartite_colour(int64_t N, const Csr& g, std::vector<int32_t>& col) {
  col.assign(N, -1);
  std::queue<int32_t> q;
  for (int64_t s = 0; s < N; ++s) {
    if (col[s] >= 0) continue;
    col[s] = 0;
    q.push((int32_t)s);
    while (!q.empty()) {
      int32_t i = q.front();
      q.pop();
      for (int64_t p = g.ptr[i]; p < g.ptr[i + 1]; ++p) {
        int32_t k = g.nbr[p];
        if (col[k] < 0) {
          col[k] = 1 - col[i];
          q.push(k);
        } else if (col[k] == col[i]) {
          return false;
        }
      }
    }
  }
  return true;
}

void greedy_colour(int64_t N, const Csr& g, const std::vector<int32_t>& visit, std::vector<int32_t>& col) {
  col.assign(N, -1);
  std::vector<int32_t> mark;
  for (int32_t i : visit) {
    mark.assign(g.ptr[i + 1] - g.ptr[i] + 2, 0);
    for (int64_t p = g.ptr[i]; p < g.ptr[i + 1]; ++p) {
      int32_t c = col[g.nbr[p]];
      if (c >= 0 && c < (int32_t)mark.size()) mark[c] = 1;
    }
    int32_t c = 0;
    while (mark[c]) ++c;
    col[i] = c;
  }
}

}  // namespace

int build_layout(const fnlh_mesh& m, const fnlh_options& o, Layout& L, std::string& err) {
  std::ostringstream es;
  const int64_t N = m.n_cells, E = m.n_edges, B = m.n_bfaces;
  if (N <= 0 || E < 0 || B < 0 || m.n_zones < 1) {
    err = "mesh: need n_cells > 0, n_edges >= 0, n_bfaces >= 0, n_zones >= 1";
    return FNLH_E_ARG;
  }
  if (N >= (int64_t)1 << 30 || E >= (int64_t)1 << 29) {
    err = "mesh: too large for 32-bit internal indices";
    return FNLH_E_ARG;
  }
  if ((E > 0 && (!m.edges || !m.area)) || !m.volume || (B > 0 && (!m.bface_cell || !m.bface_area))) {
    err = "mesh: null array";
    return FNLH_E_ARG;
  }
  if (o.storage < FNLH_F64 || o.storage > FNLH_BF16 || o.outer < FNLH_OUTER_EXACT ||
      o.outer > FNLH_OUTER_STORED || o.ordering < FNLH_ORDER_AUTO || o.ordering > FNLH_ORDER_USER ||
      o.factor_slots < 0) {
    err = "options: value out of range";
    return FNLH_E_ARG;
  }
  if (o.ordering == FNLH_ORDER_USER && !o.user_colour) {
    err = "options: ordering USER needs user_colour";
    return FNLH_E_ARG;
  }
  for (int64_t e = 0; e < E; ++e) {
    int64_t a = m.edges[2 * e], b = m.edges[2 * e + 1];
    if (a < 0 || a >= N || b < 0 || b >= N) {
      es << "mesh: edge " << e << " has a cell id out of range";
      err = es.str();
      return FNLH_E_MESH;
    }
    if (a == b) {
      es << "mesh: edge " << e << " is a self loop";
      err = es.str();
      return FNLH_E_MESH;
    }
    for (int d = 0; d < 3; ++d)
      if (!std::isfinite(m.area[3 * e + d])) {
        es << "mesh: edge " << e << " has a non-finite area";
        err = es.str();
        return FNLH_E_MESH;
      }
  }
  for (int64_t i = 0; i < N; ++i) {
    if (!(m.volume[i] > 0.0) || !std::isfinite(m.volume[i])) {
      es << "mesh: volume of cell " << i << " is not positive";
      err = es.str();
      return FNLH_E_MESH;
    }
    if (m.zone && (m.zone[i] < 0 || m.zone[i] >= m.n_zones)) {
      es << "mesh: zone of cell " << i << " out of range";
      err = es.str();
      return FNLH_E_MESH;
    }
  }
  for (int64_t f = 0; f < B; ++f) {
    if (m.bface_cell[f] < 0 || m.bface_cell[f] >= N) {
      es << "mesh: boundary face " << f << " has a cell id out of range";
      err = es.str();
      return FNLH_E_MESH;
    }
  }
  Csr g = adjacency(N, E, m.edges);
  for (int64_t i = 0; i < N; ++i)
    for (int64_t p = g.ptr[i] + 1; p < g.ptr[i + 1]; ++p)
      if (g.nbr[p] == g.nbr[p - 1]) {
        es << "mesh: duplicate edge between cells " << i << " and " << g.nbr[p];
        err = es.str();
        return FNLH_E_MESH;
      }

  L.N = N;
  L.E = E;
  L.B = B;
  L.n_zones = m.n_zones;
  std::vector<int32_t> rcm = rcm_order(N, g);
  std::vector<int32_t>& col = L.colour_user;
  if (o.ordering == FNLH_ORDER_USER) {
    col.assign(o.user_colour, o.user_colour + N);
    for (int64_t i = 0; i < N; ++i)
      if (col[i] < 0) {
        err = "ordering: negative user colour";
        return FNLH_E_MESH;
      }
    for (int64_t e = 0; e < E; ++e)
      if (col[m.edges[2 * e]] == col[m.edges[2 * e + 1]]) {
        es << "ordering: user colouring is not proper (edge " << e << ")";
        err = es.str();
        return FNLH_E_MESH;
      }
    // compact colour values, keeping their order
    std::vector<int32_t> vals(col);
    std::sort(vals.begin(), vals.end());
    vals.erase(std::unique(vals.begin(), vals.end()), vals.end());
    for (auto& c : col) c = (int32_t)(std::lower_bound(vals.begin(), vals.end(), c) - vals.begin());
    L.bipartite = vals.size() == 2;
  } else {
    bool bip = false;
    if (o.ordering == FNLH_ORDER_AUTO || o.ordering == FNLH_ORDER_BIPARTITE) {
      bip = bipartite_colour(N, g, col);
      if (!bip && o.ordering == FNLH_ORDER_BIPARTITE) {
        err = "ordering: cell graph is not bipartite";
        return FNLH_E_MESH;
      }
    }
    if (!bip) greedy_colour(N, g, rcm, col);
    int32_t mx = 0;
    for (auto c : col) mx = std::max(mx, c);
    L.bipartite = bip || mx == 1;
  }
  int32_t ncol = 0;
  for (auto c : col) ncol = std::max(ncol, c + 1);
  L.n_colours = ncol;

  // colour-major, RCM position inside each colour; every colour is padded to a
  // multiple of 64 rows so tile t is rows [64t, 64t+64) and never straddles a colour
  std::vector<int32_t> rpos(N);
  for (int64_t p = 0; p < N; ++p) rpos[rcm[p]] = (int32_t)p;
  std::vector<int32_t> byc(N);
  std::iota(byc.begin(), byc.end(), 0);
  std::stable_sort(byc.begin(), byc.end(), [&](int32_t x, int32_t y) {
    return col[x] < col[y] || (col[x] == col[y] && rpos[x] < rpos[y]);
  });
  std::vector<int64_t> count(ncol, 0);
  for (auto c : col) count[c]++;
  L.cstart.assign(ncol + 1, 0);
  L.ccount = count;
  for (int32_t c = 0; c < ncol; ++c) L.cstart[c + 1] = L.cstart[c] + (count[c] + kTile - 1) / kTile * kTile;
  const int64_t NP = L.cstart[ncol];
  L.NP = NP;
  L.perm.assign(N, -1);
  L.iperm.assign(NP, -1);
  {
    int64_t p = 0;
    for (int32_t c = 0; c < ncol; ++c) {
      for (int64_t k = 0; k < count[c]; ++k, ++p) {
        const int32_t u = byc[p];
        const int64_t row = L.cstart[c] + k;
        L.perm[u] = (int32_t)row;
        L.iperm[row] = u;
      }
    }
  }

  // tiles
  L.n_tiles = NP / kTile;
  L.ctile.assign(ncol + 1, 0);
  for (int32_t c = 0; c <= ncol; ++c) L.ctile[c] = L.cstart[c] / kTile;
  L.tile_nrows.assign(L.n_tiles, 0);
  L.tile_width.assign(L.n_tiles, 0);
  L.tile_slot0.assign(L.n_tiles, 0);
  int64_t slot = 0;
  for (int64_t t = 0; t < L.n_tiles; ++t) {
    int32_t nr = 0, w = 0;
    for (int32_t l = 0; l < kTile; ++l) {
      const int32_t u = L.iperm[t * kTile + l];
      if (u < 0) continue;
      ++nr;
      w = std::max<int32_t>(w, (int32_t)(g.ptr[u + 1] - g.ptr[u]));
    }
    L.tile_nrows[t] = nr;
    L.tile_width[t] = w;
    L.tile_slot0[t] = slot;
    slot += w;
  }
  L.n_slots = slot;
  if (slot * kTile >= ((int64_t)1 << 31)) {
    err = "mesh: too many couplings for 32-bit entry indices";
    return FNLH_E_ARG;
  }
  const int64_t nent = slot * kTile;
  L.ent_nbr.assign(nent, 0);
  L.ent_edge.assign(nent, 0);
  L.ent_rev.assign(nent, -1);
  L.edge_ent.assign(2 * E, -1);
  for (int64_t t = 0; t < L.n_tiles; ++t) {
    for (int32_t l = 0; l < kTile; ++l) {
      const int64_t row = t * kTile + l;
      const int32_t u = L.iperm[row];
      const int64_t deg = u >= 0 ? g.ptr[u + 1] - g.ptr[u] : 0;
      for (int32_t j = 0; j < L.tile_width[t]; ++j) {
        const int64_t f = (L.tile_slot0[t] + j) * kTile + l;
        if (j < deg) {
          const int64_t p = g.ptr[u] + j;
          const int64_t d = g.eid[p];
          L.ent_nbr[f] = L.perm[g.nbr[p]];
          const int64_t e = d >> 1;
          L.ent_edge[f] = (d & 1) ? -(int32_t)(e + 1) : (int32_t)(e + 1);
          L.edge_ent[d] = f;
        } else {
          L.ent_nbr[f] = (int32_t)row;  // zero block: contributes nothing
        }
      }
    }
  }
  for (int64_t d = 0; d < 2 * E; ++d) L.ent_rev[L.edge_ent[d]] = (int32_t)L.edge_ent[d ^ 1];

  L.c_deg.assign(ncol, 0);
  L.c_deg_upper.assign(ncol, 0);
  L.c_nbr.assign(ncol, 0);
  L.c_nbr_lower.assign(ncol, 0);
  L.c_nbr_upper.assign(ncol, 0);
  {
    std::vector<int32_t> stamp(N, -1);
    for (int64_t p = 0; p < N; ++p) {
      const int32_t u = byc[p];
      const int32_t c = col[u];
      for (int64_t q = g.ptr[u]; q < g.ptr[u + 1]; ++q) {
        const int32_t k = g.nbr[q];
        L.c_deg[c]++;
        if (col[k] > c) L.c_deg_upper[c]++;
        if (stamp[k] != c) {
          stamp[k] = c;
          L.c_nbr[c]++;
          if (col[k] < c) L.c_nbr_lower[c]++;
          else L.c_nbr_upper[c]++;
        }
      }
    }
  }

  L.vol.assign(NP, 1.0);
  L.zone.assign(NP, 0);
  for (int64_t u = 0; u < N; ++u) {
    L.vol[L.perm[u]] = m.volume[u];
    L.zone[L.perm[u]] = m.zone ? m.zone[u] : 0;
  }
  L.bf_ptr.assign(NP + 1, 0);
  for (int64_t f = 0; f < B; ++f) L.bf_ptr[L.perm[m.bface_cell[f]] + 1]++;
  for (int64_t i = 0; i < NP; ++i) L.bf_ptr[i + 1] += L.bf_ptr[i];
  L.bf_idx.resize(B);
  {
    std::vector<int32_t> fill(L.bf_ptr.begin(), L.bf_ptr.end() - 1);
    for (int64_t f = 0; f < B; ++f) L.bf_idx[fill[L.perm[m.bface_cell[f]]]++] = (int32_t)f;
  }
  return FNLH_OK;
}

int build_pilu(const Layout& L, const std::vector<int32_t>& part, int32_t unit_rows, PiluLayout& P,
               std::string& err) {
  const int64_t N = L.N;
  if ((int64_t)part.size() != N) {
    err = "partition-local ILU: one partition label per cell needed";
    return FNLH_E_ARG;
  }
  if (L.n_slots * kTile >= (int64_t)INT32_MAX) {
    err = "partition-local ILU: mesh too large for 32-bit entry indices";
    return FNLH_E_ARG;
  }
  P = PiluLayout();
  // in-partition neighbours of user cell u, as (neighbour id, flat SELL entry)
  auto each_coupling = [&](int64_t u, auto&& f) {
    const int64_t row = L.perm[u];
    const int64_t t = row / kTile;
    const int lane = (int)(row % kTile);
    for (int q = 0; q < L.tile_width[t]; ++q) {
      const int64_t fe = (L.tile_slot0[t] + q) * kTile + lane;
      if (L.ent_edge[fe] == 0) continue;
      const int32_t v = L.iperm[L.ent_nbr[fe]];
      if (part[v] == part[u]) f(v, fe);
    }
  };
  // partitions by ascending label
  std::vector<int32_t> labels(part.begin(), part.end());
  std::sort(labels.begin(), labels.end());
  labels.erase(std::unique(labels.begin(), labels.end()), labels.end());
  P.n_parts = (int64_t)labels.size();
  std::vector<int32_t> pidx(N);
  std::vector<int64_t> psize(P.n_parts, 0);
  for (int64_t u = 0; u < N; ++u) {
    pidx[u] = (int32_t)(std::lower_bound(labels.begin(), labels.end(), part[u]) - labels.begin());
    psize[pidx[u]]++;
  }
  for (int64_t k = 0; k < P.n_parts; ++k) P.max_part = std::max<int32_t>(P.max_part, (int32_t)psize[k]);
  // work units: consecutive partitions while they fit in unit_rows cells
  std::vector<int32_t> unit_of(P.n_parts);
  {
    int64_t rows = 0, u = -1;
    for (int64_t k = 0; k < P.n_parts; ++k) {
      if (u < 0 || rows + psize[k] > std::max<int64_t>(unit_rows, 1)) {
        ++u;
        rows = 0;
      }
      unit_of[k] = (int32_t)u;
      rows += psize[k];
    }
    P.n_units = u + 1;
  }
  // levels, visiting cells by ascending id (the natural order inside every partition)
  std::vector<int32_t> level(N, 0);
  for (int64_t u = 0; u < N; ++u) {
    int32_t lv = 0;
    each_coupling(u, [&](int32_t v, int64_t) {
      if (v < u) lv = std::max(lv, level[v] + 1);
    });
    level[u] = lv;
  }
  // positions: unit, then (level, partition, id)
  std::vector<int32_t> cells(N);
  std::iota(cells.begin(), cells.end(), 0);
  std::stable_sort(cells.begin(), cells.end(), [&](int32_t a, int32_t b) {
    const int32_t ua = unit_of[pidx[a]], ub = unit_of[pidx[b]];
    if (ua != ub) return ua < ub;
    if (level[a] != level[b]) return level[a] < level[b];
    return pidx[a] < pidx[b];
  });
  std::vector<int32_t> pos_of(N);
  for (int64_t q = 0; q < N; ++q) pos_of[cells[q]] = (int32_t)q;
  P.unit_ptr.assign(P.n_units + 1, 0);
  for (int64_t k = 0; k < P.n_parts; ++k) P.unit_ptr[unit_of[k] + 1] += (int32_t)psize[k];
  for (int64_t w = 0; w < P.n_units; ++w) {
    P.max_rows = std::max(P.max_rows, P.unit_ptr[w + 1]);
    P.unit_ptr[w + 1] += P.unit_ptr[w];
  }
  P.unit_lev.assign(P.n_units + 1, 0);
  P.lev_ptr.assign(1, 0);
  for (int64_t w = 0; w < P.n_units; ++w) {
    const int32_t a = P.unit_ptr[w], b = P.unit_ptr[w + 1];
    for (int32_t q = a; q < b; ++q)
      if (q + 1 == b || level[cells[q + 1]] != level[cells[q]]) P.lev_ptr.push_back(q + 1);
    P.unit_lev[w + 1] = (int32_t)P.lev_ptr.size() - 1;
    P.max_levels = std::max(P.max_levels, P.unit_lev[w + 1] - P.unit_lev[w]);
  }
  // packed couplings per group of 64 positions, lower neighbours first
  P.n_groups = (N + kTile - 1) / kTile;
  P.pos_row.assign(P.n_groups * kTile, -1);
  for (int64_t q = 0; q < N; ++q) P.pos_row[q] = L.perm[cells[q]];
  P.g_width.assign(P.n_groups, 0);
  P.g_slot0.assign(P.n_groups, 0);
  int64_t slot = 0;
  for (int64_t g = 0; g < P.n_groups; ++g) {
    int32_t w = 0;
    for (int lane = 0; lane < kTile; ++lane) {
      const int64_t q = g * kTile + lane;
      int32_t d = 0;
      if (q < N) each_coupling(cells[q], [&](int32_t, int64_t) { ++d; });
      w = std::max(w, d);
    }
    P.g_width[g] = w;
    P.g_slot0[g] = slot;
    slot += w;
  }
  P.n_slots = slot;
  P.e_pos.assign(P.n_slots * kTile, -1);
  P.e_row.assign(P.n_slots * kTile, -1);
  P.e_src.assign(P.n_slots * kTile, -1);
  P.e_rev.assign(P.n_slots * kTile, -1);
  std::vector<int32_t> packed_of(L.n_slots * kTile, -1);
  std::vector<std::pair<int32_t, int64_t>> list;
  for (int64_t g = 0; g < P.n_groups; ++g) {
    for (int lane = 0; lane < kTile; ++lane) {
      const int64_t q = g * kTile + lane;
      if (q >= N) continue;
      list.clear();
      each_coupling(cells[q], [&](int32_t v, int64_t fe) { list.emplace_back(pos_of[v], fe); });
      std::sort(list.begin(), list.end());
      for (size_t k = 0; k < list.size(); ++k) {
        const int64_t pe = (P.g_slot0[g] + (int64_t)k) * kTile + lane;
        P.e_pos[pe] = list[k].first;
        P.e_row[pe] = P.pos_row[list[k].first];
        P.e_src[pe] = (int32_t)list[k].second;
        packed_of[list[k].second] = (int32_t)pe;
      }
      P.n_coup += (int64_t)list.size();
    }
  }
  for (int64_t pe = 0; pe < P.n_slots * kTile; ++pe) {
    if (P.e_src[pe] < 0) continue;
    P.e_rev[pe] = packed_of[L.ent_rev[P.e_src[pe]]];
    if (P.e_rev[pe] < 0) {
      err = "partition-local ILU: coupling without its transpose";
      return FNLH_E_MESH;
    }
  }
  return FNLH_OK;
}

}  // namespace fnlh
