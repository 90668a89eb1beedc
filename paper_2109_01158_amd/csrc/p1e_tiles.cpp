// p1e_tiles.cpp -- host setup of the element tiles that the gradient kernels work on.
//
// The exact gradient at a free node is the sum of the element forces over its nodal patch
// (Section 4.2 patches, Section 6.2 forces), and the patch central differences sum
// per-element differences over the same patch (Section 6.1). Here a patch is split by
// element tiles: runs of consecutive internal elements (at most kTileElems elements touching
// at most kTileNodes distinct nodes). One workgroup evaluates a tile, keeps the tile's
// element results in LDS and sums, for every node of the tile, the entries of its patch
// that lie in the tile ("local patch row"). A node whose whole patch lies in one tile is
// complete there; the others write their tile's part to a halo slot (the slots of a node are
// consecutive, in ascending tile order), and a second pass sums the slots of each such node.
// Every sum has a fixed order.

#include <algorithm>
#include <numeric>
#include <vector>

#include "p1e_internal.h"

namespace p1e {

// conn: [k][ne] internal node of each element vertex (internal element order). Uses
// m->ninfo (internal nodes: first free DOF << 3 | free mask).
int build_tiles(p1e_mesh *m, const std::vector<int32_t> &conn) {
  const int k = m->k;
  const int64_t ne = m->ne, nn = m->nn;
  auto is_free = [&](int64_t v) { return (m->ninfo[v] & 7) != 0; };

  // ---- tiles: greedy runs of consecutive elements; ntile_of[v] = tiles that touch node v
  std::vector<int32_t> mark(nn, -1), ntile_of(nn, 0);
  std::vector<int32_t> tile_e(1, 0);
  for (int64_t e = 0; e < ne;) {
    const int32_t t = (int32_t)tile_e.size() - 1;
    const int64_t e0 = e;
    int nodes = 0;
    while (e < ne && e - e0 < kTileElems) {
      int add = 0;
      for (int l = 0; l < k; ++l) add += mark[conn[(size_t)l * ne + e]] != t;
      if (nodes + add > kTileNodes) break;
      for (int l = 0; l < k; ++l) {
        const int32_t v = conn[(size_t)l * ne + e];
        if (mark[v] != t) {
          mark[v] = t;
          ntile_of[v] += 1;
          ++nodes;
        }
      }
      ++e;
    }
    tile_e.push_back((int32_t)e);
  }
  const int64_t nt = (int64_t)tile_e.size() - 1;
  m->ntiles = nt;

  // ---- patch size of every node; patch incidences of free nodes (Section 4.2)
  std::vector<int32_t> deg(nn, 0);
  for (size_t i = 0; i < (size_t)k * ne; ++i) deg[conn[i]] += 1;
  int64_t nnz = 0;
  int maxv = 0;
  for (int64_t v = 0; v < nn; ++v)
    if (is_free(v)) {
      nnz += deg[v];
      maxv = std::max(maxv, deg[v]);
    }
  m->nnz = nnz;
  m->max_valence = maxv;

  // ---- halo rows: free nodes in several tiles or in none, in internal node order; their
  // slots are consecutive (one per tile, ascending tile)
  std::vector<int64_t> hstart(nn, -1);
  m->hrec.clear();
  int64_t nslots = 0;
  for (int64_t v = 0; v < nn; ++v)
    if (is_free(v) && ntile_of[v] != 1) {
      hstart[v] = nslots;
      m->hrec.insert(m->hrec.end(), {(int32_t)nslots, ntile_of[v], m->ninfo[v], 0});
      nslots += ntile_of[v];
    }
  m->nhalo = (int64_t)m->hrec.size() / 4;
  m->nslots = nslots;
  if (nslots >= (int64_t(1) << 29)) return fail(P1E_EINVAL, "mesh too large for halo slots");

  // ---- per tile: node records, local connectivity, local patch rows
  m->ttile.clear();
  m->trec.clear();
  m->tlent.clear();
  m->ttile.reserve(4 * (nt + 1));
  m->trec.reserve(4 * (size_t)std::accumulate(ntile_of.begin(), ntile_of.end(), int64_t(0)));
  m->tlent.reserve((size_t)k * ne + kEntAlign * nt);
  m->conn_loc.assign((size_t)k * ne, 0);
  std::vector<int32_t> loc(nn, -1), cnt, pos, fill, nodes, seen_tiles(nn, 0);
  nodes.reserve(kTileNodes);
  for (int64_t t = 0; t < nt; ++t) {
    const int64_t e0 = tile_e[t], e1 = tile_e[t + 1];
    nodes.clear();
    for (int64_t e = e0; e < e1; ++e)
      for (int l = 0; l < k; ++l) {
        const int32_t v = conn[(size_t)l * ne + e];
        if (loc[v] < 0) {
          loc[v] = 0;
          nodes.push_back(v);
        }
      }
    std::sort(nodes.begin(), nodes.end());
    const int nloc = (int)nodes.size();
    for (int a = 0; a < nloc; ++a) loc[nodes[a]] = a;
    cnt.assign(nloc, 0);
    for (int64_t e = e0; e < e1; ++e)
      for (int l = 0; l < k; ++l) {
        const int a = loc[conn[(size_t)l * ne + e]];
        m->conn_loc[(size_t)l * ne + e] = (uint16_t)a;
        cnt[a] += 1;
      }
    // local patch rows of the tile's free nodes, entries in ascending element
    const int64_t ent0 = (int64_t)m->tlent.size();
    m->ttile.insert(m->ttile.end(),
                    {(int32_t)e0, (int32_t)(m->trec.size() / 4), (int32_t)ent0, 0});
    pos.assign(nloc, 0);
    int run = 0;
    for (int a = 0; a < nloc; ++a) {
      pos[a] = run;
      if (is_free(nodes[a])) run += cnt[a];
    }
    m->tlent.resize(ent0 + (run + kEntAlign - 1) / kEntAlign * kEntAlign, 0);
    fill.assign(pos.begin(), pos.end());
    for (int64_t e = e0; e < e1; ++e)
      for (int l = 0; l < k; ++l) {
        const int a = loc[conn[(size_t)l * ne + e]];
        if (is_free(nodes[a]))  // LDS offset of the entry's result: (l kTileElems + e) d
          m->tlent[ent0 + fill[a]++] = (uint16_t)((l * kTileElems + (e - e0)) * m->d);
      }
    for (int a = 0; a < nloc; ++a) {
      const int32_t v = nodes[a];
      const bool fr = is_free(v);
      int32_t z = 0;
      if (fr) {
        const int rank = seen_tiles[v];
        const int complete = ntile_of[v] == 1;
        const int64_t slot = complete ? 0 : hstart[v] + rank;
        z = (int32_t)((slot << 2) | ((rank == 0) << 1) | complete);
      }
      const int32_t w = fr ? (pos[a] | (cnt[a] << 16)) : 0;
      m->trec.insert(m->trec.end(), {v, m->ninfo[v], z, w});
      seen_tiles[v] += 1;
      loc[v] = -1;
    }
  }
  m->ttile.insert(m->ttile.end(),
                  {(int32_t)ne, (int32_t)(m->trec.size() / 4), (int32_t)m->tlent.size(), 0});
  m->ntnodes = (int64_t)m->trec.size() / 4;
  if (m->tlent.size() >= (size_t(1) << 31)) return fail(P1E_EINVAL, "mesh too large for tiles");
  return P1E_OK;
}

}  // namespace p1e
