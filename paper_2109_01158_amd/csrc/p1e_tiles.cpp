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

// LDS slots for a tile's nodal values (a permutation of 0 .. nloc-1). The element pass reads
// the values of each element's vertices, one element per lane; the reads of R neighbouring
// lanes are served together, and two different nodes whose slots agree modulo R fall in the
// same LDS banks and are served one after the other. Greedy colouring into the R residues:
// the nodes at one vertex position in one group of R lanes (a "set") want different
// residues; the nodes with the most partners choose first, each taking the residue (with
// room left) that the fewest already placed members of its sets use. lv: [net][k] local
// vertex indices in lane order.
struct SlotScratch {
  std::vector<int32_t> deg, mstart, mem, order, color, cap, next, setn, setcnt;
};

static void assign_slots(int nloc, int net, int k, int R, const std::vector<int32_t> &lv,
                         std::vector<int32_t> &slot, SlotScratch &w) {
  const int nsets = (net + R - 1) / R * k;
  // the sets: for each group of R lanes and vertex position, its distinct nodes
  w.setn.assign((size_t)nsets * R, 0);  // members of set s at [s R, s R + size)
  std::vector<int32_t> &size = w.deg;   // reused below as the degree
  size.assign(nsets, 0);
  for (int g0 = 0, s0 = 0; g0 < net; g0 += R, s0 += k) {
    const int g1 = std::min(net, g0 + R);
    for (int l = 0; l < k; ++l) {
      int32_t *m = &w.setn[(size_t)(s0 + l) * R];
      int n = 0;
      for (int le = g0; le < g1; ++le) {
        const int a = lv[(size_t)le * k + l];
        bool seen = false;
        for (int q = 0; q < n; ++q) seen = seen || m[q] == a;
        if (!seen) m[n++] = a;
      }
      size[s0 + l] = n;
    }
  }
  // memberships of each node (node -> sets), and its number of partners
  w.mstart.assign(nloc + 1, 0);
  for (int s = 0; s < nsets; ++s)
    for (int q = 0; q < size[s]; ++q) w.mstart[w.setn[(size_t)s * R + q] + 1] += 1;
  for (int a = 0; a < nloc; ++a) w.mstart[a + 1] += w.mstart[a];
  w.mem.resize(w.mstart[nloc]);
  w.order.assign(nloc, 0);  // fill cursor for now
  std::vector<int32_t> part(nloc, 0);
  for (int s = 0; s < nsets; ++s)
    for (int q = 0; q < size[s]; ++q) {
      const int a = w.setn[(size_t)s * R + q];
      w.mem[w.mstart[a] + w.order[a]++] = s;
      part[a] += size[s] - 1;
    }
  // greedy colouring, most partners first
  std::iota(w.order.begin(), w.order.end(), 0);
  std::stable_sort(w.order.begin(), w.order.end(),
                   [&](int x, int y) { return part[x] > part[y]; });
  w.setcnt.assign((size_t)nsets * R, 0);  // placed members of set s with residue r
  w.cap.assign(R, 0);
  w.next.resize(R);
  for (int s = 0; s < nloc; ++s) w.cap[s % R] += 1;
  for (int r = 0; r < R; ++r) w.next[r] = r;
  slot.assign(nloc, 0);
  int cost[64];
  for (int a : w.order) {
    for (int r = 0; r < R; ++r) cost[r] = 0;
    for (int i = w.mstart[a]; i < w.mstart[a + 1]; ++i) {
      const int32_t *c = &w.setcnt[(size_t)w.mem[i] * R];
      for (int r = 0; r < R; ++r) cost[r] += c[r];
    }
    int best = -1;
    for (int r = 0; r < R; ++r)
      if (w.cap[r] > 0 && (best < 0 || cost[r] < cost[best] ||
                           (cost[r] == cost[best] && w.cap[r] > w.cap[best])))
        best = r;
    for (int i = w.mstart[a]; i < w.mstart[a + 1]; ++i) w.setcnt[(size_t)w.mem[i] * R + best] += 1;
    w.cap[best] -= 1;
    slot[a] = w.next[best];
    w.next[best] += R;
  }
}

// conn: [k][ne] internal node of each element vertex (internal element order). Uses
// m->ninfo (internal nodes: first free DOF << 3 | free mask). A tile touches at most
// node_cap (<= kTileNodes) nodes.
int build_tiles(p1e_mesh *m, const std::vector<int32_t> &conn, int node_cap) {
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
      if (nodes + add > node_cap) break;
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
  m->tslot.clear();
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
    // Record order: free nodes by descending number of patch-sum rounds (rounds of 8 entries,
    // two lanes per node), then the nodes without a free DOF; ascending node within each
    // group. A wavefront's patch sums take as many rounds as its longest row, so grouping
    // rows of equal length saves rounds, and the ascending runs keep the nodal loads and the
    // gradient stores contiguous.
    for (int a = 0; a < nloc; ++a) loc[nodes[a]] = a;
    cnt.assign(nloc, 0);
    for (int64_t e = e0; e < e1; ++e)
      for (int l = 0; l < k; ++l) cnt[loc[conn[(size_t)l * ne + e]]] += 1;
    {
      auto key = [&](int32_t v) { return is_free(v) ? -((cnt[loc[v]] + 7) / 8) : 1; };
      std::stable_sort(nodes.begin(), nodes.end(),
                       [&](int32_t x, int32_t y) { return key(x) < key(y); });
      std::vector<int32_t> c2(nloc);
      for (int a = 0; a < nloc; ++a) c2[a] = cnt[loc[nodes[a]]];
      cnt.swap(c2);
    }
    for (int a = 0; a < nloc; ++a) loc[nodes[a]] = a;
    for (int64_t e = e0; e < e1; ++e)
      for (int l = 0; l < k; ++l)  // slot = local index until coloured
        m->conn_loc[(size_t)l * ne + e] = (uint16_t)loc[conn[(size_t)l * ne + e]];
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
        if (is_free(nodes[a]))  // byte offset of the entry's FP32 result, (l kTileElems + e) d 4
          m->tlent[ent0 + fill[a]++] = (uint16_t)((l * kTileElems + (e - e0)) * m->d * 4);
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
      m->tslot.push_back((uint16_t)a);
      seen_tiles[v] += 1;
      loc[v] = -1;
    }
  }
  m->ttile.insert(m->ttile.end(),
                  {(int32_t)ne, (int32_t)(m->trec.size() / 4), (int32_t)m->tlent.size(), 0});
  m->ntnodes = (int64_t)m->trec.size() / 4;
  m->slots_coloured = false;
  if (m->tlent.size() >= (size_t(1) << 31)) return fail(P1E_EINVAL, "mesh too large for tiles");
  return P1E_OK;
}

// GEO_OTF: per tile node (record order) its coordinates minus the centroid of the tile's
// nodes, FP64 [sum nloc][dim]. Near the centroid the offsets are of the tile's size, so the
// edge vectors the element pass forms from them lose little even in FP32.
void tile_offsets(p1e_mesh *m, const double *coords) {
  const int dim = m->dim;
  m->txo.assign((size_t)m->ntnodes * dim, 0.0);
  for (int64_t t = 0; t < m->ntiles; ++t) {
    const int64_t r0 = m->ttile[4 * t + 1], r1 = m->ttile[4 * (t + 1) + 1];
    double c[3] = {0.0, 0.0, 0.0};
    for (int64_t r = r0; r < r1; ++r)
      for (int j = 0; j < dim; ++j) c[j] += coords[(int64_t)m->trec[4 * r] * dim + j];
    for (int j = 0; j < dim; ++j) c[j] /= (double)std::max<int64_t>(r1 - r0, 1);
    for (int64_t r = r0; r < r1; ++r)
      for (int j = 0; j < dim; ++j)
        m->txo[(size_t)r * dim + j] = coords[(int64_t)m->trec[4 * r] * dim + j] - c[j];
  }
}

// Replace the identity slots of build_tiles by coloured ones (assign_slots) in every tile:
// conn_loc and tslot are rewritten together; results do not change (only where the nodal
// values sit in LDS). Done once, when a mesh is first bound for mixed precision, whose
// 16-byte float nodal values it is tuned for.
void colour_slots(p1e_mesh *m) {
  if (m->slots_coloured) return;
  const int k = m->k;
  const int64_t ne = m->ne;
  // lanes whose vertex reads are served together: 128 bytes of nodal values (float x 4 per
  // node for d = 3, x 2 for d = 2, x 1 for d = 1)
  const int R = m->d == 3 ? 8 : m->d == 2 ? 16 : 32;
  std::vector<int32_t> lv, slot;
  SlotScratch sw;
  for (int64_t t = 0; t < m->ntiles; ++t) {
    const int64_t e0 = m->ttile[4 * t], e1 = m->ttile[4 * (t + 1)];
    const int64_t r0 = m->ttile[4 * t + 1], nloc = m->ttile[4 * (t + 1) + 1] - r0;
    lv.resize((size_t)(e1 - e0) * k);
    for (int64_t e = e0; e < e1; ++e)
      for (int l = 0; l < k; ++l)
        lv[(size_t)(e - e0) * k + l] = m->conn_loc[(size_t)l * ne + e];
    assign_slots((int)nloc, (int)(e1 - e0), k, R, lv, slot, sw);
    for (int64_t e = e0; e < e1; ++e)
      for (int l = 0; l < k; ++l)
        m->conn_loc[(size_t)l * ne + e] = (uint16_t)slot[lv[(size_t)(e - e0) * k + l]];
    for (int64_t a = 0; a < nloc; ++a) m->tslot[r0 + a] = (uint16_t)slot[a];
  }
  m->slots_coloured = true;
}

}  // namespace p1e
