// Host-side fuzz of the library's mesh setup (p1e_mesh_create, p1e_mesh_get_info,
// p1e_workspace_bytes, p1e_material_constants), built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the CPU (no GPU: the kernel launchers are stubs). Random
// structured triangle and tetrahedron meshes, jittered and permuted, of every energy kind,
// with random Dirichlet masks, values and loads, flags and geometry modes; a share of them is
// corrupted (index out of range, repeated vertex, coincident vertices, non-finite coordinate,
// bad sizes, kinds, exponents or pointers) and must be refused with the documented status.
// For the valid ones the reported counts are checked against counts made here, and the element
// tiles against their definition (white box: the library's host structures).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <numeric>
#include <random>
#include <vector>

#include "p1e.h"
#include "p1e_internal.h"

static int g_fail = 0;
#define CHECK(c, ...)                                              \
  do {                                                             \
    if (!(c)) {                                                    \
      std::fprintf(stderr, "check failed (%s:%d): %s: ", __FILE__, \
                   __LINE__, #c);                                  \
      std::fprintf(stderr, __VA_ARGS__);                           \
      std::fprintf(stderr, "\n");                                  \
      ++g_fail;                                                    \
    }                                                              \
  } while (0)

// The tiles of a built mesh against their definition: per tile at most kTileElems elements and
// the node cap, each node once; identity LDS slots before colouring; every local patch entry
// is the byte offset (l kTileElems + e) d 4 of an element result whose vertex l is the row's
// node, in ascending element, one per incidence; free nodes' records first, by descending
// number of patch-sum rounds of 8 entries, then the nodes without a free DOF, ascending node
// within each group.
static void check_tiles(const p1e_mesh *m, int cap, int it) {
  const int k = m->k, d = m->d;
  const int64_t ne = m->ne;
  std::vector<int> cnt, seen(m->nn, -1);
  for (int64_t t = 0; t < m->ntiles; ++t) {
    const int64_t e0 = m->ttile[4 * t], e1 = m->ttile[4 * t + 4];
    const int64_t r0 = m->ttile[4 * t + 1], r1 = m->ttile[4 * t + 5];
    const int64_t ent0 = m->ttile[4 * t + 2];
    const int nloc = (int)(r1 - r0);
    CHECK(e1 > e0 && e1 - e0 <= p1e::kTileElems && nloc <= cap, "iter %d tile %lld size", it,
          (long long)t);
    cnt.assign(nloc, 0);
    for (int a = 0; a < nloc; ++a) {
      const int32_t v = m->trec[4 * (r0 + a)];
      CHECK(seen[v] != (int)t, "iter %d tile %lld: node %d twice", it, (long long)t, v);
      seen[v] = (int)t;
      CHECK(m->slots_coloured || m->tslot[r0 + a] == a, "iter %d: slot", it);
    }
    auto node_at = [&](int l, int64_t e) { return m->trec[4 * (r0 + m->conn_loc[l * ne + e])]; };
    for (int64_t e = e0; e < e1; ++e)
      for (int l = 0; l < k; ++l) {
        const int a = m->conn_loc[l * ne + e];
        CHECK(a < nloc, "iter %d: local index", it);
        if (a < nloc) cnt[a] += 1;
      }
    int prev_key = 1 << 30, prev_v = -1;
    for (int a = 0; a < nloc; ++a) {
      const int32_t *rec = &m->trec[4 * (r0 + a)];
      const int32_t v = rec[0];
      const bool fr = (m->ninfo[v] & 7) != 0;
      const int key = fr ? (cnt[a] + 7) / 8 : -1;
      CHECK(key < prev_key || (key == prev_key && v > prev_v), "iter %d tile %lld: record order",
            it, (long long)t);
      prev_key = key;
      prev_v = v;
      if (!fr) {
        CHECK(rec[3] == 0, "iter %d: row of a prescribed node", it);
        continue;
      }
      const int p0 = rec[3] & 0xffff, n = rec[3] >> 16;
      CHECK(n == cnt[a], "iter %d: row length %d vs %d", it, n, cnt[a]);
      int prev_le = -1;
      for (int q = 0; q < n; ++q) {
        const int off = m->tlent[ent0 + p0 + q];
        const int idx = off / (4 * d), l = idx / p1e::kTileElems, le = idx % p1e::kTileElems;
        const bool ok = off % (4 * d) == 0 && l < k && le < e1 - e0 && le > prev_le &&
                        node_at(l, e0 + le) == v;
        CHECK(ok, "iter %d tile %lld node %d: entry %d", it, (long long)t, v, off);
        prev_le = le;
      }
    }
  }
  // halo rows: the free nodes in several tiles (or none), ascending node, each with one slot
  // per tile in ascending tile order; a record's flags say complete (one tile) and owner
  // (the first tile)
  std::vector<int> ntile(m->nn, 0), rank_in(m->nn, 0);
  for (int64_t r = 0; r < m->ntnodes; ++r) ntile[m->trec[4 * r]] += 1;
  std::vector<int64_t> first_slot(m->nn, -1);
  int64_t h = 0, slots = 0;
  for (int64_t v = 0; v < m->nn; ++v)
    if ((m->ninfo[v] & 7) && ntile[v] != 1) {
      CHECK(h < m->nhalo && m->hrec[4 * h] == slots && m->hrec[4 * h + 1] == ntile[v] &&
                m->hrec[4 * h + 2] == m->ninfo[v],
            "iter %d: halo row %lld", it, (long long)h);
      first_slot[v] = slots;
      slots += ntile[v];
      ++h;
    }
  CHECK(h == m->nhalo && slots == m->nslots, "iter %d: halo rows %lld slots %lld", it,
        (long long)h, (long long)slots);
  for (int64_t r = 0; r < m->ntnodes; ++r) {  // records in tile order
    const int32_t v = m->trec[4 * r], z = m->trec[4 * r + 2];
    const int rank = rank_in[v]++;
    if (!(m->ninfo[v] & 7)) continue;
    const bool complete = ntile[v] == 1;
    CHECK((z & 1) == (int)complete && ((z >> 1) & 1) == (int)(rank == 0) &&
              (complete || (z >> 2) == first_slot[v] + rank),
          "iter %d: record flags of node %d", it, v);
  }
}

struct Mesh {
  int dim = 2;
  std::vector<double> x;   // [nn][dim]
  std::vector<int32_t> t;  // [ne][dim+1]
  int64_t nn() const { return (int64_t)x.size() / dim; }
  int64_t ne() const { return (int64_t)t.size() / (dim + 1); }
};

// right triangles (2D) or Kuhn tetrahedra (3D) on a grid of n[0] x n[1] (x n[2]) cells
static Mesh grid(int dim, const int n[3], double h, double jitter, std::mt19937_64 &rng) {
  Mesh m;
  m.dim = dim;
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  const int nx = n[0] + 1, ny = n[1] + 1, nz = dim == 3 ? n[2] + 1 : 1;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const bool inner = i > 0 && i < nx - 1 && j > 0 && j < ny - 1 &&
                           (dim == 2 || (k > 0 && k < nz - 1));
        const double c[3] = {i * h, j * h, k * h};
        for (int a = 0; a < dim; ++a) m.x.push_back(c[a] + (inner ? jitter * h * U(rng) : 0.0));
      }
  auto id = [&](int i, int j, int k) { return (int32_t)(i + nx * (j + ny * k)); };
  if (dim == 2) {
    for (int j = 0; j < n[1]; ++j)
      for (int i = 0; i < n[0]; ++i) {
        m.t.insert(m.t.end(), {id(i, j, 0), id(i + 1, j, 0), id(i + 1, j + 1, 0)});
        m.t.insert(m.t.end(), {id(i, j, 0), id(i + 1, j + 1, 0), id(i, j + 1, 0)});
      }
  } else {
    const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    for (int k = 0; k < n[2]; ++k)
      for (int j = 0; j < n[1]; ++j)
        for (int i = 0; i < n[0]; ++i)
          for (auto &p : perm) {
            int c[3] = {i, j, k};
            const int32_t v0 = id(c[0], c[1], c[2]);
            c[p[0]] += 1;
            const int32_t v1 = id(c[0], c[1], c[2]);
            c[p[1]] += 1;
            const int32_t v2 = id(c[0], c[1], c[2]);
            m.t.insert(m.t.end(), {v0, v1, v2, id(i + 1, j + 1, k + 1)});
          }
  }
  return m;
}

static double volume(const Mesh &m, int64_t e) {
  const int d = m.dim;
  const int32_t *T = &m.t[(size_t)e * (d + 1)];
  double B[3][3] = {{0}};
  for (int l = 1; l <= d; ++l)
    for (int a = 0; a < d; ++a) B[a][l - 1] = m.x[(size_t)T[l] * d + a] - m.x[(size_t)T[0] * d + a];
  const double det = d == 2 ? B[0][0] * B[1][1] - B[0][1] * B[1][0]
                            : B[0][0] * (B[1][1] * B[2][2] - B[1][2] * B[2][1]) -
                                  B[0][1] * (B[1][0] * B[2][2] - B[1][2] * B[2][0]) +
                                  B[0][2] * (B[1][0] * B[2][1] - B[1][1] * B[2][0]);
  return std::fabs(det) / (d == 2 ? 2.0 : 6.0);
}

int main(int argc, char **argv) {
  const int iters = argc > 1 ? std::atoi(argv[1]) : 300;
  std::mt19937_64 rng(20261203);
  std::uniform_real_distribution<double> U01(0.0, 1.0);
  const int kinds[5] = {P1E_PLAPLACE, P1E_PLAPLACE_ORTHO, P1E_NEOHOOKE, P1E_SVK,
                        P1E_GINZBURG_LANDAU};
  int n_ok = 0, n_refused = 0;
  for (int it = 0; it < iters; ++it) {
    const int dim = 2 + (int)(rng() % 2);
    const int n[3] = {1 + (int)(rng() % 9), 1 + (int)(rng() % 6), 1 + (int)(rng() % 5)};
    Mesh m = grid(dim, n, 0.1 + U01(rng), (rng() % 2) ? 0.25 : 0.0, rng);
    // permute nodes and elements
    std::vector<int32_t> np(m.nn());
    std::iota(np.begin(), np.end(), 0);
    std::shuffle(np.begin(), np.end(), rng);
    std::vector<double> x2(m.x.size());
    for (int64_t i = 0; i < m.nn(); ++i)
      for (int a = 0; a < dim; ++a) x2[(size_t)np[i] * dim + a] = m.x[(size_t)i * dim + a];
    m.x.swap(x2);
    for (auto &v : m.t) v = np[v];
    const int kind = kinds[rng() % 5];
    const bool vec = kind == P1E_NEOHOOKE || kind == P1E_SVK;
    const int nc = vec ? dim : 1;
    const int64_t nn = m.nn(), ne = m.ne();
    std::vector<uint8_t> dmask((size_t)nn * nc);
    std::vector<double> dval((size_t)nn * nc), load((size_t)nn * nc);
    for (auto &b : dmask) b = U01(rng) < 0.3;
    for (auto &v : dval) v = U01(rng) - 0.5;
    for (auto &v : load) v = 10.0 * (U01(rng) - 0.5);
    p1e_mesh_desc d{};
    d.dim = dim;
    d.ncomp = nc;
    d.kind = kind;
    d.flags = (int)(rng() % 8) & (P1E_INPUT_ORDER | P1E_FULL_GEOMETRY);
    d.nn = nn;
    d.ne = ne;
    d.conn = m.t.data();
    d.coords = m.x.data();
    d.dirichlet = (rng() % 4) ? dmask.data() : nullptr;
    d.dirichlet_values = (rng() % 3) ? dval.data() : nullptr;
    d.load = (rng() % 3) ? load.data() : nullptr;
    d.p = 1.2 + 4.0 * U01(rng);
    d.C1 = 1.0 + U01(rng);
    d.D1 = 1.0 + U01(rng);
    // corruption
    int expect = P1E_OK;
    const int c = (U01(rng) < 0.4) ? 1 + (int)(rng() % 10) : 0;
    const int k = dim + 1;
    const int64_t e = (int64_t)(rng() % ne);
    switch (c) {
      case 1: m.t[(size_t)e * k + rng() % k] = (rng() % 2) ? -1 : (int32_t)nn; expect = P1E_EINVAL; break;
      case 2: m.t[(size_t)e * k + 1] = m.t[(size_t)e * k]; expect = P1E_EINVAL; break;
      case 3: {  // two vertices of element e at one position: e is degenerate
        const int32_t a = m.t[(size_t)e * k], b = m.t[(size_t)e * k + 1];
        for (int q = 0; q < dim; ++q) m.x[(size_t)b * dim + q] = m.x[(size_t)a * dim + q];
        expect = P1E_EDEGEN;
        break;
      }
      case 4: m.x[(size_t)m.t[(size_t)e * k] * dim] = NAN; expect = P1E_EDEGEN; break;
      case 5: d.ncomp = vec ? 1 : 2; expect = P1E_EINVAL; break;
      case 6: if (kind == P1E_PLAPLACE || kind == P1E_PLAPLACE_ORTHO) { d.p = 1.0; expect = P1E_EINVAL; } break;
      case 7: d.kind = 9; expect = P1E_EINVAL; break;
      case 8: d.dim = 4; expect = P1E_EINVAL; break;
      case 9: d.conn = nullptr; expect = P1E_EINVAL; break;
      case 10: d.nn = 0; expect = P1E_EINVAL; break;
    }
    p1e_mesh *h = nullptr;
    const int rc = p1e_mesh_create(&d, &h);
    if (expect != P1E_OK) {
      CHECK(rc == expect && h == nullptr, "iter %d corruption %d: rc %d, expected %d (%s)", it, c, rc,
            expect, p1e_last_error());
      ++n_refused;
      continue;
    }
    CHECK(rc == P1E_OK && h != nullptr, "iter %d: rc %d (%s)", it, rc, p1e_last_error());
    if (rc != P1E_OK) continue;
    ++n_ok;
    p1e_mesh_info info{};
    CHECK(p1e_mesh_get_info(h, &info) == P1E_OK, "info");
    // counts made here
    int64_t nfd = 0, nfree = 0, nnz = 0;
    std::vector<int32_t> deg(nn, 0);
    for (auto v : m.t) deg[v] += 1;
    double vol = 0.0;
    for (int64_t q = 0; q < ne; ++q) vol += volume(m, q);
    for (int64_t i = 0; i < nn; ++i) {
      int f = 0;
      for (int j = 0; j < nc; ++j) f += !(d.dirichlet && d.dirichlet[i * nc + j]);
      nfd += f;
      if (f) {
        ++nfree;
        nnz += deg[i];
      }
    }
    CHECK(info.nn == nn && info.ne == ne, "sizes");
    CHECK(info.n_free_dofs == nfd && info.n_free_nodes == nfree, "free %lld/%lld vs %lld/%lld",
          (long long)info.n_free_dofs, (long long)info.n_free_nodes, (long long)nfd, (long long)nfree);
    CHECK(info.nnz == nnz, "nnz %lld vs %lld", (long long)info.nnz, (long long)nnz);
    CHECK(std::fabs(info.total_volume - vol) <= 1e-12 * vol, "volume %.17g vs %.17g", info.total_volume, vol);
    CHECK(info.kind == kind && info.ncomp == nc && info.dim == dim, "kind");
    if (d.flags & P1E_FULL_GEOMETRY) CHECK(info.geometry_mode == 0, "stored geometry");
    else CHECK(info.geometry_mode == (info.geometry_classes > 0 ? 1 : 2), "geometry mode");
    const int cap = info.geometry_mode == 2 ? 512 : 1024;
    CHECK(info.n_tile_nodes <= (int64_t)cap * info.n_tiles, "tile nodes");
    CHECK(info.n_halo_slots >= 2 * info.n_halo_rows, "halo slots");  // every node is in an element
    for (int mask = 0; mask < 9; ++mask) {
      const uint64_t b = p1e_workspace_bytes(h, mask);
      const bool valid = mask >= 1 && mask <= 7;
      CHECK(valid ? b > 0 && b % info.alignment == 0 : b == 0, "workspace mask %d: %llu", mask,
            (unsigned long long)b);
    }
    check_tiles(h, cap, it);
    p1e_mesh_destroy(h);
  }
  // material constants: valid and invalid arguments
  double C1 = 0.0, D1 = 0.0;
  CHECK(p1e_material_constants(P1E_NEOHOOKE, 2e8, 0.3, &C1, &D1) == P1E_OK, "nh constants");
  CHECK(std::fabs(C1 - 2e8 / 2.6 / 2.0) <= 1e-6 * C1, "C1");
  CHECK(p1e_material_constants(P1E_SVK, 2e8, 0.5, &C1, &D1) == P1E_EINVAL, "nu = 1/2");
  CHECK(p1e_material_constants(P1E_PLAPLACE, 2e8, 0.3, &C1, &D1) == P1E_EINVAL, "kind");
  CHECK(p1e_material_constants(P1E_NEOHOOKE, -1.0, 0.3, &C1, &D1) == P1E_EINVAL, "E < 0");
  CHECK(p1e_material_constants(P1E_NEOHOOKE, 1.0, 0.3, nullptr, &D1) == P1E_EINVAL, "null");
  CHECK(p1e_mesh_create(nullptr, nullptr) == P1E_EINVAL, "null desc");
  std::printf("fuzz: %d meshes built, %d refused, %d failed checks\n", n_ok, n_refused, g_fail);
  return g_fail ? 1 : 0;
}
