// p1e_internal.h -- mesh handle layout and kernel launchers shared by the host setup
// (p1e_api.cpp, p1e_tiles.cpp), the single-mesh kernels (p1e_kernels.hip) and the batched
// engine (p1e_batch.hip, p1e_serve.cpp). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/p1e.h"

namespace p1e {

// Element tiles: one workgroup evaluates one tile of consecutive (internal) elements. The
// tile's nodal values and patch entries are staged in LDS, its element forces are written
// to LDS, and each of its nodes sums its share of the patch from LDS (Section 4.2 patches
// split by tile).
#ifndef P1E_TILE_ELEMS
#define P1E_TILE_ELEMS 1024
#endif
// XCDs of the device: each has its own L2, and the dispatcher hands consecutive workgroups
// to them in turn
#ifndef P1E_XCD_COUNT
#define P1E_XCD_COUNT 8
#endif
constexpr int kTileElems = P1E_TILE_ELEMS;  // elements per tile (at most)
constexpr int kTileNodes = P1E_TILE_ELEMS;  // distinct nodes per tile (at most)
constexpr int kEntAlign = 8;       // each tile's patch entries start on a 16-byte boundary
static_assert((4 * kTileElems) * 3 * 4 <= 65536, "patch entry byte offsets fit 16 bits");
constexpr int kBlock = 256;        // threads per block of the halo-row and vector kernels
constexpr uint64_t kAlign = 256;   // alignment of every sub-array in the bound buffer
constexpr int kMaxGeoClasses = 64; // geometry classes kept as one-byte indices
constexpr double kClassDeviation = 0x1p-42;  // largest relative record change of a class

// How the element pass gets B^-1 and |T| (Section 4.1):
//   GEO_STORED  per-element records [dim*dim+1][ne] (P1E_FULL_GEOMETRY);
//   GEO_CLASS   a table of at most kMaxGeoClasses records and a one-byte class per element;
//   GEO_OTF     formed in the tile from its nodes' coordinates, staged in LDS as offsets from
//               the tile's centroid (meshes without few enough classes); such tiles touch at
//               most kTileNodes / 2 nodes, and the offsets take the other half of the nodal
//               value slots.
enum GeoMode { GEO_STORED = 0, GEO_CLASS = 1, GEO_OTF = 2 };

// Device view of a bound mesh (all arrays in the caller's buffer). Internal numbering: the
// elements in tile order, the nodes in order of first use by the elements.
//
// Tile node record (int4), one per node of a tile, in ascending internal node:
//   x = internal node, y = (first free DOF << 3) | free-component mask,
//   z = (halo slot << 2) | owner << 1 | complete   (complete: the node's whole patch lies in
//       the tile; owner: this is the first tile of the node, which adds its b.v),
//   w = first local patch entry | entry count << 16.
// Halo row record (int4), one per free node whose patch spans several tiles (or no
// element): x = first slot, y = slot count, z = (first free DOF << 3) | mask.
struct TileMesh {
  int32_t nn = 0, ne = 0, nfd = 0;
  int32_t ntiles = 0, nhalo = 0;
  const double *wref = nullptr;  // [nn][d] per component: free -> subtrahend (x for
                                 // Neo-Hookean, 0 for the p-Laplacian), prescribed -> u
  const double *bhat = nullptr;  // [nfd] b = M f on the free DOFs
  // elements (internal order)
  const uint16_t *conn_loc = nullptr;  // [dim+1][ne] vertex -> LDS slot of its nodal value
                                       // within the tile (tslot of the node)
  // element geometry: B^-1 entries (row l-1 = grad phi_l) and |T|, either per element as
  // [dim*dim+1][ne], or (geometry classes) as a table [nclass][dim*dim+1] indexed by geo_cls
  const double *geo64 = nullptr;    // FP64
  const float *geo32 = nullptr;     // FP32 (mixed mode)
  const uint8_t *geo_cls = nullptr; // [ne] class of each element, or nullptr
  int32_t nclass = 0;
  int32_t geo_mode = GEO_STORED;
  // GEO_OTF: per tile node (record order) its coordinates minus the tile's centroid, [dim]
  const double *txo64 = nullptr;    // FP64
  const float *txo32 = nullptr;     // FP32 (mixed mode)
  // tiles
  const int4 *ttile = nullptr;  // [ntiles+1] {first element, first node record, first patch
                                //  entry, 0}; the last one closes the ranges
  const int4 *trec = nullptr;   // [sum nloc] tile node records
  const uint16_t *tslot = nullptr;  // [sum nloc] LDS slot of each tile node's nodal value
  const uint16_t *tlent = nullptr;  // local patch entries: byte offset (l kTileElems + e) d 4
                                    // of the element's FP32 result in the tile's LDS (twice
                                    // that for FP64 results), per node ascending e
  const int4 *hrec = nullptr;   // [nhalo] halo row records
  // scratch
  double *hpart = nullptr;   // [slots][d] partial patch sums of halo rows, by row, in the
                             // tiles' element type (float in mixed precision; sized for double)
  double *gw = nullptr;      // [nfd] gradient kept by p1e_energy_forces
  double2 *part = nullptr;   // [2][max(ntiles,1)] compensated partials: energy, then b.v
  int32_t *badp = nullptr;   // [max(ntiles,1)] bad-element counts
};

}  // namespace p1e

struct p1e_mesh {
  int dim = 0, d = 0, kind = 0, k = 0;
  int ortho = 0;  // P1E_PLAPLACE_ORTHO: kind P1E_PLAPLACE with the component-wise norm
  int64_t nn = 0, ne = 0, nf = 0, nfd = 0, nnz = 0;
  double p = 2.0, C1 = 0.0, D1 = 0.0;
  int max_valence = 0;
  double total_vol = 0.0, min_vol = 0.0, max_vol = 0.0, dirichlet_bv = 0.0;

  // host copies (kept so the mesh can be bound again)
  std::vector<double> geo64;       // [dim*dim+1][ne] (empty when classed)
  int nclass = 0;                  // distinct element geometries when <= kMaxGeoClasses, else 0
  double class_dev = 0.0;          // largest relative change of a record by its class
  std::vector<uint8_t> geo_cls;    // [ne] class of each element
  std::vector<double> geo_tab;     // [nclass][dim*dim+1]
  int geo_mode = p1e::GEO_STORED;  // GeoMode
  std::vector<double> txo;         // GEO_OTF: [sum nloc][dim] node offsets from tile centroids
  std::vector<int32_t> ninfo;      // [nn] internal order
  std::vector<double> wref;        // [nn][d] internal order
  std::vector<double> bhat;        // [nfd]
  std::vector<uint16_t> conn_loc;  // [k][ne]
  std::vector<int32_t> ttile;      // [ntiles+1][4]
  std::vector<int32_t> trec;       // [sum nloc][4]
  std::vector<uint16_t> tslot;     // [sum nloc]
  bool slots_coloured = false;     // tslot / conn_loc hold coloured LDS slots (colour_slots)
  std::vector<uint16_t> tlent;
  std::vector<int32_t> hrec;       // [nhalo][4]
  int64_t ntiles = 0, nhalo = 0, nslots = 0, ntnodes = 0;

  // binding
  int bound_modes = 0;
  int device = -1;
  p1e::TileMesh dev;
  int forces_prec = 0;   // precision of the gradient held in dev.gw (0 = none)
};

namespace p1e {

// thread-local error reporting (p1e_api.cpp)
int fail(int code, const std::string &msg);

// kernel timing hooks (p1e_api.cpp); no-ops unless enabled
void prof_begin(const char *name, hipStream_t s);
void prof_end(hipStream_t s);

inline int64_t nblocks(int64_t n, int per = kBlock) { return (n + per - 1) / per; }

// host setup of the element tiles, node order and halo rows (p1e_tiles.cpp)
int build_tiles(p1e_mesh *m, const std::vector<int32_t> &conn, int node_cap);
void tile_offsets(p1e_mesh *m, const double *coords);
void colour_slots(p1e_mesh *m);

// launchers (p1e_kernels.hip). All enqueue on stream and return P1E_OK or a status.
int run_energy(p1e_mesh *m, const double *vhat, int prec, double *out3, int32_t *flag,
               hipStream_t s);
int run_grad_exact(p1e_mesh *m, const double *vhat, int prec, double *g, double *out3,
                   int32_t *flag, hipStream_t s);
int run_grad_fd(p1e_mesh *m, const double *vhat, double eps, int order, double *g,
                int32_t *flag, hipStream_t s);
int run_energy_forces(p1e_mesh *m, const double *vhat, int prec, double *out3, int32_t *flag,
                      hipStream_t s);
int run_scale(p1e_mesh *m, const double *scale, double *g, hipStream_t s);
int run_scale_inplace(p1e_mesh *m, const double *scale, double *g, hipStream_t s);
// p1e_grad_exact with its scratch in the library's static per-device array
int run_grad_exact_static(p1e_mesh *m, const double *vhat, int prec, double *g, double *out3,
                          int32_t *flag, hipStream_t s);
uint64_t static_scratch_need(const p1e_mesh *m);

}  // namespace p1e

// ============================================================================ batched engine
// Many minimizations (requests) share the device: each occupies a slot whose mesh and
// L-BFGS state live in one sub-allocation of a pool. One engine step advances every active
// slot by one line-search trial with a fixed sequence of launches that read the set of
// active slots from device tables, so the sequence can be captured once in a hipGraph.
namespace p1e {

constexpr int kMaxHistory = 8;     // L-BFGS memory m <= kMaxHistory
constexpr int kVecTile = 1024;     // DOFs per tile of the vector kernels
constexpr int kMaxLineTrials = 40; // backtracking halvings per iteration
constexpr int kNPart = 4 * kMaxHistory;  // vector-reduction partials per vector tile
// per-slot L-BFGS matrices and coefficients (doubles, storage order of the history):
// s_a.y_b, y_a.y_b, then the direction's coefficients of g, of S_h and of Y_h
constexpr int kSY = 0, kYY = kMaxHistory * kMaxHistory, kCoefG = 2 * kMaxHistory * kMaxHistory,
              kCoefS = kCoefG + 1, kCoefY = kCoefS + kMaxHistory, kNSyy = kCoefY + kMaxHistory;

// per-slot scalars (double) and integers (int32), one row of kNSc / kNSt per slot
enum SlotScalar {
  SC_J = 0, SC_JT, SC_ALPHA, SC_GTD, SC_GAMMA, SC_H, SC_BV, SC_JG, SC_COEF, SC_MAXD,
  SC_A0 = 12, SC_RHO0 = SC_A0 + kMaxHistory, kNSc = SC_RHO0 + kMaxHistory
};
enum SlotInt {
  ST_MODE = 0, ST_ITER, ST_NH, ST_HEAD, ST_NEXT, ST_TRIALS, ST_BAD, ST_ACC, ST_NEEDDIR,
  ST_MAXIT, ST_STATUS, ST_EVALS, ST_RESET, ST_CLASS, ST_NEWPAIR, kNSt = 16
};
enum SlotMode { MODE_FREE = 0, MODE_INIT = 1, MODE_TRIAL = 2, MODE_DONE = 3 };
// ST_STATUS on completion
enum { SLOT_OK = 0, SLOT_STALLED = 1, SLOT_CONVERGED = 2, SLOT_BAD_START = -5 };

// element classes with their own kernel instantiations
enum ElemClass { CLS_PLAP2 = 0, CLS_PLAP3, CLS_NH2, CLS_NH3, kNumClasses };

// one slot as the batched kernels see it
struct SlotDev {
  TileMesh M;      // the slot's mesh (layout of p1e_mesh_bind inside the slot's allocation)
  double2 *vpart;  // [ntile_v][kNPart] vector-reduction partials
  double *syy;     // [kNSyy] S^T Y, Y^T Y of the stored pairs and the direction's coefficients
  int32_t ntile_h, ntile_v;
  double C1, D1, p, dirichlet_bv;
  int32_t ortho;  // p-Laplacian with the component-wise norm
  // L-BFGS vectors, nfd doubles each; S and Y hold kMaxHistory vectors each
  double *v, *g, *d, *vt, *gt, *S, *Y;
};

// tile tables: (slot, tile) pairs; element tiles and halo-row tiles grouped by class
enum TileKind { TK_TILE = 0, TK_HALO = 1, kNumTileKinds = 2 };
// counts[] layout: for kind k and class c, offset at 2*(k*kNumClasses + c), count next to it;
// the number of vector tiles at kCountVec
constexpr int kCountVec = 2 * kNumTileKinds * kNumClasses;
constexpr int kNumCounts = kCountVec + 1;

// device tables of an engine (all in the table area of its workspace)
struct EngineDev {
  SlotDev *slots;   // [max_slots]
  double *sc;       // [max_slots][kNSc]
  int32_t *st;      // [max_slots][kNSt]
  int2 *map[kNumTileKinds];  // element tiles, halo-row tiles
  int2 *vmap;       // vector tiles over all slots
  int32_t *counts;  // [kNumCounts]
  int32_t max_slots, history;
  int32_t prec;     // P1E_FP64 or P1E_MIXED
};

// enqueue one engine step on stream s (p1e_batch.hip)
int batch_step(const EngineDev &E, hipStream_t s);

}  // namespace p1e
