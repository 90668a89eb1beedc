// p1e_internal.h -- mesh handle layout and kernel launchers shared by the host setup
// (p1e_api.cpp) and the gfx950 kernels (p1e_kernels.hip). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/p1e.h"

namespace p1e {

constexpr int kBlock = 256;        // threads per block of the patch gather
constexpr int kBlockElem = 512;    // threads per block of the element kernel
#ifndef P1E_ELEM_PER_THREAD
#define P1E_ELEM_PER_THREAD 4
#endif
constexpr int kElemPerThread = P1E_ELEM_PER_THREAD;    // elements per thread (one tile)
constexpr int kElemTile = kBlockElem * kElemPerThread;  // elements per element-kernel tile
constexpr int kBlockNode = 1024;   // threads (= nodes) per block of the node prepass
constexpr uint64_t kAlign = 256;   // alignment of every sub-array in the bound buffer
constexpr int kMaxGeoClasses = 256; // geometry classes kept as one-byte indices

// Device view of a bound mesh. All arrays live in the caller's buffer.
struct DevMesh {
  // node arrays in the caller's (external) node order
  const int32_t *node_info = nullptr;  // [nn]  (first free DOF << 3) | free-component mask
  const int32_t *node_int = nullptr;   // [nn]  internal number of each node
  const double *xref = nullptr;        // [nn][dim] reference coordinates (Neo-Hookean)
  const double *vD = nullptr;          // [nn][d] prescribed values
  // element and patch arrays in internal (locality) order
  const double *bhat = nullptr;        // [n_free_dofs] b = M f on the free DOFs
  const int32_t *conn = nullptr;       // [dim+1][ne] structure of arrays
  // element geometry: B^-1 entries (row l-1 = grad phi_l) and |T|, either per element as
  // [dim*dim+1][ne], or (geometry classes) as a table [nclass][dim*dim+1] indexed by geo_cls
  const double *geo64 = nullptr;       // FP64
  const float *geo32 = nullptr;        // FP32 (mixed mode)
  const uint8_t *geo_cls = nullptr;    // [ne] class of each element, or nullptr
  int nclass = 0;
  const int32_t *row_ptr = nullptr;    // [nf+1] patch rows of free nodes
  const uint32_t *ent = nullptr;       // [nnz] (element << 2) | local vertex, ascending element
  const int32_t *row_info = nullptr;   // [nf] node_info of each free node
  void *u = nullptr;                   // scratch: nodal field [nn][ns] in internal node order,
                                       // ns = 4 if d == 3 else d
  void *r = nullptr;                   // scratch: per-element forces / differences [(dim+1)d][ne]
  double2 *part = nullptr;             // scratch: compensated block partials
  int32_t *badp = nullptr;             // scratch: bad-element counts per block
};

}  // namespace p1e

struct p1e_mesh {
  int dim = 0, d = 0, kind = 0, k = 0;
  int64_t nn = 0, ne = 0, nf = 0, nfd = 0, nnz = 0;
  double p = 2.0, C1 = 0.0, D1 = 0.0;
  int max_valence = 0;
  double total_vol = 0.0, min_vol = 0.0, max_vol = 0.0, dirichlet_bv = 0.0;

  // host copies (kept so the mesh can be bound again)
  std::vector<int32_t> conn;       // [k][ne]
  std::vector<double> geo64;       // [dim*dim+1][ne] (empty when classed)
  int nclass = 0;                  // distinct element geometries when <= kMaxGeoClasses, else 0
  std::vector<uint8_t> geo_cls;    // [ne] class of each element
  std::vector<double> geo_tab;     // [nclass][dim*dim+1]
  std::vector<int32_t> node_info;  // [nn] external order
  std::vector<int32_t> node_int;   // [nn] external -> internal node number
  std::vector<double> xref;        // [nn][dim] (Neo-Hookean only)
  std::vector<double> vD;          // [nn][d]
  std::vector<double> bhat;        // [nfd]
  std::vector<int32_t> row_ptr;    // [nf+1]
  std::vector<uint32_t> ent;       // [nnz]
  std::vector<int32_t> row_info;   // [nf]

  // binding
  int bound_modes = 0;
  int device = -1;
  p1e::DevMesh dev;
  int64_t part_cap = 0;  // number of double2 partial slots
  int forces_prec = 0;   // precision of the element forces held in scratch (0 = none)
};

namespace p1e {

// thread-local error reporting (p1e_api.cpp)
int fail(int code, const std::string &msg);

// kernel timing hooks (p1e_api.cpp); no-ops unless enabled
void prof_begin(const char *name, hipStream_t s);
void prof_end(hipStream_t s);

// number of blocks of the streaming kernels over n items
inline int64_t nblocks(int64_t n, int per = kBlock) { return (n + per - 1) / per; }
inline int64_t element_blocks(int64_t ne) { return nblocks(ne, kElemTile); }
inline int64_t node_blocks(int64_t nn) { return nblocks(nn, kBlockNode); }
// per-element scratch is padded to whole element blocks
inline int64_t padded_elements(int64_t ne) { return element_blocks(ne) * kElemTile; }

// device bytes of each scratch array for the given mode mask
uint64_t u_bytes(const p1e_mesh *m, int modes);
uint64_t r_bytes(const p1e_mesh *m, int modes);
int64_t part_slots(const p1e_mesh *m);

// launchers (p1e_kernels.hip). All enqueue on stream and return P1E_OK or a status.
int run_energy(p1e_mesh *m, const double *vhat, int prec, double *out3, int32_t *flag,
               hipStream_t s);
int run_grad_exact(p1e_mesh *m, const double *vhat, int prec, double *g, double *out3,
                   int32_t *flag, hipStream_t s);
int run_grad_fd(p1e_mesh *m, const double *vhat, double eps, double *g, int32_t *flag,
                hipStream_t s);
int run_energy_forces(p1e_mesh *m, const double *vhat, int prec, double *out3, int32_t *flag,
                      hipStream_t s);
int run_gather(p1e_mesh *m, int prec, const double *scale, double *g, hipStream_t s);

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

// per-slot scalars (double) and integers (int32), one row of kNSc / kNSt per slot
enum SlotScalar {
  SC_J = 0, SC_JT, SC_ALPHA, SC_GTD, SC_GAMMA, SC_H, SC_BV, SC_JG, SC_COEF, SC_MAXD,
  SC_A0 = 12, SC_RHO0 = SC_A0 + kMaxHistory, kNSc = SC_RHO0 + kMaxHistory
};
enum SlotInt {
  ST_MODE = 0, ST_ITER, ST_NH, ST_HEAD, ST_NEXT, ST_TRIALS, ST_BAD, ST_ACC, ST_NEEDDIR,
  ST_MAXIT, ST_STATUS, ST_EVALS, ST_RESET, ST_CLASS, kNSt = 16
};
enum SlotMode { MODE_FREE = 0, MODE_INIT = 1, MODE_TRIAL = 2, MODE_DONE = 3 };
// ST_STATUS on completion
enum { SLOT_OK = 0, SLOT_STALLED = 1, SLOT_CONVERGED = 2, SLOT_BAD_START = -5 };

// element classes with their own kernel instantiations
enum ElemClass { CLS_PLAP2 = 0, CLS_PLAP3, CLS_NH2, CLS_NH3, kNumClasses };

// one slot as the batched kernels see it
struct SlotDev {
  // mesh (layout of p1e_mesh_bind inside the slot's allocation)
  const int32_t *node_info, *node_int;
  const double *xref, *vD, *bhat;
  const int32_t *conn;
  const void *geo;  // double or float by engine precision (class table when gcls is set)
  const uint8_t *gcls;
  const int32_t *row_ptr;
  const uint32_t *ent;
  const int32_t *row_info;
  void *u, *r;
  double2 *part;   // [ntile_e] element partials, then [ntile_n] node partials
  int32_t *badp;   // [ntile_e]
  double2 *vpart;  // [ntile_v][4] vector-reduction partials
  int32_t nn, ne, nep, nf, nfd, ntile_e, ntile_n, ntile_v;
  double C1, D1, p, dirichlet_bv;
  // L-BFGS vectors, nfd doubles each; S and Y hold kMaxHistory vectors each
  double *v, *g, *d, *vt, *gt, *S, *Y;
};

// tile tables: (slot, tile) pairs; element, node and row tiles grouped by class
enum TileKind { TK_ELEM = 0, TK_NODE = 1, TK_ROW = 2 };
// counts[] layout: for kind k and class c, offset at 2*(k*kNumClasses + c), count next to it;
// the number of vector tiles at kCountVec
constexpr int kCountVec = 2 * 3 * kNumClasses;
constexpr int kNumCounts = kCountVec + 1;

// device tables of an engine (all in the table area of its workspace)
struct EngineDev {
  SlotDev *slots;   // [max_slots]
  double *sc;       // [max_slots][kNSc]
  int32_t *st;      // [max_slots][kNSt]
  int2 *map[3];     // element, node, row tiles
  int2 *vmap;       // vector tiles over all slots
  int32_t *counts;  // [kNumCounts]
  int32_t max_slots, history;
  int32_t prec;     // P1E_FP64 or P1E_MIXED
};

// enqueue one engine step on stream s (p1e_batch.hip)
int batch_step(const EngineDev &E, hipStream_t s);
// rows per patch-row tile for a class (matches the gather's lanes per row)
int rows_per_tile(int cls);

}  // namespace p1e
