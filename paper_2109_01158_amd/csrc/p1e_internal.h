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
constexpr int kBlockElem = 512;    // threads (= elements) per block of the element kernel
constexpr int kBlockNode = 1024;   // threads (= nodes) per block of the node prepass
constexpr uint64_t kAlign = 256;   // alignment of every sub-array in the bound buffer

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
  const double *geo64 = nullptr;       // [dim*dim+1][ne]: B^-1 entries (row l-1 = grad phi_l), |T|
  const float *geo32 = nullptr;        // same in FP32 (mixed mode)
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
  std::vector<double> geo64;       // [dim*dim+1][ne]
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
inline int64_t element_blocks(int64_t ne) { return nblocks(ne, kBlockElem); }
inline int64_t node_blocks(int64_t nn) { return nblocks(nn, kBlockNode); }
// per-element scratch is padded to whole element blocks
inline int64_t padded_elements(int64_t ne) { return element_blocks(ne) * kBlockElem; }

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
