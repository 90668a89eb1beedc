// p1e_kernels.hip -- gfx950 kernels of libp1e for one mesh per call, and their launchers.
//
// One call of the library is a short chain of streaming kernels on the caller's stream:
//
//   k_prepass   per node: expand the free-DOF vector into a node-major field (u = v - x for
//               Neo-Hookean, u = v for the p-Laplacian) and the partial sums of b.vhat.
//   k_element   per element: gather u at the dim+1 vertices, G = grad u (eq. Dv), the
//               density W (eqs. neoHook, pLaplacian) and |T| W into a compensated block sum
//               (eq. Denergy); optionally the element forces |T| dW/dF grad phi_l
//               (Section 6.2) or the per-element central differences of |T| W under the
//               perturbation of one row of F (Section 6.1).
//   k_finalize  one block: deterministic compensated sum of the block partials -> J.
//   k_gather    per free node: sum its patch entries (Section 4.2 patches; no atomics) and
//               subtract b, written in free-DOF order.
//
// Every array is a structure of arrays indexed by element or node, so consecutive lanes of a
// 64-wide wavefront touch consecutive addresses; only the vertex gathers of u and the patch
// gathers of element forces are indirect. The arithmetic lives in p1e_device.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "p1e_device.h"
#include "p1e_internal.h"

namespace p1e {
namespace {

using namespace dev;

// ----------------------------------------------------------------------- kernels
template <typename T, int D, bool SUB_X>
__global__ __launch_bounds__(kBlockNode) void k_prepass(int nn, const int32_t *__restrict__ node_info,
                                                        const int32_t *__restrict__ node_int,
                                                        const double *__restrict__ vhat,
                                                        const double *__restrict__ vD,
                                                        const double *__restrict__ xref,
                                                        const double *__restrict__ bhat,
                                                        T *__restrict__ u,
                                                        double2 *__restrict__ part) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int i = tile * kBlockNode + threadIdx.x;
  double s = 0.0, c = 0.0;
  int cnt = 0;
  if (i < nn) prepass_node<T, D, SUB_X>(i, node_info, node_int, vhat, vD, xref, bhat, u, s, c);
  block_reduce<kBlockNode>(s, c, cnt);
  if (threadIdx.x == 0) part[tile] = make_double2(s, c);
}

// One tile of kElemTile elements per block. With CLS the (small) table of element records
// is staged in LDS first.
template <int DIM, int D, int KIND, typename T, int MODE, bool CLS>
__global__ __launch_bounds__(kBlockElem) void k_element(int ne, int nep,
                                                        const int32_t *__restrict__ conn,
                                                        const T *__restrict__ geo,
                                                        const uint8_t *__restrict__ gcls,
                                                        int nclass,
                                                        const T *__restrict__ u,
                                                        T *__restrict__ r,
                                                        double2 *__restrict__ part,
                                                        int32_t *__restrict__ badp, Params prm) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  double s = 0.0, c = 0.0;
  int cnt = 0;
  if constexpr (CLS) {
    constexpr int REC = DIM * DIM + 1;
    __shared__ T tab[kMaxGeoClasses * REC];
    for (int q = threadIdx.x; q < nclass * REC; q += kBlockElem) tab[q] = geo[q];
    __syncthreads();
    element_tile<DIM, D, KIND, T, MODE, true>(tile, ne, nep, conn, tab, gcls, u, r, prm, s, c,
                                              cnt);
  } else {
    element_tile<DIM, D, KIND, T, MODE, false>(tile, ne, nep, conn, geo, nullptr, u, r, prm, s,
                                               c, cnt);
  }
  block_reduce<kBlockElem>(s, c, cnt);
  if (threadIdx.x == 0) {
    part[tile] = make_double2(s, c);
    badp[tile] = cnt;
  }
}

template <int K, int D, typename T, int GL, int U>
__global__ __launch_bounds__(kBlock) void k_gather(int nf, int nep,
                                                   const int32_t *__restrict__ row_ptr,
                                                   const uint32_t *__restrict__ ent,
                                                   const int32_t *__restrict__ row_info,
                                                   const T *__restrict__ r,
                                                   const double *__restrict__ bhat,
                                                   const double *__restrict__ scale,
                                                   double *__restrict__ g) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int row = tile * (kBlock / GL) + threadIdx.x / GL;
  gather_row<K, D, T, GL, U>(row, threadIdx.x % GL, nf, nep, row_ptr, ent, row_info, r, bhat,
                             scale, g);
}

// Single block of kFin threads: J_grad = sum of element partials, b.v = sum of node partials
// + the constant Dirichlet part; out3 = {J, J_grad, b.v}; flag = bad elements (J = +Inf if
// any). Each thread reads its strided partials in batches of 8 independent loads.
constexpr int kFin = 1024;

__device__ __forceinline__ void strided_pairs(int n, const double2 *__restrict__ p,
                                              const int32_t *__restrict__ cntp, double &s,
                                              double &c, int &cnt) {
  // rounds of B predicated loads, all in flight together; absent slots add (0, 0), which
  // leaves the compensated pair unchanged
  constexpr int B = 16;
  for (int i = threadIdx.x; i < n; i += B * kFin) {
    double2 q[B];
    int k[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int j = i + b * kFin;
      q[b] = j < n ? p[j] : make_double2(0.0, 0.0);
      k[b] = (cntp && j < n) ? cntp[j] : 0;
    }
#pragma unroll
    for (int b = 0; b < B; ++b) {
      pair_add(s, c, q[b].x, q[b].y);
      cnt += k[b];
    }
  }
}

__global__ __launch_bounds__(kFin) void k_finalize(int nbe, const double2 *__restrict__ pe,
                                                   const int32_t *__restrict__ badp, int nbn,
                                                   const double2 *__restrict__ pn,
                                                   double dirichlet_bv, double *out3,
                                                   int32_t *flag) {
  double s = 0.0, c = 0.0;
  int cnt = 0;
  strided_pairs(nbe, pe, badp, s, c, cnt);
  block_reduce<kFin>(s, c, cnt);
  __shared__ double jg;
  __shared__ int nbad;
  if (threadIdx.x == 0) {
    jg = s + c;
    nbad = cnt;
  }
  __syncthreads();
  s = 0.0, c = 0.0;
  int dummy = 0;
  strided_pairs(nbn, pn, nullptr, s, c, dummy);
  block_reduce<kFin>(s, c, dummy);
  if (threadIdx.x == 0) {
    pair_add(s, c, dirichlet_bv, 0.0);
    const double bv = s + c;
    const double J = nbad ? INFINITY : jg - bv;
    if (out3 != nullptr) {
      out3[0] = J;
      out3[1] = nbad ? INFINITY : jg;
      out3[2] = bv;
    }
    flag[0] = nbad;
  }
}
// ----------------------------------------------------------------------- launchers
int check_launch(const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(P1E_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  return P1E_OK;
}

Params params_of(const p1e_mesh *m, double eps) { return Params{m->C1, m->D1, m->p, eps}; }

template <typename T, int D, bool SUBX>
int launch_prepass(p1e_mesh *m, const double *vhat, double2 *pn, hipStream_t s) {
  const int nb = (int)node_blocks(m->nn);
  prof_begin("k_prepass", s);
  hipLaunchKernelGGL((k_prepass<T, D, SUBX>), dim3(nb), dim3(kBlockNode), 0, s, (int)m->nn,
                     m->dev.node_info, m->dev.node_int, vhat, m->dev.vD, m->dev.xref, m->dev.bhat, (T *)m->dev.u,
                     pn);
  prof_end(s);
  return check_launch("k_prepass");
}

template <int DIM, int D, int KIND, typename T, int MODE>
int launch_element(p1e_mesh *m, const T *geo, double eps, hipStream_t s) {
  if (m->ne == 0) return P1E_OK;
  const int nb = (int)element_blocks(m->ne);
  const char *name = MODE == MODE_ENERGY ? "k_element_energy"
                     : MODE == MODE_FORCE ? "k_element_force"
                                          : "k_element_fd";
  prof_begin(name, s);
  if (m->dev.geo_cls != nullptr)
    hipLaunchKernelGGL((k_element<DIM, D, KIND, T, MODE, true>), dim3(nb), dim3(kBlockElem), 0,
                       s, (int)m->ne, (int)padded_elements(m->ne), m->dev.conn, geo,
                       m->dev.geo_cls, m->dev.nclass, (const T *)m->dev.u, (T *)m->dev.r,
                       m->dev.part, m->dev.badp, params_of(m, eps));
  else
    hipLaunchKernelGGL((k_element<DIM, D, KIND, T, MODE, false>), dim3(nb), dim3(kBlockElem), 0,
                       s, (int)m->ne, (int)padded_elements(m->ne), m->dev.conn, geo, nullptr, 0,
                       (const T *)m->dev.u, (T *)m->dev.r, m->dev.part, m->dev.badp,
                       params_of(m, eps));
  prof_end(s);
  return check_launch(name);
}

// Lanes per patch row and entries per lane per round (3D Kuhn patches hold up to 24
// elements, 2D right-triangle patches 6); both can be set at build time.
template <int DIM>
constexpr int gather_lanes() { return DIM == 3 ? P1E_GATHER_LANES_3D : P1E_GATHER_LANES_2D; }

template <int DIM, int D, typename T>
int launch_gather(p1e_mesh *m, const double *scale, double *g, hipStream_t s) {
  if (m->nf == 0) return P1E_OK;
  constexpr int GL = gather_lanes<DIM>();
  const int rows_per_block = kBlock / GL;
  const int nb = (int)((m->nf + rows_per_block - 1) / rows_per_block);
  prof_begin("k_gather", s);
  hipLaunchKernelGGL((k_gather<DIM + 1, D, T, GL, P1E_GATHER_UNROLL>), dim3(nb), dim3(kBlock), 0, s, (int)m->nf,
                     (int)padded_elements(m->ne),
                     m->dev.row_ptr, m->dev.ent, m->dev.row_info, (const T *)m->dev.r,
                     m->dev.bhat, scale, g);
  prof_end(s);
  return check_launch("k_gather");
}

int launch_finalize(p1e_mesh *m, const double2 *pn, double *out3, int32_t *flag,
                    hipStream_t s) {
  const int nbe = m->ne ? (int)element_blocks(m->ne) : 0;
  const int nbn = (int)node_blocks(m->nn);
  prof_begin("k_finalize", s);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFin), 0, s, nbe, m->dev.part, m->dev.badp, nbn,
                     pn, m->dirichlet_bv, out3, flag);
  prof_end(s);
  return check_launch("k_finalize");
}

// node partials follow the element partials (the layout reserves 2 x part_cap slots)
double2 *node_partials(p1e_mesh *m) { return m->dev.part + m->part_cap; }

// The pipeline for one (DIM, D, KIND, T): prepass, element pass (mode), finalize, and the
// patch gather when g is given.
template <int DIM, int D, int KIND, typename T, int MODE>
int pipeline(p1e_mesh *m, const double *vhat, const T *geo, double eps, double *g,
             double *out3, int32_t *flag, hipStream_t s) {
  constexpr bool SUBX = KIND == P1E_NEOHOOKE;
  double2 *pn = node_partials(m);
  int rc = launch_prepass<T, D, SUBX>(m, vhat, pn, s);
  if (rc) return rc;
  rc = launch_element<DIM, D, KIND, T, MODE>(m, geo, eps, s);
  if (rc) return rc;
  rc = launch_finalize(m, pn, out3, flag, s);
  if (rc) return rc;
  if (MODE != MODE_ENERGY && g != nullptr) rc = launch_gather<DIM, D, T>(m, nullptr, g, s);
  return rc;
}

template <typename T, int MODE>
int dispatch(p1e_mesh *m, const double *vhat, const T *geo, double eps, double *g,
             double *out3, int32_t *flag, hipStream_t s) {
  if (m->kind == P1E_NEOHOOKE) {
    if (m->dim == 3) return pipeline<3, 3, P1E_NEOHOOKE, T, MODE>(m, vhat, geo, eps, g, out3, flag, s);
    return pipeline<2, 2, P1E_NEOHOOKE, T, MODE>(m, vhat, geo, eps, g, out3, flag, s);
  }
  if (m->dim == 3) return pipeline<3, 1, P1E_PLAPLACE, T, MODE>(m, vhat, geo, eps, g, out3, flag, s);
  return pipeline<2, 1, P1E_PLAPLACE, T, MODE>(m, vhat, geo, eps, g, out3, flag, s);
}

template <typename T>
int dispatch_gather(p1e_mesh *m, const double *scale, double *g, hipStream_t s) {
  if (m->kind == P1E_NEOHOOKE) {
    if (m->dim == 3) return launch_gather<3, 3, T>(m, scale, g, s);
    return launch_gather<2, 2, T>(m, scale, g, s);
  }
  if (m->dim == 3) return launch_gather<3, 1, T>(m, scale, g, s);
  return launch_gather<2, 1, T>(m, scale, g, s);
}

}  // namespace

int run_energy(p1e_mesh *m, const double *vhat, int prec, double *out3, int32_t *flag,
               hipStream_t s) {
  if (prec == P1E_MIXED)
    return dispatch<float, MODE_ENERGY>(m, vhat, m->dev.geo32, 0.0, nullptr, out3, flag, s);
  return dispatch<double, MODE_ENERGY>(m, vhat, m->dev.geo64, 0.0, nullptr, out3, flag, s);
}

int run_grad_exact(p1e_mesh *m, const double *vhat, int prec, double *g, double *out3,
                   int32_t *flag, hipStream_t s) {
  if (prec == P1E_MIXED)
    return dispatch<float, MODE_FORCE>(m, vhat, m->dev.geo32, 0.0, g, out3, flag, s);
  return dispatch<double, MODE_FORCE>(m, vhat, m->dev.geo64, 0.0, g, out3, flag, s);
}

int run_grad_fd(p1e_mesh *m, const double *vhat, double eps, double *g, int32_t *flag,
                hipStream_t s) {
  return dispatch<double, MODE_FD>(m, vhat, m->dev.geo64, eps, g, nullptr, flag, s);
}

int run_energy_forces(p1e_mesh *m, const double *vhat, int prec, double *out3, int32_t *flag,
                      hipStream_t s) {
  if (prec == P1E_MIXED)
    return dispatch<float, MODE_FORCE>(m, vhat, m->dev.geo32, 0.0, nullptr, out3, flag, s);
  return dispatch<double, MODE_FORCE>(m, vhat, m->dev.geo64, 0.0, nullptr, out3, flag, s);
}

int run_gather(p1e_mesh *m, int prec, const double *scale, double *g, hipStream_t s) {
  if (prec == P1E_MIXED) return dispatch_gather<float>(m, scale, g, s);
  return dispatch_gather<double>(m, scale, g, s);
}

}  // namespace p1e
