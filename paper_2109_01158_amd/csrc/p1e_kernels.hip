// p1e_kernels.hip -- gfx950 kernels of libp1e for one mesh per call, and their launchers.
//
// One call of the library is a short chain of kernels on the caller's stream:
//
//   k_tile      per element tile (one per workgroup; in FP64 a persistent grid): the tile's
//               nodal field u (u = v - x for Neo-Hookean, u = v for the p-Laplacian) staged in
//               LDS; per element G = grad u (eq. Dv), the density W (eqs. neoHook,
//               pLaplacian) and |T| W into a compensated block sum (eq. Denergy), and, by
//               mode, the element forces
//               |T| dW/dF grad phi_l (Section 6.2) or the per-element central differences
//               of |T| W under the perturbation of one row of F (Section 6.1) in LDS; then
//               per node of the tile the part of its patch sum (Section 4.2) that lies in the
//               tile, written as the gradient when the whole patch lies there, else to a halo
//               slot; and b.v of the nodes the tile meets first.
//   k_halo      per node whose patch spans several tiles: sum of its slots in tile order,
//               minus b, written in free-DOF order; its first block runs the finalize.
//   k_finalize  one block: deterministic compensated sums of the tile partials -> J (energy
//               mode; with a gradient the halo kernel does it).
//   k_scale     g = s * (gradient kept by the last p1e_energy_forces), s a device scalar.
//
// No atomics anywhere; every sum has a fixed order. The arithmetic lives in p1e_device.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <mutex>

#include "p1e_device.h"
#include "p1e_internal.h"

// Scratch of p1e_grad_exact_static: the tile partials, bad-element counts and halo partial
// sums of one call, in a fixed per-device array instead of the mesh's bound buffer. In host
// code the name is only a stand-in for the symbol: kernels get the device address that
// hipGetSymbolAddress returns for the current device (static_scratch below).
static __device__ __align__(256) unsigned char scratch[P1E_STATIC_SCRATCH_BYTES];

namespace p1e {
namespace {

using namespace dev;

// ----------------------------------------------------------------------- kernels
// threads per tile workgroup: one element and at most one node per thread, except for the
// patch differences in FP64 (more registers per element; two each)
#ifndef P1E_TILE_THREADS
#define P1E_TILE_THREADS 1024
#endif
template <typename T, int MODE>
constexpr int tile_threads() {
  return is_fd(MODE) ? (kTileElems >= 1024 ? kTileElems / 2 : kTileElems)
                         : (kTileElems > P1E_TILE_THREADS ? P1E_TILE_THREADS : kTileElems);
}
// waves per SIMD to keep registers for: two FP32 tiles fit in LDS (160 KiB), so two
// workgroups per CU (with 1024 threads: 8 waves per SIMD, at most 64 VGPRs); FP64 tiles
// run one per CU
template <typename T, int MODE>
constexpr int tile_waves_per_eu() { return sizeof(T) == 4 ? 2 * tile_threads<T, MODE>() / 256 : 1; }

// FP64 tiles (one per CU, registers to spare) run as a persistent grid that hides the
// loads of a tile's head behind the previous tile; FP32 tiles (two per CU, 64 registers)
// would spill the carried head, and run one per workgroup.
template <typename T>
constexpr bool tile_persistent() { return sizeof(T) == 8; }

template <int DIM, int D, int KIND, typename T, int MODE, int GEO>
__global__ __launch_bounds__((tile_threads<T, MODE>())) __attribute__((amdgpu_waves_per_eu(tile_waves_per_eu<T, MODE>()))) void k_tile(TileMesh M,
                                                                  const T *__restrict__ geo,
                                                                  const double *__restrict__ vhat,
                                                                  double *__restrict__ g,
                                                                  Params prm) {
  constexpr int NT = tile_threads<T, MODE>();
  using Head = typename TileSplit<DIM, NT>::Head;
  __shared__ TileShared<DIM, D, T, MODE, 1 << GEO> sh;
  if constexpr (!tile_persistent<T>()) {  // one tile per workgroup
    Head h;
    tile_head<TileSplit<DIM, NT>::NPT, NT, MODE != MODE_ENERGY>(
        M, xcd_tile(blockIdx.x, gridDim.x), h, threadIdx.x);
    tile_pass<DIM, D, KIND, T, MODE, GEO, NT>(M, h, geo, vhat, g, nullptr, prm, sh,
                                              threadIdx.x);
    return;
  }
  int end, step;
  int t = xcd_first(blockIdx.x, gridDim.x, M.ntiles, end, step);
  if (t >= end) return;
  // persistent: each tile loads the next one's head while it sums its patches
  Head h, hn;
  tile_head<TileSplit<DIM, NT>::NPT, NT, MODE != MODE_ENERGY>(M, t, h, threadIdx.x);
  for (;;) {
    const int tn = t + step < end ? t + step : -1;
    tile_pass<DIM, D, KIND, T, MODE, GEO, NT>(M, h, geo, vhat, g, nullptr, prm, sh,
                                              threadIdx.x, tn, &hn);
    if (tn < 0) break;
    h = hn;
    t = tn;
  }
}

// Deterministic compensated sums of the tiles' partials by one block of NT threads:
// J_grad = sum of the energy partials, b.v = sum of the b.v partials + the constant
// Dirichlet part; out3 = {J, J_grad, b.v} (nullable); flag = bad elements (J = +Inf if any).
template <int NT>
__device__ __forceinline__ void strided_pairs(int n, const double2 *__restrict__ p,
                                              const int32_t *__restrict__ cntp, double &s,
                                              double &c, int &cnt) {
  // rounds of B predicated loads, all in flight together; absent slots add (0, 0), which
  // leaves the compensated pair unchanged
  constexpr int B = 16;
  for (int i = threadIdx.x; i < n; i += B * NT) {
    double2 q[B];
    int k[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int j = i + b * NT;
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

template <int NT>
__device__ __forceinline__ void finalize_block(int nt, const double2 *__restrict__ part,
                                               const int32_t *__restrict__ badp,
                                               double dirichlet_bv, double *out3,
                                               int32_t *flag) {
  double s = 0.0, c = 0.0;
  int cnt = 0;
  strided_pairs<NT>(nt, part, badp, s, c, cnt);
  block_reduce<NT>(s, c, cnt);
  __shared__ double jg;
  __shared__ int nbad;
  if (threadIdx.x == 0) {
    jg = s + c;
    nbad = cnt;
  }
  __syncthreads();
  s = 0.0, c = 0.0;
  int dummy = 0;
  strided_pairs<NT>(nt, part + nt, nullptr, s, c, dummy);
  block_reduce<NT>(s, c, dummy);
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

constexpr int kFin = 1024;

__global__ __launch_bounds__(kFin) void k_finalize(int nt, const double2 *__restrict__ part,
                                                   const int32_t *__restrict__ badp,
                                                   double dirichlet_bv, double *out3,
                                                   int32_t *flag) {
  finalize_block<kFin>(nt, part, badp, dirichlet_bv, out3, flag);
}

// halo rows (blocks 1..) and, in block 0, the finalize: both only read what k_tile wrote
// (halo partials of the tiles' element type T)
template <int D, typename T>
__global__ __launch_bounds__(kBlock) void k_halo(TileMesh M, double *__restrict__ g,
                                                 double dirichlet_bv, double *out3,
                                                 int32_t *flag) {
  if (blockIdx.x == 0) {
    finalize_block<kBlock>(M.ntiles, M.part, M.badp, dirichlet_bv, out3, flag);
    return;
  }
  const int h = (blockIdx.x - 1) * kBlock + threadIdx.x;
  if (h < M.nhalo) halo_row<D, T>(M, h, g, nullptr);
}

// two DOFs per thread as one 16-byte access when g is 16-byte aligned (gw always is)
__global__ __launch_bounds__(kBlock) void k_scale(int n, const double *__restrict__ gw,
                                                  const double *__restrict__ scale,
                                                  double *__restrict__ g) {
  const int i = 2 * (blockIdx.x * kBlock + threadIdx.x);
  if (i >= n) return;
  const double sc = scale ? *scale : 1.0;
  if (i + 1 < n && (reinterpret_cast<uintptr_t>(g) & 15) == 0) {
    const double2 w = *reinterpret_cast<const double2 *>(gw + i);
    *reinterpret_cast<double2 *>(g + i) = make_double2(sc * w.x, sc * w.y);
  } else {
    g[i] = sc * gw[i];
    if (i + 1 < n) g[i + 1] = sc * gw[i + 1];
  }
}

// g *= s in place, s = *scale read by every block; nothing to do (and nothing written) when
// s == 1, where the product would return every g bitwise. Grid-stride over pairs of DOFs.
__global__ __launch_bounds__(kBlock) void k_scale_inplace(int n, const double *__restrict__ scale,
                                                          double *__restrict__ g) {
  const double sc = *scale;
  if (sc == 1.0) return;
  const bool vec = (reinterpret_cast<uintptr_t>(g) & 15) == 0;
  for (int64_t i = 2 * ((int64_t)blockIdx.x * kBlock + threadIdx.x); i < n;
       i += 2 * (int64_t)kBlock * gridDim.x) {
    if (vec && i + 1 < n) {
      double2 *p = reinterpret_cast<double2 *>(g + i);
      const double2 w = *p;
      *p = make_double2(sc * w.x, sc * w.y);
    } else {
      g[i] *= sc;
      if (i + 1 < n) g[i + 1] *= sc;
    }
  }
}

// ----------------------------------------------------------------------- launchers
int check_launch(const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(P1E_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  return P1E_OK;
}

Params params_of(const p1e_mesh *m, double eps) {
  return Params{m->C1, m->D1, m->p, eps, m->ortho, (float)(2.0 * m->C1), (float)(2.0 * m->D1)};
}

// Blocks of a persistent grid over n tiles: as many as the device holds at once (occupancy
// query, once per kernel and device), at most n, rounded up to a multiple of the XCD count.
template <typename F>
int persistent_grid(F kernel, int nt, int64_t n) {
  static int cached_dev = -1, resident = 0;  // per kernel instantiation
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (dev != cached_dev) {
    int per_cu = 0, cus = 0;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, nt, 0);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    resident = std::max(1, per_cu) * std::max(1, cus);
    cached_dev = dev;
  }
  constexpr int X = P1E_XCD_COUNT;
  const int64_t nb = std::min<int64_t>(n, resident);
  return (int)((nb + X - 1) / X * X);
}

// Every launcher takes the device view Mv of the mesh: m->dev, or a copy whose scratch
// pointers lead elsewhere (p1e_grad_exact_static).
template <int DIM, int D, int KIND, typename T, int MODE, int GEO>
void launch_tile_kernel(p1e_mesh *m, const TileMesh &Mv, const T *geo, const double *vhat,
                        double *g, double eps, hipStream_t s) {
  constexpr int NT = tile_threads<T, MODE>();
  auto kern = k_tile<DIM, D, KIND, T, MODE, GEO>;
  const int nb = tile_persistent<T>() ? persistent_grid(kern, NT, m->ntiles) : (int)m->ntiles;
  hipLaunchKernelGGL(kern, dim3(nb), dim3(NT), 0, s, Mv, geo, vhat, g, params_of(m, eps));
}

template <int DIM, int D, int KIND, typename T, int MODE>
int launch_tile(p1e_mesh *m, const TileMesh &Mv, const T *geo, const double *vhat, double *g,
                double eps, hipStream_t s) {
  if (m->ntiles == 0) return P1E_OK;
  const char *name = MODE == MODE_ENERGY ? "k_tile_energy"
                     : MODE == MODE_FORCE ? "k_tile_force"
                     : MODE == MODE_FD    ? "k_tile_fd"
                                          : "k_tile_fd4";
  prof_begin(name, s);
  if (Mv.geo_mode == GEO_CLASS)
    launch_tile_kernel<DIM, D, KIND, T, MODE, GEO_CLASS>(m, Mv, geo, vhat, g, eps, s);
  else if (Mv.geo_mode == GEO_OTF)
    launch_tile_kernel<DIM, D, KIND, T, MODE, GEO_OTF>(m, Mv, geo, vhat, g, eps, s);
  else
    launch_tile_kernel<DIM, D, KIND, T, MODE, GEO_STORED>(m, Mv, geo, vhat, g, eps, s);
  prof_end(s);
  return check_launch(name);
}

// halo rows and finalize (gradient modes)
template <int D, typename T>
int launch_halo(p1e_mesh *m, const TileMesh &Mv, double *g, double *out3, int32_t *flag,
                hipStream_t s) {
  prof_begin("k_halo", s);
  hipLaunchKernelGGL((k_halo<D, T>), dim3(1 + nblocks(m->nhalo)), dim3(kBlock), 0, s, Mv, g,
                     m->dirichlet_bv, out3, flag);
  prof_end(s);
  return check_launch("k_halo");
}

// finalize alone (energy mode)
int launch_finalize(p1e_mesh *m, const TileMesh &Mv, double *out3, int32_t *flag,
                    hipStream_t s) {
  prof_begin("k_finalize", s);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFin), 0, s, (int)m->ntiles, Mv.part, Mv.badp,
                     m->dirichlet_bv, out3, flag);
  prof_end(s);
  return check_launch("k_finalize");
}

// The pipeline for one (DIM, D, KIND, T): tiles (mode), then the finalize, together with
// the halo rows when a gradient is asked for.
template <int DIM, int D, int KIND, typename T, int MODE>
int pipeline(p1e_mesh *m, const TileMesh &Mv, const double *vhat, const T *geo, double eps,
             double *g, double *out3, int32_t *flag, hipStream_t s) {
  int rc = launch_tile<DIM, D, KIND, T, MODE>(m, Mv, geo, vhat, g, eps, s);
  if (rc) return rc;
  if (MODE != MODE_ENERGY) return launch_halo<D, T>(m, Mv, g, out3, flag, s);
  return launch_finalize(m, Mv, out3, flag, s);
}

template <typename T, int MODE>
int dispatch(p1e_mesh *m, const double *vhat, const T *geo, double eps, double *g,
             double *out3, int32_t *flag, hipStream_t s, const TileMesh *view = nullptr) {
  const TileMesh &V = view ? *view : m->dev;
  if (m->kind == P1E_NEOHOOKE) {
    if (m->dim == 3) return pipeline<3, 3, P1E_NEOHOOKE, T, MODE>(m, V, vhat, geo, eps, g, out3, flag, s);
    return pipeline<2, 2, P1E_NEOHOOKE, T, MODE>(m, V, vhat, geo, eps, g, out3, flag, s);
  }
  if (m->kind == P1E_SVK) {
    if (m->dim == 3) return pipeline<3, 3, P1E_SVK, T, MODE>(m, V, vhat, geo, eps, g, out3, flag, s);
    return pipeline<2, 2, P1E_SVK, T, MODE>(m, V, vhat, geo, eps, g, out3, flag, s);
  }
  if (m->kind == P1E_GINZBURG_LANDAU) {
    if (m->dim == 3) return pipeline<3, 1, P1E_GINZBURG_LANDAU, T, MODE>(m, V, vhat, geo, eps, g, out3, flag, s);
    return pipeline<2, 1, P1E_GINZBURG_LANDAU, T, MODE>(m, V, vhat, geo, eps, g, out3, flag, s);
  }
  if (m->dim == 3) return pipeline<3, 1, P1E_PLAPLACE, T, MODE>(m, V, vhat, geo, eps, g, out3, flag, s);
  return pipeline<2, 1, P1E_PLAPLACE, T, MODE>(m, V, vhat, geo, eps, g, out3, flag, s);
}

}  // namespace

// the geometry array of a precision: per-element records or class table, or (GEO_OTF) the
// tile nodes' coordinate offsets
const float *geo32_of(const TileMesh &M) { return M.geo_mode == GEO_OTF ? M.txo32 : M.geo32; }
const double *geo64_of(const TileMesh &M) { return M.geo_mode == GEO_OTF ? M.txo64 : M.geo64; }

int run_energy(p1e_mesh *m, const double *vhat, int prec, double *out3, int32_t *flag,
               hipStream_t s) {
  if (prec == P1E_MIXED)
    return dispatch<float, MODE_ENERGY>(m, vhat, geo32_of(m->dev), 0.0, nullptr, out3, flag, s);
  return dispatch<double, MODE_ENERGY>(m, vhat, geo64_of(m->dev), 0.0, nullptr, out3, flag, s);
}

int run_grad_exact(p1e_mesh *m, const double *vhat, int prec, double *g, double *out3,
                   int32_t *flag, hipStream_t s) {
  if (prec == P1E_MIXED)
    return dispatch<float, MODE_FORCE>(m, vhat, geo32_of(m->dev), 0.0, g, out3, flag, s);
  return dispatch<double, MODE_FORCE>(m, vhat, geo64_of(m->dev), 0.0, g, out3, flag, s);
}

int run_grad_fd(p1e_mesh *m, const double *vhat, double eps, int order, double *g,
                int32_t *flag, hipStream_t s) {
  if (order == 4)
    return dispatch<double, MODE_FD4>(m, vhat, geo64_of(m->dev), eps, g, nullptr, flag, s);
  return dispatch<double, MODE_FD>(m, vhat, geo64_of(m->dev), eps, g, nullptr, flag, s);
}

int run_energy_forces(p1e_mesh *m, const double *vhat, int prec, double *out3, int32_t *flag,
                      hipStream_t s) {
  return run_grad_exact(m, vhat, prec, m->dev.gw, out3, flag, s);
}

// Device address of `scratch` on the current device, looked up once per device (each GPU
// holds its own copy of the array at its own address); nullptr with the HIP status in *err
// if the lookup fails.
static void *static_scratch(hipError_t *err) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void *addr[kMaxDevices] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    *err = e != hipSuccess ? e : hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(mu);
  if (addr[dev] == nullptr) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      *err = e != hipSuccess ? e : hipErrorInvalidSymbol;
      return nullptr;
    }
    addr[dev] = p;
  }
  *err = hipSuccess;
  return addr[dev];
}

// Byte offsets of the three scratch arrays of a call in the static array: tile partials
// [2][ntiles] double2, bad counts [ntiles] int32, halo partials [slots][d] double, each
// 256-byte aligned. Returns the bytes needed.
static uint64_t static_layout(const p1e_mesh *m, uint64_t &part, uint64_t &badp, uint64_t &hpart) {
  auto up = [](uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; };
  const uint64_t nt1 = (uint64_t)std::max<int64_t>(m->ntiles, 1);
  part = 0;
  badp = up(32 * nt1);
  hpart = badp + up(4 * nt1);
  return hpart + 8ull * (uint64_t)m->nslots * (uint64_t)m->d;
}

uint64_t static_scratch_need(const p1e_mesh *m) {
  uint64_t a, b, c;
  return static_layout(m, a, b, c);
}

// p1e_grad_exact with the call's scratch in the static array. Every tile writes its
// partials and bad count and every halo slot is written by the one tile it belongs to before
// k_halo reads it, so nothing needs clearing first; calls that overlap on one device race on
// the array.
int run_grad_exact_static(p1e_mesh *m, const double *vhat, int prec, double *g, double *out3,
                          int32_t *flag, hipStream_t s) {
  uint64_t op, ob, oh;
  const uint64_t need = static_layout(m, op, ob, oh);
  if (need > (uint64_t)P1E_STATIC_SCRATCH_BYTES)
    return fail(P1E_ENOMEM, "mesh needs " + std::to_string(need) +
                                " bytes of scratch, more than the static array's " +
                                std::to_string((uint64_t)P1E_STATIC_SCRATCH_BYTES));
  hipError_t e;
  char *base = (char *)static_scratch(&e);
  if (base == nullptr)
    return fail(P1E_EHIP, std::string("static scratch lookup: ") + hipGetErrorString(e));
  TileMesh V = m->dev;
  V.part = (double2 *)(base + op);
  V.badp = (int32_t *)(base + ob);
  V.hpart = (double *)(base + oh);
  if (prec == P1E_MIXED)
    return dispatch<float, MODE_FORCE>(m, vhat, geo32_of(m->dev), 0.0, g, out3, flag, s, &V);
  return dispatch<double, MODE_FORCE>(m, vhat, geo64_of(m->dev), 0.0, g, out3, flag, s, &V);
}

int run_scale_inplace(p1e_mesh *m, const double *scale, double *g, hipStream_t s) {
  if (m->nfd == 0) return P1E_OK;
  prof_begin("k_scale_inplace", s);
  const int nb = (int)std::min<int64_t>(nblocks((m->nfd + 1) / 2), 1024);
  hipLaunchKernelGGL(k_scale_inplace, dim3(nb), dim3(kBlock), 0, s, (int)m->nfd, scale, g);
  prof_end(s);
  return check_launch("k_scale_inplace");
}

int run_scale(p1e_mesh *m, const double *scale, double *g, hipStream_t s) {
  if (m->nfd == 0) return P1E_OK;
  prof_begin("k_scale", s);
  hipLaunchKernelGGL(k_scale, dim3(nblocks((m->nfd + 1) / 2)), dim3(kBlock), 0, s, (int)m->nfd,
                     (const double *)m->dev.gw, scale, g);
  prof_end(s);
  return check_launch("k_scale");
}

}  // namespace p1e
