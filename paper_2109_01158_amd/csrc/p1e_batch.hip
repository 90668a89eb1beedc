// p1e_batch.hip -- batched kernels of the multi-request engine: every kernel walks a device
// table of (slot, tile) pairs with a fixed grid (grid-stride), so one launch covers all active
// requests of an element class and the launch parameters never change while requests come
// and go. Each slot's work is split into the same tiles and reduced in the same order whether
// it runs alone or among others, so its results are bitwise identical either way.
//
// One engine step advances every active slot by one L-BFGS line-search trial (memory m,
// H0 = (s.y / y.y) I, the product H g in compact form, Armijo backtracking by halving, first
// step scaled so that the largest nodal update is 0.1 h):
//   evaluate   J and grad J at the trial point vt (element tiles, halo rows, finalize; the
//              same bodies as the single-mesh path, Sections 5 and 6.2)
//   decide     accept (Armijo) or halve the step
//   update     v, g and the newest (s, y) pair of accepted slots; trial point of rejected ones
//   direction  d = -H g for slots that accepted, then the next trial point
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "p1e_device.h"
#include "p1e_internal.h"

namespace p1e {
namespace {

using namespace dev;

constexpr double kArmijo = 1e-4;
constexpr int kVB = 256;  // threads of the vector and per-slot kernels

__device__ __forceinline__ int slot_mode(const EngineDev &E, int slot) {
  return E.st[slot * kNSt + ST_MODE];
}
__device__ __forceinline__ bool evaluating(const EngineDev &E, int slot) {
  const int m = slot_mode(E, slot);
  return m == MODE_INIT || m == MODE_TRIAL;
}

// the tiles of kind K and class C: [map + off, map + off + count)
template <int K, int C>
__device__ __forceinline__ const int2 *tiles(const EngineDev &E, int &count) {
  const int off = E.counts[2 * (K * kNumClasses + C)];
  count = E.counts[2 * (K * kNumClasses + C) + 1];
  return E.map[K] + off;
}

// ----------------------------------------------------------------------- evaluation
// element tiles of every evaluating slot of class C (persistent grid over the tile table)
template <typename T>
constexpr int batch_tile_threads() {
  return sizeof(T) == 4 ? (kTileElems < 1024 ? kTileElems : 1024)
                        : (kTileElems < 512 ? kTileElems : 512);
}

template <int DIM, int D, int KIND, typename T, int C>
__global__ __launch_bounds__((batch_tile_threads<T>())) void kb_tile(EngineDev E) {
  constexpr int NT = batch_tile_threads<T>();
  __shared__ TileShared<DIM, D, T, MODE_FORCE, (1 << GEO_STORED) | (1 << GEO_CLASS) | (1 << GEO_OTF)> sh;
  int count;
  const int2 *tl = tiles<TK_TILE, C>(E, count);
  for (int t = blockIdx.x; t < count; t += gridDim.x) {
    const int2 st = tl[t];
    if (!evaluating(E, st.x)) continue;
    const SlotDev &S = E.slots[st.x];
    const Params prm{S.C1, S.D1, S.p, 0.0, S.ortho, (float)(2.0 * S.C1), (float)(2.0 * S.D1)};
    const bool otf = S.M.geo_mode == GEO_OTF;
    const T *geo = sizeof(T) == 4 ? (const T *)(otf ? (const void *)S.M.txo32 : S.M.geo32)
                                  : (const T *)(otf ? (const void *)S.M.txo64 : S.M.geo64);
    using Split = TileSplit<DIM, NT>;
    typename Split::Head h;
    tile_head<Split::NPT, NT, true>(S.M, st.y, h, threadIdx.x);
    if (S.M.geo_mode == GEO_CLASS)
      tile_pass<DIM, D, KIND, T, MODE_FORCE, GEO_CLASS, NT>(S.M, h, geo, S.vt, S.gt, nullptr,
                                                            prm, sh, threadIdx.x);
    else if (otf)
      tile_pass<DIM, D, KIND, T, MODE_FORCE, GEO_OTF, NT>(S.M, h, geo, S.vt, S.gt, nullptr,
                                                          prm, sh, threadIdx.x);
    else
      tile_pass<DIM, D, KIND, T, MODE_FORCE, GEO_STORED, NT>(S.M, h, geo, S.vt, S.gt, nullptr,
                                                             prm, sh, threadIdx.x);
  }
}

// halo rows (kBlock per tile) of every evaluating slot of class C; partials of type T
template <int D, int C, typename T>
__global__ __launch_bounds__(kBlock) void kb_halo(EngineDev E) {
  int count;
  const int2 *tl = tiles<TK_HALO, C>(E, count);
  for (int t = blockIdx.x; t < count; t += gridDim.x) {
    const int2 st = tl[t];
    if (!evaluating(E, st.x)) continue;
    const SlotDev &S = E.slots[st.x];
    const int h = st.y * kBlock + threadIdx.x;
    if (h < S.M.nhalo) halo_row<D, T>(S.M, h, S.gt, nullptr);
  }
}

// (s, c) sum of n pairs p[stride * i + off] in a fixed order; every thread of the block
// calls it, thread 0 gets the result
__device__ __forceinline__ void slot_sum(const double2 *p, int n, int stride, int off,
                                         const int32_t *cntp, double &s, double &c, int &cnt) {
  s = 0.0, c = 0.0;
  cnt = 0;
  for (int i = threadIdx.x; i < n; i += kVB) {
    const double2 q = p[(int64_t)stride * i + off];
    pair_add(s, c, q.x, q.y);
    if (cntp) cnt += cntp[i];
  }
  block_reduce<kVB>(s, c, cnt);
}

// max over n values p[stride * i + off].x, thread 0 gets it
__device__ __forceinline__ double slot_max(const double2 *p, int n, int stride, int off) {
  __shared__ double sh[kVB / 64];
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += kVB) m = fmax(m, p[(int64_t)stride * i + off].x);
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_down(m, o, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int w = 1; w < kVB / 64; ++w) m = fmax(m, sh[w]);
  __syncthreads();
  return m;
}

// one block per slot: J_t = J_grad - b.v of the trial point, and its bad-element count
__global__ __launch_bounds__(kVB) void kb_finalize(EngineDev E) {
  const int slot = blockIdx.x;
  if (!evaluating(E, slot)) return;
  const SlotDev &S = E.slots[slot];
  double s, c, s2, c2;
  int cnt, dummy;
  slot_sum(S.M.part, S.M.ntiles, 1, 0, S.M.badp, s, c, cnt);
  __syncthreads();
  slot_sum(S.M.part + S.M.ntiles, S.M.ntiles, 1, 0, nullptr, s2, c2, dummy);
  if (threadIdx.x == 0) {
    double *sc = E.sc + slot * kNSc;
    int *st = E.st + slot * kNSt;
    pair_add(s2, c2, S.dirichlet_bv, 0.0);
    const double jg = s + c, bv = s2 + c2;
    sc[SC_JG] = jg;
    sc[SC_BV] = bv;
    sc[SC_JT] = cnt ? INFINITY : jg - bv;
    st[ST_BAD] = cnt;
    st[ST_EVALS] += 1;
  }
}

// ----------------------------------------------------------------------- line search
// one thread per slot: accept the trial point (Armijo) or halve the step
__global__ __launch_bounds__(kVB) void kb_decide(EngineDev E) {
  const int slot = blockIdx.x * kVB + threadIdx.x;
  if (slot >= E.max_slots) return;
  double *sc = E.sc + slot * kNSc;
  int *st = E.st + slot * kNSt;
  const int mode = st[ST_MODE];
  int acc = 0, needdir = 0;
  if (mode == MODE_INIT) {
    if (st[ST_BAD] != 0 || !isfinite(sc[SC_JT])) {
      st[ST_MODE] = MODE_DONE;
      st[ST_STATUS] = SLOT_BAD_START;
    } else {
      sc[SC_J] = sc[SC_JT];
      acc = 1;
      needdir = st[ST_MAXIT] > 0;
      if (!needdir) st[ST_MODE] = MODE_DONE;
    }
  } else if (mode == MODE_TRIAL) {
    const double Jt = sc[SC_JT];
    const bool ok = st[ST_BAD] == 0 && isfinite(Jt) &&
                    Jt <= sc[SC_J] + kArmijo * sc[SC_ALPHA] * sc[SC_GTD];
    if (ok) {
      acc = 2;
      sc[SC_J] = Jt;
      st[ST_ITER] += 1;
      st[ST_NEXT] = (st[ST_HEAD] + 1) % E.history;
      needdir = st[ST_ITER] < st[ST_MAXIT];
      if (!needdir) {
        st[ST_MODE] = MODE_DONE;
        st[ST_STATUS] = SLOT_OK;
      }
    } else if (++st[ST_TRIALS] >= kMaxLineTrials) {
      st[ST_MODE] = MODE_DONE;
      st[ST_STATUS] = SLOT_STALLED;
    } else {
      sc[SC_ALPHA] *= 0.5;
    }
  }
  st[ST_ACC] = acc;
  st[ST_NEEDDIR] = needdir;
  st[ST_NEWPAIR] = 0;  // set by kb_hist when a new pair is kept
}

// per-tile view of a slot's vectors for the vector kernels
struct VTile {
  int slot, n, i0;
};
__device__ __forceinline__ VTile vtile(const EngineDev &E, int t) {
  const int2 st = E.vmap[t];
  VTile v;
  v.slot = st.x;
  v.n = E.slots[st.x].M.nfd;
  v.i0 = st.y * kVecTile;
  return v;
}

// accepted slots: newest (s, y) pair and v, g <- vt, gt, with the partial dots y.s, y.y, s.s;
// rejected slots: the next trial point v + alpha d
__global__ __launch_bounds__(kVB) void kb_vupdate(EngineDev E) {
  __shared__ double sh[3][2][kVB / 64];
  const int count = E.counts[kCountVec];
  for (int t = blockIdx.x; t < count; t += gridDim.x) {
    const VTile V = vtile(E, t);
    const SlotDev &S = E.slots[V.slot];
    const int *st = E.st + V.slot * kNSt;
    const int acc = st[ST_ACC], mode = st[ST_MODE];
    if (acc == 0) {
      if (mode == MODE_TRIAL) {
        const double alpha = E.sc[V.slot * kNSc + SC_ALPHA];
        for (int k = 0; k < kVecTile; k += kVB) {
          const int i = V.i0 + k + threadIdx.x;
          if (i < V.n) S.vt[i] = S.v[i] + alpha * S.d[i];
        }
      }
      continue;
    }
    double q[3][2] = {{0, 0}, {0, 0}, {0, 0}};
    const int64_t off = (int64_t)st[ST_NEXT] * V.n;
    for (int k = 0; k < kVecTile; k += kVB) {
      const int i = V.i0 + k + threadIdx.x;
      if (i < V.n) {
        const double vt = S.vt[i], gt = S.gt[i];
        if (acc == 2) {
          const double sv = vt - S.v[i], yv = gt - S.g[i];
          S.S[off + i] = sv;
          S.Y[off + i] = yv;
          double tt, e;
          two_sum(q[0][0], yv * sv, tt, e), q[0][0] = tt, q[0][1] += e;
          two_sum(q[1][0], yv * yv, tt, e), q[1][0] = tt, q[1][1] += e;
          two_sum(q[2][0], sv * sv, tt, e), q[2][0] = tt, q[2][1] += e;
        }
        S.v[i] = vt;
        S.g[i] = gt;
      }
    }
    if (acc == 2) {  // (uniform over the block) the three pairs' block sums together: the
      // shuffle trees of block_reduce, then one LDS exchange
      for (int o = 32; o > 0; o >>= 1) {
        double q2[3][2];
#pragma unroll
        for (int j = 0; j < 3; ++j)
          q2[j][0] = __shfl_down(q[j][0], o, 64), q2[j][1] = __shfl_down(q[j][1], o, 64);
#pragma unroll
        for (int j = 0; j < 3; ++j) pair_add(q[j][0], q[j][1], q2[j][0], q2[j][1]);
      }
      if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int j = 0; j < 3; ++j)
          sh[j][0][threadIdx.x >> 6] = q[j][0], sh[j][1][threadIdx.x >> 6] = q[j][1];
      __syncthreads();
      if (threadIdx.x == 0)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          for (int w = 1; w < kVB / 64; ++w) pair_add(q[j][0], q[j][1], sh[j][0][w], sh[j][1][w]);
          S.vpart[kNPart * (V.i0 / kVecTile) + j] = make_double2(q[j][0], q[j][1]);
        }
      __syncthreads();
    }
  }
}

// one block per accepted slot: keep the new pair if s.y > 1e-12 |s||y| (then rho, gamma)
__global__ __launch_bounds__(kVB) void kb_hist(EngineDev E) {
  const int slot = blockIdx.x;
  int *st = E.st + slot * kNSt;
  if (st[ST_ACC] != 2) return;
  const SlotDev &S = E.slots[slot];
  double r[3];
  for (int j = 0; j < 3; ++j) {
    double s, c;
    int cnt;
    slot_sum(S.vpart, S.ntile_v, kNPart, j, nullptr, s, c, cnt);
    r[j] = s + c;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double *sc = E.sc + slot * kNSc;
    const double ys = r[0], yy = r[1], ss = r[2];
    const int m = E.history;
    if (ys > 1e-12 * sqrt(yy * ss) && isfinite(ys) && yy > 0.0) {
      const int next = st[ST_NEXT];
      st[ST_HEAD] = next;
      st[ST_NH] = min(st[ST_NH] + 1, m);
      st[ST_NEWPAIR] = 1;
      sc[SC_RHO0 + next] = 1.0 / ys;
      sc[SC_GAMMA] = ys / yy;
    } else if (st[ST_NH] == m) {
      st[ST_NH] = m - 1;  // the oldest pair was overwritten by the rejected one
    }
  }
}

// ----------------------------------------------------------------------- direction
__device__ __forceinline__ bool needs_dir(const EngineDev &E, int slot) {
  return E.st[slot * kNSt + ST_NEEDDIR] != 0;
}

// history index of loop position i (0 = newest) or -1 if beyond the stored pairs
__device__ __forceinline__ int hist_index(const EngineDev &E, int slot, int i) {
  const int *st = E.st + slot * kNSt;
  if (i >= st[ST_NH]) return -1;
  return (st[ST_HEAD] - i + E.history) % E.history;
}

// The direction d = -H g in the compact form of the L-BFGS matrix (Byrd, Nocedal and
// Schnabel): with the stored pairs in chronological order, R the upper triangle (diagonal
// included) of S^T Y, D its diagonal and H0 = gamma I (gamma = s.y / y.y of the newest pair),
//   H g = gamma g + S w - gamma Y t,  t = R^-1 S^T g,  w = R^-T ((D + gamma Y^T Y) t - gamma Y^T g),
// the product the two-loop recursion forms, in three launches: one pass for the dot products
// S^T g and Y^T g (and, after a new pair, S^T y_new and Y^T y_new, which extend the S^T Y and
// Y^T Y kept per slot), an O(m^2) solve per slot, and one pass forming d.
constexpr int kNDot = 4 * kMaxHistory;  // dot products of the first pass, by loop position i:
// [i] s_i.g, [M + i] y_i.g, [2M + i] s_i.y_new, [3M + i] y_i.y_new (M = kMaxHistory)

// first pass: per vector tile, the partial dot products of the stored pairs with g (and with
// the new pair's y) into vpart[tile][0 .. kNDot)
__global__ __launch_bounds__(kVB) void kb_dots(EngineDev E) {
  __shared__ double sh[kVB / 64][kNDot];
  const int count = E.counts[kCountVec];
  for (int t = blockIdx.x; t < count; t += gridDim.x) {
    const VTile V = vtile(E, t);
    if (!needs_dir(E, V.slot)) continue;
    const int *st = E.st + V.slot * kNSt;
    const int nh = st[ST_NH];
    if (nh == 0) continue;  // d = -g: no dot products
    const bool newp = st[ST_NEWPAIR] != 0;
    const SlotDev &S = E.slots[V.slot];
    const double *ynew = S.Y + (int64_t)st[ST_HEAD] * V.n;
    const double *si_[kMaxHistory], *yi_[kMaxHistory];
#pragma unroll
    for (int i = 0; i < kMaxHistory; ++i) {
      const int64_t h = i < nh ? hist_index(E, V.slot, i) : 0;
      si_[i] = S.S + h * V.n;
      yi_[i] = S.Y + h * V.n;
    }
    double acc[kNDot];
#pragma unroll
    for (int q = 0; q < kNDot; ++q) acc[q] = 0.0;
    for (int k = 0; k < kVecTile; k += kVB) {
      const int j = V.i0 + k + threadIdx.x;
      if (j >= V.n) continue;
      const double gj = S.g[j], yn = newp ? ynew[j] : 0.0;
#pragma unroll
      for (int i = 0; i < kMaxHistory; ++i) {
        if (i >= nh) break;
        const double si = si_[i][j], yi = yi_[i][j];
        acc[i] = fma(si, gj, acc[i]);
        acc[kMaxHistory + i] = fma(yi, gj, acc[kMaxHistory + i]);
        acc[2 * kMaxHistory + i] = fma(si, yn, acc[2 * kMaxHistory + i]);
        acc[3 * kMaxHistory + i] = fma(yi, yn, acc[3 * kMaxHistory + i]);
      }
    }
    // every wavefront's sums into the LDS, then the wavefronts' in order (plain FP64)
#pragma unroll
    for (int q = 0; q < kNDot; ++q) {
      const int i = q % kMaxHistory, kind = q / kMaxHistory;
      if (i >= nh || (kind >= 2 && !newp)) continue;  // uniform over the block
      const double r = wave_sum(acc[q]);
      if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6][q] = r;
    }
    __syncthreads();
    const int q = threadIdx.x, i = q % kMaxHistory, kind = q / kMaxHistory;
    if (q < kNDot && i < nh && (kind < 2 || newp)) {
      double r = 0.0;
      for (int w = 0; w < kVB / 64; ++w) r += sh[w][q];
      S.vpart[(int64_t)kNPart * (V.i0 / kVecTile) + q] = make_double2(r, 0.0);
    }
    __syncthreads();
  }
}

// one block per slot: the dot products summed over the slot's tiles (fixed order), S^T Y and
// Y^T Y extended by the new pair, the compact solve, and the coefficients of the second pass
// in syy: [kCoefG] for g, [kCoefS + h] for S_h, [kCoefY + h] for Y_h (d = -g without pairs)
constexpr int kCB = 1024;  // threads of kb_compact
__global__ __launch_bounds__(kCB) void kb_compact(EngineDev E) {
  constexpr int M = kMaxHistory, CH = kCB / kNDot;  // chunks of tiles per dot product
  constexpr int U = 4;                              // loads in flight per chunk
  __shared__ double red[CH][kNDot], val[kNDot], sy[M * M], yy[M * M];
  const int slot = blockIdx.x;
  if (!needs_dir(E, slot)) return;
  const SlotDev &S = E.slots[slot];
  const int *st = E.st + slot * kNSt;
  const int nh = st[ST_NH], head = st[ST_HEAD], m = E.history;
  const bool newp = st[ST_NEWPAIR] != 0;
  double *syy = S.syy;
  if (nh > 0) {
    for (int i = threadIdx.x; i < M * M; i += kCB) {
      sy[i] = syy[kSY + i];
      yy[i] = syy[kYY + i];
    }
    const int q = threadIdx.x % kNDot, ch = threadIdx.x / kNDot;
    double s = 0.0, c = 0.0;
    const int i = q % M, kind = q / M;
    if (i < nh && (kind < 2 || newp))
      for (int t0 = ch; t0 < S.ntile_v; t0 += U * CH) {
        double x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int tt = t0 + u * CH;
          x[u] = tt < S.ntile_v ? S.vpart[(int64_t)kNPart * tt + q].x : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) pair_add(s, c, x[u], 0.0);
      }
    red[ch][q] = s + c;
    __syncthreads();
    if (threadIdx.x < kNDot) {
      double r = 0.0;
      for (int w = 0; w < CH; ++w) r += red[w][threadIdx.x];
      val[threadIdx.x] = r;
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  if (nh == 0) {
    syy[kCoefG] = -1.0;
    return;
  }
  auto hist = [&](int i) { return (head - i + m) % m; };  // loop position i, 0 = newest
  if (newp) {  // the newest pair against every stored pair (i = 0: itself)
    for (int i = 0; i < nh; ++i) {
      const int hi = hist(i);
      sy[hi * M + head] = syy[kSY + hi * M + head] = val[2 * M + i];  // s_hi . y_new
      yy[hi * M + head] = syy[kYY + hi * M + head] = val[3 * M + i];  // y_hi . y_new
      yy[head * M + hi] = syy[kYY + head * M + hi] = val[3 * M + i];
    }
  }
  // chronological position c (0 = oldest) -> storage index; loops unrolled over M with
  // predicates, so that t, w and h stay in registers
  int h[M];
#pragma unroll
  for (int c = 0; c < M; ++c) h[c] = c < nh ? hist(nh - 1 - c) : 0;
  const double gamma = E.sc[slot * kNSc + SC_GAMMA];
  double t[M], w[M];
#pragma unroll
  for (int c = M - 1; c >= 0; --c) {  // R t = S^T g (back substitution)
    double r = 0.0;
    if (c < nh) {
      r = val[nh - 1 - c];
#pragma unroll
      for (int c2 = c + 1; c2 < M; ++c2)
        if (c2 < nh) r -= sy[h[c] * M + h[c2]] * t[c2];
      r /= sy[h[c] * M + h[c]];
    }
    t[c] = r;
  }
#pragma unroll
  for (int c = 0; c < M; ++c) {  // (D + gamma Y^T Y) t - gamma Y^T g
    double r = 0.0;
    if (c < nh) {
      r = sy[h[c] * M + h[c]] * t[c] - gamma * val[M + nh - 1 - c];
#pragma unroll
      for (int c2 = 0; c2 < M; ++c2)
        if (c2 < nh) r += gamma * yy[h[c] * M + h[c2]] * t[c2];
    }
    w[c] = r;
  }
#pragma unroll
  for (int c = 0; c < M; ++c) {  // R^T w' = w (forward substitution)
    if (c < nh) {
      double r = w[c];
#pragma unroll
      for (int c2 = 0; c2 < c; ++c2) r -= sy[h[c2] * M + h[c]] * w[c2];
      w[c] = r / sy[h[c] * M + h[c]];
    }
  }
  syy[kCoefG] = -gamma;
#pragma unroll
  for (int c = 0; c < M; ++c)
    if (c < nh) {
      syy[kCoefS + h[c]] = -w[c];
      syy[kCoefY + h[c]] = gamma * t[c];
    }
}

// second pass: d = cg g + sum_i (cS_i S_i + cY_i Y_i) (loop position order), with the
// partials g.d, max|d|, g.g, max|g|
__global__ __launch_bounds__(kVB) void kb_dir(EngineDev E) {
  __shared__ double sh[6][kVB / 64];
  const int count = E.counts[kCountVec];
  for (int t = blockIdx.x; t < count; t += gridDim.x) {
    const VTile V = vtile(E, t);
    if (!needs_dir(E, V.slot)) continue;
    const SlotDev &S = E.slots[V.slot];
    const int nh = E.st[V.slot * kNSt + ST_NH];
    const double cg = S.syy[kCoefG];
    const double *si_[kMaxHistory], *yi_[kMaxHistory];
    double cs[kMaxHistory], cy[kMaxHistory];
#pragma unroll
    for (int i = 0; i < kMaxHistory; ++i) {
      const int64_t h = i < nh ? hist_index(E, V.slot, i) : 0;
      si_[i] = S.S + h * V.n;
      yi_[i] = S.Y + h * V.n;
      cs[i] = i < nh ? S.syy[kCoefS + h] : 0.0;
      cy[i] = i < nh ? S.syy[kCoefY + h] : 0.0;
    }
    double s = 0.0, c = 0.0, gg = 0.0, ggc = 0.0, md = 0.0, mg = 0.0;
    for (int k = 0; k < kVecTile; k += kVB) {
      const int j = V.i0 + k + threadIdx.x;
      if (j >= V.n) continue;
      const double gj = S.g[j];
      double dj = cg * gj;
#pragma unroll
      for (int i = 0; i < kMaxHistory; ++i) {
        if (i >= nh) break;
        dj = fma(cs[i], si_[i][j], dj);
        dj = fma(cy[i], yi_[i][j], dj);
      }
      S.d[j] = dj;
      double tt, e;
      two_sum(s, gj * dj, tt, e), s = tt, c += e;
      two_sum(gg, gj * gj, tt, e), gg = tt, ggc += e;
      md = fmax(md, fabs(dj));
      mg = fmax(mg, fabs(gj));
    }
    // the two compensated sums and the two maxima together: the shuffle trees of block_reduce
    // within each wavefront, then one LDS exchange (the same results, fewer barriers)
    for (int o = 32; o > 0; o >>= 1) {
      const double s2 = __shfl_down(s, o, 64), c2 = __shfl_down(c, o, 64);
      const double g2 = __shfl_down(gg, o, 64), gc2 = __shfl_down(ggc, o, 64);
      pair_add(s, c, s2, c2);
      pair_add(gg, ggc, g2, gc2);
      md = fmax(md, __shfl_down(md, o, 64));
      mg = fmax(mg, __shfl_down(mg, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
      const int w = threadIdx.x >> 6;
      sh[0][w] = s, sh[1][w] = c, sh[2][w] = gg, sh[3][w] = ggc, sh[4][w] = md, sh[5][w] = mg;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 1; w < kVB / 64; ++w) {
        pair_add(s, c, sh[0][w], sh[1][w]);
        pair_add(gg, ggc, sh[2][w], sh[3][w]);
        md = fmax(md, sh[4][w]);
        mg = fmax(mg, sh[5][w]);
      }
      double2 *p = S.vpart + (int64_t)kNPart * (V.i0 / kVecTile);
      p[0] = make_double2(s, c);
      p[1] = make_double2(md, 0.0);
      p[2] = make_double2(gg, ggc);
      p[3] = make_double2(mg, 0.0);
    }
    __syncthreads();
  }
}

// one block per slot: directional derivative, fallback to steepest descent, first step size
__global__ __launch_bounds__(kVB) void kb_dirfin(EngineDev E) {
  const int slot = blockIdx.x;
  if (!needs_dir(E, slot)) return;
  const SlotDev &S = E.slots[slot];
  double s, c, s2, c2;
  int cnt;
  slot_sum(S.vpart, S.ntile_v, kNPart, 0, nullptr, s, c, cnt);
  __syncthreads();
  slot_sum(S.vpart, S.ntile_v, kNPart, 2, nullptr, s2, c2, cnt);
  const double md = slot_max(S.vpart, S.ntile_v, kNPart, 1);
  const double mg = slot_max(S.vpart, S.ntile_v, kNPart, 3);
  if (threadIdx.x == 0) {
    double *sc = E.sc + slot * kNSc;
    int *st = E.st + slot * kNSt;
    double gtd = s + c, maxd = md;
    int reset = 0;
    if (!(gtd < 0.0) || !isfinite(gtd) || !(maxd > 0.0) || !isfinite(maxd)) {
      reset = 1;  // not a descent direction: restart from steepest descent
      st[ST_NH] = 0;
      gtd = -(s2 + c2);
      maxd = mg;
    }
    st[ST_RESET] = reset;
    if (!(maxd > 0.0)) {  // zero gradient: stationary point reached
      st[ST_MODE] = MODE_DONE;
      st[ST_STATUS] = SLOT_CONVERGED;
      st[ST_NEEDDIR] = 0;
      return;
    }
    sc[SC_GTD] = gtd;
    sc[SC_MAXD] = maxd;
    sc[SC_ALPHA] = st[ST_NH] == 0 ? fmin(1.0, 0.1 * sc[SC_H] / maxd) : 1.0;
    st[ST_MODE] = MODE_TRIAL;
    st[ST_TRIALS] = 0;
  }
}

// trial point vt = v + alpha d (d = -g after a restart)
__global__ __launch_bounds__(kVB) void kb_vtrial(EngineDev E) {
  const int count = E.counts[kCountVec];
  for (int t = blockIdx.x; t < count; t += gridDim.x) {
    const VTile V = vtile(E, t);
    if (!needs_dir(E, V.slot)) continue;
    const SlotDev &S = E.slots[V.slot];
    const double alpha = E.sc[V.slot * kNSc + SC_ALPHA];
    const bool reset = E.st[V.slot * kNSt + ST_RESET] != 0;
    for (int k = 0; k < kVecTile; k += kVB) {
      const int j = V.i0 + k + threadIdx.x;
      if (j < V.n) {
        double dj = S.d[j];
        if (reset) S.d[j] = dj = -S.g[j];
        S.vt[j] = S.v[j] + alpha * dj;
      }
    }
  }
}

// ----------------------------------------------------------------------- launch sequence
constexpr int kGridTile = 1024, kGridHalo = 2048, kGridVec = 2048;

template <typename T>
int eval_launches(const EngineDev &E, hipStream_t s) {
  constexpr int NT = batch_tile_threads<T>();
  hipLaunchKernelGGL((kb_tile<2, 1, P1E_PLAPLACE, T, CLS_PLAP2>), dim3(kGridTile), dim3(NT), 0, s, E);
  hipLaunchKernelGGL((kb_tile<3, 1, P1E_PLAPLACE, T, CLS_PLAP3>), dim3(kGridTile), dim3(NT), 0, s, E);
  hipLaunchKernelGGL((kb_tile<2, 2, P1E_NEOHOOKE, T, CLS_NH2>), dim3(kGridTile), dim3(NT), 0, s, E);
  hipLaunchKernelGGL((kb_tile<3, 3, P1E_NEOHOOKE, T, CLS_NH3>), dim3(kGridTile), dim3(NT), 0, s, E);
  hipLaunchKernelGGL(kb_finalize, dim3(E.max_slots), dim3(kVB), 0, s, E);
  hipLaunchKernelGGL((kb_halo<1, CLS_PLAP2, T>), dim3(kGridHalo), dim3(kBlock), 0, s, E);
  hipLaunchKernelGGL((kb_halo<1, CLS_PLAP3, T>), dim3(kGridHalo), dim3(kBlock), 0, s, E);
  hipLaunchKernelGGL((kb_halo<2, CLS_NH2, T>), dim3(kGridHalo), dim3(kBlock), 0, s, E);
  hipLaunchKernelGGL((kb_halo<3, CLS_NH3, T>), dim3(kGridHalo), dim3(kBlock), 0, s, E);
  return P1E_OK;
}

}  // namespace

int batch_step(const EngineDev &E, hipStream_t s) {
  if (E.prec == P1E_MIXED) eval_launches<float>(E, s);
  else eval_launches<double>(E, s);
  const int sb = (E.max_slots + kVB - 1) / kVB;
  hipLaunchKernelGGL(kb_decide, dim3(sb), dim3(kVB), 0, s, E);
  hipLaunchKernelGGL(kb_vupdate, dim3(kGridVec), dim3(kVB), 0, s, E);
  hipLaunchKernelGGL(kb_hist, dim3(E.max_slots), dim3(kVB), 0, s, E);
  hipLaunchKernelGGL(kb_dots, dim3(kGridVec), dim3(kVB), 0, s, E);
  hipLaunchKernelGGL(kb_compact, dim3(E.max_slots), dim3(kCB), 0, s, E);
  hipLaunchKernelGGL(kb_dir, dim3(kGridVec), dim3(kVB), 0, s, E);
  hipLaunchKernelGGL(kb_dirfin, dim3(E.max_slots), dim3(kVB), 0, s, E);
  hipLaunchKernelGGL(kb_vtrial, dim3(kGridVec), dim3(kVB), 0, s, E);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(P1E_EHIP, std::string("engine step: ") + hipGetErrorString(e));
  return P1E_OK;
}

}  // namespace p1e
