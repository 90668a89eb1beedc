// p1e_device.h -- device-side building blocks shared by the single-mesh kernels
// (p1e_kernels.hip) and the batched multi-request kernels (p1e_batch.hip): compensated sums,
// block reductions, nodal field access, the densities and their stresses (Neo-Hookean,
// p-Laplacian, St. Venant-Kirchhoff), and the bodies of the element-tile pass and of the
// halo-row pass. Not part of the public ABI.
//
// Precision. P1E_FP64 runs everything in double. P1E_MIXED evaluates the element algebra in
// float on the displacement gradient G = F - I, with the cancellation-free forms
//   |F|^2 - dim = 2 tr G + |G|^2,  det F - 1 = tr G + s2(G) + det G  (s2: sum of principal
//   2x2 minors, absent in 2D),  (det F - 1) - log det F  by log_excess (float),
//   F - F^-T = [(s2 + det G) I + (det F) G + G^T - cof G] / det F  (2D: cof terms reduce),
// forms the Neo-Hookean density from these in float, and accumulates the energies in double
// and the patch sums of the element forces in rounds: each lane adds up to four forces of its
// node in float, and the rounds in double.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "p1e_internal.h"

#ifndef P1E_STREAM_NT
#define P1E_STREAM_NT 1
#endif
namespace p1e {
namespace dev {

// Loads of arrays that one pass reads exactly once (connectivity, geometry, patch entries,
// LDS slots).
// With P1E_STREAM_NT (the default) they are marked non-temporal, leaving cache capacity to
// the data that is re-read (nodal values shared by neighbouring tiles, the halo partials
// that the halo kernel reads next).
template <typename T>
__device__ __forceinline__ T stream_load(const T *p) {
#if P1E_STREAM_NT
  return __builtin_nontemporal_load(p);
#else
  return *p;
#endif
}

// Element i of an array through a 32-bit byte offset: the access then takes the array's base
// as a scalar register pair and the offset as one vector register, instead of forming a
// 64-bit address per lane. Every array the tile kernels index this way is below 4 GiB
// (p1e_mesh_create refuses larger meshes).
template <typename T>
__device__ __forceinline__ const T *at32(const T *p, int i) {
  return reinterpret_cast<const T *>(reinterpret_cast<const char *>(p) +
                                     (uint32_t)i * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ T *at32(T *p, int i) {
  return reinterpret_cast<T *>(reinterpret_cast<char *>(p) + (uint32_t)i * (uint32_t)sizeof(T));
}

struct Params {
  double C1, D1, p, eps;
  int ortho;       // p-Laplacian with the component-wise norm of the gradient (uniform per mesh)
  float C1x2, D1x2;  // 2 C1 and 2 D1 rounded to float
};

// 2 C1 and 2 D1 in T. The float stresses take the host's roundings as uniform operands (no
// conversion per element); they equal 2 (float)C1 and 2 (float)D1, the doubling being exact.
template <typename T>
__device__ __forceinline__ T twice_c1(const Params &prm) {
  if constexpr (std::is_same<T, float>::value)
    return prm.C1x2;
  else
    return 2.0 * prm.C1;
}
template <typename T>
__device__ __forceinline__ T twice_d1(const Params &prm) {
  if constexpr (std::is_same<T, float>::value)
    return prm.D1x2;
  else
    return 2.0 * prm.D1;
}

// ----------------------------------------------------------------------- compensated sums
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
  s = a + b;
  double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// (s, c) pairs: value = s + c
__device__ __forceinline__ void pair_add(double &s, double &c, double s2, double c2) {
  double t, e;
  two_sum(s, s2, t, e);
  s = t;
  c = c + c2 + e;
}

// Block-wide deterministic reduction of (s, c) pairs and an integer count; thread 0 gets
// the result. Fixed shuffle and LDS order, so the result does not depend on timing.
template <int NT>
__device__ __forceinline__ void block_reduce(double &s, double &c, int &cnt) {
  __shared__ double sh_s[NT / 64], sh_c[NT / 64];
  __shared__ int sh_n[NT / 64];
  for (int off = 32; off > 0; off >>= 1) {
    double s2 = __shfl_down(s, off, 64);
    double c2 = __shfl_down(c, off, 64);
    pair_add(s, c, s2, c2);
  }
  if (__any(cnt != 0))  // counts are rare (bad elements): wave-uniform test
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_down(cnt, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    sh_s[wave] = s;
    sh_c[wave] = c;
    sh_n[wave] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < NT / 64; ++w) {
      pair_add(s, c, sh_s[w], sh_c[w]);
      cnt += sh_n[w];
    }
  }
}

// a double from another lane by a DPP lane permutation within rows of 16 (CTRL: quad_perm,
// row_half_mirror or row_mirror; every lane has a source)
template <int CTRL>
__device__ __forceinline__ double dpp_double(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_double(double x, int lane) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), lane),
                          __builtin_amdgcn_readlane(__double2loint(x), lane));
}

// Sum of a double over one 64-wide wavefront, the same in every lane: within each row of 16
// lanes a butterfly of DPP permutations (partners 1 and 2 within quads, then the mirrored
// half-row and row: each step adds two equal-sized partial sums), then the four row sums
// combined as (r0 + r1) + (r2 + r3). A plain FP64 tree (at most 6 ulps of the wavefront's sum
// of magnitudes) in a fixed order, without the LDS.
__device__ __forceinline__ double wave_sum(double a) {
  constexpr int kXor1 = 0xb1, kXor2 = 0x4e, kHalfMirror = 0x141, kMirror = 0x140;
  a += dpp_double<kXor1>(a);
  a += dpp_double<kXor2>(a);
  a += dpp_double<kHalfMirror>(a);
  a += dpp_double<kMirror>(a);
  return (lane_double(a, 0) + lane_double(a, 16)) + (lane_double(a, 32) + lane_double(a, 48));
}
__device__ __forceinline__ int wave_count(int n) {
  if (__any(n != 0))  // counts are rare (bad elements): wave-uniform test
    for (int off = 32; off > 0; off >>= 1) n += __shfl_xor(n, off, 64);
  return n;
}

// Compensated (TwoSum) sum of NW per-wavefront values v[0..NW) by the lanes of one wavefront;
// lane 0 gets the (sum, correction) pair.
template <int NW>
__device__ __forceinline__ double2 waves_combine(const double *v) {
  const int lane = threadIdx.x & 63;
  double s = lane < NW ? v[lane] : 0.0, c = 0.0;
#pragma unroll
  for (int off = NW / 2; off > 0; off >>= 1) {
    const double s2 = __shfl_down(s, off, 64), c2 = __shfl_down(c, off, 64);
    pair_add(s, c, s2, c2);
  }
  return make_double2(s, c);
}

// The dispatcher hands consecutive workgroups to the 8 XCDs in turn, and each XCD has its
// own L2. Renumber blocks so that every XCD works on one contiguous range of tiles: tiles
// that share nodes or elements then share an L2. Bijective on [0, nb).
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  constexpr int X = P1E_XCD_COUNT;
  const int q = nb / X, r = nb % X;
  const int x = b % X, k = b / X;
  return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// The tiles of a persistent grid of nb blocks (nb a multiple of the XCD count): block b works
// on every (nb / X)-th tile of the contiguous range of XCD b % X, the same ranges as
// xcd_tile with one block per tile. Returns the first tile (or n) and the step.
__device__ __forceinline__ int xcd_first(int b, int nb, int n, int &end, int &step) {
  constexpr int X = P1E_XCD_COUNT;
  const int q = n / X, r = n % X;
  const int x = b % X, k = b / X;
  const int lo = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
  end = lo + (x < r ? q + 1 : q);
  step = nb / X;
  return lo + k;
}

// explicit fused multiply-add: kernels are built without automatic contraction, so the
// same expression rounds the same way in every kernel that uses it
__device__ __forceinline__ float mad(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double mad(double a, double b, double c) { return fma(a, b, c); }

// ----------------------------------------------------------------------- node field access
template <typename T, int D>
struct NodeVec;
template <>
struct NodeVec<float, 3> {
  static constexpr int NS = 4;
  __device__ static void load(const float *u, int i, float o[3]) {
    float4 q = reinterpret_cast<const float4 *>(u)[i];
    o[0] = q.x, o[1] = q.y, o[2] = q.z;
  }
  __device__ static void store(float *u, int i, const float o[3]) {
    reinterpret_cast<float4 *>(u)[i] = make_float4(o[0], o[1], o[2], 0.f);
  }
};
template <>
struct NodeVec<double, 3> {
  static constexpr int NS = 4;
  __device__ static void load(const double *u, int i, double o[3]) {
    const double2 *q = reinterpret_cast<const double2 *>(u) + 2 * (int64_t)i;
    double2 a = q[0], b = q[1];
    o[0] = a.x, o[1] = a.y, o[2] = b.x;
  }
  __device__ static void store(double *u, int i, const double o[3]) {
    double2 *q = reinterpret_cast<double2 *>(u) + 2 * (int64_t)i;
    q[0] = make_double2(o[0], o[1]);
    q[1] = make_double2(o[2], 0.0);
  }
};
template <>
struct NodeVec<float, 2> {
  static constexpr int NS = 2;
  __device__ static void load(const float *u, int i, float o[2]) {
    float2 q = reinterpret_cast<const float2 *>(u)[i];
    o[0] = q.x, o[1] = q.y;
  }
  __device__ static void store(float *u, int i, const float o[2]) {
    reinterpret_cast<float2 *>(u)[i] = make_float2(o[0], o[1]);
  }
};
template <>
struct NodeVec<double, 2> {
  static constexpr int NS = 2;
  __device__ static void load(const double *u, int i, double o[2]) {
    double2 q = reinterpret_cast<const double2 *>(u)[i];
    o[0] = q.x, o[1] = q.y;
  }
  __device__ static void store(double *u, int i, const double o[2]) {
    reinterpret_cast<double2 *>(u)[i] = make_double2(o[0], o[1]);
  }
};
template <typename T>
struct NodeVec<T, 1> {
  static constexpr int NS = 1;
  __device__ static void load(const T *u, int i, T o[1]) { o[0] = u[i]; }
  __device__ static void store(T *u, int i, const T o[1]) { u[i] = o[0]; }
};

// ----------------------------------------------------------------------- densities
// A double constant handed to the arithmetic as a scalar register: the FMAs then read it as a
// uniform operand instead of materialising it in vector registers (two vector moves each).
__device__ __forceinline__ double scalar_const(double c) {
  double r;
  asm("s_mov_b64 %0, %1" : "=s"(r) : "s"(c));
  return r;
}

// num / den for a normal den of moderate size (no scaling is done): the hardware reciprocal
// refined by two Newton steps, then one residual correction of the quotient (Markstein's
// scheme), within 1 ulp; cheaper than the correctly rounded division.
__device__ __forceinline__ double quotient(double num, double den) {
  double r = __builtin_amdgcn_rcp(den);
  r = fma(r, fma(-den, r, 1.0), r);
  r = fma(r, fma(-den, r, 1.0), r);
  const double q = num * r;
  return fma(r, fma(-den, q, num), q);
}

// q(d) = d - log(1 + d) >= 0 for d > -1, in double, without the cancellation of the plain
// difference near d = 0 (where q ~ d^2 / 2). Binary exponent reduction 1 + d = 2^k m with
// m in [1/sqrt 2, sqrt 2), then log m = 2 atanh s = 2 s + 2 s^3 S(s^2), s = (m - 1)/(m + 1),
// |s| <= 0.1716, S(w) = sum_{i>=0} w^i / (2i + 3); ten terms leave a truncation error below
// 1e-16 of S.
//  k = 0: s = d / (2 + d) from d itself (1 + d is never rounded), and d - 2 s = s d exactly
//         in real arithmetic, so q = s d - 2 s^3 S: both terms positive for d < 0, the second
//         at most a twentieth of the first for d > 0.
//  k != 0: q = d - k log 2 - 2 s - 2 s^3 S - (1 + d - t)/t with t = fl(1 + d); the last term
//         undoes the rounding of t (d - (t - 1) is exact here), q >= 0.06 so no cancellation.
// About 40 double instructions, against over 100 for a general-purpose log1p.
__device__ __forceinline__ double log_excess(double d) {
  const double t = 1.0 + d;
  constexpr double kRt = 0.70710678118654752440;  // 1/sqrt 2 rounded
  int k;
  double m = frexp(t, &k);  // t = m 2^k, m in [1/2, 1)
  const bool lo = m < kRt;
  m = lo ? 2.0 * m : m;
  k = lo ? k - 1 : k;
  const bool k0 = k == 0;
  const double s = quotient(k0 ? d : m - 1.0, k0 ? 2.0 + d : m + 1.0);  // den in [1.7, 2.5]
  const double w = s * s;
  double S = 1.0 / 21.0;  // S(w) = sum w^i / (2i + 3), i = 9 .. 0 by Horner
#pragma unroll
  for (int i = 8; i >= 0; --i) S = fma(S, w, scalar_const(1.0 / (2 * i + 3)));
  const double tail = 2.0 * (s * w) * S;
  const double q0 = fma(s, d, -tail);
  constexpr double kLn2Hi = 6.93147180369123816490e-01;  // high 32 bits of log 2
  constexpr double kLn2Lo = 1.90821492927058770002e-10;  // log 2 - kLn2Hi
  const double kd = (double)k;
  const double corr = (d - (t - 1.0)) * __builtin_amdgcn_rcp(t);
  const double qk = ((((d - kd * kLn2Hi) - kd * kLn2Lo) - 2.0 * s) - tail) - corr;
  return k0 ? q0 : qk;
}

// The same q(d) in float, for the mixed-precision density (whose delta is a sum of float
// invariants): the reduction and the two forms above with float arithmetic, S(w) to w^4
// (truncation below 2e-9 of S), log 2 split into 16 high bits (k log2Hi exact for |k| < 256)
// and the rest; the quotient by the hardware reciprocal, one Newton step and one residual
// correction. Within 3 float ulps of q for |d| <= 1/4 and 12 ulps near the ends of the
// reduction interval (against a long double reference over 2e7 samples of (-1, 1000)).
__device__ __forceinline__ float log_excess(float d) {
  const float t = 1.0f + d;
  int k;
  float m = frexpf(t, &k);  // t = m 2^k, m in [1/2, 1)
  const bool lo = m < 0.70710678f;
  m = lo ? 2.0f * m : m;
  k = lo ? k - 1 : k;
  const bool k0 = k == 0;
  const float num = k0 ? d : m - 1.0f, den = k0 ? 2.0f + d : m + 1.0f;  // den in [1.7, 2.5]
  float r = __builtin_amdgcn_rcpf(den);
  r = fmaf(r, fmaf(-den, r, 1.0f), r);
  float s = num * r;
  s = fmaf(r, fmaf(-den, s, num), s);
  const float w = s * s;
  float S = 1.0f / 11.0f;  // S(w) = sum w^i / (2i + 3), i = 4 .. 0 by Horner
#pragma unroll
  for (int i = 3; i >= 0; --i) S = fmaf(S, w, 1.0f / (2 * i + 3));
  const float tail = 2.0f * (s * w) * S;
  const float q0 = fmaf(s, d, -tail);
  constexpr float kLn2Hi = 0.693145751953125f;  // 45426 / 2^16
  constexpr float kLn2Lo = 1.4286068203e-6f;     // log 2 - kLn2Hi
  const float kd = (float)k;
  const float corr = (d - (t - 1.0f)) * __builtin_amdgcn_rcpf(t);
  const float qk = ((((d - kd * kLn2Hi) - kd * kLn2Lo) - 2.0f * s) - tail) - corr;
  return k0 ? q0 : qk;
}

// log((1 + y) / (1 - y)) = 2 atanh y for |y| < 1: the log of the det F ratio of a difference
// step. For |y| < 1/64 by the odd series 2 (y + y^3/3 + ... + y^9/9) (the omitted terms are
// below 1e-19 of the sum), without division; otherwise as x - log_excess(x) = log1p(x) with
// x = 2y / (1 - y). The caller picks one form for a whole wavefront (a uniform branch).
constexpr double kSeriesBound = 0.015625;
__device__ __forceinline__ double log_ratio_series(double y) {
  const double w = y * y;
  double t = scalar_const(1.0 / 9.0);
#pragma unroll
  for (int i = 7; i >= 3; i -= 2) t = fma(t, w, scalar_const(1.0 / i));
  t = fma(t, w, 1.0);
  return 2.0 * y * t;
}
__device__ __forceinline__ double log_ratio_general(double y) {
  const double x = quotient(2.0 * y, 1.0 - y);
  return x - log_excess(x);
}

// Invariants of G = F - I used by the Neo-Hookean density and stress, in T: tr G, s2 (sum of
// the principal 2x2 minors, 0 in 2D), det G, |G|^2, and (3D) cof G. det F = 1 + tr + s2 + det G.
template <int DIM, typename T>
struct NhInv {
  T tr, s2, dG, n2;
  T cg[DIM][DIM];
};
template <int DIM, typename T>
__device__ __forceinline__ NhInv<DIM, T> nh_invariants(const T G[DIM][DIM]) {
  NhInv<DIM, T> v;
  if constexpr (DIM == 3) {
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        const int j1 = (j + 1) % 3, j2 = (j + 2) % 3, m1 = (m + 1) % 3, m2 = (m + 2) % 3;
        v.cg[j][m] = mad(G[j1][m1], G[j2][m2], -(G[j1][m2] * G[j2][m1]));
      }
    v.tr = G[0][0] + G[1][1] + G[2][2];
    v.s2 = v.cg[0][0] + v.cg[1][1] + v.cg[2][2];
    v.dG = mad(G[0][0], v.cg[0][0], mad(G[0][1], v.cg[0][1], G[0][2] * v.cg[0][2]));
  } else {
    v.tr = G[0][0] + G[1][1];
    v.s2 = T(0);
    v.dG = mad(G[0][0], G[1][1], -(G[0][1] * G[1][0]));
    v.cg[0][0] = G[1][1], v.cg[0][1] = -G[1][0], v.cg[1][0] = -G[0][1], v.cg[1][1] = G[0][0];
  }
  T n2 = T(0);
#pragma unroll
  for (int j = 0; j < DIM; ++j)
#pragma unroll
    for (int m = 0; m < DIM; ++m) n2 = mad(G[j][m], G[j][m], n2);
  v.n2 = n2;
  return v;
}

// Neo-Hookean density from the invariants (eq. neoHook), returned in double:
//   W = C1 (|G|^2 - 2 (s2 + det G) + 2 q) + D1 delta^2,  delta = det F - 1,
//   q = delta - log det F (log_excess), using |F|^2 - dim = 2 tr G + |G|^2.
// In T: for float (mixed precision) as 2W with the uniform 2 C1 and 2 D1, every term of the
// size of the float invariants it is formed from, so their own rounding already sets the
// accuracy.
template <int DIM, typename T>
__device__ __forceinline__ double nh_density(const NhInv<DIM, T> &v, const Params &prm,
                                             bool &bad) {
  const T delta = v.tr + v.s2 + v.dG;
  if (!(delta > T(-1))) {
    bad = true;
    return 0.0;
  }
  const T q = log_excess(delta);
  T W;
  if constexpr (std::is_same<T, float>::value) {
    const float a = fmaf(2.0f, q, v.n2 - 2.0f * (v.s2 + v.dG));
    W = 0.5f * fmaf(prm.D1x2 * delta, delta, prm.C1x2 * a);
  } else {
    W = prm.C1 * (v.n2 - 2.0 * (v.s2 + v.dG) + 2.0 * q) + prm.D1 * delta * delta;
  }
  if (!isfinite(W)) bad = true;
  return (double)W;
}

// Neo-Hookean density at F = I + G (eq. neoHook), returned in double.
template <int DIM, typename T>
__device__ __forceinline__ double nh_energy(const T G[DIM][DIM], const Params &prm, bool &bad) {
  return nh_density<DIM, T>(nh_invariants<DIM, T>(G), prm, bad);
}

// Density and first Piola stress P = dW/dF at F = I + G from one set of invariants:
//   P = 2 C1 (J F - cof F) / J + 2 D1 (J - 1) cof F,  J = det F,
// with (3D) J F - cof F = (s2 + det G) I + J G + G^T - cof G, cof F = (1 + tr G) I - G^T + cof G,
// so that with a = 2 C1 / J (a J = 2 C1), b = 2 D1 (J - 1):
//   P = a J G + (a - b)(G^T - cof G) + (a (s2 + det G) + b (1 + tr G)) I;
// (2D) J F - cof F = det G I + J G + G^T, cof F = I + cof G = (1 + tr G) I - G^T:
//   P = a J G + (a - b) G^T + (a det G + b (1 + tr G)) I.
// P comes out multiplied by vol (the element size, folded into the three coefficients). The
// density is bitwise the one of nh_energy.
template <int DIM, typename T>
__device__ __forceinline__ double nh_energy_stress(const T G[DIM][DIM], const Params &prm,
                                                   T vol, bool &bad, T P[DIM][DIM]) {
  const NhInv<DIM, T> v = nh_invariants<DIM, T>(G);
  const double W = nh_density<DIM, T>(v, prm, bad);
  const T delta = v.tr + v.s2 + v.dG;
  const T J = T(1) + delta;
  const T c1x2 = twice_c1<T>(prm);
  // a = 2 C1 / J (in float by the hardware reciprocal, within 1 ulp); a J = 2 C1 exactly
  T a;
  if constexpr (std::is_same<T, float>::value)
    a = c1x2 * __builtin_amdgcn_rcpf(J);
  else
    a = c1x2 / J;
  const T bcoef = twice_d1<T>(prm) * delta;
  const T alpha = c1x2 * vol, beta = (a - bcoef) * vol;
  const T gamma = mad(a, v.s2 + v.dG, bcoef * (T(1) + v.tr)) * vol;
#pragma unroll
  for (int j = 0; j < DIM; ++j)
#pragma unroll
    for (int m = 0; m < DIM; ++m) {
      const T X = DIM == 3 ? G[m][j] - v.cg[j][m] : G[m][j];
      const T p = mad(alpha, G[j][m], beta * X);
      P[j][m] = j == m ? p + gamma : p;
    }
  return W;
}

// St. Venant-Kirchhoff, the extension Section 2 names after eq. neoHook, in its textbook form
// W = C1 |E|^2 + D1 (tr E)^2 (C1 = mu, D1 = lambda / 2) with the Green-Lagrange strain taken
// from G = F - I without the cancellation of F^T F - I: E = (G + G^T + G^T G) / 2, in T.
template <int DIM, typename T>
__device__ __forceinline__ void svk_strain(const T G[DIM][DIM], T E[DIM][DIM]) {
#pragma unroll
  for (int j = 0; j < DIM; ++j)
#pragma unroll
    for (int m = j; m < DIM; ++m) {
      T acc = G[j][m] + G[m][j];
#pragma unroll
      for (int q = 0; q < DIM; ++q) acc = mad(G[q][j], G[q][m], acc);
      E[j][m] = T(0.5) * acc;
      E[m][j] = E[j][m];
    }
}
// the density from E, in double
template <int DIM, typename T>
__device__ __forceinline__ double svk_density(const T E[DIM][DIM], double C1, double D1,
                                              bool &bad) {
  double tr = 0.0, ee = 0.0;
#pragma unroll
  for (int j = 0; j < DIM; ++j) {
    tr += (double)E[j][j];
#pragma unroll
    for (int m = 0; m < DIM; ++m) ee = fma((double)E[j][m], (double)E[j][m], ee);
  }
  const double W = C1 * ee + D1 * tr * tr;
  if (!isfinite(W)) bad = true;
  return W;
}
template <int DIM, typename T>
__device__ __forceinline__ double svk_energy(const T G[DIM][DIM], double C1, double D1,
                                             bool &bad) {
  T E[DIM][DIM];
  svk_strain<DIM, T>(G, E);
  return svk_density<DIM, T>(E, C1, D1, bad);
}
// the density and vol dW/dF = vol F S with S = dW/dE = 2 C1 E + 2 D1 (tr E) I (second
// Piola-Kirchhoff stress), F = I + G; the density is bitwise the one of svk_energy
template <int DIM, typename T>
__device__ __forceinline__ double svk_energy_stress(const T G[DIM][DIM], const Params &prm,
                                                    T vol, bool &bad, T P[DIM][DIM]) {
  T E[DIM][DIM];
  svk_strain<DIM, T>(G, E);
  const double W = svk_density<DIM, T>(E, prm.C1, prm.D1, bad);
  T tr = T(0);
#pragma unroll
  for (int j = 0; j < DIM; ++j) tr += E[j][j];
  const T a = twice_c1<T>(prm) * vol, b = twice_d1<T>(prm) * vol * tr;
  T Sv[DIM][DIM];  // vol S
#pragma unroll
  for (int j = 0; j < DIM; ++j)
#pragma unroll
    for (int m = 0; m < DIM; ++m) Sv[j][m] = j == m ? mad(a, E[j][m], b) : a * E[j][m];
#pragma unroll
  for (int j = 0; j < DIM; ++j)
#pragma unroll
    for (int m = 0; m < DIM; ++m) {
      T acc = Sv[j][m];
#pragma unroll
      for (int q = 0; q < DIM; ++q) acc = mad(G[j][q], Sv[q][m], acc);
      P[j][m] = acc;
    }
  return W;
}

// s^(p/2) for s >= 0, in double. When 2p is an integer k <= 64 (the benchmarks use p = 1.5,
// 3, 5): s^(k/4) = s^floor(k/4) (s^(1/4))^(k mod 4) by products and square roots only (an
// error of a few ulps); otherwise pow. The branch depends on p alone (uniform per mesh).
__device__ __forceinline__ double half_pow(double s, double p) {
  const double k2 = 2.0 * p;
  const int k = (int)k2;
  if ((double)k == k2 && k >= 0 && k <= 64) {
    double r = 1.0;
    for (int i = 0; i < (k >> 2); ++i) r *= s;
    const int f = k & 3;
    if (f != 0) {
      const double q = sqrt(s);
      if (f == 2) {
        r *= q;
      } else {
        const double q4 = sqrt(q);
        r *= f == 1 ? q4 : q * q4;
      }
    }
    return r;
  }
  return pow(s, 0.5 * p);
}

template <int DIM, typename T>
__device__ __forceinline__ T pl_norm2(const T g[DIM]) {
  T s = T(0);
#pragma unroll
  for (int m = 0; m < DIM; ++m) s += g[m] * g[m];
  return s;
}

// p-Laplacian density |g|^p / p (eq. pLaplacian), in double; with ortho the density with the
// component-wise norm, sum_m |g_m|^p / p (the one whose minima Table 6 prints)
template <int DIM, typename T>
__device__ __forceinline__ double pl_energy(const T g[DIM], double p, bool ortho, bool &bad) {
  double W;
  if (ortho) {
    W = 0.0;
#pragma unroll
    for (int m = 0; m < DIM; ++m) W += half_pow((double)(g[m] * g[m]), p);
    W /= p;
  } else {
    W = half_pow((double)pl_norm2<DIM, T>(g), p) / p;
  }
  if (!isfinite(W)) bad = true;
  return W;
}

// the density and vol times its gradient, vol |g|^(p-2) g (0 at g = 0), from one power |g|^p
// (ortho: vol |g_m|^(p-2) g_m per component); the density is bitwise the one of pl_energy
template <int DIM, typename T>
__device__ __forceinline__ double pl_energy_stress(const T g[DIM], double p, bool ortho, T vol,
                                                   bool &bad, T P[DIM]) {
  double W;
  if (ortho) {
    W = 0.0;
#pragma unroll
    for (int m = 0; m < DIM; ++m) {
      const T s = g[m] * g[m];
      const double sp = half_pow((double)s, p);
      W += sp;
      P[m] = s > T(0) ? (T)(sp / (double)s) * vol * g[m] : T(0);
    }
    W /= p;
  } else {
    const T s = pl_norm2<DIM, T>(g);
    const double sp = half_pow((double)s, p);
    W = sp / p;
    const T sc = s > T(0) ? (T)(sp / (double)s) * vol : T(0);
#pragma unroll
    for (int m = 0; m < DIM; ++m) P[m] = sc * g[m];
  }
  if (!isfinite(W)) bad = true;
  return W;
}

// Ginzburg-Landau, the scalar first-gradient problem Section 7 names: W = C1 |grad u|^2 (here)
// plus the potential D1 int_T (u^2 - 1)^2 dx of the element's P1 field (gl_potential). With
// u = sum_l u_l lambda_l, int_T u^k dx = |T| k! dim! / (k + dim)! h_k(u_0, ..., u_dim) (h_k the
// complete homogeneous symmetric polynomial, from the power sums by Newton's identities), so
//   int_T (u^2 - 1)^2 = |T| (c4 h_4 - 2 c2 h_2 + 1),  c4 = 4! dim!/(4+dim)!, c2 = 2! dim!/(2+dim)!
// and d h_k / d u_l = h_(k-1)(u_0, ..., u_dim, u_l). Evaluated in double in both precisions.
template <int DIM>
struct GlCoef {
  static constexpr double c4 = DIM == 2 ? 1.0 / 15.0 : 1.0 / 35.0;
  static constexpr double c2 = DIM == 2 ? 1.0 / 6.0 : 1.0 / 10.0;
};
struct PowerSums {
  double p1, p2, p3, p4;
};
template <int DIM, typename T>
__device__ __forceinline__ PowerSums gl_power_sums(const T (&uu)[DIM + 1][1]) {
  PowerSums q{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int l = 0; l <= DIM; ++l) {
    const double x = (double)uu[l][0], x2 = x * x;
    q.p1 += x;
    q.p2 += x2;
    q.p3 += x2 * x;
    q.p4 += x2 * x2;
  }
  return q;
}
// h_2 and h_4 from power sums
__device__ __forceinline__ double gl_h2(const PowerSums &q) { return 0.5 * (q.p1 * q.p1 + q.p2); }
__device__ __forceinline__ double gl_h4(const PowerSums &q) {
  const double h1 = q.p1, h2 = gl_h2(q);
  const double h3 = (q.p1 * h2 + q.p2 * h1 + q.p3) / 3.0;
  return 0.25 * (q.p1 * h3 + q.p2 * h2 + q.p3 * h1 + q.p4);
}
// D1 int_T (u^2 - 1)^2 dx
template <int DIM>
__device__ __forceinline__ double gl_potential(const PowerSums &q, double vol, double D1) {
  return D1 * vol * (GlCoef<DIM>::c4 * gl_h4(q) - 2.0 * GlCoef<DIM>::c2 * gl_h2(q) + 1.0);
}
// its first and third derivatives in u_l (the potential is a quartic in u_l)
template <int DIM>
__device__ __forceinline__ double gl_potential_d1(const PowerSums &q, double x, double vol,
                                                  double D1) {
  const double x2 = x * x;
  const double r1 = q.p1 + x, r2 = q.p2 + x2, r3 = q.p3 + x2 * x;  // power sums with u_l twice
  const double h3 = (r1 * r1 * r1 + 3.0 * r1 * r2 + 2.0 * r3) / 6.0;
  return D1 * vol * (GlCoef<DIM>::c4 * h3 - 2.0 * GlCoef<DIM>::c2 * r1);
}
template <int DIM>
__device__ __forceinline__ double gl_potential_d3(const PowerSums &q, double x, double vol,
                                                  double D1) {
  return D1 * vol * GlCoef<DIM>::c4 * (18.0 * x + 6.0 * q.p1);
}

// density dispatch on a D x DIM gradient
template <int DIM, int D, int KIND, typename T>
__device__ __forceinline__ double density(const T G[D][DIM], const Params &prm, bool &bad) {
  if constexpr (KIND == P1E_NEOHOOKE) {
    return nh_energy<DIM, T>(G, prm, bad);
  } else if constexpr (KIND == P1E_SVK) {
    return svk_energy<DIM, T>(G, prm.C1, prm.D1, bad);
  } else if constexpr (KIND == P1E_GINZBURG_LANDAU) {  // the gradient part only
    const double W = prm.C1 * (double)pl_norm2<DIM, T>(G[0]);
    if (!isfinite(W)) bad = true;
    return W;
  } else {
    return pl_energy<DIM, T>(G[0], prm.p, prm.ortho != 0, bad);
  }
}


// MODE_FD: second-order central differences on +-eps; MODE_FD4: the fourth-order scheme on
// +-eps and +-2 eps, [8 (S(eps) - S(-eps)) - (S(2eps) - S(-2eps))] / (12 eps)
enum { MODE_ENERGY = 0, MODE_FORCE = 1, MODE_FD = 2, MODE_FD4 = 3 };
constexpr bool is_fd(int mode) { return mode == MODE_FD || mode == MODE_FD4; }

// one force-record entry: D words of T, loaded and stored as a single vector access
template <typename T, int D>
struct Entry {
  T v[D];
};

template <typename T, int D, int K>
__device__ __forceinline__ void store_entries(T *__restrict__ r, int nep, int e, const T *out) {
#pragma unroll
  for (int l = 0; l < K; ++l) {
    Entry<T, D> q;
#pragma unroll
    for (int j = 0; j < D; ++j) q.v[j] = out[l * D + j];
    *reinterpret_cast<Entry<T, D> *>(r + ((int64_t)l * nep + e) * D) = q;
  }
}

// Element geometry from its vertices (Section 4.1): the edge matrix
// B = [x_1 - x_0, ..., x_dim - x_0] (columns) from the vertex offsets xx[l][m] (offsets from a
// common origin), B^-1 by its adjugate (row l of B^-1 is grad phi_(l+1)) and |T| = |det B| / dim!.
template <int DIM, typename T>
__device__ __forceinline__ void simplex_geometry(const T (&xx)[DIM + 1][DIM], T Bi[DIM][DIM],
                                                 T &vol) {
  T B[DIM][DIM];
#pragma unroll
  for (int m = 0; m < DIM; ++m)
#pragma unroll
    for (int l = 0; l < DIM; ++l) B[m][l] = xx[l + 1][m] - xx[0][m];
  T det;
  if constexpr (DIM == 3) {
    T cof[3][3];  // cof[m][l]: the cofactor of B[m][l]
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        const int m1 = (m + 1) % 3, m2 = (m + 2) % 3, l1 = (l + 1) % 3, l2 = (l + 2) % 3;
        cof[m][l] = mad(B[m1][l1], B[m2][l2], -(B[m1][l2] * B[m2][l1]));
      }
    det = mad(B[0][0], cof[0][0], mad(B[0][1], cof[0][1], B[0][2] * cof[0][2]));
    T r;
    if constexpr (std::is_same<T, float>::value)
      r = __builtin_amdgcn_rcpf(det);
    else
      r = T(1) / det;
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
      for (int m = 0; m < 3; ++m) Bi[l][m] = cof[m][l] * r;
    vol = fabs(det) * T(1.0 / 6.0);
  } else {
    det = mad(B[0][0], B[1][1], -(B[0][1] * B[1][0]));
    T r;
    if constexpr (std::is_same<T, float>::value)
      r = __builtin_amdgcn_rcpf(det);
    else
      r = T(1) / det;
    Bi[0][0] = B[1][1] * r;
    Bi[0][1] = -B[0][1] * r;
    Bi[1][0] = -B[1][0] * r;
    Bi[1][1] = B[0][0] * r;
    vol = fabs(det) * T(0.5);
  }
}

// The element pass for element e < ne, given u at its vertices (uu): G = grad u (eq. Dv),
// the density (energy of the element added to (s, c), bad elements counted in cnt) and, by
// MODE, the element forces |T| dW/dF grad phi_l (Section 6.2) or the per-element central
// differences of |T| W under a perturbation of one row of F (Section 6.1), written as
// vertex-major entries r[(l nep + er) D + j].
// Geometry by GEO: (GEO_STORED) geo holds [DIM*DIM][ne] entries of B^-1 followed by [ne]
// sizes |T|; (GEO_CLASS) geo is a table of records [DIM*DIM entries of B^-1, |T|] and cls the
// element's class; (GEO_OTF) xx holds the vertices' coordinate offsets (simplex_geometry).
// FIRST: (s, c) holds nothing yet, so the element's energy is assigned instead of added
template <int DIM, int D, int KIND, typename T, int MODE, int GEO, bool FIRST = false>
__device__ __forceinline__ void element_pass(int e, int ne, const T (&uu)[DIM + 1][D],
                                             const T *__restrict__ geo, int cls,
                                             const T (&xx)[DIM + 1][DIM],
                                             T *__restrict__ r, int nep, int er,
                                             const Params &prm, double &s, double &c,
                                             int &cnt) {
  constexpr int K = DIM + 1;
  T Bi[DIM][DIM];
  T vol;
  if constexpr (GEO == GEO_OTF) {
    simplex_geometry<DIM, T>(xx, Bi, vol);
  } else if constexpr (GEO == GEO_CLASS) {
    const T *rec = geo + cls * (DIM * DIM + 1);
#pragma unroll
    for (int l = 0; l < DIM; ++l)
#pragma unroll
      for (int m = 0; m < DIM; ++m) Bi[l][m] = rec[l * DIM + m];
    vol = rec[DIM * DIM];
  } else {
#pragma unroll
    for (int l = 0; l < DIM; ++l)
#pragma unroll
      for (int m = 0; m < DIM; ++m) Bi[l][m] = stream_load(geo + (int64_t)(l * DIM + m) * ne + e);
    vol = stream_load(geo + (int64_t)(DIM * DIM) * ne + e);
  }
  // G = D Binv with D[j][l] = u_{l+1}[j] - u_0[j]   (eq. Dv, grad phi_0 = -sum of others)
  T G[D][DIM];
#pragma unroll
  for (int j = 0; j < D; ++j)
#pragma unroll
    for (int m = 0; m < DIM; ++m) {
      T acc = T(0);
#pragma unroll
      for (int l = 0; l < DIM; ++l) acc = mad(uu[l + 1][j] - uu[0][j], Bi[l][m], acc);
      G[j][m] = acc;
    }
  bool bad = false;
  double W;
  T P[D][DIM];
  NhInv<DIM, T> nv;  // (Neo-Hookean patch differences) the invariants, kept for the steps
  if constexpr (MODE == MODE_FORCE && KIND == P1E_NEOHOOKE) {
    W = nh_energy_stress<DIM, T>(G, prm, vol, bad, P);  // P = |T| dW/dF
  } else if constexpr (MODE == MODE_FORCE && KIND == P1E_SVK) {
    W = svk_energy_stress<DIM, T>(G, prm, vol, bad, P);
  } else if constexpr (MODE == MODE_FORCE && KIND == P1E_GINZBURG_LANDAU) {
    W = density<DIM, D, KIND, T>(G, prm, bad);
    const T a = twice_c1<T>(prm) * vol;  // vol dW/dgrad u = 2 C1 vol grad u
#pragma unroll
    for (int m = 0; m < DIM; ++m) P[0][m] = a * G[0][m];
  } else if constexpr (MODE == MODE_FORCE) {
    W = pl_energy_stress<DIM, T>(G[0], prm.p, prm.ortho != 0, vol, bad, P[0]);
  } else if constexpr (is_fd(MODE) && KIND == P1E_NEOHOOKE) {
    nv = nh_invariants<DIM, T>(G);
    W = nh_density<DIM, T>(nv, prm, bad);
  } else {
    W = density<DIM, D, KIND, T>(G, prm, bad);
  }
  if constexpr (MODE == MODE_FORCE) {
    T out[K * D];
#pragma unroll
    for (int j = 0; j < D; ++j) out[j] = T(0);
#pragma unroll
    for (int l = 1; l < K; ++l)
#pragma unroll
      for (int j = 0; j < D; ++j) {
        T acc = T(0);
#pragma unroll
        for (int m = 0; m < DIM; ++m) acc = mad(P[j][m], Bi[l - 1][m], acc);
        out[l * D + j] = acc;
        out[j] -= acc;
      }
    if constexpr (KIND == P1E_GINZBURG_LANDAU) {  // + d/du_l of the potential
      const PowerSums q = gl_power_sums<DIM, T>(uu);
#pragma unroll
      for (int l = 0; l < K; ++l)
        out[l] += (T)gl_potential_d1<DIM>(q, (double)uu[l][0], (double)vol, prm.D1);
    }
    store_entries<T, D, K>(r, nep, er, out);
  }
  if constexpr (is_fd(MODE)) {
    // Central differences of |T| W under v_n +- h for every DOF n of this element: only
    // row j of F changes, by +-h grad phi_l (Section 6.1). Differenced per element (h = eps,
    // and in the fourth-order scheme also 2 eps); the patch sums happen in the tile's node
    // phase and the halo rows.
    const double eps = prm.eps;
    // the scheme's combination of the differences W(+h) - W(-h) at h = eps and 2 eps
    const double inv2e = 1.0 / (2.0 * eps), inv12e = 1.0 / (12.0 * eps);
    auto scheme = [=](double d1, double d2) {
      return MODE == MODE_FD ? d1 * inv2e : (8.0 * d1 - d2) * inv12e;
    };
    T out[K * D];
    // (Neo-Hookean) det F - 1, 1 / det F and cof F = (1 + tr G) I - G^T (+ cof G in 3D),
    // dDet F / dF
    double delta = 0.0, rdet = 0.0;
    T cf[DIM][DIM];
    if constexpr (KIND == P1E_NEOHOOKE) {
      delta = (double)nv.tr + (double)nv.s2 + (double)nv.dG;
      rdet = 1.0 + delta > 0.0 ? quotient(1.0, 1.0 + delta) : -1.0;
#pragma unroll
      for (int j = 0; j < DIM; ++j)
#pragma unroll
        for (int m = 0; m < DIM; ++m) {
          const T t = (j == m ? T(1) + nv.tr : T(0)) - G[m][j];
          cf[j][m] = DIM == 3 ? t + nv.cg[j][m] : t;
        }
    }
    // (Neo-Hookean) y = c eps / det F, and the log-free part of the result, 2 |T| C1 F_j . a
    // + 2 |T| D1 (det F - 1) c, for every DOF of the element
    const double ky = eps * rdet, ka = 2.0 * (double)vol * prm.C1,
                 kc = 2.0 * (double)vol * prm.D1 * delta;
    double yv[KIND == P1E_NEOHOOKE ? K * D : 1], av[KIND == P1E_NEOHOOKE ? K * D : 1];
#pragma unroll
    for (int l = 0; l < K; ++l) {
      T a[DIM];
#pragma unroll
      for (int m = 0; m < DIM; ++m) {
        if (l == 0) {
          T t = T(0);
#pragma unroll
          for (int q = 0; q < DIM; ++q) t -= Bi[q][m];
          a[m] = t;
        } else {
          a[m] = Bi[l - 1][m];
        }
      }
      if constexpr (KIND == P1E_NEOHOOKE) {
        // F -> F +- h e_j a^T changes det F by +- h c with c = (cof F)_j . a (det F is
        // linear in each row) and |F|^2 by +- 2 h F_j . a + h^2 |a|^2, so
        //   W+ - W- = C1 (4 h F_j . a - 2 log(det F+ / det F-)) + 4 D1 h c (det F - 1),
        // with det F+ / det F- = (1 + y) / (1 - y), y = h c / det F: the same difference
        // as two density evaluations, without their cancellation, with one logarithm instead
        // of two and one division per element. Here y at h = eps and the log-free part of
        // the scheme's result, |T| (4 eps C1 F_j . a + 4 eps D1 c (det F - 1)) / (2 eps); the
        // logarithms follow for all the element's DOFs at once.
#pragma unroll
        for (int j = 0; j < D; ++j) {
          double c = 0.0, fa = (double)a[j];
#pragma unroll
          for (int m = 0; m < DIM; ++m) {
            c = fma((double)cf[j][m], (double)a[m], c);
            fa = fma((double)G[j][m], (double)a[m], fa);
          }
          yv[l * D + j] = c * ky;
          av[l * D + j] = fma(ka, fa, kc * c);
        }
        continue;
      }
      if constexpr (KIND == P1E_GINZBURG_LANDAU) {
        // |T| W(+h) - |T| W(-h) from the structure of the step: the gradient part changes by
        // C1 |T| (|g + h a|^2 - |g - h a|^2) = 4 h C1 |T| g.a, and the potential, a quartic in
        // u_l, by 2 h P' + h^3 P''' / 3 (its odd Taylor terms), both exact
        const PowerSums q = gl_power_sums<DIM, T>(uu);
        const double x = (double)uu[l][0], vd = (double)vol;
        double ga = 0.0;
#pragma unroll
        for (int m = 0; m < DIM; ++m) ga = fma((double)G[0][m], (double)a[m], ga);
        const double p1 = gl_potential_d1<DIM>(q, x, vd, prm.D1);
        const double p3 = gl_potential_d3<DIM>(q, x, vd, prm.D1);
        auto dE = [&](double h) {
          return 4.0 * h * prm.C1 * vd * ga + 2.0 * h * p1 + h * h * h * p3 / 3.0;
        };
        const double d = scheme(dE(eps), MODE == MODE_FD4 ? dE(2.0 * eps) : 0.0);
        if (!isfinite(d)) bad = true;
        out[l] = (T)d;
        continue;
      }
#pragma unroll
      for (int j = 0; j < D; ++j) {
        auto dW = [&](double h) {  // W(+h) - W(-h): two density evaluations
          T Gp[D][DIM], Gm[D][DIM];
#pragma unroll
          for (int jj = 0; jj < D; ++jj)
#pragma unroll
            for (int m = 0; m < DIM; ++m) {
              Gp[jj][m] = G[jj][m];
              Gm[jj][m] = G[jj][m];
            }
#pragma unroll
          for (int m = 0; m < DIM; ++m) {
            Gp[j][m] = mad((T)h, a[m], G[j][m]);
            Gm[j][m] = mad(-(T)h, a[m], G[j][m]);
          }
          return density<DIM, D, KIND, T>(Gp, prm, bad) - density<DIM, D, KIND, T>(Gm, prm, bad);
        };
        const double d1 = dW(eps), d2 = MODE == MODE_FD4 ? dW(2.0 * eps) : 0.0;
        out[l * D + j] = (T)((double)vol * scheme(d1, d2));
      }
    }
    if constexpr (KIND == P1E_NEOHOOKE) {
      // |T| (W+ - W-) = |T| (A - 2 C1 L(y)) at h = eps (A the log-free part, L(y) =
      // log((1 + y) / (1 - y))) and |T| (2A - 2 C1 L(2y)) at h = 2 eps, so the second-order
      // result is av - (|T| C1 / eps) L(y) and the fourth-order one
      // av - (|T| C1 / (6 eps)) (8 L(y) - L(2y)). Both det F+ and det F- must be positive
      // (|y| < 1 at the largest step). One uniform choice of the logarithm's form for every
      // DOF of the wavefront's elements.
      constexpr double ymax = MODE == MODE_FD4 ? 0.5 : 1.0;
      bool small = true;
#pragma unroll
      for (int n = 0; n < K * D; ++n) {
        const bool ok = rdet > 0.0 && fabs(yv[n]) < ymax;
        if (!ok) {
          bad = true;
          yv[n] = 0.0;
        }
        small = small && fabs(yv[n]) < ymax * kSeriesBound;
      }
      const double kl = (double)vol * prm.C1 / (MODE == MODE_FD4 ? 6.0 * eps : eps);
      auto finish = [&](auto lratio) {
#pragma unroll
        for (int n = 0; n < K * D; ++n) {
          const double lg = MODE == MODE_FD4 ? fma(8.0, lratio(yv[n]), -lratio(2.0 * yv[n]))
                                             : lratio(yv[n]);
          const double q = fma(-kl, lg, av[n]);
          if (!isfinite(q)) bad = true;
          out[n] = (T)q;
        }
      };
      if (__all(small))
        finish([](double y) { return log_ratio_series(y); });
      else
        finish([](double y) { return log_ratio_general(y); });
    }
    store_entries<T, D, K>(r, nep, er, out);
  }
  double Ee = (double)vol * W;  // the element's energy |T| W
  if constexpr (KIND == P1E_GINZBURG_LANDAU) {
    Ee += gl_potential<DIM>(gl_power_sums<DIM, T>(uu), (double)vol, prm.D1);
    if (!isfinite(Ee)) bad = true;
  }
  if (bad) {
    cnt += 1;
  } else if (FIRST) {
    s = Ee;
  } else {
    double t, err;
    two_sum(s, Ee, t, err);
    s = t;
    c += err;
  }
}

// LDS of one element tile: the element results (vertex-major, [dim+1][kTileElems][D]; first,
// so that a patch entry's byte offset is its LDS address), the staged nodal values, the
// tile's local patch entries and the geometry class table.
// 16-byte aligned: nodal values and patch entries move as 16-byte vectors.
// GSET: the geometry modes (bits 1 << GEO) the workgroup may meet. With GEO_OTF tiles (at
// most kTileNodes / 2 nodes) the first half of us holds the nodal values and the second half
// (xs) the nodes' coordinate offsets, so us has slots of max(NS, NSX) scalars.
template <int DIM, int D, typename T, int MODE, int GSET>
struct alignas(16) TileShared {
  static constexpr int K = DIM + 1, NS = NodeVec<T, D>::NS, REC = DIM * DIM + 1;
  static constexpr int NSX = NodeVec<T, DIM>::NS;
  static constexpr bool CLS = (GSET >> GEO_CLASS) & 1, OTF = (GSET >> GEO_OTF) & 1;
  static constexpr int NSU = OTF && NSX > NS ? NSX : NS;
  static constexpr int NENT = (K * kTileElems + kEntAlign - 1) / kEntAlign * kEntAlign;
  T fs[MODE == MODE_ENERGY ? 4 : K * kTileElems * D + 4];  // + a zero record at the end
  T us[kTileNodes * NSU];
  uint16_t lent[MODE == MODE_ENERGY ? kEntAlign : NENT + kEntAlign];  // + slack read past rows
  T tab[CLS ? kMaxGeoClasses * REC : 4];
  double red[2 * 16];  // per-wavefront shares: energy, then b.v
  int nbad[16];
  __device__ T *xs() { return us + (kTileNodes / 2) * NSU; }
};

// byte offset of a patch entry's element result: entries hold the offset for FP32 results
template <typename T>
__device__ __forceinline__ int ent_bytes(int raw) {
  return sizeof(T) == 4 ? raw : 2 * raw;
}

// Patch sums of a tile's free nodes (Section 4.2 patch restricted to the tile), GL lanes per
// node: the lanes of a node take every GL-th entry of its local patch row (ascending element,
// rounds of 4 whose LDS reads are issued together; absent slots read a zero record) and
// combine their sums, so every lane holds the same value. A node whose whole patch lies in
// the tile writes g = scale * (sum - b) in free-DOF order; the others write the sum to their
// halo slot. The record of a lane's first node comes from the caller (loaded before the
// element pass, so its latency is hidden); b is loaded before the LDS sums.
template <class SH>
struct DIM_OF_SH {
  static constexpr int K = SH::K;
};
template <int D, typename T, int NT, int GL, class SH>
__device__ __forceinline__ void tile_patch_sums(const TileMesh &M, int r0, int nloc,
                                                const double *__restrict__ scale,
                                                double *__restrict__ g, SH &sh, int4 rec0,
                                                const double (&b0)[D], int tid) {
  static_assert(3 * GL <= kEntAlign, "reads past a row stay within the entry slack");
  const int sub = tid % GL;
  for (int a = tid / GL; a < nloc; a += NT / GL) {
    const bool first = a < NT / GL;
    const int4 rec = first ? rec0 : *at32(M.trec, r0 + a);  // rec0, b0: loaded by the caller
    if (rec.w == 0) continue;  // no free DOF (uniform over the node's lanes)
    const int mask = rec.y & 7, fb = rec.y >> 3;
    const bool complete = rec.z & 1;
    double bj[D];  // b of a complete node's free DOFs, loaded ahead of the sums
    if (first) {
#pragma unroll
      for (int j = 0; j < D; ++j) bj[j] = b0[j];
    } else {
#pragma unroll
      for (int j = 0; j < D; ++j) {
        bj[j] = 0.0;
        if (complete && sub == 0 && ((mask >> j) & 1))
          bj[j] = *at32(M.bhat, fb + __popc(mask & ((1 << j) - 1)));
      }
    }
    double acc[D];
#pragma unroll
    for (int j = 0; j < D; ++j) acc[j] = 0.0;
    const int p0 = rec.w & 0xffff, n = rec.w >> 16;
    // entries are byte offsets into an FP32 fs (offset 0 of the LDS); FP64 results are twice
    // as far
    const char *fsb = reinterpret_cast<const char *>(sh.fs);
    const uint16_t *le = sh.lent + p0;
    constexpr int kZeroB = (DIM_OF_SH<SH>::K) * kTileElems * D * (int)sizeof(T);  // zero record
    for (int p = sub; p < n; p += 4 * GL) {
      int xb[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {  // read unconditionally (at most 3 GL past the row's end)
        const int raw = le[p + u * GL];
        xb[u] = p + u * GL < n ? ent_bytes<T>(raw) : kZeroB;
      }
      T q[4][D];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int j = 0; j < D; ++j)
          q[u][j] = *reinterpret_cast<const T *>(fsb + xb[u] + j * (int)sizeof(T));
      if constexpr (std::is_same<T, float>::value) {
        // (mixed) the round's four forces summed in float, the rounds in double
#pragma unroll
        for (int j = 0; j < D; ++j) acc[j] += (double)((q[0][j] + q[1][j]) + (q[2][j] + q[3][j]));
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int j = 0; j < D; ++j) acc[j] += (double)q[u][j];
      }
    }
    static_assert(GL == 1 || GL == 2, "one or two lanes per node");
    if constexpr (GL == 2) {  // the node's two lanes are neighbours: a DPP swap within quads
#pragma unroll
      for (int j = 0; j < D; ++j) acc[j] += dpp_double<0xb1>(acc[j]);
    }
    if (sub != 0) continue;
    if (complete) {
      const double sc = scale ? *scale : 1.0;
      int f = fb;
#pragma unroll
      for (int j = 0; j < D; ++j)
        if ((mask >> j) & 1) {
          *at32(g, f) = sc * (acc[j] - bj[j]);
          ++f;
        }
    } else {  // halo partials in the tile's element type (FP32 in mixed precision)
      T *hp = at32(reinterpret_cast<T *>(M.hpart), (rec.z >> 2) * D);
#pragma unroll
      for (int j = 0; j < D; ++j) hp[j] = (T)acc[j];
    }
  }
}

#ifndef P1E_LDS_ENERGY_SUM
#define P1E_LDS_ENERGY_SUM 1
#endif
// One element tile t of mesh M, by one workgroup of NT threads (kTileElems / NT elements and
// kTileNodes / NT node records per thread):
//  0. issue the loads that depend on nothing else: the local connectivity (and classes) of
//     the thread's elements, its node records, and the tile's local patch entries (into LDS);
//  1. stage the nodal field u (u = v - x for Neo-Hookean, u = v for the p-Laplacian) of the
//     tile's nodes in LDS (GEO_OTF: and their coordinate offsets); the tile that meets a node
//     first adds b.v of its free DOFs; in the same round trip, b of the lane's first
//     patch-sum node when that node's row is complete in the tile;
//  2. element pass of the tile's elements, vertex values read from LDS, element results
//     written to LDS; energies into (s, c);
//  3. patch sums of the tile's free nodes from LDS (tile_patch_sums);
//  4. block sums: b.v by per-wavefront plain sums taken right after staging, the energy by
//     wavefront 0 over the threads' values left in LDS (or per wavefront where they do not
//     fit), then compensated sums of the shares: energy -> part[t], b.v -> part[ntiles + t],
//     bad count.
// Every order is fixed: the results do not depend on timing. No atomics.
// geo: by GEO, the per-element geometry arrays, the class table (staged in sh.tab) or the
// tile nodes' coordinate offsets (staged in sh.xs()).
// What a tile's pass reads first: its bounds, its node records and each lane's first
// patch-sum record (the nodal loads depend on them). A persistent caller loads the next
// tile's head while the current tile sums its patches, so that a tile starts with one memory
// round trip instead of two.
template <int NPT>
struct TileHead {
  int t;
  int4 ta, tb;  // ttile[t], ttile[t + 1]
  int4 rec[NPT];
  int slot[NPT];  // LDS slot of the node's nodal value (tslot)
  int4 prec;      // (gradient modes) the record of the lane's first patch-sum node
};

// The lane's first node of the patch-sum phase: node tid / 2 (two lanes per node) when the
// tile has at most NT / 2 nodes, else node tid.
template <int NT>
__device__ __forceinline__ int patch_node(int tid, int nloc) {
  return nloc <= NT / 2 ? tid / 2 : tid;
}

// records past the tile's nodes are zero
template <int NPT, int NT, bool PATCH>
__device__ __forceinline__ void tile_head(const TileMesh &M, int t, TileHead<NPT> &h, int tid) {
  h.t = t;
  h.ta = M.ttile[t];
  h.tb = M.ttile[t + 1];
  const int r0 = h.ta.y, nloc = h.tb.y - h.ta.y;
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int a = k * NT + tid;
    h.rec[k] = a < nloc ? *at32(M.trec, r0 + a) : make_int4(0, 0, 0, 0);
    h.slot[k] = a < nloc ? (int)stream_load(at32(M.tslot, r0 + a)) : 0;  // read once
  }
  h.prec = make_int4(0, 0, 0, 0);
  if constexpr (PATCH) {
    const int a = patch_node<NT>(tid, nloc);
    if (a < nloc) h.prec = *at32(M.trec, r0 + a);
  }
}

template <int DIM, int NT>
struct TileSplit {
  static constexpr int K = DIM + 1, EPT = kTileElems / NT, NPT = kTileNodes / NT;
  static_assert(EPT * NT == kTileElems && NPT * NT == kTileNodes, "tile split");
  using Head = TileHead<NPT>;
};

template <int DIM, int D, int KIND, typename T, int MODE, int GEO, int NT, class SH>
__device__ __forceinline__ void tile_pass(const TileMesh &M,
                                          const typename TileSplit<DIM, NT>::Head &h,
                                          const T *__restrict__ geo,
                                          const double *__restrict__ vhat,
                                          double *__restrict__ g,
                                          const double *__restrict__ scale, const Params &prm,
                                          SH &sh, int tid, int tnext = -1,
                                          typename TileSplit<DIM, NT>::Head *next = nullptr) {
  constexpr int K = DIM + 1, REC = DIM * DIM + 1;
  constexpr int EPT = TileSplit<DIM, NT>::EPT, NPT = TileSplit<DIM, NT>::NPT;
  const int t = h.t;
  const int4 ta = h.ta, tb = h.tb;
  const int e0 = ta.x, net = tb.x - ta.x, r0 = ta.y, nloc = tb.y - ta.y;
  const auto &rec = h.rec;
  // 0. independent loads: the elements' local connectivity and classes (lanes past the tile's
  // end read its last element), the patch entries and the class table (to registers here,
  // to LDS once the nodal loads are in flight; the node records are the head's).
  int nd[EPT][K], cl[EPT];
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int e = e0 + min(k * NT + tid, net - 1);
#pragma unroll
    for (int l = 0; l < K; ++l) nd[k][l] = stream_load(at32(M.conn_loc + (int64_t)l * M.ne, e));
    cl[k] = GEO == GEO_CLASS ? (int)stream_load(at32(M.geo_cls, e)) : 0;
  }
  constexpr int LQ = (K * kTileElems / kEntAlign + NT - 1) / NT;  // 16-byte entry groups
  constexpr int TQ = (kMaxGeoClasses * REC + NT - 1) / NT;
  const int nlq = (tb.z - ta.z) / kEntAlign, ntq = GEO == GEO_CLASS ? M.nclass * REC : 0;
  uint4 lq[LQ];
  T tq[TQ];
  if constexpr (MODE != MODE_ENERGY) {
    const uint4 *src = reinterpret_cast<const uint4 *>(M.tlent + ta.z);
#pragma unroll
    for (int i = 0; i < LQ; ++i)
      if (i * NT + tid < nlq) lq[i] = src[i * NT + tid];
  }
  if constexpr (GEO == GEO_CLASS) {
#pragma unroll
    for (int i = 0; i < TQ; ++i)
      if (i * NT + tid < ntq) tq[i] = geo[i * NT + tid];
  }
  // 1. nodal field of the tile; b.v of the nodes this tile owns (only the owner reads b).
  // Per node all loads first (one memory round trip), then the arithmetic; component j's DOF
  // is the node's first free DOF plus the free components before j. In the same round trip,
  // b of the lane's first patch-sum node when the lane writes that node's complete row.
  double sb = 0.0, cb = 0.0;
  double pb[D];
#pragma unroll
  for (int j = 0; j < D; ++j) pb[j] = 0.0;
  if constexpr (MODE != MODE_ENERGY) {
    const int4 pr = h.prec;
    const int mask = pr.y & 7, fb = pr.y >> 3;
    if ((pr.z & 1) && (nloc > NT / 2 || (tid & 1) == 0))
#pragma unroll
      for (int j = 0; j < D; ++j)
        if ((mask >> j) & 1) pb[j] = *at32(M.bhat, fb + __popc(mask & ((1 << j) - 1)));
  }
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int a = k * NT + tid;
    const int mask = rec[k].y & 7;
    const bool own = (rec[k].z >> 1) & 1;
    double w[D], vj[D], bj[D];
    T xo[DIM];  // (GEO_OTF) the node's coordinate offset, read once
#pragma unroll
    for (int j = 0; j < D; ++j) w[j] = 0.0, vj[j] = 0.0, bj[j] = 0.0;
    if (a < nloc) {
      const int gi = rec[k].x, fb = rec[k].y >> 3;
      if constexpr (GEO == GEO_OTF) {
#pragma unroll
        for (int j = 0; j < DIM; ++j) xo[j] = stream_load(at32(geo, (r0 + a) * DIM + j));
      }
#pragma unroll
      for (int j = 0; j < D; ++j) w[j] = *at32(M.wref, gi * D + j);
#pragma unroll
      for (int j = 0; j < D; ++j)
        if ((mask >> j) & 1) {
          const int f = fb + __popc(mask & ((1 << j) - 1));
          vj[j] = *at32(vhat, f);
          if (own) bj[j] = *at32(M.bhat, f);
        }
    }
    if (k == 0) {  // registers -> LDS while the nodal loads are in flight
      if constexpr (MODE != MODE_ENERGY) {
        uint4 *dst = reinterpret_cast<uint4 *>(sh.lent);
#pragma unroll
        for (int i = 0; i < LQ; ++i)
          if (i * NT + tid < nlq) dst[i * NT + tid] = lq[i];
        if (tid < D) sh.fs[K * kTileElems * D + tid] = T(0);
      }
      if constexpr (GEO == GEO_CLASS) {
#pragma unroll
        for (int i = 0; i < TQ; ++i)
          if (i * NT + tid < ntq) sh.tab[i * NT + tid] = tq[i];
      }
    }
    if (a < nloc) {
      T o[D];
      double bvn = 0.0;  // b.v of this node's free DOFs
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const bool fr = (mask >> j) & 1;
        o[j] = (T)(fr ? vj[j] - w[j] : w[j]);
        if (fr) bvn = fma(bj[j], vj[j], bvn);
      }
      NodeVec<T, D>::store(sh.us, h.slot[k], o);
      if constexpr (GEO == GEO_OTF) NodeVec<T, DIM>::store(sh.xs(), h.slot[k], xo);
      if (own) {
        if (NPT == 1) {
          sb = bvn;
        } else {
          double t2, err;
          two_sum(sb, bvn, t2, err);
          sb = t2;
          cb += err;
        }
      }
    }
  }
  constexpr int NW = NT / 64;
  static_assert(NW <= 16, "per-wavefront shares in LDS");
  const int lane = tid & 63, wave = tid >> 6;
  {
    // this wavefront's share of b.v (none in wavefronts past the tile's nodes: uniform test)
    const double wb = (NPT > 1 || wave * 64 < nloc) ? wave_sum(sb + cb) : 0.0;
    if (lane == 0) sh.red[NW + wave] = wb;
  }
  __syncthreads();
  // 2. elements
  double s = 0.0, c = 0.0;
  int cnt = 0;
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int le = k * NT + tid;
    if (le < net) {
      T uu[K][D], xx[K][DIM];
#pragma unroll
      for (int l = 0; l < K; ++l) NodeVec<T, D>::load(sh.us, nd[k][l], uu[l]);
      if constexpr (GEO == GEO_OTF) {
#pragma unroll
        for (int l = 0; l < K; ++l) NodeVec<T, DIM>::load(sh.xs(), nd[k][l], xx[l]);
      }
      constexpr bool FIRST = EPT == 1;
      element_pass<DIM, D, KIND, T, MODE, GEO, FIRST>(e0 + le, M.ne, uu,
                                                      GEO == GEO_CLASS ? sh.tab : geo, cl[k],
                                                      xx, sh.fs, kTileElems, le, prm, s, c,
                                                      cnt);
    }
  }
  // the next tile's head: in flight while this tile sums its patches
  if (next != nullptr && tnext >= 0)
    tile_head<NPT, NT, MODE != MODE_ENERGY>(M, tnext, *next, tid);
  // The tile's energy: where the nodal-value slots (dead once the elements are done) hold a
  // double per thread, every thread leaves its element energy there and wavefront 0 adds
  // them (one column of NW values per lane, then one wavefront sum); otherwise each
  // wavefront sums its own share. All densities are nonnegative, so the plain FP64 sums are
  // within (NW + 5) u of the tile's energy; tiles are combined compensated.
  constexpr bool kLdsEnergy = P1E_LDS_ENERGY_SUM && sizeof(sh.us) >= NT * sizeof(double);
  {
    const int wn = wave_count(cnt);
    if constexpr (!kLdsEnergy) {
      const double wj = wave_sum(s + c);  // this wavefront's share of the energy
      if (lane == 0) sh.red[wave] = wj;
    }
    if (lane == 0) sh.nbad[wave] = wn;
  }
  // 3. patch sums of the tile's free nodes
  if constexpr (MODE != MODE_ENERGY || kLdsEnergy) {
    __syncthreads();
    if constexpr (kLdsEnergy) reinterpret_cast<double *>(sh.us)[tid] = EPT == 1 ? s : s + c;
    if constexpr (MODE != MODE_ENERGY) {
      if (nloc <= NT / 2)
        tile_patch_sums<D, T, NT, 2>(M, r0, nloc, scale, g, sh, h.prec, pb, tid);
      else
        tile_patch_sums<D, T, NT, 1>(M, r0, nloc, scale, g, sh, h.prec, pb, tid);
    }
  }
  // 4. partials: compensated sums of the per-wavefront shares
  __syncthreads();
  if (wave == 0) {
    double2 rj;
    if constexpr (kLdsEnergy) {
      const double *E = reinterpret_cast<const double *>(sh.us);
      double a = E[lane];
#pragma unroll
      for (int w = 1; w < NW; ++w) a += E[w * 64 + lane];
      rj = make_double2(wave_sum(a), 0.0);
    } else {
      rj = waves_combine<NW>(sh.red);
    }
    const double2 rb = waves_combine<NW>(sh.red + NW);
    if (lane == 0) {
      int n = 0;
      for (int w = 0; w < NW; ++w) n += sh.nbad[w];
      M.part[t] = rj;
      M.part[M.ntiles + t] = rb;
      M.badp[t] = n;
    }
  }
  __syncthreads();  // a persistent caller reuses the LDS for its next tile
}

// Halo row h: a free node whose patch spans several tiles (or none) sums its slots (one per
// tile, ascending tile order; partials of type T, summed in FP64) and writes
// g = scale * (sum - b).
template <int D, typename T>
__device__ __forceinline__ void halo_row(const TileMesh &M, int h, double *__restrict__ g,
                                         const double *__restrict__ scale) {
  const int4 hr = M.hrec[h];
  const int mask = hr.z & 7, fb = hr.z >> 3;
  double bv[D];  // fetched first: its latency overlaps the slot loads
  {
    int f = fb;
#pragma unroll
    for (int j = 0; j < D; ++j) bv[j] = ((mask >> j) & 1) ? M.bhat[f++] : 0.0;
  }
  double acc[D];
#pragma unroll
  for (int j = 0; j < D; ++j) acc[j] = 0.0;
  const T *hp = reinterpret_cast<const T *>(M.hpart) + (int64_t)hr.x * D;
  // slots in rounds of 4 whose loads are issued together; the sum stays sequential in tile
  // order (absent slots load nothing and add zero)
  for (int q = 0; q < hr.y; q += 4) {
    T x[4][D];
    bool ok[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      ok[u] = q + u < hr.y;
#pragma unroll
      for (int j = 0; j < D; ++j) x[u][j] = T(0);
      if (ok[u])
#pragma unroll
        for (int j = 0; j < D; ++j) x[u][j] = hp[(q + u) * D + j];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int j = 0; j < D; ++j) acc[j] += ok[u] ? (double)x[u][j] : 0.0;
  }
  const double sc = scale ? *scale : 1.0;
  int f = fb;
#pragma unroll
  for (int j = 0; j < D; ++j)
    if ((mask >> j) & 1) {
      g[f] = sc * (acc[j] - bv[j]);
      ++f;
    }
}

}  // namespace dev
}  // namespace p1e
