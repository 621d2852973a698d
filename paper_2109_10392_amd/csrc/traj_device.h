// Device helpers shared by the solver kernels: cross-lane primitives of gfx950
// (DPP row/quad permutations, permlane16/32 swaps), wave reductions and the
// workgroup -> scene lookup.
#pragma once
#include "traj_internal.h"

namespace traj {
namespace dev {

constexpr int DPP_QUAD_1032 = 0xB1;  // quad_perm [1,0,3,2]: partner lane ^ 1
constexpr int DPP_QUAD_2301 = 0x4E;  // quad_perm [2,3,0,1]: partner lane ^ 2
constexpr int DPP_ROW_MIRROR = 0x140;       // lane p <-> 15 - p within a row of 16
constexpr int DPP_ROW_HALF_MIRROR = 0x141;  // lane p <-> 7 - p within a half-row of 8

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ float rdlane(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

// lanes 0-31 of the result: a summed over lane pairs (l, l+32); lanes 32-63: b summed likewise
__device__ __forceinline__ float swap32_add(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, a), __builtin_bit_cast(unsigned, b),
                                                  false, false);
  // copy the two results out as values first: a bit_cast of the vector element
  // lvalue r[1] is lowered as element 0 by this compiler
  const unsigned r0 = r[0], r1 = r[1];
  return __builtin_bit_cast(float, r0) + __builtin_bit_cast(float, r1);
}

// within each 32-lane half: lanes 0-15 a summed over (l, l+16), lanes 16-31 b summed likewise
__device__ __forceinline__ float swap16_add(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(unsigned, a), __builtin_bit_cast(unsigned, b),
                                                  false, false);
  const unsigned r0 = r[0], r1 = r[1];
  return __builtin_bit_cast(float, r0) + __builtin_bit_cast(float, r1);
}

// lanes 32-63 receive lanes 0-31 of v (lanes 0-31 keep v)
__device__ __forceinline__ float permlane_lo_to_hi(float v) {
  const auto r = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, v), __builtin_bit_cast(unsigned, v),
                                                  false, false);
  const unsigned r0 = r[0];
  return __builtin_bit_cast(float, r0);
}

// Wave-wide minimum / maximum, returned in every lane.
__device__ __forceinline__ float wave_min(float v) {
  v = fminf(v, dpp<DPP_QUAD_1032>(v));
  v = fminf(v, dpp<DPP_QUAD_2301>(v));
  v = fminf(v, dpp<DPP_ROW_HALF_MIRROR>(v));
  v = fminf(v, dpp<DPP_ROW_MIRROR>(v));
  const auto a = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(unsigned, v), __builtin_bit_cast(unsigned, v),
                                                  false, false);
  const unsigned a0 = a[0], a1 = a[1];
  v = fminf(__builtin_bit_cast(float, a0), __builtin_bit_cast(float, a1));
  const auto b = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, v), __builtin_bit_cast(unsigned, v),
                                                  false, false);
  const unsigned b0 = b[0], b1 = b[1];
  return fminf(__builtin_bit_cast(float, b0), __builtin_bit_cast(float, b1));
}

__device__ __forceinline__ float wave_max(float v) { return -wave_min(-v); }

// Order-preserving integer key of a float: key(a) < key(b) whenever a < b (not NaN;
// -0 sorts below +0). Integer minima and maxima fold into single DPP instructions,
// where the float ones need canonicalising moves.
__device__ __forceinline__ int order_key(float x) {
  const int b = __builtin_bit_cast(int, x);
  return b ^ ((b >> 31) & 0x7fffffff);
}

template <int CTRL>
__device__ __forceinline__ int dpp_i(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, CTRL, 0xF, 0xF, false);
}

// Minimum / maximum of an integer over each DPP row of 16 lanes, in every lane of the row.
__device__ __forceinline__ int row_min_i(int v) {
  constexpr int TOP = 0x7fffffff;
  v = min(v, dpp_i<DPP_QUAD_1032>(TOP, v));
  v = min(v, dpp_i<DPP_QUAD_2301>(TOP, v));
  v = min(v, dpp_i<DPP_ROW_HALF_MIRROR>(TOP, v));
  return min(v, dpp_i<DPP_ROW_MIRROR>(TOP, v));
}

__device__ __forceinline__ int row_max_i(int v) {
  constexpr int BOTTOM = (int)0x80000000;
  v = max(v, dpp_i<DPP_QUAD_1032>(BOTTOM, v));
  v = max(v, dpp_i<DPP_QUAD_2301>(BOTTOM, v));
  v = max(v, dpp_i<DPP_ROW_HALF_MIRROR>(BOTTOM, v));
  return max(v, dpp_i<DPP_ROW_MIRROR>(BOTTOM, v));
}

__device__ __forceinline__ int rdlane_i(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

// Wave-wide minimum / maximum of an integer, in every lane.
__device__ __forceinline__ int wave_min_i(int v) {
  v = row_min_i(v);
  const auto a = __builtin_amdgcn_permlane16_swap((unsigned)v, (unsigned)v, false, false);
  const unsigned a0 = a[0], a1 = a[1];
  v = min((int)a0, (int)a1);
  const auto b = __builtin_amdgcn_permlane32_swap((unsigned)v, (unsigned)v, false, false);
  const unsigned b0 = b[0], b1 = b[1];
  return min((int)b0, (int)b1);
}

__device__ __forceinline__ int wave_max_i(int v) {
  v = row_max_i(v);
  const auto a = __builtin_amdgcn_permlane16_swap((unsigned)v, (unsigned)v, false, false);
  const unsigned a0 = a[0], a1 = a[1];
  v = max((int)a0, (int)a1);
  const auto b = __builtin_amdgcn_permlane32_swap((unsigned)v, (unsigned)v, false, false);
  const unsigned b0 = b[0], b1 = b[1];
  return max((int)b0, (int)b1);
}

// Wave-local LDS exchange. Values written by some lanes of a wave and read by
// others of the same wave: the fences and the wave barrier keep the compiler from
// moving the reads above the writes (the hardware runs one wave's LDS accesses
// in order).
__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Obstacle candidate lists. A scaled obstacle state that no trajectory sample
// reaches: (x/a - 1e30)^2 overflows to +inf, so the test q < 1 fails. A wave's
// list holds every obstacle plus seven such entries after the last candidate, so
// rounds of four can read the next round's entries before testing their own.
constexpr float UNREACHABLE = 1e30f;
constexpr int CLIST = MAX_OBS + 7;

// Compacts the scaled states `ob` of the lanes with `hit` set into list[0, cnt) in
// lane order and pads list[cnt, cnt + 7) with unreachable entries; returns cnt.
// Every lane of the wave must take part.
__device__ __forceinline__ int compact_candidates(bool hit, const float4& ob, float4* list) {
  const int lane = threadIdx.x & (WAVE - 1);
  const unsigned long long cand = __ballot(hit);
  const int cnt = __popcll(cand);
  if (hit) list[__builtin_amdgcn_mbcnt_hi((unsigned)(cand >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)cand, 0u))] = ob;
  if (lane < 7) list[cnt + lane] = make_float4(UNREACHABLE, UNREACHABLE, 0.f, 0.f);
  wave_sync_lds();
  return cnt;
}

// Obstacle polar variables at one sample inside a scaled ellipse (eqs. 15 and 22;
// q = tx^2 + ty^2 < 1 in units scaled by (1/a, 1/b)): d/du - 1 = 1/du - 1 with
// du = sqrt(q), added to s_o as (tx, ty) (1/du - 1), and the sample's squared
// obstacle residual (a tx, b ty)^2 (1/du - 1)^2. On the obstacle centre alpha =
// atan2(+0, +0) = 0 and d = 1. The hardware reciprocal square root equals the
// library's for a normal argument but reads a denormal as 0, so an offset whose q
// is below 2^-126 (under 1.1e-19 in scaled units, where the angle of eq. 22 is no
// longer resolved) counts as the centre.
__device__ __forceinline__ void obstacle_inside(float tx, float ty, float q, float a2, float b2, float& Sx,
                                                float& Sy, float& ro) {
  const bool centre = !(q >= 0x1p-126f);
  const float f = __builtin_amdgcn_rsqf(q) - 1.f;
  Sx = centre ? Sx + 1.f : fmaf(tx, f, Sx);
  Sy = centre ? Sy : fmaf(ty, f, Sy);
  ro = centre ? ro + a2 : fmaf(fmaf(a2 * tx, tx, b2 * ty * ty), f * f, ro);
}

// Minimum over each DPP row of 16 lanes, returned in every lane of the row.
__device__ __forceinline__ float row_min(float v) {
  v = fminf(v, dpp<DPP_QUAD_1032>(v));
  v = fminf(v, dpp<DPP_QUAD_2301>(v));
  v = fminf(v, dpp<DPP_ROW_HALF_MIRROR>(v));
  return fminf(v, dpp<DPP_ROW_MIRROR>(v));
}

__device__ __forceinline__ float row_max(float v) { return -row_min(-v); }

// sin and cos of |r| <= pi/2: Taylor series about 0 truncated after r^13 / r^12
// (alternating series: the truncation error is below the first omitted term,
// 6.7e-10 for sin and 6.4e-9 for cos at pi/2, under FP32's rounding of values
// near 1).
__device__ __forceinline__ void sincos_taylor(float x, float* sn, float* cs) {
  const float x2 = x * x;
  float ps = 1.6059044e-10f;                  //  1/13!
  ps = fmaf(ps, x2, -2.5052108e-08f);         // -1/11!
  ps = fmaf(ps, x2, 2.7557319e-06f);          //  1/9!
  ps = fmaf(ps, x2, -1.9841270e-04f);         // -1/7!
  ps = fmaf(ps, x2, 8.3333333e-03f);          //  1/5!
  ps = fmaf(ps, x2, -1.6666667e-01f);         // -1/3!
  *sn = fmaf(ps * x2, x, x);
  float pc = 2.0876757e-09f;                  //  1/12!
  pc = fmaf(pc, x2, -2.7557319e-07f);         // -1/10!
  pc = fmaf(pc, x2, 2.4801587e-05f);          //  1/8!
  pc = fmaf(pc, x2, -1.3888889e-03f);         // -1/6!
  pc = fmaf(pc, x2, 4.1666667e-02f);          //  1/4!
  pc = fmaf(pc, x2, -0.5f);                   // -1/2!
  *cs = fmaf(pc, x2, 1.0f);
}

// sin and cos of a heading angle. |x| <= pi/2 (every heading the method keeps):
// the Taylor kernel directly. Larger angles: reduction by multiples of pi/2 with
// a three-part split of pi/2 (Cody and Waite, with fused multiply-adds; relative
// error of the reduced argument below 1e-7 for |x| < 1e3, growing slowly beyond)
// and the quadrant's sign/swap. Non-finite input gives NaN.
__device__ __forceinline__ void sincos_heading(float x, float* sn, float* cs) {
  if (fabsf(x) <= 1.5707964f) {
    sincos_taylor(x, sn, cs);
  } else {
    constexpr float C1 = 1.570796371e+00f, C2 = -4.371138829e-08f, C3 = -1.715124510e-15f;  // pi/2
    const float k = rintf(x * 6.366197467e-01f);                                              // x / (pi/2)
    float r = fmaf(-k, C1, x);
    r = fmaf(-k, C2, r);
    r = fmaf(-k, C3, r);
    float s, c;
    sincos_taylor(r, &s, &c);
    const int quad = (int)fminf(fmaxf(k, -16777216.f), 16777216.f) & 3;
    *sn = quad == 0 ? s : (quad == 1 ? c : (quad == 2 ? -s : -c));
    *cs = quad == 0 ? c : (quad == 1 ? -s : (quad == 2 ? -c : s));
  }
}

// atan2 of a heading direction. First octant: a = min(|x|, |y|) / max(|x|, |y|)
// in [0, 1]; atan(a) = a p(a^2) with p a degree-9 polynomial in a^2, p(0) = 1,
// fitted for relative error to atan(sqrt(s)) / sqrt(s) on [0, 1] (Lawson's
// reweighted least squares on Chebyshev nodes, fit_atan2_poly.py in this folder
// with its defaults; 1.24 units in the last place at most in FP32 Horner form);
// then pi/2 - r past the diagonal, pi - r for negative x (sign bit, so -0 counts)
// and the sign of y. Special cases as IEEE atan2: (+-0, +0) -> +-0,
// (+-0, -0) -> +-pi, both infinite -> +-pi/4 or +-3pi/4, NaN in -> NaN. Tiny
// magnitudes are scaled by 2^100 (exact) before the reciprocal.
__device__ __forceinline__ float atan2_heading(float y, float x) {
  const float ax = fabsf(x), ay = fabsf(y);
  float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
  const float sc = mx < 0x1p-100f ? 0x1p+100f : 1.f;
  mx *= sc;
  mn *= sc;
  float a = mn * __builtin_amdgcn_rcpf(mx);
  a = (mn == mx) ? 1.f : a;   // equal magnitudes, both infinite included
  a = (mn == 0.f) ? 0.f : a;  // an axis (both zero included)
  const float s = a * a;
  float p = -1.79358129e-03f;
  p = fmaf(p, s, 1.09144244e-02f);
  p = fmaf(p, s, -3.11775077e-02f);
  p = fmaf(p, s, 5.79572544e-02f);
  p = fmaf(p, s, -8.40343013e-02f);
  p = fmaf(p, s, 1.09521791e-01f);
  p = fmaf(p, s, -1.42642409e-01f);
  p = fmaf(p, s, 1.99985474e-01f);
  p = fmaf(p, s, -3.33332986e-01f);
  p = fmaf(p, s, 1.0f);
  float r = a * p;
  r = (ay > ax) ? 1.57079637f - r : r;
  r = __builtin_signbit(x) ? 3.14159274f - r : r;
  r = copysignf(r, y);
  return (x != x || y != y) ? x + y : r;
}

// Wave-wide sums of 32 per-lane values: on return lane l holds the sum of value l >> 1.
// LIVE: values i and i + 16 for i >= LIVE are known to be zero in every lane (their
// first exchange is skipped).
template <int LIVE = 16>
__device__ __forceinline__ float reduce32(const float (&v)[32]) {
  const int lane = threadIdx.x & (WAVE - 1);
  float s[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) s[i] = i < LIVE ? swap32_add(v[i], v[i + 16]) : 0.f;
  float t[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) t[i] = swap16_add(s[i], s[i + 8]);
  const bool lo8 = (lane & 8) == 0;
  float u[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) u[i] = (lo8 ? t[i] : t[i + 4]) + dpp<DPP_ROW_MIRROR>(lo8 ? t[i + 4] : t[i]);
  const bool lo4 = (lane & 4) == 0;
  float w[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) w[i] = (lo4 ? u[i] : u[i + 2]) + dpp<DPP_ROW_HALF_MIRROR>(lo4 ? u[i + 2] : u[i]);
  const bool lo2 = (lane & 2) == 0;
  float z = (lo2 ? w[0] : w[1]) + dpp<DPP_QUAD_2301>(lo2 ? w[1] : w[0]);
  return z + dpp<DPP_QUAD_1032>(z);
}

// Wave-wide sums of 16 per-lane values: on return lane l holds the sum of value l >> 2.
__device__ __forceinline__ float reduce16(const float (&v)[16]) {
  const int lane = threadIdx.x & (WAVE - 1);
  float s[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) s[i] = swap32_add(v[i], v[i + 8]);
  float t[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) t[i] = swap16_add(s[i], s[i + 4]);
  const bool lo8 = (lane & 8) == 0;
  float u[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) u[i] = (lo8 ? t[i] : t[i + 2]) + dpp<DPP_ROW_MIRROR>(lo8 ? t[i + 2] : t[i]);
  const bool lo4 = (lane & 4) == 0;
  float z = (lo4 ? u[0] : u[1]) + dpp<DPP_ROW_HALF_MIRROR>(lo4 ? u[1] : u[0]);
  z += dpp<DPP_QUAD_2301>(z);
  return z + dpp<DPP_QUAD_1032>(z);
}


// Workgroup b of a launch runs on XCD b mod 8 (the dispatcher deals workgroups
// round robin over the device's eight XCDs). xcd_block(b, nb) renumbers them in
// tiles of 256: within a tile, XCD x takes the 32 consecutive work items
// [32 x, 32 x + 32), so the goal-fastest outputs of 32 neighbouring items (a
// 128-byte line per output row when an item is one goal) are all written through
// one L2, which writes the lines back whole instead of in 4-byte pieces. The
// items resident on one XCD at a time still spread over the whole range, as in
// the plain order: one contiguous range per XCD would gather neighbouring goals,
// whose costs are alike, onto the same compute units. The last partial tile keeps
// the plain order. A bijection on [0, nb).
__device__ __forceinline__ int xcd_block(int b, int nb) {
  constexpr int XCDS = 8, RUN = 32, TILE = XCDS * RUN;
  if (b >= nb / TILE * TILE) return b;
  const int r = b % TILE;
  return b - r + (r % XCDS) * RUN + r / XCDS;
}

// Work item -> (scene, first goal): scene s owns ceil(goals_s / per_item)
// consecutive items. Returns scene -1 past the last one. scan needs one int per
// wave of the workgroup.
__device__ void locate(const int32_t* goal_off, int n_scenes, int per_item, int* sh, int* scan, int block) {
  const int tid = threadIdx.x;
  const int lane = tid & (WAVE - 1), wv = tid >> 6;
  if (tid == 0) {
    sh[0] = -1;
    sh[1] = 0;
  }
  int base = 0;
  for (int c0 = 0; c0 < n_scenes; c0 += (int)blockDim.x) {
    const int s = c0 + tid;
    const int cnt = (s < n_scenes) ? (goal_off[s + 1] - goal_off[s] + per_item - 1) / per_item : 0;
    int incl = cnt;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
      const int y = __shfl_up(incl, d, WAVE);
      if (lane >= d) incl += y;
    }
    __syncthreads();
    if (lane == WAVE - 1) scan[wv] = incl;
    __syncthreads();
    int pre = 0, tot = 0;
    const int nw = (int)blockDim.x / WAVE;
    for (int w = 0; w < nw; ++w) {
      if (w < wv) pre += scan[w];
      tot += scan[w];
    }
    incl += pre;
    const int excl = incl - cnt;
    const int b = block - base;
    if (cnt > 0 && b >= excl && b < incl) {
      sh[0] = s;
      sh[1] = goal_off[s] + per_item * (b - excl);
    }
    base += tot;
    if (base > block) break;  // uniform: every thread sees the same base
  }
  __syncthreads();
}


}  // namespace dev
}  // namespace traj
