// Matrix-core building blocks shared by the two MFMA solver kernels.
//
// Layout of a 16 x 16 product tile (v_mfma_*_16x16x*): lane l of a wave holds
// column j = l % 16 and row group q = l / 16, i.e. output rows 4q + r (r = 0..3)
// of column j. In the solver the column is a goal and the rows are either 16
// time samples (after a basis evaluation) or the 11 coefficients padded to 16
// (after a contraction over time or an 11 x 11 apply). The K index of every
// product is chosen so that a lane's B operand is exactly the four values it
// already holds; the constant A operands are permuted to match when loaded.
//
// Two precisions:
//   FP32:   v_mfma_f32_16x16x4_f32 for evaluations, contractions and the heading
//           apply; v_mfma_f64_16x16x4_f64 for the x/y applies, whose constant
//           operators stay FP64.
//   BF16x3: v_mfma_f32_16x16x32_bf16 with split operands x = hi + lo (bf16 each):
//           hi*hi + lo*hi + hi*lo in two instructions (K = 32 holds hi and lo of
//           16 K values), FP32 accumulation, for the basis evaluations and the x/y
//           contractions; the heading contraction on v_mfma_f32_16x16x4_f32; the
//           x/y and heading applies (inverse x right-hand side, eqs. 18, 20) in a
//           three-way split h + m + l (bf16 each, exact for FP32 values) with the
//           six products of order >= 2^-16 in three instructions. No FP64
//           arithmetic: FP64 stays in forming and inverting the KKT matrices.
#pragma once
#include "traj_device.h"

namespace traj {
namespace mma {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int TILE = 16;   // time samples per product tile
constexpr int GCOLS = 16;  // goals per product tile

__device__ __forceinline__ f4 mma32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ d4 mma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mmabf(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ __bf16 bf_hi(float x) { return (__bf16)x; }
__device__ __forceinline__ __bf16 bf_lo(float x) { return (__bf16)(x - (float)(__bf16)x); }

// B operand of a split product from the lane's 4 values: K slots 8q + e hold
// hi(v[e]) for e < 4 and lo(v[e - 4]) for e >= 4.
__device__ __forceinline__ bf8 split_b(const f4& v) {
  bf8 b;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    b[e] = bf_hi(v[e]);
    b[e + 4] = bf_lo(v[e]);
  }
  return b;
}
// A operands of a split product from 4 values a[e] (K slots 8q + e and 8q + e + 4):
// first instruction hi(a) against (hi, lo) of B, second lo(a) against hi of B.
__device__ __forceinline__ void split_a(const float (&a)[4], bf8& first, bf8& second) {
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    first[e] = bf_hi(a[e]);
    first[e + 4] = bf_hi(a[e]);
    second[e] = bf_lo(a[e]);
    second[e + 4] = (__bf16)0.f;
  }
}

// A operand of one 16 x 16 x 16 product (K = the 16 rows of the lane group):
// four FP32 K-steps, or the two split BF16 instructions.
template <int MODE>
struct Operand;
template <>
struct Operand<TRAJ_MODE_FP32> {
  float v[4];
};
template <>
struct Operand<TRAJ_MODE_BF16X3> {
  bf8 v[2];
};

template <int MODE>
__device__ __forceinline__ void make_operand(Operand<MODE>& o, const float (&a)[4]) {
  if constexpr (MODE == TRAJ_MODE_FP32) {
#pragma unroll
    for (int e = 0; e < 4; ++e) o.v[e] = a[e];
  } else {
    split_a(a, o.v[0], o.v[1]);
  }
}

// Basis evaluation at the lane's 4 rows for coefficients c (rows 4q + r of the
// lane's column); cb is the split form of c (BF16x3 only).
template <int MODE>
__device__ __forceinline__ f4 eval(const Operand<MODE>& a, const f4& c, const bf8& cb) {
  f4 acc = {0.f, 0.f, 0.f, 0.f};
  if constexpr (MODE == TRAJ_MODE_FP32) {
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) acc = mma32(a.v[kk], c[kk], acc);
  } else {
    acc = mmabf(a.v[0], cb, acc);
    acc = mmabf(a.v[1], cb, acc);
  }
  return acc;
}

// acc += (the transposed basis tile) x s, s = per-sample values at the lane's 4 rows
template <int MODE>
__device__ __forceinline__ f4 contract(const Operand<MODE>& a, const f4& s, f4 acc) {
  if constexpr (MODE == TRAJ_MODE_FP32) {
#pragma unroll
    for (int r = 0; r < 4; ++r) acc = mma32(a.v[r], s[r], acc);
  } else {
    const bf8 sb = split_b(s);
    acc = mmabf(a.v[0], sb, acc);
    acc = mmabf(a.v[1], sb, acc);
  }
  return acc;
}

// Three-way split of an FP32 value into bf16 parts, x = h + m + l: each part takes
// the next 8 significant bits of the remainder (the subtractions are exact).
__device__ __forceinline__ void split3(float x, __bf16& h, __bf16& m, __bf16& l) {
  h = (__bf16)x;
  const float r1 = x - (float)h;
  m = (__bf16)r1;
  l = (__bf16)(r1 - (float)m);
}

// acc + A v for one 16 x 16 operator in the three-way split: lane (j, q) holds
// a[e] = A[row j][k = 4 q + e] and its column's values v[e] = v[k = 4 q + e]. K slot
// 8 q + e carries k = 4 q + e and slot 8 q + 4 + e the same k again, so the three
// instructions form h(A) (h(v) + m(v)), m(A) (h(v) + m(v)) and l(A) h(v) + h(A) l(v):
// every product of order >= 2^-16 of the leading one, FP32 accumulation, smallest
// terms first.
__device__ __forceinline__ f4 mv_split3(const float (&a)[4], const f4& v, f4 acc) {
  bf8 vhm, vhl, a_h, a_m, a_lh;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    __bf16 h, m, l;
    split3(v[e], h, m, l);
    vhm[e] = h;
    vhm[e + 4] = m;
    vhl[e] = h;
    vhl[e + 4] = l;
    split3(a[e], h, m, l);
    a_h[e] = h;
    a_h[e + 4] = h;
    a_m[e] = m;
    a_m[e + 4] = m;
    a_lh[e] = l;
    a_lh[e + 4] = h;
  }
  acc = mmabf(a_lh, vhl, acc);
  acc = mmabf(a_m, vhm, acc);
  return mmabf(a_h, vhm, acc);
}

// Row j of an NC x NC operator of the FP32 table at the lane's K values 4 q + e
// (zero outside the NC x NC block).
__device__ __forceinline__ void load_row4(const float* __restrict__ T, int n, int sq, int j, int q, float (&a)[4]) {
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int k = 4 * q + e;
    a[e] = (j < NC && k < NC) ? T[tab_square(n, sq) + j * NC + k] : 0.f;
  }
}

// The split form's x/y step for one axis: c0 + MG c + M r (eq. 18), three-way split.
__device__ __forceinline__ f4 apply_xy_split3(const float* __restrict__ T, int n, int axis, int j, int q,
                                              const f4& c0, const f4& c, const f4& r) {
  float a[4];
  load_row4(T, n, axis == 0 ? SQ_MX : SQ_MY, j, q, a);
  f4 acc = mv_split3(a, r, c0);
  load_row4(T, n, axis == 0 ? SQ_MGX : SQ_MGY, j, q, a);
  return mv_split3(a, c, acc);
}

// The split form's heading step: c0p + M_psi r (eq. 20), three-way split.
__device__ __forceinline__ f4 apply_psi_split3(const float* __restrict__ T, int n, int j, int q, const f4& c0p,
                                               const f4& r) {
  float a[4];
  load_row4(T, n, SQ_MP, j, q, a);
  return mv_split3(a, r, c0p);
}

// Operators of the FP32 form's x/y and heading applies (rows of the lane's column).
//
// The FP32 form keeps the x/y step's constant operators in FP64: they act on
// coefficients of hundreds of metres with products that cancel, their rounding
// is integrated by the multipliers (eqs. 23, 24) over the iterations, and with
// 50 obstacles an FP32 apply leaves coefficient errors of 2-4e-4 against the
// oracle. The split form, held to a decade looser gate, uses the three-way split
// above (FP32-level products) for these applies. A two-way split (about 16
// significant bits) is too coarse for both applies: the heading operator's
// entries reach ~70 and its row sums ~200 while its products cancel to angles of
// tenths of a radian.
struct XYOps {
  double mg[4], m[4];  // rows permuted for the f64 output layout
};
struct PsiOps {
  float mp[4];
};

__device__ __forceinline__ void load_xy_ops(XYOps& O, const double* __restrict__ T64, int axis, int j, int q) {
  // row permutation of the f64 16x16x4 output: register r of row group q is row 4r + q
  const int prow = 4 * (j & 3) + (j >> 2);
  const double* mg = T64 + (axis == 0 ? T64_MGX : T64_MGY);
  const double* m = T64 + (axis == 0 ? T64_MX : T64_MY);
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int k = 4 * q + kk;
    const bool ok = prow < NC && k < NC;
    O.mg[kk] = ok ? mg[prow * NC + k] : 0.0;
    O.m[kk] = ok ? m[prow * NC + k] : 0.0;
  }
}

__device__ __forceinline__ void load_psi_ops(PsiOps& O, const float* __restrict__ T, int n, int j, int q) {
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int k = 4 * q + kk;
    O.mp[kk] = (j < NC && k < NC) ? T[tab_square(n, SQ_MP) + j * NC + k] : 0.f;
  }
}

// c0 + MG c + M r for one axis, accumulated in FP64
__device__ __forceinline__ f4 apply_xy(const XYOps& O, const d4& c0d, const f4& c, const f4& r) {
  d4 acc = c0d;
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) acc = mma64(O.mg[kk], (double)c[kk], acc);
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) acc = mma64(O.m[kk], (double)r[kk], acc);
  f4 out;
#pragma unroll
  for (int k = 0; k < 4; ++k) out[k] = (float)acc[k];
  return out;
}

__device__ __forceinline__ f4 apply_psi(const PsiOps& O, const f4& c0p, const f4& r) {
  f4 acc = c0p;
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) acc = mma32(O.mp[kk], r[kk], acc);
  return acc;
}

// End-to-end line of a position coefficient vector (rows 4q + r of goal column j).
// A Bernstein basis reproduces linear coefficients exactly (sum_k B_k = 1 and
// sum_k (k/N) B_k = tau), so c_k = c0 + (cN - c0) k/N evaluates to c0 + v t with
// v = (cN - c0) / t_f, its derivative to v and its second derivative to 0. The
// split-BF16 form evaluates the coefficients relative to this line and adds the
// line back in FP32: the split (about 16 significant bits) then carries the
// deviation from uniform motion, metres, instead of positions of hundreds of metres.
struct Trend {
  float c0, d, v;  // first coefficient, last minus first, slope in time
};
static_assert(NC == 11, "the last coefficient row N = 10 is register 2 of row group 2");

__device__ __forceinline__ Trend trend_of(const f4& c, int j, float inv_tf) {
  Trend L;
  L.c0 = __shfl(c[0], j);                 // row 0: row group 0, register 0
  const float cN = __shfl(c[2], j + 32);  // row 10: row group 2, register 2
  L.d = cN - L.c0;
  L.v = L.d * inv_tf;
  return L;
}

__device__ __forceinline__ bf8 split_detrended(const f4& c, const Trend& L, int q) {
  f4 e;
#pragma unroll
  for (int r = 0; r < 4; ++r) e[r] = c[r] - fmaf(L.d, (float)(4 * q + r) * (1.f / (NC - 1)), L.c0);
  return split_b(e);
}

__device__ __forceinline__ float4 f4to(const f4& v) { return make_float4(v[0], v[1], v[2], v[3]); }
__device__ __forceinline__ f4 tof4(const float4& v) {
  f4 r = {v.x, v.y, v.z, v.w};
  return r;
}

// sum over the 4 row groups (lanes j, j+16, j+32, j+48), result in every lane
__device__ __forceinline__ float sum_rows(float v) {
  const auto a = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(unsigned, v), __builtin_bit_cast(unsigned, v),
                                                  false, false);
  const unsigned a0 = a[0], a1 = a[1];
  const float s = __builtin_bit_cast(float, a0) + __builtin_bit_cast(float, a1);
  const auto b = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, s), __builtin_bit_cast(unsigned, s),
                                                  false, false);
  const unsigned b0 = b[0], b1 = b[1];
  return __builtin_bit_cast(float, b0) + __builtin_bit_cast(float, b1);
}

// Boundary values (eq. 8b) of a goal and the particular parts M_b b of its three
// steps at the lane's coefficient rows 4q + r; with cold, also the boundary-only
// minimum-acceleration start.
// FP32 form: the x/y parts in FP64 (c0xd, c0yd); split form: in FP32 (c0x, c0y).
struct Particular {
  d4 c0xd, c0yd;
  f4 c0x, c0y;
  f4 c0p;
};

template <int MODE>
__device__ __forceinline__ void particular(const float* __restrict__ T, const double* __restrict__ T64, int n,
                                           const float* e, const float* gl, int q, Particular& P, bool cold, f4& cx,
                                           f4& cy) {
  const float bx[NX] = {e[0], e[2], e[4], gl[0]};
  const float by[NY] = {e[1], e[3], e[5], gl[1], 0.f, 0.f};
  const float bp[NP] = {e[6], e[7], 0.f, 0.f};
  const float* Bt = T + tab_bnd(n);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int k = 4 * q + r;
    P.c0xd[r] = 0.0;
    P.c0yd[r] = 0.0;
    P.c0x[r] = 0.f;
    P.c0y[r] = 0.f;
    P.c0p[r] = 0.f;
    if (cold) {  // the padding rows k >= NC too: an apply multiplies them by zero operator
      cx[r] = 0.f;  // columns, which a NaN or infinity left there would turn into NaN
      cy[r] = 0.f;
    }
    if (k < NC) {
      if constexpr (MODE == TRAJ_MODE_FP32) {
        double sx = 0.0, sy = 0.0;
        for (int i = 0; i < NX; ++i) sx = fma(T64[T64_MBX + k * NX + i], (double)bx[i], sx);
        for (int i = 0; i < NY; ++i) sy = fma(T64[T64_MBY + k * NY + i], (double)by[i], sy);
        P.c0xd[r] = sx;
        P.c0yd[r] = sy;
      } else {
        float sx = 0.f, sy = 0.f;
        for (int i = 0; i < NX; ++i) sx = fmaf(Bt[BND_MBX + k * NX + i], bx[i], sx);
        for (int i = 0; i < NY; ++i) sy = fmaf(Bt[BND_MBY + k * NY + i], by[i], sy);
        P.c0x[r] = sx;
        P.c0y[r] = sy;
      }
      float sp = 0.f;
      for (int i = 0; i < NP; ++i) sp = fmaf(Bt[BND_MBP + k * NP + i], bp[i], sp);
      P.c0p[r] = sp;
      if (cold) {
        float vx = 0.f, vy = 0.f;
        for (int i = 0; i < NX; ++i) vx = fmaf(Bt[BND_M0BX + k * NX + i], bx[i], vx);
        for (int i = 0; i < NY; ++i) vy = fmaf(Bt[BND_M0BY + k * NY + i], by[i], vy);
        cx[r] = vx;
        cy[r] = vy;
      }
    }
  }
}

}  // namespace mma
}  // namespace traj
