// Batched alternating minimisation (Algorithm 1, Sec. III-D) on the matrix cores.
//
// Mapping: one workgroup per goal group (up to 16 goals of one scene: the MFMA
// columns), one wavefront per 16-sample time tile (the MFMA rows). Every dense
// contraction of the method runs on MFMA:
//   basis evaluation    X[t][goal] = sum_k P[t][k] c[k][goal]          (eq. 6)
//   time contractions   U[k][goal] = sum_t P[t][k] S[t][goal]          (F^T g of eq. 18, P^T theta of eq. 20)
//   inverse x RHS       c_new[k][goal] = sum_i M[k][i] r[i][goal]       (eqs. 18, 20)
// with the goal index as the MFMA column. The per-sample closed forms (eqs. 21,
// 22, 15, 16) run on the vector ALU over each lane's 4 samples. A contraction's
// partial sums over one tile are added across the workgroup's waves through LDS
// in a fixed order, so every wave holds the same totals and repeats the small
// applies itself.
//
// Lane l of a wave: column (goal) j = l % 16, row group q = l / 16. It holds the
// MFMA output rows 4q + r (r = 0..3): time samples 16 w + 4q + r of goal j after
// an evaluation, coefficients 4q + r of goal j after a contraction or apply. The
// K index of every product is chosen so that a lane's operands are exactly the
// values it already holds; the constant operands are permuted to match.
//
// Two precisions:
//   FP32:   v_mfma_f32_16x16x4_f32 for evaluations, contractions and the heading
//           apply; v_mfma_f64_16x16x4_f64 for the x/y applies (their constant
//           operators stay FP64, as in the wave kernel).
//   BF16x3: v_mfma_f32_16x16x32_bf16 with split operands x = hi + lo (bf16 each):
//           hi*hi + lo*hi + hi*lo in two instructions (K = 32 holds hi and lo of
//           16 K values), FP32 accumulation, for every contraction and apply.
#include <mutex>

#include "traj_mma.h"

namespace traj {
namespace {

using namespace dev;
using namespace mma;

// Constant operands of one wave: its time tile of the three basis matrices (for
// evaluation and for the transposed contraction) and the apply operators.
template <int MODE>
struct Ops {
  Operand<MODE> ev[3];  // P, P', P'' [t = 16w + j][4q + kk]
  Operand<MODE> ct[3];  // P, P', P'' [16w + 4q + r][j]
  PsiOps psi;           // the x/y operators (FP64) are read from the tables at each use
};

template <int MODE>
__device__ __forceinline__ f4 evalO(const Ops<MODE>& O, int mi, const f4& c, const bf8& cb) {
  return eval<MODE>(O.ev[mi], c, cb);
}
template <int MODE>
__device__ __forceinline__ f4 contractO(const Ops<MODE>& O, int mi, const f4& s, f4 acc) {
  return contract<MODE>(O.ct[mi], s, acc);
}

// Sum two per-lane vectors over the workgroup's waves (fixed order: identical in
// every wave). ex: [2 buffers][W][2][64] float4.
__device__ __forceinline__ void exchange(float4* ex, int buf, int W, int w, int lane, f4& a, f4& b) {
  float4* mine = ex + ((size_t)(buf * W + w) * 2) * WAVE;
  mine[lane] = f4to(a);
  mine[WAVE + lane] = f4to(b);
  __syncthreads();
  f4 sa = {0.f, 0.f, 0.f, 0.f}, sb = {0.f, 0.f, 0.f, 0.f};
  for (int v = 0; v < W; ++v) {
    const float4* p = ex + ((size_t)(buf * W + v) * 2) * WAVE;
    sa += tof4(p[lane]);
    sb += tof4(p[WAVE + lane]);
  }
  a = sa;
  b = sb;
}

struct Consts {
  int n, m, n_pad, W;
  float rho, a, b, inv_a, inv_b, a2, b2, vmin, vmax, amax, amax2;
};

template <int MODE>
__device__ void load_ops(Ops<MODE>& O, const float* __restrict__ T, const double* __restrict__ T64, int n, int w,
                         int j, int q) {
#pragma unroll
  for (int mi = 0; mi < 3; ++mi) {
    float ev[4], ct[4];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int t = TILE * w + j, k = 4 * q + kk;
      ev[kk] = (t < n && k < NC) ? T[tab_basis(n, mi) + k * n + t] : 0.f;
      const int t2 = TILE * w + 4 * q + kk;
      ct[kk] = (t2 < n && j < NC) ? T[tab_basis(n, mi) + j * n + t2] : 0.f;
    }
    make_operand<MODE>(O.ev[mi], ev);
    make_operand<MODE>(O.ct[mi], ct);
  }
  load_psi_ops(O.psi, T, n, j, q);
}

// Per-sample closed forms for the lane's 4 samples and the contraction inputs.
struct SampleOut {
  f4 sox, soy, sax, say, ex, ey, ep;
  float r_obs, r_acc, r_nh, r_psi;
};

__device__ __forceinline__ void samples(const Consts& K, const float2* __restrict__ xi, const float4* __restrict__ box,
                                        int w, int lane, int q, bool gv, const f4& x, const f4& y, const f4& xd,
                                        const f4& yd, const f4& xdd, const f4& ydd, const f4& psi, const f4& th,
                                        SampleOut& o) {
  bool tv[4];
  float X[4], Y[4];
  // the tile's box as order-preserving integer keys (single-instruction DPP
  // minima and maxima; a strict float inequality implies the same between keys)
  constexpr int TOP = 0x7fffffff, BOTTOM = (int)0x80000000;
  int lxlo = TOP, lxhi = BOTTOM, lylo = TOP, lyhi = BOTTOM;
  o.r_obs = o.r_acc = o.r_nh = o.r_psi = 0.f;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    tv[r] = gv && (TILE * w + 4 * q + r) < K.n;
    X[r] = x[r] * K.inv_a;
    Y[r] = y[r] * K.inv_b;
    const int kx = order_key(X[r]), ky = order_key(Y[r]);
    lxlo = tv[r] ? min(lxlo, kx) : lxlo;
    lxhi = tv[r] ? max(lxhi, kx) : lxhi;
    lylo = tv[r] ? min(lylo, ky) : lylo;
    lyhi = tv[r] ? max(lyhi, ky) : lyhi;
    // velocity (eq. 21), heading direction, z - x'
    // (the hardware square root, within 1 ulp; the clamp to v_min > 0 absorbs a
    // denormal argument read as 0)
    const float v = fminf(fmaxf(__builtin_amdgcn_sqrtf(fmaf(xd[r], xd[r], yd[r] * yd[r])), K.vmin), K.vmax);
    float sn, cs;
    sincos_heading(psi[r], &sn, &cs);
    const float ex = fmaf(v, cs, -xd[r]), ey = fmaf(v, sn, -yd[r]);
    // acceleration polar variables (eq. 16; a_max >= 2^-63, so h2 > a_max^2 is a
    // normal number, where the hardware reciprocal square root is the library's)
    const float h2 = fmaf(xdd[r], xdd[r], ydd[r] * ydd[r]);
    const float fa = h2 > K.amax2 ? K.amax * __builtin_amdgcn_rsqf(h2) - 1.f : 0.f;
    const float sax = xdd[r] * fa, say = ydd[r] * fa;
    const float ep = th[r] - psi[r];
    o.ex[r] = tv[r] ? ex : 0.f;
    o.ey[r] = tv[r] ? ey : 0.f;
    o.sax[r] = tv[r] ? sax : 0.f;
    o.say[r] = tv[r] ? say : 0.f;
    o.ep[r] = tv[r] ? ep : 0.f;
    if (tv[r]) {
      o.r_acc = fmaf(sax, sax, fmaf(say, say, o.r_acc));
      o.r_nh = fmaf(ex, ex, fmaf(ey, ey, o.r_nh));
      o.r_psi = fmaf(ep, ep, o.r_psi);
    }
  }
  // obstacle polar variables (eqs. 15, 22) with exact culling against the
  // tile's obstacle boxes (inflated by the scaled half-axes + 0.1%)
  const int xlo = wave_min_i(lxlo), xhi = wave_max_i(lxhi), ylo = wave_min_i(lylo), yhi = wave_max_i(lyhi);
  bool hit = false;
  if (lane < K.m) {
    const float4 bx = box[w * K.m + lane];
    hit = (xhi > order_key(bx.x)) & (xlo < order_key(bx.y)) & (yhi > order_key(bx.z)) & (ylo < order_key(bx.w));
  }
  unsigned long long cand = __ballot(hit);
  float Sx[4] = {0.f, 0.f, 0.f, 0.f}, Sy[4] = {0.f, 0.f, 0.f, 0.f};
  const float2* base = xi + TILE * w + 4 * q;
  while (cand) {
    const int jo = __builtin_ctzll(cand);
    cand &= cand - 1;
    const float4* p = reinterpret_cast<const float4*>(base + jo * K.n_pad);
    const float4 o01 = p[0], o23 = p[1];
    const float ox[4] = {o01.x, o01.z, o23.x, o23.z};
    const float oy[4] = {o01.y, o01.w, o23.y, o23.w};
    float tx[4], ty[4], qq[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      tx[r] = X[r] - ox[r];
      ty[r] = Y[r] - oy[r];
      qq[r] = tv[r] ? fmaf(tx[r], tx[r], ty[r] * ty[r]) : 2.f;
    }
    if (fminf(fminf(qq[0], qq[1]), fminf(qq[2], qq[3])) < 1.f) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (qq[r] < 1.f) obstacle_inside(tx[r], ty[r], qq[r], K.a2, K.b2, Sx[r], Sy[r], o.r_obs);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    o.sox[r] = K.a * Sx[r];
    o.soy[r] = K.b * Sy[r];
  }
}

template <int MODE>
__global__ __launch_bounds__(768) void k_am_mfma(SolveArgs A, int G) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int sh[2];
  __shared__ int scan[16];
  const int Wl = (int)blockDim.x / WAVE;  // waves launched
  locate(A.goal_off, A.n_scenes, G, sh, scan, xcd_block((int)blockIdx.x, (int)gridDim.x));
  const int scene = sh[0];
  if (scene < 0) return;
  if (A.skip != nullptr && A.skip[scene] != 0) return;  // uniform: one scene per workgroup
  const int g0 = sh[1];
  if (g0 < 0) return;  // goal offsets out of contract: nothing to touch
  const int gcount = min(min(G, (int)A.goal_off[scene + 1] - g0), A.n_goals - g0);
  const int sid = A.shape_id[scene];
  const int o0 = A.obs_off[scene];
  const int m_scene = A.obs_off[scene + 1] - o0;
  bool bad = sid < 0 || sid >= A.n_shapes;
  ShapeDesc sd = {};
  if (!bad) sd = A.shapes[sid];
  bad = bad || !obstacles_ok(o0, m_scene, sd.m) || sd.n < NC || (sd.n + TILE - 1) / TILE > Wl;
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), w = tid >> 6;
  const int j = lane & 15, q = lane >> 4;
  if (bad) {
    if (w == 0 && q < 1 && j < gcount) {
      if (A.resid != nullptr)
        for (int k = 0; k < 4; ++k) A.resid[k * A.n_goals + g0 + j] = __builtin_nanf("");
      if (A.iters_out != nullptr) A.iters_out[g0 + j] = 0;
    }
    return;
  }
  Consts K;
  K.n = sd.n;
  K.m = sd.m;
  K.W = Wl;
  K.n_pad = TILE * Wl;
  K.rho = A.k.rho;
  K.a = A.k.a;
  K.b = A.k.b;
  K.inv_a = 1.f / K.a;
  K.inv_b = 1.f / K.b;
  K.a2 = K.a * K.a;
  K.b2 = K.b * K.b;
  K.vmin = A.k.v_min;
  K.vmax = A.k.v_max;
  K.amax = A.k.a_max;
  K.amax2 = K.amax * K.amax;
  const int n = K.n, m = K.m;
  // LDS: xi [m][n_pad] float2 | box [W][m] float4 | exchange [2][W][2][64] float4
  float2* xi = reinterpret_cast<float2*>(smem);
  float4* box = reinterpret_cast<float4*>(smem + sizeof(float2) * (size_t)m * K.n_pad);
  float4* ex = box + (size_t)Wl * m;
  int obs_marked = 0;  // a non-finite obstacle state seen by this thread
  for (int jo = tid; jo < m; jo += blockDim.x) obs_marked |= !all_finite(A.obs + 4 * (o0 + jo), 4);
  {
    const float dt = sd.t_f / (float)(n - 1);
    for (int e = tid; e < m * K.n_pad; e += blockDim.x) {
      const int jo = e / K.n_pad, i = e - jo * K.n_pad;
      const float* o = A.obs + 4 * (o0 + jo);
      if (i < n) {
        const float t = (float)i * dt;
        xi[e] = make_float2(fmaf(o[2], t, o[0]) * K.inv_a, fmaf(o[3], t, o[1]) * K.inv_b);
      } else {
        xi[e] = make_float2(1e30f, 1e30f);
      }
    }
    for (int e = tid; e < Wl * m; e += blockDim.x) {
      const int ww = e / m, jo = e - ww * m;
      const int i0 = min(TILE * ww, n - 1), i1 = min(TILE * ww + TILE - 1, n - 1);
      const float* o = A.obs + 4 * (o0 + jo);
      const float t0 = (float)i0 * dt, t1 = (float)i1 * dt;
      const float xa = fmaf(o[2], t0, o[0]) * K.inv_a, xb = fmaf(o[2], t1, o[0]) * K.inv_a;
      const float ya = fmaf(o[3], t0, o[1]) * K.inv_b, yb = fmaf(o[3], t1, o[1]) * K.inv_b;
      constexpr float R = 1.001f;
      box[e] = make_float4(fminf(xa, xb) - R, fmaxf(xa, xb) + R, fminf(ya, yb) - R, fmaxf(ya, yb) + R);
    }
  }
  if (__syncthreads_or(obs_marked) != 0 || !all_finite(A.ego + 8 * scene, 8)) {  // workgroup-uniform
    if (j < gcount) write_marked_goal(A, g0 + j, tid / 16, (int)blockDim.x / 16);
    return;
  }

  const float* T = A.tables + sd.table_off;
  const double* T64 = A.tables64 + sd.table64_off;
  Ops<MODE> O;
  load_ops<MODE>(O, T, T64, n, w, j, q);
  const bool gin = j < gcount;  // the lane's column holds a goal
  const int g = g0 + (gin ? j : 0);
  // a goal with a non-finite target is marked here and carried as a padding
  // column (on the ego's start position instead of its target), never stored
  const bool gv = gin && all_finite(A.goal + 2 * g, 2);
  if (w == 0 && gin && !gv) write_marked_goal(A, g, q, 4);
  const int NG = A.n_goals;
  const float rho = K.rho;

  // boundary values (eq. 8b) and the particular parts M_b b of each step (rows 4q + r)
  const float* e = A.ego + 8 * scene;
  const float* gl = gv ? A.goal + 2 * g : e;
  const float bx[NX] = {e[0], e[2], e[4], gl[0]};
  const float by[NY] = {e[1], e[3], e[5], gl[1], 0.f, 0.f};
  const float bp[NP] = {e[6], e[7], 0.f, 0.f};
  const float* Bt = T + tab_bnd(n);
  // the x/y parts in FP64 (FP32 form) or FP32 (split form, no FP64 arithmetic)
  d4 c0xd = {0.0, 0.0, 0.0, 0.0}, c0yd = {0.0, 0.0, 0.0, 0.0};
  f4 c0p = {0.f, 0.f, 0.f, 0.f};
  f4 c0x = c0p, c0y = c0p;
  f4 cx = c0p, cy = c0p, cp = c0p, lx = c0p, ly = c0p, lp = c0p;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int k = 4 * q + r;
    if (k < NC) {
      if constexpr (MODE == TRAJ_MODE_FP32) {
        double sx = 0.0, sy = 0.0;
        for (int i = 0; i < NX; ++i) sx = fma(T64[T64_MBX + k * NX + i], (double)bx[i], sx);
        for (int i = 0; i < NY; ++i) sy = fma(T64[T64_MBY + k * NY + i], (double)by[i], sy);
        c0xd[r] = sx;
        c0yd[r] = sy;
      } else {
        float sx = 0.f, sy = 0.f;
        for (int i = 0; i < NX; ++i) sx = fmaf(Bt[BND_MBX + k * NX + i], bx[i], sx);
        for (int i = 0; i < NY; ++i) sy = fmaf(Bt[BND_MBY + k * NY + i], by[i], sy);
        c0x[r] = sx;
        c0y[r] = sy;
      }
      float sp = 0.f;
      for (int i = 0; i < NP; ++i) sp = fmaf(Bt[BND_MBP + k * NP + i], bp[i], sp);
      c0p[r] = sp;
    }
  }
  const bool cold = (A.flags & TRAJ_INIT_FROM_STATE) == 0;
  if (cold) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int k = 4 * q + r;
      if (k < NC) {
        float sx = 0.f, sy = 0.f;
        for (int i = 0; i < NX; ++i) sx = fmaf(Bt[BND_M0BX + k * NX + i], bx[i], sx);
        for (int i = 0; i < NY; ++i) sy = fmaf(Bt[BND_M0BY + k * NY + i], by[i], sy);
        cx[r] = sx;
        cy[r] = sy;
      }
    }
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int k = 4 * q + r;
      if (k < NC) {
        cx[r] = A.c[(0 * NC + k) * NG + g];
        cy[r] = A.c[(1 * NC + k) * NG + g];
        cp[r] = A.c[(2 * NC + k) * NG + g];
        lx[r] = A.lam[(0 * NC + k) * NG + g];
        ly[r] = A.lam[(1 * NC + k) * NG + g];
        lp[r] = A.lam[(2 * NC + k) * NG + g];
      }
    }
  }

  const f4 zero = {0.f, 0.f, 0.f, 0.f};
  f4 ux, uy, ep = zero;
  float racc[4] = {0.f, 0.f, 0.f, 0.f};
  int buf = 0;
  auto split = [&](const f4& v) -> bf8 {
    if constexpr (MODE == TRAJ_MODE_BF16X3) return split_b(v);
    else return bf8{};
  };
  // positions: split relative to the end-to-end line, which is added back after
  // each evaluation (value, first derivative; the second derivative has none)
  const float inv_tf = 1.f / sd.t_f;
  float tline[4];  // times of the lane's 4 samples
#pragma unroll
  for (int r = 0; r < 4; ++r) tline[r] = (float)(TILE * w + 4 * q + r) * (sd.t_f / (float)(n - 1));
  auto split_pos = [&](const f4& v, Trend& L) -> bf8 {
    if constexpr (MODE == TRAJ_MODE_BF16X3) {
      L = trend_of(v, j, inv_tf);
      return split_detrended(v, L, q);
    } else {
      L = Trend{0.f, 0.f, 0.f};
      return bf8{};
    }
  };
  auto plus_line = [&](f4 v, const Trend& L) {
    if constexpr (MODE == TRAJ_MODE_BF16X3) {
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] += fmaf(L.v, tline[r], L.c0);
    }
    return v;
  };
  auto plus_slope = [&](f4 v, const Trend& L) {
    if constexpr (MODE == TRAJ_MODE_BF16X3) {
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] += L.v;
    }
    return v;
  };
  // one pass of the per-sample blocks at the current coefficients; returns u~
  // (summed over the workgroup) and the lane's residual partials
  auto heading = [&](f4& xd, f4& yd, f4& th, f4& W_, f4& E_) {
    Trend Lx, Ly;
    const bf8 cxb = split_pos(cx, Lx), cyb = split_pos(cy, Ly);
    xd = plus_slope(evalO<MODE>(O, 1, cx, cxb), Lx);
    yd = plus_slope(evalO<MODE>(O, 1, cy, cyb), Ly);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const bool tv = gv && (TILE * w + 4 * q + r) < n;
      th[r] = tv ? atan2_heading(yd[r], xd[r]) : 0.f;
    }
    W_ = contractO<MODE>(O, 0, th, zero);
    E_ = contractO<MODE>(O, 0, ep, zero);
    exchange(ex, buf, Wl, w, lane, W_, E_);
    buf ^= 1;
  };
  auto project = [&](const f4& xd, const f4& yd, const f4& th) {
    Trend Lx, Ly;
    const bf8 cxb = split_pos(cx, Lx), cyb = split_pos(cy, Ly), cpb = split(cp);
    const f4 x = plus_line(evalO<MODE>(O, 0, cx, cxb), Lx), y = plus_line(evalO<MODE>(O, 0, cy, cyb), Ly);
    const f4 xdd = evalO<MODE>(O, 2, cx, cxb), ydd = evalO<MODE>(O, 2, cy, cyb);
    const f4 psi = evalO<MODE>(O, 0, cp, cpb);
    SampleOut so;
    samples(K, xi, box, w, lane, q, gv, x, y, xd, yd, xdd, ydd, psi, th, so);
    ep = so.ep;
    racc[0] = so.r_obs;
    racc[1] = so.r_acc;
    racc[2] = so.r_nh;
    racc[3] = so.r_psi;
    f4 ax = contractO<MODE>(O, 0, so.sox, zero);
    ax = contractO<MODE>(O, 2, so.sax, ax);
    ax = contractO<MODE>(O, 1, so.ex, ax);
    f4 ay = contractO<MODE>(O, 0, so.soy, zero);
    ay = contractO<MODE>(O, 2, so.say, ay);
    ay = contractO<MODE>(O, 1, so.ey, ay);
    exchange(ex, buf, Wl, w, lane, ax, ay);
    buf ^= 1;
    ux = ax;
    uy = ay;
  };
  auto residuals = [&](f4& out) {
    f4 rr;
#pragma unroll
    for (int k = 0; k < 4; ++k) rr[k] = sum_rows(racc[k]);
    f4 dummy = zero;
    exchange(ex, buf, Wl, w, lane, rr, dummy);
    buf ^= 1;
    out = rr;
  };

  {
    f4 xd, yd, th, W_, E_;
    heading(xd, yd, th, W_, E_);
    if (cold) {
      if constexpr (MODE == TRAJ_MODE_FP32) cp = apply_psi(O.psi, c0p, rho * W_ + lp);
      else cp = apply_psi_split3(T, n, j, q, c0p, rho * W_ + lp);
    }
    project(xd, yd, th);
    ep = zero;  // the start has no pending heading multiplier step
  }
  int done = 0;
  bool stopped = false;
  for (int it = 0; it < A.iters; ++it) {
    // x/y step (eq. 12 through eq. 18)
    {
      // an offset the compiler cannot see through keeps the loop-invariant loads in the loop
      int opaque = 0;
      asm volatile("" : "+v"(opaque));
      if constexpr (MODE == TRAJ_MODE_FP32) {
        XYOps o;
        load_xy_ops(o, T64 + opaque, 0, j, q);
        cx = apply_xy(o, c0xd, cx, rho * ux + lx);
        load_xy_ops(o, T64 + opaque, 1, j, q);
        cy = apply_xy(o, c0yd, cy, rho * uy + ly);
      } else {
        cx = apply_xy_split3(T + opaque, n, 0, j, q, c0x, cx, rho * ux + lx);
        cy = apply_xy_split3(T + opaque, n, 1, j, q, c0y, cy, rho * uy + ly);
      }
    }
    // pending heading multiplier (eq. 24) and heading step (eq. 13 through eq. 20)
    f4 xd, yd, th, W_, E_;
    heading(xd, yd, th, W_, E_);
    lp = lp + rho * E_;
    if constexpr (MODE == TRAJ_MODE_FP32) cp = apply_psi(O.psi, c0p, rho * W_ + lp);
    else cp = apply_psi_split3(T, n, j, q, c0p, rho * W_ + lp);
    // v, (alpha, d), (alpha_a, d_a) and u~ (eqs. 14-16, 21, 22)
    project(xd, yd, th);
    // multipliers of the x/y block (eq. 23)
    lx = lx + rho * ux;
    ly = ly + rho * uy;
    done = it + 1;
    if (A.tol > 0.f && done % 5 == 0) {
      f4 rr;
      residuals(rr);
      // every goal of the group below tol (the group advances together)
      const float worst = sqrtf(worst_of(rr[0], rr[1], rr[2]));
      const bool ok = !gv || worst <= A.tol;
      if (__ballot(!ok) == 0ull) {
        stopped = true;
      }
      // the decision is identical in every wave (same totals), so the loop exits uniformly
      if (stopped) break;
    }
  }
  if (done > 0) {
    f4 E_ = contractO<MODE>(O, 0, ep, zero), dummy = zero;
    exchange(ex, buf, Wl, w, lane, E_, dummy);
    buf ^= 1;
    lp = lp + rho * E_;
  }
  f4 rr;
  residuals(rr);
  if (w == 0 && gv) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int k = 4 * q + r;
      if (k < NC) {
        A.c[(0 * NC + k) * NG + g] = cx[r];
        A.c[(1 * NC + k) * NG + g] = cy[r];
        A.c[(2 * NC + k) * NG + g] = cp[r];
        A.lam[(0 * NC + k) * NG + g] = lx[r];
        A.lam[(1 * NC + k) * NG + g] = ly[r];
        A.lam[(2 * NC + k) * NG + g] = lp[r];
      }
    }
    if (q == 0) {
      if (A.resid != nullptr)
        for (int k = 0; k < 4; ++k) A.resid[k * NG + g] = sqrtf(rr[k]);
      if (A.iters_out != nullptr) A.iters_out[g] = done;
    }
  }
}

}  // namespace

// The dynamic LDS the MFMA kernel may take is raised once per device, to the
// largest need seen, under a lock: setup reserves each handle's need, so the
// launches (which a caller may capture into a graph) make no attribute calls.
hipError_t mfma_reserve_smem(size_t smem) {
  static std::mutex lock;
  static int reserved[64] = {};  // bytes per device
  if (smem <= 65536 || smem > MFMA_SMEM_LIMIT) return hipSuccess;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> guard(lock);
  if (dev >= 0 && dev < 64 && (int)smem <= reserved[dev]) return hipSuccess;
  for (const void* fn : {(const void*)k_am_mfma<TRAJ_MODE_FP32>, (const void*)k_am_mfma<TRAJ_MODE_BF16X3>}) {
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
  }
  if (dev >= 0 && dev < 64) reserved[dev] = (int)smem;
  return hipSuccess;
}

size_t mfma_smem_bytes(int max_n, int max_m) {
  const int W = (max_n + TILE - 1) / TILE;
  const int mm = max_m > 0 ? max_m : 1;
  return sizeof(float2) * (size_t)mm * TILE * W + sizeof(float4) * (size_t)W * mm +
         sizeof(float4) * 2 * (size_t)W * 2 * WAVE;
}

hipError_t launch_solve_mfma(const SolveArgs& a, int mode, int G, int max_n, int max_m, hipStream_t stream) {
  if (a.n_goals <= 0) return hipSuccess;
  if (G < 1 || G > GCOLS) return hipErrorInvalidValue;
  const int W = (max_n + TILE - 1) / TILE;
  const int blocks = (a.n_goals + G - 1) / G + a.n_scenes;
  const size_t smem = mfma_smem_bytes(max_n, max_m);
  if (smem > MFMA_SMEM_LIMIT) return hipErrorInvalidValue;
  const void* fn = mode == TRAJ_MODE_BF16X3 ? (const void*)k_am_mfma<TRAJ_MODE_BF16X3>
                                            : (const void*)k_am_mfma<TRAJ_MODE_FP32>;
  if (smem > 65536) {
    hipError_t e = mfma_reserve_smem(smem);  // a no-op once setup has reserved it
    if (e != hipSuccess) return e;
  }
  if (mode == TRAJ_MODE_BF16X3)
    hipLaunchKernelGGL(k_am_mfma<TRAJ_MODE_BF16X3>, dim3(blocks), dim3(WAVE * W), smem, stream, a, G);
  else
    hipLaunchKernelGGL(k_am_mfma<TRAJ_MODE_FP32>, dim3(blocks), dim3(WAVE * W), smem, stream, a, G);
  return hipGetLastError();
}

}  // namespace traj
