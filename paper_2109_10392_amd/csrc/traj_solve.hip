// Batched alternating minimisation (Algorithm 1, Sec. III-D) on gfx950.
//
// Mapping: one goal per WPG wavefronts (1 or 2), lanes over time samples: wave w
// of a goal holds the samples lane + 64 (WPG s + w) of its S "slots". With one
// wave per goal a workgroup holds four goals of one scene; with two, a workgroup
// is one goal, and the two waves add their partial contractions through LDS
// after each reduction (in a fixed order, so both hold identical totals and take
// identical decisions). Each goal's iterate stays in registers for all
// iterations; nothing goes back to HBM until the end. Obstacle predictions are
// evaluated where needed from the scene's obstacles staged in LDS, pre-scaled by
// (1/a, 1/b).
//
// Per iteration, with c the coefficients of the previous x/y step:
//   x/y step (eq. 12 via eqs. 17-18). F^T g splits into a part linear in c and
//   the projection corrections, because the obstacle rows of g are
//   x + dx (d/du - 1), the acceleration rows x'' + s_a and the velocity rows
//   x' + (z - x'), with M, M_b blocks of the KKT inverse. The dense stacked F of
//   eq. 9 is never formed.
//   heading step (eq. 13 via eqs. 19-20): theta = atan2(y', x'),
//     c_psi = M_psi (rho P^T theta + lam_psi) + M_bpsi b_psi.
//   velocity (eq. 21), obstacle polar variables (eq. 22 and the 1-D minimiser of
//   eq. 15 clipped to d >= 1: d/du - 1 = max(0, 1/du - 1), du = |(dx/a, dy/b)|),
//   acceleration polar variables (eq. 16: d_a = min(a_max, |(x'', y'')|)).
//   multipliers (eq. 23): lam += rho F_ax^T (g - F_ax c) = rho u~ with
//   u~ = P^T s_o + P''^T s_a + P'^T (z - x'); (eq. 24, residual oriented as in
//   eq. 23): lam_psi += rho P^T (theta - psi). Both increments are contracted
//   from per-sample residuals, never as a difference of two large products
//   (P^T theta - P^T P c_psi): the multipliers integrate every iteration's
//   rounding, and the difference form makes FP32 drift well past 1e-4.
//   Correspondingly rho F^T g = (rho F_ax^T F_ax) c + rho u~, so the x/y step
//   is c_new = (M rho F_ax^T F_ax) c + M (rho u~ + lam) + M_b b.
// The contractions over time (P^T s, P^T theta) are lane-parallel products
// followed by a reduce-scatter across the wave (permlane swaps + DPP); the
// 11x11 applies run one output row per lane, their inputs and outputs broadcast
// through a per-wave LDS slot (one write by the home lanes, vector reads by all).
#include "traj_device.h"

namespace traj {
namespace {

using namespace dev;

constexpr int SOLVE_THREADS = WAVE * GOALS_PER_WG;

// Value slots of the two 32-way reductions (value v lands in lanes 2v, 2v+1).
// After the projections:
constexpr int R_UX = 0;     // u~_x[0..10]  -> lanes 2k
constexpr int R_OBS = 11;   // r_obs^2      -> lane 22
constexpr int R_ACC = 12;   // r_acc^2      -> lane 24
constexpr int R_NH = 13;    // r_nh^2       -> lane 26
constexpr int R_PSI = 14;   // r_psi^2      -> lane 28
constexpr int R_UY = 16;    // u~_y[0..10]  -> lanes 32 + 2k
// After the heading input:
constexpr int H_W = 0;      // P^T theta            -> lanes 2k
constexpr int H_E = 16;     // P^T (theta - psi) of the previous heading step -> lanes 32 + 2k

struct Goal {
  int n, m;
  float rho, a, b, inv_a, inv_b, a2, b2, vmin, vmax, amax, amax2, dt;
};

// Sum of one value per lane over the goal's two waves (fixed order), through a
// double-buffered LDS slot; every wave of the goal gets the same total.
__device__ __forceinline__ float pair_sum(float v, float* ex, int& buf) {
  const int lane = threadIdx.x & (WAVE - 1), wv = (threadIdx.x >> 6) & 1;
  ex[(buf * 2 + wv) * WAVE + lane] = v;
  __syncthreads();
  const float r = ex[(buf * 2 + 0) * WAVE + lane] + ex[(buf * 2 + 1) * WAVE + lane];
  buf ^= 1;
  return r;
}

// The home lanes' values of one coefficient vector: lane 2k (k < NC) holds value k
// of the lower set, lane 32 + 2k value k of the upper set. They are written to the
// wave's slot (lower set at [0, 16), upper set at [16, 32)).
__device__ __forceinline__ void put_home(float v, float* slot) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int k = (lane & 31) >> 1;
  if ((lane & 1) == 0 && k < NC) slot[(lane >> 5) * 16 + k] = v;
}

// The same in FP64: lane 2k (k < NC) writes value k of the lower set to slot[k],
// lane 32 + 2k value k of the upper set to slot[12 + k].
__device__ __forceinline__ void put_home64(double v, double* slot) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int k = (lane & 31) >> 1;
  if ((lane & 1) == 0 && k < NC) slot[(lane >> 5) * 12 + k] = v;
}

__device__ __forceinline__ void get_vec64(const double* slot, double (&v)[NC]) {
  const double2* s2 = reinterpret_cast<const double2*>(slot);
#pragma unroll
  for (int i = 0; i < NC / 2; ++i) {
    const double2 d = s2[i];
    v[2 * i] = d.x;
    v[2 * i + 1] = d.y;
  }
  v[NC - 1] = s2[NC / 2].x;
}

// The NC values at slot[0, NC) into registers (every lane reads the same words).
__device__ __forceinline__ void get_vec(const float* slot, float (&v)[NC]) {
  const float4* s4 = reinterpret_cast<const float4*>(slot);
  const float4 a = s4[0], b = s4[1], c = s4[2];
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  v[8] = c.x; v[9] = c.y; v[10] = c.z;
}

// Samples of a goal's WPG waves: wave w holds span = ceil(n / WPG) consecutive
// samples starting at w span, slot s the 64 of them from w span + 64 s (so the
// waves' shares, and their obstacle work, stay balanced).
__host__ __device__ inline int wave_span(int n, int wpg) { return (n + wpg - 1) / wpg; }
__host__ __device__ inline int slot_start(int n, int wpg, int w, int s) { return w * wave_span(n, wpg) + WAVE * s; }

// Basis rows of the lane's samples, their times, the lane's obstacle (scaled
// state) and each slot's culling boxes of it (one per row of 16 samples);
// loop-invariant, held in registers.
template <int S>
struct Lane {
  float P[S][NC], Pd[S][NC], Pdd[S][NC];
  float tm[S];
  float4 ob;
  int4 box[S][WAVE / 16];  // order keys of the box (x low, x high, y low, y high)
  bool val[S];
};

__device__ __forceinline__ float dotc(const float (&r)[NC], const float (&c)[NC]) {
  float acc = 0.f;
#pragma unroll
  for (int k = 0; k < NC; ++k) acc = fmaf(r[k], c[k], acc);
  return acc;
}

// Heading surrogate input (eq. 13): x', y', theta = atan2(y', x') per slot and the
// lane's share of P^T theta, plus P^T e_psi for the pending heading multiplier.
template <int S>
__device__ __forceinline__ void heading_input(const Lane<S>& L, const float (&cx)[NC], const float (&cy)[NC],
                                              const float (&ep)[S], float (&xd)[S], float (&yd)[S],
                                              float (&th)[S], float (&part)[32]) {
#pragma unroll
  for (int k = 0; k < 32; ++k) part[k] = 0.f;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    xd[s] = dotc(L.Pd[s], cx);
    yd[s] = dotc(L.Pd[s], cy);
    th[s] = atan2_heading(yd[s], xd[s]);
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      part[H_W + k] = fmaf(L.P[s][k], th[s], part[H_W + k]);
      part[H_E + k] = fmaf(L.P[s][k], ep[s], part[H_E + k]);
    }
  }
}

// Projections (eqs. 21, 22, 15, 16) at the current coefficients. Produces the
// lane's share of
//   u~ = P^T s_o + P''^T s_a + P'^T (z - x')   (per axis)
// where s_o, s_a are the obstacle and acceleration corrections g - F c of those
// rows and z = v (cos psi, sin psi): u~ = F_ax^T (g - F_ax c), the multiplier
// increment of eq. 23 divided by rho, formed from per-sample residuals. Also the
// squared residual components, and e_psi = theta - psi per slot for eq. 24.
template <int S, int WPG>
__device__ __forceinline__ void projections(const Goal& G, const Lane<S>& L, const float (&cx)[NC],
                                            const float (&cy)[NC], const float (&cp)[NC], const float (&xd)[S],
                                            const float (&yd)[S], const float (&th)[S], float (&ep)[S],
                                            float (&part)[32], float4* clist) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = (threadIdx.x >> 6) % WPG;
#pragma unroll
  for (int k = 0; k < 32; ++k) part[k] = 0.f;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int gs = WPG * s + wv;  // global slot of this wave's slot s
    const float x = dotc(L.P[s], cx), y = dotc(L.P[s], cy);
    const float xdd = dotc(L.Pdd[s], cx), ydd = dotc(L.Pdd[s], cy);
    const float psi = dotc(L.P[s], cp);
    // velocity, eq. 21 (the hardware square root, within 1 ulp; a denormal argument
    // reads as 0, a difference below 1.1e-19 that the clamp to v_min > 0 absorbs)
    const float v = fminf(fmaxf(__builtin_amdgcn_sqrtf(fmaf(xd[s], xd[s], yd[s] * yd[s])), G.vmin), G.vmax);
    float sn, cs;
    sincos_heading(psi, &sn, &cs);
    const float ex = fmaf(v, cs, -xd[s]), ey = fmaf(v, sn, -yd[s]);  // z - x'
    // acceleration polar variables, eq. 16: d_a = min(a_max, h), s_a = (x'', y'') (d_a / h - 1)
    const float h2 = fmaf(xdd, xdd, ydd * ydd);
    // (a_max >= 2^-63, so h2 > a_max^2 is a normal number: the hardware reciprocal
    // square root is the library's)
    const float fa = h2 > G.amax2 ? G.amax * __builtin_amdgcn_rsqf(h2) - 1.f : 0.f;
    const float sax = xdd * fa, say = ydd * fa;
    // obstacle polar variables, eqs. 15 and 22, in units scaled by (1/a, 1/b):
    // s_o = sum_j dx_j (d_j / du_j - 1), non-zero only inside an ellipse.
    // Culling at the time granularity of a DPP row (16 consecutive samples): an
    // obstacle is visited only if, for some row, its box over the row's time span
    // (inflated by the scaled half-axes plus 0.1%) meets the box of the row's
    // trajectory samples; for every other pair (x/a - xi_x)^2 + (y/b - xi_y)^2 > 1
    // holds in FP32 as well, so the result is exactly that of visiting all
    // obstacles. Whole slots (64 samples, 6.4 s) would let most obstacles of the
    // lanes a trajectory passes through into the loop.
    const float X = x * G.inv_a, Y = y * G.inv_b;
    // the row boxes in order keys (a strict float inequality implies the same one
    // between the keys, so no overlapping pair is lost)
    const int kx = order_key(X), ky = order_key(Y);
    constexpr int TOP = 0x7fffffff, BOTTOM = (int)0x80000000;
    const int xlo = row_min_i(L.val[s] ? kx : TOP), xhi = row_max_i(L.val[s] ? kx : BOTTOM);
    const int ylo = row_min_i(L.val[s] ? ky : TOP), yhi = row_max_i(L.val[s] ? ky : BOTTOM);
    // lane j tests obstacle j against each row's box: every lane stores its row's box
    // behind the wave's candidate list (all lanes, so that the last DPP step of the
    // row extremes stays fused), and every lane reads the four rows' first entries
    // back (same address per read: a broadcast). The previous reads of these words
    // fed the previous slot's candidate test, so they completed before these writes.
    int4* rbox = reinterpret_cast<int4*>(clist + CLIST);
    rbox[lane] = make_int4(xlo, xhi, ylo, yhi);
    wave_sync_lds();
    bool hit = false;
#pragma unroll
    for (int rw = 0; rw < WAVE / 16; ++rw) {
      const int4 rb = rbox[16 * rw];
      const int4 bx = L.box[s][rw];
      hit = hit | ((rb.y > bx.x) & (rb.x < bx.y) & (rb.w > bx.z) & (rb.z < bx.w));
    }
    // the candidates' scaled states, compacted in index order into the wave's list
    const int cnt = compact_candidates(hit && lane < G.m, L.ob, clist);
    const float tm = L.tm[s];
    float Sx = 0.f, Sy = 0.f, ro = 0.f;
    auto test4 = [&](const float4 (&o)[4]) {
      float tx[4], ty[4], qq[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        tx[u] = X - fmaf(o[u].z, tm, o[u].x);
        ty[u] = Y - fmaf(o[u].w, tm, o[u].y);
        qq[u] = fmaf(tx[u], tx[u], ty[u] * ty[u]);
      }
      if (fminf(fminf(qq[0], qq[1]), fminf(qq[2], qq[3])) < 1.f) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (qq[u] < 1.f) obstacle_inside(tx[u], ty[u], qq[u], G.a2, G.b2, Sx, Sy, ro);
        }
      }
    };
    // rounds of four in two alternating register sets: each round's reads are
    // issued before the previous round is tested (indices stay below cnt + 7)
    float4 oa[4], ob[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) oa[u] = clist[u];
    for (int c0 = 0; c0 < cnt; c0 += 8) {
#pragma unroll
      for (int u = 0; u < 4; ++u) ob[u] = clist[c0 + 4 + u];
      test4(oa);
      if (c0 + 4 >= cnt) break;
#pragma unroll
      for (int u = 0; u < 4; ++u) oa[u] = clist[c0 + 8 + u];
      test4(ob);
    }
    // the list is rewritten by the next slot or iteration: every lane's reads first
    wave_sync_lds();
    const float sox = G.a * Sx, soy = G.b * Sy;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      part[R_UX + k] = fmaf(L.P[s][k], sox, fmaf(L.Pdd[s][k], sax, fmaf(L.Pd[s][k], ex, part[R_UX + k])));
      part[R_UY + k] = fmaf(L.P[s][k], soy, fmaf(L.Pdd[s][k], say, fmaf(L.Pd[s][k], ey, part[R_UY + k])));
    }
    ep[s] = L.val[s] ? th[s] - psi : 0.f;
    if (L.val[s]) {
      part[R_OBS] += ro;
      part[R_ACC] += fmaf(sax, sax, say * say);
      part[R_NH] += fmaf(ex, ex, ey * ey);
      part[R_PSI] += ep[s] * ep[s];
    }
  }
}

// Per-wave LDS slots of solve_goal (floats): coefficient broadcast (x at [0, 16),
// y at [16, 32)), heading step input and output; then (doubles) the x/y step's
// operands in FP64: coefficients (x at [0, 12), y at [12, 24)) and right-hand
// sides (same layout).
constexpr int SLOT_C = 0, SLOT_P = 32, SLOT_Q = 48, SLOT_D = 64, SLOT_FLOATS = 160;

template <int S, int WPG>
__device__ void solve_goal(const SolveArgs& A, const ShapeDesc& sd, const float* __restrict__ T,
                           const float4* __restrict__ sobs, const float4* __restrict__ box, float* ex, float* slots,
                           float4* clist, int scene, int g) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = (threadIdx.x >> 6) % WPG;
  int buf = 0;
  // wave totals of a reduction (the pair's sum when a goal spans two waves)
  auto total = [&](float v) { return WPG == 2 ? pair_sum(v, ex, buf) : v; };
  const int NG = A.n_goals;
  Goal G;
  G.n = sd.n;
  G.m = sd.m;
  G.rho = A.k.rho;
  G.a = A.k.a;
  G.b = A.k.b;
  G.inv_a = 1.f / G.a;
  G.inv_b = 1.f / G.b;
  G.a2 = G.a * G.a;
  G.b2 = G.b * G.b;
  G.vmin = A.k.v_min;
  G.vmax = A.k.v_max;
  G.amax = A.k.a_max;
  G.amax2 = G.amax * G.amax;
  G.dt = sd.t_f / (float)(sd.n - 1);
  const float rho = G.rho;
  const int n = G.n;

  Lane<S> L;
  L.ob = lane < G.m ? sobs[lane] : make_float4(UNREACHABLE, UNREACHABLE, 0.f, 0.f);
  const int span = wave_span(n, WPG);
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int t = slot_start(n, WPG, wv, s) + lane;
    L.val[s] = WAVE * s + lane < span && t < n;
    const int tc = L.val[s] ? t : 0;
    L.tm[s] = (float)t * G.dt;
#pragma unroll
    for (int rw = 0; rw < WAVE / 16; ++rw) {
      const float4 b = box[((WPG * s + wv) * (WAVE / 16) + rw) * MAX_OBS + (lane < G.m ? lane : 0)];
      L.box[s][rw] = make_int4(order_key(b.x), order_key(b.y), order_key(b.z), order_key(b.w));
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      L.P[s][k] = L.val[s] ? T[tab_basis(n, 0) + k * n + tc] : 0.f;
      L.Pd[s][k] = L.val[s] ? T[tab_basis(n, 1) + k * n + tc] : 0.f;
      L.Pdd[s][k] = L.val[s] ? T[tab_basis(n, 2) + k * n + tc] : 0.f;
    }
  }
  // Home lanes: coefficient k of x lives in lanes 2k, 2k+1; of y and psi in 32+2k, 33+2k.
  // Every lane computes the rows of its index k for all three applies: x rows in the
  // lower half, y rows in the upper half, heading rows in both.
  const int k_home = min((lane & 31) >> 1, NC - 1);
  const bool upper = lane >= 32;
  // x/y step operators of the lane's axis and row in FP64 registers (loaded once),
  // heading operator row in FP32
  const double* T64 = A.tables64 + sd.table64_off;
  double rowMG[NC], rowM[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    rowMG[j] = T64[(upper ? T64_MGY : T64_MGX) + k_home * NC + j];
    rowM[j] = T64[(upper ? T64_MY : T64_MX) + k_home * NC + j];
  }
  float rMp[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) rMp[j] = T[tab_square(n, SQ_MP) + k_home * NC + j];
  // boundary values (eq. 8b) and the particular parts M_b b of each step
  const float* e = A.ego + 8 * scene;
  const float* gl = A.goal + 2 * g;
  const float bx[NX] = {e[0], e[2], e[4], gl[0]};
  const float by[NY] = {e[1], e[3], e[5], gl[1], 0.f, 0.f};
  const float bp[NP] = {e[6], e[7], 0.f, 0.f};
  const float* Bt = T + tab_bnd(n);
  double c0 = 0.0;  // particular part of the lane's axis and row
  float c0p = 0.f;
  if (!upper) {
#pragma unroll
    for (int j = 0; j < NX; ++j) c0 = fma(T64[T64_MBX + k_home * NX + j], (double)bx[j], c0);
  } else {
#pragma unroll
    for (int j = 0; j < NY; ++j) c0 = fma(T64[T64_MBY + k_home * NY + j], (double)by[j], c0);
  }
#pragma unroll
  for (int j = 0; j < NP; ++j) c0p = fmaf(Bt[BND_MBP + k_home * NP + j], bp[j], c0p);

  float* sC = slots + SLOT_C;  // coefficient broadcast
  float* sP = slots + SLOT_P;  // heading apply input
  float* sQ = slots + SLOT_Q;  // heading apply output
  double* sC64 = reinterpret_cast<double*>(slots + SLOT_D);  // x/y step operands in FP64
  double* sR64 = sC64 + 24;
  float cx[NC], cy[NC], cp[NC];
  // multipliers at their home lanes: lxy = lambda_x[k] (lower half) / lambda_y[k] (upper
  // half); lp = lambda_psi[k] (upper half)
  float lxy, lp;
  const bool cold = (A.flags & TRAJ_INIT_FROM_STATE) == 0;
  if (cold) {
    // boundary-only minimum-acceleration start, lambda = 0
    float v0 = 0.f;
    if (!upper) {
#pragma unroll
      for (int j = 0; j < NX; ++j) v0 = fmaf(Bt[BND_M0BX + k_home * NX + j], bx[j], v0);
    } else {
#pragma unroll
      for (int j = 0; j < NY; ++j) v0 = fmaf(Bt[BND_M0BY + k_home * NY + j], by[j], v0);
    }
    put_home(v0, sC);
    put_home64((double)v0, sC64);
    lxy = 0.f;
    lp = 0.f;
  } else {
    const float c_in = A.c[((upper ? 1 : 0) * NC + k_home) * NG + g];
    put_home(c_in, sC);
    put_home64((double)c_in, sC64);
    lxy = A.lam[((upper ? 1 : 0) * NC + k_home) * NG + g];
    lp = A.lam[(2 * NC + k_home) * NG + g];
  }
  wave_sync_lds();
  get_vec(sC, cx);
  get_vec(sC + 16, cy);
  if (cold) {
#pragma unroll
    for (int j = 0; j < NC; ++j) cp[j] = 0.f;
  } else {
#pragma unroll
    for (int j = 0; j < NC; ++j) cp[j] = A.c[(2 * NC + j) * NG + g];
  }

  // heading step (eq. 20) from rp = rho P^T theta + lambda_psi at the upper home lanes
  auto heading_step = [&](float rp) {
    if (upper) put_home(rp, sP - 16);  // upper set -> sP[0, NC)
    wave_sync_lds();
    float rv[NC];
    get_vec(sP, rv);
    float a0 = c0p, a1 = 0.f;
#pragma unroll
    for (int j = 0; j < NC; j += 2) a0 = fmaf(rMp[j], rv[j], a0);
#pragma unroll
    for (int j = 1; j < NC; j += 2) a1 = fmaf(rMp[j], rv[j], a1);
    if (upper) put_home(a0 + a1, sQ - 16);
    wave_sync_lds();
    get_vec(sQ, cp);
  };

  float uxy;  // u~_x[k] at lanes 2k, u~_y[k] at lanes 32+2k, residuals at lanes 22..28
  float part[32];
  float ep[S];
#pragma unroll
  for (int s = 0; s < S; ++s) ep[s] = 0.f;
  {
    // split variables of the starting point: heading QP (cold start only), v, (alpha, d),
    // (alpha_a, d_a). No multiplier is updated here.
    float xd[S], yd[S], th[S];
    heading_input<S>(L, cx, cy, ep, xd, yd, th, part);
    if (cold) {
      const float wE = total(reduce32<NC>(part));
      const float w = permlane_lo_to_hi(wE);  // P^T theta at lanes 32+2k
      heading_step(fmaf(rho, w, lp));
    }
    projections<S, WPG>(G, L, cx, cy, cp, xd, yd, th, ep, part, clist);
    uxy = total(reduce32<R_PSI + 1>(part));
#pragma unroll
    for (int s = 0; s < S; ++s) ep[s] = 0.f;  // the start has no pending heading multiplier step
  }

  int done = 0;
  for (int it = 0; it < A.iters; ++it) {
    // ---- x/y step (eq. 12 through eq. 18):
    // c_new = M (rho F^T g + lambda) + M_b b = (M rho F_ax^T F_ax) c + M (rho u~ + lambda) + M_b b
    // Each lane applies the row k_home of its half's axis in FP64 (four independent
    // accumulation chains), with the axis's c and r = rho u~ + lambda read back from LDS
    // (written there in FP64 by their home lanes: the FP32 values, widened once).
    {
      put_home64((double)fmaf(rho, uxy, lxy), sR64);
      wave_sync_lds();
      double rv[NC], cv[NC];
      get_vec64(sR64 + (upper ? 12 : 0), rv);
      get_vec64(sC64 + (upper ? 12 : 0), cv);
      double a0 = c0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
      for (int j = 0; j < NC; j += 2) {
        a0 = fma(rowMG[j], cv[j], a0);
        a1 = fma(rowM[j], rv[j], a1);
      }
#pragma unroll
      for (int j = 1; j < NC; j += 2) {
        a2 = fma(rowMG[j], cv[j], a2);
        a3 = fma(rowM[j], rv[j], a3);
      }
      const float cn = (float)((a0 + a2) + (a1 + a3));
      put_home(cn, sC);
      put_home64((double)cn, sC64);
      wave_sync_lds();
      get_vec(sC, cx);
      get_vec(sC + 16, cy);
    }
    // ---- pending heading multiplier (eq. 24 of the previous step) and heading step
    // (eq. 13 through eq. 20)
    float xd[S], yd[S], th[S];
    {
      heading_input<S>(L, cx, cy, ep, xd, yd, th, part);
      const float wE = total(reduce32<NC>(part));
      lp = fmaf(rho, wE, lp);                 // upper lanes: lambda_psi += rho P^T (theta - psi)
      const float w = permlane_lo_to_hi(wE);  // P^T theta at lanes 32+2k
      heading_step(fmaf(rho, w, lp));
    }
    // ---- v, (alpha, d), (alpha_a, d_a): eqs. 14-16, 21-22
    projections<S, WPG>(G, L, cx, cy, cp, xd, yd, th, ep, part, clist);
    uxy = total(reduce32<R_PSI + 1>(part));
    // ---- multipliers of the x/y block (eq. 23): lambda += rho F_ax^T (g - F_ax c)
    lxy = fmaf(rho, uxy, lxy);
    done = it + 1;
    if (A.tol > 0.f && done % 5 == 0) {
      const float worst = worst_of(rdlane(uxy, 2 * R_OBS), rdlane(uxy, 2 * R_ACC), rdlane(uxy, 2 * R_NH));
      if (sqrtf(worst) <= A.tol) break;
    }
  }
  if (done > 0) {
    // the heading multiplier step of the last iteration
#pragma unroll
    for (int k = 0; k < 32; ++k) part[k] = 0.f;
#pragma unroll
    for (int s = 0; s < S; ++s) {
#pragma unroll
      for (int k = 0; k < NC; ++k) part[H_E + k] = fmaf(L.P[s][k], ep[s], part[H_E + k]);
    }
    lp = fmaf(rho, total(reduce32<NC>(part)), lp);
  }

  if (WPG == 2 && wv != 0) return;  // the first wave of the goal writes
  // ---- write back from the home lanes
  const int k = (lane & 31) >> 1;
  if ((lane & 1) == 0 && k < NC) {
    float vx = 0.f, vy = 0.f, vp = 0.f;
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      if (j == k) {
        vx = cx[j];
        vy = cy[j];
        vp = cp[j];
      }
    }
    if (!upper) {
      A.c[(0 * NC + k) * NG + g] = vx;
      A.lam[(0 * NC + k) * NG + g] = lxy;
    } else {
      A.c[(1 * NC + k) * NG + g] = vy;
      A.lam[(1 * NC + k) * NG + g] = lxy;
      A.c[(2 * NC + k) * NG + g] = vp;
      A.lam[(2 * NC + k) * NG + g] = lp;
    }
  }
  if (A.resid != nullptr) {
    // residuals of the returned iterate (of the starting point when iters == 0)
    const float r_obs = rdlane(uxy, 2 * R_OBS), r_acc = rdlane(uxy, 2 * R_ACC);
    const float r_nh = rdlane(uxy, 2 * R_NH), r_psi = rdlane(uxy, 2 * R_PSI);
    if (lane < 4) {
      const float rr = lane == 0 ? r_obs : (lane == 1 ? r_acc : (lane == 2 ? r_nh : r_psi));
      A.resid[lane * NG + g] = sqrtf(rr);
    }
  }
  if (A.iters_out != nullptr && lane == 0) A.iters_out[g] = done;
}

template <int S, int WPG>
__global__ __launch_bounds__(SOLVE_THREADS) void k_am(SolveArgs A) {
  constexpr int GPW = WPG == 1 ? GOALS_PER_WG : 1;  // goals per workgroup
  constexpr int THREADS = WAVE * WPG * GPW;
  __shared__ float4 sobs[MAX_OBS];                  // the scene's obstacles, scaled by (1/a, 1/b)
  __shared__ float4 box[S * WPG * (WAVE / 16) * MAX_OBS];  // per slot, row of 16 samples and obstacle:
                                                          // x range, y range (scaled, inflated)
  __shared__ float ex[2 * 2 * WAVE];                // partial sums of a goal's two waves (double-buffered)
  __shared__ float4 slots4[GPW * WPG][SLOT_FLOATS / 4];  // each wave's broadcast slots
  __shared__ float4 clists[GPW * WPG][CLIST + WAVE];  // each wave's obstacle candidates, then its
                                                       // lanes' row boxes of the current slot
  __shared__ int sh[2];
  __shared__ int scan[GOALS_PER_WG];
  locate(A.goal_off, A.n_scenes, GPW, sh, scan, xcd_block((int)blockIdx.x, (int)gridDim.x));
  const int scene = sh[0];
  if (scene < 0) return;
  if (A.skip != nullptr && A.skip[scene] != 0) return;  // uniform: one scene per workgroup
  const int g0 = sh[1];
  if (g0 < 0) return;  // goal offsets out of contract: nothing to touch
  const int g1 = min(min(g0 + GPW, (int)A.goal_off[scene + 1]), A.n_goals);
  const int sid = A.shape_id[scene];
  const int o0 = A.obs_off[scene];
  const int m_scene = A.obs_off[scene + 1] - o0;
  bool bad = sid < 0 || sid >= A.n_shapes;
  ShapeDesc sd = {};
  if (!bad) sd = A.shapes[sid];
  bad = bad || !obstacles_ok(o0, m_scene, sd.m) || sd.n > WAVE * S * WPG || sd.n < NC;
  const int tid = threadIdx.x;
  const int g = g0 + (tid >> 6) / WPG;
  const bool writer = ((tid >> 6) % WPG) == 0;
  if (bad) {
    if (writer && A.resid != nullptr && g < g1 && (tid & 63) < 4)
      A.resid[(tid & 63) * A.n_goals + g] = __builtin_nanf("");
    if (writer && A.iters_out != nullptr && g < g1 && (tid & 63) == 0) A.iters_out[g] = 0;
    return;
  }
  const int n = sd.n, m = sd.m;
  const float dt = sd.t_f / (float)(n - 1);
  const float inv_a = 1.f / A.k.a, inv_b = 1.f / A.k.b;
  int obs_marked = 0;  // a non-finite obstacle state seen by this thread
  for (int j = tid; j < m; j += THREADS) {
    const float* o = A.obs + 4 * (o0 + j);
    obs_marked |= !all_finite(o, 4);
    sobs[j] = make_float4(o[0] * inv_a, o[1] * inv_b, o[2] * inv_a, o[3] * inv_b);
  }
  // Boxes per slot row (16 samples): the scaled prediction fma(v', t, p') is
  // monotone in the sample time, so its extremes over a row are at the row's
  // first and last sample (the same expression the projections evaluate).
  constexpr int ROWS = WAVE / 16;
  for (int e = tid; e < S * WPG * ROWS * m; e += THREADS) {
    const int gr = e / m, j = e - gr * m;  // gr = (WPG slot + wave) * ROWS + row
    const int gs = gr / ROWS, rw = gr - gs * ROWS;
    const int first = slot_start(n, WPG, gs % WPG, gs / WPG) + 16 * rw;
    const int i0 = min(first, n - 1), i1 = min(first + 15, n - 1);
    const float* o = A.obs + 4 * (o0 + j);
    const float px = o[0] * inv_a, py = o[1] * inv_b, vx = o[2] * inv_a, vy = o[3] * inv_b;
    const float t0 = (float)i0 * dt, t1 = (float)i1 * dt;
    const float xa = fmaf(vx, t0, px), xb = fmaf(vx, t1, px);
    const float ya = fmaf(vy, t0, py), yb = fmaf(vy, t1, py);
    constexpr float R = 1.001f;
    box[gr * MAX_OBS + j] = make_float4(fminf(xa, xb) - R, fmaxf(xa, xb) + R, fminf(ya, yb) - R, fmaxf(ya, yb) + R);
  }
  const bool scene_marked = __syncthreads_or(obs_marked) != 0 || !all_finite(A.ego + 8 * scene, 8);
  if (g >= g1) return;  // only with one wave per goal (a two-wave workgroup always has its goal)
  if (scene_marked || !all_finite(A.goal + 2 * g, 2)) {  // uniform over the goal's waves
    if (writer) write_marked_goal(A, g, tid & 63, WAVE);
    return;
  }
  solve_goal<S, WPG>(A, sd, A.tables + sd.table_off, sobs, box, ex,
                     reinterpret_cast<float*>(slots4[tid >> 6]), clists[tid >> 6], scene, g);
}

// Lane-layout check of the two reductions: in[R][64] -> out[64].
__global__ void k_debug_reduce(const float* in, float* out, int r) {
  const int lane = threadIdx.x;
  if (r == 32) {
    float v[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) v[i] = in[i * WAVE + lane];
    out[lane] = reduce32(v);
  } else {
    float v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = in[i * WAVE + lane];
    out[lane] = reduce16(v);
  }
}

__global__ void k_debug_atan2(const float* y, const float* x, float* out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = atan2_heading(y[i], x[i]);
}

}  // namespace

hipError_t launch_debug_atan2(const float* y, const float* x, float* out, int n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_debug_atan2, dim3((n + 255) / 256), dim3(256), 0, stream, y, x, out, n);
  return hipGetLastError();
}

hipError_t launch_debug_reduce(const float* in, float* out, int r, hipStream_t stream) {
  hipLaunchKernelGGL(k_debug_reduce, dim3(1), dim3(WAVE), 0, stream, in, out, r);
  return hipGetLastError();
}

hipError_t launch_solve(const SolveArgs& a, int max_n, int max_m, int waves, hipStream_t stream) {
  (void)max_m;
  if (a.n_goals <= 0) return hipSuccess;
  if (waves != 1 && waves != 2) return hipErrorInvalidValue;
  const int gpw = waves == 1 ? GOALS_PER_WG : 1;
  const int blocks = (a.n_goals + gpw - 1) / gpw + a.n_scenes;
  const int S = (max_n + WAVE * waves - 1) / (WAVE * waves);
  const dim3 block(WAVE * waves * gpw);
  if (waves == 1) {
    if (S <= 1) hipLaunchKernelGGL((k_am<1, 1>), dim3(blocks), block, 0, stream, a);
    else if (S == 2) hipLaunchKernelGGL((k_am<2, 1>), dim3(blocks), block, 0, stream, a);
    else hipLaunchKernelGGL((k_am<3, 1>), dim3(blocks), block, 0, stream, a);
  } else {
    if (S <= 1) hipLaunchKernelGGL((k_am<1, 2>), dim3(blocks), block, 0, stream, a);
    else hipLaunchKernelGGL((k_am<2, 2>), dim3(blocks), block, 0, stream, a);
  }
  return hipGetLastError();
}

}  // namespace traj
