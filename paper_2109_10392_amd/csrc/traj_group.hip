// Batched alternating minimisation (Algorithm 1, Sec. III-D) on the matrix
// cores, one wavefront per goal group.
//
// A wavefront owns up to 16 goals of one scene (the MFMA columns) and sweeps the
// time axis itself in 16-sample tiles, so no partial sum ever leaves the wave and
// there is no barrier in the iteration. Per iteration:
//   x/y step (eqs. 17-18)       c = MG c + M (rho u~ + lambda) + M_b b     f64 MFMA apply
//   heading sweep               per tile: x', y' (MFMA), theta = atan2, W += P^T theta
//   heading step (eqs. 19-20)   c_psi = M_psi (rho W + lambda_psi) + M_bpsi b_psi
//   projection sweep            per tile: x, y, x', y', x'', y'', psi (MFMA), the
//                               closed forms of eqs. 21, 22, 15, 16 (vector ALU),
//                               u~ += P^T s_o + P''^T s_a + P'^T (z - x') and
//                               E += P^T (theta - psi) (MFMA)
//   multipliers (eqs. 23, 24)   lambda += rho u~, lambda_psi += rho E
// The algebra is that of the other two kernels (reduced F^T g, increments
// contracted from per-sample residuals). A tile's basis operands are read from
// the packed per-shape table: one coalesced float4 per lane and matrix.
//
// Goal order. Within a scene the goals are ranked by final position (lateral,
// then longitudinal) and groups take 16 consecutive goals of that order, so the
// trajectories of a group stay close together and the box of a tile's samples,
// against which the obstacles are culled, stays small (on the dense highway
// scene about a quarter of the obstacles the index order leaves per tile).
//
// Uneven batches. The goal groups of a batch are listed by a one-workgroup list
// kernel in decreasing order of cost (16-sample tiles x (32 + obstacles)). The
// solver grid either takes them in list order, one per wavefront, or runs
// persistently: a grid that fits on the device at once, each wavefront claiming
// the next group from an atomic counter until the list is exhausted. Either way
// the most expensive groups start first and the cheapest fill the tail.
#include "traj_mma.h"

namespace traj {
namespace {

using namespace dev;
using namespace mma;

constexpr int GROUP_WAVES = 4;      // independent wavefronts per workgroup
constexpr int MAX_TILES = (MAX_TIME + TILE - 1) / TILE;
constexpr int LIST_THREADS = 1024;  // list kernel: one workgroup
constexpr int ORDER_THREADS = 1024; // goal-order kernel: one workgroup per scene
constexpr int COST_BUCKETS = 2048;  // cost keys n_tiles * (32 + m) <= 12 * 96

struct GroupArgs {
  int32_t* header;   // [0] claim counter, [1] groups listed
  int2* items;        // (scene, first position in the scene's goal order) per group, decreasing cost
  int32_t* perm;      // [n_goals]: goal index at each position of its scene's order
  int32_t* nvalid;    // [n_scenes]: goals of the scene that are solved (the first of its order)
  int capacity;       // entries of items
  int G;              // goals per group, 1..16
  int persistent;
};

__device__ __forceinline__ int group_cost(const SolveArgs& A, int scene) {
  const int sid = A.shape_id[scene];
  if (sid < 0 || sid >= A.n_shapes) return 0;
  const ShapeDesc sd = A.shapes[sid];
  const int n = min(max(sd.n, 0), MAX_TIME), m = min(max(sd.m, 0), MAX_OBS);
  return n_tiles(n) * (32 + m);
}

// Goals per group for the scenes of one shape: the shape's own size where set
// (the per-bucket autotuner's choice), else the tile's.
__device__ __forceinline__ int scene_group(const SolveArgs& A, const GroupArgs& L, int s) {
  const int sid = A.shape_id[s];
  const int gs = (sid >= 0 && sid < A.n_shapes) ? A.shapes[sid].group : 0;
  return (gs >= 1 && gs <= GCOLS) ? gs : L.G;
}

__device__ __forceinline__ void scene_goals(const SolveArgs& A, int s, int& g0, int& g1) {
  g0 = min(max((int)A.goal_off[s], 0), A.n_goals);
  g1 = min(max((int)A.goal_off[s + 1], g0), A.n_goals);
}

// Counting sort of the goal groups by decreasing cost; resets the claim counter.
// The order among groups of equal cost is unspecified (it does not change any
// result: the groups are independent).
__global__ __launch_bounds__(LIST_THREADS) void k_list(SolveArgs A, GroupArgs L) {
  __shared__ int hist[COST_BUCKETS];
  __shared__ int part[LIST_THREADS / WAVE];
  const int tid = threadIdx.x;
  for (int b = tid; b < COST_BUCKETS; b += LIST_THREADS) hist[b] = 0;
  __syncthreads();
  for (int s = tid; s < A.n_scenes; s += LIST_THREADS) {
    const int G = scene_group(A, L, s);
    const int cnt = (A.skip != nullptr && A.skip[s] != 0) ? 0 : (L.nvalid[s] + G - 1) / G;
    if (cnt > 0) atomicAdd(&hist[min(group_cost(A, s), COST_BUCKETS - 1)], cnt);
  }
  __syncthreads();
  // exclusive scan in decreasing key order: thread t owns keys 2t+1, 2t (descending
  // rank r = COST_BUCKETS - 1 - key)
  const int lane = tid & (WAVE - 1), wv = tid >> 6;
  const int k_hi = COST_BUCKETS - 1 - 2 * tid, k_lo = k_hi - 1;
  const int a = hist[k_hi], b = hist[k_lo];
  int incl = a + b;
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    const int y = __shfl_up(incl, d, WAVE);
    if (lane >= d) incl += y;
  }
  if (lane == WAVE - 1) part[wv] = incl;
  __syncthreads();
  int pre = 0, total = 0;
  for (int w = 0; w < LIST_THREADS / WAVE; ++w) {
    if (w < wv) pre += part[w];
    total += part[w];
  }
  const int excl = pre + incl - (a + b);
  __syncthreads();
  hist[k_hi] = excl;  // becomes the cursor of each bucket
  hist[k_lo] = excl + a;
  __syncthreads();
  for (int s = tid; s < A.n_scenes; s += LIST_THREADS) {
    int g0, g1;
    scene_goals(A, s, g0, g1);
    const int G = scene_group(A, L, s);
    const int cnt = (A.skip != nullptr && A.skip[s] != 0) ? 0 : (L.nvalid[s] + G - 1) / G;
    if (cnt <= 0) continue;
    int pos = atomicAdd(&hist[min(group_cost(A, s), COST_BUCKETS - 1)], cnt);
    for (int i = 0; i < cnt && pos < L.capacity; ++i, ++pos)
      L.items[pos] = make_int2(s, g0 + i * G);
  }
  if (tid == 0) {
    L.header[0] = 0;
    L.header[1] = min(total, L.capacity);
  }
}

// Total order on floats (NaN included) as unsigned keys.
__device__ __forceinline__ unsigned sort_key(float v) {
  const unsigned u = __builtin_bit_cast(unsigned, v);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Goal order of every scene: goals sorted by (y_f, x_f, index), in segments of
// ORDER_THREADS consecutive goals (a scene with more goals is ordered segment by
// segment). One workgroup per scene, bitonic sort of (key, index) pairs in LDS.
// Any permutation of a scene's goal range gives the same results; the order only
// makes the goals of a group close together.
//
// Inputs a solve cannot use are found here: a scene whose ego state (the
// boundary values of eq. 8b) or any obstacle state is not finite has every goal
// marked, a goal whose target is not finite is marked alone. The solved goals
// take the first nvalid positions of the scene's order and the marked ones the
// rest; a marked goal's outputs are written here (NaN coefficients, multipliers
// and residuals, zero iterations) and the solve never reaches it.
__global__ __launch_bounds__(ORDER_THREADS) void k_order(SolveArgs A, int32_t* __restrict__ perm,
                                                         int32_t* __restrict__ nvalid) {
  __shared__ unsigned long long key[ORDER_THREADS];
  __shared__ int idx[ORDER_THREADS];
  constexpr unsigned long long MARKED = 0xFFFFFFFF00000000ull;  // after every finite (y_f, x_f) key
  const int s = blockIdx.x;
  const int t = threadIdx.x;
  int g0, g1;
  scene_goals(A, s, g0, g1);
  int bad = t < 8 && !__builtin_isfinite(A.ego[8 * s + t]);
  // the obstacles are read only where the solve would read them (a known shape
  // with the scene's obstacle count; otherwise the solve marks the scene itself)
  const int sid = A.shape_id[s];
  const int o0 = A.obs_off[s], m_scene = A.obs_off[s + 1] - o0;
  if (sid >= 0 && sid < A.n_shapes && obstacles_ok(o0, m_scene, A.shapes[sid].m))
    for (int j = t; j < m_scene; j += ORDER_THREADS) bad |= !all_finite(A.obs + 4 * (o0 + j), 4);
  const bool scene_marked = __syncthreads_or(bad) != 0;
  auto solved = [&](int i) { return i < g1 && !scene_marked && all_finite(A.goal + 2 * i, 2); };
  int total = 0;
  for (int seg = g0; seg < g1; seg += ORDER_THREADS) total += __syncthreads_count(solved(seg + t));
  if (t == 0) nvalid[s] = total;
  int done_valid = 0, done_marked = 0;
  for (int seg = g0; seg < g1; seg += ORDER_THREADS) {
    const int cnt = min(ORDER_THREADS, g1 - seg);
    const int i = seg + t;
    const bool valid = t < cnt && solved(i);
    key[t] = valid ? (((unsigned long long)sort_key(A.goal[2 * i + 1]) << 32) | sort_key(A.goal[2 * i]))
                   : (t < cnt ? MARKED : ~0ull);
    idx[t] = t;
    const int seg_valid = __syncthreads_count(valid);
    for (int k = 2; k <= ORDER_THREADS; k <<= 1) {
      for (int jx = k >> 1; jx > 0; jx >>= 1) {
        const int l = t ^ jx;
        if (l > t) {
          const unsigned long long ka = key[t], kb = key[l];
          const int ia = idx[t], ib = idx[l];
          const bool a_gt = ka > kb || (ka == kb && ia > ib);
          if (a_gt == ((t & k) == 0)) {  // out of order for this half's direction
            key[t] = kb;
            key[l] = ka;
            idx[t] = ib;
            idx[l] = ia;
          }
        }
        __syncthreads();
      }
    }
    if (t < cnt) {
      const int pos = t < seg_valid ? g0 + done_valid + t : g0 + total + done_marked + (t - seg_valid);
      perm[pos] = seg + idx[t];
    }
    if (t < cnt && !valid) write_marked_goal(A, i, 0, 1);
    done_valid += seg_valid;
    done_marked += cnt - seg_valid;
    __syncthreads();
  }
}

struct GConsts {
  int n, m, nt;
  float rho, a, b, inv_a, inv_b, a2, b2, vmin, vmax, amax, amax2, dt, inv_tf;
};

template <int MODE>
__device__ __forceinline__ void to_operand(Operand<MODE>& o, const float4& v) {
  const float a[4] = {v.x, v.y, v.z, v.w};
  make_operand<MODE>(o, a);
}

// Validity of the lane's 4 samples of tile w and their sample times.
__device__ __forceinline__ void tile_rows(const GConsts& K, int w, int q, bool gv, bool (&tv)[4], float (&Tm)[4]) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = TILE * w + 4 * q + r;
    tv[r] = gv && i < K.n;
    Tm[r] = (float)i * K.dt;
  }
}

// Acceleration polar variables (eq. 16): d_a = min(a_max, h), h = |(x'', y'')|;
// s_a = (x'', y'') (d_a / h - 1) (zero where h <= a_max, including h = 0).
__device__ __forceinline__ void accel_forms(const GConsts& K, const bool (&tv)[4], const f4& xdd, const f4& ydd,
                                            f4& sax, f4& say, float& racc) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const float h2 = fmaf(xdd[r], xdd[r], ydd[r] * ydd[r]);
    // (a_max >= 2^-63, so h2 > a_max^2 is a normal number: the hardware reciprocal
    // square root is the library's)
    const float fa = (tv[r] && h2 > K.amax2) ? K.amax * __builtin_amdgcn_rsqf(h2) - 1.f : 0.f;
    sax[r] = xdd[r] * fa;
    say[r] = ydd[r] * fa;
    racc = fmaf(sax[r], sax[r], fmaf(say[r], say[r], racc));
  }
}

// Velocity (eq. 21) and the non-holonomic rows: z - x' with z = v (cos psi, sin psi);
// the heading residual theta - psi of eq. 24.
__device__ __forceinline__ void velocity_forms(const GConsts& K, const bool (&tv)[4], const f4& xd, const f4& yd,
                                               const f4& psi, const f4& th, f4& ex, f4& ey, f4& ep, float& r_nh,
                                               float& r_psi) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    // (the hardware square root, within 1 ulp; the clamp to v_min > 0 absorbs a
    // denormal argument read as 0)
    const float v = fminf(fmaxf(__builtin_amdgcn_sqrtf(fmaf(xd[r], xd[r], yd[r] * yd[r])), K.vmin), K.vmax);
    float sn, cs;
    sincos_heading(psi[r], &sn, &cs);
    ex[r] = tv[r] ? fmaf(v, cs, -xd[r]) : 0.f;
    ey[r] = tv[r] ? fmaf(v, sn, -yd[r]) : 0.f;
    ep[r] = tv[r] ? th[r] - psi[r] : 0.f;
    r_nh = fmaf(ex[r], ex[r], fmaf(ey[r], ey[r], r_nh));
    r_psi = fmaf(ep[r], ep[r], r_psi);
  }
}

// Obstacle polar variables (eqs. 15, 22) at the lane's 4 samples of tile w, in
// units scaled by (1/a, 1/b): s_o = sum_j dx_j (d_j / du_j - 1), non-zero only
// inside an ellipse. obs: the scene's obstacles in LDS as scaled (x, y, vx, vy).
// Only obstacles whose box over the tile's time span, inflated by the scaled
// half-axes plus 0.1%, meets the box of the tile's trajectory samples are
// visited: for every other pair the scaled distance exceeds 1 in FP32 too, so the
// result is that of visiting all obstacles. The boxes are compared as
// order-preserving integer keys (single-instruction DPP minima and maxima; a
// strict float inequality implies the same between keys), and the candidates'
// states are compacted, in index order, into the wave's list `clist`.
__device__ __forceinline__ void obstacle_forms(const GConsts& K, const float4* __restrict__ obs, float4* clist,
                                               int w, int lane, const bool (&tv)[4], const float (&Tm)[4],
                                               const f4& x, const f4& y, f4& sox, f4& soy, float& r_obs) {
  constexpr int TOP = 0x7fffffff, BOTTOM = (int)0x80000000;
  float X[4], Y[4];
  int lxlo = TOP, lxhi = BOTTOM, lylo = TOP, lyhi = BOTTOM;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    X[r] = x[r] * K.inv_a;
    Y[r] = y[r] * K.inv_b;
    const int kx = order_key(X[r]), ky = order_key(Y[r]);
    lxlo = tv[r] ? min(lxlo, kx) : lxlo;
    lxhi = tv[r] ? max(lxhi, kx) : lxhi;
    lylo = tv[r] ? min(lylo, ky) : lylo;
    lyhi = tv[r] ? max(lyhi, ky) : lyhi;
  }
  const int xlo = wave_min_i(lxlo), xhi = wave_max_i(lxhi), ylo = wave_min_i(lylo), yhi = wave_max_i(lyhi);
  bool hit = false;
  float4 ob = make_float4(UNREACHABLE, UNREACHABLE, 0.f, 0.f);
  if (lane < K.m) {
    // the scaled prediction is monotone in the sample time: its extremes over the
    // tile are at the first and last sample (same expression as below)
    ob = obs[lane];
    const int i0 = min(TILE * w, K.n - 1), i1 = min(TILE * w + TILE - 1, K.n - 1);
    const float t0 = (float)i0 * K.dt, t1 = (float)i1 * K.dt;
    const float xa = fmaf(ob.z, t0, ob.x), xb = fmaf(ob.z, t1, ob.x);
    const float ya = fmaf(ob.w, t0, ob.y), yb = fmaf(ob.w, t1, ob.y);
    constexpr float R = 1.001f;
    hit = (xhi > order_key(fminf(xa, xb) - R)) & (xlo < order_key(fmaxf(xa, xb) + R)) &
          (yhi > order_key(fminf(ya, yb) - R)) & (ylo < order_key(fmaxf(ya, yb) + R));
  }
  const int cnt = compact_candidates(hit, ob, clist);
  float Sx[4] = {0.f, 0.f, 0.f, 0.f}, Sy[4] = {0.f, 0.f, 0.f, 0.f};
  auto test1 = [&](const float4& o) {
    float tx[4], ty[4], qq[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      tx[r] = X[r] - fmaf(o.z, Tm[r], o.x);
      ty[r] = Y[r] - fmaf(o.w, Tm[r], o.y);
      qq[r] = tv[r] ? fmaf(tx[r], tx[r], ty[r] * ty[r]) : 2.f;
    }
    if (fminf(fminf(qq[0], qq[1]), fminf(qq[2], qq[3])) < 1.f) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (qq[r] < 1.f) obstacle_inside(tx[r], ty[r], qq[r], K.a2, K.b2, Sx[r], Sy[r], r_obs);
      }
    }
  };
  // rounds of two, their reads issued together (the padding keeps them in the list)
  for (int c0 = 0; c0 < cnt; c0 += 2) {
    const float4 o0 = clist[c0], o1 = clist[c0 + 1];
    test1(o0);
    test1(o1);
  }
  // the list is rewritten by the next tile: every lane's reads first
  wave_sync_lds();
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    sox[r] = K.a * Sx[r];
    soy[r] = K.b * Sy[r];
  }
}

template <int MODE>
__device__ void solve_group(const SolveArgs& A, const int32_t* __restrict__ perm, int G, int scene, int pos0,
                            int n_solved, int lane, float4* sobs, float4* sth, double* sc0, float4* clist) {
  const int j = lane & 15, q = lane >> 4;
  const int NG = A.n_goals;
  int s0, s1;
  scene_goals(A, scene, s0, s1);
  const int gcount = min(G, min(s1, s0 + n_solved) - pos0);
  if (gcount <= 0) return;
  const bool gv = j < gcount;
  const int g = perm[pos0 + (gv ? j : 0)];
  const int sid = A.shape_id[scene];
  const int o0 = A.obs_off[scene];
  const int m_scene = A.obs_off[scene + 1] - o0;
  bool bad = sid < 0 || sid >= A.n_shapes;
  ShapeDesc sd = {};
  if (!bad) sd = A.shapes[sid];
  bad = bad || !obstacles_ok(o0, m_scene, sd.m) || sd.n < NC || sd.n > MAX_TIME;
  if (bad) {
    if (gv && q == 0) {
      if (A.resid != nullptr)
        for (int k = 0; k < 4; ++k) A.resid[k * NG + g] = __builtin_nanf("");
      if (A.iters_out != nullptr) A.iters_out[g] = 0;
    }
    return;
  }
  GConsts K;
  K.n = sd.n;
  K.m = sd.m;
  K.nt = n_tiles(sd.n);
  K.dt = sd.t_f / (float)(sd.n - 1);
  K.inv_tf = 1.f / sd.t_f;
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
  const int n = K.n;
  const float rho = K.rho;
  const float* T = A.tables + sd.table_off;
  const double* T64 = A.tables64 + sd.table64_off;
  const float4* pk = reinterpret_cast<const float4*>(T + tab_pack(n));
  // the scene's obstacles into this wave's LDS slice (read back by other lanes of
  // the same wave only; the fence keeps the compiler from reordering across it)
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  if (lane < K.m) {
    const float4 o = reinterpret_cast<const float4*>(A.obs)[o0 + lane];
    sobs[lane] = make_float4(o.x * K.inv_a, o.y * K.inv_b, o.z * K.inv_a, o.w * K.inv_b);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  const float4* obs = sobs;

  // The apply operators (16 FP64 values per axis and lane) are read from the
  // tables (cache-resident) at each use instead of being held across the sweeps:
  // the addresses carry an offset the compiler cannot see through (an empty asm
  // statement), so the loop-invariant loads are not hoisted out of the loop.
  auto opaque_offset = []() {
    int opaque = 0;
    asm volatile("" : "+v"(opaque));
    return opaque;
  };
  auto xy_ops = [&](int axis) {
    XYOps o;
    load_xy_ops(o, T64 + opaque_offset(), axis, j, q);
    return o;
  };
  auto psi_ops = [&]() {
    PsiOps o;
    load_psi_ops(o, T + opaque_offset(), n, j, q);
    return o;
  };
  const f4 zero = {0.f, 0.f, 0.f, 0.f};
  f4 cx = zero, cy = zero, cp = zero, lx = zero, ly = zero, lp = zero;
  const bool cold = (A.flags & TRAJ_INIT_FROM_STATE) == 0;
  Particular P;
  particular<MODE>(T, T64, n, A.ego + 8 * scene, A.goal + 2 * g, q, P, cold, cx, cy);
  // the particular parts of the x/y step wait in LDS between applies ([axis][r][lane];
  // FP64 in the FP32 form, FP32 in the split form)
  float* sc0f = reinterpret_cast<float*>(sc0);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    if constexpr (MODE == TRAJ_MODE_FP32) {
      sc0[(0 * 4 + r) * WAVE + lane] = P.c0xd[r];
      sc0[(1 * 4 + r) * WAVE + lane] = P.c0yd[r];
    } else {
      sc0f[(0 * 4 + r) * WAVE + lane] = P.c0x[r];
      sc0f[(1 * 4 + r) * WAVE + lane] = P.c0y[r];
    }
  }
  auto c0d = [&](int axis) {
    d4 v;
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = sc0[(axis * 4 + r) * WAVE + lane];
    return v;
  };
  auto c0f = [&](int axis) {
    f4 v;
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = sc0f[(axis * 4 + r) * WAVE + lane];
    return v;
  };
  // the x/y step (eq. 18) and heading step (eq. 20) of one axis in the kernel's precision
  auto step_xy = [&](int axis, const f4& c, const f4& r) {
    if constexpr (MODE == TRAJ_MODE_FP32) return apply_xy(xy_ops(axis), c0d(axis), c, r);
    else return apply_xy_split3(T + opaque_offset(), n, axis, j, q, c0f(axis), c, r);
  };
  auto step_psi = [&](const f4& r) {
    if constexpr (MODE == TRAJ_MODE_FP32) return apply_psi(psi_ops(), P.c0p, r);
    else return apply_psi_split3(T + opaque_offset(), n, j, q, P.c0p, r);
  };
  if (!cold) {
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

  auto split = [&](const f4& v) -> bf8 {
    if constexpr (MODE == TRAJ_MODE_BF16X3) return split_b(v);
    else return bf8{};
  };
  // positions: split relative to the end-to-end line, which is added back after
  // each evaluation (value, first derivative; the second derivative has none)
  auto split_pos = [&](const f4& v, Trend& L) -> bf8 {
    if constexpr (MODE == TRAJ_MODE_BF16X3) {
      L = trend_of(v, j, K.inv_tf);
      return split_detrended(v, L, q);
    } else {
      L = Trend{0.f, 0.f, 0.f};
      return bf8{};
    }
  };
  auto plus_line = [&](f4 v, const Trend& L, const float (&t)[4]) {
    if constexpr (MODE == TRAJ_MODE_BF16X3) {
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] += fmaf(L.v, t[r], L.c0);
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
  // heading input: W = P^T theta, theta = atan2(y', x') at every sample; theta is
  // kept in this wave's LDS slice for the projection sweep that follows
  auto heading_sweep = [&]() -> f4 {
    Trend Lx, Ly;
    const bf8 cxb = split_pos(cx, Lx), cyb = split_pos(cy, Ly);
    f4 W = zero;
    float4 nd = pk[(0 * PACK_SLOTS + 1) * WAVE + lane], np = pk[(0 * PACK_SLOTS + 3) * WAVE + lane];
#pragma unroll 1
    for (int w = 0; w < K.nt; ++w) {
      const float4 vd = nd, vp = np;
      if (w + 1 < K.nt) {  // next tile's operands in flight while this one computes
        nd = pk[((w + 1) * PACK_SLOTS + 1) * WAVE + lane];
        np = pk[((w + 1) * PACK_SLOTS + 3) * WAVE + lane];
      }
      Operand<MODE> evd, ctp;
      to_operand<MODE>(evd, vd);
      to_operand<MODE>(ctp, vp);
      const f4 xd = plus_slope(eval<MODE>(evd, cx, cxb), Lx), yd = plus_slope(eval<MODE>(evd, cy, cyb), Ly);
      f4 th;
#pragma unroll
      for (int r = 0; r < 4; ++r) th[r] = (gv && TILE * w + 4 * q + r < n) ? atan2_heading(yd[r], xd[r]) : 0.f;
      sth[w * WAVE + lane] = f4to(th);
      W = contract<MODE>(ctp, th, W);
    }
    return W;
  };
  // projections at (cx, cy, cp): u~ per axis, E = P^T (theta - psi) and the
  // lane's squared residual partials (r_obs, r_acc, r_nh, r_psi). Each block's
  // per-sample values are contracted as soon as they exist.
  float racc[4];
  auto projection_sweep = [&](f4& ux, f4& uy, f4& E) {
    Trend Lx, Ly;
    const bf8 cxb = split_pos(cx, Lx), cyb = split_pos(cy, Ly), cpb = split(cp);
    ux = zero;
    uy = zero;
    E = zero;
#pragma unroll
    for (int k = 0; k < 4; ++k) racc[k] = 0.f;
    // operands of the current tile; each slot is refilled with the next tile's as
    // soon as it has been used, so the loads fly while the rest of the tile computes
    float4 op[PACK_SLOTS];
#pragma unroll
    for (int sl = 0; sl < PACK_SLOTS; ++sl) op[sl] = pk[sl * WAVE + lane];
#pragma unroll 1
    for (int w = 0; w < K.nt; ++w) {
      const bool more = w + 1 < K.nt;
      const float4* nxt = pk + (size_t)(w + 1) * PACK_SLOTS * WAVE + lane;
      bool tv[4];
      float Tm[4];
      tile_rows(K, w, q, gv, tv, Tm);
      Operand<MODE> ev, ct;
      {  // acceleration rows
        to_operand<MODE>(ev, op[2]);
        to_operand<MODE>(ct, op[5]);
        if (more) {
          op[2] = nxt[2 * WAVE];
          op[5] = nxt[5 * WAVE];
        }
        const f4 xdd = eval<MODE>(ev, cx, cxb), ydd = eval<MODE>(ev, cy, cyb);
        f4 sax, say;
        accel_forms(K, tv, xdd, ydd, sax, say, racc[1]);
        ux = contract<MODE>(ct, sax, ux);
        uy = contract<MODE>(ct, say, uy);
      }
      {  // velocity rows and the heading residual
        to_operand<MODE>(ev, op[1]);
        to_operand<MODE>(ct, op[4]);
        if (more) {
          op[1] = nxt[1 * WAVE];
          op[4] = nxt[4 * WAVE];
        }
        const f4 xd = plus_slope(eval<MODE>(ev, cx, cxb), Lx), yd = plus_slope(eval<MODE>(ev, cy, cyb), Ly);
        to_operand<MODE>(ev, op[0]);
        const f4 psi = eval<MODE>(ev, cp, cpb);
        const f4 th = tof4(sth[w * WAVE + lane]);
        f4 ex, ey, ep;
        velocity_forms(K, tv, xd, yd, psi, th, ex, ey, ep, racc[2], racc[3]);
        ux = contract<MODE>(ct, ex, ux);
        uy = contract<MODE>(ct, ey, uy);
        to_operand<MODE>(ct, op[3]);
        E = contract<MODE>(ct, ep, E);
      }
      {  // obstacle rows
        const f4 x = plus_line(eval<MODE>(ev, cx, cxb), Lx, Tm), y = plus_line(eval<MODE>(ev, cy, cyb), Ly, Tm);
        if (more) {
          op[0] = nxt[0 * WAVE];
          op[3] = nxt[3 * WAVE];
        }
        f4 sox, soy;
        obstacle_forms(K, obs, clist, w, lane, tv, Tm, x, y, sox, soy, racc[0]);
        ux = contract<MODE>(ct, sox, ux);
        uy = contract<MODE>(ct, soy, uy);
      }
    }
  };

  f4 ux, uy, E;
  // split variables of a starting point: heading QP (cold start only), v, (alpha,
  // d), (alpha_a, d_a); no multiplier is updated here
  auto start = [&](bool cold_start) {
    const f4 W = heading_sweep();
    if (cold_start) cp = step_psi(rho * W + lp);
    projection_sweep(ux, uy, E);
  };
  auto iteration = [&]() {
    // x/y step (eq. 12 through eq. 18)
    cx = step_xy(0, cx, rho * ux + lx);
    cy = step_xy(1, cy, rho * uy + ly);
    // heading step (eq. 13 through eq. 20)
    const f4 W = heading_sweep();
    cp = step_psi(rho * W + lp);
    // v, (alpha, d), (alpha_a, d_a), then the multipliers (eqs. 23, 24)
    projection_sweep(ux, uy, E);
    lx = lx + rho * ux;
    ly = ly + rho * uy;
    lp = lp + rho * E;
  };
  // max(r_obs, r_acc, r_nh) of the lane's goal at the last projection sweep
  auto worst_resid = [&]() {
    return sqrtf(worst_of(sum_rows(racc[0]), sum_rows(racc[1]), sum_rows(racc[2])));
  };
  auto store_state = [&]() {
    if (!gv) return;
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
  };
  auto load_state = [&]() {
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
  };

  start(cold);
  int done = 0;
  if (!cold && (A.flags & TRAJ_WARM_FALLBACK) != 0 && A.iters > 0) {
    // Cold start as fallback: one iteration from the given state and one from the
    // cold start; each goal keeps the one with the lower max(r_obs, r_acc, r_nh)
    // (a NaN residual loses). The warm result waits in the state arrays meanwhile.
    iteration();
    const float r_warm = worst_resid();
    store_state();
    lx = zero;
    ly = zero;
    lp = zero;
    cp = zero;
    particular<MODE>(T, T64, n, A.ego + 8 * scene, A.goal + 2 * g, q, P, true, cx, cy);
    start(true);
    iteration();
    const float r_cold = worst_resid();
    const bool warm = r_warm <= r_cold;
    if (warm && gv) load_state();
    // the next x/y step needs u~ (and the residuals) at the kept state: one more
    // projection sweep there reproduces them exactly (its E is not applied again)
    if (__ballot(warm && gv) != 0ull) projection_sweep(ux, uy, E);
    done = 1;
  }
#pragma unroll 1
  for (int it = done; it < A.iters; ++it) {
    iteration();
    done = it + 1;
    if (A.tol > 0.f && done % 5 == 0) {
      // every goal of the group at or below tol (the group advances together)
      if (__ballot(gv && !(worst_resid() <= A.tol)) == 0ull) break;
    }
  }
  float rr[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) rr[k] = sum_rows(racc[k]);
  store_state();
  if (gv) {
    if (q == 0) {
      if (A.resid != nullptr)
        for (int k = 0; k < 4; ++k) A.resid[k * NG + g] = sqrtf(rr[k]);
      if (A.iters_out != nullptr) A.iters_out[g] = done;
    }
  }
}

__device__ __forceinline__ int claim(int32_t* header) {
  int v = 0;
  if ((threadIdx.x & (WAVE - 1)) == 0) v = atomicAdd(header, 1);
  return __builtin_amdgcn_readfirstlane(v);
}

template <int MODE>
__global__ __launch_bounds__(WAVE * GROUP_WAVES, 2) void k_am_group(SolveArgs A, GroupArgs L) {
  __shared__ float4 sobs[GROUP_WAVES][MAX_OBS];           // each wave's current scene's obstacles (scaled)
  __shared__ float4 sclist[GROUP_WAVES][CLIST];           // each wave's obstacle candidates of a tile
  __shared__ float4 sth[GROUP_WAVES][MAX_TILES * WAVE];    // each wave's theta at its lanes' samples
  __shared__ double sc0[GROUP_WAVES][2 * 4 * WAVE];  // each wave's particular parts of the x/y step (FP64 in
                                                     // the FP32 form, FP32 in the split form)
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x >> 6;
  const int n_items = L.header[1];
  int idx = L.persistent ? claim(L.header) : (int)blockIdx.x * GROUP_WAVES + wv;
  // every wavefront leaves once the list is exhausted: the counter only grows
  while (idx < n_items) {
    const int2 it = L.items[idx];
    solve_group<MODE>(A, L.perm, scene_group(A, L, it.x), it.x, it.y, L.nvalid[it.x], lane, sobs[wv], sth[wv],
                      sc0[wv], sclist[wv]);
    idx = L.persistent ? claim(L.header) : n_items;
  }
}

}  // namespace

namespace {
// groups listed at most: sum_s ceil(goals_s / G) <= ceil(goals / G) + scenes
int64_t group_capacity(int n_scenes, int n_goals, int G) {
  if (G < 1) G = 1;
  return (int64_t)(n_goals + G - 1) / G + (int64_t)n_scenes;
}
}  // namespace

int64_t group_work_ints(int n_scenes, int n_goals, int G) {
  // header (4) | (scene, first position) per group | goal order [n_goals] | solved goals per scene
  return 4 + 2 * group_capacity(n_scenes, n_goals, G) + (int64_t)n_goals + (int64_t)n_scenes;
}

hipError_t group_blocks_per_cu(int mode, int* blocks) {
  const void* fn = mode == TRAJ_MODE_BF16X3 ? (const void*)k_am_group<TRAJ_MODE_BF16X3>
                                            : (const void*)k_am_group<TRAJ_MODE_FP32>;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, fn, WAVE * GROUP_WAVES, 0);
}

hipError_t launch_solve_group(const SolveArgs& a, int mode, int G, int G_min, bool persistent, int resident_blocks,
                              int32_t* work, bool reuse_order, hipStream_t stream) {
  if (a.n_goals <= 0) return hipSuccess;
  if (G < 1 || G > GCOLS || G_min < 1 || G_min > G || work == nullptr) return hipErrorInvalidValue;
  // every scene's groups hold at least G_min goals (but the last): the list fits
  const int64_t cap64 = group_capacity(a.n_scenes, a.n_goals, G_min);
  if (cap64 > (int64_t)1 << 29) return hipErrorInvalidValue;
  GroupArgs L;
  L.header = work;
  L.items = reinterpret_cast<int2*>(work + 4);
  L.perm = work + 4 + 2 * cap64;
  L.nvalid = L.perm + a.n_goals;
  L.capacity = (int)cap64;
  L.G = G;
  L.persistent = persistent ? 1 : 0;
  hipError_t e;
  if (!reuse_order) {
    hipLaunchKernelGGL(k_order, dim3(a.n_scenes), dim3(ORDER_THREADS), 0, stream, a, L.perm, L.nvalid);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_list, dim3(1), dim3(LIST_THREADS), 0, stream, a, L);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  int64_t blocks = (cap64 + GROUP_WAVES - 1) / GROUP_WAVES;
  if (persistent && resident_blocks > 0 && blocks > resident_blocks) blocks = resident_blocks;
  if (mode == TRAJ_MODE_BF16X3)
    hipLaunchKernelGGL(k_am_group<TRAJ_MODE_BF16X3>, dim3((unsigned)blocks), dim3(WAVE * GROUP_WAVES), 0, stream, a,
                       L);
  else
    hipLaunchKernelGGL(k_am_group<TRAJ_MODE_FP32>, dim3((unsigned)blocks), dim3(WAVE * GROUP_WAVES), 0, stream, a, L);
  return hipGetLastError();
}

}  // namespace traj
