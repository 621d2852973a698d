// Meta-cost ranking (Sec. III-F): eq. 25 (cruise) or eq. 26 (high speed close
// to the right lane) per goal, the heading post-filter of Sec. III (assumption
// 2: discard |psi| beyond psi_max), optionally a collision post-check against
// the constant-velocity obstacle predictions (assumption 3), then the
// lowest-index argmin per scene.
#include "traj_internal.h"

namespace traj {
namespace {

constexpr int SCORE_THREADS = WAVE * GOALS_PER_WG;

// scene of a goal: largest s with goal_off[s] <= g
__device__ int scene_of(const int32_t* goal_off, int n_scenes, int g) {
  int lo = 0, hi = n_scenes - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (goal_off[mid] <= g)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Sixteen lanes per goal (a DPP row), four goals per wavefront: lane r of a
// goal's row takes the samples r, r + 16, ...; the row's partial sums, maxima and
// minima are combined by four DPP steps. Coefficients are read once per lane
// (the goal-fastest layout keeps them coalesced); the basis rows and obstacles
// are shared by the goals of a scene.
constexpr int COST_LANES = 16;
constexpr int COST_THREADS = 256;
constexpr int COST_GOALS = COST_THREADS / COST_LANES;
static_assert(COST_LANES == TILE_T, "a goal's lanes walk the packed tiles' sample rows");

template <int CTRL>
__device__ __forceinline__ float dpp_row(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
constexpr int DPP_XOR1 = 0xB1;         // quad_perm [1,0,3,2]
constexpr int DPP_XOR2 = 0x4E;         // quad_perm [2,3,0,1]
constexpr int DPP_HALF_MIRROR = 0x141;  // p <-> 7 - p within 8 lanes
constexpr int DPP_MIRROR = 0x140;       // p <-> 15 - p within 16 lanes

// combined over the 16 lanes of a row, result in every lane of the row
__device__ __forceinline__ float row_sum(float v) {
  v += dpp_row<DPP_XOR1>(v);
  v += dpp_row<DPP_XOR2>(v);
  v += dpp_row<DPP_HALF_MIRROR>(v);
  return v + dpp_row<DPP_MIRROR>(v);
}
__device__ __forceinline__ float row_max(float v) {
  v = fmaxf(v, dpp_row<DPP_XOR1>(v));
  v = fmaxf(v, dpp_row<DPP_XOR2>(v));
  v = fmaxf(v, dpp_row<DPP_HALF_MIRROR>(v));
  return fmaxf(v, dpp_row<DPP_MIRROR>(v));
}

// Obstacle predictions staged in LDS by a workgroup whose goals all belong to
// one scene (at most this many (obstacle, sample) pairs).
constexpr int PRED_MAX = 2048;

__global__ __launch_bounds__(COST_THREADS) void k_cost(ScoreArgs A) {
  const int r = threadIdx.x & (COST_LANES - 1);
  const int g = blockIdx.x * COST_GOALS + (int)(threadIdx.x / COST_LANES);
  // The collision post-check's predictions x_j + v_j t of each (obstacle, sample)
  // pair are the same for every goal of a scene: a workgroup whose goals share
  // one scene forms them once in LDS (the same fused multiply-adds, so the same
  // values). Decided per workgroup, before any thread leaves.
  __shared__ float2 spred[PRED_MAX];
  bool staged = false;
  if (A.clear_min > 0.f && A.n_goals > 0) {
    const int ga = blockIdx.x * COST_GOALS, gz = min(ga + COST_GOALS, A.n_goals) - 1;
    const int sa = scene_of(A.goal_off, A.n_scenes, ga);
    const int id = A.shape_id[sa];
    if (sa == scene_of(A.goal_off, A.n_scenes, gz) && id >= 0 && id < A.n_shapes &&
        !(A.skip != nullptr && A.skip[sa] != 0)) {
      const ShapeDesc sd = A.shapes[id];
      const int o0 = A.obs_off[sa], m = A.obs_off[sa + 1] - o0;
      if (obstacles_ok(o0, m, sd.m) && m * sd.n <= PRED_MAX) {
        const float dt = sd.t_f / (float)(sd.n - 1);
        for (int e = threadIdx.x; e < m * sd.n; e += COST_THREADS) {
          const int j = e / sd.n, t = e - j * sd.n;
          const float4 o = reinterpret_cast<const float4*>(A.obs)[o0 + j];
          const float tm = (float)t * dt;
          spred[e] = make_float2(fmaf(o.z, tm, o.x), fmaf(o.w, tm, o.y));
        }
        staged = true;
      }
    }
  }
  __syncthreads();
  if (g >= A.n_goals) return;  // whole rows leave together
  const int s = scene_of(A.goal_off, A.n_scenes, g);
  if (A.skip != nullptr && A.skip[s] != 0) return;
  const int sid = A.shape_id[s];
  if (sid < 0 || sid >= A.n_shapes) {
    if (r == 0) A.cost[g] = __builtin_nanf("");
    return;
  }
  const ShapeDesc sd = A.shapes[sid];
  const float* T = A.tables + sd.table_off;
  const int n = sd.n, NG = A.n_goals;
  float cx[NC], cy[NC], cp[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    cx[k] = A.c[(0 * NC + k) * NG + g];
    cy[k] = A.c[(1 * NC + k) * NG + g];
    cp[k] = A.c[(2 * NC + k) * NG + g];
  }
  const float vref = A.v_ref[s];
  const float yrl = (A.kind == 1 && A.y_rl != nullptr) ? A.y_rl[s] : 0.f;
  const bool check = A.clear_min > 0.f;
  const int o0 = check ? A.obs_off[s] : 0, m = check ? A.obs_off[s + 1] - o0 : 0;
  if (check && !obstacles_ok(o0, m, sd.m)) {  // the post-check cannot read this scene's obstacles
    if (r == 0) A.cost[g] = __builtin_nanf("");
    return;
  }
  const float dt = sd.t_f / (float)(n - 1);
  const float ia = 1.f / A.a, ib = 1.f / A.b;
  // the basis rows of sample t = 16 w + r from the packed tiles: P[t][4q .. 4q + 3]
  // at lane 16 q + r of tile w's slot 0, P' in slot 1 (zero past column NC), so a
  // sample takes six 16-byte reads from one address instead of 22 strided ones
  const float4* pk = reinterpret_cast<const float4*>(T + tab_pack(n));
  float acc = 0.f, pmax = 0.f, clear = __builtin_inff();
  for (int t = r, w = 0; t < n; t += COST_LANES, ++w) {
    const float4* row = pk + w * PACK_SLOTS * WAVE + r;
    float p[4 * 3], pd[4 * 3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const float4 a = row[16 * q], b = row[WAVE + 16 * q];
      p[4 * q] = a.x; p[4 * q + 1] = a.y; p[4 * q + 2] = a.z; p[4 * q + 3] = a.w;
      pd[4 * q] = b.x; pd[4 * q + 1] = b.y; pd[4 * q + 2] = b.z; pd[4 * q + 3] = b.w;
    }
    float xd = 0.f, yd = 0.f, x = 0.f, y = 0.f, psi = 0.f;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      xd = fmaf(pd[k], cx[k], xd);
      yd = fmaf(pd[k], cy[k], yd);
      x = fmaf(p[k], cx[k], x);
      y = fmaf(p[k], cy[k], y);
      psi = fmaf(p[k], cp[k], psi);
    }
    // squared scaled distance to every obstacle's constant-velocity prediction (eq. 1e)
    if (staged) {
      for (int j = 0; j < m; ++j) {
        const float2 pr = spred[j * n + t];
        const float dx = (x - pr.x) * ia, dy = (y - pr.y) * ib;
        clear = fminf(clear, fmaf(dx, dx, dy * dy));
      }
    } else {
      const float tm = (float)t * dt;
      for (int j = 0; j < m; ++j) {
        const float4 o = reinterpret_cast<const float4*>(A.obs)[o0 + j];
        const float dx = (x - fmaf(o.z, tm, o.x)) * ia, dy = (y - fmaf(o.w, tm, o.y)) * ib;
        clear = fminf(clear, fmaf(dx, dx, dy * dy));
      }
    }
    const float v = sqrtf(fmaf(xd, xd, yd * yd));
    const float dv = v - vref;
    if (A.kind == 0) {
      acc = fmaf(dv, dv, acc);
    } else {
      const float dy = y - yrl;
      acc = fmaf(A.w1 * dv, dv, fmaf(A.w2 * dy, dy, acc));
    }
    pmax = fmaxf(pmax, fabsf(psi));
  }
  acc = row_sum(acc);
  pmax = row_max(pmax);
  clear = -row_max(-clear);
  const bool hit = check && !(sqrtf(clear) >= A.clear_min);
  if (r == 0) A.cost[g] = (pmax > A.psi_max || hit) ? __builtin_inff() : acc;
}

// One workgroup per scene: lowest index attaining the minimum finite cost. In a
// chunked solve (C.done set) the same thread then applies the stopping rule to
// the scene: it adds the chunk's iterations and marks the scene converged when
// the residual max(r_obs, r_acc, r_nh) of its best goal is at or below tol (a
// scene whose goals are all filtered keeps iterating). Converged scenes are
// skipped from the start (A.skip is the same array).
__global__ __launch_bounds__(SCORE_THREADS) void k_argmin(ScoreArgs A, ConvergeCheck C) {
  __shared__ float sv[SCORE_THREADS / WAVE];
  __shared__ int si[SCORE_THREADS / WAVE];
  const int s = blockIdx.x;
  if (A.skip != nullptr && A.skip[s] != 0) return;
  const int g0 = A.goal_off[s], g1 = min((int)A.goal_off[s + 1], A.n_goals);
  if (g0 < 0) {  // goal offsets out of contract: no goal is read
    if (threadIdx.x == 0) A.best[s] = -1;
    return;
  }
  float best = __builtin_inff();
  int bi = 0x7fffffff;
  for (int g = g0 + (int)threadIdx.x; g < g1; g += SCORE_THREADS) {
    const float c = A.cost[g];
    if (isfinite(c) && (c < best || (c == best && g - g0 < bi))) {
      best = c;
      bi = g - g0;
    }
  }
#pragma unroll
  for (int d = WAVE / 2; d > 0; d >>= 1) {
    const float ov = __shfl_xor(best, d, WAVE);
    const int oi = __shfl_xor(bi, d, WAVE);
    if (ov < best || (ov == best && oi < bi)) {
      best = ov;
      bi = oi;
    }
  }
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & (WAVE - 1)) == 0) {
    sv[wv] = best;
    si[wv] = bi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < SCORE_THREADS / WAVE; ++w) {
      if (sv[w] < best || (sv[w] == best && si[w] < bi)) {
        best = sv[w];
        bi = si[w];
      }
    }
    const int b = (bi == 0x7fffffff) ? -1 : bi;
    A.best[s] = b;
    if (C.done != nullptr && C.done[s] == 0) {
      C.scene_iters[s] += C.iters;
      const int g = g0 + b;
      if (b >= 0 && g < A.n_goals) {
        const float worst =
            worst_of(C.resid[0 * A.n_goals + g], C.resid[1 * A.n_goals + g], C.resid[2 * A.n_goals + g]);
        if (worst <= C.tol) C.done[s] = 1;
      }
    }
  }
}

// Controls of the chosen trajectory of every scene and its clearance from the
// obstacles: one wavefront per scene, lanes over time samples. accel = v' =
// (x' x'' + y' y'') / v, steer = atan(psi' h / max(v, v_floor)) (the kinematic
// relation of Sec. III), clearance = min over samples and obstacles of
// sqrt((dx/a)^2 + (dy/b)^2) with constant-velocity predictions (< 1: inside an
// obstacle ellipse, eq. 1e).
__global__ void k_controls(ControlArgs A) {
  const int s = blockIdx.x;
  const int lane = threadIdx.x;
  if (s >= A.n_scenes) return;
  const int b = A.best[s];
  const int sid = A.shape_id[s];
  const int g0 = A.goal_off[s], g1 = A.goal_off[s + 1];
  const bool bad = sid < 0 || sid >= A.n_shapes || b < 0 || g0 < 0 || g0 + b >= g1 || g0 + b >= A.n_goals ||
                   !obstacles_ok(A.obs_off[s], A.obs_off[s + 1] - A.obs_off[s], A.shapes[sid].m);
  float* acc = A.accel + (size_t)s * A.stride;
  float* st = A.steer + (size_t)s * A.stride;
  if (bad) {
    if (lane == 0) A.clearance[s] = __builtin_nanf("");
    return;
  }
  const ShapeDesc sd = A.shapes[sid];
  const float* T = A.tables + sd.table_off;
  const int n = sd.n, NG = A.n_goals, g = g0 + b;
  const int o0 = A.obs_off[s], m = A.obs_off[s + 1] - o0;
  const float dt = sd.t_f / (float)(n - 1);
  float cx[NC], cy[NC], cp[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    cx[k] = A.c[(0 * NC + k) * NG + g];
    cy[k] = A.c[(1 * NC + k) * NG + g];
    cp[k] = A.c[(2 * NC + k) * NG + g];
  }
  float clear = __builtin_inff();
  for (int t = lane; t < n && t < A.stride; t += WAVE) {
    float x = 0.f, y = 0.f, xd = 0.f, yd = 0.f, xdd = 0.f, ydd = 0.f, pd = 0.f;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const float p = T[tab_basis(n, 0) + k * n + t], q = T[tab_basis(n, 1) + k * n + t],
                  r = T[tab_basis(n, 2) + k * n + t];
      x = fmaf(p, cx[k], x);
      y = fmaf(p, cy[k], y);
      xd = fmaf(q, cx[k], xd);
      yd = fmaf(q, cy[k], yd);
      xdd = fmaf(r, cx[k], xdd);
      ydd = fmaf(r, cy[k], ydd);
      pd = fmaf(q, cp[k], pd);
    }
    const float v = sqrtf(fmaf(xd, xd, yd * yd));
    acc[t] = v > 0.f ? fmaf(xd, xdd, yd * ydd) / v : 0.f;
    st[t] = atanf(pd * A.wheelbase / fmaxf(v, A.v_floor));
    const float tm = (float)t * dt;
    for (int j = 0; j < m; ++j) {
      const float* o = A.obs + 4 * (o0 + j);
      const float dx = (x - fmaf(o[2], tm, o[0])) / A.a, dy = (y - fmaf(o[3], tm, o[1])) / A.b;
      clear = fminf(clear, sqrtf(fmaf(dx, dx, dy * dy)));
    }
  }
#pragma unroll
  for (int d = WAVE / 2; d > 0; d >>= 1) clear = fminf(clear, __shfl_xor(clear, d, WAVE));
  if (lane == 0) A.clearance[s] = clear;
}

__global__ void k_converge_reset(int32_t* done, int32_t* scene_iters, int n_scenes) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n_scenes) {
    done[s] = 0;
    scene_iters[s] = 0;
  }
}

}  // namespace

hipError_t launch_controls(const ControlArgs& a, hipStream_t stream) {
  if (a.n_scenes <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_controls, dim3(a.n_scenes), dim3(WAVE), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_converge_reset(int32_t* done, int32_t* scene_iters, int n_scenes, hipStream_t stream) {
  if (n_scenes <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_converge_reset, dim3((n_scenes + 255) / 256), dim3(256), 0, stream, done, scene_iters,
                     n_scenes);
  return hipGetLastError();
}

hipError_t launch_score(const ScoreArgs& a, int max_n, hipStream_t stream, const ConvergeCheck* check) {
  (void)max_n;
  if (a.n_goals > 0) {
    const int blocks = (a.n_goals + COST_GOALS - 1) / COST_GOALS;
    hipLaunchKernelGGL(k_cost, dim3(blocks), dim3(COST_THREADS), 0, stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const ConvergeCheck none = {};
  if (a.n_scenes > 0)
    hipLaunchKernelGGL(k_argmin, dim3(a.n_scenes), dim3(SCORE_THREADS), 0, stream, a, check ? *check : none);
  return hipGetLastError();
}

}  // namespace traj
