// Receding-horizon cycle on the GPU (the planner's use in Sec. IV: plan,
// execute the start of the chosen trajectory, plan again), for many episodes
// at once on straight roads:
//   k_mpc_goals      template goals from each ego's current state
//   k_mpc_obstacles  traffic one period ahead: Intelligent Driver Model
//                    (Treiber, Hennecke and Helbing 2000), each obstacle
//                    following the nearest vehicle ahead in its lane
//   k_mpc_ego        the ego one sample into its chosen trajectory (or a
//                    braking fallback when every goal was filtered), then the
//                    frame re-centred on the ego and collisions counted
//   k_mpc_shift      every goal's solution advanced by one period: the warm
//                    start of the next cycle.
// The period is one sample interval t_f / (n - 1) of the episode's shape.
#include "traj_internal.h"
#include "traj_mpc.h"

namespace traj {
int api_fail(int code, const char* fmt, ...);
}

namespace {

using traj::ShapeDesc;
using traj::NC;

struct MpcArgs {
  const int32_t* goal_off;
  const int32_t* obs_off;
  const int32_t* shape_id;
  const ShapeDesc* shapes;
  const float* tables;
  int n_shapes, n_scenes, n_goals, n_obs;
  const float* c;
  const int32_t* best;
  traj_episodes e;
  traj_mpc_params p;
  float a_max, ell_a, ell_b;
};

__device__ __forceinline__ float period(const MpcArgs& A, int s) {
  const int sid = A.shape_id[s];
  if (sid < 0 || sid >= A.n_shapes) return __builtin_nanf("");
  const ShapeDesc sd = A.shapes[sid];
  return sd.t_f / (float)(sd.n - 1);
}

__global__ void k_mpc_goals(MpcArgs A) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int per = A.p.n_lanes * A.p.per_lane;
  if (i >= (int64_t)A.n_scenes * per) return;
  const int s = (int)(i / per), slot = (int)(i - (int64_t)s * per);
  const int g0 = A.goal_off[s];
  if (A.goal_off[s + 1] - g0 != per || g0 + per > A.n_goals) return;
  const int sid = A.shape_id[s];
  if (sid < 0 || sid >= A.n_shapes) return;
  const float t_f = A.shapes[sid].t_f;
  const float* e = A.e.ego + 8 * s;
  float* g = A.e.goal + 2 * (g0 + slot);
  if (A.p.sampler == 1) {
    // right-lane sampler: about 60% of the goals on the right lane at different
    // distances, the rest over the other lanes at v_max t_f (Sec. III-F)
    const int n_r = (6 * per + 5) / 10, n_o = per - n_r, others = A.p.n_lanes - 1;
    int lane;
    float fr;
    if (slot < n_r || others == 0) {
      lane = 0;
      fr = n_r > 1 ? 0.2f + 0.8f * (float)min(slot, n_r - 1) / (float)(n_r - 1) : 1.f;
    } else {
      const int r = slot - n_r, per_o = (n_o + others - 1) / others;
      lane = 1 + r % others;
      fr = per_o > 1 ? 0.9f + 0.1f * (float)(r / others) / (float)(per_o - 1) : 1.f;
    }
    g[0] = fmaf(A.p.v_max * t_f, fr, e[0]);
    g[1] = (float)(lane - (A.p.n_lanes - 1) / 2) * A.p.lane_width;
    return;
  }
  const float v = fmaxf(sqrtf(fmaf(e[2], e[2], e[3] * e[3])), A.p.goal_v_floor);
  const int lane = slot / A.p.per_lane, k = slot - lane * A.p.per_lane;
  const float fr = A.p.per_lane > 1 ? 0.8f + 0.4f * (float)k / (float)(A.p.per_lane - 1) : 1.f;
  g[0] = fmaf(v * t_f, fr, e[0]);
  g[1] = (float)(lane - (A.p.n_lanes - 1) / 2) * A.p.lane_width;
}

__device__ __forceinline__ int episode_of(const int32_t* obs_off, int n_scenes, int o) {
  int lo = 0, hi = n_scenes - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (obs_off[mid] <= o)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ float idm_accel(const traj_mpc_params& p, float v, float v_des, float gap, float dv,
                                           bool free_road) {
  const float free = 1.f - powf(v / v_des, p.idm_delta);
  if (free_road) return p.idm_a * free;
  const float s_star = fmaxf(p.idm_s0 + v * p.idm_T + v * dv / (2.f * sqrtf(p.idm_a * p.idm_b)), 0.f);
  const float r = s_star / gap;
  return p.idm_a * (free - r * r);
}

// One thread per obstacle: its state one period ahead into obs_next.
__global__ void k_mpc_obstacles(MpcArgs A) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= A.n_obs) return;
  const int s = episode_of(A.obs_off, A.n_scenes, o);
  const int o0 = A.obs_off[s], o1 = A.obs_off[s + 1];
  const float dt = period(A, s);
  const float* me = A.e.obs + 4 * o;
  const float x = me[0], y = me[1], v = me[2];
  const float half = 0.5f * A.p.lane_width;
  // nearest vehicle ahead in the lane: the episode's other obstacles and its ego
  float lx = 0.f, lv = 0.f;
  bool found = false;
  for (int i = o0; i <= o1; ++i) {
    if (i == o) continue;
    const float* w = i < o1 ? A.e.obs + 4 * i : A.e.ego + 8 * s;
    if (!(fabsf(w[1] - y) < half) || !(w[0] > x)) continue;
    if (!found || w[0] < lx) {
      lx = w[0];
      lv = w[2];
      found = true;
    }
  }
  const float gap = fmaxf(lx - x - A.p.car_length, 0.1f);
  const float acc = idm_accel(A.p, v, A.e.v_des[o], gap, v - lv, !found);
  const float v_new = fmaxf(v + acc * dt, 0.f);
  float* out = A.e.obs_next + 4 * o;
  out[0] = x + 0.5f * (v + v_new) * dt;
  out[1] = y;
  out[2] = v_new;
  out[3] = me[3];
}

// One thread per episode: the ego one sample into its chosen trajectory, then
// the obstacles' new states committed in the frame re-centred on the ego.
__global__ void k_mpc_ego(MpcArgs A) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= A.n_scenes) return;
  const int sid = A.shape_id[s];
  if (sid < 0 || sid >= A.n_shapes) return;
  const ShapeDesc sd = A.shapes[sid];
  const float dt = sd.t_f / (float)(sd.n - 1);
  float* e = A.e.ego + 8 * s;
  const int b = A.best[s];
  const int g = A.goal_off[s] + b;
  float ne[8];
  if (b >= 0 && g < A.goal_off[s + 1] && g < A.n_goals) {
    const float* T = A.tables + sd.table_off;
    const int n = sd.n, NG = A.n_goals;
    for (int q = 0; q < 8; ++q) ne[q] = 0.f;
    for (int k = 0; k < NC; ++k) {
      const float p = T[traj::tab_basis(n, 0) + k * n + 1], pd = T[traj::tab_basis(n, 1) + k * n + 1],
                  pdd = T[traj::tab_basis(n, 2) + k * n + 1];
      const float cx = A.c[(0 * NC + k) * NG + g], cy = A.c[(1 * NC + k) * NG + g],
                  cp = A.c[(2 * NC + k) * NG + g];
      ne[0] = fmaf(p, cx, ne[0]);
      ne[1] = fmaf(p, cy, ne[1]);
      ne[2] = fmaf(pd, cx, ne[2]);
      ne[3] = fmaf(pd, cy, ne[3]);
      ne[4] = fmaf(pdd, cx, ne[4]);
      ne[5] = fmaf(pdd, cy, ne[5]);
      ne[6] = fmaf(p, cp, ne[6]);
      ne[7] = fmaf(pd, cp, ne[7]);
    }
  } else {
    // every goal filtered: brake along the road at a_max and stop moving
    // sideways (holding a lane change's heading would carry the ego into the
    // vehicle alongside)
    const float vx = fmaxf(e[2], 0.f);
    const float vx_new = fmaxf(vx - A.a_max * dt, 0.f);
    ne[0] = e[0] + 0.5f * (vx + vx_new) * dt;
    ne[1] = e[1];
    ne[2] = vx_new;
    ne[3] = 0.f;
    ne[4] = vx_new < vx ? -A.a_max : 0.f;
    ne[5] = 0.f;
    ne[6] = 0.f;
    ne[7] = 0.f;
    A.e.fallbacks[s] += 1;
  }
  const float shift = ne[0];
  ne[0] = 0.f;
  for (int q = 0; q < 8; ++q) e[q] = ne[q];
  A.e.travelled[s] += shift;
  A.e.shift[s] = shift;
  int hits = 0;
  for (int o = A.obs_off[s]; o < A.obs_off[s + 1]; ++o) {
    const float* src = A.e.obs_next + 4 * o;
    float* dst = A.e.obs + 4 * o;
    dst[0] = src[0] - shift;
    dst[1] = src[1];
    dst[2] = src[2];
    dst[3] = src[3];
    const float dx = dst[0] / A.ell_a, dy = (dst[1] - ne[1]) / A.ell_b;
    hits += fmaf(dx, dx, dy * dy) < 1.f;
  }
  A.e.collisions[s] += hits;
}

// Bernstein coefficients of degree NC-1 re-expressed on the interval shifted by
// u0 (the polar form of the polynomial at u0 and 1+u0):
//   S_ik = sum_q B(NC-1-i, k-q; u0) B(i, q; 1+u0),  B(n, j; u) = C(n, j) u^j (1-u)^(n-j).
// Entry e = i * NC + k. FP64: the terms alternate in sign for 1+u0 > 1.
__device__ double binom(int n, int j) {
  double r = 1.0;
  for (int m = 1; m <= j; ++m) r = r * (double)(n - j + m) / (double)m;
  return r;
}

__device__ double shift_entry(int e, double u0) {
  const int i = e / NC, k = e - i * NC, deg = NC - 1;
  const double a = u0, b = 1.0 + u0;
  double acc = 0.0;
  for (int q = 0; q <= i && q <= k; ++q) {
    const int p = k - q, na = deg - i;
    if (p > na) continue;
    double ta = binom(na, p), tb = binom(i, q);
    for (int r = 0; r < p; ++r) ta *= a;
    for (int r = 0; r < na - p; ++r) ta *= 1.0 - a;
    for (int r = 0; r < q; ++r) tb *= b;
    for (int r = 0; r < i - q; ++r) tb *= 1.0 - b;
    acc += ta * tb;
  }
  return acc;
}

// One workgroup per episode: S(u0) of the episode's shape in LDS, then every
// goal's coefficients of the three axes advanced (threads over goals; the
// goal-fastest layout makes each coefficient load and store coalesced). The
// multipliers stay as they are.
__global__ __launch_bounds__(256) void k_mpc_shift(MpcArgs A, float* c) {
  __shared__ float fwd[NC * NC];
  const int s = blockIdx.x;
  const int sid = A.shape_id[s];
  if (sid < 0 || sid >= A.n_shapes) return;
  const ShapeDesc sd = A.shapes[sid];
  const double u0 = 1.0 / (double)(sd.n - 1);
  const int t = threadIdx.x;
  if (t < NC * NC) fwd[t] = (float)shift_entry(t, u0);
  __syncthreads();
  const int g0 = max(A.goal_off[s], 0), g1 = min(A.goal_off[s + 1], A.n_goals);
  const float dx = A.e.shift[s];
  const int NG = A.n_goals;
  for (int g = g0 + t; g < g1; g += blockDim.x) {
    for (int ax = 0; ax < 3; ++ax) {
      float v[NC];
#pragma unroll
      for (int k = 0; k < NC; ++k) v[k] = c[(ax * NC + k) * NG + g];
#pragma unroll
      for (int i = 0; i < NC; ++i) {
        float cv = 0.f;
#pragma unroll
        for (int k = 0; k < NC; ++k) cv = fmaf(fwd[i * NC + k], v[k], cv);  // (S c)_i
        c[(ax * NC + i) * NG + g] = ax == 0 ? cv - dx : cv;
      }
    }
  }
}

bool params_ok(const traj_mpc_params* p) {
  return p != nullptr && p->idm_a > 0.f && p->idm_b > 0.f && p->idm_s0 >= 0.f && p->idm_T >= 0.f &&
         p->idm_delta > 0.f && p->car_length >= 0.f && p->lane_width > 0.f && p->n_lanes >= 1 && p->per_lane >= 1 &&
         p->goal_v_floor >= 0.f && (p->sampler == 0 || (p->sampler == 1 && p->v_max > 0.f));
}

}  // namespace

namespace traj {
// the handle's shape and operator tables and constants (traj_api.hip)
int handle_view(void* handle, const ShapeDesc** shapes, const float** tables, int* n_shapes, float* a_max,
                float* ell_a, float* ell_b);
}

namespace {

int fill(void* handle, const traj_batch* batch, MpcArgs* a) {
  int rc = traj::handle_view(handle, &a->shapes, &a->tables, &a->n_shapes, &a->a_max, &a->ell_a, &a->ell_b);
  if (rc != TRAJ_OK) return rc;
  if (batch->n_scenes < 0 || batch->n_goals < 0 || (batch->n_scenes > 0 && (!batch->goal_off || !batch->obs_off ||
                                                                           !batch->shape_id)))
    return traj::api_fail(TRAJ_E_INVAL, "batch arrays are NULL");
  a->goal_off = batch->goal_off;
  a->obs_off = batch->obs_off;
  a->shape_id = batch->shape_id;
  a->n_scenes = batch->n_scenes;
  a->n_goals = batch->n_goals;
  return TRAJ_OK;
}

}  // namespace

extern "C" {

int traj_mpc_goals(void* handle, const traj_batch* batch, const traj_episodes* eps, const traj_mpc_params* p,
                   void* stream) {
  if (batch == nullptr || eps == nullptr || !params_ok(p) || eps->ego == nullptr || eps->goal == nullptr)
    return traj::api_fail(TRAJ_E_INVAL, "traj_mpc_goals: bad arguments");
  MpcArgs a = {};
  int rc = fill(handle, batch, &a);
  if (rc != TRAJ_OK) return rc;
  a.e = *eps;
  a.p = *p;
  const int64_t n = (int64_t)batch->n_scenes * p->n_lanes * p->per_lane;
  if (n == 0) return TRAJ_OK;
  hipLaunchKernelGGL(k_mpc_goals, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, a);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? TRAJ_OK : traj::api_fail(TRAJ_E_HIP, "traj_mpc_goals: %s", hipGetErrorString(e));
}

int traj_mpc_step(void* handle, const traj_batch* batch, const traj_state* state, const int32_t* best,
                  const traj_episodes* eps, const traj_mpc_params* p, int n_obs, void* stream) {
  if (batch == nullptr || state == nullptr || state->c == nullptr || best == nullptr || eps == nullptr ||
      !params_ok(p) || eps->ego == nullptr || eps->obs == nullptr || eps->v_des == nullptr ||
      eps->obs_next == nullptr || eps->travelled == nullptr || eps->collisions == nullptr ||
      eps->fallbacks == nullptr || eps->shift == nullptr || n_obs < 0)
    return traj::api_fail(TRAJ_E_INVAL, "traj_mpc_step: bad arguments");
  MpcArgs a = {};
  int rc = fill(handle, batch, &a);
  if (rc != TRAJ_OK) return rc;
  a.c = state->c;
  a.best = best;
  a.e = *eps;
  a.p = *p;
  a.n_obs = n_obs;
  if (batch->n_scenes == 0) return TRAJ_OK;
  hipStream_t st = (hipStream_t)stream;
  if (n_obs > 0) hipLaunchKernelGGL(k_mpc_obstacles, dim3((n_obs + 255) / 256), dim3(256), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_mpc_ego, dim3((batch->n_scenes + 127) / 128), dim3(128), 0, st, a);
    e = hipGetLastError();
  }
  return e == hipSuccess ? TRAJ_OK : traj::api_fail(TRAJ_E_HIP, "traj_mpc_step: %s", hipGetErrorString(e));
}

int traj_mpc_shift(void* handle, const traj_batch* batch, traj_state* state, const traj_episodes* eps,
                   void* stream) {
  if (batch == nullptr || state == nullptr || state->c == nullptr || eps == nullptr || eps->shift == nullptr)
    return traj::api_fail(TRAJ_E_INVAL, "traj_mpc_shift: bad arguments");
  MpcArgs a = {};
  int rc = fill(handle, batch, &a);
  if (rc != TRAJ_OK) return rc;
  a.e = *eps;
  if (batch->n_scenes == 0 || batch->n_goals == 0) return TRAJ_OK;
  hipLaunchKernelGGL(k_mpc_shift, dim3(batch->n_scenes), dim3(256), 0, (hipStream_t)stream, a, state->c);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? TRAJ_OK : traj::api_fail(TRAJ_E_HIP, "traj_mpc_shift: %s", hipGetErrorString(e));
}

}  // extern "C"
