// Road-attached frame (Sec. III, assumption 1): the optimisation is posed along
// the road's centre-line (x = arc length s, y = signed lateral offset d) and the
// trajectories are mapped back to the global frame. The centre-line is a chain
// of constant-curvature segments; every thread walks the chain in FP64 (start
// pose of each segment in closed form), so no table or scratch memory is used.
//   k_from_global    vehicle states: global -> road frame (closest centre-line point)
//   k_to_global      points (s, d) -> global position and centre-line heading
//   k_traj_global    each scene's chosen trajectory, sampled, -> global frame
#include <math.h>

#include "traj_frenet.h"
#include "traj_internal.h"

namespace traj {
int api_fail(int code, const char* fmt, ...);
int handle_view(void* handle, const ShapeDesc** shapes, const float** tables, int* n_shapes, float* a_max,
                float* ell_a, float* ell_b);
int handle_max_n(void* handle, int* max_n);
}

namespace {

using traj::NC;
using traj::ShapeDesc;

constexpr int MAX_SEG = 64;
constexpr double STRAIGHT_K = 1e-9;  // |curvature| below this: a straight segment

struct Road {
  int n;
  float len[MAX_SEG], kap[MAX_SEG];
  double x0, y0, th0;
};

// Pose of the centre-line at arc length u along a segment that starts at
// (px, py, th) with curvature k.
__device__ __forceinline__ void advance(double px, double py, double th, double k, double u, double& qx, double& qy,
                                        double& qth) {
  if (fabs(k) < STRAIGHT_K) {
    qx = px + u * cos(th);
    qy = py + u * sin(th);
    qth = th;
  } else {
    qth = th + k * u;
    qx = px + (sin(qth) - sin(th)) / k;
    qy = py - (cos(qth) - cos(th)) / k;
  }
}

struct Foot {
  double s, d, th, k, dist;
};

// Closest point of a segment (u in [0, L]; lo / hi open the half-lines that
// continue the first and the last segment).
__device__ Foot project(double px, double py, double th, double k, double L, double S, double x, double y, bool lo,
                        bool hi) {
  Foot f;
  const double tx = cos(th), ty = sin(th);
  if (fabs(k) < STRAIGHT_K) {
    double u = (x - px) * tx + (y - py) * ty;
    if (!lo) u = fmax(u, 0.0);
    if (!hi) u = fmin(u, L);
    const double fx = px + u * tx, fy = py + u * ty;
    f.s = S + u;
    f.th = th;
    f.k = 0.0;
    f.d = tx * (y - fy) - ty * (x - fx);
    f.dist = hypot(x - fx, y - fy);
    return f;
  }
  // arc: centre of curvature on the left normal at distance 1/k
  const double cx = px - ty / k, cy = py + tx / k;
  const double wx = x - cx, wy = y - cy;
  const double r = hypot(wx, wy);
  double al = atan2(wy, wx) - atan2(py - cy, px - cx);  // angle swept from the start, wrapped to (-pi, pi]
  if (al > M_PI) al -= 2.0 * M_PI;
  if (al <= -M_PI) al += 2.0 * M_PI;
  const double u = al / k;
  if (u >= 0.0 && u <= L) {
    f.s = S + u;
    f.th = th + k * u;
    f.k = k;
    f.d = 1.0 / k - (k > 0.0 ? r : -r);
    f.dist = fabs(f.d);
    return f;
  }
  // outside the arc's angular range: the nearer end point
  double ex, ey, eth;
  advance(px, py, th, k, L, ex, ey, eth);
  const double d0 = hypot(x - px, y - py), d1 = hypot(x - ex, y - ey);
  const bool at_end = d1 < d0;
  const double fx = at_end ? ex : px, fy = at_end ? ey : py, fth = at_end ? eth : th;
  f.s = S + (at_end ? L : 0.0);
  f.th = fth;
  f.k = k;
  f.d = cos(fth) * (y - fy) - sin(fth) * (x - fx);
  f.dist = at_end ? d1 : d0;
  return f;
}

__device__ Foot closest(const Road& R, double x, double y) {
  double px = R.x0, py = R.y0, th = R.th0, S = 0.0;
  Foot best;
  best.dist = __builtin_inf();
  best.s = best.d = best.th = best.k = 0.0;
  for (int i = 0; i < R.n; ++i) {
    const double L = R.len[i], k = R.kap[i];
    // the half-line before the start belongs to segment 0 (straight continuation)
    if (i == 0) {
      const Foot f = project(px, py, th, 0.0, 0.0, 0.0, x, y, true, false);
      if (f.dist < best.dist) best = f;
    }
    const Foot f = project(px, py, th, k, L, S, x, y, false, false);
    if (f.dist < best.dist) best = f;
    double qx, qy, qth;
    advance(px, py, th, k, L, qx, qy, qth);
    px = qx;
    py = qy;
    th = qth;
    S += L;
  }
  const Foot f = project(px, py, th, 0.0, 0.0, S, x, y, false, true);
  if (f.dist < best.dist) best = f;
  return best;
}

// Centre-line pose and curvature at arc length s (straight continuation outside).
__device__ void pose_at(const Road& R, double s, double& x, double& y, double& th, double& k) {
  double px = R.x0, py = R.y0, pth = R.th0, S = 0.0;
  if (s < 0.0) {
    advance(px, py, pth, 0.0, s, x, y, th);
    k = 0.0;
    return;
  }
  for (int i = 0; i < R.n; ++i) {
    const double L = R.len[i];
    if (s <= S + L || i == R.n - 1) {
      const double u = fmin(s - S, L);
      advance(px, py, pth, R.kap[i], u, x, y, th);
      k = R.kap[i];
      if (s - S > L) {  // beyond the end
        double ex = x, ey = y, eth = th;
        advance(ex, ey, eth, 0.0, s - S - L, x, y, th);
        k = 0.0;
      }
      return;
    }
    double qx, qy, qth;
    advance(px, py, pth, R.kap[i], L, qx, qy, qth);
    px = qx;
    py = qy;
    pth = qth;
    S += L;
  }
}

__global__ void k_from_global(Road R, int kind, int n, const float* in, float* out) {  // in may alias out
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int w = kind == 0 ? 4 : 8;
  double v[8];
  for (int q = 0; q < w; ++q) v[q] = in[(size_t)i * w + q];
  const Foot f = closest(R, v[0], v[1]);
  const double tx = cos(f.th), ty = sin(f.th);
  const double den = 1.0 - f.k * f.d;
  const bool ok = den > 0.0 && f.dist == f.dist;
  const double sd = ok ? (v[2] * tx + v[3] * ty) / den : __builtin_nan("");
  const double dd = ok ? (-v[2] * ty + v[3] * tx) : __builtin_nan("");
  double o[8];
  o[0] = f.s;
  o[1] = f.d;
  o[2] = sd;
  o[3] = dd;
  if (kind == 1) {
    const double at = v[4] * tx + v[5] * ty, an = -v[4] * ty + v[5] * tx;
    o[4] = ok ? (at + 2.0 * f.k * dd * sd) / den : __builtin_nan("");
    o[5] = ok ? an - f.k * den * sd * sd : __builtin_nan("");
    o[6] = v[6] - f.th;
    o[7] = ok ? v[7] - f.k * sd : __builtin_nan("");
  }
  for (int q = 0; q < w; ++q) out[(size_t)i * w + q] = (float)o[q];
}

__global__ void k_to_global(Road R, int n, const float* __restrict__ in, float* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double s = in[2 * (size_t)i], d = in[2 * (size_t)i + 1];
  double x, y, th, k;
  pose_at(R, s, x, y, th, k);
  out[3 * (size_t)i + 0] = (float)(x - d * sin(th));
  out[3 * (size_t)i + 1] = (float)(y + d * cos(th));
  out[3 * (size_t)i + 2] = (float)th;
}

struct TrajArgs {
  const int32_t* goal_off;
  const int32_t* shape_id;
  const ShapeDesc* shapes;
  const float* tables;
  const float* c;
  const int32_t* best;
  int n_shapes, n_scenes, n_goals, stride;
  float* out;
};

// One wavefront per scene, lanes over samples.
__global__ void k_traj_global(Road R, TrajArgs A) {
  const int s = blockIdx.x;
  if (s >= A.n_scenes) return;
  const int b = A.best[s];
  const int sid = A.shape_id[s];
  if (b < 0 || sid < 0 || sid >= A.n_shapes) return;
  const int g = A.goal_off[s] + b;
  if (g >= A.goal_off[s + 1] || g >= A.n_goals) return;
  const ShapeDesc sd = A.shapes[sid];
  const float* T = A.tables + sd.table_off;
  const int n = sd.n, NG = A.n_goals;
  for (int t = threadIdx.x; t < n && t < A.stride; t += blockDim.x) {
    double x = 0.0, y = 0.0, xd = 0.0, yd = 0.0;
    for (int k = 0; k < NC; ++k) {
      const double p = T[traj::tab_basis(n, 0) + k * n + t], q = T[traj::tab_basis(n, 1) + k * n + t];
      const double cx = A.c[(0 * NC + k) * NG + g], cy = A.c[(1 * NC + k) * NG + g];
      x = fma(p, cx, x);
      y = fma(p, cy, y);
      xd = fma(q, cx, xd);
      yd = fma(q, cy, yd);
    }
    double px, py, th, kk;
    pose_at(R, x, px, py, th, kk);
    float* o = A.out + ((size_t)s * A.stride + t) * 3;
    o[0] = (float)(px - y * sin(th));
    o[1] = (float)(py + y * cos(th));
    o[2] = (float)(th + atan2(yd, (1.0 - kk * y) * xd));
  }
}

int make_road(const traj_road* r, Road* R) {
  if (r == nullptr || r->seg == nullptr || r->n_seg < 1 || r->n_seg > MAX_SEG)
    return traj::api_fail(TRAJ_E_INVAL, "road: n_seg must be in [1, %d] and seg non-NULL", MAX_SEG);
  if (!(isfinite(r->x0) && isfinite(r->y0) && isfinite(r->theta0)))
    return traj::api_fail(TRAJ_E_INVAL, "road: start pose must be finite");
  R->n = r->n_seg;
  for (int i = 0; i < r->n_seg; ++i) {
    const float L = r->seg[2 * i], k = r->seg[2 * i + 1];
    if (!(isfinite(L) && L > 0.f && isfinite(k) && fabs((double)k * L) <= M_PI + 1e-9))
      return traj::api_fail(TRAJ_E_INVAL, "road: segment %d needs length > 0 and |curvature| length <= pi", i);
    R->len[i] = L;
    R->kap[i] = k;
  }
  for (int i = r->n_seg; i < MAX_SEG; ++i) R->len[i] = R->kap[i] = 0.f;
  R->x0 = r->x0;
  R->y0 = r->y0;
  R->th0 = r->theta0;
  return TRAJ_OK;
}

int launched(const char* what) {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? TRAJ_OK : traj::api_fail(TRAJ_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace

extern "C" {

int traj_road_from_global(const traj_road* road, int kind, int n, const float* in, float* out, void* stream) {
  Road R;
  int rc = make_road(road, &R);
  if (rc != TRAJ_OK) return rc;
  if ((kind != 0 && kind != 1) || n < 0 || (n > 0 && (in == nullptr || out == nullptr)))
    return traj::api_fail(TRAJ_E_INVAL, "traj_road_from_global: kind must be 0 or 1, n >= 0, arrays non-NULL");
  if (n == 0) return TRAJ_OK;
  hipLaunchKernelGGL(k_from_global, dim3((n + 127) / 128), dim3(128), 0, (hipStream_t)stream, R, kind, n, in, out);
  return launched("traj_road_from_global");
}

int traj_road_to_global(const traj_road* road, int n, const float* in, float* out, void* stream) {
  Road R;
  int rc = make_road(road, &R);
  if (rc != TRAJ_OK) return rc;
  if (n < 0 || (n > 0 && (in == nullptr || out == nullptr)))
    return traj::api_fail(TRAJ_E_INVAL, "traj_road_to_global: n >= 0 and arrays non-NULL");
  if (n == 0) return TRAJ_OK;
  hipLaunchKernelGGL(k_to_global, dim3((n + 127) / 128), dim3(128), 0, (hipStream_t)stream, R, n, in, out);
  return launched("traj_road_to_global");
}

int traj_trajectory_to_global(void* handle, const traj_batch* batch, const traj_state* state, const int32_t* best,
                              const traj_road* road, int stride, float* out, void* stream) {
  Road R;
  int rc = make_road(road, &R);
  if (rc != TRAJ_OK) return rc;
  TrajArgs A = {};
  float a_max, ea, eb;
  rc = traj::handle_view(handle, &A.shapes, &A.tables, &A.n_shapes, &a_max, &ea, &eb);
  if (rc != TRAJ_OK) return rc;
  if (batch == nullptr || state == nullptr || best == nullptr || out == nullptr || batch->n_scenes < 0 ||
      batch->n_goals < 0 || (batch->n_scenes > 0 && (batch->goal_off == nullptr || batch->shape_id == nullptr)) ||
      (batch->n_goals > 0 && state->c == nullptr))
    return traj::api_fail(TRAJ_E_INVAL, "traj_trajectory_to_global: NULL argument");
  int max_n = 0;
  if ((rc = traj::handle_max_n(handle, &max_n)) != TRAJ_OK) return rc;
  if (stride < max_n) return traj::api_fail(TRAJ_E_INVAL, "stride %d < longest n_time %d", stride, max_n);
  if (batch->n_scenes == 0) return TRAJ_OK;
  A.goal_off = batch->goal_off;
  A.shape_id = batch->shape_id;
  A.c = state->c;
  A.best = best;
  A.n_scenes = batch->n_scenes;
  A.n_goals = batch->n_goals;
  A.stride = stride;
  A.out = out;
  hipLaunchKernelGGL(k_traj_global, dim3(batch->n_scenes), dim3(64), 0, (hipStream_t)stream, R, A);
  return launched("traj_trajectory_to_global");
}

}  // extern "C"
