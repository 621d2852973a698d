// C-ABI of libtraj: argument validation, handle ownership, kernel launches.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "traj_internal.h"

namespace traj {
hipError_t launch_debug_reduce(const float* in, float* out, int r, hipStream_t stream);
hipError_t launch_debug_atan2(const float* y, const float* x, float* out, int n, hipStream_t stream);
// raises the MFMA kernel's dynamic LDS on the current device (once per need; takes a lock)
hipError_t mfma_reserve_smem(size_t smem);
}

namespace {

using traj::ShapeDesc;

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

}  // namespace

namespace traj {
// error reporting for the entry points defined in other translation units
int api_fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}
}  // namespace traj

namespace {

int hip_fail(hipError_t e, const char* what) {
  return fail(TRAJ_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace

// Library-owned scratch of traj_solve_batch_noalloc: the group kernel's work list
// (claim counter, cost-sorted goal groups, goal order per scene, solved goals per
// scene). Every GPU the library runs on holds its own copy until the process ends.
// Host code never passes the array's name to a kernel: it uses the device address
// that resolve_scratch() takes once per device (at setup) and keeps.
static __device__ __align__(256) int32_t scratch[TRAJ_NOALLOC_WORK_INTS];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
int32_t* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on device `dev`, which must be the current device.
// Resolved on the first call for that device and kept.
hipError_t resolve_scratch(int dev, int32_t** out) {
  *out = nullptr;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (p == nullptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = static_cast<int32_t*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

struct Handle {
  traj_params p;
  std::vector<ShapeDesc> shapes;
  ShapeDesc* d_shapes = nullptr;
  float* d_tables = nullptr;
  double* d_tables64 = nullptr;
  int max_n = 0, max_m = 0;
  size_t table_floats = 0;
  traj_tile tile = {(int32_t)TRAJ_KERNEL_WAVE, 16, 1, 1};
  int resident_blocks[2] = {0, 0};  // group kernel workgroups resident at once, per precision mode
  int device = -1;                  // the device current at setup (tables and scratch live there)
  int32_t* scratch = nullptr;       // that device's address of the no-allocation scratch
};

bool finite_pos(float v) { return isfinite(v) && v > 0.f; }

// Smallest goals-per-group of the group kernel over the handle's shapes (a shape
// without its own size takes the tile's): sizes the group kernel's work list.
int min_group(const Handle* h) {
  int g = h->tile.group;
  for (const ShapeDesc& s : h->shapes)
    if (s.group >= 1 && s.group < g) g = s.group;
  return g;
}

traj::SolverConst consts(const traj_params& p) {
  traj::SolverConst k;
  k.rho = p.rho;
  k.a = p.a;
  k.b = p.b;
  k.v_min = p.v_min;
  k.v_max = p.v_max;
  k.a_max = p.a_max;
  k.psi_max = p.psi_max;
  return k;
}

int check_batch(const Handle* h, const traj_batch* b) {
  if (b == nullptr) return fail(TRAJ_E_INVAL, "batch is NULL");
  if (b->n_scenes < 0 || b->n_goals < 0) return fail(TRAJ_E_INVAL, "negative batch size");
  if (b->n_scenes == 0 && b->n_goals > 0) return fail(TRAJ_E_INVAL, "goals without scenes");
  if (b->n_goals == 0 && b->n_scenes == 0) return TRAJ_OK;
  if (!b->goal_off || !b->obs_off || !b->shape_id || !b->ego || !b->goal)
    return fail(TRAJ_E_INVAL, "batch has a NULL device array");
  if (h->max_m > 0 && b->obs == nullptr) return fail(TRAJ_E_INVAL, "batch.obs is NULL");
  return TRAJ_OK;
}

int solve_impl(Handle* h, const traj_batch* batch, traj_state* state, int iters, float tol, uint32_t flags,
               void* stream, bool reuse_order, int32_t* static_work = nullptr);
int score_impl(Handle* h, const traj_batch* batch, const traj_state* state, const traj_metacost* mc, float* cost,
               int32_t* best, void* stream, const int32_t* skip = nullptr,
               const traj::ConvergeCheck* check = nullptr);

}  // namespace

extern "C" {

const char* traj_last_error(void) { return g_err.c_str(); }

int traj_setup(const traj_params* params, const traj_shape* shapes, int n_shapes, void* stream, void** handle_out) {
  g_err.clear();
  if (params == nullptr || shapes == nullptr || handle_out == nullptr)
    return fail(TRAJ_E_INVAL, "traj_setup: NULL argument");
  *handle_out = nullptr;
  const traj_params& p = *params;
  if (p.n_coef != TRAJ_N_COEF) return fail(TRAJ_E_INVAL, "n_coef must be %d (got %d)", TRAJ_N_COEF, p.n_coef);
  if (!finite_pos(p.rho) || !finite_pos(p.a) || !finite_pos(p.b) || !finite_pos(p.v_min) || !finite_pos(p.v_max) ||
      !finite_pos(p.a_max) || !finite_pos(p.psi_max))
    return fail(TRAJ_E_INVAL, "parameters must be finite and positive");
  if (p.v_min > p.v_max) return fail(TRAJ_E_INVAL, "v_min > v_max");
  // the acceleration projection's reciprocal square root needs a_max^2 normal
  if (p.a_max < 0x1p-63f) return fail(TRAJ_E_INVAL, "a_max must be at least 2^-63");
  if (n_shapes < 1 || n_shapes > 4096) return fail(TRAJ_E_INVAL, "n_shapes must be in [1, 4096]");
  Handle* h = new (std::nothrow) Handle();
  if (h == nullptr) return fail(TRAJ_E_NOMEM, "host allocation failed");
  h->p = p;
  size_t off = 0;
  for (int i = 0; i < n_shapes; ++i) {
    const traj_shape& s = shapes[i];
    if (s.n_time < traj::NC || s.n_time > traj::MAX_TIME || !(isfinite(s.t_f) && s.t_f > 0.f) || s.n_obs < 0 ||
        s.n_obs > traj::MAX_OBS) {
      delete h;
      return fail(TRAJ_E_INVAL, "shape %d invalid (n_time in [%d, %d], t_f > 0, n_obs in [0, %d])", i, traj::NC,
                  traj::MAX_TIME, traj::MAX_OBS);
    }
    ShapeDesc d = {};
    d.n = s.n_time;
    d.m = s.n_obs;
    d.t_f = s.t_f;
    d.table_off = (int)off;
    d.table64_off = i * traj::TAB64_SIZE;
    off += (size_t)((traj::tab_size(d.n) + 63) / 64 * 64);
    h->shapes.push_back(d);
    if (d.n > h->max_n) h->max_n = d.n;
    if (d.m > h->max_m) h->max_m = d.m;
  }
  h->table_floats = off;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  if ((e = hipMalloc(&h->d_shapes, sizeof(ShapeDesc) * n_shapes)) != hipSuccess ||
      (e = hipMalloc(&h->d_tables, sizeof(float) * off)) != hipSuccess ||
      (e = hipMalloc(&h->d_tables64, sizeof(double) * traj::TAB64_SIZE * n_shapes)) != hipSuccess) {
    traj_destroy(h);
    return fail(TRAJ_E_NOMEM, "hipMalloc: %s", hipGetErrorString(e));
  }
  if ((e = hipMemcpyAsync(h->d_shapes, h->shapes.data(), sizeof(ShapeDesc) * n_shapes, hipMemcpyHostToDevice, st)) !=
          hipSuccess ||
      (e = traj::launch_setup(h->d_shapes, n_shapes, consts(p), h->d_tables, h->d_tables64, h->max_n, st)) !=
          hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess) {
    traj_destroy(h);
    return hip_fail(e, "traj_setup");
  }
  int dev = 0, cus = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess ||
      (e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) {
    traj_destroy(h);
    return hip_fail(e, "traj_setup: device query");
  }
  for (int mode = 0; mode < 2; ++mode) {
    int per_cu = 0;
    if ((e = traj::group_blocks_per_cu(mode, &per_cu)) != hipSuccess) {
      traj_destroy(h);
      return hip_fail(e, "traj_setup: occupancy query");
    }
    h->resident_blocks[mode] = cus * (per_cu > 0 ? per_cu : 1);
  }
  h->device = dev;
  if ((e = resolve_scratch(dev, &h->scratch)) != hipSuccess) {
    traj_destroy(h);
    return hip_fail(e, "traj_setup: address of the library scratch");
  }
  // the MFMA kernel's dynamic LDS for this handle's shapes (larger handles are
  // refused at dispatch)
  if ((e = traj::mfma_reserve_smem(traj::mfma_smem_bytes(h->max_n, h->max_m))) != hipSuccess) {
    traj_destroy(h);
    return hip_fail(e, "traj_setup: LDS reservation");
  }
  *handle_out = h;
  return TRAJ_OK;
}

int traj_destroy(void* handle) {
  Handle* h = (Handle*)handle;
  if (h == nullptr) return TRAJ_OK;
  // releasing is best effort: a failure leaves nothing the caller could act on
  if (h->d_shapes) (void)hipFree(h->d_shapes);
  if (h->d_tables) (void)hipFree(h->d_tables);
  if (h->d_tables64) (void)hipFree(h->d_tables64);
  delete h;
  return TRAJ_OK;
}

int traj_solve_batch(void* handle, const traj_batch* batch, traj_state* state, int iters, float tol, uint32_t flags,
                     void* stream) {
  g_err.clear();
  return solve_impl((Handle*)handle, batch, state, iters, tol, flags, stream, false);
}

int traj_solve_batch_noalloc(void* handle, const traj_batch* batch, traj_state* state, int iters, float tol,
                             uint32_t flags, void* stream) {
  g_err.clear();
  Handle* h = (Handle*)handle;
  if (h == nullptr) return fail(TRAJ_E_INVAL, "handle is NULL");
  int cur = -1;
  const hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "traj_solve_batch_noalloc: current device");
  if (cur != h->device)
    return fail(TRAJ_E_INVAL, "traj_solve_batch_noalloc: current device %d is not the handle's device %d", cur,
                h->device);
  if (h->scratch == nullptr) return fail(TRAJ_E_HIP, "traj_solve_batch_noalloc: library scratch not resolved");
  return solve_impl(h, batch, state, iters, tol, flags, stream, false, h->scratch);
}

int traj_score(void* handle, const traj_batch* batch, const traj_state* state, const traj_metacost* mc, float* cost,
               int32_t* best, void* stream) {
  g_err.clear();
  return score_impl((Handle*)handle, batch, state, mc, cost, best, stream);
}

int traj_converge(void* handle, const traj_batch* batch, traj_state* state, const traj_metacost* mc, int max_iters,
                  int chunk, float tol, uint32_t flags, float* cost, int32_t* best, int32_t* scene_iters,
                  void* stream) {
  g_err.clear();
  Handle* h = (Handle*)handle;
  if (h == nullptr) return fail(TRAJ_E_INVAL, "handle is NULL");
  int rc = check_batch(h, batch);
  if (rc != TRAJ_OK) return rc;
  if (state == nullptr || mc == nullptr) return fail(TRAJ_E_INVAL, "state / metacost is NULL");
  if (max_iters < 0 || max_iters > 100000 || chunk < 1 || chunk > 100000)
    return fail(TRAJ_E_INVAL, "max_iters must be in [0, 100000] and chunk in [1, 100000]");
  if (!(isfinite(tol) && tol > 0.f)) return fail(TRAJ_E_INVAL, "tol must be finite and > 0");
  if (batch->n_scenes == 0) return TRAJ_OK;
  if (state->scene_done == nullptr || scene_iters == nullptr || best == nullptr)
    return fail(TRAJ_E_INVAL, "state.scene_done, scene_iters and best are required");
  if (state->resid == nullptr) return fail(TRAJ_E_INVAL, "state.resid is required");
  const bool keep_done = (flags & TRAJ_KEEP_DONE) != 0;
  flags &= ~TRAJ_KEEP_DONE;
  hipStream_t st = (hipStream_t)stream;
  if (!keep_done) {
    hipError_t e = traj::launch_converge_reset(state->scene_done, scene_iters, batch->n_scenes, st);
    if (e != hipSuccess) return hip_fail(e, "traj_converge");
  }
  const uint32_t keep = TRAJ_PREC_BF16X3 | TRAJ_KERNEL_WAVE | TRAJ_KERNEL_MFMA | TRAJ_KERNEL_GROUP;
  for (int done = 0, c = 0; done < max_iters; ++c) {
    const int it = max_iters - done < chunk ? max_iters - done : chunk;
    // the first chunk starts as the caller asked; later chunks resume the state
    const uint32_t f = c == 0 ? flags : ((flags & keep) | TRAJ_INIT_FROM_STATE);
    if ((rc = solve_impl(h, batch, state, it, 0.f, f, stream, c > 0)) != TRAJ_OK) return rc;
    // scenes converged in an earlier chunk (or call, with TRAJ_KEEP_DONE) are neither
    // iterated nor re-scored; the scoring also applies the stopping rule to the others
    const traj::ConvergeCheck check = {state->resid, state->scene_done, scene_iters, it, tol};
    const int32_t* skip = (c > 0 || keep_done) ? state->scene_done : nullptr;
    if ((rc = score_impl(h, batch, state, mc, cost, best, stream, skip, &check)) != TRAJ_OK) return rc;
    done += it;
  }
  return TRAJ_OK;
}

}  // extern "C"

namespace {

// static_work: the library scratch (traj_solve_batch_noalloc), used instead of
// state->work by a group-kernel solve; NULL for traj_solve_batch.
int solve_impl(Handle* h, const traj_batch* batch, traj_state* state, int iters, float tol, uint32_t flags,
               void* stream, bool reuse_order, int32_t* static_work) {
  if (h == nullptr) return fail(TRAJ_E_INVAL, "handle is NULL");
  int rc = check_batch(h, batch);
  if (rc != TRAJ_OK) return rc;
  if (state == nullptr) return fail(TRAJ_E_INVAL, "state is NULL");
  if (iters < 0 || iters > 100000) return fail(TRAJ_E_INVAL, "iters must be in [0, 100000]");
  if (!isfinite(tol)) return fail(TRAJ_E_INVAL, "tol must be finite");
  const uint32_t kernels = TRAJ_KERNEL_WAVE | TRAJ_KERNEL_MFMA | TRAJ_KERNEL_GROUP;
  const uint32_t known = TRAJ_INIT_FROM_STATE | TRAJ_WARM_FALLBACK | TRAJ_PREC_BF16X3 | kernels;
  if ((flags & ~known) != 0) return fail(TRAJ_E_INVAL, "unknown flags 0x%x", flags);
  if ((flags & TRAJ_WARM_FALLBACK) && !(flags & TRAJ_INIT_FROM_STATE))
    return fail(TRAJ_E_INVAL, "TRAJ_WARM_FALLBACK needs TRAJ_INIT_FROM_STATE");
  uint32_t kernel = flags & kernels;
  if (kernel != 0 && (kernel & (kernel - 1)) != 0)
    return fail(TRAJ_E_INVAL, "TRAJ_KERNEL_WAVE, TRAJ_KERNEL_MFMA and TRAJ_KERNEL_GROUP are exclusive");
  if ((flags & TRAJ_PREC_BF16X3) && kernel == TRAJ_KERNEL_WAVE)
    return fail(TRAJ_E_INVAL, "TRAJ_PREC_BF16X3 runs on a matrix-core kernel only");
  if (kernel == 0) kernel = (uint32_t)h->tile.kernel;
  if ((flags & TRAJ_PREC_BF16X3) && kernel == TRAJ_KERNEL_WAVE) kernel = TRAJ_KERNEL_MFMA;
  if ((flags & TRAJ_WARM_FALLBACK) && kernel != TRAJ_KERNEL_GROUP)
    return fail(TRAJ_E_INVAL, "TRAJ_WARM_FALLBACK runs on the group kernel only");
  if (batch->n_goals == 0) return TRAJ_OK;
  if (state->c == nullptr || state->lam == nullptr) return fail(TRAJ_E_INVAL, "state.c / state.lam is NULL");
  int32_t* work = state->work;
  if (kernel == TRAJ_KERNEL_GROUP) {
    const int64_t need = traj::group_work_ints(batch->n_scenes, batch->n_goals, min_group(h));
    if (static_work != nullptr) {
      if (need > (int64_t)TRAJ_NOALLOC_WORK_INTS)
        return fail(TRAJ_E_INVAL,
                    "traj_solve_batch_noalloc: the group kernel's work list for %d scenes and %d goals (group "
                    "size %d) needs %lld int32, more than the library scratch of %d",
                    batch->n_scenes, batch->n_goals, min_group(h), (long long)need, TRAJ_NOALLOC_WORK_INTS);
      work = static_work;
    } else if (state->work == nullptr || state->work_ints < need) {
      return fail(TRAJ_E_INVAL, "the group kernel needs state.work with %lld int32 (got %lld)", (long long)need,
                  (long long)(state->work == nullptr ? 0 : state->work_ints));
    }
  }
  traj::SolveArgs a;
  a.goal_off = batch->goal_off;
  a.obs_off = batch->obs_off;
  a.shape_id = batch->shape_id;
  a.ego = batch->ego;
  a.obs = batch->obs;
  a.goal = batch->goal;
  a.c = state->c;
  a.lam = state->lam;
  a.resid = state->resid;
  a.iters_out = state->iters;
  a.skip = state->scene_done;
  a.shapes = h->d_shapes;
  a.tables = h->d_tables;
  a.tables64 = h->d_tables64;
  a.n_shapes = (int)h->shapes.size();
  a.n_scenes = batch->n_scenes;
  a.n_goals = batch->n_goals;
  a.iters = iters;
  a.flags = (int)flags;
  a.tol = tol;
  a.k = consts(h->p);
  const int mode = (flags & TRAJ_PREC_BF16X3) ? traj::TRAJ_MODE_BF16X3 : traj::TRAJ_MODE_FP32;
  hipError_t e;
  if (kernel == TRAJ_KERNEL_GROUP) {
    e = traj::launch_solve_group(a, mode, h->tile.group, min_group(h), h->tile.persistent != 0, h->resident_blocks[mode],
                                 work, reuse_order, (hipStream_t)stream);
  } else if (kernel == TRAJ_KERNEL_MFMA) {
    const size_t need = traj::mfma_smem_bytes(h->max_n, h->max_m);
    if (need > traj::MFMA_SMEM_LIMIT)
      return fail(TRAJ_E_INVAL,
                  "the MFMA kernel keeps every obstacle prediction of a horizon in LDS: the handle's longest "
                  "horizon (%d samples) with its most obstacles (%d) needs %zu bytes > %zu; use the group or "
                  "the wave kernel",
                  h->max_n, h->max_m, need, traj::MFMA_SMEM_LIMIT);
    e = traj::launch_solve_mfma(a, mode, h->tile.group, h->max_n, h->max_m, (hipStream_t)stream);
  } else {
    e = traj::launch_solve(a, h->max_n, h->max_m, h->tile.waves, (hipStream_t)stream);
  }
  if (e != hipSuccess) return hip_fail(e, "traj_solve_batch launch");
  return TRAJ_OK;
}

int score_impl(Handle* h, const traj_batch* batch, const traj_state* state, const traj_metacost* mc, float* cost,
               int32_t* best, void* stream, const int32_t* skip, const traj::ConvergeCheck* check) {
  if (h == nullptr) return fail(TRAJ_E_INVAL, "handle is NULL");
  int rc = check_batch(h, batch);
  if (rc != TRAJ_OK) return rc;
  if (state == nullptr || mc == nullptr) return fail(TRAJ_E_INVAL, "state / metacost is NULL");
  if (mc->kind != 0 && mc->kind != 1) return fail(TRAJ_E_INVAL, "metacost kind must be 0 or 1");
  if (!isfinite(mc->w1) || !isfinite(mc->w2)) return fail(TRAJ_E_INVAL, "metacost weights must be finite");
  if (!(isfinite(mc->clear_min) && mc->clear_min >= 0.f))
    return fail(TRAJ_E_INVAL, "metacost clear_min must be finite and >= 0");
  if (batch->n_scenes == 0) return TRAJ_OK;
  if (mc->v_ref == nullptr || (mc->kind == 1 && mc->y_rl == nullptr))
    return fail(TRAJ_E_INVAL, "metacost reference arrays are NULL");
  if (best == nullptr || (batch->n_goals > 0 && (cost == nullptr || state->c == nullptr)))
    return fail(TRAJ_E_INVAL, "cost / best / state.c is NULL");
  traj::ScoreArgs a;
  a.goal_off = batch->goal_off;
  a.shape_id = batch->shape_id;
  a.c = state->c;
  a.shapes = h->d_shapes;
  a.tables = h->d_tables;
  a.n_shapes = (int)h->shapes.size();
  a.n_scenes = batch->n_scenes;
  a.n_goals = batch->n_goals;
  a.kind = mc->kind;
  a.v_ref = mc->v_ref;
  a.y_rl = mc->y_rl;
  a.w1 = mc->w1;
  a.w2 = mc->w2;
  a.psi_max = h->p.psi_max;
  a.obs_off = batch->obs_off;
  a.obs = batch->obs;
  a.a = h->p.a;
  a.b = h->p.b;
  a.clear_min = mc->clear_min;
  a.skip = skip;
  a.cost = cost;
  a.best = best;
  hipError_t e = traj::launch_score(a, h->max_n, (hipStream_t)stream, check);
  if (e != hipSuccess) return hip_fail(e, "traj_score launch");
  return TRAJ_OK;
}

}  // namespace

extern "C" {

int traj_controls(void* handle, const traj_batch* batch, const traj_state* state, const int32_t* best,
                  float wheelbase, int stride, float* accel, float* steer, float* clearance, void* stream) {
  g_err.clear();
  Handle* h = (Handle*)handle;
  if (h == nullptr) return fail(TRAJ_E_INVAL, "handle is NULL");
  int rc = check_batch(h, batch);
  if (rc != TRAJ_OK) return rc;
  if (state == nullptr || state->c == nullptr || best == nullptr || accel == nullptr || steer == nullptr ||
      clearance == nullptr)
    return fail(TRAJ_E_INVAL, "traj_controls: NULL argument");
  if (!(isfinite(wheelbase) && wheelbase > 0.f)) return fail(TRAJ_E_INVAL, "wheelbase must be finite and > 0");
  if (stride < h->max_n) return fail(TRAJ_E_INVAL, "stride must be at least the longest horizon (%d)", h->max_n);
  if (batch->n_scenes == 0) return TRAJ_OK;
  traj::ControlArgs a;
  a.goal_off = batch->goal_off;
  a.obs_off = batch->obs_off;
  a.shape_id = batch->shape_id;
  a.obs = batch->obs;
  a.c = state->c;
  a.best = best;
  a.shapes = h->d_shapes;
  a.tables = h->d_tables;
  a.n_shapes = (int)h->shapes.size();
  a.n_scenes = batch->n_scenes;
  a.n_goals = batch->n_goals;
  a.stride = stride;
  a.wheelbase = wheelbase;
  a.v_floor = h->p.v_min;
  a.a = h->p.a;
  a.b = h->p.b;
  a.accel = accel;
  a.steer = steer;
  a.clearance = clearance;
  hipError_t e = traj::launch_controls(a, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "traj_controls launch");
  return TRAJ_OK;
}

int traj_set_tile(void* handle, const traj_tile* tile) {
  g_err.clear();
  Handle* h = (Handle*)handle;
  if (h == nullptr || tile == nullptr) return fail(TRAJ_E_INVAL, "NULL argument");
  if (tile->kernel != (int32_t)TRAJ_KERNEL_WAVE && tile->kernel != (int32_t)TRAJ_KERNEL_MFMA &&
      tile->kernel != (int32_t)TRAJ_KERNEL_GROUP)
    return fail(TRAJ_E_INVAL, "unknown kernel 0x%x", (unsigned)tile->kernel);
  if (tile->group < 1 || tile->group > 16) return fail(TRAJ_E_INVAL, "group must be in [1, 16]");
  if (tile->persistent != 0 && tile->persistent != 1) return fail(TRAJ_E_INVAL, "persistent must be 0 or 1");
  if (tile->waves != 1 && tile->waves != 2) return fail(TRAJ_E_INVAL, "waves must be 1 or 2");
  h->tile = *tile;
  return TRAJ_OK;
}

int traj_get_tile(void* handle, traj_tile* tile) {
  g_err.clear();
  Handle* h = (Handle*)handle;
  if (h == nullptr || tile == nullptr) return fail(TRAJ_E_INVAL, "NULL argument");
  *tile = h->tile;
  return TRAJ_OK;
}

int traj_work_ints(void* handle, int n_scenes, int n_goals, int64_t* out) {
  g_err.clear();
  Handle* h = (Handle*)handle;
  if (h == nullptr || out == nullptr) return fail(TRAJ_E_INVAL, "NULL argument");
  if (n_scenes < 0 || n_goals < 0) return fail(TRAJ_E_INVAL, "negative batch size");
  *out = traj::group_work_ints(n_scenes, n_goals, min_group(h));
  return TRAJ_OK;
}

int traj_set_shape_groups(void* handle, const int32_t* groups) {
  g_err.clear();
  Handle* h = (Handle*)handle;
  if (h == nullptr) return fail(TRAJ_E_INVAL, "NULL handle");
  int cur = -1;
  const hipError_t ed = hipGetDevice(&cur);
  if (ed != hipSuccess) return hip_fail(ed, "traj_set_shape_groups: current device");
  if (cur != h->device)
    return fail(TRAJ_E_INVAL, "traj_set_shape_groups: current device %d is not the handle's device %d", cur, h->device);
  std::vector<ShapeDesc> next = h->shapes;
  for (size_t i = 0; i < next.size(); ++i) {
    const int g = groups == nullptr ? 0 : groups[i];
    if (g < 0 || g > 16) return fail(TRAJ_E_INVAL, "shape %zu: group size %d outside 0..16", i, g);
    next[i].group = g;
  }
  const hipError_t e = hipMemcpy(h->d_shapes, next.data(), sizeof(ShapeDesc) * next.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "traj_set_shape_groups");
  h->shapes = next;
  return TRAJ_OK;
}

int traj_get_shape_groups(void* handle, int32_t* groups) {
  g_err.clear();
  Handle* h = (Handle*)handle;
  if (h == nullptr || groups == nullptr) return fail(TRAJ_E_INVAL, "NULL argument");
  for (size_t i = 0; i < h->shapes.size(); ++i) groups[i] = h->shapes[i].group;
  return TRAJ_OK;
}

int traj_debug_table_size(void* handle, int shape) {
  Handle* h = (Handle*)handle;
  if (h == nullptr || shape < 0 || shape >= (int)h->shapes.size()) return fail(TRAJ_E_SHAPE, "bad handle or shape");
  return traj::tab_size(h->shapes[shape].n);
}

int traj_debug_operators(void* handle, int shape, double* out_f64, float* out_f32, void* stream) {
  g_err.clear();
  Handle* h = (Handle*)handle;
  if (h == nullptr) return fail(TRAJ_E_INVAL, "handle is NULL");
  if (shape < 0 || shape >= (int)h->shapes.size()) return fail(TRAJ_E_SHAPE, "shape %d not set up", shape);
  const ShapeDesc& d = h->shapes[shape];
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  if (out_f64)
    e = hipMemcpyAsync(out_f64, h->d_tables64 + d.table64_off, sizeof(double) * traj::SYS_COUNT * traj::KMAX * traj::KMAX,
                       hipMemcpyDeviceToHost, st);
  if (e == hipSuccess && out_f32)
    e = hipMemcpyAsync(out_f32, h->d_tables + d.table_off, sizeof(float) * traj::tab_size(d.n), hipMemcpyDeviceToHost,
                       st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "traj_debug_operators");
  return TRAJ_OK;
}

int traj_debug_atan2(const float* y, const float* x, float* out, int n, void* stream) {
  g_err.clear();
  if (y == nullptr || x == nullptr || out == nullptr || n < 0) return fail(TRAJ_E_INVAL, "bad argument");
  hipError_t e = traj::launch_debug_atan2(y, x, out, n, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "traj_debug_atan2");
  return TRAJ_OK;
}

int traj_debug_reduce(const float* in, float* out, int r, void* stream) {
  g_err.clear();
  if (in == nullptr || out == nullptr) return fail(TRAJ_E_INVAL, "NULL argument");
  if (r != 16 && r != 32) return fail(TRAJ_E_INVAL, "r must be 16 or 32");
  hipError_t e = traj::launch_debug_reduce(in, out, r, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "traj_debug_reduce");
  return TRAJ_OK;
}

}  // extern "C"

namespace traj {
int handle_view(void* handle, const ShapeDesc** shapes, const float** tables, int* n_shapes, float* a_max,
                float* ell_a, float* ell_b) {
  Handle* h = (Handle*)handle;
  if (h == nullptr) return fail(TRAJ_E_INVAL, "handle is NULL");
  *shapes = h->d_shapes;
  *tables = h->d_tables;
  *n_shapes = (int)h->shapes.size();
  *a_max = h->p.a_max;
  *ell_a = h->p.a;
  *ell_b = h->p.b;
  return TRAJ_OK;
}

// the longest n_time of the handle's shapes (host copy, no device access)
int handle_max_n(void* handle, int* max_n) {
  Handle* h = (Handle*)handle;
  if (h == nullptr) return fail(TRAJ_E_INVAL, "handle is NULL");
  *max_n = h->max_n;
  return TRAJ_OK;
}
}  // namespace traj
