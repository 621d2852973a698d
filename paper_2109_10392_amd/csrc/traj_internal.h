// Internal layout shared by the HIP kernels and the C-ABI implementation.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "traj.h"

namespace traj {

constexpr int NC = TRAJ_N_COEF;  // Bernstein coefficients per axis
constexpr int NX = 4;            // boundary rows of x: x(0), x'(0), x''(0), x(t_f)
constexpr int NY = 6;            // boundary rows of y: + y'(t_f), y''(t_f)
constexpr int NP = 4;            // boundary rows of psi: psi(0), psi'(0), psi(t_f), psi'(t_f)
constexpr int KMAX = NC + NY;    // largest KKT system (17)
constexpr int MAX_TIME = 192;    // three 64-lane slots
constexpr int MAX_OBS = 64;
constexpr int WAVE = 64;
constexpr int GOALS_PER_WG = 4;  // one goal per wave, four waves per workgroup

// precision modes of the matrix-core kernel
constexpr int TRAJ_MODE_FP32 = 0;
constexpr int TRAJ_MODE_BF16X3 = 1;

// Per-shape FP32 table, offsets in floats from the shape's table_off.
//   basis:  P[NC][n], Pd[NC][n], Pdd[NC][n]        (coefficient-major, time fastest)
//   square: MGx, Mx, MGy, My, Mp                   (each NC x NC row-major)
//           MGx = Mx (rho F_ax^T F_ax) = Mx (rho (m P^T P + P''^T P'' + P'^T P'))
//   boundary: Mbx[NC][NX], Mby[NC][NY], Mbp[NC][NP], M0bx[NC][NX], M0by[NC][NY]
enum SquareId { SQ_MGX = 0, SQ_MX, SQ_MGY, SQ_MY, SQ_MP, SQ_COUNT };

__host__ __device__ inline int tab_basis(int n, int which) { return which * NC * n; }
__host__ __device__ inline int tab_square(int n, int id) { return 3 * NC * n + id * NC * NC; }
__host__ __device__ inline int tab_bnd(int n) { return 3 * NC * n + SQ_COUNT * NC * NC; }
// boundary sub-blocks relative to tab_bnd
constexpr int BND_MBX = 0;
constexpr int BND_MBY = BND_MBX + NC * NX;
constexpr int BND_MBP = BND_MBY + NC * NY;
constexpr int BND_M0BX = BND_MBP + NC * NP;
constexpr int BND_M0BY = BND_M0BX + NC * NX;
constexpr int BND_SIZE = BND_M0BY + NC * NY;
// Packed product tiles of the group kernel (4-float aligned, after the boundary
// blocks): [tile w][slot s][lane l] float4 for 16-sample tiles w. Lane l = 16 q + j
// of slot s < 3 holds the evaluation operand of basis s (P, P', P''): entries
// [t = 16 w + j][k = 4 q .. 4 q + 3]; slot 3 + s the contraction operand of basis s:
// entries [t = 16 w + 4 q + r][k = j], r = 0..3. Zero outside the n x NC matrix.
constexpr int TILE_T = 16;
constexpr int PACK_SLOTS = 6;
__host__ __device__ inline int n_tiles(int n) { return (n + TILE_T - 1) / TILE_T; }

// max(r_obs, r_acc, r_nh) (squared or not) of the stopping rule and of the warm
// start's fallback test; NaN when any component is NaN, which fmaxf alone would
// drop (a goal with NaN coefficients has r_obs = 0: no inside test holds).
__host__ __device__ inline float worst_of(float a, float b, float c) {
  const float m = fmaxf(fmaxf(a, b), c);
  const float s = a + b + c;  // the components are >= 0: NaN exactly when one is NaN
  return s == s ? m : __builtin_nanf("");
}
__host__ __device__ inline int tab_pack(int n) { return (tab_bnd(n) + BND_SIZE + 3) & ~3; }
__host__ __device__ inline int tab_size(int n) { return tab_pack(n) + n_tiles(n) * PACK_SLOTS * WAVE * 4; }

// FP64 table per shape: the 5 KKT inverses (KMAX x KMAX each, verification),
// then the operators of the x/y step that stay in FP64 in the solver:
//   MGx, Mx, MGy, My (NC x NC), Mbx (NC x NX), Mby (NC x NY).
// The x/y step adds these constant terms to the iterate every iteration and the
// multipliers integrate whatever they carry, so their FP32 rounding would act
// as a systematic per-iteration perturbation of the fixed point.
enum SysId { SYS_X = 0, SYS_Y, SYS_P, SYS_0X, SYS_0Y, SYS_COUNT };
constexpr int T64_INV = 0;
constexpr int T64_MGX = SYS_COUNT * KMAX * KMAX;
constexpr int T64_MX = T64_MGX + NC * NC;
constexpr int T64_MGY = T64_MX + NC * NC;
constexpr int T64_MY = T64_MGY + NC * NC;
constexpr int T64_MBX = T64_MY + NC * NC;
constexpr int T64_MBY = T64_MBX + NC * NX;
constexpr int TAB64_SIZE = T64_MBY + NC * NY;

struct ShapeDesc {
  int n;          // samples
  int m;          // obstacles
  float t_f;
  int table_off;  // float offset of the FP32 table
  int table64_off;
  int group;      // goals per group of the group kernel for scenes of this shape (0: the tile's)
};

struct SolverConst {
  float rho, a, b, v_min, v_max, a_max, psi_max;
};

struct SolveArgs {
  const int32_t* goal_off;
  const int32_t* obs_off;
  const int32_t* shape_id;
  const float* ego;
  const float* obs;
  const float* goal;
  float* c;
  float* lam;
  float* resid;
  int32_t* iters_out;
  const int32_t* skip;  // [n_scenes] or NULL: scenes with a non-zero entry are left untouched
  const ShapeDesc* shapes;
  const float* tables;
  const double* tables64;
  int n_shapes;
  int n_scenes;
  int n_goals;
  int iters;
  int flags;
  float tol;
  SolverConst k;
};

// A scene's obstacle range [obs_off[s], obs_off[s+1]) as the kernels read it: a
// non-negative start and the obstacle count of the scene's shape (at most MAX_OBS).
// Any other range is never read; the scene is marked like one of unknown shape.
__device__ __forceinline__ bool obstacles_ok(int o0, int m_scene, int m_shape) {
  return o0 >= 0 && m_scene == m_shape && m_scene >= 0 && m_scene <= MAX_OBS;
}

// Inputs a solve cannot use: a scene whose ego state (the boundary values of
// eq. 8b) or any obstacle state is not finite marks every goal of the scene; a
// goal whose target is not finite marks that goal. A marked goal's coefficients,
// multipliers and residuals become NaN and its iteration count 0 (so scoring
// never picks it); the other goals are solved as usual.
// The check reads through an offset the compiler cannot see through (an empty asm
// statement), so its loads are not merged with the solve's own later reads of the
// same values, which would keep those live across the whole solve.
__device__ __forceinline__ bool all_finite(const float* v, int count) {
  int opaque = 0;
  asm volatile("" : "+s"(opaque));
  v += opaque;
  bool ok = true;
  for (int i = 0; i < count; ++i) ok = ok && __builtin_isfinite(v[i]);
  return ok;
}

// the outputs of a marked goal, written by `parts` lanes of which this is `part`
__device__ __forceinline__ void write_marked_goal(const SolveArgs& A, int g, int part, int parts) {
  const float nan = __builtin_nanf("");
  const int NG = A.n_goals;
  for (int e = part; e < 3 * NC; e += parts) {
    A.c[e * NG + g] = nan;
    A.lam[e * NG + g] = nan;
  }
  if (part == 0) {
    if (A.resid != nullptr)
      for (int k = 0; k < 4; ++k) A.resid[k * NG + g] = nan;
    if (A.iters_out != nullptr) A.iters_out[g] = 0;
  }
}

struct ScoreArgs {
  const int32_t* goal_off;
  const int32_t* shape_id;
  const float* c;
  const ShapeDesc* shapes;
  const float* tables;
  int n_shapes;
  int n_scenes;
  int n_goals;
  int kind;
  const float* v_ref;
  const float* y_rl;
  float w1, w2, psi_max;
  // collision post-check (clear_min > 0): obstacles of the batch and the ellipse axes
  const int32_t* obs_off;
  const float* obs;
  float a, b, clear_min;
  // scenes with a non-zero entry keep their cost and best untouched (NULL: none);
  // the chunked solve passes its converged scenes, whose state no longer changes
  const int32_t* skip;
  float* cost;
  int32_t* best;
};

struct ControlArgs {
  const int32_t* goal_off;
  const int32_t* obs_off;
  const int32_t* shape_id;
  const float* obs;
  const float* c;
  const int32_t* best;
  const ShapeDesc* shapes;
  const float* tables;
  int n_shapes;
  int n_scenes;
  int n_goals;
  int stride;
  float wheelbase, v_floor, a, b;
  float* accel;
  float* steer;
  float* clearance;
};

// Launchers (defined next to their kernels). Return hipSuccess or the launch error.
hipError_t launch_setup(const ShapeDesc* d_shapes, int n_shapes, const SolverConst& k, float* d_tables,
                        double* d_tables64, int max_n, hipStream_t stream);
hipError_t launch_solve(const SolveArgs& a, int max_n, int max_m, int waves, hipStream_t stream);
hipError_t launch_solve_mfma(const SolveArgs& a, int mode, int G, int max_n, int max_m, hipStream_t stream);
size_t mfma_smem_bytes(int max_n, int max_m);
constexpr size_t MFMA_SMEM_LIMIT = 150 * 1024;  // LDS the MFMA kernel may take per workgroup
// Stopping rule of the chunked solve, applied by the argmin kernel when done is set:
// per scene not yet converged, scene_iters += iters and done = 1 once the residual
// max(r_obs, r_acc, r_nh) of its best goal is at or below tol.
struct ConvergeCheck {
  const float* resid;
  int32_t* done;
  int32_t* scene_iters;
  int iters;
  float tol;
};
hipError_t launch_score(const ScoreArgs& a, int max_n, hipStream_t stream, const ConvergeCheck* check = nullptr);
hipError_t launch_controls(const ControlArgs& a, hipStream_t stream);

// Group kernel (one wavefront per goal group, cost-sorted work list).
// work: int32 workspace of group_work_ints(n_scenes, n_goals, G) entries.
int64_t group_work_ints(int n_scenes, int n_goals, int G);
hipError_t group_blocks_per_cu(int mode, int* blocks);
// G: the tile's goals per group, used where a shape sets none; G_min: the smallest
// group size of any shape (sizes the work list).
hipError_t launch_solve_group(const SolveArgs& a, int mode, int G, int G_min, bool persistent, int resident_blocks,
                              int32_t* work, bool reuse_order, hipStream_t stream);
// Convergence bookkeeping (traj_converge): zero the per-scene flags and counters
// (the check after each chunk runs in the argmin kernel, see ConvergeCheck).
hipError_t launch_converge_reset(int32_t* done, int32_t* scene_iters, int n_scenes, hipStream_t stream);

}  // namespace traj
