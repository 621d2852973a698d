/*
 * traj_mpc.h -- receding-horizon (closed-loop) use of the batched planner of
 * traj.h, for many episodes at once on straight multi-lane roads.
 *
 * The paper (arXiv 2109.10392, Sec. IV) runs the planner in a loop: plan from
 * the current state, execute the start of the chosen trajectory, plan again,
 * among traffic. Here a cycle is one sample interval t_f / (n_time - 1) of the
 * episode's shape: the ego moves to the chosen trajectory's state one sample
 * ahead, and the other vehicles move by the Intelligent Driver Model (Treiber,
 * Hennecke and Helbing, 2000; the paper gives no traffic model, so its
 * parameters are inputs). The frame is re-centred on the ego every cycle (ego x
 * = 0; the distance is accumulated), so positions stay small.
 *
 * A cycle on the caller's stream: traj_mpc_goals -> traj_converge (or
 * traj_solve_batch) -> traj_score -> traj_mpc_step. Conventions as in traj.h.
 */
#ifndef TRAJ_MPC_H
#define TRAJ_MPC_H

#include <stdint.h>

#include "traj.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  float idm_a;        /* IDM maximum acceleration (m/s^2), > 0 */
  float idm_b;        /* IDM comfortable deceleration (m/s^2), > 0 */
  float idm_s0;       /* IDM minimum gap (m), >= 0 */
  float idm_T;        /* IDM time headway (s), >= 0 */
  float idm_delta;    /* IDM acceleration exponent, > 0 */
  float car_length;   /* bumper-to-bumper gap = leader x - follower x - car_length (m) */
  float lane_width;   /* lane centres (k - floor((n_lanes - 1) / 2)) lane_width; same lane: |dy| < lane_width / 2 */
  int32_t n_lanes;    /* goal template: lanes */
  int32_t per_lane;   /* goal template: longitudinal slots per lane */
  float goal_v_floor; /* goal template: x_f = x0 + max(|v|, goal_v_floor) t_f linspace(0.8, 1.2, per_lane) */
  int32_t sampler;    /* 0: the template (cruise, eq. 25); 1: the right-lane sampler of Sec. III-F for
                         eq. 26: of G = n_lanes per_lane goals, n_r = round(0.6 G) on the right lane
                         (lane 0, the lowest y) at x0 + v_max t_f linspace(0.2, 1, n_r); the others
                         round-robin over lanes 1 .. n_lanes-1 at x0 + v_max t_f (0.9 .. 1.0) */
  float v_max;        /* sampler 1: the scenario's maximum speed (m/s), > 0 */
} traj_mpc_params;

/* Episode state, device arrays; ego, obs and goal are the arrays the traj_batch
 * of the episodes points to. */
typedef struct {
  float *ego;          /* [S][8]: x, y, vx, vy, ax, ay, psi, psi' (advanced in place) */
  float *obs;          /* [n_obs][4]: x, y, vx, vy (advanced in place) */
  float *goal;         /* [n_goals][2] (rewritten by traj_mpc_goals) */
  const float *v_des;  /* [n_obs]: IDM desired speed of every obstacle, > 0 */
  float *obs_next;     /* [n_obs][4] scratch */
  float *travelled;    /* [S]: distance the ego moved along x (accumulated) */
  int32_t *collisions; /* [S]: obstacle-ellipse overlaps after each cycle (accumulated) */
  int32_t *fallbacks;  /* [S]: cycles in which every goal was filtered (accumulated) */
  float *shift;        /* [S]: the ego's x advance in the last traj_mpc_step (the frame's
                          re-centring; written by traj_mpc_step, read by traj_mpc_shift) */
} traj_episodes;

/*
 * traj_mpc_goals -- the goals of every episode from its ego's current state
 * (n_lanes x per_lane goals; p->sampler picks the template or the right-lane
 * sampler). Episodes with another goal count are left unchanged.
 */
int traj_mpc_goals(void *handle, const traj_batch *batch, const traj_episodes *eps, const traj_mpc_params *p,
                   void *stream);

/*
 * traj_mpc_step -- one cycle after planning: every obstacle one period ahead by
 * IDM (following the nearest vehicle ahead in its lane, the ego included; free
 * road otherwise; speed clipped at 0, ballistic position update); the ego to its
 * chosen trajectory one sample ahead (state c of goal best[s]; with best[s] < 0
 * it brakes along the road at a_max (x' -= a_max dt, floored at 0) and stops
 * moving sideways: y kept, y' = y'' = psi = psi' = 0); then the frame re-centred on the
 * ego and overlaps of obstacle ellipses with the ego centre counted.
 *   n_obs: total obstacles of the batch (= obs_off[n_scenes]).
 */
int traj_mpc_step(void *handle, const traj_batch *batch, const traj_state *state, const int32_t *best,
                  const traj_episodes *eps, const traj_mpc_params *p, int n_obs, void *stream);

/*
 * traj_mpc_shift -- warm start of the next cycle from this cycle's solutions
 * (every goal slot's final iterate), advanced by the cycle's period: a
 * trajectory of the new horizon [dt, t_f + dt] is the same polynomial, so with
 * u0 = dt / t_f = 1 / (n_time - 1) the Bernstein coefficients of each of
 * x, y, psi become c' = S c, S_ik = sum_q B(10-i, k-q; u0) B(i, q; 1+u0),
 * B(n, j; u) = C(n, j) u^j (1-u)^(n-j) (the polar form at u0 (10-i times) and
 * 1+u0 (i times)), then x' -= shift[s] (the frame re-centring; the basis sums
 * to one). The multipliers are kept as they are: of the forms tried (kept,
 * S lambda, S^-T lambda, lambda + Q (c' - c), zero) keeping them needs the
 * fewest iterations in closed loop. Call after traj_mpc_step and
 * traj_mpc_goals; solve with TRAJ_INIT_FROM_STATE (and TRAJ_WARM_FALLBACK).
 * The first iteration's x/y step puts every goal's boundary values in place
 * (eq. 8b).
 *   state: c, device [3][11][n_goals], updated in place (lam is not touched).
 *   eps: shift.
 */
int traj_mpc_shift(void *handle, const traj_batch *batch, traj_state *state, const traj_episodes *eps,
                   void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TRAJ_MPC_H */
