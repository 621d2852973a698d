/*
 * traj_frenet.h -- road-attached (centre-line) frame around the batched planner
 * of traj.h.
 *
 * The paper (arXiv 2109.10392, Sec. III, assumption 1) poses the optimisation
 * in the frame of the road's centre-line, so that a curved road looks straight:
 * x is the arc length s along the centre-line and y the signed lateral offset d
 * (left of the direction of travel positive); the trajectories are mapped back
 * to the global frame afterwards. These calls do both mappings on the device for
 * a centre-line made of segments of constant curvature (straights and circular
 * arcs) starting at a given pose.
 *
 * Conventions as in traj.h: device pointers, the caller's stream, no allocation,
 * no synchronisation; errors are TRAJ_E_INVAL (checked on the host, nothing is
 * launched) and TRAJ_E_HIP. Arithmetic inside is FP64 (global coordinates can be
 * kilometres); inputs and outputs are FP32.
 */
#ifndef TRAJ_FRENET_H
#define TRAJ_FRENET_H

#include <stdint.h>

#include "traj.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Centre-line: n_seg segments, segment i of length seg[2i] (m, > 0) and
 * curvature seg[2i+1] (1/m; > 0 turns left, 0 is straight), each arc turning by
 * at most pi (|curvature| * length <= pi), starting at (x0, y0) with heading
 * theta0 (rad). The centre-line is continued straight beyond both ends.
 * seg is a HOST array, copied at each call; 1 <= n_seg <= 64. */
typedef struct {
  int32_t n_seg;
  const float *seg;
  float x0, y0, theta0;
} traj_road;

/*
 * traj_road_from_global -- vehicle states from the global frame into the road
 * frame. Position: s and d of the closest point of the centre-line (the segment
 * with the smallest distance; ties to the lower index). With T, N the unit
 * tangent and left normal there and k the curvature:
 *   velocity      s' = (v . T) / (1 - k d),  d' = v . N
 *   acceleration  s'' = (a . T + 2 k d' s') / (1 - k d),  d'' = a . N - k (1 - k d) s'^2
 *   heading       psi_road = psi - theta(s),  psi_road' = psi' - k s'
 * (exact for constant curvature at the foot point).
 *   kind 0 (obstacles): in/out [n][4] = x, y, vx, vy -> s, d, s', d'.
 *   kind 1 (ego states): in/out [n][8] = x, y, vx, vy, ax, ay, psi, psi'
 *                        -> s, d, s', d', s'', d'', psi_road, psi_road'.
 *   in and out may be the same array. A point on an arc's centre of curvature,
 *   or with 1 - k d <= 0 at its foot point, gets NaN rates (s', d', ...).
 */
int traj_road_from_global(const traj_road *road, int kind, int n, const float *in, float *out, void *stream);

/*
 * traj_road_to_global -- points (s, d) of the road frame to the global frame:
 * out[i] = (X, Y, theta) with (X, Y) = C(s) + d N(s) and theta = theta(s) the
 * centre-line heading at s. in: device [n][2], out: device [n][3].
 */
int traj_road_to_global(const traj_road *road, int n, const float *in, float *out, void *stream);

/*
 * traj_trajectory_to_global -- the chosen trajectory of every scene (goal
 * best[s] of traj_score, planned in the road frame: x = s, y = d) at the
 * scene's samples, in the global frame: out[s][t] = (X, Y, heading), heading =
 * theta(s) + atan2(d', (1 - k d) s') the direction of motion. Samples t >= n_time
 * of the scene and scenes with best < 0 are left untouched.
 *   out: device [n_scenes][stride][3], stride >= the longest n_time of the
 *   handle.
 */
int traj_trajectory_to_global(void *handle, const traj_batch *batch, const traj_state *state, const int32_t *best,
                              const traj_road *road, int stride, float *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TRAJ_FRENET_H */
