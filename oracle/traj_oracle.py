"""FP64 CPU oracle of the batch non-holonomic trajectory optimizer.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module. It shares no code
with the HIP path and imports nothing from the product package.

What it computes is the paper's method written out plainly, in float64, with
every matrix formed explicitly as printed:

* basis (Sec. III-B, eq. 6): 10th-order Bernstein polynomials on tau = t/t_f;
* stacked matrices (eq. 7a-c): F_o is P repeated m times, obstacle-major;
* reformulated problem (eq. 8a-c, 9): Q = P''^T P'', A c = b, F c = g(...);
* Algorithm 1 (Sec. III-D, eqs. 12-16) in its order: x/y QP -> heading QP ->
  velocity -> (alpha, d) -> (alpha_a, d_a) -> multipliers (eqs. 23-24);
* the QPs are solved through their KKT systems (eqs. 17, 19) with one LU
  factorisation shared by the whole batch (eqs. 18, 20);
* closed forms: velocity (eq. 21), alpha (eq. 22), d as the clipped 1-D
  least-squares minimiser of the second half of eq. 15, (alpha_a, d_a) as in
  eq. 16;
* meta-costs (eqs. 25, 26) and the heading post-filter (Sec. III intro).

Readings where the paper is silent or garbled (documented with the design):
boundary rows, cold start, residual norms, d >= 1 rather than the printed
[0, 1] clip, etc. -- see the module functions.

Batch convention: goals are columns (the paper's [q_1 | ... | q_l]).
"""
from __future__ import annotations

from math import comb

import numpy as np
import scipy.linalg

# ----------------------------------------------------------------- basis (eq. 6)


def bernstein_matrices(n_coef: int, n_time: int, t_f: float):
    """P, P_dot, P_ddot (n_time x n_coef), Bernstein degree n_coef-1 on tau = t/t_f.

    Time grid: n_time samples linspace(0, t_f) inclusive. Derivatives are the
    exact derivatives of the Bernstein polynomials with respect to t, i.e. the
    tau-derivatives scaled by 1/t_f and 1/t_f^2.
    """
    deg = n_coef - 1
    tau = np.linspace(0.0, 1.0, n_time)

    def B(d, k):
        if k < 0 or k > d:
            return np.zeros_like(tau)
        return comb(d, k) * tau ** k * (1.0 - tau) ** (d - k)

    P = np.stack([B(deg, k) for k in range(n_coef)], axis=1)
    Pd = np.stack([deg * (B(deg - 1, k - 1) - B(deg - 1, k)) for k in range(n_coef)], axis=1) / t_f
    Pdd = np.stack([deg * (deg - 1) * (B(deg - 2, k - 2) - 2.0 * B(deg - 2, k - 1) + B(deg - 2, k))
                    for k in range(n_coef)], axis=1) / t_f ** 2
    return P, Pd, Pdd


def time_grid(n_time: int, t_f: float) -> np.ndarray:
    return np.linspace(0.0, t_f, n_time)


# ---------------------------------------------------- boundary conditions (eq. 8b)


def boundary_matrices(P, Pd, Pdd):
    """Rows of A for each axis (reading of the boundary set C_b of eq. 1c).

    x:   x(0), x'(0), x''(0), x(t_f)
    y:   y(0), y'(0), y''(0), y(t_f), y'(t_f) = 0, y''(t_f) = 0
    psi: psi(0), psi'(0), psi(t_f) = 0, psi'(t_f) = 0
    """
    A_x = np.stack([P[0], Pd[0], Pdd[0], P[-1]])
    A_y = np.stack([P[0], Pd[0], Pdd[0], P[-1], Pd[-1], Pdd[-1]])
    A_psi = np.stack([P[0], Pd[0], P[-1], Pd[-1]])
    return A_x, A_y, A_psi


def boundary_values(ego, goals):
    """b_x (4 x B), b_y (6 x B), b_psi (4 x B) from the ego state and goal positions.

    ego = (x0, y0, vx0, vy0, ax0, ay0, psi0, psidot0); goals = (x_f, y_f) per goal.
    Final lateral velocity/acceleration and final heading/heading rate are 0.
    """
    ego = np.asarray(ego, np.float64)
    goals = np.asarray(goals, np.float64)
    B = goals.shape[0]
    one = np.ones(B)
    b_x = np.stack([ego[0] * one, ego[2] * one, ego[4] * one, goals[:, 0]])
    b_y = np.stack([ego[1] * one, ego[3] * one, ego[5] * one, goals[:, 1], 0 * one, 0 * one])
    b_psi = np.stack([ego[6] * one, ego[7] * one, 0 * one, 0 * one])
    return b_x, b_y, b_psi


# ------------------------------------------------------ problem data (eqs. 7, 9)


def obstacle_predictions(obs, t):
    """xi_x, xi_y stacked obstacle-major (m*n,): constant-velocity prediction x_j + vx_j t."""
    obs = np.asarray(obs, np.float64).reshape(-1, 4)
    xi_x = (obs[:, 0:1] + obs[:, 2:3] * t[None, :]).reshape(-1)
    xi_y = (obs[:, 1:2] + obs[:, 3:4] * t[None, :]).reshape(-1)
    return xi_x, xi_y


def build_F(P, Pd, Pdd, m):
    """F = blkdiag(F_ax, F_ax), F_ax = [F_o; P''; P'], F_o = P stacked m times (eq. 9, Sec. III-B)."""
    F_o = np.concatenate([P] * m, axis=0) if m > 0 else np.zeros((0, P.shape[1]))
    F_ax = np.concatenate([F_o, Pdd, Pd], axis=0)
    Z = np.zeros_like(F_ax)
    F = np.block([[F_ax, Z], [Z, F_ax]])
    return F, F_ax


def build_g(xi_x, xi_y, a, b, d, alpha, d_a, alpha_a, v, psi):
    """g_l of eq. 9, one column per goal. d, alpha: (m*n, B); d_a, alpha_a, v, psi: (n, B)."""
    g_x = np.concatenate([xi_x[:, None] + a * d * np.cos(alpha),
                          d_a * np.cos(alpha_a),
                          v * np.cos(psi)], axis=0)
    g_y = np.concatenate([xi_y[:, None] + b * d * np.sin(alpha),
                          d_a * np.sin(alpha_a),
                          v * np.sin(psi)], axis=0)
    return np.concatenate([g_x, g_y], axis=0)


# ------------------------------------------------------------- the optimizer


class Problem:
    """Constant data of one (n_time, t_f, m) shape: basis, F, KKT factorisations (Remark 1)."""

    def __init__(self, n_time, t_f, m, params):
        p = params
        self.N = N = int(p["n_coef"])
        self.n = n_time
        self.t_f = float(t_f)
        self.m = m
        self.rho = float(p["rho"])
        self.a, self.b = float(p["a"]), float(p["b"])
        self.v_min, self.v_max = float(p["v_min"]), float(p["v_max"])
        self.a_max = float(p["a_max"])
        self.psi_max = float(p["psi_max"])
        self.t = time_grid(n_time, t_f)
        self.P, self.Pd, self.Pdd = bernstein_matrices(N, n_time, t_f)
        # cost matrix: sum of squared accelerations (eq. 8a)
        self.Q = self.Pdd.T @ self.Pdd
        self.A_x, self.A_y, self.A_psi = boundary_matrices(self.P, self.Pd, self.Pdd)
        nx, ny = self.A_x.shape[0], self.A_y.shape[0]
        self.A = np.block([[self.A_x, np.zeros((nx, N))], [np.zeros((ny, N)), self.A_y]])
        self.F, self.F_ax = build_F(self.P, self.Pd, self.Pdd, m)
        rho = self.rho
        QQ = np.block([[self.Q, np.zeros((N, N))], [np.zeros((N, N)), self.Q]])
        ne = self.A.shape[0]
        # eq. 17: [[Q + rho F^T F, A^T], [A, 0]]
        self.Q_xy = np.block([[QQ + rho * self.F.T @ self.F, self.A.T], [self.A, np.zeros((ne, ne))]])
        # eq. 19: [[Q + rho P^T P, A^T], [A, 0]]
        npsi = self.A_psi.shape[0]
        self.Q_psi = np.block([[self.Q + rho * self.P.T @ self.P, self.A_psi.T],
                               [self.A_psi, np.zeros((npsi, npsi))]])
        # cold start: the boundary-only minimum-acceleration QP
        self.Q_0 = np.block([[QQ, self.A.T], [self.A, np.zeros((ne, ne))]])
        # one factorisation each, shared by every goal (eqs. 18, 20)
        self.lu_xy = scipy.linalg.lu_factor(self.Q_xy)
        self.lu_psi = scipy.linalg.lu_factor(self.Q_psi)
        self.lu_0 = scipy.linalg.lu_factor(self.Q_0)


def _xy_rhs_b(prob, ego, goals):
    b_x, b_y, b_psi = boundary_values(ego, goals)
    return np.concatenate([b_x, b_y], axis=0), b_psi


def solve_xy(prob, g, lam_xy, b_xy):
    """Step (12) through eq. 17/18: returns c_x, c_y (N x B each) and the full KKT solution."""
    rhs = np.concatenate([prob.rho * prob.F.T @ g + lam_xy, b_xy], axis=0)
    sol = scipy.linalg.lu_solve(prob.lu_xy, rhs)
    N = prob.N
    return sol[:N], sol[N:2 * N], sol


def solve_psi(prob, theta, lam_psi, b_psi):
    """Step (13) with the convex surrogate, through eq. 19/20."""
    rhs = np.concatenate([prob.rho * prob.P.T @ theta + lam_psi, b_psi], axis=0)
    sol = scipy.linalg.lu_solve(prob.lu_psi, rhs)
    return sol[:prob.N], sol


def project_velocity(prob, xd, yd):
    """Eq. 21: v = clip(sqrt(xd^2 + yd^2), v_min, v_max)."""
    return np.clip(np.sqrt(xd ** 2 + yd ** 2), prob.v_min, prob.v_max)


def project_obstacles(prob, x, y, xi_x, xi_y):
    """Step (15): alpha by eq. 22; d as the 1-D least-squares minimiser over d >= 1.

    x, y: (n, B). Returns alpha, d of shape (m*n, B), obstacle-major rows.
    The printed clip to [0, 1] contradicts the constraint d >= 1 stated with
    eq. 4 and the feasible set of eq. 15; d >= 1 is used.
    """
    m = prob.m
    a, b = prob.a, prob.b
    X = np.tile(x, (m, 1))
    Y = np.tile(y, (m, 1))
    dx = X - xi_x[:, None]
    dy = Y - xi_y[:, None]
    alpha = np.arctan2(a * dy, b * dx)
    ca, sa = np.cos(alpha), np.sin(alpha)
    # minimiser of sum (dx - a d cos)^2 + (dy - b d sin)^2 over d (no bound), then d >= 1
    d_unc = (a * dx * ca + b * dy * sa) / (a ** 2 * ca ** 2 + b ** 2 * sa ** 2)
    d = np.maximum(1.0, d_unc)
    return alpha, d, d_unc


def project_acceleration(prob, xdd, ydd):
    """Step (16): alpha_a = atan2(y'', x''); d_a = 1-D minimiser clipped to d_a <= a_max."""
    alpha_a = np.arctan2(ydd, xdd)
    d_unc = xdd * np.cos(alpha_a) + ydd * np.sin(alpha_a)
    d_a = np.minimum(prob.a_max, d_unc)
    return alpha_a, d_a


class State:
    """Per-goal iterate: coefficients, multipliers and the split variables."""

    def __init__(self, **kw):
        self.__dict__.update(kw)


def _sweep(prob, st, xi_x, xi_y, b_psi, do_psi_qp):
    """Steps (13)-(16) from the current c_x, c_y: heading QP (optional), v, (alpha, d), (alpha_a, d_a)."""
    P, Pd, Pdd = prob.P, prob.Pd, prob.Pdd
    xd, yd = Pd @ st.c_x, Pd @ st.c_y
    st.theta = np.arctan2(yd, xd)
    if do_psi_qp:
        st.c_psi, _ = solve_psi(prob, st.theta, st.lam_psi, b_psi)
    st.v = project_velocity(prob, xd, yd)
    x, y = P @ st.c_x, P @ st.c_y
    st.alpha, st.d, st.d_unc = project_obstacles(prob, x, y, xi_x, xi_y)
    st.alpha_a, st.d_a = project_acceleration(prob, Pdd @ st.c_x, Pdd @ st.c_y)
    st.psi = P @ st.c_psi


def _g(prob, st, xi_x, xi_y):
    return build_g(xi_x, xi_y, prob.a, prob.b, st.d, st.alpha, st.d_a, st.alpha_a, st.v, st.psi)


def residuals(prob, st, g):
    """Components of F c - g (eq. 8c) per goal, plus the heading surrogate residual.

    r_obs: 2-norm over the obstacle rows of both axes; r_acc: over the P'' rows;
    r_nh: over the P' rows; r_psi: ||atan2(y', x') - P c_psi||.
    """
    m, n = prob.m, prob.n
    c = np.concatenate([st.c_x, st.c_y], axis=0)
    r = prob.F @ c - g
    L = (m + 2) * n
    rx, ry = r[:L], r[L:]
    r_obs = np.sqrt(np.sum(rx[:m * n] ** 2, 0) + np.sum(ry[:m * n] ** 2, 0))
    r_acc = np.sqrt(np.sum(rx[m * n:(m + 1) * n] ** 2, 0) + np.sum(ry[m * n:(m + 1) * n] ** 2, 0))
    r_nh = np.sqrt(np.sum(rx[(m + 1) * n:] ** 2, 0) + np.sum(ry[(m + 1) * n:] ** 2, 0))
    r_psi = np.sqrt(np.sum((st.theta - prob.P @ st.c_psi) ** 2, 0))
    return np.stack([r_obs, r_acc, r_nh, r_psi])


def cold_start(prob, ego, goals):
    """c^0 = argmin 1/2 c^T Q c s.t. A c = b (boundary-only minimum acceleration), lambda^0 = 0."""
    b_xy, b_psi = _xy_rhs_b(prob, ego, goals)
    B = goals.shape[0]
    N = prob.N
    rhs = np.concatenate([np.zeros((2 * N, B)), b_xy], axis=0)
    sol = scipy.linalg.lu_solve(prob.lu_0, rhs)
    return sol[:N], sol[N:2 * N]


def solve(prob, ego, obs, goals, iters, init=None, record=False):
    """Run Algorithm 1 for ``iters`` iterations on every goal of one scene.

    init: None for the cold start, or a dict with c_x, c_y, c_psi, lam_x,
    lam_y, lam_psi (each N x B) to resume from a stored iterate (then the
    heading QP is not re-run before the first iteration; the stored c_psi is
    used as is).

    Returns a State with c_*, lam_*, resid (4 x B, after the last iteration)
    and, if ``record``, hist (iters x 4 x B).
    """
    ego = np.asarray(ego, np.float64)
    goals = np.asarray(goals, np.float64).reshape(-1, 2)
    B = goals.shape[0]
    N = prob.N
    xi_x, xi_y = obstacle_predictions(obs, prob.t)
    b_xy, b_psi = _xy_rhs_b(prob, ego, goals)
    if init is None:
        c_x, c_y = cold_start(prob, ego, goals)
        st = State(c_x=c_x, c_y=c_y, c_psi=np.zeros((N, B)),
                   lam_x=np.zeros((N, B)), lam_y=np.zeros((N, B)), lam_psi=np.zeros((N, B)))
        _sweep(prob, st, xi_x, xi_y, b_psi, do_psi_qp=True)
    else:
        st = State(**{k: np.array(init[k], np.float64) for k in
                      ("c_x", "c_y", "c_psi", "lam_x", "lam_y", "lam_psi")})
        _sweep(prob, st, xi_x, xi_y, b_psi, do_psi_qp=False)
    g = _g(prob, st, xi_x, xi_y)
    hist = []
    st.resid = residuals(prob, st, g)  # of the starting point, replaced after each iteration
    rho = prob.rho
    for _ in range(iters):
        lam_xy = np.concatenate([st.lam_x, st.lam_y], axis=0)
        # (12) x/y QP with the g of the previous iteration
        st.c_x, st.c_y, _ = solve_xy(prob, g, lam_xy, b_xy)
        # (13)-(16)
        _sweep(prob, st, xi_x, xi_y, b_psi, do_psi_qp=True)
        g = _g(prob, st, xi_x, xi_y)
        # multipliers (eqs. 23, 24)
        c = np.concatenate([st.c_x, st.c_y], axis=0)
        lam_xy = lam_xy - rho * prob.F.T @ (prob.F @ c - g)
        st.lam_x, st.lam_y = lam_xy[:N], lam_xy[N:]
        # eq. 24 with the residual taken as (model - target), P c_psi - theta, the
        # same orientation as F c - g in eq. 23: the printed (theta - P c_psi)
        # makes the heading multiplier grow geometrically.
        st.lam_psi = st.lam_psi - rho * prob.P.T @ (prob.P @ st.c_psi - st.theta)
        st.resid = residuals(prob, st, g)
        if record:
            hist.append(st.resid.copy())
    if record:
        st.hist = np.array(hist)
    return st


# ------------------------------------------------------------ ranking (Sec. III-F)


def meta_cost(prob, c_x, c_y, c_psi, kind=0, v_ref=None, w1=1.0, w2=1.0, y_rl=0.0, obs=None, clear_min=0.0):
    """Meta-cost per goal: eq. 25 (kind 0, v_ref = v_cruise) or eq. 26 (kind 1, v_ref = v_max).

    v(t) is the speed of the final trajectory, sqrt(x'^2 + y'^2). A goal whose
    heading P c_psi exceeds psi_max in magnitude at any sample is discarded
    (cost +inf), the post-filter of Sec. III. With clear_min > 0, a goal whose
    trajectory comes closer than clear_min to an obstacle (the clearance of
    `controls`: scaled distance of eq. 1e to the constant-velocity predictions
    of assumption 3) is discarded too.
    """
    v = np.sqrt((prob.Pd @ c_x) ** 2 + (prob.Pd @ c_y) ** 2)
    if kind == 0:
        cost = np.sum((v - v_ref) ** 2, axis=0)
    else:
        y = prob.P @ c_y
        cost = np.sum(w1 * (v - v_ref) ** 2 + w2 * (y - y_rl) ** 2, axis=0)
    psi = prob.P @ c_psi
    bad = np.max(np.abs(psi), axis=0) > prob.psi_max
    if clear_min > 0.0 and obs is not None and np.asarray(obs).size > 0:
        c_x2, c_y2, c_p2 = (np.asarray(u, np.float64).reshape(prob.N, -1) for u in (c_x, c_y, c_psi))
        clear = np.array([controls(prob, obs, c_x2[:, i], c_y2[:, i], c_p2[:, i], 1.0, 1.0)[2]
                          for i in range(c_x2.shape[1])])
        bad = bad | ~(clear >= clear_min)
    return np.where(bad, np.inf, cost)


def best_goal(cost):
    """Lowest index attaining the minimum finite cost, -1 if every goal is filtered."""
    cost = np.asarray(cost, np.float64)
    finite = np.isfinite(cost)
    if not finite.any():
        return -1
    return int(np.flatnonzero(cost == np.min(cost[finite]))[0])


# ------------------------------------------------------------ controls and post-check


def controls(prob, obs, c_x, c_y, c_psi, wheelbase, v_floor):
    """Controls along one trajectory and its clearance from the obstacles.

    Acceleration is the rate of change of speed, v' = (x' x'' + y' y'') / v; the
    steering angle follows the kinematic relation the paper states for
    extracting it (Sec. III): arctan(psi' h / v), h the wheelbase, with v floored
    at v_floor (the speed bound v_min). Clearance is the smallest scaled distance
    sqrt((dx/a)^2 + (dy/b)^2) over all samples and obstacles (constant-velocity
    predictions); a value below 1 is a collision with an obstacle ellipse (eq. 1e).
    Returns (accel[n], steer[n], clearance).
    """
    xd, yd = prob.Pd @ c_x, prob.Pd @ c_y
    xdd, ydd = prob.Pdd @ c_x, prob.Pdd @ c_y
    psid = prob.Pd @ c_psi
    v = np.hypot(xd, yd)
    accel = np.where(v > 0, (xd * xdd + yd * ydd) / np.where(v > 0, v, 1.0), 0.0)
    steer = np.arctan(psid * wheelbase / np.maximum(v, v_floor))
    obs = np.asarray(obs, np.float64).reshape(-1, 4)
    if obs.shape[0] == 0:
        return accel, steer, np.inf
    x, y = prob.P @ c_x, prob.P @ c_y
    t = prob.t
    xi_x = obs[:, 0][None, :] + obs[:, 2][None, :] * t[:, None]
    xi_y = obs[:, 1][None, :] + obs[:, 3][None, :] * t[:, None]
    du = np.sqrt(((x[:, None] - xi_x) / prob.a) ** 2 + ((y[:, None] - xi_y) / prob.b) ** 2)
    return accel, steer, float(du.min())


# ------------------------------------------------------------ closed loop (receding horizon)
#
# One cycle of the receding-horizon use of the planner (Sec. IV: plan, execute
# the start of the chosen trajectory, plan again), on a straight road whose
# traffic follows the Intelligent Driver Model (Treiber, Hennecke and Helbing,
# Phys. Rev. E 62, 2000; its parameters are not given by the paper and are
# chosen here). The cycle period is one sample interval t_f / (n - 1).

IDM_DEFAULTS = dict(a=1.0, b=1.5, s0=2.0, T=1.5, delta=4.0, length=4.5, lane_width=3.5)


def mpc_goals(ego, n_lanes=4, per_lane=64, t_f=10.0, v_floor=5.0, lane_width=3.5):
    """Template goals from the current ego state: lane centres x (ego x + max(|v|,
    v_floor) t_f linspace(0.8, 1.2, per_lane)), lane-major."""
    ego = np.asarray(ego, np.float64)
    v = max(np.hypot(ego[2], ego[3]), v_floor)
    centres = (np.arange(n_lanes) - (n_lanes - 1) // 2) * lane_width
    fr = np.linspace(0.8, 1.2, per_lane)
    g = np.zeros((n_lanes * per_lane, 2))
    for k in range(n_lanes):
        g[k * per_lane:(k + 1) * per_lane, 0] = ego[0] + v * t_f * fr
        g[k * per_lane:(k + 1) * per_lane, 1] = centres[k]
    return g


def right_lane_goals(ego, v_max, n_lanes=4, per_lane=64, t_f=10.0, lane_width=3.5):
    """Goals of the high-speed right-lane scenario (Sec. III-F, for eq. 26): about
    60% of them on the right lane (the lowest y) at different distances, here
    v_max t_f linspace(0.2, 1), the rest spread over the other lanes at v_max t_f
    (from 0.9 v_max t_f up, so that no two coincide), assigned round-robin."""
    ego = np.asarray(ego, np.float64)
    G = n_lanes * per_lane
    n_r = int(np.floor(0.6 * G + 0.5))
    centres = (np.arange(n_lanes) - (n_lanes - 1) // 2) * lane_width
    g = np.zeros((G, 2))
    g[:n_r, 0] = ego[0] + v_max * t_f * np.linspace(0.2, 1.0, n_r)
    g[:n_r, 1] = centres[0]
    others = list(range(1, n_lanes))
    rest = G - n_r
    if not others:  # one lane: the rest at v_max t_f on it
        g[n_r:] = (ego[0] + v_max * t_f, centres[0])
        return g
    per_o = -(-rest // len(others))
    fr = np.linspace(0.9, 1.0, per_o) if per_o > 1 else np.ones(1)
    for r in range(rest):
        g[n_r + r, 0] = ego[0] + v_max * t_f * fr[r // len(others)]
        g[n_r + r, 1] = centres[others[r % len(others)]]
    return g


def idm_accel(v, v_des, gap, dv, p):
    """IDM acceleration; gap = None for a free road."""
    free = 1.0 - (v / v_des) ** p["delta"]
    if gap is None:
        return p["a"] * free
    s_star = p["s0"] + v * p["T"] + v * dv / (2.0 * np.sqrt(p["a"] * p["b"]))
    return p["a"] * (free - (max(s_star, 0.0) / gap) ** 2)


def idm_step(obs, ego, v_des, dt, p):
    """Obstacles after one period: each follows the nearest vehicle ahead in its
    lane (obstacles and the ego; same lane: |dy| < lane width / 2), bumper gap
    x_lead - x - length (at least 0.1 m); speed clipped at 0, ballistic position
    update. Lateral positions and velocities are kept."""
    obs = np.asarray(obs, np.float64).reshape(-1, 4)
    veh = np.vstack([obs[:, :4], np.asarray(ego, np.float64)[None, :4]])
    out = obs.copy()
    for j in range(obs.shape[0]):
        x, y, v = obs[j, 0], obs[j, 1], obs[j, 2]
        lead = None
        for i in range(veh.shape[0]):
            if i == j or abs(veh[i, 1] - y) >= p["lane_width"] / 2 or veh[i, 0] <= x:
                continue
            if lead is None or veh[i, 0] < veh[lead, 0]:
                lead = i
        if lead is None:
            acc = idm_accel(v, v_des[j], None, 0.0, p)
        else:
            gap = max(veh[lead, 0] - x - p["length"], 0.1)
            acc = idm_accel(v, v_des[j], gap, v - veh[lead, 2], p)
        v_new = max(v + acc * dt, 0.0)
        out[j, 0] = x + 0.5 * (v + v_new) * dt
        out[j, 2] = v_new
    return out


def ego_brake(ego, a_max, dt):
    """The ego's fallback when every goal is filtered: it brakes along the road at
    a_max (longitudinal speed floored at zero, the distance covered at the mean of
    the two speeds) and stops moving sideways at its lateral position."""
    ego = np.asarray(ego, np.float64)
    vx = max(ego[2], 0.0)
    vx_new = max(vx - a_max * dt, 0.0)
    return np.array([ego[0] + 0.5 * (vx + vx_new) * dt, ego[1], vx_new, 0.0,
                     -a_max if vx_new < vx else 0.0, 0.0, 0.0, 0.0])


def shift_matrix(n_coef, u0):
    """S with c' = S c: the Bernstein coefficients, on [0, 1], of the polynomial
    u -> sum_k c_k B_k(u0 + u), i.e. the same trajectory seen from a horizon that
    starts u0 t_f later. Found by collocation: both sides agree at n_coef
    distinct points of [0, 1], which fixes a polynomial of degree n_coef - 1."""
    deg = n_coef - 1
    nodes = np.linspace(0.0, 1.0, n_coef)

    def basis(u):
        return np.stack([comb(deg, k) * u ** k * (1.0 - u) ** (deg - k) for k in range(n_coef)], axis=1)

    return np.linalg.solve(basis(nodes), basis(nodes + u0))


def shift_solution(c, u0, dx):
    """Warm start of the next receding-horizon cycle from this cycle's solution.

    c: (3, n_coef, G) coefficients of x, y, psi. Returns c' = S c per axis, with
    x' shifted by -dx (the frame moved dx forward; Bernstein polynomials sum to
    one, so a constant moves every coefficient). The multipliers are not part of
    the map: they are kept as they are.
    """
    c = np.asarray(c, np.float64)
    Smat = shift_matrix(c.shape[1], u0)
    c_new = np.einsum("ik,akg->aig", Smat, c)
    c_new[0] -= np.asarray(dx, np.float64)
    return c_new


def ego_advance(prob, c_x, c_y, c_psi):
    """Ego state one sample into the chosen trajectory: (x, y, x', y', x'', y'', psi, psi')."""
    i = 1
    return np.array([prob.P[i] @ c_x, prob.P[i] @ c_y, prob.Pd[i] @ c_x, prob.Pd[i] @ c_y, prob.Pdd[i] @ c_x,
                     prob.Pdd[i] @ c_y, prob.P[i] @ c_psi, prob.Pd[i] @ c_psi])
