"""FP64 oracle of the road-attached frame (Sec. III, assumption 1): test
infrastructure only; the product path never imports it.

The frame is defined directly, without the closed forms of circular arcs that
the device uses:
  * the centre-line C(s) is the curve whose heading theta(s) is the integral of
    the curvature from the start pose; its position is integrated numerically
    (adaptive Gauss-Kronrod, scipy.integrate.quad) segment by segment, and it is
    continued straight before its start and after its end;
  * the road coordinates of a point p are the arc length s of the closest point
    of the centre-line (the nearest vertex of a 0.05 m polyline, refined by
    Brent's root finder on (p - C(s)) . T(s) = 0 with C by quadrature) and
    d = (p - C(s)) . N(s), N the left normal;
  * rates are time derivatives of (s, d) and of the heading along the vehicle's
    motion p(t) = p + v t + a t^2 / 2, taken by central differences with one
    Richardson step (valid away from the joints, where the curvature jumps).
Parity unpinned parts: none; tests/test_frenet_oracle.py pins every function
against closed forms of straight and circular roads.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, optimize


class RoadOracle:
    def __init__(self, segments, x0=0.0, y0=0.0, theta0=0.0):
        self.seg = np.asarray(segments, np.float64).reshape(-1, 2)
        self.start = (float(x0), float(y0), float(theta0))
        self.S = np.concatenate([[0.0], np.cumsum(self.seg[:, 0])])
        # heading at every segment start and position by quadrature
        th = [self.start[2]]
        for L, k in self.seg:
            th.append(th[-1] + k * L)
        self.th = np.array(th)
        pos = [(self.start[0], self.start[1])]
        for i, (L, k) in enumerate(self.seg):
            t0 = self.th[i]
            dx = integrate.quad(lambda u: math.cos(t0 + k * u), 0.0, L, epsabs=1e-13, epsrel=1e-13)[0]
            dy = integrate.quad(lambda u: math.sin(t0 + k * u), 0.0, L, epsabs=1e-13, epsrel=1e-13)[0]
            pos.append((pos[-1][0] + dx, pos[-1][1] + dy))
        self.pos = np.array(pos)

    @property
    def length(self):
        return float(self.S[-1])

    def heading(self, s):
        if s < 0.0:
            return self.th[0]
        if s >= self.length:
            return self.th[-1]
        i = int(np.searchsorted(self.S, s, side="right") - 1)
        return self.th[i] + self.seg[i, 1] * (s - self.S[i])

    def curvature(self, s):
        if s < 0.0 or s > self.length:
            return 0.0
        i = min(int(np.searchsorted(self.S, s, side="right") - 1), len(self.seg) - 1)
        return float(self.seg[i, 1])

    def point(self, s):
        """C(s) by quadrature from the start of s's segment."""
        if s < 0.0:
            t = self.th[0]
            return self.pos[0] + s * np.array([math.cos(t), math.sin(t)])
        if s >= self.length:
            t = self.th[-1]
            return self.pos[-1] + (s - self.length) * np.array([math.cos(t), math.sin(t)])
        i = int(np.searchsorted(self.S, s, side="right") - 1)
        t0, k, u = self.th[i], self.seg[i, 1], s - self.S[i]
        dx = integrate.quad(lambda w: math.cos(t0 + k * w), 0.0, u, epsabs=1e-13, epsrel=1e-13)[0]
        dy = integrate.quad(lambda w: math.sin(t0 + k * w), 0.0, u, epsabs=1e-13, epsrel=1e-13)[0]
        return self.pos[i] + np.array([dx, dy])

    def to_global(self, s, d):
        c = self.point(s)
        t = self.heading(s)
        return np.array([c[0] - d * math.sin(t), c[1] + d * math.cos(t), t])

    def _polyline(self, ext):
        """A fine polyline of the centre-line (0.05 m steps, cumulative trapezoid of
        (cos theta, sin theta)) for the coarse search only."""
        if getattr(self, "_poly_ext", -1.0) >= ext:
            return self._grid, self._pts
        grid = np.arange(-ext, self.length + ext + 0.05, 0.05)
        th = np.array([self.heading(s) for s in grid])
        c, sn = np.cos(th), np.sin(th)
        dx = np.concatenate([[0.0], np.cumsum(0.5 * (c[1:] + c[:-1]) * np.diff(grid))])
        dy = np.concatenate([[0.0], np.cumsum(0.5 * (sn[1:] + sn[:-1]) * np.diff(grid))])
        p0 = self.point(grid[0])
        self._grid, self._pts, self._poly_ext = grid, np.stack([p0[0] + dx, p0[1] + dy], 1), ext
        return self._grid, self._pts

    def project(self, x, y):
        """(s, d) of the closest centre-line point."""
        p = np.array([x, y], np.float64)
        grid, pts = self._polyline(max(200.0, 2.0 * float(np.hypot(*(p - self.pos[0])))))
        j = int(np.argmin(np.sum((pts - p) ** 2, axis=1)))
        # the foot point: (p - C(s)) . T(s) = 0, a sign change around the nearest
        # vertex (a root is found to ~1e-12 m; minimising the squared distance would
        # only locate s to the square root of its rounding)
        g = lambda s: float((p - self.point(s)) @ np.array([math.cos(self.heading(s)), math.sin(self.heading(s))]))
        lo, hi = grid[j] - 0.5, grid[j] + 0.5
        if g(lo) > 0 > g(hi):
            s = optimize.brentq(g, lo, hi, xtol=1e-13, rtol=4 * np.finfo(float).eps)
        else:
            f = lambda s: float(np.sum((self.point(s) - p) ** 2))
            s = optimize.minimize_scalar(f, bounds=(lo, hi), method="bounded", options={"xatol": 1e-11}).x
        s = float(s)
        t = self.heading(s)
        c = self.point(s)
        d = -(p[0] - c[0]) * math.sin(t) + (p[1] - c[1]) * math.cos(t)
        return s, d

    def from_global(self, state, eps=1e-3):
        """Obstacle [x, y, vx, vy] -> [s, d, s', d']; ego [8] -> [s, d, s', d', s'', d'',
        psi_road, psi_road'], rates by central differences along the motion."""
        st = np.asarray(state, np.float64)
        x, y, vx, vy = st[:4]
        ax, ay = (st[4], st[5]) if st.size == 8 else (0.0, 0.0)

        def sd_at(t):
            return np.array(self.project(x + vx * t + 0.5 * ax * t * t, y + vy * t + 0.5 * ay * t * t))

        z = sd_at(0.0)
        # central differences with one Richardson step (truncation O(h^4))
        def first(f, h):
            return (4 * (f(h / 2) - f(-h / 2)) / h - (f(h) - f(-h)) / (2 * h)) / 3

        def second(f, h):
            f0 = f(0.0)
            return (4 * (f(h / 2) - 2 * f0 + f(-h / 2)) / (h / 2) ** 2 - (f(h) - 2 * f0 + f(-h)) / h ** 2) / 3

        rate = first(sd_at, 2 * eps)
        out = [z[0], z[1], rate[0], rate[1]]
        if st.size == 8:
            # the second difference over a 10x longer step (rounding of the
            # minimiser's s, ~1e-11, would dominate at eps)
            acc = second(sd_at, 20 * eps)
            psi, psid = st[6], st[7]
            th_at = lambda t: self.heading(sd_at(t)[0])
            out += [acc[0], acc[1], psi - self.heading(z[0]), psid - first(th_at, 2 * eps)]
        return np.array(out)

    def trajectory_to_global(self, s_of_t, d_of_t, times, eps=1e-4):
        """Global (X, Y, heading of motion) of a road-frame trajectory given as functions of t."""
        out = []
        for t in times:
            g = self.to_global(s_of_t(t), d_of_t(t))
            at = lambda h: self.to_global(s_of_t(t + h), d_of_t(t + h))[:2]
            vel = (4 * (at(eps / 2) - at(-eps / 2)) / eps - (at(eps) - at(-eps)) / (2 * eps)) / 3
            out.append([g[0], g[1], math.atan2(vel[1], vel[0])])
        return np.array(out)
