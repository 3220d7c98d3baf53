"""Parallel-in-time solves of the two sweeps inside P_T (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).  Plain float64 NumPy/SciPy.

P_T^{-1} applies two block lower-triangular space-time solves by forward
substitution in time: F_u of eq. (STFu), first order in time, and C_A of
eqs. (CAspacetime)/(CAs), second order.  The paper leaves solving these
single-variable space-time systems in parallel to future work (Conclusions, and
the footnote of Sec. "Comparison with single time-step block preconditioner"),
with multigrid in time among the candidates it cites.  This module takes the
simplest two-level member of that family, Parareal (Lions, Maday and Turinici,
2001), with a coarse propagator that takes the same slabs but a cheaper spatial
solve.

A slab step is an update over a predictor from the earlier slabs:

    F_u:  x^k = x^{k-1} + S_k(g^k - A_k x^{k-1}),         A_k = F_u,k - M_u/dt,
    C_A:  y^k = p^k + S_k(s^k + C1_{k-1}/dt y^{k-1} - C2/dt^2 y^{k-2} - C0_k p^k),
          p^k = 2 y^{k-1} - y^{k-2} (k >= 2), y^0 (k = 1), 0 (k = 0),

with S_k a solve with the diagonal block (F_u,k or C0_k).  With exact S_k both
are the forward substitutions of ``SpaceTimeSystem.solve_Fu`` / ``solve_CA``.
The fine propagator F_k uses an accurate S_k, the coarse G_k a few
Chebyshev-Jacobi steps.  Parareal, iteration j -> j+1:

    x_{j+1}^k = G_k(x_{j+1}^{<k}) + F_k(x_j^{<k}) - G_k(x_j^{<k}),

starting from the coarse sweep x_0.  The corrections F_k - G_k of all slabs are
independent of each other (the time-parallel part); the coarse sweep stays
sequential.  After j iterations the first j slabs equal the fine sweep, after nt
iterations all of them do.
"""
from __future__ import annotations

import copy

import numpy as np


def chebyshev_jacobi(A, dinv, r, deg, theta, delta):
    """deg steps of the Chebyshev iteration for A x = r from x = 0, preconditioned
    by D^{-1} = diag(dinv), for D^{-1} A with eigenvalues in [theta - delta,
    theta + delta] (Saad, Iterative Methods for Sparse Linear Systems, Sec. 12.3):
    d_0 = D^{-1} r / theta; then r_i = r_{i-1} - A d_{i-1},
    rho_i = 1 / (2 sigma - rho_{i-1}) with sigma = theta / delta, rho_0 = 1 / sigma,
    d_i = rho_i rho_{i-1} d_{i-1} + (2 rho_i / delta) D^{-1} r_i; x = sum of the d_i.

    delta <= 0 stands for an ellipse with imaginary foci theta -+ i|delta|
    (Manteuffel, Numer. Math. 28, 1977): the same recursion with c = i|delta| in
    place of delta, written in g_i = rho_i / c so that only c^2 = -delta^2 enters:
    g_0 = 1 / theta, g_i = 1 / (2 theta - c^2 g_{i-1}),
    d_i = c^2 g_i g_{i-1} d_{i-1} + 2 g_i D^{-1} r_i."""
    res = np.array(r, dtype=np.float64)
    d = dinv * res / theta
    x = d.copy()
    if delta <= 0.0:
        csq = -delta * delta
        g = 1.0 / theta
        for _ in range(1, deg):
            res = res - A @ d
            g_new = 1.0 / (2.0 * theta - csq * g)
            d = csq * g_new * g * d + 2.0 * g_new * (dinv * res)
            g = g_new
            x = x + d
        return x
    sigma = theta / delta
    rho = 1.0 / sigma
    for _ in range(1, deg):
        res = res - A @ d
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * (dinv * res)
        rho = rho_new
        x = x + d
    return x


class SweepSteps:
    """The slab steps of the F_u and C_A sweeps of a ``SpaceTimeSystem``."""

    def __init__(self, sysm):
        self.sysm = sysm
        self.nt, self.dt = sysm.nt, sysm.dt
        self.C0, self.C1, self.C2 = sysm.wave_blocks()

    # spatial solves -----------------------------------------------------
    def exact_fu(self, k, r):
        s = self.sysm
        return s._factor(("Fu", k), lambda: s.slabs[k].Fu).solve(r)

    def exact_ca(self, k, r):
        return self.sysm._factor(("CA", k), lambda: self.C0[k]).solve(r)

    def cheb_fu(self, deg, intervals):
        """S_k = deg Chebyshev-Jacobi steps on F_u,k with (theta, delta) = intervals[k]."""
        def solve(k, r):
            A = self.sysm.slabs[k].Fu
            return chebyshev_jacobi(A, 1.0 / A.diagonal(), r, deg, *intervals[k])
        return solve

    def cheb_ca(self, deg, intervals):
        def solve(k, r):
            A = self.C0[k]
            return chebyshev_jacobi(A, 1.0 / A.diagonal(), r, deg, *intervals[k])
        return solve

    # slab steps (prev = (x^{k-1}, x^{k-2}), zero before the first slab) -----
    def fu_step(self, k, prev, g, solve):
        if k == 0:
            return solve(0, g)
        s, x1 = self.sysm, prev[0]
        r = g - s.slabs[k].Fu @ x1 + s.cb.Mu @ x1 / self.dt
        return x1 + solve(k, r)

    def ca_step(self, k, prev, s_k, solve):
        dt = self.dt
        y1, y2 = prev
        if k == 0:
            return solve(0, s_k)
        r = s_k + self.C1[k - 1] @ y1 / dt
        if k >= 2:
            r = r - self.C2 @ y2 / dt**2
            p = 2.0 * y1 - y2
        else:
            p = y1
        return p + solve(k, r - self.C0[k] @ p)


def _prev(x, k):
    z = np.zeros_like(x[0])
    return (x[k - 1] if k >= 1 else z, x[k - 2] if k >= 2 else z)


def sweep(step, rhs, solve):
    """Sequential sweep: x^k = step(k, (x^{k-1}, x^{k-2}), rhs^k, solve)."""
    x = np.zeros_like(rhs)
    for k in range(rhs.shape[0]):
        x[k] = step(k, _prev(x, k), rhs[k], solve)
    return x


def parareal(step, rhs, fine, coarse, iters):
    """Parareal with fine / coarse spatial solves; returns every iterate x_0..x_iters."""
    nt = rhs.shape[0]
    x = sweep(step, rhs, coarse)
    out = [x]
    for _ in range(iters):
        corr = np.array([step(k, _prev(x, k), rhs[k], fine) - step(k, _prev(x, k), rhs[k], coarse)
                         for k in range(nt)])
        xn = np.zeros_like(rhs)
        for k in range(nt):
            xn[k] = step(k, _prev(xn, k), rhs[k], coarse) + corr[k]
        x = xn
        out.append(x)
    return out


def apply_PT_inv_parareal(sysm, r, iters, fu_coarse, ca_coarse, fu_fine=None, ca_fine=None, normalise=True):
    """P_T^{-1} r of eq. (PT) with both sweeps taken by ``iters`` Parareal
    iterations (fine: exact solves unless given)."""
    st = SweepSteps(sysm)
    fu_fine = fu_fine or st.exact_fu
    ca_fine = ca_fine or st.exact_ca
    proxy = copy.copy(sysm)
    proxy.solve_Fu = lambda q: parareal(st.fu_step, q, fu_fine, fu_coarse, iters)[-1]
    proxy.solve_CA = lambda s: parareal(st.ca_step, s, ca_fine, ca_coarse, iters)[-1]
    return proxy.apply_PT_inv(r, normalise=normalise)
