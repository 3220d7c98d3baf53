"""Manufactured-solution pins of the oracle: convergence rates of the decoupled heat
(vector potential) and unsteady Stokes (velocity-pressure) sub-problems."""
import math

import numpy as np

import oracle
from oracle.fem import at_quad


def decoupled_system(n, nt, dt, mu, eta):
    """Zero velocity and constant potential: J splits into Stokes (u, p) and heat (j, A)."""
    ub = np.zeros((nt, 2, (2 * n + 1) ** 2))
    Ab = np.zeros((nt, (n + 1) ** 2))
    return oracle.SpaceTimeSystem(n, nt, dt, mu, eta, 1.0, ub, Ab, jbar=np.zeros_like(Ab))


def test_heat_part_converges_at_second_order_in_space():
    """With the backward-Euler-exact solution A^k = (1 + 2 pi^2 eta dt)^{-k} sin(pi x) sin(pi y)
    of the time-discrete heat equation, the error is purely spatial: O(h^2) for Q1."""
    eta, dt, nt = 1.0, 0.01, 3
    errs = []
    for n in (4, 8, 16):
        sysm = decoupled_system(n, nt, dt, 0.1, eta)
        mesh = sysm.mesh
        t = np.arange(n + 1) / n
        y, x = np.meshgrid(t, t, indexing="ij")
        phi = (np.sin(math.pi * x) * np.sin(math.pi * y)).ravel()[mesh.free1]
        b = np.zeros((nt, sysm.ns))
        b[0, sysm.offs[3]:] = sysm.cb.MA @ phi / dt       # initial condition enters slab 1
        xs = sysm.direct_solve(b.ravel()).reshape(nt, sysm.ns)
        err = 0.0
        for k in range(nt):
            exact = phi * (1 + 2 * math.pi**2 * eta * dt) ** (-(k + 1))
            e = xs[k, sysm.offs[3]:] - exact
            err = max(err, math.sqrt(e @ (sysm.cb.MA @ e)))
        errs.append(err)
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 1.8, (errs, rates)


def test_heat_part_converges_at_first_order_in_time():
    """Against the continuous solution exp(-2 pi^2 eta t) sin sin on a fine mesh: O(dt)."""
    eta, T, n = 1.0, 0.05, 16
    errs = []
    for nt in (2, 4, 8):
        dt = T / nt
        sysm = decoupled_system(n, nt, dt, 0.1, eta)
        mesh = sysm.mesh
        t = np.arange(n + 1) / n
        y, x = np.meshgrid(t, t, indexing="ij")
        phi = (np.sin(math.pi * x) * np.sin(math.pi * y)).ravel()[mesh.free1]
        b = np.zeros((nt, sysm.ns))
        b[0, sysm.offs[3]:] = sysm.cb.MA @ phi / dt
        xs = sysm.direct_solve(b.ravel()).reshape(nt, sysm.ns)
        e = xs[-1, sysm.offs[3]:] - phi * math.exp(-2 * math.pi**2 * eta * T)
        errs.append(math.sqrt(e @ (sysm.cb.MA @ e)))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(0.8 < r < 1.3 for r in rates), (errs, rates)


def _stokes_exact(x, y):
    """u = curl(sin^2(pi x) sin^2(pi y)) (divergence free, zero on the boundary), p = cos cos."""
    pi = math.pi
    ux = pi * np.sin(pi * x) ** 2 * np.sin(2 * pi * y)
    uy = -pi * np.sin(2 * pi * x) * np.sin(pi * y) ** 2
    p = np.cos(pi * x) * np.cos(pi * y)
    # forcing of -mu Lap u + grad p (steady), mu given by caller
    lap_ux = pi * (2 * pi**2 * np.cos(2 * pi * x) * np.sin(2 * pi * y)
                   - 4 * pi**2 * np.sin(pi * x) ** 2 * np.sin(2 * pi * y))
    lap_uy = -pi * (-4 * pi**2 * np.sin(2 * pi * x) * np.sin(pi * y) ** 2
                    + 2 * pi**2 * np.sin(2 * pi * x) * np.cos(2 * pi * y))
    px = -pi * np.sin(pi * x) * np.cos(pi * y)
    py = -pi * np.cos(pi * x) * np.sin(pi * y)
    return ux, uy, p, lap_ux, lap_uy, px, py


def test_stokes_part_converges_at_taylor_hood_rates():
    """Steady state of the unsteady Stokes part started from the exact velocity:
    velocity L2 error O(h^3) and pressure L2 error O(h^2) for Q2-Q1."""
    mu, dt, nt = 1.0, 1.0, 1
    eu, ep = [], []
    for n in (4, 8, 16):
        sysm = decoupled_system(n, nt, dt, mu, 1.0)
        mesh = sysm.mesh
        q2, h = mesh.q2, mesh.h
        # quadrature point coordinates per element
        X = mesh.ex[:, None] * h + q2.s[None] * h
        Yq = mesh.ey[:, None] * h + q2.t[None] * h
        ux, uy, p, lx, ly, px, py = _stokes_exact(X, Yq)
        W = q2.w * h * h
        fx = -mu * lx + px
        fy = -mu * ly + py
        from oracle.fem import assemble_vec
        bx = assemble_vec(mesh.c2, np.einsum("q,mq,eq->em", W, q2.N, fx), mesh.nq2)[mesh.free2]
        by = assemble_vec(mesh.c2, np.einsum("q,mq,eq->em", W, q2.N, fy), mesh.nq2)[mesh.free2]
        t2 = np.arange(2 * n + 1) / (2 * n)
        y2, x2 = np.meshgrid(t2, t2, indexing="ij")
        uxn, uyn, _, _, _, _, _ = _stokes_exact(x2.ravel(), y2.ravel())
        u0 = np.concatenate([uxn[mesh.free2], uyn[mesh.free2]])
        b = np.zeros(sysm.ns)
        b[:sysm.offs[1]] = np.concatenate([bx, by]) + sysm.cb.Mu @ u0 / dt
        xs = sysm.direct_solve(b)
        e = xs[:sysm.offs[1]] - u0
        eu.append(math.sqrt(e @ (sysm.cb.Mu @ e)))
        t1 = np.arange(n + 1) / n
        y1, x1 = np.meshgrid(t1, t1, indexing="ij")
        pe = (np.cos(math.pi * x1) * np.cos(math.pi * y1)).ravel()
        dp = xs[sysm.offs[1]:sysm.offs[2]] - pe
        dp -= (sysm.cb.Mp @ dp).sum()          # both have (near) zero mean; compare modulo constants
        ep.append(math.sqrt(dp @ (sysm.cb.Mp @ dp)))
    ru = [math.log2(eu[i] / eu[i + 1]) for i in range(2)]
    rp = [math.log2(ep[i] / ep[i + 1]) for i in range(2)]
    assert ru[-1] > 2.7, (eu, ru)
    assert rp[-1] > 1.7, (ep, rp)
