"""Pins of the oracle's Jacobian: finite differences of the recurrence residual and the
force balance of the paper's equilibria."""
import math

import numpy as np
import pytest

import oracle
from oracle.fem import Mesh
from oracle.nonlinear import slab_residual, spacetime_residual


def _random_fields(n, nt, seed):
    rng = np.random.default_rng(seed)
    nq2, nq1 = (2 * n + 1) ** 2, (n + 1) ** 2
    return (rng.standard_normal((nt, 2, nq2)), rng.standard_normal((nt, nq1)),
            rng.standard_normal((nt, nq1)), rng.standard_normal((nt, nq1)))


@pytest.mark.parametrize("n,nt", [(2, 2), (3, 3)])
def test_jacobian_equals_central_difference_of_residual(n, nt):
    """The residual is quadratic in the unknowns, so central differences are exact:
    J x = (R(base + e x) - R(base - e x)) / (2 e).  This pins every sign and placement
    of the coupling blocks (Z_j acts on j, Z_A on A) and the Newton term."""
    dt, mu, eta, mu0 = 0.1, 0.03, 0.02, 0.7
    bu, bp, bj, bA = _random_fields(n, nt, 11)
    sysm = oracle.SpaceTimeSystem(n, nt, dt, mu, eta, mu0, bu, bA, jbar=bj)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(sysm.N)
    u_init = rng.standard_normal((2, (2 * n + 1) ** 2))
    A_init = rng.standard_normal((n + 1) ** 2)
    eps = 1e-3
    Rp = spacetime_residual(sysm, (bu, bp, bj, bA), eps * x, u_init, A_init)
    Rm = spacetime_residual(sysm, (bu, bp, bj, bA), -eps * x, u_init, A_init)
    fd = (Rp - Rm) / (2 * eps)
    Jx = sysm.apply_J(x)
    assert np.linalg.norm(fd - Jx) <= 1e-10 * np.linalg.norm(Jx)
    # and the assembled matrix agrees with the apply
    J = sysm.assemble_J()
    np.testing.assert_allclose(J @ x, Jx, rtol=0, atol=1e-12 * np.abs(Jx).max())


def test_single_slab_is_single_step_jacobian():
    n = 3
    bu, _, bj, bA = _random_fields(n, 1, 2)
    sysm = oracle.SpaceTimeSystem(n, 1, 0.2, 0.1, 0.1, 1.0, bu, bA, jbar=bj)
    assert abs(sysm.assemble_J() - sysm.slab_jacobian(0)).max() == 0.0


def test_jacobian_is_block_lower_bidiagonal_in_time():
    n, nt = 2, 4
    bu, _, bj, bA = _random_fields(n, nt, 3)
    sysm = oracle.SpaceTimeSystem(n, nt, 0.1, 0.1, 0.1, 1.0, bu, bA, jbar=bj)
    J = sysm.assemble_J().toarray()
    ns = sysm.ns
    for k in range(nt):
        for l in range(nt):
            blk = J[k * ns:(k + 1) * ns, l * ns:(l + 1) * ns]
            if l not in (k, k - 1):
                assert np.abs(blk).max() == 0.0
    # sub-diagonal coupling is -M/dt on u and A only
    sub = J[ns:2 * ns, 0:ns]
    o = sysm.offs
    np.testing.assert_allclose(sub[o[0]:o[1], o[0]:o[1]], -sysm.cb.Mu.toarray() / 0.1)
    np.testing.assert_allclose(sub[o[3]:o[4], o[3]:o[4]], -sysm.cb.MA.toarray() / 0.1)
    assert np.abs(sub[o[1]:o[3], :]).max() == 0.0
    assert np.abs(sub[o[0]:o[1], o[1]:]).max() == 0.0 and np.abs(sub[o[3]:, :o[3]]).max() == 0.0


def _harris_fields(n, lam=5.0, mu0=1.0):
    """Interpolants of the Harris-sheet equilibrium (paper, tearing-mode problem),
    shifted so that the current sheet sits at y = 1/2 of the unit square."""
    t = np.arange(n + 1) / n
    y, x = np.meshgrid(t, t, indexing="ij")
    z = lam * (y - 0.5)
    A = (np.log(np.cosh(z)) / lam).ravel()
    j = (lam / np.cosh(z) ** 2 / mu0).ravel()             # j = Laplacian(A) / mu0
    p = (1.0 / (2 * mu0) / np.cosh(z) ** 2).ravel()
    return p, j, A


def _fadeev_fields(n, beta=0.2, mu0=1.0):
    """Interpolants of the island-coalescence (Fadeev) equilibrium of the paper."""
    t = np.arange(n + 1) / n
    y, x = np.meshgrid(t, t, indexing="ij")
    d = np.cosh(2 * math.pi * y) + beta * np.cos(2 * math.pi * x)
    A = (np.log(d) / (2 * math.pi)).ravel()
    j = (2 * math.pi * (1 - beta**2) / d**2 / mu0).ravel()
    p = ((1 - beta**2) / (2 * mu0) / d**2).ravel()
    return p, j, A


@pytest.mark.parametrize("fields", [_harris_fields, _fadeev_fields])
def test_equilibria_balance_lorentz_force(fields):
    """With u = 0, the momentum residual of an exact equilibrium reduces to
    grad p + j grad A, which vanishes for the paper's equilibria.  The discrete residual
    must go to zero under refinement relative to the pressure force alone.  With the
    opposite sign of the Lorentz term it would not."""
    ratios = []
    for n in (8, 16, 32):
        mesh = Mesh(n)
        p, j, A = fields(n)
        u0 = np.zeros((2, mesh.nq2))
        R = slab_residual(mesh, (u0, p, j, A), (u0, A), 1.0, 1.0, 1.0, 1.0)
        Rp_only = slab_residual(mesh, (u0, p, np.zeros_like(j), A), (u0, A), 1.0, 1.0, 1.0, 1.0)
        nu = 2 * mesh.free2.size
        ratios.append(np.linalg.norm(R[:nu]) / np.linalg.norm(Rp_only[:nu]))
    assert ratios[0] < 0.2
    assert ratios[1] < ratios[0] / 3 and ratios[2] < ratios[1] / 3
