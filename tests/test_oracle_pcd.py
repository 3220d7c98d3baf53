"""Pins of the oracle's pressure convection-diffusion blocks, eq. (Fp), against 1-D closed
forms.  The boundary treatment (pure Neumann on all pressure nodes, no Robin term) is a
reading of the paper, which defers it to the authors' earlier work; these tests pin the
arithmetic of that reading: F_p = M_p/dt + W_p(ubar) + mu K_p on every Q1 node, and the
zero-sum K_p solve."""
import numpy as np
import pytest

import oracle
from oracle.blocks import ConstantBlocks, SlabBlocks
from oracle.fem import Mesh


def p1_closed(h):
    """Linear element on an interval of length h: mass, stiffness and the convection matrix
    C[m, n] = int phi_n' phi_m."""
    M = h / 6 * np.array([[2, 1], [1, 2.0]])
    K = 1 / h * np.array([[1, -1], [-1, 1.0]])
    C = np.array([[-0.5, 0.5], [-0.5, 0.5]])
    return M, K, C


def global_1d(n):
    h = 1.0 / n
    Me, Ke, Ce = p1_closed(h)
    M, K, C = (np.zeros((n + 1, n + 1)) for _ in range(3))
    for e in range(n):
        idx = np.arange(e, e + 2)
        M[np.ix_(idx, idx)] += Me
        K[np.ix_(idx, idx)] += Ke
        C[np.ix_(idx, idx)] += Ce
    return M, K, C


@pytest.mark.parametrize("n", [2, 4])
def test_pcd_operator_for_a_constant_velocity_is_a_kronecker_sum(n):
    """With ubar = (a, b) constant, int (ubar . grad psi_n) psi_m = a M (x) C + b C (x) M
    (y factor outer, x fastest), so F_p = M_p/dt + W_p + mu K_p is fixed in closed form."""
    a, b, dt, mu, eta, mu0 = 0.7, -1.3, 0.05, 0.02, 0.03, 1.0
    mesh = Mesh(n)
    cb = ConstantBlocks(mesh, mu0)
    nq2, nq1 = (2 * n + 1) ** 2, (n + 1) ** 2
    ubar = np.stack([np.full(nq2, a), np.full(nq2, b)])
    rng = np.random.default_rng(1)
    sb = SlabBlocks(mesh, cb, ubar, rng.standard_normal(nq1), rng.standard_normal(nq1), dt, mu, eta, mu0)
    M, K, C = global_1d(n)
    Mp = np.kron(M, M)
    Kp = np.kron(K, M) + np.kron(M, K)
    Wp = a * np.kron(M, C) + b * np.kron(C, M)
    np.testing.assert_allclose(sb.Wp.toarray(), Wp, atol=1e-14)
    np.testing.assert_allclose(sb.Fp.toarray(), Mp / dt + Wp + mu * Kp, atol=1e-12)
    # the advection of the potential is the same operator restricted to interior nodes
    inner = mesh.free1
    np.testing.assert_allclose(sb.WA.toarray(), Wp[np.ix_(inner, inner)], atol=1e-14)


def test_neumann_laplacian_solve_returns_the_zero_sum_solution():
    """K_p (all nodes, natural boundary) has the constants as its null space; the bordered
    solve returns the solution of K_p q = r - mean(r) with zero sum."""
    n, nt = 3, 1
    nq2, nq1 = (2 * n + 1) ** 2, (n + 1) ** 2
    rng = np.random.default_rng(4)
    sysm = oracle.SpaceTimeSystem(n, nt, 0.1, 0.01, 0.01, 1.0, rng.standard_normal((nt, 2, nq2)),
                                  rng.standard_normal((nt, nq1)))
    M, K, _ = global_1d(n)
    Kp = np.kron(K, M) + np.kron(M, K)
    np.testing.assert_allclose(Kp @ np.ones(nq1), 0.0, atol=1e-13)
    r = rng.standard_normal(nq1)
    q = sysm.solve_Kp(r)
    assert abs(q.sum()) < 1e-12
    np.testing.assert_allclose(Kp @ q, r - r.mean(), atol=1e-12)
