"""Pins of the oracle's finite-element layer against closed forms and identities."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from oracle.blocks import ConstantBlocks, SlabBlocks, mean_field
from oracle.fem import Mesh, RefSquare


def p1_closed(h):
    """Textbook linear-element mass and stiffness on an interval of length h."""
    return h / 6 * np.array([[2, 1], [1, 2.0]]), 1 / h * np.array([[1, -1], [-1, 1.0]])


def p2_closed(h):
    """Textbook quadratic-element mass and stiffness (nodes at 0, h/2, h)."""
    M = h / 30 * np.array([[4, 2, -1], [2, 16, 2], [-1, 2, 4.0]])
    K = 1 / (3 * h) * np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7.0]])
    return M, K


def global_1d(n, deg):
    """Global 1-D mass/stiffness on [0,1] with n cells, assembled from the closed forms."""
    h = 1.0 / n
    Me, Ke = p1_closed(h) if deg == 1 else p2_closed(h)
    nn = deg * n + 1
    M = np.zeros((nn, nn))
    K = np.zeros((nn, nn))
    for e in range(n):
        idx = np.arange(deg * e, deg * e + deg + 1)
        M[np.ix_(idx, idx)] += Me
        K[np.ix_(idx, idx)] += Ke
    return M, K


@pytest.mark.parametrize("n", [1, 3, 4])
def test_mass_stiffness_are_kronecker_products(n):
    mesh = Mesh(n)
    cb = ConstantBlocks(mesh, 1.0)
    for deg, Mg, Kg in [(1, cb.M1full, cb.K1full), (2, cb.M2full, cb.K2full)]:
        M1, K1 = global_1d(n, deg)
        # x fastest: global index = ix + (deg n + 1) iy, so the y factor is the outer one.
        np.testing.assert_allclose(Mg.toarray(), np.kron(M1, M1), atol=1e-14)
        np.testing.assert_allclose(Kg.toarray(), np.kron(K1, M1) + np.kron(M1, K1), atol=1e-12)


def test_basis_partition_of_unity_and_nodal():
    for deg in (1, 2):
        ref = RefSquare(deg)
        np.testing.assert_allclose(ref.N.sum(axis=0), 1.0, atol=1e-14)
        np.testing.assert_allclose(ref.Ns.sum(axis=0), 0.0, atol=1e-13)
        np.testing.assert_allclose(ref.Nt.sum(axis=0), 0.0, atol=1e-13)
    v, _ = oracle.lagrange1d(2, np.array([0.0, 0.5, 1.0]))
    np.testing.assert_allclose(v, np.eye(3), atol=1e-15)


def test_quadrature_exactness():
    s, w = oracle.gauss01(5)
    for d in range(10):
        assert abs(np.sum(w * s**d) - 1.0 / (d + 1)) < 1e-15


def test_divergence_kills_constants_and_area():
    mesh = Mesh(5)
    cb = ConstantBlocks(mesh, 1.0)
    # B^T 1 = -int div(phi) = 0 for velocity basis functions vanishing on the boundary.
    np.testing.assert_allclose(cb.B.T @ np.ones(cb.B.shape[0]), 0.0, atol=1e-14)
    # Neumann stiffness annihilates constants; masses integrate to the area.
    np.testing.assert_allclose(cb.K1full @ np.ones(mesh.nq1), 0.0, atol=1e-12)
    np.testing.assert_allclose(cb.K2full @ np.ones(mesh.nq2), 0.0, atol=1e-12)
    assert abs(cb.M1full.sum() - 1.0) < 1e-13 and abs(cb.M2full.sum() - 1.0) < 1e-13


def test_divergence_of_q2_field_is_exact():
    # u = (x(1-x)y(1-y), 0) lies in the interior Q2 space, so B u = -int psi d/dx[x(1-x)] y(1-y).
    mesh = Mesh(4)
    cb = ConstantBlocks(mesh, 1.0)
    x2, y2 = oracle_coords(mesh)
    u = np.concatenate([(x2 * (1 - x2) * y2 * (1 - y2))[mesh.free2], np.zeros(mesh.free2.size)])
    ref = -load_q1(mesh, lambda x, y: (1 - 2 * x) * y * (1 - y))
    np.testing.assert_allclose(cb.B @ u, ref, atol=1e-14)


def oracle_coords(mesh):
    t = np.arange(2 * mesh.n + 1) / (2.0 * mesh.n)
    y, x = np.meshgrid(t, t, indexing="ij")
    return x.ravel(), y.ravel()


def load_q1(mesh, fn):
    """int fn chi_m over the mesh by an independent 8-point rule per direction."""
    s, w = np.polynomial.legendre.leggauss(8)
    s, w = (s + 1) / 2, w / 2
    out = np.zeros(mesh.nq1)
    h = mesh.h
    for e in range(mesh.ne):
        x0, y0 = mesh.ex[e] * h, mesh.ey[e] * h
        for a in range(8):
            for b in range(8):
                X, Yq = x0 + s[a] * h, y0 + s[b] * h
                chi = [(1 - s[a]) * (1 - s[b]), s[a] * (1 - s[b]), (1 - s[a]) * s[b], s[a] * s[b]]
                f = fn(X, Yq) * w[a] * w[b] * h * h
                for i in range(4):
                    out[mesh.c1[e, i]] += f * chi[i]
    return out


def test_advection_is_skew_for_divergence_free_state():
    # u = (a + b y + c x, d + e x - c y) is divergence free and exactly representable in Q2;
    # with test/trial functions vanishing on the boundary, W + W^T = -int div(u) phi phi = 0.
    n = 4
    mesh = Mesh(n)
    cb = ConstantBlocks(mesh, 1.0)
    x2, y2 = oracle_coords(mesh)
    ub = np.stack([0.3 + 0.7 * y2 + 0.2 * x2, -0.1 + 0.5 * x2 - 0.2 * y2])
    Ab = np.zeros(mesh.nq1)
    s = SlabBlocks(mesh, cb, ub, Ab, np.zeros(mesh.nq1), 0.1, 0.01, 0.01, 1.0)
    W = s.Wu.toarray()
    np.testing.assert_allclose(W + W.T, 0.0, atol=1e-13)
    WA = s.WA.toarray()
    np.testing.assert_allclose(WA + WA.T, 0.0, atol=1e-13)
    # Constant potential => no magnetic coupling blocks.
    assert abs(s.Zj).max() == 0 and abs(s.ZA).max() == 0 and abs(s.Y).max() == 0


def test_y_is_transpose_of_zj():
    # Y_{m n} = int (phi_n . grad A) chi_m and Zj_{m n} = int chi_n (grad A . phi_m).
    mesh = Mesh(3)
    cb = ConstantBlocks(mesh, 1.0)
    rng = np.random.default_rng(3)
    s = SlabBlocks(mesh, cb, rng.standard_normal((2, mesh.nq2)), rng.standard_normal(mesh.nq1),
                   rng.standard_normal(mesh.nq1), 0.1, 0.01, 0.01, 1.0)
    np.testing.assert_allclose(s.Y.toarray(), s.Zj.toarray().T[mesh.free1], atol=1e-14)


def test_mean_field_closed_form_shear_layer():
    # Bbar depends only on boundary values: for A = tanh((y-1/2)/0.1) + 0.01 cos(pi x),
    # the Q1 interpolant gives Bbar = (2 tanh 5, 0.02) exactly.
    for n in (4, 7, 32):
        mesh = Mesh(n)
        t = np.arange(n + 1) / n
        y, x = np.meshgrid(t, t, indexing="ij")
        A = (np.tanh((y - 0.5) / 0.1) + 0.01 * np.cos(math.pi * x)).ravel()
        np.testing.assert_allclose(mean_field(mesh, A), [2 * math.tanh(5.0), 0.02], rtol=0, atol=1e-13)
