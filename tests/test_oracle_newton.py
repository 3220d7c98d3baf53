"""Pins of the oracle's space-time Newton solve (eq. (recurrence) at once).

* The linearisation handed to the linear solver is the derivative of the
  residual: central differences of R at a non-zero iterate reproduce J of the
  state base + x (R is quadratic in the unknowns, so the differences are exact
  up to rounding).  This pins the assembly of the state from base + x,
  including the current, and the slab coupling of the first slab to t_0.
* The forcing rows: a constant electric field gives the row sums of the mass
  matrix on the induction rows (partition of unity); a constant momentum forcing
  gives minus those of the velocity mass matrix.
* The paper's initial current (the discrete current equation of the base
  potential) leaves the current rows with zero residual.
* Newton with exact linear solves converges quadratically to 1e-10 on both
  model problems; with GMRES + P_T to the paper's inner tolerance it still
  reaches 1e-10.
"""
import numpy as np
import pytest

from oracle.fem import Mesh
from oracle.newton import NewtonProblem, initial_current, load_vector, newton_solve
from oracle.blocks import ConstantBlocks
from paper_2309_00768_amd import inputs


def model(name, n, nt, dt):
    prob = inputs.ModelProblem(name, n, nt, dt)
    fl = inputs.model_newton_fields(prob)
    jb = initial_current(n, fl["a_base"], prob.mu0)
    base = (fl["u_base"], fl["p_base"], jb, fl["a_base"])
    return NewtonProblem(n, nt, dt, prob.mu, prob.eta, prob.mu0, base, fl["u_init"], fl["a_init"], None, fl["e"])


def test_linearisation_is_the_derivative_of_the_residual():
    P = model("island", 4, 3, 0.25)
    rng = np.random.default_rng(1)
    x = 0.1 * rng.standard_normal(P.N)
    d = rng.standard_normal(P.N)
    eps = 1e-3
    fd = (P.residual(x + eps * d) - P.residual(x - eps * d)) / (2 * eps)
    Jd = P.linearisation(x).apply_J(d)
    assert np.linalg.norm(fd - Jd) <= 1e-9 * np.linalg.norm(Jd)


def test_forcing_rows_are_mass_row_sums():
    n = 5
    mesh = Mesh(n)
    E = np.ones(mesh.nq1)
    f = np.stack([np.ones(mesh.nq2), np.zeros(mesh.nq2)])
    L = load_vector(mesh, f, E)
    nf2, nf1 = mesh.free2.size, mesh.free1.size
    # integral of an interior Q1 basis function (a hat on four squares): h^2
    assert np.allclose(L[-nf1:], (1.0 / n) ** 2, rtol=1e-13)
    # integral of an interior Q2 basis function, closed form per direction: the
    # 1-D quadratic Lagrange functions integrate to h/6 (end nodes) and 2h/3
    # (midpoint), so a vertex node gets h/3 (two intervals) and a midpoint 2h/3
    h = 1.0 / n
    I = np.arange(1, 2 * n)
    w1 = np.where(I % 2 == 0, h / 3.0, 2.0 * h / 3.0)
    expect = np.outer(w1, w1).ravel()          # row-major: y outer, x inner
    assert np.allclose(L[:nf2], -expect, rtol=1e-13)
    assert np.allclose(L[nf2:2 * nf2], 0.0)


def test_initial_current_zeroes_the_current_rows():
    P = model("tearing", 6, 2, 0.5)
    R = P.residual(np.zeros(P.N)).reshape(P.nt, P.ns)
    o = P.offs
    Rj = R[:, o[2]:o[3]]
    assert np.abs(Rj).max() <= 1e-12 * max(1.0, np.abs(R).max())


@pytest.mark.parametrize("name", ["island", "tearing"])
def test_newton_converges_on_the_model_problems(name):
    P = model(name, 8, 8, 0.125)
    x, hist, its = newton_solve(P, linear="direct")
    assert hist[-1] <= 1e-10 and len(its) <= 4
    # quadratic: the second correction squares the first residual (up to a constant)
    assert hist[2] <= 10.0 * hist[1] ** 2
    x2, hist2, its2 = newton_solve(P, linear="gmres")
    assert hist2[-1] <= 1e-10 and len(its2) <= 8
    assert np.linalg.norm(x2 - x) <= 1e-8 * np.linalg.norm(x)
