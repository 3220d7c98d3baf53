"""Pins of the oracle's parallel-in-time sweeps (Parareal over the slab steps of
the F_u and C_A sweeps of P_T).

* Chebyshev-Jacobi: after d steps from zero the preconditioned residual is the
  scaled Chebyshev polynomial T_d((theta - t) / delta) / T_d(theta / delta) of
  D^{-1} A applied to the first one (checked through the eigendecomposition of
  the symmetric D^{-1/2} A D^{-1/2}, with T_d from numpy's Chebyshev series);
  with imaginary foci theta -+ i c the same with i c for delta, checked on a
  non-normal matrix with complex eigenvalues.
* The slab steps with exact spatial solves are the forward substitutions of
  P_T's sweeps (``solve_Fu``, ``solve_CA``).
* Parareal's finite termination: after j iterations the first j slabs are the
  fine sweep's, after nt iterations every slab is, whatever the coarse solve.
* With nt iterations the P_T^{-1} built on the Parareal sweeps is P_T^{-1}.
"""
import numpy as np
import pytest
from numpy.polynomial import chebyshev as C

import oracle
from oracle import paratime
from paper_2309_00768_amd import inputs


def small_system(n, nt):
    cfg = inputs.Config("pt", n, nt, 0.1, 20.0, 30.0)
    ub, Ab = inputs.state(cfg)
    return oracle.SpaceTimeSystem(n, nt, cfg.dt, cfg.mu, cfg.eta, 1.0, ub * 3.0, Ab * 3.0)


def jacobi_interval(A):
    """Range of the real parts of the eigenvalues of D^{-1} A, widened by 10% (any
    interval serves a coarse propagator: Parareal terminates whatever it is)."""
    d = A.diagonal()
    ev = np.linalg.eigvals((A.toarray() if hasattr(A, "toarray") else A) / d[:, None]).real
    lo, hi = 0.9 * ev.min(), 1.1 * ev.max()
    return 0.5 * (hi + lo), 0.5 * (hi - lo)


@pytest.mark.parametrize("deg", [1, 2, 3, 6])
def test_chebyshev_jacobi_is_the_chebyshev_residual_polynomial(deg):
    rng = np.random.default_rng(3)
    n = 12
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T + n * np.diag(rng.uniform(1.0, 3.0, n))
    d = np.diag(A)
    Dh = 1.0 / np.sqrt(d)
    lam, V = np.linalg.eigh(Dh[:, None] * A * Dh[None, :])
    theta, delta = 0.5 * (lam.max() * 1.05 + lam.min() * 0.95), 0.5 * (lam.max() * 1.05 - lam.min() * 0.95)
    r = rng.standard_normal(n)
    x = paratime.chebyshev_jacobi(A, 1.0 / d, r, deg, theta, delta)
    Td = np.zeros(deg + 1)
    Td[deg] = 1.0
    p = C.chebval((theta - lam) / delta, Td) / C.chebval(theta / delta, Td)
    # x = A^{-1} (I - p(D^{-1} A)) r, in the symmetric frame
    x_ref = Dh * (V @ (((1.0 - p) / lam) * (V.T @ (Dh * r))))
    assert np.allclose(x, x_ref, rtol=1e-12, atol=1e-12 * np.abs(x_ref).max())


@pytest.mark.parametrize("deg", [1, 2, 5, 9])
def test_chebyshev_jacobi_on_an_ellipse_with_imaginary_foci(deg):
    """A non-normal D^{-1} A with eigenvalues well off the real axis, foci
    theta -+ i c: the residual polynomial is T_d((theta - lambda)/(i c)) /
    T_d(theta/(i c)), evaluated through the (complex) eigendecomposition."""
    rng = np.random.default_rng(8)
    n = 10
    # eigenvalues 1 +- 0.6i, 0.8 +- 0.4i, ... as 2x2 rotation blocks, in a random basis
    blocks = np.zeros((n, n))
    for k in range(n // 2):
        re, im = 0.7 + 0.1 * k, 0.2 + 0.15 * k
        blocks[2 * k:2 * k + 2, 2 * k:2 * k + 2] = [[re, im], [-im, re]]
    Q = rng.standard_normal((n, n)) + 3 * np.eye(n)
    M = Q @ blocks @ np.linalg.inv(Q)          # D^{-1} A
    d = rng.uniform(1.0, 2.0, n)
    A = d[:, None] * M
    lam, V = np.linalg.eig(M)
    assert np.abs(lam.imag).max() > 0.5
    theta, c = 0.9, 0.5                          # foci 0.9 -+ 0.5i
    r = rng.standard_normal(n)
    x = paratime.chebyshev_jacobi(A, 1.0 / d, r, deg, theta, -c)
    Td = np.zeros(deg + 1)
    Td[deg] = 1.0
    p = C.chebval((theta - lam) / (1j * c), Td) / C.chebval(theta / (1j * c), Td)
    # x = A^{-1} (I - p(D^{-1} A)) r = M^{-1} (I - p(M)) D^{-1} r
    y = np.linalg.solve(V, r / d)
    x_ref = (V @ (((1.0 - p) / lam) * y)).real
    assert np.allclose(x, x_ref, rtol=1e-10, atol=1e-10 * np.abs(x_ref).max())


def test_slab_steps_with_exact_solves_are_the_forward_substitutions():
    s = small_system(4, 5)
    st = paratime.SweepSteps(s)
    rng = np.random.default_rng(4)
    g = rng.standard_normal((s.nt, s.nu))
    a = rng.standard_normal((s.nt, s.na))
    assert np.allclose(paratime.sweep(st.fu_step, g, st.exact_fu), s.solve_Fu(g), rtol=1e-11, atol=1e-11)
    assert np.allclose(paratime.sweep(st.ca_step, a, st.exact_ca), s.solve_CA(a), rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("which", ["fu", "ca"])
def test_parareal_terminates_slab_by_slab(which):
    s = small_system(4, 6)
    st = paratime.SweepSteps(s)
    rng = np.random.default_rng(5)
    if which == "fu":
        rhs = rng.standard_normal((s.nt, s.nu))
        step, fine = st.fu_step, st.exact_fu
        coarse = st.cheb_fu(1, [jacobi_interval(s.slabs[k].Fu) for k in range(s.nt)])
    else:
        rhs = rng.standard_normal((s.nt, s.na))
        step, fine = st.ca_step, st.exact_ca
        coarse = st.cheb_ca(1, [jacobi_interval(st.C0[k]) for k in range(s.nt)])
    ref = paratime.sweep(step, rhs, fine)
    its = paratime.parareal(step, rhs, fine, coarse, s.nt)
    scale = np.abs(ref).max()
    # the coarse sweep alone is far from the fine one
    assert np.abs(its[0] - ref).max() > 1e-3 * scale
    for j, x in enumerate(its):
        err = np.abs(x - ref).max(axis=1)
        assert np.all(err[:j] <= 1e-11 * scale), (j, err)
    # one iteration is not yet the fine sweep: the later slabs still carry the coarse error
    assert np.abs(its[1] - ref)[1:].max() > 1e-8 * scale
    assert np.abs(its[-1] - ref).max() <= 1e-11 * scale


def test_parareal_PT_with_nt_iterations_is_PT():
    s = small_system(4, 5)
    st = paratime.SweepSteps(s)
    fu_c = st.cheb_fu(2, [jacobi_interval(s.slabs[k].Fu) for k in range(s.nt)])
    ca_c = st.cheb_ca(1, [jacobi_interval(st.C0[k]) for k in range(s.nt)])
    r = np.random.default_rng(6).standard_normal(s.N)
    z_ref = s.apply_PT_inv(r)
    z = paratime.apply_PT_inv_parareal(s, r, s.nt, fu_c, ca_c)
    assert np.linalg.norm(z - z_ref) <= 1e-10 * np.linalg.norm(z_ref)
    # one iteration: the first slab is already P_T's, the operator as a whole is not
    z1 = paratime.apply_PT_inv_parareal(s, r, 1, fu_c, ca_c)
    first = slice(0, s.ns)
    assert np.linalg.norm(z1[first] - z_ref[first]) <= 1e-10 * np.linalg.norm(z_ref[first])
    assert np.linalg.norm(z1 - z_ref) > 1e-6 * np.linalg.norm(z_ref)
