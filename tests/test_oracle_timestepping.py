"""Pins of the oracle's sequential time stepping with P_{T,k} (eq. (PTTS)).

* The time-stepping solution is the all-at-once solution: J is block
  lower-bidiagonal in time, so forward substitution slab by slab with
  converged step solves gives x* (checked against the direct solve and the
  bordered dense LU of the whole system at tiny sizes), and the space-time
  residual meets the tolerance the per-step absolute tolerance is scaled for.
* The one-slab system of slab k is that slab's diagonal block of J
  (eq. (jacobianSTDiscrete) with Nt = 1 gives eq. (jacobianDiscrete)).
* P_T^{-1} is block lower-triangular in time (its sweeps run forward), so
  its first slab of output depends only on the first slab of input and equals
  the single-step P_{T,1}^{-1} of that slab; for later slabs the single-step
  operator differs from P_T's diagonal only through the time couplings, which
  vanish for k = 1.
"""
import numpy as np
import pytest

import oracle
from oracle.timestepping import slab_system, solve_time_stepping, solve_windows
from paper_2309_00768_amd import inputs


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("n,nt,warm", [(3, 4, True), (4, 3, False), (8, 8, True)])
def test_time_stepping_reaches_the_all_at_once_solution(n, nt, warm):
    cfg = inputs.Config("ts", n, nt, 0.1, 100.0, 100.0)
    ub, ab = inputs.state(cfg)
    full = oracle.system_from_config(cfg, ub, ab)
    b = inputs.rhs(cfg, 3)
    xs = full.direct_solve(b)
    x, its, st = solve_time_stepping(n, nt, cfg.dt, cfg.mu, cfg.eta, cfg.mu0, ub, ab, b, rtol=1e-12,
                                     warm_start=warm)
    assert len(its) == nt and all(i >= 1 for i in its)
    bp = full.project_pressure(b)
    assert np.linalg.norm(bp - full.apply_J(x)) <= 1.0001e-12 * np.linalg.norm(bp)
    assert rel(x, xs) <= 1e-9
    # each step's residual is within the scaled absolute tolerance
    assert max(st["step_residuals"]) <= 1.0001 * st["atol"]


def test_time_stepping_matches_dense_lu_at_tiny_size():
    n, nt = 2, 3
    cfg = inputs.Config("ts", n, nt, 0.1, 10.0, 10.0)
    ub, ab = inputs.state(cfg)
    full = oracle.system_from_config(cfg, ub, ab)
    b = full.project_pressure(inputs.rhs(cfg, 4))
    # bordered dense LU: J plus one zero-mean pressure constraint per slab
    J = full.assemble_J().toarray()
    m = np.asarray(full.cb.Mp.sum(axis=0)).ravel()
    E = np.zeros((full.N, nt))
    for k in range(nt):
        E[k * full.ns + full.offs[1]: k * full.ns + full.offs[2], k] = m
    A = np.block([[J, E], [E.T, np.zeros((nt, nt))]])
    xd = np.linalg.solve(A, np.concatenate([b, np.zeros(nt)]))[:full.N]
    x, _, _ = solve_time_stepping(n, nt, cfg.dt, cfg.mu, cfg.eta, cfg.mu0, ub, ab, b, rtol=1e-13)
    assert rel(x, xd) <= 1e-10


def test_slab_system_is_the_diagonal_block_of_J():
    n, nt = 3, 3
    cfg = inputs.Config("ts", n, nt, 0.1, 100.0, 100.0)
    ub, ab = inputs.state(cfg)
    full = oracle.system_from_config(cfg, ub, ab)
    rng = np.random.default_rng(5)
    for k in range(nt):
        sk = slab_system(n, cfg.dt, cfg.mu, cfg.eta, cfg.mu0, ub[k], ab[k])
        xk = rng.standard_normal(full.ns)
        X = np.zeros((nt, full.ns))
        X[k] = xk
        yk = full.apply_J(X.ravel()).reshape(nt, full.ns)[k]
        assert rel(sk.apply_J(xk), yk) <= 1e-13


def test_first_slab_of_PT_is_the_single_step_preconditioner():
    n, nt = 3, 4
    cfg = inputs.Config("ts", n, nt, 0.1, 100.0, 100.0)
    ub, ab = inputs.state(cfg)
    full = oracle.system_from_config(cfg, ub, ab)
    rng = np.random.default_rng(6)
    R = rng.standard_normal((nt, full.ns))
    z = full.apply_PT_inv(R.ravel()).reshape(nt, full.ns)
    s0 = slab_system(n, cfg.dt, cfg.mu, cfg.eta, cfg.mu0, ub[0], ab[0])
    assert rel(s0.apply_PT_inv(R[0]), z[0]) <= 1e-12
    # and later slabs' input does not reach slab 1 (block lower-triangular in time)
    R2 = R.copy()
    R2[1:] = rng.standard_normal((nt - 1, full.ns))
    z2 = full.apply_PT_inv(R2.ravel()).reshape(nt, full.ns)
    assert rel(z2[0], z[0]) <= 1e-13


@pytest.mark.parametrize("window", [2, 3])
def test_windows_reach_the_all_at_once_solution(window):
    """Windows of W slabs in turn (7 slabs: the last window shorter) reach x*, and
    the whole residual meets the space-time tolerance."""
    cfg = inputs.Config("win", 4, 7, 0.1, 100.0, 100.0)
    ub, ab = inputs.state(cfg)
    sysm = oracle.system_from_config(cfg, ub, ab)
    b = inputs.rhs(cfg, 3)
    x, its, _ = solve_windows(cfg.n, cfg.nt, cfg.dt, cfg.mu, cfg.eta, cfg.mu0, ub, ab, b, window, rtol=1e-12)
    assert len(its) == -(-cfg.nt // window)
    xs = sysm.direct_solve(b)
    assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)


def test_one_slab_windows_are_time_stepping_and_one_window_is_all_at_once():
    cfg = inputs.Config("win1", 4, 5, 0.1, 100.0, 100.0)
    ub, ab = inputs.state(cfg)
    b = inputs.rhs(cfg, 4)
    _, its1, _ = solve_windows(cfg.n, cfg.nt, cfg.dt, cfg.mu, cfg.eta, cfg.mu0, ub, ab, b, 1, rtol=1e-10)
    _, its_ts, _ = solve_time_stepping(cfg.n, cfg.nt, cfg.dt, cfg.mu, cfg.eta, cfg.mu0, ub, ab, b, rtol=1e-10)
    assert its1 == its_ts
    _, its_all, _ = solve_windows(cfg.n, cfg.nt, cfg.dt, cfg.mu, cfg.eta, cfg.mu0, ub, ab, b, cfg.nt, rtol=1e-10)
    sysm = oracle.system_from_config(cfg, ub, ab)
    _, its_st, _ = oracle.solve_fgmres(sysm, b, rtol=1e-10)
    assert its_all == [its_st]
