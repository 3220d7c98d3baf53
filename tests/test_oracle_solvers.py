"""Pins of the oracle's solvers: dense LU, the preconditioner algebra, the exact-Schur
iteration count, GMRES, the transposed operators and the adjoint gradient."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_2309_00768_amd import inputs


def small_system(n, nt, seed=0, dt=0.1, re=20.0, s=30.0, const_A=None, jbar=None):
    cfg = inputs.Config("t", n, nt, dt, re, s, state_seed=seed)
    ub, Ab = inputs.state(cfg)
    if const_A is not None:
        Ab = np.full_like(Ab, const_A)
    return oracle.SpaceTimeSystem(n, nt, dt, cfg.mu, cfg.eta, 1.0, ub * 3.0, Ab * 3.0, jbar), cfg


def bordered_dense_J(sysm):
    """J bordered with one pressure normalisation row/column per slab (dense)."""
    J = sysm.assemble_J().toarray()
    m = np.asarray(sysm.cb.Mp.sum(axis=0)).ravel()
    E = np.zeros((sysm.N, sysm.nt))
    for k in range(sysm.nt):
        E[k * sysm.ns + sysm.offs[1]: k * sysm.ns + sysm.offs[2], k] = m
    return np.block([[J, E], [E.T, np.zeros((sysm.nt, sysm.nt))]])


@pytest.mark.parametrize("n,nt", [(2, 2), (2, 4), (4, 2), (4, 4)])
def test_direct_time_stepping_equals_dense_lu(n, nt):
    sysm, _ = small_system(n, nt)
    b = sysm.project_pressure(np.random.default_rng(1).standard_normal(sysm.N))
    K = bordered_dense_J(sysm)
    xd = np.linalg.solve(K, np.concatenate([b, np.zeros(nt)]))[:sysm.N]
    x = sysm.direct_solve(b)
    assert np.linalg.norm(x - xd) <= 1e-12 * np.linalg.norm(xd)
    # transposed direct solve against the dense transpose
    lt = np.linalg.solve(K.T, np.concatenate([b, np.zeros(nt)]))[:sysm.N]
    assert np.linalg.norm(sysm.direct_solve_T(b) - lt) <= 1e-12 * np.linalg.norm(lt)


def test_gmres_with_PT_reaches_direct_solution_cfg1():
    cfg = inputs.CONFIGS["cfg1"]
    sysm = oracle.system_from_config(cfg)
    b = inputs.rhs(cfg, 1)
    xs = sysm.direct_solve(b)
    x, its, _ = oracle.solve_fgmres(sysm, b, rtol=1e-12)
    assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)
    assert 5 < its < 300


def test_wave_operator_is_the_product_FA_Dinv_FA_plus_KA():
    """C_A assembled from its bands (eq. (CAs), band -1 with factor -1/dt) equals
    F_A D^{-1} F_A + K_A built from the lower-bidiagonal space-time F_A."""
    sysm, _ = small_system(3, 4)
    m = sysm.st_matrices()
    D = m["D"]
    prod = m["FA"] @ sp.diags(1.0 / D.diagonal()) @ m["FA"] + m["KAw"]
    assert abs(prod - m["CA"]).max() <= 1e-12 * abs(prod).max()


def dense_PT(sysm):
    """P_T of eq. (PT) as a dense matrix in slab-major order, with
    S_p = -K_p F_p^{-1} M_p and S_A = M_A F_A^{-1} C_A."""
    m = {k: v.toarray() for k, v in sysm.st_matrices().items()}
    Sp = -m["Kp"] @ np.linalg.solve(m["Fp"], m["Mp"])
    SA = m["MA"] @ np.linalg.solve(m["FA"], m["CA"])
    nu, np_, nj, na = m["Fu"].shape[0], m["Kp"].shape[0], m["Mj"].shape[0], m["MA"].shape[0]
    Z = lambda a, b: np.zeros((a, b))
    P = np.block([
        [m["Fu"], m["B"].T, m["Zj"], m["ZA"]],
        [Z(np_, nu), Sp, Z(np_, nj), Z(np_, na)],
        [Z(nj, nu), Z(nj, np_), m["Mj"], m["KjA"]],
        [Z(na, nu), Z(na, np_), Z(na, nj), SA]])
    perm = sysm.slab_major_permutation()
    return P[np.ix_(perm, perm)]


@pytest.mark.parametrize("n,nt", [(2, 3), (4, 3)])
def test_PT_inverse_inverts_dense_PT(n, nt):
    sysm, _ = small_system(n, nt)
    P = dense_PT(sysm)
    r = sysm.project_pressure(np.random.default_rng(7).standard_normal(sysm.N))
    z = sysm.apply_PT_inv(r)
    assert np.linalg.norm(P @ z - r) <= 1e-10 * np.linalg.norm(r)


def test_exact_schur_decoupled_case_converges_in_two_iterations():
    """Constant potential => j = 0 and Y = Z_j = Z_A = 0.  With the exact Schur
    complements S_p = -B F_u^{-1} B^T and S_A = F_A, J P_T^{-1} = I + N with N^2 = 0,
    so right-preconditioned GMRES converges in at most two iterations."""
    sysm, _ = small_system(4, 3, const_A=0.7, jbar=np.zeros((3, 25)))
    assert abs(sysm.slabs[0].ZA).max() < 1e-14 and abs(sysm.slabs[0].Y).max() < 1e-14
    sp_fn, sa_fn = sysm.exact_schur_inverses()
    M = lambda r: sysm.apply_PT_inv(r, schur_p=sp_fn, schur_a=sa_fn)
    b = sysm.project_pressure(np.random.default_rng(2).standard_normal(sysm.N))
    x, its, hist = oracle.gmres(sysm.apply_J, M, b, restart=30, rtol=1e-10)
    assert its <= 2, hist
    # with the paper's approximations the count is larger but finite
    x2, its2, _ = oracle.gmres(sysm.apply_J, sysm.apply_PT_inv, b, restart=30, rtol=1e-10)
    assert its2 > 2


def test_exact_schur_with_wave_sa_in_decoupled_case():
    """In the decoupled case, S_A = F_A; the wave approximation with the consistent mass
    instead of D and K_A = 0 reproduces it, so only the PCD approximation is inexact."""
    sysm, _ = small_system(3, 3, const_A=0.0)
    m = {k: v.toarray() for k, v in sysm.st_matrices().items()}
    CA_exact = m["FA"] @ np.linalg.solve(m["MA"], m["FA"])
    SA = m["MA"] @ np.linalg.solve(m["FA"], CA_exact)
    np.testing.assert_allclose(SA, m["FA"], atol=1e-10 * np.abs(m["FA"]).max())


def test_transposes_dot_tests():
    sysm, _ = small_system(3, 4)
    rng = np.random.default_rng(9)
    x = sysm.project_pressure(rng.standard_normal(sysm.N))
    y = sysm.project_pressure(rng.standard_normal(sysm.N))
    Jx, JTy = sysm.apply_J(x), sysm.apply_JT(y)
    assert abs(Jx @ y - x @ JTy) <= 1e-13 * np.linalg.norm(Jx) * np.linalg.norm(y)
    Px, PTy = sysm.apply_PT_inv(x), sysm.apply_PT_invT(y)
    assert abs(Px @ y - x @ PTy) <= 1e-11 * np.linalg.norm(Px) * np.linalg.norm(y)


def test_adjoint_gradient_matches_central_differences():
    """J(A0) = 1/2 |x_A^{Nt} - A_target|^2 with b_A^1 = (M_A/dt) A0 is exactly quadratic, so
    central differences equal the adjoint gradient (M_A/dt) lambda_A^1 up to rounding."""
    sysm, cfg = small_system(4, 5)
    rng = np.random.default_rng(4)
    f = sysm.project_pressure(rng.standard_normal(sysm.N))
    A0 = rng.standard_normal(sysm.na)
    At = rng.standard_normal(sysm.na)
    o = sysm.offs

    def forward(a0):
        b = f.copy().reshape(sysm.nt, sysm.ns)
        b[0, o[3]:o[4]] += sysm.cb.MA @ a0 / sysm.dt
        x = sysm.direct_solve(b.ravel()).reshape(sysm.nt, sysm.ns)
        return x

    def objective(a0):
        xa = forward(a0)[-1, o[3]:o[4]]
        return 0.5 * np.sum((xa - At) ** 2)

    x = forward(A0)
    g = np.zeros((sysm.nt, sysm.ns))
    g[-1, o[3]:o[4]] = x[-1, o[3]:o[4]] - At
    lam = sysm.direct_solve_T(g.ravel()).reshape(sysm.nt, sysm.ns)
    grad = sysm.cb.MA @ lam[0, o[3]:o[4]] / sysm.dt
    for d in range(4):
        v = rng.standard_normal(sysm.na)
        eps = 1e-2
        fd = (objective(A0 + eps * v) - objective(A0 - eps * v)) / (2 * eps)
        assert abs(fd - grad @ v) <= 1e-8 * max(1.0, abs(fd))
    # the forcing gradient: d/df of J is lambda_u (rows of the momentum equation)
    v = rng.standard_normal(o[1])
    eps = 1e-2

    def obj_f(df):
        b = f.copy().reshape(sysm.nt, sysm.ns)
        b[:, :o[1]] += df.reshape(1, -1)
        b[0, o[3]:o[4]] += sysm.cb.MA @ A0 / sysm.dt
        xa = sysm.direct_solve(b.ravel()).reshape(sysm.nt, sysm.ns)[-1, o[3]:o[4]]
        return 0.5 * np.sum((xa - At) ** 2)
    fd = (obj_f(eps * v) - obj_f(-eps * v)) / (2 * eps)
    assert abs(fd - lam[:, :o[1]].sum(axis=0) @ v) <= 1e-8 * max(1.0, abs(fd))
