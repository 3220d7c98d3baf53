"""Pins of the oracle's full preconditioner P and its simplification P-tilde
(eqs. (preconditioner), (preconditionerSimplified1)).

* The factor composition that drops both lower factors is P_T^{-1} itself.
* P-tilde^{-1} inverts P-tilde assembled densely from its block form, with
  Delta S_p = S_p-tilde - S_p and S_p = -B F_u^{-1} B^T.
* P^{-1} inverts P assembled densely as the product of its factors
  L_ujA Utilde_ujA F_uI^{-1} L_up Utilde_up (eqs. (jacobianApprox+LeftLU),
  (PupLU), (Utilde)).
* Decoupled case (constant potential: Y = Z_j = Z_A = 0) with the exact Schur
  complements: P and P-tilde are then J itself, so right-preconditioned GMRES
  converges in one iteration (P_T needs two: N^2 = 0, not N = 0).
"""
import numpy as np
import pytest

import oracle
from oracle import variants
from paper_2309_00768_amd import inputs


def small_system(n, nt, const_A=None, jbar=None):
    cfg = inputs.Config("v", n, nt, 0.1, 20.0, 30.0)
    ub, Ab = inputs.state(cfg)
    if const_A is not None:
        Ab = np.full_like(Ab, const_A)
    return oracle.SpaceTimeSystem(n, nt, cfg.dt, cfg.mu, cfg.eta, 1.0, ub * 3.0, Ab * 3.0, jbar)


def dense_blocks(sysm):
    m = {k: v.toarray() for k, v in sysm.st_matrices().items()}
    m["Sp_t"] = -m["Kp"] @ np.linalg.solve(m["Fp"], m["Mp"])
    m["SA_t"] = m["MA"] @ np.linalg.solve(m["FA"], m["CA"])
    m["Sp"] = -m["B"] @ np.linalg.solve(m["Fu"], m["B"].T)
    return m


def to_slab_major(sysm, P):
    perm = sysm.slab_major_permutation()
    return P[np.ix_(perm, perm)]


def test_dropping_both_lower_factors_gives_PT():
    sysm = small_system(3, 4)
    r = np.random.default_rng(1).standard_normal(sysm.N)
    z = variants.apply_inv(sysm, r, "PT")
    zt = sysm.apply_PT_inv(r)
    assert np.linalg.norm(z - zt) <= 1e-13 * np.linalg.norm(zt)


@pytest.mark.parametrize("n,nt", [(2, 3), (3, 2)])
def test_ptilde_inverse_inverts_its_block_form(n, nt):
    sysm = small_system(n, nt)
    m = dense_blocks(sysm)
    nu, np_, nj, na = m["Fu"].shape[0], m["Kp"].shape[0], m["Mj"].shape[0], m["MA"].shape[0]
    Z = lambda a, b: np.zeros((a, b))
    Pt = np.block([
        [m["Fu"], m["B"].T, m["Zj"], m["ZA"]],
        [m["B"], m["Sp_t"] - m["Sp"], Z(np_, nj), Z(np_, na)],
        [Z(nj, nu), Z(nj, np_), m["Mj"], m["KjA"]],
        [Z(na, nu), Z(na, np_), Z(na, nj), m["SA_t"]]])
    Pt = to_slab_major(sysm, Pt)
    r = sysm.project_pressure(np.random.default_rng(2).standard_normal(sysm.N))
    z = variants.apply_inv(sysm, r, "Ptilde")
    assert np.linalg.norm(Pt @ z - r) <= 1e-10 * np.linalg.norm(r)


@pytest.mark.parametrize("n,nt", [(2, 3), (3, 2)])
def test_p_inverse_inverts_the_product_of_its_factors(n, nt):
    sysm = small_system(n, nt)
    m = dense_blocks(sysm)
    nu, np_, nj, na = m["Fu"].shape[0], m["Kp"].shape[0], m["Mj"].shape[0], m["MA"].shape[0]
    Z = lambda a, b: np.zeros((a, b))
    I = np.eye
    YF = m["Y"] @ np.linalg.inv(m["Fu"])
    L_ujA = np.block([
        [I(nu), Z(nu, np_), Z(nu, nj), Z(nu, na)],
        [Z(np_, nu), I(np_), Z(np_, nj), Z(np_, na)],
        [Z(nj, nu), Z(nj, np_), I(nj), Z(nj, na)],
        [YF, Z(na, np_), -YF @ m["Zj"] @ np.linalg.inv(m["Mj"]), I(na)]])
    U_ujA = np.block([
        [m["Fu"], Z(nu, np_), m["Zj"], m["ZA"]],
        [Z(np_, nu), I(np_), Z(np_, nj), Z(np_, na)],
        [Z(nj, nu), Z(nj, np_), m["Mj"], m["KjA"]],
        [Z(na, nu), Z(na, np_), Z(na, nj), m["SA_t"]]])
    FuI_inv = np.block([
        [np.linalg.inv(m["Fu"]), Z(nu, np_ + nj + na)],
        [Z(np_ + nj + na, nu), I(np_ + nj + na)]])
    L_up = np.block([
        [I(nu), Z(nu, np_ + nj + na)],
        [m["B"] @ np.linalg.inv(m["Fu"]), I(np_), Z(np_, nj + na)],
        [Z(nj + na, nu + np_), I(nj + na)]])
    U_up = np.block([
        [m["Fu"], m["B"].T, Z(nu, nj + na)],
        [Z(np_, nu), m["Sp_t"], Z(np_, nj + na)],
        [Z(nj + na, nu + np_), I(nj + na)]])
    P = to_slab_major(sysm, L_ujA @ U_ujA @ FuI_inv @ L_up @ U_up)
    r = sysm.project_pressure(np.random.default_rng(3).standard_normal(sysm.N))
    z = variants.apply_inv(sysm, r, "P")
    assert np.linalg.norm(P @ z - r) <= 1e-9 * np.linalg.norm(r)


@pytest.mark.parametrize("variant,bound", [("P", 1), ("Ptilde", 1), ("PT", 2)])
def test_exact_schur_decoupled_case_iterations(variant, bound):
    sysm = small_system(4, 3, const_A=0.7, jbar=np.zeros((3, 25)))
    assert abs(sysm.slabs[0].Y).max() < 1e-14
    sp_fn, sa_fn = sysm.exact_schur_inverses()
    M = lambda r: variants.apply_inv(sysm, r, variant, schur_p=sp_fn, schur_a=sa_fn)
    b = sysm.project_pressure(np.random.default_rng(4).standard_normal(sysm.N))
    x, its, hist = oracle.gmres(sysm.apply_J, M, b, restart=30, rtol=1e-10)
    assert its <= bound, (variant, hist)
