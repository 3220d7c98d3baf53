"""The full space-time block preconditioner P and its simplification P-tilde.

TEST INFRASTRUCTURE ONLY (see the package header).  Plain float64 SciPy, on a
``SpaceTimeSystem`` with its exact inner solves (sequential time stepping and
sparse LU, Sec. "Performance of preconditioner").

From the approximate factorisation of the Jacobian, eq. (jacobianApprox), and
the two block LU decompositions, eqs. (PupLU) and (jacobianApprox+LeftLU):

    P^{-1}       = Utilde_up^{-1} L_up^{-1} Ubar_ujA^{-1} L_ujA^{-1}  eq. (preconditioner)
    Ptilde^{-1}  = Utilde_up^{-1} L_up^{-1} Ubar_ujA^{-1}             eq. (preconditionerSimplified1)
    P_T^{-1}     = Utilde_up^{-1}           Ubar_ujA^{-1}             eq. (PT)

(Ubar_ujA = Utilde_ujA F_uI^{-1}, eq. (barUuja), so F_uI Utilde_ujA^{-1} =
Ubar_ujA^{-1}).  Each factor's inverse is written out from its block form:

* L_ujA^{-1} (Sec. "Full approximation", step 1): x_A += Y F_u^{-1}(Z_j M_j^{-1} x_j - x_u);
* Ubar_ujA^{-1}: y_A = Stilde_A^{-1} x_A with Stilde_A^{-1} = C_A^{-1} F_A M_A^{-1}
  (eq. (ASchurApprox)), y_j = M_j^{-1}(x_j - K_jA y_A), y_u = x_u - Z_j y_j - Z_A y_A;
* L_up^{-1} (eq. (PupLU)): y_p -= B F_u^{-1} y_u;
* Utilde_up^{-1} (eq. (Utilde)): x_p = Stilde_p^{-1} y_p with
  Stilde_p^{-1} = -M_p^{-1} F_p K_p^{-1}, x_u = F_u^{-1}(y_u - B^T x_p).

P applies F_u^{-1} three times and C_A^{-1} once, Ptilde twice and once, P_T once
and once (Sec. "Block-triangular approximation").
"""
from __future__ import annotations

import numpy as np

VARIANTS = ("PT", "Ptilde", "P")


def _mass_solve(sysm, key, M, r):
    lu = sysm._factor(key, lambda: M)
    return np.array([lu.solve(r[k]) for k in range(sysm.nt)])


def lujA_inv(sysm, xu, xj, xA):
    """L_ujA^{-1}: only the A rows change."""
    cb = sysm.cb
    tj = _mass_solve(sysm, "Mj", cb.Mj, xj)
    s = sysm.solve_Fu(np.array([sysm.slabs[k].Zj @ tj[k] - xu[k] for k in range(sysm.nt)]))
    return xA + np.array([sysm.slabs[k].Y @ s[k] for k in range(sysm.nt)])


def ubar_ujA_inv(sysm, xu, xj, xA, schur_a=None):
    cb, dt, nt = sysm.cb, sysm.dt, sysm.nt
    if schur_a is not None:
        yA = schur_a(xA)
    else:
        w = _mass_solve(sysm, "MA", cb.MA, xA)
        s = np.array([sysm.slabs[k].FA @ w[k] - (cb.MA @ w[k - 1] / dt if k > 0 else 0.0) for k in range(nt)])
        yA = sysm.solve_CA(s)
    yj = _mass_solve(sysm, "Mj", cb.Mj, np.array([xj[k] - cb.KjA @ yA[k] for k in range(nt)]))
    yu = np.array([xu[k] - sysm.slabs[k].Zj @ yj[k] - sysm.slabs[k].ZA @ yA[k] for k in range(nt)])
    return yu, yj, yA


def lup_inv(sysm, yu, yp):
    """L_up^{-1}: y_p - B F_u^{-1} y_u."""
    w = sysm.solve_Fu(yu)
    return np.array([yp[k] - sysm.cb.B @ w[k] for k in range(sysm.nt)])


def utilde_up_inv(sysm, yu, yp, schur_p=None):
    cb, dt, nt = sysm.cb, sysm.dt, sysm.nt
    if schur_p is not None:
        xp = schur_p(yp)
    else:
        q = np.array([sysm.solve_Kp(yp[k]) for k in range(nt)])
        t = np.array([sysm.slabs[k].Fp @ q[k] - (cb.Mp @ q[k - 1] / dt if k > 0 else 0.0) for k in range(nt)])
        xp = -_mass_solve(sysm, "Mp", cb.Mp, t)
    xu = sysm.solve_Fu(np.array([yu[k] - cb.B.T @ xp[k] for k in range(nt)]))
    return xu, xp


def apply_inv(sysm, r, variant="P", schur_p=None, schur_a=None, normalise=True):
    """z = M^{-1} r for M = P, Ptilde or P_T (slab-major vectors; the pressure
    rows of r projected to zero sum per slab, z normalised like P_T's)."""
    if variant not in VARIANTS:
        raise ValueError(variant)
    r = sysm.project_pressure(r)
    xu, xp, xj, xA = sysm.split(r)
    if variant == "P":
        xA = lujA_inv(sysm, xu, xj, xA)
    yu, yj, yA = ubar_ujA_inv(sysm, xu, xj, xA, schur_a)
    yp = lup_inv(sysm, yu, xp) if variant in ("P", "Ptilde") else xp
    zu, zp = utilde_up_inv(sysm, yu, yp, schur_p)
    z = sysm.join(zu, zp, yj, yA)
    return sysm.normalise_pressure(z) if normalise else z
