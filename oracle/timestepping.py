"""Sequential time stepping with the single-step preconditioner P_{T,k}.

TEST INFRASTRUCTURE ONLY (see the package header).  Plain float64 SciPy.

The classical alternative to the all-at-once solve (Sec. "Comparison with
sequential time-stepping"): the slabs are solved one after the other, slab k
from its own single-step Jacobian of eq. (jacobianDiscrete),

    J_k x^k = b^k + diag(M_u/dt, 0, 0, M_A/dt) x^{k-1},

each by GMRES right-preconditioned with the single-step counterpart of P_T,
eq. (PTTS): the same factors as eq. (PT) on one slab, with the single-step
magnetic Schur approximation of eq. (ASchurApproxTS), S_A,k = M_A F_A,k^{-1}
C_A,k, whose inverse is C_A,k^{-1} F_A,k M_A^{-1}, i.e. P_T of a one-slab
system.  The linear solver of each step stops on an absolute tolerance scaled
by 1/sqrt(Nt) (the paper's balancing of the comparison), here
rtol ||b|| / sqrt(Nt): the per-step residuals are exactly the rows of the
space-time residual, so the whole solution then meets ||b - J x|| <= rtol ||b||.
Each step may start from the previous step's solution (the paper reuses it as
the next step's initial guess).

Between the two extremes, windows of W slabs can be solved one after the other,
each all at once with the P_T of eq. (PT) on its own slabs and coupled to the
previous window's last slab in the same way; window k then stops on
rtol ||b|| sqrt(W_k / Nt), which again bounds the whole space-time residual.
W = 1 is time stepping, W = Nt the all-at-once solve.
"""
from __future__ import annotations

import numpy as np

from .spacetime import SpaceTimeSystem, gmres


def slab_system(n, dt, mu, eta, mu0, ubar_k, Abar_k, jbar_k=None):
    """The one-slab system of slab k: its J is the single-step Jacobian and its
    P_T the single-step preconditioner P_{T,k} of eq. (PTTS)."""
    jb = None if jbar_k is None else jbar_k[None]
    return SpaceTimeSystem(n, 1, dt, mu, eta, mu0, ubar_k[None], Abar_k[None], jb)


def solve_time_stepping(n, nt, dt, mu, eta, mu0, ubar, Abar, b, rtol=1e-8, restart=30, maxit=2000,
                        warm_start=True, jbar=None):
    """x = J^{-1} b by sequential time stepping with P_{T,k}.

    Returns (x, iterations per step, stats) with the solution normalised like
    the all-at-once solve (pressure 1^T M_p p^k = 0 per slab).  stats holds the
    per-step true residual norms and the tolerance used."""
    first = slab_system(n, dt, mu, eta, mu0, ubar[0], Abar[0], None if jbar is None else jbar[0])
    ns = first.ns
    B = np.asarray(b, dtype=np.float64).reshape(nt, ns)
    # every slab's pressure rows projected to zero sum (the range of J)
    Bp = np.stack([first.project_pressure(B[k]) for k in range(nt)])
    atol = rtol * np.linalg.norm(Bp) / np.sqrt(nt)
    C = first.coupling()           # J_{k,k-1} = -diag(M_u/dt, 0, 0, M_A/dt), slab-invariant
    X = np.zeros((nt, ns))
    its, res = [], []
    for k in range(nt):
        sk = first if k == 0 else slab_system(n, dt, mu, eta, mu0, ubar[k], Abar[k],
                                              None if jbar is None else jbar[k])
        rhs = Bp[k] - (C @ X[k - 1] if k > 0 else 0.0)
        x0 = X[k - 1].copy() if (warm_start and k > 0) else None
        rn = np.linalg.norm(rhs)
        # the oracle's GMRES stops on a relative tolerance: express the absolute one relative to rhs
        tol = atol / rn if rn > 0 else 0.0
        xk, ik, _ = gmres(sk.apply_J, sk.apply_PT_inv, rhs, restart=restart, rtol=tol, maxit=maxit, x0=x0)
        X[k] = sk.normalise_pressure(xk)
        its.append(ik)
        res.append(float(np.linalg.norm(rhs - sk.apply_J(X[k]))))
    return X.ravel(), its, {"atol": atol, "step_residuals": res}


def solve_windows(n, nt, dt, mu, eta, mu0, ubar, Abar, b, window, rtol=1e-8, restart=30, maxit=2000,
                  warm_start=True):
    """x = J^{-1} b by windows of `window` slabs (the last one shorter), each by
    GMRES right-preconditioned with the P_T of its own slabs.

    Returns (x, iterations per window, stats) like solve_time_stepping; with a
    warm start every slab of a window starts from the previous window's last
    slab."""
    first = slab_system(n, dt, mu, eta, mu0, ubar[0], Abar[0])
    ns = first.ns
    B = np.asarray(b, dtype=np.float64).reshape(nt, ns)
    Bp = np.stack([first.project_pressure(B[k]) for k in range(nt)])
    bnorm = np.linalg.norm(Bp)
    C = first.coupling()
    X = np.zeros((nt, ns))
    its, res = [], []
    for k0 in range(0, nt, window):
        w = min(window, nt - k0)
        sw = SpaceTimeSystem(n, w, dt, mu, eta, mu0, ubar[k0:k0 + w], Abar[k0:k0 + w])
        rhs = Bp[k0:k0 + w].copy()
        if k0 > 0:
            rhs[0] -= C @ X[k0 - 1]
        rhs = rhs.ravel()
        x0 = np.tile(X[k0 - 1], w) if (warm_start and k0 > 0) else None
        atol = rtol * bnorm * np.sqrt(w / nt)
        rn = np.linalg.norm(rhs)
        tol = atol / rn if rn > 0 else 0.0
        xw, iw, _ = gmres(sw.apply_J, sw.apply_PT_inv, rhs, restart=restart, rtol=tol, maxit=maxit, x0=x0)
        X[k0:k0 + w] = sw.normalise_pressure(xw).reshape(w, ns)
        its.append(iw)
        res.append(float(np.linalg.norm(rhs - sw.apply_J(X[k0:k0 + w].ravel()))))
    return X.ravel(), its, {"step_residuals": res}
