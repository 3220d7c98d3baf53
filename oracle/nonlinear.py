"""Residual of the backward-Euler finite-element recurrence (oracle).

The paper's eq. (recurrence): for k = 1..Nt,

  Mu (u^k - u^{k-1})/dt + mu Ku u^k + B^T p^k + N_u(u^k, j^k, A^k) = f^k
  B u^k = 0
  Mj j^k + (1/mu0) KjA A^k = h^k
  MA (A^k - A^{k-1})/dt + (eta/mu0) KA A^k + N_A(u^k, A^k) = -E^k

with N_u the weak form of (u.grad)u + j grad A and N_A that of u.grad A.  This
module evaluates the left-hand side directly by quadrature of the fields (no
matrices), so that the assembled Jacobian blocks can be checked against its
derivative: the residual is quadratic in the unknowns, hence central
differences reproduce J x exactly up to rounding.
"""
from __future__ import annotations

import numpy as np

from .fem import Mesh, assemble_vec, at_quad


def slab_residual(mesh: Mesh, fields, prev, dt, mu, eta, mu0):
    """Residual rows of one slab for full nodal fields.

    ``fields`` = (u (2, nq2), p (nq1), j (nq1), A (nq1)) at time k and ``prev`` =
    (u, A) at time k-1.  Returns the residual on the unknown rows, in the slab
    order [u_x | u_y | p | j | A] (u and A rows on interior nodes only).
    """
    u, p, j, A = fields
    u0, A0 = prev
    q2, q1, h = mesh.q2, mesh.q1, mesh.h
    W = q2.w * h * h
    N2, N2x, N2y = q2.N, q2.Ns / h, q2.Nt / h
    N1, N1x, N1y = q1.N, q1.Ns / h, q1.Nt / h
    ux, uxx, uxy = at_quad(q2, mesh.c2, u[0], h)
    uy, uyx, uyy = at_quad(q2, mesh.c2, u[1], h)
    vx, _, _ = at_quad(q2, mesh.c2, u0[0], h)
    vy, _, _ = at_quad(q2, mesh.c2, u0[1], h)
    pq, _, _ = at_quad(q1, mesh.c1, p, h)
    jq, _, _ = at_quad(q1, mesh.c1, j, h)
    Aq, Ax, Ay = at_quad(q1, mesh.c1, A, h)
    Bq, _, _ = at_quad(q1, mesh.c1, A0, h)
    # momentum, component x and y:  (u - u0)/dt phi + mu grad u : grad phi - p div phi
    #                                + ((u.grad) u) . phi + j grad A . phi
    conv_x = ux * uxx + uy * uxy
    conv_y = ux * uyx + uy * uyy
    rux = np.einsum("q,mq,eq->em", W, N2, (ux - vx) / dt + conv_x + jq * Ax) \
        + mu * (np.einsum("q,mq,eq->em", W, N2x, uxx) + np.einsum("q,mq,eq->em", W, N2y, uxy)) \
        - np.einsum("q,mq,eq->em", W, N2x, pq)
    ruy = np.einsum("q,mq,eq->em", W, N2, (uy - vy) / dt + conv_y + jq * Ay) \
        + mu * (np.einsum("q,mq,eq->em", W, N2x, uyx) + np.einsum("q,mq,eq->em", W, N2y, uyy)) \
        - np.einsum("q,mq,eq->em", W, N2y, pq)
    # incompressibility: -int psi div u
    rp = -np.einsum("q,mq,eq->em", W, N1, uxx + uyy)
    # current: int j chi + (1/mu0) int grad A . grad chi
    rj = np.einsum("q,mq,eq->em", W, N1, jq) \
        + (np.einsum("q,mq,eq->em", W, N1x, Ax) + np.einsum("q,mq,eq->em", W, N1y, Ay)) / mu0
    # induction: (A - A0)/dt chi + (eta/mu0) grad A . grad chi + (u . grad A) chi
    ra = np.einsum("q,mq,eq->em", W, N1, (Aq - Bq) / dt + ux * Ax + uy * Ay) \
        + (eta / mu0) * (np.einsum("q,mq,eq->em", W, N1x, Ax) + np.einsum("q,mq,eq->em", W, N1y, Ay))
    Rux = assemble_vec(mesh.c2, rux, mesh.nq2)[mesh.free2]
    Ruy = assemble_vec(mesh.c2, ruy, mesh.nq2)[mesh.free2]
    Rp = assemble_vec(mesh.c1, rp, mesh.nq1)
    Rj = assemble_vec(mesh.c1, rj, mesh.nq1)
    Ra = assemble_vec(mesh.c1, ra, mesh.nq1)[mesh.free1]
    return np.concatenate([Rux, Ruy, Rp, Rj, Ra])


def spacetime_residual(sysm, base, x, u_init, A_init):
    """Residual of the whole recurrence at the fields ``base + x``.

    ``base`` = (u (nt, 2, nq2), p (nt, nq1), j (nt, nq1), A (nt, nq1)) are full
    nodal fields; ``x`` is a space-time vector of unknowns (interior u and A,
    all p and j) added on top of them.  ``u_init``/``A_init`` are the fields at
    t_0, which the first slab couples to.
    """
    mesh = sysm.mesh
    bu, bp, bj, bA = base
    xu, xp, xj, xa = sysm.split(x)
    nf2 = mesh.free2.size
    out = []
    prev_u, prev_A = u_init, A_init
    for k in range(sysm.nt):
        u = bu[k].copy()
        u[0, mesh.free2] += xu[k, :nf2]
        u[1, mesh.free2] += xu[k, nf2:]
        A = bA[k].copy()
        A[mesh.free1] += xa[k]
        p = bp[k] + xp[k]
        j = bj[k] + xj[k]
        out.append(slab_residual(mesh, (u, p, j, A), (prev_u, prev_A), sysm.dt, sysm.mu, sysm.eta, sysm.mu0))
        prev_u, prev_A = u, A
    return np.concatenate(out)
