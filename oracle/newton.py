"""Space-time Newton iteration on the nonlinear recurrence (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).  Plain float64 NumPy/SciPy.

The paper solves the whole backward-Euler recurrence, eq. (recurrence), at once
by Newton's method: each step linearises it about the current space-time
iterate, which gives the space-time Jacobian of eq. (jacobianSTDiscrete), and
solves that linear system with GMRES right-preconditioned by P_T (Sec.
"Performance of preconditioner": Newton to an absolute 1e-10, GMRES to a
relative 1e-2 or an absolute 1e-14).

Unknowns: the space-time vector x of the linear solver (interior u and A, all p
and j per slab) is added to base fields that carry the boundary values (u and
A Dirichlet on every side) and the initial guess; the fields at t_0 enter the
first slab.  The residual is the left-hand side of eq. (recurrence) evaluated
by quadrature (``nonlinear.slab_residual``) minus its right-hand side: the
forcing f in the momentum rows and the imposed electric field, which enters the
induction rows as +E (the recurrence carries -E on its right).  f and E are
nodal fields integrated against the test functions with the same quadrature.
"""
from __future__ import annotations

import numpy as np

from .blocks import current_from_potential
from .fem import Mesh, assemble_vec, at_quad
from .nonlinear import slab_residual
from .spacetime import SpaceTimeSystem, gmres


def load_vector(mesh: Mesh, f=None, E=None):
    """Right-hand side rows of one slab moved to the left: -(f, phi) on the
    velocity rows and +(E, chi) on the induction rows, slab order
    [u_x | u_y | p | j | A] (u and A rows on interior nodes)."""
    q2, q1, h = mesh.q2, mesh.q1, mesh.h
    W = q2.w * h * h
    nf2, nf1 = mesh.free2.size, mesh.free1.size
    ru = np.zeros(2 * nf2)
    ra = np.zeros(nf1)
    if f is not None:
        for c in range(2):
            fq, _, _ = at_quad(q2, mesh.c2, f[c], h)
            loc = np.einsum("q,mq,eq->em", W, q2.N, fq)
            ru[c * nf2:(c + 1) * nf2] = -assemble_vec(mesh.c2, loc, mesh.nq2)[mesh.free2]
    if E is not None:
        Eq, _, _ = at_quad(q1, mesh.c1, E, h)
        loc = np.einsum("q,mq,eq->em", W, q1.N, Eq)
        ra = assemble_vec(mesh.c1, loc, mesh.nq1)[mesh.free1]
    return np.concatenate([ru, np.zeros(2 * mesh.nq1), ra])


class NewtonProblem:
    """Base fields, initial fields and forcing of a space-time Newton solve.

    base = (u (nt, 2, nq2), p (nt, nq1), j (nt, nq1), A (nt, nq1)) full nodal
    fields; u_init (2, nq2), A_init (nq1) at t_0; f (nt, 2, nq2) or None,
    E (nt, nq1) or None."""

    def __init__(self, n, nt, dt, mu, eta, mu0, base, u_init, A_init, f=None, E=None):
        self.n, self.nt, self.dt, self.mu, self.eta, self.mu0 = n, nt, dt, mu, eta, mu0
        self.mesh = Mesh(n)
        self.base = base
        self.u_init, self.A_init = u_init, A_init
        self.f, self.E = f, E
        self.loads = [load_vector(self.mesh, None if f is None else f[k], None if E is None else E[k])
                      for k in range(nt)]
        nf2, nf1 = self.mesh.free2.size, self.mesh.free1.size
        self.offs = np.cumsum([0, 2 * nf2, self.mesh.nq1, self.mesh.nq1, nf1])
        self.ns = int(self.offs[-1])
        self.N = self.ns * nt

    def fields(self, x):
        """Full nodal fields (u, p, j, A) of base + x, each with a leading slab axis."""
        mesh = self.mesh
        bu, bp, bj, bA = self.base
        X = x.reshape(self.nt, self.ns)
        o = self.offs
        nf2 = mesh.free2.size
        u = bu.copy()
        u[:, 0, mesh.free2] += X[:, o[0]:o[0] + nf2]
        u[:, 1, mesh.free2] += X[:, o[0] + nf2:o[1]]
        p = bp + X[:, o[1]:o[2]]
        j = bj + X[:, o[2]:o[3]]
        A = bA.copy()
        A[:, mesh.free1] += X[:, o[3]:o[4]]
        return u, p, j, A

    def residual(self, x):
        """R(base + x): eq. (recurrence), left-hand side minus right-hand side."""
        u, p, j, A = self.fields(x)
        out = []
        prev = (self.u_init, self.A_init)
        for k in range(self.nt):
            r = slab_residual(self.mesh, (u[k], p[k], j[k], A[k]), prev, self.dt, self.mu, self.eta, self.mu0)
            out.append(r + self.loads[k])
            prev = (u[k], A[k])
        return np.concatenate(out)

    def linearisation(self, x):
        """The space-time system linearised about base + x (its J is the Jacobian of R there)."""
        u, p, j, A = self.fields(x)
        return SpaceTimeSystem(self.n, self.nt, self.dt, self.mu, self.eta, self.mu0, u, A, j)


def initial_current(mesh_n, A, mu0):
    """j with M_j j = -(1/mu0) K_jA A for every slab (the paper's initial j)."""
    from .blocks import ConstantBlocks
    cb = ConstantBlocks(Mesh(mesh_n), mu0)
    return np.stack([current_from_potential(cb, A[k], mu0) for k in range(A.shape[0])])


def newton_solve(prob: NewtonProblem, tol=1e-10, max_newton=20, linear="gmres", lin_rtol=1e-2, lin_atol=1e-14,
                 restart=30, maxit=2000):
    """Newton on R(base + x) = 0 from x = 0.  linear = "gmres" (right-preconditioned
    by P_T of each linearisation, to lin_rtol relative or lin_atol absolute) or
    "direct" (forward substitution in time with sparse LU).  Returns
    (x, residual norms before each step, linear iterations per step)."""
    x = np.zeros(prob.N)
    hist, lin_its = [], []
    for _ in range(max_newton + 1):
        r = prob.residual(x)
        rn = float(np.linalg.norm(r))
        hist.append(rn)
        if rn <= tol or len(lin_its) >= max_newton:
            break
        sysm = prob.linearisation(x)
        b = sysm.project_pressure(-r)
        if linear == "direct":
            d = sysm.direct_solve(b)
            lin_its.append(0)
        else:
            bn = np.linalg.norm(b)
            rt = max(lin_rtol, lin_atol / bn) if bn > 0 else lin_rtol
            d, its, _ = gmres(sysm.apply_J, sysm.apply_PT_inv, b, restart=restart, rtol=rt, maxit=maxit)
            d = sysm.normalise_pressure(d)
            lin_its.append(its)
        x = x + d
    return x, hist, lin_its
