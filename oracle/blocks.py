"""The single-slab operator blocks of the linearised MHD system (oracle).

Follows the paper's Sec. "Problem definition and discretisation": the
single-step Jacobian eq. (jacobianDiscrete) and the definitions of its blocks
given right after it, the Newton term of eq. (advVdelta), the pressure
convection-diffusion operator of eq. (Fp), and the averaged field B-bar and
the wave operator blocks of eqs. (CAspacetime)/(CAs).

Sign conventions (trial index n, test index m; phi = Q2 vector basis, psi = Q1
pressure basis, chi = Q1 basis of j and A):

* ``B``   = -int psi_m div(phi_n)                   (negative divergence)
* ``Wu``  =  int ((ubar . grad) phi_n) . phi_m      (advection)
* ``dWu`` =  int ((phi_n . grad) ubar) . phi_m      (Newton term, eq. advVdelta)
* ``Fu``  =  Mu/dt + mu Ku + Wu + dWu
* ``Zj``  =  int chi_n (grad Abar . phi_m)          (Lorentz term linearised in j)
* ``ZA``  =  int jbar (grad chi_n . phi_m)          (Lorentz term linearised in A)
* ``KjA`` = (1/mu0) int grad chi_n . grad chi_m     (j test on all nodes, A trial on free nodes)
* ``Y``   =  int (phi_n . grad Abar) chi_m          (induction advection linearised in u)
* ``FA``  =  MA/dt + (eta/mu0) KA + WA,  WA = int (ubar . grad chi_n) chi_m
* ``Fp``  =  Mp/dt + Wp + mu Kp, Kp the Neumann Laplacian on all pressure nodes.

The Lorentz force enters the momentum equation as +j grad A (the form that the
paper's equilibria balance against grad p; see the reading list in the design notes).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fem import Mesh, assemble, at_quad, restrict


def _w(mesh: Mesh, ref) -> np.ndarray:
    """Physical quadrature weights (same for every element of the uniform mesh)."""
    return ref.w * mesh.h * mesh.h


class ConstantBlocks:
    """Slab-independent matrices: masses, stiffnesses, divergence, mixed stiffness."""

    def __init__(self, mesh: Mesh, mu0: float):
        q2, q1, h = mesh.q2, mesh.q1, mesh.h
        E = mesh.ne
        w2, w1 = _w(mesh, q2), _w(mesh, q1)   # same 5x5 rule for both element types
        # Scalar Q2 mass and stiffness (identical on every element).
        M2e = np.einsum("q,aq,bq->ab", w2, q2.N, q2.N)
        K2e = np.einsum("q,aq,bq->ab", w2, q2.Ns, q2.Ns) / h**2 + np.einsum("q,aq,bq->ab", w2, q2.Nt, q2.Nt) / h**2
        M1e = np.einsum("q,aq,bq->ab", w1, q1.N, q1.N)
        K1e = np.einsum("q,aq,bq->ab", w1, q1.Ns, q1.Ns) / h**2 + np.einsum("q,aq,bq->ab", w1, q1.Nt, q1.Nt) / h**2
        tile = lambda Me: np.broadcast_to(Me, (E,) + Me.shape)
        self.M2full = assemble(mesh.c2, mesh.c2, tile(M2e), (mesh.nq2, mesh.nq2))
        self.K2full = assemble(mesh.c2, mesh.c2, tile(K2e), (mesh.nq2, mesh.nq2))
        self.M1full = assemble(mesh.c1, mesh.c1, tile(M1e), (mesh.nq1, mesh.nq1))
        self.K1full = assemble(mesh.c1, mesh.c1, tile(K1e), (mesh.nq1, mesh.nq1))
        # Divergence: rows pressure test psi_m (Q1), columns velocity component c trial (Q2).
        Bx = -np.einsum("q,aq,bq->ab", w2, q1_at(mesh), q2.Ns) / h
        By = -np.einsum("q,aq,bq->ab", w2, q1_at(mesh), q2.Nt) / h
        Bxf = assemble(mesh.c1, mesh.c2, tile(Bx), (mesh.nq1, mesh.nq2))
        Byf = assemble(mesh.c1, mesh.c2, tile(By), (mesh.nq1, mesh.nq2))
        f2, f1 = mesh.free2, mesh.free1
        self.M2 = restrict(self.M2full, f2, f2)
        self.K2 = restrict(self.K2full, f2, f2)
        self.Mu = sp.block_diag([self.M2, self.M2]).tocsr()
        self.Ku = sp.block_diag([self.K2, self.K2]).tocsr()
        self.B = sp.hstack([restrict(Bxf, None, f2), restrict(Byf, None, f2)]).tocsr()
        self.Mj = self.M1full.copy()
        self.KjA = restrict(self.K1full, None, f1) / mu0
        self.MA = restrict(self.M1full, f1, f1)
        self.KA = restrict(self.K1full, f1, f1)
        self.Mp = self.M1full.copy()
        self.Kp = self.K1full.copy()


def q1_at(mesh: Mesh) -> np.ndarray:
    """Q1 basis values at the Q2 reference quadrature points (same rule)."""
    return mesh.q1.N


def current_from_potential(cb: ConstantBlocks, Abar: np.ndarray, mu0: float) -> np.ndarray:
    """Current state from the discrete current equation with zero data:
    Mj jbar = -(1/mu0) K Abar (paper, the initialisation of j in Sec. "Model problems")."""
    return spla.spsolve(cb.M1full.tocsc(), -(cb.K1full @ Abar) / mu0)


def mean_field(mesh: Mesh, Abar: np.ndarray) -> np.ndarray:
    """Space average of B = curl(A k) = (dA/dy, -dA/dx) over the unit square."""
    _, ax, ay = at_quad(mesh.q1, mesh.c1, Abar, mesh.h)
    w = _w(mesh, mesh.q1)
    return np.array([np.sum(ay * w), -np.sum(ax * w)])


class SlabBlocks:
    """State-dependent blocks of one slab (velocity ubar (2, nq2), potential Abar, current jbar)."""

    def __init__(self, mesh: Mesh, cb: ConstantBlocks, ubar, Abar, jbar, dt, mu, eta, mu0):
        q2, q1, h = mesh.q2, mesh.q1, mesh.h
        w2 = _w(mesh, q2)
        ux, uxx, uxy = at_quad(q2, mesh.c2, ubar[0], h)
        uy, uyx, uyy = at_quad(q2, mesh.c2, ubar[1], h)
        # Q1 fields at the same quadrature points (the Q1 tabulation uses the same rule).
        _, Ax, Ay = at_quad(q1, mesh.c1, Abar, h)
        jq, _, _ = at_quad(q1, mesh.c1, jbar, h)
        N2, N2x, N2y = q2.N, q2.Ns / h, q2.Nt / h
        N1, N1x, N1y = q1.N, q1.Ns / h, q1.Nt / h
        f2, f1 = mesh.free2, mesh.free1
        n2, n1 = mesh.nq2, mesh.nq1

        # Advection W(ubar): int (ubar . grad phi_n) phi_m, scalar Q2, same for both components.
        adv = ux[:, None, :] * N2x[None] + uy[:, None, :] * N2y[None]          # (E, n, q)
        We = np.einsum("q,mq,enq->emn", w2, N2, adv)
        W2 = assemble(mesh.c2, mesh.c2, We, (n2, n2))
        # Newton term: block (d, c) = int phi_n phi_m d_c ubar_d.
        grads = {(0, 0): uxx, (0, 1): uxy, (1, 0): uyx, (1, 1): uyy}        # (d, c) -> d_c ubar_d
        dW = {}
        for (d, c), g in grads.items():
            e = np.einsum("q,mq,nq,eq->emn", w2, N2, N2, g)
            dW[(d, c)] = restrict(assemble(mesh.c2, mesh.c2, e, (n2, n2)), f2, f2)
        W2f = restrict(W2, f2, f2)
        self.Wu = sp.block_diag([W2f, W2f]).tocsr()
        self.dWu = sp.bmat([[dW[(0, 0)], dW[(0, 1)]], [dW[(1, 0)], dW[(1, 1)]]]).tocsr()
        self.Fu = (cb.Mu / dt + mu * cb.Ku + self.Wu + self.dWu).tocsr()

        # Lorentz blocks (rows velocity component c, test phi_m).
        Zjx = np.einsum("q,nq,eq,mq->emn", w2, N1, Ax, N2)
        Zjy = np.einsum("q,nq,eq,mq->emn", w2, N1, Ay, N2)
        self.Zj = sp.vstack([
            restrict(assemble(mesh.c2, mesh.c1, Zjx, (n2, n1)), f2, None),
            restrict(assemble(mesh.c2, mesh.c1, Zjy, (n2, n1)), f2, None)]).tocsr()
        ZAx = np.einsum("q,eq,nq,mq->emn", w2, jq, N1x, N2)
        ZAy = np.einsum("q,eq,nq,mq->emn", w2, jq, N1y, N2)
        self.ZA = sp.vstack([
            restrict(assemble(mesh.c2, mesh.c1, ZAx, (n2, n1)), f2, f1),
            restrict(assemble(mesh.c2, mesh.c1, ZAy, (n2, n1)), f2, f1)]).tocsr()
        # Y: rows A test chi_m (free), columns velocity component c trial phi_n.
        Yx = np.einsum("q,nq,eq,mq->emn", w2, N2, Ax, N1)
        Yy = np.einsum("q,nq,eq,mq->emn", w2, N2, Ay, N1)
        self.Y = sp.hstack([
            restrict(assemble(mesh.c1, mesh.c2, Yx, (n1, n2)), f1, f2),
            restrict(assemble(mesh.c1, mesh.c2, Yy, (n1, n2)), f1, f2)]).tocsr()
        # Scalar Q1 advection with the velocity state: int (ubar . grad chi_n) chi_m.
        adv1 = ux[:, None, :] * N1x[None] + uy[:, None, :] * N1y[None]
        W1e = np.einsum("q,mq,enq->emn", w2, N1, adv1)
        W1 = assemble(mesh.c1, mesh.c1, W1e, (n1, n1))
        self.WA = restrict(W1, f1, f1)
        self.FA = (cb.MA / dt + (eta / mu0) * cb.KA + self.WA).tocsr()
        self.Wp = W1
        self.Fp = (cb.Mp / dt + W1 + mu * cb.Kp).tocsr()
        self.Bbar = mean_field(mesh, Abar)
