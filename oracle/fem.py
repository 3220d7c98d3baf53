"""Finite-element building blocks of the oracle: bases, quadrature, meshes, assembly.

Discretisation (paper, Sec. "Problem definition and discretisation", recurrence
eq. (recurrence), and Sec. "Results" for the element choice): backward Euler in
time and finite elements in space.  This oracle uses Taylor-Hood Q2-Q1 for
velocity-pressure and Q1 for current and vector potential on a uniform mesh of
``n x n`` squares of the unit square.

Every integrand of the linearised operators is a polynomial of degree at most 6
in each coordinate on an affine square, so tensor Gauss-Legendre with 5 points
per direction (exact to degree 9) gives the exact Galerkin matrices.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

QUAD_PTS_1D = 5


def gauss01(m: int):
    """Gauss-Legendre points and weights mapped to [0, 1]."""
    x, w = np.polynomial.legendre.leggauss(m)
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange1d(deg: int, s: np.ndarray):
    """Values and first derivatives of the equispaced 1-D Lagrange basis of degree ``deg`` on [0, 1].

    Written from the definition L_a(s) = prod_{b != a} (s - s_b) / (s_a - s_b).
    Returns arrays of shape (deg+1, len(s)).
    """
    nodes = np.linspace(0.0, 1.0, deg + 1)
    s = np.asarray(s, dtype=float)
    val = np.empty((deg + 1, s.size))
    der = np.empty((deg + 1, s.size))
    for a in range(deg + 1):
        others = [nodes[b] for b in range(deg + 1) if b != a]
        denom = np.prod([nodes[a] - o for o in others])
        val[a] = np.prod([s - o for o in others], axis=0) / denom
        d = np.zeros_like(s)
        for i in range(len(others)):
            term = np.ones_like(s)
            for j, o in enumerate(others):
                if j != i:
                    term = term * (s - o)
            d += term
        der[a] = d / denom
    return val, der


class RefSquare:
    """Tensor-product Lagrange basis of degree ``deg`` tabulated at the tensor Gauss points.

    Local node (a, b) (a along x, b along y) has index a + (deg+1) b.  Arrays:
    ``N[i, q]``, ``Ns[i, q]`` (d/ds) and ``Nt[i, q]`` (d/dt) on the reference
    square [0,1]^2, and the weights ``w[q]`` (summing to 1).
    """

    def __init__(self, deg: int, m: int = QUAD_PTS_1D):
        s, ws = gauss01(m)
        v, d = lagrange1d(deg, s)
        nb = deg + 1
        nq = m * m
        self.deg, self.nloc, self.nq = deg, nb * nb, nq
        self.N = np.empty((nb * nb, nq))
        self.Ns = np.empty((nb * nb, nq))
        self.Nt = np.empty((nb * nb, nq))
        for b in range(nb):
            for a in range(nb):
                i = a + nb * b
                # quadrature point index: qx + m * qy
                self.N[i] = np.outer(v[b], v[a]).ravel()
                self.Ns[i] = np.outer(v[b], d[a]).ravel()
                self.Nt[i] = np.outer(d[b], v[a]).ravel()
        self.w = np.outer(ws, ws).ravel()
        self.s = np.tile(s, m)
        self.t = np.repeat(s, m)


class Mesh:
    """Uniform mesh of the unit square with ``n x n`` square cells.

    Element e = ex + n ey.  Q2 nodes live on the (2n+1)^2 grid and Q1 nodes on
    the (n+1)^2 grid, both numbered lexicographically with x fastest.
    """

    def __init__(self, n: int):
        self.n = n
        self.h = 1.0 / n
        self.nq2 = (2 * n + 1) ** 2
        self.nq1 = (n + 1) ** 2
        ex, ey = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
        ex, ey = ex.ravel(), ey.ravel()          # element order e = ex + n*ey
        self.ex, self.ey = ex, ey
        self.ne = n * n
        c2 = np.empty((self.ne, 9), dtype=np.int64)
        for b in range(3):
            for a in range(3):
                c2[:, a + 3 * b] = (2 * ex + a) + (2 * n + 1) * (2 * ey + b)
        c1 = np.empty((self.ne, 4), dtype=np.int64)
        for b in range(2):
            for a in range(2):
                c1[:, a + 2 * b] = (ex + a) + (n + 1) * (ey + b)
        self.c2, self.c1 = c2, c1
        # Interior ("free") node lists: homogeneous Dirichlet is imposed on the boundary.
        i2 = np.arange(2 * n + 1)
        m2 = (i2 > 0) & (i2 < 2 * n)
        self.free2 = np.flatnonzero(np.outer(m2, m2).ravel())
        i1 = np.arange(n + 1)
        m1 = (i1 > 0) & (i1 < n)
        self.free1 = np.flatnonzero(np.outer(m1, m1).ravel())
        self.q2 = RefSquare(2)
        self.q1 = RefSquare(1)


def assemble(rows: np.ndarray, cols: np.ndarray, local: np.ndarray, shape) -> sp.csr_matrix:
    """Sum element matrices ``local[e, a, b]`` into global (rows[e, a], cols[e, b])."""
    E, na, nb = local.shape
    R = np.broadcast_to(rows[:, :, None], (E, na, nb)).ravel()
    C = np.broadcast_to(cols[:, None, :], (E, na, nb)).ravel()
    A = sp.coo_matrix((local.ravel(), (R, C)), shape=shape).tocsr()
    A.sum_duplicates()
    return A


def assemble_vec(rows: np.ndarray, local: np.ndarray, size: int) -> np.ndarray:
    """Sum element vectors ``local[e, a]`` into a global vector at rows[e, a]."""
    out = np.zeros(size)
    np.add.at(out, rows.ravel(), local.ravel())
    return out


def at_quad(ref: RefSquare, conn: np.ndarray, nodal: np.ndarray, h: float):
    """Value and physical gradient of a nodal field at every element's quadrature points.

    Returns (val, dx, dy), each of shape (E, nq).
    """
    loc = nodal[conn]                       # (E, nloc)
    val = loc @ ref.N
    dx = (loc @ ref.Ns) / h
    dy = (loc @ ref.Nt) / h
    return val, dx, dy


def restrict(A: sp.spmatrix, rows=None, cols=None) -> sp.csr_matrix:
    """Sub-matrix on the given row and column index sets (None = all)."""
    A = A.tocsr()
    if rows is not None:
        A = A[rows, :]
    if cols is not None:
        A = A[:, cols]
    return A.tocsr()
