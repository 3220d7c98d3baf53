"""Space-time Jacobian, block preconditioner P_T, GMRES and direct solves (oracle).

References into the paper:

* space-time Jacobian J, eq. (jacobianSTDiscrete), with the block
  lower-bidiagonal F_u and F_A of eqs. (STFu)/(STFA) and the block-diagonal
  coupling blocks of eqs. (lorentz)/(STother);
* preconditioner P_T = Ubar_ujA Utilde_up, eq. (PT), whose inverse is
  Utilde_up^{-1} Ubar_ujA^{-1} with Ubar_ujA from eq. (barUuja) and Utilde_up
  from eq. (Utilde);
* pressure Schur approximation S_p ~ -K_p F_p^{-1} M_p with the space-time
  F_p of eq. (Fp);
* magnetic Schur approximation S_A^{-1} ~ C_A^{-1} F_A M_A^{-1},
  eq. (ASchurApprox), with the block lower tri-diagonal C_A of
  eqs. (CAspacetime)/(CAs) built with the diagonal of M_A;
* GMRES on J, right preconditioned (Sec. "Performance of preconditioner");
* exact inner solves: sequential time stepping for F_u and C_A and sparse LU
  for every spatial block (Sec. "Performance of preconditioner").

Unknowns of one slab are ordered [u_x | u_y | p | j | A]; the space-time vector
is slab-major.  Velocity and A use only interior nodes.  Pressure is fixed up to
a constant per slab; every solve here returns pressure with zero mean,
1^T M_p p^k = 0, and every right-hand side has its pressure rows projected to
zero sum per slab (the range of the divergence).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .blocks import ConstantBlocks, SlabBlocks, current_from_potential
from .fem import Mesh


class SpaceTimeSystem:
    """All blocks of J and P_T for one configuration and linearisation state.

    ``ubar`` has shape (nt, 2, (2n+1)^2), ``Abar`` shape (nt, (n+1)^2).  ``jbar``
    (nt, (n+1)^2) defaults to the discrete current of ``Abar``.
    """

    def __init__(self, n, nt, dt, mu, eta, mu0, ubar, Abar, jbar=None):
        self.n, self.nt, self.dt, self.mu, self.eta, self.mu0 = n, nt, dt, mu, eta, mu0
        self.mesh = Mesh(n)
        self.cb = ConstantBlocks(self.mesh, mu0)
        cb = self.cb
        self.nu = cb.Mu.shape[0]
        self.np_ = cb.Mp.shape[0]
        self.nj = cb.Mj.shape[0]
        self.na = cb.MA.shape[0]
        self.offs = np.cumsum([0, self.nu, self.np_, self.nj, self.na])
        self.ns = int(self.offs[-1])
        self.N = self.ns * nt
        if jbar is None:
            jbar = np.stack([current_from_potential(cb, Abar[k], mu0) for k in range(nt)])
        self.ubar, self.Abar, self.jbar = ubar, Abar, jbar
        self.slabs = [SlabBlocks(self.mesh, cb, ubar[k], Abar[k], jbar[k], dt, mu, eta, mu0) for k in range(nt)]
        self._lu = {}
        self._wave = None

    # ----------------------------------------------------------------- layout
    def split(self, x):
        """View a space-time vector as per-slab blocks u, p, j, A (each (nt, size))."""
        X = x.reshape(self.nt, self.ns)
        o = self.offs
        return X[:, o[0]:o[1]], X[:, o[1]:o[2]], X[:, o[2]:o[3]], X[:, o[3]:o[4]]

    def join(self, u, p, j, a):
        return np.concatenate([u, p, j, a], axis=1).ravel()

    def project_pressure(self, x):
        """Remove the per-slab mean of the pressure rows (Euclidean): the range of B."""
        u, p, j, a = (b.copy() for b in self.split(x))
        p -= p.mean(axis=1, keepdims=True)
        return self.join(u, p, j, a)

    def normalise_pressure(self, x):
        """Shift each slab's pressure so that 1^T M_p p^k = 0."""
        u, p, j, a = (b.copy() for b in self.split(x))
        m = np.asarray(self.cb.Mp.sum(axis=0)).ravel()
        p -= (p @ m)[:, None] / m.sum()
        return self.join(u, p, j, a)

    # ----------------------------------------------------------- slab matrix
    def slab_jacobian(self, k):
        """Single-step Jacobian of slab k, eq. (jacobianDiscrete)."""
        s, cb = self.slabs[k], self.cb
        return sp.bmat([
            [s.Fu, cb.B.T, s.Zj, s.ZA],
            [cb.B, None, None, None],
            [None, None, cb.Mj, cb.KjA],
            [s.Y, None, None, s.FA]]).tocsr()

    def coupling(self):
        """Sub-diagonal slab coupling: J_{k,k-1} = -diag(Mu/dt, 0, 0, MA/dt)."""
        cb = self.cb
        zp = sp.csr_matrix((self.np_, self.np_))
        zj = sp.csr_matrix((self.nj, self.nj))
        return -sp.block_diag([cb.Mu / self.dt, zp, zj, cb.MA / self.dt]).tocsr()

    def assemble_J(self):
        """The whole space-time Jacobian as one sparse matrix (small sizes only)."""
        C = self.coupling()
        blocks = [[None] * self.nt for _ in range(self.nt)]
        for k in range(self.nt):
            blocks[k][k] = self.slab_jacobian(k)
            if k > 0:
                blocks[k][k - 1] = C
        return sp.bmat(blocks).tocsr()

    # ------------------------------------------------------------- J applies
    def apply_J(self, x):
        """y = J x, eq. (jacobianSTDiscrete): per slab, the single-step Jacobian plus the
        -M/dt coupling to the previous slab for u and A."""
        u, p, j, a = self.split(x)
        cb, dt = self.cb, self.dt
        yu, yp, yj, ya = [], [], [], []
        for k in range(self.nt):
            s = self.slabs[k]
            vu = s.Fu @ u[k] + cb.B.T @ p[k] + s.Zj @ j[k] + s.ZA @ a[k]
            va = s.Y @ u[k] + s.FA @ a[k]
            if k > 0:
                vu -= cb.Mu @ u[k - 1] / dt
                va -= cb.MA @ a[k - 1] / dt
            yu.append(vu)
            yp.append(cb.B @ u[k])
            yj.append(cb.Mj @ j[k] + cb.KjA @ a[k])
            ya.append(va)
        return self.join(np.array(yu), np.array(yp), np.array(yj), np.array(ya))

    def apply_JT(self, x):
        """y = J^T x: per slab the transposed single-step Jacobian plus the -M/dt coupling
        to the next slab (the mass matrices are symmetric)."""
        u, p, j, a = self.split(x)
        cb, dt = self.cb, self.dt
        yu, yp, yj, ya = [], [], [], []
        for k in range(self.nt):
            s = self.slabs[k]
            vu = s.Fu.T @ u[k] + cb.B.T @ p[k] + s.Y.T @ a[k]
            va = s.ZA.T @ u[k] + cb.KjA.T @ j[k] + s.FA.T @ a[k]
            if k + 1 < self.nt:
                vu -= cb.Mu @ u[k + 1] / dt
                va -= cb.MA @ a[k + 1] / dt
            yu.append(vu)
            yp.append(cb.B @ u[k])
            yj.append(s.Zj.T @ u[k] + cb.Mj @ j[k])
            ya.append(va)
        return self.join(np.array(yu), np.array(yp), np.array(yj), np.array(ya))

    # ------------------------------------------------------- exact factors
    def _factor(self, key, mat_fn):
        if key not in self._lu:
            self._lu[key] = spla.splu(sp.csc_matrix(mat_fn()))
        return self._lu[key]

    def _kp_bordered(self):
        """Bordered Neumann Laplacian [[Kp, 1], [1^T, 0]] (returns the zero-sum solution)."""
        Kp = self.cb.Kp
        one = np.ones((Kp.shape[0], 1))
        return sp.bmat([[Kp, sp.csr_matrix(one)], [sp.csr_matrix(one.T), None]])

    def solve_Kp(self, r):
        lu = self._factor("Kp", self._kp_bordered)
        return lu.solve(np.append(r, 0.0))[:-1]

    def wave_blocks(self):
        """Blocks of C_A, eq. (CAs), with D the diagonal of the (interior) M_A.

        C0[k] = F_{A,k} D^{-1} F_{A,k} + (|Bbar_k|^2 / mu0) K_A         (diagonal band)
        C1[k] = M_A D^{-1} F_{A,k} + F_{A,k+1} D^{-1} M_A, k < nt-1      (band -1, block (k+1, k))
        C2    = M_A D^{-1} M_A                                            (band -2)
        The bands enter C_A with factors 1, -1/dt and +1/dt^2: these are the blocks of
        the product F_A D^{-1} F_A with the lower-bidiagonal F_A of eq. (STFA).
        """
        if self._wave is None:
            cb = self.cb
            Dinv = sp.diags(1.0 / cb.MA.diagonal())
            C0 = [(s.FA @ Dinv @ s.FA + (s.Bbar @ s.Bbar / self.mu0) * cb.KA).tocsr() for s in self.slabs]
            C1 = [(cb.MA @ Dinv @ self.slabs[k].FA + self.slabs[k + 1].FA @ Dinv @ cb.MA).tocsr()
                  for k in range(self.nt - 1)]
            C2 = (cb.MA @ Dinv @ cb.MA).tocsr()
            self._wave = (C0, C1, C2)
        return self._wave

    # ------------------------------------------------------------ P_T^{-1}
    def apply_PT_inv(self, r, normalise=True, schur_p=None, schur_a=None):
        """z = P_T^{-1} r with exact inner solves (eq. (PT)).

        Ubar_ujA^{-1} (back substitution of eq. (barUuja)):
          1. w = M_A^{-1} r_A, s = F_A w, y_A = C_A^{-1} s   (S_A^{-1} of eq. (ASchurApprox))
          2. y_j = M_j^{-1} (r_j - K_jA y_A)
          3. y_u = r_u - Z_j y_j - Z_A y_A,  y_p = r_p
        Utilde_up^{-1} (eq. (Utilde)):
          4. x_p = S_p^{-1} y_p = -M_p^{-1} F_p K_p^{-1} y_p
          5. x_u = F_u^{-1} (y_u - B^T x_p)

        ``schur_p`` / ``schur_a`` optionally replace the two Schur-complement inverses
        (callables on (nt, size) arrays), e.g. by the exact ones of ``exact_schur_inverses``.
        """
        cb, dt, nt = self.cb, self.dt, self.nt
        r = self.project_pressure(r)
        ru, rp, rj, ra = self.split(r)
        luMA = self._factor("MA", lambda: cb.MA)
        luMj = self._factor("Mj", lambda: cb.Mj)
        luMp = self._factor("Mp", lambda: cb.Mp)
        # 1. magnetic Schur complement
        if schur_a is not None:
            yA = schur_a(ra)
        else:
            w = np.array([luMA.solve(ra[k]) for k in range(nt)])
            s = np.array([self.slabs[k].FA @ w[k] - (cb.MA @ w[k - 1] / dt if k > 0 else 0.0) for k in range(nt)])
            yA = self.solve_CA(s)
        # 2.-3.
        yj = np.array([luMj.solve(rj[k] - cb.KjA @ yA[k]) for k in range(nt)])
        yu = np.array([ru[k] - self.slabs[k].Zj @ yj[k] - self.slabs[k].ZA @ yA[k] for k in range(nt)])
        # 4. pressure convection-diffusion
        if schur_p is not None:
            xp = schur_p(rp)
        else:
            q = np.array([self.solve_Kp(rp[k]) for k in range(nt)])
            t = np.array([self.slabs[k].Fp @ q[k] - (cb.Mp @ q[k - 1] / dt if k > 0 else 0.0) for k in range(nt)])
            xp = -np.array([luMp.solve(t[k]) for k in range(nt)])
        # 5. velocity
        xu = self.solve_Fu(np.array([yu[k] - cb.B.T @ xp[k] for k in range(nt)]))
        z = self.join(xu, xp, yj, yA)
        return self.normalise_pressure(z) if normalise else z

    def solve_Fu(self, q):
        """F_u x = q by sequential time stepping: F_{u,k} x^k = q^k + (M_u/dt) x^{k-1}."""
        x = np.empty_like(q)
        for k in range(self.nt):
            lu = self._factor(("Fu", k), lambda k=k: self.slabs[k].Fu)
            rhs = q[k] + (self.cb.Mu @ x[k - 1] / self.dt if k > 0 else 0.0)
            x[k] = lu.solve(rhs)
        return x

    def solve_CA(self, s):
        """C_A y = s by forward substitution over the slabs:
        C0_k y^k = s^k + (1/dt) C1_{k-1} y^{k-1} - (1/dt^2) C2 y^{k-2}."""
        C0, C1, C2 = self.wave_blocks()
        dt = self.dt
        y = np.empty_like(s)
        for k in range(self.nt):
            rhs = s[k].copy()
            if k >= 1:
                rhs += C1[k - 1] @ y[k - 1] / dt
            if k >= 2:
                rhs -= C2 @ y[k - 2] / dt**2
            lu = self._factor(("CA", k), lambda k=k: C0[k])
            y[k] = lu.solve(rhs)
        return y

    # --------------------------------------------------------- P_T^{-T}
    def apply_PT_invT(self, r, normalise=True):
        """z = P_T^{-T} r = Ubar_ujA^{-T} Utilde_up^{-T} r (the transpose of apply_PT_inv).

        Utilde_up^T is block lower triangular: x_u = F_u^{-T} r_u (backward in time),
        x_p = S_p^{-T} (r_p - B x_u) with S_p^{-T} = -K_p^{-1} F_p^T M_p^{-1}.
        Ubar_ujA^T is block lower triangular: y_j = M_j^{-1}(r_j - Z_j^T x_u),
        y_A = S_A^{-T}(r_A - Z_A^T x_u - K_jA^T y_j), S_A^{-T} = M_A^{-1} F_A^T C_A^{-T}.
        """
        cb, dt, nt = self.cb, self.dt, self.nt
        r = self.project_pressure(r)
        ru, rp, rj, ra = self.split(r)
        luMA = self._factor("MA", lambda: cb.MA)
        luMj = self._factor("Mj", lambda: cb.Mj)
        luMp = self._factor("Mp", lambda: cb.Mp)
        xu = self.solve_FuT(ru)
        g = np.array([rp[k] - cb.B @ xu[k] for k in range(nt)])
        g -= g.mean(axis=1, keepdims=True)
        v = np.array([luMp.solve(g[k]) for k in range(nt)])
        t = np.array([self.slabs[k].Fp.T @ v[k] - (cb.Mp @ v[k + 1] / dt if k + 1 < nt else 0.0)
                      for k in range(nt)])
        t -= t.mean(axis=1, keepdims=True)
        xp = -np.array([self.solve_Kp(t[k]) for k in range(nt)])
        yj = np.array([luMj.solve(rj[k] - self.slabs[k].Zj.T @ xu[k]) for k in range(nt)])
        h = np.array([ra[k] - self.slabs[k].ZA.T @ xu[k] - cb.KjA.T @ yj[k] for k in range(nt)])
        c = self.solve_CAT(h)
        f = np.array([self.slabs[k].FA.T @ c[k] - (cb.MA @ c[k + 1] / dt if k + 1 < nt else 0.0)
                      for k in range(nt)])
        yA = np.array([luMA.solve(f[k]) for k in range(nt)])
        z = self.join(xu, xp, yj, yA)
        return self.normalise_pressure(z) if normalise else z

    def solve_FuT(self, q):
        """F_u^T x = q backward in time: F_{u,k}^T x^k = q^k + (M_u/dt) x^{k+1}."""
        x = np.empty_like(q)
        for k in reversed(range(self.nt)):
            lu = self._factor(("FuT", k), lambda k=k: self.slabs[k].Fu.T)
            rhs = q[k] + (self.cb.Mu @ x[k + 1] / self.dt if k + 1 < self.nt else 0.0)
            x[k] = lu.solve(rhs)
        return x

    def solve_CAT(self, s):
        """C_A^T y = s backward in time:
        C0_k^T y^k = s^k + (1/dt) C1_k^T y^{k+1} - (1/dt^2) C2^T y^{k+2}."""
        C0, C1, C2 = self.wave_blocks()
        dt = self.dt
        y = np.empty_like(s)
        for k in reversed(range(self.nt)):
            rhs = s[k].copy()
            if k + 1 < self.nt:
                rhs += C1[k].T @ y[k + 1] / dt
            if k + 2 < self.nt:
                rhs -= C2.T @ y[k + 2] / dt**2
            lu = self._factor(("CAT", k), lambda k=k: C0[k].T)
            y[k] = lu.solve(rhs)
        return y

    # --------------------------------------------------------- direct solves
    def _bordered_slab(self, k, transpose=False):
        """Slab Jacobian bordered with the pressure normalisation 1^T M_p p = 0."""
        Jk = self.slab_jacobian(k)
        if transpose:
            Jk = Jk.T
        e = np.zeros(self.ns)
        m = np.asarray(self.cb.Mp.sum(axis=0)).ravel()
        e[self.offs[1]:self.offs[2]] = m
        e = sp.csr_matrix(e[:, None])
        return sp.bmat([[Jk, e], [e.T, None]])

    def direct_solve(self, b):
        """x* = J^{-1} b by block forward substitution in time with one sparse LU per slab:
        J_k x^k = b^k + diag(Mu/dt, 0, 0, MA/dt) x^{k-1}."""
        b = self.project_pressure(b).reshape(self.nt, self.ns)
        C = self.coupling()
        x = np.empty_like(b)
        for k in range(self.nt):
            lu = self._factor(("Jk", k), lambda k=k: self._bordered_slab(k))
            rhs = b[k] - (C @ x[k - 1] if k > 0 else 0.0)
            x[k] = lu.solve(np.append(rhs, 0.0))[:-1]
        return x.ravel()

    def direct_solve_T(self, g):
        """lambda* = J^{-T} g by block backward substitution in time:
        J_k^T lam^k = g^k + diag(Mu/dt, 0, 0, MA/dt) lam^{k+1}."""
        g = self.project_pressure(g).reshape(self.nt, self.ns)
        C = self.coupling()
        x = np.empty_like(g)
        for k in reversed(range(self.nt)):
            lu = self._factor(("JkT", k), lambda k=k: self._bordered_slab(k, transpose=True))
            rhs = g[k] - (C.T @ x[k + 1] if k + 1 < self.nt else 0.0)
            x[k] = lu.solve(np.append(rhs, 0.0))[:-1]
        return x.ravel()

    # ------------------------------------------------ space-time block matrices
    def st_bidiagonal(self, diag_blocks, sub_block):
        """Block lower-bidiagonal space-time matrix with the given diagonal blocks and a
        constant sub-diagonal block (eqs. (STFu)/(STFA)/(Fp))."""
        nt = self.nt
        rows = [[None] * nt for _ in range(nt)]
        for k in range(nt):
            rows[k][k] = diag_blocks[k]
            if k > 0:
                rows[k][k - 1] = sub_block
        return sp.bmat(rows).tocsr()

    def st_matrices(self):
        """Variable-major space-time blocks of J and P_T (small sizes only)."""
        cb, dt, nt = self.cb, self.dt, self.nt
        bd = lambda blocks: sp.block_diag(blocks).tocsr()
        m = {
            "Fu": self.st_bidiagonal([s.Fu for s in self.slabs], -cb.Mu / dt),
            "FA": self.st_bidiagonal([s.FA for s in self.slabs], -cb.MA / dt),
            "Fp": self.st_bidiagonal([s.Fp for s in self.slabs], -cb.Mp / dt),
            "B": bd([cb.B] * nt), "Zj": bd([s.Zj for s in self.slabs]), "ZA": bd([s.ZA for s in self.slabs]),
            "Mj": bd([cb.Mj] * nt), "KjA": bd([cb.KjA] * nt), "Y": bd([s.Y for s in self.slabs]),
            "MA": bd([cb.MA] * nt), "Mp": bd([cb.Mp] * nt), "Kp": bd([cb.Kp] * nt),
            "KAw": bd([(s.Bbar @ s.Bbar / self.mu0) * cb.KA for s in self.slabs]),
            "D": bd([sp.diags(cb.MA.diagonal())] * nt),
        }
        C0, C1, C2 = self.wave_blocks()
        rows = [[None] * nt for _ in range(nt)]
        for k in range(nt):
            rows[k][k] = C0[k]
            if k >= 1:
                rows[k][k - 1] = -C1[k - 1] / dt
            if k >= 2:
                rows[k][k - 2] = C2 / dt**2
        m["CA"] = sp.bmat(rows, format="csr") if nt > 1 else C0[0].tocsr()
        return m

    def slab_major_permutation(self):
        """perm such that x_slab_major = x_variable_major[perm]."""
        nt, o = self.nt, self.offs
        sizes = np.diff(o)
        var_off = np.concatenate([[0], np.cumsum(sizes * nt)])
        perm = np.empty(self.N, dtype=np.int64)
        for k in range(nt):
            for v in range(4):
                perm[k * self.ns + o[v]: k * self.ns + o[v + 1]] = var_off[v] + k * sizes[v] + np.arange(sizes[v])
        return perm

    def exact_schur_inverses(self):
        """Exact Schur complements (dense; tiny sizes only):
        S_p = -B F_u^{-1} B^T (inverted on zero-sum pressures per slab), and
        S_A = F_A - Y F_u^{-1} (Z_A - Z_j M_j^{-1} K_jA), eq. (ASchurApprox1+)."""
        m = self.st_matrices()
        Fu_inv = np.linalg.inv(m["Fu"].toarray())
        B = m["B"].toarray()
        Sp = -B @ Fu_inv @ B.T
        Z = m["ZA"].toarray() - m["Zj"].toarray() @ np.linalg.solve(m["Mj"].toarray(), m["KjA"].toarray())
        SA = m["FA"].toarray() - m["Y"].toarray() @ Fu_inv @ Z
        Sp_pinv = np.linalg.pinv(Sp, rcond=1e-12)
        SA_inv = np.linalg.inv(SA)
        nt = self.nt
        sp_fn = lambda yp: (Sp_pinv @ yp.ravel()).reshape(nt, -1)
        sa_fn = lambda ra: (SA_inv @ ra.ravel()).reshape(nt, -1)
        return sp_fn, sa_fn


def gmres(apply_A, apply_Minv, b, restart=30, rtol=1e-8, maxit=2000, x0=None, true_residual=None):
    """Right-preconditioned restarted GMRES with modified Gram-Schmidt and Givens rotations.

    Stops when the true residual ||b - A x|| <= rtol ||b|| (checked whenever the
    recurrence estimate reaches the tolerance and at every restart).  Returns
    (x, iterations, history of estimated relative residuals).
    """
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, 0, [0.0]
    its, hist = 0, []
    while its < maxit:
        r = b - apply_A(x)
        beta = np.linalg.norm(r)
        hist.append(beta / bnorm)
        if beta <= rtol * bnorm:
            break
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart))
        cs, sn = np.zeros(restart), np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        m = 0
        for j in range(restart):
            z = apply_Minv(V[j])
            Z.append(z)
            w = apply_A(z)
            for i in range(j + 1):
                H[i, j] = np.dot(V[i], w)
                w = w - H[i, j] * V[i]
            hnext = np.linalg.norm(w)
            H[j + 1, j] = hnext
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            d = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / d, H[j + 1, j] / d
            H[j, j] = d
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            m = j + 1
            hist.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) <= rtol * bnorm or its >= maxit:
                break
            V.append(w / hnext)
        y = np.linalg.solve(np.triu(H[:m, :m]), g[:m])
        for i in range(m):
            x = x + y[i] * Z[i]
        if np.linalg.norm(b - apply_A(x)) <= rtol * bnorm:
            break
    return x, its, hist


def solve_fgmres(sysm: SpaceTimeSystem, b, restart=30, rtol=1e-8, maxit=2000, precond=None):
    """GMRES on J with right preconditioner P_T (or ``precond``); pressure projected on input
    and normalised on output."""
    b = sysm.project_pressure(b)
    M = precond if precond is not None else sysm.apply_PT_inv
    x, its, hist = gmres(sysm.apply_J, M, b, restart=restart, rtol=rtol, maxit=maxit)
    return sysm.normalise_pressure(x), its, hist
