"""Pins of the oracle's current state j from the potential A (the current equation of the
paper's recurrence, eq. (recurrence), with zero data: the initialisation of j in Sec.
"Model problems").  Both checks are independent of the matrix assembly that
``current_from_potential`` uses."""
import numpy as np
import pytest

from oracle.blocks import ConstantBlocks, current_from_potential
from oracle.fem import Mesh
from oracle.nonlinear import slab_residual


@pytest.mark.parametrize("n,mu0", [(3, 1.0), (5, 0.7)])
def test_current_row_of_the_recurrence_vanishes_at_the_current_state(n, mu0):
    """The current row of the residual of eq. (recurrence), evaluated by quadrature of the
    fields (no matrices), is zero at (jbar(A), A) for any A and any other field."""
    rng = np.random.default_rng(3)
    mesh = Mesh(n)
    cb = ConstantBlocks(mesh, mu0)
    nq1, nq2 = (n + 1) ** 2, (2 * n + 1) ** 2
    A = rng.standard_normal(nq1)
    j = current_from_potential(cb, A, mu0)
    u = rng.standard_normal((2, nq2))
    p = rng.standard_normal(nq1)
    R = slab_residual(mesh, (u, p, j, A), (rng.standard_normal((2, nq2)), rng.standard_normal(nq1)),
                      0.1, 0.02, 0.03, mu0)
    nu = 2 * mesh.free2.size
    Rj = R[nu + nq1: nu + 2 * nq1]
    # scale of the two terms that cancel: int j chi
    scale = np.linalg.norm(cb.M1full @ j)
    assert scale > 1.0
    assert np.linalg.norm(Rj) <= 1e-12 * scale
    # and with the opposite sign (or a wrong 1/mu0) the row does not vanish
    R2 = slab_residual(mesh, (u, p, -j, A), (u, p), 0.1, 0.02, 0.03, mu0)
    assert np.linalg.norm(R2[nu + nq1: nu + 2 * nq1]) > 0.5 * scale


def test_current_converges_to_laplacian_of_potential_at_second_order():
    """For A = sin^2(pi x) sin^2(pi y) (zero normal derivative, so the natural boundary term of
    the current equation vanishes) the discrete current at every node tends to
    Laplace(A)/mu0 = 2 pi^2 [cos(2 pi x) sin^2(pi y) + sin^2(pi x) cos(2 pi y)] / mu0 at O(h^2)."""
    mu0 = 2.0
    errs = []
    for n in (8, 16, 32):
        mesh = Mesh(n)
        cb = ConstantBlocks(mesh, mu0)
        g = np.linspace(0.0, 1.0, n + 1)
        X, Y = np.meshgrid(g, g)          # nodes lexicographic, x fastest
        A = (np.sin(np.pi * X) ** 2 * np.sin(np.pi * Y) ** 2).ravel()
        lap = 2 * np.pi ** 2 * (np.cos(2 * np.pi * X) * np.sin(np.pi * Y) ** 2
                                + np.sin(np.pi * X) ** 2 * np.cos(2 * np.pi * Y))
        j = current_from_potential(cb, A, mu0)
        errs.append(np.abs(j - lap.ravel() / mu0).max())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 1.9), (errs, orders)
    # |Laplace(A)/mu0| reaches 2 pi^2 / 2 ~ 9.9; at n = 32 the nodal error is 0.064
    assert errs[-1] < 0.1
