"""Seeded synthetic inputs shared by the library tests, the benchmark and the oracle.

This module holds no arithmetic of the method: it only lays out node grids,
samples smooth closed-form fields at those nodes, and draws seeded random
right-hand sides.  Everything here is data handed identically to both the HIP
library and the CPU oracle.

Workload recipe (the paper's model problems, Sec. "Model problems", are
near-equilibrium magnetic states on the unit square; these seeded fields stand
in for them with the sizes of the five benchmark configurations):

* mesh: unit square, ``n x n`` square cells; velocity on the Q2 node grid
  ``(2n+1)^2`` (two components), pressure / current / vector potential on the Q1
  grid ``(n+1)^2``; lexicographic node order, x fastest;
* linearisation state ("Fourier" generator): for each of ``u_x, u_y, A``,
  ``0.1 * sum_{m=1..4} s_m cos(p_m pi x + a_m) cos(q_m pi y + b_m)
  * (1 + cos(w_m t + g_m) / 2) / 1.5`` with ``p, q ~ U{1,2,3}``, ``s = +-1``,
  ``a, b, g ~ U[0, 2pi)``, ``w ~ U[pi, 4pi]``, drawn with ``numpy.random.default_rng``;
  sampled at ``t_k = k dt`` for the slabs ``k = 1..Nt``;
* shear-layer state: ``A = tanh((y - 1/2) / 0.1) + 0.01 cos(pi x)``, constant
  in time, with the velocity from the Fourier generator;
* right-hand sides: N(0, 1) on every free unknown, slab-major;
* batch of uneven systems: n and Nt drawn per system (``batch_configs``).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class Config:
    """One space-time problem: mesh, slabs, time step and the two Reynolds numbers."""

    name: str
    n: int            # cells per side of the unit square
    nt: int           # number of backward-Euler slabs
    dt: float         # time step
    re: float         # fluid Reynolds number, viscosity mu = 1 / re
    s: float          # Lundquist number, resistivity eta = 1 / s
    mu0: float = 1.0  # magnetic permeability
    state: str = "fourier"   # "fourier" or "shear"
    state_seed: int = 0
    rhs_seeds: tuple = (1,)

    @property
    def mu(self) -> float:
        return 1.0 / self.re

    @property
    def eta(self) -> float:
        return 1.0 / self.s


# The five workloads (sizes, time steps, Reynolds numbers) of the benchmark suite.
CONFIGS = {
    "cfg1": Config("cfg1", 8, 8, 0.1, 100.0, 100.0, rhs_seeds=(1,)),
    "cfg2": Config("cfg2", 32, 32, 0.05, 100.0, 100.0, state="shear", rhs_seeds=(1, 2, 3)),
    "cfg3": Config("cfg3", 64, 128, 0.01, 100.0, 100.0, rhs_seeds=(1,)),
    "cfg3_re1000": Config("cfg3_re1000", 64, 128, 0.01, 1000.0, 1000.0, rhs_seeds=(1,)),
    "cfg5": Config("cfg5", 128, 128, 0.005, 500.0, 500.0, rhs_seeds=(1,)),
}


def batch_configs(count: int = 16, seed: int = 0, meshes=(16, 32, 48, 64, 96), max_nt: int = 256,
                  re: float = 300.0) -> list:
    """The uneven batch workload: ``count`` systems with n drawn from ``meshes``
    and Nt from {16, 32, ..., max_nt} (seeded draw), dt = 1/Nt (final time 1),
    Re = S = ``re``; system i has state seed 100 + i and right-hand-side seed 200 + i."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.choice(np.asarray(meshes)))
        nt = 16 * int(rng.integers(1, max_nt // 16 + 1))
        out.append(Config(f"batch{i}", n, nt, 1.0 / nt, re, re, state_seed=100 + i, rhs_seeds=(200 + i,)))
    return out


def slab_sizes(n: int) -> dict:
    """Unknown counts of one slab in the order [u_x | u_y | p | j | A].

    Velocity and vector potential carry homogeneous Dirichlet conditions on the
    boundary (those nodes are not unknowns); pressure and current use all nodes.
    """
    nu1 = (2 * n - 1) ** 2
    nq1 = (n + 1) ** 2
    na = (n - 1) ** 2
    sizes = {"ux": nu1, "uy": nu1, "p": nq1, "j": nq1, "A": na}
    offs, o = {}, 0
    for k in ("ux", "uy", "p", "j", "A"):
        offs[k] = o
        o += sizes[k]
    return {"sizes": sizes, "offsets": offs, "slab": o}


def q2_coords(n: int):
    """x and y of the (2n+1)^2 Q2 nodes, lexicographic with x fastest."""
    t = np.arange(2 * n + 1) / (2.0 * n)
    y, x = np.meshgrid(t, t, indexing="ij")
    return x.ravel(), y.ravel()


def q1_coords(n: int):
    """x and y of the (n+1)^2 Q1 nodes, lexicographic with x fastest."""
    t = np.arange(n + 1) / float(n)
    y, x = np.meshgrid(t, t, indexing="ij")
    return x.ravel(), y.ravel()


def _fourier_params(rng, nfields=3, modes=4):
    out = []
    for _ in range(nfields):
        modes_f = []
        for _ in range(modes):
            p = int(rng.integers(1, 4))
            q = int(rng.integers(1, 4))
            s = 1.0 if rng.random() < 0.5 else -1.0
            a, b, g = rng.uniform(0.0, 2.0 * math.pi, size=3)
            w = rng.uniform(math.pi, 4.0 * math.pi)
            modes_f.append((p, q, s, a, b, g, w))
        out.append(modes_f)
    return out


def _fourier_field(modes, x, y, t, amp=0.1):
    f = np.zeros_like(x)
    for (p, q, s, a, b, g, w) in modes:
        f += s * np.cos(p * math.pi * x + a) * np.cos(q * math.pi * y + b) * (1.0 + 0.5 * math.cos(w * t + g)) / 1.5
    return amp * f


def state(cfg: Config):
    """Linearisation state of every slab.

    Returns ``(ubar, Abar)`` with ``ubar`` of shape ``(nt, 2, (2n+1)^2)`` (Q2 nodal
    velocity, all nodes) and ``Abar`` of shape ``(nt, (n+1)^2)`` (Q1 nodal vector
    potential, all nodes), both float64 and C-contiguous.
    """
    rng = np.random.default_rng(cfg.state_seed)
    params = _fourier_params(rng)
    x2, y2 = q2_coords(cfg.n)
    x1, y1 = q1_coords(cfg.n)
    ubar = np.empty((cfg.nt, 2, x2.size))
    Abar = np.empty((cfg.nt, x1.size))
    for k in range(cfg.nt):
        t = (k + 1) * cfg.dt
        ubar[k, 0] = _fourier_field(params[0], x2, y2, t)
        ubar[k, 1] = _fourier_field(params[1], x2, y2, t)
        if cfg.state == "shear":
            Abar[k] = np.tanh((y1 - 0.5) / 0.1) + 0.01 * np.cos(math.pi * x1)
        else:
            Abar[k] = _fourier_field(params[2], x1, y1, t)
    return np.ascontiguousarray(ubar), np.ascontiguousarray(Abar)


def constant_state(cfg: Config, a_value: float = 0.0, zero_velocity: bool = False):
    """State with a spatially constant vector potential (so the current vanishes).

    The velocity comes from the Fourier generator unless ``zero_velocity``.
    """
    ubar, _ = state(cfg)
    if zero_velocity:
        ubar = np.zeros_like(ubar)
    Abar = np.full((cfg.nt, (cfg.n + 1) ** 2), float(a_value))
    return ubar, Abar


def rhs(cfg: Config, seed: int) -> np.ndarray:
    """N(0,1) right-hand side on all free unknowns, slab-major, float64."""
    n_slab = slab_sizes(cfg.n)["slab"]
    rng = np.random.default_rng(seed)
    return rng.standard_normal(cfg.nt * n_slab)


def random_vector(length: int, seed: int) -> np.ndarray:
    """Seeded N(0,1) vector of a given length (test directions, adjoint data)."""
    return np.random.default_rng(seed).standard_normal(length)


def free_a_field(cfg: Config, seed: int) -> np.ndarray:
    """A smooth Fourier-type field sampled at the interior Q1 nodes, e.g. an initial potential."""
    rng = np.random.default_rng(seed)
    params = _fourier_params(rng, nfields=1)
    x1, y1 = q1_coords(cfg.n)
    f = _fourier_field(params[0], x1, y1, 0.0).reshape(cfg.n + 1, cfg.n + 1)
    return np.ascontiguousarray(f[1:-1, 1:-1].ravel())


# --------------------------------------------------------- model problems ---
# The paper's two model problems (Sec. "Model problems") as closed-form nodal
# fields on the unit square: a magnetic equilibrium (A_eq, the pressure p_eq
# that balances its Lorentz force, and the electric field E_eq that sustains
# it against resistive diffusion), a quiet flow, and a perturbed initial
# potential.  Island coalescence lives on the unit square as in the paper;
# the tearing mode's Harris sheet is centred at y = 1/2 of the unit square
# (x-length L = 1).  Boundary values are those of the fields (Dirichlet on
# every side for u and A).


@dataclasses.dataclass(frozen=True)
class ModelProblem:
    name: str
    n: int
    nt: int
    dt: float
    mu: float = 1.0
    eta: float = 1.0
    mu0: float = 1.0


def model_fields(prob: ModelProblem):
    """(A_eq, p_eq, E_eq) at the Q1 nodes and A_init (the perturbed initial
    potential) at the Q1 nodes, float64; the flow is at rest (u = 0)."""
    x, y = q1_coords(prob.n)
    if prob.name == "island":
        beta, eps = 0.2, 1e-3
        den = np.cosh(2 * math.pi * y) + beta * np.cos(2 * math.pi * x)
        A = np.log(den) / (2 * math.pi)
        p = (1 - beta ** 2) / den ** 2 / (2 * prob.mu0)
        E = (prob.eta / prob.mu0) * 2 * math.pi * (1 - beta ** 2) / den ** 2
        A0 = A + eps * np.cos(0.5 * math.pi * y) * np.cos(math.pi * x)
    elif prob.name == "tearing":
        lam, eps, L = 5.0, 1e-3, 1.0
        ys = y - 0.5
        A = np.log(np.cosh(lam * ys)) / lam
        p = 1.0 / np.cosh(lam * ys) ** 2 / (2 * prob.mu0)
        E = (lam * prob.eta / prob.mu0) / np.cosh(lam * ys) ** 2
        A0 = A - eps * np.cos(math.pi * ys) * np.cos(2 * math.pi * x / L)
    else:
        raise ValueError(prob.name)
    return A, p - p.mean(), E, A0


def model_newton_fields(prob: ModelProblem):
    """Base fields, fields at t_0 and forcing of the model problem's space-time
    Newton solve, float64 C-contiguous:

    * base: every slab at the equilibrium (u = 0, p = p_eq, A = A_eq), except
      that A's boundary values are those of the initial potential (Dirichlet
      data, fixed in time);
    * u_init = 0, A_init = the perturbed potential;
    * E: the sustaining electric field on every slab; no momentum forcing.

    The base current is not included: it solves the discrete current equation
    of each slab's base potential (computed by the solver in use)."""
    A, p, E, A0 = model_fields(prob)
    n, nt = prob.n, prob.nt
    nq2 = (2 * n + 1) ** 2
    x, y = q1_coords(n)
    bnd = (x == 0.0) | (x == 1.0) | (y == 0.0) | (y == 1.0)
    Ab = np.where(bnd, A0, A)
    return {
        "u_base": np.zeros((nt, 2, nq2)),
        "p_base": np.ascontiguousarray(np.tile(p, (nt, 1))),
        "a_base": np.ascontiguousarray(np.tile(Ab, (nt, 1))),
        "u_init": np.zeros((2, nq2)),
        "a_init": np.ascontiguousarray(A0),
        "e": np.ascontiguousarray(np.tile(E, (nt, 1))),
    }
