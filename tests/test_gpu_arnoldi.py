"""FGMRES with delayed reorthogonalisation (``orth="delayed"``) on the GPU,
against the oracle's GMRES and direct solutions, through the C ABI.

Both Gram-Schmidt forms build an orthonormal basis of the same Krylov space
and minimise the residual over it, so with a fixed preconditioner (exact inner
solves, FP64) their iterates are the same up to rounding:

* the iterate after k steps without convergence (one cycle, and GMRES(1) over
  several cycles) equals the oracle's GMRES iterate;
* a converged solve equals the oracle's direct solution x* (and the adjoint
  solve its transposed direct solution);
* with the production FP32 preconditioner and a long restart (the automatic
  choice takes the delayed form above restart 64), also through a long residual
  plateau, the oracle's residual of the result meets the tolerance and the
  iteration count is that of CGS2 within a few;
* iteration caps are exact, a zero right-hand side gives zero, and a batch
  rejects the delayed form.
"""
import functools
import sys

import numpy as np
import pytest

import oracle
from paper_2309_00768_amd import inputs
from parity_util import assert_blocks

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@functools.lru_cache(maxsize=None)
def case(n, nt, re=100.0):
    cfg = inputs.Config(f"ar{n}x{nt}", n, nt, 0.1 if re <= 100 else 0.01, re, re)
    ub, ab = inputs.state(cfg)
    return cfg, ub, ab, oracle.system_from_config(cfg, ub, ab)


@functools.lru_cache(maxsize=None)
def system(n, nt, re=100.0, precision="fp64", adjoint=False, max_restart=30):
    from paper_2309_00768_amd import binding
    cfg, ub, ab, _ = case(n, nt, re)
    kw = {"inner": "exact"} if precision == "fp64" else {}
    plan = binding.Plan(cfg.n, cfg.nt, cfg.dt, cfg.mu, cfg.eta, cfg.mu0, ub, ab, precision=precision,
                        adjoint=adjoint, max_restart=max_restart, **kw)
    return binding.System(plan, "cuda:0")


@pytest.mark.parametrize("restart,steps", [(12, 12), (1, 3), (5, 13)])
def test_delayed_iterate_matches_oracle_gmres(restart, steps):
    say(f"[gpu] delayed reorthogonalisation: iterate after {steps} steps of GMRES({restart}) vs oracle")
    cfg, ub, ab, ref = case(8, 8)
    sysg = system(8, 8)
    b = inputs.rhs(cfg, 1)
    xr, its, _ = oracle.gmres(ref.apply_J, ref.apply_PT_inv, ref.project_pressure(b), restart=restart,
                              rtol=1e-14, maxit=steps)
    assert its == steps
    xr = ref.normalise_pressure(xr)
    for orth in ("delayed", "cgs2"):
        x, info, rc, _ = sysg.solve(dev(b), restart=restart, rtol=1e-14, maxit=steps, orth=orth)
        assert info.iterations == steps and rc != 0
        assert_blocks(x.cpu().numpy(), xr, sysg.offsets, cfg.nt, 1e-10, f"x_{steps} {orth}")


def test_delayed_converged_solve_is_direct_solution():
    say("[gpu] delayed reorthogonalisation: converged FP64 solve vs direct solution")
    cfg, ub, ab, ref = case(8, 8)
    sysg = system(8, 8)
    b = inputs.rhs(cfg, 2)
    xs = ref.direct_solve(b)
    its = {}
    for orth in ("delayed", "cgs2"):
        x, info, rc, _ = sysg.solve(dev(b), rtol=1e-13, orth=orth)
        its[orth] = info.iterations
        assert rc == 0
        assert_blocks(x.cpu().numpy(), xs, sysg.offsets, cfg.nt, 1e-10, f"x {orth}")
    say(f"    iterations {its}")
    assert abs(its["delayed"] - its["cgs2"]) <= 1


def test_delayed_adjoint_solve_is_transposed_direct_solution():
    say("[gpu] delayed reorthogonalisation: adjoint solve vs transposed direct solution")
    cfg, ub, ab, ref = case(6, 5)
    sysg = system(6, 5, adjoint=True)
    g = np.random.default_rng(31).standard_normal(ref.N)
    lam_ref = ref.direct_solve_T(g)
    lam, info, rc, _ = sysg.solve(dev(g), rtol=1e-13, adjoint=True, orth="delayed")
    assert rc == 0
    assert_blocks(lam.cpu().numpy(), lam_ref, sysg.offsets, cfg.nt, 1e-9, "lambda delayed")


def test_long_restart_fp32_automatic_delayed():
    """Re = S = 1000 on a 16 x 16 mesh, 32 slabs: the residual plateau needs a long
    restart; GMRES(150) picks the delayed form by itself."""
    say("[gpu] FP32 preconditioner, GMRES(150), automatic (delayed) vs CGS2")
    cfg, ub, ab, ref = case(16, 32, 1000.0)
    sysg = system(16, 32, 1000.0, precision="fp32", max_restart=150)
    b = inputs.rhs(cfg, 1)
    bp = ref.project_pressure(b)
    its = {}
    for orth in ("auto", "cgs2"):
        x, info, rc, _ = sysg.solve(dev(b), restart=150, rtol=1e-8, maxit=600, orth=orth)
        res = np.linalg.norm(bp - ref.apply_J(x.cpu().numpy())) / np.linalg.norm(bp)
        its[orth] = info.iterations
        say(f"    {orth}: {info.iterations} its, oracle residual {res:.2e}")
        assert rc == 0 and res <= 1.05e-8
    assert abs(its["auto"] - its["cgs2"]) <= 2


def test_long_restart_plateau_fp32_delayed():
    """Re = S = 1000, 16 x 16 mesh, 128 slabs: a plateau of about 170 iterations in
    one GMRES(200) cycle, with subdiagonal entries of the Hessenberg matrix far
    from 1 (the unit-scaled pending vector keeps the delayed form in range)."""
    say("[gpu] FP32 preconditioner, GMRES(200) through a residual plateau, delayed vs CGS2")
    cfg, ub, ab, ref = case(16, 128, 1000.0)
    sysg = system(16, 128, 1000.0, precision="fp32", max_restart=200)
    b = inputs.rhs(cfg, 1)
    bp = ref.project_pressure(b)
    its = {}
    for orth in ("delayed", "cgs2"):
        x, info, rc, _ = sysg.solve(dev(b), restart=200, rtol=1e-8, maxit=600, orth=orth)
        res = np.linalg.norm(bp - ref.apply_J(x.cpu().numpy())) / np.linalg.norm(bp)
        its[orth] = info.iterations
        say(f"    {orth}: {info.iterations} its, oracle residual {res:.2e}")
        assert rc == 0 and res <= 1.05e-8
    assert abs(its["delayed"] - its["cgs2"]) <= max(3, its["cgs2"] // 50)


def test_delayed_zero_rhs_and_caps():
    say("[gpu] delayed reorthogonalisation: zero rhs, iteration caps")
    cfg, ub, ab, ref = case(8, 8)
    sysg = system(8, 8)
    z = torch.zeros(ref.N, dtype=torch.float64, device="cuda:0")
    x, info, rc, _ = sysg.solve(z, orth="delayed")
    assert rc == 0 and info.iterations == 0 and float(x.abs().max()) == 0.0
    b = dev(inputs.rhs(cfg, 1))
    for cap in (1, 2, 7):
        _, info, rc, hist = sysg.solve(b, rtol=1e-14, maxit=cap, history=16, orth="delayed")
        assert rc != 0 and info.iterations == cap and len(hist) == cap + 1
        assert np.all(np.isfinite(hist)) and hist[-1] < hist[0]


def test_unknown_orth_is_rejected():
    from paper_2309_00768_amd import binding
    sysg = system(8, 8)
    b = dev(inputs.rhs(case(8, 8)[0], 1))
    binding.ORTH["bad"] = 3
    try:
        with pytest.raises(RuntimeError):
            sysg.solve(b, maxit=5, orth="bad")
    finally:
        del binding.ORTH["bad"]


def test_batch_rejects_delayed():
    from paper_2309_00768_amd import binding
    sysg = system(8, 8)
    batch = binding.Batch([sysg])
    b = dev(inputs.rhs(case(8, 8)[0], 1))
    with pytest.raises(RuntimeError):
        batch.solve([b], maxit=10, orth="delayed")
    _, infos, st, rc, _ = batch.solve([b], maxit=10, orth="cgs2")
    assert infos[0].iterations == 10
