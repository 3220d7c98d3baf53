"""Sequential time stepping with the single-step preconditioner P_{T,k}
(st_timestep_solve) against the oracle, through the C ABI.

* EXACT inner mode, FP64, the 8 x 8 mesh with 8 slabs: the solution at
  rtol 1e-13 equals the direct all-at-once x* per block to 1e-10, and the
  per-step FGMRES iteration counts are the oracle's time stepping's (exact
  inner solves, GMRES with P_{T,k}) up to rounding (G16: +-1 per step).
* Production inner solves, FP32 and FP64 preconditioner: the space-time
  residual recomputed by the oracle meets 1e-8, on a ragged 5-slab horizon.
* Cold and warm starts give the same solution to the tolerance.
* Windows of several slabs (windowed space-time, each window with its own P_T):
  EXACT mode equals x* with the oracle's per-window iteration counts (+-1),
  production FP32 meets the space-time tolerance.
"""
import functools
import sys

import numpy as np
import pytest

import oracle
from oracle.timestepping import solve_time_stepping, solve_windows
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
def case(n, nt, dt=0.1, re=100.0):
    cfg = inputs.Config(f"ts{n}x{nt}", n, nt, dt, re, re)
    ub, ab = inputs.state(cfg)
    return cfg, ub, ab, oracle.system_from_config(cfg, ub, ab)


def stepping(cfg, ub, ab, **kw):
    from paper_2309_00768_amd import binding
    return binding.TimeStepping(cfg.n, cfg.nt, cfg.dt, cfg.mu, cfg.eta, cfg.mu0, ub, ab, **kw)


def test_exact_time_stepping_matches_direct_solution_and_oracle_counts():
    say("[gpu] time stepping EXACT fp64 n=8 nt=8")
    cfg, ub, ab, ref = case(8, 8)
    ts = stepping(cfg, ub, ab, inner="exact")
    b = inputs.rhs(cfg, 1)
    x, infos, rc = ts.solve(dev(b), rtol=1e-13)
    its = [i.iterations for i in infos]
    _, its_ref, _ = solve_time_stepping(cfg.n, cfg.nt, cfg.dt, cfg.mu, cfg.eta, cfg.mu0, ub, ab, b, rtol=1e-13)
    say(f"    its gpu {its} oracle {its_ref}")
    assert rc == 0 and all(i.converged for i in infos)
    assert_blocks(x.cpu().numpy(), ref.direct_solve(b), ts.offsets, cfg.nt, 1e-10, "x vs x*")
    assert all(abs(a - r) <= 1 for a, r in zip(its, its_ref)), (its, its_ref)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_production_time_stepping_reaches_1e8(precision):
    say(f"[gpu] time stepping {precision} n=12 nt=5")
    cfg, ub, ab, ref = case(12, 5, dt=0.05)
    ts = stepping(cfg, ub, ab, precision=precision)
    b = inputs.rhs(cfg, 2)
    x, infos, rc = ts.solve(dev(b), rtol=1e-8)
    assert rc == 0
    bp = ref.project_pressure(b)
    res = np.linalg.norm(bp - ref.apply_J(x.cpu().numpy())) / np.linalg.norm(bp)
    say(f"    its {[i.iterations for i in infos]} residual {res:.2e}")
    assert res <= 1e-8


def test_warm_and_cold_starts_agree():
    say("[gpu] time stepping warm vs cold start n=6 nt=4")
    cfg, ub, ab, ref = case(6, 4)
    ts = stepping(cfg, ub, ab)
    b = inputs.rhs(cfg, 3)
    xw, iw, rcw = ts.solve(dev(b), rtol=1e-12, warm_start=True)
    xc, ic, rcc = ts.solve(dev(b), rtol=1e-12, warm_start=False)
    assert rcw == 0 and rcc == 0
    xs = ref.direct_solve(b)
    assert_blocks(xw.cpu().numpy(), xs, ts.offsets, cfg.nt, 1e-9, "warm")
    assert_blocks(xc.cpu().numpy(), xs, ts.offsets, cfg.nt, 1e-9, "cold")


@pytest.mark.parametrize("window", [2, 3])
def test_windowed_space_time_matches_direct_solution(window):
    """Windows of W slabs solved all at once in turn (the last one shorter:
    7 slabs in windows of 2 or 3), each coupled to the previous window's last
    slab: EXACT mode reaches the direct x* per block; production FP32 solves meet
    the space-time tolerance (oracle residual)."""
    say(f"[gpu] windowed space-time, windows of {window} slabs, n=6 nt=7")
    cfg, ub, ab, ref = case(6, 7)
    b = inputs.rhs(cfg, 1)
    ts = stepping(cfg, ub, ab, inner="exact", window=window)
    assert len(ts.systems) == -(-cfg.nt // window)
    x, infos, rc = ts.solve(dev(b), rtol=1e-13)
    assert rc == 0 and all(i.converged for i in infos)
    assert_blocks(x.cpu().numpy(), ref.direct_solve(b), ts.offsets, cfg.nt, 1e-10, f"x vs x* (windows of {window})")
    its = [i.iterations for i in infos]
    _, its_ref, _ = solve_windows(cfg.n, cfg.nt, cfg.dt, cfg.mu, cfg.eta, cfg.mu0, ub, ab, b, window, rtol=1e-13)
    say(f"    its per window gpu {its} oracle {its_ref}")
    assert all(abs(a - r) <= 1 for a, r in zip(its, its_ref)), (its, its_ref)
    ts32 = stepping(cfg, ub, ab, precision="fp32", window=window, restart=60)
    x, infos, rc = ts32.solve(dev(b), rtol=1e-8)
    bp = ref.project_pressure(b)
    res = np.linalg.norm(bp - ref.apply_J(x.cpu().numpy())) / np.linalg.norm(bp)
    say(f"    fp32: iterations per window {[i.iterations for i in infos]}, oracle residual {res:.2e}")
    assert rc == 0 and res <= 1.05e-8
