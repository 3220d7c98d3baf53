"""The full preconditioner P and P-tilde (eqs. (preconditioner),
(preconditionerSimplified1)) on the GPU against the oracle, through the C ABI.

* EXACT inner mode, FP64: P^{-1} r and P-tilde^{-1} r equal the oracle's
  compositions of exact factor inverses per block to 1e-10.
* FGMRES with each preconditioner reaches the direct solution at rtol 1e-13
  (EXACT mode) and a true residual of 1e-8 with the production inner solves
  in FP32; the iteration counts of P, P-tilde and P_T are reported (the paper
  finds them close, Sec. "Block-triangular approximation").
* The forward-only variants reject the transposed apply.
"""
import functools
import sys

import numpy as np
import pytest

import oracle
from oracle import variants
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
def case(n, nt):
    cfg = inputs.Config(f"v{n}x{nt}", n, nt, 0.1, 100.0, 100.0)
    ub, ab = inputs.state(cfg)
    return cfg, ub, ab, oracle.system_from_config(cfg, ub, ab)


def system(cfg, ub, ab, variant, **kw):
    from paper_2309_00768_amd import binding
    plan = binding.Plan(cfg.n, cfg.nt, cfg.dt, cfg.mu, cfg.eta, cfg.mu0, ub, ab, variant=variant, **kw)
    return binding.System(plan, "cuda:0")


@pytest.mark.parametrize("variant", ["Ptilde", "P"])
@pytest.mark.parametrize("n,nt", [(8, 8), (3, 5)])
def test_variant_apply_matches_oracle(variant, n, nt):
    say(f"[gpu] {variant}^-1 exact vs oracle n={n} nt={nt}")
    cfg, ub, ab, ref = case(n, nt)
    sysg = system(cfg, ub, ab, variant, inner="exact")
    r = np.random.default_rng(16).standard_normal(ref.N)
    z = sysg.apply_precond(dev(r)).cpu().numpy()
    assert_blocks(z, variants.apply_inv(ref, r, variant), sysg.offsets, nt, 1e-10, f"{variant}^-1")


@pytest.mark.parametrize("variant", ["PT", "Ptilde", "P"])
def test_variant_fgmres(variant):
    say(f"[gpu] FGMRES with {variant} n=8 nt=8")
    cfg, ub, ab, ref = case(8, 8)
    b = inputs.rhs(cfg, 1)
    xs = ref.direct_solve(b)
    sysx = system(cfg, ub, ab, variant, inner="exact")
    x, info, rc, _ = sysx.solve(dev(b), rtol=1e-13)
    say(f"    exact: its={info.iterations}")
    assert rc == 0
    assert_blocks(x.cpu().numpy(), xs, sysx.offsets, cfg.nt, 1e-10, "x vs x*")
    sys32 = system(cfg, ub, ab, variant, precision="fp32")
    x, info, rc, _ = sys32.solve(dev(b), rtol=1e-8)
    bp = ref.project_pressure(b)
    res = np.linalg.norm(bp - ref.apply_J(x.cpu().numpy())) / np.linalg.norm(bp)
    say(f"    fp32 production: its={info.iterations} residual {res:.2e}")
    assert rc == 0 and res <= 1e-8


def test_variants_are_forward_only():
    from paper_2309_00768_amd import binding
    cfg, ub, ab, ref = case(3, 2)
    sysg = system(cfg, ub, ab, "P")
    r = dev(np.ones(ref.N))
    with pytest.raises(binding.StError):
        sysg.apply_precond(r, transpose=True)
    with pytest.raises(binding.StError):
        sysg.apply_precond_noalloc(r, torch.zeros_like(r))
