"""The allocation-free preconditioner apply (st_apply_precond_noalloc) against
st_apply_precond, through the C ABI.

Two calls in a row on one GPU, the second on a smaller system, so the second
runs on the static scratch the first left behind; each must equal the
workspace-scratch apply of its own system bit for bit (same kernels, same
order), in FP64 and in FP32.  A system whose scratch exceeds the static array
is rejected before any launch.
"""
import sys

import numpy as np
import pytest

from paper_2309_00768_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def system(n, nt, precision, **kw):
    from paper_2309_00768_amd import binding
    cfg = inputs.Config(f"na{n}x{nt}", n, nt, 0.1, 100.0, 100.0)
    ub, ab = inputs.state(cfg)
    plan = binding.Plan(cfg.n, cfg.nt, cfg.dt, cfg.mu, cfg.eta, cfg.mu0, ub, ab, precision=precision, **kw)
    return binding.System(plan, "cuda:0")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("single_stream", [False, True])
def test_noalloc_precond_matches_workspace_apply(precision, single_stream):
    say(f"[gpu] st_apply_precond_noalloc {precision} single_stream={single_stream}: n=12 nt=20 then n=5 nt=3")
    for n, nt in ((12, 20), (5, 3)):
        sysg = system(n, nt, precision, single_stream=single_stream)
        r = torch.from_numpy(np.random.default_rng(20 + n).standard_normal(sysg.N)).to("cuda:0")
        z_ws = sysg.apply_precond(r)
        z_na = torch.full_like(r, float("nan"))
        sysg.apply_precond_noalloc(r, z_na)
        torch.cuda.synchronize()
        say(f"    n={n} nt={nt}: bitwise equal {torch.equal(z_ws, z_na)}")
        assert torch.equal(z_ws, z_na)
        # repeated on the scratch it just used
        z_na2 = torch.full_like(r, float("nan"))
        sysg.apply_precond_noalloc(r, z_na2)
        torch.cuda.synchronize()
        assert torch.equal(z_ws, z_na2)


def test_noalloc_rejects_a_system_beyond_the_static_scratch():
    """The 64 x 64 mesh with 128 slabs in FP64 needs about 170 MB of
    preconditioner scratch, more than the 128 MiB array: ST_ENOMEM, and the
    output is left untouched."""
    say("[gpu] st_apply_precond_noalloc size rejection (n=64 nt=128 fp64)")
    from paper_2309_00768_amd import binding
    cfg = inputs.CONFIGS["cfg3"]
    ub, ab = inputs.state(cfg)
    plan = binding.Plan(cfg.n, cfg.nt, cfg.dt, cfg.mu, cfg.eta, cfg.mu0, ub, ab, precision="fp64",
                        single_stream=True)
    sysg = binding.System(plan, "cuda:0")
    r = torch.ones(sysg.N, dtype=torch.float64, device="cuda:0")
    z = torch.zeros_like(r)
    with pytest.raises(binding.StError) as e:
        sysg.apply_precond_noalloc(r, z)
    assert e.value.code == -3
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(z)) == 0
