"""GPU parity of the HIP path against the CPU oracle (through the C ABI).

Tolerances (relative, 2-norm, asserted for the whole vector and for each of
the variable blocks u, p, j, A over all slabs): J and J^T apply 1e-12; P_T^{-1}
/ P_T^{-T} with converged inner solves 1e-10; FGMRES at rtol 1e-13 vs the
direct time-stepping solution 1e-10; production (AMG) and FP32-preconditioner
solves: true FP64 residual <= 1e-8 recomputed by the oracle.
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


@functools.lru_cache(maxsize=None)
def case(n, nt, dt=0.1, re=100.0, s=100.0, state="fourier", seed=0):
    cfg = inputs.Config(f"n{n}nt{nt}", n, nt, dt, re, s, state=state, state_seed=seed)
    ub, ab = inputs.state(cfg)
    return cfg, ub, ab, oracle.system_from_config(cfg, ub, ab)


@functools.lru_cache(maxsize=None)
def gpu_system(n, nt, precision="fp64", inner="exact", dt=0.1, re=100.0, s=100.0, state="fourier"):
    from paper_2309_00768_amd import binding
    cfg, ub, ab, _ = case(n, nt, dt, re, s, state)
    plan = binding.Plan(cfg.n, cfg.nt, cfg.dt, cfg.mu, cfg.eta, cfg.mu0, ub, ab, precision=precision, inner=inner,
                        adjoint=True)
    return binding.System(plan, "cuda:0")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


SMALL = [(8, 8), (2, 1), (3, 5), (5, 2)]


@pytest.mark.parametrize("n,nt", SMALL)
def test_jacobian_apply(n, nt):
    say(f"[gpu] J apply n={n} nt={nt}")
    cfg, ub, ab, ref = case(n, nt)
    sysg = gpu_system(n, nt)
    x = np.random.default_rng(3).standard_normal(ref.N)
    y = sysg.apply_jacobian(dev(x)).cpu().numpy()
    assert_blocks(y, ref.apply_J(x), sysg.offsets, nt, 1e-12, "J")
    yt = sysg.apply_jacobian(dev(x), transpose=True).cpu().numpy()
    assert_blocks(yt, ref.apply_JT(x), sysg.offsets, nt, 1e-12, "J^T")


@pytest.mark.parametrize("n,nt", [(8, 8), (3, 5)])
def test_precond_exact_parity(n, nt):
    say(f"[gpu] P_T^-1 exact n={n} nt={nt}")
    cfg, ub, ab, ref = case(n, nt)
    sysg = gpu_system(n, nt)
    r = np.random.default_rng(4).standard_normal(ref.N)
    z = sysg.apply_precond(dev(r)).cpu().numpy()
    assert_blocks(z, ref.apply_PT_inv(r), sysg.offsets, nt, 1e-10, "P_T^-1")
    zt = sysg.apply_precond(dev(r), transpose=True).cpu().numpy()
    assert_blocks(zt, ref.apply_PT_invT(r), sysg.offsets, nt, 1e-10, "P_T^-T")


@pytest.mark.parametrize("n,nt", [(8, 8), (3, 5)])
def test_production_stencil_sweeps_match_oracle(n, nt):
    """The sweeps the benchmark runs (structured 5x5 stencils, each step solving
    for its increment over a predictor from the earlier slabs with the combined
    coupling stencils, Chebyshev-Jacobi alone, recorded two-program replay; the
    current solves of a chunk in one workgroup) with converged spatial solves:
    degree 40 on F_u,k and 80 on C_A,k leave 2 r^d below 1e-17 on the estimated
    intervals (kappa <= 16 here), and EXACT mode converges the K_p and mass
    solves.  P_T^{-1} and P_T^{-T} then equal the oracle's exact-inner operators
    of eq. (PT) block by block."""
    say(f"[gpu] production stencil sweeps vs oracle n={n} nt={nt}")
    from paper_2309_00768_amd import binding
    cfg, ub, ab, ref = case(n, nt)
    plan = binding.Plan(cfg.n, cfg.nt, cfg.dt, cfg.mu, cfg.eta, cfg.mu0, ub, ab, inner="exact", fu_solver=40,
                        ca_solver=80, adjoint=True, sweep_format=0)
    fu_deg, ca_deg, fu_kappa, ca_kappa = plan.solver_info()
    assert (fu_deg, ca_deg) == (40, 80)
    for deg, kappa in ((fu_deg, fu_kappa), (ca_deg, ca_kappa)):
        r = (kappa ** 0.5 - 1) / (kappa ** 0.5 + 1)
        assert 2 * r ** deg < 1e-14, (deg, kappa)
    sysg = binding.System(plan, "cuda:0")
    r = np.random.default_rng(14).standard_normal(ref.N)
    z = sysg.apply_precond(dev(r)).cpu().numpy()
    assert_blocks(z, ref.apply_PT_inv(r), sysg.offsets, nt, 1e-10, "P_T^-1 stencil")
    zt = sysg.apply_precond(dev(r), transpose=True).cpu().numpy()
    assert_blocks(zt, ref.apply_PT_invT(r), sysg.offsets, nt, 1e-10, "P_T^-T stencil")


def test_fgmres_exact_cfg1_matches_direct_solution():
    say("[gpu] FGMRES exact cfg1")
    cfg, ub, ab, ref = case(8, 8)
    sysg = gpu_system(8, 8)
    b = inputs.rhs(cfg, 1)
    xs = ref.direct_solve(b)
    x, info, rc, hist = sysg.solve(dev(b), rtol=1e-13, restart=30, history=200)
    say(f"    its={info.iterations} res={info.true_rel_residual:.2e}")
    assert rc == 0 and info.converged == 1
    assert_blocks(x.cpu().numpy(), xs, sysg.offsets, cfg.nt, 1e-10, "x vs x*")


def test_adjoint_exact_cfg1_matches_backward_substitution():
    say("[gpu] adjoint exact cfg1")
    cfg, ub, ab, ref = case(8, 8)
    sysg = gpu_system(8, 8)
    g = np.random.default_rng(6).standard_normal(ref.N)
    ls = ref.direct_solve_T(g)
    lam, info, rc, _ = sysg.solve(dev(g), rtol=1e-13, adjoint=True)
    say(f"    its={info.iterations} res={info.true_rel_residual:.2e}")
    assert rc == 0
    assert_blocks(lam.cpu().numpy(), ls, sysg.offsets, cfg.nt, 1e-10, "lambda vs lambda*")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fgmres_amg_reaches_1e8(precision):
    say(f"[gpu] FGMRES amg {precision} cfg1")
    cfg, ub, ab, ref = case(8, 8)
    sysg = gpu_system(8, 8, precision=precision, inner="amg")
    b = inputs.rhs(cfg, 1)
    x, info, rc, _ = sysg.solve(dev(b), rtol=1e-8)
    say(f"    its={info.iterations} res={info.true_rel_residual:.2e}")
    assert rc == 0
    xh = x.cpu().numpy()
    bp = ref.project_pressure(b)
    assert np.linalg.norm(bp - ref.apply_J(xh)) <= 1e-8 * np.linalg.norm(bp)


@pytest.mark.parametrize("n,nt", [(8, 8), (3, 5), (6, 1)])
def test_stencil_and_sell_sweeps_agree(n, nt):
    """Sweeps with converged spatial solves (Chebyshev-Jacobi of degree 40 on
    F_u,k and 80 on C_A,k, whose estimated interval is wider) agree
    whatever the form: the stencil sweeps solve for the increment over a
    predictor with combined coupling stencils, the SELL sweeps for the whole
    slab from zero with the plain couplings.  P_T^{-1} and P_T^{-T} (FP64) agree
    to 1e-10, which checks the combined stencils against the plain blocks."""
    say(f"[gpu] stencil vs SELL sweeps n={n} nt={nt}")
    from paper_2309_00768_amd import binding
    cfg, ub, ab, ref = case(n, nt)
    out = []
    for fmt in (0, 1):
        plan = binding.Plan(cfg.n, cfg.nt, cfg.dt, cfg.mu, cfg.eta, cfg.mu0, ub, ab, fu_solver=40, ca_solver=80,
                            adjoint=True, sweep_format=fmt)
        sysg = binding.System(plan, "cuda:0")
        r = np.random.default_rng(8).standard_normal(ref.N)
        out.append((sysg.apply_precond(dev(r)).cpu().numpy(), sysg.apply_precond(dev(r), transpose=True).cpu().numpy()))
    assert_blocks(out[0][0], out[1][0], sysg.offsets, nt, 1e-10, "P_T^-1")
    assert_blocks(out[0][1], out[1][1], sysg.offsets, nt, 1e-10, "P_T^-T")


def test_long_horizon_fp32_sweeps_stay_accurate():
    """224 slabs of the uneven-batch recipe (n = 16, dt = 1/224, Re = S = 300): with
    approximate spatial solves a sweep that solves each slab from zero amplifies
    their error by the recursion (the FP32 solve then stagnates); the increment
    form keeps P_T usable and FGMRES reaches 1e-8."""
    say("[gpu] long-horizon FP32 solve n=16 nt=224")
    from paper_2309_00768_amd import binding
    cfg = inputs.batch_configs()[4]
    assert (cfg.n, cfg.nt) == (16, 224)
    ub, ab = inputs.state(cfg)
    plan = binding.Plan(cfg.n, cfg.nt, cfg.dt, cfg.mu, cfg.eta, cfg.mu0, ub, ab, precision="fp32")
    sysg = binding.System(plan, "cuda:0")
    b = dev(inputs.rhs(cfg, cfg.rhs_seeds[0]))
    x, info, rc, _ = sysg.solve(b, rtol=1e-8, maxit=1500)
    say(f"    its={info.iterations} res={info.true_rel_residual:.2e}")
    assert rc == 0 and info.true_rel_residual <= 1e-8


@pytest.mark.parametrize("precision,inner", [("fp64", "amg"), ("fp32", "amg"), ("fp64", "exact")])
def test_pipelined_sweeps_match_single_stream(precision, inner):
    """The recorded two-program pipelines (for P_T^{-1}: a C_A sweep step and an
    F_u sweep step in one launch, chunk by chunk; for P_T^{-T}: the backward F_u^T
    sweep beside the backward C_A^T sweep of the chunks already done) compute
    exactly what the step-by-step order computes, and repeated applies give
    identical results.  20 slabs in chunks of 6 leave a ragged last chunk."""
    say(f"[gpu] recorded pipeline vs step-by-step {precision} {inner}")
    from paper_2309_00768_amd import binding
    cfg, ub, ab, ref = case(8, 20)
    out = []
    for single in (False, True):
        plan = binding.Plan(cfg.n, cfg.nt, cfg.dt, cfg.mu, cfg.eta, cfg.mu0, ub, ab, precision=precision,
                            inner=inner, single_stream=single, sweep_chunk=6, sweep_chain=False, adjoint=True)
        sysg = binding.System(plan, "cuda:0")
        r = np.random.default_rng(9).standard_normal(ref.N)
        res = []
        for tr in (False, True):
            z = sysg.apply_precond(dev(r), transpose=tr)
            z2 = sysg.apply_precond(dev(r), transpose=tr)
            torch.cuda.synchronize()
            assert torch.equal(z, z2)
            res.append(z.cpu().numpy())
        out.append(res)
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("n,nt,fu,ca", [(12, 6, 4, 4), (12, 6, 7, 11), (20, 3, 5, 2), (3, 4, 1, 6)])
def test_fused_sweep_solves_match_per_step(precision, n, nt, fu, ca):
    """The tiled sweep solve (8 x 8 node tiles grown by halos in LDS, up to 4
    Chebyshev steps in the first launch of a solve and 3 in each later one)
    computes what one launch per step computes.  The meshes give ragged tiles
    (F_u grids of 23 x 23, 39 x 39 and 5 x 5 nodes; C_A grids of 11 x 11,
    19 x 19 and 2 x 2), the degrees one and several launches per solve; both
    P_T^{-1} (recorded pipeline) and P_T^{-T} are compared."""
    say(f"[gpu] fused vs per-step sweep solves {precision} n={n} nt={nt} fu={fu} ca={ca}")
    from paper_2309_00768_amd import binding
    cfg, ub, ab, ref = case(n, nt)
    out = []
    for fuse in (True, False):
        plan = binding.Plan(cfg.n, cfg.nt, cfg.dt, cfg.mu, cfg.eta, cfg.mu0, ub, ab, precision=precision,
                            fu_solver=fu, ca_solver=ca, adjoint=True, sweep_fuse=fuse, sweep_chain=False)
        sysg = binding.System(plan, "cuda:0")
        r = np.random.default_rng(10).standard_normal(ref.N)
        z = sysg.apply_precond(dev(r)).cpu().numpy()
        zt = sysg.apply_precond(dev(r), transpose=True).cpu().numpy()
        out.append((z, zt))
    tol = 1e-13 if precision == "fp64" else 1e-6
    say(f"    bitwise equal: {np.array_equal(out[0][0], out[1][0])}, {np.array_equal(out[0][1], out[1][1])}; "
        f"rel {rel(out[0][0], out[1][0]):.1e}, {rel(out[0][1], out[1][1]):.1e}")
    assert rel(out[0][0], out[1][0]) <= tol
    assert rel(out[0][1], out[1][1]) <= tol


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_autotuned_launches_give_the_same_results(precision):
    """st_create with autotune = 1 times the J slabs per wavefront, the sweep
    step rows per workgroup and the tiled solve on the system itself; whatever
    it picks, J x, P_T^{-1} r and P_T^{-T} r are bitwise those of the default
    launches."""
    say(f"[gpu] autotuned launches {precision}")
    from paper_2309_00768_amd import binding
    cfg, ub, ab, ref = case(12, 6)
    out = []
    for tune in (False, True):
        plan = binding.Plan(cfg.n, cfg.nt, cfg.dt, cfg.mu, cfg.eta, cfg.mu0, ub, ab, precision=precision,
                            adjoint=True, autotune=tune)
        sysg = binding.System(plan, "cuda:0")
        t = sysg.tuning()
        say(f"    autotune={tune}: {t}")
        assert t["j_slabs"] in (1, 4, 8) and t["step_rows"] in (64, 128, 256) and t["step_lanes"] in (1, 2)
        r = np.random.default_rng(11).standard_normal(ref.N)
        out.append([sysg.apply_jacobian(dev(r)).cpu().numpy(), sysg.apply_precond(dev(r)).cpu().numpy(),
                    sysg.apply_precond(dev(r), transpose=True).cpu().numpy()])
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-4)])
def test_chain_kernel_matches_per_step_launches(precision, tol):
    """Launched step by step on grids of at most 1024 rows, the C_A sweep and the
    current solves of a chunk run in one workgroup (k_ca_chain).  They agree with
    the per-step launches up to the summation order of the stencil and SELL forms
    of K_jA and M_j."""
    say(f"[gpu] chain kernel vs per-step launches {precision}")
    from paper_2309_00768_amd import binding
    cfg, ub, ab, ref = case(8, 20)
    out = []
    for chain in (True, False):
        plan = binding.Plan(cfg.n, cfg.nt, cfg.dt, cfg.mu, cfg.eta, cfg.mu0, ub, ab, precision=precision,
                            single_stream=True, sweep_chain=chain)
        sysg = binding.System(plan, "cuda:0")
        r = np.random.default_rng(12).standard_normal(ref.N)
        out.append(sysg.apply_precond(dev(r)).cpu().numpy())
    say(f"    rel {rel(out[0], out[1]):.1e}")
    assert rel(out[0], out[1]) <= tol


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("n,nt", [(12, 6), (3, 4), (20, 3)])
def test_two_lane_sweep_steps_match_one_lane(precision, n, nt):
    """F_u,k sweep steps with the row's two column components on two lanes
    (partial sums exchanged between the lanes) compute what one lane per row
    computes, bit for bit, in P_T^{-1} (recorded replay) and P_T^{-T}; the
    meshes leave ragged last workgroups (F_u grids of 23 x 23, 5 x 5 and
    39 x 39 nodes per component)."""
    say(f"[gpu] two-lane vs one-lane sweep steps {precision} n={n} nt={nt}")
    from paper_2309_00768_amd import binding
    cfg, ub, ab, ref = case(n, nt)
    out = []
    for lanes in (1, 2):
        plan = binding.Plan(cfg.n, cfg.nt, cfg.dt, cfg.mu, cfg.eta, cfg.mu0, ub, ab, precision=precision,
                            adjoint=True, sweep_lanes=lanes, sweep_chain=False)
        sysg = binding.System(plan, "cuda:0")
        assert sysg.tuning()["step_lanes"] == lanes
        r = np.random.default_rng(15).standard_normal(ref.N)
        out.append((sysg.apply_precond(dev(r)).cpu().numpy(), sysg.apply_precond(dev(r), transpose=True).cpu().numpy()))
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])
