"""The Chebyshev intervals (or ellipses) that the host setup chooses for the
spatial solves of the F_u and C_A sweeps, against the true spectra of
D^{-1} F_u,k and D^{-1} C_A,k from the oracle's blocks (dense eigenvalues).

The iteration with centre theta and foci theta -+ c reduces the eigencomponent
at lambda by |w + sqrt(w^2 - 1)| / (the same at 0), w = (theta - lambda) / c
(Manteuffel, Numer. Math. 28, 1977); the plan exports (theta, delta) with
c = delta for delta > 0 and c = i |delta| otherwise.

* A block with eigenvalues far off the real axis (12 x 12 mesh, 4 slabs,
  dt = 1/8, Re = S = 1000; the real interval's iteration diverges there) gets
  ellipses with imaginary foci on F_u, and the iteration contracts every
  eigenvalue of every slab, at about the factor the degree choice assumes.
* The C_A,k blocks of a member of the uneven batch get ellipses with
  imaginary foci that contract every eigenvalue.
* The cfg1 blocks keep real intervals that contract every eigenvalue.
"""
import numpy as np
import pytest

import oracle
from oracle import paratime
from paper_2309_00768_amd import inputs

binding = pytest.importorskip("paper_2309_00768_amd.binding")


def factor(ev, theta, delta):
    c = delta if delta > 0 else 1j * (-delta)

    def level(z):
        w = (theta - z) / c
        s = np.sqrt(w * w - 1 + 0j)
        return np.maximum(np.abs(w + s), np.abs(w - s))
    return float((level(ev) / level(0.0)).max())


def spectra(cfg, blocks=("Fu", "CA")):
    ub, ab = inputs.state(cfg)
    plan = binding.Plan(cfg.n, cfg.nt, cfg.dt, cfg.mu, cfg.eta, cfg.mu0, ub, ab, precision="fp32")
    ref = oracle.system_from_config(cfg, ub, ab)
    st = paratime.SweepSteps(ref)
    out = {}
    for name, ivs, block in (("Fu", plan.cheb_intervals("Fu"), lambda k: ref.slabs[k].Fu),
                             ("CA", plan.cheb_intervals("CA"), lambda k: st.C0[k])):
        if name not in blocks:
            continue
        rows = []
        for k in range(cfg.nt):
            A = block(k)
            A = A.toarray() if hasattr(A, "toarray") else np.asarray(A)
            ev = np.linalg.eigvals(A / np.diag(A)[:, None])
            theta, delta = ivs[k]
            rows.append((theta, delta, factor(ev, theta, delta), float(np.abs(ev.imag).max())))
        out[name] = rows
    fu_k, ca_k = plan.solver_info()[2:]
    return out, {"Fu": fu_k, "CA": ca_k}


def test_uneven_batch_member_wave_blocks_get_contracting_ellipses():
    """Member 2 of the uneven batch (32 x 32 mesh, 16 slabs, dt = 1/16,
    Re = S = 300): eigenvalues of D^{-1} C_A,k up to 1.1 off the real axis.  The
    chosen ellipses (imaginary foci) contract every eigenvalue of every slab."""
    out, kap = spectra(inputs.batch_configs()[2], blocks=("CA",))
    rows = out["CA"]
    assert any(d <= 0.0 for _, d, _, _ in rows)
    worst = max(f for _, _, f, _ in rows)
    print(f"C_A: worst factor {worst:.3f}, model {model_factor(kap['CA']):.3f}")
    assert worst < 1.0


def model_factor(kappa):
    sk = np.sqrt(kappa)
    return (sk - 1.0) / (sk + 1.0)


def test_non_normal_blocks_get_contracting_ellipses():
    cfg = inputs.Config("nonnormal", 12, 4, 0.125, 1000.0, 1000.0)
    out, kap = spectra(cfg)
    assert any(d <= 0.0 for _, d, _, _ in out["Fu"]), "expected imaginary foci on F_u"
    for name, rows in out.items():
        r_model = model_factor(kap[name])
        for k, (theta, delta, f, im) in enumerate(rows):
            print(f"{name}_{k}: theta {theta:.3f} delta {delta:+.3f} factor {f:.3f} (model {r_model:.3f}, "
                  f"max |Im lambda| {im:.2f})")
            assert f < 1.0
            assert f <= r_model + 0.05


def test_normal_blocks_keep_real_intervals():
    out, kap = spectra(inputs.CONFIGS["cfg1"])
    for name, rows in out.items():
        for theta, delta, f, im in rows:
            assert delta > 0.0 and f < 1.0
