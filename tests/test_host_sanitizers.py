"""The host setup (assembly, AMG, Chebyshev intervals and ellipses, packing)
built on its own with g++ under AddressSanitizer and UndefinedBehaviorSanitizer
and run on two plans: a non-normal case whose F_u,k blocks take ellipses with
imaginary foci (12 x 12 mesh, 4 slabs, dt = 1/8, Re = S = 1000) and a normal
one (8 x 8, 4 slabs, Re = S = 100).  No sanitizer report, and the setup's
choices equal those of the library build."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2309_00768_amd import inputs

binding = pytest.importorskip("paper_2309_00768_amd.binding")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2309_00768_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <vector>
#include "st.h"
int main(int argc, char** argv) {
  int n, nt; double dt, mu;
  if (sscanf(argv[1], "%d", &n) != 1 || sscanf(argv[2], "%d", &nt) != 1 || sscanf(argv[3], "%lf", &dt) != 1 ||
      sscanf(argv[4], "%lf", &mu) != 1) return 2;
  const size_t nq2 = size_t(2 * n + 1) * (2 * n + 1), nq1 = size_t(n + 1) * (n + 1);
  std::vector<double> ub(size_t(nt) * 2 * nq2), ab(size_t(nt) * nq1);
  FILE* f = fopen(argv[5], "rb");
  if (!f || fread(ub.data(), sizeof(double), ub.size(), f) != ub.size()) return 3;
  fclose(f);
  f = fopen(argv[6], "rb");
  if (!f || fread(ab.data(), sizeof(double), ab.size(), f) != ab.size()) return 3;
  fclose(f);
  st_problem p{};
  p.n = n; p.nt = nt; p.dt = dt; p.mu = mu; p.eta = mu; p.mu0 = 1.0;
  p.ubar = ub.data(); p.abar = ab.data();
  st_plan* plan = nullptr;
  if (st_plan_create(&p, &plan) != 0) return 4;
  int fd, cd; double fk, ck;
  st_plan_solver_info(plan, &fd, &cd, &fk, &ck);
  std::vector<double> iu(2 * nt), ia(2 * nt);
  st_plan_cheb_intervals(plan, 0, iu.data());
  st_plan_cheb_intervals(plan, 1, ia.data());
  printf("%d %d %.17g %.17g\n", fd, cd, fk, ck);
  for (int k = 0; k < nt; ++k) printf("%.17g %.17g %.17g %.17g\n", iu[2 * k], iu[2 * k + 1], ia[2 * k], ia[2 * k + 1]);
  st_plan_destroy(plan);
  return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("sanitized")
    src = d / "driver.cpp"
    src.write_text(DRIVER)
    exe = d / "driver"
    host = [os.path.join(CSRC, f) for f in ("plan.cpp", "setup_amg.cpp", "setup_assemble.cpp", "setup_csr.cpp")]
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"), "-I", CSRC, str(src), *host,
                    "-o", str(exe), "-lpthread"], check=True, capture_output=True, timeout=600)
    return d, exe


@pytest.mark.parametrize("n,nt,dt,re", [(12, 4, 0.125, 1000.0), (8, 4, 0.1, 100.0)])
def test_host_setup_is_clean_under_sanitizers(driver, n, nt, dt, re):
    d, exe = driver
    cfg = inputs.Config("san", n, nt, dt, re, re)
    ub, ab = inputs.state(cfg)
    fu, fa = d / f"ub_{n}.bin", d / f"ab_{n}.bin"
    np.ascontiguousarray(ub, dtype=np.float64).tofile(fu)
    np.ascontiguousarray(ab, dtype=np.float64).tofile(fa)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    p = subprocess.run([str(exe), str(n), str(nt), repr(dt), repr(cfg.mu), str(fu), str(fa)], capture_output=True,
                       text=True, timeout=600, env=env)
    assert p.returncode == 0, p.stderr[-3000:]
    assert "runtime error" not in p.stderr and "AddressSanitizer" not in p.stderr, p.stderr[-3000:]
    lines = p.stdout.split("\n")
    fd, cd = (int(v) for v in lines[0].split()[:2])
    plan = binding.Plan(cfg.n, cfg.nt, cfg.dt, cfg.mu, cfg.eta, cfg.mu0, ub, ab, precision="fp32")
    assert (fd, cd) == tuple(plan.solver_info()[:2])
    got = np.array([[float(v) for v in ln.split()] for ln in lines[1:1 + nt]])
    want = np.column_stack([np.array(plan.cheb_intervals("Fu")), np.array(plan.cheb_intervals("CA"))])
    assert np.allclose(got, want, rtol=1e-12, atol=0.0)
