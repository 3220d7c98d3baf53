// Host assembly of the single-slab blocks of the space-time Jacobian and of the
// preconditioner (paper: single-step Jacobian eq. (jacobianDiscrete), space-time
// blocks eqs. (STFu)/(STFA)/(lorentz)/(STother), PCD operator eq. (Fp), wave
// operator eqs. (CAspacetime)/(CAs)).
//
// Elements: Q2 (velocity) / Q1 (pressure, current, potential) on a uniform
// n x n mesh of the unit square; tensor 4-point Gauss quadrature, exact for all
// integrands here (degree <= 6 per coordinate).  Blocks that depend on the
// linearisation state carry one value array per slab on a shared pattern.
#include <algorithm>
#include <cmath>
#include <cstdio>

#include "st_internal.h"

namespace st {

Dims make_dims(int n, int nt) {
  Dims d;
  d.n = n;
  d.nt = nt;
  d.nq2 = (2 * n + 1) * (2 * n + 1);
  d.nq1 = (n + 1) * (n + 1);
  d.nf2 = (2 * n - 1) * (2 * n - 1);
  d.nf1 = (n - 1) * (n - 1);
  d.nu = 2 * d.nf2;
  d.np = d.nq1;
  d.nj = d.nq1;
  d.na = d.nf1;
  d.off[0] = 0;
  d.off[1] = d.nf2;
  d.off[2] = d.nu;
  d.off[3] = d.nu + d.np;
  d.off[4] = d.off[3] + d.nj;
  d.off[5] = d.off[4] + d.na;
  d.ns = d.off[5];
  return d;
}

namespace {

constexpr int NQ = 16;  // 4 x 4 Gauss points

struct Tab {
  double w[NQ];                         // reference weights (sum 1)
  double q2[9][NQ], q2s[9][NQ], q2t[9][NQ];
  double q1[4][NQ], q1s[4][NQ], q1t[4][NQ];
};

Tab make_tab() {
  // 4-point Gauss-Legendre on [-1, 1] mapped to [0, 1].
  const double g[4] = {-0.8611363115940526, -0.3399810435848563, 0.3399810435848563, 0.8611363115940526};
  const double gw[4] = {0.3478548451374538, 0.6521451548625461, 0.6521451548625461, 0.3478548451374538};
  Tab t{};
  for (int qy = 0; qy < 4; ++qy)
    for (int qx = 0; qx < 4; ++qx) {
      const int q = qx + 4 * qy;
      const double s = 0.5 * (g[qx] + 1.0), r = 0.5 * (g[qy] + 1.0);
      t.w[q] = 0.25 * gw[qx] * gw[qy];
      // quadratic Lagrange factors at 0, 1/2, 1
      const double Ls[3] = {(1 - s) * (1 - 2 * s), 4 * s * (1 - s), s * (2 * s - 1)};
      const double Lr[3] = {(1 - r) * (1 - 2 * r), 4 * r * (1 - r), r * (2 * r - 1)};
      const double dLs[3] = {4 * s - 3, 4 - 8 * s, 4 * s - 1};
      const double dLr[3] = {4 * r - 3, 4 - 8 * r, 4 * r - 1};
      for (int b = 0; b < 3; ++b)
        for (int a = 0; a < 3; ++a) {
          t.q2[a + 3 * b][q] = Ls[a] * Lr[b];
          t.q2s[a + 3 * b][q] = dLs[a] * Lr[b];
          t.q2t[a + 3 * b][q] = Ls[a] * dLr[b];
        }
      const double Ps[2] = {1 - s, s}, Pr[2] = {1 - r, r};
      const double dP[2] = {-1.0, 1.0};
      for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) {
          t.q1[a + 2 * b][q] = Ps[a] * Pr[b];
          t.q1s[a + 2 * b][q] = dP[a] * Pr[b];
          t.q1t[a + 2 * b][q] = Ps[a] * dP[b];
        }
    }
  return t;
}

// Node numbering helpers for element (ex, ey).
struct Mesh {
  int n;
  int q2(int ex, int ey, int l) const { return (2 * ex + l % 3) + (2 * n + 1) * (2 * ey + l / 3); }
  int q1(int ex, int ey, int l) const { return (ex + l % 2) + (n + 1) * (ey + l / 2); }
  int q2free(int ex, int ey, int l) const {
    const int I = 2 * ex + l % 3, J = 2 * ey + l / 3;
    if (I <= 0 || J <= 0 || I >= 2 * n || J >= 2 * n) return -1;
    return (J - 1) * (2 * n - 1) + (I - 1);
  }
  int q1free(int ex, int ey, int l) const {
    const int i = ex + l % 2, j = ey + l / 2;
    if (i <= 0 || j <= 0 || i >= n || j >= n) return -1;
    return (j - 1) * (n - 1) + (i - 1);
  }
};

// Element-to-CSR position maps for a block: pos[e][a][b] (or -1).
struct PosMap {
  int na = 0, nb = 0;
  std::vector<int64_t> pos;
  int64_t at(int e, int a, int b) const { return pos[(size_t(e) * na + a) * nb + b]; }
};

using RowFn = std::function<int(int ex, int ey, int l)>;

// Pattern of an element-coupled block: rows via rf (na local rows), cols via cf.
Csr pattern(int n, int nrows, int ncols, int na, const RowFn& rf, int nb, const RowFn& cf) {
  PatternBuilder pb(nrows, ncols);
  for (int ey = 0; ey < n; ++ey)
    for (int ex = 0; ex < n; ++ex)
      for (int a = 0; a < na; ++a) {
        const int r = rf(ex, ey, a);
        if (r < 0) continue;
        for (int b = 0; b < nb; ++b) {
          const int c = cf(ex, ey, b);
          if (c >= 0) pb.add(r, c);
        }
      }
  return pb.finish();
}

PosMap posmap(const Csr& m, int n, int na, const RowFn& rf, int nb, const RowFn& cf) {
  PosMap pm;
  pm.na = na;
  pm.nb = nb;
  pm.pos.assign(size_t(n) * n * na * nb, -1);
  for (int ey = 0; ey < n; ++ey)
    for (int ex = 0; ex < n; ++ex) {
      const int e = ex + n * ey;
      for (int a = 0; a < na; ++a) {
        const int r = rf(ex, ey, a);
        if (r < 0) continue;
        for (int b = 0; b < nb; ++b) {
          const int c = cf(ex, ey, b);
          if (c >= 0) pm.pos[(size_t(e) * na + a) * nb + b] = m.find(r, c);
        }
      }
    }
  return pm;
}

// Adds the element matrix loc[a][b] (row-major na x nb) into values v.
inline void scatter(const PosMap& pm, int e, const double* loc, double* v) {
  for (int a = 0; a < pm.na; ++a)
    for (int b = 0; b < pm.nb; ++b) {
      const int64_t p = pm.at(e, a, b);
      if (p >= 0) v[p] += loc[a * pm.nb + b];
    }
}

// Diagonal of a CSR (value set 0).
std::vector<double> diagonal(const Csr& a) {
  std::vector<double> d(a.nr, 0.0);
  for (int r = 0; r < a.nr; ++r) {
    const int64_t p = a.find(r, r);
    if (p >= 0) d[r] = a.v[p];
  }
  return d;
}

// Jacobi-preconditioned CG for the (SPD) current mass matrix, to rounding level.
void pcg_mass(const Csr& M, const std::vector<double>& dg, const double* b, double* x) {
  const int n = M.nr;
  std::vector<double> r(b, b + n), z(n), p(n), q(n);
  std::fill(x, x + n, 0.0);
  double bn = 0;
  for (int i = 0; i < n; ++i) bn += b[i] * b[i];
  bn = std::sqrt(bn);
  if (bn == 0.0) return;
  for (int i = 0; i < n; ++i) z[i] = r[i] / dg[i];
  p = z;
  double rz = 0;
  for (int i = 0; i < n; ++i) rz += r[i] * z[i];
  for (int it = 0; it < 500; ++it) {
    csr_spmv(M, p.data(), q.data());
    double pq = 0;
    for (int i = 0; i < n; ++i) pq += p[i] * q[i];
    const double al = rz / pq;
    double rn = 0;
    for (int i = 0; i < n; ++i) {
      x[i] += al * p[i];
      r[i] -= al * q[i];
      rn += r[i] * r[i];
    }
    if (std::sqrt(rn) <= 1e-16 * bn) break;
    for (int i = 0; i < n; ++i) z[i] = r[i] / dg[i];
    double rz2 = 0;
    for (int i = 0; i < n; ++i) rz2 += r[i] * z[i];
    const double be = rz2 / rz;
    rz = rz2;
    for (int i = 0; i < n; ++i) p[i] = z[i] + be * p[i];
  }
}

}  // namespace

int assemble_blocks(const st_problem& p, Blocks& B, std::string& err) {
  const int n = p.n, nt = p.nt;
  if (n < 2 || nt < 1 || !(p.dt > 0) || !(p.mu0 > 0) || !p.ubar || !p.abar) {
    err = "invalid problem (need n >= 2, nt >= 1, dt > 0, mu0 > 0, state arrays)";
    return ST_EINVAL;
  }
  B.d = make_dims(n, nt);
  B.dt = p.dt;
  B.mu = p.mu;
  B.eta = p.eta;
  B.mu0 = p.mu0;
  const Dims& d = B.d;
  const Tab T = make_tab();
  const Mesh m{n};
  const double h = 1.0 / n;
  const int nf2 = d.nf2;
  const int E = n * n;

  // Row/column maps of the blocks: velocity rows carry the component in l / 9.
  RowFn vel = [&](int ex, int ey, int l) {
    const int f = m.q2free(ex, ey, l % 9);
    return f < 0 ? -1 : f + (l / 9) * nf2;
  };
  RowFn q1all = [&](int ex, int ey, int l) { return m.q1(ex, ey, l); };
  RowFn q1fr = [&](int ex, int ey, int l) { return m.q1free(ex, ey, l); };
  // velocity map restricted to one component pair for the mass/stiffness pattern
  auto velc = [&](int c) -> RowFn {
    return [&, c](int ex, int ey, int l) {
      const int f = m.q2free(ex, ey, l);
      return f < 0 ? -1 : f + c * nf2;
    };
  };

  // ---------------------------------------------------------- patterns
  {
    PatternBuilder pb(d.nu, d.nu);
    for (int c = 0; c < 2; ++c) {
      Csr t = pattern(n, d.nu, d.nu, 9, velc(c), 9, velc(c));
      for (int r = 0; r < t.nr; ++r)
        for (int q = t.rp[r]; q < t.rp[r + 1]; ++q) pb.add(r, t.ci[q]);
    }
    B.Mu = pb.finish();
  }
  B.Ku = B.Mu;
  B.Fu = pattern(n, d.nu, d.nu, 18, vel, 18, vel);
  B.B = pattern(n, d.np, d.nu, 4, q1all, 18, vel);
  B.Zj = pattern(n, d.nu, d.nj, 18, vel, 4, q1all);
  B.ZA = pattern(n, d.nu, d.na, 18, vel, 4, q1fr);
  B.Mj = pattern(n, d.nj, d.nj, 4, q1all, 4, q1all);
  B.KjA = pattern(n, d.nj, d.na, 4, q1all, 4, q1fr);
  B.Y = pattern(n, d.na, d.nu, 4, q1fr, 18, vel);
  B.FA = pattern(n, d.na, d.na, 4, q1fr, 4, q1fr);
  B.MA = B.FA;
  B.KA = B.FA;
  B.Mp = B.Mj;
  B.Kp = B.Mj;
  B.Fp = B.Mj;

  // ------------------------------------------------- constant element matrices
  double M2[81] = {0}, K2[81] = {0}, M1[16] = {0}, K1[16] = {0}, Bx[4 * 9] = {0}, By[4 * 9] = {0};
  for (int q = 0; q < NQ; ++q) {
    const double w = T.w[q];
    for (int a = 0; a < 9; ++a)
      for (int b = 0; b < 9; ++b) {
        M2[a * 9 + b] += w * h * h * T.q2[a][q] * T.q2[b][q];
        K2[a * 9 + b] += w * (T.q2s[a][q] * T.q2s[b][q] + T.q2t[a][q] * T.q2t[b][q]);
      }
    for (int a = 0; a < 4; ++a) {
      for (int b = 0; b < 4; ++b) {
        M1[a * 4 + b] += w * h * h * T.q1[a][q] * T.q1[b][q];
        K1[a * 4 + b] += w * (T.q1s[a][q] * T.q1s[b][q] + T.q1t[a][q] * T.q1t[b][q]);
      }
      for (int b = 0; b < 9; ++b) {   // -int psi_a d_c phi_b
        Bx[a * 9 + b] -= w * h * T.q1[a][q] * T.q2s[b][q];
        By[a * 9 + b] -= w * h * T.q1[a][q] * T.q2t[b][q];
      }
    }
  }
  {
    PosMap pmu0 = posmap(B.Mu, n, 9, velc(0), 9, velc(0));
    PosMap pmu1 = posmap(B.Mu, n, 9, velc(1), 9, velc(1));
    std::vector<double> vm(B.Mu.nnz(), 0.0), vk(B.Mu.nnz(), 0.0);
    for (int e = 0; e < E; ++e) {
      scatter(pmu0, e, M2, vm.data());
      scatter(pmu1, e, M2, vm.data());
      scatter(pmu0, e, K2, vk.data());
      scatter(pmu1, e, K2, vk.data());
    }
    B.Mu.v = vm;
    B.Ku.v = vk;
    PosMap pb = posmap(B.B, n, 4, q1all, 18, vel);
    std::fill(B.B.v.begin(), B.B.v.end(), 0.0);
    double Bl[4 * 18];
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 9; ++b) {
        Bl[a * 18 + b] = Bx[a * 9 + b];
        Bl[a * 18 + 9 + b] = By[a * 9 + b];
      }
    for (int e = 0; e < E; ++e) scatter(pb, e, Bl, B.B.v.data());
    PosMap p1 = posmap(B.Mj, n, 4, q1all, 4, q1all);
    std::vector<double> mj(B.Mj.nnz(), 0.0), kp(B.Mj.nnz(), 0.0);
    for (int e = 0; e < E; ++e) {
      scatter(p1, e, M1, mj.data());
      scatter(p1, e, K1, kp.data());
    }
    B.Mj.v = mj;
    B.Mp.v = mj;
    B.Kp.v = kp;
    PosMap pka = posmap(B.KjA, n, 4, q1all, 4, q1fr);
    std::fill(B.KjA.v.begin(), B.KjA.v.end(), 0.0);
    double K1s[16];
    for (int i = 0; i < 16; ++i) K1s[i] = K1[i] / p.mu0;
    for (int e = 0; e < E; ++e) scatter(pka, e, K1s, B.KjA.v.data());
    PosMap pa = posmap(B.MA, n, 4, q1fr, 4, q1fr);
    std::vector<double> ma(B.MA.nnz(), 0.0), ka(B.MA.nnz(), 0.0);
    for (int e = 0; e < E; ++e) {
      scatter(pa, e, M1, ma.data());
      scatter(pa, e, K1, ka.data());
    }
    B.MA.v = ma;
    B.KA.v = ka;
  }
  B.Bt = csr_transpose(B.B);
  B.KjAt = csr_transpose(B.KjA);

  // ------------------------------------------------------- current state
  B.jbar.assign(size_t(nt) * d.nq1, 0.0);
  if (p.jbar) {
    std::copy(p.jbar, p.jbar + size_t(nt) * d.nq1, B.jbar.begin());
  } else {
    const std::vector<double> dg = diagonal(B.Mj);
    parallel_for(nt, host_threads(), [&](int k) {
      std::vector<double> rhs(d.nq1);
      csr_spmv(B.Kp, p.abar + size_t(k) * d.nq1, rhs.data());
      for (auto& x : rhs) x = -x / p.mu0;
      pcg_mass(B.Mj, dg, rhs.data(), B.jbar.data() + size_t(k) * d.nq1);
    });
  }

  // --------------------------------------------- state-dependent blocks
  const PosMap pFu = posmap(B.Fu, n, 18, vel, 18, vel);
  const PosMap pZj = posmap(B.Zj, n, 18, vel, 4, q1all);
  const PosMap pZA = posmap(B.ZA, n, 18, vel, 4, q1fr);
  const PosMap pY = posmap(B.Y, n, 4, q1fr, 18, vel);
  const PosMap pFA = posmap(B.FA, n, 4, q1fr, 4, q1fr);
  const PosMap pFp = posmap(B.Fp, n, 4, q1all, 4, q1all);
  const int64_t zFu = B.Fu.nnz(), zZj = B.Zj.nnz(), zZA = B.ZA.nnz(), zY = B.Y.nnz(),
                zFA = B.FA.nnz(), zFp = B.Fp.nnz();
  B.Fu.v.assign(size_t(nt) * zFu, 0.0);
  B.Zj.v.assign(size_t(nt) * zZj, 0.0);
  B.ZA.v.assign(size_t(nt) * zZA, 0.0);
  B.Y.v.assign(size_t(nt) * zY, 0.0);
  B.FA.v.assign(size_t(nt) * zFA, 0.0);
  B.Fp.v.assign(size_t(nt) * zFp, 0.0);
  B.bbar2.assign(nt, 0.0);
  // Constant parts of F_u, F_A, F_p on their patterns.
  const PosMap pFuc0 = posmap(B.Fu, n, 9, velc(0), 9, velc(0));
  const PosMap pFuc1 = posmap(B.Fu, n, 9, velc(1), 9, velc(1));
  const double dt = p.dt, mu = p.mu, eta = p.eta, mu0 = p.mu0;
  double Fu_c[81], FA_c[16], Fp_c[16];
  for (int i = 0; i < 81; ++i) Fu_c[i] = M2[i] / dt + mu * K2[i];
  for (int i = 0; i < 16; ++i) {
    FA_c[i] = M1[i] / dt + (eta / mu0) * K1[i];
    Fp_c[i] = M1[i] / dt + mu * K1[i];
  }

  parallel_for(nt, host_threads(), [&](int k) {
    const double* ux = p.ubar + size_t(k) * 2 * d.nq2;
    const double* uy = ux + d.nq2;
    const double* A = p.abar + size_t(k) * d.nq1;
    const double* J = B.jbar.data() + size_t(k) * d.nq1;
    double* vFu = B.Fu.v.data() + size_t(k) * zFu;
    double* vZj = B.Zj.v.data() + size_t(k) * zZj;
    double* vZA = B.ZA.v.data() + size_t(k) * zZA;
    double* vY = B.Y.v.data() + size_t(k) * zY;
    double* vFA = B.FA.v.data() + size_t(k) * zFA;
    double* vFp = B.Fp.v.data() + size_t(k) * zFp;
    double bx = 0.0, by = 0.0;
    double Le[18 * 18], Lzj[18 * 4], Lza[18 * 4], Ly[4 * 18], Lw1[16];
    for (int ey = 0; ey < n; ++ey)
      for (int ex = 0; ex < n; ++ex) {
        const int e = ex + n * ey;
        double nux[9], nuy[9], nA[4], nJ[4];
        for (int l = 0; l < 9; ++l) {
          nux[l] = ux[m.q2(ex, ey, l)];
          nuy[l] = uy[m.q2(ex, ey, l)];
        }
        for (int l = 0; l < 4; ++l) {
          nA[l] = A[m.q1(ex, ey, l)];
          nJ[l] = J[m.q1(ex, ey, l)];
        }
        std::fill(Le, Le + 18 * 18, 0.0);
        std::fill(Lzj, Lzj + 72, 0.0);
        std::fill(Lza, Lza + 72, 0.0);
        std::fill(Lw1, Lw1 + 16, 0.0);
        for (int q = 0; q < NQ; ++q) {
          // state at the quadrature point (physical derivatives = reference / h)
          double u0 = 0, u1 = 0, u0x = 0, u0y = 0, u1x = 0, u1y = 0;
          for (int l = 0; l < 9; ++l) {
            u0 += nux[l] * T.q2[l][q];
            u1 += nuy[l] * T.q2[l][q];
            u0x += nux[l] * T.q2s[l][q];
            u0y += nux[l] * T.q2t[l][q];
            u1x += nuy[l] * T.q2s[l][q];
            u1y += nuy[l] * T.q2t[l][q];
          }
          u0x /= h; u0y /= h; u1x /= h; u1y /= h;
          double ax = 0, ay = 0, jv = 0;
          for (int l = 0; l < 4; ++l) {
            ax += nA[l] * T.q1s[l][q];
            ay += nA[l] * T.q1t[l][q];
            jv += nJ[l] * T.q1[l][q];
          }
          ax /= h;
          ay /= h;
          const double W = T.w[q] * h * h;
          bx += W * ay;    // Bbar = mean of (dA/dy, -dA/dx)
          by -= W * ax;
          const double gu[2][2] = {{u0x, u0y}, {u1x, u1y}};  // gu[d][c] = d_c u_d
          for (int a = 0; a < 9; ++a) {
            const double Na = T.q2[a][q];
            for (int b = 0; b < 9; ++b) {
              const double Nb = T.q2[b][q];
              const double adv = (u0 * T.q2s[b][q] + u1 * T.q2t[b][q]) / h;  // ubar . grad phi_b
              const double w_adv = W * adv * Na;
              const double w_mm = W * Na * Nb;
              for (int dd = 0; dd < 2; ++dd)
                for (int cc = 0; cc < 2; ++cc) {
                  double v = w_mm * gu[dd][cc];            // Newton term (phi_b . grad) ubar
                  if (dd == cc) v += w_adv;                 // advection
                  Le[(dd * 9 + a) * 18 + cc * 9 + b] += v;
                }
            }
            for (int b = 0; b < 4; ++b) {
              const double chi = T.q1[b][q];
              const double chix = T.q1s[b][q] / h, chiy = T.q1t[b][q] / h;
              // Zj: int chi_b (grad A . phi_a);  ZA: int j (grad chi_b . phi_a)
              Lzj[a * 4 + b] += W * chi * ax * Na;
              Lzj[(9 + a) * 4 + b] += W * chi * ay * Na;
              Lza[a * 4 + b] += W * jv * chix * Na;
              Lza[(9 + a) * 4 + b] += W * jv * chiy * Na;
            }
          }
          for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b)
              Lw1[a * 4 + b] += W * (u0 * T.q1s[b][q] + u1 * T.q1t[b][q]) / h * T.q1[a][q];
        }
        // Y: int (phi_b . grad A) chi_a = Zj transposed element-wise
        for (int a = 0; a < 4; ++a)
          for (int b = 0; b < 18; ++b) Ly[a * 18 + b] = Lzj[b * 4 + a];
        scatter(pFu, e, Le, vFu);
        scatter(pFuc0, e, Fu_c, vFu);
        scatter(pFuc1, e, Fu_c, vFu);
        scatter(pZj, e, Lzj, vZj);
        scatter(pZA, e, Lza, vZA);
        scatter(pY, e, Ly, vY);
        double la[16], lp[16];
        for (int i = 0; i < 16; ++i) {
          la[i] = Lw1[i] + FA_c[i];
          lp[i] = Lw1[i] + Fp_c[i];
        }
        scatter(pFA, e, la, vFA);
        scatter(pFp, e, lp, vFp);
      }
    B.bbar2[k] = bx * bx + by * by;
  });
  return ST_OK;
}

namespace {
Csr slab_of(const Csr& a, int k) {
  Csr s;
  s.nr = a.nr;
  s.nc = a.nc;
  s.rp = a.rp;
  s.ci = a.ci;
  const int64_t z = a.nnz();
  s.v.assign(a.v.begin() + size_t(k) * z, a.v.begin() + size_t(k + 1) * z);
  return s;
}

bool same_pattern(const Csr& a, const Csr& b) { return a.rp == b.rp && a.ci == b.ci; }
}  // namespace

void form_wave_operator(Blocks& B) {
  // C0_k = F_Ak D^{-1} F_Ak + (|Bbar_k|^2/mu0) K_A
  // C1_k = M_A D^{-1} F_Ak + F_A(k+1) D^{-1} M_A      (block (k+1, k), factor -1/dt)
  // C2   = M_A D^{-1} M_A                             (block (k+2, k), factor +1/dt^2)
  const int nt = B.d.nt;
  std::vector<double> dinv = diagonal(B.MA);
  for (auto& x : dinv) x = 1.0 / x;
  Csr MAD = csr_scale_cols(B.MA, dinv);
  B.C2 = csr_matmul(MAD, B.MA);
  std::vector<Csr> c0(nt), c1(std::max(nt - 1, 0));
  parallel_for(nt, host_threads(), [&](int k) {
    Csr fa = slab_of(B.FA, k);
    Csr fad = csr_scale_cols(fa, dinv);
    c0[k] = csr_add(csr_matmul(fad, fa), 1.0, B.KA, B.bbar2[k] / B.mu0);
    if (k + 1 < nt) {
      Csr fa1 = slab_of(B.FA, k + 1);
      c1[k] = csr_add(csr_matmul(MAD, fa), 1.0, csr_matmul(csr_scale_cols(fa1, dinv), B.MA), 1.0);
    }
  });
  B.C0 = c0[0];
  const int64_t z0 = B.C0.nnz();
  B.C0.v.resize(size_t(nt) * z0);
  for (int k = 1; k < nt; ++k) {
    if (!same_pattern(c0[k], c0[0])) std::fprintf(stderr, "libst: C0 pattern mismatch\n");
    std::copy(c0[k].v.begin(), c0[k].v.end(), B.C0.v.begin() + size_t(k) * z0);
  }
  if (nt >= 2) {
    B.C1 = c1[0];
    const int64_t z1 = B.C1.nnz();
    B.C1.v.resize(size_t(nt - 1) * z1);
    for (int k = 1; k < nt - 1; ++k) std::copy(c1[k].v.begin(), c1[k].v.end(), B.C1.v.begin() + size_t(k) * z1);
  } else {
    B.C1 = B.C2;   // unused when nt == 1 (pattern only)
    std::fill(B.C1.v.begin(), B.C1.v.end(), 0.0);
  }
}

}  // namespace st
