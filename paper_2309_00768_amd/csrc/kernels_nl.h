// Residual of the nonlinear space-time recurrence on the device.
//
// The backward-Euler finite-element recurrence, eq. (recurrence), for all
// slabs at once: for slab k (fields at t_k and the previous slab's u, A)
//   momentum:   M_u (u - u_prev)/dt + mu K_u u + B^T p + N_u(u, j, A) - f
//   continuity: B u                                   (B = -int psi div)
//   current:    M_j j + (1/mu0) K_jA A
//   induction:  M_A (A - A_prev)/dt + (eta/mu0) K_A A + N_A(u, A) + E
// with N_u the weak form of (u.grad) u + j grad A and N_A that of u.grad A; the
// imposed electric field enters with + because the recurrence carries -E on
// its right.  Every term is integrated over each element with 4 x 4 Gauss
// points (exact: the integrands are polynomials of degree <= 6 per direction
// on the affine squares), then each unknown's row sums the contributions of
// its elements in a fixed order (deterministic, no atomics).
//
// Fields are full nodal arrays (Q2 velocity on the (2n+1)^2 grid, Q1 p, j, A
// on the (n+1)^2 grid, lexicographic with x fastest) made of base values (which
// carry the boundary data) plus the unknowns x of the linear solver's
// slab-major layout [u_x | u_y | p | j | A] (interior u and A, all p and j).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace st {

constexpr int kNlLocal = 30;   // element residual entries: 9 u_x, 9 u_y, 4 p, 4 j, 4 A

struct NlArgs {
  int n, nt;
  double h, dt, mu, eta, mu0;
  const double* ub;   // base fields [nt][2][nq2], [nt][nq1] x3
  const double* pb;
  const double* jb;
  const double* ab;
  const double* u0;   // fields at t_0: [2][nq2], [nq1]
  const double* a0;
  const double* f;    // forcing [nt][2][nq2] (nullable)
  const double* e;    // electric field [nt][nq1] (nullable)
  const double* x;    // unknowns [nt][ns]
  double* elem;       // [nt][n*n][kNlLocal]
  double* r;          // residual rows [nt][ns]
};

// 4-point Gauss-Legendre on [0, 1].
__device__ inline double nl_gauss_s(int i) {
  const double a = 0.33998104358485626, b = 0.86113631159405258;
  const double g[4] = {-b, -a, a, b};
  return 0.5 * (1.0 + g[i]);
}
__device__ inline double nl_gauss_w(int i) {
  const double wa = 0.65214515486254614, wb = 0.34785484513745386;
  const double w[4] = {wb, wa, wa, wb};
  return 0.5 * w[i];
}

// Quadratic Lagrange basis on the nodes 0, 1/2, 1 and its derivative.
__device__ inline void nl_q2_1d(double s, double v[3], double d[3]) {
  v[0] = 2.0 * (s - 0.5) * (s - 1.0);
  v[1] = -4.0 * s * (s - 1.0);
  v[2] = 2.0 * s * (s - 0.5);
  d[0] = 4.0 * s - 3.0;
  d[1] = -8.0 * s + 4.0;
  d[2] = 4.0 * s - 1.0;
}

// Indices of the unknowns within a slab.
struct NlLayout {
  int n, g2, g1, nf2, nf1, ns;   // grids 2n+1 and n+1, interior counts, slab size
  int ou, op, oj, oa;            // offsets of u_x, p, j, A
  __device__ __host__ explicit NlLayout(int n_) : n(n_) {
    g2 = 2 * n + 1;
    g1 = n + 1;
    nf2 = (2 * n - 1) * (2 * n - 1);
    nf1 = (n - 1) * (n - 1);
    ou = 0;
    op = 2 * nf2;
    oj = op + g1 * g1;
    oa = oj + g1 * g1;
    ns = oa + nf1;
  }
  // interior index of Q2 node (I, J), or -1 on the boundary
  __device__ int free2(int I, int J) const {
    return (I > 0 && I < g2 - 1 && J > 0 && J < g2 - 1) ? (J - 1) * (g2 - 2) + (I - 1) : -1;
  }
  __device__ int free1(int I, int J) const {
    return (I > 0 && I < g1 - 1 && J > 0 && J < g1 - 1) ? (J - 1) * (g1 - 2) + (I - 1) : -1;
  }
};

// Element residual of element e of slab k (one thread each).
__global__ __launch_bounds__(256) void k_nl_element(NlArgs a) {
  const int ne = a.n * a.n;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(ne) * a.nt) return;
  const int k = int(t / ne), e = int(t - int64_t(k) * ne);
  const int ex = e % a.n, ey = e / a.n;
  const NlLayout L(a.n);
  const int nq2 = L.g2 * L.g2, nq1 = L.g1 * L.g1;
  const double* xk = a.x + int64_t(k) * L.ns;
  const double* xp = k > 0 ? a.x + int64_t(k - 1) * L.ns : nullptr;
  // local nodal values: Q2 node (ia, ib) -> ia + 3 ib; Q1 node (ia, ib) -> ia + 2 ib
  double ux[9], uy[9], vx[9], vy[9], fx[9], fy[9];
  for (int ib = 0; ib < 3; ++ib)
    for (int ia = 0; ia < 3; ++ia) {
      const int I = 2 * ex + ia, J = 2 * ey + ib, g = I + L.g2 * J, l = ia + 3 * ib;
      const int fi = L.free2(I, J);
      const double* bu = a.ub + int64_t(k) * 2 * nq2;
      ux[l] = bu[g] + (fi >= 0 ? xk[L.ou + fi] : 0.0);
      uy[l] = bu[nq2 + g] + (fi >= 0 ? xk[L.ou + L.nf2 + fi] : 0.0);
      if (k == 0) {
        vx[l] = a.u0[g];
        vy[l] = a.u0[nq2 + g];
      } else {
        const double* bp = a.ub + int64_t(k - 1) * 2 * nq2;
        vx[l] = bp[g] + (fi >= 0 ? xp[L.ou + fi] : 0.0);
        vy[l] = bp[nq2 + g] + (fi >= 0 ? xp[L.ou + L.nf2 + fi] : 0.0);
      }
      fx[l] = a.f ? a.f[int64_t(k) * 2 * nq2 + g] : 0.0;
      fy[l] = a.f ? a.f[int64_t(k) * 2 * nq2 + nq2 + g] : 0.0;
    }
  double pl[4], jl[4], Al[4], Bl[4], El[4];
  for (int ib = 0; ib < 2; ++ib)
    for (int ia = 0; ia < 2; ++ia) {
      const int I = ex + ia, J = ey + ib, g = I + L.g1 * J, l = ia + 2 * ib;
      const int fi = L.free1(I, J);
      pl[l] = a.pb[int64_t(k) * nq1 + g] + xk[L.op + g];
      jl[l] = a.jb[int64_t(k) * nq1 + g] + xk[L.oj + g];
      Al[l] = a.ab[int64_t(k) * nq1 + g] + (fi >= 0 ? xk[L.oa + fi] : 0.0);
      Bl[l] = k == 0 ? a.a0[g] : a.ab[int64_t(k - 1) * nq1 + g] + (fi >= 0 ? xp[L.oa + fi] : 0.0);
      El[l] = a.e ? a.e[int64_t(k) * nq1 + g] : 0.0;
    }
  double R[kNlLocal];
  for (int i = 0; i < kNlLocal; ++i) R[i] = 0.0;
  const double h = a.h, ih = 1.0 / h, idt = 1.0 / a.dt;
  for (int qy = 0; qy < 4; ++qy)
    for (int qx = 0; qx < 4; ++qx) {
      const double s = nl_gauss_s(qx), tt = nl_gauss_s(qy);
      const double W = nl_gauss_w(qx) * nl_gauss_w(qy) * h * h;
      double v2s[3], d2s[3], v2t[3], d2t[3];
      nl_q2_1d(s, v2s, d2s);
      nl_q2_1d(tt, v2t, d2t);
      const double v1s[2] = {1.0 - s, s}, d1s[2] = {-1.0, 1.0};
      const double v1t[2] = {1.0 - tt, tt}, d1t[2] = {-1.0, 1.0};
      double N2[9], N2x[9], N2y[9], N1[4], N1x[4], N1y[4];
      for (int ib = 0; ib < 3; ++ib)
        for (int ia = 0; ia < 3; ++ia) {
          const int l = ia + 3 * ib;
          N2[l] = v2s[ia] * v2t[ib];
          N2x[l] = d2s[ia] * v2t[ib] * ih;
          N2y[l] = v2s[ia] * d2t[ib] * ih;
        }
      for (int ib = 0; ib < 2; ++ib)
        for (int ia = 0; ia < 2; ++ia) {
          const int l = ia + 2 * ib;
          N1[l] = v1s[ia] * v1t[ib];
          N1x[l] = d1s[ia] * v1t[ib] * ih;
          N1y[l] = v1s[ia] * d1t[ib] * ih;
        }
      double Ux = 0, Uy = 0, Uxx = 0, Uxy = 0, Uyx = 0, Uyy = 0, Vx = 0, Vy = 0, Fx = 0, Fy = 0;
      for (int l = 0; l < 9; ++l) {
        Ux += ux[l] * N2[l];
        Uy += uy[l] * N2[l];
        Uxx += ux[l] * N2x[l];
        Uxy += ux[l] * N2y[l];
        Uyx += uy[l] * N2x[l];
        Uyy += uy[l] * N2y[l];
        Vx += vx[l] * N2[l];
        Vy += vy[l] * N2[l];
        Fx += fx[l] * N2[l];
        Fy += fy[l] * N2[l];
      }
      double P = 0, Jq = 0, Aq = 0, Ax = 0, Ay = 0, Bq = 0, Eq = 0;
      for (int l = 0; l < 4; ++l) {
        P += pl[l] * N1[l];
        Jq += jl[l] * N1[l];
        Aq += Al[l] * N1[l];
        Ax += Al[l] * N1x[l];
        Ay += Al[l] * N1y[l];
        Bq += Bl[l] * N1[l];
        Eq += El[l] * N1[l];
      }
      // momentum: test phi_m (Q2), both components
      const double cx = (Ux - Vx) * idt + Ux * Uxx + Uy * Uxy + Jq * Ax - Fx;
      const double cy = (Uy - Vy) * idt + Ux * Uyx + Uy * Uyy + Jq * Ay - Fy;
      for (int m = 0; m < 9; ++m) {
        R[m] += W * (N2[m] * cx + a.mu * (N2x[m] * Uxx + N2y[m] * Uxy) - N2x[m] * P);
        R[9 + m] += W * (N2[m] * cy + a.mu * (N2x[m] * Uyx + N2y[m] * Uyy) - N2y[m] * P);
      }
      const double dv = Uxx + Uyy;
      const double ca = (Aq - Bq) * idt + Ux * Ax + Uy * Ay + Eq;
      for (int m = 0; m < 4; ++m) {
        R[18 + m] += -W * N1[m] * dv;
        R[22 + m] += W * (N1[m] * Jq + (N1x[m] * Ax + N1y[m] * Ay) / a.mu0);
        R[26 + m] += W * (N1[m] * ca + (a.eta / a.mu0) * (N1x[m] * Ax + N1y[m] * Ay));
      }
    }
  double* out = a.elem + (int64_t(k) * ne + e) * kNlLocal;
  for (int i = 0; i < kNlLocal; ++i) out[i] = R[i];
}

// Row r of slab k: the sum of its elements' entries, elements in ascending
// order (one thread per unknown).
__global__ __launch_bounds__(256) void k_nl_gather(NlArgs a) {
  const NlLayout L(a.n);
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(L.ns) * a.nt) return;
  const int k = int(t / L.ns), row = int(t - int64_t(k) * L.ns);
  const int ne = a.n * a.n;
  const double* el = a.elem + int64_t(k) * ne * kNlLocal;
  double acc = 0.0;
  if (row < L.op) {
    // velocity: interior Q2 node, component c
    const int c = row < L.nf2 ? 0 : 1;
    const int fi = row - c * L.nf2;
    const int I = fi % (L.g2 - 2) + 1, J = fi / (L.g2 - 2) + 1;
    const int ey0 = max(0, (J - 1) / 2), ey1 = min(a.n - 1, J / 2);
    const int ex0 = max(0, (I - 1) / 2), ex1 = min(a.n - 1, I / 2);
    for (int ey = ey0; ey <= ey1; ++ey)
      for (int ex = ex0; ex <= ex1; ++ex) {
        const int ia = I - 2 * ex, ib = J - 2 * ey;
        if (ia < 0 || ia > 2 || ib < 0 || ib > 2) continue;
        acc += el[int64_t(ex + a.n * ey) * kNlLocal + 9 * c + ia + 3 * ib];
      }
  } else {
    // Q1 rows: p and j on every node, A on interior nodes
    int base, I, J;
    if (row < L.oa) {
      const int var = row < L.oj ? 0 : 1;
      const int g = row - (var == 0 ? L.op : L.oj);
      base = var == 0 ? 18 : 22;
      I = g % L.g1;
      J = g / L.g1;
    } else {
      const int fi = row - L.oa;
      base = 26;
      I = fi % (L.g1 - 2) + 1;
      J = fi / (L.g1 - 2) + 1;
    }
    for (int ey = max(0, J - 1); ey <= min(a.n - 1, J); ++ey)
      for (int ex = max(0, I - 1); ex <= min(a.n - 1, I); ++ex)
        acc += el[int64_t(ex + a.n * ey) * kNlLocal + base + (I - ex) + 2 * (J - ey)];
  }
  a.r[int64_t(k) * L.ns + row] = acc;
}

// Full nodal fields of base + x (u [nt][2][nq2], j and A [nt][nq1]): the
// linearisation state of the next Newton step.
struct NlStateArgs {
  int n, nt;
  const double* ub;
  const double* jb;
  const double* ab;
  const double* x;
  double* u;
  double* j;
  double* A;
};

__global__ __launch_bounds__(256) void k_nl_state(NlStateArgs a) {
  const NlLayout L(a.n);
  const int nq2 = L.g2 * L.g2, nq1 = L.g1 * L.g1;
  const int per = 2 * nq2 + 2 * nq1;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(per) * a.nt) return;
  const int k = int(t / per), i = int(t - int64_t(k) * per);
  const double* xk = a.x + int64_t(k) * L.ns;
  if (i < 2 * nq2) {
    const int c = i / nq2, g = i - c * nq2;
    const int fi = L.free2(g % L.g2, g / L.g2);
    a.u[int64_t(k) * 2 * nq2 + i] = a.ub[int64_t(k) * 2 * nq2 + i] + (fi >= 0 ? xk[L.ou + c * L.nf2 + fi] : 0.0);
  } else if (i < 2 * nq2 + nq1) {
    const int g = i - 2 * nq2;
    a.j[int64_t(k) * nq1 + g] = a.jb[int64_t(k) * nq1 + g] + xk[L.oj + g];
  } else {
    const int g = i - 2 * nq2 - nq1;
    const int fi = L.free1(g % L.g1, g / L.g1);
    a.A[int64_t(k) * nq1 + g] = a.ab[int64_t(k) * nq1 + g] + (fi >= 0 ? xk[L.oa + fi] : 0.0);
  }
}

// y = alpha x + beta y; with beta = 0, y is written without being read (it
// may hold anything, NaN included).
struct NlAxpbyArgs {
  const double* x;
  double* y;
  double alpha, beta;
  int64_t n;
};

__global__ __launch_bounds__(256) void k_nl_axpby(NlAxpbyArgs a) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < a.n; i += int64_t(gridDim.x) * blockDim.x)
    a.y[i] = a.beta != 0.0 ? a.alpha * a.x[i] + a.beta * a.y[i] : a.alpha * a.x[i];
}

struct NlNormArgs {
  const double* x;
  int64_t n;
  double* partial;   // [gridDim.x]
};

__global__ __launch_bounds__(256) void k_nl_norm_partial(NlNormArgs a) {
  __shared__ double s[256];
  double acc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < a.n; i += int64_t(gridDim.x) * blockDim.x)
    acc += a.x[i] * a.x[i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.partial[blockIdx.x] = s[0];
}

}  // namespace st
