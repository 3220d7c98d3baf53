// Host setup of the smoothed-aggregation AMG hierarchies for the spatial blocks
// of P_T (F_u,k, the wave blocks C_A,k, and the pressure Laplacian K_p) and the
// SELL-C-sigma packer that lays matrices out for the device.
//
// Aggregation is geometric: the blocks live on structured node grids, so
// aggregates are 3 x 3 node blocks per vector component (boundary remainders
// join the last aggregate of their row/column).  The tentative prolongator is
// the aggregate indicator (it preserves constants per component); it is
// smoothed once with damped Jacobi on a reference operator (value set 0,
// inter-component couplings dropped) to give P; R = P^T and A_c = R A P per
// value set (per slab for the state-dependent blocks).  The coarsest level is
// inverted densely.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "st_internal.h"

namespace st {

namespace {

constexpr int kCoarseMax = 160;

Csr set_of(const Csr& a, int s) {
  Csr c;
  c.nr = a.nr;
  c.nc = a.nc;
  c.rp = a.rp;
  c.ci = a.ci;
  const int64_t z = a.nnz();
  c.v.assign(a.v.begin() + size_t(s) * z, a.v.begin() + size_t(s + 1) * z);
  return c;
}

std::vector<double> diag_of(const Csr& a, int s) {
  std::vector<double> d(a.nr, 0.0);
  const int64_t z = a.nnz();
  for (int r = 0; r < a.nr; ++r) {
    const int64_t p = a.find(r, r);
    if (p >= 0) d[r] = a.v[size_t(s) * z + p];
  }
  return d;
}

// Largest |eigenvalue| of D^{-1} A (value set s) by power iteration.
double lambda_max(const Csr& a, int s, const std::vector<double>& dinv) {
  const int n = a.nr;
  std::vector<double> x(n), y(n);
  for (int i = 0; i < n; ++i) x[i] = 1.0 + 0.37 * std::sin(1.7 * i + 0.3);   // deterministic start
  const int64_t z = a.nnz();
  const double* v = a.v.data() + size_t(s) * z;
  double lam = 0.0;
  for (int it = 0; it < 30; ++it) {
    double nx = 0;
    for (double t : x) nx += t * t;
    nx = std::sqrt(nx);
    for (auto& t : x) t /= nx;
    double ny = 0;
    for (int r = 0; r < n; ++r) {
      double acc = 0;
      for (int p = a.rp[r]; p < a.rp[r + 1]; ++p) acc += v[p] * x[a.ci[p]];
      y[r] = acc * dinv[r];
      ny += y[r] * y[r];
    }
    lam = std::sqrt(ny);
    std::swap(x, y);
  }
  return lam;
}

// Dense inverse by Gauss-Jordan with partial pivoting; returns false if singular.
bool dense_inverse(std::vector<double>& a, int n) {
  std::vector<double> inv(size_t(n) * n, 0.0);
  for (int i = 0; i < n; ++i) inv[size_t(i) * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(a[size_t(r) * n + c]) > std::fabs(a[size_t(piv) * n + c])) piv = r;
    if (a[size_t(piv) * n + c] == 0.0) return false;
    if (piv != c)
      for (int j = 0; j < n; ++j) {
        std::swap(a[size_t(c) * n + j], a[size_t(piv) * n + j]);
        std::swap(inv[size_t(c) * n + j], inv[size_t(piv) * n + j]);
      }
    const double d = 1.0 / a[size_t(c) * n + c];
    for (int j = 0; j < n; ++j) {
      a[size_t(c) * n + j] *= d;
      inv[size_t(c) * n + j] *= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = a[size_t(r) * n + c];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        a[size_t(r) * n + j] -= f * a[size_t(c) * n + j];
        inv[size_t(r) * n + j] -= f * inv[size_t(c) * n + j];
      }
    }
  }
  a.swap(inv);
  return true;
}

template <class T>
Span put_converted(Image& img, const std::vector<double>& v, int fp32) {
  if (fp32) {
    std::vector<float> f(v.begin(), v.end());
    return img.put(f);
  }
  return img.put(v);
}

}  // namespace

// ---------------------------------------------------------------- SELL ---
int auto_lanes(double mean) {
  // Keep each lane's loop near 6-12 entries: long per-lane loops are latency-bound
  // on small matrices, where few waves are in flight.
  int l = 1;
  while (l < 16 && mean / (2 * l) >= 6.0) l *= 2;
  return l;
}

SellGroup pack_sell(Image& img, const std::vector<const Csr*>& mats, int fp32, int sigma, int lanes) {
  SellGroup g;
  g.nseg = int(mats.size());
  g.nrows = mats[0]->nr;
  g.ncols = mats[0]->nc;
  g.fp32 = fp32;
  const int nr = g.nrows;
  // Row order: descending total row length inside windows of `sigma` rows.
  std::vector<int> total(nr, 0);
  int64_t sum = 0;
  for (const Csr* m : mats)
    for (int r = 0; r < nr; ++r) {
      total[r] += m->rp[r + 1] - m->rp[r];
      sum += m->rp[r + 1] - m->rp[r];
    }
  if (lanes <= 0) lanes = auto_lanes(nr ? double(sum) / nr : 0.0);
  g.lanes = lanes;
  const int rps = kSlice / lanes;   // rows per slice
  g.nslices = (nr + rps - 1) / rps;
  std::vector<int> order(nr);
  std::iota(order.begin(), order.end(), 0);
  const int win = sigma <= 0 ? nr : sigma;
  for (int b = 0; b < nr; b += win) {
    const int e = std::min(nr, b + win);
    std::stable_sort(order.begin() + b, order.begin() + e, [&](int x, int y) { return total[x] > total[y]; });
  }
  std::vector<int> perm(size_t(g.nslices) * rps, -1);
  for (int i = 0; i < nr; ++i) perm[i] = order[i];
  g.perm = img.put(perm);
  for (int si = 0; si < g.nseg; ++si) {
    const Csr& m = *mats[si];
    SellSeg& s = g.seg[si];
    const int64_t z = m.nnz();
    s.nsets = z ? int(m.v.size() / z) : 1;
    if (s.nsets < 1) s.nsets = 1;
    std::vector<int> sptr(g.nslices + 1, 0);
    for (int sl = 0; sl < g.nslices; ++sl) {
      int w = 0;
      for (int q = 0; q < rps; ++q) {
        const int r = perm[size_t(sl) * rps + q];
        if (r >= 0) w = std::max(w, (m.rp[r + 1] - m.rp[r] + lanes - 1) / lanes);
      }
      sptr[sl + 1] = sptr[sl] + w * kSlice;
    }
    s.total = sptr[g.nslices];
    std::vector<int> col(s.total, 0);
    std::vector<double> val(size_t(s.nsets) * s.total, 0.0);
    for (int sl = 0; sl < g.nslices; ++sl)
      for (int q = 0; q < rps; ++q) {
        const int r = perm[size_t(sl) * rps + q];
        if (r < 0) continue;
        int j = 0;
        for (int p = m.rp[r]; p < m.rp[r + 1]; ++p, ++j) {
          const int64_t at = sptr[sl] + int64_t(j / lanes) * kSlice + q * lanes + (j % lanes);
          col[at] = m.ci[p];
          for (int st = 0; st < s.nsets; ++st) val[size_t(st) * s.total + at] = m.v[size_t(st) * z + p];
        }
      }
    s.sptr = img.put(sptr);
    s.col = img.put(col);
    s.val = fp32 ? put_converted<float>(img, val, 1) : img.put(val);
  }
  return g;
}

// ------------------------------------------------------------ stencils ---
bool pack_stencil(Image& img, const Csr& m, int nsets, int gx, int gy, int ncomp, bool diag_comp, int fp32,
                  StencilOp& out, int rad, int cgx, int cgy, int shift) {
  out = StencilOp();
  if (ncomp < 1 || ncomp > 2) return false;   // the kernels sum one or two column components
  out.gx = gx;
  out.gy = gy;
  out.ncomp = ncomp;
  out.diag_comp = diag_comp ? 1 : 0;
  out.nsets = nsets;
  out.rad = rad;
  out.cgx = cgx > 0 ? cgx : gx;
  out.cgy = cgy > 0 ? cgy : gy;
  out.shift = shift;
  const int w = 2 * rad + 1;
  out.nslot = diag_comp ? w * w : w * w * ncomp;
  out.fp32 = fp32;
  const int64_t per = int64_t(gx) * gy, cper = int64_t(out.cgx) * out.cgy;
  out.rows = per * ncomp;
  if (m.nr != out.rows || m.nc != cper * ncomp) return false;
  const int64_t z = m.nnz();
  const int msets = z ? int(m.v.size() / z) : 1;
  std::vector<double> coef(size_t(nsets) * out.nslot * out.rows, 0.0);
  for (int r = 0; r < m.nr; ++r) {
    const int c = int(r / per), i = int(r % per) % gx, j = int(r % per) / gx;
    for (int p = m.rp[r]; p < m.rp[r + 1]; ++p) {
      const int col = m.ci[p];
      const int cc = int(col / cper), ii = int(col % cper) % out.cgx, jj = int(col % cper) / out.cgx;
      const int dx = ii + shift - i, dy = jj + shift - j;
      if (dx < -rad || dx > rad || dy < -rad || dy > rad) return false;
      if (diag_comp && cc != c) return false;
      const int slot = (diag_comp ? 0 : cc * w * w) + (dy + rad) * w + (dx + rad);
      for (int s = 0; s < nsets; ++s)
        coef[(size_t(s) * out.nslot + slot) * out.rows + r] = m.v[size_t(msets == 1 ? 0 : s) * z + p];
    }
  }
  out.coef = fp32 ? put_converted<float>(img, coef, 1) : img.put(coef);
  return true;
}

// --------------------------------------------------- spectral interval ---
namespace {

// Bounds of the field of values of S = D^{-1/2} A D^{-1/2} (value set s), which
// is similar to D^{-1} A and so holds its eigenvalues: the extreme eigenvalues
// of H = (S + S^T)/2 bound their real parts, ||K|| with K = (S - S^T)/2 their
// imaginary parts.  Power iterations (the estimates approach from inside).
struct FovBox {
  double re_lo = 0.0, re_hi = 0.0, im = 0.0;
};

FovBox fov_box(const Csr& a, int s) {
  const int n = a.nr;
  const int64_t z = a.nnz();
  const double* v = a.v.data() + size_t(s) * z;
  std::vector<double> dh = diag_of(a, s);
  for (auto& t : dh) t = t != 0.0 ? 1.0 / std::sqrt(std::fabs(t)) : 0.0;
  std::vector<double> t1(n), su(n), st(n);
  // su = S x, st = S^T x
  auto apply_s = [&](const std::vector<double>& x) {
    for (int i = 0; i < n; ++i) t1[i] = dh[i] * x[i];
    std::fill(st.begin(), st.end(), 0.0);
    for (int r = 0; r < n; ++r) {
      double acc = 0.0;
      for (int p = a.rp[r]; p < a.rp[r + 1]; ++p) {
        acc += v[p] * t1[a.ci[p]];
        st[a.ci[p]] += v[p] * t1[r];
      }
      su[r] = dh[r] * acc;
    }
    for (int i = 0; i < n; ++i) st[i] *= dh[i];
  };
  // power iteration on x -> op(x); returns the last ||op(x)|| for unit x
  auto power = [&](auto&& op, double phase) {
    std::vector<double> x(n), y(n);
    for (int i = 0; i < n; ++i) x[i] = 1.0 + 0.31 * std::sin(1.3 * i + phase);
    double mu = 0.0;
    for (int it = 0; it < 40; ++it) {
      double nx = 0.0;
      for (double t : x) nx += t * t;
      nx = std::sqrt(nx);
      if (nx == 0.0) break;
      for (auto& t : x) t /= nx;
      op(x, y);
      double ny = 0.0;
      for (double t : y) ny += t * t;
      mu = std::sqrt(ny);
      std::swap(x, y);
    }
    return mu;
  };
  FovBox b;
  const double hmax = power([&](const std::vector<double>& x, std::vector<double>& y) {
    apply_s(x);
    for (int i = 0; i < n; ++i) y[i] = 0.5 * (su[i] + st[i]);
  }, 0.4);
  const double sig = 1.05 * hmax;
  const double mu = power([&](const std::vector<double>& x, std::vector<double>& y) {
    apply_s(x);
    for (int i = 0; i < n; ++i) y[i] = sig * x[i] - 0.5 * (su[i] + st[i]);
  }, 1.1);
  std::vector<double> kx(n);
  const double k2 = power([&](const std::vector<double>& x, std::vector<double>& y) {
    apply_s(x);
    for (int i = 0; i < n; ++i) kx[i] = 0.5 * (su[i] - st[i]);
    apply_s(kx);
    for (int i = 0; i < n; ++i) y[i] = -0.5 * (su[i] - st[i]);   // K^T K x = -K (K x)
  }, 2.3);
  b.re_hi = hmax;
  b.re_lo = sig - mu;
  b.im = std::sqrt(std::max(k2, 0.0));
  return b;
}

// ||r_d|| / ||r_0|| after d steps of the Chebyshev iteration (centre theta,
// foci theta -+ c, c = delta or i|delta| for delta <= 0) for A x = b from
// x = 0, value set s, with a fixed pseudo-random b: a direct test of whether
// the iteration contracts on the block's spectrum.
double cheb_residual_drop(const Csr& a, int s, const std::vector<double>& dinv, double theta, double delta,
                          int d) {
  const int n = a.nr;
  const int64_t z = a.nnz();
  const double* v = a.v.data() + size_t(s) * z;
  std::vector<double> r(n), dv(n);
  double r0 = 0.0;
  uint64_t state = 0x9e3779b97f4a7c15ull;   // LCG: rough, so that every mode has weight
  for (int i = 0; i < n; ++i) {
    state = state * 6364136223846793005ull + 1442695040888963407ull;
    r[i] = double(int64_t(state >> 11) - (int64_t(1) << 52)) / double(int64_t(1) << 52);
    r0 += r[i] * r[i];
    dv[i] = dinv[i] * r[i] / theta;
  }
  double ra = delta > 0.0 ? 1.0 / (theta / delta) : 1.0 / theta, rb = ra;
  auto residual_update = [&]() {
    for (int row = 0; row < n; ++row) {
      double acc = 0.0;
      for (int p = a.rp[row]; p < a.rp[row + 1]; ++p) acc += v[p] * dv[a.ci[p]];
      r[row] -= acc;
    }
  };
  for (int step = 1; step < d; ++step) {
    residual_update();
    ra = rb;
    double c1, c2;
    if (delta > 0.0) {
      rb = 1.0 / (2.0 * (theta / delta) - ra);
      c1 = rb * ra;
      c2 = 2.0 * rb / delta;
    } else {
      const double csq = -delta * delta;
      rb = 1.0 / (2.0 * theta - csq * ra);
      c1 = csq * rb * ra;
      c2 = 2.0 * rb;
    }
    for (int i = 0; i < n; ++i) dv[i] = c1 * dv[i] + c2 * dinv[i] * r[i];
  }
  residual_update();
  double rd = 0.0;
  for (double t : r) rd += t * t;
  return r0 > 0.0 ? std::sqrt(rd / r0) : 0.0;
}

}  // namespace

void estimate_interval(Image& img, const Csr& a, int nsets, Amg& out) {
  const int n = a.nr;
  out.cheb_alone.assign(size_t(nsets) * 2, 0.0);
  std::vector<double> kap(nsets, 0.0), lmins(nsets, 0.0), lmaxs(nsets, 0.0);
  const int64_t z = a.nnz();
  parallel_for(nsets, host_threads(), [&](int s) {
    std::vector<double> di = diag_of(a, s);
    for (auto& x : di) x = x != 0.0 ? 1.0 / x : 0.0;
    const double lmax = lambda_max(a, s, di);
    // Shifted power iteration on sigma I - D^{-1} A for the low end.
    const double sig = 1.05 * lmax;
    const double* v = a.v.data() + size_t(s) * z;
    std::vector<double> x(n), y(n);
    for (int i = 0; i < n; ++i) x[i] = 1.0 + 0.29 * std::cos(0.9 * i + 0.7);
    double mu = 0.0;
    for (int it = 0; it < 80; ++it) {
      double nx = 0;
      for (double t : x) nx += t * t;
      nx = std::sqrt(nx);
      for (auto& t : x) t /= nx;
      double ny = 0;
      for (int r = 0; r < n; ++r) {
        double acc = 0;
        for (int p = a.rp[r]; p < a.rp[r + 1]; ++p) acc += v[p] * x[a.ci[p]];
        y[r] = sig * x[r] - acc * di[r];
        ny += y[r] * y[r];
      }
      mu = std::sqrt(ny);
      std::swap(x, y);
    }
    double lmin = sig - mu;
    // Widen: the power estimates approach the extreme eigenvalues from inside.
    const double lo = std::max(0.7 * lmin, 1e-3 * lmax), hi = 1.1 * lmax;
    out.cheb_alone[2 * s] = 0.5 * (hi + lo);
    out.cheb_alone[2 * s + 1] = 0.5 * (hi - lo);
    kap[s] = hi / lo;
    lmins[s] = lmin;
    lmaxs[s] = lmax;
  });
  // A non-normal block (convection, the magnetic terms of C_A at high Re and
  // long steps) can have eigenvalues far off the real axis, where the
  // iteration on the real interval contracts slower than its condition
  // number says, or not at all.  That is tested directly: 80 Chebyshev steps
  // on a fixed pseudo-random right-hand side (a component that grows by 5% a
  // step is 50 times larger after them) measure the factor per step,
  // drop^(1/80).  If it exceeds the modelled (sqrt(kappa) - 1)/(sqrt(kappa) + 1)
  // by more than 0.05 (and the drop is above rounding), the ellipse with the
  // half-widths of the (widened) field-of-values box as semi-axes is tried:
  // a along the real axis, b along the imaginary one, foci theta -+ c with
  // c^2 = a^2 - b^2 of either sign, stored as delta = c, or -|c| for
  // imaginary foci.  The better of the two by the same test is kept, and
  // the degree choice uses the larger of its measured and modelled factors
  // ((a + b) / (theta + sqrt(theta^2 - c^2)) for the ellipse).  The state
  // changes smoothly from slab to slab, so five slabs spread over the
  // horizon are tested first, and every slab only if one of them fails.
  constexpr int kTestSteps = 80;
  auto kappa_of = [](double r) { return r < 1.0 ? std::pow((1.0 + r) / (1.0 - r), 2.0) : 1e30; };
  std::vector<int> fails(nsets, 0);
  auto check = [&](int s) {
    std::vector<double> di = diag_of(a, s);
    for (auto& x : di) x = x != 0.0 ? 1.0 / x : 0.0;
    const double th = out.cheb_alone[2 * s], de = out.cheb_alone[2 * s + 1];
    const double drop = cheb_residual_drop(a, s, di, th, de, kTestSteps);
    const double sk = std::sqrt(kap[s]), r_model = (sk - 1.0) / (sk + 1.0);
    const double r_int = std::pow(drop, 1.0 / kTestSteps);
    if (drop < 1e-10 || r_int <= r_model + 0.05) return;
    fails[s] = 1;
    kap[s] = std::max(kap[s], kappa_of(r_int));
    const FovBox box = fov_box(a, s);
    const double xl = std::min(box.re_lo, lmins[s]) * 0.9, xh = std::max(box.re_hi, lmaxs[s]) * 1.05;
    const double ct = 0.5 * (xl + xh), ea = 0.5 * (xh - xl), eb = 1.15 * box.im;
    const double csq = ea * ea - eb * eb;
    if (!(xl > 0.0 && ea < ct)) return;   // the ellipse would hold the origin
    const double r_ell_model = (ea + eb) / (ct + std::sqrt(ct * ct - csq));
    const double dl = csq > 0.0 ? std::sqrt(csq) : -std::sqrt(-csq);
    const double drop_ell = cheb_residual_drop(a, s, di, ct, dl, kTestSteps);
    if (r_ell_model < 1.0 && drop_ell < drop) {
      out.cheb_alone[2 * s] = ct;
      out.cheb_alone[2 * s + 1] = dl;
      kap[s] = kappa_of(std::max(r_ell_model, std::pow(drop_ell, 1.0 / kTestSteps)));
    }
  };
  std::vector<int> sample;
  for (int q = 0; q < 5; ++q) {
    const int s = int((int64_t(nsets - 1) * q) / 4);
    if (sample.empty() || sample.back() != s) sample.push_back(s);
  }
  parallel_for(int(sample.size()), host_threads(), [&](int i) { check(sample[i]); });
  bool any = false;
  for (int s : sample) any = any || fails[s];
  if (any) {
    std::vector<int> rest;
    for (int s = 0; s < nsets; ++s)
      if (std::find(sample.begin(), sample.end(), s) == sample.end()) rest.push_back(s);
    parallel_for(int(rest.size()), host_threads(), [&](int i) { check(rest[i]); });
  }
  out.kappa = *std::max_element(kap.begin(), kap.end());
  out.cheb_alone_span = img.put(out.cheb_alone);
}

// ----------------------------------------------------------------- AMG ---
int build_amg(Image& img, const Csr& a0, int nsets, Grid2 grid, int fp32, int cheb_degree,
              int sigma, bool singular, Amg& out, std::string& err) {
  out = Amg();
  out.nsets = nsets;
  out.fp32 = fp32;
  out.cheb_degree = cheb_degree;
  out.singular = singular ? 1 : 0;
  Csr A = a0;   // current level, nsets value sets
  Grid2 g = grid;
  const int threads = host_threads();
  for (int level = 0;; ++level) {
    const int n = A.nr;
    AmgLevel L;
    L.nrows = n;
    const int64_t z = A.nnz();
    // Jacobi diagonals and Chebyshev intervals per value set.
    std::vector<double> dinv(size_t(nsets) * n), cheb(size_t(nsets) * 2);
    parallel_for(nsets, threads, [&](int s) {
      std::vector<double> d = diag_of(A, s);
      std::vector<double> di(n);
      for (int i = 0; i < n; ++i) di[i] = d[i] != 0.0 ? 1.0 / d[i] : 0.0;
      std::copy(di.begin(), di.end(), dinv.begin() + size_t(s) * n);
      const double lm = lambda_max(A, s, di);
      const double hi = 1.1 * lm, lo = hi / 10.0;
      cheb[2 * s] = 0.5 * (hi + lo);
      cheb[2 * s + 1] = 0.5 * (hi - lo);
    });
    L.A = pack_sell(img, {&A}, fp32, sigma);
    L.dinv = fp32 ? put_converted<float>(img, dinv, 1) : img.put(dinv);
    L.cheb = img.put(cheb);
    const int ax = std::max(1, g.gx / 3), ay = std::max(1, g.gy / 3);
    const int nagg = ax * ay * g.ncomp;
    const bool last = n <= kCoarseMax || nagg >= n || (ax == 1 && ay == 1);
    if (last) {
      out.lev.push_back(L);
      out.ncoarse = n;
      std::vector<double> inv(size_t(nsets) * n * n);
      bool ok = true;
      parallel_for(nsets, threads, [&](int s) {
        std::vector<double> dense(size_t(n) * n, 0.0);
        for (int r = 0; r < n; ++r)
          for (int p = A.rp[r]; p < A.rp[r + 1]; ++p) dense[size_t(r) * n + A.ci[p]] = A.v[size_t(s) * z + p];
        if (singular) {   // constant null vector: invert A + alpha 1 1^T
          double md = 0;
          for (int r = 0; r < n; ++r) md += dense[size_t(r) * n + r];
          const double alpha = md / n / n;
          for (auto& x : dense) x += alpha;
        }
        if (!dense_inverse(dense, n)) ok = false;
        // stored column-major: inv[s][j][i] = Ainv(i, j) (coalesced reads on the device)
        for (int i = 0; i < n; ++i)
          for (int j = 0; j < n; ++j) inv[size_t(s) * n * n + size_t(j) * n + i] = dense[size_t(i) * n + j];
      });
      if (!ok) {
        err = "singular coarsest AMG matrix";
        return ST_EINTERNAL;
      }
      out.coarse_inv = fp32 ? put_converted<float>(img, inv, 1) : img.put(inv);
      break;
    }
    // Aggregates: 3x3 node blocks per component.
    std::vector<int> agg(n);
    for (int c = 0; c < g.ncomp; ++c)
      for (int j = 0; j < g.gy; ++j)
        for (int i = 0; i < g.gx; ++i) {
          const int node = c * g.gx * g.gy + j * g.gx + i;
          agg[node] = c * ax * ay + std::min(j / 3, ay - 1) * ax + std::min(i / 3, ax - 1);
        }
    // Reference operator: value set 0 with inter-component entries dropped.
    const int per = g.gx * g.gy;
    std::vector<double> dref(n, 0.0);
    Csr Aref;
    Aref.nr = n;
    Aref.nc = n;
    Aref.rp.assign(n + 1, 0);
    for (int r = 0; r < n; ++r) {
      for (int p = A.rp[r]; p < A.rp[r + 1]; ++p)
        if (A.ci[p] / per == r / per) {
          Aref.ci.push_back(A.ci[p]);
          Aref.v.push_back(A.v[p]);
          if (A.ci[p] == r) dref[r] = A.v[p];
        }
      Aref.rp[r + 1] = int(Aref.ci.size());
    }
    std::vector<double> drefinv(n);
    for (int i = 0; i < n; ++i) drefinv[i] = dref[i] != 0.0 ? 1.0 / dref[i] : 0.0;
    const double omega = 4.0 / (3.0 * lambda_max(Aref, 0, drefinv));
    // P = (I - omega D^{-1} Aref) P_tent
    Csr Pt;
    Pt.nr = n;
    Pt.nc = nagg;
    Pt.rp.resize(n + 1);
    Pt.ci.resize(n);
    Pt.v.assign(n, 1.0);
    for (int i = 0; i <= n; ++i) Pt.rp[i] = i;
    for (int i = 0; i < n; ++i) Pt.ci[i] = agg[i];
    Csr DA = Aref;
    for (int r = 0; r < n; ++r)
      for (int p = DA.rp[r]; p < DA.rp[r + 1]; ++p) DA.v[p] *= omega * drefinv[r];
    Csr P = csr_add(Pt, 1.0, csr_matmul(DA, Pt), -1.0);
    Csr R = csr_transpose(P);
    L.P = pack_sell(img, {&P}, fp32, sigma);
    L.R = pack_sell(img, {&R}, fp32, sigma);
    out.lev.push_back(L);
    // Galerkin coarse operators per value set on a common pattern.
    std::vector<Csr> coarse(nsets);
    parallel_for(nsets, threads, [&](int s) {
      Csr As = set_of(A, s);
      coarse[s] = csr_matmul(R, csr_matmul(As, P));
    });
    Csr Ac = coarse[0];
    const int64_t zc = Ac.nnz();
    Ac.v.resize(size_t(nsets) * zc);
    for (int s = 1; s < nsets; ++s) {
      if (coarse[s].rp != coarse[0].rp || coarse[s].ci != coarse[0].ci) {
        err = "coarse pattern differs between value sets";
        return ST_EINTERNAL;
      }
      std::copy(coarse[s].v.begin(), coarse[s].v.end(), Ac.v.begin() + size_t(s) * zc);
    }
    A = std::move(Ac);
    g = Grid2{ax, ay, g.ncomp};
  }
  return ST_OK;
}

}  // namespace st
