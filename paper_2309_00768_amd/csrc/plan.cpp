// st_plan_*: the host-side setup of libst.  Assembles the blocks, forms the wave
// operator, builds the fused rows of J and J^T (paper, eq. (jacobianSTDiscrete)),
// the pieces of P_T (eq. (PT)) and the AMG hierarchies, and packs everything
// into a device image that st_create() uploads in one copy.
#include <algorithm>
#include <functional>
#include <cmath>
#include <cstdio>
#include <new>

#include "st_internal.h"

struct st_plan {
  st::Plan p;
};

namespace st {

namespace {

struct Piece {
  const Csr* m;
  int roff, coff;
  double scale;
};

// Rows [0, nr) built from blocks placed at (roff, coff); each block has 1 or
// `nsets` value sets (1 = broadcast to every set).
Csr fuse(int nr, int nc, int nsets, std::vector<Piece> pieces) {
  std::sort(pieces.begin(), pieces.end(), [](const Piece& a, const Piece& b) { return a.coff < b.coff; });
  Csr f;
  f.nr = nr;
  f.nc = nc;
  f.rp.assign(nr + 1, 0);
  for (int r = 0; r < nr; ++r) {
    int cnt = 0;
    for (const Piece& pc : pieces) {
      const int lr = r - pc.roff;
      if (lr >= 0 && lr < pc.m->nr) cnt += pc.m->rp[lr + 1] - pc.m->rp[lr];
    }
    f.rp[r + 1] = f.rp[r] + cnt;
  }
  const int64_t z = f.rp[nr];
  f.ci.resize(z);
  f.v.assign(size_t(nsets) * z, 0.0);
  for (int r = 0; r < nr; ++r) {
    int64_t q = f.rp[r];
    for (const Piece& pc : pieces) {
      const int lr = r - pc.roff;
      if (lr < 0 || lr >= pc.m->nr) continue;
      const int64_t zm = pc.m->nnz();
      const int msets = zm ? int(pc.m->v.size() / zm) : 1;
      for (int p = pc.m->rp[lr]; p < pc.m->rp[lr + 1]; ++p, ++q) {
        f.ci[q] = pc.m->ci[p] + pc.coff;
        for (int s = 0; s < nsets; ++s)
          f.v[size_t(s) * z + q] = pc.scale * pc.m->v[size_t(msets == 1 ? 0 : s) * zm + p];
      }
    }
  }
  return f;
}

Csr empty_rows(int nr, int nc) {
  Csr e;
  e.nr = nr;
  e.nc = nc;
  e.rp.assign(nr + 1, 0);
  return e;
}

template <class T>
Span put_diag_inv(Image& img, const Csr& a, int fp32) {
  std::vector<double> d(a.nr, 0.0);
  for (int r = 0; r < a.nr; ++r) {
    const int64_t p = a.find(r, r);
    d[r] = p >= 0 && a.v[p] != 0.0 ? 1.0 / a.v[p] : 0.0;
  }
  if (fp32) {
    std::vector<float> f(d.begin(), d.end());
    return img.put(f);
  }
  return img.put(d);
}

}  // namespace

// sum_t coef_t * m_t(value set set_t(k)) for every output set k on the union
// pattern; set_t(k) < 0 leaves term t out of set k.
struct SetTerm {
  const Csr* m;
  double coef;
  std::function<int(int)> set;
};

static Csr combine_sets(int nsets, const std::vector<SetTerm>& terms) {
  const int nr = terms[0].m->nr, nc = terms[0].m->nc;
  PatternBuilder pb(nr, nc);
  for (const SetTerm& t : terms)
    for (int r = 0; r < nr; ++r)
      for (int p = t.m->rp[r]; p < t.m->rp[r + 1]; ++p) pb.add(r, t.m->ci[p]);
  Csr out = pb.finish();
  const int64_t z = out.nnz();
  out.v.assign(size_t(nsets) * size_t(z), 0.0);
  for (const SetTerm& t : terms) {
    const int64_t tz = t.m->nnz();
    parallel_for(nsets, host_threads(), [&](int k) {
      const int s = t.set(k);
      if (s < 0) return;
      const double* src = t.m->v.data() + size_t(s) * size_t(tz);
      double* dst = out.v.data() + size_t(k) * size_t(z);
      for (int r = 0; r < nr; ++r)
        for (int p = t.m->rp[r]; p < t.m->rp[r + 1]; ++p) dst[out.find(r, t.m->ci[p])] += t.coef * src[p];
    });
  }
  return out;
}

WsLayout workspace_layout(const Plan& P) {
  WsLayout L;
  const Dims& d = P.blk.d;
  size_t cur = (P.image_bytes + 255) & ~size_t(255);
  auto take = [&](size_t bytes) {
    const size_t off = cur;
    cur = (cur + bytes + 255) & ~size_t(255);
    return off;
  };
  const size_t N = size_t(d.nt) * d.ns;
  const int m = P.max_restart;
  const size_t ts = P.fp32 ? 4 : 8;
  L.V = take(8 * N * (m + 1));
  L.Z = take(8 * N * m);
  L.w = take(8 * N);
  L.r = take(8 * N);
  L.hess = take(8 * size_t(m + 1) * (m + 1));
  // small: 64 scalars, g, cs, sn, y (m + 2 each), then the 2m dot products of
  // the Arnoldi step with delayed reorthogonalisation
  L.small = take(8 * 64 + 8 * 4 * size_t(m + 2) + 8 * 2 * size_t(m + 1));
  L.partial = take(8 * size_t(kPartialBlocks) * (2 * size_t(m) + 2));
  L.psum = take(8 * size_t(d.nt) * 2);
  L.pt_begin = L.psum;
  const size_t nt = d.nt;
  L.ru = take(ts * nt * d.nu);
  L.yu = take(ts * nt * d.nu);
  L.xu = take(ts * nt * d.nu);
  L.rp = take(ts * nt * d.np);
  L.q = take(ts * nt * d.np);
  L.t = take(ts * nt * d.np);
  L.xp = take(ts * nt * d.np);
  L.rj = take(ts * nt * d.nj);
  L.yj = take(ts * nt * d.nj);
  L.ra = take(ts * nt * d.na);
  L.wA = take(ts * nt * d.na);
  L.sA = take(ts * nt * d.na);
  L.yA = take(ts * nt * d.na);
  const size_t mm = std::max(d.np, std::max(d.nj, d.na));
  L.mr = take(ts * nt * mm);
  L.md0 = take(ts * nt * mm);
  L.md1 = take(ts * nt * mm);
  L.chr = take(ts * mm);
  L.chd0 = take(ts * mm);
  L.chd1 = take(ts * mm);
  L.mr2 = take(ts * nt * mm);
  L.md02 = take(ts * nt * mm);
  L.md12 = take(ts * nt * mm);
  L.io = take(2 * sizeof(void*));
  if (P.pint > 0)
    for (int i = 0; i < 6; ++i) {
      L.pint_u[i] = take(ts * nt * d.nu);
      L.pint_a[i] = take(ts * nt * d.na);
    }
  for (const AmgLevel& lv : P.amgKp.lev)
    for (int i = 0; i < 6; ++i) L.kp_lev.push_back(take(ts * nt * lv.nrows));
  for (const AmgLevel& lv : P.amgFu.lev)
    for (int i = 0; i < 6; ++i) L.fu_lev.push_back(take(ts * lv.nrows));
  for (const AmgLevel& lv : P.amgC0.lev)
    for (int i = 0; i < 6; ++i) L.ca_lev.push_back(take(ts * lv.nrows));
  L.end = cur;
  return L;
}

static int build_plan(Plan& P, std::string& err) {
  const st_problem& pr = P.prob;
  if (pr.j_slabs != 0 && pr.j_slabs != 1 && pr.j_slabs != 4 && pr.j_slabs != 8) {
    err = "j_slabs must be 0, 1, 4 or 8";
    return ST_EINVAL;
  }
  if (pr.sweep_fuse != 0 && pr.sweep_fuse != 1) {
    err = "sweep_fuse must be 0 or 1";
    return ST_EINVAL;
  }
  if (pr.precond_variant < 0 || pr.precond_variant > 2) {
    err = "precond_variant must be 0 (P_T), 1 (P-tilde) or 2 (P)";
    return ST_EINVAL;
  }
  if (pr.precond_variant != 0 && pr.adjoint) {
    err = "the transposed preconditioner exists for P_T only (precond_variant 0)";
    return ST_EINVAL;
  }
  if (pr.sweep_lanes < 0 || pr.sweep_lanes > 2) {
    err = "sweep_lanes must be 0, 1 or 2";
    return ST_EINVAL;
  }
  if (pr.autotune != 0 && pr.autotune != 1) {
    err = "autotune must be 0 or 1";
    return ST_EINVAL;
  }
  if (pr.time_parallel < 0 || pr.time_coarse_degree < 0) {
    err = "time_parallel and time_coarse_degree must be >= 0";
    return ST_EINVAL;
  }
  if (pr.time_parallel > 0 && (pr.adjoint || pr.precond_variant != 0 || pr.sweep_format != 0)) {
    err = "time_parallel needs P_T (precond_variant 0), no adjoint and the stencil sweeps (sweep_format 0)";
    return ST_EINVAL;
  }
  int rc = assemble_blocks(pr, P.blk, err);
  if (rc) return rc;
  form_wave_operator(P.blk);
  Blocks& b = P.blk;
  const Dims& d = b.d;
  const int nt = d.nt;
  const int sigma = pr.sell_sigma;
  P.fp32 = pr.precond_precision == ST_FP32 ? 1 : 0;
  P.exact = pr.inner_mode == ST_INNER_EXACT ? 1 : 0;
  P.inner_iters = pr.inner_iters > 0 ? pr.inner_iters : 40;
  P.mass_iters = pr.mass_iters > 0 ? pr.mass_iters : (P.exact ? 60 : 6);
  P.max_restart = pr.max_restart > 0 ? pr.max_restart : 30;
  const int cheb = pr.cheb_degree > 0 ? pr.cheb_degree : 3;
  const int fp = P.fp32;
  Image& img = P.img;

  // ---------------------------------------------------------- J (FP64)
  // Rows [u | p | j | A]; columns of the same slab (segments 0, 1) or of the
  // previous slab (segment 2).
  const int o2 = d.off[2], o3 = d.off[3], o4 = d.off[4], ns = d.ns;
  {
    Csr S = fuse(ns, ns, nt, {{&b.Fu, 0, 0, 1.0}, {&b.Zj, 0, o3, 1.0}, {&b.ZA, 0, o4, 1.0},
                              {&b.Y, o4, 0, 1.0}, {&b.FA, o4, o4, 1.0}});
    Csr C = fuse(ns, ns, 1, {{&b.Bt, 0, o2, 1.0}, {&b.B, o2, 0, 1.0}, {&b.Mj, o3, o3, 1.0},
                             {&b.KjA, o3, o4, 1.0}});
    Csr Pv = fuse(ns, ns, 1, {{&b.Mu, 0, 0, -1.0 / b.dt}, {&b.MA, o4, o4, -1.0 / b.dt}});
    // J is bandwidth bound and large: one lane per row unless asked otherwise.
    P.J = pack_sell(img, {&S, &C, &Pv}, 0, sigma, pr.j_lanes > 0 ? pr.j_lanes : 1);
  }
  if (pr.adjoint) {
    Csr FuT = csr_transpose(b.Fu), YT = csr_transpose(b.Y), ZjT = csr_transpose(b.Zj),
        ZAT = csr_transpose(b.ZA), FAT = csr_transpose(b.FA);
    Csr S = fuse(ns, ns, nt, {{&FuT, 0, 0, 1.0}, {&YT, 0, o4, 1.0}, {&ZjT, o3, 0, 1.0},
                              {&ZAT, o4, 0, 1.0}, {&FAT, o4, o4, 1.0}});
    Csr C = fuse(ns, ns, 1, {{&b.Bt, 0, o2, 1.0}, {&b.B, o2, 0, 1.0}, {&b.Mj, o3, o3, 1.0},
                             {&b.KjAt, o4, o3, 1.0}});
    Csr Pv = fuse(ns, ns, 1, {{&b.Mu, 0, 0, -1.0 / b.dt}, {&b.MA, o4, o4, -1.0 / b.dt}});
    P.JT = pack_sell(img, {&S, &C, &Pv}, 0, sigma, pr.j_lanes > 0 ? pr.j_lanes : 1);
  }

  {
    Csr MAd = b.MA;
    for (auto& v : MAd.v) v /= b.dt;
    P.MA64 = pack_sell(img, {&MAd}, 0, sigma);
  }
  // ------------------------------------------------------- P_T pieces
  P.MA = pack_sell(img, {&b.MA}, fp, sigma);
  P.dMA = put_diag_inv<double>(img, b.MA, fp);
  P.Mj = pack_sell(img, {&b.Mj}, fp, sigma);
  P.dMj = put_diag_inv<double>(img, b.Mj, fp);
  P.Mp = P.Mj;                 // M_p and M_j are the same Q1 mass matrix
  P.dMp = P.dMj;
  {
    // bidiagonal applies: segment 0 = diagonal block (per slab), segment 1 = mass (previous slab)
    Csr MAs = b.MA, Mps = b.Mp;
    for (auto& v : MAs.v) v *= -1.0 / b.dt;
    for (auto& v : Mps.v) v *= -1.0 / b.dt;
    P.FA = pack_sell(img, {&b.FA, &MAs}, fp, sigma);
    P.Fp = pack_sell(img, {&b.Fp, &Mps}, fp, sigma);
    if (pr.adjoint) {
      Csr FAT = csr_transpose(b.FA), FpT = csr_transpose(b.Fp);
      P.FAt = pack_sell(img, {&FAT, &MAs}, fp, sigma);
      P.Fpt = pack_sell(img, {&FpT, &Mps}, fp, sigma);
    }
  }
  P.KjA = pack_sell(img, {&b.KjA}, fp, sigma);
  P.Bt = pack_sell(img, {&b.Bt}, fp, sigma);
  // y_u = r_u - Zj y_j - ZA y_A + B^T (-x_p): three segments over the velocity rows
  P.Zj = pack_sell(img, {&b.Zj, &b.ZA, &b.Bt}, fp, sigma);
  P.Mu = pack_sell(img, {&b.Mu}, fp, sigma);
  {
    // C_A sweep couplings: rhs = s^k + (1/dt) C1_{k-1} y^{k-1} - (1/dt^2) C2 y^{k-2}
    P.C1 = pack_sell(img, {&b.C1, &b.C2}, fp, sigma);
  }
  P.variant = pr.precond_variant;
  if (P.variant >= 1) P.Bv = pack_sell(img, {&b.B}, fp, sigma);
  if (P.variant == 2) P.Yv = pack_sell(img, {&b.Y}, fp, sigma);
  if (pr.adjoint) {
    P.KjAt = pack_sell(img, {&b.KjAt}, fp, sigma);
    P.B = pack_sell(img, {&b.B}, fp, sigma);
    Csr ZjT = csr_transpose(b.Zj), ZAT = csr_transpose(b.ZA);
    P.Zjt = pack_sell(img, {&ZjT}, fp, sigma);
    P.ZAt = pack_sell(img, {&ZAT}, fp, sigma);
    Csr C1T = csr_transpose(b.C1), C2T = csr_transpose(b.C2);
    P.C1t = pack_sell(img, {&C1T, &C2T}, fp, sigma);
  }

  // ------------------------------------------------------------- AMG
  const int n = d.n;
  rc = build_amg(img, b.Fu, nt, Grid2{2 * n - 1, 2 * n - 1, 2}, fp, cheb, sigma, false, P.amgFu, err);
  if (rc) return rc;
  rc = build_amg(img, b.C0, nt, Grid2{n - 1, n - 1, 1}, fp, cheb, sigma, false, P.amgC0, err);
  if (rc) return rc;
  rc = build_amg(img, b.Kp, 1, Grid2{n + 1, n + 1, 1}, fp, cheb, sigma, true, P.amgKp, err);
  if (rc) return rc;
  if (pr.adjoint) {
    Csr FuT = csr_transpose(b.Fu), C0T = csr_transpose(b.C0);
    rc = build_amg(img, FuT, nt, Grid2{2 * n - 1, 2 * n - 1, 2}, fp, cheb, sigma, false, P.amgFuT, err);
    if (rc) return rc;
    rc = build_amg(img, C0T, nt, Grid2{n - 1, n - 1, 1}, fp, cheb, sigma, false, P.amgC0T, err);
    if (rc) return rc;
  }
  // Spatial solver of the two sweeps: Chebyshev-Jacobi alone when D^{-1} A is
  // well conditioned (it then needs a few kernels per slab instead of a whole
  // V-cycle), otherwise one SA-AMG V(1,1) cycle.  D^{-1} A^T has the spectrum
  // of D^{-1} A, so the transposed sweeps reuse the interval.
  estimate_interval(img, b.Fu, nt, P.amgFu);
  estimate_interval(img, b.C0, nt, P.amgC0);
  {
    const double red_fu = pr.inner_reduction > 0 ? pr.inner_reduction : 0.3;
    const double red_ca = pr.ca_reduction > 0 ? pr.ca_reduction : 0.3;
    // The degree meets the reduction target on the estimated interval, and is
    // at least kMinAlone (the sweeps solve for increments, so the error of a
    // step is not amplified by the recursion in time; measured on a 64 x 64
    // mesh with 128 slabs and on meshes of 16 to 96 cells with up to 256 slabs,
    // tighter solves do not lower the FGMRES iteration count, and C_A below
    // degree 4 raises it).  Beyond kMaxAlone steps one
    // V-cycle is cheaper per slab.
    constexpr int kMinAlone = 4, kMaxAlone = 48;
    auto pick = [&](int opt, const Amg& a, double red) -> int {
      if (opt < 0) return 0;
      if (opt > 0) return opt;   // explicit degree, also in EXACT mode
      if (P.exact) return 0;
      const double sk = std::sqrt(a.kappa), r = (sk - 1.0) / (sk + 1.0);
      const int deg = int(std::ceil(std::log(red / 2.0) / std::log(r)));
      return deg > kMaxAlone ? 0 : std::max(kMinAlone, deg);
    };
    P.fu_deg = pick(pr.fu_solver, P.amgFu, red_fu);
    P.ca_deg = pick(pr.ca_solver, P.amgC0, red_ca);
  }
  P.chunk = pr.sweep_chunk > 0 ? pr.sweep_chunk : std::max(4, (nt + 7) / 8);
  P.pint = pr.time_parallel;
  P.pint_deg = pr.time_coarse_degree > 0 ? pr.time_coarse_degree : 1;
  if (P.pint > 0 && (P.fu_deg <= 0 || P.ca_deg <= 0 || P.pint_deg >= std::min(P.fu_deg, P.ca_deg))) {
    err = "time_parallel needs Chebyshev alone on F_u,k and C_A,k, with degrees above time_coarse_degree";
    return ST_EINVAL;
  }
  // Stencil forms of the sweep operators (structured grids, 5x5 neighbourhoods).
  P.use_stencil = (P.fu_deg > 0 || P.ca_deg > 0) && pr.sweep_format == 0 ? 1 : 0;
  // Each sweep step solves for the increment over a predictor from the earlier
  // slabs (the previous slab for F_u, linear extrapolation for the second-order
  // C_A recursion), so the couplings enter combined with the diagonal block:
  //   F_u:  r0 = q^k - A_k x^{k-1},  A_k = F_u,k - M_u/dt,  x^k = x^{k-1} + F_u,k^{-1} r0;
  //   C_A:  r0 = s^k + P_k y^{k-1} + Q_k y^{k-2},  y^k = (2 y^{k-1} - y^{k-2}) + C0_k^{-1} r0,
  //         P_k = C1_{k-1}/dt - 2 C0_k,  Q_k = C0_k - C2/dt^2  (k >= 2),
  //         P_1 = C1_0/dt - C0_1,  Q_1 = 0  (predictor y^0).
  // With exact spatial solves this is the same forward substitution; with
  // approximate ones the error is that of the increment, propagated by the
  // exact (contracting) recursion.  The combinations are formed here in FP64.
  if (P.use_stencil) {
    const int gu = 2 * n - 1, ga = n - 1;
    const double dt = b.dt;
    auto same = [](int k) { return k; };
    bool ok = pack_stencil(img, b.Fu, nt, gu, gu, 2, false, fp, P.sFu);
    {
      Csr Au = combine_sets(nt, {{&b.Fu, 1.0, same}, {&b.Mu, -1.0 / dt, [](int) { return 0; }}});
      ok = ok && pack_stencil(img, Au, nt, gu, gu, 2, false, fp, P.sAu);
    }
    ok = ok && pack_stencil(img, b.C0, nt, ga, ga, 1, false, fp, P.sC0);
    {
      Csr CP = combine_sets(nt, {{&b.C1, 1.0 / dt, [](int k) { return k >= 1 ? k - 1 : -1; }},
                                 {&b.C0, -1.0, [](int k) { return k >= 1 ? k : -1; }},
                                 {&b.C0, -1.0, [](int k) { return k >= 2 ? k : -1; }}});
      Csr CQ = combine_sets(nt, {{&b.C0, 1.0, [](int k) { return k >= 2 ? k : -1; }},
                                 {&b.C2, -1.0 / (dt * dt), [](int k) { return k >= 2 ? 0 : -1; }}});
      ok = ok && pack_stencil(img, CP, nt, ga, ga, 1, false, fp, P.sCP);
      ok = ok && pack_stencil(img, CQ, nt, ga, ga, 1, false, fp, P.sCQ);
    }
    ok = ok && pack_stencil(img, b.Mj, 1, n + 1, n + 1, 1, false, fp, P.sMj, 1);
    ok = ok && pack_stencil(img, b.KjA, 1, n + 1, n + 1, 1, false, fp, P.sKjA, 1, n - 1, n - 1, 1);
    if (pr.adjoint) {
      // Backward sweeps of the transposes: predictors x^{k+1} and 2 c^{k+1} - c^{k+2}.
      Csr FuT = csr_transpose(b.Fu), C0T = csr_transpose(b.C0), C1T = csr_transpose(b.C1), C2T = csr_transpose(b.C2);
      ok = ok && pack_stencil(img, FuT, nt, gu, gu, 2, false, fp, P.sFuT);
      Csr AuT = combine_sets(nt, {{&FuT, 1.0, same}, {&b.Mu, -1.0 / dt, [](int) { return 0; }}});
      ok = ok && pack_stencil(img, AuT, nt, gu, gu, 2, false, fp, P.sAuT);
      ok = ok && pack_stencil(img, C0T, nt, ga, ga, 1, false, fp, P.sC0T);
      const int last = nt - 1;
      Csr CPT = combine_sets(nt, {{&C1T, 1.0 / dt, [last](int k) { return k <= last - 1 ? k : -1; }},
                                  {&C0T, -1.0, [last](int k) { return k <= last - 1 ? k : -1; }},
                                  {&C0T, -1.0, [last](int k) { return k <= last - 2 ? k : -1; }}});
      Csr CQT = combine_sets(nt, {{&C0T, 1.0, [last](int k) { return k <= last - 2 ? k : -1; }},
                                  {&C2T, -1.0 / (dt * dt), [last](int k) { return k <= last - 2 ? 0 : -1; }}});
      ok = ok && pack_stencil(img, CPT, nt, ga, ga, 1, false, fp, P.sCPT);
      ok = ok && pack_stencil(img, CQT, nt, ga, ga, 1, false, fp, P.sCQT);
    }
    if (!ok) {
      err = "sweep operator does not fit a 5x5 stencil";
      return ST_EINTERNAL;
    }
  }

  // pressure normalisation weights m = 1^T M_p (FP64)
  std::vector<double> m(d.np, 0.0);
  for (int r = 0; r < b.Mp.nr; ++r)
    for (int p = b.Mp.rp[r]; p < b.Mp.rp[r + 1]; ++p) m[b.Mp.ci[p]] += b.Mp.v[p];
  P.mp_rowsum = img.put(m);
  P.image_bytes = img.bytes.size();
  P.ws_bytes = workspace_layout(P).end;
  return ST_OK;
}

}  // namespace st

extern "C" {

int st_plan_create(const st_problem* p, st_plan** out) {
  if (!p || !out) return ST_EINVAL;
  *out = nullptr;
  try {
    st_plan* pl = new st_plan;
    pl->p.prob = *p;
    std::string err;
    int rc = st::build_plan(pl->p, err);
    if (rc) {
      if (!err.empty()) std::fprintf(stderr, "libst: %s\n", err.c_str());
      delete pl;
      return rc;
    }
    pl->p.prob.ubar = pl->p.prob.abar = pl->p.prob.jbar = nullptr;   // not retained
    *out = pl;
    return ST_OK;
  } catch (const std::bad_alloc&) {
    return ST_ENOMEM;
  } catch (...) {
    return ST_EINTERNAL;
  }
}

int st_plan_workspace_size(const st_plan* plan, size_t* bytes) {
  if (!plan || !bytes) return ST_EINVAL;
  *bytes = plan->p.ws_bytes;
  return ST_OK;
}

int st_plan_sizes(const st_plan* plan, int* ns, int offsets[6]) {
  if (!plan) return ST_EINVAL;
  if (ns) *ns = plan->p.blk.d.ns;
  if (offsets)
    for (int i = 0; i < 6; ++i) offsets[i] = plan->p.blk.d.off[i];
  return ST_OK;
}

int st_plan_export_block(const st_plan* plan, int block, int k, int* nrows, int* ncols, int64_t* nnz,
                         int* rowptr, int* colind, double* val) {
  if (!plan) return ST_EINVAL;
  const st::Blocks& b = plan->p.blk;
  const st::Csr* m = nullptr;
  switch (block) {
    case 0: m = &b.Fu; break;
    case 1: m = &b.Mu; break;
    case 2: m = &b.B; break;
    case 3: m = &b.Zj; break;
    case 4: m = &b.ZA; break;
    case 5: m = &b.Mj; break;
    case 6: m = &b.KjA; break;
    case 7: m = &b.Y; break;
    case 8: m = &b.FA; break;
    case 9: m = &b.MA; break;
    case 10: m = &b.KA; break;
    case 11: m = &b.Kp; break;
    case 12: m = &b.Fp; break;
    case 13: m = &b.C0; break;
    case 14: m = &b.C1; break;
    case 15: m = &b.C2; break;
    default: return ST_EINVAL;
  }
  const int64_t z = m->nnz();
  const int nsets = z ? int(m->v.size() / z) : 1;
  if (k < 0 || k >= b.d.nt || (nsets > 1 && k >= nsets)) return ST_EINVAL;
  if (nrows) *nrows = m->nr;
  if (ncols) *ncols = m->nc;
  if (nnz) *nnz = z;
  if (!rowptr) return ST_OK;
  if (!colind || !val) return ST_EINVAL;
  std::copy(m->rp.begin(), m->rp.end(), rowptr);
  std::copy(m->ci.begin(), m->ci.end(), colind);
  const size_t s = nsets > 1 ? size_t(k) : 0;
  std::copy(m->v.begin() + s * z, m->v.begin() + (s + 1) * z, val);
  return ST_OK;
}

int st_plan_solver_info(const st_plan* plan, int* fu_degree, int* ca_degree, double* fu_kappa, double* ca_kappa) {
  if (!plan) return ST_EINVAL;
  if (fu_degree) *fu_degree = plan->p.fu_deg;
  if (ca_degree) *ca_degree = plan->p.ca_deg;
  if (fu_kappa) *fu_kappa = plan->p.amgFu.kappa;
  if (ca_kappa) *ca_kappa = plan->p.amgC0.kappa;
  return ST_OK;
}

int st_plan_cheb_intervals(const st_plan* plan, int which, double* out) {
  if (!plan || !out || (which != 0 && which != 1)) return ST_EINVAL;
  const st::Amg& a = which == 0 ? plan->p.amgFu : plan->p.amgC0;
  const int nt = plan->p.blk.d.nt;
  for (int k = 0; k < nt; ++k) {
    const int s = int(a.cheb_alone.size()) >= 2 * nt ? k : 0;
    out[2 * k] = a.cheb_alone[size_t(2 * s)];
    out[2 * k + 1] = a.cheb_alone[size_t(2 * s + 1)];
  }
  return ST_OK;
}

int st_plan_jacobian_slots(const st_plan* plan, int64_t slots[3], int* nslices) {
  if (!plan) return ST_EINVAL;
  const st::SellGroup& g = plan->p.J;
  if (slots)
    for (int s = 0; s < 3; ++s) slots[s] = s < g.nseg ? g.seg[s].total : 0;
  if (nslices) *nslices = g.nslices;
  return ST_OK;
}

int st_plan_export_jbar(const st_plan* plan, double* jbar) {
  if (!plan || !jbar) return ST_EINVAL;
  std::copy(plan->p.blk.jbar.begin(), plan->p.blk.jbar.end(), jbar);
  return ST_OK;
}

int st_plan_destroy(st_plan* plan) {
  delete plan;
  return ST_OK;
}

const char* st_error_string(int code) {
  switch (code) {
    case ST_OK: return "success";
    case ST_ENOTCONV: return "not converged within maxit";
    case ST_EINVAL: return "invalid argument";
    case ST_EHIP: return "HIP runtime error";
    case ST_ENOMEM: return "out of memory or workspace too small";
    case ST_EBREAKDOWN: return "NaN/Inf breakdown";
    case ST_EINTERNAL: return "internal setup error";
    default: return "unknown status";
  }
}

}  // extern "C"
