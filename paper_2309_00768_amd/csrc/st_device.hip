// Device side of libst: st_create, the space-time operator applies, the
// preconditioner P_T^{-1} (and its transpose) and FGMRES, all on one HIP stream.
//
// Paper references: J = eq. (jacobianSTDiscrete); P_T = Ubar_ujA Utilde_up,
// eq. (PT), with Ubar_ujA from eq. (barUuja), Utilde_up from eq. (Utilde), the
// PCD operator of eq. (Fp) and the magnetic Schur approximation
// S_A^{-1} ~ C_A^{-1} F_A M_A^{-1} of eq. (ASchurApprox); GMRES on J with right
// preconditioning (Sec. "Performance of preconditioner").
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <type_traits>
#include <utility>
#include <vector>

#include "kernels.h"
#include "kernels_nl.h"
#include "kernels_vec.h"
#include "launch.h"
#include "st_internal.h"

struct st_plan {
  st::Plan p;
};

namespace st {

// ------------------------------------------------------ device mirrors ---
struct DGroup {
  const int* perm = nullptr;
  int nrows = 0, nslices = 0, nseg = 0, lanes = 1;
  const int* sptr[3] = {nullptr, nullptr, nullptr};
  const int* col[3] = {nullptr, nullptr, nullptr};
  const void* val[3] = {nullptr, nullptr, nullptr};
  int64_t vstride[3] = {0, 0, 0};
};

struct DLevel {
  int n = 0;
  DGroup A, P, R;
  const void* dinv = nullptr;
  const double* cheb = nullptr;
};

struct DAmg {
  std::vector<DLevel> lev;
  int nsets = 1, deg = 3, ncoarse = 0;
  const void* cinv = nullptr;
  std::vector<double> alone;            // host copy of the Chebyshev-alone intervals
  const double* alone_dev = nullptr;
  // scratch: 6 vectors per level (x, b, r, d0, d1, e)
  std::vector<void*> buf;
};

// One launch of a replayed program: a recorded op through its own kernel, or
// one op of each program through a paired kernel (k_two, k_two_solve);
// arguments by value.
struct ReplayItem {
  const void* fn = nullptr;
  dim3 grid;
  int block = kBlock;
  alignas(16) unsigned char args[832];
};

struct Handle {
  Plan* plan_copy = nullptr;   // scalars only (no big host arrays kept)
  Dims d;
  double dt = 0;
  int fp32 = 0, exact = 0, inner_iters = 1, mass_iters = 12, max_restart = 30, adjoint = 0;
  int fu_deg = 0, ca_deg = 0, use_stencil = 0;
  int sweep_fuse = 0;              // stencil sweep solves in tiled launches of several steps
  int first_chunk = 0;             // slabs in the first chunk of the recorded forward apply (0: chunk)
  int mj_place = 1;                // current solves: 0 the program that finishes b first, 1 b, 2 a
  int step_rows = 0;               // rows per workgroup of the sweep step kernels (0: by precision)
  int step_lanes = 1;              // lanes per row of the two-component (F_u) step kernels: 1 or 2
  char* base = nullptr;
  WsLayout L;
  // Preconditioner scratch: null = in the workspace at its layout offsets;
  // otherwise the range [L.pt_begin, L.end) is relocated to sbase (the
  // allocation-free apply, whose scratch is the library's static array).
  char* sbase = nullptr;
  int scratch_dev = -1;                  // device of the handle's workspace
  char* noalloc_scratch = nullptr;       // that device's static scratch array
  DGroup J, JT, MA, Mj, Mp, FA, FAt, Fp, Fpt, KjA, KjAt, Bt, B, Zj, Zjt, ZAt, Mu, C1, C1t, MA64;
  DGroup Yv, Bv;                   // Y and B for the lower factors of P and P-tilde
  int variant = 0;                 // 0 P_T, 1 P-tilde, 2 P
  int pint = 0, pint_deg = 1;      // Parareal iterations of the two P_T sweeps (0: forward substitution), coarse degree
  const void *dMA = nullptr, *dMj = nullptr, *dMp = nullptr;
  const double* mp_rowsum = nullptr;
  double msum = 1.0;              // 1^T M_p 1 (the area)
  DAmg amgFu, amgC0, amgKp, amgFuT, amgC0T;
  StencilOp sFu, sAu, sC0, sCP, sCQ, sFuT, sAuT, sC0T, sCPT, sCQT;   // offsets into the image
  StencilOp sMj, sKjA;
  int use_chain = 0;               // C_A sweep + M_j solves in single-workgroup chunk kernels
  double* host_small = nullptr;   // pinned
  double precond_ms = 0.0;
  int chunk = 8;
  // Recorded forward P_T^{-1}: its two programs replayed in lockstep (launch t
  // runs the next op of each program whose dependency is met) from descriptors
  // built once; the argument blocks live in the workspace, the input and
  // output vectors are read from two device slots.
  int j_slabs = 0;                 // slabs per wavefront of the J apply (0: 8)
  int pipeline = 0, pipeline_t = 0;
  std::vector<ReplayItem> pt_items, pt_items_t;   // forward and transposed applies
  const double** rslot = nullptr;
  double** zslot = nullptr;
  // Sampled event timing of one kernel of the replayed preconditioner
  // (st_profile_kernel): every prof_every-th launch of prof_fn is bracketed by
  // a pair of events from a pool; the pairs are read after each solve.
  const void* prof_fn = nullptr;
  int prof_every = 0;
  int64_t prof_seen = 0, prof_n = 0;
  double prof_ms = 0.0;
  std::vector<hipEvent_t> prof_ev;
  size_t prof_used = 0;
};

}  // namespace st

struct st_handle {
  st::Handle h;
};

namespace st {
namespace {

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) {                                                            \
      std::fprintf(stderr, "libst: %s failed: %s\n", #expr, hipGetErrorString(e_));    \
      return ST_EHIP;                                                                  \
    }                                                                                  \
  } while (0)

template <class T>
T* at(char* base, size_t off) {
  return reinterpret_cast<T*>(base + off);
}

// A preconditioner scratch buffer at layout offset off (off >= L.pt_begin).
template <class T>
T* scr(const Handle& H, size_t off) {
  return H.sbase ? reinterpret_cast<T*>(H.sbase + (off - H.L.pt_begin)) : at<T>(H.base, off);
}

DGroup mirror(char* base, const SellGroup& g) {
  DGroup d;
  d.nrows = g.nrows;
  d.nslices = g.nslices;
  d.nseg = g.nseg;
  d.lanes = g.lanes;
  if (!g.nrows) return d;
  d.perm = at<int>(base, g.perm.off);
  for (int s = 0; s < g.nseg; ++s) {
    d.sptr[s] = at<int>(base, g.seg[s].sptr.off);
    d.col[s] = at<int>(base, g.seg[s].col.off);
    d.val[s] = base + g.seg[s].val.off;
    d.vstride[s] = g.seg[s].nsets > 1 ? g.seg[s].total : 0;
  }
  return d;
}

DAmg mirror_amg(char* base, const Amg& a, const std::vector<size_t>& bufs) {
  DAmg d;
  d.nsets = a.nsets;
  d.deg = a.cheb_degree;
  d.ncoarse = a.ncoarse;
  d.cinv = base + a.coarse_inv.off;
  for (const AmgLevel& l : a.lev) {
    DLevel dl;
    dl.n = l.nrows;
    dl.A = mirror(base, l.A);
    dl.P = mirror(base, l.P);
    dl.R = mirror(base, l.R);
    dl.dinv = base + l.dinv.off;
    dl.cheb = at<double>(base, l.cheb.off);
    d.lev.push_back(dl);
  }
  for (size_t o : bufs) d.buf.push_back(base + o);
  d.alone = a.cheb_alone;
  if (!a.cheb_alone.empty()) d.alone_dev = at<double>(base, a.cheb_alone_span.off);
  return d;
}


// ---------------------------------------------------------- launchers ---
template <class T>
Seg<T> seg(const DGroup& g, int s, int set_base, int set_step, const void* x, int64_t xstride, int xshift,
           int vlo, int vhi, double alpha) {
  Seg<T> r;
  r.sptr = g.sptr[s];
  r.col = g.col[s];
  r.val = static_cast<const T*>(g.val[s]);
  r.vstride = g.vstride[s];
  r.set_base = set_base;
  r.set_step = set_step;
  r.x = x;
  r.xstride = xstride;
  r.xshift = xshift;
  r.vlo = vlo;
  r.vhi = vhi;
  r.alpha = alpha;
  return r;
}

struct Epilogue {
  int kind = 0;
  const void* dinv = nullptr;
  double theta = 1.0;
  void *r = nullptr, *d = nullptr, *x = nullptr;
};

template <class T, class TX>
void spmv(Ctx& c, const DGroup& g, int nvec, int nseg, const Seg<T>* segs, const TX* b, int64_t bstride,
          double beta, TX* y, int64_t ystride, int role = kRoleSlab, const Epilogue* ep = nullptr) {
  SpmvArgs<T, TX> a;
  std::memset(&a, 0, sizeof(a));
  a.perm = g.perm;
  a.nslices = g.nslices;
  a.lanes = g.lanes;
  a.nseg = nseg;
  a.epi = 0;
  a.dinv = nullptr;
  a.theta = 1.0;
  a.r = a.d = a.x = nullptr;
  for (int i = 0; i < nseg; ++i) a.seg[i] = segs[i];
  a.b = b;
  a.bstride = bstride;
  a.beta = beta;
  a.y = y;
  a.ystride = ystride;
  if (ep && ep->kind == 1) {
    a.epi = 1;
    a.dinv = static_cast<const T*>(ep->dinv);
    a.theta = ep->theta;
    a.r = static_cast<TX*>(ep->r);
    a.d = static_cast<TX*>(ep->d);
    a.x = static_cast<TX*>(ep->x);
  }
  dim3 grid((g.nslices + 3) / 4, nvec);
  // In a batched launch the FP64 J apply has its own body; every other product
  // runs in the preconditioner precision of the batch.
  static_assert(std::is_same<T, TX>::value, "products take and give vectors of their own precision");
  switch (role) {
    case kRoleJ:
      emit(c, std::is_same<T, double>::value ? kKSpmvJ : kKSpmvT, grid, &k_spmv<T, TX, T, kRoleJ>, a);
      break;
    case kRoleSweep: emit(c, kKSpmvT, grid, &k_spmv<T, TX, T, kRoleSweep>, a); break;
    case kRoleAmg: emit(c, kKSpmvT, grid, &k_spmv<T, TX, T, kRoleAmg>, a); break;
    default: emit(c, kKSpmvT, grid, &k_spmv<T, TX, T, kRoleSlab>, a); break;
  }
}

// y = alpha A x + beta b for a one-segment group, nvec vectors of length n.
template <class T>
void spmv1(Ctx& c, const DGroup& g, int nvec, int set_base, int set_step, const T* x, int64_t xstride,
           double alpha, const T* b, double beta, T* y, int64_t ystride, int role = kRoleSlab) {
  Seg<T> sg = seg<T>(g, 0, set_base, set_step, x, xstride, 0, 0, nvec, alpha);
  spmv<T, T>(c, g, nvec, 1, &sg, b, ystride, beta, y, ystride, role);
}

template <class T>
void cheb_launch(Ctx& c, const DGroup& A, int nvec, int set_base, int set_step, const T* dinv, int64_t dstride,
                 const double* cheb, double theta, double delta, const T* b, T* r, T* x, const T* dold, T* dnew,
                 int64_t vec, int mode, int step, int x_add, int role) {
  ChebArgs<T> a;
  std::memset(&a, 0, sizeof(a));
  a.perm = A.perm;
  a.nslices = A.nslices;
  a.lanes = A.lanes;
  a.sptr = A.sptr[0];
  a.col = A.col[0];
  a.val = static_cast<const T*>(A.val[0]);
  a.vstride = A.vstride[0];
  a.set_base = set_base;
  a.set_step = set_step;
  a.dinv = dinv;
  a.dstride = dstride;
  a.cheb = cheb;
  a.theta = theta;
  a.delta = delta;
  a.b = b;
  a.r = r;
  a.x = x;
  a.dold = dold;
  a.dnew = dnew;
  a.vec = vec;
  a.mode = mode;
  a.step = step;
  a.x_add = x_add;
  dim3 grid((A.nslices + 3) / 4, nvec);
  if (role == 1) emit(c, kKCheb, grid, &k_cheb<T, 1>, a);
  else if (role == 2) emit(c, kKCheb, grid, &k_cheb<T, 2>, a);
  else emit(c, kKCheb, grid, &k_cheb<T, 0>, a);
}

// Chebyshev-Jacobi polynomial solve of A x = b with `steps` steps from x = 0
// (or x += correction when x_add), using caller scratch r, d0, d1.
template <class T>
void cheb_solve(Ctx& c, const DGroup& A, int nvec, int set_base, int set_step, const T* dinv, int64_t dstride,
                const double* cheb, double theta, double delta, const T* b, T* x, T* r, T* d0, T* d1, int64_t vec,
                int steps, int x_add, bool final_residual, int role = 0) {
  cheb_launch<T>(c, A, nvec, set_base, set_step, dinv, dstride, cheb, theta, delta, b, r, x, nullptr, d0, vec, 0, 0,
                 x_add, role);
  T* d[2] = {d0, d1};
  for (int i = 1; i < steps; ++i)
    cheb_launch<T>(c, A, nvec, set_base, set_step, dinv, dstride, cheb, theta, delta, nullptr, r, x, d[(i - 1) % 2],
                   d[i % 2], vec, 1, i, 1, role);
  if (final_residual)
    cheb_launch<T>(c, A, nvec, set_base, set_step, dinv, dstride, cheb, theta, delta, nullptr, r, x,
                   d[(steps - 1) % 2], d[steps % 2], vec, 2, 0, 1, role);
}

// ---------------------------------------------------------------- AMG ---
// One V(1,1) cycle on level l for nvec vectors (value set set_base + v*set_step).
// Level-0 vectors may be supplied by the caller (x0, b0); x_add: x holds a guess.
template <class T>
void vcycle(Ctx& c, DAmg& a, int l, int nvec, int set_base, int set_step, T* x0, const T* b0, int x_add,
            bool need_residual) {
  DLevel& L = a.lev[l];
  const int64_t vec = L.n;   // vectors of one level are stored back to back
  T* x = (l == 0 && x0) ? x0 : static_cast<T*>(a.buf[6 * l + 0]);
  const T* b = (l == 0 && b0) ? b0 : static_cast<const T*>(a.buf[6 * l + 1]);
  T* r = static_cast<T*>(a.buf[6 * l + 2]);
  T* d0 = static_cast<T*>(a.buf[6 * l + 3]);
  T* d1 = static_cast<T*>(a.buf[6 * l + 4]);
  const T* dinv = static_cast<const T*>(L.dinv);
  const int64_t dstride = a.nsets > 1 ? L.n : 0;
  const bool coarsest = (l + 1 == int(a.lev.size()));
  if (coarsest) {
    const T* rhs = b;
    if (x_add) {   // x += Ainv (b - A x)
      spmv1<T>(c, L.A, nvec, set_base, set_step, x, vec, -1.0, b, 1.0, r, vec, kRoleAmg);
      rhs = r;
    }
    CoarseArgs<T> ca;
    std::memset(&ca, 0, sizeof(ca));
    ca.n = a.ncoarse;
    ca.inv = static_cast<const T*>(a.cinv);
    ca.istride = a.nsets > 1 ? int64_t(a.ncoarse) * a.ncoarse : 0;
    ca.set_base = set_base;
    ca.set_step = set_step;
    ca.b = rhs;
    ca.x = x;
    ca.vec = vec;
    ca.accumulate = x_add;
    emit(c, kKCoarse, dim3(nvec), &k_coarse<T>, ca);
    if (need_residual) spmv1<T>(c, L.A, nvec, set_base, set_step, x, vec, -1.0, b, 1.0, r, vec, kRoleAmg);
    return;
  }
  const int deg = a.deg;
  const int crole = l == 0 ? 1 : 2;
  // pre-smoothing (leaves r = b - A x)
  if (x_add) {
    spmv1<T>(c, L.A, nvec, set_base, set_step, x, vec, -1.0, b, 1.0, r, vec, kRoleAmg);
    cheb_solve<T>(c, L.A, nvec, set_base, set_step, dinv, dstride, L.cheb, 0, 0, nullptr, x, r, d0, d1, vec, deg, 1,
                  true, crole);
  } else {
    cheb_solve<T>(c, L.A, nvec, set_base, set_step, dinv, dstride, L.cheb, 0, 0, b, x, r, d0, d1, vec, deg, 0, true,
                  crole);
  }
  // coarse-grid correction
  DLevel& C = a.lev[l + 1];
  const int64_t cvec = C.n;
  T* cb = static_cast<T*>(a.buf[6 * (l + 1) + 1]);
  T* cx = static_cast<T*>(a.buf[6 * (l + 1) + 0]);
  spmv1<T>(c, L.R, nvec, 0, 0, r, vec, 1.0, nullptr, 0.0, cb, cvec, kRoleAmg);
  vcycle<T>(c, a, l + 1, nvec, set_base, set_step, nullptr, nullptr, 0, false);
  spmv1<T>(c, L.P, nvec, 0, 0, cx, cvec, 1.0, x, 1.0, x, vec, kRoleAmg);   // x += P x_c
  // post-smoothing
  spmv1<T>(c, L.A, nvec, set_base, set_step, x, vec, -1.0, b, 1.0, r, vec, kRoleAmg);
  cheb_solve<T>(c, L.A, nvec, set_base, set_step, dinv, dstride, L.cheb, 0, 0, nullptr, x, r, d0, d1, vec, deg, 1,
                need_residual, crole);
}

// Spatial solve A x = b with `iters` V-cycles (x starts from zero).
template <class T>
void amg_solve(Ctx& c, DAmg& a, int nvec, int set_base, int set_step, T* x, const T* b, int iters) {
  for (int it = 0; it < iters; ++it) vcycle<T>(c, a, 0, nvec, set_base, set_step, x, b, it > 0 ? 1 : 0, false);
}

// ----------------------------------------------- vector launch helpers ---
inline int grid_for(int64_t n) {
  int64_t b = (n + kBlock - 1) / kBlock;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return int(b);
}

inline void slab_sums_d(Ctx& c, const double* src, int64_t ld, int off, int len, const double* w, double* out,
                        int nt, const double* const* rslot = nullptr) {
  SlabSumsDArgs a{src, ld, off, len, w, out, rslot};
  emit(c, kKSlabSumsD, dim3(nt), &k_slab_sums_d, a);
}

template <class T>
inline void slab_sums_t(Ctx& c, const T* src, int64_t ld, int len, const double* w, double* out, int nt) {
  SlabSumsTArgs<T> a{src, ld, len, w, out};
  emit(c, kKSlabSumsT, dim3(nt), &k_slab_sums_t<T>, a);
}

template <class T>
inline void slab_shift(Ctx& c, T* x, int64_t ld, int len, int nt, const double* sums, double scale) {
  SlabShiftArgs<T> a{x, ld, len, nt, sums, scale};
  const int kind = std::is_same<T, double>::value ? kKSlabShiftD : kKSlabShiftT;
  emit(c, kind, dim3(grid_for(int64_t(len) * nt)), &k_slab_shift<T>, a);
}

// One sweep step: x = A_k^{-1} (q + coupling), the coupling given as segments
// of `cg` acting on earlier (or later) slabs.  With deg > 0 the solve is
// Chebyshev-Jacobi alone of that degree, its first step fused into the
// coupling product; otherwise the right-hand side is formed and `vc`
// V-cycles of the hierarchy are applied.
template <class T>
void sweep_step(Ctx& c, DAmg& a, const DGroup& cg, int nseg, const Seg<T>* segs, const T* q, T* x, int k, int deg,
                int vc) {
  T* rhs = static_cast<T*>(a.buf[1]);
  if (deg <= 0) {
    spmv<T, T>(c, cg, 1, nseg, segs, q, 0, 1.0, rhs, 0, kRoleSweep);
    amg_solve<T>(c, a, 1, k, 0, x, rhs, vc);
    return;
  }
  DLevel& L = a.lev[0];
  T* r = static_cast<T*>(a.buf[2]);
  T* d0 = static_cast<T*>(a.buf[3]);
  T* d1 = static_cast<T*>(a.buf[4]);
  const int64_t dstride = a.nsets > 1 ? L.n : 0;
  const T* dinv = static_cast<const T*>(L.dinv) + (a.nsets > 1 ? int64_t(k) * L.n : 0);
  Epilogue ep;
  ep.kind = 1;
  ep.dinv = dinv;
  ep.theta = a.alone[2 * (a.nsets > 1 ? k : 0)];
  ep.r = r;
  ep.d = d0;
  ep.x = x;
  spmv<T, T>(c, cg, 1, nseg, segs, q, 0, 1.0, rhs, 0, kRoleSweep, &ep);
  T* d[2] = {d0, d1};
  for (int i = 1; i < deg; ++i)
    cheb_launch<T>(c, L.A, 1, a.nsets > 1 ? k : 0, 0, static_cast<const T*>(L.dinv), dstride, a.alone_dev, 0, 0,
                   nullptr, r, x, d[(i - 1) % 2], d[i % 2], L.n, 1, i, 1, 1);
}

template <class T>
StOp<T> st_op(char* base, const StencilOp& o) {
  StOp<T> a;
  a.coef = reinterpret_cast<const T*>(base + o.coef.off);
  a.set_stride = o.nsets > 1 ? int64_t(o.nslot) * o.rows : 0;
  a.gx = o.gx;
  a.gy = o.gy;
  a.ncomp = o.ncomp;
  a.diag_comp = o.diag_comp;
  a.nslot = o.nslot;
  a.cgx = o.cgx;
  a.cgy = o.cgy;
  a.shift = o.shift;
  a.rows = o.rows;
  return a;
}

// Tiles of the fused sweep solve and the steps one launch may take: the grown
// tile (tile + 2 x radius x stencil applications) must fit the LDS arrays.
// Rows per workgroup of a sweep step kernel: a slab's grid has few rows
// (32,258 velocity rows at 64 x 64), so smaller workgroups spread a step over
// more CUs; measured at 64 x 64, FP64 steps gain from 64 rows (the P_T apply
// drops from 5.1 to 4.5 ms) and FP32 steps are latency-bound at any size.
template <class T>
constexpr int st_rows() { return sizeof(T) == 8 ? 64 : 128; }
constexpr int kSolveTile = 8;
constexpr int kSolveFirst = 4;   // steps 0..3: three applications of A
constexpr int kSolveNext = 3;    // a continuing launch also applies A to the d it reads

// Whether the fused solve handles operator A (one radius-2 stencil on a grid
// that is its own column grid, at most two components).
inline bool solve_fusable(const StencilOp& A) {
  const int hmax = 2 * std::max(kSolveFirst - 1, kSolveNext);
  return A.rad == 2 && A.ncomp <= kTileComp && A.cgx == A.gx && A.cgy == A.gy && A.shift == 0 &&
         (kSolveTile + 2 * hmax) * (kSolveTile + 2 * hmax) <= kTileExt && kSolveTile * kSolveTile <= kTileOut &&
         int64_t(A.gx) * A.gy * A.ncomp == A.rows;
}

// Launches per sweep solve of degree deg.
inline int sweep_launches(const Handle& H, int deg) {
  if (!H.sweep_fuse) return deg;
  return deg <= kSolveFirst ? 1 : 1 + (deg - kSolveFirst + kSolveNext - 1) / kSolveNext;
}

// One sweep step with Chebyshev-Jacobi alone on stencil operators:
// x = x0 + p(D^{-1} A_k) D^{-1} r0 with r0 = q + a1 S1 y1 + a2 S2 y2 the
// residual of the predictor x0 = g1 y1 + g2 y2 (x0 = 0 when !guess).  Fused:
// the tiled solve kernel, up to kSolveFirst steps in its first launch and
// kSolveNext in each later one; otherwise one kernel per step.
template <class T>
void sweep_step_stencil(Ctx& c, Handle& H, DAmg& a, const StencilOp& A, const StencilOp* S1, int set1, double a1,
                        const T* y1, const StencilOp* S2, int set2, double a2, const T* y2, const T* q, T* x, int k,
                        int deg, int role, bool guess = false, double g1 = 0.0, double g2 = 0.0,
                        const T* y3 = nullptr, double g3 = 0.0) {
  DLevel& L = a.lev[0];
  const int64_t rows = A.rows;
  T* r = static_cast<T*>(a.buf[2]);
  T* d0 = static_cast<T*>(a.buf[3]);
  T* d1 = static_cast<T*>(a.buf[4]);
  const T* dinv = static_cast<const T*>(L.dinv) + (a.nsets > 1 ? int64_t(k) * L.n : 0);
  const int iset = a.nsets > 1 ? k : 0;
  const double theta = a.alone[2 * iset], delta = a.alone[2 * iset + 1];
  StInitArgs<T> ia;
  std::memset(&ia, 0, sizeof(ia));
  ia.S1 = S1 ? st_op<T>(H.base, *S1) : StOp<T>{};
  ia.S2 = S2 ? st_op<T>(H.base, *S2) : StOp<T>{};
  ia.set1 = set1;
  ia.set2 = set2;
  ia.n1 = S1 != nullptr;
  ia.n2 = S2 != nullptr;
  ia.a1 = a1;
  ia.a2 = a2;
  ia.y1 = y1;
  ia.y2 = y2;
  ia.q = q;
  ia.dinv = dinv;
  ia.theta = theta;
  ia.r = r;
  ia.d = d0;
  ia.x = x;
  ia.rows = rows;
  ia.guess = guess ? 1 : 0;
  ia.g1 = g1;
  ia.g2 = g2;
  ia.y3 = y3;
  ia.g3 = g3;
  // Two lanes per row only for two-component operators (F_u,k and its coupling).
  auto two = [](const StencilOp* o) { return !o || (o->ncomp == 2 && !o->diag_comp); };
  const int lanes = H.step_lanes == 2 && two(&A) && two(S1) && two(S2) ? 2 : 1;
  const int rpb = std::min(H.step_rows > 0 ? H.step_rows : st_rows<T>(), kBlock / lanes);
  ia.rpb = rpb;
  ia.lanes = lanes;
  if (H.sweep_fuse && solve_fusable(A)) {
    StSolveArgs<T> sa;
    std::memset(&sa, 0, sizeof(sa));
    sa.in = ia;
    sa.A = st_op<T>(H.base, A);
    sa.set = iset;
    sa.delta = delta;
    sa.tx = sa.ty = kSolveTile;
    sa.ntx = (A.gx + kSolveTile - 1) / kSolveTile;
    const dim3 grid(unsigned(sa.ntx * ((A.gy + kSolveTile - 1) / kSolveTile)));
    // a continuing launch reads the previous launch's r and d from the other pair of buffers
    T* rb[2] = {r, static_cast<T*>(a.buf[1])};
    T* db[2] = {d0, d1};
    for (int s0 = 0, l = 0; s0 < deg; ++l) {
      sa.s0 = s0;
      sa.ns = std::min(deg - s0, s0 == 0 ? kSolveFirst : kSolveNext);
      sa.more = s0 + sa.ns < deg ? 1 : 0;
      sa.r_in = rb[(l + 1) % 2];
      sa.d_in = db[(l + 1) % 2];
      sa.in.r = rb[l % 2];
      sa.in.d = db[l % 2];
      if (role == 1) emit(c, kKStSolve, grid, &k_st_solve<T, 1>, sa);
      else emit(c, kKStSolve, grid, &k_st_solve<T, 2>, sa);
      s0 += sa.ns;
    }
    return;
  }
  const dim3 grid(unsigned((rows + rpb - 1) / rpb));
  if (role == 1) emit(c, kKStInit, grid, &k_st_init<T, 1>, ia);
  else emit(c, kKStInit, grid, &k_st_init<T, 2>, ia);
  StChebArgs<T> ca;
  std::memset(&ca, 0, sizeof(ca));
  ca.A = st_op<T>(H.base, A);
  ca.set = iset;
  ca.dinv = dinv;
  ca.rows = rows;
  ca.r = r;
  ca.x = x;
  ca.rpb = rpb;
  ca.lanes = lanes;
  T* d[2] = {d0, d1};
  ChebRec cr(theta, delta);
  for (int i = 1; i < deg; ++i) {
    double k1, k2;
    cr.next(k1, k2);
    ca.c1 = k1;
    ca.c2 = k2;
    ca.dold = d[(i - 1) % 2];
    ca.dnew = d[i % 2];
    if (role == 1) emit(c, kKStCheb, grid, &k_st_cheb<T, 1>, ca);
    else emit(c, kKStCheb, grid, &k_st_cheb<T, 2>, ca);
  }
}

// ====================================== parallel-in-time sweeps (Parareal) ===
// The two sweeps of P_T^{-1} with K Parareal iterations instead of forward
// substitution in time.  A slab step maps the earlier slabs to slab k,
//   F_u: x^k = x^{k-1} + S_k(g^k - A_k x^{k-1}),  A_k = F_u,k - M_u/dt;
//   C_A: y^k = p^k + S_k(s^k + C1_{k-1}/dt y^{k-1} - C2/dt^2 y^{k-2} - C0_k p^k),
//        p^k = 2 y^{k-1} - y^{k-2} (y^0 for k = 1, 0 for k = 0),
// with S_k Chebyshev-Jacobi on the diagonal block: the plan's degree (fine) or
// the coarse degree (coarse).  Iteration j -> j+1:
//   x_{j+1}^k = G_k(x_{j+1}^{<k}) + (F_k - G_k)(x_j^{<k}),
// from the coarse sweep x_0.  The corrections F_k - G_k = (S^fine - S^coarse) r_k
// of all slabs are computed together (SELL products and Chebyshev steps over
// every slab in one launch each: the Chebyshev iterates are nested, so the
// increments past the coarse degree are the difference); the coarse sweep runs
// slab by slab with the stencil steps, the correction added to the predictor.
template <class T>
struct ParaBufs {
  T* alt;    // the iterate not held in the output
  T* corr;   // (S^fine - S^coarse) r per slab
  T* acc;    // the first coarse-degree increments (discarded)
  T* r;
  T* d0;
  T* d1;
};

template <class T>
ParaBufs<T> para_bufs(Handle& H, const size_t* off) {
  return ParaBufs<T>{scr<T>(H, off[0]), scr<T>(H, off[1]), scr<T>(H, off[2]),
                     scr<T>(H, off[3]), scr<T>(H, off[4]), scr<T>(H, off[5])};
}

// corr = (S^fine - S^coarse) r over all nt slabs (r holds the slabs' residuals).
template <class T>
void para_correction(Ctx& c, DAmg& a, int nt, int deg_f, int deg_c, const ParaBufs<T>& pb) {
  DLevel& L = a.lev[0];
  const int64_t n = L.n;
  FillArgs f{reinterpret_cast<double*>(pb.corr), int64_t((size_t(nt) * size_t(n) * sizeof(T) + 7) / 8), 0.0};
  emit(c, kKFill, dim3(grid_for(f.n)), &k_fill, f);
  T* d[2] = {pb.d0, pb.d1};
  const int sstep = a.nsets > 1 ? 1 : 0;
  const int64_t dstride = a.nsets > 1 ? n : 0;
  for (int i = 0; i < deg_f; ++i)
    cheb_launch<T>(c, L.A, nt, 0, sstep, static_cast<const T*>(L.dinv), dstride, a.alone_dev, 0, 0, nullptr, pb.r,
                   i < deg_c ? pb.acc : pb.corr, d[(i + 1) % 2], d[i % 2], n, i == 0 ? 0 : 1, i, 0, 1);
}

// x = the F_u sweep of g (nt slabs) by K Parareal iterations.
template <class T>
void parareal_fu(Ctx& c, Handle& H, const T* g, T* x) {
  const int nt = H.d.nt, nu = H.d.nu, K = H.pint, dc = H.pint_deg;
  const double dt = H.dt;
  const ParaBufs<T> pb = para_bufs<T>(H, H.L.pint_u);
  auto buf = [&](int j) { return (j % 2) == (K % 2) ? x : pb.alt; };
  auto at = [&](T* v, int k) { return v + int64_t(k) * nu; };
  auto coarse_sweep = [&](T* y, bool corr) {
    for (int k = 0; k < nt; ++k)
      sweep_step_stencil<T>(c, H, H.amgFu, H.sFu, k >= 1 ? &H.sAu : nullptr, k, -1.0,
                            k >= 1 ? at(y, k - 1) : at(pb.corr, 0), nullptr, 0, 0.0, nullptr, g + int64_t(k) * nu,
                            at(y, k), k, dc, 1, corr || k >= 1, k >= 1 ? 1.0 : 0.0, 0.0,
                            corr ? at(pb.corr, k) : nullptr, corr ? 1.0 : 0.0);
  };
  coarse_sweep(buf(0), false);
  const DGroup& Fu = H.amgFu.lev[0].A;
  for (int j = 0; j < K; ++j) {
    const T* cur = buf(j);
    // r^k = g^k - F_u,k x^{k-1} + (1/dt) M_u x^{k-1} (k >= 1), r^0 = g^0
    Seg<T> sf = seg<T>(Fu, 0, 0, 1, cur, nu, -1, 1, nt, -1.0);
    spmv<T, T>(c, Fu, nt, 1, &sf, g, nu, 1.0, pb.r, nu, kRoleSweep);
    Seg<T> sm = seg<T>(H.Mu, 0, 0, 0, cur, nu, -1, 1, nt, 1.0 / dt);
    spmv<T, T>(c, H.Mu, nt, 1, &sm, pb.r, nu, 1.0, pb.r, nu, kRoleSweep);
    para_correction<T>(c, H.amgFu, nt, H.fu_deg, dc, pb);
    coarse_sweep(buf(j + 1), true);
  }
}

// y = the C_A sweep of s (nt slabs) by K Parareal iterations.
template <class T>
void parareal_ca(Ctx& c, Handle& H, const T* s, T* y) {
  const int nt = H.d.nt, na = H.d.na, K = H.pint, dc = H.pint_deg;
  const double dt = H.dt;
  const ParaBufs<T> pb = para_bufs<T>(H, H.L.pint_a);
  auto buf = [&](int j) { return (j % 2) == (K % 2) ? y : pb.alt; };
  auto at = [&](T* v, int k) { return v + int64_t(k) * na; };
  auto coarse_sweep = [&](T* v, bool corr) {
    for (int k = 0; k < nt; ++k)
      sweep_step_stencil<T>(c, H, H.amgC0, H.sC0, k >= 1 ? &H.sCP : nullptr, k, 1.0,
                            k >= 1 ? at(v, k - 1) : at(pb.corr, 0), k >= 2 ? &H.sCQ : nullptr, k, 1.0,
                            k >= 2 ? at(v, k - 2) : at(pb.corr, 0), s + int64_t(k) * na, at(v, k), k, dc, 2,
                            corr || k >= 1, k >= 2 ? 2.0 : (k >= 1 ? 1.0 : 0.0), k >= 2 ? -1.0 : 0.0,
                            corr ? at(pb.corr, k) : nullptr, corr ? 1.0 : 0.0);
  };
  coarse_sweep(buf(0), false);
  const DGroup& C0 = H.amgC0.lev[0].A;
  for (int j = 0; j < K; ++j) {
    const T* cur = buf(j);
    // r^k = s^k + (1/dt) C1_{k-1} y^{k-1} - (1/dt^2) C2 y^{k-2} - C0_k p^k
    Seg<T> s1[2] = {seg<T>(H.C1, 0, -1, 1, cur, na, -1, 1, nt, 1.0 / dt),
                    seg<T>(H.C1, 1, 0, 0, cur, na, -2, 2, nt, -1.0 / (dt * dt))};
    spmv<T, T>(c, H.C1, nt, 2, s1, s, na, 1.0, pb.r, na, kRoleSweep);
    Seg<T> s0[3] = {seg<T>(C0, 0, 0, 1, cur, na, -1, 2, nt, -2.0), seg<T>(C0, 0, 0, 1, cur, na, -2, 2, nt, 1.0),
                    seg<T>(C0, 0, 0, 1, cur, na, -1, 1, std::min(2, nt), -1.0)};
    spmv<T, T>(c, C0, nt, 3, s0, pb.r, na, 1.0, pb.r, na, kRoleSweep);
    para_correction<T>(c, H.amgC0, nt, H.ca_deg, dc, pb);
    coarse_sweep(buf(j + 1), true);
  }
}

// ================================================= P_T^{-1} (forward) ===
// z = P_T^{-1} r.  `c` receives the launches of program b and `ca` those of
// program a: when not recording both are the caller's stream and everything
// runs in the order written; when recording (Program: two op lists, the
// b-ops carrying how many a-ops they wait for) a = the magnetic part up to
// the C_A sweep (and the current solves when that balances the two better),
// b = the pressure part, then per chunk of slabs the velocity right-hand side
// and the F_u sweep, which wait for that chunk of the C_A sweep.  With slots,
// r and z are read from device slots instead (recorded programs).
template <class T>
int precond_forward(Handle& H, const double* r, double* z, Ctx& c, Ctx& ca, const double* const* rslot = nullptr,
                    double* const* zslot = nullptr) {
  const Dims& d = H.d;
  const int nt = d.nt;
  char* B = H.base;
  const WsLayout& L = H.L;
  T* ru = scr<T>(H, L.ru); T* yu = scr<T>(H, L.yu); T* xu = scr<T>(H, L.xu);
  T* rp = scr<T>(H, L.rp); T* q = scr<T>(H, L.q); T* t = scr<T>(H, L.t); T* xp = scr<T>(H, L.xp);
  T* rj = scr<T>(H, L.rj); T* yj = scr<T>(H, L.yj);
  T* ra = scr<T>(H, L.ra); T* w = scr<T>(H, L.wA); T* sA = scr<T>(H, L.sA); T* yA = scr<T>(H, L.yA);
  T* mr = scr<T>(H, L.mr); T* md0 = scr<T>(H, L.md0); T* md1 = scr<T>(H, L.md1);
  T* mr2 = scr<T>(H, L.mr2); T* md02 = scr<T>(H, L.md02); T* md12 = scr<T>(H, L.md12);
  double* psum = scr<double>(H, L.psum);
  const int o2 = d.off[2], o3 = d.off[3], o4 = d.off[4], ns = d.ns;
  const int nu = d.nu, np = d.np, nj = d.nj, na = d.na;
  const double dt = H.dt;
  const int vc = H.exact ? H.inner_iters : 1;       // V-cycles per spatial solve
  const int mit = H.mass_iters;
  // Q1 mass: eigenvalues of D^{-1} M lie in [1/4, 9/4] on squares; widened slightly.
  const double mlo = 0.24, mhi = 2.3, mth = 0.5 * (mhi + mlo), mde = 0.5 * (mhi - mlo);
  const bool rec = c.recording();
  const bool chain = H.use_chain && !rec;
  // Chunk boundaries: a first chunk of H.first_chunk slabs (0: C), then C each.
  const int C = rec ? std::max(1, std::min(H.chunk, nt)) : nt;
  std::vector<int> cb{0};
  for (int k = rec && H.first_chunk > 0 ? std::min(H.first_chunk, C) : C; k < nt; k += C) cb.push_back(k);
  cb.push_back(nt);
  const int nch = int(cb.size()) - 1;
  // The pressure part runs in b-ops that wait only for the split.
  auto mark = [&](Ctx& cx, int need) { cx.need = need; };

  // 0. split r, projecting the pressure rows to zero sum per slab (program a)
  slab_sums_d(ca, r, int64_t(ns), o2, np, nullptr, psum, nt, rslot);
  {
    SplitArgs<T> a{r, ns, nt, o2, o3, o4, psum, ru, rp, rj, ra, rslot};
    emit(ca, kKSplit, dim3(grid_for(int64_t(ns) * nt)), &k_split<T>, a);
  }
  const int a_split = rec ? int(ca.rec->size()) : 0;
  // 1. magnetic Schur complement: w = M_A^{-1} r_A; s = F_A w (all slabs at once)
  cheb_solve<T>(ca, H.MA, nt, 0, 0, static_cast<const T*>(H.dMA), 0, nullptr, mth, mde, ra, w, mr, md0, md1, na, mit,
                0, false);
  {
    Seg<T> sg[2] = {seg<T>(H.FA, 0, 0, 1, w, na, 0, 0, nt, 1.0), seg<T>(H.FA, 1, 0, 0, w, na, -1, 1, nt, 1.0)};
    spmv<T, T>(ca, H.FA, nt, 2, sg, nullptr, na, 0.0, sA, na);
  }
  // 2. pressure (program b, alongside the C_A sweep): q = K_p^{-1} r_p; t = F_p q;
  //    x_p = -M_p^{-1} t (xp holds M_p^{-1} t; the sign is applied where x_p is used)
  mark(c, a_split);
  amg_solve<T>(c, H.amgKp, nt, 0, 0, q, rp, vc);
  {
    Seg<T> sg[2] = {seg<T>(H.Fp, 0, 0, 1, q, np, 0, 0, nt, 1.0), seg<T>(H.Fp, 1, 0, 0, q, np, -1, 1, nt, 1.0)};
    spmv<T, T>(c, H.Fp, nt, 2, sg, nullptr, np, 0.0, t, np);
  }
  // the b-side mass solves use their own scratch: a-side ones may run alongside
  cheb_solve<T>(c, H.Mp, nt, 0, 0, static_cast<const T*>(H.dMp), 0, nullptr, mth, mde, t, xp, mr2, md02, md12, np,
                mit, 0, false);
  // 3. y_A = C_A^{-1} s: forward sweep (program a), chunk by chunk; per chunk
  //    y_j = M_j^{-1}(r_j - K_jA y_A) (the current solve, in either program),
  //    g_u = r_u - Z_j y_j - Z_A y_A - B^T x_p and x_u = F_u^{-1} g_u (forward
  //    sweep, program b, once that chunk of the C_A sweep is done)
  auto current_solve = [&](Ctx& cx, int k0, int kc, T* r_, T* d0_, T* d1_) {
    spmv1<T>(cx, H.KjA, kc, 0, 0, yA + int64_t(k0) * na, na, -1.0, rj + int64_t(k0) * nj, 1.0,
             rj + int64_t(k0) * nj, nj);
    cheb_solve<T>(cx, H.Mj, kc, 0, 0, static_cast<const T*>(H.dMj), 0, nullptr, mth, mde, rj + int64_t(k0) * nj,
                  yj + int64_t(k0) * nj, r_ + int64_t(k0) * nj, d0_ + int64_t(k0) * nj, d1_ + int64_t(k0) * nj, nj,
                  mit, 0, false);
  };
  auto ca_step = [&](Ctx& cx, int k) {
    if (H.use_stencil && H.ca_deg > 0) {
      // increment over the predictor y^0 (k = 1) or 2 y^{k-1} - y^{k-2} (k >= 2)
      sweep_step_stencil<T>(cx, H, H.amgC0, H.sC0, k >= 1 ? &H.sCP : nullptr, k, 1.0, yA + int64_t(k - 1) * na,
                            k >= 2 ? &H.sCQ : nullptr, k, 1.0, yA + int64_t(k - 2) * na, sA + int64_t(k) * na,
                            yA + int64_t(k) * na, k, H.ca_deg, 2, k >= 1, k >= 2 ? 2.0 : 1.0, k >= 2 ? -1.0 : 0.0);
    } else {
      Seg<T> sg[2];
      int nsg = 0;
      if (k >= 1) sg[nsg++] = seg<T>(H.C1, 0, k - 1, 0, yA + int64_t(k - 1) * na, 0, 0, 0, 1, 1.0 / dt);
      if (k >= 2) sg[nsg++] = seg<T>(H.C1, 1, 0, 0, yA + int64_t(k - 2) * na, 0, 0, 0, 1, -1.0 / (dt * dt));
      sweep_step<T>(cx, H.amgC0, H.C1, nsg, sg, sA + int64_t(k) * na, yA + int64_t(k) * na, k, H.ca_deg, vc);
    }
  };
  auto fu_step = [&](Ctx& cx, int k) {
    if (H.use_stencil && H.fu_deg > 0) {
      // increment over the predictor x^{k-1}: r0 = g^k - (F_u,k - M_u/dt) x^{k-1}
      sweep_step_stencil<T>(cx, H, H.amgFu, H.sFu, k >= 1 ? &H.sAu : nullptr, k, -1.0, xu + int64_t(k - 1) * nu,
                            nullptr, 0, 0.0, nullptr, yu + int64_t(k) * nu, xu + int64_t(k) * nu, k, H.fu_deg, 1,
                            k >= 1, 1.0, 0.0);
    } else {
      Seg<T> sg = seg<T>(H.Mu, 0, 0, 0, xu + int64_t(k - 1) * nu, 0, 0, 0, 1, 1.0 / dt);
      sweep_step<T>(cx, H.amgFu, H.Mu, k >= 1 ? 1 : 0, &sg, yu + int64_t(k) * nu, xu + int64_t(k) * nu, k,
                    H.fu_deg, vc);
    }
  };
  // Lockstep estimate (one op of each program per launch; a never waits): b's
  // work on a chunk starts once a has finished that chunk and b its earlier
  // work.  The current solve goes to the program that lets b finish the chunk
  // first (H.mj_place 0), or always to b (1) or to a (2).  The op counts come
  // from recording into a scratch list.
  int cs_ops = 0, fu_ops = 0;
  if (rec) {
    std::vector<Op> tmp;
    Ctx ct{nullptr, &tmp, nullptr, 0};
    current_solve(ct, 0, 1, mr2, md02, md12);
    cs_ops = int(tmp.size());
    tmp.clear();
    fu_step(ct, std::min(1, nt - 1));
    fu_ops = int(tmp.size());
  }
  int tb = rec ? a_split + int(c.rec->size()) : 0;
  if (H.pint > 0 && !rec) {
    // both sweeps by Parareal over all slabs at once: y_A, then the current
    // solves and the velocity right-hand side of every slab, then x_u
    parareal_ca<T>(ca, H, sA, yA);
    current_solve(c, 0, nt, mr2, md02, md12);
    Seg<T> sg[3] = {seg<T>(H.Zj, 0, 0, 1, yj, nj, 0, 0, nt, -1.0), seg<T>(H.Zj, 1, 0, 1, yA, na, 0, 0, nt, -1.0),
                    seg<T>(H.Zj, 2, 0, 0, xp, np, 0, 0, nt, 1.0)};
    spmv<T, T>(c, H.Zj, nt, 3, sg, ru, nu, 1.0, yu, nu);
    parareal_fu<T>(c, H, yu, xu);
  }
  for (int ch = 0; ch < nch && !(H.pint > 0 && !rec); ++ch) {
    const int k0 = cb[size_t(ch)], k1 = cb[size_t(ch) + 1], kc = k1 - k0;
    if (chain) {
      ChainArgs<T> cha;
      cha.C0 = st_op<T>(B, H.sC0);
      cha.CP = st_op<T>(B, H.sCP);
      cha.CQ = st_op<T>(B, H.sCQ);
      cha.Mj = st_op<T>(B, H.sMj);
      cha.KjA = st_op<T>(B, H.sKjA);
      cha.k0 = k0;
      cha.k1 = k1;
      cha.deg = H.ca_deg;
      cha.mit = mit;
      cha.na = na;
      cha.nj = nj;
      cha.dt = dt;
      cha.alone = H.amgC0.alone_dev;
      cha.dinvC = static_cast<const T*>(H.amgC0.lev[0].dinv);
      cha.dinv_stride = H.amgC0.nsets > 1 ? na : 0;
      cha.dinvM = static_cast<const T*>(H.dMj);
      cha.mth = mth;
      cha.mde = mde;
      cha.sA = sA;
      cha.yA = yA;
      cha.rj = rj;
      cha.yj = yj;
      cha.r = scr<T>(H, L.chr);
      cha.d0 = scr<T>(H, L.chd0);
      cha.d1 = scr<T>(H, L.chd1);
      hipLaunchKernelGGL((k_ca_chain<T>), dim3(1), dim3(kChainBlock), 0, ca.s, cha);
    } else {
      for (int k = k0; k < k1; ++k) ca_step(ca, k);
    }
    bool in_a = false;
    if (rec && !chain) {
      const int la = int(ca.rec->size());
      const int fin_a = std::max(tb, la + cs_ops) + 1 + kc * fu_ops;
      const int fin_b = std::max(tb, la) + cs_ops + 1 + kc * fu_ops;
      in_a = H.mj_place == 2 || (H.mj_place == 0 && fin_a < fin_b);
      tb = in_a ? fin_a : fin_b;
    }
    if (in_a) current_solve(ca, k0, kc, mr, md0, md1);
    mark(c, rec ? int(ca.rec->size()) : 0);
    if (!chain && !in_a) current_solve(c, k0, kc, mr2, md02, md12);
    {
      Seg<T> sg[3] = {seg<T>(H.Zj, 0, k0, 1, yj + int64_t(k0) * nj, nj, 0, 0, kc, -1.0),
                      seg<T>(H.Zj, 1, k0, 1, yA + int64_t(k0) * na, na, 0, 0, kc, -1.0),
                      seg<T>(H.Zj, 2, 0, 0, xp + int64_t(k0) * np, np, 0, 0, kc, 1.0)};
      spmv<T, T>(c, H.Zj, kc, 3, sg, ru + int64_t(k0) * nu, nu, 1.0, yu + int64_t(k0) * nu, nu);
    }
    for (int k = k0; k < k1; ++k) fu_step(c, k);
  }
  // 4. join with the pressure normalisation 1^T M_p p = 0
  mark(c, rec ? int(ca.rec->size()) : 0);
  slab_sums_t<T>(c, xp, int64_t(np), np, H.mp_rowsum, psum + nt, nt);
  {
    JoinArgs<T> a{z, ns, nt, o2, o3, o4, xu, xp, -1.0, psum + nt, H.msum, yj, yA, zslot};
    emit(c, kKJoin, dim3(grid_for(int64_t(ns) * nt)), &k_join<T>, a);
  }
  return ST_OK;
}

// ================================================ P_T^{-T} (adjoint) ====
// z = P_T^{-T} r: the backward F_u^T sweep first, then the pressure part and,
// slab by slab, the current and the backward C_A^T sweep.  As for the forward
// apply, `ca` receives program a (split, the F_u^T sweep chunk by chunk from
// the last slab, then the pressure part) and `c` program b (per chunk, once
// that chunk of x_u is done: y_j = M_j^{-1}(r_j - Z_j^T x_u), the right-hand
// side h = r_A - Z_A^T x_u - K_jA^T y_j and the C_A^T sweep; then F_A^T, M_A^{-1}
// and, after all of a, the join).  Not recording, both are the caller's stream.
template <class T>
int precond_transpose(Handle& H, const double* r, double* z, Ctx& c, Ctx& ca, const double* const* rslot = nullptr,
                      double* const* zslot = nullptr) {
  if (!H.adjoint) return ST_EINVAL;
  const Dims& d = H.d;
  const int nt = d.nt;
  char* B = H.base;
  const WsLayout& L = H.L;
  T* ru = scr<T>(H, L.ru); T* xu = scr<T>(H, L.xu);
  T* rp = scr<T>(H, L.rp); T* q = scr<T>(H, L.q); T* t = scr<T>(H, L.t); T* xp = scr<T>(H, L.xp);
  T* rj = scr<T>(H, L.rj); T* yj = scr<T>(H, L.yj);
  T* ra = scr<T>(H, L.ra); T* cA = scr<T>(H, L.wA); T* f = scr<T>(H, L.sA); T* yA = scr<T>(H, L.yA);
  T* mr = scr<T>(H, L.mr); T* md0 = scr<T>(H, L.md0); T* md1 = scr<T>(H, L.md1);
  T* mr2 = scr<T>(H, L.mr2); T* md02 = scr<T>(H, L.md02); T* md12 = scr<T>(H, L.md12);
  double* psum = scr<double>(H, L.psum);
  const int o2 = d.off[2], o3 = d.off[3], o4 = d.off[4], ns = d.ns;
  const int nu = d.nu, np = d.np, nj = d.nj, na = d.na;
  const double dt = H.dt;
  const int vc = H.exact ? H.inner_iters : 1;
  const int mit = H.mass_iters;
  const double mlo = 0.24, mhi = 2.3, mth = 0.5 * (mhi + mlo), mde = 0.5 * (mhi - mlo);
  const bool rec = c.recording();
  const int C = rec ? std::max(1, std::min(H.chunk, nt)) : nt;
  const int nch = (nt + C - 1) / C;
  auto mark = [&](Ctx& cx, int need) { cx.need = need; };

  slab_sums_d(ca, r, int64_t(ns), o2, np, nullptr, psum, nt, rslot);
  {
    SplitArgs<T> a{r, ns, nt, o2, o3, o4, psum, ru, rp, rj, ra, rslot};
    emit(ca, kKSplit, dim3(grid_for(int64_t(ns) * nt)), &k_split<T>, a);
  }
  // x_u = F_u^{-T} r_u, backward in time: F_uk^T x^k = r^k + (1/dt) M_u x^{k+1};
  // chunk ch holds slabs [k0, k1) counted from the last one.
  std::vector<int> a_end(size_t(nch), 0);
  auto chunk = [&](int ch, int& k0, int& k1) {
    k1 = nt - ch * C;
    k0 = std::max(0, k1 - C);
  };
  for (int ch = 0; ch < nch; ++ch) {
    int k0, k1;
    chunk(ch, k0, k1);
    for (int k = k1 - 1; k >= k0; --k) {
      Seg<T> sg = seg<T>(H.Mu, 0, 0, 0, xu + int64_t(k + 1) * nu, 0, 0, 0, 1, 1.0 / dt);
      if (H.use_stencil && H.fu_deg > 0)
        sweep_step_stencil<T>(ca, H, H.amgFuT, H.sFuT, k + 1 < nt ? &H.sAuT : nullptr, k, -1.0,
                              xu + int64_t(k + 1) * nu, nullptr, 0, 0.0, nullptr, ru + int64_t(k) * nu,
                              xu + int64_t(k) * nu, k, H.fu_deg, 1, k + 1 < nt, 1.0, 0.0);
      else
        sweep_step<T>(ca, H.amgFuT, H.Mu, k + 1 < nt ? 1 : 0, &sg, ru + int64_t(k) * nu, xu + int64_t(k) * nu, k,
                      H.fu_deg, vc);
    }
    a_end[size_t(ch)] = rec ? int(ca.rec->size()) : 0;
  }
  // x_p = S_p^{-T}(r_p - B x_u),  S_p^{-T} = -K_p^{-1} F_p^T M_p^{-1}  (program a)
  spmv1<T>(ca, H.B, nt, 0, 0, xu, nu, -1.0, rp, 1.0, rp, np);
  slab_sums_t<T>(ca, rp, int64_t(np), np, nullptr, psum, nt);
  slab_shift<T>(ca, rp, int64_t(np), np, nt, psum, 1.0 / np);
  cheb_solve<T>(ca, H.Mp, nt, 0, 0, static_cast<const T*>(H.dMp), 0, nullptr, mth, mde, rp, q, mr, md0, md1, np,
                mit, 0, false);
  {
    Seg<T> sg[2] = {seg<T>(H.Fpt, 0, 0, 1, q, np, 0, 0, nt, 1.0), seg<T>(H.Fpt, 1, 0, 0, q, np, 1, 0, nt - 1, 1.0)};
    spmv<T, T>(ca, H.Fpt, nt, 2, sg, nullptr, np, 0.0, t, np);
  }
  slab_sums_t<T>(ca, t, int64_t(np), np, nullptr, psum, nt);
  slab_shift<T>(ca, t, int64_t(np), np, nt, psum, 1.0 / np);
  amg_solve<T>(ca, H.amgKp, nt, 0, 0, xp, t, vc);
  const int a_all = rec ? int(ca.rec->size()) : 0;
  // per chunk (program b): y_j = M_j^{-1}(r_j - Z_j^T x_u); h = r_A - Z_A^T x_u -
  // K_jA^T y_j (in ra); c = C_A^{-T} h backward:
  // C0_k^T c^k = h^k + (1/dt) C1_k^T c^{k+1} - (1/dt^2) C2^T c^{k+2}
  for (int ch = 0; ch < nch; ++ch) {
    int k0, k1;
    chunk(ch, k0, k1);
    const int kc = k1 - k0;
    mark(c, a_end[size_t(ch)]);
    spmv1<T>(c, H.Zjt, kc, k0, 1, xu + int64_t(k0) * nu, nu, -1.0, rj + int64_t(k0) * nj, 1.0,
             rj + int64_t(k0) * nj, nj);
    cheb_solve<T>(c, H.Mj, kc, 0, 0, static_cast<const T*>(H.dMj), 0, nullptr, mth, mde, rj + int64_t(k0) * nj,
                  yj + int64_t(k0) * nj, mr2 + int64_t(k0) * nj, md02 + int64_t(k0) * nj, md12 + int64_t(k0) * nj, nj,
                  mit, 0, false);
    spmv1<T>(c, H.ZAt, kc, k0, 1, xu + int64_t(k0) * nu, nu, -1.0, ra + int64_t(k0) * na, 1.0,
             ra + int64_t(k0) * na, na);
    spmv1<T>(c, H.KjAt, kc, 0, 0, yj + int64_t(k0) * nj, nj, -1.0, ra + int64_t(k0) * na, 1.0,
             ra + int64_t(k0) * na, na);
    for (int k = k1 - 1; k >= k0; --k) {
      Seg<T> sg[2];
      int nsg = 0;
      if (k + 1 < nt) sg[nsg++] = seg<T>(H.C1t, 0, k, 0, cA + int64_t(k + 1) * na, 0, 0, 0, 1, 1.0 / dt);
      if (k + 2 < nt) sg[nsg++] = seg<T>(H.C1t, 1, 0, 0, cA + int64_t(k + 2) * na, 0, 0, 0, 1, -1.0 / (dt * dt));
      if (H.use_stencil && H.ca_deg > 0)
        sweep_step_stencil<T>(c, H, H.amgC0T, H.sC0T, k + 1 < nt ? &H.sCPT : nullptr, k, 1.0,
                              cA + int64_t(k + 1) * na, k + 2 < nt ? &H.sCQT : nullptr, k, 1.0,
                              cA + int64_t(k + 2) * na, ra + int64_t(k) * na, cA + int64_t(k) * na, k, H.ca_deg, 2,
                              k + 1 < nt, k + 2 < nt ? 2.0 : 1.0, k + 2 < nt ? -1.0 : 0.0);
      else
        sweep_step<T>(c, H.amgC0T, H.C1t, nsg, sg, ra + int64_t(k) * na, cA + int64_t(k) * na, k, H.ca_deg, vc);
    }
  }
  // f = F_A^T c; y_A = M_A^{-1} f
  {
    Seg<T> sg[2] = {seg<T>(H.FAt, 0, 0, 1, cA, na, 0, 0, nt, 1.0), seg<T>(H.FAt, 1, 0, 0, cA, na, 1, 0, nt - 1, 1.0)};
    spmv<T, T>(c, H.FAt, nt, 2, sg, nullptr, na, 0.0, f, na);
  }
  cheb_solve<T>(c, H.MA, nt, 0, 0, static_cast<const T*>(H.dMA), 0, nullptr, mth, mde, f, yA, mr2, md02, md12, na,
                mit, 0, false);
  // join with the pressure normalisation, once program a is done
  mark(c, a_all);
  slab_sums_t<T>(c, xp, int64_t(np), np, H.mp_rowsum, psum + nt, nt);
  {
    JoinArgs<T> a{z, ns, nt, o2, o3, o4, xu, xp, -1.0, psum + nt, H.msum, yj, yA, zslot};
    emit(c, kKJoin, dim3(grid_for(int64_t(ns) * nt)), &k_join<T>, a);
  }
  return ST_OK;
}

// Records P_T^{-1} (or P_T^{-T}) as programs a and b reading r, z from the slots.
int record_precond(Handle& H, Program& prog, const double* const* rslot, double* const* zslot,
                   bool transpose = false) {
  Ctx cb{nullptr, &prog.b, &prog.dep, 0};
  Ctx ca{nullptr, &prog.a, nullptr, 0};
  if (transpose)
    return H.fp32 ? precond_transpose<float>(H, nullptr, nullptr, cb, ca, rslot, zslot)
                  : precond_transpose<double>(H, nullptr, nullptr, cb, ca, rslot, zslot);
  return H.fp32 ? precond_forward<float>(H, nullptr, nullptr, cb, ca, rslot, zslot)
                : precond_forward<double>(H, nullptr, nullptr, cb, ca, rslot, zslot);
}

// Replay of the recorded forward P_T^{-1} on stream s.
// =============================== P and P-tilde (eqs. (preconditioner), ===
// (preconditionerSimplified1)), step by step on one stream:
//   P^{-1}      = Utilde_up^{-1} L_up^{-1} Ubar_ujA^{-1} L_ujA^{-1},
//   Ptilde^{-1} = Utilde_up^{-1} L_up^{-1} Ubar_ujA^{-1},
// with L_ujA^{-1}: x_A += Y F_u^{-1}(Z_j M_j^{-1} x_j - x_u) (step 1 of the paper's
// application of P) and L_up^{-1}: y_p -= B F_u^{-1} y_u (eq. (PupLU)); the
// Ubar_ujA and Utilde_up parts are P_T's.  Every F_u^{-1} is a whole forward
// sweep (the same sweep steps as P_T's).
template <class T>
void fu_sweep_all(Ctx& c, Handle& H, const T* q, T* x) {
  const int nt = H.d.nt, nu = H.d.nu;
  const int vc = H.exact ? H.inner_iters : 1;
  const double dt = H.dt;
  for (int k = 0; k < nt; ++k) {
    if (H.use_stencil && H.fu_deg > 0) {
      sweep_step_stencil<T>(c, H, H.amgFu, H.sFu, k >= 1 ? &H.sAu : nullptr, k, -1.0, x + int64_t(k - 1) * nu,
                            nullptr, 0, 0.0, nullptr, q + int64_t(k) * nu, x + int64_t(k) * nu, k, H.fu_deg, 1,
                            k >= 1, 1.0, 0.0);
    } else {
      Seg<T> sg = seg<T>(H.Mu, 0, 0, 0, x + int64_t(k - 1) * nu, 0, 0, 0, 1, 1.0 / dt);
      sweep_step<T>(c, H.amgFu, H.Mu, k >= 1 ? 1 : 0, &sg, q + int64_t(k) * nu, x + int64_t(k) * nu, k, H.fu_deg,
                    vc);
    }
  }
}

template <class T>
int precond_variant(Handle& H, const double* r, double* z, Ctx& c) {
  const Dims& d = H.d;
  const int nt = d.nt;
  char* B = H.base;
  const WsLayout& L = H.L;
  T* ru = scr<T>(H, L.ru); T* yu = scr<T>(H, L.yu); T* xu = scr<T>(H, L.xu);
  T* rp = scr<T>(H, L.rp); T* q = scr<T>(H, L.q); T* t = scr<T>(H, L.t); T* xp = scr<T>(H, L.xp);
  T* rj = scr<T>(H, L.rj); T* yj = scr<T>(H, L.yj);
  T* ra = scr<T>(H, L.ra); T* w = scr<T>(H, L.wA); T* sA = scr<T>(H, L.sA); T* yA = scr<T>(H, L.yA);
  T* mr = scr<T>(H, L.mr); T* md0 = scr<T>(H, L.md0); T* md1 = scr<T>(H, L.md1);
  double* psum = scr<double>(H, L.psum);
  const int o2 = d.off[2], o3 = d.off[3], o4 = d.off[4], ns = d.ns;
  const int nu = d.nu, np = d.np, nj = d.nj, na = d.na;
  const double dt = H.dt;
  const int vc = H.exact ? H.inner_iters : 1;
  const int mit = H.mass_iters;
  const double mlo = 0.24, mhi = 2.3, mth = 0.5 * (mhi + mlo), mde = 0.5 * (mhi - mlo);
  // split r, the pressure rows projected to zero sum per slab
  slab_sums_d(c, r, int64_t(ns), o2, np, nullptr, psum, nt);
  {
    SplitArgs<T> a{r, ns, nt, o2, o3, o4, psum, ru, rp, rj, ra, nullptr};
    emit(c, kKSplit, dim3(grid_for(int64_t(ns) * nt)), &k_split<T>, a);
  }
  auto mj_solve = [&](const T* rhs, T* out) {
    cheb_solve<T>(c, H.Mj, nt, 0, 0, static_cast<const T*>(H.dMj), 0, nullptr, mth, mde, rhs, out, mr, md0, md1,
                  nj, mit, 0, false);
  };
  if (H.variant == 2) {
    // L_ujA^{-1}: t_j = M_j^{-1} x_j; s = F_u^{-1}(Z_j t_j - x_u); x_A += Y s
    mj_solve(rj, yj);
    Seg<T> sz = seg<T>(H.Zj, 0, 0, 1, yj, nj, 0, 0, nt, 1.0);
    spmv<T, T>(c, H.Zj, nt, 1, &sz, ru, nu, -1.0, yu, nu);
    fu_sweep_all<T>(c, H, yu, xu);
    spmv1<T>(c, H.Yv, nt, 0, 1, xu, nu, 1.0, ra, 1.0, ra, na);
  }
  // Ubar_ujA^{-1}: y_A = C_A^{-1} F_A M_A^{-1} x_A; y_j = M_j^{-1}(x_j - K_jA y_A);
  // y_u = x_u - Z_j y_j - Z_A y_A
  cheb_solve<T>(c, H.MA, nt, 0, 0, static_cast<const T*>(H.dMA), 0, nullptr, mth, mde, ra, w, mr, md0, md1, na, mit,
                0, false);
  {
    Seg<T> sg[2] = {seg<T>(H.FA, 0, 0, 1, w, na, 0, 0, nt, 1.0), seg<T>(H.FA, 1, 0, 0, w, na, -1, 1, nt, 1.0)};
    spmv<T, T>(c, H.FA, nt, 2, sg, nullptr, na, 0.0, sA, na);
  }
  for (int k = 0; k < nt; ++k) {
    if (H.use_stencil && H.ca_deg > 0) {
      sweep_step_stencil<T>(c, H, H.amgC0, H.sC0, k >= 1 ? &H.sCP : nullptr, k, 1.0, yA + int64_t(k - 1) * na,
                            k >= 2 ? &H.sCQ : nullptr, k, 1.0, yA + int64_t(k - 2) * na, sA + int64_t(k) * na,
                            yA + int64_t(k) * na, k, H.ca_deg, 2, k >= 1, k >= 2 ? 2.0 : 1.0, k >= 2 ? -1.0 : 0.0);
    } else {
      Seg<T> sg[2];
      int nsg = 0;
      if (k >= 1) sg[nsg++] = seg<T>(H.C1, 0, k - 1, 0, yA + int64_t(k - 1) * na, 0, 0, 0, 1, 1.0 / dt);
      if (k >= 2) sg[nsg++] = seg<T>(H.C1, 1, 0, 0, yA + int64_t(k - 2) * na, 0, 0, 0, 1, -1.0 / (dt * dt));
      sweep_step<T>(c, H.amgC0, H.C1, nsg, sg, sA + int64_t(k) * na, yA + int64_t(k) * na, k, H.ca_deg, vc);
    }
  }
  spmv1<T>(c, H.KjA, nt, 0, 0, yA, na, -1.0, rj, 1.0, rj, nj);
  mj_solve(rj, yj);
  {
    Seg<T> sg[2] = {seg<T>(H.Zj, 0, 0, 1, yj, nj, 0, 0, nt, -1.0), seg<T>(H.Zj, 1, 0, 1, yA, na, 0, 0, nt, -1.0)};
    spmv<T, T>(c, H.Zj, nt, 2, sg, ru, nu, 1.0, yu, nu);
  }
  // L_up^{-1}: y_p = x_p - B F_u^{-1} y_u
  fu_sweep_all<T>(c, H, yu, xu);
  spmv1<T>(c, H.Bv, nt, 0, 0, xu, nu, -1.0, rp, 1.0, rp, np);
  // Utilde_up^{-1}: x_p = -M_p^{-1} F_p K_p^{-1} y_p (xp holds M_p^{-1} F_p q);
  // x_u = F_u^{-1}(y_u - B^T x_p)
  amg_solve<T>(c, H.amgKp, nt, 0, 0, q, rp, vc);
  {
    Seg<T> sg[2] = {seg<T>(H.Fp, 0, 0, 1, q, np, 0, 0, nt, 1.0), seg<T>(H.Fp, 1, 0, 0, q, np, -1, 1, nt, 1.0)};
    spmv<T, T>(c, H.Fp, nt, 2, sg, nullptr, np, 0.0, t, np);
  }
  cheb_solve<T>(c, H.Mp, nt, 0, 0, static_cast<const T*>(H.dMp), 0, nullptr, mth, mde, t, xp, mr, md0, md1, np, mit,
                0, false);
  spmv1<T>(c, H.Bt, nt, 0, 0, xp, np, 1.0, yu, 1.0, yu, nu);
  fu_sweep_all<T>(c, H, yu, xu);
  slab_sums_t<T>(c, xp, int64_t(np), np, H.mp_rowsum, psum + nt, nt);
  {
    JoinArgs<T> a{z, ns, nt, o2, o3, o4, xu, xp, -1.0, psum + nt, H.msum, yj, yA, nullptr};
    emit(c, kKJoin, dim3(grid_for(int64_t(ns) * nt)), &k_join<T>, a);
  }
  (void)B;
  return ST_OK;
}

int replay_precond(Handle& H, const double* r, double* z, hipStream_t s, bool transpose = false) {
  SetPtrsArgs sp{H.rslot, H.zslot, r, z};
  hipLaunchKernelGGL(k_set_ptrs, dim3(1), dim3(kBlock), 0, s, sp);
  for (ReplayItem& it : transpose ? H.pt_items_t : H.pt_items) {
    void* params[] = {it.args};
    const bool timed = H.prof_fn && it.fn == H.prof_fn && (H.prof_seen++ % H.prof_every) == 0 &&
                       H.prof_used + 2 <= H.prof_ev.size();
    if (timed) {
      // the events take the dispatch's own start and end times (no extra
      // packets between launches, which would break their back-to-back issue)
      (void)hipExtLaunchKernel(it.fn, it.grid, dim3(unsigned(it.block)), params, 0, s, H.prof_ev[H.prof_used],
                               H.prof_ev[H.prof_used + 1], 0);
      H.prof_used += 2;
    } else {
      (void)hipLaunchKernel(it.fn, it.grid, dim3(unsigned(it.block)), params, 0, s);
    }
  }
  return ST_OK;
}

// Adds the sampled kernel durations recorded so far (the stream is synchronised
// by the caller) and frees the pool for the next solve.
void profile_harvest(Handle& H) {
  for (size_t i = 0; i + 1 < H.prof_used; i += 2) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, H.prof_ev[i], H.prof_ev[i + 1]) == hipSuccess) {
      H.prof_ms += ms;
      H.prof_n += 1;
    }
  }
  H.prof_used = 0;
}

int apply_precond(Handle& H, const double* r, double* z, Ctx& c, bool transpose) {
  if (H.variant != 0) {
    if (transpose || c.recording()) return ST_EINVAL;
    return H.fp32 ? precond_variant<float>(H, r, z, c) : precond_variant<double>(H, r, z, c);
  }
  if (H.pint > 0) {   // Parareal sweeps: forward, step by step
    if (transpose || c.recording()) return ST_EINVAL;
    return H.fp32 ? precond_forward<float>(H, r, z, c, c) : precond_forward<double>(H, r, z, c, c);
  }
  if (!c.recording() && (transpose ? H.pipeline_t : H.pipeline)) return replay_precond(H, r, z, c.s, transpose);
  if (H.fp32)
    return transpose ? precond_transpose<float>(H, r, z, c, c) : precond_forward<float>(H, r, z, c, c);
  return transpose ? precond_transpose<double>(H, r, z, c, c) : precond_forward<double>(H, r, z, c, c);
}

// y = alpha J x + beta b  (J or J^T), FP64.  With one lane per row the
// multi-slab kernel loads the slab-invariant indices and values once for
// several slabs.
void apply_J(Handle& H, const double* x, double* y, Ctx& c, bool transpose, double alpha, const double* b) {
  const DGroup& g = transpose ? H.JT : H.J;
  const int nt = H.d.nt, ns = H.d.ns;
  Seg<double> sg[3] = {
      seg<double>(g, 0, 0, 1, x, ns, 0, 0, nt, alpha),
      seg<double>(g, 1, 0, 0, x, ns, 0, 0, nt, alpha),
      transpose ? seg<double>(g, 2, 0, 0, x, ns, 1, 0, nt - 1, alpha) : seg<double>(g, 2, 0, 0, x, ns, -1, 1, nt, alpha)};
  const int nv = H.j_slabs == 0 ? 8 : H.j_slabs;
  if (g.lanes != 1 || nv == 1) {
    spmv<double, double>(c, g, nt, 3, sg, b, ns, b ? 1.0 : 0.0, y, ns, kRoleJ);
    return;
  }
  SpmvSlabsArgs a;
  std::memset(&a, 0, sizeof(a));
  a.a.perm = g.perm;
  a.a.nslices = g.nslices;
  a.a.lanes = 1;
  a.a.nseg = 3;
  for (int i = 0; i < 3; ++i) a.a.seg[i] = sg[i];
  a.a.b = b;
  a.a.bstride = ns;
  a.a.beta = b ? 1.0 : 0.0;
  a.a.y = y;
  a.a.ystride = ns;
  a.nvec = nt;
  a.nbx = (g.nslices + 3) / 4;
  a.nblk = a.nbx * ((nt + nv - 1) / nv);
  const dim3 grid(unsigned((a.nblk + 7) / 8 * 8));
  if (nv == 8) emit(c, kKSpmvSlabs8, grid, &k_spmv_slabs<8>, a);
  else emit(c, kKSpmvSlabs4, grid, &k_spmv_slabs<4>, a);
}

// ============================================================ FGMRES ===
// Device pointers of one system's Krylov workspace for restart length m.
struct Krylov {
  int64_t N = 0;
  int m = 0, ldh = 0;
  double *V = nullptr, *Z = nullptr, *w = nullptr, *bp = nullptr, *Hc = nullptr, *sm = nullptr;
  double *g = nullptr, *cs = nullptr, *sn = nullptr, *y = nullptr, *psum = nullptr, *partial = nullptr;
  double* dots = nullptr;   // 2m dot products of a delayed-reorthogonalisation step
  const double** rslot = nullptr;   // input/output slots of the recorded preconditioner
  double** zslot = nullptr;
};

Krylov krylov(Handle& H, int m) {
  Krylov K;
  char* B = H.base;
  const WsLayout& L = H.L;
  K.N = int64_t(H.d.nt) * H.d.ns;
  K.m = m;
  K.ldh = m + 1;
  K.V = at<double>(B, L.V);
  K.Z = at<double>(B, L.Z);
  K.w = at<double>(B, L.w);
  K.bp = at<double>(B, L.r);
  K.Hc = at<double>(B, L.hess);     // column j at Hc + j*(m+1)
  K.sm = at<double>(B, L.small);
  K.g = K.sm + 64;
  K.cs = K.g + (m + 2);
  K.sn = K.cs + (m + 2);
  K.y = K.sn + (m + 2);
  K.dots = at<double>(B, L.small) + 64 + 4 * (H.max_restart + 2);
  K.psum = at<double>(B, L.psum);
  K.partial = at<double>(B, L.partial);
  K.rslot = at<const double*>(B, L.io);
  K.zslot = at<double*>(B, L.io + sizeof(void*));
  return K;
}

// out[i] = V_i . w for i < nv (mode 0 set, 2 add); mode 1: out[0] = ||w||
void emit_dots(Ctx& c, const Krylov& K, const double* V, int nv, const double* w, double* out, int mode,
               double* copy_to = nullptr) {
  MdotArgs a{V, K.N, w, K.partial};
  emit(c, kKMdot, dim3(kPartialBlocks, nv), &k_mdot_partial, a);
  ReduceArgs r{K.partial, kPartialBlocks, out, mode, copy_to};
  emit(c, kKReduce, dim3(nv), &k_reduce, r);
}

// bp = b with the pressure rows projected per slab; sm[0] = ||bp||; x = 0 unless given.
void emit_fgmres_init(Ctx& c, Handle& H, const Krylov& K, const double* b, double* x, bool zero_x) {
  const Dims& d = H.d;
  slab_sums_d(c, b, int64_t(d.ns), d.off[2], d.np, nullptr, K.psum, d.nt);
  ProjectPArgs pa{b, K.bp, d.ns, d.nt, d.off[2], d.off[3], K.psum};
  emit(c, kKProjectP, dim3(grid_for(K.N)), &k_project_p, pa);
  emit_dots(c, K, K.bp, 1, K.bp, K.sm + 0, 1);
  if (zero_x) {
    FillArgs f{x, K.N, 0.0};
    emit(c, kKFill, dim3(grid_for(K.N)), &k_fill, f);
  }
}

// V_0 = bp - J x (unnormalised); sm[0] = ||V_0||.  The J apply goes through `jac`.
template <class JacFn>
void emit_residual(Ctx& c, const Krylov& K, double* x, JacFn&& jac) {
  jac(x, K.V, -1.0, K.bp);
  emit_dots(c, K, K.V, 1, K.V, K.sm + 0, 1);
}

// V_0 /= beta; g = (beta, 0, ...).
void emit_cycle_head(Ctx& c, const Krylov& K) {
  ScaleArgs s{K.V, K.V, K.N, K.sm + 0};
  emit(c, kKScale, dim3(grid_for(K.N)), &k_scale, s);
  InitGArgs ig{K.g, K.m + 1, K.sm + 0};
  emit(c, kKInitG, dim3(1), &k_init_g, ig);
}

// After w = J z_j: CGS2 against V_0..V_j, h_{j+1,j} = ||w|| (copied to sm[1]),
// the Givens update (estimate in sm[2]) and V_{j+1} = w / h_{j+1,j}.
void emit_arnoldi(Ctx& c, const Krylov& K, int j) {
  double* hcol = K.Hc + int64_t(j) * K.ldh;
  emit_dots(c, K, K.V, j + 1, K.w, hcol, 0);
  CombineArgs u1{K.w, K.V, K.N, hcol, j + 1, -1.0};
  emit(c, kKCombine, dim3(grid_for(K.N)), &k_combine, u1);
  emit_dots(c, K, K.V, j + 1, K.w, K.y, 0);
  CombineArgs u2{K.w, K.V, K.N, K.y, j + 1, -1.0};
  emit(c, kKCombine, dim3(grid_for(K.N)), &k_combine, u2);
  // H[:, j] += second-pass coefficients (one-element partials per entry)
  ReduceArgs add{K.y, 1, hcol, 2, nullptr};
  emit(c, kKReduce, dim3(j + 1), &k_reduce, add);
  emit_dots(c, K, K.w, 1, K.w, hcol + (j + 1), 1, K.sm + 1);
  GivensArgs gv{K.Hc, j, K.ldh, K.g, K.cs, K.sn, K.sm + 2};
  emit(c, kKGivens, dim3(1), &k_givens, gv);
  if (j + 1 < K.m) {
    ScaleArgs s{K.V + int64_t(j + 1) * K.N, K.w, K.N, K.sm + 1};
    emit(c, kKScale, dim3(grid_for(K.N)), &k_scale, s);
  }
}

// Arnoldi step j with delayed reorthogonalisation (see the kernels): after
// w = J z_j, the dot pass over V_0..V_{j-1} with u_j = V_j and w, then the
// update pass writing q~ over V_j and w'' to V_{j+1}, and the Hessenberg
// entries (column j-1 completed, column j's first pass).  Without w (the
// closing pass of a cycle) only u_j = V_j is reorthogonalised and measured.
void emit_delayed_passes(Ctx& c, const Krylov& K, int j, const double* w) {
  double* u = K.V + int64_t(j) * K.N;
  if (j > 0) {
    Mdot2Args a{K.V, K.N, j, u, w, K.partial};
    emit(c, kKMdot2, dim3(kPartialBlocks, (j + kDotGroup - 1) / kDotGroup), &k_mdot2, a);
    ReduceArgs r{K.partial, kPartialBlocks, K.dots, 0, nullptr};
    emit(c, kKReduce, dim3(2 * j), &k_reduce, r);
  }
  UpdDelayedArgs up{K.V, K.N, j, K.dots, u, w, w ? K.V + int64_t(j + 1) * K.N : nullptr, K.partial};
  emit(c, kKUpdDelayed, dim3(kPartialBlocks), &k_upd_delayed, up);
  ReduceArgs r2{K.partial, kPartialBlocks, K.sm + 5, 0, nullptr};
  emit(c, kKReduce, dim3(3), &k_reduce, r2);
  FinDelayedArgs f{K.dots, K.sm + 5, K.Hc, K.ldh, j, w ? 1 : 0, K.sm};
  emit(c, kKFinDelayed, dim3(1), &k_fin_delayed, f);
}

// Givens update of the completed column j (estimate in sm[2]).
void emit_givens(Ctx& c, const Krylov& K, int j) {
  GivensArgs gv{K.Hc, j, K.ldh, K.g, K.cs, K.sn, K.sm + 2};
  emit(c, kKGivens, dim3(1), &k_givens, gv);
}

// q_j = q~ / nu over V_j, then u_{j+1} = (w'' - c q_j) / s_{j+1} in V_{j+1}.
void emit_delayed_next(Ctx& c, const Krylov& K, int j) {
  NextDelayedArgs a{K.V + int64_t(j) * K.N, K.V + int64_t(j + 1) * K.N, K.N, K.sm, K.sm + 8 + ((j + 1) & 1)};
  emit(c, kKNextDelayed, dim3(grid_for(K.N)), &k_next_delayed, a);
}

// x += Z y with y from the rotated Hessenberg system of size mused.
void emit_cycle_end(Ctx& c, const Krylov& K, double* x, int mused) {
  TrisolveArgs ts{K.Hc, mused, K.ldh, K.g, K.y};
  emit(c, kKTrisolve, dim3(1), &k_trisolve, ts);
  CombineArgs u{x, K.Z, K.N, K.y, mused, 1.0};
  emit(c, kKCombine, dim3(grid_for(K.N)), &k_combine, u);
}

// Pressure of x normalised per slab: 1^T M_p p^k = 0.
void emit_finalize(Ctx& c, Handle& H, const Krylov& K, double* x) {
  const Dims& d = H.d;
  slab_sums_d(c, x, int64_t(d.ns), d.off[2], d.np, H.mp_rowsum, K.psum, d.nt);
  slab_shift<double>(c, x + d.off[2], int64_t(d.ns), d.np, d.nt, K.psum, 1.0 / H.msum);
}

// Begin/end events recorded around each J or P_T apply of a solve, on the
// solve's stream; the destructor releases them on every return path.
struct EventPairs {
  hipStream_t s;
  std::vector<hipEvent_t> v;
  explicit EventPairs(hipStream_t st) : s(st) {}
  EventPairs(const EventPairs&) = delete;
  EventPairs& operator=(const EventPairs&) = delete;
  ~EventPairs() {
    for (hipEvent_t e : v)
      if (e) (void)hipEventDestroy(e);
  }
  void mark() {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) e = nullptr;
    if (e) (void)hipEventRecord(e, s);
    v.push_back(e);
  }
  void begin() { mark(); }
  void end() { mark(); }
  int pairs() const { return int(v.size() / 2); }
  // Sum of the pairs' durations (stream synchronised by the caller).
  double elapsed_ms() const {
    double acc = 0.0;
    for (size_t i = 0; i + 1 < v.size(); i += 2) {
      float ms = 0.f;
      if (v[i] && v[i + 1] && hipEventElapsedTime(&ms, v[i], v[i + 1]) == hipSuccess) acc += ms;
    }
    return acc;
  }
};

int fgmres(Handle& H, const double* b_in, double* x, const st_opts* o, st_info* info, hipStream_t s, bool adjoint) {
  auto t0 = std::chrono::steady_clock::now();
  const int m = o->restart > 0 ? o->restart : 30;
  if (m > H.max_restart) return ST_EINVAL;
  if (adjoint && !H.adjoint) return ST_EINVAL;
  const int maxit = o->maxit > 0 ? o->maxit : 1000;
  if (o->orth < 0 || o->orth > 2) return ST_EINVAL;
  const Krylov K = krylov(H, m);
  const bool delayed = o->orth == 2 || (o->orth == 0 && (m > kDelayedFrom || K.N >= kDelayedRows));
  Ctx c{s, nullptr};
  double* hs = H.host_small;
  EventPairs evs(s), jevs(s);
  auto jac = [&](const double* xin, double* yout, double alpha, const double* bb) {
    jevs.begin();
    apply_J(H, xin, yout, c, adjoint, alpha, bb);
    jevs.end();
  };
  auto precond = [&](const double* r, double* z) {
    evs.begin();
    apply_precond(H, r, z, c, adjoint);
    evs.end();
  };
  auto fetch = [&](const double* dev, int count) -> int {
    if (hipMemcpyAsync(hs, dev, sizeof(double) * count, hipMemcpyDeviceToHost, s) != hipSuccess) return ST_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return ST_EHIP;
    return ST_OK;
  };
  emit_fgmres_init(c, H, K, b_in, x, !o->x0_given);
  int rc = fetch(K.sm, 1);
  if (rc) return rc;
  const double bnorm = hs[0];
  if (!std::isfinite(bnorm)) return ST_EBREAKDOWN;
  const double tol = std::max(o->rtol * bnorm, o->atol);
  info->iterations = 0;
  info->restarts = 0;
  info->converged = 0;
  int its = 0, status = ST_ENOTCONV;
  double true_res = 0.0;
  if (bnorm == 0.0) {
    FillArgs f{x, K.N, 0.0};
    emit(c, kKFill, dim3(grid_for(K.N)), &k_fill, f);
    HIP_TRY(hipStreamSynchronize(s));
    info->converged = 1;
    info->true_rel_residual = 0.0;
    return ST_OK;
  }
  for (;;) {
    emit_residual(c, K, x, jac);
    rc = fetch(K.sm, 1);
    if (rc) return rc;
    const double beta = hs[0];
    true_res = beta;
    if (!std::isfinite(beta)) return ST_EBREAKDOWN;
    if (beta <= tol) {
      status = ST_OK;
      break;
    }
    if (its >= maxit) break;
    if (o->history && its < o->history_len && its == 0) o->history[0] = beta / bnorm;
    emit_cycle_head(c, K);
    int mused = 0;
    // a finished Hessenberg column: count it, record and test the estimate
    auto column_done = [&](int cols, bool& stop) -> int {
      const int rc2 = fetch(K.sm, 3);
      if (rc2) return rc2;
      ++its;
      mused = cols;
      const double est = hs[2];
      if (o->history && its < o->history_len) o->history[its] = est / bnorm;
      if (!std::isfinite(est) || !std::isfinite(hs[1])) return ST_EBREAKDOWN;
      stop = est <= tol || its >= maxit;
      return ST_OK;
    };
    bool stop = false;
    for (int j = 0; j < m && !stop; ++j) {
      precond(K.V + int64_t(j) * K.N, K.Z + int64_t(j) * K.N);
      jac(K.Z + int64_t(j) * K.N, K.w, 1.0, nullptr);
      if (!delayed) {
        emit_arnoldi(c, K, j);
        if ((rc = column_done(j + 1, stop))) return rc;
        continue;
      }
      // column j-1 completes in this step; z_j is unused if the solve stops here
      emit_delayed_passes(c, K, j, K.w);
      if (j > 0) {
        emit_givens(c, K, j - 1);
        if ((rc = column_done(j, stop))) return rc;
        if (stop) break;
      }
      emit_delayed_next(c, K, j);
    }
    if (delayed && !stop) {
      // closing pass: u_m against V_0..V_{m-1} completes column m-1
      emit_delayed_passes(c, K, m, nullptr);
      emit_givens(c, K, m - 1);
      if ((rc = column_done(m, stop))) return rc;
    }
    emit_cycle_end(c, K, x, mused);
    info->restarts++;
  }
  emit_finalize(c, H, K, x);
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipGetLastError());
  if (H.prof_fn) profile_harvest(H);
  const double pms = evs.elapsed_ms(), jms = jevs.elapsed_ms();
  info->precond_calls = evs.pairs();
  info->jacobian_calls = jevs.pairs();
  info->jacobian_seconds = jms * 1e-3;
  info->iterations = its;
  info->converged = status == ST_OK ? 1 : 0;
  info->true_rel_residual = true_res / bnorm;
  info->precond_seconds = pms * 1e-3;
  info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return status;
}

// ---------------------------------------------- sequential time stepping ---
// The slabs solved one after the other (Sec. "Comparison with sequential
// time-stepping"): slab k from its single-step Jacobian with FGMRES
// right-preconditioned by the single-step P_{T,k} of eq. (PTTS), which is P_T
// of a one-slab system, so hs[k] is a one-slab handle of slab k's state:
//   J_k x^k = b^k + diag(M_u/dt, 0, 0, M_A/dt) x^{k-1}.
// A handle of W > 1 slabs makes step k a window of W slabs solved all at once
// with its own P_T (windowed space-time), coupled to the previous window's
// last slab the same way.  Window k of W_k slabs stops on
// ||r_k|| <= max(rtol ||b||, atol) sqrt(W_k / Nt) (the window residuals are
// the rows of the space-time residual, so the whole x meets the space-time
// tolerance).  With o->x0_given every slab of a window starts from the
// previous window's last slab.
int timestep_solve(st_handle* const* hs, int nt, const double* b, double* x, const st_opts* o, st_info* infos,
                   hipStream_t s) {
  const Dims& d0 = hs[0]->h.d;
  const int ns = d0.ns;
  // window k holds slabs [first[k], first[k] + W_k) of the horizon
  std::vector<int64_t> first(size_t(nt) + 1, 0);
  for (int k = 0; k < nt; ++k) {
    const Dims& d = hs[k]->h.d;
    if (d.nt < 1 || d.ns != ns || d.n != d0.n) return ST_EINVAL;
    for (int i = 0; i < 6; ++i)
      if (d.off[i] != d0.off[i]) return ST_EINVAL;
    first[size_t(k) + 1] = first[size_t(k)] + d.nt;
  }
  const double total = double(first[size_t(nt)]);
  const int m = o->restart > 0 ? o->restart : 30;
  Ctx c{s, nullptr};
  // ||b|| with every slab's pressure rows projected to zero sum
  double bb = 0.0;
  for (int k = 0; k < nt; ++k) {
    Handle& H = hs[k]->h;
    if (m > H.max_restart) return ST_EINVAL;
    const Krylov K = krylov(H, m);
    emit_fgmres_init(c, H, K, b + first[size_t(k)] * ns, x + first[size_t(k)] * ns, false);
    HIP_TRY(hipMemcpyAsync(H.host_small, K.sm, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (!std::isfinite(H.host_small[0])) return ST_EBREAKDOWN;
    bb += H.host_small[0] * H.host_small[0];
  }
  const double tol_all = std::max(o->rtol * std::sqrt(bb), o->atol);
  int status = ST_OK;
  for (int k = 0; k < nt; ++k) {
    Handle& H = hs[k]->h;
    const int w = H.d.nt;
    const Krylov K = krylov(H, m);
    const double* bk = b + first[size_t(k)] * ns;
    double* xk = x + first[size_t(k)] * ns;
    const double* rhs = bk;
    if (k > 0) {
      // rhs = b^k - J_{k,k-1} x^{k-1} on the window's first slab (its coupling to
      // the previous window's last slab), the window's other slabs as in b;
      // formed in handle k's Arnoldi work vector (FGMRES reads its right-hand
      // side only when it projects it, before its first Arnoldi step)
      const double* xprev = x + (first[size_t(k)] - 1) * ns;
      if (w > 1)
        HIP_TRY(hipMemcpyAsync(K.w + ns, bk + ns, sizeof(double) * size_t(w - 1) * ns, hipMemcpyDeviceToDevice, s));
      Seg<double> sg = seg<double>(H.J, 2, 0, 0, xprev, ns, 0, 0, 1, -1.0);
      spmv<double, double>(c, H.J, 1, 1, &sg, bk, ns, 1.0, K.w, ns, kRoleJ);
      rhs = K.w;
      if (o->x0_given)
        for (int j = 0; j < w; ++j)
          HIP_TRY(hipMemcpyAsync(xk + int64_t(j) * ns, xprev, sizeof(double) * ns, hipMemcpyDeviceToDevice, s));
    }
    st_opts ok = *o;
    ok.restart = m;
    ok.rtol = 0.0;
    ok.atol = tol_all * std::sqrt(double(w) / total);
    ok.x0_given = (o->x0_given && k > 0) ? 1 : 0;
    ok.history = nullptr;
    ok.history_len = 0;
    const int rc = fgmres(H, rhs, xk, &ok, &infos[k], s, false);
    if (rc < 0) return rc;
    if (rc == ST_ENOTCONV) status = ST_ENOTCONV;
  }
  return status;
}

// --------------------------------------------- lockstep scheduling ---
// One member's launches in a phase: program a, program b (op i waits for
// dep[i] a-ops), then b2 (after all of a).
struct LockProg {
  const std::vector<Member>* a = nullptr;
  const std::vector<Member>* b = nullptr;
  const std::vector<int>* dep = nullptr;
  const std::vector<Member>* b2 = nullptr;
};

// Lockstep schedule: launch t takes, for every member, its next a-op and its
// next b-op when that op's dependency was met by the a-ops of earlier
// launches.  fn(args, blocks) receives each launch.
template <class Fn>
int lockstep(const std::vector<LockProg>& progs, Fn&& fn) {
  const size_t n = progs.size();
  if (2 * n > size_t(kMaxMembers)) return ST_EINVAL;
  std::vector<size_t> ia(n, 0), ib(n, 0);
  for (;;) {
    MultiArgs a;
    std::memset(&a, 0, sizeof(a));
    int64_t total = 0;
    bool left = false;
    for (size_t i = 0; i < n; ++i) {
      const LockProg& p = progs[i];
      const size_t na = p.a ? p.a->size() : 0, nb1 = p.b ? p.b->size() : 0, nb2 = p.b2 ? p.b2->size() : 0;
      const size_t done = ia[i];
      if (ia[i] < na) {
        a.m[a.nmem++] = (*p.a)[ia[i]++];
        total += a.m[a.nmem - 1].blocks;
      }
      if (ib[i] < nb1 + nb2) {
        const size_t need = ib[i] < nb1 ? (p.dep ? size_t((*p.dep)[ib[i]]) : 0) : na;
        if (need > na) return ST_EINTERNAL;
        if (need <= done) {
          a.m[a.nmem++] = ib[i] < nb1 ? (*p.b)[ib[i]] : (*p.b2)[ib[i] - nb1];
          total += a.m[a.nmem - 1].blocks;
          ++ib[i];
        }
      }
      if (ia[i] < na || ib[i] < nb1 + nb2) left = true;
    }
    if (a.nmem == 0) {
      if (!left) return ST_OK;
      continue;   // only waiting b-ops: the a-op of this member ran in the previous launch
    }
    if (total > int64_t(0x7fffffff)) return ST_EINTERNAL;
    fn(a, unsigned(total));
  }
}

// Appends the argument blocks of `ops` to `pool` (the host image of a device
// region starting at dev) and returns their launch descriptors.
inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

std::vector<Member> place(const std::vector<Op>& ops, std::vector<unsigned char>& pool, const unsigned char* dev) {
  std::vector<Member> out;
  out.reserve(ops.size());
  for (const Op& op : ops) {
    const size_t off = align_up(pool.size(), 16);
    pool.resize(off + size_t(op.size));
    std::memcpy(pool.data() + off, op.args, size_t(op.size));
    Member mb;
    mb.args = dev ? dev + off : nullptr;
    mb.kind = op.kind;
    mb.blocks = op.gx * op.gy;
    mb.gx = op.gx;
    mb.pad = 0;
    out.push_back(mb);
  }
  return out;
}

// Builds the replay of a handle's recorded forward P_T^{-1} (st_create):
// launch t runs the next op of program a and the next op of program b whose
// dependency the earlier launches met; two ops with a paired kernel (sweep
// steps, SELL Chebyshev steps and SELL products) share one k_two launch,
// anything else runs through its own kernel.
template <class T, class X, class Y>
bool try_pair(const Op& x, const Op& y, ReplayItem& it) {
  if (x.kind != X::kind || y.kind != Y::kind) return false;
  static_assert(sizeof(TwoArgs<X, Y>) <= sizeof(ReplayItem::args), "paired arguments exceed a replay item");
  TwoArgs<X, Y> p;
  std::memset(&p, 0, sizeof(p));
  std::memcpy(&p.x, x.args, sizeof(p.x));
  std::memcpy(&p.y, y.args, sizeof(p.y));
  p.xblocks = x.gx * x.gy;
  p.xgx = x.gx;
  p.ygx = y.gx;
  it.fn = reinterpret_cast<const void*>(&k_two<X, Y>);
  it.grid = dim3(unsigned(p.xblocks + y.gx * y.gy));
  std::memset(it.args, 0, sizeof(it.args));
  std::memcpy(it.args, &p, sizeof(p));
  return true;
}

template <class T, class X>
bool try_pair_x(const Op& x, const Op& y, ReplayItem& it) {
  return try_pair<T, X, BodyStInit<T>>(x, y, it) || try_pair<T, X, BodyStCheb<T>>(x, y, it) ||
         try_pair<T, X, BodyCheb<T>>(x, y, it) || try_pair<T, X, BodySpmv<T>>(x, y, it);
}

template <class T>
bool pair_ops(const Op& x, const Op& y, ReplayItem& it) {
  if (x.kind == kKStSolve && y.kind == kKStSolve) {
    // two tiled solves: their own kernel, with its wider workgroups
    if (!try_pair<T, BodyStSolve<T>, BodyStSolve<T>>(x, y, it)) return false;
    it.fn = reinterpret_cast<const void*>(&k_two_solve<T>);
    it.block = kSolveBlock;
    return true;
  }
  return try_pair_x<T, BodyStInit<T>>(x, y, it) || try_pair_x<T, BodyStCheb<T>>(x, y, it) ||
         try_pair_x<T, BodyCheb<T>>(x, y, it) || try_pair_x<T, BodySpmv<T>>(x, y, it);
}

template <class T>
int build_items(std::vector<ReplayItem>& items, const Program& prog) {
  auto single = [&](const Op& op) {
    ReplayItem it;
    it.fn = op.fn;
    it.grid = dim3(unsigned(op.gx), unsigned(op.gy));
    it.block = block_of(op.kind);
    std::memset(it.args, 0, sizeof(it.args));
    std::memcpy(it.args, op.args, size_t(op.size));
    items.push_back(it);
  };
  const size_t na = prog.a.size(), nb = prog.b.size();
  size_t ia = 0, ib = 0;
  while (ia < na || ib < nb) {
    const size_t done = ia;
    const Op* x = ia < na ? &prog.a[ia++] : nullptr;
    const Op* y = nullptr;
    if (ib < nb) {
      if (size_t(prog.dep[ib]) > na) return ST_EINTERNAL;
      if (size_t(prog.dep[ib]) <= done) y = &prog.b[ib++];
    }
    if (!x && !y) return ST_EINTERNAL;
    ReplayItem it;
    if (x && y && pair_ops<T>(*x, *y, it)) {
      items.push_back(it);
      continue;
    }
    if (x) single(*x);
    if (y) single(*y);
  }
  return ST_OK;
}

int build_pipeline(Handle& H) {
  H.rslot = at<const double*>(H.base, H.L.io);
  H.zslot = at<double*>(H.base, H.L.io + sizeof(void*));
  for (int tr = 0; tr < (H.adjoint ? 2 : 1); ++tr) {
    Program prog;
    int rc = record_precond(H, prog, H.rslot, H.zslot, tr == 1);
    if (rc) return rc;
    std::vector<ReplayItem>& items = tr ? H.pt_items_t : H.pt_items;
    items.clear();
    rc = H.fp32 ? build_items<float>(items, prog) : build_items<double>(items, prog);
    if (rc) return rc;
    (tr ? H.pipeline_t : H.pipeline) = 1;
  }
  return ST_OK;
}

// =========================================================== autotune ===
// Times, on this system's own operators, the launch choices that leave every
// result bitwise the same, and keeps the fastest: slabs per wavefront of the
// J apply (when not given), rows per workgroup of the sweep step kernels, one
// launch per sweep step against the tiled multi-step solve, and the schedule
// of the recorded forward apply (first chunk, placement of the current
// solves).  The inputs
// are two zeroed Krylov columns (the kernels' timing does not depend on the
// values).
int autotune(Handle& H, hipStream_t s, bool pipeline) {
  const int64_t N = int64_t(H.d.ns) * H.d.nt;
  double* x = at<double>(H.base, H.L.V);
  double* y = x + N;
  if (hipMemsetAsync(x, 0, size_t(N) * sizeof(double), s) != hipSuccess) return ST_EHIP;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return ST_EHIP;
  Ctx c{s, nullptr};
  int rc = ST_OK;
  auto timed = [&](auto&& fn, int reps) -> float {
    fn();
    fn();
    (void)hipEventRecord(e0, s);
    for (int i = 0; i < reps; ++i) fn();
    (void)hipEventRecord(e1, s);
    float ms = 0.0f;
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = ST_EHIP;
    return ms / float(reps);
  };
  if (H.j_slabs == 0 && H.J.lanes == 1) {
    int best = 8;
    float tbest = 1e30f;
    for (int nv : {1, 4, 8}) {
      H.j_slabs = nv;
      const float t = timed([&] { apply_J(H, x, y, c, false, 1.0, nullptr); }, 5);
      if (t < tbest) {
        tbest = t;
        best = nv;
      }
    }
    H.j_slabs = best;
  }
  if (rc == ST_OK && H.use_stencil) {
    struct Cand { int fuse, rows, lanes; };
    const Cand cands[] = {{0, 64, 1}, {0, 128, 1}, {0, 256, 1}, {0, 64, 2}, {0, 128, 2}, {1, 0, 1}};
    Cand best = cands[0];
    float tbest = 1e30f;
    for (const Cand& cd : cands) {
      H.sweep_fuse = cd.fuse;
      H.step_rows = cd.rows;
      H.step_lanes = cd.lanes;
      if (pipeline && (rc = build_pipeline(H)) != ST_OK) break;
      const float t = timed([&] { (void)apply_precond(H, x, y, c, false); }, 4);
      if (rc != ST_OK) break;
      if (t < tbest) {
        tbest = t;
        best = cd;
      }
    }
    H.sweep_fuse = best.fuse;
    H.step_rows = best.rows;
    H.step_lanes = best.lanes;
    if (rc == ST_OK && pipeline) rc = build_pipeline(H);
  }
  // the recorded forward apply's schedule: size of the first chunk (how long
  // program b waits for the C_A sweep at the start) and where the current
  // solves go
  if (rc == ST_OK && pipeline) {
    const int C = std::max(1, std::min(H.chunk, H.d.nt));
    struct Sched { int first, place; };
    const Sched cands[] = {{0, 1}, {0, 0}, {C / 2, 1}, {C / 2, 0}, {C / 4, 1}, {C / 4, 0}};
    Sched best = cands[0];
    float tbest = 1e30f;
    for (const Sched& sc : cands) {
      if (sc.first < 0 || (sc.first > 0 && sc.first >= C)) continue;
      H.first_chunk = sc.first;
      H.mj_place = sc.place;
      if ((rc = build_pipeline(H)) != ST_OK) break;
      const float t = timed([&] { (void)apply_precond(H, x, y, c, false); }, 4);
      if (rc != ST_OK) break;
      if (t < tbest) {
        tbest = t;
        best = sc;
      }
    }
    H.first_chunk = best.first;
    H.mj_place = best.place;
    if (rc == ST_OK) rc = build_pipeline(H);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc == ST_OK && hipGetLastError() != hipSuccess) rc = ST_EHIP;
  return rc;
}

// ============================================================ batches ===
// Lockstep FGMRES over several systems.  Each system's launches are recorded
// once (the preconditioner as its two programs reading the Krylov column
// from the handle's slots, one Arnoldi tail per column j that also points the
// slots at the next column, the cycle head) and again per solve for the
// launches that name the caller's b and x.  A batched phase runs the lockstep
// schedule of every member's programs, one k_group (or, for two pairable
// kinds, one k_group2) launch per op kind of a step.
struct BatchSys {
  Handle* H = nullptr;
  Krylov K;
  std::vector<Member> pa, pb, head;
  std::vector<int> pdep;
  std::vector<std::vector<Member>> tail;   // per Krylov column j
  std::vector<Member> init, resid, fin;    // per solve (b, x)
  std::vector<std::vector<Member>> end;    // per solve, index mused - 1
};

struct Batch {
  std::vector<BatchSys> sys;
  int m = 30, fp32 = 0;
  size_t out_off = 0, static_off = 0, static_bytes = 0, dyn_off = 0, dyn_bytes = 0, ws_bytes = 0;
  char* base = nullptr;
  double* out = nullptr;                 // device [nsys][4]: gathered sm[0..2]
  double* host_out = nullptr;            // pinned
  unsigned char* staging = nullptr;      // pinned, dyn_bytes
  int64_t lock_launches = 0, sep_launches = 0;   // one Arnoldi step, lockstep vs one system at a time
};

// Static programs of every member; dev = device address of the static pool (null: sizing only).
int record_static(Batch& Bt, std::vector<unsigned char>& pool, const unsigned char* dev) {
  pool.clear();
  for (size_t s = 0; s < Bt.sys.size(); ++s) {
    BatchSys& S = Bt.sys[s];
    Handle& H = *S.H;
    S.K = krylov(H, Bt.m);
    const Krylov& K = S.K;
    Program prog;
    int rc = record_precond(H, prog, K.rslot, K.zslot);
    if (rc) return rc;
    S.pa = place(prog.a, pool, dev);
    S.pb = place(prog.b, pool, dev);
    S.pdep = prog.dep;
    std::vector<Op> ops;
    Ctx c{nullptr, &ops};
    emit_cycle_head(c, K);
    SetPtrsArgs sp0{K.rslot, K.zslot, K.V, K.Z};
    emit(c, kKSetPtrs, dim3(1), &k_set_ptrs, sp0);
    S.head = place(ops, pool, dev);
    S.tail.assign(size_t(Bt.m), {});
    for (int j = 0; j < Bt.m; ++j) {
      ops.clear();
      apply_J(H, K.Z + int64_t(j) * K.N, K.w, c, false, 1.0, nullptr);
      emit_arnoldi(c, K, j);
      CopySmallArgs cs{K.sm, Bt.out + 4 * s, 3};
      emit(c, kKCopySmall, dim3(1), &k_copy_small, cs);
      if (j + 1 < Bt.m) {
        SetPtrsArgs sp{K.rslot, K.zslot, K.V + int64_t(j + 1) * K.N, K.Z + int64_t(j + 1) * K.N};
        emit(c, kKSetPtrs, dim3(1), &k_set_ptrs, sp);
      }
      S.tail[size_t(j)] = place(ops, pool, dev);
    }
  }
  return ST_OK;
}

// Per-solve programs (they name b and x); dev = device address of the dynamic pool.
void record_dynamic(Batch& Bt, std::vector<unsigned char>& pool, const unsigned char* dev, const double* const* b,
                    double* const* x, bool zero_x) {
  pool.clear();
  for (size_t s = 0; s < Bt.sys.size(); ++s) {
    BatchSys& S = Bt.sys[s];
    Handle& H = *S.H;
    const Krylov& K = S.K;
    const double* bs = b ? b[s] : nullptr;
    double* xs = x ? x[s] : nullptr;
    std::vector<Op> ops;
    Ctx c{nullptr, &ops};
    emit_fgmres_init(c, H, K, bs, xs, zero_x);
    CopySmallArgs g0{K.sm, Bt.out + 4 * s, 3};
    emit(c, kKCopySmall, dim3(1), &k_copy_small, g0);
    S.init = place(ops, pool, dev);
    ops.clear();
    emit_residual(c, K, xs, [&](const double* xin, double* yout, double alpha, const double* bb) {
      apply_J(H, xin, yout, c, false, alpha, bb);
    });
    emit(c, kKCopySmall, dim3(1), &k_copy_small, g0);
    S.resid = place(ops, pool, dev);
    S.end.assign(size_t(Bt.m), {});
    for (int mu = 1; mu <= Bt.m; ++mu) {
      ops.clear();
      emit_cycle_end(c, K, xs, mu);
      S.end[size_t(mu - 1)] = place(ops, pool, dev);
    }
    ops.clear();
    emit_finalize(c, H, K, xs);
    S.fin = place(ops, pool, dev);
  }
}

// Grouped launches of one lockstep step: the ops are grouped by kind; two
// groups of pairable kinds share one k_group2 launch, every other group runs
// as one k_group launch of its kind.
template <class T, int... K>
void group_kernels(std::vector<const void*>& out, std::integer_sequence<int, K...>) {
  out = {reinterpret_cast<const void*>(&k_group<K, T>)...};
}

template <class T>
const void* group_kernel(int kind) {
  static std::vector<const void*> table;
  if (table.empty()) {
    group_kernels<T>(table, std::make_integer_sequence<int, kKNumKinds>{});
    table[size_t(kKStSolve)] = reinterpret_cast<const void*>(&k_group_solve<T>);
  }
  return table[size_t(kind)];
}

constexpr int kNumPairable = 4;
constexpr int kPairable[kNumPairable] = {kKStInit, kKStCheb, kKCheb, kKSpmvT};

template <class T, int I, int J>
const void* group2_entry() {
  return reinterpret_cast<const void*>(&k_group2<kPairable[I], kPairable[J], T>);
}

template <class T>
const void* group2_kernel(int i, int j) {   // i < j: indices into kPairable
  static const void* table[kNumPairable][kNumPairable] = {
      {nullptr, group2_entry<T, 0, 1>(), group2_entry<T, 0, 2>(), group2_entry<T, 0, 3>()},
      {nullptr, nullptr, group2_entry<T, 1, 2>(), group2_entry<T, 1, 3>()},
      {nullptr, nullptr, nullptr, group2_entry<T, 2, 3>()},
      {nullptr, nullptr, nullptr, nullptr}};
  return table[i][j];
}

inline int pairable_index(int kind) {
  for (int i = 0; i < kNumPairable; ++i)
    if (kPairable[i] == kind) return i;
  return -1;
}

template <class T>
void launch_groups(const MultiArgs& step, hipStream_t s) {
  int kinds[kKNumKinds];
  int nk = 0;
  for (int i = 0; i < step.nmem; ++i) {
    bool seen = false;
    for (int k = 0; k < nk; ++k) seen = seen || kinds[k] == step.m[i].kind;
    if (!seen) kinds[nk++] = step.m[i].kind;
  }
  auto launch = [&](const void* fn, int k1, int k2) {
    GroupArgs g;
    std::memset(&g, 0, sizeof(g));
    int64_t total = 0;
    for (int i = 0; i < step.nmem; ++i) {
      const Member& m = step.m[i];
      if (m.kind != k1 && m.kind != k2) continue;
      g.start[g.n] = int(total);
      g.args[g.n] = m.args;
      g.gx[g.n] = m.gx;
      g.second[g.n] = m.kind == k2 && k2 != k1 ? 1 : 0;
      ++g.n;
      total += m.blocks;
    }
    g.start[g.n] = int(total);
    for (int i = g.n + 1; i <= kMaxMembersG; ++i) g.start[i] = std::numeric_limits<int>::max();
    void* params[] = {&g};
    (void)hipLaunchKernel(fn, dim3(unsigned(total)), dim3(unsigned(block_of(k1))), params, 0, s);
  };
  // pairable kinds two by two, the rest (and an odd one out) alone
  int pend = -1;
  for (int k = 0; k < nk; ++k) {
    const int pi = pairable_index(kinds[k]);
    if (pi < 0) {
      launch(group_kernel<T>(kinds[k]), kinds[k], kinds[k]);
      continue;
    }
    if (pend < 0) {
      pend = pi;
      continue;
    }
    const int a = std::min(pend, pi), b = std::max(pend, pi);
    launch(group2_kernel<T>(a, b), kPairable[a], kPairable[b]);
    pend = -1;
  }
  if (pend >= 0) launch(group_kernel<T>(kPairable[pend]), kPairable[pend], kPairable[pend]);
}

template <class T>
int run_phase(const std::vector<LockProg>& progs, hipStream_t s) {
  const int rc = lockstep(progs, [&](const MultiArgs& a, unsigned) { launch_groups<T>(a, s); });
  if (rc) return rc;
  return hipGetLastError() == hipSuccess ? ST_OK : ST_EHIP;
}

int run_phase_any(const Batch& Bt, const std::vector<LockProg>& progs, hipStream_t s) {
  return Bt.fp32 ? run_phase<float>(progs, s) : run_phase<double>(progs, s);
}

int batch_solve(Batch& Bt, const double* const* b, double* const* x, const st_opts* o, st_info* infos,
                int* statuses, hipStream_t s) {
  auto t0 = std::chrono::steady_clock::now();
  const int ns = int(Bt.sys.size());
  const int m = Bt.m;
  if ((o->restart > 0 && o->restart != m)) return ST_EINVAL;
  if (o->orth < 0 || o->orth > 1) return ST_EINVAL;   // lockstep steps use CGS2
  const int maxit = o->maxit > 0 ? o->maxit : 1000;
  for (int i = 0; i < ns; ++i)
    if (!b[i] || !x[i] || b[i] == x[i]) return ST_EINVAL;
  // per-solve programs: record, copy to the device, wait for the copy
  std::vector<unsigned char> pool;
  record_dynamic(Bt, pool, reinterpret_cast<unsigned char*>(Bt.base + Bt.dyn_off), b, x, !o->x0_given);
  if (pool.size() > Bt.dyn_bytes) return ST_EINTERNAL;
  std::memcpy(Bt.staging, pool.data(), pool.size());
  HIP_TRY(hipMemcpyAsync(Bt.base + Bt.dyn_off, Bt.staging, pool.size(), hipMemcpyHostToDevice, s));
  auto fetch = [&]() -> int {
    if (hipMemcpyAsync(Bt.host_out, Bt.out, sizeof(double) * 4 * ns, hipMemcpyDeviceToHost, s) != hipSuccess)
      return ST_EHIP;
    return hipStreamSynchronize(s) == hipSuccess ? ST_OK : ST_EHIP;
  };
  std::vector<double> bnorm(ns, 0.0), tol(ns, 0.0), true_res(ns, 0.0);
  std::vector<int> its(ns, 0), status(ns, ST_ENOTCONV), restarts(ns, 0), done(ns, 0), mused(ns, 0);
  std::vector<LockProg> progs;
  for (int i = 0; i < ns; ++i) progs.push_back(LockProg{nullptr, &Bt.sys[i].init});
  int rc = run_phase_any(Bt, progs, s);
  if (!rc) rc = fetch();
  if (rc) return rc;
  std::vector<int> active;
  for (int i = 0; i < ns; ++i) {
    bnorm[i] = Bt.host_out[4 * i];
    if (!std::isfinite(bnorm[i])) {
      status[i] = ST_EBREAKDOWN;
      done[i] = 1;
    } else if (bnorm[i] == 0.0) {
      Ctx c{s, nullptr};
      FillArgs f{x[i], Bt.sys[i].K.N, 0.0};
      emit(c, kKFill, dim3(grid_for(Bt.sys[i].K.N)), &k_fill, f);
      status[i] = ST_OK;
      done[i] = 1;
    } else {
      tol[i] = std::max(o->rtol * bnorm[i], o->atol);
      active.push_back(i);
    }
  }
  std::vector<int> finalize;
  while (!active.empty()) {
    progs.clear();
    for (int i : active) progs.push_back(LockProg{nullptr, &Bt.sys[i].resid});
    rc = run_phase_any(Bt, progs, s);
    if (!rc) rc = fetch();
    if (rc) return rc;
    std::vector<int> cyc;
    for (int i : active) {
      const double beta = Bt.host_out[4 * i];
      true_res[i] = beta;
      if (!std::isfinite(beta)) {
        status[i] = ST_EBREAKDOWN;
        done[i] = 1;
        continue;
      }
      if (beta <= tol[i]) {
        status[i] = ST_OK;
        finalize.push_back(i);
        continue;
      }
      if (its[i] >= maxit) {
        finalize.push_back(i);
        continue;
      }
      if (o->history && its[i] == 0 && o->history_len > 0) o->history[size_t(i) * o->history_len] = beta / bnorm[i];
      cyc.push_back(i);
    }
    active = cyc;
    if (active.empty()) break;
    progs.clear();
    for (int i : cyc) progs.push_back(LockProg{nullptr, &Bt.sys[i].head});
    rc = run_phase_any(Bt, progs, s);
    if (rc) return rc;
    for (int i : cyc) mused[i] = 0;
    std::vector<int> inner = cyc;
    for (int j = 0; j < m && !inner.empty(); ++j) {
      progs.clear();
      for (int i : inner) {
        BatchSys& S = Bt.sys[size_t(i)];
        progs.push_back(LockProg{&S.pa, &S.pb, &S.pdep, &S.tail[size_t(j)]});
      }
      rc = run_phase_any(Bt, progs, s);
      if (!rc) rc = fetch();
      if (rc) return rc;
      std::vector<int> next;
      for (int i : inner) {
        ++its[i];
        mused[i] = j + 1;
        const double hj = Bt.host_out[4 * i + 1], est = Bt.host_out[4 * i + 2];
        if (o->history && its[i] < o->history_len) o->history[size_t(i) * o->history_len + its[i]] = est / bnorm[i];
        if (!std::isfinite(est) || !std::isfinite(hj)) {
          status[i] = ST_EBREAKDOWN;
          done[i] = 1;
          continue;
        }
        if (est <= tol[i] || its[i] >= maxit) continue;
        next.push_back(i);
      }
      inner = next;
    }
    // close the cycle of every system still in it
    std::vector<int> cont;
    progs.clear();
    for (int i : cyc) {
      if (done[i]) continue;
      progs.push_back(LockProg{nullptr, &Bt.sys[i].end[size_t(mused[i] - 1)]});
      restarts[i]++;
      cont.push_back(i);
    }
    rc = run_phase_any(Bt, progs, s);
    if (rc) return rc;
    active = cont;
  }
  progs.clear();
  for (int i : finalize) progs.push_back(LockProg{nullptr, &Bt.sys[i].fin});
  rc = run_phase_any(Bt, progs, s);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipGetLastError());
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int worst = ST_OK;
  for (int i = 0; i < ns; ++i) {
    st_info& in = infos[i];
    in.iterations = its[i];
    in.restarts = restarts[i];
    in.converged = status[i] == ST_OK ? 1 : 0;
    in.true_rel_residual = bnorm[i] > 0.0 ? true_res[i] / bnorm[i] : 0.0;
    in.seconds = secs;
    in.precond_seconds = 0.0;
    in.jacobian_seconds = 0.0;
    in.precond_calls = its[i];
    in.jacobian_calls = its[i] + restarts[i] + (status[i] == ST_OK ? 1 : 0);
    if (statuses) statuses[i] = status[i];
    if (status[i] < 0 && worst >= 0) worst = status[i];
    else if (status[i] == ST_ENOTCONV && worst == ST_OK) worst = ST_ENOTCONV;
  }
  return worst;
}

}  // namespace
}  // namespace st

struct st_batch {
  st::Batch b;
};


// ============================================================ C ABI ===
// Scratch of the allocation-free preconditioner apply (st_apply_precond_noalloc):
// one array per GPU, placed by the code-object loader and held until the
// process ends.  In host code its name is a host-side stand-in, never a device
// address: kernels receive the address hipGetSymbolAddress returns for the
// current device.
constexpr size_t kNoAllocScratchBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace st {
namespace {

constexpr int kMaxDevices = 64;

std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array, looked up once per
// device (with that device current).
int scratch_for_current_device(int* dev_out, char** ptr_out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return ST_EHIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(::scratch));
    if (e != hipSuccess || !p) {
      std::fprintf(stderr, "libst: hipGetSymbolAddress(scratch) failed on device %d: %s\n", dev,
                   hipGetErrorString(e));
      return ST_EHIP;
    }
    g_scratch_ptr[dev] = static_cast<char*>(p);
  }
  *dev_out = dev;
  *ptr_out = g_scratch_ptr[dev];
  return ST_OK;
}

// The level buffers of a hierarchy with the preconditioner scratch relocated
// to sbase.
std::vector<void*> relocated(const Handle& H, const std::vector<size_t>& offs, char* sbase) {
  std::vector<void*> v;
  for (size_t o : offs) v.push_back(sbase + (o - H.L.pt_begin));
  return v;
}

}  // namespace
}  // namespace st

namespace st {
namespace {

// ================================================= space-time Newton ===
// Newton's method on the nonlinear recurrence, eq. (recurrence), all slabs at
// once (Sec. "Performance of preconditioner"): the residual on the device
// (kernels_nl.h), the linearisation about the current iterate assembled on the
// host into a plan and uploaded into the caller's linear workspace, its
// correction from FGMRES with P_T, and the update on the device.
struct NonlinearState {
  int n = 0, nt = 0, ns = 0;
  double dt = 0, mu = 0, eta = 0, mu0 = 0;
  int64_t N = 0;
  char* base = nullptr;
  double *ub = nullptr, *pb = nullptr, *jb = nullptr, *ab = nullptr, *u0 = nullptr, *a0 = nullptr;
  double *f = nullptr, *e = nullptr, *elem = nullptr, *r = nullptr, *b = nullptr, *d = nullptr;
  double *su = nullptr, *sj = nullptr, *sa = nullptr, *part = nullptr;
  double* host = nullptr;   // pinned: the norm partials
};

constexpr int kNlNormBlocks = 256;

struct NlLayoutHost {
  size_t ub, pb, jb, ab, u0, a0, f, e, elem, r, b, d, su, sj, sa, part, end;
};

NlLayoutHost nl_layout(const st_nl_problem& p) {
  NlLayoutHost L{};
  size_t cur = 0;
  auto take = [&](size_t bytes) {
    const size_t off = cur;
    cur = (cur + bytes + 255) & ~size_t(255);
    return off;
  };
  const size_t nt = size_t(p.nt), nq2 = size_t(2 * p.n + 1) * (2 * p.n + 1), nq1 = size_t(p.n + 1) * (p.n + 1);
  const NlLayout D(p.n);
  const size_t N = nt * size_t(D.ns);
  L.ub = take(8 * nt * 2 * nq2);
  L.pb = take(8 * nt * nq1);
  L.jb = take(8 * nt * nq1);
  L.ab = take(8 * nt * nq1);
  L.u0 = take(8 * 2 * nq2);
  L.a0 = take(8 * nq1);
  L.f = take(p.f ? 8 * nt * 2 * nq2 : 0);
  L.e = take(p.e ? 8 * nt * nq1 : 0);
  L.elem = take(8 * nt * size_t(p.n) * p.n * kNlLocal);
  L.r = take(8 * N);
  L.b = take(8 * N);
  L.d = take(8 * N);
  L.su = take(8 * nt * 2 * nq2);
  L.sj = take(8 * nt * nq1);
  L.sa = take(8 * nt * nq1);
  L.part = take(8 * kNlNormBlocks);
  L.end = cur;
  return L;
}

NlArgs nl_args(const NonlinearState& S, const double* x, double* r) {
  NlArgs a;
  a.n = S.n;
  a.nt = S.nt;
  a.h = 1.0 / S.n;
  a.dt = S.dt;
  a.mu = S.mu;
  a.eta = S.eta;
  a.mu0 = S.mu0;
  a.ub = S.ub;
  a.pb = S.pb;
  a.jb = S.jb;
  a.ab = S.ab;
  a.u0 = S.u0;
  a.a0 = S.a0;
  a.f = S.f;
  a.e = S.e;
  a.x = x;
  a.elem = S.elem;
  a.r = r;
  return a;
}

void nl_residual(const NonlinearState& S, const double* x, double* r, hipStream_t s) {
  const NlArgs a = nl_args(S, x, r);
  const int64_t ne = int64_t(S.n) * S.n * S.nt;
  hipLaunchKernelGGL(k_nl_element, dim3(unsigned((ne + 255) / 256)), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_nl_gather, dim3(unsigned((S.N + 255) / 256)), dim3(256), 0, s, a);
}

int nl_norm(NonlinearState& S, const double* x, hipStream_t s, double* out) {
  NlNormArgs a{x, S.N, S.part};
  hipLaunchKernelGGL(k_nl_norm_partial, dim3(kNlNormBlocks), dim3(256), 0, s, a);
  HIP_TRY(hipMemcpyAsync(S.host, S.part, sizeof(double) * kNlNormBlocks, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  double acc = 0.0;
  for (int i = 0; i < kNlNormBlocks; ++i) acc += S.host[i];
  *out = std::sqrt(acc);
  return ST_OK;
}

void nl_axpby(const double* x, double* y, double alpha, double beta, int64_t n, hipStream_t s) {
  NlAxpbyArgs a{x, y, alpha, beta, n};
  hipLaunchKernelGGL(k_nl_axpby, dim3(unsigned(std::min<int64_t>((n + 255) / 256, 8192))), dim3(256), 0, s, a);
}

}  // namespace
}  // namespace st

struct st_nl {
  st::NonlinearState s;
};

namespace st {
namespace {

int newton_solve(st_nl* nl, const st_problem* lin, void* lin_ws, size_t lin_ws_bytes, double* x,
                 const st_newton_opts* o, st_newton_info* info, hipStream_t s) {
  NonlinearState& S = nl->s;
  const auto t0 = std::chrono::steady_clock::now();
  const int maxn = std::min(o->max_newton > 0 ? o->max_newton : 20, ST_NEWTON_MAX);
  std::memset(info, 0, sizeof(*info));
  const size_t nq2 = size_t(2 * S.n + 1) * (2 * S.n + 1), nq1 = size_t(S.n + 1) * (S.n + 1);
  std::vector<double> hu(size_t(S.nt) * 2 * nq2), hj(size_t(S.nt) * nq1), ha(size_t(S.nt) * nq1);
  for (int it = 0;; ++it) {
    nl_residual(S, x, S.r, s);
    double rn = 0.0;
    int rc = nl_norm(S, S.r, s, &rn);
    if (rc) return rc;
    if (!std::isfinite(rn)) return ST_EBREAKDOWN;
    info->residual_norm[it] = rn;
    info->newton_iterations = it;
    if (rn <= o->atol) {
      info->converged = 1;
      break;
    }
    if (it >= maxn) break;
    // linearisation state: full nodal fields of the iterate, to the host
    NlStateArgs sa{S.n, S.nt, S.ub, S.jb, S.ab, x, S.su, S.sj, S.sa};
    const int64_t per = int64_t(2 * nq2 + 2 * nq1) * S.nt;
    hipLaunchKernelGGL(k_nl_state, dim3(unsigned((per + 255) / 256)), dim3(256), 0, s, sa);
    HIP_TRY(hipMemcpyAsync(hu.data(), S.su, 8 * hu.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(hj.data(), S.sj, 8 * hj.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(ha.data(), S.sa, 8 * ha.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const auto ts = std::chrono::steady_clock::now();
    st_problem pr = *lin;
    pr.n = S.n;
    pr.nt = S.nt;
    pr.dt = S.dt;
    pr.mu = S.mu;
    pr.eta = S.eta;
    pr.mu0 = S.mu0;
    pr.ubar = hu.data();
    pr.abar = ha.data();
    pr.jbar = hj.data();
    st_plan* plan = nullptr;
    rc = st_plan_create(&pr, &plan);
    if (rc) return rc;
    st_handle* h = nullptr;
    rc = st_create(plan, lin_ws, lin_ws_bytes, s, &h);
    st_plan_destroy(plan);
    if (rc) return rc;
    info->setup_seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - ts).count();
    // correction: J d = -r with FGMRES and P_T, from zero
    nl_axpby(S.r, S.b, -1.0, 0.0, S.N, s);
    st_opts lo = o->linear;
    lo.x0_given = 0;
    lo.history = nullptr;
    lo.history_len = 0;
    st_info li;
    std::memset(&li, 0, sizeof(li));
    rc = fgmres(h->h, S.b, S.d, &lo, &li, s, false);
    st_destroy(h);
    if (rc < 0) return rc;
    info->linear_iterations[it] = li.iterations;
    info->linear_iterations_total += li.iterations;
    nl_axpby(S.d, x, 1.0, 1.0, S.N, s);
  }
  HIP_TRY(hipStreamSynchronize(s));
  info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return info->converged ? ST_OK : ST_ENOTCONV;
}

}  // namespace
}  // namespace st

extern "C" {

int st_create(const st_plan* plan, void* ws, size_t ws_bytes, void* stream, st_handle** out) {
  using namespace st;
  if (!plan || !ws || !out) return ST_EINVAL;
  *out = nullptr;
  const Plan& P = plan->p;
  if (ws_bytes < P.ws_bytes) return ST_ENOMEM;
  if (reinterpret_cast<uintptr_t>(ws) % 256) return ST_EINVAL;
  if (P.amgFu.ncoarse > 512 || P.amgC0.ncoarse > 512 || P.amgKp.ncoarse > 512) return ST_EINTERNAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  st_handle* hh = nullptr;
  try {
    hh = new st_handle;
  } catch (...) {
    return ST_ENOMEM;
  }
  Handle& H = hh->h;
  H.d = P.blk.d;
  H.dt = P.blk.dt;
  H.fp32 = P.fp32;
  H.exact = P.exact;
  H.inner_iters = P.inner_iters;
  H.mass_iters = P.mass_iters;
  H.max_restart = P.max_restart;
  H.adjoint = P.prob.adjoint;
  H.fu_deg = P.fu_deg;
  H.ca_deg = P.ca_deg;
  H.use_stencil = P.use_stencil;
  H.sweep_fuse = P.prob.sweep_fuse == 1 ? 1 : 0;
  H.step_lanes = P.prob.sweep_lanes == 2 ? 2 : 1;
  H.j_slabs = P.prob.j_slabs;
  H.sFu = P.sFu;
  H.sAu = P.sAu;
  H.sC0 = P.sC0;
  H.sCP = P.sCP;
  H.sCQ = P.sCQ;
  H.sFuT = P.sFuT;
  H.sC0T = P.sC0T;
  H.sAuT = P.sAuT;
  H.sCPT = P.sCPT;
  H.sCQT = P.sCQT;
  H.sMj = P.sMj;
  H.sKjA = P.sKjA;
  // One workgroup covers the C_A grid with at most one row per thread: then the
  // chain kernel (no dispatch per step) beats per-step launches; on larger
  // grids one CU is too slow for it.
  H.use_chain = H.use_stencil && H.ca_deg > 0 && std::max(H.d.na, H.d.nj) <= kChainBlock && P.prob.sweep_chain >= 0 &&
                        H.sC0.ncomp == 1 && H.sCP.ncomp == 1 && H.sCQ.ncomp == 1 && H.sMj.ncomp == 1 &&
                        H.sKjA.ncomp == 1
                    ? 1
                    : 0;
  H.base = static_cast<char*>(ws);
  H.L = workspace_layout(P);
  char* base = H.base;
  if (hipMemcpyAsync(base, P.img.bytes.data(), P.img.bytes.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    delete hh;
    return ST_EHIP;
  }
  H.J = mirror(base, P.J);
  H.MA64 = mirror(base, P.MA64);
  if (H.adjoint) H.JT = mirror(base, P.JT);
  H.MA = mirror(base, P.MA);
  H.Mj = mirror(base, P.Mj);
  H.Mp = mirror(base, P.Mp);
  H.dMA = base + P.dMA.off;
  H.dMj = base + P.dMj.off;
  H.dMp = base + P.dMp.off;
  H.FA = mirror(base, P.FA);
  H.Fp = mirror(base, P.Fp);
  H.KjA = mirror(base, P.KjA);
  H.Bt = mirror(base, P.Bt);
  H.Zj = mirror(base, P.Zj);
  H.Mu = mirror(base, P.Mu);
  H.C1 = mirror(base, P.C1);
  if (H.adjoint) {
    H.FAt = mirror(base, P.FAt);
    H.Fpt = mirror(base, P.Fpt);
    H.KjAt = mirror(base, P.KjAt);
    H.B = mirror(base, P.B);
    H.Zjt = mirror(base, P.Zjt);
    H.ZAt = mirror(base, P.ZAt);
    H.C1t = mirror(base, P.C1t);
  }
  H.variant = P.variant;
  H.pint = P.pint;
  H.pint_deg = P.pint_deg;
  if (H.variant >= 1) H.Bv = mirror(base, P.Bv);
  if (H.variant == 2) H.Yv = mirror(base, P.Yv);
  H.mp_rowsum = at<double>(base, P.mp_rowsum.off);
  {
    const double* m = reinterpret_cast<const double*>(P.img.bytes.data() + P.mp_rowsum.off);
    double acc = 0.0;
    for (size_t i = 0; i < P.mp_rowsum.count; ++i) acc += m[i];
    H.msum = acc;
  }
  H.amgFu = mirror_amg(base, P.amgFu, H.L.fu_lev);
  H.amgC0 = mirror_amg(base, P.amgC0, H.L.ca_lev);
  H.amgKp = mirror_amg(base, P.amgKp, H.L.kp_lev);
  if (H.adjoint) {
    H.amgFuT = mirror_amg(base, P.amgFuT, H.L.fu_lev);
    H.amgC0T = mirror_amg(base, P.amgC0T, H.L.ca_lev);
    // the transposed blocks share the spectrum (and the interval) of the forward ones
    H.amgFuT.alone = H.amgFu.alone;
    H.amgFuT.alone_dev = H.amgFu.alone_dev;
    H.amgC0T.alone = H.amgC0.alone;
    H.amgC0T.alone_dev = H.amgC0.alone_dev;
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&H.host_small), 64 * sizeof(double), hipHostMallocDefault) !=
      hipSuccess) {
    delete hh;
    return ST_EHIP;
  }
  // About 16 chunks of slabs: the F_u sweep of a chunk starts as soon as its
  // part of the C_A sweep is done.
  H.chunk = P.chunk;
  {
    int rc = ST_OK;
    try {
      const bool recorded = P.prob.single_stream == 0 && H.variant == 0 && H.pint == 0;
      if (recorded) rc = build_pipeline(H);
      if (rc == ST_OK && P.prob.autotune == 1) rc = autotune(H, s, recorded);
    } catch (...) {
      rc = ST_ENOMEM;
    }
    if (rc) {
      (void)hipHostFree(H.host_small);
      delete hh;
      return rc;
    }
  }
  {
    // the allocation-free apply's scratch on this device (set-up, once per device)
    const int rc = scratch_for_current_device(&H.scratch_dev, &H.noalloc_scratch);
    if (rc) {
      (void)hipHostFree(H.host_small);
      delete hh;
      return rc;
    }
  }
  *out = hh;
  return ST_OK;
}

int st_destroy(st_handle* h) {
  if (!h) return ST_OK;
  if (h->h.host_small) (void)hipHostFree(h->h.host_small);
  for (hipEvent_t e : h->h.prof_ev) (void)hipEventDestroy(e);
  delete h;
  return ST_OK;
}

int st_sizes(const st_handle* h, int64_t* n_total, int* ns, int* nt) {
  if (!h) return ST_EINVAL;
  if (n_total) *n_total = int64_t(h->h.d.ns) * h->h.d.nt;
  if (ns) *ns = h->h.d.ns;
  if (nt) *nt = h->h.d.nt;
  return ST_OK;
}

int st_tuning(const st_handle* h, int* j_slabs, int* step_rows, int* sweep_fuse, int* precond_launches,
              int* step_lanes) {
  if (!h) return ST_EINVAL;
  const st::Handle& H = h->h;
  if (j_slabs) *j_slabs = H.J.lanes != 1 ? 1 : (H.j_slabs == 0 ? 8 : H.j_slabs);
  if (step_rows) *step_rows = H.step_rows > 0 ? H.step_rows : (H.fp32 ? st::st_rows<float>() : st::st_rows<double>());
  if (sweep_fuse) *sweep_fuse = H.sweep_fuse;
  if (precond_launches) *precond_launches = H.pipeline ? int(H.pt_items.size()) + 1 : 0;
  if (step_lanes) *step_lanes = H.step_lanes;
  return ST_OK;
}

int st_profile_kernel(st_handle* h, int kernel, int every) {
  using namespace st;
  if (!h || kernel < 0 || kernel > 1 || (kernel == 1 && every < 1)) return ST_EINVAL;
  Handle& H = h->h;
  H.prof_fn = nullptr;
  H.prof_seen = H.prof_n = 0;
  H.prof_ms = 0.0;
  H.prof_used = 0;
  if (kernel == 0) return ST_OK;
  if (!H.pipeline) return ST_EINVAL;
  constexpr size_t kPairs = 8192;
  while (H.prof_ev.size() < 2 * kPairs) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return ST_EHIP;
    H.prof_ev.push_back(e);
  }
  H.prof_fn = H.fp32 ? reinterpret_cast<const void*>(&k_two<BodyStCheb<float>, BodyStCheb<float>>)
                     : reinterpret_cast<const void*>(&k_two<BodyStCheb<double>, BodyStCheb<double>>);
  H.prof_every = every;
  return ST_OK;
}

int st_profile_read(const st_handle* h, double* seconds, int64_t* launches_timed, int64_t* launches_seen) {
  if (!h) return ST_EINVAL;
  if (seconds) *seconds = h->h.prof_ms * 1e-3;
  if (launches_timed) *launches_timed = h->h.prof_n;
  if (launches_seen) *launches_seen = h->h.prof_seen;
  return ST_OK;
}

int st_apply_jacobian(st_handle* h, const double* x, double* y, void* stream) {
  if (!h || !x || !y || x == y) return ST_EINVAL;
  st::Ctx c{static_cast<hipStream_t>(stream), nullptr};
  st::apply_J(h->h, x, y, c, false, 1.0, nullptr);
  return hipGetLastError() == hipSuccess ? ST_OK : ST_EHIP;
}

int st_apply_jacobian_t(st_handle* h, const double* x, double* y, void* stream) {
  if (!h || !x || !y || x == y || !h->h.adjoint) return ST_EINVAL;
  st::Ctx c{static_cast<hipStream_t>(stream), nullptr};
  st::apply_J(h->h, x, y, c, true, 1.0, nullptr);
  return hipGetLastError() == hipSuccess ? ST_OK : ST_EHIP;
}

int st_apply_precond(st_handle* h, const double* r, double* z, void* stream) {
  if (!h || !r || !z || r == z) return ST_EINVAL;
  st::Ctx c{static_cast<hipStream_t>(stream), nullptr};
  int rc = st::apply_precond(h->h, r, z, c, false);
  if (rc) return rc;
  return hipGetLastError() == hipSuccess ? ST_OK : ST_EHIP;
}

int st_apply_precond_t(st_handle* h, const double* r, double* z, void* stream) {
  if (!h || !r || !z || r == z || !h->h.adjoint) return ST_EINVAL;
  st::Ctx c{static_cast<hipStream_t>(stream), nullptr};
  int rc = st::apply_precond(h->h, r, z, c, true);
  if (rc) return rc;
  return hipGetLastError() == hipSuccess ? ST_OK : ST_EHIP;
}

int st_apply_precond_noalloc(st_handle* h, const double* r, double* z, void* stream) {
  using namespace st;
  if (!h || !r || !z || r == z) return ST_EINVAL;
  Handle& H = h->h;
  if (H.variant != 0 || H.pint != 0) return ST_EINVAL;
  const size_t need = H.L.end - H.L.pt_begin;
  if (need > ::kNoAllocScratchBytes) {
    std::fprintf(stderr,
                 "libst: st_apply_precond_noalloc: this system's preconditioner scratch (%zu bytes) exceeds the "
                 "library's static scratch (%zu bytes)\n",
                 need, ::kNoAllocScratchBytes);
    return ST_ENOMEM;
  }
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != H.scratch_dev || !H.noalloc_scratch) return ST_EINVAL;
  // Step by step on the caller's stream (the recorded programs hold workspace
  // scratch addresses), every scratch buffer relocated to the static array.
  char* const sb = H.noalloc_scratch;
  std::vector<void*> fu = relocated(H, H.L.fu_lev, sb), ca = relocated(H, H.L.ca_lev, sb),
                     kp = relocated(H, H.L.kp_lev, sb);
  std::swap(H.amgFu.buf, fu);
  std::swap(H.amgC0.buf, ca);
  std::swap(H.amgKp.buf, kp);
  H.sbase = sb;
  // st_apply_precond replays the recorded programs, which never use the chain
  // kernel; without them it runs step by step, chain kernel included: the
  // same choice here gives the same result, bit for bit.
  const int use_chain = H.use_chain;
  if (H.pipeline) H.use_chain = 0;
  Ctx c{static_cast<hipStream_t>(stream), nullptr};
  const int rc = H.fp32 ? precond_forward<float>(H, r, z, c, c) : precond_forward<double>(H, r, z, c, c);
  H.use_chain = use_chain;
  H.sbase = nullptr;
  std::swap(H.amgFu.buf, fu);
  std::swap(H.amgC0.buf, ca);
  std::swap(H.amgKp.buf, kp);
  if (rc) return rc;
  return hipGetLastError() == hipSuccess ? ST_OK : ST_EHIP;
}

int st_apply_initial_coupling(st_handle* h, const double* a0, double* y, void* stream) {
  if (!h || !a0 || !y || a0 == y) return ST_EINVAL;
  st::Ctx c{static_cast<hipStream_t>(stream), nullptr};
  st::spmv1<double>(c, h->h.MA64, 1, 0, 0, a0, 0, 1.0, nullptr, 0.0, y, 0,
                    st::kRoleSlab);
  return hipGetLastError() == hipSuccess ? ST_OK : ST_EHIP;
}

int st_fgmres_solve(st_handle* h, const double* b, double* x, const st_opts* o, st_info* info, void* stream) {
  if (!h || !b || !x || !o || !info || b == x) return ST_EINVAL;
  return st::fgmres(h->h, b, x, o, info, static_cast<hipStream_t>(stream), false);
}

int st_adjoint_solve(st_handle* h, const double* g, double* lam, const st_opts* o, st_info* info, void* stream) {
  if (!h || !g || !lam || !o || !info || g == lam) return ST_EINVAL;
  return st::fgmres(h->h, g, lam, o, info, static_cast<hipStream_t>(stream), true);
}

int st_timestep_solve(st_handle* const* hs, int nt, const double* b, double* x, const st_opts* o,
                      st_info* infos, void* stream) {
  if (!hs || nt < 1 || !b || !x || !o || !infos || b == x) return ST_EINVAL;
  for (int k = 0; k < nt; ++k)
    if (!hs[k]) return ST_EINVAL;
  try {
    return st::timestep_solve(hs, nt, b, x, o, infos, static_cast<hipStream_t>(stream));
  } catch (...) {
    return ST_ENOMEM;
  }
}

int st_batch_create(st_handle* const* hs, int nsys, int restart, st_batch** out) {
  using namespace st;
  if (!hs || !out || nsys < 1 || nsys > kMaxMembers) return ST_EINVAL;
  *out = nullptr;
  const int m = restart > 0 ? restart : 30;
  for (int i = 0; i < nsys; ++i) {
    if (!hs[i]) return ST_EINVAL;
    if (m > hs[i]->h.max_restart) return ST_EINVAL;
    if (hs[i]->h.variant != 0 || hs[i]->h.pint != 0) return ST_EINVAL;
    if (hs[i]->h.fp32 != hs[0]->h.fp32) return ST_EINVAL;
    for (int k = 0; k < i; ++k)
      if (hs[k] == hs[i]) return ST_EINVAL;
  }
  st_batch* bb = nullptr;
  try {
    bb = new st_batch;
    Batch& B = bb->b;
    B.m = m;
    B.fp32 = hs[0]->h.fp32;
    B.sys.resize(size_t(nsys));
    for (int i = 0; i < nsys; ++i) B.sys[size_t(i)].H = &hs[i]->h;
    // sizes: the programs have the same shape whatever the addresses
    std::vector<unsigned char> pool;
    const int rc = record_static(B, pool, nullptr);
    if (rc) {
      delete bb;
      return rc;
    }
    B.static_bytes = pool.size();
    std::vector<double*> fake(size_t(nsys), nullptr);
    record_dynamic(B, pool, nullptr, fake.data(), fake.data(), true);
    B.dyn_bytes = pool.size();
    B.out_off = 0;
    B.static_off = align_up(sizeof(double) * 4 * size_t(nsys), 256);
    B.dyn_off = align_up(B.static_off + B.static_bytes, 256);
    B.ws_bytes = align_up(B.dyn_off + B.dyn_bytes, 256);
    // launches of one Arnoldi step (preconditioner + J + Gram-Schmidt), all
    // members in lockstep vs each member alone
    auto count = [](const std::vector<LockProg>& progs) {
      int64_t n = 0;
      (void)lockstep(progs, [&](const MultiArgs&, unsigned) { ++n; });
      return n;
    };
    std::vector<LockProg> all;
    B.sep_launches = 0;
    for (BatchSys& S : B.sys) {
      all.push_back(LockProg{&S.pa, &S.pb, &S.pdep, &S.tail[0]});
      B.sep_launches += count({all.back()});
    }
    B.lock_launches = count(all);
  } catch (...) {
    delete bb;
    return ST_ENOMEM;
  }
  *out = bb;
  return ST_OK;
}

int st_batch_workspace_size(const st_batch* b, size_t* bytes) {
  if (!b || !bytes) return ST_EINVAL;
  *bytes = b->b.ws_bytes;
  return ST_OK;
}

int st_batch_launch_counts(const st_batch* b, int64_t* lockstep, int64_t* separate) {
  if (!b) return ST_EINVAL;
  if (lockstep) *lockstep = b->b.lock_launches;
  if (separate) *separate = b->b.sep_launches;
  return ST_OK;
}

int st_batch_upload(st_batch* b, void* ws, size_t ws_bytes, void* stream) {
  using namespace st;
  if (!b || !ws) return ST_EINVAL;
  Batch& B = b->b;
  if (ws_bytes < B.ws_bytes) return ST_ENOMEM;
  if (reinterpret_cast<uintptr_t>(ws) % 256) return ST_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  try {
    B.base = static_cast<char*>(ws);
    B.out = reinterpret_cast<double*>(B.base + B.out_off);
    std::vector<unsigned char> pool;
    if (record_static(B, pool, reinterpret_cast<unsigned char*>(B.base + B.static_off)) != ST_OK ||
        pool.size() != B.static_bytes)
      return ST_EINTERNAL;
    if (!B.host_out &&
        hipHostMalloc(reinterpret_cast<void**>(&B.host_out), sizeof(double) * 4 * B.sys.size(),
                      hipHostMallocDefault) != hipSuccess)
      return ST_EHIP;
    if (!B.staging && B.dyn_bytes &&
        hipHostMalloc(reinterpret_cast<void**>(&B.staging), B.dyn_bytes, hipHostMallocDefault) != hipSuccess)
      return ST_EHIP;
    if (hipMemcpyAsync(B.base + B.static_off, pool.data(), pool.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return ST_EHIP;
  } catch (...) {
    return ST_ENOMEM;
  }
  return ST_OK;
}

int st_fgmres_solve_batched(st_batch* b, const double* const* bvec, double* const* x, const st_opts* o,
                            st_info* infos, int* statuses, void* stream) {
  if (!b || !bvec || !x || !o || !infos || !b->b.base) return ST_EINVAL;
  try {
    return st::batch_solve(b->b, bvec, x, o, infos, statuses, static_cast<hipStream_t>(stream));
  } catch (...) {
    return ST_ENOMEM;
  }
}

int st_batch_destroy(st_batch* b) {
  if (!b) return ST_OK;
  if (b->b.host_out) (void)hipHostFree(b->b.host_out);
  if (b->b.staging) (void)hipHostFree(b->b.staging);
  delete b;
  return ST_OK;
}

int st_nl_workspace_size(const st_nl_problem* p, size_t* bytes) {
  if (!p || !bytes || p->n < 2 || p->nt < 1) return ST_EINVAL;
  *bytes = st::nl_layout(*p).end;
  return ST_OK;
}

int st_nl_create(const st_nl_problem* p, void* ws, size_t ws_bytes, void* stream, st_nl** out) {
  using namespace st;
  if (!p || !ws || !out || p->n < 2 || p->nt < 1 || !(p->dt > 0) || !p->u_base || !p->p_base || !p->j_base ||
      !p->a_base || !p->u_init || !p->a_init)
    return ST_EINVAL;
  *out = nullptr;
  const NlLayoutHost L = nl_layout(*p);
  if (ws_bytes < L.end) return ST_ENOMEM;
  if (reinterpret_cast<uintptr_t>(ws) % 256) return ST_EINVAL;
  st_nl* nl = nullptr;
  try {
    nl = new st_nl;
  } catch (...) {
    return ST_ENOMEM;
  }
  NonlinearState& S = nl->s;
  S.n = p->n;
  S.nt = p->nt;
  S.dt = p->dt;
  S.mu = p->mu;
  S.eta = p->eta;
  S.mu0 = p->mu0;
  S.ns = NlLayout(p->n).ns;
  S.N = int64_t(S.ns) * S.nt;
  S.base = static_cast<char*>(ws);
  char* B = S.base;
  S.ub = at<double>(B, L.ub);
  S.pb = at<double>(B, L.pb);
  S.jb = at<double>(B, L.jb);
  S.ab = at<double>(B, L.ab);
  S.u0 = at<double>(B, L.u0);
  S.a0 = at<double>(B, L.a0);
  S.f = p->f ? at<double>(B, L.f) : nullptr;
  S.e = p->e ? at<double>(B, L.e) : nullptr;
  S.elem = at<double>(B, L.elem);
  S.r = at<double>(B, L.r);
  S.b = at<double>(B, L.b);
  S.d = at<double>(B, L.d);
  S.su = at<double>(B, L.su);
  S.sj = at<double>(B, L.sj);
  S.sa = at<double>(B, L.sa);
  S.part = at<double>(B, L.part);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t nt = size_t(p->nt), nq2 = size_t(2 * p->n + 1) * (2 * p->n + 1), nq1 = size_t(p->n + 1) * (p->n + 1);
  bool ok = hipHostMalloc(reinterpret_cast<void**>(&S.host), sizeof(double) * kNlNormBlocks, hipHostMallocDefault) ==
            hipSuccess;
  auto up = [&](double* dst, const double* src, size_t count) {
    if (ok && src) ok = hipMemcpyAsync(dst, src, 8 * count, hipMemcpyHostToDevice, s) == hipSuccess;
  };
  up(S.ub, p->u_base, nt * 2 * nq2);
  up(S.pb, p->p_base, nt * nq1);
  up(S.jb, p->j_base, nt * nq1);
  up(S.ab, p->a_base, nt * nq1);
  up(S.u0, p->u_init, 2 * nq2);
  up(S.a0, p->a_init, nq1);
  up(S.f, p->f, nt * 2 * nq2);
  up(S.e, p->e, nt * nq1);
  if (!ok || hipStreamSynchronize(s) != hipSuccess) {
    if (S.host) (void)hipHostFree(S.host);
    delete nl;
    return ST_EHIP;
  }
  *out = nl;
  return ST_OK;
}

int st_nl_residual(st_nl* nl, const double* x, double* r, void* stream) {
  if (!nl || !x || !r || x == r) return ST_EINVAL;
  st::nl_residual(nl->s, x, r, static_cast<hipStream_t>(stream));
  return hipGetLastError() == hipSuccess ? ST_OK : ST_EHIP;
}

int st_newton_solve(st_nl* nl, const st_problem* lin, void* lin_ws, size_t lin_ws_bytes, double* x,
                    const st_newton_opts* o, st_newton_info* info, void* stream) {
  if (!nl || !lin || !lin_ws || !x || !o || !info) return ST_EINVAL;
  if (lin->n != nl->s.n || lin->nt != nl->s.nt || lin->precond_variant != 0 || lin->adjoint) return ST_EINVAL;
  try {
    return st::newton_solve(nl, lin, lin_ws, lin_ws_bytes, x, o, info, static_cast<hipStream_t>(stream));
  } catch (...) {
    return ST_ENOMEM;
  }
}

int st_nl_destroy(st_nl* nl) {
  if (!nl) return ST_OK;
  if (nl->s.host) (void)hipHostFree(nl->s.host);
  delete nl;
  return ST_OK;
}

}  // extern "C"
