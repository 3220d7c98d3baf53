// Internal host-side data structures of libst (setup, packing, device image).
#pragma once

#include <cstdint>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "../../include/st.h"

namespace st {

// ------------------------------------------------------------ host CSR ---
struct Csr {
  int nr = 0, nc = 0;
  std::vector<int> rp;      // nr+1
  std::vector<int> ci;      // nnz, sorted within each row
  std::vector<double> v;    // nnz (or nsets * nnz for per-slab values)
  int64_t nnz() const { return rp.empty() ? 0 : rp[nr]; }
  // Position of (r, c) in the pattern, or -1.
  int64_t find(int r, int c) const;
};

// Pattern from (row, col) pairs; duplicates merged, rows sorted.
class PatternBuilder {
 public:
  PatternBuilder(int nr, int nc) : nr_(nr), nc_(nc), rows_(nr) {}
  void add(int r, int c) { rows_[r].push_back(c); }
  Csr finish();
 private:
  int nr_, nc_;
  std::vector<std::vector<int>> rows_;
};

// Sparse products on a common pattern type (host, float64).
Csr csr_transpose(const Csr& a);
Csr csr_matmul(const Csr& a, const Csr& b);          // pattern + values
Csr csr_add(const Csr& a, double sa, const Csr& b, double sb);  // sa*a + sb*b
Csr csr_scale_cols(const Csr& a, const std::vector<double>& s);  // a * diag(s)
void csr_spmv(const Csr& a, const double* x, double* y);         // y = a x (set 0)

// Run f(i) for i in [0, n) on up to `threads` host threads.
void parallel_for(int n, int threads, const std::function<void(int)>& f);
int host_threads();

// ------------------------------------------------------------- problem ---
struct Dims {
  int n = 0, nt = 0;
  int nq2 = 0, nq1 = 0;     // all Q2 / Q1 nodes
  int nf2 = 0, nf1 = 0;     // interior Q2 / Q1 nodes
  int nu = 0, np = 0, nj = 0, na = 0, ns = 0;
  int off[6] = {0, 0, 0, 0, 0, 0};   // u_x, u_y, p, j, A, end
};

Dims make_dims(int n, int nt);

// Every host-assembled block.  State-dependent blocks hold one value array per
// slab (v has nt * nnz entries, slab-major); constant blocks one value array.
struct Blocks {
  Dims d;
  double dt, mu, eta, mu0;
  Csr Fu, Mu, Ku, B, Bt, Zj, ZA, Mj, KjA, KjAt, Y, FA, MA, KA, Mp, Kp, Fp;
  Csr C0, C1, C2;           // wave operator bands; C1 has nt-1 value sets (nt>=2)
  std::vector<double> jbar; // [nt][nq1]
  std::vector<double> bbar2;  // |Bbar_k|^2 per slab
};

// Assembles all blocks from the state (host, multithreaded over slabs).
int assemble_blocks(const st_problem& p, Blocks& out, std::string& err);
void form_wave_operator(Blocks& b);

// ---------------------------------------------------------- device image ---
struct Span {
  size_t off = 0;   // byte offset in the image
  size_t count = 0; // elements
};

class Image {
 public:
  template <class T>
  Span put(const T* data, size_t count) {
    Span s = reserve(count * sizeof(T));
    s.count = count;
    if (count) std::memcpy(bytes.data() + s.off, data, count * sizeof(T));
    return s;
  }
  template <class T>
  Span put(const std::vector<T>& v) { return put(v.data(), v.size()); }
  Span reserve(size_t nbytes) {
    size_t off = (bytes.size() + 255) & ~size_t(255);
    bytes.resize(off + nbytes);
    Span s;
    s.off = off;
    s.count = nbytes;
    return s;
  }
  std::vector<char> bytes;
};

// Sliced ELLPACK for wave64: a slice is one wavefront.  Each row is owned by
// `lanes` consecutive lanes (1, 2, 4, 8 or 16), so a slice holds 64/lanes rows;
// entry j of the row sits at step j/lanes, lane (row_in_slice*lanes + j%lanes).
// Several segments can share the row permutation (the fused J rows).
constexpr int kSlice = 64;

struct SellSeg {
  Span sptr;        // int32 [nslices + 1], element offsets (multiples of 64)
  Span col;         // int32 [total]
  Span val;         // T [nsets][total]
  int nsets = 1;
  int64_t total = 0;
};

struct SellGroup {
  int nrows = 0, ncols = 0, nslices = 0;
  int lanes = 1;    // lanes per row; rows per slice = 64 / lanes
  int fp32 = 0;     // value type: 0 double, 1 float
  Span perm;        // int32 [nslices * 64 / lanes]; -1 marks padding rows
  SellSeg seg[3];
  int nseg = 0;
};

// Packs CSR matrices with the same row count into one SELL group.  Each
// matrix may carry several value sets (csr.v.size() = nsets * nnz).  Rows are
// sorted by total length in windows of `sigma` rows (0 = whole matrix).
// lanes = 0 picks the lanes per row from the mean row length.
SellGroup pack_sell(Image& img, const std::vector<const Csr*>& mats, int fp32, int sigma, int lanes = 0);
int auto_lanes(double mean_row_len);

// --------------------------------------------------------------- AMG ---
struct AmgLevel {
  int nrows = 0;
  SellGroup A;            // per-set values
  Span dinv;              // T [nsets][nrows]
  Span cheb;              // double [nsets][2] = (theta, delta) of the interval
  SellGroup P;            // prolongation to this level from the next (shared)
  SellGroup R;            // restriction from this level to the next (shared)
};

struct Amg {
  int nsets = 1;
  int fp32 = 0;
  int cheb_degree = 3;
  // Spectral interval of D^{-1} A on the finest level, per value set, for
  // Chebyshev-Jacobi used alone as the spatial solver: (theta, delta).
  std::vector<double> cheb_alone;
  Span cheb_alone_span;
  double kappa = 0.0;          // largest estimated condition number over the sets
  std::vector<AmgLevel> lev;   // lev.back() is the coarsest
  int ncoarse = 0;
  Span coarse_inv;        // T [nsets][ncoarse][ncoarse] dense inverse
  int singular = 0;
};

struct Grid2 { int gx, gy, ncomp; };   // structured node grid of a block (per component)

// Builds a smoothed-aggregation hierarchy for the value sets of `a` (a.v holds
// nsets * nnz values).  `grid` gives the structured node layout used for
// aggregation (3x3 node blocks per component).
int build_amg(Image& img, const Csr& a, int nsets, Grid2 grid, int fp32, int cheb_degree,
              int sigma, bool singular, Amg& out, std::string& err);
// Estimates [lambda_min, lambda_max] of D^{-1} A per value set (finest level)
// and stores the widened Chebyshev interval in out.cheb_alone.
void estimate_interval(Image& img, const Csr& a, int nsets, Amg& out);

// ------------------------------------------------------------ stencils ---
// A block on a structured node grid stored as 5x5 stencil coefficients:
// coef[set][slot][row], slot = c_col*25 + (dy+2)*5 + (dx+2), row = c*gx*gy +
// iy*gx + ix.  Neighbours outside the grid have zero coefficients.  With
// diag_comp the columns are taken from the row's own component only (25 slots).
// Generalised: radius rad (3x3 or 5x5 neighbourhoods, w = 2 rad + 1, slot =
// c_col*w*w + (dy+rad)*w + (dx+rad)) and a column grid cgx x cgy whose node
// (ii, jj) sits at row-grid position (ii + shift, jj + shift) (e.g. interior
// nodes of the full Q1 grid: shift 1).
struct StencilOp {
  int gx = 0, gy = 0, ncomp = 1, diag_comp = 0, nsets = 0, nslot = 0, fp32 = 0;
  int rad = 2, cgx = 0, cgy = 0, shift = 0;
  int64_t rows = 0;
  Span coef;
};
// Returns false if an entry of `m` lies outside the neighbourhood.
bool pack_stencil(Image& img, const Csr& m, int nsets, int gx, int gy, int ncomp, bool diag_comp, int fp32,
                  StencilOp& out, int rad = 2, int cgx = 0, int cgy = 0, int shift = 0);

// ---------------------------------------------------------------- plan ---
struct Plan {
  st_problem prob{};
  Blocks blk;
  Image img;
  size_t ws_bytes = 0;
  int fp32 = 0;
  int inner_iters = 40, mass_iters = 12, max_restart = 30, exact = 0;
  int fu_deg = 0, ca_deg = 0;     // > 0: Chebyshev alone of this degree; 0: AMG V-cycle
  int chunk = 8;                  // slabs per chunk of the C_A / F_u sweep pipeline
  int pint = 0, pint_deg = 1;     // Parareal iterations of the two sweeps (0: forward substitution), coarse degree
  // J and J^T (FP64): segment 0 per-slab values, 1 shared, 2 previous/next slab coupling.
  SellGroup J, JT;
  // P_T pieces (precision per fp32).
  SellGroup MA, Mj, Mp;           // masses (Chebyshev-Jacobi solves)
  Span dMA, dMj, dMp;             // inverse diagonals
  SellGroup FA, FAt, Fp, Fpt;     // per-slab bidiagonal applies (diag blocks)
  SellGroup KjA, KjAt, Bt, B;     // shared couplings
  SellGroup Zj, ZA, Zjt, ZAt;     // per-slab couplings
  SellGroup Yv, Bv;               // Y (per slab) and B for the lower factors of P, P-tilde
  int variant = 0;                // 0 P_T, 1 P-tilde, 2 P
  SellGroup Mu;                   // sweep coupling of F_u
  SellGroup C1, C2, C1t, C2t;     // sweep couplings of C_A
  SellGroup MA64;                 // M_A / dt in FP64 (initial-condition coupling)
  // Stencil forms of the sweep operators (used with Chebyshev-alone sweeps).
  // sAu, sCP, sCQ (and the transposes): couplings of the increment-form sweeps.
  StencilOp sFu, sAu, sC0, sCP, sCQ, sFuT, sAuT, sC0T, sCPT, sCQT;
  StencilOp sMj, sKjA;            // 3x3 stencils of the single-workgroup C_A chain
  int use_stencil = 0;
  Amg amgFu, amgC0, amgKp;        // spatial solvers (per-slab for Fu, C0; shared Kp)
  Amg amgFuT, amgC0T;             // transposed hierarchies for the adjoint
  Span mp_rowsum;                 // double [np]: 1^T M_p (pressure normalisation)
  size_t image_bytes = 0;
};

// Scratch vectors of a handle, carved from the workspace after the image.
struct WsLayout {
  size_t V = 0, Z = 0, w = 0, r = 0, hess = 0, small = 0, partial = 0, psum = 0;
  size_t ru = 0, yu = 0, xu = 0, rp = 0, q = 0, t = 0, xp = 0, rj = 0, yj = 0;
  size_t ra = 0, wA = 0, sA = 0, yA = 0, mr = 0, md0 = 0, md1 = 0, chr = 0, chd0 = 0, chd1 = 0;
  size_t mr2 = 0, md02 = 0, md12 = 0;           // mass-solve scratch of the second program
  size_t io = 0;                                // 2 pointers: input/output slots of a recorded P_T
  size_t pint_u[6] = {0, 0, 0, 0, 0, 0};        // Parareal sweeps: other iterate, correction, coarse part,
  size_t pint_a[6] = {0, 0, 0, 0, 0, 0};        // residual, two increments (F_u / C_A, Nt slabs each)
  std::vector<size_t> kp_lev, fu_lev, ca_lev;   // 6 vectors per level each
  size_t end = 0;
  // [pt_begin, end) holds only the preconditioner's scratch (psum onwards):
  // the allocation-free apply relocates exactly this range.
  size_t pt_begin = 0;
};
constexpr int kPartialBlocks = 1024;   // blocks of the two-stage reductions
// automatic Gram-Schmidt: delayed reorthogonalisation above this restart, or
// from this many unknowns on (where reading the basis is bandwidth-bound)
constexpr int kDelayedFrom = 64;
constexpr int64_t kDelayedRows = int64_t(1) << 20;
constexpr int kOpArgBytes = 448;       // largest argument block of a recorded launch
WsLayout workspace_layout(const Plan& p);

}  // namespace st
