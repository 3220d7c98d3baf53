// HIP kernels of libst (gfx950, wave64).  Everything here is sparse or vector
// work bound by HBM bandwidth or launch latency: no MFMA.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace st {

constexpr int kWave = 64;        // CDNA wavefront = one SELL slice
constexpr int kBlock = 256;      // 4 slices per workgroup

// The sparse kernels here are latency bound: letting the compiler use up to
// 128 VGPRs (4 waves per SIMD) keeps a row's loads in flight together instead
// of serialising them to reach maximum occupancy.
#define ST_LATENCY_KERNEL __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, 4)))

// Coefficients of the Chebyshev iteration for D^{-1} A x = D^{-1} b whose
// spectrum lies in an ellipse of centre theta with foci theta -+ c (Manteuffel,
// Numer. Math. 28, 1977; Saad, Iterative Methods for Sparse Linear Systems,
// Sec. 12.3): d_0 = D^{-1} r_0 / theta, then for step i >= 1
//   d_i = c1 d_{i-1} + c2 D^{-1} r_i,  x_i = x_{i-1} + d_i.
// delta > 0: real foci, c = delta (the interval [theta - delta, theta + delta]
//   when the ellipse is flat), rho_i = 1 / (2 theta/delta - rho_{i-1}),
//   rho_0 = delta / theta, c1 = rho_i rho_{i-1}, c2 = 2 rho_i / delta.
// delta <= 0: imaginary foci, c^2 = -delta^2 (an ellipse taller than wide, for
//   spectra of non-normal blocks), g_i = rho_i / c = 1 / (2 theta - c^2 g_{i-1}),
//   g_0 = 1 / theta, c1 = c^2 g_i g_{i-1}, c2 = 2 g_i: real arithmetic only.
struct ChebRec {
  double theta, delta, a, b;   // a, b: rho (or g) of the previous and current step
  __host__ __device__ ChebRec(double th, double de) : theta(th), delta(de) {
    a = b = de > 0.0 ? 1.0 / (th / de) : 1.0 / th;
  }
  // Advances to the next step and returns its coefficients.
  __host__ __device__ void next(double& c1, double& c2) {
    a = b;
    if (delta > 0.0) {
      b = 1.0 / (2.0 * (theta / delta) - a);
      c1 = b * a;
      c2 = 2.0 * b / delta;
    } else {
      const double csq = -delta * delta;
      b = 1.0 / (2.0 * theta - csq * a);
      c1 = csq * b * a;
      c2 = 2.0 * b;
    }
  }
};

// One segment of a multi-segment SELL SpMV.  For vector v (blockIdx.y) it adds
//   alpha * A_seg(values of set `set_base + v*set_step`) * x[(v + xshift) * xstride + :]
// when vlo <= v < vhi.
template <class T>
struct Seg {
  const int* sptr;
  const int* col;
  const T* val;
  int64_t vstride;     // elements per value set (0 = one shared set)
  int set_base, set_step;
  const void* x;
  int64_t xstride;
  int xshift;
  int vlo, vhi;
  double alpha;
};

template <class T, class TX>
struct SpmvArgs {
  const int* perm;
  int nslices;
  int lanes;            // lanes per row (1, 2, 4, 8, 16)
  int nseg;
  Seg<T> seg[3];
  const TX* b;          // optional: y = sum + beta * b
  int64_t bstride;
  double beta;
  TX* y;
  int64_t ystride;
  // Epilogue 1 (first Chebyshev step of a sweep solve, one vector): with
  // q = sum + beta b, write r = q, d = dinv q / theta, x = d.
  int epi;
  const T* dinv;
  double theta;
  TX* r;
  TX* d;
  TX* x;
};

// Kernel roles get distinct symbols so that profiles separate them.
enum Role : int {
  kRoleJ = 0,        // space-time Jacobian (or its transpose)
  kRoleSlab = 1,     // slab-parallel products inside P_T
  kRoleSweep = 2,    // sweep right-hand sides (coupling to earlier slabs)
  kRoleAmg = 3,      // AMG residuals, restriction, prolongation
};

// sum_j val[j*64] * x[col[j*64]] for j < w, loads issued in batches of 8 so
// that each batch costs two memory round trips (indices and values, then the
// gathered x) instead of two per entry.
template <class T, class TX, class TA>
__device__ inline TA sell_row(const T* __restrict__ val, const int* __restrict__ col, const TX* __restrict__ x,
                              int w) {
  TA sum = TA(0);
  int j = 0;
  for (; j + 8 <= w; j += 8) {
    int c[8];
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      c[u] = col[(j + u) * 64];
      v[u] = val[(j + u) * 64];
    }
    TX xv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) xv[u] = x[c[u]];
#pragma unroll
    for (int u = 0; u < 8; ++u) sum += TA(v[u]) * TA(xv[u]);
  }
  if (j < w) {
    const int rem = w - j;   // 1..7, padded to 8 with guarded loads
    int c[8];
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      c[u] = u < rem ? col[(j + u) * 64] : 0;
      v[u] = u < rem ? val[(j + u) * 64] : T(0);
    }
    TX xv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) xv[u] = u < rem ? x[c[u]] : TX(0);
#pragma unroll
    for (int u = 0; u < 8; ++u) sum += TA(v[u]) * TA(xv[u]);
  }
  return sum;
}

template <class TA>
__device__ inline TA group_sum(TA v, int lanes) {
  for (int off = lanes / 2; off > 0; off /= 2) v += __shfl_down(v, off, lanes);
  return v;
}

// y[v][row] = sum_seg alpha_seg (A_seg x_seg)[row] + beta b[v][row]
// Workgroup bx covers slices 4 bx .. 4 bx + 3 of vector v.
template <class T, class TX, class TA>
__device__ inline void spmv_body(const SpmvArgs<T, TX>& a, int bx, int v) {
  const int slice = bx * (kBlock / kWave) + (threadIdx.x / kWave);
  if (slice >= a.nslices) return;          // uniform per wavefront
  const int lane = threadIdx.x % kWave;
  const int L = a.lanes;
  const int q = lane / L, sub = lane % L;
  const int row = a.perm[slice * (kWave / L) + q];
  TA acc = TA(0);
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    if (s >= a.nseg) break;
    const Seg<T>& g = a.seg[s];
    if (v < g.vlo || v >= g.vhi) continue;
    const int beg = g.sptr[slice];
    const int w = (g.sptr[slice + 1] - beg) / kWave;
    const T* val = g.val + (g.vstride ? int64_t(g.set_base + v * g.set_step) * g.vstride : 0) + beg + lane;
    const TX* x = static_cast<const TX*>(g.x) + int64_t(v + g.xshift) * g.xstride;
    const int* col = g.col + beg + lane;
    const TA sum = sell_row<T, TX, TA>(val, col, x, w);
    acc += TA(g.alpha) * sum;
  }
  acc = group_sum(acc, L);
  if (sub != 0 || row < 0) return;
  if (a.b) acc += TA(a.beta) * TA(a.b[int64_t(v) * a.bstride + row]);
  if (a.epi == 1) {
    const TX dd = TX(TA(a.dinv[row]) * acc / TA(a.theta));
    a.r[row] = TX(acc);
    a.d[row] = dd;
    a.x[row] = dd;
    return;
  }
  a.y[int64_t(v) * a.ystride + row] = TX(acc);
}

template <class T, class TX, class TA, int Role>
__global__ ST_LATENCY_KERNEL void k_spmv(SpmvArgs<T, TX> a) {
  spmv_body<T, TX, TA>(a, blockIdx.x, blockIdx.y);
}

// The space-time Jacobian (or its transpose) over NV consecutive slabs per
// wavefront: each column index and each slab-invariant value of a row is
// loaded once for the NV slabs, the slab-dependent values and the gathered x
// once per slab; all loads of a batch of B entries are issued together (on a
// 64 x 64 mesh with 128 slabs the loads in flight per lane pay more than
// occupancy).  One lane per
// row.  Per row and slab the products are summed in the same order as k_spmv
// (segment by segment, entries in order), so the result is the same.
struct SpmvSlabsArgs {
  SpmvArgs<double, double> a;
  int nvec;   // number of slabs
  int nbx;    // workgroups along the slices (4 slices each)
  int nblk;   // nbx x slab groups; the grid is nblk rounded up to a multiple of 8
};

// Workgroup b of the (1-D) grid -> (slice block, slab group), so that each of
// the 8 XCDs (which take workgroups round robin) runs one contiguous range of
// blocks, slab group by slab group: the x lines a slice gathers are then
// fetched into that XCD's L2 once for the neighbouring slices too, instead of
// once per XCD.  A bijection of [0, round_up(nblk, 8)); false for padding.
__device__ inline bool slabs_block(const SpmvSlabsArgs& sa, int b, int& bx, int& by) {
  const int per = (sa.nblk + 7) / 8;
  const int logical = (b % 8) * per + b / 8;
  if (logical >= sa.nblk) return false;
  bx = logical % sa.nbx;
  by = logical / sa.nbx;
  return true;
}

template <int NV, int B = 4>
__device__ inline void spmv_slabs_body(const SpmvSlabsArgs& sa, int bx, int by) {
  const SpmvArgs<double, double>& a = sa.a;
  const int nvec = sa.nvec;
  const int v0 = by * NV;
  const int slice = bx * (kBlock / kWave) + (threadIdx.x / kWave);
  if (slice >= a.nslices) return;          // uniform per wavefront
  const int lane = threadIdx.x % kWave;
  const int row = a.perm[slice * kWave + lane];
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    if (s >= a.nseg) break;
    const Seg<double>& g = a.seg[s];
    // An empty segment (the coupling of a single slab) has no slab whose data
    // is in range: skip it (uniform across the launch).
    if (g.vlo >= g.vhi) continue;
    // Slabs outside the segment's range read slab vlo's data (in bounds) and
    // their sums are dropped, so every load of a batch is issued together.
    bool on[NV];
    const double* xs[NV];
    const double* vals[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      on[v] = v0 + v < nvec && v0 + v >= g.vlo && v0 + v < g.vhi;
      const int vv = on[v] ? v0 + v : g.vlo;
      xs[v] = static_cast<const double*>(g.x) + int64_t(vv + g.xshift) * g.xstride;
      vals[v] = g.val + (g.vstride ? int64_t(g.set_base + vv * g.set_step) * g.vstride : 0);
    }
    const int beg = g.sptr[slice];
    const int w = (g.sptr[slice + 1] - beg) / kWave;
    const int* __restrict__ col = g.col + beg + lane;
    double sum[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) sum[v] = 0.0;
    for (int j = 0; j < w; j += B) {
      const int rem = w - j;
      int c[B];
      int o[B];
#pragma unroll
      for (int u = 0; u < B; ++u) {
        o[u] = beg + lane + (j + (u < rem ? u : 0)) * kWave;
        c[u] = col[(j + (u < rem ? u : 0)) * kWave];
      }
      double vv[NV][B], xv[NV][B];
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int u = 0; u < B; ++u)
          vv[v][u] = g.vstride ? __builtin_nontemporal_load(vals[v] + o[u]) : (v == 0 ? vals[v][o[u]] : 0.0);
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int u = 0; u < B; ++u) xv[v][u] = xs[v][c[u]];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
#pragma unroll
        for (int u = 0; u < B; ++u) {
          const double val = g.vstride ? vv[v][u] : vv[0][u];
          sum[v] += (u < rem ? val : 0.0) * xv[v][u];
        }
      }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v)
      if (on[v]) acc[v] += g.alpha * sum[v];
  }
  if (row < 0) return;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    if (v0 + v >= nvec) break;
    double out = acc[v];
    if (a.b) out += a.beta * a.b[int64_t(v0 + v) * a.bstride + row];
    a.y[int64_t(v0 + v) * a.ystride + row] = out;
  }
}

// Bandwidth-bound: no cap on the waves per SIMD (unlike the latency kernels).
template <int NV, int B = 4>
__global__ __launch_bounds__(kBlock) void k_spmv_slabs(SpmvSlabsArgs a) {
  int bx, by;
  if (slabs_block(a, blockIdx.x, bx, by)) spmv_slabs_body<NV, B>(a, bx, by);
}

// Fused Chebyshev-Jacobi step for A x = b (A one SELL segment), per vector v.
//   mode 0: r = b (if b), d_new = Dinv r / theta, x = d_new (or x += d_new)
//   mode 1: r -= A d_old; d_new = c1 d_old + c2 Dinv r; x += d_new   (step >= 1)
//   mode 2: r -= A d_old
template <class T>
struct ChebArgs {
  const int* perm;
  int nslices;
  int lanes;
  const int* sptr;
  const int* col;
  const T* val;
  int64_t vstride;
  int set_base, set_step;
  const T* dinv;
  int64_t dstride;      // per-set stride of dinv (0 = shared)
  const double* cheb;   // (theta, delta) per set, or null -> use theta/delta below
  double theta, delta;
  const T* b;
  T* r;
  T* x;
  const T* dold;
  T* dnew;
  int64_t vec;          // stride between vectors
  int mode, step, x_add;
};

// Role: 0 mass-matrix solves, 1 finest AMG level / single-level solves, 2 coarser AMG levels.
template <class T>
__device__ inline void cheb_body(const ChebArgs<T>& a, int bx, int v) {
  const int slice = bx * (kBlock / kWave) + (threadIdx.x / kWave);
  if (slice >= a.nslices) return;          // uniform per wavefront
  const int lane = threadIdx.x % kWave;
  const int L = a.lanes;
  const int q = lane / L, sub = lane % L;
  const int row = a.perm[slice * (kWave / L) + q];
  const int set = a.set_base + v * a.set_step;
  double theta = a.theta, delta = a.delta;
  if (a.cheb) {
    theta = a.cheb[2 * set];
    delta = a.cheb[2 * set + 1];
  }
  const int64_t o = int64_t(v) * a.vec;
  if (a.mode == 0) {
    if (sub != 0 || row < 0) return;
    const T dg = a.dinv[(a.dstride ? int64_t(set) * a.dstride : 0) + row];
    const T rr = a.b ? a.b[o + row] : a.r[o + row];
    if (a.b) a.r[o + row] = rr;
    const T d = T(dg * rr / T(theta));
    a.dnew[o + row] = d;
    a.x[o + row] = a.x_add ? a.x[o + row] + d : d;
    return;
  }
  const int beg = a.sptr[slice];
  const int w = (a.sptr[slice + 1] - beg) / kWave;
  const T* val = a.val + (a.vstride ? int64_t(set) * a.vstride : 0) + beg + lane;
  const int* col = a.col + beg + lane;
  const T* d0 = a.dold + o;
  T sum = sell_row<T, T, T>(val, col, d0, w);
  sum = group_sum(sum, L);
  if (sub != 0 || row < 0) return;
  const T rn = a.r[o + row] - sum;
  a.r[o + row] = rn;
  if (a.mode == 2) return;
  const T dg = a.dinv[(a.dstride ? int64_t(set) * a.dstride : 0) + row];
  // Chebyshev recurrence coefficients for step `step`
  ChebRec cr(theta, delta);
  double k1 = 0.0, k2 = 0.0;
  for (int i = 1; i <= a.step; ++i) cr.next(k1, k2);
  const T c1 = T(k1), c2 = T(k2);
  const T d = c1 * d0[row] + c2 * dg * rn;
  a.dnew[o + row] = d;
  a.x[o + row] += d;
}

template <class T, int Role>
__global__ ST_LATENCY_KERNEL void k_cheb(ChebArgs<T> a) {
  cheb_body<T>(a, blockIdx.x, blockIdx.y);
}

// ------------------------------------------------------------ stencils ---
// Operator on a structured node grid, 5x5 neighbourhood per component pair.
template <class T>
struct StOp {
  const T* coef;        // [set][slot][row]
  int64_t set_stride;   // nslot * rows (0 = shared)
  int gx, gy, ncomp, diag_comp, nslot;
  int cgx, cgy, shift;  // column grid (node (ii, jj) at row-grid position (ii + shift, jj + shift))
  int64_t rows;
};

// Raw buffer access (CDNA buffer resource over [base, base + bytes)): the
// base lives in scalar registers, each lane supplies a 32-bit byte offset and
// a wavefront-uniform byte offset can ride in a scalar register, so a load
// needs no 64-bit address arithmetic per lane.  Offsets past `bytes` read 0.
typedef unsigned int st_u32x2 __attribute__((ext_vector_type(2)));
constexpr int kBufFlags = 0x00020000;   // dword 3 of the resource: 32-bit raw data

__device__ inline __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, int(bytes), kBufFlags);
}
template <class T>
__device__ inline T buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff);
template <>
__device__ inline float buf_ld<float>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, int(voff), int(soff), 0));
}
template <>
__device__ inline double buf_ld<double>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, int(voff), int(soff), 0));
}
template <class T>
__device__ inline void buf_st(__amdgpu_buffer_rsrc_t r, uint32_t voff, T v);
template <>
__device__ inline void buf_st<float>(__amdgpu_buffer_rsrc_t r, uint32_t voff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, int(voff), 0, 0);
}
template <>
__device__ inline void buf_st<double>(__amdgpu_buffer_rsrc_t r, uint32_t voff, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(st_u32x2, v), r, int(voff), 0, 0);
}

// (A x)[row] for a stencil operator of radius RAD with NCC column components
// summed (1, or 2 for the coupled velocity components); every coefficient and
// neighbour load is independent of the others (one memory round trip).
// Neighbours outside the column grid have zero coefficients; their (clamped)
// addresses stay inside x.  The coefficient planes of the row's value set and
// x are read through buffer resources: the plane offset is uniform (scalar),
// the row's byte offset and the neighbours' are 32-bit (a set of planes and x
// stay below 4 GB).
template <int RAD, int NCC, class T, class TA>
__device__ inline TA stencil_row_n(const StOp<T>& A, int set, int64_t row, const T* __restrict__ x) {
  constexpr int W = 2 * RAD + 1, NS = W * W;
  constexpr uint32_t B = uint32_t(sizeof(T));
  const uint32_t per = uint32_t(A.gx) * uint32_t(A.gy), cper = uint32_t(A.cgx) * uint32_t(A.cgy);
  const uint32_t r32 = uint32_t(row);
  const uint32_t c = r32 / per;
  const uint32_t rem = r32 - c * per;
  const int i = int(rem % uint32_t(A.gx)) - A.shift, j = int(rem / uint32_t(A.gx)) - A.shift;
  const uint32_t rows = uint32_t(A.rows);
  const __amdgpu_buffer_rsrc_t rc =
      buf_rsrc(A.coef + (A.set_stride ? int64_t(set) * A.set_stride : 0), uint32_t(A.nslot) * rows * B);
  const __amdgpu_buffer_rsrc_t rx = buf_rsrc(x, uint32_t(A.ncomp) * cper * B);
  const uint32_t rb = r32 * B;
  uint32_t off[NS];
  int xs[W];
#pragma unroll
  for (int dx = -RAD; dx <= RAD; ++dx) xs[dx + RAD] = min(max(i + dx, 0), A.cgx - 1);
#pragma unroll
  for (int dy = -RAD; dy <= RAD; ++dy) {
    const int jj = min(max(j + dy, 0), A.cgy - 1) * A.cgx;
#pragma unroll
    for (int dx = -RAD; dx <= RAD; ++dx) off[(dy + RAD) * W + dx + RAD] = uint32_t(jj + xs[dx + RAD]);
  }
  T cv[NCC][NS], xv[NCC][NS];
#pragma unroll
  for (int q = 0; q < NCC; ++q) {
    const uint32_t cb = (NCC == 1 && A.diag_comp ? c : uint32_t(q)) * cper;
#pragma unroll
    for (int o = 0; o < NS; ++o) {
      cv[q][o] = buf_ld<T>(rc, rb, uint32_t(q * NS + o) * rows * B);
      xv[q][o] = buf_ld<T>(rx, (cb + off[o]) * B, 0u);
    }
  }
  // one partial sum per column component, then their sum (the order every
  // form of this product keeps, so that they agree bit for bit)
  TA acc = TA(0);
#pragma unroll
  for (int q = 0; q < NCC; ++q) {
    TA part = TA(0);
#pragma unroll
    for (int o = 0; o < NS; ++o) part += TA(cv[q][o]) * TA(xv[q][o]);
    acc = q == 0 ? part : acc + part;
  }
  return acc;
}

// The same for a two-component operator with the row's two column
// components on two neighbouring lanes (lane 2t + q sums component q of row
// t): half the loads per lane, then the partial sums are exchanged, so both
// lanes return the sum partial_0 + partial_1 of the one-lane form.
template <int RAD, class T>
__device__ inline T stencil_row_2lane(const StOp<T>& A, int set, int64_t row, const T* __restrict__ x, int q) {
  constexpr int W = 2 * RAD + 1, NS = W * W;
  constexpr uint32_t B = uint32_t(sizeof(T));
  const uint32_t per = uint32_t(A.gx) * uint32_t(A.gy), cper = uint32_t(A.cgx) * uint32_t(A.cgy);
  const uint32_t r32 = uint32_t(row);
  const uint32_t c = r32 / per;
  const uint32_t rem = r32 - c * per;
  const int i = int(rem % uint32_t(A.gx)) - A.shift, j = int(rem / uint32_t(A.gx)) - A.shift;
  const uint32_t rows = uint32_t(A.rows);
  const __amdgpu_buffer_rsrc_t rc =
      buf_rsrc(A.coef + (A.set_stride ? int64_t(set) * A.set_stride : 0), uint32_t(A.nslot) * rows * B);
  const __amdgpu_buffer_rsrc_t rx = buf_rsrc(x, uint32_t(A.ncomp) * cper * B);
  const uint32_t rb = (uint32_t(q) * uint32_t(NS) * rows + r32) * B;
  const uint32_t cb = uint32_t(q) * cper;
  uint32_t off[NS];
  int xs[W];
#pragma unroll
  for (int dx = -RAD; dx <= RAD; ++dx) xs[dx + RAD] = min(max(i + dx, 0), A.cgx - 1);
#pragma unroll
  for (int dy = -RAD; dy <= RAD; ++dy) {
    const int jj = min(max(j + dy, 0), A.cgy - 1) * A.cgx;
#pragma unroll
    for (int dx = -RAD; dx <= RAD; ++dx) off[(dy + RAD) * W + dx + RAD] = uint32_t(jj + xs[dx + RAD]);
  }
  T cv[NS], xv[NS];
#pragma unroll
  for (int o = 0; o < NS; ++o) {
    cv[o] = buf_ld<T>(rc, rb, uint32_t(o) * rows * B);
    xv[o] = buf_ld<T>(rx, (cb + off[o]) * B, 0u);
  }
  T part = T(0);
#pragma unroll
  for (int o = 0; o < NS; ++o) part += cv[o] * xv[o];
  const T other = __shfl_xor(part, 1);
  return q == 0 ? part + other : other + part;
}

// The same for any operator: one column component (diagonal-component
// operators included) or two.
template <int RAD, class T, class TA>
__device__ inline TA stencil_row(const StOp<T>& A, int set, int64_t row, const T* __restrict__ x) {
  if (A.diag_comp || A.ncomp == 1) return stencil_row_n<RAD, 1, T, TA>(A, set, row, x);
  return stencil_row_n<RAD, 2, T, TA>(A, set, row, x);
}

// Row product with one lane per row, or (lanes == 2, two-component operators)
// component q of the row on this lane; the same value either way.
template <class T>
__device__ inline T stencil_row_lanes(const StOp<T>& A, int set, int64_t row, const T* __restrict__ x, int lanes,
                                      int q) {
  if (lanes == 2) return stencil_row_2lane<2, T>(A, set, row, x, q);
  return stencil_row<2, T, T>(A, set, row, x);
}

// First step of a sweep solve with Chebyshev-Jacobi alone, fused with the
// sweep right-hand side: r = q + a1 S1 y1 + a2 S2 y2, d = Dinv r/theta and
// x = x0 + d, where the predictor x0 = g1 y1 + g2 y2 (guess != 0) or 0.  With a
// predictor the couplings S1, S2 already contain the diagonal block's action
// on it, so that r is the residual of x0.  A third term g3 y3 (g3 != 0) is
// added to x only, not to the predictor r belongs to: a Parareal correction.
template <class T>
struct StInitArgs {
  StOp<T> S1, S2;
  int set1, set2, n1, n2;   // n1/n2: whether the couplings are active
  double a1, a2;
  const T* y1;
  const T* y2;
  const T* q;
  const T* dinv;
  double theta;
  T* r;
  T* d;
  T* x;
  int64_t rows;
  int guess;
  double g1, g2;
  int rpb;              // rows per workgroup (lanes * rpb <= kBlock; fewer spread a small grid over more CUs)
  int lanes;            // 1, or 2 for two-component operators: a row's components on two lanes
  const T* y3;
  double g3;
};

template <class T>
__device__ inline void st_init_body(const StInitArgs<T>& a, int bx) {
  const int lq = a.lanes == 2 ? int(threadIdx.x & 1) : 0;
  const int t = a.lanes == 2 ? int(threadIdx.x >> 1) : int(threadIdx.x);
  if (t >= a.rpb) return;
  const int64_t row = int64_t(bx) * a.rpb + t;
  if (row >= a.rows) return;   // both lanes of a row leave together
  const uint32_t vb = uint32_t(a.rows) * uint32_t(sizeof(T)), ro = uint32_t(row) * uint32_t(sizeof(T));
  T acc = buf_ld<T>(buf_rsrc(a.q, vb), ro, 0u);
  const T dg = buf_ld<T>(buf_rsrc(a.dinv, vb), ro, 0u);
  if (a.n1) acc += T(a.a1) * stencil_row_lanes<T>(a.S1, a.set1, row, a.y1, a.lanes, lq);
  if (a.n2) acc += T(a.a2) * stencil_row_lanes<T>(a.S2, a.set2, row, a.y2, a.lanes, lq);
  const T d = dg * acc / T(a.theta);
  T x0 = T(0);
  if (a.guess) {
    x0 = T(a.g1) * buf_ld<T>(buf_rsrc(a.y1, vb), ro, 0u);
    if (a.g2 != 0.0) x0 += T(a.g2) * buf_ld<T>(buf_rsrc(a.y2, vb), ro, 0u);
    if (a.g3 != 0.0) x0 += T(a.g3) * buf_ld<T>(buf_rsrc(a.y3, vb), ro, 0u);
  }
  if (lq) return;
  buf_st<T>(buf_rsrc(a.r, vb), ro, acc);
  buf_st<T>(buf_rsrc(a.d, vb), ro, d);
  buf_st<T>(buf_rsrc(a.x, vb), ro, x0 + d);
}

template <class T, int Role>
__global__ ST_LATENCY_KERNEL void k_st_init(StInitArgs<T> a) {
  st_init_body<T>(a, blockIdx.x);
}

// Chebyshev step i >= 1 on a stencil operator: r -= A d_old; d_new = c1 d_old + c2 Dinv r; x += d_new.
template <class T>
struct StChebArgs {
  StOp<T> A;
  int set;
  const T* dinv;
  double c1, c2;
  const T* dold;
  T* dnew;
  T* r;
  T* x;
  int64_t rows;
  int rpb;              // rows per workgroup (lanes * rpb <= kBlock)
  int lanes;            // 1, or 2 for a two-component operator (see StInitArgs)
};

template <class T>
__device__ inline void st_cheb_body(const StChebArgs<T>& a, int bx) {
  const int lq = a.lanes == 2 ? int(threadIdx.x & 1) : 0;
  const int tr = a.lanes == 2 ? int(threadIdx.x >> 1) : int(threadIdx.x);
  if (tr >= a.rpb) return;
  const int64_t row = int64_t(bx) * a.rpb + tr;
  if (row >= a.rows) return;   // both lanes of a row leave together
  const uint32_t vb = uint32_t(a.rows) * uint32_t(sizeof(T)), ro = uint32_t(row) * uint32_t(sizeof(T));
  const __amdgpu_buffer_rsrc_t rd = buf_rsrc(a.dold, vb), rg = buf_rsrc(a.dinv, vb), rr_ = buf_rsrc(a.r, vb),
                               rn_ = buf_rsrc(a.dnew, vb), rx = buf_rsrc(a.x, vb);
  const T od = buf_ld<T>(rd, ro, 0u);
  const T dg = buf_ld<T>(rg, ro, 0u);
  const T rr = buf_ld<T>(rr_, ro, 0u);
  const T xo = buf_ld<T>(rx, ro, 0u);
  const T t = stencil_row_lanes<T>(a.A, a.set, row, a.dold, a.lanes, lq);
  const T rn = rr - t;
  const T d = T(a.c1) * od + T(a.c2) * dg * rn;
  if (lq) return;
  buf_st<T>(rr_, ro, rn);
  buf_st<T>(rn_, ro, d);
  buf_st<T>(rx, ro, xo + d);
}

template <class T, int Role>
__global__ ST_LATENCY_KERNEL void k_st_cheb(StChebArgs<T> a) {
  st_cheb_body<T>(a, blockIdx.x);
}

// A Chebyshev-Jacobi sweep solve (or a run of its steps) on a stencil
// operator in one launch, with no memory round trip between steps.  Each
// workgroup owns a tx x ty tile of nodes (every component) and works on the
// tile grown by a halo: a step's r and d are valid on a region one stencil
// radius smaller than the d it reads, so with h = radius x (stencil
// applications still to come) the last step of the launch is exact on the
// tile.  The grown tile's r and the two d iterates live in LDS; only x (and r
// with the last d when a later launch continues the solve) are written back.
// A continuing launch reads r and d from other buffers than those it writes,
// since its grown tile overlaps the tiles of other workgroups.
// Overlapping tiles repeat the halo work of their neighbours: with 8 x 8
// tiles and a radius-2 stencil, four steps compute 20 x 20, 16 x 16, 12 x 12
// and 8 x 8 nodes per tile.  Step 0 is st_init_body's arithmetic (residual of
// the predictor) and step i >= 1 st_cheb_body's, in the same order, so the
// result is that of the step-by-step launches.
constexpr int kSolveBlock = 512;   // threads per workgroup of the tiled solve
// No cap on the registers: capped at 128 VGPRs (two workgroups per CU) the
// kernel spills and is no faster (measured).
#define ST_SOLVE_KERNEL __launch_bounds__(kSolveBlock)
constexpr int kTileExt = 400;   // nodes of a grown tile per component (LDS capacity)
constexpr int kTileOut = 64;    // nodes of a tile per component
constexpr int kTileComp = 2;

template <class T>
struct StSolveArgs {
  StInitArgs<T> in;   // step 0; x, dinv, theta, rows; r and d receive r and the
                      // last d when a later launch continues the solve
  StOp<T> A;          // the diagonal block (row grid = column grid)
  int set;
  double delta;
  const T* r_in;      // s0 > 0: r and d_{s0-1} written by the previous launch
  const T* d_in;
  int s0, ns;         // steps [s0, s0 + ns) of the solve
  int tx, ty, ntx;    // tile size and tiles per grid row
  int more;           // 1: a later launch continues (write r and the last d)
};

// (A d)[row] for a radius-2 stencil with d held in LDS over the grown tile
// whose corner is grid node (ex0, ey0); neighbour addresses clamp to the grid
// exactly as stencil_row's do (the clamped node lies in the grown tile).
template <int NCC, class T>
__device__ inline T stencil_row_lds_n(const StOp<T>& A, int set, int64_t row, int c, int i, int j, const T* sdv,
                                      int ew, int ea, int ex0, int ey0) {
  constexpr int RAD = 2, W = 2 * RAD + 1, NS = W * W;
  const T* __restrict__ cf = A.coef + (A.set_stride ? int64_t(set) * A.set_stride : 0) + row;
  int off[NS];
#pragma unroll
  for (int dy = -RAD; dy <= RAD; ++dy) {
    const int jj = min(max(j + dy, 0), A.gy - 1) - ey0;
#pragma unroll
    for (int dx = -RAD; dx <= RAD; ++dx)
      off[(dy + RAD) * W + dx + RAD] = jj * ew + min(max(i + dx, 0), A.gx - 1) - ex0;
  }
  T cv[NCC][NS], xv[NCC][NS];
#pragma unroll
  for (int q = 0; q < NCC; ++q) {
    const T* xc = sdv + (NCC == 1 && A.diag_comp ? c : q) * ea;
    const T* __restrict__ cq = cf + int64_t(q) * NS * A.rows;
#pragma unroll
    for (int o = 0; o < NS; ++o) {
      cv[q][o] = cq[int64_t(o) * A.rows];
      xv[q][o] = xc[off[o]];
    }
  }
  T acc = T(0);
#pragma unroll
  for (int q = 0; q < NCC; ++q) {
    T part = T(0);
#pragma unroll
    for (int o = 0; o < NS; ++o) part += cv[q][o] * xv[q][o];
    acc = q == 0 ? part : acc + part;
  }
  return acc;
}

template <class T>
__device__ inline T stencil_row_lds(const StOp<T>& A, int set, int64_t row, int c, int i, int j, const T* sdv,
                                    int ew, int ea, int ex0, int ey0) {
  if (A.diag_comp || A.ncomp == 1) return stencil_row_lds_n<1, T>(A, set, row, c, i, j, sdv, ew, ea, ex0, ey0);
  return stencil_row_lds_n<2, T>(A, set, row, c, i, j, sdv, ew, ea, ex0, ey0);
}

template <class T>
__device__ inline void st_solve_body(const StSolveArgs<T>& a, int bx) {
  constexpr int RAD = 2;
  __shared__ T sr[kTileComp * kTileExt];
  __shared__ T sd[2][kTileComp * kTileExt];
  __shared__ T sx[kTileComp * kTileOut];
  const StInitArgs<T>& in = a.in;
  const int gx = a.A.gx, gy = a.A.gy, nc = a.A.ncomp;
  const int per = gx * gy;
  const int tyi = bx / a.ntx, txi = bx - tyi * a.ntx;
  const int X0 = txi * a.tx, Y0 = tyi * a.ty;
  const int s0 = a.s0, s1 = a.s0 + a.ns;       // steps [s0, s1)
  const int H = RAD * (a.ns - (s0 == 0 ? 1 : 0));
  const int ew = a.tx + 2 * H, ea = ew * (a.ty + 2 * H);
  const int ex0 = X0 - H, ey0 = Y0 - H;
  const int ta = a.tx * a.ty;
  ChebRec cr(in.theta, a.delta);
  double k1 = 0.0, k2 = 0.0;
  for (int i = 1; i < s0; ++i) cr.next(k1, k2);
  // A continued solve reads d_{s0-1} on the whole grown tile, r and x where
  // its first step computes.
  if (s0 > 0) {
    const int xa = max(ex0, 0), xb = min(ex0 + ew, gx), ya = max(ey0, 0), yb = min(ey0 + ea / ew, gy);
    const int w = xb - xa, n = nc * w * (yb - ya);
    for (int e = threadIdx.x; e < n; e += kSolveBlock) {
      const int c = e / (w * (yb - ya)), rem = e - c * w * (yb - ya);
      const int j = ya + rem / w, i = xa + rem % w;
      const int64_t row = int64_t(c) * per + int64_t(j) * gx + i;
      const int l = c * ea + (j - ey0) * ew + (i - ex0);
      sd[(s0 - 1) & 1][l] = a.d_in[row];
      sr[l] = a.r_in[row];
      if (i >= X0 && i < X0 + a.tx && j >= Y0 && j < Y0 + a.ty)
        sx[c * ta + (j - Y0) * a.tx + (i - X0)] = in.x[row];
    }
    __syncthreads();
  }
  for (int s = s0; s < s1; ++s) {
    const int h = RAD * (s1 - 1 - s);
    const int xa = max(X0 - h, 0), xb = min(X0 + a.tx + h, gx), ya = max(Y0 - h, 0), yb = min(Y0 + a.ty + h, gy);
    const int w = xb - xa, wh = w * (yb - ya), n = nc * wh;
    const bool last = s == s1 - 1;
    T c1 = T(0), c2 = T(0);
    if (s >= 1) {
      cr.next(k1, k2);
      c1 = T(k1);
      c2 = T(k2);
    }
    for (int e = threadIdx.x; e < n; e += kSolveBlock) {
      const int c = e / wh, rem = e - c * wh;
      const int j = ya + rem / w, i = xa + rem % w;
      const int64_t row = int64_t(c) * per + int64_t(j) * gx + i;
      const int l = c * ea + (j - ey0) * ew + (i - ex0);
      const bool tile = i >= X0 && i < X0 + a.tx && j >= Y0 && j < Y0 + a.ty;
      const int tl = c * ta + (j - Y0) * a.tx + (i - X0);
      T rn, d, xn = T(0);
      if (s == 0) {
        T acc = in.q[row];
        if (in.n1) acc += T(in.a1) * stencil_row<2, T, T>(in.S1, in.set1, row, in.y1);
        if (in.n2) acc += T(in.a2) * stencil_row<2, T, T>(in.S2, in.set2, row, in.y2);
        d = in.dinv[row] * acc / T(in.theta);
        rn = acc;
        if (tile) {
          T x0 = T(0);
          if (in.guess) {
            x0 = T(in.g1) * in.y1[row];
            if (in.g2 != 0.0) x0 += T(in.g2) * in.y2[row];
            if (in.g3 != 0.0) x0 += T(in.g3) * in.y3[row];
          }
          xn = x0 + d;
        }
      } else {
        const T* sdo = sd[(s - 1) & 1];
        const T od = sdo[l];
        const T dg = in.dinv[row];
        const T t = stencil_row_lds<T>(a.A, a.set, row, c, i, j, sdo, ew, ea, ex0, ey0);
        rn = sr[l] - t;
        d = c1 * od + c2 * dg * rn;
        if (tile) xn = sx[tl] + d;
      }
      if (last) {
        // the last step runs on the tile only
        in.x[row] = xn;
        if (a.more) {
          in.r[row] = rn;
          in.d[row] = d;
        }
      } else {
        sr[l] = rn;
        sd[s & 1][l] = d;
        if (tile) sx[tl] = xn;
      }
    }
    if (!last) __syncthreads();
  }
}

template <class T, int Role>
__global__ ST_SOLVE_KERNEL void k_st_solve(StSolveArgs<T> a) {
  st_solve_body<T>(a, blockIdx.x);
}

// The C_A sweep for slabs [k0, k1) in one workgroup, each slab followed by
// its current solve y_j = M_j^{-1}(r_j - K_jA y_A): Chebyshev-Jacobi of degree
// `deg` on C_A,k for the increment over the predictor (y^0 for slab 1,
// 2 y^{k-1} - y^{k-2} after; first step fused with the residual
// s^k + P_k y^{k-1} + Q_k y^{k-2} of the predictor) and of degree `mit` on
// M_j.  Only workgroup barriers: no inter-workgroup synchronisation.  Every
// operator here is a one-component stencil (checked where the kernel is
// chosen).
template <class T>
struct ChainArgs {
  StOp<T> C0, CP, CQ, Mj, KjA;
  int k0, k1, deg, mit, na, nj;
  double dt;
  const double* alone;  // (theta, delta) per slab for C_A
  const T* dinvC;       // [nt][na] (or shared when dinv_stride = 0)
  int64_t dinv_stride;
  const T* dinvM;       // [nj]
  double mth, mde;      // M_j interval
  const T* sA;
  T* yA;
  const T* rj;
  T* yj;
  T* r;
  T* d0;
  T* d1;
};

constexpr int kChainBlock = 1024;

template <class T>
__global__ __launch_bounds__(kChainBlock) void k_ca_chain(ChainArgs<T> a) {
  const int tid = threadIdx.x;
  const int na = a.na, nj = a.nj;
  for (int k = a.k0; k < a.k1; ++k) {
    const double theta = a.alone[2 * k], delta = a.alone[2 * k + 1];
    const T* dinv = a.dinvC + int64_t(k) * a.dinv_stride;
    T* yk = a.yA + int64_t(k) * na;
    const T* sk = a.sA + int64_t(k) * na;
    for (int row = tid; row < na; row += kChainBlock) {
      T acc = sk[row];
      T x0 = T(0);
      if (k >= 1) {
        const T* y1 = a.yA + int64_t(k - 1) * na;
        acc += stencil_row_n<2, 1, T, T>(a.CP, k, row, y1);
        x0 = y1[row];
      }
      if (k >= 2) {
        const T* y2 = a.yA + int64_t(k - 2) * na;
        acc += stencil_row_n<2, 1, T, T>(a.CQ, k, row, y2);
        x0 = T(2) * x0 - y2[row];
      }
      const T dd = dinv[row] * acc / T(theta);
      a.r[row] = acc;
      a.d0[row] = dd;
      yk[row] = x0 + dd;
    }
    __syncthreads();
    {
      ChebRec cr(theta, delta);
      for (int i = 1; i < a.deg; ++i) {
        double k1, k2;
        cr.next(k1, k2);
        const T c1 = T(k1), c2 = T(k2);
        const T* dold = (i - 1) % 2 ? a.d1 : a.d0;
        T* dnew = i % 2 ? a.d1 : a.d0;
        for (int row = tid; row < na; row += kChainBlock) {
          const T od = dold[row], dg = dinv[row], rr = a.r[row];
          const T rn = rr - stencil_row_n<2, 1, T, T>(a.C0, k, row, dold);
          const T dn = c1 * od + c2 * dg * rn;
          a.r[row] = rn;
          dnew[row] = dn;
          yk[row] += dn;
        }
        __syncthreads();
      }
    }
    // current: y_j = M_j^{-1} (r_j - K_jA y_A^k)
    T* jk = a.yj + int64_t(k) * nj;
    const T* rjk = a.rj + int64_t(k) * nj;
    for (int row = tid; row < nj; row += kChainBlock) {
      const T acc = rjk[row] - stencil_row_n<1, 1, T, T>(a.KjA, 0, row, yk);
      const T dd = a.dinvM[row] * acc / T(a.mth);
      a.r[row] = acc;
      a.d0[row] = dd;
      jk[row] = dd;
    }
    __syncthreads();
    {
      ChebRec cr(a.mth, a.mde);
      for (int i = 1; i < a.mit; ++i) {
        double k1, k2;
        cr.next(k1, k2);
        const T c1 = T(k1), c2 = T(k2);
        const T* dold = (i - 1) % 2 ? a.d1 : a.d0;
        T* dnew = i % 2 ? a.d1 : a.d0;
        for (int row = tid; row < nj; row += kChainBlock) {
          const T od = dold[row], dg = a.dinvM[row], rr = a.r[row];
          const T rn = rr - stencil_row_n<1, 1, T, T>(a.Mj, 0, row, dold);
          const T dn = c1 * od + c2 * dg * rn;
          a.r[row] = rn;
          dnew[row] = dn;
          jk[row] += dn;
        }
        __syncthreads();
      }
    }
  }
}

// Coarsest AMG level: x[v] (+)= Ainv(set) * b[v]; Ainv stored column-major.
constexpr int kMaxCoarse = 512;

template <class T>
struct CoarseArgs {
  int n;                // coarse size, <= kMaxCoarse
  const T* inv;
  int64_t istride;      // per-set stride of the inverses (0 = shared)
  int set_base, set_step;
  const T* b;
  T* x;
  int64_t vec;
  int accumulate;
};

template <class T>
__device__ inline void coarse_body(const CoarseArgs<T>& a, int v) {
  __shared__ T sb[kMaxCoarse];
  const int n = a.n;
  const int set = a.set_base + v * a.set_step;
  const T* A = a.inv + (a.istride ? int64_t(set) * a.istride : 0);
  for (int i = threadIdx.x; i < n; i += blockDim.x) sb[i] = a.b[int64_t(v) * a.vec + i];
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    T s = T(0);
    for (int j = 0; j < n; ++j) s += A[int64_t(j) * n + i] * sb[j];
    T* xp = a.x + int64_t(v) * a.vec + i;
    *xp = a.accumulate ? *xp + s : s;
  }
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_coarse(CoarseArgs<T> a) {
  coarse_body<T>(a, blockIdx.x);
}

// ----------------------------------------------------------- reductions ---
__device__ inline double wave_sum(double v) {
  for (int off = kWave / 2; off > 0; off /= 2) v += __shfl_down(v, off, kWave);
  return v;
}

// Block-wide sum of one double; result valid in thread 0.
__device__ inline double block_sum(double v) {
  __shared__ double part[kBlock / kWave];
  v = wave_sum(v);
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  if (l == 0) part[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kBlock / kWave; ++i) s += part[i];
  __syncthreads();
  return s;
}

}  // namespace st
