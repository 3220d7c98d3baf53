// HIP kernels of libst (gfx950, wave64).  Everything here is sparse or vector
// work bound by HBM bandwidth or launch latency: no MFMA.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace st {

constexpr int kWave = 64;        // CDNA wavefront = one SELL slice
constexpr int kBlock = 256;      // 4 slices per workgroup

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

template <class TA>
__device__ inline TA group_sum(TA v, int lanes) {
  for (int off = lanes / 2; off > 0; off /= 2) v += __shfl_down(v, off, lanes);
  return v;
}

// y[v][row] = sum_seg alpha_seg (A_seg x_seg)[row] + beta b[v][row]
template <class T, class TX, class TA, int Role>
__global__ __launch_bounds__(kBlock) void k_spmv(SpmvArgs<T, TX> a) {
  const int v = blockIdx.y;
  const int slice = blockIdx.x * (kBlock / kWave) + (threadIdx.x / kWave);
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
    TA sum = TA(0);
    for (int j = 0; j < w; ++j) sum += TA(val[j * kWave]) * TA(x[col[j * kWave]]);
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
template <class T, int Role>
__global__ __launch_bounds__(kBlock) void k_cheb(ChebArgs<T> a) {
  const int v = blockIdx.y;
  const int slice = blockIdx.x * (kBlock / kWave) + (threadIdx.x / kWave);
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
  T sum = T(0);
  for (int j = 0; j < w; ++j) sum += val[j * kWave] * d0[col[j * kWave]];
  sum = group_sum(sum, L);
  if (sub != 0 || row < 0) return;
  const T rn = a.r[o + row] - sum;
  a.r[o + row] = rn;
  if (a.mode == 2) return;
  const T dg = a.dinv[(a.dstride ? int64_t(set) * a.dstride : 0) + row];
  // Chebyshev recurrence coefficients for step `step` (rho_0 = delta/theta).
  const double sigma = theta / delta;
  double rho_prev = 1.0 / sigma, rho = rho_prev;
  for (int i = 1; i <= a.step; ++i) {
    rho_prev = rho;
    rho = 1.0 / (2.0 * sigma - rho_prev);
  }
  const T c1 = T(rho * rho_prev), c2 = T(2.0 * rho / delta);
  const T d = c1 * d0[row] + c2 * dg * rn;
  a.dnew[o + row] = d;
  a.x[o + row] += d;
}

// Coarsest AMG level: x[v] (+)= Ainv(set) * b[v]; Ainv stored column-major.
template <class T>
__global__ __launch_bounds__(kBlock) void k_coarse(int n, const T* inv, int64_t istride, int set_base, int set_step,
                                                    const T* b, T* x, int64_t vec, int accumulate) {
  __shared__ T sb[512];
  const int v = blockIdx.x;
  const int set = set_base + v * set_step;
  const T* A = inv + (istride ? int64_t(set) * istride : 0);
  for (int i = threadIdx.x; i < n; i += blockDim.x) sb[i] = b[int64_t(v) * vec + i];
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    T s = T(0);
    for (int j = 0; j < n; ++j) s += A[int64_t(j) * n + i] * sb[j];
    T* xp = x + int64_t(v) * vec + i;
    *xp = accumulate ? *xp + s : s;
  }
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
