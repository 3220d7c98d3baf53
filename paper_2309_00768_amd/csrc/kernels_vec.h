// Vector kernels of libst: the precision boundary and pressure handling of
// P_T^{-1}, and the FGMRES building blocks (multi-dot, Gram-Schmidt update,
// Givens rotations, back substitution).  Each kernel is a device body taking
// explicit workgroup coordinates (bx, by) and the x-extent gx of its grid,
// plus a thin __global__ wrapper, so that the batched launcher can run the
// same body for several systems in one launch.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "kernels.h"

namespace st {

// A recorded preconditioner program reads its input and output vectors from a
// device slot (set by k_set_ptrs before the program runs); otherwise the
// pointers in the arguments are used.
template <class P>
__device__ inline P slot_or(P const* slot, P direct) {
  return slot ? *slot : direct;
}

// Per-slab sums of src[k*ld + off + i], i < len (weights w[i] if w): out[k]; bx = k.
struct SlabSumsDArgs {
  const double* src;
  int64_t ld;
  int off, len;
  const double* w;
  double* out;
  const double* const* rslot;
};

__device__ inline void slab_sums_d_body(const SlabSumsDArgs& a, int k) {
  const double* p = slot_or(a.rslot, a.src) + int64_t(k) * a.ld + a.off;
  double acc = 0.0;
  for (int i = threadIdx.x; i < a.len; i += blockDim.x) acc += (a.w ? a.w[i] : 1.0) * p[i];
  acc = block_sum(acc);
  if (threadIdx.x == 0) a.out[k] = acc;
}

template <class T>
struct SlabSumsTArgs {
  const T* src;
  int64_t ld;
  int len;
  const double* w;
  double* out;
};

template <class T>
__device__ inline void slab_sums_t_body(const SlabSumsTArgs<T>& a, int k) {
  const T* p = a.src + int64_t(k) * a.ld;
  double acc = 0.0;
  for (int i = threadIdx.x; i < a.len; i += blockDim.x) acc += (a.w ? a.w[i] : 1.0) * double(p[i]);
  acc = block_sum(acc);
  if (threadIdx.x == 0) a.out[k] = acc;
}

// Split an FP64 slab-major vector into per-block arrays (precision T); the
// pressure rows lose their per-slab mean psum[k] / np.
template <class T>
struct SplitArgs {
  const double* r;
  int ns, nt, o2, o3, o4;
  const double* psum;
  T *ru, *rp, *rj, *ra;
  const double* const* rslot;
};

template <class T>
__device__ inline void split_body(const SplitArgs<T>& a, int bx, int gx) {
  const int64_t N = int64_t(a.ns) * a.nt;
  const int ns = a.ns, o2 = a.o2, o3 = a.o3, o4 = a.o4;
  const int np = o3 - o2, nj = o4 - o3, na = ns - o4;
  const double* r = slot_or(a.rslot, a.r);
  for (int64_t i = bx * int64_t(kBlock) + threadIdx.x; i < N; i += int64_t(gx) * kBlock) {
    const int k = int(i / ns), c = int(i % ns);
    const double v = r[i];
    if (c < o2) a.ru[int64_t(k) * o2 + c] = T(v);
    else if (c < o3) a.rp[int64_t(k) * np + (c - o2)] = T(v - a.psum[k] / np);
    else if (c < o4) a.rj[int64_t(k) * nj + (c - o3)] = T(v);
    else a.ra[int64_t(k) * na + (c - o4)] = T(v);
  }
}

// Join per-block arrays into an FP64 slab-major vector; pressure is
// psign * xp shifted so that 1^T M_p p^k = 0 (wsum[k] = m . xp^k, msum = sum m).
template <class T>
struct JoinArgs {
  double* z;
  int ns, nt, o2, o3, o4;
  const T* xu;
  const T* xp;
  double psign;
  const double* wsum;
  double msum;
  const T* yj;
  const T* ya;
  double* const* zslot;
};

template <class T>
__device__ inline void join_body(const JoinArgs<T>& a, int bx, int gx) {
  const int64_t N = int64_t(a.ns) * a.nt;
  const int ns = a.ns, o2 = a.o2, o3 = a.o3, o4 = a.o4;
  const int np = o3 - o2, nj = o4 - o3, na = ns - o4;
  double* z = slot_or(a.zslot, a.z);
  for (int64_t i = bx * int64_t(kBlock) + threadIdx.x; i < N; i += int64_t(gx) * kBlock) {
    const int k = int(i / ns), c = int(i % ns);
    double v;
    if (c < o2) v = double(a.xu[int64_t(k) * o2 + c]);
    else if (c < o3) v = a.psign * (double(a.xp[int64_t(k) * np + (c - o2)]) - a.wsum[k] / a.msum);
    else if (c < o4) v = double(a.yj[int64_t(k) * nj + (c - o3)]);
    else v = double(a.ya[int64_t(k) * na + (c - o4)]);
    z[i] = v;
  }
}

// x[k*ld + i] -= sums[k] * scale (i < len)
template <class T>
struct SlabShiftArgs {
  T* x;
  int64_t ld;
  int len, nt;
  const double* sums;
  double scale;
};

template <class T>
__device__ inline void slab_shift_body(const SlabShiftArgs<T>& a, int bx, int gx) {
  const int64_t N = int64_t(a.len) * a.nt;
  for (int64_t i = bx * int64_t(kBlock) + threadIdx.x; i < N; i += int64_t(gx) * kBlock) {
    const int k = int(i / a.len), c = int(i % a.len);
    T* p = a.x + int64_t(k) * a.ld + c;
    *p = T(double(*p) - a.sums[k] * a.scale);
  }
}

// FP64 slab-major: p rows (offset o2..o3) minus psum[k]/np, written to dst.
struct ProjectPArgs {
  const double* src;
  double* dst;
  int ns, nt, o2, o3;
  const double* psum;
};

__device__ inline void project_p_body(const ProjectPArgs& a, int bx, int gx) {
  const int64_t N = int64_t(a.ns) * a.nt;
  const int np = a.o3 - a.o2;
  for (int64_t i = bx * int64_t(kBlock) + threadIdx.x; i < N; i += int64_t(gx) * kBlock) {
    const int k = int(i / a.ns), c = int(i % a.ns);
    double v = a.src[i];
    if (c >= a.o2 && c < a.o3) v -= a.psum[k] / np;
    a.dst[i] = v;
  }
}

// partial[i * gx + bx] = sum over the workgroup's rows of V_i . w   (i = by)
struct MdotArgs {
  const double* V;
  int64_t N;
  const double* w;
  double* partial;
};

__device__ inline void mdot_body(const MdotArgs& a, int bx, int i, int gx) {
  const double* v = a.V + int64_t(i) * a.N;
  double acc = 0.0;
  for (int64_t r = bx * int64_t(kBlock) + threadIdx.x; r < a.N; r += int64_t(gx) * kBlock) acc += v[r] * a.w[r];
  acc = block_sum(acc);
  if (threadIdx.x == 0) a.partial[int64_t(i) * gx + bx] = acc;
}

// out[i] (+)= sum_b partial[i * nb + b]  (i = bx); mode 1: out[0] = sqrt(sum), mode 2: add.
struct ReduceArgs {
  const double* partial;
  int nb;
  double* out;
  int mode;
  double* copy_to;
};

__device__ inline void reduce_body(const ReduceArgs& a, int i) {
  double acc = 0.0;
  for (int b = threadIdx.x; b < a.nb; b += kBlock) acc += a.partial[int64_t(i) * a.nb + b];
  acc = block_sum(acc);
  if (threadIdx.x == 0) {
    if (a.mode == 1) acc = std::sqrt(acc);
    if (a.mode == 2) a.out[i] += acc;
    else a.out[i] = acc;
    if (a.copy_to) a.copy_to[i] = a.out[i];
  }
}

// w -= sum_{i < nv} h[i] V_i   (sign -1), or x += sum_i y[i] Z_i (sign +1)
struct CombineArgs {
  double* w;
  const double* V;
  int64_t N;
  const double* h;
  int nv;
  double sign;
};

__device__ inline void combine_body(const CombineArgs& a, int bx, int gx) {
  for (int64_t r = bx * int64_t(kBlock) + threadIdx.x; r < a.N; r += int64_t(gx) * kBlock) {
    double acc = a.w[r];
    if (a.sign < 0.0)
      for (int i = 0; i < a.nv; ++i) acc -= a.h[i] * a.V[int64_t(i) * a.N + r];
    else
      for (int i = 0; i < a.nv; ++i) acc += a.h[i] * a.V[int64_t(i) * a.N + r];
    a.w[r] = acc;
  }
}

// ------------------------------- Arnoldi with delayed reorthogonalisation ---
// Step j of a cycle holds u_j, the newest basis direction after one classical
// Gram-Schmidt pass, in V_j, and w = J z_j with z_j = P^{-1} u_j.  One read of
// the finished basis Q = V_0..V_{j-1} gives both a = Q^T u_j (the second pass
// of u_j) and b = Q^T w (the first pass of w); a second read forms
// q~ = u_j - Q a and w'' = w - Q b with ||q~||^2 and q~ . w''.  Then
// q_j = q~ / ||q~|| and u_{j+1} = w'' - (q_j . w'') q_j.  Every direction
// still gets two full passes, as in CGS2, but the basis is read twice per
// step instead of four times.
//
// The pending vector is kept at unit scale: u_{j+1} is stored as
// u_{j+1} / s_{j+1} with s_{j+1}^2 = ||w''||^2 - c^2 (its norm; ||w''|| where
// that difference loses too much to cancellation, any positive scale being
// exact), and s enters the entries that complete its Hessenberg column.
// Unscaled, the pending vector grows or shrinks by the subdiagonal entries
// step after step and leaves the floating-point range on long restarts
// when ||J P_T^{-1}|| is far from 1.

constexpr int kDotGroup = 16;   // basis vectors per workgroup of the dot pass

// partial[(2i + 0) * gx + bx] = rows of V_i . u, partial[(2i + 1) * gx + bx] =
// rows of V_i . w (0 without w), i in the workgroup's group of kDotGroup.
struct Mdot2Args {
  const double* V;
  int64_t N;
  int nv;
  const double* u;
  const double* w;   // nullptr: only V^T u
  double* partial;
};

__device__ inline void mdot2_body(const Mdot2Args& a, int bx, int grp, int gx) {
  __shared__ double part[2 * kDotGroup][kBlock / kWave];
  const int i0 = grp * kDotGroup;
  const int cnt = min(kDotGroup, a.nv - i0);
  const bool hw = a.w != nullptr;
  double au[kDotGroup], aw[kDotGroup];
#pragma unroll
  for (int g = 0; g < kDotGroup; ++g) au[g] = aw[g] = 0.0;
  const double* v0 = a.V + int64_t(i0) * a.N;
  for (int64_t r = bx * int64_t(kBlock) + threadIdx.x; r < a.N; r += int64_t(gx) * kBlock) {
    const double ur = a.u[r];
    const double wr = hw ? a.w[r] : 0.0;
#pragma unroll
    for (int g = 0; g < kDotGroup; ++g) {
      if (g < cnt) {
        const double v = v0[int64_t(g) * a.N + r];
        au[g] += v * ur;
        aw[g] += v * wr;
      }
    }
  }
  const int wv = threadIdx.x / kWave, l = threadIdx.x % kWave;
#pragma unroll
  for (int g = 0; g < kDotGroup; ++g) {
    const double su = wave_sum(au[g]), sw = wave_sum(aw[g]);
    if (l == 0) {
      part[2 * g][wv] = su;
      part[2 * g + 1][wv] = sw;
    }
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < 2 * cnt) {
    double acc = 0.0;
    for (int k = 0; k < kBlock / kWave; ++k) acc += part[t][k];
    a.partial[int64_t(2 * i0 + t) * gx + bx] = acc;
  }
}

// q~ = u - sum_i a_i V_i in place of u, w'' = w - sum_i b_i V_i into wout
// (a_i = dots[2i], b_i = dots[2i + 1], i < nv); partial[k * gx + bx] = rows of
// ||q~||^2, q~ . w'' and ||w''||^2 for k = 0, 1, 2 (the last two 0 without w).
struct UpdDelayedArgs {
  const double* V;
  int64_t N;
  int nv;
  const double* dots;
  double* u;
  const double* w;   // nullptr on the closing pass of a cycle
  double* wout;
  double* partial;
};

__device__ inline void upd_delayed_body(const UpdDelayedArgs& a, int bx, int gx) {
  double qq = 0.0, qw = 0.0, ww = 0.0;
  const bool hw = a.w != nullptr;
  for (int64_t r = bx * int64_t(kBlock) + threadIdx.x; r < a.N; r += int64_t(gx) * kBlock) {
    double su = 0.0, sw = 0.0;
#pragma unroll 4
    for (int i = 0; i < a.nv; ++i) {
      const double v = a.V[int64_t(i) * a.N + r];
      su += a.dots[2 * i] * v;
      sw += a.dots[2 * i + 1] * v;
    }
    const double q = a.u[r] - su;
    a.u[r] = q;
    qq += q * q;
    if (hw) {
      const double w2 = a.w[r] - sw;
      a.wout[r] = w2;
      qw += q * w2;
      ww += w2 * w2;
    }
  }
  qq = block_sum(qq);
  qw = block_sum(qw);
  ww = block_sum(ww);
  if (threadIdx.x == 0) {
    a.partial[bx] = qq;
    a.partial[int64_t(gx) + bx] = qw;
    a.partial[2 * int64_t(gx) + bx] = ww;
  }
}

// Hessenberg entries of step j from the reduced sums nrm = (||q~||^2, q~ . w'',
// ||w''||^2): nu = ||q~|| (1 at j = 0, where V_0 is already normalised) and
// c = q~ . w'' / nu.  With s = s_j = sm[8 + j % 2], the scale of the pending
// vector held in V_j, column j - 1 gains s a and H[j, j-1] = s nu; column j gets
// its first-pass coefficients b and H[j, j] = c (has_w), and s_{j+1} goes to
// sm[8 + (j + 1) % 2].  sm[1] = s nu, sm[3] = nu, sm[4] = c.  One workgroup.
struct FinDelayedArgs {
  const double* dots;
  const double* nrm;
  double* H;
  int ldh, j, has_w;
  double* sm;
};

__device__ inline void fin_delayed_body(const FinDelayedArgs& a) {
  const int j = a.j;
  const double nu = j == 0 ? 1.0 : std::sqrt(fmax(a.nrm[0], 0.0));
  const double s = j == 0 ? 1.0 : a.sm[8 + (j & 1)];
  for (int i = threadIdx.x; i < j; i += blockDim.x) {
    a.H[int64_t(j - 1) * a.ldh + i] += s * a.dots[2 * i];
    if (a.has_w) a.H[int64_t(j) * a.ldh + i] = a.dots[2 * i + 1];
  }
  if (threadIdx.x == 0) {
    const double c = nu > 0.0 ? a.nrm[1] / nu : 0.0;
    if (j > 0) a.H[int64_t(j - 1) * a.ldh + j] = s * nu;
    if (a.has_w) {
      a.H[int64_t(j) * a.ldh + j] = c;
      const double ww = fmax(a.nrm[2], 0.0), s2 = ww - c * c;
      a.sm[8 + ((j + 1) & 1)] = s2 > 1e-8 * ww ? std::sqrt(s2) : std::sqrt(ww);
    }
    a.sm[1] = s * nu;
    a.sm[3] = nu;
    a.sm[4] = c;
  }
}

// q_j = q~ / nu in place (zero if nu is zero), then wn = (wn - c q_j) / s_{j+1}
// (nu = sm[3], c = sm[4], s_{j+1} = *snew; zero if it is zero).
struct NextDelayedArgs {
  double* q;
  double* wn;
  int64_t N;
  const double* sm;
  const double* snew;
};

__device__ inline void next_delayed_body(const NextDelayedArgs& a, int bx, int gx) {
  const double nu = a.sm[3], c = a.sm[4], s = *a.snew;
  for (int64_t r = bx * int64_t(kBlock) + threadIdx.x; r < a.N; r += int64_t(gx) * kBlock) {
    const double q = nu != 0.0 ? a.q[r] / nu : 0.0;
    a.q[r] = q;
    a.wn[r] = s != 0.0 ? (a.wn[r] - c * q) / s : 0.0;
  }
}

// dst = src / *nrm (zero if the norm is zero)
struct ScaleArgs {
  double* dst;
  const double* src;
  int64_t N;
  const double* nrm;
};

__device__ inline void scale_body(const ScaleArgs& a, int bx, int gx) {
  const double s = *a.nrm;
  const double f = s != 0.0 ? 1.0 / s : 0.0;
  for (int64_t r = bx * int64_t(kBlock) + threadIdx.x; r < a.N; r += int64_t(gx) * kBlock) a.dst[r] = a.src[r] * f;
}

// Givens update of Hessenberg column j (rotations 0..j-1 applied, rotation j
// formed); g is the rotated right-hand side; est = |g[j+1]|.  One thread.
struct GivensArgs {
  double* H;      // column j at H + j * ldh
  int j, ldh;
  double *g, *cs, *sn, *est;
};

__device__ inline void givens_body(const GivensArgs& a) {
  if (threadIdx.x != 0) return;
  double* h = a.H + int64_t(a.j) * a.ldh;
  const int j = a.j;
  for (int i = 0; i < j; ++i) {
    const double t = a.cs[i] * h[i] + a.sn[i] * h[i + 1];
    h[i + 1] = -a.sn[i] * h[i] + a.cs[i] * h[i + 1];
    h[i] = t;
  }
  const double x = h[j], y = h[j + 1];
  const double d = std::hypot(x, y);
  const double c = d != 0.0 ? x / d : 1.0, s = d != 0.0 ? y / d : 0.0;
  a.cs[j] = c;
  a.sn[j] = s;
  h[j] = d;
  h[j + 1] = 0.0;
  a.g[j + 1] = -s * a.g[j];
  a.g[j] = c * a.g[j];
  a.est[0] = std::fabs(a.g[j + 1]);
}

// Back substitution of the rotated upper-triangular m x m system H y = g.  One thread.
struct TrisolveArgs {
  const double* H;
  int m, ldh;
  const double* g;
  double* y;
};

__device__ inline void trisolve_body(const TrisolveArgs& a) {
  if (threadIdx.x != 0) return;
  for (int i = a.m - 1; i >= 0; --i) {
    double acc = a.g[i];
    for (int l = i + 1; l < a.m; ++l) acc -= a.H[int64_t(l) * a.ldh + i] * a.y[l];
    a.y[i] = acc / a.H[int64_t(i) * a.ldh + i];
  }
}

// g = (beta, 0, ..., 0), m1 entries.
struct InitGArgs {
  double* g;
  int m1;
  const double* beta;
};

__device__ inline void init_g_body(const InitGArgs& a) {
  for (int i = threadIdx.x; i < a.m1; i += blockDim.x) a.g[i] = i == 0 ? *a.beta : 0.0;
}

// x[i] = v for i < n (also clears memory in place of a memset).
struct FillArgs {
  double* x;
  int64_t n;
  double v;
};

__device__ inline void fill_body(const FillArgs& a, int bx, int gx) {
  for (int64_t i = bx * int64_t(kBlock) + threadIdx.x; i < a.n; i += int64_t(gx) * kBlock) a.x[i] = a.v;
}

// dst[i] = src[i] for i < n (small gathers).
struct CopySmallArgs {
  const double* src;
  double* dst;
  int n;
};

__device__ inline void copy_small_body(const CopySmallArgs& a) {
  for (int i = threadIdx.x; i < a.n; i += blockDim.x) a.dst[i] = a.src[i];
}

// The input/output slots of a recorded preconditioner program: *rslot = r, *zslot = z.
struct SetPtrsArgs {
  const double** rslot;
  double** zslot;
  const double* r;
  double* z;
};

__device__ inline void set_ptrs_body(const SetPtrsArgs& a) {
  if (threadIdx.x == 0) {
    *a.rslot = a.r;
    *a.zslot = a.z;
  }
}

// ------------------------------------------------------------ wrappers ---
__global__ __launch_bounds__(kBlock) void k_slab_sums_d(SlabSumsDArgs a) { slab_sums_d_body(a, blockIdx.x); }
template <class T>
__global__ __launch_bounds__(kBlock) void k_slab_sums_t(SlabSumsTArgs<T> a) { slab_sums_t_body<T>(a, blockIdx.x); }
template <class T>
__global__ __launch_bounds__(kBlock) void k_split(SplitArgs<T> a) { split_body<T>(a, blockIdx.x, gridDim.x); }
template <class T>
__global__ __launch_bounds__(kBlock) void k_join(JoinArgs<T> a) { join_body<T>(a, blockIdx.x, gridDim.x); }
template <class T>
__global__ __launch_bounds__(kBlock) void k_slab_shift(SlabShiftArgs<T> a) {
  slab_shift_body<T>(a, blockIdx.x, gridDim.x);
}
__global__ __launch_bounds__(kBlock) void k_project_p(ProjectPArgs a) { project_p_body(a, blockIdx.x, gridDim.x); }
__global__ __launch_bounds__(kBlock) void k_mdot_partial(MdotArgs a) {
  mdot_body(a, blockIdx.x, blockIdx.y, gridDim.x);
}
__global__ __launch_bounds__(kBlock) void k_reduce(ReduceArgs a) { reduce_body(a, blockIdx.x); }
__global__ __launch_bounds__(kBlock) void k_combine(CombineArgs a) { combine_body(a, blockIdx.x, gridDim.x); }
__global__ __launch_bounds__(kBlock) void k_mdot2(Mdot2Args a) { mdot2_body(a, blockIdx.x, blockIdx.y, gridDim.x); }
__global__ __launch_bounds__(kBlock) void k_upd_delayed(UpdDelayedArgs a) {
  upd_delayed_body(a, blockIdx.x, gridDim.x);
}
__global__ __launch_bounds__(kBlock) void k_fin_delayed(FinDelayedArgs a) { fin_delayed_body(a); }
__global__ __launch_bounds__(kBlock) void k_next_delayed(NextDelayedArgs a) {
  next_delayed_body(a, blockIdx.x, gridDim.x);
}
__global__ __launch_bounds__(kBlock) void k_scale(ScaleArgs a) { scale_body(a, blockIdx.x, gridDim.x); }
__global__ __launch_bounds__(kBlock) void k_givens(GivensArgs a) { givens_body(a); }
__global__ __launch_bounds__(kBlock) void k_trisolve(TrisolveArgs a) { trisolve_body(a); }
__global__ __launch_bounds__(kBlock) void k_init_g(InitGArgs a) { init_g_body(a); }
__global__ __launch_bounds__(kBlock) void k_fill(FillArgs a) { fill_body(a, blockIdx.x, gridDim.x); }
__global__ __launch_bounds__(kBlock) void k_copy_small(CopySmallArgs a) { copy_small_body(a); }
__global__ __launch_bounds__(kBlock) void k_set_ptrs(SetPtrsArgs a) { set_ptrs_body(a); }

}  // namespace st
