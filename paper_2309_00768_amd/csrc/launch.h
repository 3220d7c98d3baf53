// Launch sink of libst.  Every kernel launch of the preconditioner and of
// FGMRES goes through emit(): it either launches the kernel on a stream
// (immediate mode) or appends the launch -- kernel, body kind, grid and
// argument block -- to a program (record mode).  Recorded programs are
// replayed with several ops per launch: two ops of one system through a
// kernel holding exactly their two bodies (k_two), or the ops of many systems
// grouped by kind (k_group, k_group2), whose workgroups find their op from a
// descriptor table passed as kernel arguments.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <vector>

#include "kernels.h"
#include "kernels_vec.h"
#include "st_internal.h"

namespace st {

// Kernel bodies a batched launch can run.  Ids of precision-dependent bodies
// refer to the preconditioner precision T of the k_group<K, T> instance.
enum Kind : int {
  kKSpmvJ = 0,      // SpmvArgs<double, double>, FP64 (J apply)
  kKSpmvT,          // SpmvArgs<T, T> (every P_T product, all roles)
  kKCheb,           // ChebArgs<T>
  kKStInit,         // StInitArgs<T>
  kKStCheb,         // StChebArgs<T>
  kKCoarse,         // CoarseArgs<T>
  kKSlabSumsD,      // SlabSumsDArgs
  kKSlabSumsT,      // SlabSumsTArgs<T>
  kKSplit,          // SplitArgs<T>
  kKJoin,           // JoinArgs<T>
  kKSlabShiftD,     // SlabShiftArgs<double>
  kKSlabShiftT,     // SlabShiftArgs<T>
  kKProjectP,       // ProjectPArgs
  kKMdot,           // MdotArgs
  kKReduce,         // ReduceArgs
  kKCombine,        // CombineArgs
  kKScale,          // ScaleArgs
  kKGivens,         // GivensArgs
  kKTrisolve,       // TrisolveArgs
  kKInitG,          // InitGArgs
  kKFill,           // FillArgs
  kKCopySmall,      // CopySmallArgs
  kKSetPtrs,        // SetPtrsArgs
  kKSpmvSlabs4,     // SpmvSlabsArgs (J apply, 4 slabs per wavefront)
  kKSpmvSlabs8,     // SpmvSlabsArgs (J apply, 8 slabs per wavefront)
  kKStSolve,        // StSolveArgs<T>
  kKMdot2,          // Mdot2Args (Arnoldi with delayed reorthogonalisation)
  kKUpdDelayed,     // UpdDelayedArgs
  kKFinDelayed,     // FinDelayedArgs
  kKNextDelayed,    // NextDelayedArgs
  kKNumKinds
};

constexpr int kMaxMembers = 64;   // two programs per system, 32 systems
constexpr int kMaxMembersG = 64;  // members of one grouped launch

// One recorded launch: its kernel (for a replay through the same kernel),
// the body kind (for a batched launch), grid and argument block.
struct Op {
  const void* fn = nullptr;
  int kind = 0;
  int gx = 1, gy = 1;
  int size = 0;
  alignas(16) unsigned char args[kOpArgBytes];
};

// A recorded preconditioner apply is two programs: `a` (the C_A sweep, and
// the current solves when they balance the two better) and `b` (the rest,
// then whatever follows the apply).  Op i of b may run only once dep[i] ops
// of a have completed in earlier launches.
struct Program {
  std::vector<Op> a, b;
  std::vector<int> dep;
};

struct Ctx {
  hipStream_t s = nullptr;
  std::vector<Op>* rec = nullptr;   // record mode when set
  std::vector<int>* dep = nullptr;  // b-side: dependency of each recorded op
  int need = 0;                     // a-ops the next recorded ops depend on
  bool recording() const { return rec != nullptr; }
};

// Workgroup size of a kind's kernels: the tiled sweep solve runs wider
// workgroups (one grown tile each), everything else kBlock.
inline int block_of(int kind) { return kind == kKStSolve ? kSolveBlock : kBlock; }

template <class A>
inline void emit(Ctx& c, int kind, dim3 grid, void (*kern)(A), const A& a) {
  static_assert(sizeof(A) <= kOpArgBytes, "kernel arguments exceed an op record");
  if (c.rec) {
    Op op;
    op.fn = reinterpret_cast<const void*>(kern);
    op.kind = kind;
    op.gx = int(grid.x);
    op.gy = int(grid.y);
    op.size = int(sizeof(A));
    std::memset(op.args, 0, sizeof(op.args));
    std::memcpy(op.args, &a, sizeof(A));
    c.rec->push_back(op);
    if (c.dep) c.dep->push_back(c.need);
    return;
  }
  void* params[] = {const_cast<A*>(&a)};
  (void)hipLaunchKernel(reinterpret_cast<const void*>(kern), grid, dim3(block_of(kind)), params, 0, c.s);
}

// ------------------------------------------------------- paired launches ---
// One op of each of the two preconditioner programs in one launch: workgroups
// [0, xblocks) run x, the rest run y.  One kernel per pair of bodies, each
// holding only its two bodies (a kernel with all of them in a switch runs
// every launch at the occupancy and register budget of the largest).
template <class T>
struct BodyStInit {
  using Args = StInitArgs<T>;
  static constexpr int kind = kKStInit;
  __device__ static void run(const Args& a, int b, int) { st_init_body<T>(a, b); }
};

template <class T>
struct BodyStCheb {
  using Args = StChebArgs<T>;
  static constexpr int kind = kKStCheb;
  __device__ static void run(const Args& a, int b, int) { st_cheb_body<T>(a, b); }
};

template <class T>
struct BodyStSolve {
  using Args = StSolveArgs<T>;
  static constexpr int kind = kKStSolve;
  __device__ static void run(const Args& a, int b, int) { st_solve_body<T>(a, b); }
};

template <class T>
struct BodyCheb {
  using Args = ChebArgs<T>;
  static constexpr int kind = kKCheb;
  __device__ static void run(const Args& a, int b, int gx) { cheb_body<T>(a, b % gx, b / gx); }
};

template <class T>
struct BodySpmv {
  using Args = SpmvArgs<T, T>;
  static constexpr int kind = kKSpmvT;
  __device__ static void run(const Args& a, int b, int gx) { spmv_body<T, T, T>(a, b % gx, b / gx); }
};

template <class X, class Y>
struct TwoArgs {
  typename X::Args x;
  typename Y::Args y;
  int xblocks, xgx, ygx;
};

template <class X, class Y>
__global__ ST_LATENCY_KERNEL void k_two(TwoArgs<X, Y> p) {
  const int b = blockIdx.x;
  if (b < p.xblocks) X::run(p.x, b, p.xgx);
  else Y::run(p.y, b - p.xblocks, p.ygx);
}

// Two tiled sweep solves (one of each program) in one launch of kSolveBlock
// workgroups.
template <class T>
__global__ ST_SOLVE_KERNEL void k_two_solve(TwoArgs<BodyStSolve<T>, BodyStSolve<T>> p) {
  const int b = blockIdx.x;
  if (b < p.xblocks) st_solve_body<T>(p.x, b);
  else st_solve_body<T>(p.y, b - p.xblocks);
}

// -------------------------------------------------------- grouped launches ---
// Body of kind K in precision T with its argument type; b is the workgroup
// index within the op's own grid of gx columns.  A grouped launch runs ops of
// one kind (k_group) or of two pairable kinds (k_group2) for several systems,
// their argument blocks read from device memory.
template <int K, class T> struct KB;
template <class T> struct KB<kKSpmvJ, T> {
  using Args = SpmvArgs<double, double>;
  __device__ static void run(const Args& a, int b, int gx) { spmv_body<double, double, double>(a, b % gx, b / gx); }
};
template <class T> struct KB<kKSpmvT, T> {
  using Args = SpmvArgs<T, T>;
  __device__ static void run(const Args& a, int b, int gx) { spmv_body<T, T, T>(a, b % gx, b / gx); }
};
template <class T> struct KB<kKCheb, T> {
  using Args = ChebArgs<T>;
  __device__ static void run(const Args& a, int b, int gx) { cheb_body<T>(a, b % gx, b / gx); }
};
template <class T> struct KB<kKStInit, T> {
  using Args = StInitArgs<T>;
  __device__ static void run(const Args& a, int b, int) { st_init_body<T>(a, b); }
};
template <class T> struct KB<kKStCheb, T> {
  using Args = StChebArgs<T>;
  __device__ static void run(const Args& a, int b, int) { st_cheb_body<T>(a, b); }
};
template <class T> struct KB<kKStSolve, T> {   // launched through k_group_solve
  using Args = StSolveArgs<T>;
  __device__ static void run(const Args&, int, int) {}
};
template <class T> struct KB<kKCoarse, T> {
  using Args = CoarseArgs<T>;
  __device__ static void run(const Args& a, int b, int) { coarse_body<T>(a, b); }
};
template <class T> struct KB<kKSlabSumsD, T> {
  using Args = SlabSumsDArgs;
  __device__ static void run(const Args& a, int b, int) { slab_sums_d_body(a, b); }
};
template <class T> struct KB<kKSlabSumsT, T> {
  using Args = SlabSumsTArgs<T>;
  __device__ static void run(const Args& a, int b, int) { slab_sums_t_body<T>(a, b); }
};
template <class T> struct KB<kKSplit, T> {
  using Args = SplitArgs<T>;
  __device__ static void run(const Args& a, int b, int gx) { split_body<T>(a, b, gx); }
};
template <class T> struct KB<kKJoin, T> {
  using Args = JoinArgs<T>;
  __device__ static void run(const Args& a, int b, int gx) { join_body<T>(a, b, gx); }
};
template <class T> struct KB<kKSlabShiftD, T> {
  using Args = SlabShiftArgs<double>;
  __device__ static void run(const Args& a, int b, int gx) { slab_shift_body<double>(a, b, gx); }
};
template <class T> struct KB<kKSlabShiftT, T> {
  using Args = SlabShiftArgs<T>;
  __device__ static void run(const Args& a, int b, int gx) { slab_shift_body<T>(a, b, gx); }
};
template <class T> struct KB<kKProjectP, T> {
  using Args = ProjectPArgs;
  __device__ static void run(const Args& a, int b, int gx) { project_p_body(a, b, gx); }
};
template <class T> struct KB<kKMdot, T> {
  using Args = MdotArgs;
  __device__ static void run(const Args& a, int b, int gx) { mdot_body(a, b % gx, b / gx, gx); }
};
template <class T> struct KB<kKReduce, T> {
  using Args = ReduceArgs;
  __device__ static void run(const Args& a, int b, int) { reduce_body(a, b); }
};
template <class T> struct KB<kKCombine, T> {
  using Args = CombineArgs;
  __device__ static void run(const Args& a, int b, int gx) { combine_body(a, b, gx); }
};
template <class T> struct KB<kKScale, T> {
  using Args = ScaleArgs;
  __device__ static void run(const Args& a, int b, int gx) { scale_body(a, b, gx); }
};
template <class T> struct KB<kKGivens, T> {
  using Args = GivensArgs;
  __device__ static void run(const Args& a, int, int) { givens_body(a); }
};
template <class T> struct KB<kKTrisolve, T> {
  using Args = TrisolveArgs;
  __device__ static void run(const Args& a, int, int) { trisolve_body(a); }
};
template <class T> struct KB<kKInitG, T> {
  using Args = InitGArgs;
  __device__ static void run(const Args& a, int, int) { init_g_body(a); }
};
template <class T> struct KB<kKFill, T> {
  using Args = FillArgs;
  __device__ static void run(const Args& a, int b, int gx) { fill_body(a, b, gx); }
};
template <class T> struct KB<kKCopySmall, T> {
  using Args = CopySmallArgs;
  __device__ static void run(const Args& a, int, int) { copy_small_body(a); }
};
template <class T> struct KB<kKSpmvSlabs4, T> {
  using Args = SpmvSlabsArgs;
  __device__ static void run(const Args& a, int b, int) {
    int bx, by;
    if (slabs_block(a, b, bx, by)) spmv_slabs_body<4>(a, bx, by);
  }
};
template <class T> struct KB<kKSpmvSlabs8, T> {
  using Args = SpmvSlabsArgs;
  __device__ static void run(const Args& a, int b, int) {
    int bx, by;
    if (slabs_block(a, b, bx, by)) spmv_slabs_body<8>(a, bx, by);
  }
};
template <class T> struct KB<kKMdot2, T> {
  using Args = Mdot2Args;
  __device__ static void run(const Args& a, int b, int gx) { mdot2_body(a, b % gx, b / gx, gx); }
};
template <class T> struct KB<kKUpdDelayed, T> {
  using Args = UpdDelayedArgs;
  __device__ static void run(const Args& a, int b, int gx) { upd_delayed_body(a, b, gx); }
};
template <class T> struct KB<kKFinDelayed, T> {
  using Args = FinDelayedArgs;
  __device__ static void run(const Args& a, int, int) { fin_delayed_body(a); }
};
template <class T> struct KB<kKNextDelayed, T> {
  using Args = NextDelayedArgs;
  __device__ static void run(const Args& a, int b, int gx) { next_delayed_body(a, b, gx); }
};
template <class T> struct KB<kKSetPtrs, T> {
  using Args = SetPtrsArgs;
  __device__ static void run(const Args& a, int, int) { set_ptrs_body(a); }
};

// An op's argument block, read from device memory word by word into scalar
// registers at the start of the workgroup: the address is the same for the
// whole workgroup, and v_readfirstlane tells the compiler that every field is
// uniform.  (Copied as a struct, parts of the block land in vector registers
// as values that may differ between lanes, and every buffer load built from
// them becomes a loop over the lanes' distinct resources.)  The blocks are
// written before the launch and only read by it.
template <class A>
__device__ inline A load_args(const unsigned char* p) {
  static_assert(sizeof(A) % 4 == 0, "argument blocks are whole words");
  constexpr int W = int(sizeof(A) / 4);
  const __attribute__((address_space(4))) uint32_t* src = (const __attribute__((address_space(4))) uint32_t*)(p);
  uint32_t w[W];
#pragma unroll
  for (int i = 0; i < W; ++i) w[i] = __builtin_amdgcn_readfirstlane(src[i]);
  A a;
  __builtin_memcpy(&a, w, sizeof(A));
  return a;
}

// The ops of one grouped launch: op i runs on workgroups [start[i],
// start[i + 1]) with its argument block args[i] (a device copy), its own grid
// width gx[i] and (k_group2) body second[i]; start[n] is the total and the
// starts after it are INT_MAX.
struct GroupArgs {
  int n;
  int pad;
  int start[kMaxMembersG + 1];
  int gx[kMaxMembersG];
  int second[kMaxMembersG];
  const unsigned char* args[kMaxMembersG];
};

// Finds the op of workgroup blockIdx.x: returns its index and the block
// within it.  A binary search over the starts (nondecreasing, INT_MAX after
// the total) for the last one at or below the workgroup: six scalar loads
// from the kernel arguments, whatever the number of ops.
__device__ inline int group_member(const GroupArgs& g, int& rem) {
  static_assert((kMaxMembersG & (kMaxMembersG - 1)) == 0, "the search halves a power of two");
  const int b = int(blockIdx.x);
  int lo = 0;
#pragma unroll
  for (int step = kMaxMembersG / 2; step > 0; step >>= 1)
    if (b >= g.start[lo + step]) lo += step;
  rem = b - g.start[lo];
  return lo;
}

template <int K, class T>
__global__ ST_LATENCY_KERNEL void k_group(GroupArgs g) {
  int rem = 0;
  const int sel = group_member(g, rem);
  using A = typename KB<K, T>::Args;
  const A a = load_args<A>(g.args[sel]);
  KB<K, T>::run(a, rem, g.gx[sel]);
}

// Tiled sweep solves of several systems (both sweeps of each) in one launch.
template <class T>
__global__ ST_SOLVE_KERNEL void k_group_solve(GroupArgs g) {
  int rem = 0;
  const int sel = group_member(g, rem);
  const StSolveArgs<T> a = load_args<StSolveArgs<T>>(g.args[sel]);
  st_solve_body<T>(a, rem);
}

template <int K1, int K2, class T>
__global__ ST_LATENCY_KERNEL void k_group2(GroupArgs g) {
  int rem = 0;
  const int sel = group_member(g, rem);
  const unsigned char* p = g.args[sel];
  const int gx = g.gx[sel];
  if (g.second[sel]) {
    using A = typename KB<K2, T>::Args;
    const A a = load_args<A>(p);
    KB<K2, T>::run(a, rem, gx);
  } else {
    using A = typename KB<K1, T>::Args;
    const A a = load_args<A>(p);
    KB<K1, T>::run(a, rem, gx);
  }
}

// ------------------------------------------------------ batch descriptors ---
// One op of a member system in a lockstep step, and the ops of one step.
struct Member {
  const unsigned char* args;   // device copy of the op's argument block
  int kind;
  int blocks;                  // gx * gy
  int gx;
  int pad;
};

struct MultiArgs {
  int nmem;
  int pad;
  Member m[kMaxMembers];
};

}  // namespace st
