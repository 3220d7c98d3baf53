/*
 * st.h -- C ABI of libst: the all-at-once space-time solve of linearised
 * incompressible resistive MHD, preconditioned by the block upper-triangular
 * space-time preconditioner P_T of Danieli, Southworth & Schroder,
 * "Space-time block preconditioning for incompressible resistive MHD"
 * (arXiv:2309.00768).
 *
 * Problem (paper, Sec. "Problem definition and discretisation"): backward
 * Euler in time with Nt slabs, Taylor-Hood Q2-Q1 velocity/pressure and Q1
 * current/vector potential on a uniform n x n mesh of the unit square.  The
 * space-time Jacobian J (eq. (jacobianSTDiscrete)) is block lower-bidiagonal
 * in time; P_T (eq. (PT)) = Ubar_ujA * Utilde_up uses the pressure
 * convection-diffusion Schur approximation (eq. (Fp)) and the wave-based
 * magnetic Schur approximation C_A (eqs. (CAspacetime), (CAs),
 * (ASchurApprox)).
 *
 * Vector layout (every vector argument): float64, device memory, slab-major,
 * length N = Nt * Ns with, per slab, [u_x | u_y | p | j | A]:
 *   u_x, u_y : (2n-1)^2 interior Q2 nodes each (homogeneous Dirichlet),
 *   p, j     : (n+1)^2 Q1 nodes (all nodes),
 *   A        : (n-1)^2 interior Q1 nodes (homogeneous Dirichlet);
 * nodes numbered lexicographically, x fastest.
 *
 * Pressure: J has one constant-pressure null vector per slab.  Every entry
 * point projects the pressure rows of its input to zero sum per slab and
 * returns pressure normalised to zero mean, 1^T M_p p^k = 0.
 *
 * Ownership and threading: all vector memory belongs to the caller.  Device
 * memory of a handle comes only from the caller's workspace `ws`.  A handle
 * is not thread-safe; calls on one handle must be serialised (one stream at a
 * time).  No C++ exception crosses this interface.
 *
 * Errors: every call returns an st_status; 0 is success.  st_error_string()
 * gives a static description.
 */
#ifndef ST_H
#define ST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum st_status {
  ST_OK = 0,
  ST_ENOTCONV = 1,      /* solver hit maxit; x holds the best iterate, info is filled */
  ST_EINVAL = -1,       /* bad argument (null pointer, size, option) */
  ST_EHIP = -2,         /* a HIP runtime call failed */
  ST_ENOMEM = -3,       /* workspace smaller than st_plan_workspace_size(), or a system
                           whose preconditioner scratch exceeds the static
                           array of st_apply_precond_noalloc */
  ST_EBREAKDOWN = -4,   /* NaN or Inf in a residual or in the Hessenberg matrix */
  ST_EINTERNAL = -5     /* setup failed (e.g. singular coarse matrix) */
} st_status;

typedef enum st_precision { ST_FP64 = 0, ST_FP32 = 1 } st_precision;

/* Inner solvers of P_T (the paper uses exact LU-based ones, Sec. "Performance
 * of preconditioner"; here they are iterative):
 *   ST_INNER_AMG   : one smoothed-aggregation V(1,1) cycle (Chebyshev-Jacobi
 *                    smoothing) per spatial solve of F_u,k, C_A,k and K_p and a
 *                    fixed Chebyshev-Jacobi polynomial for the mass matrices;
 *   ST_INNER_EXACT : the same cycles repeated (inner_iters times) as a
 *                    stationary iteration, so that every inner solve is
 *                    converged to rounding level; P_T^{-1} then agrees with the
 *                    exact-inner operator of the paper.                       */
typedef enum st_inner_mode { ST_INNER_AMG = 0, ST_INNER_EXACT = 1 } st_inner_mode;

typedef struct st_problem {
  int n;              /* cells per side of the unit square (n >= 2)           */
  int nt;             /* number of slabs (Nt >= 1)                            */
  double dt;          /* time step                                            */
  double mu;          /* viscosity (1/Re)                                     */
  double eta;         /* resistivity (1/S)                                    */
  double mu0;         /* magnetic permeability                                */
  const double* ubar; /* host, [nt][2][(2n+1)^2]: Q2 nodal velocity state     */
  const double* abar; /* host, [nt][(n+1)^2]: Q1 nodal vector-potential state */
  const double* jbar; /* host, [nt][(n+1)^2] current state, or NULL: then the
                         library solves M_j jbar = -(1/mu0) K abar per slab    */
  int precond_precision; /* st_precision of everything inside P_T           */
  int inner_mode;     /* st_inner_mode                                        */
  int inner_iters;    /* V-cycles per spatial solve in EXACT mode (0: 40)      */
  int mass_iters;     /* Chebyshev steps per mass-matrix solve (0: 6 AMG mode,
                         60 EXACT mode)                                        */
  int cheb_degree;    /* Chebyshev-Jacobi smoother degree (0: 3)              */
  int fu_solver;      /* inner solver of F_u,k: 0 auto (AMG mode: from the
                         estimated condition number of D^{-1} F_u; EXACT mode:
                         repeated V-cycles), -1 one SA-AMG V(1,1) cycle (AMG
                         mode), k > 0 Chebyshev-Jacobi of degree k alone in
                         either mode (EXACT mode then converges the K_p and
                         mass solves only)                                  */
  int ca_solver;      /* the same for the wave blocks C_A,k                   */
  int max_restart;    /* largest FGMRES restart length the workspace holds (0: 30) */
  int sell_sigma;     /* SELL sorting window in rows (0: whole matrix)        */
  int adjoint;        /* 1: also build the transposed operators (J^T, P_T^{-T}) */
  int j_lanes;        /* wavefront lanes per row of the J apply (0: auto)     */
  int sweep_format;   /* Chebyshev-alone sweeps: 0 structured 5x5 stencils,
                         each step solving for its increment over a predictor
                         from the earlier slabs (the approximate solve's error
                         is then not amplified by the recursion in time);
                         1 SELL, each step solved from zero (for comparison:
                         the two agree when the spatial solves converge)    */
  int single_stream;  /* 0: P_T^{-1} is recorded at st_create as two programs
                         (the C_A sweep; the pressure part and the F_u sweep,
                         each chunk of it waiting for that chunk of the C_A
                         sweep) and replayed with one launch carrying a step
                         of each; 1: launched step by step in program order
                         (same arithmetic)                                    */
  int sweep_chunk;    /* slabs per chunk of that pipeline (0: max(4, Nt/8))  */
  int sweep_chain;    /* 0: on grids of at most 1024 unknowns the C_A sweep and
                         the M_j solves of a chunk run in one workgroup (no
                         launch per step); -1: never (per-step launches)      */
  int j_slabs;        /* slabs per wavefront of the J apply: 0 auto (8), 1 one
                         slab per workgroup row, 4 or 8 (slab-invariant column
                         indices and values loaded once for them)           */
  int sweep_fuse;     /* stencil sweep solves: 0 one launch per Chebyshev step;
                         1 several steps per launch on 8 x 8 node tiles grown
                         by halos held in LDS (up to 4 steps in the first
                         launch of a solve, 3 in each later one; bitwise the
                         same result, slower on the measured workloads)     */
  int autotune;       /* 1: st_create times, on this system's operators, the
                         launch choices that leave every result bitwise the
                         same (slabs per wavefront of the J apply when j_slabs
                         is 0; rows per workgroup of the sweep step kernels;
                         one launch per sweep step or the tiled solve) and
                         keeps the fastest (st_tuning reports them); 0: the
                         given or default choices                          */
  int sweep_lanes;    /* stencil sweep steps on the two-component F_u,k: 0
                         default (1), 1 one lane per row, 2 the row's two
                         column components on two lanes (half the loads per
                         lane; the same result bit for bit); the autotuner
                         times both                                         */
  double inner_reduction; /* auto inner solver of F_u,k: target error reduction
                             per spatial solve (0: 0.3; degree at least 4)    */
  double ca_reduction;    /* auto inner solver of C_A,k: target reduction (0: 0.3;
                             degree at least 4)                                */
  int precond_variant;    /* the preconditioner FGMRES and st_apply_precond use:
                             0 P_T, eq. (PT) (recorded replay); 1 P-tilde, eq.
                             (preconditionerSimplified1), one more F_u sweep (the
                             L_up factor); 2 the full P, eq. (preconditioner),
                             two more F_u sweeps and an M_j solve (the L_ujA and
                             L_up factors).  1 and 2 run step by step, forward
                             only: st_apply_precond_t, the adjoint solve, the
                             allocation-free apply and batches take 0 only
                             (ST_EINVAL otherwise).                         */
  int time_parallel;      /* the two sweeps of P_T^{-1} (F_u,k and C_A,k over
                             the slabs, eqs. (STFu), (CAspacetime)): 0 forward
                             substitution in time; K >= 1 K iterations of
                             Parareal, the parallel-in-time inner solves the
                             paper leaves to future work (Conclusions; footnote
                             of Sec. "Comparison with single time-step block
                             preconditioner").  Fine propagator: the slab step
                             with the plan's Chebyshev degree; coarse: the same
                             step with time_coarse_degree Chebyshev steps.  The
                             fine steps of all slabs run together (one launch
                             per Chebyshev step), the coarse sweep slab by slab;
                             after K iterations the first K slabs equal the
                             forward substitution, after Nt all of them.  Needs
                             the stencil sweeps with Chebyshev alone on both
                             blocks (sweep_format 0 and a positive degree chosen
                             for each, else st_plan_create fails); P_T forward
                             only, step by step: not with adjoint, batches or
                             the allocation-free apply (ST_EINVAL).         */
  int time_coarse_degree; /* Chebyshev steps of the coarse propagator per slab
                             (0: 1); below both sweep degrees                 */
} st_problem;

typedef struct st_opts {
  int restart;        /* m, <= max_restart (0: 30)                            */
  int maxit;          /* total iteration cap (0: 1000)                        */
  double rtol;        /* stop when ||b - J x||_2 <= max(rtol ||b||_2, atol)   */
  double atol;
  int x0_given;       /* 1: x holds the initial guess; 0: start from zero     */
  int history_len;    /* capacity of `history` (may be 0)                     */
  double* history;    /* host; estimated relative residual per iteration      */
  int orth;           /* Gram-Schmidt of the Arnoldi steps (st_fgmres_solve,
                         st_adjoint_solve, the time-stepping and Newton solves;
                         a batch takes 1 and rejects 2):
                         0: automatic, 2 when restart > 64 or N >= 2^20
                            (bandwidth-bound basis reads), else 1;
                         1: classical Gram-Schmidt with a second pass (CGS2),
                            four reads of the basis per step;
                         2: CGS2 with the second pass of each direction delayed
                            to the next step and fused with that step's first
                            pass: two reads of the basis per step.  Each column
                            of the Hessenberg matrix completes one step later,
                            so a solve that stops inside a cycle has applied
                            P_T^{-1} and J once more than it counts
                            iterations.  Other values: ST_EINVAL.           */
} st_opts;

typedef struct st_info {
  int iterations;     /* FGMRES iterations (preconditioner applications)      */
  int restarts;
  int converged;      /* 1 if the true residual met the tolerance             */
  double true_rel_residual;  /* ||b - J x|| / ||b|| at exit (computed in FP64) */
  double seconds;     /* wall time of the solve (host clock, after sync)      */
  double precond_seconds;    /* time inside P_T^{-1} (event-timed)            */
  double jacobian_seconds;   /* time inside the J applies (event-timed)       */
  int jacobian_calls;        /* number of J applies in the solve              */
  int precond_calls;         /* number of P_T^{-1} applies in the solve       */
} st_info;

typedef struct st_plan st_plan;       /* host-side setup result             */
typedef struct st_handle st_handle;   /* device-resident system             */
typedef struct st_batch st_batch;     /* lockstep solver over several systems */

/* ---------------------------------------------------------------- setup --- */

/* Host-only setup: assembles every block of J and P_T from the state, forms the
 * wave operator blocks (eq. (CAs)), builds the AMG hierarchies and packs all
 * device data into one image.  Makes no HIP call.  `p` and its arrays are only
 * read during the call. */
int st_plan_create(const st_problem* p, st_plan** out);

/* Bytes of device workspace st_create() needs for this plan (256-aligned). */
int st_plan_workspace_size(const st_plan* plan, size_t* bytes);

/* Sizes of one slab: Ns and the block offsets [u_x, u_y, p, j, A, end]. */
int st_plan_sizes(const st_plan* plan, int* ns, int offsets[6]);

/* Debug/test export of one host-assembled block (CSR, float64) for slab k.
 * block ids: 0 Fu, 1 Mu, 2 B, 3 Zj, 4 ZA, 5 Mj, 6 KjA, 7 Y, 8 FA, 9 MA, 10 KA,
 * 11 Kp, 12 Fp, 13 C0 (diagonal band of C_A), 14 C1 (band -1, k < nt-1),
 * 15 C2 (band -2).  Call with rowptr == NULL to get nrows, ncols, nnz first. */
int st_plan_export_block(const st_plan* plan, int block, int k, int* nrows, int* ncols,
                         int64_t* nnz, int* rowptr, int* colind, double* val);

/* Inner solvers chosen by the setup: Chebyshev degree used alone on F_u,k and
 * C_A,k (0 = SA-AMG V-cycle) and the estimated condition numbers of D^{-1} A
 * (for a slab on an ellipse, or whose interval contracts slower than its
 * condition number says, the condition number of an interval with the same
 * convergence factor). */
int st_plan_solver_info(const st_plan* plan, int* fu_degree, int* ca_degree, double* fu_kappa,
                        double* ca_kappa);

/* Chebyshev-alone intervals of the sweep blocks, host: which = 0 for F_u,k,
 * 1 for C_A,k; out[2 k] = theta and out[2 k + 1] = delta of slab k (nt pairs).
 * delta > 0: the Chebyshev-Jacobi steps of that slab's spatial solve assume
 * the eigenvalues of D^{-1} A in an ellipse with foci theta -+ delta (the
 * interval [theta - delta, theta + delta] when flat); delta <= 0: foci
 * theta -+ i|delta| (a non-normal block with eigenvalues far off the real
 * axis; Manteuffel, Numer. Math. 28, 1977). */
int st_plan_cheb_intervals(const st_plan* plan, int which, double* out);

/* The current state used (either given or computed), host [nt][(n+1)^2]. */
int st_plan_export_jbar(const st_plan* plan, double* jbar);

/* Stored layout of the J apply (SELL, eq. (jacobianSTDiscrete)): entries per
 * segment including the padding of each 64-row slice, slots[0] for the
 * per-slab blocks (one value set per slab), slots[1] for the slab-invariant
 * blocks and slots[2] for the previous-slab coupling, and the number of
 * slices.  Host only; any pointer may be NULL. */
int st_plan_jacobian_slots(const st_plan* plan, int64_t slots[3], int* nslices);

int st_plan_destroy(st_plan* plan);

/* Uploads the plan into the caller's device workspace `ws` (>= workspace size
 * bytes, 256-byte aligned) on `stream` and returns a handle.  The plan may be
 * destroyed afterwards.  `stream` is a hipStream_t (NULL = default stream). */
int st_create(const st_plan* plan, void* ws, size_t ws_bytes, void* stream, st_handle** out);

/* Releases host-side state only; `ws` stays owned by the caller. */
int st_destroy(st_handle* h);

/* ---------------------------------------------------------- operators --- */

/* y = J x (eq. (jacobianSTDiscrete)); x, y device, length N, must not alias.
 * Asynchronous on `stream`. */
int st_apply_jacobian(st_handle* h, const double* x, double* y, void* stream);

/* y = J^T x: the transpose of eq. (jacobianSTDiscrete), block upper-bidiagonal
 * in time (diagonal blocks the transposed single-step Jacobians of eq.
 * (jacobianDiscrete), super-diagonal -diag(M_u/dt, 0, 0, M_A/dt), the mass
 * matrices being symmetric).  Needs a handle created with adjoint = 1 (else
 * ST_EINVAL).  Same layout, aliasing and stream rules as st_apply_jacobian. */
int st_apply_jacobian_t(st_handle* h, const double* x, double* y, void* stream);

/* z = P_T^{-1} r (eq. (PT)); internal precision per the problem; FP64 in/out.
 * r and z device, length N, must not alias.  Asynchronous on `stream`. */
int st_apply_precond(st_handle* h, const double* r, double* z, void* stream);

/* z = P_T^{-T} r: the transpose of eq. (PT), P_T^T = Utilde_up^T Ubar_ujA^T
 * with eqs. (Utilde) and (barUuja) transposed; its F_u and C_A solves become
 * backward-in-time sweeps on the transposed blocks of eqs. (STFu) and (CAs).
 * Needs adjoint = 1 (else ST_EINVAL).  FP64 in/out, device, length N, no
 * aliasing; asynchronous on `stream`. */
int st_apply_precond_t(st_handle* h, const double* r, double* z, void* stream);

/* z = P_T^{-1} r exactly as st_apply_precond computes it (the same kernels,
 * launched step by step), for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  It calls no hipMalloc, hipFree or allocating library routine:
 * the preconditioner's scratch (per-block vectors, Chebyshev and V-cycle
 * buffers, pressure sums) lives in one static device array of 128 MiB per
 * GPU, held from the library's load onto that GPU until the process ends; the
 * operators stay in the handle's workspace, r and z are the caller's (FP64,
 * device, length N, no aliasing).  The scratch a system needs is
 * workspace_size - (operators + Krylov vectors); a system needing more than
 * 128 MiB is rejected with ST_ENOMEM and a message on stderr, before any
 * launch.  The calling thread's current device must be the one the handle was
 * created on (else ST_EINVAL).  Every call on a GPU shares that GPU's array,
 * which keeps the last call's contents; nothing in it has to start at zero
 * (each buffer is written before it is read within a call).  Calls that
 * overlap on one GPU (other streams, other threads, other handles) race on
 * the array and must be serialised by the caller.  Asynchronous on `stream`. */
int st_apply_precond_noalloc(st_handle* h, const double* r, double* z, void* stream);

/* y = (M_A / dt) a0: how an initial vector potential A^0 (interior Q1 nodes,
 * length (n-1)^2, device, FP64) enters the right-hand side of the first slab
 * (the A^{k-1} term of the induction row of the paper's recurrence, eq.
 * (recurrence), moved to the right for k = 1).  M_A is symmetric, so the same
 * call maps an adjoint lambda_A^1 to the gradient with respect to A^0. */
int st_apply_initial_coupling(st_handle* h, const double* a0, double* y, void* stream);

/* ------------------------------------------------------------- solves --- */

/* Right-preconditioned FGMRES(m) on J x = b with P_T, the Krylov method the
 * paper wraps around eq. (PT) (Sec. "Performance of preconditioner", GMRES
 * right-preconditioned; flexible here because the inner solves are
 * iterative); residual, Arnoldi (CGS2, or CGS2 with delayed
 * reorthogonalisation: st_opts.orth) and the Hessenberg least-squares
 * problem in FP64 on the device.  b, x device, length N, slab-major; the
 * pressure rows of b are projected to zero sum per slab and x is normalised
 * to 1^T M_p p^k = 0.  Stops when ||b - J x||_2 <= max(rtol ||b||_2, atol) (true
 * residual).  o->restart <= the plan's max_restart (else ST_EINVAL).  Blocks
 * until done.  Returns ST_OK, ST_ENOTCONV (x = last iterate, info filled),
 * ST_EBREAKDOWN (a NaN or Inf in b or in the iteration) or another error. */
int st_fgmres_solve(st_handle* h, const double* b, double* x, const st_opts* o,
                    st_info* info, void* stream);

/* Adjoint solve J^T lam = g (the transpose of eq. (jacobianSTDiscrete), a
 * backward-in-time recurrence) with FGMRES right-preconditioned by P_T^{-T}
 * (st_apply_precond_t); the gradient of a terminal functional of A^{Nt} with
 * respect to A^0 is then st_apply_initial_coupling(lambda_A^1).  Needs
 * adjoint = 1.  Options, stopping test, outputs and status codes as for
 * st_fgmres_solve. */
int st_adjoint_solve(st_handle* h, const double* g, double* lam, const st_opts* o,
                     st_info* info, void* stream);

/* Sequential time stepping, the baseline the all-at-once solve is compared
 * with (Sec. "Comparison with sequential time-stepping"): slab k is solved
 * after slab k-1 from J_k x^k = b^k + diag(M_u/dt, 0, 0, M_A/dt) x^{k-1}, J_k the
 * single-step Jacobian of eq. (jacobianDiscrete), by FGMRES(m)
 * right-preconditioned with the single-step P_{T,k} of eq. (PTTS) (with eq.
 * (ASchurApproxTS)).  hs[k] is a handle created from a one-slab plan (Nt = 1)
 * of slab k's state, whose P_T is P_{T,k}; all handles share n.  A handle of
 * W_k > 1 slabs (a plan of those slabs' states) makes step k a window solved
 * all at once with its own P_T (windowed space-time), coupled to the previous
 * window's last slab in the same way; nt is then the number of windows and
 * Nt = sum W_k.  b, x: device, length Nt * Ns, slab-major, the same layout as
 * the all-at-once system.  Step k stops on
 * ||r_k||_2 <= max(rtol ||b||_2, atol) sqrt(W_k / Nt) (the paper's scaling of
 * the step tolerance; the step residuals are the rows of the space-time
 * residual, so x meets ||b - J x|| <= max(rtol ||b||, atol)).  With
 * o->x0_given = 1 every slab of step k >= 2 starts from the previous step's
 * last slab (the paper's warm start), else from zero.  infos[k] receives step
 * k's result.  Blocks until done.  Returns ST_OK if every step converged,
 * ST_ENOTCONV if some did not (later steps still run from that iterate), else
 * an error. */
int st_timestep_solve(st_handle* const* hs, int nt, const double* b, double* x, const st_opts* o,
                      st_info* infos, void* stream);

/* --------------------------------------------------- space-time Newton --- */
/* The nonlinear recurrence, eq. (recurrence), solved for all slabs at once by
 * Newton's method, each correction from the space-time Jacobian of eq.
 * (jacobianSTDiscrete) linearised about the current iterate and solved by
 * FGMRES with P_T (Sec. "Performance of preconditioner").
 *
 * Fields are full nodal arrays on the unit square's n x n mesh: Q2 velocity on
 * the (2n+1)^2 grid ([2][(2n+1)^2] per slab), Q1 p, j, A on the (n+1)^2 grid,
 * lexicographic with x fastest.  The unknown x (device, length nt * Ns, the
 * linear solver's slab-major layout [u_x | u_y | p | j | A]: interior u and A,
 * all p and j) is added to base fields, which carry the Dirichlet values of u
 * and A on the boundary and the initial guess; u_init and a_init are the
 * fields at t_0 that the first slab couples to.  f (momentum forcing) and e
 * (the imposed electric field E of the induction equation) are nodal fields per
 * slab, integrated against the test functions; either may be NULL (zero).
 * All pointers are host arrays, copied at st_nl_create. */
typedef struct st_nl st_nl;

typedef struct st_nl_problem {
  int n, nt;
  double dt, mu, eta, mu0;
  const double* u_base;  /* [nt][2][(2n+1)^2] */
  const double* p_base;  /* [nt][(n+1)^2] */
  const double* j_base;  /* [nt][(n+1)^2] */
  const double* a_base;  /* [nt][(n+1)^2] */
  const double* u_init;  /* [2][(2n+1)^2] */
  const double* a_init;  /* [(n+1)^2] */
  const double* f;       /* [nt][2][(2n+1)^2] or NULL */
  const double* e;       /* [nt][(n+1)^2] or NULL */
} st_nl_problem;

#define ST_NEWTON_MAX 32
typedef struct st_newton_opts {
  int max_newton;     /* Newton steps at most (0: 20; at most ST_NEWTON_MAX) */
  double atol;        /* stop when ||R(x)||_2 <= atol (the paper: 1e-10)     */
  st_opts linear;     /* FGMRES of each correction (the paper: rtol 1e-2,
                         atol 1e-14); x0_given and the history are ignored   */
} st_newton_opts;

typedef struct st_newton_info {
  int newton_iterations;                        /* corrections applied         */
  int converged;
  int linear_iterations_total;
  int linear_iterations[ST_NEWTON_MAX];         /* FGMRES iterations per step   */
  double residual_norm[ST_NEWTON_MAX + 1];      /* ||R|| before each step, and at the end */
  double seconds;                               /* wall time of the whole solve */
  double setup_seconds;                         /* of which re-assembly and upload */
} st_newton_info;

/* Device bytes st_nl_create needs (base, initial and forcing fields, element
 * residuals, three N-vectors, the linearisation state). */
int st_nl_workspace_size(const st_nl_problem* p, size_t* bytes);
/* Copies the fields into the caller's workspace `ws` (256-byte aligned) on
 * `stream` and waits for it. */
int st_nl_create(const st_nl_problem* p, void* ws, size_t ws_bytes, void* stream, st_nl** out);
/* r = R(base + x): the left-hand side of eq. (recurrence) minus its right-hand
 * side (f in the momentum rows; E, carried with a minus sign on the right of
 * the induction equation, enters the residual with a plus), by 4 x 4 Gauss
 * quadrature per element; rows in the slab-major layout of x.  x, r device,
 * no aliasing; asynchronous on `stream`. */
int st_nl_residual(st_nl* nl, const double* x, double* r, void* stream);
/* Newton from the given x (device, updated in place): each step evaluates R,
 * stops if ||R|| <= o->atol, else assembles the linearisation about base + x
 * on the host (the template `lin` supplies every option of st_problem but the
 * state and sizes; precond_variant 0, adjoint 0), uploads it into `lin_ws`
 * (the caller's, >= st_plan_workspace_size of the same problem) and applies
 * x += d with J d = -R from FGMRES.  Blocks until done.  ST_OK when converged,
 * ST_ENOTCONV after max_newton steps, else an error. */
int st_newton_solve(st_nl* nl, const st_problem* lin, void* lin_ws, size_t lin_ws_bytes, double* x,
                    const st_newton_opts* o, st_newton_info* info, void* stream);
int st_nl_destroy(st_nl* nl);

/* ------------------------------------------------------------ batches --- */
/* Many independent space-time systems (uneven n and Nt) solved together: the
 * same right-preconditioned FGMRES(m) as st_fgmres_solve on each member, run
 * in lockstep so that one launch carries the same step of every member (a
 * sweep step, a Gram-Schmidt pass, ...).  Each member's arithmetic, and so its
 * iterates and result, is the one st_fgmres_solve produces on that handle
 * with single_stream = 1 and sweep_chain = -1.
 *
 * st_batch_create: host-only; records the launch programs of the members.
 *   hs: 1..32 distinct handles with the same precond_precision, each with
 *   max_restart >= restart (0: 30).  The handles must outlive the batch and
 *   must not be used by other calls while a batched solve runs.
 * st_batch_workspace_size: device bytes the batch needs besides the handles'
 *   workspaces (argument blocks of the recorded launches).
 * st_batch_upload: copies the recorded launches into `ws` (caller-owned,
 *   256-byte aligned, >= the workspace size) on `stream` and waits for it.
 * st_batch_launch_counts: launches of one Arnoldi step (preconditioner, J and
 *   Gram-Schmidt) in lockstep and summed over members solved one at a time.  */
int st_batch_create(st_handle* const* hs, int nsys, int restart, st_batch** out);
int st_batch_workspace_size(const st_batch* b, size_t* bytes);
int st_batch_upload(st_batch* b, void* ws, size_t ws_bytes, void* stream);
int st_batch_launch_counts(const st_batch* b, int64_t* lockstep, int64_t* separate);

/* Solves J_i x_i = b_i for every member i (b, x: host arrays of nsys device
 * pointers, each of that member's length N_i).  o->restart must be 0 or the
 * batch's restart; the history buffer, if given, holds nsys rows of
 * history_len entries.  infos[i] (and statuses[i] if not NULL) receive each
 * member's result and status; seconds is the wall time of the whole batch and
 * the per-phase times are 0.  Returns ST_OK if every member converged,
 * ST_ENOTCONV if some did not, else the first error.  Blocks until done. */
int st_fgmres_solve_batched(st_batch* b, const double* const* bvec, double* const* x, const st_opts* o,
                            st_info* infos, int* statuses, void* stream);
int st_batch_destroy(st_batch* b);

/* Sizes of a created system: N, Ns, Nt. */
int st_sizes(const st_handle* h, int64_t* n_total, int* ns, int* nt);

/* Launch choices in effect for a created system (tuned when
   st_problem.autotune = 1): slabs per wavefront of the J apply, rows per
   workgroup of the sweep step kernels, 1 if the sweep solves run as tiled
   multi-step launches, the number of launches of one recorded P_T^{-1}
   apply (0 when it is launched step by step) and the lanes per row of the
   F_u,k step kernels.  Any pointer may be NULL. */
int st_tuning(const st_handle* h, int* j_slabs, int* step_rows, int* sweep_fuse, int* precond_launches,
              int* step_lanes);

/* Sampled timing of the dominant preconditioner kernel inside solves, for
 * roofline measurements.  kernel = 1 times the paired sweep-step kernel of
 * the recorded P_T^{-1} replay (one Chebyshev step of the C_A sweep, eq.
 * (CAs), and one of the F_u sweep, eq. (STFu), in one launch): every
 * `every`-th launch of it is issued with a pair of HIP events that take that
 * dispatch's start and end times (hipExtLaunchKernel; no packets between
 * launches; a pool of 8192 pairs, read after each st_fgmres_solve).  kernel = 0
 * turns it off.  Either call resets the counts.  ST_EINVAL if the handle
 * replays no recorded programs (single_stream = 1).  Host only. */
int st_profile_kernel(st_handle* h, int kernel, int every);

/* Summed event-timed duration (seconds) of the sampled launches, how many were
 * timed and how many launches of that kernel ran since st_profile_kernel. */
int st_profile_read(const st_handle* h, double* seconds, int64_t* launches_timed, int64_t* launches_seen);

const char* st_error_string(int code);

#ifdef __cplusplus
}
#endif

#endif /* ST_H */
