/*
 * cpgn.h -- C ABI of libcpgn.so: Gauss-Newton (preconditioned implicit CG) and ALS for dense
 * CP decomposition on AMD Instinct MI355X (gfx950).
 *
 * The operations follow N. Singh, L. Ma, H. Yang, E. Solomonik, "Comparison of Accuracy and
 * Scalability of Gauss-Newton and Alternating Least Squares for CP Decomposition"
 * (arXiv:1910.12331). Equation numbers refer to that paper: (1) Khatri-Rao product P^(n),
 * (2) Gamma^(n), (3) objective f, (4) Jacobian, (5) blocks of J^T J, (6) Gamma^(n,p),
 * (7) implicit matrix-vector contraction; Algorithm 1 is CP-GN and Algorithm 2 is CP-CG.
 *
 * Memory and ownership
 *   - X is a DEVICE pointer to a dense C-order tensor of shape dims[0] x ... x dims[N-1]
 *     (last index fastest).
 *   - A, G, W, Q are HOST arrays of N DEVICE pointers; entry n points to a row-major
 *     dims[n] x rank matrix (rank contiguous). Modes may have different sizes, hence the
 *     per-mode pointers.
 *   - Every buffer, including the workspace `ws`, is allocated and owned by the caller. The
 *     library allocates nothing and is re-entrant per stream; its only mutable state is each
 *     host thread's MTTKRP tile shape (cp_set_tuning) and cp_gn_step_noalloc's scratch array.
 *     Query the workspace size with cp_workspace_bytes; the workspace must be 256-byte
 *     aligned. Its contents need not be initialised and are clobbered.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream). Every call only
 *     enqueues work on that stream and returns without waiting.
 *
 * Error behaviour
 *   - The return value reports errors detectable on the host before anything is enqueued:
 *     CP_EINVAL (bad order/rank/dims/mode/method, null pointer, misaligned workspace),
 *     CP_EUNSUPPORTED (dtype combination), CP_EWORKSPACE (workspace too small), CP_EHIP (a
 *     launch failed). Nothing has been enqueued when a non-zero value is returned, except for
 *     CP_EHIP.
 *   - Failures found on the device (a non-SPD Cholesky pivot, CG breakdown <W,Q> <= 0,
 *     non-finite values) are written as a status code into device memory (the `status` field
 *     of cp_gn_stats, or `status_dev`); the caller reads it after synchronising the stream.
 *     On such a failure the factors are left unchanged.
 *   - Every call takes any rank. Up to 208 the R x R inverse (Gauss-Newton), the Cholesky
 *     factor (ALS) and the CG operand rows are held by one workgroup; above 208 they are blocked
 *     by 16 x 16 tiles in global memory (more launches per step). The triangular-solve
 *     preconditioner (CP_GN_CHOL_PRECOND) and the split and batched steps need rank <= 128.
 *
 * Precision
 *   - x_dtype equals f_dtype, CP_F64 or CP_F32; or f_dtype = CP_F32 and x_dtype = CP_BF16 or
 *     CP_BF16X3 (a bfloat16 tensor). With x_dtype = f_dtype the tensor contraction (MTTKRP,
 *     reconstruction) runs on the matrix cores in that precision with accumulation in the same
 *     precision. With a bfloat16 tensor the MTTKRP multiplies X by the inner factor rounded
 *     to bfloat16 (split into two bfloat16 parts for CP_BF16X3) on the bf16 matrix cores,
 *     accumulates in FP32 and applies the remaining Khatri-Rao factors in FP32; the residual
 *     reads X in bfloat16 and reconstructs in FP32. In every case the Grams, Gamma matrices,
 *     the CG vectors and scalars, Cholesky factors and all norms and inner products are kept in
 *     FP64 on the device.
 */
#ifndef CPGN_H
#define CPGN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CP_MAX_ORDER 8
#define CP_ABI_VERSION 1

/* Element types. CP_BF16 and CP_BF16X3 describe the tensor X only (x_dtype), with f_dtype =
   CP_F32:
     CP_BF16    X holds prod(dims) bfloat16 values.
     CP_BF16X3  X holds two planes of prod(dims) bfloat16 values each, hi then lo; the tensor is
                hi + lo (see cp_tensor_to_bf16). The contraction takes three bf16 products per
                term, hi*hi + hi*lo + lo*hi, of X's planes and a like split of the factor. */
typedef enum { CP_F64 = 0, CP_F32 = 1, CP_BF16 = 2, CP_BF16X3 = 3 } cp_dtype;

/* Return / device status codes. */
enum {
  CP_OK = 0,
  CP_EINVAL = -1,
  CP_EUNSUPPORTED = -2,
  CP_EWORKSPACE = -3,
  CP_EHIP = -4,
  CP_ENOTSPD = -5,      /* Gamma(n,n) + lambda I (or Gamma(n) + lambda I in ALS) not SPD  */
  CP_EBREAKDOWN = -6,   /* CG curvature sum <W,Q> <= 0                                     */
  CP_ENONFINITE = -7,   /* a NaN or Inf appeared in the gradient or the CG recurrences      */
  CP_ESCRATCH = -8      /* the problem needs more than the built-in scratch buffer          */
};

/* Workspace queries: one per entry point. */
enum {
  CP_OP_MTTKRP = 0,
  CP_OP_GN_GRADIENT = 1,
  CP_OP_GN_JTJ_MATVEC = 2,
  CP_OP_GN_STEP = 3,
  CP_OP_ALS_SWEEP = 4,
  CP_OP_RESIDUAL = 5,
  CP_OP_MTTKRP_ALL = 6
};

/* Residual methods for cp_residual. */
enum { CP_RESIDUAL_DIRECT = 0, CP_RESIDUAL_EXPANSION = 1 };

/* cp_gn_params.flags bits. CP_GN_DIAG_DAMPING: damp with lambda diag(J^T J) instead of lambda I
   (Section 3.2). The diagonal of J^T J in mode n's block is diag(Gamma^(n,n)) for every row
   (eq. (5)), so the CG system becomes (J^T J + lambda D) V = -G with D^(n) = diag(Gamma^(n,n)),
   and the preconditioner (Gamma^(n,n) + lambda diag(Gamma^(n,n)))^-1. */
#define CP_GN_DIAG_DAMPING 1u
/* CP_GN_CHOL_PRECOND: apply the preconditioner (Gamma^(n,n) + lambda D^(n))^-1 by a forward and a
   back triangular solve with its Cholesky factor instead of multiplying by its explicit inverse
   (the alternative Section 3.3 describes and sets aside for its parallel depth: each solve is
   sequential in R). Same CG iterates up to rounding; rank <= 128 (CP_EUNSUPPORTED above). */
#define CP_GN_CHOL_PRECOND 2u

typedef struct {
  int32_t order;                 /* N, 2 <= N <= CP_MAX_ORDER                               */
  int32_t rank;                  /* R >= 1                                                  */
  int64_t dims[CP_MAX_ORDER];    /* s_1..s_N, each >= 1; entries past N are ignored         */
  int32_t x_dtype;               /* cp_dtype of X                                           */
  int32_t f_dtype;               /* cp_dtype of the factor matrices and per-mode outputs    */
} cp_problem;

typedef struct {
  double lambda;                 /* Tikhonov damping of J^T J + lambda I (>= 0), Section 3.2 */
  double cg_tol;                 /* eps_cg: CG runs while sum||R(n)|| > eps_cg sum||G(n)||   */
  int32_t cg_maxiter;            /* cap on CG iterations (>= 0)                              */
  uint32_t flags;                /* CP_GN_DIAG_DAMPING | CP_GN_CHOL_PRECOND; others must be 0 */
} cp_gn_params;

/* Written to DEVICE memory by cp_gn_step. */
typedef struct {
  int32_t status;                /* CP_OK or a device status code                           */
  int32_t cg_iters;              /* CG iterations taken                                     */
  double grad_norm_sum;          /* sum_n ||G(n)||_F at the start of the step               */
  double cg_res_norm_sum;        /* sum_n ||R(n)||_F when CG stopped                        */
  double alpha_last;             /* last CG step length (0 if no iteration)                 */
  double beta_last;              /* last CG direction coefficient (0 if no iteration)       */
  double update_norm;            /* sqrt(sum_n ||V(n)||_F^2) of the applied update          */
} cp_gn_stats;

/* Size in bytes of the workspace entry point `op` needs for this problem. */
int cp_workspace_bytes(const cp_problem* prob, int op, size_t* bytes);

/*
 * MTTKRP, Section 2.2: M = X_(n) P^(n), with P^(n) the Khatri-Rao product of every factor but
 * A^(n) (eq. (1)); elementwise M[k,r] = sum over indices i with i_n = k of
 * X[i] * prod_{m != n} A^(m)[i_m, r].
 *   mode: n, 0-based. M: device, dims[mode] x rank, f_dtype, written.
 */
int cp_mttkrp(const cp_problem* prob, const void* X, const void* const* A, int mode, void* M,
              void* ws, size_t ws_bytes, void* stream);

/*
 * cp_mttkrp with its main kernel bracketed for timing: the HIP events `kernel_begin` and
 * `kernel_end` (hipEvent_t, created by the caller; either may be NULL) are recorded on `stream`
 * right before the first and after the last launch of the MTTKRP kernel proper, so that
 * hipEventElapsedTime gives that kernel's duration without the factor preparation before it and
 * the partial-tile reduction after it. Same result, arguments and errors as cp_mttkrp.
 */
int cp_mttkrp_marked(const cp_problem* prob, const void* X, const void* const* A, int mode,
                     void* M, void* ws, size_t ws_bytes, void* stream, void* kernel_begin,
                     void* kernel_end);

/*
 * All-mode MTTKRP: M^(n) = X_(n) P^(n) (Section 2.2, eq. (1)) for every mode n at one point, the
 * contractions that form the gradient of Algorithm 1. For an FP32/FP64 tensor of order >= 3
 * whose last mode is a multiple of 4 (16-byte aligned X), modes 0 .. N-2 come from one pass over
 * X (a dimension tree, Section 2.2: the partial contraction with A^(N-1) is shared; above order 3
 * the middle modes are formed from its FP64 per-outer-index sums, while those take at most a
 * quarter of X's bytes) and mode N-1 from a second pass; otherwise one pass per mode. The
 * gradient (cp_gn_gradient, cp_gn_step) forms its MTTKRPs the same way.
 *   M: N device pointers, M[n] is dims[n] x rank, f_dtype, written.
 */
int cp_mttkrp_all(const cp_problem* prob, const void* X, const void* const* A, void* const* M,
                  void* ws, size_t ws_bytes, void* stream);

/*
 * Gradient of f (eq. (3)) for every mode at one point, Algorithm 1:
 * G^(n) = A^(n) Gamma^(n,n) - M^(n), with Gamma^(n,n) the Hadamard product of the Grams
 * S^(m) = A^(m)T A^(m), m != n (eq. (2)).
 *   G: N device pointers, dims[n] x rank, f_dtype, written.
 *   grad_norm_sum_dev: device double, receives sum_n ||G^(n)||_F (may be NULL).
 */
int cp_gn_gradient(const cp_problem* prob, const void* X, const void* const* A, void* const* G,
                   double* grad_norm_sum_dev, void* ws, size_t ws_bytes, void* stream);

/*
 * Objective and gradient together, for a differentiable objective whose forward pass keeps the
 * gradient for its backward pass: G^(n) = A^(n) Gamma^(n,n) - M^(n) for every mode (as
 * cp_gn_gradient, the same kernels and bits), and the residual norm of eq. (3) by the expansion
 * ||X - [[A]]||^2 = ||X||^2 - 2 <M^(1), A^(1)> + sum_{r,z} prod_m S^(m)_{rz} from the same M^(1)
 * and Grams, so that f costs one extra pass over X (for ||X||^2) and no matrix work. The
 * expansion cancels as the fit becomes exact: its absolute error in ||X - [[A]]||^2 is about the
 * MTTKRP's relative accuracy times ||X||^2 (FP32 storage: ~1e-6 ||X||^2), against cp_residual's
 * direct form. A negative square is clamped to 0.
 *   G: N device pointers, dims[n] x rank, f_dtype, written.
 *   res_dev: device double[2]: [0] = ||X - [[A]]||_F by the expansion, [1] = ||X||_F.
 *   ws: at least cp_workspace_bytes(CP_OP_GN_GRADIENT).
 */
int cp_objective_gradient(const cp_problem* prob, const void* X, const void* const* A,
                          void* const* G, double* res_dev, void* ws, size_t ws_bytes,
                          void* stream);

/*
 * Damped Gauss-Newton matrix-vector product, Algorithm 2 with eqs. (5)-(7):
 * Q^(n) = lambda W^(n) + sum_p sum_{l,z} h^(n,p)_{krlz} W^(p)_{lz}, i.e. Q = (J^T J + lambda I) W.
 *   W: N device pointers (input), Q: N device pointers (output), both dims[n] x rank, f_dtype.
 */
int cp_gn_jtj_matvec(const cp_problem* prob, const void* const* A, const void* const* W,
                     double lambda, void* const* Q, void* ws, size_t ws_bytes, void* stream);

/*
 * One loop body of Algorithm 1 (CP-GN): all MTTKRPs at the current point, Grams and Gamma
 * matrices, G^(n), then Algorithm 2 (CP-CG) on (J^T J + lambda I) V = -G with the block
 * preconditioner (Gamma^(n,n) + lambda I)^-1 (Section 3.3), then A^(n) += V^(n). With
 * CP_GN_DIAG_DAMPING in params->flags, lambda I is replaced by lambda diag(J^T J) in both.
 * CG uses beta = sum<R,Z>_new / sum<R,Z>_old (standard preconditioned CG).
 *   A: N device pointers, read and overwritten in place (f_dtype).
 *   params: HOST pointer. stats: DEVICE pointer to one cp_gn_stats.
 */
int cp_gn_step(const cp_problem* prob, const void* X, void* const* A, const cp_gn_params* params,
               cp_gn_stats* stats, void* ws, size_t ws_bytes, void* stream);

/*
 * cp_gn_step with the damping read from device memory when the step runs, for callers that
 * replay the step from a captured HIP graph (its kernel arguments are then fixed): lambda_dev
 * points to one device double (>= 0, finite); params->lambda is ignored. A negative or non-finite
 * value there is reported as CP_EINVAL in stats->status and leaves the factors unchanged.
 * Everything else is as for cp_gn_step.
 */
int cp_gn_step_devlam(const cp_problem* prob, const void* X, void* const* A,
                      const cp_gn_params* params, const double* lambda_dev, cp_gn_stats* stats,
                      void* ws, size_t ws_bytes, void* stream);

/*
 * cp_gn_step without a workspace argument, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc). The
 * workspace is a device array built into the library, CP_NOALLOC_SCRATCH_BYTES long, of which
 * every GPU the library runs on holds one copy until the process ends; the call allocates
 * nothing. Its device address is looked up once per device, on the first call made with that
 * device current (hipGetSymbolAddress); the stream must belong to the current device.
 * Every call on one GPU shares that GPU's array and leaves its contents behind: calls that
 * overlap on one GPU (concurrent streams, several threads) race and must be serialised by the
 * caller. The step reads nothing from the array that it has not written in the same call.
 *   Arguments and results as for cp_gn_step.
 *   Errors: CP_ESCRATCH (before any launch) when cp_workspace_bytes(CP_OP_GN_STEP) exceeds
 *   CP_NOALLOC_SCRATCH_BYTES (64 MiB: 400^3 at rank 100 needs 30 MiB in FP32, 44 MiB in FP64);
 *   CP_EHIP when the scratch address cannot be obtained; otherwise as cp_gn_step.
 */
#define CP_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int cp_gn_step_noalloc(const cp_problem* prob, const void* X, void* const* A,
                       const cp_gn_params* params, cp_gn_stats* stats, void* stream);

/* Armijo step-size control of a Gauss-Newton step (Section 5). */
typedef struct cp_armijo_params {
  double c;             /* sufficient-decrease constant, 0 < c < 1 (e.g. 1e-4)                 */
  double shrink;        /* factor between successive step sizes, 0 < shrink < 1 (e.g. 0.5)     */
  int32_t max_trials;   /* objective evaluations at most, 0..64                                */
  uint32_t flags;       /* 0 or CP_LS_F0_GIVEN; other bits must be 0                           */
} cp_armijo_params;

/* cp_armijo_params.flags bit. CP_LS_F0_GIVEN: f(A) and ||X||_F are read from the cp_armijo_stats
   that the previous cp_gn_step_armijo call on these same factors wrote (its f and x_norm: f at
   the point it returned), instead of one more direct residual pass over X at the start. The
   caller guarantees that the factors have not changed since that call. */
#define CP_LS_F0_GIVEN 1u

typedef struct cp_armijo_stats {
  double alpha;         /* accepted step size; 0 if none was accepted                          */
  double f0;            /* f = 1/2 ||X - [[A]]||_F^2 (eq. (3)) at the start point               */
  double f;             /* f at the returned point (f0 if no step size was accepted)           */
  double gv;            /* sum_n <G(n), V(n)>: slope of f along the Gauss-Newton direction V    */
  double x_norm;        /* ||X||_F                                                             */
  int32_t trials;       /* objective evaluations made                                          */
  int32_t accepted;     /* 1 if a step size passed the test                                    */
} cp_armijo_stats;

/*
 * Gauss-Newton step with Armijo step-size control, the variant Section 5 uses for the
 * matrix-multiplication tensors. The direction V is the one cp_gn_step computes (Algorithm 1 with
 * CG, same params and damping flags); the step sizes alpha = 1, shrink, shrink^2, ... (at most
 * max_trials) are then tried in that order and the first with
 *     f(A + alpha V) <= f(A) + c alpha sum_n <G(n), V(n)>
 * (f of eq. (3) evaluated directly, G the gradient) is applied: A(n) <- A(n) + alpha V(n). No trial
 * runs when the CG status is a failure, when sum <G, V> >= 0 (no descent, e.g. V = 0 with
 * cg_maxiter = 0) or when f(A) is not finite; then, and when no trial passes, the factors are left
 * unchanged and accepted = 0. The search runs on the device without host synchronisation: every
 * trial is launched and the ones after a passing trial return at once. With max_trials = 1 it is
 * the accept-or-reject rule of a damped Gauss-Newton (Levenberg-Marquardt) iteration: the full
 * step is taken only when it decreases f enough, so a run never leaves a converging trajectory
 * when the gradient has become rounding noise. With CP_LS_F0_GIVEN in ls->flags, f(A) comes from
 * the previous call's ls_stats (read on the device, stream-ordered) and the step costs one
 * residual pass (the trial) instead of two.
 *   A: N device pointers, read and overwritten in place (f_dtype).
 *   params, ls: HOST pointers. stats: DEVICE pointer to one cp_gn_stats (update_norm is
 *   ||alpha V||). ls_stats: DEVICE pointer to one cp_armijo_stats.
 *   ws: at least cp_workspace_bytes(CP_OP_GN_STEP).
 *   Errors: CP_EINVAL for null pointers or parameters out of range (before any launch);
 *   CP_GN_CHOL_PRECOND above rank 128: CP_EUNSUPPORTED.
 */
int cp_gn_step_armijo(const cp_problem* prob, const void* X, void* const* A,
                      const cp_gn_params* params, const cp_armijo_params* ls, cp_gn_stats* stats,
                      cp_armijo_stats* ls_stats, void* ws, size_t ws_bytes, void* stream);

/*
 * The varying damping of Section 3.2 advanced once on the device (one tiny kernel, so a captured
 * graph can carry the schedule with the step). state_dev: device double[5] =
 * {lambda, lower, upper, mu, decreasing (1.0 or 0.0)}; while decreasing, lambda /= mu and the
 * direction turns when lambda <= lower; otherwise lambda *= mu and it turns when lambda >= upper.
 */
int cp_damping_advance(double* state_dev, void* stream);

/*
 * A Gauss-Newton step (Algorithm 1) split in three calls, so that the CG iterations (Algorithm 2)
 * of many independent problems share launches; for each problem the three calls together do
 * exactly what cp_gn_step_devlam does (the same kernels on the same data: bitwise the same
 * factors and stats). R <= 128, explicit-inverse preconditioner (no CP_GN_CHOL_PRECOND).
 *   cp_gn_step_begin  everything before CG on `stream`: prepared factors, the gradient of
 *                     Algorithm 1, the preconditioner of Section 3.3 (lambda_dev: device
 *                     damping as in cp_gn_step_devlam, or NULL for params->lambda), and the
 *                     problem's CG arguments, stored in its workspace `ws`.
 *   cp_gn_cg_batch    CG initialisation, cg_maxiter iterations and the final state of `count`
 *                     (<= CP_MAX_CG_BATCH) problems whose steps have begun: probs[i] and ws[i]
 *                     (ws_bytes[i] bytes) as given to cp_gn_step_begin; three launches per
 *                     iteration for the whole batch. Every problem stops at its own test.
 *   cp_gn_step_end    A += V and the step's stats (device) for one problem.
 * Stream order: begin of a problem, then the batch, then its end (join and fork the streams with
 * events when problems begin on several streams).
 */
#define CP_MAX_CG_BATCH 128
int cp_gn_step_begin(const cp_problem* prob, const void* X, void* const* A,
                     const cp_gn_params* params, const double* lambda_dev, void* ws,
                     size_t ws_bytes, void* stream);
int cp_gn_cg_batch(int count, const cp_problem* probs, void* const* ws, const size_t* ws_bytes,
                   int cg_maxiter, void* stream);
int cp_gn_step_end(const cp_problem* prob, void* const* A, cp_gn_stats* stats, void* ws,
                   size_t ws_bytes, void* stream);

/*
 * A batch program: one Gauss-Newton step (Algorithm 1, CG of Algorithm 2) of `count` independent
 * problems in shared launches. cp_gn_batch_create records, once, the launches that
 * cp_gn_step_begin and cp_gn_step_end make for each problem (and a cp_damping_advance when
 * damping_state[i] is given), with their arguments; cp_gn_batch_step then enqueues, for each
 * position in the step, one launch per kernel that runs the workgroups of every problem at that
 * position (a workgroup finds its problem from a table of workgroup offsets), with the CG of all
 * problems in between as cp_gn_cg_batch does. Each problem computes exactly what its three split
 * calls compute (bitwise the same factors, stats and damping), in about 40 launches per step
 * for the whole batch instead of about 20 per problem plus the shared CG.
 *   count: >= 1. probs[i], X[i], ws[i] (ws_bytes[i] >= cp_workspace_bytes(CP_OP_GN_STEP)): as
 *     for cp_gn_step_begin. A: count * CP_MAX_ORDER device pointers, A[i * CP_MAX_ORDER + n] the
 *     factor n of problem i (read and overwritten by each step). params: HOST pointer, shared by
 *     all problems (CP_GN_CHOL_PRECOND not supported). lambda_dev: NULL (params->lambda for all)
 *     or count device pointers (an entry may be NULL: params->lambda). damping_state: NULL or
 *     count device double[5] schedules (entries may be NULL) advanced after each step as by
 *     cp_damping_advance. stats: count device pointers to cp_gn_stats.
 *   table: caller-owned device memory for the recorded arguments, table_bytes long (16-byte
 *     aligned); *table_needed (host) receives the size required. With table NULL or too small
 *     the call returns CP_EWORKSPACE after setting *table_needed, and creates nothing.
 *   *out (host) receives the program. It refers to every pointer above (none is copied): they
 *     must stay valid and keep their sizes while the program is used. The recorded arguments are
 *     copied into `table` synchronously before the call returns.
 * Errors: CP_EINVAL (null or inconsistent arguments), CP_EUNSUPPORTED (rank above 128, bfloat16
 * storage, or the Cholesky preconditioner), CP_EWORKSPACE (workspace or table too small), or a
 * HIP error of the table copy. cp_gn_batch_step enqueues one step on `stream` (CP_EINVAL for a
 * null program); cp_gn_batch_destroy releases the host-side program (not the caller's memory).
 */
typedef struct cp_gn_batch cp_gn_batch;
int cp_gn_batch_create(int count, const cp_problem* probs, const void* const* X, void* const* A,
                       const cp_gn_params* params, double* const* lambda_dev,
                       double* const* damping_state, cp_gn_stats* const* stats,
                       void* const* ws, const size_t* ws_bytes, void* table, size_t table_bytes,
                       size_t* table_needed, cp_gn_batch** out);
int cp_gn_batch_step(cp_gn_batch* program, void* stream);
int cp_gn_batch_destroy(cp_gn_batch* program);

/*
 * Device timestamps for per-problem step latencies (p50/p99) of many problems run on several
 * streams: enqueues one one-thread kernel on `stream` that writes the device's constant-rate
 * clock to *dst_dev when it runs, so that two of them around a step bracket the step's execution
 * on the device. dst_dev: device int64_t, written. cp_device_clock_hz returns the rate of that
 * clock in *hz (host int64_t) for the current device. CP_EINVAL for a null pointer.
 */
int cp_device_timestamp(int64_t* dst_dev, void* stream);
int cp_device_clock_hz(int64_t* hz);

/*
 * One ALS sweep, Section 2.2: for n = 0..N-1 in order, A^(n) = M^(n) (Gamma^(n) + lambda I)^-1
 * with M^(n) computed from the latest factors: the FP64 Cholesky factor L L^T = Gamma^(n) +
 * lambda I, then Y L^T = M^(n) and A^(n) L = Y by blocked substitution (16-column blocks; the
 * 16 x 16 diagonal blocks of L act through their inverses). No explicit inverse of Gamma^(n).
 * For an order-3 FP32/FP64 tensor the workspace that cp_workspace_bytes(CP_OP_ALS_SWEEP) reports
 * also holds T = X x_3 A^(3) (dims[0] dims[1] x rank words): M^(1) and M^(2) are then formed from
 * T (a dimension tree: two passes over X per sweep instead of three). Given only the smaller
 * workspace of the other operations, the sweep takes one pass per mode.
 *   A: N device pointers, read and overwritten in place. lambda >= 0 (0 = plain ALS).
 *   status_dev: device int32 receiving CP_OK or CP_ENOTSPD (a pivot <= 0: that mode and the ones
 *   after it keep their factors; may be NULL). Any rank: above 208 the Cholesky factor and the
 *   substitutions are blocked by 16 x 16 tiles in global memory, one launch per block column.
 */
int cp_als_sweep(const cp_problem* prob, const void* X, void* const* A, double lambda,
                 int32_t* status_dev, void* ws, size_t ws_bytes, void* stream);

/*
 * Residual norms, Section 5 (relative residual r = ||X - [[A]]||_F / ||X||_F, fitness 1 - r).
 *   method CP_RESIDUAL_DIRECT: streams X once and rebuilds [[A]] tile by tile.
 *   method CP_RESIDUAL_EXPANSION: ||X||^2 - 2<M^(1),A^(1)> + sum_{r,z} prod_m S^(m)_{rz}; cheap
 *     but it cancels catastrophically near an exact fit (a negative square is clamped to 0).
 *   out_dev: device double[2]: out_dev[0] = ||X - [[A]]||_F, out_dev[1] = ||X||_F.
 */
int cp_residual(const cp_problem* prob, const void* X, const void* const* A, int method,
                double* out_dev, void* ws, size_t ws_bytes, void* stream);

/*
 * Storage conversion for the bfloat16 tensor forms (x_dtype CP_BF16 / CP_BF16X3); not a step of
 * the method. Rounds the n FP32 values of X to nearest bfloat16 (ties to even) into out[0..n).
 * With split != 0 it also writes the rounded remainder lo = bf16(x - hi) into out[n..2n), so
 * that hi + lo carries about 16 significant bits of x.
 *   X: device, n floats (finite). out: device, n (or 2n with split) 16-bit values, written.
 *   Returns CP_EINVAL for n < 0 or a NULL pointer with n > 0.
 */
int cp_tensor_to_bf16(const float* X, int64_t n, int split, void* out, void* stream);

/*
 * Tile shape of the FP32/FP64 MTTKRP launches (Section 2.2's contraction; not a step of the
 * method). A tuning choice for many small problems, where the best split of a mode's work over
 * wavefronts depends on the shapes: every setting computes the same contraction, but the
 * partial sums are added in a different order, so results agree to rounding, not bitwise, across
 * settings (bitwise for one setting). Zero fields take the defaults.
 *   mttkrp_min_items: least (outer index, 16-wide inner chunk) items per wavefront before a row
 *     tile's items are split over more wavefronts; 1..4096, default 16.
 *   mttkrp_wg_per_cu: workgroups per compute unit one launch aims for; 1..8, default 2.
 *   mttkrp_row_block: 16-row blocks per row tile of the FP32 kernel for modes whose inner index
 *     runs along X rows (n < N-1, 16-byte aligned rows); 2, 4 or 5, default automatic (5 where
 *     80-row tiles pad the mode less than 64-row ones, else 4). Other kernels keep their tiles.
 *   reserved: must be 0.
 * cp_set_tuning applies to the calling host thread: to the workspace sizes, launches and batch
 * programs of calls made from it afterwards (a batch program keeps the setting of its
 * cp_gn_batch_create). A workspace sized under one setting can be too small for another
 * (CP_EWORKSPACE). t == NULL restores the defaults. CP_EINVAL for a field out of range.
 * cp_get_tuning writes the calling thread's setting (zeros for defaults) to *t (host).
 */
typedef struct {
  int32_t mttkrp_min_items;
  int32_t mttkrp_wg_per_cu;
  int32_t mttkrp_row_block;
  int32_t reserved;
} cp_tuning;
int cp_set_tuning(const cp_tuning* t);
int cp_get_tuning(cp_tuning* t);

/* Static description of a status code. */
const char* cp_status_string(int status);

/* CP_ABI_VERSION of the built library. */
int cp_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CPGN_H */
