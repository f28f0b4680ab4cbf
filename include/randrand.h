/*
 * randrand.h — C ABI of the RandRAND (randomized range deflation) solver library
 * for MI355X (gfx950).
 *
 * Problem (paper, Section 1, eq. initsys): solve (A + mu I) x = b with A
 * symmetric positive semidefinite and mu >= 0, A reached through matvecs (a
 * stored dense matrix) or through its entries (a Gaussian RBF or Matern-3/2
 * kernel formed on the fly).  The preconditioner is C-RandRAND (Section 3.2,
 * eq. c_randrand_def) in its explicit-basis form (Section 4.1,
 * eq. g_randrand_explicit):
 *
 *     P = I - Pi + tau Pi A_mu^{-1} Pi = I + Q (tau T G T - T) Q^T,
 *     A_mu Omega = Q R,  G = R^{-T} (Omega^T A_mu Omega) R^{-1},  T = 2I - Q^T Q,
 *
 * used inside PCG with restarts (Algorithm RandRAND_PCG, Section 6.2).  The same
 * handle also serves preconditioned MINRES, R-RandRAND and split R-RandRAND
 * (Section 3.1, Algorithms RandRAND_CG and RandRAND_CG_split), block MINRES and
 * block CG over several right-hand sides (Section 7.2.2), and a basis-less form
 * (Section 4.1, Algorithm BL_RandRAND_PCG); see rr_method, rr_krylov and rr_basis.
 *
 * Conventions for every entry point:
 *  - All functions are extern "C", never throw, never abort, and return rr_status.
 *  - Matrices are column-major.  "device" pointers are HIP device memory on the
 *    current device; "host" pointers are ordinary host memory.
 *  - The caller owns every buffer it passes in.  Operator memory (A, pts) is
 *    borrowed by a preconditioner handle and must outlive it.  A handle owns the
 *    memory it allocates (Omega, Y, Q, the l x l factors, workspaces) and
 *    releases it in rr_precond_destroy.
 *  - Device work is enqueued on the caller's hipStream_t (passed as void*;
 *    NULL = the default stream).  rr_build_precond, rr_solve and
 *    rr_solve_batch return only after their work has completed.
 *  - On failure the function returns a non-zero rr_status; rr_last_error()
 *    returns a thread-local message describing it.  RR_EINVAL is returned
 *    before any device work is done.
 */
#ifndef RANDRAND_H
#define RANDRAND_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RR_OK = 0,
    RR_EINVAL = 1,      /* invalid argument (checked before any device work)        */
    RR_ENOMEM = 2,      /* device allocation failed or the memory budget is exceeded */
    RR_ENOTSPD = 3,     /* Cholesky failed after the whole shift ladder             */
    RR_EBREAKDOWN = 4,  /* PCG breakdown: p^T A_mu p <= 0 or r^T z <= 0            */
    RR_ENOCONV = 5,     /* maxit reached; x holds the last iterate, info is filled   */
    RR_EDEVICE = 6,     /* HIP runtime error or no usable GPU                        */
    RR_EBUSY = 7        /* resource in use                                           */
} rr_status;

/* Operator kinds (Section 1: A symmetric psd, reached by matvecs or entries). */
typedef enum { RR_OP_DENSE = 0, RR_OP_RBF = 1, RR_OP_MATERN32 = 2 } rr_op_kind;

/*
 * The operator A (not including the shift mu).
 *  DENSE:     A   device, float64, n x n column-major, leading dimension lda >= n,
 *                 symmetric (only its symmetry is assumed, not checked).
 *  RBF:       pts device, float32, structure-of-arrays d x n (pts[k*n + i] is
 *                 coordinate k of point i); A_ij = scale * exp(-kconst ||x_i - x_j||^2).
 *  MATERN32:  same layout; A_ij = scale * (1 + kconst r) exp(-kconst r), r = ||x_i - x_j||.
 *  kconst is 1/(2 sigma^2) (RBF) or sqrt(3)/ell (Matern-3/2); scale is 1 for a
 *  plain Gram matrix and 1/n for the kernel ridge normalisation (Section 7.2.2,
 *  eq. kernel).  Unused fields are ignored.
 */
typedef struct {
    int32_t kind;
    int64_t n;
    const double* A;
    int64_t lda;
    const float* pts;
    int32_t d;
    double kconst;
    double scale;
} rr_operator;

/* Test matrix Omega (Section 1.1 eq. testmatrix; Section 2).  COLSAMPLE: signed
 * uniform column sampling (column c = sgn_c e_idx_c, l distinct indices), the
 * paper's test matrix for kernel systems (Section 7.2.2, limited-memory KRR). */
typedef enum { RR_SK_GAUSSIAN = 0, RR_SK_SRHT = 1, RR_SK_COLSAMPLE = 2 } rr_sketch;
/* Representation of the deflation basis (Section 4).  EXPLICIT: Q (n x l) stored.
 * LESS: basis-less (Section 4.2, Algorithm BL_RandRAND_PCG): only R, the l x l
 * factors and the sampled indices are kept; Q^T u = R^{-T} (A_mu Omega)^T u and
 * Q d = (A_mu Omega) R^{-1} d are formed from kernel entries on every use (kernel
 * operators, COLSAMPLE test matrix, one shift; O(n + l^2) memory). */
typedef enum { RR_BASIS_EXPLICIT = 0, RR_BASIS_LESS = 1 } rr_basis;
/* Orthogonalisation of A_mu Omega: Algorithm prec_chol_qr (sketched, default) or chol_qr. */
typedef enum { RR_ORTH_SKETCHED_CHOLQR = 0, RR_ORTH_CHOLQR = 1 } rr_orth;
/*
 * Working precision.
 *  FP64:  everything float64.
 *  FP32:  matvec with float32-class entries and float64 accumulation (a float32
 *         copy of a dense A; kernel entries whose exponents are float32-accurate
 *         record products on bf16 MFMA, each term split into three bf16 pieces);
 *         sketch: kernel operators on bf16 MFMA with each kernel entry split into
 *         bf16 hi + lo (about 16 significant bits) and Omega drawn in bf16, dense
 *         operators on float64 MFMA from the float32 copy; Q, Gram, Cholesky, dots
 *         and vectors float64.
 *  MIXED: as FP32 but a dense sketch runs bf16 x bf16 -> float32 on MFMA.
 *  In FP32 and MIXED the residual at every restart is taken with the float64
 *  operator by default (outer float64 iterative refinement, rr_solve_opts.fp64_ir).
 */
typedef enum { RR_PREC_FP64 = 0, RR_PREC_FP32 = 1, RR_PREC_MIXED = 2 } rr_precision;
/*
 * tau rule (Section 3.2).
 *  OPT: tau = sqrt(mu ||E|| / lam)  (eq. optimal_rho with F = 1/mu in eq. c_randrand_tau);
 *       falls back to RHO when mu == 0.
 *  RHO: tau = rho ||E|| / lam        (eq. c_randrand_tau).
 *  NYS: tau = 1 / lambda_max(G) = ||Pi A_mu^{-1} Pi||^{-1} (eq. nys_tau).
 * ||E|| = ||(I-Pi) A_mu (I-Pi)|| and lam = lambda_max(Pi A_mu Pi A_mu^{-1} Pi) are
 * power-iteration estimates (power_iters steps each).
 */
typedef enum { RR_TAU_OPT = 0, RR_TAU_RHO = 1, RR_TAU_NYS = 2 } rr_tau_rule;

/*
 * How rr_solve uses the handle (Section 6).
 *  C:        C-RandRAND preconditioner P = I - Pi + tau Pi A_mu^{-1} Pi inside the
 *            Krylov method (Algorithm RandRAND_PCG).
 *  R:        R-RandRAND (Algorithm RandRAND_CG): the Krylov method runs on
 *            B = (I-Pi) A_mu (I-Pi) + ||E|| Pi (eq. APdef2 with tau = ||E||, eq. cnd_bound,
 *            rho = 1) and each cycle recovers x with eq. APdef3.
 *  SPLIT_R:  split R-RandRAND (Algorithm RandRAND_CG_split): the Krylov method runs on
 *            E y = (I-Pi)(I-Pi) b, E = (I-Pi) A_mu, then x = A_mu^{-1} Pi (b - A_mu y) + y.
 * Pi = Q T Q^T is the refined projector (eq. accurate_proj) and A_mu^{-1} Pi u =
 * Omega R^{-1} T Q^T u.  R and SPLIT_R need a single-shift handle with l >= 1 (R also
 * the ||E|| estimate of the OPT or RHO tau rule).
 */
typedef enum { RR_METHOD_C = 0, RR_METHOD_R = 1, RR_METHOD_SPLIT_R = 2 } rr_method;
/* Krylov method: CG (Hestenes-Stiefel) or MINRES (Paige-Saunders, preconditioned for
 * method C), both restarted after each residual drop by restart_eta.
 * BLOCK_MINRES / BLOCK_CG (rr_solve_batch with method C only): the columns under one
 * shift are solved together, in groups of at most RR_BLOCK_MAX columns (in column
 * order), over the block Krylov space of the preconditioned operator, with every
 * stored Krylov block reorthogonalised twice per step (Section 7.2.2: block
 * preconditioned MINRES with Krylov basis reorthogonalisation).  BLOCK_MINRES
 * minimises each column's residual in the norm of P (block Lanczos in that inner
 * product, block QR of the band matrix); BLOCK_CG takes the Galerkin step with
 * A_mu-orthonormal direction blocks.  A group converges when
 * max_i ||b_i - A_mu x_i|| / ||b_i|| <= tol; a restart keeps only the columns not yet
 * at tol; a cycle also ends after block_kmax steps (its stored blocks).  iters counts
 * block steps (one operator product per group block).  A group whose residual block
 * is not numerically full rank at a cycle start (a Cholesky pivot c_jj^2 <= 1e-20 S_jj
 * of its Gram matrix, e.g. equal or dependent right-hand sides) stops with
 * RR_EBREAKDOWN for its unconverged columns. */
#define RR_BLOCK_MAX 32
typedef enum { RR_KRYLOV_CG = 0, RR_KRYLOV_MINRES = 1, RR_KRYLOV_BLOCK_MINRES = 2,
               RR_KRYLOV_BLOCK_CG = 3 } rr_krylov;

/*
 * Several shifts in one handle (Section 5.1).
 *  JOINT:         one joint basis orth([Omega, A Omega]) and a 2l x l Householder QR per
 *                 shift.
 *  SHIFTED_CHOL:  one orthogonalisation of A_alpha Omega at alpha = the largest shift,
 *                 then per shift R = R_chol R_alpha with R_chol = chol of the Gram
 *                 W2 + 2 (mu - alpha) W1 + (mu - alpha)^2 W0 of A_mu Omega R_alpha^{-1}
 *                 (shifted Cholesky preconditioning), the basis
 *                 Q_mu = [Q_alpha, Omega R_alpha^{-1}] [I; (mu - alpha) I] R_chol^{-1}.
 */
typedef enum { RR_MULTI_JOINT = 0, RR_MULTI_SHIFTED_CHOL = 1 } rr_multi_shift;

typedef struct {
    int64_t l;            /* columns of Omega (sketch size); 0 = plain CG (P = I)       */
    int32_t sketch;       /* rr_sketch                                                   */
    uint64_t seed;        /* Omega: stream seed; Theta: seed+1; power starts: seed+2/+3  */
    int32_t orth;         /* rr_orth                                                     */
    int32_t prec;         /* rr_precision                                                */
    int32_t tau_rule;     /* rr_tau_rule                                                 */
    double rho;           /* RHO rule factor (default 1.0)                               */
    int32_t power_iters;  /* power iterations per estimate (default 4)                   */
    int32_t power_q;      /* q of eq. testmatrix: Omega = A^q X, q in {0, 1} (default 0) */
    int32_t multi_shift;  /* rr_multi_shift for n_mu > 1 (default JOINT)                 */
    int64_t l_max;        /* > l: adaptive sketch size (Section 5.3, eq. ad_criterion):
                             build with l, l <- min(2 l, l_max) while the ||E|| estimate
                             exceeds ad_factor (n / l_max)^(1/(2q+2)) mu and the last
                             doubling cut it below 0.9 of its previous value; single
                             shift, tau rule OPT or RHO.  0: off (default)               */
    double ad_factor;     /* f of eq. ad_criterion (default 100)                         */
    int32_t basis;        /* rr_basis (default EXPLICIT)                                 */
    int32_t reorth;       /* 1: re-orthogonalised C-RandRAND, eq. c_randrand_reorth: core
                             tau T G - T in place of tau T G T - T (default 0)           */
} rr_build_opts;

typedef struct {
    double tol;           /* stop when ||b - A_mu x|| <= tol ||b||  (default 1e-6)        */
    double restart_eta;   /* restart after each residual drop by this factor (1e-2)      */
    int32_t maxit;        /* maximum PCG iterations (default 5000)                       */
    int32_t check_every;  /* iterations per device launch batch between host checks (8)  */
    int32_t fp64_ir;      /* 1: residual at restarts with the float64 operator (outer
                             float64 refinement); -1: by precision (on unless the handle
                             works in FP64); 0: off                                      */
    double* relres_history;  /* optional host array: relative residual per iteration     */
    int32_t history_cap;     /* its length                                               */
    int32_t use_graph;    /* 1: replay each batch of iterations as a captured hipGraph   */
    int32_t certify;      /* 1: when refinement is off, one float64-operator residual
                             after convergence fills info.relres_fp64 (not counted in
                             ms_solve); with refinement on, or in FP64, the final true
                             residual is already the float64 one; 0: skip             */
    int32_t method;       /* rr_method (default C); rr_solve_batch runs C only           */
    int32_t krylov;       /* rr_krylov (default CG); rr_solve takes CG or MINRES,
                             rr_solve_batch CG, BLOCK_MINRES or BLOCK_CG               */
    int32_t block_kmax;   /* block solvers: steps per cycle, i.e. Krylov blocks kept for
                             reorthogonalisation (2 x (block_kmax + 1) n x s float64
                             blocks per group); default 128                           */
} rr_solve_opts;

typedef struct {
    int32_t iters;        /* Krylov iterations (operator products inside the cycles)      */
    int32_t restarts;     /* restarts after the first cycle                               */
    double relres_work;   /* final relative residual with the working operator            */
    double relres_fp64;   /* final relative residual with the float64 operator            */
    double tau, normE, lamhat;  /* preconditioner scale and its two estimates             */
    double orth_err;      /* ||Q^T Q - I||_max of the stored basis                        */
    double ms_build;      /* wall time of rr_build_precond                                */
    double ms_solve;      /* wall time of the solve                                       */
    int32_t status;       /* rr_status of this solve / column                             */
    int32_t graph_fallbacks;  /* 1 if use_graph was asked for but the runtime invalidated
                                 the capture, so the iterations ran as eager launches of the
                                 same kernels (same results); 0 otherwise                 */
} rr_solve_info;

/* Optional device allocator (e.g. backed by PyTorch's caching allocator). */
typedef struct {
    void* ctx;
    void* (*alloc)(void* ctx, size_t bytes, void* stream);
    void (*free)(void* ctx, void* ptr, void* stream);
} rr_allocator;

typedef struct rr_precond rr_precond;   /* opaque; immutable after build */

/* Fill option structs with defaults (l = 0 means plain CG). */
void rr_build_opts_default(rr_build_opts* o);
void rr_solve_opts_default(rr_solve_opts* o);

/*
 * Build C-RandRAND preconditioners for the shifts mus[0..n_mu-1] (host array)
 * — Algorithm RandRAND_PCG steps 1-4 (Section 6.2):
 *   Omega (Section 2) -> Y = A Omega + mu Omega -> Q R = Y (Algorithm prec_chol_qr or
 *   chol_qr) -> G (remark after Algorithm RandRAND_PCG) -> T (eq. accurate_proj) -> tau.
 * With n_mu > 1 all shifts share the joint basis orth([Omega, A Omega]) and each
 * gets a 2l x l reduced QR (Section 5.1).
 * A: operator (device memory borrowed).  alloc: NULL = hipMalloc.  out: new handle.
 * Errors: RR_EINVAL (null pointers, n < 1, l < 0, l > n, n_mu < 1, a negative or
 * non-finite mu, d < 1 for kernels, unknown enum values), RR_ENOMEM, RR_ENOTSPD,
 * RR_EDEVICE.  On error *out is NULL.
 */
rr_status rr_build_precond(const rr_operator* A, const double* mus, int32_t n_mu,
                           const rr_build_opts* opts, const rr_allocator* alloc,
                           void* hip_stream, rr_precond** out);

/*
 * Solve (A + mus[mu_index] I) x = b by C-RandRAND PCG with restarts
 * (Algorithm RandRAND_PCG steps 5-11).  b, x: device float64 vectors of length n;
 * x holds x0 on entry and the solution on exit.  info may be NULL.
 * A handle built with l = 0 runs plain CG with identical kernels.
 * Errors: RR_EINVAL (also for NaN/Inf in b), RR_EBREAKDOWN, RR_ENOCONV (x holds the
 * last iterate), RR_EDEVICE.
 */
rr_status rr_solve(const rr_precond* P, int32_t mu_index, const double* b, double* x,
                   const rr_solve_opts* opts, rr_solve_info* info, void* hip_stream);

/*
 * Solve nrhs independent systems (A + mus[mu_index_per_col[j]] I) X_j = B_j at once:
 * one PCG recurrence per column (own alpha, beta, stopping), fused launches,
 * the kernel matvec of all columns as one MFMA product (Section 5.1 joint basis
 * when the handle holds several shifts; multi-RHS block of Section 7.2.2).
 * mu_index_per_col: host int array [nrhs].  B, X: device float64 n x nrhs with
 * leading dimensions ldb, ldx >= n; X holds X0 on entry.  infos: host [nrhs] or NULL.
 * Returns RR_OK if every column converged, else the first failing column's status.
 */
rr_status rr_solve_batch(const rr_precond* P, const int32_t* mu_index_per_col,
                         const double* B, int64_t ldb, int32_t nrhs, double* X, int64_t ldx,
                         const rr_solve_opts* opts, rr_solve_info* infos, void* hip_stream);

/* ---------------------------------------------------------------- serving --- */

/* One solve request.  All pointers are HOST memory owned by the caller and must
 * stay valid until deliver() is called for the request: pts (d x n float32 SoA),
 * B (n x nrhs float64), X (n x nrhs float64, written before deliver). */
typedef struct {
    int32_t kind;         /* RR_OP_RBF or RR_OP_MATERN32                              */
    int64_t n;
    int32_t d;
    const float* pts;
    double kconst, scale, mu;
    int64_t l;            /* sketch size for this request (0 = plain CG)               */
    int32_t nrhs;
    const double* B;
    double* X;
    uint64_t id;
    uint64_t seed;
    double t_arrival;     /* seconds on the clock passed to next()                     */
} rr_request;

/* next(): return 1 and fill *out if a request has arrived by `now` (seconds since
 * rr_serve started), 0 if none is due yet, -1 when the stream has ended. */
typedef int32_t (*rr_next_fn)(void* user, double now, rr_request* out);
/* deliver(): called once per request after X has been written on the host. */
typedef void (*rr_deliver_fn)(void* user, const rr_request* req, const rr_solve_info* info,
                              double t_done);

typedef struct {
    size_t hbm_budget;    /* device bytes the server may hold for requests               */
    int32_t max_slots;    /* requests resident at once                                  */
    int32_t graph_iters;  /* PCG iterations per replayed batch                          */
    rr_build_opts build;  /* l and seed are taken per request                           */
    rr_solve_opts solve;
    const rr_allocator* alloc;  /* device allocator for every request buffer and handle
                                   (NULL: the library's stream-ordered pool); its alloc and
                                   free are called from the server's worker threads       */
    int32_t grouped;      /* k in [1, 8]: the PCG batches of the resident requests run
                             together, each batch of every request waiting at that moment
                             in one replay of grouped persistent kernels over a device
                             work list, on k replay lanes (streams) at once (requests of
                             one shift whose kernel product runs on MFMA; others replay
                             their own graph); 0: every request replays its own graph.
                             Needs graph_iters in [1, 256].                            */
} rr_serve_config;

typedef struct {
    double p50_ms, p99_ms, mean_ms;  /* arrival -> delivered latency of OK requests        */
    double solves_per_s;             /* OK requests / wall time                          */
    int64_t served;                  /* requests delivered after running (ok + failed)   */
    int64_t rejected;                /* requests refused at admission (budget, invalid)  */
    size_t hbm_peak;
    int32_t max_active;
    int64_t ok, failed;              /* delivered with status RR_OK / with an error       */
    int64_t graph_fallbacks;         /* requests whose PCG graph capture was invalidated  */
    int64_t group_replays;           /* grouped replays run (grouped = 1)                 */
    double group_mean;               /* request batches per grouped replay                */
    int32_t group_max;               /* largest number of requests in one replay          */
    double group_busy_s;             /* replay time of the grouped engine (summed over lanes) */
    double group_wait_s;             /* summed over request batches: queued to completed  */
} rr_serve_stats;

/*
 * Continuous-batching server: a persistent loop polls next(), admits requests while
 * slots and the HBM budget allow (a request larger than the whole budget is
 * rejected with status RR_ENOMEM in its deliver()), builds each request's
 * preconditioner on the device (worker threads, one stream each, builds
 * overlapping), advances the resident requests' PCG iterations in batches of
 * graph_iters (grouped = 1: the batches of every request waiting at that moment in
 * one replay of grouped kernels; grouped = 0: a graph per request) and delivers
 * each result as soon as it converges.  Per-request arithmetic does not depend on
 * what else is resident (each request keeps its own work items and reduction
 * orders in the grouped kernels), so a result is the same alone and in the mix.  Returns when next() has returned -1 and every admitted request is
 * delivered.  Returns RR_OK only if every admitted request succeeded; otherwise
 * the first failed request's status (stats->failed counts them, rr_last_error()
 * names the first).  Errors: RR_EINVAL, RR_EDEVICE, or a request's status.
 */
rr_status rr_serve(const rr_serve_config* cfg, rr_next_fn next, rr_deliver_fn deliver,
                   void* user, rr_serve_stats* stats);

/* ------------------------------------------------------------ inspection --- */

/*
 * Copy a handle's state to host memory for checking (any pointer may be NULL):
 * Q (n x l, the per-shift basis Q_mu), R (l x l), G (l x l), T (l x l),
 * scalars[4] = {tau, ||E|| estimate, lam estimate, mu}.
 */
rr_status rr_precond_export(const rr_precond* P, int32_t mu_index, double* Q_host,
                            double* R_host, double* G_host, double* T_host,
                            double* scalars_host);

/* Write Omega (n x l, float64, host) as the handle drew it. */
rr_status rr_precond_export_omega(const rr_precond* P, double* Omega_host);

/*
 * The sketch step alone (Algorithm RandRAND_PCG step 1, q = 0): Y_out (device,
 * n x l float64) = A Omega + mu Omega, computed exactly as rr_build_precond does
 * with the same options (test matrix from opts->seed, precision opts->prec).
 */
rr_status rr_sketch_apply(const rr_operator* A, double mu, const rr_build_opts* opts,
                          double* Y_out, void* hip_stream);

/* Number of rows n, columns l and shifts of a handle (any pointer may be NULL). */
rr_status rr_precond_shape(const rr_precond* P, int64_t* n, int64_t* l, int32_t* n_mu);

/*
 * Form a kernel operator densely: A_out (device, n x n, leading dimension lda)
 * = scale * K evaluated in float64 (dtype 0), float32 (1) or bf16 (2, from float64).
 */
rr_status rr_kernel_to_dense(const rr_operator* kernel_op, void* A_out, int32_t dtype,
                             int64_t lda, void* hip_stream);

/*
 * y = (A + mu I) u with the operator in the given precision (rr_precision; FP32 uses
 * float32 entries with float64 accumulation).  u, y: device float64 [n].
 */
rr_status rr_apply_operator(const rr_operator* A, double mu, int32_t prec, const double* u,
                            double* y, void* hip_stream);

/*
 * Estimate of ||A_work - A||_2, the distance between the working operator of
 * precision prec (float32 entries / the float32 copy of a dense A) and the float64
 * operator: `iters` power-iteration steps on the difference (each step one product
 * with each operator), start vector from Gaussian stream `seed`.  It enters the
 * per-result error bound for the non-float64 modes: if ||b - A_work x|| <= tol ||b||
 * then ||b - A_mu x|| <= tol ||b|| + ||dA|| ||x|| and
 * ||x - x*|| <= (tol ||b|| + ||dA|| ||x||) / lambda_min(A_mu), lambda_min(A_mu) >= mu.
 * *out_host = 0 for prec = FP64.  Errors: RR_EINVAL, RR_ENOMEM, RR_EDEVICE.
 */
rr_status rr_operator_delta_norm(const rr_operator* A, int32_t prec, int32_t iters, uint64_t seed,
                                 double* out_host, void* hip_stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): y = (A + mu I) u exactly as
 * rr_apply_operator computes it (same kernels, bitwise the same result), with every
 * buffer beyond u and y (kernel point records, the float32 copy of a dense A in
 * FP32/MIXED, partial sums) taken from a static device scratch array of
 * rr_noalloc_scratch_bytes() = 64 MiB that each GPU holds until the process ends.
 * It calls no allocator and does not synchronise: the work is enqueued on
 * hip_stream and the caller synchronises.  All calls on one GPU share that array and
 * it keeps the last call's contents, so calls that overlap on one GPU (on different
 * streams or threads) race.  Limit: the layout must fit the scratch (kernel
 * operators up to about n = 32,768 at d <= 16; dense FP32/MIXED up to n of about
 * 4,000; dense FP64 any n).  Errors: RR_EINVAL (as rr_apply_operator, and for an
 * operator too large for the scratch, before any device work), RR_EDEVICE.
 */
rr_status rr_apply_operator_noalloc(const rr_operator* A, double mu, int32_t prec, const double* u,
                                    double* y, void* hip_stream);
/* Size in bytes of the per-GPU scratch array behind rr_apply_operator_noalloc. */
size_t rr_noalloc_scratch_bytes(void);

/*
 * Y = (A + mu I) U for nr columns at once (U, Y: device float64, n x nr,
 * column-major, leading dimension n; 1 <= nr <= 4096).  Kernel operators form each
 * entry once per group of up to 8 (FP32) or 2 (FP64) columns; in FP32 the entry
 * K_ij of a pair of row blocks is formed once and used for both y_i and y_j.
 * Same errors as rr_apply_operator.  This is the operator product of every PCG
 * step (Algorithm RandRAND_PCG) applied to a block of vectors.
 */
rr_status rr_apply_operator_block(const rr_operator* A, double mu, int32_t prec, const double* U,
                                  int32_t nr, double* Y, void* hip_stream);

/*
 * Fill out (device, rows x cols, float64, column-major) with the method's random
 * test matrix: kind 0 = Gaussian stream `seed` (element i + c*rows),
 * kind 1 = SRHT columns (D, sampled Hadamard rows) for n = rows, l = cols.
 */
rr_status rr_random_matrix(int32_t kind, uint64_t seed, int64_t rows, int64_t cols,
                           double* out, void* hip_stream);

/*
 * S = Theta Y with the second-level sketch of Algorithm prec_chol_qr (Section 4.2)
 * exactly as the build draws it for Omega stream `seed`: Theta is the sparse sign
 * embedding of stream seed+1 with 2k rows and min(8, 2k) entries +-1 per column,
 * one in each of that many row blocks (block t = rows [floor(2kt/z), floor(2k(t+1)/z))),
 * row and sign from one generator word per (column, block).  Y: device, n x k
 * float64 column-major (ld n), borrowed.  S: device, 2k x k float64 column-major
 * (ld 2k), written.  Each S[r, c] is summed over the columns of Theta in increasing
 * order.  Errors: RR_EINVAL (null pointers, n < 1, k < 1), RR_ENOMEM, RR_EDEVICE.
 * Asynchronous on the stream.
 */
rr_status rr_theta_apply(uint64_t seed, int64_t n, int64_t k, const double* Y, double* S,
                         void* hip_stream);

/*
 * The build's Cholesky step on a caller matrix (inspection of the factorisation
 * that Algorithms chol_qr / prec_chol_qr and the core R_Omega use): R (device,
 * k x k float64, column-major, ld k) = upper factor of sym(W) + alpha I with
 * R^T R = sym(W) + alpha I, where alpha = 0 if sym(W) factors, else the first of
 * 10^e max_i |W_ii| (e = -14 .. -1) that does.  W (device, k x k) is borrowed and
 * not modified.  alpha_host (may be NULL) receives alpha.  Errors: RR_EINVAL,
 * RR_ENOTSPD (the whole ladder failed), RR_EDEVICE.  Returns after the work.
 */
rr_status rr_cholesky_ladder(const double* W, int64_t k, double* R, double* alpha_host,
                             void* hip_stream);

/*
 * lambda_max of a symmetric positive semidefinite k x k float64 matrix G (device,
 * column-major, ld k, borrowed), exactly as the NYS tau rule computes
 * 1 / tau = lambda_max(G) (eq. nys_tau): Lanczos with full reorthogonalisation
 * from the Gaussian start vector of stream `seed`, stopped when the Ritz residual
 * bound is below 1e-14 lambda or after k steps.  out_host[3] = {lambda_max,
 * residual bound (|theta - lambda| <= it), Lanczos steps}.  1 <= k <= 1536.
 * Errors: RR_EINVAL, RR_EDEVICE.  Returns after the work.
 */
rr_status rr_lambda_max(const double* G, int64_t k, uint64_t seed, double* out_host, void* hip_stream);

/*
 * Kernel timing for measurement (off by default).  rr_profile_enable(1) clears the
 * counters and makes the launchers of the hot kernels bracket every launch with
 * HIP events on the launch stream; rr_profile_read(slot, &count, &total_ms)
 * returns the number of timed launches and their summed device time, leaving out
 * launches shorter than a tenth of the slot's median (iterations past convergence,
 * which the device-side stop flag turns into no-ops).  Slots:
 * 0 = float32 kernel matvec (first stage), 1 = float32 kernel-GEMM sketch,
 * 2 = float32 dense matvec, 3 = bf16 dense sketch, 4 = projections,
 * 5 = float64 kernel matrix-matrix product of the batched solve, 6 = float64 kernel
 * matvec (first stage; restart residuals of the float64 refinement), 7 = float64 dense
 * matvec; the serving loop's grouped iterations (run as plain launches while timing
 * is on): 8 = kernel products, 9 = their finish, 10 = projections, 11 = x, r and p
 * updates (one timed span per iteration and class).
 */
void rr_profile_enable(int32_t on);
rr_status rr_profile_read(int32_t slot, int64_t* count, double* total_ms);

void rr_precond_destroy(rr_precond* P);
const char* rr_status_string(rr_status s);
const char* rr_last_error(void);
/* Library version string. */
const char* rr_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RANDRAND_H */
