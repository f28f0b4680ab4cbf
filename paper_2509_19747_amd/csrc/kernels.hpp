// Host-side launchers for the gfx950 kernels.  Every launcher enqueues work on
// the given stream and returns immediately; argument shapes are validated by the
// caller (the C-ABI layer) before any launcher is reached.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rr {

enum Dtype { DT_F64 = 0, DT_F32 = 1, DT_BF16 = 2 };

// Per-solve device scalar state of one PCG recurrence.  Kernels read the
// scalars they need and return immediately once `stop` is non-zero, so a batch
// of iterations launched ahead of a host check becomes a no-op past the exit.
struct CgState {
    double alpha, beta, rho, rr, pw, target2;
    int32_t stop;       // 0 running, 1 reached target (restart/converged), 2 breakdown, 3 maxit
    int32_t iters;
    int32_t maxit;
    int32_t hist_cap;
    double* hist;       // device array of ||r||^2 per iteration (may be null)
};
enum { STOP_NONE = 0, STOP_TARGET = 1, STOP_BREAKDOWN = 2, STOP_MAXIT = 3 };

// Per-column state of the batched solve (one PCG recurrence per column).
struct BState {
    double alpha, beta, rho, rr, pw, target2;
    int32_t run;      // 1 while the column iterates in the current cycle
    int32_t code;     // STOP_* reason the column left the cycle
    int32_t iters;
    int32_t maxit;
};

// Device scalar state of one preconditioned MINRES recurrence (kernels_krylov.hip).
struct MrState {
    double beta, oldb, alfa, dbar, epsln, phibar, cs, sn, phi, gamma, delta, oldeps, rr, target2;
    int32_t stop, iters, maxit, k;   // k: steps in the current cycle
    int32_t hist_cap;
    double* hist;                    // ||res||^2 per iteration (may be null)
};

// ----------------------------------------------------------- random matrices
void launch_gauss_fill(void* out, int dtype, int64_t rows, int64_t cols, int64_t ld,
                       uint64_t seed, hipStream_t st);
void launch_srht_prepare(int64_t n, int64_t l, uint64_t seed, int64_t s, int32_t* perm_ws,
                         int32_t* rows_out, float* D_out, hipStream_t st);
void launch_srht_fill(void* out, int dtype, int64_t n, int64_t l, int64_t ld, const float* D,
                      const int32_t* rows, hipStream_t st);
// dbits[w] bit b = 1 when D[32 w + b] < 0 (i < n), words ceil(n / 32).
void launch_srht_dbits(int64_t n, const float* D, uint32_t* dbits, hipStream_t st);
// C (l x l, ldc) = Y^T Omega for the SRHT Omega of Hadamard size s (sampled rows, sign
// bits of D), Y n x l (float32 or float64, leading dimension ldy), by chunked
// Walsh-Hadamard transforms of the columns of D o Y; ws: srht_yt_omega_ws_doubles.
int64_t srht_yt_omega_ws_doubles(int64_t n, int64_t l, int64_t s);
void launch_srht_yt_omega(int ydt, int64_t n, int64_t l, int64_t s, const void* Y, int64_t ldy,
                          const uint32_t* dbits, const int32_t* rows, double* ws, double* C, int64_t ldc,
                          hipStream_t st);
// S (2k x k, column-major, lds) = Theta Y for the sparse sign embedding of stream
// `seed` (THETA_NNZ nonzeros per column, one per row block); Yt: Y row-major in
// float64 (Yt[i * ldy + c], i < n, c < k).
constexpr int THETA_NNZ = 8;
int theta_nnz(int64_t k);
void launch_theta_apply(int64_t n, int64_t k, uint64_t seed, const double* Yt, int64_t ldy, double* S,
                        int64_t lds, hipStream_t st);
// The same over rows [row0, row0 + rows) of Y (Yt holds those rows), adding into S
// when accumulate: S = Theta Y is then summed over row blocks.
void launch_theta_apply_rows(int64_t rows, int64_t row0, int64_t k, uint64_t seed, const double* Yt, int64_t ldy,
                             double* S, int64_t lds, bool accumulate, hipStream_t st);
// out[c + i * ldo] = (double) in[i + c * ldi] (i < rows, c < cols): a column-major
// matrix of dtype float64 / float32 written row-major in float64.
void launch_transpose_f64(int dtype, int64_t rows, int64_t cols, const void* in, int64_t ldi, double* out,
                          int64_t ldo, hipStream_t st);

// ------------------------------------------------------------------- GEMM
// C = alpha * op(A) op(B) + beta * C, float64 accumulation, op = transpose if tr*.
// A element type dta (F64/F32/BF16), B element type dtb (F64/F32).  Splits the K
// dimension over `splits` slices through workspace `ws` (splits*M*N doubles) and
// reduces them in a fixed order (deterministic).
size_t gemm_ws_doubles(int64_t M, int64_t N, int64_t K);
void launch_gemm(int dta, bool trA, int dtb, bool trB, int64_t M, int64_t N, int64_t K,
                 const void* A, int64_t lda, const void* B, int64_t ldb, double* C, int64_t ldc,
                 double alpha, double beta, double* ws, size_t ws_doubles, hipStream_t st);

// The same on float64 MFMA for float64/float32 operands with M, N >= 32 (returns
// false, doing nothing, otherwise); launch_gemm tries it first.
bool launch_gemm_mfma(int dta, bool trA, int dtb, bool trB, int64_t M, int64_t N, int64_t K,
                      const void* A, int64_t lda, const void* B, int64_t ldb, double* C,
                      int64_t ldc, double alpha, double beta, double* ws, size_t wsd,
                      hipStream_t st);
// C (M x M) = A^T A for float64 A (K x M, column-major): only the tiles on and
// above the diagonal are multiplied, then mirrored, so C is exactly symmetric.
// Returns false (nothing launched) when the MFMA path does not apply (M < 32 or K < 16).
bool launch_gemm_ata(int64_t M, int64_t K, const double* A, int64_t lda, double* C, int64_t ldc,
                     double* ws, size_t wsd, hipStream_t st);
// C = op(A) B (float64) for B upper triangular with zeros stored below its diagonal
// (column block j reads only rows k < its last column); false when the sizes are
// too small for the MFMA kernel.
bool launch_gemm_upper_b(bool trA, int64_t M, int64_t N, int64_t K, const double* A, int64_t lda,
                         const double* B, int64_t ldb, double* C, int64_t ldc, double* ws, size_t wsd,
                         hipStream_t st);

// ------------------------------------------------------ small dense helpers
void launch_symmetrize(double* A, int64_t l, int64_t lda, hipStream_t st);
void launch_add_diag(double* A, int64_t l, int64_t lda, double alpha, hipStream_t st);
void launch_add_diag_dev(double* A, int64_t l, int64_t lda, const double* alpha_dev, hipStream_t st);
void launch_two_minus(double* T, int64_t l, int64_t ldt, hipStream_t st);   // T = 2I - T
void launch_zero_lower(double* A, int64_t l, int64_t lda, hipStream_t st);
void launch_copy_mat(int dtype_src, const void* src, int64_t lds, int dtype_dst, void* dst,
                     int64_t ldd, int64_t rows, int64_t cols, hipStream_t st);
// C = a*A + b*B (all float64, same shape)
void launch_axpby_mat(double a, const double* A, int64_t lda, double b, const double* B,
                      int64_t ldb, double* C, int64_t ldc, int64_t rows, int64_t cols,
                      hipStream_t st);
void launch_scale_mat(double* A, int64_t lda, int64_t rows, int64_t cols, double s, hipStream_t st);
// max |A^T A - I| style check: out = max_ij |M_ij - delta_ij| (one double on device)
void launch_max_abs_minus_identity(const double* M, int64_t l, int64_t ldm, double* out, hipStream_t st);

// ------------------------------------------------- block Krylov solvers
// Right-hand sides per block of block MINRES / block CG (small matrices s x s,
// column-major, leading dimension s).
constexpr int BLOCK_MAX_S = 32;
// S = C^T C (S symmetrised first), C upper and C^{-1}; *flag = 1 (C, C^{-1} zero)
// when a pivot fails c_jj^2 > 1e-20 S_jj.
void launch_blk_chol(int s, const double* S, double* C, double* Ci, int32_t* flag, hipStream_t st);
// One block-QR step of block MINRES (see kernels_block.hip); G slots 2s x 2s.
void launch_bmr_qr(int s, int k, const double* M, const double* Cprev, const double* Cnew, const int32_t* brk,
                   const double* Gm2, const double* Gm1, double* Gk, double* phibar, double* R2, double* R1,
                   double* Rinv, double* phi, hipStream_t st);
// D_k = (Z - D1 R1 - D2 R2) Rinv, ADk likewise from U, Y += D_k phi, Rres -= ADk phi
// (D1/AD1, D2/AD2 may be null: zero blocks).  n x s blocks, leading dimension n.
void launch_bmr_rows(int64_t n, int s, const double* Z, const double* U, const double* D1, const double* D2,
                     const double* AD1, const double* AD2, const double* R1, const double* R2,
                     const double* Rinv, const double* phi, double* Dk, double* ADk, double* Y, double* Rres,
                     hipStream_t st);
// dst(:, j) = src(:, idx[j]);  dst(:, idx[j]) (+)= src(:, j)
void launch_blk_gather(int64_t n, int s, const double* src, int64_t lds, const int32_t* idx, double* dst,
                       hipStream_t st);
void launch_blk_scatter(int64_t n, int s, const double* src, const int32_t* idx, double* dst, int64_t ldd,
                        bool add, hipStream_t st);

// ------------------------------------------------------- factorizations
// In-place upper Cholesky of an l x l spd matrix (A = R^T R, R stored in the upper
// triangle, lower part zeroed).  *status (device int) is set non-zero on failure.
void launch_cholesky_upper(double* A, int64_t l, int64_t lda, int32_t* status, double* ws,
                           size_t ws_doubles, hipStream_t st);
// R factor (positive diagonal) of a Householder QR of S (m x k, m >= k), S is
// overwritten.  R: k x k, ldr.  ws: householder_ws_doubles(m, k) doubles (blocked
// panels with compact-WY GEMM updates; a smaller ws falls back to one reflector
// per launch, which needs none).
size_t householder_ws_doubles(int64_t m, int64_t k);
bool householder_blocked_ok(int64_t m, int64_t k);
void launch_householder_r(double* S, int64_t m, int64_t k, int64_t lds, double* R, int64_t ldr,
                          double* ws, size_t wsd, hipStream_t st);
// Householder QR with explicit Q (m x k, ldq) and R (k x k): used for the reduced
// 2l x l QR of the joint basis.  S is overwritten.  ws: >= max(m*k + k,
// householder_ws_doubles(m, k)) doubles.
void launch_householder_qr(double* S, int64_t m, int64_t k, int64_t lds, double* Q, int64_t ldq,
                           double* R, int64_t ldr, double* ws, size_t wsd, hipStream_t st);
void launch_householder_r_blocked(double* S, int64_t m, int64_t k, int64_t lds, double* R,
                                  int64_t ldr, double* ws, size_t wsd, hipStream_t st);
void launch_householder_qr_blocked(double* S, int64_t m, int64_t k, int64_t lds, double* Q,
                                   int64_t ldq, double* R, int64_t ldr, double* ws, size_t wsd,
                                   hipStream_t st);
// lambda_max of a symmetric psd k x k matrix G (k <= lanczos_max_dim()) by Lanczos
// with full reorthogonalisation in one workgroup; start vector from Gaussian stream
// `seed`.  out3 (device): {lambda_max, Ritz residual bound, steps}.  ws:
// lanczos_ws_doubles(k) doubles.
int lanczos_max_dim();
size_t lanczos_ws_doubles(int64_t k);
void launch_lanczos_lmax(const double* G, int64_t ldg, int64_t k, uint64_t seed, double* ws, double* out3,
                         hipStream_t st);
// X = R^{-1} for an upper-triangular l x l R.
void launch_tri_inv_upper(const double* R, int64_t l, int64_t ldr, double* X, int64_t ldx,
                          hipStream_t st);

// -------------------------------------------------------------- matvecs
// Dense symmetric y = A u + mu u (A float64 or float32, column-major), and
// per-block partials of u^T y in dot_part[nblocks].  Returns nblocks.
int dense_matvec_blocks(int64_t n);
void launch_dense_matvec(int dta, int64_t n, const void* A, int64_t lda, const double* u,
                         double mu, double* y, double* dot_part, const int32_t* stop,
                         hipStream_t st);

// Kernel operator y = scale*K u + mu u with K from points (float32 or float64
// evaluation, float64 accumulation), partials of u^T y.
struct KernelOp {
    int kind;            // 1 RBF, 2 Matern-3/2
    int64_t n;
    int d;
    const float* pts;    // d x n SoA
    const float* sqn;    // |x_i|^2 in float32 (length n), precomputed
    const float* xa;     // point records: n x dm floats, coordinates then zero padding
    int dm;              // record length kernel_record_len(d) in {4, 8, 16, 32}
    double kconst, scale;
    const double* xd = nullptr;   // float64 point records: n x dm doubles (coordinates, zeros)
    const double* hd = nullptr;   // -g |x_i|^2 / 2 in float64 (g of kernel_g64)
};
// float64 exponent scale g: an RBF entry is exp2(-g r^2 / 2) with g = 2 kconst log2(e);
// a Matern-3/2 entry uses g = 1 (the record product is then -r^2 / 2).
double kernel_g64(int kind, double kconst);
// xd[i*dm + k] = (double) pts[k*n + i] (k < d, zeros after), hd[i] = -g |x_i|^2 / 2.
void launch_point_records64(const float* pts, int64_t n, int d, int dm, double g, double* xd, double* hd,
                            hipStream_t st);
// Symmetric float64 kernel matvec (entries in float64: record products on the vector
// ALU, table-driven exp2), nr in {1, 2}; needs op.xd and op.hd.
size_t kernel_sym64_ws_doubles(int64_t n, int d, int nr);
// Float64 symmetric kernel matvec with the exponents' Gram products on float64 MFMA
// (the MFMA kernel's items and slots: kernel_mma_ok, kernel_mma_ws_doubles).
void launch_kernel_matvec_mma64(const KernelOp& op, const double* u, int nr, double mu, double* y,
                                double* dot_part, double* ws, const int32_t* stop, hipStream_t st);
void launch_kernel_matvec_sym64(const KernelOp& op, const double* u, int nr, double mu, double* y,
                                double* dot_part, double* ws, const int32_t* stop, hipStream_t st);
// Record length (floats) of a d-dimensional point: the next of 4, 8, 16, 32.
int kernel_record_len(int d);
// xa[i*dm + k] = pts[k*n + i] for k < d, 0 for d <= k < dm.
void launch_point_records(const float* pts, int64_t n, int d, int dm, float* xa, hipStream_t st);
int kernel_matvec_blocks(int64_t n);
// Workspace (doubles) of launch_kernel_matvec(_multi) for up to nr columns.
size_t kernel_matvec_ws_doubles(int64_t n, int d, int nr);
// The same for one precision only (fp64: the float64 operator on point records;
// otherwise the float32-class operator): what launch_kernel_matvec_multi uses then.
size_t kernel_matvec_ws_doubles_for(int64_t n, int d, int nr, bool fp64);
void launch_kernel_matvec(const KernelOp& op, bool fp64, const double* u, double mu, double* y,
                          double* dot_part, double* ws, const int32_t* stop, hipStream_t st);
// nr >= 1 right-hand sides at once: u, y are n x nr (leading dimension n);
// dot partials of column q at dot_part[q * kernel_matvec_blocks(n) + b].  Each
// kernel entry is evaluated once per group of up to 8 (float32) or 2 (float64)
// columns and applied to every column of the group.
// estimate: float32 sums allowed (power iterations of the tau estimates).
void launch_kernel_matvec_multi(const KernelOp& op, bool fp64, const double* u, int nr, double mu,
                                double* y, double* dot_part, double* ws, const int32_t* stop,
                                hipStream_t st, bool estimate = false);
// Symmetric kernel matvec with the pair terms on bf16 MFMA (three-piece split,
// float32-class entries, float64 sums), nr in {1, 2} (kernels_ksym_mma.hip).
bool kernel_mma_ok(int64_t n, int d);
size_t kernel_mma_ws_doubles(int64_t n, int nr);
// Work-item plan of the MFMA kernel product (row blocks nb, column blocks per run m,
// column ranges S, items per column block of the launch).
struct KmmaPlanInfo {
    int nb, m, S;
    int64_t items;
};
KmmaPlanInfo kernel_mma_plan_info(int64_t n);
// Columns one MFMA kernel product may carry with float64 sums (4 for records of up to
// 16 terms, else 2); each column's arithmetic is the same whatever the width.
int kernel_mma_max_cols(int dm);
// a32: float32 products and partial sums (estimate grade, power iterations).
void launch_kernel_matvec_mma(const KernelOp& op, const double* u, int nr, double mu, double* y,
                              double* dot_part, double* ws, const int32_t* stop, hipStream_t st,
                              bool a32 = false);
// Symmetric float32 matvec, nr in {1, 2, 4, 8} (kernels_ksym.hip).
size_t kernel_sym_ws_doubles(int64_t n, int d, int nr);
// a32: float32 products and sums (estimate grade, nr <= 2), for power iterations.
void launch_kernel_matvec_sym(const KernelOp& op, const double* u, int nr, double mu, double* y,
                              double* dot_part, double* ws, const int32_t* stop, hipStream_t st,
                              bool a32 = false);
void launch_sqnorms(const float* pts, int64_t n, int d, float* sqn, hipStream_t st);
// Dense formation A_out = scale*K in float64 (dtype 0) / float32 (1) / bf16 (2).
void launch_kernel_to_dense(const KernelOp& op, void* out, int dtype, int64_t lda, hipStream_t st);
// Kernel-GEMM on BF16 MFMA with hi/lo-split kernel entries; B (n x m, ldb a
// multiple of 8 and >= round8(n), rows [n, round8(n)) zero) holds bf16 values
// (the test matrix, exact in bf16); Y float32.
// srht_rows / srht_dbits (both or neither): Omega is the SRHT with these sampled
// Hadamard rows (m) and sign bits of D (bit i%32 of word i/32, set for D_i = -1);
// its B fragments are then generated in registers instead of read from Bbf16
// (Bbf16 still supplies the mu * Omega term).
void launch_kernel_gemm_bf16x2(const KernelOp& op, const void* Bbf16, int64_t ldb, int64_t m,
                               double mu, float* Y, int64_t ldy, float* ws, hipStream_t st,
                               const int32_t* srht_rows = nullptr, const uint32_t* srht_dbits = nullptr);
// Workspace (floats) of launch_kernel_gemm_bf16x2 for n points and m columns (0: none).
size_t kernel_sketch_ws_floats(int64_t n, int64_t m);
// Same in float64 on the vector ALU (small problems / float64 mode).
void launch_kernel_gemm_f64(const KernelOp& op, const double* B, int64_t ldb, int64_t m,
                            double mu, double* Y, int64_t ldy, hipStream_t st);
// Dense bf16 GEMM on MFMA: Y(float32, n x m) = A(bf16, n x n) * B(bf16, n x m) + mu*Bf
void launch_dense_gemm_bf16(int64_t n, int64_t m, const void* A, int64_t lda, const void* B,
                            int64_t ldb, double mu, float* Y, int64_t ldy, hipStream_t st);

// ------------------------------------------------------------ batched solve
// W = scale*K P + diag(mucol) P for m columns on float64 MFMA; entries in float32
// (the same values as the single-vector matvec) or, with f64_entries, float64.
void launch_kernel_matmat_f64(const KernelOp& op, bool f64_entries, const double* mucol,
                              const double* P, int64_t ldp, int64_t m, double* W, int64_t ldw,
                              hipStream_t st);
void launch_add_shift_cols(int64_t n, int64_t m, const double* mucol, const double* P, int64_t ldp,
                           double* W, int64_t ldw, hipStream_t st);
int coldot_chunks(int64_t n);
void launch_coldot(int64_t n, int64_t m, const double* A, int64_t lda, const double* B, int64_t ldb,
                   double* part, hipStream_t st);
// Per-column block partials: partial c of column j at p[c * cs + j * js], c < nch.
struct ColParts {
    const double* p;
    int nch;
    int64_t cs, js;
};
void launch_bstate_start(ColParts part, int64_t m, BState* st, const int32_t* start,
                         const double* target2, int32_t maxit, hipStream_t s);
// Blocks per column of the fused x/r and p updates (rr_part of the x/r update holds
// bxr_blocks(n) partials per column, at rr_part[j * bxr_blocks(n) + block]).
int bxr_blocks(int64_t n);
// The x/r update with alpha folded in (alpha_j = rho_j / sum of pw's partials, formed
// by every block) and the p update with beta folded in (beta_j = sum of rz's partials
// / rho_j); the last block of each column records the scalars and stop tests and
// resets its counter: cnt holds m int32 that are zero between launches.  More than 32
// columns: the updates write their partials and a second launch (one block per column)
// records the scalars from the same sums (no per-block device-scope fence).
void launch_bxr_fused(int64_t n, int64_t m, double* X, int64_t ldx, double* R, const double* P,
                      const double* W, BState* st, ColParts pw, double* rr_part, int32_t* cnt, hipStream_t s);
void launch_bp_fused(int64_t n, int64_t m, const double* Z, double* P, BState* st, ColParts rz, int32_t* cnt,
                     hipStream_t s);
// dst[:, di[c]] = src[:, si[c]] for c < ncols (a null index list is the identity).
void launch_copy_cols(int64_t n, int64_t ncols, const int32_t* si, const double* src, int64_t lds,
                      const int32_t* di, double* dst, int64_t ldd, hipStream_t s);
void launch_copy_flagged(int64_t n, int64_t m, const double* src, int64_t lds, double* dst,
                         int64_t ldd, const int32_t* flag, hipStream_t s);
void launch_bresid(int64_t n, int64_t m, const double* B, int64_t ldb, const double* T, double* Rt,
                   hipStream_t s);
void launch_select_cols(int64_t k, int64_t m, const double* Dall, const int32_t* mu_idx, double* D,
                        hipStream_t s);

// ------------------------------------------------------ projections
// c_part[chunk * k + j] = sum_{i in chunk} Q[i, j] r[i]; returns number of chunks.
int gemv_t_chunks(int64_t n, int64_t k);
int64_t gemv_t_rows_per_chunk_of(int64_t n, int64_t k);   // rows of each of those chunks
void launch_gemv_t(int64_t n, int64_t k, const double* Q, int64_t ldq, const double* r,
                   double* c_part, int nchunks, const int32_t* stop, hipStream_t st);
// nr = 1 or 2 vectors (R: n x nr, leading dimension ldr); vector q's partials at
// c_part + q * nchunks * k.
void launch_gemv_t_multi(int nr, int64_t n, int64_t k, const double* Q, int64_t ldq, const double* R,
                         int64_t ldr, double* c_part, int nchunks, const int32_t* stop, hipStream_t st);
// d = Kc * c with c = sum over chunks of c_part (Kc symmetric k x k).
void launch_core_apply(int64_t k, const double* Kc, int64_t ldk, const double* c_part,
                       int nchunks, double* d, const int32_t* stop, hipStream_t st);
// The same for a pair of columns: d[0:k] from K0 and c_part[0 : nchunks*k],
// d[k:2k] from K1 and c_part[nchunks*k : 2*nchunks*k] (one launch).
void launch_core_apply_pair(int64_t k, const double* K0, const double* K1, int64_t ldk,
                            const double* c_part, int nchunks, double* d, const int32_t* stop,
                            hipStream_t st);
// Pair plus a third product on the second column: d[2k:3k) = K2 c_1, and c_1 itself
// into c1_out (k doubles).
// ncols columns with one core: d[q k : (q+1) k) = Kc c_q, c_q from column q of c_part.
void launch_core_apply_cols(int64_t k, const double* Kc, int64_t ldk, const double* c_part, int nchunks,
                            int ncols, double* d, hipStream_t st);
void launch_core_apply_triple(int64_t k, const double* K0, const double* K1, const double* K2, int64_t ldk,
                              const double* c_part, int nchunks, double* d, double* c1_out, hipStream_t st);
// z = rcoef*r + Q d, and per-block partials of r^T z.
int qd_blocks(int64_t n);
void launch_qd(int64_t n, int64_t k, const double* Q, int64_t ldq, const double* d,
               const double* r, double rcoef, double* z, double* rz_part, const int32_t* stop,
               hipStream_t st);
// Z[:, q] = rc_q R[:, q] + Q D[:, q] for nr = 1 or 2 (D: k x nr, leading dimension k;
// R, Z: leading dimension ldr); partials of column q at rz_part + q * qd_blocks(n).
void launch_qd_multi(int nr, int64_t n, int64_t k, const double* Q, int64_t ldq, const double* D,
                     const double* R, int64_t ldr, double rc0, double rc1, double* Z, double* rz_part,
                     const int32_t* stop, hipStream_t st);
// v = v / sqrt(sum(part)); lam_out[0] = sqrt(sum(part))  (power-iteration step)
// v0 = src0 / ||src0|| (||src0||^2 from count0 partials) and v1 = src1 / sqrt(a^T b) (k
// entries) in one launch; the norms go to lam0 and lam1.
void launch_normalize_pair(int64_t n, double* v0, const double* src0, const double* part0, int count0,
                           double* lam0, double* v1, const double* src1, const double* a, const double* b,
                           int64_t k, double* lam1, hipStream_t st);
void launch_normalize(int64_t n, double* v, const double* src, const double* part, int count,
                      double* lam_out, hipStream_t st);

// ----------------------------------------------------------- CG updates
int vec_blocks(int64_t n);
// x += alpha p; r -= alpha w; partial ||r||^2
void launch_xr_update(int64_t n, double* x, double* r, const double* p, const double* w,
                      CgState* s, double* rr_part, hipStream_t st);
// p = z + beta p
void launch_p_update(int64_t n, const double* z, double* p, const CgState* s, hipStream_t st);
// r = b - w, partial ||r||^2
void launch_residual(int64_t n, const double* b, const double* w, double* r, double* rr_part,
                     hipStream_t st);
void launch_copy_vec(int64_t n, const double* src, double* dst, hipStream_t st);
void launch_dot_part(int64_t n, const double* a, const double* b, double* part, hipStream_t st);
// single-block scalar steps
void launch_scal_alpha(const double* part, int count, CgState* s, hipStream_t st);
void launch_scal_rr(const double* part, int count, CgState* s, hipStream_t st);
void launch_scal_beta(const double* part, int count, CgState* s, hipStream_t st);
void launch_scal_set(const double* part, int count, double* out, hipStream_t st);  // out = sum
void launch_state_init(CgState* s, const double* rz_part, int rz_count, double target2,
                       int32_t maxit, int32_t iters, double* hist, int32_t hist_cap,
                       hipStream_t st);
// Finite check of a vector: *flag = 1 if any entry is NaN/Inf.
// *flag = 1 if v holds a NaN or Inf; *nonzero = 1 (when given) if any entry is not 0.
void launch_nonfinite(int64_t n, const double* v, int32_t* flag, hipStream_t st, int32_t* nonzero = nullptr);

// ------------------------------------------- basis-less kernel blocks
// Signed column sampling: sgn[c] = D[idx[c]], pos[i] = c if i = idx[c] else -1.
void launch_colsample_prep(int64_t n, int64_t l, const float* D, const int32_t* idx, double* sgn, int32_t* pos,
                           hipStream_t st);
// dense Omega (ld x l, dtype) with Omega[idx[c], c] = sgn[c]
void launch_colsample_fill(int dtype, int64_t n, int64_t l, int64_t ld, const int32_t* idx, const double* sgn,
                           void* out, hipStream_t st);
// out[c] = sgn_c (scale K(x_idx_c, :) v + mu v_idx_c)  (= (A_mu Omega)^T v)
void launch_kblock_rows(const KernelOp& op, bool f64, const int32_t* idx, const double* sgn, int64_t l,
                        const double* v, double mu, double* out, const int32_t* stop, hipStream_t st);
// z = rcoef r + (A_mu Omega) d, with kblock_cols_blocks(n) partials of r^T z (rz_part may be null;
// r may be null for z = (A_mu Omega) d)
int kblock_cols_blocks(int64_t n);
void launch_kblock_cols(const KernelOp& op, bool f64, const int32_t* idx, const double* sgn, const int32_t* pos,
                        int64_t l, const double* d, double mu, const double* r, double rcoef, double* z,
                        double* rz_part, const int32_t* stop, hipStream_t st);
// rows of A_mu Omega, row-major (out[i * ldo + c]): rows r0 .. r0 + rows - 1, or the rows
// rowidx[i] scaled by rowsgn[i] (Omega^T A_mu Omega for rowidx = idx, rowsgn = sgn)
void launch_kblock_y(const KernelOp& op, bool f64, const int32_t* idx, const double* sgn, int64_t l, double mu,
                     int64_t r0, int64_t rows, const int32_t* rowidx, const double* rowsgn, double* out,
                     int64_t ldo, hipStream_t st);

// ------------------------------------------------ general Krylov engine
void launch_mr_init(const double* part, int count, MrState* s, double target2, int32_t maxit, int32_t iters,
                    double* hist, int32_t hist_cap, hipStream_t st);
void launch_mr_v(int64_t n, const double* z, double* v, const MrState* s, hipStream_t st);
void launch_mr_t(int64_t n, const double* av, const double* r1, const double* v, double* t, const MrState* s,
                 double* part, hipStream_t st);
void launch_mr_alfa(const double* part, int count, MrState* s, hipStream_t st);
void launch_mr_shift(int64_t n, const double* t, double* r1, double* r2, const MrState* s, hipStream_t st);
void launch_mr_rot(const double* part, int count, MrState* s, hipStream_t st);
void launch_mr_update(int64_t n, const double* v, const double* av, double* w, double* w2, double* aw,
                      double* aw2, double* y, double* res, const MrState* s, double* part, hipStream_t st);
void launch_mr_rr(const double* part, int count, MrState* s, hipStream_t st);
// dst = src with vec_blocks(n) partials of ||src||^2
void launch_copy_dot(int64_t n, const double* src, double* dst, double* part, const int32_t* stop, hipStream_t st);
// vec_blocks(n) partials of a^T b (no-op once *stop is set)
void launch_dot_part_stop(int64_t n, const double* a, const double* b, double* part, const int32_t* stop,
                          hipStream_t st);
// d = K1 c1 + K2 c2 (symmetric k x k cores, c's as chunk partials; k <= 4096)
void launch_core_apply2(int64_t k, const double* K1, const double* K2, int64_t ldk, const double* c1_part,
                        const double* c2_part, int nchunks, double* d, const int32_t* stop, hipStream_t st);

}  // namespace rr
