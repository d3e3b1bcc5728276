/*
 * nyspcg.h -- C ABI of the MI355X (gfx950) randomized Nystrom PCG library.
 *
 * Solves the regularised psd system (A + mu I) x = b of Section 1.1 of
 * Frangella, Tropp & Udell, "Randomized Nystrom Preconditioning", with the
 * randomized Nystrom approximation (Section 2.2, algorithm "Randomized Nystrom
 * Approximation"), the Nystrom preconditioner (Section 5.1.2, eq. (NysPre)) and
 * left-preconditioned CG (Section 5.2, algorithm "Nystrom PCG").
 *
 * Conventions shared by every entry point
 *   - Every array argument is a DEVICE pointer owned by the caller, unless the
 *     comment says "host".  Matrices are row-major with an explicit leading
 *     dimension counted in elements.  The library never allocates or frees
 *     device memory: each call takes a workspace (ws, ws_bytes) sized by
 *     nys_workspace_size(); a too-small workspace returns NYS_ERR_WORKSPACE.
 *     Its only allocation is 256 bytes of pinned host memory per calling host
 *     thread, made once and kept until the process ends, into which the
 *     device writes the flags that nys_factor and nys_pcg_solve* poll.
 *   - `stream` is the caller's hipStream_t (NULL = default stream).  Work is
 *     enqueued on it in order.  nys_pcg_solve* synchronise that stream to
 *     read convergence and failure flags.  nys_sketch and nys_factor read
 *     theirs from pinned host memory as the device writes them and return
 *     once their last kernels are enqueued: their outputs are complete when
 *     the stream reaches that point (they synchronise the stream only when
 *     the pinned memory could not be had, and nys_factor also with
 *     NYS_VERBOSE set).  Calls documented as synchronising say so; the
 *     others do not.
 *     nys_pcg_solve with opts.device_info = 1 neither synchronises nor reads
 *     device memory on the host, so it can be captured into a HIP graph.
 *   - Inputs are never written, except the buffers documented as in/out.
 *   - Errors are returned as nys_status codes; no C++ exception crosses the
 *     ABI.  nys_last_error() returns a message for the last non-OK status of
 *     the calling thread.
 *   - Calls that share a workspace must not overlap on different streams.
 */
#ifndef NYSPCG_H
#define NYSPCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NYS_OK = 0,
  NYS_NOT_CONVERGED = 1,   /* iteration cap reached; X holds the last iterate  */
  NYS_ERR_ARG = -1,        /* invalid argument (shape, mu < 0, tol <= 0, ...)  */
  NYS_ERR_NOT_PSD = -2,    /* Cholesky of Omega^T Y_nu failed after retries    */
  NYS_ERR_BREAKDOWN = -3,  /* p^T (A + mu I) p <= 0: system not positive definite */
  NYS_ERR_DEVICE = -4,     /* HIP runtime error, or a device-side time-out     */
  NYS_ERR_WORKSPACE = -5   /* workspace smaller than nys_workspace_size()      */
} nys_status;

typedef enum { NYS_F64 = 0, NYS_F32 = 1 } nys_dtype;

/* Arithmetic used by the sketch, the matvec and the CG vectors.  Every mode
 * returns x in float64 and is judged by the float64 true relative residual. */
typedef enum {
  NYS_PREC_FP64 = 0,            /* all float64                                   */
  NYS_PREC_FP32 = 1,            /* float32 vectors/matvec, no refinement (tol >= 1e-5) */
  NYS_PREC_FP32_REFINE64 = 2,   /* float32 inner PCG; float64 residual b-(A+mu I)x
                                   and update x += d in an outer refinement loop   */
  NYS_PREC_BF16X3_REFINE64 = 3  /* as 2, with RBF Gram tiles split into three
                                   bf16 products on MFMA (float32 accumulation)    */
} nys_precision;

/* The operator A (Section 1.1: A is reached only through products). */
typedef enum {
  NYS_OP_DENSE = 0,   /* explicit symmetric A: data is n x n                   */
  NYS_OP_XTX = 1,     /* ridge normal equations A = scale X^T X (Section 1.3,
                         eq. (RidgeRegression)): data X is rows x n            */
  NYS_OP_RBF = 2,     /* Gaussian kernel K_ij = exp(-|x_i-x_j|^2/(2 sigma^2))
                         (kernel ridge regression, Section 6.5): data is n x d,
                         one point per row                                     */
  NYS_OP_CALLBACK = 3 /* A given only as a product routine of the caller
                         (Section 1.1: the method needs nothing but products
                         with A): `apply` below; data, rows, cols, ld unused   */
} nys_op_kind;

/* Product routine of an NYS_OP_CALLBACK operator: W = A V for k columns,
 * V and W row-major n x k blocks (device pointers, leading dimensions ldv and
 * ldw in elements) of type `dtype` (NYS_F64 or NYS_F32), enqueued on `stream`
 * (the hipStream_t of the library call; the routine must not synchronise it
 * when the call is being captured into a graph).  The library applies scale
 * and the shift itself: it uses scale * W + mu V.  The routine returns 0 on
 * success; any other value makes the library call return NYS_ERR_DEVICE.  A
 * routine that does not support NYS_F32 should return nonzero for it: the
 * float32 inner solves of the reduced-precision modes call it with NYS_F32,
 * everything else with NYS_F64.  It may be called from inside any library
 * call that takes the operator, on the calling host thread. */
typedef int32_t (*nys_apply_fn)(void* ctx, int64_t k, int32_t dtype, const void* V, int64_t ldv, void* W,
                                int64_t ldw, void* stream);

typedef struct {
  int32_t kind;      /* nys_op_kind                                           */
  int32_t dtype;     /* storage type of `data`: NYS_F64 or NYS_F32            */
  int64_t n;         /* system dimension                                      */
  const void* data;  /* device, row-major, see nys_op_kind                    */
  int64_t rows;      /* rows of data (DENSE: n; XTX: m; RBF: n)               */
  int64_t cols;      /* cols of data (DENSE: n; XTX: n; RBF: d)               */
  int64_t ld;        /* leading dimension of data, >= cols                    */
  double sigma;      /* RBF bandwidth (> 0); ignored otherwise                */
  double scale;      /* A = scale * (base operator); must be > 0              */
  nys_apply_fn apply;/* NYS_OP_CALLBACK: the product routine; NULL otherwise  */
  void* ctx;         /* NYS_OP_CALLBACK: passed to apply unchanged            */
  const double* weights; /* NYS_OP_XTX only, nullable: device float64 row
                         weights d (rows entries, each finite and >= 0, not
                         checked by the products), A = scale X^T D X with
                         D = diag(d) -- the data term of a generalised linear
                         model's Hessian (Section 6.3, approximate
                         cross-validation).  Applied in the arithmetic of each
                         product (float64 in the float64 products and
                         residuals, rounded to float32 in the float32 ones).
                         Not available to nys_sketch_columns or the gX output
                         of nys_pcg_backward (NYS_ERR_ARG); must be NULL for
                         the other kinds.                                     */
} nys_operator;

/* Factored Nystrom approximation A_hat = U diag(lam) U^T (output of the
 * randomized Nystrom approximation).  It does not depend on mu, so one
 * preconditioner serves a whole mu grid and the adjoint solve. */
typedef struct {
  int64_t n, ell;
  void* U;           /* device, n x ell row-major (ldu), orthonormal columns  */
  int64_t ldu;
  int32_t dtype;     /* storage of U: NYS_F64 or NYS_F32 (float32 halves the
                        apply traffic of the mixed-precision modes)           */
  int32_t pad_;
  double* lam;       /* device, ell float64, descending, >= 0                 */
  double nu;         /* host: shift used by the factorisation (output)        */
} nys_precond;

typedef struct {
  double tol;          /* stop when ||b - (A+mu I)x||_2 <= tol ||b||_2          */
  int32_t maxit;       /* iteration cap per (inner) solve; 0 selects 500        */
  int32_t prec;        /* nys_precision                                         */
  int32_t max_refine;  /* refinement modes: cap on outer steps; 0 selects 10    */
  int32_t check_every; /* iterations between host polls of the convergence flags;
                          <= 0: chosen from the measured iteration time (1 .. 32) */
  double inner_tol;    /* refinement modes: relative reduction asked of each
                          inner solve; 0 selects 1e-4                          */
  int32_t device_info; /* 0: the call waits for the device and fills the host
                          arrays of nys_solve_info.  1: nothing is read back and
                          the stream is never synchronised (graph capture):
                          the info arrays are DEVICE arrays written by the last
                          kernels of the call, and the iteration counts are
                          fixed in advance (see nys_pcg_solve)                  */
  int32_t pad_;
} nys_solve_opts;

typedef struct {
  int32_t* iters;      /* host (device when opts.device_info = 1), one per
                          column: PCG iterations (all inner)                    */
  double* relres;      /* host (device when opts.device_info = 1), one per
                          column: final relative residual (float64 true
                          residual in refinement modes and with device_info,
                          recursive otherwise)                                  */
  int32_t* status;     /* host (device when opts.device_info = 1), one per
                          column: nys_status                                    */
  int32_t refine_steps;/* output: outer refinement steps taken                  */
  int32_t total_iters; /* output: iteration sweeps executed (max over columns)  */
} nys_solve_info;

/* Bytes of workspace that suffice for every call below on operator A with
 * sketch size ell, ncols simultaneous right-hand sides and precision prec. */
size_t nys_workspace_size(const nys_operator* A, int64_t ell, int64_t ncols, int32_t prec);

/* Standard normal n x ell test matrix (Section 2.2, algorithm "Randomized
 * Nystrom Approximation", first step) from a counter-based generator:
 * Philox4x32-10 (Salmon et al., SC 2011) with key = seed, counter = entry/2,
 * and the Box-Muller transform of two 53-bit uniforms.  Entry (i, j) depends
 * only on (seed, i*ell + j).  out: device float64, n x ell, leading dim ld. */
nys_status nys_gaussian(uint64_t seed, int64_t n, int64_t ell, double* out, int64_t ld,
                        void* stream);

/* Sketch (algorithm "Randomized Nystrom Approximation", steps 1-3):
 * Omega = orth(Omega0) (thin QR factor Q by CholeskyQR: one pass for a drawn
 * Gaussian with n >= 3 ell, two passes otherwise) and Y = A Omega.  omega0: device float64 n x ell (ld = ell) or NULL to draw it
 * with nys_gaussian(seed).  Omega_out, Y_out: device float64 n x ell (ld = ell).
 * prec selects the arithmetic of Y = A Omega (FP64, FP32 or BF16X3 tiles);
 * Omega is float64 in every mode.  Errors: NYS_ERR_ARG (1 <= ell <= min(n, 2048)
 * violated, bad operator), NYS_ERR_NOT_PSD (Omega0 rank deficient).
 * Waits for the CholeskyQR pivot flags, then returns with Y = A Omega still
 * enqueued on the stream (see the stream note at the top). */
nys_status nys_sketch(const nys_operator* A, int64_t ell, uint64_t seed, const double* omega0,
                      double* Omega_out, double* Y_out, int32_t prec, void* ws, size_t ws_bytes,
                      void* stream);

/* Factor (same algorithm, steps 4-9): nu = eps(||Y||_F) (spacing of the
 * float64 number), Y_nu = Y + nu Omega, C = chol(Omega^T Y_nu), B = Y_nu C^{-1},
 * [U, Sigma] = thin SVD of B, lam = max(0, Sigma^2 - nu), descending.
 * prec: arithmetic of the sketch that produced Y.  For a reduced-precision
 * sketch (relative error up to u = 2^-20 for float32 tiles, 2^-15 for bf16x3
 * tiles) the shift is raised to max(eps(||Y||_F), u ||Y||_F) so that the core
 * matrix stays positive definite; the shift is removed again from lam.
 * Y is overwritten.  P: P->n, P->ell, P->U, P->ldu, P->dtype, P->lam set by
 * the caller (1 <= P->ell <= min(n, 2048), else NYS_ERR_ARG; the same bound
 * holds for every call that takes a preconditioner); P->nu is written (host).
 * A failed Cholesky is retried with nu <- 10 nu up to three times, then
 * NYS_ERR_NOT_PSD.  Waits for the Cholesky's pivot flag and the eigensolver's
 * sweep flags, then returns with the last kernels (U, lam) still enqueued on
 * the stream (see the stream note at the top). */
nys_status nys_factor(const double* Omega, double* Y, nys_precond* P, int32_t prec, void* ws,
                      size_t ws_bytes, void* stream);

/* Z = (A + mu I) V for k columns (row-major n x k).  prec NYS_PREC_FP64
 * computes in float64 (float32 operator data is promoted exactly; V, Z
 * float64).  Other modes compute in float32 with float32 V, Z: X^T X and
 * dense operators for one contiguous vector; RBF operators for any k, with
 * the Gram tiles in float32 (NYS_PREC_FP32, NYS_PREC_FP32_REFINE64) or split
 * into three bf16 products (NYS_PREC_BF16X3_REFINE64), d <= 32.  Used for
 * right-hand sides, true residuals and tests of the product kernels. */
nys_status nys_op_apply(const nys_operator* A, double mu, const void* V, int64_t k, int64_t ldv,
                        void* Z, int64_t ldz, int32_t prec, void* ws, size_t ws_bytes, void* stream);

/* Z = P^{-1} R with eq. (NysPre):
 *   P^{-1} = (lam_l + mu) U (Lambda + mu I)^{-1} U^T + (I - U U^T),
 * for k columns (row-major n x k), all float64.  Requires lam_l + mu > 0. */
nys_status nys_precond_apply(const nys_precond* P, double mu, const double* R, int64_t k,
                             int64_t ldr, double* Z, int64_t ldz, void* ws, size_t ws_bytes,
                             void* stream);

/* Nystrom PCG (Section 5.2, algorithm "Nystrom PCG") for nmu*nrhs independent
 * systems that share A and P: column c = m*nrhs + r solves
 * (A + mu[m] I) x = B[:, r] (Section 5.2.3, Block Nystrom PCG, read as independent
 * columns; the mu grid reuses one preconditioner, which does not depend on mu).
 * mu: host array of nmu values >= 0.  B: device float64 n x nrhs (ldb).
 * X: device float64 n x (nmu*nrhs) (ldx); on entry the initial guesses, on exit
 * the solutions.  info: host arrays of nmu*nrhs entries (may be NULL).
 * Returns NYS_OK when every column met tol, NYS_NOT_CONVERGED when some hit
 * the cap, NYS_ERR_BREAKDOWN when p^T v <= 0 occurred.
 *
 * Device-info form (o->device_info = 1), for callers that capture the call
 * into a HIP graph or cannot wait for the device: the host only checks the
 * arguments and enqueues kernels (no synchronisation, no device-to-host copy,
 * no memset node).  Every mu must be > 0.  No column is dropped early and
 * nothing is decided on the host: the float64 and float32 modes run exactly
 * maxit iterations, the refinement modes exactly max_refine outer steps of
 * maxit inner iterations each; a column that has met its tolerance (or broken
 * down) is frozen by device flags, so the remaining iterations change nothing
 * for it.  In the float64 mode no correction solve follows.  At the end
 * info->iters / relres / status (device arrays of nmu*nrhs entries; may be
 * NULL pointers individually) receive the iterations each column ran, its
 * float64 true relative residual, and NYS_OK (true residual <= tol),
 * NYS_NOT_CONVERGED or NYS_ERR_BREAKDOWN; info->refine_steps and
 * info->total_iters (host fields) receive the fixed counts.  The return
 * value only reports argument errors (NYS_OK once everything is enqueued). */
nys_status nys_pcg_solve(const nys_operator* A, const nys_precond* P, const double* mu, int64_t nmu,
                         const double* B, int64_t nrhs, int64_t ldb, double* X, int64_t ldx,
                         const nys_solve_opts* o, nys_solve_info* info, void* ws, size_t ws_bytes,
                         void* stream);

/* Allocation-free form of nys_pcg_solve, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments and results as nys_pcg_solve in its
 * device-info form (o->device_info must be 1, else NYS_ERR_ARG), without the
 * workspace: the call uses a static device array of
 * nys_noalloc_scratch_bytes() bytes (64 MiB) that the library holds on each
 * GPU it runs on until the process ends.  A solve whose workspace
 * (nys_workspace_size for the same operator, rank and column count) exceeds
 * that returns NYS_ERR_WORKSPACE before anything is enqueued.  The call makes
 * no device or pinned-host allocation, no hipFree and no memset; the first
 * call on a device looks the array's address up once (before capture, make
 * one call on each device outside it).  Every call on one GPU shares that
 * GPU's array, whatever its stream: calls that overlap in time on one GPU
 * race and give undefined results.  The array keeps the last call's contents;
 * the call initialises everything it reads. */
nys_status nys_pcg_solve_noalloc(const nys_operator* A, const nys_precond* P, const double* mu, int64_t nmu,
                                 const double* B, int64_t nrhs, int64_t ldb, double* X, int64_t ldx,
                                 const nys_solve_opts* o, nys_solve_info* info, void* stream);
size_t nys_noalloc_scratch_bytes(void);

/* Ragged batch: nprob independent systems (A_k + mu_k I) x_k = b_k, each with
 * its own operator and preconditioner, solved together (one iteration sweep
 * advances every unfinished problem).  ops, Ps, mu, B, X: host arrays of
 * nprob entries; B[k], X[k] are device float64 vectors of length ops[k].n.
 * ws must hold nys_workspace_size_ragged(ops, Ps, nprob, prec) bytes.
 * info arrays have nprob entries. */
size_t nys_workspace_size_ragged(const nys_operator* ops, const nys_precond* Ps, int32_t nprob,
                                 int32_t prec);
nys_status nys_pcg_solve_ragged(const nys_operator* ops, const nys_precond* Ps, const double* mu,
                                const double* const* B, double* const* X, int32_t nprob,
                                const nys_solve_opts* o, nys_solve_info* info, void* ws,
                                size_t ws_bytes, void* stream);

/* Adjoint of x = (A + mu I)^{-1} b for a scalar loss L with gradient gx =
 * dL/dx (the paper does not treat differentiation; these are the
 * implicit-function formulas).  Solves (A + mu I) lambda = gx with the same
 * preconditioner P, then
 *   gb      (device, n)  = lambda                           = dL/db
 *   *gmu    (host)       = -lambda^T x                      = dL/dmu
 *   *gsigma (host, RBF)  = -lambda^T (dK/dsigma) x,  dK_ij/dsigma =
 *                          K_ij |x_i - x_j|^2 / sigma^3     (implicit part of dL/dsigma)
 *   gX      (device, XTX, rows x n, nullable) = -scale (X x lambda^T + X lambda x^T)
 * x, gx: device float64 n.  gsigma / gX may be NULL.  Synchronises stream. */
nys_status nys_pcg_backward(const nys_operator* A, const nys_precond* P, double mu, const double* x,
                            const double* gx, double* gb, double* gmu, double* gsigma, double* gX,
                            const nys_solve_opts* o, nys_solve_info* info, void* ws,
                            size_t ws_bytes, void* stream);

/* Rectangular RBF products for losses on held-out points (validation set Xv,
 * nv x d, same storage type as the data of A; training points X of A, n x d).
 * All vectors are device float64.
 *   wvec == NULL, transpose = 0:  out (nv) = K(Xv, X) v,       v has n entries
 *   wvec == NULL, transpose = 1:  out (n)  = K(Xv, X)^T v,     v has nv entries
 *   wvec != NULL (transpose must be 0; dsig_out, host, must be non-NULL):
 *       out (nv) = (dK(Xv, X)/dsigma) wvec,  wvec has n entries,
 *       *dsig_out = v^T out,                 v has nv entries,
 *   with dK_ij/dsigma = K_ij |xv_i - x_j|^2 / sigma^3 (the explicit sigma
 *   dependence of a validation loss).  The call reads exactly these lengths;
 *   shorter buffers are undefined behaviour.  Synchronises the stream only in
 *   the wvec form. */
nys_status nys_rbf_cross(const nys_operator* A, const void* Xv, int64_t nv, int64_t ldxv,
                         int32_t transpose, const double* v, double* out, const double* wvec,
                         double* dsig_out, void* ws, size_t ws_bytes, void* stream);

/* ---- Sketch from sampled columns (Section "Random projection versus
 * column sampling"; the paper's kernel ridge regression experiments) ---- */

/* Bytes of workspace for nys_sketch_columns with ell sampled columns. */
size_t nys_workspace_size_columns(const nys_operator* A, int64_t ell);

/* Column-sampling sketch: Omega = I[:, S] (a test matrix with 1-sparse
 * columns; already orthonormal, so the QR step of the base algorithm leaves
 * it as it is) and Y = A Omega = A[:, S], for the ell indices S = idx
 * (device int64, distinct, in [0, n); drawn by the caller, e.g. uniformly
 * without replacement).  RBF operators evaluate the ell kernel columns
 * directly (O(n ell d) work instead of ell products), dense operators gather
 * them, X^T X operators form scale X^T X[:, S] with one GEMM.  All float64
 * (float32 operator data is promoted exactly).  Omega_out, Y_out: device
 * float64 n x ell (ld = ell); pass them to nys_factor (prec NYS_PREC_FP64) to
 * complete the approximation.  Errors: NYS_ERR_ARG (indices out of range or
 * repeated, ell outside [1, n], bad operator).  Synchronises the stream once
 * (index check). */
nys_status nys_sketch_columns(const nys_operator* A, int64_t ell, const int64_t* idx, double* Omega_out,
                              double* Y_out, void* ws, size_t ws_bytes, void* stream);

/* ---- Weighted normal equations X^T D X (Section 6.3, "Approximate
 * cross-validation": the Hessian of a regularised generalised linear model,
 * e.g. logistic weights d_i = p_i (1 - p_i)) ---- */

/* Bytes of workspace for nys_weight_rows (a device flag). */
size_t nys_workspace_size_weight_rows(void);

/* Xw = D^{1/2} X for D = diag(d): row i of Xw is sqrt(d_i) times row i of X,
 * so that an NYS_OP_XTX operator on Xw (rows x cols, leading dimension ldw,
 * the same dtype) is A = scale X^T D X.  Weights are folded once; every later
 * product is the one-pass X^T X product.  X, Xw: device, dtype NYS_F64 or
 * NYS_F32, row-major with leading dimensions ldx, ldw >= cols; Xw may be X
 * (in place, ldw == ldx) or a buffer that does not overlap it.  d: device
 * float64, rows entries, each finite and >= 0 (checked on the device before
 * anything is written).  sqrt(d_i) is rounded to the data type once, so a
 * float32 Xw carries one more float32 rounding per entry.  Errors:
 * NYS_ERR_ARG (shapes, dtype, a negative or non-finite weight: X and Xw are
 * left unchanged), NYS_ERR_WORKSPACE.  Synchronises the stream once. */
nys_status nys_weight_rows(int64_t rows, int64_t cols, int32_t dtype, const void* X, int64_t ldx,
                           const double* d, void* Xw, int64_t ldw, void* ws, size_t ws_bytes, void* stream);

/* ---- Block Nystrom PCG (Section "Block Nystrom PCG") ---- */

/* Bytes of workspace for nys_block_pcg_solve with preconditioner rank ell and
 * s right-hand sides (1 <= s <= 64; 0 otherwise). */
size_t nys_workspace_size_block(const nys_operator* A, int64_t ell, int64_t s);

/* Coupled block PCG for (A + mu I) X = B with s right-hand sides sharing mu:
 * O'Leary's preconditioned block CG recurrences (alpha = (D^T A_mu D)^{-1}
 * Z^T R, beta = (Z^T R)_old^{-1} (Z^T R)_new, s x s Cholesky solves) with the
 * Nystrom preconditioner of eq. (NysPre), after Feng, Owen and Peric's
 * orthogonalisation of B (thin QR B = Q T0 by CholeskyQR2; the block iteration
 * solves for Q and X = Xt T0).  Unlike nys_pcg_solve, whose columns are
 * independent, the columns share one block Krylov space.  Float64 only
 * (o->prec must be NYS_PREC_FP64); X0 = 0 (X is output only).  Stops when
 * every column's residual (the recursive residual mapped back through T0)
 * meets o->tol relative to its column of B, checked every o->check_every
 * iterations (<= 0: every 8), so the count can pass the first converged step
 * by up to check_every - 1.  B: device float64 n x s (ldb), full
 * column rank, else NYS_ERR_ARG.  info arrays: s entries (iters = the block's
 * iteration count).  Returns NYS_OK, NYS_NOT_CONVERGED (cap) or
 * NYS_ERR_BREAKDOWN (an s x s system lost definiteness before convergence).
 * Synchronises the stream at every check. */
nys_status nys_block_pcg_solve(const nys_operator* A, const nys_precond* P, double mu, const double* B, int64_t s,
                               int64_t ldb, double* X, int64_t ldx, const nys_solve_opts* o, nys_solve_info* info,
                               void* ws, size_t ws_bytes, void* stream);

/* ---- Nystrom sketch-and-solve (Section "Nystrom sketch-and-solve") ---- */

/* Bytes of workspace for nys_sketch_solve with n x ell U and k columns. */
size_t nys_workspace_size_sketch_solve(int64_t n, int64_t ell, int64_t k);

/* Solves the proxy system (A_hat + mu I) X = B, A_hat = U diag(lam) U^T, by
 * the Woodbury form of the lemma on approximate regularized inversion, eq.
 * (Woodbury): X = U (Lambda + mu I)^{-1} U^T B + (1/mu)(I - U U^T) B.  The
 * paper's point is that this is NOT a solve of (A + mu I) X = B: its error is
 * set by how well A_hat approximates A against mu (theorem on sketch-and-solve),
 * unlike nys_pcg_solve.  B, X: device float64 n x k (ldb, ldx >= k), must not
 * alias; mu > 0.  U float64 or float32 (promoted).  ws:
 * nys_workspace_size_sketch_solve(n, ell, k) bytes.  Errors: NYS_ERR_ARG. */
nys_status nys_sketch_solve(const nys_precond* P, double mu, const double* B, int64_t k, int64_t ldb, double* X,
                            int64_t ldx, void* ws, size_t ws_bytes, void* stream);

/* ---- Adaptive rank selection (Section "Adaptive rank selection") ---- */

/* Stopping criteria of nys_nystrom_adaptive. */
typedef enum {
  NYS_ADA_ERR = 0,      /* Strategy 1: estimate of ||E|| <= tau mu                   */
  NYS_ADA_ERR_LAM = 1,  /* Strategy 1 with the theorem's second condition:
                           ||E|| estimate <= tau mu and lam_l <= tau mu / 11        */
  NYS_ADA_RATIO = 2     /* Strategy 2: lam_l <= tau mu (no power estimate)           */
} nys_ada_criterion;

/* Bytes of workspace for nys_nystrom_adaptive with sketch sizes up to ell_max
 * (also enough for nys_power_err_est with P->ell <= ell_max). */
size_t nys_workspace_size_adaptive(const nys_operator* A, int64_t ell_max, int32_t prec);

/* Randomized power estimate of ||E||, E = A - U diag(lam) U^T (Appendix,
 * algorithm "Randomized Power method for estimating ||E||"):
 *   v0 = g / ||g||; q times: v = A v0 - U (lam .* (U^T v0)), E = v0^T v,
 *   v0 = v / ||v||.
 * g: device float64 n, the random start vector (an input; nys_gaussian draws
 * one).  *est (host) receives the last E, a lower bound of ||E|| that
 * approaches it as q grows.  prec: NYS_PREC_FP64 forms A v0 in float64; the
 * other modes form it as nys_op_apply does in that mode (from a float32 copy of
 * v0); everything else is float64.  ws: nys_workspace_size_adaptive(A, P->ell,
 * prec) bytes suffice.  Errors: NYS_ERR_ARG (q < 1, shapes).  Synchronises. */
nys_status nys_power_err_est(const nys_operator* A, const nys_precond* P, int32_t q, const double* g,
                             double* est, int32_t prec, void* ws, size_t ws_bytes, void* stream);

/* Adaptive randomized Nystrom approximation (Appendix, algorithm "Adaptive
 * Randomized Nystrom Approximation"; Strategy 2 with criterion NYS_ADA_RATIO).
 * Starting from ell0 columns, the sketch size doubles (each new block of test
 * columns is drawn, orthonormalised on its own and sketched; the earlier
 * blocks and their sketch are kept) until the criterion holds with
 * tol = tau mu; a doubling past ell_max is cut to ell_max, and that last
 * approximation is returned without an estimate.  Every stage is factored as
 * nys_factor does.  Random draws: block j (j = 0, 1, ...) is
 * nys_gaussian(seed + 2j), the start vector of the j-th estimate
 * nys_gaussian(seed + 2j + 1, n, 1).
 * Omega, Y: device float64 n x ld (ld >= ell_max), written: on return their
 *   first P->ell columns hold the accepted test matrix and sketch.
 * P: caller sets n, U (capacity n x ldu, ldu >= ell_max), ldu, dtype and lam
 *   (capacity ell_max); the call sets P->ell (the chosen sketch size), P->nu
 *   and fills U, lam.
 * *err_out (host): the estimate of ||E|| for the returned approximation (NaN
 *   for NYS_ADA_RATIO and when ell_max was reached).
 * Returns NYS_OK when the criterion held, NYS_NOT_CONVERGED when ell_max was
 * reached first (U, lam then hold the rank-ell_max approximation), or an
 * error of nys_sketch / nys_factor.  ws: nys_workspace_size_adaptive(A,
 * ell_max, prec) bytes.  Synchronises the stream. */
nys_status nys_nystrom_adaptive(const nys_operator* A, int64_t ell0, int64_t ell_max, int32_t q, double tau,
                                double mu, int32_t criterion, uint64_t seed, double* Omega, double* Y,
                                int64_t ld, nys_precond* P, double* err_out, int32_t prec, void* ws,
                                size_t ws_bytes, void* stream);

/* Measurement hook.  nys_timing_begin enables, for calls made afterwards on
 * the calling host thread, HIP events recorded on the launch stream
 * immediately before and after each launch of the one-pass X^T X product
 * kernel (the dominant kernel of the ridge solve).  nys_timing_end waits for
 * the recorded events, returns the mean launch duration in milliseconds and
 * the number of launches timed, releases the events and disables timing.
 * Timing costs two event records per launch; it is off by default.
 * Errors: NYS_ERR_ARG (end without begin), NYS_ERR_DEVICE (event failure). */
nys_status nys_timing_begin(void);
nys_status nys_timing_end(double* avg_ms, int64_t* launches);

/* Message for the last non-OK status returned on this thread. */
const char* nys_last_error(void);

/* Library version string. */
const char* nys_version(void);

/* ---- Autotuner of the tile shapes of the RBF block products ---- */

/* The reduced-precision RBF block product V = K P (the sketch Y = K Omega and
 * the products of the batched solves) has several tile shapes: a register
 * kernel with 16, 32 or 64 columns per workgroup, an LDS kernel with 128 or
 * 256, and a split over points sized for 4, 8 or 16 workgroups per compute
 * unit, and for the LDS kernel one or two 16-row fragments per wave.  Without
 * tuning a built-in rule picks one from the column count.
 * nys_autotune times every shape on the caller's operator (n, d), precision
 * mode and each column count ks[i] (2 <= ks[i] <= 4096, nks <= 64) on stream
 * (which it synchronises), and records the fastest in a process-wide table;
 * a later product with k columns on the same n, d and Gram precision takes
 * the entry with the smallest tuned column count >= k (none: the built-in
 * rule).  The shape changes neither the arithmetic of an entry of K nor the
 * result beyond float32 summation order.  The table persists through a text
 * file: nys_autotune_load merges a file (lines "rbf_kv n d mode k reg cf bpc
 * microseconds fr", fr optional; a malformed line rejects the whole file,
 * NYS_ERR_ARG),
 * nys_autotune_save writes the table.  If the environment variable
 * NYS_AUTOTUNE_CACHE names a file, it is loaded before the first lookup and
 * rewritten after each nys_autotune call.  A is an NYS_OP_RBF operator with
 * d <= 32; prec a reduced-precision mode (NYS_PREC_BF16X3_REFINE64 tunes the
 * bf16x3 Gram, the float32 modes the float32 Gram).  ws: at least
 * nys_workspace_size_autotune(A, max ks) bytes.  This is the project's own
 * tuner; the paper has no counterpart. */
size_t nys_workspace_size_autotune(const nys_operator* A, int64_t kmax);
nys_status nys_autotune(const nys_operator* A, int32_t prec, const int64_t* ks, int32_t nks, void* ws,
                        size_t ws_bytes, void* stream);
/* The shape a product with k columns would use now: choice[0] = 1 for the
 * register kernel (0: LDS kernel), choice[1] = column tiles of 16 per
 * workgroup, choice[2] = workgroups per compute unit, choice[3] = row
 * fragments of 16 per wave of the LDS kernel (1 or 2; 1 for the register
 * kernel); *tuned (nullable) = 1 when it comes from the table.  Host only. */
nys_status nys_autotune_query(const nys_operator* A, int32_t prec, int64_t k, int32_t* choice, int32_t* tuned);
int64_t nys_autotune_entries(void);
nys_status nys_autotune_clear(void);
nys_status nys_autotune_load(const char* path);
nys_status nys_autotune_save(const char* path);

#ifdef __cplusplus
}
#endif

#endif /* NYSPCG_H */
