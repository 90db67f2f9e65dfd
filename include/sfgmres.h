/*
 * sfgmres.h -- C ABI of the MI355X (gfx950) sketched-FGMRES solver.
 *
 * Solves A x = b for a square sparse nonsymmetric A in CSR form by flexible
 * GMRES (Guettel & Pearson, "Stabilizing randomized GMRES through flexible
 * GMRES", arXiv 2506.18408, Algorithm 1) whose variable preconditioner is one
 * cycle of sketched GMRES (eq. (1.2) and Section 3): a truncated-Arnoldi
 * Krylov basis B_k of K_k(A, v_j), the sparse sign sketch S, and the sketched
 * least-squares solve z_j = B_k (S A B_k)^+ (S v_j), with the inner dimension
 * k limited by the rules C1 (k <= m), C2 (cond(S A B_k) <= threshold) and C3
 * (the FGMRES residual predicted by the bound of eq. (2.2) is below tol).
 *
 * Conventions for every entry point
 *  - All n- and nnz-sized arrays are DEVICE pointers (HIP device memory on
 *    the current device), owned by the caller, which must keep them alive
 *    and unmodified until the call returns.  Host arrays are marked "host".
 *  - Every call enqueues its GPU work on the caller's HIP stream `stream`
 *    (NULL = the default stream) and returns after that work is complete.
 *    The solves also use a second stream owned by the handle (default
 *    priority, non-blocking), for the inner cycle's slot reductions and
 *    decision kernels; it is ordered against `stream` by events, and the
 *    caller's stream waits for all of its work before the call returns.
 *  - The library allocates no device memory: the caller provides one
 *    workspace of at least the size returned by sfgmres_workspace_bytes,
 *    256-byte aligned.  It allocates only a small pinned host status block,
 *    one stream and a few events per handle (in sfgmres_create and on the
 *    first solve).
 *  - Return codes: 0 = success; > 0 = success with a warning (the result is
 *    valid); < 0 = error, in which case output arrays may be partially
 *    written and sfgmres_last_error(h) describes the problem.  No C++
 *    exception crosses this interface.
 *  - A handle serialises its calls: one call at a time per handle; distinct
 *    handles may be used from distinct host threads.
 */
#ifndef SFGMRES_H
#define SFGMRES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---------------------------------------------------- */
#define SFGMRES_OK               0   /* converged to tol                                  */
#define SFGMRES_NOT_CONVERGED    1   /* max_outer reached; x holds the best (last) iterate */
#define SFGMRES_ERR_INVALID     -1   /* invalid argument                                   */
#define SFGMRES_ERR_HIP         -2   /* a HIP runtime call failed                          */
#define SFGMRES_ERR_WORKSPACE   -3   /* workspace missing, too small or misaligned         */
#define SFGMRES_ERR_NONFINITE   -4   /* NaN/Inf met in a norm or in the outer recurrence   */
#define SFGMRES_ERR_BREAKDOWN   -5   /* S A v_j = 0 (the inner problem is singular), or
                                        h_{j+1,j} = 0 with a singular H_j (z_j = 0)           */
#define SFGMRES_ERR_TIMEOUT     -6   /* the device made no progress for 60 s                */

/* ---- precision modes ------------------------------------------------- */
#define SFGMRES_FP64   0  /* everything in float64                                           */
#define SFGMRES_MIXED  1  /* float32 A values, inner SpMV inputs/outputs and inner basis B;
                             float64 sketch accumulation, sketched QR/least squares,
                             z = B y accumulation, outer SpMV, Gram-Schmidt and Givens       */

/* ---- outer iterations (sfgmres_options.outer) ------------------------ */
#define SFGMRES_OUTER_FGMRES    0  /* Algorithm 1 (default)                               */
#define SFGMRES_OUTER_RESTARTED 1  /* restarted sGMRES (the paper's comparison method)    */

/* ---- preconditioning (sfgmres_options.precond) ----------------------- */
#define SFGMRES_PRECOND_NONE    0  /* (default)                                            */
#define SFGMRES_PRECOND_ILU0    1  /* zero-fill ILU, right preconditioning (Section 4.4, the
                                      "-p" rows of Table 1), in a multicolour elimination
                                      order; needs sorted columns and every diagonal entry
                                      in the pattern; FGMRES outer only                     */

/* ---- sketch operand of the inner SpMV (sfgmres_options.sketch_source) - */
#define SFGMRES_SKETCH_AUTO     0  /* (default) GEN for an FP64 solve with zeta <= 8 and short
                                      rows (at most 8 nonzeros) whose matrix has more than
                                      512 MiB of values and indices, else TABLE            */
#define SFGMRES_SKETCH_TABLE    1  /* read each column of S from a packed table (12 bytes per
                                      column per 8 nonzeros) built at the start of the solve */
#define SFGMRES_SKETCH_GEN      2  /* generate each column of S (Philox + Floyd) inside the
                                      fused SpMV: FP64 and zeta <= 8 only.  The same S, so
                                      results are bit for bit those of TABLE               */

/* ---- matrix storage of the inner SpMV (sfgmres_options.matrix_format) - */
#define SFGMRES_MATRIX_AUTO     0  /* (default) by diagonal when every nonzero lies on at most
                                      8 diagonals j - i, rows hold at most 8 nonzeros and the
                                      diagonals hold less than 1.5 nnz values (stencils in
                                      lexicographic order); CSR otherwise.  The copy is built
                                      at the start of every solve, in the workspace        */
#define SFGMRES_MATRIX_CSR      1  /* always the caller's CSR (no copy, smaller workspace)  */

/* ---- inner stop reasons (sfgmres_info.stop_reason) ------------------- */
#define SFGMRES_STOP_C1         1  /* k reached m                                  */
#define SFGMRES_STOP_C2         2  /* cond estimate of S A B_i exceeded threshold: k = i-1 */
#define SFGMRES_STOP_C3         3  /* predicted outer residual <= tol * ||b||     */
#define SFGMRES_STOP_BREAKDOWN  4  /* truncated Arnoldi produced an exact zero     */
#define SFGMRES_STOP_FORCED     5  /* k replayed from sfgmres_info.forced_k        */
#define SFGMRES_STOP_MID        6  /* two-level FGMRES: inner_k holds the lower
                                      level's outer steps                         */

/* Limits checked by every entry point. */
#define SFGMRES_MAX_ZETA   16     /* nonzeros per sketch column                   */
#define SFGMRES_MAX_S      1024   /* sketch rows                                  */
#define SFGMRES_MAX_M      512    /* inner basis dimension                        */
#define SFGMRES_MAX_T      8      /* Arnoldi truncation window                    */
#define SFGMRES_MAX_OUTER  2000   /* outer FGMRES steps                           */

/* A in CSR: int32 row_ptr[n+1] (row_ptr[0] = 0, non-decreasing,
 * row_ptr[n] = nnz), int32 col_idx[nnz] in [0, n), float64 val[nnz].
 * Columns need not be sorted; duplicates are summed by the SpMV. */
typedef struct sfgmres_csr {
  int64_t n;
  int64_t nnz;
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const double* val;
} sfgmres_csr;

typedef struct sfgmres_options {
  int32_t precision;            /* SFGMRES_FP64 (default) or SFGMRES_MIXED                       */
  int32_t max_outer;            /* outer FGMRES steps, default 100                               */
  double  cond_threshold;       /* C2 threshold on the condition estimate (Sec. 3); 0 = default:
                                   1e15 in FP64 (the paper's value), 1e15 u64/u32 = 1e15 2^-29
                                   ~ 1.86e6 in mixed precision, where the basis is FP32          */
  int32_t record_true_residual; /* 1: also compute ||b - A x_j|| after every outer step (+1 SpMV
                                   and one n x j combination per step), default 0                */
  int32_t profile;              /* N > 0: time the inner SpMV+sketch launch of every N-th
                                   inner step (steps N-1, 2N-1, ...) with HIP events recorded
                                   at the kernel's own start and end; default 0 (off)            */
  int32_t lookahead;            /* inner steps the host enqueues ahead of the last column the
                                   device has decided, 0..64; raised to at least `panel`;
                                   0 = default (2 panel)                                         */
  int32_t panel;                /* columns appended to the sketched QR per decision launch,
                                   0..8; 0 = default (8).  The stopping rule is applied after
                                   every column whatever the panel; up to panel - 1 inner steps
                                   past the stop are computed and discarded                      */
  int32_t outer;                /* SFGMRES_OUTER_FGMRES (default): Algorithm 1, sGMRES cycles as
                                   the flexible preconditioner of FGMRES.  SFGMRES_OUTER_RESTARTED:
                                   restarted sGMRES, the comparison method of Section 4 (each
                                   cycle solves A z = r_j / ||r_j|| and x <- x + ||r_j|| z; C3
                                   uses ||r_j|| as its factor).  The adjoint solve follows it too */
  int32_t identity_sketch;      /* 1: S = I instead of the random sketch (a test option: needs
                                   s == n and zeta == 1).  The sketched least-squares problem of
                                   eq. (1.2) then minimises the true inner residual, so the
                                   inner cycle is GMRES(k) on a truncated-Arnoldi basis of the
                                   same Krylov space.  Default 0                                 */
  int32_t phase_timers;         /* 1: time the phases of the solve with HIP events on the
                                   caller's stream into sfgmres_info.phase_ms; default 0        */
  int32_t precond;              /* SFGMRES_PRECOND_NONE (default) or SFGMRES_PRECOND_ILU0:
                                   M = L U, the zero-fill incomplete factorisation of A in the
                                   order of a Jones-Plassmann colouring of A + A^T (one parallel
                                   level per colour); the inner cycle works on A M^{-1} and
                                   z_j = M^{-1} B_k y_k, so residuals stay b - A x.  Built on
                                   the device at the start of every solve (of A^T for the
                                   adjoint), factored in float64; with precision MIXED the
                                   triangular solves read a float32 copy of the factor values
                                   and keep their intermediate vector in float32 (products and
                                   sums in float64), like the matrix and the vectors of the
                                   inner SpMV.  SFGMRES_ERR_INVALID for unsorted columns or a
                                   missing diagonal entry, SFGMRES_ERR_BREAKDOWN for a zero
                                   pivot                                                          */
  int32_t mid_outer;            /* 0 (default): one sGMRES cycle per outer step.  N > 0: two-level
                                   FGMRES (Section 5's multi-level FGMRES): z_j is the result of a
                                   lower-level FGMRES solve of A z = v_j (zero initial guess, the
                                   same sGMRES cycles, preconditioner and precision) of at most N
                                   outer steps, which stops once eq. (2.2) predicts the top-level
                                   tolerance: ||r~_{j-1}|| ||v_j - A z|| <= tol ||b||.  The
                                   workspace then also holds the lower level's.  FGMRES outer only;
                                   info.inner_k[j] = the lower level's outer steps,
                                   info.total_inner = all sGMRES inner steps                     */
  int32_t sketch_source;        /* SFGMRES_SKETCH_AUTO (default), _TABLE or _GEN: where the fused
                                   inner SpMV takes the columns of S from (a speed choice only)  */
  int32_t matrix_format;        /* SFGMRES_MATRIX_AUTO (default) or _CSR: how the fused inner
                                   SpMV reads A.  The diagonal copy sums every row in the same
                                   order as CSR, so results are bit for bit those of CSR      */
} sfgmres_options;

/* Solve diagnostics.  Scalars are always written; each per-step array is a
 * HOST array of the stated length, or NULL to skip it. */
typedef struct sfgmres_info {
  int32_t outer_iters;              /* J, outer steps taken                          */
  int32_t converged;                /* 1 if the implicit residual reached tol        */
  int32_t total_inner;              /* sum of the inner dimensions k_j               */
  int32_t status;                   /* return code of the call                       */
  double  rel_residual;             /* |g_{J+1}| / ||b||, the minimised residual     */
  double  true_rel_residual;        /* ||b - A x|| / ||b|| of the returned x (float64) */
  double* residual_history;         /* [max_outer+1]: |g_{j+1}| / ||b||, entry 0 = ||r0||/||b|| */
  double* true_residual_history;    /* [max_outer]: ||b - A x_j||/||b|| (record_true_residual) */
  int32_t* inner_k;                 /* [max_outer]: k_j                              */
  int32_t* stop_reason;             /* [max_outer]: SFGMRES_STOP_*                   */
  double* cond_at_stop;             /* [max_outer]: condition estimate of S A B_{k_j} */
  double* inner_sketched_residual;  /* [max_outer]: ||S(v_j - A z_j)|| at k_j        */
  double* inner_true_residual;      /* [max_outer]: ||v_j - A z_j||                  */
  double* ffom_residual;            /* [max_outer]: FFOM residual norm, eq. (2.1), absolute */
  const int32_t* forced_k;          /* input [max_outer] or NULL: replay these inner
                                       dimensions (k_j steps, no C1-C3 tests); every
                                       entry in [0, m], 0 = not forced (SFGMRES_ERR_INVALID
                                       otherwise)                                      */
  double  spmv_ms;                  /* profile: summed duration of the timed inner
                                       SpMV+sketch launches that did work              */
  int64_t spmv_launches;            /* profile: number of those launches              */
  double  solve_ms;                 /* host wall time of the call                      */
  double* bound;                    /* [max_outer]: the right side of eq. (2.2) for step j,
                                       ||r~_{j-1}|| ||v_j - A z_j|| (absolute; ||r~_0|| =
                                       beta), which bounds the minimised residual |g_{j+1}| */
  double* delta_bound;              /* [max_outer]: delta_j of the recursive bound eq. (2.3),
                                       delta_j = ||v_j - A z_j|| / sqrt(1 - delta_{j-1}^2),
                                       delta_0 = 0, so that |g_{j+1}| <= delta_j |g_j| while
                                       every delta so far is < 1; NaN once 1 - delta^2 <= 0 */
  double* ffom_x;                   /* DEVICE [n] output or NULL: the FFOM iterate of the
                                       last outer step J (Algorithm 1, "FFOM" line),
                                       x~_J = x0 + Z_J H_J^{-1} beta e_1; NaN entries when H_J
                                       is singular.  FGMRES outer only (the restarted outer
                                       leaves it untouched)                                 */
  double  phase_ms[8];              /* phase_timers: summed GPU time per phase, ms:
                                       [0] set-up (tiles, sketch, FP32 values, r0, S v_1),
                                       [1] inner steps of the cycles (until each cycle's last
                                           decision is in), [2] y = R^{-1} d and z_j = B y,
                                       [3] outer SpMV, Gram-Schmidt, Givens, v_{j+1} and S v,
                                       [4] diagnostic true residuals (record_true_residual),
                                       [5] final iterate, its true residual, FFOM iterate,
                                       [6] adjoint: CSR(A^T), [7] adjoint: dL/dA            */
  int32_t sketch_generated;         /* 1 if the inner SpMV generated the columns of S
                                       (sketch_source), 0 if it read the packed table    */
  int32_t dia_diagonals;            /* diagonals of the inner SpMV's copy of A (0: CSR) */
  int32_t matrix_streamed;          /* 1 if the inner SpMV read the CSR values and indices
                                       with streaming (non-temporal) loads              */
  int32_t reserved_i;
  double  reserved[2];
} sfgmres_info;

typedef struct sfgmres_ctx* sfgmres_handle;

/* Fill *opt with the defaults listed above.  Returns SFGMRES_OK. */
int sfgmres_default_options(sfgmres_options* opt);

/* Workspace bytes needed by sfgmres_solve (adjoint = 0) or
 * sfgmres_solve_adjoint (adjoint = 1) for a problem with n unknowns, nnz
 * nonzeros, inner dimension m, window t, sketch rows s and zeta nonzeros per
 * sketch column under *opt (NULL = defaults).  Writes the size to *bytes.
 * The workspace holds, among others, the inner basis (n x (m+1), float64 or
 * float32), the outer bases V and Z (n x (max_outer+1) each, float64), the
 * packed sketch (12 ceil(zeta/8) bytes per column of S), with matrix_format
 * AUTO room for the matrix by diagonal (8 diagonals of n values in the inner
 * SpMV's precision), with precond ILU0 the factors and their colour-ordered
 * copy, with mid_outer the lower level's whole workspace and, for the
 * adjoint, CSR(A^T). */
int sfgmres_workspace_bytes(int64_t n, int64_t nnz, int32_t m, int32_t t, int32_t s, int32_t zeta,
                            const sfgmres_options* opt, int32_t adjoint, size_t* bytes);

/* Create a handle bound to the current HIP device (with its decision
 * stream).  Returns SFGMRES_ERR_HIP if the runtime cannot provide them. */
int sfgmres_create(sfgmres_handle* h);

/* Release a handle (NULL is ignored). */
void sfgmres_destroy(sfgmres_handle h);

/* Text of the last error on h (never NULL; "" if none).  Valid until the
 * next call on h. */
const char* sfgmres_last_error(sfgmres_handle h);

/* Solve A x = b (Algorithm 1 with an sGMRES inner cycle, Section 3).
 *   A      : CSR as above (device arrays).
 *   b      : [n] right-hand side.
 *   x0     : [n] initial guess or NULL for zero.
 *   x      : [n] output solution (may alias x0).
 *   m      : inner basis dimension cap k_max (rule C1), 1 <= m < s.
 *   t      : Arnoldi truncation window (Section 4.1), 0 <= t <= min(m, SFGMRES_MAX_T);
 *            t = 0 builds a normalised power basis.
 *   s      : sketch rows, m < s <= SFGMRES_MAX_S.
 *   zeta   : nonzeros per sketch column, 1 <= zeta <= min(s, SFGMRES_MAX_ZETA).
 *   tol    : relative tolerance on ||b - A x|| / ||b||, > 0.
 *   seed   : 64-bit seed of the sketch (Philox4x32-10 key).
 *   opt    : options or NULL for defaults.
 *   info   : diagnostics (host struct) or NULL.
 *   ws, ws_bytes : device workspace (see above).
 *   stream : hipStream_t of the caller, as void*.
 * Returns SFGMRES_OK or SFGMRES_NOT_CONVERGED with x written, or an error.
 * ||b|| = 0 returns x = 0 and OK; ||b - A x0|| <= tol ||b|| returns x = x0. */
int sfgmres_solve(sfgmres_handle h, const sfgmres_csr* A, const double* b, const double* x0,
                  double* x, int32_t m, int32_t t, int32_t s, int32_t zeta, double tol,
                  uint64_t seed, const sfgmres_options* opt, sfgmres_info* info,
                  void* ws, size_t ws_bytes, void* stream);

/* Adjoint solve for reverse-mode differentiation of x = A^{-1} b: builds
 * CSR(A^T) in the workspace, solves A^T lambda = g with the same method and
 * parameters (same sketch seed), and, if x and grad_val are non-NULL, writes
 * grad_val[p] = -lambda[row(p)] * x[col(p)] for every nonzero p of A (the
 * gradient of L with respect to A's values when g = dL/dx); dL/db = lambda.
 *   g       : [n] input, lambda : [n] output, x : [n] forward solution or NULL,
 *   grad_val: [nnz] output or NULL.
 * Other arguments and return codes as sfgmres_solve; info describes the
 * transposed solve. */
int sfgmres_solve_adjoint(sfgmres_handle h, const sfgmres_csr* A, const double* g,
                          double* lambda, const double* x, double* grad_val, int32_t m,
                          int32_t t, int32_t s, int32_t zeta, double tol, uint64_t seed,
                          const sfgmres_options* opt, sfgmres_info* info, void* ws,
                          size_t ws_bytes, void* stream);

/* Write CSR(A^T) and the value map perm (val_T[q] = val[perm[q]]): row_ptr_t
 * [n+1], col_idx_t [nnz], val_t [nnz] (may be NULL), perm [nnz] -- device
 * arrays.  Rows of A^T list their columns in ascending order.  Needs
 * sfgmres_transpose_workspace_bytes of workspace. */
int sfgmres_transpose_workspace_bytes(int64_t n, int64_t nnz, size_t* bytes);
int sfgmres_transpose(sfgmres_handle h, const sfgmres_csr* A, int32_t* row_ptr_t,
                      int32_t* col_idx_t, double* val_t, int32_t* perm, void* ws,
                      size_t ws_bytes, void* stream);

/* Matrix powers for the t = 0 basis (Section 5: precomputing a few powers
 * A, A^2, ..., A^p, which the t = 0 variant can do since its basis needs no
 * inner products): Y[:, l-1] = A^l u for l = 1..p (p <= 8), with
 * C[:, l-1] = S A^l u (the s sketch rows, S as in sfgmres_sketch_materialize)
 * and norm2[l-1] = ||A^l u||^2.  The rows are split into slabs of at least
 * the matrix bandwidth max |i - j| (and at least slab_rows; 0 = a default
 * that keeps about 160 MB between a slab's first and last level) and one
 * launch computes slab tau - 2(l-1) of every level l, so each slab of A is
 * read p times within a few launches (from the last-level cache after the
 * first).  u, Y (n x p, column-major, leading dimension ldy >= n), C (s x p),
 * norm2 [p]: device arrays.  A test and measurement export; needs
 * sfgmres_powers_workspace_bytes of workspace. */
int sfgmres_powers_workspace_bytes(int64_t n, int64_t nnz, int32_t p, int32_t s, int32_t zeta,
                                   size_t* bytes);
int sfgmres_matrix_powers(sfgmres_handle h, const sfgmres_csr* A, const double* u, int32_t p,
                          int32_t s, int32_t zeta, uint64_t seed, int64_t slab_rows, double* Y,
                          int64_t ldy, double* C, double* norm2, void* ws, size_t ws_bytes,
                          void* stream);

/* The zero-fill ILU factorisation that SFGMRES_PRECOND_ILU0 builds (Section
 * 4.4's right preconditioner), as a test export: lu [nnz] receives the
 * factor values on A's pattern (entries whose column has a lower colour
 * than their row hold L, unit diagonal implied; the others hold U) and
 * color [n] the Jones-Plassmann colour of every row, which fixes the
 * elimination order (colour, then index).  Device arrays; needs
 * sfgmres_ilu_workspace_bytes of workspace.  Errors as for the option. */
int sfgmres_ilu_workspace_bytes(int64_t n, int64_t nnz, size_t* bytes);
int sfgmres_ilu0(sfgmres_handle h, const sfgmres_csr* A, double* lu, int32_t* color, void* ws,
                 size_t ws_bytes, void* stream);

/* Workspace bytes of sfgmres_sketch_materialize and sfgmres_sketch_apply
 * for an s x n sketch with zeta nonzeros per column. */
int sfgmres_sketch_workspace_bytes(int64_t n, int32_t s, int32_t zeta, size_t* bytes);

/* The sketch S (s x n) defined by (seed, s, zeta), as the solver generates
 * it (Section 4.1's sparse sketch with zeta nonzeros per column): for every
 * column r, rows[r*zeta + d] in [0, s) (distinct over d) and
 * signs[r*zeta + d] in {-1, +1}; the nonzero value is signs/sqrt(zeta).
 * Column r's entries come from Philox4x32-10 with key (seed mod 2^32,
 * seed div 2^32) and counter (r, block, 0, 0) by Floyd's sampling.
 * rows [n*zeta] int32, signs [n*zeta] int8: device arrays. */
int sfgmres_sketch_materialize(sfgmres_handle h, int64_t n, int32_t s, int32_t zeta,
                               uint64_t seed, int32_t* rows, int8_t* signs, void* ws,
                               size_t ws_bytes, void* stream);

/* out[s] = S w for w [n] (float64), with the packed sketch and the sketch
 * kernel the solver uses for S v_j. */
int sfgmres_sketch_apply(sfgmres_handle h, int64_t n, int32_t s, int32_t zeta, uint64_t seed,
                         const double* w, double* out, void* ws, size_t ws_bytes,
                         void* stream);

/* One inner step's fused kernel on its own: w = scale * A u, c = S w (s
 * entries), dots[l] = <w, U_l> for the `nwin` vectors U_l (columns of the
 * n x nwin column-major array U, leading dimension ldu), norm2 = ||w||^2.
 * u, w, U: float64 [n].  c: [s], dots: [nwin] (nwin <= SFGMRES_MAX_T),
 * norm2: [1] device outputs.  Needs sfgmres_spmv_workspace_bytes. */
int sfgmres_spmv_workspace_bytes(int64_t n, int64_t nnz, int32_t s, int32_t zeta,
                                 size_t* bytes);
int sfgmres_spmv_sketch(sfgmres_handle h, const sfgmres_csr* A, const double* u, double scale,
                        double* w, int32_t s, int32_t zeta, uint64_t seed, const double* U,
                        int64_t ldu, int32_t nwin, double* c, double* dots, double* norm2,
                        void* ws, size_t ws_bytes, void* stream);

/* Allocation-free variant of sfgmres_spmv_sketch, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the same kernels and results (bit for
 * bit), with no workspace argument.  Its workspace is a static device array
 * of sfgmres_noalloc_scratch_bytes (64 MiB) that every GPU the library runs
 * on holds until the process ends; problems whose workspace
 * (sfgmres_spmv_workspace_bytes) exceeds it are rejected with
 * SFGMRES_ERR_WORKSPACE before any launch.  The call allocates nothing
 * (no hipMalloc or hipFree, no allocating library routine).  Every call on
 * one GPU shares that GPU's array: calls that overlap on one GPU (other
 * streams or host threads) race and must be serialised by the caller.
 * Arguments, layouts and the other return codes as sfgmres_spmv_sketch; the
 * handle's device must be current. */
int sfgmres_noalloc_scratch_bytes(size_t* bytes);
int sfgmres_spmv_sketch_noalloc(sfgmres_handle h, const sfgmres_csr* A, const double* u,
                                double scale, double* w, int32_t s, int32_t zeta, uint64_t seed,
                                const double* U, int64_t ldu, int32_t nwin, double* c,
                                double* dots, double* norm2, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* SFGMRES_H */
