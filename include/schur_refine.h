/*
 * schur_refine.h - C interface of the MI355X (gfx950) library for the iterative
 * refinement of Schur decompositions (Bujanovic, Kressner, Schroder, "Iterative
 * Refinement of Schur decompositions", arXiv 2203.10879).
 *
 * Problem (Section 2, Algorithm 1 and Algorithm 4): given A and a nearly unitary
 * Q-hat such that Q-hat^H A Q-hat is nearly upper triangular, compute a unitary Q
 * (to high precision, hp) with Q^H A Q upper triangular. Each pass evaluates
 * That = Q^H A Q in hp, splits it into its upper part T and strictly lower part E,
 * solves the triangular matrix equation stril(T L - L T) = -E (Section 2.1,
 * eq. (7)) in low precision (lp), and applies the merged Newton-Schulz update
 * Q <- 1/2 Q (2I + 2W - Y - YW + W^2 + W^3), W = L - L^H, Y = Q^H Q - I
 * (Section 2.4, eq. (alg:eq:NSmerged)). Before the loop Q-hat is orthogonalised by
 * one Newton-Schulz step (eq. (alg:eq:NS)).
 *
 * Tiers: hp = FP64 (native FP64 MFMA, optionally compensated accumulation, or an
 * Ozaki-style split on INT8/BF16 MFMA) with lp = FP32; hp = double-double with
 * lp = FP64 (schur_refine_dd).
 *
 * Conventions for every entry point:
 *  - Matrices are n x n, column-major, leading dimension n, complex128 stored as
 *    interleaved (re, im) doubles (C99 double _Complex / hipDoubleComplex layout),
 *    unless a parameter says complex64 (interleaved floats).
 *  - Matrix pointers are DEVICE pointers owned by the caller; the library never
 *    frees them. Host pointers are marked "host".
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream). Work is
 *    enqueued on it; the refinement entry points synchronise it to read residuals.
 *  - Return value: SR_OK (0) or a positive outcome code (the last iterate is still
 *    written), or a negative error code (outputs untouched when validation fails).
 *  - No exceptions cross the interface. Calls on different streams with different
 *    workspaces may run concurrently; calls sharing a workspace must not overlap.
 */
#ifndef SCHUR_REFINE_H
#define SCHUR_REFINE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SR_OK = 0,             /* relative stril residual reached tol                      */
  SR_NOT_CONVERGED = 1,  /* `iters` passes done without reaching tol                 */
  SR_STAGNATED = 2,      /* residual stopped decreasing at the hp accumulation floor */
  SR_BREAKDOWN = 3,      /* non-finite value, or two equal diagonal entries of T
                            (Theorem 1: the solve is then singular)                  */
  SR_DIVERGED = 4,       /* residual rose on two consecutive passes                  */
  SR_EINVAL = -1,        /* invalid argument                                         */
  SR_EHIP = -2,          /* a HIP runtime call failed                                */
  SR_ENOMEM = -3,        /* workspace too small or allocation failed                 */
  SR_ENOSYS = -4         /* option not supported by the library                      */
} sr_status;

typedef enum {
  SR_GEMM_FP64 = 0,       /* native FP64 MFMA                                         */
  SR_GEMM_OZAKI_I8 = 1,   /* Ozaki split on INT8 MFMA, INT32 accumulation, for P = A Q,
                             the start's Newton-Schulz products and Q * Delta; That and
                             Y = Q^H Q - I stay native FP64 (the split form of the
                             residual products named for the precision comparison)     */
  SR_GEMM_OZAKI_BF16 = 2, /* Ozaki split on BF16 MFMA: not built (SR_ENOSYS); INT8
                             digits give the same exactness at twice the MFMA rate    */
  SR_GEMM_OZAKI_I8_ALL = 3, /* as SR_GEMM_OZAKI_I8, and That and Y from digit slices too
                             (Y from the column slices of Q made for P); the slice
                             sums are combined in FP64                                 */
  SR_GEMM_OZAKI_CRT = 4   /* every hp product (P, That, Y, the start, Q Delta) as an
                             Ozaki scheme II product on INT8 MFMA: rows and columns
                             scaled to integers of `slices` bits, their residues
                             modulo N pairwise coprime moduli <= 256 multiplied
                             exactly, the product recovered by the Chinese
                             remainder theorem (N = 16 for 55 bits at n <= 4096,
                             against 28 slice pairs for 7 digits)                   */
} sr_gemm_mode;

typedef struct {
  int gemm;               /* sr_gemm_mode for the hp products                         */
  int slices;             /* SR_GEMM_OZAKI_I8(_ALL): 8-bit digits per operand of P = A Q and
                             of the start's Gram matrix, slice pairs up to s + t =
                             slices + 1 (0 = default 7, at most 16);
                             SR_GEMM_OZAKI_CRT: bits of the scaled integers of the
                             main products (0 = default 55, at most 55)               */
  int update_slices;      /* SR_GEMM_OZAKI_I8: digits per operand of Q * Delta
                             (0 = chosen per update from ||Delta||_F, 2..7);
                             SR_GEMM_OZAKI_CRT: bits (0 = from ||Delta||_F, 12..55)   */
  int compensated;        /* 1: two-level K accumulation in the FP64 products P, That
                             and Y: the MFMA accumulators sum chunks of 32 K terms
                             (16 real, for the real products), which are then added
                             into running totals                                      */
  int gate_lp_terms;      /* 1: skip YW, W^2, W^3 whose Frobenius bound is below
                             0.1 u_hp (Section 2.4 notes the high-order terms may
                             fall below roundoff)                                      */
  int trunc;              /* 1: zero any computed entry of L above 1e-5 in modulus
                             (Example 4 device); 0: off                                */
  int timing;             /* 1: time the hp products and the solve with HIP events on
                             `stream` (fills the ms_* fields of sr_info)               */
  void* workspace;        /* device workspace of >= sr_workspace_bytes(n, opts)
                             bytes, or NULL to let the library allocate and cache one  */
  size_t workspace_bytes;
  void* stream;           /* hipStream_t                                               */
  int strict_stop;        /* 1: a pass with residual <= tol ends the refinement only
                             after at least one update whose correction was
                             negligible to second order, ||W||_F^2 <= u_hp (u_hp =
                             2^-53, or 2^-104 in the double-double tier); until then
                             passes continue (no stagnation or divergence test while
                             the residual is below tol). For matrices whose entries
                             span many orders of magnitude (graded, companion), where
                             the normwise residual reaches tol, even at the start,
                             while small parts of Q still move.
                             0 (default): the residual alone decides                 */
  int solver;             /* solve of the triangular equation in the FP32 tier
                             (schur_refine): SR_SOLVER_WAVEFRONT (0, default) or
                             SR_SOLVER_RECURSIVE (1, Algorithm 3); other entry points
                             take only 0 (SR_ENOSYS otherwise)                        */
  int rec_leaf;           /* SR_SOLVER_RECURSIVE: largest node solved without a split,
                             in rows (rounded up to the 16-row tile; 0 = 64)           */
  int skip_orth;          /* schur_refine only (SR_ENOSYS elsewhere). 1: skip the
                             product Y = Q^H Q - I of an update when Q (I + W) is
                             already unitary in hp (Section 2.4, the remark after the
                             merged update): the next ||Y|| predicted from the last
                             computed Y and W by the Newton-Schulz identity (Lemma 2)
                             is below u_hp and ||W||_F^2 <= u_hp; the update then takes
                             Y = 0. Never twice in a row; if the prediction holds but
                             ||W||^2 is larger, Y is formed after the solve. 0: off
                             (default)                                                 */
  int lp_digits;          /* schur_refine with a split form of the hp products
                             (SR_GEMM_OZAKI_*; SR_EINVAL with SR_GEMM_FP64, SR_ENOSYS in
                             the other entry points when nonzero): 0 (default) forms
                             the lp products W^2, W^3, YW in FP32 on MFMA; 1..7 forms
                             them from that many balanced 8-bit digits per operand on
                             INT8 MFMA (pairs s + t <= lp_digits + 1), W^2 and W^3 over
                             the tiles on and above the diagonal, rounded once to
                             complex64. The digit error is relative to the row and
                             column maxima of W (about k 2^(-8 lp_digits) max|w_i.|
                             max|w_.j|), FP32's to its entries: 4 digits keep the pass
                             counts of FP32 on the test matrices, 3 can cost a pass.
                             Sizes below 1024 keep FP32.                               */
} sr_opts;

typedef enum {
  SR_SOLVER_WAVEFRONT = 0, /* tile wavefront over the whole strictly lower part (an
                              order of Algorithm 2 by tile anti-diagonals)             */
  SR_SOLVER_RECURSIVE = 1  /* Algorithm 3: split at half the tiles, a triangular
                              Sylvester equation for the lower-left block, two
                              updates of E by FP32 MFMA products, recursion on the
                              diagonal blocks                                         */
} sr_solver;

typedef struct {
  int status;             /* sr_status of the call                                    */
  int iters;              /* passes = evaluations of That (the paper's iterations)    */
  int updates;            /* Q updates done (= iters - 1 when converged)              */
  int hp_gemms;           /* hp products counted as in the paper: 2 + 4(iters-1) + 2  */
  int lp_products;        /* lp products launched (W^2, W^3, YW; (W^2 - Y) W for both) */
  double resid;           /* last ||stril(That)||_F / ||A||_F, computed in hp         */
  double orth;            /* ||Q^H Q - I||_F of the last Y formed (0 if none)         */
  double resid_hist[16];  /* residual of passes 1..min(iters,16)                      */
  double norm_w_hist[16]; /* ||W||_F of updates 1..16                                 */
  float ms_total;         /* device time of the call (HIP events)                     */
  float ms_hp_gemm;       /* with opts.timing: summed time of the hp product launches  */
  int hp_gemm_launches;   /* with opts.timing: number of hp product launches timed     */
  float ms_solve;         /* with opts.timing: summed time of the triangular solves    */
  int update_slices_hist[16]; /* Ozaki modes: digits (SR_GEMM_OZAKI_CRT: bits) used by
                             the Newton-Schulz start (entry 0) and by updates 1..15   */
  int hp_gemm_herm_launches; /* with opts.timing: how many of the timed launches were
                             the Hermitian products Y = Q^H Q - I, which form only the
                             tiles on and above the diagonal (half the work)          */
  float ms_hp_gemm_herm;  /* with opts.timing: the part of ms_hp_gemm they took        */
  float ms_oz_full;       /* with opts.timing in an Ozaki mode: time of the full n x n x n
                             split products with opts->slices digits per operand (P =
                             A Q in every pass; That too with SR_GEMM_OZAKI_I8_ALL and
                             SR_GEMM_OZAKI_CRT, and in schur_refine_dd and
                             schur_refine_td), the INT8
                             product kernel alone (its digit splits are in ms_hp_gemm
                             only)                                                     */
  int oz_full_launches;   /* number of launches timed in ms_oz_full                     */
  int oz_full_pairs;      /* slice pairs per such launch (s + t <= slices + 1), or the
                             number of moduli with SR_GEMM_OZAKI_CRT                   */
} sr_info;

/* Default options: FP64 MFMA, compensated accumulation on, gating on, no trunc. */
void sr_default_opts(sr_opts* opts);

/* Bytes of device workspace schur_refine needs for size n under `opts`. */
size_t sr_workspace_bytes(int n, const sr_opts* opts);

/* Refine one Schur decomposition (Algorithm 4 from its second step).
 *  A  (in,  device, complex128 n x n): the matrix, read only.
 *  Q  (in/out, device, complex128 n x n): in: the start Q-hat (nearly unitary, e.g.
 *     FP32 Schur vectors widened to complex128); out: the refined Q.
 *  T  (out, device, complex128 n x n): triu(Q^H A Q) of the last pass; its strictly
 *     lower part is set to zero.
 *  n >= 1; iters >= 1: maximum number of passes; tol > 0: stop when
 *  ||stril(Q^H A Q)||_F / ||A||_F <= tol (computed in hp).
 *  opts may be NULL (defaults); info (host) may be NULL.
 *  n = 1: T = A, Q = q / |q|, one pass. */
int schur_refine(const void* A, void* Q, void* T, int n, int iters, double tol,
                 const sr_opts* opts, sr_info* info);

/* Refine `batch` independent decompositions of possibly different sizes (the
 * FP64 tier of schur_refine on each).
 *  n (host, int[batch]); A, Q, T (host arrays of `batch` device pointers), each
 *  matrix laid out as in schur_refine. info (host, sr_info[batch]) may be NULL
 *  (the ms_* fields are not filled).
 *  Each pass runs as one fixed sequence of grouped launches over the whole batch
 *  (persistent tile-table products, the solve by tile diagonal across the batch,
 *  one block per matrix for the elementwise steps) with device-side loop control;
 *  two passes are captured in a HIP graph and replayed (the graph is kept for the
 *  next call, see sr_batched_graph_builds). The tile edge (64 or 32) of each size
 *  bucket is chosen by timing both on the first batch that contains the bucket
 *  (kept for the process). opts->gemm must be SR_GEMM_FP64. The work is ordered
 *  after the caller's stream, and the call returns after it completed. With a
 *  caller workspace the call allocates no device memory (one pinned host word per
 *  host thread is made on the thread's first call).
 *  Returns the worst (largest) outcome over the batch, or a negative error. */
int schur_refine_batched(int batch, const int* n, const void* const* A, void* const* Q,
                         void* const* T, int iters, double tol, const sr_opts* opts,
                         sr_info* info);

/* Bytes of device workspace schur_refine_batched needs (opts->workspace; when it
 * is NULL the call allocates and frees its own). */
size_t sr_workspace_bytes_batched(int batch, const int* n, const sr_opts* opts);

/* Tile edge the batched autotuner chose for matrices of size n (-1: not tuned). */
int sr_batched_tile_edge(int n);

/* Persistent blocks per CU the autotuner chose for matrices of size n (1, 2, 4 or 8;
 * -1: not tuned). The autotuner times, once per size bucket (n <= 32, 64, 128, 192,
 * 256, larger), the grouped product P = A Q of up to 256 of the bucket's matrices for
 * both tile edges and grids of 1, 2, 4 and 8 blocks per CU, and keeps the fastest;
 * among choices within 3% of it, the one with the most blocks per CU. */
int sr_batched_tile_grid(int n);

/* Tuning table persistence. A file holds a header line and one line per device and
 * bucket ("<arch>/<CUs> <bucket> <edge> <blocks per CU> <ms>"). sr_tuning_save writes
 * the current device's table (keeping other devices' lines already in the file;
 * returns the number of entries written); sr_tuning_load reads the current device's
 * lines into the table (returns the number read; SR_EINVAL for a missing or foreign
 * file; loaded buckets are not timed again). With the environment variable
 * SR_TUNING_FILE set, the file is loaded before the first tuning and written after
 * each new one. sr_tuning_reset empties the table (and does not reload the file);
 * sr_tuning_runs counts the buckets timed in this process. */
int sr_tuning_save(const char* path);
int sr_tuning_load(const char* path);
void sr_tuning_reset(void);
int sr_tuning_runs(void);

/* Number of two-pass graphs schur_refine_batched has captured and instantiated in
 * this process. A call with a caller-owned workspace keeps its graph (per host
 * thread) and the next call on that thread replays it without a new capture when
 * the workspace address, the sizes, the tile edges, iters, tol and the options are
 * unchanged (the matrices' addresses may differ). */
int sr_batched_graph_builds(void);

/* Double-double tier (Section 3 refines to higher than working precision the same
 * way): A = A_hi + A_lo, Q = Q_hi + Q_lo, T = T_hi + T_lo (all device, complex128
 * n x n, each pair a double-double matrix). Every hp product (P = A Q, That, Y, the
 * Newton-Schulz start and Q Delta) is an Ozaki split product of the double-double
 * operands on INT8 MFMA with double-double accumulation; the solve and the lp
 * products YW, W^2, W^3 run in FP64, gated against 0.1 * 2^-104 (W^3 - YW as one
 * product (W^2 - Y) W when both pass).
 *  opts->slices: 8-bit digits per operand of the hp products (0 = 14, at most 32).
 *    The digits of a row or column are relative to its largest entry, so a matrix
 *    whose rows or columns span many orders of magnitude needs more digits to keep
 *    its small entries to double-double accuracy (14 digits cover about 111 bits);
 *  opts->update_slices: digits of Q Delta: 0 = the same as opts->slices (the digits
 *    of Q are relative to its row maxima, and the Schur vectors of a badly scaled
 *    matrix have entries far below them); -1 = chosen from ||Delta|| (2..14, for
 *    well-scaled matrices); otherwise the count given (at most 32);
 *  opts->gemm and opts->compensated are ignored. The stagnation floor is
 *  100 * 2^-104 * sqrt(n). Outputs and statuses as for schur_refine. */
int schur_refine_dd(const void* A_hi, const void* A_lo, void* Q_hi, void* Q_lo, void* T_hi,
                    void* T_lo, int n, int iters, double tol, const sr_opts* opts,
                    sr_info* info);

/* Bytes of device workspace schur_refine_dd needs for size n under `opts`. */
size_t sr_workspace_bytes_dd(int n, const sr_opts* opts);

/* Triple-double tier (more than two cells per number: Section 3 holds an hp number in
 * several doubles, 2 for quadruple and 6 for 100 digits; Section 4 names further
 * precision levels): every hp value is a renormalized expansion of
 * three complex128 arrays (A[0] + A[1] + A[2], likewise Q and T; column-major,
 * leading dimension n, device memory; Q in/out, T out). hp products: Ozaki splits of
 * the three-term operands into opts->slices 8-bit digits (0 = 20, at least 20, at
 * most 32) on INT8 MFMA with a three-term FP64 accumulation (about 150 bits: the
 * tolerance should stay above about 1e-44); lp = FP64 (solve and lp products) as in
 * the double-double tier. n >= 2 and (slices + 4) 3 n^2 < 2^31, i.e. n <= 5400 with 20
 * digits (the product kernel's 32-bit plane offsets; SR_EINVAL otherwise). Other outcomes as
 * schur_refine (stagnation measured against u = 2^-150). opts->gemm must be
 * SR_GEMM_FP64 and opts->solver, skip_orth 0 (SR_ENOSYS otherwise). */
int schur_refine_td(const void* const* A, void* const* Q, void* const* T, int n, int iters, double tol,
                    const sr_opts* opts, sr_info* info);

/* Bytes of device workspace schur_refine_td needs for size n. */
size_t sr_workspace_bytes_td(int n, const sr_opts* opts);

/* Real Schur variant (Section 3 extends the method to the real Schur form: T is
 * quasi-upper-triangular, with 2 x 2 diagonal blocks holding complex conjugate
 * pairs). A, Q, T: real n x n, float64, column-major, leading dimension n (device).
 * blocks (host, int[n], may be NULL = none): blocks[i] = 1 when rows and columns
 * i, i + 1 form a 2 x 2 diagonal block of the start's quasi-triangular form (as a
 * real Schur decomposition such as LAPACK sgees returns it), else 0; a block may not
 * start at the last row nor overlap the next (SR_EINVAL). The structure is kept:
 * E is the block strictly lower part of That (every entry below the diagonal except
 * the subdiagonal entry of a 2 x 2 block), T the rest, and the correction L solves
 * the block form of the triangular equation, T_II L_IJ - L_IJ T_JJ = -(E_IJ +
 * sum_{K>I} T_IK L_KJ - sum_{K<J} L_IK T_KJ), I > J. FP64 tier: the products on FP64
 * MFMA (compensated by default), the solve in FP32 (each 2 x 2 block triangularized
 * by a 2 x 2 unitary, the complex sweep run on the result, the correction mapped
 * back), the merged update as in schur_refine. opts->gemm must be SR_GEMM_FP64
 * (SR_ENOSYS otherwise); opts->trunc is ignored. Outputs and statuses as for
 * schur_refine (the residual is the block strictly lower one); T is written with its
 * block strictly lower part zero. n = 1: T = A, Q = sign(q). */
int schur_refine_real(const void* A, void* Q, void* T, const int* blocks, int n, int iters, double tol,
                      const sr_opts* opts, sr_info* info);

/* Bytes of device workspace schur_refine_real needs for size n. */
size_t sr_workspace_bytes_real(int n, const sr_opts* opts);

/* Static description of a status code. */
const char* sr_status_string(int status);

/* ---------------------------------------------------------------------------
 * Stage entry points: the steps of one pass, callable on their own (a caller may
 * drive the loop itself). All pointers are device pointers; `ws` is a workspace of
 * at least sr_workspace_bytes(n, NULL) bytes; `stream` as above. They return SR_OK
 * or a negative error code and do not synchronise the stream unless stated.
 * ------------------------------------------------------------------------- */

/* C = op(A) B (+ Cin), complex128, native FP64 MFMA (Section 2.4: the hp products).
 * op(A) is m x k: opa = 0 uses A (m x k, leading dim lda), opa = 1 uses the
 * conjugate transpose of A (k x m, leading dim lda). B is k x n (ldb), C is m x n
 * (ldc). Cin (may be NULL) is added when given (ldcin). compensated = 1 selects
 * chunked accumulation with error-free combination. C must not overlap A, B, Cin. */
int sr_zgemm(int opa, int m, int n, int k, const void* A, int lda, const void* B, int ldb,
             const void* Cin, int ldcin, void* C, int ldc, int compensated, void* stream);

/* Real products of the real Schur variant: C = op(A) B (+ Cin), float64 on FP64
 * MFMA, op(A) = A (opa = 0) or A^T (opa = 1), other arguments as sr_zgemm. */
int sr_dgemm(int opa, int m, int n, int k, const void* A, int lda, const void* B, int ldb,
             const void* Cin, int ldcin, void* C, int ldc, int compensated, void* stream);

/* The FP32 block solve of the real variant: T_lp (float32 n x n, quasi-upper-
 * triangular with the 2 x 2 blocks marked by `blocks`, host, as for
 * schur_refine_real), E_lp (float32, its block strictly lower part read), L_lp
 * (float32 out: the block strictly lower solution, zeros elsewhere). ws: device
 * workspace of >= sr_trisolve_real_ws_bytes(n) bytes. Synchronises the stream;
 * returns SR_BREAKDOWN when two blocks share an eigenvalue or a value is not
 * finite, SR_EINVAL for invalid markers. */
size_t sr_trisolve_real_ws_bytes(int n);
int sr_trisolve_real(const void* T_lp, const void* E_lp, void* L_lp, const int* blocks, int n, void* ws,
                     size_t ws_bytes, void* stream);

/* The FP32 solve of sr_trisolve by the recursive block algorithm (Section 2.1,
 * Algorithm 3 and eqs. (11)-(12)): the node of tile rows [lo, hi) splits at
 * mid = lo + (hi - lo) / 2 (16-row tiles); the triangular Sylvester equation
 * T22 X - X T11 = -E21 of its lower-left block is solved tile by tile in anti-diagonal
 * order; E11 += stril(T12 X) and E22 -= stril(X T12) follow as FP32 MFMA products;
 * the two diagonal blocks recurse, down to nodes of at most leaf_rows rows (rounded up
 * to whole tiles; 0 = 64), solved in the same tile order. All nodes of one depth share
 * the launches. Arguments as sr_trisolve; E_lp is not modified. ws: device workspace
 * of >= sr_trisolve_rec_ws_bytes(n, leaf_rows) bytes (SR_ENOMEM if smaller).
 * Synchronises the stream; SR_BREAKDOWN as sr_trisolve. */
size_t sr_trisolve_rec_ws_bytes(int n, int leaf_rows);
int sr_trisolve_rec(const void* T_lp, const void* E_lp, void* L_lp, int n, int leaf_rows, float trunc, void* ws,
                    size_t ws_bytes, void* stream);

/* C = A B, complex64, FP32 MFMA (the lp products YW, W^2, W^3 of Algorithm 4). */
int sr_cgemm(int m, int n, int k, const void* A, int lda, const void* B, int ldb, void* C,
             int ldc, void* stream);

/* Residual products and split (Algorithm 4, the That, E and T steps):
 * P = A Q, That = Q^H P; T (complex128) = triu(That) with zeros below;
 * T_lp, E_lp (complex64 n x n) = triu(That), stril(That) rounded to FP32;
 * eps (host, may be NULL) = ||stril(That)||_F / ||A||_F. Synchronises `stream` when
 * eps is requested. */
int sr_residual(const void* A, const void* Q, int n, void* T, void* T_lp, void* E_lp,
                double* eps, int compensated, void* ws, void* stream);

/* Triangular matrix equation stril(T L - L T) = -E (Section 2.1, eq. (7)) in FP32.
 * T_lp: complex64, upper triangle (incl. diagonal) read; E_lp: complex64, strictly
 * lower part read (the buffer is not modified); L_lp: complex64 out, strictly lower
 * solution, zeros elsewhere. trunc > 0 zeroes computed entries above trunc in
 * modulus. Returns SR_BREAKDOWN (after synchronising) if two diagonal entries of T
 * coincide or a non-finite value appears; otherwise SR_OK without synchronising. */
int sr_trisolve(const void* T_lp, const void* E_lp, void* L_lp, int n, float trunc,
                void* ws, void* stream);

/* The FP32 solve of sr_trisolve without allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops, harnesses
 * that forbid hipMalloc). Same kernels and the same result as sr_trisolve (bit
 * for bit), but its scratch (the partial sums passed between the solve's launches)
 * is a fixed device array inside the library, one per GPU, kept until the process
 * ends, and the call never synchronises.
 *  T_lp, E_lp, L_lp, n, trunc: as for sr_trisolve (device, complex64 n x n).
 *  status (device, one unsigned, caller-owned): cleared by the call, then set to a
 *    nonzero value if two diagonal entries of T coincide or a non-finite value
 *    appears (sr_trisolve's SR_BREAKDOWN); read it after the stream has run.
 *  n must be <= 4096 (the array holds 20 MiB): larger n returns SR_ENOMEM without
 *  launching anything; null pointers or n < 1 return SR_EINVAL.
 * Every call on one GPU uses the same array, so calls that may overlap on one GPU
 * (other streams, other threads) race and must be ordered by the caller. */
int sr_trisolve_static(const void* T_lp, const void* E_lp, void* L_lp, int n, float trunc,
                       unsigned* status, void* stream);

/* Reordering of the start (Section 2.4, the paragraph on the reordering of
 * Algorithm 4: clustered eigenvalues are moved next to each other, in the order of
 * their projections onto a random line). A: complex128 n x n (read); Q: complex128
 * n x n start, in/out. With T = triu(Q^H A Q) (FP64), unitary swaps of adjacent
 * diagonal entries put the eigenvalues in increasing order of
 * Re(lambda e^{-i theta}); Q is replaced by Q G_1 G_2 ... (the swaps in
 * odd-even transposition order, n phases). theta: the line's direction, chosen by
 * the caller (e.g. at random). perm (device int[n], may be NULL): the original
 * diagonal position of each entry of the new order. ws: device workspace of at
 * least sr_reorder_ws_bytes(n) bytes, caller-owned. Returns SR_EINVAL for null
 * pointers, n < 1, a non-finite theta or a short workspace; otherwise SR_OK without
 * synchronising. */
size_t sr_reorder_ws_bytes(int n);
int sr_reorder_start(const void* A, void* Q, int n, double theta, int* perm, void* ws, size_t ws_bytes,
                     void* stream);

/* The same equation in FP64 (the solve of the double-double tier): T, E, L are
 * complex128 with the roles above; no truncation. Same outcomes. */
int sr_trisolve64(const void* T, const void* E, void* L, int n, void* ws, void* stream);

/* Merged Newton-Schulz update (Algorithm 4, the W, Y, Sigma and Q steps) given L:
 * W = L - L^H, Y = Q^H Q - I (hp), lp products (gated when gate != 0; W^3 - YW as
 * one product (W^2 - Y) W when both pass),
 * Delta = 1/2 Sigma - I = W - Y/2 + (-YW + W^2 + W^3)/2, Q_out = Q + Q Delta.
 * L_lp complex64; Q, Q_out complex128 (must not overlap). norms (host, may be NULL,
 * double[2]) receives ||W||_F and ||Y||_F (synchronises). */
int sr_update(const void* Q, const void* L_lp, void* Q_out, int n, int gate,
              int compensated, double* norms, void* ws, void* stream);

/* Newton-Schulz step Q = 1/2 Qh (3I - Qh^H Qh) = Qh + Qh (-(Qh^H Qh - I)/2)
 * (Algorithm 4, before the loop). Qh, Q complex128, must not overlap. */
int sr_ns_init(const void* Qh, void* Q, int n, int compensated, void* ws, void* stream);

/* Ozaki split product (the hp products of Section 3 built from an Ozaki-scheme
 * splitting) on INT8 MFMA: C = op(A) B (+ Cin), complex128, arguments as sr_zgemm.
 * op(A) is split into slices_a slices of balanced 8-bit digits per row, B into
 * slices_b per column (each with a power-of-two scale per row / column, about
 * 8 * slices - 1 bits below the row / column maximum); slice pairs (s, t) with
 * s + t <= dmax are multiplied exactly in int32 and combined in FP64. dmax =
 * slices_a + slices_b keeps every pair. Outputs with fewer than 256 tiles of
 * 128 x 128 require min(slices_a, slices_b) * k * 2^14 < 2^31 (SR_EINVAL
 * otherwise); larger ones are exact for every k.
 * ws: device workspace of >= sr_ozaki_ws_bytes(...). */
size_t sr_ozaki_ws_bytes(int m, int n, int k, int slices_a, int slices_b);
int sr_ozaki_zgemm(int opa, int m, int n, int k, const void* A, int lda, const void* B, int ldb,
                   const void* Cin, int ldcin, void* C, int ldc, int slices_a, int slices_b,
                   int dmax, void* ws, size_t ws_bytes, void* stream);

/* Double-double operands and result: C_hi + C_lo = op(A_hi + A_lo) (B_hi + B_lo)
 * (+ Cin_hi + Cin_lo), each pair stored as two complex128 matrices with a shared
 * leading dimension. The digits are taken from the exact double-double values, the
 * pair sums are exact in int32 and are accumulated in double-double, so with 14
 * digits per operand and dmax = 15 the result carries about 2^-106 relative to the
 * row and column maxima. A_lo, B_lo, Cin_lo may be NULL (zero). ws as above. */
int sr_ozaki_zgemm_dd(int opa, int m, int n, int k, const void* A_hi, const void* A_lo, int lda,
                      const void* B_hi, const void* B_lo, int ldb, const void* Cin_hi,
                      const void* Cin_lo, int ldcin, void* C_hi, void* C_lo, int ldc,
                      int slices_a, int slices_b, int dmax, void* ws, size_t ws_bytes,
                      void* stream);

/* Triple-double operands and result (the hp products of the triple-double tier):
 * C[0] + C[1] + C[2] = op(A[0] + A[1] + A[2]) (B[0] + B[1] + B[2]) (+ Cin[0] + Cin[1]
 * + Cin[2]); each argument is an array of three device pointers to complex128
 * column-major matrices sharing one leading dimension (terms largest first). The
 * digits (`slices` 8-bit digits per operand, at least 1, at most 32; pairs s + t <=
 * slices + 1) are taken from the exact three-term values, the pair sums are exact
 * in int32 and are accumulated in a three-term FP64 expansion, so with 22 digits the
 * result carries about 2^-150 relative to the row and column maxima. k >= 1, every
 * pointer of A and B set and (slices + 4) 3 max(m, n) k < 2^31 (SR_EINVAL otherwise). Cin may be NULL; when given, all
 * three of its pointers are set. ws: device workspace of >=
 * sr_ozaki_ws_bytes(m, n, k, slices, slices). */
int sr_ozaki_zgemm_td(int opa, int m, int n, int k, const void* const* A, int lda, const void* const* B,
                      int ldb, const void* const* Cin, int ldcin, void* const* C, int ldc, int slices,
                      void* ws, size_t ws_bytes, void* stream);

/* The lp products on INT8 digits (sr_opts.lp_digits): C = A B for complex64 A (m x
 * k), B (k x n), C (m x n), column-major device memory, from `slices` balanced 8-bit
 * digits per operand (1..7; pairs s + t <= slices + 1) with exact int32 pair sums
 * folded in FP64 and rounded once to complex64. herm = 1 (-1): the product is
 * Hermitian (skew-Hermitian), only the elements i <= j are formed and each is stored
 * with its conjugate (negated conjugate) at (j, i); m == n required. The kernel
 * takes at least 256 output tiles of 64 x 64 (m n >= 2^20): SR_EINVAL below that, and
 * for other bad arguments. ws: device workspace of >= sr_ozaki_ws_bytes(m, n, k,
 * slices, slices). */
int sr_ozaki_cgemm(int m, int n, int k, const void* A, int lda, const void* B, int ldb, void* C, int ldc,
                   int slices, int herm, void* ws, size_t ws_bytes, void* stream);

/* Ozaki scheme II product (the hp products of Section 3 from an Ozaki-type scheme,
 * here its CRT form) on INT8 MFMA: C = op(A) B (+ Cin), complex128, arguments as
 * sr_zgemm. Every row of op(A) and column of B is scaled by a power of two to
 * integers of at most `bits` bits (rounded to nearest: an error of at most 2^-bits
 * of the row / column maximum per entry); the residues of those integers modulo
 * N = sr_crt_moduli(k, bits) pairwise coprime moduli <= 256 are multiplied exactly
 * in int32, and each output is recovered from its N residues by the Chinese
 * remainder theorem and rounded once to FP64. Requires k < 65536 and N <= 20
 * (SR_EINVAL otherwise); bits <= 55 for full FP64 operands.
 * ws: device workspace of >= sr_crt_ws_bytes(m, n, k, bits). */
int sr_crt_moduli(int k, int bits);
size_t sr_crt_ws_bytes(int m, int n, int k, int bits);
int sr_crt_zgemm(int opa, int m, int n, int k, const void* A, int lda, const void* B, int ldb,
                 const void* Cin, int ldcin, void* C, int ldc, int bits, void* ws, size_t ws_bytes,
                 void* stream);

/* Diagnostic: one matrix-core instruction (kind 0: v_mfma_f64_16x16x4f64, kind 1:
 * v_mfma_f32_16x16x4f32) on a 16x4 A and a 4x16 B (row-major, host), fed and read
 * back with the lane layout the GEMM kernels assume; D (16x16 row-major, host)
 * equals A B exactly for small integers when that layout is right. */
int sr_diag_mfma(int kind, const double* A, const double* B, double* D);

#ifdef __cplusplus
}
#endif
#endif
