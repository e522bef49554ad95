/*
 * CPU oracle for the iterative refinement of Schur decompositions
 * (Bujanovic, Kressner, Schroder, arXiv 2203.10879).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg call it. It shares no code with the GPU library and the GPU
 * library never calls it.
 *
 * Arithmetic: high precision (hp) is IEEE binary128 (__float128, libquadmath).
 * Low precision (lp) is selectable: float, double or binary128.
 *
 * Storage: n x n complex matrices, column-major, entry (i, j) at index i + j*n
 * (0-based). An hp complex value is the record {__float128 re, im} (32 bytes).
 * Double-double values travel as two complex128 arrays (hi, lo) with
 * value = hi + lo.
 *
 * Parity status of each entry point (what pins it) is stated beside it.
 */
#ifndef SCHUR_REFINE_ORACLE_H
#define SCHUR_REFINE_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { __float128 re, im; } orc_qc;

enum { ORC_LP_FLOAT = 0, ORC_LP_DOUBLE = 1, ORC_LP_QUAD = 2 };

/* Refinement outcome codes. */
enum {
  ORC_OK = 0,            /* relative stril residual reached tol                 */
  ORC_NOT_CONVERGED = 1, /* maxit passes done without reaching tol              */
  ORC_BREAKDOWN = 3,     /* non-finite value, or t_ii == t_jj in the solve       */
  ORC_DIVERGED = 4       /* residual rose on two consecutive passes             */
};

/* Refinement option bits. */
enum {
  ORC_FULL_NS = 1,  /* keep the W^2 Y and W^2 Y W terms of the merged update  */
  ORC_TRUNC = 2     /* large-entry truncation while computing L (Example 4)  */
};

/* Conversions. lo may be NULL (treated as zero / not written). */
void orc_from_dd(long count, const double* hi, const double* lo, orc_qc* out);
void orc_to_dd(long count, const orc_qc* in, double* hi, double* lo);

/* C = op(A) * B in binary128; op(A) is m x k, stored as A (opa = 0, m x k) or as
 * the conjugate transpose of a k x m matrix (opa = 1). B is k x n, C is m x n.
 * Pinned by exact Gaussian-integer products. */
void orc_gemm(int opa, int m, int n, int k, const orc_qc* A, const orc_qc* B, orc_qc* C);

/* Solve stril(T L - L T) = -E for strictly lower triangular L (Section 2.1,
 * eq. (7), entry formula (9) with the column index of L read as j; Algorithm 2).
 * T (upper part incl. diagonal) and E (strictly lower part) are rounded to the
 * low precision `lp`, the substitution runs in lp, and L is returned exactly.
 * order 0: Algorithm 2's column order; order 1: subdiagonal wavefront order
 * (entries with larger i - j first), which also satisfies the order condition (10).
 * trunc > 0: any computed entry with modulus above trunc is set to zero (the
 * Example 4 device: later entries see the zero). Returns ORC_OK or ORC_BREAKDOWN.
 * Pinned by the Kronecker-form linear system, closed forms, and Theorem 1; the
 * truncation by exact rational substitution that zeroes as computed. */
int orc_trisolve(int lp, int order, int n, const orc_qc* T, const orc_qc* E, orc_qc* L,
                 double trunc);

/* One Newton-Schulz step Q = 1/2 Qh (3I - Qh^H Qh) in hp (eq. (alg:eq:NS)).
 * Pinned by Lemma 2's identity Qn^H Qn - I = -3/4 Y^2 + 1/4 Y^3. */
void orc_ns(int n, const orc_qc* Qh, orc_qc* Q);

/* Merged orthogonalisation of Q (I + W) (Section 2.4, eq. (alg:eq:NSmerged)):
 * Y = Q^H Q - I in hp; the products Y W, W^2, W^3 (and W^2 Y, W^2 Y W when
 * full != 0) in lp; Sigma = 2I + 2W - Y - YW + W^2 + W^3 (+ W^2 Y + W^2 Y W)
 * summed in hp; Qn = 1/2 Q Sigma in hp.
 * Pinned against the unmerged Newton-Schulz step of Q (I + W) (lp = quad), and for
 * lp = float and double by the size of the lp rounding of the products (bounded
 * from both sides, scaling with the lp unit roundoff). */
void orc_ns_merged(int lp, int n, const orc_qc* Q, const orc_qc* W, int full, orc_qc* Qn);

/* Algorithm 4 from the start Qh: one Newton-Schulz step, then passes of
 * { That = Q^H (A Q); E = stril(That), T = That - E; eps = ||E||_F / ||A||_F;
 *   stop when eps <= tol; solve for L in lp (Algorithm 2); W = L - L^H;
 *   merged Newton-Schulz update of Q }.
 * A pass is one evaluation of That; hist[p] receives eps of pass p (maxit slots);
 * *iters the number of passes. Qout receives the final Q, Tout = triu(That) of
 * the last pass. Returns an ORC_* outcome.
 * Pinned by exact Schur forms (Walsh-Hadamard test matrices), brute force at
 * small n, the quadratic decrease of eps (Theorem 2), and a start rotated far
 * from the Schur basis for the DIVERGED rule. */
int orc_refine(int lp, int n, const orc_qc* A, const orc_qc* Qh, int maxit, double tol,
               int flags, orc_qc* Qout, orc_qc* Tout, double* hist, int* iters);

/* Evaluation in hp of a computed pair (Q, T) for A (the checks of Section 3):
 * out[0] = ||stril(Q^H A Q)||_F / ||A||_F, out[1] = ||Q^H Q - I||_F,
 * out[2] = ||T - triu(Q^H A Q)||_F (0 when T is NULL), out[3] = ||A||_F. */
void orc_eval(int n, const orc_qc* A, const orc_qc* Q, const orc_qc* T, double out[4]);

/* Row-sampled evaluation for large n: for the rows i in rows[0..nr), row i of
 * Q^H A Q is (q_i^H A) Q and row i of Q^H Q - I is q_i^H Q - e_i^T.
 * out[0] = sqrt(n/nr * sum_i ||stril row_i||^2) / ||A||_F (unbiased estimate of
 * the relative stril residual), out[1] = max_i ||stril row_i|| / ||A||_F,
 * out[2] = sqrt(n/nr * sum_i ||row_i(Q^H Q - I)||^2), out[3] = ||A||_F. */
void orc_eval_rows(int n, const orc_qc* A, const orc_qc* Q, int nr, const int* rows,
                   double out[4]);

/* Complex Schur decomposition of A rounded to lp by the shifted QR algorithm
 * (Householder Hessenberg reduction, then single-shift QR sweeps with Wilkinson
 * shifts and deflation), arithmetic in lp. Returns Z, S with A ~ Z S Z^H, the
 * values widened exactly to hp. Returns 0, or 1 if an eigenvalue did not
 * converge within 30 n sweeps. Pinned by its residual and by eigenvalues of
 * matrices with known spectrum. */
int orc_schur_qr(int lp, int n, const orc_qc* A, orc_qc* Z, orc_qc* S);

/* Reordering of the start (Section 2.4, the paragraph on the solve of Algorithm 4's loop):
 * the Schur form T = triu(Qh^H A Qh) is reordered by unitary swaps of adjacent
 * diagonal entries so that the eigenvalues appear in increasing order of their
 * projection Re(lambda e^{-i theta}) onto the line with direction e^{i theta}
 * (clustered eigenvalues become neighbours). Swaps follow odd-even transposition
 * order: phase p = 0 .. n-1 swaps every pair (i, i+1), i = p mod 2, whose keys are
 * out of order (keys are computed once, in double, and travel with their
 * entries). A swap of [[a, b], [0, d]] uses the unitary G whose first column is
 * the eigenvector (b, d - a) / r of d. Returns Qout = Qh G_1 G_2 ... and perm[k] =
 * the original diagonal position of the entry now at k. Pinned by the property
 * checks that fix the result independently of the steps: Qout unitary,
 * Qout^H A Qout upper triangular to the start's residual, its diagonal in key
 * order; and the 2 x 2 closed form. */
void orc_reorder(int n, const orc_qc* A, const orc_qc* Qh, double theta, orc_qc* Qout, int* perm);

/* Real Schur variant (Section 3: the method extended to the real Schur form, whose
 * triangular factor has 2 x 2 diagonal blocks holding complex conjugate pairs).
 * Matrices are real: complex records with zero imaginary parts. blk (n ints): blk[i]
 * = 1 when rows and columns i, i + 1 form one 2 x 2 diagonal block, 0 otherwise (NULL:
 * no 2 x 2 blocks). The block strictly lower part of a matrix is every (i, j), i > j,
 * except the subdiagonal entry of a 2 x 2 block.
 *
 * orc_trisolve_real: the block form of the triangular matrix equation, block
 * stril(T L - L T) = -E, for block strictly lower L, in lp (see trisolve_real in
 * oracle_lp.inc). Returns ORC_OK or ORC_BREAKDOWN (a singular small equation: two
 * blocks sharing an eigenvalue, or an invalid marker). Pinned by the scalar solve on
 * 1 x 1 blocks and by exact rational solutions of the full Kronecker system.
 *
 * orc_refine_real: Algorithm 4 with the block strictly lower part as E, the block
 * solve, W = L - L^T and the merged update (the same steps on real data).
 * Pinned by exact real Schur forms with 2 x 2 blocks (the invariant subspaces and
 * the block eigenvalues recovered), the FP32-lp convergence law, and agreement with
 * the complex refinement when every block is 1 x 1.
 *
 * orc_eval_real: orc_eval with the block strictly lower part. */
int orc_trisolve_real(int lp, int n, const int* blk, const orc_qc* T, const orc_qc* E, orc_qc* L);
int orc_refine_real(int lp, int n, const orc_qc* A, const orc_qc* Qh, const int* blk, int maxit, double tol,
                    orc_qc* Qout, orc_qc* Tout, double* hist, int* iters);
void orc_eval_real(int n, const orc_qc* A, const orc_qc* Q, const orc_qc* T, const int* blk, double out[4]);

#ifdef __cplusplus
}
#endif
#endif
