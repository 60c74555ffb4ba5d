/*
 * bgu_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, FP64 CPU reference of the Givens bidiagonal update (BGU) of
 * Brust & Saunders, "Fast and Accurate SVD-Type Updating in Streaming Data",
 * Section 3.4 ("Givens Low Rank") and Algorithm 2, together with the dense
 * factorizations used to check it (Householder and Golub-Kahan
 * bidiagonalization of Section 2, one-sided Jacobi singular values).
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  The GPU library shares no code, header,
 * table or helper with it.
 *
 * Conventions: matrices are column-major FP64 with an explicit leading
 * dimension; vectors and matrix indices in comments are 1-based as in the
 * paper, array offsets in code are 0-based.
 */
#ifndef BGU_ORACLE_H
#define BGU_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_ESTRUCT (-10) /* a band/zero-pattern assertion failed */
#define ORC_ESPAN (-11)   /* tracking: r = 1 with b or c in the span of the tracked basis */

/* flags for orc_bgu_pass / orc_bgu_update */
#define ORC_CHECK_PHASES 1 /* assert the zero pattern after each phase */
#define ORC_CHECK_EVERY 2  /* assert the one-bulge invariant after every rotation (tiny n) */
#define ORC_FULL_ROT 4     /* rotate whole rows/columns of the working matrix, not a window */
#define ORC_NO_QP 8        /* do not accumulate into Q and P (schedule/structure studies) */
#define ORC_CHECK_WINDOW 16 /* assert before each rotation that the rotated rows (columns) of
                             * the working matrix are zero outside columns i-1..i+3 (rows
                             * j-2..j+2): the pairs a rotation can change */

/* One recorded rotation: side 0 = left (rows i,i+1 of the working matrix,
 * columns i,i+1 of Q), side 1 = right (columns i,i+1, columns of P).
 * phase: 0 spike, 1 elimination phase, 2 band-to-bidiagonal phase. */
typedef struct {
    int32_t side;
    int32_t phase;
    int64_t i;
    double c;
    double s;
} orc_rot;

/* out[i] = sum_j A(j,i) x[j] accumulated as acc = fma(A(j,i), x[j], acc),
 * j ascending from acc = 0: the projections Q^T b and P^T c of
 * eq. (bidiagsubproblem) in a fixed summation order. */
void orc_project(int64_t rows, int64_t cols, const double *A, int64_t lda,
                 const double *x, double *out);

/* Rotation generator of eq. (giv1): mode 1 annihilates the first entry
 * ([c -s; s c][a;b] = [0;r]), mode 2 annihilates the second
 * ([c -s; s c][a;b] = [r;0]). r = +sqrt(a^2+b^2); identity if the target is 0. */
void orc_givens(double a, double b, int mode, double *c, double *s, double *r);

/* (x, y) <- (c x - s y, s x + c y) evaluated as fma(c,x,-(s*y)), fma(s,x,c*y). */
void orc_rot2(double c, double s, double *x, double *y);

/* One rank-1 BGU pass on the already projected vectors u (length m) and
 * v (length n): Bd + u v^T = Q1 Bd+ P1^T, Q <- Q Q1, P <- P P1
 * (eq. bidiagplus).  d has n entries, e has n-1.  u and v are overwritten.
 * trace (optional, capacity trace_cap) receives every rotation in order;
 * counts (optional, 6 entries) receives
 * {left, right, phase0, phase1, phase2, phase-2 chains that rotate}.
 * Returns ORC_OK, ORC_EINVAL or ORC_ESTRUCT. */
int orc_bgu_pass(int64_t m, int64_t n, double *Q, int64_t ldq, double *d,
                 double *e, double *P, int64_t ldp, double *u, double *v,
                 int flags, orc_rot *trace, int64_t trace_cap, int64_t *counts);

/* The same pass applied to a subset of rows: Q holds qrows rows of the
 * m x m factor (leading dimension ldq >= qrows), P holds prows rows of the
 * n x n factor.  Rotations act on columns, so each row is updated exactly as
 * in the full pass. */
int orc_bgu_pass_rows(int64_t m, int64_t n, double *Q, int64_t qrows,
                      int64_t ldq, double *d, double *e, double *P,
                      int64_t prows, int64_t ldp, double *u, double *v,
                      int flags, orc_rot *trace, int64_t trace_cap,
                      int64_t *counts);

/* Rank-r update A + B C^T (eq. main) as r rank-1 passes (Section 3.2, eq. (rk1)): for
 * column i = 1..r, u = Q^T B(:,i), v = P^T C(:,i) with the current Q, P,
 * then one pass.  B is m x r (ldb), C is n x r (ldc). */
int orc_bgu_update(int64_t m, int64_t n, double *Q, int64_t ldq, double *d,
                   double *e, double *P, int64_t ldp, const double *B,
                   int64_t ldb, const double *C, int64_t ldc, int r, int flags);

/* flags for orc_track_update / orc_track_finish */
#define ORC_TRACK_KEEP_ALL 1 /* both sides augmented: return the rank r+1 factorization */

/* Subspace tracking (Section 4, eqs. (lrup)-(bdlrup)): the thin rank-r
 * factorization A = U B V^T (U m x r, V n x r orthonormal columns, B upper
 * bidiagonal with d (r), e (r-1)) updated with b c^T.
 *
 * orc_track_complement: x_hat = A^T x, x_perp = x - A x_hat, its norm
 * (eq. defup).  Every sum is a sequential fma from 0, rows ascending;
 * (A z)_i = sum_j A(i,j) z_j as fma, j ascending.  With s0 = x^T x and
 * s1 = x_perp^T x_perp: if 2 s1 >= s0 the first pass stands; otherwise one
 * more pass against the same basis (s = A^T x_perp, x_perp <- x_perp - A s,
 * x_hat <- x_hat + s, s2 the new squared norm) and the norm is sqrt(s2) if
 * 2 s2 >= s1, else 0: x lies in span(A) to working precision (the "twice
 * is enough" test of Kahan and Parlett; Parlett, The Symmetric Eigenvalue
 * Problem, section 6-9).  The norm is also 0 when the squared norm it
 * would take is at most (tau ||x||)^2 = tau * tau * s0 with tau = rows *
 * 2^-53 (the worst-case rounding error of the projection sums: such a
 * complement has no meaningful direction).  sums (optional, 3 entries):
 * s0, s1, s2 (-1 without a second pass).
 *
 * orc_track_finish: the rest of the update from given projections b_hat,
 * c_hat (r each), norms delta, gamma >= 0 and unit complements qb =
 * b_perp/delta (m), qc = c_perp/gamma (n; each read only when its norm is
 * positive).  A side with a positive norm is augmented by its complement
 * (eq. qrlr); the middle matrix of eq. (equivlrup) is
 *   both augmented:  [B 0; 0 0] + [b_hat; delta][c_hat; gamma]^T, (r+1)^2;
 *   only the left:   [B; 0] + [b_hat; delta] c_hat^T, (r+1) x r;
 *   only the right:  [B 0] + b_hat [c_hat; gamma]^T, r x (r+1), run as its
 *                    transpose with rows and columns reversed (again upper
 *                    bidiagonal plus rank 1, (r+1) x r);
 *   neither:         B + b_hat c_hat^T, r x r;
 * one BGU pass (orc_bgu_pass, Q = P = I) factors it.  Only when both sides
 * are augmented is the result of rank r+1; unless ORC_TRACK_KEEP_ALL the
 * row and column k of Bbar with the smallest column norm (d_k^2 + e_{k-1}^2
 * as fma(d_k, d_k, e_{k-1}*e_{k-1}); ties: the highest k) are removed and
 * the superdiagonal entry joining k-1 and k+1 is 0.  Otherwise the result
 * is rank r with nothing removed (the paper's unaugmented case).
 * U2(:, j) = [U, qb] Q2(:, keep_j), each entry a sequential fma over U's
 * columns in order and the appended column last (none for an unaugmented
 * side); V2 the same with P2; in the reversed case U2 = U J P3 J and
 * V2 = [V, qc] diag(J,1) Q3(:, 1:r) J (J: reversal of r entries).
 * info (optional, 4 entries): delta, gamma, the removed index (-1 if none),
 * the output rank.  Requires m, n >= r.  Returns ORC_ESPAN, changing no
 * output, when r = 1 and a side is not augmented (no pass on a 2 x 1 or
 * 1 x 1 matrix).
 *
 * orc_track_update: orc_track_complement on both sides, the complements
 * divided by their norms, then orc_track_finish.
 * U2 is m x k, V2 n x k, d2 k entries, e2 k-1, k = r or r+1. */
int orc_track_complement(int64_t rows, int64_t r, const double *A, int64_t lda,
                         const double *x, double *xhat, double *xperp, double *norm,
                         double *sums);
int orc_track_finish(int64_t m, int64_t n, int64_t r, const double *U, int64_t ldu,
                     const double *d, const double *e, const double *V, int64_t ldv,
                     const double *bh, const double *ch, double delta, double gamma,
                     const double *qb, const double *qc, int flags, double *U2,
                     int64_t ldu2, double *d2, double *e2, double *V2, int64_t ldv2,
                     double *info);
int orc_track_update(int64_t m, int64_t n, int64_t r, const double *U, int64_t ldu,
                     const double *d, const double *e, const double *V, int64_t ldv,
                     const double *b, const double *c, int flags, double *U2,
                     int64_t ldu2, double *d2, double *e2, double *V2, int64_t ldv2,
                     double *info);

/* Householder bidiagonalization A = Q B P^T (Section 2, eq. (house)),
 * m >= n >= 1.  Q is m x m, P is n x n (P e1 = e1), d n entries, e n-1. */
int orc_bidiag_householder(int64_t m, int64_t n, const double *A, int64_t lda,
                           double *Q, double *d, double *e, double *P);

/* Golub-Kahan (Lanczos) bidiagonalization from the unit start vector p1
 * (Section 2, recurrences for A P = Q B and A^T Q = P B^T), with full
 * reorthogonalization.  Returns the n diagonal and n-1 superdiagonal
 * entries of B. */
int orc_bidiag_gk(int64_t m, int64_t n, const double *A, int64_t lda,
                  const double *p1, double *d, double *e);

/* Singular values of A (m x n, m >= n) by one-sided Jacobi, descending. */
int orc_jacobi_sv(int64_t m, int64_t n, const double *A, int64_t lda,
                  double *sigma);

/* Test hook: plant a deliberate mistake (0 = none) so the test suite can
 * show that its pins catch it.  See the MUT_* list in bgu_oracle.c. */
void orc_set_mutation(int which);

#ifdef __cplusplus
}
#endif
#endif
