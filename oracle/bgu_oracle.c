/*
 * bgu_oracle.c -- TEST INFRASTRUCTURE ONLY (see bgu_oracle.h).
 *
 * A plain FP64 reference of the Givens bidiagonal update of Brust &
 * Saunders (Section 3.4, Algorithm 2 "BGU"), written for a reader holding the
 * paper.  The working matrix W = Bd is kept dense (N x n, row-major), the
 * rotations are generated and applied one at a time in schedule order, and
 * every rotation is applied to two whole columns of Q or P.  There is no
 * blocking, fusion or reordering.
 *
 * Where the paper leaves the method open, this file takes these readings
 * (each one is restated where it is used):
 *  - Phase 1 (the rotation order of the missing phase-1 figure): for
 *    k = 1..n-1 a right rotation zeroes v_k, then a left rotation zeroes u_k
 *    (k <= N-2); every fill entry outside the band with one sub- and two
 *    superdiagonals is chased up-left through rows and columns whose u, v
 *    entries are already zero.
 *  - The spike for m > n ("reflectors in reverse order") runs first, on
 *    pairs (m-1,m) ... (n+1,n+2); it touches only u and Q.
 *  - The "permutation" for gamma_k != 0, gamma_{k+1} = 0 is the c = 0 case of
 *    the rotation generator (a signed swap, a proper rotation).
 *  - r = +sqrt(fma(a, a, b*b)); the annihilated entry is set to exactly 0 and
 *    the survivor to r; a rotation whose target is already 0 is the identity.
 *  - Phase 2 eliminates, for j = 1..n, the subdiagonal entry (j+1,j) and the
 *    second superdiagonal entry (j,j+2), each followed by a down-right chase;
 *    for m = n this starts the 2n-3 bulge chases the paper counts.
 *  - Rank r is r rank-1 passes, each projecting its column with the current
 *    Q and P (Section 3.2, eq. (rk1), "repeating the process").
 *  - Floating point: explicit fma where written, every other operation
 *    rounded on its own (built with -ffp-contract=off), IEEE sqrt and division.
 */
#include "bgu_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---- deliberate-mistake hook (tests only) ------------------------------- */
enum {
    MUT_NONE = 0,
    MUT_ROT_SIGN = 1,       /* y' = fma(s, x, -(c*y)) */
    MUT_FOLD_DROP = 2,      /* fold forgets the u_N v_n term */
    MUT_CHASE_INDEX = 3,    /* up-left chase steps by 2 instead of 3 */
    MUT_PROJECT_TRANS = 4,  /* project with Q instead of Q^T */
    MUT_Z2_SIGN = 5,        /* mode-2 generator returns s = +b/r */
    MUT_SKIP_Q = 6,         /* left rotations are not accumulated into Q */
    MUT_PHASE2_SKIP_2B = 7, /* phase 2 skips the second-superdiagonal elimination */
    MUT_TRACK_RESID = 8,    /* tracking: b_perp = b + Q1 b_hat */
    MUT_TRACK_NO_DELTA = 9, /* tracking: the middle update vector ends in 0, not delta */
    MUT_TRACK_KEEP = 10,    /* tracking: drops the column of largest norm */
    MUT_TRACK_ONE_PASS = 11,/* tracking: never a second orthogonalization pass */
    MUT_TRACK_FLIP_E = 12   /* tracking, right side only augmented: e not reversed */
};
static int g_mut = MUT_NONE;
void orc_set_mutation(int which) { g_mut = which; }

/* ---- primitives: eq. (giv), (giv1) -------------------------------------- */

void orc_rot2(double c, double s, double *x, double *y)
{
    double x0 = *x, y0 = *y;
    *x = fma(c, x0, -(s * y0));
    if (g_mut == MUT_ROT_SIGN)
        *y = fma(s, x0, -(c * y0));
    else
        *y = fma(s, x0, c * y0);
}

void orc_givens(double a, double b, int mode, double *c, double *s, double *r)
{
    double target = (mode == 1) ? a : b;
    if (target == 0.0) {
        *c = 1.0;
        *s = 0.0;
        *r = (mode == 1) ? b : a;
        return;
    }
    /* Keep a^2 + b^2 inside the exponent range by an exact power-of-two
     * scaling when the larger magnitude is extreme. */
    double big = fabs(a) > fabs(b) ? fabs(a) : fabs(b);
    double sc = 1.0, unsc = 1.0;
    if (big > 0x1p500) {
        sc = 0x1p-600;
        unsc = 0x1p600;
    } else if (big < 0x1p-500) {
        sc = 0x1p600;
        unsc = 0x1p-600;
    }
    double as = a * sc, bs = b * sc;
    double rs = sqrt(fma(as, as, bs * bs));
    if (mode == 1) { /* [c -s; s c][a;b] = [0; r]  ->  c = b/r, s = a/r */
        *c = bs / rs;
        *s = as / rs;
    } else { /* [c -s; s c][a;b] = [r; 0]  ->  c = a/r, s = -b/r */
        *c = as / rs;
        *s = (g_mut == MUT_Z2_SIGN) ? (bs / rs) : -(bs / rs);
    }
    *r = rs * unsc;
}

/* ---- projection: eq. (bidiagsubproblem) --------------------------------- */

void orc_project(int64_t rows, int64_t cols, const double *A, int64_t lda,
                 const double *x, double *out)
{
    for (int64_t i = 0; i < cols; ++i) {
        double acc = 0.0;
        for (int64_t j = 0; j < rows; ++j) {
            double a = (g_mut == MUT_PROJECT_TRANS && j < cols && i < rows)
                           ? A[i + j * lda]
                           : A[j + i * lda];
            acc = fma(a, x[j], acc);
        }
        out[i] = acc;
    }
}

/* ---- the BGU pass ------------------------------------------------------- */

typedef struct {
    int64_t m, n, N;  /* N = n if m == n, else n + 1 (active rows after the spike) */
    double *W;        /* N x n, row-major: W(i,j) = W[(i-1)*n + (j-1)] */
    double *u, *v;    /* u(1..m), v(1..n) stored at u[i-1], v[j-1] */
    double *Q, *P;
    int64_t ldq, ldp;
    int64_t qrows, prows; /* rows of Q and P that are rotated */
    int flags;
    int phase;
    orc_rot *trace;
    int64_t trace_cap, ntrace;
    int64_t cnt[6];
    int bad;          /* set when a structural assertion fails */
} bgu;

#define WEL(S, i, j) ((S)->W[((i) - 1) * (S)->n + ((j) - 1)])

static void record(bgu *S, int side, int64_t i, double c, double s)
{
    if (S->trace && S->ntrace < S->trace_cap) {
        orc_rot *t = &S->trace[S->ntrace];
        t->side = side;
        t->phase = S->phase;
        t->i = i;
        t->c = c;
        t->s = s;
    }
    S->ntrace++;
    S->cnt[side]++;
    S->cnt[2 + S->phase]++;
}

/* Entries outside the band with two subdiagonals and three superdiagonals
 * must always be exactly zero, and at most one entry may sit outside the
 * band with one subdiagonal and two superdiagonals (the bulge). */
static void check_every(bgu *S)
{
    int64_t outside = 0;
    for (int64_t i = 1; i <= S->N; ++i)
        for (int64_t j = 1; j <= S->n; ++j) {
            double w = WEL(S, i, j);
            if (w == 0.0)
                continue;
            int64_t off = j - i;
            if (off < -2 || off > 3)
                S->bad = 1;
            else if (off < -1 || off > 2)
                outside++;
        }
    if (outside > 1)
        S->bad = 1;
}

/* Left(i): rows i, i+1 of W (columns i-2..i+4 hold every nonzero the
 * schedule can create, or all columns with ORC_FULL_ROT), entries i, i+1 of
 * u, and columns i, i+1 of Q: Q <- Q G^T keeps A = Q W P^T. */
static void left(bgu *S, int64_t i, double c, double s)
{
    if ((S->flags & ORC_CHECK_WINDOW) && i + 1 <= S->N)
        for (int64_t j = 1; j <= S->n; ++j)
            if ((j < i - 1 || j > i + 3) && (WEL(S, i, j) != 0.0 || WEL(S, i + 1, j) != 0.0))
                S->bad = 1;
    if (i + 1 <= S->N) {
        int64_t lo = 1, hi = S->n;
        if (!(S->flags & ORC_FULL_ROT)) {
            lo = i - 2 > 1 ? i - 2 : 1;
            hi = i + 4 < S->n ? i + 4 : S->n;
        }
        for (int64_t j = lo; j <= hi; ++j)
            orc_rot2(c, s, &WEL(S, i, j), &WEL(S, i + 1, j));
    }
    orc_rot2(c, s, &S->u[i - 1], &S->u[i]);
    if (!(S->flags & ORC_NO_QP) && g_mut != MUT_SKIP_Q) {
        double *qi = S->Q + (i - 1) * S->ldq, *qj = S->Q + i * S->ldq;
        for (int64_t r = 0; r < S->qrows; ++r)
            orc_rot2(c, s, &qi[r], &qj[r]);
    }
    record(S, 0, i, c, s);
}

/* Right(j): columns j, j+1 of W (rows j-3..j+3, or all rows), entries
 * j, j+1 of v, and columns j, j+1 of P: P <- P G keeps A = Q W P^T. */
static void right(bgu *S, int64_t j, double c, double s)
{
    if (S->flags & ORC_CHECK_WINDOW)
        for (int64_t i = 1; i <= S->N; ++i)
            if ((i < j - 2 || i > j + 2) && (WEL(S, i, j) != 0.0 || WEL(S, i, j + 1) != 0.0))
                S->bad = 1;
    int64_t lo = 1, hi = S->N;
    if (!(S->flags & ORC_FULL_ROT)) {
        lo = j - 3 > 1 ? j - 3 : 1;
        hi = j + 3 < S->N ? j + 3 : S->N;
    }
    for (int64_t i = lo; i <= hi; ++i)
        orc_rot2(c, s, &WEL(S, i, j), &WEL(S, i, j + 1));
    orc_rot2(c, s, &S->v[j - 1], &S->v[j]);
    if (!(S->flags & ORC_NO_QP)) {
        double *pi = S->P + (j - 1) * S->ldp, *pj = S->P + j * S->ldp;
        for (int64_t r = 0; r < S->prows; ++r)
            orc_rot2(c, s, &pi[r], &pj[r]);
    }
    record(S, 1, j, c, s);
}

/* Generate from the pair (*x, *y) in the given mode, apply it as a left
 * (side 0) or right (side 1) rotation with first index i, then set the
 * annihilated entry to exactly 0 and the survivor to r. */
static void zap(bgu *S, int side, int64_t i, double *x, double *y, int mode)
{
    double c, s, r;
    orc_givens(*x, *y, mode, &c, &s, &r);
    if (side == 0)
        left(S, i, c, s);
    else
        right(S, i, c, s);
    if (mode == 1) {
        *x = 0.0;
        *y = r;
    } else {
        *x = r;
        *y = 0.0;
    }
    if (S->flags & ORC_CHECK_EVERY)
        check_every(S);
}

/* Phase 1, up-left chase of a fill entry at (i, i+3): a left rotation on
 * rows i, i+1 removes it and creates (i+1, i-1); a right rotation on
 * columns i-1, i removes that and creates (i-3, i); repeat from i-3.  Every
 * row and column touched here has u and v already zero, so those zeros
 * survive. */
static void chase_up_q3(bgu *S, int64_t i)
{
    int64_t step = (g_mut == MUT_CHASE_INDEX) ? 2 : 3;
    while (i >= 1) {
        zap(S, 0, i, &WEL(S, i, i + 3), &WEL(S, i + 1, i + 3), 1);
        if (i == 1)
            break;
        zap(S, 1, i - 1, &WEL(S, i + 1, i - 1), &WEL(S, i + 1, i), 1);
        i -= step;
    }
}

/* Phase 1, fill entry at (i, i-2) left by the left rotation that zeroed
 * u_{i-1}: a right rotation on columns i-2, i-1 removes it and creates
 * (i-4, i-1), which chase_up_q3 continues. */
static void chase_up_p2(bgu *S, int64_t i)
{
    if (i - 2 < 1)
        return;
    zap(S, 1, i - 2, &WEL(S, i, i - 2), &WEL(S, i, i - 1), 1);
    chase_up_q3(S, i - 4);
}

/* Phase 2, down-right chase: the caller's left rotation on rows i, i+1 has
 * just created the fill entry (i, i+3).  A right rotation on columns i+2,
 * i+3 removes it and creates (i+4, i+2) below the subdiagonal; a left
 * rotation on rows i+3, i+4 removes that and creates (i+3, i+6); repeat
 * until the bulge leaves the matrix. */
static void chase_down_q3(bgu *S, int64_t i)
{
    while (i + 3 <= S->n) {
        zap(S, 1, i + 2, &WEL(S, i, i + 2), &WEL(S, i, i + 3), 2);
        if (i + 4 > S->N)
            break;
        zap(S, 0, i + 3, &WEL(S, i + 3, i + 2), &WEL(S, i + 4, i + 2), 2);
        i += 3;
    }
}

static int band_ok(bgu *S, int64_t lo_off, int64_t hi_off)
{
    for (int64_t i = 1; i <= S->N; ++i)
        for (int64_t j = 1; j <= S->n; ++j) {
            int64_t off = j - i;
            if ((off < lo_off || off > hi_off) && WEL(S, i, j) != 0.0)
                return 0;
        }
    return 1;
}

int orc_bgu_pass(int64_t m, int64_t n, double *Q, int64_t ldq, double *d,
                 double *e, double *P, int64_t ldp, double *u, double *v,
                 int flags, orc_rot *trace, int64_t trace_cap, int64_t *counts)
{
    if (ldq < m || ldp < n)
        return ORC_EINVAL;
    return orc_bgu_pass_rows(m, n, Q, m, ldq, d, e, P, n, ldp, u, v, flags,
                             trace, trace_cap, counts);
}

int orc_bgu_pass_rows(int64_t m, int64_t n, double *Q, int64_t qrows,
                      int64_t ldq, double *d, double *e, double *P,
                      int64_t prows, int64_t ldp, double *u, double *v,
                      int flags, orc_rot *trace, int64_t trace_cap,
                      int64_t *counts)
{
    if (m < n || n < 2 || qrows < 0 || prows < 0 || ldq < qrows ||
        ldp < prows || !d || !e || !u || !v)
        return ORC_EINVAL;
    if (!(flags & ORC_NO_QP) && (!Q || !P))
        return ORC_EINVAL;
    bgu S;
    memset(&S, 0, sizeof S);
    S.m = m;
    S.n = n;
    S.N = (m == n) ? n : n + 1;
    S.u = u;
    S.v = v;
    S.Q = Q;
    S.P = P;
    S.ldq = ldq;
    S.ldp = ldp;
    S.qrows = qrows;
    S.prows = prows;
    S.flags = flags;
    S.trace = trace;
    S.trace_cap = trace_cap;
    S.W = (double *)calloc((size_t)(S.N * n), sizeof(double));
    if (!S.W)
        return ORC_ENOMEM;
    for (int64_t i = 1; i <= n; ++i)
        WEL(&S, i, i) = d[i - 1];
    for (int64_t i = 1; i < n; ++i)
        WEL(&S, i, i + 1) = e[i - 1];

    /* Phase 0, the spike (m > n): rotations on u entries (j-1, j) for
     * j = m..n+2 fold u(n+1:m) into u(n+1).  Rows beyond n of Bd are zero,
     * so only u and Q change. */
    S.phase = 0;
    for (int64_t j = m; j >= n + 2; --j)
        zap(&S, 0, j - 1, &S.u[j - 2], &S.u[j - 1], 2);

    /* Phase 1: alternate eliminations in v and u, keeping W banded. */
    S.phase = 1;
    for (int64_t k = 1; k <= n - 1; ++k) {
        /* right rotation on columns k, k+1 zeroes v_k; fill at (k-2, k+1) */
        zap(&S, 1, k, &S.v[k - 1], &S.v[k], 1);
        if (k >= 3)
            chase_up_q3(&S, k - 2);
        /* left rotation on rows k, k+1 zeroes u_k; fill at (k+1, k-1) */
        if (k <= S.N - 2) {
            zap(&S, 0, k, &S.u[k - 1], &S.u[k], 1);
            if (k >= 2)
                chase_up_p2(&S, k + 1);
        }
    }
    if (flags & ORC_CHECK_PHASES) {
        if (!band_ok(&S, -1, 2))
            S.bad = 1;
        for (int64_t i = 1; i <= S.N - 2; ++i)
            if (S.u[i - 1] != 0.0)
                S.bad = 1;
        for (int64_t j = 1; j <= n - 1; ++j)
            if (S.v[j - 1] != 0.0)
                S.bad = 1;
        for (int64_t i = S.N + 1; i <= m; ++i)
            if (S.u[i - 1] != 0.0)
                S.bad = 1;
    }

    /* Fold: u v^T now only touches column n, rows N-1 and N. */
    {
        int64_t N = S.N;
        WEL(&S, N - 1, n) = fma(S.u[N - 2], S.v[n - 1], WEL(&S, N - 1, n));
        if (g_mut != MUT_FOLD_DROP)
            WEL(&S, N, n) = fma(S.u[N - 1], S.v[n - 1], WEL(&S, N, n));
        for (int64_t i = 0; i < m; ++i)
            S.u[i] = 0.0;
        for (int64_t j = 0; j < n; ++j)
            S.v[j] = 0.0;
    }

    /* Phase 2: band (one sub-, two superdiagonals) to upper bidiagonal. */
    S.phase = 2;
    for (int64_t j = 1; j <= n; ++j) {
        int64_t before = S.cnt[4];
        if (j + 1 <= S.N) {
            zap(&S, 0, j, &WEL(&S, j, j), &WEL(&S, j + 1, j), 2);
            chase_down_q3(&S, j);
        }
        int64_t mid = S.cnt[4];
        if (j + 2 <= n && g_mut != MUT_PHASE2_SKIP_2B) {
            zap(&S, 1, j + 1, &WEL(&S, j, j + 1), &WEL(&S, j, j + 2), 2);
            if (j + 3 <= S.N) {
                zap(&S, 0, j + 2, &WEL(&S, j + 2, j + 1), &WEL(&S, j + 3, j + 1), 2);
                chase_down_q3(&S, j + 2);
            }
        }
        S.cnt[5] += (mid > before) + (S.cnt[4] > mid);
    }
    if ((flags & (ORC_CHECK_PHASES | ORC_CHECK_EVERY)) && !band_ok(&S, 0, 1))
        S.bad = 1;

    for (int64_t i = 1; i <= n; ++i)
        d[i - 1] = WEL(&S, i, i);
    for (int64_t i = 1; i < n; ++i)
        e[i - 1] = WEL(&S, i, i + 1);
    free(S.W);
    if (counts)
        memcpy(counts, S.cnt, sizeof S.cnt);
    return S.bad ? ORC_ESTRUCT : ORC_OK;
}

int orc_bgu_update(int64_t m, int64_t n, double *Q, int64_t ldq, double *d,
                   double *e, double *P, int64_t ldp, const double *B,
                   int64_t ldb, const double *C, int64_t ldc, int r, int flags)
{
    if (m < n || n < 2 || r < 1 || !Q || !P || !B || !C || ldb < m || ldc < n)
        return ORC_EINVAL;
    double *u = (double *)malloc(sizeof(double) * (size_t)m);
    double *v = (double *)malloc(sizeof(double) * (size_t)n);
    if (!u || !v) {
        free(u);
        free(v);
        return ORC_ENOMEM;
    }
    int st = ORC_OK;
    for (int i = 0; i < r && st == ORC_OK; ++i) {
        orc_project(m, m, Q, ldq, B + (int64_t)i * ldb, u);
        orc_project(n, n, P, ldp, C + (int64_t)i * ldc, v);
        st = orc_bgu_pass(m, n, Q, ldq, d, e, P, ldp, u, v, flags & ~ORC_NO_QP,
                          NULL, 0, NULL);
    }
    free(u);
    free(v);
    return st;
}

/* ---- subspace tracking: Section 4, eqs. (lrup)-(bdlrup) ----------------- */

/* a^T b over rows entries: a sequential fma from 0, rows ascending. */
static double plain_dot(int64_t rows, const double *a, const double *b)
{
    double p = 0.0;
    for (int64_t i = 0; i < rows; ++i)
        p = fma(a[i], b[i], p);
    return p;
}

/* y = x - A z with (A z)_i = sum_j A(i,j) z_j as fma, j ascending from 0. */
static void minus_span(int64_t rows, int64_t r, const double *A, int64_t lda,
                       const double *x, const double *z, double *y)
{
    for (int64_t i = 0; i < rows; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < r; ++j)
            s = fma(A[i + j * lda], z[j], s);
        y[i] = (g_mut == MUT_TRACK_RESID) ? x[i] + s : x[i] - s;
    }
}

int orc_track_complement(int64_t rows, int64_t r, const double *A, int64_t lda,
                         const double *x, double *xhat, double *xperp, double *norm,
                         double *sums)
{
    if (rows < 1 || r < 1 || lda < rows || !A || !x || !xhat || !xperp || !norm)
        return ORC_EINVAL;
    double *s = (double *)malloc(sizeof(double) * (size_t)r);
    double *y = (double *)malloc(sizeof(double) * (size_t)rows);
    if (!s || !y) {
        free(s);
        free(y);
        return ORC_ENOMEM;
    }
    /* first pass (eq. defup) */
    for (int64_t j = 0; j < r; ++j)
        xhat[j] = plain_dot(rows, A + j * lda, x);
    minus_span(rows, r, A, lda, x, xhat, xperp);
    const double s0 = plain_dot(rows, x, x);
    const double s1 = plain_dot(rows, xperp, xperp);
    double s2 = -1.0;
    /* a complement no larger than the worst-case rounding error of the
     * projection sums, rows * 2^-53 * ||x||, carries no direction */
    const double tau = (double)rows * 0x1p-53;
    const double floor2 = tau * tau * s0;
    if (2.0 * s1 >= s0 || g_mut == MUT_TRACK_ONE_PASS) {
        *norm = s1 > floor2 ? sqrt(s1) : 0.0;
    } else {
        /* second pass against the same basis ("twice is enough") */
        for (int64_t j = 0; j < r; ++j)
            s[j] = plain_dot(rows, A + j * lda, xperp);
        minus_span(rows, r, A, lda, xperp, s, y);
        for (int64_t j = 0; j < r; ++j)
            xhat[j] = xhat[j] + s[j];
        s2 = plain_dot(rows, y, y);
        for (int64_t i = 0; i < rows; ++i)
            xperp[i] = y[i];
        *norm = (s2 > floor2 && 2.0 * s2 >= s1) ? sqrt(s2) : 0.0;
    }
    if (sums) {
        sums[0] = s0;
        sums[1] = s1;
        sums[2] = s2;
    }
    free(s);
    free(y);
    return ORC_OK;
}

/* out(:, j) = sum_l A(:, l) M(rmap(l), cmap(j)) over l = 0..r-1 (fma, l
 * ascending), then + w M(r, cmap(j)) when w is given.  rmap is the
 * identity, or l -> r-1-l when rev; cmap is j -> keep[j]. */
static void track_product(int64_t rows, int64_t r, const double *A, int64_t lda,
                          const double *w, const double *M, int64_t ldm, int rev,
                          const int64_t *keep, int64_t ncols, double *out, int64_t ldo)
{
    for (int64_t j = 0; j < ncols; ++j) {
        const double *mc = M + keep[j] * ldm;
        for (int64_t i = 0; i < rows; ++i) {
            double acc = 0.0;
            for (int64_t l = 0; l < r; ++l)
                acc = fma(A[i + l * lda], mc[rev ? r - 1 - l : l], acc);
            out[i + j * ldo] = w ? fma(w[i], mc[r], acc) : acc;
        }
    }
}

int orc_track_finish(int64_t m, int64_t n, int64_t r, const double *U, int64_t ldu,
                     const double *d, const double *e, const double *V, int64_t ldv,
                     const double *bh, const double *ch, double delta, double gamma,
                     const double *qb, const double *qc, int flags, double *U2,
                     int64_t ldu2, double *d2, double *e2, double *V2, int64_t ldv2,
                     double *info)
{
    const int keep_all = (flags & ORC_TRACK_KEEP_ALL) != 0;
    const int ab = delta > 0.0, ac = gamma > 0.0;
    if (r < 1 || m < r || n < r || ldu < m || ldv < n || ldu2 < m || ldv2 < n || !U || !d ||
        !V || !bh || !ch || !U2 || !d2 || !V2 || (r > 1 && !e) || (ab && !qb) || (ac && !qc) ||
        !(delta >= 0.0) || !(gamma >= 0.0) || (((r > 1) || (keep_all && ab && ac)) && !e2))
        return ORC_EINVAL;
    if ((!ab || !ac) && r < 2)
        return ORC_ESPAN; /* a 1 x 1 or 2 x 1 middle matrix has no BGU pass */
    const int64_t R = r + 1;
    const int64_t mm = ab ? R : r, mn = ac ? R : r; /* middle matrix mm x mn */
    /* the BGU pass runs on a tall or square matrix: the wide case (left
     * side not augmented, right side augmented) runs on its transpose with
     * rows and columns reversed, which is again upper bidiagonal plus a
     * rank-1 term */
    const int flip = !ab && ac;
    const int64_t pm = flip ? R : mm, pn = flip ? r : mn;
    double *Qm = (double *)calloc((size_t)(pm * pm), sizeof(double));
    double *Pm = (double *)calloc((size_t)(pn * pn), sizeof(double));
    double *dm = (double *)calloc((size_t)R, sizeof(double));
    double *em = (double *)calloc((size_t)R, sizeof(double));
    double *u = (double *)calloc((size_t)R, sizeof(double));
    double *v = (double *)calloc((size_t)R, sizeof(double));
    int64_t *keep = (int64_t *)malloc(sizeof(int64_t) * (size_t)R);
    int st = ORC_OK;
    if (!Qm || !Pm || !dm || !em || !u || !v || !keep) {
        st = ORC_ENOMEM;
        goto out;
    }
    for (int64_t i = 0; i < pm; ++i)
        Qm[i + i * pm] = 1.0;
    for (int64_t i = 0; i < pn; ++i)
        Pm[i + i * pn] = 1.0;
    if (!flip) {
        /* eq. (equivlrup): [B 0; 0 0] + [b_hat; delta][c_hat; gamma]^T, the
         * row (column) of the unaugmented side left out */
        for (int64_t i = 0; i < r; ++i) {
            dm[i] = d[i];
            u[i] = bh[i];
            v[i] = ch[i];
        }
        for (int64_t i = 0; i + 1 < r; ++i)
            em[i] = e[i];
        if (ab)
            u[r] = (g_mut == MUT_TRACK_NO_DELTA) ? 0.0 : delta;
        if (ac)
            v[r] = gamma;
    } else {
        /* M = [B 0] + b_hat [c_hat; gamma]^T (r x (r+1)); with J the
         * reversal of r entries, M^T = diag(J, 1) ([J B^T J; 0] + [J c_hat;
         * gamma] (J b_hat)^T) J and J B^T J is upper bidiagonal with d and e
         * reversed */
        for (int64_t i = 0; i < r; ++i) {
            dm[i] = d[r - 1 - i];
            u[i] = ch[r - 1 - i];
            v[i] = bh[r - 1 - i];
        }
        for (int64_t i = 0; i + 1 < r; ++i)
            em[i] = (g_mut == MUT_TRACK_FLIP_E) ? e[i] : e[r - 2 - i];
        u[r] = gamma;
    }
    st = orc_bgu_pass(pm, pn, Qm, pm, dm, em, Pm, pn, u, v, 0, NULL, 0, NULL);
    if (st != ORC_OK)
        goto out;
    int64_t kdrop = -1, nk = 0;
    if (ab && ac && !keep_all) {
        /* truncation: drop the row and column of smallest column norm
         * (squared norm d_k^2 + e_{k-1}^2 as fma(d_k, d_k, e_{k-1} * e_{k-1}));
         * ties drop the highest index */
        kdrop = R - 1;
        double best = fma(dm[R - 1], dm[R - 1], em[R - 2] * em[R - 2]);
        for (int64_t k = R - 2; k >= 0; --k) {
            double nk2 = (k == 0) ? dm[0] * dm[0] : fma(dm[k], dm[k], em[k - 1] * em[k - 1]);
            if (g_mut == MUT_TRACK_KEEP ? nk2 > best : nk2 < best) {
                best = nk2;
                kdrop = k;
            }
        }
    }
    const int64_t full = (ab && ac) ? R : r; /* columns of the updated bidiagonal */
    for (int64_t k = 0; k < full; ++k)
        if (k != kdrop)
            keep[nk++] = k;
    if (!flip) {
        for (int64_t j = 0; j < nk; ++j)
            d2[j] = dm[keep[j]];
        for (int64_t j = 0; j + 1 < nk; ++j)
            e2[j] = (keep[j + 1] == keep[j] + 1) ? em[keep[j]] : 0.0;
        /* eq. (bdlrup): the thin factors [U, b_perp/delta] Q2(:, keep) and
         * [V, c_perp/gamma] P2(:, keep); an unaugmented side has no
         * appended column */
        track_product(m, r, U, ldu, ab ? qb : NULL, Qm, pm, 0, keep, nk, U2, ldu2);
        track_product(n, r, V, ldv, ac ? qc : NULL, Pm, pn, 0, keep, nk, V2, ldv2);
    } else {
        /* the pass gave M^T = diag(J,1) Q3 [Bbar; 0] P3^T J, so
         * M = (J P3 J) (J Bbar^T J) (diag(J,1) Q3(:, 1:r) J)^T with
         * J Bbar^T J upper bidiagonal: d, e reversed back, U2 = U J P3 J,
         * V2 = [V, c_perp/gamma] diag(J,1) Q3(:, 1:r) J */
        for (int64_t j = 0; j < r; ++j) {
            d2[j] = dm[r - 1 - j];
            keep[j] = r - 1 - j;
        }
        for (int64_t j = 0; j + 1 < r; ++j)
            e2[j] = em[r - 2 - j];
        track_product(m, r, U, ldu, NULL, Pm, pn, 1, keep, r, U2, ldu2);
        track_product(n, r, V, ldv, qc, Qm, pm, 1, keep, r, V2, ldv2);
    }
    if (info) {
        info[0] = delta;
        info[1] = gamma;
        info[2] = (double)kdrop;
        info[3] = (double)nk;
    }
out:
    free(Qm);
    free(Pm);
    free(dm);
    free(em);
    free(u);
    free(v);
    free(keep);
    return st;
}

int orc_track_update(int64_t m, int64_t n, int64_t r, const double *U, int64_t ldu,
                     const double *d, const double *e, const double *V, int64_t ldv,
                     const double *b, const double *c, int flags, double *U2,
                     int64_t ldu2, double *d2, double *e2, double *V2, int64_t ldv2,
                     double *info)
{
    if (r < 1 || m < r || n < r || ldu < m || ldv < n || !U || !V || !b || !c)
        return ORC_EINVAL;
    double *bh = (double *)calloc((size_t)r, sizeof(double));
    double *ch = (double *)calloc((size_t)r, sizeof(double));
    double *bp = (double *)malloc(sizeof(double) * (size_t)m);
    double *cp = (double *)malloc(sizeof(double) * (size_t)n);
    int st = ORC_OK;
    double delta = 0.0, gamma = 0.0;
    if (!bh || !ch || !bp || !cp) {
        st = ORC_ENOMEM;
        goto out;
    }
    /* eq. (defup): projections onto the tracked bases and their complements */
    st = orc_track_complement(m, r, U, ldu, b, bh, bp, &delta, NULL);
    if (st == ORC_OK)
        st = orc_track_complement(n, r, V, ldv, c, ch, cp, &gamma, NULL);
    if (st != ORC_OK)
        goto out;
    /* eq. (qrlr): the appended columns b_perp / delta and c_perp / gamma */
    if (delta > 0.0)
        for (int64_t i = 0; i < m; ++i)
            bp[i] = bp[i] / delta;
    if (gamma > 0.0)
        for (int64_t i = 0; i < n; ++i)
            cp[i] = cp[i] / gamma;
    st = orc_track_finish(m, n, r, U, ldu, d, e, V, ldv, bh, ch, delta, gamma, bp, cp, flags,
                          U2, ldu2, d2, e2, V2, ldv2, info);
out:
    free(bh);
    free(ch);
    free(bp);
    free(cp);
    return st;
}

/* ---- dense checks: Section 2 -------------------------------------------- */

/* Householder vector for x (length len): on return x holds v with v_1 = 1
 * scaled, *beta = 2 / (v^T v), and the return value is the new leading entry
 * alpha = -sign(x_1) ||x|| (H x = alpha e1, H = I - beta v v^T). */
static double house(int64_t len, double *x, double *beta)
{
    double nrm2 = 0.0;
    for (int64_t k = 0; k < len; ++k)
        nrm2 += x[k] * x[k];
    double nrm = sqrt(nrm2);
    if (nrm == 0.0) {
        *beta = 0.0;
        return 0.0;
    }
    double alpha = (x[0] >= 0.0) ? -nrm : nrm;
    x[0] -= alpha;
    double vtv = 0.0;
    for (int64_t k = 0; k < len; ++k)
        vtv += x[k] * x[k];
    *beta = (vtv == 0.0) ? 0.0 : 2.0 / vtv;
    return alpha;
}

int orc_bidiag_householder(int64_t m, int64_t n, const double *A, int64_t lda,
                           double *Q, double *d, double *e, double *P)
{
    if (m < n || n < 1 || lda < m)
        return ORC_EINVAL;
    double *R = (double *)malloc(sizeof(double) * (size_t)(m * n));
    double *x = (double *)malloc(sizeof(double) * (size_t)(m > n ? m : n));
    if (!R || !x) {
        free(R);
        free(x);
        return ORC_ENOMEM;
    }
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i)
            R[i + j * m] = A[i + j * lda];
    for (int64_t j = 0; j < m; ++j)
        for (int64_t i = 0; i < m; ++i)
            Q[i + j * m] = (i == j);
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i)
            P[i + j * n] = (i == j);

    for (int64_t k = 0; k < n; ++k) {
        /* left reflector on rows k..m-1 zeroes R(k+1:m, k) */
        int64_t len = m - k;
        double beta;
        for (int64_t t = 0; t < len; ++t)
            x[t] = R[k + t + k * m];
        double alpha = house(len, x, &beta);
        if (beta != 0.0) {
            for (int64_t j = k; j < n; ++j) {
                double w = 0.0;
                for (int64_t t = 0; t < len; ++t)
                    w += x[t] * R[k + t + j * m];
                w *= beta;
                for (int64_t t = 0; t < len; ++t)
                    R[k + t + j * m] -= w * x[t];
            }
            for (int64_t i = 0; i < m; ++i) { /* Q <- Q H */
                double w = 0.0;
                for (int64_t t = 0; t < len; ++t)
                    w += Q[i + (k + t) * m] * x[t];
                w *= beta;
                for (int64_t t = 0; t < len; ++t)
                    Q[i + (k + t) * m] -= w * x[t];
            }
            R[k + k * m] = alpha;
            for (int64_t t = 1; t < len; ++t)
                R[k + t + k * m] = 0.0;
        }
        d[k] = R[k + k * m];
        if (k + 1 >= n)
            break;
        /* right reflector on columns k+1..n-1 zeroes R(k, k+2:n) */
        len = n - k - 1;
        for (int64_t t = 0; t < len; ++t)
            x[t] = R[k + (k + 1 + t) * m];
        alpha = house(len, x, &beta);
        if (beta != 0.0) {
            for (int64_t i = k; i < m; ++i) {
                double w = 0.0;
                for (int64_t t = 0; t < len; ++t)
                    w += R[i + (k + 1 + t) * m] * x[t];
                w *= beta;
                for (int64_t t = 0; t < len; ++t)
                    R[i + (k + 1 + t) * m] -= w * x[t];
            }
            for (int64_t i = 0; i < n; ++i) { /* P <- P G */
                double w = 0.0;
                for (int64_t t = 0; t < len; ++t)
                    w += P[i + (k + 1 + t) * n] * x[t];
                w *= beta;
                for (int64_t t = 0; t < len; ++t)
                    P[i + (k + 1 + t) * n] -= w * x[t];
            }
            R[k + (k + 1) * m] = alpha;
            for (int64_t t = 1; t < len; ++t)
                R[k + (k + 1 + t) * m] = 0.0;
        }
        e[k] = R[k + (k + 1) * m];
    }
    free(R);
    free(x);
    return ORC_OK;
}

int orc_bidiag_gk(int64_t m, int64_t n, const double *A, int64_t lda,
                  const double *p1, double *d, double *e)
{
    if (m < n || n < 1 || lda < m)
        return ORC_EINVAL;
    double *Pv = (double *)calloc((size_t)(n * n), sizeof(double));
    double *Qv = (double *)calloc((size_t)(m * n), sizeof(double));
    double *w = (double *)malloc(sizeof(double) * (size_t)(m > n ? m : n));
    if (!Pv || !Qv || !w) {
        free(Pv);
        free(Qv);
        free(w);
        return ORC_ENOMEM;
    }
    for (int64_t i = 0; i < n; ++i)
        Pv[i] = p1[i];
    for (int64_t k = 0; k < n; ++k) {
        /* q_k = A p_k - beta_{k-1} q_{k-1}, reorthogonalized, alpha_k = ||q_k|| */
        double *pk = Pv + k * n, *qk = Qv + k * m;
        for (int64_t i = 0; i < m; ++i) {
            double s = 0.0;
            for (int64_t j = 0; j < n; ++j)
                s += A[i + j * lda] * pk[j];
            w[i] = s;
        }
        for (int pass = 0; pass < 2; ++pass)
            for (int64_t t = 0; t < k; ++t) {
                double *qt = Qv + t * m, h = 0.0;
                for (int64_t i = 0; i < m; ++i)
                    h += qt[i] * w[i];
                for (int64_t i = 0; i < m; ++i)
                    w[i] -= h * qt[i];
            }
        double a = 0.0;
        for (int64_t i = 0; i < m; ++i)
            a += w[i] * w[i];
        a = sqrt(a);
        d[k] = a;
        for (int64_t i = 0; i < m; ++i)
            qk[i] = (a != 0.0) ? w[i] / a : 0.0;
        if (k + 1 >= n)
            break;
        /* p_{k+1} = A^T q_k - alpha_k p_k, reorthogonalized, beta_k = ||p_{k+1}|| */
        for (int64_t j = 0; j < n; ++j) {
            double s = 0.0;
            for (int64_t i = 0; i < m; ++i)
                s += A[i + j * lda] * qk[i];
            w[j] = s;
        }
        for (int pass = 0; pass < 2; ++pass)
            for (int64_t t = 0; t <= k; ++t) {
                double *pt = Pv + t * n, h = 0.0;
                for (int64_t j = 0; j < n; ++j)
                    h += pt[j] * w[j];
                for (int64_t j = 0; j < n; ++j)
                    w[j] -= h * pt[j];
            }
        double b = 0.0;
        for (int64_t j = 0; j < n; ++j)
            b += w[j] * w[j];
        b = sqrt(b);
        e[k] = b;
        for (int64_t j = 0; j < n; ++j)
            Pv[(k + 1) * n + j] = (b != 0.0) ? w[j] / b : 0.0;
    }
    free(Pv);
    free(Qv);
    free(w);
    return ORC_OK;
}

static int cmp_desc(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x < y) - (x > y);
}

int orc_jacobi_sv(int64_t m, int64_t n, const double *A, int64_t lda,
                  double *sigma)
{
    if (m < n || n < 1 || lda < m)
        return ORC_EINVAL;
    double *U = (double *)malloc(sizeof(double) * (size_t)(m * n));
    if (!U)
        return ORC_ENOMEM;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i)
            U[i + j * m] = A[i + j * lda];
    const double tol = 1e-15;
    for (int sweep = 0; sweep < 60; ++sweep) {
        int rotated = 0;
        for (int64_t p = 0; p < n - 1; ++p)
            for (int64_t q = p + 1; q < n; ++q) {
                double *up = U + p * m, *uq = U + q * m;
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int64_t i = 0; i < m; ++i) {
                    al += up[i] * up[i];
                    be += uq[i] * uq[i];
                    ga += up[i] * uq[i];
                }
                if (ga == 0.0 || fabs(ga) <= tol * sqrt(al * be))
                    continue;
                rotated = 1;
                double zeta = (be - al) / (2.0 * ga);
                double t = (zeta >= 0.0 ? 1.0 : -1.0) /
                           (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
                for (int64_t i = 0; i < m; ++i) {
                    double x = up[i], y = uq[i];
                    up[i] = c * x - s * y;
                    uq[i] = s * x + c * y;
                }
            }
        if (!rotated)
            break;
    }
    for (int64_t j = 0; j < n; ++j) {
        double s = 0.0;
        for (int64_t i = 0; i < m; ++i)
            s += U[i + j * m] * U[i + j * m];
        sigma[j] = sqrt(s);
    }
    qsort(sigma, (size_t)n, sizeof(double), cmp_desc);
    free(U);
    return ORC_OK;
}
