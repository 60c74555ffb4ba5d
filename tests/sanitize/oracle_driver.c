/* Runs the oracle's C entry points on small inputs under the sanitizers:
 * Householder and Golub-Kahan bidiagonalization, one-sided Jacobi, rank-r
 * updates (m = n and m > n), single passes with a short trace and counts,
 * row-subset passes, and the tracking update with both, one and neither
 * side augmented.  Each result is checked against a plain property so
 * that the runs mean something; exit status 0 when every check holds. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/bgu_oracle.h"

static int g_fail = 0;
#define CHECK(c)                                                             \
    do {                                                                     \
        if (!(c)) {                                                          \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++g_fail;                                                        \
        }                                                                    \
    } while (0)

static uint64_t g_state = 88172645463325252ull;
static double rnd(void) /* xorshift64, uniform on (-1, 1) */
{
    g_state ^= g_state << 13;
    g_state ^= g_state >> 7;
    g_state ^= g_state << 17;
    return (double)(g_state >> 11) * 0x1p-52 - 1.0;
}

static double *fill(int64_t k)
{
    double *x = malloc(sizeof(double) * (size_t)(k > 0 ? k : 1));
    for (int64_t i = 0; i < k; ++i) x[i] = rnd();
    return x;
}

/* ||A - Q [diag(d) + superdiag(e); 0] P^T||_F with Q m x m, P n x n */
static double recon(int64_t m, int64_t n, const double *A, const double *Q, const double *d, const double *e,
                    const double *P)
{
    double err = 0.0;
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) {
            double s = 0.0;
            for (int64_t k = 0; k < n; ++k) {
                double qb = Q[i + k * m] * d[k] + (k > 0 ? Q[i + (k - 1) * m] * e[k - 1] : 0.0);
                s += qb * P[j + k * n];
            }
            err += (A[i + j * m] - s) * (A[i + j * m] - s);
        }
    return sqrt(err);
}

static void updates(int64_t m, int64_t n)
{
    double *A = fill(m * n), *Q = calloc((size_t)(m * m), 8), *P = calloc((size_t)(n * n), 8);
    double *d = calloc((size_t)n, 8), *e = calloc((size_t)n, 8);
    CHECK(orc_bidiag_householder(m, n, A, m, Q, d, e, P) == 0);
    CHECK(recon(m, n, A, Q, d, e, P) < 1e-12);
    const int r = 3;
    double *B = fill(m * r), *C = fill(n * r);
    CHECK(orc_bgu_update(m, n, Q, m, d, e, P, n, B, m, C, n, r, 0) == 0);
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j)
            for (int k = 0; k < r; ++k) A[i + j * m] += B[i + k * m] * C[j + k * n];
    CHECK(recon(m, n, A, Q, d, e, P) < 1e-11);
    /* one pass with a trace shorter than the pass, and the counts */
    double *u = fill(m), *v = fill(n);
    orc_rot tr[5];
    int64_t counts[6];
    CHECK(orc_bgu_pass(m, n, Q, m, d, e, P, n, u, v, 0, tr, 5, counts) == 0);
    CHECK(counts[0] + counts[1] >= 5 && tr[0].c * tr[0].c + tr[0].s * tr[0].s > 0.99);
    /* a pass on two rows of Q and one row of P equals those rows of a full pass */
    double *Q2 = malloc(sizeof(double) * (size_t)(m * m)), *P2 = malloc(sizeof(double) * (size_t)(n * n));
    double *d2 = malloc(sizeof(double) * (size_t)n), *e2 = malloc(sizeof(double) * (size_t)n);
    memcpy(Q2, Q, sizeof(double) * (size_t)(m * m));
    memcpy(P2, P, sizeof(double) * (size_t)(n * n));
    memcpy(d2, d, sizeof(double) * (size_t)n);
    memcpy(e2, e, sizeof(double) * (size_t)n);
    double *ur = fill(m), *vr = fill(n);
    double *u2 = malloc(sizeof(double) * (size_t)m), *v2 = malloc(sizeof(double) * (size_t)n);
    memcpy(u2, ur, sizeof(double) * (size_t)m);
    memcpy(v2, vr, sizeof(double) * (size_t)n);
    double Qs[2 * 64], Ps[64];
    for (int64_t j = 0; j < m; ++j) {
        Qs[0 + 2 * j] = Q[0 + j * m];
        Qs[1 + 2 * j] = Q[(m - 1) + j * m];
    }
    for (int64_t j = 0; j < n; ++j) Ps[j] = P[1 + j * n];
    CHECK(orc_bgu_pass_rows(m, n, Qs, 2, 2, d, e, Ps, 1, 1, ur, vr, 0, NULL, 0, NULL) == 0);
    CHECK(orc_bgu_pass(m, n, Q2, m, d2, e2, P2, n, u2, v2, 0, NULL, 0, NULL) == 0);
    for (int64_t j = 0; j < m; ++j) CHECK(Qs[2 * j] == Q2[j * m] && Qs[1 + 2 * j] == Q2[(m - 1) + j * m]);
    for (int64_t j = 0; j < n; ++j) CHECK(Ps[j] == P2[1 + j * n]);
    for (int64_t j = 0; j < n; ++j) CHECK(d[j] == d2[j]);
    /* bad arguments are refused */
    CHECK(orc_bgu_pass(n, m + 1, Q, m, d, e, P, n, u, v, 0, NULL, 0, NULL) != 0);
    free(A), free(Q), free(P), free(d), free(e), free(B), free(C), free(u), free(v);
    free(Q2), free(P2), free(d2), free(e2), free(ur), free(vr), free(u2), free(v2);
}

static void dense(void)
{
    const int64_t m = 12, n = 7;
    double *A = fill(m * n), *d = calloc((size_t)n, 8), *e = calloc((size_t)n, 8), *sv = calloc((size_t)n, 8);
    double *p1 = calloc((size_t)n, 8);
    p1[0] = 1.0;
    CHECK(orc_bidiag_gk(m, n, A, m, p1, d, e) == 0);
    CHECK(orc_jacobi_sv(m, n, A, m, sv) == 0);
    double fa = 0.0, fb = 0.0, fs = 0.0;
    for (int64_t i = 0; i < m * n; ++i) fa += A[i] * A[i];
    for (int64_t i = 0; i < n; ++i) fb += d[i] * d[i] + (i + 1 < n ? e[i] * e[i] : 0.0);
    for (int64_t i = 0; i < n; ++i) fs += sv[i] * sv[i];
    CHECK(fabs(fa - fb) < 1e-12 * fa && fabs(fa - fs) < 1e-12 * fa);
    for (int64_t i = 1; i < n; ++i) CHECK(sv[i] <= sv[i - 1]);
    free(A), free(d), free(e), free(sv), free(p1);
}

static void tracking(void)
{
    const int64_t m = 14, n = 10, r = 4;
    /* U = first r columns of I_m, V = first r columns of I_n */
    double *U = calloc((size_t)(m * r), 8), *V = calloc((size_t)(n * r), 8);
    for (int64_t j = 0; j < r; ++j) {
        U[j + j * m] = 1.0;
        V[j + j * n] = 1.0;
    }
    double d[4] = {4, 3, 2, 1}, e[3] = {0.5, 0.25, 0.125};
    double *U2 = calloc((size_t)(m * (r + 1)), 8), *V2 = calloc((size_t)(n * (r + 1)), 8);
    double d2[5], e2[5], info[4];
    double *b = fill(m), *c = fill(n);
    CHECK(orc_track_update(m, n, r, U, m, d, e, V, n, b, c, 0, U2, m, d2, e2, V2, n, info) == 0);
    CHECK(info[0] > 0 && info[1] > 0 && info[2] >= 0 && info[3] == r);
    CHECK(orc_track_update(m, n, r, U, m, d, e, V, n, b, c, ORC_TRACK_KEEP_ALL, U2, m, d2, e2, V2, n, info) == 0);
    CHECK(info[3] == r + 1);
    /* b in span(U): the left side is not augmented; both in span: neither */
    double bs[14] = {0}, cs[10] = {0};
    bs[1] = 2.0;
    cs[2] = -1.0;
    CHECK(orc_track_update(m, n, r, U, m, d, e, V, n, bs, c, 0, U2, m, d2, e2, V2, n, info) == 0);
    CHECK(info[0] == 0.0 && info[1] > 0 && info[2] == -1);
    CHECK(orc_track_update(m, n, r, U, m, d, e, V, n, b, cs, 0, U2, m, d2, e2, V2, n, info) == 0);
    CHECK(info[1] == 0.0 && info[2] == -1);
    CHECK(orc_track_update(m, n, r, U, m, d, e, V, n, bs, cs, 0, U2, m, d2, e2, V2, n, info) == 0);
    CHECK(info[0] == 0.0 && info[1] == 0.0);
    /* U2^T U2 = I */
    for (int64_t i = 0; i < r; ++i)
        for (int64_t j = 0; j < r; ++j) {
            double s = 0.0;
            for (int64_t k = 0; k < m; ++k) s += U2[k + i * m] * U2[k + j * m];
            CHECK(fabs(s - (i == j)) < 1e-13);
        }
    free(U), free(V), free(U2), free(V2), free(b), free(c);
}

int main(void)
{
    updates(6, 6);
    updates(9, 5);
    updates(33, 20);
    dense();
    tracking();
    if (g_fail) {
        fprintf(stderr, "%d checks failed\n", g_fail);
        return 1;
    }
    printf("oracle: all checks passed\n");
    return 0;
}
