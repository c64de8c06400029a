/*
 * CPU oracle for the A^t A product (packed lower triangle of C = A^t A).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The GPU library shares
 * no code with it.
 *
 * Contents
 *   ora_classical      plain definition: C[i(i+1)/2 + j] = sum_k A[k,i] A[k,j],
 *                      k ascending, one running sum per entry (Section 3:
 *                      the block equations hold because this is the exact
 *                      product; the output is the lower triangle, n(n+1)/2
 *                      entries).
 *   ora_classical_mt   the same definition, tiled over (i, j) and threaded, with
 *                      the identical per-entry k order, so it is bitwise equal
 *                      to ora_classical.  Used as the timed CPU baseline.
 *   ora_ata            the ATA recursion of Algorithm 1 (Section 3), with the
 *                      rectangular Strassen routine HASA for the off-diagonal
 *                      block; counts scalar multiplications and additions.
 *   ora_hasa           HASA alone: D = X Y for X (M x K), Y (K x N), Strassen
 *                      (1969) or Winograd (1971) seven-product recursion with
 *                      zero padding of odd quadrants.
 *   ora_potrf, ora_potrs, ora_atb
 *                      consumers of the product for the normal equations of
 *                      least squares (Section 1): the Cholesky factor of packed
 *                      C, the two triangular solves, and A^t b, each by its
 *                      textbook definition.
 *
 * Build with -O2 -ffp-contract=off: no fused multiply-add, IEEE round to
 * nearest even on every operation, so results are reproducible.
 *
 * Readings of the paper taken here (each listed with its reason in the design
 * notes of the repository):
 *   - the base case "m or n at most the cutoff" is read as m <= c || n <= c;
 *   - the base-case product sums k in ascending order;
 *   - HASA (whose pseudocode the paper cites but does not print) splits each of
 *     M, K, N into ceil/floor halves, treats every smaller quadrant as padded
 *     with zeros to the ceil size, forms seven products recursively and crops;
 *     it stops at min(M, K, N) <= c, and optionally after max_depth levels;
 *   - the Strassen products follow the seven-product listing of the HASA-P
 *     subsection with its first and seventh products corrected to Strassen's
 *     (A11 + A22)(B11 + B22) and (A12 - A22)(B21 + B22): as printed those two
 *     do not reproduce A B with the printed quadrant sums.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>

/* Compile-time mutants.  The test-suite builds the oracle with ORA_MUTANT=k
 * (k >= 1), each planting one plausible mistake, and checks that the pins
 * reject every one of them.  The default build (ORA_MUTANT=0) has none. */
#ifndef ORA_MUTANT
#define ORA_MUTANT 0
#endif
#include <stdlib.h>
#include <string.h>

typedef int64_t i64;

typedef struct {
    i64 mults;      /* scalar multiplications */
    i64 adds;       /* scalar additions/subtractions (matrix sums, assembly) */
    i64 ata_leaves; /* base-case mult() calls of Algorithm 1 */
    i64 hasa_leaves;/* classical products at the bottom of HASA */
    i64 hasa_calls; /* HASA invocations from Algorithm 1 */
    i64 max_hasa_depth;
} ora_counts;

enum { ORA_STRASSEN = 0, ORA_WINOGRAD = 1 };

static inline i64 tri(i64 n) { return n * (n + 1) / 2; }

/* ------------------------------------------------------------------------ */
/* Plain definition                                                          */
/* ------------------------------------------------------------------------ */

void ora_classical(const double *A, i64 m, i64 n, i64 lda, double *C)
{
    for (i64 i = 0; i < n; ++i) {
        for (i64 j = 0; j <= i; ++j) {
            double s = 0.0;
            for (i64 k = (ORA_MUTANT == 8 && m > 1) ? 1 : 0; k < m; ++k)
                s += A[k * lda + i] * A[k * lda + j];
            C[tri(i) + j] = s;
        }
    }
}

/* Threaded, tiled version of the same definition.  Computes packed rows
 * [i0, i1) of C into C_rows (entry (i, j) at tri(i) - tri(i0) + j). */
#define ORA_TB 48

typedef struct {
    const double *A;
    i64 m, n, lda, i0, i1;
    double *C;
    i64 *next_tile; /* shared work counter (row tile index) */
    pthread_mutex_t *mu;
} mt_job;

static void mt_tile(const mt_job *jb, i64 ib0, i64 ib1, i64 jb0, i64 jb1)
{
    double acc[ORA_TB][ORA_TB];
    double ai[ORA_TB], aj[ORA_TB];
    const i64 ni = ib1 - ib0, nj = jb1 - jb0;
    for (i64 a = 0; a < ni; ++a)
        for (i64 b = 0; b < nj; ++b) acc[a][b] = 0.0;
    for (i64 k = 0; k < jb->m; ++k) {
        const double *row = jb->A + k * jb->lda;
        for (i64 a = 0; a < ni; ++a) ai[a] = row[ib0 + a];
        for (i64 b = 0; b < nj; ++b) aj[b] = row[jb0 + b];
        for (i64 a = 0; a < ni; ++a) {
            const double x = ai[a];
            for (i64 b = 0; b < nj; ++b) acc[a][b] += x * aj[b];
        }
    }
    const i64 base = tri(jb->i0);
    for (i64 a = 0; a < ni; ++a) {
        const i64 i = ib0 + a;
        for (i64 b = 0; b < nj; ++b) {
            const i64 j = jb0 + b;
            if (j <= i) jb->C[tri(i) - base + j] = acc[a][b];
        }
    }
}

static void *mt_worker(void *arg)
{
    mt_job *jb = (mt_job *)arg;
    const i64 nrt = (jb->i1 - jb->i0 + ORA_TB - 1) / ORA_TB;
    for (;;) {
        pthread_mutex_lock(jb->mu);
        i64 t = (*jb->next_tile)++;
        pthread_mutex_unlock(jb->mu);
        if (t >= nrt) break;
        /* hand out the longest row tiles first */
        const i64 rt = nrt - 1 - t;
        const i64 ib0 = jb->i0 + rt * ORA_TB;
        i64 ib1 = ib0 + ORA_TB;
        if (ib1 > jb->i1) ib1 = jb->i1;
        for (i64 jb0 = 0; jb0 < ib1; jb0 += ORA_TB) {
            i64 jb1 = jb0 + ORA_TB;
            if (jb1 > ib1) jb1 = ib1;
            mt_tile(jb, ib0, ib1, jb0, jb1);
        }
    }
    return NULL;
}

int ora_classical_mt(const double *A, i64 m, i64 n, i64 lda, i64 i0, i64 i1,
                     double *C_rows, int nthreads)
{
    if (i0 < 0 || i1 > n || i0 > i1 || nthreads < 1) return -1;
    i64 next = 0;
    pthread_mutex_t mu;
    pthread_mutex_init(&mu, NULL);
    mt_job jb = {A, m, n, lda, i0, i1, C_rows, &next, &mu};
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    if (!th) return -2;
    int started = 0;
    for (int t = 0; t < nthreads; ++t)
        if (pthread_create(&th[t], NULL, mt_worker, &jb) == 0) ++started;
    if (started == 0) mt_worker(&jb);
    for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
    free(th);
    pthread_mutex_destroy(&mu);
    return started;
}

/* ------------------------------------------------------------------------ */
/* Dense helpers for the recursion (row-major, explicit leading dimensions)  */
/* ------------------------------------------------------------------------ */

static double *zalloc(i64 count)
{
    if (count <= 0) count = 1;
    return (double *)calloc((size_t)count, sizeof(double));
}

/* Copy the r x c block at src (ld ls) into a zero-padded pr x pc buffer. */
static double *padded_copy(const double *src, i64 ls, i64 r, i64 c, i64 pr, i64 pc)
{
    double *d = zalloc(pr * pc);
    for (i64 i = 0; i < r; ++i)
        for (i64 j = 0; j < c; ++j) d[i * pc + j] = src[i * ls + j];
    return d;
}

/* d = x + s*y elementwise on r x c contiguous buffers (s = +1 or -1). */
static double *msum(const double *x, const double *y, double s, i64 r, i64 c, ora_counts *cnt)
{
    double *d = zalloc(r * c);
    for (i64 t = 0; t < r * c; ++t) d[t] = (s > 0) ? x[t] + y[t] : x[t] - y[t];
    cnt->adds += r * c;
    return d;
}

/* ------------------------------------------------------------------------ */
/* HASA: D (M x N, ld ldd) = X (M x K, ld ldx) * Y (K x N, ld ldy)            */
/* ------------------------------------------------------------------------ */

typedef struct {
    i64 cutoff;
    int variant;
    int max_depth; /* < 0: unlimited */
} ora_cfg;

static void hasa_rec(const double *X, i64 ldx, const double *Y, i64 ldy, i64 M, i64 K, i64 N,
                     double *D, i64 ldd, const ora_cfg *cfg, int depth, ora_counts *cnt)
{
    i64 mn = M < K ? M : K;
    if (N < mn) mn = N;
    if (depth > cnt->max_hasa_depth) cnt->max_hasa_depth = depth;
    if (mn <= cfg->cutoff || (cfg->max_depth >= 0 && depth >= cfg->max_depth)) {
        /* classical product, k ascending */
        for (i64 i = 0; i < M; ++i)
            for (i64 j = 0; j < N; ++j) {
                double s = 0.0;
                for (i64 k = 0; k < K; ++k) s += X[i * ldx + k] * Y[k * ldy + j];
                D[i * ldd + j] = s;
            }
        cnt->mults += M * K * N;
        cnt->hasa_leaves += 1;
        return;
    }
    const i64 M1 = (M + 1) / 2, M2 = M / 2;
    const i64 K1 = (K + 1) / 2, K2 = K / 2;
    const i64 N1 = (N + 1) / 2, N2 = N / 2;
    /* zero-padded quadrants, all M1 x K1 (X) and K1 x N1 (Y) */
    double *X11 = padded_copy(X, ldx, M1, K1, M1, K1);
    double *X12 = padded_copy(X + K1, ldx, M1, K2, M1, K1);
    double *X21 = padded_copy(X + M1 * ldx, ldx, M2, K1, M1, K1);
    double *X22 = padded_copy(X + M1 * ldx + K1, ldx, M2, K2, M1, K1);
    double *Y11 = padded_copy(Y, ldy, K1, N1, K1, N1);
    double *Y12 = padded_copy(Y + N1, ldy, K1, N2, K1, N1);
    double *Y21 = padded_copy(Y + K1 * ldy, ldy, K2, N1, K1, N1);
    double *Y22 = padded_copy(Y + K1 * ldy + N1, ldy, K2, N2, K1, N1);
    const i64 sx = M1 * K1, sy = K1 * N1, sd = M1 * N1;
    double *P[7];
    for (int p = 0; p < 7; ++p) P[p] = zalloc(sd);
    double *D11 = zalloc(sd), *D12 = zalloc(sd), *D21 = zalloc(sd), *D22 = zalloc(sd);
    (void)sx;
    (void)sy;

    if (cfg->variant == ORA_STRASSEN) {
        /* Strassen 1969 */
        double *a, *b;
        a = msum(X11, ORA_MUTANT == 5 ? X12 : X22, +1, M1, K1, cnt);
        b = msum(Y11, Y22, +1, K1, N1, cnt);
        hasa_rec(a, K1, b, N1, M1, K1, N1, P[0], N1, cfg, depth + 1, cnt); free(a); free(b);
        a = msum(X21, X22, +1, M1, K1, cnt);
        hasa_rec(a, K1, Y11, N1, M1, K1, N1, P[1], N1, cfg, depth + 1, cnt); free(a);
        b = msum(Y12, Y22, -1, K1, N1, cnt);
        hasa_rec(X11, K1, b, N1, M1, K1, N1, P[2], N1, cfg, depth + 1, cnt); free(b);
        b = msum(Y21, Y11, -1, K1, N1, cnt);
        hasa_rec(X22, K1, b, N1, M1, K1, N1, P[3], N1, cfg, depth + 1, cnt); free(b);
        a = msum(X11, X12, +1, M1, K1, cnt);
        hasa_rec(a, K1, Y22, N1, M1, K1, N1, P[4], N1, cfg, depth + 1, cnt); free(a);
        a = msum(X21, X11, -1, M1, K1, cnt); b = msum(Y11, Y12, +1, K1, N1, cnt);
        hasa_rec(a, K1, b, N1, M1, K1, N1, P[5], N1, cfg, depth + 1, cnt); free(a); free(b);
        a = msum(ORA_MUTANT == 6 ? X11 : X12, X22, -1, M1, K1, cnt);
        b = msum(Y21, Y22, ORA_MUTANT == 6 ? -1 : +1, K1, N1, cnt);
        hasa_rec(a, K1, b, N1, M1, K1, N1, P[6], N1, cfg, depth + 1, cnt); free(a); free(b);
        /* D11 = M1 + M4 - M5 + M7, D12 = M3 + M5, D21 = M2 + M4,
         * D22 = M1 - M2 + M3 + M6 */
        for (i64 t = 0; t < sd; ++t) {
            D11[t] = ((P[0][t] + P[3][t]) - P[4][t]) + P[6][t];
            D12[t] = P[2][t] + P[4][t];
            D21[t] = P[1][t] + P[3][t];
            D22[t] = ((P[0][t] - (ORA_MUTANT == 2 ? -P[1][t] : P[1][t])) + P[2][t]) + P[5][t];
        }
        cnt->adds += 8 * sd;
    } else {
        /* Winograd 1971: 7 products, 15 additions */
        double *S1 = msum(X21, X22, +1, M1, K1, cnt);
        double *S2 = msum(S1, X11, -1, M1, K1, cnt);
        double *S3 = msum(X11, X21, -1, M1, K1, cnt);
        double *S4 = msum(X12, S2, -1, M1, K1, cnt);
        double *T1 = msum(Y12, Y11, -1, K1, N1, cnt);
        double *T2 = msum(Y22, T1, -1, K1, N1, cnt);
        double *T3 = msum(Y22, Y12, -1, K1, N1, cnt);
        double *T4 = msum(T2, Y21, -1, K1, N1, cnt);
        hasa_rec(X11, K1, Y11, N1, M1, K1, N1, P[0], N1, cfg, depth + 1, cnt);
        hasa_rec(X12, K1, Y21, N1, M1, K1, N1, P[1], N1, cfg, depth + 1, cnt);
        hasa_rec(S4, K1, Y22, N1, M1, K1, N1, P[2], N1, cfg, depth + 1, cnt);
        hasa_rec(X22, K1, T4, N1, M1, K1, N1, P[3], N1, cfg, depth + 1, cnt);
        hasa_rec(S1, K1, T1, N1, M1, K1, N1, P[4], N1, cfg, depth + 1, cnt);
        hasa_rec(S2, K1, T2, N1, M1, K1, N1, P[5], N1, cfg, depth + 1, cnt);
        hasa_rec(S3, K1, T3, N1, M1, K1, N1, P[6], N1, cfg, depth + 1, cnt);
        /* U2 = P1 + P6, U3 = U2 + P7, U4 = U2 + P5;
         * D11 = P1 + P2, D12 = U4 + P3, D21 = U3 - P4, D22 = U3 + P5 */
        for (i64 t = 0; t < sd; ++t) {
            const double u2 = P[0][t] + P[5][t];
            const double u3 = (ORA_MUTANT == 7) ? u2 - P[6][t] : u2 + P[6][t];
            const double u4 = u2 + P[4][t];
            D11[t] = P[0][t] + P[1][t];
            D12[t] = u4 + P[2][t];
            D21[t] = u3 - P[3][t];
            D22[t] = u3 + P[4][t];
        }
        cnt->adds += 7 * sd;
        free(S1); free(S2); free(S3); free(S4);
        free(T1); free(T2); free(T3); free(T4);
    }
    /* crop the padded quadrants into D */
    for (i64 i = 0; i < M1; ++i)
        for (i64 j = 0; j < N1; ++j) D[i * ldd + j] = D11[i * N1 + j];
    for (i64 i = 0; i < M1; ++i)
        for (i64 j = 0; j < N2; ++j) D[i * ldd + N1 + j] = D12[i * N1 + j];
    for (i64 i = 0; i < M2; ++i)
        for (i64 j = 0; j < N1; ++j) D[(M1 + i) * ldd + j] = D21[i * N1 + j];
    for (i64 i = 0; i < M2; ++i)
        for (i64 j = 0; j < N2; ++j) D[(M1 + i) * ldd + N1 + j] = D22[i * N1 + j];

    for (int p = 0; p < 7; ++p) free(P[p]);
    free(D11); free(D12); free(D21); free(D22);
    free(X11); free(X12); free(X21); free(X22);
    free(Y11); free(Y12); free(Y21); free(Y22);
}

void ora_hasa(const double *X, i64 ldx, const double *Y, i64 ldy, i64 M, i64 K, i64 N,
              double *D, i64 ldd, i64 cutoff, int variant, int max_depth, ora_counts *cnt)
{
    ora_cfg cfg = {cutoff, variant, max_depth};
    ora_counts local;
    memset(&local, 0, sizeof local);
    hasa_rec(X, ldx, Y, ldy, M, K, N, D, ldd, &cfg, 0, cnt ? cnt : &local);
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1: ATA                                                          */
/* ------------------------------------------------------------------------ */

/* base case: lower triangle of the block's A^t A, k ascending */
static void mult(const double *A, i64 m, i64 n, i64 lda, double *C, ora_counts *cnt)
{
    ora_classical(A, m, n, lda, C);
    cnt->mults += m * tri(n);
    cnt->ata_leaves += 1;
}

/* Explicit transpose of the r x c block at src (ld ls) into a c x r buffer.
 * Algorithm 1 transposes A12 and A22 before calling HASA. */
static double *transpose(const double *src, i64 ls, i64 r, i64 c)
{
    double *d = zalloc(r * c);
    for (i64 i = 0; i < r; ++i)
        for (i64 j = 0; j < c; ++j) d[j * r + i] = src[i * ls + j];
    return d;
}

static void ata_rec(const double *A, i64 m, i64 n, i64 lda, double *C, const ora_cfg *cfg,
                    ora_counts *cnt)
{
    if (m <= cfg->cutoff || n <= cfg->cutoff) {
        mult(A, m, n, lda, C, cnt);
        return;
    }
    const i64 m1 = (m + 1) / 2, m2 = m / 2, n1 = (n + 1) / 2, n2 = n / 2;
    const double *A11 = A, *A12 = A + n1, *A21 = A + (ORA_MUTANT == 4 ? m2 : m1) * lda,
                 *A22 = A + m1 * lda + n1;
    double *S1 = zalloc(tri(n1)), *S2 = zalloc(tri(n1));
    double *S3 = zalloc(tri(n2)), *S4 = zalloc(tri(n2));
    double *S5 = zalloc(n2 * n1), *S6 = zalloc(n2 * n1);
    ata_rec(A11, m1, n1, lda, S1, cfg, cnt);
    ata_rec(A21, m2, n1, lda, S2, cfg, cnt);
    ata_rec(A12, m1, n2, lda, S3, cfg, cnt);
    ata_rec(A22, m2, n2, lda, S4, cfg, cnt);
    double *T12 = transpose(A12, lda, m1, n2); /* n2 x m1 */
    double *T22 = transpose(A22, lda, m2, n2); /* n2 x m2 */
#if ORA_MUTANT == 3
    if (n1 == n2) {
        double *T11 = transpose(A11, lda, m1, n1);
        hasa_rec(T11, m1, A12, lda, n1, m1, n2, S5, n1, cfg, 0, cnt);
        free(T11);
    } else
#endif
    hasa_rec(T12, m1, A11, lda, n2, m1, n1, S5, n1, cfg, 0, cnt);
    hasa_rec(T22, m2, A21, lda, n2, m2, n1, S6, n1, cfg, 0, cnt);
    cnt->hasa_calls += 2;
    /* C = [[S1 + S2, .], [S5 + S6, S3 + S4]] in packed lower storage */
    for (i64 i = 0; i < n1; ++i)
        for (i64 j = 0; j <= i; ++j)
            C[tri(i) + j] = S1[tri(i) + j] + (ORA_MUTANT == 1 ? 0.0 : S2[tri(i) + j]);
    for (i64 i = 0; i < n2; ++i) {
        const i64 gi = n1 + i;
        for (i64 j = 0; j < n1; ++j) C[tri(gi) + j] = S5[i * n1 + j] + S6[i * n1 + j];
        for (i64 j = 0; j <= i; ++j) C[tri(gi) + n1 + j] = S3[tri(i) + j] + S4[tri(i) + j];
    }
    cnt->adds += tri(n1) + tri(n2) + n1 * n2;
    free(S1); free(S2); free(S3); free(S4); free(S5); free(S6);
    free(T12); free(T22);
}

void ora_ata(const double *A, i64 m, i64 n, i64 lda, double *C, i64 cutoff, int variant,
             int max_depth, ora_counts *cnt)
{
    ora_cfg cfg = {cutoff, variant, max_depth};
    ora_counts local;
    memset(&local, 0, sizeof local);
    ora_counts *c = cnt ? cnt : &local;
    if (n <= 0) return;
    if (m <= 0) {
        for (i64 t = 0; t < tri(n); ++t) C[t] = 0.0;
        return;
    }
    ata_rec(A, m, n, lda, C, &cfg, c);
}

/* Multiplication count of Algorithm 1 without touching data (same recursion
 * as ora_ata).  Used to check closed forms on sizes too large to multiply. */
static i64 hasa_count(i64 M, i64 K, i64 N, const ora_cfg *cfg, int depth)
{
    i64 mn = M < K ? M : K;
    if (N < mn) mn = N;
    if (mn <= cfg->cutoff || (cfg->max_depth >= 0 && depth >= cfg->max_depth)) return M * K * N;
    return 7 * hasa_count((M + 1) / 2, (K + 1) / 2, (N + 1) / 2, cfg, depth + 1);
}

static i64 ata_count(i64 m, i64 n, const ora_cfg *cfg)
{
    if (m <= cfg->cutoff || n <= cfg->cutoff) return m * tri(n);
    const i64 m1 = (m + 1) / 2, m2 = m / 2, n1 = (n + 1) / 2, n2 = n / 2;
    return ata_count(m1, n1, cfg) + ata_count(m2, n1, cfg) + ata_count(m1, n2, cfg) +
           ata_count(m2, n2, cfg) + hasa_count(n2, m1, n1, cfg, 0) + hasa_count(n2, m2, n1, cfg, 0);
}

i64 ora_ata_mult_count(i64 m, i64 n, i64 cutoff, int max_depth)
{
    ora_cfg cfg = {cutoff, ORA_STRASSEN, max_depth};
    if (m <= 0 || n <= 0) return 0;
    return ata_count(m, n, &cfg);
}

/* ------------------------------------------------------------------------
 * Consumers of the product (Section 1 names the normal equations of least
 * squares as a use of A^t A).  Textbook definitions, no blocking.
 * ------------------------------------------------------------------------ */

/* Cholesky factor of the packed lower SPD matrix C, in place, row by row
 * (Cholesky-Banachiewicz): for j < i,
 *   L[i][j] = (C[i][j] - sum_{k<j} L[i][k] L[j][k]) / L[j][j],
 *   L[i][i] = sqrt(C[i][i] - sum_{k<i} L[i][k]^2),
 * each sum taken with k ascending.  Returns 0, or p + 1 for the first row p
 * whose pivot C[p][p] - sum is not positive; the rows from p on are then
 * left as they stand. */
i64 ora_potrf(double *C, i64 n)
{
    for (i64 i = 0; i < n; ++i) {
        double *Li = C + tri(i);
        for (i64 j = 0; j < i; ++j) {
            const double *Lj = C + tri(j);
            double s = 0.0;
            for (i64 k = (ORA_MUTANT == 9 && j > 0) ? 1 : 0; k < j; ++k) s += Li[k] * Lj[k];
            Li[j] = (Li[j] - s) / (ORA_MUTANT == 10 ? Li[i] : Lj[j]);
        }
        double s = 0.0;
        for (i64 k = 0; k < i; ++k) s += Li[k] * Li[k];
        const double d = Li[i] - s;
        if (!(d > 0.0)) return i + 1;
        Li[i] = sqrt(d);
    }
    return 0;
}

/* Solve L L^t X = B in place for the packed lower factor L (n x n) and the
 * row-major n x nrhs right-hand sides B (row stride ldb): forward
 * substitution L Y = B, then back substitution L^t X = Y. */
void ora_potrs(const double *L, i64 n, double *B, i64 nrhs, i64 ldb)
{
    for (i64 r = 0; r < nrhs; ++r) {
        for (i64 i = 0; i < n; ++i) {
            double s = 0.0;
            for (i64 k = 0; k < i; ++k) s += L[tri(i) + k] * B[k * ldb + r];
            B[i * ldb + r] = (B[i * ldb + r] - s) / L[tri(i) + i];
        }
        for (i64 i = n - 1; i >= 0; --i) {
            double s = 0.0;
            for (i64 k = i + 1; k < n; ++k) s += L[tri(k) + i] * B[k * ldb + r];
            const double num = B[i * ldb + r] - s;
            B[i * ldb + r] = ORA_MUTANT == 11 ? num : num / L[tri(i) + i];
        }
    }
}

/* out[j][r] = sum_i A[i][j] B[i][r], i ascending: the right-hand side A^t b
 * of the normal equations (A m x n row stride lda, B m x nrhs row stride ldb,
 * out n x nrhs row stride ldo). */
void ora_atb(const double *A, i64 m, i64 n, i64 lda, const double *B, i64 nrhs, i64 ldb, double *out, i64 ldo)
{
    for (i64 j = 0; j < n; ++j)
        for (i64 r = 0; r < nrhs; ++r) {
            double s = 0.0;
            for (i64 i = (ORA_MUTANT == 12 && m > 1) ? 1 : 0; i < m; ++i) s += A[i * lda + j] * B[i * ldb + r];
            out[j * ldo + r] = s;
        }
}
