/*
 * ht_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, sequential CPU reference for the reduction of an
 * r-Hessenberg-triangular pencil (H,T) to Hessenberg-triangular form
 * (Steel & Vandebril, "Parallel two-stage reduction to Hessenberg-triangular
 * form", Section 3.1 and the unblocked stage-two algorithm of the appendix),
 * plus the stage-one reduction of a dense pencil to r-Hessenberg-triangular
 * form (Section 2.2 and the blocked stage-one algorithm of the appendix).
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no code, header or constant with
 * the HIP implementation.  Everything is fp64 (complex: pairs of fp64), column
 * major, element (i,j) (0-based) at p[i + j*ld].  Build with FMA contraction
 * disabled (-ffp-contract=off) so that results are reproducible.
 *
 * Conventions (the paper is silent on them; the readings are listed in the
 * design notes):
 *   - Householder reflectors follow LAPACK's xLARFG: G = I - tau v v^H with
 *     v(0) = 1, G^H x = beta e0, beta real, beta = -sgn(Re x0) ||x||,
 *     sgn(+0) = sgn(-0) = +1, tau = 0 when x(1:) = 0 and Im x0 = 0.
 *   - Left updates use G^H (X <- G^H X), accumulation is Q <- Q G, so that
 *     the input pencil equals Q (H,T) Z^H on exit.
 *   - The opposite (right) reflector is built from the first row of the
 *     orthogonal RQ factor of the diagonal block of T.  That row is fixed only
 *     up to a unimodular scalar, so its direction y is normalised to make the
 *     first nonzero entry real and positive before xLARFG is applied to it.
 *   - Entries annihilated by a reflector are written as exact zeros.
 *
 * Threads: oracle_set_threads(t) lets the reflector applications split their
 * independent columns (left updates) or rows (right updates) over t OpenMP
 * threads.  Every entry then sees exactly the operation sequence of the
 * one-thread run, so the results are bitwise equal for any t (a test checks
 * this); the default is one thread.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { double re, im; } zdbl;

#ifdef _OPENMP
#include <omp.h>
#endif

static int g_threads = 1;
/* minimum number of independent vectors before a reflector application is
 * split over threads */
#define PAR_MIN 512

void oracle_set_threads(int t) { g_threads = t < 1 ? 1 : t; }
int oracle_get_threads(void) { return g_threads; }

/* ---------- explicit complex arithmetic (no reliance on C complex rules) -- */
static zdbl zmk(double re, double im) { zdbl z; z.re = re; z.im = im; return z; }
static zdbl zadd(zdbl a, zdbl b) { return zmk(a.re + b.re, a.im + b.im); }
static zdbl zsub(zdbl a, zdbl b) { return zmk(a.re - b.re, a.im - b.im); }
static zdbl zmul(zdbl a, zdbl b) { return zmk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re); }
static zdbl zconj(zdbl a) { return zmk(a.re, -a.im); }
/* conj(a) * b, the term of a Hermitian inner product */
static zdbl zcmul(zdbl a, zdbl b) { return zmk(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re); }
/* 1 / (c + i d) by Smith's method */
static zdbl zrecip(zdbl z) {
    double c = z.re, d = z.im;
    if (fabs(c) >= fabs(d)) {
        double e = d / c, f = c + d * e;
        return zmk((1.0 + 0.0 * e) / f, (0.0 - 1.0 * e) / f);
    } else {
        double e = c / d, f = d + c * e;
        return zmk((1.0 * e + 0.0) / f, (0.0 * e - 1.0) / f);
    }
}

static double sgn_re(double a) { return a >= 0.0 ? 1.0 : -1.0; }

/* ------------------------------------------------------------------------ */
/* Householder generation, LAPACK xLARFG convention.  x has m-1 entries.     */
/* On exit *alpha = beta, x = v(1:m-1).                                      */
/* ------------------------------------------------------------------------ */
void oracle_larfg_d(int64_t m, double *alpha, double *x, double *tau)
{
    if (m <= 1) { *tau = 0.0; return; }
    double ss = 0.0;
    for (int64_t i = 0; i < m - 1; ++i) ss += x[i] * x[i];
    if (ss == 0.0) { *tau = 0.0; return; }
    double a = *alpha;
    double beta = -sgn_re(a) * sqrt(a * a + ss);
    *tau = (beta - a) / beta;
    double scal = 1.0 / (a - beta);
    for (int64_t i = 0; i < m - 1; ++i) x[i] = x[i] * scal;
    *alpha = beta;
}

void oracle_larfg_z(int64_t m, zdbl *alpha, zdbl *x, zdbl *tau)
{
    if (m <= 1 && alpha->im == 0.0) { *tau = zmk(0.0, 0.0); return; }
    double ss = 0.0;
    for (int64_t i = 0; i < m - 1; ++i) ss += x[i].re * x[i].re + x[i].im * x[i].im;
    zdbl a = *alpha;
    if (ss == 0.0 && a.im == 0.0) { *tau = zmk(0.0, 0.0); return; }
    double beta = -sgn_re(a.re) * sqrt((a.re * a.re + a.im * a.im) + ss);
    *tau = zmk((beta - a.re) / beta, -a.im / beta);
    zdbl scal = zrecip(zsub(a, zmk(beta, 0.0)));
    for (int64_t i = 0; i < m - 1; ++i) x[i] = zmul(x[i], scal);
    *alpha = zmk(beta, 0.0);
}

/* ------------------------------------------------------------------------ */
/* Direction of the first row of the orthogonal factor of an RQ              */
/* factorisation B = R Qt (B is m x m, copied, not modified).                */
/* y = conj(Qt(0,:))^T, normalised so that its first nonzero entry is real   */
/* and positive.  Householder RQ, last row first: for row i a reflector U_i  */
/* acting on columns 0..i maps B(i,0:i) to a multiple of e_i; then           */
/* B Ut = R with Ut = U_{m-1} ... U_1, Qt = Ut^H and y = Ut e0.              */
/* ------------------------------------------------------------------------ */
int oracle_rq_dir_d(int64_t m, const double *B, int64_t ldb, double *y)
{
    double *W = (double *)malloc(sizeof(double) * m * m);
    double *U = (double *)malloc(sizeof(double) * m * m);   /* reflector vectors, col i for row i */
    double *tu = (double *)malloc(sizeof(double) * m);
    double *b = (double *)malloc(sizeof(double) * m);
    if (!W || !U || !tu || !b) { free(W); free(U); free(tu); free(b); return -1; }
    for (int64_t c = 0; c < m; ++c)
        for (int64_t i = 0; i < m; ++i) W[i + c * m] = B[i + c * ldb];
    for (int64_t i = m - 1; i >= 1; --i) {
        /* b = row i, columns 0..i; alpha = b[i], x = b[0..i-1] */
        for (int64_t c = 0; c <= i; ++c) b[c] = W[i + c * m];
        double alpha = b[i], tau;
        oracle_larfg_d(i + 1, &alpha, b, &tau);
        double *u = U + i * m;
        for (int64_t c = 0; c < i; ++c) u[c] = b[c];
        u[i] = 1.0;
        tu[i] = tau;
        /* rows 0..i-1:  W(r, 0:i) -= tau * (W(r,0:i) u) u^T */
        for (int64_t rr = 0; rr < i; ++rr) {
            double s = 0.0;
            for (int64_t c = 0; c <= i; ++c) s += W[rr + c * m] * u[c];
            s *= tau;
            for (int64_t c = 0; c <= i; ++c) W[rr + c * m] -= s * u[c];
        }
    }
    for (int64_t c = 0; c < m; ++c) y[c] = 0.0;
    y[0] = 1.0;
    for (int64_t i = 1; i < m; ++i) {          /* y <- U_i y, U_1 first */
        double *u = U + i * m;
        double s = 0.0;
        for (int64_t c = 0; c <= i; ++c) s += u[c] * y[c];
        s *= tu[i];
        for (int64_t c = 0; c <= i; ++c) y[c] -= s * u[c];
    }
    int64_t p = 0;
    while (p < m && y[p] == 0.0) ++p;
    if (p < m && y[p] < 0.0)
        for (int64_t c = 0; c < m; ++c) y[c] = -y[c];
    free(W); free(U); free(tu); free(b);
    return 0;
}

int oracle_rq_dir_z(int64_t m, const zdbl *B, int64_t ldb, zdbl *y)
{
    zdbl *W = (zdbl *)malloc(sizeof(zdbl) * m * m);
    zdbl *U = (zdbl *)malloc(sizeof(zdbl) * m * m);
    zdbl *tu = (zdbl *)malloc(sizeof(zdbl) * m);
    zdbl *b = (zdbl *)malloc(sizeof(zdbl) * m);
    if (!W || !U || !tu || !b) { free(W); free(U); free(tu); free(b); return -1; }
    for (int64_t c = 0; c < m; ++c)
        for (int64_t i = 0; i < m; ++i) W[i + c * m] = B[i + c * ldb];
    for (int64_t i = m - 1; i >= 1; --i) {
        /* b = conj(row i)^T, columns 0..i; U^H b = beta e_i  <=>  row_i U = beta e_i^T */
        for (int64_t c = 0; c <= i; ++c) b[c] = zconj(W[i + c * m]);
        zdbl alpha = b[i], tau;
        oracle_larfg_z(i + 1, &alpha, b, &tau);
        zdbl *u = U + i * m;
        for (int64_t c = 0; c < i; ++c) u[c] = b[c];
        u[i] = zmk(1.0, 0.0);
        tu[i] = tau;
        /* rows 0..i-1:  W(r,0:i) <- W(r,0:i) (I - tau u u^H) */
        for (int64_t rr = 0; rr < i; ++rr) {
            zdbl s = zmk(0.0, 0.0);
            for (int64_t c = 0; c <= i; ++c) s = zadd(s, zmul(W[rr + c * m], u[c]));
            s = zmul(s, tau);
            for (int64_t c = 0; c <= i; ++c) W[rr + c * m] = zsub(W[rr + c * m], zmul(s, zconj(u[c])));
        }
    }
    for (int64_t c = 0; c < m; ++c) y[c] = zmk(0.0, 0.0);
    y[0] = zmk(1.0, 0.0);
    for (int64_t i = 1; i < m; ++i) {          /* y <- U_i y */
        zdbl *u = U + i * m;
        zdbl s = zmk(0.0, 0.0);
        for (int64_t c = 0; c <= i; ++c) s = zadd(s, zcmul(u[c], y[c]));
        s = zmul(s, tu[i]);
        for (int64_t c = 0; c <= i; ++c) y[c] = zsub(y[c], zmul(s, u[c]));
    }
    int64_t p = 0;
    while (p < m && y[p].re == 0.0 && y[p].im == 0.0) ++p;
    if (p < m) {
        double a = sqrt(y[p].re * y[p].re + y[p].im * y[p].im);
        zdbl ph = zmk(y[p].re / a, -y[p].im / a);      /* conj(y_p)/|y_p| */
        for (int64_t c = 0; c < m; ++c) y[c] = zmul(y[c], ph);
        y[p].im = 0.0;
    }
    free(W); free(U); free(tu); free(b);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Reflector application kernels (plain loops).                              */
/* ------------------------------------------------------------------------ */
/* X(rows a..a+m-1, cols c0..c1) <- (I - tau v v^T) X : left, real */
static void left_d(double *X, int64_t ld, int64_t a, int64_t m, int64_t c0, int64_t c1,
                   const double *v, double tau)
{
    if (tau == 0.0) return;
#pragma omp parallel for schedule(static) num_threads(g_threads) if (g_threads > 1 && c1 - c0 + 1 >= PAR_MIN)
    for (int64_t c = c0; c <= c1; ++c) {
        double *col = X + a + c * ld;
        double s = 0.0;
        for (int64_t i = 0; i < m; ++i) s += v[i] * col[i];
        s *= tau;
        for (int64_t i = 0; i < m; ++i) col[i] -= s * v[i];
    }
}
/* X(rows r0..r1, cols a..a+m-1) <- X (I - tau v v^T) : right, real */
static void right_d(double *X, int64_t ld, int64_t a, int64_t m, int64_t r0, int64_t r1,
                    const double *v, double tau)
{
    if (tau == 0.0 || r1 < r0) return;
    int64_t nr = r1 - r0 + 1;
    double *s = (double *)calloc((size_t)nr, sizeof(double));
    /* rows are independent: each chunk of rows runs the same column loops */
#pragma omp parallel for schedule(static) num_threads(g_threads) if (g_threads > 1 && nr >= PAR_MIN)
    for (int64_t i0 = 0; i0 < nr; i0 += 256) {
        int64_t ie = i0 + 256 < nr ? i0 + 256 : nr;
        for (int64_t j = 0; j < m; ++j) {
            const double *col = X + r0 + (a + j) * ld;
            for (int64_t i = i0; i < ie; ++i) s[i] += col[i] * v[j];
        }
        for (int64_t j = 0; j < m; ++j) {
            double *col = X + r0 + (a + j) * ld;
            double tv = tau * v[j];
            for (int64_t i = i0; i < ie; ++i) col[i] -= s[i] * tv;
        }
    }
    free(s);
}
/* complex: left uses G^H = I - conj(tau) v v^H */
static void left_z(zdbl *X, int64_t ld, int64_t a, int64_t m, int64_t c0, int64_t c1,
                   const zdbl *v, zdbl tau)
{
    if (tau.re == 0.0 && tau.im == 0.0) return;
    zdbl ct = zconj(tau);
#pragma omp parallel for schedule(static) num_threads(g_threads) if (g_threads > 1 && c1 - c0 + 1 >= PAR_MIN)
    for (int64_t c = c0; c <= c1; ++c) {
        zdbl *col = X + a + c * ld;
        zdbl s = zmk(0.0, 0.0);
        for (int64_t i = 0; i < m; ++i) s = zadd(s, zcmul(v[i], col[i]));
        s = zmul(ct, s);
        for (int64_t i = 0; i < m; ++i) col[i] = zsub(col[i], zmul(s, v[i]));
    }
}
/* complex: right uses G = I - tau v v^H:  X <- X - tau (X v) v^H */
static void right_z(zdbl *X, int64_t ld, int64_t a, int64_t m, int64_t r0, int64_t r1,
                    const zdbl *v, zdbl tau)
{
    if ((tau.re == 0.0 && tau.im == 0.0) || r1 < r0) return;
    int64_t nr = r1 - r0 + 1;
    zdbl *s = (zdbl *)calloc((size_t)nr, sizeof(zdbl));
#pragma omp parallel for schedule(static) num_threads(g_threads) if (g_threads > 1 && nr >= PAR_MIN)
    for (int64_t i0 = 0; i0 < nr; i0 += 256) {
        int64_t ie = i0 + 256 < nr ? i0 + 256 : nr;
        for (int64_t j = 0; j < m; ++j) {
            const zdbl *col = X + r0 + (a + j) * ld;
            for (int64_t i = i0; i < ie; ++i) s[i] = zadd(s[i], zmul(col[i], v[j]));
        }
        for (int64_t j = 0; j < m; ++j) {
            zdbl *col = X + r0 + (a + j) * ld;
            zdbl tv = zmul(tau, zconj(v[j]));
            for (int64_t i = i0; i < ie; ++i) col[i] = zsub(col[i], zmul(s[i], tv));
        }
    }
    free(s);
}

/* ------------------------------------------------------------------------ */
/* Stage two (unblocked algorithm of the appendix; Section 3.1).             */
/* 1-based index map of the paper, for sweep j = 1..n-2 and block k:         */
/*   n_blocks = 1 + floor((n-j-2)/r), jb = j + max(0,(k-1)r+1),              */
/*   i1 = j+kr+1, i2 = min(j+(k+1)r,n), i3 = min(j+(k+2)r,n).                */
/* Runs sweeps 1..jmax (jmax < 0: all).  Q, Z may be NULL.  Adds the number  */
/* of counted flops (4 * reflector length * vectors updated per reflector    */
/* application over the ranges the algorithm states, the left reflector on   */
/* H(i1:i2, jb:n) including the column it reduces; complex x4) to *flops     */
/* when flops != NULL.                                                       */
/* Entries outside the r-HT pattern are not read: they are overwritten by 0. */
/* ------------------------------------------------------------------------ */
static void zero_outside_d(int64_t n, int64_t r, double *H, double *T, int64_t ld)
{
    for (int64_t c = 0; c < n; ++c) {
        for (int64_t i = c + r + 1; i < n; ++i) H[i + c * ld] = 0.0;
        for (int64_t i = c + 1; i < n; ++i) T[i + c * ld] = 0.0;
    }
}
static void zero_final_d(int64_t n, double *H, double *T, int64_t ld)
{
    for (int64_t c = 0; c < n; ++c) {
        for (int64_t i = c + 2; i < n; ++i) H[i + c * ld] = 0.0;
        for (int64_t i = c + 1; i < n; ++i) T[i + c * ld] = 0.0;
    }
}
static void zero_outside_z(int64_t n, int64_t r, zdbl *H, zdbl *T, int64_t ld)
{
    for (int64_t c = 0; c < n; ++c) {
        for (int64_t i = c + r + 1; i < n; ++i) H[i + c * ld] = zmk(0.0, 0.0);
        for (int64_t i = c + 1; i < n; ++i) T[i + c * ld] = zmk(0.0, 0.0);
    }
}
static void zero_final_z(int64_t n, zdbl *H, zdbl *T, int64_t ld)
{
    for (int64_t c = 0; c < n; ++c) {
        for (int64_t i = c + 2; i < n; ++i) H[i + c * ld] = zmk(0.0, 0.0);
        for (int64_t i = c + 1; i < n; ++i) T[i + c * ld] = zmk(0.0, 0.0);
    }
}

int oracle_stage2_d(int64_t n, int64_t r, double *H, double *T, double *Q, double *Z,
                    int64_t ld, int64_t jmax, double *flops)
{
    if (n < 0) return -1;
    if (r < 1) return -2;
    if (ld < (n > 1 ? n : 1)) return -3;
    if (n == 0) return 0;
    zero_outside_d(n, r, H, T, ld);
    double *v = (double *)malloc(sizeof(double) * (size_t)(r + 1));
    double *w = (double *)malloc(sizeof(double) * (size_t)(r + 1));
    double *blk = (double *)malloc(sizeof(double) * (size_t)(r * r));
    if (!v || !w || !blk) { free(v); free(w); free(blk); return 1; }
    double fl = 0.0;
    int64_t jlast = (jmax < 0 || jmax > n - 2) ? n - 2 : jmax;
    for (int64_t j = 1; j <= jlast; ++j) {                       /* 1-based sweep index */
        int64_t nblocks = 1 + (n - j - 2) / r;
        for (int64_t k = 0; k < nblocks; ++k) {
            int64_t jb = j + ((k - 1) * r + 1 > 0 ? (k - 1) * r + 1 : 0);
            int64_t i1 = j + k * r + 1;
            int64_t i2 = j + (k + 1) * r < n ? j + (k + 1) * r : n;
            int64_t i3 = j + (k + 2) * r < n ? j + (k + 2) * r : n;
            int64_t m = i2 - i1 + 1;
            int64_t a = i1 - 1, cb = jb - 1;                    /* 0-based */
            /* left reflector reducing H(i1:i2, jb) */
            double alpha = H[a + cb * ld], tau;
            for (int64_t i = 1; i < m; ++i) v[i] = H[a + i + cb * ld];
            oracle_larfg_d(m, &alpha, v + 1, &tau);
            v[0] = 1.0;
            H[a + cb * ld] = alpha;
            for (int64_t i = 1; i < m; ++i) H[a + i + cb * ld] = 0.0;
            left_d(H, ld, a, m, cb + 1, n - 1, v, tau);          /* H <- G^H H */
            left_d(T, ld, a, m, a, n - 1, v, tau);               /* T <- G^H T */
            fl += 4.0 * m * (double)(n - jb + 1) + 4.0 * m * (double)(n - i1 + 1);
            if (Q) { right_d(Q, ld, a, m, 0, n - 1, v, tau); fl += 4.0 * m * n; }   /* Q <- Q G */
            /* opposite reflector from the RQ factorisation of T(i1:i2, i1:i2) */
            for (int64_t c = 0; c < m; ++c)
                for (int64_t i = 0; i < m; ++i) blk[i + c * m] = T[a + i + (a + c) * ld];
            if (oracle_rq_dir_d(m, blk, m, w) != 0) { free(v); free(w); free(blk); return 1; }
            double al2 = w[0], sig;
            oracle_larfg_d(m, &al2, w + 1, &sig);
            w[0] = 1.0;
            right_d(H, ld, a, m, 0, i3 - 1, w, sig);             /* H <- H W */
            right_d(T, ld, a, m, 0, i2 - 1, w, sig);             /* T <- T W */
            for (int64_t i = 1; i < m; ++i) T[a + i + a * ld] = 0.0;
            fl += 4.0 * m * (double)i3 + 4.0 * m * (double)i2;
            if (Z) { right_d(Z, ld, a, m, 0, n - 1, w, sig); fl += 4.0 * m * n; }  /* Z <- Z W */
        }
    }
    if (jlast == n - 2 || n <= 2) zero_final_d(n, H, T, ld);
    if (flops) *flops += fl;
    free(v); free(w); free(blk);
    return 0;
}

int oracle_stage2_z(int64_t n, int64_t r, zdbl *H, zdbl *T, zdbl *Q, zdbl *Z,
                    int64_t ld, int64_t jmax, double *flops)
{
    if (n < 0) return -1;
    if (r < 1) return -2;
    if (ld < (n > 1 ? n : 1)) return -3;
    if (n == 0) return 0;
    zero_outside_z(n, r, H, T, ld);
    zdbl *v = (zdbl *)malloc(sizeof(zdbl) * (size_t)(r + 1));
    zdbl *w = (zdbl *)malloc(sizeof(zdbl) * (size_t)(r + 1));
    zdbl *blk = (zdbl *)malloc(sizeof(zdbl) * (size_t)(r * r));
    if (!v || !w || !blk) { free(v); free(w); free(blk); return 1; }
    double fl = 0.0;
    int64_t jlast = (jmax < 0 || jmax > n - 2) ? n - 2 : jmax;
    for (int64_t j = 1; j <= jlast; ++j) {
        int64_t nblocks = 1 + (n - j - 2) / r;
        for (int64_t k = 0; k < nblocks; ++k) {
            int64_t jb = j + ((k - 1) * r + 1 > 0 ? (k - 1) * r + 1 : 0);
            int64_t i1 = j + k * r + 1;
            int64_t i2 = j + (k + 1) * r < n ? j + (k + 1) * r : n;
            int64_t i3 = j + (k + 2) * r < n ? j + (k + 2) * r : n;
            int64_t m = i2 - i1 + 1;
            int64_t a = i1 - 1, cb = jb - 1;
            zdbl alpha = H[a + cb * ld], tau;
            for (int64_t i = 1; i < m; ++i) v[i] = H[a + i + cb * ld];
            oracle_larfg_z(m, &alpha, v + 1, &tau);
            v[0] = zmk(1.0, 0.0);
            H[a + cb * ld] = alpha;
            for (int64_t i = 1; i < m; ++i) H[a + i + cb * ld] = zmk(0.0, 0.0);
            left_z(H, ld, a, m, cb + 1, n - 1, v, tau);
            left_z(T, ld, a, m, a, n - 1, v, tau);
            fl += 16.0 * m * (double)(n - jb + 1) + 16.0 * m * (double)(n - i1 + 1);
            if (Q) { right_z(Q, ld, a, m, 0, n - 1, v, tau); fl += 16.0 * m * n; }
            for (int64_t c = 0; c < m; ++c)
                for (int64_t i = 0; i < m; ++i) blk[i + c * m] = T[a + i + (a + c) * ld];
            if (oracle_rq_dir_z(m, blk, m, w) != 0) { free(v); free(w); free(blk); return 1; }
            zdbl al2 = w[0], sig;
            oracle_larfg_z(m, &al2, w + 1, &sig);
            w[0] = zmk(1.0, 0.0);
            right_z(H, ld, a, m, 0, i3 - 1, w, sig);
            right_z(T, ld, a, m, 0, i2 - 1, w, sig);
            for (int64_t i = 1; i < m; ++i) T[a + i + a * ld] = zmk(0.0, 0.0);
            fl += 16.0 * m * (double)i3 + 16.0 * m * (double)i2;
            if (Z) { right_z(Z, ld, a, m, 0, n - 1, w, sig); fl += 16.0 * m * n; }
        }
    }
    if (jlast == n - 2 || n <= 2) zero_final_z(n, H, T, ld);
    if (flops) *flops += fl;
    free(v); free(w); free(blk);
    return 0;
}

/* Counted flops of the whole stage two (with Q and Z), without running it. */
double oracle_stage2_flops(int64_t n, int64_t r, int is_complex)
{
    double fl = 0.0;
    for (int64_t j = 1; j <= n - 2; ++j) {
        int64_t nblocks = 1 + (n - j - 2) / r;
        for (int64_t k = 0; k < nblocks; ++k) {
            int64_t jb = j + ((k - 1) * r + 1 > 0 ? (k - 1) * r + 1 : 0);
            int64_t i1 = j + k * r + 1;
            int64_t i2 = j + (k + 1) * r < n ? j + (k + 1) * r : n;
            int64_t i3 = j + (k + 2) * r < n ? j + (k + 2) * r : n;
            double m = (double)(i2 - i1 + 1);
            fl += 4.0 * m * ((double)(n - jb + 1) + (double)(n - i1 + 1) + (double)n
                             + (double)i3 + (double)i2 + (double)n);
        }
    }
    return is_complex ? 4.0 * fl : fl;
}

/* ======================================================================== */
/* Stage one (Section 2.2; blocked stage-one algorithm of the appendix),     */
/* preceded by the QR factorisation of B (the experiments of Section 4       */
/* replace B by the R of its QR factorisation).  1-based index map:          */
/*   panels j = 1, 1+nb, ... <= n-2 (nb = r), j2 = min(n, j+nb-1),           */
/*   n_blocks = ceil((n-nb-j+1) / ((p-1) nb)), blocks k = n_blocks-1 .. 0:   */
/*   i1 = j+nb+k(p-1)nb, i2 = min(n, i1+p nb-1).                             */
/* Left: QR of A(i1:i2, j:j2) by Householder reflectors, each applied at     */
/* once to A (the columns right of it), B (columns i1..n) and Q.  Right,     */
/* per block from the bottom: RQ of B(i1:i2, i1:i2) = Rt Qt, LQ of the first */
/* min(nb, i2-i1+1) rows of Qt by reflectors P_t applied from the right,     */
/* Qt(1:nb,:) P_0 ... P_{nb-1} = L; the same P_t are applied to A (all rows),*/
/* B (rows 1..i2) and Z, which makes the first nb columns of the B block     */
/* upper triangular (written as exact zeros).  p >= 2.                       */
/* ======================================================================== */

/* Householder RQ of the m x m matrix W (modified): for i = m-1..1 a
 * reflector U_i on columns 0..i maps row i to a multiple of e_i (the same
 * reflectors as oracle_rq_dir_*); Y <- I U_{m-1} ... U_1, so that
 * B = Rt Qt with Qt = Y^H. */
static void rq_accum_d(int64_t m, double *W, double *Y, double *u)
{
    for (int64_t c = 0; c < m; ++c)
        for (int64_t i = 0; i < m; ++i) Y[i + c * m] = (i == c) ? 1.0 : 0.0;
    for (int64_t i = m - 1; i >= 1; --i) {
        for (int64_t c = 0; c <= i; ++c) u[c] = W[i + c * m];
        double alpha = u[i], tau;
        oracle_larfg_d(i + 1, &alpha, u, &tau);
        u[i] = 1.0;
        if (tau == 0.0) continue;
        for (int pass = 0; pass < 2; ++pass) {
            double *X = pass ? Y : W;
            int64_t rows = pass ? m : i;
            for (int64_t rr = 0; rr < rows; ++rr) {
                double s = 0.0;
                for (int64_t c = 0; c <= i; ++c) s += X[rr + c * m] * u[c];
                s *= tau;
                for (int64_t c = 0; c <= i; ++c) X[rr + c * m] -= s * u[c];
            }
        }
    }
}

static void rq_accum_z(int64_t m, zdbl *W, zdbl *Y, zdbl *u)
{
    for (int64_t c = 0; c < m; ++c)
        for (int64_t i = 0; i < m; ++i) Y[i + c * m] = zmk(i == c ? 1.0 : 0.0, 0.0);
    for (int64_t i = m - 1; i >= 1; --i) {
        for (int64_t c = 0; c <= i; ++c) u[c] = zconj(W[i + c * m]);
        zdbl alpha = u[i], tau;
        oracle_larfg_z(i + 1, &alpha, u, &tau);
        u[i] = zmk(1.0, 0.0);
        if (tau.re == 0.0 && tau.im == 0.0) continue;
        for (int pass = 0; pass < 2; ++pass) {
            zdbl *X = pass ? Y : W;
            int64_t rows = pass ? m : i;
            for (int64_t rr = 0; rr < rows; ++rr) {
                zdbl s = zmk(0.0, 0.0);
                for (int64_t c = 0; c <= i; ++c) s = zadd(s, zmul(X[rr + c * m], u[c]));
                s = zmul(s, tau);
                for (int64_t c = 0; c <= i; ++c) X[rr + c * m] = zsub(X[rr + c * m], zmul(s, zconj(u[c])));
            }
        }
    }
}

int oracle_rhess_d(int64_t n, int64_t r, int64_t p, double *A, double *B, double *Q, double *Z,
                   int64_t ld, double *flops)
{
    if (n < 0) return -1;
    if (r < 1) return -2;
    if (p < 2) return -3;
    if (ld < (n > 1 ? n : 1)) return -8;
    if (n == 0) return 0;
    const int64_t nb = r < n - 1 ? r : (n > 1 ? n - 1 : 1);
    const int64_t mb = p * nb;                               /* largest block order */
    double *v = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    double *W = (double *)malloc(sizeof(double) * (size_t)(mb * mb));
    double *Y = (double *)malloc(sizeof(double) * (size_t)(mb * mb));
    double *M = (double *)malloc(sizeof(double) * (size_t)(nb * mb));
    double *u = (double *)malloc(sizeof(double) * (size_t)(mb + 1));
    if (!v || !W || !Y || !M || !u) { free(v); free(W); free(Y); free(M); free(u); return 1; }
    double fl = 0.0;
    /* QR of B: B = Q_B R, A <- Q_B^H A, Q <- Q Q_B */
    for (int64_t c = 0; c + 1 < n; ++c) {
        const int64_t m = n - c;
        double alpha = B[c + c * ld], tau;
        for (int64_t i = 1; i < m; ++i) v[i] = B[c + i + c * ld];
        oracle_larfg_d(m, &alpha, v + 1, &tau);
        v[0] = 1.0;
        B[c + c * ld] = alpha;
        for (int64_t i = 1; i < m; ++i) B[c + i + c * ld] = 0.0;
        left_d(B, ld, c, m, c + 1, n - 1, v, tau);
        left_d(A, ld, c, m, 0, n - 1, v, tau);
        fl += 4.0 * m * (double)(n - c - 1) + 4.0 * m * n;
        if (Q) { right_d(Q, ld, c, m, 0, n - 1, v, tau); fl += 4.0 * m * n; }
    }
    for (int64_t j = 1; j <= n - 2; j += nb) {
        const int64_t j2 = j + nb - 1 < n ? j + nb - 1 : n;
        const int64_t num = n - nb - j + 1;
        if (num <= 0) break;
        const int64_t nblk = (num + (p - 1) * nb - 1) / ((p - 1) * nb);
        /* left: QR of the blocks of the panel, from the bottom */
        for (int64_t k = nblk - 1; k >= 0; --k) {
            const int64_t i1 = j + nb + k * (p - 1) * nb;
            const int64_t i2 = i1 + p * nb - 1 < n ? i1 + p * nb - 1 : n;
            const int64_t rows = i2 - i1 + 1, cols = j2 - j + 1;
            for (int64_t s = 0; s < rows && s < cols; ++s) {
                const int64_t a = i1 - 1 + s, c = j - 1 + s, m = rows - s;
                double alpha = A[a + c * ld], tau;
                for (int64_t i = 1; i < m; ++i) v[i] = A[a + i + c * ld];
                oracle_larfg_d(m, &alpha, v + 1, &tau);
                v[0] = 1.0;
                A[a + c * ld] = alpha;
                for (int64_t i = 1; i < m; ++i) A[a + i + c * ld] = 0.0;
                left_d(A, ld, a, m, c + 1, n - 1, v, tau);
                left_d(B, ld, a, m, i1 - 1, n - 1, v, tau);
                fl += 4.0 * m * (double)(n - c - 1) + 4.0 * m * (double)(n - i1 + 1);
                if (Q) { right_d(Q, ld, a, m, 0, n - 1, v, tau); fl += 4.0 * m * n; }
            }
        }
        /* right: RQ + LQ per block, from the bottom */
        for (int64_t k = nblk - 1; k >= 0; --k) {
            const int64_t i1 = j + nb + k * (p - 1) * nb;
            const int64_t i2 = i1 + p * nb - 1 < n ? i1 + p * nb - 1 : n;
            const int64_t m = i2 - i1 + 1, nr = nb < m ? nb : m, a = i1 - 1;
            for (int64_t c = 0; c < m; ++c)
                for (int64_t i = 0; i < m; ++i) W[i + c * m] = B[a + i + (a + c) * ld];
            rq_accum_d(m, W, Y, u);
            fl += 4.0 / 3.0 * (double)m * m * m + 2.0 * (double)m * m * m;
            for (int64_t t = 0; t < nr; ++t)                  /* M = Qt(0:nr,:) = Y(:,0:nr)^H */
                for (int64_t c = 0; c < m; ++c) M[t + c * nr] = Y[c + t * m];
            for (int64_t t = 0; t < nr; ++t) {
                const int64_t len = m - t;
                double alpha = M[t + t * nr], tau;
                for (int64_t c = 1; c < len; ++c) v[c] = M[t + (t + c) * nr];
                oracle_larfg_d(len, &alpha, v + 1, &tau);
                v[0] = 1.0;
                M[t + t * nr] = alpha;
                for (int64_t c = 1; c < len; ++c) M[t + (t + c) * nr] = 0.0;
                if (tau == 0.0) continue;
                for (int64_t rr = t + 1; rr < nr; ++rr) {      /* M(rr, t:m) <- M P_t */
                    double s = 0.0;
                    for (int64_t c = 0; c < len; ++c) s += M[rr + (t + c) * nr] * v[c];
                    s *= tau;
                    for (int64_t c = 0; c < len; ++c) M[rr + (t + c) * nr] -= s * v[c];
                }
                right_d(A, ld, a + t, len, 0, n - 1, v, tau);
                right_d(B, ld, a + t, len, 0, i2 - 1, v, tau);
                fl += 4.0 * len * (double)n + 4.0 * len * (double)i2;
                if (Z) { right_d(Z, ld, a + t, len, 0, n - 1, v, tau); fl += 4.0 * len * n; }
            }
            for (int64_t c = 0; c < nr; ++c)
                for (int64_t i = c + 1; i < m; ++i) B[a + i + (a + c) * ld] = 0.0;
        }
    }
    /* exact zeros of the output contract: A r-Hessenberg, B upper triangular */
    for (int64_t c = 0; c < n; ++c) {
        for (int64_t i = c + nb + 1; i < n; ++i) A[i + c * ld] = 0.0;
        for (int64_t i = c + 1; i < n; ++i) B[i + c * ld] = 0.0;
    }
    if (flops) *flops += fl;
    free(v); free(W); free(Y); free(M); free(u);
    return 0;
}

int oracle_rhess_z(int64_t n, int64_t r, int64_t p, zdbl *A, zdbl *B, zdbl *Q, zdbl *Z,
                   int64_t ld, double *flops)
{
    if (n < 0) return -1;
    if (r < 1) return -2;
    if (p < 2) return -3;
    if (ld < (n > 1 ? n : 1)) return -8;
    if (n == 0) return 0;
    const int64_t nb = r < n - 1 ? r : (n > 1 ? n - 1 : 1);
    const int64_t mb = p * nb;
    zdbl *v = (zdbl *)malloc(sizeof(zdbl) * (size_t)(n + 1));
    zdbl *W = (zdbl *)malloc(sizeof(zdbl) * (size_t)(mb * mb));
    zdbl *Y = (zdbl *)malloc(sizeof(zdbl) * (size_t)(mb * mb));
    zdbl *M = (zdbl *)malloc(sizeof(zdbl) * (size_t)(nb * mb));
    zdbl *u = (zdbl *)malloc(sizeof(zdbl) * (size_t)(mb + 1));
    if (!v || !W || !Y || !M || !u) { free(v); free(W); free(Y); free(M); free(u); return 1; }
    double fl = 0.0;
    for (int64_t c = 0; c + 1 < n; ++c) {
        const int64_t m = n - c;
        zdbl alpha = B[c + c * ld], tau;
        for (int64_t i = 1; i < m; ++i) v[i] = B[c + i + c * ld];
        oracle_larfg_z(m, &alpha, v + 1, &tau);
        v[0] = zmk(1.0, 0.0);
        B[c + c * ld] = alpha;
        for (int64_t i = 1; i < m; ++i) B[c + i + c * ld] = zmk(0.0, 0.0);
        left_z(B, ld, c, m, c + 1, n - 1, v, tau);
        left_z(A, ld, c, m, 0, n - 1, v, tau);
        fl += 4.0 * (4.0 * m * (double)(n - c - 1) + 4.0 * m * n);
        if (Q) { right_z(Q, ld, c, m, 0, n - 1, v, tau); fl += 16.0 * m * n; }
    }
    for (int64_t j = 1; j <= n - 2; j += nb) {
        const int64_t j2 = j + nb - 1 < n ? j + nb - 1 : n;
        const int64_t num = n - nb - j + 1;
        if (num <= 0) break;
        const int64_t nblk = (num + (p - 1) * nb - 1) / ((p - 1) * nb);
        for (int64_t k = nblk - 1; k >= 0; --k) {
            const int64_t i1 = j + nb + k * (p - 1) * nb;
            const int64_t i2 = i1 + p * nb - 1 < n ? i1 + p * nb - 1 : n;
            const int64_t rows = i2 - i1 + 1, cols = j2 - j + 1;
            for (int64_t s = 0; s < rows && s < cols; ++s) {
                const int64_t a = i1 - 1 + s, c = j - 1 + s, m = rows - s;
                zdbl alpha = A[a + c * ld], tau;
                for (int64_t i = 1; i < m; ++i) v[i] = A[a + i + c * ld];
                oracle_larfg_z(m, &alpha, v + 1, &tau);
                v[0] = zmk(1.0, 0.0);
                A[a + c * ld] = alpha;
                for (int64_t i = 1; i < m; ++i) A[a + i + c * ld] = zmk(0.0, 0.0);
                left_z(A, ld, a, m, c + 1, n - 1, v, tau);
                left_z(B, ld, a, m, i1 - 1, n - 1, v, tau);
                fl += 4.0 * (4.0 * m * (double)(n - c - 1) + 4.0 * m * (double)(n - i1 + 1));
                if (Q) { right_z(Q, ld, a, m, 0, n - 1, v, tau); fl += 16.0 * m * n; }
            }
        }
        for (int64_t k = nblk - 1; k >= 0; --k) {
            const int64_t i1 = j + nb + k * (p - 1) * nb;
            const int64_t i2 = i1 + p * nb - 1 < n ? i1 + p * nb - 1 : n;
            const int64_t m = i2 - i1 + 1, nr = nb < m ? nb : m, a = i1 - 1;
            for (int64_t c = 0; c < m; ++c)
                for (int64_t i = 0; i < m; ++i) W[i + c * m] = B[a + i + (a + c) * ld];
            rq_accum_z(m, W, Y, u);
            fl += 4.0 * (4.0 / 3.0 * (double)m * m * m + 2.0 * (double)m * m * m);
            for (int64_t t = 0; t < nr; ++t)                  /* M = Qt(0:nr,:) = Y(:,0:nr)^H */
                for (int64_t c = 0; c < m; ++c) M[t + c * nr] = zconj(Y[c + t * m]);
            for (int64_t t = 0; t < nr; ++t) {
                const int64_t len = m - t;
                /* reflector from conj(row t): (row t) P_t = beta e_0^T */
                zdbl alpha = zconj(M[t + t * nr]), tau;
                for (int64_t c = 1; c < len; ++c) v[c] = zconj(M[t + (t + c) * nr]);
                oracle_larfg_z(len, &alpha, v + 1, &tau);
                v[0] = zmk(1.0, 0.0);
                M[t + t * nr] = alpha;
                for (int64_t c = 1; c < len; ++c) M[t + (t + c) * nr] = zmk(0.0, 0.0);
                if (tau.re == 0.0 && tau.im == 0.0) continue;
                for (int64_t rr = t + 1; rr < nr; ++rr) {      /* M(rr, t:m) <- M P_t */
                    zdbl s = zmk(0.0, 0.0);
                    for (int64_t c = 0; c < len; ++c) s = zadd(s, zmul(M[rr + (t + c) * nr], v[c]));
                    s = zmul(s, tau);
                    for (int64_t c = 0; c < len; ++c) M[rr + (t + c) * nr] = zsub(M[rr + (t + c) * nr], zmul(s, zconj(v[c])));
                }
                right_z(A, ld, a + t, len, 0, n - 1, v, tau);
                right_z(B, ld, a + t, len, 0, i2 - 1, v, tau);
                fl += 4.0 * (4.0 * len * (double)n + 4.0 * len * (double)i2);
                if (Z) { right_z(Z, ld, a + t, len, 0, n - 1, v, tau); fl += 16.0 * len * n; }
            }
            for (int64_t c = 0; c < nr; ++c)
                for (int64_t i = c + 1; i < m; ++i) B[a + i + (a + c) * ld] = zmk(0.0, 0.0);
        }
    }
    for (int64_t c = 0; c < n; ++c) {
        for (int64_t i = c + nb + 1; i < n; ++i) A[i + c * ld] = zmk(0.0, 0.0);
        for (int64_t i = c + 1; i < n; ++i) B[i + c * ld] = zmk(0.0, 0.0);
    }
    if (flops) *flops += fl;
    free(v); free(W); free(Y); free(M); free(u);
    return 0;
}
