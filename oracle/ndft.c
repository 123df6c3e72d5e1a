/*
 * TEST INFRASTRUCTURE ONLY -- the oracle.  Nothing in the product path may
 * include, link or call this file; only tests/, the smoke check and the
 * CPU-baseline leg of bench.py load it (through oracle/__init__.py).
 *
 * Plain FP64 direct evaluation of the 3-D trigonometric sums that the
 * nonequispaced FFT approximates.  Everything here is the definition written
 * out, with no window, no oversampled grid and no FFT:
 *
 *   trafo   (type 2, Sec. 2.2.1 of the paper, the NFFT problem statement):
 *       f_j = sum_{k in I_N} fhat_k * exp(-2 pi i k . x_j)
 *   adjoint (type 1; the transpose-conjugate of the same matrix):
 *       fhat_k = sum_j f_j * exp(+2 pi i k . x_j)
 *   grad    (derivative of f_j with respect to its own point; the Lambda
 *            multipliers of eq. (Lambda) in the NFFT sign convention):
 *       df_j/dx_{j,d} = sum_k (-2 pi i k_d) fhat_k exp(-2 pi i k . x_j)
 *
 * with I_N = prod_d {-N_d/2, ..., N_d/2 - 1}, N_d even (Sec. 2, definition of
 * I_N; the frequency of array index i_d is k_d = i_d - N_d/2, the shifted
 * index k_d - 1 - N_d/2 of eq. (fs) / eq. (Fs)).
 *
 * The evaluation order follows the "one-loop" construction of eq. (Fs): for
 * each point build one exponential vector per dimension, E^d[i] =
 * exp(-2 pi i k_d x_d), and form the triple sum
 *     sum_{k1} E^1 sum_{k2} E^2 sum_{k3} E^3 fhat.
 * Storage: fhat is C order (N0, N1, N2), the last axis contiguous, complex
 * numbers interleaved (re, im).  Points are (M, 3) row-major, column d paired
 * with array axis d.
 *
 * Phase accuracy: k*x is reduced modulo 1 exactly (two-product with fma, then
 * subtraction of the nearest integer, which is exact), so the table entries
 * carry ~1e-16 absolute phase error at any |k|.
 *
 * Threads: points (trafo, grad) or slabs of k0 (adjoint) are split over
 * POSIX threads; every output element is written by exactly one thread.
 * The sampled adjoint (a few coefficients, many points) splits the points;
 * each thread sums its points into its own row of partial sums, and the rows
 * are added in thread order.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static const double TWO_PI = 6.283185307179586476925286766559;

/* E[i] = exp(sgn * 2 pi i k x) for k = i - Nd/2, i = 0..Nd-1. */
static void phase_vector(int64_t Nd, double x, double sgn, double *re, double *im)
{
    for (int64_t i = 0; i < Nd; ++i) {
        double k = (double)(i - Nd / 2);
        double p = k * x;
        double e = fma(k, x, -p);          /* k*x = p + e exactly         */
        double r = (p - rint(p)) + e;      /* k*x mod 1, in [-1/2, 1/2]   */
        re[i] = cos(TWO_PI * r);
        im[i] = sgn * sin(TWO_PI * r);
    }
}

typedef struct {
    const int64_t *N;
    const double *fhat;    /* interleaved complex, C order          */
    const double *x;       /* (M,3)                                  */
    double *out;           /* trafo: (M) complex; grad: (M,3) complex */
    int64_t M;
    int64_t j0, j1;        /* point range for this thread            */
    int64_t k0lo, k0hi;    /* adjoint: slab range of axis 0          */
    const double *f;       /* adjoint input values                   */
} job_t;

/* ---- type 2: f_j = sum_k fhat_k exp(-2 pi i k.x_j) ---------------------- */
static void *trafo_worker(void *arg)
{
    job_t *jb = (job_t *)arg;
    const int64_t N0 = jb->N[0], N1 = jb->N[1], N2 = jb->N[2];
    double *e0r = malloc(sizeof(double) * N0), *e0i = malloc(sizeof(double) * N0);
    double *e1r = malloc(sizeof(double) * N1), *e1i = malloc(sizeof(double) * N1);
    double *e2r = malloc(sizeof(double) * N2), *e2i = malloc(sizeof(double) * N2);
    for (int64_t j = jb->j0; j < jb->j1; ++j) {
        const double *xj = jb->x + 3 * j;
        phase_vector(N0, xj[0], -1.0, e0r, e0i);
        phase_vector(N1, xj[1], -1.0, e1r, e1i);
        phase_vector(N2, xj[2], -1.0, e2r, e2i);
        double ar = 0.0, ai = 0.0;
        for (int64_t a = 0; a < N0; ++a) {
            double s1r = 0.0, s1i = 0.0;
            for (int64_t b = 0; b < N1; ++b) {
                const double *row = jb->fhat + 2 * ((a * N1 + b) * N2);
                double s2r = 0.0, s2i = 0.0;
                for (int64_t c = 0; c < N2; ++c) {
                    double fr = row[2 * c], fi = row[2 * c + 1];
                    s2r += fr * e2r[c] - fi * e2i[c];
                    s2i += fr * e2i[c] + fi * e2r[c];
                }
                s1r += e1r[b] * s2r - e1i[b] * s2i;
                s1i += e1r[b] * s2i + e1i[b] * s2r;
            }
            ar += e0r[a] * s1r - e0i[a] * s1i;
            ai += e0r[a] * s1i + e0i[a] * s1r;
        }
        jb->out[2 * j] = ar;
        jb->out[2 * j + 1] = ai;
    }
    free(e0r); free(e0i); free(e1r); free(e1i); free(e2r); free(e2i);
    return NULL;
}

/* ---- derivative: df_j/dx_{j,d} = sum_k (-2 pi i k_d) fhat_k exp(-2 pi i k.x_j) */
static void *grad_worker(void *arg)
{
    job_t *jb = (job_t *)arg;
    const int64_t N0 = jb->N[0], N1 = jb->N[1], N2 = jb->N[2];
    double *e0r = malloc(sizeof(double) * N0), *e0i = malloc(sizeof(double) * N0);
    double *e1r = malloc(sizeof(double) * N1), *e1i = malloc(sizeof(double) * N1);
    double *e2r = malloc(sizeof(double) * N2), *e2i = malloc(sizeof(double) * N2);
    for (int64_t j = jb->j0; j < jb->j1; ++j) {
        const double *xj = jb->x + 3 * j;
        phase_vector(N0, xj[0], -1.0, e0r, e0i);
        phase_vector(N1, xj[1], -1.0, e1r, e1i);
        phase_vector(N2, xj[2], -1.0, e2r, e2i);
        /* t[d] accumulates sum_k k_d fhat_k E(k), d = 0, 1, 2 */
        double t0r = 0, t0i = 0, t1r = 0, t1i = 0, t2r = 0, t2i = 0;
        for (int64_t a = 0; a < N0; ++a) {
            double k0 = (double)(a - N0 / 2);
            double s1r = 0, s1i = 0, u1r = 0, u1i = 0, v1r = 0, v1i = 0;
            for (int64_t b = 0; b < N1; ++b) {
                double k1 = (double)(b - N1 / 2);
                const double *row = jb->fhat + 2 * ((a * N1 + b) * N2);
                double s2r = 0, s2i = 0, v2r = 0, v2i = 0;
                for (int64_t c = 0; c < N2; ++c) {
                    double k2 = (double)(c - N2 / 2);
                    double fr = row[2 * c], fi = row[2 * c + 1];
                    double pr = fr * e2r[c] - fi * e2i[c];
                    double pi = fr * e2i[c] + fi * e2r[c];
                    s2r += pr;       s2i += pi;
                    v2r += k2 * pr;  v2i += k2 * pi;
                }
                double qr = e1r[b] * s2r - e1i[b] * s2i;
                double qi = e1r[b] * s2i + e1i[b] * s2r;
                s1r += qr;      s1i += qi;
                u1r += k1 * qr; u1i += k1 * qi;
                v1r += e1r[b] * v2r - e1i[b] * v2i;
                v1i += e1r[b] * v2i + e1i[b] * v2r;
            }
            double qr = e0r[a] * s1r - e0i[a] * s1i;
            double qi = e0r[a] * s1i + e0i[a] * s1r;
            t0r += k0 * qr; t0i += k0 * qi;
            t1r += e0r[a] * u1r - e0i[a] * u1i;
            t1i += e0r[a] * u1i + e0i[a] * u1r;
            t2r += e0r[a] * v1r - e0i[a] * v1i;
            t2i += e0r[a] * v1i + e0i[a] * v1r;
        }
        /* multiply by -2 pi i:  (-2 pi i)(tr + i ti) = 2 pi ti - 2 pi i tr */
        double *o = jb->out + 6 * j;
        o[0] = TWO_PI * t0i;  o[1] = -TWO_PI * t0r;
        o[2] = TWO_PI * t1i;  o[3] = -TWO_PI * t1r;
        o[4] = TWO_PI * t2i;  o[5] = -TWO_PI * t2r;
    }
    free(e0r); free(e0i); free(e1r); free(e1i); free(e2r); free(e2i);
    return NULL;
}

/* ---- type 1: fhat_k = sum_j f_j exp(+2 pi i k.x_j), slab [k0lo, k0hi) --- */
static void *adjoint_worker(void *arg)
{
    job_t *jb = (job_t *)arg;
    const int64_t N0 = jb->N[0], N1 = jb->N[1], N2 = jb->N[2];
    double *e0r = malloc(sizeof(double) * N0), *e0i = malloc(sizeof(double) * N0);
    double *e1r = malloc(sizeof(double) * N1), *e1i = malloc(sizeof(double) * N1);
    double *e2r = malloc(sizeof(double) * N2), *e2i = malloc(sizeof(double) * N2);
    for (int64_t j = 0; j < jb->M; ++j) {
        const double *xj = jb->x + 3 * j;
        const double fr = jb->f[2 * j], fi = jb->f[2 * j + 1];
        phase_vector(N0, xj[0], +1.0, e0r, e0i);
        phase_vector(N1, xj[1], +1.0, e1r, e1i);
        phase_vector(N2, xj[2], +1.0, e2r, e2i);
        for (int64_t a = jb->k0lo; a < jb->k0hi; ++a) {
            double ar = fr * e0r[a] - fi * e0i[a];
            double ai = fr * e0i[a] + fi * e0r[a];
            for (int64_t b = 0; b < N1; ++b) {
                double br = ar * e1r[b] - ai * e1i[b];
                double bi = ar * e1i[b] + ai * e1r[b];
                double *row = jb->out + 2 * ((a * N1 + b) * N2);
                for (int64_t c = 0; c < N2; ++c) {
                    row[2 * c] += br * e2r[c] - bi * e2i[c];
                    row[2 * c + 1] += br * e2i[c] + bi * e2r[c];
                }
            }
        }
    }
    free(e0r); free(e0i); free(e1r); free(e1i); free(e2r); free(e2i);
    return NULL;
}

static int check_args(const int64_t N[3], int64_t M)
{
    if (M < 0) return -1;
    for (int d = 0; d < 3; ++d)
        if (N[d] < 2 || (N[d] % 2) != 0) return -1;
    return 0;
}

static int run_over_points(void *(*fn)(void *), const int64_t N[3], const double *fhat,
                           int64_t M, const double *x, double *out, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if ((int64_t)nthreads > M) nthreads = (int)(M > 0 ? M : 1);
    pthread_t th[256];
    job_t jobs[256];
    for (int t = 0; t < nthreads; ++t) {
        memset(&jobs[t], 0, sizeof(job_t));
        jobs[t].N = N; jobs[t].fhat = fhat; jobs[t].x = x; jobs[t].out = out; jobs[t].M = M;
        jobs[t].j0 = M * t / nthreads;
        jobs[t].j1 = M * (t + 1) / nthreads;
    }
    for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, fn, &jobs[t]);
    fn(&jobs[0]);
    for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
    return 0;
}

int oracle_ndft_trafo(const int64_t N[3], const double *fhat, int64_t M, const double *x,
                      double *f, int nthreads)
{
    if (check_args(N, M)) return -1;
    if (M == 0) return 0;
    return run_over_points(trafo_worker, N, fhat, M, x, f, nthreads);
}

int oracle_ndft_grad(const int64_t N[3], const double *fhat, int64_t M, const double *x,
                     double *df, int nthreads)
{
    if (check_args(N, M)) return -1;
    if (M == 0) return 0;
    return run_over_points(grad_worker, N, fhat, M, x, df, nthreads);
}

int oracle_ndft_adjoint(const int64_t N[3], int64_t M, const double *x, const double *f,
                        double *fhat, int nthreads)
{
    if (check_args(N, M)) return -1;
    memset(fhat, 0, sizeof(double) * 2 * N[0] * N[1] * N[2]);
    if (M == 0) return 0;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if (nthreads > N[0]) nthreads = (int)N[0];
    pthread_t th[256];
    job_t jobs[256];
    for (int t = 0; t < nthreads; ++t) {
        memset(&jobs[t], 0, sizeof(job_t));
        jobs[t].N = N; jobs[t].x = x; jobs[t].f = f; jobs[t].out = fhat; jobs[t].M = M;
        jobs[t].k0lo = N[0] * t / nthreads;
        jobs[t].k0hi = N[0] * (t + 1) / nthreads;
    }
    for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, adjoint_worker, &jobs[t]);
    adjoint_worker(&jobs[0]);
    for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
    return 0;
}

/* ---- sampled type 1: fhat at K given indices, sum over all points ------- */
/* k x mod 1 with the exact reduction of phase_vector                        */
static double reduced_phase(double k, double x)
{
    double p = k * x;
    double e = fma(k, x, -p);
    return (p - rint(p)) + e;
}

typedef struct {
    const int64_t *N, *kidx;
    const double *x, *f;
    int64_t K, j0, j1;
    double *acc;           /* 2 K partial sums of this thread           */
} atjob_t;

static void *adjoint_at_worker(void *arg)
{
    atjob_t *jb = (atjob_t *)arg;
    for (int64_t j = jb->j0; j < jb->j1; ++j) {
        const double *xj = jb->x + 3 * j;
        const double fr = jb->f[2 * j], fi = jb->f[2 * j + 1];
        for (int64_t q = 0; q < jb->K; ++q) {
            double r = 0.0;
            for (int d = 0; d < 3; ++d)
                r += reduced_phase((double)(jb->kidx[3 * q + d] - jb->N[d] / 2), xj[d]);
            r -= rint(r);
            const double c = cos(TWO_PI * r), sn = sin(TWO_PI * r);   /* exp(+2 pi i k.x) */
            jb->acc[2 * q] += fr * c - fi * sn;
            jb->acc[2 * q + 1] += fr * sn + fi * c;
        }
    }
    return NULL;
}

/* out[q] = sum_j f_j exp(+2 pi i k_q . x_j) for the K array-index triples
 * kidx[3q .. 3q+2] (frequency k_d = kidx - N_d/2). */
int oracle_ndft_adjoint_at(const int64_t N[3], int64_t M, const double *x, const double *f, int64_t K,
                           const int64_t *kidx, double *out, int nthreads)
{
    if (check_args(N, M) || K < 0) return -1;
    for (int64_t q = 0; q < K; ++q)
        for (int d = 0; d < 3; ++d)
            if (kidx[3 * q + d] < 0 || kidx[3 * q + d] >= N[d]) return -1;
    memset(out, 0, sizeof(double) * 2 * K);
    if (M == 0 || K == 0) return 0;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if ((int64_t)nthreads > M) nthreads = (int)M;
    double *acc = calloc((size_t)nthreads * 2 * K, sizeof(double));
    if (!acc) return -2;
    pthread_t th[256];
    atjob_t jobs[256];
    for (int t = 0; t < nthreads; ++t) {
        jobs[t].N = N; jobs[t].kidx = kidx; jobs[t].x = x; jobs[t].f = f; jobs[t].K = K;
        jobs[t].j0 = M * t / nthreads;
        jobs[t].j1 = M * (t + 1) / nthreads;
        jobs[t].acc = acc + (size_t)t * 2 * K;
    }
    for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, adjoint_at_worker, &jobs[t]);
    adjoint_at_worker(&jobs[0]);
    for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
    for (int t = 0; t < nthreads; ++t)
        for (int64_t i = 0; i < 2 * K; ++i) out[i] += acc[(size_t)t * 2 * K + i];
    free(acc);
    return 0;
}
