/*
 * Plain FP64 rank-Greville (Staub & Steinmann, Algorithm 1) in C.
 *
 * TEST INFRASTRUCTURE ONLY: this is the reference the HIP path is checked
 * against and the timed CPU baseline.  It shares no code with the product
 * library.  Straight loops over row-major arrays, no BLAS, no blocking, no
 * fast-math, exactly the steps of Algorithm 1 in the paper's order:
 *
 *   gamma   = Ct Gamma                                  (projection, Sec. 2.1)
 *   Gamma_r = Gamma - C^T gamma                         (rejection, Sec. 2.1)
 *   rank test of Section 3: dependent iff ||Gamma_r|| < eps or
 *             ||Gamma_r|| < eps ||Gamma||;  eps < 0 selects the paper's
 *             default (m^2 r + m r + m) * 2^-52 at the current rank r
 *   independent (Theorems 4, 6):  K = Gamma_r / ||Gamma_r||^2,
 *             C <- [C; Gamma^T], Ct <- [Ct - gamma K^T; K^T],
 *             Pinv <- diag(Pinv, 1)
 *   dependent (Theorems 5, 6):  zeta = Pinv gamma, d = 1 + gamma^T zeta,
 *             K = Ct^T zeta / d, Pinv <- Pinv - zeta zeta^T / d
 *   X <- X + K (y - Gamma^T X)                          (X before the update)
 *
 * Build: gcc -O2 -fPIC -shared -pthread rg_ref.c -o librg_ref.so -lm
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int m, cap, r;
    double eps;          /* < 0: default of Section 3 */
    double *X;           /* m */
    double *C, *Ct;      /* cap x m, row-major */
    double *Pinv;        /* cap x cap, row-major, leading dimension cap */
    double *gamma, *Gr, *zeta, *K;  /* work vectors */
    int overflow;        /* rank would exceed cap */
} rgo_state;

rgo_state *rgo_new(int m, int cap, double eps)
{
    if (m <= 0 || cap <= 0) return NULL;
    rgo_state *s = (rgo_state *)calloc(1, sizeof(rgo_state));
    if (!s) return NULL;
    s->m = m; s->cap = cap; s->r = 0; s->eps = eps;
    s->X = (double *)calloc((size_t)m, sizeof(double));
    s->C = (double *)calloc((size_t)cap * m, sizeof(double));
    s->Ct = (double *)calloc((size_t)cap * m, sizeof(double));
    s->Pinv = (double *)calloc((size_t)cap * cap, sizeof(double));
    s->gamma = (double *)calloc((size_t)cap, sizeof(double));
    s->zeta = (double *)calloc((size_t)cap, sizeof(double));
    s->Gr = (double *)calloc((size_t)m, sizeof(double));
    s->K = (double *)calloc((size_t)m, sizeof(double));
    if (!s->X || !s->C || !s->Ct || !s->Pinv || !s->gamma || !s->zeta || !s->Gr || !s->K) {
        free(s->X); free(s->C); free(s->Ct); free(s->Pinv);
        free(s->gamma); free(s->zeta); free(s->Gr); free(s->K); free(s);
        return NULL;
    }
    return s;
}

void rgo_free(rgo_state *s)
{
    if (!s) return;
    free(s->X); free(s->C); free(s->Ct); free(s->Pinv);
    free(s->gamma); free(s->zeta); free(s->Gr); free(s->K); free(s);
}

/* One call of UpdateLeastSquares.  Returns 1 if the row was independent,
 * 0 if dependent, -1 if the rank would exceed the capacity (state unchanged). */
static int rgo_update(rgo_state *s, const double *G, double y)
{
    const int m = s->m, r = s->r, cap = s->cap;
    double *C = s->C, *Ct = s->Ct, *P = s->Pinv, *X = s->X;
    double *gamma = s->gamma, *Gr = s->Gr, *zeta = s->zeta, *K = s->K;

    for (int k = 0; k < r; ++k) {                 /* gamma = Ct Gamma */
        double a = 0.0;
        for (int j = 0; j < m; ++j) a += Ct[(size_t)k * m + j] * G[j];
        gamma[k] = a;
    }
    for (int j = 0; j < m; ++j) {                 /* Gamma_r = Gamma - C^T gamma */
        double a = G[j];
        for (int k = 0; k < r; ++k) a -= C[(size_t)k * m + j] * gamma[k];
        Gr[j] = a;
    }
    double nr2 = 0.0, ng2 = 0.0;
    for (int j = 0; j < m; ++j) { nr2 += Gr[j] * Gr[j]; ng2 += G[j] * G[j]; }
    double eps = s->eps;
    if (eps < 0.0) eps = ((double)m * m * r + (double)m * r + m) * 0x1p-52;
    const double nr = sqrt(nr2), ng = sqrt(ng2);
    /* an exactly zero rejection is dependent for every eps: with eps = 0 this
     * is Algorithm 1's exact test Gamma_r == 0 (the Python oracle's eps = 0) */
    const int dependent = (nr2 == 0.0) || (nr < eps) || (nr < eps * ng);

    double dy = y;                                /* a priori residual */
    for (int j = 0; j < m; ++j) dy -= G[j] * X[j];

    if (!dependent) {
        if (r == cap) return -1;
        for (int j = 0; j < m; ++j) K[j] = Gr[j] / nr2;
        for (int k = 0; k < r; ++k)
            for (int j = 0; j < m; ++j) Ct[(size_t)k * m + j] -= gamma[k] * K[j];
        for (int j = 0; j < m; ++j) {
            C[(size_t)r * m + j] = G[j];
            Ct[(size_t)r * m + j] = K[j];
        }
        for (int k = 0; k < r; ++k) { P[(size_t)r * cap + k] = 0.0; P[(size_t)k * cap + r] = 0.0; }
        P[(size_t)r * cap + r] = 1.0;
        s->r = r + 1;
    } else {
        for (int i = 0; i < r; ++i) {
            double a = 0.0;
            for (int k = 0; k < r; ++k) a += P[(size_t)i * cap + k] * gamma[k];
            zeta[i] = a;
        }
        double d = 1.0;
        for (int k = 0; k < r; ++k) d += gamma[k] * zeta[k];
        for (int j = 0; j < m; ++j) {
            double a = 0.0;
            for (int k = 0; k < r; ++k) a += Ct[(size_t)k * m + j] * zeta[k];
            K[j] = a / d;
        }
        for (int i = 0; i < r; ++i)
            for (int k = 0; k < r; ++k) P[(size_t)i * cap + k] -= zeta[i] * zeta[k] / d;
    }
    for (int j = 0; j < m; ++j) X[j] += K[j] * dy;
    return dependent ? 0 : 1;
}

/* Push k rows (row-major k x m) with targets y.  decisions (nullable) gets
 * 1/0 per row.  Returns 0, or -1 if the capacity was hit (processing stops
 * at that row; s->overflow is set). */
int rgo_push(rgo_state *s, const double *A, const double *y, int64_t k, uint8_t *decisions)
{
    if (!s || s->overflow) return -1;
    for (int64_t i = 0; i < k; ++i) {
        int d = rgo_update(s, A + (size_t)i * s->m, y[i]);
        if (d < 0) { s->overflow = 1; return -1; }
        if (decisions) decisions[i] = (uint8_t)d;
    }
    return 0;
}

int rgo_rank(const rgo_state *s) { return s ? s->r : -1; }

/* Copy out X (m), C and Ct (r x m), Pinv (r x r, packed leading dim r). */
void rgo_get(const rgo_state *s, double *X, double *C, double *Ct, double *Pinv)
{
    const int m = s->m, r = s->r;
    if (X) memcpy(X, s->X, sizeof(double) * (size_t)m);
    if (C) memcpy(C, s->C, sizeof(double) * (size_t)r * m);
    if (Ct) memcpy(Ct, s->Ct, sizeof(double) * (size_t)r * m);
    if (Pinv)
        for (int i = 0; i < r; ++i)
            for (int k = 0; k < r; ++k) Pinv[(size_t)i * r + k] = s->Pinv[(size_t)i * s->cap + k];
}

/* ---- independent streams over a thread pool (dynamic, longest first) ---- */

typedef struct {
    int B;
    const int *m, *cap;
    const int64_t *row_ptr, *a_off, *order;
    const double *A, *Y;
    double eps;
    double *X;           /* packed, offsets x_off */
    const int64_t *x_off;
    int *rank;
    int *status;
    int64_t next;
    pthread_mutex_t mu;
} rgo_batch_job;

static void *rgo_worker(void *arg)
{
    rgo_batch_job *job = (rgo_batch_job *)arg;
    for (;;) {
        pthread_mutex_lock(&job->mu);
        int64_t t = job->next++;
        pthread_mutex_unlock(&job->mu);
        if (t >= job->B) break;
        int64_t b = job->order ? job->order[t] : t;
        int m = job->m[b];
        int cap = job->cap ? job->cap[b] : m;
        rgo_state *s = rgo_new(m, cap, job->eps);
        if (!s) { job->status[b] = -2; continue; }
        int64_t n = job->row_ptr[b + 1] - job->row_ptr[b];
        job->status[b] = rgo_push(s, job->A + job->a_off[b], job->Y + job->row_ptr[b], n, NULL);
        memcpy(job->X + job->x_off[b], s->X, sizeof(double) * (size_t)m);
        job->rank[b] = s->r;
        rgo_free(s);
    }
    return NULL;
}

/* Solve B independent streams from scratch.  Stream b has m[b] columns,
 * rows row_ptr[b] .. row_ptr[b+1]-1 of the packed targets Y, and its rows
 * start at element a_off[b] of A (row-major n_b x m[b]).  X is packed with
 * offsets x_off.  order (nullable) gives the processing order.  Returns the
 * number of threads used. */
int rgo_solve_batch(int B, const int *m, const int *cap, const int64_t *row_ptr, const int64_t *a_off,
                    const double *A, const double *Y, double eps, const int64_t *order,
                    const int64_t *x_off, double *X, int *rank, int *status, int nthreads)
{
    rgo_batch_job job;
    job.B = B; job.m = m; job.cap = cap; job.row_ptr = row_ptr; job.a_off = a_off; job.order = order;
    job.A = A; job.Y = Y; job.eps = eps; job.X = X; job.x_off = x_off; job.rank = rank; job.status = status;
    job.next = 0;
    pthread_mutex_init(&job.mu, NULL);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > B) nthreads = B > 0 ? B : 1;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    int started = 0;
    for (int i = 0; i < nthreads; ++i)
        if (pthread_create(&th[i], NULL, rgo_worker, &job) == 0) ++started;
    if (started == 0) rgo_worker(&job);
    for (int i = 0; i < started; ++i) pthread_join(th[i], NULL);
    free(th);
    pthread_mutex_destroy(&job.mu);
    return started > 0 ? started : 1;
}
