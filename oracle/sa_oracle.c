/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, sequential reference for the sampling half of the self-adaptive
 * Ising machine: one simulated-annealing run of the software p-bit machine per
 * replica (Sec. III-B, Eq. Ii_eq and Eq. mi_eq, sequential Gibbs updates under a
 * linear beta schedule).  Only tests/, the smoke check and the bench's CPU
 * baseline may load this file's library; the product never does.
 *
 * All arithmetic is integer.  The encoding (slack bits, scales, penalty, beta
 * grid, threshold table) is built by oracle.py and handed in as plain arrays.
 *
 * Per visit of site i the local field is the energy difference of the
 * normalised Lagrangian (Eq. Lagrange_energy with the penalty of
 * Eq. penalty_energy), scaled by D = 256 s_f s_g^2 so it is an exact integer:
 *
 *   Z_i = -D [ L(x with x_i=1) - L(x with x_i=0) ]
 *       = 256 s_g^2 dprofit_i - s_f Pq (|g1|^2 - |g0|^2) - s_f s_g lq.(g1 - g0)
 *
 * where g0, g1 are the constraint residuals A x - b with x_i forced to 0 / 1.
 * The p-bit input is I_i = Z_i / (2D) in normalised units; the update of
 * Eq. mi_eq is realised as x_i <- [u24 < Theta[idx]] with
 * idx = round(beta_t I_i * 256) taken from the integer beta grid.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;

#define THETA_HALF 2304

typedef struct {
    int32_t n_ext;        /* spins including slack bits */
    int32_t m;            /* constraints */
    int32_t T;            /* sweeps per run */
    int32_t S;            /* beta grid shift */
    const int64_t *W;     /* n_ext*n_ext pair profits, zero diagonal */
    const int64_t *h;     /* n_ext single-item profits */
    const int64_t *A;     /* m*n_ext extended constraint matrix */
    const int64_t *b;     /* m capacities */
    int64_t s_f, s_g, pq; /* profit scale, constraint scale, 256*P */
    const int64_t *B;     /* T beta grid values */
    const int32_t *theta; /* 2*THETA_HALF+1 thresholds, index j+THETA_HALF */
    uint64_t seed;
    uint32_t inst;
} oracle_prog;

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the
 * two-multiplier S-box with a Weyl-sequence key schedule. */
static void philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void oracle_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    philox4x32_10(ctr, key, out);
}

/* floor(v / 2^s) for signed 128-bit v, written as a division so it does not
 * depend on the compiler's shift of negative numbers. */
static i128 floor_div_pow2(i128 v, int s)
{
    i128 d = (i128)1 << s;
    i128 q = v / d;
    if ((v % d) != 0 && v < 0) q -= 1;
    return q;
}

/* Threshold index for field Z at sweep t: clamp(floor((Z*B_t + 2^(S-1)) / 2^S)). */
int32_t oracle_index(const oracle_prog *p, int64_t Z, int32_t t)
{
    i128 v = (i128)Z * (i128)p->B[t] + ((i128)1 << (p->S - 1));
    i128 q = floor_div_pow2(v, p->S);
    if (q > THETA_HALF) q = THETA_HALF;
    if (q < -THETA_HALF) q = -THETA_HALF;
    return (int32_t)q;
}

/* Z_i for state x (bytes 0/1) with residuals g = A x - b and multipliers lq. */
int64_t oracle_local_field(const oracle_prog *p, const uint8_t *x, const int64_t *g,
                           const int32_t *lq, int32_t i)
{
    const int32_t n = p->n_ext;
    /* profit gained by switching item i on, others fixed */
    i128 dprofit = p->h[i];
    for (int32_t j = 0; j < n; ++j)
        if (j != i && x[j]) dprofit += p->W[(int64_t)i * n + j];
    /* constraint terms at x_i = 0 and x_i = 1 */
    i128 dpen = 0, dlam = 0;
    for (int32_t k = 0; k < p->m; ++k) {
        int64_t a = p->A[(int64_t)k * n + i];
        i128 g0 = (i128)g[k] - (i128)a * x[i];
        i128 g1 = g0 + a;
        dpen += g1 * g1 - g0 * g0;
        dlam += (i128)lq[k] * (g1 - g0);
    }
    i128 s_g2 = (i128)p->s_g * p->s_g;
    i128 dL = -(i128)256 * s_g2 * dprofit + (i128)p->s_f * p->pq * dpen
              + (i128)p->s_f * p->s_g * dlam;
    return (int64_t)(-dL);
}

/* One annealing run of one replica; x_out gets n_ext bytes, g_out m residuals. */
static void sa_run_one(const oracle_prog *p, const int32_t *lq, int32_t k, int32_t r,
                       uint8_t *x, int64_t *g)
{
    const int32_t n = p->n_ext;
    const uint32_t nq = (uint32_t)((n + 3) / 4);
    const uint32_t key[2] = {(uint32_t)p->seed, (uint32_t)(p->seed >> 32)};
    uint32_t rnd[4] = {0, 0, 0, 0};
    memset(x, 0, (size_t)n);
    for (int32_t c = 0; c < p->m; ++c) g[c] = -p->b[c];
    for (int32_t t = 0; t < p->T; ++t) {
        for (int32_t i = 0; i < n; ++i) {
            if (i % 4 == 0) {
                uint32_t ctr[4] = {(uint32_t)t * nq + (uint32_t)(i / 4), (uint32_t)k,
                                   (uint32_t)r, p->inst};
                philox4x32_10(ctr, key, rnd);
            }
            uint32_t u24 = rnd[i % 4] >> 8;
            int64_t Z = oracle_local_field(p, x, g, lq, i);
            int32_t idx = oracle_index(p, Z, t);
            uint8_t xn = (uint8_t)(u24 < (uint32_t)p->theta[idx + THETA_HALF]);
            if (xn != x[i]) {
                int64_t delta = (int64_t)xn - (int64_t)x[i];
                for (int32_t c = 0; c < p->m; ++c) g[c] += delta * p->A[(int64_t)c * n + i];
                x[i] = xn;
            }
        }
    }
}

typedef struct {
    const oracle_prog *p;
    const int32_t *lq;
    int32_t k, r0, r1, base;
    uint8_t *x_out;
    int64_t *g_out;
} job;

static void *worker(void *arg)
{
    job *j = (job *)arg;
    for (int32_t r = j->r0; r < j->r1; ++r) {
        int64_t off = r - j->base;
        sa_run_one(j->p, j->lq, j->k, r, j->x_out + off * j->p->n_ext, j->g_out + off * j->p->m);
    }
    return NULL;
}

/* Runs replicas r0 .. r0+nrep-1 of round k; replicas are split statically
 * over nthreads POSIX threads.  Returns 0 on success. */
int oracle_sa_round(const oracle_prog *p, const int32_t *lq, int32_t k, int32_t r0, int32_t nrep,
                    uint8_t *x_out, int64_t *g_out, int32_t nthreads)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > nrep) nthreads = nrep > 0 ? nrep : 1;
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    job *jobs = (job *)calloc((size_t)nthreads, sizeof(job));
    if (!th || !jobs) { free(th); free(jobs); return -1; }
    int32_t per = nrep / nthreads, extra = nrep % nthreads, start = r0;
    for (int32_t t = 0; t < nthreads; ++t) {
        int32_t cnt = per + (t < extra ? 1 : 0);
        jobs[t] = (job){p, lq, k, start, start + cnt, r0, x_out, g_out};
        start += cnt;
        pthread_create(&th[t], NULL, worker, &jobs[t]);
    }
    for (int32_t t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    free(th);
    free(jobs);
    return 0;
}
