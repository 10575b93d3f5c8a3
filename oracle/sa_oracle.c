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
 *
 * Parallel tempering as the Ising machine inside the same loop (the machine is
 * interchangeable, Sec. III-B): chains of L replicas held at the fixed
 * temperatures of a ladder sweep exactly as above, and after every sweep the
 * replicas at adjacent ladder positions swap positions with the Metropolis
 * probability min(1, exp((beta_a - beta_b)(L_a - L_b))) of the product of
 * their Boltzmann laws; the energies L are evaluated from the Lagrangian's
 * definition.
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

/* clamp(floor((Z*B + 2^(S-1)) / 2^S)) for an explicit grid value B. */
static int32_t index_for(const oracle_prog *p, int64_t Z, int64_t B)
{
    i128 v = (i128)Z * (i128)B + ((i128)1 << (p->S - 1));
    i128 q = floor_div_pow2(v, p->S);
    if (q > THETA_HALF) q = THETA_HALF;
    if (q < -THETA_HALF) q = -THETA_HALF;
    return (int32_t)q;
}

/* D L_n(x) of the normalised Lagrangian (Eq. Lagrange_energy) from its
 * definition: -256 s_g^2 profit(x) + s_f Pq |g|^2 + s_f s_g lq.g, with
 * g = A x - b recomputed from x and the profit summed over every pair once. */
i128 oracle_energy(const oracle_prog *p, const uint8_t *x, const int32_t *lq)
{
    const int32_t n = p->n_ext;
    i128 profit = 0;
    for (int32_t i = 0; i < n; ++i) {
        if (!x[i]) continue;
        profit += p->h[i];
        for (int32_t j = i + 1; j < n; ++j)
            if (x[j]) profit += p->W[(int64_t)i * n + j];
    }
    i128 sq = 0, lg = 0;
    for (int32_t k = 0; k < p->m; ++k) {
        i128 g = -(i128)p->b[k];
        for (int32_t i = 0; i < n; ++i)
            if (x[i]) g += p->A[(int64_t)k * n + i];
        sq += g * g;
        lg += (i128)lq[k] * g;
    }
    return -(i128)256 * p->s_g * p->s_g * profit + (i128)p->s_f * p->pq * sq + (i128)p->s_f * p->s_g * lg;
}

/* oracle_energy as two 64-bit words (high signed, low unsigned) for callers
 * without a 128-bit type. */
void oracle_energy_words(const oracle_prog *p, const uint8_t *x, const int32_t *lq, int64_t *hi, uint64_t *lo)
{
    const i128 e = oracle_energy(p, x, lq);
    *hi = (int64_t)(e >> 64);
    *lo = (uint64_t)e;
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

/* ---- parallel tempering ---------------------------------------------------
 * Chain c holds replicas c L .. c L + L - 1, replica c L + j starting at ladder
 * position j.  Round k: every replica starts at x = 0; sweep t runs each
 * replica over all sites (the annealing draws above) at the grid value of its
 * current position, Bl[pos]; then for each position tau with tau = t (mod 2),
 * tau + 1 < L, the replicas a at tau and b at tau + 1 swap positions when
 *   j = floor(2 (Bl[tau] - Bl[tau+1]) (E_a - E_b) / 2^S) >= 0, or
 *   u24 < X[max(j, -XLEN + 1) + XLEN - 1],   X[i] = round(2^24 e^(i/256)),
 * where E = D L_n (oracle_energy) and 2 dB dE / 2^S = 256 (beta_tau -
 * beta_tau+1)(L_a - L_b) on the grid, u24 the top 24 bits of word 0 of
 * Philox(t, k | 2^31, c L + tau, instance).  slot_out[r] is replica r's final
 * position. */
#define XLEN 4609

typedef struct {
    const oracle_prog *p;
    const int32_t *lq;
    const int64_t *Bl;
    const int32_t *X;
    int32_t k, L, c0, c1;
    uint8_t *x_out;
    int64_t *g_out;
    int32_t *slot_out;
} pt_job;

static void pt_chain(const pt_job *j, int32_t c)
{
    const oracle_prog *p = j->p;
    const int32_t n = p->n_ext, L = j->L;
    const uint32_t nq = (uint32_t)((n + 3) / 4);
    const uint32_t key[2] = {(uint32_t)p->seed, (uint32_t)(p->seed >> 32)};
    int32_t owner[64], pos[64];
    for (int32_t q = 0; q < L; ++q) owner[q] = pos[q] = q;
    for (int32_t q = 0; q < L; ++q) {
        uint8_t *x = j->x_out + (int64_t)(c * L + q - j->c0 * L) * n;
        int64_t *g = j->g_out + (int64_t)(c * L + q - j->c0 * L) * p->m;
        memset(x, 0, (size_t)n);
        for (int32_t m = 0; m < p->m; ++m) g[m] = -p->b[m];
    }
    for (int32_t t = 0; t < p->T; ++t) {
        for (int32_t q = 0; q < L; ++q) {
            const int32_t r = c * L + q;
            uint8_t *x = j->x_out + (int64_t)(r - j->c0 * L) * n;
            int64_t *g = j->g_out + (int64_t)(r - j->c0 * L) * p->m;
            const int64_t B = j->Bl[pos[q]];
            uint32_t rnd[4] = {0, 0, 0, 0};
            for (int32_t i = 0; i < n; ++i) {
                if (i % 4 == 0) {
                    uint32_t ctr[4] = {(uint32_t)t * nq + (uint32_t)(i / 4), (uint32_t)j->k, (uint32_t)r, p->inst};
                    philox4x32_10(ctr, key, rnd);
                }
                uint32_t u24 = rnd[i % 4] >> 8;
                int64_t Z = oracle_local_field(p, x, g, j->lq, i);
                int32_t idx = index_for(p, Z, B);
                uint8_t xn = (uint8_t)(u24 < (uint32_t)p->theta[idx + THETA_HALF]);
                if (xn != x[i]) {
                    int64_t delta = (int64_t)xn - (int64_t)x[i];
                    for (int32_t m = 0; m < p->m; ++m) g[m] += delta * p->A[(int64_t)m * n + i];
                    x[i] = xn;
                }
            }
        }
        for (int32_t tau = t % 2; tau + 1 < L; tau += 2) {
            const int32_t a = owner[tau], b = owner[tau + 1];
            const uint8_t *xa = j->x_out + (int64_t)(c * L + a - j->c0 * L) * n;
            const uint8_t *xb = j->x_out + (int64_t)(c * L + b - j->c0 * L) * n;
            const i128 dE = oracle_energy(p, xa, j->lq) - oracle_energy(p, xb, j->lq);
            const i128 dB = (i128)j->Bl[tau] - (i128)j->Bl[tau + 1];
            const i128 q = floor_div_pow2(2 * dB * dE, p->S);
            int accept = q >= 0;
            if (!accept) {
                uint32_t ctr[4] = {(uint32_t)t, (uint32_t)j->k | 0x80000000u, (uint32_t)(c * L + tau), p->inst};
                uint32_t w[4];
                philox4x32_10(ctr, key, w);
                const int32_t i = q < -(XLEN - 1) ? 0 : (int32_t)q + XLEN - 1;
                accept = (w[0] >> 8) < (uint32_t)j->X[i];
            }
            if (accept) {
                owner[tau] = b;
                owner[tau + 1] = a;
                pos[a] = tau + 1;
                pos[b] = tau;
            }
        }
    }
    for (int32_t q = 0; q < L; ++q) j->slot_out[c * L + q - j->c0 * L] = pos[q];
}

static void *pt_worker(void *arg)
{
    pt_job *j = (pt_job *)arg;
    for (int32_t c = j->c0; c < j->c1; ++c) pt_chain(j, c);
    return NULL;
}

/* Chains c0 .. c0 + nchains - 1 of round k (replicas c0 L .. ), split over
 * nthreads POSIX threads.  Returns 0 on success. */
int oracle_pt_round(const oracle_prog *p, const int32_t *lq, int32_t k, int32_t L, const int64_t *Bl,
                    const int32_t *X, int32_t c0, int32_t nchains, uint8_t *x_out, int64_t *g_out,
                    int32_t *slot_out, int32_t nthreads)
{
    if (L < 2 || L > 64) return -1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > nchains) nthreads = nchains > 0 ? nchains : 1;
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    pt_job *jobs = (pt_job *)calloc((size_t)nthreads, sizeof(pt_job));
    if (!th || !jobs) { free(th); free(jobs); return -1; }
    int32_t per = nchains / nthreads, extra = nchains % nthreads, start = c0;
    for (int32_t t = 0; t < nthreads; ++t) {
        int32_t cnt = per + (t < extra ? 1 : 0);
        /* a job's outputs start at its own first chain */
        const int64_t off = (int64_t)(start - c0) * L;
        jobs[t] = (pt_job){p, lq, Bl, X, k, L, start, start + cnt, x_out + off * p->n_ext, g_out + off * p->m,
                           slot_out + off};
        start += cnt;
        pthread_create(&th[t], NULL, pt_worker, &jobs[t]);
    }
    for (int32_t t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    free(th);
    free(jobs);
    return 0;
}
