// Host side of libpbit: the instance compiler ("program the Ising machine")
// and the C ABI declared in include/pbit.h.
//
// Encoding (Sec. IV-A and IV-B): each constraint a_k.x <= b_k gets
// Q_k = floor(log2 b_k + 1) slack bits of weight 2^q so that it reads
// a_k.x + slack_k - b_k = 0; slack bits carry no profit.  The Lagrangian of
// Eq. Lagrange_energy (penalty of Eq. penalty_energy) in normalised units,
//   L_n = -profit/s_f + P_n |g|^2 / s_g^2 + lambda_n . g / s_g,
// with P_n = Pq/256, lambda_n = lq/256 and D = 256 s_f s_g^2, has the exact
// integer flip field Z_i = -D (L_n(x_i=1) - L_n(x_i=0))
//   = 256 s_g^2 (h_i + sum_j W_ij x_j) - 2 s_f Pq a_i.g - s_f s_g a_i.lq
//     - s_f Pq |a_i|^2 (1 - 2 x_i).
// Only the first and third terms vary per replica; the rest is folded into
// per-site constants K0_i (x_i = 0) and K1_i (x_i = 1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/pbit.h"
#include "pbit_types.h"
#include "net_layout.h"

namespace pbit {
hipError_t launch_sweep_quad(const DevInstance &d, int nb, int waves_per_block, hipStream_t stream);
hipError_t launch_sweep_quad_pc(const DevInstance &d, int nb, int producers, hipStream_t stream);
hipError_t launch_sweep_linear_pc_a(const DevInstance &d, bool wide, hipStream_t stream);
hipError_t launch_sweep_linear_pc_b(const DevInstance &d, bool wide, hipStream_t stream);
hipError_t launch_sweep_linear_pc_c(const DevInstance &d, bool wide, hipStream_t stream);
hipError_t launch_sweep_linear_pc_d(const DevInstance &d, bool wide, hipStream_t stream);
hipError_t launch_sweep_linear_a(const DevInstance &d, bool wide, int wpb, bool resident, hipStream_t stream);
hipError_t launch_sweep_linear_b(const DevInstance &d, bool wide, int wpb, bool resident, hipStream_t stream);
hipError_t launch_sweep_linear_c(const DevInstance &d, bool wide, int wpb, bool resident, hipStream_t stream);
hipError_t launch_sweep_linear_d(const DevInstance &d, bool wide, int wpb, bool resident, hipStream_t stream);
hipError_t launch_round_reduce(const DevInstance &d, hipStream_t stream);
hipError_t launch_lambda_update(const DevInstance &d, int mode, const int32_t *values,
                                hipStream_t stream);
hipError_t launch_round_reduce_batch(const DevInstance *insts, int count, hipStream_t stream);
hipError_t launch_lambda_update_batch(const DevInstance *insts, int count, int mode, hipStream_t stream);
hipError_t launch_reset_counter(int *counter, hipStream_t stream);
hipError_t launch_sweep_batch(bool linear, const DevInstance *insts, const int4 *items, int n_items, int *counter,
                              int blocks, size_t lds, hipStream_t stream);
hipError_t sweep_batch_prepare(bool linear, size_t lds, int *blocks_per_cu);
const void *sweep_batch_kernel(bool linear);
const void *round_reduce_batch_kernel();
const void *lambda_update_batch_kernel();
const void *reset_counter_kernel();
int reduce_threads();
int batch_linear_m(int m);
int batch_variant_code(int variant, int nb, int m);
hipError_t launch_lambda_set_batch(const DevInstance *insts, int count, const int32_t *values, hipStream_t stream);
hipError_t launch_batch_snapshot(const DevInstance *insts, int count, unsigned char *out, hipStream_t stream);
hipError_t net_launch_forward(const uint16_t *w, const uint16_t *x, const uint16_t *ctx, const int *set_rows,
                              const int *set_n, int S, int rows, uint16_t *H1, uint16_t *H2, uint16_t *Z,
                              uint16_t *G1, float *t, hipStream_t st);
hipError_t net_launch_backward(const uint16_t *w, const uint16_t *x, const int *set_rows, const int *set_n, int S,
                               int rows, const uint16_t *H1, const uint16_t *H2, const uint16_t *Z,
                               const uint16_t *G1, const float *t, const float *y, float *dP, float *partial,
                               int groups, float *grad, float *loss, hipStream_t st);
hipError_t net_launch_adam(float *wm, float *m, float *v, const float *g, uint16_t *wb, float lr, float b1,
                           float b2, float eps, float bc1, float bc2, hipStream_t st);
hipError_t net_launch_cast(const float *wm, uint16_t *wb, hipStream_t st);
hipError_t net_launch_to_lambda(const float *t, const double *scale, const int *dest, int S, int *lam,
                                hipStream_t st);
}  // namespace pbit

using namespace pbit;

namespace {

typedef __int128 i128;
typedef unsigned __int128 u128;

thread_local std::string g_error;

pbit_status fail(pbit_status st, const std::string &msg)
{
    g_error = msg;
    return st;
}

const i128 kZBudget = (i128)1 << 61;
const int64_t kLqCap = (int64_t)1 << 24;

// floor(num * 2^s / den) and the remainder, by binary long division.
u128 shifted_div(u128 num, int s, u128 den, u128 *rem)
{
    u128 q = num / den, r = num % den;
    for (int b = 0; b < s; ++b) {
        r <<= 1;
        q <<= 1;
        if (r >= den) {
            r -= den;
            q |= 1;
        }
    }
    *rem = r;
    return q;
}

// round(num * 2^s / den) half up, num >= 0.
u128 round_shifted(u128 num, int s, u128 den)
{
    u128 r;
    u128 q = shifted_div(num, s, den, &r);
    if (2 * r >= den) q += 1;
    return q;
}

int bit_length(int64_t v)
{
    int q = 0;
    while (v > 0) {
        ++q;
        v >>= 1;
    }
    return q;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Threshold table: round(2^24 / (1 + exp(-2 j / 256))) in 80-bit long double.
// X[i] = round(2^24 exp((i - 4608) / 256)): the Metropolis acceptance of a
// replica exchange on the 2^-8 grid of its exponent.
bool make_exchange_table(std::vector<int32_t> &x)
{
    x.resize(kXLen);
    for (int i = 0; i < kXLen; ++i) {
        const long double v = 16777216.0L * expl((long double)(i - (kXLen - 1)) / 256.0L);
        const long double fl = floorl(v);
        const long double fr = v - fl;
        if (i != kXLen - 1 && fabsl(fr - 0.5L) < 1e-9L) return false;  // too close to a tie to trust
        x[i] = (int32_t)fl + (fr > 0.5L ? 1 : 0);
    }
    return true;
}

bool make_theta(std::vector<int32_t> &t)
{
    t.resize(kThetaLen);
    for (int j = -kThetaHalf; j <= kThetaHalf; ++j) {
        const long double v = 16777216.0L / (1.0L + expl(-2.0L * (long double)j / 256.0L));
        const long double fl = floorl(v);
        const long double fr = v - fl;
        if (j != 0 && fabsl(fr - 0.5L) < 1e-9L) return false;  // too close to a tie to trust
        t[j + kThetaHalf] = (int32_t)fl + (fr > 0.5L ? 1 : 0);
    }
    return true;
}

struct Layout {
    size_t theta, btab, zsweep, bladder, xtab, J, acol, kbase, sa2, b, hprof, slack_off, slack_q;  // constants
    size_t kconst /* per-site records */, lam_acc, lam_q, round_k, G, best, best_x, feas;          // state
    size_t rx, rg, rprofit, rfeas, rslot;                                  // outputs
    size_t upload_end, total;
};

struct Plan {
    int kind = 0, n = 0, m = 0, n_ext = 0, n_pad = 0, words = 0, owords = 0, nb = 0;
    int variant = 0, T = 0, R = 0, S = 0, nq = 0;
    int64_t s_f = 1, s_g = 1, pq = 0, lq_max = 0;
    int32_t sg2 = 0, k2 = 0;       // scaled by 2^u
    int32_t zsh = 0, ish = 0, hclo = 0, hchi = 0;
    int64_t irnd = 0;
    int64_t sfsg = 0, eta_num = 0, lam_den = 1;
    int32_t eta_h = 0, eta_kcap = 0;
    int pt = 0;                    // parallel tempering chain length L (0: annealing)
    int samples = 0;               // samples per round the multiplier step averages (R, or R / L)
    int n_rec = 0;                 // per-site records (padding included)
    std::vector<int64_t> site;     // [n_rec][4]: K0, K1 (filled on the device), c, meta
    uint64_t seed = 0;
    uint32_t inst = 0;
    std::vector<int32_t> theta, btab, acol, hprof, slack_off, slack_q;
    std::vector<ZtSweep> zsweep;   // [T] field-threshold constants of the split kernels
    std::vector<int32_t> bladder;  // [64] parallel tempering ladder on the beta grid (first pt used)
    std::vector<int32_t> xtab;     // [kXLen] exchange acceptance 2^24 exp(j / 256), j = -4608 .. 0
    std::vector<int64_t> kbase, sa2, b;
    std::vector<int8_t> J;  // n_pad x (n_pad + 16)
    Layout L{};
};

pbit_status make_plan(const pbit_problem *p, const pbit_params *par, Plan &P)
{
    if (!p || !par) return fail(PBIT_EINVAL, "null problem or params");
    if (p->kind != PBIT_QKP && p->kind != PBIT_MKP) return fail(PBIT_EINVAL, "unknown problem kind");
    if (p->n < 1 || p->n > 4096) return fail(PBIT_EINVAL, "n must be in [1, 4096]");
    if (p->m < 1 || p->m > kMaxM) return fail(PBIT_EINVAL, "m must be in [1, 32]");
    if (!p->profit || !p->weight || !p->capacity) return fail(PBIT_EINVAL, "null problem array");
    if (par->replicas < 1 || par->replicas > (1 << 24)) return fail(PBIT_EINVAL, "replicas out of range");
    if (par->sweeps < 1 || par->sweeps > (1 << 24)) return fail(PBIT_EINVAL, "sweeps out of range");
    if (par->beta_num < 0 || par->beta_den < 1) return fail(PBIT_EINVAL, "beta must be a non-negative rational");
    if (par->eta_num < 0 || par->eta_den < 1) return fail(PBIT_EINVAL, "eta must be a non-negative rational");
    if (par->p_q < -1) return fail(PBIT_EINVAL, "p_q must be -1 or >= 0");
    if (par->p_q == -1 && (par->alpha_num < 0 || par->alpha_den < 1))
        return fail(PBIT_EINVAL, "alpha must be a non-negative rational");
    if (p->kind == PBIT_QKP && par->p_q == -1 && (p->density_num < 0 || p->density_den < 1))
        return fail(PBIT_EINVAL, "density must be a non-negative rational");
    if (par->pt_slots != 0) {
        const int L = par->pt_slots;
        if (p->kind != PBIT_QKP) return fail(PBIT_EINVAL, "parallel tempering is built for the quadratic kernel");
        if (L < 2 || L > 64 || 64 % L != 0 || par->replicas % L != 0)
            return fail(PBIT_EINVAL, "pt_slots must divide 64 and the replica count, and be >= 2");
        if (par->beta_num == 0 || par->fixed_beta)
            return fail(PBIT_EINVAL, "parallel tempering needs beta_max > 0 and no fixed-beta mode");
    }

    const int n = p->n, m = p->m;
    P.kind = p->kind;
    P.n = n;
    P.m = m;
    P.T = par->sweeps;
    P.R = par->replicas;
    P.seed = par->seed;
    P.inst = par->instance_id;
    P.pt = par->pt_slots;
    P.samples = P.pt ? P.R / P.pt : P.R;

    // item data
    std::vector<int64_t> h(n, 0);
    std::vector<int32_t> W;  // n x n, zero diagonal (quadratic only)
    int64_t s_f = 0;
    if (p->kind == PBIT_QKP) {
        W.assign((size_t)n * n, 0);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const int32_t v = p->profit[(size_t)i * n + j];
                if (v != p->profit[(size_t)j * n + i]) return fail(PBIT_EINVAL, "QKP profit matrix is not symmetric");
                if (v < -127 || v > 127) return fail(PBIT_ERANGE, "QKP profits must lie in [-127, 127]");
                s_f = std::max<int64_t>(s_f, std::llabs(v));
                if (i == j) h[i] = v;
                else W[(size_t)i * n + j] = v;
            }
    } else {
        for (int i = 0; i < n; ++i) {
            h[i] = p->profit[i];
            s_f = std::max<int64_t>(s_f, std::llabs(h[i]));
        }
    }
    P.s_f = std::max<int64_t>(s_f, 1);

    int64_t s_g = 0;
    for (int k = 0; k < m; ++k) {
        const int64_t bk = p->capacity[k];
        if (bk < 0 || bk >= ((int64_t)1 << 31)) return fail(PBIT_ERANGE, "capacities must lie in [0, 2^31)");
        s_g = std::max(s_g, bk);
        for (int i = 0; i < n; ++i) {
            const int32_t a = p->weight[(size_t)k * n + i];
            if (a < 0) return fail(PBIT_EINVAL, "weights must be non-negative");
            s_g = std::max<int64_t>(s_g, a);
        }
    }
    P.s_g = std::max<int64_t>(s_g, 1);

    // slack extension
    std::vector<int> Q(m);
    int n_ext = n;
    P.slack_off.resize(m);
    P.slack_q.resize(m);
    P.b.resize(m);
    for (int k = 0; k < m; ++k) {
        Q[k] = bit_length(p->capacity[k]);
        P.slack_off[k] = n_ext;
        P.slack_q[k] = Q[k];
        P.b[k] = p->capacity[k];
        n_ext += Q[k];
    }
    P.n_ext = n_ext;
    P.words = (n_ext + 31) / 32;
    P.owords = (n + 31) / 32;
    P.nq = (n_ext + 3) / 4;
    if (P.words > kMaxWords) return fail(PBIT_ERANGE, "more than 2048 spins");
    // Philox counter word 0 is t * nq + i / 4 (uint32): a wrap would replay
    // earlier sweeps' draws instead of a fresh one per update (Sec. III-B)
    if ((uint64_t)P.T * (uint64_t)P.nq > ((uint64_t)1 << 32))
        return fail(PBIT_ERANGE, "sweeps x ceil(n_ext / 4) exceed the 32-bit Philox counter word");
    P.n_rec = P.words * 32 + 32;
    P.acol.assign((size_t)P.n_rec * m, 0);
    for (int k = 0; k < m; ++k) {
        for (int i = 0; i < n; ++i) P.acol[(size_t)i * m + k] = p->weight[(size_t)k * n + i];
        for (int q = 0; q < Q[k]; ++q) P.acol[(size_t)(P.slack_off[k] + q) * m + k] = 1 << q;
    }

    // penalty: 256*P given, or the rule P = alpha d N (N counts slack spins)
    if (par->p_q >= 0) {
        P.pq = par->p_q;
    } else {
        i128 num, den;
        if (p->kind == PBIT_QKP) {
            num = (i128)256 * par->alpha_num * p->density_num * n_ext;
            den = (i128)par->alpha_den * p->density_den;
        } else {
            num = (i128)256 * par->alpha_num * 2 * n_ext;
            den = (i128)par->alpha_den * (n_ext + 1);
        }
        const i128 v = (2 * num + den) / (2 * den);
        if (v >= ((i128)1 << 40)) return fail(PBIT_ERANGE, "penalty too large");
        P.pq = (int64_t)v;
    }

    // bounds of the exact fields: |Z| < 2^62 for every state and |lambda_q| <= lq_max
    int64_t amax = 0, sqmax = 0, gmax = 0, fmax = 0;
    std::vector<int64_t> gmk(m);
    for (int k = 0; k < m; ++k) {
        int64_t tot = 0;
        for (int i = 0; i < n_ext; ++i) tot += P.acol[(size_t)i * m + k];
        gmk[k] = std::max<int64_t>(P.b[k], tot - P.b[k]);
        gmax = std::max(gmax, gmk[k]);
    }
    for (int i = 0; i < n_ext; ++i) {
        int64_t e = 0, sq = 0;
        for (int k = 0; k < m; ++k) {
            const int64_t a = P.acol[(size_t)i * m + k];
            e += a;
            sq += a * a;
        }
        amax = std::max(amax, e);
        sqmax = std::max(sqmax, sq);
        int64_t f = i < n ? std::llabs(h[i]) : 0;
        if (i < n && !W.empty())
            for (int j = 0; j < n; ++j) f += std::llabs(W[(size_t)i * n + j]);
        fmax = std::max(fmax, f);
    }
    const i128 sg2 = (i128)P.s_g * P.s_g;
    const i128 zmax0 = (i128)256 * sg2 * fmax + (i128)P.s_f * P.pq * ((i128)2 * amax * gmax + sqmax);
    if (zmax0 >= kZBudget) return fail(PBIT_ERANGE, "instance fields exceed the 2^61 budget");
    if (amax == 0) {
        P.lq_max = kLqCap;
    } else {
        const i128 lq = (kZBudget - zmax0) / ((i128)P.s_f * P.s_g * amax);
        P.lq_max = (int64_t)std::min<i128>(lq, kLqCap);
    }
    if (P.lq_max < 256) return fail(PBIT_ERANGE, "multiplier range below 1.0");

    // kernel variant and its narrower integer paths
    if (p->kind == PBIT_QKP) {
        if (m != 1) return fail(PBIT_ERANGE, "quadratic instances take exactly one constraint");
        if (n_ext > kMaxQuadBlocks * 32) return fail(PBIT_ERANGE, "quadratic instances need n_ext <= 352");
        if (sg2 >= ((i128)1 << 31)) return fail(PBIT_ERANGE, "quadratic instances need s_g^2 < 2^31");
        if ((i128)amax * gmax >= ((i128)1 << 31) || amax >= (1 << 23) || gmax >= (1 << 23))
            return fail(PBIT_ERANGE, "residual products exceed the 24-bit multiply path");
        P.variant = kQuad;
        P.nb = (n_ext + 31) / 32;
        P.n_pad = P.nb * 32;
    } else {
        bool narrow = gmax < ((int64_t)1 << 23);
        for (int i = 0; i < n && narrow; ++i) {
            i128 s = 0;
            for (int k = 0; k < m; ++k) {
                const int64_t a = P.acol[(size_t)i * m + k];
                if (a >= ((int64_t)1 << 23)) narrow = false;
                s += (i128)a * gmk[k];
            }
            if (s >= ((i128)1 << 31)) narrow = false;
        }
        P.variant = narrow ? kLinear : kLinearWide;
        P.n_pad = P.words * 32;
    }
    const i128 k2 = (i128)2 * P.s_f * P.pq;
    P.sfsg = P.s_f * P.s_g;

    // multiplier step: acc += round(2^32 eta_num G / (eta_den R' s_g)), G <= R' gmax, R'
    // the samples per round
    const i128 lam_den = (i128)par->eta_den * P.samples * P.s_g;
    if ((i128)par->eta_num * P.samples * gmax >= ((i128)1 << 62) || lam_den >= ((i128)1 << 62))
        return fail(PBIT_ERANGE, "multiplier step exceeds 64-bit bounds");
    if (((i128)par->eta_num * gmax << 32) >= ((i128)1 << 62) * par->eta_den * P.s_g)
        return fail(PBIT_ERANGE, "multiplier step too large");
    P.eta_num = par->eta_num;
    P.lam_den = (int64_t)lam_den;
    // diminishing step eta H / (H + k): numerator eta_num G H, denominator lam_den (H + k)
    if (par->eta_decay_rounds < 0 || par->eta_decay_rounds > (1 << 20))
        return fail(PBIT_EINVAL, "eta_decay_rounds must lie in [0, 2^20]");
    P.eta_h = par->eta_decay_rounds;
    if (P.eta_h > 0) {
        if ((i128)par->eta_num * P.samples * gmax * P.eta_h >= ((i128)1 << 62))
            return fail(PBIT_ERANGE, "diminishing multiplier step exceeds 64-bit bounds");
        const i128 kc = (((i128)1 << 62) - 1) / lam_den - P.eta_h;
        if (kc < 1) return fail(PBIT_ERANGE, "diminishing multiplier step exceeds 64-bit bounds");
        P.eta_kcap = (int32_t)std::min<i128>(kc, (i128)INT32_MAX);
    }

    // beta grid: B_t = round(2^S beta_t / (2 s_f s_g^2)), S the smallest giving B_{T-1} >= 2^30
    const u128 den = (u128)2 * P.s_f * (u128)sg2;
    const bool flat = par->fixed_beta || P.T == 1;
    P.btab.assign(P.T, 0);
    if (par->beta_num == 0) {
        P.S = 32;
    } else {
        int S = 1;
        while (round_shifted((u128)par->beta_num, S, den * (u128)par->beta_den) < ((u128)1 << 30)) {
            if (++S > 94) return fail(PBIT_ERANGE, "beta grid shift out of range");
        }
        P.S = S;
        for (int t = 0; t < P.T; ++t) {
            u128 v;
            if (flat) v = round_shifted((u128)par->beta_num, S, den * (u128)par->beta_den);
            else v = round_shifted((u128)par->beta_num * (u128)t, S, den * (u128)par->beta_den * (u128)(P.T - 1));
            P.btab[t] = (int32_t)v;
        }
    }

    // The kernels carry 2^u Z with S + u >= 34 so that the index needs one
    // 64-bit shift (see theta_index); u > 0 only for instances of tiny scale.
    const int zsh = P.S >= 34 ? 0 : 34 - P.S;
    const i128 zfull = zmax0 + (i128)P.s_f * P.s_g * amax * P.lq_max;
    if ((zfull << zsh) >= ((i128)1 << 62)) return fail(PBIT_ERANGE, "scaled fields exceed 2^62");
    if ((k2 << zsh) >= ((i128)1 << 31)) return fail(PBIT_ERANGE, "2 s_f Pq must stay below 2^31");
    if (P.variant == kQuad && (sg2 << zsh) >= ((i128)1 << 31))
        return fail(PBIT_ERANGE, "quadratic instances need s_g^2 < 2^31");
    P.zsh = zsh;
    P.k2 = (int32_t)(k2 << zsh);
    P.sg2 = (int32_t)std::min<i128>(sg2 << zsh, INT32_MAX);
    P.ish = P.S + zsh - 32;
    P.irnd = (int64_t)1 << (P.S + zsh - 33);
    // split kernels: threshold on the carried field, Zt = ceil(n 2^E / B_t),
    // E = ish + 31, from A = floor(2^E / B_t) and rho = 2^E mod B_t (field_threshold)
    P.zsweep.assign(P.T, ZtSweep{});
    {
        const int E = P.ish + 31;
        if (E > 126) return fail(PBIT_ERANGE, "beta grid shift out of range");
        for (int t = 0; t < P.T; ++t) {
            ZtSweep &z = P.zsweep[t];
            const int32_t B = P.btab[t];
            if (B <= 0) {
                z.sat = 1;
                continue;
            }
            const u128 A = ((u128)1 << E) / (u128)B;
            if (A >= ((u128)1 << 62)) {
                z.sat = 1;
                continue;
            }
            const u128 rho = ((u128)1 << E) % (u128)B;
            z.fast = A < ((u128)1 << 48) ? 1 : 0;
            z.a_hi = (int32_t)(A >> 31);
            z.a_lo = (int32_t)(A & 0x7FFFFFFFu);
            z.rho = (int32_t)rho;
            z.bt = B;
            z.rb = (double)(int32_t)rho / (double)B;
        }
    }
    if (P.ish <= 31) {
        P.hclo = -(int32_t)(1u << (P.ish - 1));
        P.hchi = (int32_t)((1u << (P.ish - 1)) - 1u);
    } else {
        P.hclo = INT32_MIN;
        P.hchi = INT32_MAX;
    }

    // parallel tempering: ladder beta_max (j + 1) / L on the beta grid, exchange
    // table, and the multiplier range narrowed so that every energy difference
    // D (L(x) - L(0)), carried as 2^u, stays below 2^61
    P.bladder.assign(64, 0);
    P.xtab.assign(kXLen, 0);
    if (P.pt) {
        const u128 den = (u128)2 * P.s_f * (u128)sg2;
        for (int j = 0; j < P.pt; ++j)
            P.bladder[j] = (int32_t)round_shifted((u128)par->beta_num * (u128)(j + 1), P.S,
                                                  den * (u128)par->beta_den * (u128)P.pt);
        if (!make_exchange_table(P.xtab)) return fail(PBIT_ERANGE, "exchange table rounding undecidable");
        i128 prof = 0;
        for (int i = 0; i < n; ++i) prof += std::llabs(h[i]);
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) prof += std::llabs(W[(size_t)i * n + j]);
        i128 sq = 0, lin = 0;
        for (int k = 0; k < m; ++k) {
            sq += (i128)gmk[k] * gmk[k] + (i128)P.b[k] * P.b[k];
            lin += (i128)gmk[k] + P.b[k];
        }
        const i128 room = (kZBudget >> zsh) - ((i128)256 * sg2 * prof + (i128)P.s_f * P.pq * sq);
        if (room <= 0) return fail(PBIT_ERANGE, "parallel tempering energies exceed the 2^61 budget");
        const i128 lam = (i128)P.s_f * P.s_g * lin;
        if (lam > 0) P.lq_max = (int64_t)std::min<i128>(P.lq_max, room / lam);
        if (P.lq_max < 256) return fail(PBIT_ERANGE, "multiplier range below 1.0");
    }

    // per-site records: c_i = change of Z_i when the preceding visit (site i-1)
    // goes 0 -> 1; meta = (a_i, -1 for a site the loop visits, 0 for padding)
    P.site.assign((size_t)P.n_rec * 4, 0);
    for (int i = 1; i < n_ext; ++i) {
        const bool quad = P.variant == kQuad;
        bool chained;
        if (quad) chained = (i % 32) != 0;
        else if (i < n) chained = (i % 32) != 0;
        else {
            // slack bit q >= 1 of the same constraint
            int k = 0;
            while (k + 1 < m && i >= P.slack_off[k + 1]) ++k;
            chained = i > P.slack_off[k] && i < P.slack_off[k] + P.slack_q[k];
        }
        if (!chained) continue;
        i128 aa = 0;
        for (int k = 0; k < m; ++k) aa += (i128)P.acol[(size_t)i * m + k] * P.acol[(size_t)(i - 1) * m + k];
        i128 c = -k2 * aa;
        if (quad && i < n && i - 1 < n) c += (i128)256 * sg2 * W[(size_t)i * n + (i - 1)];
        P.site[(size_t)i * 4 + 2] = (int64_t)(c << zsh);
    }
    for (int i = 0; i < P.n_rec; ++i) {
        const bool visited = P.variant == kQuad ? i < n_ext : i < n;
        const int32_t a = (P.variant == kQuad && i < n_ext) ? P.acol[(size_t)i * m] : 0;
        P.site[(size_t)i * 4 + 3] = (int64_t)(((uint64_t)(visited ? 0xFFFFFFFFu : 0u) << 32) | (uint32_t)a);
    }

    // per-site constants independent of lambda
    P.kbase.resize(n_ext);
    P.sa2.resize(n_ext);
    for (int i = 0; i < n_ext; ++i) {
        int64_t sq = 0;
        for (int k = 0; k < m; ++k) {
            const int64_t a = P.acol[(size_t)i * m + k];
            sq += a * a;
        }
        const i128 Sa = (i128)P.s_f * P.pq * sq;
        const int64_t hi = i < n ? h[i] : 0;
        P.kbase[i] = (int64_t)((i128)256 * sg2 * hi - Sa);
        P.sa2[i] = (int64_t)(2 * Sa);
    }
    P.hprof.resize(n);
    for (int i = 0; i < n; ++i) P.hprof[i] = (int32_t)h[i];
    if (P.variant == kQuad) {
        // slabs of 32 rows (row stride n_pad + 16 bytes), slab stride 1 KB x (nb + 1).
        // The diagonal 32 x 32 chunk of a slab is split in two: its strictly lower
        // part (j < i, the in-block corrections with the current states) stays in
        // place; the rest (j >= i, the block-start field) goes to the spare bytes,
        // columns 0..15 of row r into the row's 16 padding bytes, columns 16..31
        // into the slab's tail at 32 ls + 16 r.
        const int ls = P.n_pad + 16;
        const size_t slab = (size_t)1024 * (P.nb + 1);
        P.J.assign((size_t)P.nb * slab, 0);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const int r = i % 32, cj = j % 32;
                size_t at = (size_t)r * ls + j;
                if (j / 32 == i / 32 && cj >= r)
                    at = cj < 16 ? (size_t)r * ls + P.n_pad + cj : (size_t)32 * ls + (size_t)r * 16 + (cj - 16);
                P.J[(size_t)(i / 32) * slab + at] = (int8_t)W[(size_t)i * n + j];
            }
    }
    if (!make_theta(P.theta)) return fail(PBIT_ERANGE, "threshold table rounding undecidable");

    // workspace layout
    Layout &L = P.L;
    size_t o = 0;
    auto put = [&o](size_t bytes) {
        const size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    L.theta = put(kThetaLen * 4);
    L.btab = put((size_t)P.T * 4);
    L.zsweep = put((size_t)P.T * sizeof(ZtSweep));
    L.bladder = put(64 * 4);
    L.xtab = put((size_t)kXLen * 4);
    L.J = put(P.J.size());
    L.acol = put(P.acol.size() * 4);
    L.kbase = put((size_t)n_ext * 8);
    L.sa2 = put((size_t)n_ext * 8);
    L.b = put((size_t)m * 8);
    L.hprof = put((size_t)n * 4);
    L.slack_off = put((size_t)m * 4);
    L.slack_q = put((size_t)m * 4);
    L.lam_acc = put((size_t)m * 8);
    L.lam_q = put((size_t)m * 4);
    L.round_k = put(4);
    L.G = put((size_t)m * 8);
    L.best = put(4 * 8);
    L.best_x = put((size_t)P.words * 4);
    L.feas = put(4);
    L.kconst = put((size_t)P.n_rec * 32);
    L.upload_end = o;
    L.rx = put((size_t)P.R * P.words * 4);
    L.rg = put((size_t)P.R * m * 4);
    L.rprofit = put((size_t)P.R * 8);
    L.rfeas = put((size_t)P.R * 4);
    L.rslot = put((size_t)P.R * 4);
    L.total = o;
    return PBIT_OK;
}

void fill_plan_info(const Plan &P, pbit_plan_info *out)
{
    std::memset(out, 0, sizeof(*out));
    out->n = P.n;
    out->m = P.m;
    out->n_ext = P.n_ext;
    out->n_pad = P.n_pad;
    out->words = P.words;
    out->s_f = P.s_f;
    out->s_g = P.s_g;
    out->p_q = P.pq;
    out->shift = P.S;
    out->lq_max = (int32_t)P.lq_max;
    out->variant = P.variant;
    out->workspace_bytes = P.L.total;
    size_t o = 0;
    auto put = [&o](size_t bytes) {
        const size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    out->out_x = put((size_t)P.R * P.words * 4);
    out->out_g = put((size_t)P.R * P.m * 4);
    out->out_profit = put((size_t)P.R * 8);
    out->out_feasible = put((size_t)P.R * 4);
    out->out_G = put((size_t)P.m * 8);
    out->out_lambda = put((size_t)P.m * 4);
    out->out_round = put(4);
    out->out_sat = put(4);
    out->out_slot = put((size_t)P.R * 4);
    out->out_bytes = o;
}

const size_t kMaxLds = 160 * 1024;

// LDS of the producer/consumer linear kernel.
size_t linear_split_bytes(const Plan &P)
{
    return (size_t)kThetaBytes + kRingBytes + (size_t)(32 * P.words + 32) * 16 +
           (size_t)P.owords * 32 * P.m * 4 + (size_t)P.words * kWave * 4;
}

// LDS of the linear kernel with LDS-resident site constants for wpb waves.
size_t resident_bytes(const Plan &P, int wpb)
{
    return (size_t)kThetaBytes + (size_t)(32 * P.words + 32) * 16 + (size_t)P.owords * 32 * P.m * 4 +
           (size_t)wpb * P.words * kWave * 4;
}

int waves_per_block_default(const Plan &P)
{
    if (const char *e = std::getenv("PBIT_WAVES_PER_BLOCK")) {
        const int v = std::atoi(e);
        if (v >= 1 && v <= 4) return v;
    }
    const int waves = (P.R + kWave - 1) / kWave;
    return waves <= 256 ? 1 : 4;
}

}  // namespace

struct pbit_instance {
    Plan plan;
    DevInstance dev{};
    std::vector<unsigned char> upload;
    int device = 0;
    int wpb = 1;
    int resident = -1;    // linear kernels: 1 LDS-resident constants, 0 global, -1 whichever fits
    int split = -1;       // 1 producer/consumer workgroups, 0 not, -1 when CUs would idle (and LDS fits)
    int cus = 256;
    bool broken = false;
    bool member = false;  // owned by a batch
    int static_dev = -1;  // device whose static workspace this instance holds (-1: caller's workspace)
};

struct pbit_batch {
    std::vector<pbit_instance *> members;
    std::vector<DevInstance> dev;      // host image of the device record array
    std::vector<int4> items;           // host image of the work queue
    std::vector<int32_t> rounds;       // initial budgets
    DevInstance *d_insts = nullptr;
    int4 *d_items = nullptr;
    int *d_counter = nullptr;          // [2]: quadratic, linear queue
    int n_quad = 0;                    // items [0, n_quad) quadratic, the rest linear
    int blocks_lin = 0;
    size_t lds_lin = 0;
    int32_t *d_rounds = nullptr;
    int split_percent = 200, n_split = 0;
    int blocks = 0;
    size_t lds = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool broken = false;
    ~pbit_batch()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (pbit_instance *m : members) delete m;
    }
};

namespace {

pbit_status device_error(pbit_instance *inst, hipError_t e, const char *what)
{
    if (inst) inst->broken = true;
    return fail(PBIT_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

pbit_status check_live(pbit_instance *inst)
{
    if (!inst) return fail(PBIT_EINVAL, "null instance");
    if (inst->broken) return fail(PBIT_ESTATE, "instance is unusable after a device error");
    return PBIT_OK;
}

}  // namespace

namespace {
pbit_status create_impl(const pbit_problem *prob, const pbit_params *par, void *dev_ws, size_t ws_bytes,
                        pbit_stream stream, pbit_instance **out)
{
    if (!out) return fail(PBIT_EINVAL, "null output handle");
    pbit_instance *inst = new (std::nothrow) pbit_instance();
    if (!inst) return fail(PBIT_EINVAL, "host allocation failed");
    pbit_status st = make_plan(prob, par, inst->plan);
    if (st != PBIT_OK) {
        delete inst;
        return st;
    }
    const Plan &P = inst->plan;
    if (!dev_ws || (reinterpret_cast<uintptr_t>(dev_ws) & 255) != 0 || ws_bytes < P.L.total) {
        delete inst;
        return fail(PBIT_EWORKSPACE, "workspace missing, misaligned or smaller than pbit_workspace_bytes");
    }
    hipError_t e = hipGetDevice(&inst->device);
    hipDeviceProp_t prop;
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, inst->device);
    if (e != hipSuccess) {
        delete inst;
        return fail(PBIT_EDEVICE, std::string("device query failed: ") + hipGetErrorString(e));
    }
    inst->cus = prop.multiProcessorCount;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        delete inst;
        return fail(PBIT_EDEVICE, std::string("libpbit is built for gfx950, device is ") + prop.gcnArchName);
    }

    // host image of constants and initial state
    const Layout &L = P.L;
    inst->upload.assign(L.upload_end, 0);
    unsigned char *img = inst->upload.data();
    auto cp = [img](size_t off, const void *src, size_t bytes) {
        if (bytes) std::memcpy(img + off, src, bytes);
    };
    cp(L.theta, P.theta.data(), P.theta.size() * 4);
    cp(L.btab, P.btab.data(), P.btab.size() * 4);
    cp(L.zsweep, P.zsweep.data(), P.zsweep.size() * sizeof(ZtSweep));
    cp(L.bladder, P.bladder.data(), P.bladder.size() * 4);
    cp(L.xtab, P.xtab.data(), P.xtab.size() * 4);
    cp(L.J, P.J.data(), P.J.size());
    cp(L.acol, P.acol.data(), P.acol.size() * 4);
    cp(L.kbase, P.kbase.data(), P.kbase.size() * 8);
    cp(L.sa2, P.sa2.data(), P.sa2.size() * 8);
    cp(L.b, P.b.data(), P.b.size() * 8);
    cp(L.hprof, P.hprof.data(), P.hprof.size() * 4);
    cp(L.slack_off, P.slack_off.data(), P.slack_off.size() * 4);
    cp(L.slack_q, P.slack_q.data(), P.slack_q.size() * 4);
    cp(L.kconst, P.site.data(), P.site.size() * 8);
    const int64_t best0[4] = {INT64_MIN, 0, 0, 0};
    cp(L.best, best0, sizeof(best0));

    unsigned char *base = static_cast<unsigned char *>(dev_ws);
    DevInstance &d = inst->dev;
    d.J = reinterpret_cast<const int8_t *>(base + L.J);
    d.theta = reinterpret_cast<const int32_t *>(base + L.theta);
    d.Btab = reinterpret_cast<const int32_t *>(base + L.btab);
    d.zsweep = reinterpret_cast<const ZtSweep *>(base + L.zsweep);
    d.bladder = reinterpret_cast<const int32_t *>(base + L.bladder);
    d.xtab = reinterpret_cast<const int32_t *>(base + L.xtab);
    d.rslot = reinterpret_cast<int32_t *>(base + L.rslot);
    d.pt = P.pt;
    d.acol = reinterpret_cast<const int32_t *>(base + L.acol);
    d.kbase = reinterpret_cast<const int64_t *>(base + L.kbase);
    d.sa2 = reinterpret_cast<const int64_t *>(base + L.sa2);
    d.b = reinterpret_cast<const int64_t *>(base + L.b);
    d.hprof = reinterpret_cast<const int32_t *>(base + L.hprof);
    d.slack_off = reinterpret_cast<const int32_t *>(base + L.slack_off);
    d.slack_q = reinterpret_cast<const int32_t *>(base + L.slack_q);
    d.site = reinterpret_cast<int64_t *>(base + L.kconst);
    d.lam_acc = reinterpret_cast<int64_t *>(base + L.lam_acc);
    d.lam_q = reinterpret_cast<int32_t *>(base + L.lam_q);
    d.round_k = reinterpret_cast<int32_t *>(base + L.round_k);
    d.G = reinterpret_cast<int64_t *>(base + L.G);
    d.best = reinterpret_cast<int64_t *>(base + L.best);
    d.best_x = reinterpret_cast<uint32_t *>(base + L.best_x);
    d.feas_count = reinterpret_cast<int32_t *>(base + L.feas);
    d.lam_sat = reinterpret_cast<uint32_t *>(base + L.feas + 4);  // same 256-byte slot
    d.rx = reinterpret_cast<uint32_t *>(base + L.rx);
    d.rg = reinterpret_cast<int32_t *>(base + L.rg);
    d.rprofit = reinterpret_cast<int64_t *>(base + L.rprofit);
    d.rfeas = reinterpret_cast<int32_t *>(base + L.rfeas);
    d.n = P.n;
    d.m = P.m;
    d.n_ext = P.n_ext;
    d.n_pad = P.n_pad;
    d.words = P.words;
    d.owords = P.owords;
    d.R = P.R;
    d.T = P.T;
    d.S = P.S;
    d.nq = P.nq;
    d.sg2 = P.sg2;
    d.k2 = P.k2;
    d.zsh = P.zsh;
    d.ish = P.ish;
    d.irnd = P.irnd;
    d.hclo = P.hclo;
    d.hchi = P.hchi;
    d.sfsg = P.sfsg;
    d.lq_max = P.lq_max;
    d.eta_num = P.eta_num;
    d.eta_h = P.eta_h;
    d.eta_kcap = P.eta_kcap;
    d.lam_den = P.lam_den;
    d.seed_lo = (uint32_t)P.seed;
    d.seed_hi = (uint32_t)(P.seed >> 32);
    d.inst_id = P.inst;
    inst->wpb = waves_per_block_default(P);

    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    e = hipMemcpyAsync(dev_ws, inst->upload.data(), L.upload_end, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_lambda_update(d, 0, nullptr, s);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) {
        pbit_status r = device_error(nullptr, e, "instance upload failed");
        delete inst;
        return r;
    }
    *out = inst;
    return PBIT_OK;
}


// Multi-knapsack members are padded to a constraint count with a batch body.
struct PaddedProblem {
    pbit_problem prob{};
    std::vector<int32_t> weight;
    std::vector<int64_t> capacity;
};

struct BatchSizes {
    std::vector<PaddedProblem> padded;
    std::vector<size_t> member_bytes, off_member;
    size_t off_insts = 0, off_items = 0, off_counter = 0, off_rounds = 0, total = 0;
};

pbit_status batch_sizes(const pbit_problem *probs, const pbit_params *params, int count, BatchSizes &z)
{
    if (!probs || !params || count < 1) return fail(PBIT_EINVAL, "null arrays or count < 1");
    z.padded.resize(count);
    size_t items = 0;
    for (int i = 0; i < count; ++i) {
        PaddedProblem &pp = z.padded[i];
        pp.prob = probs[i];
        const pbit_problem &p = probs[i];
        if (p.kind == PBIT_MKP && p.m >= 1 && p.m <= kMaxM && p.n >= 1 && p.weight && p.capacity) {
            const int mb = batch_linear_m(p.m);
            if (mb != p.m) {
                pp.weight.assign((size_t)mb * p.n, 0);
                std::memcpy(pp.weight.data(), p.weight, (size_t)p.m * p.n * 4);
                pp.capacity.assign(mb, 0);
                std::memcpy(pp.capacity.data(), p.capacity, (size_t)p.m * 8);
                pp.prob.m = mb;
                pp.prob.weight = pp.weight.data();
                pp.prob.capacity = pp.capacity.data();
            }
        }
        Plan P;
        pbit_status st = make_plan(&pp.prob, &params[i], P);
        if (st != PBIT_OK) {
            g_error = "member " + std::to_string(i) + ": " + g_error;
            return st;
        }
        if (P.pt) return fail(PBIT_EINVAL, "member " + std::to_string(i) + ": parallel tempering runs as single instances");
        if (batch_variant_code(P.variant, P.nb, P.m) < 0 ||
            (P.variant != kQuad && resident_bytes(P, 4) > kMaxLds))
            return fail(PBIT_ERANGE, "member " + std::to_string(i) + ": no batch body for this instance shape");
        z.member_bytes.push_back(P.L.total);
        items += (size_t)(P.variant == kQuad ? (P.R + 255) / 256 : (P.R + 63) / 64);  // split tiles hold 64
    }
    size_t o = 0;
    auto put = [&o](size_t bytes) {
        const size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    z.off_insts = put((size_t)count * sizeof(DevInstance));
    z.off_items = put(items * sizeof(int4));
    z.off_counter = put(8);
    z.off_rounds = put((size_t)count * 4);
    for (int i = 0; i < count; ++i) z.off_member.push_back(put(z.member_bytes[i]));
    z.total = o;
    return PBIT_OK;
}

pbit_status check_batch(pbit_batch *b)
{
    if (!b) return fail(PBIT_EINVAL, "null batch");
    if (b->broken) return fail(PBIT_ESTATE, "batch is unusable after a device error");
    return PBIT_OK;
}

pbit_status batch_error(pbit_batch *b, hipError_t e, const char *what)
{
    b->broken = true;
    for (pbit_instance *m : b->members) m->broken = true;
    return fail(PBIT_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// One batch round as a graph of kernel nodes: counter reset, the two family
// kernels side by side, round reduce, multiplier step (the work-queue
// counters are cleared by a kernel, not a memset node).
hipError_t build_round_graph(pbit_batch *b)
{
    hipGraph_t g = nullptr;
    hipError_t e = hipGraphCreate(&g, 0);
    if (e != hipSuccess) return e;
    DevInstance *insts = b->d_insts;
    int4 *items_q = b->d_items;
    int4 *items_l = b->d_items + b->n_quad;
    int *counter_q = b->d_counter;
    int *counter_l = b->d_counter + 1;
    int n_quad = b->n_quad;
    int n_lin = (int)b->items.size() - b->n_quad;
    int mode = 1;
    void *a_reset[] = {&counter_q};
    void *a_lin[] = {&insts, &items_l, &n_lin, &counter_l};
    void *a_quad[] = {&insts, &items_q, &n_quad, &counter_q};
    void *a_reduce[] = {&insts};
    void *a_lambda[] = {&insts, &mode};
    const int count = (int)b->members.size();
    auto add = [&](const void *func, dim3 grid, dim3 block, size_t lds, void **args, const hipGraphNode_t *deps,
                   size_t ndeps, hipGraphNode_t *node) {
        hipKernelNodeParams p{};
        p.func = const_cast<void *>(func);
        p.gridDim = grid;
        p.blockDim = block;
        p.sharedMemBytes = (unsigned)lds;
        p.kernelParams = args;
        p.extra = nullptr;
        return hipGraphAddKernelNode(node, g, deps, ndeps, &p);
    };
    // reset -> {linear family, quadratic family} -> reduce -> multiplier step;
    // the two family kernels are independent nodes and run side by side
    hipGraphNode_t reset = nullptr, sweeps[2] = {nullptr, nullptr}, reduce = nullptr, lambda = nullptr;
    size_t nsweep = 0;
    e = add(reset_counter_kernel(), dim3(1), dim3(64), 0, a_reset, nullptr, 0, &reset);
    if (e == hipSuccess && n_lin > 0)
        e = add(sweep_batch_kernel(true), dim3(b->blocks_lin), dim3(256), b->lds_lin, a_lin, &reset, 1, &sweeps[nsweep++]);
    if (e == hipSuccess && n_quad > 0)
        e = add(sweep_batch_kernel(false), dim3(b->blocks), dim3(256), b->lds, a_quad, &reset, 1, &sweeps[nsweep++]);
    if (e == hipSuccess)
        e = add(round_reduce_batch_kernel(), dim3(count), dim3(reduce_threads()), 0, a_reduce,
                nsweep ? sweeps : &reset, nsweep ? nsweep : 1, &reduce);
    if (e == hipSuccess)
        e = add(lambda_update_batch_kernel(), dim3(count), dim3(256), 0, a_lambda, &reduce, 1, &lambda);
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        hipGraphDestroy(g);
        b->exec = nullptr;
        return e;
    }
    b->graph = g;
    return hipSuccess;
}


// ---- lambda_0 set encoder: workspace layout and host features ----------------
struct NetWs {
    size_t H1, H2, Z, G1, dP, part, total;
    int groups;
};

NetWs net_ws(int sets, int rows)
{
    NetWs w{};
    size_t o = 0;
    auto put = [&o](size_t bytes) {
        const size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    w.groups = std::min(sets, 64);
    w.H1 = put((size_t)rows * kNetH * 2);
    w.H2 = put((size_t)rows * kNetH * 2);
    w.Z = put((size_t)sets * kNetZ * 2);
    w.G1 = put((size_t)sets * kNetH * 2);
    w.dP = put((size_t)sets * kNetH * 4);
    w.part = put((size_t)w.groups * kNetPhiParams * 4);
    w.total = o;
    return w;
}

bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

uint16_t to_bf16(double v)
{
    const float f = (float)v;
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

pbit_status check_net_shape(int sets, int rows)
{
    if (sets < 1 || rows < 32 || rows % 32 != 0) return fail(PBIT_EINVAL, "sets >= 1 and rows a positive multiple of 32");
    return PBIT_OK;
}

// Workspace of allocation-free instances (pbit_create_instance_static): one
// array per device, resident until the process ends.  Host code never passes
// the symbol itself to a kernel or copy: it takes the device address of each
// device's copy with hipGetSymbolAddress once, with that device current.
constexpr size_t kStaticWsBytes = (size_t)16 << 20;
constexpr int kStaticMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kStaticWsBytes];

struct StaticSlot {
    void *ptr = nullptr;  // device address of this device's scratch array
    bool held = false;    // a live instance uses it
};
std::mutex g_static_mu;
StaticSlot g_static[kStaticMaxDevices];

}  // namespace

extern "C" {

const char *pbit_last_error(void) { return g_error.c_str(); }

pbit_status pbit_theta_table(int32_t *theta)
{
    if (!theta) return fail(PBIT_EINVAL, "null output");
    std::vector<int32_t> t;
    if (!make_theta(t)) return fail(PBIT_ERANGE, "threshold table rounding undecidable");
    std::memcpy(theta, t.data(), t.size() * 4);
    return PBIT_OK;
}

pbit_status pbit_exchange_table(int32_t *x)
{
    if (!x) return fail(PBIT_EINVAL, "null output");
    std::vector<int32_t> t;
    if (!make_exchange_table(t)) return fail(PBIT_ERANGE, "exchange table rounding undecidable");
    std::memcpy(x, t.data(), t.size() * 4);
    return PBIT_OK;
}

pbit_status pbit_plan(const pbit_problem *prob, const pbit_params *par, pbit_plan_info *out)
{
    if (!out) return fail(PBIT_EINVAL, "null output");
    Plan P;
    const pbit_status st = make_plan(prob, par, P);
    if (st != PBIT_OK) return st;
    fill_plan_info(P, out);
    return PBIT_OK;
}

size_t pbit_workspace_bytes(const pbit_problem *prob, const pbit_params *par)
{
    Plan P;
    if (make_plan(prob, par, P) != PBIT_OK) return 0;
    return P.L.total;
}

pbit_status pbit_create_instance(const pbit_problem *prob, const pbit_params *par, void *dev_ws,
                                 size_t ws_bytes, pbit_stream stream, pbit_instance **out)
{
    return create_impl(prob, par, dev_ws, ws_bytes, stream, out);
}

size_t pbit_static_workspace_bytes(void) { return kStaticWsBytes; }

pbit_status pbit_create_instance_static(const pbit_problem *prob, const pbit_params *par, pbit_stream stream,
                                        pbit_instance **out)
{
    if (!out) return fail(PBIT_EINVAL, "null output handle");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(PBIT_EDEVICE, std::string("device query failed: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kStaticMaxDevices) return fail(PBIT_EINVAL, "device index beyond the static workspace table");
    Plan P;
    pbit_status st = make_plan(prob, par, P);
    if (st != PBIT_OK) return st;
    if (P.L.total > kStaticWsBytes)
        return fail(PBIT_EWORKSPACE, "instance needs " + std::to_string(P.L.total) +
                                         " workspace bytes, more than the static workspace of " +
                                         std::to_string(kStaticWsBytes) + "; use pbit_create_instance");
    std::lock_guard<std::mutex> lock(g_static_mu);
    StaticSlot &slot = g_static[dev];
    if (slot.held) return fail(PBIT_ESTATE, "the static workspace of this device is held by a live instance");
    if (!slot.ptr) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(PBIT_EDEVICE, std::string("static workspace address lookup failed: ") + hipGetErrorString(e));
        slot.ptr = ptr;
    }
    st = create_impl(prob, par, slot.ptr, kStaticWsBytes, stream, out);
    if (st != PBIT_OK) return st;
    (*out)->static_dev = dev;
    slot.held = true;
    return PBIT_OK;
}

pbit_status pbit_sample_round(pbit_instance *inst, pbit_stream stream)
{
    pbit_status st = check_live(inst);
    if (st != PBIT_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const DevInstance &d = inst->dev;
    hipError_t e;
    switch (inst->plan.variant) {
        case kQuad: {
            const bool pc = inst->split >= 1 || (inst->split < 0 && (d.R + kWave - 1) / kWave <= inst->cus);
            // six producers (two waves per SIMD) by default: with the visiting
            // wave reading its operands ahead the producers bound the round
            // (measured: 10 blocks 114.8 -> 90.7 ms, 4 blocks 8.7 -> 6.5 ms);
            // parallel tempering is built with six only
            const int producers = inst->split == 1 && d.pt == 0 ? 3 : 6;
            e = pc ? launch_sweep_quad_pc(d, inst->plan.nb, producers, s)
                   : launch_sweep_quad(d, inst->plan.nb, inst->wpb, s);
            break;
        }
        default: {
            const bool wide = inst->plan.variant == kLinearWide;
            const bool split = inst->split == 1 ||
                               (inst->split < 0 && (d.R + kWave - 1) / kWave <= inst->cus &&
                                linear_split_bytes(inst->plan) <= kMaxLds);
            if (split) {
                if (d.m <= 6) e = launch_sweep_linear_pc_a(d, wide, s);
                else if (d.m <= 12) e = launch_sweep_linear_pc_b(d, wide, s);
                else if (d.m <= 20) e = launch_sweep_linear_pc_c(d, wide, s);
                else e = launch_sweep_linear_pc_d(d, wide, s);
                break;
            }
            const bool res = inst->resident == 1 ||
                             (inst->resident < 0 && resident_bytes(inst->plan, inst->wpb) <= kMaxLds);
            if (d.m <= 6) e = launch_sweep_linear_a(d, wide, inst->wpb, res, s);
            else if (d.m <= 12) e = launch_sweep_linear_b(d, wide, inst->wpb, res, s);
            else if (d.m <= 20) e = launch_sweep_linear_c(d, wide, inst->wpb, res, s);
            else e = launch_sweep_linear_d(d, wide, inst->wpb, res, s);
        }
    }
    if (e == hipSuccess) e = launch_round_reduce(d, s);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return device_error(inst, e, "sample_round launch failed");
    return PBIT_OK;
}

pbit_status pbit_update_lambda(pbit_instance *inst, pbit_stream stream)
{
    pbit_status st = check_live(inst);
    if (st != PBIT_OK) return st;
    hipError_t e = launch_lambda_update(inst->dev, 1, nullptr, reinterpret_cast<hipStream_t>(stream));
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return device_error(inst, e, "update_lambda launch failed");
    return PBIT_OK;
}

pbit_status pbit_set_lambda(pbit_instance *inst, const int32_t *lambda_q, pbit_stream stream)
{
    pbit_status st = check_live(inst);
    if (st != PBIT_OK) return st;
    if (!lambda_q) return fail(PBIT_EINVAL, "null lambda");
    int32_t v[kMaxM] = {0};
    const int64_t cap = inst->plan.lq_max;
    for (int k = 0; k < inst->plan.m; ++k) v[k] = (int32_t)std::max<int64_t>(-cap, std::min<int64_t>(cap, lambda_q[k]));
    hipError_t e = launch_lambda_update(inst->dev, 2, v, reinterpret_cast<hipStream_t>(stream));
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return device_error(inst, e, "set_lambda launch failed");
    return PBIT_OK;
}

pbit_status pbit_get_lambda(pbit_instance *inst, int32_t *lambda_q, pbit_stream stream)
{
    pbit_status st = check_live(inst);
    if (st != PBIT_OK) return st;
    if (!lambda_q) return fail(PBIT_EINVAL, "null output");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(lambda_q, inst->dev.lam_q, (size_t)inst->plan.m * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_error(inst, e, "get_lambda failed");
    return PBIT_OK;
}

pbit_status pbit_best_feasible(pbit_instance *inst, int64_t *profit, uint8_t *x, int32_t *round,
                               int32_t *replica, pbit_stream stream)
{
    pbit_status st = check_live(inst);
    if (st != PBIT_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int64_t best[4];
    std::vector<uint32_t> bits(inst->plan.words);
    hipError_t e = hipMemcpyAsync(best, inst->dev.best, sizeof(best), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(bits.data(), inst->dev.best_x, bits.size() * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_error(inst, e, "best_feasible failed");
    if (best[3] == 0) return PBIT_NOFEAS;
    if (profit) *profit = best[0];
    if (round) *round = (int32_t)best[1];
    if (replica) *replica = (int32_t)best[2];
    if (x)
        for (int i = 0; i < inst->plan.n; ++i) x[i] = (uint8_t)((bits[i >> 5] >> (i & 31)) & 1u);
    return PBIT_OK;
}

pbit_status pbit_round_outputs(pbit_instance *inst, void *dev_out, size_t bytes, pbit_stream stream)
{
    pbit_status st = check_live(inst);
    if (st != PBIT_OK) return st;
    pbit_plan_info info;
    fill_plan_info(inst->plan, &info);
    if (!dev_out || bytes < info.out_bytes) return fail(PBIT_EWORKSPACE, "output buffer too small");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    unsigned char *o = static_cast<unsigned char *>(dev_out);
    const DevInstance &d = inst->dev;
    const Plan &P = inst->plan;
    struct Piece {
        size_t off;
        const void *src;
        size_t bytes;
    } pieces[] = {
        {info.out_x, d.rx, (size_t)P.R * P.words * 4}, {info.out_g, d.rg, (size_t)P.R * P.m * 4},
        {info.out_profit, d.rprofit, (size_t)P.R * 8}, {info.out_feasible, d.rfeas, (size_t)P.R * 4},
        {info.out_G, d.G, (size_t)P.m * 8},            {info.out_lambda, d.lam_q, (size_t)P.m * 4},
        {info.out_round, d.round_k, 4},                {info.out_sat, d.lam_sat, 4},
        {info.out_slot, d.rslot, (size_t)P.R * 4},
    };
    for (const Piece &pc : pieces) {
        hipError_t e = hipMemcpyAsync(o + pc.off, pc.src, pc.bytes, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return device_error(inst, e, "round_outputs copy failed");
    }
    return PBIT_OK;
}

pbit_status pbit_destroy_instance(pbit_instance *inst)
{
    if (!inst) return fail(PBIT_EINVAL, "null instance");
    if (inst->member) return fail(PBIT_EINVAL, "instance is a batch member; destroy the batch");
    if (inst->static_dev >= 0) {
        std::lock_guard<std::mutex> lock(g_static_mu);
        g_static[inst->static_dev].held = false;
    }
    delete inst;
    return PBIT_OK;
}

pbit_status pbit_instance_info(const pbit_instance *inst, pbit_plan_info *out)
{
    if (!inst || !out) return fail(PBIT_EINVAL, "null instance or output");
    fill_plan_info(inst->plan, out);
    return PBIT_OK;
}

pbit_status pbit_set_tiling(pbit_instance *inst, int32_t waves_per_block, int32_t lds_resident, int32_t split)
{
    pbit_status st = check_live(inst);
    if (st != PBIT_OK) return st;
    const bool quad = inst->plan.variant == kQuad;
    const int wpb = waves_per_block == 0 ? waves_per_block_default(inst->plan) : waves_per_block;
    const bool ok = quad ? (wpb == 1 || wpb == 4) : (wpb >= 1 && wpb <= 4);
    if (!ok) return fail(PBIT_EINVAL, "waves per block must be 1 or 4 (quadratic) or 1..4 (linear)");
    if (lds_resident < -1 || lds_resident > 1) return fail(PBIT_EINVAL, "lds_resident must be -1, 0 or 1");
    if (split < -1 || split > (quad ? 2 : 1))
        return fail(PBIT_EINVAL, "split must be -1, 0 or 1 (and 2 for the quadratic kernel)");
    if (split == 1 && !quad && linear_split_bytes(inst->plan) > kMaxLds)
        return fail(PBIT_ERANGE, "site constants do not fit LDS for the split layout");
    if (!quad && lds_resident == 1 && resident_bytes(inst->plan, wpb) > kMaxLds)
        return fail(PBIT_ERANGE, "site constants do not fit LDS at this tiling");
    inst->wpb = wpb;
    inst->resident = quad ? -1 : lds_resident;
    inst->split = split;
    return PBIT_OK;
}

size_t pbit_batch_workspace_bytes(const pbit_problem *probs, const pbit_params *params, int32_t count)
{
    BatchSizes z;
    if (batch_sizes(probs, params, count, z) != PBIT_OK) return 0;
    return z.total;
}

pbit_status pbit_create_batch(const pbit_problem *probs, const pbit_params *params, int32_t count,
                              const int32_t *rounds, const pbit_batch_layout *layout, void *dev_ws,
                              size_t ws_bytes, pbit_stream stream, pbit_batch **out)
{
    if (!out) return fail(PBIT_EINVAL, "null output handle");
    pbit_batch_layout lay{0, 0, -1, 0};
    if (layout) lay = *layout;
    if (lay.blocks_quad < 0 || lay.blocks_linear < 0) return fail(PBIT_EINVAL, "grid sizes must be >= 0");
    if (lay.split_percent < -1) return fail(PBIT_EINVAL, "split_percent must be >= -1");
    if (lay.split_percent == -1) lay.split_percent = 200;
    BatchSizes z;
    pbit_status st = batch_sizes(probs, params, count, z);
    if (st != PBIT_OK) return st;
    if (!dev_ws || (reinterpret_cast<uintptr_t>(dev_ws) & 255) != 0 || ws_bytes < z.total)
        return fail(PBIT_EWORKSPACE, "workspace missing, misaligned or smaller than pbit_batch_workspace_bytes");
    if (rounds)
        for (int i = 0; i < count; ++i)
            if (rounds[i] < 0) return fail(PBIT_EINVAL, "round budgets must be >= 0");

    pbit_batch *b = new (std::nothrow) pbit_batch();
    if (!b) return fail(PBIT_EINVAL, "host allocation failed");
    unsigned char *base = static_cast<unsigned char *>(dev_ws);
    b->d_insts = reinterpret_cast<DevInstance *>(base + z.off_insts);
    b->d_items = reinterpret_cast<int4 *>(base + z.off_items);
    b->d_counter = reinterpret_cast<int *>(base + z.off_counter);
    b->d_rounds = reinterpret_cast<int32_t *>(base + z.off_rounds);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);

    struct Cost {
        int64_t cost;
        int4 item;
    };
    std::vector<Cost> q;
    std::vector<int64_t> lin_cost(count, -1);
    int64_t lin_total = 0;
    for (int i = 0; i < count; ++i) {
        pbit_instance *m = nullptr;
        st = create_impl(&z.padded[i].prob, &params[i], base + z.off_member[i], z.member_bytes[i], stream, &m);
        if (st != PBIT_OK) {
            g_error = "member " + std::to_string(i) + ": " + g_error;
            delete b;  // members created so far are released by the destructor
            return st;
        }
        m->member = true;
        m->dev.rounds_left = b->d_rounds + i;
        b->members.push_back(m);
        b->dev.push_back(m->dev);
        b->rounds.push_back(rounds ? rounds[i] : INT32_MAX);
        const Plan &P = m->plan;
        if (P.variant != kQuad) {
            // chain cost of a plain 256-replica tile, in visit-cycles (roughly)
            lin_cost[i] = (int64_t)P.T * P.n_ext * (64 + 6 * P.m);
            lin_total += lin_cost[i] * ((P.R + 255) / 256);
        }
    }
    int cus = 0, dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (cus < 1) cus = 1;
    // Which linear members run as split tiles: a split tile visits about twice
    // as fast but takes four waves per 64 replicas, i.e. twice the work per
    // replica.  Only members whose plain chain exceeds twice the average linear
    // load per CU would bound the round, so only they are split (a threshold
    // chosen by measurement on the mixed workload, where it splits the N=500
    // M=30 members: splitting also those at about 1.9 times the load, or none,
    // both lengthened its rounds).
    std::vector<char> split(count, 0);
    const int64_t load = lin_total / cus;
    int n_split = 0;
    for (int i = 0; i < count; ++i) {
        split[i] = lay.split_percent > 0 && lin_cost[i] >= 0 &&
                   (i128)lin_cost[i] * 100 > (i128)lay.split_percent * load &&
                   linear_split_bytes(b->members[i]->plan) <= kMaxLds;
        n_split += split[i];
    }
    for (int i = 0; i < count; ++i) {
        const Plan &P = b->members[i]->plan;
        const int code = batch_variant_code(P.variant, P.nb, P.m);
        if (P.variant == kQuad) {
            const int64_t cost = ((int64_t)1 << 60) + (int64_t)P.T * P.n_ext * (96 + 8 * P.nb);
            for (int r0 = 0; r0 < P.R; r0 += 256) q.push_back({cost, make_int4(i, r0, code, 0)});
            b->lds = std::max(b->lds, (size_t)kThetaBytes + (size_t)P.nb * 1024 + (size_t)2048 * (P.nb + 1));
            b->n_quad += (P.R + 255) / 256;
        } else if (split[i]) {
            const int64_t cost = lin_cost[i] / 2;
            for (int r0 = 0; r0 < P.R; r0 += 64) q.push_back({cost, make_int4(i, r0, code | kBatchSplit, 0)});
            b->lds_lin = std::max(b->lds_lin, linear_split_bytes(P));
        } else {
            for (int r0 = 0; r0 < P.R; r0 += 256) q.push_back({lin_cost[i], make_int4(i, r0, code, 0)});
            b->lds_lin = std::max(b->lds_lin, resident_bytes(P, 4));
        }
    }
    std::stable_sort(q.begin(), q.end(), [](const Cost &x, const Cost &y) { return x.cost > y.cost; });
    for (const Cost &c : q) b->items.push_back(c.item);

    int per_cu = 1, per_cu_lin = 1;
    const int n_quad = b->n_quad, n_lin = (int)b->items.size() - b->n_quad;
    if (e == hipSuccess && n_quad > 0) e = sweep_batch_prepare(false, b->lds, &per_cu);
    if (e == hipSuccess && n_lin > 0) e = sweep_batch_prepare(true, b->lds_lin, &per_cu_lin);
    if (e == hipSuccess && (per_cu < 1 || per_cu_lin < 1)) e = hipErrorInvalidConfiguration;
    const int bq = lay.blocks_quad, bl = lay.blocks_linear;
    b->blocks = n_quad == 0 ? 0 : (bq > 0 ? std::min(bq, n_quad) : std::min(n_quad, cus * per_cu));
    b->blocks_lin = n_lin == 0 ? 0 : (bl > 0 ? std::min(bl, n_lin) : std::min(n_lin, cus * per_cu_lin));
    b->split_percent = lay.split_percent;
    b->n_split = n_split;
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_insts, b->dev.data(), b->dev.size() * sizeof(DevInstance), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_items, b->items.data(), b->items.size() * sizeof(int4), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_rounds, b->rounds.data(), b->rounds.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_reset_counter(b->d_counter, s);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) {
        pbit_status r = device_error(nullptr, e, "batch upload failed");
        delete b;
        return r;
    }
    *out = b;
    return PBIT_OK;
}

pbit_status pbit_batch_sample_round(pbit_batch *b, pbit_stream stream)
{
    pbit_status st = check_batch(b);
    if (st != PBIT_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int count = (int)b->members.size();
    const int n_lin = (int)b->items.size() - b->n_quad;
    hipError_t e = launch_reset_counter(b->d_counter, s);
    if (e == hipSuccess && b->n_quad > 0)
        e = launch_sweep_batch(false, b->d_insts, b->d_items, b->n_quad, b->d_counter, b->blocks, b->lds, s);
    if (e == hipSuccess && n_lin > 0)
        e = launch_sweep_batch(true, b->d_insts, b->d_items + b->n_quad, n_lin, b->d_counter + 1, b->blocks_lin,
                               b->lds_lin, s);
    if (e == hipSuccess) e = launch_round_reduce_batch(b->d_insts, count, s);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return batch_error(b, e, "batch sample_round launch failed");
    return PBIT_OK;
}

pbit_status pbit_batch_update_lambda(pbit_batch *b, pbit_stream stream)
{
    pbit_status st = check_batch(b);
    if (st != PBIT_OK) return st;
    hipError_t e = launch_lambda_update_batch(b->d_insts, (int)b->members.size(), 1,
                                              reinterpret_cast<hipStream_t>(stream));
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return batch_error(b, e, "batch update_lambda launch failed");
    return PBIT_OK;
}

pbit_status pbit_batch_run(pbit_batch *b, int32_t rounds, int32_t use_graph, pbit_stream stream)
{
    pbit_status st = check_batch(b);
    if (st != PBIT_OK) return st;
    if (rounds < 0) return fail(PBIT_EINVAL, "rounds must be >= 0");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (!use_graph) {
        for (int k = 0; k < rounds; ++k) {
            st = pbit_batch_sample_round(b, stream);
            if (st == PBIT_OK) st = pbit_batch_update_lambda(b, stream);
            if (st != PBIT_OK) return st;
        }
        return PBIT_OK;
    }
    if (!b->exec) {
        hipError_t e = build_round_graph(b);
        if (e != hipSuccess) return batch_error(b, e, "building the round graph failed");
    }
    for (int k = 0; k < rounds; ++k) {
        hipError_t e = hipGraphLaunch(b->exec, s);
        if (e != hipSuccess) return batch_error(b, e, "graph launch failed");
    }
    return PBIT_OK;
}

pbit_status pbit_batch_member(pbit_batch *b, int32_t index, pbit_instance **member)
{
    if (!b || !member) return fail(PBIT_EINVAL, "null batch or output");
    if (index < 0 || index >= (int)b->members.size()) return fail(PBIT_EINVAL, "member index out of range");
    *member = b->members[index];
    return PBIT_OK;
}

pbit_status pbit_batch_rounds_left(pbit_batch *b, int32_t *rounds_left, pbit_stream stream)
{
    pbit_status st = check_batch(b);
    if (st != PBIT_OK) return st;
    if (!rounds_left) return fail(PBIT_EINVAL, "null output");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(rounds_left, b->d_rounds, b->members.size() * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return batch_error(b, e, "rounds_left failed");
    return PBIT_OK;
}

pbit_status pbit_batch_shape(const pbit_batch *b, int32_t *items, int32_t *blocks, size_t *lds_bytes)
{
    if (!b) return fail(PBIT_EINVAL, "null batch");
    if (items) *items = (int32_t)b->items.size();
    if (blocks) *blocks = b->blocks + b->blocks_lin;
    if (lds_bytes) *lds_bytes = std::max(b->lds, b->lds_lin);
    return PBIT_OK;
}

pbit_status pbit_batch_layout_used(const pbit_batch *b, pbit_batch_layout *out)
{
    if (!b || !out) return fail(PBIT_EINVAL, "null batch or output");
    out->blocks_quad = b->blocks;
    out->blocks_linear = b->blocks_lin;
    out->split_percent = b->split_percent;
    out->split_members = b->n_split;
    return PBIT_OK;
}

pbit_status pbit_destroy_batch(pbit_batch *b)
{
    if (!b) return fail(PBIT_EINVAL, "null batch");
    delete b;
    return PBIT_OK;
}

int32_t pbit_net_param_count(void) { return kNetParams; }

size_t pbit_net_workspace_bytes(int32_t sets, int32_t rows)
{
    if (check_net_shape(sets, rows) != PBIT_OK) return 0;
    return net_ws(sets, rows).total;
}

pbit_status pbit_net_pack(const pbit_problem *probs, const pbit_params *params, int32_t count, int32_t *sets_out,
                          int32_t *rows_out, uint16_t *x, uint16_t *ctx, int32_t *set_rows, int32_t *set_n,
                          double *scale, int32_t *dest)
{
    if (!probs || !params || count < 1 || !sets_out || !rows_out) return fail(PBIT_EINVAL, "null arguments");
    int sets = 0, rows = 0;
    std::vector<Plan> plans(count);
    for (int i = 0; i < count; ++i) {
        pbit_status st = make_plan(&probs[i], &params[i], plans[i]);
        if (st != PBIT_OK) {
            g_error = "member " + std::to_string(i) + ": " + g_error;
            return st;
        }
        sets += probs[i].m;
        rows += probs[i].m * ((probs[i].n + 31) / 32) * 32;
    }
    *sets_out = sets;
    *rows_out = rows;
    if (!x) return PBIT_OK;  // size query
    if (!ctx || !set_rows || !set_n || !scale || !dest) return fail(PBIT_EINVAL, "null output array");
    std::memset(x, 0, (size_t)rows * kNetF * 2);
    std::memset(ctx, 0, (size_t)sets * kNetCtx * 2);
    int s = 0, r = 0;
    for (int i = 0; i < count; ++i) {
        const pbit_problem &p = probs[i];
        const Plan &P = plans[i];
        const int n = p.n, m = p.m;
        std::vector<double> h(n), rho(n), wsum(n, 0.0);
        double s_f = 0.0;
        if (p.kind == PBIT_QKP) {
            for (int a = 0; a < n; ++a) {
                for (int b = 0; b < n; ++b) {
                    const double v = p.profit[(size_t)a * n + b];
                    s_f = std::max(s_f, std::fabs(v));
                    if (a != b) wsum[a] += v;
                }
                h[a] = p.profit[(size_t)a * n + a];
            }
        } else {
            for (int a = 0; a < n; ++a) {
                h[a] = p.profit[a];
                s_f = std::max(s_f, std::fabs(h[a]));
            }
        }
        s_f = std::max(s_f, 1.0);
        double s_g = 1.0;
        for (int k = 0; k < m; ++k) {
            s_g = std::max(s_g, (double)p.capacity[k]);
            for (int a = 0; a < n; ++a) s_g = std::max(s_g, (double)p.weight[(size_t)k * n + a]);
        }
        double half = 0.0;
        for (int a = 0; a < n; ++a) {
            rho[a] = h[a] + wsum[a];
            half += h[a] + 0.5 * wsum[a];
        }
        std::vector<double> mean_ratio(n, 0.0);
        for (int a = 0; a < n; ++a) {
            double acc = 0.0;
            for (int k = 0; k < m; ++k)
                acc += (double)p.weight[(size_t)k * n + a] / std::max((double)p.capacity[k], 1.0);
            mean_ratio[a] = acc / m;
        }
        const double d = p.kind == PBIT_QKP ? (double)p.density_num / (double)p.density_den
                                            : 2.0 / (P.n_ext + 1);
        const double c6[6] = {std::log((double)P.n_ext) / 8.0, d, ((double)P.pq / 256.0) / P.n_ext,
                              ((double)params[i].beta_num / params[i].beta_den) / 50.0, m / 32.0,
                              p.kind == PBIT_QKP ? 0.0 : 1.0};
        const int span = ((n + 31) / 32) * 32;
        std::vector<double> eff(n);
        std::vector<int> order(n);
        for (int k = 0; k < m; ++k, ++s) {
            set_rows[s] = r;
            set_n[s] = n;
            dest[s] = i * kMaxM + k;
            double asum = 0.0;
            const double bk = std::max((double)p.capacity[k], 1.0);
            for (int a = 0; a < n; ++a) {
                const double ak = p.weight[(size_t)k * n + a];
                asum += ak;
                uint16_t *row = x + (size_t)(r + a) * kNetF;
                row[0] = to_bf16(rho[a] / (s_f * n));
                row[1] = to_bf16(n * (ak / bk));
                row[2] = to_bf16(n * mean_ratio[a]);
                row[3] = to_bf16(h[a] / s_f);
            }
            const double rho_bar = half / (asum > 0 ? asum : 1.0);
            // profit per unit of weight k (half-marginal profit), relative to rho_bar
            for (int a = 0; a < n; ++a) {
                const double ak = p.weight[(size_t)k * n + a];
                eff[a] = ak == 0 ? HUGE_VAL : (h[a] + 0.5 * wsum[a]) / ak;
                double f4;
                if (eff[a] == HUGE_VAL) f4 = 8.0;
                else if (eff[a] <= 0.0 || rho_bar <= 0.0) f4 = -8.0;
                else f4 = std::min(8.0, std::max(-8.0, std::log(eff[a] / rho_bar)));
                x[(size_t)(r + a) * kNetF + 4] = to_bf16(f4);
            }
            // greedy fill of constraint k alone: decreasing efficiency, ties by index
            for (int a = 0; a < n; ++a) order[a] = a;
            std::sort(order.begin(), order.end(),
                      [&eff](int u, int v) { return eff[u] != eff[v] ? eff[u] > eff[v] : u < v; });
            double used = 0.0, e_break = 0.0;
            int taken = 0;
            for (int a : order) {
                const double ak = p.weight[(size_t)k * n + a];
                if (used + ak > (double)p.capacity[k]) {
                    e_break = eff[a];
                    break;
                }
                used += ak;
                ++taken;
            }
            const double c9[9] = {c6[0], c6[1], c6[2], c6[3], c6[4], c6[5],
                                  rho_bar > 0 ? e_break / rho_bar : 0.0,
                                  (double)p.capacity[k] / (asum > 0 ? asum : 1.0), (double)taken / n};
            for (int c = 0; c < 9; ++c) ctx[(size_t)s * kNetCtx + c] = to_bf16(c9[c]);
            scale[s] = 256.0 * rho_bar * s_g / s_f;
            r += span;
        }
    }
    set_rows[s] = r;
    return PBIT_OK;
}

pbit_status pbit_net_cast(const float *w, uint16_t *w_bf16, pbit_stream stream)
{
    if (!w || !w_bf16) return fail(PBIT_EINVAL, "null buffer");
    hipError_t e = net_launch_cast(w, w_bf16, reinterpret_cast<hipStream_t>(stream));
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return fail(PBIT_EDEVICE, std::string("net_cast: ") + hipGetErrorString(e));
    return PBIT_OK;
}

pbit_status pbit_net_forward(const uint16_t *w_bf16, const uint16_t *x, const uint16_t *ctx,
                             const int32_t *set_rows, const int32_t *set_n, int32_t sets, int32_t rows, void *ws,
                             size_t ws_bytes, float *t, pbit_stream stream)
{
    pbit_status st = check_net_shape(sets, rows);
    if (st != PBIT_OK) return st;
    if (!w_bf16 || !x || !ctx || !set_rows || !set_n || !t) return fail(PBIT_EINVAL, "null buffer");
    if (!aligned(w_bf16, 16) || !aligned(x, 16)) return fail(PBIT_EINVAL, "weights and inputs must be 16-byte aligned");
    const NetWs L = net_ws(sets, rows);
    if (!ws || !aligned(ws, 256) || ws_bytes < L.total) return fail(PBIT_EWORKSPACE, "net workspace too small");
    unsigned char *b = static_cast<unsigned char *>(ws);
    hipError_t e = net_launch_forward(w_bf16, x, ctx, set_rows, set_n, sets, rows,
                                      reinterpret_cast<uint16_t *>(b + L.H1), reinterpret_cast<uint16_t *>(b + L.H2),
                                      reinterpret_cast<uint16_t *>(b + L.Z), reinterpret_cast<uint16_t *>(b + L.G1),
                                      t, reinterpret_cast<hipStream_t>(stream));
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return fail(PBIT_EDEVICE, std::string("net_forward: ") + hipGetErrorString(e));
    return PBIT_OK;
}

pbit_status pbit_net_backward(const uint16_t *w_bf16, const uint16_t *x, const int32_t *set_rows,
                              const int32_t *set_n, int32_t sets, int32_t rows, const float *t, const float *y,
                              void *ws, size_t ws_bytes, float *grad, float *loss, pbit_stream stream)
{
    pbit_status st = check_net_shape(sets, rows);
    if (st != PBIT_OK) return st;
    if (!w_bf16 || !x || !set_rows || !set_n || !t || !y || !grad || !loss) return fail(PBIT_EINVAL, "null buffer");
    if (!aligned(w_bf16, 16) || !aligned(x, 16)) return fail(PBIT_EINVAL, "weights and inputs must be 16-byte aligned");
    const NetWs L = net_ws(sets, rows);
    if (!ws || !aligned(ws, 256) || ws_bytes < L.total) return fail(PBIT_EWORKSPACE, "net workspace too small");
    unsigned char *b = static_cast<unsigned char *>(ws);
    hipError_t e = net_launch_backward(
        w_bf16, x, set_rows, set_n, sets, rows, reinterpret_cast<const uint16_t *>(b + L.H1),
        reinterpret_cast<const uint16_t *>(b + L.H2), reinterpret_cast<const uint16_t *>(b + L.Z),
        reinterpret_cast<const uint16_t *>(b + L.G1), t, y, reinterpret_cast<float *>(b + L.dP),
        reinterpret_cast<float *>(b + L.part), L.groups, grad, loss, reinterpret_cast<hipStream_t>(stream));
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return fail(PBIT_EDEVICE, std::string("net_backward: ") + hipGetErrorString(e));
    return PBIT_OK;
}

pbit_status pbit_net_adam_step(float *w, float *m, float *v, const float *grad, uint16_t *w_bf16, int32_t step,
                               float lr, pbit_stream stream)
{
    if (!w || !m || !v || !grad || !w_bf16) return fail(PBIT_EINVAL, "null buffer");
    if (step < 1) return fail(PBIT_EINVAL, "step counts from 1");
    const double b1 = 0.9, b2 = 0.999;
    const float bc1 = (float)(1.0 - std::pow(b1, step)), bc2 = (float)(1.0 - std::pow(b2, step));
    hipError_t e = net_launch_adam(w, m, v, grad, w_bf16, lr, (float)b1, (float)b2, 1e-8f, bc1, bc2,
                                   reinterpret_cast<hipStream_t>(stream));
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return fail(PBIT_EDEVICE, std::string("net_adam_step: ") + hipGetErrorString(e));
    return PBIT_OK;
}

pbit_status pbit_net_to_lambda(const float *t, const double *scale, const int32_t *dest, int32_t sets,
                               int32_t *lambda_q, pbit_stream stream)
{
    if (!t || !scale || !dest || !lambda_q || sets < 1) return fail(PBIT_EINVAL, "null buffer or sets < 1");
    hipError_t e = net_launch_to_lambda(t, scale, dest, sets, lambda_q, reinterpret_cast<hipStream_t>(stream));
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return fail(PBIT_EDEVICE, std::string("net_to_lambda: ") + hipGetErrorString(e));
    return PBIT_OK;
}

pbit_status pbit_batch_set_lambdas(pbit_batch *b, const int32_t *lambda_q, pbit_stream stream)
{
    pbit_status st = check_batch(b);
    if (st != PBIT_OK) return st;
    if (!lambda_q) return fail(PBIT_EINVAL, "null lambda array");
    hipError_t e = launch_lambda_set_batch(b->d_insts, (int)b->members.size(), lambda_q,
                                           reinterpret_cast<hipStream_t>(stream));
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return batch_error(b, e, "batch set_lambdas launch failed");
    return PBIT_OK;
}

pbit_status pbit_batch_snapshot(pbit_batch *b, void *dev_out, pbit_stream stream)
{
    pbit_status st = check_batch(b);
    if (st != PBIT_OK) return st;
    if (!dev_out) return fail(PBIT_EINVAL, "null output");
    hipError_t e = launch_batch_snapshot(b->d_insts, (int)b->members.size(), static_cast<unsigned char *>(dev_out),
                                         reinterpret_cast<hipStream_t>(stream));
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return batch_error(b, e, "batch snapshot launch failed");
    return PBIT_OK;
}

}  // extern "C"
