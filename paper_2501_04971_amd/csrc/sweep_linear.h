// Annealing run for linear-profit instances with M constraints (the
// multidimensional knapsack of Sec. IV-B): the p-bit machine of Sec. III-B, one
// replica per lane.
//
// With no pair profits the field of site i for replica r reduces to
//   Z_i = K_{x_i,i} - 2 s_f Pq (a_i . g)
// where g = A_ext x - b is the replica's residual vector (M int32 values in
// VGPRs) and K_{0,i}, K_{1,i} fold in h_i, the penalty's self term and the
// Lagrange term of the current lambda.  A flip of site i moves g by +-a_i,
// O(M) work; the penalty is never expanded into couplings.
//
// Original sites are visited 32 at a time with the replica's bits for the
// block in one VGPR (the full bit vector lives in LDS, one word per lane per
// block).  Slack sites of constraint k only touch g_k (a = 2^q e_k), so they are
// visited in a loop over k unrolled at compile time with their bits kept in one
// VGPR per constraint.
#pragma once
#include "device_common.h"

namespace pbit {

template <int M, bool WIDE>
__device__ __forceinline__ int64_t constraint_field(const int32_t *ac, const int32_t (&g)[M], int64_t k2)
{
    // 2 s_f Pq a_i.g (scaled), the only replica-dependent part of an item's field
    if (WIDE) {
        int64_t dd = 0;
#pragma unroll
        for (int k = 0; k < M; ++k) dd += (int64_t)ac[k] * (int64_t)g[k];
        return dd * k2;
    }
    int32_t dd = 0;
#pragma unroll
    for (int k = 0; k < M; ++k) dd += __mul24(ac[k], g[k]);
    return (int64_t)dd * k2;
}

// Round epilogue of one replica: profit of the original bits, feasible iff
// g_k <= slack_k for every k (i.e. the original inequality holds), final state
// words (slack bits merged in) and residuals.
template <int M>
__device__ __forceinline__ void linear_score(const DevInstance &d, int r, uint32_t *xl, int lane,
                                             const int32_t (&g)[M], const uint32_t (&sk)[M])
{
    const bool live = r < d.R;
    const int n = d.n;
    int64_t profit = 0;
    for (int blk = 0; blk < d.owords; ++blk) {
        const uint32_t xw = xl[blk * kWave + lane];
#pragma unroll
        for (int s = 0; s < 32; ++s) {
            const int i = blk * 32 + s;
            if (i < n && ((xw >> s) & 1u)) profit += d.hprof[i];
        }
    }
    bool feasible = true;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        feasible = feasible && (g[k] <= (int32_t)sk[k]);
        const int off = d.slack_off[k];
        const int Qk = d.slack_q[k];
        if (Qk > 0) {
            const int w0 = off >> 5, b0 = off & 31;
            xl[w0 * kWave + lane] |= sk[k] << b0;
            if (b0 + Qk > 32) xl[(w0 + 1) * kWave + lane] |= sk[k] >> (32 - b0);
        }
    }
    if (live) {
        for (int w = 0; w < d.words; ++w) d.rx[(int64_t)r * d.words + w] = xl[w * kWave + lane];
#pragma unroll
        for (int k = 0; k < M; ++k) d.rg[(int64_t)r * d.m + k] = g[k];
        d.rprofit[r] = profit;
        d.rfeas[r] = feasible ? 1 : 0;
    }
}

// LDS bytes of linear_run for a workgroup of wpb waves and `words` state words.
inline size_t linear_lds_bytes(int wpb, int words)
{
    return (size_t)kThetaBytes + (size_t)wpb * words * kWave * 4;
}

// One annealing run (T sweeps) of the replicas rbase + [0, blockDim.x) of
// instance d, then the scoring of the final states.  smem must hold
// linear_lds_bytes(blockDim.x / 64, d.words) bytes.
template <int M, bool WIDE>
__device__ __forceinline__ void linear_run(const DevInstance &d, int rbase, unsigned char *smem)
{
    int32_t *th = reinterpret_cast<int32_t *>(smem);
    const int lane = threadIdx.x & 63;
    const int wave_in_block = threadIdx.x >> 6;
    uint32_t *xl = reinterpret_cast<uint32_t *>(smem + kThetaBytes) + wave_in_block * d.words * kWave;

    for (int e = threadIdx.x; e < kThetaLen; e += blockDim.x) th[e] = d.theta[e];
    for (int w = 0; w < d.words; ++w) xl[w * kWave + lane] = 0u;
    __syncthreads();

    const int r = rbase + threadIdx.x;
    const uint32_t kround = (uint32_t)d.round_k[0];
    const uint64_t m2 = (uint64_t)0xCD9E8D57u * (uint32_t)r;
    const int n = d.n;
    const int64_t *__restrict__ site = d.site;
    const int32_t *__restrict__ acol = d.acol;
    const int32_t *__restrict__ Btab = d.Btab;
    const int64_t k2 = d.k2;
    const int32_t ish = d.ish, hclo = d.hclo, hchi = d.hchi;
    const int64_t irnd = d.irnd;

    int32_t g[M];
    uint32_t sk[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        g[k] = -(int32_t)d.b[k];
        sk[k] = 0u;
    }

    for (int t = 0; t < d.T; ++t) {
        const int32_t Bt = Btab[t];
        const uint32_t cbase = (uint32_t)t * (uint32_t)d.nq;
        // original items, 32 per word of state
        for (int blk = 0; blk < d.owords; ++blk) {
            // a site changes only at its own visit: old states are read from this
            // copy, which keeps each record load off the chain of decisions
            const uint32_t xw0 = xl[blk * kWave + lane];
            uint32_t xw = xw0;
            const int64_t *rec = site + 4 * (blk * 32);
            const int32_t *ac0 = acol + (int64_t)(blk * 32) * M;
            uint32_t rnd[4] = {0u, 0u, 0u, 0u};
            uint32_t thA, thB, pend = 0u;
            {
                const int64_t Z = rec[xw & 1u] - constraint_field<M, WIDE>(ac0, g, k2);
                thA = (uint32_t)th[theta_index(Z, Bt, ish, irnd, hclo, hchi) + kThetaHalf];
                thB = thA;
            }
#pragma unroll
            for (int s = 0; s < 32; ++s) {
                const uint32_t xo = (xw0 >> s) & 1u;
                uint32_t nA = 0u, nB = 0u;
                if (s < 31) {
                    const int64_t *nx = rec + 4 * (s + 1);
                    const uint32_t xo1 = (xw0 >> (s + 1)) & 1u;
                    const int64_t Z0 = nx[xo1] -
                                       constraint_field<M, WIDE>(ac0 + (s + 1) * M, g, k2);
                    const int64_t Z1 = Z0 + (xo ? -nx[2] : nx[2]);
                    nA = (uint32_t)th[theta_index(Z0, Bt, ish, irnd, hclo, hchi) + kThetaHalf];
                    nB = (uint32_t)th[theta_index(Z1, Bt, ish, irnd, hclo, hchi) + kThetaHalf];
                }
                if ((s & 3) == 0)
                    philox_block(cbase + (uint32_t)((blk * 32 + s) >> 2), kround, m2, d.inst_id,
                                 d.seed_lo, d.seed_hi, rnd);
                const uint32_t u24 = rnd[s & 3] >> 8;
                const uint32_t thr = (pend ? thB : thA) & (uint32_t)(rec[4 * s + 3] >> 32);
                const uint32_t xn = u24 < thr ? 1u : 0u;
                const int32_t delta = (int32_t)xn - (int32_t)xo;
                pend = xn ^ xo;
                const int32_t *ac = ac0 + s * M;
#pragma unroll
                for (int k = 0; k < M; ++k) g[k] += delta * ac[k];
                xw = (xw & ~(1u << s)) | (xn << s);
                thA = nA;
                thB = nB;
            }
            xl[blk * kWave + lane] = xw;
        }
        // slack bits, constraint by constraint: a slack bit q of constraint k
        // has a = 2^q e_k, so its field only needs g_k
        uint32_t rnd[4] = {0u, 0u, 0u, 0u};
        int grp = -1;
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int off = d.slack_off[k];
            const int Qk = d.slack_q[k];
            if (Qk > 0) {
                uint32_t thA, thB, pend = 0u;
                {
                    const int64_t *rec = site + 4 * off;
                    const int64_t Z = rec[sk[k] & 1u] - (int64_t)g[k] * k2;
                    thA = (uint32_t)th[theta_index(Z, Bt, ish, irnd, hclo, hchi) + kThetaHalf];
                    thB = thA;
                }
                const uint32_t sk0 = sk[k];
                for (int q = 0; q < Qk; ++q) {
                    const int i = off + q;
                    const uint32_t xo = (sk0 >> q) & 1u;
                    // both thresholds of bit q+1 (the record past the last bit is padding)
                    const int64_t *nx = site + 4 * (i + 1);
                    const uint32_t xo1 = (sk0 >> (q + 1)) & 1u;
                    const int64_t Z0 = nx[xo1] - ((int64_t)g[k] * k2) * ((int64_t)2 << q);
                    const int64_t Z1 = Z0 + (xo ? -nx[2] : nx[2]);
                    const uint32_t nA = (uint32_t)th[theta_index(Z0, Bt, ish, irnd, hclo, hchi) + kThetaHalf];
                    const uint32_t nB = (uint32_t)th[theta_index(Z1, Bt, ish, irnd, hclo, hchi) + kThetaHalf];
                    if ((i >> 2) != grp) {
                        grp = i >> 2;
                        philox_block(cbase + (uint32_t)grp, kround, m2, d.inst_id, d.seed_lo,
                                     d.seed_hi, rnd);
                    }
                    const int sel = i & 3;
                    const uint32_t word = sel == 0 ? rnd[0] : sel == 1 ? rnd[1] : sel == 2 ? rnd[2] : rnd[3];
                    const uint32_t u24 = word >> 8;
                    const uint32_t thr = pend ? thB : thA;
                    const uint32_t xn = u24 < thr ? 1u : 0u;
                    const int32_t delta = (int32_t)xn - (int32_t)xo;
                    pend = xn ^ xo;
                    g[k] += delta * (1 << q);
                    sk[k] = (sk[k] & ~(1u << q)) | (xn << q);
                    thA = nA;
                    thB = nB;
                }
            }
        }
    }

    linear_score<M>(d, r, xl, lane, g, sk);
}

// LDS bytes of linear_run_lds: the threshold table, the field constants
// (K0, K1) of every site record, the coefficient rows of the original items
// and the state words of each wave.
inline size_t linear_lds_resident_bytes(int wpb, int words, int owords, int m)
{
    return (size_t)kThetaBytes + (size_t)(32 * words + 32) * 16 + (size_t)owords * 32 * m * 4 +
           (size_t)wpb * words * kWave * 4;
}

// Residual dot a_i.g from LDS coefficients (same value in every lane), summed in
// up to four independent partial sums so that the chain that waits on the last
// flip stays short.
template <int M, bool WIDE>
__device__ __forceinline__ int64_t residual_dot(const int32_t *a, const int32_t (&g)[M])
{
    constexpr int P = M < 4 ? M : 4;
    if (WIDE) {
        int64_t part[P];
#pragma unroll
        for (int p = 0; p < P; ++p) part[p] = (int64_t)a[p] * (int64_t)g[p];
#pragma unroll
        for (int k = P; k < M; ++k) part[k % P] += (int64_t)a[k] * (int64_t)g[k];
        int64_t t = 0;
#pragma unroll
        for (int p = 0; p < P; ++p) t += part[p];
        return t;
    }
    int32_t part[P];
#pragma unroll
    for (int p = 0; p < P; ++p) part[p] = mul_i24(a[p], g[p]);
#pragma unroll
    for (int k = P; k < M; ++k) part[k % P] = mad_i24(a[k], g[k], part[k % P]);
    int32_t t = 0;
#pragma unroll
    for (int p = 0; p < P; ++p) t += part[p];
    return t;
}

// Operands of one original-item visit (the item's weights and the record
// constant for its old state), read from LDS one visit ahead so that the read
// latency stays off the chain of decisions.  This pays where one wave per
// SIMD visits (the split form); two sets cost 2 (M + 2) registers, which the
// bodies with more than 16 constraints cannot spare: those read at the visit,
// and so do the bodies inside the batch kernel (whose registers are already
// full with the widest body) and the plain body, whose four waves per
// workgroup hide the latency for one another.
template <int M>
constexpr bool lin_read_ahead()
{
    return M <= 16;
}

template <int M>
struct LinOps {
    int32_t a[M];
    int64_t K;
};

template <int M>
__device__ __forceinline__ void load_lin_ops(LinOps<M> &o, const int32_t *ac, const int64_t *kr, int i,
                                             uint32_t xo)
{
    const int32_t *a = ac + i * M;
#pragma unroll
    for (int k = 0; k < M; ++k) o.a[k] = a[k];
    o.K = kr[2 * i + xo];
}

// The same annealing run with every per-site constant resident in LDS and each
// visit computed directly from the current residuals: field, threshold index,
// table lookup, decision, O(M) residual update.  No scalar-memory loads in the
// sweep, so waits on LDS never wait on scalar loads.  The host uses it whenever
// linear_lds_resident_bytes fits a workgroup.
template <int M, bool WIDE, bool AHEAD = false>
__device__ __forceinline__ void linear_run_lds(const DevInstance &d, int rbase, unsigned char *smem)
{
    const int words = d.words, owords = d.owords;
    const int n_rec = 32 * words + 32;
    int32_t *th = reinterpret_cast<int32_t *>(smem);
    int64_t *kr = reinterpret_cast<int64_t *>(smem + kThetaBytes);
    int32_t *ac = reinterpret_cast<int32_t *>(smem + kThetaBytes + (size_t)n_rec * 16);
    const int lane = threadIdx.x & 63;
    const int wave_in_block = threadIdx.x >> 6;
    uint32_t *xl = reinterpret_cast<uint32_t *>(smem + kThetaBytes + (size_t)n_rec * 16 +
                                                (size_t)owords * 32 * M * 4) +
                   wave_in_block * words * kWave;

    for (int e = threadIdx.x; e < kThetaLen; e += blockDim.x) th[e] = d.theta[e];
    for (int e = threadIdx.x; e < n_rec; e += blockDim.x) {
        kr[2 * e] = d.site[4 * e];
        kr[2 * e + 1] = d.site[4 * e + 1];
    }
    for (int e = threadIdx.x; e < owords * 32 * M; e += blockDim.x) ac[e] = d.acol[e];
    for (int w = 0; w < words; ++w) xl[w * kWave + lane] = 0u;
    __syncthreads();

    const int r = rbase + threadIdx.x;
    const uint32_t kround = (uint32_t)d.round_k[0];
    const uint64_t m2 = (uint64_t)0xCD9E8D57u * (uint32_t)r;
    const int n = d.n;
    const int32_t negk2 = -d.k2;
    const int32_t ish = d.ish, hclo = d.hclo, hchi = d.hchi;
    const int64_t irnd = d.irnd;

    int32_t g[M];
    uint32_t sk[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        g[k] = -(int32_t)d.b[k];
        sk[k] = 0u;
    }

    for (int t = 0; t < d.T; ++t) {
        const int32_t Bt = d.Btab[t];
        const uint32_t cbase = (uint32_t)t * (uint32_t)d.nq;
        for (int blk = 0; blk < owords; ++blk) {
            // a site changes only at its own visit: old states are read from this
            // copy, which keeps each record load off the chain of decisions
            const uint32_t xw0 = xl[blk * kWave + lane];
            uint32_t xw = xw0;
            const int rem = n - blk * 32;  // original items in this word (the rest are not visited here)
            uint32_t rnd[4];
            LinOps<AHEAD ? M : 1> op[2];
            if constexpr (AHEAD) load_lin_ops<M>(op[0], ac, kr, blk * 32, xw0 & 1u);
#pragma unroll
            for (int s = 0; s < 32; ++s) {
                const int i = blk * 32 + s;
                if constexpr (AHEAD) {
                    // the next visit's operands first (site blk*32 + 31 < owords*32: in bounds)
                    if (s + 1 < 32) load_lin_ops<M>(op[(s + 1) & 1], ac, kr, i + 1, (xw0 >> (s + 1)) & 1u);
                    __builtin_amdgcn_sched_barrier(0);
                }
                if ((s & 3) == 0)
                    philox_block(cbase + (uint32_t)(i >> 2), kround, m2, d.inst_id, d.seed_lo, d.seed_hi, rnd);
                const uint32_t xo = (xw0 >> s) & 1u;
                const int32_t *a = AHEAD ? op[s & 1].a : ac + i * M;
                const int64_t K = AHEAD ? op[s & 1].K : kr[2 * i + xo];
                const int64_t dd = residual_dot<M, WIDE>(a, g);
                const int64_t Z = WIDE ? K + dd * (int64_t)negk2 : K + (int64_t)(int32_t)dd * negk2;
                const uint32_t thr = (uint32_t)th[theta_index(Z, Bt, ish, irnd, hclo, hchi) + kThetaHalf] &
                                     (s < rem ? 0xFFFFFFFFu : 0u);
                const uint32_t xn = (rnd[s & 3] >> 8) < thr ? 1u : 0u;
                const int32_t delta = (int32_t)xn - (int32_t)xo;
#pragma unroll
                for (int k = 0; k < M; ++k) g[k] = WIDE ? g[k] + delta * a[k] : mad_i24(delta, a[k], g[k]);
                xw = (xw & ~(1u << s)) | (xn << s);
            }
            xl[blk * kWave + lane] = xw;
        }
        // slack bits, constraint by constraint (a = 2^q e_k: the field needs g_k only)
        uint32_t rnd[4] = {0u, 0u, 0u, 0u};
        int grp = -1;
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int off = d.slack_off[k];
            const int Qk = d.slack_q[k];
            const uint32_t sk0 = sk[k];
            for (int q = 0; q < Qk; ++q) {
                const int i = off + q;
                if ((i >> 2) != grp) {
                    grp = i >> 2;
                    philox_block(cbase + (uint32_t)grp, kround, m2, d.inst_id, d.seed_lo, d.seed_hi, rnd);
                }
                const uint32_t xo = (sk0 >> q) & 1u;
                const int64_t K = kr[2 * i + xo];
                const int64_t Z = K + (((int64_t)g[k] * negk2) << q);
                const uint32_t thr = (uint32_t)th[theta_index(Z, Bt, ish, irnd, hclo, hchi) + kThetaHalf];
                const int sel = i & 3;
                const uint32_t word = sel == 0 ? rnd[0] : sel == 1 ? rnd[1] : sel == 2 ? rnd[2] : rnd[3];
                const uint32_t xn = (word >> 8) < thr ? 1u : 0u;
                g[k] += ((int32_t)xn - (int32_t)xo) << q;
                sk[k] = (sk[k] & ~(1u << q)) | (xn << q);
            }
        }
    }
    linear_score<M>(d, r, xl, lane, g, sk);
}

template <int M, bool WIDE, bool RES>
__global__ __launch_bounds__(256) void sweep_linear(const DevInstance d)
{
    extern __shared__ __align__(16) unsigned char smem[];
    if (RES) linear_run_lds<M, WIDE>(d, blockIdx.x * blockDim.x, smem);
    else linear_run<M, WIDE>(d, blockIdx.x * blockDim.x, smem);
}

inline hipError_t launch_linear_kernel(const void *kern, const DevInstance &d, int waves_per_block,
                                       bool resident, hipStream_t stream)
{
    const int wpb = waves_per_block < 1 ? 1 : waves_per_block;
    const size_t lds = resident ? linear_lds_resident_bytes(wpb, d.words, d.owords, d.m)
                                : linear_lds_bytes(wpb, d.words);
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const int waves = (d.R + kWave - 1) / kWave;
    const int blocks = (waves + wpb - 1) / wpb;
    void *args[] = {const_cast<DevInstance *>(&d)};
    return hipLaunchKernel(kern, dim3(blocks), dim3(wpb * kWave), args, lds, stream);
}

}  // namespace pbit

#define PBIT_LINEAR_CASE(mm)                                                                \
    case mm:                                                                                \
        kern = resident ? (wide ? reinterpret_cast<const void *>(&sweep_linear<mm, true, true>) \
                                : reinterpret_cast<const void *>(&sweep_linear<mm, false, true>)) \
                        : (wide ? reinterpret_cast<const void *>(&sweep_linear<mm, true, false>) \
                                : reinterpret_cast<const void *>(&sweep_linear<mm, false, false>)); \
        break;
