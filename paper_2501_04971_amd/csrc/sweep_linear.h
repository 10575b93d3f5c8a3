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
__global__ __launch_bounds__(256) void sweep_linear(const DevInstance d)
{
    extern __shared__ __align__(16) unsigned char smem[];
    int32_t *th = reinterpret_cast<int32_t *>(smem);
    const int lane = threadIdx.x & 63;
    const int wave_in_block = threadIdx.x >> 6;
    uint32_t *xl = reinterpret_cast<uint32_t *>(smem + kThetaBytes) + wave_in_block * d.words * kWave;

    for (int e = threadIdx.x; e < kThetaLen; e += blockDim.x) th[e] = d.theta[e];
    for (int w = 0; w < d.words; ++w) xl[w * kWave + lane] = 0u;
    __syncthreads();

    const int r = (blockIdx.x * (blockDim.x >> 6) + wave_in_block) * kWave + lane;
    const uint32_t kround = (uint32_t)d.round_k[0];
    const uint64_t m2 = (uint64_t)0xCD9E8D57u * (uint32_t)r;
    const int n = d.n;
    const int64_t *__restrict__ kconst = d.kconst;
    const int32_t *__restrict__ acol = d.acol;
    const int32_t *__restrict__ Btab = d.Btab;
    const int64_t k2 = d.k2;

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
        // original items
        for (int blk = 0; blk < d.owords; ++blk) {
            uint32_t xw = xl[blk * kWave + lane];
            uint32_t rnd[4] = {0u, 0u, 0u, 0u};
#pragma unroll
            for (int s = 0; s < 32; ++s) {
                const int i = blk * 32 + s;
                if (i < n) {
                    if ((s & 3) == 0)
                        philox_block(cbase + (uint32_t)(i >> 2), kround, m2, d.inst_id, d.seed_lo,
                                     d.seed_hi, rnd);
                    const uint32_t u24 = rnd[s & 3] >> 8;
                    const uint32_t xo = (xw >> s) & 1u;
                    const int64_t K0 = kconst[2 * i];
                    const int64_t K1 = kconst[2 * i + 1];
                    const int32_t *ac = acol + (int64_t)i * M;
                    int64_t Z;
                    if (WIDE) {
                        int64_t dd = 0;
#pragma unroll
                        for (int k = 0; k < M; ++k) dd += (int64_t)ac[k] * (int64_t)g[k];
                        Z = (xo ? K1 : K0) - dd * k2;
                    } else {
                        int32_t dd = 0;
#pragma unroll
                        for (int k = 0; k < M; ++k) dd += __mul24(ac[k], g[k]);
                        Z = (xo ? K1 : K0) - (int64_t)dd * k2;
                    }
                    const int32_t idx = theta_index(Z, Bt, d.S);
                    const uint32_t xn = u24 < (uint32_t)th[idx + kThetaHalf] ? 1u : 0u;
                    const int32_t delta = (int32_t)xn - (int32_t)xo;
#pragma unroll
                    for (int k = 0; k < M; ++k) g[k] += delta * ac[k];
                    xw = (xw & ~(1u << s)) | (xn << s);
                }
            }
            xl[blk * kWave + lane] = xw;
        }
        // slack bits, constraint by constraint
        uint32_t rnd[4] = {0u, 0u, 0u, 0u};
        int grp = -1;
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int off = d.slack_off[k];
            const int Qk = d.slack_q[k];
            for (int q = 0; q < Qk; ++q) {
                const int i = off + q;
                if ((i >> 2) != grp) {
                    grp = i >> 2;
                    philox_block(cbase + (uint32_t)grp, kround, m2, d.inst_id, d.seed_lo, d.seed_hi,
                                 rnd);
                }
                const int sel = i & 3;
                const uint32_t word = sel == 0 ? rnd[0] : sel == 1 ? rnd[1] : sel == 2 ? rnd[2] : rnd[3];
                const uint32_t u24 = word >> 8;
                const uint32_t xo = (sk[k] >> q) & 1u;
                const int64_t K0 = kconst[2 * i];
                const int64_t K1 = kconst[2 * i + 1];
                const int64_t Z = (xo ? K1 : K0) - ((int64_t)g[k] * k2) * ((int64_t)1 << q);
                const int32_t idx = theta_index(Z, Bt, d.S);
                const uint32_t xn = u24 < (uint32_t)th[idx + kThetaHalf] ? 1u : 0u;
                const int32_t delta = (int32_t)xn - (int32_t)xo;
                g[k] += delta * (1 << q);
                sk[k] = (sk[k] & ~(1u << q)) | (xn << q);
            }
        }
    }

    // score: profit of the original bits, feasible iff g_k <= slack_k for all k
    const bool live = r < d.R;
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

}  // namespace pbit

namespace pbit {

inline hipError_t launch_linear_kernel(const void *kern, const DevInstance &d, int waves_per_block,
                                       hipStream_t stream)
{
    const int wpb = waves_per_block < 1 ? 1 : waves_per_block;
    const size_t lds = (size_t)kThetaBytes + (size_t)wpb * d.words * kWave * 4;
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
        kern = wide ? reinterpret_cast<const void *>(&sweep_linear<mm, true>)              \
                    : reinterpret_cast<const void *>(&sweep_linear<mm, false>);            \
        break;
