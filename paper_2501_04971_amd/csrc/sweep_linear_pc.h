// Producer/consumer form of the linear-profit annealing run (multidimensional
// knapsack), for launches that leave CUs idle: one visiting wave of 64
// replicas plus three producer waves that precompute, one block of 32 sites
// ahead, each visit's Philox draw and the equivalent threshold on the field
// product (see sweep_quad_pc.h).  Sites are visited in natural order (original
// items, then slack bits by constraint), so block c of the ring holds sites
// 32 c .. 32 c + 31 whichever loop visits them; the visiting wave meets the
// producers at a workgroup barrier whenever it crosses a multiple of 32.
// Per-site constants are LDS-resident as in linear_run_lds.  Results are
// bit-identical to linear_run.
#pragma once
#include "sweep_linear.h"
#include "sweep_quad_pc.h"

namespace pbit {

// (the host mirrors this in api.cpp, linear_split_bytes)
inline size_t linear_pc_lds_bytes(int words, int owords, int m)
{
    return (size_t)kThetaBytes + kRingBytes + (size_t)(32 * words + 32) * 16 +
           (size_t)owords * 32 * m * 4 + (size_t)words * kWave * 4;
}

template <int M, bool WIDE, bool AHEAD = lin_read_ahead<M>()>
__device__ __forceinline__ void linear_run_pc(const DevInstance &d, int rbase, unsigned char *smem)
{
    const int words = d.words, owords = d.owords;
    const int n_rec = 32 * words + 32;
    int32_t *th = reinterpret_cast<int32_t *>(smem);
    int64_t *ring = reinterpret_cast<int64_t *>(smem + kThetaBytes);
    int64_t *kr = reinterpret_cast<int64_t *>(smem + kThetaBytes + kRingBytes);
    int32_t *ac = reinterpret_cast<int32_t *>(smem + kThetaBytes + kRingBytes + (size_t)n_rec * 16);
    uint32_t *xl = reinterpret_cast<uint32_t *>(smem + kThetaBytes + kRingBytes +
                                                (size_t)n_rec * 16 + (size_t)owords * 32 * M * 4);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;

    for (int e = threadIdx.x; e < kThetaLen; e += blockDim.x) th[e] = d.theta[e];
    for (int e = threadIdx.x; e < n_rec; e += blockDim.x) {
        kr[2 * e] = d.site[4 * e];
        kr[2 * e + 1] = d.site[4 * e + 1];
    }
    for (int e = threadIdx.x; e < owords * 32 * M; e += blockDim.x) ac[e] = d.acol[e];
    for (int e = threadIdx.x; e < words * kWave; e += blockDim.x) xl[e] = 0u;
    __syncthreads();

    const int r = rbase + lane;  // every wave serves the same 64 replicas
    const uint32_t kround = (uint32_t)d.round_k[0];
    const uint64_t m2 = (uint64_t)0xCD9E8D57u * (uint32_t)r;
    const int total = d.T * words;  // ring blocks per run

    if (wave > 0) produce_thresholds<3>(d, wave - 1, 0, 0, ring, th, kround, m2);
    __syncthreads();

    // Every wave walks the same sequence of ring blocks and meets the others
    // at the one barrier per block, outside the wave-dependent branches.
    const int n = d.n, n_ext = d.n_ext;
    const int32_t negk2 = -d.k2;
    int32_t g[M];
    uint32_t sk[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        g[k] = -(int32_t)d.b[k];
        sk[k] = 0u;
    }
    // The slack layout is read once and the next block's beta multiplier one block
    // ahead: inside the persistent batch loop the compiler must assume that the
    // previous item's stores may alias these constants, so a load in the sweep would
    // be a vector load waited on at the top of the visit chain.
    int soff[M], sq[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        soff[k] = d.slack_off[k];
        sq[k] = d.slack_q[k];
    }
    int buf = 0;
    for (int c = 0; c < total; ++c) {
        const int w = c - (c / words) * words;
        if (wave == 0) {
            const int64_t *rg = ring + buf * 32 * 64;
            const int base = w * 32;
            if (w < owords) {
                // original items of this word (the tail beyond n is slack, visited below)
                // old states from the word's start (a site changes only at its own visit)
                const uint32_t xw0 = xl[w * kWave + lane];
                uint32_t xw = xw0;
                const int rem = n - base;
                // operands read one visit ahead (sites up to base + 31 < owords*32: in bounds)
                LinOps<AHEAD ? M : 1> op[2];
                int64_t ztn[2];
                if constexpr (AHEAD) {
                    load_lin_ops<M>(op[0], ac, kr, base, xw0 & 1u);
                    ztn[0] = rg[lane];
                }
#pragma unroll
                for (int s = 0; s < 32; ++s) {
                    const int i = base + s;
                    if constexpr (AHEAD) {
                        if (s + 1 < 32) {
                            load_lin_ops<M>(op[(s + 1) & 1], ac, kr, i + 1, (xw0 >> (s + 1)) & 1u);
                            ztn[(s + 1) & 1] = rg[(s + 1) * 64 + lane];
                        }
                        __builtin_amdgcn_sched_barrier(0);
                    }
                    const uint32_t xo = (xw0 >> s) & 1u;
                    const int64_t zt = AHEAD ? ztn[s & 1] : rg[s * 64 + lane];
                    const int32_t *a = AHEAD ? op[s & 1].a : ac + i * M;
                    const int64_t K = AHEAD ? op[s & 1].K : kr[2 * i + xo];
                    const int64_t dd = residual_dot<M, WIDE>(a, g);
                    const int64_t Z = WIDE ? K + dd * (int64_t)negk2 : K + (int64_t)(int32_t)dd * negk2;
                    // sites past the original items belong to the slack loop: never flip here
                    const uint32_t xn = (uint32_t)(Z >= zt) & (uint32_t)(s < rem);
                    const int32_t delta = (int32_t)xn - (int32_t)xo;
#pragma unroll
                    for (int k = 0; k < M; ++k) g[k] = WIDE ? g[k] + delta * a[k] : mad_i24(delta, a[k], g[k]);
                    xw = (xw & ~(1u << s)) | (xn << s);
                }
                xl[w * kWave + lane] = xw;
            }
            // slack bits of this block, constraint by constraint (natural order)
            const int lo = max(base, n), hi = min(base + 32, n_ext);
            if (lo < hi) {
#pragma unroll
                for (int k = 0; k < M; ++k) {
                    const int off = soff[k];
                    const int q0 = max(0, lo - off), q1 = min(sq[k], hi - off);
                    const uint32_t sk0 = sk[k];
                    for (int q = q0; q < q1; ++q) {
                        const int i = off + q;
                        const int64_t zt = rg[(i - base) * 64 + lane];
                        const uint32_t xo = (sk0 >> q) & 1u;
                        const int64_t K = kr[2 * i + xo];
                        const int64_t Z = K + (((int64_t)g[k] * negk2) << q);
                        const uint32_t xn = Z >= zt ? 1u : 0u;
                        g[k] += ((int32_t)xn - (int32_t)xo) << q;
                        sk[k] = (sk[k] & ~(1u << q)) | (xn << q);
                    }
                }
            }
        } else if (c + 1 < total) {
            const int t1 = (c + 1) / words, b1 = (c + 1) - t1 * words;
            produce_thresholds<3>(d, wave - 1, t1, b1, ring + (buf ^ 1) * 32 * 64, th, kround, m2);
        }
        buf ^= 1;
        __syncthreads();
    }
    if (wave == 0) linear_score<M>(d, r, xl, lane, g, sk);
}

}  // namespace pbit

namespace pbit {

template <int M, bool WIDE>
__global__ __launch_bounds__(256) void sweep_linear_pc(const DevInstance d)
{
    extern __shared__ __align__(16) unsigned char smem[];
    linear_run_pc<M, WIDE>(d, blockIdx.x * kWave, smem);
}

// One workgroup of 4 waves per 64 replicas.
inline hipError_t launch_linear_pc_kernel(const void *kern, const DevInstance &d, hipStream_t stream)
{
    const size_t lds = linear_pc_lds_bytes(d.words, d.owords, d.m);
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const int blocks = (d.R + kWave - 1) / kWave;
    void *args[] = {const_cast<DevInstance *>(&d)};
    return hipLaunchKernel(kern, dim3(blocks), dim3(4 * kWave), args, lds, stream);
}

}  // namespace pbit

#define PBIT_LINEAR_PC_CASE(mm)                                                             \
    case mm:                                                                                \
        kern = wide ? reinterpret_cast<const void *>(&sweep_linear_pc<mm, true>)           \
                    : reinterpret_cast<const void *>(&sweep_linear_pc<mm, false>);         \
        break;
