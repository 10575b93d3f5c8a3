// Per-round bookkeeping on the device, so a round needs no host round trip:
//  - round_reduce: keep the best feasible sample (Algorithm 1, "store feasible
//    x_k" and the final argmin), sum the residuals over replicas, advance the
//    round counter;
//  - lambda_update: the multiplier step lambda <- lambda + eta g (Algorithm 1)
//    with the replica mean of g, exact on a 2^-32 accumulator and rounded to
//    the 2^-8 grid, then refresh the per-site field constants that depend on
//    lambda.
#include <hip/hip_runtime.h>

#include "pbit_types.h"

namespace pbit {

constexpr int kReduceThreads = 256;

__device__ __forceinline__ bool better(int64_t p, int32_t r, int64_t q, int32_t s)
{
    return p > q || (p == q && r < s);
}

__device__ __forceinline__ void round_reduce_body(const DevInstance &d)
{
    __shared__ int64_t sp[kReduceThreads];
    __shared__ int32_t sr[kReduceThreads];
    __shared__ int64_t sg[kReduceThreads];
    __shared__ int32_t sf[kReduceThreads];
    const int tid = threadIdx.x;

    int64_t bp = INT64_MIN;
    int32_t br = INT32_MAX;
    int32_t nf = 0;
    // the round's samples: every replica's final state, or with parallel
    // tempering each chain's replica at the coldest ladder position
    for (int r = tid; r < d.R; r += kReduceThreads) {
        if (d.pt == 0) d.rslot[r] = 0;
        if (d.rfeas[r] && (d.pt == 0 || d.rslot[r] == d.pt - 1)) {
            ++nf;
            const int64_t p = d.rprofit[r];
            if (better(p, r, bp, br)) {
                bp = p;
                br = r;
            }
        }
    }
    sp[tid] = bp;
    sr[tid] = br;
    sf[tid] = nf;
    __syncthreads();
    for (int h = kReduceThreads / 2; h > 0; h >>= 1) {
        if (tid < h) {
            if (better(sp[tid + h], sr[tid + h], sp[tid], sr[tid])) {
                sp[tid] = sp[tid + h];
                sr[tid] = sr[tid + h];
            }
            sf[tid] += sf[tid + h];
        }
        __syncthreads();
    }
    const int32_t k = d.round_k[0];
    const bool improve = sr[0] != INT32_MAX && (d.best[3] == 0 || sp[0] > d.best[0]);
    const int32_t rbest = sr[0];
    if (improve) {
        for (int w = tid; w < d.words; w += kReduceThreads)
            d.best_x[w] = d.rx[(int64_t)rbest * d.words + w];
    }
    // residual sums, one constraint at a time
    for (int c = 0; c < d.m; ++c) {
        int64_t s = 0;
        for (int r = tid; r < d.R; r += kReduceThreads)
            if (d.pt == 0 || d.rslot[r] == d.pt - 1) s += d.rg[(int64_t)r * d.m + c];
        sg[tid] = s;
        __syncthreads();
        for (int h = kReduceThreads / 2; h > 0; h >>= 1) {
            if (tid < h) sg[tid] += sg[tid + h];
            __syncthreads();
        }
        if (tid == 0) d.G[c] = sg[0];
        __syncthreads();
    }
    __syncthreads();  // every thread has read d.best before it is rewritten
    if (tid == 0) {
        if (improve) {
            d.best[0] = sp[0];
            d.best[1] = k;
            d.best[2] = rbest;
            d.best[3] = 1;
        }
        d.feas_count[0] = sf[0];
        d.round_k[0] = k + 1;
    }
}

// round(num * 2^32 / den) half away from zero, |num| < 2^62, 0 < den < 2^62,
// result below 2^62 in magnitude (bounded when the instance is created).
__device__ int64_t round_scaled_div(int64_t num, int64_t den)
{
    const bool neg = num < 0;
    const uint64_t a = neg ? (uint64_t)(-num) : (uint64_t)num;
    const uint64_t dv = (uint64_t)den;
    uint64_t q = a / dv, rem = a % dv;
    for (int bit = 0; bit < 32; ++bit) {
        rem <<= 1;
        q <<= 1;
        if (rem >= dv) {
            rem -= dv;
            q |= 1u;
        }
    }
    if (2 * rem >= dv) q += 1;
    return neg ? -(int64_t)q : (int64_t)q;
}

struct LambdaSet {
    int32_t v[kMaxM];
};

// mode 0: refresh constants only; 1: multiplier step from d.G; 2: set lambda_q from `vals`.
__device__ __forceinline__ void lambda_update_body(const DevInstance &d, int mode, const int32_t *vals)
{
    __shared__ int32_t lq[kMaxM];
    const int tid = threadIdx.x;
    if (tid < d.m) {
        int64_t acc = d.lam_acc[tid];
        const int64_t cap = d.lq_max << 24;
        if (mode == 1) {
            // step after round k = round_k - 1: eta, or eta H / (H + k)
            int64_t num = d.eta_num * d.G[tid], den = d.lam_den;
            if (d.eta_h > 0) {
                int64_t k = (int64_t)d.round_k[0] - 1;
                k = k < 0 ? 0 : (k > d.eta_kcap ? (int64_t)d.eta_kcap : k);
                num *= d.eta_h;
                den *= d.eta_h + k;
            }
            acc += round_scaled_div(num, den);
        }
        if (mode == 2) acc = (int64_t)vals[tid] * (1 << 24);
        acc = acc > cap ? cap : acc;
        acc = acc < -cap ? -cap : acc;
        // a multiplier held at the bound no longer follows Algorithm 1's step:
        // flag it (sticky) so the caller can tell
        if (mode != 0 && (acc == cap || acc == -cap)) atomicOr(d.lam_sat, 1u << tid);
        const int32_t q = acc >= 0 ? (int32_t)((acc + (1 << 23)) >> 24)
                                   : -(int32_t)((-acc + (1 << 23)) >> 24);
        d.lam_acc[tid] = acc;
        d.lam_q[tid] = q;
        lq[tid] = q;
    }
    __syncthreads();
    for (int i = tid; i < d.n_ext; i += blockDim.x) {
        int64_t al = 0;
        for (int c = 0; c < d.m; ++c) al += (int64_t)d.acol[(int64_t)i * d.m + c] * lq[c];
        const int64_t K0 = d.kbase[i] - d.sfsg * al;
        d.site[4 * i] = K0 * ((int64_t)1 << d.zsh);
        d.site[4 * i + 1] = (K0 + d.sa2[i]) * ((int64_t)1 << d.zsh);
    }
}

__global__ __launch_bounds__(kReduceThreads) void round_reduce(const DevInstance d)
{
    round_reduce_body(d);
}

__global__ __launch_bounds__(256) void lambda_update(const DevInstance d, int mode, LambdaSet set)
{
    lambda_update_body(d, mode, set.v);
}

// Batched forms: workgroup b serves instance b.  Members whose round budget is
// spent are skipped; the multiplier step consumes one unit of the budget.
__global__ __launch_bounds__(kReduceThreads) void round_reduce_batch(const DevInstance *insts)
{
    const DevInstance d = insts[blockIdx.x];
    if (d.rounds_left && d.rounds_left[0] <= 0) return;
    round_reduce_body(d);
}

__global__ __launch_bounds__(256) void lambda_update_batch(const DevInstance *insts, int mode)
{
    const DevInstance d = insts[blockIdx.x];
    if (mode == 1 && d.rounds_left && d.rounds_left[0] <= 0) return;
    lambda_update_body(d, mode, nullptr);
    __syncthreads();
    if (mode == 1 && d.rounds_left && threadIdx.x == 0) d.rounds_left[0] -= 1;
}

// Sets member b's lambda_q from values[b * kMaxM ..] (clamped to +-lq_max).
__global__ __launch_bounds__(256) void lambda_set_batch(const DevInstance *insts, const int32_t *values)
{
    const DevInstance d = insts[blockIdx.x];
    lambda_update_body(d, 2, values + (size_t)blockIdx.x * kMaxM);
}

// Per-member summary for host-side logs: best feasible profit and round, a
// feasible flag, rounds done, and lambda_q (zero beyond m).
__global__ __launch_bounds__(64) void batch_snapshot(const DevInstance *insts, unsigned char *out)
{
    const DevInstance d = insts[blockIdx.x];
    unsigned char *rec = out + (size_t)blockIdx.x * kSnapshotBytes;
    const int tid = threadIdx.x;
    if (tid == 0) {
        *reinterpret_cast<int64_t *>(rec) = d.best[0];
        int32_t *h = reinterpret_cast<int32_t *>(rec + 8);
        h[0] = (int32_t)d.best[1];
        h[1] = (int32_t)d.best[3];
        h[2] = d.round_k[0];
        h[3] = d.feas_count[0];
        h[4] = (int32_t)d.lam_sat[0];
        h[5] = 0;
    }
    if (tid < kMaxM) reinterpret_cast<int32_t *>(rec + 32)[tid] = tid < d.m ? d.lam_q[tid] : 0;
    // sums over the last round's samples: profits of the feasible ones, |g|^2
    // of all (fixed order: lane-strided partial sums, then a tree in LDS)
    __shared__ int64_t part[2][64];
    int64_t sp = 0, sq = 0;
    for (int r = tid; r < d.R; r += 64) {
        if (d.rfeas[r]) sp += d.rprofit[r];
        for (int k = 0; k < d.m; ++k) {
            const int64_t g = d.rg[(int64_t)r * d.m + k];
            sq += g * g;
        }
    }
    part[0][tid] = sp;
    part[1][tid] = sq;
    __syncthreads();
    for (int w = 32; w > 0; w >>= 1) {
        if (tid < w) {
            part[0][tid] += part[0][tid + w];
            part[1][tid] += part[1][tid + w];
        }
        __syncthreads();
    }
    if (tid == 0) {
        reinterpret_cast<int64_t *>(rec + 160)[0] = part[0][0];
        reinterpret_cast<int64_t *>(rec + 160)[1] = part[1][0];
    }
}

hipError_t launch_lambda_set_batch(const DevInstance *insts, int count, const int32_t *values, hipStream_t stream)
{
    void *args[] = {&insts, &values};
    return hipLaunchKernel(reinterpret_cast<const void *>(&lambda_set_batch), dim3(count), dim3(256), args, 0,
                           stream);
}

hipError_t launch_batch_snapshot(const DevInstance *insts, int count, unsigned char *out, hipStream_t stream)
{
    void *args[] = {&insts, &out};
    return hipLaunchKernel(reinterpret_cast<const void *>(&batch_snapshot), dim3(count), dim3(64), args, 0,
                           stream);
}

// Clears the work-queue counters (both families).
__global__ void reset_counter(int *counter)
{
    if (threadIdx.x < 2) counter[threadIdx.x] = 0;
}

const void *round_reduce_batch_kernel() { return reinterpret_cast<const void *>(&round_reduce_batch); }
const void *lambda_update_batch_kernel() { return reinterpret_cast<const void *>(&lambda_update_batch); }
const void *reset_counter_kernel() { return reinterpret_cast<const void *>(&reset_counter); }
int reduce_threads() { return kReduceThreads; }

hipError_t launch_round_reduce_batch(const DevInstance *insts, int count, hipStream_t stream)
{
    void *args[] = {&insts};
    return hipLaunchKernel(reinterpret_cast<const void *>(&round_reduce_batch), dim3(count),
                           dim3(kReduceThreads), args, 0, stream);
}

hipError_t launch_lambda_update_batch(const DevInstance *insts, int count, int mode, hipStream_t stream)
{
    void *args[] = {&insts, &mode};
    return hipLaunchKernel(reinterpret_cast<const void *>(&lambda_update_batch), dim3(count), dim3(256),
                           args, 0, stream);
}

hipError_t launch_reset_counter(int *counter, hipStream_t stream)
{
    void *args[] = {&counter};
    return hipLaunchKernel(reinterpret_cast<const void *>(&reset_counter), dim3(1), dim3(64), args, 0,
                           stream);
}

hipError_t launch_round_reduce(const DevInstance &d, hipStream_t stream)
{
    void *args[] = {const_cast<DevInstance *>(&d)};
    return hipLaunchKernel(reinterpret_cast<const void *>(&round_reduce), dim3(1),
                           dim3(kReduceThreads), args, 0, stream);
}

hipError_t launch_lambda_update(const DevInstance &d, int mode, const int32_t *values,
                                hipStream_t stream)
{
    LambdaSet set{};
    if (values)
        for (int c = 0; c < d.m && c < kMaxM; ++c) set.v[c] = values[c];
    void *args[] = {const_cast<DevInstance *>(&d), &mode, &set};
    return hipLaunchKernel(reinterpret_cast<const void *>(&lambda_update), dim3(1), dim3(256), args,
                           0, stream);
}

}  // namespace pbit
