// Set encoder that predicts starting multipliers lambda_0 (not part of the
// paper, whose Algorithm 1 starts from lambda_0 = 0; the paper's Fig. 3 and
// Sec. IV show the multipliers settling to an instance-dependent value, which
// is what the network learns to guess).
//
// One set per (instance, constraint); one element per original variable with
// 16 input features (four used).  phi: two 128-wide ReLU layers on the matrix
// cores (bf16 operands, fp32 accumulation), mean pooling over the set, then a
// head 144 -> 128 -> 1 on the vector ALUs.  Weights and every stored activation
// are bf16; accumulation is fp32.  Backward: the head in one workgroup (sets in
// order), the phi layers per group of sets on the matrix cores into per-group
// partial gradients, reduced in a fixed order, so every result is
// deterministic.  Adam keeps fp32 master weights and writes the bf16 copy.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "net_layout.h"

namespace pbit {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef uint16_t u16;

constexpr int LS = 136;  // LDS row stride (elements) of 128-wide bf16 tiles
constexpr int LS1 = 24;  // LDS row stride of the 16-wide first-layer weights
constexpr int TS = 40;   // LDS row stride of transposed 32-row tiles

__device__ __forceinline__ u16 f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);  // nearest, ties to even (inputs are finite)
    return (u16)(u >> 16);
}

__device__ __forceinline__ float bf2f(u16 h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf8 ld8(const u16 *p)
{
    const uint4 v = *reinterpret_cast<const uint4 *>(p);
    return __builtin_bit_cast(bf8, v);
}

__device__ __forceinline__ f16v mma(bf8 a, bf8 b, f16v c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// Row of element v of a 32x32 accumulator tile held by `lane` (its column is lane & 31).
__device__ __forceinline__ int acc_row(int lane, int v) { return 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3); }

// 32 rows x 128 bf16 from an LDS tile (stride LS) to global rows of 128.
__device__ __forceinline__ void tile_out(const u16 *T, u16 *dst, int lane)
{
    const int row = lane >> 1, c0 = (lane & 1) * 64;
#pragma unroll
    for (int q = 0; q < 8; ++q)
        *reinterpret_cast<uint4 *>(dst + (size_t)row * kNetH + c0 + 8 * q) =
            *reinterpret_cast<const uint4 *>(T + row * LS + c0 + 8 * q);
}

constexpr size_t kFwdLds = (size_t)kNetH * LS1 * 2 + (size_t)kNetH * LS * 2 + 4 * (size_t)32 * LS * 2;

// grid: one workgroup per set, 256 threads.
__global__ __launch_bounds__(256) void net_forward_kernel(const u16 *__restrict__ w, const u16 *__restrict__ x,
                                                          const u16 *__restrict__ ctx,
                                                          const int *__restrict__ set_rows,
                                                          const int *__restrict__ set_n, int rows,
                                                          u16 *__restrict__ H1g, u16 *__restrict__ H2g,
                                                          u16 *__restrict__ Zg, u16 *__restrict__ G1g,
                                                          float *__restrict__ tg)
{
    extern __shared__ __align__(16) unsigned char lds[];
    u16 *sW1 = reinterpret_cast<u16 *>(lds);
    u16 *sW2 = sW1 + kNetH * LS1;
    u16 *sT = sW2 + kNetH * LS;
    __shared__ float sb1[kNetH], sb2[kNetH], sZ[kNetZ], red[kNetH];
    __shared__ float pool[4][2][kNetH];

    const int s = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int e = tid; e < kNetH * kNetF; e += 256) sW1[(e / kNetF) * LS1 + e % kNetF] = w[kOffW1 + e];
    for (int e = tid; e < kNetH * kNetH / 8; e += 256) {
        const int r = e >> 4, c = (e & 15) * 8;
        *reinterpret_cast<uint4 *>(sW2 + r * LS + c) =
            *reinterpret_cast<const uint4 *>(w + kOffW2 + r * kNetH + c);
    }
    if (tid < kNetH) {
        sb1[tid] = bf2f(w[kOffB1 + tid]);
        sb2[tid] = bf2f(w[kOffB2 + tid]);
    }
    __syncthreads();

    const int r0 = set_rows[s], r1 = set_rows[s + 1], n = set_n[s];
    const int ntile = (n + 31) / 32;
    float psum[4] = {0.f, 0.f, 0.f, 0.f};
    u16 *T = sT + wave * 32 * LS;
    for (int tl = wave; tl < ntile; tl += 4) {
        const int row0 = r0 + tl * 32;
        if (row0 + 32 > r1 || row0 + 32 > rows) break;  // malformed set table: never read past it
        const int nvalid = min(32, n - tl * 32);
        const bf8 a = ld8(x + (size_t)(row0 + (lane & 31)) * kNetF + (lane >> 5) * 8);
        // layer 1: H1 = relu(X W1^T + b1), K = 16
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            f16v acc = {};
            acc = mma(a, ld8(sW1 + (cb * 32 + (lane & 31)) * LS1 + (lane >> 5) * 8), acc);
            const int j = cb * 32 + (lane & 31);
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const float h = acc[v] + sb1[j];
                T[acc_row(lane, v) * LS + j] = f2bf(h > 0.f ? h : 0.f);
            }
        }
        tile_out(T, H1g + (size_t)row0 * kNetH, lane);
        // layer 2: H2 = relu(H1 W2^T + b2), K = 128
        f16v acc[4];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            acc[cb] = f16v{};
#pragma unroll
            for (int ks = 0; ks < 8; ++ks)
                acc[cb] = mma(ld8(T + (lane & 31) * LS + ks * 16 + (lane >> 5) * 8),
                              ld8(sW2 + (cb * 32 + (lane & 31)) * LS + ks * 16 + (lane >> 5) * 8), acc[cb]);
        }
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            const int j = cb * 32 + (lane & 31);
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int i = acc_row(lane, v);
                const float h = acc[cb][v] + sb2[j];
                const u16 hb = f2bf(h > 0.f ? h : 0.f);
                T[i * LS + j] = hb;
                if (i < nvalid) psum[cb] += bf2f(hb);
            }
        }
        tile_out(T, H2g + (size_t)row0 * kNetH, lane);
    }
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) pool[wave][lane >> 5][cb * 32 + (lane & 31)] = psum[cb];
    __syncthreads();
    if (tid < kNetH) {
        float sum = 0.f;
        for (int wv = 0; wv < 4; ++wv) sum += pool[wv][0][tid] + pool[wv][1][tid];
        const u16 pb = f2bf(sum / (float)n);
        sZ[tid] = bf2f(pb);
        Zg[(size_t)s * kNetZ + tid] = pb;
    } else if (tid < kNetZ) {
        const u16 cb = ctx[(size_t)s * kNetCtx + (tid - kNetH)];
        sZ[tid] = bf2f(cb);
        Zg[(size_t)s * kNetZ + tid] = cb;
    }
    __syncthreads();
    // head: G1 = relu(W3 z + b3), t = w4 . G1 + b4
    if (tid < kNetH) {
        float g = bf2f(w[kOffB3 + tid]);
        const u16 *row = w + kOffW3 + tid * kNetZ;
        for (int c = 0; c < kNetZ; ++c) g += bf2f(row[c]) * sZ[c];
        const u16 gb = f2bf(g > 0.f ? g : 0.f);
        G1g[(size_t)s * kNetH + tid] = gb;
        red[tid] = bf2f(w[kOffW4 + tid]) * bf2f(gb);
    }
    __syncthreads();
    for (int h = kNetH / 2; h > 0; h >>= 1) {
        if (tid < h) red[tid] += red[tid + h];
        __syncthreads();
    }
    if (tid == 0) tg[s] = red[0] + bf2f(w[kOffB4]);
}

// Head backward and the loss: one workgroup, sets in order.
__global__ __launch_bounds__(256) void net_head_backward_kernel(const u16 *__restrict__ w,
                                                                const u16 *__restrict__ Zg,
                                                                const u16 *__restrict__ G1g,
                                                                const float *__restrict__ tg,
                                                                const float *__restrict__ y, int S,
                                                                float *__restrict__ dPg,
                                                                float *__restrict__ grad,
                                                                float *__restrict__ loss)
{
    __shared__ float sdG[kNetH], sz[kNetZ];
    constexpr int Q = kNetH * kNetZ / 256;  // W3 entries per thread
    const int tid = threadIdx.x;
    float aW3[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) aW3[q] = 0.f;
    float gb3 = 0.f, gw4 = 0.f, gb4 = 0.f, lsum = 0.f;
    const float invS = 1.f / (float)S;
    for (int s = 0; s < S; ++s) {
        const float r = tg[s] - y[s];
        const float ar = fabsf(r);
        const float dt = fminf(fmaxf(r, -1.f), 1.f) * invS;
        if (tid == 0) lsum += ar <= 1.f ? 0.5f * r * r : ar - 0.5f;
        gb4 += dt;
        if (tid < kNetH) {
            const float G = bf2f(G1g[(size_t)s * kNetH + tid]);
            const float dG = G > 0.f ? dt * bf2f(w[kOffW4 + tid]) : 0.f;
            sdG[tid] = dG;
            gw4 += dt * G;
            gb3 += dG;
        }
        if (tid < kNetZ) sz[tid] = bf2f(Zg[(size_t)s * kNetZ + tid]);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int e = tid + 256 * q;
            aW3[q] += sdG[e / kNetZ] * sz[e % kNetZ];
        }
        if (tid < kNetH) {
            float dp = 0.f;
            for (int j = 0; j < kNetH; ++j) dp += bf2f(w[kOffW3 + j * kNetZ + tid]) * sdG[j];
            dPg[(size_t)s * kNetH + tid] = dp;
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) grad[kOffW3 + tid + 256 * q] = aW3[q];
    if (tid < kNetH) {
        grad[kOffB3 + tid] = gb3;
        grad[kOffW4 + tid] = gw4;
    }
    if (tid == 0) {
        grad[kOffB4] = gb4;
        loss[0] = lsum * invS;
    }
}

constexpr size_t kBwdLds = (size_t)kNetH * LS * 2 + 3 * (size_t)kNetH * TS * 2 + (size_t)32 * LS * 2 +
                           (size_t)32 * TS * 2;

// phi backward: workgroup b takes sets b, b + grid, ... and writes one partial
// gradient of (W1, b1, W2, b2).
__global__ __launch_bounds__(256) void net_phi_backward_kernel(const u16 *__restrict__ w,
                                                               const u16 *__restrict__ x,
                                                               const int *__restrict__ set_rows,
                                                               const int *__restrict__ set_n, int S, int rows,
                                                               const u16 *__restrict__ H1g,
                                                               const u16 *__restrict__ H2g,
                                                               const float *__restrict__ dPg,
                                                               float *__restrict__ partial)
{
    extern __shared__ __align__(16) unsigned char lds[];
    u16 *sW2T = reinterpret_cast<u16 *>(lds);  // [in][out]
    u16 *sH1T = sW2T + kNetH * LS;             // [in][row]
    u16 *sdH2T = sH1T + kNetH * TS;            // [out][row]
    u16 *sdH1T = sdH2T + kNetH * TS;           // [h][row]
    u16 *sdH2 = sdH1T + kNetH * TS;            // [row][out]
    u16 *sXT = sdH2 + 32 * LS;                 // [f][row], f >= 16 zero
    __shared__ float sds[kNetH];
    __shared__ float sdb1[2][kNetH];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int e = tid; e < kNetH * kNetH; e += 256) sW2T[(e % kNetH) * LS + e / kNetH] = w[kOffW2 + e];
    for (int e = tid; e < 32 * TS; e += 256) sXT[e] = 0;
    f16v acc2[4], acc1 = {};
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) acc2[cb] = f16v{};
    float db1 = 0.f, db2 = 0.f;
    __syncthreads();

    for (int s = blockIdx.x; s < S; s += gridDim.x) {
        const int r0 = set_rows[s], r1 = set_rows[s + 1], n = set_n[s];
        if (tid < kNetH) sds[tid] = bf2f(f2bf(dPg[(size_t)s * kNetH + tid] / (float)n));
        __syncthreads();
        const int ntile = (n + 31) / 32;
        for (int tl = 0; tl < ntile; ++tl) {
            const int row0 = r0 + tl * 32;
            if (row0 + 32 > r1 || row0 + 32 > rows) break;  // uniform over the workgroup
            const int nvalid = min(32, n - tl * 32);
            {
                const int row = tid >> 3, c0 = (tid & 7) * 16;
                const uint4 *h1 = reinterpret_cast<const uint4 *>(H1g + (size_t)(row0 + row) * kNetH + c0);
                const uint4 *h2 = reinterpret_cast<const uint4 *>(H2g + (size_t)(row0 + row) * kNetH + c0);
                uint4 hv[2] = {h1[0], h1[1]};
                uint4 gv[2] = {h2[0], h2[1]};
                const u16 *hs = reinterpret_cast<const u16 *>(hv);
                const u16 *gs = reinterpret_cast<const u16 *>(gv);
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    sH1T[(c0 + q) * TS + row] = hs[q];
                    const u16 d = (row < nvalid && bf2f(gs[q]) > 0.f) ? f2bf(sds[c0 + q]) : (u16)0;
                    sdH2[row * LS + c0 + q] = d;
                    sdH2T[(c0 + q) * TS + row] = d;
                }
                if (tid < 64) {
                    const uint4 xv = *reinterpret_cast<const uint4 *>(x + (size_t)(row0 + (tid >> 1)) * kNetF +
                                                                      (tid & 1) * 8);
                    const u16 *xs = reinterpret_cast<const u16 *>(&xv);
#pragma unroll
                    for (int q = 0; q < 8; ++q) sXT[((tid & 1) * 8 + q) * TS + (tid >> 1)] = xs[q];
                }
            }
            __syncthreads();
            if (tid < kNetH) {
                float a = 0.f;
                for (int rr = 0; rr < 32; ++rr) a += bf2f(sdH2T[tid * TS + rr]);
                db2 += a;
            }
            {
                // dH1 = (dH2 W2) masked by H1 > 0; this wave: columns 32*wave ..
                f16v a = {};
#pragma unroll
                for (int ks = 0; ks < 8; ++ks)
                    a = mma(ld8(sdH2 + (lane & 31) * LS + ks * 16 + (lane >> 5) * 8),
                            ld8(sW2T + (wave * 32 + (lane & 31)) * LS + ks * 16 + (lane >> 5) * 8), a);
                const int j = wave * 32 + (lane & 31);
                float cs = 0.f;
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int i = acc_row(lane, v);
                    const u16 d = bf2f(sH1T[j * TS + i]) > 0.f ? f2bf(a[v]) : (u16)0;
                    sdH1T[j * TS + i] = d;
                    cs += bf2f(d);
                }
                db1 += cs;
            }
            __syncthreads();
            // dW2[out block = wave] += dH2^T H1; dW1[h block = wave] += dH1^T X
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                const bf8 A = ld8(sdH2T + (wave * 32 + (lane & 31)) * TS + ks * 16 + (lane >> 5) * 8);
#pragma unroll
                for (int cb = 0; cb < 4; ++cb)
                    acc2[cb] = mma(A, ld8(sH1T + (cb * 32 + (lane & 31)) * TS + ks * 16 + (lane >> 5) * 8),
                                   acc2[cb]);
                acc1 = mma(ld8(sdH1T + (wave * 32 + (lane & 31)) * TS + ks * 16 + (lane >> 5) * 8),
                           ld8(sXT + (lane & 31) * TS + ks * 16 + (lane >> 5) * 8), acc1);
            }
            __syncthreads();
        }
    }
    float *pp = partial + (size_t)blockIdx.x * kNetPhiParams;
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int v = 0; v < 16; ++v)
            pp[kOffW2 + (wave * 32 + acc_row(lane, v)) * kNetH + cb * 32 + (lane & 31)] = acc2[cb][v];
    if ((lane & 31) < kNetF) {
#pragma unroll
        for (int v = 0; v < 16; ++v) pp[kOffW1 + (wave * 32 + acc_row(lane, v)) * kNetF + (lane & 31)] = acc1[v];
    }
    sdb1[lane >> 5][wave * 32 + (lane & 31)] = db1;
    __syncthreads();
    if (tid < kNetH) {
        pp[kOffB1 + tid] = sdb1[0][tid] + sdb1[1][tid];
        pp[kOffB2 + tid] = db2;
    }
}

__global__ __launch_bounds__(256) void net_reduce_kernel(const float *__restrict__ partial, int groups,
                                                         float *__restrict__ grad)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= kNetPhiParams) return;
    float s = 0.f;
    for (int b = 0; b < groups; ++b) s += partial[(size_t)b * kNetPhiParams + e];
    grad[e] = s;
}

__global__ __launch_bounds__(256) void net_adam_kernel(float *__restrict__ wm, float *__restrict__ m,
                                                       float *__restrict__ v, const float *__restrict__ g,
                                                       u16 *__restrict__ wb, int np, float lr, float b1,
                                                       float b2, float eps, float bc1, float bc2)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= np) return;
    const float gi = g[e];
    const float mi = b1 * m[e] + (1.f - b1) * gi;
    const float vi = b2 * v[e] + (1.f - b2) * gi * gi;
    m[e] = mi;
    v[e] = vi;
    const float wi = wm[e] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    wm[e] = wi;
    wb[e] = f2bf(wi);
}

__global__ __launch_bounds__(256) void net_cast_kernel(const float *__restrict__ wm, u16 *__restrict__ wb, int np)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e < np) wb[e] = f2bf(wm[e]);
}

// lambda_q = round half away from zero of t * scale (float64), clamped to +-2^30.
__global__ __launch_bounds__(256) void net_to_lambda_kernel(const float *__restrict__ t,
                                                            const double *__restrict__ scale,
                                                            const int *__restrict__ dest, int S,
                                                            int *__restrict__ lam)
{
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= S) return;
    const double v = (double)t[s] * scale[s];
    double a = floor(fabs(v) + 0.5);
    a = a > 1073741824.0 ? 1073741824.0 : a;
    lam[dest[s]] = (int)(v >= 0 ? a : -a);
}

hipError_t net_launch_forward(const u16 *w, const u16 *x, const u16 *ctx, const int *set_rows, const int *set_n,
                              int S, int rows, u16 *H1, u16 *H2, u16 *Z, u16 *G1, float *t, hipStream_t st)
{
    const void *k = reinterpret_cast<const void *>(&net_forward_kernel);
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kFwdLds);
    if (e != hipSuccess) return e;
    void *args[] = {&w, &x, &ctx, &set_rows, &set_n, &rows, &H1, &H2, &Z, &G1, &t};
    return hipLaunchKernel(k, dim3(S), dim3(256), args, kFwdLds, st);
}

hipError_t net_launch_backward(const u16 *w, const u16 *x, const int *set_rows, const int *set_n, int S, int rows,
                               const u16 *H1, const u16 *H2, const u16 *Z, const u16 *G1, const float *t,
                               const float *y, float *dP, float *partial, int groups, float *grad, float *loss,
                               hipStream_t st)
{
    void *ah[] = {&w, &Z, &G1, &t, &y, &S, &dP, &grad, &loss};
    hipError_t e = hipLaunchKernel(reinterpret_cast<const void *>(&net_head_backward_kernel), dim3(1), dim3(256),
                                   ah, 0, st);
    if (e != hipSuccess) return e;
    const void *k = reinterpret_cast<const void *>(&net_phi_backward_kernel);
    e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kBwdLds);
    if (e != hipSuccess) return e;
    void *ap[] = {&w, &x, &set_rows, &set_n, &S, &rows, &H1, &H2, &dP, &partial};
    e = hipLaunchKernel(k, dim3(groups), dim3(256), ap, kBwdLds, st);
    if (e != hipSuccess) return e;
    void *ar[] = {&partial, &groups, &grad};
    return hipLaunchKernel(reinterpret_cast<const void *>(&net_reduce_kernel),
                           dim3((kNetPhiParams + 255) / 256), dim3(256), ar, 0, st);
}

hipError_t net_launch_adam(float *wm, float *m, float *v, const float *g, u16 *wb, float lr, float b1, float b2,
                           float eps, float bc1, float bc2, hipStream_t st)
{
    int np = kNetParams;
    void *a[] = {&wm, &m, &v, &g, &wb, &np, &lr, &b1, &b2, &eps, &bc1, &bc2};
    return hipLaunchKernel(reinterpret_cast<const void *>(&net_adam_kernel), dim3((np + 255) / 256), dim3(256), a,
                           0, st);
}

hipError_t net_launch_cast(const float *wm, u16 *wb, hipStream_t st)
{
    int np = kNetParams;
    void *a[] = {&wm, &wb, &np};
    return hipLaunchKernel(reinterpret_cast<const void *>(&net_cast_kernel), dim3((np + 255) / 256), dim3(256), a,
                           0, st);
}

hipError_t net_launch_to_lambda(const float *t, const double *scale, const int *dest, int S, int *lam,
                                hipStream_t st)
{
    void *a[] = {&t, &scale, &dest, &S, &lam};
    return hipLaunchKernel(reinterpret_cast<const void *>(&net_to_lambda_kernel), dim3((S + 255) / 256),
                           dim3(256), a, 0, st);
}

}  // namespace pbit
