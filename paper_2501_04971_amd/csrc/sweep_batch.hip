// Persistent annealing kernels for a batch of instances of different kinds and
// sizes: every workgroup (4 waves = 256 replicas) takes work items (instance,
// first replica, kernel variant) from a queue ordered by decreasing estimated
// cost through one atomic counter, runs the annealing run of that replica
// tile with the body of the matching variant, and takes the next item until
// the queue is empty.  Quadratic and linear items have a kernel and a queue
// each.  All items of a round are independent, so the order in which
// workgroups take them changes no result.
#include "sweep_linear_pc.h"
#include "sweep_quad.h"

namespace pbit {

// The variant bodies of a family are inlined into that family's kernel.
template <int NB>
__device__ __forceinline__ void batch_quad(const DevInstance &d, int rbase, unsigned char *smem)
{
    quad_run<NB, 4>(d, rbase, smem);
}

// A linear item is either a plain tile (4 waves visiting 256 replicas) or a
// split tile (one wave visiting 64 replicas, three precomputing its draws and
// thresholds); the host gives the split form to the members whose chains are
// long enough to bound the round.
template <int M, bool WIDE>
__device__ __forceinline__ void batch_linear(const DevInstance &d, int rbase, bool split, unsigned char *smem)
{
    // operands read at the visit: this kernel's registers are full (see lin_read_ahead)
    if (split) linear_run_pc<M, WIDE, false>(d, rbase, smem);
    else linear_run_lds<M, WIDE, false>(d, rbase, smem);
}

#define PBIT_BQ(nb)                                                                         \
    case nb - 1:                                                                            \
        batch_quad<nb>(insts[item.x], item.y, smem);                                                   \
        break;
#define PBIT_BL(idx, mm)                                                                    \
    case 32 + 2 * idx:                                                                      \
        batch_linear<mm, false>(insts[item.x], item.y, split, smem);                        \
        break;                                                                              \
    case 33 + 2 * idx:                                                                      \
        batch_linear<mm, true>(insts[item.x], item.y, split, smem);                         \
        break;

// LINEAR = false serves the quadratic items, true the linear ones: two
// kernels, so that each family of bodies is register-allocated on its own.
template <bool LINEAR>
__global__ __launch_bounds__(256) void sweep_batch(
    const DevInstance *__restrict__ insts, const int4 *__restrict__ items, int n_items, int *__restrict__ counter)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(counter, 1);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(next);
        __syncthreads();
        if (it >= n_items) break;
        const int4 item = items[it];  // instance, first replica, variant, estimated cost
        const int *left = insts[item.x].rounds_left;
        if (left && left[0] <= 0) continue;
        if constexpr (!LINEAR) {
            switch (item.z) {
                PBIT_BQ(1) PBIT_BQ(2) PBIT_BQ(3) PBIT_BQ(4) PBIT_BQ(5) PBIT_BQ(6)
                PBIT_BQ(7) PBIT_BQ(8) PBIT_BQ(9) PBIT_BQ(10) PBIT_BQ(11)
                default:
                    break;
            }
        } else {
            const bool split = (item.z & kBatchSplit) != 0;
            switch (item.z & ~kBatchSplit) {
                PBIT_BL(0, 1) PBIT_BL(1, 2) PBIT_BL(2, 3) PBIT_BL(3, 4) PBIT_BL(4, 5) PBIT_BL(5, 6)
                PBIT_BL(6, 8) PBIT_BL(7, 10) PBIT_BL(8, 16) PBIT_BL(9, 30) PBIT_BL(10, 32)
                default:
                    break;
            }
        }
        __syncthreads();  // LDS is reused by the next item
    }
}

const void *sweep_batch_kernel(bool linear)
{
    return linear ? reinterpret_cast<const void *>(&sweep_batch<true>) : reinterpret_cast<const void *>(&sweep_batch<false>);
}

// Constraint count of the batch body that serves m constraints (0 if none).
int batch_linear_m(int m)
{
    static const int ms[11] = {1, 2, 3, 4, 5, 6, 8, 10, 16, 30, 32};
    for (int v : ms)
        if (v >= m) return v;
    return 0;
}

// Queue code of the body for a member: NB - 1 for the quadratic body,
// 32 + 2 idx (+1 with 64-bit dots) for the linear bodies (kBatchSplit added
// by the host for split tiles).
int batch_variant_code(int variant, int nb, int m)
{
    if (variant == kQuad) return nb >= 1 && nb <= kMaxQuadBlocks ? nb - 1 : -1;
    static const int ms[11] = {1, 2, 3, 4, 5, 6, 8, 10, 16, 30, 32};
    for (int idx = 0; idx < 11; ++idx)
        if (ms[idx] == m) return 32 + 2 * idx + (variant == kLinearWide ? 1 : 0);
    return -1;
}

hipError_t sweep_batch_prepare(bool linear, size_t lds, int *blocks_per_cu)
{
    const void *kern = sweep_batch_kernel(linear);
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, kern, 256, lds);
}

hipError_t launch_sweep_batch(bool linear, const DevInstance *insts, const int4 *items, int n_items, int *counter,
                              int blocks, size_t lds, hipStream_t stream)
{
    void *args[] = {&insts, &items, &n_items, &counter};
    return hipLaunchKernel(sweep_batch_kernel(linear), dim3(blocks), dim3(256), args, lds, stream);
}

}  // namespace pbit
