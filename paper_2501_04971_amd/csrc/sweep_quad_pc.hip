// Launches of the producer/consumer quadratic kernel (see sweep_quad_pc.h).
#include "sweep_quad_pc.h"

namespace pbit {

static_assert(quad_pc_lds_bytes<kMaxQuadBlocks>() <= 160 * 1024, "split layout exceeds the LDS of a CU");

template <int NB>
__global__ __launch_bounds__(256) void sweep_quad_pc(const DevInstance d)
{
    extern __shared__ __align__(16) unsigned char smem[];
    quad_run_pc<NB>(d, blockIdx.x * kWave, smem);
}

#define PBIT_QUAD_PC_CASE(nb)                                                               \
    case nb:                                                                                \
        kern = reinterpret_cast<const void *>(&sweep_quad_pc<nb>);                          \
        lds = quad_pc_lds_bytes<nb>();                                                      \
        break;

// One workgroup of 4 waves per 64 replicas.
hipError_t launch_sweep_quad_pc(const DevInstance &d, int nb, hipStream_t stream)
{
    const void *kern = nullptr;
    size_t lds = 0;
    switch (nb) {
        PBIT_QUAD_PC_CASE(1) PBIT_QUAD_PC_CASE(2) PBIT_QUAD_PC_CASE(3) PBIT_QUAD_PC_CASE(4)
        PBIT_QUAD_PC_CASE(5) PBIT_QUAD_PC_CASE(6) PBIT_QUAD_PC_CASE(7) PBIT_QUAD_PC_CASE(8)
        PBIT_QUAD_PC_CASE(9) PBIT_QUAD_PC_CASE(10) PBIT_QUAD_PC_CASE(11)
        default:
            return hipErrorInvalidValue;
    }
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const int blocks = (d.R + kWave - 1) / kWave;
    void *args[] = {const_cast<DevInstance *>(&d)};
    return hipLaunchKernel(kern, dim3(blocks), dim3(4 * kWave), args, lds, stream);
}

}  // namespace pbit
