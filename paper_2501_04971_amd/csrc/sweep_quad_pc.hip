// Launches of the producer/consumer quadratic kernel (see sweep_quad_pc.h).
#include "sweep_quad_pc.h"

namespace pbit {

static_assert(quad_pc_lds_bytes<kMaxQuadBlocks>() <= 160 * 1024, "split layout exceeds the LDS of a CU");

template <int NB, int PR, bool PT>
__global__ __launch_bounds__(quad_pc_waves<PR>() * kWave) void sweep_quad_pc(const DevInstance d)
{
    extern __shared__ __align__(16) unsigned char smem[];
    quad_run_pc<NB, PR, PT>(d, blockIdx.x * kWave, smem);
}

// PT: parallel tempering (d.pt > 0), built with six producers only
#define PBIT_QUAD_PC_CASE(nb)                                                               \
    case nb:                                                                                \
        kern = pt ? reinterpret_cast<const void *>(&sweep_quad_pc<nb, 6, true>)             \
                  : (producers == 6 ? reinterpret_cast<const void *>(&sweep_quad_pc<nb, 6, false>) \
                                    : reinterpret_cast<const void *>(&sweep_quad_pc<nb, 3, false>)); \
        lds = quad_pc_lds_bytes<nb>();                                                      \
        break;

// One workgroup per 64 replicas, with 3 producer waves (4 waves in all) or 6
// (8 waves); parallel tempering takes 6.
hipError_t launch_sweep_quad_pc(const DevInstance &d, int nb, int producers, hipStream_t stream)
{
    const bool pt = d.pt > 0;
    if (producers != 3 && producers != 6) return hipErrorInvalidValue;
    if (pt && producers != 6) return hipErrorInvalidValue;
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
    const int threads = (producers == 6 ? quad_pc_waves<6>() : quad_pc_waves<3>()) * kWave;
    void *args[] = {const_cast<DevInstance *>(&d)};
    return hipLaunchKernel(kern, dim3(blocks), dim3(threads), args, lds, stream);
}

}  // namespace pbit
