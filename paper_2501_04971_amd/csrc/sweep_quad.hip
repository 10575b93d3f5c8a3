// Single-instance launches of the quadratic annealing kernel (see sweep_quad.h).
#include "sweep_quad.h"

namespace pbit {

template <int NB, int WPB, bool PT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void sweep_quad(const DevInstance d)
{
    extern __shared__ __align__(16) unsigned char smem[];
    quad_run<NB, WPB, PT>(d, blockIdx.x * WPB * kWave, smem);
}

// PT: parallel tempering instead of annealing (d.pt > 0)
#define PBIT_QUAD_CASE(nb)                                                                          \
    case nb:                                                                                        \
        kern = pt ? (wpb == 1 ? reinterpret_cast<const void *>(&sweep_quad<nb, 1, true>)             \
                              : reinterpret_cast<const void *>(&sweep_quad<nb, 4, true>))            \
                  : (wpb == 1 ? reinterpret_cast<const void *>(&sweep_quad<nb, 1, false>)            \
                              : reinterpret_cast<const void *>(&sweep_quad<nb, 4, false>));          \
        lds = quad_lds_bytes<nb>();                                                                 \
        break;

// waves_per_block: 1 or 4 (other values round to 4)
hipError_t launch_sweep_quad(const DevInstance &d, int nb, int waves_per_block, hipStream_t stream)
{
    const void *kern = nullptr;
    size_t lds = 0;
    const int wpb = waves_per_block == 1 ? 1 : 4;
    const bool pt = d.pt > 0;
    switch (nb) {
        PBIT_QUAD_CASE(1) PBIT_QUAD_CASE(2) PBIT_QUAD_CASE(3) PBIT_QUAD_CASE(4) PBIT_QUAD_CASE(5)
        PBIT_QUAD_CASE(6) PBIT_QUAD_CASE(7) PBIT_QUAD_CASE(8) PBIT_QUAD_CASE(9) PBIT_QUAD_CASE(10)
        PBIT_QUAD_CASE(11)
        default:
            return hipErrorInvalidValue;
    }
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const int waves = (d.R + kWave - 1) / kWave;
    const int blocks = (waves + wpb - 1) / wpb;
    void *args[] = {const_cast<DevInstance *>(&d)};
    return hipLaunchKernel(kern, dim3(blocks), dim3(wpb * kWave), args, lds, stream);
}

}  // namespace pbit
