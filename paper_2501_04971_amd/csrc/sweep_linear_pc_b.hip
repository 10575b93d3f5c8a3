// Instantiations of the producer/consumer linear kernel for M in {7,8,9,10,11,12}.
#include "sweep_linear_pc.h"

namespace pbit {

hipError_t launch_sweep_linear_pc_b(const DevInstance &d, bool wide, hipStream_t stream)
{
    const void *kern = nullptr;
    switch (d.m) {
        PBIT_LINEAR_PC_CASE(7) PBIT_LINEAR_PC_CASE(8) PBIT_LINEAR_PC_CASE(9) PBIT_LINEAR_PC_CASE(10) PBIT_LINEAR_PC_CASE(11) PBIT_LINEAR_PC_CASE(12)
        default:
            return hipErrorInvalidValue;
    }
    return launch_linear_pc_kernel(kern, d, stream);
}

}  // namespace pbit
