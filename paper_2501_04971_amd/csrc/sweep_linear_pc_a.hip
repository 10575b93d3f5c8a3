// Instantiations of the producer/consumer linear kernel for M in {1,2,3,4,5,6}.
#include "sweep_linear_pc.h"

namespace pbit {

hipError_t launch_sweep_linear_pc_a(const DevInstance &d, bool wide, hipStream_t stream)
{
    const void *kern = nullptr;
    switch (d.m) {
        PBIT_LINEAR_PC_CASE(1) PBIT_LINEAR_PC_CASE(2) PBIT_LINEAR_PC_CASE(3) PBIT_LINEAR_PC_CASE(4) PBIT_LINEAR_PC_CASE(5) PBIT_LINEAR_PC_CASE(6)
        default:
            return hipErrorInvalidValue;
    }
    return launch_linear_pc_kernel(kern, d, stream);
}

}  // namespace pbit
