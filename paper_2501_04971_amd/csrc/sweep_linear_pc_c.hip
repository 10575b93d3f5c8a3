// Instantiations of the producer/consumer linear kernel for M in {13,14,15,16,17,18,19,20}.
#include "sweep_linear_pc.h"

namespace pbit {

hipError_t launch_sweep_linear_pc_c(const DevInstance &d, bool wide, hipStream_t stream)
{
    const void *kern = nullptr;
    switch (d.m) {
        PBIT_LINEAR_PC_CASE(13) PBIT_LINEAR_PC_CASE(14) PBIT_LINEAR_PC_CASE(15) PBIT_LINEAR_PC_CASE(16) PBIT_LINEAR_PC_CASE(17) PBIT_LINEAR_PC_CASE(18) PBIT_LINEAR_PC_CASE(19) PBIT_LINEAR_PC_CASE(20)
        default:
            return hipErrorInvalidValue;
    }
    return launch_linear_pc_kernel(kern, d, stream);
}

}  // namespace pbit
