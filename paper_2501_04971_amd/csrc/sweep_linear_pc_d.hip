// Instantiations of the producer/consumer linear kernel for M in {21,22,23,24,25,26,27,28,29,30,31,32}.
#include "sweep_linear_pc.h"

namespace pbit {

hipError_t launch_sweep_linear_pc_d(const DevInstance &d, bool wide, hipStream_t stream)
{
    const void *kern = nullptr;
    switch (d.m) {
        PBIT_LINEAR_PC_CASE(21) PBIT_LINEAR_PC_CASE(22) PBIT_LINEAR_PC_CASE(23) PBIT_LINEAR_PC_CASE(24) PBIT_LINEAR_PC_CASE(25) PBIT_LINEAR_PC_CASE(26) PBIT_LINEAR_PC_CASE(27) PBIT_LINEAR_PC_CASE(28) PBIT_LINEAR_PC_CASE(29) PBIT_LINEAR_PC_CASE(30) PBIT_LINEAR_PC_CASE(31) PBIT_LINEAR_PC_CASE(32)
        default:
            return hipErrorInvalidValue;
    }
    return launch_linear_pc_kernel(kern, d, stream);
}

}  // namespace pbit
