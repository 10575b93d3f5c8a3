// Instantiations of the linear sweep kernel for 21 <= M <= 32 constraints.
#include "sweep_linear.h"

namespace pbit {

hipError_t launch_sweep_linear_d(const DevInstance &d, bool wide, int waves_per_block, bool resident,
                                   hipStream_t stream)
{
    const void *kern = nullptr;
    switch (d.m) {
        PBIT_LINEAR_CASE(21) PBIT_LINEAR_CASE(22) PBIT_LINEAR_CASE(23) PBIT_LINEAR_CASE(24) PBIT_LINEAR_CASE(25) PBIT_LINEAR_CASE(26) PBIT_LINEAR_CASE(27) PBIT_LINEAR_CASE(28) PBIT_LINEAR_CASE(29) PBIT_LINEAR_CASE(30) PBIT_LINEAR_CASE(31) PBIT_LINEAR_CASE(32)
        default:
            return hipErrorInvalidValue;
    }
    return launch_linear_kernel(kern, d, waves_per_block, resident, stream);
}

}  // namespace pbit
