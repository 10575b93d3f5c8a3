// Instantiations of the linear sweep kernel for 13 <= M <= 20 constraints.
#include "sweep_linear.h"

namespace pbit {

hipError_t launch_sweep_linear_c(const DevInstance &d, bool wide, int waves_per_block, bool resident,
                                   hipStream_t stream)
{
    const void *kern = nullptr;
    switch (d.m) {
        PBIT_LINEAR_CASE(13) PBIT_LINEAR_CASE(14) PBIT_LINEAR_CASE(15) PBIT_LINEAR_CASE(16) PBIT_LINEAR_CASE(17) PBIT_LINEAR_CASE(18) PBIT_LINEAR_CASE(19) PBIT_LINEAR_CASE(20)
        default:
            return hipErrorInvalidValue;
    }
    return launch_linear_kernel(kern, d, waves_per_block, resident, stream);
}

}  // namespace pbit
