// Instantiations of the linear sweep kernel for 7 <= M <= 12 constraints.
#include "sweep_linear.h"

namespace pbit {

hipError_t launch_sweep_linear_b(const DevInstance &d, bool wide, int waves_per_block, bool resident,
                                   hipStream_t stream)
{
    const void *kern = nullptr;
    switch (d.m) {
        PBIT_LINEAR_CASE(7) PBIT_LINEAR_CASE(8) PBIT_LINEAR_CASE(9) PBIT_LINEAR_CASE(10) PBIT_LINEAR_CASE(11) PBIT_LINEAR_CASE(12)
        default:
            return hipErrorInvalidValue;
    }
    return launch_linear_kernel(kern, d, waves_per_block, resident, stream);
}

}  // namespace pbit
