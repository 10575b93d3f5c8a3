// Instantiations of the linear sweep kernel for 1 <= M <= 6 constraints.
#include "sweep_linear.h"

namespace pbit {

hipError_t launch_sweep_linear_a(const DevInstance &d, bool wide, int waves_per_block, bool resident,
                                   hipStream_t stream)
{
    const void *kern = nullptr;
    switch (d.m) {
        PBIT_LINEAR_CASE(1) PBIT_LINEAR_CASE(2) PBIT_LINEAR_CASE(3) PBIT_LINEAR_CASE(4) PBIT_LINEAR_CASE(5) PBIT_LINEAR_CASE(6)
        default:
            return hipErrorInvalidValue;
    }
    return launch_linear_kernel(kern, d, waves_per_block, resident, stream);
}

}  // namespace pbit
