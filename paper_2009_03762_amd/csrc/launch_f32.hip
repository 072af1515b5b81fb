// Pass-kernel launches of the float solvers, x side: the stencils, the
// displacement update and the kernel description.  The y and z passes and the
// strain-form x-pass of this precision live in launch_f32_yz.hip (two
// translation units, so the library's kernels compile in parallel).
#include "launch.hpp"

namespace lsfft_host {

template hipError_t Launch<float>::stencil(lsfft_solver, const lsfft::SArgs<float> &, int);
template hipError_t Launch<float>::uxpass(lsfft_solver, const lsfft::UArgs<float> &, int);
template std::string Launch<float>::describe(lsfft_solver);

}  // namespace lsfft_host
