// Pass-kernel launches of the double solvers, x side: the stencils, the
// displacement update and the kernel description.  The y and z passes and the
// strain-form x-pass of this precision live in launch_f64_yz.hip (two
// translation units, so the library's kernels compile in parallel).
#include "launch.hpp"

namespace lsfft_host {

template hipError_t Launch<double>::stencil(lsfft_solver, const lsfft::SArgs<double> &, int);
template hipError_t Launch<double>::uxpass(lsfft_solver, const lsfft::UArgs<double> &, int);
template std::string Launch<double>::describe(lsfft_solver);

}  // namespace lsfft_host
