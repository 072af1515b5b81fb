// Pass-kernel launches of the double solvers: every instantiation of the x, y,
// z, displacement-update and stencil kernels in this precision lives in this
// translation unit.
#include "launch.hpp"

namespace lsfft_host {

template struct Launch<double>;
template hipError_t Launch<double>::ypass<true>(lsfft_solver, const lsfft::YArgs<double> &, int);
template hipError_t Launch<double>::ypass<false>(lsfft_solver, const lsfft::YArgs<double> &, int);

}  // namespace lsfft_host
