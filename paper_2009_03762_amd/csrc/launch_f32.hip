// Pass-kernel launches of the float solvers: every instantiation of the x, y,
// z, displacement-update and stencil kernels in this precision lives in this
// translation unit.
#include "launch.hpp"

namespace lsfft_host {

template struct Launch<float>;
template hipError_t Launch<float>::ypass<true>(lsfft_solver, const lsfft::YArgs<float> &, int);
template hipError_t Launch<float>::ypass<false>(lsfft_solver, const lsfft::YArgs<float> &, int);

}  // namespace lsfft_host
