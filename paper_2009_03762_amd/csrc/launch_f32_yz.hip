// Pass-kernel launches of the float solvers: the y and z passes (both forms)
// and the strain-form x-pass.
#include "launch.hpp"

namespace lsfft_host {

template hipError_t Launch<float>::xpass(lsfft_solver, const lsfft::XArgs<float> &, int);
template hipError_t Launch<float>::ypass<true>(lsfft_solver, const lsfft::YArgs<float> &, int);
template hipError_t Launch<float>::ypass<false>(lsfft_solver, const lsfft::YArgs<float> &, int);
template hipError_t Launch<float>::zpass(lsfft_solver, const lsfft::ZArgs<float> &, int);
template hipError_t Launch<float>::zpass_u(lsfft_solver, const lsfft::ZArgs<float> &, int);

}  // namespace lsfft_host
