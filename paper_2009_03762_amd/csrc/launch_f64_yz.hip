// Pass-kernel launches of the double solvers: the y and z passes (both forms)
// and the strain-form x-pass.
#include "launch.hpp"

namespace lsfft_host {

template hipError_t Launch<double>::xpass(lsfft_solver, const lsfft::XArgs<double> &, int);
template hipError_t Launch<double>::ypass<true>(lsfft_solver, const lsfft::YArgs<double> &, int);
template hipError_t Launch<double>::ypass<false>(lsfft_solver, const lsfft::YArgs<double> &, int);
template hipError_t Launch<double>::zpass(lsfft_solver, const lsfft::ZArgs<double> &, int);
template hipError_t Launch<double>::zpass_u(lsfft_solver, const lsfft::ZArgs<double> &, int);

}  // namespace lsfft_host
