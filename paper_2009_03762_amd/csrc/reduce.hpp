// Reduction and stop test of one iteration, and the state reset of a solve.
// Non-template kernels: included by exactly one translation unit.
#pragma once

#include "kernels.hpp"

namespace lsfft {

__global__ __launch_bounds__(256) void k_reduce_stage(ReduceArgs a) {
  const int sysb = blockIdx.y;
  if (a.st[sysb].done) return;
  a.px += sysb * a.spx;
  a.pz += sysb * a.spz;
  a.stage += (long long)sysb * RSTAGE * 8;
  __shared__ double red[4 * 8];
  const int b = blockIdx.x;
  const long long cx = (a.nx + RSTAGE - 1) / RSTAGE, cz = (a.nz + RSTAGE - 1) / RSTAGE;
  const long long x0 = b * cx, x1 = (x0 + cx < a.nx) ? x0 + cx : a.nx;
  const long long z0 = b * cz, z1 = (z0 + cz < a.nz) ? z0 + cz : a.nz;
  double vals[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (long long i = x0 + threadIdx.x; i < x1; i += 256)
    for (int c = 0; c < 7; ++c) vals[c] += a.px[i * 8 + c];
  for (long long i = z0 + threadIdx.x; i < z1; i += 256) vals[7] += a.pz[i];
  block_sum<256>(vals, 8, red);
  if (threadIdx.x == 0)
    for (int c = 0; c < 8; ++c) a.stage[b * 8 + c] = vals[c];
}

__global__ __launch_bounds__(64) void k_reduce(ReduceArgs a) {
  const int sysb = blockIdx.y;
  if (a.st[sysb].done) return;
  a.stage += (long long)sysb * RSTAGE * 8;
  __shared__ double red[8];
  double vals[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int i = threadIdx.x; i < RSTAGE; i += 64)
    for (int c = 0; c < 8; ++c) vals[c] += a.stage[i * 8 + c];
  block_sum<64>(vals, 8, red);
  if (threadIdx.x != 0) return;
  reduce_decide(a, sysb, vals);
}

// Iterative refinement of the F32 displacement form (see k_refine_stress):
// u_b += delta, delta = 0.
__global__ __launch_bounds__(256) void k_refine_fold(double *u, double *du, const State *st, long long n) {
  const int sysb = blockIdx.y;
  if (st[sysb].done) return;
  u += sysb * n;
  du += sysb * n;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    u[i] += du[i];
    du[i] = 0.0;
  }
}

// smean of the refined sweeps: minus the mean of sigma_b (the stopping test
// subtracts smean from the mean stress of delta), from `rows` rows of 8 block
// sums per system (`stride` doubles apart) and, when the block sums leave the
// eigenstress out, its mean emean.  Fixed summation order.
__global__ __launch_bounds__(64) void k_refine_mean(const double *part, int rows, long long stride, double *smean,
                                                    const double *emean, const State *st, double N) {
  const int sysb = blockIdx.x;
  if (st[sysb].done) return;
  part += (long long)sysb * stride;
  __shared__ double red[8];
  double vals[6] = {0, 0, 0, 0, 0, 0};
  for (int i = threadIdx.x; i < rows; i += 64)
    for (int c = 0; c < 6; ++c) vals[c] += part[i * 8 + c];
  block_sum<64>(vals, 6, red);
  if (threadIdx.x == 0)
    for (int c = 0; c < 6; ++c) smean[6 * sysb + c] = -(vals[c] / N - (emean ? emean[6 * sysb + c] : 0.0));
}

__global__ void k_state_init(State *st, int count) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < count) {
    State *s = st + b;
    s->done = 0;
    s->status = 1;
    s->iters = 0;
    s->k = 0;
    s->r0 = 0.0;
    s->r = 0.0;
    for (int c = 0; c < 6; ++c) s->sig_mean[c] = 0.0;
  }
}

}  // namespace lsfft
