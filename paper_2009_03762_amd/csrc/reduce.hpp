// Reduction and stop test of one iteration, and the state reset of a solve.
// Non-template kernels: included by exactly one translation unit.
#pragma once

#include "kernels.hpp"

namespace lsfft {

// ---------------------------------------------------------------- reduction
// Two stages, both in a fixed order (deterministic): k_reduce_stage sums
// contiguous chunks of the x-pass and z-pass block sums into RSTAGE rows of
// 8 doubles; k_reduce sums those rows and takes the stop decision.
constexpr int RSTAGE = 64;

struct ReduceArgs {
  const double *px;   // x-pass block sums [system][nx][8] (6 stress sums, |d eps|^2, unused)
  int nx;
  const double *pz;   // z-pass block sums [system][nz]
  int nz;
  long long spx, spz; // strides between systems
  double *stage;      // [system][RSTAGE][8]: 6 stress sums, |d eps|^2, residual
  State *st;          // [system]
  double *hist;       // [system][hcap]
  long long hcap;
  const double *ebar_norms;  // [system] |Ebar|_F (RMS |E_*|_F for Ebar = 0 under eigenstrain)
  const double *smean;       // [system][6] mean eigenstress <C E_*> left out of the x-side sums, or null
  int maxit;
  double tol;
  int dgo;
  int disp;           // displacement form: residual from sum_x |div sigma|^2 (x-side slot 6)
  double N;
  double div_factor;
};

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
  a.st += sysb;
  a.hist += sysb * a.hcap;
  const double ebar_norm = a.ebar_norms[sysb];
  __shared__ double red[8];
  double vals[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int i = threadIdx.x; i < RSTAGE; i += 64)
    for (int c = 0; c < 8; ++c) vals[c] += a.stage[i * 8 + c];
  block_sum<64>(vals, 8, red);
  if (threadIdx.x != 0) return;
  State &s = *a.st;
  // the iteration index lives on the device, so that a captured sequence of
  // iterations can be replayed unchanged
  const int k = s.k;
  double mean[6];
  double sn = 0.0;
  for (int c = 0; c < 6; ++c) {
    mean[c] = vals[c] / a.N - (a.smean ? a.smean[6 * sysb + c] : 0.0);
    sn += (c < 3 ? 1.0 : 2.0) * mean[c] * mean[c];
  }
  double r;
  if (a.dgo) {
    r = (k == 0) ? __builtin_huge_val() : sqrt(vals[6]) / (sqrt(a.N) * ebar_norm);
  } else {
    const double num = a.disp ? sqrt(a.N * vals[6]) : sqrt(vals[7]);
    const double den = a.N * sqrt(sn);
    r = (num == 0.0) ? 0.0 : (den > 0.0 ? num / den : __builtin_huge_val());
  }
  a.hist[k] = r;
  s.r = r;
  for (int c = 0; c < 6; ++c) s.sig_mean[c] = mean[c];
  s.iters = k;
  const int first = a.dgo ? 1 : 0;
  if (k == first) s.r0 = r;
  int done = 0, status = 1;
  const bool finite = (r == r) && (r < __builtin_huge_val());
  if (a.dgo && k == 0) {
    if (k == a.maxit) { done = 1; status = 1; }
  } else if (r <= a.tol) {
    done = 1;
    status = 0;
  } else if (!a.dgo && k == a.maxit) {
    done = 1;
    status = 1;
  } else if (!finite || r > a.div_factor * fmax(s.r0, 1e-300)) {
    done = 1;
    status = 2;
  } else if (a.dgo && k == a.maxit) {
    done = 1;
    status = 1;
  }
  if (done) {
    s.status = status;
    s.done = 1;
  } else {
    s.k = k + 1;
  }
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
