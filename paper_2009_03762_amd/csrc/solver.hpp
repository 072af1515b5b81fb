// Internal header of the host library: launch-shape constants, the solver
// object behind the opaque lsfft_solver handle, and the kernel dispatch over
// the supported transform lengths (defined per precision in launch_f32.hip
// and launch_f64.hip, which build in parallel).
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "../../include/lsfft.h"
#include "disp.hpp"

using lsfft::cplx;
using lsfft::Dims;
using lsfft::State;

namespace lsfft_host {

// ------------------------------------------------------------------ sizes
// Points per thread for each transform: y and z use radix-8/4/2 passes with 8
// points per thread, x uses 4 (its six strain and six spectrum components are
// all held in registers); lengths with a factor 3 use 6 (x, z) or 12 (y),
// or the smallest multiple of 3 (of 6 on even lengths) that divides the
// length and keeps a line within the given number of threads.
#ifndef LSFFT_XE
#define LSFFT_XE 4
#endif
#ifndef LSFFT_ZE
#define LSFFT_ZE 8
#endif
#ifndef LSFFT_ZSEG
#define LSFFT_ZSEG 64
#endif
constexpr int e_pow2(int L) { return L < 8 ? L : 8; }
constexpr int e_mult3(int L, int maxtpc) {
  const int base = (L % 2 == 0) ? 6 : 3;
  for (int e = base; e < L; e += base)
    if (L % e == 0 && L / e <= maxtpc) return e;
  return L;
}
constexpr int ex_of(int L) { return (L % 3 == 0) ? (L < 6 ? L : e_mult3(L, 64)) : (L < LSFFT_XE ? L : LSFFT_XE); }
constexpr int ey_of(int n) {
  return (n % 3 == 0) ? (n < 12 ? n : (n % 12 == 0 ? 12 : e_mult3(n, 64))) : e_pow2(n);
}
constexpr int ez_of(int n) { return (n % 3 == 0) ? (n < 6 ? n : e_mult3(n, 64)) : (n < LSFFT_ZE ? n : LSFFT_ZE); }
// Columns per workgroup: at least `seg` bytes of each row (coalescing), at
// least 256 threads per workgroup.
template <typename T> constexpr int pcols_seg(int n, int E, int seg) {
  const int tpc = n / E;
  const int pmin = seg / (int)sizeof(cplx<T>);
  const int p = 256 / tpc;
  return p > pmin ? p : pmin;
}
template <typename T> constexpr int pcols(int n, int E) { return pcols_seg<T>(n, E, 128); }
template <typename T> constexpr int pcols_z(int n, int E) { return pcols_seg<T>(n, E, LSFFT_ZSEG * (int)sizeof(T) / 4); }
// z-pass of the displacement form (three components)
#ifndef LSFFT_ZUE
#define LSFFT_ZUE 8
#endif
#ifndef LSFFT_ZUSEG
#define LSFFT_ZUSEG LSFFT_ZSEG
#endif
#ifndef LSFFT_ZUE64
#define LSFFT_ZUE64 LSFFT_ZUE
#endif
// Lengths with a factor 3 from 288 take twelve points per thread where
// twelve divides them (five radix passes instead of seven at 288 and 384:
// FP64 z-pass at 384^3 966 us against 1143, FP32 288^3 225 against 241);
// below, six measured as fast or faster.
template <typename T> constexpr int ezu_of(int n) {
  const int e = sizeof(T) == 8 ? LSFFT_ZUE64 : LSFFT_ZUE;
  return (n % 3 == 0) ? (n < 6 ? n : ((n >= 288 && n % 12 == 0) ? 12 : e_mult3(n, 64))) : (n < e ? n : e);
}
template <typename T> constexpr int pcols_zu(int n, int E) {
  return pcols_seg<T>(n, E, LSFFT_ZUSEG * (int)sizeof(T) / 4);
}
// The alternative column tile of a y / z pass offered to the schedule tuner:
// twice the columns while the workgroup stays within 512 threads and 80 KB of
// LDS (two transposition buffers and the twiddles), else half of them while
// it keeps at least 64 threads; P itself when neither holds.
template <typename T> constexpr int palt(int n, int E, int P) {
  const int tpc = n / E;
  const long long lds2 = (2LL * n * (2 * P) + n) * (long long)sizeof(cplx<T>);
  if (2 * P * tpc <= 512 && lds2 <= 80 * 1024) return 2 * P;
  if (P % 2 == 0 && (P / 2) * tpc >= 64) return P / 2;
  return P;
}
constexpr int XWG = 256;
// Stencil kernel: its 2 x 3 x-transforms must fit in 256 threads (<= 32 threads each).
constexpr int es_of(int L) {
  return (L % 3 == 0) ? (L < 6 ? L : e_mult3(L, 32)) : (L < 4 ? L : (L > 128 ? L / 32 : 4));
}
// Points per thread of the register stencil's x-transforms: four on
// power-of-two lines (at most 64 threads per line, inside one wavefront),
// es_of on 3 * 2^a; lengths with a factor 9 pack their lines into
// wavefronts and may take two rounds of line transforms, so they allow up
// to 64 threads per line.
constexpr int esr_of(int L) {
  return (L % 9 == 0) ? e_mult3(L, 64) : ((L % 3 == 0) ? es_of(L) : (L < 4 ? L : 4));
}
#ifndef LSFFT_ST2
#define LSFFT_ST2 2
#endif
constexpr int ST2 = LSFFT_ST2;
// Node lines owned per y-group of a stencil workgroup: ST2, and one for FP64
// beyond 256 columns, where two would not fit in LDS.
template <typename T> constexpr int st2_of(int n1) { return (sizeof(T) == 8 && n1 > 256) ? 1 : ST2; }
// The register-resident stencil takes n1 = 2^a >= 8, 3 * 2^a in [12, 384]
// and the lengths with a factor 9 from 18 (see stencil_wg_of for their
// workgroups); 4 and 6 use the LDS stencil.
constexpr bool stencil_reg_kernel(int n1) {
  if (lsfft::pow2_len(n1)) return n1 >= 8;
  if (n1 % 3 == 0 && lsfft::pow2_len(n1 / 3)) return n1 >= 12 && n1 <= 384;
  return n1 % 9 == 0 && n1 >= 18;
}
// y-groups per register-stencil workgroup
constexpr int stencil_groups(int n1) {
  return (stencil_reg_kernel(n1) && n1 < lsfft::stencil_wg_of(n1)) ? lsfft::stencil_wg_of(n1) / n1 : 1;
}
// LDS of the stencil kernels (n1 values per line): the register-resident one
// holds one FP64 u plane (T2+2 lines x 3) per y-group, the two parts of the
// divergence exchange (T2 x 3 lines each), the transform scratch (3 T2 G
// complex lines) and the x twiddles; the other one two u planes, two sigma
// planes (T2+1 lines x 6) and the f lines.
template <typename T> constexpr long long stencil_lds(int n1) {
  const long long G = stencil_groups(n1);
  const long long t2 = st2_of<T>(n1);
  const long long ts = (long long)sizeof(T);
  if (stencil_reg_kernel(n1))
    return G * n1 * ((t2 + 2) * 3 * 8 + 2 * t2 * 3 * ts) + G * t2 * 3 * lsfft::line_scratch_of(n1 / 2) * 2 * ts +
           2LL * n1 * ts + 256;
  return G * n1 * (2 * (t2 + 2) * 3 * 8 + (2 * (t2 + 1) * 6 + t2 * 3) * ts) + 256;
}
template <typename T> constexpr bool stencil_fits(int n1) { return stencil_lds<T>(n1) <= 150000; }

// Lengths handled by the dispatch switches.  Every supported n_r (even,
// 2^a 3^b, in [4, 512]) appears for y / z; x uses n1/2.
#ifdef LSFFT_QUICK_BUILD
#define LSFFT_YZ_LENGTHS(X) X(8) X(16) X(64) X(256)
#define LSFFT_X_LENGTHS(X) X(4) X(8) X(32) X(128)
#else
#define LSFFT_YZ_LENGTHS(X)                                                                                  \
  X(4) X(6) X(8) X(12) X(16) X(18) X(24) X(32) X(36) X(48) X(54) X(64) X(72) X(96) X(108) X(128) X(144) X(162) \
  X(192) X(216) X(256) X(288) X(324) X(384) X(432) X(486) X(512)
#define LSFFT_X_LENGTHS(X)                                                                                   \
  X(2) X(3) X(4) X(6) X(8) X(9) X(12) X(16) X(18) X(24) X(27) X(32) X(36) X(48) X(54) X(64) X(72) X(81) X(96)  \
  X(108) X(128) X(144) X(162) X(192) X(216) X(243) X(256)
#endif

}  // namespace lsfft_host

struct lsfft_solver_s {
  int n[3];
  double h[3];
  double lam0, mu0;       // reference medium of system 0 (operator entry points)
  int B = 1;              // systems in the batch
  int launch_b = 1;       // systems covered by the launches being issued
  std::vector<double> lam0v, mu0v;  // reference medium of every system
  void *mem = nullptr;    // lsfft::Member<T>[B]
  double *enorm = nullptr;  // |Ebar|_F of every system
  lsfft::Strides bs{};
  long long spx = 0, spz = 0;  // doubles between systems in px / pz
  int disc, scheme, prec, M, pw;
  hipStream_t stream;
  Dims d;
  void *eps = nullptr, *lam = nullptr, *mu = nullptr, *spec = nullptr, *nyq = nullptr;
  void *tab = nullptr, *twx = nullptr, *twy = nullptr, *twz = nullptr;
  void *dgo_main = nullptr, *dgo_nyq = nullptr;
  void *u = nullptr;      // displacement (FB, AFB): [3][n3][n2][n1], FP64 in both precisions
  int disp = 0;           // 1: displacement-form path with real-space stencils
  int sZ = 0, nsb = 0, nub = 0;
  double *px = nullptr, *pz = nullptr, *pg = nullptr, *pstage = nullptr;
  int nxb = 0, nzb = 0, nyb = 0, ngb = 0;
  long long y_main_blocks = 0, z_main_blocks = 0;
  long long zu_main_blocks = 0;  // displacement-form z-pass grid
  int nzub = 0;
  State *st = nullptr;
  State *st_host = nullptr;
  double *hist = nullptr;
  int hist_cap = 0;
  int last_iters = -1;
  int tabS = 0, off[3] = {0, 0, 0};
  int timing_kernel = -1;
  std::vector<hipEvent_t> ev;
  // start / stop events of the timed kernel's next launch (null: untimed);
  // the launch records them itself, so timing adds no packets between
  // kernels
  hipEvent_t tstart = nullptr, tstop = nullptr;
  size_t ev_used = 0;
  double timing_mean = 0.0;
  int timing_count = 0;
  // FP64 warm start of an F32 displacement-form solver: a second solver in
  // F64 that borrows u, the device state and the residual history of this
  // one and runs its first `warm` iterations.
  lsfft_solver_s *twin = nullptr;
  int warm = 0;
  double until = 0.0;  // FP64 twin iterations until the residual is at most this (0 = off)
  int borrowed = 0;  // u, st, st_host and hist belong to another solver
  // Replay of captured iteration chunks: an internal stream (default
  // priority) that waits on `stream`, and the executable graph of GRAPH_CHUNK
  // iterations for the (tol, maxit) it was captured with.
  int use_graphs = 1;
  hipStream_t gstream = nullptr;
  hipEvent_t gevent = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;  // the captured chunk itself (a child node of a group solve's graph)
  double g_tol = -1.0;
  int g_maxit = -1;
  // Schedule: column-tile variant of the y pass (yv) and of the z passes
  // (zv), XCD-aware tile order (bit 0 stencil, bit 1 y pass, bit 2 z pass);
  // the stencil's planes per workgroup are sZ above.
  int yv = 0, zv = 0, xcd = 7;
  // Set while the schedule tuner times iterations: no stopping test.
  int tuning = 0;
  // Eigenstrain (T = C [E - E_*]) of the systems, when any has one: the
  // eigenstress C E_* [B][6][N] (T), its mean [B][6] (FP64) and, in the
  // displacement form, its force div^b (C E_*) at the nodes [B][3][N] (T).
  int eig = 0;
  void *sstar = nullptr, *fstar = nullptr;
  unsigned *counter = nullptr;  // displacement form: stencil workgroup arrivals [B]
  double *smean = nullptr;
  std::vector<double> estar_rms;  // RMS of |E_*|_F of each system
  // FP64 iterative refinement of the F32 displacement form: cycle length in
  // iterations (0 = off).  u holds u_b, du the correction delta that the F32
  // sweeps iterate on; fref = -F_b [B][3][N] (T) and sref [B][6] are the
  // load and the mean-stress offset of those sweeps; lam64, mu64 (and
  // sstar64 with an eigenstrain) the FP64 data of the residual evaluation,
  // rsig its cell stress [B][6][N]; mem_ref the per-system constants with
  // Ebar = 0; rpart the block sums of k_refine_stress (nrb rows per system).
  // Where the FP64 register stencil runs the evaluation instead (mem64 set:
  // Member<double>[B] of the loading, fstar64 the FP64 eigenstress force),
  // rsig and rpart are not allocated.
  int refine = 0;
  double *du = nullptr, *sref = nullptr, *lam64 = nullptr, *mu64 = nullptr, *sstar64 = nullptr, *rpart = nullptr;
  double *rsig = nullptr, *fstar64 = nullptr;
  void *fref = nullptr, *mem_ref = nullptr, *mem64 = nullptr;
  int nrb = 0;
};

namespace lsfft_host {

// The transform lengths the kernels are instantiated for: 2^a or 3 * 2^a.
// Grid lengths of the 3D solver and bar lengths of the 1D solver: even
// 2^a 3^b in [4, 512].
inline bool supported_len(int n) {
  if (n < 4 || n > 512 || (n & 1)) return false;
  int m = n;
  while (m % 2 == 0) m /= 2;
  while (m % 3 == 0) m /= 3;
  return m == 1;
}

// ------------------------------------------------------------------ tables
// exp(-2 pi i m / n) and friends, from long double with exact values at
// multiples of a quarter turn.
inline void cis_exact(long long num, long long den, long double &c, long double &s) {
  // angle 2 pi num / den
  long long q = ((num % den) + den) % den;
  if ((4 * q) % den == 0) {
    const int k = (int)((4 * q) / den) % 4;
    const long double cc[4] = {1.0L, 0.0L, -1.0L, 0.0L};
    const long double ss[4] = {0.0L, 1.0L, 0.0L, -1.0L};
    c = cc[k];
    s = ss[k];
    return;
  }
  const long double a = 2.0L * 3.14159265358979323846264338327950288L * (long double)q / (long double)den;
  c = cosl(a);
  s = sinl(a);
}

template <typename T> inline std::vector<cplx<T>> twiddles(int n) {
  std::vector<cplx<T>> w(n);
  for (int m = 0; m < n; ++m) {
    long double c, s;
    cis_exact(-m, n, c, s);
    w[m] = cplx<T>{(T)c, (T)s};
  }
  return w;
}

// Workgroup counts and tile widths of the passes (no kernels referenced).
template <typename T> struct Tiles {
  static int xgrid(int L, long long rows) {
    int tpc = 1;
    switch (L) {
#define XG(Lv) \
  case Lv:     \
    tpc = Lv / ex_of(Lv); \
    break;
      LSFFT_X_LENGTHS(XG)
#undef XG
      default:
        return 0;
    }
    const int P = lsfft::lines_per_wg(tpc, XWG);
    return (int)((rows + P - 1) / P);
  }
  // columns per y-pass workgroup of tile variant v
  static int ycols(int n, int v) {
    switch (n) {
#define YC(Nv) \
  case Nv:     \
    return v ? palt<T>(Nv, ey_of(Nv), pcols<T>(Nv, ey_of(Nv))) : pcols<T>(Nv, ey_of(Nv));
      LSFFT_YZ_LENGTHS(YC)
#undef YC
      default:
        return 0;
    }
  }
  static int zucols(int n, int v) {
    switch (n) {
#define ZUC(Nv) \
  case Nv:      \
    return v ? palt<T>(Nv, ezu_of<T>(Nv), pcols_zu<T>(Nv, ezu_of<T>(Nv))) : pcols_zu<T>(Nv, ezu_of<T>(Nv));
      LSFFT_YZ_LENGTHS(ZUC)
#undef ZUC
      default:
        return 0;
    }
  }
  static int zcols(int n, int v) {
    switch (n) {
#define ZC(Nv) \
  case Nv:     \
    return v ? palt<T>(Nv, ez_of(Nv), pcols_z<T>(Nv, ez_of(Nv))) : pcols_z<T>(Nv, ez_of(Nv));
      LSFFT_YZ_LENGTHS(ZC)
#undef ZC
      default:
        return 0;
    }
  }
};

// Launches of the pass kernels for the current grid and schedule of a
// solver; hipErrorInvalidValue for a length without an instantiation.
template <typename T> struct Launch : Tiles<T> {
  static hipError_t xpass(lsfft_solver s, const lsfft::XArgs<T> &a, int grid);
  template <bool FWD> static hipError_t ypass(lsfft_solver s, const lsfft::YArgs<T> &a, int grid);
  static hipError_t zpass(lsfft_solver s, const lsfft::ZArgs<T> &a, int grid);
  static hipError_t uxpass(lsfft_solver s, const lsfft::UArgs<T> &a, int grid);
  template <int SCH> static hipError_t stencil_s(lsfft_solver s, const lsfft::SArgs<T> &a, int grid);
  static hipError_t stencil(lsfft_solver s, const lsfft::SArgs<T> &a, int grid);
  template <int SCH> static hipError_t zpass_u_s(lsfft_solver s, const lsfft::ZArgs<T> &a, int grid);
  static hipError_t zpass_u(lsfft_solver s, const lsfft::ZArgs<T> &a, int grid);
  // The kernel instantiations (template arguments) one iteration launches,
  // in launch order, for the solver's lengths, form, scheme and schedule.
  static std::string describe(lsfft_solver s);
};

}  // namespace lsfft_host
