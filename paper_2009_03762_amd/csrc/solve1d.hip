// The 1D algorithms of Sec. 3 on the GPU: the GFP+FDD fixed point on nodal
// (TD, Sec. 3.1) or cell-centred (PCD, Sec. 3.2) samples, and the DGO
// iteration (Sec. 3.3, polarisation form).  Many independent periodic bars of
// one length are solved by one launch: a workgroup per bar keeps the bar's
// fields in registers and iterates to its own stopping test, with no host
// round trip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <mutex>
#include <vector>

#include "solver.hpp"

namespace lsfft {

template <typename T> struct Bar1dArgs {
  const T *C;              // [bar][n] stiffness samples
  const double *CH;        // [bar] reference stiffness C_H
  const double *Ebar;      // [bar] macroscopic strain
  const cplx<double> *qa;  // [n] gradient symbol per frequency (standard FFT order)
  const cplx<double> *qb;  // [n] divergence symbol
  const cplx<T> *ph;       // [n] PCD phase exp(-i pi kappa / n), or null (TD)
  const double *dgo;       // [n] DGO image factor c_p(kappa), or null (GFP)
  const cplx<T> *tw;       // [n] exp(-2 pi i m / n)
  T *E, *S;                // [bar][n] strain and stress out
  int *iters;
  double *res;
  int *status;
  double tol;
  int maxit;
  // Allocation-free entry point: stiffness read as FP64 (Cd instead of C),
  // strain and stress written as FP64 (Ed, Sd instead of E, S; either may be
  // null), per-bar outputs may be null, and each bar checks its own data
  // (check = 1): C and C_H positive and finite, Ebar finite (nonzero for the
  // DGO); a bar that fails gets status LSFFT_EINVAL and no other output.
  const double *Cd = nullptr;
  double *Ed = nullptr, *Sd = nullptr;
  int check = 0;
};

template <typename T> __device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return cplx<T>{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// Deterministic sum over the workgroup (thread order), broadcast to all.
template <int WG> __device__ __forceinline__ double bar_sum(double v, double *red) {
  __syncthreads();
  red[threadIdx.x] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < WG; ++i) s += red[i];
    red[WG] = s;
  }
  __syncthreads();
  return red[WG];
}

// One bar per workgroup, N / E threads; thread t owns samples and
// frequencies t + TPC e.  GFP (Sec. 3.1 / 3.2, the 1D form of eq. (17)):
//   E~ = F^+ (u^ q^a);  T = C (Ebar + E~);  T^ = F^- T;
//   r = |T^ q^b| / |T^(0)|, stop if r <= tol or k = maxit;
//   u^ += G T^ q^b,  G = -1 / (C_H q^a q^b) (0 where q^a q^b = 0).
// DGO (Sec. 3.3): tau = (C - C_H) E;  E' = Ebar + F^+ (Gamma^c F^- tau),
//   Gamma^c = -c_p / C_H;  r = |E' - E| / (sqrt(n) |Ebar|), stop if r <= tol
//   or k = maxit.
template <typename T, int N, int E>
__global__ __launch_bounds__(N / E) void k_bar_1d(Bar1dArgs<T> a) {
  constexpr int TPC = N / E;
  __shared__ cplx<T> twl_[N];
  __shared__ cplx<T> lds[2 * N];
  __shared__ double red[TPC + 1];
  const int bar = blockIdx.x;
  const int t = threadIdx.x;
  const double CH = a.CH[bar], Eb = a.Ebar[bar];
  T c[E];
  cplx<T> ph[E], G[E], qa[E], qb[E];
  T gd[E];
  if (a.check) {
    double bad = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const double v = a.Cd[(long long)bar * N + t + TPC * e];
      if (!(v > 0.0) || !(v < __builtin_huge_val())) bad = 1.0;
    }
    if (t == 0 && (!(CH > 0.0) || !(CH < __builtin_huge_val()) || !(fabs(Eb) < __builtin_huge_val()) ||
                   (a.dgo && Eb == 0.0)))
      bad = 1.0;
    if (bar_sum<TPC>(bad, red) != 0.0) {
      if (t == 0) {
        if (a.iters) a.iters[bar] = 0;
        if (a.res) a.res[bar] = __builtin_nan("");
        if (a.status) a.status[bar] = -1;  // LSFFT_EINVAL
      }
      return;
    }
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int j = t + TPC * e;
    c[e] = a.Cd ? (T)a.Cd[(long long)bar * N + j] : a.C[(long long)bar * N + j];
    ph[e] = a.ph ? a.ph[j] : cplx<T>{T(1), T(0)};
    qa[e] = cplx<T>{(T)a.qa[j].x, (T)a.qa[j].y};
    qb[e] = cplx<T>{(T)a.qb[j].x, (T)a.qb[j].y};
    // G = -1 / (C_H q^a q^b), formed in FP64
    const double pr = a.qa[j].x * a.qb[j].x - a.qa[j].y * a.qb[j].y;
    const double pi = a.qa[j].x * a.qb[j].y + a.qa[j].y * a.qb[j].x;
    const double d = pr * pr + pi * pi;
    G[e] = (d == 0.0) ? cplx<T>{T(0), T(0)} : cplx<T>{(T)(-pr / (CH * d)), (T)(pi / (CH * d))};
    gd[e] = a.dgo ? (T)(-a.dgo[j] / CH) : T(0);
  }
  int buf = 0;
  const cplx<T> *twl = stage_twiddles(twl_, a.tw);
  const T inv_n = T(1) / T(N);
  int k = 0;
  double r = __builtin_huge_val();  // a DGO solve with maxit = 0 has no residual
  int status = 1;
  cplx<T> v[E];
  T Ecur[E], Scur[E];
  if (!a.dgo) {
    cplx<T> u[E];
#pragma unroll
    for (int e = 0; e < E; ++e) u[e] = cplx<T>{T(0), T(0)};
    for (;;) {
      // E~ = F^+ (u^ q^a): the PCD phase exp(+i pi kappa / n) first
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = cmul(cmul(u[e], qa[e]), cplx<T>{ph[e].x, -ph[e].y});
      fft_pencil<T, N, E, false>(v, t, lds, 1, twl, 1, buf);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        Ecur[e] = (T)Eb + v[e].x * inv_n;
        Scur[e] = c[e] * Ecur[e];
        v[e] = cplx<T>{Scur[e], T(0)};
      }
      fft_pencil<T, N, E, true>(v, t, lds, 1, twl, 1, buf);
      double num = 0.0, den = 0.0;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        v[e] = cmul(v[e], ph[e]);
        const cplx<T> w = cmul(v[e], qb[e]);
        num += (double)w.x * w.x + (double)w.y * w.y;
        if (t + TPC * e == 0) den = (double)v[e].x * v[e].x + (double)v[e].y * v[e].y;
      }
      num = bar_sum<TPC>(num, red);
      den = bar_sum<TPC>(den, red);
      r = (num == 0.0) ? 0.0 : (den > 0.0 ? sqrt(num / den) : __builtin_huge_val());
      if (r <= a.tol) {
        status = 0;
        break;
      }
      if (k == a.maxit) break;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const cplx<T> du = cmul(G[e], cmul(v[e], qb[e]));
        u[e].x += du.x;
        u[e].y += du.y;
      }
      ++k;
    }
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) Ecur[e] = (T)Eb;
    const double scale = 1.0 / (sqrt((double)N) * fabs(Eb));
    while (k < a.maxit) {
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = cplx<T>{(c[e] - (T)CH) * Ecur[e], T(0)};
      fft_pencil<T, N, E, true>(v, t, lds, 1, twl, 1, buf);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const cplx<T> w = cmul(v[e], ph[e]);  // F^- of the PCD samples
        v[e] = cmul(cplx<T>{gd[e] * w.x, gd[e] * w.y}, cplx<T>{ph[e].x, -ph[e].y});
      }
      fft_pencil<T, N, E, false>(v, t, lds, 1, twl, 1, buf);
      double dd = 0.0;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const T en = (T)Eb + v[e].x * inv_n;
        const double d = (double)en - (double)Ecur[e];
        dd += d * d;
        Ecur[e] = en;
      }
      dd = bar_sum<TPC>(dd, red);
      r = sqrt(dd) * scale;
      ++k;
      if (r <= a.tol) {
        status = 0;
        break;
      }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) Scur[e] = c[e] * Ecur[e];
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const long long o = (long long)bar * N + t + TPC * e;
    if (a.E) a.E[o] = Ecur[e];
    if (a.S) a.S[o] = Scur[e];
    if (a.Ed) a.Ed[o] = (double)Ecur[e];
    if (a.Sd) a.Sd[o] = (double)Scur[e];
  }
  if (t == 0) {
    if (a.iters) a.iters[bar] = k;
    if (a.res) a.res[bar] = r;
    if (a.status) a.status[bar] = status;
  }
}

// ---------------------------------------------------------------- tables on the device
// The per-frequency tables of a 1D call computed on the device, for the
// allocation-free entry point (the host path forms the same tables in long
// double): e^{i 2 pi num / den} with exact values at quarter turns, the
// symbols of eqs. (12)-(14), the PCD phase, the DGO image factor and the
// transform twiddles.
__device__ inline void cis_exact_dev(long long num, long long den, double &c, double &s) {
  const long long q = ((num % den) + den) % den;
  if ((4 * q) % den == 0) {
    const int k = (int)((4 * q) / den) % 4;
    c = (k == 0) ? 1.0 : (k == 2 ? -1.0 : 0.0);
    s = (k == 1) ? 1.0 : (k == 3 ? -1.0 : 0.0);
    return;
  }
  sincospi(2.0 * (double)q / (double)den, &s, &c);
}

struct BarTables {
  int n, scheme, pcd, dgo, M, p;
  double h;
  cplx<double> *qa, *qb;
  void *ph, *tw;  // cplx<T>
  double *gd;
};

template <typename T> __global__ void k_bar_tables(BarTables b) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= b.n) return;
  const int n = b.n;
  const double h = b.h;
  const int kappa = (2 * j < n) ? j : j - n;  // Nyquist index read as -n/2
  double c, s, ch, sh;
  cis_exact_dev(kappa, n, c, s);
  cis_exact_dev(kappa, 2LL * n, ch, sh);
  const cplx<double> fd{(c - 1.0) / h, s / h};
  cplx<double> qa, qb;
  switch (b.scheme) {
    case LSFFT_1D_F:
      qa = {0.0, 2.0 * M_PI * kappa / (n * h)};
      qb = {0.0, -qa.y};
      break;
    case LSFFT_1D_CD:
      qa = {0.0, s / h};
      qb = {0.0, -qa.y};
      break;
    case LSFFT_1D_FD_HC:
      qa = fd;
      qb = {0.0, 2.0 * sh / h};
      break;
    default:  // LSFFT_1D_FD (and the DGO's unused symbols) with its conjugate
      qa = fd;
      qb = {fd.x, -fd.y};
      break;
  }
  b.qa[j] = qa;
  b.qb[j] = qb;
  double pc, ps;
  cis_exact_dev(-kappa, 2LL * n, pc, ps);  // exp(-i pi kappa / n)
  reinterpret_cast<cplx<T> *>(b.ph)[j] = cplx<T>{(T)pc, (T)ps};
  double tc, ts;
  cis_exact_dev(-j, n, tc, ts);  // exp(-2 pi i j / n)
  reinterpret_cast<cplx<T> *>(b.tw)[j] = cplx<T>{(T)tc, (T)ts};
  double g = 0.0;
  if (b.dgo && kappa != 0) {
    const int hi = (kappa == -n / 2) ? b.M + 1 : b.M;
    for (int nu = -b.M; nu <= hi; ++nu) {
      const long long m = (long long)kappa + (long long)nu * n;  // never 0 for kappa != 0
      double cn, sn;
      cis_exact_dev(m, 2LL * n, cn, sn);  // sin(pi m / n) with exact zeros
      const double w = sn / (M_PI * (double)m / (double)n);
      g += (b.p == 2) ? w * w : w;
    }
  }
  b.gd[j] = g;
}

// Scratch of the allocation-free entry point: one call's tables, at most
// 512 frequencies (qa, qb and the phase and twiddles as complex FP64 at most,
// the DGO factor as FP64).  Every GPU the library runs on holds one copy for
// the life of the process; in host code the name is only a stand-in for the
// device symbol, whose address each device's copy has (see
// noalloc_scratch below).
constexpr int NOALLOC_MAX_N = 512;
constexpr size_t NOALLOC_QA = 0, NOALLOC_QB = NOALLOC_QA + NOALLOC_MAX_N * 16, NOALLOC_PH = NOALLOC_QB + NOALLOC_MAX_N * 16,
                 NOALLOC_TW = NOALLOC_PH + NOALLOC_MAX_N * 16, NOALLOC_GD = NOALLOC_TW + NOALLOC_MAX_N * 16,
                 NOALLOC_BYTES = NOALLOC_GD + NOALLOC_MAX_N * 8;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

}  // namespace lsfft

namespace {

using lsfft_host::cis_exact;

#define BAR_CHECK(call)                                                                   \
  do {                                                                                    \
    hipError_t _e = (call);                                                               \
    if (_e != hipSuccess) {                                                               \
      fprintf(stderr, "lsfft: %s failed: %s\n", #call, hipGetErrorString(_e));            \
      return LSFFT_EDEVICE;                                                               \
    }                                                                                     \
  } while (0)

// Points per thread: the y-pass choice (radix-8 passes; 12 for lengths with
// a factor 3 where it divides, else the smallest multiple of 6 that does
// and keeps a bar within 64 threads).
constexpr int bar_e(int n) {
  return (n % 3 == 0) ? (n < 12 ? n : (n % 12 == 0 ? 12 : lsfft_host::e_mult3(n, 64))) : (n < 8 ? n : 8);
}

template <typename T>
hipError_t launch_bars(int n, int count, const lsfft::Bar1dArgs<T> &a, hipStream_t st) {
  switch (n) {
#define BCASE(Nv)                                                                                      \
  case Nv:                                                                                           \
    hipLaunchKernelGGL((lsfft::k_bar_1d<T, Nv, bar_e(Nv)>), dim3(count), dim3(Nv / bar_e(Nv)), 0, st, a); \
    return hipGetLastError();
    LSFFT_YZ_LENGTHS(BCASE)
#undef BCASE
    default:
      return hipErrorInvalidValue;
  }
}

// The 1D symbols of eqs. (12)-(14) at the centred index kappa of an n-point
// grid with spacing h (e^{i theta}, theta = 2 pi kappa / n):
//   F  = i 2 pi kappa / (n h),   FD = (e^{i theta} - 1) / h,
//   CD = i sin(theta) / h,       hC = 2 i sin(theta / 2) / h.
void symbol_1d(int scheme, int kappa, int n, double h, lsfft::cplx<double> &qa, lsfft::cplx<double> &qb) {
  long double c, s, ch, sh;
  cis_exact(kappa, n, c, s);
  cis_exact(kappa, 2LL * n, ch, sh);
  const long double PI = 3.14159265358979323846264338327950288L;
  lsfft::cplx<double> fd{(double)((c - 1.0L) / h), (double)(s / h)};
  switch (scheme) {
    case LSFFT_1D_F:
      qa = {0.0, (double)(2.0L * PI * kappa / (n * (long double)h))};
      qb = {qa.x, -qa.y};
      break;
    case LSFFT_1D_CD:
      qa = {0.0, (double)(s / h)};
      qb = {qa.x, -qa.y};
      break;
    case LSFFT_1D_FD_HC:
      qa = fd;
      qb = {0.0, (double)(2.0L * sh / h)};
      break;
    default:  // LSFFT_1D_FD with its conjugate
      qa = fd;
      qb = {fd.x, -fd.y};
      break;
  }
}

// sum over images nu of sinc^p(pi (kappa + nu n) / n): nu in [-M, M], and
// [-M, M+1] at the Nyquist index; 0 at kappa = 0.
double dgo_factor(int kappa, int n, int M, int p) {
  if (kappa == 0) return 0.0;
  const int hi = (kappa == -n / 2) ? M + 1 : M;
  const long double PI = 3.14159265358979323846264338327950288L;
  long double sum = 0.0L;
  for (int nu = -M; nu <= hi; ++nu) {
    const long long m = (long long)kappa + (long long)nu * n;  // never 0 for kappa != 0
    const long double x = PI * (long double)m / (long double)n;
    long double sn, cn;
    cis_exact(m, 2LL * n, cn, sn);  // sin(pi m / n) with exact zeros
    const long double w = sn / x;
    sum += (p == 2) ? w * w : w;
  }
  return (double)sum;
}

template <typename T>
lsfft_status solve_bars(const lsfft_config_1d *cfg, int count, const double *C, const double *CH,
                        const double *Ebar, double tol, int maxit, double *E_out, double *S_out, int32_t *iters,
                        double *residual, int32_t *status) {
  const int n = cfg->n;
  const double h = cfg->h > 0.0 ? cfg->h : 1.0;
  const bool dgo = cfg->scheme == LSFFT_1D_DGO;
  const bool pcd = cfg->disc == LSFFT_PCD;
  hipStream_t st = (hipStream_t)cfg->stream;
  std::vector<lsfft::cplx<double>> qa(n), qb(n);
  std::vector<lsfft::cplx<T>> ph(n);
  std::vector<double> gd(n);
  for (int j = 0; j < n; ++j) {
    const int kappa = (2 * j < n) ? j : j - n;  // Nyquist index read as -n/2
    symbol_1d(cfg->scheme, kappa, n, h, qa[j], qb[j]);
    long double c, s;
    cis_exact(-kappa, 2LL * n, c, s);  // exp(-i pi kappa / n)
    ph[j] = lsfft::cplx<T>{(T)c, (T)s};
    gd[j] = dgo ? dgo_factor(kappa, n, cfg->dgo_images, cfg->dgo_weight_power) : 0.0;
  }
  const auto tw = lsfft_host::twiddles<T>(n);
  std::vector<T> Ct((size_t)count * n);
  for (size_t i = 0; i < Ct.size(); ++i) Ct[i] = (T)C[i];
  // one device block for everything, carved below
  const size_t nb = (size_t)count * n;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  };
  const size_t oC = take(nb * sizeof(T)), oCH = take(count * sizeof(double)), oEb = take(count * sizeof(double));
  const size_t oqa = take(n * sizeof(lsfft::cplx<double>)), oqb = take(n * sizeof(lsfft::cplx<double>));
  const size_t oph = take(n * sizeof(lsfft::cplx<T>)), ogd = take(n * sizeof(double));
  const size_t otw = take(n * sizeof(lsfft::cplx<T>)), oE = take(nb * sizeof(T)), oS = take(nb * sizeof(T));
  const size_t oit = take(count * sizeof(int)), ores = take(count * sizeof(double)), ost = take(count * sizeof(int));
  char *dev = nullptr;
  BAR_CHECK(hipMalloc(&dev, off));
  auto done = [&](lsfft_status s) {
    (void)hipFree(dev);
    return s;
  };
  auto up = [&](size_t o, const void *src, size_t bytes) {
    return hipMemcpyAsync(dev + o, src, bytes, hipMemcpyHostToDevice, st);
  };
  if (up(oC, Ct.data(), nb * sizeof(T)) != hipSuccess || up(oCH, CH, count * sizeof(double)) != hipSuccess ||
      up(oEb, Ebar, count * sizeof(double)) != hipSuccess ||
      up(oqa, qa.data(), n * sizeof(lsfft::cplx<double>)) != hipSuccess ||
      up(oqb, qb.data(), n * sizeof(lsfft::cplx<double>)) != hipSuccess ||
      up(oph, ph.data(), n * sizeof(lsfft::cplx<T>)) != hipSuccess ||
      up(ogd, gd.data(), n * sizeof(double)) != hipSuccess ||
      up(otw, tw.data(), n * sizeof(lsfft::cplx<T>)) != hipSuccess)
    return done(LSFFT_EDEVICE);
  lsfft::Bar1dArgs<T> a;
  a.C = (const T *)(dev + oC);
  a.CH = (const double *)(dev + oCH);
  a.Ebar = (const double *)(dev + oEb);
  a.qa = (const lsfft::cplx<double> *)(dev + oqa);
  a.qb = (const lsfft::cplx<double> *)(dev + oqb);
  a.ph = pcd ? (const lsfft::cplx<T> *)(dev + oph) : nullptr;
  a.dgo = dgo ? (const double *)(dev + ogd) : nullptr;
  a.tw = (const lsfft::cplx<T> *)(dev + otw);
  a.E = (T *)(dev + oE);
  a.S = (T *)(dev + oS);
  a.iters = (int *)(dev + oit);
  a.res = (double *)(dev + ores);
  a.status = (int *)(dev + ost);
  a.tol = tol;
  a.maxit = maxit;
  if (launch_bars<T>(n, count, a, st) != hipSuccess) return done(LSFFT_EDEVICE);
  std::vector<T> Eh(nb), Sh(nb);
  std::vector<int> it(count), sts(count);
  std::vector<double> rs(count);
  if (hipMemcpyAsync(Eh.data(), a.E, nb * sizeof(T), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(Sh.data(), a.S, nb * sizeof(T), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(it.data(), a.iters, count * sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(rs.data(), a.res, count * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(sts.data(), a.status, count * sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return done(LSFFT_EDEVICE);
  int worst = 0;
  for (int b = 0; b < count; ++b) {
    if (iters) iters[b] = it[b];
    if (residual) residual[b] = rs[b];
    if (status) status[b] = sts[b];
    worst = sts[b] > worst ? sts[b] : worst;
  }
  for (size_t i = 0; i < nb; ++i) {
    if (E_out) E_out[i] = (double)Eh[i];
    if (S_out) S_out[i] = (double)Sh[i];
  }
  return done((lsfft_status)worst);
}

}  // namespace

namespace {

// Device address of this device's copy of the scratch array: looked up once
// per device, on the entry point's first call with that device current.
std::mutex g_scratch_mu;
void *g_scratch_ptr[64] = {};

lsfft_status noalloc_scratch(void *&ptr) {
  int dev = -1;
  BAR_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return LSFFT_EDEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    BAR_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(lsfft::scratch)));
    if (!p) return LSFFT_EDEVICE;
    g_scratch_ptr[dev] = p;
  }
  ptr = g_scratch_ptr[dev];
  return LSFFT_OK;
}

template <typename T>
lsfft_status solve_bars_noalloc(const lsfft_config_1d *cfg, int count, const double *C, const double *CH,
                                const double *Ebar, double tol, int maxit, double *E_out, double *S_out,
                                int32_t *iters, double *residual, int32_t *status) {
  void *base = nullptr;
  lsfft_status ss = noalloc_scratch(base);
  if (ss != LSFFT_OK) return ss;
  char *scr = (char *)base;
  const int n = cfg->n;
  const bool dgo = cfg->scheme == LSFFT_1D_DGO;
  hipStream_t st = (hipStream_t)cfg->stream;
  lsfft::BarTables tb;
  tb.n = n;
  tb.scheme = cfg->scheme;
  tb.pcd = cfg->disc == LSFFT_PCD;
  tb.dgo = dgo;
  tb.M = cfg->dgo_images;
  tb.p = cfg->dgo_weight_power;
  tb.h = cfg->h > 0.0 ? cfg->h : 1.0;
  tb.qa = (lsfft::cplx<double> *)(scr + lsfft::NOALLOC_QA);
  tb.qb = (lsfft::cplx<double> *)(scr + lsfft::NOALLOC_QB);
  tb.ph = scr + lsfft::NOALLOC_PH;
  tb.tw = scr + lsfft::NOALLOC_TW;
  tb.gd = (double *)(scr + lsfft::NOALLOC_GD);
  hipLaunchKernelGGL(lsfft::k_bar_tables<T>, dim3((n + 63) / 64), dim3(64), 0, st, tb);
  BAR_CHECK(hipGetLastError());
  lsfft::Bar1dArgs<T> a;
  a.C = nullptr;
  a.Cd = C;
  a.CH = CH;
  a.Ebar = Ebar;
  a.qa = tb.qa;
  a.qb = tb.qb;
  a.ph = tb.pcd ? (const lsfft::cplx<T> *)tb.ph : nullptr;
  a.dgo = dgo ? tb.gd : nullptr;
  a.tw = (const lsfft::cplx<T> *)tb.tw;
  a.E = a.S = nullptr;
  a.Ed = E_out;
  a.Sd = S_out;
  a.iters = iters;
  a.res = residual;
  a.status = status;
  a.tol = tol;
  a.maxit = maxit;
  a.check = 1;
  if (launch_bars<T>(n, count, a, st) != hipSuccess) return LSFFT_EDEVICE;
  return LSFFT_OK;
}

}  // namespace

extern "C" lsfft_status lsfft_solve_1d_noalloc(const lsfft_config_1d *cfg, int32_t count, const double *C_dev,
                                               const double *CH_dev, const double *Ebar_dev, double tol,
                                               int32_t maxit, double *E_dev, double *T_dev, int32_t *iters_dev,
                                               double *residual_dev, int32_t *status_dev) {
  if (!cfg || !C_dev || !CH_dev || !Ebar_dev || !status_dev || count < 1 || count > 65535) return LSFFT_EINVAL;
  if (cfg->n > lsfft::NOALLOC_MAX_N) {
    fprintf(stderr, "lsfft_solve_1d_noalloc: n = %d exceeds the scratch limit of %d samples per bar\n", cfg->n,
            lsfft::NOALLOC_MAX_N);
    return LSFFT_EINVAL;
  }
  if (!lsfft_host::supported_len(cfg->n) || !(cfg->h >= 0.0) || !std::isfinite(cfg->h)) return LSFFT_EINVAL;
  if (cfg->scheme < LSFFT_1D_F || cfg->scheme > LSFFT_1D_DGO) return LSFFT_EINVAL;
  if (cfg->disc != LSFFT_TD && cfg->disc != LSFFT_PCD) return LSFFT_EINVAL;
  if (cfg->prec != LSFFT_F32 && cfg->prec != LSFFT_F64) return LSFFT_EINVAL;
  if (cfg->scheme == LSFFT_1D_DGO) {
    if (cfg->disc != LSFFT_PCD || cfg->dgo_images < 0 || cfg->dgo_images > 64) return LSFFT_EINVAL;
    if (cfg->dgo_weight_power != 1 && cfg->dgo_weight_power != 2) return LSFFT_EINVAL;
  }
  if (!(tol >= 0.0) || !std::isfinite(tol) || maxit < 0 || maxit > 10000000) return LSFFT_EINVAL;
  return cfg->prec == LSFFT_F32 ? solve_bars_noalloc<float>(cfg, count, C_dev, CH_dev, Ebar_dev, tol, maxit, E_dev,
                                                            T_dev, iters_dev, residual_dev, status_dev)
                                : solve_bars_noalloc<double>(cfg, count, C_dev, CH_dev, Ebar_dev, tol, maxit, E_dev,
                                                             T_dev, iters_dev, residual_dev, status_dev);
}

extern "C" lsfft_status lsfft_solve_1d(const lsfft_config_1d *cfg, int32_t count, const double *C, const double *CH,
                                       const double *Ebar, double tol, int32_t maxit, double *E_out, double *S_out,
                                       int32_t *iters, double *residual, int32_t *status) {
  if (!cfg || !C || !CH || !Ebar || count < 1 || count > 65535) return LSFFT_EINVAL;
  if (!lsfft_host::supported_len(cfg->n) || !(cfg->h >= 0.0) || !std::isfinite(cfg->h)) return LSFFT_EINVAL;
  if (cfg->scheme < LSFFT_1D_F || cfg->scheme > LSFFT_1D_DGO) return LSFFT_EINVAL;
  if (cfg->disc != LSFFT_TD && cfg->disc != LSFFT_PCD) return LSFFT_EINVAL;
  if (cfg->prec != LSFFT_F32 && cfg->prec != LSFFT_F64) return LSFFT_EINVAL;
  if (cfg->scheme == LSFFT_1D_DGO) {
    if (cfg->disc != LSFFT_PCD || cfg->dgo_images < 0 || cfg->dgo_images > 64) return LSFFT_EINVAL;
    if (cfg->dgo_weight_power != 1 && cfg->dgo_weight_power != 2) return LSFFT_EINVAL;
  }
  if (!(tol >= 0.0) || !std::isfinite(tol) || maxit < 0 || maxit > 10000000) return LSFFT_EINVAL;
  for (long long i = 0; i < (long long)count * cfg->n; ++i)
    if (!(C[i] > 0.0) || !std::isfinite(C[i])) return LSFFT_EINVAL;
  for (int b = 0; b < count; ++b) {
    if (!(CH[b] > 0.0) || !std::isfinite(CH[b]) || !std::isfinite(Ebar[b])) return LSFFT_EINVAL;
    if (cfg->scheme == LSFFT_1D_DGO && Ebar[b] == 0.0) return LSFFT_EINVAL;
  }
  return cfg->prec == LSFFT_F32
             ? solve_bars<float>(cfg, count, C, CH, Ebar, tol, maxit, E_out, S_out, iters, residual, status)
             : solve_bars<double>(cfg, count, C, CH, Ebar, tol, maxit, E_out, S_out, iters, residual, status);
}
