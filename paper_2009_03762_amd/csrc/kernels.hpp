// Kernels of one fixed-point iteration (strain form of the 3D TD / PCD
// algorithms of Sec. 5.2 / 5.4 and of the DGO algorithm of Sec. 5.4):
//
//   k_xpass  x-lines: inverse real transform of the strain increment,
//            strain update, Hooke (Sec. 5.1), forward real transform of the
//            stress; FP64 block sums of <sigma> (and of |eps_new - eps_old|^2).
//   k_ypass  y-pencils: batched complex transform (forward or inverse).
//   k_zpass  z-pencils of all six components: forward transform, Green step
//            (green.hpp), FP64 block sums of the equilibrium residual,
//            inverse transform.
//   k_reduce single workgroup: fixed-order FP64 reduction of the block sums,
//            convergence / divergence decision, device-side stop flag.
//
// Spectrum storage: for component c, kx in [0, n1/2) in
//   main[c][k3][k2][kx]   (rows of n1/2 complex, aligned)
// and the x-Nyquist plane kx = n1/2 in
//   nyq[c][k3][k2].
// Every kernel returns at once when the stop flag is set, so iterations may
// be enqueued ahead of the host's convergence check.
#pragma once
#include "fft.hpp"
#include "green.hpp"

#ifndef LSFFT_X_PRELOAD
#define LSFFT_X_PRELOAD 1
#endif

namespace lsfft {

struct Dims {
  int n1, n2, n3, L;
  long long N, rows, comp_main, comp_nyq;
};

struct State {
  int done;
  int status;
  int iters;
  int k;        // index of the next iteration to test (advanced by k_reduce)
  double r0;    // first value of the divergence test's quantity (see reduce_decide)
  double r;
  double sig_mean[6];
};

enum { XMODE_INIT = 0, XMODE_UPDATE = 1, XMODE_DGO = 2, XMODE_EXTERNAL = 3 };

// A solver holds a batch of systems on one grid (the load cases of a cell, or
// several cells of equal size); every kernel takes its system from
// blockIdx.y.  Per-system constants live in device memory:
template <typename T> struct Member {
  double Eb[6];      // macroscopic strain, Voigt tensor components
  double hE[3][3];   // h_j Ebar_ij: the macroscopic part of an edge difference
  T lam0, mu0;       // reference medium C0
  T c1, c2, beta;    // 1/mu0, (lam0+mu0)/(mu0 (lam0+2 mu0)), (lam0+mu0)/(lam0+2 mu0)
};
// Element strides between consecutive systems of the batch.
struct Strides {
  long long field;   // one real N-voxel field (eps has 6, u has 3 of them)
  long long spec;    // complex values of the main spectrum (all components)
  long long nyq;     // complex values of the x-Nyquist plane (all components)
  long long part;    // doubles of the block partial sums
};

template <typename T> struct XArgs {
  Dims d;
  T *eps;
  const T *eps_in;   // XMODE_EXTERNAL: strain to transform (not updated)
  const T *lam;
  const T *mu;
  cplx<T> *spec;
  cplx<T> *nyq;
  const cplx<T> *tw;  // exp(-2 pi i m / n1), m = 0..n1-1
  const Member<T> *mem;
  Strides bs;
  double *partial;    // [system][gridDim.x][8]
  const State *st;    // [system]
  const T *sstar;     // eigenstress C E_* [system][6][N] (T = C [E - E_*]), or null
  int mode;
  int polarisation;   // transform (C - C0) : eps instead of C : eps
};

template <typename T> __device__ __forceinline__ void ld2(const T *p, T &a, T &b);
template <> __device__ __forceinline__ void ld2<float>(const float *p, float &a, float &b) {
  float2 v = *reinterpret_cast<const float2 *>(p);
  a = v.x;
  b = v.y;
}
template <> __device__ __forceinline__ void ld2<double>(const double *p, double &a, double &b) {
  double2 v = *reinterpret_cast<const double2 *>(p);
  a = v.x;
  b = v.y;
}
template <typename T> __device__ __forceinline__ void st2(T *p, T a, T b);
template <> __device__ __forceinline__ void st2<float>(float *p, float a, float b) {
  *reinterpret_cast<float2 *>(p) = make_float2(a, b);
}
template <> __device__ __forceinline__ void st2<double>(double *p, double a, double b) {
  *reinterpret_cast<double2 *>(p) = make_double2(a, b);
}

// Streaming (non-temporal) loads and stores of two-element values, for the
// contiguous row accesses of the x-direction kernels, which touch each value
// of u and of the spectrum once per iteration.  The y- and z-passes keep
// cached accesses: their column accesses share cache lines between
// workgroups.
template <typename T> __device__ __forceinline__ void ld2_nt(const T *p, T &a, T &b) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2 *>(p));
  a = v.x;
  b = v.y;
}
template <typename T> __device__ __forceinline__ void st2_nt(T *p, T a, T b) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  v2 v;
  v.x = a;
  v.y = b;
  __builtin_nontemporal_store(v, reinterpret_cast<v2 *>(p));
}
template <typename T> __device__ __forceinline__ cplx<T> ldc_nt(const cplx<T> *p) {
  cplx<T> v;
  ld2_nt(&p->x, v.x, v.y);
  return v;
}
template <typename T> __device__ __forceinline__ void stc_nt(cplx<T> *p, cplx<T> v) { st2_nt(&p->x, v.x, v.y); }

// Buffer resources over a field of `count` elements (raw: offsets in bytes,
// bounds-checked against the field's size, which stays below 4 GiB for every
// supported grid) and loads through them: the load adds a scalar byte offset
// to the per-thread one, so a plane-invariant per-thread offset needs no
// vector address arithmetic.
template <typename E>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_of(const E *p, long long count) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<E *>(p), 0, (int)(unsigned)(count * (long long)sizeof(E)),
                                           0x00020000);
}
__device__ __forceinline__ double load_f64(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
template <typename T> __device__ __forceinline__ T load_t(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}

// Complex values through a buffer resource (8 bytes in FP32, 16 in FP64).
template <typename T> __device__ __forceinline__ cplx<T> load_c(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  if constexpr (sizeof(T) == 4)
    return __builtin_bit_cast(cplx<T>, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
  else
    return __builtin_bit_cast(cplx<T>, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0));
}
template <typename T>
__device__ __forceinline__ void store_c(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, cplx<T> v) {
  if constexpr (sizeof(T) == 4) {
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, (int)voff, (int)soff, 0);
  } else {
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, v), r, (int)voff, (int)soff, 0);
  }
}

template <typename T> __device__ __forceinline__ T shfl(T v, int lane) { return __shfl(v, lane, 64); }

// Partner value X[(L - k) mod L] for every point k = t + TPC e held by this
// thread.  The partner of thread t is thread (TPC - t) mod TPC of the same
// pencil (same wavefront); it holds the partner point in slot E-1-e, or in
// slot (E-e) mod E when t = 0 (the pencil's own thread).
template <typename T, int E, int TPC>
__device__ __forceinline__ void partner(const cplx<T> (&v)[E], cplx<T> (&pv)[E], int t, int lane) {
  const int plane = lane - t + ((TPC - t) % TPC);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    cplx<T> send = v[E - 1 - e];
    cplx<T> got;
    if constexpr (TPC > 1) {
      got.x = shfl(send.x, plane);
      got.y = shfl(send.y, plane);
    } else {
      got = send;
    }
    pv[e] = (t == 0) ? v[(E - e) % E] : got;
  }
}

// The line transforms below run on lines that lie in one wavefront with
// scratch of their own, line_scratch<L>() points per line (every caller
// asserts 64 % TPC == 0), so their radix exchanges are ordered at wavefront
// scope.
//
// Inverse real transform of one x-line.  In: v[e] = X[k], k = t + TPC e,
// k in [0, L), and xn = X[L] (meaningful in thread t = 0).  Out: v[e] =
// (x[2m], x[2m+1]) for m = t + TPC e: the unnormalised inverse real DFT of
// length 2L, via one complex inverse transform of length L.
template <typename T, int L, int E>
__device__ __forceinline__ void c2r_line(cplx<T> (&v)[E], cplx<T> xn, int t, int lane, cplx<T> *lds,
                                         const cplx<T> *__restrict__ tw, int &buf) {
  constexpr int TPC = L / E;
  cplx<T> pv[E];
  partner<T, E, TPC>(v, pv, t, lane);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = t + TPC * e;
    if (k == 0) {
      const T a = v[e].x, b = xn.x;  // X[0] and X[L] are real for a real line
      v[e] = cplx<T>{a + b, a - b};
    } else {
      const cplx<T> xp = conjg(pv[e]);
      const cplx<T> w = conjg(tw[k]);  // exp(+2 pi i k / (2L))
      v[e] = (v[e] + xp) + mul_i(w * (v[e] - xp));
    }
  }
  fft_pencil<T, L, E, false, true, line_pad<L>()>(v, t, lds, 1, tw, 2, buf);
}

// Forward real transform of one x-line.  In: v[e] = (x[2m], x[2m+1]).
// Out: v[e] = X[k] for k = t + TPC e in [0, L), and the return value X[L]
// (in thread t = 0); with HALF false, 2 X[k] and 2 X[L] (four fewer
// multiplications per point, for callers that fold the factor into a later
// scale).
template <typename T, int L, int E, bool HALF = true>
__device__ __forceinline__ cplx<T> r2c_line(cplx<T> (&v)[E], int t, int lane, cplx<T> *lds,
                                            const cplx<T> *__restrict__ tw, int &buf) {
  constexpr int TPC = L / E;
  fft_pencil<T, L, E, true, true, line_pad<L>()>(v, t, lds, 1, tw, 2, buf);
  cplx<T> pv[E];
  partner<T, E, TPC>(v, pv, t, lane);
  cplx<T> xn{T(0), T(0)};
  constexpr T two = HALF ? T(1) : T(2);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = t + TPC * e;
    const cplx<T> z = v[e];
    if (k == 0) {
      v[e] = cplx<T>{two * (z.x + z.y), T(0)};
      xn = cplx<T>{two * (z.x - z.y), T(0)};
    } else {
      const cplx<T> zp = conjg(pv[e]);
      const cplx<T> fe = HALF ? T(0.5) * (z + zp) : z + zp;
      const cplx<T> d = HALF ? T(0.5) * (z - zp) : z - zp;
      const cplx<T> fo = cplx<T>{d.y, -d.x};  // (z - zp) / (2i), times 2 unless HALF
      v[e] = fe + tw[k] * fo;
    }
  }
  return xn;
}

template <int WG> __device__ __forceinline__ void block_sum(double *vals, int nv, double *red) {
  // fixed-order reduction: per-wavefront butterfly, then wavefronts in order.
  // A workgroup that is not whole wavefronts (some y and z tiles of lengths
  // with a factor 9) has lanes past its last thread that were never
  // launched: their values are discarded.  Lane 0 reads each lane m once, at
  // the step of m's highest set bit, when m holds the sum over lanes above
  // it only, so for a partial wavefront every value it discards is empty.
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int NW = (WG + 63) / 64;
  const int live = (WG % 64 != 0 && wave == NW - 1) ? WG - 64 * (NW - 1) : 64;
  for (int i = 0; i < nv; ++i) {
    double x = vals[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double y = __shfl_xor(x, o, 64);
      if constexpr (WG % 64 == 0)
        x += y;
      else
        x += ((lane ^ o) < live) ? y : 0.0;
    }
    if (lane == 0) red[wave * 8 + i] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 0; i < nv; ++i) {
      double s = 0.0;
      for (int w = 0; w < NW; ++w) s += red[w * 8 + i];
      vals[i] = s;
    }
  }
}

// Map a physical workgroup id to a logical tile so that each XCD (workgroups
// are dealt round-robin to the 8 XCDs) walks a contiguous range of tiles:
// neighbouring tiles then share that XCD's L2.
__device__ __forceinline__ long long xcd_tile(long long b, long long nblocks) {
  const long long per = nblocks / 8;
  if (b >= per * 8) return b;  // remainder keeps its own order
  return (b % 8) * per + b / 8;
}
// The tile of workgroup b: XCD-aware when `on`, else the launch order.
__device__ __forceinline__ long long tile_of(long long b, long long nblocks, int on) {
  return on ? xcd_tile(b, nblocks) : b;
}

// One workgroup = P x-lines of L complex points (TPC = L/E threads each).
// All global loads of the workgroup (six spectrum rows, the Nyquist values,
// the moduli and, in FP32, the old strain) are issued before any transform so
// that their latencies overlap.
// EIG: the system has an eigenstress (a.sstar); a separate instantiation,
// since its loads would otherwise size every x-pass's registers.
#ifndef LSFFT_X_WAVES
#define LSFFT_X_WAVES 3
#endif
// Three waves per SIMD for the FP32 power-of-two lengths up to 128 complex
// points per line, which fit 168 VGPRs with at most a few spilled values;
// the others keep the compiler's own choice.
template <typename T, int L, int E, bool EIG> constexpr int x_min_waves() {
  return (sizeof(T) == 4 && !EIG && E == 4 && L <= 128) ? LSFFT_X_WAVES : 1;
}
template <typename T, int L, int E, int WG, bool EIG>
__global__ __launch_bounds__(WG, (x_min_waves<T, L, E, EIG>())) void k_xpass(XArgs<T> a) {
  const int sysb = blockIdx.y;
  if (a.st && a.st[sysb].done) return;
  a.eps += sysb * 6 * a.bs.field;
  a.lam += sysb * a.bs.field;
  a.mu += sysb * a.bs.field;
  a.spec += sysb * a.bs.spec;
  a.nyq += sysb * a.bs.nyq;
  if (a.partial) a.partial += sysb * a.bs.part;
  if (EIG) a.sstar += sysb * 6 * a.bs.field;
  // the system's constants in registers
  T Ebl[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) Ebl[c] = (T)a.mem[sysb].Eb[c];
  const T lam0 = a.mem[sysb].lam0, mu0 = a.mem[sysb].mu0;
  __shared__ cplx<T> twl_[2 * L];
  constexpr int TPC = L / E;
  constexpr int P = lines_per_wg(TPC, WG);
  constexpr bool PRELOAD_EPS = (sizeof(T) == 4) && LSFFT_X_PRELOAD;
  __shared__ cplx<T> lds[line_slots<TPC, WG>() * line_scratch<L>()];
  __shared__ double red[(WG + 63) / 64 * 8];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  int p, t;
  bool live;
  line_of<TPC, P>(tid, p, t, live);
  const long long row = (long long)blockIdx.x * P + p;
  const bool valid = live && row < a.d.rows;
  const int n1 = 2 * L;
  const long long N = a.d.N;
  cplx<T> *sl = lds + p * line_scratch<L>();
  int buf = 0;
  const bool need_delta = (a.mode == XMODE_UPDATE || a.mode == XMODE_DGO);
  const bool need_old = (a.mode != XMODE_INIT);
  const T *eps_src = (a.mode == XMODE_EXTERNAL) ? a.eps_in : a.eps;
  const bool write_eps = (a.mode != XMODE_EXTERNAL);
  const cplx<T> zero{T(0), T(0)};

  cplx<T> w[6][E];
  cplx<T> xn[6];
  T lam[E][2], mu[E][2];
  T eo[PRELOAD_EPS ? 6 : 1][E][2];
  if (need_delta && valid) {
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const cplx<T> *src = a.spec + ((long long)c * a.d.rows + row) * L;
#pragma unroll
      for (int e = 0; e < E; ++e) w[c][e] = ldc_nt(src + t + TPC * e);
      xn[c] = (t == 0) ? a.nyq[(long long)c * a.d.rows + row] : zero;
    }
  } else {
#pragma unroll
    for (int c = 0; c < 6; ++c) {
#pragma unroll
      for (int e = 0; e < E; ++e) w[c][e] = zero;
      xn[c] = zero;
    }
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const long long idx = row * n1 + 2 * (t + TPC * e);
    if (valid) {
      ld2_nt(a.lam + idx, lam[e][0], lam[e][1]);
      ld2_nt(a.mu + idx, mu[e][0], mu[e][1]);
    } else {
      lam[e][0] = lam[e][1] = mu[e][0] = mu[e][1] = T(0);
    }
  }
  if constexpr (PRELOAD_EPS) {
#pragma unroll
    for (int c = 0; c < 6; ++c)
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const long long idx = row * n1 + 2 * (t + TPC * e);
        if (valid && need_old) ld2_nt(eps_src + c * N + idx, eo[c][e][0], eo[c][e][1]);
        else eo[c][e][0] = eo[c][e][1] = T(0);
      }
  }
  const cplx<T> *twl = stage_twiddles(twl_, a.tw);
  if (need_delta) {
#pragma unroll
    for (int c = 0; c < 6; ++c) c2r_line<T, L, E>(w[c], xn[c], t, lane, sl, twl, buf);
  }

  double sums[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const long long idx = row * n1 + 2 * (t + TPC * e);
    T ev[6][2];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      T o0, o1;
      if constexpr (PRELOAD_EPS) {
        o0 = eo[c][e][0];
        o1 = eo[c][e][1];
      } else {
        o0 = o1 = T(0);
        if (valid && need_old) ld2_nt(eps_src + c * N + idx, o0, o1);
      }
      T n0, n1v;
      if (a.mode == XMODE_UPDATE) {
        n0 = o0 + w[c][e].x;
        n1v = o1 + w[c][e].y;
      } else if (a.mode == XMODE_DGO) {
        n0 = Ebl[c] + w[c][e].x;
        n1v = Ebl[c] + w[c][e].y;
      } else if (a.mode == XMODE_INIT) {
        n0 = Ebl[c];
        n1v = Ebl[c];
      } else {
        n0 = o0;
        n1v = o1;
      }
      if (a.mode == XMODE_DGO && valid) {
        const double d0 = (double)n0 - (double)o0, d1 = (double)n1v - (double)o1;
        sums[6] += (c < 3 ? 1.0 : 2.0) * (d0 * d0 + d1 * d1);
      }
      if (valid && write_eps) st2_nt(a.eps + c * N + idx, n0, n1v);
      ev[c][0] = n0;
      ev[c][1] = n1v;
    }
    // eigenstress of the two voxels (T = C [E - E_*]); zero without eigenstrain
    T ss[6][2];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      ss[c][0] = ss[c][1] = T(0);
      if (EIG && valid) ld2_nt(a.sstar + c * N + idx, ss[c][0], ss[c][1]);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const T tr = ev[0][h] + ev[1][h] + ev[2][h];
      const T l = lam[e][h], m2 = T(2) * mu[e][h];
      const T lp = l - lam0, mp2 = m2 - T(2) * mu0;
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const T sg = (c < 3 ? l * tr : T(0)) + m2 * ev[c][h] - ss[c][h];
        if (valid) sums[c] += (double)sg;
        const T fin = a.polarisation ? (c < 3 ? lp * tr : T(0)) + mp2 * ev[c][h] - ss[c][h] : sg;
        if (h == 0) w[c][e].x = fin; else w[c][e].y = fin;
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const cplx<T> x_nyq = r2c_line<T, L, E>(w[c], t, lane, sl, twl, buf);
    if (valid) {
      cplx<T> *dst = a.spec + ((long long)c * a.d.rows + row) * L;
#pragma unroll
      for (int e = 0; e < E; ++e) stc_nt(dst + t + TPC * e, w[c][e]);
      if (t == 0) a.nyq[(long long)c * a.d.rows + row] = x_nyq;
    }
  }

  if (a.partial) {
    block_sum<WG>(sums, 7, red);
    if (tid == 0) {
      double *dst = a.partial + (long long)blockIdx.x * 8;
      for (int i = 0; i < 7; ++i) dst[i] = sums[i];
      dst[7] = 0.0;
    }
  }
}

// ---------------------------------------------------------------- y pass
template <typename T> struct YArgs {
  Dims d;
  cplx<T> *spec;
  cplx<T> *nyq;
  const cplx<T> *tw;  // exp(-2 pi i m / n2)
  const State *st;    // [system]
  Strides bs;
  long long main_blocks;
  int ncomp;          // components transformed (6 strain form, 3 displacement form)
  int xcd;            // 1: XCD-aware order of the column tiles
};

// Columns: main = (c, k3, kx) flattened, P consecutive per workgroup, stride
// n1/2 between y points; Nyquist plane = (c, k3) rows, stride 1.
template <typename T, int NY, int E, int P, bool FWD>
__global__ __launch_bounds__(P *(NY / E)) void k_ypass(YArgs<T> a) {
  const int sysb = blockIdx.y;
  if (a.st && a.st[sysb].done) return;
  a.spec += sysb * a.bs.spec;
  a.nyq += sysb * a.bs.nyq;
  __shared__ cplx<T> twl_[NY];
  constexpr int TPC = NY / E;
  __shared__ cplx<T> lds[2 * NY * P];
  const int tid = threadIdx.x;
  const int p = tid % P, t = tid / P;
  const int L = a.d.L;
  cplx<T> *base;
  long long stride;
  bool valid;
  if ((long long)blockIdx.x < a.main_blocks) {
    const long long col = tile_of(blockIdx.x, a.main_blocks, a.xcd) * P + p;
    const long long ncol = (long long)a.ncomp * a.d.n3 * L;
    valid = col < ncol;
    const long long slab = col / L, kx = col % L;
    base = a.spec + slab * (long long)NY * L + kx;
    stride = L;
  } else {
    const long long col = ((long long)blockIdx.x - a.main_blocks) * P + p;
    valid = col < (long long)a.ncomp * a.d.n3;
    base = a.nyq + col * NY;
    stride = 1;
  }
  cplx<T> v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = valid ? base[(t + TPC * e) * stride] : cplx<T>{T(0), T(0)};
  int buf = 0;
  const cplx<T> *twl = stage_twiddles(twl_, a.tw);
  fft_pencil<T, NY, E, FWD>(v, t, lds + p, P, twl, 1, buf);
  if (valid) {
#pragma unroll
    for (int e = 0; e < E; ++e) base[(t + TPC * e) * stride] = v[e];
  }
}

// ---------------------------------------------------------------- z pass + Green
template <typename T> struct ZArgs {
  Dims d;
  cplx<T> *spec;
  cplx<T> *nyq;
  const cplx<T> *tw;  // exp(-2 pi i m / n3)
  GreenParams<T> g;
  const Member<T> *mem;  // reference medium of each system (null: g as given)
  Strides bs;
  double *partial;    // [system][gridDim.x]
  const State *st;    // [system]
  long long main_blocks;
  int forward_only;   // 1: forward transform only (operator entry point)
  int xcd;            // 1: XCD-aware order of the column tiles
};

// The Green parameters of system b: the shared tables and the system's C0.
template <typename T> __device__ __forceinline__ void member_green(GreenParams<T> &g, const Member<T> *mem, int b) {
  if (!mem) return;
  const Member<T> &m = mem[b];
  g.lam0 = m.lam0;
  g.mu0 = m.mu0;
  g.c1 = m.c1;
  g.c2 = m.c2;
  g.beta = m.beta;
}

// SCH: the scheme, fixed at compile time for AFB (its Green step and tables
// only, sizing the kernel for that path), or -1: any scheme, from a.g.
#ifndef LSFFT_Z_WAVES
#define LSFFT_Z_WAVES 3
#endif
template <typename T, int SCH> constexpr int z_min_waves() {
  return (sizeof(T) == 4 && SCH == SCHEME_AFB) ? LSFFT_Z_WAVES : 1;
}
template <typename T, int NZ, int E, int P, int SCH>
__global__ __launch_bounds__(P *(NZ / E), (z_min_waves<T, SCH>())) void k_zpass(ZArgs<T> a) {
  const int sysb = blockIdx.y;
  if (a.st && a.st[sysb].done) return;
  a.spec += sysb * a.bs.spec;
  a.nyq += sysb * a.bs.nyq;
  if (a.partial) a.partial += sysb * a.bs.part;
  member_green(a.g, a.mem, sysb);
  __shared__ cplx<T> twl_[NZ];
  constexpr int TPC = NZ / E;
  constexpr int WG = P * TPC;
  __shared__ cplx<T> lds[2 * NZ * P];
  __shared__ double red[(WG + 63) / 64 * 8];
  const int tid = threadIdx.x;
  const int p = tid % P, t = tid / P;
  const int L = a.d.L;
  // one buffer resource per component (each below 4 GiB): the thread's
  // column and z point a fixed 32-bit byte offset, each z step a scalar one;
  // a column past the last one lies past the resource (its loads return 0)
  unsigned zstride, voff;
  int i1, i2;
  bool valid;
  const cplx<T> *cbase;
  long long cstride;
  if ((long long)blockIdx.x < a.main_blocks) {
    const unsigned col = (unsigned)(tile_of(blockIdx.x, a.main_blocks, a.xcd) * P + p);
    valid = col < (unsigned)(a.d.n2 * L);
    i2 = (int)(col / (unsigned)L);
    i1 = (int)(col % (unsigned)L);
    zstride = (unsigned)(a.d.n2 * L);
    cbase = a.spec;
    cstride = a.d.comp_main;
    voff = (col + (unsigned)t * zstride) * (unsigned)sizeof(cplx<T>);
  } else {
    const unsigned col = (unsigned)(((long long)blockIdx.x - a.main_blocks) * P + p);
    valid = col < (unsigned)a.d.n2;
    i2 = (int)col;
    i1 = L;
    zstride = (unsigned)a.d.n2;
    cbase = a.nyq;
    cstride = a.d.comp_nyq;
    voff = (col + (unsigned)t * zstride) * (unsigned)sizeof(cplx<T>);
  }
  __amdgpu_buffer_rsrc_t rs[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) rs[c] = buffer_of(cbase + c * cstride, cstride);
  auto soff = [&](int e) { return (unsigned)(TPC * e) * zstride * (unsigned)sizeof(cplx<T>); };
  cplx<T> v[6][E];
  // every load of the tile first, then the transforms
#pragma unroll
  for (int c = 0; c < 6; ++c)
#pragma unroll
    for (int e = 0; e < E; ++e) v[c][e] = load_c<T>(rs[c], voff, soff(e));
  const AxisVal<T> axx = axis_val_s<SCH>(a.g, 0, i1), axy = axis_val_s<SCH>(a.g, 1, valid ? i2 : 0);
#if LSFFT_LDS_AXIS
  __shared__ AxisVal<T> axl[NZ];
  for (int i = threadIdx.x; i < NZ; i += blockDim.x) axl[i] = axis_val_s<SCH>(a.g, 2, i);
#else
  AxisVal<T> axz[E];
#pragma unroll
  for (int e = 0; e < E; ++e) axz[e] = axis_val_s<SCH>(a.g, 2, t + TPC * e);
#endif
  int buf = 0;
  const cplx<T> *twl = stage_twiddles(twl_, a.tw);  // its barrier publishes axl too
#pragma unroll
  for (int c = 0; c < 6; ++c) fft_pencil<T, NZ, E, true>(v[c], t, lds + p, P, twl, 1, buf);
  if (a.forward_only) {
    if (valid) {
#pragma unroll
      for (int c = 0; c < 6; ++c)
#pragma unroll
        for (int e = 0; e < E; ++e) store_c<T>(rs[c], voff, soff(e), v[c][e]);
    }
    return;
  }
  double res = 0.0;
  const double wgt = (i1 == 0 || i1 == L) ? 1.0 : 2.0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    cplx<T> s[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) s[c] = v[c][e];
#if LSFFT_LDS_AXIS
    const AxisVal<T> ax[3] = {axx, axy, axl[t + TPC * e]};
#else
    const AxisVal<T> ax[3] = {axx, axy, axz[e]};
#endif
    const double r = green_point_s<SCH>(a.g, i1, valid ? i2 : 0, t + TPC * e, ax, s);
    if (valid) res += wgt * r;
#pragma unroll
    for (int c = 0; c < 6; ++c) v[c][e] = s[c];
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    fft_pencil<T, NZ, E, false>(v[c], t, lds + p, P, twl, 1, buf);
    if (valid) {
#pragma unroll
      for (int e = 0; e < E; ++e) store_c<T>(rs[c], voff, soff(e), v[c][e]);
    }
  }
  if (a.partial) {
    double vals[1] = {res};
    block_sum<WG>(vals, 1, red);
    if (tid == 0) a.partial[blockIdx.x] = vals[0];
  }
}

// ---------------------------------------------------------------- reduction
// Strain form: two kernels, both in a fixed order (deterministic):
// k_reduce_stage sums contiguous chunks of the x-pass and z-pass block sums
// into RSTAGE rows of 8 doubles; k_reduce sums those rows and takes the stop
// decision.  Displacement form: the last workgroup of the stencil launch
// does both (last_block_reduce below).
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

// The stop decision of system sysb from its summed partials vals[8] (6
// stress sums, x-side residual or |d eps|^2, z-side residual); one thread.
__device__ inline void reduce_decide(const ReduceArgs &a, int sysb, const double (&vals)[8]) {
  State &s = a.st[sysb];
  double *hist = a.hist + sysb * a.hcap;
  const double ebar_norm = a.ebar_norms[sysb];
  // the iteration index lives on the device, so that a captured sequence of
  // iterations can be replayed unchanged
  const int k = s.k;
  double mean[6];
  double sn = 0.0;
  for (int c = 0; c < 6; ++c) {
    mean[c] = vals[c] / a.N - (a.smean ? a.smean[6 * sysb + c] : 0.0);
    sn += (c < 3 ? 1.0 : 2.0) * mean[c] * mean[c];
  }
  // r: the stopping test's residual; g: the quantity whose growth past
  // div_factor times its first value means divergence (GFP: the unnormalised
  // equilibrium norm, since r itself stays bounded while the mean stress
  // grows with a diverging iterate; DGO: r, whose scale is fixed)
  double r, g;
  if (a.dgo) {
    r = (k == 0) ? __builtin_huge_val() : sqrt(vals[6]) / (sqrt(a.N) * ebar_norm);
    g = r;
  } else {
    const double num = a.disp ? sqrt(a.N * vals[6]) : sqrt(vals[7]);
    const double den = a.N * sqrt(sn);
    r = (num == 0.0) ? 0.0 : (den > 0.0 ? num / den : __builtin_huge_val());
    g = num;
  }
  hist[k] = r;
  s.r = r;
  for (int c = 0; c < 6; ++c) s.sig_mean[c] = mean[c];
  s.iters = k;
  const int first = a.dgo ? 1 : 0;
  if (k == first) s.r0 = g;
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
  } else if (!finite || g > a.div_factor * fmax(s.r0, 1e-300)) {
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

// Rows of block sums that another XCD will read inside the same launch are
// written and read with device-scope atomics: such accesses go to the
// device's coherence point, so no write-back of the whole L2 (which a
// device-scope fence would issue) is needed to publish eight doubles.
__device__ __forceinline__ void store_row_coherent(double *dst, const double *vals, int nv) {
  for (int i = 0; i < nv; ++i) __hip_atomic_store(dst + i, vals[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Called by every workgroup of a launch that wrote its row of 8 block sums
// into ra.px (system sysb) with store_row_coherent: the workgroup that arrives
// last sums every row in a fixed order (deterministic, whichever workgroup it
// is) and takes the stop decision, then rearms the system's arrival counter.
// The row's stores complete (s_waitcnt) before the arrival is counted.
template <int WG>
__device__ __forceinline__ void last_block_reduce(const ReduceArgs &ra, unsigned *counter, int sysb, double *red) {
  __shared__ int last;
  __syncthreads();  // this workgroup's row is issued (by thread 0)
  if (threadIdx.x == 0) {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    const unsigned prev = __hip_atomic_fetch_add(counter + sysb, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    last = (prev == gridDim.x - 1) ? 1 : 0;
  }
  __syncthreads();
  if (!last) return;
  const double *px = ra.px + sysb * ra.spx;
  double vals[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (long long i = threadIdx.x; i < ra.nx; i += WG)
    for (int c = 0; c < 7; ++c) vals[c] += __hip_atomic_load(px + i * 8 + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  block_sum<WG>(vals, 8, red);
  if (threadIdx.x == 0) {
    reduce_decide(ra, sysb, vals);
    counter[sysb] = 0u;
  }
}

// ---------------------------------------------------------------- pointwise helpers
// Sensitivity of J = <eps_a : C : eps_b> (= A : C_eff : B for the converged
// strains under macroscopic loads A and B) to the moduli of each voxel: the
// discrete problem minimises a quadratic energy over compatible fluctuations,
// so the derivative of the minimum is the partial derivative at the minimiser:
//   dJ/dlambda(x) = tr eps_a tr eps_b / N,   dJ/dmu(x) = 2 eps_a : eps_b / N,
// and at fixed Poisson ratio dJ/dE(x) = (lambda dJ/dlambda + mu dJ/dmu) / E
// with E = mu (3 lambda + 2 mu) / (lambda + mu).  FP64 arithmetic; any output
// may be null.
template <typename T>
__global__ void k_stiffness_gradient(const T *__restrict__ ea, const T *__restrict__ eb, const T *__restrict__ lam,
                                     const T *__restrict__ mu, T *__restrict__ dl, T *__restrict__ dm,
                                     T *__restrict__ de, long long N) {
  const double inv = 1.0 / (double)N;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x) {
    double tra = 0.0, trb = 0.0, dd = 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const double a = (double)ea[c * N + i], b = (double)eb[c * N + i];
      if (c < 3) {
        tra += a;
        trb += b;
      }
      dd += (c < 3 ? 1.0 : 2.0) * a * b;
    }
    const double gl = tra * trb * inv, gm = 2.0 * dd * inv;
    if (dl) dl[i] = (T)gl;
    if (dm) dm[i] = (T)gm;
    if (de) {
      const double l = (double)lam[i], m = (double)mu[i];
      const double E = m * (3.0 * l + 2.0 * m) / (l + m);
      de[i] = (T)((l * gl + m * gm) / E);
    }
  }
}

template <typename T>
__global__ void k_hooke_out(const T *__restrict__ eps, const T *__restrict__ lam, const T *__restrict__ mu,
                            const T *__restrict__ sstar, T *__restrict__ sig, long long N) {
  // sstar: the eigenstress C E_* [6][N], or null
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x) {
    const T e0 = eps[i], e1 = eps[N + i], e2 = eps[2 * N + i];
    const T l = lam[i], m2 = T(2) * mu[i];
    const T tr = e0 + e1 + e2;
    T s6[6] = {l * tr + m2 * e0, l * tr + m2 * e1, l * tr + m2 * e2,
               m2 * eps[3 * N + i], m2 * eps[4 * N + i], m2 * eps[5 * N + i]};
    if (sstar)
      for (int c = 0; c < 6; ++c) s6[c] -= sstar[c * N + i];
    for (int c = 0; c < 6; ++c) sig[c * N + i] = s6[c];
  }
}

// internal (main + Nyquist plane) <-> standard half spectrum [6][n3][n2][L+1]
template <typename T>
__global__ void k_to_standard(const cplx<T> *__restrict__ spec, const cplx<T> *__restrict__ nyq,
                              cplx<T> *__restrict__ out, Dims d) {
  const long long total = 6LL * d.rows * (d.L + 1);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long long)gridDim.x * blockDim.x) {
    const long long r = i / (d.L + 1);
    const int k = (int)(i % (d.L + 1));
    out[i] = (k < d.L) ? spec[r * d.L + k] : nyq[r];
  }
}

template <typename T>
__global__ void k_from_standard(const cplx<T> *__restrict__ in, cplx<T> *__restrict__ spec,
                                cplx<T> *__restrict__ nyq, Dims d) {
  const long long total = 6LL * d.rows * (d.L + 1);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long long)gridDim.x * blockDim.x) {
    const long long r = i / (d.L + 1);
    const int k = (int)(i % (d.L + 1));
    if (k < d.L) spec[r * d.L + k] = in[i];
    else nyq[r] = in[i];
  }
}

// Green step at every frequency of a standard half spectrum (operator entry point).
template <typename T>
__global__ void k_green_only(const cplx<T> *__restrict__ in, cplx<T> *__restrict__ out, GreenParams<T> g, Dims d,
                             double *partial) {
  const long long nf = d.rows * (d.L + 1);
  const long long cs = nf;
  double res = 0.0;
  for (long long f = (long long)blockIdx.x * blockDim.x + threadIdx.x; f < nf; f += (long long)gridDim.x * blockDim.x) {
    const int i1 = (int)(f % (d.L + 1));
    const long long r = f / (d.L + 1);
    const int i2 = (int)(r % d.n2), i3 = (int)(r / d.n2);
    cplx<T> s[6];
    for (int c = 0; c < 6; ++c) s[c] = in[c * cs + f];
    const double w = (i1 == 0 || i1 == d.L) ? 1.0 : 2.0;
    res += w * green_point(g, i1, i2, i3, s);
    for (int c = 0; c < 6; ++c) out[c * cs + f] = s[c];
  }
  __shared__ double red[4 * 8];
  double vals[1] = {res};
  block_sum<256>(vals, 1, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = vals[0];
}

// ---------------------------------------------------------------- DGO table
// One thread per half-spectrum frequency: P_ij = sum_nu w n_i n_j and
// Q_ijkl = sum_nu w n_i n_j n_k n_l over the periodic images of Sec. 5.4,
// weight w = prod_r sinc^p(pi (kappa_r + nu_r n_r) / n_r), n = k/|k|,
// k_r = 2 pi (kappa_r + nu_r n_r) / (n_r h_r).  nu_r in [-M, M], and
// [-M, M+1] at the Nyquist index (symmetric image set).
template <typename T>
__global__ void k_dgo_build(T *main, T *nyq, Dims d, int M, int p, double h1, double h2, double h3) {
  const long long nf = d.rows * (d.L + 1);
  const long long f = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const int i1 = (int)(f % (d.L + 1));
  const long long r = f / (d.L + 1);
  const int i2 = (int)(r % d.n2), i3 = (int)(r / d.n2);
  const int n[3] = {d.n1, d.n2, d.n3};
  const int idx[3] = {i1, i2, i3};
  const double h[3] = {h1, h2, h3};
  int kap[3];
  double sv[3];
  int hi[3];
  for (int q = 0; q < 3; ++q) {
    kap[q] = (2 * idx[q] < n[q]) ? idx[q] : idx[q] - n[q];
    sv[q] = sinpi((double)kap[q] / n[q]);
    hi[q] = (2 * kap[q] == -n[q]) ? M + 1 : M;
  }
  double P[6] = {0, 0, 0, 0, 0, 0}, Q[15];
  for (int q = 0; q < 15; ++q) Q[q] = 0.0;
  const bool dc = (kap[0] == 0 && kap[1] == 0 && kap[2] == 0);
  if (!dc) {
    for (int v3 = -M; v3 <= hi[2]; ++v3) {
      double w3, k3;
      {
        const int m = kap[2] + v3 * n[2];
        if (kap[2] == 0) { w3 = (v3 == 0) ? 1.0 : 0.0; }
        else { w3 = ((v3 & 1) ? -sv[2] : sv[2]) / (M_PI * ((double)kap[2] / n[2] + v3)); }
        k3 = 2.0 * M_PI * m / (n[2] * h[2]);
        if (p == 2) w3 *= w3;
      }
      if (w3 == 0.0) continue;
      for (int v2 = -M; v2 <= hi[1]; ++v2) {
        double w2, k2;
        {
          const int m = kap[1] + v2 * n[1];
          if (kap[1] == 0) { w2 = (v2 == 0) ? 1.0 : 0.0; }
          else { w2 = ((v2 & 1) ? -sv[1] : sv[1]) / (M_PI * ((double)kap[1] / n[1] + v2)); }
          k2 = 2.0 * M_PI * m / (n[1] * h[1]);
          if (p == 2) w2 *= w2;
        }
        if (w2 == 0.0) continue;
        for (int v1 = -M; v1 <= hi[0]; ++v1) {
          double w1, k1;
          const int m = kap[0] + v1 * n[0];
          if (kap[0] == 0) { w1 = (v1 == 0) ? 1.0 : 0.0; }
          else { w1 = ((v1 & 1) ? -sv[0] : sv[0]) / (M_PI * ((double)kap[0] / n[0] + v1)); }
          k1 = 2.0 * M_PI * m / (n[0] * h[0]);
          if (p == 2) w1 *= w1;
          if (w1 == 0.0) continue;
          const double w = w1 * w2 * w3;
          const double kk = k1 * k1 + k2 * k2 + k3 * k3;
          const double inv = 1.0 / sqrt(kk);
          const double nv[3] = {k1 * inv, k2 * inv, k3 * inv};
          P[0] += w * nv[0] * nv[0];
          P[1] += w * nv[1] * nv[1];
          P[2] += w * nv[2] * nv[2];
          P[3] += w * nv[1] * nv[2];
          P[4] += w * nv[0] * nv[2];
          P[5] += w * nv[0] * nv[1];
          for (int a4 = 0; a4 <= 4; ++a4)
            for (int b4 = 0; b4 <= 4 - a4; ++b4) {
              const int c4 = 4 - a4 - b4;
              double mnm = w;
              for (int q = 0; q < a4; ++q) mnm *= nv[0];
              for (int q = 0; q < b4; ++q) mnm *= nv[1];
              for (int q = 0; q < c4; ++q) mnm *= nv[2];
              Q[qidx(a4, b4)] += mnm;
            }
        }
      }
    }
  }
  if (i1 < d.L) {
    const long long o = ((long long)i3 * d.n2 + i2) * d.L + i1;
    const long long cs = d.rows * d.L;
    for (int q = 0; q < 6; ++q) main[q * cs + o] = (T)P[q];
    for (int q = 0; q < 15; ++q) main[(6 + q) * cs + o] = (T)Q[q];
  } else {
    const long long o = (long long)i3 * d.n2 + i2;
    const long long cs = d.rows;
    for (int q = 0; q < 6; ++q) nyq[q * cs + o] = (T)P[q];
    for (int q = 0; q < 15; ++q) nyq[(6 + q) * cs + o] = (T)Q[q];
  }
}

}  // namespace lsfft
