// Device-side building blocks: complex arithmetic and an in-workgroup
// Stockham FFT of one pencil whose L points are spread over L/E threads,
// E points per thread, exchanged through LDS between radix passes.
//
// Data distribution (input AND output, both directions): the thread with
// pencil-local index t holds points  m = t + (L/E) * e,  e = 0..E-1,  in v[e].
// So a pencil can be loaded, transformed, processed point-wise and stored
// back without any reordering.
#pragma once
#include <hip/hip_runtime.h>

namespace lsfft {

template <typename T> struct cplx {
  T x, y;
};

template <typename T> __device__ __forceinline__ cplx<T> mk(T a, T b) { return cplx<T>{a, b}; }
template <typename T> __device__ __forceinline__ cplx<T> operator+(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T> __device__ __forceinline__ cplx<T> operator-(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T> __device__ __forceinline__ cplx<T> operator*(cplx<T> a, cplx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T> __device__ __forceinline__ cplx<T> operator*(T s, cplx<T> a) { return {s * a.x, s * a.y}; }
template <typename T> __device__ __forceinline__ cplx<T> conjg(cplx<T> a) { return {a.x, -a.y}; }
// multiply by -i (forward) or +i (inverse)
template <typename T, bool FWD> __device__ __forceinline__ cplx<T> rot(cplx<T> a) {
  return FWD ? cplx<T>{a.y, -a.x} : cplx<T>{-a.y, a.x};
}
template <typename T> __device__ __forceinline__ cplx<T> mul_i(cplx<T> a) { return {-a.y, a.x}; }
template <typename T> __device__ __forceinline__ T norm2(cplx<T> a) { return a.x * a.x + a.y * a.y; }

// ---------------------------------------------------------------- radix plans
// Passes use radices from {8, 4, 3, 2}, greedily the largest that divides both
// the remaining length and E (each thread then runs E/R butterflies per pass).
template <int L, int E> struct Plan {
  static constexpr int pick(int rem) {
    return (rem % 8 == 0 && E % 8 == 0) ? 8
         : (rem % 4 == 0 && E % 4 == 0) ? 4
         : (rem % 3 == 0 && E % 3 == 0) ? 3
         : (rem % 2 == 0 && E % 2 == 0) ? 2 : 0;
  }
  static constexpr int npass() {
    int rem = L, n = 0;
    while (rem > 1) {
      int r = pick(rem);
      if (r == 0) return -1;
      rem /= r;
      ++n;
    }
    return n;
  }
  static constexpr int radix(int p) {
    int rem = L, r = 1;
    for (int i = 0; i <= p; ++i) { r = pick(rem); rem /= r; }
    return r;
  }
  static constexpr int stride(int p) {
    int s = 1;
    for (int i = 0; i < p; ++i) s *= radix(i);
    return s;
  }
  static_assert(L % E == 0, "E must divide L");
  static_assert(npass() > 0 || L == 1, "length not factorable with radices dividing E");
};

// ---------------------------------------------------------------- butterflies
// In-place DFT of R points, sign exp(-2 pi i / R) when FWD.
template <typename T, bool FWD> __device__ __forceinline__ void bfly2(cplx<T> *a) {
  cplx<T> t = a[0];
  a[0] = t + a[1];
  a[1] = t - a[1];
}

template <typename T, bool FWD> __device__ __forceinline__ void bfly3(cplx<T> *a) {
  const T c = T(-0.5);
  const T s = T(0.86602540378443864676372317075293618);  // sin(2 pi / 3)
  cplx<T> sum = a[1] + a[2], dif = a[1] - a[2];
  cplx<T> m = a[0] + c * sum;
  a[0] = a[0] + sum;
  cplx<T> r = s * rot<T, FWD>(dif);  // -i s (a1 - a2) forward
  a[1] = m + r;
  a[2] = m - r;
}

template <typename T, bool FWD> __device__ __forceinline__ void bfly4(cplx<T> *a) {
  cplx<T> t0 = a[0] + a[2], t1 = a[0] - a[2];
  cplx<T> t2 = a[1] + a[3], t3 = rot<T, FWD>(a[1] - a[3]);
  a[0] = t0 + t2;
  a[2] = t0 - t2;
  a[1] = t1 + t3;
  a[3] = t1 - t3;
}

template <typename T, bool FWD> __device__ __forceinline__ void bfly8(cplx<T> *a) {
  const T h = T(0.70710678118654752440084436210484904);  // sqrt(1/2)
  cplx<T> e[4] = {a[0], a[2], a[4], a[6]};
  cplx<T> o[4] = {a[1], a[3], a[5], a[7]};
  bfly4<T, FWD>(e);
  bfly4<T, FWD>(o);
  // twiddles W8^k, k = 1, 2, 3 (conjugated for the inverse)
  cplx<T> o1 = FWD ? cplx<T>{h * (o[1].x + o[1].y), h * (o[1].y - o[1].x)}
                   : cplx<T>{h * (o[1].x - o[1].y), h * (o[1].y + o[1].x)};
  cplx<T> o2 = rot<T, FWD>(o[2]);
  cplx<T> o3 = FWD ? cplx<T>{h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y)}
                   : cplx<T>{-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y)};
  a[0] = e[0] + o[0];
  a[4] = e[0] - o[0];
  a[1] = e[1] + o1;
  a[5] = e[1] - o1;
  a[2] = e[2] + o2;
  a[6] = e[2] - o2;
  a[3] = e[3] + o3;
  a[7] = e[3] - o3;
}

template <typename T, bool FWD, int R> __device__ __forceinline__ void bfly(cplx<T> *a) {
  if constexpr (R == 2) bfly2<T, FWD>(a);
  else if constexpr (R == 3) bfly3<T, FWD>(a);
  else if constexpr (R == 4) bfly4<T, FWD>(a);
  else if constexpr (R == 8) bfly8<T, FWD>(a);
}

// ---------------------------------------------------------------- Stockham pass
// tw: table of exp(-2 pi i m / L) at tw[m * ts], m = 0..L-1.
// lds: this pencil's scratch, two buffers of L points: point m of buffer b at
// lds[(b * L + m) * ms].  Exchanges alternate between the two buffers (the
// uniform counter `buf` carries the parity across calls), so one barrier per
// exchange suffices: a buffer is rewritten only after the barrier of the
// exchange in between, which every thread reaches after its last read of it.
// WAVE: every thread of the pencil lies in one wavefront and the scratch is
// the pencil's own, so the exchange is ordered at wavefront scope (a wave's
// LDS accesses complete in order) instead of by a workgroup barrier.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// PAD: point m of a buffer sits at slot m + m / 16 (buffers of L + L / 16
// slots), which spreads the strided writes of the early radix passes over
// the LDS banks; only for power-of-two lines with ms = 1 (see line_pad).
template <typename T, int L, int E, bool FWD, int P, bool WAVE = false, bool PAD = false>
struct StockhamPass {
  __device__ __forceinline__ static int slot(int m) { return PAD ? m + (m >> 4) : m; }
  __device__ __forceinline__ static void run(cplx<T> (&v)[E], int t, cplx<T> *lds, int ms,
                                             const cplx<T> *__restrict__ tw, int ts, int &buf) {
    using PL = Plan<L, E>;
    constexpr int NP = PL::npass();
    constexpr int R = PL::radix(P);
    constexpr int Ns = PL::stride(P);
    constexpr int NB = E / R;
    constexpr int TPC = L / E;
    constexpr bool LAST = (P + 1 == NP);
    constexpr int LP = PAD ? L + L / 16 : L;
    cplx<T> out[E];
    cplx<T> *sb = lds + (buf ? LP * ms : 0);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int j = t + TPC * b;
      cplx<T> a[R];
#pragma unroll
      for (int r = 0; r < R; ++r) a[r] = v[b + r * NB];
      const int k = (Ns > 1) ? (j % Ns) : 0;
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cplx<T> w = tw[(k * r * (L / (Ns * R))) * ts];
          if (!FWD) w.y = -w.y;
          a[r] = a[r] * w;
        }
      }
      bfly<T, FWD, R>(a);
      if (LAST) {
#pragma unroll
        for (int r = 0; r < R; ++r) out[b + r * NB] = a[r];
      } else {
        const int base = (j / Ns) * Ns * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) sb[slot(base + r * Ns) * ms] = a[r];
      }
    }
    if constexpr (LAST) {
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = out[e];
    } else {
      if constexpr (WAVE)
        wave_sync();
      else
        __syncthreads();
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = sb[slot(t + TPC * e) * ms];
      buf ^= 1;
      StockhamPass<T, L, E, FWD, P + 1, WAVE, PAD>::run(v, t, lds, ms, tw, ts, buf);
    }
  }
};

// One transform of a pencil; `buf` is the workgroup-uniform buffer parity,
// to be carried from one call to the next (start at 0).
template <typename T, int L, int E, bool FWD, bool WAVE = false, bool PAD = false>
__device__ __forceinline__ void fft_pencil(cplx<T> (&v)[E], int t, cplx<T> *lds, int ms,
                                           const cplx<T> *__restrict__ tw, int ts, int &buf) {
  if constexpr (L > 1) StockhamPass<T, L, E, FWD, 0, WAVE, PAD>::run(v, t, lds, ms, tw, ts, buf);
}

// Line transforms (one pencil per line, ms = 1): pad the exchange buffers of
// power-of-two lines of 16 points or more; their scratch is line_scratch<L>()
// points per line (two buffers).
constexpr bool line_pad_of(int L) { return L % 3 != 0 && L >= 16; }
constexpr int line_scratch_of(int L) { return 2 * (line_pad_of(L) ? L + L / 16 : L); }
template <int L> constexpr bool line_pad() { return line_pad_of(L); }
template <int L> constexpr int line_scratch() { return line_scratch_of(L); }

// Copy a twiddle table of NT entries into LDS with all threads of the
// workgroup, then synchronise.  Each radix pass reads its twiddles right
// before use; from LDS that costs tens of cycles instead of a cache round trip.
#ifndef LSFFT_LDS_TW
#define LSFFT_LDS_TW 1
#endif
template <typename T, int NT>
__device__ __forceinline__ const cplx<T> *stage_twiddles(cplx<T> (&dst)[NT], const cplx<T> *__restrict__ src) {
  // the barrier also publishes whatever else the workgroup staged before it
  if constexpr (!LSFFT_LDS_TW) {
    __syncthreads();
    return src;
  }
  for (int i = threadIdx.x; i < NT; i += blockDim.x) dst[i] = src[i];
  __syncthreads();
  return dst;
}

// Lines of TPC threads packed into wavefronts: 64 / TPC whole lines per
// wavefront, so that no line straddles two (the line transforms exchange at
// wavefront scope).  When TPC divides 64 every lane works and line p of a
// workgroup is threads [p TPC, (p + 1) TPC); otherwise the lanes past the
// last whole line of a wavefront idle.  lines_per_wg and line_slots count
// whole wavefronts (wg a multiple of 64); a workgroup with a partial last
// wavefront counts its lines itself.
constexpr int lines_per_wg(int tpc, int wg) { return (wg / 64) * (64 / tpc); }
// Line p (of NL per workgroup) and point index t of thread tid; `live` is
// false on idle lanes, which are given the dummy line NL + wavefront (their
// own scratch, nothing loaded or stored) and t < TPC.  In a partial last
// wavefront a line whose lanes were not all launched gets p >= NL too, when
// NL counts only the whole lines.
template <int TPC, int NL>
__device__ __forceinline__ void line_of(int tid, int &p, int &t, bool &live) {
  static_assert(TPC >= 1 && TPC <= 64, "a line must fit in one wavefront");
  if constexpr (64 % TPC == 0) {
    p = tid / TPC;
    t = tid % TPC;
    live = true;
  } else {
    constexpr int LPW = 64 / TPC;
    const int w = tid >> 6, l = tid & 63, q = l / TPC;
    live = q < LPW;
    t = l - q * TPC;
    p = live ? w * LPW + q : NL + w;
  }
}
// Scratch lines a workgroup of WG threads needs for lines of TPC threads
// (one dummy line per wavefront when lanes idle).
template <int TPC, int WG> constexpr int line_slots() {
  return lines_per_wg(TPC, WG) + (64 % TPC == 0 ? 0 : WG / 64);
}

// Number of LDS exchanges the transform performs (passes - 1).
template <int L, int E> constexpr int fft_exchanges() { return Plan<L, E>::npass() - 1; }

}  // namespace lsfft
