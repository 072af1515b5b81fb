// The Green step of one frequency, evaluated from per-axis tables.
//
// Input: the six Voigt tensor components of sigma_hat (or of the
// polarisation tau_hat for the DGO) at frequency (i1, i2, i3) of the
// half spectrum.  Output, in place: the strain increment
//   BASIC / AFB:  -Gamma_0(k) sigma_hat, with the isotropic closed form
//       Gamma_0(k) A = (1/mu0) sym(n (x) A n) - (lam0+mu0)/(mu0 (lam0+2 mu0)) (n.A n) n (x) n,
//     n = k/|k|, i.e. Gamma_0 = -Gamma_H of Sec. 5.4 eq. (48);
//       BASIC: k_r = 2 pi kappa_r / (n_r h_r), a Nyquist component zeroed when
//              another, non-Nyquist component is nonzero (real-field reading);
//       AFB:   k_r = (2/h_r) sin(pi kappa_r/n_r) cos(pi kappa_s/n_s) cos(pi kappa_t/n_t),
//              the real vector with q^AhC = i k and q^AFD = Phi i k (Sec. 5.3 eq. (43)),
//              so the phase Phi cancels from the strain update of eq. (34);
//       CD:    k_r = sin(2 pi kappa_r/n_r)/h_r, q^CD = i k of eq. (14) with the
//              conjugate divergence;
//       ACD:   k_r = sin(2 pi kappa_r/n_r)/h_r cos(2 pi kappa_s/n_s) cos(2 pi kappa_t/n_t),
//              the averaged central difference of Sec. 5.3 eq. (43), conjugate pair;
//   FB: q^a = a_r = (e^{i 2 pi kappa_r/n_r} - 1)/h_r, q^b = conj(a) (eq. (45)):
//       increment = -sym( K^{-1} (sigma_hat conj(a)) (x) a ),
//       K = mu0 |a|^2 I + mu0 a (x) conj(a) + lam0 conj(a) (x) a  (= -G^{-1}, eq. (34));
//   DGO: the increment is the new strain spectrum
//       eps_hat = -[ (1/mu0) sym(tau_hat P) - beta/mu0 Q : tau_hat ],
//       P = sum_nu w_nu n n, Q = sum_nu w_nu n n n n (image sums of Sec. 5.4).
// Everything is multiplied by `scale` (1/N: the inverse transforms are
// unnormalised).  Zero output at xi = 0 and where the wavevector vanishes.
// Returns |sigma_hat q^b|^2 for the equilibrium residual (0 for the DGO).
#pragma once
#include "fft.hpp"

namespace lsfft {

// 1 / x: the hardware reciprocal in FP32 (1 ulp; the Green steps' 1 / |k|^2
// and complex divisions, far from the denormal range), a division in FP64.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

enum { SCHEME_BASIC = 0, SCHEME_FB = 1, SCHEME_AFB = 2, SCHEME_DGO = 3, SCHEME_CD = 4, SCHEME_ACD = 5 };

// Table kinds, laid out tab[kind * (n1 + n2 + n3) + off[axis] + i]:
// TAB_K 2 pi kappa/(n h); TAB_SH (2/h) sin(pi kappa/n); TAB_C cos(pi kappa/n);
// TAB_AR, TAB_AI real and imaginary parts of (e^{2 pi i kappa/n} - 1)/h (the
// imaginary part is also the central-difference wavenumber sin(2 pi kappa/n)/h);
// TAB_C2 cos(2 pi kappa/n).  Zeros are exact.
enum { TAB_K = 0, TAB_SH = 1, TAB_C = 2, TAB_AR = 3, TAB_AI = 4, TAB_C2 = 5, TAB_KINDS = 6 };

template <typename T> struct GreenParams {
  int scheme;
  int n[3];
  int off[3];
  int tabS;
  const T *tab;
  T c1;     // 1 / mu0
  T c2;     // (lam0 + mu0) / (mu0 (lam0 + 2 mu0))
  T beta;   // (lam0 + mu0) / (lam0 + 2 mu0)
  T lam0, mu0;
  T scale;  // 1 / N
  // DGO tables: 21 coefficient planes (P: 6, Q: 15) of the half spectrum,
  // kx in [0, n1/2) in `dgo_main`, kx = n1/2 in `dgo_nyq`.
  const T *dgo_main;
  const T *dgo_nyq;
  long long dgo_main_stride;  // elements between coefficient planes
  long long dgo_nyq_stride;
};

// Voigt slot -> (i, j)
__device__ __forceinline__ constexpr int vi(int I) { return I == 0 ? 0 : I == 1 ? 1 : I == 2 ? 2 : I == 3 ? 1 : I == 4 ? 0 : 0; }
__device__ __forceinline__ constexpr int vj(int I) { return I == 0 ? 0 : I == 1 ? 1 : I == 2 ? 2 : I == 3 ? 2 : I == 4 ? 2 : 1; }
// (i, j) -> Voigt slot
__host__ __device__ __forceinline__ constexpr int voigt(int i, int j) {
  return i == j ? i : ((i + j) == 3 ? 3 : (i + j) == 2 ? 4 : 5);
}
// index of the fully symmetric 4th-order moment with exponent counts (a, b, c)
__host__ __device__ __forceinline__ constexpr int qidx(int a, int b) {
  return (a == 4 ? 0 : a == 3 ? 1 : a == 2 ? 3 : a == 1 ? 6 : 10) + (4 - a - b);
}
__host__ __device__ __forceinline__ constexpr int qidx4(int i, int j, int k, int l) {
  return qidx((i == 0) + (j == 0) + (k == 0) + (l == 0), (i == 1) + (j == 1) + (k == 1) + (l == 1));
}

template <typename T>
__device__ __forceinline__ T tabv(const GreenParams<T> &g, int kind, int axis, int i) {
  return g.tab[kind * g.tabS + g.off[axis] + i];
}

// Real-wavevector Green step (BASIC, AFB).  s: Voigt components, in place.
template <typename T>
__device__ __forceinline__ double green_real(const GreenParams<T> &g, const T (&k)[3], cplx<T> (&s)[6]) {
  const T kk = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
  if (kk == T(0)) {
#pragma unroll
    for (int I = 0; I < 6; ++I) s[I] = cplx<T>{T(0), T(0)};
    return 0.0;
  }
  // v = sigma k
  cplx<T> v[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    v[i] = k[0] * s[voigt(i, 0)] + k[1] * s[voigt(i, 1)] + k[2] * s[voigt(i, 2)];
  }
  const double res = (double)norm2(v[0]) + (double)norm2(v[1]) + (double)norm2(v[2]);
  const T inv = recip(kk);
  const cplx<T> kv = k[0] * v[0] + k[1] * v[1] + k[2] * v[2];
  const T a1 = -g.c1 * inv * g.scale;                  // -(1/mu0)/|k|^2
  const cplx<T> a2 = (g.c2 * inv * inv * g.scale) * kv;  // +c2 (k.v)/|k|^4
#pragma unroll
  for (int I = 0; I < 6; ++I) {
    const int i = vi(I), j = vj(I);
    cplx<T> sy = T(0.5) * (k[i] * v[j] + k[j] * v[i]);
    s[I] = a1 * sy + (k[i] * k[j]) * a2;
  }
  return res;
}

template <typename T> __device__ __forceinline__ cplx<T> cdiv(cplx<T> a, cplx<T> b) {
  const T r = recip(b.x * b.x + b.y * b.y);
  return cplx<T>{(a.x * b.x + a.y * b.y) * r, (a.y * b.x - a.x * b.y) * r};
}

// FB Green step with complex a = q^a, q^b = conj(a).
template <typename T>
__device__ __forceinline__ double green_fb(const GreenParams<T> &g, const cplx<T> (&a)[3], cplx<T> (&s)[6]) {
  const T aa = norm2(a[0]) + norm2(a[1]) + norm2(a[2]);
  if (aa == T(0)) {
#pragma unroll
    for (int I = 0; I < 6; ++I) s[I] = cplx<T>{T(0), T(0)};
    return 0.0;
  }
  cplx<T> v[3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
    v[i] = s[voigt(i, 0)] * conjg(a[0]) + s[voigt(i, 1)] * conjg(a[1]) + s[voigt(i, 2)] * conjg(a[2]);
  const double res = (double)norm2(v[0]) + (double)norm2(v[1]) + (double)norm2(v[2]);
  // K_ij = mu |a|^2 d_ij + mu a_i conj(a_j) + lam conj(a_i) a_j
  cplx<T> K[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cplx<T> e = g.mu0 * (a[i] * conjg(a[j])) + g.lam0 * (conjg(a[i]) * a[j]);
      if (i == j) e.x += g.mu0 * aa;
      K[i][j] = e;
    }
  // w = K^{-1} v by cofactors
  const cplx<T> c00 = K[1][1] * K[2][2] - K[1][2] * K[2][1];
  const cplx<T> c01 = K[1][2] * K[2][0] - K[1][0] * K[2][2];
  const cplx<T> c02 = K[1][0] * K[2][1] - K[1][1] * K[2][0];
  const cplx<T> det = K[0][0] * c00 + K[0][1] * c01 + K[0][2] * c02;
  cplx<T> adj[3][3];
  adj[0][0] = c00;
  adj[1][0] = c01;
  adj[2][0] = c02;
  adj[0][1] = K[0][2] * K[2][1] - K[0][1] * K[2][2];
  adj[1][1] = K[0][0] * K[2][2] - K[0][2] * K[2][0];
  adj[2][1] = K[0][1] * K[2][0] - K[0][0] * K[2][1];
  adj[0][2] = K[0][1] * K[1][2] - K[0][2] * K[1][1];
  adj[1][2] = K[0][2] * K[1][0] - K[0][0] * K[1][2];
  adj[2][2] = K[0][0] * K[1][1] - K[0][1] * K[1][0];
  cplx<T> w[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) w[i] = cdiv(adj[i][0] * v[0] + adj[i][1] * v[1] + adj[i][2] * v[2], det);
  const T sc = -g.scale;
#pragma unroll
  for (int I = 0; I < 6; ++I) {
    const int i = vi(I), j = vj(I);
    s[I] = (T(0.5) * sc) * (w[i] * a[j] + w[j] * a[i]);
  }
  return res;
}

// DGO step from the 21 coefficients at this frequency.
template <typename T>
__device__ __forceinline__ void green_dgo(const GreenParams<T> &g, const T *coef, long long cstride,
                                          cplx<T> (&s)[6]) {
  T P[6], Q[15];
#pragma unroll
  for (int I = 0; I < 6; ++I) P[I] = coef[I * cstride];
#pragma unroll
  for (int I = 0; I < 15; ++I) Q[I] = coef[(6 + I) * cstride];
  cplx<T> out[6];
#pragma unroll
  for (int I = 0; I < 6; ++I) {
    const int i = vi(I), j = vj(I);
    // sym(tau P)_ij = 1/2 sum_k (tau_ik P_kj + P_ik tau_kj)
    cplx<T> sp{T(0), T(0)};
#pragma unroll
    for (int k = 0; k < 3; ++k) sp = sp + P[voigt(k, j)] * s[voigt(i, k)] + P[voigt(i, k)] * s[voigt(k, j)];
    sp = T(0.5) * sp;
    // (Q : tau)_ij = sum_kl Q_ijkl tau_kl
    cplx<T> qt{T(0), T(0)};
#pragma unroll
    for (int J = 0; J < 6; ++J) {
      const int k = vi(J), l = vj(J);
      const T m = (k == l) ? T(1) : T(2);
      qt = qt + (m * Q[qidx4(i, j, k, l)]) * s[J];
    }
    out[I] = (-g.scale) * (g.c1 * sp - g.c2 * qt);
  }
#pragma unroll
  for (int I = 0; I < 6; ++I) s[I] = out[I];
}

// The two per-axis table values a Green step needs at axis index i:
// (sin, cos) for AFB, (Re, Im) of the FB symbol, the plain wavenumber for
// BASIC.  Kernels load them together with their data, before the transforms,
// so that the Green step itself reads registers only; the table kinds are
// chosen arithmetically (no branch has to merge a load result).
template <typename T> struct AxisVal {
  T p, q;
};
template <typename T> __device__ __forceinline__ AxisVal<T> axis_val(const GreenParams<T> &g, int axis, int i) {
  const int kp = g.scheme == SCHEME_AFB ? TAB_SH
               : g.scheme == SCHEME_FB  ? TAB_AR
               : (g.scheme == SCHEME_CD || g.scheme == SCHEME_ACD) ? TAB_AI : TAB_K;
  const int kq = g.scheme == SCHEME_AFB ? TAB_C
               : (g.scheme == SCHEME_FB || g.scheme == SCHEME_CD) ? TAB_AI
               : g.scheme == SCHEME_ACD ? TAB_C2 : TAB_K;
  return AxisVal<T>{tabv(g, kp, axis, i), tabv(g, kq, axis, i)};
}

// The values of every index of `axis` staged in LDS by the workgroup; a
// barrier of the caller publishes them.  Read back at each transform point
// instead of being held in registers from the start of the kernel.
#ifndef LSFFT_LDS_AXIS
#define LSFFT_LDS_AXIS 1
#endif
template <typename T, int NA>
__device__ __forceinline__ void stage_axis(AxisVal<T> (&dst)[NA], const GreenParams<T> &g, int axis) {
  for (int i = threadIdx.x; i < NA; i += blockDim.x) dst[i] = axis_val(g, axis, i);
}

// Dispatch on the scheme for spectrum indices (i1, i2, i3), i1 in [0, n1/2],
// with the per-axis table values ax[r] = axis_val(g, r, idx[r]).
template <typename T>
__device__ __forceinline__ double green_point(const GreenParams<T> &g, int i1, int i2, int i3,
                                              const AxisVal<T> (&ax)[3], cplx<T> (&s)[6]) {
  const int idx[3] = {i1, i2, i3};
  if (g.scheme == SCHEME_DGO) {
    if (i1 == 0 && i2 == 0 && i3 == 0) {
#pragma unroll
      for (int I = 0; I < 6; ++I) s[I] = cplx<T>{T(0), T(0)};
      return 0.0;
    }
    const int L = g.n[0] / 2;
    if (i1 < L) {
      const long long f = ((long long)i3 * g.n[1] + i2) * L + i1;
      green_dgo(g, g.dgo_main + f, g.dgo_main_stride, s);
    } else {
      const long long f = (long long)i3 * g.n[1] + i2;
      green_dgo(g, g.dgo_nyq + f, g.dgo_nyq_stride, s);
    }
    return 0.0;
  }
  if (g.scheme == SCHEME_FB) {
    cplx<T> a[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) a[r] = cplx<T>{ax[r].p, ax[r].q};
    return green_fb(g, a, s);
  }
  T k[3];
  if (g.scheme == SCHEME_AFB || g.scheme == SCHEME_ACD) {
    // a per-axis difference times the averaging factors of the other axes
    k[0] = ax[0].p * ax[1].q * ax[2].q;
    k[1] = ax[1].p * ax[2].q * ax[0].q;
    k[2] = ax[2].p * ax[0].q * ax[1].q;
  } else if (g.scheme == SCHEME_CD) {
#pragma unroll
    for (int r = 0; r < 3; ++r) k[r] = ax[r].p;
  } else {
    bool nyq[3];
    bool live = false;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      k[r] = ax[r].p;
      nyq[r] = (2 * idx[r] == g.n[r]);
      live = live || (!nyq[r] && k[r] != T(0));
    }
    if (live) {
#pragma unroll
      for (int r = 0; r < 3; ++r)
        if (nyq[r]) k[r] = T(0);
    }
  }
  return green_real(g, k, s);
}

// A scheme fixed at compile time (SCH >= 0: only AFB is specialised) or
// taken from g (SCH < 0): the table values and the Green step of that scheme.
template <int SCH, typename T> __device__ __forceinline__ AxisVal<T> axis_val_s(const GreenParams<T> &g, int axis, int i) {
  if constexpr (SCH == SCHEME_AFB)
    return AxisVal<T>{tabv(g, TAB_SH, axis, i), tabv(g, TAB_C, axis, i)};
  else
    return axis_val(g, axis, i);
}
template <int SCH, typename T>
__device__ __forceinline__ double green_point_s(const GreenParams<T> &g, int i1, int i2, int i3,
                                                const AxisVal<T> (&ax)[3], cplx<T> (&s)[6]) {
  if constexpr (SCH == SCHEME_AFB) {
    const T k[3] = {ax[0].p * ax[1].q * ax[2].q, ax[1].p * ax[2].q * ax[0].q, ax[2].p * ax[0].q * ax[1].q};
    return green_real(g, k, s);
  } else {
    return green_point(g, i1, i2, i3, ax, s);
  }
}

// The same, loading the table values itself.
template <typename T>
__device__ __forceinline__ double green_point(const GreenParams<T> &g, int i1, int i2, int i3, cplx<T> (&s)[6]) {
  const AxisVal<T> ax[3] = {axis_val(g, 0, i1), axis_val(g, 1, i2), axis_val(g, 2, i3)};
  return green_point(g, i1, i2, i3, ax, s);
}

}  // namespace lsfft
