// Displacement form of the TD algorithm of Sec. 5.2 for the FB and AFB
// schemes, with the finite-difference operators applied as real-space
// stencils.  One iteration:
//
//   k_uxpass    u += IDFT(Delta u_hat)            (x-lines, three components)
//   k_stencil   eps = Ebar + sym(grad^a u)  at the cells,   sigma = C : eps,
//               f = div^b sigma  at the nodes,  f_hat_x = forward x transform
//   k_ypass     forward y (three components)
//   k_zpass_u   Delta u_hat = K(q)^{-1} f_hat (x) / N,  forward + inverse z
//   k_ypass     inverse y
//
// AFB: grad^a = the average forward difference over the eight corners of a
// cell (eq. (36) carried to 3D, symbol q^AFD of eq. (43)); div^b = the
// average backward difference over the eight cells around a node (symbol
// q^ABD).  Because q^AFD = Phi q^AhC and q^ABD = conj(Phi) q^AhC with one
// scalar phase Phi, G(q^AFD, q^AhC) sigma_hat q^AhC = K(k)^{-1} sigma_hat q^ABD,
// K(k) = mu0 |k|^2 I + (lam0 + mu0) k (x) k at the rotated wavevector k
// (eq. (34)): these are exactly the iterates of the (AFD, AhC) algorithm.
// FB: grad^a = forward difference, div^b = backward difference (q^b =
// conj(q^FD) = -q^BD), K = mu0 |a|^2 I + mu0 a (x) conj(a) + lam0 conj(a) (x) a.
// The equilibrium residual needs no spectrum: sum_xi |sigma_hat q^b|^2 =
// N sum_x |f(x)|^2 (Parseval), accumulated in FP64 by k_stencil.
//
// Precision: u is stored and accumulated in FP64 whatever the solver
// precision T.  u grows like |eps| n h, so a T-rounded u would lose about
// log2(n) bits of the strain taken from its differences, and that rounding
// would build up over the iterations.  The stencils take exact FP64
// differences of neighbouring nodes and round those to T (the LDS variant
// forms the whole gradient in FP64); sigma, f, the transforms and the Green
// step run in T, with rounding relative to the strain and stress themselves.
#pragma once
#include <type_traits>

#include "kernels.hpp"

namespace lsfft {

// Delta u_hat = K^{-1} f_hat * scale at one frequency, with the per-axis
// table values ax[r] = axis_val(g, r, index_r).  The scheme (FB or AFB) is a
// template parameter: the FB inverse of a Hermitian 3 x 3 needs far more
// registers than the AFB closed form, and a kernel is sized for its
// heaviest path.
template <int SCH, typename T>
__device__ __forceinline__ void green_disp_point(const GreenParams<T> &g, const AxisVal<T> (&ax)[3],
                                                 cplx<T> (&f)[3]) {
  static_assert(SCH == SCHEME_FB || SCH == SCHEME_AFB, "displacement form: FB or AFB");
  if constexpr (SCH == SCHEME_FB) {
    cplx<T> a[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) a[r] = cplx<T>{ax[r].p, ax[r].q};
    const T aa = norm2(a[0]) + norm2(a[1]) + norm2(a[2]);
    if (aa == T(0)) {
#pragma unroll
      for (int i = 0; i < 3; ++i) f[i] = cplx<T>{T(0), T(0)};
      return;
    }
    cplx<T> K[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        cplx<T> e = g.mu0 * (a[i] * conjg(a[j])) + g.lam0 * (conjg(a[i]) * a[j]);
        if (i == j) e.x += g.mu0 * aa;
        K[i][j] = e;
      }
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
    for (int i = 0; i < 3; ++i)
      w[i] = g.scale * cdiv(adj[i][0] * f[0] + adj[i][1] * f[1] + adj[i][2] * f[2], det);
#pragma unroll
    for (int i = 0; i < 3; ++i) f[i] = w[i];
    return;
  }
  // AFB: rotated wavevector
  T k[3];
  k[0] = ax[0].p * ax[1].q * ax[2].q;
  k[1] = ax[1].p * ax[2].q * ax[0].q;
  k[2] = ax[2].p * ax[0].q * ax[1].q;
  const T kk = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
  if (kk == T(0)) {
#pragma unroll
    for (int i = 0; i < 3; ++i) f[i] = cplx<T>{T(0), T(0)};
    return;
  }
  // K^{-1} = (1 / (mu0 |k|^2)) [I - beta k (x) k / |k|^2],  beta = (lam0+mu0)/(lam0+2mu0)
  const T inv = recip(kk);
  const T a1 = g.c1 * inv * g.scale;
  const cplx<T> kf = k[0] * f[0] + k[1] * f[1] + k[2] * f[2];
  const cplx<T> a2 = (g.beta * inv) * kf;
#pragma unroll
  for (int i = 0; i < 3; ++i) f[i] = a1 * (f[i] - k[i] * a2);
}

// ---------------------------------------------------------------- u update (x-lines)
template <typename T> struct UArgs {
  Dims d;
  double *u;          // [system][3][n3][n2][n1], FP64 whatever T
  const cplx<T> *spec;
  const cplx<T> *nyq;
  const cplx<T> *tw;  // exp(-2 pi i m / n1)
  const State *st;    // [system]
  Strides bs;
};

template <typename T, int L, int E, int WG>
__global__ __launch_bounds__(WG) void k_uxpass(UArgs<T> a) {
  const int sysb = blockIdx.y;
  if (a.st && a.st[sysb].done) return;
  a.u += sysb * 3 * a.bs.field;
  a.spec += sysb * a.bs.spec;
  a.nyq += sysb * a.bs.nyq;
  __shared__ cplx<T> twl_[2 * L];
  constexpr int TPC = L / E;
  constexpr int P = lines_per_wg(TPC, WG);
  __shared__ cplx<T> lds[line_slots<TPC, WG>() * line_scratch<L>()];
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
  const cplx<T> zero{T(0), T(0)};
  cplx<T> w[3][E];
  cplx<T> xn[3];
  double uo[3][E][2];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cplx<T> *src = a.spec + ((long long)c * a.d.rows + row) * L;
#pragma unroll
    for (int e = 0; e < E; ++e) w[c][e] = valid ? ldc_nt(src + t + TPC * e) : zero;
    xn[c] = (valid && t == 0) ? a.nyq[(long long)c * a.d.rows + row] : zero;
  }
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const long long idx = row * n1 + 2 * (t + TPC * e);
      if (valid) ld2_nt(a.u + c * N + idx, uo[c][e][0], uo[c][e][1]);
      else uo[c][e][0] = uo[c][e][1] = 0.0;
    }
  const cplx<T> *twl = stage_twiddles(twl_, a.tw);
#pragma unroll
  for (int c = 0; c < 3; ++c) c2r_line<T, L, E>(w[c], xn[c], t, lane, sl, twl, buf);
  if (valid) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const long long idx = row * n1 + 2 * (t + TPC * e);
        st2_nt(a.u + c * N + idx, uo[c][e][0] + (double)w[c][e].x, uo[c][e][1] + (double)w[c][e].y);
      }
  }
}

// ---------------------------------------------------------------- stencil kernel
// One workgroup owns output node lines y in [y0, y0 + T2) for planes
// z in [z0, z0 + Z) and marches along z.  LDS holds two u planes over the
// node lines [y0-1, y0+T2], two sigma planes over the cell lines
// [y0-1, y0+T2), and the divergence f of the current plane (u planes in
// FP64, sigma and f in T).  A cell (c1, c2, c3)
// has corners (c1..c1+1, c2..c2+1, c3..c3+1); node n gathers the cells
// n - {0,1}^3 (all indices periodic).
template <typename T> struct SArgs {
  Dims d;
  const double *u;     // FP64 displacement [system][3][N]
  const T *lam;        // [system][N]
  const T *mu;
  cplx<T> *spec;
  cplx<T> *nyq;
  const cplx<T> *tw;   // exp(-2 pi i m / n1)
  const Member<T> *mem;  // Ebar, h_j Ebar_ij of each system
  Strides bs;
  double ihu[3];       // 1 / h_r for the FP64 gradient
  T ih[3];             // 1 / h_r for the divergence
  double *partial;     // [system][gridDim.x][8]: 6 stress sums, sum |f|^2
  const State *st;     // [system]
  const T *fstar;      // div sigma_* of the eigenstress at the nodes [system][3][N], or null
  ReduceArgs red;      // the iteration's reduction and stop test ...
  unsigned *counter;   // ... taken by the last workgroup: arrivals [system], or null (no reduction)
  int Z;               // planes per workgroup
  int xcd;             // 1: XCD-aware order of the tiles
  int zero_u;          // u is identically zero (first pass): the LDS variant skips its loads
  float *raw;          // FP64 register stencil only: store -f here [system][3][N] instead of transforming
                       // (the FP64 residual force of a refinement cycle), or null
};

// Offset the per-system pointers of stencil arguments to system b.
template <typename T> __device__ __forceinline__ void stencil_member(SArgs<T> &a, int b) {
  a.u += b * 3 * a.bs.field;
  a.lam += b * a.bs.field;
  a.mu += b * a.bs.field;
  a.spec += b * a.bs.spec;
  a.nyq += b * a.bs.nyq;
  if (a.partial) a.partial += b * a.bs.part;
  if (a.fstar) a.fstar += b * 3 * a.bs.field;
  if (a.raw) a.raw += b * 3 * a.bs.field;
}

template <int SCHEME> struct Stencil;

// Tile of a stencil workgroup: y-blocks fastest, then z-blocks.  In the
// XCD-aware order each XCD takes a contiguous range of tiles, so workgroups
// marching neighbouring y-blocks side by side share their halo lines in that
// XCD's L2.
__device__ __forceinline__ int stencil_tile(int xcd) { return (int)tile_of(blockIdx.x, gridDim.x, xcd); }

// Average forward difference over the cell, eq. (36) carried to 3D.
template <> struct Stencil<SCHEME_AFB> {
  template <typename T>
  __device__ __forceinline__ static void grad(const T (&c)[2][2][2], const T (&ih)[3], T (&gr)[3]) {
    // c[a][b][d]: value at corner offsets (x a, y b, z d)
    gr[0] = T(0.25) * ih[0] * ((c[1][0][0] - c[0][0][0]) + (c[1][1][0] - c[0][1][0]) + (c[1][0][1] - c[0][0][1]) +
                               (c[1][1][1] - c[0][1][1]));
    gr[1] = T(0.25) * ih[1] * ((c[0][1][0] - c[0][0][0]) + (c[1][1][0] - c[1][0][0]) + (c[0][1][1] - c[0][0][1]) +
                               (c[1][1][1] - c[1][0][1]));
    gr[2] = T(0.25) * ih[2] * ((c[0][0][1] - c[0][0][0]) + (c[1][0][1] - c[1][0][0]) + (c[0][1][1] - c[0][1][0]) +
                               (c[1][1][1] - c[1][1][0]));
  }
  // s[a][b][d]: value at the cell node - (a, b, d); returns the average
  // backward difference of component direction r.
  template <typename T>
  __device__ __forceinline__ static T div(const T (&s)[2][2][2], int r, const T (&ih)[3]) {
    if (r == 0)
      return T(0.25) * ih[0] * ((s[0][0][0] - s[1][0][0]) + (s[0][1][0] - s[1][1][0]) + (s[0][0][1] - s[1][0][1]) +
                                (s[0][1][1] - s[1][1][1]));
    if (r == 1)
      return T(0.25) * ih[1] * ((s[0][0][0] - s[0][1][0]) + (s[1][0][0] - s[1][1][0]) + (s[0][0][1] - s[0][1][1]) +
                                (s[1][0][1] - s[1][1][1]));
    return T(0.25) * ih[2] * ((s[0][0][0] - s[0][0][1]) + (s[1][0][0] - s[1][0][1]) + (s[0][1][0] - s[0][1][1]) +
                              (s[1][1][0] - s[1][1][1]));
  }
};

// The same AFB gradient from edge differences of the cell (x, l) between
// planes z (a) and z+1 (b): dx = u(x+1) - u(x) on lines l, l+1 of each plane,
// dy = u(l+1) - u(l) of the own column on each plane, dz = u(z+1) - u(z) of
// the own column on lines l, l+1.  The neighbour column's y and z
// differences follow from dy(x+1) = dy + dx(l+1) - dx(l) and dz(x+1) =
// dz + dx_b - dx_a, so no FP64 corner value is needed once the exact
// differences are taken.  The identities hold as well for differences of the
// total displacement u + Ebar x.
template <typename T>
__device__ __forceinline__ void afb_grad_edges(T dxa0, T dxa1, T dxb0, T dxb1, T dya, T dyb, T dz0, T dz1,
                                               const T (&ih)[3], T (&gr)[3]) {
  gr[0] = T(0.25) * ih[0] * ((dxa0 + dxa1) + (dxb0 + dxb1));
  gr[1] = T(0.25) * ih[1] * (T(2) * (dya + dyb) + ((dxa1 - dxa0) + (dxb1 - dxb0)));
  gr[2] = T(0.25) * ih[2] * (T(2) * (dz0 + dz1) + ((dxb0 - dxa0) + (dxb1 - dxa1)));
}

// Forward difference (gradient) / backward difference (divergence).
template <> struct Stencil<SCHEME_FB> {
  template <typename T>
  __device__ __forceinline__ static void grad(const T (&c)[2][2][2], const T (&ih)[3], T (&gr)[3]) {
    gr[0] = ih[0] * (c[1][0][0] - c[0][0][0]);
    gr[1] = ih[1] * (c[0][1][0] - c[0][0][0]);
    gr[2] = ih[2] * (c[0][0][1] - c[0][0][0]);
  }
  template <typename T>
  __device__ __forceinline__ static T div(const T (&s)[2][2][2], int r, const T (&ih)[3]) {
    if (r == 0) return ih[0] * (s[0][0][0] - s[1][0][0]);
    if (r == 1) return ih[1] * (s[0][0][0] - s[0][1][0]);
    return ih[2] * (s[0][0][0] - s[0][0][1]);
  }
};

// eps = Ebar + sym(gr) and sigma = lam tr(eps) I + 2 mu eps (Voigt order,
// tensor components), all in FP64.
__device__ __forceinline__ void cell_stress(const double (&Eb)[6], const double (&gr)[3][3], double lm, double m2,
                                            double (&sg)[6]) {
  double e[6];
  e[0] = Eb[0] + gr[0][0];
  e[1] = Eb[1] + gr[1][1];
  e[2] = Eb[2] + gr[2][2];
  e[3] = Eb[3] + 0.5 * (gr[1][2] + gr[2][1]);
  e[4] = Eb[4] + 0.5 * (gr[0][2] + gr[2][0]);
  e[5] = Eb[5] + 0.5 * (gr[0][1] + gr[1][0]);
  const double tr = e[0] + e[1] + e[2];
#pragma unroll
  for (int c = 0; c < 6; ++c) sg[c] = (c < 3 ? lm * tr : 0.0) + m2 * e[c];
}

template <typename T, int N1, int E, int SCHEME, int T2>
__global__ __launch_bounds__(256) void k_stencil(SArgs<T> a) {
  const int sysb = blockIdx.y;
  if (a.st && a.st[sysb].done) return;
  stencil_member(a, sysb);
  double Ebl[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) Ebl[c] = a.mem[sysb].Eb[c];
  constexpr int WG = 256;
  constexpr int L = N1 / 2;
  constexpr int TPC = L / E;
  constexpr int NUL = T2 + 2;   // node lines of u
  constexpr int NSL = T2 + 1;   // cell lines of sigma
  constexpr int UPL = NUL * 3 * N1;
  constexpr int SPL = NSL * 6 * N1;
  constexpr int NLW = lines_per_wg(TPC, WG);
  static_assert(T2 * 3 <= NLW, "x transforms of the workgroup's f lines do not fit");
  static_assert((T2 * 3 + 1) * line_scratch<L>() * 2 <= SPL, "transform scratch must fit in one sigma plane");
  __shared__ double U[2 * UPL];
  __shared__ T S[2 * SPL];
  __shared__ T F[T2 * 3 * N1];
  __shared__ double red[(WG + 63) / 64 * 8];
  const int tid = threadIdx.x;
  const int n2 = a.d.n2, n3 = a.d.n3;
  const long long N = a.d.N;
  const int ny_blocks = n2 / T2;
  const int tile = stencil_tile(a.xcd);
  const int y0 = (tile % ny_blocks) * T2;
  const int z0 = (tile / ny_blocks) * a.Z;
  const T ih[3] = {a.ih[0], a.ih[1], a.ih[2]};
  const double ihu[3] = {a.ihu[0], a.ihu[1], a.ihu[2]};
  double sums[8] = {0, 0, 0, 0, 0, 0, 0, 0};

  // Software pipeline: the u plane z+2 and the moduli of cell plane z+1 are
  // loaded into registers while plane z is computed, then stored to LDS /
  // used at the next step.
  constexpr int UQ = (UPL + WG - 1) / WG;          // u values per thread per plane
  constexpr int CQ = (NSL * N1 + WG - 1) / WG;     // cells per thread per plane
  double ureg[UQ];
  T lreg[CQ], mreg[CQ];
  auto fetch_u = [&](int zz) {
    const int zg = ((zz % n3) + n3) % n3;
#pragma unroll
    for (int j = 0; j < UQ; ++j) {
      const int q = tid + WG * j;
      double v = 0.0;
      if (q < UPL && !a.zero_u) {
        const int x = q % N1;
        const int lc = q / N1;  // line * 3 + comp
        const int l = lc / 3, c = lc % 3;
        const int yg = ((y0 - 1 + l) % n2 + n2) % n2;
        v = a.u[c * N + ((long long)zg * n2 + yg) * N1 + x];
      }
      ureg[j] = v;
    }
  };
  auto stash_u = [&](int pb) {
#pragma unroll
    for (int j = 0; j < UQ; ++j) {
      const int q = tid + WG * j;
      if (q < UPL) U[pb * UPL + q] = ureg[j];
    }
  };
  auto fetch_lm = [&](int zz) {
    const int zg = ((zz % n3) + n3) % n3;
#pragma unroll
    for (int j = 0; j < CQ; ++j) {
      const int q = tid + WG * j;
      if (q < NSL * N1) {
        const int x = q % N1, l = q / N1;
        const int yg = ((y0 - 1 + l) % n2 + n2) % n2;
        const long long gi = ((long long)zg * n2 + yg) * N1 + x;
        lreg[j] = a.lam[gi];
        mreg[j] = a.mu[gi];
      }
    }
  };

  fetch_u(z0 - 1);
  stash_u((z0 - 1) & 1);
  fetch_u(z0);
  fetch_lm(z0 - 1);
  for (int z = z0 - 1; z < z0 + a.Z; ++z) {
    stash_u((z + 1) & 1);
    T lcur[CQ], mcur[CQ];
#pragma unroll
    for (int j = 0; j < CQ; ++j) {
      lcur[j] = lreg[j];
      mcur[j] = mreg[j];
    }
    if (z + 2 <= z0 + a.Z) fetch_u(z + 2);
    if (z + 1 < z0 + a.Z) fetch_lm(z + 1);
    __syncthreads();
    // ---- sigma at the cells of plane c3 = z, cell lines [y0-1, y0+T2)
    {
      const double *U0 = U + (z & 1) * UPL;        // nodes at plane z
      const double *U1 = U + ((z + 1) & 1) * UPL;  // nodes at plane z + 1
      T *Sp = S + (z & 1) * SPL;
#pragma unroll
      for (int j = 0; j < CQ; ++j) {
        const int q = tid + WG * j;
        if (q >= NSL * N1) break;
        const int x = q % N1, l = q / N1;
        const int x1 = (x + 1) % N1;
        const double lm = (double)lcur[j], m2 = 2.0 * (double)mcur[j];
        double gr[3][3];  // gr[i][j] = d u_i / d x_j
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          double cv[2][2][2];
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            const int base = ((l + b) * 3 + c) * N1;
            cv[0][b][0] = U0[base + x];
            cv[1][b][0] = U0[base + x1];
            cv[0][b][1] = U1[base + x];
            cv[1][b][1] = U1[base + x1];
          }
          Stencil<SCHEME>::grad(cv, ihu, gr[c]);
        }
        double sg[6];
        cell_stress(Ebl, gr, lm, m2, sg);
#pragma unroll
        for (int c = 0; c < 6; ++c) Sp[(l * 6 + c) * N1 + x] = (T)sg[c];
        if (l >= 1 && z >= z0) {
#pragma unroll
          for (int c = 0; c < 6; ++c) sums[c] += sg[c];
        }
      }
    }
    __syncthreads();
    if (z < z0) continue;
    // ---- f = div sigma at the nodes of plane z, node lines [y0, y0+T2)
    {
      const T *S1 = S + (z & 1) * SPL;        // cells at c3 = z
      const T *S0 = S + ((z - 1) & 1) * SPL;  // cells at c3 = z - 1
      for (int q = tid; q < T2 * N1; q += WG) {
        const int x = q % N1, m = q / N1;
        const int xm = (x + N1 - 1) % N1;
        // cell lines: node line m (y0 + m) gathers cell lines y0 + m (l = m + 1) and y0 + m - 1 (l = m)
        T f3[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          T acc = T(0);
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            const int c = voigt(i, j);
            T s[2][2][2];
#pragma unroll
            for (int b = 0; b < 2; ++b) {
              const int base = ((m + 1 - b) * 6 + c) * N1;
              s[0][b][0] = S1[base + x];
              s[1][b][0] = S1[base + xm];
              s[0][b][1] = S0[base + x];
              s[1][b][1] = S0[base + xm];
            }
            acc += Stencil<SCHEME>::div(s, j, ih);
          }
          // eigenstrain: the force of the eigenstress, T = C [E - E_*]
          if (a.fstar) acc -= a.fstar[i * N + ((long long)(z % n3) * n2 + y0 + m) * N1 + x];
          f3[i] = acc;
          F[(m * 3 + i) * N1 + x] = acc;
        }
        sums[6] += (double)f3[0] * f3[0] + (double)f3[1] * f3[1] + (double)f3[2] * f3[2];
      }
    }
    __syncthreads();
    // ---- forward x transforms of the T2 x 3 f lines; scratch in the free sigma plane
    {
      int pid, t;
      bool live;
      line_of<TPC, NLW>(tid, pid, t, live);
      const bool act = live && pid < T2 * 3;
      const int m = act ? pid / 3 : 0, c = act ? pid % 3 : 0;
      cplx<T> v[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int xx = 2 * (t + TPC * e);
        v[e] = act ? cplx<T>{F[(m * 3 + c) * N1 + xx], F[(m * 3 + c) * N1 + xx + 1]} : cplx<T>{T(0), T(0)};
      }
      // idle threads share one dummy scratch area past the T2 x 3 lines
      cplx<T> *scr =
          reinterpret_cast<cplx<T> *>(S + ((z - 1) & 1) * SPL) + (act ? pid : T2 * 3) * line_scratch<L>();
      int buf = 0;
      const cplx<T> xnq = r2c_line<T, L, E, false>(v, t, tid & 63, scr, a.tw, buf);  // twice the spectrum
      if (act) {
        const int zg = z % n3;
        const long long row = (long long)zg * n2 + (y0 + m);
        cplx<T> *dst = a.spec + ((long long)c * a.d.rows + row) * L;
#pragma unroll
        for (int e = 0; e < E; ++e) dst[t + TPC * e] = v[e];
        if (t == 0) a.nyq[(long long)c * a.d.rows + row] = xnq;
      }
    }
  }
  if (a.partial) {
    block_sum<WG>(sums, 7, red);
    if (tid == 0) {
      double *dst = a.partial + (long long)blockIdx.x * 8;
      sums[7] = 0.0;
      if (a.counter)
        store_row_coherent(dst, sums, 8);  // read by the last workgroup of this launch
      else
        for (int i = 0; i < 8; ++i) dst[i] = sums[i];
    }
  }
  if (a.counter) last_block_reduce<WG>(a.red, a.counter, sysb, red);
}

// Register-resident variant for n1 = 2^a or 3 * 2^a: every thread owns one
// x column of one y-group and keeps its own displacement planes, edge
// differences and sigma planes in registers; LDS only carries the column
// exchange with the x +- 1 neighbours, the two parts of the divergence and
// the transform scratch.  The workgroup has WG = 256 threads for a
// power-of-two n1 up to 256, 192 for 3 * 2^a up to 192, the most whole
// y-groups that fit in 256 threads for lengths with a factor 9 (e.g. 252 at
// 36 columns, 144 at 144: not always whole wavefronts), n1 threads beyond,
// and holds G = WG / n1 independent y-groups when n1 < WG.  The FP64
// u exchange is single-buffered: each plane is published once and the x
// differences it yields are kept for the next step.  Two workgroup barriers
// per plane (the u exchange, the divergence parts).  The z-march is unrolled
// by two so that the per-plane buffers alternate by name (index P = z & 1)
// instead of being copied.
#ifndef LSFFT_STENCIL_WAVES
#define LSFFT_STENCIL_WAVES 1
#endif
constexpr bool pow2_len(int n) { return n > 0 && (n & (n - 1)) == 0; }
constexpr int stencil_wg_of(int n1) {
  if (n1 % 9 == 0) return n1 >= 256 ? n1 : (256 / n1) * n1;
  const int base = pow2_len(n1) ? 256 : 192;
  return n1 > base ? n1 : base;
}
// Waves per SIMD the compiler must leave room for: two for the FP32
// 192-thread kernels up to 192 columns (the 96-column AFB one would otherwise
// take 269 registers and run one wave; two waves with a small spill are
// faster), the compiler's own choice otherwise.
template <typename T, int N1> constexpr int stencil_min_waves() {
  return (sizeof(T) == 4 && !pow2_len(N1) && N1 <= 192) ? 2 : LSFFT_STENCIL_WAVES;
}
//
// FS: the system subtracts a force at the nodes (a.fstar: the eigenstress's,
// or a refinement cycle's FP64 residual); a separate instantiation, since
// its prefetch registers would otherwise size the plain kernel.
template <typename T, int N1, int E, int SCHEME, int T2, bool FS>
__global__ __launch_bounds__(stencil_wg_of(N1), (stencil_min_waves<T, N1>())) void k_stencil_reg(SArgs<T> a) {
  const int sysb = blockIdx.y;
  if (a.st && a.st[sysb].done) return;
  stencil_member(a, sysb);
  // the system's constants in registers (a reference into global memory
  // would be reloaded after every store of the march)
  double hE[3][3];
#pragma unroll
  for (int q1 = 0; q1 < 3; ++q1)
#pragma unroll
    for (int q2 = 0; q2 < 3; ++q2) hE[q1][q2] = a.mem[sysb].hE[q1][q2];
  constexpr int WG = stencil_wg_of(N1);
  constexpr int L = N1 / 2;
  constexpr int TPC = L / E;
  constexpr int G = N1 >= WG ? 1 : WG / N1;     // y-groups per workgroup
  constexpr int XV = N1 >= WG ? N1 / WG : 1;    // x columns per thread
  constexpr int NX = N1 / XV;                    // threads per group
  constexpr int NUL = T2 + 2, NSL = T2 + 1;
  constexpr int UX = G * NUL * 3 * N1;           // the exchanged u plane (FP64)
  constexpr int NPEN = G * T2 * 3;
  constexpr int NF = NPEN * N1;                  // the two divergence parts of a plane (T)
  constexpr int SCR = NPEN * line_scratch<L>();  // transform scratch (complex T)
  static_assert(G * NX == WG, "the workgroup must split evenly into x columns");
  static_assert(TPC <= 64, "a line must fit in one wavefront");
  // Whole x-lines the workgroup's wavefronts hold (64 / TPC per wavefront, a
  // partial last wavefront included) and the rounds of line transforms a
  // plane takes: one, except on some lengths with a factor 9.
  constexpr int NLW = (WG / 64) * (64 / TPC) + (WG % 64) / TPC;
  constexpr int ROUNDS = (NPEN + NLW - 1) / NLW;
  __shared__ double Ux[UX];
  __shared__ T Fv[NF];  // f_i's part from the own column, at x
  __shared__ T Fu[NF];  // f_i's part that column x takes from column x-1, at x
  __shared__ cplx<T> Scr[SCR];
  __shared__ cplx<T> twl[N1];   // the x twiddles, read by every transform below
  __shared__ double red[(WG + 63) / 64 * 8];
  const int tid = threadIdx.x;
  const int n2 = a.d.n2, n3 = a.d.n3;
  const long long N = a.d.N;
  const int ny_blocks = (n2 + G * T2 - 1) / (G * T2);
  const int tile = stencil_tile(a.xcd);
  if (a.tw)
    for (int i = tid; i < N1; i += WG) twl[i] = a.tw[i];
  const int g = tid / NX, xt = tid % NX;
  const int yg0 = (tile % ny_blocks) * G * T2 + g * T2;
  const bool gvalid = yg0 < n2;
  const int z0 = (tile / ny_blocks) * a.Z;
  // quarter inverse spacings: every AFB difference is an average of four edges
  const T q[3] = {T(0.25) * a.ih[0], T(0.25) * a.ih[1], T(0.25) * a.ih[2]};
  const T ih[3] = {a.ih[0], a.ih[1], a.ih[2]};
  double sums[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  T acc0[6];  // the even step's stress sums of a loop pass
  static_assert(XV == 1, "one x column per thread");
  // Wave priorities (FP32, two workgroups per CU): a step's loads, exchange
  // and FP64 differences first, then its stresses and divergence parts, its
  // line transforms last, so that a workgroup's latency-bound transforms
  // fill the other's issue gaps instead of competing with its arithmetic
  // (the FP64 stencil, one wave per SIMD at 256 columns, measured no gain).
  constexpr bool PRIO = sizeof(T) == 4;

  // Per-plane buffers indexed by plane parity.  u: own columns (FP64), plane
  // p in u[p & 1].  Edge differences of the TOTAL displacement u + Ebar x,
  // exact in FP64, then rounded to T (their rounding is relative to the local
  // total strain, which is small in a stiff phase, where Ebar + grad u would
  // cancel): dx[p & 1] = x differences (neighbour - own) on plane p,
  // dy[p & 1] = y differences on plane p, dz = between planes z and z+1.
  // sg[p & 1] = sigma of cell plane p; lam, mu[p & 1] = moduli of cell plane p.
  double u[2][XV][NUL][3];
  T dx[2][XV][NUL][3], dy[2][XV][NSL][3];
  T dz[XV][NUL][3];
  T sg[2][XV][NSL][6];
  T lam[2][XV][NSL], mu[2][XV][NSL];
  // Prefetches are unconditional and unselected (every index wraps, so each
  // load is in bounds; u of the first pass is zero-filled memory): a load
  // whose result had to be merged with an old register value would force a
  // wait right after it.  Groups past n2 compute on wrapped rows and store
  // nothing.  The loads go through buffer resources: the byte offset of the
  // plane and component is a scalar, the thread's column on a line a fixed
  // 32-bit register (lo8 for FP64, lo4 for T), so the march spends no vector
  // instructions on addresses.
  static_assert((long long)NX * (XV - 1) * 8 < 4096, "column offsets must fit the load's immediate");
  unsigned lo8[NUL], lo4[NSL];
#pragma unroll
  for (int l = 0; l < NUL; ++l) {
    const int yg = ((yg0 - 1 + l) % n2 + n2) % n2;
    lo8[l] = (unsigned)(yg * N1 + xt) * 8u;
    if (l < NSL) lo4[l] = (unsigned)(yg * N1 + xt) * (unsigned)sizeof(T);
  }
  const unsigned plane = (unsigned)(n2 * N1);
  const auto u_rs = buffer_of(a.u, 3 * N);
  const auto lam_rs = buffer_of(a.lam, N), mu_rs = buffer_of(a.mu, N);
  // the march reads planes z0-1 .. z0+Z+1 with z0+Z <= n3: one wrap at most
  auto zwrap = [&](int zz) { return zz < 0 ? zz + n3 : (zz >= n3 ? zz - n3 : zz); };
  auto fetch_u = [&](double (&dst)[XV][NUL][3], int zz) {
    const unsigned zg = (unsigned)zwrap(zz);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const unsigned so = (zg * plane + (unsigned)c * (unsigned)N) * 8u;
#pragma unroll
      for (int v = 0; v < XV; ++v)
#pragma unroll
        for (int l = 0; l < NUL; ++l) dst[v][l][c] = load_f64(u_rs, lo8[l] + NX * 8 * v, so);
    }
  };
  auto fetch_lm = [&](T (&dl)[XV][NSL], T (&dm)[XV][NSL], int zz) {
    const unsigned so = (unsigned)zwrap(zz) * plane * (unsigned)sizeof(T);
#pragma unroll
    for (int v = 0; v < XV; ++v)
#pragma unroll
      for (int l = 0; l < NSL; ++l) {
        dl[v][l] = load_t<T>(lam_rs, lo4[l] + NX * sizeof(T) * v, so);
        dm[v][l] = load_t<T>(mu_rs, lo4[l] + NX * sizeof(T) * v, so);
      }
  };
  auto ux_at = [&](int l, int c, int x) -> double & { return Ux[((g * NUL + l) * 3 + c) * N1 + x]; };
  auto fpart = [&](int m, int i, int x) { return ((g * T2 + m) * 3 + i) * N1 + x; };
  // y differences of plane `src`, publish it, take its x differences
  auto take_plane = [&](const double (&src)[XV][NUL][3], T (&ddx)[XV][NUL][3], T (&ddy)[XV][NSL][3]) {
#pragma unroll
    for (int v = 0; v < XV; ++v)
#pragma unroll
      for (int l = 0; l < NSL; ++l)
#pragma unroll
        for (int c = 0; c < 3; ++c) ddy[v][l][c] = (T)((src[v][l + 1][c] - src[v][l][c]) + hE[c][1]);
#pragma unroll
    for (int v = 0; v < XV; ++v)
#pragma unroll
      for (int l = 0; l < NUL; ++l)
#pragma unroll
        for (int c = 0; c < 3; ++c) ux_at(l, c, xt + NX * v) = src[v][l][c];
    __syncthreads();
#pragma unroll
    for (int v = 0; v < XV; ++v) {
      const int x1 = (xt + NX * v + 1) % N1;
#pragma unroll
      for (int l = 0; l < NUL; ++l)
#pragma unroll
        for (int c = 0; c < 3; ++c) ddx[v][l][c] = (T)((ux_at(l, c, x1) - src[v][l][c]) + hE[c][0]);
    }
  };

  // One step: sigma of cell plane z (between node planes z and z+1) and, unless
  // FIRST, f at node plane z and its x transforms.  Plane z is in u[P], plane
  // z+1 has arrived in u[P^1].
  auto step = [&](auto Pc, auto firstc, int z) {
    constexpr int P = decltype(Pc)::value, Q = P ^ 1;
    constexpr bool FIRST = decltype(firstc)::value;
#pragma unroll
    for (int v = 0; v < XV; ++v)
#pragma unroll
      for (int l = 0; l < NUL; ++l)
#pragma unroll
        for (int c = 0; c < 3; ++c) dz[v][l][c] = (T)((u[Q][v][l][c] - u[P][v][l][c]) + hE[c][2]);
    fetch_u(u[P], z + 2);
    fetch_lm(lam[Q], mu[Q], z + 1);
    // the force this plane's transforms subtract (eigenstress, or the FP64
    // residual of a refinement cycle), fetched now so that its latency
    // overlaps the step instead of stalling the transforms
    T fsv[ROUNDS][E][2];
    if constexpr (FS && !FIRST) {
      int lp, t;
      bool live;
      line_of<TPC, NLW>(tid, lp, t, live);
#pragma unroll
      for (int rd = 0; rd < ROUNDS; ++rd) {
        const int pid = rd * NLW + lp;
        if (live && lp < NLW && pid < NPEN) {
          const int pg = pid / (T2 * 3), m = (pid / 3) % T2, c = pid % 3;
          const int yrow = (tile % ny_blocks) * G * T2 + pg * T2 + m;  // groups past n2 work on wrapped rows
          const T *fs = a.fstar + c * N + ((long long)zwrap(z) * n2 + yrow % n2) * N1;
#pragma unroll
          for (int e = 0; e < E; ++e) ld2(fs + 2 * (t + TPC * e), fsv[rd][e][0], fsv[rd][e][1]);
        }
      }
    }
    // The previous step's last reads of Ux (its exchange) precede a barrier
    // of that step, its transforms' reads of Fv, Fu the one inside this
    // exchange.
    take_plane(u[Q], dx[Q], dy[Q]);
    if constexpr (PRIO) __builtin_amdgcn_s_setprio(1);
    // ---- sigma at the cells (x, lines 0..NSL-1, plane z) of this thread
#pragma unroll
    for (int v = 0; v < XV; ++v) {
      const int x = xt + NX * v;
      T gr[NSL][3][3];  // gradient of the total displacement: eps = sym(gr)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if constexpr (SCHEME == SCHEME_AFB) {
          // line sums shared by the two cells on either side of a node line
          T px[NUL], rz[NUL];
#pragma unroll
          for (int l = 0; l < NUL; ++l) {
            px[l] = dx[P][v][l][c] + dx[Q][v][l][c];
            rz[l] = T(2) * dz[v][l][c] + (dx[Q][v][l][c] - dx[P][v][l][c]);
          }
#pragma unroll
          for (int l = 0; l < NSL; ++l) {
            gr[l][c][0] = q[0] * (px[l] + px[l + 1]);
            gr[l][c][1] = q[1] * (T(2) * (dy[P][v][l][c] + dy[Q][v][l][c]) + (px[l + 1] - px[l]));
            gr[l][c][2] = q[2] * (rz[l] + rz[l + 1]);
          }
        } else {
#pragma unroll
          for (int l = 0; l < NSL; ++l) {
            gr[l][c][0] = ih[0] * dx[P][v][l][c];
            gr[l][c][1] = ih[1] * dy[P][v][l][c];
            gr[l][c][2] = ih[2] * dz[v][l][c];
          }
        }
      }
      T acc[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int l = 0; l < NSL; ++l) {
        const T lt = lam[P][v][l] * (gr[l][0][0] + gr[l][1][1] + gr[l][2][2]);
        const T m1 = mu[P][v][l];
        const T m2 = T(2) * m1;
        const T s6[6] = {lt + m2 * gr[l][0][0], lt + m2 * gr[l][1][1], lt + m2 * gr[l][2][2],
                         m1 * (gr[l][1][2] + gr[l][2][1]), m1 * (gr[l][0][2] + gr[l][2][0]),
                         m1 * (gr[l][0][1] + gr[l][1][0])};
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          sg[P][v][l][c] = s6[c];
          if (l >= 1) acc[c] += s6[c];
        }
      }
      // mean stress: the T2 owned cell lines, summed in T over the two steps
      // of a loop pass, then in FP64
      if constexpr (!FIRST) {
        if constexpr (P == 0) {
#pragma unroll
          for (int c = 0; c < 6; ++c) acc0[c] = acc[c];
        } else if (gvalid) {
#pragma unroll
          for (int c = 0; c < 6; ++c) sums[c] += (double)(acc0[c] + acc[c]);
        }
      }
    }
    if constexpr (FIRST) {
      __syncthreads();  // the exchange reads above precede the next publish
      return;
    }
    // ---- f = div sigma at the nodes (x, lines 0..T2-1, plane z).  Node line
    // m gathers cell lines m+1 and m, cell planes z (sg[P]) and z-1 (sg[Q]),
    // columns x and x-1.  Each difference operator is separable, so the part
    // of f_i that the own column contributes (fv, to Fv at x) and the part
    // the column x+1 takes from it (fu, to Fu at x+1) are formed here, and
    // the transforms below read f_i(x) = fv_i(x) - fu_i(x-1): three values
    // per node cross the column boundary instead of the six stress
    // components of two cell planes.
#pragma unroll
    for (int v = 0; v < XV; ++v) {
      const int x = xt + NX * v;
      const int x1 = (x + 1) % N1;
#pragma unroll
      for (int m = 0; m < T2; ++m) {
        T xp[3], w[3];  // x-derivative part and (y, z)-derivative part of f_i
        if constexpr (SCHEME == SCHEME_AFB) {
          // z-pair sums and differences of cell lines m, m+1, then the
          // 2 x 2 averages: S (x part), Y (y part), Z (z part)
          T S[6], Y[6], Zd[6];
#pragma unroll
          for (int c = 0; c < 6; ++c) {
            const T a0 = sg[P][v][m][c] + sg[Q][v][m][c], a1 = sg[P][v][m + 1][c] + sg[Q][v][m + 1][c];
            const T d0 = sg[P][v][m][c] - sg[Q][v][m][c], d1 = sg[P][v][m + 1][c] - sg[Q][v][m + 1][c];
            S[c] = a1 + a0;
            Y[c] = a1 - a0;
            Zd[c] = d1 + d0;
          }
          // f_0 = d1 s11 + d2 s12 + d3 s13, f_1 = d1 s12 + d2 s22 + d3 s23,
          // f_2 = d1 s13 + d2 s23 + d3 s33 (Voigt 11,22,33,23,13,12)
          xp[0] = S[0];
          xp[1] = S[5];
          xp[2] = S[4];
          w[0] = q[1] * Y[5] + q[2] * Zd[4];
          w[1] = q[1] * Y[1] + q[2] * Zd[3];
          w[2] = q[1] * Y[3] + q[2] * Zd[2];
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            Fv[fpart(m, i, x)] = q[0] * xp[i] + w[i];
            Fu[fpart(m, i, x1)] = q[0] * xp[i] - w[i];
          }
        } else {
          // backward differences: cell (x, m+1, z) minus its neighbour in x, y, z
          const T(&o)[6] = sg[P][v][m + 1];
          const T(&ym)[6] = sg[P][v][m];
          const T(&zm)[6] = sg[Q][v][m + 1];
          xp[0] = o[0];
          xp[1] = o[5];
          xp[2] = o[4];
          w[0] = ih[1] * (o[5] - ym[5]) + ih[2] * (o[4] - zm[4]);
          w[1] = ih[1] * (o[1] - ym[1]) + ih[2] * (o[3] - zm[3]);
          w[2] = ih[1] * (o[3] - ym[3]) + ih[2] * (o[2] - zm[2]);
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            Fv[fpart(m, i, x)] = ih[0] * xp[i] + w[i];
            Fu[fpart(m, i, x1)] = ih[0] * xp[i];
          }
        }
      }
    }
    __syncthreads();
    // ---- f of the G x T2 x 3 lines and their forward x transforms, each
    // line inside one wavefront (the lanes past the last whole line skip
    // them: a line's exchanges are ordered within its wavefront), in ROUNDS
    // rounds of at most NLW lines
    if constexpr (PRIO) __builtin_amdgcn_s_setprio(0);
    int lp, t;
    bool live;
    line_of<TPC, NLW>(tid, lp, t, live);
#pragma unroll
    for (int rd = 0; rd < ROUNDS; ++rd) {
      const int pid = rd * NLW + lp;
      if (!(live && lp < NLW && pid < NPEN)) continue;
      const int pg = pid / (T2 * 3), m = (pid / 3) % T2, c = pid % 3;
      const int yrow = (tile % ny_blocks) * G * T2 + pg * T2 + m;  // rows past n2 store nothing
      const int lo = ((pg * T2 + m) * 3 + c) * N1;
      cplx<T> vv[E];
      T ff = T(0);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int xx = 2 * (t + TPC * e);
        T f0 = Fv[lo + xx] - Fu[lo + xx], f1 = Fv[lo + xx + 1] - Fu[lo + xx + 1];
        if constexpr (FS) {
          f0 -= fsv[rd][e][0];
          f1 -= fsv[rd][e][1];
        }
        ff += f0 * f0 + f1 * f1;
        vv[e] = cplx<T>{f0, f1};
      }
      if constexpr (sizeof(T) == 8) {
        if (a.raw) {  // a refinement cycle's FP64 evaluation: -f in real space, rounded to FP32
          if (yrow < n2) {
            float *dst = a.raw + c * N + ((long long)zwrap(z) * n2 + yrow) * N1;
#pragma unroll
            for (int e = 0; e < E; ++e)
              *reinterpret_cast<float2 *>(dst + 2 * (t + TPC * e)) = float2{(float)-vv[e].x, (float)-vv[e].y};
          }
          continue;
        }
      }
      cplx<T> *scr = Scr + pid * line_scratch<L>();
      int buf = 0;
      const cplx<T> xnq = r2c_line<T, L, E, false>(vv, t, tid & 63, scr, twl, buf);  // twice the spectrum
      if (yrow < n2) {
        sums[6] += (double)ff;
        const long long row = (long long)zwrap(z) * n2 + yrow;
        cplx<T> *dst = a.spec + ((long long)c * a.d.rows + row) * L;
#pragma unroll
        for (int e = 0; e < E; ++e) stc_nt(dst + t + TPC * e, vv[e]);
        if (t == 0) a.nyq[(long long)c * a.d.rows + row] = xnq;
      }
    }
    if constexpr (PRIO) __builtin_amdgcn_s_setprio(2);
  };

  // prologue: plane z0-1 (odd parity, since Z and hence z0 are even) and its
  // x and y differences, plane z0 in flight, moduli of cell plane z0-1
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  using BT = std::integral_constant<bool, true>;
  using BF = std::integral_constant<bool, false>;
  fetch_u(u[1], z0 - 1);
  take_plane(u[1], dx[1], dy[1]);
  fetch_u(u[0], z0);
  fetch_lm(lam[1], mu[1], z0 - 1);
  __syncthreads();  // the neighbour reads above precede the first publish below
  step(I1{}, BT{}, z0 - 1);
  for (int z = z0; z < z0 + a.Z; z += 2) {
    step(I0{}, BF{}, z);
    step(I1{}, BF{}, z + 1);
  }
  if (a.partial) {
    block_sum<WG>(sums, 7, red);
    if (tid == 0) {
      double *dst = a.partial + (long long)blockIdx.x * 8;
      sums[7] = 0.0;
      if (a.counter)
        store_row_coherent(dst, sums, 8);  // read by the last workgroup of this launch
      else
        for (int i = 0; i < 8; ++i) dst[i] = sums[i];
    }
  }
  if (a.counter) last_block_reduce<WG>(a.red, a.counter, sysb, red);
}

// ---------------------------------------------------------------- z pass, displacement form
// Waves per SIMD the compiler must leave room for: the FP32 AFB pass fits
// in 128 VGPRs without spilling (four waves); the FB and FP64 passes would
// spill there and keep the compiler's own choice.
#ifndef LSFFT_ZU_WAVES
#define LSFFT_ZU_WAVES 4
#endif
template <typename T, int SCH> constexpr int zu_min_waves() {
  return (sizeof(T) == 4 && SCH == SCHEME_AFB) ? LSFFT_ZU_WAVES : 1;
}
template <typename T, int NZ, int E, int P, int SCH>
__global__ __launch_bounds__(P *(NZ / E), (zu_min_waves<T, SCH>())) void k_zpass_u(ZArgs<T> a) {
  const int sysb = blockIdx.y;
  if (a.st && a.st[sysb].done) return;
  a.spec += sysb * a.bs.spec;
  a.nyq += sysb * a.bs.nyq;
  member_green(a.g, a.mem, sysb);
  __shared__ cplx<T> twl_[NZ];
  constexpr int TPC = NZ / E;
  __shared__ cplx<T> lds[2 * NZ * P];
  const int tid = threadIdx.x;
  const int p = tid % P, t = tid / P;
  const int L = a.d.L;
  cplx<T> *base;
  long long zstride, cstride;
  int i1, i2;
  bool valid;
  if ((long long)blockIdx.x < a.main_blocks) {
    const long long col = tile_of(blockIdx.x, a.main_blocks, a.xcd) * P + p;
    valid = col < (long long)a.d.n2 * L;
    i2 = (int)(col / L);
    i1 = (int)(col % L);
    base = a.spec + col;
    zstride = (long long)a.d.n2 * L;
    cstride = a.d.comp_main;
  } else {
    const long long col = ((long long)blockIdx.x - a.main_blocks) * P + p;
    valid = col < a.d.n2;
    i2 = (int)col;
    i1 = L;
    base = a.nyq + col;
    zstride = a.d.n2;
    cstride = a.d.comp_nyq;
  }
  // global addressing: buffer loads with scalar z offsets (as in the strain
  // form's z-pass) issue fewer instructions here but measured 3 % slower
  cplx<T> v[3][E];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int e = 0; e < E; ++e)
      v[c][e] = valid ? base[c * cstride + (t + TPC * e) * zstride] : cplx<T>{T(0), T(0)};
  const AxisVal<T> axx = axis_val(a.g, 0, i1), axy = axis_val(a.g, 1, valid ? i2 : 0);
#if LSFFT_LDS_AXIS
  __shared__ AxisVal<T> axl[NZ];
  stage_axis(axl, a.g, 2);
#else
  AxisVal<T> axz[E];
#pragma unroll
  for (int e = 0; e < E; ++e) axz[e] = axis_val(a.g, 2, t + TPC * e);
#endif
  int buf = 0;
  const cplx<T> *twl = stage_twiddles(twl_, a.tw);  // its barrier publishes axl too
#pragma unroll
  for (int c = 0; c < 3; ++c) fft_pencil<T, NZ, E, true>(v[c], t, lds + p, P, twl, 1, buf);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    cplx<T> f[3] = {v[0][e], v[1][e], v[2][e]};
#if LSFFT_LDS_AXIS
    const AxisVal<T> ax[3] = {axx, axy, axl[t + TPC * e]};
#else
    const AxisVal<T> ax[3] = {axx, axy, axz[e]};
#endif
    green_disp_point<SCH>(a.g, ax, f);
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c][e] = f[c];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    fft_pencil<T, NZ, E, false>(v[c], t, lds + p, P, twl, 1, buf);
    if (valid) {
#pragma unroll
      for (int e = 0; e < E; ++e) base[c * cstride + (t + TPC * e) * zstride] = v[c][e];
    }
  }
}

// ---------------------------------------------------------------- outputs
// eps = Ebar + sym(grad^a u) at every cell, straight from global memory
// (FP64 arithmetic, stored in T).
template <typename T, int SCHEME>
__global__ void k_strain_from_u(const double *__restrict__ u, T *__restrict__ eps, Dims d, double e0, double e1,
                                double e2, double e3, double e4, double e5, double ih0, double ih1, double ih2) {
  const double ih[3] = {ih0, ih1, ih2};
  const long long N = d.N;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(i % d.n1);
    const long long r = i / d.n1;
    const int y = (int)(r % d.n2), z = (int)(r / d.n2);
    double gr[3][3];
    for (int c = 0; c < 3; ++c) {
      double cv[2][2][2];
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
          for (int dd = 0; dd < 2; ++dd) {
            const long long j = ((long long)((z + dd) % d.n3) * d.n2 + (y + b) % d.n2) * d.n1 + (x + a) % d.n1;
            cv[a][b][dd] = u[c * N + j];
          }
      Stencil<SCHEME>::grad(cv, ih, gr[c]);
    }
    eps[i] = (T)(e0 + gr[0][0]);
    eps[N + i] = (T)(e1 + gr[1][1]);
    eps[2 * N + i] = (T)(e2 + gr[2][2]);
    eps[3 * N + i] = (T)(e3 + 0.5 * (gr[1][2] + gr[2][1]));
    eps[4 * N + i] = (T)(e4 + 0.5 * (gr[0][2] + gr[2][0]));
    eps[5 * N + i] = (T)(e5 + 0.5 * (gr[0][1] + gr[1][0]));
  }
}

// ---------------------------------------------------------------- FP64 refinement
// Iterative refinement of an F32 displacement-form solve.  The fixed point
// keeps no memory beyond its iterate, so restarting it on the correction
// delta of u = u_b + delta, with the residual force of u_b as a fixed load,
// continues the same iteration; its rounding errors are then relative to
// the residual at the restart, not to the solution.  k_refine_fold moves
// delta into u_b; k_refine_stress evaluates, in FP64, the total stress
// sigma_b = C : (Ebar + grad^a u_b) - C E_* of every cell once, with block
// sums for its mean (k_refine_mean); k_refine_div takes its divergence
// F_b = div^b sigma_b at the nodes, both with the stencils' own operators,
// and stores -F_b in T as the load of the next FP32 sweeps (they subtract it
// from div^b C grad^a delta).
template <typename T> struct RefineArgs {
  Dims d;
  const double *u;         // folded displacement [system][3][N]
  const double *lam, *mu;  // FP64 moduli [system][N]
  const double *sstar;     // FP64 eigenstress C E_* [system][6][N], or null
  const Member<T> *mem;    // macroscopic strain of each system
  double *sig;             // cell stress sigma_b [system][6][N] (FP64 scratch)
  T *fref;                 // out: -F_b [system][3][N]
  double *part;            // out: stress sums [system][gridDim.x][8]
  const State *st;         // [system]
  double ih[3];            // 1 / h_r
};

template <typename T, int SCH> __global__ __launch_bounds__(256) void k_refine_stress(RefineArgs<T> a) {
  const int sysb = blockIdx.y;
  if (a.st[sysb].done) return;
  const long long N = a.d.N;
  const int n1 = a.d.n1, n2 = a.d.n2, n3 = a.d.n3;
  const double *u = a.u + sysb * 3 * N;
  const double *lam = a.lam + sysb * N, *mu = a.mu + sysb * N;
  const double *ss = a.sstar ? a.sstar + sysb * 6 * N : nullptr;
  double *sig = a.sig + sysb * 6 * N;
  const double *E = a.mem[sysb].Eb;
  __shared__ double red[4 * 8];
  double sums[6] = {0, 0, 0, 0, 0, 0};
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x) {
    // cell (x, y, z): corners (x..x+1, y..y+1, z..z+1)
    const int x = (int)(i % n1);
    const long long row = i / n1;
    const int y = (int)(row % n2), z = (int)(row / n2);
    const int xp = (x + 1) % n1;
    const long long r00 = row * n1, r10 = ((long long)z * n2 + (y + 1) % n2) * n1;
    const long long r01 = ((long long)((z + 1) % n3) * n2 + y) * n1;
    const long long r11 = ((long long)((z + 1) % n3) * n2 + (y + 1) % n2) * n1;
    double gr[3][3];
    for (int c = 0; c < 3; ++c) {
      const double *uc = u + c * N;
      // cv[a][b][d]: corner offsets (x a, y b, z d)
      const double cv[2][2][2] = {{{uc[r00 + x], uc[r01 + x]}, {uc[r10 + x], uc[r11 + x]}},
                                  {{uc[r00 + xp], uc[r01 + xp]}, {uc[r10 + xp], uc[r11 + xp]}}};
      Stencil<SCH>::grad(cv, a.ih, gr[c]);
    }
    double e[6];
    e[0] = E[0] + gr[0][0];
    e[1] = E[1] + gr[1][1];
    e[2] = E[2] + gr[2][2];
    e[3] = E[3] + 0.5 * (gr[1][2] + gr[2][1]);
    e[4] = E[4] + 0.5 * (gr[0][2] + gr[2][0]);
    e[5] = E[5] + 0.5 * (gr[0][1] + gr[1][0]);
    const double l = lam[i], m = mu[i], tr = e[0] + e[1] + e[2];
    for (int c = 0; c < 6; ++c) {
      double v = (c < 3 ? l * tr : 0.0) + 2.0 * m * e[c];
      if (ss) v -= ss[c * N + i];
      sig[c * N + i] = v;
      sums[c] += v;
    }
  }
  block_sum<256>(sums, 6, red);
  if (threadIdx.x == 0) {
    double *dst = a.part + ((long long)sysb * gridDim.x + blockIdx.x) * 8;
    for (int c = 0; c < 6; ++c) dst[c] = sums[c];
  }
}

template <typename T, int SCH> __global__ __launch_bounds__(256) void k_refine_div(RefineArgs<T> a) {
  const int sysb = blockIdx.y;
  if (a.st[sysb].done) return;
  const long long N = a.d.N;
  const int n1 = a.d.n1, n2 = a.d.n2, n3 = a.d.n3;
  const double *sig = a.sig + sysb * 6 * N;
  T *fref = a.fref + sysb * 3 * N;
  static constexpr int vo[3][3] = {{0, 5, 4}, {5, 1, 3}, {4, 3, 2}};  // Voigt index of (i, j)
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x) {
    // node (x, y, z) gathers the cells (x - a, y - b, z - d)
    const int x = (int)(i % n1);
    const long long row = i / n1;
    const int y = (int)(row % n2), z = (int)(row / n2);
    const int xm = (x + n1 - 1) % n1, ym = (y + n2 - 1) % n2, zm = (z + n3 - 1) % n3;
    const long long r00 = row * n1, r10 = ((long long)z * n2 + ym) * n1;
    const long long r01 = ((long long)zm * n2 + y) * n1, r11 = ((long long)zm * n2 + ym) * n1;
    double f[3] = {0.0, 0.0, 0.0};
    for (int c = 0; c < 6; ++c) {
      const double *sc = sig + c * N;
      // s[a][b][d]: the cell node - (a, b, d)
      const double sv[2][2][2] = {{{sc[r00 + x], sc[r01 + x]}, {sc[r10 + x], sc[r11 + x]}},
                                  {{sc[r00 + xm], sc[r01 + xm]}, {sc[r10 + xm], sc[r11 + xm]}}};
      for (int r = 0; r < 3; ++r)
        for (int j = 0; j < 3; ++j)
          if (vo[r][j] == c) f[r] += Stencil<SCH>::div(sv, j, a.ih);
    }
    for (int r = 0; r < 3; ++r) fref[r * N + i] = (T)(-f[r]);
  }
}

template <typename T> __global__ void k_fill_zero(T *p, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = T(0);
}

}  // namespace lsfft
