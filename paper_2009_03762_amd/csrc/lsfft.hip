// Host side of the C ABI declared in include/lsfft.h: validation, device
// buffers, per-axis tables, the launch schedule and its tuner, and the
// fixed-point loop with a device-side stop flag.  The pass kernels are
// launched through Launch<T> (launch_f32.hip, launch_f64.hip).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <chrono>
#include <vector>

#include "solver.hpp"
#include "reduce.hpp"

using namespace lsfft_host;

namespace {

int centred(int i, int n) { return (2 * i < n) ? i : i - n; }

template <typename T> std::vector<T> axis_tables(const int n[3], const double h[3], int off[3], int &S) {
  S = n[0] + n[1] + n[2];
  off[0] = 0;
  off[1] = n[0];
  off[2] = n[0] + n[1];
  std::vector<T> tab((size_t)lsfft::TAB_KINDS * S);
  const long double PI = 3.14159265358979323846264338327950288L;
  for (int r = 0; r < 3; ++r) {
    for (int i = 0; i < n[r]; ++i) {
      const int k = centred(i, n[r]);
      const long double hr = h[r];
      long double c2, s2, ch, sh;
      cis_exact(k, n[r], c2, s2);       // angle 2 pi k / n
      cis_exact(k, 2LL * n[r], ch, sh); // angle pi k / n
      tab[lsfft::TAB_K * S + off[r] + i] = (T)(2.0L * PI * k / (n[r] * hr));
      tab[lsfft::TAB_SH * S + off[r] + i] = (T)(2.0L * sh / hr);
      tab[lsfft::TAB_C * S + off[r] + i] = (T)ch;
      tab[lsfft::TAB_AR * S + off[r] + i] = (T)((c2 - 1.0L) / hr);
      tab[lsfft::TAB_AI * S + off[r] + i] = (T)(s2 / hr);
      tab[lsfft::TAB_C2 * S + off[r] + i] = (T)c2;
    }
  }
  return tab;
}

}  // namespace


namespace {

#define LSFFT_CHECK(call)                                  \
  do {                                                     \
    hipError_t _e = (call);                                \
    if (_e != hipSuccess) {                                \
      fprintf(stderr, "lsfft: %s failed: %s\n", #call,     \
              hipGetErrorString(_e));                      \
      return LSFFT_EDEVICE;                                \
    }                                                      \
  } while (0)


template <typename T> lsfft::GreenParams<T> green_params(lsfft_solver s) {
  lsfft::GreenParams<T> g;
  g.scheme = s->scheme;
  for (int r = 0; r < 3; ++r) {
    g.n[r] = s->n[r];
    g.off[r] = s->off[r];
  }
  g.tabS = s->tabS;
  g.tab = (const T *)s->tab;
  g.lam0 = (T)s->lam0;
  g.mu0 = (T)s->mu0;
  g.c1 = (T)(1.0 / s->mu0);
  g.c2 = (T)((s->lam0 + s->mu0) / (s->mu0 * (s->lam0 + 2.0 * s->mu0)));
  g.beta = (T)((s->lam0 + s->mu0) / (s->lam0 + 2.0 * s->mu0));
  g.scale = (T)(1.0 / (double)s->d.N);
  g.dgo_main = (const T *)s->dgo_main;
  g.dgo_nyq = (const T *)s->dgo_nyq;
  g.dgo_main_stride = s->d.rows * s->d.L;
  g.dgo_nyq_stride = s->d.rows;
  return g;
}

size_t esize(const lsfft_solver s) { return s->prec == LSFFT_F32 ? sizeof(float) : sizeof(double); }

hipEvent_t next_event(lsfft_solver s) {
  if (s->ev_used == s->ev.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    s->ev.push_back(e);
  }
  return s->ev[s->ev_used++];
}

// Times the launches of pass `id` in its scope.  The single-kernel passes
// (ids 0-4, launched through LSFFT_LAUNCH) record the start and stop events
// in the launch itself; the strain form's two-kernel reduction (id 5)
// records them around its launches.
struct Timed {
  lsfft_solver s;
  bool on, in_launch;
  Timed(lsfft_solver s_, int id) : s(s_), on(s_->timing_kernel == id), in_launch(id <= 4) {
    if (!on) return;
    hipEvent_t a = next_event(s);
    hipEvent_t b = a ? next_event(s) : nullptr;
    if (!b) {
      on = false;
      return;
    }
    if (in_launch) {
      s->tstart = a;
      s->tstop = b;
    } else {
      (void)hipEventRecord(a, s->stream);
    }
  }
  ~Timed() {
    if (!on) return;
    if (in_launch) {
      s->tstart = s->tstop = nullptr;
    } else {
      (void)hipEventRecord(s->ev[s->ev_used - 1], s->stream);
    }
  }
};

template <typename T> lsfft::XArgs<T> xargs(lsfft_solver s, int mode, const void *eps_in, bool with_partial) {
  lsfft::XArgs<T> a;
  a.d = s->d;
  a.eps = (T *)s->eps;
  a.eps_in = (const T *)eps_in;
  a.lam = (const T *)s->lam;
  a.mu = (const T *)s->mu;
  a.spec = (cplx<T> *)s->spec;
  a.nyq = (cplx<T> *)s->nyq;
  a.tw = (const cplx<T> *)s->twx;
  a.mem = (const lsfft::Member<T> *)s->mem;
  a.bs = s->bs;
  a.bs.part = s->spx;
  a.partial = with_partial ? s->px : nullptr;
  a.st = with_partial ? s->st : nullptr;
  a.sstar = (const T *)s->sstar;
  a.mode = mode;
  a.polarisation = (s->scheme == LSFFT_DGO) ? 1 : 0;
  return a;
}

template <typename T> lsfft::YArgs<T> yargs(lsfft_solver s, bool flag, int ncomp = 6) {
  lsfft::YArgs<T> a;
  a.ncomp = ncomp;
  a.d = s->d;
  a.spec = (cplx<T> *)s->spec;
  a.nyq = (cplx<T> *)s->nyq;
  a.tw = (const cplx<T> *)s->twy;
  a.st = flag ? s->st : nullptr;
  a.bs = s->bs;
  const int py = Launch<T>::ycols(s->n[1], s->yv);
  a.main_blocks = ((long long)ncomp * s->n[2] * s->d.L + py - 1) / py;
  a.xcd = (s->xcd >> 1) & 1;
  return a;
}

template <typename T> int ygrid(lsfft_solver s, int ncomp) {
  const int py = Launch<T>::ycols(s->n[1], s->yv);
  return (int)(((long long)ncomp * s->n[2] * s->d.L + py - 1) / py + ((long long)ncomp * s->n[2] + py - 1) / py);
}

template <typename T> lsfft::ZArgs<T> zargs(lsfft_solver s, bool flag, int forward_only) {
  lsfft::ZArgs<T> a;
  a.d = s->d;
  a.spec = (cplx<T> *)s->spec;
  a.nyq = (cplx<T> *)s->nyq;
  a.tw = (const cplx<T> *)s->twz;
  a.g = green_params<T>(s);
  a.mem = (const lsfft::Member<T> *)s->mem;
  a.bs = s->bs;
  a.bs.part = s->spz;
  a.partial = flag ? s->pz : nullptr;
  a.st = flag ? s->st : nullptr;
  a.main_blocks = s->z_main_blocks;
  a.forward_only = forward_only;
  a.xcd = (s->xcd >> 2) & 1;
  return a;
}

template <typename T> lsfft::SArgs<T> sargs(lsfft_solver s, int zero_u) {
  lsfft::SArgs<T> a;
  a.raw = nullptr;
  a.d = s->d;
  // refinement: the sweeps iterate on the correction with Ebar = 0 and the
  // FP64 residual force of the folded displacement as their load
  a.u = (const double *)(s->refine ? s->du : s->u);
  a.lam = (const T *)s->lam;
  a.mu = (const T *)s->mu;
  a.spec = (cplx<T> *)s->spec;
  a.nyq = (cplx<T> *)s->nyq;
  a.tw = (const cplx<T> *)s->twx;
  a.mem = (const lsfft::Member<T> *)(s->refine ? s->mem_ref : s->mem);
  a.bs = s->bs;
  a.bs.part = s->spx;
  for (int r = 0; r < 3; ++r) {
    a.ihu[r] = 1.0 / s->h[r];
    a.ih[r] = (T)(1.0 / s->h[r]);
  }
  a.partial = s->px;
  a.st = s->st;
  a.fstar = (const T *)(s->refine ? s->fref : s->fstar);
  a.red = lsfft::ReduceArgs{};
  a.counter = nullptr;
  a.Z = s->sZ;
  a.xcd = s->xcd & 1;
  a.zero_u = zero_u;
  return a;
}

template <typename T> lsfft::UArgs<T> uargs(lsfft_solver s) {
  lsfft::UArgs<T> a;
  a.d = s->d;
  a.u = (double *)(s->refine ? s->du : s->u);
  a.spec = (const cplx<T> *)s->spec;
  a.nyq = (const cplx<T> *)s->nyq;
  a.tw = (const cplx<T> *)s->twx;
  a.st = s->st;
  a.bs = s->bs;
  return a;
}

// eps of every system from its displacement; Eb: [B][6]
template <typename T> hipError_t strain_from_u(lsfft_solver s, const double *Eb) {
  const int blocks = (int)std::min<long long>((s->d.N + 255) / 256, 65536);
  const double ih0 = 1.0 / s->h[0], ih1 = 1.0 / s->h[1], ih2 = 1.0 / s->h[2];
  for (int b = 0; b < s->B; ++b) {
    const double *u = (const double *)s->u + (long long)b * 3 * s->d.N;
    T *eps = (T *)s->eps + (long long)b * 6 * s->d.N;
    const double *e = Eb + 6 * b;
    if (s->scheme == LSFFT_FB)
      hipLaunchKernelGGL((lsfft::k_strain_from_u<T, lsfft::SCHEME_FB>), dim3(blocks), dim3(256), 0, s->stream, u,
                         eps, s->d, e[0], e[1], e[2], e[3], e[4], e[5], ih0, ih1, ih2);
    else
      hipLaunchKernelGGL((lsfft::k_strain_from_u<T, lsfft::SCHEME_AFB>), dim3(blocks), dim3(256), 0, s->stream, u,
                         eps, s->d, e[0], e[1], e[2], e[3], e[4], e[5], ih0, ih1, ih2);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}

// Per-system constants (macroscopic strain Eb[B][6], reference medium) to the device.
template <typename T> lsfft_status upload_members(lsfft_solver s, const double *Eb) {
  std::vector<lsfft::Member<T>> m(s->B);
  std::vector<double> en(s->B);
  static const int vo[3][3] = {{0, 5, 4}, {5, 1, 3}, {4, 3, 2}};  // Voigt index of (i, j)
  for (int b = 0; b < s->B; ++b) {
    const double *e = Eb ? Eb + 6 * b : nullptr;
    double nrm = 0.0;
    for (int c = 0; c < 6; ++c) {
      m[b].Eb[c] = e ? e[c] : 0.0;
      nrm += (c < 3 ? 1.0 : 2.0) * m[b].Eb[c] * m[b].Eb[c];
    }
    en[b] = std::sqrt(nrm);
    // pure eigenstrain loading: scale the DGO stopping test by the RMS of |E_*|_F
    if (en[b] == 0.0 && s->eig) en[b] = s->estar_rms[b];
    for (int i = 0; i < 3; ++i)
      for (int r = 0; r < 3; ++r) m[b].hE[i][r] = s->h[r] * m[b].Eb[vo[i][r]];
    const double l0 = s->lam0v[b], m0 = s->mu0v[b];
    m[b].lam0 = (T)l0;
    m[b].mu0 = (T)m0;
    m[b].c1 = (T)(1.0 / m0);
    m[b].c2 = (T)((l0 + m0) / (m0 * (l0 + 2.0 * m0)));
    m[b].beta = (T)((l0 + m0) / (l0 + 2.0 * m0));
  }
  LSFFT_CHECK(hipMemcpyAsync(s->mem, m.data(), sizeof(lsfft::Member<T>) * s->B, hipMemcpyHostToDevice, s->stream));
  LSFFT_CHECK(hipMemcpyAsync(s->enorm, en.data(), sizeof(double) * s->B, hipMemcpyHostToDevice, s->stream));
  std::vector<lsfft::Member<double>> m64(s->mem64 ? s->B : 0);
  for (size_t b = 0; b < m64.size(); ++b) {
    for (int c = 0; c < 6; ++c) m64[b].Eb[c] = m[b].Eb[c];
    for (int i = 0; i < 3; ++i)
      for (int r = 0; r < 3; ++r) m64[b].hE[i][r] = m[b].hE[i][r];
    m64[b].lam0 = s->lam0v[b];
    m64[b].mu0 = s->mu0v[b];
    m64[b].c1 = 1.0 / s->mu0v[b];
    m64[b].c2 = (s->lam0v[b] + s->mu0v[b]) / (s->mu0v[b] * (s->lam0v[b] + 2.0 * s->mu0v[b]));
    m64[b].beta = (s->lam0v[b] + s->mu0v[b]) / (s->lam0v[b] + 2.0 * s->mu0v[b]);
  }
  if (s->mem64)
    LSFFT_CHECK(hipMemcpyAsync(s->mem64, m64.data(), sizeof(lsfft::Member<double>) * s->B, hipMemcpyHostToDevice,
                               s->stream));
  if (s->mem_ref) {
    for (auto &x : m) {
      for (int c = 0; c < 6; ++c) x.Eb[c] = 0.0;
      for (int i = 0; i < 3; ++i)
        for (int r = 0; r < 3; ++r) x.hE[i][r] = 0.0;
    }
    LSFFT_CHECK(hipMemcpyAsync(s->mem_ref, m.data(), sizeof(lsfft::Member<T>) * s->B, hipMemcpyHostToDevice,
                               s->stream));
  }
  // the host vectors go out of scope: wait for the copies
  LSFFT_CHECK(hipStreamSynchronize(s->stream));
  return LSFFT_OK;
}

bool all_done(const lsfft_solver s) {
  for (int b = 0; b < s->B; ++b)
    if (!s->st_host[b].done) return false;
  return true;
}

constexpr int GRAPH_CHUNK = 8;

// Capture GRAPH_CHUNK iterations (enqueued by `iteration`) on the internal
// stream and keep the executable graph; captured again when tol or maxit
// change.  The captured launches are kernels only.
template <typename F> lsfft_status ensure_graph(lsfft_solver s, double tol, int maxit, F &&iteration) {
  if (!s->gstream) {
    LSFFT_CHECK(hipStreamCreateWithFlags(&s->gstream, hipStreamNonBlocking));
    LSFFT_CHECK(hipEventCreateWithFlags(&s->gevent, hipEventDisableTiming));
  }
  if (s->gexec && s->g_tol == tol && s->g_maxit == maxit) return LSFFT_OK;
  if (s->gexec) {
    (void)hipGraphExecDestroy(s->gexec);
    s->gexec = nullptr;
  }
  if (s->graph) {
    (void)hipGraphDestroy(s->graph);
    s->graph = nullptr;
  }
  hipStream_t user = s->stream;
  s->stream = s->gstream;
  // captured chunks are never timed (a group solve may capture a handle
  // whose kernel timing is on)
  const int timing = s->timing_kernel;
  s->timing_kernel = -1;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(s->gstream, hipStreamCaptureModeThreadLocal);
  for (int j = 0; j < GRAPH_CHUNK && e == hipSuccess; ++j) e = iteration(false);
  hipError_t e2 = hipStreamEndCapture(s->gstream, &g);
  s->stream = user;
  s->timing_kernel = timing;
  if (e != hipSuccess || e2 != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    fprintf(stderr, "lsfft: graph capture failed: %s\n", hipGetErrorString(e != hipSuccess ? e : e2));
    return LSFFT_EDEVICE;
  }
  e = hipGraphInstantiate(&s->gexec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    s->gexec = nullptr;
    fprintf(stderr, "lsfft: graph instantiation failed: %s\n", hipGetErrorString(e));
    return LSFFT_EDEVICE;
  }
  s->graph = g;
  s->g_tol = tol;
  s->g_maxit = maxit;
  return LSFFT_OK;
}

// Iterations k_begin .. k_end-1 of a solve (maxit, tol as in lsfft_solve) of
// every system of the batch, whose constants upload_members has set.
// fresh: start from u = 0 / eps = Ebar with a new device state; otherwise the
// state, history and u left by an earlier phase are continued (displacement
// form), after re-evaluating the stencil on that u in this precision.
// Returns LSFFT_OK when the iterations ran, even if not every system is done.
// prepare_only: enqueue the phase's opening work (state reset, first stencil
// or x-pass with its test) and capture the chunk graph, but run no chunk: a
// group solve replays the chunks of several solvers in one graph.
template <typename T>
lsfft_status run_phase(lsfft_solver s, double tol, int maxit, int k_begin, int k_end, bool fresh,
                       bool prepare_only = false) {
  using L = Launch<T>;
  const bool dgo = (s->scheme == LSFFT_DGO);
  const bool disp = s->disp != 0;
  const int ncomp = disp ? 3 : 6;
  s->launch_b = s->B;
  lsfft::ReduceArgs ra;
  ra.px = s->px;
  ra.nx = disp ? s->nsb : s->nxb;
  ra.pz = s->pz;
  ra.nz = disp ? 0 : s->nzb;
  ra.spx = s->spx;
  ra.spz = s->spz;
  ra.stage = s->pstage;
  ra.st = s->st;
  ra.hist = s->hist;
  ra.hcap = s->hist_cap;
  ra.ebar_norms = s->enorm;
  // the stencil sums C E, not C [E - E_*]; refined sweeps sum C grad delta,
  // and sref holds minus the mean total stress of the folded displacement
  ra.smean = s->refine ? s->sref : ((disp && s->eig) ? s->smean : nullptr);
  ra.maxit = maxit;
  ra.tol = s->tuning ? -1.0 : tol;
  ra.dgo = dgo ? 1 : 0;
  ra.disp = disp ? 1 : 0;
  ra.N = (double)s->d.N;
  ra.div_factor = s->tuning ? __builtin_huge_val() : 1e6;
  // displacement form: the stencil's last workgroup takes the reduction and
  // stop test of the iterate the stencil has just evaluated
  auto with_reduce = [&](lsfft::SArgs<T> a) {
    a.red = ra;
    a.counter = s->counter;
    return a;
  };
  if (fresh) {
    hipLaunchKernelGGL(lsfft::k_state_init, dim3((s->B + 63) / 64), dim3(64), 0, s->stream, s->st, s->B);
    LSFFT_CHECK(hipGetLastError());
  }
  if (disp) {
    if (fresh) {
      const long long nu = 3 * s->d.N * s->B;
      hipLaunchKernelGGL(lsfft::k_fill_zero<double>, dim3((unsigned)std::min<long long>((nu + 255) / 256, 65536)),
                         dim3(256), 0, s->stream, (double *)(s->refine ? s->du : s->u), nu);
      LSFFT_CHECK(hipGetLastError());
    }
    Timed tm(s, 0);
    // a refinement cycle starts from delta = 0
    LSFFT_CHECK(L::stencil(s, with_reduce(sargs<T>(s, (fresh || s->refine) ? 1 : 0)), s->nsb));
  } else {
    Timed tm(s, 0);
    LSFFT_CHECK(L::xpass(s, xargs<T>(s, lsfft::XMODE_INIT, nullptr, true), s->nxb));
  }
  const lsfft::YArgs<T> ya = yargs<T>(s, true, ncomp);
  const int nyg = ygrid<T>(s, ncomp);
  lsfft::ZArgs<T> za = zargs<T>(s, true, 0);
  if (disp) {
    za.main_blocks = s->zu_main_blocks;
    za.g.scale = (T)(0.5 / (double)s->d.N);  // the stencils' real x transforms return twice the spectrum
  }
  const lsfft::XArgs<T> xa = xargs<T>(s, dgo ? lsfft::XMODE_DGO : lsfft::XMODE_UPDATE, nullptr, true);
  const lsfft::SArgs<T> sa = with_reduce(sargs<T>(s, 0));
  const lsfft::UArgs<T> ua = uargs<T>(s);
  // One iteration of every system: forward y, z-pass with the Green step,
  // (strain form: reduction and stopping test,) inverse y, then the x side:
  // displacement update and stencil, whose last workgroup reduces and tests
  // the new iterate, or the x-pass.  `last` omits the trailing stencil (the
  // next phase evaluates it, and tests that iterate, in its own precision).
  auto iteration = [&](bool last) -> hipError_t {
    hipError_t e;
    {
      Timed tm(s, 1);
      if ((e = L::template ypass<true>(s, ya, nyg)) != hipSuccess) return e;
    }
    {
      Timed tm(s, 2);
      if ((e = disp ? L::zpass_u(s, za, s->nzub) : L::zpass(s, za, s->nzb)) != hipSuccess) return e;
    }
    if (!disp) {
      Timed tm(s, 5);
      hipLaunchKernelGGL(lsfft::k_reduce_stage, dim3(lsfft::RSTAGE, s->B), dim3(256), 0, s->stream, ra);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      hipLaunchKernelGGL(lsfft::k_reduce, dim3(1, s->B), dim3(64), 0, s->stream, ra);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    {
      Timed tm(s, 3);
      if ((e = L::template ypass<false>(s, ya, nyg)) != hipSuccess) return e;
    }
    if (disp) {
      {
        Timed tm(s, 4);
        if ((e = L::uxpass(s, ua, s->nub)) != hipSuccess) return e;
      }
      if (!last) {
        Timed tm(s, 0);
        if ((e = L::stencil(s, sa, s->nsb)) != hipSuccess) return e;
      }
    } else {
      Timed tm(s, 0);
      if ((e = L::xpass(s, xa, s->nxb)) != hipSuccess) return e;
    }
    return hipSuccess;
  };
  auto read_state = [&](hipStream_t st) -> lsfft_status {
    LSFFT_CHECK(hipMemcpyAsync(s->st_host, s->st, sizeof(State) * s->B, hipMemcpyDeviceToHost, st));
    LSFFT_CHECK(hipStreamSynchronize(st));
    return LSFFT_OK;
  };
  if (prepare_only) return ensure_graph(s, tol, maxit, iteration);
  int k = k_begin;
  // The final phase of a solve replays captured chunks of iterations (its
  // iterations run to the stopping test, so a chunk may overrun: kernels of
  // a finished system return at once).  Kernel timing needs the eager path.
  const bool graphs = s->use_graphs && k_end == maxit + 1 && s->timing_kernel < 0 && k_end - k >= GRAPH_CHUNK;
  if (graphs) {
    lsfft_status gs = ensure_graph(s, tol, maxit, iteration);
    if (gs != LSFFT_OK) return gs;
    LSFFT_CHECK(hipEventRecord(s->gevent, s->stream));
    LSFFT_CHECK(hipStreamWaitEvent(s->gstream, s->gevent, 0));
    int per_sync = (tol == 0.0 || s->tuning) ? (k_end - k + GRAPH_CHUNK - 1) / GRAPH_CHUNK : 1;
    // residual and tested iterate of every system at the previous read
    std::vector<double> r_prev(s->B, -1.0);
    std::vector<int> k_prev(s->B, 0);
    for (;;) {
      for (int j = 0; j < per_sync && k < k_end; ++j, k += GRAPH_CHUNK) LSFFT_CHECK(hipGraphLaunch(s->gexec, s->gstream));
      lsfft_status rs = read_state(s->gstream);
      if (rs != LSFFT_OK) return rs;
      if (all_done(s) || k >= k_end) break;
      // Chunks between reads: doubling up to 8, but no more than the slowest
      // running system still needs at its contraction since the last read
      // (chunks enqueued past a stop return at once, yet each costs its
      // launches).
      int need = 0;
      bool known = true;
      for (int b = 0; b < s->B; ++b) {
        const State &x = s->st_host[b];
        if (x.done) continue;
        const int dk = x.k - k_prev[b];
        const double rho = (r_prev[b] > 0.0 && x.r > 0.0 && dk > 0) ? std::pow(x.r / r_prev[b], 1.0 / dk) : 1.0;
        if (!(rho < 1.0) || !(tol > 0.0)) {
          known = false;
        } else {
          const double left = std::log(tol / x.r) / std::log(rho);
          need = std::max(need, (int)std::ceil(std::max(left, 1.0) / GRAPH_CHUNK));
        }
        r_prev[b] = x.r;
        k_prev[b] = x.k;
      }
      per_sync = std::min(per_sync * 2, 8);
      if (known && need > 0) per_sync = std::min(per_sync, need);
    }
    return LSFFT_OK;
  }
  int chunk = (tol == 0.0 || s->tuning) ? k_end - k_begin : 2;
  for (;;) {
    const int nenq = std::min(chunk, k_end - k);
    for (int j = 0; j < nenq; ++j, ++k) LSFFT_CHECK(iteration(k + 1 == k_end));
    lsfft_status rs = read_state(s->stream);
    if (rs != LSFFT_OK) return rs;
    if (all_done(s) || k >= k_end) break;
    chunk = std::min(chunk * 2, 64);
  }
  return LSFFT_OK;
}

// Eb: [B][6].  Returns the largest status over the systems (OK < ENOTCONV <
// EDIVERGED) or a negative error.
// Room for the residuals of iterations 0 .. maxit of every system.
lsfft_status ensure_hist(lsfft_solver s, int maxit) {
  if (maxit + 1 > s->hist_cap) {
    if (s->hist) (void)hipFree(s->hist);
    s->hist = nullptr;
    int cap = maxit + 1 < 1024 ? 1024 : maxit + 1;
    if (hipMalloc(&s->hist, sizeof(double) * cap * (size_t)s->B) != hipSuccess) {
      s->hist_cap = 0;
      return LSFFT_ENOMEM;
    }
    s->hist_cap = cap;
  }
  return LSFFT_OK;
}

// Drop the captured iteration chunk (the schedule or the stopping rule it
// was captured with has changed).
void drop_graph(lsfft_solver s) {
  if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
  s->gexec = nullptr;
  if (s->graph) (void)hipGraphDestroy(s->graph);
  s->graph = nullptr;
  s->g_tol = -1.0;
  s->g_maxit = -1;
}

int stencil_yblocks(const lsfft_solver s, bool f64);

// Start of a refinement cycle (systems not done): fold delta into u, then in
// FP64 the divergence of the cell stress of u at the nodes, stored as the
// sweeps' load -F_b, and the mean stress: by the FP64 register stencil where
// it runs at this n1, else by the cell-stress and divergence kernels.
template <typename T> lsfft_status refine_rebase(lsfft_solver s) {
  const long long n3 = 3 * s->d.N;
  const unsigned fb = (unsigned)std::min<long long>((n3 + 255) / 256, 4096);
  hipLaunchKernelGGL(lsfft::k_refine_fold, dim3(fb, s->B), dim3(256), 0, s->stream, (double *)s->u, s->du, s->st,
                     n3);
  LSFFT_CHECK(hipGetLastError());
  if (s->mem64) {
    // the FP64 register stencil on the folded u: its divergence f (minus the
    // eigenstress force), stored as -F_b, and its stress block sums
    lsfft::SArgs<double> a;
    a.d = s->d;
    a.u = (const double *)s->u;
    a.lam = s->lam64;
    a.mu = s->mu64;
    a.spec = nullptr;
    a.nyq = nullptr;
    a.tw = nullptr;
    a.mem = (const lsfft::Member<double> *)s->mem64;
    a.bs = s->bs;
    a.bs.part = s->spx;
    for (int r = 0; r < 3; ++r) {
      a.ihu[r] = 1.0 / s->h[r];
      a.ih[r] = 1.0 / s->h[r];
    }
    a.partial = s->px;
    a.st = s->st;
    a.fstar = s->fstar64;
    a.red = lsfft::ReduceArgs{};
    a.counter = nullptr;
    a.Z = s->sZ;
    a.xcd = s->xcd & 1;
    a.zero_u = 0;
    a.raw = (float *)s->fref;
    const int nsb64 = stencil_yblocks(s, true) * (s->n[2] / s->sZ);  // its own node lines per workgroup
    LSFFT_CHECK(Launch<double>::stencil(s, a, nsb64));
    hipLaunchKernelGGL(lsfft::k_refine_mean, dim3(s->B), dim3(64), 0, s->stream, s->px, nsb64, s->spx, s->sref,
                       s->eig ? s->smean : nullptr, s->st, (double)s->d.N);
    LSFFT_CHECK(hipGetLastError());
    return LSFFT_OK;
  }
  lsfft::RefineArgs<T> a;
  a.d = s->d;
  a.u = (const double *)s->u;
  a.lam = s->lam64;
  a.mu = s->mu64;
  a.sstar = s->sstar64;
  a.mem = (const lsfft::Member<T> *)s->mem;
  a.sig = s->rsig;
  a.fref = (T *)s->fref;
  a.part = s->rpart;
  a.st = s->st;
  for (int r = 0; r < 3; ++r) a.ih[r] = 1.0 / s->h[r];
  const dim3 grid(s->nrb, s->B);
  if (s->scheme == LSFFT_FB) {
    hipLaunchKernelGGL((lsfft::k_refine_stress<T, lsfft::SCHEME_FB>), grid, dim3(256), 0, s->stream, a);
    LSFFT_CHECK(hipGetLastError());
    hipLaunchKernelGGL((lsfft::k_refine_div<T, lsfft::SCHEME_FB>), grid, dim3(256), 0, s->stream, a);
  } else {
    hipLaunchKernelGGL((lsfft::k_refine_stress<T, lsfft::SCHEME_AFB>), grid, dim3(256), 0, s->stream, a);
    LSFFT_CHECK(hipGetLastError());
    hipLaunchKernelGGL((lsfft::k_refine_div<T, lsfft::SCHEME_AFB>), grid, dim3(256), 0, s->stream, a);
  }
  LSFFT_CHECK(hipGetLastError());
  hipLaunchKernelGGL(lsfft::k_refine_mean, dim3(s->B), dim3(64), 0, s->stream, s->rpart, s->nrb,
                     (long long)s->nrb * 8, s->sref, nullptr, s->st, (double)s->d.N);
  LSFFT_CHECK(hipGetLastError());
  return LSFFT_OK;
}

// A solve with FP64 iterative refinement (F32 displacement form): cycles of
// `refine` F32 iterations on delta, each opened by a fold and an FP64
// residual evaluation whose stencil pass tests the folded iterate.  A system
// that stops inside a cycle (tolerance, maxit or divergence judged on the
// F32 sums) is resumed and re-tested at the next FP64 evaluation, so every
// final status, residual and mean stress comes from one.  fresh: start from
// u = 0; otherwise u holds an untested iterate (FP64 warm start).
template <typename T> lsfft_status run_refined(lsfft_solver s, double tol, int maxit, bool fresh) {
  const long long nu = 3 * s->d.N * s->B;
  const unsigned zb = (unsigned)std::min<long long>((nu + 255) / 256, 65536);
  if (fresh) {
    hipLaunchKernelGGL(lsfft::k_state_init, dim3((s->B + 63) / 64), dim3(64), 0, s->stream, s->st, s->B);
    LSFFT_CHECK(hipGetLastError());
    hipLaunchKernelGGL(lsfft::k_fill_zero<double>, dim3(zb), dim3(256), 0, s->stream, (double *)s->u, nu);
    LSFFT_CHECK(hipGetLastError());
  }
  hipLaunchKernelGGL(lsfft::k_fill_zero<double>, dim3(zb), dim3(256), 0, s->stream, s->du, nu);
  LSFFT_CHECK(hipGetLastError());
  LSFFT_CHECK(hipMemcpyAsync(s->st_host, s->st, sizeof(State) * s->B, hipMemcpyDeviceToHost, s->stream));
  LSFFT_CHECK(hipStreamSynchronize(s->stream));
  std::vector<int> tested(s->B);
  for (;;) {
    if (all_done(s)) break;
    // the iterate each system's FP64 evaluation tests
    for (int b = 0; b < s->B; ++b) tested[b] = s->st_host[b].k;
    lsfft_status rs = refine_rebase<T>(s);
    if (rs != LSFFT_OK) return rs;
    rs = run_phase<T>(s, tol, maxit, 0, s->refine, false);
    if (rs != LSFFT_OK) return rs;
    bool resume = false;
    for (int b = 0; b < s->B; ++b) {
      State &x = s->st_host[b];
      if (x.done && x.iters != tested[b]) {
        x.done = 0;
        x.status = 1;
        resume = true;
      }
    }
    if (resume) {
      LSFFT_CHECK(hipMemcpyAsync(s->st, s->st_host, sizeof(State) * s->B, hipMemcpyHostToDevice, s->stream));
      LSFFT_CHECK(hipStreamSynchronize(s->stream));
    }
  }
  return LSFFT_OK;
}

template <typename T>
lsfft_status run_solve(lsfft_solver s, const double *Eb, double tol, int maxit) {
  lsfft_status hs = ensure_hist(s, maxit);
  if (hs != LSFFT_OK) return hs;
  s->ev_used = 0;
  lsfft_status us = upload_members<T>(s, Eb);
  if (us != LSFFT_OK) return us;
  int k0 = 0;
  if (s->twin && (s->warm > 0 || s->until > 0.0)) {
    // FP64 iterations on the shared u, state and history: 0 .. warm-1, then
    // (f64_until) on until each system's residual is at most the switch
    // level; the F32 phase below continues every system that is not done
    lsfft_solver t = s->twin;
    t->hist = s->hist;
    t->hist_cap = s->hist_cap;
    t->timing_kernel = -1;
    us = upload_members<double>(t, Eb);
    if (us != LSFFT_OK) return us;
    bool fresh = true;
    if (s->warm > 0) {
      k0 = std::min(s->warm, maxit + 1);
      lsfft_status ps = run_phase<double>(t, tol, maxit, 0, k0, true);
      if (ps != LSFFT_OK) return ps;
      fresh = false;
    }
    if (s->until > 0.0 && (fresh || (!all_done(s) && k0 <= maxit))) {
      lsfft_status ps = run_phase<double>(t, std::max(tol, s->until), maxit, k0, maxit + 1, fresh);
      if (ps != LSFFT_OK) return ps;
      // a system that stopped on the switch level rather than on tol goes on
      // in F32 from the iterate it stopped at (tested again there)
      bool resume = false;
      int kmin = maxit + 1;
      for (int b = 0; b < s->B; ++b) {
        State &x = s->st_host[b];
        if (x.done && x.status == 0 && x.r > tol) {
          x.done = 0;
          x.status = 1;
          resume = true;
        }
        if (!x.done) kmin = std::min(kmin, x.k);
      }
      if (resume) {
        LSFFT_CHECK(hipMemcpyAsync(s->st, s->st_host, sizeof(State) * s->B, hipMemcpyHostToDevice, s->stream));
        LSFFT_CHECK(hipStreamSynchronize(s->stream));
      }
      k0 = std::max(kmin, 1);
    }
  }
  if (s->refine) {
    lsfft_status ps = run_refined<T>(s, tol, maxit, k0 == 0);
    if (ps != LSFFT_OK) return ps;
  } else if (k0 == 0 || (!all_done(s) && k0 <= maxit)) {
    lsfft_status ps = run_phase<T>(s, tol, maxit, k0, maxit + 1, k0 == 0);
    if (ps != LSFFT_OK) return ps;
  }
  if (!all_done(s)) return LSFFT_EDEVICE;
  s->last_iters = s->st_host[0].iters;
  if (s->timing_kernel >= 0 && s->ev_used >= 2) {
    double tot = 0.0;
    int cnt = 0;
    for (size_t i = 0; i + 1 < s->ev_used; i += 2) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, s->ev[i], s->ev[i + 1]) == hipSuccess) {
        tot += ms;
        ++cnt;
      }
    }
    s->timing_mean = cnt ? tot / cnt : 0.0;
    s->timing_count = cnt;
  }
  int worst = 0;
  for (int b = 0; b < s->B; ++b) worst = std::max(worst, s->st_host[b].status);
  return (lsfft_status)worst;
}

// ------------------------------------------------------------------ group solve
// Replay the captured chunks of several solvers together: one graph holding
// each solver's chunk as an independent child node, launched on `gs` until
// every system of every solver is done (a finished system's kernels return
// at once, so the chunk of a solver that is done costs launches only).  The
// opening work of each phase ran on the solvers' own streams; their later
// work waits for the group.
lsfft_status group_loop(const std::vector<lsfft_solver> &hs, hipStream_t gs, hipEvent_t ev, int max_chunks) {
  hipGraph_t g = nullptr;
  LSFFT_CHECK(hipGraphCreate(&g, 0));
  for (lsfft_solver h : hs) {
    hipGraphNode_t node;
    const hipError_t e = hipGraphAddChildGraphNode(&node, g, nullptr, 0, h->graph);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      fprintf(stderr, "lsfft: group graph: %s\n", hipGetErrorString(e));
      return LSFFT_EDEVICE;
    }
  }
  hipGraphExec_t gx = nullptr;
  hipError_t e = hipGraphInstantiate(&gx, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    fprintf(stderr, "lsfft: group graph instantiation failed: %s\n", hipGetErrorString(e));
    return LSFFT_EDEVICE;
  }
  auto fail = [&](hipError_t err) {
    (void)hipGraphExecDestroy(gx);
    fprintf(stderr, "lsfft: group solve: %s\n", hipGetErrorString(err));
    return LSFFT_EDEVICE;
  };
  for (lsfft_solver h : hs) {
    if ((e = hipEventRecord(h->gevent, h->stream)) != hipSuccess) return fail(e);
    if ((e = hipStreamWaitEvent(gs, h->gevent, 0)) != hipSuccess) return fail(e);
  }
  int launched = 0, per_sync = 1;
  for (;;) {
    for (int j = 0; j < per_sync && launched < max_chunks; ++j, ++launched)
      if ((e = hipGraphLaunch(gx, gs)) != hipSuccess) return fail(e);
    for (lsfft_solver h : hs)
      if ((e = hipMemcpyAsync(h->st_host, h->st, sizeof(State) * h->B, hipMemcpyDeviceToHost, gs)) != hipSuccess)
        return fail(e);
    if ((e = hipStreamSynchronize(gs)) != hipSuccess) return fail(e);
    bool all = true;
    for (lsfft_solver h : hs) all = all && all_done(h);
    if (all || launched >= max_chunks) break;
    per_sync = std::min(per_sync * 2, 8);
  }
  (void)hipGraphExecDestroy(gx);
  LSFFT_CHECK(hipEventRecord(ev, gs));
  for (lsfft_solver h : hs) LSFFT_CHECK(hipStreamWaitEvent(h->stream, ev, 0));
  return LSFFT_OK;
}

template <typename T> lsfft_status prepare_phase(lsfft_solver s, double tol, int maxit, int k0, bool fresh) {
  return run_phase<T>(s, tol, maxit, k0, maxit + 1, fresh, true);
}

// Solve every system of several solvers (cells of different sizes, each a
// batch of load cases) together: the FP64 phase of the solvers with an FP64
// warm start (f64_until), then every solver's own phase, each as one group
// graph per chunk of iterations.  Eb: [sum B][6] in solver order.
lsfft_status solve_group(const std::vector<lsfft_solver> &hs, const double *Eb, double tol,
                         const std::vector<int> &maxits) {
  const int n = (int)hs.size();
  int maxit_all = 0;
  for (int m : maxits) maxit_all = std::max(maxit_all, m);
  std::vector<int> k0(n, 0);
  std::vector<char> fresh(n, 1);
  long long off = 0;
  for (int i = 0; i < n; ++i) {
    lsfft_solver s = hs[i];
    const int maxit = maxits[i];
    lsfft_status st = ensure_hist(s, maxit);
    if (st != LSFFT_OK) return st;
    s->ev_used = 0;
    st = (s->prec == LSFFT_F32) ? upload_members<float>(s, Eb + 6 * off) : upload_members<double>(s, Eb + 6 * off);
    if (st != LSFFT_OK) return st;
    if (s->twin && (s->warm > 0 || s->until > 0.0)) {
      lsfft_solver t = s->twin;
      t->hist = s->hist;
      t->hist_cap = s->hist_cap;
      t->timing_kernel = -1;
      st = upload_members<double>(t, Eb + 6 * off);
      if (st != LSFFT_OK) return st;
      if (s->warm > 0) {
        k0[i] = std::min(s->warm, maxit + 1);
        st = run_phase<double>(t, tol, maxit, 0, k0[i], true);
        if (st != LSFFT_OK) return st;
        fresh[i] = 0;
      }
    }
    off += s->B;
  }
  hipStream_t gs = nullptr;
  hipEvent_t ev = nullptr;
  LSFFT_CHECK(hipStreamCreateWithFlags(&gs, hipStreamNonBlocking));
  if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
    (void)hipStreamDestroy(gs);
    return LSFFT_EDEVICE;
  }
  auto done = [&](lsfft_status st) {
    (void)hipStreamSynchronize(gs);
    (void)hipEventDestroy(ev);
    (void)hipStreamDestroy(gs);
    return st;
  };
  const int chunks = (maxit_all + 1 + GRAPH_CHUNK - 1) / GRAPH_CHUNK + 1;
  // FP64 phase down to each solver's switch level
  std::vector<lsfft_solver> grp;
  std::vector<int> who;
  for (int i = 0; i < n; ++i) {
    lsfft_solver s = hs[i];
    const int maxit = maxits[i];
    if (!s->twin || !(s->until > 0.0)) continue;
    if (!fresh[i] && (all_done(s) || k0[i] > maxit)) continue;
    lsfft_status st = prepare_phase<double>(s->twin, std::max(tol, s->until), maxit, k0[i], fresh[i]);
    if (st != LSFFT_OK) return done(st);
    grp.push_back(s->twin);
    who.push_back(i);
  }
  if (!grp.empty()) {
    lsfft_status st = group_loop(grp, gs, ev, chunks);
    if (st != LSFFT_OK) return done(st);
    for (int i : who) {
      lsfft_solver s = hs[i];
      const int maxit = maxits[i];
      bool resume = false;
      int kmin = maxit + 1;
      for (int b = 0; b < s->B; ++b) {
        State &x = s->st_host[b];
        if (x.done && x.status == 0 && x.r > tol) {
          x.done = 0;
          x.status = 1;
          resume = true;
        }
        if (!x.done) kmin = std::min(kmin, x.k);
      }
      if (resume && hipMemcpyAsync(s->st, s->st_host, sizeof(State) * s->B, hipMemcpyHostToDevice, s->stream) !=
                        hipSuccess)
        return done(LSFFT_EDEVICE);
      k0[i] = std::max(kmin, 1);
      fresh[i] = 0;
    }
  }
  // every solver's own phase
  grp.clear();
  for (int i = 0; i < n; ++i) {
    lsfft_solver s = hs[i];
    const int maxit = maxits[i];
    if (!fresh[i] && (all_done(s) || k0[i] > maxit)) continue;
    lsfft_status st = (s->prec == LSFFT_F32) ? prepare_phase<float>(s, tol, maxit, k0[i], fresh[i])
                                             : prepare_phase<double>(s, tol, maxit, k0[i], fresh[i]);
    if (st != LSFFT_OK) return done(st);
    grp.push_back(s);
  }
  if (!grp.empty()) {
    lsfft_status st = group_loop(grp, gs, ev, chunks);
    if (st != LSFFT_OK) return done(st);
  }
  off = 0;
  for (int i = 0; i < n; ++i) {
    lsfft_solver s = hs[i];
    if (!all_done(s)) return done(LSFFT_EDEVICE);
    s->last_iters = s->st_host[0].iters;
    off += s->B;
  }
  return done(LSFFT_OK);
}

// Outputs of every system: eps_out / sig_out hold [B][6][N] values (host
// doubles or device T); either may be null.  In the displacement form the
// strain is formed from u here, and only when an output needs it.  Eb: [B][6].
template <typename T>
lsfft_status finish_outputs(lsfft_solver s, void *eps_out, void *sig_out, bool host, const double *Eb) {
  if (s->disp && (eps_out || sig_out)) LSFFT_CHECK(strain_from_u<T>(s, Eb));
  const size_t n6 = 6 * (size_t)s->d.N;
  const size_t bytes = n6 * (size_t)s->B * sizeof(T);
  if (eps_out) {
    if (host) {
      std::vector<T> tmp(n6 * s->B);
      LSFFT_CHECK(hipMemcpyAsync(tmp.data(), s->eps, bytes, hipMemcpyDeviceToHost, s->stream));
      LSFFT_CHECK(hipStreamSynchronize(s->stream));
      double *o = (double *)eps_out;
      for (size_t i = 0; i < tmp.size(); ++i) o[i] = (double)tmp[i];
    } else {
      LSFFT_CHECK(hipMemcpyAsync(eps_out, s->eps, bytes, hipMemcpyDeviceToDevice, s->stream));
    }
  }
  if (sig_out) {
    T *dst = nullptr;
    if (host) {
      LSFFT_CHECK(hipMalloc(&dst, bytes));
    } else {
      dst = (T *)sig_out;
    }
    const int blocks = (int)std::min<long long>((s->d.N + 255) / 256, 65536);
    for (int b = 0; b < s->B; ++b) {
      const long long off = (long long)b * s->d.N;
      const T *ss = s->sstar ? (const T *)s->sstar + 6 * off : nullptr;
      hipLaunchKernelGGL(lsfft::k_hooke_out<T>, dim3(blocks), dim3(256), 0, s->stream, (const T *)s->eps + 6 * off,
                         (const T *)s->lam + off, (const T *)s->mu + off, ss, dst + 6 * off, s->d.N);
      LSFFT_CHECK(hipGetLastError());
    }
    if (host) {
      std::vector<T> tmp(n6 * s->B);
      LSFFT_CHECK(hipMemcpyAsync(tmp.data(), dst, bytes, hipMemcpyDeviceToHost, s->stream));
      LSFFT_CHECK(hipStreamSynchronize(s->stream));
      (void)hipFree(dst);
      double *o = (double *)sig_out;
      for (size_t i = 0; i < tmp.size(); ++i) o[i] = (double)tmp[i];
    }
  }
  LSFFT_CHECK(hipStreamSynchronize(s->stream));
  return LSFFT_OK;
}

bool finite_all(const double *p, long long n) {
  for (long long i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

template <typename T> lsfft_status upload_moduli(lsfft_solver s, const lsfft_config *cfg) {
  const size_t N = (size_t)s->d.N;
  std::vector<T> a(N), b(N);
  for (int m = 0; m < s->B; ++m) {
    for (size_t i = 0; i < N; ++i) {
      a[i] = (T)cfg[m].lambda[i];
      b[i] = (T)cfg[m].mu[i];
    }
    LSFFT_CHECK(hipMemcpy((T *)s->lam + m * N, a.data(), N * sizeof(T), hipMemcpyHostToDevice));
    LSFFT_CHECK(hipMemcpy((T *)s->mu + m * N, b.data(), N * sizeof(T), hipMemcpyHostToDevice));
  }
  return LSFFT_OK;
}

// y-blocks of a stencil plane: the register stencil packs several
// independent y-groups per workgroup when n1 is shorter than the workgroup.
int stencil_yblocks(const lsfft_solver s, bool f64 = false) {
  const int n1 = s->n[0];
  const int G = stencil_groups(n1);
  const int t2 = (s->prec == LSFFT_F32 && !f64) ? st2_of<float>(n1) : st2_of<double>(n1);
  return (s->n[1] + G * t2 - 1) / (G * t2);
}

// Grids of the passes for the solver's schedule: planes per stencil
// workgroup and the column-tile variants of the y and z passes.
template <typename T> lsfft_status set_grids(lsfft_solver s) {
  const int py = Launch<T>::ycols(s->n[1], s->yv);
  const int pzc = Launch<T>::zcols(s->n[2], s->zv);
  if (py <= 0 || pzc <= 0) return LSFFT_EINVAL;
  s->y_main_blocks = (6LL * s->n[2] * s->d.L + py - 1) / py;
  s->nyb = (int)(s->y_main_blocks + (6LL * s->n[2] + py - 1) / py);
  s->z_main_blocks = ((long long)s->n[1] * s->d.L + pzc - 1) / pzc;
  s->nzb = (int)(s->z_main_blocks + ((long long)s->n[1] + pzc - 1) / pzc);
  if (s->disp) {
    if (s->sZ < 2 || s->n[2] % s->sZ) return LSFFT_EINVAL;
    s->nsb = stencil_yblocks(s) * (s->n[2] / s->sZ);
    s->nub = s->nxb;
    const int pzu = Launch<T>::zucols(s->n[2], s->zv);
    if (pzu <= 0) return LSFFT_EINVAL;
    s->zu_main_blocks = ((long long)s->n[1] * s->d.L + pzu - 1) / pzu;
    s->nzub = (int)(s->zu_main_blocks + ((long long)s->n[1] + pzu - 1) / pzu);
  }
  return LSFFT_OK;
}

// Partial-sum slots per system that any schedule needs: x-pass or stencil
// workgroups (8 values each; two planes per stencil workgroup at least) and
// z-pass workgroups (one value each).
template <typename T> void partial_slots(const lsfft_solver s, long long &spx, long long &spz) {
  // (a refinement's FP64 evaluation runs the FP64 stencil on these block sums)
  const long long nsb_max =
      s->disp ? (long long)std::max(stencil_yblocks(s), s->refine ? stencil_yblocks(s, true) : 0) * (s->n[2] / 2) : 0;
  spx = 8LL * std::max<long long>(s->nxb, nsb_max);
  spz = 1;
  for (int v = 0; v < 2; ++v) {
    const int pzc = Launch<T>::zcols(s->n[2], v);
    spz = std::max<long long>(spz, ((long long)s->n[1] * s->d.L + pzc - 1) / pzc + ((long long)s->n[1] + pzc - 1) / pzc);
  }
}

template <typename T> lsfft_status upload_tables(lsfft_solver s) {
  std::vector<T> tab = axis_tables<T>(s->n, s->h, s->off, s->tabS);
  LSFFT_CHECK(hipMalloc(&s->tab, tab.size() * sizeof(T)));
  LSFFT_CHECK(hipMemcpy(s->tab, tab.data(), tab.size() * sizeof(T), hipMemcpyHostToDevice));
  auto wx = twiddles<T>(s->n[0]);
  auto wy = twiddles<T>(s->n[1]);
  auto wz = twiddles<T>(s->n[2]);
  LSFFT_CHECK(hipMalloc(&s->twx, wx.size() * sizeof(cplx<T>)));
  LSFFT_CHECK(hipMalloc(&s->twy, wy.size() * sizeof(cplx<T>)));
  LSFFT_CHECK(hipMalloc(&s->twz, wz.size() * sizeof(cplx<T>)));
  LSFFT_CHECK(hipMemcpy(s->twx, wx.data(), wx.size() * sizeof(cplx<T>), hipMemcpyHostToDevice));
  LSFFT_CHECK(hipMemcpy(s->twy, wy.data(), wy.size() * sizeof(cplx<T>), hipMemcpyHostToDevice));
  LSFFT_CHECK(hipMemcpy(s->twz, wz.data(), wz.size() * sizeof(cplx<T>), hipMemcpyHostToDevice));
  s->nxb = Launch<T>::xgrid(s->d.L, s->d.rows);
  if (s->nxb <= 0) return LSFFT_EINVAL;
  return set_grids<T>(s);
}

template <typename T> lsfft_status build_dgo(lsfft_solver s) {
  const size_t nm = 21 * (size_t)s->d.rows * s->d.L, nn = 21 * (size_t)s->d.rows;
  LSFFT_CHECK(hipMalloc(&s->dgo_main, nm * sizeof(T)));
  LSFFT_CHECK(hipMalloc(&s->dgo_nyq, nn * sizeof(T)));
  const long long nf = s->d.rows * (s->d.L + 1);
  hipLaunchKernelGGL(lsfft::k_dgo_build<T>, dim3((unsigned)((nf + 127) / 128)), dim3(128), 0, s->stream,
                     (T *)s->dgo_main, (T *)s->dgo_nyq, s->d, s->M, s->pw, s->h[0], s->h[1], s->h[2]);
  LSFFT_CHECK(hipGetLastError());
  LSFFT_CHECK(hipStreamSynchronize(s->stream));
  return LSFFT_OK;
}

void release(lsfft_solver s) {
  if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
  if (s->graph) (void)hipGraphDestroy(s->graph);
  s->graph = nullptr;
  if (s->gevent) (void)hipEventDestroy(s->gevent);
  if (s->gstream) (void)hipStreamDestroy(s->gstream);
  s->gexec = nullptr;
  s->gevent = nullptr;
  s->gstream = nullptr;
  if (s->twin) {
    release(s->twin);
    delete s->twin;
    s->twin = nullptr;
  }
  if (s->borrowed) {
    s->u = nullptr;
    s->st = nullptr;
    s->st_host = nullptr;
    s->hist = nullptr;
  }
  void *ptrs[] = {s->eps,  s->lam,      s->mu,      s->spec, s->nyq, s->tab,    s->twx, s->twy, s->twz, s->u,
                  s->dgo_main, s->dgo_nyq, s->px, s->pz,   s->pg,  s->pstage, s->st,  s->hist, s->mem, s->enorm,
                  s->sstar, s->fstar, s->smean, s->counter, s->du, s->sref, s->lam64, s->mu64, s->sstar64,
                  s->rpart, s->fref, s->mem_ref, s->rsig, s->fstar64, s->mem64};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  if (s->st_host) (void)hipHostFree(s->st_host);
  for (hipEvent_t e : s->ev) (void)hipEventDestroy(e);
  s->ev.clear();
}

template <typename T> lsfft_status stress_spectrum_impl(lsfft_solver s, const void *eps_dev, void *out) {
  s->launch_b = 1;  // the operator entry points act on system 0
  LSFFT_CHECK(Launch<T>::xpass(s, xargs<T>(s, lsfft::XMODE_EXTERNAL, eps_dev, false), s->nxb));
  LSFFT_CHECK(Launch<T>::template ypass<true>(s, yargs<T>(s, false), s->nyb));
  LSFFT_CHECK(Launch<T>::zpass(s, zargs<T>(s, false, 1), s->nzb));
  const long long total = 6LL * s->d.rows * (s->d.L + 1);
  const int blocks = (int)std::min<long long>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(lsfft::k_to_standard<T>, dim3(blocks), dim3(256), 0, s->stream, (const cplx<T> *)s->spec,
                     (const cplx<T> *)s->nyq, (cplx<T> *)out, s->d);
  LSFFT_CHECK(hipGetLastError());
  LSFFT_CHECK(hipStreamSynchronize(s->stream));
  return LSFFT_OK;
}

template <typename T> lsfft_status green_impl(lsfft_solver s, const void *in, void *out, double *res_sq) {
  const long long nf = s->d.rows * (s->d.L + 1);
  const int blocks = (int)std::min<long long>((nf + 255) / 256, s->ngb);
  lsfft::GreenParams<T> g = green_params<T>(s);
  g.scale = T(1);  // the operator entry point returns the unnormalised increment
  hipLaunchKernelGGL(lsfft::k_green_only<T>, dim3(blocks), dim3(256), 0, s->stream, (const cplx<T> *)in,
                     (cplx<T> *)out, g, s->d, s->pg);
  LSFFT_CHECK(hipGetLastError());
  std::vector<double> part(blocks);
  LSFFT_CHECK(hipMemcpyAsync(part.data(), s->pg, sizeof(double) * blocks, hipMemcpyDeviceToHost, s->stream));
  LSFFT_CHECK(hipStreamSynchronize(s->stream));
  double tot = 0.0;
  for (double v : part) tot += v;
  if (res_sq) *res_sq = tot;
  return LSFFT_OK;
}

// Eigenstrain of every system (T = C [E - E_*], Sec. 7), all in FP64 here:
// the eigenstress C E_* per voxel, which the strain form's Hooke step and
// the stress output subtract; its mean, which the displacement form takes
// out of its stress sums; and, in the displacement form, the force
// div^b (C E_*) at the nodes (the same cell-to-node stencil as the stencil
// kernel), which that kernel subtracts from div^b (C E).
template <typename T> lsfft_status setup_eigenstrain(lsfft_solver s, const lsfft_config *cfgs) {
  bool any = false;
  for (int m = 0; m < s->B; ++m) any = any || cfgs[m].eigenstrain != nullptr;
  if (!any) return LSFFT_OK;
  s->eig = 1;
  const long long N = s->d.N;
  const int n1 = s->n[0], n2 = s->n[1], n3 = s->n[2];
  const size_t B = (size_t)s->B;
  LSFFT_CHECK(hipMalloc(&s->sstar, B * 6 * (size_t)N * sizeof(T)));
  LSFFT_CHECK(hipMalloc(&s->smean, B * 6 * sizeof(double)));
  if (s->disp) LSFFT_CHECK(hipMalloc(&s->fstar, B * 3 * (size_t)N * sizeof(T)));
  if (s->refine) LSFFT_CHECK(hipMalloc(&s->sstar64, B * 6 * (size_t)N * sizeof(double)));
  if (s->refine && s->mem64) LSFFT_CHECK(hipMalloc(&s->fstar64, B * 3 * (size_t)N * sizeof(double)));
  std::vector<double> sd(6 * (size_t)N), fd(s->disp ? 3 * (size_t)N : 0), mean(6 * B, 0.0);
  std::vector<T> tmp(6 * (size_t)N);
  s->estar_rms.assign(B, 0.0);
  static const int vo[3][3] = {{0, 5, 4}, {5, 1, 3}, {4, 3, 2}};  // Voigt index of (i, j)
  for (size_t m = 0; m < B; ++m) {
    const double *es = cfgs[m].eigenstrain;
    const double *l = cfgs[m].lambda, *mu = cfgs[m].mu;
    double ss = 0.0;
    for (long long i = 0; i < N; ++i) {
      double e[6];
      for (int c = 0; c < 6; ++c) e[c] = es ? es[c * N + i] : 0.0;
      const double tr = e[0] + e[1] + e[2];
      for (int c = 0; c < 6; ++c) {
        sd[c * N + i] = (c < 3 ? l[i] * tr : 0.0) + 2.0 * mu[i] * e[c];
        mean[6 * m + c] += sd[c * N + i];
        ss += (c < 3 ? 1.0 : 2.0) * e[c] * e[c];
      }
    }
    for (int c = 0; c < 6; ++c) mean[6 * m + c] /= (double)N;
    s->estar_rms[m] = std::sqrt(ss / (double)N);
    for (size_t i = 0; i < tmp.size(); ++i) tmp[i] = (T)sd[i];
    LSFFT_CHECK(hipMemcpy((T *)s->sstar + m * 6 * N, tmp.data(), 6 * N * sizeof(T), hipMemcpyHostToDevice));
    if (s->refine)
      LSFFT_CHECK(hipMemcpy(s->sstar64 + m * 6 * N, sd.data(), 6 * N * sizeof(double), hipMemcpyHostToDevice));
    if (!s->disp) continue;
    // f_i = sum_j d_j sigma_ij at node (x, y, z), the upper corner of cells
    // (x - a, y - b, z - d), a, b, d in {0, 1}.  AFB: each d_j averages the
    // four cell differences across the node; with z-pair sums P and z
    // differences D of the cell stress these are 2 x 2 sums over (x, y).
    const double q[3] = {0.25 / s->h[0], 0.25 / s->h[1], 0.25 / s->h[2]};
    const double ih[3] = {1.0 / s->h[0], 1.0 / s->h[1], 1.0 / s->h[2]};
    for (int z = 0; z < n3; ++z) {
      const int zm = (z + n3 - 1) % n3;
      for (int y = 0; y < n2; ++y) {
        const int ym = (y + n2 - 1) % n2;
        const long long r00 = ((long long)z * n2 + y) * n1, r01 = ((long long)z * n2 + ym) * n1;
        const long long r10 = ((long long)zm * n2 + y) * n1, r11 = ((long long)zm * n2 + ym) * n1;
        for (int x = 0; x < n1; ++x) {
          const int xm = x ? x - 1 : n1 - 1;
          double f[3] = {0.0, 0.0, 0.0};
          for (int c = 0; c < 6; ++c) {
            const double *sc = sd.data() + c * N;
            double dd[3];
            if (s->scheme == LSFFT_AFB) {
              // [a][b]: cell column x - a, cell line y - b
              const double P[2][2] = {{sc[r00 + x] + sc[r10 + x], sc[r01 + x] + sc[r11 + x]},
                                      {sc[r00 + xm] + sc[r10 + xm], sc[r01 + xm] + sc[r11 + xm]}};
              const double D[2][2] = {{sc[r00 + x] - sc[r10 + x], sc[r01 + x] - sc[r11 + x]},
                                      {sc[r00 + xm] - sc[r10 + xm], sc[r01 + xm] - sc[r11 + xm]}};
              dd[0] = q[0] * ((P[0][0] + P[0][1]) - (P[1][0] + P[1][1]));
              dd[1] = q[1] * ((P[0][0] + P[1][0]) - (P[0][1] + P[1][1]));
              dd[2] = q[2] * ((D[0][0] + D[0][1]) + (D[1][0] + D[1][1]));
            } else {  // FB: backward differences of the cell stress
              const double own = sc[r00 + x];
              dd[0] = ih[0] * (own - sc[r00 + xm]);
              dd[1] = ih[1] * (own - sc[r01 + x]);
              dd[2] = ih[2] * (own - sc[r10 + x]);
            }
            for (int i = 0; i < 3; ++i)
              for (int j = 0; j < 3; ++j)
                if (vo[i][j] == c) f[i] += dd[j];
          }
          for (int i = 0; i < 3; ++i) fd[i * N + r00 + x] = f[i];
        }
      }
    }
    for (size_t i = 0; i < fd.size(); ++i) tmp[i] = (T)fd[i];
    LSFFT_CHECK(hipMemcpy((T *)s->fstar + m * 3 * N, tmp.data(), 3 * N * sizeof(T), hipMemcpyHostToDevice));
    if (s->fstar64)
      LSFFT_CHECK(hipMemcpy(s->fstar64 + m * 3 * N, fd.data(), 3 * N * sizeof(double), hipMemcpyHostToDevice));
  }
  LSFFT_CHECK(hipMemcpy(s->smean, mean.data(), mean.size() * sizeof(double), hipMemcpyHostToDevice));
  return LSFFT_OK;
}

bool ok_moduli(double l, double m) { return std::isfinite(l) && std::isfinite(m) && m > 0.0 && 3.0 * l + 2.0 * m > 0.0; }

// ------------------------------------------------------------------ schedule
template <typename T> void get_schedule(const lsfft_solver s, lsfft_schedule *out) {
  out->stencil_planes = s->disp ? s->sZ : 0;
  out->y_cols = Launch<T>::ycols(s->n[1], s->yv);
  out->z_cols = s->disp ? Launch<T>::zucols(s->n[2], s->zv) : Launch<T>::zcols(s->n[2], s->zv);
  out->xcd_order = s->xcd;
}

// Apply a schedule after checking it against the ones this grid offers.
template <typename T> lsfft_status set_schedule(lsfft_solver s, const lsfft_schedule *in) {
  int yv = -1, zv = -1;
  for (int v = 1; v >= 0; --v) {
    if (in->y_cols == Launch<T>::ycols(s->n[1], v)) yv = v;
    const int zc = s->disp ? Launch<T>::zucols(s->n[2], v) : Launch<T>::zcols(s->n[2], v);
    if (in->z_cols == zc) zv = v;
  }
  if (yv < 0 || zv < 0 || in->xcd_order < 0 || in->xcd_order > 7) return LSFFT_EINVAL;
  int z = 0;
  if (s->disp) {
    z = in->stencil_planes;
    if (z < 2 || z > s->n[2] || (z & 1) || s->n[2] % z) return LSFFT_EINVAL;
  } else if (in->stencil_planes != 0) {
    return LSFFT_EINVAL;
  }
  const int oz = s->sZ, oy = s->yv, ov = s->zv;
  if (s->disp) s->sZ = z;
  s->yv = yv;
  s->zv = zv;
  lsfft_status st = set_grids<T>(s);
  if (st != LSFFT_OK) {
    s->sZ = oz;
    s->yv = oy;
    s->zv = ov;
    (void)set_grids<T>(s);
    return st;
  }
  s->xcd = in->xcd_order;
  drop_graph(s);
  return LSFFT_OK;
}

// Milliseconds per iteration of the whole batch under the current schedule:
// the best of `reps` timed runs of `chunks` captured chunks of iterations
// (after one untimed run), on a unit axial macroscopic strain, with the
// stopping test off.
template <typename T> lsfft_status time_schedule(lsfft_solver s, int chunks, int reps, double &ms) {
  const int iters = chunks * GRAPH_CHUNK;
  double best = __builtin_huge_val();
  for (int r = 0; r <= reps; ++r) {
    LSFFT_CHECK(hipStreamSynchronize(s->stream));
    const auto t0 = std::chrono::steady_clock::now();
    lsfft_status ps = run_phase<T>(s, 0.0, iters - 1, 0, iters, true);
    if (ps != LSFFT_OK) return ps;
    LSFFT_CHECK(hipStreamSynchronize(s->stream));
    const double el = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (r > 0) best = std::min(best, el / iters);
  }
  ms = best;
  return LSFFT_OK;
}

// Coordinate search over the schedule knobs: stencil planes per workgroup,
// the two column tiles of the y and z passes, then each XCD-order bit; a
// change is kept when it is faster by more than 1 %.
template <typename T>
lsfft_status autotune(lsfft_solver s, int iterations, lsfft_schedule *best, double *start_ms, double *best_ms) {
  const int chunks = std::max(1, (iterations + GRAPH_CHUNK - 1) / GRAPH_CHUNK);
  const int reps = 3;
  lsfft_status st = ensure_hist(s, chunks * GRAPH_CHUNK);
  if (st != LSFFT_OK) return st;
  std::vector<double> eb(6 * (size_t)s->B, 0.0);
  for (int b = 0; b < s->B; ++b) eb[6 * b] = 1.0;
  st = upload_members<T>(s, eb.data());
  if (st != LSFFT_OK) return st;
  const int timing = s->timing_kernel;
  s->timing_kernel = -1;
  s->tuning = 1;
  drop_graph(s);
  lsfft_schedule cur;
  get_schedule<T>(s, &cur);
  double tcur = 0.0;
  st = time_schedule<T>(s, chunks, reps, tcur);
  const double t0 = tcur;
  auto trial = [&](const lsfft_schedule &c) -> lsfft_status {
    lsfft_status e = set_schedule<T>(s, &c);
    if (e != LSFFT_OK) return e;
    double t = 0.0;
    e = time_schedule<T>(s, chunks, reps, t);
    if (e != LSFFT_OK) return e;
    if (t < 0.99 * tcur) {
      cur = c;
      tcur = t;
    }
    return LSFFT_OK;
  };
  if (st == LSFFT_OK && s->disp) {
    // every even divisor of n3 up to 128: on 3 x 2^a and factor-9 grids the
    // best march is often one that is not a power of two (the number of
    // workgroups fills whole rounds of the CUs)
    const int z0 = cur.stencil_planes;
    for (int z = 2; z <= 128 && st == LSFFT_OK; z += 2) {
      if (z == z0 || s->n[2] % z) continue;
      lsfft_schedule c = cur;
      c.stencil_planes = z;
      st = trial(c);
    }
  }
  for (int v = 0; v < 2 && st == LSFFT_OK; ++v) {
    lsfft_schedule c = cur;
    c.y_cols = Launch<T>::ycols(s->n[1], v);
    if (c.y_cols != cur.y_cols) st = trial(c);
  }
  for (int v = 0; v < 2 && st == LSFFT_OK; ++v) {
    lsfft_schedule c = cur;
    c.z_cols = s->disp ? Launch<T>::zucols(s->n[2], v) : Launch<T>::zcols(s->n[2], v);
    if (c.z_cols != cur.z_cols) st = trial(c);
  }
  for (int bit = 0; bit < 3 && st == LSFFT_OK; ++bit) {
    if (bit == 0 && !s->disp) continue;
    lsfft_schedule c = cur;
    c.xcd_order = cur.xcd_order ^ (1 << bit);
    st = trial(c);
  }
  s->tuning = 0;
  s->timing_kernel = timing;
  lsfft_status fs = set_schedule<T>(s, &cur);
  if (st == LSFFT_OK) st = fs;
  if (st != LSFFT_OK) return st;
  if (best) *best = cur;
  if (start_ms) *start_ms = t0;
  if (best_ms) *best_ms = tcur;
  return LSFFT_OK;
}

}  // namespace

extern "C" {

const char *lsfft_version(void) { return "lsfft 0.1 (gfx950)"; }

const char *lsfft_status_string(lsfft_status st) {
  switch (st) {
    case LSFFT_OK: return "converged";
    case LSFFT_ENOTCONV: return "maximum iterations reached";
    case LSFFT_EDIVERGED: return "diverged";
    case LSFFT_EINVAL: return "invalid argument";
    case LSFFT_ENOMEM: return "device allocation failed";
    case LSFFT_EDEVICE: return "HIP runtime error";
  }
  return "unknown status";
}

const char *lsfft_kernel_name(int32_t id) {
  static const char *names[] = {"k_xpass", "k_ypass(forward)", "k_zpass", "k_ypass(inverse)", "k_uxpass",
                                "k_reduce"};
  return (id >= 0 && id < 6) ? names[id] : "none";
}

lsfft_status lsfft_create_batch(const lsfft_config *cfgs, int32_t count, lsfft_solver *out) {
  if (!cfgs || !out || count < 1 || count > 65535) return LSFFT_EINVAL;
  *out = nullptr;
  const lsfft_config *cfg = cfgs;
  for (int r = 0; r < 3; ++r) {
    if (!supported_len(cfg->n[r])) return LSFFT_EINVAL;
    if (!(cfg->h[r] >= 0.0) || !std::isfinite(cfg->h[r])) return LSFFT_EINVAL;
  }
  if (cfg->disc != LSFFT_TD && cfg->disc != LSFFT_PCD) return LSFFT_EINVAL;
  if (cfg->scheme < LSFFT_BASIC || cfg->scheme > LSFFT_ACD) return LSFFT_EINVAL;
  if ((cfg->scheme == LSFFT_CD || cfg->scheme == LSFFT_ACD) && cfg->form == 2) return LSFFT_EINVAL;
  if (cfg->prec != LSFFT_F64 && cfg->prec != LSFFT_F32) return LSFFT_EINVAL;
  if (cfg->form < 0 || cfg->form > 2) return LSFFT_EINVAL;
  if (cfg->f64_warmup < 0 || cfg->refine < 0) return LSFFT_EINVAL;
  if (!(cfg->f64_until >= 0.0) || !std::isfinite(cfg->f64_until)) return LSFFT_EINVAL;
  if (cfg->scheme == LSFFT_DGO) {
    if (cfg->disc != LSFFT_PCD) return LSFFT_EINVAL;
    if (cfg->dgo_images < 0 || cfg->dgo_images > 64) return LSFFT_EINVAL;
    if (cfg->dgo_weight_power != 1 && cfg->dgo_weight_power != 2) return LSFFT_EINVAL;
  }
  const long long N = (long long)cfg->n[0] * cfg->n[1] * cfg->n[2];
  for (int m = 0; m < count; ++m) {
    const lsfft_config *c = cfgs + m;
    if (!c->lambda || !c->mu) return LSFFT_EINVAL;
    // every system shares the grid and the solver options
    for (int r = 0; r < 3; ++r)
      if (c->n[r] != cfg->n[r] || c->h[r] != cfg->h[r]) return LSFFT_EINVAL;
    if (c->disc != cfg->disc || c->scheme != cfg->scheme || c->prec != cfg->prec || c->form != cfg->form ||
        c->dgo_images != cfg->dgo_images || c->dgo_weight_power != cfg->dgo_weight_power ||
        c->stream != cfg->stream || c->f64_warmup != cfg->f64_warmup || c->refine != cfg->refine ||
        c->f64_until != cfg->f64_until)
      return LSFFT_EINVAL;
    if (!ok_moduli(c->lambda0, c->mu0)) return LSFFT_EINVAL;
    // the DGO table depends on C0: one table, one reference medium
    if (cfg->scheme == LSFFT_DGO && (c->lambda0 != cfg->lambda0 || c->mu0 != cfg->mu0)) return LSFFT_EINVAL;
    for (long long i = 0; i < N; ++i)
      if (!ok_moduli(c->lambda[i], c->mu[i])) return LSFFT_EINVAL;
    if (c->eigenstrain && !finite_all(c->eigenstrain, 6 * N)) return LSFFT_EINVAL;
  }

  lsfft_solver s = new lsfft_solver_s();
  for (int r = 0; r < 3; ++r) {
    s->n[r] = cfg->n[r];
    s->h[r] = cfg->h[r] > 0.0 ? cfg->h[r] : 1.0;
  }
  s->B = count;
  s->launch_b = count;
  {
    const char *ng = std::getenv("LSFFT_NO_GRAPHS");
    s->use_graphs = (ng && ng[0] && ng[0] != '0') ? 0 : 1;
  }
  s->lam0 = cfg->lambda0;
  s->mu0 = cfg->mu0;
  for (int m = 0; m < count; ++m) {
    s->lam0v.push_back(cfgs[m].lambda0);
    s->mu0v.push_back(cfgs[m].mu0);
  }
  s->disc = cfg->disc;
  s->scheme = cfg->scheme;
  s->prec = cfg->prec;
  s->M = cfg->dgo_images;
  s->pw = cfg->dgo_weight_power;
  s->stream = (hipStream_t)cfg->stream;
  s->d.n1 = s->n[0];
  s->d.n2 = s->n[1];
  s->d.n3 = s->n[2];
  s->d.L = s->n[0] / 2;
  s->d.N = N;
  s->d.rows = (long long)s->n[1] * s->n[2];
  s->d.comp_main = s->d.rows * s->d.L;
  s->d.comp_nyq = s->d.rows;
  s->bs.field = N;
  s->bs.spec = 6 * s->d.comp_main;
  s->bs.nyq = 6 * s->d.comp_nyq;

  const size_t es = esize(s);
  const size_t cs = 2 * es;
  const size_t B = (size_t)count;
  lsfft_status st = LSFFT_OK;
  auto fail = [&](lsfft_status e) {
    release(s);
    delete s;
    return e;
  };
  if (hipMalloc(&s->eps, B * 6 * (size_t)N * es) != hipSuccess) return fail(LSFFT_ENOMEM);
  if (hipMalloc(&s->lam, B * (size_t)N * es) != hipSuccess) return fail(LSFFT_ENOMEM);
  if (hipMalloc(&s->mu, B * (size_t)N * es) != hipSuccess) return fail(LSFFT_ENOMEM);
  if (hipMalloc(&s->spec, B * 6 * (size_t)s->d.comp_main * cs) != hipSuccess) return fail(LSFFT_ENOMEM);
  if (hipMalloc(&s->nyq, B * 6 * (size_t)s->d.comp_nyq * cs) != hipSuccess) return fail(LSFFT_ENOMEM);
  if (hipMalloc(&s->st, B * sizeof(State)) != hipSuccess) return fail(LSFFT_ENOMEM);
  if (hipHostMalloc(&s->st_host, B * sizeof(State), 0) != hipSuccess) return fail(LSFFT_ENOMEM);
  if (hipMalloc(&s->mem, B * (s->prec == LSFFT_F32 ? sizeof(lsfft::Member<float>) : sizeof(lsfft::Member<double>))) !=
      hipSuccess)
    return fail(LSFFT_ENOMEM);
  if (hipMalloc(&s->enorm, B * sizeof(double)) != hipSuccess) return fail(LSFFT_ENOMEM);
  st = (s->prec == LSFFT_F32) ? upload_moduli<float>(s, cfgs) : upload_moduli<double>(s, cfgs);
  if (st != LSFFT_OK) return fail(st);
  st = (s->prec == LSFFT_F32) ? upload_tables<float>(s) : upload_tables<double>(s);
  if (st != LSFFT_OK) return fail(st);
  if (s->scheme == LSFFT_FB || s->scheme == LSFFT_AFB) {
    const bool fits = (s->prec == LSFFT_F32) ? stencil_fits<float>(s->n[0]) : stencil_fits<double>(s->n[0]);
    if (cfg->form == 2 && !fits) return fail(LSFFT_EINVAL);
    s->disp = (cfg->form == 1) ? 0 : (fits ? 1 : 0);
  }
  if (s->disp) {
    if (hipMalloc(&s->u, B * 3 * (size_t)N * sizeof(double)) != hipSuccess) return fail(LSFFT_ENOMEM);
    // planes per stencil workgroup: as many as keep >= 512 workgroups (over
    // the whole batch; one round of two per CU), at most 128, at least 2:
    // every workgroup evaluates one extra cell plane and loads two extra u
    // planes, so longer marches waste less
    const int ny = stencil_yblocks(s);
    int Z = 2;
    for (int c : {128, 64, 32, 16, 8, 4}) {
      if (s->n[2] % c == 0 && (long long)ny * (s->n[2] / c) * count >= 512) {
        Z = c;
        break;
      }
    }
    s->sZ = Z;
    if (hipMalloc(&s->counter, B * sizeof(unsigned)) != hipSuccess) return fail(LSFFT_ENOMEM);
    if (hipMemset(s->counter, 0, B * sizeof(unsigned)) != hipSuccess) return fail(LSFFT_EDEVICE);
  }
  if (cfg->refine > 0 && s->prec == LSFFT_F32) {
    if (!s->disp) return fail(LSFFT_EINVAL);
    s->refine = cfg->refine;
    const size_t n3 = B * 3 * (size_t)N;
    s->nrb = (int)std::min<long long>((N + 255) / 256, 2048);
    // the FP64 residual evaluation: the FP64 register stencil where it runs
    // at this n1, else the cell-stress and divergence kernels
    const bool reg64 = stencil_reg_kernel(s->n[0]) && stencil_fits<double>(s->n[0]);
    if (hipMalloc(&s->du, n3 * sizeof(double)) != hipSuccess) return fail(LSFFT_ENOMEM);
    if (reg64) {
      if (hipMalloc(&s->mem64, B * sizeof(lsfft::Member<double>)) != hipSuccess) return fail(LSFFT_ENOMEM);
    } else if (hipMalloc(&s->rsig, 2 * n3 * sizeof(double)) != hipSuccess) {
      return fail(LSFFT_ENOMEM);
    }
    if (hipMalloc(&s->fref, n3 * sizeof(float)) != hipSuccess) return fail(LSFFT_ENOMEM);
    if (hipMalloc(&s->sref, B * 6 * sizeof(double)) != hipSuccess) return fail(LSFFT_ENOMEM);
    if (hipMalloc(&s->lam64, B * (size_t)N * sizeof(double)) != hipSuccess) return fail(LSFFT_ENOMEM);
    if (hipMalloc(&s->mu64, B * (size_t)N * sizeof(double)) != hipSuccess) return fail(LSFFT_ENOMEM);
    if (!reg64 && hipMalloc(&s->rpart, B * (size_t)s->nrb * 8 * sizeof(double)) != hipSuccess)
      return fail(LSFFT_ENOMEM);
    if (hipMalloc(&s->mem_ref, B * sizeof(lsfft::Member<float>)) != hipSuccess) return fail(LSFFT_ENOMEM);
    // defined contents for the schedule tuner, which times the sweeps alone
    if (hipMemset(s->du, 0, n3 * sizeof(double)) != hipSuccess) return fail(LSFFT_EDEVICE);
    if (hipMemset(s->fref, 0, n3 * sizeof(float)) != hipSuccess) return fail(LSFFT_EDEVICE);
    if (hipMemset(s->sref, 0, B * 6 * sizeof(double)) != hipSuccess) return fail(LSFFT_EDEVICE);
    for (size_t m = 0; m < B; ++m) {
      if (hipMemcpy(s->lam64 + m * N, cfgs[m].lambda, N * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(s->mu64 + m * N, cfgs[m].mu, N * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
        return fail(LSFFT_EDEVICE);
    }
  }
  st = (s->prec == LSFFT_F32) ? set_grids<float>(s) : set_grids<double>(s);
  if (st != LSFFT_OK) return fail(st);
  if (s->prec == LSFFT_F32)
    partial_slots<float>(s, s->spx, s->spz);
  else
    partial_slots<double>(s, s->spx, s->spz);
  if (hipMalloc(&s->px, sizeof(double) * B * (size_t)s->spx) != hipSuccess) return fail(LSFFT_ENOMEM);
  if (hipMalloc(&s->pz, sizeof(double) * B * (size_t)s->spz) != hipSuccess) return fail(LSFFT_ENOMEM);
  if (hipMalloc(&s->pstage, sizeof(double) * B * 8 * lsfft::RSTAGE) != hipSuccess) return fail(LSFFT_ENOMEM);
  s->ngb = 1024;
  if (hipMalloc(&s->pg, sizeof(double) * (size_t)s->ngb) != hipSuccess) return fail(LSFFT_ENOMEM);
  st = (s->prec == LSFFT_F32) ? setup_eigenstrain<float>(s, cfgs) : setup_eigenstrain<double>(s, cfgs);
  if (st != LSFFT_OK) return fail(st);
  // reference media of the systems for the operator entry points and the DGO
  st = (s->prec == LSFFT_F32) ? upload_members<float>(s, nullptr) : upload_members<double>(s, nullptr);
  if (st != LSFFT_OK) return fail(st);
  if (s->scheme == LSFFT_DGO) {
    st = (s->prec == LSFFT_F32) ? build_dgo<float>(s) : build_dgo<double>(s);
    if (st != LSFFT_OK) return fail(st);
  }
  if ((cfg->f64_warmup > 0 || cfg->f64_until > 0.0) && s->prec == LSFFT_F32 && s->disp &&
      stencil_fits<double>(s->n[0])) {
    std::vector<lsfft_config> c2(cfgs, cfgs + count);
    for (auto &c : c2) {
      c.prec = LSFFT_F64;
      c.form = 2;
      c.f64_warmup = 0;
      c.f64_until = 0.0;
    }
    lsfft_solver t = nullptr;
    st = lsfft_create_batch(c2.data(), count, &t);
    if (st != LSFFT_OK) return fail(st);
    (void)hipFree(t->u);
    (void)hipFree(t->st);
    (void)hipHostFree(t->st_host);
    t->u = s->u;
    t->st = s->st;
    t->st_host = s->st_host;
    t->borrowed = 1;
    s->twin = t;
    s->warm = cfg->f64_warmup;
    s->until = cfg->f64_until;
  }
  *out = s;
  return LSFFT_OK;
}

lsfft_status lsfft_create(const lsfft_config *cfg, lsfft_solver *out) { return lsfft_create_batch(cfg, 1, out); }

static lsfft_status check_solve_args(lsfft_solver s, const double *Eb, double tol, int32_t maxit) {
  if (!s || !Eb) return LSFFT_EINVAL;
  if (!(tol >= 0.0) || !std::isfinite(tol) || maxit < 0) return LSFFT_EINVAL;
  if (!finite_all(Eb, 6LL * s->B)) return LSFFT_EINVAL;
  return LSFFT_OK;
}

// Eb [B][6]; outputs of every system: eps, sig [B][6][N], sig_mean [B][6],
// iters, residual, status [B] (each may be null).
static lsfft_status solve_common(lsfft_solver s, const double *Ebar, double tol, int32_t maxit, void *eps,
                                 void *sig, double *sig_mean, int32_t *iters, double *residual, int32_t *status,
                                 bool host) {
  lsfft_status st = check_solve_args(s, Ebar, tol, maxit);
  if (st != LSFFT_OK) return st;
  lsfft_status rs = (s->prec == LSFFT_F32) ? run_solve<float>(s, Ebar, tol, maxit)
                                           : run_solve<double>(s, Ebar, tol, maxit);
  if (rs < 0) return rs;
  lsfft_status os = (s->prec == LSFFT_F32) ? finish_outputs<float>(s, eps, sig, host, Ebar)
                                           : finish_outputs<double>(s, eps, sig, host, Ebar);
  if (os != LSFFT_OK) return os;
  for (int b = 0; b < s->B; ++b) {
    const State &x = s->st_host[b];
    if (sig_mean)
      for (int c = 0; c < 6; ++c) sig_mean[6 * b + c] = x.sig_mean[c];
    if (iters) iters[b] = x.iters;
    if (residual) residual[b] = x.r;
    if (status) status[b] = x.status;
  }
  return rs;
}

lsfft_status lsfft_solve(lsfft_solver s, const double Ebar[6], double tol, int32_t maxit, double *eps, double *sig,
                         double sig_mean[6], int32_t *iters, double *residual) {
  if (s && s->B != 1) return LSFFT_EINVAL;
  return solve_common(s, Ebar, tol, maxit, eps, sig, sig_mean, iters, residual, nullptr, true);
}

lsfft_status lsfft_solve_device(lsfft_solver s, const double Ebar[6], double tol, int32_t maxit, void *eps_dev,
                                void *sig_dev, double sig_mean[6], int32_t *iters, double *residual) {
  if (s && s->B != 1) return LSFFT_EINVAL;
  return solve_common(s, Ebar, tol, maxit, eps_dev, sig_dev, sig_mean, iters, residual, nullptr, false);
}

lsfft_status lsfft_solve_batch(lsfft_solver s, const double *Ebar, double tol, int32_t maxit, void *eps_dev,
                               void *sig_dev, double *sig_mean, int32_t *iters, double *residual, int32_t *status) {
  return solve_common(s, Ebar, tol, maxit, eps_dev, sig_dev, sig_mean, iters, residual, status, false);
}

lsfft_status lsfft_solve_group(const lsfft_solver *handles, int32_t count, const double *Ebar, double tol,
                               int32_t maxit, const int32_t *maxit_each, void *const *eps_dev, double *sig_mean,
                               int32_t *iters, double *residual, int32_t *status) {
  if (!handles || !Ebar || count < 1 || count > 64) return LSFFT_EINVAL;
  if (!(tol >= 0.0) || !std::isfinite(tol) || maxit < 0) return LSFFT_EINVAL;
  std::vector<lsfft_solver> hs(handles, handles + count);
  std::vector<int> maxits(count, maxit);
  long long total = 0;
  for (int i = 0; i < count; ++i) {
    if (maxit_each) maxits[i] = maxit_each[i];
    if (maxits[i] < 0) return LSFFT_EINVAL;
    if (!hs[i] || hs[i]->refine > 0) return LSFFT_EINVAL;
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i]) return LSFFT_EINVAL;
    total += hs[i]->B;
  }
  if (!finite_all(Ebar, 6 * total)) return LSFFT_EINVAL;
  // the group replays captured chunks: per-kernel event timing stays off
  std::vector<int> timing(count);
  for (int i = 0; i < count; ++i) {
    timing[i] = hs[i]->timing_kernel;
    hs[i]->timing_kernel = -1;
  }
  lsfft_status st = solve_group(hs, Ebar, tol, maxits);
  for (int i = 0; i < count; ++i) hs[i]->timing_kernel = timing[i];
  if (st < 0) return st;
  int worst = 0;
  long long off = 0;
  for (int i = 0; i < count; ++i) {
    lsfft_solver s = hs[i];
    void *e = eps_dev ? eps_dev[i] : nullptr;
    lsfft_status os = (s->prec == LSFFT_F32) ? finish_outputs<float>(s, e, nullptr, false, Ebar + 6 * off)
                                             : finish_outputs<double>(s, e, nullptr, false, Ebar + 6 * off);
    if (os != LSFFT_OK) return os;
    for (int b = 0; b < s->B; ++b, ++off) {
      const State &x = s->st_host[b];
      if (sig_mean)
        for (int c = 0; c < 6; ++c) sig_mean[6 * off + c] = x.sig_mean[c];
      if (iters) iters[off] = x.iters;
      if (residual) residual[off] = x.r;
      if (status) status[off] = x.status;
      worst = std::max(worst, x.status);
    }
  }
  return (lsfft_status)worst;
}

int32_t lsfft_batch_size(lsfft_solver s) { return s ? s->B : 0; }

lsfft_status lsfft_get_schedule(lsfft_solver s, lsfft_schedule *out) {
  if (!s || !out) return LSFFT_EINVAL;
  if (s->prec == LSFFT_F32)
    get_schedule<float>(s, out);
  else
    get_schedule<double>(s, out);
  return LSFFT_OK;
}

lsfft_status lsfft_set_schedule(lsfft_solver s, const lsfft_schedule *sch) {
  if (!s || !sch) return LSFFT_EINVAL;
  return (s->prec == LSFFT_F32) ? set_schedule<float>(s, sch) : set_schedule<double>(s, sch);
}

lsfft_status lsfft_autotune(lsfft_solver s, int32_t iterations, lsfft_schedule *best, double *start_ms,
                            double *best_ms) {
  if (!s || iterations < 1 || iterations > 4096) return LSFFT_EINVAL;
  return (s->prec == LSFFT_F32) ? autotune<float>(s, iterations, best, start_ms, best_ms)
                                : autotune<double>(s, iterations, best, start_ms, best_ms);
}

lsfft_status lsfft_residual_history(lsfft_solver s, double *out, int32_t cap, int32_t *count) {
  if (!s || !out || cap < 0 || s->last_iters < 0) return LSFFT_EINVAL;
  const int n = std::min(cap, s->last_iters + 1);
  if (count) *count = s->last_iters + 1;
  if (n > 0) {
    LSFFT_CHECK(hipMemcpyAsync(out, s->hist, sizeof(double) * n, hipMemcpyDeviceToHost, s->stream));
    LSFFT_CHECK(hipStreamSynchronize(s->stream));
  }
  return LSFFT_OK;
}

lsfft_status lsfft_stress_spectrum(lsfft_solver s, const void *eps_dev, void *sig_hat_dev) {
  if (!s || !eps_dev || !sig_hat_dev) return LSFFT_EINVAL;
  return (s->prec == LSFFT_F32) ? stress_spectrum_impl<float>(s, eps_dev, sig_hat_dev)
                                : stress_spectrum_impl<double>(s, eps_dev, sig_hat_dev);
}

lsfft_status lsfft_green_apply(lsfft_solver s, const void *in_dev, void *out_dev, double *res_sq) {
  if (!s || !in_dev || !out_dev) return LSFFT_EINVAL;
  return (s->prec == LSFFT_F32) ? green_impl<float>(s, in_dev, out_dev, res_sq)
                                : green_impl<double>(s, in_dev, out_dev, res_sq);
}

lsfft_status lsfft_stiffness_gradient(lsfft_solver s, const void *eps_a_dev, const void *eps_b_dev,
                                      void *dj_dlambda_dev, void *dj_dmu_dev, void *dj_dyoung_dev) {
  if (!s || !eps_a_dev || !eps_b_dev) return LSFFT_EINVAL;
  const int blocks = (int)std::min<long long>((s->d.N + 255) / 256, 65536);
  if (s->prec == LSFFT_F32)
    hipLaunchKernelGGL(lsfft::k_stiffness_gradient<float>, dim3(blocks), dim3(256), 0, s->stream,
                       (const float *)eps_a_dev, (const float *)eps_b_dev, (const float *)s->lam,
                       (const float *)s->mu, (float *)dj_dlambda_dev, (float *)dj_dmu_dev, (float *)dj_dyoung_dev,
                       s->d.N);
  else
    hipLaunchKernelGGL(lsfft::k_stiffness_gradient<double>, dim3(blocks), dim3(256), 0, s->stream,
                       (const double *)eps_a_dev, (const double *)eps_b_dev, (const double *)s->lam,
                       (const double *)s->mu, (double *)dj_dlambda_dev, (double *)dj_dmu_dev,
                       (double *)dj_dyoung_dev, s->d.N);
  LSFFT_CHECK(hipGetLastError());
  LSFFT_CHECK(hipStreamSynchronize(s->stream));
  return LSFFT_OK;
}

lsfft_status lsfft_describe(lsfft_solver s, char *buf, int32_t cap) {
  if (!s || !buf || cap < 1) return LSFFT_EINVAL;
  const std::string d = s->prec == LSFFT_F32 ? Launch<float>::describe(s) : Launch<double>::describe(s);
  if ((long long)d.size() + 1 > cap) return LSFFT_EINVAL;
  memcpy(buf, d.c_str(), d.size() + 1);
  return LSFFT_OK;
}

lsfft_status lsfft_set_timing(lsfft_solver s, int32_t kernel_id) {
  if (!s || kernel_id < -1 || kernel_id > 5) return LSFFT_EINVAL;
  s->timing_kernel = kernel_id;
  s->timing_mean = 0.0;
  s->timing_count = 0;
  return LSFFT_OK;
}

lsfft_status lsfft_get_timing(lsfft_solver s, double *mean_ms, int32_t *launches) {
  if (!s) return LSFFT_EINVAL;
  if (mean_ms) *mean_ms = s->timing_mean;
  if (launches) *launches = s->timing_count;
  return LSFFT_OK;
}

lsfft_status lsfft_destroy(lsfft_solver s) {
  if (!s) return LSFFT_OK;
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  else (void)hipDeviceSynchronize();
  release(s);
  delete s;
  return LSFFT_OK;
}

}  // extern "C"
