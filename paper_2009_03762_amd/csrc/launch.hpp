// Definitions of the pass-kernel launches, instantiated once per precision
// by launch_f32.hip and launch_f64.hip.
#pragma once
#include <hip/hip_ext.h>

#include <cstdio>

#include "solver.hpp"

// A pass launch on the solver's stream; while the solver times this pass
// (s->tstart set), the launch itself records the start and stop events.
#define LSFFT_LAUNCH(kernel, grid, block, s, a)                                                          \
  do {                                                                                                   \
    if ((s)->tstart)                                                                                     \
      hipExtLaunchKernelGGL(kernel, grid, block, 0, (s)->stream, (s)->tstart, (s)->tstop, 0, a);         \
    else                                                                                                 \
      hipLaunchKernelGGL(kernel, grid, block, 0, (s)->stream, a);                                        \
  } while (0)

namespace lsfft_host {

template <typename T>
hipError_t Launch<T>::xpass(lsfft_solver s, const lsfft::XArgs<T> &a, int grid) {
  switch (s->d.L) {
#define XCASE(Lv)                                                                                        \
case Lv:                                                                                               \
  if (a.sstar)                                                                                           \
    LSFFT_LAUNCH((lsfft::k_xpass<T, Lv, ex_of(Lv), XWG, true>), dim3(grid, s->launch_b), dim3(XWG), s, a);                                                                    \
  else                                                                                                   \
    LSFFT_LAUNCH((lsfft::k_xpass<T, Lv, ex_of(Lv), XWG, false>), dim3(grid, s->launch_b), dim3(XWG), s, a);                                                                    \
  return hipGetLastError();
    LSFFT_X_LENGTHS(XCASE)
#undef XCASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T> template <bool FWD>
hipError_t Launch<T>::ypass(lsfft_solver s, const lsfft::YArgs<T> &a, int grid) {
  switch (s->d.n2) {
#define YCASE(Nv)                                                                                      \
case Nv: {                                                                                           \
  constexpr int E = ey_of(Nv), P0 = pcols<T>(Nv, E), P1 = palt<T>(Nv, E, P0);                        \
  if (s->yv)                                                                                         \
    LSFFT_LAUNCH((lsfft::k_ypass<T, Nv, E, P1, FWD>), dim3(grid, s->launch_b), dim3(P1 * (Nv / E)), s, a);                                                                \
  else                                                                                               \
    LSFFT_LAUNCH((lsfft::k_ypass<T, Nv, E, P0, FWD>), dim3(grid, s->launch_b), dim3(P0 * (Nv / E)), s, a);                                                                \
  return hipGetLastError();                                                                          \
}
    LSFFT_YZ_LENGTHS(YCASE)
#undef YCASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t Launch<T>::zpass(lsfft_solver s, const lsfft::ZArgs<T> &a, int grid) {
  switch (s->d.n3) {
#define ZCASE(Nv)                                                                                      \
case Nv: {                                                                                           \
  constexpr int E = ez_of(Nv), P0 = pcols_z<T>(Nv, E), P1 = palt<T>(Nv, E, P0);                      \
  if (s->scheme == LSFFT_AFB && s->zv)                                                               \
    LSFFT_LAUNCH((lsfft::k_zpass<T, Nv, E, P1, lsfft::SCHEME_AFB>), dim3(grid, s->launch_b),                 \
                 dim3(P1 * (Nv / E)), s, a);                                                         \
  else if (s->scheme == LSFFT_AFB)                                                                   \
    LSFFT_LAUNCH((lsfft::k_zpass<T, Nv, E, P0, lsfft::SCHEME_AFB>), dim3(grid, s->launch_b),                 \
                 dim3(P0 * (Nv / E)), s, a);                                                         \
  else if (s->zv)                                                                                    \
    LSFFT_LAUNCH((lsfft::k_zpass<T, Nv, E, P1, -1>), dim3(grid, s->launch_b), dim3(P1 * (Nv / E)), s, a);                                                                           \
  else                                                                                               \
    LSFFT_LAUNCH((lsfft::k_zpass<T, Nv, E, P0, -1>), dim3(grid, s->launch_b), dim3(P0 * (Nv / E)), s, a);                                                                           \
  return hipGetLastError();                                                                          \
}
    LSFFT_YZ_LENGTHS(ZCASE)
#undef ZCASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t Launch<T>::uxpass(lsfft_solver s, const lsfft::UArgs<T> &a, int grid) {
  switch (s->d.L) {
#define UCASE(Lv)                                                                                         \
case Lv:                                                                                                \
  LSFFT_LAUNCH((lsfft::k_uxpass<T, Lv, ex_of(Lv), XWG>), dim3(grid, s->launch_b), dim3(XWG), s, a); \
  return hipGetLastError();
    LSFFT_X_LENGTHS(UCASE)
#undef UCASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T> template <int SCH>
hipError_t Launch<T>::stencil_s(lsfft_solver s, const lsfft::SArgs<T> &a, int grid) {
  switch (s->n[0]) {
#define SCASE(Lv)                                                                                      \
case 2 * Lv:                                                                                         \
  if constexpr (stencil_fits<T>(2 * Lv) && stencil_reg_kernel(2 * Lv)) {                            \
    if (a.fstar)                                                                                     \
      LSFFT_LAUNCH((lsfft::k_stencil_reg<T, 2 * Lv, esr_of(Lv), SCH, st2_of<T>(2 * Lv), true>),                     \
                   dim3(grid, s->launch_b), dim3(lsfft::stencil_wg_of(2 * Lv)), s, a);                                \
    else                                                                                             \
      LSFFT_LAUNCH((lsfft::k_stencil_reg<T, 2 * Lv, esr_of(Lv), SCH, st2_of<T>(2 * Lv), false>),                    \
                   dim3(grid, s->launch_b), dim3(lsfft::stencil_wg_of(2 * Lv)), s, a);                                \
    return hipGetLastError();                                                                        \
  } else if constexpr (stencil_fits<T>(2 * Lv)) {                                                    \
    LSFFT_LAUNCH((lsfft::k_stencil<T, 2 * Lv, es_of(Lv), SCH, st2_of<T>(2 * Lv)>), dim3(grid, s->launch_b),       \
                 dim3(256), s, a);                                                                                    \
    return hipGetLastError();                                                                        \
  } else {                                                                                           \
    return hipErrorInvalidValue;                                                                     \
  }
    LSFFT_X_LENGTHS(SCASE)
#undef SCASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t Launch<T>::stencil(lsfft_solver s, const lsfft::SArgs<T> &a, int grid) {
  return s->scheme == LSFFT_FB ? stencil_s<lsfft::SCHEME_FB>(s, a, grid) : stencil_s<lsfft::SCHEME_AFB>(s, a, grid);
}

template <typename T> template <int SCH>
hipError_t Launch<T>::zpass_u_s(lsfft_solver s, const lsfft::ZArgs<T> &a, int grid) {
  switch (s->d.n3) {
#define ZUCASE(Nv)                                                                                     \
case Nv: {                                                                                           \
  constexpr int E = ezu_of<T>(Nv), P0 = pcols_zu<T>(Nv, E), P1 = palt<T>(Nv, E, P0);                    \
  if (s->zv)                                                                                         \
    LSFFT_LAUNCH((lsfft::k_zpass_u<T, Nv, E, P1, SCH>), dim3(grid, s->launch_b), dim3(P1 * (Nv / E)), s, a);                                                                \
  else                                                                                               \
    LSFFT_LAUNCH((lsfft::k_zpass_u<T, Nv, E, P0, SCH>), dim3(grid, s->launch_b), dim3(P0 * (Nv / E)), s, a);                                                                \
  return hipGetLastError();                                                                          \
}
    LSFFT_YZ_LENGTHS(ZUCASE)
#undef ZUCASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t Launch<T>::zpass_u(lsfft_solver s, const lsfft::ZArgs<T> &a, int grid) {
  return s->scheme == LSFFT_FB ? zpass_u_s<lsfft::SCHEME_FB>(s, a, grid) : zpass_u_s<lsfft::SCHEME_AFB>(s, a, grid);
}

template <typename T> std::string Launch<T>::describe(lsfft_solver s) {
  const char *tn = sizeof(T) == 4 ? "float" : "double";
  const char *sch = s->scheme == LSFFT_FB ? "FB" : "AFB";
  char b[128];
  std::string x, y, z, u;
  if (s->disp) {
    switch (s->n[0]) {
#define SD(Lv)                                                                                          \
case 2 * Lv:                                                                                           \
  if (stencil_reg_kernel(2 * Lv))                                                                      \
    snprintf(b, sizeof b, "k_stencil_reg<%s,%d,%d,%s,%d>", tn, 2 * Lv, esr_of(Lv), sch, st2_of<T>(2 * Lv)); \
  else                                                                                                 \
    snprintf(b, sizeof b, "k_stencil<%s,%d,%d,%s,%d>", tn, 2 * Lv, es_of(Lv), sch, st2_of<T>(2 * Lv)); \
  x = b;                                                                                               \
  snprintf(b, sizeof b, "k_uxpass<%s,%d,%d,%d>", tn, Lv, ex_of(Lv), XWG);                              \
  u = b;                                                                                               \
  break;
      LSFFT_X_LENGTHS(SD)
#undef SD
      default:
        break;
    }
    switch (s->d.n3) {
#define ZUD(Nv)                                                                                         \
case Nv: {                                                                                            \
  constexpr int E = ezu_of<T>(Nv), P0 = pcols_zu<T>(Nv, E), P1 = palt<T>(Nv, E, P0);                     \
  snprintf(b, sizeof b, "k_zpass_u<%s,%d,%d,%d,%s>", tn, Nv, E, s->zv ? P1 : P0, sch);                    \
  z = b;                                                                                              \
  break;                                                                                              \
}
      LSFFT_YZ_LENGTHS(ZUD)
#undef ZUD
      default:
        break;
    }
  } else {
    switch (s->d.L) {
#define XD(Lv)                                                                                \
case Lv:                                                                                     \
  snprintf(b, sizeof b, "k_xpass<%s,%d,%d,%d,%d>", tn, Lv, ex_of(Lv), XWG, s->eig ? 1 : 0); \
  x = b;                                                                                     \
  break;
      LSFFT_X_LENGTHS(XD)
#undef XD
      default:
        break;
    }
    switch (s->d.n3) {
#define ZD(Nv)                                                                                    \
case Nv: {                                                                                      \
  constexpr int E = ez_of(Nv), P0 = pcols_z<T>(Nv, E), P1 = palt<T>(Nv, E, P0);                   \
  snprintf(b, sizeof b, "k_zpass<%s,%d,%d,%d>", tn, Nv, E, s->zv ? P1 : P0);                      \
  z = b;                                                                                        \
  break;                                                                                        \
}
      LSFFT_YZ_LENGTHS(ZD)
#undef ZD
      default:
        break;
    }
  }
  switch (s->d.n2) {
#define YD(Nv)                                                                                  \
case Nv: {                                                                                    \
  constexpr int E = ey_of(Nv), P0 = pcols<T>(Nv, E), P1 = palt<T>(Nv, E, P0);                 \
  snprintf(b, sizeof b, "k_ypass<%s,%d,%d,%d>", tn, Nv, E, s->yv ? P1 : P0);                    \
  y = b;                                                                                      \
  break;                                                                                      \
}
    LSFFT_YZ_LENGTHS(YD)
#undef YD
    default:
      break;
  }
  return s->disp ? x + " " + y + " " + z + " " + y + " " + u : x + " " + y + " " + z + " " + y;
}

}  // namespace lsfft_host
