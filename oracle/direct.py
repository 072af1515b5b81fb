"""Independent routes to the same discrete solutions.  TEST INFRASTRUCTURE ONLY.

The fixed points of Sec. 5.2 / Sec. 5.4 are the solutions of linear systems;
these functions solve those systems by other algorithms, so that the
fixed-point oracle can be checked against something other than itself.

* `dense_gfp`: assembles, column by column, the map
      u_check -> (F^- C : F^+ sym(u_check (x) q^a)) q^b
  on the non-singular frequencies (the discrete equilibrium operator behind
  eq. (33)-(34)) and solves  A u = -(F^- C Ebar) q^b  by dense LU.  Tiny grids.
* `dense_dgo`: assembles eps -> Ebar + F^{c+} Gamma^c F^{c-} (C - C_H) eps and
  solves (I - L) eps = Ebar by dense LU.  Tiny grids.
* `pcg_gfp`: conjugate gradients on the same equilibrium equations for a
  conjugate pair q^b = conj(q^a) (Hermitian positive semidefinite operator),
  preconditioned by the reference-medium Green function (Zeman et al. 2010
  style FFT-based CG; the paper mentions CG solvers in Sec. 1).
"""
from __future__ import annotations

import numpy as np

from . import fdd, fourier
from .green import from_voigt, sym_outer, to_voigt, green_inverse
from .solve3d import _transform, _ebar_matrix, eigenstrain_field, hooke


def _apply_equilibrium(u, lam, mu, qa, qb, disc):
    """(F^- C : F^+ sym(u (x) q^a)) q^b, complex-linear in u (no real part taken)."""
    E = _transform(sym_outer(u, qa), forward=False, disc=disc)
    T = hooke(lam, mu, E)
    That = _transform(T, forward=True, disc=disc)
    return np.einsum("...ij,...j->...i", That, qb)


def dense_gfp(lam, mu, Ebar, scheme="AFB", disc="TD", h=(1.0, 1.0, 1.0), eigenstrain=None):
    """Strain field (6, n3, n2, n1) of the discrete equilibrium, by dense LU.
    With an eigenstrain E_* the load is the stress C [Ebar - E_*]."""
    n3, n2, n1 = lam.shape
    qa, qb = fdd.scheme_pair(scheme, (n1, n2, n3), h)
    sing = fdd.singular_mask(qa, qb)
    idx = np.argwhere(~sing)
    m = idx.shape[0] * 3
    A = np.zeros((m, m), dtype=np.complex128)
    col = 0
    for (a, b, c) in idx:
        for i in range(3):
            u = np.zeros((n3, n2, n1, 3), dtype=np.complex128)
            u[a, b, c, i] = 1.0
            out = _apply_equilibrium(u, lam, mu, qa, qb, disc)
            A[:, col] = out[~sing].ravel()
            col += 1
    Eb = _ebar_matrix(Ebar)
    Es = eigenstrain_field(eigenstrain, lam.shape)
    load = np.broadcast_to(Eb, (n3, n2, n1, 3, 3)) - (Es if Es is not None else 0.0)
    T0 = hooke(lam, mu, load)
    rhs = -np.einsum("...ij,...j->...i", _transform(T0, True, disc), qb)[~sing].ravel()
    sol = np.linalg.solve(A, rhs)
    u = np.zeros((n3, n2, n1, 3), dtype=np.complex128)
    u[~sing] = sol.reshape(-1, 3)
    E = Eb + _transform(sym_outer(u, qa), forward=False, disc=disc).real
    return np.moveaxis(to_voigt(E), -1, 0)


def dense_dgo(lam, mu, Ebar, lam0, mu0, Gc, disc="PCD", eigenstrain=None):
    """DGO fixed point (I - L) eps = Ebar by dense LU; Gc as in solve3d.solve_dgo.
    With an eigenstrain E_*: (I - L) eps = Ebar - G(C E_*), G the Green map."""
    n3, n2, n1 = lam.shape
    N = n1 * n2 * n3
    dlam, dmu = lam - lam0, mu - mu0

    def G(tv):  # polarisation (6, n3, n2, n1) Voigt -> strain, same layout
        th = fourier.pcd_forward(tv) if disc == "PCD" else fourier.td_forward(tv)
        eh = np.einsum("...IJ,J...->I...", Gc, th)
        return (fourier.pcd_inverse(eh) if disc == "PCD" else fourier.td_inverse(eh)).real

    def L(ev):  # ev: (6, n3, n2, n1) Voigt -> same
        tau = hooke(dlam, dmu, from_voigt(np.moveaxis(ev, 0, -1)))
        return G(np.moveaxis(to_voigt(tau), -1, 0))

    A = np.zeros((6 * N, 6 * N))
    for j in range(6 * N):
        e = np.zeros(6 * N)
        e[j] = 1.0
        A[:, j] = e - L(e.reshape(6, n3, n2, n1)).ravel()
    rhs = np.broadcast_to(np.asarray(Ebar, dtype=np.float64)[:, None], (6, N)).ravel()
    Es = eigenstrain_field(eigenstrain, lam.shape)
    if Es is not None:
        rhs = rhs - G(np.moveaxis(to_voigt(hooke(lam, mu, Es)), -1, 0)).ravel()
    return np.linalg.solve(A, rhs).reshape(6, n3, n2, n1)


def pcg_gfp(lam, mu, Ebar, lam0, mu0, scheme="AFB_conj", tol=1e-12, maxit=5000,
            disc="TD", h=(1.0, 1.0, 1.0)):
    """Preconditioned CG for a conjugate pair; returns (eps (6,...), iterations)."""
    n3, n2, n1 = lam.shape
    qa, qb = fdd.scheme_pair(scheme, (n1, n2, n3), h)
    if not np.allclose(qb, np.conj(qa)):
        raise ValueError("pcg_gfp needs a conjugate pair q^b = conj(q^a)")
    sing = fdd.singular_mask(qa, qb)
    ok = ~sing
    K0 = -green_inverse(qa[ok], qb[ok], lam0, mu0)      # reference operator, HPD

    def prec(r):
        z = np.zeros_like(r)
        z[ok] = np.linalg.solve(K0, r[ok][..., None])[..., 0]
        return z

    def A(u):
        out = _apply_equilibrium(u, lam, mu, qa, qb, disc)
        out[sing] = 0.0
        return out

    Eb = _ebar_matrix(Ebar)
    T0 = hooke(lam, mu, np.broadcast_to(Eb, (n3, n2, n1, 3, 3)))
    b = -np.einsum("...ij,...j->...i", _transform(T0, True, disc), qb)
    b[sing] = 0.0
    u = np.zeros_like(b)
    r = b.copy()
    z = prec(r)
    p = z.copy()
    rz = np.vdot(r, z)
    bn = np.linalg.norm(b)
    it = 0
    while np.linalg.norm(r) > tol * bn and it < maxit:
        Ap = A(p)
        alpha = rz / np.vdot(p, Ap)
        u += alpha * p
        r -= alpha * Ap
        z = prec(r)
        rz_new = np.vdot(r, z)
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
    E = Eb + _transform(sym_outer(u, qa), forward=False, disc=disc).real
    return np.moveaxis(to_voigt(E), -1, 0), it
