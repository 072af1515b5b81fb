"""The 3D fixed-point algorithms, FP64.  TEST INFRASTRUCTURE ONLY.

`solve_gfp` follows the displacement-based TD algorithm of Sec. 5.2 (the 3D
trapezoidal GFP+FDD algorithm, Algorithm 2 of the trapezoidal series) and,
with disc="PCD", its cell-centred twin of Sec. 5.4 (Algorithm 2 of the PCD
series).  `solve_dgo` follows the DGO algorithm of Sec. 5.4 (Algorithm 2 of
the DGO series) in the polarisation form that the paper's footnote in Sec. 3.3
attributes to Eloh et al.

Readings taken where the paper is silent or garbled (each is also listed in
the design notes of the repository):
  * iteration indexing: u^(k+1) = u^(k) + Delta u^(k), u^(0) = 0;
  * stopping test: the relative equilibrium norm
        r_k = sqrt(sum_xi |T_check(xi) q^b(xi)|^2) / |T_check(0)|_F,
    evaluated on T^(k) before the update; the iterate returned is the one
    whose residual is reported, and `iters` counts the updates applied.  The
    paper's own test (an L1 norm of successive Green increments) is kept as
    stop="paper";
  * divergence (the paper has no rule): stop with EDIVERGED when r_k is not
    finite or the unnormalised equilibrium norm sqrt(sum |T_check q^b|^2) has
    grown past DIVERGENCE_FACTOR times its value at k = 0 (r_k itself can
    stay bounded in a diverging iteration, since the mean stress that
    normalises it grows with the iterate);
  * DGO: polarisation form eps^(k+1) = Ebar + F^{c+}[Gamma^c F^{c-}((C - C_H) eps^(k))],
    stopped on |eps^(k+1) - eps^(k)| / (sqrt(N) |Ebar|_F).

Fields are stored per voxel as full 3x3 matrices, shape (n3, n2, n1, 3, 3);
the public results use Voigt tensor components, shape (6, n3, n2, n1).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import fdd, fourier
from .green import from_voigt, green_update, sym_outer, to_voigt

OK, ENOTCONV, EDIVERGED = 0, 1, 2
DIVERGENCE_FACTOR = 1e6


@dataclass
class Result:
    eps: np.ndarray            # (6, n3, n2, n1) Voigt tensor components
    sig: np.ndarray            # (6, n3, n2, n1)
    sig_mean: np.ndarray       # (6,)
    iters: int
    residual: float
    status: int
    history: list = field(default_factory=list)


def hooke(lam, mu, eps):
    """Isotropic Hooke law of Sec. 5.1: T = lambda tr(E) I + mu (E + E^T)."""
    tr = np.trace(eps, axis1=-2, axis2=-1)
    return lam[..., None, None] * tr[..., None, None] * np.eye(3) + mu[..., None, None] * (
        eps + np.swapaxes(eps, -1, -2))


def frob(A):
    """Frobenius norm over the last two (3x3) axes and everything before them."""
    return float(np.sqrt(np.sum(np.abs(A) ** 2)))


def _transform(T, forward, disc):
    """Transform a (n3, n2, n1, 3, 3) symmetric field through its 6 Voigt components."""
    v = np.moveaxis(to_voigt(T), -1, 0)
    if disc == "TD":
        out = fourier.td_forward(v) if forward else fourier.td_inverse(v)
    elif disc == "PCD":
        out = fourier.pcd_forward(v) if forward else fourier.pcd_inverse(v)
    else:
        raise ValueError(disc)
    return from_voigt(np.moveaxis(out, 0, -1))


def equilibrium_norm(That, qb):
    """sqrt(sum |T_check q^b|^2): the unnormalised equilibrium norm."""
    div = np.einsum("...ij,...j->...i", That, qb)
    return float(np.sqrt(np.sum(np.abs(div) ** 2)))


def equilibrium_residual(That, qb, num=None):
    """sqrt(sum |T_check q^b|^2) / |T_check(0)|_F (the reading above)."""
    if num is None:
        num = equilibrium_norm(That, qb)
    den = frob(That[0, 0, 0])
    if num == 0.0:
        return 0.0
    return float(num / den) if den > 0 else float("inf")


def _ebar_matrix(Ebar):
    return from_voigt(np.asarray(Ebar, dtype=np.float64))


def _voigt_field(A):
    return np.ascontiguousarray(np.moveaxis(to_voigt(A), -1, 0))


def eigenstrain_field(eigenstrain, shape):
    """(n3, n2, n1, 3, 3) eigenstrain E_* from Voigt tensor components of shape
    (6, n3, n2, n1), or None for none."""
    if eigenstrain is None:
        return None
    e = np.asarray(eigenstrain, dtype=np.float64)
    if e.shape != (6,) + tuple(shape):
        raise ValueError("eigenstrain must have shape (6, n3, n2, n1)")
    return from_voigt(np.moveaxis(e, 0, -1))


def eigenstress(lam, mu, Es):
    """C E_*: the stress the eigenstrain removes, T = C [E - E_*] (Sec. 7)."""
    return hooke(lam, mu, Es)


def eigen_norm(Eb, Es):
    """Scale of the loading for the DGO stopping test: |Ebar|_F, or the RMS of
    |E_*|_F over the voxels when Ebar = 0 (reading: the paper normalises by
    Ebar, which a pure eigenstrain loading does not have)."""
    nE = frob(Eb)
    if nE == 0.0 and Es is not None:
        nE = frob(Es) / np.sqrt(Es.shape[0] * Es.shape[1] * Es.shape[2])
    return nE


def solve_gfp(lam, mu, Ebar, lam0, mu0, scheme="AFB", tol=1e-8, maxit=1000,
              disc="TD", h=(1.0, 1.0, 1.0), stop="equilibrium", callback=None, eigenstrain=None):
    """TD / PCD GFP+FDD fixed point (Sec. 5.2 / Sec. 5.4), displacement based.

    lam, mu: (n3, n2, n1) moduli sampled at the nodes (TD) or cell centres (PCD);
    Ebar: macroscopic strain, Voigt tensor components; lam0, mu0: C_H;
    scheme: a key of fdd.SCHEMES.  Steps per iteration, in the paper's order:
        E~ = F^+ sym(u_check (x) q^a);  T = T^(0) + C E~;  T_check = F^- T;
        Delta u = G(q^a, q^b) T_check q^b;  u_check += Delta u.
    eigenstrain: optional E_* (6, n3, n2, n1), Voigt tensor components; the
    constitutive law becomes T = C [E - E_*], i.e. T^(0) = C [Ebar - E_*]
    (Sec. 7).  The returned eps is the total strain E.
    """
    n3, n2, n1 = lam.shape
    qa, qb = fdd.scheme_pair(scheme, (n1, n2, n3), h)
    singular = fdd.singular_mask(qa, qb)
    Eb = _ebar_matrix(Ebar)
    Es = eigenstrain_field(eigenstrain, lam.shape)
    T0 = hooke(lam, mu, np.broadcast_to(Eb, (n3, n2, n1, 3, 3)))
    if Es is not None:
        T0 = T0 - eigenstress(lam, mu, Es)
    u = np.zeros((n3, n2, n1, 3), dtype=np.complex128)
    du_prev = np.zeros_like(u)
    paper_done = False
    history = []
    k = 0
    while True:
        Et = _transform(sym_outer(u, qa), forward=False, disc=disc).real
        T = T0 + hooke(lam, mu, Et)
        That = _transform(T, forward=True, disc=disc)
        num = equilibrium_norm(That, qb)
        r = equilibrium_residual(That, qb, num)
        history.append(r)
        if k == 0:
            num0 = num
        if callback is not None:
            callback(k, Eb + Et, T, r)
        if paper_done or (stop == "equilibrium" and r <= tol):
            status = OK
            break
        if k == maxit:
            status = ENOTCONV
            break
        if not np.isfinite(r) or num > DIVERGENCE_FACTOR * max(num0, 1e-300):
            status = EDIVERGED
            break
        du = green_update(That, qa, qb, lam0, mu0, singular)
        u += du
        k += 1
        if stop == "paper":
            # the paper's test: L1 norm over frequencies of |Delta u^(k) - Delta u^(k-1)|
            d = float(np.sum(np.sqrt(np.sum(np.abs(du - du_prev) ** 2, axis=-1))))
            paper_done = d < tol
            du_prev = du
    eps = Eb + Et
    sig_mean = to_voigt(T.mean(axis=(0, 1, 2)))
    return Result(_voigt_field(eps), _voigt_field(T), sig_mean, k, history[-1], status, history)


def solve_dgo(lam, mu, Ebar, lam0, mu0, Gc, tol=1e-8, maxit=1000, disc="PCD", eigenstrain=None):
    """DGO fixed point of Sec. 5.4 in polarisation form.

    Gc: (n3, n2, n1, 6, 6) discrete Green operator (green.dgo_voigt), with the
    paper's sign (Gamma_H = -sym[G A k (x) k]).  Per iteration:
        tau = (C - C_H) eps;  eps_new = Ebar + F^{c+}[ Gc F^{c-} tau ].
    eigenstrain: optional E_*; the polarisation becomes
        tau = T - C_H eps = (C - C_H) eps - C E_*   (T = C [E - E_*], Sec. 7).
    """
    n3, n2, n1 = lam.shape
    N = n1 * n2 * n3
    Eb = _ebar_matrix(Ebar)
    Es = eigenstrain_field(eigenstrain, lam.shape)
    eps = np.broadcast_to(Eb, (n3, n2, n1, 3, 3)).copy()
    dlam, dmu = lam - lam0, mu - mu0
    tau_star = eigenstress(lam, mu, Es) if Es is not None else 0.0
    nE = eigen_norm(Eb, Es)
    history = []
    r = float("inf")
    k = 0
    status = ENOTCONV
    while k < maxit:
        tau = hooke(dlam, dmu, eps) - tau_star
        tv = np.moveaxis(to_voigt(tau), -1, 0)
        th = fourier.pcd_forward(tv) if disc == "PCD" else fourier.td_forward(tv)
        eh = np.einsum("...IJ,J...->I...", Gc, th)
        ev = (fourier.pcd_inverse(eh) if disc == "PCD" else fourier.td_inverse(eh)).real
        eps_new = Eb + from_voigt(np.moveaxis(ev, 0, -1))
        r = frob(eps_new - eps) / (np.sqrt(N) * nE) if nE > 0 else 0.0
        history.append(r)
        eps = eps_new
        k += 1
        if r <= tol:
            status = OK
            break
        if not np.isfinite(r) or r > DIVERGENCE_FACTOR * max(history[0], 1e-300):
            status = EDIVERGED
            break
    T = hooke(lam, mu, eps) - tau_star
    sig_mean = to_voigt(T.mean(axis=(0, 1, 2)))
    return Result(_voigt_field(eps), _voigt_field(T), sig_mean, k, r, status, history)


def mandel(v):
    """Voigt tensor components -> Mandel vector (shear scaled by sqrt 2)."""
    v = np.asarray(v, dtype=np.float64).copy()
    v[3:] *= np.sqrt(2.0)
    return v


def effective_stiffness(solve, unit_strains):
    """6x6 Mandel effective stiffness from six solves.

    solve(Ebar) -> Result; unit_strains: (6, 6) rows are Voigt tensor strains
    with unit Mandel norm.  Column J is the Mandel vector of <sigma> under
    unit strain J.
    """
    M = np.zeros((6, 6))
    for J in range(6):
        res = solve(unit_strains[J])
        M[:, J] = mandel(res.sig_mean)
    return M
