"""The 1D algorithms of Sec. 3 and the analytic solution of Sec. 2.1, FP64.
TEST INFRASTRUCTURE ONLY (see the package docstring).

* `solve_gfp_1d`: the TD GFP+FDD algorithm of Sec. 3.1 (Algorithm 1 of the
  trapezoidal series) and, with disc="PCD", the cell-centred algorithm of
  Sec. 3.2 (Algorithm 1 of the PCD series).  Green function of eq. (17):
  G = -1 / (C_H q^a q^b), set to 0 where q^a q^b == 0.
* `solve_dgo_1d`: the DGO algorithm of Sec. 3.3 (Algorithm 1 of the DGO
  series).  form="polarisation" (default, the footnote of Sec. 3.3) or
  form="stress" (the algorithm exactly as printed, iterating on T).
* `analytic_strain`: eq. (3): E~(x)/Ebar = S~(x)/Sbar, i.e. nodal strain
  E_i = S_i Tbar with Tbar = Ebar / <S>, the exact discrete equilibrium.

Fields are 1D arrays of length n; the same iteration-index and stopping
readings as the 3D module apply.
"""
from __future__ import annotations

import numpy as np

from . import fdd
from .fourier import centred_index
from .green import sinc_weight, image_range

PAIRS_1D = {"F": ("F", "conj"), "CD": ("CD", "conj"), "FD": ("FD", "conj"),
            "FD_hC": ("FD", "hC")}


def _fwd(f, disc):
    n = f.shape[-1]
    out = np.fft.fft(f, norm="ortho")
    if disc == "PCD":
        out = out * np.exp(-1j * np.pi * centred_index(n) / n)
    return out


def _inv(fc, disc):
    n = fc.shape[-1]
    if disc == "PCD":
        fc = fc * np.exp(1j * np.pi * centred_index(n) / n)
    return np.fft.ifft(fc, norm="ortho")


def pair_1d(scheme, n, h=1.0):
    s = fdd.symbols_1d(n, h)
    a, b = PAIRS_1D[scheme]
    qa = s[a]
    qb = np.conj(qa) if b == "conj" else s[b]
    return qa, qb


def solve_gfp_1d(C, Ebar, CH, scheme="F", tol=1e-13, maxit=10000, disc="TD", h=1.0):
    """1D GFP+FDD fixed point; returns (E, T, iters, residual)."""
    n = C.shape[0]
    qa, qb = pair_1d(scheme, n, h)
    prod = qa * qb
    G = np.zeros(n, dtype=np.complex128)
    ok = prod != 0
    G[ok] = -1.0 / (CH * prod[ok])
    T0 = C * Ebar
    u = np.zeros(n, dtype=np.complex128)
    k = 0
    while True:
        Et = _inv(u * qa, disc).real
        T = T0 + C * Et
        Tc = _fwd(T, disc)
        num = np.sqrt(np.sum(np.abs(Tc * qb) ** 2))
        r = 0.0 if num == 0 else float(num / abs(Tc[0]))
        if r <= tol or k == maxit:
            break
        u += G * Tc * qb
        k += 1
    return Ebar + Et, T, k, r


def dgo_factor_1d(n, M, p=1):
    """c_p(omega) = sum over images of sinc^p(pi (kappa + nu n)/n); 0 at omega = 0."""
    kap = centred_index(n)
    c = np.zeros(n)
    for j, a in enumerate(kap):
        if a == 0:
            continue
        c[j] = sum(sinc_weight(a, v, n) ** p for v in image_range(int(a), n, M))
    return c


def solve_dgo_1d(C, Ebar, CH, M, p=1, tol=1e-13, maxit=10000, form="polarisation"):
    """1D DGO fixed point.  Gamma_H(k) A = -A / C_H in 1D, so Gamma^c = -c_p / C_H."""
    n = C.shape[0]
    Gc = -dgo_factor_1d(n, M, p) / CH
    E = np.full(n, float(Ebar))
    k = 0
    r = float("inf")
    if form == "stress":
        # exactly as printed: E_check += Gamma^c T_check, T = C E
        Ec = np.zeros(n, dtype=np.complex128)
        while k < maxit:
            T = C * E
            Tc = _fwd(T, "PCD")
            dE = Gc * Tc
            Ec += dE
            E_new = Ebar + _inv(Ec, "PCD").real
            r = float(np.linalg.norm(E_new - E) / (np.sqrt(n) * abs(Ebar)))
            E = E_new
            k += 1
            if r <= tol:
                break
        return E, C * E, k, r
    while k < maxit:
        tau = (C - CH) * E
        E_new = Ebar + _inv(Gc * _fwd(tau, "PCD"), "PCD").real
        r = float(np.linalg.norm(E_new - E) / (np.sqrt(n) * abs(Ebar)))
        E = E_new
        k += 1
        if r <= tol:
            break
    return E, C * E, k, r


def analytic_strain(C, Ebar):
    """Exact 1D equilibrium at the samples: E_i = S_i Tbar, Tbar = Ebar / <S>."""
    S = 1.0 / C
    Tbar = Ebar / S.mean()
    return S * Tbar, Tbar
