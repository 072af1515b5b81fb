"""Closed forms and bounds used to pin the oracle.  TEST INFRASTRUCTURE ONLY.

* `laminate_strain`: exact equilibrium of a material that varies along x1
  only.  Equilibrium forces T e1 to be uniform and compatibility lets only
  E11, E12, E13 fluctuate, so with layer moduli lambda(x1), mu(x1):
      E22, E33, E23 = Ebar's;  E12 = Ebar12 / (mu <1/mu>)  (likewise E13);
      E11 = (S - lambda (Ebar22 + Ebar33)) / (lambda + 2 mu),
      S = (Ebar11 + <lambda/(lambda+2mu)> (Ebar22 + Ebar33)) / <1/(lambda+2mu)>.
  Every scheme's wavevector is parallel to e1 at the frequencies such a field
  excites, so this is also the exact discrete solution of each scheme.
* `laminate_strain_eig`: the same with a layer eigenstrain E_*(x1) and the
  law T = C [E - E_*] (Sec. 7): T e1 uniform, E22, E33, E23 = Ebar's;
      E1j = E_*1j + S1j / (2 mu),  S1j = (Ebar1j - <E_*1j>) / <1/(2 mu)>  (j = 2, 3);
      E11 = (S - lambda (Ebar22 + Ebar33) + lambda tr E_* + 2 mu E_*11) / (lambda + 2 mu),
      S = (Ebar11 + <(lambda (Ebar22 + Ebar33) - lambda tr E_* - 2 mu E_*11) / (lambda + 2 mu)>)
          / <1/(lambda + 2 mu)>.
  The forcing excites the same frequencies, so it is again the exact discrete
  solution of each scheme.
* `voigt_mandel`, `reuss_mandel`: <C> and <C^{-1}>^{-1} in Mandel form.
* `hs_lower_bulk`: Hashin-Shtrikman lower bound on the bulk modulus of a
  two-phase isotropic mixture.
* `iso_mandel`: Mandel 6x6 matrix of lambda I(x)I + 2 mu I^sym.
"""
from __future__ import annotations

import numpy as np


def laminate_strain(lam1, mu1, Ebar):
    """Exact strain (6, n1) of a laminate with layer moduli lam1(x1), mu1(x1)."""
    E = np.asarray(Ebar, dtype=np.float64)
    M = lam1 + 2.0 * mu1
    S = (E[0] + np.mean(lam1 / M) * (E[1] + E[2])) / np.mean(1.0 / M)
    out = np.zeros((6,) + lam1.shape)
    out[0] = (S - lam1 * (E[1] + E[2])) / M
    out[1] = E[1]
    out[2] = E[2]
    out[3] = E[3]
    out[4] = E[4] / (mu1 * np.mean(1.0 / mu1))
    out[5] = E[5] / (mu1 * np.mean(1.0 / mu1))
    return out


def laminate_strain_eig(lam1, mu1, Ebar, estar1):
    """Exact strain (6, n1) of a laminate with layer moduli lam1(x1), mu1(x1)
    and layer eigenstrain estar1 (6, n1), Voigt tensor components."""
    E = np.asarray(Ebar, dtype=np.float64)
    es = np.asarray(estar1, dtype=np.float64)
    M = lam1 + 2.0 * mu1
    tr = es[0] + es[1] + es[2]
    g = lam1 * (E[1] + E[2]) - lam1 * tr - 2.0 * mu1 * es[0]
    S = (E[0] + np.mean(g / M)) / np.mean(1.0 / M)
    out = np.zeros((6,) + lam1.shape)
    out[0] = (S - g) / M
    out[1] = E[1]
    out[2] = E[2]
    out[3] = E[3]
    for j in (4, 5):  # E13, E12: shear stress S1j = 2 mu (E1j - E_*1j) uniform
        s1j = (E[j] - np.mean(es[j])) / np.mean(1.0 / (2.0 * mu1))
        out[j] = es[j] + s1j / (2.0 * mu1)
    return out


def iso_mandel(lam, mu):
    """Mandel 6x6 of an isotropic stiffness."""
    m = np.zeros((6, 6))
    m[:3, :3] = lam
    m += 2.0 * mu * np.eye(6)
    return m


def voigt_mandel(lam, mu):
    """Voigt bound <C> (uniform strain) in Mandel form."""
    return iso_mandel(float(np.mean(lam)), float(np.mean(mu)))


def reuss_mandel(lam, mu):
    """Reuss bound <C^{-1}>^{-1} (uniform stress) in Mandel form."""
    lam = np.ravel(lam)
    mu = np.ravel(mu)
    # isotropic compliance: S = 1/(2mu) I - lam/(2mu(3lam+2mu)) I(x)I
    a = np.mean(1.0 / (2.0 * mu))
    b = np.mean(lam / (2.0 * mu * (3.0 * lam + 2.0 * mu)))
    S = a * np.eye(6)
    S[:3, :3] -= b
    return np.linalg.inv(S)


def bulk_shear(lam, mu):
    return lam + 2.0 * mu / 3.0, mu


def hs_lower_bulk(k1, mu1, k2, f2):
    """HS lower bound on kappa for phase 1 the softer one (k1 <= k2, mu1 <= mu2)."""
    f1 = 1.0 - f2
    return k1 + f2 / (1.0 / (k2 - k1) + 3.0 * f1 / (3.0 * k1 + 4.0 * mu1))


def hs_upper_bulk(k2, mu2, k1, f1):
    """HS upper bound (phase 2 the stiffer one)."""
    f2 = 1.0 - f1
    return k2 + f1 / (1.0 / (k1 - k2) + 3.0 * f2 / (3.0 * k2 + 4.0 * mu2))


def bulk_from_mandel(M):
    """kappa_eff = (1/9) I : C_eff : I."""
    return float(np.sum(M[:3, :3]) / 9.0)
