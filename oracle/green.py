"""Green-function preconditioners.  TEST INFRASTRUCTURE ONLY.

* `green_inverse`: the 3x3 symbol of -div^b C_H grad^a, Sec. 5.2 eq. (34):
      G^{-1}(q^a, q^b) = -mu_H (q^a . q^b) I - mu_H q^a (x) q^b - lambda_H q^b (x) q^a
  (the 1D analogue is eq. (17)).  The oracle inverts it numerically, per
  frequency, with a general complex solve: no closed form is assumed.
* `green_update`: Delta u = G(q^a, q^b) T_check q^b, the Green step of the TD
  and PCD algorithms (Sec. 5.2 and Sec. 5.4), with G := 0 at the singular
  frequencies (q^a . q^b == 0), as Sec. 3.1 prescribes after Algorithm 1.
* `green_tensor_iso`, `gamma_iso`: the isotropic Green tensor of Sec. 5.4
  eq. (48) and the Lippmann-Schwinger operator defined right after it,
      Gamma_H(k) A = -sym[ G_H(k) A (k (x) k) ].
* `dgo_voigt`: the discrete Green operator of the Sec. 5.4 DGO algorithm
  (and of Sec. 3.3 in 1D): Gamma^c_omega = sum over periodic images of the
  sinc weight times Gamma_H at the image wavevector, Gamma^c_0 = 0.
"""
from __future__ import annotations

import itertools

import numpy as np

from .fourier import centred_index

VOIGT = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))


def green_inverse(qa, qb, lam0, mu0):
    """G^{-1}(q^a, q^b) of eq. (34); qa, qb: (..., 3) -> (..., 3, 3)."""
    dot = np.einsum("...r,...r->...", qa, qb)
    eye = np.eye(3)
    return (-mu0 * dot[..., None, None] * eye
            - mu0 * qa[..., :, None] * qb[..., None, :]
            - lam0 * qb[..., :, None] * qa[..., None, :])


def green_update(that, qa, qb, lam0, mu0, singular):
    """Delta u = G T_check q^b per frequency; zero where `singular` is True.

    that: (..., 3, 3) stress spectrum (full symmetric matrices),
    qa, qb: (..., 3); singular: boolean (...).
    """
    rhs = np.einsum("...ij,...j->...i", that, qb)
    du = np.zeros(rhs.shape, dtype=np.complex128)
    ok = ~singular
    if np.any(ok):
        ginv = green_inverse(qa[ok], qb[ok], lam0, mu0)
        du[ok] = np.linalg.solve(ginv, rhs[ok][..., None])[..., 0]
    return du


def sym_outer(u, q):
    """sym(u (x) q) per frequency: (..., 3), (..., 3) -> (..., 3, 3)."""
    m = u[..., :, None] * q[..., None, :]
    return 0.5 * (m + np.swapaxes(m, -1, -2))


def green_tensor_iso(k, lam0, mu0):
    """Isotropic Green tensor of eq. (48) for real k != 0: (..., 3) -> (..., 3, 3).

    G_H(k) = (mu |k|^2)^{-1} [ I - (1 + lambda/mu)/(1 + (1 + lambda/mu)) khat (x) khat ].
    """
    k2 = np.einsum("...r,...r->...", k, k)
    khat = k / np.sqrt(k2)[..., None]
    r = lam0 / mu0
    c = (1.0 + r) / (1.0 + (1.0 + r))
    return (np.eye(3) - c * khat[..., :, None] * khat[..., None, :]) / (mu0 * k2)[..., None, None]


def gamma_iso(k, lam0, mu0, A):
    """Gamma_H(k) A = -sym[G_H(k) A (k (x) k)], k real (..., 3), A (..., 3, 3)."""
    G = green_tensor_iso(k, lam0, mu0)
    Ak = np.einsum("...ij,...j->...i", A, k)
    v = np.einsum("...ij,...j->...i", G, Ak)
    return -sym_outer(v, k)


def _unit_sym(J):
    """Symmetric unit tensor of Voigt slot J (both off-diagonal entries = 1)."""
    E = np.zeros((3, 3))
    i, j = VOIGT[J]
    E[i, j] = 1.0
    E[j, i] = 1.0
    return E


def to_voigt(A):
    """(..., 3, 3) -> (..., 6) tensor components in Voigt order."""
    return np.stack([A[..., i, j] for (i, j) in VOIGT], axis=-1)


def from_voigt(v):
    """(..., 6) tensor components -> (..., 3, 3) symmetric."""
    A = np.zeros(v.shape[:-1] + (3, 3), dtype=v.dtype)
    for J, (i, j) in enumerate(VOIGT):
        A[..., i, j] = v[..., J]
        A[..., j, i] = v[..., J]
    return A


def gamma_iso_voigt(k, lam0, mu0):
    """6x6 matrix M(k) with Voigt(Gamma_H(k) A) = M(k) Voigt(A); k: (..., 3)."""
    cols = []
    for J in range(6):
        E = np.broadcast_to(_unit_sym(J), k.shape[:-1] + (3, 3))
        cols.append(to_voigt(gamma_iso(k, lam0, mu0, E)))
    return np.stack(cols, axis=-1)


def sinc_weight(kappa, nu, n):
    """sinc(pi (kappa + nu n)/n) with exact zeros at nonzero integer arguments."""
    x = kappa / n + nu
    num = kappa + nu * n
    with np.errstate(divide="ignore", invalid="ignore"):
        w = np.sin(np.pi * x) / (np.pi * x)
    w = np.where(num == 0, 1.0, w)
    w = np.where((num != 0) & (kappa % n == 0), 0.0, w)
    return w


def image_range(kappa, n, M):
    """Periodic image shifts nu for index kappa: [-M, M], or [-M, M+1] at the
    Nyquist index kappa = -n/2 so that the image set stays symmetric about 0
    (a reading: the paper's printed window [-m, m-1] is not symmetric)."""
    hi = M + 1 if (n % 2 == 0 and kappa == -n // 2) else M
    return range(-M, hi + 1)


def dgo_voigt(n, lam0, mu0, M, p=1, h=(1.0, 1.0, 1.0)):
    """DGO Gamma^c per frequency as (n3, n2, n1, 6, 6), with Gamma^c_0 = 0.

    Gamma^c_omega = sum_nu prod_r s^p(kappa_r + nu_r n_r) Gamma_H(k_nu),
    k_nu,r = 2 pi (kappa_r + nu_r n_r) / (n_r h_r), s(m) = sinc(pi m / n_r);
    p = 1 is the single sinc printed in the paper, p = 2 the squared weight of
    the consistent operator the paper cites.  The sum runs image by image,
    each image evaluated at every frequency at once (small grids only).
    """
    n1, n2, n3 = (n,) * 3 if np.isscalar(n) else n
    ns = (n1, n2, n3)
    kap = [centred_index(v) for v in ns]
    out = np.zeros((n3, n2, n1, 6, 6))
    shape = (n3, n2, n1)
    for v in itertools.product(range(-M, M + 2), repeat=3):
        w = np.ones(shape)
        k = np.zeros(shape + (3,))
        for r in range(3):
            a = kap[r]
            allowed = np.array([v[r] in image_range(int(x), ns[r], M) for x in a])
            wr = np.where(allowed, sinc_weight(a, v[r], ns[r]), 0.0) ** p
            kr = 2 * np.pi * (a + v[r] * ns[r]) / (ns[r] * h[r])
            sl = [None, None, None]
            sl[2 - r] = slice(None)
            w = w * wr[tuple(sl)]
            k[..., r] = np.broadcast_to(kr[tuple(sl)], shape)
        live = w != 0.0
        live &= np.einsum("...r,...r->...", k, k) != 0.0   # the k = 0 point (omega = 0)
        if not np.any(live):
            continue
        out[live] += w[live][:, None, None] * gamma_iso_voigt(k[live], lam0, mu0)
    out[0, 0, 0] = 0.0
    return out


def dgo_voigt_at(freq, n, lam0, mu0, M, p=1, h=(1.0, 1.0, 1.0)):
    """DGO 6x6 matrix at one frequency index triple (j1, j2, j3) (numpy order)."""
    n1, n2, n3 = n
    a = [int(centred_index(nr)[j]) for nr, j in zip((n1, n2, n3), freq)]
    if a == [0, 0, 0]:
        return np.zeros((6, 6))
    acc = np.zeros((6, 6))
    for v in itertools.product(*(image_range(a[r], (n1, n2, n3)[r], M) for r in range(3))):
        w = 1.0
        for r in range(3):
            w *= sinc_weight(a[r], v[r], (n1, n2, n3)[r])
        w = w ** p
        if w == 0.0:
            continue
        k = np.array([2 * np.pi * (a[r] + v[r] * (n1, n2, n3)[r]) / ((n1, n2, n3)[r] * h[r])
                      for r in range(3)])
        acc += w * gamma_iso_voigt(k, lam0, mu0)
    return acc
