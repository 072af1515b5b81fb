"""Test-side glue: oracle quantities in the GPU library's layouts.

Everything here calls only the CPU oracle (oracle/) and numpy; nothing
comes from the GPU path.  Half spectra follow include/lsfft.h: unnormalised
forward DFT, shape (6, n3, n2, n1/2 + 1), Voigt tensor components.
"""
import numpy as np

from oracle import fdd, fourier, green, solve3d

SCHEME_NAMES = {"basic": "basic", "fb": "FB", "afb": "AFB", "cd": "CD", "acd": "ACD"}


def hooke_voigt(lam, mu, eps):
    """(6, n3, n2, n1) strain -> stress via the oracle's Hooke law."""
    E = green.from_voigt(np.moveaxis(eps, 0, -1))
    return np.moveaxis(green.to_voigt(solve3d.hooke(lam, mu, E)), -1, 0)


def half_spectrum(field):
    """Unnormalised forward transform (oracle TD transform x sqrt(N)), kx in [0, n1/2]."""
    n3, n2, n1 = field.shape[-3:]
    full = fourier.td_forward(field) * np.sqrt(n1 * n2 * n3)
    return np.ascontiguousarray(full[..., : n1 // 2 + 1])


def full_from_half(half, n1):
    """Hermitian completion of a half spectrum along the last axis."""
    n3, n2 = half.shape[-3:-1]
    full = np.zeros(half.shape[:-1] + (n1,), dtype=np.complex128)
    full[..., : n1 // 2 + 1] = half
    for j in range(n1 // 2 + 1, n1):
        src = half[..., n1 - j]
        # X(k3, k2, -j) = conj X(-k3, -k2, j)
        src = np.conj(src[..., (-np.arange(n3)) % n3, :][..., :, (-np.arange(n2)) % n2])
        full[..., j] = src
    return full


def green_increment_half(half, scheme, lam0, mu0):
    """Strain increment -Gamma_0 sigma_hat by the oracle's general complex path
    (Sec. 5.2 eq. (34)), on a half spectrum; also sum |sigma_hat q^b|^2 over the
    full spectrum."""
    n3, n2, L1 = half.shape[-3:]
    n1 = 2 * (L1 - 1)
    full = full_from_half(half, n1)
    qa, qb = fdd.scheme_pair(SCHEME_NAMES[scheme], (n1, n2, n3))
    sing = fdd.singular_mask(qa, qb)
    T = green.from_voigt(np.moveaxis(full, 0, -1))
    du = green.green_update(T, qa, qb, lam0, mu0, sing)
    de = green.sym_outer(du, qa)
    out = np.moveaxis(green.to_voigt(de), -1, 0)[..., :L1]
    div = np.einsum("...ij,...j->...i", T, qb)
    return np.ascontiguousarray(out), float(np.sum(np.abs(div) ** 2))


def dgo_apply_half(half, Gc):
    """Gamma^c (Voigt 6x6 per frequency, paper's sign) applied to a half spectrum."""
    L1 = half.shape[-1]
    G = Gc[:, :, :L1]
    return np.einsum("...IJ,J...->I...", G, half)


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0))


def plane_errors(a, b):
    """Relative L2 errors of the strain spectrum of `a` against that of `b`
    ((..., n3, n2, n1) fields) on the planes and lines a global norm could
    hide: the Nyquist plane of each even axis and the three zero-frequency
    axis lines (the mean, index (0, 0, 0), excluded).  A plane whose
    reference content is below 1e-12 of the whole fluctuation spectrum is
    compared against that instead."""
    A = np.fft.fftn(np.asarray(a, dtype=np.float64), axes=(-3, -2, -1))
    Bf = np.fft.fftn(np.asarray(b, dtype=np.float64), axes=(-3, -2, -1))
    n3, n2, n1 = Bf.shape[-3:]
    fluct = Bf.copy()
    fluct[..., 0, 0, 0] = 0.0
    scale = np.linalg.norm(fluct.ravel())
    sel = {}
    if n1 % 2 == 0:
        sel["x_nyquist"] = (Ellipsis, slice(None), slice(None), n1 // 2)
    if n2 % 2 == 0:
        sel["y_nyquist"] = (Ellipsis, slice(None), n2 // 2, slice(None))
    if n3 % 2 == 0:
        sel["z_nyquist"] = (Ellipsis, n3 // 2, slice(None), slice(None))
    sel["x_line"] = (Ellipsis, 0, 0, slice(1, None))
    sel["y_line"] = (Ellipsis, 0, slice(1, None), 0)
    sel["z_line"] = (Ellipsis, slice(1, None), 0, 0)
    out = {}
    for name, ix in sel.items():
        d = np.linalg.norm((A[ix] - Bf[ix]).ravel())
        r = np.linalg.norm(Bf[ix].ravel())
        out[name] = float(d / max(r, 1e-12 * scale, 1e-300))
    return out
