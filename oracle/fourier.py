"""Discrete Fourier transforms of the trapezoidal (TD) and piecewise-constant
(PCD) discretisations.  TEST INFRASTRUCTURE ONLY (see the package docstring).

Conventions (all fields have their three spatial axes LAST, ordered
(x3, x2, x1), so x1 is the fastest axis):

* TD, Sec. 3.1 eqs. (9)-(10) and its tensor product Sec. 5.2 eq. (31): nodes
  x_i = (i - 1) h (0-based: i h), unitary transform
  f_check = n^{-1/2} sum_i exp(-i k x_i) f_i, inverse with exp(+i k x_i).
* PCD, Sec. 3.2 eqs. (20)-(21) and Sec. 5.4 eq. (47): samples at the cell
  centres x^c_i = (i - 1/2) h (0-based: (i + 1/2) h), same unitary kernel.
* Spectrum indexing: numpy FFT order.  Index j on an axis of length n is the
  centred wavenumber index kappa = j for j < n/2 and kappa = j - n otherwise,
  i.e. the paper's set kappa = mu - 1 - m, mu = 1..n, m = n/2, which for even
  n is [-n/2, n/2 - 1] (Sec. 3.1, after eq. (10); Appendix A).  The Nyquist
  index is therefore kappa = -n/2.

numpy.fft with norm="ortho" is exactly the unitary TD transform; it is pinned
against the brute-force triple sum `dft_bruteforce` in the tests.
"""
from __future__ import annotations

import numpy as np

AXES = (-3, -2, -1)


def centred_index(n):
    """kappa for each numpy-order spectrum index j of an axis of length n."""
    j = np.arange(n)
    return np.where(j < (n + 1) // 2, j, j - n) if n % 2 else np.where(j < n // 2, j, j - n)


def grid_shape(field):
    """(n1, n2, n3) of a field whose spatial axes are last."""
    n3, n2, n1 = field.shape[-3:]
    return n1, n2, n3


def td_forward(f):
    """TD transform F^- (unitary) over the last three axes."""
    return np.fft.fftn(f, axes=AXES, norm="ortho")


def td_inverse(fc):
    """TD inverse F^+ (unitary) over the last three axes."""
    return np.fft.ifftn(fc, axes=AXES, norm="ortho")


def _centre_phase(n1, n2, n3, h=(1.0, 1.0, 1.0)):
    """exp(-i k . h/2): the factor that moves TD nodes to PCD cell centres.

    For wavenumber index kappa on an axis, k h / 2 = pi kappa / n.
    """
    ph = []
    for n in (n1, n2, n3):
        ph.append(np.exp(-1j * np.pi * centred_index(n) / n))
    p1, p2, p3 = ph
    return p3[:, None, None] * p2[None, :, None] * p1[None, None, :]


def pcd_forward(f):
    """PCD transform F^{c-}: unitary kernel evaluated at the cell centres."""
    n1, n2, n3 = grid_shape(f)
    return td_forward(f) * _centre_phase(n1, n2, n3)


def pcd_inverse(fc):
    """PCD inverse F^{c+}."""
    n1, n2, n3 = grid_shape(fc)
    return td_inverse(fc * np.conj(_centre_phase(n1, n2, n3)))


def dft_bruteforce(f, centre=False):
    """Unitary 3D DFT by the defining triple sum, O(N^2): for tiny grids only.

    Evaluates f_check(kappa) = N^{-1/2} sum_x exp(-i k . x) f(x) with
    k_r = 2 pi kappa_r / n_r (h = 1), x_r = i_r (TD) or i_r + 1/2 (PCD,
    centre=True), written out with no FFT and no separability.
    """
    n1, n2, n3 = grid_shape(f)
    N = n1 * n2 * n3
    off = 0.5 if centre else 0.0
    xs = [(np.arange(n) + off) for n in (n1, n2, n3)]
    ks = [2.0 * np.pi * centred_index(n) / n for n in (n1, n2, n3)]
    X3, X2, X1 = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    K3, K2, K1 = np.meshgrid(ks[2], ks[1], ks[0], indexing="ij")
    x = np.stack([X1.ravel(), X2.ravel(), X3.ravel()], axis=1)      # (N, 3)
    k = np.stack([K1.ravel(), K2.ravel(), K3.ravel()], axis=1)      # (N, 3)
    kernel = np.exp(-1j * (k @ x.T)) / np.sqrt(N)                  # (Nk, Nx)
    lead = f.shape[:-3]
    flat = f.reshape(lead + (N,))
    out = flat @ kernel.T
    return out.reshape(lead + (n3, n2, n1))


def dft_matrix(n, centre=False):
    """Unitary 1D DFT matrix F^-_{kappa i} (rows: numpy-order kappa)."""
    off = 0.5 if centre else 0.0
    k = 2.0 * np.pi * centred_index(n) / n
    x = np.arange(n) + off
    return np.exp(-1j * np.outer(k, x)) / np.sqrt(n)
