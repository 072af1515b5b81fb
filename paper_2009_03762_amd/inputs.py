"""Seeded synthetic inputs for the periodic matrix-inclusion unit cell.

These generators produce per-voxel isotropic Lame moduli (lambda, mu) and
macroscopic strains.  They hold none of the solver's arithmetic: both the GPU
library and the CPU oracle consume the arrays they return, unchanged.

Array convention: every field has shape (n3, n2, n1) in C order, so the x
index i1 is the fastest-varying one; voxel (i1, i2, i3) is sampled at its
centre ((i1 + 1/2) h1, (i2 + 1/2) h2, (i3 + 1/2) h3).

Geometry follows the cubic-inclusion benchmark of Section 5 (Computational
comparisons in 3D): a centred cube, either with a sharp interface (the
interface lies between voxel centres) or a smooth tanh interface built from
the 1D inclusion density of Section 2.1 as a tensor product over x1, x2, x3.
"""
from __future__ import annotations

import numpy as np

# Voigt order used everywhere: (11, 22, 33, 23, 13, 12), tensor components.
VOIGT = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))


def lame_from_young(E, nu):
    """Isotropic Lame moduli (lambda, mu) for Young's modulus E and Poisson nu."""
    E = np.asarray(E, dtype=np.float64)
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def _shape(n):
    if np.isscalar(n):
        n = (int(n),) * 3
    n1, n2, n3 = (int(v) for v in n)
    return n1, n2, n3


def inclusion_indicator_sharp(n, side):
    """1 inside the centred cube of `side` voxels per axis, else 0.

    The cube covers voxel indices [(n_r - s_r)/2, (n_r + s_r)/2) on each axis,
    so every interface lies between two voxel centres (no sample sits on it).
    `side` may be a scalar or a per-axis triple (s1, s2, s3).
    """
    n1, n2, n3 = _shape(n)
    s1, s2, s3 = _shape(side)
    masks = []
    for nr, sr in ((n1, s1), (n2, s2), (n3, s3)):
        if (nr - sr) % 2:
            raise ValueError("n - side must be even for a centred cube")
        lo = (nr - sr) // 2
        m = np.zeros(nr)
        m[lo:lo + sr] = 1.0
        masks.append(m)
    m1, m2, m3 = masks
    return m3[:, None, None] * m2[None, :, None] * m1[None, None, :]


def inclusion_density_tanh(n, side, eps):
    """Tensor-product inclusion density nu(x1) nu(x2) nu(x3), smooth interface.

    nu(x) = phi(x; c_l) - phi(x; c_r), phi(x; c) = 1/2 + 1/2 tanh((x - c)/eps),
    with interface centres c_l = (n - s)/2 and c_r = (n + s)/2 (in voxel
    units, h = 1) and half-width eps, sampled at voxel centres x = i + 1/2.
    """
    n1, n2, n3 = _shape(n)
    s1, s2, s3 = _shape(side)
    dens = []
    for nr, sr in ((n1, s1), (n2, s2), (n3, s3)):
        x = np.arange(nr) + 0.5
        cl, cr = (nr - sr) / 2.0, (nr + sr) / 2.0
        phi = lambda c: 0.5 + 0.5 * np.tanh((x - c) / eps)
        dens.append(phi(cl) - phi(cr))
    d1, d2, d3 = dens
    return d3[:, None, None] * d2[None, :, None] * d1[None, None, :]


def cubic_inclusion(n, side, E_matrix=1.0, E_incl=10.0, nu=0.3, interface="sharp", eps=1.0):
    """Per-voxel (lambda, mu) for the centred cubic inclusion benchmark.

    Young's modulus is mixed with the inclusion density (sharp: 0/1 indicator;
    smooth: tanh density with half-width `eps` voxels); both phases share
    Poisson's ratio `nu`, so lambda and mu scale together by the contrast.
    Returns float64 arrays of shape (n3, n2, n1).
    """
    if interface == "sharp":
        d = inclusion_indicator_sharp(n, side)
    elif interface == "smooth":
        d = inclusion_density_tanh(n, side, eps)
    else:
        raise ValueError("interface must be 'sharp' or 'smooth'")
    E = E_matrix + (E_incl - E_matrix) * d
    lam, mu = lame_from_young(E, nu)
    return np.ascontiguousarray(lam), np.ascontiguousarray(mu)


def reference_medium_mean(E_matrix, E_incl, nu=0.3):
    """Reference medium C0: arithmetic mean of the two phases' Lame moduli."""
    lm, mm = lame_from_young(E_matrix, nu)
    li, mi = lame_from_young(E_incl, nu)
    return float(0.5 * (lm + li)), float(0.5 * (mm + mi))


def laminate(n, seed=0, E_range=(1.0, 100.0), nu_range=(0.1, 0.4)):
    """Random layered material: moduli vary with x1 only (layers normal to e1)."""
    n1, n2, n3 = _shape(n)
    rng = np.random.default_rng(seed)
    E = np.exp(rng.uniform(np.log(E_range[0]), np.log(E_range[1]), n1))
    nu = rng.uniform(nu_range[0], nu_range[1], n1)
    lam1, mu1 = lame_from_young(E, nu)
    lam = np.broadcast_to(lam1[None, None, :], (n3, n2, n1)).copy()
    mu = np.broadcast_to(mu1[None, None, :], (n3, n2, n1)).copy()
    return lam, mu


def random_moduli(n, seed=0, E_range=(1.0, 10.0), nu=0.3):
    """Voxelwise independent log-uniform Young's modulus (white-noise material)."""
    n1, n2, n3 = _shape(n)
    rng = np.random.default_rng(seed)
    E = np.exp(rng.uniform(np.log(E_range[0]), np.log(E_range[1]), (n3, n2, n1)))
    return lame_from_young(E, nu)


def random_strain_field(n, seed=0, scale=1e-3):
    """Random real symmetric strain field, Voigt-component major: (6, n3, n2, n1)."""
    n1, n2, n3 = _shape(n)
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal((6, n3, n2, n1))


def macro_strain(component=None, value=1.0):
    """Macroscopic strain as a Voigt 6-vector of TENSOR components.

    component: None (zero), an index 0..5 or a name '11','22','33','23','13','12'.
    A shear entry E_12 = value means E_12 = E_21 = value.
    """
    e = np.zeros(6)
    if component is None:
        return e
    names = {"11": 0, "22": 1, "33": 2, "23": 3, "13": 4, "12": 5, "xy": 5}
    idx = names[component] if isinstance(component, str) else int(component)
    e[idx] = value
    return e


def mandel_unit_strains():
    """Six unit strains in Mandel normalisation, as Voigt tensor-component 6-vectors.

    Shear unit strains have tensor components 1/sqrt(2), so that the 6x6
    effective stiffness assembled from them is the Mandel matrix.
    """
    out = np.eye(6)
    out[3:, 3:] /= np.sqrt(2.0)
    return out


def gaussian_random_field(n, corr_len=8.0, seed=7):
    """Standardised periodic Gaussian random field: white noise convolved with
    a Gaussian of standard deviation `corr_len` voxels (applied as the
    Gaussian's periodic transfer function), then shifted and scaled to zero
    mean and unit variance.  Shape (n3, n2, n1)."""
    n1, n2, n3 = _shape(n)
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n3, n2, n1))
    k3 = 2.0 * np.pi * np.fft.fftfreq(n3)[:, None, None]
    k2 = 2.0 * np.pi * np.fft.fftfreq(n2)[None, :, None]
    k1 = 2.0 * np.pi * np.fft.rfftfreq(n1)[None, None, :]
    filt = np.exp(-0.5 * corr_len ** 2 * (k1 ** 2 + k2 ** 2 + k3 ** 2))
    g = np.fft.irfftn(np.fft.rfftn(w, axes=(0, 1, 2)) * filt, s=(n3, n2, n1), axes=(0, 1, 2))
    g -= g.mean()
    return g / g.std()


def lognormal_young(n, corr_len=8.0, seed=7, log10_mean=1.0, log10_std=0.5, clip=(1.0, 100.0)):
    """Log-normal Young's modulus field E = clip(10^(log10_mean + log10_std g), clip)
    from `gaussian_random_field`."""
    g = gaussian_random_field(n, corr_len, seed)
    return np.clip(10.0 ** (log10_mean + log10_std * g), clip[0], clip[1])


def poisson_spheres(n, seed, mean_count=20, radius=(3.0, 8.0), log10_E=(0.0, 3.0), E_matrix=1.0):
    """Young's modulus field of a periodic cell with Poisson(mean_count)
    spheres: centres uniform in the cell, radii uniform in `radius` voxels,
    per-sphere log10 E uniform in `log10_E`, matrix E_matrix; a voxel belongs
    to a sphere when the periodic (minimum-image) distance of its centre to
    the sphere centre is at most the radius; overlaps keep the largest E.
    Shape (n3, n2, n1)."""
    n1, n2, n3 = _shape(n)
    rng = np.random.default_rng(seed)
    count = rng.poisson(mean_count)
    E = np.full((n3, n2, n1), float(E_matrix))
    x1 = np.arange(n1) + 0.5
    x2 = np.arange(n2) + 0.5
    x3 = np.arange(n3) + 0.5
    for _ in range(count):
        c = rng.uniform(0.0, 1.0, 3) * np.array([n1, n2, n3])
        r = rng.uniform(*radius)
        Ei = 10.0 ** rng.uniform(*log10_E)

        def d(x, c0, n0):
            t = np.abs(x - c0)
            return np.minimum(t, n0 - t)
        dist2 = (d(x3, c[2], n3)[:, None, None] ** 2 + d(x2, c[1], n2)[None, :, None] ** 2 +
                 d(x1, c[0], n1)[None, None, :] ** 2)
        E = np.where(dist2 <= r * r, np.maximum(E, Ei), E)
    return E
