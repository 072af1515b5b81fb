"""Effective wavenumbers of the finite-difference discretisations (FDD).
TEST INFRASTRUCTURE ONLY (see the package docstring).

1D symbols, Sec. 3.1 eqs. (12)-(14), with q = i k and h the grid spacing:
    q^F  = q                               (plain Fourier, "F")
    q^FD = h^{-1} (e^{q h} - 1)            (forward difference)
    q^BD = h^{-1} (1 - e^{-q h})           (backward difference)
    q^CD = h^{-1} sinh(q h)                (central difference)
    q^hC = 2 h^{-1} sinh(q h / 2)          (half-central difference)
3D averaged symbols, Sec. 5.3 eq. (43), (s, t) = (2,3), (3,1), (1,2) for r = 1,2,3:
    q^AFD_r = 1/4 q^FD_r (e^{q_s h_s} + 1)(e^{q_t h_t} + 1)
    q^ABD_r = 1/4 q^BD_r (e^{-q_s h_s} + 1)(e^{-q_t h_t} + 1)
    q^ACD_r = q^CD_r cosh(q_s h_s) cosh(q_t h_t)
    q^AhC_r = q^hC_r cosh(q_s h_s / 2) cosh(q_t h_t / 2)
Willot's rotated-scheme wavenumber, Sec. 5.3 eq. (44):
    q^R_r = 1/4 q^W_r (e^{q_s h_s} + 1)(e^{q_t h_t} + 1),
    q^W = h^{-1} tanh(q h / 2)(e^{q h} + 1)      (indeterminate at Nyquist)
Pairs (a, b) of gradient / divergence symbols: the conjugacy rule
q^b = conj(q^a) of Sec. 3.1 eq. (18) and Sec. 5.3 eq. (45), or the AFB/R pair
(a_r, b_r) = (AFD, AhC) defined at the end of Sec. 5.3.

The unit-modulus factors e^{i 2 pi kappa / n} are evaluated exactly at
multiples of a quarter turn (so e^{-i pi} + 1 is exactly 0, not 1e-16 i);
everywhere else they are numpy's exp of the rounded angle.  Exact zeros matter
because the singular-frequency rule below tests q^a . q^b == 0.
"""
from __future__ import annotations

import numpy as np

from .fourier import centred_index

# Pair definitions: scheme name -> (gradient symbol, divergence symbol rule).
# "conj" means q^b = conj(q^a) (the conjugacy rule).
SCHEMES = {
    "basic": ("F", "conj"),        # plain Fourier wavevectors (basic scheme)
    "CD": ("CD", "conj"),
    "FB": ("FD", "conj"),          # forward gradient, q^b = conj(q^FD) = -q^BD
    "FB_hC": ("FD", "hC"),         # 1D (FD, hC) choice carried to 3D; oracle-only
    "ACD": ("ACD", "conj"),
    "AFB": ("AFD", "AhC"),         # averaged forward-backward / rotated scheme
    "AFB_conj": ("AFD", "conj"),   # AFD with conjugacy, q^b = -q^ABD
}


def cis_turns(num, den):
    """exp(2 pi i num / den) for integer arrays num and integer den.

    Exact (+1, +i, -1, -i) wherever 4 num / den is an integer.
    """
    num = np.asarray(num, dtype=np.int64)
    z = np.exp(2j * np.pi * (num.astype(np.float64) / den))
    q = 4 * num
    exact = (q % den) == 0
    quarter = (q // den) % 4
    table = np.array([1.0 + 0j, 1j, -1.0 + 0j, -1j])
    z = np.where(exact, table[quarter], z)
    return z


def symbols_1d(n, h=1.0):
    """All 1D symbols of eqs. (12)-(14) for the n centred indices (numpy order)."""
    kap = centred_index(n)
    e = cis_turns(kap, n)            # e^{q h}
    ei = cis_turns(-kap, n)          # e^{-q h}
    eh = cis_turns(kap, 2 * n)       # e^{q h / 2}
    ehi = cis_turns(-kap, 2 * n)     # e^{-q h / 2}
    out = {
        "F": 1j * 2.0 * np.pi * kap / (n * h),
        "FD": (e - 1.0) / h,
        "BD": (1.0 - ei) / h,
        "CD": (e - ei) / (2.0 * h),
        "hC": (eh - ehi) / h,
        # factors used by the averaged symbols
        "ep1": e + 1.0,                 # e^{q h} + 1
        "em1": ei + 1.0,                # e^{-q h} + 1
        "cosh": 0.5 * (e + ei),         # cosh(q h)
        "cosh_half": 0.5 * (eh + ehi),  # cosh(q h / 2)
    }
    with np.errstate(divide="ignore", invalid="ignore"):
        tanh_half = (eh - ehi) / (eh + ehi)
        out["W"] = tanh_half * (e + 1.0) / h
    return out


def _grid(n):
    if np.isscalar(n):
        n = (int(n),) * 3
    return tuple(int(v) for v in n)


def _bcast(v1, v2, v3):
    """Broadcast per-axis arrays to the (n3, n2, n1) spectrum grid."""
    return (v1[None, None, :], v2[None, :, None], v3[:, None, None])


def symbols_3d(kind, n, h=(1.0, 1.0, 1.0)):
    """3D symbol vector q^kind as an array (n3, n2, n1, 3), component r = x_r.

    kind: 'F', 'FD', 'BD', 'CD', 'hC' (componentwise 1D symbols, eq. (32)),
    or the averaged 'AFD', 'ABD', 'ACD', 'AhC' of eq. (43), or 'R' of eq. (44).
    """
    n1, n2, n3 = _grid(n)
    s = [symbols_1d(nr, hr) for nr, hr in zip((n1, n2, n3), h)]
    shape = (n3, n2, n1)

    def axis(r, key):
        v = [np.ones(1), np.ones(1), np.ones(1)]
        v[r] = s[r][key]
        b = _bcast(*v)
        return np.broadcast_to(b[r], shape)

    q = np.zeros(shape + (3,), dtype=np.complex128)
    base = {"AFD": "FD", "ABD": "BD", "ACD": "CD", "AhC": "hC", "R": "W"}
    fac = {"AFD": ("ep1", 0.5), "ABD": ("em1", 0.5), "ACD": ("cosh", 1.0),
           "AhC": ("cosh_half", 1.0), "R": ("ep1", 0.5)}
    for r in range(3):
        if kind in ("F", "FD", "BD", "CD", "hC"):
            q[..., r] = axis(r, kind)
        elif kind in base:
            st = [(1, 2), (2, 0), (0, 1)][r]
            key, scale = fac[kind]
            val = axis(r, base[kind])
            for t in st:
                val = val * (scale * axis(t, key))
            q[..., r] = val
        else:
            raise ValueError(kind)
    return q


def real_field_nyquist_rule(q, n):
    """Plain-Fourier wavevector made consistent with real fields on even axes.

    At a Nyquist index kappa_r = -n_r/2 the Hermitian partner of a frequency
    has the SAME r-component, while its other components flip sign; the
    plain symbol i k then gives the partner a wavevector that is not +-k, so
    the Green update of a real field would not be real.  Reading: where an
    axis sits at its Nyquist index and some non-Nyquist component is nonzero,
    that Nyquist component is set to 0 (the nodal derivative of the real
    trigonometric interpolant of the Nyquist mode).  Frequencies whose only
    nonzero components are Nyquist ones keep i k, which is already consistent;
    so do all 1D problems, matching Sec. 3.1.
    """
    n1, n2, n3 = n
    q = q.copy()
    nyq = []
    for r, nr in enumerate((n1, n2, n3)):
        m = np.zeros((n3, n2, n1), dtype=bool)
        if nr % 2 == 0:
            kap = centred_index(nr)
            sl = [None, None, None]
            sl[2 - r] = slice(None)
            m = np.broadcast_to((kap == -nr // 2)[tuple(sl)], (n3, n2, n1))
        nyq.append(m)
    for r in range(3):
        others = [t for t in range(3) if t != r]
        other_live = np.zeros((n3, n2, n1), dtype=bool)
        for t in others:
            other_live |= (q[..., t] != 0) & ~nyq[t]
        q[..., r] = np.where(nyq[r] & other_live, 0.0, q[..., r])
    return q


def scheme_pair(scheme, n, h=(1.0, 1.0, 1.0)):
    """(q^a, q^b) arrays (n3, n2, n1, 3) for a named scheme (see SCHEMES)."""
    a, b = SCHEMES[scheme]
    qa = symbols_3d(a, n, h)
    if a == "F":
        qa = real_field_nyquist_rule(qa, _grid(n))
    qb = np.conj(qa) if b == "conj" else symbols_3d(b, n, h)
    return qa, qb


def singular_mask(qa, qb):
    """Frequencies where q^a . q^b == 0 exactly: there G is set to zero.

    Sec. 3.1 (after Algorithm 1 of the TD series) sets the Green function to
    zero where the symbols vanish; in 3D the inverse of eq. (34) exists iff
    q^a . q^b != 0 (Sec. 5.2).
    """
    return np.einsum("...r,...r->...", qa, qb) == 0
