"""Pins for the oracle's Green operators (CPU only).

The isotropic stiffness is built here as the full fourth-order tensor
C_ijkl = lambda d_ij d_kl + mu (d_ik d_jl + d_il d_jk) (Sec. 5.1), so the
acoustic tensor, the Navier symbol and the projections are formed
independently of the formulas under test.
"""
import numpy as np
import pytest

from oracle import fdd, fourier, green
from oracle.green import VOIGT


def stiffness4(lam, mu):
    d = np.eye(3)
    return (lam * np.einsum("ij,kl->ijkl", d, d)
            + mu * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d)))


def acoustic(C4, k):
    return np.einsum("ijkl,j,l->ik", C4, k, k)


def navier_symbol(C4, qa, qb):
    # -div^b C grad^a acting on u (x) q^a: u_k -> -C_ijkl (u_k qa_l) qb_j
    return -np.einsum("ijkl,l,j->ik", C4, qa, qb)


LAM0, MU0 = 2.3, 1.1


def test_green_inverse_is_navier_symbol_for_every_pair():
    C4 = stiffness4(LAM0, MU0)
    rng = np.random.default_rng(0)
    for _ in range(20):
        qa = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        qb = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        assert np.allclose(green.green_inverse(qa, qb, LAM0, MU0), navier_symbol(C4, qa, qb),
                           atol=1e-13)


def test_green_tensor_is_inverse_acoustic_tensor():
    C4 = stiffness4(LAM0, MU0)
    rng = np.random.default_rng(1)
    for _ in range(20):
        k = rng.standard_normal(3)
        G = green.green_tensor_iso(k, LAM0, MU0)
        assert np.allclose(G @ acoustic(C4, k), np.eye(3), atol=1e-12)


def _voigt_stiffness(C4):
    # 6x6 matrix acting on Voigt tensor components (shear slot = both entries)
    M = np.zeros((6, 6))
    for J, (k, l) in enumerate(VOIGT):
        E = np.zeros((3, 3))
        E[k, l] = E[l, k] = 1.0
        S = np.einsum("ijkl,kl->ij", C4, E)
        M[:, J] = [S[i, j] for (i, j) in VOIGT]
    return M


def test_gamma_is_projection_onto_compatible_strains():
    C4 = stiffness4(LAM0, MU0)
    C6 = _voigt_stiffness(C4)
    rng = np.random.default_rng(2)
    for _ in range(10):
        k = rng.standard_normal(3)
        Gm = -green.gamma_iso_voigt(k, LAM0, MU0)      # Gamma_0 = -Gamma_H
        # Gamma_0 C_0 Gamma_0 = Gamma_0
        assert np.allclose(Gm @ C6 @ Gm, Gm, atol=1e-12)
        # Gamma_0 C_0 sym(u (x) k) = sym(u (x) k)
        u = rng.standard_normal(3)
        e = green.to_voigt(green.sym_outer(u, k))
        assert np.allclose(Gm @ C6 @ e, e, atol=1e-12)
        # equilibrated stresses (sigma k = 0) are annihilated
        A = rng.standard_normal((3, 3))
        A = A + A.T
        P = np.eye(3) - np.outer(k, k) / (k @ k)
        Aeq = P @ A @ P
        assert np.allclose(Gm @ green.to_voigt(Aeq), 0, atol=1e-12)


@pytest.mark.parametrize("scheme", ["basic", "FB", "AFB", "ACD"])
def test_general_update_inverts_reference_operator(scheme):
    # Delta u for T_check = C_0 sym(v (x) q^a) must be -v (definition of G)
    C4 = stiffness4(LAM0, MU0)
    n = (8, 6, 4)
    qa, qb = fdd.scheme_pair(scheme, n)
    sing = fdd.singular_mask(qa, qb)
    rng = np.random.default_rng(3)
    v = rng.standard_normal(qa.shape) + 1j * rng.standard_normal(qa.shape)
    E = green.sym_outer(v, qa)
    T = np.einsum("ijkl,...kl->...ij", C4, E)
    du = green.green_update(T, qa, qb, LAM0, MU0, sing)
    assert np.allclose(du[~sing], -v[~sing], atol=1e-12)
    assert np.all(du[sing] == 0)


@pytest.mark.parametrize("scheme", ["basic", "AFB"])
def test_general_update_equals_closed_form_at_real_wavevector(scheme):
    # strain update sym(G T q^b (x) q^a) equals Gamma_H(k_eff) T with k_eff the
    # real vector q^b / i (basic: k; AFB: the rotated k^R), Sec. 5.4 eq. (48)
    n = (8, 6, 4)
    qa, qb = fdd.scheme_pair(scheme, n)
    sing = fdd.singular_mask(qa, qb)
    keff = (qb / 1j).real if scheme == "AFB" else (qa / 1j).real
    rng = np.random.default_rng(4)
    A = rng.standard_normal(qa.shape[:-1] + (3, 3)) + 1j * rng.standard_normal(qa.shape[:-1] + (3, 3))
    A = A + np.swapaxes(A, -1, -2)
    du = green.green_update(A, qa, qb, LAM0, MU0, sing)
    de = green.sym_outer(du, qa)
    ok = ~sing
    ref = green.gamma_iso(keff[ok], LAM0, MU0, A[ok])
    assert np.allclose(de[ok], ref, atol=1e-12)


@pytest.mark.parametrize("scheme", ["basic", "FB", "AFB"])
def test_update_of_real_field_is_real(scheme):
    # the Green step maps the transform of a real stress to that of a real strain
    n = (8, 6, 4)
    qa, qb = fdd.scheme_pair(scheme, n)
    sing = fdd.singular_mask(qa, qb)
    rng = np.random.default_rng(5)
    T = rng.standard_normal((4, 6, 8, 3, 3))
    T = T + np.swapaxes(T, -1, -2)
    Tv = np.moveaxis(green.to_voigt(T), -1, 0)
    Th = green.from_voigt(np.moveaxis(fourier.td_forward(Tv), 0, -1))
    de = green.sym_outer(green.green_update(Th, qa, qb, LAM0, MU0, sing), qa)
    back = fourier.td_inverse(np.moveaxis(green.to_voigt(de), -1, 0))
    assert np.max(np.abs(back.imag)) < 1e-13 * np.max(np.abs(back.real))


def test_plain_symbol_without_nyquist_rule_breaks_realness():
    # documents why the basic scheme needs the real-field Nyquist reading
    n = (8, 6, 4)
    qa = fdd.symbols_3d("F", n)
    qb = np.conj(qa)
    sing = fdd.singular_mask(qa, qb)
    rng = np.random.default_rng(5)
    T = rng.standard_normal((4, 6, 8, 3, 3))
    T = T + np.swapaxes(T, -1, -2)
    Tv = np.moveaxis(green.to_voigt(T), -1, 0)
    Th = green.from_voigt(np.moveaxis(fourier.td_forward(Tv), 0, -1))
    de = green.sym_outer(green.green_update(Th, qa, qb, LAM0, MU0, sing), qa)
    back = fourier.td_inverse(np.moveaxis(green.to_voigt(de), -1, 0))
    assert np.max(np.abs(back.imag)) > 1e-3 * np.max(np.abs(back.real))


@pytest.mark.parametrize("p", [1, 2])
def test_sinc_image_sums_tend_to_one(p):
    # sum_nu sinc^p(pi (x + nu)) = 1 for p = 1, 2 (partition of unity)
    n = 16
    for kappa in (1, 3, -5, 7):
        s = [sum(green.sinc_weight(kappa, v, n) ** p for v in range(-M, M + 1)) for M in (4, 64, 2048)]
        err = [abs(x - 1.0) for x in s]
        assert err[2] < err[0] and err[2] < 5e-3
    # kappa = 0: only the nu = 0 image carries weight
    assert green.sinc_weight(0, 0, n) == 1.0
    assert all(green.sinc_weight(0, v, n) == 0.0 for v in (-3, -1, 1, 2))


def test_dgo_on_axis_reduces_to_scaled_gamma():
    # at (kappa1, 0, 0) only images along e1 carry weight; all are parallel to e1
    n = (8, 6, 4)
    M, p = 3, 1
    Gc = green.dgo_voigt(n, LAM0, MU0, M, p)
    e1 = np.array([1.0, 0.0, 0.0])
    base = green.gamma_iso_voigt(e1, LAM0, MU0)
    for j1 in range(1, 8):
        a = int(fourier.centred_index(8)[j1])
        c = sum(green.sinc_weight(a, v, 8) ** p for v in green.image_range(a, 8, M))
        assert np.allclose(Gc[0, 0, j1], c * base, atol=1e-13)


def test_dgo_pointwise_matches_table_and_is_even():
    n = (6, 4, 8)
    Gc = green.dgo_voigt(n, LAM0, MU0, 2, 2)
    for f in [(1, 2, 3), (3, 0, 4), (5, 3, 7)]:
        assert np.allclose(Gc[f[2], f[1], f[0]], green.dgo_voigt_at(f, n, LAM0, MU0, 2, 2), atol=1e-13)
    # symmetric image window => Gamma^c(-xi) = Gamma^c(xi)
    for j3 in range(8):
        for j2 in range(4):
            for j1 in range(6):
                assert np.allclose(Gc[j3, j2, j1], Gc[(-j3) % 8, (-j2) % 4, (-j1) % 6], atol=1e-13)


def _energy_form(G6):
    """Symmetric part of the quadratic form -tau : Gamma tau in Voigt tensor
    components (shear entries counted twice).  The operators carry the
    paper's sign (Gamma_hat = -sym[G A k (x) k]), so -Gamma is the positive
    one."""
    W = np.diag([1.0, 1.0, 1.0, 2.0, 2.0, 2.0])
    A = -W @ G6
    return 0.5 * (A + A.T)


def test_dgo_squared_sinc_is_positive_semidefinite():
    """With squared-sinc weights the DGO is a non-negative combination of the
    continuous Gamma_0 at the image frequencies, each positive semidefinite
    for the energy tau : Gamma tau; the table must keep that at every
    frequency (a wrong sign in any image term or in Gamma_0 breaks it)."""
    n = (6, 4, 8)
    Gc = green.dgo_voigt(n, LAM0, MU0, 2, 2)
    top = max(np.abs(_energy_form(Gc[j3, j2, j1])).max() for j3 in range(8) for j2 in range(4) for j1 in range(6))
    for j3 in range(8):
        for j2 in range(4):
            for j1 in range(6):
                ev = np.linalg.eigvalsh(_energy_form(Gc[j3, j2, j1]))
                assert ev.min() >= -1e-12 * top
    # the continuous operator itself, at a generic wavevector
    ev = np.linalg.eigvalsh(_energy_form(green.gamma_iso_voigt(np.array([0.3, -1.2, 0.7]), LAM0, MU0)))
    assert ev.min() >= -1e-12 and ev.max() > 0.0


def test_dgo_single_sinc_weights_can_be_indefinite():
    """The single-sinc weights of reading R14 are signed: at M = 3 some
    frequency of a small grid has an indefinite DGO (why p = 1 may diverge)."""
    n = (6, 4, 8)
    Gc = green.dgo_voigt(n, LAM0, MU0, 3, 1)
    mins = [np.linalg.eigvalsh(_energy_form(Gc[j3, j2, j1])).min()
            for j3 in range(8) for j2 in range(4) for j1 in range(6)]
    assert min(mins) < -1e-6
