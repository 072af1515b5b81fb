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
    """The single-sinc weights of reading R9 are signed: at M = 3 some
    frequency of a small grid has an indefinite DGO (why p = 1 may diverge)."""
    n = (6, 4, 8)
    Gc = green.dgo_voigt(n, LAM0, MU0, 3, 1)
    mins = [np.linalg.eigvalsh(_energy_form(Gc[j3, j2, j1])).min()
            for j3 in range(8) for j2 in range(4) for j1 in range(6)]
    assert min(mins) < -1e-6


# ---------------------------------------------------------------------------
# Off-axis pin of the DGO image sum (Sec. 5.4, the DGO algorithm).  With
# squared weights the DGO is the continuous Gamma_0 acting on a voxelwise
# constant polarisation, averaged back over each voxel.  On a grid refined r
# times per axis that composition is computed here directly: repeat each voxel
# r^3 times, FFT, Gamma_0 at the plain continuum wavevector of every fine
# frequency, inverse FFT, average each voxel's r^3 samples, transform back.
# Exactly, this equals the image sum over the r^3 aliases kappa + nu n of each
# coarse frequency (|nu_r| <= (r - 1)/2 on odd grids), with the box filter of
# the r samples, D_r(m) = sin(pi m / n) / (r sin(pi m / (r n))), in place of
# the sinc; D_r -> sinc as r grows.  So dgo_voigt with its weight function
# replaced by D_r must reproduce the refined computation at every frequency,
# off-axis included, which pins its image wavevectors and the axis each
# weight applies to; with the sinc itself the two converge as r grows.


def _refined_gamma0(tau, r, lam0, mu0, h):
    """Voxel averages of Gamma_0 (paper's sign, eq. (48)) applied to the
    voxelwise constant field `tau` (6, n3, n2, n1), computed on an r-times
    refined grid; returned as the coarse DFT (6, n3, n2, n1), complex."""
    n3, n2, n1 = tau.shape[1:]
    fine = np.repeat(np.repeat(np.repeat(tau, r, axis=1), r, axis=2), r, axis=3)
    F = np.fft.fftn(fine, axes=(1, 2, 3))
    ks = []
    for n, hr, ax in ((n1, h[0], 2), (n2, h[1], 1), (n3, h[2], 0)):
        m = fourier.centred_index(r * n)
        shape = [1, 1, 1]
        shape[ax] = r * n
        ks.append(np.broadcast_to((2 * np.pi * m / (n * hr)).reshape(shape), (r * n3, r * n2, r * n1)))
    k = np.stack(ks, axis=-1)
    live = np.einsum("...r,...r->...", k, k) > 0.0
    T = green.from_voigt(np.moveaxis(F, 0, -1))
    out = np.zeros_like(T)
    out[live] = green.gamma_iso(k[live], lam0, mu0, T[live])
    back = np.fft.ifftn(np.moveaxis(green.to_voigt(out), -1, 0), axes=(1, 2, 3))
    avg = back.reshape(6, n3, r, n2, r, n1, r).mean(axis=(2, 4, 6))
    return np.fft.fftn(avg, axes=(1, 2, 3))


def _dirichlet(r, mirror=False, axis_len=None):
    """Box-filter weight D_r at the image m = kappa + nu n (see above).
    mirror: weight taken at kappa - nu n (a planted mistake); axis_len: a map
    n -> another axis's length (a planted mistake)."""

    def w(kappa, nu, n):
        nn = axis_len[n] if axis_len else n
        m = np.asarray(kappa - nu * nn if mirror else kappa + nu * nn, dtype=np.float64)
        with np.errstate(divide="ignore", invalid="ignore"):
            val = np.sin(np.pi * m / nn) / (r * np.sin(np.pi * m / (r * nn)))
        return np.where(m == 0, 1.0, val)

    return w


def _dgo_apply(Gc, tau):
    th = np.fft.fftn(tau, axes=(1, 2, 3))
    return np.einsum("...IJ,J...->I...", Gc, th)


N_ODD = (3, 5, 7)
H_ODD = (0.5, 1.0, 2.0)


@pytest.mark.parametrize("r", [3, 5])
def test_dgo_image_sum_equals_refined_grid_gamma0(monkeypatch, r):
    tau = np.random.default_rng(r).standard_normal((6,) + N_ODD[::-1])
    ref = _refined_gamma0(tau, r, LAM0, MU0, H_ODD)
    monkeypatch.setattr(green, "sinc_weight", _dirichlet(r))
    Gc = green.dgo_voigt(N_ODD, LAM0, MU0, (r - 1) // 2, 2, h=H_ODD)
    got = _dgo_apply(Gc, tau)
    scale = np.abs(ref).max()
    assert np.abs(got - ref).max() < 1e-12 * scale
    # most of the signal is off-axis: at least two nonzero indices
    kap = [fourier.centred_index(n) for n in N_ODD]
    off = ((kap[0][None, None, :] != 0).astype(int) + (kap[1][None, :, None] != 0) + (kap[2][:, None, None] != 0)) >= 2
    assert np.abs(ref[:, off]).max() > 0.5 * scale


@pytest.mark.parametrize("plant", ["mirrored image", "other axis length", "permuted wavevector"])
def test_dgo_refined_grid_pin_catches_planted_mistakes(monkeypatch, plant):
    r = 3
    tau = np.random.default_rng(9).standard_normal((6,) + N_ODD[::-1])
    ref = _refined_gamma0(tau, r, LAM0, MU0, H_ODD)
    if plant == "mirrored image":
        monkeypatch.setattr(green, "sinc_weight", _dirichlet(r, mirror=True))
    elif plant == "other axis length":
        monkeypatch.setattr(green, "sinc_weight", _dirichlet(r, axis_len={3: 5, 5: 7, 7: 3}))
    else:
        monkeypatch.setattr(green, "sinc_weight", _dirichlet(r))
        orig = green.gamma_iso_voigt
        monkeypatch.setattr(green, "gamma_iso_voigt", lambda k, l0, m0: orig(k[..., [1, 0, 2]], l0, m0))
    Gc = green.dgo_voigt(N_ODD, LAM0, MU0, 1, 2, h=H_ODD)
    got = _dgo_apply(Gc, tau)
    assert np.abs(got - ref).max() > 1e-3 * np.abs(ref).max()


def test_dgo_squared_sinc_is_the_limit_of_refined_grids():
    """With the sinc itself, the refined-grid result approaches dgo_voigt
    (p = 2, M = (r - 1)/2) as r grows: both tend to the full image sum (the
    gap, of the truncated tails and of D_r against the sinc, closes about
    like 1/r)."""
    tau = np.random.default_rng(4).standard_normal((6,) + N_ODD[::-1])
    errs = []
    for r in (3, 5, 9):
        ref = _refined_gamma0(tau, r, LAM0, MU0, H_ODD)
        got = _dgo_apply(green.dgo_voigt(N_ODD, LAM0, MU0, (r - 1) // 2, 2, h=H_ODD), tau)
        errs.append(np.abs(got - ref).max() / np.abs(ref).max())
    assert errs[0] > errs[1] > errs[2] and errs[2] < 0.4 * errs[0]


def test_dgo_even_grid_matches_refined_grid_off_nyquist(monkeypatch):
    """Even axes: every frequency with no Nyquist index, off-axis included,
    matches the refined computation (at a Nyquist index the refined grid's
    alias set is one-sided while the table's window is the symmetric one of
    reading R10)."""
    n, r = (6, 4, 8), 3
    tau = np.random.default_rng(2).standard_normal((6,) + n[::-1])
    ref = _refined_gamma0(tau, r, LAM0, MU0, (1.0, 1.0, 1.0))
    monkeypatch.setattr(green, "sinc_weight", _dirichlet(r))
    got = _dgo_apply(green.dgo_voigt(n, LAM0, MU0, 1, 2), tau)
    kap = [fourier.centred_index(v) for v in n]
    keep = ((kap[0][None, None, :] != -n[0] // 2) & (kap[1][None, :, None] != -n[1] // 2)
            & (kap[2][:, None, None] != -n[2] // 2))
    assert np.abs(got[:, keep] - ref[:, keep]).max() < 1e-12 * np.abs(ref).max()
