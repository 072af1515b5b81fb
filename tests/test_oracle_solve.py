"""Pins for the oracle's fixed-point solvers (CPU only).

Each solver is checked against something other than itself: closed forms
(homogeneous material, laminates, the 1D analytic solution), other
algorithms for the same discrete equations (dense LU, conjugate gradients)
and rigorous bounds (Voigt / Reuss, Hashin-Shtrikman) on the effective
stiffness.
"""
import numpy as np
import pytest

from oracle import bounds, direct, green, solve1d, solve3d
from paper_2009_03762_amd import inputs

EBAR = np.array([1e-3, 2e-4, -3e-4, 1e-4, 5e-5, 2e-4])
SCHEMES = ["basic", "FB", "AFB"]


def _ref(lam, mu):
    return 0.5 * (lam.min() + lam.max()), 0.5 * (mu.min() + mu.max())


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_homogeneous_exact_at_first_pass(scheme):
    n = (8, 6, 4)
    lam = np.full((4, 6, 8), 2.0)
    mu = np.full((4, 6, 8), 1.5)
    r = solve3d.solve_gfp(lam, mu, EBAR, 1.0, 1.0, scheme=scheme, tol=1e-12)
    assert r.iters == 0 and r.status == solve3d.OK and r.residual <= 1e-14
    assert np.allclose(r.eps, EBAR[:, None, None, None] * np.ones((1, 4, 6, 8)), atol=1e-18)


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("shape", [(8, 8, 8), (12, 4, 6)])
def test_laminate_closed_form(scheme, shape):
    n1, n2, n3 = shape
    lam, mu = inputs.laminate(shape, seed=3, E_range=(1.0, 50.0))
    l0, m0 = _ref(lam, mu)
    r = solve3d.solve_gfp(lam, mu, EBAR, l0, m0, scheme=scheme, tol=1e-13, maxit=5000)
    assert r.status == solve3d.OK
    exact = bounds.laminate_strain(lam[0, 0], mu[0, 0], EBAR)
    exact = np.broadcast_to(exact[:, None, None, :], r.eps.shape)
    assert _rel(r.eps, exact) < 1e-10


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("shape", [(4, 4, 4), (6, 4, 8)])
def test_fixed_point_equals_dense_lu(scheme, shape):
    lam, mu = inputs.random_moduli(shape, seed=7, E_range=(1.0, 20.0))
    l0, m0 = _ref(lam, mu)
    r = solve3d.solve_gfp(lam, mu, EBAR, l0, m0, scheme=scheme, tol=1e-14, maxit=5000)
    d = direct.dense_gfp(lam, mu, EBAR, scheme=scheme)
    assert r.status == solve3d.OK
    assert _rel(r.eps, d) < 1e-11


@pytest.mark.parametrize("scheme,cg", [("AFB", "AFB_conj"), ("FB", "FB"), ("basic", "basic")])
def test_fixed_point_equals_conjugate_gradients(scheme, cg):
    lam, mu = inputs.cubic_inclusion(16, 8, 1.0, 30.0)
    l0, m0 = _ref(lam, mu)
    r = solve3d.solve_gfp(lam, mu, EBAR, l0, m0, scheme=scheme, tol=1e-13, maxit=5000)
    e, it = direct.pcg_gfp(lam, mu, EBAR, l0, m0, scheme=cg, tol=1e-13)
    assert _rel(r.eps, e) < 1e-10


def test_pcd_equals_td_on_voxel_data():
    # the PCD algorithm of Sec. 5.4 differs from TD only in where C is sampled
    lam, mu = inputs.cubic_inclusion((8, 6, 4), (4, 2, 2), 1.0, 10.0)
    l0, m0 = _ref(lam, mu)
    a = solve3d.solve_gfp(lam, mu, EBAR, l0, m0, scheme="AFB", tol=0.0, maxit=7, disc="TD")
    b = solve3d.solve_gfp(lam, mu, EBAR, l0, m0, scheme="AFB", tol=0.0, maxit=7, disc="PCD")
    assert _rel(a.eps, b.eps) < 1e-13


def test_paper_stopping_rule_reaches_same_solution():
    lam, mu = inputs.cubic_inclusion(8, 4, 1.0, 10.0)
    l0, m0 = _ref(lam, mu)
    a = solve3d.solve_gfp(lam, mu, EBAR, l0, m0, scheme="AFB", tol=1e-12, maxit=3000)
    b = solve3d.solve_gfp(lam, mu, EBAR, l0, m0, scheme="AFB", tol=1e-11, maxit=3000, stop="paper")
    assert b.status == solve3d.OK
    assert _rel(a.eps, b.eps) < 1e-9


def test_afb_needs_fewer_iterations_than_basic_at_high_contrast():
    # Sec. 6.1 (convergence versus contrast): AFB/R converges much faster
    lam, mu = inputs.cubic_inclusion(16, 8, 1.0, 1000.0)
    l0, m0 = _ref(lam, mu)
    E = inputs.macro_strain("12", 1e-3)
    a = solve3d.solve_gfp(lam, mu, E, l0, m0, scheme="AFB", tol=1e-6, maxit=3000)
    b = solve3d.solve_gfp(lam, mu, E, l0, m0, scheme="basic", tol=1e-6, maxit=300)
    assert a.status == solve3d.OK
    assert b.status == solve3d.ENOTCONV
    assert a.iters < 300 // 2


def test_effective_stiffness_bounds_and_symmetry():
    E_m, E_i = 1.0, 10.0
    lam, mu = inputs.cubic_inclusion(8, 4, E_m, E_i)
    l0, m0 = inputs.reference_medium_mean(E_m, E_i)
    units = inputs.mandel_unit_strains()
    M = solve3d.effective_stiffness(
        lambda E: solve3d.solve_gfp(lam, mu, E, l0, m0, scheme="AFB", tol=1e-12, maxit=3000), units)
    tol = 1e-8 * np.linalg.norm(M)
    assert np.linalg.norm(M - M.T) < tol
    V = bounds.voigt_mandel(lam, mu)
    R = bounds.reuss_mandel(lam, mu)
    assert np.min(np.linalg.eigvalsh(V - M)) > -tol
    assert np.min(np.linalg.eigvalsh(M - R)) > -tol
    lm, mm = inputs.lame_from_young(E_m, 0.3)
    li, mi = inputs.lame_from_young(E_i, 0.3)
    k1, _ = bounds.bulk_shear(lm, mm)
    k2, _ = bounds.bulk_shear(li, mi)
    f2 = float(np.mean(lam == li))
    assert bounds.bulk_from_mandel(M) >= bounds.hs_lower_bulk(k1, mm, k2, f2) - tol


# ---------------------------------------------------------------- 1D (Sec. 3)

def _c1d(n, chi=100.0, smooth=False):
    x = np.arange(n) + 0.5
    if smooth:
        phi = lambda c: 0.5 + 0.5 * np.tanh((x - c) / (n / 100.0))
        nu = phi(n / 4) - phi(3 * n / 4)
    else:
        nu = ((x > n / 4) & (x < 3 * n / 4)).astype(float)
    S = 1.0 + (1.0 / chi - 1.0) * nu      # compliance mixing, eq. (6)
    return 1.0 / S


@pytest.mark.parametrize("scheme", ["F", "FD", "FD_hC", "CD"])
@pytest.mark.parametrize("n", [10, 50, 90])
def test_1d_all_schemes_reach_analytic_nodal_solution(scheme, n):
    C = _c1d(n)
    CH = 0.5 * (C.min() + C.max())
    E, T, it, r = solve1d.solve_gfp_1d(C, 1.0, CH, scheme=scheme, tol=1e-13)
    Ea, Tbar = solve1d.analytic_strain(C, 1.0)
    if scheme == "CD" and n % 2 == 0:
        # CD also vanishes at the Nyquist index (Sec. 3.1): that stress mode stays free
        assert r <= 1e-13
        return
    assert np.allclose(E, Ea, rtol=1e-11)
    assert np.allclose(T, Tbar, rtol=1e-11)


def test_1d_pcd_equals_td():
    C = _c1d(32)
    CH = 0.5 * (C.min() + C.max())
    a = solve1d.solve_gfp_1d(C, 1.0, CH, scheme="FD", tol=1e-13, disc="TD")
    b = solve1d.solve_gfp_1d(C, 1.0, CH, scheme="FD", tol=1e-13, disc="PCD")
    assert np.allclose(a[0], b[0], rtol=1e-12)


def test_1d_dgo_deviation_decays_with_resolution():
    # Sec. 4: DGO nodal strains deviate from the analytic ones, less as n grows
    devs = []
    for n in (10, 50, 90):
        C = _c1d(n)
        CH = 0.5 * (C.min() + C.max())
        E, T, it, r = solve1d.solve_dgo_1d(C, 1.0, CH, M=n // 2, p=1, tol=1e-14)
        Ea, _ = solve1d.analytic_strain(C, 1.0)
        devs.append(np.max(np.abs(E - Ea)) / np.max(np.abs(Ea)))
    assert devs[0] > devs[1] > devs[2] > 0


def test_1d_dgo_printed_stress_form_forces_uniform_stress():
    # iterating on the full stress (as printed) has the fixed point T = const;
    # the polarisation form does not (why the polarisation reading is taken)
    C = _c1d(20, chi=2.0)
    CH = 0.5 * (C.min() + C.max())
    E, T, it, r = solve1d.solve_dgo_1d(C, 1.0, CH, M=3, p=1, tol=1e-14, form="stress")
    assert r <= 1e-14
    assert np.ptp(T) < 1e-10 * np.mean(T)
    E2, T2, it2, r2 = solve1d.solve_dgo_1d(C, 1.0, CH, M=3, p=1, tol=1e-14)
    assert np.ptp(T2) > 1e-3 * np.mean(T2)


# ---------------------------------------------------------------- DGO (Sec. 5.4)

@pytest.mark.parametrize("p", [1, 2])
def test_dgo_fixed_point_equals_dense_lu(p):
    lam, mu = inputs.random_moduli((4, 4, 4), seed=11, E_range=(1.0, 5.0))
    l0, m0 = _ref(lam, mu)
    Gc = green.dgo_voigt((4, 4, 4), l0, m0, 2, p)
    r = solve3d.solve_dgo(lam, mu, EBAR, l0, m0, Gc, tol=1e-15, maxit=5000)
    d = direct.dense_dgo(lam, mu, EBAR, l0, m0, Gc)
    assert _rel(r.eps, d) < 1e-11


def test_dgo_laminate_reduces_to_1d_dgo():
    # on a laminate the 3D DGO decouples into 1D DGO problems (normal: C = lambda+2mu,
    # shear: C = 2mu) with reference C_H = lambda0+2mu0 and 2mu0
    n = (8, 4, 4)
    M, p = 3, 1
    lam, mu = inputs.laminate(n, seed=5, E_range=(1.0, 4.0), nu_range=(0.3, 0.3))
    l0, m0 = _ref(lam, mu)
    Gc = green.dgo_voigt(n, l0, m0, M, p)
    E = inputs.macro_strain("12", 1e-3)
    r = solve3d.solve_dgo(lam, mu, E, l0, m0, Gc, tol=1e-15, maxit=5000)
    E1, T1, it, rr = solve1d.solve_dgo_1d(2 * mu[0, 0], 1e-3, 2 * m0, M, p, tol=1e-15)
    assert np.allclose(r.eps[5, 0, 0], E1, rtol=1e-10)
    E = inputs.macro_strain("11", 1e-3)
    r = solve3d.solve_dgo(lam, mu, E, l0, m0, Gc, tol=1e-15, maxit=5000)
    # normal component: sigma11 = (lambda+2mu) e11 + lambda (e22+e33), e22 = e33 = 0
    E1, T1, it, rr = solve1d.solve_dgo_1d(lam[0, 0] + 2 * mu[0, 0], 1e-3, l0 + 2 * m0, M, p, tol=1e-15)
    assert np.allclose(r.eps[0, 0, 0], E1, rtol=1e-10)


def test_dgo_homogeneous_is_exact():
    lam = np.full((4, 4, 4), 2.0)
    mu = np.full((4, 4, 4), 1.0)
    Gc = green.dgo_voigt((4, 4, 4), 2.0, 1.0, 2, 1)
    r = solve3d.solve_dgo(lam, mu, EBAR, 2.0, 1.0, Gc, tol=1e-14, maxit=10)
    assert r.iters == 1 and np.allclose(r.eps, EBAR[:, None, None, None], atol=1e-18)


# ---------------------------------------------------------------- planted mistakes

def test_planted_sign_error_in_hooke_is_caught(monkeypatch):
    orig = solve3d.hooke

    def bad(lam, mu, eps):
        tr = np.trace(eps, axis1=-2, axis2=-1)
        return -lam[..., None, None] * tr[..., None, None] * np.eye(3) + mu[..., None, None] * (
            eps + np.swapaxes(eps, -1, -2))

    monkeypatch.setattr(solve3d, "hooke", bad)
    lam, mu = inputs.laminate((8, 4, 4), seed=3, E_range=(1.0, 10.0))
    l0, m0 = _ref(lam, mu)
    r = solve3d.solve_gfp(lam, mu, EBAR, l0, m0, scheme="AFB", tol=1e-12, maxit=3000)
    exact = bounds.laminate_strain(lam[0, 0], mu[0, 0], EBAR)
    exact = np.broadcast_to(exact[:, None, None, :], r.eps.shape)
    assert _rel(r.eps, exact) > 1e-3
    monkeypatch.setattr(solve3d, "hooke", orig)


def test_planted_transpose_in_green_inverse_is_caught(monkeypatch):
    def bad(qa, qb, lam0, mu0):
        dot = np.einsum("...r,...r->...", qa, qb)
        return (-mu0 * dot[..., None, None] * np.eye(3)
                - mu0 * qb[..., :, None] * qa[..., None, :]
                - lam0 * qa[..., :, None] * qb[..., None, :])

    # the pin: the update of T = C_0 sym(v (x) q^a) must be -v (see test_oracle_green)
    from oracle import fdd
    lam0, mu0 = 2.3, 1.1
    qa, qb = fdd.scheme_pair("FB", (8, 6, 4))
    sing = fdd.singular_mask(qa, qb)
    rng = np.random.default_rng(3)
    v = rng.standard_normal(qa.shape) + 1j * rng.standard_normal(qa.shape)
    T = solve3d.hooke(np.full(qa.shape[:-1], lam0), np.full(qa.shape[:-1], mu0), green.sym_outer(v, qa))
    good = green.green_update(T, qa, qb, lam0, mu0, sing)
    assert np.allclose(good[~sing], -v[~sing], atol=1e-12)
    monkeypatch.setattr(green, "green_inverse", bad)
    planted = green.green_update(T, qa, qb, lam0, mu0, sing)
    assert not np.allclose(planted[~sing], -v[~sing], atol=1e-6)


def _homogeneous_with_eigenstrain(shape, alpha, seed=5):
    """Homogeneous C_1 = alpha C_0 loaded by a random eigenstrain (Sec. 7): the
    error of every GFP iterate is a compatible fluctuation, and one pass maps
    it to (1 - alpha) times itself (Gamma_0 C_0 is the projection onto
    compatible fields, eq. (34) with C_1 = alpha C_0), so the equilibrium norm
    is multiplied by exactly |1 - alpha| per iteration and the mean stress
    C_1 (Ebar - <E_*>) never changes."""
    n1, n2, n3 = shape
    l0, m0 = 1.3, 0.9
    lam = np.full((n3, n2, n1), alpha * l0)
    mu = np.full((n3, n2, n1), alpha * m0)
    es = 1e-3 * np.random.default_rng(seed).standard_normal((6, n3, n2, n1))
    return lam, mu, l0, m0, es


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("alpha", [0.4, 1.7])
def test_contraction_factor_closed_form(scheme, alpha):
    lam, mu, l0, m0, es = _homogeneous_with_eigenstrain((8, 6, 4), alpha)
    r = solve3d.solve_gfp(lam, mu, EBAR, l0, m0, scheme=scheme, tol=0.0, maxit=12, eigenstrain=es)
    h = np.array(r.history)
    assert r.status == solve3d.ENOTCONV and r.iters == 12
    assert np.allclose(h[1:] / h[:-1], abs(1.0 - alpha), rtol=1e-9)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_divergence_detected_where_the_closed_form_says(scheme):
    """C_0 = C_1 / 2.5 (below half the stiffness): the equilibrium norm grows
    by exactly 1.5 per iteration and first exceeds 1e6 times its initial value
    at k = ceil(log 1e6 / log 1.5) = 35, where the oracle must stop with
    EDIVERGED; r_k grows the same way (constant mean stress)."""
    alpha = 2.5
    lam, mu, l0, m0, es = _homogeneous_with_eigenstrain((8, 6, 4), alpha)
    r = solve3d.solve_gfp(lam, mu, EBAR, l0, m0, scheme=scheme, tol=1e-8, maxit=500, eigenstrain=es)
    k_expected = int(np.ceil(np.log(solve3d.DIVERGENCE_FACTOR) / np.log(alpha - 1.0)))
    assert k_expected == 35
    assert r.status == solve3d.EDIVERGED and r.iters == k_expected
    assert np.isclose(r.history[-1] / r.history[0], 1.5 ** k_expected, rtol=1e-8)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_reference_medium_below_half_the_stiffest_phase_diverges(scheme):
    """Cubic inclusion, contrast 10: with C_0 = C_I / 5 the basic, FB and AFB
    iterations diverge (detected within 20 iterations); with C_0 = 0.55 C_I
    (above half the stiffest phase) they converge."""
    lam, mu = inputs.cubic_inclusion(8, 4, 1.0, 10.0)
    li, mi = inputs.lame_from_young(10.0, 0.3)
    bad = solve3d.solve_gfp(lam, mu, EBAR, 0.2 * li, 0.2 * mi, scheme=scheme, tol=1e-10, maxit=300)
    assert bad.status == solve3d.EDIVERGED and bad.iters <= 20
    good = solve3d.solve_gfp(lam, mu, EBAR, 0.55 * li, 0.55 * mi, scheme=scheme, tol=1e-10, maxit=300)
    assert good.status == solve3d.OK
