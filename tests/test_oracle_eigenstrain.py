"""Pins for the eigenstrain generalisation of the oracle (CPU only).

The law T = C [E - E_*] (Sec. 7) is checked against closed forms that do not
use the oracle: a laminate with layer eigenstrains, free expansion (a uniform
eigenstrain equal to Ebar leaves every material stress free), a homogeneous
cell, and the same discrete equations solved by dense LU.  A planted sign
error in the eigenstress is caught.
"""
import numpy as np
import pytest

from oracle import bounds, direct, green, solve3d
from paper_2009_03762_amd import inputs

EBAR = np.array([1e-3, 2e-4, -3e-4, 1e-4, 5e-5, 2e-4])
SCHEMES = ["basic", "FB", "AFB"]


def _ref(lam, mu):
    return 0.5 * (lam.min() + lam.max()), 0.5 * (mu.min() + mu.max())


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _layer_eigenstrain(n, seed):
    """Eigenstrain (6, n3, n2, n1) varying along x1 only, all six components."""
    n1, n2, n3 = n
    rng = np.random.default_rng(seed)
    e1 = 1e-3 * rng.standard_normal((6, n1))
    return e1, np.ascontiguousarray(np.broadcast_to(e1[:, None, None, :], (6, n3, n2, n1)))


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("shape", [(8, 8, 8), (12, 4, 6)])
def test_laminate_with_layer_eigenstrain(scheme, shape):
    lam, mu = inputs.laminate(shape, seed=3, E_range=(1.0, 50.0))
    e1, es = _layer_eigenstrain(shape, 11)
    l0, m0 = _ref(lam, mu)
    r = solve3d.solve_gfp(lam, mu, EBAR, l0, m0, scheme=scheme, tol=1e-13, maxit=5000, eigenstrain=es)
    assert r.status == solve3d.OK
    exact = bounds.laminate_strain_eig(lam[0, 0], mu[0, 0], EBAR, e1)
    exact = np.broadcast_to(exact[:, None, None, :], r.eps.shape)
    assert _rel(r.eps, exact) < 1e-10
    # T e1 is uniform and the mean stress is that of the exact field
    s = r.sig
    for c in (0, 4, 5):
        assert np.ptp(s[c]) <= 1e-10 * np.abs(s).max()


def test_laminate_closed_form_reduces_without_eigenstrain():
    lam1 = np.array([1.0, 3.0, 2.0, 5.0])
    mu1 = np.array([0.5, 1.0, 0.7, 2.0])
    a = bounds.laminate_strain(lam1, mu1, EBAR)
    b = bounds.laminate_strain_eig(lam1, mu1, EBAR, np.zeros((6, 4)))
    assert np.allclose(a, b, rtol=1e-14, atol=0)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_free_expansion_is_stress_free(scheme):
    """E_* = Ebar everywhere: E = Ebar and T = 0 in any material."""
    shape = (6, 4, 8)
    lam, mu = inputs.random_moduli(shape, seed=4, E_range=(1.0, 30.0))
    es = np.broadcast_to(EBAR[:, None, None, None], (6,) + lam.shape).copy()
    l0, m0 = _ref(lam, mu)
    r = solve3d.solve_gfp(lam, mu, EBAR, l0, m0, scheme=scheme, tol=1e-12, maxit=100, eigenstrain=es)
    assert r.status == solve3d.OK and r.iters == 0
    assert np.abs(r.sig).max() == 0.0
    assert np.allclose(r.eps, es, rtol=0, atol=1e-18)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_homogeneous_uniform_eigenstrain(scheme):
    """Homogeneous cell, uniform E_* = E0: E = Ebar, T = C [Ebar - E0] (exact)."""
    shape = (4, 6, 8)
    lam = np.full(shape[::-1], 2.0)
    mu = np.full(shape[::-1], 1.5)
    E0 = np.array([3e-4, -1e-4, 2e-4, 0.0, 1e-4, -2e-4])
    es = np.broadcast_to(E0[:, None, None, None], (6,) + lam.shape).copy()
    r = solve3d.solve_gfp(lam, mu, EBAR, 1.0, 1.0, scheme=scheme, tol=1e-12, eigenstrain=es)
    assert r.iters == 0 and r.status == solve3d.OK
    d = EBAR - E0
    tr = d[0] + d[1] + d[2]
    want = np.array([2.0 * tr + 3.0 * d[0], 2.0 * tr + 3.0 * d[1], 2.0 * tr + 3.0 * d[2],
                     3.0 * d[3], 3.0 * d[4], 3.0 * d[5]])
    assert np.allclose(r.sig_mean, want, rtol=1e-13, atol=0)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_fixed_point_with_eigenstrain_equals_dense_lu(scheme):
    shape = (4, 4, 4)
    lam, mu = inputs.random_moduli(shape, seed=7, E_range=(1.0, 20.0))
    es = 1e-3 * np.random.default_rng(5).standard_normal((6,) + lam.shape)
    l0, m0 = _ref(lam, mu)
    r = solve3d.solve_gfp(lam, mu, EBAR, l0, m0, scheme=scheme, tol=1e-14, maxit=5000, eigenstrain=es)
    d = direct.dense_gfp(lam, mu, EBAR, scheme=scheme, eigenstrain=es)
    assert r.status == solve3d.OK
    assert _rel(r.eps, d) < 1e-11


def test_dgo_with_eigenstrain_equals_dense_lu_and_laminate():
    shape = (4, 4, 4)
    lam, mu = inputs.random_moduli(shape, seed=9, E_range=(1.0, 4.0))
    es = 1e-3 * np.random.default_rng(6).standard_normal((6,) + lam.shape)
    l0, m0 = _ref(lam, mu)
    Gc = green.dgo_voigt(shape, l0, m0, M=2, p=2)
    r = solve3d.solve_dgo(lam, mu, EBAR, l0, m0, Gc, tol=1e-14, maxit=5000, eigenstrain=es)
    d = direct.dense_dgo(lam, mu, EBAR, l0, m0, Gc, eigenstrain=es)
    assert r.status == solve3d.OK
    assert _rel(r.eps, d) < 1e-10
    # pure eigenstrain loading (Ebar = 0): the stopping scale falls back to the RMS of E_*
    r0 = solve3d.solve_dgo(lam, mu, np.zeros(6), l0, m0, Gc, tol=1e-12, maxit=5000, eigenstrain=es)
    d0 = direct.dense_dgo(lam, mu, np.zeros(6), l0, m0, Gc, eigenstrain=es)
    assert r0.status == solve3d.OK and r0.iters > 1
    assert _rel(r0.eps, d0) < 1e-9


def test_planted_sign_error_in_eigenstress_is_caught(monkeypatch):
    shape = (8, 4, 4)
    lam, mu = inputs.laminate(shape, seed=3, E_range=(1.0, 50.0))
    e1, es = _layer_eigenstrain(shape, 12)
    l0, m0 = _ref(lam, mu)
    exact = bounds.laminate_strain_eig(lam[0, 0], mu[0, 0], EBAR, e1)
    real = solve3d.eigenstress
    monkeypatch.setattr(solve3d, "eigenstress", lambda l, m, E: -real(l, m, E))
    r = solve3d.solve_gfp(lam, mu, EBAR, l0, m0, scheme="AFB", tol=1e-13, maxit=5000, eigenstrain=es)
    assert _rel(r.eps, np.broadcast_to(exact[:, None, None, :], r.eps.shape)) > 1e-2
