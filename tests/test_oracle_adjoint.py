"""Pins of the oracle's adjoint sensitivity (oracle/adjoint.py) by central
finite differences of the oracle's own converged effective stiffness: no
formula is shared between the two sides of each check."""
import numpy as np
import pytest

from oracle import adjoint
from paper_2009_03762_amd import inputs

N_ = 8
NU = 0.3


def _cell(seed=3):
    E = inputs.lognormal_young(N_, corr_len=1.5, seed=seed)
    lam, mu = inputs.lame_from_young(E, NU)
    l_lo, m_lo = inputs.lame_from_young(E.min(), NU)
    l_hi, m_hi = inputs.lame_from_young(E.max(), NU)
    return E, lam, mu, 0.5 * (l_lo + l_hi), 0.5 * (m_lo + m_hi)


def _J(lam, mu, A, B, l0, m0, scheme="AFB"):
    return adjoint.objective(lam, mu, A, B, l0, m0, scheme=scheme, tol=1e-13, maxit=20000)


VOX = [(0, 0, 0), (3, 5, 1), (7, 2, 6), (4, 4, 4)]


@pytest.mark.parametrize("scheme", ["AFB", "basic"])
def test_young_gradient_matches_central_differences(scheme):
    E, lam, mu, l0, m0 = _cell()
    A = inputs.macro_strain("11", 1.0)
    J, ea, eb = _J(lam, mu, A, A, l0, m0, scheme)
    _, _, gE = adjoint.modulus_gradient(lam, mu, ea, eb)
    h = 1e-4
    for v in VOX:
        Ep, Em = E.copy(), E.copy()
        Ep[v] *= 1 + h
        Em[v] *= 1 - h
        Jp = _J(*inputs.lame_from_young(Ep, NU), A, A, l0, m0, scheme)[0]
        Jm = _J(*inputs.lame_from_young(Em, NU), A, A, l0, m0, scheme)[0]
        fd = (Jp - Jm) / (2 * h * E[v])
        assert abs(fd - gE[v]) < 1e-6 * abs(gE[v]), (v, fd, gE[v])


def test_lambda_and_mu_gradients_match_central_differences():
    E, lam, mu, l0, m0 = _cell(5)
    A = inputs.macro_strain("11", 1.0)
    B = inputs.macro_strain("22", 1.0)
    J, ea, eb = _J(lam, mu, A, B, l0, m0)
    gl, gm, _ = adjoint.modulus_gradient(lam, mu, ea, eb)
    for v in VOX[:2]:
        for which, g in (("lam", gl), ("mu", gm)):
            h = 1e-4 * (lam[v] if which == "lam" else mu[v])
            lp, mp, lm_, mm = lam.copy(), mu.copy(), lam.copy(), mu.copy()
            if which == "lam":
                lp[v] += h
                lm_[v] -= h
            else:
                mp[v] += h
                mm[v] -= h
            fd = (_J(lp, mp, A, B, l0, m0)[0] - _J(lm_, mm, A, B, l0, m0)[0]) / (2 * h)
            assert abs(fd - g[v]) < 1e-6 * np.max(np.abs(g)), (which, v, fd, g[v])


@pytest.mark.parametrize("p", [1, 2])
def test_dgo_gradients_match_central_differences(p):
    """The DGO is self-adjoint too (G symmetric, even, zero on uniform fields):
    its own primal fields give dJ/dlambda and dJ/dmu."""
    from oracle import green
    n = (4, 4, 4)
    lam, mu = inputs.random_moduli(n, seed=3, E_range=(1.0, 4.0))
    l0, m0 = 0.5 * (lam.min() + lam.max()), 0.5 * (mu.min() + mu.max())
    Gc = green.dgo_voigt(n, l0, m0, M=2, p=p)
    A = np.array([1.0, 0.0, 0.0, 0.0, 0.0, 0.0])
    B = np.array([0.0, 0.5, 0.0, 0.0, 0.0, 0.3])

    def J(lam_, mu_):
        return adjoint.objective(lam_, mu_, A, B, l0, m0, scheme="DGO", tol=1e-15, maxit=20000, Gc=Gc)

    J0, ea, eb = J(lam, mu)
    gl, gm, _ = adjoint.modulus_gradient(lam, mu, ea, eb)
    h = 1e-6
    for v in [(0, 0, 0), (1, 2, 3), (3, 1, 0)]:
        lp, lm_ = lam.copy(), lam.copy()
        lp[v] += h
        lm_[v] -= h
        fd_l = (J(lp, mu)[0] - J(lm_, mu)[0]) / (2 * h)
        mp, mm = mu.copy(), mu.copy()
        mp[v] += h
        mm[v] -= h
        fd_m = (J(lam, mp)[0] - J(lam, mm)[0]) / (2 * h)
        assert abs(fd_l - gl[v]) < 1e-6 * np.max(np.abs(gl)), (v, fd_l, gl[v])
        assert abs(fd_m - gm[v]) < 1e-6 * np.max(np.abs(gm)), (v, fd_m, gm[v])
    # and its effective stiffness is symmetric
    Jba = adjoint.objective(lam, mu, B, A, l0, m0, scheme="DGO", tol=1e-15, maxit=20000, Gc=Gc)[0]
    assert abs(J0 - Jba) < 1e-12 * abs(J0)


def test_objective_is_symmetric_in_the_loads():
    E, lam, mu, l0, m0 = _cell(7)
    A = np.array([1.0, 0.2, -0.3, 0.1, 0.05, 0.4])
    B = np.array([-0.2, 1.0, 0.1, 0.3, -0.1, 0.2])
    Jab = _J(lam, mu, A, B, l0, m0)[0]
    Jba = _J(lam, mu, B, A, l0, m0)[0]
    assert abs(Jab - Jba) < 1e-10 * abs(Jab)


def test_planted_factor_error_is_caught():
    # the shear-modulus sensitivity without its factor 2 must fail the FD pin
    E, lam, mu, l0, m0 = _cell()
    A = inputs.macro_strain("12", 1.0)
    J, ea, eb = _J(lam, mu, A, A, l0, m0)
    gm_wrong = adjoint.contract(ea, eb) / lam.size
    v = VOX[1]
    h = 1e-4 * mu[v]
    mp, mm = mu.copy(), mu.copy()
    mp[v] += h
    mm[v] -= h
    fd = (_J(lam, mp, A, A, l0, m0)[0] - _J(lam, mm, A, A, l0, m0)[0]) / (2 * h)
    assert abs(fd - gm_wrong[v]) > 0.1 * abs(fd)
