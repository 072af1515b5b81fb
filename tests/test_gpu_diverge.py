"""Divergence is a numerical status, not a fault: a reference medium softer
than half the stiffest phase makes the fixed point of Sec. 5.2 diverge, and
the GPU must stop with LSFFT_EDIVERGED at the iteration the oracle stops at.
Every kernel returns normally; the stopping test on the device decides.

Two cases: a homogeneous cell C_1 = 2.5 C_0 loaded by a random eigenstrain
(Sec. 7), whose equilibrium norm grows by exactly 1.5 per iteration, so that
the divergence test (growth past 1e6 times the first value) fires at k = 35
by the closed form; and the cubic inclusion of contrast 10 with C_0 = C_I / 5,
against the oracle's stopping iteration."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import fdd, solve3d  # noqa: E402
from paper_2009_03762_amd import inputs  # noqa: E402

from oracle_ref import rel  # noqa: E402

NAMES = {"basic": "basic", "fb": "FB", "afb": "AFB", "cd": "CD", "acd": "ACD"}
EB = np.array([1e-3, -2e-4, 3e-4, 1e-4, -1e-4, 2e-4])
CASES = [("basic", "auto"), ("afb", "strain"), ("afb", "displacement"), ("fb", "displacement"), ("fb", "strain"),
         ("cd", "auto"), ("acd", "auto")]


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2009_03762_amd import lsfft
    return lsfft


@pytest.mark.parametrize("scheme,form", CASES)
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_homogeneous_closed_form_divergence(L, scheme, form, prec):
    print(f"\n[diverge closed form] {scheme} {form} {prec}", flush=True)
    shape = (16, 12, 8)
    n1, n2, n3 = shape
    alpha, l0, m0 = 2.5, 1.3, 0.9
    lam = np.full((n3, n2, n1), alpha * l0)
    mu = np.full((n3, n2, n1), alpha * m0)
    es = 1e-3 * np.random.default_rng(5).standard_normal((6, n3, n2, n1))
    s = L.Solver(lam, mu, l0, m0, scheme=scheme, prec=prec, form=form, eigenstrain=es)
    out = s.solve(EB, tol=1e-8, maxit=500)
    hist = s.residual_history()
    s.close()
    assert out["status"] == L.EDIVERGED and out["iters"] == 35
    ratio = hist[1:] / hist[:-1]
    # FP32: rounding noise grows with the diverging mode; the ratio stays near 1.5
    assert np.allclose(ratio, 1.5, rtol=1e-9 if prec == "f64" else 2e-2)
    ref = solve3d.solve_gfp(lam, mu, EB, l0, m0, scheme=NAMES[scheme], tol=1e-8, maxit=500, eigenstrain=es)
    assert ref.status == solve3d.EDIVERGED and ref.iters == 35


@pytest.mark.parametrize("scheme,form", CASES)
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_soft_reference_medium_diverges_with_the_oracle(L, scheme, form, prec):
    print(f"\n[diverge inclusion] {scheme} {form} {prec}", flush=True)
    n = 16
    lam, mu = inputs.cubic_inclusion(n, n // 2, 1.0, 10.0)
    li, mi = inputs.lame_from_young(10.0, 0.3)
    l0, m0 = 0.2 * li, 0.2 * mi
    nums = []
    qa, qb = fdd.scheme_pair(NAMES[scheme], (n, n, n))

    def grab(k, E, T, r):
        That = solve3d._transform(T, True, "TD")
        nums.append(solve3d.equilibrium_norm(That, qb))

    ref = solve3d.solve_gfp(lam, mu, EB, l0, m0, scheme=NAMES[scheme], tol=1e-10, maxit=300, callback=grab)
    assert ref.status == solve3d.EDIVERGED and ref.iters <= 20
    # the oracle's crossing is not a near tie that rounding could move
    g = np.array(nums) / (nums[0] * solve3d.DIVERGENCE_FACTOR)
    assert g[-1] > 1.02 and g[-2] < 0.98
    s = L.Solver(lam, mu, l0, m0, scheme=scheme, prec=prec, form=form)
    out = s.solve(EB, tol=1e-10, maxit=300)
    hist = s.residual_history()
    s.close()
    assert out["status"] == L.EDIVERGED and out["iters"] == ref.iters
    assert rel(hist, np.array(ref.history)) < (1e-9 if prec == "f64" else 1e-3)
