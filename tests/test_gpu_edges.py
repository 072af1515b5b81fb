"""Edge cases of the 3D solver against the oracle, through the C ABI: the
shortest (4) and longest (512) supported axis lengths and radix-3 lengths in
every position (x lengths 4 to 512 in both stencil kernels), anisotropic grid spacing for every scheme and form (also with
an eigenstrain and for the DGO), a soft inclusion (contrast < 1), zero
macroscopic strain, maxit = 0, and a tolerance met at the first pass."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import green, solve1d, solve3d  # noqa: E402
from paper_2009_03762_amd import inputs  # noqa: E402

from oracle_ref import rel  # noqa: E402

NAMES = {"basic": "basic", "fb": "FB", "afb": "AFB", "cd": "CD", "acd": "ACD"}
EB = np.array([1e-3, -2e-4, 3e-4, 1e-4, -1e-4, 2e-4])


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2009_03762_amd import lsfft
    return lsfft


def _cell(n, chi, seed=0):
    lam, mu = inputs.random_moduli(n, seed=seed, E_range=(1.0, chi) if chi >= 1 else (chi, 1.0))
    return lam, mu, 0.5 * (lam.min() + lam.max()), 0.5 * (mu.min() + mu.max())


# (n1, n2, n3), n1 the fastest axis.  n1 = 12, 96, 192 take the register
# stencil with 192-thread workgroups (16, 2 and 1 y-groups), 384 and 512 the
# one-column-per-thread register stencil; lengths 4 to 512 and 3 x 2^a also
# sit in the y and z positions.
SHAPES = [(4, 4, 4), (8, 6, 4), (4, 4, 6), (4, 4, 512), (4, 512, 4), (512, 4, 4), (4, 6, 384), (12, 384, 8),
          (96, 6, 4), (192, 4, 6), (384, 4, 4)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("scheme,form", [("afb", "auto"), ("afb", "strain"), ("fb", "auto"), ("basic", "auto"),
                                         ("cd", "auto")])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_extreme_lengths_match_oracle(L, shape, scheme, form, prec):
    print(f"\n[edges] {shape} {scheme} {form} {prec}", flush=True)
    K = 8
    lam, mu, l0, m0 = _cell(shape, 10.0, seed=sum(shape))
    assert lam.shape == shape[::-1]
    s = L.Solver(lam, mu, l0, m0, scheme=scheme, prec=prec, form=form)
    out = s.solve(EB, tol=0.0, maxit=K)
    s.close()
    ref = solve3d.solve_gfp(lam, mu, EB, l0, m0, scheme=NAMES[scheme], tol=0.0, maxit=K)
    assert out["iters"] == K
    tol = 1e-12 if prec == "f64" else 1e-5
    assert rel(out["eps"], ref.eps) < tol
    assert rel(out["sig_mean"], ref.sig_mean) < tol


H = (0.5, 1.0, 2.0)


@pytest.mark.parametrize("scheme,form", [("afb", "displacement"), ("fb", "displacement"), ("afb", "strain"),
                                         ("fb", "strain"), ("basic", "auto"), ("cd", "auto"), ("acd", "auto")])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_anisotropic_spacing_matches_oracle(L, scheme, form, prec):
    shape = (16, 12, 8)
    print(f"\n[spacing] h={H} {scheme} {form} {prec}", flush=True)
    K = 10
    lam, mu = inputs.cubic_inclusion(shape, (8, 6, 4), 1.0, 10.0)
    l0, m0 = inputs.reference_medium_mean(1.0, 10.0)
    s = L.Solver(lam, mu, l0, m0, scheme=scheme, prec=prec, form=form, h=H)
    out = s.solve(EB, tol=0.0, maxit=K)
    s.close()
    ref = solve3d.solve_gfp(lam, mu, EB, l0, m0, scheme=NAMES[scheme], tol=0.0, maxit=K, h=H)
    tol = 1e-12 if prec == "f64" else 1e-5
    assert rel(out["eps"], ref.eps) < tol
    assert rel(out["sig"], ref.sig) < tol
    assert abs(out["residual"] - ref.residual) / ref.residual < (1e-9 if prec == "f64" else 1e-3)


@pytest.mark.parametrize("scheme,form", [("afb", "displacement"), ("fb", "displacement"), ("afb", "strain")])
def test_anisotropic_spacing_with_eigenstrain(L, scheme, form):
    shape = (16, 12, 8)
    print(f"\n[spacing+eig] {scheme} {form}", flush=True)
    lam, mu = inputs.cubic_inclusion(shape, (8, 6, 4), 1.0, 10.0)
    l0, m0 = inputs.reference_medium_mean(1.0, 10.0)
    es = 1e-3 * np.random.default_rng(2).standard_normal((6,) + lam.shape)
    s = L.Solver(lam, mu, l0, m0, scheme=scheme, prec="f64", form=form, h=H, eigenstrain=es)
    out = s.solve(EB, tol=1e-9, maxit=2000)
    s.close()
    ref = solve3d.solve_gfp(lam, mu, EB, l0, m0, scheme=NAMES[scheme], tol=1e-9, maxit=2000, h=H,
                            eigenstrain=es)
    assert out["status"] == L.OK and out["iters"] == ref.iters
    assert rel(out["eps"], ref.eps) < 1e-11


def test_anisotropic_spacing_dgo(L):
    shape = (8, 8, 8)
    print("\n[spacing dgo]", flush=True)
    lam, mu = inputs.cubic_inclusion(8, 4, 1.0, 5.0)
    l0, m0 = inputs.reference_medium_mean(1.0, 5.0)
    M, p, K = 2, 2, 10
    s = L.Solver(lam, mu, l0, m0, scheme="dgo", disc="pcd", prec="f64", dgo_images=M, dgo_weight_power=p, h=H)
    out = s.solve(EB, tol=0.0, maxit=K)
    s.close()
    Gc = green.dgo_voigt(shape, l0, m0, M, p, h=H)
    ref = solve3d.solve_dgo(lam, mu, EB, l0, m0, Gc, tol=0.0, maxit=K)
    assert rel(out["eps"], ref.eps) < 1e-12


@pytest.mark.parametrize("scheme,form", [("afb", "displacement"), ("afb", "strain"), ("basic", "auto")])
def test_soft_inclusion(L, scheme, form):
    """Contrast 1e-2 (a soft cube in a stiff matrix), converged FP64."""
    print(f"\n[soft] {scheme} {form}", flush=True)
    lam, mu = inputs.cubic_inclusion(16, 8, 1.0, 1e-2)
    l0, m0 = inputs.reference_medium_mean(1.0, 1e-2)
    s = L.Solver(lam, mu, l0, m0, scheme=scheme, prec="f64", form=form)
    out = s.solve(EB, tol=1e-9, maxit=5000)
    s.close()
    ref = solve3d.solve_gfp(lam, mu, EB, l0, m0, scheme=NAMES[scheme], tol=1e-9, maxit=5000)
    assert out["status"] == L.OK and out["iters"] == ref.iters
    assert rel(out["eps"], ref.eps) < 1e-11


@pytest.mark.parametrize("scheme,form", [("afb", "displacement"), ("afb", "strain"), ("basic", "auto"),
                                         ("fb", "displacement")])
def test_zero_load_maxit_zero_and_first_pass(L, scheme, form):
    lam, mu, l0, m0 = _cell((16, 8, 12), 10.0, seed=4)
    print(f"\n[degenerate] {scheme} {form}", flush=True)
    s = L.Solver(lam, mu, l0, m0, scheme=scheme, prec="f64", form=form)
    # zero macroscopic strain: every field is zero and the first pass is exact
    z = s.solve(np.zeros(6), tol=1e-12, maxit=50)
    assert z["status"] == L.OK and z["iters"] == 0
    assert np.abs(z["eps"]).max() == 0.0 and np.abs(z["sig"]).max() == 0.0
    # maxit = 0: the initial iterate, reported with its residual
    m = s.solve(EB, tol=1e-12, maxit=0)
    ref = solve3d.solve_gfp(lam, mu, EB, l0, m0, scheme=NAMES[scheme], tol=1e-12, maxit=0)
    assert m["status"] == L.ENOTCONV and m["iters"] == 0
    assert np.allclose(m["eps"], EB[:, None, None, None], rtol=0, atol=1e-18)
    assert abs(m["residual"] - ref.residual) <= 1e-12 * ref.residual
    # a tolerance above r_0 stops at once
    f = s.solve(EB, tol=2.0 * ref.residual, maxit=50)
    assert f["status"] == L.OK and f["iters"] == 0
    s.close()


def test_1d_anisotropic_spacing(L):
    """The 1D solver with h != 1 (the Green function scales with 1/h^2)."""
    print("\n[1d spacing]", flush=True)
    n = 48
    rng = np.random.default_rng(3)
    C = np.exp(rng.uniform(0.0, np.log(50.0), (3, n)))
    CH = 0.5 * (C.min(axis=1) + C.max(axis=1))
    out = L.solve_1d(C, CH, 1e-3, scheme="fd", disc="pcd", prec="f64", h=0.25, tol=0.0, maxit=12)
    for b in range(3):
        E = solve1d.solve_gfp_1d(C[b], 1e-3, CH[b], scheme="FD", tol=0.0, maxit=12, disc="PCD", h=0.25)[0]
        assert rel(out["E"][b], E) < 1e-12
