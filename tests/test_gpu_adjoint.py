"""GPU adjoint sensitivity (lsfft_stiffness_gradient behind a torch autograd
function) against the oracle's adjoint at 16^3, and against central finite
differences of GPU FP64 solves on 20 random voxels of the 128^3 log-normal
cell (a property that holds at any size: the adjoint gradient is the
derivative of J)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import adjoint as oadj  # noqa: E402
from paper_2009_03762_amd import inputs  # noqa: E402

NU = 0.3


@pytest.fixture(scope="module")
def A():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2009_03762_amd import adjoint
    return adjoint


def _ref_medium(E):
    l_lo, m_lo = inputs.lame_from_young(E.min(), NU)
    l_hi, m_hi = inputs.lame_from_young(E.max(), NU)
    return 0.5 * (float(l_lo) + float(l_hi)), 0.5 * (float(m_lo) + float(m_hi))


@pytest.mark.parametrize("prec,form_load", [("f64", "11"), ("f32", "11"), ("f64", "12")])
def test_gradient_matches_oracle_adjoint(A, prec, form_load):
    print(f"\n[adjoint16] prec={prec} load={form_load}", flush=True)
    E = inputs.lognormal_young(16, corr_len=2.0, seed=11)
    lam, mu = inputs.lame_from_young(E, NU)
    l0, m0 = _ref_medium(E)
    load = inputs.macro_strain(form_load, 1.0)
    J_ref, ea, eb = oadj.objective(lam, mu, load, load, l0, m0, scheme="AFB", tol=1e-12, maxit=20000)
    _, _, gE_ref = oadj.modulus_gradient(lam, mu, ea, eb)
    young = torch.tensor(E, requires_grad=True)
    J = A.effective_stiffness(young, NU, load, scheme="afb", prec=prec, tol=1e-12 if prec == "f64" else 0.0,
                              maxit=20000 if prec == "f64" else 400, f64_warmup=0 if prec == "f64" else 5)
    J.backward()
    g = young.grad.numpy()
    errJ = abs(J.item() - J_ref) / abs(J_ref)
    errg = np.linalg.norm(g - gE_ref) / np.linalg.norm(gE_ref)
    assert errJ < (1e-11 if prec == "f64" else 1e-6), errJ
    assert errg < (1e-9 if prec == "f64" else 2e-5), errg


def test_gradient_matches_finite_differences_128(A):
    """Config: 128^3 log-normal E (correlation length 8 voxels, clipped to
    [1, 100]), nu = 0.3, AFB, J = C_eff,1111; central differences (h = 1e-4
    relative) of FP64 GPU solves on 20 seeded random voxels."""
    print("\n[adjoint128] building", flush=True)
    from paper_2009_03762_amd import lsfft
    n = 128
    E = inputs.lognormal_young(n, corr_len=8.0, seed=7)
    l0, m0 = _ref_medium(E)
    load = inputs.macro_strain("11", 1.0)
    grads = {}
    for prec in ("f64", "f32"):
        young = torch.tensor(E, requires_grad=True)
        J = A.effective_stiffness(young, NU, load, lambda0=l0, mu0=m0, scheme="afb", prec=prec,
                                  tol=1e-10 if prec == "f64" else 0.0, maxit=5000 if prec == "f64" else 800,
                                  f64_warmup=0 if prec == "f64" else 5)
        J.backward()
        grads[prec] = (J.item(), young.grad.numpy())
    rng = np.random.default_rng(2024)
    vox = [tuple(int(v) for v in rng.integers(0, n, 3)) for _ in range(20)]
    h = 1e-4

    W = np.array([1.0, 1.0, 1.0, 2.0, 2.0, 2.0])

    def J_of(Ev):
        # the strain energy <eps : C : eps> equals J at convergence and is
        # stationary, so its error is quadratic in the iterate's (a mean
        # stress would be only first-order accurate)
        lam, mu = inputs.lame_from_young(Ev, NU)
        s = lsfft.Solver(lam, mu, l0, m0, scheme="afb", prec="f64")
        out = s.solve(load, tol=1e-10, maxit=5000)
        s.close()
        assert out["status"] == lsfft.OK
        return float(np.tensordot(W, out["eps"] * out["sig"], axes=(0, 0)).mean())

    g64, g32 = grads["f64"][1], grads["f32"][1]
    assert abs(grads["f32"][0] - grads["f64"][0]) < 1e-6 * abs(grads["f64"][0])
    for v in vox:
        Ep, Em = E.copy(), E.copy()
        Ep[v] *= 1 + h
        Em[v] *= 1 - h
        fd = (J_of(Ep) - J_of(Em)) / (2 * h * E[v])
        print(f"  voxel {v}: fd {fd:.6e} adjoint f64 {g64[v]:.6e} f32 {g32[v]:.6e}", flush=True)
        assert abs(fd - g64[v]) < 1e-4 * abs(fd), v
        assert abs(fd - g32[v]) < 1e-3 * abs(fd), v


@pytest.mark.parametrize("p", [1, 2])
def test_dgo_gradient_matches_oracle_and_differences(A, p):
    """The DGO's sensitivities from its own primal fields: against the oracle's
    DGO adjoint at 8^3 and against central differences of GPU DGO solves."""
    print(f"\n[adjoint dgo] p={p}", flush=True)
    from oracle import green
    n = 8
    # contrast 4: the single-sinc DGO (p = 1) diverges at high contrast
    E = np.exp(np.random.default_rng(13).uniform(0.0, np.log(4.0), (n, n, n)))
    lam, mu = inputs.lame_from_young(E, NU)
    l0, m0 = _ref_medium(E)
    load = inputs.macro_strain("11", 1.0)
    M = 2
    Gc = green.dgo_voigt((n, n, n), l0, m0, M, p)
    J_ref, ea, eb = oadj.objective(lam, mu, load, load, l0, m0, scheme="DGO", tol=1e-14, maxit=20000, Gc=Gc)
    assert np.isfinite(J_ref)
    _, _, gE_ref = oadj.modulus_gradient(lam, mu, ea, eb)

    def run(Ev, grad):
        young = torch.tensor(Ev, requires_grad=grad)
        J = A.effective_stiffness(young, NU, load, lambda0=l0, mu0=m0, scheme="dgo", prec="f64", tol=1e-14,
                                  maxit=20000, dgo_images=M, dgo_weight_power=p)
        if grad:
            J.backward()
            return J.item(), young.grad.numpy()
        return J.item(), None

    J, g = run(E, True)
    assert abs(J - J_ref) < 1e-11 * abs(J_ref)
    assert np.linalg.norm(g - gE_ref) < 1e-9 * np.linalg.norm(gE_ref)
    h = 1e-5
    for v in [(0, 0, 0), (3, 5, 1), (7, 2, 6)]:
        Ep, Em = E.copy(), E.copy()
        Ep[v] *= 1 + h
        Em[v] *= 1 - h
        fd = (run(Ep, False)[0] - run(Em, False)[0]) / (2 * h * E[v])
        assert abs(fd - g[v]) < 1e-6 * np.max(np.abs(g)), (v, fd, g[v])

