"""Every transform length of the displacement form in every axis position,
against the oracle at fixed iteration counts (Sec. 5.2, Alg. T3, with the
(AFD, AhC) and (FD, conj FD) pairs of Sec. 5.3, eq. (43)).

Shapes are written (n1, n2, n3), n1 the fastest axis; each test asserts the
array it hands over has n1 as its last extent, and names the kernel
instantiations the library launched (`lsfft_describe`), so the lengths below
reach the register stencil of n1 columns, the y pass of n2 and the z pass of
n3 that the benchmark and the batched cells run.  Moduli are voxelwise white
noise (Young's contrast 100), so every frequency plane carries signal; besides
the global relative L2 the Nyquist planes and the zero-frequency lines of the
strain spectrum are compared on their own."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import solve3d  # noqa: E402
from paper_2009_03762_amd import inputs  # noqa: E402

from oracle_ref import plane_errors, rel  # noqa: E402

NAMES = {"fb": "FB", "afb": "AFB"}
EB = np.array([1e-3, -2e-4, 3e-4, 1e-4, -1e-4, 5e-4])
LENGTHS = [48, 64, 96, 128, 192, 256]
K = 10


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2009_03762_amd import lsfft
    return lsfft


def _cell(shape, seed):
    n1, n2, n3 = shape
    lam, mu = inputs.random_moduli(shape, seed=seed, E_range=(1.0, 100.0))
    assert lam.shape == (n3, n2, n1)
    return lam, mu, 0.5 * (lam.min() + lam.max()), 0.5 * (mu.min() + mu.max())


def _tname(prec):
    return "float" if prec == "f32" else "double"


def _check(out, hist, ref, prec):
    f64 = prec == "f64"
    assert out["iters"] == K
    assert rel(out["eps"], ref.eps) < (1e-12 if f64 else 1e-5)
    assert rel(out["sig"], ref.sig) < (1e-12 if f64 else 1e-5)
    assert rel(out["sig_mean"], ref.sig_mean) < (1e-12 if f64 else 1e-6)
    assert rel(hist, np.array(ref.history)) < (1e-9 if f64 else 1e-3)
    for name, err in plane_errors(out["eps"], ref.eps).items():
        assert err < (1e-10 if f64 else 1e-4), name


@pytest.mark.parametrize("n", LENGTHS)
@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("scheme", ["afb", "fb"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_length_in_each_axis(L, n, axis, scheme, prec):
    shape = [8, 8, 8]
    shape[axis] = n
    shape = tuple(shape)
    lam, mu, l0, m0 = _cell(shape, seed=n + 7 * axis)
    s = L.Solver(lam, mu, l0, m0, scheme=scheme, prec=prec, form="displacement")
    kern = s.describe()
    print(f"\n[lengths] (n1,n2,n3)={shape} {scheme} {prec}: {kern}", flush=True)
    tn = _tname(prec)
    names = kern.split()
    assert names[0].startswith(f"k_stencil_reg<{tn},{shape[0]},")
    assert names[1].startswith(f"k_ypass<{tn},{shape[1]},")
    assert names[2].startswith(f"k_zpass_u<{tn},{shape[2]},") and names[2].endswith(f",{NAMES[scheme]}>")
    out = s.solve(EB, tol=0.0, maxit=K)
    hist = s.residual_history()
    s.close()
    ref = solve3d.solve_gfp(lam, mu, EB, l0, m0, scheme=NAMES[scheme], tol=0.0, maxit=K)
    _check(out, hist, ref, prec)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_benchmark_kernels_on_random_moduli(L, prec):
    """n1 = n3 = 256: exactly the stencil and z-pass instantiations the
    256^3 benchmark runs (same lengths, precision, scheme and tiles; the
    plane count per stencil workgroup only depends on n3), on non-laminate
    data whose spectrum fills every plane."""
    shape = (256, 16, 256)
    lam, mu, l0, m0 = _cell(shape, seed=256)
    s = L.Solver(lam, mu, l0, m0, scheme="afb", prec=prec, form="displacement")
    kern = s.describe()
    print(f"\n[lengths 256] {shape} {prec}: {kern}", flush=True)
    tn = _tname(prec)
    names = kern.split()
    if prec == "f32":
        assert names[0] == "k_stencil_reg<float,256,4,AFB,2>"
    assert names[0].startswith(f"k_stencil_reg<{tn},256,")
    assert names[2].startswith(f"k_zpass_u<{tn},256,") and names[2].endswith(",AFB>")
    out = s.solve(EB, tol=0.0, maxit=K)
    hist = s.residual_history()
    s.close()
    ref = solve3d.solve_gfp(lam, mu, EB, l0, m0, scheme="AFB", tol=0.0, maxit=K)
    _check(out, hist, ref, prec)


@pytest.mark.parametrize("n1", [192, 384])
def test_f64_warm_start_wide_x(L, n1):
    """FP64 warm start where the FP64 stencil runs 192 threads (192 columns)
    and one owned node line per y-group (384)."""
    shape = (n1, 6, 4)
    warm = 3
    lam, mu, l0, m0 = _cell(shape, seed=n1)
    s = L.Solver(lam, mu, l0, m0, scheme="afb", prec="f32", form="displacement", f64_warmup=warm)
    print(f"\n[warm wide x] {shape}: {s.describe()}", flush=True)
    assert s.describe().split()[0].startswith(f"k_stencil_reg<float,{n1},")
    out = s.solve(EB, tol=0.0, maxit=K)
    hist = s.residual_history()
    s.close()
    ref = solve3d.solve_gfp(lam, mu, EB, l0, m0, scheme="AFB", tol=0.0, maxit=K)
    assert out["iters"] == K
    assert rel(hist[:warm], np.array(ref.history[:warm])) < 1e-9
    assert rel(out["eps"], ref.eps) < 1e-5


@pytest.mark.parametrize("n1", [192, 384, 512])
def test_refined_sweeps_wide_x(L, n1):
    """FP64 refinement cycles with the 192-, 384- and 512-column register
    stencils (refinement uses them for its F32 sweeps)."""
    shape = (n1, 12, 8)
    lam, mu = inputs.cubic_inclusion(shape, (n1 // 2, 6, 4), 1.0, 10.0)
    assert lam.shape[-1] == n1
    l0, m0 = inputs.reference_medium_mean(1.0, 10.0)
    s = L.Solver(lam, mu, l0, m0, scheme="afb", prec="f32", form="displacement", refine=4)
    print(f"\n[refine wide x] {shape}: {s.describe()}", flush=True)
    assert s.describe().split()[0].startswith(f"k_stencil_reg<float,{n1},")
    out = s.solve(EB, tol=0.0, maxit=K)
    hist = s.residual_history()
    s.close()
    ref = solve3d.solve_gfp(lam, mu, EB, l0, m0, scheme="AFB", tol=0.0, maxit=K)
    assert out["iters"] == K
    assert rel(out["eps"], ref.eps) < 1e-6
    assert rel(hist, np.array(ref.history)) < 1e-3
