"""Grid lengths with a factor 9 (the even 2^a 3^b that are not 2^a or 3 * 2^a)
in every axis position, against the oracle at fixed iteration counts
(Sec. 5.2, Alg. T3; the displacement form's stencils of Sec. 5.3, eq. (43);
the strain form's Green operators of Sec. 5.1 and the DGO of Sec. 5.4).

Shapes are written (n1, n2, n3), n1 the fastest axis.  On these x lengths a
line of the real x transform takes L / E threads (L = n1 / 2), a count that
need not divide a wavefront: the kernels pack whole lines into each
wavefront and leave the remaining lanes idle, so these cases check that
packing (and the ragged last workgroup of lines) as much as the radix-3
passes.  The displacement form runs the register stencil on every one of
these x lengths; the kernel names confirm it."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import green, solve3d  # noqa: E402
from paper_2009_03762_amd import inputs  # noqa: E402

from oracle_ref import plane_errors, rel  # noqa: E402

NAMES = {"basic": "basic", "fb": "FB", "afb": "AFB", "cd": "CD", "acd": "ACD"}
EB = np.array([1e-3, -2e-4, 3e-4, 1e-4, -1e-4, 5e-4])
LENGTHS = [18, 36, 54, 108, 144, 162, 216, 288, 324, 432, 486]
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
@pytest.mark.parametrize("scheme,prec", [("afb", "f64"), ("afb", "f32"), ("fb", "f64")])
def test_length9_in_each_axis(L, n, axis, scheme, prec):
    shape = [8, 6, 4]
    shape[axis] = n
    shape = tuple(shape)
    lam, mu, l0, m0 = _cell(shape, seed=3 * n + axis)
    s = L.Solver(lam, mu, l0, m0, scheme=scheme, prec=prec)
    kern = s.describe()
    print(f"\n[lengths9] (n1,n2,n3)={shape} {scheme} {prec}: {kern}", flush=True)
    tn = "float" if prec == "f32" else "double"
    names = kern.split()
    stencil = "k_stencil" if shape[0] < 8 else "k_stencil_reg"
    assert names[0].startswith(f"{stencil}<{tn},{shape[0]},")
    assert names[1].startswith(f"k_ypass<{tn},{shape[1]},")
    assert names[2].startswith(f"k_zpass_u<{tn},{shape[2]},")
    out = s.solve(EB, tol=0.0, maxit=K)
    hist = s.residual_history()
    s.close()
    ref = solve3d.solve_gfp(lam, mu, EB, l0, m0, scheme=NAMES[scheme], tol=0.0, maxit=K)
    _check(out, hist, ref, prec)


@pytest.mark.parametrize("n1,prec", [(18, "f32"), (162, "f32"), (486, "f32"), (486, "f64")])
def test_register_stencil_rounds(L, n1, prec):
    """Workgroups that are not whole wavefronts (162 threads), two rounds of
    line transforms per plane (18 columns: 14 y-groups, 84 lines of 3
    threads; 162 columns: lines of 27 threads, two to a wavefront) and the
    widest rows (486): the register stencil against the oracle."""
    shape = (n1, 6, 4)
    lam, mu, l0, m0 = _cell(shape, seed=n1 + 1)
    s = L.Solver(lam, mu, l0, m0, scheme="afb", prec=prec, form="displacement")
    tn = "float" if prec == "f32" else "double"
    print(f"\n[lengths9 rounds] {shape} {prec}: {s.describe()}", flush=True)
    assert s.describe().split()[0].startswith(f"k_stencil_reg<{tn},{n1},")
    out = s.solve(EB, tol=0.0, maxit=K)
    hist = s.residual_history()
    s.close()
    ref = solve3d.solve_gfp(lam, mu, EB, l0, m0, scheme="AFB", tol=0.0, maxit=K)
    _check(out, hist, ref, prec)


@pytest.mark.parametrize("scheme", ["basic", "cd", "acd", "afb"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_strain_form_schemes(L, scheme, prec):
    """The strain form of every Green operator on a cell with a factor 9 or
    27 in each axis (x-pass lines of 3 threads, 21 to a wavefront)."""
    shape = (36, 18, 54)
    lam, mu, l0, m0 = _cell(shape, seed=11)
    s = L.Solver(lam, mu, l0, m0, scheme=scheme, prec=prec, form="strain")
    print(f"\n[lengths9 strain] {shape} {scheme} {prec}: {s.describe()}", flush=True)
    out = s.solve(EB, tol=0.0, maxit=K)
    hist = s.residual_history()
    s.close()
    ref = solve3d.solve_gfp(lam, mu, EB, l0, m0, scheme=NAMES[scheme], tol=0.0, maxit=K)
    _check(out, hist, ref, prec)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_dgo_length9(L, prec):
    shape = (18, 12, 36)
    M = 2
    lam, mu, l0, m0 = _cell(shape, seed=5)
    s = L.Solver(lam, mu, l0, m0, scheme="dgo", disc="pcd", prec=prec, dgo_images=M, dgo_weight_power=1)
    out = s.solve(EB, tol=0.0, maxit=K)
    s.close()
    Gc = green.dgo_voigt(shape, l0, m0, M, 1)
    ref = solve3d.solve_dgo(lam, mu, EB, l0, m0, Gc, tol=0.0, maxit=K)
    tol = 1e-12 if prec == "f64" else 1e-5
    assert out["iters"] == K
    assert rel(out["eps"], ref.eps) < tol
    assert rel(out["sig"], ref.sig) < tol


def test_converged_fp64_length9(L):
    """Converged AFB solve on a 36 x 18 x 72 cubic inclusion: the oracle's
    iteration count and solution."""
    shape = (36, 18, 72)
    lam, mu = inputs.cubic_inclusion(shape, (18, 8, 36), 1.0, 10.0)
    assert lam.shape == (72, 18, 36)
    l0, m0 = inputs.reference_medium_mean(1.0, 10.0)
    Eb = inputs.macro_strain("12", 1e-3)
    s = L.Solver(lam, mu, l0, m0, scheme="afb", prec="f64")
    out = s.solve(Eb, tol=1e-8, maxit=2000)
    s.close()
    ref = solve3d.solve_gfp(lam, mu, Eb, l0, m0, scheme="AFB", tol=1e-8, maxit=2000)
    assert out["status"] == L.OK and ref.status == solve3d.OK
    assert out["iters"] == ref.iters
    assert rel(out["eps"], ref.eps) < 1e-11
    assert rel(out["sig_mean"], ref.sig_mean) < 1e-11


@pytest.mark.parametrize("n1", [72, 18, 162])
@pytest.mark.parametrize("opt", ["warm", "refine"])
def test_f32_options_length9(L, opt, n1):
    """FP64 warm start and FP64 refinement on x lengths with a factor 9 (at
    18 and 162 columns the register stencils, the refinement's prescribed-
    force instantiation and its FP64 real-space evaluation included, run
    their line transforms in two rounds)."""
    shape = (n1, 12, 18)
    lam, mu, l0, m0 = _cell(shape, seed=n1)
    kw = {"f64_warmup": 3} if opt == "warm" else {"refine": 4}
    s = L.Solver(lam, mu, l0, m0, scheme="afb", prec="f32", form="displacement", **kw)
    print(f"\n[lengths9 {opt}] {shape}: {s.describe()}", flush=True)
    out = s.solve(EB, tol=0.0, maxit=K)
    hist = s.residual_history()
    s.close()
    ref = solve3d.solve_gfp(lam, mu, EB, l0, m0, scheme="AFB", tol=0.0, maxit=K)
    assert out["iters"] == K
    assert rel(out["eps"], ref.eps) < (1e-5 if opt == "warm" else 1e-6)
    if opt == "warm":
        assert rel(hist[:3], np.array(ref.history[:3])) < 1e-9
    else:
        assert rel(hist, np.array(ref.history)) < 1e-3


def _probe(L, h, n3):
    """Each knob's values the handle accepts (the default and its doubled or
    halved tiles, the even plane counts dividing n3)."""
    d = L.get_schedule(h)
    out = {}
    for key in ("y_cols", "z_cols"):
        vals = [d[key]]
        for c in (d[key] // 2, d[key] * 2):
            try:
                L.set_schedule(h, dict(d, **{key: c}))
                vals.append(c)
            except L.LsfftError as e:
                assert e.status == L.EINVAL
        out[key] = vals
    out["stencil_planes"] = [z for z in (2, 6, 18) if n3 % z == 0] if d["stencil_planes"] else [0]
    L.set_schedule(h, d)
    return d, out


@pytest.mark.parametrize("form,prec", [("displacement", "f32"), ("displacement", "f64"), ("strain", "f64")])
def test_offered_schedules_length9(L, form, prec):
    """Every offered tile of the y and z passes (many of them workgroups that
    are not whole wavefronts on these lengths, whose block sums feed the
    residual) and plane count gives the iterates of the default schedule."""
    shape = (36, 18, 54)
    lam, mu, l0, m0 = _cell(shape, seed=36)
    s = L.Solver(lam, mu, l0, m0, scheme="afb", prec=prec, form=form)
    d, offered = _probe(L, s.handle, shape[2])
    print(f"\n[lengths9 schedule] {form} {prec} default {d} offered {offered}", flush=True)
    assert len(offered["z_cols"]) == 2  # 28 and 56 (FP32) or 14 (FP64) columns of 9 threads
    ref = s.solve(EB, tol=0.0, maxit=K)
    hist_ref = s.residual_history()
    tol = 1e-13 if prec == "f64" else 2e-6
    for z in offered["stencil_planes"]:
        for y in offered["y_cols"]:
            for zc in offered["z_cols"]:
                for x in (0, 7):
                    sch = {"stencil_planes": z, "y_cols": y, "z_cols": zc, "xcd_order": x}
                    L.set_schedule(s.handle, sch)
                    out = s.solve(EB, tol=0.0, maxit=K)
                    assert rel(out["eps"], ref["eps"]) < tol, sch
                    assert rel(s.residual_history(), hist_ref) < (1e-9 if prec == "f64" else 1e-5), sch
    s.close()
    oref = solve3d.solve_gfp(lam, mu, EB, l0, m0, scheme="AFB", tol=0.0, maxit=K)
    assert rel(ref["eps"], oref.eps) < (1e-12 if prec == "f64" else 1e-5)


def test_batch_and_group_length9(L):
    """Two cells of different sizes with factor-9 lengths, two loads each:
    one group graph gives each batch's own iterates bit for bit, and both
    match the oracle."""
    loads = np.array([[1e-3, 0, 0, 0, 0, 0], [0, 0, 0, 0, 0, 1e-3]])
    cells = [_cell((18, 18, 18), seed=18), _cell((36, 18, 54), seed=54)]
    shapes = [(18, 18, 18), (36, 18, 54)]
    hs = [L.create_batch([c, c], scheme="afb", prec="f64") for c in cells]
    try:
        devs = [torch.zeros((2, 6) + sh[::-1], dtype=torch.float64, device="cuda") for sh in shapes]
        st, res = L.solve_group(hs, [loads, loads], 0.0, K, eps_devs=devs)
        torch.cuda.synchronize()
        eps = [d.cpu().numpy() for d in devs]
        each = []
        for h, sh in zip(hs, shapes):
            d1 = torch.zeros((2, 6) + sh[::-1], dtype=torch.float64, device="cuda")
            L.solve_batch(h, loads, 0.0, K, eps_dev=d1)
            torch.cuda.synchronize()
            each.append(d1.cpu().numpy())
    finally:
        for h in hs:
            L.destroy(h)
    for (lam, mu, l0, m0), e, e1 in zip(cells, eps, each):
        assert np.array_equal(e, e1)
        for b in range(2):
            ref = solve3d.solve_gfp(lam, mu, loads[b], l0, m0, scheme="AFB", tol=0.0, maxit=K)
            assert rel(e[b], ref.eps) < 1e-12


@pytest.mark.parametrize("n1,scheme,prec", [(18, "afb", "f32"), (54, "afb", "f64"), (162, "fb", "f64")])
def test_eigenstrain_length9(L, n1, scheme, prec):
    """An eigenstrain (Sec. 7) through the register stencil's prescribed-force
    instantiation where its line transforms take two rounds per plane."""
    shape = (n1, 6, 4)
    lam, mu, l0, m0 = _cell(shape, seed=n1 + 2)
    es = 1e-3 * np.random.default_rng(n1).standard_normal((6,) + lam.shape)
    s = L.Solver(lam, mu, l0, m0, scheme=scheme, prec=prec, form="displacement", eigenstrain=es)
    print(f"\n[lengths9 eig] {shape} {scheme} {prec}: {s.describe()}", flush=True)
    out = s.solve(EB, tol=0.0, maxit=K)
    hist = s.residual_history()
    s.close()
    ref = solve3d.solve_gfp(lam, mu, EB, l0, m0, scheme=NAMES[scheme], tol=0.0, maxit=K, eigenstrain=es)
    _check(out, hist, ref, prec)
