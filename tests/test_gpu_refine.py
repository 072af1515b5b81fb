"""FP64 iterative refinement of the F32 displacement form (lsfft_config.refine)
against the FP64 oracle.

The fixed point keeps no memory beyond its iterate, so restarting it on the
correction of a folded displacement continues the same iteration: the refined
F32 solve must follow the oracle's iterates (fixed iteration counts, every
cycle length, anisotropic spacing, an eigenstrain, a batch, an FP64 warm
start) and, at contrast 10, reach tolerances far below the residual floor
of plain F32 in the oracle's iteration count, reporting a residual and mean
stress from an FP64 evaluation.  At contrast 1e2 and above the FP32 rounding
of the first, large updates lands in the slowest modes of the iteration
(contraction about (chi - 1)/(chi + 1) per iteration), which the FP64
residual sees but refinement cannot remove faster than the iteration does:
there the refined solve needs more iterations than FP64 (not asserted)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import green, solve3d  # noqa: E402
from paper_2009_03762_amd import inputs  # noqa: E402

from oracle_ref import rel  # noqa: E402

NAMES = {"fb": "FB", "afb": "AFB"}
EB = np.array([1e-3, -2e-4, 3e-4, 1e-4, -1e-4, 5e-4])


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2009_03762_amd import lsfft
    return lsfft


def _oracle_at(lam, mu, E, l0, m0, scheme, tol, k_stop, **kw):
    """One oracle run to k_stop + 2 iterations (tol = 0): the iteration count
    it needs for `tol` (None if not within), its history, and its iterate and
    mean stress at k_stop (Voigt, (6, n3, n2, n1) and (6,))."""
    got = {}

    def grab(k, eps, T, r):
        if k == k_stop:
            got["eps"] = np.moveaxis(green.to_voigt(eps), -1, 0)
            got["sig"] = np.moveaxis(green.to_voigt(T), -1, 0)
            got["sig_mean"] = green.to_voigt(T.mean(axis=(0, 1, 2)))

    ref = solve3d.solve_gfp(lam, mu, E, l0, m0, scheme=scheme, tol=0.0, maxit=k_stop + 2, callback=grab, **kw)
    hist = np.array(ref.history)
    below = np.nonzero(hist <= tol)[0]
    return (int(below[0]) if below.size else None), hist, got


def _inclusion(shape, side, chi):
    lam, mu = inputs.cubic_inclusion(shape, side, 1.0, chi)
    l0, m0 = inputs.reference_medium_mean(1.0, chi)
    return lam, mu, l0, m0


@pytest.mark.parametrize("scheme,n,cycle,slack", [("afb", 24, 8, 2), ("afb", 32, 8, 2), ("fb", 16, 16, 2),
                                                  ("afb", 24, 16, 4)])
def test_reaches_fp64_tolerance(L, scheme, n, cycle, slack):
    """Contrast 10, tol 1e-10 (orders below the F32 floor): stop in the
    oracle's iteration count (+-2) with the oracle's iterate, where plain F32
    does not converge in three times as many iterations.  AFB cycles longer
    than 8 iterations reach the tolerance too, but a cycle whose residual
    reduction exceeds about 1e-3 meets the F32 floor of the sweeps on delta
    (measured: 59 iterations against the oracle's 56 with cycles of 16 at
    24^3 and 32^3, 74 with cycles of 32; FB loses none)."""
    tol = 1e-10
    print(f"\n[refine tol] {scheme} n={n} cycle={cycle} tol={tol}", flush=True)
    lam, mu, l0, m0 = _inclusion((n, n, n), (n // 2,) * 3, 10.0)
    s = L.Solver(lam, mu, l0, m0, scheme=scheme, prec="f32", form="displacement", refine=cycle)
    out = s.solve(EB, tol=tol, maxit=5000)
    hist = s.residual_history()
    s.close()
    k = out["iters"]
    assert out["status"] == L.OK and out["residual"] <= tol
    k_ref, h_ref, it = _oracle_at(lam, mu, EB, l0, m0, NAMES[scheme], tol, k)
    assert k_ref is not None and abs(k - k_ref) <= slack
    # eps is stored in FP32: its rounding (6e-8) is the floor of the field bar
    assert rel(out["eps"], it["eps"]) < 1e-6
    assert rel(out["sig_mean"], it["sig_mean"]) < 1e-6
    # the reported residual is an FP64 evaluation of the final iterate, whose
    # FP32 rounding (relative to the residual of its cycle) it also sees
    if slack <= 2:
        assert abs(out["residual"] - h_ref[k]) <= 0.2 * h_ref[k]
    assert hist[-1] == out["residual"]
    plain = L.Solver(lam, mu, l0, m0, scheme=scheme, prec="f32", form="displacement")
    p = plain.solve(EB, tol=tol, maxit=3 * k, fields=False)
    plain.close()
    assert p["status"] == L.ENOTCONV and p["residual"] > 10 * tol


@pytest.mark.parametrize("cycle", [1, 7, 64])
@pytest.mark.parametrize("scheme", ["afb", "fb"])
def test_fixed_iterations_every_cycle_length(L, cycle, scheme):
    """Cycles of 1 and 7 iterations, and one longer than the solve (plain F32
    sweeps after one FP64 evaluation, confirmed at maxit)."""
    print(f"\n[refine cycle] {scheme} m={cycle}", flush=True)
    K = 20
    lam, mu, l0, m0 = _inclusion((16, 12, 24), (8, 6, 12), 1e3)
    s = L.Solver(lam, mu, l0, m0, scheme=scheme, prec="f32", form="displacement", refine=cycle)
    out = s.solve(EB, tol=0.0, maxit=K)
    hist = s.residual_history()
    s.close()
    ref = solve3d.solve_gfp(lam, mu, EB, l0, m0, scheme=NAMES[scheme], tol=0.0, maxit=K)
    h_ref = np.array(ref.history)
    assert out["status"] == L.ENOTCONV and out["iters"] == K and len(hist) == K + 1
    # FP32 rounding of the updates is white in u; its residual, relative to
    # the residual at the start of the cycle, grows like (n/2)^2 x 2^-24
    if cycle > K:
        assert rel(out["eps"], ref.eps) < 1e-5
        assert rel(out["sig_mean"], ref.sig_mean) < 1e-5
        assert rel(hist, h_ref) < 5e-2
    else:
        assert rel(out["sig_mean"], ref.sig_mean) < 1e-6
        assert rel(out["eps"], ref.eps) < 1e-6
        assert rel(hist, h_ref) < 1e-3
        assert abs(hist[-1] - h_ref[-1]) <= 1e-3 * h_ref[-1]


@pytest.mark.parametrize("shape,scheme,eig", [((4, 8, 8), "afb", False), ((6, 12, 8), "fb", False),
                                              ((6, 8, 12), "afb", True)])
def test_cell_kernel_evaluation(L, shape, scheme, eig):
    """x-lines of 4 and 6 points, where the FP64 register stencil does not run
    and each cycle's FP64 residual comes from the cell-stress and divergence
    kernels instead: converged refined solves against the oracle."""
    print(f"\n[refine cell kernels] {shape} {scheme} eig={eig}", flush=True)
    side = tuple(n // 2 if (n - n // 2) % 2 == 0 else n // 2 - 1 for n in shape)  # centred cubes
    lam, mu, l0, m0 = _inclusion(shape, side, 10.0)
    es = 1e-3 * np.random.default_rng(5).standard_normal((6,) + lam.shape) if eig else None
    s = L.Solver(lam, mu, l0, m0, scheme=scheme, prec="f32", form="displacement", refine=8, eigenstrain=es)
    assert s.describe().split()[0].startswith("k_stencil<float")
    out = s.solve(EB, tol=1e-10, maxit=2000)
    s.close()
    ref = solve3d.solve_gfp(lam, mu, EB, l0, m0, scheme=scheme.upper(), tol=1e-10, maxit=2000, eigenstrain=es)
    assert out["status"] == L.OK and abs(out["iters"] - ref.iters) <= 1
    assert rel(out["eps"], ref.eps) < 1e-6
    assert rel(out["sig_mean"], ref.sig_mean) < 1e-6


def test_fp32_floor_status(L):
    """The F32 displacement form's residual floor (about (n/2)^2 x 2^-24, 6e-5
    at 64^3, contrast 1e3): a tolerance below it ends ENOTCONV after maxit
    with the fields at FP64 accuracy, one above it stops OK, and f64_until
    with refinement certifies the tolerance below it."""
    print("\n[floor status]", flush=True)
    lam, mu, l0, m0 = _inclusion((64, 64, 64), (32, 32, 32), 1e3)
    s = L.Solver(lam, mu, l0, m0, scheme="afb", prec="f32", f64_warmup=5)
    lo = s.solve(EB, tol=1e-7, maxit=400)
    hi = s.solve(EB, tol=1e-3, maxit=400)
    s.close()
    s = L.Solver(lam, mu, l0, m0, scheme="afb", prec="f64")
    ref = s.solve(EB, tol=1e-10, maxit=3000)
    s.close()
    s = L.Solver(lam, mu, l0, m0, scheme="afb", prec="f32", f64_until=3e-5, refine=8)
    cert = s.solve(EB, tol=1e-7, maxit=3000)
    s.close()
    assert lo["status"] == L.ENOTCONV and lo["iters"] == 400 and lo["residual"] > 1e-7
    assert rel(lo["eps"], ref["eps"]) < 1e-5
    assert hi["status"] == L.OK and hi["residual"] <= 1e-3
    assert cert["status"] == L.OK and cert["residual"] <= 1e-7
    assert rel(cert["eps"], ref["eps"]) < 1e-5


def test_anisotropic_spacing(L):
    print("\n[refine spacing]", flush=True)
    h = (0.5, 1.0, 2.0)
    lam, mu, l0, m0 = _inclusion((16, 12, 8), (8, 6, 4), 10.0)
    s = L.Solver(lam, mu, l0, m0, scheme="afb", prec="f32", form="displacement", refine=5, h=h)
    out = s.solve(EB, tol=1e-10, maxit=2000)
    s.close()
    ref = solve3d.solve_gfp(lam, mu, EB, l0, m0, scheme="AFB", tol=1e-10, maxit=2000, h=h)
    assert out["status"] == L.OK and abs(out["iters"] - ref.iters) <= 1
    assert rel(out["eps"], ref.eps) < 1e-6


@pytest.mark.parametrize("scheme", ["afb", "fb"])
def test_eigenstrain(L, scheme):
    print(f"\n[refine eigenstrain] {scheme}", flush=True)
    lam, mu, l0, m0 = _inclusion((16, 16, 16), (8, 8, 8), 10.0)
    es = 1e-3 * np.random.default_rng(11).standard_normal((6,) + lam.shape)
    s = L.Solver(lam, mu, l0, m0, scheme=scheme, prec="f32", form="displacement", refine=16, eigenstrain=es)
    out = s.solve(EB, tol=1e-10, maxit=5000)
    s.close()
    k = out["iters"]
    assert out["status"] == L.OK
    k_ref, _, it = _oracle_at(lam, mu, EB, l0, m0, NAMES[scheme], 1e-10, k, eigenstrain=es)
    assert k_ref is not None and abs(k - k_ref) <= 2
    assert rel(out["eps"], it["eps"]) < 1e-6
    assert rel(out["sig"], it["sig"]) < 1e-6


def test_batch_stops_each_system_on_its_own(L):
    """Three load cases of one cell and a zero load: each stops on its own
    FP64-confirmed test, at the oracle's iteration count."""
    print("\n[refine batch]", flush=True)
    lam, mu, l0, m0 = _inclusion((16, 16, 16), (8, 8, 8), 10.0)
    loads = [EB, np.array([0, 0, 0, 0, 0, 1e-3]), np.zeros(6), np.array([2e-3, 0, 0, 0, 0, 0])]
    h = L.create_batch([(lam, mu, l0, m0)] * len(loads), scheme="afb", prec="f32", form="displacement", refine=12)
    try:
        dev = torch.zeros((len(loads), 6) + lam.shape, dtype=torch.float32, device="cuda")
        st, sm, it, r, bst = L.solve_batch(h, np.stack(loads), 1e-10, 5000, eps_dev=dev)
        torch.cuda.synchronize()
        eps = dev.cpu().double().numpy()
    finally:
        L.destroy(h)
    for b, E in enumerate(loads):
        if not np.any(E):
            assert it[b] == 0 and bst[b] == L.OK and np.abs(eps[b]).max() == 0.0
            continue
        assert bst[b] == L.OK and r[b] <= 1e-10
        k_ref, _, got = _oracle_at(lam, mu, E, l0, m0, "AFB", 1e-10, int(it[b]))
        assert k_ref is not None and abs(int(it[b]) - k_ref) <= 2
        assert rel(eps[b], got["eps"]) < 1e-6
        assert rel(sm[b], got["sig_mean"]) < 1e-6


def test_with_f64_warm_start(L):
    print("\n[refine + warm start]", flush=True)
    lam, mu, l0, m0 = _inclusion((16, 16, 16), (8, 8, 8), 10.0)
    s = L.Solver(lam, mu, l0, m0, scheme="afb", prec="f32", form="displacement", refine=8, f64_warmup=5)
    out = s.solve(EB, tol=1e-10, maxit=5000)
    hist = s.residual_history()
    s.close()
    k = out["iters"]
    assert out["status"] == L.OK
    k_ref, h_ref, it = _oracle_at(lam, mu, EB, l0, m0, "AFB", 1e-10, k)
    assert k_ref is not None and abs(k - k_ref) <= 2
    assert rel(hist[:5], h_ref[:5]) < 1e-9
    assert rel(out["eps"], it["eps"]) < 1e-6


def test_degenerate_cases(L):
    print("\n[refine degenerate]", flush=True)
    lam, mu, l0, m0 = _inclusion((16, 8, 12), (8, 4, 6), 10.0)
    s = L.Solver(lam, mu, l0, m0, scheme="afb", prec="f32", form="displacement", refine=4)
    z = s.solve(np.zeros(6), tol=1e-12, maxit=50)
    assert z["status"] == L.OK and z["iters"] == 0 and np.abs(z["eps"]).max() == 0.0
    m = s.solve(EB, tol=1e-12, maxit=0)
    ref = solve3d.solve_gfp(lam, mu, EB, l0, m0, scheme="AFB", tol=1e-12, maxit=0)
    assert m["status"] == L.ENOTCONV and m["iters"] == 0
    # the first residual comes from the FP64 evaluation
    assert abs(m["residual"] - ref.residual) <= 1e-6 * ref.residual
    f = s.solve(EB, tol=2.0 * ref.residual, maxit=50)
    assert f["status"] == L.OK and f["iters"] == 0
    s.close()


def test_f64_ignores_refine_and_strain_form_rejects_it(L):
    lam, mu, l0, m0 = _inclusion((8, 8, 8), (4, 4, 4), 10.0)
    a = L.Solver(lam, mu, l0, m0, scheme="afb", prec="f64", refine=8)
    b = L.Solver(lam, mu, l0, m0, scheme="afb", prec="f64")
    oa, ob = a.solve(EB, tol=0.0, maxit=6), b.solve(EB, tol=0.0, maxit=6)
    a.close()
    b.close()
    assert np.array_equal(oa["eps"], ob["eps"])
    for kw in (dict(scheme="afb", form="strain"), dict(scheme="basic"), dict(scheme="cd")):
        with pytest.raises(L.LsfftError) as e:
            L.create(lam, mu, l0, m0, prec="f32", refine=8, **kw)
        assert e.value.status == L.EINVAL


def test_tuned_schedule_keeps_the_refined_solve(L):
    """The schedule tuner times the refined sweeps of the handle; the solve
    after tuning stops at the same iteration with the same fields (only the
    order of FP64 partial sums may change)."""
    print("\n[refine + autotune]", flush=True)
    lam, mu, l0, m0 = _inclusion((16, 16, 32), (8, 8, 16), 10.0)
    s = L.Solver(lam, mu, l0, m0, scheme="afb", prec="f32", form="displacement", refine=8)
    a = s.solve(EB, tol=1e-10, maxit=2000)
    sch, _, _ = L.autotune(s.handle, 8)
    b = s.solve(EB, tol=1e-10, maxit=2000)
    s.close()
    assert a["status"] == b["status"] == L.OK
    assert abs(a["iters"] - b["iters"]) <= 1
    assert rel(b["eps"], a["eps"]) < 1e-6
    assert set(sch) == {"stencil_planes", "y_cols", "z_cols", "xcd_order"}


def test_batch_mixing_eigenstrain(L):
    """A refined batch in which one system has an eigenstrain and one has
    none: each follows its own oracle solve."""
    print("\n[refine batch eigenstrain]", flush=True)
    lam, mu, l0, m0 = _inclusion((12, 16, 16), (6, 8, 8), 10.0)
    es = 1e-3 * np.random.default_rng(21).standard_normal((6,) + lam.shape)
    h = L.create_batch([(lam, mu, l0, m0, es), (lam, mu, l0, m0)], scheme="afb", prec="f32", form="displacement",
                       refine=8)
    try:
        dev = torch.zeros((2, 6) + lam.shape, dtype=torch.float32, device="cuda")
        st, sm, it, r, bst = L.solve_batch(h, np.stack([EB, 2 * EB]), 1e-9, 3000, eps_dev=dev)
        torch.cuda.synchronize()
        eps = dev.cpu().double().numpy()
    finally:
        L.destroy(h)
    for b, (E, e_star) in enumerate(((EB, es), (2 * EB, None))):
        assert bst[b] == L.OK and r[b] <= 1e-9
        k_ref, _, got = _oracle_at(lam, mu, E, l0, m0, "AFB", 1e-9, int(it[b]), eigenstrain=e_star)
        assert k_ref is not None and abs(int(it[b]) - k_ref) <= 2
        assert rel(eps[b], got["eps"]) < 1e-6
        assert rel(sm[b], got["sig_mean"]) < 1e-6


@pytest.mark.parametrize("scheme", ["afb", "fb"])
def test_f64_until_certifies_tolerance_at_high_contrast(L, scheme):
    """Contrast 1e3, tol 1e-7: FP64 iterations until r <= 300 tol (the same
    residuals as the oracle's), then refined F32 cycles of 8 whose stop is an
    FP64 evaluation; the solve stops OK at r <= tol within 3 iterations of the
    oracle's count, with the oracle's iterate."""
    tol = 1e-7
    print(f"\n[f64_until] {scheme} tol={tol}", flush=True)
    lam, mu, l0, m0 = _inclusion((24, 24, 24), (12, 12, 12), 1e3)
    s = L.Solver(lam, mu, l0, m0, scheme=scheme, prec="f32", form="displacement", refine=8, f64_until=300 * tol)
    out = s.solve(EB, tol=tol, maxit=5000)
    hist = s.residual_history()
    s.close()
    k = out["iters"]
    assert out["status"] == L.OK and out["residual"] <= tol
    k_ref, h_ref, it = _oracle_at(lam, mu, EB, l0, m0, NAMES[scheme], tol, k)
    assert k_ref is not None and abs(k - k_ref) <= 3
    # the FP64 phase: the oracle's residuals until the switch
    ksw = int(np.nonzero(h_ref <= 300 * tol)[0][0])
    assert rel(hist[:ksw + 1], h_ref[:ksw + 1]) < 1e-9
    assert rel(out["eps"], it["eps"]) < 1e-6
    assert rel(out["sig_mean"], it["sig_mean"]) < 1e-6


def test_f64_until_batch_switches_each_system_on_its_own(L):
    """Four load cases of one cell, contrast 1e2: each system leaves its FP64
    phase at its own iteration and stops on its own FP64-confirmed test; a
    zero load stops at once."""
    print("\n[f64_until batch]", flush=True)
    tol = 1e-8
    lam, mu, l0, m0 = _inclusion((16, 16, 16), (8, 8, 8), 1e2)
    loads = [EB, np.array([0, 0, 0, 0, 0, 1e-3]), np.zeros(6), np.array([2e-3, 0, 0, 0, 0, 0])]
    h = L.create_batch([(lam, mu, l0, m0)] * len(loads), scheme="afb", prec="f32", form="displacement", refine=8,
                       f64_until=300 * tol)
    try:
        dev = torch.zeros((len(loads), 6) + lam.shape, dtype=torch.float32, device="cuda")
        st, sm, it, r, bst = L.solve_batch(h, np.stack(loads), tol, 5000, eps_dev=dev)
        torch.cuda.synchronize()
        eps = dev.cpu().double().numpy()
    finally:
        L.destroy(h)
    for b, E in enumerate(loads):
        if not np.any(E):
            assert it[b] == 0 and bst[b] == L.OK and np.abs(eps[b]).max() == 0.0
            continue
        assert bst[b] == L.OK and r[b] <= tol
        k_ref, _, got = _oracle_at(lam, mu, E, l0, m0, "AFB", tol, int(it[b]))
        assert k_ref is not None and abs(int(it[b]) - k_ref) <= 3
        assert rel(eps[b], got["eps"]) < 1e-6
        assert rel(sm[b], got["sig_mean"]) < 1e-6


def test_f64_until_edge_cases(L):
    """A switch level above r_0 (no FP64 iteration is needed: the F32 phase
    starts at k = 0), a switch level below tol (the solve stays in FP64
    throughout and matches F64), together with f64_warmup (at least that
    many FP64 iterations), and invalid levels."""
    print("\n[f64_until edges]", flush=True)
    lam, mu, l0, m0 = _inclusion((16, 12, 8), (8, 6, 4), 10.0)
    ref = solve3d.solve_gfp(lam, mu, EB, l0, m0, scheme="AFB", tol=1e-9, maxit=2000)
    a = L.Solver(lam, mu, l0, m0, scheme="afb", prec="f32", form="displacement", refine=8, f64_until=1e3)
    oa = a.solve(EB, tol=1e-9, maxit=2000)
    a.close()
    assert oa["status"] == L.OK and abs(oa["iters"] - ref.iters) <= 2 and rel(oa["eps"], ref.eps) < 1e-6
    b = L.Solver(lam, mu, l0, m0, scheme="afb", prec="f32", form="displacement", f64_until=1e-12)
    ob = b.solve(EB, tol=1e-9, maxit=2000)
    hb = b.residual_history()
    b.close()
    assert ob["status"] == L.OK and ob["iters"] == ref.iters
    assert rel(hb, np.array(ref.history)) < 1e-9
    c = L.Solver(lam, mu, l0, m0, scheme="afb", prec="f32", form="displacement", refine=8, f64_warmup=20,
                 f64_until=1e3)
    oc = c.solve(EB, tol=1e-9, maxit=2000)
    hc = c.residual_history()
    c.close()
    assert oc["status"] == L.OK and rel(hc[:20], np.array(ref.history[:20])) < 1e-9
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(L.LsfftError) as e:
            L.create(lam, mu, l0, m0, scheme="afb", prec="f32", form="displacement", f64_until=bad)
        assert e.value.status == L.EINVAL
