"""Batched solves (lsfft_create_batch / lsfft_solve_batch): several systems on
one grid solved by the same kernel launches.  Checked against one-system
solves of the same library and against the oracle; systems stop on their own
tests."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import solve3d  # noqa: E402
from paper_2009_03762_amd import inputs  # noqa: E402

from oracle_ref import rel  # noqa: E402


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2009_03762_amd import lsfft
    return lsfft


def _dt(prec):
    return torch.float64 if prec == "f64" else torch.float32


def _cells(shape, contrasts):
    out = []
    for chi in contrasts:
        lam, mu = inputs.cubic_inclusion(shape, tuple(v // 2 for v in shape), 1.0, chi)
        l0, m0 = inputs.reference_medium_mean(1.0, chi)
        out.append((lam, mu, l0, m0))
    return out


def _batch_solve(L, systems, Ebs, prec, tol, maxit, **kw):
    h = L.create_batch(systems, prec=prec, **kw)
    shape = systems[0][0].shape
    B = len(systems)
    eps = torch.zeros((B, 6) + shape, dtype=_dt(prec), device="cuda")
    sig = torch.zeros_like(eps)
    st, sm, it, r, sts = L.solve_batch(h, Ebs, tol, maxit, eps, sig)
    L.destroy(h)
    return st, sm, it, r, sts, eps.cpu().double().numpy(), sig.cpu().double().numpy()


@pytest.mark.parametrize("scheme,form", [("afb", "displacement"), ("fb", "displacement"), ("afb", "strain"),
                                         ("basic", "auto")])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_cells_batch_matches_single_solves(L, scheme, form, prec):
    """Three cells of different contrast (different moduli and C0), fixed iterations."""
    print(f"\n[batch cells] {scheme} {form} {prec}", flush=True)
    shape = (16, 12, 8)
    systems = _cells(shape, (3.0, 10.0, 30.0))
    Ebs = np.array([[1e-3, 0, 0, 0, 0, 0], [0, 0, 0, 0, 0, 2e-3], [1e-3, -5e-4, 2e-4, 1e-4, 3e-4, -2e-4]])
    K = 10
    st, sm, it, r, sts, eps, sig = _batch_solve(L, systems, Ebs, prec, 0.0, K, scheme=scheme, form=form)
    tol = 1e-13 if prec == "f64" else 1e-6
    for b, (lam, mu, l0, m0) in enumerate(systems):
        s = L.Solver(lam, mu, l0, m0, scheme=scheme, prec=prec, form=form)
        one = s.solve(Ebs[b], tol=0.0, maxit=K)
        s.close()
        assert it[b] == K and sts[b] == L.ENOTCONV
        assert rel(eps[b], one["eps"]) < tol
        assert rel(sig[b], one["sig"]) < tol
        assert rel(sm[b], one["sig_mean"]) < tol
        assert abs(r[b] - one["residual"]) <= 1e-9 * one["residual"]
    # and against the oracle (different formulation of the same iteration)
    lam, mu, l0, m0 = systems[1]
    ref = solve3d.solve_gfp(lam, mu, Ebs[1], l0, m0, scheme={"basic": "basic", "fb": "FB", "afb": "AFB"}[scheme],
                            tol=0.0, maxit=K)
    assert rel(eps[1], ref.eps) < (1e-12 if prec == "f64" else 1e-5)


def test_systems_stop_independently(L):
    """A homogeneous cell (exact at the first pass) beside an inclusion cell:
    the first stops at iteration 0, the second converges later, and both
    results are those of one-system solves."""
    shape = (16, 16, 16)
    (lam, mu, l0, m0), = _cells(shape, (10.0,))
    hom = (np.full(lam.shape, 2.0), np.full(lam.shape, 1.5), 1.0, 1.0)
    systems = [hom, (lam, mu, l0, m0), hom]
    Ebs = np.array([[1e-3, 0, 0, 0, 0, 2e-4], [1e-3, 0, 0, 0, 0, 0], [0, 0, 1e-3, 0, 0, 0]])
    st, sm, it, r, sts, eps, sig = _batch_solve(L, systems, Ebs, "f64", 1e-9, 500, scheme="afb")
    assert st == L.OK and list(sts) == [L.OK] * 3
    assert it[0] == 0 and it[2] == 0 and it[1] > 10
    for b in (0, 2):
        assert np.allclose(eps[b], Ebs[b][:, None, None, None], atol=1e-18)
    s = L.Solver(lam, mu, l0, m0, scheme="afb", prec="f64")
    one = s.solve(Ebs[1], tol=1e-9, maxit=500)
    s.close()
    assert one["iters"] == it[1]
    assert rel(eps[1], one["eps"]) < 1e-13


@pytest.mark.parametrize("prec,warm", [("f64", 0), ("f32", 0), ("f32", 3)])
def test_effective_stiffness_in_one_batch(L, prec, warm):
    """The six Mandel unit loads of one cell as one batch -> C_eff against the oracle."""
    n = 16
    lam, mu = inputs.cubic_inclusion(n, n // 2, 1.0, 10.0, interface="smooth")
    l0, m0 = inputs.reference_medium_mean(1.0, 10.0)
    units = inputs.mandel_unit_strains()
    ref = solve3d.effective_stiffness(
        lambda E: solve3d.solve_gfp(lam, mu, E, l0, m0, scheme="AFB", tol=1e-12, maxit=5000), units)
    h = L.create_batch([(lam, mu, l0, m0)] * 6, scheme="afb", prec=prec, f64_warmup=warm)
    st, sm, it, r, sts = L.solve_batch(h, units, 1e-12 if prec == "f64" else 1e-7, 5000)
    L.destroy(h)
    got = np.stack([solve3d.mandel(sm[J]) for J in range(6)], axis=1)
    assert rel(got, ref) < (1e-11 if prec == "f64" else 1e-6)


def test_dgo_batch_matches_single(L):
    shape = (8, 8, 8)
    lam, mu = inputs.cubic_inclusion(8, 4, 1.0, 5.0)
    l0, m0 = inputs.reference_medium_mean(1.0, 5.0)
    lam2 = lam * 1.3
    mu2 = mu * 1.3
    systems = [(lam, mu, l0, m0), (lam2, mu2, l0, m0)]
    Ebs = np.array([[0, 0, 0, 0, 0, 1e-3], [1e-3, 0, 0, 0, 0, 0]])
    st, sm, it, r, sts, eps, sig = _batch_solve(L, systems, Ebs, "f64", 0.0, 8, scheme="dgo", disc="pcd",
                                                dgo_images=2, dgo_weight_power=2)
    for b, (la, m_, a0, b0) in enumerate(systems):
        s = L.Solver(la, m_, a0, b0, scheme="dgo", disc="pcd", prec="f64", dgo_images=2, dgo_weight_power=2)
        one = s.solve(Ebs[b], tol=0.0, maxit=8)
        s.close()
        assert rel(eps[b], one["eps"]) < 1e-13


def test_single_entry_points_reject_batch_handles(L):
    (lam, mu, l0, m0), = _cells((8, 8, 8), (2.0,))
    h = L.create_batch([(lam, mu, l0, m0)] * 2, prec="f64")
    assert L.batch_size(h) == 2
    with pytest.raises(L.LsfftError) as e:
        L.solve(h, np.zeros(6), 1e-6, 5)
    assert e.value.status == L.EINVAL
    L.destroy(h)


@pytest.mark.parametrize("prec,form", [("f64", "displacement"), ("f32", "strain")])
def test_graph_replay_matches_eager(L, prec, form, monkeypatch):
    """Solves replaying captured iteration chunks give the same bits as eager
    launches, on repeated solves of one handle with other work in between."""
    shape = (16, 16, 16)
    systems = _cells(shape, (10.0, 30.0))
    Ebs = np.array([[1e-3, 0, 0, 0, 0, 0], [0, 0, 0, 0, 0, 1e-3]])
    res = {}
    for mode in ("graphs", "eager"):
        if mode == "eager":
            monkeypatch.setenv("LSFFT_NO_GRAPHS", "1")
        else:
            monkeypatch.delenv("LSFFT_NO_GRAPHS", raising=False)
        h = L.create_batch(systems, scheme="afb", prec=prec, form=form)
        outs = []
        for rep in range(3):
            eps = torch.zeros((2, 6) + shape, dtype=_dt(prec), device="cuda")
            tol = 1e-9 if rep != 1 else 0.0
            st, sm, it, r, sts = L.solve_batch(h, Ebs * (1 + rep), tol, 60 + 5 * rep, eps)
            torch.cuda.synchronize()
            junk = torch.randn(1 << 20, device="cuda").sum().item()  # eager work between replays
            outs.append((it.copy(), sm.copy(), eps.cpu().numpy()))
        L.destroy(h)
        res[mode] = outs
    for (ia, sa_, ea), (ib, sb, eb) in zip(res["graphs"], res["eager"]):
        assert np.array_equal(ia, ib)
        assert np.array_equal(sa_, sb)
        assert np.array_equal(ea, eb)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_handles_on_streams_solve_concurrently(L, prec):
    """Separate handles, each on its own stream, solved at the same time from
    host threads (the library call releases the GIL): every result equals the
    same handle's solve on its own, bit for bit."""
    from concurrent.futures import ThreadPoolExecutor
    print(f"\n[streams] {prec}", flush=True)
    shapes = [(16, 16, 16), (24, 12, 32), (8, 8, 8)]
    Eb = np.array([1e-3, 0.0, 0.0, 0.0, 0.0, 5e-4])
    jobs = []
    for k, shape in enumerate(shapes):
        systems = _cells(shape, (10.0, 1e2))
        stream = torch.cuda.Stream()
        h = L.create_batch(systems, scheme="afb", prec=prec, stream=stream)
        dev = torch.zeros((len(systems), 6) + shape, dtype=_dt(prec), device="cuda")
        jobs.append((h, stream, np.tile(Eb, (len(systems), 1)), dev))

    def run(job):
        h, stream, Ebs, dev = job
        return L.solve_batch(h, Ebs, 1e-9, 3000, eps_dev=dev)

    try:
        alone = []
        for job in jobs:
            out = run(job)
            torch.cuda.synchronize()
            alone.append((out, job[3].cpu().numpy()))
        for job in jobs:
            job[3].zero_()
        torch.cuda.synchronize()
        with ThreadPoolExecutor(max_workers=len(jobs)) as pool:
            together = list(pool.map(run, jobs))
        torch.cuda.synchronize()
        for (a, eps_a), b, job in zip(alone, together, jobs):
            assert np.array_equal(a[2], b[2])            # iterations per system
            assert np.array_equal(a[1], b[1])            # mean stress
            assert np.array_equal(eps_a, job[3].cpu().numpy())
    finally:
        for job in jobs:
            L.destroy(job[0])
