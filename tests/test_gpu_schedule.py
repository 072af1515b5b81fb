"""Launch schedules (lsfft_get_schedule / lsfft_set_schedule / lsfft_autotune):
every schedule a grid offers gives the same iterates as the default one, the
tuner leaves a valid schedule in force, and invalid schedules are refused.
The default-schedule solves these are compared with are themselves checked
against the oracle in the parity tests; one case here repeats that check."""
import itertools

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


def _cell(n, chi):
    """Cubic inclusion of half the cell on the grid n = (n1, n2, n3); arrays of
    shape (n3, n2, n1)."""
    lam, mu = inputs.cubic_inclusion(n, tuple(v // 2 for v in n), 1.0, chi)
    l0, m0 = inputs.reference_medium_mean(1.0, chi)
    return lam, mu, l0, m0


def _accepts(L, h, sch):
    try:
        L.set_schedule(h, sch)
        return True
    except L.LsfftError as e:
        assert e.status == L.EINVAL
        return False


def _offered(L, h, n3):
    """The values of each knob the handle accepts, found by probing."""
    d = L.get_schedule(h)
    out = {}
    for key, cands in (("y_cols", (d["y_cols"] // 2, d["y_cols"] * 2)),
                       ("z_cols", (d["z_cols"] // 2, d["z_cols"] * 2))):
        vals = [d[key]]
        for c in cands:
            if c > 0 and _accepts(L, h, dict(d, **{key: c})):
                vals.append(c)
        out[key] = vals
    if d["stencil_planes"]:
        out["stencil_planes"] = [z for z in (2, 4, 8, 16, 32) if n3 % z == 0]
    else:
        out["stencil_planes"] = [0]
    L.set_schedule(h, d)
    assert L.get_schedule(h) == d
    return d, out


CASES = [("afb", "displacement", "f64"), ("afb", "displacement", "f32"), ("fb", "displacement", "f64"),
         ("afb", "strain", "f64"), ("basic", "auto", "f32")]


@pytest.mark.parametrize("scheme,form,prec", CASES)
def test_every_offered_schedule_gives_the_same_iterates(L, scheme, form, prec):
    """Fixed 12 iterations on an inclusion cell with n = (24, 16, 32) (n1 not
    a power of two: the LDS stencil) under every combination of the offered
    knobs."""
    lam, mu, l0, m0 = _cell((24, 16, 32), 30.0)
    Eb = np.array([1e-3, -2e-4, 3e-4, 1e-4, -1e-4, 2e-4])
    K = 12
    s = L.Solver(lam, mu, l0, m0, scheme=scheme, prec=prec, form=form)
    d, offered = _offered(L, s.handle, lam.shape[0])
    print(f"\n[schedule] {scheme} {form} {prec} default {d} offered {offered}", flush=True)
    ref = s.solve(Eb, tol=0.0, maxit=K)
    assert len(offered["y_cols"]) == 2 and len(offered["z_cols"]) == 2
    tol = 1e-13 if prec == "f64" else 2e-6
    worst = 0.0
    for z, y, zc, x in itertools.product(offered["stencil_planes"], offered["y_cols"], offered["z_cols"], (0, 7)):
        sch = {"stencil_planes": z, "y_cols": y, "z_cols": zc, "xcd_order": x}
        L.set_schedule(s.handle, sch)
        assert L.get_schedule(s.handle) == sch
        out = s.solve(Eb, tol=0.0, maxit=K)
        assert out["iters"] == K
        e = rel(out["eps"], ref["eps"])
        worst = max(worst, e)
        assert e < tol, (sch, e)
        assert rel(out["sig_mean"], ref["sig_mean"]) < tol
        assert abs(out["residual"] - ref["residual"]) <= 1e-9 * ref["residual"]
    print(f"  largest field difference to the default schedule: {worst:.3e}", flush=True)
    s.close()


def test_set_schedule_refuses_what_the_grid_does_not_offer(L):
    lam, mu, l0, m0 = _cell((24, 16, 32), 10.0)  # n3 = 32
    print("\n[schedule] invalid schedules", flush=True)
    s = L.Solver(lam, mu, l0, m0, scheme="afb", prec="f64", form="displacement")
    d = L.get_schedule(s.handle)
    bad = [dict(d, stencil_planes=3), dict(d, stencil_planes=12), dict(d, stencil_planes=0),
           dict(d, stencil_planes=64), dict(d, y_cols=d["y_cols"] + 1), dict(d, z_cols=0),
           dict(d, xcd_order=8), dict(d, xcd_order=-1)]
    print(f"  default {d}", flush=True)
    for b in bad:
        try:
            L.set_schedule(s.handle, b)
        except L.LsfftError as e:
            assert e.status == L.EINVAL
        else:
            pytest.fail(f"accepted {b}")
        assert L.get_schedule(s.handle) == d
    s.close()
    t = L.Solver(lam, mu, l0, m0, scheme="afb", prec="f64", form="strain")
    dt = L.get_schedule(t.handle)
    assert dt["stencil_planes"] == 0
    with pytest.raises(L.LsfftError):
        L.set_schedule(t.handle, dict(dt, stencil_planes=2))
    with pytest.raises(L.LsfftError):
        L.autotune(t.handle, 0)
    t.close()


@pytest.mark.parametrize("scheme,form,prec", [("afb", "displacement", "f32"), ("afb", "strain", "f64"),
                                              ("afb", "displacement", "f64")])
def test_autotuned_schedule_converges_like_the_default(L, scheme, form, prec):
    """64^3 cubic inclusion, contrast 1e3: tune, then solve (FP64: to 1e-8; F32:
    a fixed 150 iterations, its residual meets a floor near 1e-4 at this
    contrast) and compare with a default-schedule handle and, in FP64, the
    oracle's fixed-iteration result."""
    lam, mu, l0, m0 = _cell((64, 64, 64), 1e3)
    Eb = np.array([1.0, 0, 0, 0, 0, 0])
    tol, maxit, want = (1e-8, 2000, L.OK) if prec == "f64" else (0.0, 150, L.ENOTCONV)
    print(f"\n[autotune] {scheme} {form} {prec} 64^3", flush=True)
    a = L.Solver(lam, mu, l0, m0, scheme=scheme, prec=prec, form=form)
    best, t0, t1 = L.autotune(a.handle, 8)
    print(f"  start {t0:.4f} ms/iter -> {t1:.4f} ms/iter with {best}", flush=True)
    assert L.get_schedule(a.handle) == best
    assert 0 < t1 <= t0
    out = a.solve(Eb, tol=tol, maxit=maxit)
    b = L.Solver(lam, mu, l0, m0, scheme=scheme, prec=prec, form=form)
    ref = b.solve(Eb, tol=tol, maxit=maxit)
    print(f"  tuned: status {out['status']} after {out['iters']}; default: {ref['status']} after {ref['iters']}",
          flush=True)
    assert out["status"] == want and ref["status"] == want
    assert abs(out["iters"] - ref["iters"]) <= 1
    assert rel(out["eps"], ref["eps"]) < (1e-12 if prec == "f64" else 1e-6)
    # a second tune starts from the tuned schedule and keeps a valid one
    best2, t0b, t1b = L.autotune(a.handle, 8)
    assert L.get_schedule(a.handle) == best2
    K = 6
    got = a.solve(Eb, tol=0.0, maxit=K)
    a.close()
    b.close()
    if prec == "f64":
        o = solve3d.solve_gfp(lam, mu, Eb, l0, m0, scheme="AFB", tol=0.0, maxit=K)
        assert rel(got["eps"], o.eps) < 1e-12


def test_schedule_changes_between_graph_replays(L):
    """Solves that replay captured iteration chunks, with the schedule changed
    and changed back between them (and eager solves in between), all give
    the default schedule's result."""
    lam, mu, l0, m0 = _cell((32, 32, 32), 100.0)
    Eb = np.array([0, 0, 0, 0, 0, 1.0])
    print("\n[schedule] graph replays across schedule changes", flush=True)
    s = L.Solver(lam, mu, l0, m0, scheme="afb", prec="f64", form="displacement")
    d, offered = _offered(L, s.handle, lam.shape[0])
    ref = s.solve(Eb, tol=1e-9, maxit=1000)
    alt = {"stencil_planes": offered["stencil_planes"][0], "y_cols": offered["y_cols"][-1],
           "z_cols": offered["z_cols"][-1], "xcd_order": 2}
    for sch in (alt, d, alt, d):
        L.set_schedule(s.handle, sch)
        for _ in range(2):
            out = s.solve(Eb, tol=1e-9, maxit=1000)
            assert out["iters"] == ref["iters"]
            assert rel(out["eps"], ref["eps"]) < 1e-13
            eager = s.solve(Eb, tol=0.0, maxit=3)
            assert eager["iters"] == 3
    s.close()


def test_batch_autotune(L):
    """A batch of three cells of different contrast: tuned batch solve equal
    to the default-schedule batch solve."""
    systems = [_cell((32, 24, 16), c) for c in (3.0, 30.0, 300.0)]
    shape = systems[0][0].shape
    Ebs = np.array([[1e-3, 0, 0, 0, 0, 0], [0, 0, 0, 0, 0, 2e-3], [1e-3, -5e-4, 2e-4, 1e-4, 3e-4, -2e-4]])
    print("\n[autotune] batch of 3 cells", flush=True)
    res = []
    for tune in (False, True):
        h = L.create_batch(systems, prec="f64", scheme="afb", form="displacement")
        if tune:
            best, t0, t1 = L.autotune(h, 8)
            print(f"  start {t0:.4f} ms/iter -> {t1:.4f} ms/iter with {best}", flush=True)
        eps = torch.zeros((3, 6) + shape, dtype=torch.float64, device="cuda")
        st, sm, it, r, sts = L.solve_batch(h, Ebs, 1e-9, 2000, eps, None)
        L.destroy(h)
        res.append((st, sm, it, eps.cpu().numpy()))
    assert res[0][0] == L.OK and res[1][0] == L.OK
    assert np.all(np.abs(res[0][2] - res[1][2]) <= 1)
    assert rel(res[1][3], res[0][3]) < 1e-11
    assert rel(res[1][1], res[0][1]) < 1e-11
