"""Pins for the oracle's transforms and finite-difference symbols (CPU only).

Transforms are pinned against the defining triple sum; symbols against the
difference stencils they are the modal form of (Sec. 3.1 eq. (12), Sec. 5.3
eqs. (36)-(39) carried to 3D), applied to sampled plane waves.
"""
import numpy as np
import pytest

from oracle import fdd, fourier


@pytest.mark.parametrize("shape", [(4, 4, 4), (4, 6, 2), (6, 4, 8)])
@pytest.mark.parametrize("centre", [False, True])
def test_transform_matches_bruteforce_dft(shape, centre):
    n1, n2, n3 = shape
    rng = np.random.default_rng(1)
    f = rng.standard_normal((2, n3, n2, n1))
    ref = fourier.dft_bruteforce(f, centre=centre)
    got = fourier.pcd_forward(f) if centre else fourier.td_forward(f)
    assert np.max(np.abs(got - ref)) < 1e-12


@pytest.mark.parametrize("n", [4, 5, 6, 8])
def test_inverse_is_inverse(n):
    # F^+ F^- = identity (Appendix A, cardinality of the TD basis)
    F = fourier.dft_matrix(n)
    assert np.allclose(F.conj().T @ F, np.eye(n), atol=1e-13)
    Fc = fourier.dft_matrix(n, centre=True)
    assert np.allclose(Fc.conj().T @ Fc, np.eye(n), atol=1e-13)
    rng = np.random.default_rng(0)
    f = rng.standard_normal((n, n + 1, n + 2))
    assert np.allclose(fourier.pcd_inverse(fourier.pcd_forward(f)).real, f, atol=1e-13)


def test_centred_index_is_paper_set():
    # kappa = mu - 1 - m, mu = 1..n, m = n/2: {-n/2, ..., n/2 - 1}
    for n in (4, 8, 10):
        assert sorted(fourier.centred_index(n).tolist()) == list(range(-n // 2, n // 2))


def _plane_wave(k, x):
    return np.exp(1j * k * x)


@pytest.mark.parametrize("n", [6, 8])
@pytest.mark.parametrize("h", [1.0, 0.7])
def test_1d_symbols_are_stencil_eigenvalues(n, h):
    s = fdd.symbols_1d(n, h)
    kap = fourier.centred_index(n)
    x = np.linspace(0.1, 3.0, 7)
    for j, a in enumerate(kap):
        k = 2 * np.pi * a / (n * h)
        f = lambda y: _plane_wave(k, y)
        stencils = {
            "FD": (f(x + h) - f(x)) / h,
            "BD": (f(x) - f(x - h)) / h,
            "CD": (f(x + h) - f(x - h)) / (2 * h),
            "hC": (f(x + h / 2) - f(x - h / 2)) / h,
        }
        for key, val in stencils.items():
            assert np.allclose(val, s[key][j] * f(x), atol=1e-12), (key, a)
        # plain Fourier derivative
        assert np.isclose(s["F"][j], 1j * k)


def test_exact_zeros_at_nyquist_and_dc():
    n = 8
    s = fdd.symbols_1d(n)
    kap = fourier.centred_index(n)
    nyq = np.where(kap == -n // 2)[0][0]
    assert s["FD"][nyq] == -2.0 and s["BD"][nyq] == 2.0
    assert s["CD"][nyq] == 0.0 and s["ep1"][nyq] == 0.0
    assert s["FD"][0] == 0.0 and s["hC"][0] == 0.0
    assert s["cosh_half"][nyq] == 0.0


def _averaged_stencil(kind, f, x, h):
    """The cell-averaged differences of eqs. (36)-(39), carried to 3D (eq. (43))."""
    out = []
    for r in range(3):
        s, t = [(1, 2), (2, 0), (0, 1)][r]
        e = np.eye(3)
        if kind == "AFD":
            d = lambda y: (f(y + h[r] * e[r]) - f(y)) / h[r]
            offs = [(0, 0), (1, 0), (0, 1), (1, 1)]
            scale = 1.0
        elif kind == "ABD":
            d = lambda y: (f(y) - f(y - h[r] * e[r])) / h[r]
            offs = [(0, 0), (-1, 0), (0, -1), (-1, -1)]
            scale = 1.0
        elif kind == "ACD":
            d = lambda y: (f(y + h[r] * e[r]) - f(y - h[r] * e[r])) / (2 * h[r])
            offs = [(-1, -1), (1, -1), (-1, 1), (1, 1)]
            scale = 1.0
        elif kind == "AhC":
            d = lambda y: (f(y + 0.5 * h[r] * e[r]) - f(y - 0.5 * h[r] * e[r])) / h[r]
            offs = [(-1, -1), (1, -1), (-1, 1), (1, 1)]
            scale = 0.5
        acc = 0
        for (a, b) in offs:
            acc = acc + d(x + scale * a * h[s] * e[s] + scale * b * h[t] * e[t])
        out.append(acc / 4.0)
    return np.array(out)


@pytest.mark.parametrize("kind", ["AFD", "ABD", "ACD", "AhC"])
def test_3d_averaged_symbols_are_stencil_eigenvalues(kind):
    n = (4, 6, 8)
    h = (1.0, 0.8, 1.3)
    q = fdd.symbols_3d(kind, n, h)
    rng = np.random.default_rng(2)
    pts = rng.uniform(0, 3, (5, 3))
    kap = [fourier.centred_index(v) for v in n]
    for j3 in range(n[2]):
        for j2 in range(0, n[1], 2):
            for j1 in range(n[0]):
                k = np.array([2 * np.pi * kap[0][j1] / (n[0] * h[0]),
                              2 * np.pi * kap[1][j2] / (n[1] * h[1]),
                              2 * np.pi * kap[2][j3] / (n[2] * h[2])])
                f = lambda y: np.exp(1j * (y @ k))
                for x in pts:
                    got = _averaged_stencil(kind, f, x, h)
                    assert np.allclose(got, q[j3, j2, j1] * f(x), atol=1e-12)


def test_abd_shifted_equals_ahc():
    # eq. (40): ABD at x + h/2 (every axis) equals AhC at x; a shift by +h_r/2
    # multiplies a mode by exp(i pi kappa_r / n_r) on each axis
    n = (6, 4, 8)
    h = (1.0, 0.5, 2.0)
    qabd = fdd.symbols_3d("ABD", n, h)
    qahc = fdd.symbols_3d("AhC", n, h)
    e = [np.exp(1j * np.pi * fourier.centred_index(v) / v) for v in n]
    ph = e[2][:, None, None] * e[1][None, :, None] * e[0][None, None, :]
    assert np.allclose(qabd * ph[..., None], qahc, atol=1e-13)


def test_willot_w_equals_fd_off_nyquist_and_afd_is_phase_times_ahc():
    n = (8, 6, 4)
    qafd = fdd.symbols_3d("AFD", n)
    qahc = fdd.symbols_3d("AhC", n)
    qr = fdd.symbols_3d("R", n)
    kap = [fourier.centred_index(v) for v in n]
    nyq = np.zeros((n[2], n[1], n[0]), dtype=bool)
    for r in range(3):
        sl = [None, None, None]
        sl[2 - r] = slice(None)
        nyq |= np.broadcast_to((kap[r] == -n[r] // 2)[tuple(sl)], nyq.shape)
    # Sec. 5.3 after eq. (44): q^W = q^FD except at the Nyquist index
    assert np.allclose(qr[~nyq], qafd[~nyq], atol=1e-12)
    # scalar phase Phi = exp(1/2 sum_r q_r h_r): q^AFD = Phi q^AhC
    th = [np.pi * k / v for k, v in zip(kap, n)]
    Phi = np.exp(1j * (th[2][:, None, None] + th[1][None, :, None] + th[0][None, None, :]))
    assert np.allclose(qafd, Phi[..., None] * qahc, atol=1e-13)
    # q^AhC is i times a real vector (the rotated wavevector)
    assert np.max(np.abs(qahc.real)) < 1e-15


@pytest.mark.parametrize("n", [4, 8, 10])
def test_afb_singular_set_size(n):
    qa, qb = fdd.scheme_pair("AFB", n)
    sing = fdd.singular_mask(qa, qb)
    # xi = 0 plus every frequency with at least two Nyquist indices
    assert int(sing.sum()) == 3 * n - 1
    for s in ("basic", "FB"):
        qa, qb = fdd.scheme_pair(s, n)
        assert int(fdd.singular_mask(qa, qb).sum()) == 1


