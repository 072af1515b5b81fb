"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/lsfft.h declares, and rejects invalid input with
LSFFT_EINVAL before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2009_03762_amd import lsfft
    return lsfft


def declared_functions():
    src = open(os.path.join(ROOT, "include", "lsfft.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lsfft_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 10
    lib = ctypes.CDLL(L._LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(L.EXPORTS) == set(names)


def test_strings(L):
    assert "gfx950" in L.version()
    assert L.status_string(L.OK) == "converged"
    assert L.status_string(L.EINVAL) == "invalid argument"
    assert L.kernel_name(0) == "k_xpass"


def _mat(shape, lam=1.0, mu=1.0):
    n1, n2, n3 = shape
    return np.full((n3, n2, n1), lam), np.full((n3, n2, n1), mu)


# Supported: even 2^a 3^b in [4, 512] on every axis.  Rejected: a factor 5 or
# 7, odd lengths (27 = 3^3, 9), lengths past 512 (768, 1024) or below 4.
@pytest.mark.parametrize("shape", [(10, 8, 8), (8, 7, 8), (8, 8, 1024), (2, 8, 8), (8, 8, 27), (9, 8, 8),
                                   (8, 40, 8), (8, 8, 768), (8, 8, 972)])
def test_unsupported_sizes_rejected(L, shape):
    lam, mu = _mat(shape)
    with pytest.raises(L.LsfftError) as e:
        L.create(lam, mu, 1.0, 1.0)
    assert e.value.status == L.EINVAL


@pytest.mark.parametrize("lam,mu", [(np.nan, 1.0), (1.0, 0.0), (1.0, -1.0), (-1.0, 1.0), (1.0, np.inf)])
def test_bad_moduli_rejected(L, lam, mu):
    la, mu_ = _mat((8, 8, 8))
    la[1, 2, 3] = lam
    mu_[1, 2, 3] = mu
    with pytest.raises(L.LsfftError) as e:
        L.create(la, mu_, 1.0, 1.0)
    assert e.value.status == L.EINVAL


@pytest.mark.parametrize("kw", [dict(lambda0=1.0, mu0=0.0), dict(lambda0=-1.0, mu0=1.0),
                                dict(scheme="dgo", disc="td"), dict(scheme="dgo", disc="pcd", dgo_images=-1),
                                dict(scheme="dgo", disc="pcd", dgo_weight_power=3),
                                dict(scheme=7), dict(prec=5), dict(disc=4), dict(h=(1.0, -1.0, 1.0)),
                                dict(form=3), dict(f64_warmup=-1), dict(refine=-1), dict(scheme=6),
                                dict(scheme="cd", form=2),
                                dict(scheme="acd", form="displacement")])
def test_bad_config_rejected(L, kw):
    lam, mu = _mat((8, 8, 8))
    args = dict(lambda0=1.0, mu0=1.0)
    args.update(kw)
    l0, m0 = args.pop("lambda0"), args.pop("mu0")
    with pytest.raises(L.LsfftError) as e:
        L.create(lam, mu, l0, m0, **args)
    assert e.value.status == L.EINVAL


def test_null_handles(L):
    Eb = np.zeros(6)
    with pytest.raises(L.LsfftError) as e:
        L.solve(None, Eb, 1e-6, 10)
    assert e.value.status == L.EINVAL
    assert L.destroy(None) == L.OK
    with pytest.raises(L.LsfftError):
        L.set_timing(None, 0)


def test_macro_strain_must_have_six_components(L):
    with pytest.raises(ValueError):
        L.solve(None, np.zeros(3), 1e-6, 10)
    with pytest.raises(ValueError):
        L.solve_device(None, 1.0, 1e-6, 10)


def test_batch_configs_must_agree(L):
    lam, mu = _mat((8, 8, 8))
    lam2, mu2 = _mat((8, 8, 16))
    with pytest.raises(L.LsfftError) as e:
        L.create_batch([(lam, mu, 1.0, 1.0), (lam2, mu2, 1.0, 1.0)])
    assert e.value.status == L.EINVAL
    with pytest.raises(L.LsfftError) as e:   # the DGO table needs one reference medium
        L.create_batch([(lam, mu, 1.0, 1.0), (lam, mu, 1.1, 1.0)], scheme="dgo", disc="pcd")
    assert e.value.status == L.EINVAL
    with pytest.raises(L.LsfftError) as e:
        L.create_batch([])
    assert e.value.status == L.EINVAL
    assert L.batch_size(None) == 0


@pytest.mark.parametrize("kw", [dict(scheme="dgo", disc="td"), dict(scheme="dgo", disc="pcd", dgo_images=65),
                                dict(scheme="dgo", disc="pcd", dgo_weight_power=0), dict(scheme=5),
                                dict(disc=2), dict(prec=3), dict(h=-1.0), dict(tol=-1.0), dict(maxit=-1),
                                dict(maxit=20000000)])
def test_1d_bad_options_rejected(L, kw):
    C = np.linspace(1.0, 2.0, 16)
    with pytest.raises(L.LsfftError) as e:
        L.solve_1d(C, 1.5, 1e-3, **kw)
    assert e.value.status == L.EINVAL


@pytest.mark.parametrize("C,CH,Eb", [(np.ones(10), 1.0, 1.0), (np.ones(1024), 1.0, 1.0),
                                     (np.array([1.0, -1.0, 1.0, 1.0]), 1.0, 1.0),
                                     (np.array([1.0, np.nan, 1.0, 1.0]), 1.0, 1.0),
                                     (np.ones(8), 0.0, 1.0), (np.ones(8), 1.0, np.inf)])
def test_1d_bad_inputs_rejected(L, C, CH, Eb):
    with pytest.raises(L.LsfftError) as e:
        L.solve_1d(C, CH, Eb)
    assert e.value.status == L.EINVAL


def test_1d_dgo_needs_a_macroscopic_strain(L):
    with pytest.raises(L.LsfftError) as e:
        L.solve_1d(np.ones(8), 1.0, 0.0, scheme="dgo", disc="pcd")
    assert e.value.status == L.EINVAL


def test_bench_refuses_more_than_one_gpu():
    """bench.py is a one-GPU measurement: --gpus above 1 exits with status 2
    and says so, before touching any device."""
    import subprocess
    import sys
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU" in out.stderr
