"""The seeded input generators: the spherical Bessel table against scipy, the
torch evaluation of the radial covariance against the numpy one, and the
covariance's defining properties (symmetric, positive semi-definite)."""
import numpy as np
import pytest

from paper_0909_0009_amd import inputs


def test_bessel_table_matches_scipy():
    """j_l(x) for l <= 300 on both recurrence branches (downward below
    x = L + 60, upward above), against scipy.special.spherical_jn, to 1e-11
    of each l's largest value over the points."""
    from scipy.special import spherical_jn
    L = 300
    x = np.concatenate([np.geomspace(1e-3, 350.0, 400), np.linspace(361.0, 3000.0, 200)])
    J = inputs.sph_bessel_table(L, x)
    ref = np.stack([spherical_jn(l, x) for l in range(L + 1)])
    scale = np.maximum(np.max(np.abs(ref), axis=1, keepdims=True), 1e-300)
    assert np.max(np.abs(J - ref) / scale) <= 1e-11


def test_torch_covariance_matches_numpy():
    torch = pytest.importorskip("torch")
    r, _ = inputs.radial_nodes(17)
    C = inputs.covariance(60, r)
    Ct = inputs.covariance_torch(60, r, "cpu", kchunk=512)
    assert np.max(np.abs(C - Ct)) <= 1e-13 * np.max(np.abs(C))
    assert torch is not None


def test_covariance_is_symmetric_positive_semidefinite():
    r, _ = inputs.radial_nodes(24)
    C = inputs.covariance(20, r)
    for l in (0, 5, 20):
        assert np.allclose(C[l], C[l].T, rtol=0, atol=1e-15 * np.max(np.abs(C[l])))
        ev = np.linalg.eigvalsh(C[l])
        assert ev.min() >= -1e-12 * ev.max()
