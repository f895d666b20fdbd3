"""Pins of the cubic KSW statistic's oracle (oracle/ksw.py, Sect. 4): the
sky integral of A B^2 on the grid against the exact Gaunt sum, against the
closed form of constant maps, grid independence above the exact grid, and
the statistic's cubic scaling and radial sum."""
import math

import numpy as np
import pytest

from oracle import ksw
from paper_0909_0009_amd import inputs


def _rand_alm(L, seed):
    rng = np.random.default_rng(seed)
    n = inputs.nlm(L)
    a = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    _, ms = inputs.lm_arrays(L)
    a[ms == 0] = a[ms == 0].real
    return a


def _one_node_tables(L, A, B):
    """Tables that make the filtered maps of node 0 equal A and B exactly:
    cinv = identity on T, alpha^T = beta^T = 1, data aT = A, aE = B would mix;
    instead the data carry A in T and B in E, alpha picks T and beta picks E."""
    alpha = np.zeros((2, L + 1, 1))
    beta = np.zeros((2, L + 1, 1))
    alpha[0, :, 0] = 1.0
    beta[1, :, 0] = 1.0
    cinv = np.broadcast_to(np.eye(2), (L + 1, 2, 2)).copy()
    return alpha, beta, cinv


@pytest.mark.parametrize("L", [2, 4])
def test_sky_integral_matches_gaunt_sum(orc, L):
    A, B = _rand_alm(L, 10 + L), _rand_alm(L, 20 + L)
    al, be, ci = _one_node_tables(L, A, B)
    got = ksw.cubic_statistic(L, [1.0], [1.0], al, be, ci, A, B)["S"]
    ref = ksw.sky_integral_gaunt(L, A, B)
    assert abs(got - ref) <= 1e-12 * abs(ref)


def test_constant_maps_closed_form(orc):
    """Only the (0,0) coefficients: A = A00/sqrt(4 pi), B = B00/sqrt(4 pi), so
    int A B^2 = A00 B00^2 / sqrt(4 pi)."""
    L = 3
    A = np.zeros(inputs.nlm(L), dtype=complex)
    B = np.zeros_like(A)
    A[0], B[0] = 1.7, -0.6
    al, be, ci = _one_node_tables(L, A, B)
    got = ksw.cubic_statistic(L, [1.0], [1.0], al, be, ci, A, B)["S"]
    assert abs(got - 1.7 * 0.36 / math.sqrt(4 * math.pi)) <= 1e-14


def test_grid_independence_and_scaling(orc):
    """Above the exact grid the result does not change; S is cubic in the
    data and the radial sum weights each node by w r^2."""
    L, N = 10, 5
    p = inputs.problem(L, N, cache=False)
    al, be, ci = inputs.ksw_tables(p)
    aT, aE = _rand_alm(L, 1), _rand_alm(L, 2)
    s0 = ksw.cubic_statistic(L, p["r"], p["w"], al, be, ci, aT, aE)
    s1 = ksw.cubic_statistic(L, p["r"], p["w"], al, be, ci, aT, aE, ntheta=29, nphi=47)
    assert abs(s0["S"] - s1["S"]) <= 1e-12 * s0["S_abs"]
    s2 = ksw.cubic_statistic(L, p["r"], p["w"], al, be, ci, -2.0 * aT, -2.0 * aE)
    assert abs(s2["S"] + 8.0 * s0["S"]) <= 1e-12 * 8.0 * s0["S_abs"]
    rad = p["w"] * p["r"] ** 2
    assert abs(np.sum(rad * s0["per_node"]) - s0["S"]) <= 1e-15 * s0["S_abs"]


def test_tables_reproduce_model_spectrum():
    """beta = C W on the nodes, and (C^-1)_l is the pseudo-inverse of the
    model spectrum W^T C W for l >= 2 (zero below): S C^+ S = S and
    C^+ S C^+ = C^+."""
    L, N = 12, 9
    p = inputs.problem(L, N, cache=False)
    al, be, ci = inputs.ksw_tables(p)
    wr2 = p["w"] * p["r"] ** 2
    for l in (2, 7, 12):
        S = np.array([[np.sum(al[x, l] * wr2 * be[y, l]) for y in range(2)] for x in range(2)])
        assert np.allclose(S @ ci[l] @ S, S, rtol=0, atol=1e-9 * np.abs(S).max())
        assert np.allclose(ci[l] @ S @ ci[l], ci[l], rtol=0, atol=1e-9 * np.abs(ci[l]).max())
        assert np.allclose(ci[l], ci[l].T)
    assert not np.any(ci[:2])
