"""Pins of the quadrature-design oracle (oracle/quadrature.py, Sect. 3): the
error formula against a Monte Carlo of the weighted sum, its eigenpair form,
the optimal weights against perturbations and closed forms, and the greedy
design against its one-node closed form and monotonicity."""
import numpy as np
import pytest

from oracle import quadrature as q
from paper_0909_0009_amd import inputs


def _spd(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    return A @ A.T / n + 0.05 * np.eye(n)


def test_error_formula_matches_eigenpair_form():
    C = _spd(12, 1)
    rng = np.random.default_rng(2)
    a, nodes, w = rng.standard_normal(12), [3, 7, 10], rng.standard_normal(3)
    e1 = q.expected_error(C, a, nodes, w)
    e2 = q.expected_error_eigen(C, a, nodes, w)
    assert abs(e1 - e2) <= 1e-12 * abs(e1)


def test_error_formula_matches_monte_carlo():
    """Draw Phi ~ N(0, C) on the fine grid and average (I_hat - I)^2."""
    n, K = 10, 200_000
    C = _spd(n, 3)
    rng = np.random.default_rng(4)
    a = rng.standard_normal(n)
    nodes, w = [1, 4, 8], rng.standard_normal(3)
    Lc = np.linalg.cholesky(C)
    phi = rng.standard_normal((K, n)) @ Lc.T
    d = phi[:, nodes] @ w - phi @ a
    mc = np.mean(d * d)
    # (I_hat - I) is Gaussian: the sample mean of its square has relative
    # standard error sqrt(2 / K)
    pred = q.expected_error(C, a, nodes, w)
    assert abs(mc - pred) <= 5.0 * np.sqrt(2.0 / K) * pred


def test_optimal_weights_are_a_minimum():
    C = _spd(15, 5)
    rng = np.random.default_rng(6)
    a = rng.standard_normal(15)
    nodes = [0, 2, 9, 14]
    w = q.optimal_weights(C, a, nodes)
    e0 = q.expected_error(C, a, nodes, w)
    assert abs(e0 - q.optimal_error(C, a, nodes)) <= 1e-12 * abs(e0)
    for k in range(20):
        dw = 1e-3 * rng.standard_normal(4)
        assert q.expected_error(C, a, nodes, w + dw) > e0


def test_all_nodes_reproduce_the_fine_sum():
    C = _spd(8, 7)
    a = np.random.default_rng(8).standard_normal(8)
    nodes = list(range(8))
    w = q.optimal_weights(C, a, nodes)
    assert np.allclose(w, a, rtol=1e-10, atol=1e-12)
    assert abs(q.optimal_error(C, a, nodes)) <= 1e-10 * float(a @ C @ a)


def test_greedy_first_node_closed_form_and_monotone():
    """One node j with its optimal weight leaves a^T C a - (C a)_j^2 / C_jj,
    so the first greedy choice maximises the sum of (C a)_j^2 / C_jj."""
    probs = [(_spd(20, 10 + s), np.random.default_rng(20 + s).standard_normal(20))
             for s in range(3)]
    nodes, errs = q.greedy_nodes(probs, 6)
    gain = sum((C @ a) ** 2 / np.diag(C) for C, a in probs)
    assert nodes[0] == int(np.argmax(gain))
    assert len(set(nodes)) == 6
    assert all(e2 <= e1 * (1 + 1e-12) for e1, e2 in zip(errs, errs[1:]))
    total0 = sum(float(a @ C @ a) for C, a in probs)
    assert errs[0] < total0


def test_design_on_the_synthetic_inputs():
    """The synthetic covariance and transfer tables on a 48-shell fine grid:
    T and E problems for l = 2..5 with equal weights.  The first node sits
    at the transfer tables' peak (r = 14000 Mpc), and twelve greedy nodes
    leave a tenth or less of the summed relative error of twelve evenly
    spaced shells with their own optimal weights."""
    L = 5
    r = np.linspace(13000.0, 15000.0, 48)
    C = inputs.covariance(L, r)
    alpha, beta = inputs.transfer_tables(L, r)
    probs = []
    for l in range(2, L + 1):
        for X in (alpha, beta):
            probs.append((C[l], q.fine_weights(r, X[l])))
    scale = [float(a @ Cl @ a) for Cl, a in probs]
    rel = [(Cl / s, a) for (Cl, a), s in zip(probs, scale)]
    nodes, errs = q.greedy_nodes(rel, 12)
    even = list(np.linspace(0, 47, 12).round().astype(int))
    err_even = sum(q.optimal_error(Cl, a, even) for Cl, a in rel)
    assert abs(r[nodes[0]] - 14000.0) < 100.0
    assert errs[-1] < 0.1 * err_even


def _tight_problems(L=4, ntot=120, spacing=2.0):
    """T and E problems for l = 2..L on a fine grid spaced `spacing` Mpc
    around 14000 Mpc (far below the correlation length), each scaled to unit
    a^T C a."""
    r = 14000.0 + spacing * (np.arange(ntot) - ntot // 2)
    C = inputs.covariance(L, r)
    alpha, beta = inputs.transfer_tables(L, r)
    probs = []
    for l in range(2, L + 1):
        for X in (alpha, beta):
            a = q.fine_weights(r, X[l])
            probs.append((C[l] / float(a @ C[l] @ a), a))
    return probs


def test_design_on_a_tight_grid_stays_nonnegative():
    """On a 2 Mpc grid the conditional variances collapse to rounding noise
    after about two dozen nodes.  The design must then stop gaining: the
    error curve stays >= 0, never rises, equals a from-scratch recomputation
    of every step's error (eigendecomposition solve on each problem's
    independent nodes), and the independent sets stop growing while further
    nodes are still chosen."""
    probs = _tight_problems()
    n = 40
    nodes, errs = q.greedy_nodes(probs, n)
    errs = np.array(errs)
    total = len(probs)
    assert np.all(errs >= 0.0)
    assert np.all(np.diff(errs) <= 1e-13 * total)
    again = np.array(q.design_errors(probs, nodes))
    assert np.max(np.abs(again - errs)) <= 1e-12 * total
    sets = q.effective_sets(probs, nodes)
    assert max(len(s) for s in sets) < n
    # the dependent nodes of a problem get weight 0 there; the weights of the
    # independent ones reproduce the error
    W = q.design_weights(probs, nodes)
    for p, ((C, a), B) in enumerate(zip(probs, sets)):
        dep = [k for k, j in enumerate(nodes) if j not in B]
        assert np.all(W[p, dep] == 0.0)
        e = q.expected_error(C, a, nodes, W[p])
        assert abs(e - q.optimal_error(C, a, B)) <= 1e-12


def test_dependent_duplicate_shell_gets_no_weight():
    """A fine grid whose last shell repeats the first: once one copy is a node
    the other is dependent (conditional variance 0) and gains nothing."""
    C0 = _spd(10, 30)
    idx = list(range(10)) + [0]
    C = C0[np.ix_(idx, idx)]
    a = np.random.default_rng(31).standard_normal(11)
    nodes, errs = q.greedy_nodes([(C, a)], 11)
    sets = q.effective_sets([(C, a)], nodes)
    assert len(sets[0]) == 10 and not ({0, 10} <= set(sets[0]))
    assert abs(errs[-1]) <= 1e-10 * float(a @ C @ a)
