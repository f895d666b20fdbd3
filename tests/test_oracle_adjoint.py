"""Pins of the oracle's adjoint: central finite differences of its own forward
(exact for a loss quadratic in the noise), and an independent dense model of
the whole map generator built from scipy's Y_lm and numpy's Gauss-Legendre
rule, differentiated by torch autograd."""
import math

import numpy as np
import pytest
import torch
from scipy import special

from paper_0909_0009_amd import inputs


def nlm(L):
    return (L + 1) * (L + 2) // 2


def rand_c(shape, rng):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def small_problem(orc, L, N, mean=0, seed=0):
    rng = np.random.default_rng(seed)
    r, w = inputs.radial_nodes(N)
    A = rng.standard_normal((L + 1, N, N)) * 1e-3
    F = np.tril(A)
    alpha = rng.standard_normal((L + 1, N)) * 1e-7
    beta = rng.standard_normal((L + 1, N)) * 1e-7
    beta[:2] = 0
    P = orc.Problem(L, r, w, F, alpha, beta, mean_mode=mean)
    n = inputs.noise(L, N, 77 + seed)
    return P, n


def loss(P, n, fnl, gT, gE):
    o = P.forward(n, fnl)
    return float(np.real(np.vdot(gT, o["aT"]) + np.vdot(gE, o["aE"])))


@pytest.mark.parametrize("mean", [0, 1])
def test_adjoint_matches_central_differences(orc, mean):
    L, N, fnl = 6, 4, 37.0
    P, n = small_problem(orc, L, N, mean)
    rng = np.random.default_rng(5)
    gT, gE = rand_c(nlm(L), rng), rand_c(nlm(L), rng)
    gn, gf = P.adjoint(n, fnl, gT, gE)
    _, ms = inputs.lm_arrays(L)
    assert np.all(gn[:, ms == 0].imag == 0)
    for t in range(6):
        d = rand_c(n.shape, np.random.default_rng(100 + t))
        h = 1e-3
        num = (loss(P, n + h * d, fnl, gT, gE) - loss(P, n - h * d, fnl, gT, gE)) / (2 * h)
        ana = float(np.real(np.vdot(gn, d)))
        assert abs(num - ana) < 1e-9 * (abs(ana) + 1e-30), (t, num, ana)
    # single components, including an m = 0 imaginary part (ignored input)
    for (j, i, part) in ((0, 0, 1), (1, 3, 1j), (N - 1, nlm(L) - 1, 1), (2, 0, 1j)):
        d = np.zeros_like(n)
        d[j, i] = part
        h = 1e-3
        num = (loss(P, n + h * d, fnl, gT, gE) - loss(P, n - h * d, fnl, gT, gE)) / (2 * h)
        ana = float(np.real(np.vdot(gn, d)))
        assert abs(num - ana) < 1e-9 * max(abs(ana), 1e-12 * np.max(np.abs(gn))), (j, i, num, ana)
    # f_NL enters linearly
    h = 1.0
    num = (loss(P, n, fnl + h, gT, gE) - loss(P, n, fnl - h, gT, gE)) / (2 * h)
    assert abs(num - gf) < 1e-10 * abs(gf)


def dense_model(L, ntheta, nphi, r, w, F, alpha, beta, mean):
    """Dense torch model: Y matrices from scipy sph_harm_y on numpy's
    Gauss-Legendre rule; returns a function (n_re, n_im, fnl) -> (aT, aE)
    as (re, im) pairs."""
    xr, wr = np.polynomial.legendre.leggauss(ntheta)
    th = np.arccos(xr)
    ph = 2 * np.pi * np.arange(nphi) / nphi
    ls, ms = inputs.lm_arrays(L)
    T, Pp = np.meshgrid(th, ph, indexing="ij")
    # real basis: field = sum_lm c_m (Re a cos(m phi) lam - Im a sin(m phi) lam)
    Bre = np.empty((nlm(L), ntheta * nphi))
    Bim = np.empty((nlm(L), ntheta * nphi))
    for q, (l, m) in enumerate(zip(ls, ms)):
        Y = special.sph_harm_y(l, m, T, Pp).ravel()   # includes e^{i m phi}
        c = 1.0 if m == 0 else 2.0
        Bre[q] = c * Y.real
        Bim[q] = -c * Y.imag if m > 0 else 0.0
    pw = np.repeat(wr * 2 * np.pi / nphi, nphi)
    # analysis: a_lm = sum_pix pw Y*_lm map
    Are = np.empty((nlm(L), ntheta * nphi))
    Aim = np.empty((nlm(L), ntheta * nphi))
    for q, (l, m) in enumerate(zip(ls, ms)):
        Y = special.sph_harm_y(l, m, T, Pp).ravel()
        Are[q] = pw * Y.real
        Aim[q] = -pw * Y.imag if m > 0 else 0.0
    tt = lambda a: torch.tensor(a, dtype=torch.float64)
    Bre, Bim, Are, Aim, pw_t = tt(Bre), tt(Bim), tt(Are), tt(Aim), tt(pw)
    Ft = tt(F)[ls]                                   # [nlm, N, N]
    base = w * r ** 2
    WT = tt(alpha * base[None, :])[ls]               # [nlm, N]
    WE = tt(beta * base[None, :])[ls]
    m0 = tt((ms == 0).astype(float))
    ensemble = tt(np.einsum("l,lij->i", (2 * np.arange(L + 1) + 1) / (4 * np.pi), F ** 2))

    def run(nre, nim, fnl):
        nim = nim * (1 - m0)[None, :]
        pre = torch.einsum("qij,jq->iq", Ft, nre)
        pim = torch.einsum("qij,jq->iq", Ft, nim)
        f = pre @ Bre + pim @ Bim                    # [N, pix]
        sq = f * f
        if mean == 0:
            mu = (sq * pw_t).sum(1) / (4 * np.pi)
        else:
            mu = ensemble
        g = sq - mu[:, None]
        nre_ = g @ Are.T
        nim_ = g @ Aim.T
        aTr = (WT.T * (pre + fnl * nre_)).sum(0)
        aTi = (WT.T * (pim + fnl * nim_)).sum(0)
        aEr = (WE.T * (pre + fnl * nre_)).sum(0)
        aEi = (WE.T * (pim + fnl * nim_)).sum(0)
        return aTr, aTi, aEr, aEi

    return run


@pytest.mark.parametrize("mean", [0, 1])
def test_forward_and_adjoint_match_dense_autograd_model(orc, mean):
    L, N, fnl = 4, 3, 55.0
    P, n = small_problem(orc, L, N, mean, seed=3)
    model = dense_model(L, P.ntheta, P.nphi, P.r, P.w, P.filter, P.alpha, P.beta, mean)
    nre = torch.tensor(n.real.copy(), requires_grad=True)
    nim = torch.tensor(n.imag.copy(), requires_grad=True)
    f = torch.tensor(fnl, dtype=torch.float64, requires_grad=True)
    aTr, aTi, aEr, aEi = model(nre, nim, f)
    o = P.forward(n, fnl)
    sc = np.max(np.abs(o["aT"]))
    assert np.max(np.abs(aTr.detach().numpy() + 1j * aTi.detach().numpy() - o["aT"])) < 1e-12 * sc
    sc = np.max(np.abs(o["aE"]))
    assert np.max(np.abs(aEr.detach().numpy() + 1j * aEi.detach().numpy() - o["aE"])) < 1e-12 * sc
    rng = np.random.default_rng(9)
    gT, gE = rand_c(nlm(L), rng), rand_c(nlm(L), rng)
    tl = ((aTr * torch.tensor(gT.real)).sum() + (aTi * torch.tensor(gT.imag)).sum()
          + (aEr * torch.tensor(gE.real)).sum() + (aEi * torch.tensor(gE.imag)).sum())
    tl.backward()
    ref_n = nre.grad.numpy() + 1j * nim.grad.numpy()
    gn, gf = P.adjoint(n, fnl, gT, gE)
    assert np.max(np.abs(gn - ref_n)) < 1e-11 * np.max(np.abs(ref_n))
    assert abs(gf - f.grad.item()) < 1e-11 * abs(gf)
