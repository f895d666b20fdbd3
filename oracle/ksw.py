"""Plain FP64 oracle of the cubic KSW statistic S_prim of Sect. 4.

TEST INFRASTRUCTURE ONLY (like the rest of oracle/): it states what an
implementation of the statistic must compute, step by step, on the exact
Gauss-Legendre grid, using the oracle's own synthesis (fnl_oracle.c).

For data a^T_lm, a^E_lm and every radial node r_k the two filtered maps are

    A(r_k, n) = sum_{i,j in T,E} sum_lm (C^-1)^{ij}_l alpha^i_l(r_k) a^j_lm Y_lm(n),
    B(r_k, n) = sum_{i,j in T,E} sum_lm (C^-1)^{ij}_l beta^i_l(r_k)  a^j_lm Y_lm(n),

and the statistic is the radial quadrature of the sky integral of A B^2,

    S_prim = sum_k w_k r_k^2 int d^2n A(r_k, n) B(r_k, n)^2.

A B^2 has degree 3L along every ring and in cos theta, so a grid of
ceil((3L+1)/2) Gauss-Legendre rings and 3L+1 pixels per ring integrates it
exactly: the result is the closed form sum_lm c_m Re(conj(A_lm) [B^2]_lm).
"""
import numpy as np

from . import fnl_oracle as orc


def filtered_coeffs(L, tab, cinv, aT, aE, k):
    """Harmonic coefficients of a filtered map at node k: tab is alpha (for A)
    or beta (for B), [2][L+1][Nk] (T then E); cinv [L+1][2][2]."""
    ls = np.repeat(np.arange(L + 1), np.arange(1, L + 2))
    aT = np.asarray(aT, dtype=np.complex128)
    aE = np.asarray(aE, dtype=np.complex128)
    # inverse-covariance weighted data, per l: abar^i = sum_j (C^-1)^{ij} a^j
    barT = cinv[ls, 0, 0] * aT + cinv[ls, 0, 1] * aE
    barE = cinv[ls, 1, 0] * aT + cinv[ls, 1, 1] * aE
    return tab[0][ls, k] * barT + tab[1][ls, k] * barE


def cubic_statistic(L, r, w, alpha, beta, cinv, aT, aE, ntheta=None, nphi=None):
    """S_prim and its scale S_abs = sum_k w_k r_k^2 int |A| B^2 (the size of
    the terms that cancel in S_prim), plus the per-node sky integrals.
    Nodes whose tables are all zero are skipped (their integral is 0)."""
    alpha = np.asarray(alpha, dtype=np.float64)
    beta = np.asarray(beta, dtype=np.float64)
    cinv = np.asarray(cinv, dtype=np.float64)
    Nk = len(r)
    nth = orc.default_ntheta(L) if ntheta is None else int(ntheta)
    nph = orc.default_nphi(L) if nphi is None else int(nphi)
    x, wg = orc.gl_grid(nth)
    pix = wg[:, None] * (2.0 * np.pi / nph)
    per_node = np.zeros(Nk)
    per_abs = np.zeros(Nk)
    for k in range(Nk):
        if not (np.any(alpha[:, :, k]) or np.any(beta[:, :, k])):
            continue
        A = orc.synth(L, nth, nph, filtered_coeffs(L, alpha, cinv, aT, aE, k))
        B = orc.synth(L, nth, nph, filtered_coeffs(L, beta, cinv, aT, aE, k))
        per_node[k] = float(np.sum(pix * A * B * B))
        per_abs[k] = float(np.sum(pix * np.abs(A) * B * B))
    rad = np.asarray(w, dtype=np.float64) * np.asarray(r, dtype=np.float64) ** 2
    return {"S": float(np.sum(rad * per_node)), "S_abs": float(np.sum(rad * per_abs)),
            "per_node": per_node}


def sky_integral_gaunt(L, A, B):
    """int A B^2 dOmega from the harmonic coefficients alone, by the exact
    Gaunt sum of oracle/gaunt.py: sum_lm c_m Re(conj(A_lm) [B^2]_lm)."""
    from . import gaunt
    sq = np.array(gaunt.square_coeffs(B, L))
    A = np.asarray(A, dtype=np.complex128).copy()
    ls = np.repeat(np.arange(L + 1), np.arange(1, L + 2))
    ms = np.arange(ls.size) - ls * (ls + 1) // 2
    A[ms == 0] = A[ms == 0].real
    c = np.where(ms == 0, 1.0, 2.0)
    return float(np.sum(c * (np.conj(A) * sq).real))
