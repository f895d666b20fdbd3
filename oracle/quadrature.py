"""Plain FP64 oracle of the optimal radial quadrature of Sect. 3.

TEST INFRASTRUCTURE ONLY (like the rest of oracle/): it states what an
implementation of the quadrature design must compute, in numpy, step by step.

For one multipole and one transfer table, the line-of-sight integral
I = int dr r^2 alpha(r) Phi(r) (Eq. los_int) is first a fine sum
I = sum_k a_k Phi(r_k) over N_tot shells, a_k = fine quadrature weight *
r_k^2 alpha(r_k).  A coarse estimate uses N of those shells with weights w:
I_hat = sum_i w_i Phi(r_{s_i}).  With C the covariance of Phi on the fine
grid (Eq. cov_phi), the expected quadratic error (Eq. mean_err) is

    E(w) = a^T C a - 2 w^T (C a)_S + w^T C_SS w,

where a^T C a = sum_k lambda_k (a^T phi_k)^2 over the eigenpairs of C, the
paper's first term.  Setting dE/dw = 0 gives the linear system
C_SS w = (C a)_S (the paper's optimal-weight equations), and there
E = a^T C a - w^T C_SS w, the paper's form of Eq. mean_err.  The greedy
design adds, one node at a time, the fine shell that most lowers the sum of
the optimal errors over all problems (multipoles, and T and E with equal
weights).
"""
import numpy as np


def trapezoid_weights(r):
    """Trapezoid weights of a sorted grid (the fine sum's dr)."""
    r = np.asarray(r, dtype=np.float64)
    w = np.zeros_like(r)
    if r.size > 1:
        d = np.diff(r)
        w[:-1] += 0.5 * d
        w[1:] += 0.5 * d
    return w


def fine_weights(r, alpha):
    """a_k = dr_k r_k^2 alpha(r_k): the fine-grid form of Eq. los_int."""
    r = np.asarray(r, dtype=np.float64)
    return trapezoid_weights(r) * r * r * np.asarray(alpha, dtype=np.float64)


def expected_error(C, a, nodes, w):
    """E(w) = a^T C a - 2 w^T (C a)_S + w^T C_SS w (Eq. mean_err for any w)."""
    C = np.asarray(C, dtype=np.float64)
    a = np.asarray(a, dtype=np.float64)
    S = np.asarray(nodes, dtype=np.int64)
    w = np.asarray(w, dtype=np.float64)
    Ca = C @ a
    return float(a @ Ca - 2.0 * (w @ Ca[S]) + w @ C[np.ix_(S, S)] @ w)


def expected_error_eigen(C, a, nodes, w):
    """The same error written with the eigenpairs (lambda_k, phi_k) of C, as
    the paper does: sum_k lambda_k (a^T phi_k - w^T phi_k[S])^2."""
    lam, phi = np.linalg.eigh(np.asarray(C, dtype=np.float64))
    S = np.asarray(nodes, dtype=np.int64)
    proj = np.asarray(a, dtype=np.float64) @ phi - np.asarray(w, dtype=np.float64) @ phi[S, :]
    return float(np.sum(lam * proj * proj))


def optimal_weights(C, a, nodes):
    """Solve C_SS w = (C a)_S (the condition dE/dw_i = 0) by a symmetric
    eigendecomposition of C_SS: eigenvalues at or below 1e-14 of the largest
    are left out (a least-squares solution), so a set whose covariance is
    singular up to rounding still gives finite weights."""
    C = np.asarray(C, dtype=np.float64)
    S = np.asarray(nodes, dtype=np.int64)
    rhs = (C @ np.asarray(a, dtype=np.float64))[S]
    lam, U = np.linalg.eigh(C[np.ix_(S, S)])
    keep = lam > 1e-14 * max(float(lam.max()), 0.0)
    return U[:, keep] @ ((U[:, keep].T @ rhs) / lam[keep])


def optimal_error(C, a, nodes):
    """E at the optimal weights: a^T C a - w^T C_SS w."""
    C = np.asarray(C, dtype=np.float64)
    a = np.asarray(a, dtype=np.float64)
    S = np.asarray(nodes, dtype=np.int64)
    if S.size == 0:
        return float(a @ C @ a)
    w = optimal_weights(C, a, S)
    return float(a @ C @ a - w @ C[np.ix_(S, S)] @ w)


# A shell whose variance conditional on the nodes already chosen is at most
# DEPENDENT_TOL times its own variance C_jj carries no information the set
# does not already hold (on a fine grid spaced well below the correlation
# length this happens after a few dozen nodes): it adds nothing to that
# problem, and its weight there is 0.
DEPENDENT_TOL = 1e-10


def conditional_variance(C, basis, j):
    """d_j = C_jj - C_jB C_BB^{-1} C_Bj for the shells B already in use."""
    C = np.asarray(C, dtype=np.float64)
    if len(basis) == 0:
        return float(C[j, j])
    B = np.asarray(basis, dtype=np.int64)
    c = C[B, j]
    return float(C[j, j] - c @ np.linalg.solve(C[np.ix_(B, B)], c))


def effective_sets(problems, nodes):
    """Replay a node order: for each problem, the nodes that were not
    dependent (conditional variance above DEPENDENT_TOL C_jj) when added."""
    out = []
    for C, _ in problems:
        B = []
        for j in nodes:
            if conditional_variance(C, B, j) > DEPENDENT_TOL * float(np.asarray(C)[j, j]):
                B.append(int(j))
        out.append(B)
    return out


def design_errors(problems, nodes):
    """Summed optimal error after each step of a given node order, each
    problem using only its effective nodes (recomputed from scratch at every
    step with the eigendecomposition solve)."""
    errs = []
    for k in range(1, len(nodes) + 1):
        sets = effective_sets(problems, nodes[:k])
        errs.append(sum(optimal_error(C, a, B) for (C, a), B in zip(problems, sets)))
    return errs


def design_weights(problems, nodes):
    """[P][n] optimal weights of a node order: each problem's weights solve its
    effective set's system; dependent nodes get weight 0."""
    sets = effective_sets(problems, nodes)
    W = np.zeros((len(problems), len(nodes)))
    for p, ((C, a), B) in enumerate(zip(problems, sets)):
        if B:
            wB = optimal_weights(C, a, B)
            for w, j in zip(wB, B):
                W[p, list(nodes).index(j)] = w
    return W


def greedy_nodes(problems, n):
    """Greedy node design.  problems: list of (C, a) pairs on one fine grid
    (one per multipole and transfer table; T and E enter with equal weight).
    Returns (nodes in the order chosen, total optimal error after each
    step).  Each step tries every fine shell not yet chosen and keeps the
    one whose addition leaves the smallest summed error (the lowest index
    among equal ones); in a problem where the shell is dependent on that
    problem's nodes (see DEPENDENT_TOL) it changes nothing."""
    ntot = np.asarray(problems[0][0]).shape[0]
    chosen, errors = [], []
    basis = [[] for _ in problems]
    for _ in range(n):
        best, best_err = -1, np.inf
        for j in range(ntot):
            if j in chosen:
                continue
            err = 0.0
            for (C, a), B in zip(problems, basis):
                indep = conditional_variance(C, B, j) > DEPENDENT_TOL * float(np.asarray(C)[j, j])
                err += optimal_error(C, a, B + [j] if indep else B)
            if err < best_err:
                best, best_err = j, err
        chosen.append(best)
        errors.append(best_err)
        for p, (C, a) in enumerate(problems):
            if conditional_variance(C, basis[p], best) > DEPENDENT_TOL * float(np.asarray(C)[best, best]):
                basis[p].append(best)
    return chosen, errors
