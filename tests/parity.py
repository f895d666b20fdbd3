"""Error metric shared by the GPU parity tests.

err_l = sqrt(sum_m c_m |a - ref|^2) / sqrt(sum_m c_m |ref|^2), c_0 = 1, c_m = 2,
evaluated per multipole for each output separately.  Multipoles whose
reference power is zero up to rounding (E at l < 2; the sample-mean-removed
Phi_NL,00) are checked absolutely against the largest per-l reference norm.
"""
import numpy as np


def per_l_errors(a, ref, L):
    a = np.asarray(a).reshape(-1)
    ref = np.asarray(ref).reshape(-1)
    ls = np.repeat(np.arange(L + 1), np.arange(1, L + 2))
    ms = np.arange(ls.size) - ls * (ls + 1) // 2
    c = np.where(ms == 0, 1.0, 2.0)
    num = np.sqrt(np.bincount(ls, weights=c * np.abs(a - ref) ** 2, minlength=L + 1))
    den = np.sqrt(np.bincount(ls, weights=c * np.abs(ref) ** 2, minlength=L + 1))
    scale = den.max() if den.max() > 0 else 1.0
    zero = den <= 1e-12 * scale
    err = np.where(zero, num / scale, num / np.where(zero, 1.0, den))
    return err


def max_rel_err(a, ref, L):
    return float(per_l_errors(a, ref, L).max())


def assert_close(a, ref, L, tol, what=""):
    e = per_l_errors(a, ref, L)
    worst = int(np.argmax(e))
    assert e[worst] <= tol, f"{what}: max per-l relative rms error {e[worst]:.3e} at l={worst} > {tol}"
    return float(e[worst])
