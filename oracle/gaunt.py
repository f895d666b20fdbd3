"""Brute-force Phi_NL from Gaunt integrals (test infrastructure only).

For a real band-limited field Phi = sum_{l,m} Phi_lm Y_lm (all m, with
Phi_{l,-m} = (-1)^m conj(Phi_lm)), the harmonic coefficients of its square are

    [Phi^2]_lm = sum_{l1 m1 l2 m2} Phi_l1m1 Phi_l2m2  int Y_l1m1 Y_l2m2 Y*_lm dOmega,

    int Y_l1m1 Y_l2m2 Y*_lm = (-1)^m sqrt((2l1+1)(2l2+1)(2l+1)/(4 pi))
                              (l1 l2 l; 0 0 0) (l1 l2 l; m1 m2 -m).

Phi_NL = Phi^2 - <Phi^2> (Eq. phinldef) differs from [Phi^2] only at l = 0.
The Wigner 3j symbols come from Racah's closed formula evaluated in exact
rational arithmetic (the square root is taken once, at the end), so this is
the plain algebraic definition with no quadrature at all.  The prefactor is
the I_{l1 l2 l3} of the bispectrum normalisation in Sect. 4 (Eq. fast_est).
"""
import math
from fractions import Fraction
from functools import lru_cache


@lru_cache(maxsize=None)
def _fact(n):
    return math.factorial(n)


@lru_cache(maxsize=None)
def wigner3j_exact(j1, j2, j3, m1, m2, m3):
    """(sign * S, P) with 3j = sign*S*sqrt(P), S and P exact Fractions."""
    if m1 + m2 + m3 != 0:
        return Fraction(0), Fraction(0)
    if j3 < abs(j1 - j2) or j3 > j1 + j2:
        return Fraction(0), Fraction(0)
    if abs(m1) > j1 or abs(m2) > j2 or abs(m3) > j3:
        return Fraction(0), Fraction(0)
    delta = Fraction(_fact(j1 + j2 - j3) * _fact(j1 - j2 + j3) * _fact(-j1 + j2 + j3),
                     _fact(j1 + j2 + j3 + 1))
    pre = delta * (_fact(j1 + m1) * _fact(j1 - m1) * _fact(j2 + m2) * _fact(j2 - m2)
                   * _fact(j3 + m3) * _fact(j3 - m3))
    kmin = max(0, j2 - j3 - m1, j1 - j3 + m2)
    kmax = min(j1 + j2 - j3, j1 - m1, j2 + m2)
    s = Fraction(0)
    for k in range(kmin, kmax + 1):
        den = (_fact(k) * _fact(j3 - j2 + k + m1) * _fact(j3 - j1 + k - m2)
               * _fact(j1 + j2 - j3 - k) * _fact(j1 - k - m1) * _fact(j2 - k + m2))
        s += Fraction((-1) ** k, den)
    sign = -1 if (j1 - j2 - m3) % 2 else 1
    return sign * s, pre


def wigner3j(j1, j2, j3, m1, m2, m3):
    s, p = wigner3j_exact(j1, j2, j3, m1, m2, m3)
    if s == 0:
        return 0.0
    return float(s) * math.sqrt(float(p))


@lru_cache(maxsize=None)
def gaunt(l1, m1, l2, m2, l, m):
    """int Y_l1m1 Y_l2m2 Y*_lm dOmega, evaluated exactly then rounded once."""
    if m1 + m2 != m or (l1 + l2 + l) % 2:
        return 0.0
    s0, p0 = wigner3j_exact(l1, l2, l, 0, 0, 0)
    s1, p1 = wigner3j_exact(l1, l2, l, m1, m2, -m)
    if s0 == 0 or s1 == 0:
        return 0.0
    sq = p0 * p1 * (2 * l1 + 1) * (2 * l2 + 1) * (2 * l + 1)
    val = float(s0 * s1) * math.sqrt(float(sq)) / math.sqrt(4.0 * math.pi)
    return -val if m % 2 else val


def _full(alm, L):
    """Phi_lm for all -l <= m <= l from the m >= 0 half (real field)."""
    d = {}
    for l in range(L + 1):
        for m in range(l + 1):
            v = complex(alm[l * (l + 1) // 2 + m])
            if m == 0:
                v = complex(v.real, 0.0)
            d[(l, m)] = v
            if m > 0:
                d[(l, -m)] = (-1) ** m * v.conjugate()
    return d


def square_coeffs(alm, L, lout=None):
    """[Phi^2]_lm for 0 <= m <= l <= lout (default L) by the Gaunt sum."""
    lout = L if lout is None else lout
    full = _full(alm, L)
    out = []
    for l in range(lout + 1):
        for m in range(l + 1):
            acc = 0j
            for l1 in range(L + 1):
                for l2 in range(abs(l - l1), min(L, l + l1) + 1):
                    if (l1 + l2 + l) % 2:
                        continue
                    for m1 in range(-l1, l1 + 1):
                        m2 = m - m1
                        if abs(m2) > l2:
                            continue
                        g = gaunt(l1, m1, l2, m2, l, m)
                        if g:
                            acc += full[(l1, m1)] * full[(l2, m2)] * g
            out.append(acc)
    return out


def phi_nl_sample(alm, L):
    """Phi_NL with the sky-mean subtraction: the square's (0,0) term removed."""
    sq = square_coeffs(alm, L)
    sq[0] = 0j
    return sq


def wigner3j_float(j1, j2, j3, m1, m2, m3):
    """The same Racah formula in FP64: log-factorials (lgamma) for every
    factor, the alternating sum added exactly-rounded (math.fsum).  For the
    brute force at l ~ 32, where exact rationals get slow; checked against
    wigner3j_exact at small l."""
    if m1 + m2 + m3 != 0 or j3 < abs(j1 - j2) or j3 > j1 + j2:
        return 0.0
    if abs(m1) > j1 or abs(m2) > j2 or abs(m3) > j3:
        return 0.0
    lf = lambda n: math.lgamma(n + 1.0)
    half = 0.5 * (lf(j1 + j2 - j3) + lf(j1 - j2 + j3) + lf(-j1 + j2 + j3) - lf(j1 + j2 + j3 + 1)
                  + lf(j1 + m1) + lf(j1 - m1) + lf(j2 + m2) + lf(j2 - m2) + lf(j3 + m3) + lf(j3 - m3))
    kmin = max(0, j2 - j3 - m1, j1 - j3 + m2)
    kmax = min(j1 + j2 - j3, j1 - m1, j2 + m2)
    terms = []
    for k in range(kmin, kmax + 1):
        lg = half - (lf(k) + lf(j3 - j2 + k + m1) + lf(j3 - j1 + k - m2) + lf(j1 + j2 - j3 - k)
                     + lf(j1 - k - m1) + lf(j2 - k + m2))
        terms.append((-1.0) ** k * math.exp(lg))
    sign = -1.0 if (j1 - j2 - m3) % 2 else 1.0
    return sign * math.fsum(terms)


@lru_cache(maxsize=None)
def gaunt_float(l1, m1, l2, m2, l, m):
    """int Y_l1m1 Y_l2m2 Y*_lm dOmega with wigner3j_float."""
    if m1 + m2 != m or (l1 + l2 + l) % 2:
        return 0.0
    w0 = wigner3j_float(l1, l2, l, 0, 0, 0)
    if w0 == 0.0:
        return 0.0
    w1 = wigner3j_float(l1, l2, l, m1, m2, -m)
    val = math.sqrt((2 * l1 + 1) * (2 * l2 + 1) * (2 * l + 1) / (4.0 * math.pi)) * w0 * w1
    return -val if m % 2 else val


def square_coeffs_float(alm, L, outputs):
    """[Phi^2]_lm at the listed (l, m) outputs, by the Gaunt sum in FP64."""
    full = _full(alm, L)
    out = []
    for l, m in outputs:
        acc = 0j
        for l1 in range(L + 1):
            for l2 in range(abs(l - l1), min(L, l + l1) + 1):
                if (l1 + l2 + l) % 2:
                    continue
                for m1 in range(-l1, l1 + 1):
                    m2 = m - m1
                    if abs(m2) > l2:
                        continue
                    gv = gaunt_float(l1, m1, l2, m2, l, m)
                    if gv:
                        acc += full[(l1, m1)] * full[(l2, m2)] * gv
        out.append(acc)
    return out
