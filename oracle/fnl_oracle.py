"""ctypes binding of the FP64 CPU oracle (test infrastructure only).

Arrays are numpy; complex coefficient arrays are complex128 in the alm order
idx(l, m) = l(l+1)/2 + m.  See fnl_oracle.h for the conventions.
"""
import ctypes
import math

import numpy as np

from . import build as _build

MEAN_SAMPLE = 0
MEAN_ENSEMBLE = 1

_lib = None


class _Problem(ctypes.Structure):
    _fields_ = [("lmax", ctypes.c_int), ("nshell", ctypes.c_int),
                ("ntheta", ctypes.c_int), ("nphi", ctypes.c_int),
                ("mean_mode", ctypes.c_int),
                ("r", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("filter", ctypes.c_void_p), ("alpha", ctypes.c_void_p),
                ("beta", ctypes.c_void_p)]


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(_build.ensure_built())
        vp, ip, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        _lib.orc_gl_grid.argtypes = [ip, vp, vp]
        _lib.orc_gl_grid.restype = ip
        _lib.orc_lambda_all.argtypes = [ip, dp, vp]
        _lib.orc_lambda_all.restype = None
        _lib.orc_synth.argtypes = [ip, ip, ip, vp, vp, vp]
        _lib.orc_synth.restype = None
        _lib.orc_anal.argtypes = [ip, ip, ip, vp, vp, vp, vp]
        _lib.orc_anal.restype = None
        _lib.orc_filter.argtypes = [ctypes.POINTER(_Problem), vp, vp]
        _lib.orc_filter.restype = None
        _lib.orc_forward.argtypes = [ctypes.POINTER(_Problem), vp, dp] + [vp] * 9
        _lib.orc_forward.restype = ip
        _lib.orc_adjoint.argtypes = [ctypes.POINTER(_Problem), vp, dp, vp, vp, vp, vp]
        _lib.orc_philox4x32_10.argtypes = [vp, vp, vp]
        _lib.orc_philox4x32_10.restype = None
        _lib.orc_noise.argtypes = [ip, ip, ctypes.c_ulonglong, vp]
        _lib.orc_noise.restype = None
        _lib.orc_adjoint.restype = ip
        _lib.orc_spin_lambda.argtypes = [ip, ip, ip, dp, vp]
        _lib.orc_spin_lambda.restype = None
        _lib.orc_synth_qu.argtypes = [ip, ip, ip, vp, vp, vp, vp]
        _lib.orc_synth_qu.restype = None
    return _lib


def nlm(L):
    return (L + 1) * (L + 2) // 2


def _ptr(a):
    return None if a is None else a.ctypes.data


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def default_ntheta(L):
    """Smallest ring count that integrates a product of three band-L fields."""
    return (3 * L + 2) // 2


def default_nphi(L):
    """3L+1 pixels per ring: the square of a band-L field is not aliased."""
    return 3 * L + 1


def gl_grid(n):
    x = np.empty(n)
    w = np.empty(n)
    if lib().orc_gl_grid(n, _ptr(x), _ptr(w)) != 0:
        raise ValueError("bad order")
    return x, w


def lambda_all(L, x):
    out = np.empty(nlm(L))
    lib().orc_lambda_all(L, float(x), _ptr(out))
    return out


def synth(L, ntheta, nphi, alm):
    x, _ = gl_grid(ntheta)
    alm = _c128(alm)
    out = np.empty((ntheta, nphi))
    lib().orc_synth(L, ntheta, nphi, _ptr(x), _ptr(alm), _ptr(out))
    return out


def spin_lambda(L, m, s, x):
    """sl_lm(x) for l = 0..L (spin-weighted Legendre functions, one m and s)."""
    out = np.empty(L + 1)
    lib().orc_spin_lambda(int(L), int(m), int(s), float(x), _ptr(out))
    return out


def synth_qu(L, x, nphi, almE):
    """Stokes Q, U maps [len(x)][nphi] of a pure-E field on the rings x."""
    x = _f64(x)
    almE = _c128(almE)
    Q = np.empty((x.size, nphi))
    U = np.empty((x.size, nphi))
    lib().orc_synth_qu(int(L), x.size, int(nphi), _ptr(x), _ptr(almE), _ptr(Q), _ptr(U))
    return Q, U


def synth_rings(L, x, nphi, alm):
    """Scalar synthesis on an arbitrary ring list x (orc_synth)."""
    x = _f64(x)
    alm = _c128(alm)
    out = np.empty((x.size, nphi))
    lib().orc_synth(int(L), x.size, int(nphi), _ptr(x), _ptr(alm), _ptr(out))
    return out


def anal(L, ntheta, nphi, m):
    x, w = gl_grid(ntheta)
    m = _f64(m)
    assert m.shape == (ntheta, nphi)
    out = np.empty(nlm(L), dtype=np.complex128)
    lib().orc_anal(L, ntheta, nphi, _ptr(x), _ptr(w), _ptr(m), _ptr(out))
    return out


class Problem:
    """Inputs of one map generator (r, w, filter, alpha, beta) plus the grid."""

    def __init__(self, lmax, r, w, filt, alpha, beta, ntheta=None, nphi=None,
                 mean_mode=MEAN_SAMPLE):
        self.lmax = int(lmax)
        self.r = _f64(r)
        self.w = _f64(w)
        self.nshell = self.r.shape[0]
        self.filter = _f64(filt)
        self.alpha = _f64(alpha)
        self.beta = _f64(beta)
        N, L = self.nshell, self.lmax
        assert self.filter.shape == (L + 1, N, N)
        assert self.alpha.shape == (L + 1, N) and self.beta.shape == (L + 1, N)
        self.ntheta = default_ntheta(L) if ntheta is None else int(ntheta)
        self.nphi = default_nphi(L) if nphi is None else int(nphi)
        self.mean_mode = int(mean_mode)

    def _struct(self):
        return _Problem(self.lmax, self.nshell, self.ntheta, self.nphi, self.mean_mode,
                        _ptr(self.r), _ptr(self.w), _ptr(self.filter),
                        _ptr(self.alpha), _ptr(self.beta))

    def filter_apply(self, noise):
        noise = _c128(noise)
        out = np.empty((self.nshell, nlm(self.lmax)), dtype=np.complex128)
        st = self._struct()
        lib().orc_filter(ctypes.byref(st), _ptr(noise), _ptr(out))
        return out

    def forward(self, noise, fnl, want_phi=False, want_mu=False):
        """Return a dict with aT, aE, aT_lin, aE_lin, aT_nl, aE_nl (and phiL,
        phiNL, mu on request)."""
        L, N = self.lmax, self.nshell
        noise = _c128(noise)
        assert noise.shape == (N, nlm(L))
        outs = {k: np.empty(nlm(L), dtype=np.complex128)
                for k in ("aT", "aE", "aT_lin", "aE_lin", "aT_nl", "aE_nl")}
        phiL = np.empty((N, nlm(L)), dtype=np.complex128) if want_phi else None
        phiNL = np.empty((N, nlm(L)), dtype=np.complex128) if want_phi else None
        mu = np.empty(N) if want_mu else None
        st = self._struct()
        rc = lib().orc_forward(ctypes.byref(st), _ptr(noise), float(fnl),
                               _ptr(outs["aT"]), _ptr(outs["aE"]),
                               _ptr(outs["aT_lin"]), _ptr(outs["aE_lin"]),
                               _ptr(outs["aT_nl"]), _ptr(outs["aE_nl"]),
                               _ptr(phiL), _ptr(phiNL), _ptr(mu))
        if rc != 0:
            raise ValueError("oracle forward rejected its arguments")
        if want_phi:
            outs["phiL"], outs["phiNL"] = phiL, phiNL
        if want_mu:
            outs["mu"] = mu
        return outs

    def adjoint(self, noise, fnl, gT, gE):
        L, N = self.lmax, self.nshell
        noise, gT, gE = _c128(noise), _c128(gT), _c128(gE)
        gn = np.empty((N, nlm(L)), dtype=np.complex128)
        gf = np.zeros(1)
        st = self._struct()
        rc = lib().orc_adjoint(ctypes.byref(st), _ptr(noise), float(fnl), _ptr(gT), _ptr(gE),
                               _ptr(gn), _ptr(gf))
        if rc != 0:
            raise ValueError("oracle adjoint rejected its arguments")
        return gn, float(gf[0])


def radial_weights(problem):
    """W^X_li = w_i r_i^2 X_l(r_i) (quadrature form of Eq. phi2alm_r)."""
    base = problem.w * problem.r ** 2
    return problem.alpha * base[None, :], problem.beta * base[None, :]


SQRT4PI = math.sqrt(4.0 * math.pi)


def philox4x32_10(ctr, key):
    """Philox4x32-10 of a 4-word counter under a 2-word key -> 4 words."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty(4, dtype=np.uint32)
    lib().orc_philox4x32_10(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def seeded_noise(L, N, seed):
    """Counter-based noise [N][n_lm] complex128 of one realization seed
    (definition in fnl_oracle.h, orc_noise)."""
    out = np.empty((N, nlm(L)), dtype=np.complex128)
    lib().orc_noise(int(L), int(N), int(seed), out.ctypes.data)
    return out
