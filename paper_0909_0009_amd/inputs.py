"""Seeded synthetic inputs for the local-f_NL map generator.

This module only *builds inputs*: radial nodes and weights, the radial filter
(a square root of the potential's radial covariance, Sect. 2, Eq. cov_phi),
synthetic transfer tables and white noise.  It holds none of the map
generator's arithmetic (filter application, transforms, square, radial sum)
and is shared by the oracle tests and the HIP path alike.

The paper's inputs come from CAMB (WMAP5+BAO+SN transfer functions, 70
optimised nodes; Sect. 3).  Those are not available here, so the stand-ins
have the same shapes and structure:

* nodes r_i uniform in [13000, 15000] Mpc, trapezoid weights;
* covariance C_l(r_i, r_j) = (2/pi) int dk k^2 P(k) j_l(k r_i) j_l(k r_j) with
  P(k) = A k^-3 (k/0.05)^(ns-1), A = 1.7e-8, ns = 0.96 on k in [1e-5, 0.2]
  (4096 log-spaced nodes, trapezoid rule in ln k).  This is Eq. cov_phi:
  4 pi Delta^2(k)/k = (2/pi) k^2 P(k);
* filter F_l = Cholesky(C_l + 1e-12 max diag(C_l) I), lower triangular (the
  paper's P^{1/2}; the jitter keeps N = 200 numerically positive definite);
* transfer tables alpha_l(r), beta_l(r): a Gaussian in r (centre 14000 Mpc,
  width 150 Mpc) times a seeded smooth l-envelope; beta_0 = beta_1 = 0;
* noise n_lm(r_j): complex unit Gaussian (E|n|^2 = 1), real for m = 0.
"""
import hashlib
import math
import os

import numpy as np

# --------------------------------------------------------------- configs

CONFIGS = {
    # plain method, tiny
    "tiny": dict(lmax=32, nshell=16, ntheta=49, nphi=128, fnl=100.0),
    # plain method, medium
    "medium": dict(lmax=256, nshell=64, ntheta=385, nphi=768, fnl=100.0),
    # paper scale: lmax 1024 with 200 nodes
    "paper": dict(lmax=1024, nshell=200, ntheta=1537, nphi=3072, fnl=100.0),
    # differentiation workload
    "grad": dict(lmax=512, nshell=96, ntheta=769, nphi=1536, fnl=100.0),
}

BATCH_LMAX_CHOICES = (128, 256, 512, 1024)

TRANSFER_SEED = 7
NOISE_SEED_BASE = 1000
TARGET_SEED = 2
BATCH_SEED = 33


def nlm(L):
    return (L + 1) * (L + 2) // 2


def min_ntheta(L):
    """ceil((3L+1)/2): rings needed to integrate a cubic product exactly."""
    return (3 * L + 2) // 2


def batch_mix(count=32, seed=BATCH_SEED):
    """(lmax, nshell) per realization of the uneven batching workload."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        L = int(rng.choice(BATCH_LMAX_CHOICES))
        N = int(rng.integers(64, 201))
        out.append((L, N))
    return out


def lm_arrays(L):
    """l and m of every coefficient in the order idx = l(l+1)/2 + m."""
    ls = np.repeat(np.arange(L + 1), np.arange(1, L + 2))
    ms = np.arange(nlm(L)) - ls * (ls + 1) // 2
    return ls, ms


# ------------------------------------------------------------ radial grid

def radial_nodes(N, rmin=13000.0, rmax=15000.0):
    """Uniform nodes, inclusive, with trapezoid weights."""
    r = np.linspace(rmin, rmax, N)
    if N == 1:
        return r, np.ones(1)
    h = (rmax - rmin) / (N - 1)
    w = np.full(N, h)
    w[0] = w[-1] = 0.5 * h
    return r, w


# ------------------------------------------------ spherical Bessel table

def sph_bessel_table(L, x):
    """j_l(x) for l = 0..L at every x > 0 (1-D), shape [L+1, x.size].

    For x > L + 60 the upward recurrence from j_0, j_1 is stable over l <= L.
    Otherwise Miller's downward recurrence is used, started at
    l = max(x) + 60 + 8 max(x)^(1/3) (beyond which j_l is below 1e-30 of its
    peak) but not above L + 200, with rescaling against overflow and
    normalisation by the identity sum_l (2l+1) j_l(x)^2 = 1; the sign is taken
    from whichever of j_0, j_1 is larger in magnitude.
    """
    x = np.asarray(x, dtype=np.float64).ravel()
    out = np.zeros((L + 1, x.size))
    up = x > L + 60.0
    if np.any(up):
        xs = x[up]
        j0 = np.sin(xs) / xs
        j1 = np.sin(xs) / xs ** 2 - np.cos(xs) / xs
        out[0, up] = j0
        if L >= 1:
            out[1, up] = j1
        jm, jc = j0, j1
        for l in range(1, L):
            jn = (2 * l + 1) / xs * jc - jm
            out[l + 1, up] = jn
            jm, jc = jc, jn
    dn = ~up
    if np.any(dn):
        xs = x[dn]
        Ls = max(L, 1)                      # keep j_1 for the sign test
        xmax = float(np.max(xs))
        top = int(min(Ls + 200, xmax + 60 + 8 * xmax ** (1 / 3)))
        top = max(top, 2)
        t_next = np.zeros_like(xs)          # t_{l+1}
        t_cur = np.full_like(xs, 1e-100)    # t_l at l = top
        scale = np.zeros(xs.size, dtype=np.int64)
        stored = np.zeros((Ls + 1, xs.size))
        stored_scale = np.zeros((Ls + 1, xs.size), dtype=np.int64)
        norm = (2 * top + 1) * t_cur ** 2
        for l in range(top, 0, -1):
            t_prev = (2 * l + 1) / xs * t_cur - t_next   # t_{l-1}
            t_next, t_cur = t_cur, t_prev
            norm = norm + (2 * l - 1) * t_cur ** 2
            big = np.abs(t_cur) > 1e120
            if np.any(big):
                t_cur = np.where(big, t_cur * 1e-120, t_cur)
                t_next = np.where(big, t_next * 1e-120, t_next)
                norm = np.where(big, norm * 1e-240, norm)
                scale = scale + big
            if l - 1 <= Ls:
                stored[l - 1] = t_cur
                stored_scale[l - 1] = scale
        # bring every stored value to the final scale; two or more rescales
        # later it is below 1e-240 of the peak and is dropped
        lag = scale[None, :] - stored_scale
        stored *= np.where(lag == 0, 1.0, np.where(lag == 1, 1e-120, 0.0))
        mag = 1.0 / np.sqrt(norm)
        j0 = np.sin(xs) / xs
        j1 = np.sin(xs) / xs ** 2 - np.cos(xs) / xs
        use0 = np.abs(j0) >= np.abs(j1)
        sign = np.sign(np.where(use0, j0 * stored[0], j1 * stored[1]))
        sign[sign == 0] = 1.0
        out[:, dn] = stored[:L + 1] * (mag * sign)[None, :]
    return out


# ------------------------------------------------------------- covariance

# The k quadrature is summed in KGROUPS fixed contiguous groups of k chunks,
# each group in order, then the group sums in order: the result does not
# depend on how many worker threads evaluate the groups.
KGROUPS = 8


def _cov_group(L, r, k, D, q0s, kchunk):
    N = r.size
    C = np.zeros((L + 1, N, N))
    for q0 in q0s:
        kc = k[q0:q0 + kchunk]
        x = np.outer(r, kc)                       # [N, kc]
        J = sph_bessel_table(L, x.ravel()).reshape(L + 1, N, kc.size)
        JD = J * D[q0:q0 + kchunk][None, None, :]
        C += np.matmul(JD, J.transpose(0, 2, 1))
    return C


def _cov_group_task(args):
    return _cov_group(*args)


def input_workers():
    """Worker threads for input generation (FNLSIM_INPUT_WORKERS, else the
    usable cores, at most KGROUPS)."""
    env = os.environ.get("FNLSIM_INPUT_WORKERS")
    if env:
        return max(1, int(env))
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    return max(1, min(KGROUPS, ncpu))


def covariance(L, r, A=1.7e-8, ns=0.96, kmin=1e-5, kmax=0.2, nk=4096, kchunk=64, workers=None):
    """C_l(r_i, r_j) for l = 0..L, shape [L+1, N, N] (Eq. cov_phi)."""
    r = np.asarray(r, dtype=np.float64)
    k = np.geomspace(kmin, kmax, nk)
    h = math.log(kmax / kmin) / (nk - 1)
    dlnk = np.full(nk, h)
    dlnk[0] = dlnk[-1] = 0.5 * h
    # dk k^2 P(k) = dlnk * A (k/0.05)^(ns-1);  prefactor 2/pi
    D = (2.0 / math.pi) * A * (k / 0.05) ** (ns - 1.0) * dlnk
    starts = list(range(0, nk, kchunk))
    per = -(-len(starts) // KGROUPS)
    groups = [starts[g * per:(g + 1) * per] for g in range(KGROUPS)]
    groups = [g for g in groups if g]
    tasks = [(L, r, k, D, g, kchunk) for g in groups]
    workers = input_workers() if workers is None else workers
    # threads (numpy releases the GIL inside its array loops); every matmul
    # runs on one BLAS thread, so the sums do not depend on the thread count
    import concurrent.futures

    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1, user_api="blas"):
        if workers > 1 and len(tasks) > 1:
            with concurrent.futures.ThreadPoolExecutor(min(workers, len(tasks))) as ex:
                parts = list(ex.map(_cov_group_task, tasks))
        else:
            parts = [_cov_group_task(t) for t in tasks]
    C = parts[0]
    for P in parts[1:]:
        C += P
    return C


def _sph_bessel_table_torch(L, x):
    """sph_bessel_table with torch FP64 tensors on the tensor's device: the
    same upward / Miller downward recurrences, normalisation and sign rule."""
    import torch
    out = torch.zeros((L + 1, x.numel()), dtype=torch.float64, device=x.device)
    up = x > L + 60.0
    if bool(up.any()):
        xs = x[up]
        j0 = torch.sin(xs) / xs
        j1 = torch.sin(xs) / xs ** 2 - torch.cos(xs) / xs
        rows = [j0] + ([j1] if L >= 1 else [])
        jm, jc = j0, j1
        for l in range(1, L):
            jn = (2 * l + 1) / xs * jc - jm
            rows.append(jn)
            jm, jc = jc, jn
        out[:, up] = torch.stack(rows[:L + 1])
    dn = ~up
    if bool(dn.any()):
        xs = x[dn]
        Ls = max(L, 1)
        xmax = float(xs.max())
        top = max(int(min(Ls + 200, xmax + 60 + 8 * xmax ** (1 / 3))), 2)
        t_next = torch.zeros_like(xs)
        t_cur = torch.full_like(xs, 1e-100)
        scale = torch.zeros(xs.numel(), dtype=torch.int64, device=x.device)
        stored = torch.zeros((Ls + 1, xs.numel()), dtype=torch.float64, device=x.device)
        stored_scale = torch.zeros((Ls + 1, xs.numel()), dtype=torch.int64, device=x.device)
        norm = (2 * top + 1) * t_cur ** 2
        for l in range(top, 0, -1):
            t_prev = (2 * l + 1) / xs * t_cur - t_next
            t_next, t_cur = t_cur, t_prev
            norm = norm + (2 * l - 1) * t_cur ** 2
            big = t_cur.abs() > 1e120
            # rescale where needed (a no-op elsewhere; no host sync per step)
            f = torch.where(big, torch.full_like(t_cur, 1e-120), torch.ones_like(t_cur))
            t_cur = t_cur * f
            t_next = t_next * f
            norm = norm * f * f
            scale = scale + big.to(torch.int64)
            if l - 1 <= Ls:
                stored[l - 1] = t_cur
                stored_scale[l - 1] = scale
        lag = scale[None, :] - stored_scale
        one = torch.ones_like(stored)
        stored = stored * torch.where(lag == 0, one, torch.where(lag == 1, 1e-120 * one, 0.0 * one))
        mag = 1.0 / torch.sqrt(norm)
        j0 = torch.sin(xs) / xs
        j1 = torch.sin(xs) / xs ** 2 - torch.cos(xs) / xs
        use0 = j0.abs() >= j1.abs()
        sign = torch.sign(torch.where(use0, j0 * stored[0], j1 * stored[1]))
        sign[sign == 0] = 1.0
        out[:, dn] = stored[:L + 1] * (mag * sign)[None, :]
    return out


def covariance_torch(L, r, device, A=1.7e-8, ns=0.96, kmin=1e-5, kmax=0.2, nk=4096, kchunk=1024,
                     as_tensor=False):
    """covariance() evaluated with torch FP64 on `device` (a GPU makes the
    paper-scale tables take about a second instead of minutes): the same k
    grid, trapezoid rule in ln k and Bessel recurrences; sums in another
    order, so the result agrees with covariance() to rounding.  as_tensor
    returns the device tensor instead of a host array."""
    import torch
    r_np = np.asarray(r, dtype=np.float64)
    k_np = np.geomspace(kmin, kmax, nk)
    h = math.log(kmax / kmin) / (nk - 1)
    dlnk = np.full(nk, h)
    dlnk[0] = dlnk[-1] = 0.5 * h
    D_np = (2.0 / math.pi) * A * (k_np / 0.05) ** (ns - 1.0) * dlnk
    rt = torch.from_numpy(r_np).to(device)
    N = r_np.size
    C = torch.zeros((L + 1, N, N), dtype=torch.float64, device=device)
    for q0 in range(0, nk, kchunk):
        kc = torch.from_numpy(k_np[q0:q0 + kchunk]).to(device)
        Dc = torch.from_numpy(D_np[q0:q0 + kchunk]).to(device)
        J = _sph_bessel_table_torch(L, torch.outer(rt, kc).reshape(-1)).reshape(L + 1, N, kc.numel())
        JD = (J * Dc[None, None, :]).contiguous()
        C += torch.matmul(JD, J.transpose(1, 2).contiguous())
        del J, JD
    if not bool(torch.isfinite(C).all()):
        raise FloatingPointError("covariance_torch produced a non-finite value")
    if as_tensor:
        return C
    out = C.cpu().numpy()
    del C
    return out


def filter_from_covariance(C, jitter=1e-12):
    """Lower-triangular F_l with F_l F_l^T = C_l + jitter * max diag(C_l) I."""
    L1, N, _ = C.shape
    eye = np.eye(N)
    F = np.empty_like(C)
    for l in range(L1):
        d = float(np.max(np.diag(C[l])))
        F[l] = np.linalg.cholesky(C[l] + jitter * d * eye)
    return F


# --------------------------------------------------------- transfer tables

def transfer_tables(L, r, seed=TRANSFER_SEED, centre=14000.0, width=150.0):
    """alpha_l(r_i), beta_l(r_i): Gaussian in r times a smooth l-envelope
    e_l = 1 + 0.3 sum_{q=1..3} u_q sin(2 pi q l / L + psi_q)."""
    rng = np.random.default_rng(seed)
    uT = rng.uniform(0.0, 1.0, 3)
    pT = rng.uniform(0.0, 2.0 * math.pi, 3)
    uE = rng.uniform(0.0, 1.0, 3)
    pE = rng.uniform(0.0, 2.0 * math.pi, 3)
    ell = np.arange(L + 1, dtype=np.float64)
    Ls = max(L, 1)
    eT = 1.0 + 0.3 * sum(uT[q] * np.sin(2 * math.pi * (q + 1) * ell / Ls + pT[q]) for q in range(3))
    eE = 1.0 + 0.3 * sum(uE[q] * np.sin(2 * math.pi * (q + 1) * ell / Ls + pE[q]) for q in range(3))
    g = np.exp(-((np.asarray(r) - centre) ** 2) / (2.0 * width ** 2))
    alpha = eT[:, None] * g[None, :]
    beta = eE[:, None] * g[None, :]
    beta[:min(2, L + 1)] = 0.0
    return alpha, beta


# ----------------------------------------------------- estimator tables

def ksw_tables(p):
    """Tables of the cubic KSW statistic (Sect. 4) on the problem's radial
    nodes, as stand-ins for the CAMB-derived ones:

    * alpha^i_l(r_k): the transfer tables themselves (i = T, E), [2][L+1][N];
    * beta^i_l(r_k) = 4 pi int dk Delta^2(k)/k g^i_l(k) j_l(k r_k), which for
      alpha of the same g equals int dr r^2 C_l(r_k, r) alpha^i_l(r); on the
      nodes, sum_j C_l(r_k, r_j) w_j r_j^2 alpha^i_l(r_j), [2][L+1][N];
    * (C^-1)_l: the inverse of the model spectrum matrix [[TT, TE], [TE, EE]],
      C^{ij}_l = sum_{k,k'} W^i_lk C_l(r_k, r_k') W^j_lk' with W = w r^2 alpha,
      [L+1][2][2]; zero for l < 2 (monopole and dipole are left out, and EE
      vanishes there).  The synthetic T and E tables share one radial
      profile, so this matrix has rank one (E carries no information T
      lacks); its Moore-Penrose pseudo-inverse (eigenvalues below 1e-10 of
      the largest dropped) stands in for the inverse.
    """
    C = p["cov"]
    L1, N = p["alpha"].shape
    wr2 = p["w"] * p["r"] ** 2
    alpha = np.stack([p["alpha"], p["beta"]])
    W = alpha * wr2[None, None, :]
    beta = np.einsum("lkj,xlj->xlk", C, W)
    spec = np.einsum("xlk,ylk->lxy", W, beta)
    cinv = np.zeros((L1, 2, 2))
    for l in range(2, L1):
        S = 0.5 * (spec[l] + spec[l].T)
        lam, U = np.linalg.eigh(S)
        keep = lam > 1e-10 * lam.max()
        cinv[l] = (U[:, keep] / lam[keep]) @ U[:, keep].T
    return alpha, beta, cinv


def model_spectrum(p):
    """[L+1][2][2] T/E model spectrum C^{ij}_l = sum_kk' W^i_lk C_l(r_k, r_k') W^j_lk'
    with W = w r^2 alpha (alpha = the T and E transfer tables)."""
    wr2 = p["w"] * p["r"] ** 2
    W = np.stack([p["alpha"], p["beta"]]) * wr2[None, None, :]
    return np.einsum("xli,lij,ylj->lxy", W, p["cov"], W)


def gaussian_data(p, seed):
    """Seeded Gaussian T+E harmonic data with the model spectrum: a^X_lm with
    E[a^i a^j*] = C^{ij}_l, complex for m > 0 (E|z|^2 = 1 per draw) and real
    for m = 0; returns (aT, aE) [n_lm] complex128."""
    spec = model_spectrum(p)
    L = spec.shape[0] - 1
    ls, ms = lm_arrays(L)
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((2, ls.size, 2))
    s = 1.0 / math.sqrt(2.0)
    zc = np.where(ms == 0, z[:, :, 0], s * z[:, :, 0]) + 1j * np.where(ms == 0, 0.0, s * z[:, :, 1])
    out = np.zeros((2, ls.size), dtype=np.complex128)
    for l in range(L + 1):
        lam, U = np.linalg.eigh(0.5 * (spec[l] + spec[l].T))
        M = U * np.sqrt(np.maximum(lam, 0.0))[None, :]
        sel = ls == l
        out[:, sel] = M @ zc[:, sel]
    return out[0], out[1]


# ------------------------------------------------------------------ noise

def noise(L, N, seed, dtype=np.complex128, out=None):
    """n_lm(r_j), shape [N, n_lm]: (Z0 + i Z1)/sqrt(2) for m > 0, Z0 for m = 0,
    with Z = default_rng(seed).standard_normal((N, n_lm, 2)) drawn shell by
    shell (the same stream as one draw of the whole array)."""
    rng = np.random.default_rng(seed)
    n = nlm(L)
    _, ms = lm_arrays(L)
    m0 = ms == 0
    if out is None:
        out = np.empty((N, n), dtype=dtype)
    s = 1.0 / math.sqrt(2.0)
    for j in range(N):
        z = rng.standard_normal((n, 2))
        re = np.where(m0, z[:, 0], z[:, 0] * s)
        im = np.where(m0, 0.0, z[:, 1] * s)
        out[j].real = re
        out[j].imag = im
    return out


def realization_seed(index):
    return NOISE_SEED_BASE + int(index)


# ------------------------------------------------------------ full problem

def _cache_dir():
    d = os.environ.get("FNLSIM_INPUT_CACHE")
    if not d:
        d = os.path.join(os.path.expanduser("~"), ".cache", "fnlsim_inputs")
    os.makedirs(d, exist_ok=True)
    return d


def problem(L, N, seed=TRANSFER_SEED, cache=True, device=None):
    """dict(r, w, filter, alpha, beta, cov) for band limit L and N nodes.
    device: None evaluates the covariance with numpy on the host; a torch
    device (e.g. "cuda") evaluates it there (covariance_torch); the two agree
    to rounding and are cached apart."""
    tag = "v2" if device is None else "v2t"
    key = hashlib.sha1(f"{tag}|{L}|{N}|{seed}".encode()).hexdigest()[:16]
    path = os.path.join(_cache_dir(), f"problem_L{L}_N{N}_{key}.npz") if cache else None
    if path and os.path.exists(path):
        with np.load(path, allow_pickle=False) as z:
            return {k: z[k] for k in z.files}
    r, w = radial_nodes(N)
    C = covariance(L, r) if device is None else covariance_torch(L, r, device)
    F = filter_from_covariance(C)
    alpha, beta = transfer_tables(L, r, seed)
    out = dict(r=r, w=w, filter=F, alpha=alpha, beta=beta, cov=C)
    if path:
        tmp = path + f".tmp{os.getpid()}.npz"
        np.savez(tmp, **out)
        os.replace(tmp, path)
    return out
