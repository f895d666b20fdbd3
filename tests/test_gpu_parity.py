"""GPU parity: the HIP library against the FP64 CPU oracle, element by element
(per-l relative rms, each output separately), through the C ABI.

Bars: FP64 path <= 1e-10, FP32 matrix-core path <= 1e-5.
"""
import math

import numpy as np
import pytest

from paper_0909_0009_amd import inputs
from tests.parity import assert_close

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5}


@pytest.fixture(scope="module")
def fs():
    import torch
    from paper_0909_0009_amd import build, fnlsim
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    if not __import__("os").path.exists(fnlsim.LIB_PATH):
        build.build()
    fnlsim.lib()
    return fnlsim


def _problem(L, N):
    return inputs.problem(L, N)


def _sim(fs, p, L, precision="fp64", **kw):
    return fs.Simulator(L, p["r"], p["w"], p["filter"], p["alpha"], p["beta"],
                        precision=precision, **kw)


def _oracle(orc, p, L, alpha=None, beta=None, mean=0, ntheta=None, nphi=None):
    return orc.Problem(L, p["r"], p["w"], p["filter"],
                       p["alpha"] if alpha is None else alpha,
                       p["beta"] if beta is None else beta,
                       mean_mode=mean, ntheta=ntheta, nphi=nphi)


def _dev(noise, precision):
    import torch
    dt = torch.complex128 if precision == "fp64" else torch.complex64
    return torch.from_numpy(noise).to(dt).cuda()


def _check_all(got, ref, L, tol, tag):
    aT, aE, aTn, aEn = [g.cpu().numpy().reshape(-1) for g in got]
    errs = {}
    errs["aT"] = assert_close(aT, ref["aT"], L, tol, tag + " aT")
    errs["aE"] = assert_close(aE, ref["aE"], L, tol, tag + " aE")
    errs["aT_nl"] = assert_close(aTn, ref["aT_nl"], L, tol, tag + " aT_nl")
    errs["aE_nl"] = assert_close(aEn, ref["aE_nl"], L, tol, tag + " aE_nl")
    print(tag, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    return errs


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_tiny_config(fs, orc, precision):
    cfg = inputs.CONFIGS["tiny"]
    L, N = cfg["lmax"], cfg["nshell"]
    p = _problem(L, N)
    sim = _sim(fs, p, L, precision, n_ring=cfg["ntheta"], n_phi=cfg["nphi"])
    noise = inputs.noise(L, N, inputs.realization_seed(0))
    if precision == "fp32":
        noise = noise.astype(np.complex64).astype(np.complex128)
    got = sim.forward(_dev(noise, precision), cfg["fnl"], want_nl=True)
    ref = _oracle(orc, p, L).forward(noise, cfg["fnl"])
    _check_all(got, ref, L, TOL[precision], f"tiny {precision}")


def test_debug_stages_tiny(fs, orc):
    import torch
    cfg = inputs.CONFIGS["tiny"]
    L, N = cfg["lmax"], cfg["nshell"]
    p = _problem(L, N)
    sim = _sim(fs, p, L, "fp64", n_ring=cfg["ntheta"], n_phi=cfg["nphi"])
    noise = inputs.noise(L, N, inputs.realization_seed(0))
    P = _oracle(orc, p, L)
    phiL = P.filter_apply(noise)
    got = sim.debug_stage(fs.SIM_STAGE_FILTER, _dev(noise, "fp64")).cpu().numpy()
    for i in range(N):
        assert_close(got[i], phiL[i], L, 1e-12, f"filter shell {i}")
    out = P.forward(noise, 0.0, want_phi=True)
    nl = sim.debug_stage(fs.SIM_STAGE_NONLIN, torch.from_numpy(phiL).cuda()).cpu().numpy()
    for i in range(N):
        assert_close(nl[i], out["phiNL"][i], L, 1e-11, f"Phi_NL shell {i}")
    maps = sim.debug_stage(fs.SIM_STAGE_MAPS, torch.from_numpy(phiL).cuda()).cpu().numpy()
    for i in (0, N // 2, N - 1):
        ref = orc.synth(L, sim.n_ring, sim.n_phi, phiL[i])
        assert np.max(np.abs(maps[i] - ref)) < 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_medium_config(fs, orc, precision):
    cfg = inputs.CONFIGS["medium"]
    L, N = cfg["lmax"], cfg["nshell"]
    p = _problem(L, N)
    sim = _sim(fs, p, L, precision, n_ring=cfg["ntheta"], n_phi=cfg["nphi"])
    noise = inputs.noise(L, N, inputs.realization_seed(0))
    if precision == "fp32":
        noise = noise.astype(np.complex64).astype(np.complex128)
    got = sim.forward(_dev(noise, precision), cfg["fnl"], want_nl=True)
    ref = _oracle(orc, p, L).forward(noise, cfg["fnl"])
    _check_all(got, ref, L, TOL[precision], f"medium {precision}")


EDGE = [
    # (L, N, n_ring, n_phi, mean, R)
    (1, 1, 0, 0, 0, 1),
    (2, 3, 0, 0, 0, 1),
    (17, 7, 0, 0, 0, 1),        # odd L: n_phi = 54, no alias; ragged tiles
    (32, 16, 0, 0, 1, 1),       # ensemble mean
    (32, 16, 60, 100, 0, 1),    # larger grid than the minimum
    (40, 33, 0, 0, 0, 2),       # 66 columns (padded tile), two realizations
    (64, 5, 0, 0, 0, 1),        # few shells, many l
    (6, 300, 0, 0, 0, 1),       # N > 256: the filter runs two rounds of row-tile pairs
]


@pytest.mark.parametrize("L,N,nring,nphi,mean,R", EDGE)
def test_edge_shapes_fp64(fs, orc, L, N, nring, nphi, mean, R):
    p = _problem(L, N)
    sim = _sim(fs, p, L, "fp64", n_ring=nring, n_phi=nphi,
               mean="ensemble" if mean else "sample")
    noises = [inputs.noise(L, N, 4000 + k) for k in range(R)]
    fnl = [30.0 + 10 * k for k in range(R)]
    import torch
    batch = torch.from_numpy(np.stack(noises)).cuda()
    got = sim.forward(batch, fnl, want_nl=True)
    P = _oracle(orc, p, L, mean=mean)
    for k in range(R):
        ref = P.forward(noises[k], fnl[k])
        _check_all([g[k] for g in got], ref, L, TOL["fp64"], f"edge L={L} N={N} r={k}")


# the same shapes on the FP32 path (noise rounded to FP32 on both sides):
# ragged tiles, padded columns, N > 256 and the smallest l range, where the
# FP32 polar-skip threshold and the per-K-step polar start decide tile edges
@pytest.mark.parametrize("L,N,nring,nphi,mean,R", EDGE)
def test_edge_shapes_fp32(fs, orc, L, N, nring, nphi, mean, R):
    p = _problem(L, N)
    sim = _sim(fs, p, L, "fp32", n_ring=nring, n_phi=nphi,
               mean="ensemble" if mean else "sample")
    noises = [inputs.noise(L, N, 5000 + k).astype(np.complex64).astype(np.complex128)
              for k in range(R)]
    fnl = [30.0 + 10 * k for k in range(R)]
    import torch
    batch = torch.from_numpy(np.stack(noises)).to(torch.complex64).cuda()
    got = sim.forward(batch, fnl, want_nl=True)
    P = _oracle(orc, p, L, mean=mean)
    for k in range(R):
        ref = P.forward(noises[k], fnl[k])
        _check_all([g[k] for g in got], ref, L, TOL["fp32"], f"edge fp32 L={L} N={N} r={k}")


def test_forward_rejects_empty_and_null_then_still_runs(fs, orc):
    """R = 0 and null outputs are SIM_EINVAL through the C ABI, with no device
    work; the context then still gives the oracle's result."""
    import torch
    L, N = 8, 3
    p = _problem(L, N)
    sim = _sim(fs, p, L, "fp64")
    noise = inputs.noise(L, N, 77)
    x = torch.from_numpy(noise[None]).cuda()
    f = np.array([40.0])
    aT = torch.empty((1, sim.n_lm), dtype=torch.complex128, device="cuda")
    aE = torch.empty_like(aT)
    lib = fs.lib()
    assert lib.sim_forward(sim._h, x.data_ptr(), 0, f.ctypes.data, aT.data_ptr(), aE.data_ptr(),
                           None, None) == fs.SIM_EINVAL
    assert lib.sim_forward(sim._h, x.data_ptr(), 1, f.ctypes.data, None, aE.data_ptr(),
                           None, None) == fs.SIM_EINVAL
    assert lib.sim_forward(sim._h, None, 1, f.ctypes.data, aT.data_ptr(), aE.data_ptr(),
                           None, None) == fs.SIM_EINVAL
    assert lib.sim_last_error(sim._h)  # the reason is reported
    got = sim.forward(x, 40.0, want_nl=True)
    ref = _oracle(orc, p, L).forward(noise, 40.0)
    _check_all([g[0] for g in got], ref, L, TOL["fp64"], "after rejected calls")


# Paper workload: 200 nodes = 400 real columns in five 80-column tiles of the
# Legendre kernels (40 shells each); one kept shell per tile, the last one
# included.
PAPER_KEEP = [0, 45, 93, 140, 199]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_paper_scale_sampled_shells(fs, orc, precision):
    """Full lmax = 1024, 200 nodes, 1537 x 3072 grid in the benchmark's launch
    configuration, at f_NL = 0 and 100; the transfer tables are zeroed except
    on one node of every column tile, so the oracle only has to evaluate
    those shells (the linear part still sums the filter over all nodes)."""
    cfg = inputs.CONFIGS["paper"]
    L, N = cfg["lmax"], cfg["nshell"]
    p = _problem(L, N)
    keep = PAPER_KEEP
    al = np.zeros_like(p["alpha"])
    be = np.zeros_like(p["beta"])
    al[:, keep] = p["alpha"][:, keep]
    be[:, keep] = p["beta"][:, keep]
    sim = fs.Simulator(L, p["r"], p["w"], p["filter"], al, be, precision=precision,
                       n_ring=cfg["ntheta"], n_phi=cfg["nphi"])
    assert sim.col_tile == 80 and sorted({2 * s // 80 for s in keep}) == [0, 1, 2, 3, 4]
    noise = inputs.noise(L, N, inputs.realization_seed(0))
    if precision == "fp32":
        noise = noise.astype(np.complex64).astype(np.complex128)
    ref = _oracle(orc, p, L, alpha=al, beta=be).forward(noise, cfg["fnl"])
    dev = _dev(noise, precision)
    got = sim.forward(dev, cfg["fnl"], want_nl=True)
    _check_all(got, ref, L, TOL[precision], f"paper {precision} f_NL={cfg['fnl']}")
    got0 = sim.forward(dev, 0.0, want_nl=True)
    ref0 = dict(ref, aT=ref["aT_lin"], aE=ref["aE_lin"])
    _check_all(got0, ref0, L, TOL[precision], f"paper {precision} f_NL=0")


def test_many_shells_fp32(fs, orc):
    """N = 300 (10 row tiles, two rounds of tile pairs in the filter, 600
    columns) on the FP32 path."""
    L, N = 7, 300
    p = _problem(L, N)
    sim = _sim(fs, p, L, "fp32")
    noise = inputs.noise(L, N, 55).astype(np.complex64).astype(np.complex128)
    got = sim.forward(_dev(noise, "fp32"), 70.0, want_nl=True)
    ref = _oracle(orc, p, L).forward(noise, 70.0)
    _check_all(got, ref, L, TOL["fp32"], "N=300 fp32")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_dense_filter(fs, orc, precision):
    """The ABI takes any real filter, not only a Cholesky factor: a dense F
    (upper triangle non-zero) takes the full contraction."""
    L, N = 20, 70
    p = _problem(L, N)
    rng = np.random.default_rng(5)
    F = p["filter"] + np.triu(rng.standard_normal((L + 1, N, N)), 1) * 1e-6
    sim = fs.Simulator(L, p["r"], p["w"], F, p["alpha"], p["beta"], precision=precision)
    noise = inputs.noise(L, N, 31)
    if precision == "fp32":
        noise = noise.astype(np.complex64).astype(np.complex128)
    got = sim.forward(_dev(noise, precision), 60.0, want_nl=True)
    ref = orc.Problem(L, p["r"], p["w"], F, p["alpha"], p["beta"]).forward(noise, 60.0)
    _check_all(got, ref, L, TOL[precision], f"dense filter {precision}")


@pytest.mark.parametrize("L,N,nphi", [(40, 33, 0), (256, 64, 0), (64, 5, 200)])
@pytest.mark.parametrize("rs", [1, 2])
def test_fp32_ring_shells_per_block(fs, orc, L, N, nphi, rs):
    """Both ring-stage block shapes of the FP32 data path (1 or 2 shells per
    block, the launch shape the autotuner chooses between) give the oracle's
    result: planned and run-time FFT lengths, an odd shell count."""
    p = _problem(L, N)
    sim = fs.Simulator(L, p["r"], p["w"], p["filter"], p["alpha"], p["beta"], n_phi=nphi,
                       precision="fp32", ring_shells=rs)
    assert sim.ring_shells == rs
    noise = inputs.noise(L, N, 91).astype(np.complex64).astype(np.complex128)
    got = sim.forward(_dev(noise, "fp32"), 60.0, want_nl=True)
    ref = _oracle(orc, p, L, nphi=nphi or None).forward(noise, 60.0)
    _check_all(got, ref, L, TOL["fp32"], f"L={L} N={N} nphi={nphi} ring shells {rs}")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_tuned_column_tile(fs, orc, precision):
    """The set-up autotuner (one context per column tile, fastest kept) gives
    the oracle's result, and the untuned context's to rounding."""
    L, N = 40, 33
    p = _problem(L, N)
    tuned = _sim(fs, p, L, precision, tune=True)
    plain = _sim(fs, p, L, precision)
    assert tuned.col_tile in (16, 32, 48, 64, 80) and plain.col_tile in (16, 32, 48, 64, 80)
    assert tuned.ring_shells in ((1, 2) if precision == "fp32" else (1,))
    noise = inputs.noise(L, N, 77)
    if precision == "fp32":
        noise = noise.astype(np.complex64).astype(np.complex128)
    got = tuned.forward(_dev(noise, precision), 40.0, want_nl=True)
    ref = _oracle(orc, p, L).forward(noise, 40.0)
    _check_all(got, ref, L, TOL[precision], f"tuned (tile {tuned.col_tile}) {precision}")
    base = plain.forward(_dev(noise, precision), 40.0, want_nl=True)
    for g, b in zip(got, base):
        assert_close(g.cpu().numpy().reshape(-1), b.cpu().numpy().reshape(-1), L,
                     1e-12 if precision == "fp64" else 1e-6, "tuned vs untuned")
