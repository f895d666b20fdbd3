"""GPU reverse pass (differentiation form): the hand-written adjoint against the
CPU FP64 oracle adjoint, against central differences of the GPU forward, and
through torch.autograd.Function."""
import numpy as np
import pytest

from paper_0909_0009_amd import inputs
from tests.parity import assert_close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fs():
    import os

    import torch
    from paper_0909_0009_amd import build, fnlsim
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    if not os.path.exists(fnlsim.LIB_PATH):
        build.build()
    fnlsim.lib()
    return fnlsim


def rand_c(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _per_l_all_shells(g, ref, L):
    """Per-l relative rms of a [N][n_lm] gradient, norms over all shells and m."""
    ls, ms = inputs.lm_arrays(L)
    c = np.where(ms == 0, 1.0, 2.0)
    num = np.sqrt(np.bincount(ls, weights=c * np.sum(np.abs(g - ref) ** 2, axis=0)))
    den = np.sqrt(np.bincount(ls, weights=c * np.sum(np.abs(ref) ** 2, axis=0)))
    return float(np.max(num / den))


def _per_shell_errors(g, ref, L):
    """Per input shell j: max over l of ||g_j - ref_j||_l / ||ref_j||_l, and the
    same error measured against the largest shell's norm at that l."""
    ls, ms = inputs.lm_arrays(L)
    c = np.where(ms == 0, 1.0, 2.0)
    num = np.stack([np.sqrt(np.bincount(ls, weights=c * np.abs(g[j] - ref[j]) ** 2, minlength=L + 1))
                    for j in range(ref.shape[0])])
    den = np.stack([np.sqrt(np.bincount(ls, weights=c * np.abs(ref[j]) ** 2, minlength=L + 1))
                    for j in range(ref.shape[0])])
    top = np.maximum(den.max(axis=0), 1e-300)
    rel = np.where(den > 0, num / np.where(den > 0, den, 1.0), np.where(num > 0, np.inf, 0.0))
    return rel.max(axis=1), (num / top[None, :]).max(axis=1), den.max(axis=1) / top.max()


def _compare_grad(gn, ref_gn, gf, ref_gf, L, tol, tag):
    worst = 0.0
    if tol < 1e-8:
        # FP64: every input shell separately
        for i in range(ref_gn.shape[0]):
            if np.max(np.abs(ref_gn[i])) == 0:
                continue
            worst = max(worst, assert_close(gn[i], ref_gn[i], L, tol, f"{tag} grad shell {i}"))
    else:
        # FP32: every input shell separately (per-l relative rms of that
        # shell's own gradient), with the aggregate over all shells and the
        # error against the largest shell's gradient reported beside it
        agg = _per_l_all_shells(gn, ref_gn, L)
        rel, vs_top, size = _per_shell_errors(gn, ref_gn, L)
        order = np.argsort(rel)[::-1][:4]
        print(tag, f"aggregate {agg:.1e}; worst shells (shell, own-norm error, error vs "
              "largest shell, norm vs largest):",
              [(int(j), f"{rel[j]:.1e}", f"{vs_top[j]:.1e}", f"{size[j]:.1e}") for j in order],
              flush=True)
        worst = float(np.max(rel))
        assert worst <= tol, f"{tag} grad of shell {int(np.argmax(rel))}: {worst:.3e} > {tol}"
    rel = abs(gf - ref_gf) / max(abs(ref_gf), 1e-300)
    assert rel <= tol, f"{tag} grad_fnl {gf} vs {ref_gf} ({rel:.2e})"
    print(tag, f"grad_n {worst:.2e} grad_fnl {rel:.2e}", flush=True)


CASES = [
    # (L, N, n_ring, n_phi, mean, fnl, precision)
    (16, 8, 0, 0, "sample", 100.0, "fp64"),      # n_phi = 48 = 3L: alias term
    (16, 8, 0, 0, "ensemble", 100.0, "fp64"),
    (16, 8, 0, 0, "sample", 0.0, "fp64"),
    (21, 5, 0, 0, "sample", 37.0, "fp64"),       # odd L: no alias, ragged tiles
    (32, 16, 0, 0, "sample", 100.0, "fp32"),
    (32, 16, 0, 0, "ensemble", 100.0, "fp32"),
    (6, 300, 0, 0, "sample", 60.0, "fp64"),      # N > 256: filter rounds, forward and transposed
]


@pytest.mark.parametrize("L,N,nring,nphi,mean,fnl,precision", CASES)
def test_backward_matches_oracle_adjoint(fs, orc, L, N, nring, nphi, mean, fnl, precision):
    import torch
    p = inputs.problem(L, N)
    sim = fs.Simulator(L, p["r"], p["w"], p["filter"], p["alpha"], p["beta"], n_ring=nring,
                       n_phi=nphi, mean=mean, precision=precision)
    noise = inputs.noise(L, N, 123)
    if precision == "fp32":
        noise = noise.astype(np.complex64).astype(np.complex128)
    nlm = sim.n_lm
    gT = rand_c(nlm, 1)
    gE = rand_c(nlm, 2)
    dt = torch.complex128 if precision == "fp64" else torch.complex64
    gn, gf = sim.backward(torch.from_numpy(noise).to(dt).cuda(), fnl,
                          torch.from_numpy(gT).cuda(), torch.from_numpy(gE).cuda())
    P = orc.Problem(L, p["r"], p["w"], p["filter"], p["alpha"], p["beta"],
                    mean_mode=1 if mean == "ensemble" else 0)
    ref_gn, ref_gf = P.adjoint(noise, fnl, gT, gE)
    tol = 1e-10 if precision == "fp64" else 1e-5
    g = gn.cpu().numpy().reshape(N, nlm).astype(np.complex128)
    _compare_grad(g, ref_gn, float(gf[0]), ref_gf, L, tol, f"L={L} N={N} {mean} {precision}")
    _, ms = inputs.lm_arrays(L)
    assert np.all(g[:, ms == 0].imag == 0)


def test_backward_two_realizations_and_central_differences(fs):
    """R = 2 in one call, and the directional derivative of the GPU forward
    (central difference: exact for a loss quadratic in the noise)."""
    import torch
    L, N, fnl = 12, 6, 80.0
    p = inputs.problem(L, N)
    sim = fs.Simulator(L, p["r"], p["w"], p["filter"], p["alpha"], p["beta"])
    nlm = sim.n_lm
    n = torch.from_numpy(np.stack([inputs.noise(L, N, 7), inputs.noise(L, N, 8)])).cuda()
    gT = torch.from_numpy(np.stack([rand_c(nlm, 3), rand_c(nlm, 4)])).cuda()
    gE = torch.from_numpy(np.stack([rand_c(nlm, 5), rand_c(nlm, 6)])).cuda()
    gn, gf = sim.backward(n, [fnl, fnl], gT, gE)

    def loss(nn, f):
        aT, aE = sim.forward(nn, f)
        return float((torch.sum(torch.conj(gT) * aT) + torch.sum(torch.conj(gE) * aE)).real)

    d = torch.from_numpy(np.stack([rand_c((N, nlm), 9), rand_c((N, nlm), 10)])).cuda()
    h = 1e-2
    num = (loss(n + h * d, [fnl, fnl]) - loss(n - h * d, [fnl, fnl])) / (2 * h)
    ana = float(torch.sum(torch.conj(gn) * d).real)
    assert abs(num - ana) <= 1e-9 * abs(ana), (num, ana)
    numf = (loss(n, [fnl + 1, fnl + 1]) - loss(n, [fnl - 1, fnl - 1])) / 2
    assert abs(numf - (gf[0] + gf[1])) <= 1e-9 * abs(numf)
    # each realization's gradient equals its own single-realization call
    g0, f0 = sim.backward(n[0:1], fnl, gT[0:1], gE[0:1])
    assert torch.equal(g0[0], gn[0]) and f0[0] == gf[0]


def test_autograd_function(fs):
    """torch.autograd through the map generator: the loss of the
    differentiation workload, sum_lm c_m |a^T - t|^2 / C_l."""
    import torch
    L, N = 24, 10
    p = inputs.problem(L, N)
    sim = fs.Simulator(L, p["r"], p["w"], p["filter"], p["alpha"], p["beta"])
    n = torch.from_numpy(inputs.noise(L, N, 11)).cuda().unsqueeze(0).requires_grad_(True)
    f = torch.tensor([100.0], dtype=torch.float64, requires_grad=True)
    t, _ = sim.forward(torch.from_numpy(inputs.noise(L, N, inputs.TARGET_SEED)).cuda(), 100.0)
    W = p["alpha"] * (p["w"] * p["r"] ** 2)[None, :]
    V = np.einsum("li,lij->lj", W, p["filter"])
    Cl = np.sum(V * V, axis=1)
    ls, ms = inputs.lm_arrays(L)
    wgt = torch.from_numpy(np.where(ms == 0, 1.0, 2.0) / Cl[ls]).cuda()
    aT, aE = fs.simulate(sim, n, f)
    lossv = torch.sum(wgt * torch.abs(aT[0] - t[0]) ** 2)
    lossv.backward()
    gT = (2 * wgt * (aT[0] - t[0])).detach().unsqueeze(0)
    gn, gf = sim.backward(n.detach(), 100.0, gT, torch.zeros_like(gT))
    assert torch.allclose(n.grad, gn, rtol=0, atol=1e-12 * float(gn.abs().max()))
    assert abs(f.grad.item() - gf[0]) <= 1e-12 * abs(gf[0])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_grad_workload_sampled_shells(fs, orc, precision):
    """lmax 512, 96 nodes, 769 x 1536 grid (the differentiation workload), with
    the transfer tables zeroed except on one node per column tile so the
    CPU adjoint stays cheap; loss as in the workload with a target from a second seed."""
    import torch
    cfg = inputs.CONFIGS["grad"]
    L, N, fnl = cfg["lmax"], cfg["nshell"], cfg["fnl"]
    p = inputs.problem(L, N)
    keep = [3, 45, 92]   # one node in each of the three 64-column tiles
    al = np.zeros_like(p["alpha"])
    be = np.zeros_like(p["beta"])
    al[:, keep] = p["alpha"][:, keep]
    be[:, keep] = p["beta"][:, keep]
    sim = fs.Simulator(L, p["r"], p["w"], p["filter"], al, be, n_ring=cfg["ntheta"],
                       n_phi=cfg["nphi"], precision=precision)
    noise = inputs.noise(L, N, inputs.realization_seed(0))
    if precision == "fp32":
        noise = noise.astype(np.complex64).astype(np.complex128)
    dt = torch.complex128 if precision == "fp64" else torch.complex64
    nz = torch.from_numpy(noise).to(dt).cuda()
    tgt = inputs.noise(L, N, inputs.TARGET_SEED)
    P = orc.Problem(L, p["r"], p["w"], p["filter"], al, be)
    t = P.forward(tgt, fnl)["aT"]
    a = P.forward(noise, fnl)["aT"]
    W = al * (p["w"] * p["r"] ** 2)[None, :]
    V = np.einsum("li,lij->lj", W, p["filter"])
    Cl = np.sum(V * V, axis=1)
    ls, ms = inputs.lm_arrays(L)
    gT = 2 * np.where(ms == 0, 1.0, 2.0) / Cl[ls] * (a - t)
    gE = np.zeros_like(gT)
    gn, gf = sim.backward(nz, fnl, torch.from_numpy(gT).cuda(), torch.from_numpy(gE).cuda())
    ref_gn, ref_gf = P.adjoint(noise, fnl, gT, gE)
    tol = 1e-10 if precision == "fp64" else 1e-5
    _compare_grad(gn.cpu().numpy().reshape(N, -1).astype(np.complex128), ref_gn, float(gf[0]),
                  ref_gf, L, tol, f"grad workload {precision}")


def test_backward_regrows_its_workspace(fs):
    """R = 1, then R = 2 (the per-realization f_NL workspace grows), then
    R = 1 again on one context: every call gives the same gradients for the
    same realization."""
    import torch
    L, N = 10, 6
    p = inputs.problem(L, N)
    sim = fs.Simulator(L, p["r"], p["w"], p["filter"], p["alpha"], p["beta"])
    nlm = sim.n_lm
    n = torch.from_numpy(np.stack([inputs.noise(L, N, 17), inputs.noise(L, N, 18)])).cuda()
    gT = torch.from_numpy(np.stack([rand_c(nlm, 21), rand_c(nlm, 22)])).cuda()
    gE = torch.from_numpy(np.stack([rand_c(nlm, 23), rand_c(nlm, 24)])).cuda()
    gn1, gf1 = sim.backward(n[:1], [40.0], gT[:1], gE[:1])
    gn2, gf2 = sim.backward(n, [40.0, -15.0], gT, gE)
    gn3, gf3 = sim.backward(n[:1], [40.0], gT[:1], gE[:1])
    assert torch.equal(gn1[0], gn2[0]) and torch.equal(gn3, gn1)
    assert gf1[0] == gf2[0] == gf3[0]
    ref_gn, ref_gf = sim.backward(n[1:], [-15.0], gT[1:], gE[1:])
    assert torch.equal(ref_gn[0], gn2[1]) and ref_gf[0] == gf2[1]
