"""Batching form: several contexts with uneven lmax and node counts run as one
grouped launch per stage, captured in a HIP graph; every realization must equal
its own single-context forward pass, on the first call and on graph replays
with new inputs."""
import ctypes

import numpy as np
import pytest

from paper_0909_0009_amd import inputs
from tests.parity import assert_close

pytestmark = pytest.mark.gpu

MIX = [(48, 9), (16, 5), (64, 12), (32, 20), (40, 7), (24, 16)]


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


def _batch(fs, sims):
    arr = (ctypes.c_void_p * len(sims))(*[s.handle.value for s in sims])
    h = ctypes.c_void_p()
    rc = fs.lib().sim_batch_create(arr, len(sims), ctypes.byref(h))
    assert rc == 0, fs.lib().sim_last_error(None)
    return h


def _run_batch(fs, h, noises, fnls, outs):
    n = len(noises)
    nz = (ctypes.c_void_p * n)(*[x.data_ptr() for x in noises])
    aT = (ctypes.c_void_p * n)(*[o[0].data_ptr() for o in outs])
    aE = (ctypes.c_void_p * n)(*[o[1].data_ptr() for o in outs])
    f = np.ascontiguousarray(fnls, dtype=np.float64)
    rc = fs.lib().sim_batch_forward(h, nz, f.ctypes.data, aT, aE)
    assert rc == 0


@pytest.mark.parametrize("form", ["grouped", "branches", "auto"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_equals_sequential(fs, precision, form, monkeypatch):
    if form != "auto":
        monkeypatch.setenv("FNLSIM_BATCH_FORM", form)
    else:
        monkeypatch.delenv("FNLSIM_BATCH_FORM", raising=False)
    import torch
    dt = torch.complex128 if precision == "fp64" else torch.complex64
    sims, probs = [], []
    for L, N in MIX:
        p = inputs.problem(L, N)
        probs.append(p)
        sims.append(fs.Simulator(L, p["r"], p["w"], p["filter"], p["alpha"], p["beta"],
                                 precision=precision))
    h = _batch(fs, sims)
    try:
        for call in range(3):   # capture, then two replays with new inputs
            noises = [torch.from_numpy(inputs.noise(L, N, 900 + 10 * call + i)).to(dt).cuda()
                      for i, (L, N) in enumerate(MIX)]
            fnls = [50.0 + call + i for i in range(len(MIX))]
            outs = [(torch.empty((1, s.n_lm), dtype=torch.complex128, device="cuda"),
                     torch.empty((1, s.n_lm), dtype=torch.complex128, device="cuda"))
                    for s in sims]
            _run_batch(fs, h, noises, fnls, outs)
            torch.cuda.synchronize()
            exact = 0
            for i, s in enumerate(sims):
                rT, rE = s.forward(noises[i], fnls[i])
                torch.cuda.synchronize()
                exact += int(torch.equal(rT, outs[i][0]) and torch.equal(rE, outs[i][1]))
                L = MIX[i][0]
                assert_close(outs[i][0].cpu().numpy(), rT.cpu().numpy(), L, 1e-13, f"batch aT {i}")
                assert_close(outs[i][1].cpu().numpy(), rE.cpu().numpy(), L, 1e-13, f"batch aE {i}")
            print(f"{form} call {call}: {exact}/{len(sims)} realizations bitwise equal", flush=True)
            assert exact == len(sims)
        m = ctypes.c_int(-2)
        fs.lib().sim_batch_get_mode(h, ctypes.byref(m), None, None)
        assert m.value == {"grouped": 0, "branches": 1}.get(form, m.value) and m.value in (0, 1)
    finally:
        fs.lib().sim_batch_destroy(h)


def test_batch_rejects_a_repeated_context(fs):
    p = inputs.problem(16, 5)
    a = fs.Simulator(16, p["r"], p["w"], p["filter"], p["alpha"], p["beta"])
    arr = (ctypes.c_void_p * 2)(a.handle.value, a.handle.value)
    h = ctypes.c_void_p()
    assert fs.lib().sim_batch_create(arr, 2, ctypes.byref(h)) == fs.SIM_EINVAL


def test_batch_rejects_mixed_precision(fs):
    p = inputs.problem(16, 5)
    a = fs.Simulator(16, p["r"], p["w"], p["filter"], p["alpha"], p["beta"], precision="fp64")
    b = fs.Simulator(16, p["r"], p["w"], p["filter"], p["alpha"], p["beta"], precision="fp32")
    arr = (ctypes.c_void_p * 2)(a.handle.value, b.handle.value)
    h = ctypes.c_void_p()
    assert fs.lib().sim_batch_create(arr, 2, ctypes.byref(h)) == fs.SIM_EINVAL


@pytest.mark.parametrize("form", ["grouped", "branches"])
def test_batch_with_one_shell_ring_blocks(fs, form, monkeypatch):
    """FP32 contexts fixed to one shell per ring block (sim_opts.ring_shells =
    1, a shape the autotuner may pick): the grouped form's ring launches keep
    the default two-shell blocks and the branch form runs each context's own
    launches; both equal the sequential passes bit for bit."""
    monkeypatch.setenv("FNLSIM_BATCH_FORM", form)
    import torch
    sims = []
    for L, N in MIX[:4]:
        p = inputs.problem(L, N)
        sims.append(fs.Simulator(L, p["r"], p["w"], p["filter"], p["alpha"], p["beta"],
                                 precision="fp32", ring_shells=1))
        assert sims[-1].ring_shells == 1
    h = _batch(fs, sims)
    try:
        noises = [torch.from_numpy(inputs.noise(L, N, 700 + i)).to(torch.complex64).cuda()
                  for i, (L, N) in enumerate(MIX[:4])]
        fnls = [40.0 + i for i in range(4)]
        outs = [(torch.empty((1, s.n_lm), dtype=torch.complex128, device="cuda"),
                 torch.empty((1, s.n_lm), dtype=torch.complex128, device="cuda")) for s in sims]
        _run_batch(fs, h, noises, fnls, outs)
        torch.cuda.synchronize()
        for i, s in enumerate(sims):
            rT, rE = s.forward(noises[i], fnls[i])
            torch.cuda.synchronize()
            assert torch.equal(rT, outs[i][0]) and torch.equal(rE, outs[i][1]), f"{form} context {i}"
    finally:
        fs.lib().sim_batch_destroy(h)
