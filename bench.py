"""Benchmark of the local-f_NL map generator on one MI355X.

One step = one full forward pass of the hot path (filter, Legendre synthesis,
ring FFT stage with the square and mean removal, Legendre analysis, radial
quadrature, combine) for one T+E realization at the paper-scale workload
(lmax 1024, 200 radial nodes, 1537 x 3072 Gauss-Legendre grid).  The
headline value is the FP32 matrix-core path (FP64 recurrence and radial
sums); the FP64 path is measured on the same inputs and reported beside it.

Prints one JSON line.  Inputs are seeded and synthetic (see
paper_0909_0009_amd/inputs.py) and resident in HBM before timing starts.
"""
import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "T+E map realizations/sec at lmax=1024 (mixed vs FP64 GPU path, same error)"

PEAK = {  # MI355X published dense peaks
    "hbm_GBs": 8000.0,
    "fp64_mfma_TFs": 78.6,
    "fp32_mfma_TFs": 157.3,
    "bf16_mfma_TFs": 2500.0,
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def stage_work(sim, stage, precision):
    """Algorithmic work of one launch of a stage: (bound, amount, unit)."""
    L, N = sim.lmax, sim.nshell
    nlm = (L + 1) * (L + 2) // 2
    C = 2 * N
    esize = 8 if precision == "fp64" else 4
    if stage in ("synth", "anal"):
        # every lambda_lm(x_p) multiplies each of the 2N real columns once
        return "mfma", 2.0 * sim.n_pair * nlm * C, "flop"
    if stage == "filter":
        return "mfma", 4.0 * N * N * nlm, "flop"
    if stage == "ring":
        # read the synthesis spectra, write the analysis spectra (E and O)
        return "hbm", 2.0 * sim.n_pair * (L + 1) * 2 * C * esize, "byte"
    if stage == "radial_lin":
        return "hbm", N * nlm * 2.0 * esize + 2 * nlm * 16.0, "byte"
    return "hbm", 0.0, "byte"


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "internal.h", "device_common.h"):
        with open(os.path.join(ROOT, "paper_0909_0009_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(stage, precision):
    """HBM bytes per launch of a stage's kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE record (profiles/hbm_traffic.json), or None when
    the kernel sources have changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_sha256") != kernel_source_hash():
        return None
    T = "float" if precision == "fp32" else "double"
    pat = re.compile(rf"^k_{stage}<{T}[,>]")
    # the filter's stored-noise instantiation (", true>" marks the seeded one)
    hits = [v for k, v in rec["kernels"].items()
            if pat.match(k) and not (stage == "filter" and k.endswith(", true>"))]
    return round(hits[0]["traffic_bytes"]) if len(hits) == 1 else None


def roofline(sim, stages, precision, steps):
    """Roofline object for the stage with the largest total time."""
    dom = max(stages, key=lambda k: stages[k][0])
    tot_ms, n = stages[dom]
    avg_s = tot_ms / max(n, 1) / 1e3
    bound, work, unit = stage_work(sim, dom, precision)
    if bound == "mfma":
        achieved = work / avg_s / 1e12
        peak = PEAK["fp64_mfma_TFs"] if precision == "fp64" else PEAK["fp32_mfma_TFs"]
        u = "TFLOP/s"
    else:
        achieved = work / avg_s / 1e9
        peak = PEAK["hbm_GBs"]
        u = "GB/s"
    return dom, {"bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": u,
                 "frac": round(achieved / peak, 4), "traffic": measured_traffic(dom, precision),
                 "traffic_unit": "byte",
                 "kernel": dom, "avg_launch_ms": round(avg_s * 1e3, 4),
                 "work_per_launch": work, "work_unit": unit}


def time_path(torch, fnlsim, p, cfg, noise_np, precision, steps, warmup):
    L, N = cfg["lmax"], cfg["nshell"]
    sim = fnlsim.Simulator(L, p["r"], p["w"], p["filter"], p["alpha"], p["beta"],
                           n_ring=cfg["ntheta"], n_phi=cfg["nphi"], precision=precision)
    dt = torch.complex128 if precision == "fp64" else torch.complex64
    noise = torch.from_numpy(noise_np).to(dt).cuda()
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        out = sim.forward(noise, cfg["fnl"])
    torch.cuda.synchronize()
    sim.profile(True)
    sim.profile_read()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        out = sim.forward(noise, cfg["fnl"])
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    stages = sim.profile_read()
    sim.profile(False)
    aT, aE = out
    # the non-linear parts alone (outside the timed region): they carry the
    # error of the matrix-core transforms, which the linear part hides
    nl = sim.forward(noise, cfg["fnl"], want_nl=True)
    res = dict(ms=ms, stages=stages, aT=aT.cpu().numpy().ravel(), aE=aE.cpu().numpy().ravel(),
               aT_nl=nl[2].cpu().numpy().ravel(), aE_nl=nl[3].cpu().numpy().ravel(),
               sim=sim, ws=sim.workspace_bytes)
    del noise, nl
    return res


def split_bf16_leg(r, ref, precision, L):
    """Timing and error of a split-BF16 form of the Legendre transforms.
    The matrix cores issue nprod BF16 products per FP32 product; the rate
    of those products is set against the dense BF16 peak."""
    nprod = 3 if precision == "bf16x3" else 6
    sim = r["sim"]
    legs = {}
    for st in ("synth", "anal"):
        tot, n = r["stages"][st]
        avg_s = tot / max(n, 1) / 1e3
        _, work, _ = stage_work(sim, st, "fp32")
        legs[st] = {"avg_launch_ms": round(avg_s * 1e3, 4),
                    "algorithmic_TFs": round(work / avg_s / 1e12, 2),
                    "bf16_products_TFs": round(nprod * work / avg_s / 1e12, 2),
                    "frac_of_bf16_peak": round(nprod * work / avg_s / 1e12 / PEAK["bf16_mfma_TFs"], 4)}
    err_nl = None
    if ref is not None:
        err_nl = max(per_l_rel_err(r["aT_nl"], ref["aT_nl"], L),
                     per_l_rel_err(r["aE_nl"], ref["aE_nl"], L))
    return {"value": round(1000.0 / r["ms"], 4), "ms_per_step": round(r["ms"], 4),
            "stages_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in r["stages"].items()},
            "legendre": legs, "nl_max_rel_err_vs_fp64": err_nl}


def time_seeded(torch, sim, cfg, steps, warmup):
    """The same forward with counter-based noise generated inside the linear
    radial sum and the filter (sim_forward_seeded): no noise buffer is read.
    A new seed per step."""
    stream = torch.cuda.current_stream()
    for k in range(warmup):
        sim.forward_seeded([1000 + k], cfg["fnl"])
    torch.cuda.synchronize()
    sim.profile(True)
    sim.profile_read()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for k in range(steps):
        sim.forward_seeded([2000 + k], cfg["fnl"])
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    st = sim.profile_read()
    sim.profile(False)
    elem = 8 if sim.precision == "fp32" else 16
    # the generator alone (sim_noise: one realization's noise written to HBM)
    nvals = sim.nshell * sim.n_lm
    buf = sim.noise([1])
    torch.cuda.synchronize()
    e0.record(stream)
    for k in range(steps):
        buf = sim.noise([3000 + k])
    e1.record(stream)
    torch.cuda.synchronize()
    gen_ms = e0.elapsed_time(e1) / steps
    del buf
    return {"value": round(1000.0 / ms, 4), "unit": "maps/s", "ms_per_step": round(ms, 4),
            "stages_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in st.items()},
            "noise_bytes_not_stored": elem * nvals,
            "sim_noise_ms": round(gen_ms, 4),
            "sim_noise_values_per_s": round(nvals / gen_ms * 1e3, 1)}


def time_quadrature(torch, fnlsim, inputs, L=1024, ntot=400, n=70):
    """Greedy radial-quadrature design (sim_quadrature_design) at the size of
    a full design: the synthetic covariance of Eq. cov_phi on a 400-shell
    fine grid over [13000, 15000] Mpc (evaluated on the GPU), P = 2 (L + 1)
    problems (l = 0..1024, T and E) with the fine-sum weights dr r^2 X_l(r)
    of the synthetic transfer tables, each scaled to unit a^T C a; 70 nodes.
    The call is synchronous; the best of 3 after one warm-up."""
    import numpy as np
    r = np.linspace(13000.0, 15000.0, ntot)
    C = inputs.covariance_torch(L, r, "cuda", as_tensor=True)
    alpha, beta = inputs.transfer_tables(L, r)
    dr = np.zeros(ntot)
    dr[:-1] += 0.5 * np.diff(r)
    dr[1:] += 0.5 * np.diff(r)
    P = 2 * (L + 1)
    a = torch.empty((P, ntot), dtype=torch.float64, device="cuda")
    a[0::2] = torch.from_numpy(dr * r * r * alpha).cuda()
    a[1::2] = torch.from_numpy(dr * r * r * beta).cuda()
    # T and E problems of one multipole share C_l (sim_quadrature_design_shared);
    # each problem is scaled to unit a^T C a through its a
    cidx = np.arange(P) // 2
    a2 = a.view(L + 1, 2, ntot)
    s = torch.einsum("lxi,lij,lxj->lx", a2, C, a2).reshape(P)
    s = torch.where(s > 0, s, torch.ones_like(s))
    a /= torch.sqrt(s)[:, None]
    torch.cuda.synchronize()
    fnlsim.quadrature_design(C, a, n, cidx=cidx)
    best = float("inf")
    for _ in range(3):
        t0 = time.perf_counter()
        nodes, err, _ = fnlsim.quadrature_design(C, a, n, cidx=cidx)
        best = min(best, time.perf_counter() - t0)
    del C, a
    # algorithmic bytes: each C_l read once (b = C a), then per step k the
    # gains read e per problem and (d, C_jj) per multipole; the update reads
    # the k earlier columns of the multipole's factor and row sel of C_l,
    # writes column k, updates d (per multipole) and e (per problem)
    pn = 8.0 * P * ntot
    sn = 8.0 * (L + 1) * ntot
    byts = 8.0 * (L + 1) * ntot * ntot + sum(3 * pn + sn * (k + 6) for k in range(n))
    return {"ms": round(best * 1e3, 3), "problems": P, "fine_shells": ntot, "nodes": n,
            "algorithmic_bytes": byts, "achieved_GBps": round(byts / best / 1e9, 1),
            "final_error_rel": float(err[-1] / (err[0] + 1e-300)),
            "error_curve_10_30_50_70": [float(err[k - 1]) for k in (10, 30, 50, 70)],
            "workload": "synthetic covariance of Eq. cov_phi on 400 fine shells over "
                        "[13000, 15000] Mpc, l = 0..1024 x (T, E) problems scaled to unit "
                        "a^T C a (T and E share C_l), 70 greedy nodes"}


def time_fwd_bwd(torch, fnlsim, inputs, precision, steps, warmup):
    """Forward + hand-written reverse pass per step at the differentiation
    workload (lmax 512, 96 nodes, 769 x 1536 grid), one realization."""
    import numpy as np
    cfg = inputs.CONFIGS["grad"]
    L, N = cfg["lmax"], cfg["nshell"]
    p = inputs.problem(L, N)
    sim = fnlsim.Simulator(L, p["r"], p["w"], p["filter"], p["alpha"], p["beta"],
                           n_ring=cfg["ntheta"], n_phi=cfg["nphi"], precision=precision)
    dt = torch.complex128 if precision == "fp64" else torch.complex64
    noise = torch.from_numpy(inputs.noise(L, N, inputs.realization_seed(0))).to(dt).cuda()
    rng = np.random.default_rng(3)
    gT = torch.from_numpy(rng.standard_normal((1, sim.n_lm)) + 1j * rng.standard_normal((1, sim.n_lm))).cuda()
    gE = torch.zeros_like(gT)
    stream = torch.cuda.current_stream()

    def step():
        sim.forward(noise, cfg["fnl"])
        sim.backward(noise, cfg["fnl"], gT, gE)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    # five Legendre transforms per step (forward synthesis and analysis; the
    # reverse pass's adjoint synthesis, Phi_L recomputation and adjoint
    # analysis), each 2 n_pair n_lm (2N) flop
    lflop = 5 * 2.0 * sim.n_pair * sim.n_lm * 2 * N
    peak = PEAK["fp64_mfma_TFs"] if precision == "fp64" else PEAK["fp32_mfma_TFs"]
    sim.close()
    return {"value": round(1000.0 / ms, 3), "unit": "fwd+bwd maps/s", "ms_per_step": round(ms, 4),
            "legendre_flop_per_step": lflop,
            "legendre_TFLOPs_over_whole_step": round(lflop / ms / 1e9, 2),
            "frac_of_mfma_peak_whole_step": round(lflop / ms / 1e9 / peak, 4),
            "workload": f"lmax={L}, {N} radial nodes, {cfg['ntheta']}x{cfg['nphi']} grid, "
                        f"gradients w.r.t. the noise and f_NL"}


def time_batch(torch, fnlsim, inputs, precision, steps, warmup):
    """Uneven batching workload: 32 realizations with lmax in {128, 256, 512,
    1024} and 64..200 nodes, one grouped graph-captured launch per stage,
    against the same 32 forward passes issued one after another."""
    mix = inputs.batch_mix()
    dt = torch.complex128 if precision == "fp64" else torch.complex64
    sims, noises, fnls = [], [], []
    t0 = time.time()
    probs = {}
    for i, (L, N) in enumerate(mix):
        if (L, N) not in probs:
            probs[(L, N)] = inputs.problem(L, N, device="cuda")
            log(f"batch input {i + 1}/{len(mix)}: lmax {L}, {N} nodes ({time.time() - t0:.0f} s)")
    log(f"batch inputs ready in {time.time() - t0:.1f} s")
    for i, (L, N) in enumerate(mix):
        p = probs[(L, N)]
        sims.append(fnlsim.Simulator(L, p["r"], p["w"], p["filter"], p["alpha"], p["beta"],
                                     precision=precision))
        noises.append(torch.from_numpy(inputs.noise(L, N, inputs.realization_seed(i))).to(dt).cuda())
        fnls.append(50.0)
    batch = fnlsim.Batch(sims)
    outs = batch.forward(noises, fnls)
    stream = torch.cuda.current_stream()

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    ms_b = timed(lambda: batch.forward(noises, fnls, outs))
    ms_s = timed(lambda: [s.forward(x, f) for s, x, f in zip(sims, noises, fnls)])
    # the batched result equals the per-context one
    worst = 0.0
    for s, x, f, o in zip(sims, noises, fnls, outs):
        aT, aE = s.forward(x, f)
        worst = max(worst, float((aT - o[0]).abs().max() / aT.abs().max()),
                    float((aE - o[1]).abs().max() / aE.abs().max()))
    batch.close()
    for s in sims:
        s.close()
    return {"realizations": len(mix), "batched_ms": round(ms_b, 3), "sequential_ms": round(ms_s, 3),
            "batched_maps_per_s": round(1000.0 * len(mix) / ms_b, 2),
            "sequential_maps_per_s": round(1000.0 * len(mix) / ms_s, 2),
            "speedup": round(ms_s / ms_b, 3), "max_rel_diff_vs_sequential": worst,
            "workload": "32 realizations, lmax in {128,256,512,1024}, 64..200 nodes "
                        "(default_rng(33)), n_theta = ceil((3L+1)/2), n_phi = 3L, f_NL = 50"}


def time_ksw(torch, fnlsim, inputs, p, cfg, aT, aE, precision, steps, warmup):
    """Cubic KSW statistic S_prim (Sect. 4) of one T+E realization at the
    paper workload: the filtered maps A and B of all 200 radial nodes (400
    syntheses on the 1537 x 3072 grid), the sky integral of A B^2 and the
    radial sum, per step."""
    L = cfg["lmax"]
    al, be, ci = inputs.ksw_tables(p)
    st = fnlsim.KswStatistic(L, p["r"], p["w"], al, be, ci, n_ring=cfg["ntheta"],
                             n_phi=cfg["nphi"], precision=precision)
    tT = torch.from_numpy(aT).cuda().reshape(1, -1)
    tE = torch.from_numpy(aE).cuda().reshape(1, -1)
    for _ in range(warmup):
        st(tT, tE)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        S = st(tT, tE)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    st.close()
    return {"ms": round(ms, 4), "statistics_per_s": round(1000.0 / ms, 3),
            "S_prim": float(S[0]), "precision": precision,
            "workload": f"lmax={L}, {len(p['r'])} radial nodes, {cfg['ntheta']}x{cfg['nphi']} grid"}


def time_tqu(torch, fnlsim, p, cfg, aT, aE, steps, warmup):
    """T, Q, U maps of one realization at the paper workload (FP64)."""
    L = cfg["lmax"]
    sim = fnlsim.Simulator(L, p["r"][:1], p["w"][:1], p["filter"][:, :1, :1], p["alpha"][:, :1],
                           p["beta"][:, :1], n_ring=cfg["ntheta"], n_phi=cfg["nphi"])
    tT = torch.from_numpy(aT).cuda().reshape(1, -1)
    tE = torch.from_numpy(aE).cuda().reshape(1, -1)
    for _ in range(warmup):
        sim.tqu_maps(tT, tE)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        sim.tqu_maps(tT, tE)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    sim.close()
    return {"ms": round(ms, 4), "realizations_per_s": round(1000.0 / ms, 2),
            "map_bytes": 3 * cfg["ntheta"] * cfg["nphi"] * 8,
            "workload": f"lmax={L}, T+Q+U on {cfg['ntheta']}x{cfg['nphi']} (FP64)"}


def per_l_rel_err(a, ref, L):
    import numpy as np
    ls = np.repeat(np.arange(L + 1), np.arange(1, L + 2))
    ms = np.arange(ls.size) - ls * (ls + 1) // 2
    c = np.where(ms == 0, 1.0, 2.0)
    num = np.sqrt(np.bincount(ls, weights=c * np.abs(a - ref) ** 2))
    den = np.sqrt(np.bincount(ls, weights=c * np.abs(ref) ** 2))
    ok = den > 1e-12 * den.max()
    return float(np.max(num[ok] / den[ok]))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _omp_threads(n):
    """Set the OpenMP thread count of the oracle's runtime (libgomp) for the
    following parallel regions; returns False if it cannot be set."""
    import ctypes
    try:
        gomp = ctypes.CDLL("libgomp.so.1")
        gomp.omp_set_num_threads(int(n))
        return True
    except OSError:
        return False


def cpu_baseline(p, cfg, noise_np, nsample, nsample1=1):
    """The FP64 oracle as it stands, on `nsample` of the N shells (transfer
    tables zeroed elsewhere: the oracle then evaluates only those shells).
    Work per shell is identical, so maps/s = 1 / (t * N / nsample).  Timed
    on every usable host thread, then on one thread with `nsample1` shells."""
    import numpy as np
    from oracle import fnl_oracle
    L, N = cfg["lmax"], cfg["nshell"]

    def run(ns):
        keep = np.linspace(N // 4, 3 * N // 4, ns).astype(int)
        al = np.zeros_like(p["alpha"])
        be = np.zeros_like(p["beta"])
        al[:, keep] = p["alpha"][:, keep]
        be[:, keep] = p["beta"][:, keep]
        P = fnl_oracle.Problem(L, p["r"], p["w"], p["filter"], al, be)
        fnl_oracle.lib()
        t0 = time.perf_counter()
        P.forward(noise_np, cfg["fnl"])
        return time.perf_counter() - t0

    try:
        threads = len(os.sched_getaffinity(0))
    except AttributeError:
        threads = os.cpu_count()
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or threads
    _omp_threads(threads)
    t = run(nsample)
    one = None
    if nsample1 and _omp_threads(1):
        t1 = run(nsample1)
        _omp_threads(threads)
        one = {"value": 1.0 / (t1 * N / nsample1), "unit": "maps/s", "cores": 1,
               "sample": f"{nsample1} of {N} shells in {t1:.1f} s, scaled by {N}/{nsample1}"}
    return {"value": 1.0 / (t * N / nsample), "unit": "maps/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{nsample} of {N} shells at lmax {L} (filter rows, synthesis, square, "
                      f"analysis and radial sums of those shells) in {t:.1f} s, scaled by "
                      f"{N}/{nsample}",
            "one_core": one,
            "paper_context": {"value": 8.3e-4, "unit": "maps/s",
                              "hardware": "one Intel Xeon core at 2.33 GHz",
                              "workload": "lmax 1024, HEALPix nside 512, 70 radial shells "
                                          "(about 20 minutes per T+E map)",
                              "shells_per_s": 0.058,
                              "note": "the paper's own timing, not the same workload "
                                      "(70 instead of 200 shells, HEALPix instead of the "
                                      "exact Gauss-Legendre grid): compare per shell"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="paper", choices=["paper", "medium", "grad", "tiny"])
    ap.add_argument("--cpu-shells", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fp32-only", action="store_true", help="skip the FP64 path (profiling runs)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="run one plain device copy of this many MiB first (counter calibration)")
    ap.add_argument("--no-grad", action="store_true", help="skip the fwd+bwd leg (lmax 512)")
    ap.add_argument("--no-quad", action="store_true",
                    help="skip the radial-quadrature design leg")
    ap.add_argument("--no-seeded", action="store_true",
                    help="skip the counter-based-noise forward leg")
    ap.add_argument("--no-split-bf16", action="store_true",
                    help="skip the split-BF16 forms of the Legendre transforms")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the uneven 32-realization batch leg")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the map generator runs on a single MI355X here; "
              "realizations shard across GPUs with no communication, so N > 1 is not measured.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_0909_0009_amd import fnlsim, inputs

    if args.calib_copy_mb:
        # a plain copy of known size: reads and writes exactly nbytes each
        nbytes = args.calib_copy_mb << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {nbytes} bytes read and written")
        del src, dst

    cfg = dict(inputs.CONFIGS[args.workload])
    L, N = cfg["lmax"], cfg["nshell"]
    t0 = time.time()
    p = inputs.problem(L, N)
    noise_np = inputs.noise(L, N, inputs.realization_seed(0))
    log(f"inputs ready in {time.time() - t0:.1f} s")

    r32 = time_path(torch, fnlsim, p, cfg, noise_np, "fp32", args.steps, args.warmup)
    log(f"fp32: {r32['ms']:.3f} ms/step")
    dom, roof = roofline(r32["sim"], r32["stages"], "fp32", args.steps)
    stages32 = {k: round(v[0] / max(v[1], 1), 4) for k, v in r32["stages"].items()}
    seeded = None
    if not args.no_seeded:
        seeded = {"fp32": time_seeded(torch, r32["sim"], cfg, args.steps, args.warmup)}
        log(f"seeded fp32: {seeded['fp32']['ms_per_step']:.3f} ms/step")
    r32["sim"].close()
    torch.cuda.empty_cache()
    fp64 = None
    err = None
    err_nl = None
    if not args.fp32_only:
        r64 = time_path(torch, fnlsim, p, cfg, noise_np, "fp64", args.steps, args.warmup)
        log(f"fp64: {r64['ms']:.3f} ms/step")
        dom64, roof64 = roofline(r64["sim"], r64["stages"], "fp64", args.steps)
        if seeded is not None:
            seeded["fp64"] = time_seeded(torch, r64["sim"], cfg, args.steps, args.warmup)
            log(f"seeded fp64: {seeded['fp64']['ms_per_step']:.3f} ms/step")
        fp64 = {"value": round(1000.0 / r64["ms"], 4), "ms_per_step": round(r64["ms"], 4),
                "shells_per_s": round(1000.0 / r64["ms"] * N, 2),
                "stages_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in r64["stages"].items()},
                "roofline": roof64}
        # error of the mixed path against the FP64 GPU path (which matches the
        # FP64 oracle to <= 1e-10 at this workload)
        err = max(per_l_rel_err(r32["aT"], r64["aT"], L), per_l_rel_err(r32["aE"], r64["aE"], L))
        err_nl = max(per_l_rel_err(r32["aT_nl"], r64["aT_nl"], L),
                     per_l_rel_err(r32["aE_nl"], r64["aE_nl"], L))
        r64["sim"].close()
        torch.cuda.empty_cache()
    split = None
    if not args.no_split_bf16:
        split = {}
        for pr in ("bf16x3", "bf16x6"):
            rb = time_path(torch, fnlsim, p, cfg, noise_np, pr, args.steps, args.warmup)
            split[pr] = split_bf16_leg(rb, r64 if fp64 is not None else None, pr, L)
            rb["sim"].close()
            del rb
            torch.cuda.empty_cache()
        log(f"split bf16: {split}")

    grad = None
    if not args.no_grad:
        grad = {"fp32": time_fwd_bwd(torch, fnlsim, inputs, "fp32", args.steps, args.warmup)}
        if not args.fp32_only:
            grad["fp64"] = time_fwd_bwd(torch, fnlsim, inputs, "fp64", args.steps, args.warmup)
        log(f"fwd+bwd: {grad}")
        torch.cuda.empty_cache()
    ksw = None
    tqu = None
    if args.workload == "paper":
        ksw = {pr: time_ksw(torch, fnlsim, inputs, p, cfg, r32["aT"], r32["aE"], pr, args.steps,
                            args.warmup) for pr in ("fp32", "fp64")}
        log(f"ksw: {ksw}")
        tqu = time_tqu(torch, fnlsim, p, cfg, r32["aT"], r32["aE"], args.steps, args.warmup)
        log(f"tqu: {tqu}")
        torch.cuda.empty_cache()
    quad = None
    if not args.no_quad:
        quad = time_quadrature(torch, fnlsim, inputs)
        log(f"quadrature design: {quad['ms']} ms")
        torch.cuda.empty_cache()
    batch = None
    if not args.no_batch:
        batch = {"fp32": time_batch(torch, fnlsim, inputs, "fp32", args.steps, args.warmup)}
        log(f"batch: {batch}")
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(p, cfg, noise_np, args.cpu_shells)
        log(f"cpu baseline: {cpu['value']:.3e} maps/s on {cpu['cores']} threads")

    value = 1000.0 / r32["ms"]
    line = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "maps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r32["ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: lmax={L}, {N} radial nodes, "
                               f"{cfg['ntheta']}x{cfg['nphi']} Gauss-Legendre grid, "
                               f"1 T+E realization per step, f_NL={cfg['fnl']}",
                   "precision": "fp32 matrix cores; fp64 recurrence, mean and radial sums"},
        "shells_per_s": round(value * N, 2),
        "stages_ms": stages32,
        "roofline": roof,
        "fp64": fp64,
        "mixed_vs_fp64_max_rel_err": err,
        "mixed_vs_fp64_nl_max_rel_err": err_nl,
        "split_bf16": split,
        "seeded": seeded,
        "ksw_cubic_statistic": ksw,
        "tqu_maps": tqu,
        "quadrature_design": quad,
        "fwd_bwd": grad,
        "batch": batch,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
