"""Throughput of the interpolation + Im Sigma hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: the realistic fcc system (2 atoms, 8 Wannier bands, 6 modes,
6^3 coarse grid -> 279 Wigner-Seitz vectors each for electrons and phonons,
fine 20^3 k x 20^3 q = 6.4e7 k.q pairs, T = 300 K, sigma = 20 meV, mu at
mid-gap + 0.1 eV), synthetic seeded inputs resident in HBM before the timed
region.  A step is one epw_imsigma call over all pairs: phases, every
eigensolve, both contractions, both rotations and the reduction.

The headline value is the float64 forward; the float32 (and, where built,
split-bf16) forward and the backward are reported alongside.  One JSON line
goes to stdout.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "k·q pairs/sec for interp+Im Σ_nk (FP64 vs FP32/split-BF16) and backward, 1 GPU"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "split_bf16": 2500.0}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def setup(device):
    from paper_1604_03525_amd import epw
    from paper_1604_03525_amd import inputs as I
    m = I.realistic_model()
    R, nd = epw.epw_ws_vectors(m.metric, m.coarse)
    HR, DR, gR = I.realistic_arrays(R, R)
    k = epw.epw_grid_points(m.kgrid)
    kq = epw.epw_kq_index(m.kgrid, m.qgrid)
    sysd = epw.System(R, nd, R, nd, HR, DR, gR, device)
    pts = epw.Points(k, k, kq, device=device)
    return m, sysd, pts, (R, nd, HR, DR, gR, k)


def mfma_issue_rate(nk, nq, ne, nm, nb, ms, bk, folded=False):
    """TFLOP/s the matrix units execute in the fused kernel's R_e -> k sum on
    the padded band blocks: unfolded, three real products per complex product
    (6 MFMA flops per 8 algorithmic ones) over K = N_e padded to the K step
    bk; folded by pairs (R, -R) (a set closed under R -> -R, as Wigner-Seitz
    sets are), four real products per entry of the halved sum (8 MFMA flops)
    over K = (N_e + 1) / 2 padded to bk."""
    nbp = 1
    while nbp < nb:
        nbp *= 2
    k = (ne + 1) // 2 if folded else ne
    kp = (k + bk - 1) // bk * bk
    return (8.0 if folded else 6.0) * nk * nq * kp * nm * nbp * nbp / (ms * 1e-3) / 1e12


def fused_flops(nk, nq, ne, nm, nb):
    """Algorithmic flops of the dominant kernel over all its launches:
    the R_e -> k contraction (8 flops per complex multiply-add) plus the
    two n_b x n_b rotations per (k, q, nu)."""
    return 8.0 * nk * nq * ne * nm * nb * nb + 16.0 * nk * nq * nm * nb ** 3


def timed(fn, steps, warmup, torch):
    from paper_1604_03525_amd import epw
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    epw.epw_timing_enable(True)
    t0 = time.perf_counter()
    for i in range(steps):
        fn()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stages = {}
    for name, sid in (("eigh", 0), ("gemm_rp", 1), ("moderot", 2), ("fused", 3), ("backward", 4),
                      ("spectral", 5), ("pair_gemm", 6), ("pair_eigh", 7), ("bwd_gemm", 8)):
        ms, n = epw.epw_timing_read(sid)
        stages[name] = (ms, n)
    epw.epw_timing_enable(False)
    return dt, stages


# HBM traffic of the dominant kernel, from the rocprofv3 FETCH_SIZE / WRITE_SIZE
# counters recorded in this profile (scaled by the counts of a plain 1 GiB
# device copy, see --copy-calibration).  It describes the kernel sources whose
# hash it records: once those change, the figure is reported as null.
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "fused_k_kernel_fcc20.md")
MOBILITY_PROFILE = os.path.join(ROOT, "profiles", "fused_k_kernel_mobility_shard.md")
TRAFFIC_SOURCES = ["paper_1604_03525_amd/csrc/k_vertex.hip", "paper_1604_03525_amd/csrc/cgemm.h",
                   "paper_1604_03525_amd/csrc/api.cpp"]


def sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def recorded_traffic(dtype, profile=None):
    """Bytes per launch of the fused kernel for `dtype` (from `profile`, by
    default the fcc 20^3 record), or None when the profile is missing or was
    taken on other kernel sources."""
    if profile is None:
        profile = TRAFFIC_PROFILE
    try:
        with open(profile) as f:
            for line in f:
                if line.startswith("traffic-record: "):
                    rec = json.loads(line[len("traffic-record: "):])
                    if rec.get("sources_sha256") != sources_sha256():
                        return None
                    return rec.get("bytes_per_launch", {}).get(dtype)
    except (OSError, ValueError):
        return None
    return None


def copy_calibration(torch):
    """A plain device copy of 1 GiB (two launches): the reference dispatch
    whose FETCH_SIZE / WRITE_SIZE counts calibrate the traffic counters."""
    x = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(2):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": x.numel() * 4}), flush=True)


def peak_gemm(torch, n=8192, reps=10):
    """Library GEMM rates (torch.matmul, n x n x n) in FP64, FP32 and BF16: a
    check of the datasheet MFMA peaks used as roofline denominators."""
    out = {}
    for name, dt in (("fp64", torch.float64), ("fp32", torch.float32), ("bf16", torch.bfloat16)):
        a = torch.randn(n, n, device="cuda:0").to(dt)
        b = torch.randn(n, n, device="cuda:0").to(dt)
        c = a @ b
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            c = a @ b
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name] = {"ms": ms, "tflops": 2.0 * n ** 3 / (ms * 1e-3) / 1e12}
        log("bench: peak gemm %s %.2f TFLOP/s" % (name, out[name]["tflops"]))
        del a, b, c
    print(json.dumps({"peak_gemm": out, "n": n}), flush=True)


def backward_gemm_flops(nk, nq, ne, np_, nm, nb):
    """Algorithmic flops of the adjoint's contractions (8 per complex
    multiply-add): the recomputed R_p -> q and R_e -> k products, their two
    conjugate-transposed sums (over k for dL/dg_nu(R_e,q), over q for
    dL/dg(R_e,R_p)) and the k-set sum of dL/dH(R_e)."""
    a5 = 8.0 * nq * np_ * ne * nm * nb * nb
    a7 = 8.0 * nk * nq * ne * nm * nb * nb
    return 2.0 * (a5 + a7) + 8.0 * ne * nk * nb * nb


def pair_eigh_flops(n):
    """Arithmetic of one n x n complex Jacobi sweep of the two-sided method
    (flops = real additions and multiplications): each of the n(n-1)/2
    rotations of a sweep rewrites two rows and two columns of A (4n complex
    entries, each 2 complex-by-real products, one complex phase product and
    one complex addition: 14 flops) and two columns of V (2n entries, 14 flops
    each).  The eigensolver computes only the half of A above the diagonal and
    mirrors it, so it executes about two thirds of this count."""
    return n * (n - 1) / 2 * (4 * n + 2 * n) * 14.0


def mobility_shard(dev, dtypes, bwd_dtypes, steps, warmup, torch):
    """One 4096-q chunk of the mobility-scale system, i.e. the per-GPU shard of
    a q-sharded run: fcc, 3 atoms, 16 bands, 9 modes, 617 + 617 WS vectors,
    8000 k in the 0.3 eV window above the conduction band minimum x the first
    4096 of 125,000 random q, off-grid k+q (H interpolated and diagonalised per
    pair), normalised by N_q = 125,000.  H and D carry the scale constants of
    the model (12 eV bandwidth and a 65 meV top phonon on the coarse grid; mu
    mid-gap on a 40^3 grid).  g(R_e,R_p) (14 GB) is drawn on the device."""
    import numpy as np
    from paper_1604_03525_amd import epw
    from paper_1604_03525_amd import inputs as I
    m = I.mobility_model()
    x = m.extra
    R, nd = epw.epw_ws_vectors(m.metric, m.coarse)
    H0, D0 = I.mobility_arrays(R)
    Ht = torch.as_tensor(H0, device=dev)
    Dt = torch.as_tensor(D0, device=dev)
    cbm, mu = I.C5_CBM, I.C5_MU
    cand = I.mobility_k_candidates(65536, x["seed_k"])
    e, _ = epw.epw_interp_bands(Ht, R, nd, cand)
    mask = ((e >= cbm) & (e <= cbm + x["window"])).any(dim=1).cpu().numpy()
    k = cand[mask][: x["nk"]]
    q = I.random_points(x["nq"], x["seed_q"])[: x["chunk"]]
    gR = I.random_vertex_device(R, R, m.vectors, m.nm, m.nb, seed=x["seed_g"], g0=0.05, decay=1.0, device=dev)
    sysd = epw.System(R, nd, R, nd, Ht, Dt, gR, dev)
    del gR
    pts = epw.Points(k, q, None, device=dev)
    ws = epw.Workspace(dev)
    pairs = len(k) * len(q)
    out = {"workload": "mobility-scale shard: fcc 3 atoms, nb=16, nm=9, WS 617+617, %d window k x %d random q "
                       "(the first chunk of %d), off-grid k+q, T=300 K, sigma=10 meV" % (len(k), len(q), x["nq"]),
           "nk": len(k), "nq": len(q), "pairs": pairs, "mu_eV": mu, "cbm_eV": cbm}
    ff = fused_flops(len(k), len(q), len(R), m.nm, m.nb)
    for dt in dtypes:
        log("bench: mobility shard %s forward" % dt)
        par = epw.make_params(T=m.T, mu=mu, sigma=m.sigma, nq_norm=float(x["nq"]), dtype=dt)
        dtv, stv = timed(lambda: epw.epw_imsigma(sysd, pts, par, workspace=ws), steps, warmup, torch)
        fms, fnn = stv["fused"]
        ach = ff * steps / (fms * 1e-3) / 1e12 if fms > 0 else None
        gms, gn = stv["pair_gemm"]
        ems, en = stv["pair_eigh"]
        eig_tf = pairs * steps * 7.0 * pair_eigh_flops(m.nb) / (ems * 1e-3) / 1e12 if ems > 0 else None
        rec = {"value": pairs * steps / dtv, "unit": "k·q pairs/s", "ms_per_step": 1e3 * dtv / steps,
               "roofline": {"bound": "mfma", "kernel": "fused_k_kernel", "achieved": ach,
                            "peak": PEAK_TFLOPS[dt], "unit": "TFLOP/s",
                            "frac": ach / PEAK_TFLOPS[dt] if ach else None,
                            "traffic": recorded_traffic(dt, MOBILITY_PROFILE),
                            "launches": fnn, "avg_launch_ms": fms / fnn if fnn else None},
               "pair_states_ms_per_step": {"h_kq_gemm": gms / steps, "eigh": ems / steps},
               "pair_eigh_fp64_valu": {"achieved": eig_tf, "peak": PEAK_TFLOPS["fp64"], "unit": "TFLOP/s",
                                       "frac": eig_tf / PEAK_TFLOPS["fp64"] if eig_tf else None,
                                       "count": "7 Jacobi sweeps of pair_eigh_flops(16) per pair"},
               "stages_ms_per_step": {s_: v[0] / steps for s_, v in stv.items()}}
        if dt == "split_bf16" and ach:
            rec["roofline"]["frac_of_split_peak"] = ach / (PEAK_TFLOPS[dt] / 3.0)
        out[dt] = rec
    w = torch.rand((len(k), m.nb), dtype=torch.float64, device=dev, generator=torch.Generator(device=dev).manual_seed(1))
    for dt in bwd_dtypes:
        log("bench: mobility shard %s backward" % dt)
        par = epw.make_params(T=m.T, mu=mu, sigma=m.sigma, nq_norm=float(x["nq"]), dtype=dt)
        dtb, stb = timed(lambda: epw.epw_imsigma_backward(sysd, pts, par, w, workspace=ws), 1, 0, torch)
        out["backward_" + dt] = {"value": pairs / dtb, "unit": "k·q pairs/s", "ms_per_step": 1e3 * dtb,
                                 "outputs": "dL/dg(R_e,R_p), dL/dH(R_e), dL/domega",
                                 "stages_ms_per_step": {s_: v[0] for s_, v in stb.items()}}
    for s_ in ("fp32", "split_bf16"):
        if s_ in out and "fp64" in out:
            out[s_]["speedup_vs_fp64"] = out[s_]["value"] / out["fp64"]["value"]
    del sysd
    torch.cuda.empty_cache()
    return out


def spectral_flops(nk, nq, nw, nm, nb):
    """Algorithmic flops of the frequency-resolved sum (Eq. (3) on a grid):
    per (k, pole family (q, nu, m), frequency incl. omega = 0) 14 flops for the
    two complex poles (two subtractions, two x^2 + d^2, two reciprocals, the
    weights and the real and imaginary sums) plus a complex update of every
    band n (4 flops)."""
    return float(nk) * (nw + 1) * nq * nm * nb * (14.0 + 4.0 * nb)


def spectral_run(sysd, model, dev, steps, warmup, torch):
    """Frequency-resolved Sigma_nk(omega) (Eq. (3)) and A_nk(omega)
    (Eq. (10)) on the spectral workload: the realistic system, 64 k on
    Gamma-X, 10^5 random q (off-grid k+q), 512 frequencies, FP64."""
    from paper_1604_03525_amd import epw
    from paper_1604_03525_amd import inputs as I
    wl = I.spectral_workload()
    pts = epw.Points(wl["k"], wl["q"], None, device=dev)
    w = torch.as_tensor(wl["wgrid"], device=dev)
    par = epw.make_params(T=model.T, mu=model.mu, sigma=model.sigma)
    ws = epw.Workspace(dev)
    nk, nq, nw = len(wl["k"]), len(wl["q"]), len(wl["wgrid"])
    log("bench: spectral function (%d k x %d q x %d frequencies)" % (nk, nq, nw))
    dt, st = timed(lambda: epw.spectral_function(sysd, pts, par, w, workspace=ws), steps, warmup, torch)
    sms, sn = st["spectral"]
    fl = spectral_flops(nk, nq, nw, sysd.nm, sysd.nb) * steps
    ach = fl / (sms * 1e-3) / 1e12 if sms > 0 else None
    return {"value": nk * nq * steps / dt, "unit": "k·q pairs/s", "ms_per_step": 1e3 * dt / steps,
            "dtype": "fp64", "workload": "realistic fcc system, %d k on Gamma-X x %d random q (off-grid k+q), "
                                         "%d frequencies on [-1, 1] eV, delta = 20 meV" % (nk, nq, nw),
            "outputs": "Sigma_nk(omega) complex (Eq. 3), Sigma_nk(0), A_nk(omega) (Eq. 10)",
            "spectral_kernel": {"kernel": "sigma_omega_kernel", "bound": "alu", "achieved": ach,
                                "peak": PEAK_TFLOPS["fp64"], "unit": "TFLOP/s",
                                "frac": ach / PEAK_TFLOPS["fp64"] if ach else None,
                                "launches": sn, "avg_launch_ms": sms / sn if sn else None},
            "stages_ms_per_step": {s_: v[0] / steps for s_, v in st.items()}}


def cpu_baseline(host, model, seconds_target=15.0):
    """The FP64 oracle on a bounded sample: a few k points against all q."""
    import numpy as np
    from threadpoolctl import threadpool_info
    from oracle import selfenergy
    R, nd, HR, DR, gR, k = host
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    nk_s = 0
    t0 = time.perf_counter()
    rng = np.random.default_rng(0)
    idx = rng.choice(len(k), 64, replace=False)
    while time.perf_counter() - t0 < seconds_target and nk_s < 64:
        selfenergy.imsigma(HR, R, nd, DR, R, nd, gR, k[idx[nk_s:nk_s + 1]], k, model.T, model.mu,
                           model.sigma)
        nk_s += 1
    dt = time.perf_counter() - t0
    pairs = nk_s * len(k)
    # the same oracle on one BLAS thread, one k point against all q
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        t1 = time.perf_counter()
        selfenergy.imsigma(HR, R, nd, DR, R, nd, gR, k[idx[:1]], k, model.T, model.mu, model.sigma)
        dt1 = time.perf_counter() - t1
    cpu = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next(l.split(":", 1)[1].strip() for l in f if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {"value": pairs / dt, "unit": "k·q pairs/s", "cores": int(threads), "kind": "oracle",
            "sample": "%d k points x all %d q of the same workload (%.1f s, FP64 NumPy, %s, %d CPUs visible)"
                      % (nk_s, len(k), dt, cpu, os.cpu_count() or 0),
            "single_thread": {"value": len(k) / dt1, "unit": "k·q pairs/s", "cores": 1,
                              "sample": "1 k point x all %d q (%.1f s)" % (len(k), dt1)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--variants",
                    default="fp32,split_bf16,backward,backward_fp32,backward_split_bf16,mobility,phonon,resigma,"
                            "polar,transport,spectral",
                    help="comma list of fp32, split_bf16, backward, backward_fp32, backward_split_bf16, mobility "
                         "(one 4096-q shard of the mobility-scale system), mobility_forward (its forward legs "
                         "only), phonon, resigma, polar, transport, spectral")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration) and exit")
    ap.add_argument("--peak-gemm", action="store_true",
                    help="only time library GEMMs (8192^3, FP64 / FP32 / BF16) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (a sharded run "
              "would give each GPU whole q chunks and sum the partial Im Sigma once); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1604_03525_amd import epw
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(torch)
        return
    if args.peak_gemm:
        peak_gemm(torch)
        return
    dev = torch.device("cuda:0")
    model, sysd, pts, host = setup(dev)
    nk, nq = pts.k.shape[0], pts.q.shape[0]
    ne, nm, nb = sysd.Re.shape[0], sysd.nm, sysd.nb
    pairs = nk * nq
    ws = epw.Workspace(dev)

    def run(dtype):
        par = epw.make_params(T=model.T, mu=model.mu, sigma=model.sigma, dtype=dtype)
        out = torch.empty((nk, nb), dtype=torch.float64, device=dev)
        return lambda: epw.epw_imsigma(sysd, pts, par, out=out, workspace=ws)

    log("bench: fp64 forward, %d steps after %d warmup" % (args.steps, args.warmup))
    dt, st = timed(run("fp64"), args.steps, args.warmup, torch)
    ms_step = 1e3 * dt / args.steps
    value = pairs * args.steps / dt
    fms, fn = st["fused"]
    flops = fused_flops(nk, nq, ne, nm, nb) * args.steps
    achieved = flops / (fms * 1e-3) / 1e12 if fms > 0 else None
    result = {
        "metric": METRIC, "value": value, "unit": "k·q pairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded random fcc model, see paper_1604_03525_amd/inputs.py)",
        "config": {"workload": "fcc 2 atoms, nb=8, nm=6, WS 279+279, 20^3 k x 20^3 q grid, "
                               "T=300 K, sigma=20 meV, FP64 forward",
                   "nk": nk, "nq": nq, "pairs": pairs, "nb": nb, "nm": nm, "nRe": ne,
                   "parallelism": "1 GPU"},
        "roofline": {"bound": "mfma", "kernel": "fused_k_kernel (R_e->k contraction + rotation + reduction)",
                     "achieved": achieved, "peak": PEAK_TFLOPS["fp64"], "unit": "TFLOP/s",
                     "frac": (achieved / PEAK_TFLOPS["fp64"]) if achieved else None,
                     "traffic": recorded_traffic("fp64"),
                     "launches": fn, "avg_launch_ms": fms / fn if fn else None,
                     "convention": "achieved = algorithmic flops (8 per complex multiply-add of the R_e->k sum, "
                                   "plus the two band rotations) per second; the kernel sums over the pairs "
                                   "(R, -R) of the Wigner-Seitz set, c B+ + i s B- per pair with two real "
                                   "MFMAs per R vector (4 MFMA flops per 8 algorithmic), so frac can reach 2; "
                                   "mfma_issue_frac is the matrix units' own rate",
                     "mfma_issue_frac": mfma_issue_rate(nk, nq, ne, nm, nb, fms / args.steps, 8, folded=True)
                     / PEAK_TFLOPS["fp64"] if fms > 0 else None},
        "stages_ms_per_step": {k: v[0] / args.steps for k, v in st.items()},
    }
    variants = {}
    # secondary variants (everything but the precisions of the headline
    # forward) take at most 3 timed steps after at most 1 warm-up, so the
    # default run stays within a few minutes
    ksteps, kwarm = min(args.steps, 3), min(args.warmup, 1)
    kflops = fused_flops(nk, nq, ne, nm, nb) * ksteps
    for var in [v for v in args.variants.split(",") if v]:
        try:
            if var in ("fp32", "split_bf16"):
                log("bench: %s forward" % var)
                dtv, stv = timed(run(var), args.steps, args.warmup, torch)
                fmsv, fnv = stv["fused"]
                ach = flops / (fmsv * 1e-3) / 1e12 if fmsv > 0 else None
                variants[var] = {"value": pairs * args.steps / dtv, "ms_per_step": 1e3 * dtv / args.steps,
                                 "speedup_vs_fp64": (pairs * args.steps / dtv) / value,
                                 "fused_tflops": ach, "fused_frac_of_peak": ach / PEAK_TFLOPS[var] if ach else None,
                                 "fused_avg_launch_ms": fmsv / fnv if fnv else None,
                                 "fused_traffic": recorded_traffic(var)}
                if var == "split_bf16" and ach:
                    # three BF16 products per real product: 24 MFMA flops per complex
                    # multiply-add (8 algorithmic), so the split form tops out at 1/3 of the
                    # BF16 peak in algorithmic flops; also the rate against the FP32 peak
                    variants[var]["fused_frac_of_split_peak"] = ach / (PEAK_TFLOPS[var] / 3.0)
                    variants[var]["effective_fp32_frac"] = ach / PEAK_TFLOPS["fp32"]
            elif var in ("backward", "backward_fp32", "backward_split_bf16"):
                bdt = {"backward": "fp64", "backward_fp32": "fp32", "backward_split_bf16": "split_bf16"}[var]
                log("bench: %s backward" % bdt)
                par = epw.make_params(T=model.T, mu=model.mu, sigma=model.sigma, dtype=bdt)
                w = torch.rand((nk, nb), dtype=torch.float64, device=dev)
                dtb, stb = timed(lambda: epw.epw_imsigma_backward(sysd, pts, par, w, workspace=ws),
                                 ksteps, kwarm, torch)
                bms, bn = stb["bwd_gemm"]
                bfl = backward_gemm_flops(nk, nq, ne, ne, nm, nb) * ksteps
                bach = bfl / (bms * 1e-3) / 1e12 if bms > 0 else None
                bpeak = PEAK_TFLOPS["fp64" if bdt == "fp64" else "fp32"]
                variants[var] = {"value": pairs * ksteps / dtb, "ms_per_step": 1e3 * dtb / ksteps,
                                 "steps": ksteps, "dtype": bdt,
                                 "outputs": "dL/dg(R_e,R_p), dL/dH(R_e), dL/domega",
                                 "ratio_to_forward": (1e3 * dtb / ksteps) / ms_step if bdt == "fp64" else None,
                                 "roofline": {"bound": "mfma",
                                              "kernel": "adjoint contractions (%s)"
                                              % ("cgemm_generic_kernel, bf16_gemm_kernel" if bdt == "split_bf16"
                                                 else "fused_k_kernel recompute, ksum_fold_kernel, "
                                                      "cgemm_generic_kernel"),
                                              "convention": None if bdt == "split_bf16" else
                                              "algorithmic flops (8 per complex multiply-add); the R_e <-> k "
                                              "sums run folded by the pairs (R, -R) with two real MFMAs per "
                                              "R vector, so frac can exceed 1",
                                              "achieved": bach, "peak": bpeak, "unit": "TFLOP/s",
                                              "frac": bach / bpeak if bach else None, "traffic": None,
                                              "launches": bn, "gemm_ms_per_step": bms / ksteps,
                                              "peak_note": "split-bf16 runs its R_p <-> q sums in float32: "
                                                           "rated against the float32 peak" if bdt == "split_bf16"
                                              else None},
                                 "stages_ms_per_step": {s_: v[0] / ksteps for s_, v in stb.items()}}
            elif var == "phonon":
                log("bench: phonon linewidth and lambda (fp64)")
                par = epw.make_params(T=model.T, mu=model.mu, sigma=model.sigma)
                dtp, stp = timed(lambda: epw.epw_phonon_selfenergy(sysd, pts, par, workspace=ws),
                                 ksteps, kwarm, torch)
                fmsp, fnp = stp["fused"]
                achp = kflops / (fmsp * 1e-3) / 1e12 if fmsp > 0 else None
                variants[var] = {"value": pairs * ksteps / dtp, "ms_per_step": 1e3 * dtp / ksteps,
                                 "dtype": "fp64", "outputs": "Pi''_q,nu (Eq. 9) and lambda_q,nu (Eq. 11)",
                                 "fused_tflops": achp, "fused_frac_of_peak": achp / PEAK_TFLOPS["fp64"] if achp else None}
            elif var == "resigma":
                log("bench: on-shell Re Sigma and Sigma~' (fp64)")
                par = epw.make_params(T=model.T, mu=model.mu, sigma=model.sigma)
                dtr, str_ = timed(lambda: epw.epw_resigma(sysd, pts, par, workspace=ws),
                                  ksteps, kwarm, torch)
                fmsr, fnr = str_["fused"]
                achr = kflops / (fmsr * 1e-3) / 1e12 if fmsr > 0 else None
                variants[var] = {"value": pairs * ksteps / dtr, "ms_per_step": 1e3 * dtr / ksteps,
                                 "dtype": "fp64", "outputs": "Sigma'_nk on shell (Eq. 3) and Sigma~'_nk (Eq. 5)",
                                 "fused_tflops": achr, "fused_frac_of_peak": achr / PEAK_TFLOPS["fp64"] if achr else None}
            elif var == "transport":
                log("bench: transport coupling lambda_tr with lambda and Pi'' (fp64)")
                from paper_1604_03525_amd import inputs as I
                # eps_F 0.3 eV into the valence bands (the headline mu is mid-gap)
                par = epw.make_params(T=model.T, mu=model.mu - 0.3, sigma=0.05)
                dtt, stt = timed(lambda: epw.epw_transport_coupling(sysd, pts, par, I.FCC_VECTORS, want_pi=True,
                                                                    workspace=ws), ksteps, kwarm, torch)
                fmst, fnt = stt["fused"]
                acht = kflops / (fmst * 1e-3) / 1e12 if fmst > 0 else None
                variants[var] = {"value": pairs * ksteps / dtt, "ms_per_step": 1e3 * dtt / ksteps,
                                 "dtype": "fp64", "outputs": "lambda_tr (Eq. 55), lambda (Eq. 11), Pi'' (Eq. 9)",
                                 "mu_shift_eV": -0.3, "sigma_eV": 0.05,
                                 "fused_tflops": acht, "fused_frac_of_peak": acht / PEAK_TFLOPS["fp64"] if acht else None}
            elif var == "polar":
                log("bench: fp64 forward with the polar long-range term")
                from paper_1604_03525_amd import inputs as I
                R_, nd_, HR_, DR_, gR_, _ = host
                sysp = epw.System(R_, nd_, R_, nd_, HR_, DR_, gR_, dev, polar=I.polar_params())
                par = epw.make_params(T=model.T, mu=model.mu, sigma=model.sigma)
                outp = torch.empty((nk, nb), dtype=torch.float64, device=dev)
                dtq, stq = timed(lambda: epw.epw_imsigma(sysp, pts, par, out=outp, workspace=ws), ksteps,
                                 kwarm, torch)
                variants[var] = {"value": pairs * ksteps / dtq, "ms_per_step": 1e3 * dtq / ksteps,
                                 "dtype": "fp64", "outputs": "Im Sigma_nk with g = g^S + g^L (Sec. 4)",
                                 "stages_ms_per_step": {s_: v[0] / ksteps for s_, v in stq.items()}}
                del sysp
            elif var == "spectral":
                variants[var] = spectral_run(sysd, model, dev, ksteps, kwarm, torch)
            elif var == "mobility":
                variants[var] = mobility_shard(dev, ("fp64", "fp32", "split_bf16"), ("fp32", "split_bf16"), 1, 0,
                                               torch)
            elif var == "mobility_forward":
                variants[var] = mobility_shard(dev, ("fp64", "fp32", "split_bf16"), (), 1, 0, torch)
        except epw.EpwError as e:
            variants[var] = {"unavailable": str(e)}
    result["variants"] = variants
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle sample)")
        result["cpu_baseline"] = cpu_baseline(host, model)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
