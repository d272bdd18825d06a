"""Throughput benchmark: detector-samples/s of the full simulation on one GPU.

One step = one gtod_simulate_tod call covering the whole observation of the
workload: the PINK job (1/f noise for every (pixel, channel) series,
written into the TOD) and the SIGNAL job (pointing, screen, table +
airmass, cascade, filterbank contraction, photon noise) over every
(pixel, sample), added into it.
Inputs (screen, tables, filter matrices, source cube) are resident in HBM
before the timed region; outputs stay in HBM.

Prints one JSON line.  See `python bench.py --help`.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("detector-samples/s (t×pix×chan) at ≤1e-6 rel err vs "
          "FP64; p50/p99 request ms")
PEAK = {"fp32": 157.3e12, "split": 2.5e15}   # dense MFMA FLOP/s (MI355X)
HBM_PEAK = 8.0e12
SKYDIP_PWV = (0.25, 2.75)
ARCSEC = 3.141592653589793 / 180.0 / 3600.0
REDUCE_R_OUT = 30 * ARCSEC       # outer ring of the 7x7 grid is off source
REDUCE_MAP = (31, 150 * ARCSEC)  # nodes per axis, half extent

WORKLOADS = {
    "c2": "single-pixel spectrometer: 1 px raster +-60\" at 0.5 deg/s, "
          "347-channel filterbank R=500 220-440 GHz, 3000 bins, 600 s at "
          "160 Hz (96000 samples), 512x65536 PWV screen, 6-stage cascade, "
          "Gaussian source with 350 GHz line, photon + 1/f noise",
    "c3": "IFU: 7x7 = 49 px at 12\" pitch, daisy r=90\", 347-channel "
          "filterbank R=500 220-440 GHz, 3000 bins, 1 h at 160 Hz (576000 "
          "samples), 1024x262144 PWV screen, 6-stage cascade, Gaussian "
          "source with 350 GHz line, photon + 1/f noise (knee 1 Hz, alpha 1)",
    "c4": "IFU as c3 plus a faint 60\" Gaussian source (1e-4 of the "
          "loading), split hi+lo BF16 contraction",
    "c5": "serving stream: 256 seeded requests, Poisson arrivals 20/s, "
          "pixels in {1,7,19 hex; 49 square}, channels in {64,347,720}, "
          "bins 1000-4000, 10-600 s at 160 Hz, 4 shared resident "
          "512x65536 screens, daisy, HBM-budget admission, split BF16, "
          "continuous batching over 4 streams",
}


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default=None, choices=["fp32", "split"])
    ap.add_argument("--workspace-gib", type=float, default=8.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--kelvin", type=int, default=0, metavar="N",
                    help="output in kelvin: calibrate by an N-point skydip "
                         "(PWV 0.25-2.75 mm at the scan elevation) before "
                         "the timed steps")
    ap.add_argument("--to-disk", default=None, metavar="DIR",
                    help="instead of the in-HBM steps, time one out-of-core "
                         "run (gtod_simulate_to_disk) of the workload cut "
                         "to --disk-seconds, written to DIR (removed after)")
    ap.add_argument("--disk-seconds", type=float, default=360.0)
    ap.add_argument("--prep", action="store_true",
                    help="time the input preparation instead: source-beam "
                         "convolution of the 121x121x3000 intensity cube and "
                         "footprint smoothing of the 1024x262144 screen")
    ap.add_argument("--reduce", action="store_true",
                    help="after the simulation steps, time gtod_reduce "
                         "(common-mode subtraction + 31x31 inverse-variance "
                         "maps) on the Kelvin TOD; needs --kelvin")
    ap.add_argument("--headline-only", action="store_true",
                    help="with the default c3 workload, skip the c4 "
                         "(split BF16) and c5 (serving) measurements that "
                         "the JSON line otherwise carries beside it")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 1 GiB device copy first (counter "
                         "calibration for HBM byte counts)")
    return ap.parse_args()


def scenario(name):
    from workloads import configs
    return {"c2": configs.c2, "c3": configs.c3, "c4": configs.c4}[name]()


def _cores():
    """Threads the oracle's BLAS/FFT pools use."""
    try:
        import numpy  # noqa: F401  (loads the BLAS pool)
        from threadpoolctl import threadpool_info
        return int(max([i.get("num_threads", 1) for i in threadpool_info()]
                       or [1]))
    except Exception:  # pragma: no cover
        return os.cpu_count() or 1


def cpu_baseline(sc, target_s):
    """The FP64 oracle, as it is, on a bounded sample of the same workload:
    all pixels over a window of samples in the middle of the observation,
    plus two full 1/f series; scaled to detector-samples/s."""
    import oracle
    threads = _cores()
    mid = sc.t_total // 2
    # size the window from the marginal cost per sample (each call also
    # rebuilds the oracle's channel responses, a fixed cost)
    t0 = time.perf_counter()
    oracle.tod.simulate(sc, mid, mid + 8)
    t8 = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.tod.simulate(sc, mid, mid + 40)
    t40 = time.perf_counter() - t0
    per_sample = max((t40 - t8) / 32, 1e-6)
    n = int(max(40, min(sc.t_total - mid,
                        (target_s * 0.85 - t8) / per_sample)))
    t0 = time.perf_counter()
    oracle.tod.simulate(sc, mid, mid + n)
    t_sig = time.perf_counter() - t0
    nep2 = oracle.tod.reference_nep2(sc)
    A = oracle.pink.amplitude(nep2, sc.pink_alpha, sc.pink_knee_hz)
    t0 = time.perf_counter()
    for k in (0, sc.K - 1):
        oracle.pink.series(sc.seed, 0, k, A[k], sc.pink_alpha[k], sc.t_total,
                           sc.f_sample_hz)
    t_pink_series = (time.perf_counter() - t0) / 2
    det = sc.n_pix * sc.K * n
    per_det = t_sig / det + t_pink_series / sc.t_total
    return {"value": 1.0 / per_det, "unit": "detector-samples/s",
            "cores": int(threads), "kind": "oracle",
            "sample": (f"{sc.n_pix} px x {sc.K} ch x {n} samples of the "
                       f"signal path ({t_sig:.1f} s) plus two full "
                       f"{sc.t_total}-sample 1/f series "
                       f"({t_pink_series:.2f} s each), combined per "
                       f"detector-sample")}


def run_to_disk(args, g, torch):
    """One out-of-core run: pixel groups streamed device -> pinned host ->
    .npy files; reports end-to-end detector-samples/s and bytes/s."""
    import shutil
    from workloads import configs
    T = int(round(args.disk_seconds * configs.F_SAMPLE))
    mk = {"c2": configs.c2, "c3": configs.c3, "c4": configs.c4}[args.workload]
    sc = mk(t_total=T)
    prec = g.PREC_SPLIT_BF16 if (args.precision or ("split" if args.workload
                                                    == "c4" else "fp32")) \
        == "split" else g.PREC_FP32
    ctx = g.sim_init(device=0, precision=prec,
                     workspace_bytes=int(args.workspace_gib * (1 << 30)))
    run = g.ScenarioRun(ctx, sc)
    dummy = g.Outputs(tod=torch.empty(1, device="cuda"), t0=0, length=T)
    sig, pk = run.signal_job(dummy), run.pink_job(dummy.tod)
    out_dir = os.path.join(args.to_disk, "gtod_sink_bench")
    per_pix = sc.K * T * 4 + T * 4
    dev = 2 * 7 * per_pix                      # two slabs of 7 pixels
    res = {}
    try:
        wall, nbytes, groups, G = g.simulate_to_disk(
            ctx, sig, pk, out_dir, device_bytes=dev, host_bytes=1 << 30)
        det = sc.n_pix * sc.K * T
        res = {"metric": "out-of-core detector-samples/s (device -> pinned "
                         "host -> .npy files)",
               "value": det / wall, "unit": "detector-samples/s",
               "bytes_per_s": nbytes / wall, "bytes": nbytes,
               "wall_s": wall, "groups": groups, "pixels_per_group": G,
               "config": {"workload": f"{args.workload} cut to {T} samples",
                          "dir": args.to_disk, "device_bytes": dev,
                          "host_bytes": 1 << 30}}
    finally:
        shutil.rmtree(out_dir, ignore_errors=True)
        g.free(ctx)
    print(json.dumps(res), flush=True)


FP64_PEAK = 78.6e12


def run_prep(args, g, torch, steps=3):
    """Input preparation at the sizes of the IFU workload: source-beam
    convolution (Eq. convolve_src) of a 121 x 121 x 3000 specific-intensity
    cube over +-150 arcsec, and footprint smoothing (5 m aperture, -10 dB
    taper) of the 1024 x 262144 PWV screen."""
    import numpy as np
    from workloads import configs, gen
    sc = configs.c3()
    nu = sc.spectral.nu_hz
    n, half = 121, 150 * ARCSEC
    d = 2 * half / (n - 1)
    I = torch.from_numpy(gen.intensity_cube(nu, n, half, seed=8)).cuda()
    scr = torch.from_numpy(sc.screen.pwv_mm).cuda()
    ctx = g.sim_init(device=0, workspace_bytes=int(args.workspace_gib * (1 << 30)))
    stream = torch.cuda.current_stream()
    el0 = configs.THETA0 - half
    calls = {
        "src_conv": lambda: g.convolve_source(ctx, I, nu, d, el0, d, 5.0, -10.0),
        "screen_conv": lambda: g.convolve_screen(ctx, scr, 0.2, 0.2, 5.0, -10.0),
    }
    res = {"metric": "input preparation (section 2.2)", "config": {
        "source": f"{n}x{n}x{nu.size} intensity cube, +-150 arcsec",
        "screen": "x".join(map(str, sc.screen.pwv_mm.shape)) + " FP64, 0.2 m cells",
        "aperture": "R_tel 5 m, edge taper -10 dB"}}
    for name, fn in calls.items():
        fn()
        torch.cuda.synchronize()
        g.profile_enable(ctx, True)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(stream)
        for _ in range(steps):
            out = fn()
        ev[1].record(stream)
        torch.cuda.synchronize()
        prof = g.profile_read(ctx)
        g.profile_enable(ctx, False)
        del out
        ms = ev[0].elapsed_time(ev[1]) / steps
        kern = {}
        for k, (kms, nl, units) in prof.items():
            if nl:
                kern[k] = {"launches": nl, "avg_ms": kms / nl, "total_ms": kms,
                           "work_per_s": units / (kms / 1e3)}
        main = kern[name]
        res[name] = {"ms_per_call": ms, "kernels": kern,
                     "roofline": {"kernel": name, "bound": "alu",
                                  "achieved": main["work_per_s"] / 1e12,
                                  "peak": FP64_PEAK / 1e12, "unit": "TFLOP/s",
                                  "frac": main["work_per_s"] / FP64_PEAK,
                                  "traffic": None}}
        print(f"# {name}: {ms:.2f} ms", file=sys.stderr, flush=True)
    g.free(ctx)
    print(json.dumps(res), flush=True)


def cpu_skydip(sc, n):
    """Seconds the oracle takes for the same skydip calibration."""
    from oracle import skydip as osd
    t = time.perf_counter()
    osd.skydip(sc, sc.scan.theta0, *SKYDIP_PWV, n)
    return time.perf_counter() - t


def run_reduce(args, g, torch, ctx, run, sc, out, stream, steps=3):
    """Time gtod_reduce on the Kelvin TOD of the last simulation step."""
    n, half = REDUCE_MAP
    ts = torch.empty_like(out.tod)
    mp = torch.zeros((sc.K, n, n), dtype=torch.float64, device="cuda")
    wt = torch.zeros_like(mp)
    d = run.reduce_desc(out.tod, REDUCE_R_OUT, t_star=ts, maps=(mp, wt),
                        map_n=n, map_half_rad=half, pwv=out.pwv)
    g.reduce(ctx, d, stream)
    torch.cuda.synchronize()
    g.profile_enable(ctx, True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(stream)
    for _ in range(steps):
        g.reduce(ctx, d, stream)
    ev[1].record(stream)
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / steps
    prof = g.profile_read(ctx)
    g.profile_enable(ctx, False)
    kern = {k: v for k, v in kernel_table(prof).items()
            if k in ("common", "grid")}
    dom = max(kern, key=lambda k: kern[k]["total_ms"])
    k = kern[dom]
    det = sc.n_pix * sc.K * sc.t_total
    finite = int(torch.isfinite(mp).sum().item())
    del ts
    return {"det_samples_per_s": det / (ms / 1e3), "ms_per_call": ms,
            "calls": steps, "map_nodes": n,
            "map_half_arcsec": half / ARCSEC,
            "r_out_arcsec": REDUCE_R_OUT / ARCSEC,
            "finite_map_cells": finite, "kernels": kern,
            "roofline": {"kernel": dom, "bound": "hbm",
                         "achieved": k["alg_gbs"], "peak": HBM_PEAK / 1e9,
                         "unit": "GB/s", "frac": k["alg_gbs"] * 1e9 / HBM_PEAK,
                         "traffic": None}}


def cpu_reduce(sc, seconds_hint=None):
    """The oracle's common-mode subtraction and gridding on one channel of
    every spaxel over 120000 samples of a synthetic Kelvin TOD."""
    import numpy as np
    from oracle import reduce as orr
    T = min(sc.t_total, 120000)
    rng = np.random.default_rng(0)
    tb = (20.0 + rng.normal(0, 0.01, (sc.n_pix, 1, T))).astype(np.float32)
    n, half = REDUCE_MAP
    t = time.perf_counter()
    ts = orr.common_mode(sc, tb, 1.0, REDUCE_R_OUT, channels=[sc.K // 2])
    orr.combine(*orr.spaxel_maps(sc, ts, half, n))
    dt = time.perf_counter() - t
    return {"value": sc.n_pix * T / dt, "unit": "detector-samples/s",
            "kind": "oracle", "cores": _cores(),
            "sample": f"1 channel x {sc.n_pix} spaxels x {T} samples"}


def copy_gbs(torch, n_bytes=1 << 30, reps=5):
    """Device-to-device copy bandwidth (bytes read + written per second),
    the practical ceiling for the elementwise kernels."""
    src = torch.ones(n_bytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(reps):
        dst.copy_(src)
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / reps
    del src, dst
    return 2.0 * n_bytes / (ms / 1e3) / 1e9


def d2h_gbs(torch, tod, n_bytes=1 << 30, reps=3):
    """Device-to-host copy of part of the TOD into pinned memory (GB/s);
    reported beside the result, never as it."""
    flat = tod.reshape(-1)[: n_bytes // 4]
    host = torch.empty(flat.numel(), dtype=torch.float32, pin_memory=True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    host.copy_(flat, non_blocking=True)
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(reps):
        host.copy_(flat, non_blocking=True)
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / reps
    return flat.numel() * 4 / (ms / 1e3) / 1e9


def elementwise(kern, workload, copy, sc):
    """HBM view of the elementwise kernels (panel, 1/f passes): algorithmic
    GB/s against the 8 TB/s peak and against the measured copy bandwidth,
    plus the measured fetch+write bytes where a profile holds them.

    The panel's algorithmic bytes are what any panel kernel must move: the
    dP row it writes (4 F bytes) and the screen cells (32 bytes) per row,
    plus one read of the source cube per launch.  The library's per-row
    count (20 F + 32: four corner spectra per row) describes a kernel that
    reads every row's corners from memory; in cube-cell order the corners
    come mostly from the caches, so that count is not a traffic bound."""
    out = {}
    for name in ("panel", "pink_pass1", "pink_pass2"):
        if name not in kern:
            continue
        gbs = kern[name]["alg_gbs"]
        if name == "pink_pass2":
            # the library counts 16 bytes per complex point (a scratch read
            # and two TOD samples); the TOD keeps only t_total of the
            # transform's N samples, so the store is 8 t_total / N bytes
            n_fft = 1 << max(1, (sc.t_total - 1).bit_length())
            gbs *= (8.0 + 8.0 * min(1.0, sc.t_total / n_fft)) / 16.0
        if name == "panel":
            k = kern[name]
            rows = k["alg_gbs"] * 1e9 * k["avg_ms"] / 1e3 / (20.0 * sc.F + 32.0)
            cube = 0.0 if sc.source is None else sc.source.cube.size * 4.0
            gbs = (rows * (4.0 * sc.F + 32.0) + cube) / (k["avg_ms"] / 1e3) / 1e9
        d = {"alg_gbs": gbs, "frac_hbm_peak": gbs * 1e9 / HBM_PEAK,
             "frac_copy": gbs / copy}
        tf = os.path.join(ROOT, "profiles", f"traffic_{name}_{workload}.json")
        if os.path.exists(tf):
            b = json.load(open(tf))["bytes_per_launch"]
            meas = b / (kern[name]["avg_ms"] / 1e3) / 1e9
            d.update({"measured_gbs": meas,
                      "measured_frac_hbm_peak": meas * 1e9 / HBM_PEAK})
        out[name] = d
    return out


def end_to_end(value, sc, prec_name):
    """Detector-samples/s against the whole-path bound: the contraction at
    its matrix-core peak (6 F FLOP per detector-sample; the split path runs
    7 BF16 products for every 3) and the algorithmic HBM bytes per
    detector-sample ((16 F + 4 K) / K: four source spectra per row and the
    output)."""
    F, K = sc.F, sc.K
    flop = 6.0 * F * (7.0 / 3.0 if prec_name == "split" else 1.0)
    compute = PEAK[prec_name] / flop
    hbm = HBM_PEAK / ((16.0 * F + 4.0 * K) / K)
    bound = min(compute, hbm)
    return {"compute_bound": compute, "hbm_bound": hbm, "frac": value / bound}


def kernel_table(prof):
    """Per-kernel figures from the library's event timing, with the
    algorithmic work the library reports per kernel (FLOP for the
    contractions, bytes for the panel and the reduction kernels, complex
    points for the 1/f passes: an 8-byte scratch write in pass 1; a
    scratch read plus two TOD samples, 16 bytes, in pass 2, which
    `elementwise` scales to the TOD samples a series keeps)."""
    kern = {}
    for name, (ms, n, units) in prof.items():
        if n == 0:
            continue
        d = {"launches": n, "avg_ms": ms / n, "total_ms": ms}
        sec = ms / 1e3
        if name.startswith("gemm"):
            d["alg_tflops"] = units / sec / 1e12
        elif name in ("panel", "common", "grid"):
            d["alg_gbs"] = units / sec / 1e9
        else:
            d["alg_gbs"] = (8.0 if name == "pink_pass1" else 16.0) * units / sec / 1e9
        kern[name] = d
    return kern


def roofline(kern, workload):
    dom = max(kern, key=lambda k: kern[k]["total_ms"])
    dd = kern[dom]
    if dom.startswith("gemm"):
        peak = PEAK["split" if dom.endswith("bf16") else "fp32"] / 1e12
        roof = {"bound": "mfma", "achieved": dd["alg_tflops"], "peak": peak,
                "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": dd["alg_gbs"],
                "peak": HBM_PEAK / 1e9, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["kernel"] = dom
    roof["traffic"] = None
    tf = os.path.join(ROOT, "profiles", f"traffic_{dom}_{workload}.json")
    if os.path.exists(tf):
        roof["traffic"] = json.load(open(tf)).get("bytes_per_launch")
    return roof


def run_c5(args, g, torch):
    """Serving workload: returns (result dict, representative scenario)."""
    from paper_2604_23305_amd.serve import Engine, Request
    from workloads import configs
    prec = g.PREC_SPLIT_BF16 if (args.precision or "split") == "split" \
        else g.PREC_FP32
    reqs = configs.c5_requests()
    screens = configs.c5_screens()
    ctx = g.sim_init(device=0, precision=prec, workspace_bytes=4 << 30)
    scr_ids = [g.load_screen(ctx, s.pwv_mm, s.dx_m, s.dy_m, s.ix0, s.iy0,
                             s.h_column_m, s.wind_mps) for s in screens]
    sp_cache, src_cache, spec_ids, cubes = {}, {}, {}, {}
    requests, scen = [], {}
    for r in reqs:
        sc = configs.c5_scenario(r, screens, sp_cache, src_cache)
        key = (r["K"], r["F"])
        run = g.ScenarioRun(ctx, sc, screen_id=scr_ids[r["screen"]],
                            spec_id=spec_ids.get(key), cube=cubes.get(r["F"]))
        spec_ids[key] = run.spec_id
        cubes[r["F"]] = run.cube
        requests.append(Request.from_run(run, r["rid"], r["arrival_s"]))
        scen[r["rid"]] = sc
    torch.cuda.synchronize()
    print(f"# c5 setup: {len(requests)} requests, {len(spec_ids)} spectral "
          "setups resident", file=sys.stderr, flush=True)
    # warm-up: the four smallest requests, all arrived at once
    warm = sorted(requests, key=lambda q: q.det_samples)[:4]
    # the timed engine reuses the warm-up engine's streams, whose workspaces
    # are then already allocated
    streams = [torch.cuda.Stream() for _ in range(4)]
    Engine(ctx, streams=streams, hbm_budget_bytes=150 << 30).run(
        [Request(**{k: getattr(q, k) for k in (
            "rid", "arrival_s", "spec_id", "screen_id", "K", "n_pix", "dphi",
            "dtheta", "t_total", "seed", "scan_kind", "scan_params", "phi0",
            "theta0", "cube", "cube_grid", "pink_alpha", "pink_knee_hz",
            "photon_noise", "precision")}) for q in warm], realtime=False)
    g.profile_enable(ctx, True)
    eng = Engine(ctx, streams=streams, hbm_budget_bytes=150 << 30)
    stats = eng.run(requests, realtime=True)
    prof = g.profile_read(ctx)
    g.profile_enable(ctx, False)
    summ = stats.summary()
    mid = sorted(reqs, key=lambda q: q["n_pix"] * q["K"] * q["t_total"])
    rep = scen[mid[len(mid) // 2]["rid"]]
    g.free(ctx)
    return summ, prof, rep, ("split" if prec == g.PREC_SPLIT_BF16 else "fp32")


def measure(g, torch, ctx, jobs, stream, steps, warmup, label):
    """Warm-up calls, then `steps` timed calls of the whole simulation, each
    one gtod_simulate_tod call on `stream`; per-kernel times come from the
    library's events on that stream."""
    for w in range(warmup):
        g.simulate_tod(ctx, jobs, stream)
        torch.cuda.synchronize()
        print(f"# {label}: warmup {w} done", file=sys.stderr, flush=True)
    g.profile_enable(ctx, True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for s in range(steps):
        g.simulate_tod(ctx, jobs, stream)
        ev[s + 1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = g.profile_read(ctx)
    g.profile_enable(ctx, False)
    step_ms = [ev[s].elapsed_time(ev[s + 1]) for s in range(steps)]
    print(f"# {label}: timed {steps} steps in {elapsed:.3f} s",
          file=sys.stderr, flush=True)
    return elapsed, step_ms, kernel_table(prof)


def latency(step_ms):
    import numpy as np
    return {"p50": float(np.percentile(step_ms, 50)),
            "p99": float(np.percentile(step_ms, 99)),
            "min": float(np.min(step_ms)), "max": float(np.max(step_ms))}


def c4_measure(args, g, torch, ctx, run3, sc3, stream):
    """The split-precision IFU workload on the context, screen and spectral
    setup of the c3 run (c4 differs only by its faint extended source and
    noise seed): the same whole-simulation steps, hi+lo BF16 contraction."""
    from workloads import configs
    sc = configs.c4(reuse_screen=sc3.screen)
    run = g.ScenarioRun(ctx, sc, screen_id=run3.screen_id,
                        spec_id=run3.spec_id)
    out = run.alloc()
    jobs = [run.pink_job(out.tod, accumulate=False),
            run.signal_job(out, precision=g.PREC_SPLIT_BF16, accumulate=True)]
    elapsed, step_ms, kern = measure(g, torch, ctx, jobs, stream, args.steps,
                                     args.warmup, "c4")
    del out, run
    value = sc.n_pix * sc.K * sc.t_total * args.steps / elapsed
    res = {"value": value, "unit": "detector-samples/s",
           "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": elapsed * 1e3 / args.steps, "dtype": "bf16x2",
           "config": {"workload": f"c4: {WORKLOADS['c4']}",
                      "pixels": sc.n_pix, "channels": sc.K,
                      "freq_bins": sc.F, "samples": sc.t_total,
                      "precision": "split"},
           "latency_ms": latency(step_ms),
           "roofline": roofline(kern, "c4"),
           "end_to_end": end_to_end(value, sc, "split"),
           "kernels": kern}
    return res, sc


def c5_measure(args, g, torch):
    """The serving stream, summarised for the c3 line."""
    summ, prof, rep, prec_name = run_c5(args, g, torch)
    kern = kernel_table(prof)
    return {"value": summ["det_samples_per_s"], "unit": "detector-samples/s",
            "makespan_ms": summ["makespan_s"] * 1e3,
            "requests": summ["requests"], "det_samples": summ["det_samples"],
            "dtype": "f32" if prec_name == "fp32" else "bf16x2",
            "config": {"workload": f"c5: {WORKLOADS['c5']}",
                       "precision": prec_name},
            "latency_ms": {"p50": summ["p50_ms"], "p99": summ["p99_ms"],
                           "mean": summ["mean_ms"],
                           "what": "scheduled arrival to the completion "
                                   "event of the request's last job, "
                                   "outputs in HBM"},
            "roofline": roofline(kern, "c5"), "kernels": kern}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not "
              "supported (rows and 1/f series are independent, so the "
              "simulation shards by pixel or by request with no exchange "
              "between GPUs)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2604_23305_amd as g

    if args.workload == "c5":
        summ, prof, rep, prec_name = run_c5(args, g, torch)
        kern = kernel_table(prof)
        res = {"metric": METRIC, "value": summ["det_samples_per_s"],
               "unit": "detector-samples/s", "n_gpus": 1, "steps": 1,
               "warmup": 1, "ms_per_step": summ["makespan_s"] * 1e3,
               "higher_is_better": True, "scaling": "weak",
               "vs_baseline": None,
               "dtype": "f32" if prec_name == "fp32" else "bf16x2",
               "data": "synthetic",
               "config": {"workload": f"c5: {WORKLOADS['c5']}",
                          "requests": summ["requests"],
                          "det_samples": summ["det_samples"],
                          "precision": prec_name,
                          "parallelism": "single GPU, 4 streams"},
               "latency_ms": {"p50": summ["p50_ms"], "p99": summ["p99_ms"],
                              "mean": summ["mean_ms"]},
               "roofline": roofline(kern, "c5"), "kernels": kern}
        torch.cuda.empty_cache()
        if not args.no_cpu_baseline:
            res["cpu_baseline"] = cpu_baseline(rep, args.cpu_seconds)
            res["cpu_baseline"]["sample"] = (
                f"request {rep.name} ({rep.n_pix} px, {rep.K} ch, "
                f"{rep.F} bins): " + res["cpu_baseline"]["sample"])
        print(json.dumps(res), flush=True)
        return
    if args.to_disk:
        run_to_disk(args, g, torch)
        return
    if args.prep:
        run_prep(args, g, torch)
        return
    if args.calib_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    copy = copy_gbs(torch)
    prec_name = args.precision or ("split" if args.workload == "c4" else "fp32")
    prec = g.PREC_SPLIT_BF16 if prec_name == "split" else g.PREC_FP32
    t_setup = time.perf_counter()
    sc = scenario(args.workload)
    ctx = g.sim_init(device=0, precision=prec,
                     workspace_bytes=int(args.workspace_gib * (1 << 30)))
    run = g.ScenarioRun(ctx, sc)
    if args.reduce and not args.kelvin:
        print("--reduce needs --kelvin N", file=sys.stderr)
        sys.exit(2)
    out = run.alloc(with_pwv=args.reduce)
    kel = None
    if args.kelvin:
        times = []
        for _ in range(3):
            t = time.perf_counter()
            g.skydip(ctx, run.spec_id, sc.K, sc.scan.theta0, *SKYDIP_PWV,
                     args.kelvin)
            times.append(time.perf_counter() - t)
        kel = {"sweep_points": args.kelvin, "pwv_mm": list(SKYDIP_PWV),
               "elevation_deg": float(np.degrees(sc.scan.theta0)),
               "skydip_ms": min(times) * 1e3}
    kflag = bool(args.kelvin)
    # the 1/f job writes the TOD and the signal job's contraction epilogue
    # adds into it (the order the serving engine uses): the one extra TOD
    # read then sits in the matrix-core-bound kernel, not in the
    # memory-bound 1/f pass
    jobs = [run.pink_job(out.tod, accumulate=False, kelvin=kflag),
            run.signal_job(out, kelvin=kflag, accumulate=True)]
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_setup
    print(f"# setup {setup_s:.1f} s; workload {args.workload} ({prec_name})",
          file=sys.stderr, flush=True)

    elapsed, step_ms, kern = measure(g, torch, ctx, jobs, stream, args.steps,
                                     args.warmup, args.workload)
    det_per_step = sc.n_pix * sc.K * sc.t_total
    value = det_per_step * args.steps / elapsed
    roof = roofline(kern, args.workload)
    red = run_reduce(args, g, torch, ctx, run, sc, out, stream) \
        if args.reduce else None

    res = {
        "metric": METRIC,
        "value": value,
        "unit": "detector-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec_name == "fp32" else "bf16x2",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}",
                   "pixels": sc.n_pix, "channels": sc.K, "freq_bins": sc.F,
                   "samples": sc.t_total, "precision": prec_name,
                   "tod_unit": "K" if kel else "W",
                   "parallelism": "single GPU"},
        "latency_ms": latency(step_ms),
        "roofline": roof,
        "elementwise": elementwise(kern, args.workload, copy, sc),
        "end_to_end": end_to_end(value, sc, prec_name),
        "copy_gbs": copy,
        "d2h_gbs": d2h_gbs(torch, out.tod),
        "kernels": kern,
    }
    extras = (args.workload == "c3" and not args.headline_only
              and not kel and not red)
    sc4 = None
    if extras:
        del out
        res["c4"], sc4 = c4_measure(args, g, torch, ctx, run, sc, stream)
        res["c4"]["vs_c3_fp32"] = res["c4"]["value"] / value
    g.free(ctx)
    if not extras:
        del out
    torch.cuda.empty_cache()
    if extras:
        res["c5"] = c5_measure(args, g, torch)
        torch.cuda.empty_cache()
    if kel:
        res["kelvin"] = kel
    if red:
        res["reduce"] = red
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(sc, args.cpu_seconds)
        if sc4 is not None:
            res["c4"]["cpu_baseline"] = cpu_baseline(sc4, args.cpu_seconds / 2)
        if kel:
            kel["skydip_oracle_ms"] = cpu_skydip(sc, args.kelvin) * 1e3
        if red:
            red["cpu_baseline"] = cpu_reduce(sc)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
