#!/usr/bin/env python3
"""Throughput of the time-domain Gaussian log-likelihood on one MI355X.

Workload (two detectors x N = 16384 samples at 4096 Hz, 4 s; 4096 chirp templates
per launch; analytic-PSD ACF with nugget 1e-6; seeded synthetic data standing in
for LIGO strain): every step scores all templates against both detectors and
returns the network logL per template.  One step runs the per-evaluation hot
path with the factors resident in HBM: template gather and BF16 hi/lo split,
the two BF16x3 whitening products, the FP64 FFT refinement and the FP64
reductions (mixed precision), or the blocked FP64 triangular solve with fused
reductions (FP64).  The one-time costs (covariance assembly, FP64 Cholesky,
whitening operator and its split, whitened data) are timed separately.

Prints one JSON line.  `value` is the mixed-precision evals/s (one eval = one
template against all detectors); the FP64 path on the same GPU is reported
beside it, with |dlogL| of mixed vs FP64 over every template and of both vs the
FP64 CPU oracle on a sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "logL evals/s @N=16384, mixed vs FP64 at |ΔlogL|≤1e-3; p50/p99 latency"
PEAK_BF16 = 2.5e15       # dense BF16 matrix-core peak, FLOP/s
PEAK_FP64 = 78.6e12      # FP64 matrix-core peak, FLOP/s
PEAK_HBM = 8.0e12        # HBM3E bandwidth, bytes/s


# HBM traffic of a kernel comes from rocprofv3 counter runs (FETCH_SIZE and WRITE_SIZE,
# scaled by a copy kernel of known size); the committed summary records the bytes per
# launch together with a hash of the kernel sources, and is used only while they match.
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "traffic_c2.md")
KERNEL_SOURCES = ["paper_2603_06010_amd/csrc/kernels_mixed.hip",
                  "paper_2603_06010_amd/csrc/kernels_f64.hip",
                  "paper_2603_06010_amd/csrc/tda_api.hip",
                  "paper_2603_06010_amd/csrc/tda_internal.h"]


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


PROFILE_UTIL = os.path.join(ROOT, "profiles", "utilisation_c2.md")


def profiled_clock(name):
    """(sustained shader clock in GHz, matrix-core busy fraction at that clock) of timing
    record `name` from the committed counter summary, or None (other kernel sources)."""
    try:
        with open(PROFILE_UTIL) as fh:
            lines = fh.read().splitlines()
    except OSError:
        return None
    sha = kernel_sources_sha256()
    for line in lines:
        parts = line.strip().split()
        if len(parts) >= 5 and parts[0] == "clock" and parts[1] == name:
            kv = dict(p.split("=", 1) for p in parts[2:] if "=" in p)
            if kv.get("sources_sha256") != sha:
                return None
            return float(kv["ghz"]), float(kv["mfma_util"])
    return None


def profiled_traffic(name):
    """Bytes per launch (fetched + written) of timing record `name`, or None."""
    try:
        with open(PROFILE_TRAFFIC) as fh:
            lines = fh.read().splitlines()
    except OSError:
        return None
    sha = kernel_sources_sha256()
    for line in lines:
        parts = line.strip().strip("`").split()
        if len(parts) >= 5 and parts[0] == "traffic" and parts[1] == name:
            kv = dict(p.split("=", 1) for p in parts[2:] if "=" in p)
            if kv.get("sources_sha256") != sha:
                return None
            return int(kv["fetch_bytes"]) + int(kv["write_bytes"])
    return None


def _pct(x, p):
    return float(np.percentile(np.asarray(x), p))


def host_cpu():
    """Physical cores (lscpu core/socket pairs), logical CPUs, the CPUs this process may
    use, and the BLAS library numpy/scipy call (threadpoolctl)."""
    import subprocess
    info = {"logical_cpus": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0))}
    try:
        out = subprocess.run(["lscpu", "-p=CORE,SOCKET"], capture_output=True, text=True,
                             timeout=10).stdout
        pairs = {tuple(l.split(",")) for l in out.splitlines() if l and not l.startswith("#")}
        info["physical_cores"] = len(pairs) or None
    except Exception:
        info["physical_cores"] = None
    try:
        from threadpoolctl import threadpool_info
        blas = [i for i in threadpool_info() if i.get("user_api") == "blas"]
        info["blas"] = [{"library": i.get("internal_api"), "version": i.get("version"),
                         "threads": i.get("num_threads"), "arch": i.get("architecture")}
                        for i in blas]
    except Exception:
        info["blas"] = None
    return info


_POOL = {}


def _pool_init(paths, d_np):
    """Worker set-up: the oracle's factors, memory-mapped from files the parent wrote."""
    import oracle
    fs = []
    for p in paths:
        meta = json.load(open(p + ".json"))
        Ls = [np.load(f"{p}.L{k}.npy", mmap_mode="r") for k in range(meta["n_seg"])]
        idx = [np.load(f"{p}.idx{k}.npy") for k in range(meta["n_seg"])]
        fs.append(oracle.Factor(meta["N"], [tuple(x) for x in meta["segments"]], idx, Ls,
                                meta["logdet"], meta["n_eff"]))
    _POOL["fs"], _POOL["d"] = fs, d_np


def _pool_eval(h_row):
    """One template per call, every detector (the paper's recommended CPU set-up)."""
    import oracle
    return float(oracle.loglik_network(_POOL["fs"], _POOL["d"], h_row[None, :])[0])


def cpu_pool_baseline(inst, fs, sample, n_proc):
    """The oracle in a process pool of n_proc single-threaded workers, one template per call
    (Sec. III.B, Sec. V: a pool of size equal to the cores, one BLAS thread each).  The
    factors go to the workers through memory-mapped files (one copy in the page cache)."""
    import multiprocessing as mp
    import shutil
    import tempfile
    need = sum(L.nbytes for f in fs for L in f.L)
    base = "/dev/shm" if shutil.disk_usage("/dev/shm").free > 2 * need else None
    tmp = tempfile.mkdtemp(prefix="tda_pool_", dir=base)
    try:
        paths = []
        for k, f in enumerate(fs):
            p = os.path.join(tmp, f"det{k}")
            for j, (L, idx) in enumerate(zip(f.L, f.idx)):
                np.save(f"{p}.L{j}.npy", L)
                np.save(f"{p}.idx{j}.npy", idx)
            json.dump({"N": f.N, "segments": [list(x) for x in f.segments], "n_seg": len(f.L),
                       "logdet": f.logdet, "n_eff": f.n_eff}, open(p + ".json", "w"))
            paths.append(p)
        env_keys = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
        saved = {k: os.environ.get(k) for k in env_keys}
        for k in env_keys:
            os.environ[k] = "1"
        try:
            ctx = mp.get_context("spawn")
            with ctx.Pool(n_proc, initializer=_pool_init, initargs=(paths, inst.d)) as pool:
                pool.map(_pool_eval, [inst.H[0]] * n_proc)  # warm-up: workers page L in
                t = time.perf_counter()
                ref = pool.map(_pool_eval, list(inst.H[:sample]), chunksize=1)
                wall = time.perf_counter() - t
        finally:
            for k, v in saved.items():
                if v is None:
                    os.environ.pop(k, None)
                else:
                    os.environ[k] = v
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return np.array(ref), {
        "value": sample / wall, "unit": "evals/s", "cores": n_proc, "kind": "oracle",
        "sample": f"{sample} of the {inst.B} templates x {inst.n_det} detectors, one template per "
                  f"call in a pool of {n_proc} processes with one BLAS thread each",
    }


def cpu_baseline(inst, sample, fs_cache):
    """Time the FP64 oracle (as it is) on `sample` templates against both detectors."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 0) for i in threadpool_info()] or [0])
    except Exception:
        threads = 0
    cores = threads or len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    fs = [oracle.factor(inst.acf, inst.N, inst.masks[k]) for k in range(inst.n_det)]
    t_factor = time.perf_counter() - t0
    fs_cache.extend(fs)
    Hs = inst.H[:sample]
    oracle.loglik_network(fs, inst.d, Hs[:2])  # warm-up
    reps, t = 0, 0.0
    while reps < 3 or (t < 10.0 and reps < 10):
        t1 = time.perf_counter()
        ref = oracle.loglik_network(fs, inst.d, Hs)
        t += time.perf_counter() - t1
        reps += 1
    return ref, {
        "value": sample * reps / t,
        "unit": "evals/s",
        "cores": int(cores),
        "kind": "oracle",
        "sample": f"{sample} of the {inst.B} templates x {inst.n_det} detectors, N={inst.N}, "
                  f"{reps} repetitions after 1 warm-up of one batched triangular solve per "
                  f"detector (BLAS threads = {threads or 'unknown'}); factorisation "
                  f"({t_factor:.1f} s, once per detector) excluded like on the GPU",
        "factor_s": t_factor,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--templates", type=int, default=4096)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--fp64-steps", type=int, default=None)
    ap.add_argument("--cpu-sample", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c5", action="store_true", help="c2: leave out the short served leg")
    ap.add_argument("--core-only", action="store_true",
                    help="c2: only the batched mixed and FP64 evaluations (for profiling runs); "
                         "every other leg is null (same as --legs none)")
    ap.add_argument("--legs", default="gs,acf,cdo,terms,wres,stress,c3,c4,c5",
                    help="c2: the legs run beside the mixed and FP64 evaluations, comma-"
                         "separated from gs, acf, cdo, terms, wres, stress, c3, c4, c5 (or none)")
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c4", "c5"],
                    help="c2 (default): two detectors x N=16384, 4096 templates per launch; "
                         "c3: one detector x N=32768 with 3 gaps, 8192 templates; "
                         "c4: 64 ragged instances in one batched evaluation; "
                         "c5: request server over 32 resident datasets")
    ap.add_argument("--duration", type=float, default=4.0, help="c5: seconds of request trace")
    ap.add_argument("--rate", type=float, default=20000.0, help="c5: mean requests per second")
    ap.add_argument("--rates", default="0.01,0.025,0.05,0.1,1.0",
                    help="c5: offered loads of the sweep, as fractions of --rate")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after timing, run one device copy of this many MiB (reference "
                         "kernel for hardware byte counters)")
    args = ap.parse_args()
    legs = set() if args.core_only else {x.strip() for x in args.legs.split(",")} - {"none", ""}
    if args.no_c5:
        legs.discard("c5")
    args.leg = lambda name: name in legs
    if args.gpus != 1:
        print("bench.py: measures one GPU only; run with --gpus 1 (templates and datasets "
              "shard across GPUs with no exchange in the hot loop)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2603_06010_amd as tda
    import synth

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(2)
    tda.load_library()
    dev = torch.device("cuda", 0)
    log = lambda *a: print("[bench]", *a, file=sys.stderr, flush=True)  # noqa: E731
    if args.workload == "c3":
        return bench_c3(args, tda, torch, synth, dev, log)
    if args.workload == "c4":
        return bench_c4(args, tda, torch, synth, dev, log)
    if args.workload == "c5":
        return bench_c5(args, tda, torch, synth, dev, log)

    t0 = time.perf_counter()
    w = synth.c2_workload(B=args.templates, n=args.n)
    inst = w.instances[0]
    log(f"inputs ready in {time.perf_counter() - t0:.1f} s: N={inst.N} B={inst.B} det={inst.n_det}")
    d = [torch.from_numpy(inst.d[k]).to(dev) for k in range(inst.n_det)]
    H = torch.from_numpy(inst.H).to(dev)

    setup = {}
    tda.timing_read(reset=True)
    tda.timing_enable(True)
    t0 = time.perf_counter()
    hs = [tda.Handle(inst.acf, inst.N, inst.masks[k], precision="mixed") for k in range(inst.n_det)]
    torch.cuda.synchronize()
    setup["cov_build_s"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    for h in hs:
        h.factor()
    torch.cuda.synchronize()
    setup["factor_and_operator_s"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    for h, dk in zip(hs, d):
        h.set_data(dk)
    torch.cuda.synchronize()
    setup["whitened_data_s"] = time.perf_counter() - t0
    tda.timing_enable(False)
    kt_setup = tda.timing_read(reset=True)
    n_eff = [h.info()["n_eff"] for h in hs]
    n_pad = [h.info()["n_pad"] for h in hs]
    setup["one_time"] = one_time_costs(kt_setup, n_eff, n_pad)
    log("setup", setup)

    out = {p: torch.empty(inst.B, dtype=torch.float64, device=dev) for p in ("mixed", "fp64")}
    items = {p: [(h, dk, H, out[p]) for h, dk in zip(hs, d)] for p in out}

    def run(prec, steps, warmup):
        for _ in range(warmup):
            tda.loglik_multi(items[prec], precision=prec)
        torch.cuda.synchronize()
        tda.timing_read(reset=True)
        tda.timing_enable(True)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(steps)]
        torch.cuda.synchronize()
        t = time.perf_counter()
        for a, b in evs:
            a.record()
            tda.loglik_multi(items[prec], precision=prec)
            b.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        tda.timing_enable(False)
        kt = tda.timing_read(reset=True)
        lat = [a.elapsed_time(b) for a, b in evs]
        return wall, lat, kt

    wall_m, lat_m, kt_m = run("mixed", args.steps, args.warmup)
    log(f"mixed: {wall_m / args.steps * 1e3:.3f} ms/step", kt_m)
    fsteps = args.fp64_steps or max(3, args.steps // 4)
    wall_f, lat_f, kt_f = run("fp64", fsteps, 1)
    log(f"fp64: {wall_f / fsteps * 1e3:.3f} ms/step", kt_f)
    res_m = out["mixed"].cpu().numpy()
    res_f = out["fp64"].cpu().numpy()
    d_mf = np.abs(res_m - res_f)

    # Gohberg-Semencul FP64 path on the same inputs (segments without excluded samples)
    gs = None
    if args.leg("gs") and not any(m is not None and np.any(m) for m in inst.masks):
        t0 = time.perf_counter()
        hg = [tda.Handle(inst.acf, inst.N, inst.masks[k], precision="gs").factor()
              for k in range(inst.n_det)]
        torch.cuda.synchronize()
        gs_setup = time.perf_counter() - t0
        out["gs"] = torch.empty(inst.B, dtype=torch.float64, device=dev)
        items["gs"] = [(h, dk, H, out["gs"]) for h, dk in zip(hg, d)]
        wall_g, lat_g, kt_g = run("gs", args.steps, args.warmup)
        log(f"gs: {wall_g / args.steps * 1e3:.3f} ms/step", kt_g)
        res_g = out["gs"].cpu().numpy()
        gs = {"value": inst.B * args.steps / wall_g, "unit": "evals/s",
              "ms_per_step": wall_g / args.steps * 1e3,
              "latency_ms": {"p50": _pct(lat_g, 50), "p99": _pct(lat_g, 99)},
              "max_abs_dlogL_vs_fp64_gpu": float(np.abs(res_g - res_f).max()),
              "kernels_ms": {k: v[1] / v[0] for k, v in kt_g.items()},
              "setup_s": gs_setup}
        for h in hg:
            h.close()

    acf_line = cdo = snr_terms = wres = stress = c3_line = c4_line = c5_line = None
    if args.leg("acf"):
        # autocovariance estimation from a 256 s stretch of noise at 4096 Hz (2^20 samples):
        # Welch with 8 s segments and the direct estimator, both to the 16384 lags of the
        # N = 16384 covariance
        xs = torch.from_numpy(synth.stationary_noise(np.random.default_rng(7), 1 << 20, 1)[0]).to(dev)
        acf_line = {}
        for meth, seg in (("welch", 32768), ("direct", None)):
            tda.acf_estimate(xs, 16384, method=meth, seg_len=seg)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(3):
                est = tda.acf_estimate(xs, 16384, method=meth, seg_len=seg)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t) / 3 * 1e3
            n_x = xs.shape[0]
            macs = ((n_x - seg) // (seg // 2) + 1) * seg * 16384 if seg else n_x * 16384
            true = synth.make_acf(8)
            acf_line[meth] = {"ms": ms, "gmac_per_s": macs / ms * 1e-6,
                              "max_abs_err_first_8_lags_vs_true": float(np.abs(est[:8].cpu().numpy() - true).max())}
        acf_line["input"] = "2^20 samples of noise with the benchmark covariance; 16384 lags; Welch 32768-sample segments"
        log("acf", acf_line)
        del xs

    if args.leg("cdo"):
        # explicit-inverse FP64 evaluation (the paper's CDO form) on the same mixed handles:
        # one call per detector, network sum on the host side of the comparison
        csteps = max(3, args.steps // 4)
        cdo_out = [h.loglik(dk, H, precision="cdo") for h, dk in zip(hs, d)]
        torch.cuda.synchronize()
        tda.timing_read(reset=True)
        tda.timing_enable(True)
        t = time.perf_counter()
        for _ in range(csteps):
            cdo_out = [h.loglik(dk, H, precision="cdo") for h, dk in zip(hs, d)]
        torch.cuda.synchronize()
        wall_c = time.perf_counter() - t
        tda.timing_enable(False)
        kt_c = tda.timing_read(reset=True)
        res_c = sum(o.cpu().numpy() for o in cdo_out)
        cc, tc = kt_c["cdo_f64"]
        ach_c = float(sum(n * n for n in n_eff)) / len(n_eff) * inst.B / (tc / cc * 1e-3)
        cdo = {"value": inst.B * csteps / wall_c, "unit": "evals/s", "ms_per_step": wall_c / csteps * 1e3,
               "steps": csteps, "max_abs_dlogL_vs_fp64_gpu": float(np.abs(res_c - res_f).max()),
               "kernels_ms": {k: v[1] / v[0] for k, v in kt_c.items()},
               "roofline": {"bound": "mfma", "kernel": "cdo_f64", "achieved": ach_c / 1e12,
                            "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s", "frac": ach_c / PEAK_FP64,
                            "avg_ms": tc / cc}}
        log("cdo", cdo)
        del cdo_out

    if args.leg("terms"):
        # inner products behind the SNRs (tda_loglik_terms): mixed per detector, timed, and
        # compared with the FP64 evaluation of the same terms on the GPU
        tsteps = max(3, args.steps // 4)
        terms_m = [h.loglik_terms(dk, H, precision="mixed") for h, dk in zip(hs, d)]
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(tsteps):
            terms_m = [h.loglik_terms(dk, H, precision="mixed") for h, dk in zip(hs, d)]
        torch.cuda.synchronize()
        wall_t = time.perf_counter() - t
        terms_f = [h.loglik_terms(dk, H, precision="fp64") for h, dk in zip(hs, d)]
        torch.cuda.synchronize()
        dh_m = sum(x[1] for x in terms_m).cpu().numpy()
        hh_m = sum(x[2] for x in terms_m).cpu().numpy()
        dh_f = sum(x[1] for x in terms_f).cpu().numpy()
        hh_f = sum(x[2] for x in terms_f).cpu().numpy()
        rho_m, rho_f = dh_m / np.sqrt(hh_m), dh_f / np.sqrt(hh_f)
        snr_terms = {"value": inst.B * tsteps / wall_t, "unit": "evals/s (logL + <d,h> + <h,h>, "
                     "network sums)", "ms_per_step": wall_t / tsteps * 1e3, "steps": tsteps,
                     "max_abs_d_dh_mixed_vs_fp64_gpu": float(np.abs(dh_m - dh_f).max()),
                     "max_abs_d_hh_mixed_vs_fp64_gpu": float(np.abs(hh_m - hh_f).max()),
                     "max_abs_d_rho_mf_mixed_vs_fp64_gpu": float(np.abs(rho_m - rho_f).max()),
                     "rho_mf_range": [float(rho_f.min()), float(rho_f.max())]}
        log("snr terms", snr_terms)
        del terms_m, terms_f

    if args.leg("wres"):
        # whitened residuals (tda_whitened_residual) of one detector: the FP64 solve plus the
        # export of L^-1 (d - h) for every template; the export kernel against the HBM peak
        wsteps = 3
        out_w, W = hs[0].whitened_residual(d[0], H)
        torch.cuda.synchronize()
        tda.timing_read(reset=True)
        tda.timing_enable(True)
        t = time.perf_counter()
        for _ in range(wsteps):
            out_w, W = hs[0].whitened_residual(d[0], H)
        torch.cuda.synchronize()
        wall_w = time.perf_counter() - t
        tda.timing_enable(False)
        kt_w = tda.timing_read(reset=True)
        ref_w = hs[0].loglik(d[0], H, precision="fp64")
        exp_ms = kt_w["whiten_export"][1] / kt_w["whiten_export"][0]
        exp_bytes = 16.0 * W.shape[0] * W.shape[1]  # 8 B read and 8 B written per entry
        wres = {"ms_per_call": wall_w / wsteps * 1e3, "templates": int(W.shape[0]),
                "n_eff": int(W.shape[1]), "export_ms": exp_ms,
                "export_GB_per_s": exp_bytes / exp_ms / 1e6,
                "export_frac_of_hbm_peak": exp_bytes / exp_ms / 1e-3 / PEAK_HBM,
                "logL_identical_to_fp64": bool(torch.equal(out_w, ref_w))}
        log("whitened residuals", wres)
        del W, out_w, ref_w

    # the same workload at smaller nuggets down to the stress nugget (kappa(C) up to 2.9e8),
    # and the gapped one-detector N = 32768 workload (where Gohberg-Semencul cannot apply)
    if args.leg("stress"):
        stress = stress_leg(args, tda, torch, synth, dev, log)
    if args.leg("c3"):
        c3_line = run_c3(args, tda, torch, synth, dev, log, steps=5, fsteps=2)
    def guarded(name, fn):
        # a leg that fails (say, out of device memory) is reported in the line, not fatal
        try:
            return fn()
        except Exception as e:  # noqa: BLE001
            log(f"{name} failed: {type(e).__name__}: {e}")
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
            return {"error": f"{type(e).__name__}: {e}"}

    if args.leg("c5"):
        # a short served leg: 2 s of requests at 5 % of the offered load (below saturation,
        # where latency is the server's own) and at the full, overloaded rate.  It runs
        # before the ragged batch, whose many handles leave the device memory fragmented
        # enough to cut the server's batches.
        c5_line = guarded("c5", lambda: run_c5(args, tda, torch, synth, dev, log, 2.0,
                                               [0.05, 1.0], ("mixed",)))
    if args.leg("c4"):
        # the 64-instance ragged batch (one batched evaluation per step, compact handles)
        c4_line = guarded("c4", lambda: run_c4(args, tda, torch, synth, dev, log, 4, 1))
        c4_line.pop("wall", None)

    evals_m = inst.B * args.steps / wall_m
    evals_f = inst.B * fsteps / wall_f
    if gs is not None:
        # the Toeplitz (Gohberg-Semencul) route needs gap-free segments; on this gap-free
        # workload it is the fastest exact-enough method, while gapped data (the c3 key)
        # take the Cholesky paths
        gs["speedup_vs_mixed"] = gs["value"] / evals_m
        gs["applies_to"] = "segments without gaps (Toeplitz covariance)"

    # dominant kernel of the mixed step and its roofline (algorithmic flops: one
    # triangular product = N_eff^2 flops per template and detector)
    dom = max((k for k in kt_m if k.startswith("trmm")), key=lambda k: kt_m[k][1])
    cnt, tot = kt_m[dom]
    alg_flops = float(sum(n * n for n in n_eff)) * inst.B
    achieved = alg_flops / (tot / cnt * 1e-3)
    # frac: the dominant kernel alone (one product launch); step_frac: the whole step's
    # algorithmic rate (the same N_eff^2 B flops over ms_per_step)
    step_rate = alg_flops / (wall_m / args.steps)
    roofline = {"bound": "mfma", "kernel": dom, "achieved": achieved / 1e12,
                "peak": PEAK_BF16 / 1e12, "unit": "TFLOP/s", "frac": achieved / PEAK_BF16,
                "traffic": profiled_traffic(dom), "traffic_unit": "bytes per launch",
                "avg_ms": tot / cnt, "issued_frac": 3 * achieved / PEAK_BF16,
                "step_achieved": step_rate / 1e12, "step_frac": step_rate / PEAK_BF16,
                "alg_flops_per_step": alg_flops}
    clk = profiled_clock(dom)
    if clk is not None:
        # under sustained BF16 matrix load the chip runs below the 2.4 GHz the published peak
        # assumes; the counter run gives the clock this kernel held and its matrix-core busy
        # fraction at that clock (profiles/utilisation_c2.md)
        roofline["sustained_clock_ghz"] = clk[0]
        roofline["frac_at_sustained_clock"] = achieved / (PEAK_BF16 * clk[0] / 2.4)
        roofline["mfma_busy_at_sustained_clock"] = clk[1]
    dom_f = "trsm_f64"
    cf, tf = kt_f[dom_f]
    ach_f = alg_flops / (tf / cf * 1e-3)

    line = {
        "metric": METRIC,
        "value": evals_m,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall_m / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3+f64",
        "data": "synthetic",
        "config": {"workload": f"two detectors x N={inst.N} (fs=4096 Hz), {inst.B} chirp templates "
                               f"per launch, analytic-PSD ACF + nugget {synth.EPS_PRIMARY:g}, no gaps",
                   "n_det": inst.n_det, "N": inst.N, "templates_per_launch": inst.B,
                   "n_eff": n_eff,
                   "template_amplitudes": "network SNR 8-30 by the band-limited (20-2048 Hz) "
                                          "frequency-domain convention; the time-domain h^T C^-1 h "
                                          "the library evaluates is larger (sharp chirp ends)"},
        "latency_ms": {"p50": _pct(lat_m, 50), "p99": _pct(lat_m, 99),
                       "unit": "one launch of all templates"},
        "fp64": {"value": evals_f, "unit": "evals/s", "ms_per_step": wall_f / fsteps * 1e3,
                 "steps": fsteps, "latency_ms": {"p50": _pct(lat_f, 50), "p99": _pct(lat_f, 99)},
                 "roofline": {"bound": "mfma", "kernel": dom_f, "achieved": ach_f / 1e12,
                              "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
                              "frac": ach_f / PEAK_FP64, "avg_ms": tf / cf}},
        "speedup_mixed_vs_fp64": evals_m / evals_f,
        "gs_fp64": gs,
        "cdo_fp64": cdo,
        "acf_estimate": acf_line,
        "snr_terms": snr_terms,
        "whitened_residual": wres,
        "accuracy_stress": stress,
        "c3": c3_line,
        "c4": c4_line,
        "c5_served": c5_line,
        "accuracy": {"max_abs_dlogL_mixed_vs_fp64_gpu": float(d_mf.max()),
                     "p99_abs_dlogL_mixed_vs_fp64_gpu": _pct(d_mf, 99),
                     "templates_compared": int(inst.B)},
        "roofline": roofline,
        "kernels_ms": {k: v[1] / v[0] for k, v in kt_m.items()},
        "setup_s": setup,
    }
    if args.calib_copy_mib:
        nel = args.calib_copy_mib * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        line["calib_copy_bytes"] = 2 * nel * 8
        del src, dst
    if not args.no_cpu_baseline:
        fs = []
        ref, cb = cpu_baseline(inst, args.cpu_sample, fs)
        cb["host"] = host_cpu()
        n_proc = min([x for x in (cb["host"]["physical_cores"], cb["host"]["affinity_cpus"], 16)
                      if x])
        try:
            ref_p, pool = cpu_pool_baseline(inst, fs, args.cpu_sample, n_proc)
            pool["max_abs_dlogL_vs_batched_oracle"] = float(np.abs(ref_p - ref).max())
            cb["pool"] = pool
            log("cpu pool baseline", pool)
        except Exception as e:  # reported, never fatal to the GPU line
            cb["pool"] = {"error": repr(e)}
        line["cpu_baseline"] = cb
        line["accuracy"]["max_abs_dlogL_mixed_vs_oracle"] = float(np.abs(res_m[:len(ref)] - ref).max())
        line["accuracy"]["max_abs_dlogL_fp64_vs_oracle"] = float(np.abs(res_f[:len(ref)] - ref).max())
        line["accuracy"]["oracle_sample"] = len(ref)
    print(json.dumps(line), flush=True)
    for h in hs:
        h.close()


def one_time_costs(kt, n_eff, n_pad):
    """Assembly and Cholesky figures from the timed set-up launches: the assembly writes
    n_pad^2 doubles per detector (the dense block, lower part used); the Cholesky does
    N_eff^3 / 3 algorithmic flops per detector."""
    res = {}
    if "assemble" in kt:
        c, t = kt["assemble"]
        byts = float(sum(n * n for n in n_pad)) * 8.0
        res["assembly"] = {"ms": t, "launches": c, "bytes": byts, "GB_per_s": byts / t * 1e-6,
                           "frac_hbm_peak": byts / (t * 1e-3) / PEAK_HBM}
    if "cholesky" in kt:
        c, t = kt["cholesky"]
        fl = float(sum(n ** 3 for n in n_eff)) / 3.0
        res["cholesky"] = {"ms": t, "launches": c, "flops": fl, "TFLOP_per_s": fl / t * 1e-9,
                           "frac_fp64_peak": fl / (t * 1e-3) / PEAK_FP64}
    for k in ("data_check", "data_whiten"):
        if k in kt:
            res[k + "_ms"] = kt[k][1]
    return res


def _base_line(args, value, unit, wall, steps, config, dtype):
    return {"metric": METRIC, "value": value, "unit": unit, "n_gpus": 1, "steps": steps,
            "warmup": args.warmup, "ms_per_step": wall / max(steps, 1) * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": "synthetic", "config": config}


GOLD = os.path.join(ROOT, "tests", "golden")


def _gold(name):
    """Stored oracle values for sampled templates (written by tests/golden/make_golden.py,
    which calls only the oracle), or None."""
    try:
        return json.load(open(os.path.join(GOLD, f"{name}_sample.json")))
    except OSError:
        return None


def stress_leg(args, tda, torch, synth, dev, log):
    """Two detectors x N at smaller nuggets, down to the stress nugget 1e-8 (kappa(C) up to
    2.9e8): mixed vs FP64 over every template at each nugget (where mixed stops meeting
    1e-3), and at 1e-8 also Gohberg-Semencul and the explicit inverse vs FP64 and all paths
    against the stored oracle rows."""
    sweep, res = [], {}
    for eps in (1e-7, 3e-8, synth.EPS_STRESS):
        w = synth.c2_workload(eps=eps, B=args.templates, n=args.n)
        inst = w.instances[0]
        d = [torch.from_numpy(x).to(dev) for x in inst.d]
        H = torch.from_numpy(inst.H).to(dev)
        hs = [tda.Handle(inst.acf, inst.N, m, precision="mixed").factor() for m in inst.masks]
        out = {p: torch.empty(inst.B, dtype=torch.float64, device=dev) for p in ("mixed", "fp64")}
        for p in out:
            tda.loglik_multi([(h, dk, H, out[p]) for h, dk in zip(hs, d)], precision=p)
        torch.cuda.synchronize()
        rm, rf = out["mixed"].cpu().numpy(), out["fp64"].cpu().numpy()
        lo, hi = synth.eig_bounds(eps)
        dm = np.abs(rm - rf)
        pt = {"eps": eps, "kappa_bound": hi / lo,
              "max_abs_dlogL_mixed_vs_fp64_gpu": float(dm.max()),
              "p99_abs_dlogL_mixed_vs_fp64_gpu": _pct(dm, 99),
              "templates_above_1e-3": int(np.sum(dm > 1e-3)),
              "min_dlogL_mixed_minus_fp64": float((rm - rf).min())}
        sweep.append(pt)
        log("nugget", pt)
        if eps == synth.EPS_STRESS:
            t = time.perf_counter()
            for _ in range(3):
                tda.loglik_multi([(h, dk, H, out["mixed"]) for h, dk in zip(hs, d)],
                                 precision="mixed")
            torch.cuda.synchronize()
            res = dict(pt)
            res["templates_compared"] = int(inst.B)
            res["mixed_ms_per_step"] = (time.perf_counter() - t) / 3 * 1e3
            res["meets_1e-3_vs_fp64"] = bool(dm.max() <= 1e-3)
            rc = sum(h.loglik(dk, H, precision="cdo") for h, dk in zip(hs, d)).cpu().numpy()
            hg = [tda.Handle(inst.acf, inst.N, None, precision="gs").factor() for _ in hs]
            og = torch.empty(inst.B, dtype=torch.float64, device=dev)
            tda.loglik_multi([(h, dk, H, og) for h, dk in zip(hg, d)], precision="gs")
            rg = og.cpu().numpy()
            res["max_abs_dlogL_gs_vs_fp64_gpu"] = float(np.abs(rg - rf).max())
            res["max_abs_dlogL_cdo_vs_fp64_gpu"] = float(np.abs(rc - rf).max())
            gold = _gold("c2_stress")
            if gold and gold["N"] == inst.N and gold["eps"] == eps and inst.B > max(gold["rows"]):
                rows, want = np.array(gold["rows"]), np.array(gold["loglik"])
                for k, r in (("mixed", rm), ("fp64", rf), ("gs", rg), ("cdo", rc)):
                    res[f"max_abs_dlogL_{k}_vs_oracle"] = float(np.abs(r[rows] - want).max())
                res["oracle_rows"] = len(rows)
            for h in hg:
                h.close()
        for h in hs:
            h.close()
        del d, H
    res["nugget_sweep"] = sweep
    ok = [p["kappa_bound"] for p in sweep if p["max_abs_dlogL_mixed_vs_fp64_gpu"] <= 1e-3]
    bad = [p["kappa_bound"] for p in sweep if p["max_abs_dlogL_mixed_vs_fp64_gpu"] > 1e-3]
    res["mixed_meets_1e-3_up_to_kappa"] = max(ok) if ok else None
    res["mixed_misses_1e-3_from_kappa"] = min(bad) if bad else None
    log("stress nugget", res)
    return res


def run_c3(args, tda, torch, synth, dev, log, steps, fsteps):
    """One detector, N = 32768 with 3 gaps (the masked covariance C[mask, mask], one
    segment whose circulant refines with split transforms), 8192 templates per launch:
    mixed and FP64 evaluations through the same handle, and the stored oracle rows."""
    t0 = time.perf_counter()
    w = synth.c3_workload()
    inst = w.instances[0]
    log(f"c3 inputs in {time.perf_counter() - t0:.1f} s")
    d = torch.from_numpy(inst.d[0]).to(dev)
    H = torch.from_numpy(inst.H).to(dev)
    tda.timing_read(reset=True)
    tda.timing_enable(True)
    t0 = time.perf_counter()
    h = tda.Handle(inst.acf, inst.N, inst.masks[0], precision="mixed").factor()
    h.set_data(d)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    tda.timing_enable(False)
    info = h.info()
    one_time = one_time_costs(tda.timing_read(reset=True), [info["n_eff"]], [info["n_pad"]])
    log(f"c3 setup {setup:.1f} s, n_eff {info['n_eff']}")
    res = {}
    for p in ("mixed", "fp64"):
        out = torch.empty(inst.B, dtype=torch.float64, device=dev)
        for _ in range(args.warmup if p == "mixed" else 1):
            h.loglik(d, H, out=out, precision=p)
        torch.cuda.synchronize()
        tda.timing_read(reset=True)
        tda.timing_enable(True)
        n = steps if p == "mixed" else fsteps
        t = time.perf_counter()
        for _ in range(n):
            h.loglik(d, H, out=out, precision=p)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        tda.timing_enable(False)
        res[p] = (wall, n, tda.timing_read(reset=True), out.cpu().numpy())
        log(f"c3 {p}: {wall / n * 1e3:.2f} ms/step")
    h.close()
    wall, n, kt, rm = res["mixed"]
    fw, fn, _, rf = res["fp64"]
    alg = float(info["n_eff"]) ** 2 * inst.B
    line = {"value": inst.B * n / wall, "unit": "evals/s", "ms_per_step": wall / n * 1e3,
            "steps": n,
            "config": {"workload": f"one detector x N={inst.N} with 3 gaps (64-512 samples), "
                                   f"{inst.B} chirp templates per launch", "n_eff": info["n_eff"]},
            "fp64": {"value": inst.B * fn / fw, "unit": "evals/s", "ms_per_step": fw / fn * 1e3,
                     "steps": fn},
            "step_frac_bf16": alg / (wall / n) / PEAK_BF16,
            "kernels_ms": {k: v[1] / v[0] for k, v in kt.items()},
            "setup_s": setup, "one_time": one_time}
    line["speedup_mixed_vs_fp64"] = line["value"] / line["fp64"]["value"]
    dm = np.abs(rm - rf)
    line["accuracy"] = {"max_abs_dlogL_mixed_vs_fp64_gpu": float(dm.max()),
                        "p99_abs_dlogL_mixed_vs_fp64_gpu": _pct(dm, 99)}
    gold = _gold("c3")
    if gold and gold["N"] == inst.N:
        rows, want = np.array(gold["rows"]), np.array(gold["loglik"])
        line["accuracy"]["max_abs_dlogL_mixed_vs_oracle"] = float(np.abs(rm[rows] - want).max())
        line["accuracy"]["max_abs_dlogL_fp64_vs_oracle"] = float(np.abs(rf[rows] - want).max())
        line["accuracy"]["oracle_rows"] = len(rows)
    log("c3", line)
    return line


def bench_c3(args, tda, torch, synth, dev, log):
    """The gapped one-detector workload alone (see run_c3)."""
    c3 = run_c3(args, tda, torch, synth, dev, log, args.steps, max(2, args.steps // 4))
    line = _base_line(args, c3["value"], "evals/s", c3["ms_per_step"] * c3["steps"] * 1e-3,
                      c3["steps"], c3.pop("config"), "bf16x3+f64")
    line.update({k: v for k, v in c3.items() if k not in ("value", "unit", "ms_per_step", "steps")})
    print(json.dumps(line), flush=True)


def run_c4(args, tda, torch, synth, dev, log, steps_m, warmup):
    """64 ragged instances (N ~ U{2048..32768}, 0-2 gaps per detector, 1-2 detectors,
    256 templates each) evaluated in one batched launch sequence per step.  The mixed pass
    keeps only the BF16 operators of its handles (compact); the FP64 pass builds FP64
    handles afterwards (both sets at once would exceed HBM).  Returns the key set of the
    line (value, config, fp64, accuracy, kernels, setup)."""
    t0 = time.perf_counter()
    w = synth.c4_workload()
    log(f"c4 inputs in {time.perf_counter() - t0:.1f} s")
    n_eval = sum(inst.B for inst in w.instances)
    Hs = [torch.from_numpy(inst.H).to(dev) for inst in w.instances]
    ds = [[torch.from_numpy(inst.d[k]).to(dev) for k in range(inst.n_det)] for inst in w.instances]
    res = {}
    for p in ("mixed", "fp64"):
        t0 = time.perf_counter()
        items, outs, keep = [], [], []
        for inst, H, dks in zip(w.instances, Hs, ds):
            o = torch.empty(inst.B, dtype=torch.float64, device=dev)
            for k in range(inst.n_det):
                h = tda.Handle(inst.acf, inst.N, inst.masks[k], precision=p,
                               compact=(p == "mixed")).factor()
                if p == "mixed":
                    h.set_data(dks[k])
                items.append((h, dks[k], H, o))
                keep.append(h)
            outs.append(o)
        torch.cuda.synchronize()
        setup = time.perf_counter() - t0
        log(f"c4 {p}: setup {setup:.1f} s, {len(items)} detector items, {n_eval} evals per step")
        for _ in range(warmup):
            tda.loglik_multi(items, precision=p)
        torch.cuda.synchronize()
        tda.timing_read(reset=True)
        tda.timing_enable(True)
        t = time.perf_counter()
        steps = steps_m if p == "mixed" else max(2, steps_m // 4)
        for _ in range(steps):
            tda.loglik_multi(items, precision=p)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        tda.timing_enable(False)
        res[p] = (wall, steps, tda.timing_read(reset=True),
                  np.concatenate([o.cpu().numpy() for o in outs]), setup, len(items))
        for h in keep:
            h.close()
        del items, keep
        torch.cuda.synchronize()
        log(f"c4 {p}: {wall / steps * 1e3:.2f} ms/step")
    wall, steps, kt, rm, setup, n_items = res["mixed"]
    fw, fs, fkt, rf, fsetup, _ = res["fp64"]
    c4 = {"value": n_eval * steps / wall, "unit": "evals/s", "ms_per_step": wall / steps * 1e3,
          "steps": steps, "wall": wall,
          "config": {"workload": "64 ragged instances, N~U{2048..32768}, 0-2 gaps, 1-2 detectors, "
                                 "256 templates each, one batched evaluation per step",
                     "instances": len(w.instances), "detector_items": n_items},
          "fp64": {"value": n_eval * fs / fw, "unit": "evals/s", "ms_per_step": fw / fs * 1e3,
                   "setup_s": fsetup},
          "accuracy": {"max_abs_dlogL_mixed_vs_fp64_gpu": float(np.abs(rm - rf).max()),
                       "p99_abs_dlogL_mixed_vs_fp64_gpu": _pct(np.abs(rm - rf), 99),
                       "evals_compared": int(rm.size)},
          "kernels_ms": {k: v[1] / v[0] for k, v in kt.items()},
          "setup_s": setup}
    c4["speedup_mixed_vs_fp64"] = c4["value"] / c4["fp64"]["value"]
    # the handles took their memory through torch's caching allocator; give it back
    torch.cuda.empty_cache()
    return c4


def bench_c4(args, tda, torch, synth, dev, log):
    """The ragged batch alone (see run_c4)."""
    c4 = run_c4(args, tda, torch, synth, dev, log, args.steps, args.warmup)
    line = _base_line(args, c4["value"], "evals/s", c4.pop("wall"), c4["steps"], c4.pop("config"),
                      "bf16x3+f64")
    line.update({k: v for k, v in c4.items() if k not in ("value", "unit", "steps", "ms_per_step")})
    print(json.dumps(line), flush=True)


def _serve_trace(srv, req, Hs, out_dev, torch):
    """Replay a request trace against a server in real time; returns (wall, stats, templates)."""
    n = len(req["t"])
    counts = req["count"]
    out = torch.empty(int(counts.sum()), dtype=torch.float64, device=out_dev)
    offs = np.concatenate([[0], np.cumsum(counts)[:-1]])
    bank = Hs[0].shape[0]
    tickets = []
    srv.stats(reset=True)
    t_start = time.perf_counter()
    for k in range(n):
        delay = req["t"][k] - (time.perf_counter() - t_start)
        if delay > 0:
            time.sleep(delay)
        ds = int(req["dataset"][k])
        c = int(counts[k])
        r0 = min(int(req["start"][k]), bank - c)
        tk = None
        while tk is None:
            tk = srv.submit(ds, Hs[ds][r0:r0 + c], out[offs[k]:offs[k] + c])
        tickets.append(tk)
    for tk in tickets:
        srv.wait(tk, 600.0)
    wall = time.perf_counter() - t_start
    return wall, srv.stats(), int(counts.sum())


def run_c5(args, tda, torch, synth, dev, log, duration, fracs, precisions):
    """Request server: 32 resident single-detector datasets (N in 4096..65536), Poisson
    arrivals of 1-64-template requests from 512 simulated walkers, at the offered loads
    `fracs` (fractions of --rate) for `duration` seconds each; the FP64 server (if asked
    for) replays every 20th request of the full trace."""
    t0 = time.perf_counter()
    w = synth.c5_workload(duration_s=duration, rate_hz=args.rate)
    log(f"c5 inputs in {time.perf_counter() - t0:.1f} s")
    # the batched evaluations before this leg keep workspaces sized for their largest
    # batch; the server's slots need that memory for their own
    tda.release_workspaces()
    torch.cuda.empty_cache()
    # the server runs the default product variant: tuning trials for every coalesced
    # batch shape would otherwise land inside the latency measurements
    saved = os.environ.get("TDA_AUTOTUNE")
    os.environ["TDA_AUTOTUNE"] = "0"
    sweep, res = [], {}
    for prec in precisions:
        t0 = time.perf_counter()
        srv = tda.Server(precision=prec, n_slots=3, max_batch=2048, staging_bytes=256 << 20)
        keep, Hs = [], []
        for inst in w.instances:
            h = tda.Handle(inst.acf, inst.N, inst.masks[0], precision=prec,
                           compact=(prec == "mixed")).factor()
            dk = torch.from_numpy(inst.d[0]).to(dev)
            H = torch.from_numpy(inst.H).to(dev)
            srv.add_dataset(h, dk)
            keep.append((h, dk))
            Hs.append(H)
        torch.cuda.synchronize()
        # the handles took their memory through torch's caching allocator, which keeps what
        # the compaction released; hand it back for the server's own workspaces
        torch.cuda.empty_cache()
        setup = time.perf_counter() - t0
        log(f"c5 {prec}: setup {setup:.1f} s")
        try:
            _c5_serve(args, srv, w, prec, fracs, duration, Hs, dev, torch, synth, log, sweep, res,
                      setup)
        finally:
            srv.close()
        del keep, Hs
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    if saved is None:
        os.environ.pop("TDA_AUTOTUNE", None)
    else:
        os.environ["TDA_AUTOTUNE"] = saved
    return _c5_line(args, res, sweep, duration, fracs)


def _c5_serve(args, srv, w, prec, fracs, duration, Hs, dev, torch, synth, log, sweep, res, setup):
    """The timed traces of one server (run_c5)."""
    # untimed warm-up (code loading, first allocations)
    _serve_trace(srv, synth.c5_requests(args.rate * min(fracs), 0.5, trace=99), Hs, dev, torch)
    if prec == "mixed":
        for i, f in enumerate(fracs):
            req = w.requests if f == 1.0 else synth.c5_requests(args.rate * f, duration,
                                                                 trace=i + 1)
            wall, st, tmpl = _serve_trace(srv, req, Hs, dev, torch)
            point = {"offered_evals_per_s": tmpl / duration,
                     "achieved_evals_per_s": tmpl / wall, "requests": len(req["t"]),
                     "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
                     "mean_templates_per_launch": st["mean_templates_per_launch"]}
            # the server kept up when the trace drained within 10 % of its length
            point["below_saturation"] = bool(wall <= 1.1 * duration)
            sweep.append(point)
            log(f"c5 mixed at {f:g} x {args.rate:g} req/s: {point}")
            if f == max(fracs):
                res[prec] = (wall, st, setup, len(req["t"]), tmpl)
    else:
        req = {k: v[::20] for k, v in w.requests.items()}
        wall, st, tmpl = _serve_trace(srv, req, Hs, dev, torch)
        res[prec] = (wall, st, setup, len(req["t"]), tmpl)
        log(f"c5 fp64: {st}")


def _c5_line(args, res, sweep, duration, fracs):
    wall, st, setup, n, tmpl = res["mixed"]
    top = max(fracs)
    line = {"value": tmpl / wall, "unit": "evals/s",
            "config": {"workload": f"request server: 32 resident datasets N in 4096..65536, "
                                   f"Poisson {args.rate * top:g} req/s x {duration:g} s, 1-64 "
                                   f"templates per request, 512 walkers", "requests": n,
                       "templates": tmpl},
            "latency_ms": {"p50": st["p50_ms"], "p99": st["p99_ms"], "max": st["max_ms"],
                           "unit": "submit to results written"},
            "offered_evals_per_s": tmpl / duration, "server": st, "load_sweep": sweep,
            "setup_s": setup}
    if "fp64" in res:
        fw, fst, fsetup, fn, ftmpl = res["fp64"]
        line["fp64"] = {"value": ftmpl / fw, "unit": "evals/s", "offered_fraction": 1 / 20,
                        "latency_ms": {"p50": fst["p50_ms"], "p99": fst["p99_ms"]},
                        "setup_s": fsetup}
    return line


def bench_c5(args, tda, torch, synth, dev, log):
    """The request server alone over the --rates sweep (see run_c5)."""
    fracs = [float(x) for x in args.rates.split(",") if x.strip()]
    c5 = run_c5(args, tda, torch, synth, dev, log, args.duration, fracs, ("mixed", "fp64"))
    wall = c5["server"]["busy_s"] or 1.0
    line = _base_line(args, c5["value"], "evals/s", wall, 1, c5.pop("config"), "bf16x3+f64")
    line.update({k: v for k, v in c5.items() if k not in ("value", "unit")})
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
