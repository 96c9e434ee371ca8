"""Benchmark: one step = one complete pass of the hot path on the device.

Default workload: the large multichannel image, P=3 channels of 4096x4096,
K=25 atoms of 3x32x32 (Gaussian, unit norm), Bernoulli(5e-4) x Exp(1)
activations, noise sigma=0.05, lambda = 0.1 lambda_max, at its configured
precision: FP32 incremental beta/z, the beta initialisation on the BF16
matrix cores with FP32 accumulation, one FP64 drift correction of beta and the
FP64 objective/KKT check; then the dictionary statistics ztz (K x K x 63 x 63)
and ztX of the solved z.  A step runs DtD and its apply table, the beta
initialisation, the LGCD + soft-lock rounds to the sweep certificate
(tol = 1e-5 lambda), the verification (strict KKT <= 1e-4 lambda), any polish
pass it asks for, and the statistics.  Inputs are resident in HBM before the
timed region starts.

Prints one JSON line.  value = accepted coordinate updates per second over the
timed steps; ms_per_step = one whole step; time_to_kkt_tol_ms = the solve.
Other workloads: --workload image_1024 (1024x1024, K=25 atoms 16x16, on its
configured 16x16 worker grid), signal_1d, batch_images, serving, corr, ablation.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_1901_09235_amd", "csrc")


def kernel_source_digest() -> str:
    """Digest of the source that defines the round kernel: counter results are
    only used while that kernel is unchanged."""
    import hashlib
    with open(os.path.join(CSRC, "dcdl_device.h"), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def stored_traffic(workload: str, grid, tile):
    """HBM bytes per launch of the round kernel from the committed rocprofv3
    FETCH_SIZE/WRITE_SIZE runs, if they were taken on the current sources and
    on the same worker grid and sub-domain tile."""
    path = os.path.join(PROFILES, f"traffic_lgcd_rounds_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_digest") != kernel_source_digest():
        return None
    if rec.get("grid") != list(grid) or rec.get("tile") != list(tile):
        return None
    return rec


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="image_rgb_4096",
                    choices=["image_1024", "signal_1d", "image_rgb_4096", "batch_images", "serving", "corr",
                             "ablation"])
    ap.add_argument("--requests", type=int, default=2000, help="measured requests of the serving workload")
    ap.add_argument("--serve-warmup", type=int, default=200, help="warm-up requests of the serving workload")
    ap.add_argument("--pool", type=int, default=48, help="distinct request signals of the serving workload")
    ap.add_argument("--budgets", default="0,2048,512",
                    help="serving: HBM admission budgets in MiB to sweep (0: the server default)")
    ap.add_argument("--rate", type=float, default=200.0, help="Poisson arrival rate of the serving workload")
    ap.add_argument("--rates", default="", help="serving: comma-separated offered rates to sweep (e.g. 200,600,1200)")
    ap.add_argument("--admit", type=int, default=0,
                    help="server: workgroups of the admitted requests at most (0: one launch, -1: unbounded)")
    ap.add_argument("--max-workers", type=int, default=0, help="server: workgroups per request at most")
    ap.add_argument("--slice", type=int, default=0, help="server: rounds per launch")
    ap.add_argument("--batch-n", type=int, default=256, help="instances of the batch workload")
    ap.add_argument("--plain", type=int, default=-1,
                    help="batch workload: also time this many instances one solve per call "
                         "(-1: all of them, 0: skip)")
    ap.add_argument("--size", type=int, default=0, help="override the image side (testing)")
    ap.add_argument("--grid", type=int, nargs="*", default=None)
    ap.add_argument("--tile", type=int, nargs="*", default=None)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--inner", type=int, default=0, help="sub-domain visits per worker per round (0: 1)")
    ap.add_argument("--no-autotune", action="store_true", help="batch: skip the autotuner (defaults)")
    ap.add_argument("--ablation-cap", type=float, default=30.0,
                    help="ablation: wall-clock cap of one solve in seconds")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-grid16", action="store_true",
                    help="image_1024: skip the extra solve on a 16 x 16 worker grid (profiling runs)")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="side of the oracle's crop (0: 192 for the RGB image, 128 for the 1024^2 image)")
    ap.add_argument("--cpu-kkt-every", type=int, default=8,
                    help="oracle baseline: sweeps between its strict-KKT evaluations")
    ap.add_argument("--precision", default="",
                    help="beta initialisation contraction: bf16, bf16x3, f64, direct or auto "
                         "(default: bf16 for the RGB image, auto otherwise)")
    ap.add_argument("--fix-after", type=int, default=-1,
                    help="sweeps before the one FP64 drift correction of beta (0: none before the check; "
                         "-1: the workload's default)")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the untimed solves at the other initialisation precisions / worker grid")
    ap.add_argument("--probe-mib", type=int, default=1024, help="copy-probe size (0: skip)")
    return ap.parse_args()


def make_workload(args):
    from paper_1901_09235_amd import synth
    if args.workload == "signal_1d":
        return synth.signal_1d()
    if args.workload == "image_rgb_4096":
        return synth.image_4096_rgb(size=args.size or 4096)
    return synth.image_1024(size=args.size or 1024)


def algorithmic_bytes(patched_positions, visit_positions, checked_positions, K, s_beta, s_move):
    """Bytes the method itself moves in the round kernel (see the design notes).
    Per patched position of an accepted update: K beta values read and written
    and K DtD entries read (eq. beta_update).  Per position of a visited
    sub-domain and per position inspected by a soft-lock test: one cached
    best-move entry read."""
    return patched_positions * K * 3 * s_beta + (visit_positions + checked_positions) * s_move


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(args):
    """The FP64 oracle (plain sequential C, one thread) timed on one pinned
    host core, on a bounded crop of the workload's own recipe.  Runs before
    any GPU call; the process's CPU affinity is restored afterwards.

    Two oracle runs on the same crop: the first gives the time to the sweep
    tolerance (beta from X plus the sweeps), the second evaluates the strict
    FP64 KKT every --cpu-kkt-every sweeps (evaluations not timed) and gives the
    sweep time at which it first reads <= 1e-4 lambda."""
    import oracle
    from paper_1901_09235_amd import synth
    wl = args.workload
    if wl == "signal_1d":
        pb = synth.signal_1d()
        sample = "the whole 1-D signal (T=5000, K=5, L=64)"
    elif wl == "image_rgb_4096":
        side = args.cpu_sample or 192
        pb = synth.image_4096_rgb(size=side)
        sample = f"3x{side}x{side} crop of the RGB recipe (K=25 atoms 3x32x32, seed 3000)"
    else:
        side = args.cpu_sample or 128
        pb = synth.image_1024(size=side)
        sample = f"{side}x{side} crop of the 1024^2 recipe (K=25 atoms 16x16, seed 2000)"
    prev = os.sched_getaffinity(0)
    core = min(prev)
    os.sched_setaffinity(0, {core})
    try:
        lam = pb.lambda_frac * oracle.lambda_max(pb.X, pb.D)
        tol = pb.tol_rel if pb.tol_abs else pb.tol_rel * lam
        t0 = time.perf_counter()
        _, info = oracle.lgcd(pb.X, pb.D, lam, tol)
        wall = time.perf_counter() - t0
        init_s = wall - info["t_solve_s"]
        _, ik = oracle.lgcd(pb.X, pb.D, lam, tol, kkt_every=args.cpu_kkt_every, kkt_target=1e-4)
    finally:
        os.sched_setaffinity(0, prev)
    t_kkt = init_s + ik["t_kkt_s"] if ik["t_kkt_s"] >= 0 else None
    return {"value": info["n_updates"] / wall, "unit": "updates/s", "cores": 1, "kind": "oracle",
            "sample": sample, "pinned_core": core, "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
            "time_to_tol_s": round(wall, 4), "time_to_kkt_1e-4_s": None if t_kkt is None else round(t_kkt, 4),
            "kkt_resolution_sweeps": args.cpu_kkt_every, "init_s": round(init_s, 4),
            "updates": info["n_updates"], "sweeps": info["n_sweeps"],
            "note": "oracle beta init by direct FP64 loops, then sequential LGCD sweeps"}


def run_batch(args):
    """Batching pattern: n uneven images sharing a dictionary, solved in one
    persistent launch per step, beside the plain form (one solve per call)."""
    import numpy as np
    import torch
    import paper_1901_09235_amd as dl
    from paper_1901_09235_amd import synth

    t0 = time.perf_counter()
    D_np, pbs = synth.batch_images(n=args.batch_n)
    t_gen = time.perf_counter() - t0
    D = torch.from_numpy(D_np).to("cuda", dtype=torch.float32).contiguous()
    Xs = [torch.from_numpy(pb.X).to("cuda", dtype=torch.float32).contiguous() for pb in pbs]
    lams = [pb.lambda_frac * dl.dicodile_lambda_max(X, D) for pb, X in zip(pbs, Xs)]
    tols = [1e-5 * l for l in lams]
    zs = [torch.empty((D.shape[0], X.shape[1] - D.shape[2] + 1, X.shape[2] - D.shape[3] + 1),
                      dtype=torch.float32, device="cuda") for X in Xs]
    bopts = {}
    tune = None
    if args.threads or args.tile:
        if args.threads:
            bopts["threads"] = args.threads
        if args.tile:
            bopts["tile"] = tuple(args.tile) if len(args.tile) > 1 else args.tile[0]
    elif not args.no_autotune:
        bopts, tune = dl.dicodile_csc_batch_autotune(Xs, D, lams, tols)
        print(f"# autotuned {bopts} in {tune['t_tune_s']:.1f} s", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        dl.dicodile_csc_batch(Xs, D, lams, tols, z_outs=zs, **bopts)
    torch.cuda.synchronize()
    t_default = None
    if tune is not None and (tuple(bopts.get("tile", ())) != (2 * D.shape[2], 2 * D.shape[3])
                             or bopts.get("threads", 256) != 256 or bopts.get("workers", 0)):
        # the default configuration beside the tuned one (outside the timed region)
        t0 = time.perf_counter()
        _, _, bd = dl.dicodile_csc_batch(Xs, D, lams, tols, z_outs=zs)
        torch.cuda.synchronize()
        t_default = time.perf_counter() - t0
    binfos, t0 = [], time.perf_counter()
    for _ in range(args.steps):
        _, infos, binfo = dl.dicodile_csc_batch(Xs, D, lams, tols, z_outs=zs, **bopts)
        binfos.append(binfo)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    if any(b["n_converged"] != len(pbs) for b in binfos):
        raise SystemExit(f"batch did not converge: {binfos[-1]}")
    n_plain = len(pbs) if args.plain < 0 else min(args.plain, len(pbs))
    t_plain = None
    plain_kkt = 0.0
    if n_plain > 0:
        t0 = time.perf_counter()
        for X, z, lam, tol in list(zip(Xs, zs, lams, tols))[:n_plain]:
            _, info = dl.dicodile_csc(X, D, lam, tol, z_out=z, max_rounds=50_000_000, timeout_s=120)
            plain_kkt = max(plain_kkt, info["kkt"])
            if info["status"] != "OK":
                raise SystemExit(f"plain solve did not converge: {info}")
        torch.cuda.synchronize()
        t_plain = (time.perf_counter() - t0) / n_plain * len(pbs)
    upd = binfos[-1]["n_updates"]
    out = {
        "metric": "CSC time-to-KKT-tol & coord updates/s; batched vs plain",
        "value": len(pbs) / dt, "unit": "instances/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batch_{len(pbs)}_images_128-1024_K16_L12", "dictionary": list(D.shape),
                   "lambda": "0.1 lambda_max each", "tol": "1e-5 lambda each",
                   "positions": int(sum((X.shape[1] - 11) * (X.shape[2] - 11) for X in Xs))},
        "updates_per_s": upd / dt,
        "max_kkt": max(i["kkt"] for i in infos),
        "batched_phase_ms": {"setup": binfos[-1]["t_setup_s"] * 1e3, "rounds": binfos[-1]["t_rounds_s"] * 1e3,
                             "check": binfos[-1]["t_check_s"] * 1e3},
        "roofline": _rounds_roofline(infos, binfos[-1]["t_rounds_s"], D.shape[0]),
        "workers": binfos[-1]["workers"], "launches": binfos[-1]["n_passes"],
        "used_graph": binfos[-1]["used_graph"],
        "batch_opts": {k: (list(v) if isinstance(v, tuple) else v) for k, v in bopts.items()},
        "autotune": tune,
        "default_config_s": t_default,
        "plain_s_for_all": t_plain,
        "plain_instances_timed": n_plain,
        "batched_over_plain": (t_plain / dt) if t_plain else None,
        "generation_s": t_gen,
    }
    stored = stored_gap("batch_256_images_128-1024_K16_L12")
    if stored is not None and len(pbs) == 256:
        out["objective_gap_vs_oracle"] = stored.get("summary")
    print(json.dumps(out), flush=True)


def _percentiles(v):
    import numpy as np
    a = np.sort(np.asarray(v, dtype=np.float64))
    return {"p50_ms": float(np.percentile(a, 50) * 1e3), "p99_ms": float(np.percentile(a, 99) * 1e3),
            "mean_ms": float(a.mean() * 1e3), "max_ms": float(a.max() * 1e3)}


def _rounds_roofline(infos, t_rounds, K, s_beta=4, s_move=8):
    """HBM roofline of the round kernel from per-solve counters summed over
    solves and the round kernel's event time over the same solves."""
    patched = sum(i["n_patched"] for i in infos)
    visit_pos = sum(i["n_visits"] * i["tile"][0] * i["tile"][1] for i in infos)
    checked = sum(i["n_checked"] for i in infos)
    alg = algorithmic_bytes(patched, visit_pos, checked, K, s_beta, s_move)
    ach = alg / max(t_rounds, 1e-12) / 1e9
    return {"bound": "hbm", "kernel": "lgcd_rounds", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": None, "seconds": t_rounds,
            "counts": {"n_patched": patched, "visit_positions": visit_pos, "n_checked": checked}}


def run_serving(args):
    """Serving pattern: Poisson arrivals of multichannel 1-D requests of
    log-uniform length sharing one dictionary, served by continuous batching
    (dicodile_server_*), beside the plain form: the same arrivals solved one
    call at a time in arrival order.  Latency = arrival -> z ready.  Swept over
    offered rates (--rates); at the first rate the HBM admission budget is also
    swept (--budgets).  The request signals come from a pool of distinct
    seeded requests, reused cyclically; every request is solved in full into
    its own output."""
    import threading
    import numpy as np
    import torch
    import paper_1901_09235_amd as dl
    from paper_1901_09235_amd import synth

    t0 = time.perf_counter()
    D_np = synth.serving_dictionary()
    pool = [synth.serving_request(j, D_np) for j in range(args.pool)]
    t_gen = time.perf_counter() - t0
    print(f"# generated {len(pool)} request signals in {t_gen:.1f} s", file=sys.stderr, flush=True)
    D = torch.from_numpy(D_np).to("cuda", dtype=torch.float32).contiguous()
    Xs = [torch.from_numpy(pb.X).to("cuda", dtype=torch.float32).contiguous() for pb in pool]
    lams = [pb.lambda_frac * dl.dicodile_lambda_max(X, D) for pb, X in zip(pool, Xs)]
    L = D.shape[2]
    K = D.shape[0]
    n_warm, n_meas = args.serve_warmup, args.requests
    n = n_warm + n_meas
    which = [i % len(pool) for i in range(n)]
    # one output per in-flight request: a ring deep enough for any backlog here,
    # a multiple of the pool so that slot i % ring always holds signal i % pool
    ring = len(pool) * max(1, 2048 // len(pool))
    zs = [torch.empty((K, Xs[i % len(pool)].shape[1] - L + 1), dtype=torch.float32, device="cuda")
          for i in range(ring)]
    torch.cuda.synchronize()
    max_len = max(X.shape[1] for X in Xs)

    def serve(rate, budget_mib):
        arrivals = synth.serving_arrivals(n, rate_hz=rate)
        sopts = dict(max_len=max_len)
        if budget_mib > 0:
            sopts["hbm_budget_bytes"] = budget_mib << 20
        if args.max_workers:
            sopts["max_workers"] = args.max_workers
        if args.slice:
            sopts["slice_rounds"] = args.slice
        if args.admit:
            sopts["admit_workers"] = args.admit
        srv = dl.Server(D, **sopts)
        results, tickets, sub_at = [None] * n, [None] * n, [0.0] * n
        ready = threading.Semaphore(0)

        def collect():
            for i in range(n):
                ready.acquire()
                results[i] = srv.wait(tickets[i])[1]
        try:
            th = threading.Thread(target=collect, daemon=True)
            th.start()
            start = time.monotonic() + 0.05
            for i in range(n):
                if i >= ring:  # the output slot is reused: its earlier request must be done
                    while results[i - ring] is None:
                        time.sleep(1e-4)
                delay = start + arrivals[i] - time.monotonic()
                if delay > 0:
                    time.sleep(delay)
                sub_at[i] = time.monotonic()
                j = which[i]
                tickets[i] = srv.submit(Xs[j], lams[j], 1e-5 * lams[j], z_out=zs[i % ring])
                ready.release()
            th.join()
            st = srv.stats()
        finally:
            srv.close()
        meas = range(n_warm, n)
        bad = [results[i] for i in meas if results[i]["status"] != "OK"]
        if bad:
            raise SystemExit(f"{len(bad)} served requests did not converge: {bad[0]}")
        lat = [(sub_at[i] - (start + arrivals[i])) + results[i]["t_total_s"] for i in meas]
        done = [sub_at[i] + results[i]["t_total_s"] for i in meas]
        span = max(done) - (start + arrivals[n_warm])
        out = dict(_percentiles(lat), requests_per_s=n_meas / span, offered_rate_hz=rate,
                   budget_mib=budget_mib or "default", max_kkt=max(results[i]["kkt"] for i in meas),
                   queue_p99_ms=_percentiles([results[i]["t_init_s"] for i in meas])["p99_ms"],
                   peak_active=st["peak_active"], peak_workers=st["peak_workers"], launches=st["n_launches"],
                   rounds_busy_frac=st["t_rounds_s"] / max(1e-9, st["t_busy_s"]),
                   roofline=_rounds_roofline([results[i] for i in range(n)], st["t_rounds_s"], K))
        obj = {which[i]: results[i]["objective"] for i in meas}
        print(f"# served {n_meas} requests at {rate:g}/s, budget {budget_mib} MiB: {out['requests_per_s']:.1f} "
              f"req/s, p50 {out['p50_ms']:.1f} ms, p99 {out['p99_ms']:.1f} ms", file=sys.stderr, flush=True)
        return out, obj

    def plain(rate, served_obj):
        arrivals = synth.serving_arrivals(n, rate_hz=rate)
        n_plain = n_meas if args.plain < 0 else min(args.plain, n_meas)
        if n_plain <= 0:
            return None, 0.0
        for X, lam in zip(Xs[:2], lams[:2]):  # warm-up
            dl.dicodile_csc(X, D, lam, 1e-5 * lam)
        torch.cuda.synchronize()
        plat, pdone = [], []
        gap = 0.0
        start = time.monotonic() + 0.05
        for i in range(n_plain):
            delay = start + arrivals[i] - time.monotonic()
            if delay > 0:
                time.sleep(delay)
            j = which[i]
            _, info = dl.dicodile_csc(Xs[j], D, lams[j], 1e-5 * lams[j], z_out=zs[i % ring],
                                      max_rounds=50_000_000, timeout_s=120)
            if info["status"] != "OK":
                raise SystemExit(f"plain solve did not converge: {info}")
            now = time.monotonic()
            plat.append(now - (start + arrivals[i]))
            pdone.append(now)
            if (i + 1) % 500 == 0:
                print(f"# plain form at {rate:g}/s: {i + 1} requests", file=sys.stderr, flush=True)
            if j in served_obj:
                gap = max(gap, abs(info["objective"] - served_obj[j]) / info["objective"])
        pspan = pdone[-1] - (start + arrivals[0])
        out = dict(_percentiles(plat), requests=n_plain, requests_per_s=n_plain / pspan, offered_rate_hz=rate)
        print(f"# plain form at {rate:g}/s: {n_plain} requests in {pspan:.2f} s, p50 {out['p50_ms']:.1f} ms, "
              f"p99 {out['p99_ms']:.1f} ms", file=sys.stderr, flush=True)
        return out, gap

    rates = [float(r) for r in args.rates.split(",")] if args.rates else [args.rate]
    budgets = [int(b) for b in args.budgets.split(",")]
    per_rate = []
    budget_sweep = []
    gap = 0.0
    for ri, rate in enumerate(rates):
        served, served_obj = serve(rate, budgets[0])
        if ri == 0:
            budget_sweep = [served] + [serve(rate, b)[0] for b in budgets[1:]]
        pl, g = plain(rate, served_obj)
        gap = max(gap, g)
        per_rate.append({"offered_rate_hz": rate, "served": served, "plain": pl,
                         "served_over_plain_throughput": served["requests_per_s"] / pl["requests_per_s"] if pl else None})
    head = per_rate[0]
    lens = [Xs[j].shape[1] for j in which]
    out = {
        "metric": "served requests/s with p50/p99 latency (arrival -> z at KKT tol), continuous batching vs plain",
        "value": head["served"]["requests_per_s"], "unit": "requests/s", "n_gpus": 1, "steps": n_meas,
        "warmup": n_warm, "ms_per_step": 1e3 / head["served"]["requests_per_s"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"serving_poisson{rates[0]:g}_P32_K40_L128_T1e4-5e5",
                   "requests": n_meas, "warmup_requests": n_warm, "distinct_signals": len(pool),
                   "offered_rates_hz": rates, "lambda": "0.2 lambda_max each", "tol": "1e-5 lambda each",
                   "mean_T": float(np.mean(lens))},
        "roofline": head["served"]["roofline"],
        "served": head["served"],
        "plain": head["plain"],
        "rates": per_rate,
        "budget_sweep": budget_sweep,
        "max_objective_gap_served_vs_plain": gap,
        "generation_s": t_gen,
    }
    stored = stored_gap("serving_P32_K40_L128_T1e4-5e5")
    if stored is not None:
        out["objective_gap_vs_oracle"] = stored.get("summary")
    print(json.dumps(out), flush=True)


def fft64_bytes(P, T, K, L, KS, s_beta):
    """HBM bytes of one FP64 correlation by FFT, pass by pass, for an image
    (P, T1, T2) and K atoms (L1, L2): transform sizes are the powers of two
    covering T, spectra hold N1 x F2p complex values (F2p = N2/2 + 1 padded to
    16).  Returned per epilogue mode, and the dictionary spectra (once per
    solve)."""
    T1, T2 = T
    N1, N2 = 1 << (T1 - 1).bit_length(), 1 << (T2 - 1).bit_length()
    M2 = N2 // 2
    F2p = (M2 + 1 + 15) // 16 * 16
    sp = 16.0 * N1 * F2p
    H, W = T1 - L[0] + 1, T2 - L[1] + 1
    HW = H * W
    fwd = P * (8.0 * T1 * T2 + sp) + 2 * 2 * P * sp            # rows, two column passes
    prod = (P + K * P) * sp + K * sp                              # products fused with the first inverse pass
    inv = K * sp + K * sp * H / N1 + K * (H * F2p * 16.0 + 8.0 * HW)  # second inverse pass, rows
    ep_g = 8.0 * K * HW                                           # G read
    beta = fwd + prod + inv + ep_g + HW * KS * (s_beta + s_beta)  # + z read, beta written
    kkt = fwd + prod + inv + ep_g + HW * KS * 3 * s_beta          # + z and kept beta read, beta written
    return {"beta": beta, "kkt": kkt, "dict_spectra": K * P * sp}


MFMA_PEAK_TFS = {"f64": 78.6, "bf16": 2500.0, "bf16x3": 2500.0 / 3, "direct": 157.3}


def run_corr_bench(args):
    """The dense contraction G = corr(X, D) (beta initialisation, drift
    correction, KKT check) in each precision on the workloads' shapes: call
    time (HIP events around the call on its stream), algorithmic TFLOP/s
    (2 K P |Theta| per valid position) and the error of each precision
    against the FP64 contraction on the same data."""
    import torch
    import paper_1901_09235_amd as dl
    shapes = {
        "serving_max_P32_T500000_K40_L128": (32, (500000,), 40, (128,)),
        "image_rgb_4096_K25_L32": (3, (4096, 4096), 25, (32, 32)),
        "image_1024_K25_L16": (1, (1024, 1024), 25, (16, 16)),
    }
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1234)
    res = {}
    for name, (P, T, K, L) in shapes.items():
        X = torch.randn((P,) + T, generator=gen, device="cuda", dtype=torch.float32)
        D = torch.randn((K, P) + L, generator=gen, device="cuda", dtype=torch.float32)
        D /= D.flatten(1).norm(dim=1).view((K,) + (1,) * (D.dim() - 1))
        positions = 1
        for t, l in zip(T, L):
            positions *= t - l + 1
        flop = 2.0 * K * P * positions * int(torch.tensor(L).prod())
        out = {}
        ref = None
        for prec in ("f64", "bf16x3", "bf16", "direct", "f64_fft"):
            if prec == "direct" and flop > 2e11:
                continue
            if prec == "f64_fft" and len(T) != 2:
                continue
            G = dl.dicodile_corr(X, D, prec=prec)  # warm-up
            torch.cuda.synchronize()
            reps = 3
            st = torch.cuda.current_stream()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            for _ in range(reps):
                dl.dicodile_corr(X, D, prec=prec, out=G, stream=st.cuda_stream)
            e1.record(st)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            tfs = flop / (ms * 1e-3) / 1e12
            if prec == "f64_fft":
                # by FFT: HBM-bound; the call also builds the dictionary spectra and
                # converts X to FP64 (the epilogue writes beta without z)
                fb = fft64_bytes(P, T, K, L, K, 4)
                byt = fb["beta"] + fb["dict_spectra"] + 12.0 * P * T[0] * T[1]
                rec = {"ms": ms, "equivalent_tflops": tfs, "bytes": byt, "achieved_gbs": byt / (ms * 1e-3) / 1e9,
                       "peak_gbs": HBM_PEAK_GBS, "frac": byt / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
            else:
                rec = {"ms": ms, "tflops": tfs, "peak_tflops": MFMA_PEAK_TFS[prec], "frac": tfs / MFMA_PEAK_TFS[prec]}
            if prec == "f64":
                ref = G.double()
            else:
                rec["max_err_rel_to_max"] = float((G.double() - ref).abs().max() / ref.abs().max())
            out[prec] = rec
            print(f"# {name} {prec}: {ms:.3f} ms, {tfs:.1f} TFLOP/s", file=sys.stderr, flush=True)
            del G
        res[name] = {"gflop": flop / 1e9, "precisions": out}
        del X, D
        torch.cuda.empty_cache()
    # the dense formulation of the dictionary statistics on the RGB workload:
    # phi[k, k', tau] = sum_w Z_k[w] Z_k'[w + tau] is, per lag tau, a K x K
    # product over all valid positions, and there are (2L1-1)(2L2-1) lags.  One
    # such product (contiguous operands: no shift copies, so a lower bound) is
    # timed with the vendor GEMM and scaled to every lag; the library computes
    # phi from the non-zeros instead (dict_stats_ms on the headline line).
    K, H, W, L = 25, 4065, 4065, 32
    lags = (2 * L - 1) ** 2
    dense = {"lags": lags, "positions": H * W, "flop_per_lag": 2.0 * K * K * H * W}
    for name, dt in (("fp32", torch.float32), ("bf16", torch.bfloat16)):
        A = torch.randn((K, H * W), generator=gen, device="cuda", dtype=torch.float32).to(dt)
        B = torch.randn((H * W, K), generator=gen, device="cuda", dtype=torch.float32).to(dt)
        C = A @ B  # warm-up
        torch.cuda.synchronize()
        st = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(5):
            C = A @ B
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 5
        dense[name] = {"gemm_ms": ms, "tflops": dense["flop_per_lag"] / (ms * 1e-3) / 1e12,
                       "projected_phi_ms": ms * lags}
        print(f"# dense phi lag product {name}: {ms:.3f} ms per lag, {ms * lags:.0f} ms for all lags",
              file=sys.stderr, flush=True)
        del A, B, C
        torch.cuda.empty_cache()
    # the library's nnz-driven form on a z of the workload's recipe
    # (Bernoulli(5e-4) x Exp(1) on 25 x 4065^2): its time and its useful flops
    # (2 per non-zero pair within a lag window for phi, 2 P L1 L2 per non-zero
    # for psi), beside the dense form's flops at the dtype peaks
    Z = (torch.rand((K, H, W), generator=gen, device="cuda") < 5e-4).float()
    Z *= -torch.log(torch.rand((K, H, W), generator=gen, device="cuda"))
    X = torch.randn((3, 4096, 4096), generator=gen, device="cuda", dtype=torch.float32)
    nzc = (Z != 0).sum(dim=0).float()
    box = torch.nn.functional.avg_pool2d(nzc[None, None], 2 * L - 1, stride=1, padding=L - 1,
                                         count_include_pad=True)[0, 0] * float((2 * L - 1) ** 2)
    pairs = float((nzc.double() * box.round().double()).sum())
    nnz = int(nzc.sum())
    dl.dicodile_dict_stats(Z, X, (L, L))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        dl.dicodile_dict_stats(Z, X, (L, L))
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / 3 * 1e3
    useful = 2.0 * pairs + 2.0 * nnz * 3 * L * L
    dense_flop = dense["flop_per_lag"] * lags + 2.0 * K * 3 * L * L * H * W
    dense["nnz_form"] = {"nnz": nnz, "pairs_within_window": pairs, "useful_gflop": useful / 1e9, "ms": ms,
                         "useful_tflops": useful / (ms * 1e-3) / 1e12}
    dense["dense_form_tflop"] = dense_flop / 1e12
    dense["dense_floor_ms"] = {k: dense_flop / (MFMA_PEAK_TFS[k] * 1e12) * 1e3 for k in ("bf16", "f64")}
    dense["dense_floor_ms"]["fp32_vector"] = dense_flop / 157.3e12 * 1e3
    for name in ("fp32", "bf16"):
        dense[name]["useful_tflops_projected"] = useful / (dense[name]["projected_phi_ms"] * 1e-3) / 1e12
    print(f"# nnz-driven ztz/ztX: {ms:.2f} ms, {nnz} non-zeros, {pairs:.3g} pairs, "
          f"{useful / (ms * 1e-3) / 1e9:.1f} useful GFLOP/s", file=sys.stderr, flush=True)
    del Z, X
    res["dense_phi_rgb_4096"] = dense
    best = res["serving_max_P32_T500000_K40_L128"]["precisions"]["f64"]
    line = {
        "metric": "dense correlation corr(X, D) throughput on the matrix cores", "value": best["tflops"],
        "unit": "TFLOP/s", "n_gpus": 1, "steps": 3, "warmup": 1, "ms_per_step": best["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "corr_serving_max_P32_T500000_K40_L128"},
        "roofline": {"bound": "mfma", "kernel": "corr_mfma<F64>", "achieved": best["tflops"], "peak": 78.6,
                     "unit": "TFLOP/s", "frac": best["tflops"] / 78.6, "traffic": None},
        "shapes": res,
    }
    print(json.dumps(line), flush=True)


def _solve_record(dl, torch, pb, cap, **opts):
    """One timed solve of a synthetic problem (FP32, lambda and tol from its
    recipe); the library's own clock (t_total_s) covers init, rounds and the
    FP64 check."""
    X = torch.from_numpy(pb.X).to("cuda", dtype=torch.float32).contiguous()
    D = torch.from_numpy(pb.D).to("cuda", dtype=torch.float32).contiguous()
    lam = pb.lambda_frac * dl.dicodile_lambda_max(X, D)
    tol = pb.tol_rel * lam
    try:
        _, info = dl.dicodile_csc(X, D, lam, tol, max_rounds=1 << 30, timeout_s=cap, **opts)
    except dl.DicodileError as e:
        return {"status": str(e).split(":")[0], "opts": {k: v for k, v in opts.items()}}
    return {"status": info["status"], "t_s": info["t_total_s"], "t_rounds_s": info["t_cd_s"],
            "updates": info["n_updates"], "rounds": info["n_rounds"], "sweeps": info["n_sweeps"],
            "softlocked": info["n_softlocked"], "objective": info["objective"], "kkt": info["kkt"],
            "grid": list(info["grid"]), "tile": list(info["tile"])}


def run_ablation(args):
    """Sec. 5's comparisons re-run on synthetic inputs (the paper's own data
    for the image experiments is not available):
      * selection rules with one worker (LGCD, randomized and greedy CD) on the
        paper's 1-D recipe (P=7, K=25, L=250, T = 150 L and 750 L);
      * the soft-lock ablation on 512x512 images with 7x7 workers and with
        workers of about one sub-domain, without the soft-lock test (divergence
        guard on) and with, for K=25 i.i.d. Gaussian atoms 16x16 and for K=4
        smooth (strongly overlapping) atoms 10x10;
      * the line vs grid split of a 512x512 image with K=5 atoms 8x8.
    Every solve is capped at --ablation-cap seconds of wall clock."""
    import torch
    import paper_1901_09235_amd as dl
    from paper_1901_09235_amd import synth
    cap = args.ablation_cap
    _solve_record(dl, torch, synth.paper_signal_1d(T=4000), cap, grid=1)  # warm-up: library set-up
    res = {"rules_1d": {}, "soft_lock": {}, "split": {"line": {}, "grid": {}}}
    for mult in (150, 750):
        pb = synth.paper_signal_1d(T=mult * 250)
        for rule in ("lgcd", "random", "greedy"):
            r = _solve_record(dl, torch, pb, cap, grid=1, strategy=rule, seed=1)
            res["rules_1d"][f"T{mult}L_{rule}"] = r
            print(f"# rules T={mult}L {rule}: {r}", file=sys.stderr, flush=True)
        ref = res["rules_1d"][f"T{mult}L_lgcd"].get("objective")
        for rule in ("random", "greedy"):
            r = res["rules_1d"][f"T{mult}L_{rule}"]
            if ref and "objective" in r:
                r["objective_gap_vs_lgcd"] = (r["objective"] - ref) / abs(ref)
    import numpy as np
    for atoms in ("gaussian", "smooth"):
        if atoms == "smooth":
            Dab = synth.smooth_dictionary(np.random.Generator(np.random.PCG64(8002)), 4, 1, (10, 10))
            pb = synth.make_problem("ablation_softlock_512_K4_L10_smooth", 8000, P=1, T=(512, 512), K=4,
                                    L=(10, 10), rho=0.01, amp="uniform", sigma=0.1, D=Dab)
        else:
            pb = synth.make_problem("ablation_softlock_512_K25_L16_gaussian", 8000, P=1, T=(512, 512), K=25,
                                    L=(16, 16), rho=0.002, amp="uniform", sigma=0.1)
        # 7x7 workers as in the paper, and workers of about one sub-domain each
        fine = (25, 25) if atoms == "smooth" else (31, 31)
        for grid in ((7, 7), fine):
            for name, kw in (("no_soft_lock", dict(no_soft_lock=True, div_guard=1e3)), ("soft_lock", {})):
                r = _solve_record(dl, torch, pb, cap, grid=grid, **kw)
                res["soft_lock"][f"{atoms}_{grid[0]}x{grid[1]}_{name}"] = r
                print(f"# soft-lock ablation, {atoms} atoms, {grid[0]}x{grid[1]} workers, {name}: {r}",
                      file=sys.stderr, flush=True)
    pb = synth.make_problem("ablation_split_512_K5_L8", 8001, P=1, T=(512, 512), K=5, L=(8, 8),
                            rho=0.002, amp="uniform", sigma=0.1)
    for w in (1, 2, 4, 8, 16, 32, 63):
        r = _solve_record(dl, torch, pb, cap, grid=(1, w))
        res["split"]["line"][w] = r
        print(f"# line split W={w}: {r}", file=sys.stderr, flush=True)
    for w in (1, 2, 4, 8, 16, 32):
        r = _solve_record(dl, torch, pb, cap, grid=(w, w))
        res["split"]["grid"][w * w] = r
        print(f"# grid split W={w * w}: {r}", file=sys.stderr, flush=True)
    head = res["rules_1d"]["T750L_lgcd"]
    line = {
        "metric": "time to tolerance of the selection-rule and partition ablations", "value": head.get("t_s"),
        "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": 1e3 * head.get("t_s", float("nan")),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "ablation_rules_T750L_lgcd_1worker", "cap_s": cap},
        "results": res,
    }
    print(json.dumps(line), flush=True)


def stored_gap(workload: str):
    """Objective gap of this workload's GPU result against the FP64 oracle, as
    recorded by the full-size parity test (tests/test_gpu_gap.py) on the
    current round-kernel sources; None when absent or stale."""
    path = os.path.join(PROFILES, f"objective_gap_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_digest") != kernel_source_digest():
        return None
    return rec


def corr_flop(g_positions, K, P, taps):
    """Algorithmic flops of one corr(R, D) over the valid domain: 2 K P |Theta| per position."""
    return 2.0 * K * P * taps * g_positions


def run_solve(args):
    import numpy as np
    import torch
    import paper_1901_09235_amd as dl

    pb = make_workload(args)
    rgb = args.workload == "image_rgb_4096"
    f64 = pb.dtype == "f64"
    tdt = torch.float64 if f64 else torch.float32
    X = torch.from_numpy(pb.X).to("cuda", dtype=tdt).contiguous()
    D = torch.from_numpy(pb.D).to("cuda", dtype=tdt).contiguous()
    lm = dl.dicodile_lambda_max(X, D)
    lam = pb.lambda_frac * lm
    tol = pb.tol_rel if pb.tol_abs else pb.tol_rel * lam
    z = torch.empty((D.shape[0],) + tuple(s - l + 1 for s, l in zip(X.shape[1:], D.shape[2:])),
                    dtype=tdt, device="cuda")
    K, P = D.shape[0], D.shape[1]
    L = tuple(D.shape[2:])
    taps = int(np.prod(L))
    positions = int(np.prod(z.shape[1:]))
    prec = args.precision or ("bf16" if rgb else "auto")
    fix_after = args.fix_after if args.fix_after >= 0 else (4 if rgb and prec == "bf16" else 0)
    opts = dict(max_rounds=50_000_000, timeout_s=120.0, beta_prec=prec)
    if fix_after > 0:
        opts.update(refresh_every=fix_after, refresh_limit=1)
    if args.grid:
        opts["grid"] = tuple(args.grid) if len(args.grid) > 1 else args.grid[0]
    elif args.workload == "image_1024":
        opts["grid"] = (16, 16)  # the workload's configured worker grid
    if args.tile:
        opts["tile"] = tuple(args.tile) if len(args.tile) > 1 else args.tile[0]
    if args.threads:
        opts["threads"] = args.threads
    if args.inner:
        opts["inner"] = args.inner

    copy_gbs = None
    if args.probe_mib > 0:
        n = args.probe_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        sec = dl.dicodile_copy_probe(dst, src, repeats=5)
        copy_gbs = 2 * n * 4 / sec / 1e9
        del src, dst

    def step():
        _, info = dl.dicodile_csc(X, D, lam, tol, z_out=z, **opts)
        t_stats = None
        if rgb:
            s0 = torch.cuda.Event(enable_timing=True)
            s1 = torch.cuda.Event(enable_timing=True)
            st = torch.cuda.current_stream()
            s0.record(st)
            dl.dicodile_dict_stats(z, X, L, stream=st.cuda_stream)
            s1.record(st)
            s1.synchronize()
            t_stats = s0.elapsed_time(s1) * 1e-3
        return info, t_stats

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    infos, stats_t = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        info, ts = step()
        infos.append(info)
        stats_t.append(ts)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for info in infos:
        if info["status"] != "OK":
            raise SystemExit(f"solve did not converge: {info}")

    s_beta = 8 if f64 else 4
    s_move = 16 if f64 else 8
    upd = sum(i["n_updates"] for i in infos)
    t_cd = sum(i["t_cd_s"] for i in infos)
    tile = infos[0]["tile"]
    n_visit_pos = sum(i["n_visits"] for i in infos) * tile[0] * tile[1]
    n_checked = sum(i["n_checked"] for i in infos)
    n_patched = sum(i["n_patched"] for i in infos)
    # positions read per visit: a full sub-domain (ragged edges counted full)
    alg = algorithmic_bytes(n_patched, n_visit_pos, n_checked, K, s_beta, s_move)
    kernels = {
        "lgcd_rounds": {"bound": "hbm", "kernel": "lgcd_rounds", "achieved": alg / t_cd / 1e9,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": alg / t_cd / 1e9 / HBM_PEAK_GBS,
                        "traffic": None, "seconds": t_cd / args.steps, "launches": infos[-1]["n_passes"],
                        "bytes_per_step": alg / args.steps,
                        "counts_per_step": {"n_patched": n_patched / args.steps,
                                            "n_visits": sum(i["n_visits"] for i in infos) / args.steps,
                                            "visit_positions": n_visit_pos / args.steps,
                                            "n_checked": n_checked / args.steps},
                        "bytes_formula": "n_patched*K*3*s_beta + (visit_positions + n_checked)*s_move"},
    }
    fl = corr_flop(positions, K, P, taps)
    init_prec = {0: "auto", 1: "f64", 2: "bf16", 3: "bf16x3", 4: "direct", 5: "f64_fft"}.get(infos[-1]["init_prec"], "?")
    t_init = sum(i["t_init_corr_s"] for i in infos)
    if t_init > 0:
        peak = MFMA_PEAK_TFS.get(init_prec, 157.3)
        ach = fl * args.steps / t_init / 1e12
        kernels[f"corr_mfma_{init_prec}_init"] = {
            "bound": "mfma", "kernel": f"corr_mfma<{init_prec}> (beta initialisation)", "achieved": ach,
            "peak": peak, "unit": "TFLOP/s", "frac": ach / peak, "traffic": None,
            "seconds": t_init / args.steps, "launches": 1, "flop_per_launch": fl}
    t64 = sum(i["t_corr64_s"] for i in infos)
    n64 = sum(i["n_corr64"] for i in infos)
    n_fft = sum(i["n_fft64"] for i in infos) - sum(1 for i in infos if i["init_prec"] == 5)
    if t64 > 0 and n_fft > 0:
        # FP64 contractions by FFT: HBM bytes of their passes as designed (the
        # drift correction writes beta, the check reads the kept beta and
        # rewrites it), plus the dictionary spectra once per solve
        KS = K if f64 else (K + 3) // 4 * 4
        fb = fft64_bytes(P, tuple(X.shape[1:]), K, L, KS, s_beta)
        byt = (fb["beta"] + fb["kkt"] * (n64 / args.steps - 1) + fb["dict_spectra"]) * args.steps
        kernels["corr_fft64"] = {
            "bound": "hbm", "kernel": "FP64 correlation by FFT (fft_rows_r2c, fft_cols, fft_product, "
                                      "fft_rows_c2r, fft_epilogue)",
            "achieved": byt / t64 / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": byt / t64 / 1e9 / HBM_PEAK_GBS, "traffic": None, "seconds": t64 / args.steps,
            "launches": n64 / args.steps, "bytes_per_launch": {k: v for k, v in fb.items()},
            "bytes_formula": "passes of dcdl_fft.h: spectra 16 N1 F2p bytes each (see DESIGN.md)"}
    elif t64 > 0:
        ach = fl * n64 / t64 / 1e12
        kernels["corr_mfma_f64"] = {
            "bound": "mfma", "kernel": "corr_mfma<f64> (drift correction and KKT check)", "achieved": ach,
            "peak": 78.6, "unit": "TFLOP/s", "frac": ach / 78.6, "traffic": None,
            "seconds": t64 / args.steps, "launches": n64 / args.steps, "flop_per_launch": fl,
            "mfma_row_fill": K / (16.0 * ((K + 15) // 16))}
    t_inc = sum(i["t_check_inc_s"] for i in infos)
    n_inc = sum(i["n_check_inc"] for i in infos)
    if t_inc > 0:
        # per changed coordinate: K (2L1-1)(2L2-1) FP64 update-table entries read
        # and as many FMAs (the changed count comes from the last check of each solve)
        U = int(np.prod([2 * l - 1 for l in L]))
        byt = sum(i["n_changed"] for i in infos) * K * U * 8.0
        kernels["check_inc"] = {
            "bound": "hbm", "kernel": "g_update_kkt (incremental FP64 check)", "achieved": byt / t_inc / 1e9,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": byt / t_inc / 1e9 / HBM_PEAK_GBS, "traffic": None,
            "seconds": t_inc / args.steps, "launches": n_inc / args.steps,
            "changed_coordinates": infos[-1]["n_changed"]}
    dominant = max(kernels, key=lambda k: kernels[k]["seconds"])
    tr = stored_traffic(pb.name, list(infos[-1]["grid"]), list(tile))
    if tr is not None and tr.get("fix_after") == fix_after and tr.get("beta_init") == init_prec:
        # HBM bytes of the round kernel's launches in one step, as the algorithmic
        # bytes_per_step are counted
        kernels["lgcd_rounds"]["traffic"] = tr["bytes_per_step"]
        kernels["lgcd_rounds"]["traffic_source"] = tr["source"]
    last = infos[-1]
    t_solve = sum(i["t_total_s"] for i in infos) / args.steps
    out = {
        "metric": "CSC time-to-KKT-tol & coord updates/s",
        "value": upd / dt,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if f64 else "f32",
        "data": "synthetic",
        "config": {"workload": pb.name, "shape": list(pb.X.shape), "atoms": list(pb.D.shape),
                   "lambda": "%.1f lambda_max" % pb.lambda_frac, "tol": tol, "grid": list(last["grid"]),
                   "tile": list(last["tile"]), "beta_init": init_prec,
                   "drift_fix_after_sweeps": fix_after or None,
                   "step": "solve + dict stats" if rgb else "solve",
                   "parallelism": "1 GPU, workgroup grid"},
        "time_to_kkt_tol_ms": t_solve * 1e3,
        "updates_per_step": upd / args.steps,
        "kkt": last["kkt"],
        "objective": last["objective"],
        "beta_drift_at_first_check": last["beta_drift"],
        "nonzeros": last["n_nonzero"],
        "rounds": last["n_rounds"],
        "passes": last["n_passes"],
        "softlock_rejection": last["n_softlocked"] / max(1, last["n_candidates"]),
        "phase_ms": {"init": last["t_init_s"] * 1e3, "rounds": last["t_cd_s"] * 1e3,
                     "check_and_fix": last["t_check_s"] * 1e3},
        "roofline": dict(kernels[dominant], name=dominant),
        "roofline_kernels": kernels,
        "hbm_copy_gbs": copy_gbs,
        "worker_phase_us_per_round": {
            k: last[f"t_worker_{k}_s"] / max(1, last["n_rounds"]) * 1e6
            for k in ("wait", "select", "collect", "apply")},
    }
    if rgb:
        out["dict_stats_ms"] = float(np.mean(stats_t)) * 1e3
        out["dict_stats_shapes"] = {"ztz": [K, K] + [2 * l - 1 for l in L], "ztX": [K, P] + list(L)}
    gap = stored_gap(pb.name)
    if gap is not None:
        out["objective_gap_vs_oracle"] = gap.get("summary")
    if not args.no_variants:
        variants = {}
        if rgb:
            # other initialisations, and the configured one with its FP64
            # contractions on the matrix cores instead of by FFT
            for vp, fa, fm in (("bf16x3", 0, "auto"), ("bf16", 0, "auto"), ("f64_fft", 0, "auto"),
                               (prec, fix_after, "mfma")):
                if vp == prec and fa == fix_after and fm == "auto":
                    continue
                vo = dict(opts, beta_prec=vp, fp64_method=fm)
                vo.pop("refresh_every", None)
                vo.pop("refresh_limit", None)
                if fa > 0:
                    vo.update(refresh_every=fa, refresh_limit=1)
                _, iv = dl.dicodile_csc(X, D, lam, tol, z_out=z, **vo)
                variants[f"init_{vp}_fix{fa}" + ("_fp64_mfma" if fm == "mfma" else "")] = {
                    "status": iv["status"], "time_to_kkt_tol_ms": iv["t_total_s"] * 1e3,
                    "rounds": iv["n_rounds"], "passes": iv["n_passes"], "kkt": iv["kkt"],
                    "objective_rel_diff": (iv["objective"] - last["objective"]) / abs(last["objective"]),
                    "t_init_corr_ms": iv["t_init_corr_s"] * 1e3, "t_corr64_ms": iv["t_corr64_s"] * 1e3,
                    "n_corr64": iv["n_corr64"], "n_fft64": iv["n_fft64"],
                    "beta_drift_at_first_check": iv["beta_drift"]}
        elif args.workload == "image_1024" and not args.grid:
            # the library's own worker grid beside the configured 16 x 16 one
            vo = dict(opts)
            vo.pop("grid")
            _, iv = dl.dicodile_csc(X, D, lam, tol, z_out=z, **vo)
            variants["library_grid"] = {"status": iv["status"], "time_to_kkt_tol_ms": iv["t_total_s"] * 1e3,
                                        "grid": list(iv["grid"]), "tile": list(iv["tile"]),
                                        "rounds": iv["n_rounds"], "kkt": iv["kkt"],
                                        "rounds_ms": iv["t_cd_s"] * 1e3}
        out["variants"] = variants
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported by this build "
              "(each box has one MI355X and the solver has no multi-GPU path).", file=sys.stderr)
        sys.exit(2)
    if args.workload == "corr":
        return run_corr_bench(args)
    if args.workload == "ablation":
        return run_ablation(args)
    if args.workload == "serving":
        return run_serving(args)
    if args.workload == "batch_images":
        return run_batch(args)
    # the oracle's baseline runs first, pinned to one core, before any GPU call
    cpu = None if args.no_cpu_baseline else cpu_baseline(args)
    if cpu is not None:
        print(f"# cpu baseline: {cpu}", file=sys.stderr, flush=True)
    out = run_solve(args)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
