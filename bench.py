#!/usr/bin/env python3
"""Benchmark: energy + adjoint gradient evaluations per second of the p=4 QAOA
estimator on the 26-vertex random tree (Pruefer sequence, seed 3), H_red observable,
complex64 amplitudes, one MI355X.

One step = one energy + adjoint-gradient evaluation (the whole hot path: phase tables,
every forward and backward statevector sweep, the FP64 reductions) at one of the 32
seeded parameter points, through the resident evaluator (aaq_resident_execute: device
parameters and outputs, forward-state checkpoints); ``--api host`` times the synchronous
aaq_energy_grad_checkpointed call instead, ``--grad-mode uncompute`` the two-buffer mode.  Prints ONE JSON line.  Alongside the headline number it reports
the roofline of the dominant kernel class (HIP start and end events carried in the dispatch
of each of its launches in the timed region, on the stream the kernel runs on; the
warm-up times every class to find it), the FP64 CPU oracle timed on the host cores, and H_red vs H_C
in the three aggregation modes.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "<H>+adjoint-grad evals/s (n=26,p=4), % HBM roofline, H_red vs H_C"
PEAK_HBM_GBS = 8000.0  # MI355X HBM3E
KERNEL_SOURCES = ["paper_2410_22247_amd/csrc/aaq_engine.h", "paper_2410_22247_amd/csrc/aaq_kernels.hip",
                  "paper_2410_22247_amd/csrc/aaq_internal.h"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic.json")


def load_traffic(kclass: str, path: str = TRAFFIC_JSON):
    """HBM bytes per launch from the committed rocprofv3 counter runs, or None when
    they were taken on other kernel sources."""
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_hash():
        return None
    k = t.get("kernels", {}).get(kclass)
    return None if k is None else k.get("hbm_bytes_per_launch")


def kernel_class(name: str):
    """Timing class of a kernel symbol (the classes aaq_timing_read reports)."""
    for pre, two, one in (("aaq::k_sweep<", "sweep_2state", "sweep_1state"),
                          ("aaq::k_bsweep<", "sweep_2state", "sweep_1state")):
        if pre in name:
            ns = name.split(pre, 1)[1].split(",")[1].strip()
            return two if ns == "2" else one
    if "aaq::k_bsweep_k<" in name:
        # <R, route, tile bits, shape>: two states when the shape loads or creates lambda
        # (bits 2 and 5 of the shape word)
        kind = int(name.split("aaq::k_bsweep_k<", 1)[1].split(">", 1)[0].split(",")[3].strip().rstrip("u"))
        return "sweep_2state" if kind & ((1 << 2) | (1 << 5)) else "sweep_1state"
    for key, cls in (("k_units", "units"), ("k_reduce", "reduce"), ("k_bsweep_out", "reduce"),
                     ("k_plan_tables", "tables"), ("k_tables", "tables"), ("k_zz_pass", "zz_pass")):
        if key in name:
            return cls
    return None


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def write_traffic(fetch_csv: str, write_csv: str, copy_bytes: int = 512 << 20, out_path: str = TRAFFIC_JSON):
    """profiles/traffic.json from two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE, KiB per
    dispatch) of `bench.py --copy-calibration`: each counter is scaled by the ratio of the
    algorithmic bytes of the 512 MiB calibration copy to what the counter reports for it."""
    import csv

    out = {"kernel_sha": kernel_hash(), "copy_bytes": copy_bytes, "kernels": {}, "factors": {}}
    per = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = list(csv.DictReader(open(path)))
        copies = [float(r["Counter_Value"]) * 1024 for r in rows if "copyBuffer" in r["Kernel_Name"]]
        ref = max(copies)
        factor = copy_bytes / ref
        out["factors"][counter] = {"copy_counter_bytes": ref, "factor": factor}
        for r in rows:
            c = kernel_class(r["Kernel_Name"])
            if c is None:
                continue
            per.setdefault(c, {}).setdefault(counter, []).append(float(r["Counter_Value"]) * 1024 * factor)
    for c, d in per.items():
        if "FETCH_SIZE" in d and "WRITE_SIZE" in d:
            f = sum(d["FETCH_SIZE"]) / len(d["FETCH_SIZE"])
            w = sum(d["WRITE_SIZE"]) / len(d["WRITE_SIZE"])
            out["kernels"][c] = {"launches": len(d["FETCH_SIZE"]), "fetch_bytes_per_launch": f,
                                 "write_bytes_per_launch": w, "hbm_bytes_per_launch": f + w}
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--cpu-runs", type=int, default=5, help="timed oracle evaluations (median reported)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run 3 plain 512 MiB device copies (reference for HBM byte counters)")
    ap.add_argument("--workload", default="c3", choices=["c3", "c1", "c2", "c4", "c5a", "c5b", "lc", "sample", "weighted", "adam"],
                    help="c3 (default): the n=26 p=4 energy+gradient headline; the others print their own line")
    ap.add_argument("--grad-mode", default="checkpoint", choices=["checkpoint", "uncompute"],
                    help="checkpoint: forward states kept in HBM, backward sweeps read them (default); "
                         "uncompute: backward sweeps recompute psi in place (two state buffers)")
    ap.add_argument("--api", default="resident", choices=["resident", "host"],
                    help="resident (default): parameters and outputs stay in device memory and evaluations queue "
                         "back to back (aaq_resident_*); host: one synchronous aaq_energy_grad call per step with "
                         "host parameters and host results")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="no GPU work: turn two rocprofv3 --pmc counter_collection.csv files into profiles/traffic.json")
    args = ap.parse_args()
    if args.write_traffic:
        write_traffic(*args.write_traffic)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2410_22247_amd as A
    from workloads.configs import config3

    if args.workload != "c3":
        import bench_configs

        print(json.dumps(bench_configs.run(args.workload, args)), flush=True)
        return

    if args.copy_calibration:
        src = torch.empty(64 << 20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    wp, p, gams, bets = config3(32)
    pr = A.Problem.from_workload(wp)
    torch.cuda.set_device(0)
    ckpt = args.grad_mode == "checkpoint"
    est = A.Estimator(pr, p, A.AAQ_OBS_HRED, A.AAQ_PREC_C64, grad=True, checkpoint=ckpt)
    stream = torch.cuda.current_stream()
    res = None
    if args.api == "resident":
        res = A.Resident(pr, p, A.AAQ_OBS_HRED, with_grad=True, checkpoint=ckpt)
        dparams = torch.from_numpy(np.concatenate([gams, bets], 1)).to("cuda")  # [32][2p], resident before timing
        dout = torch.zeros(max(args.steps, args.warmup, 1), 2 + 2 * p, dtype=torch.float64, device="cuda")

    def step(k):
        if res is not None:
            res.execute(dparams[k % 32], dout[k])
        else:
            est.energy_grad(gams[k % 32], bets[k % 32])

    # warm-up with every kernel class timed: the class breakdown, and the dominant class
    # (by summed event time) whose launches alone carry events in the timed region
    A.aaq_timing_classes(None)
    A.aaq_timing_read(reset=True)
    A.aaq_timing_enable(True)
    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    A.aaq_timing_enable(False)
    wtiming = A.aaq_timing_read(reset=True)
    dom = max(wtiming, key=lambda c: wtiming[c]["total_ms"]) if wtiming else None

    # ---------------------------------------------------------------- timed region
    A.aaq_timing_classes([dom] if dom else None)
    A.aaq_timing_read(reset=True)
    A.aaq_timing_enable(True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for k in range(args.steps):
        step(k)
    ev1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    A.aaq_timing_enable(False)
    timing = A.aaq_timing_read(reset=True)
    A.aaq_timing_classes(None)
    wall = t1 - t0
    ms_per_step = 1e3 * wall / args.steps
    value = args.steps / wall

    # the stored state: half of it with the spin-flip symmetry (n <= 29 in complex64)
    half = A.aaq_get_half_state() and (8 << wp.n) <= (1 << 32)
    state_bytes = 8 << (wp.n - (1 if half else 0))

    # the dominant class's launches in the timed region (every class there without a warm-up)
    if dom is None:
        dom = max(timing, key=lambda c: timing[c]["total_ms"])
    d = timing[dom]
    per_launch_bytes = d["bytes"] / d["launches"]
    avg_ms = d["total_ms"] / d["launches"]
    achieved = per_launch_bytes / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    traffic = load_traffic(dom)
    # per-evaluation class breakdown from the warm-up (the timed region's own without one)
    brk, brk_steps = (wtiming, args.warmup) if wtiming else (timing, args.steps)
    sweep_bytes = sum(brk[c]["bytes"] for c in brk)
    sweep_ms = sum(brk[c]["total_ms"] for c in ("sweep_1state", "sweep_2state") if c in brk)

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {
            "workload": "random tree n=26 (Pruefer, seed 3), p=4, H_red (20 orbit terms), energy + adjoint gradient, "
                        "complex64, 32 seeded (gamma, beta) points cycled",
            "n": 26, "p": 4, "observable": "H_red", "edges": int(wp.m), "orbits": int(wp.orbits.count),
            "tile_sets": A.aaq_num_sets(26),
            "tile_bits": A.aaq_get_tile_bits(26, A.AAQ_PREC_C64, True),
            "gradient_mode": args.grad_mode,
            "state": ("half: amplitudes with bit n-1 = 0 stored and swept (spin-flip symmetry psi(~z) = psi(z)), "
                      "sums doubled" if half else "full"),
            "api": ("resident: device parameters and outputs, evaluations queued without host synchronisation"
                    if res is not None else "host: synchronous call per evaluation"),
        },
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "achieved": round(achieved, 1),
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4),
            "traffic": traffic,
            "bytes_per_launch": per_launch_bytes,
            "avg_launch_ms": round(avg_ms, 5),
            "launches": d["launches"],
        },
        # every class over the warm-up evaluations (only the dominant class carries events
        # in the timed region)
        "kernel_timing": {"steps": brk_steps, "timed_region": brk is timing,
                          **{c: {"launches": v["launches"], "ms": round(v["total_ms"], 3),
                                 "GB/s": round(v["bytes"] / (v["total_ms"] * 1e-3) / 1e9, 1) if v["bytes"] else None}
                             for c, v in brk.items()}},
        # the stricter per-evaluation figure: the method's lower bound on state traffic for
        # energy + gradient (6 p S: one read and one write of psi per layer forward, psi and
        # lambda per layer backward; S = the stored state) over the whole evaluation time
        "eval_lower_bound": {"bytes": 6 * p * state_bytes,
                             "GB/s": round(6 * p * state_bytes / (ms_per_step * 1e-3) / 1e9, 1),
                             "frac": round(6 * p * state_bytes / (ms_per_step * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)},
        "sweep_bytes_per_eval": sweep_bytes / brk_steps,
        "sweep_GBps_per_eval": round(sweep_bytes / (sweep_ms * 1e-3) / 1e9, 1) if sweep_ms else None,
        "event_ms_per_step": round(ev0.elapsed_time(ev1) / args.steps, 4),
    }

    # ---------------------------------------------------------------- H_red vs H_C
    if not args.no_extras:
        ext = {}

        def rate(fn, reps=10, blocks=5):
            """Calls per second: the median over `blocks` timed blocks of `reps` calls, after
            one untimed call."""
            fn()
            torch.cuda.synchronize()
            rates = []
            for _ in range(blocks):
                t = time.perf_counter()
                for _ in range(reps):
                    fn()
                torch.cuda.synchronize()
                rates.append(reps / (time.perf_counter() - t))
            return float(np.median(rates))

        g0, b0 = gams[0], bets[0]
        ests = {agg: A.Estimator(pr, p, A.AAQ_OBS_HRED, A.AAQ_PREC_C64, grad=False, agg=agg)
                for agg in (A.AAQ_AGG_FUSED, A.AAQ_AGG_PER_TERM, A.AAQ_AGG_PASS_PER_TERM)}
        names = {A.AAQ_AGG_FUSED: "fused", A.AAQ_AGG_PER_TERM: "per_term", A.AAQ_AGG_PASS_PER_TERM: "pass_per_term"}
        for agg, es in ests.items():
            r_red = rate(lambda: es.energy(g0, b0, obs=A.AAQ_OBS_HRED))
            r_hc = rate(lambda: es.energy(g0, b0, obs=A.AAQ_OBS_HC))
            ext[f"energy_{names[agg]}"] = {"H_red_evals_s": round(r_red, 2), "H_C_evals_s": round(r_hc, 2),
                                           "speedup": round(r_red / r_hc, 3)}
        del ests
        r_red = rate(lambda: est.energy_grad(g0, b0, obs=A.AAQ_OBS_HRED))
        r_hc = rate(lambda: est.energy_grad(g0, b0, obs=A.AAQ_OBS_HC))
        ext["energy_grad_fused"] = {"H_red_evals_s": round(r_red, 2), "H_C_evals_s": round(r_hc, 2),
                                    "speedup": round(r_red / r_hc, 3)}
        ext["orbit_ratio_E_over_OE"] = round(wp.m / wp.orbits.count, 3)
        out["hred_vs_hc"] = ext
        if res is not None:
            # the same evaluations through the synchronous host API: rate and largest difference
            k_chk = min(args.steps, 4)
            got = dout[:k_chk].cpu().numpy()
            diff = 0.0
            for k in range(k_chk):
                e, dg, db, nrm = est.energy_grad(gams[k % 32], bets[k % 32])
                want = np.concatenate([[e, nrm], dg, db])
                diff = max(diff, float(np.max(np.abs(got[k] - want) / np.maximum(np.abs(want), 1e-300))))
            out["host_api"] = {"evals_s": round(rate(lambda: est.energy_grad(g0, b0)), 2),
                               "max_rel_diff_vs_resident": diff}
            # the resident evaluations without the per-launch timing events of the timed region
            out["resident_untimed_evals_s"] = round(rate(lambda: res.execute(dparams[0], dout[0])), 2)
        if half:
            # the same evaluation with every amplitude stored and swept (host API both ways)
            flat = lambda r: np.concatenate([[r[0]], r[1], r[2]])
            want = flat(est.energy_grad(g0, b0))
            r_half = rate(lambda: est.energy_grad(g0, b0))
            A.aaq_set_half_state(0)
            try:
                est_full = A.Estimator(pr, p, A.AAQ_OBS_HRED, A.AAQ_PREC_C64, grad=True, checkpoint=ckpt)
                got = flat(est_full.energy_grad(g0, b0))
                r_full = rate(lambda: est_full.energy_grad(g0, b0))
                del est_full
            finally:
                A.aaq_set_half_state(1)
            out["full_state"] = {"evals_s": round(r_full, 2), "half_state_evals_s": round(r_half, 2),
                                 "speedup": round(r_half / r_full, 3),
                                 "max_rel_diff_vs_half": float(np.max(np.abs(got - want)) / np.max(np.abs(want)))}

    # ---------------------------------------------------------------- CPU oracle baseline
    if not args.no_cpu_baseline:
        import oracle as O

        terms = wp.terms(1)
        runs = max(1, args.cpu_runs)
        O.energy_grad(wp.n, wp.edges(), terms, gams[0], bets[0])  # warm-up (page-in, thread start)
        ts = []
        for k in range(runs):
            t = time.perf_counter()
            O.energy_grad(wp.n, wp.edges(), terms, gams[(k + 1) % 32], bets[(k + 1) % 32])
            ts.append(time.perf_counter() - t)
        med = float(np.median(ts))
        out["cpu_baseline"] = {
            "value": round(1.0 / med, 4),
            "unit": "evals/s",
            "cores": O.num_threads(),
            "kind": "oracle",
            "sample": f"median of {runs} timed full-state FP64 energy + adjoint-gradient evaluations of the same "
                      f"workload (n=26, p=4, H_red) at points 2..{runs + 1} of the 32, after one untimed evaluation; "
                      f"{sum(ts):.1f} s timed",
            "runs": runs,
            "median_s": round(med, 3),
            "min_s": round(min(ts), 3),
            "max_s": round(max(ts), 3),
            "threads": O.num_threads(),
            "affinity_cpus": len(os.sched_getaffinity(0)),
            "cpu_model": cpu_model(),
        }
        out["gpu_over_cpu"] = round(value * med, 1)

    out["kernel_sha"] = kernel_hash()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
