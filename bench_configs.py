"""Secondary benchmark workloads (bench.py --workload ...), each printing one JSON line.

c1   15-vertex binary tree, p=1, 16x16 (gamma, beta) grid, complex128, both observables,
     one batched plan per observable; parity against the p=1 closed form.
c2   K_16 p=1, star n=20 p=2, the networkx 3-regular graph n=22 (seed 7) p=3; 256 seeded
     points each, both observables, complex64, batched plans against one call per point;
     parity at every point against the Dicke / hub x Dicke subspace formulas (K_16, star)
     and the stored full-state FP64 oracle energies (3-regular).
c4   512 mixed graphs (trees, stars, K_n, 3-regular; n = 8..18), p=2, energy + adjoint
     gradient per graph in one HIP-graph replay of a plan built with the autotuner's
     options vs a loop of single calls; parity of all 512 against the stored FP64 oracle.
c5a  random tree n=34, p=1, complex64 forward energy (2^34 amplitudes, 128 GiB) for
     H_red and H_C; parity against the p=1 closed form.
c5b  random tree n=33, p=2, energy + adjoint gradient (two 64 GiB states); parity
     against the light-cone FP64 adjoint.
lc   light-cone evaluation (each orbit representative's <ZZ> on its distance-p cone, one
     batched plan per instance) of the n=26 p=4, n=34 p=1 and n=33 p=2 trees: energy +
     gradient evals/s for H_red and H_C against the full-state sweeps, parity against the
     light-cone FP64 adjoint.
sample  forward pass keeping the state + inverse-CDF sampling at the n=26 p=4 and n=33
     p=2 tree sizes (2^10 and 2^20 shots); sampled approximation ratios.
weighted  the n=26 p=4 tree with integer edge weights 1..4 (seeded): energy + gradient
     (checkpoints) through the run-time sweep path, against the same tree unweighted,
     and the weighted light-cone evaluation; parity against the weighted light-cone
     FP64 adjoint.
adam  the n=26 p=4 tree: 200 Adam steps (lr 0.01) maximising <H_red> from the first seeded
     point, device-resident (parameters, optimizer and outputs on the GPU) and through the
     synchronous host API; <H_C> and the expectation ratio at the end.
"""
import math
import time

import numpy as np
import torch

import paper_2410_22247_amd as A
from workloads import configs as C


def _timed(fn, reps, blocks=5):
    """Seconds per call: the median over `blocks` timed blocks of `reps` calls, after one
    untimed call."""
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(blocks):
        t = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t) / reps)
    return float(np.median(ts))


def _golden(name):
    import json
    import os

    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden", name)) as f:
        return json.load(f)


def _oracle_rate(fn, count, runs=5, threads=0):
    """Median over `runs` timed runs (after one warm-up call) of `count` oracle
    evaluations fn(i), as evaluations per second; threads > 0 pins the oracle's thread
    count for the measurement.  Returns (rate, threads used)."""
    import oracle as O

    full = O.num_threads()
    if threads:
        O.set_num_threads(threads)
    try:
        fn(0)
        ts = []
        for _ in range(runs):
            t = time.perf_counter()
            for i in range(count):
                fn(i)
            ts.append(time.perf_counter() - t)
        return count / float(np.median(ts)), O.num_threads()
    finally:
        O.set_num_threads(full)


def _plan_rate(units, p, obs, grad, gam, bet, prec=A.AAQ_PREC_C64, reps=10, **opts):
    plan = A.Plan(units, p, obs, with_grad=grad, prec=prec, **opts)
    plan.params.copy_(torch.from_numpy(np.concatenate([gam, bet], 1)))
    dt = _timed(plan.execute, reps)
    out = plan.execute().cpu().numpy()
    plan.close()
    return len(units) / dt, out


def c1(args):
    wp, p, gam, bet = C.config1()
    pr = A.Problem.from_workload(wp)
    g, b = gam[:, 0], bet[:, 0]
    cf = 7 + 0.25 * np.sin(4 * b) * np.sin(g) * (8 + 2 * np.cos(g) + 18 * np.cos(g) ** 2)
    res = {}
    for name, obs in (("H_C", A.AAQ_OBS_HC), ("H_red", A.AAQ_OBS_HRED)):
        rate, out = _plan_rate([pr] * 256, 1, obs, False, gam, bet, prec=A.AAQ_PREC_C128)
        err = np.abs(out[:, 0] - cf)
        res[name] = {"evals_s": round(rate, 1), "max_abs_err_vs_closed_form": float(err.max()),
                     "max_abs_err_interior": float(err.reshape(16, 16)[1:15, 1:15].max())}
        res[name + "_energies"] = out[:, 0]
    diff = float(np.max(np.abs(res["H_C_energies"] - res["H_red_energies"])))
    del res["H_C_energies"], res["H_red_energies"]
    import oracle as O

    terms = wp.terms(A.AAQ_OBS_HRED)
    ev = lambda i: O.energy(wp.n, wp.edges(), terms, gam[i], bet[i])  # noqa: E731
    r_all, t_all = _oracle_rate(ev, 256)
    r_one, _ = _oracle_rate(ev, 256, threads=1)
    return {"workload": "c1: binary tree n=15 p=1, 256-point grid, complex128", "unit": "evals/s", "results": res,
            "max_abs_HC_minus_Hred": diff,
            "cpu_oracle": {"evals_s": round(r_all, 1), "threads": t_all, "evals_s_1_thread": round(r_one, 1),
                           "kind": "FP64 full-state oracle, H_red energy, all 256 points, median of 5 runs"}}


AGG_NAMES = {A.AAQ_AGG_FUSED: "fused", A.AAQ_AGG_PER_TERM: "per_term", A.AAQ_AGG_PASS_PER_TERM: "pass_per_term"}


def _agg_modes(pr, p, g, b, reps, blocks, ref_of=None):
    """Energy rates of H_red and H_C in the three aggregation modes (one Estimator per mode,
    freed before the next: at n = 34 each holds a 128 GiB state buffer); with `ref_of`, the
    relative error of each mode's energy against ref_of(obs)."""
    out = {}
    for agg, name in AGG_NAMES.items():
        est = A.Estimator(pr, p, A.AAQ_OBS_HRED, A.AAQ_PREC_C64, grad=False, agg=agg)
        m = {}
        for oname, obs in (("H_red", A.AAQ_OBS_HRED), ("H_C", A.AAQ_OBS_HC)):
            dt = _timed(lambda: est.energy(g, b, obs=obs, agg=agg), reps, blocks=blocks)
            m[f"{oname}_evals_s"] = round(1.0 / dt, 3)
            if ref_of is not None:
                e = est.energy(g, b, obs=obs, agg=agg)[0]
                m[f"{oname}_rel_err"] = abs(e - ref_of(obs)) / abs(ref_of(obs))
        m["speedup"] = round(m["H_red_evals_s"] / m["H_C_evals_s"], 3)
        out[name] = m
        del est
        torch.cuda.empty_cache()
    return out


def c2(args):
    from oracle import reduced as R
    import oracle as O

    res = {}
    for name, wp, p, gam, bet in C.config2():
        pr = A.Problem.from_workload(wp)
        r = {}
        for oname, obs in (("H_C", A.AAQ_OBS_HC), ("H_red", A.AAQ_OBS_HRED)):
            if name == "K16":
                ref = np.array([R.complete_graph_energy(16, gam[i], bet[i]) for i in range(256)])
            elif name == "star20":
                ref = np.array([R.star_energy(19, gam[i], bet[i]) for i in range(256)])
            else:  # the stored full-state FP64 oracle energies of the frozen networkx graph
                ref = np.asarray(_golden("random_regular_3_22_seed7.json")["energy_hc" if obs == 0 else "energy_hred"])
            rate, out = _plan_rate([pr] * 256, p, obs, False, gam, bet)
            est = A.Estimator(pr, p, obs, A.AAQ_PREC_C64, grad=False)

            def plain():
                for i in range(256):
                    est.energy(gam[i], bet[i])

            dt_plain = _timed(plain, 1, blocks=3)
            single = np.array([est.energy(gam[i], bet[i])[0] for i in range(256)])
            del est
            r[oname] = {"batched_evals_s": round(rate, 1), "plain_evals_s": round(256 / dt_plain, 1),
                        "batched_over_plain": round(rate * dt_plain / 256, 2),
                        "max_rel_err_batched": float(np.max(np.abs(out[:, 0] - ref) / np.abs(ref))),
                        "max_rel_err_plain": float(np.max(np.abs(single - ref) / np.abs(ref)))}
        r["speedup_Hred_over_HC_batched"] = round(r["H_red"]["batched_evals_s"] / r["H_C"]["batched_evals_s"], 3)
        r["aggregation_modes_single_calls"] = _agg_modes(pr, p, gam[0], bet[0], 20, 5)
        r["orbit_ratio_E_over_OE"] = round(wp.m / wp.orbits.count, 3)
        terms = wp.terms(A.AAQ_OBS_HRED)
        cnt = {"K16": 64, "star20": 8}.get(name, 2)
        rate_o, thr = _oracle_rate(lambda i: O.energy(wp.n, wp.edges(), terms, gam[i], bet[i]), cnt)
        r["cpu_oracle"] = {"evals_s": round(rate_o, 2), "threads": thr,
                           "kind": f"FP64 full-state oracle, H_red energy, first {cnt} points, median of 5 runs"}
        res[name] = r
    return {"workload": "c2: K16 p=1, star20 p=2, networkx 3-regular n=22 (seed 7) p=3; 256 points each, "
                        "complex64; batched plans (graph replay) against one call per point; errors over all "
                        "256 points", "unit": "evals/s", "results": res}


def c4(args):
    import oracle as O

    probs, p, gam, bet = C.config4()
    prs = [A.Problem.from_workload(w) for w in probs]
    prm = np.concatenate([gam, bet], 1)
    # every candidate timed over 20 replays (a replay takes about 0.3 ms)
    plan = A.Plan.autotuned(prs, p, A.AAQ_OBS_HRED, True, params=prm, reps=20)
    plan.params.copy_(torch.from_numpy(prm))
    dt = _timed(plan.execute, 20)
    out = plan.execute().cpu().numpy()
    tuned = plan.tuned_opts
    plan.close()
    rate = len(prs) / dt
    default_rate, _ = _plan_rate(prs, p, A.AAQ_OBS_HRED, True, gam, bet, reps=20)
    single_rate, out_single = _plan_rate(prs, p, A.AAQ_OBS_HRED, True, gam, bet, reps=3, single_launch=True)
    # plain: one aaq_energy_grad call per graph
    ests = {}
    keys = [(pr.n, tuple(probs[i].graph.edges)) for i, pr in enumerate(prs)]
    for i, pr in enumerate(prs):
        if keys[i] not in ests:
            ests[keys[i]] = A.Estimator(pr, p, A.AAQ_OBS_HRED, A.AAQ_PREC_C64, grad=True)

    def plain():
        for i in range(len(prs)):
            ests[keys[i]].energy_grad(gam[i], bet[i])

    dt_plain = _timed(plain, 1, blocks=3)
    ref = _golden("mixed512_p2_references.json")["units"]
    e_ref = np.array([r["energy"] for r in ref])
    g_ref = np.array([r["dgamma"] + r["dbeta"] for r in ref])
    rel_e = np.abs(out[:, 0] - e_ref) / np.abs(e_ref)
    rel_g = np.linalg.norm(out[:, 2:] - g_ref, axis=1) / np.linalg.norm(g_ref, axis=1)
    rate_o, thr = _oracle_rate(lambda k: O.energy_grad(probs[k].n, probs[k].edges(), probs[k].terms(1), gam[k],
                                                       bet[k]), len(probs))
    return {"workload": "c4: 512 mixed graphs n=8..18, p=2, H_red energy + adjoint gradient", "unit": "evals/s",
            "cpu_oracle": {"evals_s": round(rate_o, 1), "threads": thr,
                           "kind": "FP64 full-state oracle energy + adjoint gradient, all 512 instances, median of "
                                   "5 runs"},
            "batched_evals_s": round(rate, 1), "batched_default_opts_evals_s": round(default_rate, 1),
            "single_launch_evals_s": round(single_rate, 1),
            "single_launch_max_rel_err_energy": float(np.max(np.abs(out_single[:, 0] - e_ref) / np.abs(e_ref))),
            "tuned_opts": tuned, "plain_evals_s": round(len(prs) / dt_plain, 1),
            "batched_over_plain": round(rate * dt_plain / len(prs), 2),
            "max_rel_err_energy": float(rel_e.max()), "max_rel_err_grad": float(rel_g.max()),
            "instances_checked": len(prs)}


def c5a(args):
    from oracle import reduced as R

    wp, p, gam, bet = C.config5a(4)
    pr = A.Problem.from_workload(wp)
    est = A.Estimator(pr, p, A.AAQ_OBS_HRED, A.AAQ_PREC_C64, grad=False)
    res = {}
    for oname, obs in (("H_red", A.AAQ_OBS_HRED), ("H_C", A.AAQ_OBS_HC)):
        A.aaq_timing_read(reset=True)
        A.aaq_timing_enable(True)
        dt = _timed(lambda: est.energy(gam[0], bet[0], obs=obs), 2)
        A.aaq_timing_enable(False)
        tm = A.aaq_timing_read(reset=True)
        errs = []
        for k in range(len(gam)):
            e = est.energy(gam[k], bet[k], obs=obs)[0]
            ref = R.p1_energy(wp.n, wp.edges(), wp.terms(obs), gam[k, 0], bet[k, 0])
            errs.append(abs(e - ref) / abs(ref))
        res[oname] = {"s_per_eval": round(dt, 4), "max_rel_err_vs_closed_form": float(max(errs)),
                      "sweep_GBps": {c: round(v["bytes"] / (v["total_ms"] * 1e-3) / 1e9, 1)
                                     for c, v in tm.items() if v["bytes"]}}
    del est
    torch.cuda.empty_cache()
    ref_of = {obs: R.p1_energy(wp.n, wp.edges(), wp.terms(obs), gam[0, 0], bet[0, 0])
              for obs in (A.AAQ_OBS_HC, A.AAQ_OBS_HRED)}
    res["aggregation_modes"] = _agg_modes(pr, p, gam[0], bet[0], 1, 3, ref_of=ref_of.__getitem__)
    res["orbit_ratio_E_over_OE"] = round(wp.m / wp.orbits.count, 3)
    return {"workload": "c5a: random tree n=34 (seed 5) p=1, complex64 energy, 2^34 amplitudes", "results": res}


def c5b(args):
    from oracle import reduced as R

    wp, p, gam, bet = C.config5b(2)
    pr = A.Problem.from_workload(wp)
    est = A.Estimator(pr, p, A.AAQ_OBS_HRED, A.AAQ_PREC_C64, grad=True)
    res = {}
    for oname, obs in (("H_red", A.AAQ_OBS_HRED), ("H_C", A.AAQ_OBS_HC)):
        A.aaq_timing_read(reset=True)
        A.aaq_timing_enable(True)
        dt = _timed(lambda: est.energy_grad(gam[0], bet[0], obs=obs), 2)
        A.aaq_timing_enable(False)
        tm = A.aaq_timing_read(reset=True)
        e, dg, db, nrm = est.energy_grad(gam[1], bet[1], obs=obs)
        e_lc, dg_lc, db_lc, mb = R.light_cone_energy_grad(wp.n, wp.edges(), wp.terms(obs), gam[1], bet[1])
        g, gr = np.concatenate([dg, db]), np.concatenate([dg_lc, db_lc])
        res[oname] = {"s_per_eval": round(dt, 4), "rel_err_energy": abs(e - e_lc) / abs(e_lc),
                      "rel_err_grad": float(np.linalg.norm(g - gr) / np.linalg.norm(gr)), "light_cone_max_ball": mb,
                      "sweep_GBps": {c: round(v["bytes"] / (v["total_ms"] * 1e-3) / 1e9, 1)
                                     for c, v in tm.items() if v["bytes"]}}
    return {"workload": "c5b: random tree n=33 (seed 5) p=2, complex64 energy + adjoint gradient", "results": res}


def lc(args):
    from oracle import reduced as R

    res = {}
    for name, fn, npts in (("c3 n=26 p=4", C.config3, 8), ("c5a n=34 p=1", C.config5a, 8),
                           ("c5b n=33 p=2", C.config5b, 4)):
        wp, p, gam, bet = fn(npts)
        pr = A.Problem.from_workload(wp)
        r = {}
        for oname, obs in (("H_red", A.AAQ_OBS_HRED), ("H_C", A.AAQ_OBS_HC)):
            L = A.LightCone(pr, p, obs, with_grad=True)
            L.params.copy_(torch.from_numpy(np.concatenate([gam[0], bet[0]])))
            reps = 200 if wp.n != 26 else 50
            dt = _timed(L.execute, reps)
            errs_e, errs_g = [], []
            for k in range(min(npts, 4)):
                e, dg, db, _ = L.energy_grad(gam[k], bet[k])
                e_lc, dg_lc, db_lc, _ = R.light_cone_energy_grad(wp.n, wp.edges(), wp.terms(obs), gam[k], bet[k])
                g, gr = np.concatenate([dg, db]), np.concatenate([dg_lc, db_lc])
                errs_e.append(abs(e - e_lc) / abs(e_lc))
                errs_g.append(float(np.linalg.norm(g - gr) / np.linalg.norm(gr)))
            L.close()
            # the same cones with each small-unit launch on a stream of its own
            Ls = A.LightCone(pr, p, obs, with_grad=True, small_streams=True)
            Ls.params.copy_(torch.from_numpy(np.concatenate([gam[0], bet[0]])))
            dts = _timed(Ls.execute, reps)
            Ls.close()
            r[oname] = {"units": L.units, "max_cone_qubits": L.max_qubits, "cone_amplitudes": L.amplitudes,
                        "evals_s": round(1.0 / dt, 1), "small_streams_evals_s": round(1.0 / dts, 1),
                        "max_rel_err_energy": float(max(errs_e)), "max_rel_err_grad": float(max(errs_g))}
        r["speedup_Hred_over_HC"] = round(r["H_red"]["evals_s"] / r["H_C"]["evals_s"], 3)
        res[name] = r
    return {"workload": "lc: light-cone x orbit evaluation (energy + adjoint gradient, complex64), device-resident "
                        "parameters and outputs, graph replay", "unit": "evals/s", "results": res}


def sample(args):
    """Final-state sampling at the n=26 p=4 and n=33 p=2 tree sizes: forward sweeps that keep
    the state, then inverse-CDF draws; sampled approximation ratios against C_max = |E|."""
    res = {}
    for name, fn in (("c3 n=26 p=4", C.config3), ("c5b n=33 p=2", C.config5b)):
        wp, p, gam, bet = fn(1)
        pr = A.Problem.from_workload(wp)
        cmax = len(wp.edges())  # trees are bipartite
        for shots in (1 << 10, 1 << 20):
            s = A.Sampler(pr, p, shots)
            s.uniform.copy_(torch.rand(shots, dtype=torch.float64, generator=torch.Generator().manual_seed(shots)))
            best, mean = A.aaq_sample(pr, gam[0], bet[0], A.AAQ_PREC_C64, s.uniform, s.state, s.ws, s.samples,
                                      s.cuts)
            dt = _timed(lambda: A.aaq_sample(pr, gam[0], bet[0], A.AAQ_PREC_C64, s.uniform, s.state, s.ws,
                                             s.samples, s.cuts), 5 if wp.n > 30 else 20)
            res[f"{name} shots={shots}"] = {"calls_s": round(1.0 / dt, 2), "shots_s": round(shots / dt, 1),
                                            "best_cut": best, "mean_cut": mean, "R_best": best / cmax,
                                            "R_mean": mean / cmax}
            del s
            torch.cuda.empty_cache()
    return {"workload": "sample: forward pass keeping the state + inverse-CDF sampling (complex64 state, FP64 CDF)",
            "unit": "calls/s", "results": res}


def weighted(args):
    from oracle import reduced as R

    wp0, p, gam, bet = C.config3(4)
    g = wp0.graph
    w = np.random.default_rng(26).integers(1, 5, g.m).astype(np.int32)
    wp = C.make_problem(g, weights=w)
    res = {"total_weight": int(w.sum()), "orbits": wp.orbits.count}
    for name, prob in (("weighted", wp), ("unweighted", wp0)):
        pr = A.Problem.from_workload(prob)
        est = A.Estimator(pr, p, A.AAQ_OBS_HRED, A.AAQ_PREC_C64, grad=True, checkpoint=True)
        k = [0]

        def step():
            est.energy_grad(gam[k[0] % 4], bet[k[0] % 4])
            k[0] += 1

        dt = _timed(step, 20)
        r = {"evals_s": round(1.0 / dt, 2)}
        if name == "weighted":
            errs_e, errs_g = [], []
            for j in range(2):
                e, dg, db, _ = est.energy_grad(gam[j], bet[j])
                e_lc, dg_lc, db_lc, _ = R.light_cone_energy_grad(wp.n, wp.edges(), wp.terms(A.AAQ_OBS_HRED), gam[j],
                                                                 bet[j], weights=w)
                errs_e.append(abs(e - e_lc) / abs(e_lc))
                errs_g.append(float(np.linalg.norm(np.concatenate([dg - dg_lc, db - db_lc]))
                                    / np.linalg.norm(np.concatenate([dg_lc, db_lc]))))
            r["max_rel_err_energy"] = float(max(errs_e))
            r["max_rel_err_grad"] = float(max(errs_g))
            L = A.LightCone(pr, p, A.AAQ_OBS_HRED, with_grad=True)
            L.params.copy_(torch.from_numpy(np.concatenate([gam[0], bet[0]])))
            r["light_cone_evals_s"] = round(1.0 / _timed(L.execute, 50), 1)
            L.close()
        res[name] = r
        del est
        torch.cuda.empty_cache()
    return {"workload": "weighted: n=26 p=4 tree, integer edge weights 1..4, H_red energy + gradient (complex64, "
                        "checkpoints)", "unit": "evals/s", "results": res}


def adam(args):
    from paper_2410_22247_amd.autograd import adam_maximize, adam_maximize_resident

    wp, p, gam, bet = C.config3(1)
    pr = A.Problem.from_workload(wp)
    steps, lr = 200, 0.01
    res = A.Resident(pr, p, A.AAQ_OBS_HRED, with_grad=True, checkpoint=True)
    adam_maximize_resident(res, gam[0], bet[0], steps=3, lr=lr)  # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    g_r, b_r, h_r = adam_maximize_resident(res, gam[0], bet[0], steps=steps, lr=lr)
    t_res = time.perf_counter() - t
    res.close()
    est = A.Estimator(pr, p, A.AAQ_OBS_HRED, A.AAQ_PREC_C64, grad=True, checkpoint=True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    g_h, b_h, h_h = adam_maximize(est, gam[0], bet[0], steps=steps, lr=lr)
    t_host = time.perf_counter() - t
    e_hc = est.energy_grad(g_r, b_r, obs=A.AAQ_OBS_HC)[0]
    e_red = est.energy_grad(g_r, b_r)[0]
    cmax = len(wp.edges())  # trees are bipartite
    return {"workload": "adam: n=26 p=4 tree, 200 Adam steps (lr 0.01) maximising <H_red> from the first seeded "
                        "point (complex64, checkpoints)", "unit": "ms/step",
            "results": {"resident_ms_per_step": round(1e3 * t_res / steps, 3),
                        "host_api_ms_per_step": round(1e3 * t_host / steps, 3),
                        "energy_start": float(h_r[0, 0]), "energy_end_H_red": float(e_red),
                        "energy_end_H_C": float(e_hc), "expectation_ratio_end": float(e_hc / cmax),
                        "max_abs_diff_trajectories": float(np.max(np.abs(h_r[:, 0] - h_h))),
                        "gamma_end": g_r.tolist(), "beta_end": b_r.tolist()}}


def run(name, args):
    torch.cuda.set_device(0)
    return {"c1": c1, "c2": c2, "c4": c4, "c5a": c5a, "c5b": c5b, "lc": lc, "sample": sample, "weighted": weighted, "adam": adam}[name](args)
