"""Per-kernel timing (aaq_timing_enable / aaq_timing_read): every launch carries a start
and an end event in its dispatch; the read sums them per kernel class.

CPU: reading with nothing timed.
GPU: one checkpointed evaluation is timed with the expected launch count and
algorithmic state bytes per class and positive times, in both state modes, and its
results are bit-identical to the untimed evaluation's; a plan captured into a graph
while timing is on gives the untimed plan's results and records no timed launches
(kernels recorded into a graph carry no events)."""
import math

import numpy as np
import pytest

import paper_2410_22247_amd as A
from workloads import graphs as G
from workloads.configs import OBS_HRED, make_problem

C64 = A.AAQ_PREC_C64
AAQ_ERR_INVALID_ARG = 1


def test_timing_read_empty():
    A.aaq_timing_enable(False)
    A.aaq_timing_read(reset=True)
    assert A.aaq_timing_read(reset=True) == {}


def test_timing_class_mask_checked():
    lib = A._lib.lib()
    for bad in (-1, 1 << len(A.api.TIMING_CLASSES)):
        assert lib.aaq_timing_classes(bad) == AAQ_ERR_INVALID_ARG
    A.aaq_timing_classes(["sweep_2state", "reduce"])
    A.aaq_timing_classes(None)
    with pytest.raises(ValueError):
        A.aaq_timing_classes(["no_such_class"])


@pytest.mark.gpu
@pytest.mark.parametrize("half", [1, 0])
def test_timing_counts_and_bytes(half):
    import torch

    g = G.prufer_tree(20, 3)
    pr = A.Problem.from_workload(make_problem(g))
    p = 3
    rng = np.random.default_rng(5)
    gam, bet = rng.uniform(0, math.pi, p), rng.uniform(0, math.pi / 2, p)
    A.aaq_set_half_state(half)
    try:
        est = A.Estimator(pr, p, OBS_HRED, C64, grad=True, checkpoint=True)
        r0 = est.energy_grad(gam, bet)
        torch.cuda.synchronize()
        A.aaq_timing_read(reset=True)
        A.aaq_timing_enable(True)
        try:
            r1 = est.energy_grad(gam, bet)
            torch.cuda.synchronize()
        finally:
            A.aaq_timing_enable(False)
        t = A.aaq_timing_read(reset=True)
    finally:
        A.aaq_set_half_state(1)
    assert r0[0] == r1[0] and r0[3] == r1[3]
    assert np.array_equal(r0[1], r1[1]) and np.array_equal(r0[2], r1[2])
    L = A.aaq_get_tile_bits(g.n, C64, True)  # the tile size in force (a test may have set it)
    k = 1 + -(-(g.n - L) // (L - 5))  # set 0: L qubits; every later set: L - 5 active qubits
    assert k >= 2
    m = p * (k - 1)  # forward sweeps after the first
    # forward: the first sweep writes S, the other one-state sweeps read and write;
    # the turnaround reads psi and writes lambda, every backward sweep but the last
    # reads psi and lambda and writes lambda, the last reads both.  S = the stored state:
    # the full 2^n amplitudes, or 2^(n-1) where the half state applies
    assert t["sweep_1state"]["launches"] == m
    S = t["sweep_1state"]["bytes"] / (1 + 2 * (m - 1))
    assert S in ((8 << g.n), (8 << (g.n - 1)) if half else (8 << g.n))
    assert t["sweep_2state"]["launches"] == m + 1
    assert t["sweep_2state"]["bytes"] == (2 + 3 * (m - 1) + 2) * S
    assert t["tables"]["launches"] == 1 and t["reduce"]["launches"] == 1
    for c in ("sweep_1state", "sweep_2state", "tables", "reduce"):
        assert t[c]["total_ms"] > 0, c

    # one class selected: only its launches carry events, with the same counts and bytes
    A.aaq_set_half_state(half)
    try:
        A.aaq_timing_classes(["sweep_2state"])
        A.aaq_timing_read(reset=True)
        A.aaq_timing_enable(True)
        try:
            r2 = est.energy_grad(gam, bet)
            torch.cuda.synchronize()
        finally:
            A.aaq_timing_enable(False)
            A.aaq_timing_classes(None)
        t2 = A.aaq_timing_read(reset=True)
    finally:
        A.aaq_set_half_state(1)
    assert list(t2) == ["sweep_2state"]
    assert t2["sweep_2state"]["launches"] == t["sweep_2state"]["launches"]
    assert t2["sweep_2state"]["bytes"] == t["sweep_2state"]["bytes"]
    assert t2["sweep_2state"]["total_ms"] > 0
    assert r2[0] == r0[0] and np.array_equal(r2[1], r0[1]) and np.array_equal(r2[2], r0[2])


@pytest.mark.gpu
def test_timing_skips_captured_plan():
    import torch

    graphs = [G.star(7), G.prufer_tree(12, 1), G.binary_tree(15), G.prufer_tree(17, 4)]
    prs = [A.Problem.from_workload(make_problem(g)) for g in graphs]
    p = 2
    rng = np.random.default_rng(17)
    prm = torch.from_numpy(np.concatenate([rng.uniform(0, math.pi, (len(prs), p)),
                                           rng.uniform(0, math.pi / 2, (len(prs), p))], 1)).cuda()
    s = torch.cuda.Stream()
    ref_plan = A.Plan(prs, p, OBS_HRED, with_grad=True, use_graph=False)
    ref = ref_plan.execute(params=prm).clone()
    torch.cuda.synchronize()
    A.aaq_timing_read(reset=True)
    A.aaq_timing_enable(True)
    try:
        plan = A.Plan(prs, p, OBS_HRED, with_grad=True, use_graph=True)
        outs = []
        for _ in range(3):  # capture on the first execute, replays after
            with torch.cuda.stream(s):
                o = plan.execute(stream=s, params=prm)
            s.synchronize()
            outs.append(o.clone())
        torch.cuda.synchronize()
    finally:
        A.aaq_timing_enable(False)
    t = A.aaq_timing_read(reset=True)
    assert t == {}
    for o in outs:
        assert torch.equal(o, ref)
    plan.close()
    ref_plan.close()
