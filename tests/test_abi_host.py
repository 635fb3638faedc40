"""The C-ABI library on the host: it loads, exports every function declared in
include/aaqaoa.h, and its host-side validation returns the documented status
for each bad input (no GPU needed: validation runs before any HIP call)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2410_22247_amd as A
from paper_2410_22247_amd import _lib
from workloads import graphs as G
from workloads.configs import make_problem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "aaqaoa.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(aaq_[a-z_]+)\s*\(", src))
    return sorted(names)


def test_library_exports_every_declared_function():
    L = _lib.lib()
    names = header_functions()
    assert len(names) >= 15
    for nm in names:
        assert hasattr(L, nm), nm
    assert set(_lib.EXPORTS) == set(names)


def test_version_and_status_strings():
    assert "gfx950" in A.aaq_version()
    L = _lib.lib()
    for s in range(8):
        assert L.aaq_status_string(s)


def prob(g):
    return A.Problem.from_workload(make_problem(g))


def status_of(fn, *args, **kw):
    try:
        fn(*args, **kw)
    except A.AAQError as e:
        return e.status
    return 0


def test_validation_error_codes():
    ok = prob(G.binary_tree(7))
    assert status_of(A.aaq_validate, ok, 2) == 0
    assert status_of(A.aaq_validate, ok, 0) == 1
    assert status_of(A.aaq_validate, ok, 65) == 1
    assert status_of(A.aaq_validate, A.Problem(0, np.zeros((0, 2))), 1) == 1
    assert status_of(A.aaq_validate, A.Problem(35, np.zeros((0, 2))), 1) == 1
    assert status_of(A.aaq_validate, A.Problem(3, [[0, 3]]), 1) == 2          # vertex out of range
    assert status_of(A.aaq_validate, A.Problem(3, [[1, 1]]), 1) == 2          # self-loop
    assert status_of(A.aaq_validate, A.Problem(3, [[0, 1], [1, 0]]), 1) == 2  # duplicate edge
    # orbits: sizes must sum to |E|, representatives must be edges, sizes >= 1
    e = [[0, 1], [1, 2], [2, 0]]
    assert status_of(A.aaq_validate, A.Problem(3, e, [0], [3]), 1) == 0
    assert status_of(A.aaq_validate, A.Problem(3, e, [0], [2]), 1) == 3
    assert status_of(A.aaq_validate, A.Problem(3, e, [5], [3]), 1) == 3
    assert status_of(A.aaq_validate, A.Problem(3, e, [0, 1], [3, 0]), 1) == 3
    assert status_of(A.aaq_validate, A.Problem(3, e, [0, 0], [2, 1]), 1) == 3
    # edge_orbit consistency
    assert status_of(A.aaq_validate, A.Problem(3, e, [0, 1], [2, 1], [0, 0, 1]), 1) == 3  # rep 1 lies in orbit 0
    assert status_of(A.aaq_validate, A.Problem(3, e, [0, 2], [2, 1], [0, 0, 1]), 1) == 0
    assert status_of(A.aaq_validate, A.Problem(3, e, [0, 2], [2, 1], [0, 1, 1]), 1) == 3
    # a graph with no edges has no orbits
    assert status_of(A.aaq_validate, A.Problem(4, np.zeros((0, 2)), [], []), 1) == 0


def test_entry_points_reject_bad_arguments_before_touching_the_gpu():
    pr = prob(G.binary_tree(9))
    L = _lib.lib()
    e = ctypes.c_double()
    g = np.array([0.1, 0.2])
    b = np.array([0.3, 0.4])
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    # null state
    st = L.aaq_energy(pr.ref(), 2, dp(g), dp(b), 1, 0, 0, None, 0, fake, 1 << 20, None, ctypes.byref(e), None, None)
    assert st == 1
    # state too small
    st = L.aaq_energy(pr.ref(), 2, dp(g), dp(b), 1, 0, 0, fake, 16, fake, 1 << 20, None, ctypes.byref(e), None, None)
    assert st == 5
    # workspace too small
    st = L.aaq_energy(pr.ref(), 2, dp(g), dp(b), 1, 0, 0, fake, 1 << 20, fake, 8, None, ctypes.byref(e), None, None)
    assert st == 5
    # non-finite parameters
    gn = np.array([np.nan, 0.2])
    st = L.aaq_energy(pr.ref(), 2, dp(gn), dp(b), 1, 0, 0, fake, 1 << 20, fake, 1 << 20, None, ctypes.byref(e), None,
                      None)
    assert st == 4
    # bad enums
    st = L.aaq_energy(pr.ref(), 2, dp(g), dp(b), 7, 0, 0, fake, 1 << 20, fake, 1 << 20, None, ctypes.byref(e), None, None)
    assert st == 1
    st = L.aaq_energy(pr.ref(), 2, dp(g), dp(b), 1, 9, 0, fake, 1 << 20, fake, 1 << 20, None, ctypes.byref(e), None, None)
    assert st == 1
    # gradients need a lambda buffer; outputs untouched on error
    dg = np.full(2, 7.0)
    db = np.full(2, 7.0)
    e.value = 3.5
    st = L.aaq_energy_grad(pr.ref(), 2, dp(g), dp(b), 1, 0, fake, 1 << 20, None, 0, fake, 1 << 20, None,
                           ctypes.byref(e), dp(dg), dp(db), None)
    assert st == 1 and e.value == 3.5 and (dg == 7).all() and (db == 7).all()
    assert b"lambda" in L.aaq_last_error_message()


def test_workspace_and_state_sizes():
    pr = prob(G.prufer_tree(26, 3))
    assert A.aaq_state_bytes(pr) == 8 << 26
    assert A.aaq_state_bytes(pr, A.AAQ_PREC_C128) == 16 << 26
    w_e = A.aaq_workspace_size(pr, 4, False)
    w_g = A.aaq_workspace_size(pr, 4, True)
    assert 0 < w_e < w_g < (64 << 20)
    assert A.aaq_num_sets(26) == 3 and A.aaq_num_sets(13) == 1 and A.aaq_num_sets(14) == 2
    assert A.aaq_num_sets(34) == 4 and A.aaq_num_sets(33) == 4


def test_tile_sets_for_every_size_and_tile():
    """The planner's tile sets (qubits from 26 up spread over the later sets) are built for
    every n up to the largest and both tile sizes without tripping its own checks, and the
    set counts are those of the capacity rule: one full set of L qubits, the others L - 5."""
    for prec in (A.AAQ_PREC_C64, A.AAQ_PREC_C128):
        for tb in (12, 13):
            for n in range(2, 35):
                pr = prob(G.prufer_tree(n, n) if n > 2 else G.complete(2))
                A.aaq_set_tile_bits(n, prec, True, tb)
                try:
                    assert A.aaq_workspace_size(pr, 2, True, prec=prec) > 0
                finally:
                    A.aaq_set_tile_bits(n, prec, True, 0)
    for n in range(2, 35):
        k = A.aaq_num_sets(n)
        best = min(1 if n <= L else 1 + -(-(n - L) // (L - 5)) for L in (12, 13))
        assert k == best, (n, k, best)


def test_plan_workspace_size_host_only():
    probs = [prob(G.star(7)), prob(G.complete(9)), prob(G.prufer_tree(16, 2))]
    w = A.aaq_plan_workspace_size(probs, 2, A.AAQ_OBS_HRED, True)
    # the n = 16 unit (two tile sets, p = 2) keeps its p (k - 1) = 2 forward states and lambda,
    # each over the stored half state of 2^15 amplitudes
    assert w > 3 * (8 << 15)
    assert A.aaq_plan_workspace_size(probs, 2, A.AAQ_OBS_HRED, False) < w  # no lambda, no checkpoints
    A.aaq_set_half_state(0)
    try:
        assert A.aaq_plan_workspace_size(probs, 2, A.AAQ_OBS_HRED, True) > 3 * (8 << 16)  # every amplitude stored
    finally:
        A.aaq_set_half_state(1)
    assert status_of(A.aaq_plan_workspace_size, probs, 0, A.AAQ_OBS_HRED, True) == 1
    # plan options outside their ranges
    for bad in ({"tile_bits_large": 11}, {"min_tile_bits_small": 14}, {"workgroups": -1}, {"max_small_n": 11}):
        assert status_of(A.aaq_plan_workspace_size, probs, 2, A.AAQ_OBS_HRED, True, **bad) == 1
    for field in ("small_streams", "single_launch"):
        o = A.api._opts()
        setattr(o, field, 2)
        sz = ctypes.c_size_t()
        st = _lib.lib().aaq_plan_workspace_size(A.api._problem_array(probs), len(probs), 2, A.AAQ_OBS_HRED, 1,
                                                 ctypes.byref(o), ctypes.byref(sz))
        assert st == 1, field
    # the small-unit streams change the launches, not the workspace
    assert A.aaq_plan_workspace_size(probs, 2, A.AAQ_OBS_HRED, True, small_streams=True) == w
    # a 13-qubit unit as batched sweep steps needs its states in the workspace; beside a
    # larger unit that is the default, alone it is not
    p13 = [prob(G.binary_tree(13)), prob(G.prufer_tree(16, 2))]
    w13 = A.aaq_plan_workspace_size(p13, 2, A.AAQ_OBS_HRED, True, max_small_n=13)
    w12 = A.aaq_plan_workspace_size(p13, 2, A.AAQ_OBS_HRED, True, max_small_n=12)
    assert w12 > w13 + 2 * (8 << 12)
    assert A.aaq_plan_workspace_size(p13, 2, A.AAQ_OBS_HRED, True) == w12
    alone = [prob(G.binary_tree(13))]
    assert A.aaq_plan_workspace_size(alone, 2, A.AAQ_OBS_HRED, True) == \
        A.aaq_plan_workspace_size(alone, 2, A.AAQ_OBS_HRED, True, max_small_n=13)
