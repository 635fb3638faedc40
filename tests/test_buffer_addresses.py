"""State buffers at any device address.

The sweeps reach a state buffer through a buffer descriptor built from the buffer's
address.  These tests place the state, lambda and checkpoint buffers at device addresses
whose bit 31 is set and at addresses where it is clear. The buffers are views into one
allocation of 4 GiB plus the buffers, so both cases occur whatever the allocator returns.
Energy and gradient are compared with the FP64 oracle, with and without the spin-flip
half state (tolerances as in test_gpu_parity)."""
import math

import numpy as np
import pytest

import oracle as O
import paper_2410_22247_amd as A
from workloads import graphs as G
from workloads.configs import OBS_HRED, make_problem

C64 = A.AAQ_PREC_C64


def views_at(big, bit31: int, sizes):
    """Consecutive views of `big` (uint8) of the given byte sizes, each 2^20-aligned,
    the first at a multiple of 2^31 whose bit 31 equals `bit31`, all inside one 2^31
    window (so every view's address has the same bit 31)."""
    base, size = big.data_ptr(), big.numel()
    span = sum((s + (1 << 20) - 1) >> 20 << 20 for s in sizes)
    assert span < (1 << 31)
    k = -(-base >> 31)  # first multiple of 2^31 at or above base
    while ((k & 1) != bit31) or (k << 31) + span > base + size:
        k += 1
        assert (k << 31) <= base + size, "no window of the requested parity"
    off = (k << 31) - base
    out = []
    for s in sizes:
        v = big[off:off + s]
        assert ((v.data_ptr() >> 31) & 1) == bit31
        out.append(v)
        off += (s + (1 << 20) - 1) >> 20 << 20
    return out


@pytest.mark.gpu
@pytest.mark.parametrize("half", [1, 0])
@pytest.mark.parametrize("bit31", [0, 1])
def test_buffers_at_either_bit31(bit31, half):
    import torch

    g = G.prufer_tree(20, 3)
    wp = make_problem(g)
    pr = A.Problem.from_workload(wp)
    p = 2
    rng = np.random.default_rng(31)
    gam, bet = rng.uniform(0, math.pi, p), rng.uniform(0, math.pi / 2, p)
    e_ref, dg_ref, db_ref = O.energy_grad(g.n, g.edge_array(), wp.terms(OBS_HRED), gam, bet)
    g_ref = np.concatenate([dg_ref, db_ref])
    sb = A.aaq_state_bytes(pr, C64)
    cb = A.aaq_checkpoint_bytes(pr, p, C64)
    wb = A.aaq_workspace_size(pr, p, True, OBS_HRED)
    ws = torch.empty(wb, dtype=torch.uint8, device="cuda")
    big = torch.empty((1 << 32) + cb + sb + (4 << 20), dtype=torch.uint8, device="cuda")
    A.aaq_set_half_state(half)
    try:
        ckpt, lam = views_at(big, bit31, [cb, sb])
        for call in ("uncompute", "checkpoints"):
            if call == "uncompute":
                e, dg, db, nrm = A.aaq_energy_grad(pr, gam, bet, OBS_HRED, C64, ckpt[:sb], lam, ws)
            else:
                e, dg, db, nrm = A.aaq_energy_grad_checkpointed(pr, gam, bet, OBS_HRED, C64, ckpt, lam, ws)
            assert abs(e - e_ref) <= 1e-5 * abs(e_ref), (call, e, e_ref)
            assert np.linalg.norm(np.concatenate([dg, db]) - g_ref) <= 1e-5 * np.linalg.norm(g_ref), call
            assert abs(nrm - 1) <= 1e-5
        e, _, nrm = A.aaq_energy(pr, gam, bet, OBS_HRED, A.AAQ_AGG_FUSED, C64, ckpt[:sb], ws)
        assert abs(e - e_ref) <= 1e-5 * abs(e_ref)
    finally:
        A.aaq_set_half_state(1)
    del big
    torch.cuda.empty_cache()
