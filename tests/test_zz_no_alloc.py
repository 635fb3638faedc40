"""aaq_energy_grad_noalloc, the entry point for callers that cannot allocate device memory:
through the C ABI, two calls in a row (the second on a smaller instance) give the outputs of
aaq_energy_grad on the same inputs (the same kernels and plan: identical bits) and the FP64
oracle's within the path's tolerances; a problem whose workspace exceeds the static
maximum is refused on the host."""
import numpy as np
import pytest

import oracle as O
import paper_2410_22247_amd as A
from workloads import graphs as G
from workloads.configs import OBS_HRED, make_problem


def test_oversize_refused_on_host():
    big = A.Problem.from_workload(make_problem(G.prufer_tree(30, 1)))
    assert A.aaq_workspace_size(big, 8, True, OBS_HRED) > (64 << 20)
    with pytest.raises(A.AAQError) as e:
        A.aaq_energy_grad_noalloc(big, np.full(8, 0.3), np.full(8, 0.2), OBS_HRED, A.AAQ_PREC_C64, None, None, stream=0)
    assert e.value.status == 5
    small = A.Problem.from_workload(make_problem(G.prufer_tree(10, 1)))
    with pytest.raises(A.AAQError) as e:
        A.aaq_energy_grad_noalloc(small, [np.nan], [0.2], OBS_HRED, A.AAQ_PREC_C64, None, None, stream=0)
    assert e.value.status == 4


@pytest.mark.gpu
def test_noalloc_matches_energy_grad_twice():
    import torch

    cases = [(G.prufer_tree(22, 7), 3, np.array([0.4, 1.3, 2.2]), np.array([0.9, 0.5, 0.25])),
             (G.binary_tree(15), 2, np.array([0.7, 1.9]), np.array([0.3, 1.1]))]
    for g, p, gam, bet in cases:  # the second call is on a smaller instance
        wp = make_problem(g)
        pr = A.Problem.from_workload(wp)
        sb = A.aaq_state_bytes(pr)
        st = torch.empty(sb, dtype=torch.uint8, device="cuda")
        lam = torch.empty(sb, dtype=torch.uint8, device="cuda")
        ws = torch.empty(A.aaq_workspace_size(pr, p, True, OBS_HRED), dtype=torch.uint8, device="cuda")
        e0, dg0, db0, n0 = A.aaq_energy_grad(pr, gam, bet, OBS_HRED, A.AAQ_PREC_C64, st, lam, ws)
        e1, dg1, db1, n1 = A.aaq_energy_grad_noalloc(pr, gam, bet, OBS_HRED, A.AAQ_PREC_C64, st, lam)
        assert e1 == e0 and n1 == n0 and np.array_equal(dg1, dg0) and np.array_equal(db1, db0)
        e_ref, dg_ref, db_ref = O.energy_grad(g.n, g.edge_array(), wp.terms(OBS_HRED), gam, bet)
        gr, gv = np.concatenate([dg_ref, db_ref]), np.concatenate([dg1, db1])
        assert abs(e1 - e_ref) <= 1e-5 * abs(e_ref)
        assert np.linalg.norm(gv - gr) <= 1e-5 * np.linalg.norm(gr)
        assert np.all(np.abs(gv - gr) <= 1e-5 * np.maximum(np.abs(gr), np.linalg.norm(gr)))
        assert abs(n1 - 1) <= 1e-5
        del st, lam, ws
        torch.cuda.synchronize()
