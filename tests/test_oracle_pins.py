"""The FP64 oracle pinned to things other than itself: brute-force cut
enumeration, closed forms (p = 1 formula, Dicke and star subspaces), exact
identities of the paper (Eq. exact, Eqs. A2/A3, reverse causal cone),
invariants, and three independent gradient routes."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import derivs as D
from oracle import reduced as R
from workloads import graphs as G
from workloads.configs import OBS_HC, OBS_HRED, make_problem
from workloads.orbits import automorphism_generators


def rand_graph(n, pe, seed):
    rng = np.random.default_rng(seed)
    es = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < pe]
    return G.Graph(n, es or [(0, 1)])


SMALL = [G.binary_tree(10), G.complete(6), rand_graph(8, 0.5, 3), G.star(7), G.cycle(9),
         G.generalized_petersen(5, 2)]


# ------------------------------------------------------------------ cut values
@pytest.mark.parametrize("g", SMALL, ids=lambda g: g.name or "rand")
def test_cut_values_brute_force(g):
    z = np.arange(1 << g.n)
    bits = (z[:, None] >> np.arange(g.n)[None, :]) & 1
    want = np.zeros(1 << g.n, dtype=np.int64)
    for u, v in g.edges:
        want += bits[:, u] ^ bits[:, v]
    got = O.cut_values(g.n, g.edge_array())
    assert np.array_equal(got, want)
    assert got[0] == 0
    assert np.array_equal(got, got[(1 << g.n) - 1 - z])  # C(complement z) = C(z)


def test_cut_closed_forms():
    for n in (4, 7, 10):
        c = O.cut_values(n, G.complete(n).edge_array())
        k = np.array([bin(z).count("1") for z in range(1 << n)])
        assert np.array_equal(c, k * (n - k))
        assert c.max() == n * n // 4
    L = 9
    c = O.cut_values(L + 1, G.star(L).edge_array())
    for z in range(1 << (L + 1)):
        kl = bin(z >> 1).count("1")
        assert c[z] == ((L - kl) if z & 1 else kl)
    t = G.binary_tree(12)
    assert O.cut_values(12, t.edge_array()).max() == t.m  # trees are bipartite: C_max = |E|


def test_cut_values_at_indices():
    """The per-index cut values (for states too large for the full table) equal the full
    table on small graphs, weighted or not, and at 34 vertices follow the closed forms of
    K_n and the star and the complement symmetry."""
    for g in SMALL:
        z = np.arange(1 << g.n)
        assert np.array_equal(O.cut_values_at(z, g.edge_array()), O.cut_values(g.n, g.edge_array()))
    for g, w in weighted_graphs()[:4]:
        z = np.arange(1 << g.n)
        assert np.array_equal(O.cut_values_at(z, g.edge_array(), w), O.cut_values(g.n, g.edge_array(), w))
    n = 34
    rng = np.random.default_rng(11)
    z = rng.integers(0, 1 << n, 4096, dtype=np.uint64)
    k = np.array([bin(int(x)).count("1") for x in z])
    assert np.array_equal(O.cut_values_at(z, G.complete(n).edge_array()), k * (n - k))
    kl = np.array([bin(int(x) >> 1).count("1") for x in z])
    assert np.array_equal(O.cut_values_at(z, G.star(n - 1).edge_array()), np.where(z & np.uint64(1), n - 1 - kl, kl))
    t = G.prufer_tree(n, 5)
    full = np.uint64((1 << n) - 1)
    assert np.array_equal(O.cut_values_at(z, t.edge_array()), O.cut_values_at(full ^ z, t.edge_array()))
    prob = make_problem(G.binary_tree(11))
    zz = np.arange(1 << 11)
    assert np.array_equal(O.term_values_at(zz, prob.terms(OBS_HRED)), O.term_values(11, prob.terms(OBS_HRED)))


def test_term_values_weighted():
    prob = make_problem(G.binary_tree(11))
    h = O.term_values(11, prob.terms(OBS_HRED))
    z = np.arange(1 << 11)
    want = np.zeros(1 << 11)
    for i, j, w in zip(*prob.terms(OBS_HRED)):
        want += w * (((z >> i) ^ (z >> j)) & 1)
    assert np.array_equal(h, want)


# ------------------------------------------------------------------ state invariants
def test_state_norm_and_symmetries():
    g = G.binary_tree(13)
    gam, bet = [0.7, -0.3, 1.1], [0.2, 0.9, -0.4]
    psi = O.state(g.n, g.edge_array(), gam, bet)
    assert abs(np.vdot(psi, psi).real - 1) < 1e-12
    z = np.arange(1 << g.n)
    # global bit flip (complement) symmetry of H_C, H_M and |+>
    assert np.max(np.abs(psi - psi[(1 << g.n) - 1 - z])) < 1e-14
    # Eq. A2: A|psi> = |psi> for every automorphism
    for phi in automorphism_generators(g):
        img = np.zeros_like(z)
        for v in range(g.n):
            img |= ((z >> v) & 1) << phi[v]
        assert np.max(np.abs(psi[img] - psi)) < 1e-14


def test_state_special_angles():
    g = rand_graph(8, 0.5, 1)
    psi = O.state(g.n, g.edge_array(), [0.8, 0.3], [0.0, 0.0])  # no mixing: pure phases
    assert np.allclose(np.abs(psi) ** 2, 2.0 ** -g.n, atol=1e-15)
    cuts = O.cut_values(g.n, g.edge_array())
    assert np.allclose(psi, 2.0 ** (-g.n / 2) * np.exp(-1j * 1.1 * cuts), atol=1e-14)
    psi = O.state(g.n, g.edge_array(), [0.0, 0.0], [0.5, 0.9])  # |+> is a mixer eigenvector
    assert np.allclose(psi, psi[0], atol=1e-14) and abs(abs(psi[0]) - 2.0 ** (-g.n / 2)) < 1e-15


def test_per_gate_numpy_simulator_agrees():
    for g in SMALL[:4]:
        prob = make_problem(g)
        gam, bet = [0.4, 1.3], [0.7, 0.25]
        a = O.energy(g.n, g.edge_array(), prob.terms(OBS_HC), gam, bet)
        b = D.per_gate_energy(g.n, g.edge_array(), prob.terms(OBS_HC), gam, bet)
        assert abs(a - b) < 1e-11


# ------------------------------------------------------------------ energies
@pytest.mark.parametrize("g", [G.binary_tree(15), G.complete(6), rand_graph(9, 0.45, 3), G.star(8),
                               G.generalized_petersen(5, 2), G.prufer_tree(12, 4)],
                         ids=lambda g: g.name or "rand")
def test_p1_closed_form(g):
    prob = make_problem(g)
    e = g.edge_array()
    for gam in np.linspace(-1.3, 2.9, 5):
        for bet in np.linspace(-0.6, 1.4, 5):
            full = O.energy(g.n, e, prob.terms(OBS_HC), [gam], [bet])
            cf = R.p1_energy(g.n, e, prob.terms(OBS_HC), gam, bet)
            assert abs(full - cf) < 1e-12, (gam, bet)


def test_p1_t15_worked_values():
    # binary tree on 15 vertices, p = 1: E = 7 + (1/4) sin4b sing (8 + 2 cosg + 18 cos^2 g)
    g = G.binary_tree(15)
    prob = make_problem(g)
    for gam, bet in [(math.pi / 3, math.pi / 8), (0.3, 0.2), (2.0, 1.1)]:
        cf = 7 + 0.25 * math.sin(4 * bet) * math.sin(gam) * (8 + 2 * math.cos(gam) + 18 * math.cos(gam) ** 2)
        assert abs(O.energy(15, g.edge_array(), prob.terms(OBS_HC), [gam], [bet]) - cf) < 1e-12
    # borders of the config-1 grid: sin(gamma) = 0 or sin(4 beta) = 0 -> |E|/2
    for gam in (0.0, math.pi):
        assert abs(O.energy(15, g.edge_array(), prob.terms(OBS_HC), [gam], [0.37]) - 7) < 1e-12
    for bet in (0.0, math.pi / 2):
        assert abs(O.energy(15, g.edge_array(), prob.terms(OBS_HC), [0.81], [bet]) - 7) < 1e-12


@pytest.mark.parametrize("n,p", [(6, 1), (7, 2), (8, 3)])
def test_complete_graph_dicke(n, p):
    g = G.complete(n)
    prob = make_problem(g)
    rng = np.random.default_rng(n)
    gam, bet = rng.uniform(-1, 2, p), rng.uniform(-1, 2, p)
    full = O.energy(n, g.edge_array(), prob.terms(OBS_HC), gam, bet)
    assert abs(full - R.complete_graph_energy(n, gam, bet)) < 1e-11
    # H_red = one edge times 120-style weight n(n-1)/2
    red = O.energy(n, g.edge_array(), prob.terms(OBS_HRED), gam, bet)
    assert abs(red - full) < 1e-11


@pytest.mark.parametrize("L,p", [(5, 1), (8, 2), (9, 3)])
def test_star_subspace(L, p):
    g = G.star(L)
    prob = make_problem(g)
    rng = np.random.default_rng(L)
    gam, bet = rng.uniform(-1, 2, p), rng.uniform(-1, 2, p)
    full = O.energy(L + 1, g.edge_array(), prob.terms(OBS_HC), gam, bet)
    assert abs(full - R.star_energy(L, gam, bet)) < 1e-11


def test_symmetry_identities():
    g = rand_graph(9, 0.4, 7)
    prob = make_problem(g)
    t = prob.terms(OBS_HC)
    gam, bet = np.array([0.3, 1.2]), np.array([0.8, -0.2])
    e0 = O.energy(g.n, g.edge_array(), t, gam, bet)
    assert abs(O.energy(g.n, g.edge_array(), t, -gam, -bet) - e0) < 1e-12
    # the sign of gamma matters on its own (no accidental symmetry in the convention)
    assert abs(O.energy(g.n, g.edge_array(), t, -gam, bet) - e0) > 1e-3
    # period pi/2 in beta at p = 1
    a = O.energy(g.n, g.edge_array(), t, [0.9], [0.3])
    b = O.energy(g.n, g.edge_array(), t, [0.9], [0.3 + math.pi / 2])
    assert abs(a - b) < 1e-12


@pytest.mark.parametrize("g", [G.binary_tree(15), G.binary_tree(13), G.complete(7), G.circulant(11, [1, 2]),
                               G.generalized_petersen(5, 2), G.prufer_tree(13, 2)], ids=lambda g: g.name)
def test_exact_identity_hred_equals_hc(g):
    """Eq. exact: <H_red> = <H_C> on the Aut(G)-invariant state, for any choice of representatives."""
    rng = np.random.default_rng(1)
    p = 2
    gam, bet = rng.uniform(-1, 2, p), rng.uniform(-1, 2, p)
    prob = make_problem(g)
    e = g.edge_array()
    ehc, edir, zz, nrm = O.energy(g.n, e, prob.terms(OBS_HC), gam, bet, full=True)
    assert abs(ehc - edir) < 1e-11 and abs(nrm - 1) < 1e-12
    for trial in range(3):
        pr = make_problem(g, rep_rng=np.random.default_rng(trial))
        assert abs(O.energy(g.n, e, pr.terms(OBS_HRED), gam, bet) - ehc) < 1e-11
    # Eq. A3: per-edge <ZZ> equal inside each orbit
    for orb in prob.orbits.orbits:
        vals = zz[orb]
        assert np.ptp(vals) < 1e-12
    # and the identity fails for a non-orbit grouping (the finder is not vacuous)
    if prob.orbits.count > 1:
        ti, tj, tw = prob.terms(OBS_HRED)
        wrong = (ti, tj, np.roll(tw, 1))
        if not np.array_equal(np.roll(tw, 1), tw):
            assert abs(O.energy(g.n, e, wrong, gam, bet) - ehc) > 1e-6


def test_light_cone_equals_full_state():
    g = G.binary_tree(15)
    prob = make_problem(g)
    for p in (1, 2):
        rng = np.random.default_rng(p)
        gam, bet = rng.uniform(0, 3, p), rng.uniform(0, 1.5, p)
        full = O.energy(15, g.edge_array(), prob.terms(OBS_HC), gam, bet)
        lc = R.light_cone_energy(15, g.edge_array(), prob.terms(OBS_HC), gam, bet)
        assert abs(full - lc) < 1e-12
    g = G.prufer_tree(16, 9)
    prob = make_problem(g)
    gam, bet = [0.4, 1.1, 0.2], [0.3, 0.6, 1.0]
    e1, dg1, db1 = O.energy_grad(16, g.edge_array(), prob.terms(OBS_HRED), gam, bet)
    e2, dg2, db2, mb = R.light_cone_energy_grad(16, g.edge_array(), prob.terms(OBS_HRED), gam, bet)
    assert abs(e1 - e2) < 1e-11 and np.allclose(dg1, dg2, atol=1e-11) and np.allclose(db1, db2, atol=1e-11)


def test_zero_expectation_single_z():
    g = G.binary_tree(9)
    psi = O.state(9, g.edge_array(), [0.5, 1.0], [0.3, 0.7])
    z = np.arange(1 << 9)
    for v in range(9):
        sign = 1 - 2 * ((z >> v) & 1)
        assert abs(np.sum(np.abs(psi) ** 2 * sign)) < 1e-14


# ------------------------------------------------------------------ gradients
@pytest.mark.parametrize("g,obs", [(G.binary_tree(10), OBS_HRED), (rand_graph(8, 0.5, 5), OBS_HC),
                                   (G.complete(6), OBS_HRED)], ids=["tree10", "rand8", "K6"])
def test_gradient_three_routes(g, obs):
    prob = make_problem(g)
    e = g.edge_array()
    t = prob.terms(obs)
    gam, bet = [0.45, 1.2, -0.3], [0.35, -0.15, 0.8]
    en, dg, db, dev = O.energy_grad(g.n, e, t, gam, bet, with_dev=True)
    assert dev < 1e-12  # the backward sweep returns psi to |+>
    assert abs(en - O.energy(g.n, e, t, gam, bet)) < 1e-12
    f = lambda gg, bb: O.energy(g.n, e, t, gg, bb)
    fdg, fdb = D.central_fd(f, gam, bet, h=1e-4)
    assert np.allclose(dg, fdg, atol=2e-7) and np.allclose(db, fdb, atol=2e-7)
    lg, lb = D.layer_shift(g.n, e, t, gam, bet)
    assert np.allclose(dg, lg, atol=1e-10) and np.allclose(db, lb, atol=1e-10)
    pg, pb = D.per_gate_shift(g.n, e, t, gam, bet)
    assert np.allclose(dg, pg, atol=1e-10) and np.allclose(db, pb, atol=1e-10)


def test_gradient_p1_closed_form_and_hred_identity():
    g = G.binary_tree(15)
    prob = make_problem(g)
    e = g.edge_array()
    for gam, bet in [(0.7, 0.3), (2.2, 1.1)]:
        en, dg, db = O.energy_grad(15, e, prob.terms(OBS_HC), [gam], [bet])
        cg, cb = R.p1_dEdgamma_dbeta(15, e, prob.terms(OBS_HC), gam, bet)
        assert abs(dg[0] - cg) < 1e-7 and abs(db[0] - cb) < 1e-7
        en2, dg2, db2 = O.energy_grad(15, e, prob.terms(OBS_HRED), [gam], [bet])
        assert abs(en - en2) < 1e-12 and abs(dg[0] - dg2[0]) < 1e-11 and abs(db[0] - db2[0]) < 1e-11


# ------------------------------------------------------------------ final-state sampling
def test_sample_uniform_state_closed_form():
    """gamma = 0 (and beta = 0) leave |psi|^2 uniform: the inverse CDF is floor(u 2^n)."""
    g = G.prufer_tree(9, 2)
    u = np.concatenate([np.random.default_rng(0).random(200), [0.0, 1.0 - 2.0 ** -53, 0.5]])
    for gam, bet in ((np.zeros(2), np.array([0.3, 1.1])), (np.array([0.4, 2.0]), np.zeros(2))):
        z, c, cdf = O.sample(g.n, g.edge_array(), gam, bet, u)
        assert np.allclose(cdf, np.arange(1, 513) / 512, rtol=0, atol=1e-13)
        # floor(u 2^n), except where u sits within rounding of a multiple of 2^-n
        want = np.floor(u * 512).astype(np.int64)
        near = np.abs(u * 512 - np.round(u * 512)) < 1e-9
        assert np.all((z == want) | near)
        assert np.array_equal(c, O.cut_values(g.n, g.edge_array())[z])


def test_sample_frequencies_and_mean_cut():
    """On an even grid of M uniforms, bitstring z is drawn within 1 of M |psi(z)|^2 times
    and the mean sampled cut lies within |E|/M of <H_C> (an independently pinned energy)."""
    g = rand_graph(7, 0.5, 11)
    gam, bet = np.array([0.7, 0.2]), np.array([0.35, 0.9])
    M = 1 << 16
    u = (np.arange(M) + 0.5) / M
    z, c, _ = O.sample(g.n, g.edge_array(), gam, bet, u)
    prob = np.abs(O.state(g.n, g.edge_array(), gam, bet)) ** 2
    cnt = np.bincount(z.astype(np.int64), minlength=1 << g.n)
    assert np.all(np.abs(cnt - M * prob) <= 1.0 + 1e-9)
    e = O.energy(g.n, g.edge_array(), make_problem(g).terms(OBS_HC), gam, bet)
    assert abs(c.mean() - e) <= 2 * g.m / M * (1 << g.n)  # each bitstring's count is off by < 1
    assert np.all(np.diff(z.astype(np.int64)) >= 0)  # monotone in u


# ------------------------------------------------------------------ weighted cut (integer w_ij)
def weighted_graphs():
    """(graph, integer weights) pairs: weights drawn per edge, per orbit of Aut(G) (so every
    automorphism preserves them), and with triangles."""
    out = []
    rng = np.random.default_rng(5)
    for g in (G.complete(5), rand_graph(8, 0.5, 3), G.cycle(7), G.generalized_petersen(5, 2), G.binary_tree(10)):
        out.append((g, rng.integers(1, 6, g.m).astype(np.int32)))
    for g in (G.binary_tree(15), G.star(7), G.complete(6)):
        wp = make_problem(g)
        out.append((g, (1 + 2 * np.asarray(wp.orbits.orbit_of) % 5).astype(np.int32)))
    return out


@pytest.mark.parametrize("g,w", weighted_graphs(), ids=lambda x: getattr(x, "name", None) or "w")
def test_weighted_cut_values_brute_force(g, w):
    z = np.arange(1 << g.n)
    bits = (z[:, None] >> np.arange(g.n)[None, :]) & 1
    want = np.zeros(1 << g.n, dtype=np.int64)
    for (u, v), we in zip(g.edges, w):
        want += int(we) * (bits[:, u] ^ bits[:, v])
    assert np.array_equal(O.cut_values(g.n, g.edge_array(), w), want)
    assert np.array_equal(O.cut_values(g.n, g.edge_array(), np.ones(g.m)), O.cut_values(g.n, g.edge_array()))


@pytest.mark.parametrize("g,w", weighted_graphs(), ids=lambda x: getattr(x, "name", None) or "w")
def test_weighted_p1_closed_form(g, w):
    """The single-layer Ising formula against the full-state oracle, every edge term."""
    rng = np.random.default_rng(g.n)
    ti, tj, _ = make_problem(g).terms(OBS_HC)
    for _ in range(3):
        gam, bet = float(rng.uniform(0, math.pi)), float(rng.uniform(0, math.pi / 2))
        _, _, zz, _ = O.energy(g.n, g.edge_array(), (ti, tj, np.ones(len(ti))), [gam], [bet], full=True,
                               weights=w)
        want = [R.p1_weighted_zz(g.n, g.edge_array(), w, int(i), int(j), gam, bet) for i, j in zip(ti, tj)]
        assert np.allclose(zz, want, rtol=0, atol=1e-12)
        # unit weights reduce the formula to the unweighted closed form
        e1 = R.p1_weighted_energy(g.n, g.edge_array(), np.ones(g.m), (ti, tj, np.ones(len(ti))), gam, bet)
        assert abs(e1 - R.p1_energy(g.n, g.edge_array(), (ti, tj, np.ones(len(ti))), gam, bet)) < 1e-12


def test_weighted_state_scaling_and_unit_weights():
    """psi(k w, gamma / k) = psi(w, gamma): a weight enters the phase only as gamma w."""
    g = rand_graph(8, 0.4, 9)
    w = np.random.default_rng(2).integers(1, 4, g.m).astype(np.int32)
    gam, bet = np.array([0.3, 0.8]), np.array([0.5, 0.2])
    a = O.state(g.n, g.edge_array(), gam, bet, weights=w)
    b = O.state(g.n, g.edge_array(), gam / 3, bet, weights=3 * w)
    assert np.allclose(a, b, rtol=0, atol=1e-13)
    assert np.array_equal(O.state(g.n, g.edge_array(), gam, bet, weights=np.ones(g.m)),
                          O.state(g.n, g.edge_array(), gam, bet))


@pytest.mark.parametrize("g", [G.binary_tree(15), G.star(7), G.complete(6), G.generalized_petersen(5, 2)],
                         ids=lambda g: g.name)
def test_weighted_exact_identity_and_gradient(g):
    """Weights constant on the edge orbits of Aut(G): every automorphism preserves them, so
    <H_red> = <H_C> with H_red weights orbit size x edge weight (energy and gradient), and the
    adjoint gradient matches central differences of the energy."""
    wp = make_problem(g)
    w = (1 + 2 * np.asarray(wp.orbits.orbit_of) % 5).astype(np.int32)
    ti, tj, _ = wp.terms(OBS_HC)
    hc = (ti, tj, w.astype(np.float64))
    rep = wp.orbit_rep()
    hred = (ti[rep], tj[rep], (wp.orbit_size() * w[rep]).astype(np.float64))
    gam, bet = np.array([0.4, 1.1]), np.array([0.7, 0.3])
    e_c, dg_c, db_c = O.energy_grad(g.n, g.edge_array(), hc, gam, bet, weights=w)
    e_r, dg_r, db_r = O.energy_grad(g.n, g.edge_array(), hred, gam, bet, weights=w)
    assert abs(e_c - e_r) < 1e-12 and np.allclose(dg_c, dg_r, atol=1e-11) and np.allclose(db_c, db_r, atol=1e-11)
    assert abs(e_c - O.energy(g.n, g.edge_array(), hc, gam, bet, weights=w)) < 1e-12
    h = 1e-5
    for l in range(2):
        d = np.zeros(2)
        d[l] = h
        fd_g = (O.energy(g.n, g.edge_array(), hc, gam + d, bet, weights=w)
                - O.energy(g.n, g.edge_array(), hc, gam - d, bet, weights=w)) / (2 * h)
        fd_b = (O.energy(g.n, g.edge_array(), hc, gam, bet + d, weights=w)
                - O.energy(g.n, g.edge_array(), hc, gam, bet - d, weights=w)) / (2 * h)
        assert abs(fd_g - dg_c[l]) < 1e-6 * max(1.0, abs(dg_c[l]))
        assert abs(fd_b - db_c[l]) < 1e-6 * max(1.0, abs(db_c[l]))


def test_weighted_light_cone_equals_full_state():
    g = G.prufer_tree(14, 6)
    w = np.random.default_rng(1).integers(1, 5, g.m).astype(np.int32)
    ti, tj, _ = make_problem(g).terms(OBS_HC)
    hc = (ti, tj, w.astype(np.float64))
    gam, bet = np.array([0.6, 0.25]), np.array([0.35, 0.9])
    e, dg, db = O.energy_grad(g.n, g.edge_array(), hc, gam, bet, weights=w)
    e2, dg2, db2, _ = R.light_cone_energy_grad(g.n, g.edge_array(), hc, gam, bet, weights=w)
    assert abs(e - e2) < 1e-11 and np.allclose(dg, dg2, atol=1e-10) and np.allclose(db, db2, atol=1e-10)
