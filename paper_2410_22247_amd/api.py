"""Python binding of the C ABI in include/aaqaoa.h.

Functions named ``aaq_*`` mirror the C entry points one to one and only marshal
arguments (device buffers are torch tensors, streams are torch streams).  Every
step of the computation runs in the HIP library; a non-zero status raises
``AAQError``.  ``Estimator`` and ``Plan`` are thin conveniences that allocate the
device buffers with torch and call the same entry points.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np

from . import _lib

AAQ_OBS_HC, AAQ_OBS_HRED = 0, 1
AAQ_AGG_FUSED, AAQ_AGG_PER_TERM, AAQ_AGG_PASS_PER_TERM = 0, 1, 2
AAQ_PREC_C64, AAQ_PREC_C128 = 0, 1


class AAQError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"aaqaoa status {status}: {message}")
        self.status = status


def _check(st: int):
    if st != 0:
        L = _lib.lib()
        raise AAQError(st, f"{L.aaq_status_string(st).decode()}: {L.aaq_last_error_message().decode()}")


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32).reshape(-1))


def _ptr_i32(a: Optional[np.ndarray]):
    if a is None:
        return ctypes.POINTER(ctypes.c_int32)()
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


class Problem:
    """A MaxCut instance and its Aut(G) edge orbits, as the C struct ``aaq_problem``.

    ``edges``: (m, 2) vertex pairs; ``orbit_rep``: representative edge index per
    orbit; ``orbit_size``: orbit sizes; ``edge_orbit``: orbit id per edge or None;
    ``edge_weight``: integer edge weights (weighted MaxCut) or None for all 1.
    The numpy arrays are kept alive by this object."""

    def __init__(self, n: int, edges, orbit_rep=None, orbit_size=None, edge_orbit=None, edge_weight=None):
        self.n = int(n)
        self.edges = _i32(edges)
        m = self.edges.size // 2
        if orbit_rep is None:  # every edge its own orbit
            orbit_rep, orbit_size = np.arange(m), np.ones(m)
        self.orbit_rep = _i32(orbit_rep)
        self.orbit_size = _i32(orbit_size)
        self.edge_orbit = None if edge_orbit is None else _i32(edge_orbit)
        self.edge_weight = None if edge_weight is None else _i32(edge_weight)
        self.c = _lib.CProblem(self.n, m, _ptr_i32(self.edges), self.orbit_rep.size, _ptr_i32(self.orbit_rep),
                               _ptr_i32(self.orbit_size), _ptr_i32(self.edge_orbit), _ptr_i32(self.edge_weight))

    @property
    def num_edges(self) -> int:
        return self.edges.size // 2

    @property
    def num_orbits(self) -> int:
        return self.orbit_rep.size

    def num_terms(self, obs: int) -> int:
        return self.num_edges if obs == AAQ_OBS_HC else self.num_orbits

    @classmethod
    def from_edges(cls, n: int, edges, edge_weight=None) -> "Problem":
        """An instance whose Aut(G) edge orbits (weight-preserving ones with weights) are
        computed by the library (aaq_edge_orbits)."""
        of, rep, size = aaq_edge_orbits(n, edges, edge_weight)
        return cls(n, edges, rep, size, of, edge_weight)

    @classmethod
    def from_workload(cls, prob) -> "Problem":
        """From any object with n, edges(), orbit_rep(), orbit_size(), edge_orbit() (and an
        optional ``weights`` attribute)."""
        return cls(prob.n, prob.edges(), prob.orbit_rep(), prob.orbit_size(), prob.edge_orbit(),
                   getattr(prob, "weights", None))

    def ref(self):
        return ctypes.byref(self.c)


def _params(gamma, beta):
    g = np.ascontiguousarray(np.asarray(gamma, dtype=np.float64).reshape(-1))
    b = np.ascontiguousarray(np.asarray(beta, dtype=np.float64).reshape(-1))
    if g.size != b.size:
        raise ValueError("gamma and beta must have the same length p")
    return g, b


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _dev(t):
    """(pointer, bytes) of a torch device tensor, or (None, 0)."""
    if t is None:
        return None, 0
    return ctypes.c_void_p(t.data_ptr()), t.numel() * t.element_size()


def _stream(stream):
    if stream is None:
        import torch

        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


# ------------------------------------------------------------------ mirrors of the C ABI
def aaq_version() -> str:
    return _lib.lib().aaq_version().decode()


def aaq_validate(prob: Problem, p: int) -> None:
    _check(_lib.lib().aaq_validate(prob.ref(), int(p)))


def aaq_state_bytes(prob: Problem, prec: int = AAQ_PREC_C64) -> int:
    out = ctypes.c_size_t()
    _check(_lib.lib().aaq_state_bytes(prob.ref(), int(prec), ctypes.byref(out)))
    return out.value


def aaq_workspace_size(prob: Problem, p: int, with_grad: bool, obs: int = AAQ_OBS_HRED, agg: int = AAQ_AGG_FUSED,
                       prec: int = AAQ_PREC_C64) -> int:
    out = ctypes.c_size_t()
    _check(_lib.lib().aaq_workspace_size(prob.ref(), int(p), int(bool(with_grad)), int(obs), int(agg), int(prec),
                                         ctypes.byref(out)))
    return out.value


def aaq_energy(prob: Problem, gamma, beta, obs: int, agg: int, prec: int, d_state, d_ws, stream=None):
    """Returns (energy, zz or None, norm)."""
    g, b = _params(gamma, beta)
    e, nrm = ctypes.c_double(), ctypes.c_double()
    T = prob.num_terms(obs)
    zz = np.zeros(max(T, 1)) if agg != AAQ_AGG_FUSED else None
    sp, sb = _dev(d_state)
    wp, wb = _dev(d_ws)
    _check(_lib.lib().aaq_energy(prob.ref(), g.size, _dp(g), _dp(b), int(obs), int(agg), int(prec), sp, sb, wp, wb,
                                 _stream(stream), ctypes.byref(e), _dp(zz) if zz is not None else None,
                                 ctypes.byref(nrm)))
    return e.value, (zz[:T] if zz is not None else None), nrm.value


def aaq_energy_grad(prob: Problem, gamma, beta, obs: int, prec: int, d_state, d_lambda, d_ws, stream=None):
    """Returns (energy, dE/dgamma[p], dE/dbeta[p], norm)."""
    g, b = _params(gamma, beta)
    p = g.size
    e, nrm = ctypes.c_double(), ctypes.c_double()
    dg, db = np.zeros(p), np.zeros(p)
    sp, sb = _dev(d_state)
    lp, lb = _dev(d_lambda)
    wp, wb = _dev(d_ws)
    _check(_lib.lib().aaq_energy_grad(prob.ref(), p, _dp(g), _dp(b), int(obs), int(prec), sp, sb, lp, lb, wp, wb,
                                      _stream(stream), ctypes.byref(e), _dp(dg), _dp(db), ctypes.byref(nrm)))
    return e.value, dg, db, nrm.value


def aaq_energy_grad_noalloc(prob: Problem, gamma, beta, obs: int, prec: int, d_state, d_lambda, stream=None):
    """aaq_energy_grad with the library's static per-GPU workspace (no workspace argument, no
    allocation inside the call); returns (energy, dE/dgamma[p], dE/dbeta[p], norm)."""
    g, b = _params(gamma, beta)
    p = g.size
    e, nrm = ctypes.c_double(), ctypes.c_double()
    dg, db = np.zeros(p), np.zeros(p)
    sp, sb = _dev(d_state)
    lp, lb = _dev(d_lambda)
    _check(_lib.lib().aaq_energy_grad_noalloc(prob.ref(), p, _dp(g), _dp(b), int(obs), int(prec), sp, sb, lp, lb,
                                              _stream(stream), ctypes.byref(e), _dp(dg), _dp(db), ctypes.byref(nrm)))
    return e.value, dg, db, nrm.value


def aaq_checkpoint_bytes(prob: Problem, p: int, prec: int = AAQ_PREC_C64) -> int:
    out = ctypes.c_size_t()
    _check(_lib.lib().aaq_checkpoint_bytes(prob.ref(), int(p), int(prec), ctypes.byref(out)))
    return out.value


def aaq_energy_grad_checkpointed(prob: Problem, gamma, beta, obs: int, prec: int, d_ckpt, d_lambda, d_ws,
                                 stream=None):
    """aaq_energy_grad with forward-state checkpoints in d_ckpt; returns (energy, dE/dgamma, dE/dbeta, norm)."""
    g, b = _params(gamma, beta)
    p = g.size
    e, nrm = ctypes.c_double(), ctypes.c_double()
    dg, db = np.zeros(p), np.zeros(p)
    cp, cb = _dev(d_ckpt)
    lp, lb = _dev(d_lambda)
    wp, wb = _dev(d_ws)
    _check(_lib.lib().aaq_energy_grad_checkpointed(prob.ref(), p, _dp(g), _dp(b), int(obs), int(prec), cp, cb, lp, lb,
                                                   wp, wb, _stream(stream), ctypes.byref(e), _dp(dg), _dp(db),
                                                   ctypes.byref(nrm)))
    return e.value, dg, db, nrm.value


def aaq_cut_values(prob: Problem, obs: int, d_ws, d_out, stream=None) -> None:
    wp, wb = _dev(d_ws)
    op, _ = _dev(d_out)
    _check(_lib.lib().aaq_cut_values(prob.ref(), int(obs), wp, wb, op, _stream(stream)))


def aaq_cut_values_layout(prob: Problem, obs: int, set_index: int, arrangement: int, prec: int, d_ws, d_out,
                          stream=None) -> None:
    wp, wb = _dev(d_ws)
    op, _ = _dev(d_out)
    _check(_lib.lib().aaq_cut_values_layout(prob.ref(), int(obs), int(set_index), int(arrangement), int(prec), wp, wb,
                                            op, _stream(stream)))


def aaq_num_sets(n: int, prec: int = AAQ_PREC_C64) -> int:
    return int(_lib.lib().aaq_num_sets(int(n), int(prec)))


def _opts(use_graph=True, workgroups=0, sort_units=True, prec=AAQ_PREC_C64, tile_bits_large=0,
          min_tile_bits_small=0, single_launch=False, small_streams=False, max_small_n=0):
    o = _lib.CPlanOpts()
    _lib.lib().aaq_plan_default_opts(ctypes.byref(o))
    o.use_graph, o.workgroups, o.sort_units, o.prec = int(use_graph), int(workgroups), int(sort_units), int(prec)
    o.tile_bits_large, o.min_tile_bits_small = int(tile_bits_large), int(min_tile_bits_small)
    o.single_launch = int(bool(single_launch))
    o.small_streams = int(bool(small_streams))
    o.max_small_n = int(max_small_n)
    return o


def _opts_dict(o) -> dict:
    return {"use_graph": bool(o.use_graph), "workgroups": int(o.workgroups), "sort_units": bool(o.sort_units),
            "prec": int(o.prec), "tile_bits_large": int(o.tile_bits_large),
            "min_tile_bits_small": int(o.min_tile_bits_small), "single_launch": bool(o.single_launch),
            "small_streams": bool(o.small_streams), "max_small_n": int(o.max_small_n)}


def aaq_set_tile_bits(n: int, prec: int, with_grad: bool, tile_bits: int) -> None:
    _check(_lib.lib().aaq_set_tile_bits(int(n), int(prec), int(bool(with_grad)), int(tile_bits)))


def aaq_get_tile_bits(n: int, prec: int, with_grad: bool) -> int:
    return int(_lib.lib().aaq_get_tile_bits(int(n), int(prec), int(bool(with_grad))))


def aaq_autotune(prob: Problem, p: int, with_grad: bool, obs: int, prec: int, d_state, d_lam, d_ws, reps: int = 3,
                 stream=None):
    """Times both tile sizes for this problem class, keeps the faster; returns (tile_bits, {12: ms, 13: ms})."""
    sp, sb = _dev(d_state)
    lp, lb = _dev(d_lam) if d_lam is not None else (None, 0)
    wp, wb = _dev(d_ws)
    best = ctypes.c_int()
    ms = (ctypes.c_double * 2)()
    _check(_lib.lib().aaq_autotune(prob.ref(), int(p), int(bool(with_grad)), int(obs), int(prec), sp, sb, lp, lb, wp,
                                   wb, _stream(stream), int(reps), ctypes.byref(best), ms))
    return best.value, {12: ms[0], 13: ms[1]}


def aaq_plan_autotune(probs: Sequence[Problem], p: int, obs: int, with_grad: bool, d_ws, d_params, d_out,
                      reps: int = 3, stream=None, **base):
    """Fastest plan options for these units (dict for Plan(**opts)) and its ms per execution."""
    arr = _problem_array(probs)
    o = _opts(**base)
    best = _lib.CPlanOpts()
    ms = ctypes.c_double()
    wp, wb = _dev(d_ws)
    pp, _ = _dev(d_params)
    op, _ = _dev(d_out)
    _check(_lib.lib().aaq_plan_autotune(arr, len(probs), int(p), int(obs), int(bool(with_grad)), ctypes.byref(o), wp,
                                        wb, pp, op, _stream(stream), int(reps), ctypes.byref(best),
                                        ctypes.byref(ms)))
    return _opts_dict(best), ms.value


def _problem_array(probs: Sequence[Problem]):
    arr = (_lib.CProblem * len(probs))()
    for i, pr in enumerate(probs):
        arr[i] = pr.c
    return arr


def aaq_plan_workspace_size(probs: Sequence[Problem], p: int, obs: int, with_grad: bool, **opts) -> int:
    arr = _problem_array(probs)
    o = _opts(**opts)
    out = ctypes.c_size_t()
    _check(_lib.lib().aaq_plan_workspace_size(arr, len(probs), int(p), int(obs), int(bool(with_grad)), ctypes.byref(o),
                                              ctypes.byref(out)))
    return out.value


def aaq_plan_create(probs: Sequence[Problem], p: int, obs: int, with_grad: bool, d_ws, stream=None, **opts):
    arr = _problem_array(probs)
    o = _opts(**opts)
    wp, wb = _dev(d_ws)
    h = ctypes.c_void_p()
    _check(_lib.lib().aaq_plan_create(arr, len(probs), int(p), int(obs), int(bool(with_grad)), ctypes.byref(o), wp, wb,
                                      _stream(stream), ctypes.byref(h)))
    return h


def aaq_plan_execute(plan, d_params, d_out, stream=None) -> None:
    pp, _ = _dev(d_params)
    op, _ = _dev(d_out)
    _check(_lib.lib().aaq_plan_execute(plan, pp, op, _stream(stream)))


def aaq_plan_destroy(plan) -> None:
    if plan:
        _lib.lib().aaq_plan_destroy(plan)


def aaq_sample_workspace_size(prob: Problem, p: int, prec: int = AAQ_PREC_C64) -> int:
    out = ctypes.c_size_t()
    _check(_lib.lib().aaq_sample_workspace_size(prob.ref(), int(p), int(prec), ctypes.byref(out)))
    return out.value


def aaq_sample(prob: Problem, gamma, beta, prec: int, d_uniform, d_state, d_ws, d_samples, d_cuts, stream=None):
    """Draws len(d_uniform) bitstrings into d_samples (uint64) and their cut values into d_cuts
    (int32); returns (best cut, mean cut)."""
    g, b = _params(gamma, beta)
    up, ub = _dev(d_uniform)
    sp, sb = _dev(d_state)
    wp, wb = _dev(d_ws)
    zp, _ = _dev(d_samples)
    cp, _ = _dev(d_cuts)
    best, mean = ctypes.c_double(), ctypes.c_double()
    _check(_lib.lib().aaq_sample(prob.ref(), g.size, _dp(g), _dp(b), int(prec), ub // 8, up, sp, sb, wp, wb,
                                 _stream(stream), zp, cp, ctypes.byref(best), ctypes.byref(mean)))
    return best.value, mean.value


def aaq_edge_orbits(n: int, edges, edge_weight=None):
    """Edge orbits of Aut(G) computed by the library: (orbit_of[m], orbit_rep[k], orbit_size[k]);
    with integer ``edge_weight`` the orbits of the weight-preserving automorphisms."""
    e = _i32(edges)
    m = e.size // 2
    w = None if edge_weight is None else _i32(edge_weight)
    if w is not None and w.size != m:
        raise ValueError("one weight per edge")
    of = np.zeros(max(m, 1), dtype=np.int32)
    rep = np.zeros(max(m, 1), dtype=np.int32)
    size = np.zeros(max(m, 1), dtype=np.int32)
    k = ctypes.c_int32()
    _check(_lib.lib().aaq_edge_orbits(int(n), m, _ptr_i32(e), _ptr_i32(w), _ptr_i32(of), ctypes.byref(k),
                                      _ptr_i32(rep), _ptr_i32(size)))
    return of[:m].copy(), rep[:k.value].copy(), size[:k.value].copy()


def aaq_rcc_eta(n: int, edges, orbit_of, p: int, rep=None, vertex_cover: bool = False, qubits: bool = False):
    """eta_p, the fraction of edges outside the union of the representatives' reverse causal
    cones; with ``rep=None`` the exact mean over uniformly drawn representatives.  With
    ``qubits`` also the qubit-elimination fraction, with ``vertex_cover`` (needs ``rep``)
    also uint8[n], the qubits of the union: returns eta, or a tuple in that order."""
    e = _i32(edges)
    m = e.size // 2
    of = _i32(orbit_of)
    if of.size != m:
        raise ValueError("one orbit id per edge")
    k = int(of.max()) + 1 if m else 0
    r = None if rep is None else _i32(rep)
    if r is not None and r.size != k:
        raise ValueError("one representative per orbit")
    eta, qe = ctypes.c_double(), ctypes.c_double()
    cov = np.zeros(max(int(n), 1), dtype=np.uint8) if vertex_cover else None
    _check(_lib.lib().aaq_rcc_eta(int(n), m, _ptr_i32(e), _ptr_i32(of), k, _ptr_i32(r), int(p), ctypes.byref(eta),
                                  ctypes.byref(qe) if qubits else None,
                                  cov.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)) if cov is not None else None))
    out = (eta.value,) + ((qe.value,) if qubits else ()) + ((cov[:n].copy(),) if vertex_cover else ())
    return out if len(out) > 1 else out[0]


def aaq_resident_workspace_size(prob: Problem, p: int, obs: int, with_grad: bool, checkpoint: bool = False,
                                prec: int = AAQ_PREC_C64):
    """(workspace bytes, state bytes) of a resident evaluator."""
    wb, sb = ctypes.c_size_t(), ctypes.c_size_t()
    _check(_lib.lib().aaq_resident_workspace_size(prob.ref(), int(p), int(obs), int(bool(with_grad)),
                                                  int(bool(checkpoint)), int(prec), ctypes.byref(wb), ctypes.byref(sb)))
    return wb.value, sb.value


def aaq_resident_create(prob: Problem, p: int, obs: int, with_grad: bool, checkpoint: bool, prec: int, d_state, d_lam,
                        d_ws, stream=None):
    sp, sb = _dev(d_state)
    lp, lb = _dev(d_lam)
    wp, wb = _dev(d_ws)
    h = ctypes.c_void_p()
    _check(_lib.lib().aaq_resident_create(prob.ref(), int(p), int(obs), int(bool(with_grad)), int(bool(checkpoint)),
                                          int(prec), sp, sb, lp, lb, wp, wb, _stream(stream), ctypes.byref(h)))
    return h


def aaq_resident_execute(handle, d_params, d_out, stream=None) -> None:
    pp, _ = _dev(d_params)
    op, _ = _dev(d_out)
    _check(_lib.lib().aaq_resident_execute(handle, pp, op, _stream(stream)))


def aaq_resident_destroy(handle) -> None:
    _lib.lib().aaq_resident_destroy(handle)


def aaq_set_half_state(enable: bool) -> None:
    """Process-wide switch of the spin-flip half state (on by default)."""
    _lib.lib().aaq_set_half_state(int(bool(enable)))


def aaq_get_half_state() -> bool:
    return bool(_lib.lib().aaq_get_half_state())


def aaq_lightcone_info(prob: Problem, p: int, obs: int = AAQ_OBS_HRED):
    """(units, largest cone in qubits, total amplitudes of all cone states)."""
    u, mq, amp = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    _check(_lib.lib().aaq_lightcone_info(prob.ref(), int(p), int(obs), ctypes.byref(u), ctypes.byref(mq),
                                         ctypes.byref(amp)))
    return u.value, mq.value, amp.value


def aaq_lightcone_workspace_size(prob: Problem, p: int, obs: int, with_grad: bool, **opts) -> int:
    o = _opts(**opts)
    out = ctypes.c_size_t()
    _check(_lib.lib().aaq_lightcone_workspace_size(prob.ref(), int(p), int(obs), int(bool(with_grad)), ctypes.byref(o),
                                                   ctypes.byref(out)))
    return out.value


def aaq_lightcone_create(prob: Problem, p: int, obs: int, with_grad: bool, d_ws, stream=None, **opts):
    o = _opts(**opts)
    wp, wb = _dev(d_ws)
    h = ctypes.c_void_p()
    _check(_lib.lib().aaq_lightcone_create(prob.ref(), int(p), int(obs), int(bool(with_grad)), ctypes.byref(o), wp, wb,
                                           _stream(stream), ctypes.byref(h)))
    return h


def aaq_lightcone_execute(handle, d_params, d_out, stream=None) -> None:
    pp, _ = _dev(d_params)
    op, _ = _dev(d_out)
    _check(_lib.lib().aaq_lightcone_execute(handle, pp, op, _stream(stream)))


def aaq_lightcone_destroy(handle) -> None:
    if handle:
        _lib.lib().aaq_lightcone_destroy(handle)


def aaq_timing_enable(on: bool) -> None:
    _check(_lib.lib().aaq_timing_enable(int(bool(on))))


TIMING_CLASSES = ("sweep_1state", "sweep_2state", "tables", "reduce", "zz_pass", "units")


def aaq_timing_classes(classes=None) -> None:
    """Time only the named kernel classes while timing is on (None: every class)."""
    if classes is None:
        mask = (1 << len(TIMING_CLASSES)) - 1
    else:
        mask = 0
        for c in classes:
            mask |= 1 << TIMING_CLASSES.index(c)
    _check(_lib.lib().aaq_timing_classes(mask))


def aaq_timing_read(reset: bool = True) -> dict:
    """{class: {"launches", "total_ms", "bytes"}} accumulated since the last reset."""
    arr = (_lib.CKernelTiming * 16)()
    cnt = ctypes.c_int()
    _check(_lib.lib().aaq_timing_read(arr, 16, ctypes.byref(cnt), int(bool(reset))))
    return {arr[k].name.decode(): {"launches": int(arr[k].launches), "total_ms": float(arr[k].total_ms),
                                   "bytes": float(arr[k].bytes)} for k in range(min(cnt.value, 16))}


# ------------------------------------------------------------------ conveniences
class Estimator:
    """Owns the device buffers (torch) for repeated evaluations of one instance."""

    def __init__(self, prob: Problem, p: int, obs: int = AAQ_OBS_HRED, prec: int = AAQ_PREC_C64, grad: bool = True,
                 agg: int = AAQ_AGG_FUSED, device: str = "cuda", checkpoint: bool = False):
        """checkpoint=True: gradients use aaq_energy_grad_checkpointed (the state buffer then
        holds the forward states, aaq_checkpoint_bytes)."""
        import torch

        self.prob, self.p, self.obs, self.prec, self.agg = prob, int(p), obs, prec, agg
        self.checkpoint = bool(checkpoint and grad)
        sb = aaq_state_bytes(prob, prec)
        if self.checkpoint:
            sb = max(sb, aaq_checkpoint_bytes(prob, p, prec))
        # large enough for either observable, so one Estimator serves H_C and H_red
        wb = max(max(aaq_workspace_size(prob, p, grad, o, AAQ_AGG_FUSED, prec),
                     aaq_workspace_size(prob, p, False, o, agg, prec)) for o in (AAQ_OBS_HC, AAQ_OBS_HRED))
        self.state = torch.empty(sb, dtype=torch.uint8, device=device)
        self.lam = torch.empty(sb, dtype=torch.uint8, device=device) if grad else None
        self.ws = torch.empty(wb, dtype=torch.uint8, device=device)

    def energy(self, gamma, beta, obs: Optional[int] = None, agg: Optional[int] = None, stream=None):
        return aaq_energy(self.prob, gamma, beta, self.obs if obs is None else obs, self.agg if agg is None else agg,
                          self.prec, self.state, self.ws, stream)

    def energy_grad(self, gamma, beta, obs: Optional[int] = None, stream=None):
        if self.lam is None:
            raise ValueError("Estimator was built without gradient buffers")
        if self.checkpoint:
            return aaq_energy_grad_checkpointed(self.prob, gamma, beta, self.obs if obs is None else obs, self.prec,
                                                self.state, self.lam, self.ws, stream)
        return aaq_energy_grad(self.prob, gamma, beta, self.obs if obs is None else obs, self.prec, self.state,
                               self.lam, self.ws, stream)


class Plan:
    """Batched evaluation of many (instance, parameter point) units."""

    def __init__(self, probs: Sequence[Problem], p: int, obs: int = AAQ_OBS_HRED, with_grad: bool = True,
                 device: str = "cuda", stream=None, **opts):
        import torch

        self.count, self.p, self.with_grad = len(probs), int(p), with_grad
        self._probs = list(probs)
        wb = aaq_plan_workspace_size(self._probs, p, obs, with_grad, **opts)
        self.ws = torch.empty(wb, dtype=torch.uint8, device=device)
        self.handle = aaq_plan_create(self._probs, p, obs, with_grad, self.ws, stream, **opts)
        self.params = torch.zeros(self.count, 2 * self.p, dtype=torch.float64, device=device)
        self.out = torch.zeros(self.count, 2 + 2 * self.p, dtype=torch.float64, device=device)

    @staticmethod
    def autotuned(probs: Sequence[Problem], p: int, obs: int = AAQ_OBS_HRED, with_grad: bool = True, params=None,
                  reps: int = 3, device: str = "cuda", **base) -> "Plan":
        """A plan built with the options aaq_plan_autotune measures fastest for these units
        (parameters: a [count][2p] float64 tensor or array, default all 0.5)."""
        import itertools

        import torch

        probs = list(probs)
        cands = itertools.product((12, 13), (10, 12, 13))
        wb = max(aaq_plan_workspace_size(probs, p, obs, with_grad, **dict(base, tile_bits_large=tl,
                                                                          min_tile_bits_small=ts))
                 for tl, ts in cands)
        ws = torch.empty(wb, dtype=torch.uint8, device=device)
        prm = torch.full((len(probs), 2 * p), 0.5, dtype=torch.float64, device=device)
        if params is not None:
            prm.copy_(torch.as_tensor(params, dtype=torch.float64))
        out = torch.zeros(len(probs), 2 + 2 * p, dtype=torch.float64, device=device)
        opts, ms = aaq_plan_autotune(probs, p, obs, with_grad, ws, prm, out, reps=reps, **base)
        del ws
        plan = Plan(probs, p, obs, with_grad, device=device, **opts)
        plan.tuned_opts, plan.tuned_ms = opts, ms
        return plan

    def execute(self, stream=None, params=None, out=None):
        aaq_plan_execute(self.handle, self.params if params is None else params, self.out if out is None else out,
                         stream)
        return self.out if out is None else out

    def close(self):
        if self.handle:
            aaq_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class LightCone:
    """Light-cone evaluation of one instance (aaq_lightcone_*): owns the workspace and
    the parameter / output buffers (torch)."""

    def __init__(self, prob: Problem, p: int, obs: int = AAQ_OBS_HRED, with_grad: bool = True, device: str = "cuda",
                 stream=None, **opts):
        import torch

        self.prob, self.p, self.obs, self.with_grad = prob, int(p), obs, with_grad
        self.units, self.max_qubits, self.amplitudes = aaq_lightcone_info(prob, p, obs)
        wb = aaq_lightcone_workspace_size(prob, p, obs, with_grad, **opts)
        self.ws = torch.empty(wb, dtype=torch.uint8, device=device)
        self.handle = aaq_lightcone_create(prob, p, obs, with_grad, self.ws, stream, **opts)
        self.params = torch.zeros(2 * self.p, dtype=torch.float64, device=device)
        self.out = torch.zeros(2 + 2 * self.p, dtype=torch.float64, device=device)

    def execute(self, stream=None):
        aaq_lightcone_execute(self.handle, self.params, self.out, stream)
        return self.out

    def energy_grad(self, gamma, beta, stream=None):
        """Synchronous convenience: (energy, dE/dgamma, dE/dbeta, mean norm) as numpy."""
        import torch

        g, b = _params(gamma, beta)
        self.params.copy_(torch.from_numpy(np.concatenate([g, b])))
        o = self.execute(stream).cpu().numpy()
        return o[0], o[2:2 + self.p].copy(), o[2 + self.p:].copy(), o[1]

    def close(self):
        if self.handle:
            aaq_lightcone_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Sampler:
    """Final-state sampling of one instance (aaq_sample): owns the state, workspace and
    sample buffers (torch)."""

    def __init__(self, prob: Problem, p: int, shots: int, prec: int = AAQ_PREC_C64, device: str = "cuda"):
        import torch

        self.prob, self.p, self.shots, self.prec = prob, int(p), int(shots), prec
        self.state = torch.empty(aaq_state_bytes(prob, prec), dtype=torch.uint8, device=device)
        self.ws = torch.empty(aaq_sample_workspace_size(prob, p, prec), dtype=torch.uint8, device=device)
        self.uniform = torch.zeros(self.shots, dtype=torch.float64, device=device)
        self.samples = torch.zeros(self.shots, dtype=torch.int64, device=device)
        self.cuts = torch.zeros(self.shots, dtype=torch.int32, device=device)

    def sample(self, gamma, beta, uniform=None, stream=None):
        """(samples, cuts, best, mean); `uniform` (numpy or torch, length shots) is copied in
        when given, else the buffer's current contents are used."""
        import torch

        if uniform is not None:
            self.uniform.copy_(torch.as_tensor(np.asarray(uniform, dtype=np.float64)))
        best, mean = aaq_sample(self.prob, gamma, beta, self.prec, self.uniform, self.state, self.ws, self.samples,
                                self.cuts, stream)
        return self.samples.cpu().numpy().view(np.uint64), self.cuts.cpu().numpy(), best, mean


class Resident:
    """Device-resident evaluation of one instance (aaq_resident_*): owns the state, lambda
    and workspace buffers (torch).  ``execute(params, out)`` takes device float64 tensors
    [2p] (gamma then beta) and [2 + 2p] (energy, norm, dgamma, dbeta) and returns without
    synchronising."""

    def __init__(self, prob: Problem, p: int, obs: int = AAQ_OBS_HRED, with_grad: bool = True,
                 checkpoint: bool = False, prec: int = AAQ_PREC_C64, device: str = "cuda", stream=None):
        import torch

        self.prob, self.p, self.obs, self.with_grad = prob, int(p), obs, with_grad
        wb, sb = aaq_resident_workspace_size(prob, p, obs, with_grad, checkpoint, prec)
        self.state = torch.empty(sb, dtype=torch.uint8, device=device)
        self.lam = torch.empty(aaq_state_bytes(prob, prec), dtype=torch.uint8, device=device) if with_grad else None
        self.ws = torch.empty(wb, dtype=torch.uint8, device=device)
        self.handle = aaq_resident_create(prob, p, obs, with_grad, checkpoint, prec, self.state, self.lam, self.ws,
                                          stream)
        self.params = torch.zeros(2 * self.p, dtype=torch.float64, device=device)
        self.out = torch.zeros(2 + 2 * self.p, dtype=torch.float64, device=device)

    def execute(self, params=None, out=None, stream=None):
        o = self.out if out is None else out
        aaq_resident_execute(self.handle, self.params if params is None else params, o, stream)
        return o

    def energy_grad(self, gamma, beta, stream=None):
        """Synchronous convenience: (energy, dE/dgamma, dE/dbeta, norm) as numpy."""
        import torch

        g, b = _params(gamma, beta)
        self.params.copy_(torch.from_numpy(np.concatenate([g, b])))
        o = self.execute(stream=stream).cpu().numpy()
        return o[0], o[2:2 + self.p].copy(), o[2 + self.p:].copy(), o[1]

    def close(self):
        if self.handle:
            aaq_resident_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
