"""FP64 CPU oracle for MaxCut QAOA statevector simulation.

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this package; the library and its
Python binding never do.  The oracle shares no code with the HIP path.

``qaoa_oracle.c`` holds the full-state FP64 simulator (cut values, ansatz,
per-term <ZZ>, energy, plain adjoint gradient).  ``reduced.py`` holds the
independent reduced formulations used to pin it (p = 1 closed form, Dicke
subspace of K_n, hub x Dicke subspace of the star, light cone), and
``derivs.py`` the finite-difference and parameter-shift drivers.

Every function is pinned by a ``-m "not gpu"`` test except where a docstring
says "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None


def lib():
    """Load liboracle.so, building it with gcc if it is not there yet (ORACLE_LIB names
    another build of the same source, e.g. a sanitizer build from ``oracle/build.py``)."""
    global _LIB
    if _LIB is None:
        path = os.environ.get("ORACLE_LIB") or _build.LIB
        if path == _build.LIB and not os.path.exists(path):
            _build.build()
        L = ctypes.CDLL(path)
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        dptr = ctypes.POINTER(ctypes.c_double)
        ci = ctypes.c_int
        wp = ctypes.c_void_p  # optional int32 weights (NULL: all 1)
        L.orc_cut_values.argtypes = [ci, ci, i32p, wp, i32p]
        L.orc_term_values.argtypes = [ci, ci, i32p, i32p, f64p, f64p]
        L.orc_state.argtypes = [ci, ci, i32p, wp, ci, f64p, f64p, f64p]
        L.orc_zz.argtypes = [ci, f64p, ci, i32p, i32p, f64p]
        L.orc_energy.argtypes = [ci, ci, i32p, wp, ci, i32p, i32p, f64p, ci, f64p, f64p, dptr, dptr, f64p, dptr]
        L.orc_energy_grad.argtypes = [ci, ci, i32p, wp, ci, i32p, i32p, f64p, ci, f64p, f64p, dptr, f64p, f64p,
                                      dptr]
        L.orc_num_threads.argtypes = []
        L.orc_set_num_threads.argtypes = [ci]
        L.orc_set_num_threads.restype = None
        for f in ("orc_cut_values", "orc_term_values", "orc_state", "orc_zz", "orc_energy", "orc_energy_grad",
                  "orc_num_threads"):
            getattr(L, f).restype = ci
        _LIB = L
    return _LIB


def _edges(edges) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))


def _weights(weights, m):
    """(keep-alive array, pointer) of the int32 edge weights, or (None, None) for all 1."""
    if weights is None:
        return None, None
    w = np.ascontiguousarray(np.asarray(weights, dtype=np.int32).reshape(-1))
    if w.shape[0] != m:
        raise ValueError("one weight per edge")
    return w, w.ctypes.data_as(ctypes.c_void_p)


def _terms(terms):
    ti, tj, tw = terms
    return (np.ascontiguousarray(np.asarray(ti, dtype=np.int32)),
            np.ascontiguousarray(np.asarray(tj, dtype=np.int32)),
            np.ascontiguousarray(np.asarray(tw, dtype=np.float64)))


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(t: int) -> None:
    """Thread count of the oracle's parallel loops from now on."""
    lib().orc_set_num_threads(int(t))


def cut_values(n: int, edges, weights=None) -> np.ndarray:
    """C(z) = sum_e w_e [z_u != z_v] for every z in [0, 2^n), by looping over the edges
    (w_e = 1 unless integer ``weights`` are given: the MaxCut H_P with its w_ij)."""
    e = _edges(edges)
    w, wp = _weights(weights, e.shape[0])
    out = np.empty(1 << n, dtype=np.int32)
    rc = lib().orc_cut_values(n, e.shape[0], e, wp, out)
    if rc != 0:
        raise ValueError("orc_cut_values failed")
    return out


def cut_values_at(z, edges, weights=None) -> np.ndarray:
    """C(z) = sum_e w_e [z_u != z_v] at the given indices only (any shape, n <= 64), edge by
    edge in numpy: the values a state too large for the full table is checked on."""
    z = np.asarray(z, dtype=np.uint64)
    e = _edges(edges)
    w, _ = _weights(weights, e.shape[0])
    if w is None:
        w = np.ones(e.shape[0], dtype=np.int32)
    out = np.zeros(z.shape, dtype=np.int64)
    for (u, v), we in zip(e.reshape(-1, 2), w):
        out += int(we) * (((z >> np.uint64(u)) ^ (z >> np.uint64(v))) & np.uint64(1)).astype(np.int64)
    return out


def term_values_at(z, terms) -> np.ndarray:
    """h(z) = sum_t w_t [z_i != z_j] at the given indices only."""
    z = np.asarray(z, dtype=np.uint64)
    ti, tj, tw = _terms(terms)
    out = np.zeros(z.shape, dtype=np.float64)
    for i, j, w in zip(ti, tj, tw):
        out += float(w) * (((z >> np.uint64(i)) ^ (z >> np.uint64(j))) & np.uint64(1)).astype(np.float64)
    return out


def term_values(n: int, terms) -> np.ndarray:
    """h(z) = sum_t w_t [z_i != z_j] for every z."""
    ti, tj, tw = _terms(terms)
    out = np.empty(1 << n, dtype=np.float64)
    rc = lib().orc_term_values(n, ti.shape[0], ti, tj, tw, out)
    if rc != 0:
        raise ValueError("orc_term_values failed")
    return out


def state(n: int, edges, gamma, beta, weights=None) -> np.ndarray:
    """The p-layer QAOA state as a complex128 vector of length 2^n (cost phase
    exp(-i gamma C(z)) with the weighted cut when ``weights`` are given)."""
    e = _edges(edges)
    w, wp = _weights(weights, e.shape[0])
    g = np.ascontiguousarray(np.asarray(gamma, dtype=np.float64).reshape(-1))
    b = np.ascontiguousarray(np.asarray(beta, dtype=np.float64).reshape(-1))
    out = np.empty(2 << n, dtype=np.float64)
    rc = lib().orc_state(n, e.shape[0], e, wp, g.shape[0], g, b, out)
    if rc != 0:
        raise ValueError("orc_state failed")
    return out.view(np.complex128)


def sample(n: int, edges, gamma, beta, uniform, weights=None):
    """Final-state sampling by inverse CDF (the paper's read-out of the QAOA state): for
    each u in [0, 1), the smallest integer z with CDF(z) > u, where CDF(z) is the FP64
    running sum of |psi(y)|^2 over y <= z divided by the total.  Returns (z, C(z), CDF)."""
    psi = state(n, edges, gamma, beta, weights)
    cdf = np.cumsum(np.abs(psi) ** 2)
    cdf /= cdf[-1]
    u = np.clip(np.asarray(uniform, dtype=np.float64), 0.0, np.nextafter(1.0, 0.0))
    z = np.minimum(np.searchsorted(cdf, u, side="right"), (1 << n) - 1)
    return z.astype(np.uint64), cut_values(n, edges, weights)[z], cdf


def zz(n: int, psi: np.ndarray, terms) -> np.ndarray:
    ti, tj, _ = _terms(terms)
    buf = np.ascontiguousarray(psi.astype(np.complex128)).view(np.float64)
    out = np.empty(ti.shape[0], dtype=np.float64)
    lib().orc_zz(n, buf, ti.shape[0], ti, tj, out)
    return out


def energy(n: int, edges, terms, gamma, beta, full: bool = False, weights=None):
    """<H> for the observable given by ``terms`` = (i, j, w): sum_t (w_t/2)(1 - <Z_i Z_j>_t).

    With ``full`` also returns the direct route sum_z |psi|^2 h(z), the per-term
    <ZZ> vector and the norm.  ``weights``: integer edge weights of the cost phase."""
    e = _edges(edges)
    w, wp = _weights(weights, e.shape[0])
    ti, tj, tw = _terms(terms)
    g = np.ascontiguousarray(np.asarray(gamma, dtype=np.float64).reshape(-1))
    b = np.ascontiguousarray(np.asarray(beta, dtype=np.float64).reshape(-1))
    et, ed, nrm = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    zzv = np.zeros(max(ti.shape[0], 1), dtype=np.float64)
    rc = lib().orc_energy(n, e.shape[0], e, wp, ti.shape[0], ti, tj, tw, g.shape[0], g, b, ctypes.byref(et),
                          ctypes.byref(ed), zzv, ctypes.byref(nrm))
    if rc != 0:
        raise ValueError("orc_energy failed")
    if full:
        return et.value, ed.value, zzv[: ti.shape[0]].copy(), nrm.value
    return et.value


def energy_grad(n: int, edges, terms, gamma, beta, with_dev: bool = False, weights=None):
    """(energy, dE/dgamma[p], dE/dbeta[p]) by the plain FP64 adjoint sweep (``weights``:
    integer edge weights of the cost phase)."""
    e = _edges(edges)
    w, wp = _weights(weights, e.shape[0])
    ti, tj, tw = _terms(terms)
    g = np.ascontiguousarray(np.asarray(gamma, dtype=np.float64).reshape(-1))
    b = np.ascontiguousarray(np.asarray(beta, dtype=np.float64).reshape(-1))
    p = g.shape[0]
    en, dev = ctypes.c_double(), ctypes.c_double()
    dg = np.zeros(p, dtype=np.float64)
    db = np.zeros(p, dtype=np.float64)
    rc = lib().orc_energy_grad(n, e.shape[0], e, wp, ti.shape[0], ti, tj, tw, p, g, b, ctypes.byref(en), dg, db,
                               ctypes.byref(dev))
    if rc != 0:
        raise ValueError("orc_energy_grad failed")
    if with_dev:
        return en.value, dg, db, dev.value
    return en.value, dg, db
