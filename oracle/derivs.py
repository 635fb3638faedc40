"""Derivative drivers around the FP64 oracle (TEST INFRASTRUCTURE ONLY).

* ``central_fd``: (E(theta + h e_k) - E(theta - h e_k)) / (2h).
* ``layer_shift``: the general parameter-shift rule for a parameter whose
  generator has integer spectrum differences 1..R (Wierichs, Izaac, Wang, Lin,
  Quantum 6, 677 (2022)):
      f'(x) = sum_{mu=1}^{2R} f(x + x_mu) (-1)^(mu-1) / (4 R sin^2(x_mu / 2)),
      x_mu = (2 mu - 1) pi / (2R).
  For gamma_l the generator H_C has integer eigenvalues 0..|E| (R = |E|); for
  beta_l the generator sum X has eigenvalues n - 2k, so in x = 2 beta the
  frequencies are 1..n (R = n) and dE/dbeta = 2 df/dx.
* ``per_gate_shift``: every cost gate e^{-i gamma [z_u != z_v]} (frequency 1)
  and every mixer gate e^{-i beta X_q} (frequency 2) shifted on its own, using a
  separate small NumPy simulator with one angle per gate (n <= 14).  That
  simulator is a second, independent implementation of the ansatz.
"""
from __future__ import annotations

import math
from typing import Callable

import numpy as np

from . import energy as _energy


def central_fd(f: Callable[[np.ndarray, np.ndarray], float], gamma, beta, h: float = 1e-4):
    gamma = np.asarray(gamma, dtype=np.float64).reshape(-1)
    beta = np.asarray(beta, dtype=np.float64).reshape(-1)
    p = gamma.shape[0]
    dg = np.zeros(p)
    db = np.zeros(p)
    for k in range(p):
        e = np.zeros(p)
        e[k] = h
        dg[k] = (f(gamma + e, beta) - f(gamma - e, beta)) / (2 * h)
        db[k] = (f(gamma, beta + e) - f(gamma, beta - e)) / (2 * h)
    return dg, db


def shift_points(R: int):
    mu = np.arange(1, 2 * R + 1)
    x = (2 * mu - 1) * math.pi / (2 * R)
    coef = (-1.0) ** (mu - 1) / (4 * R * np.sin(x / 2) ** 2)
    return x, coef


def layer_shift(n: int, edges, terms, gamma, beta):
    """Gradient by the layer-level general parameter-shift rule (plain energy calls)."""
    gamma = np.asarray(gamma, dtype=np.float64).reshape(-1)
    beta = np.asarray(beta, dtype=np.float64).reshape(-1)
    p = gamma.shape[0]
    m = int(np.asarray(edges).reshape(-1, 2).shape[0])
    E = lambda g, b: _energy(n, edges, terms, g, b)
    dg = np.zeros(p)
    db = np.zeros(p)
    xg, cg = shift_points(max(m, 1))
    xb, cb = shift_points(n)
    for k in range(p):
        for x, c in zip(xg, cg):
            g = gamma.copy()
            g[k] += x
            dg[k] += c * E(g, beta)
        for x, c in zip(xb, cb):
            b = beta.copy()
            b[k] += x / 2
            db[k] += 2 * c * E(gamma, b)
    return dg, db


# ------------------------------------------------------------------ per-gate simulator
def _per_gate_energy(n, edges, terms, gam_gate, bet_gate):
    """gam_gate[l, e]: angle of edge e's cost gate in layer l; bet_gate[l, q]: mixer angle."""
    edges = np.asarray(edges).reshape(-1, 2)
    z = np.arange(1 << n)
    bits = (z[:, None] >> np.arange(n)[None, :]) & 1
    diff = [bits[:, u] != bits[:, v] for u, v in edges]
    psi = np.full(1 << n, 2.0 ** (-n / 2), dtype=np.complex128)
    for l in range(gam_gate.shape[0]):
        for e in range(edges.shape[0]):
            psi = psi * np.where(diff[e], np.exp(-1j * gam_gate[l, e]), 1.0)
        for q in range(n):
            c, s = math.cos(bet_gate[l, q]), math.sin(bet_gate[l, q])
            t = psi.reshape(1 << (n - 1 - q), 2, 1 << q)
            a, b = t[:, 0, :].copy(), t[:, 1, :].copy()
            t[:, 0, :] = c * a - 1j * s * b
            t[:, 1, :] = -1j * s * a + c * b
            psi = t.reshape(-1)
    ti, tj, tw = terms
    h = np.zeros(1 << n)
    for i, j, w in zip(ti, tj, tw):
        h += float(w) * (bits[:, int(i)] != bits[:, int(j)])
    return float(np.sum(np.abs(psi) ** 2 * h))


def per_gate_energy(n, edges, terms, gamma, beta):
    gamma = np.asarray(gamma, dtype=np.float64).reshape(-1)
    beta = np.asarray(beta, dtype=np.float64).reshape(-1)
    m = np.asarray(edges).reshape(-1, 2).shape[0]
    return _per_gate_energy(n, edges, terms, np.repeat(gamma[:, None], m, 1), np.repeat(beta[:, None], n, 1))


def per_gate_shift(n, edges, terms, gamma, beta):
    if n > 14:
        raise ValueError("per-gate simulator is meant for n <= 14")
    gamma = np.asarray(gamma, dtype=np.float64).reshape(-1)
    beta = np.asarray(beta, dtype=np.float64).reshape(-1)
    p = gamma.shape[0]
    m = np.asarray(edges).reshape(-1, 2).shape[0]
    G0 = np.repeat(gamma[:, None], m, 1)
    B0 = np.repeat(beta[:, None], n, 1)
    dg = np.zeros(p)
    db = np.zeros(p)
    for l in range(p):
        for e in range(m):
            Gp, Gm = G0.copy(), G0.copy()
            Gp[l, e] += math.pi / 2
            Gm[l, e] -= math.pi / 2
            dg[l] += 0.5 * (_per_gate_energy(n, edges, terms, Gp, B0) - _per_gate_energy(n, edges, terms, Gm, B0))
        for q in range(n):
            Bp, Bm = B0.copy(), B0.copy()
            Bp[l, q] += math.pi / 4
            Bm[l, q] -= math.pi / 4
            db[l] += _per_gate_energy(n, edges, terms, G0, Bp) - _per_gate_energy(n, edges, terms, G0, Bm)
    return dg, db
