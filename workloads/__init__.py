"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This package builds graphs, their Aut(G) edge orbits and parameter arrays.  It
holds none of the method's arithmetic (no state evolution, no expectation); the
orbit finder is the host-side preprocessing that precedes the estimator
(Algorithm 1 of the paper).
"""
from .graphs import Graph  # noqa: F401
