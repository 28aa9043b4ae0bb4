"""MI355X (gfx950) exact maximum clique for large sparse graphs.

A from-scratch GPU implementation of the method of Rossi, Gleich, Gebremedhin
and Patwary (arXiv 1302.6256): k-core peeling, the greedy heuristic clique,
core-number pruning of every neighbourhood, and per-vertex branch and bound
with colouring bounds and a shared bound.  The compute path is the C-ABI
library ``libpmc.so`` (HIP kernels, see ``csrc/``); ``pmc`` is its binding.
"""
from . import pmc  # noqa: F401
from .pmc import core_numbers, heuristic, max_clique, prune_orient  # noqa: F401
