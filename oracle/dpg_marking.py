"""Plain CPU oracle of the Dörfler marking that drives the paper's adaptive
refinement (§4.2, the Fichera case, and its refinement table: refinement
fraction 0.30, coarsening fraction 0.05).

TEST INFRASTRUCTURE ONLY.  Only ``tests/`` may import this module.  It shares
no code with the HIP library.

Cells are ranked by their indicator (the residual norm of each cell, or any
nonnegative per-cell value the caller passes, e.g. its square).  Reading of
the rule:
  * ranking: decreasing value, equal values by increasing cell index;
  * refinement: the shortest prefix of the ranking whose sum reaches
    refine_fraction of the total, i.e. cell i (at position j) is refined
    when the sum of the values ranked before it is below refine_fraction T;
  * coarsening: taken from the other end, the longest run of the smallest
    values whose sum stays within coarsen_fraction of the total, i.e. a cell
    is coarsened when T minus the sum ranked before it is at most
    coarsen_fraction T (and it is not refined);
  * sums run in ranking order, the total T being the sum of all of them.
Returns one flag per cell: +1 refine, -1 coarsen, 0 keep.
"""
from __future__ import annotations

import numpy as np


def dorfler_mark(values, refine_fraction: float, coarsen_fraction: float):
    v = [float(x) for x in values]
    n = len(v)
    order = sorted(range(n), key=lambda i: (-v[i], i))
    total = 0.0
    for i in order:
        total += v[i]
    flags = np.zeros(n, np.int8)
    before = 0.0
    for i in order:
        if before < refine_fraction * total:
            flags[i] = 1
        elif total - before <= coarsen_fraction * total:
            flags[i] = -1
        before += v[i]
    return flags
