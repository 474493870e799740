"""Float inputs whose FP64 squared distances tie only when every product and
every sum is rounded on its own.

For the query (c, c) the points A = (x, y) and B = (y, x) have the same two
rounded squares, so the index-order sums fl(fl(tx^2) + fl(ty^2)) and
fl(fl(ty^2) + fl(tx^2)) are equal and the top K orders the pair by id.  A
fused multiply-add in the second step (fl(fl(tx^2) + ty^2) against
fl(fl(ty^2) + tx^2), computed here in exact rational arithmetic) separates
them; the pairs kept are those where it does, with the id order set against
the fused order, so an implementation that fuses ranks the pair the other way.
"""
from fractions import Fraction

import numpy as np


def _fused_second_step(first_sq: float, t: float) -> float:
    return float(Fraction(first_sq) + Fraction(t) * Fraction(t))


def tie_pairs(seed: int, c: float, npairs: int, tries: int = 4000):
    """npairs (first, second) float32 points of two coordinates, in id order, or
    None when `tries` draws do not find them (some c leave every square exact)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(tries):
        if len(out) == npairs:
            break
        x, y = (float(v) for v in rng.uniform(0.25, 1.0, 2).astype(np.float32))
        tx, ty = x - c, y - c
        fa = _fused_second_step(tx * tx, ty)  # A = (x, y) with a fused second step
        fb = _fused_second_step(ty * ty, tx)  # B = (y, x)
        if fa == fb:
            continue
        a_pt, b_pt = (x, y), (y, x)
        # the smaller id gets the larger fused value
        out.append((b_pt, a_pt) if fa < fb else (a_pt, b_pt))
    return out if len(out) == npairs else None


def tie_workload(seed: int = 17, nq: int = 3, npairs: int = 4):
    """(data float32 [2 * nq * npairs, 2], queries float32 [nq, 2]); query j is
    (c_j, c_j) with c_j in [0.01, 0.1), and its pairs separate under fusion."""
    rng = np.random.default_rng(seed)
    cs, rows = [], []
    while len(cs) < nq:
        c = rng.uniform(0.01, 0.1, 1).astype(np.float32)[0]
        pairs = tie_pairs(seed * 100 + len(cs), float(c), npairs)
        if pairs is None:
            continue
        cs.append(c)
        for first, second in pairs:
            rows += [first, second]
    cs = np.asarray(cs, dtype=np.float32)
    data = np.asarray(rows, dtype=np.float32)
    queries = np.stack([cs, cs], axis=1).astype(np.float32)
    return data, queries
