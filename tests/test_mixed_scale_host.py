"""The mixed-scale scene reaches every tier of the broad-phase hash at the
default cell size (2 x the mean primitive box extent): primitives within
64 cells (one thread each), primitives of more than 64 but at most 4096
cells and at most 64 cells per axis (one wavefront each), and primitives
wider than 64 cells on some axis (tested against every query)."""
import numpy as np

import oracle as O
from scenes import mixed_scale_scene


def _spans(sc, idx, cs):
    x = O.embed(sc, sc.q)
    x1 = O.embed(sc, sc.q + sc.dq)
    h = 0.5 * sc.dhat
    p = np.concatenate([x[idx], x1[idx]], axis=1)
    lo, hi = p.min(axis=1) - h, p.max(axis=1) + h
    cell = cs * (hi - lo).sum(axis=0).max() / len(idx)
    return np.floor(hi / cell) - np.floor(lo / cell) + 1


def test_mixed_scale_scene_reaches_every_hash_tier():
    sc = mixed_scale_scene()
    for idx in (sc.faces, sc.edges):
        s = _spans(sc, idx, 2.0)
        n = s.prod(axis=1)
        small = n <= 64
        huge = (s > 64).any(axis=1) | (n > 4096)
        big = ~small & ~huge
        assert small.sum() > 1000 and big.sum() >= 4 and huge.sum() >= 1
