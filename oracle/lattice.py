"""D2Q49 lattice velocities and their numbering (oracle side).

The paper's D2Q49 set holds every lattice displacement with |v_x|, |v_y| <= 3
(Fig. 1b caption: the central node 0 and the vectors to the surrounding
nodes; its "0 to 49" is read as the 49 indices 0..48).  The numbering figure is
missing, so this oracle fixes it by a rule that reproduces the six D2Q25 sets
the Results section lists (0 | 1-4 | 5-8 | 9-12 | 13-20 | 21-24, one
displacement length each): sort by |v|^2, then by polar angle measured
counter-clockwise from +x in [0, 2 pi).
"""
from __future__ import annotations

import math

import numpy as np

NQ = 49
OVERFLOW = 49


def d2q49() -> np.ndarray:
    """[49, 2] int32 table of (v_x, v_y) in the oracle's numbering."""
    vs = [(vx, vy) for vx in range(-3, 4) for vy in range(-3, 4)]

    def key(v):
        ang = math.atan2(v[1], v[0])
        if ang < 0:
            ang += 2 * math.pi
        return (v[0] * v[0] + v[1] * v[1], ang)

    vs.sort(key=key)
    return np.ascontiguousarray(np.array(vs, dtype=np.int32))


def shells(table: np.ndarray | None = None):
    """List of index arrays, one per |v|^2 shell, in ascending |v|^2."""
    t = d2q49() if table is None else table
    r2 = t[:, 0] ** 2 + t[:, 1] ** 2
    return [np.nonzero(r2 == v)[0] for v in sorted(set(r2.tolist()))]
