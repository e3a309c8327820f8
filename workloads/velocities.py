"""Discrete velocity sets, used here only to name link directions.

A cut link is identified by (fluid node, direction index i); the index refers
to the velocity orderings below, which the oracle and the HIP library each
define again in their own tables (a test checks that all three agree).

* D2Q9: the ordering printed in the paper's Appendix (D2Q9 model).
* D3Q19: rest, the six axis vectors, then the twelve edge vectors, in the
  ordering of d'Humieres et al. (2002), the reference the paper cites for
  its 3D MRT models.
* D3Q15: the ordering printed in the paper's Appendix (D3Q15 model).
"""

import numpy as np

_D2Q9 = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1),
         (1, 1), (-1, 1), (-1, -1), (1, -1)]

_D3Q19 = [(0, 0, 0),
          (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
          (1, 1, 0), (-1, 1, 0), (1, -1, 0), (-1, -1, 0),
          (1, 0, 1), (-1, 0, 1), (1, 0, -1), (-1, 0, -1),
          (0, 1, 1), (0, -1, 1), (0, 1, -1), (0, -1, -1)]

_D3Q15 = [(0, 0, 0),
          (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
          (1, 1, 1), (-1, 1, 1), (1, -1, 1), (-1, -1, 1),
          (1, 1, -1), (-1, 1, -1), (1, -1, -1), (-1, -1, -1)]

VELOCITIES = {
    "D2Q9": np.array(_D2Q9, dtype=np.int64),
    "D3Q19": np.array(_D3Q19, dtype=np.int64),
    "D3Q15": np.array(_D3Q15, dtype=np.int64),
}


def opposite(lattice):
    """Index map i -> i-bar with e_{i-bar} = -e_i."""
    e = VELOCITIES[lattice]
    out = np.empty(len(e), dtype=np.int64)
    for i, v in enumerate(e):
        out[i] = int(np.nonzero((e == -v).all(axis=1))[0][0])
    return out


def dim(lattice):
    return VELOCITIES[lattice].shape[1]
