"""Velocity sets, weights and MRT moment matrices.

D2Q9: velocities, weights and M exactly as printed in the paper's Appendix
(D2Q9 model, M of Lallemand and Luo).  D3Q15: as printed in the Appendix.
D3Q19: not in the paper; velocities and weights are the standard D3Q19 set
and the rows of M are the moment polynomials of d'Humieres et al. (2002),
the reference the paper cites for its 3D MRT models.  Pinned by the
orthogonality of M, the diagonal of M M^T, and the weight moments
sum w = 1, sum w e_a e_b = delta_ab / 3 (tests/test_oracle_lattice.py).
"""

from dataclasses import dataclass
import numpy as np


@dataclass(frozen=True)
class Lattice:
    name: str
    e: np.ndarray        # (Q, D) int
    w: np.ndarray        # (Q,) float64
    M: np.ndarray        # (Q, Q) float64

    @property
    def Q(self):
        return self.e.shape[0]

    @property
    def D(self):
        return self.e.shape[1]

    @property
    def opp(self):
        out = np.empty(self.Q, dtype=np.int64)
        for i in range(self.Q):
            out[i] = int(np.nonzero((self.e == -self.e[i]).all(1))[0][0])
        return out

    @property
    def Minv(self):
        return np.linalg.inv(self.M)


def _d2q9():
    e = np.array([[0, 1, 0, -1, 0, 1, -1, -1, 1],
                  [0, 0, 1, 0, -1, 1, 1, -1, -1]], dtype=np.int64).T
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    M = np.array([
        [1, 1, 1, 1, 1, 1, 1, 1, 1],
        [-4, -1, -1, -1, -1, 2, 2, 2, 2],
        [4, -2, -2, -2, -2, 1, 1, 1, 1],
        [0, 1, 0, -1, 0, 1, -1, -1, 1],
        [0, -2, 0, 2, 0, 1, -1, -1, 1],
        [0, 0, 1, 0, -1, 1, 1, -1, -1],
        [0, 0, -2, 0, 2, 1, 1, -1, -1],
        [0, 1, -1, 1, -1, 0, 0, 0, 0],
        [0, 0, 0, 0, 0, 1, -1, 1, -1]], dtype=np.float64)
    return Lattice("D2Q9", e, w, M)


def _d3q15():
    e = np.array([
        [0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1],
        [0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1],
        [0, 0, 0, 0, 0, 1, -1, 1, 1, 1, 1, -1, -1, -1, -1]], dtype=np.int64).T
    w = np.array([2 / 9] + [1 / 9] * 6 + [1 / 72] * 8)
    M = np.array([
        [1] * 15,
        [-2, -1, -1, -1, -1, -1, -1, 1, 1, 1, 1, 1, 1, 1, 1],
        [16, -4, -4, -4, -4, -4, -4, 1, 1, 1, 1, 1, 1, 1, 1],
        [0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1],
        [0, -4, 4, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1],
        [0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1],
        [0, 0, 0, -4, 4, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1],
        [0, 0, 0, 0, 0, 1, -1, 1, 1, 1, 1, -1, -1, -1, -1],
        [0, 0, 0, 0, 0, -4, 4, 1, 1, 1, 1, -1, -1, -1, -1],
        [0, 2, 2, -1, -1, -1, -1, 0, 0, 0, 0, 0, 0, 0, 0],
        [0, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 0, 0, 0, 0],
        [0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1],
        [0, 0, 0, 0, 0, 0, 0, 1, 1, -1, -1, -1, -1, 1, 1],
        [0, 0, 0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, -1, 1],
        [0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1, -1, 1, 1, -1]], dtype=np.float64)
    return Lattice("D3Q15", e, w, M)


def _d3q19():
    e = np.array([(0, 0, 0),
                  (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
                  (1, 1, 0), (-1, 1, 0), (1, -1, 0), (-1, -1, 0),
                  (1, 0, 1), (-1, 0, 1), (1, 0, -1), (-1, 0, -1),
                  (0, 1, 1), (0, -1, 1), (0, 1, -1), (0, -1, -1)], dtype=np.int64)
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    ex, ey, ez = (e[:, a].astype(np.float64) for a in range(3))
    e2 = ex * ex + ey * ey + ez * ez
    rows = [
        np.ones(19),
        19 * e2 - 30,
        (21 * e2 * e2 - 53 * e2 + 24) / 2,
        ex, (5 * e2 - 9) * ex,
        ey, (5 * e2 - 9) * ey,
        ez, (5 * e2 - 9) * ez,
        3 * ex * ex - e2, (3 * e2 - 5) * (3 * ex * ex - e2),
        ey * ey - ez * ez, (3 * e2 - 5) * (ey * ey - ez * ez),
        ex * ey, ey * ez, ex * ez,
        (ey * ey - ez * ez) * ex, (ez * ez - ex * ex) * ey, (ex * ex - ey * ey) * ez,
    ]
    M = np.array(rows, dtype=np.float64)
    return Lattice("D3Q19", e, w, M)


LATTICES = {"D2Q9": _d2q9(), "D3Q15": _d3q15(), "D3Q19": _d3q19()}


def get(name):
    return LATTICES[name]
