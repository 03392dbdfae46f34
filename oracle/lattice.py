"""Velocity sets for the oracle (test infrastructure only).

D2Q9 follows eq. (VelocitySet) of Sec. II in the paper's order, with the
weights stated right after eq. (Single_Phase_EDF): 4/9, 1/9 (x4), 1/36 (x4),
c_s^2 = 1/3.

D3Q19 is the three-dimensional extension (not in the paper): weights 1/3,
1/18 (x6), 1/36 (x12).  Its direction order is an interface shared with the
GPU library's population layout: rest, then the six axis directions as
opposite pairs (+x, -x, +y, -y, +z, -z), then the twelve edge directions as
opposite pairs (xy plane, xz plane, yz plane).

Vectors are given as (c_x, c_y[, c_z]).  Field arrays are stored with the
spatial axes reversed, (y, x) in 2-D and (z, y, x) in 3-D, so that x is the
fastest-varying index as in the GPU library.
"""
import numpy as np


class Lattice:
    def __init__(self, name, c, w):
        self.name = name
        self.c = np.array(c, dtype=np.int64)
        self.w = np.array(w, dtype=np.float64)
        self.Q, self.d = self.c.shape
        self.cs2 = 1.0 / 3.0
        opp = []
        for i in range(self.Q):
            j = [k for k in range(self.Q) if np.array_equal(self.c[k], -self.c[i])]
            assert len(j) == 1
            opp.append(j[0])
        self.opp = np.array(opp, dtype=np.int64)

    def axis_of(self, alpha):
        """Array axis (in a field array) that carries velocity component alpha."""
        return self.d - 1 - alpha

    def __repr__(self):
        return self.name


D2Q9 = Lattice(
    "D2Q9",
    [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)],
    [4.0 / 9.0] + [1.0 / 9.0] * 4 + [1.0 / 36.0] * 4,
)

D3Q19 = Lattice(
    "D3Q19",
    [
        (0, 0, 0),
        (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
        (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
        (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
        (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1),
    ],
    [1.0 / 3.0] + [1.0 / 18.0] * 6 + [1.0 / 36.0] * 12,
)

LATTICES = {"D2Q9": D2Q9, "D3Q19": D3Q19}
