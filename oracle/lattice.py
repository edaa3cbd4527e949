"""D3Q19 velocity set and weights (paper, Sec. II, Eq. (2): the LB equation is
written on the D3Q19 lattice, the fourth-order-isotropic 19-velocity model).

Directions: the rest vector, the 6 face neighbours and the 12 edge
neighbours; weights 1/3, 1/18 and 1/36; speed of sound squared 1/3.
Opposite directions are adjacent (1<->2, 3<->4, ...)."""
from fractions import Fraction

import numpy as np

C = np.array([
    (0, 0, 0),
    (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
    (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
    (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
    (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1),
], dtype=np.int64)

W_EXACT = [Fraction(1, 3)] + [Fraction(1, 18)] * 6 + [Fraction(1, 36)] * 12
W = np.array([float(w) for w in W_EXACT])
CS2 = 1.0 / 3.0
Q = 19
OPP = np.array([0] + [i + 1 if i % 2 == 1 else i - 1 for i in range(1, Q)], dtype=np.int64)
