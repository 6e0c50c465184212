"""Triangle quadrature rules in barycentric coordinates (weights sum to 1;
multiply by the triangle area).

* ``RULE7``: Radon's 7-point rule, exact for polynomials of degree <= 5
  (Stroud T2:5-1): the centroid with weight 9/40 and two orbits of three
  points built from (6 -+ sqrt 15)/21 with weights (155 -+ sqrt 15)/1200.
* ``RULE3``: 3-point rule at (2/3, 1/6, 1/6) and permutations, weights 1/3,
  exact for degree <= 2.
"""

import math

import numpy as np


def _rule7():
    s15 = math.sqrt(15.0)
    a1 = (6.0 - s15) / 21.0
    b1 = 1.0 - 2.0 * a1
    w1 = (155.0 - s15) / 1200.0
    a2 = (6.0 + s15) / 21.0
    b2 = 1.0 - 2.0 * a2
    w2 = (155.0 + s15) / 1200.0
    bary = [(1 / 3, 1 / 3, 1 / 3),
            (b1, a1, a1), (a1, b1, a1), (a1, a1, b1),
            (b2, a2, a2), (a2, b2, a2), (a2, a2, b2)]
    w = [9.0 / 40.0, w1, w1, w1, w2, w2, w2]
    return np.array(bary), np.array(w)


def _rule3():
    bary = [(2 / 3, 1 / 6, 1 / 6), (1 / 6, 2 / 3, 1 / 6), (1 / 6, 1 / 6, 2 / 3)]
    return np.array(bary), np.full(3, 1.0 / 3.0)


RULE7 = _rule7()
RULE3 = _rule3()


def points(tv, rule):
    """Quadrature points for triangles tv (K, 3, 3): returns (K, q, 3)."""
    bary, _ = rule
    return np.einsum("qi,kid->kqd", bary, tv)
