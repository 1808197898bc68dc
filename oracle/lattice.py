"""Velocity sets of the paper (Sec. 2.1: first-neighbour stencils built on third-order
quadrature, D2Q9 and D3Q27) and the lattice sound speed c_s = dr/(sqrt(3) dt) with
dr = dt = 1, so c_s^2 = 1/3.

Population ordering is the library's interface format: index i of velocity
(cx, cy, cz) is (cx+1) + 3 (cy+1) + 9 (cz+1)  (D2Q9: cz = 0, i = (cx+1) + 3 (cy+1)).
The opposite of i is Q-1-i.
"""
import itertools

import torch

CS2 = 1.0 / 3.0

# Quadrature weights by speed class (number of non-zero velocity components).
_W2 = {0: 4.0 / 9.0, 1: 1.0 / 9.0, 2: 1.0 / 36.0}
_W3 = {0: 8.0 / 27.0, 1: 2.0 / 27.0, 2: 1.0 / 54.0, 3: 1.0 / 216.0}


class Lattice:
    """c: (Q, D) float64 velocities, w: (Q,) weights, opp: (Q,) opposite index."""

    def __init__(self, name):
        self.name = name
        if name == "D2Q9":
            self.D = 2
            vel = [(cx, cy) for cy in (-1, 0, 1) for cx in (-1, 0, 1)]
            w = [_W2[sum(1 for a in v if a != 0)] for v in vel]
        elif name == "D3Q27":
            self.D = 3
            vel = [(cx, cy, cz) for cz in (-1, 0, 1) for cy in (-1, 0, 1) for cx in (-1, 0, 1)]
            w = [_W3[sum(1 for a in v if a != 0)] for v in vel]
        else:
            raise ValueError(name)
        self.Q = len(vel)
        self.c = torch.tensor(vel, dtype=torch.float64)
        self.ci = torch.tensor(vel, dtype=torch.int64)
        self.w = torch.tensor(w, dtype=torch.float64)
        self.opp = torch.tensor(
            [vel.index(tuple(-a for a in v)) for v in vel], dtype=torch.int64)
        # Moment exponents (a, b[, c]) with every exponent in {0, 1, 2}: Q of them, the
        # complete moment basis of a first-neighbour tensor-product velocity set.
        self.exps = list(itertools.product(range(3), repeat=self.D))
        # Dense moment matrix M[j, i] = prod_d c_{i,d}^{a_{j,d}}  (Sec. 2.2, matrix M).
        M = torch.ones(self.Q, self.Q, dtype=torch.float64)
        for j, e in enumerate(self.exps):
            for d in range(self.D):
                M[j] *= self.c[:, d] ** e[d]
        self.M = M
        self.Minv = torch.linalg.inv(M)


D2Q9 = Lattice("D2Q9")
D3Q27 = Lattice("D3Q27")


def get(name):
    return {"D2Q9": D2Q9, "D3Q27": D3Q27}[name]
