"""Curved walls for both solvers (the paper's "proper treatment of curved boundaries",
Sec. 1, used for the obstacles of Sec. 3.1 and the burner of Sec. 3.2; the methods are
not given, so this is a reading: parity unpinned against the paper, pinned against
viscous decay rates between off-lattice walls and in a circular cavity in the tests).

Test infrastructure: see the package header.

The wall is the zero level of a signed distance phi given at the nodes (phi >= 0 fluid,
phi < 0 solid).  Along a link or grid line from a fluid node r to a solid node s the wall
sits at the fraction q = phi(r) / (phi(r) - phi(s)) in [0, 1) of the way (phi linear
between the two nodes).

Lattice Boltzmann (linearly interpolated bounce-back of Bouzidi, Firdaouss and Lallemand,
Phys. Fluids 13, 2001): population i arriving at fluid node r from the solid node r - c_i
is built from post-collision values,
    q <  1/2:  g_i(r) = 2q g*_ib(r) + (1 - 2q) g*_ib(r + c_i)
    q >= 1/2:  g_i(r) = g*_ib(r) / (2q) + (1 - 1/(2q)) g*_i(r)
with ib the opposite of i; q = 1/2 is the halfway bounce-back g_i(r) = g*_ib(r).  Where
q < 1/2 and r + c_i is not a fluid node, the halfway value is used.

Finite differences (ghost values along grid lines, zero normal gradient): a stencil point
across the wall takes the value at its mirror image about the wall on the same grid line,
linearly interpolated between the fluid nodes on the other side.  An image that falls
between the wall and the nearest fluid node (at distance p < 0 from it) takes the value
of the even quadratic a + b d^2 in the wall distance d through the two nearest fluid
nodes, v0 + (v1 - v0) p/(2 - p), which has zero gradient at the wall.  With the wall
halfway (q = 1/2) this is the plain mirror rule.  Density ghosts for grad(rho) are the
ideal-gas density of the ghost scalars.
"""
import torch


def fraction(phi_fluid, phi_solid):
    """q of the wall between a fluid node and a solid node."""
    return phi_fluid / (phi_fluid - phi_solid)


def lerp(a, b, p):
    """(1 - p) a + p b, exact at p = 0 and p = 1."""
    return (1.0 - p) * a + p * b


def bounce_back(q, g_opp_here, g_opp_next, g_same_here, next_fluid):
    """g_i(r) of an interpolated bounce-back link (tensors of one population)."""
    near = lerp(g_opp_next, g_opp_here, 2.0 * q)                # 2q here + (1-2q) next
    qq = torch.where(q >= 0.5, q, torch.ones_like(q))
    far = g_opp_here / (2.0 * qq) + (1.0 - 1.0 / (2.0 * qq)) * g_same_here
    near = torch.where(next_fluid, near, g_opp_here)
    return torch.where(q < 0.5, near, far)


def mirror_value(p, v0, v1, v2):
    """Value at the image point at distance p (-1 < p <= 2, counted from node 0 away from
    the wall) on the line of nodes v0, v1, v2."""
    inner = lerp(v0, v1, torch.where(p >= 0.0, p, p / (2.0 - p)))
    outer = lerp(v1, v2, torch.clamp(p - 1.0, min=0.0))
    return torch.where(p <= 1.0, inner, outer)
