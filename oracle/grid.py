"""Geometry bookkeeping for the oracle: neighbour values with periodic wrap and the
classification of neighbour positions (fluid / solid / inlet ghost / outlet ghost).

Grids are (nz, ny, nx) tensors (nz = 1 for 2-D); axis d = 0, 1, 2 is x, y, z and lives
in tensor dimension -1, -2, -3.  Domain faces are ordered (-x, +x, -y, +y, -z, +z)."""
import torch

FLUID, SOLID, INLET, OUTLET = 0, 1, 2, 3
FACE_CODES = {"periodic": None, "wall": SOLID, "inlet": INLET, "outlet": OUTLET}


class Grid:
    def __init__(self, params, solid=None, phi=None):
        self.nx, self.ny, self.nz = params["nx"], params["ny"], params["nz"]
        self.shape = (self.nz, self.ny, self.nx)
        self.D = 2 if params["lattice"] == "D2Q9" else 3
        self.faces = list(params["face_bc"])
        if solid is None:
            solid = torch.zeros(self.shape, dtype=torch.bool)
        self.solid = solid.to(torch.bool).reshape(self.shape)
        self.fluid = ~self.solid
        # signed wall distance at the nodes (curved walls), or None (staircase walls)
        self.phi = None if phi is None else phi.to(torch.float64).reshape(self.shape)
        idx = torch.meshgrid(torch.arange(self.nz), torch.arange(self.ny),
                             torch.arange(self.nx), indexing="ij")
        self.coord = [idx[2], idx[1], idx[0]]          # x, y, z index of every cell
        self.n = [self.nx, self.ny, self.nz]

    @staticmethod
    def tdim(d):
        return -1 - d

    def shift(self, t, d, k):
        """Value of t at cell i + k e_d (periodic wrap)."""
        return torch.roll(t, shifts=-k, dims=self.tdim(d))

    def shift_vec(self, t, offs):
        """Value of t at cell i + offs (offs per axis, periodic wrap)."""
        for d, k in enumerate(offs):
            if k:
                t = self.shift(t, d, k)
        return t

    def face_of(self, d, k):
        """Per cell: None-or-face-code if i + k e_d leaves the domain through a
        non-periodic face; returns (outside mask, code tensor)."""
        pos = self.coord[d] + k
        low, high = pos < 0, pos >= self.n[d]
        code = torch.full(self.shape, -1, dtype=torch.int64)
        for mask, face in ((low, self.faces[2 * d]), (high, self.faces[2 * d + 1])):
            fc = FACE_CODES[face]
            if fc is not None:
                code = torch.where(mask, torch.full_like(code, fc), code)
        return code >= 0, code

    def solid_cell(self, d, k):
        """Position i + k e_d is a solid cell inside the domain (not beyond a face)."""
        outside, _ = self.face_of(d, k)
        return self.shift(self.solid, d, k) & ~outside

    def status(self, d, k):
        """Classification of position i + k e_d for every cell i."""
        outside, code = self.face_of(d, k)
        inner = torch.where(self.shift(self.solid, d, k), SOLID, FLUID)
        return torch.where(outside, code, inner)
