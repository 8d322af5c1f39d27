"""Structured hexahedral mesh topology (oracle; test infrastructure only).

The paper uses a partition of the domain into hexahedra T, its faces E_h and
outer normals (Sec. 2), macro-elements made of 2x2x2 hexahedra (Sec. 3,
figure macroel).  Numbering is a choice of this project:

* node (i,j,k)  -> i + (nx+1)*(j + (ny+1)*k)
* cell (i,j,k)  -> i + nx*(j + ny*k)
* faces: all x-normal faces (i in 0..nx, j<ny, k<nz) numbered
  i + (nx+1)*(j + ny*k); then y-normal faces (offset n_fx) i + nx*(j + (ny+1)*k);
  then z-normal faces (offset n_fx+n_fy) i + nx*(j + ny*k)
* local cell nodes a = 0..7 at offsets (a&1, (a>>1)&1, (a>>2)&1)
* local cell faces (-x, +x, -y, +y, -z, +z)
* displacement dof = 3*node + component; system order [u; p; pi]
"""
from __future__ import annotations

import numpy as np


class Mesh:
    def __init__(self, nx: int, ny: int, nz: int, coords: np.ndarray):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.coords = np.asarray(coords, dtype=np.float64)
        self.n_nodes = (nx + 1) * (ny + 1) * (nz + 1)
        self.n_cells = nx * ny * nz
        self.n_fx = (nx + 1) * ny * nz
        self.n_fy = nx * (ny + 1) * nz
        self.n_fz = nx * ny * (nz + 1)
        self.n_faces = self.n_fx + self.n_fy + self.n_fz
        assert self.coords.shape == (self.n_nodes, 3)
        k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        self.ci, self.cj, self.ck = i.ravel(), j.ravel(), k.ravel()
        self.cell_nodes = np.empty((self.n_cells, 8), dtype=np.int64)
        for a in range(8):
            di, dj, dk = a & 1, (a >> 1) & 1, (a >> 2) & 1
            self.cell_nodes[:, a] = self.node_id(self.ci + di, self.cj + dj, self.ck + dk)
        self.cell_faces = np.empty((self.n_cells, 6), dtype=np.int64)
        self.cell_faces[:, 0] = self.fx_id(self.ci, self.cj, self.ck)
        self.cell_faces[:, 1] = self.fx_id(self.ci + 1, self.cj, self.ck)
        self.cell_faces[:, 2] = self.fy_id(self.ci, self.cj, self.ck)
        self.cell_faces[:, 3] = self.fy_id(self.ci, self.cj + 1, self.ck)
        self.cell_faces[:, 4] = self.fz_id(self.ci, self.cj, self.ck)
        self.cell_faces[:, 5] = self.fz_id(self.ci, self.cj, self.ck + 1)

    # -- ids -----------------------------------------------------------------
    def node_id(self, i, j, k):
        return i + (self.nx + 1) * (j + (self.ny + 1) * k)

    def cell_id(self, i, j, k):
        return i + self.nx * (j + self.ny * k)

    def fx_id(self, i, j, k):
        return i + (self.nx + 1) * (j + self.ny * k)

    def fy_id(self, i, j, k):
        return self.n_fx + i + self.nx * (j + (self.ny + 1) * k)

    def fz_id(self, i, j, k):
        return self.n_fx + self.n_fy + i + self.nx * (j + self.ny * k)

    def face_cells(self, f):
        """Cells sharing face f (one or two)."""
        nx, ny, nz = self.nx, self.ny, self.nz
        if f < self.n_fx:
            i, r = f % (nx + 1), f // (nx + 1)
            j, k = r % ny, r // ny
            cand = [(i - 1, j, k), (i, j, k)]
        elif f < self.n_fx + self.n_fy:
            g = f - self.n_fx
            i, r = g % nx, g // nx
            j, k = r % (ny + 1), r // (ny + 1)
            cand = [(i, j - 1, k), (i, j, k)]
        else:
            g = f - self.n_fx - self.n_fy
            i, r = g % nx, g // nx
            j, k = r % ny, r // ny
            cand = [(i, j, k - 1), (i, j, k)]
        return [self.cell_id(a, b, c) for (a, b, c) in cand
                if 0 <= a < nx and 0 <= b < ny and 0 <= c < nz]

    # -- node / face sets ------------------------------------------------------
    def node_ijk(self):
        k, j, i = np.meshgrid(np.arange(self.nz + 1), np.arange(self.ny + 1),
                              np.arange(self.nx + 1), indexing="ij")
        return i.ravel(), j.ravel(), k.ravel()

    def bottom_nodes(self):
        i, j, k = self.node_ijk()
        return np.nonzero(k == 0)[0]

    def top_faces(self):
        """z-normal faces on the plane k = nz (drained boundary)."""
        i, j = np.meshgrid(np.arange(self.nx), np.arange(self.ny), indexing="xy")
        return np.sort(self.fz_id(i.ravel(), j.ravel(), self.nz))

    def top_cells(self):
        return np.nonzero(self.ck == self.nz - 1)[0]

    def boundary_faces(self):
        f = []
        for j in range(self.ny):
            for k in range(self.nz):
                f += [self.fx_id(0, j, k), self.fx_id(self.nx, j, k)]
        for i in range(self.nx):
            for k in range(self.nz):
                f += [self.fy_id(i, 0, k), self.fy_id(i, self.ny, k)]
        for i in range(self.nx):
            for j in range(self.ny):
                f += [self.fz_id(i, j, 0), self.fz_id(i, j, self.nz)]
        return np.array(sorted(f), dtype=np.int64)

    def cell_coords(self):
        """(n_cells, 8, 3) node coordinates of every hexahedron."""
        return self.coords[self.cell_nodes]

    def macro_elements(self):
        """Macro-elements: aligned 2x2x2 blocks of cells (Sec. 3).  Returns an
        (n_macro, 8) array of cell ids with local order (a&1, (a>>1)&1, (a>>2)&1)."""
        assert self.nx % 2 == 0 and self.ny % 2 == 0 and self.nz % 2 == 0
        K, J, I = np.meshgrid(np.arange(self.nz // 2), np.arange(self.ny // 2),
                              np.arange(self.nx // 2), indexing="ij")
        I, J, K = I.ravel(), J.ravel(), K.ravel()
        out = np.empty((I.size, 8), dtype=np.int64)
        for a in range(8):
            out[:, a] = self.cell_id(2 * I + (a & 1), 2 * J + ((a >> 1) & 1), 2 * K + ((a >> 2) & 1))
        return out
