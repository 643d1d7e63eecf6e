"""Tensor-product mesh, facet tables and the implicit/explicit split (oracle; test infrastructure only).

Sec. 3.1 (mesh, skeleton, normals) and Sec. 4 (T = T^im U T^ex, interface
Gamma_i).  Elements are lexicographic with x fastest; element (i, j) covers
[x_i, x_{i+1}] x [y_j, y_{j+1}].  The characteristic length of the IP penalty
(eq. penalty_coefficient_ip) is l_T = |T| / |dT|.
"""
from __future__ import annotations

import numpy as np

from paper_2607_16044_amd.workloads import BC_PERIODIC, BC_FARFIELD, BC_WALL, Workload

# HDG facet kinds (Sec. 4.1.2 and App. B.2-B.3)
KIND_INTERIOR = 0
KIND_INTERFACE = 1
KIND_FARFIELD = 2
KIND_WALL = 3

OPPOSITE = np.array([1, 0, 3, 2])


class Mesh:
    def __init__(self, wl: Workload):
        self.wl = wl
        nx, ny = wl.nx, wl.ny
        self.nx, self.ny = nx, ny
        self.E = nx * ny
        ii, jj = np.meshgrid(np.arange(nx), np.arange(ny))
        ii = ii.reshape(-1)
        jj = jj.reshape(-1)
        self.ei, self.ej = ii, jj
        self.x0 = wl.xgrid[ii]
        self.y0 = wl.ygrid[jj]
        self.hx = wl.xgrid[ii + 1] - wl.xgrid[ii]
        self.hy = wl.ygrid[jj + 1] - wl.ygrid[jj]
        self.area = self.hx * self.hy
        self.lchar = self.area / (2.0 * (self.hx + self.hy))
        self.implicit = wl.implicit_flags().astype(bool)
        per_x = wl.bc[0] == BC_PERIODIC
        per_y = wl.bc[2] == BC_PERIODIC
        # neighbour element per local face (-1 = boundary) and boundary condition type
        self.nbr = -np.ones((self.E, 4), dtype=int)
        self.bctype = np.full((self.E, 4), -1, dtype=int)
        for e in range(self.E):
            i, j = ii[e], jj[e]
            cand = [(i - 1, j, 0), (i + 1, j, 1), (i, j - 1, 2), (i, j + 1, 3)]
            for (a, b, f) in cand:
                if 0 <= a < nx and 0 <= b < ny:
                    self.nbr[e, f] = a + nx * b
                elif f < 2 and per_x:
                    self.nbr[e, f] = (a % nx) + nx * b
                elif f >= 2 and per_y:
                    self.nbr[e, f] = a + nx * (b % ny)
                else:
                    self.bctype[e, f] = wl.bc[f]
        # global facets: (eL, fL, eR, fR); L = lower coordinate side
        facets = []
        nvx = nx if per_x else nx + 1
        for j in range(ny):
            for i in range(nvx):
                eR = i + nx * j if i < nx else -1
                if i > 0:
                    eL = (i - 1) + nx * j
                elif per_x:
                    eL = (nx - 1) + nx * j
                else:
                    eL = -1
                facets.append((eL, 1, eR, 0))
        nhy = ny if per_y else ny + 1
        for j in range(nhy):
            for i in range(nx):
                eR = i + nx * j if j < ny else -1
                if j > 0:
                    eL = i + nx * (j - 1)
                elif per_y:
                    eL = i + nx * (ny - 1)
                else:
                    eL = -1
                facets.append((eL, 3, eR, 2))
        self.facets = np.array(facets, dtype=int)
        self.n_facets = len(facets)
        # element face -> global facet
        self.efacet = -np.ones((self.E, 4), dtype=int)
        for F, (eL, fL, eR, fR) in enumerate(self.facets):
            if eL >= 0:
                self.efacet[eL, fL] = F
            if eR >= 0:
                self.efacet[eR, fR] = F
        # HDG facets: touching at least one implicit element
        self.hdg_index = -np.ones(self.n_facets, dtype=int)
        hdg = []
        for F, (eL, fL, eR, fR) in enumerate(self.facets):
            sides = [e for e in (eL, eR) if e >= 0]
            if any(self.implicit[e] for e in sides):
                self.hdg_index[F] = len(hdg)
                hdg.append(F)
        self.hdg_facets = np.array(hdg, dtype=int)
        self.n_hdg = len(hdg)
        # HDG facet kind as seen from an implicit element's face
        self.face_kind = np.full((self.E, 4), -1, dtype=int)
        for e in range(self.E):
            if not self.implicit[e]:
                continue
            for f in range(4):
                nb = self.nbr[e, f]
                if nb >= 0:
                    self.face_kind[e, f] = KIND_INTERIOR if self.implicit[nb] else KIND_INTERFACE
                else:
                    self.face_kind[e, f] = KIND_FARFIELD if self.bctype[e, f] == BC_FARFIELD else KIND_WALL
        self.im_elems = np.nonzero(self.implicit)[0]
        self.ex_elems = np.nonzero(~self.implicit)[0]
        for e in self.ex_elems:
            for f in range(4):
                if self.nbr[e, f] < 0 and self.bctype[e, f] == BC_WALL:
                    raise ValueError("adiabatic walls are supported on implicit elements only")

    def node_coords(self, basis):
        """Physical coordinates (E, nn) of the element nodes."""
        n1 = basis.k + 1
        a = np.arange(basis.nn) % n1
        b = np.arange(basis.nn) // n1
        X = self.x0[:, None] + 0.5 * (basis.nodes[a][None, :] + 1.0) * self.hx[:, None]
        Y = self.y0[:, None] + 0.5 * (basis.nodes[b][None, :] + 1.0) * self.hy[:, None]
        return X, Y
