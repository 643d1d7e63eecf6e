"""Seeded synthetic workloads shared by the HIP path, the tests and the oracle.

This module only describes inputs: mesh coordinates, region flags, physical
constants, the initial condition as a function of position, seeded noise and
the time-step rule. It holds none of the discretisation's arithmetic (no
basis, quadrature, flux or time-integration formula) and imports nothing from
the rest of the package, so that the oracle and the HIP path can both consume
it without sharing code.

Workloads (shapes follow the experiments of the paper, Sec. 5):

* ``vortex``: 2D Euler isentropic vortex on the periodic square [0,10]^2,
  16x16 quads, uniform in x; in y the middle four rows are compressed 20x and
  are the implicit strip (Sec. 5.1.2 uses an implicit band through which a
  vortex is advected).  Degree 2, Lax-Friedrichs flux, ARS(2,2,2), 20 steps.
* ``boundary_layer``: 2D Navier-Stokes flat-plate boundary layer on
  [0,2]x[0,0.5], 256x128 quads, wall-normal geometric stretching (ratio 1.12,
  first-cell aspect ratio 1000, capped so the rows fill the height); the first
  16 wall rows are implicit HDG-MX, the rest explicit DG-IP.  Degree 4,
  ARS(3,4,3), 200 steps (the stiffness study of Sec. 5.2 on a Cartesian
  analogue).
* ``boundary_layer_small`` and ``vortex_small``: the same physics on meshes
  small enough for the oracle's monolithic Newton solve.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Dict, Optional

import numpy as np

BC_PERIODIC = 0
BC_FARFIELD = 1
BC_WALL = 2

FLUX_VIJAYASUNDARAM = 0   # DG flux of the paper (characteristic upwinding at the mean state)
FLUX_LAX_FRIEDRICHS = 1   # DG flux named by the vortex workload
HDG_FLUX_FVS = 0          # S_c = A_n^+(Uhat)
HDG_FLUX_LF = 1           # S_c = lambda_max(Uhat) I

HDG_IP = 0
HDG_MX = 1


@dataclasses.dataclass
class Workload:
    name: str
    xgrid: np.ndarray            # (nx+1,) strictly increasing
    ygrid: np.ndarray            # (ny+1,)
    bc: tuple                    # (-x, +x, -y, +y) in BC_*
    implicit: np.ndarray         # (ny, nx) bool, element (i, j) at [j, i]
    degree: int
    gamma: float
    R: float
    mu: float
    Pr: float
    viscous: bool
    u_inf: np.ndarray            # conservative free-stream state (4,)
    dg_flux: int
    hdg_flux: int
    hdg_variant: int
    tableau: str                 # "ARS222" | "ARS343"
    dt: float
    steps: int
    ic: Callable                 # ic(x, y, elem_index, node_index) -> (4, ...) conservative
    alpha_dg: float = 1.0
    alpha_hdg: float = 10.0

    @property
    def nx(self) -> int:
        return len(self.xgrid) - 1

    @property
    def ny(self) -> int:
        return len(self.ygrid) - 1

    @property
    def n_elem(self) -> int:
        return self.nx * self.ny

    @property
    def nodes_per_elem(self) -> int:
        return (self.degree + 1) ** 2

    @property
    def n_dof(self) -> int:
        return self.n_elem * self.nodes_per_elem * 4

    @property
    def stages(self) -> int:
        return {"ARS222": 2, "ARS343": 3}[self.tableau]

    def implicit_flags(self) -> np.ndarray:
        """Per-element implicit flag, lexicographic with x fastest (uint8)."""
        return self.implicit.reshape(-1).astype(np.uint8)


def _conservative(rho, u, v, p, gamma):
    return np.stack([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


# ----------------------------------------------------------------------------
# isentropic vortex
# ----------------------------------------------------------------------------

def vortex_ic(gamma: float, beta: float, uinf: float, vinf: float, xc: float = 5.0, yc: float = 5.0):
    """Steady isentropic vortex in radial equilibrium, advected by (uinf, vinf)."""
    def ic(x, y, elem=None, node=None):
        dx = x - xc
        dy = y - yc
        r2 = dx * dx + dy * dy
        f = beta / (2.0 * math.pi) * np.exp(0.5 * (1.0 - r2))
        u = uinf - f * dy
        v = vinf + f * dx
        T = 1.0 - (gamma - 1.0) * beta * beta / (8.0 * gamma * math.pi ** 2) * np.exp(1.0 - r2)
        rho = T ** (1.0 / (gamma - 1.0))
        p = rho * T
        return _conservative(rho, u, v, p, gamma)
    return ic


def _strip_grid_y(ny: int, strip_rows: int, compression: float, L: float = 10.0):
    """Rows of equal height H except a centred strip of rows of height H/compression."""
    H = L / ((ny - strip_rows) + strip_rows / compression)
    j0 = (ny - strip_rows) // 2
    h = np.full(ny, H)
    h[j0:j0 + strip_rows] = H / compression
    y = np.concatenate([[0.0], np.cumsum(h)])
    y[-1] = L
    return y, j0


def _euler_dt(wl_grid_x, wl_grid_y, implicit, k, ic, gamma, cfl=0.5):
    """Explicit-region time step: dt = cfl / max_T (k+1)^2 (|u|+c)/h_min, the wave speed
    sampled on a 5x5 grid of points of each explicit element."""
    xs, ys = np.asarray(wl_grid_x), np.asarray(wl_grid_y)
    jj, ii = np.nonzero(~np.asarray(implicit))
    if len(ii) == 0:
        return np.inf
    t = np.linspace(0.0, 1.0, 5)
    X = xs[ii, None, None] + (xs[ii + 1] - xs[ii])[:, None, None] * t[None, None, :]
    Y = ys[jj, None, None] + (ys[jj + 1] - ys[jj])[:, None, None] * t[None, :, None]
    X, Y = np.broadcast_arrays(X, Y)
    U = ic(X, Y)
    rho = U[0]
    u = U[1] / rho
    v = U[2] / rho
    p = (gamma - 1.0) * (U[3] - 0.5 * rho * (u * u + v * v))
    s = (np.sqrt(u * u + v * v) + np.sqrt(gamma * p / rho)).reshape(len(ii), -1).max(axis=1)
    h = np.minimum(xs[ii + 1] - xs[ii], ys[jj + 1] - ys[jj])
    return cfl / np.max((k + 1) ** 2 * s / h)


def vortex(nx: int = 16, ny: int = 16, k: int = 2, strip_rows: int = 4, compression: float = 20.0,
           beta: float = 5.0, steps: int = 20, name: str = "vortex", dt_scale: float = 1.0) -> Workload:
    gamma = 1.4
    x = np.linspace(0.0, 10.0, nx + 1)
    y, j0 = _strip_grid_y(ny, strip_rows, compression)
    implicit = np.zeros((ny, nx), dtype=bool)
    implicit[j0:j0 + strip_rows, :] = True
    speed = 0.5 * math.sqrt(gamma)          # Mach 0.5 with rho = p = 1
    uinf = vinf = speed / math.sqrt(2.0)
    ic = vortex_ic(gamma, beta, uinf, vinf)
    dt = _euler_dt(x, y, implicit, k, ic, gamma) * dt_scale
    u_inf = _conservative(np.array(1.0), np.array(uinf), np.array(vinf), np.array(1.0), gamma).astype(float)
    return Workload(name=name, xgrid=x, ygrid=y, bc=(BC_PERIODIC,) * 4, implicit=implicit, degree=k,
                    gamma=gamma, R=1.0, mu=0.0, Pr=0.72, viscous=False, u_inf=u_inf,
                    dg_flux=FLUX_LAX_FRIEDRICHS, hdg_flux=HDG_FLUX_LF, hdg_variant=HDG_IP,
                    tableau="ARS222", dt=dt, steps=steps, ic=ic)


# ----------------------------------------------------------------------------
# flat-plate boundary layer
# ----------------------------------------------------------------------------

def boundary_layer_rows(ny: int, h0: float, ratio: float, height: Optional[float]):
    """Wall-normal row heights h_j = min(h0 ratio^j, h_cap) with h_cap chosen so that sum h = height.

    With ``height=None`` the rows are purely geometric (no cap)."""
    j = np.arange(ny)
    g = h0 * ratio ** j
    if height is None:
        return np.concatenate([[0.0], np.cumsum(g)])
    lo, hi = h0, height
    for _ in range(200):
        cap = 0.5 * (lo + hi)
        if np.minimum(g, cap).sum() > height:
            hi = cap
        else:
            lo = cap
    h = np.minimum(g, 0.5 * (lo + hi))
    y = np.concatenate([[0.0], np.cumsum(h)])
    y[-1] = height
    return y


def boundary_layer(nx: int = 256, ny: int = 128, k: int = 4, implicit_rows: int = 16, Lx: float = 2.0,
                   height: Optional[float] = 0.5, Re: float = 1.0e4, Ma: float = 0.3, Pr: float = 0.72,
                   steps: int = 200, seed: int = 2, noise: float = 0.01, name: str = "boundary_layer",
                   hdg_variant: int = HDG_MX, tableau: str = "ARS343", dt_scale: float = 1.0,
                   x0: float = 0.0, noise_kind: str = "smooth") -> Workload:
    """Flat-plate boundary layer.  noise_kind "smooth": the perturbation is a seeded
    random-phase Fourier field; "node": independent uniform draws in [-1, 1] at every
    node (the same seed, one draw per velocity component and node in the order the nodes
    are passed), both of amplitude `noise` and damped by the profile."""
    if noise_kind not in ("smooth", "node"):
        raise ValueError("noise_kind is 'smooth' or 'node'")
    gamma = 1.4
    hx = Lx / nx
    h0 = (2.0 / 256.0) / 1000.0          # first-cell aspect ratio 1000 at the reference spacing 2/256
    x = x0 + np.linspace(0.0, Lx, nx + 1)
    y = boundary_layer_rows(ny, h0, 1.12, height)
    implicit = np.zeros((ny, nx), dtype=bool)
    implicit[:implicit_rows, :] = True
    R = 1.0 / (gamma * Ma * Ma)
    p_inf = 1.0 / (gamma * Ma * Ma)
    mu = 1.0 / Re
    rng = np.random.default_rng(seed)
    # smooth seeded perturbation: random-phase Fourier modes over the reference plate [0,2]x[0,0.5]
    n_modes = 8
    kx = rng.integers(1, 9, size=(2, n_modes))
    ky = rng.integers(1, 5, size=(2, n_modes))
    ph = rng.uniform(0.0, 2.0 * math.pi, size=(2, n_modes))

    def xi(c, X, Y):
        s = np.zeros_like(X)
        for m in range(n_modes):
            s = s + np.sin(2.0 * math.pi * (kx[c, m] * X / 2.0 + ky[c, m] * Y / 0.5) + ph[c, m])
        return s / n_modes

    def ic(X, Y, elem=None, node=None):
        delta = 1.85 * np.sqrt((X + 0.05) / Re)
        base = np.tanh(Y / delta)
        if noise_kind == "node":
            draws = np.random.default_rng(seed).uniform(-1.0, 1.0, size=(2,) + np.shape(X))
            n0, n1 = draws[0], draws[1]
        else:
            n0, n1 = xi(0, X, Y), xi(1, X, Y)
        # 1% perturbation of the free-stream speed, damped by the profile so the wall stays no-slip
        u = base * (1.0 + noise * n0)
        v = noise * base * n1
        rho = np.ones_like(u)
        p = np.full_like(u, p_inf)
        return _conservative(rho, u, v, p, gamma)

    # time step from the first explicit row (Z18 rule: convective + viscous limit)
    cp = gamma * R / (gamma - 1.0)
    hmin = min(hx, float(np.min(np.diff(y)[implicit_rows:]))) if implicit_rows < ny else hx
    c = math.sqrt(gamma * p_inf)
    lam = (k + 1) ** 2 * ((1.0 + c) / hmin + (k + 1) ** 2 * max(4.0 / 3.0, gamma / Pr) * mu / hmin ** 2)
    dt = 0.5 / lam * dt_scale
    del cp
    u_inf = _conservative(np.array(1.0), np.array(1.0), np.array(0.0), np.array(p_inf), gamma).astype(float)
    return Workload(name=name, xgrid=x, ygrid=y, bc=(BC_FARFIELD, BC_FARFIELD, BC_WALL, BC_FARFIELD),
                    implicit=implicit, degree=k, gamma=gamma, R=R, mu=mu, Pr=Pr, viscous=True, u_inf=u_inf,
                    dg_flux=FLUX_VIJAYASUNDARAM, hdg_flux=HDG_FLUX_FVS, hdg_variant=hdg_variant,
                    tableau=tableau, dt=dt, steps=steps, ic=ic)


def farfield_mach_direction(gamma: float, Ma: float) -> np.ndarray:
    """d u_inf / d Ma of the boundary-layer far-field state (rho = |u| = 1, p = 1 / (gamma Ma^2)):
    only the energy changes, by dp/dMa / (gamma - 1)."""
    return np.array([0.0, 0.0, 0.0, -2.0 / (gamma * (gamma - 1.0) * Ma ** 3)])


def vortex_ensemble(n: int = 512, seed: int = 4, steps: int = 5, nmin: int = 8, nmax: int = 48):
    """Independent isentropic-vortex instances: square meshes N x N with N uniform in
    [nmin, nmax], degree uniform in {1, 2, 3, 4}, vortex strength uniform in [1, 5], a centred
    implicit strip of 1..6 rows (at most N - 2) compressed by a factor uniform in [5, 50]."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        N = int(rng.integers(nmin, nmax + 1))
        k = int(rng.integers(1, 5))
        beta = float(rng.uniform(1.0, 5.0))
        rows = min(int(rng.integers(1, 7)), N - 2)
        comp = float(rng.uniform(5.0, 50.0))
        out.append(vortex(nx=N, ny=N, k=k, strip_rows=rows, compression=comp, beta=beta, steps=steps,
                          name=f"vortex_ensemble_{i}"))
    return out


def get(name: str) -> Workload:
    """Named workloads (sizes as in the design document)."""
    table: Dict[str, Callable[[], Workload]] = {
        "vortex": lambda: vortex(),
        "vortex_small": lambda: vortex(nx=6, ny=6, k=2, strip_rows=2, steps=3, name="vortex_small"),
        "boundary_layer": lambda: boundary_layer(noise_kind="node"),
        "boundary_layer_smooth": lambda: boundary_layer(name="boundary_layer_smooth"),
        "boundary_layer_small": lambda: boundary_layer(nx=6, ny=6, k=2, implicit_rows=2, Lx=6 * 2.0 / 256,
                                                       height=None, steps=2, name="boundary_layer_small"),
    }
    return table[name]()


# ---------------------------------------------------------------------------
# 3D (hexahedra): the explicit DG residual of the Navier-Stokes channel
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Workload3D:
    """A Cartesian hexahedral mesh x(nx+1) x y(ny+1) x z(nz+1), element (i, j, l) at index
    i + nx (j + ny l), five conservative variables (rho, rho u, rho v, rho w, rho E); the
    boundary of each side is BC_PERIODIC or BC_FARFIELD (all elements explicit)."""
    name: str
    xgrid: np.ndarray
    ygrid: np.ndarray
    zgrid: np.ndarray
    bc: tuple                    # (-x, +x, -y, +y, -z, +z)
    degree: int
    gamma: float
    R: float
    mu: float
    Pr: float
    viscous: bool
    u_inf: np.ndarray            # (5,)
    dg_flux: int
    ic: Callable                 # ic(x, y, z) -> (5, ...) conservative
    alpha_dg: float = 1.0

    @property
    def nx(self) -> int:
        return len(self.xgrid) - 1

    @property
    def ny(self) -> int:
        return len(self.ygrid) - 1

    @property
    def nz(self) -> int:
        return len(self.zgrid) - 1

    @property
    def n_elem(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def nodes_per_elem(self) -> int:
        return (self.degree + 1) ** 3

    @property
    def n_dof(self) -> int:
        return self.n_elem * self.nodes_per_elem * 5


def conservative3d(rho, u, v, w, p, gamma):
    return np.stack([rho, rho * u, rho * v, rho * w,
                     p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)])


def channel3d(nx: int = 64, ny: int = 32, nz: int = 32, k: int = 3, Re: float = 3000.0, Ma: float = 0.2,
              Pr: float = 0.72, beta: float = 4.0610, seed: int = 3, amp: float = 0.05, viscous: bool = True,
              flux: int = FLUX_VIJAYASUNDARAM, name: str = "channel3d") -> Workload3D:
    """The 3D channel [0, 4 pi] x [-1, 1] x [0, 2 pi] with tanh-stretched rows
    y_j = tanh(beta (2 j / ny - 1)) / tanh(beta) (first-cell aspect ratio about 500 at
    ny = 32), periodic in x and z, Re 3000 on the half-height and bulk velocity, Ma 0.2.
    Initial state: Poiseuille u = 1.5 (1 - y^2) plus sinusoidal perturbations of u, v, w
    with random phases (seed 3), amplitude 5 %, damped by (1 - y^2); rho = 1, p = p_inf.
    The explicit residual is exercised on all elements, the y = +-1 sides being far-field
    boundaries at the wall-layer state (the wall layers themselves are the implicit
    HDG-IP region of the channel, which this engine builds in 2D only)."""
    gamma = 1.4
    Lx, Lz = 4.0 * math.pi, 2.0 * math.pi
    x = np.linspace(0.0, Lx, nx + 1)
    j = np.arange(ny + 1)
    y = np.tanh(beta * (2.0 * j / ny - 1.0)) / math.tanh(beta)
    z = np.linspace(0.0, Lz, nz + 1)
    R = 1.0 / (gamma * Ma * Ma)
    p_inf = 1.0 / (gamma * Ma * Ma)
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0.0, 2.0 * math.pi, size=(3, 3))
    kx = [1, 2, 3]
    kz = [2, 1, 3]

    def pert(c, X, Y, Z):
        s = np.zeros_like(X)
        for m in range(3):
            s = s + np.sin(kx[m] * 2.0 * math.pi * X / Lx + kz[m] * 2.0 * math.pi * Z / Lz + ph[c, m])
        return s / 3.0

    def ic(X, Y, Z):
        damp = 1.0 - Y * Y
        u = 1.5 * damp + amp * damp * pert(0, X, Y, Z)
        v = amp * damp * pert(1, X, Y, Z)
        w = amp * damp * pert(2, X, Y, Z)
        return conservative3d(np.ones_like(X), u, v, w, np.full_like(X, p_inf), gamma)

    u_inf = conservative3d(np.array(1.0), np.array(0.0), np.array(0.0), np.array(0.0), np.array(p_inf),
                           gamma).astype(float)
    return Workload3D(name=name, xgrid=x, ygrid=y, zgrid=z,
                      bc=(BC_PERIODIC, BC_PERIODIC, BC_FARFIELD, BC_FARFIELD, BC_PERIODIC, BC_PERIODIC),
                      degree=k, gamma=gamma, R=R, mu=(1.0 / Re) if viscous else 0.0, Pr=Pr, viscous=viscous,
                      u_inf=u_inf, dg_flux=flux, ic=ic)


def smooth_box3d(n=(3, 3, 3), k: int = 2, viscous: bool = True, mu: float = 0.02, flux: int = FLUX_VIJAYASUNDARAM,
                 bc=(BC_PERIODIC,) * 6, stretch: float = 0.0, name: str = "box3d") -> Workload3D:
    """Unit cube with a smooth state varying in all three directions (all velocity
    components nonzero); `stretch` > 0 grades the y rows geometrically."""
    gamma = 1.4
    nx, ny, nz = n
    x = np.linspace(0.0, 1.0, nx + 1)
    if stretch > 0.0:
        h = (1.0 + stretch) ** np.arange(ny)
        y = np.concatenate([[0.0], np.cumsum(h)]) / h.sum()
    else:
        y = np.linspace(0.0, 1.0, ny + 1)
    z = np.linspace(0.0, 1.0, nz + 1)
    tp = 2.0 * math.pi

    def ic(X, Y, Z):
        rho = 1.0 + 0.2 * np.sin(tp * X) * np.cos(tp * Z) + 0.1 * np.cos(tp * Y)
        u = 0.3 + 0.1 * np.cos(tp * (X + Y))
        v = 0.2 - 0.1 * np.sin(tp * (X + Z))
        w = -0.1 + 0.15 * np.sin(tp * (Y - Z))
        p = 2.5 + 0.3 * np.cos(tp * Y) * np.sin(tp * Z)
        return conservative3d(rho, u, v, w, p, gamma)

    u_inf = conservative3d(np.array(1.0), np.array(0.3), np.array(0.2), np.array(-0.1), np.array(2.5), gamma)
    return Workload3D(name=name, xgrid=x, ygrid=y, zgrid=z, bc=tuple(bc), degree=k, gamma=gamma, R=1.0,
                      mu=mu if viscous else 0.0, Pr=0.72, viscous=viscous, u_inf=np.asarray(u_inf, float),
                      dg_flux=flux, ic=ic)
