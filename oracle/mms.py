"""Manufactured solution and its source term (oracle; test infrastructure only).

Sec. 5.1.1 verifies the IMEX schemes with a manufactured solution: the equations get a
source S = dU_e/dt + div(F^c(U_e) - F^nu(U_e, grad U_e)) so that U_e solves them, and the
error of the discrete solution against U_e is measured over time-step sizes.  The solution
is the smooth travelling wave the paper takes from the literature,
    U_e = (s, s, s, s^2),   s = sin(pi (kx x + ky y) - omega pi t) + 4,
(so u = v = 1 and E = s).  Here S is evaluated point by point: dU_e/dt and grad U_e in closed
form, the divergence of the flux by the complex step in x and in y separately (an exact
derivative of the analytic flux, to rounding).

Discrete source: b[e][v][n] = int_T S_v(x, t) phi_n dx with the volume rule; with it the
semi-discrete equations read M dU/dt = -R + b.
"""
from __future__ import annotations

import numpy as np

from . import physics as ph
from .basis import Basis
from .dg import Geometry
from .mesh import Mesh


def exact_state(x, y, t, kx, ky, omega):
    """U_e at (x, y, t): (4, ...)."""
    s = np.sin(np.pi * (kx * x + ky * y) - omega * np.pi * t) + 4.0
    return np.stack([s, s, s, s * s])


def exact_gradient(x, y, t, kx, ky, omega):
    """grad U_e (4, 2, ...) in closed form."""
    arg = np.pi * (kx * x + ky * y) - omega * np.pi * t
    s = np.sin(arg) + 4.0
    ds = np.cos(arg)
    dU = np.stack([ds, ds, ds, 2.0 * s * ds])          # d U_e / d arg
    return np.stack([dU * (np.pi * kx), dU * (np.pi * ky)], axis=1)


def source(x, y, t, kx, ky, omega, gas: ph.Gas, h=1e-30):
    """S = dU_e/dt + d/dx (F^c - F^nu)_x + d/dy (F^c - F^nu)_y at points (x, y): (4, ...)."""
    x = np.asarray(x, dtype=float)
    y = np.asarray(y, dtype=float)
    arg = np.pi * (kx * x + ky * y) - omega * np.pi * t
    s = np.sin(arg) + 4.0
    ds = np.cos(arg)
    dUdt = np.stack([ds, ds, ds, 2.0 * s * ds]) * (-omega * np.pi)

    def flux(xx, yy, d):
        U = exact_state(xx, yy, t, kx, ky, omega)
        G = exact_gradient(xx, yy, t, kx, ky, omega)
        return ph.convective_flux(U, gas)[:, d] - ph.viscous_flux(U, G, gas)[:, d]
    ddx = np.imag(flux(x + 1j * h, y, 0)) / h
    ddy = np.imag(flux(x, y + 1j * h, 1)) / h
    return dUdt + ddx + ddy


def source_load(t, kx, ky, omega, mesh: Mesh, basis: Basis, gas: ph.Gas):
    """b[e][v][n] = int_T S_v(x, t) phi_n dx (E, 4, nn) with the volume Gauss rule."""
    geo = Geometry(mesh, basis)
    Q = basis.nq
    qi = np.arange(Q * Q) % Q
    qj = np.arange(Q * Q) // Q
    X = mesh.x0[:, None] + 0.5 * (basis.qx[qi][None, :] + 1.0) * mesh.hx[:, None]
    Y = mesh.y0[:, None] + 0.5 * (basis.qx[qj][None, :] + 1.0) * mesh.hy[:, None]
    S = source(X, Y, t, kx, ky, omega, gas)                        # (4, E, Qv)
    w = basis.wvol[None, :] * geo.jac[:, None]
    return np.einsum("veq,qn,eq->evn", S, basis.phi, w)
