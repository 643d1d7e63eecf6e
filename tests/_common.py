"""Helpers shared by the tests: library availability and workload variants."""
import math
import os

import numpy as np
import pytest

from paper_2607_16044_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2607_16044_amd", "libimexhdg.so")


def ensure_built():
    if not os.path.exists(LIB):
        from paper_2607_16044_amd import build
        build.build()
    return LIB


def gpu_engine(wl, **kw):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    ensure_built()
    from paper_2607_16044_amd.binding import Engine
    return Engine(wl, **kw)


def smooth_square(n=4, k=2, viscous=True, mu=0.02, variant=W.HDG_IP, implicit_rows=(), lf=False,
                  bc=(W.BC_PERIODIC,) * 4, tableau="ARS222", dt=1e-3):
    """Periodic unit square with a smooth non-trivial state (used for parity checks)."""
    x = np.linspace(0.0, 1.0, n + 1)
    implicit = np.zeros((n, n), dtype=bool)
    for j in implicit_rows:
        implicit[j, :] = True

    def ic(X, Y, elem=None, node=None):
        tp = 2.0 * math.pi
        rho = 1.0 + 0.2 * np.sin(tp * X) * np.cos(tp * Y)
        u = 0.3 + 0.1 * np.cos(tp * (X + Y))
        v = 0.2 - 0.1 * np.sin(tp * X)
        p = 2.5 + 0.3 * np.cos(tp * Y)
        return np.stack([rho, rho * u, rho * v, p / 0.4 + 0.5 * rho * (u * u + v * v)])
    uinf = np.array([1.0, 0.3, 0.2, 2.5 / 0.4 + 0.5 * (0.09 + 0.04)])
    return W.Workload(name="square", xgrid=x, ygrid=x.copy(), bc=bc, implicit=implicit, degree=k, gamma=1.4, R=1.0,
                      mu=mu if viscous else 0.0, Pr=0.72, viscous=viscous, u_inf=uinf,
                      dg_flux=W.FLUX_LAX_FRIEDRICHS if lf else W.FLUX_VIJAYASUNDARAM,
                      hdg_flux=W.HDG_FLUX_LF if lf else W.HDG_FLUX_FVS, hdg_variant=variant, tableau=tableau, dt=dt,
                      steps=1, ic=ic)


def rel_err(a, b):
    """Largest relative error of a against b.  States laid out [element or facet][field][node]
    (3D arrays with the four conservative fields on axis 1) are compared field by field, each
    field relative to its own largest magnitude, and the worst field is returned, so a small
    field (rho v near a wall) is held to the same relative bar as rho E.  Other arrays (element
    blocks, flat vectors) are compared relative to their largest magnitude."""
    a = np.asarray(a)
    b = np.asarray(b)
    if a.ndim == 3 and a.shape[1] == 4:
        return max(rel_err(a[:, v], b[:, v]) for v in range(4))
    if a.size == 0:
        return 0.0
    scale = np.maximum(np.abs(b).max(), 1e-300)
    return float(np.abs(a - b).max() / scale)


MMS = (2.0, 2.0, 200.0)          # kx, ky, omega of the manufactured solution (Sec. 5.1.1)


def mms_workload(n=8, k=2, implicit_cols=(), variant=W.HDG_MX, tableau="ARS222", dt=1e-4, mu=0.01, lf=False):
    """Periodic unit square for the manufactured solution: U_e = (s, s, s, s^2),
    s = sin(pi (kx x + ky y) - omega pi t) + 4 (u = v = 1), gamma 1.4, Pr 0.72, mu 0.01;
    implicit_cols: the element columns of the implicit region (the paper takes the middle
    half, x in [0.25, 0.75])."""
    from oracle.mms import exact_state          # noqa: F401  (the same closed form, for the tests)
    x = np.linspace(0.0, 1.0, n + 1)
    implicit = np.zeros((n, n), dtype=bool)
    for i in implicit_cols:
        implicit[:, i] = True
    kx, ky, om = MMS

    def ic(X, Y, elem=None, node=None):
        s = np.sin(np.pi * (kx * X + ky * Y)) + 4.0
        return np.stack([s, s, s, s * s])
    return W.Workload(name="mms", xgrid=x, ygrid=x.copy(), bc=(W.BC_PERIODIC,) * 4, implicit=implicit, degree=k,
                      gamma=1.4, R=1.0, mu=mu, Pr=0.72, viscous=True, u_inf=np.array([4.0, 4.0, 4.0, 16.0]),
                      dg_flux=W.FLUX_LAX_FRIEDRICHS if lf else W.FLUX_VIJAYASUNDARAM,
                      hdg_flux=W.HDG_FLUX_LF if lf else W.HDG_FLUX_FVS, hdg_variant=variant, tableau=tableau,
                      dt=dt, steps=1, ic=ic)
