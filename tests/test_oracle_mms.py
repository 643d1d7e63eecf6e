"""The oracle's manufactured-solution source (Sec. 5.1.1), CPU only.

* The source S = dU_e/dt + div(F^c - F^nu) at random points against central finite
  differences in t, x and y of the closed-form solution and flux (independent of the
  complex-step derivative the oracle uses).
* Consistency of the discrete source: for the exact solution interpolated on an explicit
  periodic mesh, M^-1 (b - R^DG) converges to dU_e/dt under refinement, i.e. the source
  makes U_e a solution of the discrete equations up to the truncation error.
* The IMEX step with the source keeps the oracle's conservation ledger exact (the totals
  change by the interface defect plus the integrated source, which vanishes over whole
  periods of the wave).
"""
import numpy as np

from _common import MMS, mms_workload
from oracle import physics as ph
from oracle.ark import IMEXSolver
from oracle.basis import Basis
from oracle.dg import Geometry, apply_minv, dg_residual
from oracle.mesh import Mesh
from oracle.mms import exact_gradient, exact_state, source, source_load


def test_source_against_finite_differences():
    gas = ph.Gas(1.4, 1.0, 0.01, 0.72)
    kx, ky, om = MMS
    rng = np.random.default_rng(1)
    x, y, t = rng.random(20), rng.random(20), 1e-3 * rng.random()
    h = 1e-5

    def flux(xx, yy, d):
        U = exact_state(xx, yy, t, kx, ky, om)
        G = exact_gradient(xx, yy, t, kx, ky, om)
        return ph.convective_flux(U, gas)[:, d] - ph.viscous_flux(U, G, gas)[:, d]
    fd = ((exact_state(x, y, t + h * 1e-3, kx, ky, om) - exact_state(x, y, t - h * 1e-3, kx, ky, om)) / (2e-3 * h)
          + (flux(x + h, y, 0) - flux(x - h, y, 0)) / (2 * h) + (flux(x, y + h, 1) - flux(x, y - h, 1)) / (2 * h))
    S = source(x, y, t, kx, ky, om, gas)
    assert np.abs(S - fd).max() < 1e-6 * np.abs(S).max()
    # the closed-form gradient against differences of the state
    G = exact_gradient(x, y, t, kx, ky, om)
    gx = (exact_state(x + h, y, t, kx, ky, om) - exact_state(x - h, y, t, kx, ky, om)) / (2 * h)
    assert np.abs(G[:, 0] - gx).max() < 1e-7 * np.abs(G).max()


def test_discrete_source_makes_the_exact_solution_consistent():
    kx, ky, om = MMS
    t = 3e-4
    errs = []
    for n in (8, 16):
        wl = mms_workload(n=n, k=3)
        mesh, basis = Mesh(wl), Basis(3)
        gas = ph.Gas(wl.gamma, wl.R, wl.mu, wl.Pr)
        X, Y = mesh.node_coords(basis)
        U = np.moveaxis(exact_state(X, Y, t, kx, ky, om), 0, 1).copy()
        R = dg_residual(U, None, wl, mesh, basis, gas)
        b = source_load(t, kx, ky, om, mesh, basis, gas)
        geo = Geometry(mesh, basis)
        dudt = apply_minv(b - R, basis, geo)
        arg = np.pi * (kx * X + ky * Y) - om * np.pi * t
        c = np.cos(arg)
        s = np.sin(arg) + 4.0
        ex = np.moveaxis(np.stack([c, c, c, 2 * s * c]), 0, 1) * (-om * np.pi)
        errs.append(np.sqrt(np.mean((dudt - ex) ** 2)) / np.sqrt(np.mean(ex ** 2)))
    print(errs)
    assert errs[1] < 0.15 * errs[0] and errs[1] < 1e-3


def test_ledger_with_source():
    wl = mms_workload(n=4, k=2, implicit_cols=(1, 2), dt=2e-4)
    s = IMEXSolver(wl)
    s.mms = MMS
    for _ in range(2):
        m0 = s.totals()
        s.step()
        L = s.ledger[-1]
        resid = s.totals() - m0 - L["interface"] - L["boundary"] - L["source"]
        assert np.all(np.abs(resid) <= 1e-12 * np.abs(m0)), resid
        # over whole periods of the wave the integrated source vanishes (both dU_e/dt and the
        # flux divergence integrate to zero on the periodic square)
        assert np.abs(L["source"]).max() < 1e-12 * np.abs(m0).max()
