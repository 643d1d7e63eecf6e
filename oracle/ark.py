"""ARS tableaux and the geometry-split IMEX step (oracle; test infrastructure only).

Sec. 4.2.2 and App. C (Alg. imex_scheme_update): the explicit (s+1)-stage ERK
and the s-stage SDIRK are synchronised by padding (cbar_{i+1} = c_i).  Per
stage i: R^DG_i = R^DG(y^ex_i, y^im_{i-1}); y^ex_{i+1} from eq. erk_stage_update;
then the implicit stage y^im_i from eqs. dirk_stage_update_* with interface
data y^ex_{i+1}.  After the loop: the final explicit update (eq.
erk_solution_update) unless the ERK is FSAL, and U^im_{n+1} = y^im_s when the
SDIRK is stiffly accurate (eq. dirk_solution_update otherwise).

The ARS schemes are those of Ascher, Ruuth and Spiteri (1997) that the paper
adopts (Sec. 4.2.2); their constants are not printed in the paper and are
written here from that reference.  For ARS(3,4,3) the published 10-digit
decimals are used with the explicit row sums made exact (c-bar consistency).
"""
from __future__ import annotations

import math

import numpy as np

from . import physics as ph
from .basis import Basis
from .dg import Geometry, apply_minv, dg_residual, mass_matrix
from .hdg import HDGSystem, init_facets, init_mixed
from .mesh import Mesh, BC_FARFIELD


class Tableau:
    def __init__(self, name: str):
        self.name = name
        if name == "ARS222":
            g = 1.0 - 1.0 / math.sqrt(2.0)
            d = 1.0 - 1.0 / (2.0 * g)
            self.s = 2
            self.Ae = np.array([[0.0, 0.0, 0.0], [g, 0.0, 0.0], [d, 1.0 - d, 0.0]])
            self.be = np.array([d, 1.0 - d, 0.0])
            self.Ai = np.array([[g, 0.0], [1.0 - g, g]])
            self.bi = np.array([1.0 - g, g])
        elif name == "ARS343":
            r = np.roots([6.0, -18.0, 9.0, -1.0])
            r = np.real(r[(np.abs(np.imag(r)) < 1e-12)])
            g = float(r[(r > 0.4) & (r < 0.5)][0])
            b1 = -1.5 * g * g + 4.0 * g - 0.25
            b2 = 1.5 * g * g - 5.0 * g + 1.25
            a32 = 0.3966543747
            a42 = a43 = 0.5529291479
            self.s = 3
            self.Ae = np.array([[0.0, 0.0, 0.0, 0.0],
                                [g, 0.0, 0.0, 0.0],
                                [(1.0 + g) / 2.0 - a32, a32, 0.0, 0.0],
                                [1.0 - a42 - a43, a42, a43, 0.0]])
            self.be = np.array([0.0, b1, b2, g])
            self.Ai = np.array([[g, 0.0, 0.0], [(1.0 - g) / 2.0, g, 0.0], [b1, b2, g]])
            self.bi = np.array([b1, b2, g])
        else:
            raise ValueError(name)
        self.ce = self.Ae.sum(axis=1)
        self.ci = self.Ai.sum(axis=1)
        self.fsal = bool(np.array_equal(self.be, self.Ae[-1])) and self.ce[-1] == 1.0
        self.stiffly_accurate = bool(np.array_equal(self.bi, self.Ai[-1])) and self.ci[-1] == 1.0


class IMEXSolver:
    """The oracle's full IMEX integrator on one workload."""

    def __init__(self, wl, U0=None):
        self.wl = wl
        self.mesh = Mesh(wl)
        self.basis = Basis(wl.degree)
        self.gas = ph.Gas(wl.gamma, wl.R, wl.mu, wl.Pr)
        self.geo = Geometry(self.mesh, self.basis)
        self.tab = Tableau(wl.tableau)
        self.system = HDGSystem(wl, self.mesh, self.basis, self.gas)
        self.M = mass_matrix(self.basis, self.geo)
        if U0 is None:
            U0 = self.initial_state()
        self.U = np.array(U0, dtype=float)
        self.Uhat = init_facets(self.U, self.mesh, self.basis)
        self.Q = init_mixed(self.U, self.Uhat, self.system)
        self.newton_its = []
        self.ledger = []
        self.mms = None          # (kx, ky, omega): manufactured-solution source (Sec. 5.1.1)
        self.t = 0.0             # time of the current state

    def initial_state(self):
        X, Y = self.mesh.node_coords(self.basis)
        E, nn = X.shape
        elem = np.repeat(np.arange(E)[:, None], nn, axis=1)
        node = np.repeat(np.arange(nn)[None, :], E, axis=0)
        U = self.wl.ic(X, Y, elem, node)                # (4, E, nn)
        return np.moveaxis(U, 0, 1).copy()

    def mass_apply(self, U):
        return np.einsum("enm,evm->evn", self.M, U)

    def dg(self, Y, Q, fluxes=None):
        """R^DG; with a list fluxes, appends the flux of R^DG out of the explicit region
        through the interface faces and through the far-field faces ((4,) each)."""
        faces = {} if fluxes is not None else None
        R = dg_residual(Y, Q, self.wl, self.mesh, self.basis, self.gas, faces=faces)
        if fluxes is not None:
            mesh = self.mesh
            itf, bnd = np.zeros(4), np.zeros(4)
            for f in range(4):
                s, w = faces[f]
                flux = np.einsum("veq,eq->ev", s, w)
                nb = mesh.nbr[:, f]
                explicit = ~mesh.implicit
                itf += flux[explicit & (nb >= 0) & mesh.implicit[np.maximum(nb, 0)]].sum(axis=0)
                bnd += flux[explicit & (nb < 0) & (mesh.bctype[:, f] == BC_FARFIELD)].sum(axis=0)
            fluxes.append((itf, bnd))
        return R

    def totals(self, U=None):
        """Conserved totals sum_T int_T U (4,)."""
        return np.einsum("enm,evm->v", self.M, self.U if U is None else U)

    def step(self):
        """One IMEX step (Alg. imex_scheme_update).  Also appends to self.ledger the
        interface flux-defect ledger of the step: the change of the conserved totals that
        the update formulas imply, split into (i) the interface term
            -dt [ sum_j be_j Phi^DG_j + sum_j bi_j Phi^HDG_j ]  over the faces of Gamma_i,
        Phi^DG_j the flux of R^DG_j out of the explicit elements and Phi^HDG_j that of
        R^HDG_j out of the implicit elements through those faces (the two sides evaluate
        the interface with different stage data, so they do not cancel), and (ii) the same
        sums over the physical boundary faces.  Interior DG faces and (at the converged
        stages) interior HDG facets cancel, so the totals change by (i) + (ii) up to
        roundoff and the Newton tolerance."""
        tab, dt = self.tab, self.wl.dt
        ex, im = self.mesh.ex_elems, self.mesh.im_elems
        Un = self.U.copy()
        Y = self.U.copy()
        Rdg, Rhdg = [], []
        fdg, fhdg = [], []
        src = []                 # (stage weight of each side, load) for the ledger
        its = []

        def load(tt):
            from .mms import source_load
            return source_load(tt, *self.mms, self.mesh, self.basis, self.gas)
        for i in range(1, tab.s + 1):
            Rdg.append(self.dg(Y, self.Q, fdg))
            if self.mms is not None:
                # the source at the explicit stage time (R^DG - b at t_n + cbar_i dt)
                b = load(self.t + tab.ce[i - 1] * dt)
                Rdg[-1] = Rdg[-1] - b
                src.append(("ex", tab.be[i - 1], b))
            acc = sum(tab.Ae[i, j] * Rdg[j] for j in range(i))
            Y[ex] = Un[ex] - dt * apply_minv(acc[ex], self.basis, _sub(self.geo, ex))
            if len(im):
                rhs = self.mass_apply(Un)[im]
                for j in range(i - 1):
                    rhs = rhs - dt * tab.Ai[i - 1, j] * Rhdg[j]
                dta = dt * tab.Ai[i - 1, i - 1]
                bi = None
                if self.mms is not None:
                    # the source at the implicit stage time: M y + dt a_ii (R^HDG(y) - b) = rhs
                    bi = load(self.t + tab.ci[i - 1] * dt)[im]
                    rhs = rhs + dta * bi
                    src.append(("im", tab.bi[i - 1], bi))
                n_it, Rh = self.system.newton(Y, self.Q, self.Uhat, dta, rhs)
                its.append(n_it)
                Rhdg.append(Rh if bi is None else Rh - bi)
                fhdg.append(self.system.face_fluxes(Y, self.Q, self.Uhat, self.system.stage_data(Y, dta, rhs)))
        if tab.fsal:
            self.U[ex] = Y[ex]
        else:
            Rdg.append(self.dg(Y, self.Q, fdg))
            if self.mms is not None:
                b = load(self.t + tab.ce[tab.s] * dt)
                Rdg[-1] = Rdg[-1] - b
                src.append(("ex", tab.be[tab.s], b))
            acc = sum(tab.be[j] * Rdg[j] for j in range(tab.s + 1))
            self.U[ex] = Un[ex] - dt * apply_minv(acc[ex], self.basis, _sub(self.geo, ex))
        if len(im):
            if tab.stiffly_accurate:
                self.U[im] = Y[im]
            else:
                acc = sum(tab.bi[j] * Rhdg[j] for j in range(tab.s))
                self.U[im] = Un[im] - dt * apply_minv(acc, self.basis, _sub(self.geo, im))
        self.newton_its.append(its)
        itf, bnd = np.zeros(4), np.zeros(4)
        for j, (a, b) in enumerate(fdg):
            itf -= dt * tab.be[j] * a
            bnd -= dt * tab.be[j] * b
        for j, (a, b) in enumerate(fhdg):
            itf -= dt * tab.bi[j] * a
            bnd -= dt * tab.bi[j] * b
        srcs = np.zeros(4)
        for side, wgt, b in src:
            srcs += dt * wgt * (b[ex] if side == "ex" else b).sum(axis=(0, 2))
        self.ledger.append({"interface": itf, "boundary": bnd, "source": srcs})
        self.t += dt

    def run(self, steps=None):
        for _ in range(self.wl.steps if steps is None else steps):
            self.step()
        return self.U


class _sub:
    """Geometry restricted to a subset of elements."""

    def __init__(self, geo: Geometry, elems):
        self.jac = geo.jac[elems]
        self.sx = geo.sx[elems]
        self.sy = geo.sy[elems]
        self.fjac = geo.fjac[elems]


def step_jvp(solver: IMEXSolver, dU, dUhat, duinf=None, h=1e-30):
    """Forward-mode derivative of one IMEX step from the solver's current (U_n, Uhat_n):
    returns (U_{n+1}, Uhat_{n+1}, dU_{n+1}, dUhat_{n+1}) along the direction (dU, dUhat) of
    the initial state and, optionally, duinf of the far-field state (u_inf + p duinf at
    p = 0).  The solver itself is not advanced.

    Each step of Alg. imex_scheme_update is differentiated in turn:
    * the mixed variables of U_n lifted from (U_n, Uhat_n), the explicit residuals R^DG_i
      and the final explicit update by the complex step (an exact derivative of the
      real-analytic residuals, to rounding);
    * each implicit stage through its converged root z_i = (y_i, q_i, yhat_i) of
      F(z; rhs_i, y^ex_{i+1}, p) = 0 by the implicit-function theorem,
      dz_i = -J(z_i)^-1 dF/d(rhs_i, y^ex_{i+1}, p), with the monolithic Jacobian J and
      the right-hand side derivative by the complex step at fixed z_i;
    * R^HDG_i at the root and the later right-hand sides rhs_j = M U_n - dt sum a_jk R^HDG_k
      by the same rules.
    Parity: the adjoint of the step satisfies <Ubar, dU> + <Uhatbar, dUhat> + pbar dp =
    <Ubar_{n+1}, dU_{n+1}> + <Uhatbar_{n+1}, dUhat_{n+1}> for every direction."""
    if getattr(solver, "mms", None) is not None:
        raise NotImplementedError("step_jvp does not carry the manufactured-solution source")
    import dataclasses as _dc
    import scipy.sparse.linalg as _spla

    from .dg import dg_residual as _dgr
    tab, dt = solver.tab, solver.wl.dt
    wl0 = solver.wl
    sysm = solver.system
    ex, im = solver.mesh.ex_elems, solver.mesh.im_elems
    du = np.zeros(4) if duinf is None else np.asarray(duinf, dtype=float)
    wl_c = _dc.replace(wl0, u_inf=wl0.u_inf + 1j * h * du)    # complex far-field state
    basis, mesh, gas = solver.basis, solver.mesh, solver.gas

    def dgr(Y, Q, dY, dQ):
        Yc = Y + 1j * h * dY
        Qc = None if Q is None else Q + 1j * h * dQ
        R = _dgr(Yc, Qc, wl_c, mesh, basis, gas)
        return np.real(R), np.imag(R) / h

    def minv(X, elems):
        return apply_minv(X[elems], basis, _sub(solver.geo, elems))

    Un = solver.U.copy()
    Hn = solver.Uhat.copy()
    dUn = np.array(dU, dtype=float)
    dHn = np.array(dUhat, dtype=float)
    Qc = init_mixed(Un + 1j * h * dUn, Hn + 1j * h * dHn, sysm)
    Q, dQ = np.real(Qc), np.imag(Qc) / h
    Y, dY = Un.copy(), dUn.copy()
    H, dH = Hn.copy(), dHn.copy()
    Rdg, dRdg, Rh, dRh = [], [], [], []
    Mn, dMn = solver.mass_apply(Un), solver.mass_apply(dUn)
    for i in range(1, tab.s + 1):
        R, dR = dgr(Y, Q if sysm.mx else None, dY, dQ)
        Rdg.append(R)
        dRdg.append(dR)
        acc = sum(tab.Ae[i, j] * Rdg[j] for j in range(i))
        dacc = sum(tab.Ae[i, j] * dRdg[j] for j in range(i))
        Y[ex] = Un[ex] - dt * minv(acc, ex)
        dY[ex] = dUn[ex] - dt * minv(dacc, ex)
        if not len(im):
            continue
        rhs = Mn[im] - sum(dt * tab.Ai[i - 1, j] * Rh[j] for j in range(i - 1)) if i > 1 else Mn[im].copy()
        drhs = dMn[im] - sum(dt * tab.Ai[i - 1, j] * dRh[j] for j in range(i - 1)) if i > 1 else dMn[im].copy()
        dta = dt * tab.Ai[i - 1, i - 1]
        sysm.newton(Y, Q, H, dta, rhs)                      # the root (in place)
        z = sysm.pack(Y, Q, H)
        sd = sysm.stage_data(Y, dta, rhs)
        J = sysm.jacobian(z, sd)
        # dF/d(rhs, y^ex, p) along (drhs, dy^ex, dp) at fixed z
        sd_c = sysm.stage_data(Y + 1j * h * dY, dta, rhs + 1j * h * drhs)
        sysm.wl = wl_c
        try:
            Fc, _ = _residual_complex(sysm, z, sd_c)
        finally:
            sysm.wl = wl0
        dz = _spla.spsolve(J.tocsc(), -np.imag(Fc) / h)
        dYim = np.zeros_like(Y)
        dQim = np.zeros_like(Q)
        dHim = np.zeros_like(H)
        sysm.unpack(dz, dYim, dQim, dHim)
        dY[im] = dYim[im]
        if sysm.mx:
            dQ = dQim
        dH = dHim
        # R^HDG at the root and its derivative (z and the stage data move together)
        sysm.wl = wl_c
        try:
            _, Rc = _residual_complex(sysm, z + 1j * h * dz, sd_c)
        finally:
            sysm.wl = wl0
        Rh.append(np.real(Rc))
        dRh.append(np.imag(Rc) / h)
    U1, dU1 = Y.copy(), dY.copy()
    if not tab.fsal:
        R, dR = dgr(Y, Q if sysm.mx else None, dY, dQ)
        Rdg.append(R)
        dRdg.append(dR)
        acc = sum(tab.be[j] * Rdg[j] for j in range(tab.s + 1))
        dacc = sum(tab.be[j] * dRdg[j] for j in range(tab.s + 1))
        U1[ex] = Un[ex] - dt * minv(acc, ex)
        dU1[ex] = dUn[ex] - dt * minv(dacc, ex)
    if len(im) and not tab.stiffly_accurate:
        raise NotImplementedError("implicit tableaux that are not stiffly accurate")
    return U1, H, dU1, dH


def _residual_complex(sysm, z, sd):
    """HDGSystem.residual for complex z or stage data (the global assembly in complex)."""
    zl = z[sysm.locmap]
    out, Rh = sysm.local_out(zl, sd)
    F = np.zeros(sysm.N, dtype=complex)
    np.add.at(F, sysm.locmap.reshape(-1), out.reshape(-1))
    return F, Rh
