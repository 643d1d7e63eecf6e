"""Implicit HDG stage system and its Newton solve (oracle; test infrastructure only).

Stage equations of the SDIRK part (eqs. dirk_stage_update_solution / _facet /
_mixed):
    f = M y + dt a_ii R^HDG(y, yhat, ytilde) - rhs = 0       (element rows)
    g = Rtilde(y, yhat, ytilde)                        = 0   (mixed rows, HDG-MX)
    h = Rhat(y, yhat, ytilde, y^ex_{i+1})              = 0   (facet rows)
with rhs = M U_n - dt sum_{j<i} a_ij R^HDG_j.

R^HDG per implicit element:
  HDG-IP (eq. bilinear_form_interior_hdg_ip_element): volume term, the
  convective flux Fhat*(U, Uhat) on all of dT, and on dT minus walls the
  viscous surface, adjoint and penalty terms with K evaluated at Uhat
  (alpha = 10); wall faces use K_w (App. B.2.2).
  HDG-MX (eq. bilinear_form_hdg_mixed): volume term with F^nu(U, eps, phi) and
  int_dT (Fhat* - F^{nu,*}_n) . V with F^{nu,*}_n = F^nu_n(Uhat, eps, phi) - S_d (U - Uhat),
  S_d = diag(0, mu, mu, kappa) (eq. viscous_numerical_flux).
Facet rows:
  interior facets: the transmission forms (eq. bilinear_form_interior_hdg_ip_facet, MX form),
  interface facets: int (Uhat - U^ex) . Vhat (eq. interface_bilinearform_implicit_facet),
  far-field facets: int (A^+(Uhat)(Uhat - U) - A^-(Uhat)(Uhat - U_inf)) . Vhat (App. B.2.1),
  walls: HDG-IP Uhat = U_w = (rho, 0, 0, rho e_i) of the element trace (App. B.2.2);
         HDG-MX (rhohat - rho, rhohat u, kappa phi.n - kappa (rhoE - rhoEhat)) (App. B.3.2).
Mixed rows (HDG-MX): the eps and phi equations of eq. bilinear_form_hdg_mixed with
symmetric test tensors; eps : zeta counts the off-diagonal entry twice.

Newton (Sec. 4.3): the monolithic system over (U, Q, Uhat) of all implicit
elements and HDG facets is linearised with the exact Jacobian (complex-step
derivatives of each element's local residual, assembled globally) and solved
with a sparse direct factorisation -- no static condensation, so that the
condensed HIP path is checked against an independent route to the same root.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import physics as ph
from .basis import Basis
from .dg import Geometry, face_eval, outer_n, test_face, test_volume, vol_eval
from .mesh import KIND_FARFIELD, KIND_INTERFACE, KIND_INTERIOR, KIND_WALL, Mesh, OPPOSITE
from paper_2607_16044_amd.workloads import HDG_FLUX_LF, HDG_MX

# symmetric test tensors for (eps11, eps12, eps22)
SYM_BASIS = [np.array([[1.0, 0.0], [0.0, 0.0]]),
             np.array([[0.0, 1.0], [1.0, 0.0]]),
             np.array([[0.0, 0.0], [0.0, 1.0]])]


class BatchGeometry:
    def __init__(self, geo: Geometry, mesh: Mesh, elems):
        self.jac = geo.jac[elems]
        self.sx = geo.sx[elems]
        self.sy = geo.sy[elems]
        self.fjac = geo.fjac[elems]
        self.lchar = mesh.lchar[elems]


class StageData:
    """Per-stage data of the implicit elements: interface traces, dt a_ii and rhs."""

    def __init__(self, kind, uex_fq, dt_a, rhs):
        self.kind = kind          # (B, 4) facet kinds
        self.uex_fq = uex_fq      # (B, 4, 4, Qf) explicit traces on interface faces
        self.dt_a = dt_a
        self.rhs = rhs            # (B, 4, nn)


def local_residual(U, Q, Uh, sd: StageData, wl, basis: Basis, bg: BatchGeometry, gas: ph.Gas, faces=None):
    """Element-local stage residual.

    U (B, 4, nn), Q (B, 5, nn) or None, Uh (B, 4 faces, 4, k+1).
    Returns f (B, 4, nn), g (B, 5, nn) or None, h (B, 4 faces, 4, k+1), Rh (B, 4, nn).
    faces: optional dict; faces[f] receives (s, w), the part of R^HDG's face-f integrand
    tested against V itself ((4, B, Qf)) and the face quadrature weights ((B, Qf)).
    """
    k = basis.k
    mx = wl.hdg_variant == HDG_MX and wl.viscous
    Uq, Gq = vol_eval(U, basis, bg)
    vol = -ph.convective_flux(Uq, gas)
    if wl.viscous:
        if mx:
            Qq = np.einsum("qn,ecn->ceq", basis.phi, Q)
            vol = vol + ph.viscous_flux_mixed(Uq, Qq[:3], Qq[3:], gas)
        else:
            vol = vol + ph.viscous_flux(Uq, Gq, gas)
    Rh = test_volume(vol, basis, bg)
    B = U.shape[0]
    h = np.zeros((B, 4, 4, k + 1), dtype=np.result_type(U, Uh, sd.uex_fq, sd.rhs, wl.u_inf, float))
    tau = wl.alpha_hdg * (k + 1) ** 2 / bg.lchar
    uinf = wl.u_inf.reshape(4, 1, 1)
    wf_all = []
    for f in range(4):
        n = Basis.NORMALS[f]
        kind = sd.kind[:, f]
        Uf, Gf = face_eval(U, f, basis, bg)
        Uhq = np.einsum("qm,bvm->vbq", basis.psi, Uh[:, f])
        if wl.hdg_flux == HDG_FLUX_LF:
            Fc = ph.flux_hdg_lf(Uf, Uhq, n, gas)
        else:
            Fc = ph.flux_hdg_fvs(Uf, Uhq, n, gas)
        s = Fc
        g = None
        t_int = -Fc
        eps_f = phi_f = None
        if wl.viscous:
            if mx:
                Qf = np.einsum("qn,ecn->ceq", basis.fphi[f], Q)
                eps_f, phi_f = Qf[:3], Qf[3:]
                Sd = np.array([0.0, gas.mu, gas.mu, gas.kappa]).reshape(4, 1, 1)
                Fvs = ph.normal_flux(ph.viscous_flux_mixed(Uhq, eps_f, phi_f, gas), n) - Sd * (Uf - Uhq)
                s = Fc - Fvs
                t_int = Fc - Fvs
            else:
                wall = (kind == KIND_WALL)[None, None, :, None]
                Gj = outer_n(Uf - Uhq, n)
                Kg = ph.viscous_flux(Uhq, Gf, gas)
                Kj = ph.viscous_flux(Uhq, Gj, gas)
                Kg_w = ph.viscous_flux(Uhq, Gf, gas, adiabatic_normal=n)
                Kj_w = ph.viscous_flux(Uhq, Gj, gas, adiabatic_normal=n)
                Kg = np.where(wall, Kg_w, Kg)
                Kj = np.where(wall, Kj_w, Kj)
                tq = tau[None, :, None]
                visc_s = -ph.normal_flux(Kg, n) + tq * ph.normal_flux(Kj, n)
                s = Fc + visc_s
                g = -Kj
                t_int = -Fc + ph.normal_flux(Kg, n) - tq * ph.normal_flux(Kj, n)
        if faces is not None:
            faces[f] = (s, basis.qw[None, :] * bg.fjac[:, f][:, None])
        Rh = Rh + test_face(s, g, f, basis, bg)
        # facet rows
        Uex = np.moveaxis(sd.uex_fq[:, f], 0, 1)                 # (4, B, Qf)
        t_itf = Uhq - Uex
        Ap, Am = ph.char_split(Uhq, n, gas)
        t_far = ph.matvec(Ap, Uhq - Uf) - ph.matvec(Am, Uhq - np.broadcast_to(uinf, Uf.shape))
        if mx:
            rho = Uf[0]
            phin = phi_f[0] * n[0] + phi_f[1] * n[1]
            t_wall = np.stack([Uhq[0] - rho, Uhq[1], Uhq[2],
                               gas.kappa * phin - gas.kappa * (Uf[3] - Uhq[3])])
        else:
            rho = Uf[0]
            rhoei = Uf[3] - 0.5 * (Uf[1] ** 2 + Uf[2] ** 2) / rho
            Uw = np.stack([rho, 0.0 * rho, 0.0 * rho, rhoei])
            t_wall = Uhq - Uw
        kb = kind[None, :, None]
        t = np.where(kb == KIND_INTERIOR, t_int,
                     np.where(kb == KIND_INTERFACE, t_itf,
                              np.where(kb == KIND_FARFIELD, t_far, t_wall)))
        wf = basis.qw[None, :] * bg.fjac[:, f][:, None]
        wf_all.append(wf)
        h[:, f] = np.einsum("vbq,qm,bq->bvm", t, basis.psi, wf)
    # element rows
    wv = basis.wvol[None, :] * bg.jac[:, None]
    MU = np.einsum("veq,qn,eq->evn", Uq, basis.phi, wv)
    f_rows = MU + sd.dt_a * Rh - sd.rhs
    g_rows = None
    if mx:
        g_rows = mixed_residual(U, Q, Uh, basis, bg, gas, wf_all)
    return f_rows, g_rows, h, Rh


def mixed_residual(U, Q, Uh, basis: Basis, bg: BatchGeometry, gas: ph.Gas, wf_all):
    """Rtilde: the eps and phi equations of eq. bilinear_form_hdg_mixed."""
    rho, u, v, E, p, theta, c, H = ph.primitives(np.einsum("qn,evn->veq", basis.phi, U), gas)
    vel = [u, v]
    Qq = np.einsum("qn,ecn->ceq", basis.phi, Q)
    epsq = np.array([[Qq[0], Qq[1]], [Qq[1], Qq[2]]])            # (2, 2, B, Qv)
    phiq = Qq[3:]
    wv = basis.wvol[None, :] * bg.jac[:, None]
    dphi = [np.einsum("qn,e->eqn", basis.dxi, bg.sx), np.einsum("qn,e->eqn", basis.deta, bg.sy)]
    B = U.shape[0]
    g = np.zeros((B, 5, basis.nn), dtype=np.result_type(U, Q, Uh, float))
    for cidx, Esym in enumerate(SYM_BASIS):
        Zt = Esym - np.trace(Esym) / 3.0 * np.eye(2)
        epsE = sum(epsq[i, j] * Esym[i, j] for i in range(2) for j in range(2))
        g[:, cidx] += np.einsum("eq,qn,eq->en", epsE, basis.phi, wv)
        for i in range(2):
            for j in range(2):
                if Zt[i, j] != 0.0:
                    g[:, cidx] += Zt[i, j] * np.einsum("eq,eqn,eq->en", vel[i], dphi[j], wv)
    for d in range(2):
        g[:, 3 + d] += np.einsum("eq,qn,eq->en", phiq[d], basis.phi, wv)
        g[:, 3 + d] += np.einsum("eq,eqn,eq->en", theta, dphi[d], wv)
    for f in range(4):
        n = Basis.NORMALS[f]
        Uhq = np.einsum("qm,bvm->vbq", basis.psi, Uh[:, f])
        _, uh, vh, _, _, thh, _, _ = ph.primitives(Uhq, gas)
        velh = [uh, vh]
        wf = wf_all[f]
        for cidx, Esym in enumerate(SYM_BASIS):
            Zt = Esym - np.trace(Esym) / 3.0 * np.eye(2)
            for i in range(2):
                for j in range(2):
                    if Zt[i, j] != 0.0 and n[j] != 0.0:
                        g[:, cidx] -= Zt[i, j] * n[j] * np.einsum("eq,qn,eq->en", velh[i], basis.fphi[f], wf)
        for d in range(2):
            if n[d] != 0.0:
                g[:, 3 + d] -= n[d] * np.einsum("eq,qn,eq->en", thh, basis.fphi[f], wf)
    return g


class HDGSystem:
    """Global numbering of the monolithic stage system and its Newton solve."""

    def __init__(self, wl, mesh: Mesh, basis: Basis, gas: ph.Gas):
        self.wl, self.mesh, self.basis, self.gas = wl, mesh, basis, gas
        self.geo = Geometry(mesh, basis)
        self.mx = wl.hdg_variant == HDG_MX and wl.viscous
        self.elems = mesh.im_elems
        self.B = len(self.elems)
        self.bg = BatchGeometry(self.geo, mesh, self.elems)
        nn, k1 = basis.nn, basis.k + 1
        self.nU = 4 * nn
        self.nQ = 5 * nn if self.mx else 0
        self.nF = 4 * k1
        B = self.B
        self.offQ = B * self.nU
        self.offH = B * (self.nU + self.nQ)
        self.N = self.offH + mesh.n_hdg * self.nF
        pos = np.arange(B)
        loc = []
        loc.append(pos[:, None] * self.nU + np.arange(self.nU)[None, :])
        if self.mx:
            loc.append(self.offQ + pos[:, None] * self.nQ + np.arange(self.nQ)[None, :])
        hidx = mesh.hdg_index[mesh.efacet[self.elems]].reshape(B, 4)        # (B, 4)
        assert np.all(hidx >= 0)
        loc.append((self.offH + hidx[:, :, None] * self.nF + np.arange(self.nF)[None, None, :]).reshape(B, 4 * self.nF))
        self.locmap = np.concatenate(loc, axis=1)                           # (B, nloc)
        self.nloc = self.locmap.shape[1]
        self.kind = mesh.face_kind[self.elems]

    # -- packing ----------------------------------------------------------
    def pack(self, U_all, Q_all, Uhat):
        z = np.zeros(self.N, dtype=np.result_type(U_all, Uhat, float) if Q_all is None
                     else np.result_type(U_all, Q_all, Uhat, float))
        z[:self.offQ] = U_all[self.elems].reshape(-1)
        if self.mx:
            z[self.offQ:self.offH] = Q_all[self.elems].reshape(-1)
        z[self.offH:] = Uhat.reshape(-1)
        return z

    def unpack(self, z, U_all, Q_all, Uhat):
        nn, k1 = self.basis.nn, self.basis.k + 1
        U_all[self.elems] = z[:self.offQ].reshape(self.B, 4, nn)
        if self.mx:
            Q_all[self.elems] = z[self.offQ:self.offH].reshape(self.B, 5, nn)
        Uhat[:] = z[self.offH:].reshape(-1, 4, k1)

    def split_local(self, zl):
        nn, k1 = self.basis.nn, self.basis.k + 1
        B = zl.shape[0]
        U = zl[:, :self.nU].reshape(B, 4, nn)
        o = self.nU
        Q = None
        if self.mx:
            Q = zl[:, o:o + self.nQ].reshape(B, 5, nn)
            o += self.nQ
        Uh = zl[:, o:].reshape(B, 4, 4, k1)
        return U, Q, Uh

    def local_out(self, zl, sd, faces=None):
        U, Q, Uh = self.split_local(zl)
        f, g, h, Rh = local_residual(U, Q, Uh, sd, self.wl, self.basis, self.bg, self.gas, faces=faces)
        parts = [f.reshape(self.B, -1)]
        if self.mx:
            parts.append(g.reshape(self.B, -1))
        parts.append(h.reshape(self.B, -1))
        return np.concatenate(parts, axis=1), Rh

    # -- stage data ---------------------------------------------------------
    def stage_data(self, U_all, dt_a, rhs_im):
        mesh, basis = self.mesh, self.basis
        B = self.B
        uex = np.zeros((B, 4, 4, basis.nq), dtype=np.result_type(U_all, float))
        for f in range(4):
            nb = mesh.nbr[self.elems, f]
            itf = self.kind[:, f] == KIND_INTERFACE
            if np.any(itf):
                vals, _ = face_eval(U_all, OPPOSITE[f], basis, self.geo)       # (4, E, Qf)
                uex[itf, f] = np.moveaxis(vals[:, nb[itf]], 0, 1)
        return StageData(self.kind, uex, dt_a, rhs_im)

    def face_fluxes(self, U_all, Q_all, Uhat, sd):
        """Flux of R^HDG out of the implicit region through its interface faces and through
        its physical boundary faces (far field and walls): two (4,) vectors, each the sum
        over those faces of int_F s . 1 ds with s the face integrand tested against V (the
        element rows tested with V = 1 sum to these face integrals: the volume term and the
        adjoint term, tested against grad V, vanish)."""
        z = self.pack(U_all, Q_all, Uhat)
        faces = {}
        self.local_out(z[self.locmap], sd, faces=faces)
        itf = np.zeros(4)
        bnd = np.zeros(4)
        for f in range(4):
            s, w = faces[f]
            flux = np.einsum("vbq,bq->bv", s, w)
            itf += flux[self.kind[:, f] == KIND_INTERFACE].sum(axis=0)
            bnd += flux[(self.kind[:, f] == KIND_FARFIELD) | (self.kind[:, f] == KIND_WALL)].sum(axis=0)
        return itf, bnd

    # -- residual and Jacobian ---------------------------------------------
    def residual(self, z, sd):
        zl = z[self.locmap]
        out, Rh = self.local_out(zl, sd)
        F = np.zeros(self.N)
        np.add.at(F, self.locmap.reshape(-1), out.reshape(-1))
        return F, Rh

    def local_jacobian(self, z, sd, hstep=1e-30):
        """Complex-step Jacobian of every element's local residual: (B, nloc, nloc)."""
        zl = z[self.locmap].astype(complex)
        J = np.zeros((self.B, self.nloc, self.nloc))
        for j in range(self.nloc):
            zp = zl.copy()
            zp[:, j] += 1j * hstep
            out, _ = self.local_out(zp, sd)
            J[:, :, j] = out.imag / hstep
        return J

    def jacobian(self, z, sd):
        J = self.local_jacobian(z, sd)
        rows = np.repeat(self.locmap[:, :, None], self.nloc, axis=2).reshape(-1)
        cols = np.repeat(self.locmap[:, None, :], self.nloc, axis=1).reshape(-1)
        return sp.csc_matrix((J.reshape(-1), (rows, cols)), shape=(self.N, self.N))

    def newton(self, U_all, Q_all, Uhat, dt_a, rhs_im, rtol=1e-12, maxit=30):
        """Solve the stage system in place; returns (iterations, R^HDG of implicit elements).

        Stops once the increments of U and Uhat are below rtol times the largest
        |U| and |Uhat| (the mixed variables follow from them)."""
        sd = self.stage_data(U_all, dt_a, rhs_im)
        z = self.pack(U_all, Q_all, Uhat)
        its = 0
        sU = np.max(np.abs(z[:self.offQ]))
        sH = np.max(np.abs(z[self.offH:])) if self.N > self.offH else 1.0
        for its in range(1, maxit + 1):
            F, _ = self.residual(z, sd)
            J = self.jacobian(z, sd)
            rs = 1.0 / np.maximum(abs(J).max(axis=1).toarray().ravel(), 1e-300)
            Dr = sp.diags(rs)
            dz = spla.spsolve((Dr @ J).tocsc(), -rs * F)
            z = z + dz
            if (np.max(np.abs(dz[:self.offQ])) <= rtol * sU and
                    (self.N == self.offH or np.max(np.abs(dz[self.offH:])) <= rtol * sH)):
                break
        else:
            raise RuntimeError("oracle Newton did not converge")
        self.unpack(z, U_all, Q_all, Uhat)
        _, Rh = self.residual(z, sd)
        return its, Rh


def init_facets(U_all, mesh: Mesh, basis: Basis):
    """Initial facet state: mean of the adjacent element traces at the facet nodes.

    Interface facets take the explicit element's trace (their Dirichlet value);
    boundary facets the single adjacent trace."""
    k1 = basis.k + 1
    Uhat = np.zeros((mesh.n_hdg, 4, k1))
    for hf, F in enumerate(mesh.hdg_facets):
        eL, fL, eR, fR = mesh.facets[F]
        sides = [(e, f) for (e, f) in ((eL, fL), (eR, fR)) if e >= 0]
        ex = [(e, f) for (e, f) in sides if not mesh.implicit[e]]
        use = ex if ex else sides
        acc = np.zeros((4, k1))
        for (e, f) in use:
            acc += np.einsum("mn,vn->vm", basis.trace_at_fnodes[f], U_all[e])
        Uhat[hf] = acc / len(use)
    return Uhat


def init_mixed(U_all, Uhat, system: HDGSystem):
    """Mixed variables solving Rtilde = 0 for given (U, Uhat).

    Rtilde is affine in Q: Rtilde(Q) = Rtilde(0) + A Q, with A probed column by column."""
    nn = system.basis.nn
    Q_all = np.zeros((U_all.shape[0], 5, nn), dtype=np.result_type(U_all, Uhat, float))
    if not system.mx or system.B == 0:
        return Q_all
    z = system.pack(U_all, Q_all, Uhat)
    U, Q, Uh = system.split_local(z[system.locmap])
    wf_all = [system.basis.qw[None, :] * system.bg.fjac[:, f][:, None] for f in range(4)]
    g0 = mixed_residual(U, np.zeros_like(Q), Uh, system.basis, system.bg, system.gas, wf_all)
    A = np.zeros((system.B, 5 * nn, 5 * nn))
    for j in range(5 * nn):
        Qp = np.zeros_like(Q)
        Qp[:, j // nn, j % nn] = 1.0
        # the coefficients of Q are mass-matrix terms, real for complex (U, Uhat) as well
        A[:, :, j] = np.real(mixed_residual(U, Qp, Uh, system.basis, system.bg, system.gas, wf_all)
                             - g0).reshape(system.B, -1)
    sol = np.linalg.solve(A, -g0.reshape(system.B, -1, 1))[..., 0]
    Q_all[system.elems] = sol.reshape(system.B, 5, nn)
    return Q_all


def wall_shear(Q_all, mesh: Mesh, basis: Basis, gas: ph.Gas) -> float:
    """Integral over the implicit region's adiabatic walls of the wall shear
    mu (du/dy + dv/dx) = 2 mu eps_12, with eps_12 the stored off-diagonal strain of the
    HDG-MX mixed variables (Sec. 3.5) evaluated at the face Gauss points (the integrand of
    a time-averaged wall-shear objective)."""
    J = 0.0
    for e in mesh.im_elems:
        for f in range(4):
            if mesh.face_kind[e, f] != KIND_WALL:
                continue
            ds = 0.5 * (mesh.hy[e] if f < 2 else mesh.hx[e])
            eps12 = basis.fphi[f] @ Q_all[e, 1]
            J += 2.0 * gas.mu * float(np.sum(basis.qw * eps12)) * ds
    return J
