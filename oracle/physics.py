"""Compressible-flow fluxes and numerical fluxes (oracle; test infrastructure only).

Sec. 2: conservative variables U = (rho, rho u, rho v, rho E), convective flux
F^c and viscous flux F^nu (eq. inviscid_viscous_fluxes), ideal gas p = rho R theta,
Fourier heat flux q = -kappa grad(theta), Newtonian stress with lambda = -2mu/3,
kappa = c_p mu / Pr.

The quasi-linear form F^nu_i = K_ij dU/dx_j (eq. definition_jacobians) is used
through ``viscous_flux(W, G)``: the viscous flux evaluated at state W with the
conservative gradient replaced by G.  Because F^nu is linear in the gradient,
viscous_flux(W, G) = K(W) G for any G; every K-product of the IP forms is such
an evaluation.

All functions are complex-step safe: branches (max, |.|, sign of an
eigenvalue) are decided on the real part, and only analytic operations act on
the values.  State arrays carry the variable on axis 0; fluxes are (4, 2, ...)
with axis 1 the direction.
"""
from __future__ import annotations

import numpy as np


class Gas:
    def __init__(self, gamma: float, R: float, mu: float, Pr: float):
        self.gamma = gamma
        self.R = R
        self.mu = mu
        self.Pr = Pr
        self.cv = R / (gamma - 1.0)
        self.cp = gamma * R / (gamma - 1.0)
        self.kappa = self.cp * mu / Pr
        self.lam = -2.0 * mu / 3.0


def rabs(x):
    return np.where(np.real(x) >= 0, x, -x)


def rmax(a, b):
    return np.where(np.real(a) >= np.real(b), a, b)


def primitives(U, gas: Gas):
    rho = U[0]
    u = U[1] / rho
    v = U[2] / rho
    E = U[3] / rho
    ek = 0.5 * (u * u + v * v)
    ei = E - ek
    theta = ei / gas.cv
    p = rho * gas.R * theta
    c = np.sqrt(gas.gamma * gas.R * theta)
    H = E + p / rho
    return rho, u, v, E, p, theta, c, H


def convective_flux(U, gas: Gas):
    rho, u, v, E, p, theta, c, H = primitives(U, gas)
    F = np.empty((4, 2) + np.shape(rho), dtype=np.result_type(U, float))
    F[0, 0] = rho * u
    F[1, 0] = rho * u * u + p
    F[2, 0] = rho * v * u
    F[3, 0] = rho * H * u
    F[0, 1] = rho * v
    F[1, 1] = rho * u * v
    F[2, 1] = rho * v * v + p
    F[3, 1] = rho * H * v
    return F


def normal_flux(F, n):
    """F_n = sum_i F_i n_i for a (4, 2, ...) flux and a normal (2,) or (2, ...)."""
    return F[:, 0] * n[0] + F[:, 1] * n[1]


def _stress_and_heat(gu, gv, gtheta, gas: Gas):
    div = gu[0] + gv[1]
    t11 = 2.0 * gas.mu * gu[0] + gas.lam * div
    t22 = 2.0 * gas.mu * gv[1] + gas.lam * div
    t12 = gas.mu * (gu[1] + gv[0])
    q = [-gas.kappa * gtheta[0], -gas.kappa * gtheta[1]]
    return t11, t12, t22, q


def viscous_flux(W, G, gas: Gas, adiabatic_normal=None):
    """F^nu at state W with conservative gradient G (4, 2, ...): equals K(W) G.

    With ``adiabatic_normal`` = n the heat flux is replaced by q - (q.n) n (the
    adiabatic-wall flux F^{nu,w} of eq. adiabatic_viscous_flux_compact).
    """
    rho = W[0]
    u = W[1] / rho
    v = W[2] / rho
    E = W[3] / rho
    gu = [(G[1, d] - u * G[0, d]) / rho for d in range(2)]
    gv = [(G[2, d] - v * G[0, d]) / rho for d in range(2)]
    gE = [(G[3, d] - E * G[0, d]) / rho for d in range(2)]
    gei = [gE[d] - u * gu[d] - v * gv[d] for d in range(2)]
    gtheta = [gei[d] / gas.cv for d in range(2)]
    t11, t12, t22, q = _stress_and_heat(gu, gv, gtheta, gas)
    if adiabatic_normal is not None:
        n = adiabatic_normal
        qn = q[0] * n[0] + q[1] * n[1]
        q = [q[0] - qn * n[0], q[1] - qn * n[1]]
    F = np.empty((4, 2) + np.shape(rho), dtype=np.result_type(W, G, float))
    F[0, 0] = 0.0
    F[1, 0] = t11
    F[2, 0] = t12
    F[3, 0] = t11 * u + t12 * v - q[0]
    F[0, 1] = 0.0
    F[1, 1] = t12
    F[2, 1] = t22
    F[3, 1] = t12 * u + t22 * v - q[1]
    return F


def viscous_flux_mixed(W, eps, phi, gas: Gas):
    """F^nu(U, eps, phi) of Sec. 3.5; eps = (e11, e12, e22), phi = grad(theta)."""
    rho = W[0]
    u = W[1] / rho
    v = W[2] / rho
    m2 = 2.0 * gas.mu
    F = np.empty((4, 2) + np.shape(rho), dtype=np.result_type(W, eps, phi, float))
    F[0, 0] = 0.0
    F[1, 0] = m2 * eps[0]
    F[2, 0] = m2 * eps[1]
    F[3, 0] = m2 * (eps[0] * u + eps[1] * v) + gas.kappa * phi[0]
    F[0, 1] = 0.0
    F[1, 1] = m2 * eps[1]
    F[2, 1] = m2 * eps[2]
    F[3, 1] = m2 * (eps[1] * u + eps[2] * v) + gas.kappa * phi[1]
    return F


def _as_last(W):
    return np.moveaxis(W, 0, -1)


def char_split(W, n, gas: Gas):
    """A_n^+ and A_n^- at state W (Sec. 3.2, eq. inviscid_jacobian_eigendecomposition).

    A_n = P Lambda P^-1 with the closed-form right eigenvectors of the 2D Euler
    normal Jacobian (eigenvalues u_n - c, u_n, u_n, u_n + c); P^-1 by a
    numerical inverse.  Lambda^+ = max(lambda, 0), Lambda^- = min(lambda, 0).
    Returns arrays of shape (..., 4, 4).
    """
    rho, u, v, E, p, theta, c, H = primitives(W, gas)
    nx, ny = n[0], n[1]
    un = u * nx + v * ny
    ut = -u * ny + v * nx
    one = np.ones_like(rho)
    zero = np.zeros_like(rho)
    nxa = nx * one
    nya = ny * one
    cols = [
        [one, u - c * nxa, v - c * nya, H - c * un],
        [one, u, v, 0.5 * (u * u + v * v)],
        [zero, -nya, nxa, ut],
        [one, u + c * nxa, v + c * nya, H + c * un],
    ]
    P = np.stack([np.stack(col, axis=-1) for col in cols], axis=-1)   # (..., 4 rows, 4 cols)
    lam = np.stack([un - c, un, un, un + c], axis=-1)
    lp = np.where(np.real(lam) > 0, lam, 0.0 * lam)
    lm = np.where(np.real(lam) < 0, lam, 0.0 * lam)
    Pinv = np.linalg.inv(P)
    Ap = np.einsum("...ij,...j,...jk->...ik", P, lp, Pinv)
    Am = np.einsum("...ij,...j,...jk->...ik", P, lm, Pinv)
    return Ap, Am


def matvec(A, x):
    """(..., 4, 4) times a state (4, ...) -> state (4, ...)."""
    return np.moveaxis(np.einsum("...ij,...j->...i", A, _as_last(x)), -1, 0)


def flux_vijayasundaram(U, UN, n, gas: Gas):
    """DG numerical flux A_n^+(Ubar) U + A_n^-(Ubar) U^- (eq. upwinding_Vijayasundaram_sdg)."""
    Ap, Am = char_split(0.5 * (U + UN), n, gas)
    return matvec(Ap, U) + matvec(Am, UN)


def max_wave_speed(W, n, gas: Gas):
    rho, u, v, E, p, theta, c, H = primitives(W, gas)
    return rabs(u * n[0] + v * n[1]) + c


def flux_lax_friedrichs(U, UN, n, gas: Gas):
    """Local Lax-Friedrichs: mean of the normal fluxes plus lambda_max/2 times the jump."""
    lam = rmax(max_wave_speed(U, n, gas), max_wave_speed(UN, n, gas))
    Fn = normal_flux(convective_flux(U, gas), n)
    FnN = normal_flux(convective_flux(UN, gas), n)
    return 0.5 * (Fn + FnN) + 0.5 * lam * (U - UN)


def flux_hdg_fvs(U, Uh, n, gas: Gas):
    """HDG convective flux F_n(Uhat) + A_n^+(Uhat)(U - Uhat) (eq. inviscid_numerical_flux)."""
    Ap, Am = char_split(Uh, n, gas)
    return normal_flux(convective_flux(Uh, gas), n) + matvec(Ap, U - Uh)


def flux_hdg_lf(U, Uh, n, gas: Gas):
    """HDG convective flux with S_c = lambda_max(Uhat) I."""
    lam = max_wave_speed(Uh, n, gas)
    return normal_flux(convective_flux(Uh, gas), n) + lam * (U - Uh)


def farfield_dg_flux(U, Uinf, n, gas: Gas):
    """A_n(U) U_Gamma = A_n^+(U) U + A_n^-(U) U_inf (App. B.1.1, characteristic boundary state)."""
    Ap, Am = char_split(U, n, gas)
    return matvec(Ap, U) + matvec(Am, Uinf)
