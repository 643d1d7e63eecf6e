"""Pins of the oracle's basis, quadrature and flux functions (CPU only).

Each check compares against something other than the oracle itself: exact
integrals, the Lagrange property, the inviscid and viscous Jacobian matrices
printed in App. A of the paper (with the two sign fixes stated there), closed
forms of the eigen-decomposition, and flux consistency identities.
"""
import math

import numpy as np
import pytest

from oracle import physics as ph
from oracle.basis import Basis, quad_points


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_quadrature_exactness_and_lagrange(k):
    b = Basis(k)
    assert b.nq == {1: 2, 2: 4, 3: 5, 4: 7}[k]
    assert 2 * b.nq - 1 >= 3 * k
    for m in range(2 * b.nq):
        exact = 0.0 if m % 2 else 2.0 / (m + 1)
        assert abs(np.sum(b.qw * b.qx ** m) - exact) < 1e-14
    # Lagrange property at the nodes and exact interpolation of polynomials of degree <= k
    from oracle.basis import lagrange
    L, D = lagrange(b.nodes, b.nodes)
    assert np.allclose(L, np.eye(k + 1), atol=1e-14)
    for j in range(k + 1):
        vals = b.nodes ** j
        Lq, Dq = lagrange(b.nodes, b.qx)
        assert np.allclose(Lq @ vals, b.qx ** j, atol=1e-13)
        assert np.allclose(Dq @ vals, j * b.qx ** max(j - 1, 0) if j else 0 * b.qx, atol=1e-12)


@pytest.mark.parametrize("k", [1, 2, 4])
def test_mass_matrix_diagonal(k):
    b = Basis(k)
    M = np.einsum("q,qn,qm->nm", b.wvol, b.phi, b.phi)
    off = M - np.diag(np.diag(M))
    assert np.abs(off).max() < 1e-14
    assert abs(M.sum() - 4.0) < 1e-13                # |[-1,1]^2|
    expect = np.outer(b.node_w, b.node_w).reshape(-1)  # w_a w_b with n = a + (k+1) b
    assert np.allclose(np.diag(M), expect.T.reshape(-1), atol=1e-14)


GAS = ph.Gas(1.4, 1.0 / (1.4 * 0.3 ** 2), 1e-2, 0.72)


def _state(rng, n=5):
    rho = rng.uniform(0.5, 1.5, n)
    u = rng.uniform(-1, 1, n)
    v = rng.uniform(-1, 1, n)
    p = rng.uniform(5, 10, n)
    return np.stack([rho, rho * u, rho * v, p / 0.4 + 0.5 * rho * (u * u + v * v)])


def _cs_jacobian(fun, U, h=1e-30):
    cols = []
    for j in range(4):
        Up = U.astype(complex)
        Up[j] += 1j * h
        cols.append(np.imag(fun(Up)) / h)
    return np.stack(cols, axis=-1)


def test_inviscid_jacobians_match_appendix():
    rng = np.random.default_rng(0)
    U = _state(rng)
    g = GAS.gamma
    gb = g - 1.0
    rho, u, v, E, p, theta, c, H = ph.primitives(U, GAS)
    ek = 0.5 * (u * u + v * v)
    z = 0 * u
    o = z + 1
    # App. A.1, with row 1 of A_1 read as (0, 1, 0, 0)
    A1 = np.array([[z, o, z, z],
                   [gb * ek - u * u, (3 - g) * u, -gb * v, gb * o],
                   [-u * v, v, u, z],
                   [u * (gb * ek - H), H - gb * u * u, -gb * u * v, g * u]])
    A2 = np.array([[z, z, o, z],
                   [-u * v, v, u, z],
                   [gb * ek - v * v, -gb * u, (3 - g) * v, gb * o],
                   [v * (gb * ek - H), -gb * u * v, H - gb * v * v, g * v]])
    for d, A in enumerate([A1, A2]):
        J = _cs_jacobian(lambda W: ph.convective_flux(W, GAS)[:, d], U)    # (4, n, 4)
        assert np.allclose(np.moveaxis(J, 1, 0), np.moveaxis(A, 2, 0), atol=1e-12)
        # degree-1 homogeneity: A_i U = F_i^c
        AU = np.einsum("ijn,jn->in", A, U)
        assert np.allclose(AU, ph.convective_flux(U, GAS)[:, d], atol=1e-12)


def test_viscous_jacobians_match_appendix():
    rng = np.random.default_rng(1)
    U = _state(rng)
    mu, lam = GAS.mu, GAS.lam
    alpha = GAS.kappa / GAS.cv
    mub = mu + lam
    lamb = lam + 2 * mu
    rho, u, v, E, p, theta, c, H = ph.primitives(U, GAS)
    ek = 0.5 * (u * u + v * v)
    ei = E - ek
    z = 0 * u
    # App. A.2, with the energy entry of the rho column of K11 and K22 read as +alpha (e_k - e_i)
    K11 = np.array([[z, z, z, z],
                    [-lamb * u, lamb + z, z, z],
                    [-mu * v, z, mu + z, z],
                    [-mu * v * v - lamb * u * u + alpha * (ek - ei), (lamb - alpha) * u, (mu - alpha) * v, alpha + z]]) / rho
    K12 = np.array([[z, z, z, z],
                    [-lam * v, z, lam + z, z],
                    [-mu * u, mu + z, z, z],
                    [-mub * u * v, mu * v, lam * u, z]]) / rho
    K21 = np.array([[z, z, z, z],
                    [-mu * v, z, mu + z, z],
                    [-lam * u, lam + z, z, z],
                    [-mub * u * v, lam * v, mu * u, z]]) / rho
    K22 = np.array([[z, z, z, z],
                    [-mu * u, mu + z, z, z],
                    [-lamb * v, z, lamb + z, z],
                    [-mu * u * u - lamb * v * v + alpha * (ek - ei), (mu - alpha) * u, (lamb - alpha) * v, alpha + z]]) / rho
    K = {(0, 0): K11, (0, 1): K12, (1, 0): K21, (1, 1): K22}
    for (i, j), Kij in K.items():
        for b in range(4):
            G = np.zeros((4, 2) + U.shape[1:])
            G[b, j] = 1.0
            col = ph.viscous_flux(U, G, GAS)[:, i]       # column b of K_ij
            assert np.allclose(col, Kij[:, b], atol=1e-13), (i, j, b)


def test_mixed_flux_equals_primal_flux():
    """F^nu(U, eps, phi) with eps = sym grad u - div u / 3 I and phi = grad theta equals F^nu(U, grad U)."""
    rng = np.random.default_rng(2)
    U = _state(rng)
    G = rng.standard_normal((4, 2, U.shape[1]))
    # primitive gradients by complex step of the maps U -> u, v, theta along G
    h = 1e-30
    pg = []
    for d in range(2):
        Up = U.astype(complex) + 1j * h * G[:, d]
        rho, u, v, E, p, theta, c, H = ph.primitives(Up, GAS)
        pg.append((np.imag(u) / h, np.imag(v) / h, np.imag(theta) / h))
    ux, vx, tx = pg[0]
    uy, vy, ty = pg[1]
    div = ux + vy
    eps = np.stack([ux - div / 3, 0.5 * (uy + vx), vy - div / 3])
    phi = np.stack([tx, ty])
    assert np.allclose(ph.viscous_flux_mixed(U, eps, phi, GAS), ph.viscous_flux(U, G, GAS), atol=1e-12)


def test_characteristic_split():
    rng = np.random.default_rng(3)
    U = _state(rng)
    for n in [np.array([1.0, 0.0]), np.array([0.0, -1.0]), np.array([0.6, 0.8])]:
        Ap, Am = ph.char_split(U, n, GAS)
        An = _cs_jacobian(lambda W: ph.normal_flux(ph.convective_flux(W, GAS), n), U)
        An = np.moveaxis(An, 1, 0)
        assert np.allclose(Ap + Am, An, atol=1e-11)
        assert np.allclose(Ap @ Am, 0.0, atol=1e-10)
        rho, u, v, E, p, theta, c, H = ph.primitives(U, GAS)
        un = u * n[0] + v * n[1]
        lam = np.stack([un - c, un, un, un + c], axis=-1)
        for e in range(U.shape[1]):
            ev = np.sort(np.linalg.eigvals(Ap[e]).real)
            assert np.allclose(ev, np.sort(np.maximum(lam[e], 0)), atol=1e-10)
            evm = np.sort(np.linalg.eigvals(Am[e]).real)
            assert np.allclose(evm, np.sort(np.minimum(lam[e], 0)), atol=1e-10)
    # supersonic along n: A^+ = A_n
    rho = np.array([1.0, 1.2])
    uu = np.array([8.0, 9.0])
    pp = np.array([6.0, 7.0])
    Us = np.stack([rho, rho * uu, 0 * rho, pp / 0.4 + 0.5 * rho * uu * uu])
    n = np.array([1.0, 0.0])
    Ap, Am = ph.char_split(Us, n, GAS)
    assert np.abs(Am).max() < 1e-12


def test_numerical_flux_consistency_and_conservation():
    rng = np.random.default_rng(4)
    U = _state(rng)
    V = _state(rng)
    n = np.array([0.6, -0.8])
    Fn = ph.normal_flux(ph.convective_flux(U, GAS), n)
    for flux in (ph.flux_vijayasundaram, ph.flux_lax_friedrichs):
        assert np.allclose(flux(U, U, n, GAS), Fn, atol=1e-12)
        assert np.allclose(flux(U, V, n, GAS), -flux(V, U, -n, GAS), atol=1e-12)
    for flux in (ph.flux_hdg_fvs, ph.flux_hdg_lf):
        assert np.allclose(flux(U, U, n, GAS), Fn, atol=1e-12)
    # FVS HDG flux equals A^+(Uh) U + A^-(Uh) Uh
    Ap, Am = ph.char_split(V, n, GAS)
    assert np.allclose(ph.flux_hdg_fvs(U, V, n, GAS), ph.matvec(Ap, U) + ph.matvec(Am, V), atol=1e-11)
    # far-field flux with U = U_inf is the physical flux
    assert np.allclose(ph.farfield_dg_flux(U, U, n, GAS), Fn, atol=1e-11)


def test_quad_points_rule():
    assert [quad_points(k) for k in (1, 2, 3, 4, 5)] == [2, 4, 5, 7, 8]
    assert math.isclose(GAS.kappa, GAS.cp * GAS.mu / GAS.Pr)
