"""Nodal tensor-product basis and quadrature (oracle; test infrastructure only).

Reading of the paper: the broken space P^k(T) of Sec. 3.1 is taken on quads as
the tensor-product space Q^k with a nodal Lagrange basis at the (k+1)
Gauss-Legendre points per direction; facets carry P^k(F) with the same nodes.
Integrals use Gauss-Legendre with Q = ceil((3k+1)/2) points per direction, the
"over-integration up to order 3k" of Sec. 5.  Everything here is the plain
definition: products of 1D Lagrange polynomials evaluated point by point.
"""
from __future__ import annotations

import math

import numpy as np


def gauss_legendre(npts: int):
    """Gauss-Legendre points and weights on [-1, 1] (library routine)."""
    x, w = np.polynomial.legendre.leggauss(npts)
    return x, w


def quad_points(k: int) -> int:
    """Points per direction for exactness up to degree 3k: smallest Q with 2Q-1 >= 3k."""
    return int(math.ceil((3 * k + 1) / 2))


def lagrange(nodes: np.ndarray, x: np.ndarray):
    """Values L[i, a] = l_a(x_i) and derivatives D[i, a] = l_a'(x_i) of the Lagrange polynomials."""
    x = np.asarray(x, dtype=float)
    m = len(nodes)
    L = np.ones((len(x), m))
    D = np.zeros((len(x), m))
    for a in range(m):
        for b in range(m):
            if b != a:
                L[:, a] *= (x - nodes[b]) / (nodes[a] - nodes[b])
        for c in range(m):
            if c == a:
                continue
            term = np.full(len(x), 1.0 / (nodes[a] - nodes[c]))
            for b in range(m):
                if b != a and b != c:
                    term *= (x - nodes[b]) / (nodes[a] - nodes[b])
            D[:, a] += term
    return L, D


class Basis:
    """Reference-element tables for degree k.

    Node n = a + (k+1) b sits at (xi_a, xi_b); volume point q = i + Q j sits at
    (z_i, z_j).  Local faces: 0 = {xi=-1}, 1 = {xi=+1}, 2 = {eta=-1}, 3 = {eta=+1}
    with outward normals (-1,0), (1,0), (0,-1), (0,1); points on a face are
    ordered by increasing tangential coordinate.
    """

    NORMALS = np.array([[-1.0, 0.0], [1.0, 0.0], [0.0, -1.0], [0.0, 1.0]])

    def __init__(self, k: int, nq: int | None = None):
        self.k = k
        self.nq = quad_points(k) if nq is None else nq
        self.nodes, self.node_w = gauss_legendre(k + 1)
        self.qx, self.qw = gauss_legendre(self.nq)
        L, D = lagrange(self.nodes, self.qx)
        self.L1, self.D1 = L, D                        # (Q, k+1)
        Lm, Dm = lagrange(self.nodes, np.array([-1.0]))
        Lp, Dp = lagrange(self.nodes, np.array([1.0]))
        n1 = k + 1
        self.nn = n1 * n1
        Q = self.nq
        # volume tables (Q*Q, nn)
        self.phi = np.zeros((Q * Q, self.nn))
        self.dxi = np.zeros((Q * Q, self.nn))
        self.deta = np.zeros((Q * Q, self.nn))
        self.wvol = np.zeros(Q * Q)
        for j in range(Q):
            for i in range(Q):
                q = i + Q * j
                self.wvol[q] = self.qw[i] * self.qw[j]
                for b in range(n1):
                    for a in range(n1):
                        n = a + n1 * b
                        self.phi[q, n] = L[i, a] * L[j, b]
                        self.dxi[q, n] = D[i, a] * L[j, b]
                        self.deta[q, n] = L[i, a] * D[j, b]
        # face tables (4, Q, nn): value and reference derivatives at face points
        self.fphi = np.zeros((4, Q, self.nn))
        self.fdxi = np.zeros((4, Q, self.nn))
        self.fdeta = np.zeros((4, Q, self.nn))
        ends = {0: (Lm[0], Dm[0]), 1: (Lp[0], Dp[0])}
        for f in range(4):
            e_val, e_der = ends[f % 2]
            for i in range(Q):
                for b in range(n1):
                    for a in range(n1):
                        n = a + n1 * b
                        if f < 2:   # xi fixed, eta = z_i
                            self.fphi[f, i, n] = e_val[a] * L[i, b]
                            self.fdxi[f, i, n] = e_der[a] * L[i, b]
                            self.fdeta[f, i, n] = e_val[a] * D[i, b]
                        else:       # eta fixed, xi = z_i
                            self.fphi[f, i, n] = L[i, a] * e_val[b]
                            self.fdxi[f, i, n] = D[i, a] * e_val[b]
                            self.fdeta[f, i, n] = L[i, a] * e_der[b]
        # facet basis at face points (Q, k+1) and element traces at facet nodes (4, k+1, nn)
        self.psi = L.copy()
        Ln, _ = lagrange(self.nodes, self.nodes)
        self.trace_at_fnodes = np.zeros((4, n1, self.nn))
        for f in range(4):
            e_val, _ = ends[f % 2]
            for m in range(n1):
                for b in range(n1):
                    for a in range(n1):
                        n = a + n1 * b
                        if f < 2:
                            self.trace_at_fnodes[f, m, n] = e_val[a] * Ln[m, b]
                        else:
                            self.trace_at_fnodes[f, m, n] = Ln[m, a] * e_val[b]

    def mass_1d_facet(self):
        """Facet mass matrix int psi_m psi_l on [-1,1] with the Q-point rule."""
        return np.einsum("i,im,il->ml", self.qw, self.psi, self.psi)
