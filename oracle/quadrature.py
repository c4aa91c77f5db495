"""1D quadrature rules and Lagrange bases.

The FE basis is spectral: Lagrange polynomials on Gauss-Lobatto-Legendre
(GLL) nodes, so that GLL quadrature makes the FE overlap diagonal (Sec. III.A,
text before eqnorthCGLL).  Integrals of the Hamiltonian use a tensor
Gauss-Legendre rule with q = p + 1 points per direction (reading of the
paper's silence on the H quadrature; exact for the stiffness on affine cells).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg


def legendre_values(n: int, x: np.ndarray) -> np.ndarray:
    """P_n(x) by the three-term recurrence (n >= 0)."""
    x = np.asarray(x, dtype=np.float64)
    p0 = np.ones_like(x)
    if n == 0:
        return p0
    p1 = x.copy()
    for k in range(1, n):
        p0, p1 = p1, ((2 * k + 1) * x * p1 - k * p0) / (k + 1)
    return p1


def gll_rule(p: int):
    """GLL nodes (ascending) and weights for degree p (p + 1 points).

    Nodes: -1, 1 and the roots of P_p'.  Weights: 2 / (p (p + 1) P_p(x)^2).
    """
    if p < 1:
        raise ValueError("p >= 1")
    c = np.zeros(p + 1)
    c[p] = 1.0
    dc = npleg.legder(c)
    inner = np.sort(np.real(npleg.legroots(dc))) if p >= 2 else np.zeros(0)
    x = np.concatenate([[-1.0], inner, [1.0]])
    # polish interior roots with Newton on P_p'
    for _ in range(3):
        if p >= 2:
            d1 = npleg.legval(x[1:-1], dc)
            d2 = npleg.legval(x[1:-1], npleg.legder(dc))
            x[1:-1] -= d1 / d2
    w = 2.0 / (p * (p + 1) * legendre_values(p, x) ** 2)
    return x, w


def gauss_rule(q: int):
    """Gauss-Legendre nodes (ascending) and weights, q points."""
    x, w = npleg.leggauss(q)
    return x, w


def lagrange_basis(nodes: np.ndarray, x: np.ndarray):
    """Values ell_a(x_b) and derivatives ell_a'(x_b) of the Lagrange basis on `nodes`.

    Returns (V, D) with V[b, a] = ell_a(x_b), D[b, a] = ell_a'(x_b), from the
    product formula.
    """
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    n = nodes.size
    V = np.ones((x.size, n))
    D = np.zeros((x.size, n))
    for a in range(n):
        others = [j for j in range(n) if j != a]
        denom = np.prod([nodes[a] - nodes[j] for j in others])
        for b in range(x.size):
            V[b, a] = np.prod([x[b] - nodes[j] for j in others]) / denom
            s = 0.0
            for k in others:
                s += np.prod([x[b] - nodes[j] for j in others if j != k])
            D[b, a] = s / denom
    return V, D


class Reference1D:
    """1D reference data for degree p: GLL nodes/weights, Gauss rule, B1 and D1.

    B1[b, a] = ell_a(eta_b) (GLL basis at Gauss point b); D1[b, a] = ell_a'(eta_b).
    """

    def __init__(self, p: int):
        self.p = p
        self.xi, self.what = gll_rule(p)
        self.q = p + 1
        self.eta, self.w = gauss_rule(self.q)
        self.B1, self.D1 = lagrange_basis(self.xi, self.eta)
