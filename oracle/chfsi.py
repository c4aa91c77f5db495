"""Chebyshev-filtered subspace iteration (Sec. IV of the paper).

One pass: filter Ytilde = p_m(Ht) Y (damps the unwanted part of the spectrum
mapped to [-1, 1], amplifies the wanted part below it), orthonormalize, then
Rayleigh-Ritz (project, diagonalize, rotate; eqnProjKS).  Readings where the
paper is silent (it cites the method rather than stating it):

* spectrum bounds: k-step Lanczos with full reorthogonalization;
  a0 = smallest Ritz value of T_k, b = largest + beta_k;
* filter: the scaled three-term recurrence, which returns
  T_m(tau(Ht)) X / T_m(tau(a0)), tau(t) = (t - c) / e, e = (b - a)/2,
  c = (b + a)/2 -- the unscaled filter divided by one scalar (same span);
* orthonormalization: Cholesky-Gram-Schmidt Q = Y L^-*, L L^* = Y^* Y (the
  R factor of a QR factorization with positive diagonal), formed from the
  Jacobi-scaled Gram matrix (identical Q in exact arithmetic), repeated once
  when max|Q^* Q - I| > 1e-12; breakdown is declared when a squared pivot of
  the scaled (unit-diagonal) Gram matrix is at or below n * 2^-52;
* Rayleigh-Ritz in the symmetric form: Q^* Q = I so the projected overlap is
  the identity; the next block is the Ritz vectors Q U (same span as Q);
* pass 1 uses a = (a0 + b) / 2; later passes a0 = theta_1, a = theta_nv of the
  previous pass, b fixed.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


class CholeskyBreakdown(RuntimeError):
    def __init__(self, column: int):
        super().__init__(f"Gram matrix not positive definite at column {column}")
        self.column = column


def lanczos_bounds(apply, v0: np.ndarray, k: int = 10):
    """k-step Lanczos with full reorthogonalization (twice) -> (a0, b, alpha, beta)."""
    v = v0 / np.linalg.norm(v0)
    V = [v]
    alpha, beta = [], []
    b_prev = 0.0
    v_prev = np.zeros_like(v)
    for j in range(k):
        w = apply(V[-1])
        a = float(np.real(np.vdot(V[-1], w)))
        alpha.append(a)
        w = w - a * V[-1] - b_prev * v_prev
        Vm = np.stack(V, axis=1)
        for _ in range(2):
            w = w - Vm @ (np.conj(Vm.T) @ w)
        bj = float(np.linalg.norm(w))
        beta.append(bj)
        scale = max(max(abs(x) for x in alpha), max(beta))
        if bj < 1e-14 * scale:
            break
        v_prev = V[-1]
        b_prev = bj
        V.append(w / bj)
    n = len(alpha)
    T = np.diag(alpha) + np.diag(beta[: n - 1], 1) + np.diag(beta[: n - 1], -1)
    th = np.linalg.eigvalsh(T)
    return float(th[0]), float(th[-1] + beta[n - 1]), np.array(alpha), np.array(beta)


def filter_coefficients(m: int, a: float, b: float, a0: float):
    """Scalars of the scaled recurrence: returns (e, c, sigma[1..m])."""
    e = (b - a) / 2.0
    c = (b + a) / 2.0
    s1 = e / (a0 - c)
    sig = [s1]
    for _ in range(1, m):
        sig.append(1.0 / (2.0 / s1 - sig[-1]))
    return e, c, np.array(sig)


def chebyshev_filter(apply, X: np.ndarray, m: int, a: float, b: float, a0: float) -> np.ndarray:
    """Y_m = T_m(tau(Ht)) X / T_m(tau(a0)) by the scaled three-term recurrence (m >= 1)."""
    e, c, sig = filter_coefficients(m, a, b, a0)
    Yprev = X
    Y = (sig[0] / e) * (apply(X) - c * X)
    for k in range(1, m):
        Ynew = (2.0 * sig[k] / e) * (apply(Y) - c * Y) - (sig[k - 1] * sig[k]) * Yprev
        Yprev, Y = Y, Ynew
    return Y


def chebyshev_T(m: int, t: np.ndarray) -> np.ndarray:
    """T_m(t) from its closed forms on and off [-1, 1]."""
    t = np.asarray(t, dtype=np.float64)
    out = np.empty_like(t)
    inside = np.abs(t) <= 1.0
    out[inside] = np.cos(m * np.arccos(t[inside]))
    hi = t > 1.0
    out[hi] = np.cosh(m * np.arccosh(t[hi]))
    lo = t < -1.0
    out[lo] = (-1.0) ** m * np.cosh(m * np.arccosh(-t[lo]))
    return out


def cholgs_once(Y: np.ndarray):
    G = np.conj(Y.T) @ Y
    G = 0.5 * (G + np.conj(G.T))
    dg = np.real(np.diag(G)).copy()
    if np.any(~(dg > 0.0)):
        raise CholeskyBreakdown(int(np.nonzero(~(dg > 0.0))[0][0]))
    d = 1.0 / np.sqrt(dg)
    Gs = d[:, None] * G * d[None, :]
    try:
        Ls = np.linalg.cholesky(Gs)
    except np.linalg.LinAlgError:
        # locate the failing column the way a right-looking Cholesky would
        n = Gs.shape[0]
        col = n - 1
        for j in range(1, n + 1):
            try:
                np.linalg.cholesky(Gs[:j, :j])
            except np.linalg.LinAlgError:
                col = j - 1
                break
        raise CholeskyBreakdown(col)
    # numerical rank deficiency: a pivot of the unit-diagonal scaled Gram matrix at or below n u
    piv = np.real(np.diag(Ls)) ** 2
    small = np.nonzero(~(piv > Gs.shape[0] * np.finfo(float).eps))[0]
    if small.size:
        raise CholeskyBreakdown(int(small[0]))
    # Q = (Y d) Ls^-*  <=>  Ls Q^* = (Y d)^*
    QH = sla.solve_triangular(Ls, np.conj((Y * d[None, :]).T), lower=True)
    return np.conj(QH.T), (Ls / d[:, None])


def cholgs(Y: np.ndarray, tol: float = 1e-12):
    """Cholesky-Gram-Schmidt: Q with Q^* Q = I and span(Q) = span(Y); repeated once if needed.

    Returns (Q, repeated).
    """
    Q, _ = cholgs_once(Y)
    err = np.max(np.abs(np.conj(Q.T) @ Q - np.eye(Q.shape[1])))
    if err > tol:
        Q, _ = cholgs_once(Q)
        return Q, True
    return Q, False


def rayleigh_ritz(apply, Q: np.ndarray):
    """Ritz values (ascending) and vectors X = Q U of Ht on span(Q), Q orthonormal."""
    W = apply(Q)
    Hq = np.conj(Q.T) @ W
    Hq = 0.5 * (Hq + np.conj(Hq.T))
    th, U = np.linalg.eigh(Hq)
    return th, Q @ U


def chfsi(apply, X0: np.ndarray, v0: np.ndarray, m: int, passes: int, lanczos_k: int = 10):
    """Full ChFSI run -> dict with bounds, per-pass Ritz values, final vectors."""
    a0L, b, _, _ = lanczos_bounds(apply, v0, lanczos_k)
    a0, a = a0L, 0.5 * (a0L + b)
    X = X0
    hist = []
    for _ in range(passes):
        Y = chebyshev_filter(apply, X, m, a, b, a0)
        Q, _ = cholgs(Y)
        th, X = rayleigh_ritz(apply, Q)
        hist.append(dict(a=a, b=b, a0=a0, theta=th))
        a0, a = float(th[0]), float(th[-1])
    return dict(a0_lanczos=a0L, b=b, passes=hist, X=X, theta=hist[-1]["theta"])
