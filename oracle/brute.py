"""Brute-force solvers of entropic OT that do not use Sinkhorn iterations.

TEST INFRASTRUCTURE ONLY (used to pin the oracle; never by the product path).

* ``dual_max``   - maximises the concave dual of Eq. (eval-dual) / Eq.
                   (dual-theta), Sec. 2-3, with a generic trust-region
                   Newton method from SciPy, with the gauge alpha_1 = 0
                   that makes the maximiser unique (App. B).
* ``primal_2x2`` - for n = m = 2 the feasible plans form a segment; the
                   primal Eq. (reg-ot) is strictly convex on it and its
                   minimiser is found by bisection on the derivative.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import minimize

F64 = np.float64


def dual_objective(alpha, beta, K, a, b, eps):
    """a^T alpha + b^T beta - eps e^{alpha/eps}^T K e^{beta/eps} + eps."""
    ea = np.exp(alpha / eps)
    eb = np.exp(beta / eps)
    return float(a @ alpha + b @ beta - eps * ea @ K @ eb + eps)


def dual_max(K, a, b, eps):
    """Maximise the entropic OT dual over (alpha, beta) with alpha_1 = 0.
    Returns (value, alpha, beta)."""
    K = np.asarray(K, F64)
    a = np.asarray(a, F64)
    b = np.asarray(b, F64)
    n, m = K.shape

    def unpack(z):
        alpha = np.concatenate([[0.0], z[:n - 1]])
        beta = z[n - 1:]
        return alpha, beta

    def f(z):
        al, be = unpack(z)
        return -dual_objective(al, be, K, a, b, eps)

    def grad(z):
        al, be = unpack(z)
        ea, eb = np.exp(al / eps), np.exp(be / eps)
        P = ea[:, None] * K * eb[None, :]
        ga = a - P.sum(1)
        gb = b - P.sum(0)
        return -np.concatenate([ga[1:], gb])

    def hess(z):
        al, be = unpack(z)
        ea, eb = np.exp(al / eps), np.exp(be / eps)
        P = ea[:, None] * K * eb[None, :]
        H = np.zeros((n + m, n + m))
        H[:n, :n] = np.diag(P.sum(1))
        H[n:, n:] = np.diag(P.sum(0))
        H[:n, n:] = P
        H[n:, :n] = P.T
        H /= eps
        return H[1:, 1:]

    # start: beta from the first-order condition with alpha = 0
    z0 = np.concatenate([np.zeros(n - 1), eps * np.log(b / K.sum(0))])
    res = minimize(f, z0, jac=grad, hess=hess, method="trust-exact",
                   options={"gtol": 1e-15, "maxiter": 10000})
    al, be = unpack(res.x)
    return -float(res.fun), al, be


def primal_2x2(K, a, b, eps):
    """Exact entropic OT for n = m = 2 by bisection on the single free plan
    entry p = P_11 (P_12 = a1 - p, P_21 = b1 - p, P_22 = a2 - b1 + p).
    Returns (value, P)."""
    K = np.asarray(K, F64)
    a = np.asarray(a, F64)
    b = np.asarray(b, F64)
    C = -eps * np.log(K)
    lo = max(0.0, b[0] - a[1])
    hi = min(a[0], b[0])

    def dfdp(p):
        return (C[0, 0] - C[0, 1] - C[1, 0] + C[1, 1]
                + eps * (math.log(p) - math.log(a[0] - p)
                         - math.log(b[0] - p) + math.log(a[1] - b[0] + p)))

    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if dfdp(mid) > 0:
            hi = mid
        else:
            lo = mid
    p = 0.5 * (lo + hi)
    P = np.array([[p, a[0] - p], [b[0] - p, a[1] - b[0] + p]])
    H = -(P * (np.log(P) - 1.0)).sum()
    return float((P * C).sum() - eps * H + eps), P
