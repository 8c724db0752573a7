"""FP64 CPU reference oracle for linear-time Sinkhorn divergences with
positive features (Scetbon & Cuturi, "Linear Time Sinkhorn Divergences
using Positive Features").

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: it exists so that tests, the smoke check and the CPU
baseline of the benchmark can compare the GPU library against a plain,
slow, obviously correct implementation.  It shares no code with the HIP
library and does not import it.

Everything is float64 NumPy.  Inputs given as float32 arrays are upcast, so
both sides see the same numbers.  No blocking, fusion or reordering beyond
what the definitions state.

Pins (tests/test_oracle_pins.py, run without a GPU):
  * lambert_q                - the defining identity of W0 (closed form).
  * gaussian_log_features    - Gauss-Hermite quadrature of the integral
                               representation of the Gaussian kernel
                               (Lemma 1); convergence of K_theta to the
                               Gaussian kernel as r grows (Prop. 3.1).
  * sinkhorn                 - marginals, u^T K v = 1, brute-force dual
                               maximisation, 2x2 primal bisection,
                               primal/dual equality.
  * w_hat / divergence       - translation closed form for the exact
                               Gaussian kernel, symmetry, permutation.
  * divergence_grad          - central finite differences; large-r limit
                               of the squared-Euclidean Sinkhorn gradient;
                               divergence_grad_scaled equals it where both
                               apply.
  * divergence_grad_anchors  - central finite differences of the divergence
                               with respect to every anchor coordinate.
  * accelerated_sinkhorn     - (tests/test_accelerated.py) reaches the
                               optimum of Algorithm 1 with a plan of the
                               right marginals; weak duality and the
                               accelerated gap bound A_k (phi_k - phi*) <=
                               ||eta*||^2/2 at every step; rank-one closed
                               form; first step against finite differences;
                               line-search doubling.  divergence_grad_accelerated
                               reuses divergence_grad's formulas (pinned there)
                               on these points.
  * arccos_kernel            - 2-D numerical integration of the defining
                               integral; arccos_features - convergence of the
                               feature products to the kernel as r grows.
No function here is "parity unpinned".
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional

import numpy as np
from scipy.special import lambertw

__all__ = [
    "lambert_q", "sigma2_from_q", "q_from_sigma2", "divergence_grad_anchors",
    "gaussian_log_features", "gaussian_features", "gaussian_features_scaled",
    "gaussian_kernel", "rf_kernel",
    "arccos_log_features", "arccos_features", "arccos_kernel", "arccos_features_scaled",
    "SinkhornResult", "sinkhorn", "sinkhorn_dense", "sinkhorn_factored",
    "AcceleratedResult", "accelerated_sinkhorn", "dual_value",
    "w_hat", "w_hat_scaled", "Divergence", "divergence",
    "divergence_scaled", "divergence_from_kernels",
    "primal_objective", "divergence_grad", "grad_x_exact_kernel",
    "divergence_grad_accelerated", "divergence_grad_scaled", "grads_from_scalings",
]

F64 = np.float64


# --------------------------------------------------------------------------
# Bandwidth of the Gaussian feature map (Lemma 1, Sec. 3.2; proof in App. A)
# --------------------------------------------------------------------------
def lambert_q(R: float, eps: float, d: int) -> float:
    """q = R^2 / (2 eps d W0(R^2 / (eps d))), W0 the principal real branch
    of the Lambert function (Lemma 1, for points in the ball B(0, R))."""
    z = (R * R) / (eps * d)
    w = float(lambertw(z, 0).real)
    return (R * R) / (2.0 * eps * d * w)


def sigma2_from_q(q: float, eps: float) -> float:
    """Anchor variance sigma^2 = q eps / 4 (Lemma 1)."""
    return q * eps / 4.0


def q_from_sigma2(sigma2: float, eps: float) -> float:
    """Inverse of sigma2_from_q, for workloads that fix sigma^2 directly."""
    return 4.0 * sigma2 / eps


# --------------------------------------------------------------------------
# Positive features for the Gaussian kernel k(x,y) = exp(-||x-y||^2/eps)
# --------------------------------------------------------------------------
def gaussian_log_features(X, U, eps: float, q: float,
                          chunk: Optional[int] = None) -> np.ndarray:
    """log phi_theta(x_i)_k for the Gaussian feature map.

    The per-anchor map (Lemma 1, in the form derived in its proof, App. A):
        phi(x, u) = (2q)^{d/4} exp(-2||x - u||^2 / eps) exp(||u||^2 / (eps q))
    and the finite feature vector of Eq. (general), Sec. 3.2:
        phi_theta(x) = r^{-1/2} (phi(x, u_1), ..., phi(x, u_r)).
    Squared distances are taken as direct differences.  Returns (n, r).
    """
    X = np.asarray(X, F64)
    U = np.asarray(U, F64)
    n, d = X.shape
    r = U.shape[0]
    const = -0.5 * math.log(r) + 0.25 * d * math.log(2.0 * q)
    unorm = (U * U).sum(1) / (eps * q)
    out = np.empty((n, r), F64)
    if chunk is None:                    # rows per block of differences (<= 256 MB)
        chunk = max(1, min(4096, (1 << 25) // max(1, r * d)))
    for s in range(0, n, chunk):
        diff = X[s:s + chunk, None, :] - U[None, :, :]
        d2 = (diff * diff).sum(-1)
        out[s:s + chunk] = const - (2.0 / eps) * d2 + unorm[None, :]
    return out


def gaussian_features(X, U, eps: float, q: float) -> np.ndarray:
    """Features phi_theta(x_i) as rows, (n, r); K_theta = Phi_x Phi_y^T."""
    return np.exp(gaussian_log_features(X, U, eps, q))


def gaussian_features_scaled(X, U, eps: float, q: float):
    """Row-scaled features: Phi = diag(exp(s)) Phi_tilde with
    s_i = max_k log phi_theta(x_i)_k, so every entry of Phi_tilde lies in
    (0, 1].  The scaling is absorbed exactly by the Sinkhorn scalings
    (u_tilde = u * exp(s)); it is not in the paper and only keeps the
    entries representable.  Returns (Phi_tilde (n, r), s (n,))."""
    E = gaussian_log_features(X, U, eps, q)
    s = E.max(axis=1)
    return np.exp(E - s[:, None]), s


# --------------------------------------------------------------------------
# Perturbed arc-cosine features (Sec. 3.2, "Arc-cosine kernels"; the lemma on
# the decomposition of the arc-cosine kernel in the appendix)
# --------------------------------------------------------------------------
def arccos_log_features(X, U, s: int, sigma: float, kappa: float) -> np.ndarray:
    """Natural log of the r + 1 features of the perturbed arc-cosine kernel
    k_{s,kappa} = k_s + kappa, for anchors U (rows u_k, drawn from
    N(0, sigma^2 I), sigma > 1):
        phi_k(x) = r^{-1/2} sigma^{d/2} sqrt(2) max(0, u_k^T x)^s
                   exp(-||u_k||^2 (1 - 1/sigma^2) / 4),   k = 1..r,
        phi_{r+1}(x) = sqrt(kappa).
    The factor sqrt(2) belongs to Theta_s(w) = sqrt(2) max(0, w)^s as the
    kernel is defined in Sec. 3.2 (with it the map reproduces k_s).  A
    rectified zero has log -inf; max(0, w)^0 is 1 for w > 0 and 0 else."""
    X = np.asarray(X, F64)
    U = np.asarray(U, F64)
    r, d = U.shape
    proj = X @ U.T
    with np.errstate(divide="ignore"):
        if s == 0:
            lp = np.where(proj > 0, 0.0, -np.inf)
        else:
            lp = s * np.log(np.maximum(proj, 0.0))
    c = (-0.5 * math.log(r) + 0.5 * d * math.log(sigma) + 0.5 * math.log(2.0)
         - 0.25 * (1.0 - 1.0 / sigma ** 2) * (U * U).sum(1))
    out = np.empty((X.shape[0], r + 1))
    out[:, :r] = lp + c[None, :]
    out[:, r] = 0.5 * math.log(kappa)
    return out


def arccos_features(X, U, s: int, sigma: float, kappa: float) -> np.ndarray:
    return np.exp(arccos_log_features(X, U, s, sigma, kappa))


def arccos_kernel(X, Y, s: int, kappa: float) -> np.ndarray:
    """Closed form of k_s (Cho & Saul, 2009): (1/pi) ||x||^s ||y||^s J_s(t)
    with t the angle between x and y and
        J_0 = pi - t,  J_1 = sin t + (pi - t) cos t,
        J_2 = 3 sin t cos t + (pi - t)(1 + 2 cos^2 t);  plus kappa."""
    X = np.asarray(X, F64)
    Y = np.asarray(Y, F64)
    nx = np.linalg.norm(X, axis=1)[:, None]
    ny = np.linalg.norm(Y, axis=1)[None, :]
    c = np.clip((X @ Y.T) / (nx * ny), -1.0, 1.0)
    t = np.arccos(c)
    if s == 0:
        J = np.pi - t
    elif s == 1:
        J = np.sin(t) + (np.pi - t) * c
    elif s == 2:
        J = 3.0 * np.sin(t) * c + (np.pi - t) * (1.0 + 2.0 * c * c)
    else:
        raise ValueError("closed form only for s in {0, 1, 2}")
    return (nx ** s) * (ny ** s) * J / np.pi + kappa


def arccos_features_scaled(X, U, s: int, sigma: float, kappa: float):
    """Row-scaled arc-cosine features: (Phi~, s) with phi = e^s Phi~ and the
    row maximum of Phi~ equal to 1 (the constant feature keeps it > 0)."""
    L = arccos_log_features(X, U, s, sigma, kappa)
    m = L.max(1)
    return np.exp(L - m[:, None]), m


def gaussian_kernel(X, Y, eps: float) -> np.ndarray:
    """Exact Gibbs kernel of the squared Euclidean cost, exp(-||x-y||^2/eps)."""
    X = np.asarray(X, F64)
    Y = np.asarray(Y, F64)
    diff = X[:, None, :] - Y[None, :, :]
    return np.exp(-(diff * diff).sum(-1) / eps)


def rf_kernel(X, Y, U, eps: float, q: float) -> np.ndarray:
    """K_theta = Xi^T Zeta = Phi_x Phi_y^T (Sec. 3.1)."""
    return gaussian_features(X, U, eps, q) @ gaussian_features(Y, U, eps, q).T


# --------------------------------------------------------------------------
# Algorithm 1 (Sinkhorn), Sec. 2
# --------------------------------------------------------------------------
@dataclasses.dataclass
class SinkhornResult:
    u: np.ndarray          # row scaling
    v: np.ndarray          # column scaling
    iters: int             # number of (v-update, u-update) pairs done
    err: float             # ||v o K^T u - b||_1 after the last u-update
    converged: bool


def sinkhorn(apply_K: Callable, apply_Kt: Callable, a, b, tol: float = 1e-6,
             max_iter: int = 2000, fixed_iter: int = 0,
             u0: Optional[np.ndarray] = None) -> SinkhornResult:
    """Algorithm 1: starting from a positive u, repeat
           v <- b / K^T u,   u <- a / K v
    until ||v o K^T u - b||_1 < tol (tested after each u-update).

    ``apply_K(v) = K v`` and ``apply_Kt(u) = K^T u``.  With ``fixed_iter``
    > 0 exactly that many iterations are done and the error is only
    reported.  Otherwise at most ``max_iter`` iterations are done.
    """
    a = np.asarray(a, F64)
    b = np.asarray(b, F64)
    u = np.ones_like(a) if u0 is None else np.asarray(u0, F64).copy()
    Ktu = apply_Kt(u)
    limit = fixed_iter if fixed_iter > 0 else max_iter
    err = math.inf
    v = None
    k = 0
    converged = False
    for k in range(1, limit + 1):
        v = b / Ktu
        u = a / apply_K(v)
        Ktu = apply_Kt(u)
        err = float(np.abs(v * Ktu - b).sum())
        if fixed_iter <= 0 and err < tol:
            converged = True
            break
    if fixed_iter > 0:
        converged = err < tol
    return SinkhornResult(u, v, k, err, converged)


@dataclasses.dataclass
class AcceleratedResult:
    eta1: np.ndarray        # returned dual point (log row scaling)
    eta2: np.ndarray        # returned dual point (log column scaling)
    iters: int              # accepted steps
    trials: int             # gradient evaluations (one K and one K^T product each)
    err: float              # ||grad phi||_1 at the last momentum point evaluated
    converged: bool
    zeta1: np.ndarray       # momentum sequence after the last accepted step
    zeta2: np.ndarray
    blocks: list            # block (1 or 2) minimised at every accepted step
    Ls: list                # accepted Lipschitz estimate of every step
    As: list                # A_k after every accepted step
    phis: list              # phi(eta^k) after every accepted step
    margins: list           # |G1 - G2| / (G1 + G2) of the block choice, every trial
    ls_margins: list        # |decrease - required| / required of the test, every trial


def accelerated_sinkhorn(apply_K: Callable, apply_Kt: Callable, a, b, tol: float = 1e-6,
                         max_iter: int = 2000, fixed_iter: int = 0,
                         L0: float = 1.0) -> AcceleratedResult:
    """Accelerated Sinkhorn: accelerated alternating minimisation (the
    remark on acceleration in Sec. 3.1 and the accelerated algorithm of the
    appendix, read from its description where the printed listing is
    garbled).  It minimises the convex smooth function
        phi(eta1, eta2) = log <e^eta1, K e^eta2> - <eta1, a> - <eta2, b>,
    i.e. -F/eps for the dual F of Eq. (dual-smooth).  Starting from
    eta = zeta = 0, A = 0, step k tries the Lipschitz estimate L_k / 2,
    then doubles it until the sufficient-decrease test passes:
        a_{k+1} = 1/(2L) + sqrt(1/(4L^2) + A_k/L),  A_{k+1} = A_k + a_{k+1},
        tau = a_{k+1} / A_{k+1},  lambda = tau zeta + (1 - tau) eta,
        eta' = exact minimiser of phi over the block of lambda with the
               larger gradient norm (a Sinkhorn half-step from lambda), the
               other block kept at lambda,
        accept when phi(eta') <= phi(lambda) - ||grad phi(lambda)||^2 / (2L);
    an accepted step sets zeta <- zeta - a_{k+1} grad phi(lambda),
    eta <- eta'.  grad phi(lambda) is the marginal mismatch of the plan
    diag(e^lambda1) K diag(e^lambda2) / <e^lambda1, K e^lambda2>.

    Stopping: when ||grad phi(lambda)||_1 < tol at an evaluated momentum
    point, the block minimiser from that point is returned (it lowers phi
    whatever the test says).  With fixed_iter > 0 exactly that many steps
    are accepted and eta after the last one is returned.  Exponentials are
    formed after subtracting the maximum (exact in float64)."""
    a = np.asarray(a, F64)
    b = np.asarray(b, F64)
    n, m = len(a), len(b)
    eta1, eta2 = np.zeros(n), np.zeros(m)
    zeta1, zeta2 = np.zeros(n), np.zeros(m)
    A, L = 0.0, float(L0)
    trials, blocks, Ls, As, phis, margins, ls_margins = 0, [], [], [], [], [], []
    err = math.inf

    def phi_at(l1, l2):
        s1, s2 = l1.max(), l2.max()
        c = float(np.exp(l1 - s1) @ apply_K(np.exp(l2 - s2)))
        return math.log(c) + s1 + s2 - l1 @ a - l2 @ b

    def evaluate(l1, l2):
        # gradient of phi at lambda and the block minimisers from lambda
        s1, s2 = l1.max(), l2.max()
        e1, e2 = np.exp(l1 - s1), np.exp(l2 - s2)
        Ke2, Kte1 = apply_K(e2), apply_Kt(e1)         # K e^l2 / e^s2, K^T e^l1 / e^s1
        c = float(e1 @ Ke2)
        g1 = e1 * Ke2 / c - a
        g2 = e2 * Kte1 / c - b
        G1, G2 = float(g1 @ g1), float(g2 @ g2)
        margins.append(abs(G1 - G2) / (G1 + G2) if G1 + G2 > 0 else 0.0)
        if G1 >= G2:
            block, n1, n2 = 1, np.log(a) - np.log(Ke2) - s2, l2
        else:
            block, n1, n2 = 2, l1, np.log(b) - np.log(Kte1) - s1
        return g1, g2, block, n1, n2

    k = 0
    while True:
        if fixed_iter > 0 and k == fixed_iter:
            return AcceleratedResult(eta1, eta2, k, trials, err, False, zeta1, zeta2,
                                     blocks, Ls, As, phis, margins, ls_margins)
        if fixed_iter <= 0 and k == max_iter:
            return AcceleratedResult(eta1, eta2, k, trials, err, False, zeta1, zeta2,
                                     blocks, Ls, As, phis, margins, ls_margins)
        Lt = L / 2.0
        while True:
            ak = 1.0 / (2.0 * Lt) + math.sqrt(1.0 / (4.0 * Lt * Lt) + A / Lt)
            tau = ak / (A + ak)
            l1 = tau * zeta1 + (1.0 - tau) * eta1
            l2 = tau * zeta2 + (1.0 - tau) * eta2
            g1, g2, block, n1, n2 = evaluate(l1, l2)
            trials += 1
            err = float(np.abs(g1).sum() + np.abs(g2).sum())
            if fixed_iter <= 0 and err < tol:
                return AcceleratedResult(n1, n2, k, trials, err, True, zeta1, zeta2,
                                         blocks, Ls, As, phis, margins, ls_margins)
            phi_new = phi_at(n1, n2)
            need = float(g1 @ g1 + g2 @ g2) / (2.0 * Lt)
            drop = phi_at(l1, l2) - phi_new
            ls_margins.append(abs(drop - need) / need if need > 0 else math.inf)
            if drop >= need:
                break
            Lt *= 2.0
            if not Lt < 1e300:      # the test cannot pass in this precision
                return AcceleratedResult(eta1, eta2, k, trials, err, False, zeta1, zeta2,
                                         blocks, Ls, As, phis, margins, ls_margins)
        zeta1 = zeta1 - ak * g1
        zeta2 = zeta2 - ak * g2
        eta1, eta2 = n1, n2
        A, L = A + ak, Lt
        k += 1
        blocks.append(block)
        Ls.append(Lt)
        As.append(A)
        phis.append(phi_new)


def dual_value(eta1, eta2, K, a, b, eps: float) -> float:
    """eps (<eta1, a> + <eta2, b> - log <e^eta1, K e^eta2>): the dual of
    Eq. (dual-smooth), a lower bound of the regularised OT value that equals
    it at the optimum."""
    s1, s2 = eta1.max(), eta2.max()
    c = float(np.exp(eta1 - s1) @ (K @ np.exp(eta2 - s2)))
    return float(eps * (eta1 @ a + eta2 @ b - math.log(c) - s1 - s2))


def sinkhorn_dense(K, a, b, **kw) -> SinkhornResult:
    """Algorithm 1 on a materialised n x m kernel matrix."""
    K = np.asarray(K, F64)
    return sinkhorn(lambda v: K @ v, lambda u: K.T @ u, a, b, **kw)


def sinkhorn_factored(Phix, Phiy, a, b, **kw) -> SinkhornResult:
    """Algorithm 1 on K = Phix Phiy^T applied as two skinny products, the
    r(n+m) form of Sec. 3.1."""
    Phix = np.asarray(Phix, F64)
    Phiy = np.asarray(Phiy, F64)
    return sinkhorn(lambda v: Phix @ (Phiy.T @ v),
                    lambda u: Phiy @ (Phix.T @ u), a, b, **kw)


def w_hat(u, v, a, b, eps: float) -> float:
    """Dual estimate eps (a^T log u + b^T log v) of Eq. (dual-estimate),
    Sec. 2 (valid because u^T K v = 1 after any Sinkhorn update)."""
    a = np.asarray(a, F64)
    b = np.asarray(b, F64)
    return float(eps * (a @ np.log(u) + b @ np.log(v)))


def primal_objective(P, K, eps: float) -> float:
    """<P, C> - eps H(P) + eps with C = -eps log K and
    H(P) = -sum P (log P - 1), Eq. (reg-ot), Sec. 2."""
    P = np.asarray(P, F64)
    C = -eps * np.log(np.asarray(K, F64))
    H = -(P * (np.log(P) - 1.0)).sum()
    return float((P * C).sum() - eps * H + eps)


# --------------------------------------------------------------------------
# Sinkhorn divergence, Eq. (reg-sdiv), Sec. 2
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Divergence:
    value: float           # W_bar = W(mu,nu) - (W(mu,mu) + W(nu,nu)) / 2
    w_xy: float
    w_xx: float
    w_yy: float
    xy: SinkhornResult
    xx: SinkhornResult
    yy: SinkhornResult


def divergence_from_kernels(Kxy, Kxx, Kyy, a, b, eps, **kw) -> Divergence:
    """Debiased divergence from three dense kernels: three runs of
    Algorithm 1 and their dual estimates (Eq. reg-sdiv, Eq. dual-estimate)."""
    xy = sinkhorn_dense(Kxy, a, b, **kw)
    xx = sinkhorn_dense(Kxx, a, a, **kw)
    yy = sinkhorn_dense(Kyy, b, b, **kw)
    wxy = w_hat(xy.u, xy.v, a, b, eps)
    wxx = w_hat(xx.u, xx.v, a, a, eps)
    wyy = w_hat(yy.u, yy.v, b, b, eps)
    return Divergence(wxy - 0.5 * (wxx + wyy), wxy, wxx, wyy, xy, xx, yy)


def divergence(X, Y, a, b, U, eps: float, q: float, tol: float = 1e-6,
               max_iter: int = 2000, fixed_iter: int = 0,
               dense: Optional[bool] = None) -> Divergence:
    """Sinkhorn divergence with the positive-feature kernel K_theta.

    Each of the three problems (x,y), (x,x), (y,y) runs Algorithm 1 from
    u0 = exp(-s_x) (a positive start, allowed by Sec. 2), where s_x is the
    per-point maximum log-feature.  Dense K_theta when n*m is small
    (``dense=None`` picks dense for n*m <= 4e7), otherwise the factored
    product.  The unscaled features are used, so this is plain Algorithm 1
    on K_theta; it needs exp(log-features) representable in float64.
    """
    Ex = gaussian_log_features(X, U, eps, q)
    Ey = gaussian_log_features(Y, U, eps, q)
    sx = Ex.max(1)
    sy = Ey.max(1)
    Px, Py = np.exp(Ex), np.exp(Ey)
    n, m = Px.shape[0], Py.shape[0]
    if dense is None:
        dense = n * m <= 4e7 and n * n <= 4e7 and m * m <= 4e7
    kw = dict(tol=tol, max_iter=max_iter, fixed_iter=fixed_iter)
    if dense:
        def run(A, B, wa, wb, s0):
            return sinkhorn_dense(A @ B.T, wa, wb, u0=np.exp(-s0), **kw)
    else:
        def run(A, B, wa, wb, s0):
            return sinkhorn_factored(A, B, wa, wb, u0=np.exp(-s0), **kw)
    xy = run(Px, Py, a, b, sx)
    xx = run(Px, Px, a, a, sx)
    yy = run(Py, Py, b, b, sy)
    wxy = w_hat(xy.u, xy.v, a, b, eps)
    wxx = w_hat(xx.u, xx.v, a, a, eps)
    wyy = w_hat(yy.u, yy.v, b, b, eps)
    return Divergence(wxy - 0.5 * (wxx + wyy), wxy, wxx, wyy, xy, xx, yy)


def w_hat_scaled(ut, vt, a, b, sx, sy, eps: float) -> float:
    """Dual estimate for the row-scaled problem.  With Phi = diag(e^s) Phi~,
    the scalings of K_theta are u = u~ e^{-s_x}, v = v~ e^{-s_y}, so
    eps(a^T log u + b^T log v) = eps(a^T log u~ + b^T log v~)
                                 - eps(a^T s_x + b^T s_y)."""
    a = np.asarray(a, F64)
    b = np.asarray(b, F64)
    return float(eps * (a @ np.log(ut) + b @ np.log(vt))
                 - eps * (a @ np.asarray(sx, F64) + b @ np.asarray(sy, F64)))


def divergence_scaled(X, Y, a, b, U, eps: float, q: float, tol: float = 1e-6,
                      max_iter: int = 2000, fixed_iter: int = 0,
                      dense: Optional[bool] = None, features=None) -> Divergence:
    """Same quantity as ``divergence`` computed on the row-scaled features:
    Algorithm 1 on K~ = Phi~_x Phi~_y^T from u~0 = 1 (the image of
    u0 = exp(-s_x) under the scaling), then ``w_hat_scaled``.  The iterates
    are those of ``divergence`` times exp(s); unlike ``divergence`` it
    never forms exp of a raw log-feature, so it also covers workloads whose
    raw features underflow float64 (small eps, large d).  The returned
    SinkhornResult scalings are the scaled ones (u~, v~).  ``features``
    may hold (Phi~_x, s_x, Phi~_y, s_y) already computed by
    gaussian_features_scaled for these X, Y."""
    if features is None:
        Px, sx = gaussian_features_scaled(X, U, eps, q)
        Py, sy = gaussian_features_scaled(Y, U, eps, q)
    else:
        Px, sx, Py, sy = features
    n, m = Px.shape[0], Py.shape[0]
    if dense is None:
        dense = n * m <= 4e7 and n * n <= 4e7 and m * m <= 4e7
    kw = dict(tol=tol, max_iter=max_iter, fixed_iter=fixed_iter)
    if dense:
        def run(A, B, wa, wb):
            return sinkhorn_dense(A @ B.T, wa, wb, **kw)
    else:
        def run(A, B, wa, wb):
            return sinkhorn_factored(A, B, wa, wb, **kw)
    xy = run(Px, Py, a, b)
    xx = run(Px, Px, a, a)
    yy = run(Py, Py, b, b)
    wxy = w_hat_scaled(xy.u, xy.v, a, b, sx, sy, eps)
    wxx = w_hat_scaled(xx.u, xx.v, a, a, sx, sx, eps)
    wyy = w_hat_scaled(yy.u, yy.v, b, b, sy, sy, eps)
    return Divergence(wxy - 0.5 * (wxx + wyy), wxy, wxx, wyy, xy, xx, yy)


# --------------------------------------------------------------------------
# Gradients (Prop. 3.2 and the chain rule that follows it, Sec. 3.3)
# --------------------------------------------------------------------------
def _grad_points_one_side(Xs, U, eps, Phi, p, g):
    """Gradient of W_hat with respect to the points of one side.

    Prop. 3.2 gives dW/dK = -eps u v^T at the optimum.  With
    K_ij = sum_k phi_k(x_i) phi_k(y_j) and, from the feature map,
    d phi_k(x)/dx = -(4/eps)(x - u_k) phi_k(x), the chain rule gives for a
    point on the row side (p = u, g = Phi_y^T v):
        dW/dx_i = 4 p_i sum_k phi_k(x_i) g_k (x_i - u_k).
    The same expression with p = v, g = Phi_x^T u holds for the column side.
    """
    Xs = np.asarray(Xs, F64)
    U = np.asarray(U, F64)
    wphi = Phi * g[None, :]                      # phi_k(x_i) g_k
    term1 = wphi.sum(1)[:, None] * Xs            # sum_k phi g  x_i
    term2 = wphi @ U                             # sum_k phi g  u_k
    return 4.0 * p[:, None] * (term1 - term2)


def divergence_grad(X, Y, a, b, U, eps: float, q: float, tol: float = 1e-13,
                    max_iter: int = 100000, fixed_iter: int = 0):
    """Gradients of the divergence with respect to X, a, Y, b.

    Point gradients: the envelope gradient of Prop. 3.2 pushed through the
    feature map (the gradient formula with respect to the point locations
    in Sec. 3.3).  A point of X enters W(mu, nu) on the row side and
    W(mu, mu) on both sides, so
        dW_bar/dX = G_row(xy) - (G_row(xx) + G_col(xx)) / 2.
    Weight gradients: by the envelope theorem on Eq. (eval-dual),
    dW/da = alpha* = eps log u (row side) and eps log v (column side); the
    dual optimum is unique only up to a constant shift (App. B), so the
    gradient is returned centred (mean removed), i.e. projected on the
    tangent space {sum da = 0} of the simplex.
    Returns (dX, da, dY, db, Divergence).
    """
    Phx = gaussian_features(X, U, eps, q)
    Phy = gaussian_features(Y, U, eps, q)
    sx = gaussian_log_features(X, U, eps, q).max(1)
    sy = gaussian_log_features(Y, U, eps, q).max(1)
    kw = dict(tol=tol, max_iter=max_iter, fixed_iter=fixed_iter)
    xy = sinkhorn_dense(Phx @ Phy.T, a, b, u0=np.exp(-sx), **kw)
    xx = sinkhorn_dense(Phx @ Phx.T, a, a, u0=np.exp(-sx), **kw)
    yy = sinkhorn_dense(Phy @ Phy.T, b, b, u0=np.exp(-sy), **kw)
    wxy = w_hat(xy.u, xy.v, a, b, eps)
    wxx = w_hat(xx.u, xx.v, a, a, eps)
    wyy = w_hat(yy.u, yy.v, b, b, eps)
    div = Divergence(wxy - 0.5 * (wxx + wyy), wxy, wxx, wyy, xy, xx, yy)

    dX, da, dY, db = grads_from_scalings(X, Y, U, eps, Phx, Phy, (xy.u, xy.v),
                                          (xx.u, xx.v), (yy.u, yy.v))
    return dX, da, dY, db, div


def divergence_grad_scaled(X, Y, a, b, U, eps: float, q: float, tol: float = 1e-13,
                           max_iter: int = 100000, fixed_iter: int = 0, dense=None):
    """divergence_grad computed on the row-scaled features (for inputs whose
    raw features underflow float64, e.g. large d): the gradient formulas only
    use products u_i phi_k(x_i) = u~_i Phi~_ik and Phi^T v = Phi~^T v~, and
    log u_xy - (log u_xx + log v_xx)/2 = log u~_xy - (log u~_xx + log v~_xx)/2
    (the log-scales cancel), so they apply unchanged to the scaled run of
    divergence_scaled.  Returns (dX, da, dY, db, Divergence)."""
    Px, sx = gaussian_features_scaled(X, U, eps, q)
    Py, sy = gaussian_features_scaled(Y, U, eps, q)
    div = divergence_scaled(X, Y, a, b, U, eps, q, tol=tol, max_iter=max_iter,
                            fixed_iter=fixed_iter, dense=dense, features=(Px, sx, Py, sy))
    dX, da, dY, db = grads_from_scalings(X, Y, U, eps, Px, Py, (div.xy.u, div.xy.v),
                                          (div.xx.u, div.xx.v), (div.yy.u, div.yy.v))
    return dX, da, dY, db, div


def grads_from_scalings(X, Y, U, eps, Phx, Phy, sxy, sxx, syy):
    """The gradient formulas of divergence_grad applied to the scalings
    (u, v) of the three terms."""
    dX = (_grad_points_one_side(X, U, eps, Phx, sxy[0], Phy.T @ sxy[1])
          - 0.5 * (_grad_points_one_side(X, U, eps, Phx, sxx[0], Phx.T @ sxx[1])
                   + _grad_points_one_side(X, U, eps, Phx, sxx[1], Phx.T @ sxx[0])))
    dY = (_grad_points_one_side(Y, U, eps, Phy, sxy[1], Phx.T @ sxy[0])
          - 0.5 * (_grad_points_one_side(Y, U, eps, Phy, syy[0], Phy.T @ syy[1])
                   + _grad_points_one_side(Y, U, eps, Phy, syy[1], Phy.T @ syy[0])))
    da = eps * (np.log(sxy[0]) - 0.5 * (np.log(sxx[0]) + np.log(sxx[1])))
    db = eps * (np.log(sxy[1]) - 0.5 * (np.log(syy[0]) + np.log(syy[1])))
    return dX, da - da.mean(), dY, db - db.mean()


def divergence_grad_accelerated(X, Y, a, b, U, eps: float, q: float, fixed_iter: int,
                                L0: float = 1.0):
    """divergence_grad with each term's dual point taken from
    accelerated_sinkhorn after `fixed_iter` accepted steps from zero on the
    row-scaled factored kernel K~ = Phi~_x Phi~_y^T (features divided by
    their row maxima e^s).  The point eta~ on K~ is the point eta~ - s on
    the unscaled kernel: u = e^(eta~1 - s_x), v = e^(eta~2 - s_y) enter the
    same gradient formulas, and each term's value is the dual F of
    Eq. (dual-smooth) there, F(eta~ - s) = F~(eta~) - eps (<s_x, a> + <s_y, b>).
    Returns (dX, da, dY, db, (W_bar, W_xy, W_xx, W_yy), (res_xy, res_xx,
    res_yy))."""
    a = np.asarray(a, F64)
    b = np.asarray(b, F64)
    Phx = gaussian_features(X, U, eps, q)
    Phy = gaussian_features(Y, U, eps, q)
    Px, sx = gaussian_features_scaled(X, U, eps, q)
    Py, sy = gaussian_features_scaled(Y, U, eps, q)
    runs, vals, sc = [], [], []
    for P, Q, p, g, sp, sq in ((Px, Py, a, b, sx, sy), (Px, Px, a, a, sx, sx),
                               (Py, Py, b, b, sy, sy)):
        res = accelerated_sinkhorn(lambda v, P=P, Q=Q: P @ (Q.T @ v),
                                   lambda u, P=P, Q=Q: Q @ (P.T @ u), p, g,
                                   fixed_iter=fixed_iter, L0=L0)
        runs.append(res)
        vals.append(dual_value(res.eta1, res.eta2, P @ Q.T, p, g, eps)
                    - eps * (sp @ p + sq @ g))
        sc.append((np.exp(res.eta1 - sp), np.exp(res.eta2 - sq)))
    dX, da, dY, db = grads_from_scalings(X, Y, U, eps, Phx, Phy, *sc)
    value = (vals[0] - 0.5 * (vals[1] + vals[2]), vals[0], vals[1], vals[2])
    return dX, da, dY, db, value, tuple(runs)


def _grad_anchors_one_solve(Zr, Zc, U, eps, q, Pr, Pc, p, g):
    """Gradient of W_hat of one solve with respect to the anchors.

    With K_ij = sum_k phi_k(z_i) phi_k(z'_j) and, from the log-feature of
    Lemma 1, d log phi_k(z) / d u_k = (4/eps)(z - u_k) + (2/(eps q)) u_k,
    the envelope gradient dW/dK = -eps p g^T of Prop. 3.2 gives
        dW/du_k = -eps [ (sum_j g_j phi_k(z'_j)) sum_i p_i phi_k(z_i) dlog phi_k(z_i)
                        + (sum_i p_i phi_k(z_i)) sum_j g_j phi_k(z'_j) dlog phi_k(z'_j) ].
    """
    Zr = np.asarray(Zr, F64)
    Zc = np.asarray(Zc, F64)
    U = np.asarray(U, F64)
    Wr = p[:, None] * Pr                          # p_i phi_k(z_i)
    Wc = g[:, None] * Pc                          # g_j phi_k(z'_j)
    zr = Wr.sum(0)
    zc = Wc.sum(0)
    dr = (4.0 / eps) * (Wr.T @ Zr - zr[:, None] * U) + (2.0 / (eps * q)) * zr[:, None] * U
    dc = (4.0 / eps) * (Wc.T @ Zc - zc[:, None] * U) + (2.0 / (eps * q)) * zc[:, None] * U
    return -eps * (zc[:, None] * dr + zr[:, None] * dc)


def divergence_grad_anchors(X, Y, a, b, U, eps: float, q: float, tol: float = 1e-13,
                            max_iter: int = 100000, fixed_iter: int = 0):
    """Gradient of the divergence with respect to the anchors U (r x d),
    with q held fixed: dW_bar/dU = G(xy) - (G(xx) + G(yy)) / 2, each G from
    the envelope gradient of Prop. 3.2 through the feature map.
    Returns (dU, Divergence)."""
    Phx = gaussian_features(X, U, eps, q)
    Phy = gaussian_features(Y, U, eps, q)
    sx = gaussian_log_features(X, U, eps, q).max(1)
    sy = gaussian_log_features(Y, U, eps, q).max(1)
    kw = dict(tol=tol, max_iter=max_iter, fixed_iter=fixed_iter)
    xy = sinkhorn_dense(Phx @ Phy.T, a, b, u0=np.exp(-sx), **kw)
    xx = sinkhorn_dense(Phx @ Phx.T, a, a, u0=np.exp(-sx), **kw)
    yy = sinkhorn_dense(Phy @ Phy.T, b, b, u0=np.exp(-sy), **kw)
    wxy = w_hat(xy.u, xy.v, a, b, eps)
    wxx = w_hat(xx.u, xx.v, a, a, eps)
    wyy = w_hat(yy.u, yy.v, b, b, eps)
    div = Divergence(wxy - 0.5 * (wxx + wyy), wxy, wxx, wyy, xy, xx, yy)
    dU = (_grad_anchors_one_solve(X, Y, U, eps, q, Phx, Phy, xy.u, xy.v)
          - 0.5 * (_grad_anchors_one_solve(X, X, U, eps, q, Phx, Phx, xx.u, xx.v)
                   + _grad_anchors_one_solve(Y, Y, U, eps, q, Phy, Phy, yy.u, yy.v)))
    return dU, div


def grad_x_exact_kernel(X, Y, a, b, eps: float, tol: float = 1e-13,
                        max_iter: int = 100000):
    """Gradient of W(mu, nu) in X for the exact squared-Euclidean cost:
    dW/dx_i = sum_j P_ij 2 (x_i - y_j) = 2 (a_i x_i - sum_j P_ij y_j),
    P the optimal plan.  The limit r -> infinity of the feature gradient."""
    X = np.asarray(X, F64)
    Y = np.asarray(Y, F64)
    K = gaussian_kernel(X, Y, eps)
    res = sinkhorn_dense(K, a, b, tol=tol, max_iter=max_iter)
    P = res.u[:, None] * K * res.v[None, :]
    return 2.0 * (P.sum(1)[:, None] * X - P @ Y)
