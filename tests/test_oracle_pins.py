"""Pins of the FP64 oracle against facts fixed by the paper and by
mathematics, independent of the oracle's own code (no GPU needed).

Each test names the passage of the paper it checks.  They are chosen so
that a dropped term, a wrong sign, a transposed operand or a wrong constant
anywhere in the oracle fails at least one of them.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2006_07057_amd import inputs

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _rng(seed):
    return np.random.default_rng(seed)


# ------------------------------------------------------------------ Lemma 1
@pytest.mark.parametrize("R,eps,d", [(1.0, 1.0, 1), (4.0, 0.1, 3),
                                     (2.5, 0.05, 64), (30.0, 10.0, 784),
                                     (1e-3, 1.0, 2)])
def test_lambert_q_defining_identity(R, eps, d):
    """Lemma 1: q = z / (2 W0(z)) with z = R^2/(eps d).  Since
    W0(z) e^{W0(z)} = z, this is equivalent to 2q log(2q) = z and q > 1/2,
    an identity that does not use any Lambert routine."""
    q = oracle.lambert_q(R, eps, d)
    z = R * R / (eps * d)
    assert q > 0.5
    assert 2 * q * math.log(2 * q) == pytest.approx(z, rel=1e-12, abs=1e-15)


def test_lambert_known_values():
    """W0(1) is the omega constant 0.567143290409783872...; W0(e) = 1."""
    # z = R^2/(eps d) = e  ->  W0 = 1  ->  q = e/2
    q = oracle.lambert_q(math.sqrt(math.e), 1.0, 1)
    assert q == pytest.approx(math.e / 2, rel=1e-14)
    q1 = oracle.lambert_q(1.0, 1.0, 1)
    assert q1 == pytest.approx(1.0 / (2 * 0.5671432904097838730), rel=1e-14)


def _gh_rule(k, d, tau):
    """Tensor probabilists' Gauss-Hermite rule for N(0, tau^2 I_d):
    E f(u) ~ sum_i w_i f(u_i).  Returns nodes (k^d, d), weights (k^d,)."""
    t, w = np.polynomial.hermite_e.hermegauss(k)
    w = w / math.sqrt(2 * math.pi)
    grids = np.meshgrid(*([t] * d), indexing="ij")
    nodes = tau * np.stack([g.ravel() for g in grids], 1)
    weights = np.ones(nodes.shape[0])
    for g in np.meshgrid(*([w] * d), indexing="ij"):
        weights = weights * g.ravel()
    return nodes, weights


def _quadrature_kernel(pts, eps, q, k, d):
    """E_{u~rho} phi(x,u) phi(y,u), rho = N(0, sigma^2 I), sigma^2 = q eps/4
    (Lemma 1), by Gauss-Hermite quadrature.  The rule is taken for
    N(0, tau^2 I) with tau^2 = eps/8, the width of the integrand, and the
    density ratio rho/N(0, tau^2) is folded into the weights, so the
    remaining integrand is exp(linear) and the rule converges to rounding.
    The anchors are the nodes; r * weight replaces the 1/r of phi_theta."""
    s2 = oracle.sigma2_from_q(q, eps)
    tau2 = eps / 8.0
    U, w = _gh_rule(k, d, math.sqrt(tau2))
    u2 = (U * U).sum(1)
    ratio = (tau2 / s2) ** (d / 2) * np.exp(-u2 / (2 * s2) + u2 / (2 * tau2))
    r = U.shape[0]
    L = oracle.gaussian_log_features(pts, U, eps, q)
    return (np.exp(L[:, None, :] + L[None, :, :]) * (r * w * ratio)).sum(-1)


@pytest.mark.parametrize("eps,q", [(1.0, 1.0), (0.5, 8.0), (2.0, 3.3),
                                   (0.3, 0.75)])
def test_feature_map_reproduces_gaussian_kernel_1d(eps, q):
    """Lemma 1: k(x,y) = exp(-|x-y|^2/eps) = E_{u~N(0, q eps/4)}
    phi(x,u) phi(y,u), for any q > 1/2."""
    pts = np.array([[-0.7], [0.0], [0.35], [1.1]])
    quad = _quadrature_kernel(pts, eps, q, 80, 1)
    exact = oracle.gaussian_kernel(pts, pts, eps)
    np.testing.assert_allclose(quad, exact, rtol=1e-12, atol=0)


def test_feature_map_reproduces_gaussian_kernel_2d():
    """Lemma 1 in d = 2 (tensor rule): checks the (2q)^{d/4} factor, which
    a 1-D test cannot tell apart from (2q)^{1/4}."""
    pts = np.array([[0.1, -0.2], [0.5, 0.4], [-0.6, 0.3]])
    for eps, q in ((0.8, 2.0), (0.5, 8.0)):
        quad = _quadrature_kernel(pts, eps, q, 50, 2)
        exact = oracle.gaussian_kernel(pts, pts, eps)
        np.testing.assert_allclose(quad, exact, rtol=1e-11, atol=0)


def test_rf_kernel_unbiased_and_error_shrinks_with_r():
    """Eq. (general) with i.i.d. anchors: K_theta is an unbiased Monte-Carlo
    estimate of k, and (Prop. 3.1) the ratio error sup|K_theta/k - 1|
    shrinks like r^{-1/2}.  Median over anchor seeds."""
    rng = _rng(1)
    X = rng.standard_normal((12, 2)) * 0.5
    Y = rng.standard_normal((10, 2)) * 0.5 + 0.3
    eps = 1.0
    R = inputs.max_norm(X, Y)
    q = oracle.lambert_q(R, eps, 2)
    s2 = oracle.sigma2_from_q(q, eps)
    K = oracle.gaussian_kernel(X, Y, eps)
    errs = {}
    for r in (64, 1024, 16384):
        e = []
        for seed in range(9):
            U = np.sqrt(s2) * inputs.standard_normal_anchors(seed, r, 2)
            e.append(np.abs(oracle.rf_kernel(X, Y, U, eps, q) / K - 1).max())
        errs[r] = float(np.median(e))
    assert errs[1024] < errs[64] / 2.0
    assert errs[16384] < errs[1024] / 2.0
    assert errs[16384] < 0.25 * errs[64] * 1.0
    # unbiasedness: average of many independent small-r estimates
    acc = np.zeros_like(K)
    N = 400
    for seed in range(N):
        U = np.sqrt(s2) * inputs.standard_normal_anchors(1000 + seed, 32, 2)
        acc += oracle.rf_kernel(X, Y, U, eps, q)
    ratio = acc / N / K
    assert abs(np.median(ratio) - 1) < 0.03


def test_scaled_features_reconstruct():
    """The row scaling is exact: Phi = diag(e^s) Phi~ and max_k Phi~_ik = 1."""
    rng = _rng(2)
    X = rng.standard_normal((20, 3))
    U = rng.standard_normal((16, 3))
    P = oracle.gaussian_features(X, U, 0.7, 1.3)
    Pt, s = oracle.gaussian_features_scaled(X, U, 0.7, 1.3)
    np.testing.assert_allclose(Pt * np.exp(s)[:, None], P, rtol=1e-13)
    np.testing.assert_allclose(Pt.max(1), 1.0, rtol=0, atol=0)


# ------------------------------------------------------------- Algorithm 1
def _small_problem(seed, n, m, d=2, r=16, eps=0.5):
    rng = _rng(seed)
    X = rng.standard_normal((n, d))
    Y = rng.standard_normal((m, d)) + 0.5
    a = rng.dirichlet(np.ones(n))
    b = rng.dirichlet(np.ones(m))
    q = oracle.lambert_q(inputs.max_norm(X, Y), eps, d)
    U = np.sqrt(oracle.sigma2_from_q(q, eps)) * rng.standard_normal((r, d))
    return X, Y, a, b, U, eps, q


def test_sinkhorn_marginals_and_unit_mass():
    """Alg. 1 fixed point: after the u-update the row marginal of
    P = diag(u) K diag(v) is a exactly; at exit the column error is below
    the tolerance; u^T K v = 1 (the remark after Eq. (eval-dual))."""
    X, Y, a, b, U, eps, q = _small_problem(3, 9, 7)
    K = oracle.rf_kernel(X, Y, U, eps, q)
    res = oracle.sinkhorn_dense(K, a, b, tol=1e-12, max_iter=100000)
    assert res.converged
    P = res.u[:, None] * K * res.v[None, :]
    np.testing.assert_allclose(P.sum(1), a, rtol=1e-13)
    assert np.abs(P.sum(0) - b).sum() < 1e-12
    assert res.u @ K @ res.v == pytest.approx(1.0, abs=1e-13)
    # fixed-iteration mode: exactly that many pairs, mass 1 already
    r5 = oracle.sinkhorn_dense(K, a, b, fixed_iter=5)
    assert r5.iters == 5
    assert r5.u @ K @ r5.v == pytest.approx(1.0, abs=1e-13)


def test_sinkhorn_matches_2x2_bisection():
    """Brute force for n = m = 2: the plan has one free entry; the primal
    Eq. (reg-ot) minimised by bisection must equal the dual estimate
    Eq. (dual-estimate) of the converged Alg. 1."""
    for seed in range(5):
        rng = _rng(10 + seed)
        K = np.exp(-rng.uniform(0, 3, size=(2, 2)))
        a = rng.dirichlet(np.ones(2))
        b = rng.dirichlet(np.ones(2))
        eps = rng.uniform(0.2, 2.0)
        val, P = brute.primal_2x2(K, a, b, eps)
        res = oracle.sinkhorn_dense(K, a, b, tol=1e-15, max_iter=100000)
        assert oracle.w_hat(res.u, res.v, a, b, eps) == pytest.approx(
            val, rel=1e-11, abs=1e-13)
        Ps = res.u[:, None] * K * res.v[None, :]
        np.testing.assert_allclose(Ps, P, rtol=1e-9, atol=1e-14)


@pytest.mark.parametrize("n,m", [(3, 5), (8, 8), (6, 2)])
def test_sinkhorn_matches_dual_maximiser(n, m):
    """Eq. (dual-theta): a generic Newton trust-region maximiser of the
    concave dual gives the same value as Alg. 1 + Eq. (dual-estimate), and
    alpha* = eps log u* up to the constant shift of App. B."""
    X, Y, a, b, U, eps, q = _small_problem(20 + n, n, m, r=6)
    K = oracle.rf_kernel(X, Y, U, eps, q)
    val, al, be = brute.dual_max(K, a, b, eps)
    res = oracle.sinkhorn_dense(K, a, b, tol=1e-15, max_iter=1000000)
    assert oracle.w_hat(res.u, res.v, a, b, eps) == pytest.approx(
        val, rel=1e-10, abs=1e-12)
    la = eps * np.log(res.u)
    np.testing.assert_allclose(la - la[0], al, rtol=1e-7, atol=1e-9)


def test_primal_dual_equality():
    """No duality gap for positive kernels (Sec. 3.1): the primal objective
    of Eq. (reg-ot) at P = diag(u)K diag(v) equals Eq. (dual-estimate)."""
    X, Y, a, b, U, eps, q = _small_problem(4, 40, 30, r=32)
    K = oracle.rf_kernel(X, Y, U, eps, q)
    res = oracle.sinkhorn_dense(K, a, b, tol=1e-14, max_iter=1000000)
    P = res.u[:, None] * K * res.v[None, :]
    assert oracle.primal_objective(P, K, eps) == pytest.approx(
        oracle.w_hat(res.u, res.v, a, b, eps), rel=1e-10)


def test_factored_equals_dense():
    """Sec. 3.1: K_theta = Xi^T Zeta, so the factored r(n+m) iteration is
    the dense one re-associated; iterates agree to rounding."""
    X, Y, a, b, U, eps, q = _small_problem(5, 50, 40, r=24)
    Px = oracle.gaussian_features(X, U, eps, q)
    Py = oracle.gaussian_features(Y, U, eps, q)
    rd = oracle.sinkhorn_dense(Px @ Py.T, a, b, fixed_iter=50)
    rf = oracle.sinkhorn_factored(Px, Py, a, b, fixed_iter=50)
    np.testing.assert_allclose(rf.u, rd.u, rtol=1e-12)
    np.testing.assert_allclose(rf.v, rd.v, rtol=1e-12)
    assert rf.err == pytest.approx(rd.err, rel=1e-8, abs=1e-15)


def test_scaled_iteration_equals_unscaled():
    """The row-scaled problem from u~0 = 1 is Alg. 1 from u0 = e^{-s_x}:
    the iterates differ exactly by the factors e^{s}, and the dual
    estimates coincide."""
    rng = _rng(6)
    X = rng.standard_normal((30, 2))
    Y = rng.standard_normal((25, 2)) + 1.0
    a = rng.dirichlet(np.ones(30))
    b = rng.dirichlet(np.ones(25))
    eps, q = 0.5, 8.0
    U = rng.standard_normal((40, 2))
    d1 = oracle.divergence(X, Y, a, b, U, eps, q, fixed_iter=30)
    d2 = oracle.divergence_scaled(X, Y, a, b, U, eps, q, fixed_iter=30)
    _, sx = oracle.gaussian_features_scaled(X, U, eps, q)
    _, sy = oracle.gaussian_features_scaled(Y, U, eps, q)
    np.testing.assert_allclose(d2.xy.u * np.exp(-sx), d1.xy.u, rtol=1e-11)
    np.testing.assert_allclose(d2.xy.v * np.exp(-sy), d1.xy.v, rtol=1e-11)
    for f in ("value", "w_xy", "w_xx", "w_yy"):
        assert getattr(d2, f) == pytest.approx(getattr(d1, f), rel=1e-11,
                                               abs=1e-12)


def test_dual_range_bound():
    """App. B lemma: max alpha* - min alpha* <= eps R(K) with
    R(K) = -log(iota min K / max K), iota = min(a_i, b_j)."""
    X, Y, a, b, U, eps, q = _small_problem(7, 20, 15, r=12)
    K = oracle.rf_kernel(X, Y, U, eps, q)
    res = oracle.sinkhorn_dense(K, a, b, tol=1e-14, max_iter=1000000)
    iota = min(a.min(), b.min())
    RK = -math.log(iota * K.min() / K.max())
    la, lb = np.log(res.u), np.log(res.v)
    assert la.max() - la.min() <= RK + 1e-9
    assert lb.max() - lb.min() <= RK + 1e-9


# ------------------------------------------------------- divergence (reg-sdiv)
def test_divergence_translation_closed_form():
    """Exact Gaussian kernel (the r -> infinity limit, squared Euclidean
    cost): for nu = mu shifted by m with the same weights, the cross term
    -2 m^T (x_i - x_j) of the cost is separable and integrates to zero, so
    W(mu, nu) = W(mu, mu) + ||m||^2 and W(nu, nu) = W(mu, mu); hence the
    divergence of Eq. (reg-sdiv) is exactly ||m||^2."""
    rng = _rng(8)
    for eps in (0.3, 1.0, 4.0):
        X = rng.standard_normal((25, 2))
        shift = np.array([0.7, -1.2])
        Y = X + shift
        a = rng.dirichlet(np.ones(25))
        kw = dict(tol=1e-13, max_iter=1000000)
        dv = oracle.divergence_from_kernels(
            oracle.gaussian_kernel(X, Y, eps), oracle.gaussian_kernel(X, X, eps),
            oracle.gaussian_kernel(Y, Y, eps), a, a, eps, **kw)
        assert dv.value == pytest.approx(float(shift @ shift), rel=1e-9)
        assert dv.w_xx == pytest.approx(dv.w_yy, rel=1e-9)


def test_divergence_symmetry_and_self_zero():
    """W(mu,nu) = W(nu,mu) (swap X<->Y with a<->b transposes K); the
    divergence of a measure with itself (any point order) is 0."""
    X, Y, a, b, U, eps, q = _small_problem(9, 30, 22, r=20)
    kw = dict(tol=1e-13, max_iter=1000000)
    d1 = oracle.divergence(X, Y, a, b, U, eps, q, **kw)
    d2 = oracle.divergence(Y, X, b, a, U, eps, q, **kw)
    assert d1.value == pytest.approx(d2.value, rel=1e-10)
    assert d1.w_xy == pytest.approx(d2.w_xy, rel=1e-10)
    perm = _rng(1).permutation(30)
    d0 = oracle.divergence(X, X[perm], a, a[perm], U, eps, q, **kw)
    assert abs(d0.value) < 1e-11


def test_divergence_permutation_invariance():
    """Jointly permuting (x_i, a_i) permutes the rows of K and leaves every
    term of Eq. (reg-sdiv) unchanged."""
    X, Y, a, b, U, eps, q = _small_problem(11, 26, 19, r=20)
    kw = dict(tol=1e-12, max_iter=1000000)
    d1 = oracle.divergence(X, Y, a, b, U, eps, q, **kw)
    p = _rng(2).permutation(26)
    d2 = oracle.divergence(X[p], Y, a[p], b, U, eps, q, **kw)
    assert d1.value == pytest.approx(d2.value, rel=1e-10)


# --------------------------------------------------------------- gradients
def _fd(f, x0, h):
    g = np.zeros_like(x0)
    for idx in np.ndindex(x0.shape):
        xp = x0.copy()
        xm = x0.copy()
        xp[idx] += h
        xm[idx] -= h
        g[idx] = (f(xp) - f(xm)) / (2 * h)
    return g


def test_gradients_match_finite_differences():
    """Prop. 3.2 + the chain rule of Sec. 3.3 (both sides of the self
    terms): central differences of the converged divergence in X, Y, and
    in a, b along directions that stay on the simplex."""
    X, Y, a, b, U, eps, q = _small_problem(12, 6, 5, r=10, eps=0.7)
    kw = dict(tol=1e-14, max_iter=1000000)
    dX, da, dY, db, _ = oracle.divergence_grad(X, Y, a, b, U, eps, q, **kw)

    def fX(Xp):
        return oracle.divergence(Xp, Y, a, b, U, eps, q, **kw).value

    def fY(Yp):
        return oracle.divergence(X, Yp, a, b, U, eps, q, **kw).value

    np.testing.assert_allclose(dX, _fd(fX, X, 1e-5), rtol=1e-6, atol=1e-9)
    np.testing.assert_allclose(dY, _fd(fY, Y, 1e-5), rtol=1e-6, atol=1e-9)
    h = 1e-6
    for i, j in [(0, 1), (2, 5), (4, 3)]:
        e = np.zeros(6)
        e[i], e[j] = 1.0, -1.0
        fd = (oracle.divergence(X, Y, a + h * e, b, U, eps, q, **kw).value
              - oracle.divergence(X, Y, a - h * e, b, U, eps, q, **kw).value
              ) / (2 * h)
        assert da @ e == pytest.approx(fd, rel=1e-6, abs=1e-9)
    for i, j in [(0, 4), (1, 2)]:
        e = np.zeros(5)
        e[i], e[j] = 1.0, -1.0
        fd = (oracle.divergence(X, Y, a, b + h * e, U, eps, q, **kw).value
              - oracle.divergence(X, Y, a, b - h * e, U, eps, q, **kw).value
              ) / (2 * h)
        assert db @ e == pytest.approx(fd, rel=1e-6, abs=1e-9)
    assert abs(da.sum()) < 1e-12 and abs(db.sum()) < 1e-12


def _frozen_value(X, Y, a, b, U, eps, q, sc):
    """The dual estimates' combination with the scalings of the three solves
    frozen at sc = ((u_xy, v_xy), (u_xx, v_xx), (u_yy, v_yy)): for one solve
    on K = Phi_r Phi_c^T with weights (p, g),
        D = eps (p^T log u + g^T log v) - eps u^T K v,
    the dual objective of Eq. (eval-dual) written with the scalings (its
    value at a Sinkhorn iterate is the dual estimate plus the constant
    -eps u^T K v = -eps).  Returns D_xy - (D_xx + D_yy) / 2."""
    Px = oracle.gaussian_features(X, U, eps, q)
    Py = oracle.gaussian_features(Y, U, eps, q)
    out = 0.0
    for (P, Q, p, g), (u, v), c in zip(((Px, Py, a, b), (Px, Px, a, a), (Py, Py, b, b)),
                                       sc, (1.0, -0.5, -0.5)):
        out += c * eps * (p @ np.log(u) + g @ np.log(v) - u @ (P @ (Q.T @ v)))
    return out


def test_fixed_iteration_gradients_are_frozen_scaling_derivatives():
    """Off convergence (5 iterations, where the two sides of a self-problem
    still differ: u_xx != v_xx), the gradient readings the GPU is compared
    with at fixed iteration counts (both sides of the self terms, weight
    gradient eps(log u_xy - (log u_xx + log v_xx)/2)) are exactly the
    derivatives of the dual objective with the iterates' scalings held
    fixed (Prop. 3.2's envelope form dW/dK = -eps u v^T applied at those
    scalings).  Central differences of that frozen function in X, Y, U and
    along simplex directions of a, b pin the formulas at any iteration
    count; using one side twice, or dropping log v_xx, fails here."""
    X, Y, a, b, U, eps, q = _small_problem(19, 7, 6, r=9, eps=0.7)
    dX, da, dY, db, div = oracle.divergence_grad(X, Y, a, b, U, eps, q, fixed_iter=5)
    sc = ((div.xy.u, div.xy.v), (div.xx.u, div.xx.v), (div.yy.u, div.yy.v))
    assert np.max(np.abs(np.log(div.xx.u / div.xx.v))) > 1e-3   # really off convergence
    f = lambda **kw: _frozen_value(kw.get("X", X), kw.get("Y", Y), kw.get("a", a),
                                   kw.get("b", b), kw.get("U", U), eps, q, sc)
    np.testing.assert_allclose(dX, _fd(lambda Z: f(X=Z), X, 1e-5), rtol=1e-7, atol=1e-10)
    np.testing.assert_allclose(dY, _fd(lambda Z: f(Y=Z), Y, 1e-5), rtol=1e-7, atol=1e-10)
    dU, _ = oracle.divergence_grad_anchors(X, Y, a, b, U, eps, q, fixed_iter=5)
    np.testing.assert_allclose(dU, _fd(lambda Z: f(U=Z), U, 1e-5), rtol=1e-7, atol=1e-10)
    h = 1e-3      # the frozen function is linear in the weights
    for wts, grad, key in ((a, da, "a"), (b, db, "b")):
        for i, j in [(0, 1), (2, 4), (5, 3)]:
            e = np.zeros(len(wts))
            e[i], e[j] = 1.0, -1.0
            fd = (f(**{key: wts + h * e}) - f(**{key: wts - h * e})) / (2 * h)
            assert grad @ e == pytest.approx(fd, rel=1e-9, abs=1e-12), (key, i, j)


def test_scaled_gradient_equals_unscaled_and_fd_at_large_d():
    """divergence_grad_scaled equals divergence_grad where raw features are
    representable, and at d = 128 (raw features below float64 range for
    part of the anchors) it matches a central difference of
    divergence_scaled along a random direction."""
    X, Y, a, b, U, eps, q = _small_problem(12, 9, 4, r=16, eps=0.7)
    kw = dict(tol=1e-14, max_iter=1000000)
    ref = oracle.divergence_grad(X, Y, a, b, U, eps, q, **kw)
    got = oracle.divergence_grad_scaled(X, Y, a, b, U, eps, q, **kw)
    for g, r_ in zip(got[:4], ref[:4]):
        np.testing.assert_allclose(g, r_, rtol=1e-9, atol=1e-12)
    rng = np.random.default_rng(8)
    n, m, d, r = 10, 8, 128, 24
    X = rng.standard_normal((n, d))
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    Y = rng.standard_normal((m, d))
    Y /= np.linalg.norm(Y, axis=1, keepdims=True)
    a = rng.dirichlet(np.ones(n))
    b = rng.dirichlet(np.ones(m))
    eps = 1.0
    q = oracle.lambert_q(1.0, eps, d)
    U = rng.standard_normal((r, d)) * math.sqrt(oracle.sigma2_from_q(q, eps))
    dX, da, dY, db, _ = oracle.divergence_grad_scaled(X, Y, a, b, U, eps, q, **kw)
    D = rng.standard_normal(X.shape)
    h = 1e-5
    fd = (oracle.divergence_scaled(X + h * D, Y, a, b, U, eps, q, **kw).value
          - oracle.divergence_scaled(X - h * D, Y, a, b, U, eps, q, **kw).value) / (2 * h)
    assert float((dX * D).sum()) == pytest.approx(fd, rel=1e-6, abs=1e-10)


def test_anchor_gradient_matches_finite_differences():
    """Gradient with respect to the anchors (q fixed): central differences
    of the converged divergence in every anchor coordinate."""
    X, Y, a, b, U, eps, q = _small_problem(14, 7, 6, r=5, eps=0.8)
    kw = dict(tol=1e-14, max_iter=1000000)
    dU, div = oracle.divergence_grad_anchors(X, Y, a, b, U, eps, q, **kw)
    assert div.value == pytest.approx(oracle.divergence(X, Y, a, b, U, eps, q, **kw).value,
                                      rel=1e-12)

    def fU(Up):
        return oracle.divergence(X, Y, a, b, Up, eps, q, **kw).value

    np.testing.assert_allclose(dU, _fd(fU, U, 1e-5), rtol=1e-6, atol=1e-9)


def test_point_gradient_large_r_limit():
    """As r grows K_theta -> exp(-||x-y||^2/eps) and the row-side feature
    gradient of W(mu,nu) tends to the squared-Euclidean Sinkhorn gradient
    2(a_i x_i - sum_j P_ij y_j).  The error must shrink with r."""
    rng = _rng(13)
    X = rng.standard_normal((7, 2)) * 0.4
    Y = rng.standard_normal((6, 2)) * 0.4 + 0.2
    a = rng.dirichlet(np.ones(7))
    b = rng.dirichlet(np.ones(6))
    eps = 1.0
    q = oracle.lambert_q(inputs.max_norm(X, Y), eps, 2)
    s2 = oracle.sigma2_from_q(q, eps)
    exact = oracle.grad_x_exact_kernel(X, Y, a, b, eps)
    errs = {}
    for r in (100, 10000):
        e = []
        for seed in range(5):
            U = np.sqrt(s2) * inputs.standard_normal_anchors(50 + seed, r, 2)
            Px = oracle.gaussian_features(X, U, eps, q)
            Py = oracle.gaussian_features(Y, U, eps, q)
            res = oracle.sinkhorn_dense(Px @ Py.T, a, b, tol=1e-13,
                                        max_iter=1000000)
            g = Px * (Py.T @ res.v)[None, :]
            G = 4 * res.u[:, None] * (g.sum(1)[:, None] * X - g @ U)
            e.append(np.linalg.norm(G - exact) / np.linalg.norm(exact))
        errs[r] = float(np.median(e))
    assert errs[10000] < errs[100] / 3.0
    assert errs[10000] < 0.1


# --------------------------------------------------------- arc-cosine kernel
@pytest.mark.parametrize("s", [0, 1, 2])
def test_arccos_closed_form_matches_defining_integral(s):
    """k_s(x, y) = E_{u ~ N(0, I)} Theta_s(u.x) Theta_s(u.y) with
    Theta_s(w) = sqrt(2) max(0, w)^s, integrated numerically in polar
    coordinates (d = 2), against the closed form in J_s."""
    from scipy import integrate
    rng = _rng(40 + s)
    X = rng.standard_normal((3, 2))
    Y = rng.standard_normal((2, 2))
    K = oracle.arccos_kernel(X, Y, s, kappa=0.0)
    radial, _ = integrate.quad(lambda p: p ** (2 * s + 1) * math.exp(-p * p / 2), 0, np.inf)
    alpha = np.linspace(0.0, 2 * np.pi, 400001)[:-1]
    dirs = np.stack([np.cos(alpha), np.sin(alpha)], 1)
    for i, x in enumerate(X):
        for j, y in enumerate(Y):
            px, py = dirs @ x, dirs @ y
            if s == 0:
                ang = np.mean((px > 0) & (py > 0))
            else:
                ang = np.mean(np.maximum(px, 0) ** s * np.maximum(py, 0) ** s)
            val = 2.0 * radial * ang          # (1/2pi) d alpha, rho e^{-rho^2/2} d rho
            assert K[i, j] == pytest.approx(val, rel=1e-5, abs=1e-9)


@pytest.mark.parametrize("s", [0, 1, 2])
def test_arccos_feature_map_integrates_to_kernel_1d(s):
    """d = 1: integrating phi(x, u) phi(y, u) against rho = N(0, sigma^2)
    (the importance weights of the lemma) gives k_s + kappa."""
    from scipy import integrate
    sigma, kappa = 1.7, 0.3
    for x, y in [(0.8, 1.3), (-0.5, -2.0), (0.7, -1.1)]:
        def phi(z, u):
            w = max(0.0, u * z)
            base = w ** s if s > 0 else (1.0 if w > 0 else 0.0)
            return (sigma ** 0.5) * math.sqrt(2.0) * base * math.exp(-u * u * (1 - 1 / sigma ** 2) / 4)
        dens = lambda u: math.exp(-u * u / (2 * sigma ** 2)) / (sigma * math.sqrt(2 * math.pi))
        val = sum(integrate.quad(lambda u: phi(x, u) * phi(y, u) * dens(u), lo, hi)[0]
                  for lo, hi in ((-np.inf, 0.0), (0.0, np.inf))) + kappa
        ref = oracle.arccos_kernel(np.array([[x]]), np.array([[y]]), s, kappa)[0, 0]
        assert val == pytest.approx(ref, rel=1e-7, abs=1e-10)


def test_arccos_features_converge_to_kernel():
    """Products of the r + 1 features are unbiased for k_{s,kappa} and their
    error shrinks like r^{-1/2} (Prop. 3.1 for this map)."""
    rng = _rng(50)
    X = rng.standard_normal((5, 3)) * 0.7
    Y = rng.standard_normal((4, 3)) * 0.7
    s, sigma, kappa = 1, 1.4, 0.5
    K = oracle.arccos_kernel(X, Y, s, kappa)
    errs = {}
    for r in (256, 16384):
        e = []
        for seed in range(8):
            U = _rng(1000 + seed).standard_normal((r, 3)) * sigma
            Kr = oracle.arccos_features(X, U, s, sigma, kappa) @ oracle.arccos_features(Y, U, s, sigma, kappa).T
            e.append(np.abs(Kr / K - 1).mean())
        errs[r] = np.median(e)
    assert errs[16384] < errs[256] / 4
    # unbiased: the mean over many small draws is close to the kernel
    acc = np.zeros_like(K)
    T = 400
    for seed in range(T):
        U = _rng(5000 + seed).standard_normal((32, 3)) * sigma
        acc += oracle.arccos_features(X, U, s, sigma, kappa) @ oracle.arccos_features(Y, U, s, sigma, kappa).T
    assert np.abs(acc / T / K - 1).max() < 0.05
