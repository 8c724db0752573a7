"""Accelerated Sinkhorn (the acceleration remark of Sec. 3.1 and the
accelerated algorithm of the appendix): pins of the oracle against facts
that do not come from its own code, and (GPU) parity of the device solver
with it."""
import math

import numpy as np
import pytest

import oracle
from paper_2006_07057_amd import inputs

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _clouds(seed, n=40, m=35, d=2):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, d))
    Y = rng.standard_normal((m, d)) + 1.0
    a = rng.dirichlet(np.ones(n))
    b = rng.dirichlet(np.ones(m))
    return X, Y, a, b


def _phi(K, a, b, e1, e2):
    """The minimised function, written from its definition."""
    return math.log(np.exp(e1) @ K @ np.exp(e2)) - e1 @ a - e2 @ b


def _acc(K, a, b, **kw):
    return oracle.accelerated_sinkhorn(lambda v: K @ v, lambda u: K.T @ u, a, b, **kw)


def _sinkhorn_optimum(K, a, b, eps):
    sk = oracle.sinkhorn_dense(K, a, b, tol=1e-12, max_iter=400000)
    assert sk.converged
    return sk, oracle.w_hat(sk.u, sk.v, a, b, eps)


@pytest.mark.parametrize("eps", [1.0, 0.1])
def test_acc_oracle_reaches_algorithm1_optimum(eps):
    """Both algorithms solve the same dual problem (Eq. dual-smooth is a
    reformulation of the dual of Eq. reg-ot): the dual value of the
    accelerated point equals Algorithm 1's estimate at convergence, and the
    plan diag(e^eta1) K diag(e^eta2) it returns has the marginals a, b."""
    X, Y, a, b = _clouds(0)
    K = oracle.gaussian_kernel(X, Y, eps)
    _, W = _sinkhorn_optimum(K, a, b, eps)
    res = _acc(K, a, b, tol=1e-9, max_iter=5000)
    assert res.converged
    assert oracle.dual_value(res.eta1, res.eta2, K, a, b, eps) == pytest.approx(W, rel=1e-10)
    P = np.exp(res.eta1)[:, None] * K * np.exp(res.eta2)[None, :]
    assert np.abs(P.sum(1) - a).sum() + np.abs(P.sum(0) - b).sum() < 1e-8


@pytest.mark.parametrize("eps", [1.0, 0.1])
def test_acc_oracle_weak_duality_and_rate(eps):
    """Every iterate is a dual point, so eps * (-phi) never exceeds the
    optimum (weak duality).  The estimate-sequence argument behind
    accelerated alternating minimisation bounds the gap by
    A_k (phi(eta^k) - phi*) <= ||eta* - eta^0||^2 / 2 for the optimum eta*
    nearest to the start eta^0 = 0; a wrong momentum weight, step sign or
    test breaks it."""
    X, Y, a, b = _clouds(1)
    K = oracle.gaussian_kernel(X, Y, eps)
    sk, W = _sinkhorn_optimum(K, a, b, eps)
    al, be = np.log(sk.u), np.log(sk.v)
    # optima form the line (al + t, be - t); the nearest one to 0
    t = (be.sum() - al.sum()) / (len(al) + len(be))
    R2 = ((al + t) ** 2).sum() + ((be - t) ** 2).sum()
    phistar = -W / eps
    res = _acc(K, a, b, fixed_iter=200)
    assert res.iters == 200 and len(res.As) == 200
    for A, ph in zip(res.As, res.phis):
        assert -eps * ph <= W + 1e-12 * abs(W)
        assert A * (ph - phistar) <= 0.5 * R2 * (1 + 1e-9)
    # A_k grows at least like k^2 / (4 L_max) for accelerated methods
    assert res.As[-1] >= 200 ** 2 / (4.0 * max(res.Ls)) * 0.99


def test_acc_oracle_rank_one_closed_form():
    """For K = x y^T every coupling diag(u) K diag(v) is rank one, the
    optimal plan is a b^T and the dual optimum is
    sum a log(a/x) + sum b log(b/y) (eps = 1)."""
    rng = np.random.default_rng(2)
    x = rng.uniform(0.2, 3.0, 30)
    y = rng.uniform(0.2, 3.0, 25)
    a = rng.dirichlet(np.ones(30))
    b = rng.dirichlet(np.ones(25))
    K = np.outer(x, y)
    res = _acc(K, a, b, tol=1e-10, max_iter=5000)
    assert res.converged
    ref = float(a @ np.log(a / x) + b @ np.log(b / y))
    assert oracle.dual_value(res.eta1, res.eta2, K, a, b, 1.0) == pytest.approx(ref, rel=1e-11)


def test_acc_oracle_first_step():
    """From eta = zeta = 0 with A_0 = 0, the first step has a_1 = 1/L_1 and
    tau = 1, so lambda = 0: it minimises phi exactly over the block with
    the larger gradient at 0 (that block's marginal becomes exact) and moves
    zeta to -grad phi(0) / L_1.  The gradient is checked by central finite
    differences of phi written from its definition."""
    X, Y, a, b = _clouds(3, n=12, m=9)
    K = oracle.gaussian_kernel(X, Y, 0.5)
    L0 = 2.0e6                                  # the first trial (L0/2) passes
    res = _acc(K, a, b, fixed_iter=1, L0=L0)
    assert res.iters == 1 and res.trials == 1
    L1 = L0 / 2
    assert res.Ls == [L1] and res.As[0] == pytest.approx(1.0 / L1, rel=1e-14)
    n, m = len(a), len(b)
    h = 1e-6
    g = np.zeros(n + m)
    for i in range(n + m):
        e = np.zeros(n + m)
        e[i] = h
        g[i] = (_phi(K, a, b, e[:n], e[n:]) - _phi(K, a, b, -e[:n], -e[n:])) / (2 * h)
    np.testing.assert_allclose(np.concatenate([res.zeta1, res.zeta2]), -g / L1,
                               rtol=1e-6, atol=1e-12 / L1)
    blk = 1 if g[:n] @ g[:n] >= g[n:] @ g[n:] else 2
    assert res.blocks == [blk]
    P = np.exp(res.eta1)[:, None] * K * np.exp(res.eta2)[None, :]
    if blk == 1:
        np.testing.assert_allclose(P.sum(1), a, rtol=1e-13)
        np.testing.assert_array_equal(res.eta2, np.zeros(m))
    else:
        np.testing.assert_allclose(P.sum(0), b, rtol=1e-13)
        np.testing.assert_array_equal(res.eta1, np.zeros(n))


def test_acc_oracle_line_search_doubles():
    """A tiny starting estimate cannot pass the sufficient-decrease test
    (the function is smooth with a constant of order 1), so the first step
    doubles L until it does: the accepted L_1 is L_0/2 times a power of two
    and took that many extra trials."""
    X, Y, a, b = _clouds(4, n=15, m=11)
    K = oracle.gaussian_kernel(X, Y, 1.0)
    L0 = 1e-6
    res = _acc(K, a, b, fixed_iter=1, L0=L0)
    p = math.log2(res.Ls[0] / (L0 / 2))
    assert p == int(p) and p >= 1
    assert res.trials == int(p) + 1
