"""Accelerated Sinkhorn (the acceleration remark of Sec. 3.1 and the
accelerated algorithm of the appendix): pins of the oracle against facts
that do not come from its own code, and (GPU) parity of the device solver
with it."""
import math

import numpy as np
import pytest

import oracle
from paper_2006_07057_amd import inputs
from parity import check_divergence, check_gradient, check_value

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


# --------------------------------------------------------------- C ABI
def test_acc_argument_errors():
    """Argument checks happen on the host before anything is enqueued."""
    import ctypes
    from paper_2006_07057_amd import _lib
    L = _lib.lib()
    P = 0x1000
    spec = _lib.sk_solve_spec(P, P, P, P, 0, 0, P, P, P, P, P, 10, 12, 8, 1.0)
    lin = _lib.sk_solve_opts(1e-6, 100, 0, 0, _lib.SK_RANGE_LINEAR)
    ext = _lib.sk_solve_opts(1e-6, 100, 0, 0, _lib.SK_RANGE_EXTENDED)
    warm = _lib.sk_solve_opts(1e-6, 100, 0, 1, _lib.SK_RANGE_LINEAR)
    f = L.sinkhorn_solve_accelerated
    ws = ctypes.c_void_p(P)
    assert f(ctypes.byref(spec), ctypes.byref(lin), 0.0, None, ws, 1 << 30, None) == _lib.SK_EINVAL
    assert f(ctypes.byref(spec), ctypes.byref(lin), float("inf"), None, ws, 1 << 30,
             None) == _lib.SK_EINVAL
    assert f(ctypes.byref(spec), ctypes.byref(ext), 1.0, None, ws, 1 << 30, None) == _lib.SK_ENOTSUP
    assert f(ctypes.byref(spec), ctypes.byref(warm), 1.0, None, ws, 1 << 30, None) == _lib.SK_ENOTSUP
    assert f(ctypes.byref(spec), ctypes.byref(lin), 1.0, None, ws, 16, None) == _lib.SK_ENOMEM
    assert f(ctypes.byref(spec), ctypes.byref(lin), 1.0, None, None, 1 << 30, None) == _lib.SK_EINVAL
    empty = _lib.sk_solve_spec(P, P, P, P, 0, 0, P, P, P, P, P, 0, 12, 8, 1.0)
    assert f(ctypes.byref(empty), ctypes.byref(lin), 1.0, None, ws, 1 << 30, None) == _lib.SK_EINVAL
    assert L.sinkhorn_solve_accelerated_workspace_size(ctypes.byref(empty)) == 0
    bad_r = _lib.sk_solve_spec(P, P, P, P, 0, 0, P, P, P, P, P, 10, 12, 6, 1.0)
    assert f(ctypes.byref(bad_r), ctypes.byref(lin), 1.0, None, ws, 1 << 30, None) == _lib.SK_ENOTSUP
    assert L.sinkhorn_solve_accelerated_workspace_size(ctypes.byref(bad_r)) == 0
    assert L.sinkhorn_solve_accelerated_workspace_size(ctypes.byref(spec)) > 0


# ---------------------------------------------------------- GPU parity
def _gpu_api():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2006_07057_amd import api as A
    A.lib()
    return A


def _features(n, m, r, seed, eps=0.5):
    """Row-normalised positive features of two Gaussian clouds (float32,
    linear layout) and the float64 values the oracle sees."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, 2))
    Y = rng.standard_normal((m, 2)) + 1.0
    U = rng.standard_normal((r, 2))
    Ex = oracle.gaussian_log_features(X, U, eps, 8.0)
    Ey = oracle.gaussian_log_features(Y, U, eps, 8.0)
    Fx = np.exp(Ex - Ex.max(1)[:, None]).astype(np.float32)
    Fy = np.exp(Ey - Ey.max(1)[:, None]).astype(np.float32)
    a = inputs.dirichlet_weights(rng, n)
    b = inputs.dirichlet_weights(rng, m)
    return Fx, Fy, a, b


def _run_solve(A, Fx, Fy, a, b, **kw):
    import torch
    d = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    n, r = Fx.shape
    m = Fy.shape[0]
    t = dict(Prow=d(Fx), Pcol=d(Fy), a=d(a), b=d(b),
             u=torch.zeros(2 * n, dtype=torch.float32, device="cuda"),
             v=torch.zeros(2 * m, dtype=torch.float32, device="cuda"),
             w=torch.zeros(2 * r, dtype=torch.float32, device="cuda"),
             z=torch.zeros(2 * r, dtype=torch.float32, device="cuda"),
             info=torch.zeros(A.INFO_BYTES, dtype=torch.uint8, device="cuda"),
             trials=torch.zeros(1, dtype=torch.int32, device="cuda"))
    spec = A.solve_spec(t["Prow"], t["Pcol"], t["a"], t["b"], t["u"], t["v"], t["w"],
                        t["z"], t["info"], eps=1.0)
    A.solve_accelerated(spec, trials=t["trials"], **kw)
    torch.cuda.synchronize()
    info = A.parse_infos(t["info"])[0]
    out = {k: t[k].cpu().numpy().astype(np.float64) for k in ("u", "v", "w", "z")}
    out["u"], out["v"] = out["u"][:n], out["v"][:m]
    out["w"], out["z"] = out["w"][:r], out["z"][:r]
    return out, info, int(t["trials"].cpu()[0])


def _gauge_free(lu, lv):
    """(log u_i - log u_0, log u_0 + log v_j): the plan diag(u) K diag(v)
    is invariant under u -> u t, v -> v / t."""
    return lu - lu[0], lu[0] + lv


@pytest.mark.gpu
@pytest.mark.parametrize("n,m,r,steps", [(300, 257, 128, 1), (300, 257, 128, 12),
                                         (1000, 1400, 64, 40), (2500, 1900, 1024, 25),
                                         (3, 2, 4, 6), (20000, 15000, 512, 8)])
def test_acc_fixed_steps_match_oracle(n, m, r, steps):
    """A fixed number of accepted steps from eta = zeta = 0: the same step
    count, blocks and line-search path as the float64 oracle (gradient
    evaluations agree), the same dual point up to the plan's gauge, the
    r-vectors of the returned scalings and the dual value."""
    A = _gpu_api()
    Fx, Fy, a, b = _features(n, m, r, seed=n + r)
    res, info, trials = _run_solve(A, Fx, Fy, a, b, fixed_iter=steps)
    Px, Py = Fx.astype(np.float64), Fy.astype(np.float64)
    ref = oracle.accelerated_sinkhorn(lambda v: Px @ (Py.T @ v), lambda u: Py @ (Px.T @ u),
                                      a, b, fixed_iter=steps)
    assert info["status"] == 0 and info["iters"] == steps
    assert trials == ref.trials
    lu, lv = np.log(res["u"]), np.log(res["v"])
    gu, gv = _gauge_free(lu, lv)
    ru, rv = _gauge_free(ref.eta1, ref.eta2)
    np.testing.assert_allclose(gu, ru, rtol=0, atol=5e-4)
    np.testing.assert_allclose(gv, rv, rtol=0, atol=5e-4)
    np.testing.assert_allclose(res["w"], Py.T @ res["v"], rtol=2e-5, atol=1e-30)
    np.testing.assert_allclose(res["z"], Px.T @ res["u"], rtol=2e-5, atol=1e-30)
    K = Px @ Py.T if n * m <= 4_000_000 else None
    if K is not None:
        F = oracle.dual_value(ref.eta1, ref.eta2, K, a, b, 1.0)
        check_value(f"accelerated fixed-step dual value {n}x{m}", info["w_hat"], F)


@pytest.mark.gpu
@pytest.mark.parametrize("n,m,r", [(800, 700, 128), (2000, 1500, 256), (1500, 1500, 1024)])
def test_acc_tolerance_mode_reaches_optimum(n, m, r):
    """Stopping at a momentum point whose gradient has L1 norm < tol: the
    returned pair's marginals are within a few tol of (a, b) and its dual
    value equals the float64 optimum (Algorithm 1 run to 1e-10) within
    1e-5."""
    A = _gpu_api()
    Fx, Fy, a, b = _features(n, m, r, seed=7 * n + r)
    res, info, trials = _run_solve(A, Fx, Fy, a, b, tol=1e-6, max_iter=20000)
    Px, Py = Fx.astype(np.float64), Fy.astype(np.float64)
    assert info["status"] == 0, info
    assert trials >= info["iters"] >= 1
    u, v = res["u"], res["v"]
    row = u * (Px @ (Py.T @ v))
    col = v * (Py @ (Px.T @ u))
    err = np.abs(row - a).sum() + np.abs(col - b).sum()
    assert err < 5e-6
    assert info["err"] == pytest.approx(err, rel=0.05, abs=2e-7)
    K = Px @ Py.T
    sk = oracle.sinkhorn_dense(K, a, b, tol=1e-10, max_iter=200000)
    W = oracle.w_hat(sk.u, sk.v, a, b, 1.0)
    assert info["w_hat"] == pytest.approx(W, rel=1e-5)


@pytest.mark.gpu
@pytest.mark.parametrize("n,m,r", [(1, 1, 4), (1, 7, 8), (9, 1, 4), (2, 3, 4096),
                                   (700, 500, 4096)])
def test_acc_degenerate_and_largest_shapes(n, m, r):
    """Single-point clouds (one marginal is exact from the first block
    step) and the largest feature count (r = 4096): fixed steps against
    the oracle, and tolerance mode reaching the float64 optimum."""
    A = _gpu_api()
    Fx, Fy, a, b = _features(n, m, r, seed=3 * n + m + r)
    Px, Py = Fx.astype(np.float64), Fy.astype(np.float64)
    ref = oracle.accelerated_sinkhorn(lambda v: Px @ (Py.T @ v), lambda u: Py @ (Px.T @ u),
                                      a, b, fixed_iter=6)
    res, info, trials = _run_solve(A, Fx, Fy, a, b, fixed_iter=6)
    assert info["status"] == 0 and info["iters"] == 6
    assert trials == ref.trials
    gu, gv = _gauge_free(np.log(res["u"]), np.log(res["v"]))
    ru, rv = _gauge_free(ref.eta1, ref.eta2)
    np.testing.assert_allclose(gu, ru, rtol=0, atol=5e-4)
    np.testing.assert_allclose(gv, rv, rtol=0, atol=5e-4)
    res, info, _ = _run_solve(A, Fx, Fy, a, b, tol=1e-6, max_iter=20000)
    assert info["status"] == 0, info
    K = Px @ Py.T
    sk = oracle.sinkhorn_dense(K, a, b, tol=1e-10, max_iter=200000)
    assert info["w_hat"] == pytest.approx(oracle.w_hat(sk.u, sk.v, a, b, 1.0), rel=1e-5)


@pytest.mark.gpu
def test_acc_rank_one_kernel():
    """The rank-one degenerate case (every row of the features equal up to
    scale, r = 4 identical columns): the optimum is the product coupling, of
    dual value sum a log(a / x) + sum b log(b / y) for K = x y^T."""
    A = _gpu_api()
    rng = np.random.default_rng(17)
    n, m, r = 300, 200, 4
    x = rng.uniform(0.2, 1.0, n).astype(np.float32)
    y = rng.uniform(0.2, 1.0, m).astype(np.float32)
    Fx = np.repeat(x[:, None], r, axis=1).astype(np.float32)
    Fy = np.repeat(y[:, None], r, axis=1).astype(np.float32)
    a = inputs.dirichlet_weights(rng, n)
    b = inputs.dirichlet_weights(rng, m)
    res, info, _ = _run_solve(A, Fx, Fy, a, b, tol=1e-6, max_iter=5000)
    assert info["status"] == 0
    xs, ys = r * x.astype(np.float64), y.astype(np.float64)     # K = (r x) y^T
    ref = float(a @ np.log(a / xs) + b @ np.log(b / ys))
    assert info["w_hat"] == pytest.approx(ref, rel=1e-5)


def _div_inputs(seed, n, m, d, r, eps):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, d)).astype(np.float32)
    Y = (rng.standard_normal((m, d)) + 0.4).astype(np.float32)
    a = inputs.dirichlet_weights(rng, n)
    b = inputs.dirichlet_weights(rng, m)
    q = oracle.lambert_q(inputs.max_norm(X, Y), eps, d)
    U = inputs.gaussian_anchors(seed + 1, r, d, oracle.sigma2_from_q(q, eps))
    return X, Y, a, b, U, q


@pytest.mark.gpu
@pytest.mark.parametrize("n,m,d,r,eps", [(300, 250, 3, 256, 0.7), (1000, 900, 2, 128, 0.5)])
def test_acc_divergence_matches_converged_oracle(n, m, d, r, eps):
    """The divergence with accelerated solves run to tol = 1e-6 equals the
    converged float64 divergence (Algorithm 1) within 1e-5."""
    import torch
    A = _gpu_api()
    X, Y, a, b, U, q = _div_inputs(n + r, n, m, d, r, eps)
    dv = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    out, st = A.divergence_accelerated(dv(X), dv(Y), dv(a), dv(b), dv(U), eps, q,
                                       tol=1e-6, max_iter=20000)
    g = out.cpu().numpy()
    infos = st.infos()
    assert list(infos["status"]) == [0, 0, 0], infos
    meta = st.meta()
    assert meta[0] == 0 and np.all(meta[1:] >= infos["iters"])   # linear layout
    ref = oracle.divergence_scaled(X, Y, a, b, U, eps, q, tol=1e-11, max_iter=200000)
    check_divergence(f"accelerated tol 1e-6 {n}x{m} d={d} r={r}", g, ref)


@pytest.mark.gpu
@pytest.mark.parametrize("seed,n,m,d,r,eps,steps", [(556, 300, 250, 3, 256, 0.7, 30),
                                                    (1132, 1000, 900, 2, 128, 0.5, 35),
                                                    # a long trajectory (about 120
                                                    # gradient evaluations per solve)
                                                    (32, 300, 260, 2, 128, 1.0, 64)])
def test_acc_divergence_gradients_match_oracle(seed, n, m, d, r, eps, steps):
    """After a fixed number of accepted steps, the three dual points, the
    dual values and the adjoint's gradients (dX, da, dY, db) match the
    oracle's accelerated run pushed through the same gradient formulas
    (values within 1e-5, gradients within 1e-4)."""
    import torch
    A = _gpu_api()
    X, Y, a, b, U, q = _div_inputs(seed, n, m, d, r, eps)
    dv = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    out, st = A.divergence_accelerated(dv(X), dv(Y), dv(a), dv(b), dv(U), eps, q,
                                       fixed_iter=steps)
    g = out.cpu().numpy()
    infos = st.infos()
    assert list(infos["status"]) == [0, 0, 0] and list(infos["iters"]) == [steps] * 3
    rX, ra, rY, rb, vals, runs = oracle.divergence_grad_accelerated(X, Y, a, b, U, eps, q,
                                                                   fixed_iter=steps)
    # The trajectory is unique only where no decision is a near tie: float32
    # row sums move the sufficient-decrease test by about 1e-7 / ||grad||
    # relative and the block choice by about 1e-7.  The symmetric terms
    # W(mu,mu), W(nu,nu) tie exactly at the first block choice; either choice
    # gives the mirror-image trajectory, with the same value and the same
    # (symmetric) gradient contributions.
    for res, symmetric in zip(runs, (False, True, True)):
        ms = res.margins[1:] if symmetric else res.margins
        assert min(ms) > 1e-4, "oracle path has a near tie: pick another case"
        assert min(res.ls_margins) > 1e-2, "oracle path has a near tie: pick another case"
    assert list(st.meta()[1:]) == [rr.trials for rr in runs]
    lab = f"accelerated {steps} steps {n}x{m} d={d} r={r}"
    check_divergence(lab, g, vals)
    dX, da, dY, db = [t.cpu().numpy().astype(np.float64) for t in A.divergence_backward(st)]
    for nm, gg, rr in (("dX", dX, rX), ("da", da, ra), ("dY", dY, rY), ("db", db, rb)):
        check_gradient(f"{lab} {nm}", gg, rr)


@pytest.mark.gpu
def test_acc_full_size_properties():
    """The benchmarked shape (two 4-component mixtures in R^3, n = m = 10^6,
    r = 1024, eps = 0.1 is too far for the float32 linear layout, so the
    2-D Gaussian pair at eps = 0.5 is used at that size): properties that
    hold at any size, checked with plain torch float32 products outside the
    library: status, the returned pair's marginal errors, w = Pcol^T v and
    z = Prow^T u, and a dual value no larger than Algorithm 1's."""
    import torch
    A = _gpu_api()
    n = m = 1_000_000
    c = inputs.gauss2d(5, n=n, m=m)
    eps = 0.5
    s2 = 1.0
    q = oracle.q_from_sigma2(s2, eps)
    U = inputs.gaussian_anchors(5, 1024, 2, s2)
    dv = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    X, Y, a, b, Ud = dv(c.X), dv(c.Y), dv(c.a), dv(c.b), dv(U)
    out, st = A.divergence_accelerated(X, Y, a, b, Ud, eps, q, tol=1e-5, max_iter=3000)
    infos = st.infos()
    assert list(infos["status"]) == [0, 0, 0], infos
    u, v, w, z = st.scalings(0)
    u, v = u[:n], v[:m]
    Px, Py = st.phix, st.phiy
    wz = (Py.t() @ v).double()
    zz = (Px.t() @ u).double()
    torch.testing.assert_close(w[:1024].double(), wz, rtol=1e-4, atol=0)
    torch.testing.assert_close(z[:1024].double(), zz, rtol=1e-4, atol=0)
    row = (u.double() * (Px @ w[:1024]).double() - a.double()).abs().sum().item()
    col = (v.double() * (Py @ z[:1024]).double() - b.double()).abs().sum().item()
    assert row + col < 5e-5
    out2, st2 = A.divergence(X, Y, a, b, Ud, eps, q, tol=1e-5, max_iter=3000,
                             range=A.LINEAR)
    g, g2 = out.cpu().numpy(), out2.cpu().numpy()
    for k in range(1, 4):
        assert g[k] == pytest.approx(g2[k], rel=1e-5)


def test_acc_oracle_gradients_at_convergence():
    """Run far enough, the accelerated dual points give the converged
    divergence and its gradients (divergence_grad, pinned by finite
    differences elsewhere)."""
    rng = np.random.default_rng(21)
    n, m, d, r, eps = 30, 25, 2, 64, 1.0
    X = rng.standard_normal((n, d))
    Y = rng.standard_normal((m, d)) + 0.3
    a = rng.dirichlet(np.full(n, 20.0))   # no near-zero weights: every
    b = rng.dirichlet(np.full(m, 20.0))   # potential is well determined
    q = oracle.lambert_q(float(max(np.linalg.norm(X, axis=1).max(),
                                   np.linalg.norm(Y, axis=1).max())), eps, d)
    U = rng.standard_normal((r, d)) * math.sqrt(oracle.sigma2_from_q(q, eps))
    rX, ra, rY, rb, div = oracle.divergence_grad(X, Y, a, b, U, eps, q)
    gX, ga, gY, gb, vals, runs = oracle.divergence_grad_accelerated(X, Y, a, b, U, eps, q,
                                                                   fixed_iter=600)
    assert max(res.err for res in runs) < 1e-8
    assert vals[0] == pytest.approx(div.value, rel=1e-9, abs=1e-12)
    for gg, rr in ((gX, rX), (ga, ra), (gY, rY), (gb, rb)):
        assert np.linalg.norm(gg - rr) <= 1e-6 * np.linalg.norm(rr)
