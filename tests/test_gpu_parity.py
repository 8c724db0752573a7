"""GPU parity tests: the HIP library (through the C ABI) against the FP64
oracle on the same seeded float32 inputs.

Tolerances: divergences within 1e-5 relative, gradients within 1e-4
relative (L2), features within a bound derived from float32 rounding of
the exponent (see _feature_tol).  Both numeric domains of the solver are
exercised: the extended range (default) and plain float32 (LINEAR).
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2006_07057_amd import inputs
from parity import DIV_RTOL, GRAD_RTOL, check_divergence, check_gradient, check_value

pytestmark = pytest.mark.gpu

EXT, LIN = 0, 1
RANGES = [pytest.param(EXT, id="ext"), pytest.param(LIN, id="lin")]
LOG2E = 1.0 / math.log(2.0)


def _say(*a):
    print("[gpu-test]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2006_07057_amd import api as A
    A.lib()  # fail loudly if the library is missing
    return A


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _feature_tol(X, U, eps, q):
    """Per-row absolute bound on the float32 exponent error.  E_ik is
    formed from a float32 squared distance (d+1 roundings), a float32
    product with 2/eps and a float32 sum with c_k; the error of E_ik - s_i
    is then at most a small multiple of 2^-24 times the magnitudes
    involved."""
    X = np.asarray(X, np.float64)
    U = np.asarray(U, np.float64)
    d = X.shape[1]
    d2 = ((X[:, None, :] - U[None, :, :]) ** 2).sum(-1)
    E = oracle.gaussian_log_features(X, U, eps, q)
    c = np.abs(E + (2.0 / eps) * d2)
    mag = (2.0 / eps) * d2 * (d + 3) + c + np.abs(E)
    if d >= 32 and d % 4 == 0:
        # matrix-core path: E - s is formed from c_k + (4/eps) x.u with the
        # dot product accumulated over d float32 terms, and s adds the
        # float32 product (2/eps)||x||^2
        dot = np.abs(X) @ np.abs(U).T
        xn = (X ** 2).sum(1)[:, None]
        un = (U ** 2).sum(1)[None, :]
        mag = mag + (4.0 / eps) * dot * (d + 3) + (2.0 / eps) * (xn + un) + np.abs(c)
    return 8 * 2.0 ** -24 * (mag.max(1) + 1.0)


@pytest.mark.parametrize("rng_mode", RANGES)
@pytest.mark.parametrize("n,d,r,eps,q", [
    (1000, 2, 128, 0.5, 8.0),        # the small 2-D workload
    (1037, 3, 1024, 0.1, 9.17),      # mixture-like shape, ragged n
    (333, 1, 4, 1.0, 1.0),           # tiny r, 64 rows per wave load
    (257, 16, 100, 0.5, 2.0),        # r not a power of two
    (130, 3, 37, 0.7, 3.0),          # r % 4 != 0 (scalar path)
    (200, 64, 256, 5.0, 0.7),        # d = 64, anchors staged in LDS
    (150, 128, 2048, 1.0, 0.504),    # d = 128, anchors read from memory
    (64, 2, 4096, 0.5, 8.0),         # largest r
])
def test_features_match_oracle(api, n, d, r, eps, q, rng_mode):
    _say("features", n, d, r, eps, rng_mode)
    rng = np.random.default_rng(n + d + r)
    X = rng.standard_normal((n, d)).astype(np.float32)
    U = (math.sqrt(oracle.sigma2_from_q(q, eps)) *
         rng.standard_normal((r, d))).astype(np.float32)
    Phi, s = api.features(dev(X), dev(U), eps, q, range=rng_mode)
    torch.cuda.synchronize()
    Pg, sg = host(Phi), host(s)
    E = oracle.gaussian_log_features(X, U, eps, q)
    so = E.max(1)
    tol = _feature_tol(X, U, eps, q)
    assert np.all(np.abs(sg - so) <= tol), np.max(np.abs(sg - so) / tol)
    if rng_mode == EXT:
        Lo = (E - so[:, None]) * LOG2E
        err = np.abs(Pg - Lo)
        assert np.all(err <= 2 * LOG2E * tol[:, None] + 4e-7 * np.abs(Lo)), err.max()
        assert np.all(Pg <= 0.0)
    else:
        Po = np.exp(E - so[:, None])
        big = Po > 1e-30
        rel = np.abs(Pg - Po) / np.where(big, Po, 1.0)
        assert np.all(rel[big] <= 2 * np.broadcast_to(tol[:, None], Po.shape)[big] + 4e-7)
        assert np.all(np.abs(Pg - Po)[~big] <= 1e-30)
        assert np.all(Pg <= 1.0) and np.all(Pg >= 0.0)


@pytest.mark.parametrize("rng_mode", RANGES)
@pytest.mark.parametrize("n,m,r,iters", [(1000, 1000, 128, 50), (777, 1203, 64, 30),
                                         (5000, 3000, 256, 20), (40000, 30000, 512, 10),
                                         (3, 2, 4, 5)])
def test_solve_matches_oracle_fixed_iterations(api, n, m, r, iters, rng_mode):
    """Algorithm 1 from u = 1 for a fixed number of iterations on features
    produced by the oracle (rounded to float32; log2 features for the
    extended range): scalings, r-vectors, iteration count and error."""
    _say("solve", n, m, r, iters, rng_mode)
    rng = np.random.default_rng(n + m)
    X = rng.standard_normal((n, 2))
    Y = rng.standard_normal((m, 2)) + 1.0
    U = rng.standard_normal((r, 2))
    Ex = oracle.gaussian_log_features(X, U, 0.5, 8.0)
    Ey = oracle.gaussian_log_features(Y, U, 0.5, 8.0)
    Lx = Ex - Ex.max(1)[:, None]
    Ly = Ey - Ey.max(1)[:, None]
    if rng_mode == EXT:
        Gx, Gy = (Lx * LOG2E).astype(np.float32), (Ly * LOG2E).astype(np.float32)
        Px = np.exp2(Gx.astype(np.float64))
        Py = np.exp2(Gy.astype(np.float64))
    else:
        Gx, Gy = np.exp(Lx).astype(np.float32), np.exp(Ly).astype(np.float32)
        Px, Py = Gx.astype(np.float64), Gy.astype(np.float64)
    a = inputs.dirichlet_weights(rng, n)
    b = inputs.dirichlet_weights(rng, m)
    res = api.solve(dev(Gx), dev(Gy), dev(a), dev(b), fixed_iter=iters,
                    range=rng_mode)
    info = res.info()
    ref = oracle.sinkhorn_factored(Px, Py, a, b, fixed_iter=iters)
    assert info["status"] == 0 and info["iters"] == iters
    lu = api.host_log_scaling(res.u, rng_mode)
    lv = api.host_log_scaling(res.v, rng_mode)
    np.testing.assert_allclose(lu, np.log(ref.u), rtol=0, atol=2e-4)
    np.testing.assert_allclose(lv, np.log(ref.v), rtol=0, atol=2e-4)
    lw = api.host_log_scaling(res.w, rng_mode)
    lz = api.host_log_scaling(res.z, rng_mode)
    np.testing.assert_allclose(lw, np.log(Py.T @ ref.v), rtol=0, atol=2e-4)
    np.testing.assert_allclose(lz, np.log(Px.T @ ref.u), rtol=0, atol=2e-4)
    wo = oracle.w_hat(ref.u, ref.v, a, b, 1.0)
    check_value(f"solve w_hat {n}x{m} r={r} it={iters} range={rng_mode}", info["w_hat"], wo)
    assert info["err"] == pytest.approx(ref.err, rel=0.05, abs=2e-6)


def _divergence_inputs(kind, seed=0, **kw):
    if kind == "gauss2d":
        c = inputs.gauss2d(seed, **kw)
        eps, s2, r = 0.5, 1.0, 128
        q = oracle.q_from_sigma2(s2, eps)
    elif kind == "gmm3d":
        c = inputs.gmm3d(seed, **kw)
        eps, r = 0.1, 1024
        q = oracle.lambert_q(inputs.max_norm(c.X, c.Y), eps, 3)
        s2 = oracle.sigma2_from_q(q, eps)
    else:
        raise ValueError(kind)
    U = inputs.gaussian_anchors(seed, r, c.X.shape[1], s2)
    return c, U, eps, q


@pytest.mark.parametrize("rng_mode", RANGES)
def test_divergence_small_gaussians_200_iterations(api, rng_mode):
    """The 2-D Gaussian workload: n = m = 1000, r = 128, sigma^2 = 1,
    200 fixed iterations; GPU float32 vs oracle float64 (dense K_theta)."""
    _say("divergence gauss2d 200 fixed", rng_mode)
    c, U, eps, q = _divergence_inputs("gauss2d")
    out, st = api.divergence(dev(c.X), dev(c.Y), dev(c.a), dev(c.b), dev(U),
                             eps, q, fixed_iter=200, range=rng_mode)
    g = host(out)
    ref = oracle.divergence(c.X, c.Y, c.a, c.b, U, eps, q, fixed_iter=200)
    check_divergence(f"gauss2d 200 fixed range={rng_mode}", g, ref)
    infos = st.infos()
    assert list(infos["iters"]) == [200, 200, 200]
    assert list(infos["status"]) == [0, 0, 0]


@pytest.mark.parametrize("rng_mode", RANGES)
def test_divergence_tolerance_mode(api, rng_mode):
    """Stop test of Algorithm 1 at tol = 1e-6: both sides converge and agree
    within 1e-5; the reported error is below the tolerance and the
    iteration counts agree to a few iterations (float32 vs float64 may
    cross the threshold at slightly different iterations)."""
    _say("divergence gauss2d tol", rng_mode)
    c, U, eps, q = _divergence_inputs("gauss2d")
    out, st = api.divergence(dev(c.X), dev(c.Y), dev(c.a), dev(c.b), dev(U),
                             eps, q, tol=1e-6, max_iter=5000, range=rng_mode)
    g = host(out)
    ref = oracle.divergence(c.X, c.Y, c.a, c.b, U, eps, q, tol=1e-6, max_iter=5000)
    infos = st.infos()
    assert list(infos["status"]) == [0, 0, 0]
    assert np.all(infos["err"] < 1e-6)
    for k, rr in enumerate((ref.xy, ref.xx, ref.yy)):
        assert abs(int(infos["iters"][k]) - rr.iters) <= max(3, rr.iters // 20)
    check_divergence(f"gauss2d tol 1e-6 range={rng_mode}", g, ref)


def test_separated_mixtures_extended_range_converges(api):
    """Two 4-component mixtures in R^3 at eps = 0.1 (clusters far apart, the
    mixture workload at n = m = 3000): the extended range converges to the
    float64 oracle's divergence within 1e-5 at tol = 1e-6."""
    _say("separated mixtures")
    c, U, eps, q = _divergence_inputs("gmm3d", seed=0, n=3000, m=3000)
    args = (dev(c.X), dev(c.Y), dev(c.a), dev(c.b), dev(U), eps, q)
    out, st = api.divergence(*args, tol=1e-6, max_iter=3000, range=EXT)
    infos = st.infos()
    assert list(infos["status"]) == [0, 0, 0], infos
    ref = oracle.divergence_scaled(c.X, c.Y, c.a, c.b, U, eps, q, tol=1e-6,
                                   max_iter=3000, dense=False)
    g = host(out)
    _say("iters", infos["iters"], ref.xy.iters, ref.xx.iters, ref.yy.iters)
    check_divergence("separated mixtures 3000 tol 1e-6", g, ref)


def _marginal_checks(c, U, eps, q, st, rows, tol):
    """Properties of the converged (x, y) solve that hold at any size,
    checked in float64 on the host with features recomputed by the oracle
    (independently of the GPU's features) on sampled points:
      * row marginal (exact after the u-update of Algorithm 1):
        u_i sum_k phi_k(x_i) w_k = a_i,
      * column marginal of the returned pair within the stop tolerance:
        v_j sum_k phi_k(y_j) z_k ~ b_j,
    with (u, v, w, z) the GPU's scalings and r-vectors.  The tolerance
    covers float32 feature rounding of exponents of a few hundred."""
    lu, lv = st.log_scalings(0)
    _, _, w, z = st.scalings(0)
    lw = api_host_log(w, st.range)
    lz = api_host_log(z, st.range)
    rng = np.random.default_rng(7)
    ii = rng.choice(len(c.a), size=min(rows, len(c.a)), replace=False)
    jj = rng.choice(len(c.b), size=min(rows, len(c.b)), replace=False)
    sx = st.sx.cpu().numpy().astype(np.float64)
    sy = st.sy.cpu().numpy().astype(np.float64)
    Ex = oracle.gaussian_log_features(c.X[ii], U, eps, q)
    Ey = oracle.gaussian_log_features(c.Y[jj], U, eps, q)
    # log of u_i phi_k(x_i) w_k with the GPU's scaled u (u = u~ e^{-s})
    row = np.exp(lu[ii, None] - sx[ii, None] + Ex + lw[None, :]).sum(1)
    np.testing.assert_allclose(row, c.a[ii].astype(np.float64), rtol=1e-3)
    col = np.exp(lv[jj, None] - sy[jj, None] + Ey + lz[None, :]).sum(1)
    np.testing.assert_allclose(col, c.b[jj].astype(np.float64), rtol=1e-3)


def api_host_log(t, range_):
    from paper_2006_07057_amd import api as A
    return A.host_log_scaling(t, range_)


def test_linear_overflow_detected_extended_converges(api):
    """Mixture workload at n = m = 20000: the float32 scalings of the
    (x, y) problem overflow, which the linear domain reports as SK_ERANGE
    (no silent NaN); the extended range converges and its solution passes
    float64 marginal checks on sampled points."""
    _say("linear overflow vs extended range")
    c, U, eps, q = _divergence_inputs("gmm3d", seed=0, n=20000, m=20000)
    args = (dev(c.X), dev(c.Y), dev(c.a), dev(c.b), dev(U), eps, q)
    _, st_lin = api.divergence(*args, tol=1e-6, max_iter=3000, range=LIN)
    assert st_lin.infos()["status"][0] == 3
    out, st = api.divergence(*args, tol=1e-6, max_iter=3000, range=EXT)
    infos = st.infos()
    assert list(infos["status"]) == [0, 0, 0], infos
    assert np.all(infos["err"] < 1e-6)
    _marginal_checks(c, U, eps, q, st, 500, 1e-6)


def test_full_size_mixture_properties(api):
    """The benchmark configuration itself (n = m = 10^6 points in R^3,
    r = 1024, eps = 0.1, tol 1e-6, at most 2000 iterations, extended range,
    the same entry point and launch as the benchmark): every solve ends
    with status OK or SK_ENOTCONV, the reported error of converged solves
    is below the tolerance, the divergence is the float64 combination of
    the three dual estimates, features of sampled rows match the oracle,
    and the (x, y) solution passes float64 marginal checks on sampled
    points."""
    _say("full-size mixture workload")
    c, U, eps, q = _divergence_inputs("gmm3d", seed=0)
    args = (dev(c.X), dev(c.Y), dev(c.a), dev(c.b), dev(U), eps, q)
    out, st = api.divergence(*args, tol=1e-6, max_iter=2000, range=EXT)
    infos = st.infos()
    g = host(out)
    _say("infos", infos, "W_bar", g[0])
    assert set(int(s) for s in infos["status"]) <= {0, 4}
    for k in range(3):
        if infos["status"][k] == 0:
            assert infos["err"][k] < 1e-6
    assert g[0] == pytest.approx(g[1] - 0.5 * (g[2] + g[3]), rel=1e-12)
    # features of sampled rows against the oracle
    rng = np.random.default_rng(3)
    ii = rng.choice(len(c.a), size=256, replace=False)
    E = oracle.gaussian_log_features(c.X[ii], U, eps, q)
    so = E.max(1)
    sg = st.sx.cpu().numpy().astype(np.float64)[ii]
    tol = _feature_tol(c.X[ii], U, eps, q)
    assert np.all(np.abs(sg - so) <= tol)
    Lg = st.phix[torch.from_numpy(ii).cuda()].cpu().numpy().astype(np.float64)
    Lo = (E - so[:, None]) * LOG2E
    assert np.all(np.abs(Lg - Lo) <= 2 * LOG2E * tol[:, None] + 4e-7 * np.abs(Lo))
    if infos["status"][0] == 0:
        _marginal_checks(c, U, eps, q, st, 300, 1e-6)


@pytest.mark.parametrize("rng_mode", RANGES)
@pytest.mark.parametrize("n,m,d,r,eps", [
    (1037, 555, 3, 100, 0.5), (90, 140, 1, 4, 1.0), (2000, 1500, 16, 512, 2.0),
    (513, 511, 2, 1024, 0.3), (300, 200, 5, 2048, 1.0), (120, 130, 2, 4096, 0.5),
    (64, 64, 2, 12, 0.5), (1, 1, 2, 8, 1.0),
])
def test_divergence_shapes(api, n, m, d, r, eps, rng_mode):
    """Ragged sizes across every solver class (30 fixed iterations)."""
    _say("divergence shapes", n, m, d, r, eps, rng_mode)
    rng = np.random.default_rng(n * 7 + m)
    X = rng.standard_normal((n, d)).astype(np.float32)
    Y = (rng.standard_normal((m, d)) + 0.5).astype(np.float32)
    a = inputs.dirichlet_weights(rng, n)
    b = inputs.dirichlet_weights(rng, m)
    q = oracle.lambert_q(inputs.max_norm(X, Y), eps, d)
    U = inputs.gaussian_anchors(n + m, r, d, oracle.sigma2_from_q(q, eps))
    out, st = api.divergence(dev(X), dev(Y), dev(a), dev(b), dev(U), eps, q,
                             fixed_iter=30, range=rng_mode)
    g = host(out)
    ref = oracle.divergence_scaled(X, Y, a, b, U, eps, q, fixed_iter=30)
    check_divergence(f"shapes {n}x{m} d={d} r={r} eps={eps} range={rng_mode}", g, ref)


@pytest.mark.parametrize("rng_mode", RANGES)
def test_divergence_multi_workgroup_groups(api, rng_mode):
    """Large enough that every solve spans many workgroups (group barriers
    and the cross-workgroup reduction are exercised), compared with the
    factored oracle at fixed iterations."""
    _say("divergence multi-workgroup", rng_mode)
    c, U, eps, q = _divergence_inputs("gmm3d", seed=3, n=60000, m=50000)
    out, st = api.divergence(dev(c.X), dev(c.Y), dev(c.a), dev(c.b), dev(U),
                             eps, q, fixed_iter=8, range=rng_mode)
    g = host(out)
    ref = oracle.divergence_scaled(c.X, c.Y, c.a, c.b, U, eps, q, fixed_iter=8,
                                   dense=False)
    check_divergence(f"multi-workgroup 60000x50000 range={rng_mode}", g, ref)


@pytest.mark.parametrize("n,m,d,r,eps,kind", [
    (300, 260, 784, 512, 10.0, "pixels"),    # pixel-like, matrix-core features
    (400, 400, 128, 256, 1.0, "sphere"),     # unit-normalised Gaussian vectors
])
def test_large_d_divergence_matches_oracle(api, n, m, d, r, eps, kind):
    """End to end through the matrix-core feature path (d >= 32)."""
    _say("large-d divergence", kind, n, m, d, r)
    if kind == "pixels":
        c = inputs.pixels(3, n=n, m=m, d=d)
    else:
        c = inputs.sphere(3, n=n, m=m, d=d)
    q = oracle.lambert_q(inputs.max_norm(c.X, c.Y), eps, d)
    U = inputs.gaussian_anchors(3, r, d, oracle.sigma2_from_q(q, eps))
    out, st = api.divergence(dev(c.X), dev(c.Y), dev(c.a), dev(c.b), dev(U), eps, q,
                             fixed_iter=100)
    ref = oracle.divergence_scaled(c.X, c.Y, c.a, c.b, U, eps, q, fixed_iter=100)
    check_divergence(f"large-d {kind} {n}x{m} d={d} r={r}", host(out), ref)


@pytest.mark.parametrize("rng_mode", RANGES)
def test_batched_equals_single(api, rng_mode):
    """Several uneven problems in one batched call give the results of each
    problem alone.  A launch that packs more than three solves sizes their
    workgroup gangs by work share, so each solve's rows are split over a
    different number of workgroups than alone: equal up to float32 rounding
    of the partial sums (and of the stop test near the tolerance)."""
    _say("batched vs single", rng_mode)
    probs = []
    rng = np.random.default_rng(5)
    for (n, m, d, r, eps) in [(1000, 800, 2, 128, 0.5), (5000, 7000, 3, 256, 0.2),
                              (300, 300, 16, 64, 1.0), (20000, 15000, 3, 1024, 0.1),
                              (100, 4000, 2, 128, 0.5)]:
        X = rng.standard_normal((n, d)).astype(np.float32)
        Y = (rng.standard_normal((m, d)) + 0.3).astype(np.float32)
        a = inputs.dirichlet_weights(rng, n)
        b = inputs.dirichlet_weights(rng, m)
        q = oracle.lambert_q(inputs.max_norm(X, Y), eps, d)
        U = inputs.gaussian_anchors(n, r, d, oracle.sigma2_from_q(q, eps))
        probs.append((dev(X), dev(Y), dev(a), dev(b), dev(U), eps, q))
    outb, sts = api.divergence_batched(probs, tol=1e-6, max_iter=3000,
                                       range=rng_mode)
    ob = host(outb)
    for i, P in enumerate(probs):
        o1, s1 = api.divergence(*P, tol=1e-6, max_iter=3000, range=rng_mode)
        o1 = host(o1)
        np.testing.assert_allclose(ob[i], o1, rtol=1e-6, atol=1e-9)
        for ib, i1 in zip(sts[i].infos()["iters"], s1.infos()["iters"]):
            assert abs(int(ib) - int(i1)) <= max(3, 0.05 * int(i1)), (i, ib, i1)


@pytest.mark.parametrize("rng_mode", RANGES)
def test_gradients_match_oracle(api, rng_mode):
    """Adjoint kernels vs the oracle's gradient formula at the same (fixed)
    iteration count."""
    _say("gradients", rng_mode)
    rng = np.random.default_rng(11)
    n, m, d, r, eps = 300, 250, 3, 256, 0.7
    X = rng.standard_normal((n, d)).astype(np.float32)
    Y = (rng.standard_normal((m, d)) + 0.4).astype(np.float32)
    a = inputs.dirichlet_weights(rng, n)
    b = inputs.dirichlet_weights(rng, m)
    q = oracle.lambert_q(inputs.max_norm(X, Y), eps, d)
    U = inputs.gaussian_anchors(1, r, d, oracle.sigma2_from_q(q, eps))
    out, st = api.divergence(dev(X), dev(Y), dev(a), dev(b), dev(U), eps, q,
                             fixed_iter=300, range=rng_mode)
    dX, da, dY, db = [host(t) for t in api.divergence_backward(st)]
    rX, ra, rY, rb, div = oracle.divergence_grad(X, Y, a, b, U, eps, q,
                                                 fixed_iter=300)
    check_divergence(f"gradients d=3 range={rng_mode}", host(out), div)
    for nm, gg, rr in (("dX", dX, rX), ("da", da, ra), ("dY", dY, rY), ("db", db, rb)):
        check_gradient(f"gradients d=3 {nm} range={rng_mode}", gg, rr)


@pytest.mark.parametrize("rng_mode", RANGES)
@pytest.mark.parametrize("n,m,d,r,eps,kind", [
    (300, 250, 36, 100, 1.0, "normal"),     # 2 tiles + 4 coordinates, ragged k chunk
    (129, 383, 8, 64, 0.5, "normal"),       # half of one tile
    (260, 140, 128, 256, 1.0, "sphere"),    # 8 tiles in one workgroup
    (200, 180, 784, 512, 10.0, "pixels"),   # 7 column blocks of 7 tiles
    (130, 150, 6, 4096, 1.0, "normal"),     # per-row kernel, anchors not in LDS
])
def test_gradients_match_oracle_wide_points(api, rng_mode, n, m, d, r, eps, kind):
    """Point and weight gradients for d >= 8 (the matrix-core adjoint) vs
    the oracle's formula on the row-scaled features at the same fixed
    iteration count; row counts leave partial 128-row blocks, r leaves a
    partial 32-feature chunk, d leaves partial 16-coordinate tiles.  d = 6
    (not a multiple of 4) with r = 4096 takes the per-row kernel with the
    anchors read from memory (d r exceeds its LDS staging)."""
    _say("wide gradients", rng_mode, n, m, d, r)
    rng = np.random.default_rng(23 + d)
    if kind == "pixels":
        c = inputs.pixels(31, n=n, m=m, d=d)
        X, Y, a, b = c.X, c.Y, c.a, c.b
    elif kind == "sphere":
        c = inputs.sphere(31, n=n, m=m, d=d)
        X, Y, a, b = c.X, c.Y, c.a, c.b
    else:
        X = (0.4 * rng.standard_normal((n, d))).astype(np.float32)
        Y = (0.4 * rng.standard_normal((m, d)) + 0.1).astype(np.float32)
        a = inputs.dirichlet_weights(rng, n)
        b = inputs.dirichlet_weights(rng, m)
    q = oracle.lambert_q(inputs.max_norm(X, Y), eps, d)
    U = inputs.gaussian_anchors(3, r, d, oracle.sigma2_from_q(q, eps))
    out, st = api.divergence(dev(X), dev(Y), dev(a), dev(b), dev(U), eps, q,
                             fixed_iter=200, range=rng_mode)
    dX, da, dY, db = [host(t) for t in api.divergence_backward(st)]
    rX, ra, rY, rb, div = oracle.divergence_grad_scaled(X, Y, a, b, U, eps, q,
                                                        fixed_iter=200)
    lab = f"wide gradients {kind} d={d} r={r} range={rng_mode}"
    check_divergence(lab, host(out), div)
    for nm, gg, rr in (("dX", dX, rX), ("da", da, ra), ("dY", dY, rY), ("db", db, rb)):
        check_gradient(f"{lab} {nm}", gg, rr)


@pytest.mark.parametrize("rng_mode", RANGES)
def test_point_gradient_accumulates_single_terms(api, rng_mode):
    """The single-term entry point with accumulation, for d >= 8: summing
    the three weighted terms of dW_bar/dX one call at a time gives the
    three-term result of the divergence backward."""
    _say("single-term accumulate", rng_mode)
    rng = np.random.default_rng(41)
    n, m, d, r, eps = 270, 200, 20, 68, 1.0
    X = (0.4 * rng.standard_normal((n, d))).astype(np.float32)
    Y = (0.4 * rng.standard_normal((m, d)) + 0.1).astype(np.float32)
    a = inputs.dirichlet_weights(rng, n)
    b = inputs.dirichlet_weights(rng, m)
    q = oracle.lambert_q(inputs.max_norm(X, Y), eps, d)
    U = inputs.gaussian_anchors(4, r, d, oracle.sigma2_from_q(q, eps))
    Xd, Ud = dev(X), dev(U)
    out, st = api.divergence(Xd, dev(Y), dev(a), dev(b), Ud, eps, q, fixed_iter=150,
                             range=rng_mode)
    dX3 = host(api.divergence_backward(st, need=(True, False, False, False))[0])
    u0, _, w0, _ = st.scalings(0)
    u1, v1, w1, z1 = st.scalings(1)
    acc = None
    for p, g, cf in ((u0, w0, 1.0), (u1, w1, -0.5), (v1, z1, -0.5)):
        acc = api.features_backward(Xd, Ud, st.phix, p, g, coef=cf, dX=acc,
                                    accumulate=acc is not None, range=st.range)
    got = host(acc)
    assert np.linalg.norm(got - dX3) <= 1e-5 * np.linalg.norm(dX3)


@pytest.mark.parametrize("rng_mode", RANGES)
@pytest.mark.parametrize("n,m,d,r,eps", [(300, 250, 3, 256, 0.7), (500, 420, 2, 64, 0.5),
                                         (260, 300, 16, 100, 1.0)])
def test_anchor_gradients_match_oracle(api, rng_mode, n, m, d, r, eps):
    """Anchor gradient (q fixed) vs the oracle's closed form at the same
    fixed iteration count; r = 100 leaves part of a column sweep empty,
    d = 16 takes several coordinate chunks."""
    _say("anchor gradients", rng_mode, n, m, d, r)
    rng = np.random.default_rng(17 + d)
    X = rng.standard_normal((n, d)).astype(np.float32)
    Y = (rng.standard_normal((m, d)) + 0.4).astype(np.float32)
    a = inputs.dirichlet_weights(rng, n)
    b = inputs.dirichlet_weights(rng, m)
    q = oracle.lambert_q(inputs.max_norm(X, Y), eps, d)
    U = inputs.gaussian_anchors(2, r, d, oracle.sigma2_from_q(q, eps))
    out, st = api.divergence(dev(X), dev(Y), dev(a), dev(b), dev(U), eps, q,
                             fixed_iter=300, range=rng_mode)
    dU = host(api.divergence_backward_anchors(st))
    rU, div = oracle.divergence_grad_anchors(X, Y, a, b, U, eps, q, fixed_iter=300)
    lab = f"anchor gradients d={d} r={r} range={rng_mode}"
    check_divergence(lab, host(out), div)
    check_gradient(lab + " dU", dU, rU)


@pytest.mark.parametrize("rng_mode", RANGES)
@pytest.mark.parametrize("n,m,d,r,eps", [
    (300, 250, 36, 132, 1.0),      # partial anchor block and coordinate tile
    (4100, 3100, 12, 64, 1.0),     # twelve row slices, ragged rows
    (260, 140, 128, 256, 0.5),     # 8 coordinate tiles, two anchor blocks
    (150, 170, 200, 68, 2.0),      # 13 tiles: 2 column blocks of 7
])
def test_anchor_gradients_wide_points(api, rng_mode, n, m, d, r, eps):
    """Anchor gradient for d >= 8 (the matrix-core product H^T Z over row
    slices) vs the oracle's closed form at the same fixed iteration count."""
    _say("wide anchor gradients", rng_mode, n, m, d, r)
    rng = np.random.default_rng(29 + d)
    X = (0.4 * rng.standard_normal((n, d))).astype(np.float32)
    Y = (0.4 * rng.standard_normal((m, d)) + 0.1).astype(np.float32)
    a = inputs.dirichlet_weights(rng, n)
    b = inputs.dirichlet_weights(rng, m)
    q = oracle.lambert_q(inputs.max_norm(X, Y), eps, d)
    U = inputs.gaussian_anchors(5, r, d, oracle.sigma2_from_q(q, eps))
    out, st = api.divergence(dev(X), dev(Y), dev(a), dev(b), dev(U), eps, q,
                             fixed_iter=150, range=rng_mode)
    dU = host(api.divergence_backward_anchors(st))
    rU, div = oracle.divergence_grad_anchors(X, Y, a, b, U, eps, q, fixed_iter=150)
    lab = f"wide anchor gradients d={d} r={r} range={rng_mode}"
    check_divergence(lab, host(out), div)
    check_gradient(lab + " dU", dU, rU)


def test_anchor_gradient_autograd(api):
    _say("anchor autograd")
    c, U, eps, q = _divergence_inputs("gauss2d", n=300, m=280)
    Ud = dev(U).requires_grad_(True)
    W = api.sinkhorn_divergence(dev(c.X), dev(c.Y), dev(c.a), dev(c.b), Ud, eps, q,
                                fixed_iter=120)
    (2.0 * W).backward()
    rU, div = oracle.divergence_grad_anchors(c.X, c.Y, c.a, c.b, U, eps, q, fixed_iter=120)
    gU = host(Ud.grad)
    check_gradient("anchor autograd dU", gU, 2 * rU)


@pytest.mark.parametrize("rng_mode", RANGES)
def test_autograd_function(api, rng_mode):
    """torch.autograd.Function wrapper: backward through the adjoint kernels,
    scaled by the incoming gradient."""
    _say("autograd", rng_mode)
    c, U, eps, q = _divergence_inputs("gauss2d", n=400, m=300)
    X = dev(c.X).requires_grad_(True)
    a = dev(c.a).requires_grad_(True)
    W = api.sinkhorn_divergence(X, dev(c.Y), a, dev(c.b), dev(U), eps, q,
                                fixed_iter=100, range=rng_mode)
    (3.0 * W).backward()
    rX, ra, _, _, div = oracle.divergence_grad(c.X, c.Y, c.a, c.b, U, eps, q,
                                               fixed_iter=100)
    check_divergence(f"autograd range={rng_mode}", [W.item()], div, terms=False)
    check_gradient(f"autograd dX range={rng_mode}", host(X.grad), 3 * rX)
    check_gradient(f"autograd da range={rng_mode}", host(a.grad), 3 * ra)


@pytest.mark.parametrize("rng_mode", RANGES)
def test_status_codes(api, rng_mode):
    """Weights outside the simplex (Sec. 2: positive entries summing to 1)
    end the affected solves with SK_EINVAL before any iteration, checked in
    float64 on the device: a zero weight, a negative one, a NaN, and a sum
    off by 1e-4 (a sum off by 1e-6 is accepted).  The solve that does not
    use the bad vector is unaffected.  An iteration cap below what the
    tolerance needs gives SK_ENOTCONV with the error reported."""
    _say("status codes", rng_mode)
    c, U, eps, q = _divergence_inputs("gauss2d", n=200, m=200)
    bad = []
    for kind in ("zero", "negative", "nan", "sum"):
        a = c.a.astype(np.float64)
        if kind == "zero":
            a[5] = 0.0
        elif kind == "negative":
            a[5], a[6] = -a[5], a[6] + 2 * a[5]
        elif kind == "nan":
            a[5] = np.nan
        else:
            a = a * (1.0 + 1e-4)
        bad.append((kind, a.astype(np.float32)))
    for kind, a in bad:
        out, st = api.divergence(dev(c.X), dev(c.Y), dev(a), dev(c.b), dev(U), eps,
                                 q, fixed_iter=10, range=rng_mode)
        infos = st.infos()
        assert list(infos["status"]) == [1, 1, 0], (kind, infos)
        assert list(infos["iters"][:2]) == [0, 0] and np.isnan(host(out)[0]), kind
    a = (c.a.astype(np.float64) * (1.0 + 1e-6)).astype(np.float32)
    out, st = api.divergence(dev(c.X), dev(c.Y), dev(a), dev(c.b), dev(U), eps, q,
                             fixed_iter=10, range=rng_mode)
    assert list(st.infos()["status"]) == [0, 0, 0]
    out, st = api.divergence(dev(c.X), dev(c.Y), dev(c.a), dev(c.b), dev(U),
                             eps, q, tol=1e-12, max_iter=3, range=rng_mode)
    infos = st.infos()
    assert list(infos["status"]) == [4, 4, 4]
    assert list(infos["iters"]) == [3, 3, 3]
    assert np.all(infos["err"] > 1e-12)


def test_divergence_assemble_matches_the_divergence_call(api):
    """sinkhorn_divergence_assemble on the three records a divergence left in
    its state reproduces that call's (W_bar, W_xy, W_xx, W_yy) bit for bit;
    two problems assembled in one call."""
    _say("assemble")
    outs, recs = [], []
    for seed in (0, 1):
        c, U, eps, q = _divergence_inputs("gauss2d", seed=seed, n=300, m=250)
        out, st = api.divergence(dev(c.X), dev(c.Y), dev(c.a), dev(c.b), dev(U), eps, q,
                                 fixed_iter=50)
        L = st.layout
        outs.append(host(out))
        recs.append(st.buf[L.info:L.info + 3 * api.INFO_BYTES].clone())
    got = host(api.divergence_assemble(torch.cat(recs), 2))
    assert np.array_equal(got, np.stack(outs))
