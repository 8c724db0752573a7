"""Batched solves with warm start and the continuous-batching server.

CPU tests cover the admission policy and the statistics; GPU tests check
that packed launches reproduce single launches, that continuing from a
returned scaling continues Algorithm 1, and that every request served in a
mix of overlapping requests gets the result it gets alone (and the oracle's).
"""
import math

import numpy as np
import pytest

import oracle
from paper_2006_07057_amd import inputs
from parity import check_divergence

serve = pytest.importorskip("paper_2006_07057_amd.serve")



# ------------------------------------------------------------------ host
def test_admission_is_fifo_and_respects_the_budget():
    foot = [30, 20, 40, 10, 5]
    plan = serve.plan_admission(foot, live_bytes=0, live_count=0, budget=95,
                                reserve=10)
    # 30 + 20 + 40 = 90 > 95 - 10: the third waits, and so does every later
    # request (no overtaking)
    assert plan == ["admit", "admit"]
    assert serve.plan_admission(foot[2:], 50, 2, 95, 10) == []
    assert serve.plan_admission(foot[2:], 0, 0, 95, 10) == ["admit", "admit", "admit"]


def test_admission_rejects_only_what_can_never_fit():
    # too large for the whole budget: rejected when nothing else is live ...
    assert serve.plan_admission([500, 10], 0, 0, 100, 0) == ["reject", "admit"]
    # ... but waits (is not rejected) while other requests hold memory
    assert serve.plan_admission([500, 10], 60, 1, 100, 0) == []


@pytest.mark.parametrize("seed", range(5))
def test_admission_never_exceeds_budget(seed):
    rng = np.random.default_rng(seed)
    foot = list(rng.integers(1, 60, size=40))
    live, count, budget, reserve = 0, 0, 200, 7
    queue = list(foot)
    while queue:
        plan = serve.plan_admission(queue, live, count, budget, reserve)
        assert plan, "a request that fits an empty device must be admitted"
        for dec in plan:
            f = queue.pop(0)
            if dec == "admit":
                live += f
                count += 1
                assert live + reserve <= budget
        # retire everything (the next epoch frees memory)
        live, count = 0, 0


def test_latency_stats():
    R = serve.Result
    res = [R(0, 0, 1.0, (0,) * 3, (1,) * 3, 0.0, 0.0, 1.0, 1),
           R(1, 0, 1.0, (0,) * 3, (1,) * 3, 0.5, 0.5, 2.5, 1),
           R(2, 4, math.nan, (0,) * 3, (1,) * 3, 1.0, 1.0, 3.0, 1)]
    st = serve.latency_stats(res)
    assert st["ok"] == 2 and st["failed"] == {4: 1}
    assert st["p50_ms"] == pytest.approx(1500.0)
    assert st["divergences_per_s"] == pytest.approx(2 / 3.0)


# ------------------------------------------------------------------- GPU
def _torch():
    import torch
    return torch


def _solve_inputs(seed, n, m, d, r, eps=0.5, sigma2=1.0):
    torch = _torch()
    from paper_2006_07057_amd import api
    c = inputs.gauss2d(seed, n=n, m=m, d=d)
    U = inputs.gaussian_anchors(seed, r, d, sigma2)
    t = lambda x: torch.from_numpy(x).cuda()
    q = 4.0 * sigma2 / eps
    Px, _ = api.features(t(c.X), t(U), eps, q)
    Py, _ = api.features(t(c.Y), t(U), eps, q)
    return Px, Py, t(c.a), t(c.b)


def _buffers(n, m, r):
    torch = _torch()
    f = lambda k: torch.empty(2 * k, dtype=torch.float32, device="cuda")
    info = torch.zeros(24, dtype=torch.uint8, device="cuda")
    return f(n), f(m), f(r), f(r), info


@pytest.mark.gpu
def test_solve_batched_equals_single_launches_bit_exact():
    from paper_2006_07057_amd import api
    shapes = [(3000, 2500, 3, 128), (700, 900, 2, 128), (5000, 4000, 3, 256),
              (1200, 1200, 16, 64)]
    probs = [_solve_inputs(i, *s) for i, s in enumerate(shapes)]
    singles = [api.solve(Px, Py, a, b, fixed_iter=25) for (Px, Py, a, b) in probs]
    bufs, specs = [], []
    for (Px, Py, a, b), (n, m, d, r) in zip(probs, shapes):
        B = _buffers(n, m, r)
        bufs.append(B)
        specs.append(api.solve_spec(Px, Py, a, b, *B, eps=1.0))
    api.solve_batched(specs, fixed_iter=25)
    for S, B in zip(singles, bufs):
        for x, y in zip((S.u, S.v, S.w, S.z), B[:4]):
            assert np.array_equal(x.cpu().numpy(), y.cpu().numpy())
        assert api.parse_infos(B[4])[0]["w_hat"] == S.info()["w_hat"]


@pytest.mark.gpu
def test_warm_start_continues_algorithm_1():
    """K1 iterations, then K2 more from the returned u, against the oracle's
    K1 + K2 iterations from the same start."""
    from paper_2006_07057_amd import api
    n, m, d, r = 1500, 1300, 2, 128
    Px, Py, a, b = _solve_inputs(7, n, m, d, r)
    u, v, w, z, info = _buffers(n, m, r)
    sp = api.solve_spec(Px, Py, a, b, u, v, w, z, info)
    api.solve_batched([sp], fixed_iter=40)
    api.solve_batched([sp], fixed_iter=35, warm_start=True)
    got_u = api.host_log_scaling(u, api.EXTENDED)
    got_v = api.host_log_scaling(v, api.EXTENDED)
    Lx = Px.double().cpu().numpy() * math.log(2.0)
    Ly = Py.double().cpu().numpy() * math.log(2.0)
    ref = oracle.sinkhorn_factored(np.exp(Lx), np.exp(Ly), a.double().cpu().numpy(),
                                   b.double().cpu().numpy(), fixed_iter=75)
    # the pair (u, v) is unique up to (c u, v / c): compare u v^T invariants
    shift = np.mean(got_u - np.log(ref.u))
    assert np.allclose(got_u - shift, np.log(ref.u), atol=2e-4)
    assert np.allclose(got_v + shift, np.log(ref.v), atol=2e-4)


def _specs(count, seed, lo=300, hi=3000):
    return inputs.request_stream(seed=seed, count=count, rate=3000.0, lo=lo, hi=hi,
                                 d_menu=(2, 3, 16), r_menu=(64, 128, 256),
                                 eps_menu=(0.5, 5.0))


@pytest.mark.gpu
def test_server_mix_matches_alone_and_overlaps():
    torch = _torch()
    from paper_2006_07057_amd import api
    reqs = [serve.from_spec(s) for s in _specs(12, seed=11)]
    srv = serve.Server(hbm_budget=2 << 30, epoch_iters=12)
    res = {r.rid: r for r in srv.run(reqs)}
    assert len(res) == len(reqs)
    # work of requests admitted at different times shared packed launches
    joined = [e for e in srv.epoch_log if e["admitted"] and
              len(set(e["live"]) - set(e["admitted"])) > 0]
    assert joined, "no request joined requests already on the device"
    assert max(len(e["live"]) for e in srv.epoch_log) >= 3
    for q in reqs:
        r = res[q.rid]
        assert r.status == 0, (q.rid, r.status)
        t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
        out, st = api.divergence(t(q.X), t(q.Y), t(q.a), t(q.b), t(q.U), q.eps, q.q)
        check_divergence(f"served vs alone request {q.rid}", (r.w_bar,) + r.w_hat,
                         tuple(out.cpu().numpy()))
        # the stopping iteration agrees up to the float32 rounding of the
        # marginal error near the tolerance (~1e-7 absolute against 1e-6)
        alone_iters = [int(i) for i in st.infos()["iters"]]
        assert all(abs(i - j) <= max(3, 0.05 * j) for i, j in zip(r.iters, alone_iters)), \
            (q.rid, r.iters, alone_iters)


@pytest.mark.gpu
def test_server_results_match_oracle():
    specs = _specs(4, seed=5, lo=200, hi=600)
    reqs = [serve.from_spec(s) for s in specs]
    srv = serve.Server(hbm_budget=1 << 30, epoch_iters=20)
    res = {r.rid: r for r in srv.run(reqs)}
    for sp in specs:
        # the oracle forms its own bandwidth and anchors from the request's
        # seeded draws (nothing taken from the library)
        cl = inputs.request_arrays(sp)
        q = oracle.lambert_q(inputs.max_norm(cl.X, cl.Y), sp.eps, sp.d)
        U = inputs.gaussian_anchors(sp.seed, sp.r, sp.d, oracle.sigma2_from_q(q, sp.eps))
        ref = oracle.divergence_scaled(cl.X, cl.Y, cl.a, cl.b, U, sp.eps, q,
                                       tol=1e-6, max_iter=2000)
        r = res[sp.rid]
        check_divergence(f"served vs oracle request {sp.rid}", (r.w_bar,) + r.w_hat, ref)


@pytest.mark.gpu
def test_server_budget_limits_live_requests():
    reqs = [serve.from_spec(s) for s in _specs(8, seed=2, lo=1500, hi=2500)]
    foot = [serve.footprint_bytes(q.X.shape[0], q.Y.shape[0], q.X.shape[1], q.U.shape[0])
            for q in reqs]
    budget = int(2.5 * max(foot)) + (80 << 20)
    srv = serve.Server(hbm_budget=budget, epoch_iters=25)
    res = srv.run(reqs)
    assert len(res) == len(reqs) and all(r.status == 0 for r in res)
    assert all(e["bytes"] + srv.reserve <= budget for e in srv.epoch_log)
    # the budget, not the arrivals, limited how many requests were live
    assert max(len(e["live"]) for e in srv.epoch_log) < len(reqs)
    assert any(r.admitted > r.arrival + 1e-4 for r in res)
