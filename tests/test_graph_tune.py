"""HIP-graph capture of a divergence step, and the launch-planning
autotuner.  CPU tests cover the tuning table's storage; GPU tests replay the
captured graph against eager runs and check that tuning changes timing, not
results."""
import json

import numpy as np
import pytest

import oracle
from paper_2006_07057_amd import autotune, inputs


def test_class_of():
    assert autotune.class_of(1) == 4
    assert autotune.class_of(128) == 128
    assert autotune.class_of(129) == 256
    assert autotune.class_of(4096) == 4096
    with pytest.raises(ValueError):
        autotune.class_of(4097)


def test_table_save_load_roundtrip(tmp_path):
    from paper_2006_07057_amd import api
    autotune.reset()
    default = api.tune_get(256)
    table = {256: 512 << 10, 1024: 4 << 20}
    p = str(tmp_path / "tune.json")
    with open(p, "w") as f:
        # a table written before layouts were tuned: targets only
        json.dump({"device": None, "targets": {str(k): v for k, v in table.items()}}, f)
    assert autotune.load(p) == {256: (0, 512 << 10), 1024: (0, 4 << 20)}
    assert api.tune_get(200) == 512 << 10      # same class as 256
    assert api.tune_get(1000) == 4 << 20
    assert api.tune_get(64) == default
    with open(p, "w") as f:
        json.dump({"targets": {"1024": 4 << 20}, "layouts": {"1024": 1}}, f)
    assert autotune.load(p) == {1024: (1, 4 << 20)}
    assert api.tune_get_layout(1000) == 1 and api.tune_get_layout(512) == 0
    autotune.save(str(tmp_path / "again.json"))
    back = json.load(open(tmp_path / "again.json"))
    assert int(back["targets"]["256"]) == 512 << 10 and int(back["targets"]["64"]) == default
    assert int(back["layouts"]["1024"]) == 1 and int(back["layouts"]["256"]) == 0
    autotune.reset()
    assert api.tune_get(256) == default and api.tune_get_layout(1024) == 0


def test_layouts_per_class():
    """Every class lists its compiled lane layouts, the default first, each
    covering the class's largest r (4 G C = rmax)."""
    from paper_2006_07057_amd import api
    for c in autotune.CLASS_RMAX:
        lays = api.solver_layouts(c)
        assert len(lays) >= 1
        for (G, C, U, W) in lays:
            assert 4 * G * C == c and 64 % G == 0 and U >= 1 and W >= 1
    assert len(api.solver_layouts(512)) == 2 and len(api.solver_layouts(1024)) == 2


def test_table_rejects_bad_entries(tmp_path):
    from paper_2006_07057_amd import api
    p = str(tmp_path / "bad.json")
    with open(p, "w") as f:
        json.dump({"targets": {"100": 1024}}, f)   # not a class
    with pytest.raises(ValueError):
        autotune.load(p)
    with open(p, "w") as f:
        json.dump({"targets": {"4096": 1024}, "layouts": {"4096": 3}}, f)   # no such layout
    with pytest.raises(ValueError):
        autotune.load(p)
    autotune.reset()
    with pytest.raises(Exception):
        api.tune_set(5000, 1024)
    with pytest.raises(Exception):
        api.tune_set(64, -1)
    with pytest.raises(Exception):
        api.tune_set_layout(4096, 1)
    with pytest.raises(Exception):
        api.tune_set_layout(512, -1)


# ------------------------------------------------------------------- GPU
def _inputs(seed, n, m, d, r):
    c = inputs.gauss2d(seed, n=n, m=m, d=d)
    U = inputs.gaussian_anchors(0, r, d, 1.0)   # same anchors for every call
    return c.X, c.Y, c.a, c.b, U


@pytest.mark.gpu
def test_graph_replays_match_eager():
    import torch
    from paper_2006_07057_amd import api
    n, m, d, r, eps = 2000, 1500, 3, 128, 0.5
    q = 4.0 / eps
    G = api.DivergenceGraph(n, m, d, r, eps, q, tol=1e-6, max_iter=2000)
    t = lambda x: torch.from_numpy(x).cuda()
    noise = torch.randn(512, 512, device="cuda")
    for rep in range(4):
        X, Y, a, b, U = (t(x) for x in _inputs(10 + rep, n, m, d, r))
        out_g, grads_g = G(X, Y, a, b, U)
        out_g = out_g.cpu().numpy().copy()
        grads_g = [g.cpu().numpy().copy() for g in grads_g]
        # eager work and synchronisation between replays
        for _ in range(3):
            noise = torch.tanh(noise @ noise.T)
        torch.cuda.synchronize()
        out_e, st = api.divergence(X, Y, a, b, U, eps, q, tol=1e-6, max_iter=2000)
        grads_e = api.divergence_backward(st)
        np.testing.assert_array_equal(out_g, out_e.cpu().numpy())
        for g1, g2 in zip(grads_g, grads_e):
            np.testing.assert_array_equal(g1, g2.cpu().numpy())


@pytest.mark.gpu
def test_batched_graph_replays_match_eager():
    """A packed batch of uneven problems (several feature-count classes)
    captured once with its adjoint: every replay, with eager work between
    replays, equals an eager batched call bit for bit."""
    import torch
    from paper_2006_07057_amd import api
    rng = np.random.default_rng(7)
    shapes = []
    for i in range(12):
        n, m = (int(x) for x in rng.integers(500, 5000, size=2))
        d = int(rng.choice([2, 3]))
        r = int(rng.choice([64, 256, 1024]))
        shapes.append((n, m, d, r, 0.5, 8.0))
    G = api.BatchedDivergenceGraph(shapes, tol=1e-6, max_iter=2000)
    t = lambda x: torch.from_numpy(x).cuda()
    noise = torch.randn(512, 512, device="cuda")
    for rep in range(3):
        probs = [tuple(t(x) for x in _inputs(100 * rep + i, n, m, d, r))
                 for i, (n, m, d, r, _, _) in enumerate(shapes)]
        out_g, grads_g = G(probs)
        out_g = out_g.cpu().numpy().copy()
        grads_g = [[g.cpu().numpy().copy() for g in gs] for gs in grads_g]
        for _ in range(3):
            noise = torch.tanh(noise @ noise.T)
        torch.cuda.synchronize()
        out_e, states = api.divergence_batched(
            [p + (0.5, 8.0) for p in probs], tol=1e-6, max_iter=2000)
        np.testing.assert_array_equal(out_g, out_e.cpu().numpy())
        for gs, st in zip(grads_g, states):
            for g1, g2 in zip(gs, api.divergence_backward(st)):
                np.testing.assert_array_equal(g1, g2.cpu().numpy())


@pytest.mark.gpu
def test_graph_matches_oracle():
    import torch
    from paper_2006_07057_amd import api
    n, m, d, r, eps = 400, 300, 2, 64, 0.5
    q = 4.0 / eps
    X, Y, a, b, U = _inputs(3, n, m, d, r)
    G = api.DivergenceGraph(n, m, d, r, eps, q, fixed_iter=150, backward=False)
    t = lambda x: torch.from_numpy(x).cuda()
    out, _ = G(t(X), t(Y), t(a), t(b), t(U))
    ref = oracle.divergence_scaled(X, Y, a, b, U, eps, q, fixed_iter=150)
    assert float(out[0].item()) == pytest.approx(ref.value, rel=1e-5)


@pytest.mark.gpu
def test_autotune_changes_timing_not_results():
    import torch
    from paper_2006_07057_amd import api
    autotune.reset()
    n, r = 40000, 128
    Px, Py, a, b = autotune._problem(n, n, r, 3, 0.5, 0, api.EXTENDED, torch.device("cuda"))
    ref = api.solve(Px, Py, a, b, fixed_iter=30)
    ref_u = api.host_log_scaling(ref.u, api.EXTENDED)
    times = autotune.tune_class(r, n, candidates=(64 << 10, 256 << 10, 4 << 20), iters=10)
    assert set(times) == {(0, 64 << 10), (0, 256 << 10), (0, 4 << 20)}
    assert all(t > 0 for t in times.values())
    assert (api.tune_get_layout(r), api.tune_get(r)) == min(times, key=times.get)
    got = api.solve(Px, Py, a, b, fixed_iter=30)
    got_u = api.host_log_scaling(got.u, api.EXTENDED)
    np.testing.assert_allclose(got_u, ref_u, rtol=0, atol=2e-5)
    assert got.info()["w_hat"] == pytest.approx(ref.info()["w_hat"], rel=1e-6)
    autotune.reset()


@pytest.mark.gpu
@pytest.mark.parametrize("r", [64, 200, 512, 1024])
@pytest.mark.parametrize("rng", [0, 1])
def test_alternative_layouts_match_oracle(r, rng):
    """Each compiled lane layout other than the default, selected through
    the tuning table, gives the oracle's divergence (Eq. reg-sdiv) within
    1e-5 at 100 fixed iterations, and the default's result to float32
    rounding; both numeric domains, several workgroups per solve."""
    import torch
    from paper_2006_07057_amd import api
    from parity import check_divergence
    n, m, d, eps = 3000, 2500, 3, 0.5
    X, Y, a, b, U = _inputs(11, n, m, d, r)
    q = oracle.q_from_sigma2(1.0, eps)
    t = lambda x: torch.from_numpy(x).cuda()
    args = (t(X), t(Y), t(a), t(b), t(U), eps, q)
    ref = oracle.divergence_scaled(X, Y, a, b, U.astype(np.float64), eps, q, fixed_iter=100)
    autotune.reset()
    api.tune_set(r, 16 << 10)              # several workgroups per solve
    try:
        base, _ = api.divergence(*args, fixed_iter=100, range=rng)
        base = base.cpu().numpy()
        for v in range(1, len(api.solver_layouts(r))):
            api.tune_set_layout(r, v)
            out, _ = api.divergence(*args, fixed_iter=100, range=rng)
            out = out.cpu().numpy()
            check_divergence(f"layout {api.solver_layouts(r)[v]} r={r} range={rng}", out, ref)
            np.testing.assert_allclose(out[1:], base[1:], rtol=1e-6)
    finally:
        autotune.reset()
