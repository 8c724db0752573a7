"""Stored expected values (tests/golden/*.json, written by
tests/golden/make_golden.py from the float64 oracle): the oracle still
reproduces them, the library's host Lambert routine matches them, and the
GPU library matches them within the parity tolerances."""
import ctypes
import importlib.util
import json
import os

import numpy as np
import pytest

import oracle
from paper_2006_07057_amd import inputs
from parity import check_divergence

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(name):
    with open(os.path.join(HERE, name + ".json")) as f:
        return json.load(f)


def _maker():
    spec = importlib.util.spec_from_file_location("make_golden",
                                                  os.path.join(HERE, "make_golden.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("name", ["gauss2d_1k", "lambert_q", "accelerated_small"])
def test_oracle_reproduces_golden(name):
    """Regression guard: the oracle as it stands writes the same values."""
    fresh = getattr(_maker(), name)()
    stored = _load(name)
    assert sorted(fresh) == sorted(stored)
    for k, v in stored.items():
        if isinstance(v, float):
            assert fresh[k] == pytest.approx(v, rel=1e-12, abs=1e-300), k
        elif k == "cases":
            for cf, cs in zip(fresh[k], v):
                assert cf["q"] == pytest.approx(cs["q"], rel=1e-13)
        else:
            assert fresh[k] == v, k


def test_library_lambert_q_matches_golden():
    """sinkhorn_gaussian_q (host code of the library, Halley's iteration)
    against the oracle's Lambert values."""
    from paper_2006_07057_amd import _lib
    L = _lib.lib()
    for c in _load("lambert_q")["cases"]:
        q = ctypes.c_double(0.0)
        assert L.sinkhorn_gaussian_q(c["R"], c["eps"], c["d"], ctypes.byref(q)) == 0
        assert q.value == pytest.approx(c["q"], rel=1e-12)


@pytest.mark.gpu
@pytest.mark.parametrize("rng_mode", [0, 1], ids=["ext", "lin"])
def test_gpu_gauss2d_matches_golden(rng_mode):
    import torch
    from paper_2006_07057_amd import api
    g = _load("gauss2d_1k")
    c = inputs.gauss2d(0, n=1000, m=1000)
    U = inputs.gaussian_anchors(0, g["r"], 2, 1.0)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    out, _ = api.divergence(t(c.X), t(c.Y), t(c.a), t(c.b), t(U), g["eps"], g["q"],
                            fixed_iter=g["fixed_iter"], range=rng_mode)
    o = out.cpu().numpy()
    check_divergence(f"golden gauss2d_1k range={rng_mode}", o,
                     (g["W_bar"], g["W_xy"], g["W_xx"], g["W_yy"]))


@pytest.mark.gpu
def test_gpu_accelerated_matches_golden():
    import torch
    from paper_2006_07057_amd import api
    g = _load("accelerated_small")
    assert g["min_block_margin"] > 1e-4 and g["min_test_margin"] > 1e-2
    Fx, Fy, a, b = _maker().accelerated_inputs()
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    n, r = Fx.shape
    m = Fy.shape[0]
    P, Q, at, bt = t(Fx), t(Fy), t(a), t(b)
    u = torch.zeros(2 * n, device="cuda")
    v = torch.zeros(2 * m, device="cuda")
    w = torch.zeros(2 * r, device="cuda")
    z = torch.zeros(2 * r, device="cuda")
    info = torch.zeros(api.INFO_BYTES, dtype=torch.uint8, device="cuda")
    tr = torch.zeros(1, dtype=torch.int32, device="cuda")
    spec = api.solve_spec(P, Q, at, bt, u, v, w, z, info, eps=1.0)
    api.solve_accelerated(spec, fixed_iter=g["steps"], trials=tr)
    rec = api.parse_infos(info)[0]
    assert rec["status"] == 0 and rec["iters"] == g["steps"]
    assert int(tr.cpu()[0]) == g["trials"]
    assert rec["w_hat"] == pytest.approx(g["dual_value"], rel=1e-5)


@pytest.mark.gpu
def test_gpu_gmm3d_1m_matches_golden():
    """The 10^6-point mixture workload at full size (two 4-component Gaussian
    mixtures in R^3, r = 1024, eps = 0.1), inputs and anchors made as the
    benchmark makes them, through the entry point and launch the benchmark
    times, against the factored float64 oracle's stored values: 100 fixed
    iterations (every term and W_bar within 1e-5), and the stop test at
    tol = 1e-6 with at most 2000 iterations (W_bar and the terms within
    1e-5; iteration counts within the float32 jitter of the stopping index
    near the tolerance)."""
    import torch
    from paper_2006_07057_amd import api
    g = _load("gmm3d_1m")
    c = inputs.gmm3d(0)
    U, q = api.gaussian_anchors(inputs.standard_normal_anchors(0, 1024, 3), 0.1,
                                R=inputs.max_norm(c.X, c.Y))
    assert q == pytest.approx(g["q"], rel=1e-13)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    X, Y, a, b, Ud = t(c.X), t(c.Y), t(c.a), t(c.b), t(U)
    for key, kw in (("fixed_100", dict(fixed_iter=100)),
                    ("tol_1e-6", dict(tol=1e-6, max_iter=2000))):
        ref = g[key]
        out, st = api.divergence(X, Y, a, b, Ud, 0.1, q, **kw)
        o = out.cpu().numpy()
        infos = st.infos()
        print(f"[golden] gmm3d_1m {key}: iters gpu {list(infos['iters'])} "
              f"oracle {ref['iters']}", flush=True)
        assert list(infos["status"]) == [0, 0, 0]
        check_divergence(f"gmm3d_1m {key}", o,
                         (ref["W_bar"], ref["W_xy"], ref["W_xx"], ref["W_yy"]))
        for it, rit in zip(infos["iters"], ref["iters"]):
            assert abs(int(it) - rit) <= max(3, rit // 20), (key, it, rit)
