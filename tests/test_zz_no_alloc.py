"""The allocation-free solve entry point (sinkhorn_solve_noalloc, static
device scratch) against sinkhorn_solve with a caller workspace: identical
scalings, r-vectors and solve records, on two calls in a row (the second on
a smaller problem, so the scratch holds the first call's leftovers), and
size/argument rejection before any device work."""
import ctypes

import numpy as np
import pytest

from paper_2006_07057_amd import _lib, inputs


def _api():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2006_07057_amd import api
    api.lib()
    return torch, api


def _problem(torch, api, seed, n, m, d, r, eps, rng_mode):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, d)).astype(np.float32)
    Y = (rng.standard_normal((m, d)) + 0.5).astype(np.float32)
    a = inputs.dirichlet_weights(rng, n)
    b = inputs.dirichlet_weights(rng, m)
    U, q = api.gaussian_anchors(inputs.standard_normal_anchors(seed, r, d), eps,
                                R=inputs.max_norm(X, Y))
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    Px, _ = api.features(t(X), t(U), eps, q, range=rng_mode)
    Py, _ = api.features(t(Y), t(U), eps, q, range=rng_mode)
    return Px, Py, t(a), t(b)


def _outputs(torch, n, m, r):
    f = lambda k: torch.full((2 * k,), float("nan"), dtype=torch.float32, device="cuda")
    return f(n), f(m), f(r), f(r), torch.zeros(24, dtype=torch.uint8, device="cuda")


def _call(torch, api, fn, P, opts, outs, ws=None):
    Px, Py, a, b = P
    n, r = Px.shape
    m = Py.shape[0]
    u, v, w, z, info = outs
    args = [api._ptr(Px), n, api._ptr(Py), m, r, api._ptr(a), api._ptr(b), ctypes.byref(opts),
            api._ptr(u), api._ptr(v), api._ptr(w), api._ptr(z), api._ptr(info)]
    if ws is not None:
        args += [api._ptr(ws), ws.numel()]
    args.append(api._stream())
    return fn(*args)


@pytest.mark.gpu
@pytest.mark.parametrize("rng_mode", [0, 1], ids=["ext", "lin"])
def test_noalloc_solve_equals_workspace_solve(rng_mode):
    torch, api = _api()
    L = _lib.lib()
    cases = [(1, 30000, 41000, 3, 1024, 0.5, dict(tol=1e-6, max_iter=500)),
             (2, 1500, 900, 2, 256, 0.7, dict(fixed_iter=60))]
    for seed, n, m, d, r, eps, kw in cases:       # second call: smaller problem
        P = _problem(torch, api, seed, n, m, d, r, eps, rng_mode)
        opts = api._opts(kw.get("tol", 1e-6), kw.get("max_iter", 2000),
                         kw.get("fixed_iter", 0), False, rng_mode)
        need = L.sinkhorn_solve_workspace_size(n, m, r)
        assert 0 < need <= _lib.SK_NOALLOC_SCRATCH_BYTES
        ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        ref = _outputs(torch, n, m, r)
        got = _outputs(torch, n, m, r)
        assert _call(torch, api, L.sinkhorn_solve, P, opts, ref, ws) == _lib.SK_OK
        assert _call(torch, api, L.sinkhorn_solve_noalloc, P, opts, got) == _lib.SK_OK
        torch.cuda.synchronize()
        k = 2 if rng_mode == 0 else 1
        for x, y, cnt in zip(ref[:4], got[:4], (n, m, r, r)):
            assert torch.equal(x[:k * cnt], y[:k * cnt])
        ri = api.parse_infos(ref[4])[0]
        gi = api.parse_infos(got[4])[0]
        assert ri["status"] in (0, 4) and ri.tobytes() == gi.tobytes(), (ri, gi)


def test_noalloc_rejects_before_device_work():
    """Argument errors and sizes whose workspace exceeds the static scratch
    are returned synchronously (no pointer is dereferenced)."""
    L = _lib.lib()
    P = ctypes.c_void_p(0x1000)
    o = _lib.sk_solve_opts(1e-6, 100, 0, 0, 0)
    args = [P, 10, P, 12, 8, P, P, ctypes.byref(o), P, P, P, P, P, None]
    assert L.sinkhorn_solve_noalloc(*args[:0], None, *args[1:]) == _lib.SK_EINVAL
    bad = list(args); bad[4] = 6
    assert L.sinkhorn_solve_noalloc(*bad) == _lib.SK_ENOTSUP
    big = list(args); big[1] = big[3] = 100_000; big[4] = 4096
    assert L.sinkhorn_solve_workspace_size(100_000, 100_000, 4096) > _lib.SK_NOALLOC_SCRATCH_BYTES
    assert L.sinkhorn_solve_noalloc(*big) == _lib.SK_ENOMEM
