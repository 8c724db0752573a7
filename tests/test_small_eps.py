"""The small-eps cells of the request stream (the regime where, as the
experiments of Sec. 4 note, Sinkhorn needs many iterations and plain float32
scalings leave their range): eps = 0.05 with d = 16 and d = 64, and
eps = 0.5 with d = 64, on requests of the stream itself (seeded, n and m
between 1e3 and 2.5e3).  The extended-range domain is compared with the
float64 oracle at a fixed iteration count and at the stop test (tol 1e-6)
with a cap high enough for Algorithm 1 to converge in float64: the oracle
needs up to 2.5e4 iterations on these self-problems, far above the
stream's cap of 2000 (so requests there end with SK_ENOTCONV in float32 and
float64 alike)."""
import sys

import numpy as np
import pytest

import oracle
from paper_2006_07057_amd import inputs
from parity import check_divergence

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

# request ids of inputs.request_stream(seed=0) (2048 requests at 500/s):
# (eps, d, r) = (0.05, 16, 64), (0.05, 64, 256), (0.5, 64, 256)
RIDS = [869, 1260, 1312]


def _say(*a):
    print("[gpu-test]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def api():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2006_07057_amd import api as A
    A.lib()
    return A


@pytest.fixture(scope="module")
def stream():
    return {q.rid: q for q in inputs.request_stream(seed=0, count=2048, rate=500.0)}


def _case(api, spec):
    import torch
    cl = inputs.request_arrays(spec)
    R = inputs.max_norm(cl.X, cl.Y)
    U, q = api.gaussian_anchors(inputs.standard_normal_anchors(spec.seed, spec.r, spec.d),
                                spec.eps, R=R)
    # the oracle's own bandwidth and anchors from the same draws
    qo = oracle.lambert_q(R, spec.eps, spec.d)
    Uo = inputs.gaussian_anchors(spec.seed, spec.r, spec.d, oracle.sigma2_from_q(qo, spec.eps))
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    return cl, (t(cl.X), t(cl.Y), t(cl.a), t(cl.b), t(U), spec.eps, q), Uo, qo


@pytest.mark.parametrize("rid", RIDS)
def test_small_eps_fixed_iterations(api, stream, rid):
    spec = stream[rid]
    _say("small eps fixed", rid, spec.eps, spec.d, spec.r, spec.n, spec.m)
    cl, args, Uo, qo = _case(api, spec)
    out, st = api.divergence(*args, fixed_iter=300)
    assert list(st.infos()["status"]) == [0, 0, 0]
    ref = oracle.divergence_scaled(cl.X, cl.Y, cl.a, cl.b, Uo, spec.eps, qo, fixed_iter=300)
    check_divergence(f"small eps {spec.eps} d={spec.d} r={spec.r} rid={rid} 300 fixed",
                     out.cpu().numpy(), ref)


@pytest.mark.parametrize("rid", RIDS)
def test_small_eps_converged(api, stream, rid):
    spec = stream[rid]
    _say("small eps tol", rid, spec.eps, spec.d, spec.r, spec.n, spec.m)
    cl, args, Uo, qo = _case(api, spec)
    out, st = api.divergence(*args, tol=1e-6, max_iter=40000)
    infos = st.infos()
    ref = oracle.divergence_scaled(cl.X, cl.Y, cl.a, cl.b, Uo, spec.eps, qo, tol=1e-6,
                                   max_iter=40000)
    _say("iterations gpu", list(infos["iters"]), "oracle",
         [ref.xy.iters, ref.xx.iters, ref.yy.iters], "err gpu", list(infos["err"]))
    assert list(infos["status"]) == [0, 0, 0], infos
    assert max(ref.xy.iters, ref.xx.iters, ref.yy.iters) > 2000 or spec.eps == 0.5
    check_divergence(f"small eps {spec.eps} d={spec.d} r={spec.r} rid={rid} tol 1e-6",
                     out.cpu().numpy(), ref)
