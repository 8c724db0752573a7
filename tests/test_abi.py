"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point declared in include/sinkhorn.h, validates arguments before
touching the device, and its host helpers agree with the oracle."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle
from paper_2006_07057_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sinkhorn.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int64_t|int|size_t|const char\*)\s+"
                                 r"(sinkhorn_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libsinkhorn.so is not built (python -m "
                    "paper_2006_07057_amd.build)")
    return _lib.lib()


def test_header_declares_the_entry_points():
    names = _declared()
    for must in ("sinkhorn_features", "sinkhorn_solve", "sinkhorn_divergence",
                 "sinkhorn_divergence_batched", "sinkhorn_features_backward",
                 "sinkhorn_divergence_backward", "sinkhorn_gaussian_q"):
        assert must in names


def test_library_exports_every_declared_symbol(L):
    for name in _declared():
        assert hasattr(L, name), name
        assert name in _lib.SIGNATURES, f"binding misses {name}"


def test_strerror_and_version(L):
    for s in range(8):
        assert L.sinkhorn_strerror(s).decode().startswith("SK_")
    assert b"gfx950" in L.sinkhorn_version()


@pytest.mark.parametrize("R,eps,d", [(1.0, 1.0, 1), (4.0, 0.1, 3),
                                     (2.5, 0.05, 64), (30.0, 10.0, 784),
                                     (1e-3, 1.0, 2), (math.sqrt(math.e), 1, 1)])
def test_gaussian_q_matches_oracle(L, R, eps, d):
    q = ctypes.c_double()
    assert L.sinkhorn_gaussian_q(R, eps, d, ctypes.byref(q)) == _lib.SK_OK
    assert q.value == pytest.approx(oracle.lambert_q(R, eps, d), rel=1e-13)


def test_gaussian_q_rejects_bad_arguments(L):
    q = ctypes.c_double()
    assert L.sinkhorn_gaussian_q(0.0, 1.0, 2, ctypes.byref(q)) == _lib.SK_EINVAL
    assert L.sinkhorn_gaussian_q(1.0, -1.0, 2, ctypes.byref(q)) == _lib.SK_EINVAL
    assert L.sinkhorn_gaussian_q(1.0, 1.0, 0, ctypes.byref(q)) == _lib.SK_EINVAL
    assert L.sinkhorn_gaussian_q(1.0, 1.0, 2, None) == _lib.SK_EINVAL


def _problem(n=10, m=12, d=2, r=8, eps=0.5, q=2.0, ptr=0x1000):
    return _lib.sk_problem(ptr, ptr, ptr, ptr, ptr, n, m, d, r, eps, q)


def test_argument_errors_return_before_any_device_work(L):
    P = ctypes.c_void_p(0x1000)
    o = _lib.sk_solve_opts(1e-6, 100, 0, 0, 0)
    # features
    assert L.sinkhorn_features(None, 10, 2, P, 8, 0.5, 2.0, 0, P, P, None) == _lib.SK_EINVAL
    assert L.sinkhorn_features(P, 0, 2, P, 8, 0.5, 2.0, 0, P, P, None) == _lib.SK_EINVAL
    assert L.sinkhorn_features(P, 10, 2, P, 8, 0.0, 2.0, 0, P, P, None) == _lib.SK_EINVAL
    assert L.sinkhorn_features(P, 10, 2, P, 8, 0.5, 0.4, 1, P, P, None) == _lib.SK_EINVAL
    assert L.sinkhorn_features(P, 10, 2, P, 8, 0.5, 2.0, 2, P, P, None) == _lib.SK_EINVAL
    assert L.sinkhorn_features(P, 10, 2, P, 5000, 0.5, 2.0, 0, P, P, None) == _lib.SK_ENOTSUP
    # solve
    args = [P, 10, P, 12, 8, P, P, ctypes.byref(o), P, P, P, P, P, P, 1 << 20, None]
    bad = list(args); bad[0] = None
    assert L.sinkhorn_solve(*bad) == _lib.SK_EINVAL
    bad = list(args); bad[4] = 6
    assert L.sinkhorn_solve(*bad) == _lib.SK_ENOTSUP
    bad = list(args); bad[4] = 8192
    assert L.sinkhorn_solve(*bad) == _lib.SK_ENOTSUP
    o2 = _lib.sk_solve_opts(-1.0, 100, 0, 0, 0)
    bad = list(args); bad[7] = ctypes.byref(o2)
    assert L.sinkhorn_solve(*bad) == _lib.SK_EINVAL
    o3 = _lib.sk_solve_opts(1e-6, 0, 0, 0, 0)
    bad = list(args); bad[7] = ctypes.byref(o3)
    assert L.sinkhorn_solve(*bad) == _lib.SK_EINVAL
    o4 = _lib.sk_solve_opts(1e-6, 10, 0, 0, 7)   # unknown numeric domain
    bad = list(args); bad[7] = ctypes.byref(o4)
    assert L.sinkhorn_solve(*bad) == _lib.SK_EINVAL
    bad = list(args); bad[14] = 16   # workspace too small
    assert L.sinkhorn_solve(*bad) == _lib.SK_ENOMEM
    # divergence
    p = _problem()
    lay = _lib.sk_state_layout()
    assert L.sinkhorn_state_layout(10, 12, 8, ctypes.byref(lay)) == _lib.SK_OK
    ws = L.sinkhorn_divergence_workspace_size(ctypes.byref(p))
    assert ws > 0
    assert L.sinkhorn_divergence(ctypes.byref(p), ctypes.byref(o), P, P,
                                 lay.total - 1, P, ws, None) == _lib.SK_ENOMEM
    assert L.sinkhorn_divergence(ctypes.byref(p), ctypes.byref(o), P, P,
                                 lay.total, P, ws - 1, None) == _lib.SK_ENOMEM
    for field, val, code in (("eps", 0.0, _lib.SK_EINVAL), ("q", 0.5, _lib.SK_EINVAL),
                             ("r", 6, _lib.SK_ENOTSUP), ("n", 0, _lib.SK_EINVAL),
                             ("X", 0, _lib.SK_EINVAL)):
        pb = _problem()
        setattr(pb, field, val)
        assert L.sinkhorn_divergence(ctypes.byref(pb), ctypes.byref(o), P, P,
                                     lay.total, P, ws, None) == code, field
        assert L.sinkhorn_divergence_workspace_size(ctypes.byref(pb)) == 0
    # batched
    arr = (_lib.sk_problem * 2)(_problem(), _problem(n=0))
    assert L.sinkhorn_batched_workspace_size(arr, 2) == 0
    # backward
    assert L.sinkhorn_divergence_backward(ctypes.byref(p), None, None, P, P, P, P,
                                          P, 1 << 20, None) == _lib.SK_EINVAL
    assert L.sinkhorn_features_backward(P, 10, 2, P, 6, P, P, P, 1.0, 0, 0, P,
                                        None) == _lib.SK_ENOTSUP
    assert L.sinkhorn_features_backward(P, 10, 2, P, 8, P, P, P, 1.0, 0, 5, P,
                                        None) == _lib.SK_EINVAL


def test_state_layout_is_aligned_and_disjoint(L):
    n, m, r = 1037, 555, 100
    lay = _lib.sk_state_layout()
    assert L.sinkhorn_state_layout(n, m, r, ctypes.byref(lay)) == _lib.SK_OK
    pieces = [(lay.phix, 4 * n * r), (lay.phiy, 4 * m * r), (lay.sx, 4 * n),
              (lay.sy, 4 * m), (lay.info, 72), (lay.out, 32), (lay.meta, 16)]
    rows_u, rows_v = (n, n, m), (m, n, m)
    for k in range(3):   # pair layout [E | M]: 8 bytes per entry
        pieces += [(lay.u[k], 8 * rows_u[k]), (lay.v[k], 8 * rows_v[k]),
                   (lay.w[k], 8 * r), (lay.z[k], 8 * r)]
    pieces.sort()
    for (o1, s1), (o2, _) in zip(pieces, pieces[1:]):
        assert o1 % 256 == 0 and o1 + s1 <= o2
    assert pieces[-1][0] + pieces[-1][1] <= lay.total


def test_workspace_sizes_grow_with_the_problem(L):
    small = L.sinkhorn_solve_workspace_size(1000, 1000, 128)
    big = L.sinkhorn_solve_workspace_size(1_000_000, 1_000_000, 1024)
    assert 0 < small < big
    assert L.sinkhorn_solve_workspace_size(0, 10, 8) == 0
    # bounded by the slot buffer, not by n: no quadratic growth
    assert big < 64 * 2 ** 20


# ------------------------------------------------- anchors, assembly, arccos
@pytest.mark.parametrize("r,d,eps,sigma2", [(128, 2, 0.5, 1.0), (64, 16, 0.05, 0.3)])
def test_gaussian_anchors_with_given_variance(L, r, d, eps, sigma2):
    """sigma^2 given: U = float32(sqrt(sigma^2) Z) exactly as the seeded
    generator's own anchors, and q = 4 sigma^2 / eps (Lemma 1's relation)."""
    from paper_2006_07057_amd import inputs
    Z = inputs.standard_normal_anchors(3, r, d)
    U = np.empty((r, d), np.float32)
    q = ctypes.c_double()
    assert L.sinkhorn_gaussian_anchors(Z.ctypes.data, r, d, eps, sigma2, 0.0,
                                       U.ctypes.data, ctypes.byref(q)) == _lib.SK_OK
    assert np.array_equal(U, inputs.gaussian_anchors(3, r, d, sigma2))
    assert q.value == oracle.q_from_sigma2(sigma2, eps)


@pytest.mark.parametrize("R,eps,d", [(4.0, 0.1, 3), (30.0, 10.0, 784), (1.0, 1.0, 128)])
def test_gaussian_anchors_with_lambert_bandwidth(L, R, eps, d):
    """sigma^2 from Lemma 1's q for the ball of radius R: q matches the
    oracle's Lambert value and the anchors the oracle would draw from the
    same normals (within one float32 rounding: q may differ in its last
    bits between the two Lambert evaluations)."""
    from paper_2006_07057_amd import inputs
    r = 64
    Z = inputs.standard_normal_anchors(5, r, d)
    U = np.empty((r, d), np.float32)
    q = ctypes.c_double()
    assert L.sinkhorn_gaussian_anchors(Z.ctypes.data, r, d, eps, 0.0, R,
                                       U.ctypes.data, ctypes.byref(q)) == _lib.SK_OK
    qo = oracle.lambert_q(R, eps, d)
    assert q.value == pytest.approx(qo, rel=1e-13)
    Uo = inputs.gaussian_anchors(5, r, d, oracle.sigma2_from_q(qo, eps))
    np.testing.assert_allclose(U, Uo, rtol=2 ** -23, atol=0)


def test_new_entry_points_reject_bad_arguments(L):
    P = ctypes.c_void_p(0x1000)
    Z = np.zeros((4, 2))
    U = np.empty((4, 2), np.float32)
    q = ctypes.c_double()
    f = L.sinkhorn_gaussian_anchors
    assert f(None, 4, 2, 0.5, 1.0, 0.0, U.ctypes.data, ctypes.byref(q)) == _lib.SK_EINVAL
    assert f(Z.ctypes.data, 0, 2, 0.5, 1.0, 0.0, U.ctypes.data, ctypes.byref(q)) == _lib.SK_EINVAL
    assert f(Z.ctypes.data, 4, 2, 0.0, 1.0, 0.0, U.ctypes.data, ctypes.byref(q)) == _lib.SK_EINVAL
    assert f(Z.ctypes.data, 4, 2, 0.5, 0.0, 0.0, U.ctypes.data, ctypes.byref(q)) == _lib.SK_EINVAL
    assert f(Z.ctypes.data, 4, 2, 0.5, math.inf, 0.0, U.ctypes.data,
             ctypes.byref(q)) == _lib.SK_EINVAL
    assert L.sinkhorn_divergence_assemble(None, 1, P, None) == _lib.SK_EINVAL
    assert L.sinkhorn_divergence_assemble(P, 0, P, None) == _lib.SK_EINVAL
    assert L.sinkhorn_divergence_assemble(P, 1, None, None) == _lib.SK_EINVAL
    o = _lib.sk_solve_opts(1e-6, 100, 0, 0, _lib.SK_RANGE_LINEAR)
    p = _problem(r=7)                          # r + 1 = 8 columns
    ws = L.sinkhorn_divergence_arccos_workspace_size(ctypes.byref(p))
    assert ws > 0
    lay = _lib.sk_state_layout()
    assert L.sinkhorn_state_layout(10, 12, 8, ctypes.byref(lay)) == _lib.SK_OK
    g = L.sinkhorn_divergence_arccos
    assert g(ctypes.byref(_problem(r=8)), 1, 1.5, 0.5, ctypes.byref(o), P, P, lay.total,
             P, ws, None) == _lib.SK_ENOTSUP   # 9 columns
    assert g(ctypes.byref(p), 9, 1.5, 0.5, ctypes.byref(o), P, P, lay.total, P, ws,
             None) == _lib.SK_EINVAL
    assert g(ctypes.byref(p), 1, 1.0, 0.5, ctypes.byref(o), P, P, lay.total, P, ws,
             None) == _lib.SK_EINVAL
    assert g(ctypes.byref(p), 1, 1.5, 0.5, ctypes.byref(o), P, P, lay.total - 1, P, ws,
             None) == _lib.SK_ENOMEM
    assert g(ctypes.byref(p), 1, 1.5, 0.5, ctypes.byref(o), P, P, lay.total, P, ws - 1,
             None) == _lib.SK_ENOMEM
    ox = _lib.sk_solve_opts(1e-6, 100, 0, 0, _lib.SK_RANGE_EXTENDED)
    assert g(ctypes.byref(p), 1, 1.5, 0.5, ctypes.byref(ox), P, P, lay.total, P, ws,
             None) == _lib.SK_ENOTSUP
