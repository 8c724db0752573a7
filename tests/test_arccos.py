"""Perturbed arc-cosine features (Sec. 3.2 and the decomposition lemma of the
appendix): argument checks on the host, and parity of the HIP feature map
and of a divergence built on it with the oracle."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2006_07057_amd import _lib, inputs
from parity import check_divergence


def test_arccos_argument_errors():
    L = _lib.lib()
    P = ctypes.c_void_p(0x1000)
    f = L.sinkhorn_features_arccos
    assert f(None, 10, 3, P, 7, 1, 1.5, 0.5, P, P, None) == _lib.SK_EINVAL
    assert f(P, 10, 3, P, 7, -1, 1.5, 0.5, P, P, None) == _lib.SK_EINVAL
    assert f(P, 10, 3, P, 7, 1, 1.0, 0.5, P, P, None) == _lib.SK_EINVAL   # sigma <= 1
    assert f(P, 10, 3, P, 7, 1, 1.5, 0.0, P, P, None) == _lib.SK_EINVAL   # kappa <= 0
    assert f(P, 10, 3, P, 4096, 1, 1.5, 0.5, P, P, None) == _lib.SK_ENOTSUP


def _data(seed, n, m, d, r, sigma):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, d)).astype(np.float32)
    Y = (rng.standard_normal((m, d)) + 0.5).astype(np.float32)
    U = (sigma * rng.standard_normal((r, d))).astype(np.float32)
    return X, Y, U


@pytest.mark.gpu
@pytest.mark.parametrize("s", [0, 1, 2])
@pytest.mark.parametrize("d,r", [(3, 127), (16, 255), (2, 1023),
                                 # per-row kernel reading anchors from global
                                 # memory (d (r + 1) > 12288 floats of staging)
                                 (7, 2047),
                                 # matrix-core projections (d >= 8, d % 4 == 0):
                                 # r + 1 = 101 columns (unaligned rows), pixel width,
                                 # 16 column blocks
                                 (36, 100), (784, 127), (128, 1023)])
def test_arccos_features_match_oracle(s, d, r):
    import torch
    from paper_2006_07057_amd import api
    sigma, kappa = 1.5, 0.5
    X, _, U = _data(s + d, 300, 10, d, r, sigma)
    Phi, ls = api.features_arccos(torch.from_numpy(X).cuda(), torch.from_numpy(U).cuda(),
                                  s, sigma, kappa)
    Pg, lg = Phi.cpu().numpy().astype(np.float64), ls.cpu().numpy().astype(np.float64)
    Po, lo = oracle.arccos_features_scaled(X, U, s, sigma, kappa)
    assert Pg.shape == (300, r + 1)
    # Per-element float32 bound on log phi: the projection u.x is a float32
    # dot product of d terms (relative error <= (d + 2) 2^-24 sum|x_e u_e| /
    # |u.x|, times s for the power), plus the roundings of the constant,
    # the logarithm and the row maximum.  Projections within that error of
    # zero may land on either side of the rectifier.
    U64, X64 = U.astype(np.float64), X.astype(np.float64)
    proj = X64 @ U64.T
    scale = np.abs(X64) @ np.abs(U64).T
    u = 2.0 ** -24
    Lo = oracle.arccos_log_features(X, U, s, sigma, kappa)
    cond = np.zeros_like(Po)
    with np.errstate(divide="ignore", invalid="ignore"):
        cond[:, :r] = np.where(np.abs(proj) > 0, s * (d + 2) * u * scale / np.abs(proj), np.inf)
    tol_el = 8 * (cond + u * (np.abs(np.where(np.isfinite(Lo), Lo, 0)) + 10))
    amax = Lo.argmax(1)
    tol_row = tol_el[np.arange(len(amax)), amax][:, None]
    ambiguous = np.zeros_like(Po, dtype=bool)
    ambiguous[:, :r] = np.abs(proj) <= 8 * (d + 2) * u * scale
    ok = ~ambiguous
    bound = (tol_el + tol_row) * np.maximum(Po, 0.0)
    assert np.all(np.abs(Pg - Po)[ok] <= bound[ok] + 1e-30)
    assert np.all(np.abs(lg - lo) <= tol_row[:, 0] * (1 + np.abs(lo)))
    assert np.all(Pg[:, :r][(Po[:, :r] == 0) & ok[:, :r]] == 0.0)
    assert np.all(Pg[:, r] > 0)


@pytest.mark.gpu
@pytest.mark.parametrize("s", [1, 2])
@pytest.mark.parametrize("d", [3, 16])
def test_arccos_divergence_matches_oracle(s, d):
    import torch
    from paper_2006_07057_amd import api
    sigma, kappa, eps = 1.4, 0.5, 0.5
    n, m, r = 300, 260, 127
    X, Y, U = _data(10 + s, n, m, d, r, sigma)
    rng = np.random.default_rng(3)
    a = inputs.dirichlet_weights(rng, n)
    b = inputs.dirichlet_weights(rng, m)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    w_bar, infos = api.divergence_arccos(t(X), t(Y), t(a), t(b), t(U), s, sigma, kappa, eps,
                                         fixed_iter=200)
    Px, sx = oracle.arccos_features_scaled(X, U, s, sigma, kappa)
    Py, sy = oracle.arccos_features_scaled(Y, U, s, sigma, kappa)
    ws = []
    for (P, Q, p, g, sp, sq) in ((Px, Py, a, b, sx, sy), (Px, Px, a, a, sx, sx),
                                 (Py, Py, b, b, sy, sy)):
        res = oracle.sinkhorn_factored(P, Q, p, g, fixed_iter=200)
        ws.append(oracle.w_hat_scaled(res.u, res.v, p, g, sp, sq, eps))
    ref = ws[0] - 0.5 * (ws[1] + ws[2])
    assert list(infos["status"]) == [0, 0, 0]
    check_divergence(f"arccos divergence s={s} d={d}",
                     [w_bar] + [infos["w_hat"][k] for k in range(3)],
                     (ref, ws[0], ws[1], ws[2]))
