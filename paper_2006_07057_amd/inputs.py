"""Seeded synthetic inputs for the point-cloud workloads.

This module only draws random numbers: point clouds, probability weights,
anchor draws and request schedules.  It holds none of the arithmetic of the
Sinkhorn method (no features, no kernel, no scalings), so both the GPU path
and the FP64 reference oracle can consume the very same arrays.

Every array handed to the device is float32 (the compute type of the GPU
path); the oracle upcasts the same float32 values to float64.

Workloads (shapes follow the experiments of Sec. 4 and App. C of the paper:
Gaussian clouds in R^2, mixtures in R^3, unit-normalised vectors and
pixel-like vectors for the mini-batch OT-GAN objective; the paper's own
datasets are not used and none of their items are reproduced):

* ``gauss2d``   - x ~ N(0, I_2), y ~ N(1.5*1, I_2), uniform weights.
* ``gmm3d``     - two 4-component Gaussian mixtures in R^3, component means
                  ~ U[-2, 2]^3 drawn independently per cloud, covariance
                  0.3*I, equal component probabilities, uniform weights.
* ``stream``    - Poisson request stream; per request n, m log-uniform,
                  d, r, eps from fixed menus, Dirichlet(1) weights,
                  x ~ N(0, I), y ~ N(mu, I) with mu ~ U[0, 1]^d.
* ``sphere``    - i.i.d. N(0, I_d) rows normalised to unit norm.
* ``pixels``    - i.i.d. U[0, 1]^d rows (pixel-like vectors).
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np

__all__ = [
    "Cloud", "Request",
    "gauss2d", "gmm3d", "sphere", "pixels",
    "gaussian_anchors", "standard_normal_anchors",
    "uniform_weights", "dirichlet_weights",
    "request_stream", "request_arrays", "pixel_batch_sizes",
    "max_norm", "max_norm_device", "counter_uniform", "pixels_counter", "pixel_batch",
]


@dataclasses.dataclass
class Cloud:
    """Two weighted point clouds: X (n, d), Y (m, d), weights a (n,), b (m,)."""
    X: np.ndarray
    Y: np.ndarray
    a: np.ndarray
    b: np.ndarray


def _f32(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float32))


def uniform_weights(n: int) -> np.ndarray:
    """Uniform probability vector 1/n in float32."""
    return np.full(n, 1.0 / n, dtype=np.float32)


def dirichlet_weights(rng: np.random.Generator, n: int) -> np.ndarray:
    """Dirichlet(1) probability vector (normalised in float64, stored float32)."""
    g = rng.standard_exponential(n)
    w = g / g.sum()
    w = np.maximum(w, 1e-30)          # keep every entry strictly positive
    return _f32(w)


def gauss2d(seed: int = 0, n: int = 1000, m: int = 1000, shift: float = 1.5,
            d: int = 2) -> Cloud:
    """x ~ N(0, I_d), y ~ N(shift*1, I_d), uniform weights."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, d))
    Y = rng.standard_normal((m, d)) + shift
    return Cloud(_f32(X), _f32(Y), uniform_weights(n), uniform_weights(m))


def _gmm(rng, n, d, k, cov):
    means = rng.uniform(-2.0, 2.0, size=(k, d))
    comp = rng.integers(0, k, size=n)
    return means[comp] + np.sqrt(cov) * rng.standard_normal((n, d))


def gmm3d(seed: int = 0, n: int = 1_000_000, m: int = 1_000_000, d: int = 3,
          k: int = 4, cov: float = 0.3) -> Cloud:
    """Two independent k-component Gaussian mixtures, uniform weights."""
    rng = np.random.default_rng(seed)
    X = _gmm(rng, n, d, k, cov)
    Y = _gmm(rng, m, d, k, cov)
    return Cloud(_f32(X), _f32(Y), uniform_weights(n), uniform_weights(m))


def sphere(seed: int = 0, n: int = 8192, m: int = 8192, d: int = 128) -> Cloud:
    """Unit-normalised Gaussian vectors in R^d, uniform weights."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, d))
    Y = rng.standard_normal((m, d))
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    Y /= np.linalg.norm(Y, axis=1, keepdims=True)
    return Cloud(_f32(X), _f32(Y), uniform_weights(n), uniform_weights(m))


def pixels(seed: int = 0, n: int = 4096, m: int = 4096, d: int = 784) -> Cloud:
    """Pixel-like vectors: i.i.d. U[0, 1]^d rows, uniform weights."""
    rng = np.random.default_rng(seed)
    X = rng.uniform(0.0, 1.0, size=(n, d))
    Y = rng.uniform(0.0, 1.0, size=(m, d))
    return Cloud(_f32(X), _f32(Y), uniform_weights(n), uniform_weights(m))


# ---------------------------------------------- counter-based pixel points
# Points of the mixed pixel batch (0.3 TB in all) are made where they are
# used: on the device for the GPU path, on the host for the oracle, from the
# same integer counter hash, so both sides get bit-identical arrays without
# moving them.  The hash is the 32-bit finaliser of MurmurHash3 (Appleby,
# public domain), applied twice; every product is kept below 2^48 so that
# int64 arithmetic (numpy or torch, host or device) is exact.
_M32 = 0xFFFFFFFF


def _mul32(h, c: int):
    """(h * c) mod 2^32 for 0 <= h < 2^32, through two 16-bit halves of c."""
    lo, hi = c & 0xFFFF, c >> 16
    return ((h * lo) + (((h * hi) & 0xFFFF) << 16)) & _M32


def _fmix32(h):
    h = h ^ (h >> 16)
    h = _mul32(h, 0x85EBCA6B)
    h = h ^ (h >> 13)
    h = _mul32(h, 0xC2B2AE35)
    return h ^ (h >> 16)


def _salt(key: int, cloud: int) -> int:
    import numpy as _np
    return int(_fmix32(_np.int64((2 * key + cloud) & _M32)))


def counter_uniform(key: int, cloud: int, rows: int, d: int, device=None,
                    block: int = 1 << 16):
    """rows x d float32 values in [0, 1): entry (i, j) is
    (h >> 8) 2^-24 with h = fmix32(fmix32((i d + j) xor s) + s mod 2^32) and
    s a salt of (key, cloud).  device None: a numpy array; else a torch
    tensor made on that device (blocks of `block` rows)."""
    if rows * d >= 1 << 32:
        raise ValueError("counter range exceeds 32 bits")
    s = _salt(key, cloud)
    if device is None:
        out = np.empty((rows, d), dtype=np.float32)
        for i0 in range(0, rows, block):
            i1 = min(rows, i0 + block)
            c = np.arange(i0 * d, i1 * d, dtype=np.int64)
            h = _fmix32((_fmix32(c ^ s) + s) & _M32)
            out[i0:i1] = ((h >> 8).astype(np.float32) * np.float32(2.0 ** -24)).reshape(i1 - i0, d)
        return out
    import torch
    out = torch.empty((rows, d), dtype=torch.float32, device=device)
    for i0 in range(0, rows, block):
        i1 = min(rows, i0 + block)
        c = torch.arange(i0 * d, i1 * d, dtype=torch.int64, device=device)
        h = _fmix32((_fmix32(c ^ s) + s) & _M32)
        out[i0:i1] = ((h >> 8).to(torch.float32) * (2.0 ** -24)).view(i1 - i0, d)
    return out


def pixels_counter(key: int, n: int, m: int, d: int = 784, device=None):
    """Pixel-like clouds X (n x d), Y (m x d) with entries in [0, 1) from
    counter_uniform (bit-identical on host and device) and uniform float32
    weights.  device None: numpy arrays; else torch tensors on it."""
    X = counter_uniform(key, 0, n, d, device)
    Y = counter_uniform(key, 1, m, d, device)
    if device is None:
        return Cloud(X, Y, uniform_weights(n), uniform_weights(m))
    import torch
    a = torch.full((n,), 1.0 / n, dtype=torch.float32, device=device)
    b = torch.full((m,), 1.0 / m, dtype=torch.float32, device=device)
    return Cloud(X, Y, a, b)


def pixel_batch(seed: int = 0, count: int = 256, lo: int = 2 ** 12, hi: int = 2 ** 20,
                r_menu=(512, 4096)):
    """The mixed pixel batch: per problem (index, n, m, r, key) with n, m
    log-uniform in [lo, hi], r uniform over r_menu (pixel_batch_sizes) and
    `key` seeding its points (pixels_counter) and anchor draws
    (standard_normal_anchors)."""
    sizes = pixel_batch_sizes(seed=seed, count=count, lo=lo, hi=hi, r_menu=r_menu)
    return [(i, n, m, r, 1000 + 1000 * seed + i) for i, (n, m, r) in enumerate(sizes)]


def max_norm_device(*tensors, rows: int = 1 << 16) -> float:
    """Largest Euclidean row norm over device point arrays, in float64
    (blocks of `rows` rows)."""
    best = 0.0
    for T in tensors:
        for i in range(0, T.shape[0], rows):
            blk = T[i:i + rows].double()
            best = max(best, float((blk * blk).sum(1).max().sqrt().item()))
    return best


def standard_normal_anchors(seed: int, r: int, d: int) -> np.ndarray:
    """r x d standard normal draws (float64), the raw randomness of the anchors."""
    rng = np.random.default_rng([seed, 0xA5C4])
    return rng.standard_normal((r, d))


def gaussian_anchors(seed: int, r: int, d: int, sigma2: float) -> np.ndarray:
    """Anchors u_1..u_r ~ N(0, sigma2 * I_d), i.i.d., float32 (r, d)."""
    return _f32(np.sqrt(sigma2) * standard_normal_anchors(seed, r, d))


def max_norm(*arrays: np.ndarray) -> float:
    """Largest Euclidean row norm over the given point arrays (float64)."""
    return float(max(np.sqrt((np.asarray(A, np.float64) ** 2).sum(1)).max()
                     for A in arrays))


# ---------------------------------------------------------------- serving
@dataclasses.dataclass
class Request:
    """One divergence request of the serving stream."""
    rid: int
    arrival: float      # seconds since stream start
    n: int
    m: int
    d: int
    r: int
    eps: float
    seed: int


def request_stream(seed: int = 0, count: int = 2048, rate: float = 500.0,
                   lo: int = 2 ** 10, hi: int = 2 ** 17,
                   d_menu=(2, 3, 16, 64), r_menu=(64, 256, 1024),
                   eps_menu=(0.05, 0.5, 5.0)) -> List[Request]:
    """Poisson arrivals (mean rate ``rate``/s); sizes log-uniform in [lo, hi]."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]
    ln = rng.uniform(np.log(lo), np.log(hi), size=count)
    lm = rng.uniform(np.log(lo), np.log(hi), size=count)
    ds = rng.choice(np.asarray(d_menu), size=count)
    rs = rng.choice(np.asarray(r_menu), size=count)
    es = rng.choice(np.asarray(eps_menu), size=count)
    seeds = rng.integers(0, 2 ** 31 - 1, size=count)
    out = []
    for i in range(count):
        out.append(Request(i, float(t[i]), int(round(np.exp(ln[i]))),
                           int(round(np.exp(lm[i]))), int(ds[i]), int(rs[i]),
                           float(es[i]), int(seeds[i])))
    return out


def request_arrays(req: Request) -> Cloud:
    """Materialise one request: x ~ N(0, I), y ~ N(mu, I), mu ~ U[0,1]^d,
    Dirichlet(1) weights."""
    rng = np.random.default_rng(req.seed)
    X = rng.standard_normal((req.n, req.d))
    mu = rng.uniform(0.0, 1.0, size=req.d)
    Y = rng.standard_normal((req.m, req.d)) + mu
    a = dirichlet_weights(rng, req.n)
    b = dirichlet_weights(rng, req.m)
    return Cloud(_f32(X), _f32(Y), a, b)


def pixel_batch_sizes(seed: int = 0, count: int = 256, lo: int = 2 ** 12,
                      hi: int = 2 ** 20, r_menu=(512, 4096)):
    """Sizes of the mixed pixel batch: (n, m, r) per problem, n and m drawn
    independently log-uniform in [lo, hi], r uniform over ``r_menu``."""
    rng = np.random.default_rng(seed)
    ln = rng.uniform(np.log(lo), np.log(hi), size=count)
    lm = rng.uniform(np.log(lo), np.log(hi), size=count)
    rs = rng.choice(np.asarray(r_menu), size=count)
    return [(int(round(np.exp(x))), int(round(np.exp(y))), int(z))
            for x, y, z in zip(ln, lm, rs)]
