"""Autotuner for the persistent solver's launch planning.

The solver splits each solve's rows over g workgroups with
g = ceil(max(n, m) * r * 4 / target), where ``target`` (feature bytes each
workgroup streams per half-step) is a per-class entry of the library's
tuning table (``sinkhorn_tune_set``).  More workgroups mean more memory
parallelism but a costlier grid barrier (every half-step ends with two) and
more partial vectors to reduce; the best target depends on the class's lane
layout and on the problem sizes served.  This module measures candidate
targets on the device with the library's own launch timing, installs the
fastest, and stores the table as JSON so later processes can load it
without re-measuring.

Only launch planning is tuned: the arithmetic of each solve is the same
for every target (partial sums are only grouped differently, which changes
results by float32 rounding).
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, Iterable, Optional, Sequence

import numpy as np
import torch

from . import api, inputs

DEFAULT_CANDIDATES = (32 << 10, 64 << 10, 128 << 10, 256 << 10, 512 << 10,
                      1 << 20, 4 << 20, 16 << 20)
CLASS_RMAX = (4, 8, 16, 32, 64, 128, 256, 512, 768, 1024, 1536, 2048, 3072, 4096)


def class_of(r: int) -> int:
    for c in CLASS_RMAX:
        if r <= c:
            return c
    raise ValueError(f"r={r} exceeds the largest solver class")


def _problem(n: int, m: int, r: int, d: int, eps: float, seed: int, rng: int, dev):
    c = inputs.gauss2d(seed, n=n, m=m, d=d)
    # anchors with Lemma 1's bandwidth for these points (valid for every
    # eps and d)
    U, q = api.gaussian_anchors(inputs.standard_normal_anchors(seed, r, d), eps,
                                R=inputs.max_norm(c.X, c.Y))
    t = lambda x: torch.from_numpy(x).to(dev)
    Px, _ = api.features(t(c.X), t(U), eps, q, range=rng)
    Py, _ = api.features(t(c.Y), t(U), eps, q, range=rng)
    return Px, Py, t(c.a), t(c.b)


def time_solve(Px, Py, a, b, iters: int, reps: int, rng: int) -> float:
    """Best-of-reps duration (ms) of one solver launch of `iters` fixed
    iterations, timed by the library's events on the launch stream."""
    best = math.inf
    ws = None
    for _ in range(reps):
        api.profile(True)
        out = api.solve(Px, Py, a, b, fixed_iter=iters, range=rng, workspace=ws)
        torch.cuda.synchronize()
        ms, cnt, _ = api.profile_read(api.PROF_SOLVER)
        api.profile(False)
        best = min(best, ms / max(cnt, 1))
    return best


def tune_class(r: int, n: int, m: Optional[int] = None, d: int = 3, eps: float = 0.5,
               candidates: Sequence[int] = DEFAULT_CANDIDATES, iters: int = 20,
               reps: int = 2, rng: int = api.EXTENDED, seed: int = 0,
               device: str = "cuda:0") -> Dict[int, float]:
    """Time every candidate target for the class serving r on a synthetic
    problem of shape (n, m, r), install the fastest, and return
    {target: ms per launch}."""
    m = n if m is None else m
    dev = torch.device(device)
    Px, Py, a, b = _problem(n, m, r, d, eps, seed, rng, dev)
    times = {}
    for tgt in candidates:
        api.tune_set(r, int(tgt))
        times[int(tgt)] = time_solve(Px, Py, a, b, iters, reps, rng)
    best = min(times, key=times.get)
    api.tune_set(r, best)
    return times


def tune(shapes: Iterable[tuple], **kw) -> Dict[int, int]:
    """Tune each class once on the given shapes ((n, m, r) tuples; the
    first shape seen for a class is used).  Returns {class rmax: target}."""
    table = {}
    for (n, m, r) in shapes:
        c = class_of(r)
        if c in table:
            continue
        times = tune_class(r, n, m, **kw)
        table[c] = min(times, key=times.get)
    return table


def current_table() -> Dict[int, int]:
    return {c: api.tune_get(c) for c in CLASS_RMAX}


def save(path: str, table: Optional[Dict[int, int]] = None) -> None:
    table = current_table() if table is None else table
    doc = {"device": torch.cuda.get_device_name(0) if torch.cuda.is_available() else None,
           "targets": {str(k): int(v) for k, v in sorted(table.items())}}
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(doc, f, indent=1)
    os.replace(tmp, path)


def load(path: str) -> Dict[int, int]:
    """Install a stored table (host-only: no device work)."""
    with open(path) as f:
        doc = json.load(f)
    table = {int(k): int(v) for k, v in doc["targets"].items()}
    for c, tgt in table.items():
        if c not in CLASS_RMAX or tgt < 0:
            raise ValueError(f"bad tuning entry {c}: {tgt}")
        api.tune_set(c, tgt)
    return table


def reset() -> None:
    for c in CLASS_RMAX:
        api.tune_set(c, 0)
