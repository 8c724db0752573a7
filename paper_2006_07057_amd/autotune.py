"""Autotuner for the persistent solver's launch plan and lane layouts.

Two choices per solver class (feature-count class, indexed by its largest
r) are tuned, both entries of the library's tuning table:

* the lane layout (``sinkhorn_solver_layouts`` / ``sinkhorn_tune_set_layout``):
  G lanes per feature row, C float4 chunks per lane, U rows per batch and
  the occupancy W the kernels were compiled for; and
* the target (``sinkhorn_tune_set``): the feature bytes each workgroup
  streams per half-step, which sets the gang size
  g = ceil(max(n, m) * r * 4 / target).  More workgroups mean more memory
  parallelism but costlier grid barriers and more partial vectors.

Candidates are timed on the device with the library's own launch events,
on problems with the workload's own shapes and generators (``tune_class``
takes the shape and the generator kind), the fastest pair is installed, and
the table is stored as JSON so later processes load it without
re-measuring.  Only the grouping of sums changes between candidates: every
layout and target computes the same iteration, so results differ by float32
rounding only.
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


def _problem(n: int, m: int, r: int, d: int, eps: float, seed: int, rng: int, dev,
             kind: str = "gauss2d"):
    """Features of one synthetic problem of the given shape.  kind: the
    workload generator (gauss2d: N(0, I) against a shifted N, any d;
    pixels: the pixel batch's counter-based U[0, 1)^d points)."""
    if kind == "pixels":
        c = inputs.pixels_counter(1000 + seed, n, m, d, device=dev)
        R = inputs.max_norm_device(c.X, c.Y)
        X, Y, a, b = c.X, c.Y, c.a, c.b
    else:
        h = inputs.gauss2d(seed, n=n, m=m, d=d)
        R = inputs.max_norm(h.X, h.Y)
        t = lambda x: torch.from_numpy(x).to(dev)
        X, Y, a, b = t(h.X), t(h.Y), t(h.a), t(h.b)
    # anchors with Lemma 1's bandwidth for these points (valid for every
    # eps and d)
    U, q = api.gaussian_anchors(inputs.standard_normal_anchors(seed, r, d), eps, R=R)
    Ud = torch.from_numpy(U).to(dev)
    Px, _ = api.features(X, Ud, eps, q, range=rng)
    Py, _ = api.features(Y, Ud, eps, q, range=rng)
    return Px, Py, a, b


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
               device: str = "cuda:0", kind: str = "gauss2d",
               layouts: Optional[Sequence[int]] = None) -> Dict[tuple, float]:
    """Time every (layout variant, target) pair for the class serving r on a
    synthetic problem of shape (n, m, r) from generator `kind`, install the
    fastest, and return {(variant, target): ms per launch}."""
    m = n if m is None else m
    dev = torch.device(device)
    Px, Py, a, b = _problem(n, m, r, d, eps, seed, rng, dev, kind)
    variants = range(len(api.solver_layouts(r))) if layouts is None else layouts
    times = {}
    for v in variants:
        api.tune_set_layout(r, int(v))
        for tgt in candidates:
            api.tune_set(r, int(tgt))
            times[(int(v), int(tgt))] = time_solve(Px, Py, a, b, iters, reps, rng)
    best = min(times, key=times.get)
    api.tune_set_layout(r, best[0])
    api.tune_set(r, best[1])
    return times


def tune(shapes: Iterable[tuple], **kw) -> Dict[int, tuple]:
    """Tune each class once on the given shapes ((n, m, r) tuples; the
    first shape seen for a class is used).  Returns {class rmax: (layout,
    target)}."""
    table = {}
    for (n, m, r) in shapes:
        c = class_of(r)
        if c in table:
            continue
        times = tune_class(r, n, m, **kw)
        table[c] = min(times, key=times.get)
    return table


def current_table() -> Dict[int, tuple]:
    """{class rmax: (layout variant, target bytes)} as installed."""
    return {c: (api.tune_get_layout(c), api.tune_get(c)) for c in CLASS_RMAX}


def save(path: str, table: Optional[Dict[int, tuple]] = None, notes=None) -> None:
    table = current_table() if table is None else table
    doc = {"device": torch.cuda.get_device_name(0) if torch.cuda.is_available() else None,
           "targets": {str(k): int(v[1]) for k, v in sorted(table.items())},
           "layouts": {str(k): int(v[0]) for k, v in sorted(table.items())}}
    if notes is not None:
        doc["notes"] = notes
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(doc, f, indent=1)
    os.replace(tmp, path)


def load(path: str) -> Dict[int, tuple]:
    """Install a stored table (host-only: no device work).  Tables written
    before layouts were tuned hold targets only (layout 0)."""
    with open(path) as f:
        doc = json.load(f)
    targets = {int(k): int(v) for k, v in doc["targets"].items()}
    layouts = {int(k): int(v) for k, v in doc.get("layouts", {}).items()}
    table = {}
    for c, tgt in targets.items():
        lay = layouts.get(c, 0)
        if c not in CLASS_RMAX or tgt < 0 or not 0 <= lay < len(api.solver_layouts(c)):
            raise ValueError(f"bad tuning entry {c}: target {tgt}, layout {lay}")
        api.tune_set(c, tgt)
        api.tune_set_layout(c, lay)
        table[c] = (lay, tgt)
    return table


def reset() -> None:
    for c in CLASS_RMAX:
        api.tune_set(c, 0)
        api.tune_set_layout(c, 0)
