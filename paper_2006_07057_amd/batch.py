"""Batches of divergences larger than device memory, run in waves.

The mini-batch objective of Sec. 4 averages many independent divergence
terms; the paper computes them in batches "because of memory limitation on
GPUs".  A batch whose features alone exceed HBM (the 256 pixel-like
problems with n, m up to 2^20 and r = 4096 hold about 0.9 TB of features)
is split into waves: each wave is a set of problems whose device footprint
(inputs, the state of ``sinkhorn_state_layout``, the gradient output and a
share of the solver workspace) fits the HBM budget.  A wave's inputs are
made on the device, its divergences run in one ``sinkhorn_divergence_batched``
call (packed persistent launches, one per feature-count class), its
gradients with respect to X in one backward call per problem, and its memory
is released before the next wave.

The planning is host code; every arithmetic step of the method runs in the
library's kernels.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional, Sequence

import torch

from . import api


@dataclasses.dataclass
class BatchProblem:
    """Sizes of one problem of a batch (its inputs are made by the caller's
    `make` callback when its wave runs)."""
    index: int
    n: int
    m: int
    d: int
    r: int


def footprint_bytes(n: int, m: int, d: int, r: int, grad_x: bool = True) -> int:
    """Device bytes one problem holds while its wave runs."""
    L = api.state_layout(n, m, r)
    inputs = 4 * (n * d + m * d + n + m + r * d)
    grads = 4 * n * d if grad_x else 0
    work = 8 * (max(n, m) + r) * 3 + 4096          # second v, w buffers per solve
    return int(L.total) + inputs + grads + work


def plan_waves(footprints: Sequence[int], budget: int) -> List[List[int]]:
    """First-fit decreasing: problems sorted by footprint (largest first)
    go into the first wave with room.  Returns waves as lists of problem
    indices (each wave in ascending index order).  A problem larger than
    the whole budget cannot run and raises."""
    order = sorted(range(len(footprints)), key=lambda i: (-footprints[i], i))
    waves: List[List[int]] = []
    room: List[int] = []
    for i in order:
        f = int(footprints[i])
        if f > budget:
            raise ValueError(f"problem {i} needs {f} bytes, above the budget {budget}")
        for w in range(len(waves)):
            if f <= room[w]:
                waves[w].append(i)
                room[w] -= f
                break
        else:
            waves.append([i])
            room.append(budget - f)
    return [sorted(w) for w in waves]


@dataclasses.dataclass
class WaveResult:
    wave: int
    indices: List[int]
    out: torch.Tensor            # (count, 4) float64 on the device
    states: list                 # api.DivergenceState per problem
    grads: List[Optional[torch.Tensor]]   # dX per problem (or None)
    ms: float                    # device time of the wave's compute


def run_waves(problems: Sequence[BatchProblem], make: Callable, budget: int,
              tol: float = 1e-6, max_iter: int = 2000, fixed_iter: int = 0,
              grad_x: bool = True, on_wave: Optional[Callable[[WaveResult], None]] = None,
              device: str = "cuda:0") -> List[List[int]]:
    """Run every problem of the batch, wave by wave, within `budget` device
    bytes.  make(problem) -> (X, Y, a, b, U, eps, q) device tensors and
    floats for that problem (called when its wave starts, outside the timed
    region).  on_wave(result) receives each wave's results (W_bar and the
    three estimates per problem, states, dX) before its memory is released.
    The compute of a wave (features, solves, reductions, gradients) is timed
    with events on the launch stream; its buffers (states, workspace,
    outputs) are allocated before the timed region.  Returns the wave plan."""
    dev = torch.device(device)
    foot = [footprint_bytes(p.n, p.m, p.d, p.r, grad_x) for p in problems]
    # the packed launches' partial r-vectors and descriptors are shared by
    # the wave: keep 256 MiB of the budget for them
    waves = plan_waves(foot, budget - (256 << 20))
    ws = None
    for w, idx in enumerate(waves):
        probs = [make(problems[i]) for i in idx]
        states = api.batched_states(probs)
        need = api.batched_workspace_bytes(states)
        if ws is None or ws.numel() < need:
            ws = None
            ws = torch.empty(need, dtype=torch.uint8, device=dev)
        out = torch.empty((len(idx), 4), dtype=torch.float64, device=dev)
        gbuf = [torch.empty_like(st.X) if grad_x else None for st in states]
        stream = torch.cuda.current_stream(dev)
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        out, states = api.divergence_batched(probs, tol=tol, max_iter=max_iter,
                                             fixed_iter=fixed_iter, workspace=ws,
                                             states=states, out=out)
        grads = [api.divergence_backward(st, need=(True, False, False, False),
                                         out=(gb, None, None, None))[0]
                 if grad_x else None for st, gb in zip(states, gbuf)]
        t1.record(stream)
        t1.synchronize()
        res = WaveResult(w, list(idx), out, states, grads, t0.elapsed_time(t1))
        if on_wave is not None:
            on_wave(res)
        del probs, out, states, grads, gbuf, res
    return waves
