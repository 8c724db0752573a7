"""Serving loop for divergence requests on one GPU: admission by HBM budget
and continuous batching.

A request is one debiased divergence (three runs of Algorithm 1: (X, Y),
(X, X), (Y, Y)).  The server keeps every admitted request resident in device
memory (inputs, features, scalings and r-vectors in one state buffer laid
out by ``sinkhorn_state_layout``) and advances all live solves together in
*epochs*: one call of ``sinkhorn_solve_batched`` packs every unfinished solve
of every live request into persistent launches and runs at most
``epoch_iters`` iterations of each, continuing from the scaling the previous
epoch left in its u buffer (warm start).  Between epochs, converged solves
retire, finished requests free their memory, and requests that arrived
meanwhile are admitted as the HBM budget allows, so new work joins work
already on the device instead of waiting for it to drain.

Continuing Algorithm 1 from u^(K) produces the same iterates as an
uninterrupted run (up to rounding), and the stopping test is evaluated after
every iteration in both cases, so a request's result is the one it would get
alone.  The iteration cap is applied at epoch granularity (rounded up to a
multiple of ``epoch_iters``).

The scheduling logic is host code; every arithmetic step of the method runs
in the library's kernels.
"""
from __future__ import annotations

import collections
import ctypes
import dataclasses
import math
import time
from typing import Callable, Deque, List, Optional, Sequence

import numpy as np
import torch

from . import api
from ._lib import (lib, check, SK_OK, SK_ENOMEM, SK_ENOTCONV, SK_RANGE_EXTENDED)

_SOLVE_NAMES = ("xy", "xx", "yy")


@dataclasses.dataclass
class Request:
    """One divergence request (host arrays; float32 points, weights and
    anchors).  ``arrival`` is in seconds from the start of a run."""
    X: np.ndarray
    Y: np.ndarray
    a: np.ndarray
    b: np.ndarray
    U: np.ndarray
    eps: float
    q: float
    arrival: float = 0.0
    rid: int = -1


@dataclasses.dataclass
class Result:
    rid: int
    status: int
    w_bar: float
    w_hat: tuple
    iters: tuple
    arrival: float
    admitted: float
    finished: float
    epochs: int

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def from_spec(spec, sigma2: Optional[float] = None) -> Request:
    """Materialise a synthetic request description (``inputs.Request``):
    points and weights from its seed, and anchors of Lemma 1 from the
    request's standard normal draws through sinkhorn_gaussian_anchors (q
    from the Lambert rule with R = largest norm over both clouds, unless
    sigma2 is given)."""
    from . import inputs
    cloud = inputs.request_arrays(spec)
    Z = inputs.standard_normal_anchors(spec.seed, spec.r, spec.d)
    if sigma2 is None:
        U, q = api.gaussian_anchors(Z, spec.eps, R=inputs.max_norm(cloud.X, cloud.Y))
    else:
        U, q = api.gaussian_anchors(Z, spec.eps, sigma2=sigma2)
    return Request(cloud.X, cloud.Y, cloud.a, cloud.b, U, spec.eps, q,
                   arrival=spec.arrival, rid=spec.rid)


def footprint_bytes(n: int, m: int, d: int, r: int) -> int:
    """Device bytes a request holds while live: its state buffer, its inputs
    and its share of the solver workspace (second v and w buffers)."""
    L = api.state_layout(n, m, r)
    inputs = 4 * (n * d + m * d + n + m + r * d)
    work = 3 * (8 * max(n, m) + 8 * r + 1024)
    return int(L.total) + inputs + work


def plan_admission(footprints: Sequence[int], live_bytes: int, live_count: int,
                   budget: int, reserve: int) -> List[str]:
    """First-come-first-served admission by device-memory budget.  Walks the
    queue (footprints in arrival order) and returns a decision for its
    leading requests: "admit" while the request fits next to what is live,
    "reject" for a request that cannot fit even on an empty device; stops at
    the first request that must wait for memory to free up."""
    out: List[str] = []
    for f in footprints:
        if live_bytes + f + reserve <= budget:
            out.append("admit")
            live_bytes += f
            live_count += 1
        elif live_count == 0:
            out.append("reject")
        else:
            break
    return out


class _Live:
    def __init__(self, req: Request, dev, rng: int, now: float):
        self.req = req
        n, d = req.X.shape
        m = req.Y.shape[0]
        r = req.U.shape[0]
        self.n, self.m, self.d, self.r = n, m, d, r
        t = lambda x: torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(dev)
        self.X, self.Y, self.a, self.b, self.U = t(req.X), t(req.Y), t(req.a), t(req.b), t(req.U)
        self.layout = api.state_layout(n, m, r)
        self.buf = torch.empty(self.layout.total, dtype=torch.uint8, device=dev)
        self.bytes = footprint_bytes(n, m, d, r)
        self.done = [False, False, False]
        self.iters = [0, 0, 0]
        self.status = SK_OK
        self.admitted = now
        self.epochs = 0
        L = self.layout
        stream = api._stream(dev)
        for (P, s, pts, cnt) in ((L.phix, L.sx, self.X, n), (L.phiy, L.sy, self.Y, m)):
            check(lib().sinkhorn_features(
                api._ptr(pts), cnt, d, api._ptr(self.U), r, float(req.eps),
                float(req.q), int(rng), ctypes.c_void_p(self.buf.data_ptr() + P),
                ctypes.c_void_p(self.buf.data_ptr() + s), stream), "sinkhorn_features")
        # u^(0) = 1 for the three solves (then every epoch warm-starts)
        for k in range(3):
            rows = (n, n, m)[k]
            u = self._f32(L.u[k], 2 * rows)
            if rng == SK_RANGE_EXTENDED:
                u[:rows].zero_()
                u[rows:].fill_(1.0)
            else:
                u[:rows].fill_(1.0)

    def _f32(self, off, count):
        return self.buf[off:off + 4 * count].view(torch.float32)

    def keep_record(self, k: int, rec: torch.Tensor):
        """Store solve k's final device record in the state (device copy)."""
        o = self.layout.info + k * api.INFO_BYTES
        self.buf[o:o + api.INFO_BYTES].copy_(rec)

    def assemble(self):
        """W_bar and the three estimates into the state's out block, on the
        device (sinkhorn_divergence_assemble); returns that float64 view."""
        L = self.layout
        out = self.buf[L.out:L.out + 32].view(torch.float64).view(1, 4)
        api.divergence_assemble(self.buf[L.info:L.info + 3 * api.INFO_BYTES], 1, out)
        return out

    def spec(self, k: int, info_ptr: int):
        L, n, m, r = self.layout, self.n, self.m, self.r
        base = self.buf.data_ptr()
        rows = (L.phix, L.phix, L.phiy)[k]
        cols = (L.phiy, L.phix, L.phiy)[k]
        srow = (L.sx, L.sx, L.sy)[k]
        scol = (L.sy, L.sx, L.sy)[k]
        wa = (self.a, self.a, self.b)[k]
        wb = (self.b, self.a, self.b)[k]
        nr = (n, n, m)[k]
        nc = (m, n, m)[k]
        return api.sk_solve_spec(base + rows, base + cols, wa.data_ptr(), wb.data_ptr(),
                                 base + srow, base + scol, base + L.u[k], base + L.v[k],
                                 base + L.w[k], base + L.z[k], info_ptr, nr, nc, r,
                                 float(self.req.eps))


class Server:
    """Continuous-batching divergence server (see the module docstring).

    hbm_budget   device bytes the live requests may hold (default: half of
                 the free device memory when the server starts);
    epoch_iters  iterations each live solve advances per packed launch;
    tol, max_iter, range  as for ``api.divergence``.
    """

    def __init__(self, hbm_budget: Optional[int] = None, epoch_iters: int = 50,
                 tol: float = 1e-6, max_iter: int = 2000, range: int = api.EXTENDED,
                 device: str = "cuda:0", clock: Callable[[], float] = time.perf_counter):
        self.dev = torch.device(device)
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info(self.dev)
            hbm_budget = free // 2
        self.budget = int(hbm_budget)
        self.reserve = 80 << 20  # per-launch partial slots and descriptors
        self.epoch_iters = int(epoch_iters)
        self.tol, self.max_iter, self.range = float(tol), int(max_iter), int(range)
        self.clock = clock
        self.t0 = clock()
        self.queue: Deque[Request] = collections.deque()
        self.live: List[_Live] = []
        self.live_bytes = 0
        self.workspace: Optional[torch.Tensor] = None
        self.results: List[Result] = []
        self.epoch_log: List[dict] = []
        self._next_id = 0

    # ---------------------------------------------------------- requests
    def now(self) -> float:
        return self.clock() - self.t0

    def submit(self, req: Request) -> int:
        if req.rid < 0:
            req.rid = self._next_id
        self._next_id = max(self._next_id, req.rid + 1)
        self.queue.append(req)
        return req.rid

    def busy(self) -> bool:
        return bool(self.queue) or bool(self.live)

    # ---------------------------------------------------------- admission
    def _admit(self) -> List[int]:
        foot = [footprint_bytes(q.X.shape[0], q.Y.shape[0], q.X.shape[1], q.U.shape[0])
                for q in self.queue]
        plan = plan_admission(foot, self.live_bytes, len(self.live), self.budget,
                              self.reserve)
        admitted = []
        for decision in plan:
            req = self.queue.popleft()
            t = self.now()
            if decision == "admit":
                lv = _Live(req, self.dev, self.range, t)
                self.live.append(lv)
                self.live_bytes += lv.bytes
                admitted.append(req.rid)
            else:
                self.results.append(Result(req.rid, SK_ENOMEM, math.nan, (math.nan,) * 3,
                                           (0, 0, 0), req.arrival, t, t, 0))
        return admitted

    # ---------------------------------------------------------- one epoch
    def step(self) -> List[Result]:
        """Admit what fits, advance every live solve by one epoch, retire
        finished requests.  Returns the requests finished in this epoch."""
        admitted = self._admit()
        if not self.live:
            return []
        live_ids = [lv.req.rid for lv in self.live]
        bytes_in_use = self.live_bytes
        jobs = [(lv, k) for lv in self.live for k in range(3) if not lv.done[k]]
        infos = torch.zeros(api.INFO_BYTES * len(jobs), dtype=torch.uint8, device=self.dev)
        base = infos.data_ptr()
        specs = [lv.spec(k, base + j * api.INFO_BYTES) for j, (lv, k) in enumerate(jobs)]
        self.workspace = api.solve_batched(specs, tol=self.tol, max_iter=self.epoch_iters,
                                           warm_start=True, range=self.range,
                                           workspace=self.workspace, device=self.dev)
        rec = api.parse_infos(infos)  # synchronises
        for j, (lv, k) in enumerate(jobs):
            it, st = int(rec["iters"][j]), int(rec["status"][j])
            lv.iters[k] += it
            if st == SK_OK:
                lv.done[k] = True
            elif st == SK_ENOTCONV:
                if lv.iters[k] >= self.max_iter:
                    lv.done[k] = True
                    lv.status = SK_ENOTCONV
            else:
                lv.done[k] = True
                lv.status = st
            if lv.done[k]:
                lv.keep_record(k, infos[j * api.INFO_BYTES:(j + 1) * api.INFO_BYTES])
        for lv in self.live:
            lv.epochs += 1
        t = self.now()
        keep, done = [], []
        for lv in self.live:
            (done if all(lv.done) else keep).append(lv)
        finished = []
        if done:
            # W_bar of every finished request assembled on the device, read
            # back in one transfer
            vals = torch.cat([lv.assemble() for lv in done]).cpu().numpy()
            for lv, v in zip(done, vals):
                finished.append(Result(lv.req.rid, lv.status, float(v[0]),
                                       tuple(float(x) for x in v[1:]), tuple(lv.iters),
                                       lv.req.arrival, lv.admitted, t, lv.epochs))
                self.live_bytes -= lv.bytes
        self.live = keep
        self.results.extend(finished)
        self.epoch_log.append({"t": t, "solves": len(jobs), "admitted": admitted,
                               "finished": [r.rid for r in finished],
                               "live": live_ids, "bytes": bytes_in_use})
        return finished

    # ---------------------------------------------------------- replay
    def run(self, requests: Sequence[Request], idle_sleep: float = 2e-4,
            progress: Optional[Callable[["Server"], None]] = None) -> List[Result]:
        """Replay requests at their arrival times (seconds from now) and serve
        them until all are done.  Returns the results in completion order.
        ``progress`` is called after every epoch."""
        pending = collections.deque(sorted(requests, key=lambda q: q.arrival))
        self.t0 = self.clock()
        start = len(self.results)
        while pending or self.busy():
            now = self.now()
            while pending and pending[0].arrival <= now:
                self.submit(pending.popleft())
            if self.busy():
                self.step()
                if progress is not None:
                    progress(self)
            elif pending:
                time.sleep(min(idle_sleep, max(0.0, pending[0].arrival - now)))
        return self.results[start:]


def latency_stats(results: Sequence[Result]) -> dict:
    """Throughput and latency percentiles (arrival to result) of a run."""
    ok = [r for r in results if r.status == SK_OK]
    lat = np.array([r.latency for r in ok]) if ok else np.zeros(0)
    span = (max(r.finished for r in results) - min(r.arrival for r in results)
            if results else 0.0)
    return {
        "requests": len(results),
        "ok": len(ok),
        "failed": {int(s): sum(1 for r in results if r.status == s)
                   for s in sorted({r.status for r in results if r.status != SK_OK})},
        "divergences_per_s": len(ok) / span if span > 0 else math.nan,
        "p50_ms": float(np.percentile(lat, 50) * 1e3) if len(lat) else math.nan,
        "p99_ms": float(np.percentile(lat, 99) * 1e3) if len(lat) else math.nan,
        "span_s": span,
    }
