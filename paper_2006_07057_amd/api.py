"""PyTorch-facing binding of the C ABI.

Every function here only checks and marshals arguments (device pointers,
sizes, the current HIP stream) and calls the HIP library; all arithmetic of
the method runs in the library's kernels.  PyTorch provides device memory
and streams.  Names follow the C ABI (sinkhorn_features, sinkhorn_solve,
sinkhorn_divergence, ...) with the ``sinkhorn_`` prefix dropped.

Numeric domain (``range``): EXTENDED (default) stores features as log2
values and scalings / r-vectors as [exponent | mantissa] halves (twice the
length); LINEAR stores plain float32 values.  ``host_log_scaling`` decodes
either layout on the host for inspection.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import (lib, check, sk_problem, sk_solve_opts, sk_solve_spec,
                   sk_state_layout, SK_RANGE_EXTENDED, SK_RANGE_LINEAR)

EXTENDED, LINEAR = SK_RANGE_EXTENDED, SK_RANGE_LINEAR

INFO_DTYPE = np.dtype([("iters", "<i4"), ("status", "<i4"), ("err", "<f8"),
                       ("w_hat", "<f8")])
INFO_BYTES = INFO_DTYPE.itemsize  # 24


def _stream(device=None):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _need(t: torch.Tensor, name: str, dtype=torch.float32, shape=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device (cuda) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {shape}")
    return t


def _opts(tol=1e-6, max_iter=2000, fixed_iter=0, warm_start=False,
          range=EXTENDED):
    return sk_solve_opts(float(tol), int(max_iter), int(fixed_iter),
                         int(bool(warm_start)), int(range))


def _width(range):
    return 2 if range == EXTENDED else 1


def parse_infos(raw: torch.Tensor) -> np.ndarray:
    """Decode device sk_solve_info records (synchronises)."""
    return raw.detach().cpu().numpy().view(INFO_DTYPE)


def host_log_scaling(t: torch.Tensor, range: int) -> np.ndarray:
    """Natural log of a scaling or r-vector stored by the library, on the
    host (float64).  For inspection and tests; synchronises."""
    a = t.detach().cpu().numpy().astype(np.float64)
    if range == EXTENDED:
        k = a.shape[0] // 2
        with np.errstate(divide="ignore"):
            return (a[:k] + np.log2(a[k:])) * math.log(2.0)
    with np.errstate(divide="ignore"):
        return np.log(a)


# ------------------------------------------------------------------ (a1)
def gaussian_q(R: float, eps: float, d: int) -> float:
    """Lemma 1 bandwidth q (host computation in the library)."""
    q = ctypes.c_double()
    check(lib().sinkhorn_gaussian_q(float(R), float(eps), int(d),
                                    ctypes.byref(q)), "sinkhorn_gaussian_q")
    return q.value


def gaussian_anchors(Z: np.ndarray, eps: float, sigma2: Optional[float] = None,
                     R: Optional[float] = None):
    """Anchors of Lemma 1 from standard normal draws Z (r x d, the caller's
    seeded randomness): U = sqrt(sigma2) Z with sigma2 given, or with
    sigma2 = q eps / 4 and q Lemma 1's bandwidth for points of norm <= R.
    Host call into the library; returns (U float32 (r, d), q)."""
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    if Z.ndim != 2:
        raise ValueError("Z must be r x d")
    r, d = Z.shape
    if (sigma2 is None) == (R is None):
        raise ValueError("give exactly one of sigma2 and R")
    U = np.empty((r, d), dtype=np.float32)
    q = ctypes.c_double()
    check(lib().sinkhorn_gaussian_anchors(Z.ctypes.data, r, d, float(eps),
                                          float(sigma2) if sigma2 is not None else 0.0,
                                          float(R) if R is not None else 0.0,
                                          U.ctypes.data, ctypes.byref(q)),
          "sinkhorn_gaussian_anchors")
    return U, q.value


# ------------------------------------------------------------------ (a2)
def features(X: torch.Tensor, U: torch.Tensor, eps: float, q: float,
             range: int = EXTENDED):
    """Row-scaled Gaussian features: returns (Phi (n, r), s (n,)) with
    phi_theta(x_i) = exp(s_i) Phi[i] (LINEAR) or exp(s_i) 2^Phi[i]
    (EXTENDED, log2 features)."""
    _need(X, "X")
    _need(U, "U")
    n, d = X.shape
    r = U.shape[0]
    if U.shape[1] != d:
        raise ValueError("U must be r x d with the same d as X")
    Phi = torch.empty((n, r), dtype=torch.float32, device=X.device)
    s = torch.empty((n,), dtype=torch.float32, device=X.device)
    check(lib().sinkhorn_features(_ptr(X), n, d, _ptr(U), r, float(eps),
                                  float(q), int(range), _ptr(Phi), _ptr(s),
                                  _stream(X.device)), "sinkhorn_features")
    return Phi, s


def features_arccos(X: torch.Tensor, U: torch.Tensor, s: int, sigma: float,
                    kappa: float):
    """Row-scaled perturbed arc-cosine features (linear domain): returns
    (Phi (n, r + 1), logscale (n,)); the last column is the constant
    feature sqrt(kappa)."""
    _need(X, "X")
    _need(U, "U")
    n, d = X.shape
    r = U.shape[0]
    if U.shape[1] != d:
        raise ValueError("U must be r x d with the same d as X")
    Phi = torch.empty((n, r + 1), dtype=torch.float32, device=X.device)
    ls = torch.empty((n,), dtype=torch.float32, device=X.device)
    check(lib().sinkhorn_features_arccos(_ptr(X), n, d, _ptr(U), r, int(s), float(sigma),
                                         float(kappa), _ptr(Phi), _ptr(ls),
                                         _stream(X.device)), "sinkhorn_features_arccos")
    return Phi, ls


def divergence_arccos(X, Y, a, b, U, s: int, sigma: float, kappa: float, eps: float,
                      tol=1e-6, max_iter=2000, fixed_iter=0):
    """Debiased divergence for the arc-cosine kernel (cost -eps log k_{s,kappa})
    through sinkhorn_divergence_arccos: features of both clouds, the three
    solves in one packed launch (linear domain), W_bar on the device.
    Returns (W_bar, infos) (synchronises)."""
    _check_problem_tensors(X, Y, a, b, U)
    n, d = X.shape
    m, r = Y.shape[0], U.shape[0]
    dev = X.device
    prob = sk_problem(X.data_ptr(), Y.data_ptr(), a.data_ptr(), b.data_ptr(),
                      U.data_ptr(), n, m, d, r, float(eps), 0.0)
    L = state_layout(n, m, r + 1)
    state = torch.empty(L.total, dtype=torch.uint8, device=dev)
    need = int(lib().sinkhorn_divergence_arccos_workspace_size(ctypes.byref(prob)))
    if need == 0:
        raise _lib.SinkhornError(_lib.SK_ENOTSUP, "sinkhorn_divergence_arccos_workspace_size")
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    out = torch.empty(4, dtype=torch.float64, device=dev)
    o = _opts(tol, max_iter, fixed_iter, False, LINEAR)
    check(lib().sinkhorn_divergence_arccos(ctypes.byref(prob), int(s), float(sigma),
                                           float(kappa), ctypes.byref(o), _ptr(out),
                                           _ptr(state), state.numel(), _ptr(ws), ws.numel(),
                                           _stream(dev)), "sinkhorn_divergence_arccos")
    rec = parse_infos(state[L.info:L.info + 3 * INFO_BYTES])
    return float(out[0].item()), rec


def divergence_assemble(infos: torch.Tensor, count: int,
                        out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """W_bar and the three dual estimates of `count` divergences from their
    device solve records (3 consecutive sk_solve_info per problem, as bytes)
    via sinkhorn_divergence_assemble.  Returns a device float64 tensor
    (count, 4) = (W_bar, W_xy, W_xx, W_yy) (asynchronous)."""
    if infos.dtype != torch.uint8 or not infos.is_cuda or not infos.is_contiguous():
        raise ValueError("infos must be a contiguous device uint8 tensor")
    if infos.numel() < 3 * count * INFO_BYTES:
        raise ValueError("infos holds fewer than 3 * count records")
    if out is None:
        out = torch.empty((count, 4), dtype=torch.float64, device=infos.device)
    check(lib().sinkhorn_divergence_assemble(_ptr(infos), int(count), _ptr(out),
                                             _stream(infos.device)),
          "sinkhorn_divergence_assemble")
    return out


# -------------------------------------------------------------- (a3)(a4)
@dataclasses.dataclass
class SolveResult:
    u: torch.Tensor
    v: torch.Tensor
    w: torch.Tensor
    z: torch.Tensor
    info_raw: torch.Tensor
    range: int

    def info(self):
        return parse_infos(self.info_raw)[0]


def solve(Phix: torch.Tensor, Phiy: torch.Tensor, a: torch.Tensor,
          b: torch.Tensor, tol: float = 1e-6, max_iter: int = 2000,
          fixed_iter: int = 0, u0: Optional[torch.Tensor] = None,
          range: int = EXTENDED,
          workspace: Optional[torch.Tensor] = None) -> SolveResult:
    """Algorithm 1 on K = Phix Phiy^T (asynchronous; read .info() to sync).
    In the EXTENDED range Phix/Phiy are log2 features and u, v, w, z come
    back as [exponent | mantissa] arrays."""
    _need(Phix, "Phix")
    _need(Phiy, "Phiy")
    n, r = Phix.shape
    m = Phiy.shape[0]
    if Phiy.shape[1] != r:
        raise ValueError("Phix and Phiy need the same number of features")
    _need(a, "a", shape=(n,))
    _need(b, "b", shape=(m,))
    dev = Phix.device
    k = _width(range)
    u = u0.clone() if u0 is not None else torch.empty(k * n, dtype=torch.float32, device=dev)
    v = torch.empty(k * m, dtype=torch.float32, device=dev)
    w = torch.empty(k * r, dtype=torch.float32, device=dev)
    z = torch.empty(k * r, dtype=torch.float32, device=dev)
    info = torch.zeros(INFO_BYTES, dtype=torch.uint8, device=dev)
    need = lib().sinkhorn_solve_workspace_size(n, m, r)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    o = _opts(tol, max_iter, fixed_iter, u0 is not None, range)
    check(lib().sinkhorn_solve(_ptr(Phix), n, _ptr(Phiy), m, r, _ptr(a), _ptr(b),
                               ctypes.byref(o), _ptr(u), _ptr(v), _ptr(w),
                               _ptr(z), _ptr(info), _ptr(workspace),
                               workspace.numel(), _stream(dev)),
          "sinkhorn_solve")
    return SolveResult(u, v, w, z, info, range)


# ------------------------------------------------------------------ (a5)
def state_layout(n: int, m: int, r: int) -> sk_state_layout:
    L = sk_state_layout()
    check(lib().sinkhorn_state_layout(n, m, r, ctypes.byref(L)),
          "sinkhorn_state_layout")
    return L


class DivergenceState:
    """Device state of one divergence (features, scalings, infos), kept for
    the backward pass and for inspection."""

    def __init__(self, X, Y, a, b, U, eps, q):
        self.X, self.Y, self.a, self.b, self.U = X, Y, a, b, U
        self.eps, self.q = float(eps), float(q)
        self.n, self.d = X.shape
        self.m = Y.shape[0]
        self.r = U.shape[0]
        self.range = EXTENDED
        self.layout = state_layout(self.n, self.m, self.r)
        self.buf = torch.empty(self.layout.total, dtype=torch.uint8,
                               device=X.device)
        self.problem = sk_problem(X.data_ptr(), Y.data_ptr(), a.data_ptr(),
                                  b.data_ptr(), U.data_ptr(), self.n, self.m,
                                  self.d, self.r, self.eps, self.q)

    def _view(self, off, count, dtype=torch.float32):
        nbytes = count * torch.tensor([], dtype=dtype).element_size()
        return self.buf[off:off + nbytes].view(dtype)

    @property
    def phix(self):
        return self._view(self.layout.phix, self.n * self.r).view(self.n, self.r)

    @property
    def phiy(self):
        return self._view(self.layout.phiy, self.m * self.r).view(self.m, self.r)

    @property
    def sx(self):
        return self._view(self.layout.sx, self.n)

    @property
    def sy(self):
        return self._view(self.layout.sy, self.m)

    def scalings(self, k):
        """(u, v, w, z) of solve k: 0 = (x,y), 1 = (x,x), 2 = (y,y), in the
        layout of the domain used (pairs in the EXTENDED range)."""
        rows = (self.n, self.n, self.m)[k]
        cols = (self.m, self.n, self.m)[k]
        L = self.layout
        c = _width(self.range)
        return (self._view(L.u[k], c * rows), self._view(L.v[k], c * cols),
                self._view(L.w[k], c * self.r), self._view(L.z[k], c * self.r))

    def log_scalings(self, k):
        """Natural logs of (u, v) of solve k on the host (float64)."""
        u, v, _, _ = self.scalings(k)
        return host_log_scaling(u, self.range), host_log_scaling(v, self.range)

    def infos(self) -> np.ndarray:
        return parse_infos(self.buf[self.layout.info:self.layout.info +
                                    3 * INFO_BYTES])

    @property
    def out(self):
        return self._view(self.layout.out, 4, torch.float64)

    def meta(self) -> np.ndarray:
        """int32[4]: numeric domain, then the gradient evaluations of the
        three accelerated solves (zeros for Algorithm 1)."""
        return self._view(self.layout.meta, 4, torch.int32).cpu().numpy()


def _check_problem_tensors(X, Y, a, b, U):
    _need(X, "X")
    _need(Y, "Y")
    _need(U, "U")
    n, d = X.shape
    m = Y.shape[0]
    if Y.shape[1] != d or U.shape[1] != d:
        raise ValueError("X, Y and U need the same dimension d")
    _need(a, "a", shape=(n,))
    _need(b, "b", shape=(m,))


def divergence_workspace_bytes(state: DivergenceState) -> int:
    return int(lib().sinkhorn_divergence_workspace_size(ctypes.byref(state.problem)))


def divergence(X, Y, a, b, U, eps, q, tol=1e-6, max_iter=2000, fixed_iter=0,
               range=EXTENDED, workspace: Optional[torch.Tensor] = None,
               state: Optional[DivergenceState] = None):
    """Debiased divergence.  Returns (out, state) with out a device float64
    tensor [W_bar, W_xy, W_xx, W_yy] (asynchronous)."""
    _check_problem_tensors(X, Y, a, b, U)
    if state is None:
        state = DivergenceState(X, Y, a, b, U, eps, q)
    state.range = int(range)
    need = divergence_workspace_bytes(state)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=X.device)
    out = torch.empty(4, dtype=torch.float64, device=X.device)
    o = _opts(tol, max_iter, fixed_iter, False, range)
    check(lib().sinkhorn_divergence(ctypes.byref(state.problem), ctypes.byref(o),
                                    _ptr(out), _ptr(state.buf),
                                    state.buf.numel(), _ptr(workspace),
                                    workspace.numel(), _stream(X.device)),
          "sinkhorn_divergence")
    state.workspace = workspace
    return out, state


def divergence_backward(state: DivergenceState,
                        grad_out: Optional[torch.Tensor] = None,
                        need=(True, True, True, True), out=None):
    """Gradients (dX, da, dY, db) of the divergence held in `state`.
    out: optional (dX, da, dY, db) tensors to write (None entries are
    allocated where `need` asks for them)."""
    dev = state.X.device
    o = tuple(out) if out is not None else (None, None, None, None)
    dX = (o[0] if o[0] is not None else torch.empty_like(state.X)) if need[0] else None
    da = (o[1] if o[1] is not None else torch.empty_like(state.a)) if need[1] else None
    dY = (o[2] if o[2] is not None else torch.empty_like(state.Y)) if need[2] else None
    db = (o[3] if o[3] is not None else torch.empty_like(state.b)) if need[3] else None
    for t, ref, nm in ((dX, state.X, "dX"), (da, state.a, "da"), (dY, state.Y, "dY"),
                       (db, state.b, "db")):
        if t is not None:
            _need(t, nm, shape=tuple(ref.shape))
    ws = getattr(state, "workspace", None)
    if ws is None or ws.numel() < 32768:
        ws = torch.empty(32768, dtype=torch.uint8, device=dev)
    if grad_out is not None:
        grad_out = grad_out.detach().to(device=dev, dtype=torch.float32).reshape(1).contiguous()
    check(lib().sinkhorn_divergence_backward(
        ctypes.byref(state.problem), _ptr(state.buf), _ptr(grad_out), _ptr(dX),
        _ptr(da), _ptr(dY), _ptr(db), _ptr(ws), ws.numel(), _stream(dev)),
        "sinkhorn_divergence_backward")
    return dX, da, dY, db


def divergence_backward_anchors(state: DivergenceState,
                                grad_out: Optional[torch.Tensor] = None):
    """Gradient dU (r x d) of the divergence held in `state` with respect to
    the anchors (q fixed)."""
    dev = state.X.device
    dU = torch.empty_like(state.U)
    need = int(lib().sinkhorn_divergence_backward_anchors_workspace_size(
        ctypes.byref(state.problem)))
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    if grad_out is not None:
        grad_out = grad_out.detach().to(device=dev, dtype=torch.float32).reshape(1).contiguous()
    check(lib().sinkhorn_divergence_backward_anchors(
        ctypes.byref(state.problem), _ptr(state.buf), _ptr(grad_out), _ptr(dU), _ptr(ws),
        ws.numel(), _stream(dev)), "sinkhorn_divergence_backward_anchors")
    return dU


def features_backward(X, U, Phi, p, g, coef=1.0, dX=None, accumulate=False,
                      range=EXTENDED):
    """dX (+)= coef * 4 p_i (x_i (Phi_i . g) - sum_k Phi_ik g_k u_k)."""
    n, d = X.shape
    r = U.shape[0]
    if dX is None:
        dX = torch.zeros_like(X)
    check(lib().sinkhorn_features_backward(_ptr(X), n, d, _ptr(U), r, _ptr(Phi),
                                           _ptr(p), _ptr(g), float(coef),
                                           int(accumulate), int(range),
                                           _ptr(dX), _stream(X.device)),
          "sinkhorn_features_backward")
    return dX


# ------------------------------------------------------------------ (a6)
class DivergenceGraph:
    """One divergence step (features, the three solves, the float64
    assembly and optionally the adjoint) captured once as a HIP graph and
    replayed, for repeated calls on fixed shapes (an optimisation loop over
    point locations, a fixed-shape serving batch).  Every launch of the step
    is a library kernel; none of them allocates, copies or sets memory, so
    the captured graph is exactly the eager sequence.  Inputs are copied
    into the graph's static buffers before each replay; results are the
    static output tensors (overwritten by the next replay)."""

    def __init__(self, n, m, d, r, eps, q, tol=1e-6, max_iter=2000, fixed_iter=0,
                 range=EXTENDED, backward=True, device="cuda:0"):
        dev = torch.device(device)
        f32 = dict(dtype=torch.float32, device=dev)
        self.X = torch.zeros((n, d), **f32)
        self.Y = torch.zeros((m, d), **f32)
        self.a = torch.full((n,), 1.0 / n, **f32)
        self.b = torch.full((m,), 1.0 / m, **f32)
        self.U = torch.zeros((r, d), **f32)
        self.kw = dict(tol=tol, max_iter=max_iter, fixed_iter=fixed_iter, range=range)
        self.eps, self.q, self.backward = float(eps), float(q), bool(backward)
        self.state = DivergenceState(self.X, self.Y, self.a, self.b, self.U, eps, q)
        self.state.range = int(range)
        need = max(divergence_workspace_bytes(self.state), 32768)
        self.workspace = torch.empty(need, dtype=torch.uint8, device=dev)
        self.out = torch.empty(4, dtype=torch.float64, device=dev)
        self.grads = tuple(torch.empty_like(t) for t in (self.X, self.a, self.Y, self.b))
        self.graph = None

    def _step(self, stream):
        o = _opts(self.kw["tol"], self.kw["max_iter"], self.kw["fixed_iter"], False,
                  self.kw["range"])
        st = self.state
        check(lib().sinkhorn_divergence(ctypes.byref(st.problem), ctypes.byref(o),
                                        _ptr(self.out), _ptr(st.buf), st.buf.numel(),
                                        _ptr(self.workspace), self.workspace.numel(),
                                        stream), "sinkhorn_divergence")
        if self.backward:
            dX, da, dY, db = self.grads
            check(lib().sinkhorn_divergence_backward(
                ctypes.byref(st.problem), _ptr(st.buf), _ptr(None), _ptr(dX), _ptr(da),
                _ptr(dY), _ptr(db), _ptr(self.workspace), self.workspace.numel(), stream),
                "sinkhorn_divergence_backward")

    def capture(self):
        dev = self.X.device
        side = torch.cuda.Stream(device=dev)
        side.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(side):  # one eager run before capture
            self._step(_stream(dev))
        torch.cuda.current_stream(dev).wait_stream(side)
        torch.cuda.synchronize(dev)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._step(_stream(dev))
        return self

    def __call__(self, X, Y, a=None, b=None, U=None):
        """Copy the inputs in and replay (asynchronous).  Returns
        (out [W_bar, W_xy, W_xx, W_yy], (dX, da, dY, db) or None)."""
        if self.graph is None:
            self.capture()
        self.X.copy_(X)
        self.Y.copy_(Y)
        if a is not None:
            self.a.copy_(a)
        if b is not None:
            self.b.copy_(b)
        if U is not None:
            self.U.copy_(U)
        self.graph.replay()
        return self.out, (self.grads if self.backward else None)


class BatchedDivergenceGraph:
    """A batch of divergences of fixed, uneven shapes (the packed persistent
    launches of sinkhorn_divergence_batched, then optionally the adjoint of
    every problem) captured once as a HIP graph and replayed.  ``shapes``
    holds (n, m, d, r, eps, q) per problem.  Inputs are copied into static
    buffers before each replay; ``out`` (count x 4) and the gradients are
    static tensors overwritten by the next replay."""

    def __init__(self, shapes: Sequence[tuple], tol=1e-6, max_iter=2000, fixed_iter=0,
                 range=EXTENDED, backward=True, device="cuda:0"):
        dev = torch.device(device)
        f32 = dict(dtype=torch.float32, device=dev)
        self.inputs, self.states = [], []
        for (n, m, d, r, eps, q) in shapes:
            X = torch.zeros((n, d), **f32)
            Y = torch.zeros((m, d), **f32)
            a = torch.full((n,), 1.0 / n, **f32)
            b = torch.full((m,), 1.0 / m, **f32)
            U = torch.zeros((r, d), **f32)
            st = DivergenceState(X, Y, a, b, U, eps, q)
            st.range = int(range)
            self.inputs.append((X, Y, a, b, U))
            self.states.append(st)
        count = len(self.states)
        self.kw = dict(tol=tol, max_iter=max_iter, fixed_iter=fixed_iter, range=range)
        self.backward = bool(backward)
        self._arr = (sk_problem * count)(*[s.problem for s in self.states])
        self._ptrs = (ctypes.c_void_p * count)(*[s.buf.data_ptr() for s in self.states])
        need = int(lib().sinkhorn_batched_workspace_size(self._arr, count))
        if need == 0:
            raise ValueError("invalid batch")
        self.workspace = torch.empty(max(need, 32768), dtype=torch.uint8, device=dev)
        self.out = torch.empty((count, 4), dtype=torch.float64, device=dev)
        self.grads = [tuple(torch.empty_like(t) for t in (X, a, Y, b))
                      for (X, Y, a, b, _) in self.inputs]
        self.graph = None

    def _step(self, stream):
        o = _opts(self.kw["tol"], self.kw["max_iter"], self.kw["fixed_iter"], False,
                  self.kw["range"])
        count = len(self.states)
        check(lib().sinkhorn_divergence_batched(self._arr, count, ctypes.byref(o),
                                                _ptr(self.out), self._ptrs,
                                                _ptr(self.workspace), self.workspace.numel(),
                                                stream), "sinkhorn_divergence_batched")
        if self.backward:
            for st, (dX, da, dY, db) in zip(self.states, self.grads):
                check(lib().sinkhorn_divergence_backward(
                    ctypes.byref(st.problem), _ptr(st.buf), _ptr(None), _ptr(dX), _ptr(da),
                    _ptr(dY), _ptr(db), _ptr(self.workspace), self.workspace.numel(),
                    stream), "sinkhorn_divergence_backward")

    def capture(self):
        dev = self.out.device
        side = torch.cuda.Stream(device=dev)
        side.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(side):  # one eager run before capture
            self._step(_stream(dev))
        torch.cuda.current_stream(dev).wait_stream(side)
        torch.cuda.synchronize(dev)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._step(_stream(dev))
        return self

    def __call__(self, problems: Sequence[tuple]):
        """problems: (X, Y, a, b, U) per problem, shapes as captured.  Copies
        them in and replays (asynchronous).  Returns (out, grads or None)."""
        if self.graph is None:
            self.capture()
        if len(problems) != len(self.inputs):
            raise ValueError("batch size differs from the captured one")
        for src, dst in zip(problems, self.inputs):
            for s_, d_ in zip(src, dst):
                if tuple(s_.shape) != tuple(d_.shape):
                    raise ValueError("shape differs from the captured one")
                d_.copy_(s_)
        self.graph.replay()
        return self.out, (self.grads if self.backward else None)


def batched_states(problems: Sequence[tuple], range=EXTENDED):
    """Device states of a batch (allocated here, filled by
    divergence_batched)."""
    states: List[DivergenceState] = []
    for P in problems:
        _check_problem_tensors(*P[:5])
        st = DivergenceState(*P)
        st.range = int(range)
        states.append(st)
    return states


def batched_workspace_bytes(states: Sequence[DivergenceState]) -> int:
    arr = (sk_problem * len(states))(*[s.problem for s in states])
    return int(lib().sinkhorn_batched_workspace_size(arr, len(states)))


def divergence_batched(problems: Sequence[tuple], tol=1e-6, max_iter=2000,
                       fixed_iter=0, range=EXTENDED,
                       workspace: Optional[torch.Tensor] = None,
                       states: Optional[Sequence[DivergenceState]] = None,
                       out: Optional[torch.Tensor] = None):
    """Many divergences in batched launches.  ``problems`` holds tuples
    (X, Y, a, b, U, eps, q).  Returns (out (count, 4) float64, states).
    states / out / workspace: optional buffers made beforehand
    (batched_states, batched_workspace_bytes), so that the call allocates
    nothing."""
    if states is None:
        states = batched_states(problems, range)
    else:
        states = list(states)
        if len(states) != len(problems):
            raise ValueError("one state per problem")
        for st in states:
            st.range = int(range)
    count = len(states)
    dev = states[0].X.device
    arr = (sk_problem * count)(*[s.problem for s in states])
    need = int(lib().sinkhorn_batched_workspace_size(arr, count))
    if need == 0:
        raise ValueError("invalid batch")
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    if out is None:
        out = torch.empty((count, 4), dtype=torch.float64, device=dev)
    else:
        _need(out, "out", dtype=torch.float64, shape=(count, 4))
    ptrs = (ctypes.c_void_p * count)(*[s.buf.data_ptr() for s in states])
    o = _opts(tol, max_iter, fixed_iter, False, range)
    check(lib().sinkhorn_divergence_batched(arr, count, ctypes.byref(o),
                                            _ptr(out), ptrs, _ptr(workspace),
                                            workspace.numel(), _stream(dev)),
          "sinkhorn_divergence_batched")
    for s in states:
        s.workspace = workspace
    return out, states


def solve_spec(Prow, Pcol, a, b, u, v, w, z, info, eps=1.0, srow=None,
               scol=None) -> sk_solve_spec:
    """Descriptor of one solve for solve_batched (pointers of the given
    device tensors; keep the tensors alive while the launch runs).  u, v, w,
    z hold 8 bytes per entry; info holds one 24-byte record."""
    n, r = Prow.shape
    m = Pcol.shape[0]
    return sk_solve_spec(Prow.data_ptr(), Pcol.data_ptr(), a.data_ptr(),
                         b.data_ptr(), srow.data_ptr() if srow is not None else 0,
                         scol.data_ptr() if scol is not None else 0,
                         u.data_ptr(), v.data_ptr(), w.data_ptr(), z.data_ptr(),
                         info.data_ptr(), n, m, r, float(eps))


def solve_batched_workspace_bytes(specs: Sequence[sk_solve_spec]) -> int:
    arr = (sk_solve_spec * len(specs))(*specs)
    return int(lib().sinkhorn_solve_batched_workspace_size(arr, len(specs)))


def solve_batched(specs: Sequence[sk_solve_spec], tol=1e-6, max_iter=2000,
                  fixed_iter=0, warm_start=False, range=EXTENDED,
                  workspace: Optional[torch.Tensor] = None, device=None):
    """Run many solves in packed persistent launches (asynchronous).
    Returns the workspace tensor used (reuse it for the next call)."""
    count = len(specs)
    arr = (sk_solve_spec * count)(*specs)
    need = int(lib().sinkhorn_solve_batched_workspace_size(arr, count))
    if need == 0:
        raise ValueError("invalid solve specs")
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else device
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    o = _opts(tol, max_iter, fixed_iter, warm_start, range)
    check(lib().sinkhorn_solve_batched(arr, count, ctypes.byref(o),
                                       _ptr(workspace), workspace.numel(),
                                       _stream(dev)), "sinkhorn_solve_batched")
    return workspace


def solve_accelerated_workspace_bytes(spec: sk_solve_spec) -> int:
    return int(lib().sinkhorn_solve_accelerated_workspace_size(ctypes.byref(spec)))


def solve_accelerated(spec: sk_solve_spec, tol=1e-6, max_iter=2000, fixed_iter=0,
                      L0=1.0, trials: Optional[torch.Tensor] = None,
                      workspace: Optional[torch.Tensor] = None, device=None):
    """Accelerated Sinkhorn on one factored kernel whose features are in the
    linear layout (asynchronous).  trials: optional device int32 tensor of
    one element receiving the number of gradient evaluations.  Returns the
    workspace tensor used."""
    need = solve_accelerated_workspace_bytes(spec)
    if need == 0:
        raise ValueError("invalid solve spec")
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else device
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    if trials is not None:
        _need(trials, "trials", dtype=torch.int32, shape=(1,))
    o = _opts(tol, max_iter, fixed_iter, False, LINEAR)
    check(lib().sinkhorn_solve_accelerated(ctypes.byref(spec), ctypes.byref(o), float(L0),
                                           _ptr(trials), _ptr(workspace), workspace.numel(),
                                           _stream(dev)), "sinkhorn_solve_accelerated")
    return workspace


def divergence_accelerated(X, Y, a, b, U, eps, q, tol=1e-6, max_iter=2000, fixed_iter=0,
                           L0=1.0, workspace: Optional[torch.Tensor] = None,
                           state: Optional[DivergenceState] = None):
    """Debiased divergence with each term solved by accelerated Sinkhorn
    (linear-layout features).  Returns (out, state) as divergence() does;
    divergence_backward applies to the state."""
    _check_problem_tensors(X, Y, a, b, U)
    if state is None:
        state = DivergenceState(X, Y, a, b, U, eps, q)
    state.range = LINEAR
    need = int(lib().sinkhorn_divergence_accelerated_workspace_size(
        ctypes.byref(state.problem)))
    if need == 0:
        raise ValueError("invalid problem")
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=X.device)
    out = torch.empty(4, dtype=torch.float64, device=X.device)
    o = _opts(tol, max_iter, fixed_iter, False, LINEAR)
    check(lib().sinkhorn_divergence_accelerated(
        ctypes.byref(state.problem), ctypes.byref(o), float(L0), _ptr(out), _ptr(state.buf),
        state.buf.numel(), _ptr(workspace), workspace.numel(), _stream(X.device)),
        "sinkhorn_divergence_accelerated")
    state.workspace = workspace
    return out, state


def tune_set(r: int, target_bytes: int):
    """Set the feature bytes per workgroup for the solver class serving r
    (0 restores the default)."""
    check(lib().sinkhorn_tune_set(int(r), int(target_bytes)), "sinkhorn_tune_set")


def tune_get(r: int) -> int:
    v = int(lib().sinkhorn_tune_get(int(r)))
    if v < 0:
        raise ValueError(f"no solver class for r={r}")
    return v


def solver_layouts(r: int):
    """Lane layouts compiled for the solver class serving r, as a list of
    (G, C, U, W) tuples; index = variant (0 is the default)."""
    cnt = int(lib().sinkhorn_solver_layouts(int(r), None, 0))
    if cnt < 0:
        raise ValueError(f"no solver class for r={r}")
    buf = (ctypes.c_int32 * (4 * max(cnt, 1)))()
    lib().sinkhorn_solver_layouts(int(r), ctypes.cast(buf, ctypes.c_void_p), cnt)
    return [tuple(int(buf[4 * i + k]) for k in range(4)) for i in range(cnt)]


def tune_set_layout(r: int, variant: int):
    """Select the lane layout variant of the solver class serving r."""
    check(lib().sinkhorn_tune_set_layout(int(r), int(variant)), "sinkhorn_tune_set_layout")


def tune_get_layout(r: int) -> int:
    v = int(lib().sinkhorn_tune_get_layout(int(r)))
    if v < 0:
        raise ValueError(f"no solver class for r={r}")
    return v


# ------------------------------------------------------- instrumentation
PROF_SOLVER, PROF_FEATURES, PROF_ADJOINT = 0, 1, 2


def profile(enable: bool = True):
    """Start (and clear) or stop per-launch event timing in the library."""
    check(lib().sinkhorn_profile(int(bool(enable))), "sinkhorn_profile")


def profile_read(kind: int):
    """(total_ms, launches, max_ms) of the recorded launches of one kind."""
    tot, mx = ctypes.c_double(), ctypes.c_double()
    cnt = ctypes.c_int64()
    check(lib().sinkhorn_profile_read(int(kind), ctypes.byref(tot),
                                      ctypes.byref(cnt), ctypes.byref(mx)),
          "sinkhorn_profile_read")
    return tot.value, cnt.value, mx.value


# ------------------------------------------------------------------ (a8)
class _SinkhornDivergenceFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X, Y, a, b, U, eps, q, tol, max_iter, fixed_iter, range):
        out, state = divergence(X, Y, a, b, U, eps, q, tol, max_iter,
                                fixed_iter, range)
        ctx.state = state
        return out[0]

    @staticmethod
    def backward(ctx, g):
        need = (ctx.needs_input_grad[0], ctx.needs_input_grad[2],
                ctx.needs_input_grad[1], ctx.needs_input_grad[3])
        dX, da, dY, db = divergence_backward(ctx.state, g, need)
        dU = divergence_backward_anchors(ctx.state, g) if ctx.needs_input_grad[4] else None
        return dX, dY, da, db, dU, None, None, None, None, None, None


def sinkhorn_divergence(X, Y, a, b, U, eps, q, tol=1e-6, max_iter=2000,
                        fixed_iter=0, range=EXTENDED):
    """Differentiable debiased Sinkhorn divergence (float64 scalar tensor);
    gradients flow to X, Y, a, b and the anchors U (q held fixed) through the
    library's adjoint kernels."""
    return _SinkhornDivergenceFn.apply(X, Y, a, b, U, eps, q, tol, max_iter,
                                       fixed_iter, range)
