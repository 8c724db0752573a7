"""Acceptance checks of the GPU parity tests, in one place.

Divergences (Eq. reg-sdiv): each of the three dual estimates
W_hat (Eq. dual-estimate) must match the oracle's within DIV_RTOL relative,
and W_bar within DIV_RTOL relative, with no absolute allowance (also where
W_bar is 1e-6 of the terms it is the difference of); every call prints the
achieved errors, so the margin is visible in the log.

Gradients (Prop. 3.2 and the point gradient of Sec. 3.3): relative L2
error within GRAD_RTOL and, per entry, |g_i - r_i| <= GRAD_RTOL |r_i| +
GRAD_RTOL max|r| (a relative bound with an absolute floor of
GRAD_RTOL max|r|).

Set SK_PARITY_LOG to a file path to also append every check as one JSON
line (the tests assert either way).
"""
import json
import math
import os
import sys

import numpy as np

DIV_RTOL = 1e-5
GRAD_RTOL = 1e-4
GRAD_ENTRY_FLOOR = 1e-4


def _log(rec):
    print("[parity]", json.dumps(rec), file=sys.stderr, flush=True)
    path = os.environ.get("SK_PARITY_LOG")
    if path:
        with open(path, "a") as f:
            f.write(json.dumps(rec) + "\n")


def _ref4(ref):
    if hasattr(ref, "w_xy"):
        return (float(ref.value), float(ref.w_xy), float(ref.w_xx), float(ref.w_yy))
    return tuple(float(x) for x in ref)


def check_divergence(label, got, ref, terms=True, rtol=DIV_RTOL):
    """got: (W_bar, W_xy, W_xx, W_yy) from the device (or just W_bar when
    terms=False); ref: oracle Divergence or the same 4-tuple."""
    r = _ref4(ref)
    g = [float(x) for x in np.ravel(np.asarray(got, dtype=np.float64))]
    err = abs(g[0] - r[0])
    rec = {"check": "divergence", "label": label, "W_bar": g[0], "W_bar_ref": r[0],
           "W_bar_rel": err / abs(r[0]) if r[0] != 0 else math.inf}
    if terms:
        rec["terms_rel"] = [abs(g[k] - r[k]) / abs(r[k]) for k in (1, 2, 3)]
        rec["terms_ref"] = list(r[1:])
    _log(rec)
    if terms:
        for k, name in ((1, "W_xy"), (2, "W_xx"), (3, "W_yy")):
            assert abs(g[k] - r[k]) <= rtol * abs(r[k]), (label, name, g[k], r[k])
    assert err <= rtol * abs(r[0]), (label, g[0], r[0], err)
    return rec


def check_value(label, got, ref, rtol=DIV_RTOL, atol=0.0):
    """One scalar (a single dual estimate, a dual value) within rtol."""
    got, ref = float(got), float(ref)
    err = abs(got - ref)
    _log({"check": "value", "label": label, "got": got, "ref": ref,
          "rel": err / abs(ref) if ref != 0 else math.inf, "atol": atol})
    assert err <= rtol * abs(ref) + atol, (label, got, ref, err)


def check_gradient(label, g, r, rtol=GRAD_RTOL, entry_floor=GRAD_ENTRY_FLOOR):
    g = np.asarray(g, np.float64)
    r = np.asarray(r, np.float64)
    rel = float(np.linalg.norm(g - r) / np.linalg.norm(r))
    mx = float(np.abs(r).max())
    dev = np.abs(g - r)
    entry = float((dev / (rtol * np.abs(r) + entry_floor * mx)).max())
    _log({"check": "gradient", "label": label, "rel_l2": rel,
          "max_entry_err_over_max": float(dev.max() / mx), "entry_ratio": entry})
    assert rel <= rtol, (label, rel)
    assert entry <= 1.0, (label, "per-entry", entry)
