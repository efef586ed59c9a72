"""Comparison helpers shared by the GPU parity tests (no method arithmetic).

Every field is compared by its relative L2 difference.  Two numbers are
kept per field:

- ``raw``: ||gpu - ref|| / ||ref||, the plain relative L2 difference;
- ``rel``: the value the tolerances are asserted on.  It equals ``raw``
  except that each velocity component is measured against the velocity
  scale of the reference state itself, the RMS over all its components,
  when the component is smaller than that (a component that is almost zero
  in a given flow, e.g. the radial velocity of a nearly axial flow, is not
  divided by its own near-zero norm).  No other floor is applied.
"""
import math

import numpy as np

VEL_KEYS = ("u", "v", "w")


def _norm(a):
    return float(np.linalg.norm(np.asarray(a, dtype=np.float64)))


def rel_l2(a, b, floor=0.0):
    """||a - b|| / max(||b||, floor * sqrt(size))."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = max(_norm(b), floor * math.sqrt(b.size))
    return _norm(a - b) / den if den > 0 else _norm(a - b)


def state_keys(prob):
    return ["p", "u", "v"] + (["w"] if prob["dim"] == 3 else []) + ["phi"]


def compare_states(prob, gpu, ref):
    """Per-field relative L2 differences: returns (rel, raw) dictionaries."""
    keys = state_keys(prob)
    vel = [k for k in keys if k in VEL_KEYS]
    vel_rms = math.sqrt(sum(_norm(ref[k]) ** 2 for k in vel) / len(vel))
    rel, raw = {}, {}
    for k in keys:
        num = _norm(np.asarray(gpu[k], dtype=np.float64) - np.asarray(ref[k], dtype=np.float64))
        den = _norm(ref[k])
        raw[k] = num / den if den > 0 else num
        if k in VEL_KEYS:
            den = max(den, vel_rms)
        rel[k] = num / den if den > 0 else num
    return rel, raw


def fmt(d):
    return " ".join(f"{k}={v:.2e}" for k, v in d.items())
