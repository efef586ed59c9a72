"""Comparison helpers shared by the GPU parity tests (no method arithmetic)."""
import math

import numpy as np


def velocity_scale(prob):
    """Characteristic velocity used as the floor of relative norms of fields
    that may be almost zero (spurious currents of a static drop)."""
    if prob["sigma"] > 0 and prob["eta_l"] > 0:
        return prob["sigma"] / prob["eta_l"]
    g = math.sqrt(sum(x * x for x in prob["g"]))
    return max(math.sqrt(g * prob["n"][0]), 1e-3)


def rel_l2(a, b, floor=0.0):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = max(float(np.linalg.norm(b)), floor * math.sqrt(b.size))
    return float(np.linalg.norm(a - b)) / den if den > 0 else float(np.linalg.norm(a - b))


def compare_states(prob, gpu, ref):
    """Relative L2 differences per field: velocities and pressure floored by
    the characteristic velocity U_c and dynamic pressure rho_L U_c^2."""
    U = velocity_scale(prob)
    out = {}
    keys = ["p", "u", "v", "phi"] + (["w"] if prob["dim"] == 3 else [])
    for k in keys:
        floor = {"p": prob["rho_l"] * U * U, "phi": 0.0}.get(k, U)
        out[k] = rel_l2(gpu[k], ref[k], floor)
    return out
