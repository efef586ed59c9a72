"""Replays of the paper's experiments (Sec. 4) on the GPU with the paper's
diagnostics, computed by the library's reduction kernels:

- the benchmark configurations at full size and length: the static drop
  (mass drift, kinetic energy, spurious velocity, pressure difference), the
  Rayleigh-Taylor case (bubble and spike fronts) and the rising bubble (gas
  centroid, top and bottom, rise velocity);
- capillary wave (Sec. 4.1, Re 1000, r_rho = r_eta = 20) on the paper's two
  meshes: the scaled interface displacement h~ = (h_eq - h_0) / A_p at
  y = 0, in T_c;
- falling drop (axisymmetric, Eo 144, Oh 0.0466): centroid velocity U_drop
  and aspect ratio Th / Wh (axial thickness over radial width), in
  U_c' = sqrt(g D), T_c' = sqrt(D / g);
- axisymmetric and 3-D coalescence (r_rho 50, r_eta 58.8): the radius R_r of
  the liquid bridge at z = 0 (axisymmetric) or the half length R_x of the
  drop on the x axis (3-D), and the centroid velocity of the drop in the box
  (along the line of centres in the axisymmetric case, across it in 3-D),
  in R, U_ci, T_ci; each case also records the other's length (the 3-D
  bridge radius on x = 0, the axisymmetric half length on the axis), so that
  the two geometries can be compared on the same flow;
- the 3-D coalescence with each of the paper's two ablations of its scheme
  (no transverse pressure average at Oh 0.3, zero bulk viscosity at
  Oh 0.037) beside its control, with the largest grid-scale (checkerboard)
  pressure amplitude, in units of the Laplace pressure 2 sigma / R;
- Rayleigh-Taylor (At 0.5, Re 256 / 3000): bubble front (smallest crossing
  on y = 0) and spike front (largest crossing on y = 1/2), in L_c, T_c.

Run `python -m paper_2011_00814_amd.replays [names] --out FILE`; each case
prints one JSON line with its time series.  The paper gives these curves as
figures only, so the series are self-consistency and regression data.
"""
from __future__ import annotations

import argparse
import json
import math
import time

from . import gpe as G
from . import workloads as W


def _falling(prec):
    return W.falling_drop_axisym(precision=prec)


def _config1(prec):
    prob, st = W.static_drop_2d(precision=prec)
    return prob, st, {"L": 16.0, "U": 1.0, "T": 1.0}           # time in steps


def _config2(prec):
    prob, st = W.rayleigh_taylor_2d(precision=prec)
    lam = float(prob["n"][0])
    U = math.sqrt(-prob["g"][1] * lam)
    return prob, st, {"L": lam, "U": U, "T": lam / U}            # T_c = lambda / sqrt(g lambda)


def _config3(prec):
    prob, st = W.rising_bubble_3d(precision=prec)
    return prob, st, {"L": 32.0, "D": 32.0, "kind": "gravity"}      # U = sqrt(g D), T = sqrt(D / g)


CASES = {
    # name: (builder(precision) -> (prob, state, scales), end time in the case's time unit, outputs)
    # the benchmark configurations at full size and length: static drop 64^2 for 1000 steps,
    # Rayleigh-Taylor 256 x 1024 for 20,000 steps (3.9 T_c), rising bubble 128 x 128 x 256 for
    # 10,000 steps (9.4 T_c)
    "config1_static_drop": (_config1, 1000.0, 10),
    "config2_rt": (_config2, 20000.0 / 5120.0, 10),
    "config3_rising_bubble": (_config3, 10000.0 / math.sqrt(32.0 / 2.8125e-5), 10),
    "capillary_wave": (lambda p: W.capillary_wave(precision=p), 30.0, 30),
    "capillary_wave_fine": (
        lambda p: W.capillary_wave(NL=128, Nt=1920, Cn=0.03125, Pe=4e4, precision=p), 30.0, 30),
    "falling_drop": (_falling, 12.0, 24),
    "coalescence_axisym_oh0.037": (lambda p: W.coalescence_axisym(Oh=0.037, precision=p), 4.0, 20),
    "coalescence_axisym_oh0.119": (lambda p: W.coalescence_axisym(Oh=0.119, precision=p), 4.0, 20),
    "coalescence_axisym_oh0.3": (lambda p: W.coalescence_axisym(Oh=0.3, precision=p), 4.0, 20),
    "coalescence_3d_oh0.119": (lambda p: W.coalescence_3d_replay(Oh=0.119, precision=p), 4.0, 20),
    # the paper's two ablations of the 3-D scheme, each beside its control:
    # no transverse pressure average at Oh 0.3 (the paper's default D3Q15)
    # and zero bulk viscosity at Oh 0.037
    "coalescence_3d_oh0.3": (lambda p: W.coalescence_3d_replay(Oh=0.3, lattice=15, precision=p), 4.0, 20),
    "coalescence_3d_oh0.3_nopavg": (
        lambda p: W.coalescence_3d_replay(Oh=0.3, lattice=15, scheme=1, precision=p), 0.05, 50),
    "coalescence_3d_oh0.037": (lambda p: W.coalescence_3d_replay(Oh=0.037, precision=p), 4.0, 20),
    "coalescence_3d_oh0.037_nobulk": (
        lambda p: W.coalescence_3d_replay(Oh=0.037, scheme=2, precision=p), 0.8, 16),
    "rt_re256": (lambda p: W.rt_paper(Re=256.0, precision=p), 4.5, 18),
    "rt_re3000": (lambda p: W.rt_paper(Re=3000.0, precision=p), 3.5, 14),
}


def checkerboard(p) -> float:
    """Largest amplitude of the grid-scale (-1)^(i+j+k) mode of a 3-D field:
    the alternating sum over each 2 x 2 x 2 block of cells, divided by 8 (a
    pure checkerboard of amplitude A gives A; a smooth field gives a third
    mixed derivative)."""
    d = p[1:] - p[:-1]
    d = d[:, 1:] - d[:, :-1]
    d = d[:, :, 1:] - d[:, :, :-1]
    return float(abs(d).max()) / 8.0


def observe(name: str, s: G.Solver, prob: dict, sc: dict) -> dict:
    """The paper's diagnostics of case `name` for the current state of s."""
    st = s.phase_stats()
    out = {"volume": st["volume"]}
    if name.startswith("config"):
        d = s.diagnostics(check=False)
        out.update(mass=d["mass"], mass_abs0=d["mass_abs0"], ke=d["ke"], umax=d["umax"] / sc["U"])
    if name == "config1_static_drop":
        p = s.get("p")
        nx, ny = prob["n"][0], prob["n"][1]
        R = math.sqrt(st["volume"] / math.pi)                   # radius of the liquid region
        out["R_eff"] = R
        out["dp_over_sigma_R"] = (p[0, ny // 2, nx // 2] - p[0, 0, 0]) / (prob["sigma"] / R)
    elif name == "config2_rt":
        nx = prob["n"][0]
        # bubble (light fluid rising) on column x = 0, spike (heavy falling) on x = lambda / 2,
        # relative to the initial mid-height, in lambda
        y_mid = 0.5 * prob["n"][1]
        out["bubble"] = (s.line_crossings(1, 0)[1] - y_mid) / sc["L"]
        out["spike"] = (s.line_crossings(1, nx // 2)[0] - y_mid) / sc["L"]
    elif name == "config3_rising_bubble":
        nx, ny, nz = prob["n"]
        ncell = float(nx * ny * nz)
        vg = ncell - st["volume"]                               # gas cells
        # gas centroid from the box's moment minus the liquid's; rise velocity
        # of the gas as the closed box's zero net flux implies, -V_l w_l / V_g
        out["z_gas"] = (ncell * 0.5 * nz - st["volume"] * st["centroid"][2]) / vg / sc["L"]
        out["w_gas"] = -st["volume"] * st["velocity"][2] / vg / sc["U"]
        ext = s.interface_extent()
        out["z_bottom"], out["z_top"] = ext[2][0] / sc["L"], ext[2][1] / sc["L"]
    elif name.startswith("capillary_wave"):
        # interface on the first cell row (y = 1/2 cell); the mode's amplitude
        # there is cos(k / 2) times that on y = 0, where the paper measures it
        h0 = s.line_crossings(0, 0)[0]
        out["h_tilde"] = (sc["h_eq"] - h0) / (sc["A_p"] * math.cos(sc["k"] / 2.0))
    elif name == "falling_drop":
        ext = s.interface_extent()
        out["U_drop"] = st["velocity"][0] / sc["U"]
        out["z_c"] = st["centroid"][0] / sc["L"]
        out["aspect"] = (ext[0][1] - ext[0][0]) / (2.0 * ext[1][1])
    elif name.startswith("coalescence_axisym"):
        out["R_r"] = s.line_crossings(1, 0)[1] / sc["L"]
        out["U_drop"] = st["velocity"][0] / sc["U"]
        # half length on the axis: the 3-D case's R_x
        out["R_axis"] = s.line_crossings(0, 0)[1] / sc["L"]
    elif name.startswith("coalescence_3d"):
        out["R_x"] = s.line_crossings(0, 0, 0)[1] / sc["L"]
        out["W_drop"] = st["velocity"][2] / sc["U"]
        # bridge radius on the contact plane x = 0 (along y at z = 0): the
        # axisymmetric case's R_r
        out["R_neck"] = s.line_crossings(1, 0, 0)[1] / sc["L"]
        # grid-scale pressure mode in units of the drop's Laplace pressure 2 sigma / R
        out["p_cb"] = checkerboard(s.get("p")) / (2.0 * prob["sigma"] / sc["L"])
    elif name.startswith("rt"):
        ny = prob["n"][1]
        out["bubble"] = s.line_crossings(0, 0)[0] / sc["L"]
        out["spike"] = s.line_crossings(0, ny - 1)[1] / sc["L"]
    return out


def run(name: str, precision: str = "fp64", t_end: float | None = None, n_out: int | None = None,
        device: str = "cuda:0") -> dict:
    build, t_def, n_def = CASES[name]
    prob, state, sc = build(precision)
    # a problem statement in dimensionless groups is mapped to lattice units
    # by the library (gpe_params_from_dimensionless), as the solver does
    prob = G.lattice_problem(prob)
    sc = W.reporting_units(sc, prob)
    t_end = t_def if t_end is None else t_end
    n_out = n_def if n_out is None else n_out
    total = int(round(t_end * sc["T"]))
    s = G.Solver(prob, state, device=device)
    nx, ny, nz = prob["n"]
    series = [dict(t=0.0, **observe(name, s, prob, sc))]
    vol0 = series[0]["volume"]
    done, wall = 0, 0.0
    for q in range(1, n_out + 1):
        target = total * q // n_out
        t0 = time.perf_counter()
        s.run(target - done)
        s.synchronize()
        wall += time.perf_counter() - t0
        done = target
        d = s.diagnostics(check=False)
        row = dict(t=done / sc["T"], **observe(name, s, prob, sc))
        row["finite"] = d["finite"]
        series.append(row)
        if not d["finite"]:
            break
    s.close()
    for row in series:
        row["volume"] = row["volume"] / vol0 if vol0 else math.nan
        if "mass" in row:
            row["mass_drift"] = abs(row["mass"] - series[0]["mass"]) / row["mass_abs0"]
    return {"case": name, "precision": precision, "grid": list(prob["n"]), "steps": done,
            "steps_per_time_unit": sc["T"], "wall_s": round(wall, 3),
            "mlups": round(nx * ny * nz * done / max(wall, 1e-9) / 1e6, 1), "series": series}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="*", default=list(CASES))
    ap.add_argument("--precision", default="fp64", choices=("fp64", "fp32"))
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    G.lib()
    results = []
    for name in args.names:
        r = run(name, args.precision)
        results.append(r)
        print(json.dumps(r), flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(results, fh, indent=1)


if __name__ == "__main__":
    main()
