"""The paper's experiments on the GPU (marked gpu): the diagnostics kernels
against their CPU reference on GPU-produced states, reduced-size replays
against the oracle, and the first stretch of each full-size replay.
"""
import math
import sys

import numpy as np
import pytest

from paper_2011_00814_amd import workloads as W
from tests.parity_util import compare_states

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpe():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2011_00814_amd import gpe as G

    G.lib()
    return G


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


SMALL = {
    "falling_drop": lambda prec: W.falling_drop_axisym(NL=10, precision=prec),
    "coalescence_axisym": lambda prec: W.coalescence_axisym(NL=12, precision=prec),
    "coalescence_3d": lambda prec: W.coalescence_3d_replay(NL=10, precision=prec),
    "rt_re256": lambda prec: W.rt_paper(NL=32, precision=prec),
}


def _diag_ref(prob, st):
    from oracle import diag_oracle as D

    vol, c, v = D.phase_stats(prob, st)
    ext = D.interface_extent(prob, st)
    return vol, c, v, ext


def _close(a, b, tol):
    return (math.isnan(a) and math.isnan(b)) or abs(a - b) <= tol * max(1.0, abs(b))


@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_diagnostics_kernels_match_reference(gpe, name, precision):
    from oracle import diag_oracle as D

    prob, st, sc = SMALL[name](precision)
    _say(f"[replay diag] {name} {precision} n={prob['n']}")
    s = gpe.Solver(prob, st)
    s.run(30)
    s.synchronize()
    cur = s.state()  # the GPU's own state, converted to FP64
    vol, c, v, ext = _diag_ref(prob, cur)
    ps = s.phase_stats()
    got_ext = s.interface_extent()
    assert _close(ps["volume"], vol, 1e-13)
    for a in range(3):
        assert _close(ps["centroid"][a], c[a], 1e-12) and _close(ps["velocity"][a], v[a], 1e-10), a
        for q in range(2):
            assert _close(got_ext[a][q], ext[a][q], 1e-12), (a, q)
    dim = prob["dim"]
    for axis in range(dim):
        n_other = [prob["n"][b] for b in range(dim) if b != axis]
        for i0 in (0, n_other[0] // 2, n_other[0] - 1):
            i1 = 0 if dim == 2 else n_other[1] // 3
            ref = D.line_crossings(prob, cur, axis, i0, i1)
            got = s.line_crossings(axis, i0, i1)
            assert _close(got[0], ref[0], 1e-12) and _close(got[1], ref[1], 1e-12), (axis, i0, i1)
    with pytest.raises(gpe.GpeError):
        s.line_crossings(0, prob["n"][1], 0)  # index beyond the grid
    s.close()


@pytest.mark.parametrize("name", list(SMALL))
def test_reduced_replays_match_oracle(gpe, oracle, name):
    prob, st, sc = SMALL[name]("fp64")
    nsteps = 60
    _say(f"[replay parity] {name} n={prob['n']} steps={nsteps}")
    ref = oracle.run(prob, st, nsteps)
    s = gpe.Solver(prob, st)
    s.run(nsteps)
    s.synchronize()
    out = s.state()
    s.close()
    errs, raw = compare_states(prob, out, ref)
    assert all(e <= 1e-11 for e in errs.values()), (errs, raw)


@pytest.mark.parametrize("name,frac", [("falling_drop", 0.1), ("coalescence_axisym_oh0.119", 0.1),
                                       ("coalescence_3d_oh0.119", 0.05), ("rt_re256", 0.1)])
def test_full_size_replay_start(gpe, name, frac):
    from paper_2011_00814_amd import replays as R

    _say(f"[replay full] {name} first {frac} of the run")
    t_end = R.CASES[name][1] * frac
    r = R.run(name, "fp64", t_end=t_end, n_out=4)
    ser = r["series"]
    assert all(row.get("finite", 1) == 1 for row in ser)
    assert all(abs(row["volume"] - 1.0) < 0.02 for row in ser), [row["volume"] for row in ser]
    if name == "falling_drop":
        # the drop accelerates from rest along +z and stays nearly spherical
        u = [row["U_drop"] for row in ser]
        assert u[0] == 0.0 and all(b > a for a, b in zip(u[1:], u[2:])) and u[-1] > 0.03
        assert all(abs(row["aspect"] - 1.0) < 0.1 for row in ser)
    elif name.startswith("coalescence_axisym"):
        rr = [row["R_r"] for row in ser]
        assert all(b > a for a, b in zip(rr, rr[1:]))       # the bridge widens
    elif name.startswith("coalescence_3d"):
        rx = [row["R_x"] for row in ser]
        assert rx[-1] < rx[0] <= 2.0 + 1e-9                 # the merged drop shortens along x
    else:
        assert ser[-1]["spike"] > ser[0]["spike"] and ser[-1]["bubble"] < ser[0]["bubble"]


@pytest.mark.parametrize("oh", ["0.037", "0.119", "0.3"])
def test_axisymmetric_and_3d_coalescence_agree(gpe, oh):
    """The same coalescence computed in axisymmetric geometry (D2Q9 CH
    stencils, cylindrical terms) and in 3-D (one eighth of the domain;
    D3Q19, or the paper's D3Q15 at Oh 0.3): the bridge radius and the half
    length along the line of centres agree over the whole run."""
    from paper_2011_00814_amd import replays as R

    _say(f"[replay cross] coalescence Oh {oh} axisymmetric vs 3-D, t <= 4 T_ci")
    a = R.run(f"coalescence_axisym_oh{oh}", "fp64", t_end=4.0, n_out=8)["series"]
    b = R.run(f"coalescence_3d_oh{oh}", "fp64", t_end=4.0, n_out=8)["series"]
    assert len(a) == len(b) == 9
    for ra, rb in zip(a[1:], b[1:]):
        # measured: within 0.0024 R (bridge) and 0.005 R (half length) at the three Oh
        assert abs(ra["R_r"] - rb["R_neck"]) < 0.01, (ra, rb)
        assert abs(ra["R_axis"] - rb["R_x"]) < 0.01, (ra, rb)
    # the drops merge: the half length falls from 2 R below the radius of
    # the merged drop, 2^(1/3) R, during the first oscillation
    assert min(r["R_x"] for r in b) < 2 ** (1 / 3)


def test_paper_ablations_3d_coalescence(gpe):
    """The paper's two ablations of its 3-D scheme (Sec. 4, drop coalescence
    in 3-D), at the paper's resolution: without the transverse pressure
    average the Oh = 0.3 run (D3Q15) blows up through a grid-scale pressure
    mode at t ~ 0.02 T_ci, while the paper's scheme stays smooth; with zero
    bulk viscosity the Oh = 0.037 run grows a checkerboard pressure mode
    by t = 0.4 T_ci that the paper's scheme does not have."""
    from paper_2011_00814_amd import replays as R

    _say("[replay ablation] no pressure average, Oh 0.3, t <= 0.05 T_ci")
    bad = R.run("coalescence_3d_oh0.3_nopavg", "fp64", t_end=0.05, n_out=10)["series"]
    good = R.run("coalescence_3d_oh0.3", "fp64", t_end=0.05, n_out=10)["series"]
    assert all(row.get("finite", 1) == 1 for row in good)
    assert max(row["p_cb"] for row in good) < 0.1
    assert bad[-1].get("finite", 1) == 0                   # stopped by the instability
    assert bad[-1]["t"] <= 0.05 + 1e-12 and bad[1]["p_cb"] < 1.0
    _say("[replay ablation] zero bulk viscosity, Oh 0.037, t <= 0.4 T_ci")
    nob = R.run("coalescence_3d_oh0.037_nobulk", "fp64", t_end=0.4, n_out=4)["series"]
    ref = R.run("coalescence_3d_oh0.037", "fp64", t_end=0.4, n_out=4)["series"]
    assert all(row.get("finite", 1) == 1 for row in nob + ref)
    assert nob[-1]["p_cb"] > 1.0 and ref[-1]["p_cb"] < 0.01
    assert nob[-1]["p_cb"] > 100.0 * ref[-1]["p_cb"]


def test_capillary_wave_meshes_against_prosperetti(gpe, oracle):
    """The capillary wave (Sec. 4.1) on the paper's two meshes against the
    closed-form solution over 30 T_c: the coarse mesh within the bounds the
    oracle meets, the refined mesh closer to it (the paper's refinement
    study), and the coarse series equal to the oracle's."""
    from paper_2011_00814_amd import replays as R
    from tests.closed_forms import prosperetti

    def errors(name, series):
        prob, _, sc = R.CASES[name][0]("fp64")
        prob = gpe.lattice_problem(prob)  # the parameters the solver ran with
        return [(row["t"], row["h_tilde"] - prosperetti(row["t"] * sc["T"], prob["sigma"], sc["k"],
                                                         prob["rho_l"], prob["rho_g"], prob["eta_l"]))
                for row in series[1:]]

    _say("[replay] capillary wave N_L = 64 and 128, 30 T_c")
    coarse = R.run("capillary_wave", "fp64")["series"]
    fine = R.run("capillary_wave_fine", "fp64")["series"]
    assert all(row.get("finite", 1) == 1 for row in coarse + fine)
    ec, ef = errors("capillary_wave", coarse), errors("capillary_wave_fine", fine)
    assert max(abs(e) for t, e in ec if t <= 3) < 0.06 and max(abs(e) for _, e in ec) < 0.13, ec
    # measured: largest deviation 0.118 (N_L = 64) and 0.079 (N_L = 128)
    assert max(abs(e) for _, e in ef) < 0.8 * max(abs(e) for _, e in ec), (ec, ef)
    # the first 3 T_c of the coarse mesh against the oracle
    prob, st, sc = R.CASES["capillary_wave"][0]("fp64")
    state = st
    for q in range(1, 4):
        state = oracle.run(prob, state, int(sc["T"]))
        row = state["phi"][0, 0]
        i = int(np.where((row[:-1] < 0) & (row[1:] >= 0))[0][0])
        h0 = i + 0.5 + row[i] / (row[i] - row[i + 1])
        ref = (sc["h_eq"] - h0) / (sc["A_p"] * math.cos(sc["k"] / 2.0))
        assert abs(coarse[q]["h_tilde"] - ref) < 1e-9, (q, coarse[q]["h_tilde"], ref)


def test_baseline_configs_full_length(gpe):
    """The three benchmark configurations at full size and length: the
    static drop 64^2 (1000 steps, FP64), Rayleigh-Taylor 256 x 1024 (20,000
    steps, FP64 and FP32) and the rising bubble 128 x 128 x 256 (10,000
    steps, FP32), with the quantities they record."""
    from paper_2011_00814_amd import replays as R

    _say("[replay] configuration 1: static drop 64^2, 1000 steps")
    c1 = R.run("config1_static_drop", "fp64")["series"]
    assert all(row.get("finite", 1) == 1 for row in c1)
    assert max(row["mass_drift"] for row in c1) < 1e-12
    assert c1[-1]["umax"] < 1e-3                    # spurious currents decay (measured 9e-5)

    _say("[replay] configuration 2: Rayleigh-Taylor 256 x 1024, 20,000 steps")
    rt = {p: R.run("config2_rt", p)["series"] for p in ("fp64", "fp32")}
    a = rt["fp64"]
    assert all(row.get("finite", 1) == 1 for row in a + rt["fp32"])
    assert max(row["mass_drift"] for row in a) < 1e-12
    assert max(row["mass_drift"] for row in rt["fp32"]) < 1e-6   # measured 2.9e-7 over 20,000 steps
    assert all(q["bubble"] > p["bubble"] for p, q in zip(a, a[1:]))   # the bubble rises
    assert all(q["spike"] < p["spike"] for p, q in zip(a, a[1:]))     # the spike falls faster
    assert a[-1]["bubble"] > 0.7 and a[-1]["spike"] < -1.1            # measured 0.797, -1.274
    for p, q in zip(a, rt["fp32"]):
        assert abs(p["bubble"] - q["bubble"]) < 1e-3 and abs(p["spike"] - q["spike"]) < 1e-3

    _say("[replay] configuration 3: rising bubble 128 x 128 x 256, 10,000 steps")
    b = R.run("config3_rising_bubble", "fp32")["series"]
    assert all(row.get("finite", 1) == 1 for row in b)
    assert max(row["mass_drift"] for row in b) < 2e-7     # measured 4.8e-8 after 10,000 steps
    z = [row["z_gas"] for row in b]
    t = [row["t"] for row in b]
    assert all(q > p for p, q in zip(z, z[1:]))
    rise = [(z2 - z1) / (t2 - t1) for z1, z2, t1, t2 in zip(z[1:], z[2:], t[1:], t[2:])]
    assert all(0.5 < v < 0.7 for v in rise), rise   # measured 0.57-0.58 sqrt(g D) after 1 T_c
    assert b[-1]["z_top"] < 8.0                      # below the top wall (8 D)
