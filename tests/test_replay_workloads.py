"""The paper's experiment set-ups (Sec. 4), stated in their dimensionless
groups and mapped to lattice units by the oracle's own mapping, reproduce
those groups; the replay driver's cases are well formed."""
import math

import numpy as np
import pytest

from oracle.problem import lattice_problem
from paper_2011_00814_amd import workloads as W


def _lattice(built):
    prob, st, sc = built
    lat = lattice_problem(prob)
    return lat, st, W.reporting_units(sc, lat)


def test_falling_drop_groups():
    p, st, sc = _lattice(W.falling_drop_axisym(NL=50))
    NL, D = 50.0, 100.0
    assert p["n"] == (1200, 400, 1) and p["axisym"] == 1
    assert p["bc"][:4] == (W.WALL, W.WALL, W.SYMMETRY, W.WALL)
    rho_g = p["rho_g"]
    assert abs(1.0 / rho_g - 1.15) < 1e-12 and p["eta_l"] == p["eta_g"]
    Eo = p["g"][0] * (1.0 - rho_g) * D * D / p["sigma"]
    Oh = p["eta_l"] / math.sqrt(D * p["sigma"])
    assert abs(Eo - 144.0) < 1e-9 and abs(Oh - 0.0466) < 1e-12
    assert abs(p["sigma"] / p["eta_l"] - NL / 4000.0) < 1e-15       # U_c = sigma / eta_L, N_t = 4000
    assert abs(p["width"] / NL - 0.06) < 1e-15                       # Cn
    assert abs((NL / 4000.0) * NL * NL / p["mob"] - 1000.0) < 1e-9   # Pe
    assert p["rho_ref"] == rho_g and p["g"][1] == 0.0
    assert abs(sc["T"] - math.sqrt(D / p["g"][0])) < 1e-9 and abs(sc["U"] * sc["T"] - D) < 1e-9
    # drop of radius R at (2R, 0)
    assert st["phi"][0, 0, 100] > 0.99 and st["phi"][0, 0, 160] < -0.99


@pytest.mark.parametrize("Oh,Nt", [(0.037, 400), (0.119, 400), (0.3, 2000)])
def test_coalescence_axisym_groups(Oh, Nt):
    p, st, sc = _lattice(W.coalescence_axisym(NL=40, Oh=Oh))
    assert p["n"] == (120, 120, 1) and p["bc"][:4] == (W.SYMMETRY,) * 4 and p["ch_transport"] == 1
    Uc = 40.0 / Nt
    assert abs(p["eta_l"] / math.sqrt(p["sigma"] * 40.0) - Oh) < 1e-12
    assert abs(p["sigma"] / p["eta_l"] - Uc) < 1e-15
    assert abs(1.0 / p["rho_g"] - 50.0) < 1e-12 and abs(p["eta_l"] / p["eta_g"] - 58.8) < 1e-12
    # capillary-inertial scales
    assert abs(sc["U"] - math.sqrt(p["sigma"] / 40.0)) < 1e-15 and abs(sc["T"] - 40.0 / sc["U"]) < 1e-9
    assert abs(sc["T"] * Oh - Nt) < 1e-6  # T_ci = T_c / Oh


@pytest.mark.parametrize("Re,r_eta", [(256.0, 3.0), (3000.0, 1.0)])
def test_rt_paper_groups(Re, r_eta):
    p, st, sc = _lattice(W.rt_paper(NL=256, Re=Re))
    assert p["n"] == (1024, 128, 1) and p["bc"][:4] == (W.WALL, W.WALL, W.SYMMETRY, W.SYMMETRY)
    Uc = 256.0 / 51200.0
    assert abs(math.sqrt(p["g"][0] * 256.0) - Uc) < 1e-15            # U_c = sqrt(lambda g)
    assert abs(Uc * 256.0 / p["eta_l"] - Re) < 1e-9 and abs(p["eta_l"] / p["eta_g"] - r_eta) < 1e-12
    assert abs((1 - p["rho_g"]) / (1 + p["rho_g"]) - 0.5) < 1e-12      # At
    assert p["sigma"] == 0.0 and p["width"] == 4.0 and p["rho_ref"] == p["rho_g"]
    # interface x = h(y): at y = 0 (bubble side) h = 1.9, at y = 1/2 (spike side) h = 2.1
    x = np.arange(1024) + 0.5
    for j, h in ((0, 1.9), (127, 2.1)):
        y = (j + 0.5) / 256.0
        hh = (2.0 + 0.1 * math.cos(2 * math.pi * (y + 0.5))) * 256.0
        assert abs(hh / 256.0 - h) < 2e-3
        k = int(np.argmax(st["phi"][0, j] < 0))
        assert x[k - 1] < hh < x[k]


def test_replay_cases_are_defined():
    from paper_2011_00814_amd import replays as R

    for name, (build, t_end, n_out) in R.CASES.items():
        assert t_end > 0 and n_out > 0, name


@pytest.mark.parametrize("Oh,Nt,scheme", [(0.037, 400, 2), (0.119, 400, 0), (0.3, 2000, 1)])
def test_coalescence_3d_replay_groups(Oh, Nt, scheme):
    p, st, sc = _lattice(W.coalescence_3d_replay(NL=12, Oh=Oh, scheme=scheme))
    NL = 12.0
    assert p["n"] == (36, 36, 36) and p["bc"] == (W.SYMMETRY,) * 6 and p["scheme"] == scheme
    assert abs(p["eta_l"] / math.sqrt(p["sigma"] * NL) - Oh) < 1e-12
    # the paper's N_t = c N_L (c = 10, or 50 at Oh 0.3) steps per T_c, T_ci = T_c / Oh
    assert abs(sc["T"] * Oh - Nt * NL / 40.0) < 1e-6


def test_checkerboard_measure():
    from paper_2011_00814_amd.replays import checkerboard

    k, j, i = np.meshgrid(np.arange(6), np.arange(5), np.arange(7), indexing="ij")
    cb = (-1.0) ** (i + j + k)
    smooth = 0.3 + 0.1 * i - 0.2 * j + 0.05 * k + 0.01 * i * j + 0.02 * (i * i + k * k)
    assert abs(checkerboard(2.5e-3 * cb) - 2.5e-3) < 1e-15
    assert checkerboard(smooth) < 1e-15               # no i j k term: no response
    assert abs(checkerboard(i * j * k * 1.0) - 1.0 / 8.0) < 1e-15  # third mixed derivative
    assert abs(checkerboard(smooth + 1e-3 * cb) - 1e-3) < 1e-12


def test_rising_bubble_groups():
    """Configuration 3 (3-D rising bubble): D = 32, U_c = sqrt(g D) = 0.03,
    Eo = 10, Mo = 1e-4, density and viscosity ratio 10, M = 0.02."""
    p = lattice_problem(W.rising_bubble_3d()[0])
    D, drho = 32.0, 0.9
    g = -p["g"][2]
    assert p["g"][0] == 0.0 and p["g"][1] == 0.0
    assert abs(math.sqrt(g * D) - 0.03) < 1e-15
    assert abs(g * drho * D * D / p["sigma"] - 10.0) < 1e-12
    assert abs(g * drho * p["eta_l"] ** 4 / p["sigma"] ** 3 - 1e-4) < 1e-16
    assert abs(p["rho_g"] - 0.1) < 1e-16 and abs(p["eta_l"] / p["eta_g"] - 10.0) < 1e-12
    assert abs(p["mob"] - 0.02) < 1e-15 and p["width"] == 2.0 and p["rho_ref"] == 1.0


def test_capillary_wave_groups():
    """Sec. 4.1 on both meshes: Re 1000 with U_c = sigma / eta_L, r = 20."""
    for NL, Nt, Cn, Pe in ((64, 384, 1 / 16, 2e4), (128, 1920, 1 / 32, 4e4)):
        p, st, sc = W.capillary_wave(NL=NL, Nt=Nt, Cn=Cn, Pe=Pe)
        p = lattice_problem(p)
        Uc = NL / Nt
        assert abs(Uc * NL / p["eta_l"] - 1000.0) < 1e-9 and abs(p["sigma"] / p["eta_l"] - Uc) < 1e-15
        assert abs(1 / p["rho_g"] - 20.0) < 1e-12 and abs(p["eta_l"] / p["eta_g"] - 20.0) < 1e-12
        assert abs(Uc * NL * NL / p["mob"] - Pe) < 1e-6 * Pe and abs(p["width"] - Cn * NL) < 1e-15
