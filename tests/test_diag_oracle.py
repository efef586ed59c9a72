"""Pins of the CPU reference of the experiment diagnostics
(oracle/diag_oracle.py) against closed forms: exact volumes and centroids of
box-shaped regions (with the axisymmetric r weight summed in closed form),
uniform and linear velocity fields, exact crossings of linear profiles and
of a sphere's tanh profile on the line through its centre."""
import math

import numpy as np
import pytest

from oracle import diag_oracle as D
from paper_2011_00814_amd import workloads as W


def test_box_region_volume_centroid_and_uniform_velocity_3d():
    prob = W.base_problem(dim=3, n=(10, 8, 6), bc=(1, 1, 2, 2, 0, 0))
    st = W.zero_state(prob)
    st["phi"][:] = -1.0
    st["phi"][1:4, 2:7, 3:9] = 0.7  # z 1..3, y 2..6, x 3..8
    for k, val in zip("uvw", (0.3, -0.2, 0.1)):
        st[k][:] = val
    # the boundary-normal faces on walls / symmetry planes are 0, but the box
    # lies inside, so every centre mean there is the uniform value
    st["u"][:, :, 0] = 0.0
    st["v"][:, 0, :] = 0.0
    vol, c, v = D.phase_stats(prob, st)
    assert vol == 3 * 5 * 6
    assert np.allclose(c, (6.0, 4.5, 2.5), atol=1e-14)
    assert np.allclose(v, (0.3, -0.2, 0.1), atol=1e-15)


def test_axisymmetric_weight_and_linear_velocity():
    # region: r-rows 0..J-1, z columns 2..7; sum of r over rows = J^2 / 2 per column
    nz, nr, J = 12, 9, 5
    prob = W.base_problem(dim=2, n=(nz, nr, 1), bc=(1, 1, 2, 1, 0, 0), axisym=1)
    st = W.zero_state(prob)
    st["phi"][:] = -1.0
    st["phi"][0, :J, 2:8] = 1.0
    # axial face velocity linear in z: u_face(i) = i  ->  centre mean i + 1/2
    st["u"][0] = np.arange(nz)[None, :] * np.ones((nr, 1))
    vol, c, v = D.phase_stats(prob, st)
    assert vol == pytest.approx(6 * J * J / 2, abs=1e-12)
    assert c[0] == pytest.approx(5.0, abs=1e-12)
    # r-weighted centroid: sum (j+1/2)^2 / sum (j+1/2) over rows 0..J-1
    rr = np.arange(J) + 0.5
    assert c[1] == pytest.approx(float((rr ** 2).sum() / rr.sum()), abs=1e-12)
    assert v[0] == pytest.approx(5.0, abs=1e-12)  # mean of i + 1/2 over columns 2..7
    assert math.isnan(c[2])


def test_crossings_of_linear_profiles_are_exact():
    prob = W.base_problem(dim=2, n=(20, 3, 1), bc=(1, 1, 1, 1, 0, 0))
    st = W.zero_state(prob)
    x = np.arange(20) + 0.5
    for j, (a, b) in enumerate(((4.3, 15.8), (7.0, 12.25), (9.2, 10.9))):
        # a tent: positive between a and b, slope 1 on both sides
        st["phi"][0, j] = np.minimum(x - a, b - x)
    for j, (a, b) in enumerate(((4.3, 15.8), (7.0, 12.25), (9.2, 10.9))):
        f, l = D.line_crossings(prob, st, 0, j)
        assert f == pytest.approx(a, abs=1e-13) and l == pytest.approx(b, abs=1e-13)
    ext = D.interface_extent(prob, st)
    assert ext[0][0] == pytest.approx(4.3, abs=1e-13) and ext[0][1] == pytest.approx(15.8, abs=1e-13)
    assert math.isnan(ext[2][0])


def test_sphere_extent_through_its_centre():
    n, R, Wd = 40, 11.3, 3.0
    prob = W.base_problem(dim=3, n=(n, n, n))
    x, y, z = W._centres(prob)
    c = (20.5, 18.5, 21.5)  # on cell-centre lines
    r = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
    st = W.zero_state(prob)
    st["phi"] = np.tanh(2 * (R - r) / Wd)
    # on the line through the centre the profile is tanh(2 (R - |x - c|) / W),
    # odd about each crossing, so linear interpolation between the two
    # centres errs by O(dx^3 (2/W)^2) ~ 0.01 cell
    f, l = D.line_crossings(prob, st, 0, 18, 21)
    assert f == pytest.approx(c[0] - R, abs=0.02) and l == pytest.approx(c[0] + R, abs=0.02)
    ext = D.interface_extent(prob, st)
    for a in range(3):
        assert ext[a][0] == pytest.approx(c[a] - R, abs=0.02) and ext[a][1] == pytest.approx(c[a] + R, abs=0.02)
    # the extent is attained on the line through the centre
    assert ext[0] == (f, l)
    vol, cen, _ = D.phase_stats(prob, st)
    assert abs(vol - 4 / 3 * math.pi * R ** 3) < 0.01 * vol
    assert np.allclose(cen, c, atol=1e-9)


def test_periodic_centre_velocity_wraps():
    prob = W.base_problem(dim=2, n=(6, 4, 1), bc=(0, 0, 1, 1, 0, 0))
    st = W.zero_state(prob)
    st["phi"][:] = 1.0
    st["u"][0, :, :] = np.arange(6)[None, :]
    # centre means (i + (i+1) % 6) / 2: 0.5, 1.5, ..., 4.5, 2.5 -> mean 15/6
    _, _, v = D.phase_stats(prob, st)
    assert v[0] == pytest.approx(15 / 6, abs=1e-15)
