"""Host-side checks of the batched ensemble (no GPU): the input recipe of the
ensemble workload against closed forms and its own constraints, and the
C-ABI's batch validation and workspace sizing."""
import ctypes
import math

import numpy as np
import pytest

from paper_2011_00814_amd import workloads as W


@pytest.fixture(scope="module")
def G():
    from paper_2011_00814_amd import gpe

    gpe.lib()
    return gpe


def test_d2q9_laplacian_spectrum_maximum_is_16_over_3():
    """The recipe's CH bound uses lam = 16/3: brute-force maximum over a fine
    wavenumber grid of 6 sum_i w_i (1 - cos(k . e_i)) with the D2Q9 weights."""
    k = np.linspace(0, math.pi, 241)
    kx, ky = np.meshgrid(k, k, indexing="ij")
    s = np.zeros_like(kx)
    for ex in (-1, 0, 1):
        for ey in (-1, 0, 1):
            nnz = abs(ex) + abs(ey)
            if nnz == 0:
                continue
            w = 1 / 9 if nnz == 1 else 1 / 36
            s += w * (1 - np.cos(kx * ex + ky * ey))
    assert abs(6 * s.max() - 16 / 3) < 1e-12


def test_recipe_dt_bounds():
    # CH-limited: nu small -> dt = 0.8 * 2 / (M lam (8a + kappa lam)) with
    # a = 3/8, kappa = 3/4 (W = 2): 8a = 3, kappa lam = 4
    assert abs(W.recipe_dt(1, 1, 1e-3, 1e-3, 0.05, 2.0) - 0.8 * 2 / (0.05 * 16 / 3 * 7)) < 1e-15
    # viscosity-limited: nu_max = eta_g / rho_g
    dt = W.recipe_dt(1.0, 0.01, 0.1, 0.01, 0.05, 2.0)
    assert abs(dt - 0.8 * 2.5127 / (3 * 1.0 * 8)) < 1e-15
    assert W.recipe_dt(1, 1, 0, 0, 0, 2.0) == 1.0


def test_ellipse_profile():
    prob = W.base_problem(dim=2, n=(64, 64, 1))
    phi = W.ellipse_phi(prob, 10.0, 0.2, (32.0, 32.0), 2.0)
    # at the centre: tanh(2 R / W); zero level set on the semi-axes
    assert abs(phi[0, 31, 31] - math.tanh(2 * 10 * (1 - math.hypot(0.5 / 12, 0.5 / 8)) / 2)) < 1e-14
    x = 32.0 + 12.0  # a = 12: the cell centre x = 43.5 is 0.5 inside
    assert phi[0, 31, 43] > 0 > phi[0, 31, 44]
    assert phi[0, 31 + 8, 31] > 0 > phi[0, 31 + 9, 31]  # b = 8 (y = 39.5 inside, 40.5 outside)
    assert np.allclose(phi, phi[:, :, ::-1]) and np.allclose(phi, phi[:, ::-1, :])


def test_ensemble_recipe_constraints_and_determinism():
    a = W.ensemble_cases(512, seed=0)
    b = W.ensemble_cases(512, seed=0)
    assert [x["n"] for x in a] == [x["n"] for x in b] and [x["dt"] for x in a] == [x["dt"] for x in b]
    sizes = [x["n"][0] for x in a]
    assert set(sizes) == set(W.ENSEMBLE_SIZES)
    for x in a:
        N = x["n"][0]
        R = x["init"]["radius"]
        assert 10 <= R <= 30 and 1.2 * R + 2 * 2.0 <= 0.45 * N
        assert 1 <= x["meta"]["r_rho"] <= 100 and 1 <= x["meta"]["r_eta"] <= 50
        assert abs(x["cs2"] * 3 * x["dt"] ** 2 - 1) < 1e-12 and 0 < x["dt"] <= 1
        assert x["bc"] == (0,) * 6 and x["precision"] == "fp32"
    assert W.ensemble_cases(8, seed=1)[0]["n"] != a[0]["n"] or W.ensemble_cases(8, seed=1)[0]["dt"] != a[0]["dt"]


def test_every_recipe_case_passes_the_library_stability_check(G):
    for x in W.ensemble_cases(512, seed=0):
        P = G.params_from_problem(x)
        h = ctypes.c_void_p()
        rc = G.lib().gpe_init_state(ctypes.byref(P), None, 0, None, None, None, ctypes.byref(h))
        assert rc == G.GPE_EWORKSPACE  # valid and stable; only the workspace is missing


def test_ensemble_workspace_and_batch_validation(G):
    cases = W.ensemble_cases(6, seed=3)
    P = [G.params_from_problem(x) for x in cases]
    total = G.gpe_ensemble_workspace_bytes(P)
    assert total >= sum(G.gpe_workspace_bytes(p) for p in P)
    # header: 3 flow + 2 CH argument blocks per case, tiles, flags, tables
    assert total - sum(G.gpe_workspace_bytes(p) for p in P) < 1 << 20
    assert G.gpe_ensemble_workspace_bytes([]) == 0
    # the batch kernels implement the conservative CH transport only
    adv = G.params_from_problem(dict(W.ensemble_cases(2, seed=0)[0], ch_transport=1))
    assert G.gpe_workspace_bytes(adv) > 0
    assert G.gpe_ensemble_workspace_bytes([P[0], adv]) == 0
    mixed = [G.params_from_problem(dict(cases[0], precision="fp64"))] + P[1:]
    assert G.gpe_ensemble_workspace_bytes(mixed) == 0
    prob3, _ = W.rising_bubble_3d(nx=32, ny=32, nz=32, precision="fp32")
    assert G.gpe_ensemble_workspace_bytes(P + [G.params_from_problem(prob3)]) == 0
    bad = G.params_from_problem(dict(cases[0]))
    bad.n[0] = 2
    assert G.gpe_ensemble_workspace_bytes([bad]) == 0
    # create: invalid batch -> EINVAL, missing workspace -> EWORKSPACE
    h = ctypes.c_void_p()
    arr = (G.gpe_params * 1)(bad)
    assert G.lib().gpe_ensemble_create(arr, 1, None, 0, None, ctypes.byref(h)) == G.GPE_EINVAL
    arr = (G.gpe_params * len(P))(*P)
    assert G.lib().gpe_ensemble_create(arr, len(P), None, 0, None, ctypes.byref(h)) == G.GPE_EWORKSPACE
    assert not G.lib().gpe_ensemble_case(None, 0)


def test_ellipse_init_kind_validation(G):
    x = dict(W.ensemble_cases(1, seed=0)[0])
    x["init"] = dict(x["init"], amp=1.0)
    P = G.params_from_problem(x)
    assert G.gpe_workspace_bytes(P) == 0  # |amp| < 1 required
