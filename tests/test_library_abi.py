"""Host-side checks of the C-ABI library (no GPU needed, no compute calls):
the library loads and exports every function include/gpe.h declares, the
problem-statement mapping and workspace sizing behave as documented, and
invalid parameter sets are rejected."""
import ctypes

import pytest

from paper_2011_00814_amd import workloads as W


@pytest.fixture(scope="module")
def G():
    from paper_2011_00814_amd import gpe

    try:
        gpe.lib()
    except (ImportError, OSError) as e:  # library not built in this checkout
        pytest.fail(f"libgpe.so not loadable: {e}")
    return gpe


def test_exports_every_header_symbol(G):
    names = G.header_functions()
    assert len(names) == 23
    L = G.lib()
    for n in names:
        assert hasattr(L, n), n


def test_exports_every_learn_header_symbol(G):
    from paper_2011_00814_amd import learn

    names = learn.header_functions()
    assert len(names) == 15
    L = G.lib()
    for n in names:
        assert hasattr(L, n), n


def test_struct_sizes_match_header_layout(G):
    # 8-byte aligned layouts with no implicit padding
    assert ctypes.sizeof(G.gpe_params) == 4 * 14 + 8 * 13 + 4 * 2 + 8 * 6
    assert ctypes.sizeof(G.gpe_problem) == 4 * 14 + 8 * 11 + 4 * 2
    assert ctypes.sizeof(G.gpe_diag) == 8 * 9 + 4 * 2


def test_params_from_dimensionless_capillary_wave(G):
    """The paper's capillary-wave set-up: N_L = 64, N_t = 384, Re = 1000,
    r = 20, Cn = 0.0625, Pe = 2e4, U_c = sigma / eta_L."""
    pr = G.gpe_problem()
    pr.geometry, pr.precision = G.GPE_GEOM_2D, G.GPE_FP64
    pr.n[:] = [64, 32, 1]
    pr.bc[:] = [1, 1, 2, 2, 0, 0]
    pr.lattice = 9
    pr.capillary_scale = 1
    pr.N_L, pr.N_t, pr.r_rho, pr.r_eta, pr.Re, pr.Pe, pr.Cn = 64, 384, 20, 20, 1000, 2e4, 0.0625
    P = G.gpe_params_from_dimensionless(pr)
    Uc = 64 / 384
    assert P.dt == 1.0 and abs(P.cs2 - 1 / 3) < 1e-16
    assert abs(P.eta_l - Uc * 64 / 1000) < 1e-15
    assert abs(P.sigma - Uc * P.eta_l) < 1e-16
    assert abs(P.mobility - Uc * 64 * 64 / 2e4) < 1e-15
    assert P.width == 4.0 and abs(P.rho_g - 0.05) < 1e-16 and abs(P.eta_g - P.eta_l / 20) < 1e-16


def test_params_from_dimensionless_gravity_and_reference_density(G):
    pr = G.gpe_problem()
    pr.geometry, pr.precision = G.GPE_GEOM_2D, G.GPE_FP32
    pr.n[:] = [256, 1024, 1]
    pr.bc[:] = [0, 0, 1, 1, 0, 0]
    pr.lattice = 9
    pr.N_L, pr.N_t, pr.r_rho, pr.r_eta, pr.Re, pr.Pe, pr.Cn = 256, 5120, 3, 1, 3000, 8e4, 2 / 256
    pr.G[:] = [0, -1, 0]
    pr.rho_ref_kind = 2
    P = G.gpe_params_from_dimensionless(pr)
    Uc = 256 / 5120
    assert abs(P.g[1] + Uc * Uc / 256) < 1e-18
    assert abs(P.rho_ref - 1 / 3) < 1e-16 and P.sigma == 0.0


def test_workspace_bytes(G):
    prob, _ = W.static_drop_2d()
    P = G.params_from_problem(prob)
    n = 64 * 64 * 8
    align = lambda b: (b + 255) // 256 * 256
    # 2-D: 3 state + 3 + 3 stage fields, phi*, one CH stage buffer, the kept CH increment, 2 face sums
    assert G.gpe_workspace_bytes(P) == 14 * align(n) + align((512 * 8 + 8) * 8)
    prob3, _ = W.rising_bubble_3d(nx=256, ny=256, nz=256, precision="fp32")
    P3 = G.params_from_problem(prob3)
    n3 = 256 ** 3 * 4
    assert G.gpe_workspace_bytes(P3) == 19 * n3 + align((512 * 8 + 8) * 8)


@pytest.mark.parametrize("mutate", [
    lambda P: setattr(P, "geometry", 7),
    lambda P: P.n.__setitem__(0, 2),
    lambda P: P.n.__setitem__(2, 4),            # 2-D must have n[2] == 1
    lambda P: P.bc.__setitem__(0, 1),           # periodic on one side only
    lambda P: setattr(P, "lattice", 15),        # 3-D lattice in 2-D
    lambda P: setattr(P, "dt", 0.0),
    lambda P: setattr(P, "width", -1.0),
    lambda P: setattr(P, "rho_g", 0.0),
    lambda P: setattr(P, "ch_transport", 2),    # only 0 (conservative) and 1 (advective)
    lambda P: setattr(P, "scheme", 1),          # ablation variants are 3-D only
])
def test_invalid_params_rejected(G, mutate):
    prob, _ = W.static_drop_2d()
    P = G.params_from_problem(prob)
    assert G.gpe_workspace_bytes(P) > 0
    mutate(P)
    assert G.gpe_workspace_bytes(P) == 0


@pytest.mark.parametrize("scheme,ok", [(0, True), (1, True), (2, True), (3, True), (4, False), (-1, False)])
def test_scheme_flags_3d(G, scheme, ok):
    prob, _ = W.rising_bubble_3d(nx=8, ny=8, nz=8)
    P = G.params_from_problem(dict(prob, scheme=scheme))
    assert (G.gpe_workspace_bytes(P) > 0) == ok


def test_axisym_requires_axis_symmetry_bc(G):
    prob, _ = W.axisym_drop()
    P = G.params_from_problem(prob)
    assert G.gpe_workspace_bytes(P) > 0
    P.bc[2] = 1
    assert G.gpe_workspace_bytes(P) == 0


def test_strerror(G):
    for code in (0, -1, -2, -3, -4, -5):
        assert G.gpe_strerror(code) and "unknown" not in G.gpe_strerror(code)


def _stability_code(G, prob):
    """gpe_init_state checks the stability estimates before it touches the
    workspace: with a NULL workspace it returns GPE_EUNSTABLE or
    GPE_EWORKSPACE without any device call."""
    P = G.params_from_problem(prob)
    h = ctypes.c_void_p()
    return G.lib().gpe_init_state(ctypes.byref(P), None, 0, None, None, None, ctypes.byref(h))


def test_gpu_test_workloads_pass_stability_estimate(G):
    from tests import test_gpu_parity as T

    probs = [T._case(name)[0] for name in T.CASES]
    probs += [W.static_drop_2d()[0], W.rising_bubble_3d(nx=256, ny=256, nz=256)[0],
              W.rayleigh_taylor_2d()[0], W.rising_bubble_3d()[0]]
    for dim, bc in ((2, (1, 1, 2, 2, 0, 0)), (3, (1, 1, 0, 0, 2, 2))):
        n = (70, 37, 1) if dim == 2 else (40, 19, 40)
        probs.append(W.base_problem(dim=dim, n=n, bc=bc, rho_l=1.0, rho_g=0.25, eta_l=0.03,
                                    eta_g=0.01, sigma=0.01, mob=0.02))
    for prob in probs:
        assert _stability_code(G, prob) == G.GPE_EWORKSPACE, prob


def test_unstable_time_step_rejected_on_host(G):
    prob, _ = W.static_drop_2d()
    prob["mob"] = 0.2
    assert _stability_code(G, prob) == G.GPE_EUNSTABLE
    prob["allow_unstable"] = 1
    assert _stability_code(G, prob) == G.GPE_EWORKSPACE
