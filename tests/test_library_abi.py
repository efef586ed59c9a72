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
    assert len(names) == 26
    L = G.lib()
    for n in names:
        assert hasattr(L, n), n


def test_exports_every_learn_header_symbol(G):
    from paper_2011_00814_amd import learn

    names = learn.header_functions()
    assert len(names) == 16
    L = G.lib()
    for n in names:
        assert hasattr(L, n), n


def test_struct_sizes_match_header_layout(G):
    # 8-byte aligned layouts with no implicit padding
    assert ctypes.sizeof(G.gpe_params) == 4 * 14 + 8 * 13 + 4 * 4 + 8 * 6
    assert ctypes.sizeof(G.gpe_problem) == 4 * 20 + 8 * 19
    assert ctypes.sizeof(G.gpe_diag) == 8 * 9 + 4 * 2


def _base(**kw):
    st = W.statement(dim=2, n=(64, 32, 1), bc=(1, 1, 2, 2, 0, 0), N_L=64.0, N_t=384.0, r_rho=20.0, r_eta=20.0,
                     visc="Re", Re=1000.0, st="capillary", Pe=2e4, Cn=0.0625)
    st.update(kw)
    return st


def test_params_from_dimensionless_capillary_wave(G):
    """The paper's capillary-wave set-up: N_L = 64, N_t = 384, Re = 1000,
    r = 20, Cn = 0.0625, Pe = 2e4, U_c = sigma / eta_L."""
    P = G.gpe_params_from_dimensionless(G.problem_struct(_base()))
    Uc = 64 / 384
    assert P.dt == 1.0 and abs(P.cs2 - 1 / 3) < 1e-16
    assert abs(P.eta_l - Uc * 64 / 1000) < 1e-15
    assert abs(P.sigma - Uc * P.eta_l) < 1e-16
    assert abs(P.mobility - Uc * 64 * 64 / 2e4) < 1e-15
    assert P.width == 4.0 and abs(P.rho_g - 0.05) < 1e-16 and abs(P.eta_g - P.eta_l / 20) < 1e-16


# Each alternative of the problem statement against its definition, the
# group computed back from the lattice parameters (Sec. 4 set-ups).
ALTERNATIVES = {
    # Ma instead of N_t: U_c = Ma c_s, c_s^2 = 1/3
    "Ma": (dict(Ma=0.05, N_t=None), lambda P, U: abs(P.sigma / P.eta_l - 0.05 / 3 ** 0.5) < 1e-16),
    # Oh on the radius with the capillary velocity (coalescence)
    "Oh": (dict(visc="Oh", Oh=0.119), lambda P, U: abs(P.eta_l / (P.sigma * 64) ** 0.5 - 0.119) < 1e-13),
    # Oh and Eo on the diameter, gravity from Eo (falling drop)
    "Oh_Eo_gravity": (dict(visc="Oh", Oh=0.0466, gravity="Eo", Eo=144.0, L_g=2.0, G=(1.0, 0.0, 0.0), r_rho=1.15),
                      lambda P, U: abs(P.g[0] * (1 - P.rho_g) * 128 ** 2 / P.sigma - 144) < 1e-9
                      and abs(P.eta_l / (P.sigma * 128) ** 0.5 - 0.0466) < 1e-13 and P.g[1] == 0.0),
    # We instead of the capillary velocity
    "We": (dict(st="We", We=12.5), lambda P, U: abs(U * U * 64 / P.sigma - 12.5) < 1e-12),
    # sigma in lattice units and eta_L from U_c = sigma / eta_L (static drop)
    "sigma": (dict(st="sigma", sigma=1e-3, visc="capillary", Ma=0.05, N_t=None),
              lambda P, U: P.sigma == 1e-3 and abs(P.eta_l - 1e-3 / (0.05 / 3 ** 0.5)) < 1e-16),
    # Fr: |g| = U_c^2 / (Fr^2 L_c) along the given direction
    "Fr": (dict(gravity="Fr", Fr=0.5, G=(0.0, -2.0, 0.0)), lambda P, U: abs(P.g[1] + U * U / (0.25 * 64)) < 1e-18),
    # Eo and Mo with gravity from Fr (rising bubble)
    "Eo_Mo": (dict(gravity="Fr", Fr=1.0, G=(0.0, -1.0, 0.0), st="Eo", Eo=10.0, visc="Mo", Mo=1e-4, r_rho=10.0),
              lambda P, U: abs(-P.g[1] * 0.9 * 64 ** 2 / P.sigma - 10) < 1e-12
              and abs(-P.g[1] * 0.9 * P.eta_l ** 4 / P.sigma ** 3 - 1e-4) < 1e-16),
    # Mo with the capillary velocity: eta_L = Mo rho_L^2 U_c^3 / (g drho)
    "Mo_capillary": (dict(gravity="Fr", Fr=1.0, G=(0.0, -1.0, 0.0), visc="Mo", Mo=1e-4, r_rho=10.0),
                     lambda P, U: abs(-P.g[1] * 0.9 * P.eta_l ** 4 / P.sigma ** 3 - 1e-4) < 1e-16
                     and abs(P.sigma / P.eta_l - U) < 1e-16),
    # an arbitrary reference density
    "rho_ref": (dict(rho_ref=0.37), lambda P, U: P.rho_ref == 0.37),
    "rho_ref_gas": (dict(rho_ref="gas"), lambda P, U: P.rho_ref == P.rho_g),
}


@pytest.mark.parametrize("name", list(ALTERNATIVES))
def test_params_from_dimensionless_alternatives(G, name):
    from oracle.problem import lattice_problem

    kw, check = ALTERNATIVES[name]
    st = _base(**{k: v for k, v in kw.items() if v is not None})
    for k, v in kw.items():
        if v is None:
            st.pop(k)
    P = G.gpe_params_from_dimensionless(G.problem_struct(st))
    U = 64 / 384 if "N_t" in st else 0.05 / 3 ** 0.5
    assert check(P, U), name
    # the oracle's own mapping gives the same values
    ref = lattice_problem(st)
    got = G.lattice_problem(st)
    for k in ("dt", "cs2", "rho_l", "rho_g", "eta_l", "eta_g", "sigma", "mob", "width", "rho_ref"):
        assert abs(got[k] - ref[k]) <= 1e-15 * abs(ref[k]), (name, k, got[k], ref[k])
    for a in range(3):
        assert abs(got["g"][a] - ref["g"][a]) <= 1e-15 * abs(ref["g"][a]), (name, a)


@pytest.mark.parametrize("kw", [
    dict(visc="capillary"),                             # sigma and eta_L each defined by the other
    dict(gravity="Eo", Eo=10.0, st="Eo", G=(1.0, 0.0, 0.0)),  # Eo used for both sigma and g
    dict(st="Eo", Eo=10.0),                             # Eo without gravity
    dict(visc="Mo", Mo=1e-4),                           # Mo without gravity
    dict(gravity="Fr", Fr=1.0, G=(0.0, -1.0, 0.0), visc="Mo", Mo=1e-4, r_rho=1.0),  # Mo with rho_L = rho_G
    dict(gravity="Fr", Fr=0.0, G=(0.0, -1.0, 0.0)),    # Fr must be positive
    dict(Re=0.0),
    dict(Cn=0.0),
    dict(N_L=0.0),
])
def test_params_from_dimensionless_rejects_undetermined(G, kw):
    st = _base(**kw)
    with pytest.raises(G.GpeError) as e:
        G.gpe_params_from_dimensionless(G.problem_struct(st))
    assert e.value.code == G.GPE_EINVAL


STATEMENT_WORKLOADS = {
    "capillary_wave": lambda: W.capillary_wave()[0],
    "capillary_wave_fine": lambda: W.capillary_wave(NL=128, Nt=1920, Cn=0.03125, Pe=4e4)[0],
    "falling_drop": lambda: W.falling_drop_axisym()[0],
    "coalescence_axisym_oh0.037": lambda: W.coalescence_axisym(Oh=0.037)[0],
    "coalescence_axisym_oh0.3": lambda: W.coalescence_axisym(Oh=0.3)[0],
    "coalescence_3d": lambda: W.coalescence_3d(),
    "coalescence_3d_replay": lambda: W.coalescence_3d_replay(NL=12, Oh=0.3, scheme=1)[0],
    "rt_re256": lambda: W.rt_paper(Re=256.0)[0],
    "rt_re3000": lambda: W.rt_paper(Re=3000.0)[0],
    "rising_bubble": lambda: W.rising_bubble_3d()[0],
    "rising_bubble_small": lambda: W.rising_bubble_3d(nx=40, ny=19, nz=45, R=7.0, zc=17.0, Fr=0.5)[0],
}


@pytest.mark.parametrize("name", list(STATEMENT_WORKLOADS))
def test_solver_mapping_equals_oracle_mapping(G, name):
    """Every workload stated in dimensionless groups reaches the solver
    through gpe_params_from_dimensionless (gpe.lattice_problem) and the
    oracle through its own mapping: the lattice parameters agree to
    round-off (measured: bitwise)."""
    from oracle.problem import lattice_problem

    st = STATEMENT_WORKLOADS[name]()
    assert W.is_statement(st)
    got, ref = G.lattice_problem(st), lattice_problem(st)
    for k in ("dt", "cs2", "rho_l", "rho_g", "eta_l", "eta_g", "sigma", "mob", "width", "rho_ref"):
        assert abs(got[k] - ref[k]) <= 1e-15 * abs(ref[k]), (k, got[k], ref[k])
    for a in range(3):
        assert abs(got["g"][a] - ref["g"][a]) <= 1e-15 * abs(ref["g"][a])
    for k in ("dim", "axisym", "n", "bc", "lattice", "precision"):
        assert got[k] == ref[k]
    # and the solver's parameter block is built from the mapped values
    P = G.params_from_problem(got)
    assert P.eta_l == got["eta_l"] and P.sigma == got["sigma"] and P.mobility == got["mob"]


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
    # FP32 x rows padded to a multiple of 64 elements from 64 cells on:
    # 130 -> 192, 70 -> 128; narrower grids (40) and FP64 keep dense rows
    prob4, _ = W.rising_bubble_3d(nx=130, ny=19, nz=45, R=7.0, zc=17.0, precision="fp32")
    P4 = G.params_from_problem(prob4)
    assert G.gpe_workspace_bytes(P4) == 19 * align(192 * 19 * 45 * 4) + align((512 * 8 + 8) * 8)
    prob6, _ = W.rising_bubble_3d(nx=40, ny=19, nz=45, R=7.0, zc=17.0, precision="fp32")
    P6 = G.params_from_problem(prob6)
    assert G.gpe_workspace_bytes(P6) == 19 * align(40 * 19 * 45 * 4) + align((512 * 8 + 8) * 8)
    prob5, _ = W.static_drop_2d(n=70, precision="fp32")
    P5 = G.params_from_problem(prob5)
    assert G.gpe_workspace_bytes(P5) == 14 * align(128 * 70 * 4) + align((512 * 8 + 8) * 8)
    prob7, _ = W.static_drop_2d(n=70, precision="fp64")
    P7 = G.params_from_problem(prob7)
    assert G.gpe_workspace_bytes(P7) == 14 * align(70 * 70 * 8) + align((512 * 8 + 8) * 8)


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
    lambda P: setattr(P, "zchunk", -1),         # 0 = automatic, else planes per work-group
])
def test_invalid_params_rejected(G, mutate):
    prob, _ = W.static_drop_2d()
    P = G.params_from_problem(prob)
    assert G.gpe_workspace_bytes(P) > 0
    mutate(P)
    assert G.gpe_workspace_bytes(P) == 0


@pytest.mark.parametrize("scheme,ok", [(0, True), (1, True), (2, True), (3, True), (4, False), (-1, False)])
def test_scheme_flags_3d(G, scheme, ok):
    prob = G.lattice_problem(W.rising_bubble_3d(nx=8, ny=8, nz=8)[0])
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


def test_hbm_stream_probe_rejects_invalid_arguments(G):
    """gpe_hbm_stream validates its arguments before it launches anything
    (the pointers here are never dereferenced)."""
    L = G.lib()
    A, B = ctypes.c_void_p(0x10000), ctypes.c_void_p(0x20000)
    bad = [
        (G.GPE_STREAM_COPY, A, B, 0, 1),                       # no bytes
        (G.GPE_STREAM_COPY, A, B, 24, 1),                      # not a multiple of 16
        (G.GPE_STREAM_COPY, ctypes.c_void_p(None), B, 64, 1),  # no destination
        (G.GPE_STREAM_READ, A, ctypes.c_void_p(None), 64, 1),  # no source to read
        (G.GPE_STREAM_COPY, ctypes.c_void_p(0x10008), B, 64, 1),  # misaligned destination
        (G.GPE_STREAM_COPY, A, ctypes.c_void_p(0x20004), 64, 1),  # misaligned source
        (G.GPE_STREAM_COPY, A, B, 64, -1),                     # negative work-group count
        (7, A, B, 64, 1),                                      # unknown mode
    ]
    for mode, dst, src, nbytes, wg in bad:
        assert L.gpe_hbm_stream(mode, dst, src, nbytes, wg, None) == G.GPE_EINVAL, (mode, nbytes, wg)
