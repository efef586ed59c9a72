"""Seeded synthetic workloads: problem dictionaries and initial states.

This module holds no arithmetic of the method itself.  It only writes down
parameter values (lattice units, dx = 1) and builds initial fields (tanh
interface profiles, seeded perturbations), shaped like the paper's test
problems (Sec. 4: static drop / capillary wave, Rayleigh-Taylor instability,
rising bubble / drop in 3-D).  Both the GPU path and the CPU oracle consume
what it produces; it imports neither.

A problem dictionary comes in one of two forms:

- lattice units (the benchmark configurations that are specified that way,
  the ensemble and the synthetic test cases)::

    dim, axisym, n=(nx, ny, nz), bc=(x-lo, x-hi, y-lo, y-hi, z-lo, z-hi),
    lattice, dt, cs2, rho_l, rho_g, eta_l, eta_g, sigma, mob, width,
    g=(gx, gy, gz), rho_ref, precision ("fp64" | "fp32")

- a problem statement in the paper's dimensionless groups (its Sec. 4
  set-ups and the rising bubble of the 3-D configuration): the structural
  keys (dim, axisym, n, bc, lattice, precision, ...) and N_L, N_t or Ma,
  r_rho, r_eta, the viscosity group (visc = "Re" | "Oh" | "Mo" | "capillary"),
  the surface-tension group (st = "none" | "We" | "Eo" | "sigma" |
  "capillary"), gravity ("G" | "Fr" | "Eo", with G a vector or direction),
  L_g, Pe, Cn, rho_ref ("zero" | "liquid" | "gas" | value).  This module
  never converts a statement to lattice units: the solver maps it with the
  library's gpe_params_from_dimensionless, the CPU reference with its own
  mapping.  Initial fields are built from the statement (interface width
  W = Cn N_L).

Boundary codes: 0 periodic, 1 no-slip wall, 2 symmetry plane / axis.
Arrays are float64 numpy arrays of shape (nz, ny, nx) (nz = 1 in 2-D).
"""
from __future__ import annotations

import math

import numpy as np

PERIODIC, WALL, SYMMETRY = 0, 1, 2


def _centres(prob):
    nx, ny, nz = prob["n"]
    z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5,
                          indexing="ij")
    return x, y, z


def zero_state(prob) -> dict:
    nx, ny, nz = prob["n"]
    sh = (nz, ny, nx)
    st = {k: np.zeros(sh) for k in ("p", "u", "v", "phi")}
    st["w"] = np.zeros(sh) if prob["dim"] == 3 else None
    return st


def base_problem(dim=2, n=(64, 64, 1), bc=(0, 0, 0, 0, 0, 0), **kw) -> dict:
    prob = dict(
        dim=dim, axisym=0, n=tuple(int(v) for v in n), bc=tuple(bc),
        lattice=9 if dim == 2 else 15, dt=1.0, cs2=1.0 / 3.0,
        rho_l=1.0, rho_g=1.0, eta_l=0.05, eta_g=0.05, sigma=0.0, mob=0.0,
        width=2.0, g=(0.0, 0.0, 0.0), rho_ref=0.0, precision="fp64",
    )
    prob.update(kw)
    return prob


def statement(dim=2, n=(64, 64, 1), bc=(0, 0, 0, 0, 0, 0), **kw) -> dict:
    """A problem statement in dimensionless groups (see the module docstring)."""
    prob = dict(dim=dim, axisym=0, n=tuple(int(v) for v in n), bc=tuple(bc),
                lattice=9 if dim == 2 else 15, precision="fp64")
    prob.update(kw)
    return prob


def is_statement(prob: dict) -> bool:
    return "N_L" in prob


def reporting_units(sc: dict, lat: dict) -> dict:
    """Complete the units a replay reports in from the lattice-unit
    parameters `lat` of its problem: kind "gravity" gives U = sqrt(|g| D),
    T = sqrt(D / |g|) (D = sc["D"]); kind "capillary" gives the
    capillary-inertial U = sqrt(sigma / (rho_L L)), T = L / U; other
    scales are returned as they are."""
    out = dict(sc)
    kind = out.pop("kind", None)
    if kind == "gravity":
        g = math.sqrt(sum(x * x for x in lat["g"]))
        out["U"], out["T"] = math.sqrt(g * out["D"]), math.sqrt(out["D"] / g)
    elif kind == "capillary":
        out["U"] = math.sqrt(lat["sigma"] / (lat["rho_l"] * out["L"]))
        out["T"] = out["L"] / out["U"]
    return out


# --------------------------------------------------------------------------
# The benchmark configurations (lattice units, dt = dx = 1, cs^2 = 1/3)
# --------------------------------------------------------------------------
def static_drop_2d(n=64, R=16.0, W=2.0, precision="fp64"):
    """2-D static drop, periodic n x n: density ratio 10, viscosity ratio 10,
    sigma = 1e-3, M = 0.05, W = 2, Ma = U_c / c_s = 0.05 with U_c = sigma/eta_L
    (so eta_L = sigma / (0.05 c_s)); drop of radius R centred; profile
    tanh((R - r) / (sqrt(2) W)) taken literally from the configuration."""
    cs = math.sqrt(1.0 / 3.0)
    sigma = 1e-3
    eta_l = sigma / (0.05 * cs)
    prob = base_problem(
        dim=2, n=(n, n, 1), bc=(PERIODIC,) * 6, rho_l=1.0, rho_g=0.1,
        eta_l=eta_l, eta_g=eta_l / 10.0, sigma=sigma, mob=0.05, width=W,
        precision=precision)
    x, y, _ = _centres(prob)
    r = np.sqrt((x - n / 2) ** 2 + (y - n / 2) ** 2)
    st = zero_state(prob)
    st["phi"] = np.tanh((R - r) / (math.sqrt(2.0) * W))
    return prob, st


def rayleigh_taylor_2d(nx=256, ny=1024, precision="fp64", amp_frac=0.1, W=2.0, in_kernel_init=False):
    """2-D Rayleigh-Taylor: x periodic, no-slip walls at y = 0 and y = ny;
    Atwood 0.5 (rho_G = 1/3), viscosity ratio 1, Re = 3000 on lambda = nx with
    U_c = sqrt(g lambda) = 0.05, sigma = 0, Pe = 8e4 (M = U_c lambda^2 / Pe),
    rho_ref = rho_G; heavy fluid (phi = +1) on top of the cosine-perturbed
    interface y0 = ny/2 + amp_frac*nx*cos(2 pi x / nx) (the in-kernel layer
    profile, init kind 3, with in_kernel_init; then no state is built)."""
    lam = float(nx)
    Uc = 0.05
    g = Uc * Uc / lam
    eta = Uc * lam / 3000.0
    prob = base_problem(
        dim=2, n=(nx, ny, 1), bc=(PERIODIC, PERIODIC, WALL, WALL, 0, 0),
        rho_l=1.0, rho_g=1.0 / 3.0, eta_l=eta, eta_g=eta, sigma=0.0,
        mob=Uc * lam * lam / 8e4, width=W, g=(0.0, -g, 0.0), rho_ref=1.0 / 3.0,
        precision=precision)
    if in_kernel_init:
        prob["init"] = {"kind": 3, "center": (0.0, ny / 2, 0.0), "amp": amp_frac * nx, "width": W}
        return prob, None
    x, y, _ = _centres(prob)
    y0 = ny / 2 + amp_frac * nx * np.cos(2 * math.pi * x / nx)
    st = zero_state(prob)
    st["phi"] = np.tanh(2.0 * (y - y0) / W)
    return prob, st


def rising_bubble_3d(nx=128, ny=128, nz=256, R=16.0, zc=48.0, precision="fp32", W=2.0,
                     mob=0.02, Fr=1.0, in_kernel_init=False):
    """3-D rising bubble, no-slip walls on all faces, as a statement: L_c =
    D = 2R = 32 cells, U_c = 0.03 (N_t = D / U_c) with U_c = sqrt(g D)
    (Fr = 1); density and viscosity ratio 10, Eotvos 10, Morton 1e-4 on D,
    Cn = W / D, Pe = U_c D^2 / mob, rho_ref = rho_L, D3Q15; gas bubble of
    radius R at (nx/2, ny/2, zc), phi = tanh(2 (r - R) / W) (the in-kernel
    profile of init kind 2 with in_kernel_init, then no state is built)."""
    D = 2.0 * R
    Uc = 0.03
    prob = statement(
        dim=3, n=(nx, ny, nz), bc=(WALL,) * 6, precision=precision,
        N_L=D, N_t=D / Uc, r_rho=10.0, r_eta=10.0, visc="Mo", Mo=1e-4, st="Eo", Eo=10.0,
        gravity="Fr", Fr=Fr, G=(0.0, 0.0, -1.0), Pe=Uc * D * D / mob, Cn=W / D, rho_ref="liquid")
    if in_kernel_init:
        prob["init"] = {"kind": 2, "center": (nx / 2, ny / 2, zc), "radius": R, "width": W}
        return prob, None
    x, y, z = _centres(prob)
    r = np.sqrt((x - nx / 2) ** 2 + (y - ny / 2) ** 2 + (z - zc) ** 2)
    st = zero_state(prob)
    st["phi"] = np.tanh(2.0 * (r - R) / W)
    return prob, st


def axisym_drop(nz=96, nr=32, R=10.0, zc=40.0, precision="fp64"):
    """Axisymmetric drop (x = axial, y = radial, axis at y = 0): density ratio
    1.15 falling-drop-like physics with gravity along the axis."""
    prob = base_problem(
        dim=2, n=(nz, nr, 1), bc=(WALL, WALL, SYMMETRY, WALL, 0, 0),
        rho_l=1.0, rho_g=1.0 / 1.15, eta_l=0.02, eta_g=0.02, sigma=2e-3,
        mob=0.03, width=3.0, g=(-1e-5, 0.0, 0.0), rho_ref=1.0 / 1.15,
        precision=precision)
    prob["axisym"] = 1
    x, y, _ = _centres(prob)
    r = np.sqrt((x - zc) ** 2 + y ** 2)
    st = zero_state(prob)
    st["phi"] = -np.tanh(2.0 * (r - R) / prob["width"])
    return prob, st


# --------------------------------------------------------------------------
# Seeded perturbations for parity tests
# --------------------------------------------------------------------------
def smooth_noise(shape, seed, amp, modes=4):
    """Sum of a few random low Fourier modes (periodic in every axis), seeded."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    out = np.zeros(shape)
    for _ in range(modes):
        kx = rng.integers(1, 4) * 2 * math.pi / nx
        ky = rng.integers(0, 4) * 2 * math.pi / ny
        kz = (rng.integers(0, 4) * 2 * math.pi / nz) if nz > 1 else 0.0
        ph = rng.uniform(0, 2 * math.pi)
        out += rng.uniform(-1, 1) * np.cos(kx * x + ky * y + kz * z + ph)
    return amp * out / modes


def perturbed(prob, st, seed=0, uamp=1e-3, pamp=1e-4):
    """Add seeded smooth velocity and pressure perturbations to a state; the
    boundary-normal faces of non-periodic axes are set to 0."""
    out = {k: (None if v is None else v.copy()) for k, v in st.items()}
    sh = out["phi"].shape
    out["p"] = out["p"] + smooth_noise(sh, seed * 7 + 1, pamp)
    comps = ["u", "v"] + (["w"] if prob["dim"] == 3 else [])
    for a, key in enumerate(comps):
        f = out[key] + smooth_noise(sh, seed * 7 + 2 + a, uamp)
        if prob["bc"][2 * a] != PERIODIC:
            idx = [slice(None)] * 3
            idx[2 - a] = 0
            f[tuple(idx)] = 0.0
        out[key] = f
    return out


# --------------------------------------------------------------------------
# Ensemble of independent 2-D drops (input of the batched engine)
# --------------------------------------------------------------------------
ENSEMBLE_SIZES = (64, 96, 128, 192, 256)
ENSEMBLE_ASPECT = 0.2  # semi-axes R (1 + 0.2) along x and R (1 - 0.2) along y


def ellipse_phi(prob, R, amp, center=None, W=None):
    """Elliptic drop: phi = tanh(2 R (1 - rho) / W) with
    rho = |((x - x0) / a, (y - y0) / b)|, a = R (1 + amp), b = R (1 - amp)."""
    nx, ny, _ = prob["n"]
    W = prob["width"] if W is None else W
    x0, y0 = (nx / 2.0, ny / 2.0) if center is None else center[:2]
    x, y, _ = _centres(prob)
    rho = np.sqrt(((x - x0) / (R * (1.0 + amp))) ** 2 + ((y - y0) / (R * (1.0 - amp))) ** 2)
    return np.tanh(2.0 * R * (1.0 - rho) / W)


def recipe_dt(rho_l, rho_g, eta_l, eta_g, mob, W, dim=2):
    """Time step of the ensemble recipe: 0.8 times the largest step the
    linear stability estimates allow, capped at 1, with c_s^2 = 1/(3 dt^2).

    With that sound speed the acoustic bound 2 c_s dt / sqrt(3) <= 1 holds at
    every dt (it equals 2/3), so only two bounds remain:
      viscous (compressive mode, eigenvalue 3 nu |k|^2 <= 12 nu in 2-D, the
      TVD-RK3 real-axis limit 2.5127):  dt <= 2.5127 / (3 nu_max 4 dim);
      Cahn-Hilliard (linearised about phi = +-1, M lam (8a + kappa lam),
      TVD-RK2 real-axis limit 2), lam = 16/3 the largest eigenvalue of
      minus the D2Q9 isotropic Laplacian (at wavenumber (pi, pi): the four
      axis links give 6 * 4 * (1/9) * 2, the diagonals 0), a = 3/(4W),
      kappa = 3W/8:  dt <= 2 / (M lam (8a + kappa lam))."""
    nu_max = max(eta_l / rho_l, eta_g / rho_g)
    dt_visc = 2.5127 / (3.0 * nu_max * 4.0 * dim) if nu_max > 0 else math.inf
    lam = 16.0 / 3.0
    a, kappa = 3.0 / (4.0 * W), 3.0 * W / 8.0
    ch = mob * lam * (8.0 * a + kappa * lam)
    dt_ch = 2.0 / ch if ch > 0 else math.inf
    return min(1.0, 0.8 * min(dt_visc, dt_ch))


def ensemble_cases(count=512, seed=0, precision="fp32", sizes=ENSEMBLE_SIZES):
    """`count` independent periodic 2-D elliptic drops (numpy PCG64 seed):
    N uniform over `sizes`; R ~ U(10, 30) redrawn until 1.2 R + 2 W <= 0.45 N;
    density ratio exp U(0, ln 100); viscosity ratio exp U(0, ln 50);
    Laplace number La ~ U(1, 20) (U_c = sigma / eta_L, so Re = We = La on R);
    Mach 0.05 at dt = 1 (U_c = 0.05 / sqrt(3)), sigma = U_c^2 R / La,
    eta_L = sigma / U_c; M = 0.05, W = 2; dt from recipe_dt, c_s^2 = 1/(3 dt^2).
    Returns a list of problem dictionaries whose "init" entry asks for the
    in-kernel elliptic drop (kind 4, the same profile as ellipse_phi)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W, M = 2.0, 0.05
    Uc = 0.05 / math.sqrt(3.0)
    out = []
    for _ in range(count):
        N = int(sizes[int(rng.integers(len(sizes)))])
        while True:
            R = float(rng.uniform(10.0, 30.0))
            if 1.2 * R + 2.0 * W <= 0.45 * N:
                break
        r_rho = math.exp(rng.uniform(0.0, math.log(100.0)))
        r_eta = math.exp(rng.uniform(0.0, math.log(50.0)))
        La = float(rng.uniform(1.0, 20.0))
        sigma = Uc * Uc * R / La
        eta_l = sigma / Uc
        rho_g, eta_g = 1.0 / r_rho, eta_l / r_eta
        dt = recipe_dt(1.0, rho_g, eta_l, eta_g, M, W)
        prob = base_problem(
            dim=2, n=(N, N, 1), bc=(PERIODIC,) * 6, rho_l=1.0, rho_g=rho_g, eta_l=eta_l,
            eta_g=eta_g, sigma=sigma, mob=M, width=W, dt=dt, cs2=1.0 / (3.0 * dt * dt),
            precision=precision)
        prob["init"] = {"kind": 4, "center": (N / 2.0, N / 2.0, 0.0), "radius": R,
                        "amp": ENSEMBLE_ASPECT, "width": W}
        prob["meta"] = {"R": R, "r_rho": r_rho, "r_eta": r_eta, "La": La}
        out.append(prob)
    return out


def ensemble_state(prob) -> dict:
    """Initial state of an ensemble case as arrays (for the oracle)."""
    st = zero_state(prob)
    ini = prob["init"]
    st["phi"] = ellipse_phi(prob, ini["radius"], ini["amp"], ini["center"], ini["width"])
    return st


# --------------------------------------------------------------------------
# Multi-mode Rayleigh-Taylor pairs (fine grid and the grid coarser by f) for
# the learned coarse correction
# --------------------------------------------------------------------------
def rt_multimode(seed, nx=256, ny=1024, factor=1, precision="fp32", modes=6, amp_frac=0.05,
                 Re=3000.0, Pe=8e4, W=2.0, Uc=0.05, At=None):
    """The Rayleigh-Taylor set-up of `rayleigh_taylor_2d` with a seeded
    Atwood number At ~ U(0.2, 0.8) (unless given) and a multi-mode
    interface y0(x) = ny/2 + sum_k A_k cos(2 pi k x / nx + theta_k),
    k = 1..modes, theta_k ~ U(0, 2 pi), A_k = amp_frac nx w_k with
    w_k ~ U(0, 1) normalised to sum 1 (fine-grid cells).

    factor > 1 returns the same physics on the (nx/f) x (ny/f) grid in its own
    lattice units (dx = dt = 1 there, so the lattice velocity U_c is kept and
    c_s^2 = 1/3): lambda = nx/f, g = U_c^2/lambda, eta = U_c lambda / Re,
    M = U_c lambda^2 / Pe, interface width W coarse cells.  The returned state
    is the fine initial state (the coarse run starts from its restriction)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    At = float(rng.uniform(0.2, 0.8)) if At is None else float(At)
    theta = rng.uniform(0.0, 2.0 * math.pi, size=modes)
    wts = rng.uniform(0.0, 1.0, size=modes)
    wts = wts / wts.sum()
    rho_g = (1.0 - At) / (1.0 + At)
    nxf, nyf = nx // factor, ny // factor
    lam = float(nxf)
    g = Uc * Uc / lam
    eta = Uc * lam / Re
    prob = base_problem(
        dim=2, n=(nxf, nyf, 1), bc=(PERIODIC, PERIODIC, WALL, WALL, 0, 0),
        rho_l=1.0, rho_g=rho_g, eta_l=eta, eta_g=eta, sigma=0.0,
        mob=Uc * lam * lam / Pe, width=W, g=(0.0, -g, 0.0), rho_ref=rho_g, precision=precision)
    prob["meta"] = {"At": At, "seed": seed, "factor": factor}
    fine = base_problem(dim=2, n=(nx, ny, 1), width=W)
    x, y, _ = _centres(fine)
    y0 = ny / 2.0 + sum(amp_frac * nx * wts[k] * np.cos(2 * math.pi * (k + 1) * x / nx + theta[k])
                        for k in range(modes))
    st = zero_state(fine)
    st["phi"] = np.tanh(2.0 * (y - y0) / W)
    return prob, st


# --------------------------------------------------------------------------
# The paper's 3-D drop coalescence (Sec. 4, 3-D coalescence; its timing case)
# --------------------------------------------------------------------------
def coalescence_3d(n=120, Oh=0.119, lattice=15, precision="fp64", N_t_per_L=10.0):
    """One eighth of two equal drops touching, as a statement: box
    [0, 3 L_c]^3 of n^3 cells (N_L = n / 3 cells per L_c = drop radius),
    symmetry planes on all six faces, drop centre (L_c, 0, 0) so that it
    touches its mirror image at x = 0; r_rho = 50, r_eta = 58.8,
    Oh = eta_L / sqrt(rho_L sigma L_c) with the capillary velocity
    U_c = sigma / eta_L (Re = We = 1 / Oh^2), Cn = 0.1, Pe = 8e3,
    N_t = N_t_per_L * N_L steps per T_c = L_c / U_c (N_t = 400 at N_L = 40),
    no gravity; phi = -tanh(2 (r - R) / W) (in-kernel drop, init kind 1).
    The paper's parameters exceed this library's (conservative) RK4
    stability estimate by a few per cent, hence allow_unstable.  CH
    convection in the advective form as printed (ch_transport = 1): with a
    gas 50 times lighter the conservative form lets phi grow at the grid
    scale in the bulk gas."""
    NL = n / 3.0
    W = 0.1 * NL
    prob = statement(
        dim=3, n=(n, n, n), bc=(SYMMETRY,) * 6, lattice=lattice, precision=precision,
        N_L=NL, N_t=N_t_per_L * NL, r_rho=50.0, r_eta=58.8, visc="Oh", Oh=Oh, st="capillary",
        Pe=8e3, Cn=0.1, allow_unstable=1, ch_transport=1)
    prob["init"] = {"kind": 1, "center": (NL, 0.0, 0.0), "radius": NL, "width": W}
    return prob


def coalescence_state(prob) -> dict:
    """Initial state of `coalescence_3d` as arrays (for the oracle)."""
    ini = prob["init"]
    x, y, z = _centres(prob)
    c = ini["center"]
    r = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
    st = zero_state(prob)
    st["phi"] = -np.tanh(2.0 * (r - ini["radius"]) / ini["width"])
    return st


# --------------------------------------------------------------------------
# The paper's experiments (Sec. 4), in lattice units: L_c = N_L cells,
# T_c = N_t steps (dx = dt = 1, U_c = N_L / N_t, c_s^2 = 1/3), sigma_ref = 1.
# Each returns (prob, state, scales): `scales` holds the length, velocity
# and time units the paper reports its diagnostics in.
# --------------------------------------------------------------------------
def capillary_wave(NL=64, Nt=384, Cn=0.0625, Pe=2e4, Re=1000.0, ratio=20.0, precision="fp64"):
    """Capillary wave in 2-D (Sec. 4.1): unit square with L_c = side length,
    gas on the left, liquid on the right, no-slip walls at x = 0 and 1; the
    lower half 0 <= y <= 1/2 with symmetry planes at y = 0 and 1/2; interface
    h(y) = 1/2 + A_p cos(k (y + 1/2)), A_p = 0.01, k = 2 pi; Re = 1000,
    r_rho = r_eta = 20 (equal kinematic viscosities), U_c = sigma / eta_L.
    The paper's meshes: N_L = 64, N_t = 384, Cn = 1/16, Pe = 2e4 and the
    refined N_L = 128, N_t = 1920, Cn = 1/32, Pe = 4e4.  Returns (statement,
    state, scales) with the wave's A_p and k in lattice units."""
    prob = statement(dim=2, n=(NL, NL // 2, 1), bc=(WALL, WALL, SYMMETRY, SYMMETRY, 0, 0), precision=precision,
                     N_L=NL, N_t=Nt, r_rho=ratio, r_eta=ratio, visc="Re", Re=Re, st="capillary", Pe=Pe, Cn=Cn)
    W = Cn * NL
    x, y, _ = _centres(prob)
    k = 2.0 * math.pi / NL
    Ap = 0.01 * NL
    st = zero_state(prob)
    st["phi"] = np.tanh(2.0 * (x - (0.5 * NL + Ap * np.cos(k * (y + 0.5 * NL)))) / W)
    scales = {"L": float(NL), "U": NL / Nt, "T": float(Nt), "A_p": Ap, "k": k, "h_eq": 0.5 * NL}
    return prob, st, scales


def falling_drop_axisym(NL=50, precision="fp64", ch_transport=0):
    """Falling drop (Sec. 4): axisymmetric [0, 24 R] x [0, 8 R] (z, r) with
    L_c = R; the axis r = 0 is a symmetry line, the other three sides are
    no-slip walls; r_rho = 1.15, r_eta = 1, Eo = g (rho_L - rho_G) D^2 /
    sigma = 144, Oh = eta_L / sqrt(rho_L D sigma) = 0.0466 (both on D = 2R)
    with U_c = sigma / eta_L; N_t = 80 N_L (c = 80), Cn = 0.06, Pe = 1000;
    gravity along +z on the drop only (rho_ref = rho_G); drop centred at
    (2R, 0).  Reported in U_c' = sqrt(g D), T_c' = sqrt(D / g)."""
    prob = statement(
        dim=2, n=(int(24 * NL), int(8 * NL), 1), bc=(WALL, WALL, SYMMETRY, WALL, 0, 0), precision=precision,
        axisym=1, N_L=NL, N_t=80.0 * NL, r_rho=1.15, r_eta=1.0, visc="Oh", Oh=0.0466, st="capillary",
        gravity="Eo", Eo=144.0, L_g=2.0, G=(1.0, 0.0, 0.0), Pe=1000.0, Cn=0.06, rho_ref="gas",
        ch_transport=ch_transport)
    W = 0.06 * NL
    x, y, _ = _centres(prob)
    r = np.sqrt((x - 2.0 * NL) ** 2 + y ** 2)
    st = zero_state(prob)
    st["phi"] = -np.tanh(2.0 * (r - NL) / W)
    scales = {"L": float(NL), "D": 2.0 * NL, "kind": "gravity"}
    return prob, st, scales


def coalescence_axisym(NL=40, Oh=0.119, precision="fp64", N_t=None):
    """Axisymmetric drop coalescence (Sec. 4): [0, 3 R] x [0, 3 R] (z, r),
    symmetry on all sides, drop of radius R = L_c centred at (R, 0) touching
    its mirror image at z = 0; r_rho = 50, r_eta = 58.8, Oh = eta_L /
    sqrt(rho_L sigma R) with U_c = sigma / eta_L, N_t = 10 N_L (50 N_L for
    Oh = 0.3), Cn = 0.1, Pe = 8e3; advective CH transport (light gas).
    Reported in U_ci = sqrt(sigma / (rho_L R)), T_ci = R / U_ci."""
    Nt = float(N_t) if N_t else (50.0 if Oh >= 0.3 else 10.0) * NL
    prob = statement(
        dim=2, n=(int(3 * NL), int(3 * NL), 1), bc=(SYMMETRY,) * 4 + (0, 0), precision=precision, axisym=1,
        N_L=NL, N_t=Nt, r_rho=50.0, r_eta=58.8, visc="Oh", Oh=Oh, st="capillary", Pe=8e3, Cn=0.1,
        ch_transport=1)
    W = 0.1 * NL
    x, y, _ = _centres(prob)
    r = np.sqrt((x - NL) ** 2 + y ** 2)
    st = zero_state(prob)
    st["phi"] = -np.tanh(2.0 * (r - NL) / W)
    return prob, st, {"L": float(NL), "kind": "capillary"}


def coalescence_3d_replay(NL=40, Oh=0.119, lattice=19, precision="fp64", scheme=0):
    """The 3-D coalescence (Sec. 4) as a replay: the set-up of coalescence_3d
    with the host-built initial field and the paper's N_t (10 N_L, 50 N_L for
    Oh = 0.3), reported in U_ci, T_ci like the axisymmetric case.  D3Q19 by
    default: with D3Q15 and N_t = 10 N_L the paper's parameters lie beyond the
    RK4 stability limit of the CH sub-step.  scheme: gpe_scheme ablation
    flags (1: no transverse pressure average, 2: zero bulk viscosity)."""
    c = 50.0 if Oh >= 0.3 else 10.0
    prob = coalescence_3d(n=int(3 * NL), Oh=Oh, lattice=lattice, precision=precision, N_t_per_L=c)
    prob = dict(prob, scheme=scheme)
    st = coalescence_state(prob)
    prob.pop("init")
    return prob, st, {"L": float(NL), "kind": "capillary"}


def rt_paper(NL=256, Re=256.0, precision="fp64", ch_transport=0):
    """Rayleigh-Taylor instability as the paper sets it up (Sec. 4): the lower
    half [0, 4] x [0, 1/2] of the domain in L_c = L_y = lambda, no-slip walls
    at x = 0 and 4, symmetry at y = 0 and 1/2; At = 0.5 (r_rho = 3); Re = 256
    with r_eta = 3 (r_nu = 1) or Re = 3000 with r_eta = 1; U_c = sqrt(lambda
    g) (Fr = 1), N_t = 200 N_L (c = 200), Cn = 1/64, Pe = 8e4, sigma = 0;
    liquid on the left of x = h(y) = 2 + 0.1 cos(2 pi (y + 1/2)), gravity
    along +x on the liquid (rho_ref = rho_G).  Reported in L_c, U_c, T_c."""
    Nt = 200.0 * NL
    prob = statement(
        dim=2, n=(int(4 * NL), int(NL // 2), 1), bc=(WALL, WALL, SYMMETRY, SYMMETRY, 0, 0), precision=precision,
        N_L=NL, N_t=Nt, r_rho=3.0, r_eta=3.0 if Re < 1000 else 1.0, visc="Re", Re=Re, st="none",
        gravity="Fr", Fr=1.0, G=(1.0, 0.0, 0.0), Pe=8e4, Cn=1.0 / 64.0, rho_ref="gas",
        ch_transport=ch_transport)
    W = NL / 64.0
    x, y, _ = _centres(prob)
    h = (2.0 + 0.1 * np.cos(2.0 * math.pi * (y / NL + 0.5))) * NL
    st = zero_state(prob)
    st["phi"] = -np.tanh(2.0 * (x - h) / W)
    return prob, st, {"L": float(NL), "U": NL / Nt, "T": Nt}
