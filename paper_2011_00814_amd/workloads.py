"""Seeded synthetic workloads: problem dictionaries and initial states.

This module holds no arithmetic of the method itself.  It only writes down
parameter values (lattice units, dx = 1) and builds initial fields (tanh
interface profiles, seeded perturbations), shaped like the paper's test
problems (Sec. 4: static drop / capillary wave, Rayleigh-Taylor instability,
rising bubble / drop in 3-D).  Both the GPU path and the CPU oracle consume
what it produces; it imports neither.

A problem dictionary has the keys::

    dim, axisym, n=(nx, ny, nz), bc=(x-lo, x-hi, y-lo, y-hi, z-lo, z-hi),
    lattice, dt, cs2, rho_l, rho_g, eta_l, eta_g, sigma, mob, width,
    g=(gx, gy, gz), rho_ref, precision ("fp64" | "fp32")

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


def rayleigh_taylor_2d(nx=256, ny=1024, precision="fp64", amp_frac=0.1, W=2.0):
    """2-D Rayleigh-Taylor: x periodic, no-slip walls at y = 0 and y = ny;
    Atwood 0.5 (rho_G = 1/3), viscosity ratio 1, Re = 3000 on lambda = nx with
    U_c = sqrt(g lambda) = 0.05, sigma = 0, Pe = 8e4 (M = U_c lambda^2 / Pe),
    rho_ref = rho_G; heavy fluid (phi = +1) on top of the cosine-perturbed
    interface y0 = ny/2 + amp_frac*nx*cos(2 pi x / nx)."""
    lam = float(nx)
    Uc = 0.05
    g = Uc * Uc / lam
    eta = Uc * lam / 3000.0
    prob = base_problem(
        dim=2, n=(nx, ny, 1), bc=(PERIODIC, PERIODIC, WALL, WALL, 0, 0),
        rho_l=1.0, rho_g=1.0 / 3.0, eta_l=eta, eta_g=eta, sigma=0.0,
        mob=Uc * lam * lam / 8e4, width=W, g=(0.0, -g, 0.0), rho_ref=1.0 / 3.0,
        precision=precision)
    x, y, _ = _centres(prob)
    y0 = ny / 2 + amp_frac * nx * np.cos(2 * math.pi * x / nx)
    st = zero_state(prob)
    st["phi"] = np.tanh(2.0 * (y - y0) / W)
    return prob, st


def rising_bubble_3d(nx=128, ny=128, nz=256, R=16.0, zc=48.0, precision="fp32", W=2.0,
                     mob=0.02):
    """3-D rising bubble, no-slip walls on all faces: density and viscosity
    ratio 10, D = 2R = 32, U_c = sqrt(g D) = 0.03, Eotvos 10, Morton 1e-4,
    W = 2, M = 0.02, rho_ref = rho_L, D3Q15; gas bubble of radius R at
    (nx/2, ny/2, zc)."""
    D = 2.0 * R
    Uc = 0.03
    g = Uc * Uc / D
    drho = 0.9
    sigma = g * drho * D * D / 10.0
    eta_l = (1e-4 * sigma ** 3 / (g * drho)) ** 0.25
    prob = base_problem(
        dim=3, n=(nx, ny, nz), bc=(WALL,) * 6, rho_l=1.0, rho_g=0.1,
        eta_l=eta_l, eta_g=eta_l / 10.0, sigma=sigma, mob=mob, width=W,
        g=(0.0, 0.0, -g), rho_ref=1.0, precision=precision)
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
