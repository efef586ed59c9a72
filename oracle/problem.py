"""The oracle's own mapping from a problem statement in dimensionless groups
to lattice-unit parameters (arXiv 2011.00814, Sec. 4: the numerical set-up
of each test problem).

TEST INFRASTRUCTURE ONLY: used by the oracle binding (oracle.run and
friends accept either form of a problem dictionary) and by the tests.  It
is written from the paper and shares no code with the GPU library, whose
C-ABI does the same mapping for the solver; a CPU test checks that the two
agree.

Lattice units: the characteristic length L_c is N_L cells and the
characteristic time T_c = L_c / U_c is N_t steps, so dx = dt = 1 and
U_c = N_L / N_t; the sound speed is c_s = dx / (sqrt(3) dt), so c_s^2 = 1/3;
rho_L = 1; the reference surface tension of the chemical potential is 1, so
that a Peclet number Pe = U_c L_c^2 / M gives the mobility.

A statement is a dictionary with the structural keys of a lattice problem
(dim, axisym, n, bc, lattice, precision, optional ch_transport, scheme,
allow_unstable, init, flags, ch_rk) and::

    N_L          cells per L_c
    N_t or Ma    steps per T_c, or the Mach number U_c / c_s
    r_rho, r_eta density and viscosity ratios (liquid over gas)
    visc         "Re" | "Oh" | "Mo" | "capillary"    (and the value under that key)
    st           "none" | "We" | "Eo" | "sigma" | "capillary"
    gravity      "G" (default) | "Fr" | "Eo";  G: vector in U_c^2 / L_c, or a direction
    L_g          length of Oh, Eo and Mo in units of L_c (default 1)
    Pe, Cn       Peclet and Cahn numbers
    rho_ref      "zero" | "liquid" | "gas" | a number (in units of rho_L)
"""
from __future__ import annotations

import math

STRUCTURAL = ("dim", "axisym", "n", "bc", "lattice", "precision", "ch_transport", "scheme",
              "allow_unstable", "init", "flags", "ch_rk", "meta", "zchunk")


def is_statement(prob: dict) -> bool:
    return "N_L" in prob


def lattice_problem(st: dict) -> dict:
    """Lattice-unit problem dictionary of a dimensionless statement (a
    lattice-unit dictionary is returned unchanged)."""
    if not is_statement(st):
        return st
    L = float(st["N_L"])
    # characteristic velocity in cells per step
    if "N_t" in st:
        U = L / float(st["N_t"])
    else:
        U = float(st["Ma"]) / math.sqrt(3.0)
    rho_l = 1.0
    rho_g = rho_l / float(st["r_rho"])
    drho = rho_l - rho_g
    Lg = L * float(st.get("L_g", 1.0))
    G = [float(x) for x in st.get("G", (0.0, 0.0, 0.0))]
    Gnorm = math.sqrt(sum(x * x for x in G))
    unit = [x / Gnorm for x in G] if Gnorm > 0 else [0.0, 0.0, 0.0]

    gravity = st.get("gravity", "G")
    g = None                       # magnitude of the body force, once known
    if gravity == "G":
        g = Gnorm * U * U / L      # G measured in U_c^2 / L_c
    elif gravity == "Fr":
        g = U * U / (float(st["Fr"]) ** 2 * L)   # Fr = U_c / sqrt(g L_c)

    kind = st.get("st", "none")
    sigma = None
    if kind == "none":
        sigma = 0.0
    elif kind == "We":             # We = rho_L U_c^2 L_c / sigma
        sigma = rho_l * U * U * L / float(st["We"])
    elif kind == "sigma":
        sigma = float(st["sigma"])
    elif kind == "Eo":             # Eo = g (rho_L - rho_G) L_g^2 / sigma
        sigma = g * drho * Lg * Lg / float(st["Eo"])

    visc = st["visc"]
    if visc == "Re":               # Re = rho_L U_c L_c / eta_L
        eta = rho_l * U * L / float(st["Re"])
    elif visc == "Oh":             # Oh = eta_L / sqrt(rho_L sigma L_g)
        Oh = float(st["Oh"])
        if kind == "capillary":    # sigma = U_c eta_L: Oh^2 = eta_L / (rho_L U_c L_g)
            eta = Oh * Oh * rho_l * U * Lg
        else:
            eta = Oh * math.sqrt(rho_l * sigma * Lg)
    elif visc == "Mo":             # Mo = g (rho_L - rho_G) eta_L^4 / (rho_L^2 sigma^3)
        Mo = float(st["Mo"])
        if kind == "capillary":    # with sigma = U_c eta_L, Mo = g drho eta_L / (rho_L^2 U_c^3)
            eta = Mo * rho_l ** 2 * U ** 3 / (g * drho)
        else:
            eta = (Mo * rho_l ** 2 * sigma ** 3 / (g * drho)) ** 0.25
    elif visc == "capillary":      # U_c = sigma / eta_L
        eta = sigma / U
    else:
        raise ValueError(f"unknown viscosity group {visc!r}")
    if kind == "capillary":
        sigma = U * eta
    if gravity == "Eo":            # the body force from Eo once sigma is known
        g = float(st["Eo"]) * sigma / (drho * Lg * Lg)

    ref = st.get("rho_ref", "zero")
    rho_ref = {"zero": 0.0, "liquid": rho_l, "gas": rho_g}[ref] if isinstance(ref, str) else float(ref) * rho_l

    out = {k: st[k] for k in STRUCTURAL if k in st}
    out.setdefault("axisym", 0)
    out.setdefault("precision", "fp64")
    out.update(dt=1.0, cs2=1.0 / 3.0, rho_l=rho_l, rho_g=rho_g, eta_l=eta, eta_g=eta / float(st["r_eta"]),
               sigma=sigma, mob=(U * L * L / float(st["Pe"])) if float(st.get("Pe", 0.0)) > 0 else 0.0,
               width=float(st["Cn"]) * L, g=tuple(g * x for x in unit), rho_ref=rho_ref)
    return out
