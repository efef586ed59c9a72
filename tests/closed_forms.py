"""Closed-form solutions the oracle and the GPU replays are checked against."""
import math

import numpy as np


def prosperetti(t, sigma, k, rho_l, rho_g, nu):
    """Scaled interface displacement (h_eq - h_0(t)) / A_p of a small capillary
    wave between two fluids of equal kinematic viscosity nu (Sec. 4.1, the
    closed-form solution, after Prosperetti): erfc terms over the four roots
    z_i of the quartic in z, evaluated through the Faddeeva function."""
    from scipy.special import erfc, wofz
    w0 = math.sqrt(sigma * k ** 3 / (rho_l + rho_g))
    eps = nu * k * k / w0
    beta = rho_l * rho_g / (rho_l + rho_g) ** 2
    z = np.roots([1, -4 * beta * math.sqrt(eps * w0), 2 * (1 - 6 * beta) * eps * w0,
                  4 * (1 - 3 * beta) * (eps * w0) ** 1.5, (1 - 4 * beta) * (eps * w0) ** 2 + w0 * w0])
    tp = w0 * t
    val = 4 * (1 - 4 * beta) * eps ** 2 / (8 * (1 - 4 * beta) * eps ** 2 + 1) * erfc(math.sqrt(eps * tp))
    for i in range(4):
        Zi = np.prod([z[j] - z[i] for j in range(4) if j != i])
        # exp((z^2 - eps w0) t) erfc(z sqrt t) = exp(-eps w0 t) w(i z sqrt t)
        val += (z[i] * w0 * w0 / (Zi * (z[i] ** 2 - eps * w0)) * math.exp(-eps * tp)
                * wofz(1j * z[i] * math.sqrt(t))).real
    return val
