"""Manufactured steady solution of the convergence study (oracle; test infrastructure).

Sec. 3.1, eq. analytical_solution: phi = kappa (x + y),
U = [s, s, s, s^2] with s = sin(phi) + C2 (so rho = s, v = (1, 1), eps = s^2).

The source printed under it does not satisfy the PDE: re-deriving
S = div(F_c - F_v)(U) with p = (gamma-1)(eps - rho|v|^2/2) gives momentum
terms with -kappa (gamma-1) cos(phi) where the paper prints -kappa (gamma-1)/2
cos(phi), and an energy term with -2 kappa (gamma-1) cos(phi) where it prints
-kappa (gamma-1) cos(phi).  The source below is the re-derived one; a CPU test
re-derives it symbolically from the primitive form of the fluxes.
"""
import numpy as np


def exact_state(x, y, kappa=25.0, C2=200.0):
    s = np.sin(kappa * (x + y)) + C2
    return np.stack([s, s, s, s * s])


def source(x, y, gamma=1.4, Pr=0.72, mu=0.01, kappa=25.0, C2=200.0):
    """S with dU/dt + div(F_c - F_v) = S holding for exact_state (steady)."""
    phi = kappa * (x + y)
    g1 = gamma - 1.0
    c, sn, s2 = np.cos(phi), np.sin(phi), np.sin(2.0 * phi)
    mom = kappa * g1 * s2 + (2.0 * kappa - kappa * g1 + 2.0 * kappa * C2 * g1) * c
    ene = (2.0 * kappa * gamma * s2 + (4.0 * kappa * gamma * C2 - 2.0 * kappa * g1) * c
           + 2.0 * gamma * mu * kappa ** 2 / Pr * sn)
    return np.stack([2.0 * kappa * c, mom, mom, ene])
