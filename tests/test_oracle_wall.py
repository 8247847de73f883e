"""Pins of the adiabatic wall (Sec. 2.2.4: velocity prescribed, Neumann
conditions on pressure and temperature): no heat crosses a wall face.

A closed annulus (wall faces on both circles) filled with fluid at rest at
uniform pressure but a radial temperature profile: every boundary flux of
energy vanishes (no advection through a fixed wall, no stress work at rest,
no conduction through an adiabatic wall), so the discrete total energy --
like mass -- has zero rate of change up to rounding, while heat still
diffuses inside (the local rates are far from zero).  With the interior's
conductive flux carried through the wall the total would change at the rate
of the wall heat flux; the test plants that and sees it."""
import numpy as np
import pytest

import meshgen as mg
from oracle import physics as ph
from oracle.overint import DGOracleOI
from tests.oracle_helpers import build


def _annulus_at_rest(p, gamma=1.4):
    m = mg.ogrid(16, 4, 0.5, 2.0, 1.2)
    ft = m["face_tag"].copy()
    ft[ft == mg.TAG_FAR] = mg.TAG_WALL
    dg = build(m, p, mu=5e-2, theta=1.0, C_pen=1.0, face_tag=ft)
    r = np.hypot(dg.mesh.x, dg.mesh.y)
    pr = np.full_like(r, 1.0 / gamma)
    T = 1.0 / gamma * (1.0 + 0.2 * np.sin(2.0 * r) + 0.05 * dg.mesh.x)
    rho = pr / T
    zero = np.zeros_like(r)
    U = np.stack([rho, zero, zero, pr / (gamma - 1.0)])
    return dg, U


@pytest.mark.parametrize("p", [2, 3, 4])
def test_closed_adiabatic_annulus_conserves_energy(p):
    dg, U = _annulus_at_rest(p)
    R = dg.rhs(U)
    tot = dg.integral(R)
    scale = np.abs(R[3]).max()
    assert scale > 1e-4                      # heat diffuses inside
    assert abs(tot[0]) < 1e-13 * np.abs(R[0]).max() + 1e-16
    assert abs(tot[3]) < 1e-12 * scale


def test_over_integrated_annulus_conserves_energy():
    dg, U = _annulus_at_rest(3)
    R = DGOracleOI(dg.mesh, dg.phys).rhs(U)
    assert abs(dg.integral(R)[3]) < 1e-12 * np.abs(R[3]).max()


def test_a_conducting_wall_would_not(monkeypatch):
    """The planted mistake: the wall's viscous flux with the conduction of
    the interior gradient (the literal G(U^b) grad U+) changes the total."""
    dg, U = _annulus_at_rest(3)
    real = ph.viscous_flux

    def conducting(U_, Ux, Uy, mu, Pr, gamma):
        return real(U_, Ux, Uy, mu, dg.phys.Pr if np.isinf(Pr) else Pr, gamma)

    monkeypatch.setattr(ph, "viscous_flux", conducting)
    R = dg.rhs(U)
    assert abs(dg.integral(R)[3]) > 1e-6 * np.abs(R[3]).max()
