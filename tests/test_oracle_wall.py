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


def _face_weights(t):
    """Weights of the exact integral over [-1, 1] of the polynomial
    interpolant through the points t (monomial moments)."""
    n = len(t)
    V = np.vander(t, n, increasing=True)
    mom = np.array([(1.0 - (-1.0) ** (j + 1)) / (j + 1) for j in range(n)])
    return np.linalg.solve(V.T, mom)


@pytest.mark.parametrize("p", [2, 3, 4])
def test_printed_wall_flux_carries_the_heat_flux(p):
    """The printed wall flux G(U^b) grad U+ (option): at rest every wall
    term except conduction vanishes, so the total energy changes at the rate
    of the heat let through the wall, the face integral of k grad(e) . n
    with k = mu gamma / Pr.  Uniform pressure and a density polynomial of
    degree 2 <= p make the nodal gradient exact, grad e = -E grad(rho) /
    rho^2; the wall faces, their nodes, normals and quadrature are found
    here from the vertices alone."""
    gamma, mu, Pr = 1.4, 5e-2, 0.72
    m = mg.ogrid(16, 4, 0.5, 2.0, 1.2)
    ft = m["face_tag"].copy()
    ft[ft == mg.TAG_FAR] = mg.TAG_WALL
    dg = build(m, p, mu=mu, Pr=Pr, gamma=gamma, theta=1.0, C_pen=1.0, face_tag=ft,
               wall_heat_flux=True)
    x, y = dg.mesh.x, dg.mesh.y
    a, b = 0.1, 0.05
    rho = 1.0 + a * x + b * y * y
    E = np.full_like(x, 1.0 / (gamma * (gamma - 1.0)))
    zero = np.zeros_like(x)
    U = np.stack([rho, zero, zero, E])
    R = dg.rhs(U)
    got = dg.integral(R)

    k_cond = mu * gamma / Pr
    VX, VY, EToV = m["VX"], m["VY"], m["EToV"]
    want = 0.0
    nface = 0
    for k, f in zip(*np.nonzero(ft == mg.TAG_WALL)):
        v = EToV[k]
        (x0, y0), (x1, y1) = (VX[v[f]], VY[v[f]]), (VX[v[(f + 1) % 3]], VY[v[(f + 1) % 3]])
        x2, y2 = VX[v[(f + 2) % 3]], VY[v[(f + 2) % 3]]
        dx, dy = x1 - x0, y1 - y0
        L = np.hypot(dx, dy)
        n = np.array([dy, -dx]) / L
        if n @ np.array([x2 - x0, y2 - y0]) > 0:
            n = -n
        # the element's nodes on this face: collinear with its vertices
        cross = (x[:, k] - x0) * dy - (y[:, k] - y0) * dx
        on = np.abs(cross) < 1e-12 * L * L
        assert on.sum() == p + 1
        t = 2.0 * ((x[on, k] - x0) * dx + (y[on, k] - y0) * dy) / (L * L) - 1.0
        xn, yn = x[on, k], y[on, k]
        r = 1.0 + a * xn + b * yn * yn
        gx, gy = -E[0, 0] * a / r ** 2, -E[0, 0] * 2.0 * b * yn / r ** 2
        want += 0.5 * L * _face_weights(t) @ (k_cond * (gx * n[0] + gy * n[1]))
        nface += 1
    assert nface == 2 * 16
    assert abs(want) > 1e-3
    assert abs(got[0]) < 1e-13 * np.abs(R[0]).max() + 1e-16
    assert abs(got[3] - want) < 1e-11 * abs(want), (got[3], want)


def test_printed_wall_flux_over_integrated():
    """The over-integrated form integrates the same wall heat flux exactly at
    the face Gauss points; for the degree-2 density it meets the nodal form's
    total within the interpolation error of E / rho^2 on the faces."""
    m = mg.ogrid(16, 4, 0.5, 2.0, 1.2)
    ft = m["face_tag"].copy()
    ft[ft == mg.TAG_FAR] = mg.TAG_WALL
    dg = build(m, 4, mu=5e-2, theta=1.0, C_pen=1.0, face_tag=ft, wall_heat_flux=True)
    x, y = dg.mesh.x, dg.mesh.y
    rho = 1.0 + 0.1 * x + 0.05 * y * y
    zero = np.zeros_like(x)
    U = np.stack([rho, zero, zero, np.full_like(x, 1.0 / (1.4 * 0.4))])
    nodal = dg.integral(dg.rhs(U))[3]
    oi = dg.integral(DGOracleOI(dg.mesh, dg.phys).rhs(U))[3]
    assert abs(nodal) > 1e-3
    assert abs(oi - nodal) < 1e-3 * abs(nodal)
    dg0 = build(m, 4, mu=5e-2, theta=1.0, C_pen=1.0, face_tag=ft)
    R0 = DGOracleOI(dg0.mesh, dg0.phys).rhs(U)
    assert abs(dg0.integral(R0)[3]) < 1e-12 * np.abs(R0[3]).max()
