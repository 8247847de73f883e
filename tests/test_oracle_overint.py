"""Pins of the over-integrated oracle (oracle/overint.py) against what the
mathematics fixes: exactness of its quadrature rules (closed-form monomial
integrals), agreement with the nodal oracle wherever both integrate exactly
(fluxes that are polynomials of degree <= p on every element), free-stream
preservation and discrete conservation."""
import numpy as np
import pytest

import meshgen as mg
from oracle.overint import (DGOracleOI, rule_points, simplex_monomial_integral,
                            triangle_rule)
from tests.oracle_helpers import build, uniform


def build_oi(mesh, p, **kw):
    dg = build(mesh, p, **kw)
    return DGOracleOI(dg.mesh, dg.phys), dg


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_triangle_rule_is_exact_to_degree_3p(p):
    q = rule_points(p)
    r, s, w = triangle_rule(q)
    assert np.all(w > 0) and np.all(r + s <= 1e-14) and np.all(r >= -1) and np.all(s >= -1)
    worst = 0.0
    for a in range(3 * p + 1):
        for b in range(3 * p + 1 - a):
            exact = simplex_monomial_integral(a, b)
            worst = max(worst, abs(np.sum(w * r ** a * s ** b) - exact))
    assert worst < 1e-13
    # and not beyond 2q - 1: some monomial of degree 2q is integrated inexactly
    deg = 2 * q
    errs = [abs(np.sum(w * r ** a * s ** (deg - a)) - simplex_monomial_integral(a, deg - a))
            for a in range(deg + 1)]
    assert max(errs) > 1e-10


def test_monomial_closed_form():
    # area, first moments (centroid (-1/3, -1/3)) and one second moment by hand
    assert simplex_monomial_integral(0, 0) == pytest.approx(2.0)
    assert simplex_monomial_integral(1, 0) == pytest.approx(-2.0 / 3.0)
    assert simplex_monomial_integral(0, 1) == pytest.approx(-2.0 / 3.0)
    # int r^2 over {r, s >= -1, r + s <= 0}: int_{-1}^{1} r^2 (-r + 1) dr = 2/3
    assert simplex_monomial_integral(2, 0) == pytest.approx(2.0 / 3.0)


def polynomial_flux_state(dg, gamma=1.4):
    """Constant density and pressure, velocity linear in x and y: every flux
    (advective, viscous, wall-free interior faces) is a polynomial of degree
    <= 3 in x and y, and the state is continuous across faces."""
    x, y = dg.mesh.x, dg.mesh.y
    rho = np.ones_like(x)
    u = 0.2 + 0.05 * x - 0.03 * y
    v = -0.04 + 0.02 * x + 0.06 * y
    p = np.full_like(x, 1.0 / gamma)
    return np.stack([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


@pytest.mark.parametrize("p", [3, 4])
def test_equals_nodal_oracle_for_polynomial_fluxes(p):
    m = mg.ogrid(12, 4, 0.5, 4.0, 1.3)
    oi, dg = build_oi(m, p, mu=2e-2)
    U = polynomial_flux_state(dg)
    R_oi = oi.rhs(U, vw=(0.01, -0.02))
    R_nd, parts = dg.rhs(U, vw=(0.01, -0.02), return_parts=True)
    inner = ~dg.mesh.is_boundary.any(axis=1)
    assert inner.sum() > 20
    # the residual is a difference of volume and surface terms: bound the
    # roundoff by the larger term (normalised bound of the parity reading)
    scale = max(np.abs(parts["vol"][:, :, inner]).max(), np.abs(parts["surf"][:, :, inner]).max())
    assert np.abs(R_oi[:, :, inner] - R_nd[:, :, inner]).max() <= 1e-13 * scale


def test_differs_from_nodal_when_the_flux_is_not_resolved():
    # at p = 2 the degree-3 fluxes are aliased by nodal interpolation
    m = mg.ogrid(12, 4, 0.5, 4.0, 1.3)
    oi, dg = build_oi(m, 2, mu=2e-2)
    U = polynomial_flux_state(dg)
    inner = ~dg.mesh.is_boundary.any(axis=1)
    R_oi, R_nd = oi.rhs(U), dg.rhs(U)
    d = np.abs(R_oi[:, :, inner] - R_nd[:, :, inner]).max()
    assert d > 1e-8 * np.abs(R_nd[:, :, inner]).max()


@pytest.mark.parametrize("p", [1, 3, 4, 6])
@pytest.mark.parametrize("vw", [(0.0, 0.0), (0.04, -0.13)])
def test_free_stream_preserved(p, vw):
    oi, dg = build_oi(mg.periodic_square(3, 3, 2.0, 2.0), p)
    U = uniform(dg, dg.phys.U_inf)
    assert np.abs(oi.rhs(U, vw)).max() < 1e-12 * p * p
    m = mg.ogrid(10, 4, 0.5, 4.0, 1.3)
    ft = m["face_tag"].copy()
    ft[ft == 1] = 2
    oi, dg = build_oi(m, p, face_tag=ft)
    U = uniform(dg, dg.phys.U_inf)
    assert np.abs(oi.rhs(U, vw)).max() < 1e-11 * p * p


@pytest.mark.parametrize("p", [2, 4, 5])
def test_conservation_periodic(p):
    oi, dg = build_oi(mg.periodic_square(4, 3, 3.0, 2.0), p, mu=0.05)
    x, y = dg.mesh.x, dg.mesh.y
    rng = np.random.default_rng(p)
    U = mg.fourier_modes(x, y, rng, L=1.0, amp=0.05) + 0.01 * rng.standard_normal((4,) + x.shape)
    R = oi.rhs(U, vw=(0.02, 0.01))
    assert np.abs(dg.integral(R)).max() < 1e-12 * np.abs(R).max()


def test_higher_rule_changes_only_the_aliasing():
    # a smooth non-polynomial state: the over-integrated result moves towards
    # the exact integral as the rule grows, and less than the nodal one differs
    m = mg.periodic_square(4, 4, 10.0, 10.0)
    dg = build(m, 4, mu=3e-3)
    x, y = dg.mesh.x, dg.mesh.y
    U = mg.fourier_modes(x, y, np.random.default_rng(5), L=10.0, amp=0.05)
    R12 = DGOracleOI(dg.mesh, dg.phys).rhs(U)
    R18 = DGOracleOI(dg.mesh, dg.phys, pf=18).rhs(U)
    R24 = DGOracleOI(dg.mesh, dg.phys, pf=24).rhs(U)
    Rn = dg.rhs(U)
    d_oi = np.abs(R12 - R24).max()
    assert np.abs(R18 - R24).max() < d_oi
    assert d_oi < np.abs(Rn - R24).max()
