"""Pins of the curved-element oracle (oracle/curved.py) against facts that do
not depend on it: the affine oracle where nothing is curved, free-stream
preservation and exact linear fields (the isoparametric property), areas by
Green's theorem on the boundary curves, the exactness of the mass matrices,
a state at rest whose momentum and mass tendencies vanish exactly, the
wall force of a linear pressure field (the divergence theorem over the body
the curved wall encloses), and the order at which the residual of an exact
steady vortex between curved slip walls falls."""
import numpy as np
import pytest
from scipy.special import roots_legendre

import meshgen as mg
from oracle.curved import CurvedMesh, DGOracleCurved, wall_force
from oracle.overint import OverIntegration
from tests.oracle_helpers import build


def _retag(m, old, new):
    m = dict(m)
    ft = m["face_tag"].copy()
    ft[ft == old] = new
    m["face_tag"] = ft
    return m


def _curved(m, p, tag=mg.TAG_WALL, **over):
    dg = build(m, p, **over)
    e, xy = mg.curve_wall(m, dg.mesh.x, dg.mesh.y, tag=tag)
    cm = CurvedMesh(dg.mesh, e, xy)
    return dg, DGOracleCurved(cm, dg.phys), e


@pytest.mark.parametrize("p", [1, 2, 4])
def test_nothing_curved_is_the_affine_oracle(p):
    """No element replaced, or elements replaced by their own straight-sided
    node positions: the nodal oracle's right-hand side, wall force and
    integral to rounding (moving wall, far field, SIPG)."""
    m = mg.ogrid(10, 4, 0.5, 4.0, 1.3)
    dg = build(m, p, mu=5e-3, C_pen=1.0)
    U = mg.noisy_free_stream((4,) + dg.mesh.x.shape, dg.phys.U_inf, np.random.default_rng(3), amp=1e-2)
    vw = (0.01, -0.02)
    want = dg.rhs(U, vw)
    scale = np.abs(want).max(axis=(1, 2))
    wall = np.nonzero((m["face_tag"] == mg.TAG_WALL).any(axis=1))[0]
    xy = np.stack([dg.mesh.x[:, wall].T, dg.mesh.y[:, wall].T], axis=1)
    for e, pos in ((np.zeros(0, dtype=int), np.zeros((0, 2, dg.ref.Np))), (wall, xy)):
        dc = DGOracleCurved(CurvedMesh(dg.mesh, e, pos), dg.phys)
        got = dc.rhs(U, vw)
        assert np.all(np.abs(got - want).max(axis=(1, 2)) <= 1e-13 * scale)
        from oracle.fsi import wall_force as wf
        assert np.abs(wall_force(dc, U, vw) - wf(dg, U, vw)).max() < 1e-14
        assert np.abs(dc.integral(U) - dg.integral(U)).max() < 1e-12 * np.abs(dg.integral(U)).max()


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_free_stream_is_preserved_on_curved_faces(p):
    """Both circles of an O-grid curved (far-field tags): the uniform state
    is an exact steady solution of the discretisation, which holds only if
    the nodal metric terms, the face normals and sJ come from the same map."""
    m = _retag(mg.ogrid(12, 4, 0.5, 3.0, 1.3), mg.TAG_WALL, mg.TAG_FAR)
    dg, dc, e = _curved(m, p, tag=mg.TAG_FAR, mu=5e-3, C_pen=1.0)
    assert len(e) == 24
    U = np.broadcast_to(dg.phys.U_inf[:, None, None], (4,) + dg.mesh.x.shape).copy()
    R, parts = dc.rhs(U, return_parts=True)
    terms = max(np.abs(parts[k]).max() for k in ("vol", "surf"))
    assert terms > 1.0
    assert np.abs(R).max() < 1e-12 * terms


def test_straight_normals_on_curved_faces_break_the_free_stream():
    """The planted mistake: the straight faces' normals kept on the curved
    faces (metric terms per node) no longer balance the volume term."""
    m = _retag(mg.ogrid(12, 4, 0.5, 3.0, 1.3), mg.TAG_WALL, mg.TAG_FAR)
    dg, dc, e = _curved(m, 3, tag=mg.TAG_FAR, mu=5e-3, C_pen=1.0)
    cm = dc.mesh
    for k in e:
        for f in range(3):
            if m["face_tag"][k, f] == mg.TAG_FAR:
                cm.nx[f, :, k] = dg.mesh.nx[f, k]
                cm.ny[f, :, k] = dg.mesh.ny[f, k]
    U = np.broadcast_to(dg.phys.U_inf[:, None, None], (4,) + dg.mesh.x.shape).copy()
    assert np.abs(dc.rhs(U)).max() > 1e-4


def _green_area(m, cm, p):
    """Area inside the boundary curves: sum over boundary faces of
    int x dy along the face's polynomial interpolant (face nodes' own
    parameter, numpy polynomial fits), traversed as the elements run."""
    ref = cm.ref
    xg, wg = roots_legendre(2 * p + 4)
    total = 0.0
    for k, f in zip(*np.nonzero(m["face_tag"] != mg.TAG_INTERIOR)):
        nodes = ref.Fmask[f]
        r, s = ref.r[nodes], ref.s[nodes]
        xi = r if f == 0 else (s if f == 1 else -s)
        cx = np.polynomial.polynomial.polyfit(xi, cm.x[nodes, k], p)
        cy = np.polynomial.polynomial.polyfit(xi, cm.y[nodes, k], p)
        X = np.polynomial.polynomial.polyval(xg, cx)
        dY = np.polynomial.polynomial.polyval(xg, np.polynomial.polynomial.polyder(cy))
        total += wg @ (X * dY)
    return total


@pytest.mark.parametrize("p", [2, 3, 5])
def test_areas_and_mass_matrices(p):
    m = mg.ogrid(10, 3, 0.5, 2.0, 1.3)
    dg, dc, e = _curved(m, p)
    cm = dc.mesh
    green = _green_area(m, cm, p)
    # the curved wall bulges into the body: less fluid than the straight mesh
    assert green < dg.mesh.area.sum()
    assert abs(cm.area.sum() - green) < 1e-12 * green
    # mass matrices: symmetric, positive definite, integrating 1 to |K|, and
    # unchanged by a rule of higher degree (exactness)
    assert np.abs(cm.MK - np.transpose(cm.MK, (0, 2, 1))).max() < 1e-15
    assert np.all(np.linalg.eigvalsh(cm.MK) > 0.0)
    one = np.ones(dg.ref.Np)
    assert np.abs(np.einsum("i,kij,j->k", one, cm.MK, one) - cm.area).max() < 1e-14 * cm.area.max()
    oi = OverIntegration(dg.ref, pf=6 * p)
    Jq = (oi.Drq @ cm.x) * (oi.Dsq @ cm.y) - (oi.Dsq @ cm.x) * (oi.Drq @ cm.y)
    MK2 = np.einsum("q,qk,qi,qj->kij", oi.wq, Jq, oi.Iq, oi.Iq)
    assert np.abs(MK2 - cm.MK).max() < 1e-14 * np.abs(cm.MK).max()
    # affine elements: M^K = J M
    flat = np.setdiff1d(np.arange(dg.mesh.K), e)
    assert np.abs(cm.MK[flat] - dg.mesh.J[flat, None, None] * dg.ref.M[None]).max() < 1e-14
    # curved face lengths: at least the chord, and the arc to the interpolation error
    for k in e:
        f = int(np.nonzero(m["face_tag"][k] == mg.TAG_WALL)[0][0])
        arc = 0.5 * 2.0 * np.pi / 10
        assert cm.face_len[f, k] > dg.mesh.face_len[f, k]
        assert abs(cm.face_len[f, k] - arc) < 1e-2 ** (p - 1) * arc


@pytest.mark.parametrize("p", [2, 4])
def test_linear_fields_have_exact_gradients(p):
    """a + b x + c y is in the isoparametric space: its nodal gradient is
    (b, c) at every node, curved elements included."""
    m = mg.ogrid(10, 3, 0.5, 2.0, 1.3)
    dg, dc, e = _curved(m, p)
    cm = dc.mesh
    coef = np.array([[1.0, 0.3, -0.2], [0.1, -0.5, 0.7], [-0.4, 0.2, 0.9], [2.0, 0.05, 0.11]])
    U = coef[:, 0, None, None] + coef[:, 1, None, None] * cm.x + coef[:, 2, None, None] * cm.y
    Ux, Uy = dc.gradient(U)
    assert np.abs(Ux - coef[:, 1, None, None]).max() < 1e-12
    assert np.abs(Uy - coef[:, 2, None, None]).max() < 1e-12
    # the straight-sided metrics on the curved elements would not be exact
    Ux2 = dg.mesh.rx * np.einsum("ij,fjk->fik", dg.ref.Dr, U) + dg.mesh.sx * np.einsum(
        "ij,fjk->fik", dg.ref.Ds, U)
    assert np.abs(Ux2[:, :, e] - coef[:, 1, None, None]).max() > 1e-3


@pytest.mark.parametrize("p", [2, 3, 4])
def test_rest_with_linear_density_in_a_curved_annulus(p):
    """Fluid at rest between two curved walls, uniform pressure, density
    linear in x and y (exactly represented): mass and momentum tendencies
    vanish at every node (pressure balanced through the curved walls), and
    heat diffuses inside while the adiabatic walls keep the total energy."""
    gamma = 1.4
    m = _retag(mg.ogrid(14, 4, 0.5, 2.0, 1.2), mg.TAG_FAR, mg.TAG_WALL)
    dg, dc, e = _curved(m, p, mu=5e-2, theta=1.0, C_pen=1.0)
    assert len(e) == 28
    cm = dc.mesh
    rho = 1.0 + 0.1 * cm.x - 0.05 * cm.y
    zero = np.zeros_like(rho)
    U = np.stack([rho, zero, zero, np.full_like(rho, 1.0 / (gamma * (gamma - 1.0)))])
    R, parts = dc.rhs(U, return_parts=True)
    terms = max(np.abs(parts[k]).max() for k in ("vol", "surf", "theta"))
    assert np.abs(R[:3]).max() < 1e-12 * terms
    assert np.abs(R[3]).max() > 1e-4
    tot = dc.integral(R)
    assert abs(tot[3]) < 1e-12 * np.abs(R[3]).max()


@pytest.mark.parametrize("p", [2, 3, 4])
def test_wall_force_of_a_linear_pressure(p):
    """At rest with p = a + b x: the force on the body is -b times the area
    the curved wall encloses (divergence theorem; n sJ is a polynomial along
    each face, so the face quadrature is exact), that area by Green's theorem
    on the wall's interpolant."""
    gamma = 1.4
    m = mg.ogrid(10, 3, 0.5, 2.0, 1.3)
    dg, dc, e = _curved(m, p, mu=1e-3)
    cm = dc.mesh
    a, b = 1.0 / gamma, 0.05
    pres = a + b * cm.x
    zero = np.zeros_like(pres)
    U = np.stack([np.ones_like(pres), zero, zero, pres / (gamma - 1.0)])
    F = wall_force(dc, U)
    # the body's area: the wall faces traversed as the fluid elements run
    # (clockwise about the body) give minus the body's area
    ref = dg.ref
    xg, wg = roots_legendre(2 * p + 4)
    body = 0.0
    for k, f in zip(*np.nonzero(m["face_tag"] == mg.TAG_WALL)):
        nodes = ref.Fmask[f]
        r, s = ref.r[nodes], ref.s[nodes]
        xi = r if f == 0 else (s if f == 1 else -s)
        cx = np.polynomial.polynomial.polyfit(xi, cm.x[nodes, k], p)
        cy = np.polynomial.polynomial.polyfit(xi, cm.y[nodes, k], p)
        body -= wg @ (np.polynomial.polynomial.polyval(xg, cx)
                      * np.polynomial.polynomial.polyval(xg, np.polynomial.polynomial.polyder(cy)))
    assert abs(body - np.pi * 0.25) < 5e-2 * np.pi * 0.25
    assert abs(F[0] + b * body) < 1e-13
    assert abs(F[1]) < 1e-13


def _potential_vortex(x, y, gamma=1.4, circ=0.5):
    """u_theta = circ / (2 pi r), homentropic (c_inf = 1 at infinity): an exact
    steady solution of the Euler equations between circular slip walls."""
    r2 = x * x + y * y
    ut = circ / (2.0 * np.pi * np.sqrt(r2))
    u, v = -ut * y / np.sqrt(r2), ut * x / np.sqrt(r2)
    c2 = 1.0 - 0.5 * (gamma - 1.0) * ut * ut
    rho = c2 ** (1.0 / (gamma - 1.0))
    pr = rho ** gamma / gamma
    return np.stack([rho, rho * u, rho * v, pr / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


def _annulus_walls(nt, nr):
    m = _retag(mg.ogrid(nt, nr, 0.5, 1.5, 1.0), mg.TAG_FAR, mg.TAG_WALL)
    return m


def vortex_residuals(p, levels=((8, 2), (16, 4), (32, 8))):
    """Mass-norm residual of the exact state on straight and curved annuli."""
    out = []
    for nt, nr in levels:
        m = _annulus_walls(nt, nr)
        dg, dc, _ = _curved(m, p, mu=0.0, C_pen=1.0)
        rs = dg.l2_norm(dg.rhs(_potential_vortex(dg.mesh.x, dg.mesh.y))).max()
        R = dc.rhs(_potential_vortex(dc.mesh.x, dc.mesh.y))
        rc = np.sqrt(np.einsum("fik,kij,fjk->f", R, dc.mesh.MK, R)).max()
        out.append((rs, rc))
    return np.array(out)


@pytest.mark.parametrize("p", [2, 3, 4])
def test_curved_walls_converge_on_an_exact_vortex(p):
    """With mu = 0 the wall flux is the slip wall's (pressure only) and the
    potential vortex is steady: the discrete residual of the exact state
    measures the consistency error.  Curved walls: it falls at order about p
    (rates above p - 0.5 over two refinements); straight walls (polygons):
    the wall normals are wrong by O(h) and it stalls (rates below 1)."""
    r = vortex_residuals(p)
    rate_s = np.log2(r[:-1, 0] / r[1:, 0])
    rate_c = np.log2(r[:-1, 1] / r[1:, 1])
    assert np.all(rate_c > p - 0.5), rate_c
    assert np.all(rate_s < 1.0), rate_s
    assert r[-1, 1] < 0.1 * r[-1, 0]
