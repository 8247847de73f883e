"""Pins of the CFL time-step oracle (oracle/cfl.py, eq. cfl_general with the
bound of eq. rayleigh_bound) against what geometry and the mathematics fix:
the inscribed radius and trace-inverse constant of right triangles by hand,
the wave speed of a uniform state, the divergence of a linear velocity
field, the neighbour maximum of G_K, and the bound itself against the
spectrum of the linearised right-hand side on a small mesh."""
import math

import numpy as np
import pytest

import meshgen as mg
from oracle.cfl import CFLOracle, inradius, trace_inverse_max
from tests.oracle_helpers import build, uniform


def cfl(mesh, p, **kw):
    dg = build(mesh, p, **kw)
    return CFLOracle(dg.mesh, dg.phys), dg


def test_inradius_and_trace_inverse_of_right_triangles():
    # every element of the split square is a right isosceles triangle with
    # legs h: inscribed radius (a + b - c) / 2, longest edge h sqrt 2
    h = 0.25
    for p in (1, 3, 5):
        c, dg = cfl(mg.periodic_square(8, 8, 2.0, 2.0), p)
        assert np.allclose(inradius(dg.mesh), (2.0 * h - h * math.sqrt(2.0)) / 2.0, rtol=1e-14)
        Np = (p + 1) * (p + 2) // 2
        assert np.allclose(trace_inverse_max(dg.mesh), Np * h * math.sqrt(2.0) / (h * h / 2.0),
                           rtol=1e-14)


@pytest.mark.parametrize("vw", [(0.0, 0.0), (0.03, -0.07)])
def test_uniform_state(vw):
    # rho = 1, p = 1/gamma: sound speed 1; |v - v_w| from the free stream
    c, dg = cfl(mg.periodic_square(3, 3, 1.0, 1.0), 2)
    U = uniform(dg, mg.free_stream(0.2))
    parts = c.parts(U, vw)
    assert np.allclose(parts["beta"], math.hypot(0.2 - vw[0], vw[1]) + 1.0, rtol=1e-14)
    assert np.abs(parts["beta1"]).max() < 1e-12
    # no jumps: every face sees one state, and G_K is that state's value
    assert np.ptp(parts["G"]) < 1e-15 * parts["G"].max()


@pytest.mark.parametrize("p", [1, 2, 4])
def test_divergence_of_a_linear_velocity_field(p):
    m = mg.ogrid(10, 4, 0.5, 3.0, 1.2)
    c, dg = cfl(m, p)
    x, y = dg.mesh.x, dg.mesh.y
    u = 0.1 + 0.03 * x - 0.02 * y
    v = -0.05 + 0.01 * x + 0.05 * y
    rho = np.ones_like(x)
    pr = np.full_like(x, 1.0 / 1.4)
    U = np.stack([rho, rho * u, rho * v, pr / 0.4 + 0.5 * rho * (u * u + v * v)])
    parts = c.parts(U)
    assert np.allclose(parts["beta1"], 0.5 * abs(0.03 + 0.05), rtol=1e-10)


def test_G_takes_the_neighbour_maximum():
    # lower density in one element raises mu/rho there; its face neighbours
    # inherit its value, elements further away do not
    c, dg = cfl(mg.periodic_square(4, 4, 1.0, 1.0), 2, mu=1e-2)
    U = uniform(dg, mg.free_stream(0.2))
    k0 = 5
    U[:, :, k0] *= 0.5          # rho halved, same velocity, pressure halved
    parts = c.parts(U)
    nb = dg.mesh.EToE[k0]
    assert np.all(parts["G"][nb] == parts["G"][k0])
    far = [k for k in range(dg.mesh.K) if k != k0 and k not in nb]
    assert np.all(parts["G"][far] < parts["G"][k0])
    assert parts["G"][k0] == pytest.approx(2.0 * parts["G"][far].min(), rel=1e-12)


def test_sigma_is_the_rhs_penalty():
    c, dg = cfl(mg.ogrid(12, 4, 0.5, 4.0, 1.3), 3, mu=5e-3)
    rng = np.random.default_rng(4)
    U = mg.noisy_free_stream((4, dg.ref.Np, dg.mesh.K), dg.phys.U_inf, rng, amp=1e-2)
    _, rp = dg.rhs(U, (0.0, 0.02), return_parts=True)
    assert np.array_equal(c.parts(U, (0.0, 0.02))["sigma"], rp["sigma"].max(axis=0))


def test_bound_covers_the_spectrum():
    """Lambda of eq. rayleigh_bound (C_grad = 1) against the eigenvalues of
    the right-hand side linearised about a free stream on a small mesh
    (central differences): every |lambda| lies below Lambda."""
    for p, mu in ((1, 5e-2), (2, 2e-2), (3, 1e-3)):
        c, dg = cfl(mg.periodic_square(2, 2, 1.0, 1.0), p, mu=mu, C_pen=1.0)
        U0 = uniform(dg, mg.free_stream(0.3))
        n = U0.size
        J = np.empty((n, n))
        eps = 1e-6
        for i in range(n):
            d = np.zeros(n)
            d[i] = eps
            J[:, i] = ((dg.rhs(U0 + d.reshape(U0.shape)) - dg.rhs(U0 - d.reshape(U0.shape)))
                       / (2.0 * eps)).ravel()
        lam_max = np.abs(np.linalg.eigvals(J)).max()
        lam, dt = c.time_step(U0, C_cfl=1.0)
        assert lam_max <= lam, (p, lam_max, lam)
        assert dt == pytest.approx(1.0 / lam)
