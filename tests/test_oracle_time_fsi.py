"""Pins of the oracle's time integrator, rigid-body step, force and manufactured source (CPU).

* LSERK: the 2N-storage coefficients, converted to a Butcher tableau, satisfy
  all eight order conditions of order 4, and the stage times c_i are its row
  sums; the step has order 4 on y' = lambda y.
* Newmark (beta = 1/4, gamma = 1/2): undamped free vibration conserves
  (y'^2 + omega^2 y^2)/2, a constant load relaxes to F/K with damping.
* Force: a uniform pressure on a closed polygonal wall exerts no force; a
  linear pressure p0 + a.x exerts -a |polygon| (divergence theorem).
* Manufactured source: re-derived here symbolically from the textbook
  Navier-Stokes fluxes (sympy), independently of the oracle's flux code.
"""
import math

import numpy as np
import pytest

import meshgen as mg
from oracle import fsi, manufactured
from oracle.dg import LSERK_A, LSERK_B, LSERK_C
from tests.oracle_helpers import build, uniform


def _butcher(Acoef, Bcoef):
    s = len(Acoef)
    a = np.zeros((s + 1, s))
    for i in range(1, s + 1):
        for j in range(1, i + 1):
            tot = 0.0
            for l in range(j, i + 1):
                pr = 1.0
                for m in range(j + 1, l + 1):
                    pr *= Acoef[m - 1]
                tot += Bcoef[l - 1] * pr
            a[i, j - 1] = tot
    return a[:s, :], a[s, :]


def test_lserk_order_conditions():
    a, b = _butcher(LSERK_A, LSERK_B)
    c = a.sum(axis=1)
    assert np.abs(c - np.array(LSERK_C)).max() < 1e-15
    conds = [b.sum() - 1, b @ c - 1 / 2, b @ c ** 2 - 1 / 3, b @ a @ c - 1 / 6,
             b @ c ** 3 - 1 / 4, b @ (c * (a @ c)) - 1 / 8, b @ a @ c ** 2 - 1 / 12,
             b @ a @ a @ c - 1 / 24]
    assert max(abs(x) for x in conds) < 1e-15
    assert LSERK_A[0] == 0.0


def test_lserk_fourth_order_on_linear_ode():
    lam = -1.0 + 2.0j
    errs = []
    for n in (10, 20, 40):
        dt = 1.0 / n
        y = 1.0 + 0j
        for _ in range(n):
            k1 = 0j
            for a, b in zip(LSERK_A, LSERK_B):
                k1 = a * k1 + dt * lam * y
                y = y + b * k1
        errs.append(abs(y - np.exp(lam)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates.min() > 3.8


def test_newmark_energy_and_static_limit():
    M, C, K = 1.0, 0.0, (2 * math.pi * 0.3) ** 2
    y, yd, ydd = 1.0, 0.0, -K * 1.0
    e0 = 0.5 * (yd ** 2 + K * y ** 2)
    for _ in range(500):
        y, yd, ydd = fsi.newmark_step(y, yd, ydd, 0.0, 0.05, M, C, K)
    assert abs(0.5 * (yd ** 2 + K * y ** 2) - e0) < 1e-12 * e0
    y, yd, ydd = 0.0, 0.0, 0.0
    for _ in range(4000):
        y, yd, ydd = fsi.newmark_step(y, yd, ydd, 0.7, 0.05, M, 0.5, K)
    assert abs(y - 0.7 / K) < 1e-9


@pytest.mark.parametrize("p", [1, 3])
def test_force_closed_forms(p):
    nt = 16
    R0 = 0.5
    dg = build(mg.ogrid(nt, 3, R0, 3.0, 1.2), p, U_inf=mg.free_stream(0.0))
    x, y = dg.mesh.x, dg.mesh.y
    area = 0.5 * nt * R0 ** 2 * math.sin(2 * math.pi / nt)
    gam = dg.phys.gamma
    for a, b, p0 in [(0.0, 0.0, 0.7), (0.03, -0.05, 0.7)]:
        pres = p0 + a * x + b * y
        U = np.stack([np.ones_like(x), 0 * x, 0 * x, pres / (gam - 1.0)])
        F = fsi.wall_force(dg, U)
        assert abs(F[0] + a * area) < 1e-13 and abs(F[1] + b * area) < 1e-13
        assert abs(F[2]) < 1e-13


def test_viv_coefficients():
    Mr, Cr, Kr, inv_m = fsi.viv_coefficients(5.0, 10.0, 0.01, 0.2)
    fn = 0.2 / 5.0
    assert Mr == 1.0 and abs(Cr - 4 * math.pi * fn * 0.01) < 1e-15
    assert abs(Kr - 1.1 * (2 * math.pi * fn) ** 2) < 1e-15
    assert abs(inv_m - 1.0 / (10.0 * math.pi / 4.0)) < 1e-15


def test_manufactured_source_symbolic():
    sp = pytest.importorskip("sympy")
    x, y = sp.symbols("x y", real=True)
    g, Pr, mu, kap, C2 = sp.Rational(7, 5), sp.Rational(18, 25), sp.Rational(1, 100), 25, 200
    s = sp.sin(kap * (x + y)) + C2
    rho, u, v, E = s, sp.Integer(1), sp.Integer(1), s * s     # U = [s, s, s, s^2]
    p = (g - 1) * (E - rho * (u * u + v * v) / 2)
    e = E / rho - (u * u + v * v) / 2
    txx = mu * (sp.Rational(4, 3) * sp.diff(u, x) - sp.Rational(2, 3) * sp.diff(v, y))
    tyy = mu * (sp.Rational(4, 3) * sp.diff(v, y) - sp.Rational(2, 3) * sp.diff(u, x))
    txy = mu * (sp.diff(u, y) + sp.diff(v, x))
    kq = mu * g / Pr
    Fx = [rho * u - 0, rho * u * u + p - txx, rho * u * v - txy,
          u * (E + p) - (u * txx + v * txy + kq * sp.diff(e, x))]
    Fy = [rho * v, rho * u * v - txy, rho * v * v + p - tyy,
          v * (E + p) - (u * txy + v * tyy + kq * sp.diff(e, y))]
    S = [sp.diff(Fx[i], x) + sp.diff(Fy[i], y) for i in range(4)]
    f = sp.lambdify((x, y), S, "numpy")
    rng = np.random.default_rng(0)
    X, Y = rng.uniform(0, 1, 20), rng.uniform(0, 1, 20)
    want = np.array([np.broadcast_to(c, X.shape) for c in f(X, Y)], dtype=float)
    got = manufactured.source(X, Y, gamma=1.4, Pr=0.72, mu=0.01)
    assert np.abs(got - want).max() < 1e-9 * np.abs(want).max()
