"""Pins of the oracle's pointwise physics (CPU).

* The viscous flux, computed by the oracle from primitive gradients, must equal
  the paper's printed G-block tables (Sec. 2.1), typed in here -- an independent
  route to the same operator, which also fixes the equation-of-state reading.
* The eigen-based Roe flux must satisfy the Rankine-Hugoniot property of the
  Roe matrix (Sec. 2.2.1), consistency, conservation symmetry, and agree with
  the textbook wave-strength form of the Roe flux (typed in here).
* ||N G N^T||_2 has a closed form at rest and is rotation invariant.
"""
import math

import numpy as np
import pytest

from oracle import physics as ph

GAMMA, PR, MU = 1.4, 0.72, 0.013


def random_states(rng, n, M=0.3):
    rho = 1.0 + 0.2 * rng.uniform(-1, 1, n)
    u = M * rng.uniform(-1.5, 1.5, n)
    v = M * rng.uniform(-1.5, 1.5, n)
    p = 1.0 / GAMMA * (1.0 + 0.2 * rng.uniform(-1, 1, n))
    return ph.conservative(rho, u, v, p, GAMMA)


def paper_g_blocks(U):
    """The four 4x4 blocks G11, G12, G21, G22 as printed in Sec. 2.1."""
    rho = U[0]
    v1, v2 = U[1] / rho, U[2] / rho
    eps = U[3]
    k = GAMMA / PR
    vv = v1 * v1 + v2 * v2
    z = np.zeros_like(rho)
    g41 = [-v * v / 3.0 - vv - k * (eps / rho - vv) for v in (v1, v2)]
    G11 = [[z, z, z, z],
           [-4.0 / 3.0 * v1, 4.0 / 3.0 + z, z, z],
           [-v2, z, 1.0 + z, z],
           [g41[0], (4.0 / 3.0 - k) * v1, (1.0 - k) * v2, k + z]]
    G12 = [[z, z, z, z],
           [2.0 / 3.0 * v2, z, -2.0 / 3.0 + z, z],
           [-v1, 1.0 + z, z, z],
           [-v1 * v2 / 3.0, v2, -2.0 / 3.0 * v1, z]]
    G21 = [[z, z, z, z],
           [-v2, z, 1.0 + z, z],
           [2.0 / 3.0 * v1, -2.0 / 3.0 + z, z, z],
           [-v1 * v2 / 3.0, -2.0 / 3.0 * v2, v1, z]]
    G22 = [[z, z, z, z],
           [-v1, 1.0 + z, z, z],
           [-4.0 / 3.0 * v2, z, 4.0 / 3.0 + z, z],
           [g41[1], (1.0 - k) * v1, (4.0 / 3.0 - k) * v2, k + z]]
    f = MU / rho
    return [np.array(B) * f for B in (G11, G12, G21, G22)]


def test_viscous_flux_equals_printed_g_tables():
    rng = np.random.default_rng(1)
    U = random_states(rng, 200)
    Ux = rng.standard_normal(U.shape)
    Uy = rng.standard_normal(U.shape)
    fx, fy = ph.viscous_flux(U, Ux, Uy, MU, PR, GAMMA)
    G11, G12, G21, G22 = paper_g_blocks(U)
    gx = np.einsum('ijn,jn->in', G11, Ux) + np.einsum('ijn,jn->in', G12, Uy)
    gy = np.einsum('ijn,jn->in', G21, Ux) + np.einsum('ijn,jn->in', G22, Uy)
    assert np.abs(fx - gx).max() < 1e-14 * (1 + np.abs(gx).max())
    assert np.abs(fy - gy).max() < 1e-14 * (1 + np.abs(gy).max())
    G = ph.g_matrix(U, MU, PR, GAMMA)
    assert np.abs(np.moveaxis(G[..., 0:4, 4:8], 0, -1) - G12).max() < 1e-15


def textbook_roe(UL, UR, nx, ny, vw):
    """Roe flux in wave-strength form (Roe 1981; LeVeque ch. 15), moving-frame eigenvalues."""
    rl, ul, vl, pl = ph.primitives(UL, GAMMA)
    rr, ur, vr, pr = ph.primitives(UR, GAMMA)
    hl, hr = (UL[3] + pl) / rl, (UR[3] + pr) / rr
    sl, sr = np.sqrt(rl), np.sqrt(rr)
    rt = sl * sr
    ut = (sl * ul + sr * ur) / (sl + sr)
    vt = (sl * vl + sr * vr) / (sl + sr)
    ht = (sl * hl + sr * hr) / (sl + sr)
    ct = np.sqrt((GAMMA - 1.0) * (ht - 0.5 * (ut * ut + vt * vt)))
    qn = ut * nx + vt * ny
    qt = -ut * ny + vt * nx
    vwn = vw[0] * nx + vw[1] * ny
    dr, dp = rr - rl, pr - pl
    dqn = (ur - ul) * nx + (vr - vl) * ny
    dqt = -(ur - ul) * ny + (vr - vl) * nx
    a1 = (dp - rt * ct * dqn) / (2 * ct * ct)
    a2 = dr - dp / (ct * ct)
    a3 = rt * dqt
    a4 = (dp + rt * ct * dqn) / (2 * ct * ct)
    one = np.ones_like(ut)
    r1 = np.stack([one, ut - ct * nx, vt - ct * ny, ht - ct * qn])
    r2 = np.stack([one, ut, vt, 0.5 * (ut * ut + vt * vt)])
    r3 = np.stack([0 * one, -ny * one, nx * one, qt])
    r4 = np.stack([one, ut + ct * nx, vt + ct * ny, ht + ct * qn])
    diss = (np.abs(qn - ct - vwn) * a1 * r1 + np.abs(qn - vwn) * (a2 * r2 + a3 * r3)
            + np.abs(qn + ct - vwn) * a4 * r4)
    fl = ph.normal_flux(UL, nx, ny, vw, GAMMA)
    fr = ph.normal_flux(UR, nx, ny, vw, GAMMA)
    return 0.5 * (fl + fr) - 0.5 * diss


@pytest.mark.parametrize("vw", [(0.0, 0.0), (0.07, -0.11)])
def test_roe_flux_against_wave_strength_form(vw):
    rng = np.random.default_rng(2)
    n = 300
    UL, UR = random_states(rng, n), random_states(rng, n)
    ang = rng.uniform(0, 2 * math.pi, n)
    nx, ny = np.cos(ang), np.sin(ang)
    # include axis-aligned normals and equal-velocity pairs (repeated eigenvalues)
    nx[:20], ny[:20] = 1.0, 0.0
    UR[:, 20:40] = UL[:, 20:40] * (1 + 1e-3)
    got = ph.roe_flux(UL, UR, nx, ny, vw, GAMMA)
    want = textbook_roe(UL, UR, nx, ny, vw)
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()


def test_roe_properties():
    rng = np.random.default_rng(3)
    n = 200
    UL, UR = random_states(rng, n), random_states(rng, n)
    ang = rng.uniform(0, 2 * math.pi, n)
    nx, ny = np.cos(ang), np.sin(ang)
    vw = (0.05, 0.02)
    # consistency F(u, u) = F_n(u)
    assert np.abs(ph.roe_flux(UL, UL, nx, ny, vw, GAMMA)
                  - ph.normal_flux(UL, nx, ny, vw, GAMMA)).max() < 1e-14
    # Rankine-Hugoniot property of the Roe matrix (Sec. 2.2.1)
    A = ph.flux_jacobian(ph.roe_average(UL, UR, GAMMA), nx, ny, vw, GAMMA)
    dF = ph.normal_flux(UR, nx, ny, vw, GAMMA) - ph.normal_flux(UL, nx, ny, vw, GAMMA)
    AdU = np.einsum('nij,jn->in', A, UR - UL)
    assert np.abs(AdU - dF).max() < 1e-13
    # conservation: F(UL, UR, n) = -F(UR, UL, -n)
    f1 = ph.roe_flux(UL, UR, nx, ny, vw, GAMMA)
    f2 = ph.roe_flux(UR, UL, -nx, -ny, vw, GAMMA)
    assert np.abs(f1 + f2).max() < 1e-13


def test_abs_matrix_matches_eigendecomposition():
    rng = np.random.default_rng(4)
    R = rng.standard_normal((50, 4, 4)) + 4 * np.eye(4)
    lam = rng.uniform(-2, 2, (50, 4))
    A = R @ (lam[..., :, None] * np.linalg.inv(R))
    w = rng.standard_normal((50, 4))
    want = np.einsum('nij,nj->ni', R @ (np.abs(lam)[..., :, None] * np.linalg.inv(R)), w)
    assert np.abs(ph.abs_matrix_apply(A, w) - want).max() < 1e-9 * np.abs(want).max()


def test_normal_diffusion_norm_closed_form_and_rotation():
    rng = np.random.default_rng(5)
    # at rest with n = (1, 0): ||A|| = mu/rho max(4/3, sqrt(g41^2 + (gamma/Pr)^2))
    rho = 1.0 + 0.3 * rng.uniform(size=20)
    p = 0.7 + 0.3 * rng.uniform(size=20)
    U = ph.conservative(rho, 0 * rho, 0 * rho, p, GAMMA)
    got = ph.normal_diffusion_norm(U, np.ones(20), np.zeros(20), MU, PR, GAMMA)
    k = GAMMA / PR
    g41 = -k * U[3] / rho
    want = MU / rho * np.maximum(4.0 / 3.0, np.hypot(g41, k))
    assert np.abs(got - want).max() < 1e-14
    # rotating velocity and normal together leaves the norm unchanged
    U = random_states(rng, 100)
    ang = rng.uniform(0, 2 * math.pi, 100)
    nx, ny = np.cos(ang), np.sin(ang)
    a = ph.normal_diffusion_norm(U, nx, ny, MU, PR, GAMMA)
    t = rng.uniform(0, 2 * math.pi, 100)
    c, s = np.cos(t), np.sin(t)
    Ur = U.copy()
    Ur[1], Ur[2] = c * U[1] - s * U[2], s * U[1] + c * U[2]
    b = ph.normal_diffusion_norm(Ur, c * nx - s * ny, s * nx + c * ny, MU, PR, GAMMA)
    assert np.abs(a - b).max() < 1e-14
