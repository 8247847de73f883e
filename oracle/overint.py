"""Over-integrated weak-form right-hand side (oracle; test infrastructure).

The weak form of eq. weak_form / eq. weak_matrices_calc with every integral
taken by a quadrature rule exact for polynomials of degree p_f = 3p on the
element and on each face, instead of integrating the nodal interpolants of
the fluxes (Sec. 2.2, the oversampling remedy for aliasing the paper cites
for subsonic flows):

  M^K dU/dt = sum_q w_q J F(U_h, grad U_h)(x_q) . grad l_i(x_q)
              - sum_e sum_g w_g sJ H_m(x_g) l_i(x_g)
              + sum_e sum_g w_g sJ H_theta(x_g) . grad l_i(x_g)

with U_h and grad U_h evaluated at the quadrature points from the nodal
values, and every flux (Roe, viscous average, penalty, theta term, boundary
ghosts) formed there exactly as the nodal oracle forms it at face nodes.

Readings:

* Volume rule: the collapsed-coordinate (Duffy) product rule, Gauss-Legendre
  in a and Gauss-Jacobi (weight 1 - b) in b with q = ceil((p_f + 1) / 2)
  points each, exact for degree 2q - 1 >= p_f on the reference triangle.
  The paper names symmetric rules with fewer points; any P_{p_f}-exact rule
  gives the same integral for polynomial integrands, and for the rational
  fluxes the difference is of the size of the remaining aliasing error.
* Face rule: Gauss-Legendre with the same q, in the face parameter xi that
  runs counter-clockwise; the neighbour sees the shared face with xi -> -xi,
  and the rule is symmetric, so its point q - 1 - g is the own point g.
* G-bar_e is the largest ||N G N^T||_2 over the face's quadrature points on
  both sides (the face's evaluation points take the place of its nodes).

The library primitives used are Gauss-Jacobi and Gauss-Legendre points and
weights (scipy.special.roots_jacobi) and the nodal basis of oracle.nodes.
"""
import math
from fractions import Fraction

import numpy as np
from scipy.special import roots_jacobi

from . import physics as ph
from .dg import DGOracle
from .mesh import TAG_WALL, TAG_FAR
from .nodes import vandermonde_2d, grad_vandermonde_2d


def rule_points(p, pf=None):
    """Number of points per direction of the degree-pf rules (pf = 3p)."""
    pf = 3 * p if pf is None else pf
    return (pf + 2) // 2


def triangle_rule(q):
    """Collapsed Gauss product rule on the reference triangle
    {r, s >= -1, r + s <= 0}: points (r, s) and weights, q^2 points, exact for
    degree 2q - 1.  r = (1 + a)(1 - b)/2 - 1, s = b, dr ds = (1 - b)/2 da db."""
    a, wa = roots_jacobi(q, 0.0, 0.0)
    b, wb = roots_jacobi(q, 1.0, 0.0)      # weight (1 - b)
    A, B = np.meshgrid(a, b, indexing="ij")
    W = np.outer(wa, wb) * 0.5
    r = 0.5 * (1.0 + A) * (1.0 - B) - 1.0
    return r.ravel(), B.ravel(), W.ravel()


def face_points(f, xi):
    """Reference coordinates of the face parameter xi on face f (face f joins
    vertices f and f + 1; xi runs counter-clockwise, as the face nodes do)."""
    if f == 0:
        return xi, -np.ones_like(xi)
    if f == 1:
        return -xi, xi
    return -np.ones_like(xi), -xi


class OverIntegration:
    """Quadrature points of one order and the nodal basis evaluated there."""

    def __init__(self, ref, pf=None):
        N = ref.N
        self.q = rule_points(N, pf)
        vinv = np.linalg.inv(ref.V)
        r, s, w = triangle_rule(self.q)
        self.wq = w
        self.Iq = vandermonde_2d(N, r, s) @ vinv              # l_j(x_q)
        Vr, Vs = grad_vandermonde_2d(N, r, s)
        self.Drq, self.Dsq = Vr @ vinv, Vs @ vinv             # d_r l_j(x_q), d_s l_j(x_q)
        xi, wg = roots_jacobi(self.q, 0.0, 0.0)
        self.wg = wg
        self.If, self.Drf, self.Dsf = [], [], []
        for f in range(3):
            fr, fs = face_points(f, xi)
            self.If.append(vandermonde_2d(N, fr, fs) @ vinv)
            Vr, Vs = grad_vandermonde_2d(N, fr, fs)
            self.Drf.append(Vr @ vinv)
            self.Dsf.append(Vs @ vinv)


class DGOracleOI(DGOracle):
    """The nodal oracle's physics with over-integrated volume and face terms."""

    def __init__(self, mesh, phys, pf=None):
        super().__init__(mesh, phys)
        self.oi = OverIntegration(mesh.ref, pf)

    def _at_faces(self, A, mats):
        """(C, Np, K) nodal field -> (C, 3, q, K) values at the face points."""
        return np.stack([np.einsum("gj,cjk->cgk", mats[f], A) for f in range(3)], axis=1)

    def rhs(self, U, vw=(0.0, 0.0), source=None, return_parts=False):
        m, p, ref, oi = self.mesh, self.phys, self.ref, self.oi
        vw = np.asarray(vw, dtype=np.float64)
        g = p.gamma
        K, q = m.K, oi.q
        Minv = ref.Minv
        # ---- volume: int_K F . grad l_i by the triangle rule
        Uq = np.einsum("qj,cjk->cqk", oi.Iq, U)
        Urq = np.einsum("qj,cjk->cqk", oi.Drq, U)
        Usq = np.einsum("qj,cjk->cqk", oi.Dsq, U)
        Uxq = m.rx * Urq + m.sx * Usq
        Uyq = m.ry * Urq + m.sy * Usq
        Fx, Fy = self.total_flux(Uq, Uxq, Uyq, vw)
        Fr = m.rx * Fx + m.ry * Fy
        Fs = m.sx * Fx + m.sy * Fy
        w = oi.wq[None, :, None]
        vol = np.einsum("ij,cjk->cik", Minv,
                        np.einsum("qi,cqk->cik", oi.Drq, w * Fr) + np.einsum("qi,cqk->cik", oi.Dsq, w * Fs))
        # ---- face points: own values, the other side's values (mirrored point)
        Up = self._at_faces(U, oi.If)
        Urp = self._at_faces(U, oi.Drf)
        Usp = self._at_faces(U, oi.Dsf)
        rx, ry, sx, sy = (a[None, None, None, :] for a in (m.rx, m.ry, m.sx, m.sy))
        Uxp = rx * Urp + sx * Usp
        Uyp = ry * Urp + sy * Usp
        kn = np.where(m.EToE >= 0, m.EToE, np.arange(K)[:, None]).T     # (3, K)
        fn = np.where(m.EToE >= 0, m.EToF, np.arange(3)[None, :]).T
        gm = np.arange(q)[::-1]
        Um = Up[:, fn[:, None, :], gm[None, :, None], kn[:, None, :]]
        Uxm = Uxp[:, fn[:, None, :], gm[None, :, None], kn[:, None, :]]
        Uym = Uyp[:, fn[:, None, :], gm[None, :, None], kn[:, None, :]]
        tag = m.face_tag.T[None, :, None, :] * np.ones((1, 1, q, 1), dtype=np.int64)
        wall = (tag == TAG_WALL)[0]
        far = (tag == TAG_FAR)[0]
        interior = ~(wall | far)
        Ub_wall = ph.wall_state(Up, vw, g)
        Ub_far = np.broadcast_to(p.U_inf[:, None, None, None], Up.shape)
        Uo = np.where(wall[None], Ub_wall, np.where(far[None], Ub_far, Um))
        nx = m.nx[:, None, :]
        ny = m.ny[:, None, :]
        # advective numerical flux
        Fc = ph.roe_flux(Up, Uo, nx, ny, vw, g)
        Fc = np.where(wall[None], ph.normal_flux(Uo, nx, ny, vw, g), Fc)
        # viscous normal flux
        vxp, vyp = ph.viscous_flux(Up, Uxp, Uyp, p.mu, p.Pr, g)
        vxm, vym = ph.viscous_flux(Uo, Uxm, Uym, p.mu, p.Pr, g)
        vxw, vyw = ph.viscous_flux(Uo, Uxp, Uyp, p.mu, p.Pr_wall, g)    # wall (adiabatic by default)
        vn = np.where(interior[None], 0.5 * ((vxp + vxm) * nx + (vyp + vym) * ny),
                      np.where(wall[None], vxw * nx + vyw * ny, vxp * nx + vyp * ny))
        # penalty: G-bar_e over the face's quadrature points, both sides
        a = ph.normal_diffusion_norm(Up, nx, ny, p.mu, p.Pr, g)
        b = ph.normal_diffusion_norm(Uo, nx, ny, p.mu, p.Pr, g)
        gbar = np.maximum(a.max(axis=1), b.max(axis=1))
        sigma = self.penalty(gbar)
        jump = Up - Uo
        Hm = Fc - vn + sigma[None, :, None, :] * jump
        Fscale = m.Fscale[None, :, None, :]
        wg = oi.wg[None, None, :, None]
        surf = np.zeros_like(U)
        for f in range(3):
            surf -= np.einsum("gi,cgk->cik", oi.If[f], (wg * Fscale * Hm)[:, f])
        surf = np.einsum("ij,cjk->cik", Minv, surf)
        # theta term: c_e theta G(U*)^T (n (x) [U]) against grad l_i
        Ustar = np.where(wall[None], Uo, Up)
        G = ph.g_matrix(Ustar, p.mu, p.Pr, g)
        G = np.where(wall[..., None, None], ph.g_matrix(Ustar, p.mu, p.Pr_wall, g), G)
        nvec = np.concatenate([np.moveaxis(jump, 0, -1) * m.nx[:, None, :, None],
                               np.moveaxis(jump, 0, -1) * m.ny[:, None, :, None]], axis=-1)
        qv = np.einsum("...ji,...j->...i", G, nvec)
        ce = np.where(interior, 0.5, 1.0)[..., None]
        qv = p.theta * ce * qv
        qx = np.moveaxis(qv[..., 0:4], -1, 0)
        qy = np.moveaxis(qv[..., 4:8], -1, 0)
        qr = wg * Fscale * (rx * qx + ry * qy)
        qs = wg * Fscale * (sx * qx + sy * qy)
        tht = np.zeros_like(U)
        for f in range(3):
            tht += np.einsum("gi,cgk->cik", oi.Drf[f], qr[:, f]) + np.einsum("gi,cgk->cik", oi.Dsf[f], qs[:, f])
        tht = np.einsum("ij,cjk->cik", Minv, tht)
        out = vol + surf + tht
        if source is not None:
            out = out + source
        if return_parts:
            return out, dict(vol=vol, surf=surf, theta=tht, sigma=sigma, gbar=gbar)
        return out


def simplex_monomial_integral(a, b):
    """int over the reference triangle of r^a s^b, in closed form: with
    r = 2 x - 1, s = 2 y - 1 on the unit simplex (dr ds = 4 dx dy) and
    int x^i y^j = i! j! / (i + j + 2)!; summed in exact rational arithmetic
    (the alternating binomial sum cancels heavily at high degree)."""
    total = Fraction(0)
    for i in range(a + 1):
        for j in range(b + 1):
            c = math.comb(a, i) * math.comb(b, j) * 2 ** (i + j) * (-1) ** (a - i + b - j)
            total += Fraction(c * math.factorial(i) * math.factorial(j), math.factorial(i + j + 2))
    return float(4 * total)
