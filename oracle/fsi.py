"""Body force and rigid-body Newmark step (oracle; test infrastructure).

* Force (Alg. 3, "Calculate Aerodynamic Forces"): the paper gives no formula.
  Reading: the traction the fluid exerts on the body, integrated over the wall
  faces with the face mass quadrature, F = sum_e int_e (p+ n - tau n) ds, with n
  the fluid element's outward normal (pointing into the body) and tau the
  viscous stress of the wall flux, i.e. the momentum rows of G(U^b) grad U+.
  Mz is the moment of that traction about the origin (the body centre).
* Rigid body (eq. 1dof_oscillator): Newmark with beta_N = 1/4, gamma_N = 1/2;
  coefficients M_r = 1, C_r = 4 pi f_n xi, K_r = (1 + 1/m*)(2 pi f_n)^2,
  F_r = Lift / m (Sec. 3.3.1).
"""
import math

import numpy as np

from . import physics as ph
from .mesh import TAG_WALL


def wall_force(dg, U, vw=(0.0, 0.0), centre=(0.0, 0.0)):
    """(Fx, Fy, Mz) on the body: sum over wall faces of the face-quadrature traction."""
    m, ref, p = dg.mesh, dg.ref, dg.phys
    vw = np.asarray(vw, dtype=np.float64)
    Ux, Uy = dg.gradient(U)
    Fx = Fy = Mz = 0.0
    for k, f in zip(*np.where(m.face_tag == TAG_WALL)):
        nodes = ref.Fmask[f]
        Up = U[:, nodes, k]
        Ub = ph.wall_state(Up, vw, p.gamma)
        _, _, _, pres = ph.primitives(Up, p.gamma)
        vx, vy = ph.viscous_flux(Ub, Ux[:, nodes, k], Uy[:, nodes, k], p.mu, p.Pr, p.gamma)
        nx, ny = m.nx[f, k], m.ny[f, k]
        tx = pres * nx - (vx[1] * nx + vy[1] * ny)
        ty = pres * ny - (vx[2] * nx + vy[2] * ny)
        w = ref.wface[f] * m.sJ[f, k]
        xs = m.x[nodes, k] - centre[0]
        ys = m.y[nodes, k] - centre[1]
        Fx += float(np.dot(w, tx))
        Fy += float(np.dot(w, ty))
        Mz += float(np.dot(w, xs * ty - ys * tx))
    return np.array([Fx, Fy, Mz])


def viv_coefficients(U_star, m_star, xi, v_inf, D=1.0, rho=1.0):
    """(M_r, C_r, K_r, 1/m) of the 1-DOF oscillator for reduced velocity U* = v_inf/(f_n D)."""
    f_n = v_inf / (U_star * D)
    m = m_star * rho * math.pi * D * D / 4.0
    return 1.0, 4.0 * math.pi * f_n * xi, (1.0 + 1.0 / m_star) * (2.0 * math.pi * f_n) ** 2, 1.0 / m


def newmark_step(y, yd, ydd, F_new, dt, M, C, K, beta=0.25, gam=0.5):
    """One Newmark-beta step of M y'' + C y' + K y = F; returns (y, y', y'') at t + dt."""
    lhs = M + gam * dt * C + beta * dt * dt * K
    rhs = (F_new - C * (yd + (1.0 - gam) * dt * ydd)
           - K * (y + dt * yd + (0.5 - beta) * dt * dt * ydd))
    ydd_n = rhs / lhs
    yd_n = yd + dt * ((1.0 - gam) * ydd + gam * ydd_n)
    y_n = y + dt * yd + 0.5 * dt * dt * ((1.0 - 2.0 * beta) * ydd + 2.0 * beta * ydd_n)
    return y_n, yd_n, ydd_n
