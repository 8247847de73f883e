"""A sweep of elastically mounted cylinders advanced as one batch.

Each instance is a cylinder free to move transversely, a 1-DOF oscillator
M_r y'' + C_r y' + K_r y = F_r (eq. 1dof_oscillator) with M_r = 1,
C_r = 4 pi f_n xi, K_r = (1 + 1/m*) (2 pi f_n)^2, F_r = lift / m,
m = m* rho_inf pi D^2 / 4 and f_n = |v_inf| / (U* D) from the reduced velocity
U* (Sec. 3.3.1).  The coupling is the weak one of Alg. 3, per step: the
Newmark step (beta 1/4, gamma 1/2, host FP64) under the last force gives the
displacement increment dy, the wall velocity for the step is v_w = (0, dy/dt),
all instances take one RK step with their own dt and v_w (one launch per
stage for the whole batch), then the forces are evaluated on the new states.
"""
import math

import numpy as np

from . import _lib as L
from .solver import Batch, Solver


def oscillator(U_star, m_star, xi, v_inf, rho_inf=1.0, D=1.0):
    """(M_r, C_r, K_r, 1/m) for reduced velocity U*, mass ratio m*, damping xi."""
    f_n = v_inf / (U_star * D)
    m = m_star * rho_inf * math.pi * D * D / 4.0
    return 1.0, 4.0 * math.pi * f_n * xi, (1.0 + 1.0 / m_star) * (2.0 * math.pi * f_n) ** 2, 1.0 / m


class VIVSweep:
    """cases: list of dicts with keys mesh, p, U_star, m_star, xi (and
    optionally D).  Physics is shared; precision is a dg_precision mode."""

    def __init__(self, cases, gamma, Pr, mu, theta, penalty_mode, C_pen, U_inf,
                 precision=L.DG_FP64):
        U_inf = np.asarray(U_inf, dtype=np.float64)
        self.n = len(cases)
        self.solvers = [Solver(c["p"], c["mesh"], gamma=gamma, Pr=Pr, mu=mu, theta=theta,
                               penalty_mode=penalty_mode, C_pen=C_pen, U_inf=U_inf,
                               precision=precision) for c in cases]
        self.batch = Batch(self.solvers)
        v_inf = float(np.hypot(U_inf[1], U_inf[2]) / U_inf[0])
        self.coef = [oscillator(c["U_star"], c["m_star"], c["xi"], v_inf, U_inf[0], c.get("D", 1.0))
                     for c in cases]
        self.osc = np.array(self.coef, dtype=np.float64)  # M, C, K, 1/m per instance
        self.body = np.zeros((self.n, 3))   # y, y', y'' per instance
        self.vw = np.zeros((self.n, 2))
        self.F = np.zeros((self.n, 3))      # Fx, Fy, Mz on the current states
        self.t = 0.0

    def set_state(self, i, U, stream=None):
        self.batch.set_state(i, U, stream)

    def get_state(self, i, out=None, stream=None):
        return self.batch.get_state(i, out, stream)

    def update_forces(self, stream=None):
        self.F = np.ascontiguousarray(self.batch.force(self.vw, stream))
        return self.F

    def step(self, dt, stream=None):
        """Newmark under the last forces, one RK step of every instance with
        the resulting wall velocities, forces on the new states -- one library
        call for the whole batch."""
        dts = np.broadcast_to(np.asarray(dt, dtype=np.float64), (self.n,)).copy()
        self.vw = self.batch.coupled_step(self.osc, self.body, self.F, dts, stream)
        self.t += float(dts.max())
        return self.F

    def close(self):
        self.batch.close()
        for s in self.solvers:
            s.close()
