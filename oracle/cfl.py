"""Time step from the CFL condition (oracle; test infrastructure).

Eq. cfl_general fixes delta t = C_CFL / Lambda, with Lambda the bound of
eq. rayleigh_bound (Appendix "On the CFL condition") on the numerical range
of the DG operator:

  Lambda = max_K ( 3/2 C_inv,2(K) G_K + (d + 1) C_inv,K (3 sigma_K + beta_K) + beta'_K ),  d = 2,

with
  C_inv,K     = max over the faces e of K of C_inv(e, K, p) = (p+1)(p+2)|e| / (2|K|)
                (the trace inverse constant of Sec. 2.2.3),
  C_inv,2(K)  = C_grad p^4 / rho_K^2, rho_K the radius of the inscribed circle
                (the classical inverse estimate; C_grad the generic constant),
  sigma_K     = max over the faces of K of the penalty sigma_e the RHS uses,
  beta_K      = max over the nodes of K of |v - v_w| + sqrt(gamma p / rho)
                (the vector b_ns of eq. cfl_general),
  beta'_K     = 1/2 max over the nodes of K of |div (v - v_w)|,
  G_K         = max over K and its face neighbours of the node maximum of ||G||.

Readings (the appendix leaves these open):
* ||G|| at a node is max(||e_x^T G e_x||_2, ||e_y^T G e_y||_2), the
  directional norm of Sec. 2.2.3 in the two coordinate directions (within a
  constant of the operator norm; the constant is absorbed in C_grad).
* div v is the divergence of the nodal interpolant of v = (rho v) / rho,
  differentiated with the element's nodal derivative matrices (v_w is uniform
  and drops out).
* sigma_e is recomputed from the state at hand exactly as the right-hand side
  does (G-bar_e over both sides of the face, boundary ghosts included).
"""
import numpy as np

from . import physics as ph
from .dg import DGOracle


def inradius(mesh):
    """rho_K = 2 |K| / perimeter(K) per element."""
    return 2.0 * mesh.area / mesh.face_len.sum(axis=0)


def trace_inverse_max(mesh):
    """C_inv,K = max_e (p+1)(p+2)|e| / (2|K|) per element."""
    N = mesh.ref.N
    return ((N + 1) * (N + 2) * mesh.face_len / (2.0 * mesh.area[None, :])).max(axis=0)


class CFLOracle(DGOracle):
    def parts(self, U, vw=(0.0, 0.0), C_grad=1.0):
        """Per-element pieces of Lambda: dict of (K,) arrays."""
        m, p, ref = self.mesh, self.phys, self.ref
        g = p.gamma
        vw = np.asarray(vw, dtype=np.float64)
        rho, u, v, pr = ph.primitives(U, g)
        beta = np.hypot(u - vw[0], v - vw[1]) + np.sqrt(g * pr / rho)
        beta_K = beta.max(axis=0)
        ux = m.rx * (ref.Dr @ u) + m.sx * (ref.Ds @ u)
        vy = m.ry * (ref.Dr @ v) + m.sy * (ref.Ds @ v)
        beta1_K = 0.5 * np.abs(ux + vy).max(axis=0)
        gx = ph.normal_diffusion_norm(U, 1.0, 0.0, p.mu, p.Pr, g)
        gy = ph.normal_diffusion_norm(U, 0.0, 1.0, p.mu, p.Pr, g)
        g_loc = np.maximum(gx, gy).max(axis=0)
        nbr = np.where(m.EToE >= 0, m.EToE, np.arange(m.K)[:, None])
        G_K = np.maximum(g_loc, g_loc[nbr].max(axis=1))
        Ux, Uy = self.gradient(U)
        sigma = self.penalty(self.gbar(self.face_states(U, Ux, Uy, vw)))
        sigma_K = sigma.max(axis=0)
        N = ref.N
        cinv2 = C_grad * N ** 4 / inradius(m) ** 2
        cinv = trace_inverse_max(m)
        lam = 1.5 * cinv2 * G_K + 3.0 * cinv * (3.0 * sigma_K + beta_K) + beta1_K
        return dict(beta=beta_K, beta1=beta1_K, G=G_K, sigma=sigma_K, cinv=cinv, cinv2=cinv2,
                    Lambda=lam)

    def time_step(self, U, vw=(0.0, 0.0), C_cfl=1.0, C_grad=1.0):
        """(Lambda, C_CFL / Lambda)."""
        lam = float(self.parts(U, vw, C_grad)["Lambda"].max())
        return lam, C_cfl / lam
