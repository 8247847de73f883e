"""Weak-form nodal IP-DG right-hand side and low-storage RK (oracle; test infrastructure).

Follows the semi-discrete weak form (eq. weak_form) element by element
(eq. dg_on_K): with Phi = l_i e_k on the own element K = K+ (the paper's
"+" side; "-" is the neighbour),

  M^K dU/dt = int_K F . grad l_i  -  int_dK H_m l_i  +  int_dK H_theta . grad l_i

where F = F_c - v_w (x) U - G grad U, and on each face (own outward normal n)

  H_m     = F^_c(U+, U-) - {G grad U} . n + sigma_e (U+ - U-)
  H_theta = c_e theta G(U*)^T (n (x) (U+ - U-)).

Readings (paper silent or garbled at these points):

* Roe upwinding enters with + 1/2 |A~| (U+ - U-), the dissipative sign.
* The theta term carries the average's 1/2 on interior faces (c_e = 1/2) and 1
  on boundary faces, with G taken at the own trace U+ (wall: at the ghost U^b),
  following Table "jump and average" and eq. ip_flux.
* Viscous average {G grad U} = (G(U+) grad U+ + G(U-) grad U-) / 2; on the far
  field G(U+) grad U+, on the wall G(U^b) grad U+ (the printed wall flux)
  without its heat conduction, and the wall's theta term with G(U^b) likewise
  without conduction: the wall is adiabatic (Neumann conditions on pressure
  and temperature, Sec. 2.2.4), and the printed G(U^b) grad U+ would carry
  the interior's conductive flux through it.  The printed form, with
  conduction, is kept as an option (Physics.wall_heat_flux).
* grad U is the broken element gradient (no lifting operator).
* G-bar_e = max over the face nodes of both sides (boundary: own trace and
  ghost) of ||N G N^T||_2; recomputed from the current state at every call.
* Penalty "paper" (eq. penalty_final): sigma_e = C1 (1+theta)^2 (d+1) G-bar_e
  max_{+-} C_inv(e, K+-, p), C_inv = (p+1)(p+2)|e| / (2|K|); boundary faces use
  the own element only.  Penalty "standard": sigma_e = C (p+1)^2 G-bar_e /
  min_{+-} h_e, h_e = 2|K|/|e| (a diffusivity is needed for the units).
* Far field: U^b = U_inf, Roe flux and IP terms with that ghost.
"""
import numpy as np

from . import physics as ph
from .mesh import TAG_WALL, TAG_FAR

PENALTY_PAPER, PENALTY_STANDARD = 0, 1

# Carpenter & Kennedy (1994) five-stage fourth-order 2N-storage coefficients
# (NASA TM-109112, solution 3): K1 <- A_i K1 + dt R(K0), K0 <- K0 + B_i K1.
LSERK_A = (0.0,
           -567301805773.0 / 1357537059087.0,
           -2404267990393.0 / 2016746695238.0,
           -3550918686646.0 / 2091501179385.0,
           -1275806237668.0 / 842570457699.0)
LSERK_B = (1432997174477.0 / 9575080441755.0,
           5161836677717.0 / 13612068292357.0,
           1720146321549.0 / 2090206949498.0,
           3134564353537.0 / 4481467310338.0,
           2277821191437.0 / 14882151754819.0)
LSERK_C = (0.0,
           1432997174477.0 / 9575080441755.0,
           2526269341429.0 / 6820363962896.0,
           2006345519317.0 / 3224310063776.0,
           2802321613138.0 / 2924317926251.0)


class Physics:
    """wall_heat_flux: False (default) the adiabatic wall reading -- the wall's
    viscous flux and theta term without heat conduction; True the printed
    wall flux G(U^b) grad U+ with the interior's conduction, and G(U^b) in
    the theta term."""

    def __init__(self, gamma=1.4, Pr=0.72, mu=1e-3, theta=1.0, penalty_mode=PENALTY_PAPER,
                 C_pen=0.01, U_inf=(1.0, 0.2, 0.0, 1.0 / (1.4 * 0.4) + 0.02),
                 wall_heat_flux=False):
        self.gamma = float(gamma)
        self.Pr = float(Pr)
        self.mu = float(mu)
        self.theta = float(theta)
        self.penalty_mode = int(penalty_mode)
        self.C_pen = float(C_pen)
        self.U_inf = np.asarray(U_inf, dtype=np.float64)
        self.wall_heat_flux = bool(wall_heat_flux)

    @property
    def Pr_wall(self):
        """The Prandtl number the wall faces' viscous terms use (infinite: no
        conduction)."""
        return self.Pr if self.wall_heat_flux else np.inf


class DGOracle:
    def __init__(self, mesh, phys):
        self.mesh = mesh
        self.ref = mesh.ref
        self.phys = phys

    # -- helpers ---------------------------------------------------------
    def gradient(self, U):
        """Broken gradient: d_x = r_x D_r + s_x D_s, d_y = r_y D_r + s_y D_s (affine maps)."""
        m, ref = self.mesh, self.ref
        Ur = np.einsum('ij,fjk->fik', ref.Dr, U)
        Us = np.einsum('ij,fjk->fik', ref.Ds, U)
        return m.rx * Ur + m.sx * Us, m.ry * Ur + m.sy * Us

    def traces(self, A):
        """Own and neighbour traces of a nodal field (C, Np, K) -> 2 x (C, 3, Nfp, K)."""
        m = self.mesh
        own = A[:, self.ref.Fmask, :]
        nbr = A[:, m.nbr_node, m.nbr_elem]
        return own, nbr

    def total_flux(self, U, Ux, Uy, vw):
        p = self.phys
        fx, fy = ph.advective_flux(U, p.gamma)
        vx, vy = ph.viscous_flux(U, Ux, Uy, p.mu, p.Pr, p.gamma)
        return fx - vw[0] * U - vx, fy - vw[1] * U - vy

    def face_states(self, U, Ux, Uy, vw):
        """Own/other traces with boundary ghosts; returns dict of (4,3,Nfp,K) arrays."""
        m, p = self.mesh, self.phys
        Up, Um = self.traces(U)
        Uxp, Uxm = self.traces(Ux)
        Uyp, Uym = self.traces(Uy)
        tag = m.face_tag.T[None, :, None, :] * np.ones((1, 1, self.ref.Nfp, 1), dtype=np.int64)
        wall = (tag == TAG_WALL)
        far = (tag == TAG_FAR)
        Ub_wall = ph.wall_state(Up, vw, p.gamma)
        Ub_far = np.broadcast_to(p.U_inf[:, None, None, None], Up.shape)
        Uo = np.where(wall, Ub_wall, np.where(far, Ub_far, Um))
        return dict(Up=Up, Uo=Uo, Uxp=Uxp, Uyp=Uyp, Uxm=Uxm, Uym=Uym, wall=wall[0], far=far[0])

    def gbar(self, fs):
        """G-bar_e per face (3, K): max of ||N G N^T||_2 over face nodes and both sides."""
        m, p = self.mesh, self.phys
        nx = m.nx[:, None, :]
        ny = m.ny[:, None, :]
        a = ph.normal_diffusion_norm(fs['Up'], nx, ny, p.mu, p.Pr, p.gamma)
        b = ph.normal_diffusion_norm(fs['Uo'], nx, ny, p.mu, p.Pr, p.gamma)
        return np.maximum(a.max(axis=1), b.max(axis=1))

    def cinv(self):
        """C_inv(e, K, p) = (p+1)(p+d)|e| / (d|K|), d = 2, per own face (3, K)
        (eq. trace_inverse_estimate)."""
        m, N = self.mesh, self.ref.N
        d = 2
        return (N + 1) * (N + d) * m.face_len / (d * m.area[None, :])

    def penalty(self, gbar):
        """sigma_e per face (3, K) (eq. penalty_final or the literature form)."""
        m, p, ref = self.mesh, self.phys, self.ref
        N = ref.N
        cinv_own = self.cinv()
        kn = np.where(m.EToE >= 0, m.EToE, np.arange(m.K)[:, None]).T      # (3, K)
        fn = np.where(m.EToE >= 0, m.EToF, np.arange(3)[None, :]).T
        cinv_nbr = cinv_own[fn, kn]
        cinv = np.maximum(cinv_own, cinv_nbr)
        if p.penalty_mode == PENALTY_PAPER:
            d = 2
            return p.C_pen * (1.0 + p.theta) ** 2 * (d + 1) * gbar * cinv
        h_own = 2.0 * m.area[None, :] / m.face_len
        h_min = np.minimum(h_own, h_own[fn, kn])
        return p.C_pen * (N + 1) ** 2 * gbar / h_min

    # -- the right-hand side ----------------------------------------------
    def rhs(self, U, vw=(0.0, 0.0), source=None, return_parts=False):
        """dU/dt = (M^K)^-1 R (eq. dg_on_K), weak form; U has shape (4, Np, K)."""
        m, p, ref = self.mesh, self.phys, self.ref
        vw = np.asarray(vw, dtype=np.float64)
        g = p.gamma
        Ux, Uy = self.gradient(U)
        Fx, Fy = self.total_flux(U, Ux, Uy, vw)
        # volume: (1/J) M^-1 int_K F . grad l_i = Drw (rx Fx + ry Fy) + Dsw (sx Fx + sy Fy)
        Fr = m.rx * Fx + m.ry * Fy
        Fs = m.sx * Fx + m.sy * Fy
        vol = np.einsum('ij,fjk->fik', ref.Drw, Fr) + np.einsum('ij,fjk->fik', ref.Dsw, Fs)

        fs = self.face_states(U, Ux, Uy, vw)
        nx = m.nx[:, None, :]
        ny = m.ny[:, None, :]
        Up, Uo = fs['Up'], fs['Uo']
        wall, far = fs['wall'], fs['far']
        interior = ~(wall | far)
        # advective numerical flux
        Fc = ph.roe_flux(Up, Uo, nx, ny, vw, g)
        Fc_wall = ph.normal_flux(Uo, nx, ny, vw, g)
        Fc = np.where(wall[None], Fc_wall, Fc)
        # viscous normal flux (average of products inside, one-sided on the boundary)
        vxp, vyp = ph.viscous_flux(Up, fs['Uxp'], fs['Uyp'], p.mu, p.Pr, g)
        vxm, vym = ph.viscous_flux(Uo, fs['Uxm'], fs['Uym'], p.mu, p.Pr, g)
        # adiabatic wall: the stress and its work, no heat conduction (Pr -> inf);
        # or the printed G(U^b) grad U+ with conduction
        vxw, vyw = ph.viscous_flux(Uo, fs['Uxp'], fs['Uyp'], p.mu, p.Pr_wall, g)
        vn_int = 0.5 * ((vxp + vxm) * nx + (vyp + vym) * ny)
        vn_far = vxp * nx + vyp * ny
        vn_wall = vxw * nx + vyw * ny
        vn = np.where(interior[None], vn_int, np.where(wall[None], vn_wall, vn_far))
        # penalty
        gbar = self.gbar(fs)
        sigma = self.penalty(gbar)
        jump = Up - Uo
        Hm = Fc - vn + sigma[None, :, None, :] * jump
        Fscale = m.Fscale[None, :, None, :]
        Np, Nfp, K = ref.Np, ref.Nfp, m.K
        surf = -np.einsum('ij,fjk->fik', ref.LIFT, (Fscale * Hm).reshape(4, 3 * Nfp, K))
        # theta term: c_e theta G(U*)^T (n (x) [U]), lifted with M^-1 D^T E
        Ustar = np.where(wall[None], Uo, Up)
        G = ph.g_matrix(Ustar, p.mu, p.Pr, g)                      # (3, Nfp, K, 8, 8)
        G = np.where(wall[..., None, None], ph.g_matrix(Ustar, p.mu, p.Pr_wall, g), G)
        nvec = np.concatenate([np.moveaxis(jump, 0, -1) * m.nx[:, None, :, None],
                               np.moveaxis(jump, 0, -1) * m.ny[:, None, :, None]], axis=-1)
        q = np.einsum('...ji,...j->...i', G, nvec)                 # G^T (n (x) [U])
        ce = np.where(interior, 0.5, 1.0)[..., None]
        q = p.theta * ce * q
        qx = np.moveaxis(q[..., 0:4], -1, 0)
        qy = np.moveaxis(q[..., 4:8], -1, 0)
        qr = Fscale * (m.rx[None, None, None, :] * qx + m.ry[None, None, None, :] * qy)
        qs = Fscale * (m.sx[None, None, None, :] * qx + m.sy[None, None, None, :] * qy)
        tht = (np.einsum('ij,fjk->fik', ref.LIFTr, qr.reshape(4, 3 * Nfp, K))
               + np.einsum('ij,fjk->fik', ref.LIFTs, qs.reshape(4, 3 * Nfp, K)))
        out = vol + surf + tht
        if source is not None:
            out = out + source
        if return_parts:
            def lift(h):
                return -np.einsum('ij,fjk->fik', ref.LIFT, (Fscale * h).reshape(4, 3 * Nfp, K))
            parts = dict(vol=vol, surf=surf, theta=tht, sigma=sigma, gbar=gbar,
                         surf_adv=lift(Fc), surf_visc=lift(-vn),
                         surf_pen=lift(sigma[None, :, None, :] * jump),
                         Hm=Hm, qx=qx, qy=qy, Fx=Fx, Fy=Fy)
            return out, parts
        return out

    def lserk_step(self, U, dt, vw=(0.0, 0.0), source=None, K1=None):
        """One five-stage low-storage RK step (Alg. 1 with the stage loop written out)."""
        K0 = U.copy()
        K1 = np.zeros_like(U) if K1 is None else K1.copy()
        for a, b in zip(LSERK_A, LSERK_B):
            K1 = a * K1 + dt * self.rhs(K0, vw, source)
            K0 = K0 + b * K1
        return K0, K1

    # -- diagnostics -------------------------------------------------------
    def integral(self, A):
        """int_Omega A dx per field: sum_K J 1^T M A_K."""
        w = self.ref.M.sum(axis=0)
        return np.einsum('j,fjk,k->f', w, A, self.mesh.J)

    def l2_norm(self, A):
        """sqrt(sum_K J A_K^T M A_K) per field."""
        MA = np.einsum('ij,fjk->fik', self.ref.M, A)
        return np.sqrt(np.einsum('fik,fik,k->f', A, MA, self.mesh.J))
