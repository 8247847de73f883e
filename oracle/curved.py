"""Isoparametric (curved) elements: geometry and weak-form right-hand side
(oracle; test infrastructure).

The paper's elements are images of the reference triangle under an affine
or isoparametric map T_K (Sec. 2.2); its experiments use affine maps and it
states that the scheme accepts curvilinear elements, citing the nodal DG
literature.  Here an element's map is the degree-p polynomial interpolant of
given node positions, x(r, s) = sum_j x_j l_j(r, s), and eq. dg_on_K is
applied to it:

  M^K dU/dt = int_K F . grad l_i  -  int_dK H_m l_i  +  int_dK H_theta . grad l_i

Readings (the paper gives no curved-element formulas):

* Metric terms at the nodes from the derivatives of the map's interpolant,
  x_r = D_r x, ...; J = x_r y_s - x_s y_r, r_x = y_s / J, r_y = -x_s / J,
  s_x = -y_r / J, s_y = x_r / J.  grad U at a node is r_x d_r U + s_x d_s U
  (exact for the polynomial U o T_K).
* Collocation of the fluxes, as the nodal scheme does on affine elements:
  the volume integral is int_K^ I(F~_r) d_r l_i + I(F~_s) d_s l_i with the
  contravariant fluxes F~_r = J (r_x F_x + r_y F_y), F~_s = J (s_x F_x +
  s_y F_y) interpolated from the nodes; the face integrals integrate the
  interpolants of sJ H_m and of sJ (r_x q_x + r_y q_y), sJ (s_x q_x + s_y q_y)
  (q = c_e theta G^T (n (x) [U])) over the reference face parameter, with
  the face mass matrix; n and sJ = |dx/dxi| at each face node from the map's
  tangent there.
* M^K = int_K^ l_i l_j J, exact (J has degree 2p - 2; the collapsed Gauss
  rule with 2p points per direction is exact to degree 4p - 1).
* The penalty's C_inv = (p+1)(p+2)|e|/(2|K|) takes the curved face length
  |e| = int |dx/dxi| dxi (32-point Gauss-Legendre: the integrand is the
  square root of a polynomial) and the curved area |K| = int_K^ J.

On an affine element all of this is the nodal oracle's arithmetic
(M^K = J M, F~ = J (r_x F_x + r_y F_y), sJ / J = Fscale).
"""
import numpy as np
from scipy.special import roots_jacobi

from . import physics as ph
from .dg import DGOracle
from .mesh import TAG_WALL
from .nodes import grad_jacobi_p, vandermonde_1d
from .overint import OverIntegration


FACE_LENGTH_POINTS = 32


def face_tangent(f, xr, xs, yr, ys):
    """d(x, y)/dxi on face f (face f joins vertices f and f+1, xi running
    counter-clockwise: face 0 r = xi, face 1 (r, s) = (-xi, xi), face 2
    s = -xi)."""
    if f == 0:
        return xr, yr
    if f == 1:
        return xs - xr, ys - yr
    return -xs, -ys


def _face_xi(ref, f):
    """The reference face parameter of face f's nodes (in Fmask order)."""
    r, s = ref.r[ref.Fmask[f]], ref.s[ref.Fmask[f]]
    return r if f == 0 else (s if f == 1 else -s)


class CurvedMesh:
    """An affine Mesh with the node positions of some elements replaced.

    The affine mesh supplies the connectivity (the replaced elements must keep
    their faces shared with other elements conforming: the same node positions
    on both sides) and the boundary tags; geometry is per node for every
    element.  elems: indices of the replaced elements; xy: (n, 2, Np) their
    node positions (library node order)."""

    def __init__(self, mesh, elems, xy):
        ref = mesh.ref
        self.base = mesh
        self.ref = ref
        self.K = mesh.K
        for name in ("period", "face_tag", "EToE", "EToF", "nbr_node", "nbr_elem", "nbr_face",
                     "is_boundary"):
            setattr(self, name, getattr(mesh, name))
        elems = np.asarray(elems, dtype=np.int64)
        xy = np.asarray(xy, dtype=np.float64).reshape(len(elems), 2, ref.Np)
        if len(set(elems.tolist())) != len(elems):
            raise ValueError("an element is listed twice")
        self.curved = np.zeros(self.K, dtype=bool)
        self.curved[elems] = True
        self.x = mesh.x.copy()
        self.y = mesh.y.copy()
        self.x[:, elems] = xy[:, 0, :].T
        self.y[:, elems] = xy[:, 1, :].T
        self._check_conforming()
        # metric terms at the nodes
        xr, xs = ref.Dr @ self.x, ref.Ds @ self.x
        yr, ys = ref.Dr @ self.y, ref.Ds @ self.y
        self.J = xr * ys - xs * yr
        if np.any(self.J <= 0.0):
            raise ValueError("an element's map has a non-positive Jacobian at a node")
        self.rx, self.ry = ys / self.J, -xs / self.J
        self.sx, self.sy = -yr / self.J, xr / self.J
        # normals and surface Jacobians at the face nodes
        Fm = ref.Fmask
        self.nx = np.zeros((3, ref.Nfp, self.K))
        self.ny = np.zeros((3, ref.Nfp, self.K))
        self.sJ = np.zeros((3, ref.Nfp, self.K))
        for f in range(3):
            tx, ty = face_tangent(f, xr[Fm[f]], xs[Fm[f]], yr[Fm[f]], ys[Fm[f]])
            L = np.hypot(tx, ty)
            self.nx[f], self.ny[f], self.sJ[f] = ty / L, -tx / L, L
        # mass matrices, areas and face lengths
        oi = OverIntegration(ref, pf=4 * ref.N - 2)
        xrq, xsq = oi.Drq @ self.x, oi.Dsq @ self.x
        yrq, ysq = oi.Drq @ self.y, oi.Dsq @ self.y
        Jq = xrq * ysq - xsq * yrq                                # (Nq, K)
        if np.any(Jq <= 0.0):
            raise ValueError("an element's map has a non-positive Jacobian inside")
        self.MK = np.einsum("q,qk,qi,qj->kij", oi.wq, Jq, oi.Iq, oi.Iq)
        self.area = np.einsum("q,qk->k", oi.wq, Jq)
        self.face_len = np.zeros((3, self.K))
        xg, wg = roots_jacobi(FACE_LENGTH_POINTS, 0.0, 0.0)
        for f in range(3):
            xi = _face_xi(ref, f)
            # derivative of the face interpolant at the Gauss points
            V = vandermonde_1d(ref.N, xi)
            dVg = np.stack([grad_jacobi_p(xg, 0.0, 0.0, j) for j in range(ref.N + 1)], axis=1)
            Dg = dVg @ np.linalg.inv(V)            # d/dxi of the face nodes' Lagrange basis
            tx = Dg @ self.x[Fm[f]]
            ty = Dg @ self.y[Fm[f]]
            self.face_len[f] = wg @ np.hypot(tx, ty)

    def _check_conforming(self, tol=1e-10):
        """Face nodes shared with a neighbour coincide on both sides."""
        ref = self.ref
        Fm = ref.Fmask
        scale = max(np.ptp(self.x), np.ptp(self.y), 1.0)
        for k in np.nonzero(self.curved)[0]:
            for f in range(3):
                kn = self.EToE[k, f]
                if kn < 0:
                    continue
                mine = Fm[f]
                theirs = self.nbr_node[f, :, k]
                dx = self.x[mine, k] - self.x[theirs, kn]
                dy = self.y[mine, k] - self.y[theirs, kn]
                if self.period[0] > 0 or self.period[1] > 0:
                    dx -= np.round(dx / self.period[0]) * self.period[0] if self.period[0] > 0 else 0.0
                    dy -= np.round(dy / self.period[1]) * self.period[1] if self.period[1] > 0 else 0.0
                if np.hypot(dx, dy).max() > tol * scale:
                    raise ValueError("face (%d,%d) of a curved element does not conform" % (k, f))


class DGOracleCurved(DGOracle):
    """The nodal oracle's physics on a CurvedMesh (per-node geometry)."""

    def gradient(self, U):
        m, ref = self.mesh, self.ref
        Ur = np.einsum('ij,fjk->fik', ref.Dr, U)
        Us = np.einsum('ij,fjk->fik', ref.Ds, U)
        return m.rx * Ur + m.sx * Us, m.ry * Ur + m.sy * Us

    def gbar(self, fs):
        m, p = self.mesh, self.phys
        a = ph.normal_diffusion_norm(fs['Up'], m.nx, m.ny, p.mu, p.Pr, p.gamma)
        b = ph.normal_diffusion_norm(fs['Uo'], m.nx, m.ny, p.mu, p.Pr, p.gamma)
        return np.maximum(a.max(axis=1), b.max(axis=1))

    def rhs(self, U, vw=(0.0, 0.0), source=None, return_parts=False):
        if source is not None:
            raise ValueError("no source term on curved meshes")
        m, p, ref = self.mesh, self.phys, self.ref
        vw = np.asarray(vw, dtype=np.float64)
        g = p.gamma
        Np, Nfp, K = ref.Np, ref.Nfp, m.K
        Fm = ref.Fmask
        Ux, Uy = self.gradient(U)
        Fx, Fy = self.total_flux(U, Ux, Uy, vw)
        # volume: int_K^ I(F~_r) d_r l_i + I(F~_s) d_s l_i = D_r^T M F~_r + D_s^T M F~_s
        Fr = m.J * (m.rx * Fx + m.ry * Fy)
        Fs = m.J * (m.sx * Fx + m.sy * Fy)
        DrTM, DsTM = ref.Dr.T @ ref.M, ref.Ds.T @ ref.M
        vol = np.einsum('ij,fjk->fik', DrTM, Fr) + np.einsum('ij,fjk->fik', DsTM, Fs)

        fs = self.face_states(U, Ux, Uy, vw)
        nx, ny = m.nx, m.ny                                          # (3, Nfp, K)
        Up, Uo = fs['Up'], fs['Uo']
        wall, far = fs['wall'], fs['far']
        interior = ~(wall | far)
        Fc = ph.roe_flux(Up, Uo, nx, ny, vw, g)
        Fc = np.where(wall[None], ph.normal_flux(Uo, nx, ny, vw, g), Fc)
        vxp, vyp = ph.viscous_flux(Up, fs['Uxp'], fs['Uyp'], p.mu, p.Pr, g)
        vxm, vym = ph.viscous_flux(Uo, fs['Uxm'], fs['Uym'], p.mu, p.Pr, g)
        vxw, vyw = ph.viscous_flux(Uo, fs['Uxp'], fs['Uyp'], p.mu, p.Pr_wall, g)
        vn_int = 0.5 * ((vxp + vxm) * nx + (vyp + vym) * ny)
        vn = np.where(interior[None], vn_int,
                      np.where(wall[None], vxw * nx + vyw * ny, vxp * nx + vyp * ny))
        gbar = self.gbar(fs)
        sigma = self.penalty(gbar)
        jump = Up - Uo
        Hm = Fc - vn + sigma[None, :, None, :] * jump
        sJ = m.sJ[None]
        surf = -np.einsum('ij,fjk->fik', ref.E, (sJ * Hm).reshape(4, 3 * Nfp, K))
        # theta term
        Ustar = np.where(wall[None], Uo, Up)
        G = ph.g_matrix(Ustar, p.mu, p.Pr, g)
        G = np.where(wall[..., None, None], ph.g_matrix(Ustar, p.mu, p.Pr_wall, g), G)
        nvec = np.concatenate([np.moveaxis(jump, 0, -1) * nx[..., None],
                               np.moveaxis(jump, 0, -1) * ny[..., None]], axis=-1)
        q = np.einsum('...ji,...j->...i', G, nvec)
        ce = np.where(interior, 0.5, 1.0)[..., None]
        q = p.theta * ce * q
        qx = np.moveaxis(q[..., 0:4], -1, 0)
        qy = np.moveaxis(q[..., 4:8], -1, 0)
        rxf, ryf = m.rx[Fm][None], m.ry[Fm][None]
        sxf, syf = m.sx[Fm][None], m.sy[Fm][None]
        qr = sJ * (rxf * qx + ryf * qy)
        qs = sJ * (sxf * qx + syf * qy)
        DrTE, DsTE = ref.Dr.T @ ref.E, ref.Ds.T @ ref.E
        tht = (np.einsum('ij,fjk->fik', DrTE, qr.reshape(4, 3 * Nfp, K))
               + np.einsum('ij,fjk->fik', DsTE, qs.reshape(4, 3 * Nfp, K)))

        def solve(b):
            # (M^K)^-1 per element
            return np.einsum('kij,fjk->fik', np.linalg.inv(m.MK), b)

        out = solve(vol + surf + tht)
        if return_parts:
            parts = dict(vol=solve(vol), surf=solve(surf), theta=solve(tht), sigma=sigma, gbar=gbar)
            return out, parts
        return out

    def integral(self, A):
        """int_Omega A dx per field: sum_K 1^T M^K A_K."""
        return np.einsum('kij,fjk->f', self.mesh.MK, A)


def wall_force(dg, U, vw=(0.0, 0.0), centre=(0.0, 0.0)):
    """(Fx, Fy, Mz) on the body: the face-quadrature traction with the normal
    and sJ of each wall face node (oracle.fsi.wall_force with per-node
    face geometry)."""
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
        nx, ny = m.nx[f, :, k], m.ny[f, :, k]
        tx = pres * nx - (vx[1] * nx + vy[1] * ny)
        ty = pres * ny - (vx[2] * nx + vy[2] * ny)
        w = ref.wface[f] * m.sJ[f, :, k]
        xs = m.x[nodes, k] - centre[0]
        ys = m.y[nodes, k] - centre[1]
        Fx += float(np.dot(w, tx))
        Fy += float(np.dot(w, ty))
        Mz += float(np.dot(w, xs * ty - ys * tx))
    return np.array([Fx, Fy, Mz])
