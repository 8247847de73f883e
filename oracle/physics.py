"""Pointwise physics of the 2D compressible Navier-Stokes system (oracle; test infrastructure).

State U = [rho, rho v1, rho v2, eps] with eps the total energy per unit
volume (Sec. 2.1, eq. cnp).  Readings of garbled passages:

* Equation of state: p = (gamma - 1)(eps - rho |v|^2 / 2).  The printed form
  is garbled; this is the only form consistent with the (4,1) entries of the
  viscous blocks G_ii printed beside it.
* Total enthalpy H = (eps + p) / rho (printed as eps + p/rho).
* Viscous flux: the paper writes F_v = G(U) grad U with four 4x4 blocks.  The
  oracle does not type those tables in; it evaluates the physical stress
  tau = mu (grad v + grad v^T - 2/3 div v I) and heat flux
  (mu gamma / Pr) grad e, e = eps/rho - |v|^2/2, from primitive gradients --
  algebraically the same operator -- and obtains G itself column by column
  from the linearity of F_v in grad U.
* Roe matrix: the flux Jacobian at the Roe-averaged state, found by complex-
  step differentiation of the flux, and |A| = R |Lambda| R^-1 from a numerical
  eigen-decomposition (no closed-form wave strengths).
"""
import numpy as np


def primitives(U, gamma):
    rho = U[0]
    u = U[1] / rho
    v = U[2] / rho
    p = (gamma - 1.0) * (U[3] - 0.5 * rho * (u * u + v * v))
    return rho, u, v, p


def conservative(rho, u, v, p, gamma):
    return np.stack([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


def advective_flux(U, gamma):
    """F_c,x and F_c,y (eq. cnp and the display below it)."""
    rho, u, v, p = primitives(U, gamma)
    E = U[3]
    fx = np.stack([rho * u, rho * u * u + p, rho * u * v, u * (E + p)])
    fy = np.stack([rho * v, rho * u * v, rho * v * v + p, v * (E + p)])
    return fx, fy


def normal_flux(U, nx, ny, vw, gamma):
    """N (F_c(U) - v_w (x) U): advective flux through a face of normal n, moving frame."""
    fx, fy = advective_flux(U, gamma)
    vwn = vw[0] * nx + vw[1] * ny
    return fx * nx + fy * ny - vwn * U


def viscous_flux(U, Ux, Uy, mu, Pr, gamma):
    """F_v = G(U) grad U via primitive gradients (see module docstring)."""
    rho = U[0]
    u = U[1] / rho
    v = U[2] / rho
    ux = (Ux[1] - u * Ux[0]) / rho
    uy = (Uy[1] - u * Uy[0]) / rho
    vx = (Ux[2] - v * Ux[0]) / rho
    vy = (Uy[2] - v * Uy[0]) / rho
    ex = (Ux[3] - U[3] / rho * Ux[0]) / rho - u * ux - v * vx
    ey = (Uy[3] - U[3] / rho * Uy[0]) / rho - u * uy - v * vy
    txx = mu * (4.0 / 3.0 * ux - 2.0 / 3.0 * vy)
    tyy = mu * (4.0 / 3.0 * vy - 2.0 / 3.0 * ux)
    txy = mu * (uy + vx)
    k = mu * gamma / Pr
    zero = np.zeros_like(rho)
    fx = np.stack([zero, txx, txy, u * txx + v * txy + k * ex])
    fy = np.stack([zero, txy, tyy, u * txy + v * tyy + k * ey])
    return fx, fy


def g_matrix(U, mu, Pr, gamma):
    """The 8x8 matrix G(U) with [F_v,x; F_v,y] = G [d_x U; d_y U], shape (..., 8, 8).

    Built column by column: F_v is linear in grad U for a fixed U.
    """
    U = np.asarray(U, dtype=np.float64)
    shape = U.shape[1:]
    G = np.zeros(shape + (8, 8))
    for c in range(8):
        gx = np.zeros_like(U)
        gy = np.zeros_like(U)
        if c < 4:
            gx[c] = 1.0
        else:
            gy[c - 4] = 1.0
        fx, fy = viscous_flux(U, gx, gy, mu, Pr, gamma)
        G[..., 0:4, c] = np.moveaxis(fx, 0, -1)
        G[..., 4:8, c] = np.moveaxis(fy, 0, -1)
    return G


def normal_diffusion_norm(U, nx, ny, mu, Pr, gamma):
    """|| N G(U) N^T ||_2 with N = n^T (x) I_4, the quantity maximised in G-bar_e (Sec. 2.2.3)."""
    G = g_matrix(U, mu, Pr, gamma)
    nx = np.asarray(nx)[..., None, None]
    ny = np.asarray(ny)[..., None, None]
    A = (nx * nx * G[..., 0:4, 0:4] + nx * ny * G[..., 0:4, 4:8]
         + ny * nx * G[..., 4:8, 0:4] + ny * ny * G[..., 4:8, 4:8])
    return np.linalg.norm(A, ord=2, axis=(-2, -1))


def roe_average(UL, UR, gamma):
    """Roe-averaged conservative state: sqrt(rho)-weighted velocity and enthalpy."""
    rl, ul, vl, pl = primitives(UL, gamma)
    rr, ur, vr, pr = primitives(UR, gamma)
    hl = (UL[3] + pl) / rl
    hr = (UR[3] + pr) / rr
    sl, sr = np.sqrt(rl), np.sqrt(rr)
    rho = sl * sr
    u = (sl * ul + sr * ur) / (sl + sr)
    v = (sl * vl + sr * vr) / (sl + sr)
    h = (sl * hl + sr * hr) / (sl + sr)
    # eps from rho h = eps + p and p = (gamma-1)(eps - rho|v|^2/2)
    eps = (rho * h + (gamma - 1.0) * 0.5 * rho * (u * u + v * v)) / gamma
    return np.stack([rho, rho * u, rho * v, eps])


def flux_jacobian(U, nx, ny, vw, gamma, h=1e-30):
    """d(normal_flux)/dU at U by complex-step differentiation, shape (..., 4, 4)."""
    U = np.asarray(U, dtype=np.float64)
    shape = U.shape[1:]
    A = np.zeros(shape + (4, 4))
    for c in range(4):
        Uc = U.astype(np.complex128)
        Uc[c] = Uc[c] + 1j * h
        fn = normal_flux(Uc, nx, ny, vw, gamma)
        A[..., :, c] = np.moveaxis(fn.imag / h, 0, -1)
    return A


def abs_matrix_apply(A, w):
    """|A| w for diagonalisable A with real spectrum, by the spectral (Sylvester) formula.

    |A| = sum_k |mu_k| prod_{j != k} (A - mu_j I) / (mu_k - mu_j) over the distinct
    eigenvalues mu_k (numerical eigenvalues; a pair closer than 1e-8 of the
    spectral scale is one eigenvalue).  This equals R |Lambda| R^-1 without forming
    eigenvectors, which LAPACK returns parallel for an exactly repeated eigenvalue.
    A: (..., n, n); w: (..., n).
    """
    lam = np.sort(np.linalg.eigvals(A).real, axis=-1)
    n = lam.shape[-1]
    scale = np.abs(lam).max(axis=-1) + 1.0
    gaps = np.diff(lam, axis=-1)
    worst = np.argmin(gaps, axis=-1)
    merged = np.take_along_axis(gaps, worst[..., None], -1)[..., 0] < 1e-8 * scale
    eye = np.eye(n)

    def lagrange(nodes):
        out = np.zeros(w.shape)
        m = nodes.shape[-1]
        for k in range(m):
            v = w.copy()
            coef = np.abs(nodes[..., k])
            for j in range(m):
                if j == k:
                    continue
                mj = nodes[..., j][..., None, None]
                v = np.einsum('...ij,...j->...i', A - mj * eye, v)
                coef = coef / (nodes[..., k] - nodes[..., j])
            out = out + coef[..., None] * v
        return out

    with np.errstate(divide='ignore', invalid='ignore'):
        full = lagrange(lam)
    keep = np.ones(lam.shape, dtype=bool)
    np.put_along_axis(keep, (worst + 1)[..., None], False, -1)
    reduced_nodes = lam[keep].reshape(lam.shape[:-1] + (n - 1,))
    with np.errstate(divide='ignore', invalid='ignore'):
        reduced = lagrange(reduced_nodes)
    return np.where(merged[..., None], reduced, full)


def roe_dissipation(UL, UR, nx, ny, vw, gamma):
    """|A~ - (v_w.n) I| (UL - UR), A~ the Roe matrix, by spectral calculus on its eigenvalues."""
    Ur = roe_average(UL, UR, gamma)
    A = flux_jacobian(Ur, nx, ny, vw, gamma)
    dU = np.moveaxis(UL - UR, 0, -1)
    return np.moveaxis(abs_matrix_apply(A, dU), -1, 0)


def roe_flux(UL, UR, nx, ny, vw, gamma):
    """Roe flux (eq. roe_flux), dissipative reading: mean normal flux + |A~|(U+ - U-)/2.

    UL is the own ("+") state, UR the neighbour ("-") state, n the own outward normal.
    """
    fl = normal_flux(UL, nx, ny, vw, gamma)
    fr = normal_flux(UR, nx, ny, vw, gamma)
    return 0.5 * (fl + fr) + 0.5 * roe_dissipation(UL, UR, nx, ny, vw, gamma)


def wall_state(Uin, vw, gamma):
    """Ghost state of the moving adiabatic wall: Q^b = [rho+, v_w, p+] (Sec. 2.2.4)."""
    rho, _, _, p = primitives(Uin, gamma)
    one = np.ones_like(rho)
    return conservative(rho, vw[0] * one, vw[1] * one, p, gamma)
