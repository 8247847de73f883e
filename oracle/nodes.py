"""Reference-element machinery of the nodal DG basis (oracle; test infrastructure).

The paper builds its nodal basis on the reference triangle
K^ = {(-1,-1), (1,-1), (-1,1)} (Sec. 2.2) from Warburton's warp-and-blend
interpolation nodes and the Dubiner/Proriol/Koornwinder (PKD) orthonormal
basis (Sec. 1; Sec. 2.2, "Weak matrices and nodal formulation"); all local
matrices are formed once on K^ because the element maps are affine.  This
module writes those constructions out directly:

* orthonormal Jacobi polynomials by their three-term recurrence,
* Legendre-Gauss-Lobatto points as the roots of P'_N (library root finder),
* Warburton's warp & blend node construction (J. Eng. Math. 56, 2006),
* the PKD basis in collapsed coordinates and its exact r/s derivatives,
* V, Vr, Vs, Dr = Vr V^-1, Ds, M = (V V^T)^-1, the face mass matrix E,
  LIFT = M^-1 E and the theta-term lifts M^-1 Dr^T E, M^-1 Ds^T E.

Node order: nodes are numbered row by row from the bottom edge s = -1 up to
the top vertex; inside a row, by increasing r.  Faces are numbered
0: s = -1 (vertex 0 -> 1), 1: r + s = 0 (vertex 1 -> 2), 2: r = -1
(vertex 2 -> 0), and the nodes of every face are listed in that
counter-clockwise direction.
"""
import math

import numpy as np
from scipy.special import roots_jacobi, gammaln

# Warburton's optimised blending exponents alpha_opt(N), N = 1..15, from
# Table 1 of "An explicit construction of interpolation nodes on the simplex"
# (T. Warburton, J. Eng. Math. 56 (2006)).  Larger N use 5/3.
ALPHA_OPT = (0.0, 0.0, 1.4152, 0.1001, 0.2751, 0.9800, 1.0999, 1.2832,
             1.3648, 1.4773, 1.4959, 1.5743, 1.5770, 1.6223, 1.6258)


def alpha_opt(N):
    return ALPHA_OPT[N - 1] if 1 <= N <= len(ALPHA_OPT) else 5.0 / 3.0


def jacobi_p(x, alpha, beta, n):
    """Orthonormal Jacobi polynomial P_n^(alpha,beta)(x) on [-1, 1].

    Normalised so that int (1-x)^alpha (1+x)^beta P_m P_n dx = delta_mn and
    evaluated with the three-term recurrence of the orthonormal family
    x P_k = a_{k+1} P_{k+1} + b_k P_k + a_k P_{k-1}.
    """
    x = np.asarray(x, dtype=np.float64)
    a, b = float(alpha), float(beta)
    log_g0 = ((a + b + 1.0) * math.log(2.0) + gammaln(a + 1.0) + gammaln(b + 1.0)
              - gammaln(a + b + 2.0))
    p_prev = np.full(x.shape, math.exp(-0.5 * log_g0))
    if n == 0:
        return p_prev
    p_cur = (((a + b + 2.0) * x + (a - b)) / 2.0) * p_prev \
        / math.sqrt((a + 1.0) * (b + 1.0) / (a + b + 3.0))
    if n == 1:
        return p_cur
    a_k = 2.0 / (a + b + 2.0) * math.sqrt((a + 1.0) * (b + 1.0) / (a + b + 3.0))
    for k in range(1, n):
        h = 2.0 * k + a + b
        a_next = 2.0 / (h + 2.0) * math.sqrt((k + 1.0) * (k + 1.0 + a + b) * (k + 1.0 + a)
                                             * (k + 1.0 + b) / ((h + 1.0) * (h + 3.0)))
        b_k = -(a * a - b * b) / (h * (h + 2.0))
        p_next = ((x - b_k) * p_cur - a_k * p_prev) / a_next
        p_prev, p_cur, a_k = p_cur, p_next, a_next
    return p_cur


def grad_jacobi_p(x, alpha, beta, n):
    """d/dx of the orthonormal P_n^(alpha,beta): sqrt(n(n+a+b+1)) P_{n-1}^(a+1,b+1)."""
    x = np.asarray(x, dtype=np.float64)
    if n == 0:
        return np.zeros(x.shape)
    return math.sqrt(n * (n + alpha + beta + 1.0)) * jacobi_p(x, alpha + 1.0, beta + 1.0, n - 1)


def gauss_lobatto(N):
    """Legendre-Gauss-Lobatto points on [-1, 1]: +-1 and the roots of P'_N."""
    if N == 1:
        return np.array([-1.0, 1.0])
    interior, _ = roots_jacobi(N - 1, 1.0, 1.0)
    return np.concatenate(([-1.0], np.sort(interior), [1.0]))


def vandermonde_1d(N, r):
    r = np.asarray(r, dtype=np.float64)
    return np.stack([jacobi_p(r, 0.0, 0.0, j) for j in range(N + 1)], axis=1)


def _warp_factor(N, rout):
    """Warburton's 1D warp: LGL minus equispaced, interpolated, divided by the blend."""
    r_lgl = gauss_lobatto(N)
    r_eq = np.linspace(-1.0, 1.0, N + 1)
    v_eq = vandermonde_1d(N, r_eq)
    p_out = vandermonde_1d(N, rout)           # (len(rout), N+1)
    lagr = np.linalg.solve(v_eq.T, p_out.T)    # Lagrange basis on r_eq at rout
    warp = lagr.T @ (r_lgl - r_eq)
    interior = np.abs(rout) < 1.0 - 1.0e-10
    denom = 1.0 - (interior * rout) ** 2
    return warp / denom + warp * (interior - 1.0)


def nodes_equilateral(N):
    """Warp & blend nodes on the equilateral triangle (-1,-1/sqrt3),(1,-1/sqrt3),(0,2/sqrt3)."""
    alpha = alpha_opt(N)
    l1, l3 = [], []
    for i in range(N + 1):          # row index (distance from the bottom edge)
        for j in range(N + 1 - i):  # position along the row
            l1.append(i / N)
            l3.append(j / N)
    l1 = np.array(l1)
    l3 = np.array(l3)
    l2 = 1.0 - l1 - l3
    x = -l2 + l3
    y = (-l2 - l3 + 2.0 * l1) / math.sqrt(3.0)
    blend1, blend2, blend3 = 4.0 * l2 * l3, 4.0 * l1 * l3, 4.0 * l1 * l2
    w1 = blend1 * _warp_factor(N, l3 - l2) * (1.0 + (alpha * l1) ** 2)
    w2 = blend2 * _warp_factor(N, l1 - l3) * (1.0 + (alpha * l2) ** 2)
    w3 = blend3 * _warp_factor(N, l2 - l1) * (1.0 + (alpha * l3) ** 2)
    x = x + w1 + math.cos(2.0 * math.pi / 3.0) * w2 + math.cos(4.0 * math.pi / 3.0) * w3
    y = y + math.sin(2.0 * math.pi / 3.0) * w2 + math.sin(4.0 * math.pi / 3.0) * w3
    return x, y


def equilateral_to_rs(x, y):
    """Barycentric map from the equilateral triangle to K^ (vertex order kept)."""
    l1 = (math.sqrt(3.0) * y + 1.0) / 3.0
    l2 = (-3.0 * x - math.sqrt(3.0) * y + 2.0) / 6.0
    l3 = (3.0 * x - math.sqrt(3.0) * y + 2.0) / 6.0
    return -l2 + l3 - l1, -l2 - l3 + l1


def nodes_rs(N):
    return equilateral_to_rs(*nodes_equilateral(N))


def rs_to_ab(r, s):
    """Collapsed coordinates a = 2(1+r)/(1-s) - 1 (a = -1 at the top vertex), b = s."""
    r = np.asarray(r, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    a = np.where(np.abs(s - 1.0) > 1e-14, 2.0 * (1.0 + r) / np.where(s != 1.0, 1.0 - s, 1.0) - 1.0, -1.0)
    return a, s


def mode_indices(N):
    return [(i, j) for i in range(N + 1) for j in range(N + 1 - i)]


def pkd_mode(a, b, i, j):
    """Orthonormal PKD mode sqrt(2) P_i(a) P_j^(2i+1,0)(b) (1-b)^i on K^."""
    return math.sqrt(2.0) * jacobi_p(a, 0, 0, i) * jacobi_p(b, 2 * i + 1, 0, j) * (1.0 - b) ** i


def pkd_mode_grad(a, b, i, j):
    """Exact (d/dr, d/ds) of pkd_mode, by the chain rule through (a, b).

    da/dr = 2/(1-b), da/ds = (1+a)/(1-b), db/ds = 1; the factor (1-b)^i absorbs
    the 1/(1-b) so the expressions stay finite at the top vertex.
    """
    f, df = jacobi_p(a, 0, 0, i), grad_jacobi_p(a, 0, 0, i)
    g, dg = jacobi_p(b, 2 * i + 1, 0, j), grad_jacobi_p(b, 2 * i + 1, 0, j)
    om = 1.0 - b
    om_im1 = om ** (i - 1) if i >= 1 else np.zeros_like(b)
    ddr = 2.0 * df * g * om_im1
    dds = df * (1.0 + a) * g * om_im1 + f * dg * om ** i - i * f * g * om_im1
    return math.sqrt(2.0) * ddr, math.sqrt(2.0) * dds


def vandermonde_2d(N, r, s):
    a, b = rs_to_ab(r, s)
    return np.stack([pkd_mode(a, b, i, j) for (i, j) in mode_indices(N)], axis=1)


def grad_vandermonde_2d(N, r, s):
    a, b = rs_to_ab(r, s)
    cols = [pkd_mode_grad(a, b, i, j) for (i, j) in mode_indices(N)]
    return np.stack([c[0] for c in cols], axis=1), np.stack([c[1] for c in cols], axis=1)


def face_masks(N, r, s, tol=1e-10):
    """Node indices of the three faces, each in counter-clockwise order."""
    f0 = np.where(np.abs(s + 1.0) < tol)[0]
    f0 = f0[np.argsort(r[f0])]                 # (-1,-1) -> (1,-1)
    f1 = np.where(np.abs(r + s) < tol)[0]
    f1 = f1[np.argsort(s[f1])]                 # (1,-1) -> (-1,1)
    f2 = np.where(np.abs(r + 1.0) < tol)[0]
    f2 = f2[np.argsort(-s[f2])]                # (-1,1) -> (-1,-1)
    return np.stack([f0, f1, f2])


class RefElement:
    """All reference-element operators for polynomial order N (Sec. 2.2, eq. weak_matrices_calc)."""

    def __init__(self, N):
        self.N = N
        self.Np = (N + 1) * (N + 2) // 2
        self.Nfp = N + 1
        self.r, self.s = nodes_rs(N)
        self.V = vandermonde_2d(N, self.r, self.s)
        self.Vr, self.Vs = grad_vandermonde_2d(N, self.r, self.s)
        vinv = np.linalg.inv(self.V)
        self.Dr = self.Vr @ vinv
        self.Ds = self.Vs @ vinv
        self.Minv = self.V @ self.V.T
        self.M = np.linalg.inv(self.Minv)
        self.Fmask = face_masks(N, self.r, self.s)
        # face mass: 1D mass matrix in the face's own parameter xi in [-1, 1]
        # (the physical face length enters through sJ = |e| / 2)
        self.E = np.zeros((self.Np, 3 * self.Nfp))
        for f in range(3):
            if f == 0:
                xi = self.r[self.Fmask[f]]
            elif f == 1:
                xi = self.s[self.Fmask[f]]
            else:
                xi = -self.s[self.Fmask[f]]
            v1 = vandermonde_1d(N, xi)
            m1 = np.linalg.inv(v1 @ v1.T)
            for i in range(self.Nfp):
                self.E[self.Fmask[f][i], f * self.Nfp:(f + 1) * self.Nfp] += m1[i]
        self.LIFT = self.Minv @ self.E
        self.LIFTr = self.Minv @ self.Dr.T @ self.E
        self.LIFTs = self.Minv @ self.Ds.T @ self.E
        # weak-form derivative operators M^-1 Dr^T M, M^-1 Ds^T M
        self.Drw = self.Minv @ self.Dr.T @ self.M
        self.Dsw = self.Minv @ self.Ds.T @ self.M
        # face quadrature weights in xi (row sums of each face mass matrix)
        self.wface = np.array([self.E[self.Fmask[f], f * self.Nfp:(f + 1) * self.Nfp].sum(axis=1)
                               for f in range(3)])
