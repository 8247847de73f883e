"""Seeded synthetic inputs shared by the oracle tests and the HIP path.

This module only produces input data: vertex coordinates, triangle lists,
face tags, periods, flow parameters and initial states evaluated at caller-
supplied node coordinates.  It holds none of the discretisation's arithmetic
(no basis, no operators, no fluxes), so both sides of every parity test can
consume it.

The paper meshes its domains with a commercial mesher; those meshes are not
available, so these generators stand in for them with the sizes of the
workloads the method is measured on:

* periodic split-quad squares (manufactured / vortex / Fourier-mode cases),
* graded O-grids around a unit-diameter cylinder (wall at r = 1/2, circular
  far field), each quad split along a diagonal into two triangles.

Nondimensionalisation: rho_inf = 1, sound speed c_inf = 1 (p_inf = 1/gamma),
v_inf = (M, 0), mu = rho_inf |v_inf| L / Re.
"""
import math

import numpy as np

TAG_INTERIOR, TAG_WALL, TAG_FAR = 0, 1, 2
SEED_BASE = 20250825


def rng_for(config_index, salt=0):
    return np.random.default_rng(SEED_BASE + int(config_index) + 1000 * int(salt))


# --------------------------------------------------------------------------
# meshes
# --------------------------------------------------------------------------
def periodic_square(nx, ny, Lx, Ly, x0=0.0, y0=0.0):
    """nx x ny quads on [x0, x0+Lx] x [y0, y0+Ly], each split into 2 CCW triangles.

    Returns dict(VX, VY, EToV, face_tag, period).  The two triangles of quad
    (i, j) are (v00, v10, v11) and (v00, v11, v01).
    """
    xs = x0 + Lx * np.arange(nx + 1) / nx
    ys = y0 + Ly * np.arange(ny + 1) / ny
    VX = np.repeat(xs[None, :], ny + 1, axis=0).ravel()
    VY = np.repeat(ys[:, None], nx + 1, axis=1).ravel()

    def vid(i, j):
        return j * (nx + 1) + i

    tris = []
    for j in range(ny):
        for i in range(nx):
            a, b, c, d = vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)
            tris.append((a, b, c))
            tris.append((a, c, d))
    EToV = np.array(tris, dtype=np.int32)
    face_tag = np.zeros(EToV.shape, dtype=np.int8)
    return dict(VX=VX, VY=VY, EToV=EToV, face_tag=face_tag, period=(float(Lx), float(Ly)))


def ogrid(ntheta, nr, R0=0.5, R1=30.0, ratio=1.05):
    """O-grid around a cylinder: ntheta x nr quads, radial spacing growing by `ratio`.

    Element order: radial ring outer, angle inner, two triangles per quad, so
    the two elements of a quad and the angular neighbours are adjacent in memory.
    Faces on r = R0 are tagged wall (1), faces on r = R1 far field (2).
    """
    if ratio == 1.0:
        dr = np.full(nr, (R1 - R0) / nr)
    else:
        dr0 = (R1 - R0) * (ratio - 1.0) / (ratio ** nr - 1.0)
        dr = dr0 * ratio ** np.arange(nr)
    radii = R0 + np.concatenate(([0.0], np.cumsum(dr)))
    radii[-1] = R1
    th = 2.0 * math.pi * np.arange(ntheta) / ntheta
    VX = (radii[:, None] * np.cos(th)[None, :]).ravel()
    VY = (radii[:, None] * np.sin(th)[None, :]).ravel()

    def vid(i, j):
        return i * ntheta + (j % ntheta)

    tris, tags = [], []
    for i in range(nr):
        for j in range(ntheta):
            a, b, c, d = vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)
            # (r_i,th_j) -> (r_i+1,th_j) -> (r_i+1,th_j+1) -> (r_i,th_j+1) is CCW
            tris.append((a, b, c))
            tags.append((TAG_INTERIOR, TAG_FAR if i + 1 == nr else TAG_INTERIOR, TAG_INTERIOR))
            tris.append((a, c, d))
            tags.append((TAG_INTERIOR, TAG_INTERIOR, TAG_WALL if i == 0 else TAG_INTERIOR))
    return dict(VX=VX, VY=VY, EToV=np.array(tris, dtype=np.int32),
                face_tag=np.array(tags, dtype=np.int8), period=(0.0, 0.0))


def curve_wall(mesh, x, y, center=(0.0, 0.0), tag=TAG_WALL):
    """Node positions of isoparametric elements whose `tag` faces lie on
    circles about `center` (the cylinder's wall): for every element with such
    a face, the positions of all its nodes, so that the element's map is the
    polynomial interpolant of those positions.

    x, y: (Np, K) node coordinates of the straight-sided mesh (any node set;
    only the positions are used).  For a face from vertex a to vertex b on the
    circle through them, a node with barycentric coordinates (la, lb, lc) in
    the straight triangle moves by (la + lb)^2 (A(xi) - C(xi)), xi = lb / (la +
    lb): C is the chord point and A the circle point at the same fraction of
    the angle from a to b.  Face nodes land on the circle; nodes on the two
    other edges do not move (xi is 0 or 1 there), so those edges stay straight
    and the mesh stays conforming.  Returns (elems, xy): element indices
    (int32) and their node positions, shape (n, 2, Np).
    """
    VX = np.asarray(mesh["VX"], dtype=np.float64)
    VY = np.asarray(mesh["VY"], dtype=np.float64)
    EToV = np.asarray(mesh["EToV"])
    ft = np.asarray(mesh["face_tag"])
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    cx, cy = float(center[0]), float(center[1])
    elems, out = [], []
    for k in range(EToV.shape[0]):
        faces = [f for f in range(3) if ft[k, f] == tag]
        if not faces:
            continue
        px, py = x[:, k].copy(), y[:, k].copy()
        for f in faces:
            a, b, c = EToV[k, f], EToV[k, (f + 1) % 3], EToV[k, (f + 2) % 3]
            # barycentric coordinates of the straight-sided positions
            det = (VX[b] - VX[a]) * (VY[c] - VY[a]) - (VX[c] - VX[a]) * (VY[b] - VY[a])
            lb = ((x[:, k] - VX[a]) * (VY[c] - VY[a]) - (VX[c] - VX[a]) * (y[:, k] - VY[a])) / det
            lc = ((VX[b] - VX[a]) * (y[:, k] - VY[a]) - (x[:, k] - VX[a]) * (VY[b] - VY[a])) / det
            lab = 1.0 - lc
            xi = np.where(lab > 1e-12, lb / np.where(lab > 1e-12, lab, 1.0), 0.0)
            xi = np.clip(xi, 0.0, 1.0)
            ra = math.hypot(VX[a] - cx, VY[a] - cy)
            rb = math.hypot(VX[b] - cx, VY[b] - cy)
            R = 0.5 * (ra + rb)
            ta = math.atan2(VY[a] - cy, VX[a] - cx)
            dth = math.atan2(VY[b] - cy, VX[b] - cx) - ta
            dth = (dth + math.pi) % (2.0 * math.pi) - math.pi
            th = ta + xi * dth
            Ax, Ay = cx + R * np.cos(th), cy + R * np.sin(th)
            Cx = (1.0 - xi) * VX[a] + xi * VX[b]
            Cy = (1.0 - xi) * VY[a] + xi * VY[b]
            w = lab * lab
            px += w * (Ax - Cx)
            py += w * (Ay - Cy)
        elems.append(k)
        out.append(np.stack([px, py]))
    return np.array(elems, dtype=np.int32), np.array(out, dtype=np.float64).reshape(len(elems), 2, x.shape[0])


def growth_ratio(R0, R1, nr, h_wall):
    """Geometric growth ratio q > 1 of nr radial cells from R0 to R1 whose
    first cell is h_wall thick: h_wall (q^nr - 1) / (q - 1) = R1 - R0, solved
    by bisection (requires h_wall < (R1 - R0) / nr)."""
    L = R1 - R0
    if not (0.0 < h_wall < L / nr):
        raise ValueError("h_wall must lie in (0, (R1 - R0) / nr)")
    lo, hi = 1.0 + 1e-12, 2.0
    while h_wall * (hi ** nr - 1.0) / (hi - 1.0) < L:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if h_wall * (mid ** nr - 1.0) / (mid - 1.0) < L:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


# --------------------------------------------------------------------------
# flow parameters
# --------------------------------------------------------------------------
def free_stream(M, gamma=1.4, angle=0.0):
    """Conservative free stream with rho = 1, c = 1, |v| = M."""
    rho = 1.0
    p = 1.0 / gamma
    u, v = M * math.cos(angle), M * math.sin(angle)
    return np.array([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


def physics_params(Re, M, L=1.0, gamma=1.4, Pr=0.72):
    return dict(gamma=gamma, Pr=Pr, mu=M * L / Re, U_inf=free_stream(M, gamma))


# --------------------------------------------------------------------------
# initial states at given node coordinates (arrays of any common shape)
# --------------------------------------------------------------------------
def isentropic_vortex(x, y, M=0.3, beta=5.0, R=1.0, xc=5.0, yc=5.0, gamma=1.4, Lper=None):
    """Isentropic vortex of strength beta and radius R centred at (xc, yc) in the free stream.

    delta v = beta/(2 pi) exp((1 - r^2/R^2)/2) (-(y-yc), x-xc)/R,
    T = p/rho = 1/gamma - (gamma-1) beta^2 exp(1 - r^2/R^2) / (8 gamma pi^2),
    rho = (gamma T)^(1/(gamma-1)), p = rho T.  Returns (4, ...) conservative.
    With Lper set, the nearest periodic image of the centre is used.
    """
    dx = x - xc
    dy = y - yc
    if Lper is not None:
        dx = dx - Lper * np.round(dx / Lper)
        dy = dy - Lper * np.round(dy / Lper)
    r2 = (dx * dx + dy * dy) / (R * R)
    f = np.exp(0.5 * (1.0 - r2))
    u = M - beta / (2.0 * math.pi) * f * dy / R
    v = beta / (2.0 * math.pi) * f * dx / R
    T = 1.0 / gamma - (gamma - 1.0) * beta ** 2 * np.exp(1.0 - r2) / (8.0 * gamma * math.pi ** 2)
    rho = (gamma * T) ** (1.0 / (gamma - 1.0))
    p = rho * T
    return np.stack([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


def noisy_free_stream(shape, U_inf, rng, amp=1e-3):
    """U = U_inf (1 + amp xi), xi ~ U(-1, 1) per node and field; shape = (4, ...)."""
    xi = rng.uniform(-1.0, 1.0, size=shape)
    return np.asarray(U_inf).reshape((4,) + (1,) * (len(shape) - 1)) * (1.0 + amp * xi)


def wake_kick(x, y, U_inf, amp=0.1, xc=1.5, R=0.5, gamma=1.4):
    """Free stream with a transverse velocity blob behind the cylinder,
    v += amp |v_inf| exp(-((x - xc)^2 + y^2) / R^2) (density and pressure of
    the free stream): breaks the up-down symmetry so that shedding starts
    early instead of growing from rounding."""
    U_inf = np.asarray(U_inf, dtype=np.float64)
    rho = U_inf[0]
    u, v = U_inf[1] / rho, U_inf[2] / rho
    p = (gamma - 1.0) * (U_inf[3] - 0.5 * rho * (u * u + v * v))
    vel = math.hypot(u, v)
    vv = v + amp * vel * np.exp(-((x - xc) ** 2 + y ** 2) / (R * R))
    uu = np.full(np.shape(x), u)
    r = np.full(np.shape(x), rho)
    return np.stack([r, r * uu, r * vv, p / (gamma - 1.0) + 0.5 * r * (uu * uu + vv * vv)])


def fourier_modes(x, y, rng, L=10.0, amp=1e-2, q0=(1.0, 0.3, 0.0, 1.0 / 1.4), gamma=1.4, nmodes=3):
    """Smooth periodic state: each primitive q0 + amp sum_m a_m sin(2 pi k_m.x / L + phi_m)."""
    prim = []
    for base in q0:
        val = np.full(np.shape(x), float(base))
        for _ in range(nmodes):
            k = rng.integers(1, 4, size=2)
            a = rng.uniform(-1.0, 1.0) / nmodes
            ph = rng.uniform(0.0, 2.0 * math.pi)
            val = val + amp * a * np.sin(2.0 * math.pi * (k[0] * x + k[1] * y) / L + ph)
        prim.append(val)
    rho, u, v, p = prim
    return np.stack([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


# --------------------------------------------------------------------------
# the workloads
# --------------------------------------------------------------------------
def workload(name, p=None):
    """Mesh + physics of a named workload; `p` overrides the default order."""
    if name == "vortex512":
        mesh = periodic_square(16, 16, 10.0, 10.0)
        phys = physics_params(Re=100.0, M=0.3, L=1.0)
        return dict(mesh=mesh, p=3 if p is None else p, penalty_mode=1, C_pen=1.0, theta=1.0, **phys)
    if name == "cylinder20k":
        mesh = ogrid(80, 128, 0.5, 30.0, 1.05)
        phys = physics_params(Re=100.0, M=0.2, L=1.0)
        return dict(mesh=mesh, p=4 if p is None else p, penalty_mode=0, C_pen=1.0, theta=1.0, **phys)
    if name == "cylinder327k":
        # the same O-grid refined 4x in each direction: K = 327,680, FP64 states
        # well beyond the 256 MB last-level cache
        mesh = ogrid(320, 512, 0.5, 30.0, 1.0 + 0.05 / 4)
        phys = physics_params(Re=100.0, M=0.2, L=1.0)
        return dict(mesh=mesh, p=4 if p is None else p, penalty_mode=0, C_pen=1.0, theta=1.0, **phys)
    if name == "periodic51k":
        mesh = periodic_square(160, 160, 10.0, 10.0)
        phys = physics_params(Re=100.0, M=0.3, L=1.0)
        return dict(mesh=mesh, p=6 if p is None else p, penalty_mode=0, C_pen=1.0, theta=1.0, **phys)
    if name == "shedding20k":
        # stand-in for the stationary-cylinder mesh of the shedding study
        # (about 20k cells, 17 mm first layer at the wall, far field 50 D
        # away): an O-grid of 128 x 80 quads, K = 20,480, interior penalty
        # with theta = 0 (IIP) and C1 = 0.01, Re = 200, M = 0.1
        mesh = ogrid(128, 80, 0.5, 50.0, growth_ratio(0.5, 50.0, 80, 0.017))
        phys = physics_params(Re=200.0, M=0.1, L=1.0)
        return dict(mesh=mesh, p=3 if p is None else p, penalty_mode=0, C_pen=0.01, theta=0.0, **phys)
    raise KeyError(name)


def viv_sweep_cases(n=16, seed_index=2):
    """Seeded instances of a transverse-VIV sweep: per instance an O-grid with
    ntheta in [40, 100] and nr in [64, 160] cells (K = 2 ntheta nr), order p in
    {4, 5, 6}, reduced velocity U* = linspace(3, 8, n), mass ratio 10, no
    structural damping.  Returns (cases, physics) for Re = 100, M = 0.2."""
    rng = rng_for(seed_index)
    cases = []
    for i, U_star in enumerate(np.linspace(3.0, 8.0, n)):
        nt = int(rng.integers(40, 101))
        nr = int(rng.integers(64, 161))
        p = int(rng.choice([4, 5, 6]))
        cases.append(dict(ntheta=nt, nr=nr, p=p, U_star=float(U_star), m_star=10.0, xi=0.0,
                          mesh=ogrid(nt, nr, 0.5, 30.0, 1.05)))
    phys = physics_params(Re=100.0, M=0.2, L=1.0)
    return cases, dict(penalty_mode=0, C_pen=1.0, theta=1.0, **phys)


def mlp_init(rng, n_in, n_hidden, n_out):
    """Seeded initial parameters of an n_in -> n_hidden -> n_hidden -> n_out
    network as one float32 vector W1 b1 W2 b2 W3 b3 (W row-major [out][in]):
    weights N(0, 2 / fan_in), biases zero."""
    parts = []
    for fi, fo in ((n_in, n_hidden), (n_hidden, n_hidden), (n_hidden, n_out)):
        parts.append(rng.standard_normal((fo, fi)) * math.sqrt(2.0 / fi))
        parts.append(np.zeros(fo))
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)
