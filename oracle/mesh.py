"""Affine triangle geometry and face connectivity (oracle; test infrastructure).

Each triangle K is the image of K^ under the affine map T_K (Sec. 2.2), so
its Jacobian, metric terms and face normals are constants per element and
per face.  Connectivity -- the map E^e of eq. dg_on_K that pairs the nodes
of a face with the neighbour's -- is found here by plain coordinate
matching of face nodes (periodic faces: coordinates taken modulo the
period), which needs no assumption about vertex numbering or orientation.
"""
import numpy as np

TAG_INTERIOR, TAG_WALL, TAG_FAR = 0, 1, 2


class Mesh:
    """Geometry and connectivity of a conforming straight-sided triangle mesh.

    VX, VY: vertex coordinates; EToV: (K, 3) vertex indices, counter-clockwise;
    face_tag: (K, 3) int, face f joins local vertices f and (f+1) % 3, 0 means
    interior (or periodic), 1 wall, 2 far field; period: (px, py), 0 = none.
    """

    def __init__(self, ref, VX, VY, EToV, face_tag=None, period=(0.0, 0.0)):
        self.ref = ref
        VX = np.asarray(VX, dtype=np.float64)
        VY = np.asarray(VY, dtype=np.float64)
        EToV = np.asarray(EToV, dtype=np.int64)
        K = EToV.shape[0]
        self.K = K
        self.period = (float(period[0]), float(period[1]))
        self.face_tag = np.zeros((K, 3), dtype=np.int64) if face_tag is None else np.asarray(face_tag, dtype=np.int64)
        x1, x2, x3 = VX[EToV[:, 0]], VX[EToV[:, 1]], VX[EToV[:, 2]]
        y1, y2, y3 = VY[EToV[:, 0]], VY[EToV[:, 1]], VY[EToV[:, 2]]
        r, s = ref.r[:, None], ref.s[:, None]
        # x = T_K(r, s): vertex 0 at (-1,-1), vertex 1 at (1,-1), vertex 2 at (-1,1)
        self.x = 0.5 * (-(r + s) * x1 + (1.0 + r) * x2 + (1.0 + s) * x3)
        self.y = 0.5 * (-(r + s) * y1 + (1.0 + r) * y2 + (1.0 + s) * y3)
        xr, xs = 0.5 * (x2 - x1), 0.5 * (x3 - x1)
        yr, ys = 0.5 * (y2 - y1), 0.5 * (y3 - y1)
        self.J = xr * ys - xs * yr
        if np.any(self.J <= 0.0):
            raise ValueError("mesh has an element with non-positive Jacobian (clockwise vertices)")
        self.rx, self.ry = ys / self.J, -xs / self.J
        self.sx, self.sy = -yr / self.J, xr / self.J
        # outward normals from the edge vectors: edge f runs from vertex f to f+1,
        # the outward normal of a counter-clockwise polygon is (dy, -dx)/|edge|
        px = [x1, x2, x3]
        py = [y1, y2, y3]
        self.nx = np.zeros((3, K))
        self.ny = np.zeros((3, K))
        self.sJ = np.zeros((3, K))
        for f in range(3):
            dx = px[(f + 1) % 3] - px[f]
            dy = py[(f + 1) % 3] - py[f]
            length = np.hypot(dx, dy)
            self.nx[f] = dy / length
            self.ny[f] = -dx / length
            self.sJ[f] = 0.5 * length          # |e| / 2: ref face parameter spans [-1, 1]
        self.Fscale = self.sJ / self.J[None, :]
        self.area = 2.0 * self.J               # |K|; |K^| = 2
        self.face_len = 2.0 * self.sJ          # |e|
        self._connect()

    def _wrap(self, x, y):
        px, py = self.period
        if px > 0.0:
            x = np.mod(x, px)
            x = np.where(np.abs(x - px) < 1e-9 * px, 0.0, x)
        if py > 0.0:
            y = np.mod(y, py)
            y = np.where(np.abs(y - py) < 1e-9 * py, 0.0, y)
        return x, y

    def _connect(self):
        ref, K = self.ref, self.K
        Fm = ref.Fmask
        fx = self.x[Fm]                        # (3, Nfp, K)
        fy = self.y[Fm]
        wx, wy = self._wrap(fx, fy)
        scale = max(np.ptp(self.x), np.ptp(self.y), 1.0)
        tol = 1e-8 * scale
        # face key: wrapped face-centroid coordinates rounded to the tolerance
        cx, cy = self._wrap(fx.mean(axis=1), fy.mean(axis=1))
        table = {}
        for k in range(K):
            for f in range(3):
                key = (int(np.round(cx[f, k] / tol)), int(np.round(cy[f, k] / tol)))
                table.setdefault(key, []).append((k, f))
        self.EToE = -np.ones((K, 3), dtype=np.int64)
        self.EToF = -np.ones((K, 3), dtype=np.int64)
        for k in range(K):
            for f in range(3):
                key = (int(np.round(cx[f, k] / tol)), int(np.round(cy[f, k] / tol)))
                cands = [c for dk in (-1, 0, 1) for dl in (-1, 0, 1)
                         for c in table.get((key[0] + dk, key[1] + dl), []) if c != (k, f)]
                if self.face_tag[k, f] != TAG_INTERIOR:
                    if cands:
                        raise ValueError("boundary face (%d,%d) has a neighbour" % (k, f))
                    continue
                if len(cands) != 1:
                    raise ValueError("interior face (%d,%d) has %d matches" % (k, f, len(cands)))
                self.EToE[k, f], self.EToF[k, f] = cands[0]
        # node-to-node map: for own face node (f, j, k) the matching neighbour node
        Nfp = ref.Nfp
        self.nbr_node = np.zeros((3, Nfp, K), dtype=np.int64)   # volume node index in neighbour
        self.nbr_elem = np.zeros((3, Nfp, K), dtype=np.int64)
        self.nbr_face = np.zeros((3, K), dtype=np.int64)
        for k in range(K):
            for f in range(3):
                kn, fn = self.EToE[k, f], self.EToF[k, f]
                if kn < 0:
                    self.nbr_node[f, :, k] = Fm[f]
                    self.nbr_elem[f, :, k] = k
                    self.nbr_face[f, k] = f
                    continue
                self.nbr_face[f, k] = fn
                # one translation per face pair (zero, or a multiple of the period
                # across a periodic seam), then nearest-node matching
                sx = fx[f, :, k].mean() - fx[fn, :, kn].mean()
                sy = fy[f, :, k].mean() - fy[fn, :, kn].mean()
                for j in range(Nfp):
                    d = np.hypot(fx[fn, :, kn] + sx - fx[f, j, k], fy[fn, :, kn] + sy - fy[f, j, k])
                    m = int(np.argmin(d))
                    if d[m] > tol:
                        raise ValueError("face nodes of (%d,%d) do not match" % (k, f))
                    self.nbr_node[f, j, k] = Fm[fn][m]
                    self.nbr_elem[f, j, k] = kn
        self.is_boundary = self.EToE < 0
