// Host set-up of isoparametric (curved) elements in FP64.
//
// An element's map T_K: K^ -> K (Sec. 2.2 allows affine or isoparametric
// maps) is the degree-p interpolant of the node positions the caller gives.
// For the curved elements and every element sharing a face with one (the set
// S, whose face terms read a curved element's metric terms) this builds, per
// node, the metric terms of the map and J; per face node, the unit normal and
// sJ = |dx/dxi| from the map's tangent; the element mass matrix
// M^K = int_K^ l_i l_j J (a collapsed Gauss rule with 2p points per
// direction, exact for J's degree 2p - 2 plus 2p) and P_K = (M^K)^-1 M.  The
// penalty's geometric factor C_inv = (p+1)(p+2)|e|/(2|K|) takes the curved
// face length (32-point Gauss-Legendre of |dx/dxi|) and area of every curved
// element, on its own faces and on its neighbours' shared faces.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <set>

#include "dg_internal.h"

namespace dgmi {
namespace {

constexpr int kFaceLengthPoints = 32;

// Reference face parameter xi of face node j of face f (counter-clockwise):
// face 0 r = xi, face 1 (r, s) = (-xi, xi), face 2 s = -xi.
double face_xi(const RefOps& ref, int f, int j) {
  const int n = ref.Fmask[f * ref.Nfp + j];
  return f == 0 ? ref.r[n] : (f == 1 ? ref.s[n] : -ref.s[n]);
}

// d(x, y)/dxi on face f from the map's derivatives at a point of that face.
void face_tangent(int f, double xr, double xs, double yr, double ys, double& tx, double& ty) {
  if (f == 0) {
    tx = xr;
    ty = yr;
  } else if (f == 1) {
    tx = xs - xr;
    ty = ys - yr;
  } else {
    tx = -xs;
    ty = -ys;
  }
}

}  // namespace

bool build_curved_tables(const RefOps& ref, const Physics& ph, int64_t n, const int32_t* elems,
                         const double* xy, MeshTables& t, std::string& err) {
  const int N = ref.N, Np = ref.Np, Nfp = ref.Nfp;
  const int64_t K = t.K;
  char msg[256];
  t.cslot.clear();
  t.celem.clear();
  t.cnode.clear();
  t.cface.clear();
  t.cP.clear();
  t.carea.clear();
  if (n <= 0) return true;
  std::vector<char> curved(K, 0);
  for (int64_t i = 0; i < n; ++i) {
    if (elems[i] < 0 || elems[i] >= K) {
      err = "curved element index out of range";
      return false;
    }
    if (curved[elems[i]]) {
      err = "a curved element is listed twice";
      return false;
    }
    curved[elems[i]] = 1;
  }
  // periodic translation of every shared face (from the straight positions)
  std::vector<double> shift(K * 3 * 2, 0.0);
  for (int64_t k = 0; k < K; ++k)
    for (int f = 0; f < 3; ++f) {
      const int64_t kf = k * 3 + f;
      if (t.tag[kf] != 0) continue;
      const int64_t kn = t.nbr[kf];
      const int fn = t.nbr_face[kf];
      double sx = 0.0, sy = 0.0;
      for (int j = 0; j < Nfp; ++j) {
        const int a = ref.Fmask[f * Nfp + j], b = ref.Fmask[fn * Nfp + j];
        sx += t.x[k * Np + a] - t.x[kn * Np + b];
        sy += t.y[k * Np + a] - t.y[kn * Np + b];
      }
      shift[2 * kf] = sx / Nfp;
      shift[2 * kf + 1] = sy / Nfp;
    }
  double scale = 1.0;
  for (int64_t i = 0; i < K * Np; ++i) scale = std::max({scale, std::fabs(t.x[i]), std::fabs(t.y[i])});
  for (int64_t i = 0; i < n; ++i) {
    const int64_t k = elems[i];
    for (int m = 0; m < Np; ++m) {
      t.x[k * Np + m] = xy[(i * 2 + 0) * Np + m];
      t.y[k * Np + m] = xy[(i * 2 + 1) * Np + m];
    }
  }
  // conforming shared faces: the same node positions on both sides
  for (int64_t k = 0; k < K; ++k) {
    if (!curved[k]) continue;
    for (int f = 0; f < 3; ++f) {
      const int64_t kf = k * 3 + f;
      if (t.tag[kf] != 0) continue;
      const int64_t kn = t.nbr[kf];
      const int fn = t.nbr_face[kf];
      for (int j = 0; j < Nfp; ++j) {
        const int a = ref.Fmask[f * Nfp + j], b = ref.Fmask[fn * Nfp + (Nfp - 1 - j)];
        const double dx = t.x[k * Np + a] - t.x[kn * Np + b] - shift[2 * kf];
        const double dy = t.y[k * Np + a] - t.y[kn * Np + b] - shift[2 * kf + 1];
        if (std::sqrt(dx * dx + dy * dy) > 1e-10 * scale) {
          std::snprintf(msg, sizeof msg, "face (%lld,%d) of a curved element does not conform with (%lld,%d)",
                        (long long)k, f, (long long)kn, fn);
          err = msg;
          return false;
        }
      }
    }
  }
  // the set S: curved elements and their face neighbours, in element order
  std::set<int64_t> S;
  for (int64_t k = 0; k < K; ++k) {
    if (!curved[k]) continue;
    S.insert(k);
    for (int f = 0; f < 3; ++f)
      if (t.tag[k * 3 + f] == 0) S.insert(t.nbr[k * 3 + f]);
  }
  const int64_t ns = (int64_t)S.size();
  t.cslot.assign(K, -1);
  t.celem.assign(S.begin(), S.end());
  for (int64_t i = 0; i < ns; ++i) t.cslot[t.celem[i]] = (int32_t)i;
  t.cnode.assign(ns * 5 * Np, 0.0);
  t.cface.assign(ns * 3 * 3 * Nfp, 0.0);
  t.cP.assign(ns * Np * Np, 0.0);
  t.carea.assign(ns, 0.0);

  // rules: the element mass matrix (2p points per direction) and face lengths
  const int q = 2 * N;
  std::vector<double> xa, wa, xb, wb, rq, sq, wq;
  gauss_jacobi_rule(q, 0.0, 0.0, xa, wa);
  gauss_jacobi_rule(q, 1.0, 0.0, xb, wb);
  for (int i = 0; i < q; ++i)
    for (int j = 0; j < q; ++j) {
      rq.push_back(0.5 * (1.0 + xa[i]) * (1.0 - xb[j]) - 1.0);
      sq.push_back(xb[j]);
      wq.push_back(0.5 * wa[i] * wb[j]);
    }
  const int Nq = q * q;
  std::vector<double> Lq, Lrq, Lsq;
  if (!lagrange_at(ref, rq, sq, Lq, Lrq, Lsq)) {
    err = "singular Vandermonde matrix";
    return false;
  }
  std::vector<double> xg, wg;
  gauss_jacobi_rule(kFaceLengthPoints, 0.0, 0.0, xg, wg);
  // d/dxi of the 1D Lagrange basis of each face's nodes at the Gauss points
  std::vector<double> Dg(3 * kFaceLengthPoints * Nfp);
  for (int f = 0; f < 3; ++f) {
    std::vector<double> V1(Nfp * Nfp);
    for (int j = 0; j < Nfp; ++j)
      for (int m = 0; m <= N; ++m) V1[j * Nfp + m] = legendre(face_xi(ref, f, j), m);
    if (!invert_matrix(V1, Nfp)) {
      err = "singular face Vandermonde matrix";
      return false;
    }
    for (int g = 0; g < kFaceLengthPoints; ++g)
      for (int j = 0; j < Nfp; ++j) {
        double v = 0.0;
        for (int m = 0; m <= N; ++m) v += dlegendre(xg[g], m) * V1[m * Nfp + j];
        Dg[(f * kFaceLengthPoints + g) * Nfp + j] = v;
      }
  }

  // effective Fscale |e| / |K| of every face (straight: the geometry table's)
  std::vector<double> fs_eff(K * 3);
  for (int64_t k = 0; k < K; ++k)
    for (int f = 0; f < 3; ++f) fs_eff[k * 3 + f] = t.geo[k * kGeoStride + 4 + 4 * f + 2];

  for (int64_t i = 0; i < ns; ++i) {
    const int64_t k = t.celem[i];
    const double* X = &t.x[k * Np];
    const double* Y = &t.y[k * Np];
    double* nd = &t.cnode[i * 5 * Np];
    std::vector<double> xr(Np), xs(Np), yr(Np), ys(Np);
    for (int a = 0; a < Np; ++a) {
      double v1 = 0, v2 = 0, v3 = 0, v4 = 0;
      for (int m = 0; m < Np; ++m) {
        v1 += ref.Dr[a * Np + m] * X[m];
        v2 += ref.Ds[a * Np + m] * X[m];
        v3 += ref.Dr[a * Np + m] * Y[m];
        v4 += ref.Ds[a * Np + m] * Y[m];
      }
      xr[a] = v1;
      xs[a] = v2;
      yr[a] = v3;
      ys[a] = v4;
      const double J = v1 * v4 - v2 * v3;
      if (!(J > 0.0)) {
        std::snprintf(msg, sizeof msg, "element %lld: non-positive Jacobian at node %d", (long long)k, a);
        err = msg;
        return false;
      }
      nd[0 * Np + a] = v4 / J;   // rx
      nd[1 * Np + a] = -v2 / J;  // ry
      nd[2 * Np + a] = -v3 / J;  // sx
      nd[3 * Np + a] = v1 / J;   // sy
      nd[4 * Np + a] = J;
    }
    double* fc = &t.cface[i * 3 * 3 * Nfp];
    for (int f = 0; f < 3; ++f)
      for (int j = 0; j < Nfp; ++j) {
        const int a = ref.Fmask[f * Nfp + j];
        double tx, ty;
        face_tangent(f, xr[a], xs[a], yr[a], ys[a], tx, ty);
        const double L = std::sqrt(tx * tx + ty * ty);
        fc[0 * 3 * Nfp + f * Nfp + j] = ty / L;
        fc[1 * 3 * Nfp + f * Nfp + j] = -tx / L;
        fc[2 * 3 * Nfp + f * Nfp + j] = L;
      }
    // mass matrix, area, P = (M^K)^-1 M
    std::vector<double> MK(Np * Np, 0.0);
    double area = 0.0;
    for (int g = 0; g < Nq; ++g) {
      double a1 = 0, a2 = 0, a3 = 0, a4 = 0;
      for (int m = 0; m < Np; ++m) {
        a1 += Lrq[g * Np + m] * X[m];
        a2 += Lsq[g * Np + m] * X[m];
        a3 += Lrq[g * Np + m] * Y[m];
        a4 += Lsq[g * Np + m] * Y[m];
      }
      const double J = a1 * a4 - a2 * a3;
      if (!(J > 0.0)) {
        std::snprintf(msg, sizeof msg, "element %lld: non-positive Jacobian inside", (long long)k);
        err = msg;
        return false;
      }
      const double w = wq[g] * J;
      area += w;
      for (int a = 0; a < Np; ++a)
        for (int b = 0; b < Np; ++b) MK[a * Np + b] += w * Lq[g * Np + a] * Lq[g * Np + b];
    }
    t.carea[i] = area;
    if (!invert_matrix(MK, Np)) {
      err = "singular element mass matrix";
      return false;
    }
    double* P = &t.cP[i * Np * Np];
    for (int a = 0; a < Np; ++a)
      for (int b = 0; b < Np; ++b) {
        double v = 0.0;
        for (int m = 0; m < Np; ++m) v += MK[a * Np + m] * ref.M[m * Np + b];
        P[a * Np + b] = v;
      }
    if (curved[k])
      for (int f = 0; f < 3; ++f) {
        double len = 0.0;
        for (int g = 0; g < kFaceLengthPoints; ++g) {
          double tx = 0.0, ty = 0.0;
          for (int j = 0; j < Nfp; ++j) {
            const int a = ref.Fmask[f * Nfp + j];
            const double d = Dg[(f * kFaceLengthPoints + g) * Nfp + j];
            tx += d * X[a];
            ty += d * Y[a];
          }
          len += wg[g] * std::sqrt(tx * tx + ty * ty);
        }
        fs_eff[k * 3 + f] = len / area;
      }
  }
  // penalty geometric factors with the curved lengths and areas (the same
  // formula as the straight set-up: C_inv = Np |e| / |K|, h_e = 2 |K| / |e|)
  for (int64_t k = 0; k < K; ++k)
    for (int f = 0; f < 3; ++f) {
      const int64_t kf = k * 3 + f;
      const double own = fs_eff[kf];
      const double other = t.tag[kf] == 0 ? fs_eff[t.nbr[kf] * 3 + t.nbr_face[kf]] : own;
      const double fs_max = std::max(own, other);
      double sg;
      if (ph.penalty_mode == 0)
        sg = ph.C_pen * (1.0 + ph.theta) * (1.0 + ph.theta) * 3.0 * Np * fs_max;
      else
        sg = ph.C_pen * (N + 1) * (N + 1) * 0.5 * fs_max;
      t.geo[k * kGeoStride + 4 + 4 * f + 3] = sg;
    }
  // wall face node coordinates (moments) on the curved positions
  t.wall_xy.clear();
  for (int32_t kf : t.wall_faces) {
    const int64_t k = kf / 3;
    const int f = kf % 3;
    for (int j = 0; j < Nfp; ++j) {
      const int a = ref.Fmask[f * Nfp + j];
      t.wall_xy.push_back(t.x[k * Np + a]);
      t.wall_xy.push_back(t.y[k * Np + a]);
    }
  }
  return true;
}

}  // namespace dgmi
