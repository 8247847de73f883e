// Host set-up in FP64: reference-element operators, affine geometry, face
// connectivity and the penalty's geometric factors.
//
// The paper builds the nodal basis from Warburton's warp & blend nodes and
// the Dubiner/Proriol/Koornwinder orthonormal basis, forms every local
// matrix once on the reference triangle (affine maps, Sec. 2.2 and eq.
// weak_matrices_calc) and pairs the nodes of shared faces through the map
// E^e of eq. dg_on_K.  Everything here runs once per mesh on the host.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <cstdio>
#include <unordered_map>

#include "dg_internal.h"

namespace dgmi {
namespace {

// Warburton's optimised blending exponents alpha_opt(N), N = 1..15
// (J. Eng. Math. 56 (2006), Table 1); larger N use 5/3.
const double kAlphaOpt[15] = {0.0, 0.0, 1.4152, 0.1001, 0.2751, 0.9800, 1.0999, 1.2832,
                              1.3648, 1.4773, 1.4959, 1.5743, 1.5770, 1.6223, 1.6258};

// Orthonormal Jacobi polynomial P_n^(a,b)(x), three-term recurrence.
double jacobi(double x, double a, double b, int n) {
  double g0 = std::pow(2.0, a + b + 1.0) * std::tgamma(a + 1.0) * std::tgamma(b + 1.0) /
              std::tgamma(a + b + 2.0);
  double pm = 1.0 / std::sqrt(g0);
  if (n == 0) return pm;
  double pc = 0.5 * ((a + b + 2.0) * x + (a - b)) * pm / std::sqrt((a + 1.0) * (b + 1.0) / (a + b + 3.0));
  if (n == 1) return pc;
  double aold = 2.0 / (a + b + 2.0) * std::sqrt((a + 1.0) * (b + 1.0) / (a + b + 3.0));
  for (int k = 1; k < n; ++k) {
    double h = 2.0 * k + a + b;
    double anew = 2.0 / (h + 2.0) *
                  std::sqrt((k + 1.0) * (k + 1.0 + a + b) * (k + 1.0 + a) * (k + 1.0 + b) /
                            ((h + 1.0) * (h + 3.0)));
    double bk = -(a * a - b * b) / (h * (h + 2.0));
    double pn = ((x - bk) * pc - aold * pm) / anew;
    pm = pc;
    pc = pn;
    aold = anew;
  }
  return pc;
}

double djacobi(double x, double a, double b, int n) {
  if (n == 0) return 0.0;
  return std::sqrt(n * (n + a + b + 1.0)) * jacobi(x, a + 1.0, b + 1.0, n - 1);
}

// Legendre-Gauss-Lobatto points: -1, the roots of P'_N (Newton with
// deflation on P_{N-1}^(1,1)), +1.
std::vector<double> lgl_points(int N) {
  std::vector<double> x(N + 1);
  x[0] = -1.0;
  x[N] = 1.0;
  int n = N - 1;
  std::vector<double> roots;
  for (int k = 0; k < n; ++k) {
    double z = -std::cos(M_PI * (k + 1.0) / N);
    for (int it = 0; it < 200; ++it) {
      double f = jacobi(z, 1.0, 1.0, n);
      double df = djacobi(z, 1.0, 1.0, n);
      double s = 0.0;
      for (double r : roots) s += 1.0 / (z - r);
      double dz = f / (df - f * s);
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    roots.push_back(z);
  }
  std::sort(roots.begin(), roots.end());
  for (int k = 0; k < n; ++k) x[k + 1] = roots[k];
  return x;
}

// Warp function of the 1D LGL vs equispaced displacement, blended to zero
// at the end points.
double warp_factor(int N, const std::vector<double>& rlgl, double rout) {
  double warp = 0.0;
  for (int i = 0; i <= N; ++i) {
    double xi = -1.0 + 2.0 * i / N;
    double l = 1.0;
    for (int j = 0; j <= N; ++j) {
      if (j == i) continue;
      double xj = -1.0 + 2.0 * j / N;
      l *= (rout - xj) / (xi - xj);
    }
    warp += l * (rlgl[i] - xi);
  }
  // scaled by the blend's 1/(1 - r^2); the warp vanishes at the edge end points
  if (std::fabs(rout) < 1.0 - 1.0e-10) return warp / (1.0 - rout * rout);
  return 0.0;
}

void warp_blend_nodes(int N, std::vector<double>& r, std::vector<double>& s) {
  double alpha = (N >= 1 && N <= 15) ? kAlphaOpt[N - 1] : 5.0 / 3.0;
  std::vector<double> rlgl = lgl_points(N);
  r.clear();
  s.clear();
  const double sq3 = std::sqrt(3.0);
  for (int i = 0; i <= N; ++i) {
    for (int j = 0; j <= N - i; ++j) {
      double L1 = double(i) / N, L3 = double(j) / N, L2 = 1.0 - L1 - L3;
      double x = -L2 + L3, y = (-L2 - L3 + 2.0 * L1) / sq3;
      double b1 = 4.0 * L2 * L3, b2 = 4.0 * L1 * L3, b3 = 4.0 * L1 * L2;
      double w1 = b1 * warp_factor(N, rlgl, L3 - L2) * (1.0 + (alpha * L1) * (alpha * L1));
      double w2 = b2 * warp_factor(N, rlgl, L1 - L3) * (1.0 + (alpha * L2) * (alpha * L2));
      double w3 = b3 * warp_factor(N, rlgl, L2 - L1) * (1.0 + (alpha * L3) * (alpha * L3));
      x += w1 + std::cos(2.0 * M_PI / 3.0) * w2 + std::cos(4.0 * M_PI / 3.0) * w3;
      y += std::sin(2.0 * M_PI / 3.0) * w2 + std::sin(4.0 * M_PI / 3.0) * w3;
      // equilateral -> reference triangle (barycentric coordinates kept)
      double l1 = (sq3 * y + 1.0) / 3.0;
      double l2 = (-3.0 * x - sq3 * y + 2.0) / 6.0;
      double l3 = (3.0 * x - sq3 * y + 2.0) / 6.0;
      r.push_back(-l2 + l3 - l1);
      s.push_back(-l2 - l3 + l1);
    }
  }
}

// PKD mode sqrt(2) P_i(a) P_j^(2i+1,0)(b) (1-b)^i and its exact r/s derivatives.
void pkd(double r, double s, int i, int j, double& v, double& dr, double& ds) {
  double a = (std::fabs(s - 1.0) > 1e-14) ? 2.0 * (1.0 + r) / (1.0 - s) - 1.0 : -1.0;
  double b = s;
  double f = jacobi(a, 0, 0, i), df = djacobi(a, 0, 0, i);
  double g = jacobi(b, 2 * i + 1, 0, j), dg = djacobi(b, 2 * i + 1, 0, j);
  double om = 1.0 - b;
  double om_i = std::pow(om, i);
  double om_im1 = (i >= 1) ? std::pow(om, i - 1) : 0.0;
  v = std::sqrt(2.0) * f * g * om_i;
  dr = std::sqrt(2.0) * 2.0 * df * g * om_im1;
  ds = std::sqrt(2.0) * (df * (1.0 + a) * g * om_im1 + f * dg * om_i - i * f * g * om_im1);
}

// In-place inverse of an n x n row-major matrix (Gauss-Jordan, partial pivoting).
bool invert(std::vector<double>& A, int n) {
  std::vector<double> inv(n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (std::fabs(A[piv * n + c]) < 1e-300) return false;
    if (piv != c)
      for (int k = 0; k < n; ++k) {
        std::swap(A[c * n + k], A[piv * n + k]);
        std::swap(inv[c * n + k], inv[piv * n + k]);
      }
    double d = 1.0 / A[c * n + c];
    for (int k = 0; k < n; ++k) {
      A[c * n + k] *= d;
      inv[c * n + k] *= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double m = A[r * n + c];
      if (m == 0.0) continue;
      for (int k = 0; k < n; ++k) {
        A[r * n + k] -= m * A[c * n + k];
        inv[r * n + k] -= m * inv[c * n + k];
      }
    }
  }
  A.swap(inv);
  return true;
}

std::vector<double> matmul(const std::vector<double>& A, const std::vector<double>& B, int n, int k,
                           int m) {
  std::vector<double> C(n * m, 0.0);
  for (int i = 0; i < n; ++i)
    for (int l = 0; l < k; ++l) {
      double a = A[i * k + l];
      for (int j = 0; j < m; ++j) C[i * m + j] += a * B[l * m + j];
    }
  return C;
}

std::vector<double> transpose(const std::vector<double>& A, int n, int m) {
  std::vector<double> T(m * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < m; ++j) T[j * n + i] = A[i * m + j];
  return T;
}

}  // namespace

bool build_ref_ops(int N, RefOps& o, std::string& err) {
  if (N < 1 || N > kMaxOrder) {
    err = "polynomial order out of range";
    return false;
  }
  o.N = N;
  o.Np = (N + 1) * (N + 2) / 2;
  o.Nfp = N + 1;
  const int Np = o.Np, Nfp = o.Nfp, NF = 3 * Nfp;
  warp_blend_nodes(N, o.r, o.s);
  std::vector<double> V(Np * Np), Vr(Np * Np), Vs(Np * Np);
  for (int n = 0; n < Np; ++n) {
    int col = 0;
    for (int i = 0; i <= N; ++i)
      for (int j = 0; j <= N - i; ++j, ++col) {
        double v, dr, ds;
        pkd(o.r[n], o.s[n], i, j, v, dr, ds);
        V[n * Np + col] = v;
        Vr[n * Np + col] = dr;
        Vs[n * Np + col] = ds;
      }
  }
  std::vector<double> Vinv = V;
  if (!invert(Vinv, Np)) {
    err = "singular Vandermonde matrix";
    return false;
  }
  o.Dr = matmul(Vr, Vinv, Np, Np, Np);
  o.Ds = matmul(Vs, Vinv, Np, Np, Np);
  std::vector<double> Minv = matmul(V, transpose(V, Np, Np), Np, Np, Np);
  // reference mass matrix M = (V V^T)^-1 = V^-T V^-1 (for norms of states)
  o.M = matmul(transpose(Vinv, Np, Np), Vinv, Np, Np, Np);
  // face node lists from the row structure of the node numbering:
  // row i starts at off(i) = i(N+1) - i(i-1)/2 and holds N+1-i nodes
  o.Fmask.assign(3 * Nfp, 0);
  auto off = [N](int i) { return i * (N + 1) - i * (i - 1) / 2; };
  for (int j = 0; j < Nfp; ++j) {
    o.Fmask[0 * Nfp + j] = j;                   // s = -1, r increasing
    o.Fmask[1 * Nfp + j] = off(j) + (N - j);    // r + s = 0, s increasing
    o.Fmask[2 * Nfp + j] = off(N - j);          // r = -1, s decreasing
  }
  // face mass: 1D mass matrix in the face parameter xi in [-1, 1]
  std::vector<double> E(Np * NF, 0.0);
  o.wface.assign(NF, 0.0);
  for (int f = 0; f < 3; ++f) {
    std::vector<double> V1(Nfp * Nfp);
    for (int i = 0; i < Nfp; ++i) {
      int n = o.Fmask[f * Nfp + i];
      double xi = (f == 0) ? o.r[n] : (f == 1 ? o.s[n] : -o.s[n]);
      for (int k = 0; k < Nfp; ++k) V1[i * Nfp + k] = jacobi(xi, 0, 0, k);
    }
    std::vector<double> M1 = matmul(V1, transpose(V1, Nfp, Nfp), Nfp, Nfp, Nfp);
    if (!invert(M1, Nfp)) {
      err = "singular face Vandermonde";
      return false;
    }
    for (int i = 0; i < Nfp; ++i)
      for (int k = 0; k < Nfp; ++k) {
        E[o.Fmask[f * Nfp + i] * NF + f * Nfp + k] += M1[i * Nfp + k];
        o.wface[f * Nfp + i] += M1[i * Nfp + k];
      }
  }
  o.LIFT = matmul(Minv, E, Np, Np, NF);
  o.LIFTr = matmul(matmul(Minv, transpose(o.Dr, Np, Np), Np, Np, Np), E, Np, Np, NF);
  o.LIFTs = matmul(matmul(Minv, transpose(o.Ds, Np, Np), Np, Np, Np), E, Np, Np, NF);
  return true;
}

// Gauss points and weights of the weight (1 - x)^a (1 + x)^b on [-1, 1]:
// the roots of P_q^(a,b) (Newton with deflation from Chebyshev-like starts)
// and w_i = 1 / sum_{k<q} p_k(x_i)^2 with the orthonormal p_k (Christoffel
// numbers).
static void gauss_jacobi(int q, double a, double b, std::vector<double>& x, std::vector<double>& w) {
  x.clear();
  for (int k = 0; k < q; ++k) {
    double z = -std::cos(M_PI * (k + 0.5) / q);
    for (int it = 0; it < 300; ++it) {
      double f = jacobi(z, a, b, q), df = djacobi(z, a, b, q), sum = 0.0;
      for (double r : x) sum += 1.0 / (z - r);
      double dz = f / (df - f * sum);
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x.push_back(z);
  }
  std::sort(x.begin(), x.end());
  w.assign(q, 0.0);
  for (int i = 0; i < q; ++i) {
    double sum = 0.0;
    for (int k = 0; k < q; ++k) {
      double v = jacobi(x[i], a, b, k);
      sum += v * v;
    }
    w[i] = 1.0 / sum;
  }
}

// Basis values and derivatives at points (r, s): rows = points, cols = nodes.
static void basis_at(const RefOps& ref, const std::vector<double>& Vinv, const std::vector<double>& r,
                     const std::vector<double>& s, std::vector<double>& L, std::vector<double>& Lr,
                     std::vector<double>& Ls) {
  const int N = ref.N, Np = ref.Np, n = (int)r.size();
  std::vector<double> V(n * Np), Vr(n * Np), Vs(n * Np);
  for (int k = 0; k < n; ++k) {
    int col = 0;
    for (int i = 0; i <= N; ++i)
      for (int j = 0; j <= N - i; ++j, ++col) {
        double v, dr, ds;
        pkd(r[k], s[k], i, j, v, dr, ds);
        V[k * Np + col] = v;
        Vr[k * Np + col] = dr;
        Vs[k * Np + col] = ds;
      }
  }
  L = matmul(V, Vinv, n, Np, Np);
  Lr = matmul(Vr, Vinv, n, Np, Np);
  Ls = matmul(Vs, Vinv, n, Np, Np);
}

bool build_oi_ops(const RefOps& ref, OIOps& o, std::string& err) {
  const int N = ref.N, Np = ref.Np, Nfp = ref.Nfp;
  const int q = oi_points(N);
  o.q = q;
  o.Nq = q * q;
  // nodal Vandermonde and its inverse, M^-1 = V V^T
  std::vector<double> V(Np * Np), dummy_r(Np * Np), dummy_s(Np * Np);
  for (int n = 0; n < Np; ++n) {
    int col = 0;
    for (int i = 0; i <= N; ++i)
      for (int j = 0; j <= N - i; ++j, ++col) pkd(ref.r[n], ref.s[n], i, j, V[n * Np + col], dummy_r[n * Np + col], dummy_s[n * Np + col]);
  }
  std::vector<double> Vinv = V;
  if (!invert(Vinv, Np)) {
    err = "singular Vandermonde matrix";
    return false;
  }
  const std::vector<double> Minv = matmul(V, transpose(V, Np, Np), Np, Np, Np);
  // element rule: collapsed coordinates, Gauss-Legendre in a, Gauss-Jacobi
  // (weight 1 - b) in b; r = (1 + a)(1 - b)/2 - 1, s = b, dr ds = (1 - b)/2 da db
  std::vector<double> xa, wa, xb, wb;
  gauss_jacobi(q, 0.0, 0.0, xa, wa);
  gauss_jacobi(q, 1.0, 0.0, xb, wb);
  std::vector<double> rq, sq;
  o.wq.clear();
  for (int i = 0; i < q; ++i)
    for (int j = 0; j < q; ++j) {
      rq.push_back(0.5 * (1.0 + xa[i]) * (1.0 - xb[j]) - 1.0);
      sq.push_back(xb[j]);
      o.wq.push_back(0.5 * wa[i] * wb[j]);
    }
  basis_at(ref, Vinv, rq, sq, o.Iq, o.Drq, o.Dsq);
  const int Nq = o.Nq;
  // M^-1 (D^T W): the weights folded in
  std::vector<double> DrW(Np * Nq), DsW(Np * Nq);
  for (int i = 0; i < Np; ++i)
    for (int k = 0; k < Nq; ++k) {
      DrW[i * Nq + k] = o.Drq[k * Np + i] * o.wq[k];
      DsW[i * Nq + k] = o.Dsq[k * Np + i] * o.wq[k];
    }
  o.Wr = matmul(Minv, DrW, Np, Np, Nq);
  o.Ws = matmul(Minv, DsW, Np, Np, Nq);
  // face rule: Gauss-Legendre in the counter-clockwise face parameter xi;
  // face 0 (xi, -1), face 1 (-xi, xi), face 2 (-1, -xi)
  gauss_jacobi(q, 0.0, 0.0, o.xg, o.wg);
  std::vector<double> rf, sf;
  for (int f = 0; f < 3; ++f)
    for (int g = 0; g < q; ++g) {
      const double xi = o.xg[g];
      rf.push_back(f == 0 ? xi : (f == 1 ? -xi : -1.0));
      sf.push_back(f == 0 ? -1.0 : (f == 1 ? xi : -xi));
    }
  std::vector<double> If;
  basis_at(ref, Vinv, rf, sf, If, o.Drf, o.Dsf);
  // the face-node part of face 0's rows: the 1D interpolation from the face
  // nodes (counter-clockwise) to the points, the same on every face
  o.If1.assign(q * Nfp, 0.0);
  for (int g = 0; g < q; ++g)
    for (int i = 0; i < Nfp; ++i) o.If1[g * Nfp + i] = If[g * Np + ref.Fmask[i]];
  const int NG = 3 * q;
  std::vector<double> LW(Np * NG), LrW(Np * NG), LsW(Np * NG);
  for (int i = 0; i < Np; ++i)
    for (int k = 0; k < NG; ++k) {
      const double w = o.wg[k % q];
      LW[i * NG + k] = If[k * Np + i] * w;
      LrW[i * NG + k] = o.Drf[k * Np + i] * w;
      LsW[i * NG + k] = o.Dsf[k * Np + i] * w;
    }
  o.LIFTq = matmul(Minv, LW, Np, Np, NG);
  o.LIFTrq = matmul(Minv, LrW, Np, Np, NG);
  o.LIFTsq = matmul(Minv, LsW, Np, Np, NG);
  return true;
}

void pack_oi(const RefOps& ref, const OIOps& o, std::vector<double>& out) {
  const int Np = ref.Np, Nq = o.Nq, NG = 3 * o.q;
  out.clear();
  // B operand of the 16x16x4 instruction: lane l of fragment (t, s) holds
  // Op[16 t + l % 16][4 s + l / 16] (rows = outputs, cols = the k index)
  auto emit = [&](const std::vector<double>& M, int rows, int cols) {
    const int nt = (rows + 15) / 16, ks = (cols + 3) / 4;
    for (int t = 0; t < nt; ++t)
      for (int s = 0; s < ks; ++s)
        for (int l = 0; l < 64; ++l) {
          int row = 16 * t + l % 16, col = 4 * s + l / 16;
          out.push_back((row < rows && col < cols) ? M[row * cols + col] : 0.0);
        }
  };
  emit(o.Iq, Nq, Np);
  emit(o.Drq, Nq, Np);
  emit(o.Dsq, Nq, Np);
  emit(o.Wr, Np, Nq);
  emit(o.Ws, Np, Nq);
  emit(o.LIFTq, Np, NG);
  emit(o.LIFTrq, Np, NG);
  emit(o.LIFTsq, Np, NG);
  for (int k = 0; k < NG; ++k)
    for (int j = 0; j < Np; ++j) {
      out.push_back(o.Drf[k * Np + j]);
      out.push_back(o.Dsf[k * Np + j]);
    }
  out.insert(out.end(), o.If1.begin(), o.If1.end());
}

namespace {
struct KeyHash {
  size_t operator()(const std::pair<int64_t, int64_t>& k) const {
    return std::hash<int64_t>()(k.first * 1000003LL) ^ std::hash<int64_t>()(k.second);
  }
};
}  // namespace

bool build_mesh_tables(const RefOps& ref, const Physics& ph, int64_t Nv, const double* VX,
                       const double* VY, int64_t K, const int32_t* EToV, const int8_t* face_tag,
                       const double period[2], MeshTables& t, std::string& err) {
  const int N = ref.N, Np = ref.Np, Nfp = ref.Nfp;
  char msg[256];
  t.K = K;
  t.geo.assign(K * kGeoStride, 0.0);
  t.nbr.assign(K * 3, -1);
  t.nbr_face.assign(K * 3, -1);
  t.tag.assign(K * 3, 0);
  t.conn.assign(K * 3, 0);
  t.x.assign(K * Np, 0.0);
  t.y.assign(K * Np, 0.0);
  t.wall_faces.clear();
  double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
  for (int64_t v = 0; v < Nv; ++v) {
    xmin = std::min(xmin, VX[v]);
    xmax = std::max(xmax, VX[v]);
    ymin = std::min(ymin, VY[v]);
    ymax = std::max(ymax, VY[v]);
  }
  const double scale = std::max({xmax - xmin, ymax - ymin, 1.0});
  const double tol = 1e-8 * scale;
  std::vector<double> Jv(K), sJ(K * 3), cx(K * 3), cy(K * 3);
  for (int64_t k = 0; k < K; ++k) {
    int32_t v[3] = {EToV[3 * k], EToV[3 * k + 1], EToV[3 * k + 2]};
    for (int c = 0; c < 3; ++c)
      if (v[c] < 0 || v[c] >= Nv) {
        std::snprintf(msg, sizeof msg, "element %lld has vertex index out of range", (long long)k);
        err = msg;
        return false;
      }
    double x1 = VX[v[0]], x2 = VX[v[1]], x3 = VX[v[2]];
    double y1 = VY[v[0]], y2 = VY[v[1]], y3 = VY[v[2]];
    double xr = 0.5 * (x2 - x1), xs = 0.5 * (x3 - x1), yr = 0.5 * (y2 - y1), ys = 0.5 * (y3 - y1);
    double J = xr * ys - xs * yr;
    if (!(J > 0.0)) {
      std::snprintf(msg, sizeof msg, "element %lld has J <= 0 (vertices not counter-clockwise)",
                    (long long)k);
      err = msg;
      return false;
    }
    Jv[k] = J;
    double* g = &t.geo[k * kGeoStride];
    g[0] = ys / J;   // rx
    g[1] = -xs / J;  // ry
    g[2] = -yr / J;  // sx
    g[3] = xr / J;   // sy
    double px[3] = {x1, x2, x3}, py[3] = {y1, y2, y3};
    for (int f = 0; f < 3; ++f) {
      double dx = px[(f + 1) % 3] - px[f], dy = py[(f + 1) % 3] - py[f];
      double len = std::sqrt(dx * dx + dy * dy);
      g[4 + 4 * f + 0] = dy / len;
      g[4 + 4 * f + 1] = -dx / len;
      sJ[k * 3 + f] = 0.5 * len;
      g[4 + 4 * f + 2] = 0.5 * len / J;  // Fscale = sJ / J
      cx[k * 3 + f] = 0.5 * (px[f] + px[(f + 1) % 3]);
      cy[k * 3 + f] = 0.5 * (py[f] + py[(f + 1) % 3]);
      int tg = face_tag ? face_tag[k * 3 + f] : 0;
      if (tg < 0 || tg > 2) {
        err = "face tag out of range";
        return false;
      }
      t.tag[k * 3 + f] = (int8_t)tg;
    }
    for (int n = 0; n < Np; ++n) {
      double r = ref.r[n], s = ref.s[n];
      t.x[k * Np + n] = 0.5 * (-(r + s) * x1 + (1.0 + r) * x2 + (1.0 + s) * x3);
      t.y[k * Np + n] = 0.5 * (-(r + s) * y1 + (1.0 + r) * y2 + (1.0 + s) * y3);
    }
  }
  // face pairing by wrapped face midpoint (covers shared vertices and periodic seams)
  const double px = period ? period[0] : 0.0, py = period ? period[1] : 0.0;
  auto wrap = [tol](double v, double per) {
    if (per <= 0.0) return v;
    double w = std::fmod(v, per);
    if (w < 0) w += per;
    if (std::fabs(w - per) < tol) w = 0.0;
    return w;
  };
  std::unordered_map<std::pair<int64_t, int64_t>, std::vector<int64_t>, KeyHash> table;
  std::vector<std::pair<int64_t, int64_t>> keys(K * 3);
  for (int64_t kf = 0; kf < K * 3; ++kf) {
    double wx = wrap(cx[kf], px), wy = wrap(cy[kf], py);
    keys[kf] = {(int64_t)std::llround(wx / tol), (int64_t)std::llround(wy / tol)};
    table[keys[kf]].push_back(kf);
  }
  for (int64_t kf = 0; kf < K * 3; ++kf) {
    int64_t k = kf / 3;
    int f = int(kf % 3);
    std::vector<int64_t> cand;
    for (int dk = -1; dk <= 1; ++dk)
      for (int dl = -1; dl <= 1; ++dl) {
        auto it = table.find({keys[kf].first + dk, keys[kf].second + dl});
        if (it == table.end()) continue;
        for (int64_t c : it->second)
          if (c != kf) cand.push_back(c);
      }
    if (t.tag[kf] != 0) {
      if (!cand.empty()) {
        std::snprintf(msg, sizeof msg, "boundary face (%lld,%d) is shared", (long long)k, f);
        err = msg;
        return false;
      }
      t.nbr[kf] = (int32_t)k;
      t.nbr_face[kf] = f;
      if (t.tag[kf] == 1) t.wall_faces.push_back((int32_t)kf);
      continue;
    }
    if (cand.size() != 1) {
      std::snprintf(msg, sizeof msg, "interior face (%lld,%d) has %d matching faces", (long long)k,
                    f, (int)cand.size());
      err = msg;
      return false;
    }
    int64_t kn = cand[0] / 3;
    int fn = int(cand[0] % 3);
    // the neighbour's face nodes must coincide with ours in reverse order
    // (conforming counter-clockwise elements; translation across a seam)
    double shx = cx[kf] - cx[cand[0]], shy = cy[kf] - cy[cand[0]];
    for (int j = 0; j < Nfp; ++j) {
      int a = ref.Fmask[f * Nfp + j], b = ref.Fmask[fn * Nfp + (Nfp - 1 - j)];
      double dx = t.x[k * Np + a] - t.x[kn * Np + b] - shx;
      double dy = t.y[k * Np + a] - t.y[kn * Np + b] - shy;
      if (std::sqrt(dx * dx + dy * dy) > tol) {
        std::snprintf(msg, sizeof msg, "face (%lld,%d) is not conforming with (%lld,%d)",
                      (long long)k, f, (long long)kn, fn);
        err = msg;
        return false;
      }
    }
    t.nbr[kf] = (int32_t)kn;
    t.nbr_face[kf] = fn;
  }
  // penalty geometric factor per face (sigma_e = sigma_geo * Gbar_e)
  for (int64_t k = 0; k < K; ++k) {
    for (int f = 0; f < 3; ++f) {
      int64_t kf = k * 3 + f;
      double fs_own = t.geo[k * kGeoStride + 4 + 4 * f + 2];
      double fs_nbr = fs_own;
      if (t.tag[kf] == 0) fs_nbr = t.geo[t.nbr[kf] * kGeoStride + 4 + 4 * t.nbr_face[kf] + 2];
      double fs_max = std::max(fs_own, fs_nbr);
      double sg;
      if (ph.penalty_mode == 0) {
        // C1 (1+theta)^2 (d+1) max C_inv, C_inv = Np |e| / |K| = Np Fscale
        sg = ph.C_pen * (1.0 + ph.theta) * (1.0 + ph.theta) * 3.0 * Np * fs_max;
      } else {
        // C (p+1)^2 / min h_e, h_e = 2|K|/|e| = 2 / Fscale
        sg = ph.C_pen * (N + 1) * (N + 1) * 0.5 * fs_max;
      }
      t.geo[k * kGeoStride + 4 + 4 * f + 3] = sg;
      t.conn[kf] = (t.nbr[kf] << 4) | (t.nbr_face[kf] << 2) | t.tag[kf];
    }
  }
  t.wall_xy.clear();
  for (int32_t kf : t.wall_faces) {
    int64_t k = kf / 3;
    int f = kf % 3;
    for (int j = 0; j < Nfp; ++j) {
      int n = ref.Fmask[f * Nfp + j];
      t.wall_xy.push_back(t.x[k * Np + n]);
      t.wall_xy.push_back(t.y[k * Np + n]);
    }
  }
  if (K >= (int64_t(1) << 27)) {
    err = "too many elements for the packed connectivity";
    return false;
  }
  return true;
}

void pack_ops(const RefOps& ref, std::vector<double>& out) {
  out.clear();
  out.insert(out.end(), ref.Dr.begin(), ref.Dr.end());
  out.insert(out.end(), ref.Ds.begin(), ref.Ds.end());
  out.insert(out.end(), ref.LIFT.begin(), ref.LIFT.end());
  out.insert(out.end(), ref.LIFTr.begin(), ref.LIFTr.end());
  out.insert(out.end(), ref.LIFTs.begin(), ref.LIFTs.end());
  out.insert(out.end(), ref.wface.begin(), ref.wface.end());
}

void pack_frags(const RefOps& ref, std::vector<double>& out) {
  const int Np = ref.Np, NF = 3 * ref.Nfp;
  const int NT = (Np + 15) / 16, KS = (Np + 3) / 4, KF = (NF + 3) / 4;
  out.clear();
  auto emit = [&](const std::vector<double>& M, int cols, int ksteps) {
    for (int t = 0; t < NT; ++t)
      for (int s = 0; s < ksteps; ++s)
        for (int l = 0; l < 64; ++l) {
          int row = 16 * t + l % 16, col = 4 * s + l / 16;
          out.push_back((row < Np && col < cols) ? M[row * cols + col] : 0.0);
        }
  };
  emit(ref.Dr, Np, KS);
  emit(ref.Ds, Np, KS);
  emit(ref.LIFT, NF, KF);
  emit(ref.LIFTr, NF, KF);
  emit(ref.LIFTs, NF, KF);
}

void pack_frags32(const RefOps& ref, std::vector<float>& out) {
  std::vector<double> d;
  pack_frags(ref, d);
  out.assign(d.begin(), d.end());
}

void pack_frags_bf16(const RefOps& ref, std::vector<uint16_t>& out) {
  const int Np = ref.Np, NF = 3 * ref.Nfp;
  const int NT = (Np + 15) / 16, KS = (Np + 15) / 16, KF = (NF + 15) / 16;
  out.clear();
  auto bf16 = [](double v) {
    float f = (float)v;
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
  };
  auto emit = [&](const std::vector<double>& M, int cols, int ksteps) {
    for (int t = 0; t < NT; ++t)
      for (int s = 0; s < ksteps; ++s)
        for (int l = 0; l < 64; ++l)
          for (int j = 0; j < 4; ++j) {
            const int row = 16 * t + l % 16, col = 16 * s + 4 * (l / 16) + j;
            out.push_back((row < Np && col < cols) ? bf16(M[row * cols + col]) : (uint16_t)0);
          }
  };
  emit(ref.Dr, Np, KS);
  emit(ref.Ds, Np, KS);
  emit(ref.LIFT, NF, KF);
  emit(ref.LIFTr, NF, KF);
  emit(ref.LIFTs, NF, KF);
}

// Helpers for the curved-element set-up (curved_setup.cpp).
void gauss_jacobi_rule(int q, double a, double b, std::vector<double>& x, std::vector<double>& w) {
  gauss_jacobi(q, a, b, x, w);
}

bool lagrange_at(const RefOps& ref, const std::vector<double>& r, const std::vector<double>& s,
                 std::vector<double>& L, std::vector<double>& Lr, std::vector<double>& Ls) {
  const int N = ref.N, Np = ref.Np;
  std::vector<double> V(Np * Np), vr(Np * Np), vs(Np * Np);
  for (int n = 0; n < Np; ++n) {
    int col = 0;
    for (int i = 0; i <= N; ++i)
      for (int j = 0; j <= N - i; ++j, ++col)
        pkd(ref.r[n], ref.s[n], i, j, V[n * Np + col], vr[n * Np + col], vs[n * Np + col]);
  }
  if (!invert(V, Np)) return false;
  basis_at(ref, V, r, s, L, Lr, Ls);
  return true;
}

bool invert_matrix(std::vector<double>& A, int n) { return invert(A, n); }

double legendre(double x, int n) { return jacobi(x, 0.0, 0.0, n); }
double dlegendre(double x, int n) { return djacobi(x, 0.0, 0.0, n); }

size_t ops_packed_size(int N) {
  size_t Np = (N + 1) * (N + 2) / 2, NF = 3 * (N + 1);
  return 2 * Np * Np + 3 * Np * NF + NF;
}

// Order-change maps between the nodal bases of orders lo < hi on the
// reference triangle.  P (Np_lo x Np_hi): the L2 projection onto degree <= lo
// (the orthonormal modal coefficients V_hi^-1 u truncated to the modes
// i + j <= lo), evaluated at the order-lo nodes.  I (Np_hi x Np_lo): the
// order-lo polynomial evaluated at the order-hi nodes.
bool build_order_maps(int lo, int hi, std::vector<double>& P, std::vector<double>& I,
                      std::string& err) {
  if (lo < 1 || hi <= lo || hi > kMaxOrder) {
    err = "orders must satisfy 1 <= lo < hi <= 8";
    return false;
  }
  const int nl = (lo + 1) * (lo + 2) / 2, nh = (hi + 1) * (hi + 2) / 2;
  std::vector<double> rl, sl, rh, sh;
  warp_blend_nodes(lo, rl, sl);
  warp_blend_nodes(hi, rh, sh);
  auto vander = [](int N, const std::vector<double>& r, const std::vector<double>& s, int maxdeg,
                   int& ncol) {
    std::vector<double> V;
    const int n = (int)r.size();
    ncol = 0;
    for (int i = 0; i <= N; ++i)
      for (int j = 0; j <= N - i; ++j)
        if (i + j <= maxdeg) ++ncol;
    V.assign((size_t)n * ncol, 0.0);
    for (int m = 0; m < n; ++m) {
      int col = 0;
      for (int i = 0; i <= N; ++i)
        for (int j = 0; j <= N - i; ++j) {
          if (i + j > maxdeg) continue;
          double v, dr, ds;
          pkd(r[m], s[m], i, j, v, dr, ds);
          V[(size_t)m * ncol + col++] = v;
        }
    }
    return V;
  };
  int c;
  std::vector<double> Vh = vander(hi, rh, sh, hi, c);
  if (!invert(Vh, nh)) {
    err = "singular Vandermonde matrix";
    return false;
  }
  // rows of V_hi^-1 of the kept modes, in mode order
  std::vector<double> keep_rows;
  {
    int row = 0;
    for (int i = 0; i <= hi; ++i)
      for (int j = 0; j <= hi - i; ++j, ++row)
        if (i + j <= lo) keep_rows.insert(keep_rows.end(), Vh.begin() + (size_t)row * nh,
                                          Vh.begin() + (size_t)(row + 1) * nh);
  }
  // the kept order-hi modes are the order-lo modes (same (i, j), same order)
  std::vector<double> Psi_l = vander(hi, rl, sl, lo, c);  // nl x nl
  P = matmul(Psi_l, keep_rows, nl, nl, nh);
  std::vector<double> Vl = vander(lo, rl, sl, lo, c);
  if (!invert(Vl, nl)) {
    err = "singular Vandermonde matrix";
    return false;
  }
  std::vector<double> Psi_h = vander(lo, rh, sh, lo, c);  // nh x nl
  I = matmul(Psi_h, Vl, nh, nl, nl);
  return true;
}

}  // namespace dgmi
