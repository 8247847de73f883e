// Pointwise physics of the 2D compressible Navier-Stokes system, device side.
//
// State U = [rho, m1, m2, eps] (m = rho v, eps = total energy per volume),
// p = (gamma-1)(eps - |m|^2/(2 rho)) (Sec. 2.1; the printed equation of state
// is garbled, this form is the one the printed (4,1) entries of the viscous
// blocks require).  The viscous flux is applied through the paper's four
// 4x4 blocks G11, G12, G21, G22 (Sec. 2.1), written out with their zero
// pattern through a factorisation (below); the theta term needs their
// transposes, and the penalty's diffusion scale needs ||n^T G n||_2
// (Sec. 2.2.3).
#pragma once

#include <hip/hip_runtime.h>

namespace dgmi {

struct Gas {
  double gamma, gm1, igm1, mu, k;  // igm1 = 1/(gamma-1), k = gamma / Pr
};

__device__ __forceinline__ double pressure(const double U[4], double ir, double gm1) {
  return gm1 * (U[3] - 0.5 * (U[1] * U[1] + U[2] * U[2]) * ir);
}

// Per-state quantities shared by the viscous operators: 1/rho, velocity,
// mu/rho, eps/rho - |v|^2 and the (4,1) entries of G11 and G22.
struct VState {
  double ir, v1, v2, m, ek, g41a, g41b;
};

__device__ __forceinline__ VState vstate(const Gas& g, const double U[4]) {
  VState s;
  s.ir = 1.0 / U[0];
  s.v1 = U[1] * s.ir;
  s.v2 = U[2] * s.ir;
  s.m = g.mu * s.ir;
  const double vv = s.v1 * s.v1 + s.v2 * s.v2;
  s.ek = U[3] * s.ir - vv;  // eps/rho - |v|^2, as in the printed (4,1) entries
  s.g41a = -s.v1 * s.v1 * (1.0 / 3.0) - vv - g.k * s.ek;
  s.g41b = -s.v2 * s.v2 * (1.0 / 3.0) - vv - g.k * s.ek;
  return s;
}

// F_c,x, F_c,y minus the moving-frame term v_w (x) U, dotted with n:
// the advective flux through a face of normal n.
__device__ __forceinline__ void normal_adv_flux(const double U[4], double ir, double nx, double ny,
                                                double vwn, double gm1, double F[4]) {
  double u = U[1] * ir, v = U[2] * ir;
  double p = gm1 * (U[3] - 0.5 * (U[1] * u + U[2] * v));
  double qn = u * nx + v * ny - vwn;
  F[0] = U[0] * qn;
  F[1] = U[1] * qn + p * nx;
  F[2] = U[2] * qn + p * ny;
  F[3] = U[3] * qn + p * (u * nx + v * ny);
}

// The printed blocks factor as G_ab = (mu/rho) C_ab T with the same 3x4 map
// T = [[-v1, 1, 0, 0], [-v2, 0, 1, 0], [-ek, -v1, -v2, 1]] in both directions:
// T d_a U = rho (d_a v1, d_a v2, d_a e) (ek = eps/rho - |v|^2), and C_ab the
// constant-coefficient stress / heat-flux weights.  Both operators below use
// that factorisation; expanding it reproduces every printed entry.
//
// F_v = G(U) grad U: Fx = G11 dUx + G12 dUy, Fy = G21 dUx + G22 dUy.
__device__ __forceinline__ void viscous_flux(const Gas& g, const VState& st, const double dx[4],
                                             const double dy[4], double Fx[4], double Fy[4]) {
  const double v1 = st.v1, v2 = st.v2, m = st.m, k = g.k;
  const double c43 = 4.0 / 3.0, c23 = 2.0 / 3.0;
  // rho-scaled primitive gradients T dU
  const double ux = dx[1] - v1 * dx[0], vx = dx[2] - v2 * dx[0];
  const double uy = dy[1] - v1 * dy[0], vy = dy[2] - v2 * dy[0];
  const double ex = dx[3] - st.ek * dx[0] - v1 * dx[1] - v2 * dx[2];
  const double ey = dy[3] - st.ek * dy[0] - v1 * dy[1] - v2 * dy[2];
  const double txx = c43 * ux - c23 * vy, tyy = c43 * vy - c23 * ux, txy = uy + vx;
  Fx[0] = 0.0;
  Fx[1] = m * txx;
  Fx[2] = m * txy;
  Fx[3] = m * (v1 * txx + v2 * txy + k * ex);
  Fy[0] = 0.0;
  Fy[1] = m * txy;
  Fy[2] = m * tyy;
  Fy[3] = m * (v1 * txy + v2 * tyy + k * ey);
}

// q = G(U)^T (n (x) w) = (mu/rho) (T^T z_x, T^T z_y) with z = C^T (n (x) w):
// qx = nx G11^T w + ny G21^T w, qy = nx G12^T w + ny G22^T w.
__device__ __forceinline__ void viscous_transpose(const Gas& g, const VState& st, double nx,
                                                  double ny, const double w[4], double qx[4],
                                                  double qy[4]) {
  const double v1 = st.v1, v2 = st.v2, m = st.m, k = g.k;
  const double c43 = 4.0 / 3.0, c23 = 2.0 / 3.0;
  const double W1 = w[1] + v1 * w[3], W2 = w[2] + v2 * w[3];
  const double sxy = nx * W2 + ny * W1;
  // weights of the rho-scaled primitive gradients (u, v, e) in x and in y
  const double zux = c43 * nx * W1 - c23 * ny * W2, zvx = sxy, zex = k * nx * w[3];
  const double zuy = sxy, zvy = c43 * ny * W2 - c23 * nx * W1, zey = k * ny * w[3];
  qx[0] = m * (-v1 * zux - v2 * zvx - st.ek * zex);
  qx[1] = m * (zux - v1 * zex);
  qx[2] = m * (zvx - v2 * zex);
  qx[3] = m * zex;
  qy[0] = m * (-v1 * zuy - v2 * zvy - st.ek * zey);
  qy[1] = m * (zuy - v1 * zey);
  qy[2] = m * (zvy - v2 * zey);
  qy[3] = m * zey;
}

// Largest eigenvalue of a symmetric 3x3 matrix by the closed-form
// trigonometric solution of its characteristic cubic.
__device__ __noinline__ double sym3_lambda_max_trig(double s00, double s11, double s22,
                                                       double s01, double s02, double s12) {
  double q = (s00 + s11 + s22) * (1.0 / 3.0);
  double p1 = s01 * s01 + s02 * s02 + s12 * s12;
  double d0 = s00 - q, d1 = s11 - q, d2 = s22 - q;
  double p2 = d0 * d0 + d1 * d1 + d2 * d2 + 2.0 * p1;
  if (p2 <= 0.0) return q;
  double pp = sqrt(p2 * (1.0 / 6.0));
  double ip = 1.0 / pp;
  double b00 = d0 * ip, b11 = d1 * ip, b22 = d2 * ip;
  double b01 = s01 * ip, b02 = s02 * ip, b12 = s12 * ip;
  double det = b00 * (b11 * b22 - b12 * b12) - b01 * (b01 * b22 - b12 * b02) +
               b02 * (b01 * b12 - b11 * b02);
  double r = 0.5 * det;
  r = r < -1.0 ? -1.0 : (r > 1.0 ? 1.0 : r);
  return q + 2.0 * pp * cos(acos(r) * (1.0 / 3.0));
}

// ||A||_2 for A = nx^2 G11 + nx ny (G12 + G21) + ny^2 G22.  The first row of
// A is zero, so ||A||_2 = (mu/rho) sqrt(lambda_max(B B^T)) for the 3x4 block B
// of its lower rows.  lambda_max of the symmetric positive semi-definite
// S = B B^T: Newton on its characteristic cubic from the Frobenius norm of S,
// an upper bound within a few per cent of lambda_max when the top eigenvalue
// is well separated (iterates decrease monotonically to the largest root).
// If the last step is not negligible -- a near-double top eigenvalue, where
// Newton converges only linearly -- the closed-form trigonometric solution is
// used instead.
__device__ __forceinline__ double normal_diffusion_norm(const Gas& g, const VState& st, double nx,
                                                        double ny) {
  const double v1 = st.v1, v2 = st.v2, k = g.k;
  const double c43 = 4.0 / 3.0, c23 = 2.0 / 3.0, c13 = 1.0 / 3.0;
  double xx = nx * nx, xy = nx * ny, yy = ny * ny;
  // rows of B (the fourth column of the momentum rows is zero)
  double a0 = -(c43 * xx + yy) * v1 - c13 * xy * v2, a1 = c43 * xx + yy, a2 = c13 * xy;
  double b0 = -(xx + c43 * yy) * v2 - c13 * xy * v1, b1 = c13 * xy, b2 = xx + c43 * yy;
  double e0 = xx * st.g41a + yy * st.g41b - c23 * xy * v1 * v2;
  double e1 = (c43 - k) * v1 * xx + c13 * v2 * xy + (1.0 - k) * v1 * yy;
  double e2 = (1.0 - k) * v2 * xx + c13 * v1 * xy + (c43 - k) * v2 * yy;
  double e3 = k * (xx + yy);
  double s00 = a0 * a0 + a1 * a1 + a2 * a2;
  double s11 = b0 * b0 + b1 * b1 + b2 * b2;
  double s22 = e0 * e0 + e1 * e1 + e2 * e2 + e3 * e3;
  double s01 = a0 * b0 + a1 * b1 + a2 * b2;
  double s02 = a0 * e0 + a1 * e1 + a2 * e2;
  double s12 = b0 * e0 + b1 * e1 + b2 * e2;
  // characteristic polynomial lambda^3 - c2 lambda^2 + c1 lambda - c0
  double c2 = s00 + s11 + s22;
  double c1 = s00 * s11 + s00 * s22 + s11 * s22 - s01 * s01 - s02 * s02 - s12 * s12;
  double c0 = s00 * (s11 * s22 - s12 * s12) - s01 * (s01 * s22 - s12 * s02) +
              s02 * (s01 * s12 - s11 * s02);
  double lam = sqrt(s00 * s00 + s11 * s11 + s22 * s22 +
                    2.0 * (s01 * s01 + s02 * s02 + s12 * s12));
  double step = 0.0;
#pragma unroll
  for (int it = 0; it < 5; ++it) {
    double f = ((lam - c2) * lam + c1) * lam - c0;
    double df = (3.0 * lam - 2.0 * c2) * lam + c1;
    // the step only needs an approximate reciprocal: Newton corrects the rest
    double r = __builtin_amdgcn_rcp(df);
    r = r * (2.0 - df * r);
    step = (df > 0.0) ? f * r : 0.0;
    lam -= step;
  }
  if (!(fabs(step) <= 1e-15 * lam)) lam = sym3_lambda_max_trig(s00, s11, s22, s01, s02, s12);
  return st.m * sqrt(lam > 0.0 ? lam : 0.0);
}

// Roe flux, own state Ul ("+"), other state Ur ("-"), own outward normal n,
// moving frame: mean normal flux + (1/2)|A~ - (v_w.n) I|(Ul - Ur), with the
// dissipation in wave-strength form (Roe averages of velocity and total
// enthalpy; eigenvalues (v~.n - v_w.n) and (v~.n - v_w.n) +- c~).
__device__ __forceinline__ void roe_flux(const double Ul[4], double irl, const double Ur[4],
                                         double irr, double nx, double ny, double vwn, double gm1,
                                         double F[4]) {
  double fl[4], fr[4];
  normal_adv_flux(Ul, irl, nx, ny, vwn, gm1, fl);
  normal_adv_flux(Ur, irr, nx, ny, vwn, gm1, fr);
  double ul = Ul[1] * irl, vl = Ul[2] * irl, ur = Ur[1] * irr, vr = Ur[2] * irr;
  double pl = gm1 * (Ul[3] - 0.5 * (Ul[1] * ul + Ul[2] * vl));
  double pr = gm1 * (Ur[3] - 0.5 * (Ur[1] * ur + Ur[2] * vr));
  double hl = (Ul[3] + pl) * irl, hr = (Ur[3] + pr) * irr;
  double sl = sqrt(Ul[0]), sr = sqrt(Ur[0]);
  double iw = 1.0 / (sl + sr);
  double rt = sl * sr;
  double ut = (sl * ul + sr * ur) * iw, vt = (sl * vl + sr * vr) * iw;
  double ht = (sl * hl + sr * hr) * iw;
  double c2 = gm1 * (ht - 0.5 * (ut * ut + vt * vt));
  double ct = sqrt(c2);
  double qn = ut * nx + vt * ny, qt = -ut * ny + vt * nx;
  // jumps taken as (other - own)
  double dr = Ur[0] - Ul[0], dp = pr - pl;
  double dqn = (ur - ul) * nx + (vr - vl) * ny;
  double dqt = -(ur - ul) * ny + (vr - vl) * nx;
  double ic2 = 1.0 / c2;
  double a1 = 0.5 * (dp - rt * ct * dqn) * ic2;
  double a2 = dr - dp * ic2;
  double a3 = rt * dqt;
  double a4 = 0.5 * (dp + rt * ct * dqn) * ic2;
  double l1 = fabs(qn - ct - vwn), l2 = fabs(qn - vwn), l4 = fabs(qn + ct - vwn);
  double w1 = l1 * a1, w2 = l2 * a2, w3 = l2 * a3, w4 = l4 * a4;
  double d0 = w1 + w2 + w4;
  double d1 = w1 * (ut - ct * nx) + w2 * ut - w3 * ny + w4 * (ut + ct * nx);
  double d2 = w1 * (vt - ct * ny) + w2 * vt + w3 * nx + w4 * (vt + ct * ny);
  double d3 = w1 * (ht - ct * qn) + w2 * 0.5 * (ut * ut + vt * vt) + w3 * qt + w4 * (ht + ct * qn);
  F[0] = 0.5 * (fl[0] + fr[0] - d0);
  F[1] = 0.5 * (fl[1] + fr[1] - d1);
  F[2] = 0.5 * (fl[2] + fr[2] - d2);
  F[3] = 0.5 * (fl[3] + fr[3] - d3);
}

}  // namespace dgmi
