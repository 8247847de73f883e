// Pointwise physics of the 2D compressible Navier-Stokes system, device side.
//
// State U = [rho, m1, m2, eps] (m = rho v, eps = total energy per volume),
// p = (gamma-1)(eps - |m|^2/(2 rho)) (Sec. 2.1; the printed equation of state
// is garbled, this form is the one the printed (4,1) entries of the viscous
// blocks require).  The viscous flux is applied through the paper's four
// 4x4 blocks G11, G12, G21, G22 (Sec. 2.1), written out with their zero
// pattern; the theta term needs their transposes, and the penalty's
// diffusion scale needs ||n^T G n||_2 (Sec. 2.2.3).
#pragma once

#include <hip/hip_runtime.h>

namespace dgmi {

struct Gas {
  double gamma, gm1, mu, k;  // k = gamma / Pr
};

__device__ __forceinline__ double pressure(const double U[4], double gm1) {
  return gm1 * (U[3] - 0.5 * (U[1] * U[1] + U[2] * U[2]) / U[0]);
}

// F_c,x, F_c,y minus the moving-frame term v_w (x) U, dotted with n:
// the advective flux through a face of normal n.
__device__ __forceinline__ void normal_adv_flux(const double U[4], double nx, double ny, double vwn,
                                                double gm1, double F[4]) {
  double ir = 1.0 / U[0];
  double u = U[1] * ir, v = U[2] * ir;
  double p = gm1 * (U[3] - 0.5 * (U[1] * u + U[2] * v));
  double qn = u * nx + v * ny - vwn;
  F[0] = U[0] * qn;
  F[1] = U[1] * qn + p * nx;
  F[2] = U[2] * qn + p * ny;
  F[3] = U[3] * qn + p * (u * nx + v * ny);
}

// F_v = G(U) grad U via the printed blocks: Fx = G11 dUx + G12 dUy,
// Fy = G21 dUx + G22 dUy (first rows of every block are zero).
__device__ __forceinline__ void viscous_flux(const Gas& g, const double U[4], const double dx[4],
                                             const double dy[4], double Fx[4], double Fy[4]) {
  double ir = 1.0 / U[0];
  double v1 = U[1] * ir, v2 = U[2] * ir;
  double m = g.mu * ir, k = g.k;
  double vv = v1 * v1 + v2 * v2;
  double ek = U[3] * ir - vv;  // eps/rho - |v|^2, as in the printed (4,1) entries
  double g41a = -v1 * v1 * (1.0 / 3.0) - vv - k * ek;
  double g41b = -v2 * v2 * (1.0 / 3.0) - vv - k * ek;
  const double c43 = 4.0 / 3.0, c23 = 2.0 / 3.0, c13 = 1.0 / 3.0;
  double txx = -c43 * v1 * dx[0] + c43 * dx[1] + c23 * v2 * dy[0] - c23 * dy[2];
  double txy = -v2 * dx[0] + dx[2] - v1 * dy[0] + dy[1];
  double tyy = c23 * v1 * dx[0] - c23 * dx[1] - c43 * v2 * dy[0] + c43 * dy[2];
  double ex = g41a * dx[0] + (c43 - k) * v1 * dx[1] + (1.0 - k) * v2 * dx[2] + k * dx[3] -
              c13 * v1 * v2 * dy[0] + v2 * dy[1] - c23 * v1 * dy[2];
  double ey = -c13 * v1 * v2 * dx[0] - c23 * v2 * dx[1] + v1 * dx[2] + g41b * dy[0] +
              (1.0 - k) * v1 * dy[1] + (c43 - k) * v2 * dy[2] + k * dy[3];
  Fx[0] = 0.0;
  Fx[1] = m * txx;
  Fx[2] = m * txy;
  Fx[3] = m * ex;
  Fy[0] = 0.0;
  Fy[1] = m * txy;
  Fy[2] = m * tyy;
  Fy[3] = m * ey;
}

// q = G(U)^T (n (x) w): qx = nx G11^T w + ny G21^T w, qy = nx G12^T w + ny G22^T w.
__device__ __forceinline__ void viscous_transpose(const Gas& g, const double U[4], double nx,
                                                  double ny, const double w[4], double qx[4],
                                                  double qy[4]) {
  double ir = 1.0 / U[0];
  double v1 = U[1] * ir, v2 = U[2] * ir;
  double m = g.mu * ir, k = g.k;
  double vv = v1 * v1 + v2 * v2;
  double ek = U[3] * ir - vv;  // eps/rho - |v|^2, as in the printed (4,1) entries
  double g41a = -v1 * v1 * (1.0 / 3.0) - vv - k * ek;
  double g41b = -v2 * v2 * (1.0 / 3.0) - vv - k * ek;
  const double c43 = 4.0 / 3.0, c23 = 2.0 / 3.0, c13 = 1.0 / 3.0;
  double w1 = w[1], w2 = w[2], w3 = w[3];
  // G11^T w, G21^T w, G12^T w, G22^T w (component 3 of G21^T, G12^T is zero)
  double a0 = -c43 * v1 * w1 - v2 * w2 + g41a * w3, a1 = c43 * w1 + (c43 - k) * v1 * w3,
         a2 = w2 + (1.0 - k) * v2 * w3, a3 = k * w3;
  double b0 = -v2 * w1 + c23 * v1 * w2 - c13 * v1 * v2 * w3, b1 = -c23 * w2 - c23 * v2 * w3,
         b2 = w1 + v1 * w3;
  double c0 = c23 * v2 * w1 - v1 * w2 - c13 * v1 * v2 * w3, c1 = w2 + v2 * w3,
         c2 = -c23 * w1 - c23 * v1 * w3;
  double d0 = -v1 * w1 - c43 * v2 * w2 + g41b * w3, d1 = w1 + (1.0 - k) * v1 * w3,
         d2 = c43 * w2 + (c43 - k) * v2 * w3, d3 = k * w3;
  qx[0] = m * (nx * a0 + ny * b0);
  qx[1] = m * (nx * a1 + ny * b1);
  qx[2] = m * (nx * a2 + ny * b2);
  qx[3] = m * (nx * a3);
  qy[0] = m * (nx * c0 + ny * d0);
  qy[1] = m * (nx * c1 + ny * d1);
  qy[2] = m * (nx * c2 + ny * d2);
  qy[3] = m * (ny * d3);
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
__device__ __forceinline__ double normal_diffusion_norm(const Gas& g, const double U[4], double nx,
                                                        double ny) {
  double ir = 1.0 / U[0];
  double v1 = U[1] * ir, v2 = U[2] * ir;
  double k = g.k;
  double vv = v1 * v1 + v2 * v2;
  double ek = U[3] * ir - vv;  // eps/rho - |v|^2, as in the printed (4,1) entries
  double g41a = -v1 * v1 * (1.0 / 3.0) - vv - k * ek;
  double g41b = -v2 * v2 * (1.0 / 3.0) - vv - k * ek;
  const double c43 = 4.0 / 3.0, c23 = 2.0 / 3.0, c13 = 1.0 / 3.0;
  double xx = nx * nx, xy = nx * ny, yy = ny * ny;
  // rows of B (the fourth column of the momentum rows is zero)
  double a0 = -(c43 * xx + yy) * v1 - c13 * xy * v2, a1 = c43 * xx + yy, a2 = c13 * xy;
  double b0 = -(xx + c43 * yy) * v2 - c13 * xy * v1, b1 = c13 * xy, b2 = xx + c43 * yy;
  double e0 = xx * g41a + yy * g41b - c23 * xy * v1 * v2;
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
  for (int it = 0; it < 6; ++it) {
    double f = ((lam - c2) * lam + c1) * lam - c0;
    double df = (3.0 * lam - 2.0 * c2) * lam + c1;
    step = (df > 0.0) ? f / df : 0.0;
    lam -= step;
  }
  if (!(fabs(step) <= 1e-15 * lam)) lam = sym3_lambda_max_trig(s00, s11, s22, s01, s02, s12);
  return g.mu * ir * sqrt(lam > 0.0 ? lam : 0.0);
}

// Roe flux, own state Ul ("+"), other state Ur ("-"), own outward normal n,
// moving frame: mean normal flux + (1/2)|A~ - (v_w.n) I|(Ul - Ur), with the
// dissipation in wave-strength form (Roe averages of velocity and total
// enthalpy; eigenvalues (v~.n - v_w.n) and (v~.n - v_w.n) +- c~).
__device__ __forceinline__ void roe_flux(const double Ul[4], const double Ur[4], double nx,
                                         double ny, double vwn, double gm1, double F[4]) {
  double fl[4], fr[4];
  normal_adv_flux(Ul, nx, ny, vwn, gm1, fl);
  normal_adv_flux(Ur, nx, ny, vwn, gm1, fr);
  double irl = 1.0 / Ul[0], irr = 1.0 / Ur[0];
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
