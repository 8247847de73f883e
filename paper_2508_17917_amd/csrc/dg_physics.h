// Pointwise physics of the 2D compressible Navier-Stokes system, device side,
// for a real type T (double, or float in the perturbation form).
//
// State U = [rho, m1, m2, eps] (m = rho v, eps = total energy per volume),
// p = (gamma-1)(eps - |m|^2/(2 rho)) (Sec. 2.1; the printed equation of state
// is garbled, this form is the one the printed (4,1) entries of the viscous
// blocks require).  The viscous flux is applied through the paper's four
// 4x4 blocks G11, G12, G21, G22 (Sec. 2.1) via a factorisation (below); the
// theta term needs their transposes, and the penalty's diffusion scale needs
// ||n^T G n||_2 (Sec. 2.2.3).
//
// Perturbation form: with U = U_inf + U', every advective flux is evaluated
// as F(U_inf + U') - F(U_inf) written without cancellation (differences of
// O(1) quantities are formed algebraically from the perturbations), so that
// a low-Mach perturbation keeps its relative precision in FP32.  The
// constant F(U_inf) drops out of the divergence and of every face term (the
// Roe flux of (U_inf, U_inf) is F_n(U_inf)); gradients are those of U'.
#pragma once

#include <hip/hip_runtime.h>

namespace dgmi {

template <typename T>
struct Gas {
  T gamma, gm1, igm1, mu, k;  // igm1 = 1/(gamma-1), k = gamma / Pr
};

// The gas as seen by the viscous terms of a wall face: the same stress, and
// the conduction k_wall -- 0 for the adiabatic wall (Sec. 2.2.4: Neumann
// conditions on pressure and temperature there), so that neither the wall's
// viscous flux nor its theta term carries heat through the wall; gamma / Pr
// for the printed wall flux G(U^b) grad U+.
template <typename T>
__device__ __forceinline__ Gas<T> gas_wall(const Gas<T>& g, T k_wall) {
  Gas<T> w = g;
  w.k = k_wall;
  return w;
}

// Free-stream quantities used by the perturbation form.
template <typename T>
struct Base {
  T rho, mx, my, E, p, ux, uy;
};

template <typename T>
__device__ __forceinline__ T rcp_approx(T x);
template <>
__device__ __forceinline__ double rcp_approx<double>(double x) {
  return __builtin_amdgcn_rcp(x);
}
template <>
__device__ __forceinline__ float rcp_approx<float>(float x) {
  return __builtin_amdgcn_rcpf(x);
}

// Reciprocal and square root at the accuracy each real type needs: binary64
// from the hardware reciprocal estimate refined by two Newton steps (within
// about 1 ulp: far inside the FP64 parity bound, and cheaper than the
// correctly rounded division); binary32 with the single hardware
// instructions (1 ulp).
template <typename T>
__device__ __forceinline__ T rcp(T x);
template <>
__device__ __forceinline__ double rcp<double>(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}
template <>
__device__ __forceinline__ float rcp<float>(float x) {
  return __builtin_amdgcn_rcpf(x);
}
template <typename T>
__device__ __forceinline__ T root(T x);
template <>
__device__ __forceinline__ double root<double>(double x) {
  return sqrt(x);
}
template <>
__device__ __forceinline__ float root<float>(float x) {
  return __builtin_amdgcn_sqrtf(x);
}

// Primitive view of one face state.  rho, u, v, p, H are the full state
// (Roe averages, eigenvalues); jr, ju, jv, jp are what jumps are taken of:
// the full values in the plain form, the perturbations in the perturbation
// form (U_inf cancels from every jump either way).
template <typename T>
struct Prim {
  T rho, ir, u, v, p, H;
  T jr, ju, jv, jp;
};

// Plain form: full state U.
template <typename T>
__device__ __forceinline__ Prim<T> prim_plain(const T U[4], T gm1) {
  Prim<T> s;
  s.rho = U[0];
  s.ir = rcp(U[0]);
  s.u = U[1] * s.ir;
  s.v = U[2] * s.ir;
  s.p = gm1 * (U[3] - T(0.5) * (U[1] * s.u + U[2] * s.v));
  s.H = (U[3] + s.p) * s.ir;
  s.jr = s.rho;
  s.ju = s.u;
  s.jv = s.v;
  s.jp = s.p;
  return s;
}

// Perturbation form: full state Uf = U_inf + Ud and the perturbation Ud.
template <typename T>
__device__ __forceinline__ Prim<T> prim_pert(const T Uf[4], const T Ud[4], const Base<T>& b,
                                             T gm1) {
  Prim<T> s;
  s.rho = Uf[0];
  s.ir = rcp(Uf[0]);
  s.u = Uf[1] * s.ir;
  s.v = Uf[2] * s.ir;
  // u' = (m' - rho' u0) / rho; kinetic-energy perturbation from products of
  // perturbation-sized terms
  s.ju = (Ud[1] - Ud[0] * b.ux) * s.ir;
  s.jv = (Ud[2] - Ud[0] * b.uy) * s.ir;
  const T dke = T(0.5) * (b.mx * s.ju + b.my * s.jv + Ud[1] * b.ux + Ud[2] * b.uy + Ud[1] * s.ju +
                          Ud[2] * s.jv);
  s.jp = gm1 * (Ud[3] - dke);
  s.jr = Ud[0];
  s.p = b.p + s.jp;
  s.H = (Uf[3] + s.p) * s.ir;
  return s;
}

// Advective flux through a face of normal n in the moving frame,
// N (F_c(U) - v_w (x) U).  Plain form: of the full state.
template <typename T>
__device__ __forceinline__ void normal_flux_plain(const T U[4], const Prim<T>& s, T nx, T ny, T vwn,
                                                  T F[4]) {
  const T un = s.u * nx + s.v * ny;
  const T qn = un - vwn;
  F[0] = U[0] * qn;
  F[1] = U[1] * qn + s.p * nx;
  F[2] = U[2] * qn + s.p * ny;
  F[3] = U[3] * qn + s.p * un;
}

// Perturbation form: N(F_c(U) - v_w U) - N(F_c(U_inf) - v_w U_inf), from the
// perturbation Ud and the primitive view s (s.ju, s.jv, s.jp = u', v', p').
template <typename T>
__device__ __forceinline__ void normal_flux_pert(const T Ud[4], const Prim<T>& s, const Base<T>& b,
                                                 T nx, T ny, T vwn, T F[4]) {
  const T qnd = s.ju * nx + s.jv * ny;  // (u - u0).n
  const T q0n = b.ux * nx + b.uy * ny;  // u0.n
  const T Ep = Ud[3] + s.jp;            // (eps + p)'
  F[0] = Ud[1] * nx + Ud[2] * ny - vwn * Ud[0];
  F[1] = b.mx * qnd + Ud[1] * (q0n + qnd) + s.jp * nx - vwn * Ud[1];
  F[2] = b.my * qnd + Ud[2] * (q0n + qnd) + s.jp * ny - vwn * Ud[2];
  F[3] = qnd * (b.E + b.p) + Ep * (q0n + qnd) - vwn * Ud[3];
}

// Per-state quantities shared by the viscous operators: 1/rho, velocity,
// mu/rho and eps/rho - |v|^2.
template <typename T>
struct VState {
  T ir, v1, v2, m, ek;
};

template <typename T>
__device__ __forceinline__ VState<T> vstate(const Gas<T>& g, const T U[4]) {
  VState<T> s;
  s.ir = rcp(U[0]);
  s.v1 = U[1] * s.ir;
  s.v2 = U[2] * s.ir;
  s.m = g.mu * s.ir;
  const T vv = s.v1 * s.v1 + s.v2 * s.v2;
  s.ek = U[3] * s.ir - vv;  // eps/rho - |v|^2, as in the printed (4,1) entries
  return s;
}

// The printed blocks factor as G_ab = (mu/rho) C_ab T with the same 3x4 map
// T = [[-v1, 1, 0, 0], [-v2, 0, 1, 0], [-ek, -v1, -v2, 1]] in both directions:
// T d_a U = rho (d_a v1, d_a v2, d_a e) (ek = eps/rho - |v|^2), and C_ab the
// constant-coefficient stress / heat-flux weights.  Both operators below use
// that factorisation; expanding it reproduces every printed entry.
//
// F_v = G(U) grad U: Fx = G11 dUx + G12 dUy, Fy = G21 dUx + G22 dUy.
template <typename T>
__device__ __forceinline__ void viscous_flux(const Gas<T>& g, const VState<T>& st, const T dx[4],
                                             const T dy[4], T Fx[4], T Fy[4]) {
  const T v1 = st.v1, v2 = st.v2, m = st.m, k = g.k;
  const T c43 = T(4.0 / 3.0), c23 = T(2.0 / 3.0);
  // rho-scaled primitive gradients T dU
  const T ux = dx[1] - v1 * dx[0], vx = dx[2] - v2 * dx[0];
  const T uy = dy[1] - v1 * dy[0], vy = dy[2] - v2 * dy[0];
  const T ex = dx[3] - st.ek * dx[0] - v1 * dx[1] - v2 * dx[2];
  const T ey = dy[3] - st.ek * dy[0] - v1 * dy[1] - v2 * dy[2];
  const T txx = c43 * ux - c23 * vy, tyy = c43 * vy - c23 * ux, txy = uy + vx;
  Fx[0] = T(0);
  Fx[1] = m * txx;
  Fx[2] = m * txy;
  Fx[3] = m * (v1 * txx + v2 * txy + k * ex);
  Fy[0] = T(0);
  Fy[1] = m * txy;
  Fy[2] = m * tyy;
  Fy[3] = m * (v1 * txy + v2 * tyy + k * ey);
}

// The same flux projected on n: Fn = Fx nx + Fy ny, formed from the normal
// stress and heat-flux components directly.
template <typename T>
__device__ __forceinline__ void viscous_normal_flux(const Gas<T>& g, const VState<T>& st,
                                                    const T dx[4], const T dy[4], T nx, T ny,
                                                    T Fn[4]) {
  const T v1 = st.v1, v2 = st.v2, m = st.m, k = g.k;
  const T c43 = T(4.0 / 3.0), c23 = T(2.0 / 3.0);
  const T ux = dx[1] - v1 * dx[0], vx = dx[2] - v2 * dx[0];
  const T uy = dy[1] - v1 * dy[0], vy = dy[2] - v2 * dy[0];
  const T ex = dx[3] - st.ek * dx[0] - v1 * dx[1] - v2 * dx[2];
  const T ey = dy[3] - st.ek * dy[0] - v1 * dy[1] - v2 * dy[2];
  const T txx = c43 * ux - c23 * vy, tyy = c43 * vy - c23 * ux, txy = uy + vx;
  const T tn1 = txx * nx + txy * ny, tn2 = txy * nx + tyy * ny;
  Fn[0] = T(0);
  Fn[1] = m * tn1;
  Fn[2] = m * tn2;
  Fn[3] = m * (v1 * tn1 + v2 * tn2 + k * (ex * nx + ey * ny));
}

// q = G(U)^T (n (x) w) = (mu/rho) (T^T z_x, T^T z_y) with z = C^T (n (x) w):
// qx = nx G11^T w + ny G21^T w, qy = nx G12^T w + ny G22^T w.
template <typename T>
__device__ __forceinline__ void viscous_transpose(const Gas<T>& g, const VState<T>& st, T nx, T ny,
                                                  const T w[4], T qx[4], T qy[4]) {
  const T v1 = st.v1, v2 = st.v2, m = st.m, k = g.k;
  const T c43 = T(4.0 / 3.0), c23 = T(2.0 / 3.0);
  const T W1 = w[1] + v1 * w[3], W2 = w[2] + v2 * w[3];
  const T sxy = nx * W2 + ny * W1;
  // weights of the rho-scaled primitive gradients (u, v, e) in x and in y
  const T zux = c43 * nx * W1 - c23 * ny * W2, zvx = sxy, zex = k * nx * w[3];
  const T zuy = sxy, zvy = c43 * ny * W2 - c23 * nx * W1, zey = k * ny * w[3];
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
__device__ __noinline__ double sym3_lambda_max_trig(double s00, double s11, double s22, double s01,
                                                    double s02, double s12) {
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
template <typename T>
__device__ __forceinline__ T normal_diffusion_norm(const Gas<T>& g, const VState<T>& st, T nx,
                                                   T ny) {
  // B in the face frame: rotating the momentum rows and columns by the same
  // orthogonal map (x, y) -> (n, t) leaves its singular values unchanged, and
  // for the unit normal its rows become
  //   (-4/3 v_n, 4/3, 0, 0), (-v_t, 0, 1, 0), (e0, (4/3 - k) v_n, (1 - k) v_t, k)
  // with v_n = v.n, v_t = v.t and e0 = -(4/3 v_n^2 + v_t^2 + k ek) (the
  // energy row's density entry, the same in both frames).
  const T k = g.k;
  const T c43 = T(4.0 / 3.0);
  const T vn = st.v1 * nx + st.v2 * ny, vt = st.v2 * nx - st.v1 * ny;
  const T vn2 = vn * vn, vt2 = vt * vt;
  const T e0 = -(c43 * vn2 + vt2 + k * st.ek);
  const T a = c43 - k, b = T(1) - k;
  const T s00 = T(16.0 / 9.0) * (vn2 + T(1));
  const T s11 = vt2 + T(1);
  const T s22 = e0 * e0 + a * a * vn2 + b * b * vt2 + k * k;
  const T s01 = c43 * vn * vt;
  const T s02 = c43 * vn * (a - e0);
  const T s12 = vt * (b - e0);
  // characteristic polynomial lambda^3 - c2 lambda^2 + c1 lambda - c0
  const T c2 = s00 + s11 + s22;
  const T c1 = s00 * s11 + s00 * s22 + s11 * s22 - s01 * s01 - s02 * s02 - s12 * s12;
  const T c0 = s00 * (s11 * s22 - s12 * s12) - s01 * (s01 * s22 - s12 * s02) +
               s02 * (s01 * s12 - s11 * s02);
  T lam = root(s00 * s00 + s11 * s11 + s22 * s22 + T(2) * (s01 * s01 + s02 * s02 + s12 * s12));
  T step = T(0);
  // quadratic convergence from the close upper bound: three steps reach the
  // binary32 tolerance, five the binary64 one (else the fallback below)
  constexpr int kIters = sizeof(T) == 8 ? 5 : 3;
#pragma unroll
  for (int it = 0; it < kIters; ++it) {
    const T f = ((lam - c2) * lam + c1) * lam - c0;
    const T df = (T(3) * lam - T(2) * c2) * lam + c1;
    // the step only needs an approximate reciprocal: Newton corrects the rest
    T r = rcp_approx<T>(df);
    r = r * (T(2) - df * r);
    step = (df > T(0)) ? f * r : T(0);
    lam -= step;
  }
  const T tol = (sizeof(T) == 8) ? T(1e-15) : T(1e-6);
  if (!(fabs(step) <= tol * lam))
    lam = (T)sym3_lambda_max_trig((double)s00, (double)s11, (double)s22, (double)s01, (double)s02,
                                  (double)s12);
  return st.m * root(lam > T(0) ? lam : T(0));
}

// Roe flux: mean of the two normal fluxes FL (own, "+") and FR (other, "-")
// plus (1/2)|A~ - (v_w.n) I|(U+ - U-), the dissipation in wave-strength form
// (Roe averages of velocity and total enthalpy; eigenvalues v~.n - v_w.n and
// v~.n - v_w.n +- c~), with wave strengths from the jumps of sR - sL.
template <typename T>
__device__ __forceinline__ void roe_flux(const Prim<T>& sl, const Prim<T>& sr, const T FL[4],
                                         const T FR[4], T nx, T ny, T vwn, T gm1, T F[4]) {
  const T ql = root(sl.rho), qr = root(sr.rho);
  const T iw = rcp(ql + qr);
  const T rt = ql * qr;
  const T ut = (ql * sl.u + qr * sr.u) * iw, vt = (ql * sl.v + qr * sr.v) * iw;
  const T ht = (ql * sl.H + qr * sr.H) * iw;
  const T c2 = gm1 * (ht - T(0.5) * (ut * ut + vt * vt));
  const T ct = root(c2);
  const T qn = ut * nx + vt * ny, qt = -ut * ny + vt * nx;
  // jumps taken as (other - own)
  const T dr = sr.jr - sl.jr, dp = sr.jp - sl.jp;
  const T du = sr.ju - sl.ju, dv = sr.jv - sl.jv;
  const T dqn = du * nx + dv * ny;
  const T dqt = -du * ny + dv * nx;
  const T ic2 = rcp(c2);
  const T a1 = T(0.5) * (dp - rt * ct * dqn) * ic2;
  const T a2 = dr - dp * ic2;
  const T a3 = rt * dqt;
  const T a4 = T(0.5) * (dp + rt * ct * dqn) * ic2;
  const T l1 = fabs(qn - ct - vwn), l2 = fabs(qn - vwn), l4 = fabs(qn + ct - vwn);
  const T w1 = l1 * a1, w2 = l2 * a2, w3 = l2 * a3, w4 = l4 * a4;
  const T d0 = w1 + w2 + w4;
  const T d1 = w1 * (ut - ct * nx) + w2 * ut - w3 * ny + w4 * (ut + ct * nx);
  const T d2 = w1 * (vt - ct * ny) + w2 * vt + w3 * nx + w4 * (vt + ct * ny);
  const T d3 = w1 * (ht - ct * qn) + w2 * T(0.5) * (ut * ut + vt * vt) + w3 * qt + w4 * (ht + ct * qn);
  F[0] = T(0.5) * (FL[0] + FR[0] - d0);
  F[1] = T(0.5) * (FL[1] + FR[1] - d1);
  F[2] = T(0.5) * (FL[2] + FR[2] - d2);
  F[3] = T(0.5) * (FL[3] + FR[3] - d3);
}

}  // namespace dgmi
