// HIP kernels for gfx950: the fused right-hand side + low-storage RK stage,
// and the wall-force reduction.
//
// One workgroup owns a tile of EPB elements at a time (grid-stride over
// tiles, operators staged in LDS once per workgroup).  Per tile, in the
// order of Alg. 2 (with the neighbour exchange replaced by reads of the
// neighbours' nodal states, which on one GPU are resident in HBM/L2):
//   A  own states, neighbour states and geometry -> LDS
//   B  volume nodes: broken gradient grad U = (rx Dr + sx Ds, ry Dr + sy Ds) U,
//      total flux F = F_c - v_w (x) U - G grad U, contravariant (Fr, Fs)
//   C  face nodes: neighbour trace and gradient (reversed face node order),
//      boundary ghosts (Sec. 2.2.4), G-bar_e (max over the face of
//      ||n^T G n||_2 on both sides), sigma_e, Roe flux, viscous average,
//      penalty, theta term
//   D  volume nodes: R = -(Dr Fr + Ds Fs) + LIFT h + LIFTr qr + LIFTs qs
//      (strong form; M^-1 and 1/J folded into the operators and Fscale),
//      then K1 <- a K1 + dt R, U_out <- U_in + b K1 (Alg. 1).
// Every element writes only its own nodes; faces are evaluated once from
// each side, so there are no atomics and results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <cstdio>

#include "dg_internal.h"
#include "dg_physics.h"

namespace dgmi {

template <int N>
struct Order {
  static constexpr int Np = (N + 1) * (N + 2) / 2;
  static constexpr int Nfp = N + 1;
  static constexpr int NF = 3 * (N + 1);
  static constexpr int ITEMS = Np > NF ? Np : NF;
  static constexpr int THREADS = 128;
  static constexpr int EPB = THREADS / ITEMS;
  static constexpr int HSZ = (12 * NF > 12 * Np) ? 12 * NF : 12 * Np;  // per element, sN | sH
};

// Node index of face node j (counter-clockwise) on face f; rows of the node
// numbering start at i(N+1) - i(i-1)/2.
template <int N>
__device__ __forceinline__ int face_node(int f, int j) {
  if (f == 0) return j;
  if (f == 1) return j * (N + 1) - j * (j - 1) / 2 + (N - j);
  int i = N - j;
  return i * (N + 1) - i * (i - 1) / 2;
}

template <int N>
__global__ __launch_bounds__(128) void stage_kernel(DeviceTables t, KernelPhysics ph,
                                                    const double* __restrict__ Uin,
                                                    double* __restrict__ Uout,
                                                    double* __restrict__ K1, double a, double b,
                                                    double dt, int rhs_only) {
  using O = Order<N>;
  constexpr int Np = O::Np, Nfp = O::Nfp, NF = O::NF, EPB = O::EPB, T = O::THREADS;
  constexpr int S = 4 * Np;  // doubles per element state

  __shared__ double sDr[Np * Np], sDs[Np * Np];
  __shared__ double sL[Np * NF], sLr[Np * NF], sLs[Np * NF];
  __shared__ double sU[EPB][4][Np];
  __shared__ double sG[EPB][8][Np];   // grad U: x-derivatives 0..3, y 4..7
  __shared__ double sF[EPB][8][Np];   // contravariant flux: Fr 0..3, Fs 4..7
  __shared__ double sX[EPB][O::HSZ];  // phase A/C: neighbour states; C/D: face terms
  __shared__ double sNorm[EPB][NF];
  __shared__ double sGeo[EPB][kGeoStride];
  __shared__ double sNGeo[EPB][3][4];
  __shared__ int sConn[EPB][3];

  const int tid = threadIdx.x;
  const int64_t K = t.K;
  const int64_t ntiles = (K + EPB - 1) / EPB;

  for (int i = tid; i < Np * Np; i += T) {
    sDr[i] = t.ops[i];
    sDs[i] = t.ops[Np * Np + i];
  }
  for (int i = tid; i < Np * NF; i += T) {
    sL[i] = t.ops[2 * Np * Np + i];
    sLr[i] = t.ops[2 * Np * Np + Np * NF + i];
    sLs[i] = t.ops[2 * Np * Np + 2 * Np * NF + i];
  }

  Gas gas;
  gas.gamma = ph.gamma;
  gas.gm1 = ph.gamma - 1.0;
  gas.mu = ph.mu;
  gas.k = ph.gamma / ph.Pr;
  const double theta = ph.theta;

  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t e0 = tile * EPB;
    const int nel = (int)((K - e0) < EPB ? (K - e0) : EPB);
    __syncthreads();  // previous tile done with LDS (and operators staged)
    // ---- A: own states, geometry, connectivity
    for (int i = tid; i < nel * S; i += T) (&sU[0][0][0])[i] = Uin[e0 * S + i];
    for (int i = tid; i < nel * kGeoStride; i += T) (&sGeo[0][0])[i] = t.geo[e0 * kGeoStride + i];
    for (int i = tid; i < nel * 3; i += T) (&sConn[0][0])[i] = t.conn[e0 * 3 + i];
    __syncthreads();
    // neighbour states (boundary faces point at the element itself) and metrics
    for (int i = tid; i < nel * 3 * S; i += T) {
      int ef = i / S, r = i - ef * S;
      int nb = sConn[ef / 3][ef % 3] >> 4;
      sX[ef / 3][(ef % 3) * S + r] = Uin[(int64_t)nb * S + r];
    }
    for (int i = tid; i < nel * 12; i += T) {
      int ef = i / 4, c = i - ef * 4;
      int nb = sConn[ef / 3][ef % 3] >> 4;
      sNGeo[ef / 3][ef % 3][c] = t.geo[(int64_t)nb * kGeoStride + c];
    }
    __syncthreads();

    // ---- B: gradient and contravariant flux at volume nodes
    {
      const int e = tid / Np, n = tid - (tid / Np) * Np;
      if (e < nel) {
        double ur[4] = {0, 0, 0, 0}, us[4] = {0, 0, 0, 0};
#pragma unroll 4
        for (int m = 0; m < Np; ++m) {
          double dr = sDr[n * Np + m], ds = sDs[n * Np + m];
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            double u = sU[e][c][m];
            ur[c] += dr * u;
            us[c] += ds * u;
          }
        }
        const double rx = sGeo[e][0], ry = sGeo[e][1], sx = sGeo[e][2], sy = sGeo[e][3];
        double U[4], dx[4], dy[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          U[c] = sU[e][c][n];
          dx[c] = rx * ur[c] + sx * us[c];
          dy[c] = ry * ur[c] + sy * us[c];
          sG[e][c][n] = dx[c];
          sG[e][4 + c][n] = dy[c];
        }
        double fvx[4], fvy[4];
        viscous_flux(gas, U, dx, dy, fvx, fvy);
        double ir = 1.0 / U[0];
        double u = U[1] * ir, v = U[2] * ir;
        double p = gas.gm1 * (U[3] - 0.5 * (U[1] * u + U[2] * v));
        double Fx[4], Fy[4];
        Fx[0] = U[0] * (u - ph.vw[0]);
        Fx[1] = U[1] * (u - ph.vw[0]) + p;
        Fx[2] = U[2] * (u - ph.vw[0]);
        Fx[3] = U[3] * (u - ph.vw[0]) + p * u;
        Fy[0] = U[0] * (v - ph.vw[1]);
        Fy[1] = U[1] * (v - ph.vw[1]);
        Fy[2] = U[2] * (v - ph.vw[1]) + p;
        Fy[3] = U[3] * (v - ph.vw[1]) + p * v;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          double fx = Fx[c] - fvx[c], fy = Fy[c] - fvy[c];
          sF[e][c][n] = rx * fx + ry * fy;
          sF[e][4 + c][n] = sx * fx + sy * fy;
        }
      }
    }
    __syncthreads();

    // ---- C: face nodes
    const int fe = tid / NF, fn = tid - (tid / NF) * NF;
    const bool fvalid = fe < nel;
    const int f = fn / Nfp, j = fn - (fn / Nfp) * Nfp;
    double Up[4], Uo[4], gxp[4], gyp[4], gxm[4], gym[4];
    double nx = 0, ny = 0, fsc = 0, sgeo = 0;
    int tag = 0;
    if (fvalid) {
      const int n = face_node<N>(f, j);
      const int conn = sConn[fe][f];
      tag = conn & 3;
      const int nf = (conn >> 2) & 3;
      nx = sGeo[fe][4 + 4 * f];
      ny = sGeo[fe][5 + 4 * f];
      fsc = sGeo[fe][6 + 4 * f];
      sgeo = sGeo[fe][7 + 4 * f];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        Up[c] = sU[fe][c][n];
        gxp[c] = sG[fe][c][n];
        gyp[c] = sG[fe][4 + c][n];
      }
      if (tag == 0) {
        const int n2 = face_node<N>(nf, Nfp - 1 - j);
        const double* nbU = &sX[fe][f * S];
        double ur[4] = {0, 0, 0, 0}, us[4] = {0, 0, 0, 0};
#pragma unroll 4
        for (int m = 0; m < Np; ++m) {
          double dr = sDr[n2 * Np + m], ds = sDs[n2 * Np + m];
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            double u = nbU[c * Np + m];
            ur[c] += dr * u;
            us[c] += ds * u;
          }
        }
        const double rx = sNGeo[fe][f][0], ry = sNGeo[fe][f][1];
        const double sx = sNGeo[fe][f][2], sy = sNGeo[fe][f][3];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          Uo[c] = nbU[c * Np + n2];
          gxm[c] = rx * ur[c] + sx * us[c];
          gym[c] = ry * ur[c] + sy * us[c];
        }
      } else if (tag == 1) {
        // moving adiabatic wall: Q^b = [rho+, v_w, p+]
        double p = pressure(Up, gas.gm1);
        Uo[0] = Up[0];
        Uo[1] = Up[0] * ph.vw[0];
        Uo[2] = Up[0] * ph.vw[1];
        Uo[3] = p / gas.gm1 + 0.5 * Up[0] * (ph.vw[0] * ph.vw[0] + ph.vw[1] * ph.vw[1]);
      } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) Uo[c] = ph.U_inf[c];
      }
      double a1 = normal_diffusion_norm(gas, Up, nx, ny);
      double a2 = normal_diffusion_norm(gas, Uo, nx, ny);
      sNorm[fe][fn] = a1 > a2 ? a1 : a2;
    }
    __syncthreads();
    if (fvalid) {
      double gbar = 0.0;
#pragma unroll
      for (int jj = 0; jj < Nfp; ++jj) {
        double v = sNorm[fe][f * Nfp + jj];
        gbar = v > gbar ? v : gbar;
      }
      const double sigma = sgeo * gbar;
      const double vwn = ph.vw[0] * nx + ph.vw[1] * ny;
      double Fc[4];
      if (tag == 1) {
        double p = pressure(Up, gas.gm1);
        Fc[0] = 0.0;
        Fc[1] = p * nx;
        Fc[2] = p * ny;
        Fc[3] = p * vwn;
      } else {
        roe_flux(Up, Uo, nx, ny, vwn, gas.gm1, Fc);
      }
      double vxa[4], vya[4], vn[4];
      if (tag == 0) {
        double vxb[4], vyb[4];
        viscous_flux(gas, Up, gxp, gyp, vxa, vya);
        viscous_flux(gas, Uo, gxm, gym, vxb, vyb);
#pragma unroll
        for (int c = 0; c < 4; ++c) vn[c] = 0.5 * ((vxa[c] + vxb[c]) * nx + (vya[c] + vyb[c]) * ny);
      } else {
        viscous_flux(gas, tag == 1 ? Uo : Up, gxp, gyp, vxa, vya);
#pragma unroll
        for (int c = 0; c < 4; ++c) vn[c] = vxa[c] * nx + vya[c] * ny;
      }
      // Fscale * (own total normal flux): -Fs (face 0), Fr + Fs (face 1), -Fr (face 2)
      const int n = face_node<N>(f, j);
      double w[4], h[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        double fr = sF[fe][c][n], fs = sF[fe][4 + c][n];
        double own = (f == 0) ? -fs : (f == 1 ? fr + fs : -fr);
        w[c] = Up[c] - Uo[c];
        double Hm = Fc[c] - vn[c] + sigma * w[c];
        h[c] = own - fsc * Hm;
      }
      double qx[4], qy[4];
      viscous_transpose(gas, tag == 1 ? Uo : Up, nx, ny, w, qx, qy);
      const double ce = theta * (tag == 0 ? 0.5 : 1.0) * fsc;
      const double rx = sGeo[fe][0], ry = sGeo[fe][1], sx = sGeo[fe][2], sy = sGeo[fe][3];
      // sX is re-used for the face terms: every neighbour read preceded the barrier above
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        sX[fe][c * NF + fn] = h[c];
        sX[fe][(4 + c) * NF + fn] = ce * (rx * qx[c] + ry * qy[c]);
        sX[fe][(8 + c) * NF + fn] = ce * (sx * qx[c] + sy * qy[c]);
      }
    }
    __syncthreads();

    // ---- D: volume divergence + lift + RK update
    {
      const int e = tid / Np, n = tid - (tid / Np) * Np;
      if (e < nel) {
        double R[4] = {0, 0, 0, 0};
#pragma unroll 4
        for (int m = 0; m < Np; ++m) {
          double dr = sDr[n * Np + m], ds = sDs[n * Np + m];
#pragma unroll
          for (int c = 0; c < 4; ++c) R[c] -= dr * sF[e][c][m] + ds * sF[e][4 + c][m];
        }
#pragma unroll 4
        for (int m = 0; m < NF; ++m) {
          double l = sL[n * NF + m], lr = sLr[n * NF + m], ls = sLs[n * NF + m];
#pragma unroll
          for (int c = 0; c < 4; ++c)
            R[c] += l * sX[e][c * NF + m] + lr * sX[e][(4 + c) * NF + m] +
                    ls * sX[e][(8 + c) * NF + m];
        }
        const int64_t base = (e0 + e) * S + n;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int64_t idx = base + c * Np;
          if (rhs_only) {
            K1[idx] = R[c];
          } else {
            double k = (a == 0.0) ? dt * R[c] : a * K1[idx] + dt * R[c];
            K1[idx] = k;
            Uout[idx] = sU[e][c][n] + b * k;
          }
        }
      }
    }
  }
}

// Wall force: one workgroup walks the wall faces in a fixed order; each
// thread accumulates its share, then a fixed-shape tree reduction in LDS.
template <int N>
__global__ __launch_bounds__(256) void force_kernel(DeviceTables t, KernelPhysics ph,
                                                    const double* __restrict__ U,
                                                    double* __restrict__ out) {
  using O = Order<N>;
  constexpr int Np = O::Np, Nfp = O::Nfp, S = 4 * Np;
  __shared__ double red[3][256];
  Gas gas;
  gas.gamma = ph.gamma;
  gas.gm1 = ph.gamma - 1.0;
  gas.mu = ph.mu;
  gas.k = ph.gamma / ph.Pr;
  const double* Dr = t.ops;
  const double* Ds = t.ops + Np * Np;
  const double* wface = t.ops + 2 * Np * Np + 3 * Np * 3 * Nfp;
  double fx = 0.0, fy = 0.0, mz = 0.0;
  const int total = t.nwall * Nfp;
  for (int i = threadIdx.x; i < total; i += blockDim.x) {
    const int wf = t.wall[i / Nfp];
    const int j = i % Nfp;
    const int64_t k = wf / 3;
    const int f = wf % 3;
    const int n = face_node<N>(f, j);
    const double* Uk = U + k * S;
    const double* g = t.geo + k * kGeoStride;
    double ur[4] = {0, 0, 0, 0}, us[4] = {0, 0, 0, 0};
    for (int m = 0; m < Np; ++m) {
      double dr = Dr[n * Np + m], ds = Ds[n * Np + m];
      for (int c = 0; c < 4; ++c) {
        ur[c] += dr * Uk[c * Np + m];
        us[c] += ds * Uk[c * Np + m];
      }
    }
    double Up[4], dx[4], dy[4];
    for (int c = 0; c < 4; ++c) {
      Up[c] = Uk[c * Np + n];
      dx[c] = g[0] * ur[c] + g[2] * us[c];
      dy[c] = g[1] * ur[c] + g[3] * us[c];
    }
    double p = pressure(Up, gas.gm1);
    double Ub[4] = {Up[0], Up[0] * ph.vw[0], Up[0] * ph.vw[1],
                    p / gas.gm1 + 0.5 * Up[0] * (ph.vw[0] * ph.vw[0] + ph.vw[1] * ph.vw[1])};
    double vx[4], vy[4];
    viscous_flux(gas, Ub, dx, dy, vx, vy);
    const double nx = g[4 + 4 * f], ny = g[5 + 4 * f];
    const double sJ = g[6 + 4 * f] / (g[0] * g[3] - g[1] * g[2]);  // Fscale * J
    const double w = wface[f * Nfp + j] * sJ;
    const double tx = p * nx - (vx[1] * nx + vy[1] * ny);
    const double ty = p * ny - (vx[2] * nx + vy[2] * ny);
    const double xw = t.wall_xy[2 * i], yw = t.wall_xy[2 * i + 1];
    fx += w * tx;
    fy += w * ty;
    mz += w * (xw * ty - yw * tx);
  }
  red[0][threadIdx.x] = fx;
  red[1][threadIdx.x] = fy;
  red[2][threadIdx.x] = mz;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int c = 0; c < 3; ++c) out[c] = red[c][0];
}

namespace {
template <int N>
int launch_stage_n(const DeviceTables& t, const KernelPhysics& ph, const double* Uin, double* Uout,
                   double* K1, double a, double b, double dt, int rhs_only, hipStream_t s,
                   std::string& err) {
  using O = Order<N>;
  int64_t ntiles = (t.K + O::EPB - 1) / O::EPB;
  int grid = (int)(ntiles < 8192 ? ntiles : 8192);
  if (grid < 1) return 0;
  hipLaunchKernelGGL(stage_kernel<N>, dim3(grid), dim3(O::THREADS), 0, s, t, ph, Uin, Uout, K1, a,
                     b, dt, rhs_only);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    err = std::string("stage kernel launch: ") + hipGetErrorString(e);
    return -3;
  }
  return 0;
}
template <int N>
int launch_force_n(const DeviceTables& t, const KernelPhysics& ph, const double* U, double* out,
                   hipStream_t s, std::string& err) {
  hipLaunchKernelGGL(force_kernel<N>, dim3(1), dim3(256), 0, s, t, ph, U, out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    err = std::string("force kernel launch: ") + hipGetErrorString(e);
    return -3;
  }
  return 0;
}
}  // namespace

int launch_stage(int N, const DeviceTables& t, const KernelPhysics& ph, const double* Uin,
                 double* Uout, double* K1, double a, double b, double dt, int rhs_only,
                 void* stream, std::string& err) {
  hipStream_t s = (hipStream_t)stream;
  switch (N) {
    case 1: return launch_stage_n<1>(t, ph, Uin, Uout, K1, a, b, dt, rhs_only, s, err);
    case 2: return launch_stage_n<2>(t, ph, Uin, Uout, K1, a, b, dt, rhs_only, s, err);
    case 3: return launch_stage_n<3>(t, ph, Uin, Uout, K1, a, b, dt, rhs_only, s, err);
    case 4: return launch_stage_n<4>(t, ph, Uin, Uout, K1, a, b, dt, rhs_only, s, err);
    case 5: return launch_stage_n<5>(t, ph, Uin, Uout, K1, a, b, dt, rhs_only, s, err);
    case 6: return launch_stage_n<6>(t, ph, Uin, Uout, K1, a, b, dt, rhs_only, s, err);
    default: err = "polynomial order not built"; return -5;
  }
}

int launch_force(int N, const DeviceTables& t, const KernelPhysics& ph, const double* U,
                 double* out, void* stream, std::string& err) {
  hipStream_t s = (hipStream_t)stream;
  switch (N) {
    case 1: return launch_force_n<1>(t, ph, U, out, s, err);
    case 2: return launch_force_n<2>(t, ph, U, out, s, err);
    case 3: return launch_force_n<3>(t, ph, U, out, s, err);
    case 4: return launch_force_n<4>(t, ph, U, out, s, err);
    case 5: return launch_force_n<5>(t, ph, U, out, s, err);
    case 6: return launch_force_n<6>(t, ph, U, out, s, err);
    default: err = "polynomial order not built"; return -5;
  }
}

}  // namespace dgmi
