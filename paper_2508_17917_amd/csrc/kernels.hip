// HIP kernels for gfx950: the fused right-hand side + low-storage RK stage,
// and the wall-force reduction.
//
// Stage kernel, per wavefront and tile of four elements, in the order of
// Alg. 2 (the neighbour exchange becomes reads of the neighbours' nodal
// states, resident in HBM / L2 on one GPU):
//   1  own states, neighbour states and geometry -> LDS
//   2  broken gradient on the FP64 matrix cores: rows (element, field),
//      columns nodes, [dU/dr, dU/ds] = U [Dr^T, Ds^T]; the output lane owns one
//      node of one element with all four fields -> total flux
//      F = F_c - v_w (x) U - G grad U and its contravariant components
//   3  face nodes (one lane each): neighbour trace and gradient (reversed face
//      node order), boundary ghosts (Sec. 2.2.4), G-bar_e = max over the face of
//      ||n^T G n||_2 on both sides, sigma_e, Roe flux, viscous average,
//      penalty and theta term
//   4  strong-form residual on the matrix cores,
//      R = -(Dr Fr + Ds Fs) + LIFT h + LIFTr qr + LIFTs qs
//      (M^-1 and 1/J folded into the operators and Fscale), then
//      K1 <- a K1 + dt R, U_out <- U_in + b K1 (Alg. 1).
// Every element writes only its own nodes and each face is evaluated from both
// sides, so there are no atomics and results are bitwise reproducible.
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
  static constexpr int S = 4 * Np;               // doubles per element state
  static constexpr int NT = (Np + 15) / 16;      // 16-node output tiles
  static constexpr int KS = (Np + 3) / 4;        // k-steps over volume nodes
  static constexpr int KF = (NF + 3) / 4;        // k-steps over face nodes
  static constexpr int RS = 4 * KS + 1;          // padded LDS row (odd: no bank aliasing)
  static constexpr int HRS = 4 * KF + 1;
  static constexpr int FIT = (4 * NF + 63) / 64; // face items per lane
  static constexpr int WAVES = (N <= 4) ? 4 : 2;
  static constexpr int THREADS = 64 * WAVES;
  // per-wave LDS (doubles)
  static constexpr int U_SZ = 16 * RS;           // own state, row 4c + e
  static constexpr int F_SZ = 32 * RS;           // contravariant flux Fr rows | Fs rows
  static constexpr int N_SZ = 12 * S;            // neighbour states [e][f][c][n]
  static constexpr int H_SZ = 48 * HRS;          // face terms h | qr | qs, row 4c + e
  static constexpr int X_SZ = N_SZ > H_SZ ? N_SZ : H_SZ;
  static constexpr int NORM_SZ = 4 * NF;
  static constexpr int VN_SZ = 16 * NF;          // mean viscous normal flux per face node
  static constexpr int WAVE_SZ = U_SZ + F_SZ + X_SZ + NORM_SZ + VN_SZ + 64 + 48;
  // operator fragments (per workgroup)
  static constexpr int FD = NT * KS * 64;        // one Dr-type fragment set
  static constexpr int FL = NT * KF * 64;        // one LIFT-type fragment set
  static constexpr int FRAG_SZ = 2 * FD + 3 * FL;
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

typedef double d4 __attribute__((ext_vector_type(4)));

// D += A B for A 16x4, B 4x16, D 16x16 (FP64 matrix core).  Lane l supplies
// A[l%16][l/16] and B[l/16][l%16] and holds D[l/16 + 4v][l%16], v = 0..3.
// With rows ordered (field c, element e) -> 4c + e, lane l therefore ends up
// with node l%16 of element l/16, all four fields in v = c.
__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// LDS ordering among the lanes of one wavefront (no workgroup barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double lane_read(double v, int src) {
  int lo = __builtin_amdgcn_ds_bpermute(src << 2, __double2loint(v));
  int hi = __builtin_amdgcn_ds_bpermute(src << 2, __double2hiint(v));
  return __hiloint2double(hi, lo);
}

// State on the other side of a face node: the neighbour's trace (interior,
// periodic), the moving adiabatic wall's ghost Q^b = [rho+, v_w, p+], or the
// far-field state (Sec. 2.2.4).  nb points at the neighbour's node, stride Np.
__device__ __forceinline__ void ghost_state(int tag, const double up[4], const double* nb, int Np,
                                            double vwx, double vwy, const double* Uinf,
                                            const Gas& gas, double uo[4]) {
  if (tag == 0) {
#pragma unroll
    for (int c = 0; c < 4; ++c) uo[c] = nb[c * Np];
  } else if (tag == 1) {
    const double p = pressure(up, 1.0 / up[0], gas.gm1);
    uo[0] = up[0];
    uo[1] = up[0] * vwx;
    uo[2] = up[0] * vwy;
    uo[3] = p * gas.igm1 + 0.5 * up[0] * (vwx * vwx + vwy * vwy);
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c) uo[c] = Uinf[c];
  }
}

// The fused right-hand side + LSERK stage.  Each wavefront owns tiles of four
// elements (16 MFMA rows = 4 fields x 4 elements); the workgroup only shares
// the operator fragments.  Tiles are handed out in contiguous ranges per XCD
// (workgroup b runs on XCD b % 8) so neighbour reads stay in that XCD's L2.
template <int N>
__global__ __launch_bounds__(Order<N>::THREADS) __attribute__((amdgpu_waves_per_eu(2))) void stage_kernel(
    DeviceTables t, KernelPhysics ph, const double* __restrict__ Uin, double* __restrict__ Uout,
    double* __restrict__ K1, double a, double b, double dt, int rhs_only) {
  using O = Order<N>;
  constexpr int Np = O::Np, Nfp = O::Nfp, NF = O::NF, S = O::S, NT = O::NT, KS = O::KS,
                KF = O::KF, RS = O::RS, HRS = O::HRS, FIT = O::FIT;
  constexpr int OFF_DR = 0, OFF_DS = O::FD, OFF_L = 2 * O::FD, OFF_LR = 2 * O::FD + O::FL,
                OFF_LS = 2 * O::FD + 2 * O::FL;
  __shared__ double sFrag[O::FRAG_SZ];
  __shared__ double sWave[O::WAVES][O::WAVE_SZ];
  __shared__ int sConnW[O::WAVES][12];

  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < O::FRAG_SZ; i += O::THREADS) sFrag[i] = t.frag[i];
  for (int i = lane; i < O::WAVE_SZ; i += 64) sWave[wid][i] = 0.0;  // zero pads once
  __syncthreads();

  double* sU = &sWave[wid][0];
  double* sFr = sU + O::U_SZ;
  double* sFs = sFr + 16 * RS;
  double* sX = sU + O::U_SZ + O::F_SZ;   // neighbour states, later face terms
  double* sH = sX;
  double* sQr = sX + 16 * HRS;
  double* sQs = sX + 32 * HRS;
  double* sNorm = sX + O::X_SZ;
  double* sVn = sNorm + O::NORM_SZ;      // [4 NF][4]
  double* sGeo = sVn + O::VN_SZ;         // [4][16]
  double* sNGeo = sGeo + 64;             // [4][3][4]
  int* sConn = sConnW[wid];              // [4][3]

  Gas gas;
  gas.gamma = ph.gamma;
  gas.gm1 = ph.gamma - 1.0;
  gas.igm1 = 1.0 / (ph.gamma - 1.0);
  gas.mu = ph.mu;
  gas.k = ph.gamma / ph.Pr;
  const double theta = ph.theta;
  const double vwx = ph.vw[0], vwy = ph.vw[1];

  const int64_t K = t.K;
  const int64_t ntiles = (K + 3) / 4;
  const int xcd = blockIdx.x & 7;
  const int nbx = gridDim.x >> 3;
  const int64_t tb = ntiles * xcd / 8, te = ntiles * (xcd + 1) / 8;
  const int64_t w0 = (int64_t)(blockIdx.x >> 3) * O::WAVES + wid;
  const int64_t wstride = (int64_t)nbx * O::WAVES;

  const int arow = lane & 15, acol = lane >> 4;  // A-operand row (4c + e), k offset
  const int re = lane >> 4, rn = lane & 15;      // output: element re, node 16 t + rn
  // state loads: value r = lane + 64 q of an element block is field r / Np,
  // node r % Np
  constexpr int NQ = (S + 63) / 64;
  bool lr_ok[NQ];
  int lds_u[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int r = lane + 64 * q;
    lr_ok[q] = r < S;
    lds_u[q] = lr_ok[q] ? (4 * (r / Np)) * RS + (r - (r / Np) * Np) : 0;
  }

  for (int64_t tile = tb + w0; tile < te; tile += wstride) {
    const int64_t e0 = tile * 4;
    const int nel = (int)((K - e0) < 4 ? (K - e0) : 4);
    wave_sync();
    // ---- own states, geometry, connectivity.  Lane l owns values r = l + 64 q
    // of every element block, so addresses are a per-lane constant plus a
    // wave-uniform base, and every load is issued before the first use.
    double ru[4][NQ];
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        ru[e][q] = (lr_ok[q] && e < nel) ? Uin[(e0 + e) * S + lane + 64 * q] : 0.0;
    const double rg = (lane < nel * kGeoStride) ? t.geo[e0 * kGeoStride + lane] : 0.0;
    const int rc = (lane < nel * 3) ? t.conn[e0 * 3 + lane] : 0;
    if (lane < nel * 3) sConn[lane] = rc;
    wave_sync();
    // ---- neighbour states (a boundary face points at the element itself) and
    // metrics, in two batches of six blocks (bounded register use)
    const double rng = (lane < nel * 12) ? t.geo[(int64_t)(sConn[lane >> 2] >> 4) * kGeoStride + (lane & 3)] : 0.0;
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        if (lr_ok[q] && e < nel) sU[lds_u[q] + e * RS] = ru[e][q];
    if (lane < nel * kGeoStride) sGeo[lane] = rg;
#pragma nounroll
    for (int h = 0; h < 2; ++h) {
      double rnb[6][NQ];
#pragma unroll
      for (int b = 0; b < 6; ++b) {
        const int ef = 6 * h + b;  // uniform across the wave
        const int64_t nb = (int64_t)(sConn[ef] >> 4) * S;
#pragma unroll
        for (int q = 0; q < NQ; ++q)
          rnb[b][q] = (lr_ok[q] && ef < 3 * nel) ? Uin[nb + lane + 64 * q] : 0.0;
      }
#pragma unroll
      for (int b = 0; b < 6; ++b) {
        const int ef = 6 * h + b;
#pragma unroll
        for (int q = 0; q < NQ; ++q)
          if (lr_ok[q] && ef < 3 * nel) sX[ef * S + lane + 64 * q] = rnb[b][q];
      }
    }
    if (lane < nel * 12) sNGeo[lane] = rng;
    wave_sync();

    // ---- gradient on the matrix cores, then the volume flux per node
    double gxk[NT][4], gyk[NT][4];
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) {
      d4 aR = {0.0, 0.0, 0.0, 0.0}, aS = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const double av = sU[arow * RS + 4 * s + acol];
        aR = mfma(av, sFrag[OFF_DR + (tt * KS + s) * 64 + lane], aR);
        aS = mfma(av, sFrag[OFF_DS + (tt * KS + s) * 64 + lane], aS);
      }
      const int n = 16 * tt + rn;
      const bool ok = (re < nel) && (n < Np);
      const double* g = sGeo + re * kGeoStride;
      const double rx = ok ? g[0] : 0.0, ry = ok ? g[1] : 0.0;
      const double sx = ok ? g[2] : 0.0, sy = ok ? g[3] : 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        gxk[tt][c] = rx * aR[c] + sx * aS[c];
        gyk[tt][c] = ry * aR[c] + sy * aS[c];
      }
      if (ok) {
        double U[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) U[c] = sU[(4 * c + re) * RS + n];
        double fvx[4], fvy[4];
        const VState st = vstate(gas, U);
        viscous_flux(gas, st, gxk[tt], gyk[tt], fvx, fvy);
        const double u = st.v1, v = st.v2;
        const double p = gas.gm1 * (U[3] - 0.5 * (U[1] * u + U[2] * v));
        const double qu = u - vwx, qv = v - vwy;
        double Fx[4] = {U[0] * qu, U[1] * qu + p, U[2] * qu, U[3] * qu + p * u};
        double Fy[4] = {U[0] * qv, U[1] * qv, U[2] * qv + p, U[3] * qv + p * v};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double fx = Fx[c] - fvx[c], fy = Fy[c] - fvy[c];
          sFr[(4 * c + re) * RS + n] = rx * fx + ry * fy;
          sFs[(4 * c + re) * RS + n] = sx * fx + sy * fy;
        }
      }
    }
    wave_sync();

    // ---- face nodes, pass 1: traces, ghosts, ||n^T G n||_2 on both sides and the
    // mean viscous normal flux (one lane per face node)
#pragma unroll
    for (int q = 0; q < FIT; ++q) {
      const int it = lane + 64 * q;
      int e = it / NF;
      const int fn = it - e * NF;
      const bool ok = (it < 4 * NF) && (e < nel);
      e = e < 4 ? e : 3;
      const int f = fn / Nfp, j = fn - f * Nfp;
      const int n = face_node<N>(f, j);
      // own gradient at the face node, from the lane that computed it
      double gxp[4], gyp[4];
      const int src = 16 * e + (n & 15);
#pragma unroll
      for (int tt = 0; tt < NT; ++tt) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double vx = lane_read(gxk[tt][c], src), vy = lane_read(gyk[tt][c], src);
          if ((n >> 4) == tt) {
            gxp[c] = vx;
            gyp[c] = vy;
          }
        }
      }
      if (ok) {
        const int conn = sConn[e * 3 + f];
        const int tag = conn & 3, nf = (conn >> 2) & 3;
        const double* g = sGeo + e * kGeoStride;
        const double nx = g[4 + 4 * f], ny = g[5 + 4 * f];
        double up[4], uo[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) up[c] = sU[(4 * c + e) * RS + n];
        const int n2 = (tag == 0) ? face_node<N>(nf, Nfp - 1 - j) : n;
        const double* nbU = sX + (e * 3 + f) * S;
        ghost_state(tag, up, nbU + n2, Np, vwx, vwy, ph.U_inf, gas, uo);
        const VState sp = vstate(gas, up), so = vstate(gas, uo);
        // one side at a time: the two evaluations need not be live together
        double nrm = 0.0;
#pragma nounroll
        for (int side = 0; side < 2; ++side) {
          const double a1 = normal_diffusion_norm(gas, side == 0 ? sp : so, nx, ny);
          nrm = a1 > nrm ? a1 : nrm;
        }
        sNorm[e * NF + fn] = nrm;
        // "other side" gradient from the staged neighbour (wall: the element itself)
        double ur[4] = {0, 0, 0, 0}, us[4] = {0, 0, 0, 0};
        const int dbase = ((n2 >> 4) * KS) * 64 + (n2 & 15);
#pragma unroll 4
        for (int m = 0; m < Np; ++m) {
          const int fi = dbase + (m >> 2) * 64 + (m & 3) * 16;
          const double dr = sFrag[OFF_DR + fi], ds = sFrag[OFF_DS + fi];
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const double uu = nbU[c * Np + m];
            ur[c] += dr * uu;
            us[c] += ds * uu;
          }
        }
        const double* ng = sNGeo + (e * 3 + f) * 4;
        double gxm[4], gym[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          gxm[c] = ng[0] * ur[c] + ng[2] * us[c];
          gym[c] = ng[1] * ur[c] + ng[3] * us[c];
        }
        // mean of G(U+) grad U+ and G(U-) grad U- inside; G(U^b) grad U+ on the
        // wall (grad U+ from the staged copy of the element itself); G(U+) grad U+
        // on the far field
        double vx[4], vy[4], vn[4];
        if (tag == 1) {
          viscous_flux(gas, so, gxm, gym, vx, vy);
#pragma unroll
          for (int c = 0; c < 4; ++c) vn[c] = vx[c] * nx + vy[c] * ny;
        } else {
          viscous_flux(gas, sp, gxp, gyp, vx, vy);
#pragma unroll
          for (int c = 0; c < 4; ++c) vn[c] = vx[c] * nx + vy[c] * ny;
          if (tag == 0) {
            viscous_flux(gas, so, gxm, gym, vx, vy);
#pragma unroll
            for (int c = 0; c < 4; ++c) vn[c] = 0.5 * (vn[c] + vx[c] * nx + vy[c] * ny);
          }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) sVn[(e * NF + fn) * 4 + c] = vn[c];
      }
    }
    wave_sync();
    // ---- face nodes, pass 2: gather what the Roe flux, penalty and theta term
    // need, then (after every read of the neighbour area) write the face terms
    double fup[FIT][4], fuo[FIT][4], fvn[FIT][4], fgb[FIT];
#pragma unroll
    for (int q = 0; q < FIT; ++q) {
      const int it = lane + 64 * q;
      const int e = it / NF;
      const int fn = it - e * NF;
      if ((it < 4 * NF) && (e < nel)) {
        const int f = fn / Nfp, j = fn - f * Nfp;
        const int n = face_node<N>(f, j);
        const int conn = sConn[e * 3 + f];
        const int tag = conn & 3, nf = (conn >> 2) & 3;
#pragma unroll
        for (int c = 0; c < 4; ++c) fup[q][c] = sU[(4 * c + e) * RS + n];
        const int n2 = face_node<N>(nf, Nfp - 1 - j);
        ghost_state(tag, fup[q], sX + (e * 3 + f) * S + n2, Np, vwx, vwy, ph.U_inf, gas, fuo[q]);
#pragma unroll
        for (int c = 0; c < 4; ++c) fvn[q][c] = sVn[(e * NF + fn) * 4 + c];
        double gbar = 0.0;
#pragma unroll
        for (int jj = 0; jj < Nfp; ++jj) {
          const double v = sNorm[e * NF + f * Nfp + jj];
          gbar = v > gbar ? v : gbar;
        }
        fgb[q] = gbar;
      }
    }
    wave_sync();
#pragma unroll
    for (int q = 0; q < FIT; ++q) {
      const int it = lane + 64 * q;
      const int e = it / NF;
      const int fn = it - e * NF;
      if ((it < 4 * NF) && (e < nel)) {
        const int f = fn / Nfp, j = fn - f * Nfp;
        const int n = face_node<N>(f, j);
        const int tag = sConn[e * 3 + f] & 3;
        const double* g = sGeo + e * kGeoStride;
        const double nx = g[4 + 4 * f], ny = g[5 + 4 * f], fsc = g[6 + 4 * f];
        const double sigma = g[7 + 4 * f] * fgb[q];
        const double vwn = vwx * nx + vwy * ny;
        const VState sp = vstate(gas, fup[q]);
        const VState so = vstate(gas, fuo[q]);
        double Fc[4];
        if (tag == 1) {
          const double p = pressure(fup[q], sp.ir, gas.gm1);
          Fc[0] = 0.0;
          Fc[1] = p * nx;
          Fc[2] = p * ny;
          Fc[3] = p * vwn;
        } else {
          roe_flux(fup[q], sp.ir, fuo[q], so.ir, nx, ny, vwn, gas.gm1, Fc);
        }
        double w[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          // Fscale * own total normal flux from the contravariant flux:
          // face 0: -Fs, face 1: Fr + Fs, face 2: -Fr
          const double fr = sFr[(4 * c + e) * RS + n], fs = sFs[(4 * c + e) * RS + n];
          const double own = (f == 0) ? -fs : (f == 1 ? fr + fs : -fr);
          w[c] = fup[q][c] - fuo[q][c];
          sH[(4 * c + e) * HRS + fn] = own - fsc * (Fc[c] - fvn[q][c] + sigma * w[c]);
        }
        double qx[4], qy[4];
        viscous_transpose(gas, tag == 1 ? so : sp, nx, ny, w, qx, qy);
        const double ce = theta * (tag == 0 ? 0.5 : 1.0) * fsc;
        const double rx = g[0], ry = g[1], sx = g[2], sy = g[3];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          sQr[(4 * c + e) * HRS + fn] = ce * (rx * qx[c] + ry * qy[c]);
          sQs[(4 * c + e) * HRS + fn] = ce * (sx * qx[c] + sy * qy[c]);
        }
      }
    }
    for (int i = lane; i < 48 * (HRS - NF); i += 64) {
      const int row = i / (HRS - NF);
      sX[row * HRS + NF + (i - row * (HRS - NF))] = 0.0;
    }
    wave_sync();

    // ---- divergence and lifts on the matrix cores, then the RK stage; the
    // K1 loads are issued first so the matrix work covers their latency
    double rk[NT][4];
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) {
      const int n = 16 * tt + rn;
#pragma unroll
      for (int c = 0; c < 4; ++c)
        rk[tt][c] = (!rhs_only && a != 0.0 && re < nel && n < Np) ? K1[(e0 + re) * S + c * Np + n] : 0.0;
    }
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) {
      d4 aD = {0.0, 0.0, 0.0, 0.0}, aL = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        aD = mfma(sFr[arow * RS + 4 * s + acol], sFrag[OFF_DR + (tt * KS + s) * 64 + lane], aD);
        aD = mfma(sFs[arow * RS + 4 * s + acol], sFrag[OFF_DS + (tt * KS + s) * 64 + lane], aD);
      }
#pragma unroll
      for (int s = 0; s < KF; ++s) {
        const int fi = (tt * KF + s) * 64 + lane;
        aL = mfma(sH[arow * HRS + 4 * s + acol], sFrag[OFF_L + fi], aL);
        aL = mfma(sQr[arow * HRS + 4 * s + acol], sFrag[OFF_LR + fi], aL);
        aL = mfma(sQs[arow * HRS + 4 * s + acol], sFrag[OFF_LS + fi], aL);
      }
      const int n = 16 * tt + rn;
      if (re < nel && n < Np) {
        const int64_t base = (e0 + re) * S + n;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double R = aL[c] - aD[c];
          const int64_t idx = base + c * Np;
          if (rhs_only) {
            K1[idx] = R;
          } else {
            const double k = (a == 0.0) ? dt * R : a * rk[tt][c] + dt * R;
            K1[idx] = k;
            Uout[idx] = sU[(4 * c + re) * RS + n] + b * k;
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
  gas.igm1 = 1.0 / (ph.gamma - 1.0);
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
    double p = pressure(Up, 1.0 / Up[0], gas.gm1);
    double Ub[4] = {Up[0], Up[0] * ph.vw[0], Up[0] * ph.vw[1],
                    p * gas.igm1 + 0.5 * Up[0] * (ph.vw[0] * ph.vw[0] + ph.vw[1] * ph.vw[1])};
    double vx[4], vy[4];
    viscous_flux(gas, vstate(gas, Ub), dx, dy, vx, vy);
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
  const int64_t ntiles = (t.K + 3) / 4;
  // persistent: about two workgroups per CU, a multiple of 8 (one range per XCD)
  int64_t want = (ntiles + O::WAVES - 1) / O::WAVES;
  int grid = (int)(want < 512 ? want : 512);
  grid = ((grid + 7) / 8) * 8;
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
