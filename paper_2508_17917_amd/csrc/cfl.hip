// Time step from the CFL condition (eq. cfl_general): the bound Lambda of
// eq. rayleigh_bound on the numerical range of the DG operator, evaluated on
// the current state,
//
//   Lambda = max_K ( 3/2 C_inv,2(K) G_K + 3 C_inv,K (3 sigma_K + beta_K) + beta'_K ),
//
// C_inv,K = Np max_e |e|/|K| (the trace inverse constant), C_inv,2(K) =
// C_grad p^4 / rho_K^2 (rho_K = 2|K| / perimeter), sigma_K the largest face
// penalty of K as the right-hand side forms it, beta_K the largest
// |v - v_w| + c over the nodes of K, beta'_K half the largest |div v|, and G_K
// the largest directional norm ||e_a^T G e_a||_2 (a = x, y) over the nodes
// of K and of its face neighbours.
//
// Two launches: the first (one thread per element and node) forms the
// per-element node maxima and, per face, the largest ||n^T G n||_2 over the
// face's own nodes (and the boundary ghost); the second (one thread per
// element) combines each element with its neighbours and reduces Lambda to
// one value (maximum of non-negative doubles, order-independent, taken with
// an integer atomic on their bits).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "dg_internal.h"
#include "dg_physics.h"

namespace dgmi {

namespace {

constexpr int kCflThreads = 256;

// Node j (counter-clockwise) of face f in the reference node numbering
// (rows of the numbering start at i(N+1) - i(i-1)/2).
template <int N>
__device__ __forceinline__ int cfl_face_node(int f, int j) {
  if (f == 0) return j;
  if (f == 1) return j * (N + 1) - j * (j - 1) / 2 + (N - j);
  const int i = N - j;
  return i * (N + 1) - i * (i - 1) / 2;
}

// maximum that keeps a NaN from either side (so that an unphysical state is
// reported rather than dropped)
__device__ __forceinline__ double vmax(double a, double b) { return (a > b || a != a) ? a : b; }

// side[k*3 + f]: max ||n^T G n||_2 over face f's nodes of element k (with
// the ghost state on wall and far-field faces); loc[k*3 + 0..2]: g_K (node max
// of the directional norms), beta_K, beta'_K.  One thread per (element, node),
// floor(256 / Np) elements per workgroup; the per-element maxima are taken
// through LDS by the element's node-0 thread.
template <int N>
__global__ __launch_bounds__(kCflThreads) void cfl_local_kernel(DeviceTables t, KernelPhysics ph,
                                                                const double* __restrict__ U,
                                                                double* __restrict__ side,
                                                                double* __restrict__ loc,
                                                                double* __restrict__ result) {
  constexpr int Np = (N + 1) * (N + 2) / 2, Nfp = N + 1, NF = 3 * Nfp;
  constexpr int EPB = kCflThreads / Np;
  __shared__ double su[EPB * Np], sv[EPB * Np], sb[EPB * Np], sg[EPB * Np], sd[EPB * Np];
  __shared__ double sf[EPB * NF];
  const int e = threadIdx.x / Np, n = threadIdx.x % Np;
  const int64_t k = (int64_t)blockIdx.x * EPB + e;
  const bool act = e < EPB && k < t.K;
  if (blockIdx.x == 0 && threadIdx.x == 0) result[0] = 0.0;
  Gas<double> gas;
  gas.gamma = ph.gamma;
  gas.gm1 = ph.gamma - 1.0;
  gas.igm1 = 1.0 / (ph.gamma - 1.0);
  gas.mu = ph.mu;
  gas.k = ph.gamma / ph.Pr;
  const double* Uk = U + k * 4 * Np;
  const double* g = t.geo + k * kGeoStride;
  const int es = e * Np;
  if (act) {
    const double S[4] = {Uk[n], Uk[Np + n], Uk[2 * Np + n], Uk[3 * Np + n]};
    const double ir = 1.0 / S[0];
    const double u = S[1] * ir, v = S[2] * ir;
    const double p = gas.gm1 * (S[3] - 0.5 * (S[1] * u + S[2] * v));
    const double du = u - ph.vw[0], dv = v - ph.vw[1];
    su[es + n] = u;
    sv[es + n] = v;
    sb[es + n] = sqrt(du * du + dv * dv) + sqrt(gas.gamma * p * ir);
    const VState<double> st = vstate(gas, S);
    sg[es + n] = vmax(normal_diffusion_norm(gas, st, 1.0, 0.0),
                      normal_diffusion_norm(gas, st, 0.0, 1.0));
  }
  __syncthreads();
  if (act) {
    const double* Dr = t.ops;
    const double* Ds = t.ops + Np * Np;
    double ur = 0.0, us = 0.0, vr = 0.0, vs = 0.0;
#pragma unroll
    for (int m = 0; m < Np; ++m) {
      const double dr = Dr[n * Np + m], ds = Ds[n * Np + m];
      ur += dr * su[es + m];
      us += ds * su[es + m];
      vr += dr * sv[es + m];
      vs += ds * sv[es + m];
    }
    sd[es + n] = fabs(g[0] * ur + g[2] * us + g[1] * vr + g[3] * vs);
    for (int i = n; i < NF; i += Np) {
      const int f = i / Nfp, j = i % Nfp;
      const int node = cfl_face_node<N>(f, j);
      const double nx = g[4 + 4 * f], ny = g[5 + 4 * f];
      const int tag = t.conn[k * 3 + f] & 3;
      const double S[4] = {Uk[node], Uk[Np + node], Uk[2 * Np + node], Uk[3 * Np + node]};
      double sfv = normal_diffusion_norm(gas, vstate(gas, S), nx, ny);
      if (tag == 1) {
        // wall ghost: own density and pressure, wall velocity
        const double p = gas.gm1 * (S[3] - 0.5 * (S[1] * S[1] + S[2] * S[2]) / S[0]);
        const double B[4] = {S[0], S[0] * ph.vw[0], S[0] * ph.vw[1],
                             p * gas.igm1 + 0.5 * S[0] * (ph.vw[0] * ph.vw[0] + ph.vw[1] * ph.vw[1])};
        sfv = vmax(sfv, normal_diffusion_norm(gas, vstate(gas, B), nx, ny));
      } else if (tag == 2) {
        sfv = vmax(sfv, normal_diffusion_norm(gas, vstate(gas, ph.U_inf), nx, ny));
      }
      sf[e * NF + i] = sfv;
    }
  }
  __syncthreads();
  if (act && n == 0) {
    double gm = 0.0, be = 0.0, dv = 0.0;
    for (int m = 0; m < Np; ++m) {
      gm = vmax(gm, sg[es + m]);
      be = vmax(be, sb[es + m]);
      dv = vmax(dv, sd[es + m]);
    }
    loc[k * 3 + 0] = gm;
    loc[k * 3 + 1] = be;
    loc[k * 3 + 2] = 0.5 * dv;
    for (int f = 0; f < 3; ++f) {
      double m = 0.0;
      for (int j = 0; j < Nfp; ++j) m = vmax(m, sf[e * NF + f * Nfp + j]);
      side[k * 3 + f] = m;
    }
  }
}

__global__ __launch_bounds__(kCflThreads) void cfl_reduce_kernel(DeviceTables t, int N, double C_grad,
                                                                 const double* __restrict__ side,
                                                                 const double* __restrict__ loc,
                                                                 double* __restrict__ result) {
  __shared__ double part[kCflThreads / 64];
  const int64_t k = (int64_t)blockIdx.x * kCflThreads + threadIdx.x;
  double lam = 0.0;
  if (k < t.K) {
    const double* g = t.geo + k * kGeoStride;
    const int Np = (N + 1) * (N + 2) / 2;
    double sigma = 0.0, G = loc[k * 3], fmax = 0.0, fsum = 0.0;
    for (int f = 0; f < 3; ++f) {
      const int32_t c = t.conn[k * 3 + f];
      const int64_t nb = c >> 4;
      const int nf = (c >> 2) & 3;
      const double gbar = vmax(side[k * 3 + f], side[nb * 3 + nf]);
      sigma = vmax(sigma, g[7 + 4 * f] * gbar);
      G = vmax(G, loc[nb * 3]);
      fmax = vmax(fmax, g[6 + 4 * f]);
      fsum += g[6 + 4 * f];
    }
    const double cinv = Np * fmax;
    // C_grad p^4 / rho_K^2 with rho_K = 2 / sum_f Fscale_f
    const double p2 = (double)N * (double)N;
    const double cinv2 = C_grad * p2 * p2 * 0.25 * fsum * fsum;
    lam = 1.5 * cinv2 * G + 3.0 * cinv * (3.0 * sigma + loc[k * 3 + 1]) + loc[k * 3 + 2];
  }
  for (int o = 32; o > 0; o >>= 1) lam = vmax(lam, __shfl_down(lam, o, 64));
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = lam;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = part[0];
    for (int w = 1; w < kCflThreads / 64; ++w) m = vmax(m, part[w]);
    // non-negative doubles order as their bit patterns (a NaN compares
    // above every finite value and is reported by the caller)
    atomicMax((unsigned long long*)result, (unsigned long long)__double_as_longlong(m));
  }
}

template <int N>
int launch_cfl_n(const DeviceTables& t, const KernelPhysics& ph, const double* U, double C_grad,
                 double* work, hipStream_t s, std::string& err) {
  constexpr int EPB = kCflThreads / ((N + 1) * (N + 2) / 2);
  const unsigned lblocks = (unsigned)((t.K + EPB - 1) / EPB);
  const unsigned blocks = (unsigned)((t.K + kCflThreads - 1) / kCflThreads);
  double* side = work;
  double* loc = work + 3 * t.K;
  double* result = work + 6 * t.K;
  hipLaunchKernelGGL(cfl_local_kernel<N>, dim3(lblocks), dim3(kCflThreads), 0, s, t, ph, U, side,
                     loc, result);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    hipLaunchKernelGGL(cfl_reduce_kernel, dim3(blocks), dim3(kCflThreads), 0, s, t, N, C_grad, side,
                       loc, result);
    e = hipGetLastError();
  }
  if (e != hipSuccess) {
    err = std::string("CFL kernels: ") + hipGetErrorString(e);
    return -3;
  }
  return 0;
}

}  // namespace

size_t cfl_work_size(int64_t K) { return (size_t)(6 * K + 1); }

int launch_cfl(int N, const DeviceTables& t, const KernelPhysics& ph, const double* U, double C_grad,
               double* work, void* stream, std::string& err) {
  if (t.K <= 0) {
    err = "empty mesh";
    return -1;
  }
  hipStream_t s = (hipStream_t)stream;
  switch (N) {
    case 1: return launch_cfl_n<1>(t, ph, U, C_grad, work, s, err);
    case 2: return launch_cfl_n<2>(t, ph, U, C_grad, work, s, err);
    case 3: return launch_cfl_n<3>(t, ph, U, C_grad, work, s, err);
    case 4: return launch_cfl_n<4>(t, ph, U, C_grad, work, s, err);
    case 5: return launch_cfl_n<5>(t, ph, U, C_grad, work, s, err);
    case 6: return launch_cfl_n<6>(t, ph, U, C_grad, work, s, err);
    default: err = "order outside 1..6"; return -5;
  }
}

}  // namespace dgmi
