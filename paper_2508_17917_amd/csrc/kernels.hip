// HIP kernels for gfx950: the fused right-hand side + low-storage RK stage,
// and the wall-force reduction.
//
// Stage kernel, per wavefront and tile of four element slots, in the order of
// Alg. 2 (the neighbour exchange becomes reads of the neighbours' nodal
// states, resident in HBM / L2 on one GPU):
//   1  own states, neighbour states and geometry -> LDS
//   2  broken gradient on the matrix cores: rows (element, field), columns
//      nodes, [dU/dr, dU/ds] = U [Dr^T, Ds^T]; the output lane owns one node
//      of one element with all four fields -> total flux
//      F = F_c - v_w (x) U - G grad U and its contravariant components
//   3  face nodes (one lane each): neighbour trace and gradient (reversed face
//      node order), boundary ghosts (Sec. 2.2.4), G-bar_e = max over the face of
//      ||n^T G n||_2 on both sides, sigma_e, Roe flux, viscous average,
//      penalty and theta term
//   4  strong-form residual on the matrix cores,
//      R = -(Dr Fr + Ds Fs) + LIFT h + LIFTr qr + LIFTs qs
//      (M^-1 and 1/J folded into the operators and Fscale), then
//      K1 <- a K1 + dt R, U_out <- U_in + b K1 (Alg. 1) in FP64.
// Every element writes only its own nodes and each face is evaluated from both
// sides, so there are no atomics and results are bitwise reproducible.
//
// Variants (template parameters): the real type T of the right-hand side
// (double, float) and the form (plain: the state itself; perturbation: the
// state minus the free stream, fluxes as cancellation-free differences).  The
// RK registers K0 = U and K1 are FP64 in every variant.
#include <hip/hip_runtime.h>

#include <cstdio>

#include "dg_internal.h"
#include "dg_physics.h"

namespace dgmi {

// Real types of the right-hand side: double, float, or float with the
// operator products on the bfloat16 matrix cores (FP32 accumulation).
struct bf16ops {};
template <typename X>
struct Real {
  typedef X type;
  static constexpr bool bf = false;
};
template <>
struct Real<bf16ops> {
  typedef float type;
  static constexpr bool bf = true;
};

template <int N, typename X>
struct Order {
  typedef typename Real<X>::type T;
  static constexpr bool BF = Real<X>::bf;
  static constexpr int Np = (N + 1) * (N + 2) / 2;
  static constexpr int Nfp = N + 1;
  static constexpr int NF = 3 * (N + 1);
  static constexpr int S = 4 * Np;               // values per element state
  static constexpr int NT = (Np + 15) / 16;      // 16-node output tiles
  static constexpr int KS = (Np + 3) / 4;        // k-steps over volume nodes
  static constexpr int KF = (NF + 3) / 4;        // k-steps over face nodes
  static constexpr int KS16 = (Np + 15) / 16;    // bfloat16 k-steps (16 deep)
  static constexpr int KF16 = (NF + 15) / 16;
  // padded LDS rows (odd: no bank aliasing), long enough for the k-steps
  static constexpr int RS = (BF && 16 * KS16 > 4 * KS ? 16 * KS16 : 4 * KS) + 1;
  static constexpr int HRS = (BF && 16 * KF16 > 4 * KF ? 16 * KF16 : 4 * KF) + 1;
  static constexpr int EPT = elements_per_tile(N);  // elements per tile (4 slots)
  static constexpr int FIT = (EPT * NF + 63) / 64;  // face items per lane
  // the volume flux in one pass over (element, node) pairs packed onto the
  // lanes, where they fit 64 lanes but the matrix-core layout (16 node
  // columns x 4 element slots per output tile) needs several tiles: p = 5
  // (3 x 21 of 64 lanes in one pass instead of 63 of 128 in two)
  static constexpr bool PACK = (EPT * Np <= 64) && (NT > 1);
  // default waves per workgroup (each wave owns its own tiles; the workgroup
  // shares the operator fragments)
  // (4 measured fastest for every order and form on MI355X: the fragments
  // are shared by more waves, and at p >= 5 in FP64 LDS and registers allow
  // one workgroup per CU either way)
  static constexpr int WAVES = 4;
  // waves per SIMD the register allocation must allow: 3 for FP32 at p <= 4
  // (a few spills, measured faster than 2 and than 4), else 2
  static constexpr int MIN_WAVES_EU = (sizeof(T) == 4 && N <= 4) ? 3 : 2;
  // the next tile's own data issued before the face pass where the
  // registers allow (K1 / K0 of the tile always are)
  static constexpr bool EARLY_OWN = N <= 4;
  // per-wave LDS (elements of T)
  static constexpr int U_SZ = 16 * RS;           // own state
  static constexpr int F_SZ = 32 * RS;           // contravariant flux Fr rows | Fs rows
  static constexpr int N_SZ = 12 * S;            // neighbour states [e][f][c][n]
  static constexpr int H_SZ = 48 * HRS;          // face terms h | qr | qs
  static constexpr int X_SZ = N_SZ > H_SZ ? N_SZ : H_SZ;
  static constexpr int NORM_SZ = 4 * NF;
  static constexpr int WAVE_SZ = U_SZ + F_SZ + X_SZ + NORM_SZ + 64 + 48;
  // operator fragments (per workgroup)
  // one Dr-type / LIFT-type fragment set, in elements of T (bfloat16: four
  // values per lane, i.e. two floats' worth)
  static constexpr int FD = BF ? NT * KS16 * 64 * 2 : NT * KS * 64;
  static constexpr int FL = BF ? NT * KF16 * 64 * 2 : NT * KF * 64;
  static constexpr int FRAG_SZ = 2 * FD + 3 * FL;
  // matrix-core row of (field c, element e): the FP64 instruction returns rows
  // l/16 + 4v to lane l, the FP32 one rows 4(l/16) + v; either way lane l ends
  // up with element l/16 and field v
  static constexpr int ROWC = sizeof(T) == 8 ? 4 : 1;
  static constexpr int ROWE = sizeof(T) == 8 ? 1 : 4;
};

// Fourth word of a raw buffer descriptor on gfx9-family devices: 32-bit data
// format (untyped loads need a valid one), no swizzle, no index stride.
constexpr int kBufferWord3 = 0x00020000;

// A raw buffer descriptor over n consecutive records of `bytes_each` bytes
// starting at record r0 of the array at p (built on the scalar unit when its
// arguments are uniform).  Accesses past the n records read 0 and write
// nothing (the hardware's range check), so n <= 0 gives an empty range.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t records(const void* p, int64_t r0, int64_t n,
                                                          int bytes_each) {
  const int bytes = n > 0 ? (int)(n * bytes_each) : 0;
  return __builtin_amdgcn_make_buffer_rsrc((void*)((const char*)p + r0 * bytes_each), (short)0, bytes,
                                           kBufferWord3);
}
__device__ __forceinline__ double buf_load_f64(__amdgpu_buffer_rsrc_t r, int byte_off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 0));
}

// Node index of face node j (counter-clockwise) on face f; rows of the node
// numbering start at i(N+1) - i(i-1)/2.
template <int N>
__device__ __forceinline__ int face_node(int f, int j) {
  if (f == 0) return j;
  if (f == 1) return j * (N + 1) - j * (j - 1) / 2 + (N - j);
  int i = N - j;
  return i * (N + 1) - i * (i - 1) / 2;
}

template <typename T>
struct Vec4 {
  typedef T type __attribute__((ext_vector_type(4)));
};

// D += A B for A 16x4, B 4x16, D 16x16 on the matrix cores.  Lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; it holds D[l/16 + 4v][l%16] (FP64) or
// D[4(l/16) + v][l%16] (FP32), v = 0..3.
__device__ __forceinline__ Vec4<double>::type mfma(double a, double b, Vec4<double>::type c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ Vec4<float>::type mfma(float a, float b, Vec4<float>::type c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// bfloat16 operands (16x16x16, FP32 accumulation): lane l supplies
// A[l%16][4(l/16) + j] and B[4(l/16) + j][l%16]; the result layout is that of
// the FP32 instruction.
typedef short bf16x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ unsigned short to_bf16(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest, ties to even
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ bf16x4_t bf16_row(const float* p) {
  return bf16x4_t{(short)to_bf16(p[0]), (short)to_bf16(p[1]), (short)to_bf16(p[2]),
                  (short)to_bf16(p[3])};
}
__device__ __forceinline__ bf16x4_t bf16_frag(const float* frag, int lane) {
  const uint2 w = ((const uint2*)frag)[lane];
  return bf16x4_t{(short)(w.x & 0xffff), (short)(w.x >> 16), (short)(w.y & 0xffff),
                  (short)(w.y >> 16)};
}
__device__ __forceinline__ Vec4<float>::type mfma_bf16(bf16x4_t a, bf16x4_t b,
                                                       Vec4<float>::type c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
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
__device__ __forceinline__ float lane_read(float v, int src) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}

template <typename T, bool PERT>
__device__ __forceinline__ void full_state(const T u[4], const Base<T>& b, T uf[4]) {
  if (PERT) {
    uf[0] = b.rho + u[0];
    uf[1] = b.mx + u[1];
    uf[2] = b.my + u[2];
    uf[3] = b.E + u[3];
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c) uf[c] = u[c];
  }
}

template <typename T, bool PERT>
__device__ __forceinline__ Prim<T> prim_of(const T uf[4], const T u[4], const Base<T>& b, T gm1) {
  return PERT ? prim_pert(uf, u, b, gm1) : prim_plain(uf, gm1);
}

template <typename T, bool PERT>
__device__ __forceinline__ void normal_flux(const T uf[4], const T u[4], const Prim<T>& s,
                                            const Base<T>& b, T nx, T ny, T vwn, T F[4]) {
  if (PERT)
    normal_flux_pert(u, s, b, nx, ny, vwn, F);
  else
    normal_flux_plain(uf, s, nx, ny, vwn, F);
}

// Value of the state on the other side of a face node (in what the kernel
// stores: the state, or its perturbation from U_inf): the neighbour's trace
// (interior, periodic), the moving adiabatic wall's ghost Q^b = [rho+, v_w,
// p+], or the far field U_inf (Sec. 2.2.4).  nb points at the neighbour's
// node, stride Np; up is the own value, upf the own full state.
template <typename T, bool PERT>
__device__ __forceinline__ void ghost_state(int tag, const T up[4], const T upf[4], const T* nb,
                                            int Np, T vwx, T vwy, const Gas<T>& gas,
                                            const Base<T>& b, T uo[4]) {
  if (tag == 0) {
#pragma unroll
    for (int c = 0; c < 4; ++c) uo[c] = nb[c * Np];
  } else if (tag == 1) {
    const T rho = upf[0];
    const T kw = T(0.5) * rho * (vwx * vwx + vwy * vwy);
    const Prim<T> s = prim_of<T, PERT>(upf, up, b, gas.gm1);
    if (!PERT) {
      uo[0] = rho;
      uo[1] = rho * vwx;
      uo[2] = rho * vwy;
      uo[3] = s.p * gas.igm1 + kw;
    } else {
      uo[0] = up[0];
      uo[1] = rho * vwx - b.mx;
      uo[2] = rho * vwy - b.my;
      // eps_b - eps_inf = p'/(gamma-1) + rho |v_w|^2/2 - rho_inf |u_inf|^2/2
      uo[3] = s.jp * gas.igm1 + kw - T(0.5) * (b.mx * b.ux + b.my * b.uy);
    }
  } else {
    if (PERT) {
#pragma unroll
      for (int c = 0; c < 4; ++c) uo[c] = T(0);
    } else {
      uo[0] = b.rho;
      uo[1] = b.mx;
      uo[2] = b.my;
      uo[3] = b.E;
    }
  }
}

template <typename X>
__device__ __forceinline__ const typename Real<X>::type* frag_of(const DeviceTables& t);
template <>
__device__ __forceinline__ const double* frag_of<double>(const DeviceTables& t) {
  return t.frag;
}
template <>
__device__ __forceinline__ const float* frag_of<float>(const DeviceTables& t) {
  return t.frag32;
}
// bfloat16 fragments, moved as 32-bit words (never used as floats)
template <>
__device__ __forceinline__ const float* frag_of<bf16ops>(const DeviceTables& t) {
  return (const float*)t.frag16;
}

// K1 (and, in the perturbation form, K0) of output lane (element slot re,
// nodes 16 tt + rn) of the tile at element e0, into registers; returns whether
// the element is outside the curved set.  K1 is read only when the stage uses
// it (a != 0, not a bare right-hand side): otherwise the load reads the
// element's own state, which the tile has just brought into the cache, and is
// not used.
template <int N, typename X, bool PERT>
__device__ __forceinline__ bool load_k(const DeviceTables& t, const double* __restrict__ Uin,
                                       const double* __restrict__ K1, double a, int rhs_only,
                                       int64_t e0, int nel, int re, int rn,
                                       double (&rk)[Order<N, X>::NT][4],
                                       double (&r0)[Order<N, X>::NT][4]) {
  using O = Order<N, X>;
  constexpr int Np = O::Np, S = O::S;
  // descriptors over the tile's elements: the lane's offsets are constants
  const __amdgpu_buffer_rsrc_t rk_d = records((a != 0.0 && !rhs_only) ? K1 : Uin, e0, nel, S * 8);
  const __amdgpu_buffer_rsrc_t r0_d = records(Uin, e0, nel, S * 8);
#pragma unroll
  for (int tt = 0; tt < O::NT; ++tt) {
    const int n = 16 * tt + rn < Np ? 16 * tt + rn : Np - 1;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int off = (re * S + c * Np + n) * 8;
      rk[tt][c] = buf_load_f64(rk_d, off);
      r0[tt][c] = PERT ? buf_load_f64(r0_d, off) : 0.0;
    }
  }
  const int64_t ke = (e0 + re) < t.K ? (e0 + re) : t.K - 1;
  return t.cslot == nullptr || t.cslot[ke] < 0;
}

// The wall force (the traction of eq. force_integral: pressure minus the
// viscous normal stress, and its moment about the origin) at wall face node i
// (node i % Nfp of face t.wall[i / Nfp]) of the state U: the node's quadrature
// weight times sJ times (tx, ty, x ty - y tx), in FP64 in every form.  UNR:
// the unroll factor of the node's derivative loop (the same operations in the
// same order whatever it is; a smaller one holds fewer registers where the
// force runs inside the stage kernel).
constexpr int kForceThreads = 64;
template <int N, int UNR = (N + 1) * (N + 2) / 2>
__device__ __forceinline__ void wall_node_force(const DeviceTables& t, const KernelPhysics& ph,
                                                const double* __restrict__ U, int i, double& fx,
                                                double& fy, double& mz) {
  using O = Order<N, double>;
  constexpr int Np = O::Np, Nfp = O::Nfp, S = 4 * Np;
  Gas<double> gas;
  gas.gamma = ph.gamma;
  gas.gm1 = ph.gamma - 1.0;
  gas.igm1 = 1.0 / (ph.gamma - 1.0);
  gas.mu = ph.mu;
  gas.k = ph.gamma / ph.Pr;
  const double* Dr = t.ops;
  const double* Ds = t.ops + Np * Np;
  const double* wface = t.ops + 2 * Np * Np + 3 * Np * 3 * Nfp;
  const int wf = t.wall[i / Nfp];
  const int j = i % Nfp;
  const int64_t k = wf / 3;
  const int f = wf % 3;
  const int n = face_node<N>(f, j);
  const double* Uk = U + k * S;
  const double* g = t.geo + k * kGeoStride;
  // metric terms at the node, normal and sJ at the face node: per node on
  // the elements of the curved set, the element's constants elsewhere
  double rx = g[0], ry = g[1], sx = g[2], sy = g[3];
  double nx = g[4 + 4 * f], ny = g[5 + 4 * f];
  double sJ = g[6 + 4 * f] / (g[0] * g[3] - g[1] * g[2]);  // Fscale * J
  const int cs = t.cslot ? t.cslot[k] : -1;
  if (cs >= 0) {
    const double* nd = t.cnode + (int64_t)cs * 5 * Np;
    const double* fc = t.cface + (int64_t)cs * 9 * Nfp;
    rx = nd[n];
    ry = nd[Np + n];
    sx = nd[2 * Np + n];
    sy = nd[3 * Np + n];
    nx = fc[f * Nfp + j];
    ny = fc[3 * Nfp + f * Nfp + j];
    sJ = fc[6 * Nfp + f * Nfp + j];
  }
  double ur[4] = {0, 0, 0, 0}, us[4] = {0, 0, 0, 0};
#pragma unroll UNR
  for (int m = 0; m < Np; ++m) {
    const double dr = Dr[n * Np + m], ds = Ds[n * Np + m];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      ur[c] += dr * Uk[c * Np + m];
      us[c] += ds * Uk[c * Np + m];
    }
  }
  double Up[4], dx[4], dy[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    Up[c] = Uk[c * Np + n];
    dx[c] = rx * ur[c] + sx * us[c];
    dy[c] = ry * ur[c] + sy * us[c];
  }
  const double p = gas.gm1 * (Up[3] - 0.5 * (Up[1] * Up[1] + Up[2] * Up[2]) / Up[0]);
  double Ub[4] = {Up[0], Up[0] * ph.vw[0], Up[0] * ph.vw[1],
                  p * gas.igm1 + 0.5 * Up[0] * (ph.vw[0] * ph.vw[0] + ph.vw[1] * ph.vw[1])};
  double vx[4], vy[4];
  viscous_flux(gas, vstate(gas, Ub), dx, dy, vx, vy);
  const double w = wface[f * Nfp + j] * sJ;
  const double tx = p * nx - (vx[1] * nx + vy[1] * ny);
  const double ty = p * ny - (vx[2] * nx + vy[2] * ny);
  const double xw = t.wall_xy[2 * i], yw = t.wall_xy[2 * i + 1];
  fx = w * tx;
  fy = w * ty;
  mz = w * (xw * ty - yw * tx);
}

// The force from the nblk partials an earlier launch wrote, in block order:
// lane c < 3 writes component c (eight loads in flight at a time, the sum
// itself in block order, as the ticket's last wave adds them).
__device__ __forceinline__ void force_sum(const double* __restrict__ part, double* out,
                                          unsigned nblk) {
  const int lane = threadIdx.x & 63;
  if (lane < 3) {
    double sum = 0.0;
    for (unsigned b = 0; b < nblk; b += 8) {
      double v[8];
#pragma unroll
      for (unsigned q = 0; q < 8; ++q) v[q] = b + q < nblk ? part[3 * (b + q) + lane] : 0.0;
#pragma unroll
      for (unsigned q = 0; q < 8; ++q)
        if (b + q < nblk) sum += v[q];
    }
    out[lane] = sum;
  }
}

// One wave's share of the wall force: nodes 64 blk .. 64 blk + 63 of the nblk
// blocks of 64 that cover the wall face nodes, reduced by a fixed shuffle
// tree into partial blk.  With TICKET the last wave to finish (an atomic
// ticket) sums the partials in block order into out[0..2] and resets the
// ticket; without, the partials are left for a later launch to sum (the
// ticket's device-scope fences write back and invalidate the L2 of the
// wave's XCD, and its chain of round trips outlasts a stage launch's first
// tiles).  The order of every sum is fixed by the wall face list alone, so
// the total does not depend on which waves ran the blocks or in which launch.
template <int N, int UNR = (N + 1) * (N + 2) / 2, bool TICKET = true>
__device__ __forceinline__ void force_wave(const DeviceTables& t, const KernelPhysics& ph,
                                           const double* __restrict__ U, double* __restrict__ out,
                                           unsigned blk, unsigned nblk) {
  const int lane = threadIdx.x & 63;
  double fx = 0.0, fy = 0.0, mz = 0.0;
  const int i = (int)blk * kForceThreads + lane;
  if (i < t.nwall * (N + 1)) wall_node_force<N, UNR>(t, ph, U, i, fx, fy, mz);
  for (int o = 32; o > 0; o >>= 1) {
    fx += __shfl_down(fx, o, 64);
    fy += __shfl_down(fy, o, 64);
    mz += __shfl_down(mz, o, 64);
  }
  if (lane == 0) {
    t.force_part[3 * blk + 0] = fx;
    t.force_part[3 * blk + 1] = fy;
    t.force_part[3 * blk + 2] = mz;
  }
  if constexpr (!TICKET) return;
  unsigned last = 0;
  if (lane == 0) {
    __threadfence();
    last = atomicAdd(t.force_ticket, 1u) == nblk - 1;
  }
  last = __shfl(last, 0, 64);
  if (last && lane < 3) {
    __threadfence();
    const volatile double* part = t.force_part;
    double sum = 0.0;
    for (unsigned b = 0; b < nblk; ++b) sum += part[3 * b + lane];
    out[lane] = sum;
    if (lane == 0) atomicExch(t.force_ticket, 0u);
  }
}

// The fused right-hand side + LSERK stage for the tiles tile0, tile0 + stride,
// ... < tile_end of one mesh, run by one wavefront.  A tile has four element
// slots (16 matrix-core rows = 4 fields x 4 elements) and holds EPT elements:
// four, or three at orders 5 and 6 so that its face nodes fit one pass over
// the lanes (the fourth slot then idles like those of a ragged last tile).
// sFrag holds the operator
// fragments (shared by the workgroup), sU this wave's LDS area (WAVE_SZ
// elements, pads zeroed once), sConn 12 ints of this wave.
template <int N, typename X, bool PERT>
__device__ __forceinline__ void stage_tiles(const DeviceTables& t, const KernelPhysics& ph,
                                            const double* __restrict__ Uin,
                                            double* __restrict__ Uout, double* __restrict__ K1,
                                            double a, double b, double dt, int rhs_only,
                                            const typename Real<X>::type* sFrag,
                                            typename Real<X>::type* sU, int* sConn,
                                            int64_t tile0, int64_t tile_end, int64_t stride) {
  typedef typename Real<X>::type T;
  using O = Order<N, X>;
  constexpr bool BF = O::BF;
  constexpr int KS16 = O::KS16, KF16 = O::KF16;
  typedef typename Vec4<T>::type V4;
  constexpr int Np = O::Np, Nfp = O::Nfp, NF = O::NF, S = O::S, NT = O::NT, KS = O::KS,
                KF = O::KF, RS = O::RS, HRS = O::HRS, FIT = O::FIT, ROWC = O::ROWC,
                ROWE = O::ROWE, EPT = O::EPT;
  constexpr bool PACK = O::PACK;
  constexpr int OFF_DR = 0, OFF_DS = O::FD, OFF_L = 2 * O::FD, OFF_LR = 2 * O::FD + O::FL,
                OFF_LS = 2 * O::FD + 2 * O::FL;
  const int lane = threadIdx.x & 63;

  T* sFr = sU + O::U_SZ;
  T* sFs = sFr + 16 * RS;
  T* sX = sU + O::U_SZ + O::F_SZ;   // neighbour states, later face terms
  T* sH = sX;
  T* sQr = sX + 16 * HRS;
  T* sQs = sX + 32 * HRS;
  T* sNorm = sX + O::X_SZ;
  T* sGeo = sNorm + O::NORM_SZ;     // [4][16]
  T* sNGeo = sGeo + 64;             // [4][3][4]

  Gas<T> gas;
  gas.gamma = (T)ph.gamma;
  gas.gm1 = (T)ph.gm1;
  gas.igm1 = (T)ph.igm1;
  gas.mu = (T)ph.mu;
  gas.k = (T)ph.k;
  const T theta = (T)ph.theta;
  const T k_wall = (T)ph.k_wall;
  const T vwx = (T)ph.vw[0], vwy = (T)ph.vw[1];
  Base<T> base;
  base.rho = (T)ph.U_inf[0];
  base.mx = (T)ph.U_inf[1];
  base.my = (T)ph.U_inf[2];
  base.E = (T)ph.U_inf[3];
  base.p = (T)ph.p_inf;
  base.ux = (T)ph.u_inf;
  base.uy = (T)ph.v_inf;
  const int64_t K = t.K;

  const int arow = lane & 15, acol = lane >> 4;  // A-operand row, k offset
  const int re = lane >> 4, rn = lane & 15;      // output: element re, node 16 t + rn
  // state loads: value r = lane + 64 q of an element block is field r / Np,
  // node r % Np
  constexpr int NQ = (S + 63) / 64;
  bool lr_ok[NQ];
  int lds_u[NQ];
  double uinf_q[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int r = lane + 64 * q;
    lr_ok[q] = r < S;
    lds_u[q] = lr_ok[q] ? ROWC * (r / Np) * RS + (r - (r / Np) * Np) : 0;
    const int c = r / Np;  // selects, not an indexed load: ph may be a local copy
    const double u_c = c == 0 ? ph.U_inf[0] : (c == 1 ? ph.U_inf[1] : (c == 2 ? ph.U_inf[2] : ph.U_inf[3]));
    uinf_q[q] = (PERT && lr_ok[q]) ? u_c : 0.0;
  }

  // The global loads of a tile are software-pipelined: a tile's own states,
  // geometry and connectivity are issued at the end of the previous tile
  // (after that tile's K1 / K0 loads, before its final matrix-core phase),
  // and its neighbour states before its volume phase, so that their latency
  // overlaps computation.  Every load is unconditional, its address clamped
  // into the arrays (element K - 1, the block's last value, the tables' last
  // entry) where the lane has nothing to load: with no control flow around
  // the loads, the wait before each value's first use covers only the loads
  // issued before it, not those issued ahead for later phases.  Values of
  // clamped lanes are never stored.
  constexpr int NB1 = NQ == 1 ? 12 : 6;  // neighbour blocks issued before the volume phase
  constexpr bool SPLIT = NB1 < 12;
  int vidx[NQ];                          // this lane's value within an element block
#pragma unroll
  for (int q = 0; q < NQ; ++q) vidx[q] = lr_ok[q] ? lane + 64 * q : S - 1;
  double ru[EPT][NQ];
  double rg = 0.0;
  int rc = 0;
  // through descriptors over the tile's elements (past the last element a
  // load reads 0, and such values are never stored)
  auto load_own = [&](int64_t tl) {
    const int64_t b = tl * EPT;
    const int64_t nb = K - b < EPT ? K - b : EPT;
    const __amdgpu_buffer_rsrc_t ud = records(Uin, b, nb, S * 8);
#pragma unroll
    for (int e = 0; e < EPT; ++e)
#pragma unroll
      for (int q = 0; q < NQ; ++q) ru[e][q] = buf_load_f64(ud, (e * S + vidx[q]) * 8);
    rg = buf_load_f64(records(t.geo, b, nb, kGeoStride * 8), lane * 8);
    rc = __builtin_amdgcn_raw_buffer_load_b32(records(t.conn, b, nb, 3 * 4), lane * 4, 0, 0);
  };
  load_own(tile0);

  for (int64_t tile = tile0; tile < tile_end; tile += stride) {
    const int64_t e0 = tile * EPT;
    const int nel = (int)((K - e0) < EPT ? (K - e0) : EPT);
    wave_sync();
    // ---- own states, geometry, connectivity (loaded ahead).  Lane l owns
    // values r = l + 64 q of every element block, so addresses are a per-lane
    // constant plus a wave-uniform base.
    if (lane < nel * 3) sConn[lane] = rc;
#pragma unroll
    for (int e = 0; e < EPT; ++e)
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        if (lr_ok[q] && e < nel) sU[lds_u[q] + ROWE * e * RS] = (T)(ru[e][q] - uinf_q[q]);
    if (lane < nel * kGeoStride) sGeo[lane] = (T)rg;
    wave_sync();
    // ---- neighbour states (a boundary face points at the element itself) and
    // metrics: the first NB1 blocks are issued now and stored after the volume
    // phase, the rest (high orders: bounded register use) after that
    // neighbour element of face slot i of the tile (slots beyond the tile's
    // elements: its first element, a valid address whose data go unused)
    auto nbr_elem = [&](int i) -> int64_t {
      return i < 3 * nel ? (int64_t)(sConn[i < 12 ? i : 0] >> 4) : e0;
    };
    // the same for a slot index uniform across the wave, as a scalar: lane i
    // of the wave holds the connectivity of face slot i (loaded with the
    // tile's own data), so the neighbour's address is formed on the scalar
    // unit and each load is a scalar base plus the lane's fixed offset
    const int nel_u = __builtin_amdgcn_readfirstlane(nel);
    const int e0_u = __builtin_amdgcn_readfirstlane((int)e0);
    auto nbr_elem_u = [&](int i) -> int {
      const int conn = __builtin_amdgcn_readlane(rc, i < 12 ? i : 0);
      return i < 3 * nel_u ? conn >> 4 : e0_u;
    };
    // value vidx[q] of element block ne (a scalar): a buffer load whose
    // descriptor spans that block only (built on the scalar unit), the lane's
    // fixed byte offset as the vector operand
    auto load_block = [&](int ne, int q) -> double {
      const __amdgpu_buffer_rsrc_t r =
          __builtin_amdgcn_make_buffer_rsrc((void*)(Uin + (int64_t)ne * S), (short)0, S * 8, kBufferWord3);
      return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vidx[q] * 8, 0, 0));
    };
    const double rng = t.geo[nbr_elem(lane >> 2) * kGeoStride + (lane & 3)];
    double rnb[NB1][NQ];
#pragma unroll
    for (int bb = 0; bb < NB1; ++bb) {
      const int nb = nbr_elem_u(bb);
#pragma unroll
      for (int q = 0; q < NQ; ++q) rnb[bb][q] = load_block(nb, q);
    }

    // ---- gradient on the matrix cores, then the volume flux per node:
    // F = F_c - v_w (x) U - G grad U at node n of element slot e, stored as
    // its contravariant components
    auto volume_flux = [&](int e, int n, const T gx[4], const T gy[4], T rx, T ry, T sx, T sy) {
      T u[4], uf[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) u[c] = sU[(ROWC * c + ROWE * e) * RS + n];
      full_state<T, PERT>(u, base, uf);
      T fvx[4], fvy[4];
      const VState<T> st = vstate(gas, uf);
      viscous_flux(gas, st, gx, gy, fvx, fvy);
      const Prim<T> pr = prim_of<T, PERT>(uf, u, base, gas.gm1);
      T Fx[4], Fy[4];
      normal_flux<T, PERT>(uf, u, pr, base, T(1), T(0), vwx, Fx);
      normal_flux<T, PERT>(uf, u, pr, base, T(0), T(1), vwy, Fy);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const T fx = Fx[c] - fvx[c], fy = Fy[c] - fvy[c];
        sFr[(ROWC * c + ROWE * e) * RS + n] = rx * fx + ry * fy;
        sFs[(ROWC * c + ROWE * e) * RS + n] = sx * fx + sy * fy;
      }
    };
    T gxk[NT][4], gyk[NT][4];
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) {
      V4 aR = {T(0), T(0), T(0), T(0)}, aS = {T(0), T(0), T(0), T(0)};
      if constexpr (BF) {
#pragma unroll
        for (int s = 0; s < KS16; ++s) {
          const bf16x4_t av = bf16_row((const float*)sU + arow * RS + 16 * s + 4 * acol);
          aR = mfma_bf16(av, bf16_frag((const float*)sFrag + OFF_DR + (tt * KS16 + s) * 128, lane), aR);
          aS = mfma_bf16(av, bf16_frag((const float*)sFrag + OFF_DS + (tt * KS16 + s) * 128, lane), aS);
        }
      } else {
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          const T av = sU[arow * RS + 4 * s + acol];
          aR = mfma(av, sFrag[OFF_DR + (tt * KS + s) * 64 + lane], aR);
          aS = mfma(av, sFrag[OFF_DS + (tt * KS + s) * 64 + lane], aS);
        }
      }
      const int n = 16 * tt + rn;
      const bool ok = (re < nel) && (n < Np);
      const T* g = sGeo + re * kGeoStride;
      const T rx = ok ? g[0] : T(0), ry = ok ? g[1] : T(0);
      const T sx = ok ? g[2] : T(0), sy = ok ? g[3] : T(0);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        gxk[tt][c] = rx * aR[c] + sx * aS[c];
        gyk[tt][c] = ry * aR[c] + sy * aS[c];
      }
      if (!SPLIT && !PACK && ok) volume_flux(re, n, gxk[tt], gyk[tt], rx, ry, sx, sy);
    }
    // high orders: the first neighbour blocks go to LDS and the rest are issued
    // between the matrix-core gradient and the volume flux, which covers them
    double rnb2[12 - NB1 > 0 ? 12 - NB1 : 1][NQ];
    if constexpr (SPLIT) {
#pragma unroll
      for (int bb = 0; bb < NB1; ++bb)
#pragma unroll
        for (int q = 0; q < NQ; ++q)
          if (lr_ok[q] && bb < 3 * nel) sX[bb * S + lane + 64 * q] = (T)(rnb[bb][q] - uinf_q[q]);
#pragma unroll
      for (int bb = 0; bb < 12 - NB1; ++bb) {
        const int nb = nbr_elem_u(NB1 + bb);
#pragma unroll
        for (int q = 0; q < NQ; ++q) rnb2[bb][q] = load_block(nb, q);
      }
      if constexpr (!PACK) {
#pragma unroll
        for (int tt = 0; tt < NT; ++tt) {
          const int n = 16 * tt + rn;
          if ((re < nel) && (n < Np)) {
            const T* g = sGeo + re * kGeoStride;
            volume_flux(re, n, gxk[tt], gyk[tt], g[0], g[1], g[2], g[3]);
          }
        }
      }
    }
    if constexpr (PACK) {
      // the tile's (element, node) pairs packed onto the lanes, one pass: the
      // lane of pair (e, n) fetches that node's gradient from the lane of the
      // matrix-core layout that holds it
      const int e = lane / Np, n = lane - e * Np;
      const int src = 16 * (e < 4 ? e : 3) + (n & 15);
      T gx[4], gy[4];
#pragma unroll
      for (int tt = 0; tt < NT; ++tt) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const T vx = lane_read(gxk[tt][c], src), vy = lane_read(gyk[tt][c], src);
          if ((n >> 4) == tt) {
            gx[c] = vx;
            gy[c] = vy;
          }
        }
      }
      if (e < nel) {
        const T* g = sGeo + e * kGeoStride;
        volume_flux(e, n, gx, gy, g[0], g[1], g[2], g[3]);
      }
    }
    if constexpr (!SPLIT) {
#pragma unroll
      for (int bb = 0; bb < NB1; ++bb)
#pragma unroll
        for (int q = 0; q < NQ; ++q)
          if (lr_ok[q] && bb < 3 * nel) sX[bb * S + lane + 64 * q] = (T)(rnb[bb][q] - uinf_q[q]);
    } else {
#pragma unroll
      for (int bb = 0; bb < 12 - NB1; ++bb) {
        const int ef = NB1 + bb;
#pragma unroll
        for (int q = 0; q < NQ; ++q)
          if (lr_ok[q] && ef < 3 * nel) sX[ef * S + lane + 64 * q] = (T)(rnb2[bb][q] - uinf_q[q]);
      }
    }
    if (lane < nel * 12) sNGeo[lane] = (T)rng;
    wave_sync();
    // K1 / K0 of the tile's outputs and the next tile's own data: at low orders
    // in FP32 the registers allow issuing them here, so that the face pass
    // covers their latency
    double rk[NT][4], r0[NT][4];
    bool mine;  // not an element of the curved set (which the curved kernel writes)
    mine = load_k<N, X, PERT>(t, Uin, K1, a, rhs_only, e0, nel, re, rn, rk, r0);
    if constexpr (O::EARLY_OWN) load_own(tile + stride);

    // ---- face nodes, one lane each (the EPT elements' 3(p+1) face nodes fit
    // the 64 lanes at every order built).  First half: traces, ghosts,
    // ||n^T G n||_2 on both sides, the neighbour's gradient at the node and
    // the mean viscous normal flux; the node's states and the viscous flux stay
    // in registers across the one wave sync that G-bar_e (a maximum over the
    // face's nodes) needs.  Second half: G-bar_e, sigma_e, Roe flux, penalty
    // and theta term, written over the neighbour area (every read of it is
    // done before the sync).
    static_assert(FIT == 1, "the face nodes of a tile must fit one pass over the lanes");
    {
      int e = lane / NF;
      const int fn = lane - e * NF;
      const bool ok = (lane < EPT * NF) && (e < nel);
      e = e < 4 ? e : 3;
      const int f = fn / Nfp, j = fn - f * Nfp;
      const int n = face_node<N>(f, j);
      // own gradient at the face node, from the lane that computed it
      T gxp[4], gyp[4];
      const int src = 16 * e + (n & 15);
#pragma unroll
      for (int tt = 0; tt < NT; ++tt) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const T vx = lane_read(gxk[tt][c], src), vy = lane_read(gyk[tt][c], src);
          if ((n >> 4) == tt) {
            gxp[c] = vx;
            gyp[c] = vy;
          }
        }
      }
      T up[4] = {T(0), T(0), T(0), T(0)}, uo[4] = {T(0), T(0), T(0), T(0)};
      T vn[4] = {T(0), T(0), T(0), T(0)};
      T nx = T(0), ny = T(0);
      int tag = 0;
      VState<T> sp = {}, so = {};
      if (ok) {
        const int conn = sConn[e * 3 + f];
        tag = conn & 3;
        const int nf = (conn >> 2) & 3;
        const T* g = sGeo + e * kGeoStride;
        nx = g[4 + 4 * f];
        ny = g[5 + 4 * f];
        T upf[4], uof[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) up[c] = sU[(ROWC * c + ROWE * e) * RS + n];
        full_state<T, PERT>(up, base, upf);
        const int n2 = (tag == 0) ? face_node<N>(nf, Nfp - 1 - j) : n;
        const T* nbU = sX + (e * 3 + f) * S;
        ghost_state<T, PERT>(tag, up, upf, nbU + n2, Np, vwx, vwy, gas, base, uo);
        full_state<T, PERT>(uo, base, uof);
        sp = vstate(gas, upf);
        so = vstate(gas, uof);
        // one side at a time: the two evaluations need not be live together
        T nrm = T(0);
#pragma nounroll
        for (int side = 0; side < 2; ++side) {
          const T a1 = normal_diffusion_norm(gas, side == 0 ? sp : so, nx, ny);
          nrm = a1 > nrm ? a1 : nrm;
        }
        sNorm[e * NF + fn] = nrm;
        // "other side" gradient from the staged neighbour (wall: the element itself)
        T ur[4] = {T(0), T(0), T(0), T(0)}, us[4] = {T(0), T(0), T(0), T(0)};
        const int dbase = ((n2 >> 4) * KS) * 64 + (n2 & 15);
#pragma unroll 4
        for (int m = 0; m < Np; ++m) {
          T dr, ds;
          if constexpr (BF) {
            // D_r[n2][m] in the bfloat16 fragment order (four values per lane)
            const unsigned short* f16 = (const unsigned short*)sFrag;
            const int wi = (((n2 >> 4) * KS16 + (m >> 4)) * 64 + 16 * ((m & 15) >> 2) + (n2 & 15)) * 4 +
                           (m & 3);
            dr = __uint_as_float((unsigned)f16[2 * OFF_DR + wi] << 16);
            ds = __uint_as_float((unsigned)f16[2 * OFF_DS + wi] << 16);
          } else {
            const int fi = dbase + (m >> 2) * 64 + (m & 3) * 16;
            dr = sFrag[OFF_DR + fi];
            ds = sFrag[OFF_DS + fi];
          }
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const T uu = nbU[c * Np + m];
            ur[c] += dr * uu;
            us[c] += ds * uu;
          }
        }
        const T* ng = sNGeo + (e * 3 + f) * 4;
        T gxm[4], gym[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          gxm[c] = ng[0] * ur[c] + ng[2] * us[c];
          gym[c] = ng[1] * ur[c] + ng[3] * us[c];
        }
        // mean of G(U+) grad U+ and G(U-) grad U- inside; G(U^b) grad U+ on the
        // wall (grad U+ from the staged copy of the element itself); G(U+) grad U+
        // on the far field
        if (tag == 1) {
          // adiabatic wall: stress and its work, no heat conduction
          viscous_normal_flux(gas_wall(gas, k_wall), so, gxm, gym, nx, ny, vn);
        } else {
          viscous_normal_flux(gas, sp, gxp, gyp, nx, ny, vn);
          if (tag == 0) {
            T vm[4];
            viscous_normal_flux(gas, so, gxm, gym, nx, ny, vm);
#pragma unroll
            for (int c = 0; c < 4; ++c) vn[c] = T(0.5) * (vn[c] + vm[c]);
          }
        }
      }
      wave_sync();
      if (ok) {
        const T* g = sGeo + e * kGeoStride;
        const T fsc = g[6 + 4 * f];
        // G-bar_e: largest norm over the face nodes of both sides
        T gbar = T(0);
#pragma unroll
        for (int jj = 0; jj < Nfp; ++jj) {
          const T v = sNorm[e * NF + f * Nfp + jj];
          gbar = v > gbar ? v : gbar;
        }
        const T sigma = g[7 + 4 * f] * gbar;
        const T vwn = vwx * nx + vwy * ny;
        T upf[4], uof[4];
        full_state<T, PERT>(up, base, upf);
        full_state<T, PERT>(uo, base, uof);
        const Prim<T> pp = prim_of<T, PERT>(upf, up, base, gas.gm1);
        T Fc[4];
        if (tag == 1) {
          // pressure through the moving wall (minus the free-stream flux in the
          // perturbation form)
          if (!PERT) {
            Fc[0] = T(0);
            Fc[1] = pp.p * nx;
            Fc[2] = pp.p * ny;
            Fc[3] = pp.p * vwn;
          } else {
            const T q0n = base.ux * nx + base.uy * ny - vwn;
            Fc[0] = -base.rho * q0n;
            Fc[1] = pp.jp * nx - base.mx * q0n;
            Fc[2] = pp.jp * ny - base.my * q0n;
            Fc[3] = pp.jp * vwn - (base.E + base.p) * q0n;
          }
        } else {
          const Prim<T> po = prim_of<T, PERT>(uof, uo, base, gas.gm1);
          T FL[4], FR[4];
          normal_flux<T, PERT>(upf, up, pp, base, nx, ny, vwn, FL);
          normal_flux<T, PERT>(uof, uo, po, base, nx, ny, vwn, FR);
          roe_flux(pp, po, FL, FR, nx, ny, vwn, gas.gm1, Fc);
        }
        // Fscale * own total normal flux from the contravariant flux:
        // face 0: -Fs, face 1: Fr + Fs, face 2: -Fr
        const T cfr = f == 0 ? T(0) : (f == 1 ? T(1) : T(-1));
        const T cfs = f == 2 ? T(0) : (f == 1 ? T(1) : T(-1));
        T fr[4], fs[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          fr[c] = sFr[(ROWC * c + ROWE * e) * RS + n];
          fs[c] = sFs[(ROWC * c + ROWE * e) * RS + n];
        }
        T w[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const T own = cfr * fr[c] + cfs * fs[c];
          w[c] = up[c] - uo[c];
          sH[(ROWC * c + ROWE * e) * HRS + fn] = own - fsc * (Fc[c] - vn[c] + sigma * w[c]);
        }
        T qx[4], qy[4];
        viscous_transpose(tag == 1 ? gas_wall(gas, k_wall) : gas, tag == 1 ? so : sp, nx, ny, w, qx, qy);
        const T ce = theta * (tag == 0 ? T(0.5) : T(1)) * fsc;
        const T rx = g[0], ry = g[1], sx = g[2], sy = g[3];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          sQr[(ROWC * c + ROWE * e) * HRS + fn] = ce * (rx * qx[c] + ry * qy[c]);
          sQs[(ROWC * c + ROWE * e) * HRS + fn] = ce * (sx * qx[c] + sy * qy[c]);
        }
      }
    }
    for (int i = lane; i < 48 * (HRS - NF); i += 64) {
      const int row = i / (HRS - NF);
      sX[row * HRS + NF + (i - row * (HRS - NF))] = T(0);
    }
    wave_sync();

    // ---- divergence and lifts on the matrix cores, then the RK stage in FP64;
    // the K1 / K0 loads (unless issued before the face pass), then those of
    // the next tile's own data, are issued first so the matrix work covers
    // their latency.
    if constexpr (!O::EARLY_OWN) load_own(tile + stride);
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) {
      V4 aD = {T(0), T(0), T(0), T(0)}, aL = {T(0), T(0), T(0), T(0)};
      if constexpr (BF) {
        const float* fr = (const float*)sFrag;
#pragma unroll
        for (int s = 0; s < KS16; ++s) {
          const int fo = (tt * KS16 + s) * 128;
          aD = mfma_bf16(bf16_row((const float*)sFr + arow * RS + 16 * s + 4 * acol),
                         bf16_frag(fr + OFF_DR + fo, lane), aD);
          aD = mfma_bf16(bf16_row((const float*)sFs + arow * RS + 16 * s + 4 * acol),
                         bf16_frag(fr + OFF_DS + fo, lane), aD);
        }
#pragma unroll
        for (int s = 0; s < KF16; ++s) {
          const int fo = (tt * KF16 + s) * 128;
          const int ao = arow * HRS + 16 * s + 4 * acol;
          aL = mfma_bf16(bf16_row((const float*)sH + ao), bf16_frag(fr + OFF_L + fo, lane), aL);
          aL = mfma_bf16(bf16_row((const float*)sQr + ao), bf16_frag(fr + OFF_LR + fo, lane), aL);
          aL = mfma_bf16(bf16_row((const float*)sQs + ao), bf16_frag(fr + OFF_LS + fo, lane), aL);
        }
      } else {
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
      }
      const int n = 16 * tt + rn;
      if (re < nel && n < Np && mine) {
        const int64_t base_i = (e0 + re) * S + n;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double R = (double)(aL[c] - aD[c]);
          const int64_t idx = base_i + c * Np;
          if (rhs_only) {
            K1[idx] = R;
          } else {
            const double k = (a != 0.0) ? a * rk[tt][c] + dt * R : dt * R;
            K1[idx] = k;
            const double u0 = PERT ? r0[tt][c] : (double)sU[(ROWC * c + ROWE * re) * RS + n];
            Uout[idx] = u0 + b * k;
          }
        }
      }
    }
  }
}

// Isoparametric elements and their face neighbours (the curved set S), in
// FP64 in every form: one element per wavefront, per-node metric terms,
// per-face-node normals and sJ, and the element's P = (M^K)^-1 M.
// With J inside the contravariant flux and sJ in the face terms, the
// strong-form residual X = -(D_r F~_r + D_s F~_s) + LIFT h + LIFT_r q_r +
// LIFT_s q_s is M times the weak form's integrals, and R = P X (on an affine
// element P = M / (J M), the stage kernel's arithmetic).  The stage kernel's
// straight tiles leave these elements unwritten, and this body reads only the
// input state and its own element's K1, so both run in the same launch: the
// stage kernel's leading workgroups take the curved set, one element per
// wave, on the SIMDs beside the straight tiles.  lds: the wave's area,
// curved_lds_doubles(N) doubles.
constexpr int curved_lds_doubles(int N) {
  return 29 * ((N + 1) * (N + 2) / 2) + 39 * (N + 1);
}
// workgroups of W waves that take the curved set, a multiple of 8 (so the
// straight tiles' workgroups keep their XCD numbering)
__host__ __device__ inline int curved_workgroups(int ncurved, int W) {
  return ncurved > 0 ? ((ncurved + W - 1) / W + 7) / 8 * 8 : 0;
}
// workgroups of W waves for the wall force in a stage launch: one wave per 64
// wall face nodes (the partials of the launch's input state), then the wave
// that sums a previous launch's partials; a multiple of 8, or none
__host__ __device__ inline int force_workgroups(const DeviceTables& t, int Nfp, int W) {
  const int nblk = (t.nwall * Nfp + kForceThreads - 1) / kForceThreads;
  if (nblk <= 0 || (!t.force_parts && t.force_fin == nullptr)) return 0;
  return ((nblk + 1 + W - 1) / W + 7) / 8 * 8;
}
template <int N>
__device__ __forceinline__ void curved_element(const DeviceTables& t, const KernelPhysics& ph,
                                               const double* __restrict__ Uin,
                                               double* __restrict__ Uout,
                                               double* __restrict__ K1, double a, double b,
                                               double dt, int rhs_only, int slot, double* lds) {
  constexpr int Np = (N + 1) * (N + 2) / 2, Nfp = N + 1, NFN = 3 * Nfp, S = 4 * Np;
  double* sU = lds;
  double* sGx = sU + S;
  double* sGy = sGx + S;
  double* sFr = sGy + S;
  double* sFs = sFr + S;
  double* sX = sFs + S;
  double* sNd = sX + S;
  double* sH = sNd + 5 * Np;
  double* sQr = sH + 4 * NFN;
  double* sQs = sQr + 4 * NFN;
  double* sNorm = sQs + 4 * NFN;
  static_assert(6 * S + 5 * Np + 13 * NFN == curved_lds_doubles(N), "curved LDS layout");
  const int lane = threadIdx.x & 63;
  const int64_t k = t.celem[slot];
  const double* Dr = t.ops;
  const double* Ds = t.ops + Np * Np;
  const double* LIFT = t.ops + 2 * Np * Np;
  const double* LIFTr = LIFT + Np * NFN;
  const double* LIFTs = LIFTr + Np * NFN;
  const double* nd = t.cnode + (int64_t)slot * 5 * Np;
  const double* fc = t.cface + (int64_t)slot * 3 * NFN;
  Gas<double> gas;
  gas.gamma = ph.gamma;
  gas.gm1 = ph.gm1;
  gas.igm1 = ph.igm1;
  gas.mu = ph.mu;
  gas.k = ph.k;
  Base<double> base;
  base.rho = ph.U_inf[0];
  base.mx = ph.U_inf[1];
  base.my = ph.U_inf[2];
  base.E = ph.U_inf[3];
  base.p = ph.p_inf;
  base.ux = ph.u_inf;
  base.uy = ph.v_inf;
  const double vwx = ph.vw[0], vwy = ph.vw[1];

  #pragma unroll 1
  for (int i = lane; i < S; i += 64) sU[i] = Uin[k * S + i];
  #pragma unroll 1
  for (int i = lane; i < 5 * Np; i += 64) sNd[i] = nd[i];
  wave_sync();
  // gradient at the nodes with each node's metric terms
  #pragma unroll 1
  for (int i = lane; i < S; i += 64) {
    const int c = i / Np, n = i - c * Np;
    double ur = 0.0, us = 0.0;
    #pragma unroll 4
    for (int m = 0; m < Np; ++m) {
      ur += Dr[n * Np + m] * sU[c * Np + m];
      us += Ds[n * Np + m] * sU[c * Np + m];
    }
    sGx[i] = sNd[n] * ur + sNd[2 * Np + n] * us;
    sGy[i] = sNd[Np + n] * ur + sNd[3 * Np + n] * us;
  }
  wave_sync();
  // total flux at the nodes, contravariant with J
  #pragma unroll 1
  for (int n = lane; n < Np; n += 64) {
    double u[4], gx[4], gy[4];
    for (int c = 0; c < 4; ++c) {
      u[c] = sU[c * Np + n];
      gx[c] = sGx[c * Np + n];
      gy[c] = sGy[c * Np + n];
    }
    double fvx[4], fvy[4], Fx[4], Fy[4];
    viscous_flux(gas, vstate(gas, u), gx, gy, fvx, fvy);
    const Prim<double> pr = prim_plain(u, gas.gm1);
    normal_flux_plain(u, pr, 1.0, 0.0, vwx, Fx);
    normal_flux_plain(u, pr, 0.0, 1.0, vwy, Fy);
    const double rx = sNd[n], ry = sNd[Np + n], sx = sNd[2 * Np + n], sy = sNd[3 * Np + n];
    const double J = sNd[4 * Np + n];
    for (int c = 0; c < 4; ++c) {
      const double fx = Fx[c] - fvx[c], fy = Fy[c] - fvy[c];
      sFr[c * Np + n] = J * (rx * fx + ry * fy);
      sFs[c * Np + n] = J * (sx * fx + sy * fy);
    }
  }
  wave_sync();
  // face nodes, one lane each: traces, ghosts, norms, the other side's
  // gradient (with that element's metric terms at its node), viscous mean
  const bool fl = lane < NFN;
  const int l = fl ? lane : 0;
  const int f = l / Nfp, j = l - f * Nfp;
  const int n = face_node<N>(f, j);
  const int conn = t.conn[k * 3 + f];
  const int tag = conn & 3, nf = (conn >> 2) & 3;
  const int64_t kn = conn >> 4;
  const double nx = fc[l], ny = fc[NFN + l], sJ = fc[2 * NFN + l];
  double up[4] = {0.0, 0.0, 0.0, 0.0}, uo[4] = {0.0, 0.0, 0.0, 0.0};
  double vn[4] = {0.0, 0.0, 0.0, 0.0};
  VState<double> sp = {}, so = {};
  if (fl) {
    double gxp[4], gyp[4], gxm[4], gym[4];
    for (int c = 0; c < 4; ++c) {
      up[c] = sU[c * Np + n];
      gxp[c] = sGx[c * Np + n];
      gyp[c] = sGy[c * Np + n];
      gxm[c] = gxp[c];
      gym[c] = gyp[c];
    }
    if (tag == 0) {
      const int n2 = face_node<N>(nf, Nfp - 1 - j);
      const double* Un = Uin + kn * S;
      double ur[4] = {0, 0, 0, 0}, us[4] = {0, 0, 0, 0};
      #pragma unroll 4
      for (int m = 0; m < Np; ++m) {
        const double dr = Dr[n2 * Np + m], ds = Ds[n2 * Np + m];
        for (int c = 0; c < 4; ++c) {
          ur[c] += dr * Un[c * Np + m];
          us[c] += ds * Un[c * Np + m];
        }
      }
      const int cs = t.cslot[kn];
      double rx, ry, sx, sy;
      if (cs >= 0) {
        const double* nd2 = t.cnode + (int64_t)cs * 5 * Np;
        rx = nd2[n2];
        ry = nd2[Np + n2];
        sx = nd2[2 * Np + n2];
        sy = nd2[3 * Np + n2];
      } else {
        const double* g2 = t.geo + kn * kGeoStride;
        rx = g2[0];
        ry = g2[1];
        sx = g2[2];
        sy = g2[3];
      }
      for (int c = 0; c < 4; ++c) {
        uo[c] = Un[c * Np + n2];
        gxm[c] = rx * ur[c] + sx * us[c];
        gym[c] = ry * ur[c] + sy * us[c];
      }
    } else {
      // wall or far field: the ghost (no neighbour value is read)
      ghost_state<double, false>(tag, up, up, sU + n, Np, vwx, vwy, gas, base, uo);
    }
    sp = vstate(gas, up);
    so = vstate(gas, uo);
    const double a1 = normal_diffusion_norm(gas, sp, nx, ny);
    const double a2 = normal_diffusion_norm(gas, so, nx, ny);
    sNorm[l] = a1 > a2 ? a1 : a2;
    if (tag == 1) {
      // wall: G(U^b) grad U+ (conduction as the wall flux mode sets it)
      viscous_normal_flux(gas_wall(gas, ph.k_wall), so, gxp, gyp, nx, ny, vn);
    } else {
      viscous_normal_flux(gas, sp, gxp, gyp, nx, ny, vn);
      if (tag == 0) {
        double vm[4];
        viscous_normal_flux(gas, so, gxm, gym, nx, ny, vm);
        for (int c = 0; c < 4; ++c) vn[c] = 0.5 * (vn[c] + vm[c]);
      }
    }
  }
  wave_sync();
  if (fl) {
    double gbar = 0.0;
    #pragma unroll 1
    for (int jj = 0; jj < Nfp; ++jj) gbar = sNorm[f * Nfp + jj] > gbar ? sNorm[f * Nfp + jj] : gbar;
    const double sigma = t.geo[k * kGeoStride + 7 + 4 * f] * gbar;
    const double vwn = vwx * nx + vwy * ny;
    const Prim<double> pp = prim_plain(up, gas.gm1);
    double Fc[4];
    if (tag == 1) {
      Fc[0] = 0.0;
      Fc[1] = pp.p * nx;
      Fc[2] = pp.p * ny;
      Fc[3] = pp.p * vwn;
    } else {
      const Prim<double> po = prim_plain(uo, gas.gm1);
      double FL[4], FR[4];
      normal_flux_plain(up, pp, nx, ny, vwn, FL);
      normal_flux_plain(uo, po, nx, ny, vwn, FR);
      roe_flux(pp, po, FL, FR, nx, ny, vwn, gas.gm1, Fc);
    }
    // sJ times the own normal flux, from the contravariant flux (J inside):
    // face 0: -Fs, face 1: Fr + Fs, face 2: -Fr
    const double cfr = f == 0 ? 0.0 : (f == 1 ? 1.0 : -1.0);
    const double cfs = f == 2 ? 0.0 : (f == 1 ? 1.0 : -1.0);
    double w[4];
    for (int c = 0; c < 4; ++c) {
      w[c] = up[c] - uo[c];
      const double own = cfr * sFr[c * Np + n] + cfs * sFs[c * Np + n];
      sH[c * NFN + l] = own - sJ * (Fc[c] - vn[c] + sigma * w[c]);
    }
    double qx[4], qy[4];
    viscous_transpose(tag == 1 ? gas_wall(gas, ph.k_wall) : gas, tag == 1 ? so : sp, nx, ny, w, qx, qy);
    const double ce = ph.theta * (tag == 0 ? 0.5 : 1.0) * sJ;
    const double rx = sNd[n], ry = sNd[Np + n], sx = sNd[2 * Np + n], sy = sNd[3 * Np + n];
    for (int c = 0; c < 4; ++c) {
      sQr[c * NFN + l] = ce * (rx * qx[c] + ry * qy[c]);
      sQs[c * NFN + l] = ce * (sx * qx[c] + sy * qy[c]);
    }
  }
  wave_sync();
  // strong-form residual, then R = P X and the stage
  #pragma unroll 1
  for (int i = lane; i < S; i += 64) {
    const int c = i / Np, m0 = i - c * Np;
    double x = 0.0;
    #pragma unroll 4
    for (int m = 0; m < Np; ++m) x -= Dr[m0 * Np + m] * sFr[c * Np + m] + Ds[m0 * Np + m] * sFs[c * Np + m];
    #pragma unroll 4
    for (int q = 0; q < NFN; ++q)
      x += LIFT[m0 * NFN + q] * sH[c * NFN + q] + LIFTr[m0 * NFN + q] * sQr[c * NFN + q] +
           LIFTs[m0 * NFN + q] * sQs[c * NFN + q];
    sX[i] = x;
  }
  wave_sync();
  const double* P = t.cP + (int64_t)slot * Np * Np;
  #pragma unroll 1
  for (int i = lane; i < S; i += 64) {
    const int c = i / Np, m0 = i - c * Np;
    double R = 0.0;
    #pragma unroll 4
    for (int m = 0; m < Np; ++m) R += P[m0 * Np + m] * sX[c * Np + m];
    const int64_t idx = k * S + i;
    if (rhs_only) {
      K1[idx] = R;
    } else {
      const double kk = (a != 0.0) ? a * K1[idx] + dt * R : dt * R;
      K1[idx] = kk;
      Uout[idx] = sU[i] + b * kk;
    }
  }
}

// Copy the operator fragments of order N into LDS and zero the pad columns
// (nodes Np .. RS - 1) of the state and flux rows of this workgroup's wave
// areas: the matrix-core products read them against zero operator entries,
// so they must hold finite values, and no tile writes them.  (Rows of absent
// elements only feed outputs that are never stored; the face-term pads are
// zeroed per tile, since the neighbour states overwrite them.)
template <int N, typename X, int W>
__device__ __forceinline__ void stage_lds_init(const typename Real<X>::type* __restrict__ frag,
                                               typename Real<X>::type* sFrag,
                                               typename Real<X>::type* sWave) {
  typedef typename Real<X>::type T;
  using O = Order<N, X>;
  constexpr int PAD = O::RS - O::Np;    // pad columns per row
  constexpr int ROWS = 48;              // 16 state rows, then 32 flux rows
  for (int i = threadIdx.x; i < O::FRAG_SZ; i += 64 * W) sFrag[i] = frag[i];
  for (int i = threadIdx.x; i < W * ROWS * PAD; i += 64 * W) {
    const int w = i / (ROWS * PAD), r = (i / PAD) % ROWS, c = i % PAD;
    sWave[w * O::WAVE_SZ + r * O::RS + O::Np + c] = T(0);
  }
  __syncthreads();
}

// Single mesh.  Tiles are handed out in contiguous ranges per XCD (workgroup b
// runs on XCD b % 8, the grid is a multiple of 8) so that neighbour reads stay
// in that XCD's L2; within a range the waves stride over the tiles (a
// persistent grid) or take one tile each (a grid of one tile per wave).
template <int N, typename X, bool PERT, int W>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(Order<N, X>::MIN_WAVES_EU))) void
stage_kernel(DeviceTables t, KernelPhysics ph, const double* __restrict__ Uin,
             double* __restrict__ Uout, double* __restrict__ K1, double a, double b, double dt,
             int rhs_only) {
  typedef typename Real<X>::type T;
  using O = Order<N, X>;
  __shared__ __attribute__((aligned(16))) T sFrag[O::FRAG_SZ];
  __shared__ __attribute__((aligned(16))) T sWave[W * O::WAVE_SZ];
  __shared__ int sConnW[W * 12];
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: tile indices stay scalar
  // the leading workgroups evaluate the curved set (one element per wave, in
  // the wave's LDS area), the rest the straight tiles
  const int ncw = curved_workgroups(t.ncurved, W);
  static_assert((O::WAVE_SZ * sizeof(T)) / 8 >= curved_lds_doubles(N) + 1,
                "the curved element's arrays must fit a wave's LDS area");
  if ((int)blockIdx.x < ncw) {
    const int slot = (int)blockIdx.x * W + wid;
    if (slot < t.ncurved) {
      const uintptr_t at = ((uintptr_t)(sWave + wid * O::WAVE_SZ) + 7) & ~(uintptr_t)7;
      curved_element<N>(t, ph, Uin, Uout, K1, a, b, dt, rhs_only, slot, (double*)at);
    }
    return;
  }
  // then, where the caller asks for them, the wall force partials of the
  // input state (the previous step's output, which this launch only reads):
  // one wave per 64 wall face nodes; and the sum of the partials a previous
  // launch left, by the wave after them
  const int nfw = force_workgroups(t, O::Nfp, W);
  if ((int)blockIdx.x < ncw + nfw) {
    const unsigned nblk = (unsigned)((t.nwall * O::Nfp + kForceThreads - 1) / kForceThreads);
    const unsigned wv = (blockIdx.x - ncw) * W + wid;
    // the node's derivative loop unrolled by eight: two rounds of loads at
    // p = 4, and no more registers than the stage kernel holds
    if (t.force_parts && wv < nblk) force_wave<N, 8, false>(t, ph, Uin, nullptr, wv, nblk);
    if (t.force_fin != nullptr && wv == nblk) force_sum(t.force_part, t.force_fin, nblk);
    return;
  }
  stage_lds_init<N, X, W>(frag_of<X>(t), sFrag, sWave);
  const unsigned bx = blockIdx.x - ncw - nfw, gx = gridDim.x - ncw - nfw;
  const int64_t ntiles = (t.K + O::EPT - 1) / O::EPT;
  const int xcd = bx & 7;
  const int64_t tb = ntiles * xcd / 8, te = ntiles * (xcd + 1) / 8;
  const int64_t w0 = (int64_t)(bx >> 3) * W + wid;
  const int64_t wstride = (int64_t)(gx >> 3) * W;
  stage_tiles<N, X, PERT>(t, ph, Uin, Uout, K1, a, b, dt, rhs_only, sFrag, sWave + wid * O::WAVE_SZ,
                          sConnW + 12 * wid, tb + w0, te, wstride);
}

// ---------------------------------------------------------------------------
// Over-integrated stage (FP64, plain form): the weak form with every integral
// taken by rules exact for degree 3p -- a collapsed Gauss rule of q^2 points on
// the element and Gauss-Legendre with q points on each face -- instead of the
// nodal interpolants of the fluxes (the anti-aliasing remedy of Sec. 2.2):
//   R = M^-1 [ sum_q w_q (F_r d_r l_i + F_s d_s l_i)(x_q)
//              - sum_faces sum_g w_g Fscale H_m l_i (x_g)
//              + sum_faces sum_g w_g Fscale (q_r d_r l_i + q_s d_s l_i)(x_g) ]
// with M^-1 and the weights folded into the operators.  Per tile:
//   1  own and neighbour states, geometry (as the nodal kernel, no pipelining)
//   2  element points in chunks of 16: U, d_r U, d_s U there on the matrix
//      cores, the total flux pointwise, and the chunk's part of the weighted
//      divergence accumulated at once (only one chunk of flux lives in LDS)
//   3  face points, one lane each: both sides' values (face-node
//      interpolation) and gradients (rows of the point derivative matrices),
//      ghosts, ||n^T G n||_2, viscous average; then G-bar_e over the face's
//      points, sigma_e, Roe, penalty and theta terms
//   4  the three weighted lifts on the matrix cores into the same
//      accumulator, then the RK stage in FP64.
// The operator fragments are read from global memory (L2-resident); only the
// face-point derivative rows sit in LDS.
template <int N>
struct OIOrder {
  using O = Order<N, double>;
  static constexpr int Np = O::Np, Nfp = O::Nfp, S = O::S, NT = O::NT, KS = O::KS, RS = O::RS;
  static constexpr int q = oi_points(N), Nq = q * q, NG = 3 * q;
  static constexpr int NQT = (Nq + 15) / 16;   // 16-point chunks of the element rule
  static constexpr int KQ = (Nq + 3) / 4;      // k-steps over the element points
  static constexpr int KG = (NG + 3) / 4;      // k-steps over the face points
  static constexpr int EPT = (64 / NG) < 4 ? ((64 / NG) > 0 ? 64 / NG : 1) : 4;
  static constexpr int FRS = 17;               // padded LDS row of one flux chunk
  static constexpr int GRS = 4 * KG + 1;       // padded LDS row of the face terms
  static constexpr int U_SZ = 16 * RS, F_SZ = 32 * FRS;
  static constexpr int N_SZ = 12 * S, H_SZ = 48 * GRS;
  static constexpr int X_SZ = N_SZ > H_SZ ? N_SZ : H_SZ;
  static constexpr int NORM_SZ = 4 * NG, VN_SZ = 16 * NG;
  static constexpr int WAVE_SZ = (U_SZ + F_SZ + X_SZ + NORM_SZ + VN_SZ + 64 + 48 + 3) / 4 * 4;
  // global fragment offsets (doubles), in the order the host packs them
  static constexpr int FI = NQT * KS * 64, FW = NT * KQ * 64, FL = NT * KG * 64;
  static constexpr int OFF_IQ = 0, OFF_DRQ = FI, OFF_DSQ = 2 * FI, OFF_WR = 3 * FI,
                       OFF_WS = 3 * FI + FW, OFF_LQ = 3 * FI + 2 * FW, OFF_LRQ = OFF_LQ + FL,
                       OFF_LSQ = OFF_LQ + 2 * FL, OFF_DRSF = OFF_LQ + 3 * FL,
                       OFF_IF1 = OFF_DRSF + 2 * NG * Np, TOTAL = OFF_IF1 + q * Nfp;
  static constexpr int LDS_TAB = 2 * NG * Np + q * Nfp;  // face-point tables in LDS
};

template <int N>
__device__ __forceinline__ void oi_tiles(const DeviceTables& t, const KernelPhysics& ph,
                                         const double* __restrict__ Uin, double* __restrict__ Uout,
                                         double* __restrict__ K1, double a, double b, double dt,
                                         int rhs_only, const double* sTab, double* sU, int* sConn,
                                         int64_t tile0, int64_t tile_end, int64_t stride) {
  typedef double T;
  using P = OIOrder<N>;
  using O = Order<N, double>;
  typedef Vec4<double>::type V4;
  constexpr int Np = P::Np, Nfp = P::Nfp, S = P::S, NT = P::NT, KS = P::KS, RS = P::RS, q = P::q,
                Nq = P::Nq, NG = P::NG, NQT = P::NQT, KQ = P::KQ, KG = P::KG, EPT = P::EPT,
                FRS = P::FRS, GRS = P::GRS, ROWC = O::ROWC, ROWE = O::ROWE;
  const int lane = threadIdx.x & 63;
  const double* G = t.oi;
  const double* sDRS = sTab;               // [NG][Np] (d_r, d_s) pairs
  const double* sIf1 = sTab + 2 * NG * Np; // [q][Nfp]
  T* sF = sU + P::U_SZ;                    // flux chunk: F_r rows | F_s rows
  T* sX = sF + P::F_SZ;                    // neighbour states, later face terms
  T* sH = sX;
  T* sQr = sX + 16 * GRS;
  T* sQs = sX + 32 * GRS;
  T* sNorm = sX + P::X_SZ;
  T* sVn = sNorm + P::NORM_SZ;             // [4 fields][4 NG]
  T* sGeo = sVn + P::VN_SZ;
  T* sNGeo = sGeo + 64;

  Gas<T> gas;
  gas.gamma = ph.gamma;
  gas.gm1 = ph.gamma - 1.0;
  gas.igm1 = 1.0 / (ph.gamma - 1.0);
  gas.mu = ph.mu;
  gas.k = ph.gamma / ph.Pr;
  const T theta = ph.theta, vwx = ph.vw[0], vwy = ph.vw[1];
  const T k_wall = ph.k_wall;
  Base<T> base;
  {
    const double r0 = ph.U_inf[0], ux0 = ph.U_inf[1] / r0, uy0 = ph.U_inf[2] / r0;
    base.rho = r0;
    base.mx = ph.U_inf[1];
    base.my = ph.U_inf[2];
    base.E = ph.U_inf[3];
    base.p = (ph.gamma - 1.0) * (ph.U_inf[3] - 0.5 * (ph.U_inf[1] * ux0 + ph.U_inf[2] * uy0));
    base.ux = ux0;
    base.uy = uy0;
  }
  const int64_t K = t.K;
  const int arow = lane & 15, acol = lane >> 4;
  const int re = lane >> 4, rn = lane & 15;
  constexpr int NQL = (S + 63) / 64;
  int lds_u[NQL];
  bool lr_ok[NQL];
#pragma unroll
  for (int qq = 0; qq < NQL; ++qq) {
    const int r = lane + 64 * qq;
    lr_ok[qq] = r < S;
    lds_u[qq] = lr_ok[qq] ? ROWC * (r / Np) * RS + (r - (r / Np) * Np) : 0;
  }

  for (int64_t tile = tile0; tile < tile_end; tile += stride) {
    const int64_t e0 = tile * EPT;
    const int nel = (int)((K - e0) < EPT ? (K - e0) : EPT);
    wave_sync();
    // ---- 1: own states, geometry, connectivity; neighbour states and metrics
    if (lane < nel * 3) sConn[lane] = t.conn[e0 * 3 + lane];
    if (lane < nel * kGeoStride) sGeo[lane] = t.geo[e0 * kGeoStride + lane];
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int qq = 0; qq < NQL; ++qq)
        if (lr_ok[qq] && e < nel) sU[lds_u[qq] + ROWE * e * RS] = Uin[(e0 + e) * S + lane + 64 * qq];
    wave_sync();
    if (lane < nel * 12) sNGeo[lane] = t.geo[(int64_t)(sConn[lane >> 2] >> 4) * kGeoStride + (lane & 3)];
    for (int bb = 0; bb < 3 * nel; ++bb) {
      const int64_t nb = (int64_t)(sConn[bb] >> 4) * S;
#pragma unroll
      for (int qq = 0; qq < NQL; ++qq)
        if (lr_ok[qq]) sX[bb * S + lane + 64 * qq] = Uin[nb + lane + 64 * qq];
    }
    wave_sync();

    // ---- 2: element points, chunk by chunk; the divergence accumulates in acc
    V4 acc[NT];
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) acc[tt] = V4{0.0, 0.0, 0.0, 0.0};
    for (int tq = 0; tq < NQT; ++tq) {
      V4 aU = {0.0, 0.0, 0.0, 0.0}, aR = aU, aS = aU;
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const T av = sU[arow * RS + 4 * s + acol];
        const int fo = (tq * KS + s) * 64 + lane;
        aU = mfma(av, G[P::OFF_IQ + fo], aU);
        aR = mfma(av, G[P::OFF_DRQ + fo], aR);
        aS = mfma(av, G[P::OFF_DSQ + fo], aS);
      }
      const int k = 16 * tq + rn;
      T Fr[4] = {0.0, 0.0, 0.0, 0.0}, Fs[4] = {0.0, 0.0, 0.0, 0.0};
      if (re < nel && k < Nq) {
        const T* g = sGeo + re * kGeoStride;
        const T rx = g[0], ry = g[1], sx = g[2], sy = g[3];
        T u[4], gx[4], gy[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          u[c] = aU[c];
          gx[c] = rx * aR[c] + sx * aS[c];
          gy[c] = ry * aR[c] + sy * aS[c];
        }
        T fvx[4], fvy[4], Fx[4], Fy[4];
        viscous_flux(gas, vstate(gas, u), gx, gy, fvx, fvy);
        const Prim<T> pr = prim_plain(u, gas.gm1);
        normal_flux<T, false>(u, u, pr, base, 1.0, 0.0, vwx, Fx);
        normal_flux<T, false>(u, u, pr, base, 0.0, 1.0, vwy, Fy);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const T fx = Fx[c] - fvx[c], fy = Fy[c] - fvy[c];
          Fr[c] = rx * fx + ry * fy;
          Fs[c] = sx * fx + sy * fy;
        }
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        sF[(ROWC * c + ROWE * re) * FRS + rn] = Fr[c];
        sF[(16 + ROWC * c + ROWE * re) * FRS + rn] = Fs[c];
      }
      wave_sync();
#pragma unroll
      for (int tt = 0; tt < NT; ++tt)
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const int s = 4 * tq + s4;
          if (s < KQ) {
            const int fo = (tt * KQ + s) * 64 + lane;
            acc[tt] = mfma(sF[arow * FRS + 4 * s4 + acol], G[P::OFF_WR + fo], acc[tt]);
            acc[tt] = mfma(sF[(16 + arow) * FRS + 4 * s4 + acol], G[P::OFF_WS + fo], acc[tt]);
          }
        }
      wave_sync();
    }

    // ---- 3: face points, one lane each
    const int e = lane / NG < 3 ? lane / NG : 3;
    const int fg = lane - (lane / NG) * NG;
    const bool ok = lane < EPT * NG && (lane / NG) < nel;
    const int f = fg / q, gp = fg - f * q;
    T up[4] = {0.0, 0.0, 0.0, 0.0}, uo[4] = {0.0, 0.0, 0.0, 0.0};
    int tag = 0;
    if (ok) {
      const int conn = sConn[e * 3 + f];
      tag = conn & 3;
      const int nf = (conn >> 2) & 3;
      const T* g = sGeo + e * kGeoStride;
      const T nx = g[4 + 4 * f], ny = g[5 + 4 * f];
      // own value and gradient at the point
      T ur[4] = {0.0, 0.0, 0.0, 0.0}, us[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
      for (int j = 0; j < Np; ++j) {
        const T dr = sDRS[2 * (fg * Np + j)], ds = sDRS[2 * (fg * Np + j) + 1];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const T v = sU[(ROWC * c + ROWE * e) * RS + j];
          ur[c] += dr * v;
          us[c] += ds * v;
        }
      }
#pragma unroll
      for (int i = 0; i < Nfp; ++i) {
        const T w = sIf1[gp * Nfp + i];
        const int n = face_node<N>(f, i);
#pragma unroll
        for (int c = 0; c < 4; ++c) up[c] += w * sU[(ROWC * c + ROWE * e) * RS + n];
      }
      T gxp[4], gyp[4], gxm[4], gym[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        gxp[c] = g[0] * ur[c] + g[2] * us[c];
        gyp[c] = g[1] * ur[c] + g[3] * us[c];
        gxm[c] = gxp[c];
        gym[c] = gyp[c];
      }
      if (tag == 0) {
        // the neighbour's value and gradient at its mirrored point
        const T* nbU = sX + (e * 3 + f) * S;
        const int gm = q - 1 - gp, row = nf * q + gm;
        T vr[4] = {0.0, 0.0, 0.0, 0.0}, vs[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
        for (int j = 0; j < Np; ++j) {
          const T dr = sDRS[2 * (row * Np + j)], ds = sDRS[2 * (row * Np + j) + 1];
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const T v = nbU[c * Np + j];
            vr[c] += dr * v;
            vs[c] += ds * v;
          }
        }
#pragma unroll
        for (int i = 0; i < Nfp; ++i) {
          const T w = sIf1[gm * Nfp + i];
          const int n = face_node<N>(nf, i);
#pragma unroll
          for (int c = 0; c < 4; ++c) uo[c] += w * nbU[c * Np + n];
        }
        const T* ng = sNGeo + (e * 3 + f) * 4;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          gxm[c] = ng[0] * vr[c] + ng[2] * vs[c];
          gym[c] = ng[1] * vr[c] + ng[3] * vs[c];
        }
      } else {
        ghost_state<T, false>(tag, up, up, nullptr, 1, vwx, vwy, gas, base, uo);
      }
      const VState<T> sp = vstate(gas, up), so = vstate(gas, uo);
      const T n1 = normal_diffusion_norm(gas, sp, nx, ny), n2 = normal_diffusion_norm(gas, so, nx, ny);
      sNorm[e * NG + fg] = n1 > n2 ? n1 : n2;
      T vn[4];
      if (tag == 1) {
        // adiabatic wall: stress and its work, no heat conduction
        viscous_normal_flux(gas_wall(gas, k_wall), so, gxp, gyp, nx, ny, vn);
      } else {
        viscous_normal_flux(gas, sp, gxp, gyp, nx, ny, vn);
        if (tag == 0) {
          T vm[4];
          viscous_normal_flux(gas, so, gxm, gym, nx, ny, vm);
#pragma unroll
          for (int c = 0; c < 4; ++c) vn[c] = 0.5 * (vn[c] + vm[c]);
        }
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) sVn[c * 4 * NG + e * NG + fg] = vn[c];
    }
    wave_sync();
    if (ok) {
      const T* g = sGeo + e * kGeoStride;
      const T nx = g[4 + 4 * f], ny = g[5 + 4 * f], fsc = g[6 + 4 * f];
      T gbar = 0.0;
#pragma unroll
      for (int jj = 0; jj < q; ++jj) {
        const T v = sNorm[e * NG + f * q + jj];
        gbar = v > gbar ? v : gbar;
      }
      const T sigma = g[7 + 4 * f] * gbar;
      const T vwn = vwx * nx + vwy * ny;
      const Prim<T> pp = prim_plain(up, gas.gm1);
      T Fc[4];
      if (tag == 1) {
        Fc[0] = 0.0;
        Fc[1] = pp.p * nx;
        Fc[2] = pp.p * ny;
        Fc[3] = pp.p * vwn;
      } else {
        const Prim<T> po = prim_plain(uo, gas.gm1);
        T FL[4], FR[4];
        normal_flux<T, false>(up, up, pp, base, nx, ny, vwn, FL);
        normal_flux<T, false>(uo, uo, po, base, nx, ny, vwn, FR);
        roe_flux(pp, po, FL, FR, nx, ny, vwn, gas.gm1, Fc);
      }
      T w[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        w[c] = up[c] - uo[c];
        sH[(ROWC * c + ROWE * e) * GRS + fg] = -fsc * (Fc[c] - sVn[c * 4 * NG + e * NG + fg] + sigma * w[c]);
      }
      T qx[4], qy[4];
      viscous_transpose(tag == 1 ? gas_wall(gas, k_wall) : gas, vstate(gas, tag == 1 ? uo : up), nx, ny, w, qx, qy);
      const T ce = theta * (tag == 0 ? 0.5 : 1.0) * fsc;
      const T rx = g[0], ry = g[1], sx = g[2], sy = g[3];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        sQr[(ROWC * c + ROWE * e) * GRS + fg] = ce * (rx * qx[c] + ry * qy[c]);
        sQs[(ROWC * c + ROWE * e) * GRS + fg] = ce * (sx * qx[c] + sy * qy[c]);
      }
    }
    for (int i = lane; i < 48 * (GRS - NG); i += 64) {
      const int row = i / (GRS - NG);
      sX[row * GRS + NG + (i - row * (GRS - NG))] = 0.0;
    }
    wave_sync();

    // ---- 4: lifts into the accumulator, then the RK stage
#pragma unroll
    for (int tt = 0; tt < NT; ++tt)
#pragma unroll
      for (int s = 0; s < KG; ++s) {
        const int fo = (tt * KG + s) * 64 + lane;
        const int ao = arow * GRS + 4 * s + acol;
        acc[tt] = mfma(sH[ao], G[P::OFF_LQ + fo], acc[tt]);
        acc[tt] = mfma(sQr[ao], G[P::OFF_LRQ + fo], acc[tt]);
        acc[tt] = mfma(sQs[ao], G[P::OFF_LSQ + fo], acc[tt]);
      }
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) {
      const int n = 16 * tt + rn;
      if (re < nel && n < Np) {
        const int64_t base_i = (e0 + re) * S + n;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double R = acc[tt][c];
          const int64_t idx = base_i + c * Np;
          if (rhs_only) {
            K1[idx] = R;
          } else {
            const double kk = (a == 0.0) ? dt * R : a * K1[idx] + dt * R;
            K1[idx] = kk;
            Uout[idx] = sU[(ROWC * c + ROWE * re) * RS + n] + b * kk;
          }
        }
      }
    }
  }
}

template <int N, int W>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(1))) void
oi_stage_kernel(DeviceTables t, KernelPhysics ph, const double* __restrict__ Uin,
                double* __restrict__ Uout, double* __restrict__ K1, double a, double b, double dt,
                int rhs_only) {
  using P = OIOrder<N>;
  __shared__ __attribute__((aligned(16))) double sTab[P::LDS_TAB];
  __shared__ __attribute__((aligned(16))) double sWave[W * P::WAVE_SZ];
  __shared__ int sConnW[W * 12];
  for (int i = threadIdx.x; i < P::LDS_TAB; i += 64 * W) sTab[i] = t.oi[P::OFF_DRSF + i];
  for (int i = threadIdx.x; i < W * P::WAVE_SZ; i += 64 * W) sWave[i] = 0.0;
  __syncthreads();
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: tile indices stay scalar
  const int64_t ntiles = (t.K + P::EPT - 1) / P::EPT;
  const int xcd = blockIdx.x & 7;
  const int64_t tb = ntiles * xcd / 8, te = ntiles * (xcd + 1) / 8;
  const int64_t w0 = (int64_t)(blockIdx.x >> 3) * W + wid;
  const int64_t wstride = (int64_t)(gridDim.x >> 3) * W;
  oi_tiles<N>(t, ph, Uin, Uout, K1, a, b, dt, rhs_only, sTab, sWave + wid * P::WAVE_SZ,
              sConnW + 12 * wid, tb + w0, te, wstride);
}

// Many meshes in one launch.  The instances are grouped by order; group g
// owns the workgroups [block_begin, block_begin + nblocks) (multiples of 8)
// and numbers the tiles of its instances consecutively.  Per-instance dt and
// v_w, and the parity of the state buffers, come from device memory, so a
// captured graph of the five stages stays valid from step to step.
template <int N, typename X, bool PERT, int W>
__device__ __forceinline__ void batch_group(const BatchItem* __restrict__ items,
                                            const BatchStep* __restrict__ steps, int par,
                                            const BatchGroup& g, int stage, double a, double b,
                                            unsigned char* smem) {
  typedef typename Real<X>::type T;
  using O = Order<N, X>;
  T* sFrag = (T*)smem;
  T* sWave = sFrag + O::FRAG_SZ;
  int* sConnW = (int*)(sWave + W * O::WAVE_SZ);
  stage_lds_init<N, X, W>(frag_of<X>(items[g.first_item].t), sFrag, sWave);
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: tile indices stay scalar
  const int local = blockIdx.x - g.block_begin;
  const int xcd = local & 7;
  const int64_t tb = g.ntiles * xcd / 8, te = g.ntiles * (xcd + 1) / 8;
  const int64_t wstride = (int64_t)(g.nblocks >> 3) * W;
  int i = g.first_item;
  for (int64_t tile = tb + (int64_t)(local >> 3) * W + wid; tile < te; tile += wstride) {
    while (tile >= items[i].tile_end) ++i;  // tiles only increase
    const BatchItem& it = items[i];
    KernelPhysics ph = it.ph;
    ph.vw[0] = steps[i].vw[0];
    ph.vw[1] = steps[i].vw[1];
    const int src = (par + stage) & 1;
    stage_tiles<N, X, PERT>(it.t, ph, it.buf[src], it.buf[src ^ 1], it.K1, a, b, steps[i].dt, 0,
                            sFrag, sWave + wid * O::WAVE_SZ, sConnW + 12 * wid,
                            tile - it.tile_begin, tile - it.tile_begin + 1, 1);
  }
}

template <typename X, int W>
struct BatchLds {
  template <int N>
  static constexpr size_t of() {
    return (Order<N, X>::FRAG_SZ + W * Order<N, X>::WAVE_SZ) * sizeof(typename Real<X>::type) +
           W * 12 * sizeof(int);
  }
  static constexpr size_t mx(size_t x, size_t y) { return x > y ? x : y; }
  static constexpr size_t bytes =
      mx(mx(mx(of<1>(), of<2>()), mx(of<3>(), of<4>())), mx(of<5>(), of<6>()));
};

template <typename T, bool PERT, int W>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(2))) void
batch_stage_kernel(const BatchItem* __restrict__ items, const BatchStep* __restrict__ steps,
                   const int* __restrict__ parity, BatchGroups G, int stage, double a, double b) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[BatchLds<T, W>::bytes];
  // the group of this workgroup, selected without dynamic indexing of the
  // by-value argument (which would place a copy of it in scratch memory)
  BatchGroup g = G.g[0];
#pragma unroll
  for (int k = 1; k < kMaxOrder; ++k)
    if (k < G.ng && (int)blockIdx.x >= G.g[k].block_begin) g = G.g[k];
  const int par = parity[0];
  switch (g.p) {
    case 1: batch_group<1, T, PERT, W>(items, steps, par, g, stage, a, b, smem); break;
    case 2: batch_group<2, T, PERT, W>(items, steps, par, g, stage, a, b, smem); break;
    case 3: batch_group<3, T, PERT, W>(items, steps, par, g, stage, a, b, smem); break;
    case 4: batch_group<4, T, PERT, W>(items, steps, par, g, stage, a, b, smem); break;
    case 5: batch_group<5, T, PERT, W>(items, steps, par, g, stage, a, b, smem); break;
    case 6: batch_group<6, T, PERT, W>(items, steps, par, g, stage, a, b, smem); break;
    default: break;
  }
}

// One order group per launch, sized for its own order: LDS and registers of
// order N only (the kernel above is sized for the largest order it may meet),
// so low orders keep the occupancy of the single-mesh kernel.
template <int N, typename X, bool PERT, int W>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(Order<N, X>::MIN_WAVES_EU))) void
batch_order_kernel(const BatchItem* __restrict__ items, const BatchStep* __restrict__ steps,
                   const int* __restrict__ parity, BatchGroup g, int stage, double a, double b) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[BatchLds<X, W>::template of<N>()];
  batch_group<N, X, PERT, W>(items, steps, parity[0], g, stage, a, b, smem);
}

// Wall force: one thread per wall face node (in the fixed order of the wall
// face list), a fixed-shape wave reduction per workgroup, per-workgroup
// partials, and the last workgroup to finish (an atomic ticket) sums the
// partials in workgroup order and resets the ticket: deterministic, one
// launch, no host synchronisation and no wait inside the kernel.
// Workgroup blk of the nblk that cover one mesh's wall face nodes.
template <int N>
__device__ __forceinline__ void force_block(const DeviceTables& t, const KernelPhysics& ph,
                                            const double* __restrict__ U, double* __restrict__ out,
                                            unsigned blk, unsigned nblk) {
  force_wave<N>(t, ph, U, out, blk, nblk);
}

template <int N>
__global__ __launch_bounds__(kForceThreads) void force_kernel(DeviceTables t, KernelPhysics ph,
                                                              const double* __restrict__ U,
                                                              double* __restrict__ out) {
  force_block<N>(t, ph, U, out, blockIdx.x, gridDim.x);
}

// Many meshes of one order: instance i owns the workgroups
// [block_begin_i, block_begin_i + nblocks_i), each instance reduced through
// its own partials and ticket.
template <int N>
__global__ __launch_bounds__(kForceThreads) void batch_force_kernel(const ForceItem* __restrict__ items,
                                                                    int count) {
  int i = 0;
  while (i + 1 < count && (int)blockIdx.x >= items[i + 1].block_begin) ++i;
  const ForceItem& it = items[i];
  force_block<N>(it.t, it.ph, it.U, it.out, blockIdx.x - it.block_begin, it.nblocks);
}

namespace {
constexpr int kMaxDev = 64;

int device_cus(int dev) {
  static int cache[kMaxDev] = {0};
  if (dev < 0 || dev >= kMaxDev) dev = 0;
  if (cache[dev] == 0) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
      cus = 256;
    cache[dev] = cus;
  }
  return cache[dev];
}

int current_device() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) dev = 0;
  return dev;
}

// Workgroups of a kernel that are resident on the whole device at once
// (occupancy query, cached per device and kernel).
template <typename F>
int resident_blocks(F kernel, int threads, int* cache) {
  const int dev = current_device();
  if (cache[dev] == 0) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess ||
        per_cu <= 0)
      per_cu = 1;
    cache[dev] = per_cu * device_cus(dev);
  }
  return cache[dev];
}

int launch_error(std::string& err, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    err = std::string(what) + ": " + hipGetErrorString(e);
    return -3;
  }
  return 0;
}

// Grid of the single-mesh stage kernel: persistent (at most the resident
// workgroups) or one tile per wave; a multiple of 8 either way.
int64_t stage_grid(int64_t ntiles, int waves, int resident, int mode) {
  const int64_t want = (ntiles + waves - 1) / waves;
  int64_t grid;
  if (mode == 1) {
    grid = (want + 7) / 8 * 8;
  } else if (mode >= 2) {
    // `mode` tiles per wave (at most the resident workgroups): every wave
    // does the same number of tiles, none waits on a partly filled last round
    const int64_t g = (ntiles + (int64_t)waves * mode - 1) / ((int64_t)waves * mode);
    grid = g < resident ? g : resident;
    grid = grid >= 8 ? (grid + 7) / 8 * 8 : 8;
    if (grid > resident) grid = resident / 8 * 8;
  } else {
    grid = want < resident ? want : resident;
    grid = grid >= 8 ? grid / 8 * 8 : 8;
  }
  return grid < 8 ? 8 : grid;
}

template <int N, typename T, bool PERT, int W>
int launch_stage_t(const StageTuning& tune, const DeviceTables& t, const KernelPhysics& ph,
                   const double* Uin, double* Uout, double* K1, double a, double b, double dt,
                   int rhs_only, hipStream_t s, std::string& err) {
  static int cache[kMaxDev] = {0};
  const int resident = resident_blocks(stage_kernel<N, T, PERT, W>, 64 * W, cache);
  constexpr int EPT = elements_per_tile(N);
  // the curved set's workgroups lead the grid, then the force's; a
  // persistent grid leaves the curved set its resident slots, but not the
  // force, which is done within a few microseconds: the tiles keep every
  // slot, and the last tile workgroup of each XCD (the fewest tiles per wave)
  // starts in the force workgroup's slot when that leaves, instead of one
  // CU per XCD holding a workgroup fewer and its SIMDs a tile more each
  const int ncw = curved_workgroups(t.ncurved, W);
  const int nfw = force_workgroups(t, N + 1, W);
  const int straight_resident = resident - ncw >= 8 ? resident - ncw : 8;
  const int64_t grid =
      stage_grid((t.K + EPT - 1) / EPT, W, straight_resident, tune.grid) + ncw + nfw;
  hipLaunchKernelGGL((stage_kernel<N, T, PERT, W>), dim3((unsigned)grid), dim3(64 * W), 0, s, t,
                     ph, Uin, Uout, K1, a, b, dt, rhs_only);
  return launch_error(err, "stage kernel launch");
}

template <int N, typename T, bool PERT>
int launch_stage_w(const StageTuning& tune, const DeviceTables& t, const KernelPhysics& ph,
                   const double* Uin, double* Uout, double* K1, double a, double b, double dt,
                   int rhs_only, hipStream_t s, std::string& err) {
  const int w = tune.waves ? tune.waves : Order<N, T>::WAVES;
  if (w == 2)
    return launch_stage_t<N, T, PERT, 2>(tune, t, ph, Uin, Uout, K1, a, b, dt, rhs_only, s, err);
  if (w == 4)
    return launch_stage_t<N, T, PERT, 4>(tune, t, ph, Uin, Uout, K1, a, b, dt, rhs_only, s, err);
  err = "waves per workgroup must be 2 or 4";
  return -1;
}

template <int N, int W>
int launch_oi_t(const StageTuning& tune, const DeviceTables& t, const KernelPhysics& ph,
                const double* Uin, double* Uout, double* K1, double a, double b, double dt,
                int rhs_only, hipStream_t s, std::string& err) {
  static int cache[kMaxDev] = {0};
  const int resident = resident_blocks(oi_stage_kernel<N, W>, 64 * W, cache);
  constexpr int EPT = OIOrder<N>::EPT;
  const int64_t grid = stage_grid((t.K + EPT - 1) / EPT, W, resident, tune.grid);
  hipLaunchKernelGGL((oi_stage_kernel<N, W>), dim3((unsigned)grid), dim3(64 * W), 0, s, t, ph, Uin,
                     Uout, K1, a, b, dt, rhs_only);
  return launch_error(err, "over-integrated stage kernel launch");
}

template <int N>
int launch_oi_w(const StageTuning& tune, const DeviceTables& t, const KernelPhysics& ph,
                const double* Uin, double* Uout, double* K1, double a, double b, double dt,
                int rhs_only, hipStream_t s, std::string& err) {
  if (!t.oi || t.oi_len != OIOrder<N>::TOTAL) {
    err = "over-integration tables not set up for this order";
    return -7;
  }
  const int w = tune.waves ? tune.waves : 2;
  if (w == 2) return launch_oi_t<N, 2>(tune, t, ph, Uin, Uout, K1, a, b, dt, rhs_only, s, err);
  if (w == 4) return launch_oi_t<N, 4>(tune, t, ph, Uin, Uout, K1, a, b, dt, rhs_only, s, err);
  err = "waves per workgroup must be 2 or 4";
  return -1;
}

template <int N>
int launch_stage_n(int form, const StageTuning& tune, const DeviceTables& t,
                   const KernelPhysics& ph, const double* Uin, double* Uout, double* K1, double a,
                   double b, double dt, int rhs_only, hipStream_t s, std::string& err) {
  switch (form) {
    case 0:
      return launch_stage_w<N, double, false>(tune, t, ph, Uin, Uout, K1, a, b, dt, rhs_only, s, err);
    case 1:
      return launch_stage_w<N, double, true>(tune, t, ph, Uin, Uout, K1, a, b, dt, rhs_only, s, err);
    case 2:
      return launch_stage_w<N, float, true>(tune, t, ph, Uin, Uout, K1, a, b, dt, rhs_only, s, err);
    case 3:
      return launch_stage_w<N, bf16ops, true>(tune, t, ph, Uin, Uout, K1, a, b, dt, rhs_only, s, err);
    case kFormOverint:
      return launch_oi_w<N>(tune, t, ph, Uin, Uout, K1, a, b, dt, rhs_only, s, err);
    default: err = "precision mode not built"; return -5;
  }
}

template <int N>
int launch_force_n(const DeviceTables& t, const KernelPhysics& ph, const double* U, double* out,
                   hipStream_t s, std::string& err) {
  const int blocks = (t.nwall * (N + 1) + kForceThreads - 1) / kForceThreads;
  if (blocks < 1 || blocks > t.force_blocks) {
    err = "wall force: workgroup count outside the set-up partial buffer";
    return -1;
  }
  hipLaunchKernelGGL(force_kernel<N>, dim3(blocks), dim3(kForceThreads), 0, s, t, ph, U, out);
  return launch_error(err, "force kernel launch");
}

template <int N, typename X, bool PERT, int W>
int launch_batch_order_t(const BatchItem* items, const BatchStep* steps, const int* parity,
                         const BatchGroup& g, int blocks, int stage, double a, double b,
                         hipStream_t s, std::string& err) {
  hipLaunchKernelGGL((batch_order_kernel<N, X, PERT, W>), dim3((unsigned)blocks), dim3(64 * W), 0, s,
                     items, steps, parity, g, stage, a, b);
  return launch_error(err, "batched stage kernel launch");
}

template <int N, typename X, bool PERT>
int launch_batch_order_w(int waves, const BatchItem* items, const BatchStep* steps,
                         const int* parity, const BatchGroup& g, int blocks, int stage, double a,
                         double b, hipStream_t s, std::string& err) {
  return waves == 4
             ? launch_batch_order_t<N, X, PERT, 4>(items, steps, parity, g, blocks, stage, a, b, s, err)
             : launch_batch_order_t<N, X, PERT, 2>(items, steps, parity, g, blocks, stage, a, b, s, err);
}

template <int N>
int launch_batch_order_n(int form, int waves, const BatchItem* items, const BatchStep* steps,
                         const int* parity, const BatchGroup& g, int blocks, int stage, double a,
                         double b, hipStream_t s, std::string& err) {
  switch (form) {
    case 0: return launch_batch_order_w<N, double, false>(waves, items, steps, parity, g, blocks, stage, a, b, s, err);
    case 1: return launch_batch_order_w<N, double, true>(waves, items, steps, parity, g, blocks, stage, a, b, s, err);
    case 2: return launch_batch_order_w<N, float, true>(waves, items, steps, parity, g, blocks, stage, a, b, s, err);
    case 3: return launch_batch_order_w<N, bf16ops, true>(waves, items, steps, parity, g, blocks, stage, a, b, s, err);
    default: err = "precision mode not built"; return -5;
  }
}

template <int N, typename X, bool PERT>
int batch_order_resident_x(int waves) {
  static int cache4[kMaxDev] = {0}, cache2[kMaxDev] = {0};
  return waves == 4 ? resident_blocks(batch_order_kernel<N, X, PERT, 4>, 256, cache4)
                    : resident_blocks(batch_order_kernel<N, X, PERT, 2>, 128, cache2);
}

template <int N>
int batch_order_resident_n(int form, int waves) {
  switch (form) {
    case 0: return batch_order_resident_x<N, double, false>(waves);
    case 1: return batch_order_resident_x<N, double, true>(waves);
    case 3: return batch_order_resident_x<N, bf16ops, true>(waves);
    default: return batch_order_resident_x<N, float, true>(waves);
  }
}

template <typename T, bool PERT, int W>
int launch_batch_t(const BatchItem* items, const BatchStep* steps, const int* parity,
                   const BatchGroups& G, int blocks, int stage, double a, double b, hipStream_t s,
                   std::string& err) {
  hipLaunchKernelGGL((batch_stage_kernel<T, PERT, W>), dim3((unsigned)blocks), dim3(64 * W), 0, s,
                     items, steps, parity, G, stage, a, b);
  return launch_error(err, "batched stage kernel launch");
}

template <typename T, bool PERT, int W>
int batch_resident_t() {
  static int cache[kMaxDev] = {0};
  return resident_blocks(batch_stage_kernel<T, PERT, W>, 64 * W, cache);
}
}  // namespace

int launch_stage(int N, int form, const StageTuning& tune, const DeviceTables& t,
                 const KernelPhysics& ph, const double* Uin, double* Uout, double* K1, double a,
                 double b, double dt, int rhs_only, void* stream, std::string& err) {
  hipStream_t s = (hipStream_t)stream;
  if (t.ncurved > 0 && form == kFormOverint) {
    err = "curved elements are not built for the over-integrated stage";
    return -5;
  }
  int rc;
  switch (N) {
    case 1: rc = launch_stage_n<1>(form, tune, t, ph, Uin, Uout, K1, a, b, dt, rhs_only, s, err); break;
    case 2: rc = launch_stage_n<2>(form, tune, t, ph, Uin, Uout, K1, a, b, dt, rhs_only, s, err); break;
    case 3: rc = launch_stage_n<3>(form, tune, t, ph, Uin, Uout, K1, a, b, dt, rhs_only, s, err); break;
    case 4: rc = launch_stage_n<4>(form, tune, t, ph, Uin, Uout, K1, a, b, dt, rhs_only, s, err); break;
    case 5: rc = launch_stage_n<5>(form, tune, t, ph, Uin, Uout, K1, a, b, dt, rhs_only, s, err); break;
    case 6: rc = launch_stage_n<6>(form, tune, t, ph, Uin, Uout, K1, a, b, dt, rhs_only, s, err); break;
    default: err = "polynomial order not built"; return -5;
  }
  return rc;
}

int default_waves(int, int) { return 4; }

int batch_order_resident_blocks(int N, int form, int waves) {
  switch (N) {
    case 1: return batch_order_resident_n<1>(form, waves);
    case 2: return batch_order_resident_n<2>(form, waves);
    case 3: return batch_order_resident_n<3>(form, waves);
    case 4: return batch_order_resident_n<4>(form, waves);
    case 5: return batch_order_resident_n<5>(form, waves);
    case 6: return batch_order_resident_n<6>(form, waves);
    default: return 0;
  }
}

int launch_batch_order_stage(int N, int form, int waves, const BatchItem* items,
                             const BatchStep* steps, const int* parity, const BatchGroup& g,
                             int blocks, int stage, double a, double b, void* stream,
                             std::string& err) {
  if (waves != 2 && waves != 4) {
    err = "waves per workgroup must be 2 or 4";
    return -1;
  }
  hipStream_t s = (hipStream_t)stream;
  switch (N) {
    case 1: return launch_batch_order_n<1>(form, waves, items, steps, parity, g, blocks, stage, a, b, s, err);
    case 2: return launch_batch_order_n<2>(form, waves, items, steps, parity, g, blocks, stage, a, b, s, err);
    case 3: return launch_batch_order_n<3>(form, waves, items, steps, parity, g, blocks, stage, a, b, s, err);
    case 4: return launch_batch_order_n<4>(form, waves, items, steps, parity, g, blocks, stage, a, b, s, err);
    case 5: return launch_batch_order_n<5>(form, waves, items, steps, parity, g, blocks, stage, a, b, s, err);
    case 6: return launch_batch_order_n<6>(form, waves, items, steps, parity, g, blocks, stage, a, b, s, err);
    default: err = "polynomial order not built"; return -5;
  }
}

int batch_resident_blocks(int form, int waves) {
  if (form == 0) return waves == 4 ? batch_resident_t<double, false, 4>() : batch_resident_t<double, false, 2>();
  if (form == 1) return waves == 4 ? batch_resident_t<double, true, 4>() : batch_resident_t<double, true, 2>();
  if (form == 3) return waves == 4 ? batch_resident_t<bf16ops, true, 4>() : batch_resident_t<bf16ops, true, 2>();
  return waves == 4 ? batch_resident_t<float, true, 4>() : batch_resident_t<float, true, 2>();
}

int launch_batch_stage(int form, int waves, const BatchItem* items, const BatchStep* steps,
                       const int* parity, const BatchGroups& G, int blocks, int stage, double a,
                       double b, void* stream, std::string& err) {
  hipStream_t s = (hipStream_t)stream;
  if (waves != 2 && waves != 4) {
    err = "waves per workgroup must be 2 or 4";
    return -1;
  }
  const bool w4 = waves == 4;
  switch (form) {
    case 0:
      return w4 ? launch_batch_t<double, false, 4>(items, steps, parity, G, blocks, stage, a, b, s, err)
                : launch_batch_t<double, false, 2>(items, steps, parity, G, blocks, stage, a, b, s, err);
    case 1:
      return w4 ? launch_batch_t<double, true, 4>(items, steps, parity, G, blocks, stage, a, b, s, err)
                : launch_batch_t<double, true, 2>(items, steps, parity, G, blocks, stage, a, b, s, err);
    case 2:
      return w4 ? launch_batch_t<float, true, 4>(items, steps, parity, G, blocks, stage, a, b, s, err)
                : launch_batch_t<float, true, 2>(items, steps, parity, G, blocks, stage, a, b, s, err);
    case 3:
      return w4 ? launch_batch_t<bf16ops, true, 4>(items, steps, parity, G, blocks, stage, a, b, s, err)
                : launch_batch_t<bf16ops, true, 2>(items, steps, parity, G, blocks, stage, a, b, s, err);
    default: err = "precision mode not built"; return -5;
  }
}

int force_blocks_for(int N, int nwall) {
  return (nwall * (N + 1) + kForceThreads - 1) / kForceThreads;
}

template <int N>
int launch_batch_force_n(const ForceItem* items, int count, int blocks, hipStream_t s,
                         std::string& err) {
  hipLaunchKernelGGL(batch_force_kernel<N>, dim3(blocks), dim3(kForceThreads), 0, s, items, count);
  return launch_error(err, "batched force kernel launch");
}

int launch_batch_force(int N, const ForceItem* items, int count, int blocks, void* stream,
                       std::string& err) {
  if (count < 1 || blocks < count) {
    err = "batched force: no instances or fewer workgroups than instances";
    return -1;
  }
  hipStream_t s = (hipStream_t)stream;
  switch (N) {
    case 1: return launch_batch_force_n<1>(items, count, blocks, s, err);
    case 2: return launch_batch_force_n<2>(items, count, blocks, s, err);
    case 3: return launch_batch_force_n<3>(items, count, blocks, s, err);
    case 4: return launch_batch_force_n<4>(items, count, blocks, s, err);
    case 5: return launch_batch_force_n<5>(items, count, blocks, s, err);
    case 6: return launch_batch_force_n<6>(items, count, blocks, s, err);
    default: err = "order not built"; return -5;
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
