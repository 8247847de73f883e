// Learned-closure kernels for gfx950: a per-element MLP
// (n_in -> H -> GELU -> H -> GELU -> n_out) trained and evaluated with
// bfloat16 operands on the matrix cores (FP32 accumulation; 16x16x16 in the
// layer-by-layer kernels, the double-depth 16x16x32 in the fused training
// step) and FP32 master weights, plus the per-element order-change maps that
// make its samples.
//
// Matrix-core operand layout (v_mfma_f32_16x16x16_bf16): lane l supplies
// A[l%16][4(l/16) + j] and B[4(l/16) + j][l%16], j = 0..3, and receives
// D[4(l/16) + v][l%16], v = 0..3.
#include <hip/hip_runtime.h>

#include "mlp_internal.h"

namespace dgmi {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16, round to nearest, ties to even
__device__ __forceinline__ unsigned short f2bf(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

// GELU (erf form) and its derivative from one exponential:
//   gelu(z) = z Phi(z), gelu'(z) = Phi(z) + z phi(z), Phi(z) = (1 + erf(z/sqrt2))/2,
// with erfc(x) = (a1 t + ... + a5 t^5) exp(-x^2), t = 1/(1 + p x), x >= 0
// (Abramowitz and Stegun, formula 7.1.26; absolute error <= 1.5e-7, far below
// the bfloat16 rounding of everything the layers store).  Phi(z) is taken as
// erfc(|x|)/2 on the negative side, so there is no cancellation there.
__device__ __forceinline__ void gelu_pair(float z, float& g, float& gp) {
  const float x = fabsf(z) * 0.70710678118654752f;
  const float e = __expf(-x * x);                 // exp(-z^2/2)
  const float t = __builtin_amdgcn_rcpf(1.0f + 0.3275911f * x);
  const float poly =
      t * (0.254829592f + t * (-0.284496736f + t * (1.421413741f + t * (-1.453152027f + t * 1.061405429f))));
  const float half_erfc = 0.5f * poly * e;        // Phi(-|z|)
  const float Phi = z >= 0.f ? 1.0f - half_erfc : half_erfc;
  g = z * Phi;
  gp = Phi + z * e * 0.39894228040143268f;        // 1/sqrt(2 pi)
}

// ---------------------------------------------------------------- dense layer
// out[B x N] = epilogue(A[B x K] W^T) with W[N x K] bfloat16 (row stride
// ldw), staged in LDS.  One wave computes 16 rows x all N = 16 NT columns;
// waves stride over the 16-row tiles.
//   A: bfloat16 [B][lda], or (NORM_IN) raw FP32 inputs normalised on the fly,
//      (x - mean) / std for columns < kvalid, 0 beyond (the normalised
//      bfloat16 copy is stored to Aout for the weight gradient).
enum DenseEpi { EPI_GELU = 0, EPI_OUT = 1, EPI_LOSS = 2, EPI_DGELU = 3 };

struct DenseArgs {
  const void* A;
  int64_t lda;
  const float* in_mean;      // NORM_IN
  const float* in_rstd;
  unsigned short* Aout;      // NORM_IN: normalised copy, ld = K
  int kvalid;
  const unsigned short* W;   // [N][ldw]
  int K, ldw;
  const float* bias;         // [N] (EPI_GELU, EPI_OUT, EPI_LOSS)
  int nvalid;                // valid output columns
  unsigned short* Gd;        // GELU derivative at the pre-activations, bfloat16 [B][N]:
                             // EPI_GELU output (skipped when null), EPI_DGELU input
  unsigned short* H;         // EPI_GELU / EPI_LOSS / EPI_DGELU output bfloat16 [B][N]
  float* Y;                  // EPI_OUT output [B][ldy]
  int64_t ldy;
  const float* T;            // EPI_LOSS raw targets [B][ldt]
  int64_t ldt;
  const float* out_mean;     // EPI_OUT / EPI_LOSS
  const float* out_std;
  float loss_scale;          // EPI_LOSS: 2 / (B n_out)
  double* loss_part;         // EPI_LOSS: one per workgroup
  int64_t B;
};

constexpr int KSMAX = 8;        // dense layers take K <= 128 inputs
constexpr int kDenseWaves = 8;  // one 16-row tile per wave; the workgroup shares the weights

template <int NT, int EPI, bool NORM_IN>
__global__ __launch_bounds__(64 * kDenseWaves) void dense_kernel(DenseArgs g) {
  constexpr int N = 16 * NT;
  extern __shared__ unsigned char smem[];
  const int K = g.K;
  const int ldl = K + 4;  // padded LDS row: rows start 2 banks apart
  unsigned short* sW = (unsigned short*)smem;
  double* sLoss = (double*)(smem + ((N * ldl * 2 + 15) / 16) * 16);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int ar = lane & 15, ak = 4 * (lane >> 4);
  const int64_t ntiles = (g.B + 15) / 16;
  const int64_t stride = (int64_t)gridDim.x * kDenseWaves;
  const int nks = K / 16;
  // a tile's inputs in registers: the whole A row slice (K <= 16 KSMAX) and
  // what the epilogue reads (the stored GELU derivative, the targets for the
  // loss), all issued together so that one memory latency covers them
  bf16x4 a[KSMAX];
  float ez[NT][4];
  auto load_tile = [&](int64_t tl) {
    const int64_t row = tl * 16 + ar;
    const bool rok = row < g.B;
#pragma unroll
    for (int ks = 0; ks < KSMAX; ++ks) {
      a[ks] = bf16x4{0, 0, 0, 0};
      if (ks >= nks) continue;
      const int k0 = ks * 16 + ak;
      if (NORM_IN) {
        const float* X = (const float*)g.A;
        unsigned short h[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int k = k0 + j;
          const float x = (rok && k < g.kvalid) ? (X[row * g.lda + k] - g.in_mean[k]) * g.in_rstd[k] : 0.f;
          h[j] = f2bf(x);
        }
        if (rok)
          *(uint2*)(g.Aout + row * K + k0) =
              make_uint2((unsigned)h[0] | ((unsigned)h[1] << 16), (unsigned)h[2] | ((unsigned)h[3] << 16));
        a[ks] = bf16x4{(short)h[0], (short)h[1], (short)h[2], (short)h[3]};
      } else if (rok) {
        const unsigned short* A = (const unsigned short*)g.A;
        const uint2 v = *(const uint2*)(A + row * g.lda + k0);
        a[ks] = bf16x4{(short)(v.x & 0xffff), (short)(v.x >> 16), (short)(v.y & 0xffff), (short)(v.y >> 16)};
      }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int c0 = t * 16 + ak;
      if (EPI == EPI_DGELU) {
        uint2 w = make_uint2(0u, 0u);
        if (rok) w = *(const uint2*)(g.Gd + row * N + c0);
        ez[t][0] = bf2f((unsigned short)(w.x & 0xffff));
        ez[t][1] = bf2f((unsigned short)(w.x >> 16));
        ez[t][2] = bf2f((unsigned short)(w.y & 0xffff));
        ez[t][3] = bf2f((unsigned short)(w.y >> 16));
      } else if (EPI == EPI_LOSS) {
        // four consecutive targets: one 16-byte load where the row stride and
        // the columns allow it
        const float* tp = g.T + row * g.ldt + c0;
        if (rok && c0 + 3 < g.nvalid && (g.ldt & 3) == 0 && (((uintptr_t)g.T) & 15) == 0) {
          const float4 q = *(const float4*)tp;
          ez[t][0] = q.x; ez[t][1] = q.y; ez[t][2] = q.z; ez[t][3] = q.w;
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v) ez[t][v] = (rok && c0 + v < g.nvalid) ? tp[v] : 0.f;
        }
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) ez[t][v] = 0.f;
      }
    }
  };
  int64_t tile = (int64_t)blockIdx.x * kDenseWaves + wid;
  load_tile(tile);
  // weights: 8-byte words (K and ldw are multiples of 16, rows 8-byte aligned),
  // all of a thread's loads in flight together
  const int kw = K / 4;
#pragma unroll 8
  for (int i = threadIdx.x; i < N * kw; i += blockDim.x) {
    const int n = i / kw, k = 4 * (i - n * kw);
    *(uint2*)(sW + n * ldl + k) = *(const uint2*)(g.W + (int64_t)n * g.ldw + k);
  }
  __syncthreads();
  double loss = 0.0;
  for (; tile < ntiles; tile += stride) {
    f32x4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KSMAX; ++ks) {
      if (ks >= nks) break;
      const int k0 = ks * 16 + ak;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const uint2 w = *(const uint2*)(sW + (t * 16 + ar) * ldl + k0);
        const bf16x4 b{(short)(w.x & 0xffff), (short)(w.x >> 16), (short)(w.y & 0xffff), (short)(w.y >> 16)};
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(b, a[ks], acc[t], 0, 0, 0);
      }
    }
    // the product is formed transposed (weights as the row operand), so lane l
    // holds sample row l%16 of the tile and the four consecutive output columns
    // 16 t + 4(l/16) + v: the bfloat16 outputs go out as one 8-byte store each
    const int64_t r = tile * 16 + ar;
    const bool rok = r < g.B;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int c0 = t * 16 + ak;
      unsigned short h[4] = {0, 0, 0, 0}, hd[4] = {0, 0, 0, 0};
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int col = c0 + v;
        const float s = acc[t][v];
        if (EPI == EPI_GELU) {
          const float z = s + g.bias[col];
          float act, der;
          gelu_pair(z, act, der);
          h[v] = f2bf(act);
          hd[v] = f2bf(der);
        } else if (EPI == EPI_OUT) {
          if (rok && col < g.nvalid) g.Y[r * g.ldy + col] = g.out_mean[col] + g.out_std[col] * (s + g.bias[col]);
        } else if (EPI == EPI_LOSS) {
          float d = 0.f;
          if (rok && col < g.nvalid) {
            const float tn = (ez[t][v] - g.out_mean[col]) / g.out_std[col];
            const float res = s + g.bias[col] - tn;
            loss += (double)res * (double)res;
            d = g.loss_scale * res;
          }
          h[v] = f2bf(d);
        } else {  // EPI_DGELU
          h[v] = f2bf(s * ez[t][v]);
        }
      }
      if (EPI != EPI_OUT && rok) {
        *(uint2*)(g.H + r * N + c0) =
            make_uint2((unsigned)h[0] | ((unsigned)h[1] << 16), (unsigned)h[2] | ((unsigned)h[3] << 16));
        if (EPI == EPI_GELU && g.Gd)
          *(uint2*)(g.Gd + r * N + c0) =
              make_uint2((unsigned)hd[0] | ((unsigned)hd[1] << 16), (unsigned)hd[2] | ((unsigned)hd[3] << 16));
      }
    }
    if (tile + stride < ntiles) load_tile(tile + stride);
  }
  if (EPI == EPI_LOSS) {
    // fixed-shape reduction of the squared residuals of this workgroup
    for (int o = 32; o > 0; o >>= 1) loss += __shfl_down(loss, o, 64);
    if (lane == 0) sLoss[wid] = loss;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < kDenseWaves; ++w) t += sLoss[w];
      g.loss_part[blockIdx.x] = t;
    }
  }
}

// ---------------------------------------------------------------- weight gradient
// part[blk] <- (sum over this workgroup's samples of G[b][n] A[b][k]) for
// n < nvalid, k < kvalid, followed by the bias part sum_b G[b][n].  Samples
// are staged 64 at a time in LDS (the k-index of the products); wave w owns
// the 16-row output tiles [w TNW, (w + 1) TNW) against all TK column tiles.
struct WgradArgs {
  const unsigned short* G;   // [B][NG]
  const unsigned short* A;   // [B][KA]
  int NG, KA, nvalid, kvalid;
  int64_t B, chunk;          // samples per workgroup (multiple of 64)
  float* part;               // [gridDim][nvalid * kvalid + nvalid]
};

template <int TNW, int TK>
__global__ __launch_bounds__(256) void wgrad_kernel(WgradArgs g) {
  extern __shared__ unsigned char smem[];
  const int NG = g.NG, KA = 16 * TK;
  const int ldg = NG + 4, lda = KA + 4;
  unsigned short* sG = (unsigned short*)smem;   // [64][ldg]
  unsigned short* sA = sG + 64 * ldg;           // [64][lda]
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int tn = NG / 16;
  f32x4 acc[TNW][TK];
#pragma unroll
  for (int i = 0; i < TNW; ++i)
#pragma unroll
    for (int t = 0; t < TK; ++t) acc[i][t] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;  // thread t < NG: bias column t
  const int64_t b0 = (int64_t)blockIdx.x * g.chunk;
  const int64_t b1 = b0 + g.chunk < g.B ? b0 + g.chunk : g.B;
  // A chunk of 64 samples is 16 NG + 16 KA 8-byte words (NG, KA <= 128): at
  // most eight of each per thread, held in registers so that the next chunk's
  // loads are in flight during this chunk's matrix-core work
  constexpr int PW = 8;
  const int gw = NG / 4, aw = KA / 4;
  uint2 pg[PW], pa[PW];
  auto fetch = [&](int64_t c) {
#pragma unroll
    for (int j = 0; j < PW; ++j) {
      const int i = threadIdx.x + 256 * j;
      const int rg = i / gw, ra = i / aw;
      pg[j] = (i < 16 * NG && c + rg < b1) ? *(const uint2*)(g.G + (c + rg) * NG + 4 * (i - rg * gw))
                                           : make_uint2(0u, 0u);
      pa[j] = (i < 16 * KA && c + ra < b1) ? *(const uint2*)(g.A + (c + ra) * KA + 4 * (i - ra * aw))
                                           : make_uint2(0u, 0u);
    }
  };
  if (b0 < b1) fetch(b0);
#pragma unroll 1
  for (int64_t c = b0; c < b1; c += 64) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PW; ++j) {
      const int i = threadIdx.x + 256 * j;
      const int rg = i / gw, ra = i / aw;
      if (i < 16 * NG) *(uint2*)(sG + rg * ldg + 4 * (i - rg * gw)) = pg[j];
      if (i < 16 * KA) *(uint2*)(sA + ra * lda + 4 * (i - ra * aw)) = pa[j];
    }
    __syncthreads();
    if (c + 64 < b1) fetch(c + 64);
    if (threadIdx.x < NG) {
      // sequential over the samples (fixed order); the LDS reads are issued
      // ahead of the adds
#pragma unroll
      for (int r0 = 0; r0 < 64; r0 += 16) {
        float v[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = bf2f(sG[(r0 + r) * ldg + threadIdx.x]);
#pragma unroll
        for (int r = 0; r < 16; ++r) bsum += v[r];
      }
    }
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      // A operand: row n, k-index sample; B operand: k-index sample, column k
      const int sb = ks * 16 + 4 * (lane >> 4);
      bf16x4 bfr[TK];
#pragma unroll
      for (int t = 0; t < TK; ++t) {
        const int col = 16 * t + (lane & 15);
        bfr[t] = bf16x4{(short)sA[(sb + 0) * lda + col], (short)sA[(sb + 1) * lda + col],
                        (short)sA[(sb + 2) * lda + col], (short)sA[(sb + 3) * lda + col]};
      }
#pragma unroll
      for (int i = 0; i < TNW; ++i) {
        const int nt = wid * TNW + i;
        if (nt >= tn) break;
        const int row = 16 * nt + (lane & 15);
        const bf16x4 afr{(short)sG[(sb + 0) * ldg + row], (short)sG[(sb + 1) * ldg + row],
                         (short)sG[(sb + 2) * ldg + row], (short)sG[(sb + 3) * ldg + row]};
#pragma unroll
        for (int t = 0; t < TK; ++t)
          acc[i][t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(afr, bfr[t], acc[i][t], 0, 0, 0);
      }
    }
  }
  float* out = g.part + (int64_t)blockIdx.x * ((int64_t)g.nvalid * g.kvalid + g.nvalid);
#pragma unroll
  for (int i = 0; i < TNW; ++i) {
    const int nt = wid * TNW + i;
    if (nt >= tn) break;
#pragma unroll
    for (int t = 0; t < TK; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int n = 16 * nt + 4 * (lane >> 4) + v, k = 16 * t + (lane & 15);
        if (n < g.nvalid && k < g.kvalid) out[n * g.kvalid + k] = acc[i][t][v];
      }
  }
  if (threadIdx.x < g.nvalid) out[(int64_t)g.nvalid * g.kvalid + threadIdx.x] = bsum;
}

// ---------------------------------------------------------------- fused training step
// One training step's forward pass, loss, backward pass and weight gradients
// in one launch, for the shapes in_pad = 16 KIT, H = 16 HT, out_pad = 16 OT.
// A workgroup of four waves takes 64 samples at a time, one 16-row tile per
// wave.  A wave's tile goes through the three layers in registers: the
// transposed products (weights as the row operand) leave lane l with sample
// l%16 and four consecutive output columns, which are exactly its B operand
// for the next layer, and the GELU derivatives stay in FP32 registers for the
// backward pass.  What the weight gradients need -- the normalised inputs,
// both hidden activations and the three output gradients -- is written to LDS
// transposed ([column][sample], bfloat16), so that after a barrier every
// wave reads its operands as 8-byte words: wave w accumulates the output
// tiles of dW1, dW2 with row tiles w and w + 4, and of dW3 with row tile w,
// over the block's 64 samples on the matrix cores.  The bias gradients are
// per-thread sums over the same arrays (fixed order).  At the end each
// workgroup writes its whole gradient (the parameter vector's layout) as one
// partial; reduce_parts_kernel sums them in a fixed order.  HBM traffic per
// sample: the inputs and targets only.
struct TrainArgs {
  const float* X;
  int64_t ldx;
  const float* T;
  int64_t ldt;
  int64_t B, chunk;          // samples; samples per workgroup (multiple of 64)
  int n_in, n_out;
  const float* in_mean;
  const float* in_rstd;
  const float* out_mean;
  const float* out_std;
  const unsigned short* W1;  // [H][ldw1]
  const unsigned short* W2;  // [H][ldw2]
  const unsigned short* W3;  // [out_pad][ldw3]
  int ldw1, ldw2, ldw3;
  const float* b1;
  const float* b2;
  const float* b3;
  float loss_scale;          // 2 / (B n_out)
  double* loss_part;         // one per workgroup
  float* part;               // [gridDim][stride]: W1 b1 W2 b2 W3 b3
  int64_t stride;
  int64_t woff[3], boff[3];
};

__device__ __forceinline__ bf16x4 bf4(const float v[4]) {
  return bf16x4{(short)f2bf(v[0]), (short)f2bf(v[1]), (short)f2bf(v[2]), (short)f2bf(v[3])};
}
__device__ __forceinline__ bf16x4 ld_bf4(const unsigned short* p) {
  const uint2 w = *(const uint2*)p;
  return bf16x4{(short)(w.x & 0xffff), (short)(w.x >> 16), (short)(w.y & 0xffff), (short)(w.y >> 16)};
}

// gfx950's double-depth instruction (v_mfma_f32_16x16x32_bf16): lane l supplies
// eight k-slots of A row l%16 and of B column l%16, and slot j of lane group
// l/16 of A meets slot j of the same group of B, so any assignment of the 32
// k values to (group, slot) that both operands share gives the product.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ f32x4 mma32(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
// slots 0-3 from lo, 4-7 from hi
__device__ __forceinline__ bf16x8 cat8(bf16x4 lo, bf16x4 hi) {
  return __builtin_bit_cast(bf16x8, (s16x8)__builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7));
}
// eight consecutive bfloat16 values (16-byte aligned)
__device__ __forceinline__ bf16x8 ld_bf8(const unsigned short* p) {
  return __builtin_bit_cast(bf16x8, *(const u32x4*)p);
}

template <int KIT, int HT, int OT>
struct TrainShape {
  static constexpr int KI = 16 * KIT, H = 16 * HT, NO = 16 * OT;
  static constexpr int L1 = KI + 4, L2 = H + 4, L3 = H + 4;  // weight rows in LDS
  static constexpr int LT = 64 + 8;  // transposed rows (samples; 16-byte aligned, no bank aliasing)
  static constexpr int W_SZ = H * L1 + H * L2 + NO * L3;
  static constexpr int T_SZ = LT * (KI + 4 * H + NO);
};

template <int KIT, int HT, int OT>
__global__ __launch_bounds__(256) void train_kernel(TrainArgs g) {
  using S = TrainShape<KIT, HT, OT>;
  constexpr int KI = S::KI, H = S::H, NO = S::NO, L1 = S::L1, L2 = S::L2, L3 = S::L3, LT = S::LT;
  static_assert(HT == 8 && OT <= 4, "shape not built: waves take row tiles wid and wid + 4");
  static_assert(KIT % 2 == 0 && OT % 2 == 0, "the double-depth products pair k-tiles");
  __shared__ __attribute__((aligned(16))) unsigned short sW[S::W_SZ];
  __shared__ __attribute__((aligned(16))) unsigned short sT[S::T_SZ];
  __shared__ double sLoss[4];
  unsigned short* sW1 = sW;
  unsigned short* sW2 = sW1 + H * L1;
  unsigned short* sW3 = sW2 + H * L2;
  unsigned short* tX = sT;                 // [KI][LT]
  unsigned short* tH1 = tX + KI * LT;      // [H][LT]
  unsigned short* tH2 = tH1 + H * LT;
  unsigned short* tZ1 = tH2 + H * LT;      // dZ1
  unsigned short* tZ2 = tZ1 + H * LT;      // dZ2
  unsigned short* tDY = tZ2 + H * LT;      // [NO][LT]
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int ar = lane & 15, ak = 4 * (lane >> 4);

  // weights into LDS, 8-byte words
  for (int i = threadIdx.x; i < H * (KI / 4); i += 256) {
    const int n = i / (KI / 4), k = 4 * (i - n * (KI / 4));
    *(uint2*)(sW1 + n * L1 + k) = *(const uint2*)(g.W1 + (int64_t)n * g.ldw1 + k);
  }
  for (int i = threadIdx.x; i < H * (H / 4); i += 256) {
    const int n = i / (H / 4), k = 4 * (i - n * (H / 4));
    *(uint2*)(sW2 + n * L2 + k) = *(const uint2*)(g.W2 + (int64_t)n * g.ldw2 + k);
  }
  for (int i = threadIdx.x; i < NO * (H / 4); i += 256) {
    const int n = i / (H / 4), k = 4 * (i - n * (H / 4));
    *(uint2*)(sW3 + n * L3 + k) = *(const uint2*)(g.W3 + (int64_t)n * g.ldw3 + k);
  }

  f32x4 acc1[2][KIT], acc2[2][HT], acc3[HT];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
#pragma unroll
    for (int t = 0; t < KIT; ++t) acc1[i][t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < HT; ++t) acc2[i][t] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
#pragma unroll
  for (int t = 0; t < HT; ++t) acc3[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum[2] = {0.f, 0.f};  // bias entries threadIdx.x and threadIdx.x + 256
  double loss = 0.0;

  const int64_t s_begin = (int64_t)blockIdx.x * g.chunk;
  const int64_t s_end = s_begin + g.chunk < g.B ? s_begin + g.chunk : g.B;
  // a tile's inputs and targets (raw FP32), loaded one block ahead
  float xr[KIT][4], tr[OT][4];
  auto load = [&](int64_t s0) {
    const int64_t row = s0 + 16 * wid + ar;
    const bool rok = row < s_end;
#pragma unroll
    for (int ks = 0; ks < KIT; ++ks)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = 16 * ks + ak + j;
        xr[ks][j] = (rok && k < g.n_in) ? g.X[row * g.ldx + k] : 0.f;
      }
#pragma unroll
    for (int t = 0; t < OT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int c = 16 * t + ak + v;
        tr[t][v] = (rok && c < g.n_out) ? g.T[row * g.ldt + c] : 0.f;
      }
  };
  if (s_begin < s_end) load(s_begin);
  __syncthreads();

#pragma unroll 1
  for (int64_t s0 = s_begin; s0 < s_end; s0 += 64) {
    const int64_t row = s0 + 16 * wid + ar;
    const bool rok = row < s_end;
    const int col = 16 * wid + ar;  // this lane's sample column in the transposed arrays
    // ---- forward: normalised inputs (zero beyond n_in and past the end)
    bf16x4 a1[KIT];
#pragma unroll
    for (int ks = 0; ks < KIT; ++ks) {
      float v[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = 16 * ks + ak + j;
        v[j] = (rok && k < g.n_in) ? (xr[ks][j] - g.in_mean[k]) * g.in_rstd[k] : 0.f;
      }
      a1[ks] = bf4(v);
#pragma unroll
      for (int j = 0; j < 4; ++j) tX[(16 * ks + ak + j) * LT + col] = (unsigned short)a1[ks][j];
    }
    float d1[HT][4], d2[HT][4];  // GELU derivatives at the pre-activations
    bf16x4 h1[HT], h2[HT];
    // the HT output tiles as independent accumulator chains (k-steps outer)
    f32x4 acc[HT];
#pragma unroll
    for (int t = 0; t < HT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    // the double-depth products take k-tiles 2q (slots 0-3) and 2q + 1 (slots
    // 4-7): lane group g holds k = 16 (2q) + 4g + j and 16 (2q + 1) + 4g + j,
    // exactly the values the previous product left in the lane
#pragma unroll
    for (int q = 0; q < KIT / 2; ++q) {
      const bf16x8 b = cat8(a1[2 * q], a1[2 * q + 1]);
#pragma unroll
      for (int t = 0; t < HT; ++t) {
        const unsigned short* w = sW1 + (16 * t + ar) * L1 + 32 * q + ak;
        acc[t] = mma32(cat8(ld_bf4(w), ld_bf4(w + 16)), b, acc[t]);
      }
    }
#pragma unroll
    for (int t = 0; t < HT; ++t) {
      float v[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) gelu_pair(acc[t][j] + g.b1[16 * t + ak + j], v[j], d1[t][j]);
      h1[t] = bf4(v);
#pragma unroll
      for (int j = 0; j < 4; ++j) tH1[(16 * t + ak + j) * LT + col] = (unsigned short)h1[t][j];
    }
#pragma unroll
    for (int t = 0; t < HT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < HT / 2; ++q) {
      const bf16x8 b = cat8(h1[2 * q], h1[2 * q + 1]);
#pragma unroll
      for (int t = 0; t < HT; ++t) {
        const unsigned short* w = sW2 + (16 * t + ar) * L2 + 32 * q + ak;
        acc[t] = mma32(cat8(ld_bf4(w), ld_bf4(w + 16)), b, acc[t]);
      }
    }
#pragma unroll
    for (int t = 0; t < HT; ++t) {
      float v[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) gelu_pair(acc[t][j] + g.b2[16 * t + ak + j], v[j], d2[t][j]);
      h2[t] = bf4(v);
#pragma unroll
      for (int j = 0; j < 4; ++j) tH2[(16 * t + ak + j) * LT + col] = (unsigned short)h2[t][j];
    }
    // ---- output layer and loss: dY = 2 (y - t_n) / (B n_out), normalised units
    bf16x4 dy[OT];
#pragma unroll
    for (int t = 0; t < OT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < HT / 2; ++q) {
      const bf16x8 b = cat8(h2[2 * q], h2[2 * q + 1]);
#pragma unroll
      for (int t = 0; t < OT; ++t) {
        const unsigned short* w = sW3 + (16 * t + ar) * L3 + 32 * q + ak;
        acc[t] = mma32(cat8(ld_bf4(w), ld_bf4(w + 16)), b, acc[t]);
      }
    }
#pragma unroll
    for (int t = 0; t < OT; ++t) {
      float v[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int c = 16 * t + ak + j;
        v[j] = 0.f;
        if (rok && c < g.n_out) {
          const float tn = (tr[t][j] - g.out_mean[c]) / g.out_std[c];
          const float res = acc[t][j] + g.b3[c] - tn;
          loss += (double)res * (double)res;
          v[j] = g.loss_scale * res;
        }
      }
      dy[t] = bf4(v);
#pragma unroll
      for (int j = 0; j < 4; ++j) tDY[(16 * t + ak + j) * LT + col] = (unsigned short)dy[t][j];
    }
    // the next block's inputs, in flight during the backward pass
    if (s0 + 64 < s_end) load(s0 + 64);
    // ---- backward: dZ2 = (dY W3) gelu'(Z2), dZ1 = (dZ2 W2) gelu'(Z1); the
    // transposed weights are read from the row-major copies, four rows apart
    bf16x4 z2[HT];
#pragma unroll
    for (int t = 0; t < HT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < OT / 2; ++q) {
      const bf16x8 b = cat8(dy[2 * q], dy[2 * q + 1]);
#pragma unroll
      for (int t = 0; t < HT; ++t) {
        const unsigned short* w = sW3 + (32 * q + ak) * L3 + 16 * t + ar;
        const unsigned short* v = w + 16 * L3;
        const s16x8 wt{(short)w[0], (short)w[L3], (short)w[2 * L3], (short)w[3 * L3],
                       (short)v[0], (short)v[L3], (short)v[2 * L3], (short)v[3 * L3]};
        acc[t] = mma32(__builtin_bit_cast(bf16x8, wt), b, acc[t]);
      }
    }
#pragma unroll
    for (int t = 0; t < HT; ++t) {
      float v[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j] = acc[t][j] * d2[t][j];
      z2[t] = bf4(v);
#pragma unroll
      for (int j = 0; j < 4; ++j) tZ2[(16 * t + ak + j) * LT + col] = (unsigned short)z2[t][j];
    }
#pragma unroll
    for (int t = 0; t < HT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < HT / 2; ++q) {
      const bf16x8 b = cat8(z2[2 * q], z2[2 * q + 1]);
#pragma unroll
      for (int t = 0; t < HT; ++t) {
        const unsigned short* w = sW2 + (32 * q + ak) * L2 + 16 * t + ar;
        const unsigned short* v = w + 16 * L2;
        const s16x8 wt{(short)w[0], (short)w[L2], (short)w[2 * L2], (short)w[3 * L2],
                       (short)v[0], (short)v[L2], (short)v[2 * L2], (short)v[3 * L2]};
        acc[t] = mma32(__builtin_bit_cast(bf16x8, wt), b, acc[t]);
      }
    }
#pragma unroll
    for (int t = 0; t < HT; ++t) {
      float v[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j] = acc[t][j] * d1[t][j];
      const bf16x4 z1 = bf4(v);
#pragma unroll
      for (int j = 0; j < 4; ++j) tZ1[(16 * t + ak + j) * LT + col] = (unsigned short)z1[j];
    }
    __syncthreads();
    // ---- weight gradients of the block: dW[n][k] += sum_s dZ[s][n] A[s][k],
    // the samples as the double-depth k (lane group g: samples 32 ks + 8g ..
    // 32 ks + 8g + 7, one 16-byte read per operand)
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const int sb = 32 * ks + 2 * ak;  // samples sb .. sb + 7 of the block
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int nt = wid + 4 * i;
        const bf16x8 az1 = ld_bf8(tZ1 + (16 * nt + ar) * LT + sb);
        const bf16x8 az2 = ld_bf8(tZ2 + (16 * nt + ar) * LT + sb);
#pragma unroll
        for (int kt = 0; kt < KIT; ++kt) acc1[i][kt] = mma32(az1, ld_bf8(tX + (16 * kt + ar) * LT + sb), acc1[i][kt]);
#pragma unroll
        for (int kt = 0; kt < HT; ++kt) acc2[i][kt] = mma32(az2, ld_bf8(tH1 + (16 * kt + ar) * LT + sb), acc2[i][kt]);
      }
      if (wid < OT) {
        const bf16x8 ady = ld_bf8(tDY + (16 * wid + ar) * LT + sb);
#pragma unroll
        for (int kt = 0; kt < HT; ++kt) acc3[kt] = mma32(ady, ld_bf8(tH2 + (16 * kt + ar) * LT + sb), acc3[kt]);
      }
    }
    // bias gradients: thread t sums its rows of dZ1 | dZ2 | dY over the block
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int e = threadIdx.x + 256 * r;
      if (e < 2 * H + NO) {
        const unsigned short* rowp = e < H ? tZ1 + e * LT : (e < 2 * H ? tZ2 + (e - H) * LT : tDY + (e - 2 * H) * LT);
        float sum = 0.f;
#pragma unroll
        for (int s = 0; s < 64; s += 4) {
          const bf16x4 q = ld_bf4(rowp + s);
          sum += ((bf2f((unsigned short)q[0]) + bf2f((unsigned short)q[1])) + bf2f((unsigned short)q[2])) +
                 bf2f((unsigned short)q[3]);
        }
        bsum[r] += sum;
      }
    }
    __syncthreads();
  }

  // ---- this workgroup's partial: the whole gradient vector
  float* out = g.part + (int64_t)blockIdx.x * g.stride;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int nt = wid + 4 * i;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int n = 16 * nt + ak + v;
#pragma unroll
      for (int kt = 0; kt < KIT; ++kt) {
        const int k = 16 * kt + ar;
        if (k < g.n_in) out[g.woff[0] + (int64_t)n * g.n_in + k] = acc1[i][kt][v];
      }
#pragma unroll
      for (int kt = 0; kt < HT; ++kt) out[g.woff[1] + (int64_t)n * H + 16 * kt + ar] = acc2[i][kt][v];
    }
  }
  if (wid < OT) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int n = 16 * wid + ak + v;
      if (n < g.n_out)
#pragma unroll
        for (int kt = 0; kt < HT; ++kt) out[g.woff[2] + (int64_t)n * H + 16 * kt + ar] = acc3[kt][v];
    }
  }
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int e = threadIdx.x + 256 * r;
    if (e < H) out[g.boff[0] + e] = bsum[r];
    else if (e < 2 * H) out[g.boff[1] + (e - H)] = bsum[r];
    else if (e < 2 * H + g.n_out) out[g.boff[2] + (e - 2 * H)] = bsum[r];
  }
  for (int o = 32; o > 0; o >>= 1) loss += __shfl_down(loss, o, 64);
  if (lane == 0) sLoss[wid] = loss;
  __syncthreads();
  if (threadIdx.x == 0) g.loss_part[blockIdx.x] = ((sLoss[0] + sLoss[1]) + sLoss[2]) + sLoss[3];
}

// gradient = sum over the workgroup partials in a fixed order: wave w of a
// workgroup sums the partials p = w mod 4 in increasing p for 64 consecutive
// entries, then the four wave sums are added in wave order
__global__ __launch_bounds__(256) void reduce_parts_kernel(const float* __restrict__ part, int nparts,
                                                           int64_t stride, int64_t n,
                                                           float* __restrict__ out) {
  __shared__ float sw[4][64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  float s = 0.f;
  if (i < n) {
    int p = wid;
    for (; p + 28 < nparts; p += 32) {
      float v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = part[(int64_t)(p + 4 * j) * stride + i];
#pragma unroll
      for (int j = 0; j < 8; ++j) s += v[j];
    }
    for (; p < nparts; p += 4) s += part[(int64_t)p * stride + i];
  }
  sw[wid][lane] = s;
  __syncthreads();
  if (wid == 0 && i < n) out[i] = ((sw[0][lane] + sw[1][lane]) + sw[2][lane]) + sw[3][lane];
}

// Adam with bias correction on the FP32 master parameters; the bfloat16 copies
// (row-major W[N][ldw] and transposed WT[K][ldwt]) of every weight entry are
// refreshed.  Layout of the parameter vector: W1 b1 W2 b2 W3 b3, W row-major
// [n_out_l][n_in_l] (unpadded).
__global__ void adam_kernel(MlpDev d, float lr, float beta1, float beta2, float eps, float bc1,
                            float bc2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.nparams) return;
  const float gr = d.grad[i];
  const float m = beta1 * d.m[i] + (1.f - beta1) * gr;
  const float v = beta2 * d.v[i] + (1.f - beta2) * gr * gr;
  d.m[i] = m;
  d.v[i] = v;
  const float p = d.params[i] - lr * (m / bc1) / (sqrtf(v / bc2) + eps);
  d.params[i] = p;
  // which weight entry (biases have no bfloat16 copy)
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    const int64_t off = d.woff[l];
    const int rows = d.wrows[l], cols = d.wcols[l];
    if (i >= off && i < off + (int64_t)rows * cols) {
      const int r = (int)((i - off) / cols), c = (int)((i - off) % cols);
      const unsigned short h = f2bf(p);
      d.wb[l][r * d.ldw[l] + c] = h;
      d.wt[l][c * d.ldwt[l] + r] = h;
    }
  }
}

// bfloat16 copies of every weight from the master parameters (after a set)
__global__ void refresh_bf16_kernel(MlpDev d) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.nparams) return;
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    const int64_t off = d.woff[l];
    const int rows = d.wrows[l], cols = d.wcols[l];
    if (i >= off && i < off + (int64_t)rows * cols) {
      const int r = (int)((i - off) / cols), c = (int)((i - off) % cols);
      const unsigned short h = f2bf(d.params[i]);
      d.wb[l][r * d.ldw[l] + c] = h;
      d.wt[l][c * d.ldwt[l] + r] = h;
    }
  }
}

// per-column sum and sum of squares (FP64) of rows [blk*chunk, ...): lane =
// column (cols <= 64), waves stride over rows; one partial per workgroup
__global__ __launch_bounds__(256) void column_stats_kernel(const float* __restrict__ A, int64_t rows,
                                                           int64_t ld, int cols, int64_t chunk,
                                                           double* __restrict__ part) {
  __shared__ double s1[4][64], s2[4][64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  const int64_t r1 = r0 + chunk < rows ? r0 + chunk : rows;
  double a = 0.0, b = 0.0;
  if (lane < cols)
    for (int64_t r = r0 + wid; r < r1; r += 4) {
      const double x = A[r * ld + lane];
      a += x;
      b += x * x;
    }
  s1[wid][lane] = a;
  s2[wid][lane] = b;
  __syncthreads();
  if (threadIdx.x < 64) {
    part[((int64_t)blockIdx.x * 64 + threadIdx.x) * 2] =
        s1[0][threadIdx.x] + s1[1][threadIdx.x] + s1[2][threadIdx.x] + s1[3][threadIdx.x];
    part[((int64_t)blockIdx.x * 64 + threadIdx.x) * 2 + 1] =
        s2[0][threadIdx.x] + s2[1][threadIdx.x] + s2[2][threadIdx.x] + s2[3][threadIdx.x];
  }
}

// ---------------------------------------------------------------- order maps
// One thread per (element, field).  Samples x = [P (U - U_inf) field-major,
// rx ry sx sy] (from_hi) or [(U_lo - U_inf), rx ry sx sy]; targets
// t = U_hi - I P U_hi; apply: U_hi = I U_lo + Y.  A thread's input row and
// intermediate row live in LDS columns (thread t at word t of every row, so the
// lanes of a wave touch consecutive banks); the operator entries are
// wave-uniform loads.  Sums run in increasing node order.
constexpr int kMapThreads = 64;

__device__ __forceinline__ double field_of(const double v[4], int f) {
  return f == 0 ? v[0] : (f == 1 ? v[1] : (f == 2 ? v[2] : v[3]));
}

__global__ __launch_bounds__(kMapThreads) void closure_features_kernel(ClosureDev c, const double* __restrict__ U,
                                                                       int from_hi, float* __restrict__ X,
                                                                       int64_t ldx) {
  __shared__ double sv[kMaxNodes * kMapThreads];
  const int64_t gid = (int64_t)blockIdx.x * kMapThreads + threadIdx.x;
  const int64_t k = gid >> 2;
  const int f = (int)(gid & 3);
  if (k >= c.K) return;
  const int nl = c.np_lo, nh = c.np_hi;
  const double u0 = field_of(c.U_inf, f);
  float* x = X + k * ldx;
  if (from_hi == 2) {
    // the free stream's sample: no deviation from U_inf
    for (int m = 0; m < nl; ++m) x[f * nl + m] = 0.0f;
  } else if (from_hi) {
    const double* u = U + (k * 4 + f) * nh;
    double* col = sv + threadIdx.x;
#pragma unroll 8
    for (int n = 0; n < nh; ++n) col[n * kMapThreads] = u[n] - u0;
    for (int m = 0; m < nl; ++m) {
      double acc = 0.0;
      for (int n = 0; n < nh; ++n) acc += c.P[m * nh + n] * col[n * kMapThreads];
      x[f * nl + m] = (float)acc;
    }
  } else {
    const double* u = U + (k * 4 + f) * nl;
    for (int m = 0; m < nl; ++m) x[f * nl + m] = (float)(u[m] - u0);
  }
  x[4 * nl + f] = (float)c.geo[k * kGeoStride + f];
}

__global__ __launch_bounds__(kMapThreads) void closure_targets_kernel(ClosureDev c, const double* __restrict__ U,
                                                                      float* __restrict__ T, int64_t ldt) {
  __shared__ double sv[2 * kMaxNodes * kMapThreads];
  const int64_t gid = (int64_t)blockIdx.x * kMapThreads + threadIdx.x;
  const int64_t k = gid >> 2;
  const int f = (int)(gid & 3);
  if (k >= c.K) return;
  const int nl = c.np_lo, nh = c.np_hi;
  const double* u = U + (k * 4 + f) * nh;
  double* col = sv + threadIdx.x;                             // the row
  double* lo = sv + kMaxNodes * kMapThreads + threadIdx.x;    // P row
#pragma unroll 8
  for (int n = 0; n < nh; ++n) col[n * kMapThreads] = u[n];
  for (int m = 0; m < nl; ++m) {
    double acc = 0.0;
    for (int n = 0; n < nh; ++n) acc += c.P[m * nh + n] * col[n * kMapThreads];
    lo[m * kMapThreads] = acc;
  }
  for (int n = 0; n < nh; ++n) {
    double acc = 0.0;
    for (int m = 0; m < nl; ++m) acc += c.I[n * nl + m] * lo[m * kMapThreads];
    T[k * ldt + f * nh + n] = (float)(col[n * kMapThreads] - acc);
  }
}

__global__ __launch_bounds__(kMapThreads) void closure_restrict_kernel(ClosureDev c, const double* __restrict__ Uhi,
                                                                       double* __restrict__ Ulo) {
  __shared__ double sv[kMaxNodes * kMapThreads];
  const int64_t gid = (int64_t)blockIdx.x * kMapThreads + threadIdx.x;
  const int64_t k = gid >> 2;
  const int f = (int)(gid & 3);
  if (k >= c.K) return;
  const int nl = c.np_lo, nh = c.np_hi;
  const double* u = Uhi + (k * 4 + f) * nh;
  double* col = sv + threadIdx.x;
#pragma unroll 8
  for (int n = 0; n < nh; ++n) col[n * kMapThreads] = u[n];
  for (int m = 0; m < nl; ++m) {
    double acc = 0.0;
    for (int n = 0; n < nh; ++n) acc += c.P[m * nh + n] * col[n * kMapThreads];
    Ulo[(k * 4 + f) * nl + m] = acc;
  }
}

__global__ __launch_bounds__(kMapThreads) void closure_apply_kernel(ClosureDev c, const double* __restrict__ Ulo,
                                                                    const float* __restrict__ Y,
                                                                    const float* __restrict__ Y0, int64_t ldy,
                                                                    double* __restrict__ Uhi) {
  __shared__ double sv[kMaxNodes * kMapThreads];
  const int64_t gid = (int64_t)blockIdx.x * kMapThreads + threadIdx.x;
  const int64_t k = gid >> 2;
  const int f = (int)(gid & 3);
  if (k >= c.K) return;
  const int nl = c.np_lo, nh = c.np_hi;
  const double* u = Ulo + (k * 4 + f) * nl;
  double* col = sv + threadIdx.x;
#pragma unroll 8
  for (int m = 0; m < nl; ++m) col[m * kMapThreads] = u[m];
  for (int n = 0; n < nh; ++n) {
    double acc = 0.0;
    for (int m = 0; m < nl; ++m) acc += c.I[n * nl + m] * col[m * kMapThreads];
    const int64_t i = k * ldy + f * nh + n;
    Uhi[(k * 4 + f) * nh + n] = acc + (Y ? (double)Y[i] - (Y0 ? (double)Y0[i] : 0.0) : 0.0);
  }
}

// Drift samples of the order-lo corrector: T[k][f Np_lo + n] = U_ref - U at
// node n of field f (one thread per element and field; FP64 difference,
// rounded once to FP32).
__global__ __launch_bounds__(kMapThreads) void closure_drift_kernel(ClosureDev c, const double* __restrict__ Uref,
                                                                    const double* __restrict__ U,
                                                                    float* __restrict__ T, int64_t ldt) {
  const int64_t gid = (int64_t)blockIdx.x * kMapThreads + threadIdx.x;
  const int64_t k = gid >> 2;
  const int f = (int)(gid & 3);
  if (k >= c.K) return;
  const int nl = c.np_lo;
  const double* a = Uref + (k * 4 + f) * nl;
  const double* b = U + (k * 4 + f) * nl;
  for (int n = 0; n < nl; ++n) T[k * ldt + f * nl + n] = (float)(a[n] - b[n]);
}

// The corrector's update of an order-lo state: U += Y - Y0 (rows as above;
// Y0, the network's output for the free-stream sample, may be NULL).
__global__ __launch_bounds__(kMapThreads) void closure_correct_kernel(ClosureDev c, const float* __restrict__ Y,
                                                                      const float* __restrict__ Y0,
                                                                      int64_t ldy, double* __restrict__ U) {
  const int64_t gid = (int64_t)blockIdx.x * kMapThreads + threadIdx.x;
  const int64_t k = gid >> 2;
  const int f = (int)(gid & 3);
  if (k >= c.K) return;
  const int nl = c.np_lo;
  double* u = U + (k * 4 + f) * nl;
  for (int n = 0; n < nl; ++n) {
    const int64_t i = k * ldy + f * nl + n;
    u[n] += (double)Y[i] - (Y0 ? (double)Y0[i] : 0.0);
  }
}

// ---------------------------------------------------------------- launchers
namespace {
int lerr(std::string& err, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    err = std::string(what) + ": " + hipGetErrorString(e);
    return -3;
  }
  return 0;
}

size_t dense_lds(int N, int K) {
  return ((size_t)N * (K + 4) * 2 + 15) / 16 * 16 + kDenseWaves * sizeof(double);
}

template <int NT, int EPI, bool NORM>
int dense_go(const DenseArgs& a, int blocks, hipStream_t s, std::string& err) {
  hipLaunchKernelGGL((dense_kernel<NT, EPI, NORM>), dim3(blocks), dim3(64 * kDenseWaves), dense_lds(16 * NT, a.K), s, a);
  return lerr(err, "dense kernel launch");
}

int dense(int NT, int epi, bool norm, const DenseArgs& a, int blocks, hipStream_t s, std::string& err) {
  if (NT == 8) {
    if (epi == EPI_GELU) return norm ? dense_go<8, EPI_GELU, true>(a, blocks, s, err)
                                     : dense_go<8, EPI_GELU, false>(a, blocks, s, err);
    if (epi == EPI_DGELU) return dense_go<8, EPI_DGELU, false>(a, blocks, s, err);
  } else if (NT == 4) {
    if (epi == EPI_OUT) return dense_go<4, EPI_OUT, false>(a, blocks, s, err);
    if (epi == EPI_LOSS) return dense_go<4, EPI_LOSS, false>(a, blocks, s, err);
    if (epi == EPI_GELU) return norm ? dense_go<4, EPI_GELU, true>(a, blocks, s, err)
                                     : dense_go<4, EPI_GELU, false>(a, blocks, s, err);
    if (epi == EPI_DGELU) return dense_go<4, EPI_DGELU, false>(a, blocks, s, err);
  }
  err = "dense layer shape not built";
  return -5;
}

template <int TNW, int TK>
int wgrad_go(const WgradArgs& a, int blocks, hipStream_t s, std::string& err) {
  const size_t lds = (size_t)64 * (a.NG + 4) * 2 + (size_t)64 * (16 * TK + 4) * 2;
  hipLaunchKernelGGL((wgrad_kernel<TNW, TK>), dim3(blocks), dim3(256), lds, s, a);
  return lerr(err, "weight-gradient kernel launch");
}

int wgrad(const WgradArgs& a, int blocks, hipStream_t s, std::string& err) {
  const int tn = a.NG / 16, tk = a.KA / 16;
  const int tnw = (tn + 3) / 4;  // n-tiles per wave
  if (tnw == 1) {
    if (tk == 1) return wgrad_go<1, 1>(a, blocks, s, err);
    if (tk == 2) return wgrad_go<1, 2>(a, blocks, s, err);
    if (tk == 4) return wgrad_go<1, 4>(a, blocks, s, err);
    if (tk == 8) return wgrad_go<1, 8>(a, blocks, s, err);
  } else if (tnw == 2) {
    if (tk == 1) return wgrad_go<2, 1>(a, blocks, s, err);
    if (tk == 2) return wgrad_go<2, 2>(a, blocks, s, err);
    if (tk == 4) return wgrad_go<2, 4>(a, blocks, s, err);
    if (tk == 8) return wgrad_go<2, 8>(a, blocks, s, err);
  }
  err = "weight-gradient shape not built";
  return -5;
}

// one 16-row tile per wave (grid-stride beyond 1024 workgroups, the size of the
// loss partial buffer)
int dense_blocks(int64_t B) {
  const int64_t tiles = (B + 15) / 16;
  const int64_t b = (tiles + kDenseWaves - 1) / kDenseWaves;
  return (int)(b < 1024 ? (b > 0 ? b : 1) : 1024);
}
}  // namespace

int mlp_forward(const MlpDev& d, const float* X, int64_t ldx, int64_t B, float* Y, int64_t ldy,
                void* stream, std::string& err) {
  hipStream_t s = (hipStream_t)stream;
  const int blocks = dense_blocks(B);
  const int NTH = d.H / 16, NTO = d.out_pad / 16;
  DenseArgs a{};
  a.B = B;
  // layer 1 (normalised inputs)
  a.A = X; a.lda = ldx; a.in_mean = d.in_mean; a.in_rstd = d.in_rstd; a.Aout = d.Xn;
  a.kvalid = d.n_in; a.W = d.wb[0]; a.K = d.in_pad; a.ldw = d.ldw[0]; a.bias = d.params + d.boff[0];
  a.H = d.H1;
  int rc = dense(NTH, EPI_GELU, true, a, blocks, s, err);
  if (rc) return rc;
  // layer 2
  a = DenseArgs{}; a.B = B;
  a.A = d.H1; a.lda = d.H; a.W = d.wb[1]; a.K = d.H; a.ldw = d.ldw[1]; a.bias = d.params + d.boff[1];
  a.H = d.H2;
  rc = dense(NTH, EPI_GELU, false, a, blocks, s, err);
  if (rc) return rc;
  // layer 3 (denormalised outputs)
  a = DenseArgs{}; a.B = B;
  a.A = d.H2; a.lda = d.H; a.W = d.wb[2]; a.K = d.H; a.ldw = d.ldw[2]; a.bias = d.params + d.boff[2];
  a.nvalid = d.n_out; a.Y = Y; a.ldy = ldy; a.out_mean = d.out_mean; a.out_std = d.out_std;
  return dense(NTO, EPI_OUT, false, a, blocks, s, err);
}

namespace {
template <int KIT, int HT, int OT>
int train_go(const TrainArgs& a, int blocks, hipStream_t s, std::string& err) {
  hipLaunchKernelGGL((train_kernel<KIT, HT, OT>), dim3(blocks), dim3(256), 0, s, a);
  return lerr(err, "training kernel launch");
}

// The fused training step for the shapes it is built for (in_pad 32,
// H 128, up to 64 outputs); returns 1 (nothing launched) for others.  The
// output tiles cover n_out rounded up to 32 (two tiles at most 32 outputs,
// else four), the rows of the stored output weights beyond that unread.
int train_fused(const MlpDev& d, const float* X, int64_t ldx, const float* T, int64_t ldt,
                int64_t B, int* loss_parts, hipStream_t s, std::string& err) {
  const int KIT = d.in_pad / 16, HT = d.H / 16, OT = d.n_out <= 32 ? 2 : 4;
  if (KIT != 2 || HT != 8 || d.n_out > 64 || 16 * OT > d.out_pad) return 1;
  // workgroups: 256 (one per CU) at most, each a whole number of 64-sample
  // blocks, and no more whole-gradient partials than the buffer holds
  const int64_t cap = (int64_t)d.nparts * ((int64_t)d.H * d.H + d.H) / d.nparams;
  const int64_t maxwg = cap < 256 ? cap : 256;
  if (maxwg < 1) return 1;
  const int64_t chunk = ((B + maxwg - 1) / maxwg + 63) / 64 * 64;
  const int blocks = (int)((B + chunk - 1) / chunk);
  if (blocks > 1024) return 1;  // the loss partial buffer
  TrainArgs a{};
  a.X = X; a.ldx = ldx; a.T = T; a.ldt = ldt; a.B = B; a.chunk = chunk;
  a.n_in = d.n_in; a.n_out = d.n_out;
  a.in_mean = d.in_mean; a.in_rstd = d.in_rstd; a.out_mean = d.out_mean; a.out_std = d.out_std;
  a.W1 = d.wb[0]; a.W2 = d.wb[1]; a.W3 = d.wb[2];
  a.ldw1 = d.ldw[0]; a.ldw2 = d.ldw[1]; a.ldw3 = d.ldw[2];
  a.b1 = d.params + d.boff[0]; a.b2 = d.params + d.boff[1]; a.b3 = d.params + d.boff[2];
  a.loss_scale = (float)(2.0 / ((double)B * d.n_out));
  a.loss_part = d.loss_part;
  a.part = d.part;
  a.stride = d.nparams;
  for (int l = 0; l < 3; ++l) {
    a.woff[l] = d.woff[l];
    a.boff[l] = d.boff[l];
  }
  int rc = OT == 4 ? train_go<2, 8, 4>(a, blocks, s, err) : train_go<2, 8, 2>(a, blocks, s, err);
  if (rc) return rc;
  if (loss_parts) *loss_parts = blocks;
  hipLaunchKernelGGL(reduce_parts_kernel, dim3((unsigned)((d.nparams + 63) / 64)), dim3(256), 0, s,
                     (const float*)d.part, blocks, (int64_t)d.nparams, (int64_t)d.nparams, d.grad);
  return lerr(err, "reduce kernel launch");
}
}  // namespace

int mlp_backward(const MlpDev& d, const float* X, int64_t ldx, const float* T, int64_t ldt,
                 int64_t B, int* loss_parts, void* stream, std::string& err) {
  hipStream_t s = (hipStream_t)stream;
  if (d.fused) {
    const int rc = train_fused(d, X, ldx, T, ldt, B, loss_parts, s, err);
    if (rc != 1) return rc;
  }
  const int blocks = dense_blocks(B);
  if (loss_parts) *loss_parts = blocks;  // the loss layer writes one partial per workgroup
  const int NTH = d.H / 16, NTO = d.out_pad / 16;
  DenseArgs a{};
  a.B = B;
  a.A = X; a.lda = ldx; a.in_mean = d.in_mean; a.in_rstd = d.in_rstd; a.Aout = d.Xn;
  a.kvalid = d.n_in; a.W = d.wb[0]; a.K = d.in_pad; a.ldw = d.ldw[0]; a.bias = d.params + d.boff[0];
  a.Gd = d.G1; a.H = d.H1;
  int rc = dense(NTH, EPI_GELU, true, a, blocks, s, err);
  if (rc) return rc;
  a = DenseArgs{}; a.B = B;
  a.A = d.H1; a.lda = d.H; a.W = d.wb[1]; a.K = d.H; a.ldw = d.ldw[1]; a.bias = d.params + d.boff[1];
  a.Gd = d.G2; a.H = d.H2;
  if ((rc = dense(NTH, EPI_GELU, false, a, blocks, s, err))) return rc;
  // output layer + loss: dY = 2 (y - t) / (B n_out) in normalised units
  a = DenseArgs{}; a.B = B;
  a.A = d.H2; a.lda = d.H; a.W = d.wb[2]; a.K = d.H; a.ldw = d.ldw[2]; a.bias = d.params + d.boff[2];
  a.nvalid = d.n_out; a.T = T; a.ldt = ldt; a.out_mean = d.out_mean; a.out_std = d.out_std;
  a.loss_scale = (float)(2.0 / ((double)B * d.n_out)); a.loss_part = d.loss_part; a.H = d.dY;
  if ((rc = dense(NTO, EPI_LOSS, false, a, blocks, s, err))) return rc;
  // dZ2 = (dY W3) * gelu'(Z2): W3^T is [H][out_pad]; gelu' as stored by the forward pass
  a = DenseArgs{}; a.B = B;
  a.A = d.dY; a.lda = d.out_pad; a.W = d.wt[2]; a.K = d.out_pad; a.ldw = d.ldwt[2];
  a.Gd = d.G2; a.H = d.dZ2;
  if ((rc = dense(NTH, EPI_DGELU, false, a, blocks, s, err))) return rc;
  // dZ1 = (dZ2 W2) * gelu'(Z1)
  a = DenseArgs{}; a.B = B;
  a.A = d.dZ2; a.lda = d.H; a.W = d.wt[1]; a.K = d.H; a.ldw = d.ldwt[1];
  a.Gd = d.G1; a.H = d.dZ1;
  if ((rc = dense(NTH, EPI_DGELU, false, a, blocks, s, err))) return rc;
  // weight gradients: partials per workgroup, then a fixed-order sum
  const int64_t chunk = ((B + d.nparts - 1) / d.nparts + 63) / 64 * 64;
  const int parts = (int)((B + chunk - 1) / chunk);
  struct L { const unsigned short* G; int NG; int nv; const unsigned short* A; int KA; int kv; int64_t off; };
  const L layers[3] = {{d.dZ1, d.H, d.H, d.Xn, d.in_pad, d.n_in, d.woff[0]},
                       {d.dZ2, d.H, d.H, d.H1, d.H, d.H, d.woff[1]},
                       {d.dY, d.out_pad, d.n_out, d.H2, d.H, d.H, d.woff[2]}};
  for (int l = 0; l < 3; ++l) {
    WgradArgs w{};
    w.G = layers[l].G; w.NG = layers[l].NG; w.nvalid = layers[l].nv;
    w.A = layers[l].A; w.KA = layers[l].KA; w.kvalid = layers[l].kv;
    w.B = B; w.chunk = chunk; w.part = d.part;
    if ((rc = wgrad(w, parts, s, err))) return rc;
    const int64_t n = (int64_t)w.nvalid * w.kvalid + w.nvalid;  // W then b: contiguous
    hipLaunchKernelGGL(reduce_parts_kernel, dim3((unsigned)((n + 63) / 64)), dim3(256), 0, s,
                       (const float*)d.part, parts, n, n, d.grad + layers[l].off);
    if ((rc = lerr(err, "reduce kernel launch"))) return rc;
  }
  return 0;
}

int mlp_adam(const MlpDev& d, float lr, float beta1, float beta2, float eps, int step, void* stream,
             std::string& err) {
  const float bc1 = 1.f - powf(beta1, (float)step), bc2 = 1.f - powf(beta2, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((d.nparams + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, d, lr, beta1, beta2, eps, bc1, bc2);
  return lerr(err, "adam kernel launch");
}

int mlp_refresh_bf16(const MlpDev& d, void* stream, std::string& err) {
  hipLaunchKernelGGL(refresh_bf16_kernel, dim3((unsigned)((d.nparams + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, d);
  return lerr(err, "refresh kernel launch");
}

int column_stats(const float* A, int64_t rows, int64_t ld, int cols, double* part, int nparts,
                 void* stream, std::string& err) {
  const int64_t chunk = (rows + nparts - 1) / nparts;
  hipLaunchKernelGGL(column_stats_kernel, dim3(nparts), dim3(256), 0, (hipStream_t)stream, A, rows,
                     ld, cols, chunk > 0 ? chunk : 1, part);
  return lerr(err, "column statistics kernel launch");
}

dim3 map_grid(int64_t K) { return dim3((unsigned)((4 * K + kMapThreads - 1) / kMapThreads)); }

int closure_features(const ClosureDev& c, const double* U, int from_hi, float* X, int64_t ldx,
                     void* stream, std::string& err) {
  hipLaunchKernelGGL(closure_features_kernel, map_grid(c.K), dim3(kMapThreads), 0,
                     (hipStream_t)stream, c, U, from_hi, X, ldx);
  return lerr(err, "closure features kernel launch");
}

int closure_targets(const ClosureDev& c, const double* U, float* T, int64_t ldt, void* stream,
                    std::string& err) {
  hipLaunchKernelGGL(closure_targets_kernel, map_grid(c.K), dim3(kMapThreads), 0,
                     (hipStream_t)stream, c, U, T, ldt);
  return lerr(err, "closure targets kernel launch");
}

int closure_restrict(const ClosureDev& c, const double* Uhi, double* Ulo, void* stream,
                     std::string& err) {
  hipLaunchKernelGGL(closure_restrict_kernel, map_grid(c.K), dim3(kMapThreads), 0,
                     (hipStream_t)stream, c, Uhi, Ulo);
  return lerr(err, "closure restrict kernel launch");
}

int closure_apply(const ClosureDev& c, const double* Ulo, const float* Y, const float* Y0,
                  int64_t ldy, double* Uhi, void* stream, std::string& err) {
  hipLaunchKernelGGL(closure_apply_kernel, map_grid(c.K), dim3(kMapThreads), 0,
                     (hipStream_t)stream, c, Ulo, Y, Y0, ldy, Uhi);
  return lerr(err, "closure apply kernel launch");
}

int closure_drift(const ClosureDev& c, const double* Uref, const double* U, float* T, int64_t ldt,
                  void* stream, std::string& err) {
  hipLaunchKernelGGL(closure_drift_kernel, map_grid(c.K), dim3(kMapThreads), 0,
                     (hipStream_t)stream, c, Uref, U, T, ldt);
  return lerr(err, "closure drift kernel launch");
}

int closure_correct(const ClosureDev& c, const float* Y, const float* Y0, int64_t ldy, double* U,
                    void* stream, std::string& err) {
  hipLaunchKernelGGL(closure_correct_kernel, map_grid(c.K), dim3(kMapThreads), 0,
                     (hipStream_t)stream, c, Y, Y0, ldy, U);
  return lerr(err, "closure correct kernel launch");
}

}  // namespace dgmi
