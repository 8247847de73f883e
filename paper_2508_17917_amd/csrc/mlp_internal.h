// Internal declarations of the learned-closure kernels (mlp.hip) and their
// C-ABI (closure.cpp).
#pragma once

#include <cstdint>
#include <string>

#include "dg_internal.h"

namespace dgmi {

constexpr int kMaxNodes = (kMaxOrder + 1) * (kMaxOrder + 2) / 2;

// Device view of one network and its training buffers.
struct MlpDev {
  int n_in, H, n_out;          // layer widths
  int in_pad, out_pad;         // padded to multiples of 16 (matrix-core k / n steps)
  int64_t nparams;             // W1 b1 W2 b2 W3 b3, W row-major [out_l][in_l]
  int64_t woff[3], boff[3];    // offsets of W_l and b_l in the parameter vector
  int wrows[3], wcols[3];
  float* params;               // FP32 master parameters
  float* grad;                 // FP32 gradient of the last backward
  float* m;                    // Adam moments
  float* v;
  unsigned short* wb[3];       // bfloat16 W_l, row-major, row stride ldw[l]
  unsigned short* wt[3];       // bfloat16 W_l^T, row stride ldwt[l]
  int ldw[3], ldwt[3];
  const float* in_mean;        // normalisation (device)
  const float* in_rstd;
  const float* out_mean;
  const float* out_std;
  // activations, [max_batch][width]
  unsigned short* Xn;          // normalised inputs, bfloat16 [B][in_pad]
  unsigned short* G1;          // GELU derivative at the pre-activations, bfloat16 [B][H]
  unsigned short* G2;
  unsigned short* H1;          // activations, bfloat16 [B][H]
  unsigned short* H2;
  unsigned short* dY;          // [B][out_pad]
  unsigned short* dZ2;         // [B][H]
  unsigned short* dZ1;
  float* part;                 // weight-gradient partials [nparts][...]
  int nparts;
  int fused;                   // training step in one fused kernel where built (else layer by layer)
  double* loss_part;           // [1024]
};

int mlp_forward(const MlpDev& d, const float* X, int64_t ldx, int64_t B, float* Y, int64_t ldy,
                void* stream, std::string& err);
int mlp_backward(const MlpDev& d, const float* X, int64_t ldx, const float* T, int64_t ldt,
                 int64_t B, int* loss_parts, void* stream, std::string& err);
int mlp_adam(const MlpDev& d, float lr, float beta1, float beta2, float eps, int step, void* stream,
             std::string& err);
int mlp_refresh_bf16(const MlpDev& d, void* stream, std::string& err);
int column_stats(const float* A, int64_t rows, int64_t ld, int cols, double* part, int nparts,
                 void* stream, std::string& err);

// Order-change maps of a closure on one mesh (device).
struct ClosureDev {
  int np_lo, np_hi;
  int64_t K;
  const double* P;     // [np_lo][np_hi]
  const double* I;     // [np_hi][np_lo]
  const double* geo;   // the mesh's geometry table (K x 16)
  double U_inf[4];
};

int closure_features(const ClosureDev& c, const double* U, int from_hi, float* X, int64_t ldx,
                     void* stream, std::string& err);
int closure_targets(const ClosureDev& c, const double* U, float* T, int64_t ldt, void* stream,
                    std::string& err);
int closure_restrict(const ClosureDev& c, const double* Uhi, double* Ulo, void* stream,
                     std::string& err);
int closure_apply(const ClosureDev& c, const double* Ulo, const float* Y, const float* Y0,
                  int64_t ldy, double* Uhi, void* stream, std::string& err);
// order-lo corrector: drift rows T = Uref - U, and U += Y - Y0
int closure_drift(const ClosureDev& c, const double* Uref, const double* U, float* T, int64_t ldt,
                  void* stream, std::string& err);
int closure_correct(const ClosureDev& c, const float* Y, const float* Y0, int64_t ldy, double* U,
                    void* stream, std::string& err);

}  // namespace dgmi
