// The context behind the opaque dg_ctx handle, and helpers shared by the
// C-ABI sources (dgmi_abi.cpp, batch.cpp, tune.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/dgmi.h"
#include "dg_internal.h"

namespace dgmi {
// Carpenter & Kennedy (1994) five-stage, fourth-order 2N-storage coefficients
// (NASA TM-109112): K1 <- A_i K1 + dt R(K0), K0 <- K0 + B_i K1 (Alg. 1).
constexpr double kRkA[5] = {0.0, -567301805773.0 / 1357537059087.0,
                            -2404267990393.0 / 2016746695238.0,
                            -3550918686646.0 / 2091501179385.0,
                            -1275806237668.0 / 842570457699.0};
constexpr double kRkB[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                            1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                            2277821191437.0 / 14882151754819.0};
}  // namespace dgmi

struct dg_ctx {
  int N = 0;
  int precision = 0;
  dgmi::StageTuning tune;
  dgmi::Physics phys;
  bool have_phys = false;
  std::vector<double> VX, VY;
  std::vector<int32_t> EToV;
  std::vector<int8_t> tag;
  double period[2] = {0.0, 0.0};
  int64_t Nv = 0, K = 0;
  bool have_mesh = false;
  dgmi::RefOps ref;
  dgmi::MeshTables mesh;
  bool host_ready = false;
  int device = -1;
  double* d_geo = nullptr;
  int32_t* d_conn = nullptr;
  double* d_ops = nullptr;
  double* d_frag = nullptr;
  double* d_oi = nullptr;         // over-integration fragments and tables
  int64_t oi_len = 0;
  dgmi::OIOps oi;
  bool overint = false;
  float* d_frag32 = nullptr;
  uint16_t* d_frag16 = nullptr;
  int32_t* d_wall = nullptr;
  double* d_wall_xy = nullptr;
  double* d_scratch = nullptr;
  double* d_force = nullptr;
  double* d_force_part = nullptr;
  unsigned* d_force_ticket = nullptr;
  double* d_cfl = nullptr;          // CFL work: 3K face maxima, 3K element maxima, result
  double* h_cfl = nullptr;          // pinned host word for the CFL result
  double* noalloc_scratch = nullptr;  // this device's static scratch array (not owned)
  // isoparametric elements given by dg_set_curved_elements, and their tables
  std::vector<int32_t> curved_elems;
  std::vector<double> curved_xy;
  int32_t* d_cslot = nullptr;
  int32_t* d_celem = nullptr;
  double* d_cnode = nullptr;
  double* d_cface = nullptr;
  double* d_cP = nullptr;
  int force_blocks = 0;
  bool dev_ready = false;
  std::string err;
};

namespace dgmi {
int ctx_fail(dg_ctx* c, int code, const std::string& msg);
int ctx_hip_fail(dg_ctx* c, hipError_t e, const char* what);
DeviceTables ctx_tables(const dg_ctx* c);
// the form launch_stage runs for this context (its precision mode, or the
// over-integrated FP64 stage)
inline int ctx_form(const dg_ctx* c) { return c->overint ? kFormOverint : c->precision; }
KernelPhysics ctx_phys(const dg_ctx* c, const double vw[2]);
// noalloc.hip: device address of the static scratch array on the current
// device (looked up once per device); its size in bytes
int noalloc_scratch_address(double** out, std::string& err);
size_t noalloc_scratch_bytes();
}  // namespace dgmi
