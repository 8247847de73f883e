// Allocation-free multi-step entry point: dg_rk_steps with every buffer
// beyond the caller's inputs and outputs (the stage ping-pong state, the wall
// force's per-workgroup partials and its ticket) in a file-scope device array
// instead of memory the library allocates, for callers that cannot allocate
// (code under HIP graph capture, tight serving loops).
//
// The array exists once per device for the life of the process.  Its device
// address is looked up once per device at set-up (dg_setup, with that device
// current) and kept; host code uses only that address, never the array's name
// (which on the host is a stand-in, not a device pointer).  Every call on a
// device shares the array: calls that overlap on one device (different
// streams, threads or contexts) race on it.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "dg_ctx.h"

namespace {

// 64 MiB: the stage state of K * Np <= about 2 million nodes (every order of
// the 20k-element cylinder mesh, the 51k-element periodic mesh at p = 6)
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr size_t kScratchDoubles = kScratchBytes / sizeof(double);
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_mu;
double* g_addr[kMaxDevices] = {};

// The wall-force ticket must be zero before a force launch (the launch's last
// workgroup resets it); a one-thread fill kernel clears it, and the force
// outputs of a mesh without walls, with no memset node in a captured graph.
__global__ void fill_zero_kernel(double* __restrict__ a, int n) {
  const int i = threadIdx.x;
  if (i < n) a[i] = 0.0;
}

// Layout of the array for one call: [state K*4*Np][partials 3*blocks][ticket]
struct Carve {
  double* state;
  double* part;
  unsigned* ticket;
  size_t doubles;
};

Carve carve(double* base, size_t state_doubles, int blocks) {
  Carve c;
  c.state = base;
  c.part = base + state_doubles;
  // ticket on its own 256-byte line after the partials
  size_t t = state_doubles + 3 * (size_t)(blocks > 0 ? blocks : 1);
  t = (t + 31) / 32 * 32;
  c.ticket = (unsigned*)(base + t);
  c.doubles = t + 32;
  return c;
}

}  // namespace

namespace dgmi {

size_t noalloc_scratch_bytes() { return kScratchBytes; }

// Device address of the array on the current device (looked up on the first
// call per device, then cached).  Returns 0 or a dg_status.
int noalloc_scratch_address(double** out, std::string& err) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    err = std::string("hipGetDevice: ") + hipGetErrorString(e);
    return DG_EHIP;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    err = "device index beyond the static scratch table";
    return DG_EUNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return DG_EHIP;
    }
    g_addr[dev] = (double*)p;
  }
  *out = g_addr[dev];
  return DG_OK;
}

}  // namespace dgmi

extern "C" int dg_rk_steps_noalloc(dg_ctx* c, double* U, double* K1, int nsteps, double dt,
                                   const double v_w[2], double* force_dev, void* stream) {
  if (!c) return DG_EINVAL;
  if (!c->dev_ready) return dgmi::ctx_fail(c, DG_ESTATE, "dg_setup has not completed on this context");
  if (!c->noalloc_scratch)
    return dgmi::ctx_fail(c, DG_ESTATE, "no static scratch address for this context's device");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != c->device)
    return dgmi::ctx_fail(c, DG_EINVAL, "the context's device must be current");
  if (!U || !K1 || U == K1) return dgmi::ctx_fail(c, DG_EINVAL, "U and K1 must be distinct device arrays");
  if (nsteps < 0) return dgmi::ctx_fail(c, DG_EINVAL, "nsteps must be non-negative");
  if (!std::isfinite(dt)) return dgmi::ctx_fail(c, DG_EINVAL, "dt is not finite");
  const size_t state_doubles = (size_t)c->K * 4 * c->ref.Np;
  const Carve cv = carve(c->noalloc_scratch, state_doubles, c->force_blocks);
  if (cv.doubles > kScratchDoubles)
    return dgmi::ctx_fail(c, DG_EINVAL,
                          "state of " + std::to_string(state_doubles * sizeof(double)) +
                              " bytes exceeds the static scratch of " +
                              std::to_string(kScratchBytes) + " bytes");
  hipStream_t s = (hipStream_t)stream;
  std::string err;
  dgmi::DeviceTables t = dgmi::ctx_tables(c);
  t.force_part = cv.part;
  t.force_ticket = cv.ticket;
  const dgmi::KernelPhysics k = dgmi::ctx_phys(c, v_w);
  const bool walls = !c->mesh.wall_faces.empty();
  if (force_dev && walls) {
    // the ticket word is the low half of one double
    hipLaunchKernelGGL(fill_zero_kernel, dim3(1), dim3(64), 0, s, (double*)cv.ticket, 1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return dgmi::ctx_hip_fail(c, e, "clearing the force ticket");
  }
  double* bufs[2] = {U, cv.state};
  int cur = 0;
  for (int n = 0; n < nsteps; ++n) {
    for (int i = 0; i < 5; ++i) {
      const int rc = dgmi::launch_stage(c->N, dgmi::ctx_form(c), c->tune, t, k, bufs[(cur + i) & 1],
                                        bufs[(cur + i + 1) & 1], K1, dgmi::kRkA[i], dgmi::kRkB[i], dt,
                                        0, stream, err);
      if (rc != 0) return dgmi::ctx_fail(c, rc, err);
    }
    cur ^= 1;
    if (force_dev) {
      if (walls) {
        const int rc = dgmi::launch_force(c->N, t, k, bufs[cur], force_dev + 3 * (int64_t)n, stream, err);
        if (rc != 0) return dgmi::ctx_fail(c, rc, err);
      } else {
        hipLaunchKernelGGL(fill_zero_kernel, dim3(1), dim3(64), 0, s, force_dev + 3 * (int64_t)n, 3);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return dgmi::ctx_hip_fail(c, e, "zero force launch");
      }
    }
  }
  if (cur == 1) {
    hipError_t e = hipMemcpyAsync(U, cv.state, state_doubles * sizeof(double),
                                  hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return dgmi::ctx_hip_fail(c, e, "hipMemcpyAsync");
  }
  return DG_OK;
}
