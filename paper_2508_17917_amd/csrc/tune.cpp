// Launch-shape selection of the stage kernel: set/get, and an autotuner that
// times every shape on the context's own mesh, with a JSON-lines cache.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "dg_ctx.h"

namespace {

struct CacheEntry {
  char arch[96];
  int p, precision;
  long long K;
  int waves, grid;
  double us;
};

bool parse_line(const char* line, CacheEntry& e) {
  return std::sscanf(line,
                     "{\"arch\": \"%95[^\"]\", \"p\": %d, \"precision\": %d, \"K\": %lld, "
                     "\"waves\": %d, \"grid\": %d, \"us\": %lf}",
                     e.arch, &e.p, &e.precision, &e.K, &e.waves, &e.grid, &e.us) == 7;
}

// Closest cached entry (in K, within a factor 2) for this architecture,
// order and precision.
bool cache_lookup(const char* path, const char* arch, int p, int precision, long long K,
                  CacheEntry& best) {
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  double bestd = 0.0;
  while (std::fgets(line, sizeof line, f)) {
    CacheEntry e;
    if (!parse_line(line, e)) continue;
    if (std::strcmp(e.arch, arch) != 0 || e.p != p || e.precision != precision) continue;
    if (e.K > 2 * K || 2 * e.K < K) continue;
    const double d = e.K > K ? (double)e.K / K : (double)K / e.K;
    if (!found || d < bestd) {
      best = e;
      bestd = d;
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

bool valid_shape(int waves, int grid) {
  return (waves == 0 || waves == 2 || waves == 4) && (grid >= 0 && grid <= 3);
}

}  // namespace

extern "C" {

int dg_set_tuning(dg_ctx* c, int waves, int grid) {
  if (!c) return DG_EINVAL;
  if (!valid_shape(waves, grid)) return dgmi::ctx_fail(c, DG_EINVAL, "waves 0/2/4, grid 0..3");
  c->tune.waves = waves;
  c->tune.grid = grid;
  return DG_OK;
}

int dg_get_tuning(const dg_ctx* c, int* waves, int* grid) {
  if (!c || !waves || !grid) return DG_EINVAL;
  *waves = c->tune.waves ? c->tune.waves : (c->overint ? 2 : dgmi::default_waves(c->N, c->precision));
  *grid = c->tune.grid;
  return DG_OK;
}

int dg_autotune(dg_ctx* c, const double* U, int reps, const char* cache_path, void* stream,
                double* best_us) {
  if (!c) return DG_EINVAL;
  if (!c->dev_ready) return dgmi::ctx_fail(c, DG_ESTATE, "dg_setup has not completed");
  if (!U || reps < 1) return dgmi::ctx_fail(c, DG_EINVAL, "U is NULL or reps < 1");
  hipDeviceProp_t prop;
  hipError_t e = hipGetDeviceProperties(&prop, c->device);
  if (e != hipSuccess) return dgmi::ctx_hip_fail(c, e, "hipGetDeviceProperties");
  char arch[96];
  std::snprintf(arch, sizeof arch, "%s", prop.gcnArchName);
  for (char* q = arch; *q; ++q)
    if (*q == '"' || *q == '\\') *q = '_';
  if (cache_path) {
    CacheEntry hit;
    if (cache_lookup(cache_path, arch, c->N, dgmi::ctx_form(c), (long long)c->K, hit)) {
      c->tune.waves = hit.waves;
      c->tune.grid = hit.grid;
      if (best_us) *best_us = 0.0;
      return DG_OK;
    }
  }
  hipStream_t s = (hipStream_t)stream;
  const size_t bytes = (size_t)c->K * 4 * c->ref.Np * sizeof(double);
  double* K1 = nullptr;
  e = hipMalloc((void**)&K1, bytes);
  if (e != hipSuccess) return dgmi::ctx_hip_fail(c, e, "hipMalloc");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  int rc = DG_OK;
  double best = 1e300;
  dgmi::StageTuning pick;
  const dgmi::DeviceTables t = dgmi::ctx_tables(c);
  const double vw0[2] = {0.0, 0.0};
  const dgmi::KernelPhysics ph = dgmi::ctx_phys(c, vw0);
  std::string err;
  if (e != hipSuccess) rc = dgmi::ctx_hip_fail(c, e, "hipEventCreate");
  if (rc == DG_OK && (e = hipMemsetAsync(K1, 0, bytes, s)) != hipSuccess)
    rc = dgmi::ctx_hip_fail(c, e, "hipMemsetAsync");
  // two sweeps over the shapes, each shape's best time kept: the candidates
  // are often within a few per cent, and one sweep's clock drift or noise
  // could pick the slower one
  constexpr int kShapes = 8;
  double shape_us[kShapes];
  for (double& x : shape_us) x = 1e300;
  for (int sweep = 0; sweep < 2 && rc == DG_OK; ++sweep)
  for (int w : {2, 4})
    for (int grid = 0; grid < 4 && rc == DG_OK; ++grid) {
      dgmi::StageTuning tune;
      tune.waves = w;
      tune.grid = grid;
      // a later RK stage (A_2 != 0), as four of the five are: reads U and K1,
      // writes scratch and K1
      auto go = [&]() {
        return dgmi::launch_stage(c->N, dgmi::ctx_form(c), tune, t, ph, U, c->d_scratch, K1,
                                  dgmi::kRkA[1], dgmi::kRkB[1], 1e-7, 0, s, err);
      };
      for (int r = 0; r < 3 && rc == DG_OK; ++r)
        if (go() != 0) rc = dgmi::ctx_fail(c, DG_EHIP, err);
      if (rc != DG_OK) break;
      (void)hipEventRecord(e0, s);
      for (int r = 0; r < reps && rc == DG_OK; ++r)
        if (go() != 0) rc = dgmi::ctx_fail(c, DG_EHIP, err);
      (void)hipEventRecord(e1, s);
      e = hipEventSynchronize(e1);
      if (e != hipSuccess) {
        rc = dgmi::ctx_hip_fail(c, e, "hipEventSynchronize");
        break;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      const double us = 1e3 * ms / reps;
      double& sb = shape_us[(w == 4 ? 4 : 0) + grid];
      if (rc == DG_OK && us < sb) sb = us;
      if (rc == DG_OK && sweep == 1 && sb < best) {
        best = sb;
        pick = tune;
      }
    }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(K1);
  if (rc != DG_OK) return rc;
  c->tune = pick;
  if (best_us) *best_us = best;
  if (cache_path) {
    FILE* f = std::fopen(cache_path, "a");
    if (!f) return dgmi::ctx_fail(c, DG_EINVAL, std::string("cannot append to ") + cache_path);
    std::fprintf(f,
                 "{\"arch\": \"%s\", \"p\": %d, \"precision\": %d, \"K\": %lld, \"waves\": %d, "
                 "\"grid\": %d, \"us\": %.3f}\n",
                 arch, c->N, dgmi::ctx_form(c), (long long)c->K, pick.waves, pick.grid, best);
    std::fclose(f);
  }
  return DG_OK;
}

}  // extern "C"
