// C-ABI of the learned closure: the MLP (create, parameters, normalisation,
// forward, backward, Adam) and the order-change maps that make its samples.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "dg_ctx.h"
#include "mlp_internal.h"

struct dg_mlp {
  dgmi::MlpDev d{};
  int64_t max_batch = 0;
  int step = 0;
  std::vector<void*> allocs;
  float* norm = nullptr;  // in_mean | in_rstd | out_mean | out_std, 64 each
  std::string err;
};

struct dg_closure {
  dgmi::ClosureDev c{};
  double* dP = nullptr;
  double* dI = nullptr;
  int n_features = 0, n_targets = 0;
  std::string err;
};

namespace {

std::string g_mlp_error;

int mfail(dg_mlp* m, int code, const std::string& msg) {
  if (m)
    m->err = msg;
  else
    g_mlp_error = msg;
  return code;
}

int mhip(dg_mlp* m, hipError_t e, const char* what) {
  return mfail(m, DG_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

int cfail(dg_closure* c, int code, const std::string& msg) {
  if (c)
    c->err = msg;
  else
    g_mlp_error = msg;
  return code;
}

int round16(int x) { return (x + 15) / 16 * 16; }

template <typename T>
hipError_t dalloc(dg_mlp* m, T** p, size_t count) {
  hipError_t e = hipMalloc((void**)p, count * sizeof(T) > 0 ? count * sizeof(T) : sizeof(T));
  if (e != hipSuccess) return e;
  m->allocs.push_back(*p);
  return hipMemset(*p, 0, count * sizeof(T));
}

void mrelease(dg_mlp* m) {
  for (void* p : m->allocs) (void)hipFree(p);
  m->allocs.clear();
}

int mlp_build(dg_mlp* m, int n_in, int n_hidden, int n_out, int64_t max_batch) {
  dgmi::MlpDev& d = m->d;
  d.n_in = n_in;
  d.H = n_hidden;
  d.n_out = n_out;
  d.in_pad = round16(n_in);
  d.out_pad = 64;
  m->max_batch = max_batch;
  const int rows[3] = {n_hidden, n_hidden, n_out}, cols[3] = {n_in, n_hidden, n_hidden};
  int64_t off = 0;
  for (int l = 0; l < 3; ++l) {
    d.wrows[l] = rows[l];
    d.wcols[l] = cols[l];
    d.woff[l] = off;
    d.boff[l] = off + (int64_t)rows[l] * cols[l];
    off = d.boff[l] + rows[l];
  }
  d.nparams = off;
  d.ldw[0] = d.in_pad;
  d.ldwt[0] = n_hidden;
  d.ldw[1] = n_hidden;
  d.ldwt[1] = n_hidden;
  d.ldw[2] = n_hidden;
  d.ldwt[2] = d.out_pad;
  const int wb_rows[3] = {n_hidden, n_hidden, d.out_pad};
  const int wt_rows[3] = {d.in_pad, n_hidden, n_hidden};
  d.nparts = 512;  // weight-gradient workgroups: two per CU at most batch sizes
  d.fused = 1;
  const int64_t B = max_batch;
  const int64_t part_len = (int64_t)n_hidden * n_hidden + n_hidden;
  hipError_t e;
  if ((e = dalloc(m, &d.params, d.nparams)) != hipSuccess ||
      (e = dalloc(m, &d.grad, d.nparams)) != hipSuccess ||
      (e = dalloc(m, &d.m, d.nparams)) != hipSuccess ||
      (e = dalloc(m, &d.v, d.nparams)) != hipSuccess ||
      (e = dalloc(m, &d.wb[0], (size_t)wb_rows[0] * d.ldw[0])) != hipSuccess ||
      (e = dalloc(m, &d.wb[1], (size_t)wb_rows[1] * d.ldw[1])) != hipSuccess ||
      (e = dalloc(m, &d.wb[2], (size_t)wb_rows[2] * d.ldw[2])) != hipSuccess ||
      (e = dalloc(m, &d.wt[0], (size_t)wt_rows[0] * d.ldwt[0])) != hipSuccess ||
      (e = dalloc(m, &d.wt[1], (size_t)wt_rows[1] * d.ldwt[1])) != hipSuccess ||
      (e = dalloc(m, &d.wt[2], (size_t)wt_rows[2] * d.ldwt[2])) != hipSuccess ||
      (e = dalloc(m, &m->norm, 4 * 64)) != hipSuccess ||
      (e = dalloc(m, &d.Xn, (size_t)B * d.in_pad)) != hipSuccess ||
      (e = dalloc(m, &d.G1, (size_t)B * n_hidden)) != hipSuccess ||
      (e = dalloc(m, &d.G2, (size_t)B * n_hidden)) != hipSuccess ||
      (e = dalloc(m, &d.H1, (size_t)B * n_hidden)) != hipSuccess ||
      (e = dalloc(m, &d.H2, (size_t)B * n_hidden)) != hipSuccess ||
      (e = dalloc(m, &d.dY, (size_t)B * d.out_pad)) != hipSuccess ||
      (e = dalloc(m, &d.dZ2, (size_t)B * n_hidden)) != hipSuccess ||
      (e = dalloc(m, &d.dZ1, (size_t)B * n_hidden)) != hipSuccess ||
      (e = dalloc(m, &d.part, (size_t)d.nparts * part_len)) != hipSuccess ||
      (e = dalloc(m, &d.loss_part, 1024)) != hipSuccess)
    return e == hipErrorOutOfMemory ? mfail(m, DG_ENOMEM, "device allocation failed")
                                    : mhip(m, e, "allocating network buffers");
  d.in_mean = m->norm;
  d.in_rstd = m->norm + 64;
  d.out_mean = m->norm + 128;
  d.out_std = m->norm + 192;
  // identity normalisation until one is set
  std::vector<float> h(256, 0.f);
  for (int i = 0; i < 64; ++i) h[64 + i] = h[192 + i] = 1.f;
  e = hipMemcpy(m->norm, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice);
  return e == hipSuccess ? DG_OK : mhip(m, e, "hipMemcpy");
}

int check_batch(dg_mlp* m, const void* X, int64_t ldx, int64_t B) {
  if (!X) return mfail(m, DG_EINVAL, "input array is NULL");
  if (B < 1 || B > m->max_batch) return mfail(m, DG_EINVAL, "batch size outside 1..max_batch");
  if (ldx < m->d.n_in) return mfail(m, DG_EINVAL, "input row stride below the input width");
  return DG_OK;
}

}  // namespace

extern "C" {

int dg_mlp_create(int n_in, int n_hidden, int n_out, int64_t max_batch, dg_mlp** out) {
  g_mlp_error.clear();
  if (!out) return DG_EINVAL;
  *out = nullptr;
  if (n_in < 1 || n_in > 64 || (n_hidden != 64 && n_hidden != 128) || n_out < 1 || n_out > 64 ||
      max_batch < 1)
    return mfail(nullptr, DG_EUNSUPPORTED,
                 "widths: 1 <= n_in <= 64, n_hidden 64 or 128, 1 <= n_out <= 64");
  dg_mlp* m = new (std::nothrow) dg_mlp();
  if (!m) return DG_ENOMEM;
  int rc = mlp_build(m, n_in, n_hidden, n_out, max_batch);
  if (rc != DG_OK) {
    g_mlp_error = m->err;
    mrelease(m);
    delete m;
    return rc;
  }
  *out = m;
  return DG_OK;
}

int64_t dg_mlp_num_params(const dg_mlp* m) { return m ? m->d.nparams : 0; }

int dg_mlp_set_params(dg_mlp* m, const float* host, int64_t count) {
  if (!m) return DG_EINVAL;
  if (!host || count != m->d.nparams) return mfail(m, DG_EINVAL, "need exactly num_params floats");
  const size_t bytes = (size_t)count * sizeof(float);
  hipError_t e = hipMemcpy(m->d.params, host, bytes, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(m->d.m, 0, bytes);
  if (e == hipSuccess) e = hipMemset(m->d.v, 0, bytes);
  if (e != hipSuccess) return mhip(m, e, "setting parameters");
  m->step = 0;
  std::string err;
  if (dgmi::mlp_refresh_bf16(m->d, nullptr, err) != 0) return mfail(m, DG_EHIP, err);
  e = hipDeviceSynchronize();
  return e == hipSuccess ? DG_OK : mhip(m, e, "hipDeviceSynchronize");
}

int dg_mlp_get_params(dg_mlp* m, float* host, int64_t count) {
  if (!m) return DG_EINVAL;
  if (!host || count != m->d.nparams) return mfail(m, DG_EINVAL, "need exactly num_params floats");
  hipError_t e = hipMemcpy(host, m->d.params, (size_t)count * sizeof(float), hipMemcpyDeviceToHost);
  return e == hipSuccess ? DG_OK : mhip(m, e, "hipMemcpy");
}

int dg_mlp_get_grad(dg_mlp* m, float* host, int64_t count) {
  if (!m) return DG_EINVAL;
  if (!host || count != m->d.nparams) return mfail(m, DG_EINVAL, "need exactly num_params floats");
  hipError_t e = hipMemcpy(host, m->d.grad, (size_t)count * sizeof(float), hipMemcpyDeviceToHost);
  return e == hipSuccess ? DG_OK : mhip(m, e, "hipMemcpy");
}

int dg_mlp_set_normalization(dg_mlp* m, const float* in_mean, const float* in_std,
                             const float* out_mean, const float* out_std) {
  if (!m) return DG_EINVAL;
  if (!in_mean || !in_std || !out_mean || !out_std) return mfail(m, DG_EINVAL, "NULL argument");
  std::vector<float> h(256, 0.f);
  for (int i = 0; i < 64; ++i) h[64 + i] = h[192 + i] = 1.f;
  for (int i = 0; i < m->d.n_in; ++i) {
    if (!(in_std[i] > 0.f) || !std::isfinite(in_mean[i]))
      return mfail(m, DG_EINVAL, "input standard deviations must be positive");
    h[i] = in_mean[i];
    h[64 + i] = 1.f / in_std[i];
  }
  for (int i = 0; i < m->d.n_out; ++i) {
    if (!(out_std[i] > 0.f) || !std::isfinite(out_mean[i]))
      return mfail(m, DG_EINVAL, "output standard deviations must be positive");
    h[128 + i] = out_mean[i];
    h[192 + i] = out_std[i];
  }
  hipError_t e = hipMemcpy(m->norm, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice);
  return e == hipSuccess ? DG_OK : mhip(m, e, "hipMemcpy");
}

int dg_mlp_forward(dg_mlp* m, const float* X, int64_t ldx, int64_t B, float* Y, int64_t ldy,
                   void* stream) {
  if (!m) return DG_EINVAL;
  int rc = check_batch(m, X, ldx, B);
  if (rc != DG_OK) return rc;
  if (!Y || ldy < m->d.n_out) return mfail(m, DG_EINVAL, "output array NULL or stride too small");
  std::string err;
  rc = dgmi::mlp_forward(m->d, X, ldx, B, Y, ldy, stream, err);
  return rc == 0 ? DG_OK : mfail(m, rc, err);
}

int dg_mlp_backward(dg_mlp* m, const float* X, int64_t ldx, const float* T, int64_t ldt, int64_t B,
                    double* loss, void* stream) {
  if (!m) return DG_EINVAL;
  int rc = check_batch(m, X, ldx, B);
  if (rc != DG_OK) return rc;
  if (!T || ldt < m->d.n_out) return mfail(m, DG_EINVAL, "target array NULL or stride too small");
  std::string err;
  int blocks = 0;
  rc = dgmi::mlp_backward(m->d, X, ldx, T, ldt, B, &blocks, stream, err);
  if (rc != 0) return mfail(m, rc, err);
  if (loss) {
    std::vector<double> h(blocks);
    hipError_t e = hipMemcpyAsync(h.data(), m->d.loss_part, blocks * sizeof(double),
                                  hipMemcpyDeviceToHost, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return mhip(m, e, "loss read-back");
    double s = 0.0;
    for (double x : h) s += x;
    *loss = s / ((double)B * m->d.n_out);
  }
  return DG_OK;
}

int dg_mlp_set_schedule(dg_mlp* m, int fused) {
  if (!m) return DG_EINVAL;
  if (fused != 0 && fused != 1) return mfail(m, DG_EINVAL, "schedule must be 0 (layer by layer) or 1 (fused)");
  m->d.fused = fused;
  return DG_OK;
}

int dg_mlp_adam(dg_mlp* m, float lr, float beta1, float beta2, float eps, void* stream) {
  if (!m) return DG_EINVAL;
  if (!(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) ||
      !(eps > 0.f))
    return mfail(m, DG_EINVAL, "Adam hyper-parameters out of range");
  m->step += 1;
  std::string err;
  int rc = dgmi::mlp_adam(m->d, lr, beta1, beta2, eps, m->step, stream, err);
  return rc == 0 ? DG_OK : mfail(m, rc, err);
}

int dg_column_stats(const float* A, int64_t rows, int64_t ld, int cols, double* mean, double* stdev,
                    void* stream) {
  if (!A || !mean || !stdev || rows < 1 || cols < 1 || cols > 64 || ld < cols) return DG_EINVAL;
  const int nparts = 256;
  double* part = nullptr;
  if (hipMalloc((void**)&part, (size_t)nparts * 64 * 2 * sizeof(double)) != hipSuccess)
    return DG_ENOMEM;
  std::string err;
  int rc = dgmi::column_stats(A, rows, ld, cols, part, nparts, stream, err);
  std::vector<double> h((size_t)nparts * 64 * 2);
  hipError_t e = hipSuccess;
  if (rc == 0) {
    e = hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                       (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  }
  (void)hipFree(part);
  if (rc != 0 || e != hipSuccess) return DG_EHIP;
  for (int c = 0; c < cols; ++c) {
    double s1 = 0.0, s2 = 0.0;
    for (int p = 0; p < nparts; ++p) {
      s1 += h[((size_t)p * 64 + c) * 2];
      s2 += h[((size_t)p * 64 + c) * 2 + 1];
    }
    const double mu = s1 / rows;
    const double var = s2 / rows - mu * mu;
    mean[c] = mu;
    stdev[c] = std::sqrt(var > 0.0 ? var : 0.0);
  }
  return DG_OK;
}

const char* dg_mlp_last_error(const dg_mlp* m) { return m ? m->err.c_str() : g_mlp_error.c_str(); }

void dg_mlp_destroy(dg_mlp* m) {
  if (!m) return;
  mrelease(m);
  delete m;
}

int dg_closure_create(const dg_ctx* lo, const dg_ctx* hi, dg_closure** out) {
  g_mlp_error.clear();
  if (!out) return DG_EINVAL;
  *out = nullptr;
  if (!lo || !hi || !lo->dev_ready || !hi->dev_ready)
    return cfail(nullptr, DG_ESTATE, "both contexts must be set up (dg_setup)");
  if (lo->N >= hi->N) return cfail(nullptr, DG_EINVAL, "the first context must have the lower order");
  // same mesh: equal element count, metrics, normals and face scales (the
  // penalty's geometric factor, the fourth entry of each face, depends on the
  // order)
  bool same = lo->K == hi->K && lo->mesh.geo.size() == hi->mesh.geo.size();
  for (size_t i = 0; same && i < hi->mesh.geo.size(); ++i)
    if ((i % dgmi::kGeoStride) < 4 || (i % dgmi::kGeoStride) % 4 != 3)
      same = lo->mesh.geo[i] == hi->mesh.geo[i];
  if (!same) return cfail(nullptr, DG_EINVAL, "the two contexts must hold the same mesh");
  std::vector<double> P, I;
  std::string err;
  if (!dgmi::build_order_maps(lo->N, hi->N, P, I, err)) return cfail(nullptr, DG_EUNSUPPORTED, err);
  dg_closure* c = new (std::nothrow) dg_closure();
  if (!c) return DG_ENOMEM;
  hipError_t e;
  if ((e = hipMalloc((void**)&c->dP, P.size() * sizeof(double))) != hipSuccess ||
      (e = hipMalloc((void**)&c->dI, I.size() * sizeof(double))) != hipSuccess ||
      (e = hipMemcpy(c->dP, P.data(), P.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(c->dI, I.data(), I.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess) {
    if (c->dP) (void)hipFree(c->dP);
    if (c->dI) (void)hipFree(c->dI);
    delete c;
    return cfail(nullptr, DG_EHIP, std::string("uploading order maps: ") + hipGetErrorString(e));
  }
  c->c.np_lo = lo->ref.Np;
  c->c.np_hi = hi->ref.Np;
  c->c.K = hi->K;
  c->c.P = c->dP;
  c->c.I = c->dI;
  c->c.geo = dgmi::ctx_tables(hi).geo;
  for (int i = 0; i < 4; ++i) c->c.U_inf[i] = hi->phys.U_inf[i];
  c->n_features = 4 * lo->ref.Np + 4;
  c->n_targets = 4 * hi->ref.Np;
  *out = c;
  return DG_OK;
}

int dg_closure_sizes(const dg_closure* c, int* n_features, int* n_targets) {
  if (!c || !n_features || !n_targets) return DG_EINVAL;
  *n_features = c->n_features;
  *n_targets = c->n_targets;
  return DG_OK;
}

int dg_closure_features(dg_closure* c, const double* U, int from_hi, float* X, int64_t ldx,
                        void* stream) {
  if (!c) return DG_EINVAL;
  if (from_hi < 0 || from_hi > 2) return cfail(c, DG_EINVAL, "from_hi must be 0, 1 or 2");
  if ((!U && from_hi != 2) || !X || ldx < c->n_features)
    return cfail(c, DG_EINVAL, "NULL array or stride too small");
  std::string err;
  int rc = dgmi::closure_features(c->c, U, from_hi, X, ldx, stream, err);
  return rc == 0 ? DG_OK : cfail(c, rc, err);
}

int dg_closure_targets(dg_closure* c, const double* U_hi, float* T, int64_t ldt, void* stream) {
  if (!c) return DG_EINVAL;
  if (!U_hi || !T || ldt < c->n_targets) return cfail(c, DG_EINVAL, "NULL array or stride too small");
  std::string err;
  int rc = dgmi::closure_targets(c->c, U_hi, T, ldt, stream, err);
  return rc == 0 ? DG_OK : cfail(c, rc, err);
}

int dg_closure_restrict(dg_closure* c, const double* U_hi, double* U_lo, void* stream) {
  if (!c) return DG_EINVAL;
  if (!U_hi || !U_lo) return cfail(c, DG_EINVAL, "NULL array");
  std::string err;
  int rc = dgmi::closure_restrict(c->c, U_hi, U_lo, stream, err);
  return rc == 0 ? DG_OK : cfail(c, rc, err);
}

int dg_closure_apply(dg_closure* c, const double* U_lo, const float* Y, const float* Y0,
                     int64_t ldy, double* U_hi, void* stream) {
  if (!c) return DG_EINVAL;
  if (!U_lo || !U_hi || (Y && ldy < c->n_targets) || (Y0 && !Y))
    return cfail(c, DG_EINVAL, "NULL array or stride too small");
  std::string err;
  int rc = dgmi::closure_apply(c->c, U_lo, Y, Y0, ldy, U_hi, stream, err);
  return rc == 0 ? DG_OK : cfail(c, rc, err);
}

int dg_closure_drift_targets(dg_closure* c, const double* U_ref, const double* U_lo, float* T,
                             int64_t ldt, void* stream) {
  if (!c) return DG_EINVAL;
  const int n = c->n_features - 4;
  if (!U_ref || !U_lo || !T || ldt < n) return cfail(c, DG_EINVAL, "NULL array or stride too small");
  std::string err;
  int rc = dgmi::closure_drift(c->c, U_ref, U_lo, T, ldt, stream, err);
  return rc == 0 ? DG_OK : cfail(c, rc, err);
}

int dg_closure_correct(dg_closure* c, const float* Y, const float* Y0, int64_t ldy, double* U_lo,
                       void* stream) {
  if (!c) return DG_EINVAL;
  const int n = c->n_features - 4;
  if (!Y || !U_lo || ldy < n) return cfail(c, DG_EINVAL, "NULL array or stride too small");
  std::string err;
  int rc = dgmi::closure_correct(c->c, Y, Y0, ldy, U_lo, stream, err);
  return rc == 0 ? DG_OK : cfail(c, rc, err);
}

const char* dg_closure_last_error(const dg_closure* c) {
  return c ? c->err.c_str() : g_mlp_error.c_str();
}

void dg_closure_destroy(dg_closure* c) {
  if (!c) return;
  if (c->dP) (void)hipFree(c->dP);
  if (c->dI) (void)hipFree(c->dI);
  delete c;
}

}  // extern "C"
