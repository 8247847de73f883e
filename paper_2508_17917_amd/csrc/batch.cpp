// Batches of contexts advanced together: one stage launch for all instances,
// the five stages of a step replayed from a captured HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "dg_ctx.h"

struct dg_batch {
  int n = 0;
  int form = 0;
  int device = -1;
  std::vector<dg_ctx*> ctx;
  std::vector<int> item_of;           // instance -> item (items sorted by order)
  std::vector<double*> A, B, K1;      // per instance
  std::vector<dgmi::BatchGroup> groups;
  dgmi::BatchItem* d_items = nullptr;
  dgmi::BatchStep* d_steps = nullptr;
  int* d_parity = nullptr;
  dgmi::BatchStep* h_steps = nullptr; // pinned staging
  int* h_parity = nullptr;
  double* d_force = nullptr;
  double* h_force = nullptr;
  dgmi::ForceItem* d_fitems = nullptr;  // wall-force launch descriptors
  dgmi::ForceItem* h_fitems = nullptr;  // pinned staging
  dgmi::BatchItem* h_items = nullptr;   // pinned staging of the item table
  bool caller_items = false;            // d_items point at caller-owned states
  std::vector<int> inst_of;             // item -> instance
  hipEvent_t upload_ev = nullptr;
  bool upload_pending = false;
  int mode = 0, waves = 0, grid = 0, use_graph = 1;
  // launch plan for the current shape
  std::vector<dgmi::BatchGroups> launches;
  std::vector<int> launch_blocks;
  int plan_waves = 2;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int parity = 0;
  std::string err;
};

namespace {

std::string g_batch_error;  // message of the last failed dg_batch_create

int bfail(dg_batch* b, int code, const std::string& msg) {
  if (b) b->err = msg;
  return code;
}

int bhip(dg_batch* b, hipError_t e, const char* what) {
  return bfail(b, DG_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

int np_of(int p) { return (p + 1) * (p + 2) / 2; }

void drop_graph(dg_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

void release(dg_batch* b) {
  drop_graph(b);
  if (b->upload_ev) (void)hipEventSynchronize(b->upload_ev);
  for (auto* v : {&b->A, &b->B, &b->K1})
    for (double* p : *v)
      if (p) (void)hipFree(p);
  void* dev[] = {b->d_items, b->d_steps, b->d_parity, b->d_force, b->d_fitems};
  for (void* p : dev)
    if (p) (void)hipFree(p);
  if (b->h_steps) (void)hipHostFree(b->h_steps);
  if (b->h_parity) (void)hipHostFree(b->h_parity);
  if (b->h_items) (void)hipHostFree(b->h_items);
  if (b->h_force) (void)hipHostFree(b->h_force);
  if (b->h_fitems) (void)hipHostFree(b->h_fitems);
  if (b->upload_ev) (void)hipEventDestroy(b->upload_ev);
  if (b->cap) (void)hipStreamDestroy(b->cap);
}

// Work of one tile of order p relative to the others (operator products and
// face work both grow like Np (Np + 3 Nfp)); used to share the resident
// workgroups of a single launch among the order groups.
double tile_cost(int p) {
  return (double)dgmi::elements_per_tile(p) * np_of(p) * (np_of(p) + 3 * (p + 1));
}

// Workgroups for each group and the launches of one stage, for the current
// shape.  Group block counts are multiples of 8 (one tile range per XCD).
int plan(dg_batch* b) {
  const int W = b->waves ? b->waves : 4;
  if (W != 2 && W != 4) return bfail(b, DG_EINVAL, "waves per workgroup must be 2 or 4");
  b->plan_waves = W;
  const int resident = dgmi::batch_resident_blocks(b->form, W);
  const int ng = (int)b->groups.size();
  std::vector<int64_t> need(ng), nb(ng);
  double total = 0.0;
  for (int g = 0; g < ng; ++g) {
    need[g] = ((b->groups[g].ntiles + W - 1) / W + 7) / 8 * 8;
    total += b->groups[g].ntiles * tile_cost(b->groups[g].p);
  }
  for (int g = 0; g < ng; ++g) {
    int64_t blocks;
    if (b->grid == 1) {
      blocks = need[g];
    } else if (b->mode == 1) {
      const int res = dgmi::batch_order_resident_blocks(b->groups[g].p, b->form, W);
      blocks = std::min<int64_t>(need[g], res / 8 * 8);
    } else {
      const double share = b->groups[g].ntiles * tile_cost(b->groups[g].p) / total;
      blocks = std::min<int64_t>(need[g], (int64_t)(share * resident) / 8 * 8);
    }
    nb[g] = std::max<int64_t>(8, blocks);
  }
  b->launches.clear();
  b->launch_blocks.clear();
  if (b->mode == 0) {
    dgmi::BatchGroups G{};
    G.ng = ng;
    int64_t off = 0;
    for (int g = 0; g < ng; ++g) {
      G.g[g] = b->groups[g];
      G.g[g].block_begin = (int)off;
      G.g[g].nblocks = (int)nb[g];
      off += nb[g];
    }
    if (off > 0x7fffffff) return bfail(b, DG_EINVAL, "batch too large for one launch");
    b->launches.push_back(G);
    b->launch_blocks.push_back((int)off);
  } else {
    for (int g = 0; g < ng; ++g) {
      dgmi::BatchGroups G{};
      G.ng = 1;
      G.g[0] = b->groups[g];
      G.g[0].block_begin = 0;
      G.g[0].nblocks = (int)nb[g];
      b->launches.push_back(G);
      b->launch_blocks.push_back((int)nb[g]);
    }
  }
  return DG_OK;
}

int launch_stage_i(dg_batch* b, int stage, hipStream_t s) {
  std::string err;
  for (size_t l = 0; l < b->launches.size(); ++l) {
    // one launch for all groups, or one per group in a kernel sized for its order
    const dgmi::BatchGroups& G = b->launches[l];
    int rc = b->mode == 0
                 ? dgmi::launch_batch_stage(b->form, b->plan_waves, b->d_items, b->d_steps,
                                            b->d_parity, G, b->launch_blocks[l], stage,
                                            dgmi::kRkA[stage], dgmi::kRkB[stage], s, err)
                 : dgmi::launch_batch_order_stage(G.g[0].p, b->form, b->plan_waves, b->d_items,
                                                  b->d_steps, b->d_parity, G.g[0],
                                                  b->launch_blocks[l], stage, dgmi::kRkA[stage],
                                                  dgmi::kRkB[stage], s, err);
    if (rc != 0) return bfail(b, rc, err);
  }
  return DG_OK;
}

int launch_step(dg_batch* b, hipStream_t s) {
  for (int i = 0; i < 5; ++i) {
    int rc = launch_stage_i(b, i, s);
    if (rc != DG_OK) return rc;
  }
  return DG_OK;
}

int capture(dg_batch* b) {
  drop_graph(b);
  hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return bhip(b, e, "hipStreamBeginCapture");
  int rc = launch_step(b, b->cap);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(b->cap, &g);
  if (rc != DG_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return bhip(b, e, "hipStreamEndCapture");
  b->graph = g;
  e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    drop_graph(b);
    return bhip(b, e, "hipGraphInstantiate");
  }
  return DG_OK;
}

// Stage the per-instance parameters and the parity, and copy them to the
// device on `s` (the previous upload is waited for before the pinned area is
// rewritten).
// With Uc / K1c (caller-owned states), the item table is rewritten to point
// at them (state buffer 0 and K1; buffer 1 the batch's second buffer) and the
// stages start from buffer 0; without, it points back at the batch's own
// buffers if a caller-state step changed it.
int upload(dg_batch* b, const double* dt, const double* vw, hipStream_t s,
           double* const* Uc = nullptr, double* const* K1c = nullptr) {
  if (b->upload_pending) {
    hipError_t e = hipEventSynchronize(b->upload_ev);
    if (e != hipSuccess) return bhip(b, e, "hipEventSynchronize");
    b->upload_pending = false;
  }
  const bool want_caller = Uc != nullptr;
  if (want_caller || b->caller_items) {
    for (int i = 0; i < b->n; ++i) {
      dgmi::BatchItem& it = b->h_items[b->item_of[i]];
      it.buf[0] = want_caller ? Uc[i] : b->A[i];
      it.buf[1] = b->B[i];
      it.K1 = want_caller ? K1c[i] : b->K1[i];
    }
    hipError_t e = hipMemcpyAsync(b->d_items, b->h_items, b->n * sizeof(dgmi::BatchItem),
                                  hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return bhip(b, e, "item upload");
    b->caller_items = want_caller;
  }
  for (int i = 0; i < b->n; ++i) {
    dgmi::BatchStep& st = b->h_steps[b->item_of[i]];
    st.dt = dt ? dt[i] : 0.0;
    st.vw[0] = vw ? vw[2 * i] : 0.0;
    st.vw[1] = vw ? vw[2 * i + 1] : 0.0;
    st.pad = 0.0;
  }
  *b->h_parity = want_caller ? 0 : b->parity;
  hipError_t e = hipMemcpyAsync(b->d_steps, b->h_steps, b->n * sizeof(dgmi::BatchStep),
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_parity, b->h_parity, sizeof(int), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipEventRecord(b->upload_ev, s);
  if (e != hipSuccess) return bhip(b, e, "parameter upload");
  b->upload_pending = true;
  return DG_OK;
}

int check_instance(dg_batch* b, int i) {
  if (!b) return DG_EINVAL;
  if (i < 0 || i >= b->n) return bfail(b, DG_EINVAL, "instance index out of range");
  return DG_OK;
}

size_t state_bytes(const dg_ctx* c) { return (size_t)c->K * 4 * c->ref.Np * sizeof(double); }

}  // namespace

extern "C" {

static int batch_build(dg_batch* b, dg_ctx* const* ctxs, int n);

int dg_batch_create(dg_ctx* const* ctxs, int n, dg_batch** out) {
  g_batch_error.clear();
  if (!out) return DG_EINVAL;
  *out = nullptr;
  if (!ctxs || n < 1) {
    g_batch_error = "need at least one context";
    return DG_EINVAL;
  }
  dg_batch* b = new (std::nothrow) dg_batch();
  if (!b) return DG_ENOMEM;
  int rc = batch_build(b, ctxs, n);
  if (rc != DG_OK) {
    g_batch_error = b->err;
    release(b);
    delete b;
    return rc;
  }
  *out = b;
  return DG_OK;
}

static int batch_build(dg_batch* b, dg_ctx* const* ctxs, int n) {
  b->n = n;
  b->ctx.assign(ctxs, ctxs + n);
  // an instance's wall force is reduced through its context's partials and
  // ticket: two instances on one context would race on them
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j)
      if (ctxs[i] && ctxs[i] == ctxs[j])
        return bfail(b, DG_EINVAL, "a context appears twice in the batch");
  for (int i = 0; i < n; ++i) {
    dg_ctx* c = ctxs[i];
    if (!c || !c->dev_ready) return bfail(b, DG_ESTATE, "every context must be set up (dg_setup)");
    if (c->precision != ctxs[0]->precision)
      return bfail(b, DG_EINVAL, "contexts of a batch must share the precision mode");
    if (c->overint)
      return bfail(b, DG_EUNSUPPORTED, "over-integrated contexts are not batched");
    if (!c->mesh.celem.empty())
      return bfail(b, DG_EUNSUPPORTED, "contexts with curved elements are not batched");
  }
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return bhip(b, e, "hipGetDevice");
  b->device = dev;
  for (int i = 0; i < n; ++i)
    if (ctxs[i]->device != dev) return bfail(b, DG_EINVAL, "contexts must live on the current device");
  b->form = ctxs[0]->precision;
  // items sorted by order (stable), grouped
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return ctxs[x]->N < ctxs[y]->N; });
  b->item_of.assign(n, 0);
  b->inst_of = idx;
  std::vector<dgmi::BatchItem> items(n);
  b->A.assign(n, nullptr);
  b->B.assign(n, nullptr);
  b->K1.assign(n, nullptr);
  for (int j = 0; j < n; ++j) {
    const int i = idx[j];
    dg_ctx* c = ctxs[i];
    b->item_of[i] = j;
    const size_t bytes = state_bytes(c);
    if ((e = hipMalloc((void**)&b->A[i], bytes)) != hipSuccess ||
        (e = hipMalloc((void**)&b->B[i], bytes)) != hipSuccess ||
        (e = hipMalloc((void**)&b->K1[i], bytes)) != hipSuccess ||
        (e = hipMemset(b->A[i], 0, bytes)) != hipSuccess ||
        (e = hipMemset(b->B[i], 0, bytes)) != hipSuccess ||
        (e = hipMemset(b->K1[i], 0, bytes)) != hipSuccess)
      return e == hipErrorOutOfMemory ? bfail(b, DG_ENOMEM, "device allocation failed")
                                      : bhip(b, e, "allocating batch states");
    dgmi::BatchItem& it = items[j];
    it.t = dgmi::ctx_tables(c);
    it.ph = dgmi::ctx_phys(c, nullptr);
    it.buf[0] = b->A[i];
    it.buf[1] = b->B[i];
    it.K1 = b->K1[i];
    const int ept = dgmi::elements_per_tile(c->N);
    const int64_t ntiles = (c->K + ept - 1) / ept;
    if (b->groups.empty() || b->groups.back().p != c->N) {
      dgmi::BatchGroup g{};
      g.p = c->N;
      g.first_item = j;
      g.n_items = 0;
      g.ntiles = 0;
      b->groups.push_back(g);
    }
    dgmi::BatchGroup& g = b->groups.back();
    it.tile_begin = g.ntiles;
    it.tile_end = g.ntiles + ntiles;
    g.ntiles += ntiles;
    g.n_items += 1;
  }
  if ((int)b->groups.size() > dgmi::kMaxOrder) return bfail(b, DG_EINVAL, "too many order groups");
  if ((e = hipMalloc((void**)&b->d_items, n * sizeof(dgmi::BatchItem))) != hipSuccess ||
      (e = hipMemcpy(b->d_items, items.data(), n * sizeof(dgmi::BatchItem),
                     hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMalloc((void**)&b->d_steps, n * sizeof(dgmi::BatchStep))) != hipSuccess ||
      (e = hipMemset(b->d_steps, 0, n * sizeof(dgmi::BatchStep))) != hipSuccess ||
      (e = hipMalloc((void**)&b->d_parity, sizeof(int))) != hipSuccess ||
      (e = hipMemset(b->d_parity, 0, sizeof(int))) != hipSuccess ||
      (e = hipMalloc((void**)&b->d_force, 4 * n * sizeof(double))) != hipSuccess ||
      (e = hipHostMalloc((void**)&b->h_steps, n * sizeof(dgmi::BatchStep))) != hipSuccess ||
      (e = hipHostMalloc((void**)&b->h_parity, sizeof(int))) != hipSuccess ||
      (e = hipHostMalloc((void**)&b->h_force, 4 * n * sizeof(double))) != hipSuccess ||
      (e = hipMalloc((void**)&b->d_fitems, n * sizeof(dgmi::ForceItem))) != hipSuccess ||
      (e = hipHostMalloc((void**)&b->h_fitems, n * sizeof(dgmi::ForceItem))) != hipSuccess ||
      (e = hipHostMalloc((void**)&b->h_items, n * sizeof(dgmi::BatchItem))) != hipSuccess ||
      (e = hipEventCreateWithFlags(&b->upload_ev, hipEventDisableTiming)) != hipSuccess ||
      (e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking)) != hipSuccess)
    return bhip(b, e, "allocating batch tables");
  std::copy(items.begin(), items.end(), b->h_items);
  return plan(b);
}

int dg_batch_set_state(dg_batch* b, int i, const double* U, void* stream) {
  int rc = check_instance(b, i);
  if (rc != DG_OK) return rc;
  if (!U) return bfail(b, DG_EINVAL, "U is NULL");
  double* dst = b->parity ? b->B[i] : b->A[i];
  hipError_t e = hipMemcpyAsync(dst, U, state_bytes(b->ctx[i]), hipMemcpyDeviceToDevice,
                                (hipStream_t)stream);
  return e == hipSuccess ? DG_OK : bhip(b, e, "hipMemcpyAsync");
}

int dg_batch_get_state(dg_batch* b, int i, double* U, void* stream) {
  int rc = check_instance(b, i);
  if (rc != DG_OK) return rc;
  if (!U) return bfail(b, DG_EINVAL, "U is NULL");
  const double* src = b->parity ? b->B[i] : b->A[i];
  hipError_t e = hipMemcpyAsync(U, src, state_bytes(b->ctx[i]), hipMemcpyDeviceToDevice,
                                (hipStream_t)stream);
  return e == hipSuccess ? DG_OK : bhip(b, e, "hipMemcpyAsync");
}

int dg_batch_rk_step(dg_batch* b, const double* dt, const double* v_w, void* stream) {
  if (!b) return DG_EINVAL;
  if (!dt || !v_w) return bfail(b, DG_EINVAL, "dt and v_w are required");
  for (int i = 0; i < b->n; ++i)
    if (!std::isfinite(dt[i]) || !std::isfinite(v_w[2 * i]) || !std::isfinite(v_w[2 * i + 1]))
      return bfail(b, DG_EINVAL, "dt or v_w not finite");
  hipStream_t s = (hipStream_t)stream;
  int rc = upload(b, dt, v_w, s);
  if (rc != DG_OK) return rc;
  if (b->use_graph) {
    if (!b->exec) {
      rc = capture(b);
      if (rc != DG_OK) return rc;
    }
    hipError_t e = hipGraphLaunch(b->exec, s);
    if (e != hipSuccess) return bhip(b, e, "hipGraphLaunch");
  } else {
    rc = launch_step(b, s);
    if (rc != DG_OK) return rc;
  }
  b->parity ^= 1;  // five stages: the state now sits in the other buffer
  return DG_OK;
}

int dg_batch_rk_step_states(dg_batch* b, double* const* U, double* const* K1, const double* dt,
                            const double* v_w, void* stream) {
  if (!b) return DG_EINVAL;
  if (!U || !K1 || !dt || !v_w) return bfail(b, DG_EINVAL, "U, K1, dt and v_w are required");
  for (int i = 0; i < b->n; ++i) {
    if (!U[i] || !K1[i] || U[i] == K1[i])
      return bfail(b, DG_EINVAL, "each instance needs distinct U and K1 device arrays");
    if (!std::isfinite(dt[i]) || !std::isfinite(v_w[2 * i]) || !std::isfinite(v_w[2 * i + 1]))
      return bfail(b, DG_EINVAL, "dt or v_w not finite");
    for (int j = 0; j < i; ++j)
      if (U[j] == U[i] || K1[j] == K1[i] || U[j] == K1[i] || K1[j] == U[i])
        return bfail(b, DG_EINVAL, "two instances share a state or K1 array");
  }
  hipStream_t s = (hipStream_t)stream;
  int rc = upload(b, dt, v_w, s, U, K1);
  if (rc != DG_OK) return rc;
  if (b->use_graph) {
    if (!b->exec) {
      rc = capture(b);
      if (rc != DG_OK) return rc;
    }
    hipError_t e = hipGraphLaunch(b->exec, s);
    if (e != hipSuccess) return bhip(b, e, "hipGraphLaunch");
  } else {
    rc = launch_step(b, s);
    if (rc != DG_OK) return rc;
  }
  // five stages from buffer 0 end in buffer 1: copy each state back
  for (int i = 0; i < b->n; ++i) {
    hipError_t e = hipMemcpyAsync(U[i], b->B[i], state_bytes(b->ctx[i]), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return bhip(b, e, "hipMemcpyAsync");
  }
  return DG_OK;
}

int dg_batch_force(dg_batch* b, const double* v_w, double* out, void* stream) {
  if (!b) return DG_EINVAL;
  if (!out) return bfail(b, DG_EINVAL, "out is NULL");
  hipStream_t s = (hipStream_t)stream;
  std::string err;
  // one launch per order group over the instances that have wall faces; the
  // others report zero
  struct Launch { int N, first, count, blocks; };
  std::vector<Launch> launches;
  int pos = 0;
  for (const dgmi::BatchGroup& g : b->groups) {
    const int first = pos;
    int blocks = 0;
    for (int j = g.first_item; j < g.first_item + g.n_items; ++j) {
      const int i = b->inst_of[j];
      dg_ctx* c = b->ctx[i];
      if (c->mesh.wall_faces.empty()) {
        hipError_t e = hipMemsetAsync(b->d_force + 4 * i, 0, 3 * sizeof(double), s);
        if (e != hipSuccess) return bhip(b, e, "hipMemsetAsync");
        continue;
      }
      const double vw[2] = {v_w ? v_w[2 * i] : 0.0, v_w ? v_w[2 * i + 1] : 0.0};
      dgmi::ForceItem& f = b->h_fitems[pos++];
      f.t = dgmi::ctx_tables(c);
      f.ph = dgmi::ctx_phys(c, vw);
      f.U = b->parity ? b->B[i] : b->A[i];
      f.out = b->d_force + 4 * i;
      f.block_begin = blocks;
      f.nblocks = c->force_blocks;
      blocks += c->force_blocks;
    }
    if (pos > first) launches.push_back({g.p, first, pos - first, blocks});
  }
  if (pos > 0) {
    // the staging is free again: the previous call ended with a synchronisation
    hipError_t e = hipMemcpyAsync(b->d_fitems, b->h_fitems, pos * sizeof(dgmi::ForceItem),
                                  hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return bhip(b, e, "uploading force descriptors");
  }
  for (const Launch& l : launches) {
    int rc = dgmi::launch_batch_force(l.N, b->d_fitems + l.first, l.count, l.blocks, s, err);
    if (rc != 0) return bfail(b, rc, err);
  }
  hipError_t e = hipMemcpyAsync(b->h_force, b->d_force, 4 * b->n * sizeof(double),
                                hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return bhip(b, e, "force read-back");
  for (int i = 0; i < b->n; ++i)
    for (int k = 0; k < 3; ++k) out[3 * i + k] = b->h_force[4 * i + k];
  return DG_OK;
}

int dg_batch_coupled_step(dg_batch* b, const double* osc, double* body, double* F,
                          const double* dt, double* v_w_out, void* stream) {
  if (!b) return DG_EINVAL;
  if (!osc || !body || !F || !dt) return bfail(b, DG_EINVAL, "osc, body, F and dt are required");
  const int n = b->n;
  std::vector<double> st(3 * n), vw(2 * n);
  for (int i = 0; i < n; ++i) {
    const double* o = osc + 4 * i;
    double* y = st.data() + 3 * i;
    y[0] = body[3 * i];
    y[1] = body[3 * i + 1];
    y[2] = body[3 * i + 2];
    if (dg_newmark_step(y, F[3 * i + 1] * o[3], dt[i], o[0], o[1], o[2]) != DG_OK)
      return bfail(b, DG_EINVAL, "Newmark step: non-positive dt or singular oscillator");
    vw[2 * i] = 0.0;
    vw[2 * i + 1] = (y[0] - body[3 * i]) / dt[i];
  }
  for (int k = 0; k < 3 * n; ++k) body[k] = st[k];
  int rc = dg_batch_rk_step(b, dt, vw.data(), stream);
  if (rc != DG_OK) return rc;
  rc = dg_batch_force(b, vw.data(), F, stream);
  if (rc != DG_OK) return rc;
  if (v_w_out)
    for (int k = 0; k < 2 * n; ++k) v_w_out[k] = vw[k];
  return DG_OK;
}

int dg_batch_configure(dg_batch* b, int mode, int waves, int grid, int use_graph) {
  if (!b) return DG_EINVAL;
  if ((mode != 0 && mode != 1) || (waves != 0 && waves != 2 && waves != 4) ||
      (grid != 0 && grid != 1))
    return bfail(b, DG_EINVAL, "mode 0/1, waves 0/2/4, grid 0/1");
  b->mode = mode;
  b->waves = waves;
  b->grid = grid;
  b->use_graph = use_graph ? 1 : 0;
  drop_graph(b);
  return plan(b);
}

int dg_batch_get_config(const dg_batch* b, int* mode, int* waves, int* grid, int* use_graph) {
  if (!b) return DG_EINVAL;
  if (mode) *mode = b->mode;
  if (waves) *waves = b->plan_waves;
  if (grid) *grid = b->grid;
  if (use_graph) *use_graph = b->use_graph;
  return DG_OK;
}

int dg_batch_autotune(dg_batch* b, int reps, void* stream, double* best_us) {
  if (!b) return DG_EINVAL;
  if (reps < 1) return bfail(b, DG_EINVAL, "reps must be positive");
  hipStream_t s = (hipStream_t)stream;
  // a finite dt for the timed launches; the first stage (A_1 = 0) writes only
  // the other state buffer and K1
  std::vector<double> dt(b->n, 1e-7), vw(2 * b->n, 0.0);
  int rc = upload(b, dt.data(), vw.data(), s);
  if (rc != DG_OK) return rc;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) return bhip(b, e, "hipEventCreate");
  const int keep_graph = b->use_graph;
  double best = 1e300;
  int bm = 0, bw = 0, bg = 0;
  for (int mode = 0; mode < 2 && rc == DG_OK; ++mode)
    for (int w : {2, 4})
      for (int grid = 0; grid < 2 && rc == DG_OK; ++grid) {
        b->mode = mode;
        b->waves = w;
        b->grid = grid;
        rc = plan(b);
        for (int r = 0; r < 3 && rc == DG_OK; ++r) rc = launch_stage_i(b, 0, s);
        if (rc != DG_OK) break;
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < reps && rc == DG_OK; ++r) rc = launch_stage_i(b, 0, s);
        (void)hipEventRecord(e1, s);
        e = hipEventSynchronize(e1);
        if (e != hipSuccess) {
          rc = bhip(b, e, "hipEventSynchronize");
          break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        const double us = 1e3 * ms / reps;
        if (rc == DG_OK && us < best) {
          best = us;
          bm = mode;
          bw = w;
          bg = grid;
        }
      }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != DG_OK) return rc;
  if (best_us) *best_us = best;
  return dg_batch_configure(b, bm, bw, bg, keep_graph);
}

const char* dg_batch_last_error(const dg_batch* b) {
  return b ? b->err.c_str() : g_batch_error.c_str();
}

void dg_batch_destroy(dg_batch* b) {
  if (!b) return;
  release(b);
  delete b;
}

}  // extern "C"
