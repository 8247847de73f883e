// C-ABI of the library: context lifetime, host set-up, device tables and
// launches.  Every entry point returns a dg_status and records a message;
// nothing throws across the boundary.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "dg_ctx.h"

namespace {

std::string g_create_error;

int fail(dg_ctx* c, int code, const std::string& msg) {
  if (c)
    c->err = msg;
  else
    g_create_error = msg;
  return code;
}

int hip_fail(dg_ctx* c, hipError_t e, const char* what) {
  return fail(c, DG_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

void free_device(dg_ctx* c) {
  void* ptrs[] = {c->d_geo,  c->d_conn,    c->d_ops,     c->d_frag,       c->d_frag32,
                  c->d_frag16, c->d_wall, c->d_wall_xy, c->d_scratch, c->d_force,
                  c->d_force_part, c->d_force_ticket, c->d_oi, c->d_cfl,
                  c->d_cslot, c->d_celem, c->d_cnode, c->d_cface, c->d_cP};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (c->h_cfl) (void)hipHostFree(c->h_cfl);
  c->h_cfl = nullptr;
  c->d_geo = nullptr;
  c->d_conn = nullptr;
  c->d_ops = nullptr;
  c->d_frag = nullptr;
  c->d_frag32 = nullptr;
  c->d_frag16 = nullptr;
  c->d_wall = nullptr;
  c->d_wall_xy = nullptr;
  c->d_scratch = nullptr;
  c->d_force = nullptr;
  c->d_force_part = nullptr;
  c->d_force_ticket = nullptr;
  c->d_oi = nullptr;
  c->d_cfl = nullptr;
  c->d_cslot = nullptr;
  c->d_celem = nullptr;
  c->d_cnode = nullptr;
  c->d_cface = nullptr;
  c->d_cP = nullptr;
  c->force_blocks = 0;
  c->dev_ready = false;
}

template <typename T>
hipError_t upload(T** dst, const std::vector<T>& src) {
  size_t bytes = src.size() * sizeof(T);
  if (bytes == 0) bytes = sizeof(T);
  hipError_t e = hipMalloc((void**)dst, bytes);
  if (e != hipSuccess) return e;
  if (!src.empty()) e = hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
  return e;
}

dgmi::DeviceTables tables(const dg_ctx* c) {
  dgmi::DeviceTables t;
  t.geo = c->d_geo;
  t.conn = c->d_conn;
  t.ops = c->d_ops;
  t.frag = c->d_frag;
  t.oi = c->d_oi;
  t.oi_len = c->oi_len;
  t.frag32 = c->d_frag32;
  t.frag16 = c->d_frag16;
  t.wall = c->d_wall;
  t.wall_xy = c->d_wall_xy;
  t.K = c->K;
  t.nwall = (int)c->mesh.wall_faces.size();
  t.force_part = c->d_force_part;
  t.force_ticket = c->d_force_ticket;
  t.force_blocks = c->force_blocks;
  if (!c->mesh.celem.empty()) {
    t.cslot = c->d_cslot;
    t.celem = c->d_celem;
    t.cnode = c->d_cnode;
    t.cface = c->d_cface;
    t.cP = c->d_cP;
    t.ncurved = (int)c->mesh.celem.size();
  }
  return t;
}

dgmi::KernelPhysics kphys(const dg_ctx* c, const double vw[2]) {
  dgmi::KernelPhysics k;
  k.gamma = c->phys.gamma;
  k.Pr = c->phys.Pr;
  k.mu = c->phys.mu;
  k.theta = c->phys.theta;
  for (int i = 0; i < 4; ++i) k.U_inf[i] = c->phys.U_inf[i];
  k.vw[0] = vw ? vw[0] : 0.0;
  k.vw[1] = vw ? vw[1] : 0.0;
  k.gm1 = k.gamma - 1.0;
  k.igm1 = 1.0 / (k.gamma - 1.0);
  k.k = k.gamma / k.Pr;
  k.u_inf = k.U_inf[1] / k.U_inf[0];
  k.v_inf = k.U_inf[2] / k.U_inf[0];
  const double ke = k.U_inf[1] * k.u_inf + k.U_inf[2] * k.v_inf;
  k.p_inf = k.gm1 * (k.U_inf[3] - 0.5 * ke);
  k.k_wall = c->phys.wall_flux == DG_WALL_PRINTED ? k.k : 0.0;
  return k;
}

int check_ready(dg_ctx* c) {
  if (!c) return fail(c, DG_EINVAL, "null context");
  if (!c->dev_ready) return fail(c, DG_ESTATE, "dg_setup has not completed on this context");
  return DG_OK;
}

}  // namespace

namespace dgmi {
int ctx_fail(dg_ctx* c, int code, const std::string& msg) { return fail(c, code, msg); }
int ctx_hip_fail(dg_ctx* c, hipError_t e, const char* what) { return hip_fail(c, e, what); }
DeviceTables ctx_tables(const dg_ctx* c) { return tables(c); }
KernelPhysics ctx_phys(const dg_ctx* c, const double vw[2]) { return kphys(c, vw); }
}  // namespace dgmi

extern "C" {

int dg_create(int p, int precision, dg_ctx** out) {
  if (!out) return fail(nullptr, DG_EINVAL, "out is NULL");
  *out = nullptr;
  if (p < 1 || p > 6) return fail(nullptr, DG_EUNSUPPORTED, "polynomial order must be in 1..6");
  if (precision != DG_FP64 && precision != DG_FP64_PERT && precision != DG_FP32_PERT &&
      precision != DG_FP32_PERT_BF16OPS)
    return fail(nullptr, DG_EUNSUPPORTED, "unsupported precision mode");
  dg_ctx* c = new (std::nothrow) dg_ctx();
  if (!c) return fail(nullptr, DG_ENOMEM, "out of host memory");
  c->N = p;
  c->precision = precision;
  *out = c;
  return DG_OK;
}

int dg_set_physics(dg_ctx* c, double gamma, double Pr, double mu, double theta, int penalty_mode,
                   double C_pen, const double U_inf[4]) {
  if (!c) return fail(c, DG_EINVAL, "null context");
  if (!U_inf) return fail(c, DG_EINVAL, "U_inf is NULL");
  if (!(gamma > 1.0) || !(Pr > 0.0) || !(mu >= 0.0) || !(theta >= -1.0 && theta <= 1.0) ||
      (penalty_mode != DG_PENALTY_PAPER && penalty_mode != DG_PENALTY_STANDARD) || !(C_pen >= 0.0))
    return fail(c, DG_EINVAL, "physics parameter out of range");
  if (!(U_inf[0] > 0.0)) return fail(c, DG_EINVAL, "far-field density must be positive");
  c->phys.gamma = gamma;
  c->phys.Pr = Pr;
  c->phys.mu = mu;
  c->phys.theta = theta;
  c->phys.penalty_mode = penalty_mode;
  c->phys.C_pen = C_pen;
  for (int i = 0; i < 4; ++i) c->phys.U_inf[i] = U_inf[i];
  c->have_phys = true;
  c->host_ready = false;
  return DG_OK;
}

int dg_set_wall_flux(dg_ctx* c, int mode) {
  if (!c) return DG_EINVAL;
  if (mode != DG_WALL_ADIABATIC && mode != DG_WALL_PRINTED)
    return fail(c, DG_EINVAL, "wall flux mode must be DG_WALL_ADIABATIC or DG_WALL_PRINTED");
  c->phys.wall_flux = mode;
  return DG_OK;
}

int dg_set_mesh(dg_ctx* c, int64_t Nv, const double* VX, const double* VY, int64_t K,
                const int32_t* EToV, const int8_t* face_tag, const double period[2]) {
  if (!c) return fail(c, DG_EINVAL, "null context");
  if (Nv < 3 || K < 1 || !VX || !VY || !EToV) return fail(c, DG_EINVAL, "empty or NULL mesh arrays");
  c->VX.assign(VX, VX + Nv);
  c->VY.assign(VY, VY + Nv);
  c->EToV.assign(EToV, EToV + 3 * K);
  if (face_tag)
    c->tag.assign(face_tag, face_tag + 3 * K);
  else
    c->tag.assign(3 * K, 0);
  c->period[0] = period ? period[0] : 0.0;
  c->period[1] = period ? period[1] : 0.0;
  c->Nv = Nv;
  c->K = K;
  c->have_mesh = true;
  c->host_ready = false;
  c->curved_elems.clear();
  c->curved_xy.clear();
  return DG_OK;
}

int dg_set_curved_elements(dg_ctx* c, int64_t n, const int32_t* elems, const double* xy) {
  if (!c) return fail(c, DG_EINVAL, "null context");
  if (!c->have_mesh) return fail(c, DG_ESTATE, "dg_set_mesh must precede dg_set_curved_elements");
  if (n < 0 || (n > 0 && (!elems || !xy))) return fail(c, DG_EINVAL, "NULL or negative curved-element arrays");
  if (n > 0 && c->overint)
    return fail(c, DG_EUNSUPPORTED, "curved elements are not built for the over-integrated stage");
  std::vector<char> seen(c->K, 0);
  for (int64_t i = 0; i < n; ++i) {
    if (elems[i] < 0 || elems[i] >= c->K) return fail(c, DG_EINVAL, "curved element index out of range");
    if (seen[elems[i]]) return fail(c, DG_EINVAL, "a curved element is listed twice");
    seen[elems[i]] = 1;
  }
  const int Np = (c->N + 1) * (c->N + 2) / 2;
  for (int64_t i = 0; i < n * 2 * Np; ++i)
    if (!std::isfinite(xy[i])) return fail(c, DG_EINVAL, "non-finite curved node position");
  c->curved_elems.assign(elems, elems + n);
  c->curved_xy.assign(xy, xy + n * 2 * Np);
  c->host_ready = false;
  return DG_OK;
}

int dg_setup_host(dg_ctx* c) {
  if (!c) return fail(c, DG_EINVAL, "null context");
  if (!c->have_phys || !c->have_mesh)
    return fail(c, DG_ESTATE, "dg_set_physics and dg_set_mesh must precede set-up");
  std::string err;
  if (!dgmi::build_ref_ops(c->N, c->ref, err)) return fail(c, DG_EUNSUPPORTED, err);
  if (!dgmi::build_oi_ops(c->ref, c->oi, err)) return fail(c, DG_EUNSUPPORTED, err);
  if (!dgmi::build_mesh_tables(c->ref, c->phys, c->Nv, c->VX.data(), c->VY.data(), c->K,
                               c->EToV.data(), c->tag.data(), c->period, c->mesh, err))
    return fail(c, DG_EMESH, err);
  if (!dgmi::build_curved_tables(c->ref, c->phys, (int64_t)c->curved_elems.size(),
                                 c->curved_elems.data(), c->curved_xy.data(), c->mesh, err))
    return fail(c, DG_EMESH, err);
  c->host_ready = true;
  return DG_OK;
}

int dg_setup(dg_ctx* c) {
  if (!c) return fail(c, DG_EINVAL, "null context");
  if (!c->host_ready) {
    int rc = dg_setup_host(c);
    if (rc != DG_OK) return rc;
  }
  free_device(c);
  hipError_t e = hipGetDevice(&c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipGetDevice");
  std::vector<double> ops, frag, oi;
  std::vector<float> frag32;
  std::vector<uint16_t> frag16;
  dgmi::pack_ops(c->ref, ops);
  dgmi::pack_frags(c->ref, frag);
  dgmi::pack_frags32(c->ref, frag32);
  dgmi::pack_frags_bf16(c->ref, frag16);
  dgmi::pack_oi(c->ref, c->oi, oi);
  c->oi_len = (int64_t)oi.size();
  if ((e = upload(&c->d_geo, c->mesh.geo)) != hipSuccess ||
      (e = upload(&c->d_conn, c->mesh.conn)) != hipSuccess ||
      (e = upload(&c->d_ops, ops)) != hipSuccess ||
      (e = upload(&c->d_frag, frag)) != hipSuccess ||
      (e = upload(&c->d_frag32, frag32)) != hipSuccess ||
      (e = upload(&c->d_frag16, frag16)) != hipSuccess ||
      (e = upload(&c->d_oi, oi)) != hipSuccess ||
      (e = upload(&c->d_wall, c->mesh.wall_faces)) != hipSuccess ||
      (e = upload(&c->d_wall_xy, c->mesh.wall_xy)) != hipSuccess ||
      (!c->mesh.celem.empty() &&
       ((e = upload(&c->d_cslot, c->mesh.cslot)) != hipSuccess ||
        (e = upload(&c->d_celem, c->mesh.celem)) != hipSuccess ||
        (e = upload(&c->d_cnode, c->mesh.cnode)) != hipSuccess ||
        (e = upload(&c->d_cface, c->mesh.cface)) != hipSuccess ||
        (e = upload(&c->d_cP, c->mesh.cP)) != hipSuccess))) {
    free_device(c);
    return hip_fail(c, e, "uploading set-up tables");
  }
  size_t state = (size_t)c->K * 4 * c->ref.Np * sizeof(double);
  c->force_blocks = dgmi::force_blocks_for(c->N, (int)c->mesh.wall_faces.size());
  const int fb = c->force_blocks > 0 ? c->force_blocks : 1;
  if ((e = hipMalloc((void**)&c->d_scratch, state)) != hipSuccess ||
      (e = hipMalloc((void**)&c->d_force, 4 * sizeof(double))) != hipSuccess ||
      (e = hipMalloc((void**)&c->d_force_part, 3 * fb * sizeof(double))) != hipSuccess ||
      (e = hipMalloc((void**)&c->d_force_ticket, sizeof(unsigned))) != hipSuccess ||
      (e = hipMalloc((void**)&c->d_cfl, dgmi::cfl_work_size(c->K) * sizeof(double))) != hipSuccess ||
      (e = hipHostMalloc((void**)&c->h_cfl, sizeof(double), hipHostMallocDefault)) != hipSuccess ||
      (e = hipMemset(c->d_force_ticket, 0, sizeof(unsigned))) != hipSuccess) {
    free_device(c);
    return e == hipErrorOutOfMemory ? fail(c, DG_ENOMEM, "device allocation failed")
                                    : hip_fail(c, e, "hipMalloc");
  }
  // the allocation-free entry point's static array on this device (a lookup,
  // no allocation); left unset if the lookup fails, which that entry point
  // then reports
  {
    std::string serr;
    if (dgmi::noalloc_scratch_address(&c->noalloc_scratch, serr) != DG_OK) c->noalloc_scratch = nullptr;
  }
  c->dev_ready = true;
  return DG_OK;
}

int dg_set_overintegration(dg_ctx* c, int on) {
  if (!c) return DG_EINVAL;
  if (on && c->precision != DG_FP64)
    return fail(c, DG_EUNSUPPORTED, "over-integration runs in the plain FP64 form only");
  if (on && (c->N < 1 || c->N > 6)) return fail(c, DG_EUNSUPPORTED, "over-integration is built for p = 1..6");
  if (on && !c->curved_elems.empty())
    return fail(c, DG_EUNSUPPORTED, "over-integration is not built for curved elements");
  c->overint = on != 0;
  return DG_OK;
}

int64_t dg_num_elements(const dg_ctx* c) { return c ? c->K : 0; }
int dg_num_nodes(const dg_ctx* c) { return c ? (c->N + 1) * (c->N + 2) / 2 : 0; }
int dg_num_face_nodes(const dg_ctx* c) { return c ? c->N + 1 : 0; }

int dg_get_host_table(const dg_ctx* cc, const char* name, double* out, int64_t count) {
  dg_ctx* c = const_cast<dg_ctx*>(cc);
  if (!c || !name || !out) return fail(c, DG_EINVAL, "NULL argument");
  if (!c->host_ready) return fail(c, DG_ESTATE, "host set-up not done");
  std::vector<double> v;
  const dgmi::RefOps& r = c->ref;
  const dgmi::MeshTables& m = c->mesh;
  std::string n(name);
  if (n == "r") v = r.r;
  else if (n == "s") v = r.s;
  else if (n == "Dr") v = r.Dr;
  else if (n == "Ds") v = r.Ds;
  else if (n == "M") v = r.M;
  else if (n == "LIFT") v = r.LIFT;
  else if (n == "LIFTr") v = r.LIFTr;
  else if (n == "LIFTs") v = r.LIFTs;
  else if (n == "wface") v = r.wface;
  else if (n == "Fmask") v.assign(r.Fmask.begin(), r.Fmask.end());
  else if (n == "geo") v = m.geo;
  else if (n == "nbr") v.assign(m.nbr.begin(), m.nbr.end());
  else if (n == "nbr_face") v.assign(m.nbr_face.begin(), m.nbr_face.end());
  else if (n == "curved_slot") {
    v.assign(m.cslot.begin(), m.cslot.end());
    if (v.empty()) v.assign(c->K, -1.0);
  }
  else if (n == "curved_elem") v.assign(m.celem.begin(), m.celem.end());
  else if (n == "curved_node") v = m.cnode;
  else if (n == "curved_face") v = m.cface;
  else if (n == "curved_P") v = m.cP;
  else if (n == "curved_area") v = m.carea;
  else if (n == "oi_wq") v = c->oi.wq;
  else if (n == "oi_xg") v = c->oi.xg;
  else if (n == "oi_wg") v = c->oi.wg;
  else if (n == "oi_Iq") v = c->oi.Iq;
  else if (n == "oi_Drq") v = c->oi.Drq;
  else if (n == "oi_Dsq") v = c->oi.Dsq;
  else if (n == "oi_Wr") v = c->oi.Wr;
  else if (n == "oi_Ws") v = c->oi.Ws;
  else if (n == "oi_If1") v = c->oi.If1;
  else if (n == "oi_Drf") v = c->oi.Drf;
  else if (n == "oi_Dsf") v = c->oi.Dsf;
  else if (n == "oi_LIFTq") v = c->oi.LIFTq;
  else if (n == "oi_LIFTrq") v = c->oi.LIFTrq;
  else if (n == "oi_LIFTsq") v = c->oi.LIFTsq;
  else return fail(c, DG_EINVAL, "unknown table " + n);
  if ((int64_t)v.size() != count)
    return fail(c, DG_EINVAL, "table " + n + " has " + std::to_string(v.size()) + " entries");
  std::memcpy(out, v.data(), v.size() * sizeof(double));
  return DG_OK;
}

int dg_get_nodes(const dg_ctx* cc, double* x, double* y) {
  dg_ctx* c = const_cast<dg_ctx*>(cc);
  if (!c || !x || !y) return fail(c, DG_EINVAL, "NULL argument");
  if (!c->host_ready) return fail(c, DG_ESTATE, "host set-up not done");
  std::memcpy(x, c->mesh.x.data(), c->mesh.x.size() * sizeof(double));
  std::memcpy(y, c->mesh.y.data(), c->mesh.y.size() * sizeof(double));
  return DG_OK;
}

int dg_rhs(dg_ctx* c, const double* U, double* R, const double v_w[2], void* stream) {
  int rc = check_ready(c);
  if (rc != DG_OK) return rc;
  if (!U || !R || U == R) return fail(c, DG_EINVAL, "U and R must be distinct device arrays");
  std::string err;
  rc = dgmi::launch_stage(c->N, dgmi::ctx_form(c), c->tune, tables(c), kphys(c, v_w), U, nullptr, R, 0.0, 0.0, 1.0, 1, stream,
                          err);
  return rc == 0 ? DG_OK : fail(c, rc, err);
}

int dg_rk_stage(dg_ctx* c, const double* Uin, double* Uout, double* K1, double a, double b,
                double dt, const double v_w[2], void* stream) {
  int rc = check_ready(c);
  if (rc != DG_OK) return rc;
  if (!Uin || !Uout || !K1 || Uin == Uout || K1 == Uin || K1 == Uout)
    return fail(c, DG_EINVAL, "U_in, U_out and K1 must be distinct device arrays");
  std::string err;
  rc = dgmi::launch_stage(c->N, dgmi::ctx_form(c), c->tune, tables(c), kphys(c, v_w), Uin, Uout, K1, a, b, dt, 0, stream, err);
  return rc == 0 ? DG_OK : fail(c, rc, err);
}

int dg_rk_step(dg_ctx* c, double* U, double* K1, double dt, const double v_w[2], void* stream) {
  int rc = check_ready(c);
  if (rc != DG_OK) return rc;
  if (!U || !K1 || U == K1) return fail(c, DG_EINVAL, "U and K1 must be distinct device arrays");
  if (!std::isfinite(dt)) return fail(c, DG_EINVAL, "dt is not finite");
  std::string err;
  dgmi::DeviceTables t = tables(c);
  dgmi::KernelPhysics k = kphys(c, v_w);
  double* bufs[2] = {U, c->d_scratch};
  for (int i = 0; i < 5; ++i) {
    rc = dgmi::launch_stage(c->N, dgmi::ctx_form(c), c->tune, t, k, bufs[i & 1], bufs[(i + 1) & 1], K1, dgmi::kRkA[i], dgmi::kRkB[i], dt, 0,
                            stream, err);
    if (rc != 0) return fail(c, rc, err);
  }
  size_t bytes = (size_t)c->K * 4 * c->ref.Np * sizeof(double);
  hipError_t e = hipMemcpyAsync(U, c->d_scratch, bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(c, e, "hipMemcpyAsync");
  return DG_OK;
}

int dg_rk_steps(dg_ctx* c, double* U, double* K1, int nsteps, double dt, const double v_w[2],
                double* force_dev, void* stream) {
  int rc = check_ready(c);
  if (rc != DG_OK) return rc;
  if (!U || !K1 || U == K1) return fail(c, DG_EINVAL, "U and K1 must be distinct device arrays");
  if (nsteps < 0) return fail(c, DG_EINVAL, "nsteps must be non-negative");
  if (!std::isfinite(dt)) return fail(c, DG_EINVAL, "dt is not finite");
  std::string err;
  const dgmi::DeviceTables t = tables(c);
  const dgmi::KernelPhysics k = kphys(c, v_w);
  const bool walls = !c->mesh.wall_faces.empty();
  // the state alternates between U and the scratch buffer: five stages per
  // step, so it sits in the other buffer after every step
  double* bufs[2] = {U, c->d_scratch};
  // the force after step n: its partials by leading waves of step n + 1's
  // first stage launch, whose input is that state, their sum in block order
  // by a leading wave of the second (the nodal stage kernel; the
  // over-integrated stage launches it apart); the last step's by a launch of
  // its own
  const bool fuse = force_dev && walls && !c->overint;
  int cur = 0;
  for (int n = 0; n < nsteps; ++n) {
    for (int i = 0; i < 5; ++i) {
      dgmi::DeviceTables ti = t;
      if (fuse && n > 0 && i == 0) ti.force_parts = true;
      if (fuse && n > 0 && i == 1) ti.force_fin = force_dev + 3 * (int64_t)(n - 1);
      rc = dgmi::launch_stage(c->N, dgmi::ctx_form(c), c->tune, ti, k, bufs[(cur + i) & 1],
                              bufs[(cur + i + 1) & 1], K1, dgmi::kRkA[i], dgmi::kRkB[i], dt, 0,
                              stream, err);
      if (rc != 0) return fail(c, rc, err);
    }
    cur ^= 1;
    if (fuse && n == nsteps - 1) {
      rc = dgmi::launch_force(c->N, t, k, bufs[cur], force_dev + 3 * (int64_t)n, stream, err);
      if (rc != 0) return fail(c, rc, err);
    } else if (force_dev && !fuse) {
      if (walls) {
        rc = dgmi::launch_force(c->N, t, k, bufs[cur], force_dev + 3 * (int64_t)n, stream, err);
        if (rc != 0) return fail(c, rc, err);
      } else {
        hipError_t e = hipMemsetAsync(force_dev + 3 * (int64_t)n, 0, 3 * sizeof(double),
                                      (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(c, e, "hipMemsetAsync");
      }
    }
  }
  if (cur == 1) {
    const size_t bytes = (size_t)c->K * 4 * c->ref.Np * sizeof(double);
    hipError_t e = hipMemcpyAsync(U, c->d_scratch, bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "hipMemcpyAsync");
  }
  return DG_OK;
}

int dg_force(dg_ctx* c, const double* U, const double v_w[2], double out[3], void* stream) {
  int rc = check_ready(c);
  if (rc != DG_OK) return rc;
  if (!U || !out) return fail(c, DG_EINVAL, "NULL argument");
  if (c->mesh.wall_faces.empty()) {
    out[0] = out[1] = out[2] = 0.0;
    return DG_OK;
  }
  std::string err;
  rc = dgmi::launch_force(c->N, tables(c), kphys(c, v_w), U, c->d_force, stream, err);
  if (rc != 0) return fail(c, rc, err);
  double h[3];
  hipError_t e = hipMemcpyAsync(h, c->d_force, 3 * sizeof(double), hipMemcpyDeviceToHost,
                                (hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(c, e, "force read-back");
  out[0] = h[0];
  out[1] = h[1];
  out[2] = h[2];
  return DG_OK;
}

int dg_cfl_time_step(dg_ctx* c, const double* U, const double v_w[2], double C_cfl, double C_grad,
                     double out[2], void* stream) {
  int rc = check_ready(c);
  if (rc != DG_OK) return rc;
  if (!U || !out) return fail(c, DG_EINVAL, "NULL argument");
  if (!(C_cfl > 0.0) || !(C_grad >= 0.0)) return fail(c, DG_EINVAL, "C_cfl must be > 0, C_grad >= 0");
  std::string err;
  rc = dgmi::launch_cfl(c->N, tables(c), kphys(c, v_w), U, C_grad, c->d_cfl, stream, err);
  if (rc != 0) return fail(c, rc, err);
  hipError_t e = hipMemcpyAsync(c->h_cfl, c->d_cfl + 6 * c->K, sizeof(double),
                                hipMemcpyDeviceToHost, (hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(c, e, "CFL read-back");
  const double lam = *c->h_cfl;
  if (!std::isfinite(lam) || !(lam > 0.0)) return fail(c, DG_ENONFINITE, "CFL bound is not finite and positive");
  out[0] = lam;
  out[1] = C_cfl / lam;
  return DG_OK;
}

int dg_force_device(dg_ctx* c, const double* U, const double v_w[2], double* out_dev,
                    void* stream) {
  int rc = check_ready(c);
  if (rc != DG_OK) return rc;
  if (!U || !out_dev) return fail(c, DG_EINVAL, "NULL argument");
  if (c->mesh.wall_faces.empty()) {
    hipError_t e = hipMemsetAsync(out_dev, 0, 3 * sizeof(double), (hipStream_t)stream);
    return e == hipSuccess ? DG_OK : hip_fail(c, e, "hipMemsetAsync");
  }
  std::string err;
  rc = dgmi::launch_force(c->N, tables(c), kphys(c, v_w), U, out_dev, stream, err);
  return rc == 0 ? DG_OK : fail(c, rc, err);
}

int dg_newmark_step(double st[3], double F_new, double dt, double M, double C, double K) {
  if (!st || !(dt > 0.0)) return DG_EINVAL;
  const double beta = 0.25, gam = 0.5;
  double lhs = M + gam * dt * C + beta * dt * dt * K;
  if (lhs == 0.0) return DG_EINVAL;
  double y = st[0], yd = st[1], ydd = st[2];
  double rhs = F_new - C * (yd + (1.0 - gam) * dt * ydd) - K * (y + dt * yd + (0.5 - beta) * dt * dt * ydd);
  double ydd_n = rhs / lhs;
  st[0] = y + dt * yd + 0.5 * dt * dt * ((1.0 - 2.0 * beta) * ydd + 2.0 * beta * ydd_n);
  st[1] = yd + dt * ((1.0 - gam) * ydd + gam * ydd_n);
  st[2] = ydd_n;
  return DG_OK;
}

const char* dg_last_error(const dg_ctx* c) { return c ? c->err.c_str() : g_create_error.c_str(); }

void dg_destroy(dg_ctx* c) {
  if (!c) return;
  if (c->dev_ready || c->d_geo) free_device(c);
  delete c;
}

}  // extern "C"
