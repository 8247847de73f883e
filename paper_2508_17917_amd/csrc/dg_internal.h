// Internal declarations shared by the host set-up, the C-ABI and the kernels.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace dgmi {

constexpr int kMaxOrder = 8;
constexpr int kGeoStride = 16;   // doubles per element in the geometry table

// Elements per tile of the stage kernel (one wavefront's unit of work): four,
// or three at orders 5 and 6, where four elements' 3(p + 1) face nodes each
// (72, 84) would take two passes over the 64 lanes and three (54, 63) take one.
constexpr int elements_per_tile(int N) { return (N == 5 || N == 6) ? 3 : 4; }

// Reference-element operators, row-major, FP64 (built once on K^).
struct RefOps {
  int N = 0, Np = 0, Nfp = 0;
  std::vector<double> r, s;            // Np
  std::vector<double> Dr, Ds;          // Np x Np
  std::vector<double> M;               // Np x Np reference mass matrix
  std::vector<double> LIFT;            // Np x 3Nfp, M^-1 E
  std::vector<double> LIFTr, LIFTs;    // Np x 3Nfp, M^-1 Dr^T E, M^-1 Ds^T E
  std::vector<int> Fmask;              // 3 x Nfp, counter-clockwise per face
  std::vector<double> wface;           // 3 x Nfp face quadrature weights in xi
};

// Over-integration operators of order N (quadrature exact for degree 3N on
// the element and on each face), row-major, FP64.
struct OIOps {
  int q = 0, Nq = 0;                   // points per direction; q^2 element points
  std::vector<double> wq;              // Nq element weights
  std::vector<double> xg, wg;          // q Gauss points and weights in the face parameter
  std::vector<double> Iq, Drq, Dsq;    // Nq x Np: l_j, d_r l_j, d_s l_j at the element points
  std::vector<double> Wr, Ws;          // Np x Nq: M^-1 (d_r l_i w)^T, M^-1 (d_s l_i w)^T
  std::vector<double> If1;             // q x Nfp: face-node values -> face points (any face)
  std::vector<double> Drf, Dsf;        // 3q x Np: d_r l_j, d_s l_j at the face points
  std::vector<double> LIFTq, LIFTrq, LIFTsq;  // Np x 3q: M^-1 (l_i w)^T, M^-1 (d_r l_i w)^T, ...
};
// launch_stage's form for the over-integrated FP64 stage (the precision modes
// are 0..3)
constexpr int kFormOverint = 4;
// the order's over-integration points per direction (degree 3N exact)
constexpr int oi_points(int N) { return (3 * N + 2) / 2; }

struct Physics {
  double gamma = 1.4, Pr = 0.72, mu = 0.0, theta = 1.0;
  int penalty_mode = 0;
  double C_pen = 0.01;
  double U_inf[4] = {1.0, 0.0, 0.0, 1.0};
  int wall_flux = 0;  // dg_wall_flux
};

// Mesh tables built on the host.
struct MeshTables {
  int64_t K = 0;
  std::vector<double> geo;        // K x 16: rx ry sx sy | (nx ny Fscale sigma_geo) x 3
  std::vector<int32_t> conn;      // K x 3 packed: nbr << 4 | nbr_face << 2 | tag
  std::vector<int32_t> nbr;       // K x 3 neighbour element (self on boundary)
  std::vector<int32_t> nbr_face;  // K x 3
  std::vector<int8_t> tag;        // K x 3
  std::vector<double> x, y;       // K x Np node coordinates
  std::vector<int32_t> wall_faces;  // list of k*3+f with tag wall
  std::vector<double> wall_xy;      // (x, y) of each wall face node, face-major
  // isoparametric elements (curved_setup.cpp): the set S of the curved
  // elements and their face neighbours, evaluated by the curved body with
  // per-node geometry; cslot[k] is k's slot in S or -1
  std::vector<int32_t> cslot;       // K (empty: no curved element)
  std::vector<int32_t> celem;       // |S|: element of each slot
  std::vector<double> cnode;        // |S| x 5 x Np: rx, ry, sx, sy, J at the nodes
  std::vector<double> cface;        // |S| x 3 x 3Nfp: nx, ny, sJ at the face nodes
  std::vector<double> cP;           // |S| x Np x Np: (M^K)^-1 M, row-major
  std::vector<double> carea;        // |S|: |K|
};

// host_setup.cpp
bool build_ref_ops(int N, RefOps& out, std::string& err);
bool build_oi_ops(const RefOps& ref, OIOps& out, std::string& err);
// matrix-core fragments of the over-integration operators, then the face-point
// tables: (D_r, D_s) pairs of the 3q face-point rows, and If1
void pack_oi(const RefOps& ref, const OIOps& oi, std::vector<double>& out);
bool build_mesh_tables(const RefOps& ref, const Physics& phys, int64_t Nv, const double* VX,
                       const double* VY, int64_t K, const int32_t* EToV, const int8_t* face_tag,
                       const double period[2], MeshTables& out, std::string& err);

bool build_order_maps(int lo, int hi, std::vector<double>& P, std::vector<double>& I,
                      std::string& err);

// curved_setup.cpp: replace the node positions of n elements (xy: n x 2 x Np,
// x then y per element) by those of their isoparametric maps and build the
// curved tables, the curved elements' penalty factors and wall coordinates
bool build_curved_tables(const RefOps& ref, const Physics& phys, int64_t n, const int32_t* elems,
                         const double* xy, MeshTables& t, std::string& err);
// host_setup.cpp helpers shared with it
void gauss_jacobi_rule(int q, double a, double b, std::vector<double>& x, std::vector<double>& w);
bool lagrange_at(const RefOps& ref, const std::vector<double>& r, const std::vector<double>& s,
                 std::vector<double>& L, std::vector<double>& Lr, std::vector<double>& Ls);
bool invert_matrix(std::vector<double>& A, int n);
double legendre(double x, int n);   // orthonormal Legendre polynomial
double dlegendre(double x, int n);

// Device-side view handed to the kernels.
struct DeviceTables {
  const double* geo = nullptr;     // K x 16
  const int32_t* conn = nullptr;   // K x 3
  const double* ops = nullptr;     // packed operators (pack_ops)
  const double* oi = nullptr;      // over-integration fragments and tables (pack_oi)
  int64_t oi_len = 0;              // its length in doubles
  const double* frag = nullptr;    // operator fragments in matrix-core lane order (pack_frags)
  const float* frag32 = nullptr;   // the same fragments rounded to FP32 (FP32 form)
  const unsigned short* frag16 = nullptr;  // bfloat16 fragments of the 16x16x16 instruction
  const int32_t* wall = nullptr;   // wall face list (k*3 + f)
  const double* wall_xy = nullptr; // node coordinates of the wall faces, (x, y) per face node
  int64_t K = 0;
  int nwall = 0;
  // isoparametric elements (see MeshTables): null / 0 without any
  const int32_t* cslot = nullptr;
  const int32_t* celem = nullptr;
  const double* cnode = nullptr;
  const double* cface = nullptr;
  const double* cP = nullptr;
  int ncurved = 0;                  // |S|
  double* force_part = nullptr;     // per-workgroup partials of the wall force
  unsigned* force_ticket = nullptr; // workgroups done (the last resets it to 0)
  int force_blocks = 0;             // capacity of force_part, in workgroups
  // the wall force inside stage launches: with force_parts, leading waves of
  // the launch write the force partials of its input state to force_part
  // (plain stores: no ticket, no fence); with force_fin, one leading wave adds
  // the partials a previous launch wrote, in block order, into force_fin[0..2]
  bool force_parts = false;
  double* force_fin = nullptr;
};

struct KernelPhysics {
  double gamma, Pr, mu, theta;
  double U_inf[4];
  double vw[2];
  // derived once on the host (wave-uniform constants the kernels would
  // otherwise divide out per lane): gamma - 1, 1/(gamma - 1), gamma/Pr, and
  // the free stream's pressure and velocity
  double gm1, igm1, k, p_inf, u_inf, v_inf;
  // conduction on wall faces: 0 (adiabatic wall, the default) or gamma/Pr
  // (the printed wall flux)
  double k_wall;
};

// Launch shape of the stage kernel: waves (= elements / 4) per workgroup, 0
// for the default of the order and form; grid 0 persistent (the resident
// workgroups stride over the tiles), 1 one tile per wave, 2 or 3 that many
// tiles per wave (within the resident workgroups).
struct StageTuning {
  int waves = 0;
  int grid = 0;
};

// kernels.hip.  form: 0 plain FP64, 1 perturbation FP64, 2 perturbation FP32,
// 3 perturbation FP32 with bfloat16 operator products (the dg_precision values).
int launch_stage(int N, int form, const StageTuning& tune, const DeviceTables& t,
                 const KernelPhysics& ph, const double* U_in, double* U_out, double* K1, double a,
                 double b, double dt, int rhs_only, void* stream, std::string& err);
int default_waves(int N, int form);

// Batched stages over many meshes (one launch per stage).
struct BatchItem {              // one instance, in device memory
  DeviceTables t;
  KernelPhysics ph;             // v_w is taken from the step parameters
  double* buf[2];               // state ping-pong buffers
  double* K1;
  int64_t tile_begin, tile_end; // its tiles in the numbering of its group
};
struct ForceItem {              // one instance's wall force in a batched launch (device memory)
  DeviceTables t;
  KernelPhysics ph;             // with the wall velocity of the state
  const double* U;
  double* out;                  // Fx, Fy, Mz
  int block_begin, nblocks;     // its workgroups within the launch of its order
};
struct BatchStep {              // per instance and step, in device memory
  double dt;
  double vw[2];
  double pad;
};
struct BatchGroup {             // instances of one order
  int p;
  int first_item, n_items;
  int block_begin, nblocks;     // multiples of 8
  int64_t ntiles;
};
struct BatchGroups {
  int ng;
  BatchGroup g[kMaxOrder];
};
int batch_resident_blocks(int form, int waves);
// the same for the one-order kernel of a group launched on its own
int batch_order_resident_blocks(int N, int form, int waves);
// one stage of one order group (g.block_begin = 0), in a kernel sized for order N
int launch_batch_order_stage(int N, int form, int waves, const BatchItem* items,
                             const BatchStep* steps, const int* parity, const BatchGroup& g,
                             int blocks, int stage, double a, double b, void* stream,
                             std::string& err);
// stage i of a step reads buf[(parity + i) & 1] and writes the other buffer
int launch_batch_stage(int form, int waves, const BatchItem* items, const BatchStep* steps,
                       const int* parity, const BatchGroups& G, int blocks, int stage, double a,
                       double b, void* stream, std::string& err);
// one thread per wall face node, 64 per workgroup
int force_blocks_for(int N, int nwall);
// the wall forces of `count` instances of order N in one launch of `blocks`
// workgroups (items in device memory, block ranges consecutive from 0)
int launch_batch_force(int N, const ForceItem* items, int count, int blocks, void* stream,
                       std::string& err);
// cfl.hip: Lambda of the CFL bound on the state U into work[6K] (work holds
// cfl_work_size(K) doubles)
size_t cfl_work_size(int64_t K);
int launch_cfl(int N, const DeviceTables& t, const KernelPhysics& ph, const double* U, double C_grad,
               double* work, void* stream, std::string& err);
int launch_force(int N, const DeviceTables& t, const KernelPhysics& ph, const double* U,
                 double* out_dev, void* stream, std::string& err);
// operator packing: Dr | Ds | LIFT | LIFTr | LIFTs | wface
size_t ops_packed_size(int N);
void pack_ops(const RefOps& ref, std::vector<double>& out);
// Dr | Ds | LIFT | LIFTr | LIFTs as B-operand fragments of the 16x16x4 FP64
// matrix instruction: for output tile t (nodes 16t..16t+15) and k-step s,
// lane l holds Op[16t + l%16][4s + l/16] (zero outside the matrix).
void pack_frags(const RefOps& ref, std::vector<double>& out);
// The FP32 matrix instruction (16x16x4 f32) takes its B operand in the same
// lane order, so the FP32 fragments are the FP64 ones rounded.
void pack_frags32(const RefOps& ref, std::vector<float>& out);
// Dr | Ds | LIFT | LIFTr | LIFTs as bfloat16 B-operand fragments of the
// 16x16x16 instruction: for output tile t and 16-deep k-step s, lane l holds
// Op[16t + l%16][16s + 4(l/16) + j], j = 0..3 (round to nearest even, zero
// outside the matrix).
void pack_frags_bf16(const RefOps& ref, std::vector<uint16_t>& out);

}  // namespace dgmi
