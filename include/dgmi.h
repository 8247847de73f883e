/*
 * dgmi -- nodal interior-penalty DG right-hand side for the 2D compressible
 * Navier-Stokes equations on triangles, hand-written for MI355X (gfx950).
 *
 * Method: Zafeiris, Georgoulis & Papadakis, "Parallel nodal interior-penalty
 * discontinuous Galerkin methods for the subsonic compressible Navier-Stokes
 * equations" (arXiv 2508.17917).  Section/equation references below are to
 * that paper.
 *
 * Conventions shared by every call
 *   - State U = [rho, rho v1, rho v2, eps] (Sec. 2.1, eq. cnp), eps = total
 *     energy per unit volume, p = (gamma-1)(eps - rho|v|^2/2).
 *   - Nodal layout at the boundary: U[K][4][Np], row-major, element-major:
 *     one element's 4 x Np block is contiguous.  Np = (p+1)(p+2)/2.
 *   - Nodes on the reference triangle {(-1,-1),(1,-1),(-1,1)} are Warburton's
 *     warp & blend nodes, numbered row by row from the edge s = -1 upward,
 *     by increasing r inside a row; dg_get_nodes returns their physical
 *     coordinates.
 *   - Face f of element k joins local vertices f and (f+1)%3 (vertices
 *     counter-clockwise); face tags: 0 interior or periodic, 1 moving
 *     adiabatic wall, 2 far field (Sec. 2.1 boundary split).
 *   - Device pointers are plain HIP device addresses (e.g. a torch tensor's
 *     data_ptr()); `stream` is a hipStream_t (NULL = default stream).  The
 *     caller owns U, K1 and R; the library owns its operator, geometry and
 *     connectivity tables from dg_setup until dg_destroy, plus one state-
 *     sized scratch buffer used by dg_rk_step.
 *   - Every call returns a dg_status; none aborts or throws across the ABI.
 *     dg_last_error gives the message of the last failing call on a context.
 *   - Calls on one context are not thread-safe; different contexts are
 *     independent.
 */
#ifndef DGMI_H
#define DGMI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dg_ctx dg_ctx;

typedef enum dg_status {
  DG_OK = 0,
  DG_EINVAL = -1,        /* bad argument (NULL pointer, size, range)            */
  DG_ENOMEM = -2,        /* host or device allocation failed                    */
  DG_EHIP = -3,          /* a HIP runtime call failed (message has the reason)  */
  DG_EMESH = -4,         /* non-conforming face, J <= 0 (clockwise element),    *
                          * unmatched periodic face, or bad face tag            */
  DG_EUNSUPPORTED = -5,  /* polynomial order or precision not built             */
  DG_ENONFINITE = -6,    /* non-finite value found by a health check            */
  DG_ESTATE = -7         /* call out of order (e.g. dg_rhs before dg_setup)     */
} dg_status;

/* Arithmetic of the right-hand side.  The RK registers (the state U and
 * K1 of Alg. 1) are binary64 in every mode; in the perturbation modes the
 * kernel works on U' = U - U_inf (U_inf the far-field state of
 * dg_set_physics), writing every flux as F(U_inf + U') - F(U_inf) without
 * cancellation (the constant F(U_inf) has no divergence and cancels from
 * every face term), so that the small deviations of a low-Mach flow from
 * the free stream keep their relative precision in binary32. */
typedef enum dg_precision {
  DG_FP64 = 0,           /* every step in IEEE binary64                         */
  DG_FP64_PERT = 1,      /* perturbation form, binary64 (equal to DG_FP64 up    *
                          * to rounding; a check on the perturbation algebra)   */
  DG_FP32_PERT = 2,      /* perturbation form, binary32 right-hand side,        *
                          * binary32 matrix-core products, binary64 RK update   */
  DG_FP32_PERT_BF16OPS = 3 /* as DG_FP32_PERT, but the operator products (Dr, *
                          * Ds, LIFT, LIFTr, LIFTs) on the bfloat16 matrix      *
                          * cores with binary32 accumulation                    */
} dg_precision;

typedef enum dg_penalty_mode {
  /* sigma_e = C1 (1+theta)^2 (d+1) Gbar_e max_{+-} C_inv(e,K+-,p),
   * C_inv = (p+1)(p+2)|e|/(2|K|)                        (eq. penalty_final) */
  DG_PENALTY_PAPER = 0,
  /* sigma_e = C (p+1)^2 Gbar_e / min_{+-} h_e, h_e = 2|K|/|e|  (literature
   * form of Sec. 2.2.3 with the diffusion scale Gbar_e supplying the units) */
  DG_PENALTY_STANDARD = 1
} dg_penalty_mode;

/* Viscous flux on the moving wall (Sec. 2.2.4).  The printed wall flux
 * G(U^b) grad U+ (and G(U^b) in the wall's theta term) carries the
 * interior's heat conduction through the wall, while the same section calls
 * the wall adiabatic (Neumann conditions on pressure and temperature).
 * DG_WALL_ADIABATIC (the default): the stress and its work, no conduction;
 * DG_WALL_PRINTED: G(U^b) grad U+ as printed, with conduction. */
typedef enum dg_wall_flux {
  DG_WALL_ADIABATIC = 0,
  DG_WALL_PRINTED = 1
} dg_wall_flux;

/* Create a context for polynomial order p (1 <= p <= 6) and a dg_precision mode.  *out receives the
 * context (owned by the caller, released with dg_destroy).  No GPU work. */
int dg_create(int p, int precision, dg_ctx** out);

/* Physics of eq. cnp and the IP flux (eq. ip_flux): gamma, Prandtl number,
 * constant dynamic viscosity mu, theta in [-1,1] (1 SIPG, 0 IIPG, -1 NIPG),
 * penalty mode and its constant, far-field state U_inf[4] (Sec. 2.2.4,
 * ghost state on far-field faces).  Host only. */
int dg_set_physics(dg_ctx* ctx, double gamma, double Pr, double mu, double theta,
                   int penalty_mode, double C_pen, const double U_inf[4]);

/* Isoparametric (curved) elements (Sec. 2.2: T_K affine or isoparametric).
 * elems: n element indices (host, int32, each once, in [0, K)); xy: host
 * array n x 2 x Np, for element elems[i] the x then the y coordinates of its
 * Np nodes in the library's node order (dg_get_nodes gives the straight
 * positions).  The element's map is the degree-p interpolant of these
 * positions; its faces shared with other elements must keep the other side's
 * node positions (a conforming mesh; checked at set-up, DG_EMESH otherwise,
 * also for a non-positive Jacobian).  Per-node metric terms, per-face-node
 * normals and sJ, the mass matrix int l_i l_j J and the penalty's C_inv with
 * the curved face length and area are built by the host set-up; the curved
 * elements and their face neighbours are evaluated in FP64 in every precision
 * mode, one element per wave in the stage launch's leading workgroups (the
 * wall force uses the same geometry).  n = 0
 * removes them.  Host only; after dg_set_mesh (which clears them) and before
 * dg_setup_host / dg_setup.  DG_EINVAL for bad indices or non-finite
 * positions, DG_EUNSUPPORTED with over-integration; batches refuse such
 * contexts. */
int dg_set_curved_elements(dg_ctx* ctx, int64_t n, const int32_t* elems, const double* xy);

/* The wall's viscous flux (a dg_wall_flux mode; default DG_WALL_ADIABATIC).
 * Host only; any time after dg_create, taking effect at the next launch (a
 * batch keeps the modes its contexts had at dg_batch_create); DG_EINVAL for
 * another mode. */
int dg_set_wall_flux(dg_ctx* ctx, int mode);

/* Mesh T of straight-sided triangles (Sec. 2.2): Nv vertices (VX, VY host
 * arrays of length Nv), K triangles (EToV host array K*3, counter-clockwise
 * vertex indices), face_tag host array K*3 (see conventions), period[2] the
 * periods in x and y of a periodic mesh (0 = not periodic; interior faces on
 * opposite sides are then matched by translation).  The arrays are copied.
 * Host only; connectivity is built here (DG_EMESH on failure). */
int dg_set_mesh(dg_ctx* ctx, int64_t Nv, const double* VX, const double* VY,
                int64_t K, const int32_t* EToV, const int8_t* face_tag,
                const double period[2]);

/* Host part of the set-up, in FP64: warp & blend nodes, PKD Vandermonde V,
 * Dr = Vr V^-1, Ds = Vs V^-1, M^-1 = V V^T, face mass E, LIFT = M^-1 E and
 * the theta-term lifts M^-1 Dr^T E, M^-1 Ds^T E (Sec. 2.2, eq.
 * weak_matrices_calc, built once on the reference element), geometric
 * factors of the affine maps, face normals, and the penalty's geometric
 * factors.  Needs dg_set_physics and dg_set_mesh.  No GPU work. */
int dg_setup_host(dg_ctx* ctx);

/* dg_setup_host (if not done) followed by the upload of every table to the
 * current HIP device and allocation of the scratch state buffer. */
int dg_setup(dg_ctx* ctx);

/* Over-integration (Sec. 2.2, the oversampling remedy for aliasing of the
 * rational fluxes): with on != 0, every later dg_rhs, dg_rk_stage, dg_rk_step,
 * dg_rk_steps and dg_autotune of this context evaluates the weak form of eq.
 * weak_matrices_calc with quadrature exact for degree 3p -- a collapsed
 * Gauss product rule of q^2 points on the element and Gauss-Legendre with q
 * points on each face, q = floor((3p + 2) / 2) -- instead of the nodal
 * interpolants of the fluxes; G-bar_e is then the maximum over the face's
 * quadrature points.  Same boundary conditions, penalty and theta term.
 * Plain FP64 form (precision DG_FP64) and p = 1..6 only, else
 * DG_EUNSUPPORTED; such contexts cannot be batched.  Any time after
 * dg_create; on = 0 returns to the nodal evaluation.  The tables it needs are
 * built by dg_setup_host / dg_setup in every case ("oi_*" host tables). */
int dg_set_overintegration(dg_ctx* ctx, int on);

/* Sizes: number of elements K, nodes per element Np, nodes per face Nfp. */
int64_t dg_num_elements(const dg_ctx* ctx);
int dg_num_nodes(const dg_ctx* ctx);
int dg_num_face_nodes(const dg_ctx* ctx);

/* Host copy of a set-up table for inspection (after dg_setup_host).  name:
 * "r", "s" (Np), "Dr", "Ds", "M" (Np*Np, row-major; M the reference mass
 * matrix (V V^T)^-1), "LIFT", "LIFTr", "LIFTs"
 * (Np*3Nfp), "Fmask" (3*Nfp, as doubles), "wface" (3*Nfp face quadrature
 * weights), "geo" (K*16: rx ry sx sy, then per face nx ny Fscale
 * sigma_geo), "nbr" (K*3 neighbour element, as doubles), "nbr_face"
 * (K*3); the curved set S (dg_set_curved_elements): "curved_slot" (K: the
 * element's slot in S, or -1), "curved_elem" (|S|), "curved_node"
 * (|S|*5*Np: rx ry sx sy J at the nodes), "curved_face" (|S|*3*3Nfp: nx, ny,
 * sJ at the face nodes), "curved_P" (|S|*Np*Np: (M^K)^-1 M), "curved_area"
 * (|S|); the
 * over-integration tables (q points per direction, Nq = q^2): "oi_wq" (Nq
 * element weights), "oi_xg", "oi_wg" (q face points and weights), "oi_Iq",
 * "oi_Drq", "oi_Dsq" (Nq*Np: l_j and its r/s derivatives at the element
 * points), "oi_Wr", "oi_Ws" (Np*Nq: M^-1 (d l_i w)^T), "oi_If1" (q*Nfp: face
 * nodes to face points), "oi_Drf", "oi_Dsf" (3q*Np, face f's points in rows
 * f*q..), "oi_LIFTq", "oi_LIFTrq", "oi_LIFTsq" (Np*3q: M^-1 (l_i w)^T and with
 * d_r l_i, d_s l_i).  count must equal the table size; out is a host array of
 * that many doubles. */
int dg_get_host_table(const dg_ctx* ctx, const char* name, double* out, int64_t count);

/* Physical node coordinates, host arrays x[K*Np], y[K*Np] (element-major). */
int dg_get_nodes(const dg_ctx* ctx, double* x, double* y);

/* Right-hand side R = dU/dt = (M^K)^-1 R_K of eq. dg_on_K for every element,
 * in strong form (algebraically equal to the weak form): volume divergence
 * through Dr/Ds, face gather with Roe flux (eq. roe_flux), SIPG/IIPG viscous
 * flux with penalty (eq. ip_flux, eq. penalty_final), boundary ghosts
 * (Sec. 2.2.4), LIFT.  U, R: device arrays [K][4][Np] of doubles (must not
 * alias).  v_w: host pointer to the rigid-frame velocity (Sec. 2.1, eq. cnp).
 * Asynchronous on `stream`. */
int dg_rhs(dg_ctx* ctx, const double* U, double* R, const double v_w[2], void* stream);

/* One five-stage low-storage RK step (Alg. 1, coefficients of Carpenter &
 * Kennedy's 2N-storage (5,4) scheme), in place: U <- U(t + dt); K1 is the
 * second 2N register (device [K][4][Np], overwritten; need not be
 * initialised since A_1 = 0).  v_w fixed over the step (Alg. 3).  Uses the
 * library's scratch state buffer; asynchronous on `stream`. */
int dg_rk_step(dg_ctx* ctx, double* U, double* K1, double dt, const double v_w[2],
               void* stream);

/* nsteps RK steps (as dg_rk_step, v_w fixed), with the wall force (as
 * dg_force_device, the same bits) after each step written to
 * force_dev[3 n .. 3 n + 2] when force_dev (device, 3 nsteps doubles) is not
 * NULL.  The force after step n < nsteps - 1 is evaluated inside step
 * n + 1's stage launches: its partials by leading workgroups of the first,
 * whose input is that state, and their sum, in the same order, by a leading
 * wave of the second; the last step's by a launch of its own (the
 * over-integrated stage: one force launch per step).  The state alternates between U and the scratch
 * buffer from step to step, so it is copied back into U only when nsteps is
 * odd (dg_rk_step copies every step).  Asynchronous on `stream`. */
int dg_rk_steps(dg_ctx* ctx, double* U, double* K1, int nsteps, double dt, const double v_w[2],
                double* force_dev, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): dg_rk_steps
 * with the same arguments and results (bitwise), whose stage ping-pong state
 * and wall-force partials live in a static device array of 64 MiB per device
 * instead of the context's set-up buffers.  It calls no hipMalloc, hipFree or
 * allocating routine and no memset.  The state [K][4][Np] of doubles plus the
 * force partials must fit the 64 MiB (K * Np up to about 2 million), else
 * DG_EINVAL.  The context's device must be current.  Every call on a device
 * shares that device's array (which keeps the last call's contents): calls
 * that overlap on one device, on any streams, contexts or threads, race and
 * must be serialised by the caller.  Asynchronous on `stream`. */
int dg_rk_steps_noalloc(dg_ctx* ctx, double* U, double* K1, int nsteps, double dt,
                        const double v_w[2], double* force_dev, void* stream);

/* One RK stage: K1 <- a K1 + dt R(U_in); U_out <- U_in + b K1.  U_in and
 * U_out must not alias (neighbours read U_in).  Asynchronous. */
int dg_rk_stage(dg_ctx* ctx, const double* U_in, double* U_out, double* K1,
                double a, double b, double dt, const double v_w[2], void* stream);

/* Force and moment exerted by the fluid on the wall faces (Alg. 3, "Calculate
 * Aerodynamic Forces"): out[0..2] = (Fx, Fy, Mz) about the origin, the face-
 * quadrature integral of p+ n - tau(U^b, grad U+) n with n the fluid's
 * outward normal.  FP64, deterministic order.  Synchronises `stream`; out is
 * a host array of 3 doubles. */
int dg_force(dg_ctx* ctx, const double* U, const double v_w[2], double out[3], void* stream);

/* As dg_force, but asynchronous: the three doubles are written to the device
 * array out_dev on `stream` (for monitoring the force every step without a
 * host synchronisation). */
int dg_force_device(dg_ctx* ctx, const double* U, const double v_w[2], double* out_dev,
                    void* stream);

/* Time step from the CFL condition (eq. cfl_general; Alg. 3, "Calculate Time
 * Step"): out[0] = Lambda, the bound of eq. rayleigh_bound on the numerical
 * range of the operator at the state U (binary64 [K][4][Np], device) with
 * wall velocity v_w,
 *   Lambda = max_K (3/2 C_inv,2(K) G_K + 3 C_inv,K (3 sigma_K + beta_K) + beta'_K),
 * C_inv,K = Np max_e |e|/|K|, C_inv,2(K) = C_grad p^4 / rho_K^2 (rho_K the
 * inscribed radius, C_grad the generic constant of the inverse estimate),
 * sigma_K the largest face penalty of K as the right-hand side forms it,
 * beta_K = max over K's nodes of |v - v_w| + c, beta'_K = 1/2 max |div v|
 * (nodal derivative of the interpolated velocity), G_K the largest
 * directional norm ||e_a^T G e_a||_2 (a = x, y) over the nodes of K and its
 * face neighbours; out[1] = C_cfl / Lambda.  C_cfl > 0 and C_grad >= 0, else
 * DG_EINVAL; a non-finite bound gives DG_ENONFINITE (an unphysical state:
 * negative pressure or density, NaN).  out is a host array of 2 doubles.
 * Uses the context's work buffer (6K + 1 doubles, set up by dg_setup), so
 * two calls of one context must not overlap on different streams;
 * synchronises `stream`. */
int dg_cfl_time_step(dg_ctx* ctx, const double* U, const double v_w[2], double C_cfl, double C_grad,
                     double out[2], void* stream);

/* Host Newmark-beta step (beta 1/4, gamma 1/2) of M y'' + C y' + K y = F
 * (eq. 1dof_oscillator): state[3] = (y, y', y'') at t, updated to t + dt
 * with the load F_new. */
int dg_newmark_step(double state[3], double F_new, double dt, double M, double C, double K);

/* ---- Launch shape and its autotuner --------------------------------------
 * The stage kernel's launch shape: waves per workgroup (2 or 4; each wave
 * owns tiles of 4 elements, the workgroup shares the operator fragments held
 * in LDS; 0 = the default for the order and precision) and the grid (0 =
 * persistent: the resident workgroups stride over the tiles, 1 = one tile per
 * wave, 2 or 3 = that many tiles per wave, within the resident workgroups).
 * Results do not depend on the shape (bitwise).  Host only. */
int dg_set_tuning(dg_ctx* ctx, int waves, int grid);
int dg_get_tuning(const dg_ctx* ctx, int* waves, int* grid);

/* Time every launch shape on this context's mesh (two sweeps over the
 * shapes, reps launches of a K1-reading RK stage per shape and sweep, each
 * shape's best kept; reading U, a device state [K][4][Np], writing only
 * library scratch) and keep the fastest.  With cache_path non-NULL, a matching entry of that
 * JSON-lines file (same device architecture, order, precision and element
 * count within a factor 2) is used instead of timing, and a new measurement
 * is appended to it.  Allocates a temporary device register; synchronises
 * `stream`.  *best_us (may be NULL) receives the chosen shape's time per
 * launch in microseconds (0 when taken from the cache). */
int dg_autotune(dg_ctx* ctx, const double* U, int reps, const char* cache_path, void* stream,
                double* best_us);

/* ---- Batches ---------------------------------------------------------------
 * A batch advances n set-up contexts (same precision and HIP device; orders,
 * meshes and physics may differ; e.g. the instances of a parameter sweep)
 * together: every RK stage of every instance runs in one launch (instances
 * grouped by order, each group owning a range of workgroups), and the five
 * stages of a step are captured once as a HIP graph and replayed.  Per-step
 * dt and v_w of each instance are uploaded into device memory before each
 * replay, so the graph stays valid.  The batch owns each instance's state
 * (two ping-pong buffers, the current one alternating from step to step) and
 * its K1 register; results equal those of dg_rk_step on each context
 * (bitwise).  The contexts must outlive the batch and must not be set up
 * again meanwhile. */
typedef struct dg_batch dg_batch;

/* Create a batch of the n contexts ctxs[0..n-1] (all set up by dg_setup,
 * each at most once: DG_EINVAL for a repeated context).  Allocates device
 * memory (3 states per instance) and pinned host memory. */
int dg_batch_create(dg_ctx* const* ctxs, int n, dg_batch** out);

/* Copy instance i's state in from / out to a device array [K_i][4][Np_i]
 * (asynchronous on `stream`). */
int dg_batch_set_state(dg_batch* b, int i, const double* U, void* stream);
int dg_batch_get_state(dg_batch* b, int i, double* U, void* stream);

/* One LSERK step of every instance: dt[i] and v_w[2i], v_w[2i+1] are host
 * arrays of n and 2n doubles.  Asynchronous on `stream` (the previous step's
 * parameter upload is waited for before the pinned staging area is
 * rewritten). */
int dg_batch_rk_step(dg_batch* b, const double* dt, const double* v_w, void* stream);

/* One LSERK step of every instance on caller-owned device arrays: U[i] and
 * K1[i] (arrays of n device pointers, each [K_i][4][Np_i] FP64, distinct
 * from each other and across instances), dt and v_w as dg_batch_rk_step.
 * The same launches and graph as dg_batch_rk_step (the item table is
 * rewritten on `stream` to point at these arrays; the batch's second state
 * buffer of each instance is the stage ping-pong partner, and the result is
 * copied back into U[i] at the end, as dg_rk_step does), so results equal
 * dg_rk_step on each context bitwise.  The batch-owned states are not
 * preserved by this call (load them again with dg_batch_set_state before
 * dg_batch_rk_step, dg_batch_force or dg_batch_coupled_step).  Asynchronous
 * on `stream`; DG_EINVAL for a NULL, shared or repeated array or a
 * non-finite dt / v_w. */
int dg_batch_rk_step_states(dg_batch* b, double* const* U, double* const* K1, const double* dt,
                            const double* v_w, void* stream);

/* Force and moment on each instance's wall faces (as dg_force), out a host
 * array of 3n doubles.  Synchronises `stream`. */
int dg_batch_force(dg_batch* b, const double* v_w, double* out, void* stream);

/* One step of the weakly coupled fluid-structure loop (Alg. 3) for every
 * instance, each a 1-DOF oscillator M y'' + C y' + K y = s F_y
 * (eq. 1dof_oscillator, Sec. 3.3.1): the host Newmark step (as
 * dg_newmark_step) under the last lift, the wall velocity for the step
 * v_w = (0, (y_new - y)/dt), one RK step of the whole batch (as
 * dg_batch_rk_step) and the forces on the new states (as dg_batch_force).
 * Host arrays: osc n x 4 (M, C, K, s), body n x 3 (y, y', y'') updated in
 * place, F n x 3 whose lifts F[3i+1] are read and which receives the new
 * forces, dt n doubles, v_w_out n x 2 doubles receiving the wall velocities
 * (may be NULL).  Synchronises `stream`.  DG_EINVAL (nothing changed) for a
 * NULL array, a non-positive dt or a singular oscillator; after a failure
 * of the step itself body may already hold the new displacements. */
int dg_batch_coupled_step(dg_batch* b, const double* osc, double* body, double* F,
                          const double* dt, double* v_w_out, void* stream);

/* Launch shape: mode 0 one launch per stage for all instances, 1 one launch
 * per order group (in a kernel sized for that order); waves as
 * dg_set_tuning, grid 0 persistent or 1 one tile per wave; use_graph 0 launches the
 * stages directly instead of replaying the captured graph. */
int dg_batch_configure(dg_batch* b, int mode, int waves, int grid, int use_graph);

/* The batch's current launch shape (as dg_batch_configure takes it; after
 * dg_batch_autotune, the one it picked).  Any pointer may be NULL. */
int dg_batch_get_config(const dg_batch* b, int* mode, int* waves, int* grid, int* use_graph);

/* Time every (mode, waves, grid) on the batch (reps first-stage launches
 * each; the states are left unchanged, K1 is overwritten) and keep the
 * fastest.  Synchronises `stream`.  *best_us (may be NULL) receives its time
 * per stage in microseconds. */
int dg_batch_autotune(dg_batch* b, int reps, void* stream, double* best_us);

/* Message of the last failing call on b; with b NULL, of the last failed
 * dg_batch_create (which releases everything it allocated and sets *out to
 * NULL). */
const char* dg_batch_last_error(const dg_batch* b);

/* Release the batch (not its contexts).  NULL is a no-op. */
void dg_batch_destroy(dg_batch* b);

/* ---- Learned closure --------------------------------------------------------
 * A per-element network corrects an order-lo solution toward the order-hi
 * one (a spec extension; the paper has no closure).  A sample of
 * element k is x = [Pi_lo(U - U_inf) (Np_lo nodes x 4 fields, field-major),
 * rx, ry, sx, sy]; its target the part of the order-hi state that order lo
 * cannot represent, t = U_hi - I Pi_lo U_hi (Np_hi x 4, field-major), where
 * Pi_lo is the L2 projection onto degree <= lo at the order-lo nodes and I
 * the interpolation back to the order-hi nodes.  The corrected state is
 * I U_lo + y.  The network is y = W3 g(W2 g(W1 x + b1) + b2) + b3 (g the
 * exact-erf GELU) on per-column normalised x and t, trained on the mean
 * squared error with Adam; its products run on the matrix cores with
 * bfloat16 operands and FP32 accumulation, its parameters are FP32. */
typedef struct dg_mlp dg_mlp;
typedef struct dg_closure dg_closure;

/* Network of widths n_in (1..64) -> n_hidden (64 or 128) -> n_hidden ->
 * n_out (1..64), with buffers for batches of up to max_batch samples.
 * Parameters start at zero; set them with dg_mlp_set_params. */
int dg_mlp_create(int n_in, int n_hidden, int n_out, int64_t max_batch, dg_mlp** out);
int64_t dg_mlp_num_params(const dg_mlp* m);

/* Parameters as one host FP32 vector W1 b1 W2 b2 W3 b3 (W_l row-major
 * [width out][width in]).  Setting them resets the Adam state.  Both calls
 * synchronise the device. */
int dg_mlp_set_params(dg_mlp* m, const float* host, int64_t count);
int dg_mlp_get_params(dg_mlp* m, float* host, int64_t count);
/* Gradient of the last dg_mlp_backward, same layout (synchronises). */
int dg_mlp_get_grad(dg_mlp* m, float* host, int64_t count);

/* Per-column normalisation: inputs (x - in_mean) / in_std, targets
 * (t - out_mean) / out_std; outputs are returned denormalised.  Host arrays
 * of n_in and n_out floats (standard deviations positive). */
int dg_mlp_set_normalization(dg_mlp* m, const float* in_mean, const float* in_std,
                             const float* out_mean, const float* out_std);

/* Y[b][0..n_out) = network(X[b][0..n_in)) for b < B: X device FP32 with row
 * stride ldx, Y device FP32 with row stride ldy.  Asynchronous. */
int dg_mlp_forward(dg_mlp* m, const float* X, int64_t ldx, int64_t B, float* Y, int64_t ldy,
                   void* stream);

/* Gradient of the mean squared error (over B x n_out normalised entries)
 * against raw targets T (device FP32, row stride ldt), kept for dg_mlp_adam
 * (partials per workgroup summed in a fixed order: reproducible).  With loss
 * non-NULL the loss is returned on the host (synchronises).  For
 * n_in <= 32, H = 128 and n_out <= 64 the step runs as one fused kernel
 * (forward, loss, backward and weight gradients per 16-row tile, activations
 * in registers and LDS; HBM traffic the inputs and targets) unless
 * dg_mlp_set_schedule chose the layer-by-layer schedule. */
/* Training schedule of dg_mlp_backward: 1 (the default) the fused kernel
 * where it is built, 0 layer by layer (each layer's activations stored and
 * re-read).  Both give the same gradient up to the order of the sums and the
 * FP32 (fused) or bfloat16 (stored) GELU derivatives.  DG_EINVAL otherwise. */
int dg_mlp_set_schedule(dg_mlp* m, int fused);

int dg_mlp_backward(dg_mlp* m, const float* X, int64_t ldx, const float* T, int64_t ldt,
                    int64_t B, double* loss, void* stream);

/* One Adam step (Kingma & Ba, bias-corrected) with the last gradient;
 * refreshes the bfloat16 weight copies.  Asynchronous. */
int dg_mlp_adam(dg_mlp* m, float lr, float beta1, float beta2, float eps, void* stream);

const char* dg_mlp_last_error(const dg_mlp* m);
void dg_mlp_destroy(dg_mlp* m);

/* Mean and standard deviation (population) of each of the first cols (<= 64)
 * columns of a device FP32 array of rows x ld; host outputs.  Allocates a
 * temporary device buffer; synchronises. */
int dg_column_stats(const float* A, int64_t rows, int64_t ld, int cols, double* mean,
                    double* stdev, void* stream);

/* Order-change maps between two set-up contexts on the same mesh, lo->N <
 * hi->N (U_inf of hi).  The contexts must outlive the closure. */
int dg_closure_create(const dg_ctx* lo, const dg_ctx* hi, dg_closure** out);
int dg_closure_sizes(const dg_closure* c, int* n_features, int* n_targets);
/* Samples of every element into X (device FP32, row stride ldx >=
 * n_features) from an order-hi state (from_hi = 1, restricted), an order-lo
 * state (from_hi = 0), or the free stream (from_hi = 2: the state columns
 * zero, U unused and may be NULL).  Asynchronous. */
int dg_closure_features(dg_closure* c, const double* U, int from_hi, float* X, int64_t ldx,
                        void* stream);
/* Targets of every element from an order-hi state (T row stride >=
 * n_targets).  Asynchronous. */
int dg_closure_targets(dg_closure* c, const double* U_hi, float* T, int64_t ldt, void* stream);
/* U_lo = Pi_lo U_hi, the order-lo state of an order-hi one (device
 * [K][4][Np_lo]).  Asynchronous. */
int dg_closure_restrict(dg_closure* c, const double* U_hi, double* U_lo, void* stream);
/* U_hi = I U_lo + Y - Y0 (Y may be NULL: interpolation only; Y0, the
 * network's output for the free-stream samples, may be NULL).  With Y0 the
 * reconstruction of a free-stream element is exactly the interpolation.
 * Asynchronous. */
int dg_closure_apply(dg_closure* c, const double* U_lo, const float* Y, const float* Y0,
                     int64_t ldy, double* U_hi, void* stream);
/* The order-lo solve corrected toward the order-hi one (a learned m-step
 * corrector, an extension not in the paper): every m steps of the order-lo
 * solver, U_lo += net(x) - net(x0) with x the sample of U_lo and x0 the
 * free stream's (so that a free-stream element is left alone, as both
 * solvers leave it), the network trained on the
 * drift of m order-lo steps from the restriction of an order-hi state,
 * t = Pi_lo U_hi(t + m dt) - Phi_lo^m(Pi_lo U_hi(t)).  Rows of 4 Np_lo values
 * (field-major, Np_lo nodes per field; n_features - 4 of dg_closure_sizes).
 * dg_closure_drift_targets: T[k] = U_ref - U_lo per element (device order-lo
 * states [K][4][Np_lo], FP64 difference rounded to FP32); dg_closure_correct:
 * U_lo += Y - Y0 (device FP32 rows of one row stride ldy; Y0 may be NULL).
 * Asynchronous. */
int dg_closure_drift_targets(dg_closure* c, const double* U_ref, const double* U_lo, float* T,
                             int64_t ldt, void* stream);
int dg_closure_correct(dg_closure* c, const float* Y, const float* Y0, int64_t ldy, double* U_lo,
                       void* stream);
const char* dg_closure_last_error(const dg_closure* c);
void dg_closure_destroy(dg_closure* c);

/* Message of the last failing call on ctx ("" if none).  Valid until the next
 * call on ctx.  ctx may be NULL (then a message about creation failures). */
const char* dg_last_error(const dg_ctx* ctx);

/* Release every host and device resource of ctx.  NULL is a no-op. */
void dg_destroy(dg_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* DGMI_H */
