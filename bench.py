"""Throughput of the DG right-hand side + low-storage RK stage on one MI355X.

Workload (default, cylinder20k): flow past a unit-diameter cylinder, O-grid
of 80 x 128 cells (radial ratio 1.05, wall r = 0.5, far field r = 30) split
into K = 20480 triangles, p = 4 (Np = 15), Re = 100, M = 0.2, SIPG, paper
penalty, free stream plus seeded 1e-3 uniform noise per node and field.
The default run also measures the rest of the metric's range and the
out-of-cache mesh, each with plain FP64 beside it, and reports them as
sub-objects of the same line: "orders" (cylinder20k at p = 5 and 6) and
"cylinder327k" (the same O-grid refined 4 x 4, K = 327,680, p = 4, states
beyond the last-level cache).
Other workloads (--workload): cylinder327k, periodic51k (160x160x2 periodic
triangles, p = 6, three seeded Fourier modes of amplitude 1e-2), viv16 (16
elastically mounted cylinders, K = 5k-31k each, p in {4, 5, 6}, U* in [3, 8],
coupled to a host Newmark step every step, advanced as one batch) and
closure20k (the learned closure: order-4 snapshots, bfloat16 training
throughput, gain at Re = 120).

A step is one pass of the hot path: the five fused RHS + stage launches of
one LSERK step and the wall-force integral (viv16: plus the host Newmark step
and the new wall velocity, as the coupling needs).  value = DOF-updates/s =
sum 4 Np K x 5 x steps / time of the K timed steps (HIP events), inputs
resident in HBM.

Forms (--form): fp64 (plain, every step binary64), fp64-pert and fp32-pert
(the right-hand side on U - U_inf with cancellation-free flux differences, in
binary64 or binary32; the RK registers stay binary64), bf16-ops.  Plain FP64
is run beside the chosen form from the same initial state for the same
steps; the stated error is the per-field L2 norm (with the mass matrix,
sum_K J_K dU^T M dU) of the difference of the final states, relative to that
of the plain FP64 state's deviation from U_inf, largest over the four fields.

Roofline: the stage kernel's average launch time (HIP events on its stream)
against HBM (algorithmic bytes), the matrix cores (operator products at the
form's matrix peak) and the vector ALU (pointwise flops), the binding roof
reported; measured HBM traffic per launch from the committed counter
summaries when they match the current kernel sources, else null.
cpu_baseline: the FP64 NumPy oracle on the host (RHS + stage update per
order, one thread and the default pools, host core count).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--p P] [--form F]
                       [--workload W] [--quick] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "DG RHS DOF-updates/s at p=4–6, chosen form vs plain FP64 at stated L2 err"
METRIC_OI = "DG RHS DOF-updates/s, over-integrated (degree-3p quadrature) FP64 vs the nodal FP64 stage"
# MI355X published peaks: HBM3E 8 TB/s; dense matrix cores FP64 78.6, FP32
# 157.3, bfloat16 2500 TFLOP/s; vector ALU 256 CUs x 4 SIMDs x 16 lanes x 2
# (FMA) x 2.4 GHz = 78.6 TFLOP/s for FP64 and for FP32 without packed
# instructions (packed FP32 is not used in this build)
HBM_PEAK_GBS = 8000.0
VALU_PEAK_TFLOPS = 78.6
MFMA_PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}
FORMS = {"fp64": 0, "fp64-pert": 1, "fp32-pert": 2, "bf16-ops": 3}
MFMA_DTYPE = {"fp64": "f64", "fp64-pert": "f64", "fp32-pert": "f32", "bf16-ops": "bf16"}
PROFILES = os.path.join(ROOT, "profiles")


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def algorithmic_bytes_per_element(Np):
    # K0 read, K1 read, K1 write, K0 write (4 x 4 Np doubles) + geometry
    # (16 doubles) + packed connectivity (3 int32)
    return 4 * 4 * Np * 8 + 16 * 8 + 3 * 4


def gemm_flops_per_element(Np, Nfp):
    """Operator products of one RHS per element (matrix cores): gradient and
    divergence 2 x 16 Np^2 (D_r, D_s on 4 fields, both ways), the three lifts
    24 Np (3 Nfp)."""
    return 32 * Np * Np + 24 * Np * 3 * Nfp


def pointwise_flops_per_element(Np, Nfp):
    """Pointwise FP64 flops of one RHS + stage per element (vector ALU),
    counted from the method: volume-node flux 75 Np, face nodes (16 Np + 460)
    per node of the 3 Nfp (neighbour gradient at the node 16 Np; two
    ||n^T G n||_2 ~200, two viscous normal fluxes ~80, Roe ~110, penalty and
    residual ~20, theta term ~50), stage update 16 Np."""
    NF = 3 * Nfp
    return 75 * Np + (16 * Np + 460) * NF + 16 * Np


def algorithmic_flops_per_element(Np, Nfp):
    return gemm_flops_per_element(Np, Nfp) + pointwise_flops_per_element(Np, Nfp)


def roofline(Np, Nfp, K, t_launch, form, traffic=None, overint=False):
    """The stage kernel against each roof it could be bound by -- HBM
    (algorithmic bytes at 8 TB/s), the matrix cores (operator products at the
    form's matrix peak) and the vector ALU (pointwise flops at 78.6 TFLOP/s),
    each taken alone as a lower bound on the launch time -- and the binding
    one (the largest bound).  frac = that bound / the measured launch time."""
    nbytes = algorithmic_bytes_per_element(Np) * K
    if overint:
        gemm, pw = (x * K for x in oi_flops_per_element(Np, Nfp))
    else:
        gemm = gemm_flops_per_element(Np, Nfp) * K
        pw = pointwise_flops_per_element(Np, Nfp) * K
    mdt = MFMA_DTYPE[form]
    t = {"hbm": nbytes / (HBM_PEAK_GBS * 1e9),
         "mfma": gemm / (MFMA_PEAK_TFLOPS[mdt] * 1e12),
         "alu": pw / (VALU_PEAK_TFLOPS * 1e12)}
    bound = max(t, key=t.get)
    if bound == "hbm":
        achieved, peak, unit = nbytes / t_launch / 1e9, HBM_PEAK_GBS, "GB/s"
    elif bound == "mfma":
        achieved, peak, unit = gemm / t_launch / 1e12, MFMA_PEAK_TFLOPS[mdt], "TFLOP/s"
    else:
        achieved, peak, unit = pw / t_launch / 1e12, VALU_PEAK_TFLOPS, "TFLOP/s"
    return {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak, "traffic": traffic,
            "avg_launch_us": t_launch * 1e6,
            "bytes_per_launch": nbytes, "gemm_flops_per_launch": gemm,
            "pointwise_flops_per_launch": pw,
            "frac_hbm": t["hbm"] / t_launch,
            "frac_mfma_%s" % mdt: t["mfma"] / t_launch,
            "frac_valu": t["alu"] / t_launch}


def closure_bytes_per_sample(n_in, H, n_out):
    """HBM bytes per sample of one training step of the layer-by-layer
    schedule: every stored quantity written once and read once by each
    consumer.  Inputs FP32 (n_in) and targets FP32 (n_out); the normalised
    inputs (padded to 16), activations, GELU derivatives and back-propagated
    gradients bfloat16 (output gradient padded to 64).  Forward: read x, write
    x_n, g1, h1; read h1, write g2, h2; read h2 and t, write dy.  Backward:
    read dy and g2, write dz2; read dz2 and g1, write dz1.  Weight gradients:
    read (dz1, x_n), (dz2, h1), (dy, h2).  The per-step weight traffic and the
    weight-gradient partials do not grow with the batch and are left out."""
    in_pad, out_pad = (n_in + 15) // 16 * 16, 64
    fwd = 4 * n_in + 2 * in_pad + 2 * H + 2 * H + 2 * H + 2 * H + 2 * H + 2 * H + 4 * n_out + 2 * out_pad
    bwd = 2 * out_pad + 2 * H + 2 * H + 2 * H + 2 * H + 2 * H
    wgr = 2 * H + 2 * in_pad + 2 * H + 2 * H + 2 * out_pad + 2 * H
    return fwd + bwd + wgr


def closure_roofline(bytes_sample, flops_sample, samples, t):
    """A training run against HBM (its algorithmic bytes) and the bfloat16
    matrix cores (its flops), each a lower bound on the time; the larger
    binds."""
    tb = bytes_sample * samples / (HBM_PEAK_GBS * 1e9)
    tf = flops_sample * samples / (MFMA_PEAK_TFLOPS["bf16"] * 1e12)
    if tb >= tf:
        bound, ach, peak, unit = "hbm", bytes_sample * samples / t / 1e9, HBM_PEAK_GBS, "GB/s"
    else:
        bound, ach, peak, unit = "mfma", flops_sample * samples / t / 1e12, MFMA_PEAK_TFLOPS["bf16"], "TFLOP/s"
    return {"bound": bound, "achieved": ach, "peak": peak, "unit": unit, "frac": ach / peak,
            "traffic": None,
            "kernel": "train_kernel (forward, loss, backward, weight gradients) + "
                      "reduce_parts_kernel + adam_kernel (one training step)",
            "bytes_per_sample": bytes_sample, "flops_per_sample": flops_sample,
            "frac_hbm": tb / t, "frac_mfma_bf16": tf / t}


def oi_flops_per_element(Np, Nfp):
    """(operator products, pointwise) FP64 flops of one over-integrated RHS +
    stage per element (q points per direction, q^2 element points, 3q face
    points), counted from the method: U, d_r U, d_s U at the element points
    3 x 8 Nq Np, weighted divergence 2 x 8 Np Nq, three lifts 24 Np 3q on the
    matrix cores; volume flux 75 per element point, per face point both
    sides' value and gradient 2 (8 Nfp + 16 Np) plus the face fluxes 460 as in
    the nodal count, stage update 16 Np on the vector ALU."""
    p = Nfp - 1
    q = (3 * p + 2) // 2
    Nq, NG = q * q, 3 * q
    return (24 * Nq * Np + 16 * Np * Nq + 24 * Np * NG,
            75 * Nq + (32 * Np + 16 * Nfp + 460) * NG + 16 * Np)


def kernel_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "dg_physics.h"):
        with open(os.path.join(ROOT, "paper_2508_17917_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, p, form):
    """HBM bytes per stage launch from the committed rocprofv3 counter
    summaries (FETCH_SIZE and WRITE_SIZE, each scaled by its reading for a
    plain device copy of known size): a line
      traffic: workload=W p=P form=F sources=H bytes=B
    in a profiles/*.md file.  None unless one matches this workload, order,
    form and the current kernel sources (counters of other sources do not
    describe this kernel)."""
    import glob
    import re
    want = kernel_sources_hash()
    pat = re.compile(r"traffic: workload=(\S+) p=(\d+) form=(\S+) sources=(\S+) bytes=([0-9.eE+]+)")
    for path in sorted(glob.glob(os.path.join(PROFILES, "*.md"))):
        with open(path) as fh:
            for line in fh:
                m = pat.search(line)
                if (m and m.group(1) == workload and int(m.group(2)) == p and m.group(3) == form
                        and m.group(4) == want):
                    return float(m.group(5))
    return None


def cpu_baseline(w, orders, overint=False):
    """The oracle as it stands (NumPy FP64) on the host cores: per order, one
    weak-form RHS of the full workload followed by its LSERK stage update
    (K1 <- A_2 K1 + dt R, U <- U + B_2 K1), timed with the BLAS/OpenMP pools
    limited to one thread and at their defaults.  DOF-updates/s = 4 Np K per
    RHS + stage / wall time.  The oracle's arithmetic is NumPy einsum and
    elementwise work, which runs on one thread either way."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits

    import meshgen as mg
    from oracle.dg import LSERK_A, LSERK_B, DGOracle, Physics
    from oracle.mesh import Mesh
    from oracle.nodes import RefElement

    host_cores = len(os.sched_getaffinity(0))
    pools = sorted({i.get("num_threads", 1) for i in threadpool_info()}) or [1]
    m = w["mesh"]
    per = {}
    total = 0.0
    for p in orders:
        ref = RefElement(p)
        mesh = Mesh(ref, m["VX"], m["VY"], m["EToV"], m["face_tag"], m["period"])
        dg = DGOracle(mesh, Physics(gamma=w["gamma"], Pr=w["Pr"], mu=w["mu"], theta=w["theta"],
                                    penalty_mode=w["penalty_mode"], C_pen=w["C_pen"],
                                    U_inf=w["U_inf"]))
        if overint:
            from oracle.overint import DGOracleOI
            dg = DGOracleOI(dg.mesh, dg.phys)
        U = mg.noisy_free_stream((4, ref.Np, mesh.K), w["U_inf"], mg.rng_for(1))
        K1 = np.zeros_like(U)
        dofs = 4 * ref.Np * mesh.K
        rates = {}
        for label, lim in (("1_thread", 1), ("default_threads", None)):
            with threadpool_limits(limits=lim):
                t0 = time.perf_counter()
                K1n = LSERK_A[1] * K1 + 1e-7 * dg.rhs(U)
                U1 = U + LSERK_B[1] * K1n
                el = time.perf_counter() - t0
            assert np.isfinite(U1).all()
            rates[label] = dofs / el
            total += el
        per[str(p)] = {"1_thread": rates["1_thread"], "default_threads": rates["default_threads"],
                       "K": mesh.K, "Np": ref.Np}
    head = per[str(orders[0])]
    return {"value": head["1_thread"], "unit": "DOF-updates/s", "cores": 1, "kind": "oracle",
            "sample": "one %sweak-form RHS + LSERK stage update of the full K=%d workload per "
                      "order p=%s, NumPy FP64, 1 thread and the default pools (%.1f s in all); "
                      "value: p=%d, 1 thread"
                      % ("over-integrated " if overint else "", head["K"],
                         ",".join(str(q) for q in orders), total, orders[0]),
            "host_cores": host_cores, "default_pool_threads": pools[-1],
            "per_order": per}


def stable_dt(mesh, p, mu, rho=1.0, C=0.01):
    """A time step inside the viscous/penalty stability limit, C h0^2 / (nu
    (p+1)^4) with h0 the shortest element edge (measured limit near 3e-7 for
    cylinder20k at p = 4, where this gives 6.7e-8)."""
    import numpy as np
    VX, VY, E = mesh["VX"], mesh["VY"], np.asarray(mesh["EToV"])
    h0 = min(np.hypot(VX[E[:, a]] - VX[E[:, b]], VY[E[:, a]] - VY[E[:, b]]).min()
             for a, b in ((0, 1), (1, 2), (2, 0)))
    return C * h0 * h0 / ((mu / rho) * (p + 1) ** 4)


def mass_norms(solver, D):
    """Per-field (sum_K J_K d^T M d)^(1/2) of a device state difference D."""
    import numpy as np
    Np, K = solver.Np, solver.K
    M = solver.table("M").reshape(Np, Np)
    geo = solver.table("geo").reshape(K, 16)
    J = 1.0 / (geo[:, 0] * geo[:, 3] - geo[:, 1] * geo[:, 2])
    d = D.cpu().numpy()
    return np.sqrt(np.einsum("kcn,nm,kcm,k->c", d, M, d, J))


def make_solver(w, p, mesh, precision, overint=False, curved=None):
    from paper_2508_17917_amd import Solver
    return Solver(p, mesh, gamma=w["gamma"], Pr=w["Pr"], mu=w["mu"], theta=w["theta"],
                  penalty_mode=w["penalty_mode"], C_pen=w["C_pen"], U_inf=w["U_inf"],
                  precision=precision, overintegration=overint, curved=curved)


def curved_bytes_per_element(Np, Nfp):
    """Algorithmic HBM bytes per element of the curved set: the state read,
    K1 read and written, the new state written (4 x 4 Np doubles), the node
    table (rx, ry, sx, sy, J: 5 Np), the face table (nx, ny, sJ: 9 Nfp), P
    (Np^2), the penalty factors and connectivity (16 doubles, 3 int32)."""
    return 4 * 4 * Np * 8 + 5 * Np * 8 + 9 * Nfp * 8 + Np * Np * 8 + 16 * 8 + 3 * 4


def stage_time(s, U, dt, stream, nl=100):
    """Average duration of the stage kernel alone (HIP events on its stream),
    on scratch copies so the caller's state is left alone."""
    import torch
    Ua, Ub = U.clone(), torch.empty_like(U)
    Kb = torch.zeros_like(U)
    for _ in range(5):
        s.rk_stage(Ua, Ub, Kb, -0.4, 0.3, dt, stream=stream)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(nl):
        s.rk_stage(Ua, Ub, Kb, -0.4, 0.3, dt, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / nl


def settle(s, U, dt, stream, ms=50.0, max_launches=4000):
    """Set-up, before the autotuner and the warmup steps: stage launches on
    scratch copies until `ms` of GPU time have passed.  After an idle host
    phase the GPU needs some milliseconds of continuous work before stage
    launches run at their steady speed (the first 5-10 ms run up to 5 % slower),
    so a short timed region right after set-up would time that ramp rather
    than the kernel, and the autotuner would compare shapes at two speeds."""
    import torch
    Ua, Ub = U.clone(), torch.empty_like(U)
    Kb = torch.zeros_like(U)
    done, n = 0.0, 0
    while done < ms and n < max_launches:
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(25):
            s.rk_stage(Ua, Ub, Kb, -0.4, 0.3, dt, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        done += e0.elapsed_time(e1)
        n += 25


def run_single(w, U0, precision, steps, warmup, dt, overint=False, curved=None):
    """One mesh: warmup + steps LSERK steps, each followed by the wall-force
    integral into device memory (one library call per phase; the state
    alternates between two buffers, so no per-step copy).  Returns (final
    state, timed seconds, stage kernel seconds, solver)."""
    import torch
    s = make_solver(w, w["p"], w["mesh"], precision, overint, curved)
    U = U0.clone()
    K1 = torch.zeros_like(U)
    F = torch.zeros((warmup + steps, 3), dtype=torch.float64, device=U.device)
    stream = torch.cuda.current_stream()
    # launch shape from the autotuner (set-up, outside the timed region)
    settle(s, U, dt, stream)
    s.autotune(U, reps=20, stream=stream)
    s.rk_steps(U, K1, warmup, dt, force=F[:warmup], stream=stream)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    s.rk_steps(U, K1, steps, dt, force=F[warmup:], stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    t_steps = ev0.elapsed_time(ev1) / 1e3
    t_launch = stage_time(s, U, dt, stream)
    return U, t_steps, t_launch, s


def tuning_of(s):
    w, g = s.get_tuning()
    return "%d waves/workgroup, %s" % (w, ("persistent grid", "one tile per wave",
                                            "two tiles per wave", "three tiles per wave")[g])


def run_viv(cases, phys, states, precision, steps, warmup, dts, batched):
    """Coupled sweep: per step Newmark under the last force, v_w = dy/dt, one
    RK step of every instance (batched: one launch per stage for all; else one
    launch per stage and instance), forces.  Returns (states, timed seconds,
    stage seconds or None, solvers, batch launch shape or None)."""
    import numpy as np
    import torch

    from paper_2508_17917_amd import _lib as L
    from paper_2508_17917_amd.viv import VIVSweep, oscillator
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    if batched:
        sw = VIVSweep([dict(c) for c in cases], precision=precision, **phys)
        for i, U in enumerate(states):
            sw.set_state(i, U)
        t_launch = sw.batch.autotune(reps=20) / 1e6
        mode, waves, grid, _ = sw.batch.get_config()
        shape = "%s, %d waves/workgroup, %s" % (
            ("one launch per stage for all orders", "one launch per order group and stage")[mode],
            waves, ("persistent grid", "one tile per wave")[grid])
        sw.update_forces()
        for _ in range(warmup):
            sw.step(dts)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(steps):
            sw.step(dts)
        ev1.record(stream)
        torch.cuda.synchronize()
        out = [sw.get_state(i) for i in range(len(cases))]
        torch.cuda.synchronize()
        return out, ev0.elapsed_time(ev1) / 1e3, t_launch, sw.solvers, shape
    U_inf = np.asarray(phys["U_inf"])
    solvers = [make_solver(dict(phys), c["p"], c["mesh"], precision) for c in cases]
    Us = [U.clone() for U in states]
    K1s = [torch.zeros_like(U) for U in Us]
    v_inf = float(np.hypot(U_inf[1], U_inf[2]) / U_inf[0])
    coef = [oscillator(c["U_star"], c["m_star"], c["xi"], v_inf, U_inf[0]) for c in cases]
    body = np.zeros((len(cases), 3))
    vw = np.zeros((len(cases), 2))
    F = np.array([s.force(U) for s, U in zip(solvers, Us)])

    def step():
        for i, s in enumerate(solvers):
            M, C, Kr, inv_m = coef[i]
            st = L.dg_newmark_step(body[i], F[i, 1] * inv_m, dts[i], M, C, Kr)
            vw[i] = (0.0, (st[0] - body[i, 0]) / dts[i])
            body[i] = st
            s.rk_step(Us[i], K1s[i], dts[i], v_w=vw[i], stream=stream)
            F[i] = s.force(Us[i], v_w=vw[i], stream=stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    return Us, ev0.elapsed_time(ev1) / 1e3, None, solvers, None


def rel_l2(solvers, got, ref, U_inf):
    """Largest over fields of ||got - ref||_M / ||ref - U_inf||_M, summed over
    instances."""
    import numpy as np
    import torch
    num = np.zeros(4)
    den = np.zeros(4)
    for s, a, b in zip(solvers, got, ref):
        uinf = torch.tensor(np.asarray(U_inf), dtype=torch.float64, device=b.device).view(1, 4, 1)
        num += mass_norms(s, a - b) ** 2
        den += mass_norms(s, b - uinf) ** 2
    return float(np.sqrt(num / np.maximum(den, 1e-300)).max())


def run_closure(args):
    """Learned closure on cylinder20k: order-4 runs of impulsively started
    flows at seeded Re in [60, 150] (FP64 plain form), snapshots every m = 40
    steps over 10^4 steps per Re; per snapshot the reconstruction samples of
    the order-4 state and the corrector samples of the drift of 40 order-2
    steps from the previous snapshot's restriction; bfloat16 training of both
    networks on the GPU (the corrector's training timed); evaluation at
    Re = 120 against the plain order-4 solve: the plain and the corrected
    order-2 solves (correction every 40 steps) after 40, 120 and 200 steps.
    Both sample sets carry free-stream rows with zero targets (four per
    element), and both corrections subtract the networks' free-stream
    outputs."""
    import numpy as np
    import torch

    import meshgen as mg
    from paper_2508_17917_amd import Solver
    from paper_2508_17917_amd.closure import Closure
    base = mg.workload("cylinder20k")
    mesh = base["mesh"]
    K = len(mesh["EToV"])
    n_runs = 8
    per_run = max(2, args.snapshots // n_runs)
    m, dt = 40, 1e-7
    every = m
    Res = np.sort(mg.rng_for(4).uniform(60.0, 150.0, n_runs))
    n_free = 4 * K      # free-stream rows with zero targets, four per element
    N = n_runs * per_run * K + n_free
    Nc = n_runs * (per_run - 1) * K + n_free
    X = torch.empty((N, 28), dtype=torch.float32, device="cuda")
    T = torch.empty((N, 60), dtype=torch.float32, device="cuda")
    Xc = torch.empty((Nc, 28), dtype=torch.float32, device="cuda")
    Tc = torch.empty((Nc, 24), dtype=torch.float32, device="cuda")

    def pair(Re):
        ph = mg.physics_params(Re=Re, M=0.2)
        mk = lambda p: Solver(p, mesh, gamma=ph["gamma"], Pr=ph["Pr"], mu=ph["mu"], theta=1.0,
                              penalty_mode=0, C_pen=1.0, U_inf=ph["U_inf"])
        return mk(2), mk(4), ph["U_inf"]

    def uniform_state(hi, U_inf):
        u = np.broadcast_to(np.asarray(U_inf)[None, :, None], (hi.K, 4, hi.Np))
        return torch.from_numpy(np.ascontiguousarray(u)).cuda()

    cl, keep = None, []
    row = rowc = 0
    t0 = time.perf_counter()
    for Re in Res:
        lo, hi, U_inf = pair(Re)
        if cl is None:
            cl = Closure(lo, hi, max_batch=args.batch,
                         params=mg.mlp_init(mg.rng_for(4, salt=1), 28, 128, 60))
            cl.make_corrector(mg.mlp_init(mg.rng_for(4, salt=2), 28, 128, 24))
        else:
            cl.rebind(lo, hi)
        keep.append((lo, hi))
        U = uniform_state(hi, U_inf)
        K1 = torch.zeros_like(U)
        U2 = None
        for j in range(per_run):
            hi.rk_steps(U, K1, every, dt)
            cl.features(U, True, out=X[row:row + K])
            cl.targets(U, out=T[row:row + K])
            row += K
            if U2 is not None:
                cl.drift_rows(U2, U, X=Xc[rowc:rowc + K], T=Tc[rowc:rowc + K])
                rowc += K
            U2 = cl.restrict(U)
            K12 = torch.zeros_like(U2)
            lo.rk_steps(U2, K12, m, dt)
    X0, _ = cl.free_rows(60, reps=4)
    X[row:row + n_free] = X0
    T[row:row + n_free] = 0.0
    Xc[rowc:rowc + n_free] = X0
    Tc[rowc:rowc + n_free] = 0.0
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    log("closure data: %d snapshots, %d + %d samples, %.1f s" % (n_runs * per_run, N, Nc, t_data))
    cl.fit_normalization(X, T)
    cl.fit_corrector_normalization(Xc, Tc)
    stream = torch.cuda.current_stream()
    cl.train(X, T, epochs=args.epochs, batch=args.batch, lr=1e-3, seed=0, loss_every=10 ** 9)
    cl.train_corrector(Xc, Tc, epochs=1, batch=args.batch, lr=1e-3, seed=0,
                       loss_every=10 ** 9)  # warm-up
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    losses = cl.train_corrector(Xc, Tc, epochs=args.epochs, batch=args.batch, lr=1e-3, seed=1,
                                loss_every=200)
    ev1.record(stream)
    torch.cuda.synchronize()
    t_train = ev0.elapsed_time(ev1) / 1e3
    steps = args.epochs * (Nc // args.batch)
    samples = steps * args.batch
    flops_sample = 2.0 * (28 * 128 + 128 * 128 + 128 * 24)
    # the training step runs as one fused kernel: its algorithmic HBM bytes
    # are the inputs and targets (FP32), its flops three passes of the network
    bytes_sample = 4 * (28 + 24)
    # both schedules on the same rows, 20 steps each (the trained network)
    sched = {}
    from paper_2508_17917_amd import _lib as L
    Bt = min(args.batch, Xc.shape[0])
    for fused in (1, 0):
        L.dg_mlp_set_schedule(cl.mc, fused)
        L.dg_mlp_backward(cl.mc, Xc[:Bt], Tc[:Bt], want_loss=False)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(20):
            L.dg_mlp_backward(cl.mc, Xc[:Bt], Tc[:Bt], want_loss=False)
        ev1.record(stream)
        torch.cuda.synchronize()
        sched["fused" if fused else "layer_by_layer"] = {
            "us_per_backward": ev0.elapsed_time(ev1) * 1e3 / 20,
            "hbm_bytes_per_sample": bytes_sample if fused else closure_bytes_per_sample(28, 128, 24)}
    L.dg_mlp_set_schedule(cl.mc, 1)
    # evaluation at Re = 120
    lo, hi, U_inf = pair(120.0)
    cl.rebind(lo, hi)
    U4 = uniform_state(hi, U_inf)
    K14 = torch.zeros_like(U4)
    hi.rk_steps(U4, K14, per_run * every // 2, dt)
    Up = cl.restrict(U4)
    Uc = Up.clone()
    K1p, K1c = torch.zeros_like(Up), torch.zeros_like(Up)
    M2, M4 = lo.table("M").reshape(6, 6), hi.table("M").reshape(15, 15)
    geo = hi.table("geo").reshape(hi.K, 16)
    J = 1.0 / (geo[:, 0] * geo[:, 3] - geo[:, 1] * geo[:, 2])

    def norm(D, M):
        d = D.cpu().numpy()
        return float(np.sqrt(np.einsum("kcn,nm,kcm,k->", d, M, d, J)))

    evals = [{"steps": 0, "interp_err": norm(cl.interpolate(Up) - U4, M4),
              "reconstruction_err": norm(cl.correct(Up) - U4, M4)}]
    evals[0]["ratio"] = evals[0]["reconstruction_err"] / evals[0]["interp_err"]
    done, phase = 0, 0
    for n in (40, 120, 200):
        hi.rk_steps(U4, K14, n - done, dt)
        lo.rk_steps(Up, K1p, n - done, dt)
        phase = cl.corrected_steps(Uc, K1c, n - done, dt, m, phase=phase)
        done = n
        ref = cl.restrict(U4)
        ep, ec = norm(Up - ref, M2), norm(Uc - ref, M2)
        e4p, e4c = norm(cl.interpolate(Up) - U4, M4), norm(cl.correct(Uc) - U4, M4)
        evals.append({"steps": n, "order2_err_plain": ep, "order2_err_corrected": ec,
                      "ratio": ec / ep, "order4_err_interpolated_plain": e4p,
                      "order4_err_corrected_reconstructed": e4c, "ratio_order4": e4c / e4p,
                      "fallback": cl.needs_fallback(Uc)})
    # inference: samples + corrector network + update for every element
    for _ in range(3):
        cl.correct_lo(Uc)
    ev0.record(stream)
    for _ in range(20):
        cl.correct_lo(Uc)
    ev1.record(stream)
    torch.cuda.synchronize()
    t_inf = ev0.elapsed_time(ev1) / 1e3 / 20
    out = {
        "metric": "closure MLP training samples/s (bfloat16 matrix cores, FP32 accumulation)",
        "value": samples / t_train, "unit": "samples/s", "n_gpus": 1,
        "steps": steps, "warmup": Nc // args.batch, "ms_per_step": t_train * 1e3 / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "closure20k: order-2 corrector 28->128->128->24 GELU MLP, "
                               "applied every %d steps; %d order-4 snapshots every %d steps "
                               "of impulsively started cylinder20k flows at Re in [60,150] "
                               "(%d runs, %d steps each), %d corrector samples, batch %d, %d "
                               "epochs; evaluated at Re=120" % (
                                   m, n_runs * per_run, every, n_runs, per_run * every, Nc,
                                   args.batch, args.epochs),
                   "samples": Nc, "loss_first": losses[0] if losses else None,
                   "loss_last": losses[-1] if losses else None, "data_s": t_data,
                   "eval": evals, "inference_us_per_correction": t_inf * 1e6,
                   "inference_elements_per_s": K / t_inf},
        "roofline": closure_roofline(bytes_sample, 3 * flops_sample, samples, t_train),
        "schedules": sched,
    }
    cl.close()
    for a, b in keep:
        a.close()
        b.close()
    lo.close()
    hi.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--p", type=int, default=None)
    ap.add_argument("--form", choices=sorted(FORMS), default="fp32-pert")
    ap.add_argument("--compare-forms", action="store_true",
                    help="also run every other form and report its rate and L2 error")
    ap.add_argument("--snapshots", type=int, default=2000, help="closure20k: training snapshots")
    ap.add_argument("--epochs", type=int, default=8, help="closure20k: training epochs")
    ap.add_argument("--batch", type=int, default=65536, help="closure20k: minibatch size")
    ap.add_argument("--workload", choices=["cylinder20k", "cylinder327k", "periodic51k", "viv16",
                                           "closure20k"],
                    default="cylinder20k")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick", action="store_true",
                    help="cylinder20k: the headline order only (no p = 5, 6 and cylinder327k "
                         "sub-objects, CPU baseline at the headline order only)")
    ap.add_argument("--overint", action="store_true",
                    help="single-mesh workloads: the over-integrated FP64 stage (degree-3p "
                         "quadrature), the nodal FP64 stage beside it")
    ap.add_argument("--curved", action="store_true",
                    help="single-mesh workloads: curve the wall layer (isoparametric elements)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 512 MiB device-to-device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the element partition would shard by domain decomposition)", file=sys.stderr)
        sys.exit(2)

    import torch

    import meshgen as mg

    if args.overint:
        if args.workload in ("closure20k", "viv16"):
            print("--overint applies to the single-mesh workloads", file=sys.stderr)
            sys.exit(2)
        args.form = "fp64"
        args.compare_forms = False
    prec = FORMS[args.form]
    if args.workload == "closure20k":
        run_closure(args)
        return
    if args.workload == "viv16":
        out = viv_report(args, prec)
    else:
        orders = [args.p] if args.p is not None else [mg.workload(args.workload)["p"]]
        head = measure(args.workload, orders[0], args.form, args.steps, args.warmup,
                       overint=args.overint, compare_forms=args.compare_forms, cfl=True,
                       curved=args.curved)
        out = head.pop("line")
        # the rest of the metric: the other orders on the same mesh, and the
        # out-of-cache mesh at the headline order (same steps, same forms)
        if args.workload == "cylinder20k" and args.p is None and not args.overint and not args.quick:
            sub = {}
            for p in (5, 6):
                r = measure("cylinder20k", p, args.form, args.steps, args.warmup)
                sub["p%d" % p] = r["summary"]
            out["orders"] = sub
            r = measure("cylinder327k", 4, args.form, args.steps, args.warmup)
            out["cylinder327k"] = r["summary"]
            # the headline mesh with its wall layer curved (isoparametric):
            # the curved kernel's cost is the stage time over the straight one
            r = measure("cylinder20k", 4, args.form, args.steps, args.warmup, curved=True)
            cw = r["summary"]
            straight_us = out["roofline"]["avg_launch_us"]
            over_us = cw["roofline"]["avg_launch_us"] - straight_us
            cw["straight_stage_us"] = straight_us
            cw["curved_overhead_us"] = over_us
            if over_us > 0:
                gbs = cw["curved_bytes_per_launch"] / (over_us * 1e-6) / 1e9
                cw["curved_kernel_roofline"] = {
                    "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": gbs / HBM_PEAK_GBS,
                    "note": "curved set (the curved elements and their face neighbours, one "
                            "element per wave in the stage launch's leading workgroups): its "
                            "algorithmic bytes over the stage time it adds; latency-bound"}
            out["curved_wall"] = cw
        if not args.no_cpu_baseline and args.workload == "cylinder20k":
            log("cpu baseline (oracle)")
            corders = [orders[0]] if (args.p is not None or args.quick or args.overint) else [4, 5, 6]
            out["cpu_baseline"] = cpu_baseline(mg.workload("cylinder20k"), corders,
                                               overint=args.overint)
    if args.copy_probe:
        # a plain copy kernel of known size: 512 MiB read + 512 MiB written per copy,
        # out of any cache, for scaling the FETCH_SIZE / WRITE_SIZE counters
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = src.numel() * 8
        del src, dst
    print(json.dumps(out), flush=True)


def initial_state(wname, w, p):
    """Seeded synthetic state of a single-mesh workload, (K, 4, Np) on the GPU."""
    import numpy as np
    import torch

    import meshgen as mg
    Np = (p + 1) * (p + 2) // 2
    K = len(w["mesh"]["EToV"])
    if wname == "periodic51k":
        # smooth field: three seeded Fourier modes of amplitude 1e-2
        sv = make_solver(w, p, w["mesh"], FORMS["fp64"])
        x, y = sv.nodes()
        sv.close()
        U0n = mg.fourier_modes(x.T, y.T, mg.rng_for(3), L=10.0, amp=1e-2,
                               q0=(1.0, 0.3, 0.0, 1.0 / w["gamma"]), gamma=w["gamma"])
    else:
        U0n = mg.noisy_free_stream((4, Np, K), w["U_inf"], mg.rng_for(1))
    return torch.from_numpy(np.ascontiguousarray(np.transpose(U0n, (2, 0, 1)))).cuda()


def describe(wname, K, p, form):
    Np = (p + 1) * (p + 2) // 2
    if wname == "periodic51k":
        return ("%s: periodic [0,10]^2, 160x160x2 -> K=%d triangles, p=%d (Np=%d), Re=100, "
                "M=0.3, 3 seeded Fourier modes (amplitude 1e-2), %s form" % (wname, K, p, Np, form))
    return ("%s: O-grid %s cells (ratio %s, r 0.5..30) -> K=%d triangles, p=%d (Np=%d), Re=100, "
            "M=0.2, SIPG, free stream + 1e-3 seeded noise, %s form"
            % (wname, "80x128" if wname == "cylinder20k" else "320x512",
               "1.05" if wname == "cylinder20k" else "1.0125", K, p, Np, form))


def measure(wname, p, form, steps, warmup, overint=False, compare_forms=False, cfl=False,
            curved=False):
    """One mesh and order: the chosen form and plain FP64 beside it from the
    same state (warmup + steps LSERK steps with the wall force after each), the
    stage kernel's launch time of each, the L2 difference, the roofline.
    curved: the wall layer's elements isoparametric (meshgen.curve_wall); the
    stage time then covers both launches of a stage.
    Returns {"line": the full bench record, "summary": its per-order digest}."""
    import numpy as np
    import torch

    import meshgen as mg
    w = mg.workload(wname, p)
    Np = (p + 1) * (p + 2) // 2
    K = len(w["mesh"]["EToV"])
    U0 = initial_state(wname, w, p)
    # SIPG with C1 = 1 on the 2.9e-3 wall layer at p = 4 is penalty-limited
    # near 3e-7; 1e-7 keeps the impulsively started state bounded
    dt = min(1e-7 if wname != "periodic51k" else 1.0, stable_dt(w["mesh"], p, w["mu"]) * 1.5)
    cv = mg.curve_wall if curved else None
    log("%s p=%d form %s, warmup %d, steps %d%s" % (wname, p, form, warmup, steps,
                                                    ", wall layer curved" if curved else ""))
    U, t_steps, t_launch, s = run_single(w, U0, FORMS[form], steps, warmup, dt, overint=overint,
                                         curved=cv)
    finite = bool(torch.isfinite(U).all().item())
    if form != "fp64" or overint:
        log("plain fp64 beside it")
        U64, t64, tl64, s64 = run_single(w, U0, FORMS["fp64"], steps, warmup, dt, curved=cv)
    else:
        U64, t64, tl64, s64 = U, t_steps, t_launch, s
    err = rel_l2([s64], [U], [U64], w["U_inf"])
    dofs = 4 * Np * K
    desc = describe(wname, K, p, form)
    if overint:
        desc = desc.replace("fp64 form", "fp64 form, over-integrated (degree-%d quadrature, %d "
                            "element and %d face points)" % (3 * p, ((3 * p + 2) // 2) ** 2,
                                                             3 * ((3 * p + 2) // 2)))
    config = {"workload": desc, "K": K, "p": p, "dofs": dofs, "form": form, "dt": dt,
              "finite": finite, "launch_shape": tuning_of(s), "launch_shape_fp64": tuning_of(s64)}
    if compare_forms:
        forms = {}
        for name in FORMS:
            if name in ("fp64", form):
                continue
            log("form %s" % name)
            Uf, tf, tlf, sf = run_single(w, U0, FORMS[name], steps, warmup, dt)
            forms[name] = {"value": dofs * 5 * steps / tf, "avg_launch_us": tlf * 1e6,
                           "l2_rel_err": rel_l2([s64], [Uf], [U64], w["U_inf"])}
            sf.close()
        config["other_forms"] = forms
    kernel = ("oi_stage_kernel<%d> (over-integrated, fp64)" % p if overint
              else "stage_kernel<%d, %s>" % (p, form))
    traffic = None if overint else measured_traffic(wname, p, form)
    roof = roofline(Np, p + 1, K, t_launch, "fp64" if overint else form, traffic, overint)
    roof["kernel"] = kernel
    roof64 = roofline(Np, p + 1, K, tl64, "fp64", measured_traffic(wname, p, "fp64"))
    value = dofs * 5 * steps / t_steps
    cmp_key = "vs_nodal_fp64" if overint else "vs_plain_fp64"
    cmp = {"value": dofs * 5 * steps / t64, "avg_launch_us": tl64 * 1e6, "speedup": t64 / t_steps,
           ("l2_rel_diff" if overint else "l2_rel_err"): err,
           "l2_norm": "max over fields of ||U - U_fp64||_M / ||U_fp64 - U_inf||_M",
           "steps_compared": warmup + steps,
           "roofline": {k: roof64[k] for k in ("bound", "achieved", "peak", "unit", "frac",
                                                "traffic", "frac_hbm", "frac_mfma_f64",
                                                "frac_valu")}}
    line = {
        "metric": METRIC_OI if overint else METRIC,
        "value": value, "unit": "DOF-updates/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": t_steps * 1e3 / steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if form in ("fp32-pert", "bf16-ops") else "f64",
        "data": "synthetic", "config": config, cmp_key: cmp, "roofline": roof,
    }
    if cfl:
        # the CFL time step of Alg. 3 on the final state (outside the timed
        # region): the bound's value and the cost of one call (two kernels and
        # a synchronising read-back)
        lam, _ = s.cfl_time_step(U)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(20):
            s.cfl_time_step(U)
        line["cfl_time_step"] = {"Lambda": lam, "us_per_call": (time.perf_counter() - t0) / 20 * 1e6,
                                 "note": "dg_cfl_time_step on the final state, C_grad = 1; not in "
                                         "the timed steps"}
    summary = {"workload": "%s p=%d" % (wname, p), "K": K, "dofs": dofs, "form": form,
               "value": value, "ms_per_step": t_steps * 1e3 / steps,
               "plain_fp64_value": cmp["value"], "speedup_vs_fp64": cmp["speedup"],
               "l2_rel_err": err, "finite": finite,
               "roofline": {k: roof[k] for k in ("bound", "achieved", "peak", "unit", "frac",
                                                  "traffic", "kernel", "avg_launch_us", "frac_hbm",
                                                  "frac_valu")},
               "roofline_fp64": cmp["roofline"], "fp64_avg_launch_us": tl64 * 1e6,
               "launch_shape": config["launch_shape"]}
    if curved:
        slot = s.table("curved_slot")
        ns = int((slot >= 0).sum())
        nc = int((np.asarray(w["mesh"]["face_tag"]) == mg.TAG_WALL).any(axis=1).sum())
        summary["workload"] += ", wall layer curved"
        summary["curved_elements"] = nc
        summary["curved_set"] = ns
        summary["curved_bytes_per_launch"] = curved_bytes_per_element(Np, p + 1) * ns
    s.close()
    if s64 is not s:
        s64.close()
    del U, U64, U0
    torch.cuda.empty_cache()
    return {"line": line, "summary": summary}


def viv_report(args, prec):
    import numpy as np
    import torch

    import meshgen as mg
    cases, phys = mg.viv_sweep_cases()
    if args.p is not None:
        for c in cases:
            c["p"] = args.p
    U_inf = phys["U_inf"]
    states, dts, desc, nbytes, gemm, pw, dofs = [], [], [], 0.0, 0.0, 0.0, 0
    for i, c in enumerate(cases):
        Np = (c["p"] + 1) * (c["p"] + 2) // 2
        K = len(c["mesh"]["EToV"])
        U0 = mg.noisy_free_stream((4, Np, K), U_inf, mg.rng_for(2, salt=i + 1))
        states.append(torch.from_numpy(np.ascontiguousarray(np.transpose(U0, (2, 0, 1)))).cuda())
        dts.append(min(1e-7, stable_dt(c["mesh"], c["p"], phys["mu"])))
        gemm += gemm_flops_per_element(Np, c["p"] + 1) * K
        pw += pointwise_flops_per_element(Np, c["p"] + 1) * K
        nbytes += algorithmic_bytes_per_element(Np) * K
        dofs += 4 * Np * K
        desc.append("%dx%d p%d" % (c["ntheta"], c["nr"], c["p"]))
    dts = np.array(dts)
    log("viv16 (%s): chosen form %s batched" % (", ".join(desc), args.form))
    U, t_steps, t_launch, solvers, shape = run_viv(cases, phys, states, prec, args.steps,
                                                   args.warmup, dts, batched=True)
    log("plain fp64 beside it (one launch per stage and instance)")
    U64, t64, _, solvers64, _ = run_viv(cases, phys, states, FORMS["fp64"], args.steps,
                                        args.warmup, dts, batched=False)
    finite = all(bool(torch.isfinite(u).all().item()) for u in U)
    err = rel_l2(solvers64, U, U64, U_inf)
    config = {"workload": "viv16: 16 elastically mounted cylinders (m*=10, xi=0, U* = "
                          "linspace(3,8)), O-grids %s, total K=%d, Re=100, M=0.2, SIPG, "
                          "coupled to host Newmark each step, batched (the stages of a "
                          "step replayed from a HIP graph), %s form" % (
                              ", ".join(desc), sum(s.K for s in solvers64), args.form),
              "instances": len(cases), "dofs": dofs, "form": args.form,
              "launch_shape": shape, "dt": [float(x) for x in dts], "finite": finite}
    kernel = ("batch_stage_kernel<%s>" if shape.startswith("one launch per stage")
              else "batch_order_kernel<p, %s> (one launch per order)") % args.form
    mdt = MFMA_DTYPE[args.form]
    t = {"hbm": nbytes / (HBM_PEAK_GBS * 1e9), "mfma": gemm / (MFMA_PEAK_TFLOPS[mdt] * 1e12),
         "alu": pw / (VALU_PEAK_TFLOPS * 1e12)}
    bound = max(t, key=t.get)
    unit = {"hbm": "GB/s"}.get(bound, "TFLOP/s")
    achieved = {"hbm": nbytes / t_launch / 1e9, "mfma": gemm / t_launch / 1e12,
                "alu": pw / t_launch / 1e12}[bound]
    peak = {"hbm": HBM_PEAK_GBS, "mfma": MFMA_PEAK_TFLOPS[mdt], "alu": VALU_PEAK_TFLOPS}[bound]
    value = dofs * 5 * args.steps / t_steps
    return {
        "metric": METRIC, "value": value, "unit": "DOF-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": t_steps * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.form in ("fp32-pert", "bf16-ops") else "f64", "data": "synthetic",
        "config": config,
        "vs_plain_fp64": {"value": dofs * 5 * args.steps / t64, "speedup": t64 / t_steps,
                          "l2_rel_err": err,
                          "l2_norm": "max over fields of ||U - U_fp64||_M / ||U_fp64 - U_inf||_M",
                          "steps_compared": args.warmup + args.steps},
        "roofline": {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
                     "frac": achieved / peak, "traffic": None, "kernel": kernel,
                     "avg_launch_us": t_launch * 1e6, "bytes_per_launch": nbytes,
                     "frac_hbm": t["hbm"] / t_launch, "frac_valu": t["alu"] / t_launch},
    }


if __name__ == "__main__":
    main()
