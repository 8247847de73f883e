"""The paper's flow studies, run on the library's kernels.

* Stationary cylinder, p-sensitivity (Sec. 3.2.1): mean and RMS of the lift
  and drag coefficients of eq. lift_drag over a window past the transient,
  the Strouhal number from a DFT of the lift, and the differences
  delta_p f = f(p + 1) - f(p) between successive orders; optionally the
  wake-centreline vorticity at a common shedding phase compared between
  orders, any Reynolds number (the validation range 100..250), and the
  heuristic search for the largest stable time step per order.
* Elastically mounted cylinder (Sec. 3.3): per reduced velocity U*, the
  maximum amplitude, the maximum lift coefficient and the primary frequency
  of the displacement (DFT) over a sampling window, all instances advanced
  as one batch with the weak coupling of Alg. 3.

Time steps follow the CFL condition of eq. cfl_general (dg_cfl_time_step,
recomputed every `cfl_every` steps from the current state).  Times are in
convective units t* = t |v_inf| / D (the library works in units of D / c_inf;
the paper's seconds with D = 1 m and |v_inf| = 1 m/s are convective units).

Run as  python -m paper_2508_17917_amd.studies {cylinder,viv,dtmax} ...
from the repository root (the synthetic meshes come from the meshgen module
there).
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import _lib as L
from .solver import Solver
from .viv import VIVSweep

FORMS = {"fp64": L.DG_FP64, "fp64-pert": L.DG_FP64_PERT, "fp32-pert": L.DG_FP32_PERT,
         "bf16-ops": L.DG_FP32_PERT_BF16OPS}


# --------------------------------------------------------------------------
# post-processing (host)
# --------------------------------------------------------------------------
def free_stream_speed(U_inf):
    U_inf = np.asarray(U_inf, dtype=np.float64)
    return float(math.hypot(U_inf[1], U_inf[2]) / U_inf[0])


def force_coefficients(F, U_inf, D=1.0):
    """(C_D, C_L) of eq. lift_drag from force rows F[..., (Fx, Fy, ...)]:
    drag along the free stream, lift perpendicular to it (90 degrees
    counter-clockwise), both over 1/2 rho_inf |v_inf|^2 D."""
    U_inf = np.asarray(U_inf, dtype=np.float64)
    rho = U_inf[0]
    vx, vy = U_inf[1] / rho, U_inf[2] / rho
    v = math.hypot(vx, vy)
    ex, ey = vx / v, vy / v
    q = 0.5 * rho * v * v * D
    F = np.asarray(F)
    return (F[..., 0] * ex + F[..., 1] * ey) / q, (-F[..., 0] * ey + F[..., 1] * ex) / q


def window(t, a, t0, t1):
    m = (t >= t0) & (t <= t1)
    if m.sum() < 2:
        raise ValueError("no samples in the window [%g, %g]" % (t0, t1))
    return t[m], a[m]


def window_stats(t, a, t0, t1):
    """mean, root mean square and maximum magnitude of a over [t0, t1]."""
    _, w = window(t, a, t0, t1)
    return float(w.mean()), float(np.sqrt(np.mean(w * w))), float(np.abs(w).max())


def dominant_frequency(t, a, t0, t1, pad=16):
    """Frequency of the largest DFT magnitude of a (mean removed, Hann
    window, zero-padded `pad` times) over [t0, t1], refined by a parabola
    through the peak bin and its neighbours.  Uniform sampling assumed."""
    tw, w = window(t, a, t0, t1)
    dt = (tw[-1] - tw[0]) / (len(tw) - 1)
    x = (w - w.mean()) * np.hanning(len(w))
    n = pad * len(x)
    mag = np.abs(np.fft.rfft(x, n))
    i = int(np.argmax(mag[1:])) + 1
    if 1 <= i < len(mag) - 1:
        y0, y1, y2 = mag[i - 1], mag[i], mag[i + 1]
        den = y0 - 2.0 * y1 + y2
        d = 0.5 * (y0 - y2) / den if den != 0.0 else 0.0
    else:
        d = 0.0
    return (i + d) / (n * dt)


def p_differences(rows, keys):
    """delta_p f = f(p + 1) - f(p) for consecutive orders in rows (sorted by p)."""
    rows = sorted(rows, key=lambda r: r["p"])
    out = []
    for a, b in zip(rows[:-1], rows[1:]):
        out.append(dict(p=a["p"], **{"d_" + k: b[k] - a[k] for k in keys}))
    return out


# --------------------------------------------------------------------------
# stationary cylinder
# --------------------------------------------------------------------------
class CylinderRun:
    """One order of the stationary-cylinder study: a solver, a state and its
    force history (coefficients recorded every `record_every` steps)."""

    def __init__(self, mesh, p, phys, U0, precision=L.DG_FP32_PERT, C_cfl=8.0, C_grad=1.0,
                 cfl_every=2000, record_every=10, overint=False, kick=None):
        import torch
        self.phys = phys
        # everything a checkpoint must agree on to be resumed by this run
        self.settings = dict(precision=int(precision), overint=bool(overint), C_cfl=float(C_cfl),
                             C_grad=float(C_grad), cfl_every=int(cfl_every),
                             record_every=int(record_every),
                             kick=None if kick is None else float(kick),
                             gamma=float(phys["gamma"]), Pr=float(phys["Pr"]),
                             mu=float(phys["mu"]), theta=float(phys["theta"]),
                             penalty_mode=int(phys["penalty_mode"]), C_pen=float(phys["C_pen"]),
                             U_inf=[float(v) for v in phys["U_inf"]])
        self.s = Solver(p, mesh, gamma=phys["gamma"], Pr=phys["Pr"], mu=phys["mu"],
                        theta=phys["theta"], penalty_mode=phys["penalty_mode"], C_pen=phys["C_pen"],
                        U_inf=phys["U_inf"], precision=precision, overintegration=overint)
        self.p = p
        self.U = torch.from_numpy(np.ascontiguousarray(U0)).cuda()
        self.K1 = torch.zeros_like(self.U)
        self.F = torch.zeros(3 * cfl_every, dtype=torch.float64, device="cuda")
        self.C_cfl, self.C_grad = C_cfl, C_grad
        self.cfl_every, self.record_every = cfl_every, record_every
        self.vel = free_stream_speed(phys["U_inf"])
        self.s.autotune(self.U, reps=10)   # launch shape of the stage kernel
        self.t = 0.0          # library units
        self.steps = 0
        self.t_rec, self.CD, self.CL, self.dts = [], [], [], []
        self.log_every = 25

    def advance(self, t_end_conv, log=None, max_wall=None):
        """Step until the convective time t_end_conv (or, with max_wall, until
        that many seconds of wall time have passed: see `done`); False if the
        state stopped being finite."""
        import torch
        t0 = time.time()
        while not self.done(t_end_conv):
            if max_wall is not None and time.time() - t0 > max_wall:
                break
            _, dt = self.s.cfl_time_step(self.U, C_cfl=self.C_cfl, C_grad=self.C_grad)
            n = self.cfl_every
            self.s.rk_steps(self.U, self.K1, n, dt, force=self.F)
            F = self.F.view(n, 3).cpu().numpy()
            if not np.isfinite(F).all():
                return False
            sel = np.arange(self.record_every - 1, n, self.record_every)
            cd, cl = force_coefficients(F[sel], self.phys["U_inf"])
            self.t_rec.append((self.t + (sel + 1) * dt) * self.vel)
            self.CD.append(cd)
            self.CL.append(cl)
            self.dts.append(dt * self.vel)
            self.t += n * dt
            self.steps += n
            if log is not None and len(self.dts) % self.log_every == 0:
                log("p=%d t*=%.2f steps=%d dt*=%.4g C_D=%.4f C_L=%+.4f (%.0f s)"
                    % (self.p, self.t * self.vel, self.steps, dt * self.vel, cd[-1], cl[-1],
                       time.time() - t0))
        torch.cuda.synchronize()
        return True

    def done(self, t_end_conv):
        """The stepping loop's own end condition."""
        return not (self.t < t_end_conv / self.vel)

    def series(self):
        return np.concatenate(self.t_rec), np.concatenate(self.CD), np.concatenate(self.CL)

    def save(self, path, wall_s=0.0):
        """Checkpoint: the state, the clock, the step count, the recorded
        series, the run's settings and the wall time spent so far (the CFL
        step is recomputed from the state, so a resumed run takes the same
        steps as an uninterrupted one)."""
        import json
        t, cd, cl = self.series() if self.t_rec else (np.zeros(0), np.zeros(0), np.zeros(0))
        np.savez(path, U=self.U.cpu().numpy(), p=self.p, K=self.s.K, t=self.t, steps=self.steps,
                 t_rec=t, CD=cd, CL=cl, dts=np.asarray(self.dts, dtype=np.float64),
                 settings=json.dumps(self.settings, sort_keys=True), wall_s=float(wall_s))

    def load(self, path):
        """Resume from a checkpoint of this order, mesh and settings (else
        ValueError); returns the wall time the checkpointed segments took."""
        import json
        import torch
        z = np.load(path)
        if int(z["p"]) != self.p or int(z["K"]) != self.s.K or z["U"].shape != tuple(self.U.shape):
            raise ValueError("checkpoint of another order or mesh")
        if "settings" not in z.files or json.loads(str(z["settings"])) != json.loads(
                json.dumps(self.settings, sort_keys=True)):
            raise ValueError("checkpoint taken with other settings (form, physics, CFL or "
                             "initial kick) than this run's")
        self.U.copy_(torch.from_numpy(z["U"]))
        self.t, self.steps = float(z["t"]), int(z["steps"])
        self.t_rec, self.CD, self.CL = [z["t_rec"]], [z["CD"]], [z["CL"]]
        self.dts = [float(d) for d in z["dts"]]
        return float(z["wall_s"])

    def summary(self, t0, t1):
        t, cd, cl = self.series()
        cd_m, cd_rms, _ = window_stats(t, cd, t0, t1)
        cl_m, cl_rms, cl_max = window_stats(t, cl, t0, t1)
        return dict(p=self.p, steps=self.steps, dt=float(np.median(self.dts)),
                    CL_mean=cl_m, CL_rms=cl_rms, CD_mean=cd_m, CD_rms=cd_rms, CL_max=cl_max,
                    St=dominant_frequency(t, cl, t0, t1))

    def advance_to_phase(self, chunk=20, max_steps=400000):
        """Step on (fixed dt, the force after every step) until the lift
        crosses zero upwards, to within `chunk` steps: the common shedding
        phase of the snapshots compared between orders."""
        import torch
        _, dt = self.s.cfl_time_step(self.U, C_cfl=self.C_cfl, C_grad=self.C_grad)
        F = torch.zeros(3 * chunk, dtype=torch.float64, device="cuda")
        last = None
        for _ in range(max_steps // chunk):
            self.s.rk_steps(self.U, self.K1, chunk, dt, force=F)
            self.t += chunk * dt
            self.steps += chunk
            cl = force_coefficients(F.view(chunk, 3).cpu().numpy(), self.phys["U_inf"])[1]
            if not np.isfinite(cl).all():
                return False
            seq = cl if last is None else np.concatenate(([last], cl))
            if np.any((seq[:-1] < 0.0) & (seq[1:] >= 0.0)):
                return True
            last = cl[-1]
        return False

    def centreline_vorticity(self):
        """(x, omega) at the nodes on the wake centreline y = 0, x > 0 (the
        O-grid's theta = 0 grid line from the wall to the far field: whole
        edges of p + 1 face nodes, each shared by the elements on both sides,
        whose values are averaged), omega = dv/dx - du/dy from the element's
        nodal derivative matrices and metric terms."""
        U = self.U.cpu().numpy()                                  # (K, 4, Np)
        K, Np = self.s.K, self.s.Np
        Dr = self.s.table("Dr").reshape(Np, Np)
        Ds = self.s.table("Ds").reshape(Np, Np)
        geo = self.s.table("geo").reshape(K, 16)
        x, y = self.s.nodes()
        u = U[:, 1] / U[:, 0]
        v = U[:, 2] / U[:, 0]
        ur, us = u @ Dr.T, u @ Ds.T
        vr, vs = v @ Dr.T, v @ Ds.T
        rx, ry, sx, sy = (geo[:, i:i + 1] for i in range(4))
        om = (rx * vr + sx * vs) - (ry * ur + sy * us)
        on = (np.abs(y) < 1e-9) & (x > 0.0)
        xs, ws = x[on], om[on]
        key = np.round(xs, 9)
        ux = np.unique(key)
        wavg = np.array([ws[key == k].mean() for k in ux])
        return ux, wavg

    def close(self):
        self.s.close()


def _edge_resample(x, w, p, xs):
    """Values at xs of the piecewise polynomial through (x, w): the sorted
    centreline nodes of order p come in edges of p + 1 nodes sharing their
    end nodes, and on each edge the trace is the degree-p Lagrange
    interpolant of its nodes (linear when the count does not fit)."""
    n = len(x)
    if p < 1 or (n - 1) % p != 0:
        return np.interp(xs, x, w)
    ends = x[::p]
    e = np.clip(np.searchsorted(ends, xs, side="right") - 1, 0, len(ends) - 2)
    idx = e[:, None] * p + np.arange(p + 1)[None, :]
    xn, wn = x[idx], w[idx]
    out = np.zeros(len(xs))
    for j in range(p + 1):
        lj = np.ones(len(xs))
        for k in range(p + 1):
            if k != j:
                lj *= (xs - xn[:, k]) / (xn[:, j] - xn[:, k])
        out += lj * wn[:, j]
    return out


def centreline_differences(lines, x0=2.0, x1=40.0, n=8001):
    """||delta_p omega|| in L2(I_x) and L_inf(I_x), I_x = (x0, x1), between
    successive orders: each order's centreline vorticity (keyed by p) is
    resampled onto n uniform points of I_x through its own edge polynomials."""
    xs = np.linspace(x0, x1, n)
    ps = sorted(lines)
    res = {p: _edge_resample(np.asarray(lines[p][0]), np.asarray(lines[p][1]), p, xs) for p in ps}
    out = []
    for a, b in zip(ps[:-1], ps[1:]):
        d = res[b] - res[a]
        out.append(dict(p=a, L2=float(np.sqrt(np.trapezoid(d * d, xs))), Linf=float(np.abs(d).max())))
    return out


def cylinder_study(mesh, phys, ps, t_end, t0, t1, precision=L.DG_FP32_PERT, C_cfl=8.0, C_grad=1.0,
                   kick=0.1, log=None, series_out=None, overint=False, vorticity=False,
                   checkpoint=None, max_wall=None):
    """Strouhal number (f D / |v_inf| = the lift's frequency in convective
    units, D = 1), mean and RMS of C_L and C_D over
    [t0, t1] for every order in ps, and their differences between orders."""
    import meshgen as mg
    if max_wall is not None and checkpoint is None:
        raise ValueError("a wall-time limit needs a checkpoint path")
    rows, series, lines = [], {}, {}
    for p in ps:
        s0 = Solver(p, mesh, gamma=phys["gamma"], Pr=phys["Pr"], mu=phys["mu"], device=False,
                    U_inf=phys["U_inf"])
        x, y = s0.nodes()
        s0.close()
        U0 = np.transpose(mg.wake_kick(x, y, phys["U_inf"], amp=kick, gamma=phys["gamma"]), (1, 0, 2))
        run = CylinderRun(mesh, p, phys, U0, precision, C_cfl, C_grad, overint=overint, kick=kick)
        ck = None if checkpoint is None else "%s_p%d.npz" % (checkpoint, p)
        wall_before = 0.0
        if ck is not None and os.path.exists(ck):
            wall_before = run.load(ck)
            if log is not None:
                log("p=%d resumed from %s at t*=%.2f" % (p, ck, run.t * run.vel))
        w0 = time.time()
        ok = run.advance(t_end, log, max_wall)
        # wall time of every segment of the run, so the rate covers all its steps
        wall = wall_before + (time.time() - w0)
        if not ok:
            rows.append(dict(p=p, finite=False, steps=run.steps))
            run.close()
            continue
        if not run.done(t_end):
            # wall-time limit reached (the loop ends early only then): keep the
            # checkpoint, report progress
            if ck is None:
                raise RuntimeError("run stopped before t* = %g without a checkpoint path" % t_end)
            run.save(ck, wall)
            rows.append(dict(p=p, finite=True, complete=False, steps=run.steps,
                             t=run.t * run.vel, checkpoint=ck))
            run.close()
            continue
        r = run.summary(t0, t1)
        r.update(finite=True, wall_s=wall,
                 dof_updates_per_s=5.0 * 4 * run.s.Np * run.s.K * run.steps / wall)
        if vorticity:
            if run.advance_to_phase():
                lines[p] = run.centreline_vorticity()
                r["phase_t"] = run.t * run.vel
        rows.append(r)
        if series_out is not None:
            series[p] = run.series()
        if log is not None:
            log("p=%d done: St=%.4f C_D mean %.4f rms %.4f C_L mean %+.5f rms %.4f, %d steps, %.1f s"
                % (p, r["St"], r["CD_mean"], r["CD_rms"], r["CL_mean"], r["CL_rms"], run.steps, wall))
        run.close()
    good = [r for r in rows if r.get("finite") and r.get("complete", True)]
    diffs = p_differences(good, ["CL_mean", "CL_rms", "CD_mean", "CD_rms", "St"])
    if vorticity and series_out is not None and lines:
        np.savez_compressed(series_out.replace(".npz", "") + "_vorticity.npz",
                            **{"p%d_%s" % (p, k): v for p, ln in lines.items()
                               for k, v in zip(("x", "omega"), ln)})
    if series_out is not None and series:
        np.savez_compressed(series_out, **{"p%d_%s" % (p, k): v for p, ser in series.items()
                                           for k, v in zip(("t", "CD", "CL"), ser)})
    res = dict(rows=rows, differences=diffs)
    if vorticity:
        res["vorticity_differences"] = centreline_differences(lines) if len(lines) > 1 else []
    return res


def max_stable_step(mesh, phys, p, C_values, t_end, precision=L.DG_FP32_PERT, C_grad=1.0, kick=0.1,
                    log=None):
    """The largest C_CFL of C_values (tried in increasing order, stopping at
    the first failure) for which a run from the wake-kick state stays finite
    up to the convective time t_end, and its time step in convective units:
    the heuristic search the paper reports its admissible time steps from."""
    import meshgen as mg
    s0 = Solver(p, mesh, gamma=phys["gamma"], Pr=phys["Pr"], mu=phys["mu"], device=False,
                U_inf=phys["U_inf"])
    x, y = s0.nodes()
    s0.close()
    U0 = np.transpose(mg.wake_kick(x, y, phys["U_inf"], amp=kick, gamma=phys["gamma"]), (1, 0, 2))
    best = None
    for C in sorted(C_values):
        run = CylinderRun(mesh, p, phys, U0, precision, C, C_grad)
        ok = run.advance(t_end)
        dt = float(np.median(run.dts)) if run.dts else None
        run.close()
        if log is not None:
            log("p=%d C_CFL=%g: %s (dt* %s)" % (p, C, "stable" if ok else "not finite",
                                                 "%.4g" % dt if dt else "-"))
        if not ok:
            break
        best = (C, dt)
    return dict(p=p, C_cfl=None if best is None else best[0], dt=None if best is None else best[1],
                t_end=t_end, tried=sorted(C_values))


# --------------------------------------------------------------------------
# elastically mounted cylinder
# --------------------------------------------------------------------------
def viv_study(mesh, phys, p, U_stars, t_end, t0, t1, m_star=1.0, xi=0.01,
              precision=L.DG_FP32_PERT, C_cfl=8.0, C_grad=1.0, kick=0.1, cfl_every=2000,
              record_every=10, log=None, series_out=None):
    """Per U*: max |y| / D, max |C_L| and the primary frequency of y over
    [t0, t1] (convective units), as f D / |v_inf| and as f / f_n; all
    instances share the mesh, the order and one time step (the smallest of
    their CFL steps)."""
    import torch

    import meshgen as mg
    cases = [dict(mesh=mesh, p=p, U_star=float(u), m_star=m_star, xi=xi) for u in U_stars]
    sw = VIVSweep(cases, phys["gamma"], phys["Pr"], phys["mu"], phys["theta"], phys["penalty_mode"],
                  phys["C_pen"], phys["U_inf"], precision=precision)
    vel = free_stream_speed(phys["U_inf"])
    x, y = sw.solvers[0].nodes()
    U0 = torch.from_numpy(np.ascontiguousarray(
        np.transpose(mg.wake_kick(x, y, phys["U_inf"], amp=kick, gamma=phys["gamma"]), (1, 0, 2)))).cuda()
    for i in range(sw.n):
        sw.set_state(i, U0)
    # launch plan of the batch (one kernel for all orders or one sized for
    # each order group, waves, grid) from timed trials; every plan gives the
    # same bits
    sw.batch.autotune(reps=10)
    sw.update_forces()
    n = sw.n
    t_lib, steps = 0.0, 0
    rec_t, rec_y, rec_cl = [], [], []
    w0 = time.time()
    finite = True
    while t_lib * vel < t_end:
        dts = np.empty(n)
        for i in range(n):
            Ui = sw.get_state(i)
            dts[i] = sw.solvers[i].cfl_time_step(Ui, v_w=tuple(sw.vw[i]), C_cfl=C_cfl, C_grad=C_grad)[1]
        dt = float(dts.min())       # one clock for the whole sweep
        for k in range(cfl_every):
            sw.step(dt)
            if (k + 1) % record_every == 0:
                rec_t.append((t_lib + (k + 1) * dt) * vel)
                rec_y.append(sw.body[:, 0].copy())
                rec_cl.append(force_coefficients(sw.F, phys["U_inf"])[1])
        t_lib += cfl_every * dt
        steps += cfl_every
        if not (np.isfinite(sw.F).all() and np.isfinite(sw.body).all()):
            finite = False
            break
        if log is not None and (steps // cfl_every) % 25 == 0:
            log("viv t*=%.2f steps=%d dt*=%.4g max|y|=%.4f (%.0f s)"
                % (t_lib * vel, steps, dt * vel, np.abs(sw.body[:, 0]).max(), time.time() - w0))
    wall = time.time() - w0
    t = np.array(rec_t)
    Y = np.array(rec_y)
    CL = np.array(rec_cl)
    rows = []
    for i, u in enumerate(U_stars):
        # natural frequency in convective units: f_n D / |v_inf| = 1 / U*
        r = dict(U_star=float(u), f_n=1.0 / float(u))
        if finite:
            _, _, amax = window_stats(t, Y[:, i], t0, t1)
            _, _, clmax = window_stats(t, CL[:, i], t0, t1)
            f = dominant_frequency(t, Y[:, i], t0, t1)     # convective units
            r.update(A_max=amax, CL_max=clmax, f_prim=f, f_ratio=f * float(u))
        rows.append(r)
    if series_out is not None and finite:
        np.savez_compressed(series_out, t=t, y=Y, CL=CL, U_star=np.asarray(U_stars, dtype=float))
    dofs = sum(s.K * 4 * s.Np for s in sw.solvers)
    sw.close()
    return dict(rows=rows, finite=finite, steps=steps, wall_s=wall,
                dof_updates_per_s=5.0 * dofs * steps / wall)


# --------------------------------------------------------------------------
def _log(msg):
    print("[study] " + msg, file=sys.stderr, flush=True)


def main(argv=None):
    import meshgen as mg
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    sub = ap.add_subparsers(dest="study", required=True)
    for name in ("cylinder", "viv", "dtmax"):
        a = sub.add_parser(name)
        a.add_argument("--t-end", type=float, required=True, help="convective time")
        if name == "dtmax":
            a.add_argument("--p", type=int, nargs="+", default=[1, 2, 3, 4, 5])
            a.add_argument("--c-values", type=float, nargs="+", required=True,
                           help="C_CFL values to try, in increasing order")
        a.add_argument("--window", type=float, nargs=2, required=(name != "dtmax"),
                       default=None, help="t0 t1, convective")
        a.add_argument("--form", default="fp32-pert", choices=sorted(FORMS))
        a.add_argument("--c-cfl", type=float, default=8.0)
        a.add_argument("--c-grad", type=float, default=1.0)
        a.add_argument("--kick", type=float, default=0.1)
        a.add_argument("--c-pen", type=float, default=None, help="penalty constant (default 0.01)")
        a.add_argument("--theta", type=float, default=None, help="theta (default 0, IIP)")
        a.add_argument("--re", type=float, default=None,
                       help="Reynolds number |v_inf| D / nu (default 200)")
        a.add_argument("--out", default=None, help="JSON result file")
        a.add_argument("--series", default=None, help=".npz file for the recorded series")
        if name == "dtmax":
            continue
        if name == "cylinder":
            a.add_argument("--p", type=int, nargs="+", default=[1, 2, 3, 4])
            a.add_argument("--overint", action="store_true",
                           help="over-integrated weak form (plain FP64 form only)")
            a.add_argument("--checkpoint", default=None,
                           help="path prefix of per-order checkpoints: resume from one "
                                "if present; with --max-wall, save one when time runs out")
            a.add_argument("--max-wall", type=float, default=None,
                           help="wall seconds per order before checkpointing")
            a.add_argument("--vorticity", action="store_true",
                           help="after t-end, advance to an upward zero crossing of the lift "
                                "and compare the wake-centreline vorticity between orders")
        else:
            a.add_argument("--p", type=int, default=3)
            a.add_argument("--ustar", type=float, nargs="+", required=True)
            a.add_argument("--m-star", type=float, default=1.0)
            a.add_argument("--xi", type=float, default=0.01)
    args = ap.parse_args(argv)
    w = mg.workload("shedding20k")
    phys = {k: w[k] for k in ("gamma", "Pr", "mu", "theta", "penalty_mode", "C_pen", "U_inf")}
    if args.c_pen is not None:
        phys["C_pen"] = args.c_pen
    if args.theta is not None:
        phys["theta"] = args.theta
    Re = 200.0
    if args.re is not None:
        # mu = rho_inf |v_inf| D / Re (D = 1)
        Re = args.re
        phys["mu"] = phys["U_inf"][0] * free_stream_speed(phys["U_inf"]) / Re
    t0, t1 = args.window if args.window is not None else (None, None)
    if args.study == "dtmax":
        rows = [max_stable_step(w["mesh"], phys, p, args.c_values, args.t_end, FORMS[args.form],
                                args.c_grad, args.kick, log=_log) for p in args.p]
        res = dict(rows=rows)
    elif args.study == "cylinder":
        res = cylinder_study(w["mesh"], phys, args.p, args.t_end, t0, t1, FORMS[args.form],
                             args.c_cfl, args.c_grad, args.kick, log=_log, series_out=args.series,
                             overint=args.overint, vorticity=args.vorticity,
                             checkpoint=args.checkpoint, max_wall=args.max_wall)
        res["overint"] = bool(args.overint)
    else:
        res = viv_study(w["mesh"], phys, args.p, args.ustar, args.t_end, t0, t1, args.m_star,
                        args.xi, FORMS[args.form], args.c_cfl, args.c_grad, args.kick, log=_log,
                        series_out=args.series)
    res.update(study=args.study, mesh="shedding20k: O-grid 128x80 cells, first layer 0.017 D, "
               "far field at 50 D, K=20480", Re=Re, M=0.1, form=args.form, C_cfl=args.c_cfl,
               C_grad=args.c_grad, C_pen=phys["C_pen"], theta=phys["theta"], window=[t0, t1],
               t_end=args.t_end)
    line = json.dumps(res, default=float)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
