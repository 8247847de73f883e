"""Convenience wrapper over the C-ABI: one context, state in torch device tensors.

Layout of every nodal tensor: (K, 4, Np) float64, contiguous, on a HIP
device -- the boundary layout of the library.
"""
import numpy as np

from . import _lib as L


class Solver:
    def __init__(self, p, mesh, gamma=1.4, Pr=0.72, mu=0.0, theta=1.0, penalty_mode=0, C_pen=0.01,
                 U_inf=(1.0, 0.0, 0.0, 1.0), device=True, precision=L.DG_FP64,
                 overintegration=False, wall_flux=L.DG_WALL_ADIABATIC, curved=None):
        """curved: isoparametric elements, as (elems, xy) with xy of shape
        (n, 2, Np), or a function f(mesh, x, y) of the mesh and its straight
        node coordinates x, y (each (Np, K)) returning that pair (e.g.
        meshgen.curve_wall)."""
        self.p = int(p)
        self.precision = int(precision)
        self.h = L.dg_create(self.p, self.precision)
        try:
            if overintegration:
                L.dg_set_overintegration(self.h, True)
            L.dg_set_physics(self.h, gamma, Pr, mu, theta, penalty_mode, C_pen, U_inf)
            L.dg_set_wall_flux(self.h, wall_flux)
            L.dg_set_mesh(self.h, mesh["VX"], mesh["VY"], mesh["EToV"], mesh.get("face_tag"),
                          mesh.get("period", (0.0, 0.0)))
            if curved is not None:
                if callable(curved):
                    L.dg_setup_host(self.h)
                    x, y = L.dg_get_nodes(self.h)
                    Np = L.dg_num_nodes(self.h)
                    curved = curved(mesh, x.reshape(-1, Np).T, y.reshape(-1, Np).T)
                L.dg_set_curved_elements(self.h, curved[0], curved[1])
            if device:
                L.dg_setup(self.h)
            else:
                L.dg_setup_host(self.h)
        except Exception:
            L.dg_destroy(self.h)
            self.h = None
            raise
        self.K = L.dg_num_elements(self.h)
        self.Np = L.dg_num_nodes(self.h)
        self.Nfp = L.dg_num_face_nodes(self.h)

    # -- host-side helpers
    def nodes(self):
        x, y = L.dg_get_nodes(self.h)
        return x.reshape(self.K, self.Np), y.reshape(self.K, self.Np)

    def table(self, name):
        sizes = {"r": self.Np, "s": self.Np, "Dr": self.Np ** 2, "Ds": self.Np ** 2,
                 "M": self.Np ** 2,
                 "LIFT": self.Np * 3 * self.Nfp, "LIFTr": self.Np * 3 * self.Nfp,
                 "LIFTs": self.Np * 3 * self.Nfp, "Fmask": 3 * self.Nfp, "wface": 3 * self.Nfp,
                 "geo": self.K * 16, "nbr": self.K * 3, "nbr_face": self.K * 3,
                 "curved_slot": self.K}
        nc = int((self.table("curved_slot") >= 0).sum()) if name.startswith("curved_") and \
            name != "curved_slot" else 0
        sizes.update({"curved_elem": nc, "curved_node": nc * 5 * self.Np,
                      "curved_face": nc * 9 * self.Nfp, "curved_P": nc * self.Np ** 2,
                      "curved_area": nc})
        q = (3 * self.p + 2) // 2
        Nq, NG = q * q, 3 * q
        sizes.update({"oi_wq": Nq, "oi_xg": q, "oi_wg": q, "oi_Iq": Nq * self.Np,
                      "oi_Drq": Nq * self.Np, "oi_Dsq": Nq * self.Np, "oi_Wr": self.Np * Nq,
                      "oi_Ws": self.Np * Nq, "oi_If1": q * self.Nfp, "oi_Drf": NG * self.Np,
                      "oi_Dsf": NG * self.Np, "oi_LIFTq": self.Np * NG, "oi_LIFTrq": self.Np * NG,
                      "oi_LIFTsq": self.Np * NG})
        return L.dg_get_host_table(self.h, name, sizes[name])

    def set_overintegration(self, on):
        """Switch the quadrature-based (degree-3p) evaluation on or off."""
        L.dg_set_overintegration(self.h, on)

    def set_wall_flux(self, mode):
        """Wall viscous flux: DG_WALL_ADIABATIC (no conduction through the
        wall) or DG_WALL_PRINTED (G(U^b) grad U+ with the interior's
        conduction); takes effect at the next call."""
        L.dg_set_wall_flux(self.h, mode)

    # -- device calls
    def empty_state(self):
        import torch
        return torch.empty((self.K, 4, self.Np), dtype=torch.float64, device="cuda")

    def rhs(self, U, R=None, v_w=(0.0, 0.0), stream=None):
        if R is None:
            R = self.empty_state()
        L.dg_rhs(self.h, U, R, v_w, stream)
        return R

    def rk_step(self, U, K1, dt, v_w=(0.0, 0.0), stream=None):
        L.dg_rk_step(self.h, U, K1, dt, v_w, stream)
        return U

    def rk_steps(self, U, K1, nsteps, dt, v_w=(0.0, 0.0), force=None, stream=None):
        """nsteps steps; with `force` (device float64, 3 nsteps) the wall force
        after every step."""
        L.dg_rk_steps(self.h, U, K1, nsteps, dt, v_w, force, stream)
        return U

    def rk_stage(self, U_in, U_out, K1, a, b, dt, v_w=(0.0, 0.0), stream=None):
        L.dg_rk_stage(self.h, U_in, U_out, K1, a, b, dt, v_w, stream)

    def force(self, U, v_w=(0.0, 0.0), stream=None):
        return L.dg_force(self.h, U, v_w, stream)

    def force_device(self, U, out, v_w=(0.0, 0.0), stream=None):
        """Force into the device tensor out[0:3] without synchronising."""
        L.dg_force_device(self.h, U, out, v_w, stream)
        return out

    def cfl_time_step(self, U, v_w=(0.0, 0.0), C_cfl=1.0, C_grad=1.0, stream=None):
        """(Lambda, C_cfl / Lambda): the CFL bound at the state U."""
        return L.dg_cfl_time_step(self.h, U, v_w, C_cfl, C_grad, stream)

    # -- launch shape
    def set_tuning(self, waves=0, grid=0):
        L.dg_set_tuning(self.h, waves, grid)

    def get_tuning(self):
        return L.dg_get_tuning(self.h)

    def autotune(self, U, reps=20, cache_path=None, stream=None):
        return L.dg_autotune(self.h, U, reps, cache_path, stream)

    def close(self):
        if self.h is not None:
            L.dg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several solvers advanced together (one launch per RK stage for all of
    them, the five stages replayed as a captured HIP graph).  The batch owns
    the states: load them with set_state, read them with get_state."""

    def __init__(self, solvers):
        self.solvers = list(solvers)
        self.n = len(self.solvers)
        self.b = L.dg_batch_create([s.h for s in self.solvers])

    def set_state(self, i, U, stream=None):
        L.dg_batch_set_state(self.b, i, U, stream)

    def get_state(self, i, out=None, stream=None):
        if out is None:
            out = self.solvers[i].empty_state()
        L.dg_batch_get_state(self.b, i, out, stream)
        return out

    def rk_step(self, dt, v_w, stream=None):
        L.dg_batch_rk_step(self.b, dt, v_w, stream)

    def rk_step_states(self, U, K1, dt, v_w, stream=None):
        """One step of every instance on caller-owned states (lists of device
        tensors U[i], K1[i]); the batch-owned states are not preserved."""
        L.dg_batch_rk_step_states(self.b, U, K1, dt, v_w, stream)

    def force(self, v_w=None, stream=None):
        return L.dg_batch_force(self.b, self.n, v_w, stream)

    def coupled_step(self, osc, body, F, dt, stream=None):
        """Newmark (host) of every instance under its lift in F, one RK step
        with the resulting wall velocities, the new forces into F; body and F
        are updated in place (float64 n x 3).  Returns the wall velocities."""
        return L.dg_batch_coupled_step(self.b, osc, body, F, dt, stream)

    def configure(self, mode=0, waves=0, grid=0, use_graph=True):
        L.dg_batch_configure(self.b, mode, waves, grid, 1 if use_graph else 0)

    def autotune(self, reps=10, stream=None):
        return L.dg_batch_autotune(self.b, reps, stream)

    def get_config(self):
        """(mode, waves, grid, use_graph) of the current launch shape."""
        return L.dg_batch_get_config(self.b)

    def close(self):
        if self.b is not None:
            L.dg_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def to_device_layout(U_oracle):
    """(4, Np, K) oracle layout -> (K, 4, Np) contiguous numpy array."""
    return np.ascontiguousarray(np.transpose(U_oracle, (2, 0, 1)))


def from_device_layout(U_dev):
    return np.ascontiguousarray(np.transpose(np.asarray(U_dev), (1, 2, 0)))
