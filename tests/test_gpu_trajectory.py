"""Trajectory parity: 100 LSERK steps on the GPU against 100 steps of the
oracle (its weak-form right-hand side, its LSERK loop and its wall-force
quadrature after every step), from the same seeded state on a graded O-grid
with wall and far field, a moving wall, p = 4, dt = 4 / Lambda (the CFL bound
of the oracle; |lambda| dt about 1).

Bounds, relative to the largest perturbation |U - U_inf| of each field after
100 steps (and to the largest force component):
* plain FP64: 1e-12 (the per-RHS parity bound; rounding differences grow
  about linearly over the steps, 6e-14 measured after 100 steps), forces
  1e-11 (the moment is a small difference of face terms);
* FP32 perturbation form: 2e-6 (1.6e-7 measured), forces 5e-6 — the FP32
  right-hand side's error of a few 1e-8 of the perturbation per step,
  accumulated over 100 steps with a factor 10 of margin."""
import numpy as np
import pytest

import meshgen as mg
from oracle import fsi
from oracle.cfl import CFLOracle
from tests.oracle_helpers import build
from tests.test_gpu_parity import _say, _to_dev, _torch

pytestmark = pytest.mark.gpu

N_STEPS = 100
CHECKS = (1, 10, 50, 100)


@pytest.fixture(scope="module")
def trajectory():
    mesh = mg.ogrid(12, 5, 0.5, 6.0, 1.3)
    dg = build(mesh, 4, mu=2e-3, penalty_mode=0, C_pen=1.0)
    U0 = mg.noisy_free_stream((4,) + dg.mesh.x.shape, dg.phys.U_inf, np.random.default_rng(3),
                              amp=1e-2)
    _, dt = CFLOracle(dg.mesh, dg.phys).time_step(U0, C_cfl=4.0)
    vw = (0.0, 0.01)
    U = U0.copy()
    forces, snaps = [], {}
    for n in range(N_STEPS):
        U, _ = dg.lserk_step(U, dt, vw)
        forces.append(fsi.wall_force(dg, U, vw))
        if n + 1 in CHECKS:
            snaps[n + 1] = U.copy()
    pert = np.abs(snaps[N_STEPS] - dg.phys.U_inf[:, None, None]).max(axis=(1, 2))
    return dict(mesh=mesh, dg=dg, U0=U0, dt=dt, vw=vw, forces=np.array(forces), snaps=snaps,
                pert=pert)


@pytest.mark.parametrize("precision,tol,ftol", [(0, 1e-12, 1e-11), (2, 2e-6, 5e-6)],
                         ids=["fp64", "fp32-pert"])
def test_hundred_steps_follow_the_oracle(trajectory, precision, tol, ftol):
    torch = _torch()
    from paper_2508_17917_amd import Solver
    tr = trajectory
    dg = tr["dg"]
    _say("trajectory K=%d p=4 precision=%d steps=%d" % (dg.mesh.K, precision, N_STEPS))
    s = Solver(4, tr["mesh"], gamma=dg.phys.gamma, Pr=dg.phys.Pr, mu=dg.phys.mu,
               theta=dg.phys.theta, penalty_mode=dg.phys.penalty_mode, C_pen=dg.phys.C_pen,
               U_inf=dg.phys.U_inf, precision=precision)
    U = _to_dev(torch, tr["U0"])
    K1 = torch.zeros_like(U)
    F = torch.zeros((N_STEPS, 3), dtype=torch.float64, device="cuda")
    done = 0
    for m in CHECKS:
        s.rk_steps(U, K1, m - done, tr["dt"], v_w=tr["vw"], force=F[done:m])
        done = m
        got = np.transpose(U.cpu().numpy(), (1, 2, 0))
        err = np.abs(got - tr["snaps"][m]).max(axis=(1, 2)) / tr["pert"]
        assert np.all(err <= tol), (m, err)
    Fo = tr["forces"]
    ferr = np.abs(F.cpu().numpy() - Fo).max(axis=0) / np.abs(Fo).max(axis=0)
    assert np.all(ferr <= ftol), ferr
    s.close()
