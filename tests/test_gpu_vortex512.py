"""The plain-method workload at its full size against the oracle (needs an MI355X).

vortex512: the viscous isentropic vortex (strength 5, radius 1) on the
periodic [0,10]^2 split-quad mesh of 512 triangles, p = 3, Re = 100, M = 0.3,
literature penalty (C = 1), theta = 1 (SIPG), 200 LSERK steps at
dt = 0.3 / Lambda (CFL bound of the initial state).  The oracle's states after
10, 100 and 200 steps are stored in tests/golden/vortex512_p3_oracle.npz,
written by tests/golden/make_vortex512.py from the oracle alone (a CPU test
re-runs its first 10 steps).

Bound, per field, relative to the largest perturbation |U - U_inf| after the
step (as the trajectory test): plain FP64 1e-12 after 200 steps; the FP32
perturbation form 2e-6.
"""
import os

import numpy as np
import pytest

import meshgen as mg
from tests.test_gpu_parity import _say, _to_dev, _torch

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "vortex512_p3_oracle.npz")


@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (2, 2e-6)], ids=["fp64", "fp32-pert"])
def test_vortex512_two_hundred_steps(precision, tol):
    torch = _torch()
    from paper_2508_17917_amd import Solver
    g = np.load(GOLDEN)
    w = mg.workload("vortex512")
    _say("vortex512 K=512 p=3 precision=%d 200 steps dt=%.6e" % (precision, float(g["dt"])))
    s = Solver(w["p"], w["mesh"], gamma=w["gamma"], Pr=w["Pr"], mu=w["mu"], theta=w["theta"],
               penalty_mode=w["penalty_mode"], C_pen=w["C_pen"], U_inf=w["U_inf"],
               precision=precision)
    try:
        x, y = s.nodes()
        # the GPU's node coordinates give the same initial state as the oracle's
        U0 = mg.isentropic_vortex(x.T, y.T, M=0.3, Lper=10.0)
        assert np.abs(U0 - g["U0"]).max() < 1e-13
        U = _to_dev(torch, g["U0"])
        K1 = torch.zeros_like(U)
        U_inf = np.asarray(w["U_inf"])[:, None, None]
        done = 0
        for m in g["steps"]:
            s.rk_steps(U, K1, int(m) - done, float(g["dt"]))
            done = int(m)
            got = np.transpose(U.cpu().numpy(), (1, 2, 0))
            want = g["U%d" % m]
            pert = np.abs(want - U_inf).max(axis=(1, 2))
            err = np.abs(got - want).max(axis=(1, 2)) / pert
            print("[vortex512] step %d err/pert per field %s" % (m, np.array2string(err, precision=2)),
                  flush=True)
            assert np.all(err <= tol), (m, err)
    finally:
        s.close()
