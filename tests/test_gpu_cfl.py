"""GPU parity of the CFL bound (dg_cfl_time_step, eq. cfl_general with the
Lambda of eq. rayleigh_bound) against the oracle (oracle/cfl.py) on the
parity cases' meshes and states (periodic, wall and far field, moving wall,
p = 2..6) and on the full shedding mesh: Lambda agrees to 1e-12 relative
(both sides take the same maxima of the same FP64 quantities; they differ
in the rounding of the sums and of the 3x3 eigenvalue problem)."""
import numpy as np
import pytest

import meshgen as mg
from oracle.cfl import CFLOracle
from tests.oracle_helpers import build
from tests.test_gpu_parity import CASES, _say, _solver, _state, _to_dev, _torch

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_cfl_bound_parity(case):
    torch = _torch()
    name, mk, p, over, recipe, vw = case
    mesh = mk()
    dg = build(mesh, p, **over)
    U = _state(dg, recipe, 5)
    c = CFLOracle(dg.mesh, dg.phys)
    _say("cfl %s K=%d p=%d" % (name, dg.mesh.K, p))
    s = _solver(mesh, p, dg.phys)
    Ud = _to_dev(torch, U)
    for C_grad in (1.0, 0.0, 0.3):
        want, _ = c.time_step(U, vw, C_cfl=1.0, C_grad=C_grad)
        lam, dt = s.cfl_time_step(Ud, v_w=vw, C_cfl=0.7, C_grad=C_grad)
        assert abs(lam - want) <= 1e-12 * want, (C_grad, lam, want)
        assert dt == 0.7 / lam
    s.close()


def test_cfl_bound_at_full_size():
    """The shedding mesh (K = 20,480, wall and far field) at p = 3, a noisy
    free stream with a moving wall."""
    torch = _torch()
    w = mg.workload("shedding20k")
    dg = build(w["mesh"], 3, gamma=w["gamma"], Pr=w["Pr"], mu=w["mu"], theta=w["theta"],
               penalty_mode=w["penalty_mode"], C_pen=w["C_pen"], U_inf=w["U_inf"])
    U = mg.noisy_free_stream((4,) + dg.mesh.x.shape, dg.phys.U_inf, mg.rng_for(7), amp=1e-2)
    vw = (0.0, 0.004)
    want, _ = CFLOracle(dg.mesh, dg.phys).time_step(U, vw)
    _say("cfl shedding20k K=%d p=3" % dg.mesh.K)
    s = _solver(w["mesh"], 3, dg.phys)
    lam, _ = s.cfl_time_step(_to_dev(torch, U), v_w=vw)
    assert abs(lam - want) <= 1e-12 * want, (lam, want)
    s.close()


def test_cfl_rejects_bad_arguments():
    torch = _torch()
    from paper_2508_17917_amd import _lib as L
    mesh = mg.periodic_square(2, 2, 1.0, 1.0)
    dg = build(mesh, 2)
    s = _solver(mesh, 2, dg.phys)
    U = _to_dev(torch, _state(dg, "noise", 1))
    for bad in (dict(C_cfl=0.0), dict(C_cfl=-1.0), dict(C_grad=-1.0)):
        with pytest.raises(L.DGError):
            s.cfl_time_step(U, **bad)
    U[0, 0, 0] = float("nan")
    with pytest.raises(L.DGError):
        s.cfl_time_step(U)
    s.close()


@pytest.mark.parametrize("p", [1, 6])
def test_cfl_bound_parity_edge_orders(p):
    """The lowest and highest built orders (p = 1: several face nodes per
    thread, 85 elements per workgroup; p = 6: nine) on a graded O-grid with
    wall and far field and a moving wall."""
    torch = _torch()
    mesh = mg.ogrid(10, 4, 0.5, 4.0, 1.3)
    dg = build(mesh, p, mu=2e-3, penalty_mode=0, C_pen=1.0)
    U = _state(dg, "noise", 13)
    vw = (0.01, -0.02)
    want, _ = CFLOracle(dg.mesh, dg.phys).time_step(U, vw)
    _say("cfl edge order K=%d p=%d" % (dg.mesh.K, p))
    s = _solver(mesh, p, dg.phys)
    lam, _ = s.cfl_time_step(_to_dev(torch, U), v_w=vw)
    assert abs(lam - want) <= 1e-12 * want, (p, lam, want)
    s.close()
