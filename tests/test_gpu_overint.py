"""GPU parity of the over-integrated stage (degree-3p quadrature on elements
and faces, FP64) against the over-integrated oracle (oracle/overint.py),
with the tolerance of the nodal parity tests: per field
    max |R_gpu - R_oracle| <= max(1e-12 max|R_oracle,f|, 1e-13 T_f),
T_f the largest of the oracle's volume, surface and theta contributions.
Both sides evaluate the weak form with the same rules, so the difference is
the rounding of the sums."""
import numpy as np
import pytest

import meshgen as mg
from oracle.overint import DGOracleOI
from tests.oracle_helpers import build
from tests.test_gpu_parity import CASES, _check, _from_dev, _say, _state, _to_dev, _torch, term_scale

pytestmark = pytest.mark.gpu


def _oi_solver(mesh, p, phys):
    from paper_2508_17917_amd import Solver
    return Solver(p, mesh, gamma=phys.gamma, Pr=phys.Pr, mu=phys.mu, theta=phys.theta,
                  penalty_mode=phys.penalty_mode, C_pen=phys.C_pen, U_inf=phys.U_inf,
                  overintegration=True)


def _oracle(mesh, p, over):
    dg = build(mesh, p, **over)
    return DGOracleOI(dg.mesh, dg.phys), dg


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_overintegrated_rhs_parity(case):
    torch = _torch()
    name, mk, p, over, recipe, vw = case
    mesh = mk()
    oi, dg = _oracle(mesh, p, over)
    U = _state(dg, recipe, 7)
    want, parts = oi.rhs(U, vw, return_parts=True)
    _say("overint rhs %s K=%d p=%d" % (name, dg.mesh.K, p))
    s = _oi_solver(mesh, p, dg.phys)
    Ud = _to_dev(torch, U)
    R = s.rhs(Ud, v_w=vw)
    torch.cuda.synchronize()
    _check(_from_dev(R), want, what=name, terms=term_scale(parts))
    # every launch shape gives the same bits; switched off, the nodal result
    for waves in (2, 4):
        for grid in (0, 1, 2, 3):
            s.set_tuning(waves, grid)
            assert torch.equal(s.rhs(Ud, v_w=vw), R), (waves, grid)
    s.set_overintegration(False)
    Rn = s.rhs(Ud, v_w=vw)
    torch.cuda.synchronize()
    _check(_from_dev(Rn), dg.rhs(U, vw), what=name + " nodal", terms=term_scale(dg.rhs(U, vw, return_parts=True)[1]))
    s.close()


@pytest.mark.parametrize("case", CASES[:3], ids=[c[0] for c in CASES[:3]])
def test_overintegrated_rk_step_parity(case):
    torch = _torch()
    name, mk, p, over, recipe, vw = case
    mesh = mk()
    oi, dg = _oracle(mesh, p, over)
    U = _state(dg, recipe, 11)
    dt = 1e-4
    want, _ = oi.lserk_step(U, dt, vw)
    terms = dt * term_scale(oi.rhs(U, vw, return_parts=True)[1])
    _say("overint rk_step %s K=%d p=%d" % (name, dg.mesh.K, p))
    s = _oi_solver(mesh, p, dg.phys)
    Ud = _to_dev(torch, U)
    K1 = torch.zeros_like(Ud)
    s.rk_step(Ud, K1, dt, v_w=vw)
    torch.cuda.synchronize()
    _check(_from_dev(Ud) - U, want - U, tol=1e-11, what=name, terms=10 * terms)
    s.close()


def test_overintegration_at_full_size_is_conservative():
    """A periodic mesh of 10,240 elements at p = 4 (many tiles, ragged last
    tile): discrete conservation of the over-integrated right-hand side."""
    torch = _torch()
    mesh = mg.periodic_square(64, 80, 10.0, 10.0)
    dg = build(mesh, 4, mu=1e-3)
    U = mg.fourier_modes(dg.mesh.x, dg.mesh.y, np.random.default_rng(3), L=10.0, amp=0.05,
                         q0=(1.0, 0.3, 0.0, 1.0 / 1.4))
    _say("overint conservation K=%d p=4" % dg.mesh.K)
    s = _oi_solver(mesh, 4, dg.phys)
    R = _from_dev(s.rhs(_to_dev(torch, U)))
    tot = dg.integral(R)
    assert np.abs(tot).max() < 1e-12 * np.abs(R).max() * np.sqrt(dg.mesh.K)
    s.close()


def test_batch_rejects_overintegrated_contexts():
    _torch()
    from paper_2508_17917_amd import Batch, _lib as L
    mesh = mg.periodic_square(2, 2, 1.0, 1.0)
    dg = build(mesh, 2)
    s = _oi_solver(mesh, 2, dg.phys)
    with pytest.raises(L.DGError):
        Batch([s])
    s.close()
