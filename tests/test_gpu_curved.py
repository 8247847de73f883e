"""GPU parity of curved (isoparametric) elements against the curved oracle
(oracle/curved.py), needs an MI355X.

The wall layer of O-grids is curved onto the cylinder (meshgen.curve_wall);
the library evaluates the curved elements and their face neighbours in FP64
in every form (one element per wave in the stage launch's leading
workgroups) and the rest as straight tiles of the same launch.
Bounds: those of the nodal parity tests (plain FP64: per field
max(1e-12 max|R|, 1e-13 T_f)), of the perturbation forms (1e-5 T'_f in
FP32), and bitwise reproducibility across launch shapes and entry points.
"""
import numpy as np
import pytest

import meshgen as mg
from oracle.curved import CurvedMesh, DGOracleCurved, wall_force
from oracle.dg import LSERK_A, LSERK_B
from tests.oracle_helpers import build, uniform
from tests.test_gpu_parity import _check, _from_dev, _say, _to_dev, _torch, term_scale
from tests.test_gpu_precision import TOL32, pert_term_scale
from tests.test_gpu_precision import _check as _check_pert

pytestmark = pytest.mark.gpu


def _retag(m, old, new):
    m = dict(m)
    ft = m["face_tag"].copy()
    ft[ft == old] = new
    m["face_tag"] = ft
    return m


CASES = [
    # name, mesh builder, p, physics overrides, curved tag, state recipe, v_w
    ("cylinder-p4", lambda: mg.ogrid(12, 5, 0.5, 6.0, 1.3), 4,
     dict(mu=2e-3, penalty_mode=0, C_pen=1.0), mg.TAG_WALL, "noise", (0.0, 0.0)),
    ("cylinder-moving-p3", lambda: mg.ogrid(10, 4, 0.5, 5.0, 1.3), 3,
     dict(mu=5e-3, penalty_mode=0, C_pen=1.0), mg.TAG_WALL, "noise", (0.013, -0.021)),
    ("cylinder-p5-iipg", lambda: mg.ogrid(9, 4, 0.5, 5.0, 1.3), 5,
     dict(mu=2e-3, penalty_mode=0, C_pen=0.01, theta=0.0), mg.TAG_WALL, "noise", (0.0, 0.0)),
    ("cylinder-p6-standard", lambda: mg.ogrid(8, 3, 0.5, 4.0, 1.3), 6,
     dict(mu=3e-3, penalty_mode=1, C_pen=1.0), mg.TAG_WALL, "noise", (0.0, 0.0)),
    ("cylinder-p2-nipg", lambda: mg.ogrid(14, 4, 0.5, 5.0, 1.3), 2,
     dict(mu=1e-2, penalty_mode=0, C_pen=1.0, theta=-1.0), mg.TAG_WALL, "noise", (0.0, 0.0)),
    ("cylinder-p1", lambda: mg.ogrid(16, 5, 0.5, 5.0, 1.3), 1,
     dict(mu=1e-2, penalty_mode=0, C_pen=1.0), mg.TAG_WALL, "noise", (0.0, 0.0)),
    ("annulus-far-p4", lambda: _retag(mg.ogrid(12, 4, 0.5, 3.0, 1.3), mg.TAG_WALL, mg.TAG_FAR), 4,
     dict(mu=5e-3, penalty_mode=0, C_pen=1.0), mg.TAG_FAR, "noise", (0.0, 0.0)),
]


def _curved_oracle(mesh, p, over, tag):
    dg = build(mesh, p, **over)
    e, xy = mg.curve_wall(mesh, dg.mesh.x, dg.mesh.y, tag=tag)
    dc = DGOracleCurved(CurvedMesh(dg.mesh, e, xy), dg.phys)
    return dg, dc, (e, xy)


def _solver(mesh, p, phys, curved, **kw):
    from paper_2508_17917_amd import Solver
    return Solver(p, mesh, gamma=phys.gamma, Pr=phys.Pr, mu=phys.mu, theta=phys.theta,
                  penalty_mode=phys.penalty_mode, C_pen=phys.C_pen, U_inf=phys.U_inf,
                  curved=curved, **kw)


def _state(dc, seed):
    cm = dc.mesh
    return mg.noisy_free_stream((4,) + cm.x.shape, dc.phys.U_inf, np.random.default_rng(seed), amp=1e-2)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_curved_rhs_parity(case):
    torch = _torch()
    name, mk, p, over, tag, recipe, vw = case
    mesh = mk()
    dg, dc, curved = _curved_oracle(mesh, p, over, tag)
    U = _state(dc, 7)
    want, parts = dc.rhs(U, vw, return_parts=True)
    # the curved geometry matters at this state: the straight oracle differs
    # (at p = 1 the map through the vertices is the affine one)
    straight = dg.rhs(U, vw)
    if p >= 2:
        assert np.abs(straight - want).max() > 1e-6 * np.abs(want).max()
    else:
        assert np.abs(straight - want).max() < 1e-12 * np.abs(want).max()
    _say("curved rhs %s K=%d p=%d curved=%d" % (name, dg.mesh.K, p, len(curved[0])))
    s = _solver(mesh, p, dg.phys, curved)
    Ud = _to_dev(torch, U)
    R = s.rhs(Ud, v_w=vw)
    torch.cuda.synchronize()
    _check(_from_dev(R), want, what="curved " + name, terms=term_scale(parts))
    # bitwise: again, and in every launch shape of the stage kernel
    assert torch.equal(s.rhs(Ud, v_w=vw), R)
    for waves in (2, 4):
        for grid in (0, 1, 2, 3):
            s.set_tuning(waves, grid)
            assert torch.equal(s.rhs(Ud, v_w=vw), R), (waves, grid)
    s.close()


@pytest.mark.parametrize("case", CASES[:3], ids=[c[0] for c in CASES[:3]])
def test_curved_perturbation_forms(case):
    """The curved set runs in FP64 in every form; the rest in the form."""
    from paper_2508_17917_amd import DG_FP32_PERT, DG_FP64_PERT
    torch = _torch()
    name, mk, p, over, tag, recipe, vw = case
    mesh = mk()
    dg, dc, curved = _curved_oracle(mesh, p, over, tag)
    U = _state(dc, 9)
    want, parts = dc.rhs(U, vw, return_parts=True)
    Ud = _to_dev(torch, U)
    _say("curved rhs fp64-pert %s" % name)
    s = _solver(mesh, p, dg.phys, curved, precision=DG_FP64_PERT)
    R = s.rhs(Ud, v_w=vw)
    torch.cuda.synchronize()
    _check_pert(_from_dev(R), want, 1e-12, 0.1 * term_scale(parts), "curved fp64-pert " + name)
    s.close()
    _say("curved rhs fp32-pert %s" % name)
    s = _solver(mesh, p, dg.phys, curved, precision=DG_FP32_PERT)
    R = s.rhs(Ud, v_w=vw)
    torch.cuda.synchronize()
    # perturbation-term scale from the curved oracle's parts minus the free stream's
    _, p0 = dc.rhs(uniform(dc, dc.phys.U_inf), vw, return_parts=True)
    terms = np.array([max(np.abs(parts[k][f] - p0[k][f]).max() for k in ("vol", "surf", "theta"))
                      for f in range(4)])
    _check_pert(_from_dev(R), want, TOL32, terms, "curved fp32-pert " + name)
    s.close()


@pytest.mark.parametrize("case", CASES[:2], ids=[c[0] for c in CASES[:2]])
def test_curved_rk_step_and_stage_chain(case):
    torch = _torch()
    name, mk, p, over, tag, recipe, vw = case
    mesh = mk()
    dg, dc, curved = _curved_oracle(mesh, p, over, tag)
    U = _state(dc, 11)
    dt = 1e-4
    K0 = U.copy()
    K1 = np.zeros_like(U)
    for a, b in zip(LSERK_A, LSERK_B):
        K1 = a * K1 + dt * dc.rhs(K0, vw)
        K0 = K0 + b * K1
    terms = dt * term_scale(dc.rhs(U, vw, return_parts=True)[1])
    _say("curved rk_step %s" % name)
    s = _solver(mesh, p, dg.phys, curved)
    Ud = _to_dev(torch, U)
    K1d = torch.full_like(Ud, float("nan"))
    s.rk_step(Ud, K1d, dt, v_w=vw)
    torch.cuda.synchronize()
    _check(_from_dev(Ud) - U, K0 - U, tol=1e-11, what="curved rk_step " + name, terms=10 * terms)
    Ua = _to_dev(torch, U)
    Ub = torch.empty_like(Ua)
    K1b = torch.zeros_like(Ua)
    for i, (a, b) in enumerate(zip(LSERK_A, LSERK_B)):
        src, dst = (Ua, Ub) if i % 2 == 0 else (Ub, Ua)
        s.rk_stage(src, dst, K1b, a, b, dt, v_w=vw)
    torch.cuda.synchronize()
    assert torch.equal(Ub, Ud)
    s.close()


def test_curved_free_stream_is_preserved():
    torch = _torch()
    mesh = _retag(mg.ogrid(12, 4, 0.5, 3.0, 1.3), mg.TAG_WALL, mg.TAG_FAR)
    for p in (2, 4, 6):
        dg, dc, curved = _curved_oracle(mesh, p, dict(mu=5e-3, C_pen=1.0), mg.TAG_FAR)
        U = uniform(dc, dc.phys.U_inf)
        _, parts = dc.rhs(_state(dc, 3), return_parts=True)
        terms = max(np.abs(parts[k]).max() for k in ("vol", "surf"))
        _say("curved free stream p=%d" % p)
        s = _solver(mesh, p, dg.phys, curved)
        R = _from_dev(s.rhs(_to_dev(torch, U)))
        assert np.abs(R).max() < 1e-12 * terms, np.abs(R).max()
        s.close()


def test_curved_wall_force_and_steps_with_forces():
    torch = _torch()
    mesh = mg.ogrid(16, 4, 0.5, 5.0, 1.3)
    for p, vw in ((3, (0.0, 0.0)), (4, (0.01, -0.02))):
        dg, dc, curved = _curved_oracle(mesh, p, dict(mu=5e-3, penalty_mode=0, C_pen=1.0), mg.TAG_WALL)
        U = _state(dc, 5)
        want = wall_force(dc, U, vw)
        _say("curved force p=%d" % p)
        s = _solver(mesh, p, dg.phys, curved)
        Ud = _to_dev(torch, U)
        got = s.force(Ud, v_w=vw)
        scale = (1.0 / 1.4) * np.pi
        assert np.abs(got - want).max() <= 1e-12 * scale, (got, want)
        # the multi-step call with a force after every step = single steps
        n = 3
        Ua, Ka = _to_dev(torch, U), torch.zeros_like(Ud)
        Fa = torch.zeros(3 * n, dtype=torch.float64, device="cuda")
        s.rk_steps(Ua, Ka, n, 1e-4, v_w=vw, force=Fa)
        Ub, Kb = _to_dev(torch, U), torch.zeros_like(Ud)
        Fb = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
        for i in range(n):
            s.rk_step(Ub, Kb, 1e-4, v_w=vw)
            s.force_device(Ub, Fb[i], v_w=vw)
        torch.cuda.synchronize()
        assert torch.equal(Ua, Ub) and torch.equal(Fa.view(n, 3), Fb)
        s.close()


def test_curved_rhs_cylinder20k_full_size():
    """The benchmark mesh with its wall layer curved (80 curved elements),
    p = 4, against the curved oracle."""
    torch = _torch()
    w = mg.workload("cylinder20k")
    over = dict(gamma=w["gamma"], Pr=w["Pr"], mu=w["mu"], theta=w["theta"],
                penalty_mode=w["penalty_mode"], C_pen=1.0, U_inf=w["U_inf"])
    dg, dc, curved = _curved_oracle(w["mesh"], w["p"], over, mg.TAG_WALL)
    assert len(curved[0]) == 80
    U = mg.noisy_free_stream((4,) + dc.mesh.x.shape, dc.phys.U_inf, mg.rng_for(1))
    want, parts = dc.rhs(U, return_parts=True)
    _say("curved rhs cylinder20k K=%d" % dg.mesh.K)
    s = _solver(w["mesh"], w["p"], dg.phys, curved)
    R = s.rhs(_to_dev(torch, U))
    torch.cuda.synchronize()
    _check(_from_dev(R), want, what="curved cylinder20k", terms=term_scale(parts))
    s.close()


def test_batches_refuse_curved_contexts():
    from paper_2508_17917_amd import Batch, _lib as L
    _torch()
    mesh = mg.ogrid(8, 2, 0.5, 2.0, 1.3)
    dg, dc, curved = _curved_oracle(mesh, 3, dict(mu=5e-3, C_pen=1.0), mg.TAG_WALL)
    s = _solver(mesh, 3, dg.phys, curved)
    with pytest.raises(L.DGError) as err:
        Batch([s])
    assert err.value.code == L.DG_EUNSUPPORTED
    s.close()


def test_gpu_residual_of_an_exact_vortex_converges_with_curved_walls():
    """The library's right-hand side of the exact potential vortex between
    two walls (mu = 0: slip walls) on three nested annuli at p = 3: with the
    walls curved its mass norm falls at order above 2.5, with straight walls
    it stalls (below 1) -- the same rates as the oracle's."""
    torch = _torch()
    from tests.test_oracle_curved import _annulus_walls, _potential_vortex
    res = []
    for nt, nr in ((8, 2), (16, 4), (32, 8)):
        mesh = _annulus_walls(nt, nr)
        dg, dc, curved = _curved_oracle(mesh, 3, dict(mu=0.0, C_pen=1.0), mg.TAG_WALL)
        row = []
        for cv, geo in ((None, dg), (curved, dc)):
            _say("vortex residual %dx%d curved=%s" % (nt, nr, cv is not None))
            s = _solver(mesh, 3, dg.phys, cv)
            x, y = s.nodes()
            U = _potential_vortex(x.T, y.T)
            R = _from_dev(s.rhs(_to_dev(torch, U)))
            if cv is None:
                row.append(geo.l2_norm(R).max())
            else:
                row.append(np.sqrt(np.einsum("fik,kij,fjk->f", R, geo.mesh.MK, R)).max())
            s.close()
        res.append(row)
    r = np.array(res)
    rate_s = np.log2(r[:-1, 0] / r[1:, 0])
    rate_c = np.log2(r[:-1, 1] / r[1:, 1])
    _say("rates straight %s curved %s" % (rate_s, rate_c))
    assert np.all(rate_c > 2.5) and np.all(rate_s < 1.0)
