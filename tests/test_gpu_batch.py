"""GPU tests of batches (one stage launch for many meshes, graph-replayed
steps), of the launch-shape autotuner and of the coupled VIV sweep.

A batch step must give what dg_rk_step gives on each instance alone: the
arithmetic of an element does not depend on the launch that runs it.  Each
graph replay is checked against eager per-instance steps taken between the
replays.  The coupled sweep is checked against the oracle's coupling loop
(Alg. 3 order: Newmark under the last force, v_w = dy/dt, RK step, force).
"""
import numpy as np
import pytest

import meshgen as mg
from oracle import fsi
from tests.oracle_helpers import build

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(msg):
    print("[gpu-case] " + msg, flush=True)


def _to_dev(torch, U):
    return torch.from_numpy(np.ascontiguousarray(np.transpose(U, (2, 0, 1)))).cuda()


def _from_dev(T):
    return np.transpose(T.cpu().numpy(), (1, 2, 0))


# uneven meshes, mixed orders (two instances share p = 4), per-instance physics
INSTANCES = [
    (lambda: mg.ogrid(10, 4, 0.5, 5.0, 1.3), 4, 2e-3),
    (lambda: mg.ogrid(12, 5, 0.5, 6.0, 1.3), 5, 3e-3),
    (lambda: mg.periodic_square(4, 3, 4.0, 3.0), 3, 2e-3),
    (lambda: mg.ogrid(9, 3, 0.5, 4.0, 1.3), 6, 4e-3),
    (lambda: mg.ogrid(8, 6, 0.5, 6.0, 1.2), 4, 2.5e-3),
]


def _make(precision):
    from paper_2508_17917_amd import Solver
    U_inf = mg.free_stream(0.2)
    out = []
    for k, (mk, p, mu) in enumerate(INSTANCES):
        mesh = mk()
        s = Solver(p, mesh, gamma=1.4, Pr=0.72, mu=mu, theta=1.0, penalty_mode=0, C_pen=1.0,
                   U_inf=U_inf, precision=precision)
        rng = np.random.default_rng(100 + k)
        U = mg.noisy_free_stream((4, s.Np, s.K), U_inf, rng)
        out.append((s, U))
    return out


def _params(step, n):
    dt = np.array([1e-4 * (1.0 + 0.1 * i) * (1.0 + 0.05 * step) for i in range(n)])
    vw = np.array([[0.0, 0.01 * np.sin(0.7 * i + step)] for i in range(n)])
    return dt, vw


SHAPES = [  # mode, waves, grid, graph
    (0, 0, 0, True), (0, 4, 1, True), (1, 2, 0, True), (1, 4, 1, False), (0, 2, 1, False),
]


@pytest.mark.parametrize("precision", [0, 2], ids=["fp64", "fp32-pert"])
def test_batch_steps_equal_single_instance_steps(precision):
    torch = _torch()
    from paper_2508_17917_amd import Batch
    inst = _make(precision)
    n = len(inst)
    for shape in SHAPES:
        _say("batch precision=%d shape=%s n=%d K=%s" % (precision, shape, n,
                                                        [s.K for s, _ in inst]))
        b = Batch([s for s, _ in inst])
        b.configure(*shape[:3], use_graph=shape[3])
        assert b.get_config() == (shape[0], shape[1] or 4, shape[2], int(shape[3]))
        ref, K1s = [], []
        for i, (s, U) in enumerate(inst):
            Ud = _to_dev(torch, U)
            b.set_state(i, Ud)
            ref.append(Ud.clone())
            K1s.append(torch.zeros_like(Ud))
        for step in range(3):
            dt, vw = _params(step, n)
            b.rk_step(dt, vw)
            # eager single-instance steps between the replays
            for i, (s, _) in enumerate(inst):
                s.rk_step(ref[i], K1s[i], dt[i], v_w=vw[i])
            torch.cuda.synchronize()
            for i, (s, _) in enumerate(inst):
                got = b.get_state(i)
                torch.cuda.synchronize()
                diff = float((got - ref[i]).abs().max())
                assert torch.equal(got, ref[i]), "shape %s step %d instance %d: max diff %.3e" % (
                    shape, step, i, diff)
        # forces on the batch states equal the single-instance forces
        vw = _params(3, n)[1]
        F = b.force(vw)
        for i, (s, _) in enumerate(inst):
            assert np.array_equal(F[i], s.force(ref[i], v_w=vw[i]))
        b.close()
    for s, _ in inst:
        s.close()


@pytest.mark.parametrize("precision", [0, 2], ids=["fp64", "fp32-pert"])
def test_batch_steps_on_caller_owned_states(precision):
    """dg_batch_rk_step_states: the same launches (and graph) on the caller's
    U and K1 arrays give dg_rk_step's bits on each instance; batch-owned
    steps still work afterwards once the states are loaded again."""
    torch = _torch()
    from paper_2508_17917_amd import Batch
    inst = _make(precision)
    n = len(inst)
    for shape in ((1, 4, 0, True), (0, 2, 1, False)):
        _say("batch caller states precision=%d shape=%s" % (precision, shape))
        b = Batch([s for s, _ in inst])
        b.configure(*shape[:3], use_graph=shape[3])
        Us = [_to_dev(torch, U) for _, U in inst]
        K1s = [torch.zeros_like(U) for U in Us]
        ref = [U.clone() for U in Us]
        Kref = [torch.zeros_like(U) for U in Us]
        for step in range(3):
            dt, vw = _params(step, n)
            b.rk_step_states(Us, K1s, dt, vw)
            for i, (s, _) in enumerate(inst):
                s.rk_step(ref[i], Kref[i], dt[i], v_w=vw[i])
            torch.cuda.synchronize()
            for i in range(n):
                assert torch.equal(Us[i], ref[i]), (shape, step, i)
                assert torch.equal(K1s[i], Kref[i]), (shape, step, i)
        # back to batch-owned states
        for i in range(n):
            b.set_state(i, Us[i])
        dt, vw = _params(5, n)
        b.rk_step(dt, vw)
        for i, (s, _) in enumerate(inst):
            s.rk_step(ref[i], torch.zeros_like(ref[i]), dt[i], v_w=vw[i])
        torch.cuda.synchronize()
        for i in range(n):
            assert torch.equal(b.get_state(i), ref[i]), ("batch-owned after", shape, i)
        b.close()
    for s, _ in inst:
        s.close()


def test_batch_states_argument_checks():
    torch = _torch()
    from paper_2508_17917_amd import Batch, Solver, _lib as L
    mesh = mg.ogrid(8, 3, 0.5, 4.0, 1.3)
    sol = [Solver(3, mesh, mu=2e-3, C_pen=1.0, U_inf=mg.free_stream(0.2)) for _ in range(2)]
    inst = [(s, mg.noisy_free_stream((4, s.Np, s.K), mg.free_stream(0.2), np.random.default_rng(7)))
            for s in sol]
    b = Batch([s for s, _ in inst])
    Us = [_to_dev(torch, U) for _, U in inst]
    K1s = [torch.zeros_like(U) for U in Us]
    dt, vw = _params(0, 2)
    with pytest.raises(ValueError):
        b.rk_step_states(Us[:1], K1s, dt, vw)
    with pytest.raises(ValueError):
        b.rk_step_states([Us[0], Us[1][:1]], K1s, dt, vw)   # too small
    with pytest.raises(L.DGError) as e:
        b.rk_step_states([Us[0], Us[0]], K1s, dt, vw)       # shared array
    assert e.value.code == L.DG_EINVAL
    with pytest.raises(L.DGError) as e:
        b.rk_step_states(Us, Us, dt, vw)                     # U is K1
    assert e.value.code == L.DG_EINVAL
    b.close()
    for s, _ in inst:
        s.close()


def test_batch_autotune_keeps_results():
    torch = _torch()
    from paper_2508_17917_amd import Batch
    inst = _make(2)
    n = len(inst)
    b = Batch([s for s, _ in inst])
    ref, K1s = [], []
    for i, (s, U) in enumerate(inst):
        Ud = _to_dev(torch, U)
        b.set_state(i, Ud)
        ref.append(Ud.clone())
        K1s.append(torch.zeros_like(Ud))
    _say("batch autotune")
    us = b.autotune(reps=5)
    assert us > 0.0
    mode, waves, grid, _ = b.get_config()
    assert mode in (0, 1) and waves in (2, 4) and grid in (0, 1)
    # the timed first-stage launches leave the states alone
    for i in range(n):
        assert torch.equal(b.get_state(i), ref[i])
    dt, vw = _params(0, n)
    b.rk_step(dt, vw)
    for i, (s, _) in enumerate(inst):
        s.rk_step(ref[i], K1s[i], dt[i], v_w=vw[i])
    torch.cuda.synchronize()
    for i in range(n):
        assert torch.equal(b.get_state(i), ref[i])
    b.close()
    for s, _ in inst:
        s.close()


def test_single_autotune_and_cache(tmp_path):
    torch = _torch()
    from paper_2508_17917_amd import Solver
    w = mg.workload("cylinder20k")
    path = str(tmp_path / "tune.jsonl")
    for precision in (0, 2):
        s = Solver(4, w["mesh"], gamma=w["gamma"], Pr=w["Pr"], mu=w["mu"], theta=w["theta"],
                   penalty_mode=w["penalty_mode"], C_pen=w["C_pen"], U_inf=w["U_inf"],
                   precision=precision)
        U = _to_dev(torch, mg.noisy_free_stream((4, s.Np, s.K), w["U_inf"], mg.rng_for(1)))
        R0 = s.rhs(U)
        _say("autotune precision=%d" % precision)
        us = s.autotune(U, reps=10, cache_path=path)
        assert us > 0.0
        shape = s.get_tuning()
        assert shape[0] in (2, 4) and shape[1] in (0, 1, 2, 3)
        # a second context finds the entry in the cache without timing
        s2 = Solver(4, w["mesh"], gamma=w["gamma"], Pr=w["Pr"], mu=w["mu"], theta=w["theta"],
                    penalty_mode=w["penalty_mode"], C_pen=w["C_pen"], U_inf=w["U_inf"],
                    precision=precision)
        assert s2.autotune(U, reps=10, cache_path=path) == 0.0
        assert s2.get_tuning() == shape
        # every shape gives the same bits
        for wv in (2, 4):
            for grid in (0, 1, 2, 3):
                s.set_tuning(wv, grid)
                assert torch.equal(s.rhs(U), R0), (precision, wv, grid)
        s.close()
        s2.close()
    lines = open(path).read().strip().splitlines()
    assert len(lines) == 2 and all('"p": 4' in ln for ln in lines)


def test_viv_sweep_matches_oracle_coupling():
    torch = _torch()
    from paper_2508_17917_amd.viv import VIVSweep
    phys = dict(gamma=1.4, Pr=0.72, mu=1e-2, theta=1.0, penalty_mode=0, C_pen=1.0)
    U_inf = mg.free_stream(0.2)
    cases = [dict(mesh=mg.ogrid(10, 4, 0.5, 5.0, 1.3), p=3, U_star=4.0, m_star=10.0, xi=0.0),
             dict(mesh=mg.ogrid(12, 4, 0.5, 5.0, 1.3), p=4, U_star=6.5, m_star=10.0, xi=0.0)]
    sweep = VIVSweep(cases, U_inf=U_inf, **phys)
    oracles, states = [], []
    for i, c in enumerate(cases):
        dg = build(c["mesh"], c["p"], U_inf=U_inf, **phys)
        U = mg.noisy_free_stream((4,) + dg.mesh.x.shape, U_inf, np.random.default_rng(7 + i))
        oracles.append(dg)
        states.append(U)
        sweep.set_state(i, _to_dev(torch, U))
    sweep.update_forces()
    body = np.zeros((2, 3))
    F = np.array([fsi.wall_force(dg, U) for dg, U in zip(oracles, states)])
    v_inf = np.hypot(U_inf[1], U_inf[2]) / U_inf[0]
    coef = [fsi.viv_coefficients(c["U_star"], c["m_star"], c["xi"], v_inf) for c in cases]
    dt = 2e-4
    _say("viv coupled sweep, 3 steps")
    for step in range(3):
        got_F = sweep.step(dt)
        for i, dg in enumerate(oracles):
            M, C, K, inv_m = coef[i]
            y, yd, ydd = fsi.newmark_step(*body[i], F[i, 1] * inv_m, dt, M, C, K)
            vw = (0.0, (y - body[i, 0]) / dt)
            body[i] = (y, yd, ydd)
            states[i], _ = dg.lserk_step(states[i], dt, vw)
            F[i] = fsi.wall_force(dg, states[i], vw)
        scale = (1.0 / 1.4) * np.pi
        assert np.abs(got_F - F).max() <= 1e-11 * scale, (step, got_F, F)
        assert np.abs(sweep.body - body).max() <= 1e-11 * np.abs(body).max() + 1e-300
        for i in range(2):
            U = _from_dev(sweep.get_state(i))
            assert np.abs(U - states[i]).max() <= 1e-12 * np.abs(states[i]).max()
    sweep.close()


def test_batch_viv16_full_size_equals_single_instances():
    """The 16-instance sweep at full size (230k elements, p 4-6): one batched
    step (graph replay) equals single-instance steps, bitwise."""
    torch = _torch()
    from paper_2508_17917_amd import Batch, Solver
    cases, phys = mg.viv_sweep_cases()
    solvers, states = [], []
    for i, c in enumerate(cases):
        s = Solver(c["p"], c["mesh"], precision=2, **phys)
        U = mg.noisy_free_stream((4, s.Np, s.K), phys["U_inf"], mg.rng_for(2, salt=i + 1))
        solvers.append(s)
        states.append(_to_dev(torch, U))
    _say("viv16 batch K=%d" % sum(s.K for s in solvers))
    b = Batch(solvers)
    for i, U in enumerate(states):
        b.set_state(i, U)
    dt = np.full(len(cases), 1e-8)
    vw = np.array([[0.0, 0.001 * i] for i in range(len(cases))])
    b.rk_step(dt, vw)
    for i, s in enumerate(solvers):
        K1 = torch.zeros_like(states[i])
        s.rk_step(states[i], K1, dt[i], v_w=vw[i])
    torch.cuda.synchronize()
    for i in range(len(cases)):
        assert torch.equal(b.get_state(i), states[i]), i
    b.close()
    for s in solvers:
        s.close()


def test_coupled_step_equals_its_parts():
    """dg_batch_coupled_step (Newmark, batch RK step, batch forces in one call)
    gives the same bits as the three steps taken one call at a time."""
    torch = _torch()
    from paper_2508_17917_amd import Batch, Solver
    from paper_2508_17917_amd import _lib as L
    from paper_2508_17917_amd.viv import oscillator
    phys = dict(gamma=1.4, Pr=0.72, mu=1e-2, theta=1.0, penalty_mode=0, C_pen=1.0,
                U_inf=mg.free_stream(0.2))
    meshes = [(mg.ogrid(10, 4, 0.5, 5.0, 1.3), 3), (mg.ogrid(12, 4, 0.5, 5.0, 1.3), 4),
              (mg.ogrid(9, 4, 0.5, 5.0, 1.3), 5)]
    batches, Us = [], []
    for copy in range(2):
        solvers = [Solver(p, m, precision=2, **phys) for m, p in meshes]
        b = Batch(solvers)
        for i, s in enumerate(solvers):
            U = mg.noisy_free_stream((4, s.Np, s.K), phys["U_inf"], mg.rng_for(3, salt=i))
            b.set_state(i, _to_dev(torch, U))
        batches.append((b, solvers))
    n = len(meshes)
    osc = np.array([oscillator(u, 10.0, 0.01, 0.2) for u in (4.0, 5.5, 7.0)])
    dt = np.array([1e-4, 2e-4, 1.5e-4])
    body_a, body_b = np.zeros((n, 3)), np.zeros((n, 3))
    F_a = np.ascontiguousarray(batches[0][0].force())
    F_b = batches[1][0].force()
    assert np.array_equal(F_a, F_b)
    _say("coupled step vs parts, %d instances, 3 steps" % n)
    for step in range(3):
        vw_a = batches[0][0].coupled_step(osc, body_a, F_a, dt)
        vw_b = np.zeros((n, 2))
        for i in range(n):
            M, C, K, s = osc[i]
            st = L.dg_newmark_step(body_b[i], F_b[i, 1] * s, dt[i], M, C, K)
            vw_b[i] = (0.0, (st[0] - body_b[i, 0]) / dt[i])
            body_b[i] = st
        batches[1][0].rk_step(dt, vw_b)
        F_b = batches[1][0].force(vw_b)
        assert np.array_equal(vw_a, vw_b) and np.array_equal(body_a, body_b), step
        assert np.array_equal(F_a, F_b), step
        for i in range(n):
            assert torch.equal(batches[0][0].get_state(i), batches[1][0].get_state(i)), (step, i)
    with pytest.raises(L.DGError):
        batches[0][0].coupled_step(osc, body_a, F_a, np.array([1e-4, 0.0, 1e-4]))
    for b, solvers in batches:
        b.close()
        for s in solvers:
            s.close()
