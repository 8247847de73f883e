"""The flow-study driver on the GPU (short runs of the shedding mesh): the
stationary-cylinder runner records finite force coefficients on the CFL
clock and its summary is self-consistent; the VIV sweep advances a batch of
two reduced velocities and reports per-instance statistics."""
import numpy as np
import pytest

import meshgen as mg

pytestmark = pytest.mark.gpu


def _phys():
    w = mg.workload("shedding20k")
    return w, {k: w[k] for k in ("gamma", "Pr", "mu", "theta", "penalty_mode", "C_pen", "U_inf")}


def test_cylinder_study_short_run():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2508_17917_amd import studies
    w, phys = _phys()
    print("[gpu-case] cylinder study p=1 K=%d" % len(w["mesh"]["EToV"]), flush=True)
    res = studies.cylinder_study(w["mesh"], phys, [1], t_end=0.8, t0=0.2, t1=0.8)
    r = res["rows"][0]
    assert r["finite"] and r["steps"] >= 2000
    # the recorded drag starts at the impulsive-start value and stays finite
    assert np.isfinite([r["CD_mean"], r["CD_rms"], r["CL_mean"], r["CL_rms"], r["St"]]).all()
    assert r["CD_rms"] >= abs(r["CD_mean"]) - 1e-12
    assert res["differences"] == []


def test_viv_study_short_run():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2508_17917_amd import studies
    w, phys = _phys()
    mesh = mg.ogrid(32, 16, 0.5, 20.0, mg.growth_ratio(0.5, 20.0, 16, 0.05))
    print("[gpu-case] viv study p=2 two instances K=%d" % len(mesh["EToV"]), flush=True)
    res = studies.viv_study(mesh, phys, 2, [3.0, 5.0], t_end=1.0, t0=0.2, t1=1.0, cfl_every=200,
                            record_every=1)
    assert res["finite"] and res["steps"] >= 200
    for r, u in zip(res["rows"], (3.0, 5.0)):
        assert r["U_star"] == u and r["f_n"] == pytest.approx(1.0 / u)
        assert np.isfinite([r["A_max"], r["CL_max"], r["f_prim"]]).all()


def test_centreline_vorticity_on_the_shedding_mesh():
    """The wake-centreline samples are the O-grid's theta = 0 grid line from
    the wall (x = 0.5) to the far field (x = 50), 80 whole edges of p + 1
    nodes, and carry the vorticity of the wake-kick state (a transverse
    velocity blob around x = 1.5)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2508_17917_amd import Solver, studies
    w, phys = _phys()
    s0 = Solver(2, w["mesh"], device=False, U_inf=phys["U_inf"])
    x, y = s0.nodes()
    s0.close()
    U0 = np.transpose(mg.wake_kick(x, y, phys["U_inf"], amp=0.1), (1, 0, 2))
    print("[gpu-case] centreline vorticity p=2", flush=True)
    run = studies.CylinderRun(w["mesh"], 2, phys, U0)
    xs, om = run.centreline_vorticity()
    run.close()
    assert len(xs) == 80 * 2 + 1 and np.all(np.diff(xs) > 0)
    assert xs[0] == pytest.approx(0.5) and xs[-1] == pytest.approx(50.0)
    assert np.isfinite(om).all()
    # dv/dx of the blob: positive on its upstream flank, negative downstream
    assert om[np.argmin(np.abs(xs - 2.0))] < 0.0


def test_largest_stable_step_search():
    """The ladder stops at the first C_CFL whose run stops being finite: 4 is
    stable on a small O-grid at p = 1, 400 (|lambda| dt of order 100) is not
    (the state turns non-finite within a few steps; no kernel faults)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2508_17917_amd import studies
    w, phys = _phys()
    mesh = mg.ogrid(32, 16, 0.5, 20.0, mg.growth_ratio(0.5, 20.0, 16, 0.05))
    print("[gpu-case] largest stable step p=1 K=%d" % len(mesh["EToV"]), flush=True)
    r = studies.max_stable_step(mesh, phys, 1, [4.0, 400.0, 800.0], t_end=0.5)
    assert r["C_cfl"] == 4.0 and r["dt"] > 0.0


def test_checkpoint_resume_is_bitwise(tmp_path):
    """A run checkpointed at a chunk boundary and resumed in a fresh runner
    takes the same CFL steps and ends in the same bits, with the same
    recorded force series, as the uninterrupted run."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2508_17917_amd import Solver, studies
    w, phys = _phys()
    mesh = mg.ogrid(32, 16, 0.5, 20.0, mg.growth_ratio(0.5, 20.0, 16, 0.05))
    s0 = Solver(2, mesh, device=False, U_inf=phys["U_inf"])
    x, y = s0.nodes()
    s0.close()
    U0 = np.transpose(mg.wake_kick(x, y, phys["U_inf"], amp=0.1), (1, 0, 2))
    print("[gpu-case] checkpoint and resume p=2 K=%d" % len(mesh["EToV"]), flush=True)
    kw = dict(C_cfl=4.0, cfl_every=200, record_every=5)
    a = studies.CylinderRun(mesh, 2, phys, U0, **kw)
    assert a.advance(0.3)
    path = str(tmp_path / "ck.npz")
    a.save(path)
    a.close()
    b = studies.CylinderRun(mesh, 2, phys, U0, **kw)
    b.load(path)
    assert b.advance(0.6)
    c = studies.CylinderRun(mesh, 2, phys, U0, **kw)
    assert c.advance(0.6)
    assert b.steps == c.steps and b.t == c.t
    assert torch.equal(b.U, c.U)
    for sb, sc in zip(b.series(), c.series()):
        assert np.array_equal(sb, sc)
    with pytest.raises(ValueError):
        studies.CylinderRun(mesh, 3, phys, np.zeros((len(mesh["EToV"]), 4, 10)) + 1.0, **kw).load(path)
    b.close()
    c.close()
