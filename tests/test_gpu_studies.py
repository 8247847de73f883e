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
