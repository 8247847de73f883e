"""Host logic of the flow studies (paper_2508_17917_amd.studies) and of
their synthetic inputs: force coefficients of eq. lift_drag, window
statistics, the DFT frequency estimate, differences between orders, the
graded O-grid of the shedding mesh and its initial state."""
import math

import numpy as np
import pytest

import meshgen as mg
from paper_2508_17917_amd.studies import (dominant_frequency, force_coefficients, p_differences,
                                          window_stats)


def test_force_coefficients_along_and_across_the_stream():
    U = mg.free_stream(0.1)
    q = 0.5 * 1.0 * 0.1 ** 2
    cd, cl = force_coefficients(np.array([[2.0 * q, 0.5 * q, 0.0]]), U)
    assert cd[0] == pytest.approx(2.0) and cl[0] == pytest.approx(0.5)
    # a stream at 30 degrees: drag along it, lift 90 degrees counter-clockwise
    a = math.radians(30.0)
    U = mg.free_stream(0.1, angle=a)
    F = np.array([[q * (1.5 * math.cos(a) - 0.2 * math.sin(a)), q * (1.5 * math.sin(a) + 0.2 * math.cos(a)), 0.0]])
    cd, cl = force_coefficients(F, U)
    assert cd[0] == pytest.approx(1.5) and cl[0] == pytest.approx(0.2)


def test_window_stats_of_a_sine():
    t = np.linspace(0.0, 100.0, 100001)
    a = 0.3 + np.sin(2.0 * math.pi * 0.2 * t)
    m, rms, amax = window_stats(t, a, 20.0, 70.0)     # ten whole periods
    assert m == pytest.approx(0.3, abs=1e-4)
    assert rms == pytest.approx(math.sqrt(0.09 + 0.5), abs=1e-4)
    assert amax == pytest.approx(1.3, abs=1e-6)


@pytest.mark.parametrize("f0", [0.1987, 0.2, 0.37])
def test_dominant_frequency(f0):
    rng = np.random.default_rng(0)
    t = np.arange(0.0, 120.0, 0.01)
    a = 0.8 * np.sin(2.0 * math.pi * f0 * t + 0.4) + 0.1 * np.sin(2.0 * math.pi * 2 * f0 * t) \
        + 0.01 * rng.standard_normal(t.shape) + 2.0
    assert dominant_frequency(t, a, 30.0, 120.0) == pytest.approx(f0, rel=2e-3)


def test_p_differences():
    rows = [dict(p=3, a=1.0), dict(p=1, a=4.0), dict(p=2, a=2.5)]
    d = p_differences(rows, ["a"])
    assert [r["p"] for r in d] == [1, 2]
    assert [r["d_a"] for r in d] == [-1.5, -1.5]


def test_shedding_mesh_grading():
    q = mg.growth_ratio(0.5, 50.0, 80, 0.017)
    assert 0.017 * (q ** 80 - 1.0) / (q - 1.0) == pytest.approx(49.5, rel=1e-12)
    w = mg.workload("shedding20k")
    m = w["mesh"]
    r = np.hypot(m["VX"], m["VY"]).reshape(81, 128)[:, 0]
    assert r[1] - r[0] == pytest.approx(0.017, rel=1e-9)
    assert r[-1] == 50.0 and len(m["EToV"]) == 20480
    assert w["theta"] == 0.0 and w["C_pen"] == 0.01
    assert w["mu"] == pytest.approx(0.1 / 200.0)
    with pytest.raises(ValueError):
        mg.growth_ratio(0.5, 50.0, 80, 1.0)


def test_wake_kick():
    x = np.linspace(-3.0, 5.0, 81)
    y = np.zeros_like(x)
    U = mg.wake_kick(x, y, mg.free_stream(0.1), amp=0.1)
    rho = U[0]
    v = U[2] / rho
    p = 0.4 * (U[3] - 0.5 * (U[1] ** 2 + U[2] ** 2) / rho)
    assert np.allclose(rho, 1.0) and np.allclose(p, 1.0 / 1.4) and np.allclose(U[1] / rho, 0.1)
    assert v.max() == pytest.approx(0.01, rel=1e-12) and x[np.argmax(v)] == pytest.approx(1.5)


def test_study_command_line():
    from paper_2508_17917_amd import studies
    for study in ("cylinder", "viv", "dtmax"):
        with pytest.raises(SystemExit) as e:
            studies.main([study, "--help"])
        assert e.value.code == 0
    with pytest.raises(SystemExit) as e:
        studies.main(["viv", "--t-end", "1", "--window", "0", "1"])   # --ustar is required
    assert e.value.code == 2


def test_centreline_differences():
    from paper_2508_17917_amd.studies import centreline_differences
    # linear profiles: reproduced exactly by every order's resampling
    x = np.linspace(0.0, 50.0, 2001)
    lines = {3: (x, 0.3 * x - 1.0), 4: (x, 0.3 * x - 0.9), 5: (x, 0.3 * x - 0.9)}
    d = centreline_differences(lines)
    assert [r["p"] for r in d] == [3, 4]
    assert d[0]["L2"] == pytest.approx(0.1 * math.sqrt(38.0), rel=1e-9)
    assert d[0]["Linf"] == pytest.approx(0.1, rel=1e-12)
    assert d[1]["L2"] < 1e-12 and d[1]["Linf"] < 1e-12


def test_edge_resampling_is_exact_for_the_edge_polynomials():
    from paper_2508_17917_amd.studies import _edge_resample
    rng = np.random.default_rng(0)
    p = 4
    ends = np.cumsum(rng.uniform(0.3, 1.5, 12))
    # Gauss-Lobatto-like interior nodes on every edge, shared end nodes
    ref = np.array([-1.0, -0.6546536707, 0.0, 0.6546536707, 1.0])
    x = np.concatenate([0.5 * (a + b) + 0.5 * (b - a) * ref[:-1] for a, b in zip(ends[:-1], ends[1:])]
                       + [ends[-1:]])
    # a cubic is reproduced exactly by every degree-4 edge interpolant
    coef = rng.standard_normal(4)
    w = sum(coef[k] * x ** k for k in range(4))
    xs = np.linspace(ends[0], ends[-1], 777)
    want = sum(coef[k] * xs ** k for k in range(4))
    got = _edge_resample(x, w, p, xs)
    assert np.allclose(got, want, rtol=1e-9, atol=1e-9)
    # and linear resampling would not be
    assert not np.allclose(np.interp(xs, x, w), want, rtol=1e-6, atol=1e-6)


def _fake_run(p=3, K=12, Np=10, **over):
    """A CylinderRun without a solver or GPU: the attributes that done(),
    save() and load() use, on host tensors."""
    import types

    import torch
    from paper_2508_17917_amd.studies import CylinderRun
    run = object.__new__(CylinderRun)
    run.p, run.vel = p, 0.1
    run.s = types.SimpleNamespace(K=K, Np=Np)
    run.U = torch.arange(K * 4 * Np, dtype=torch.float64).reshape(K, 4, Np)
    run.t, run.steps = 0.0, 0
    run.t_rec, run.CD, run.CL, run.dts = [], [], [], []
    run.settings = dict(precision=2, overint=False, C_cfl=16.0, C_grad=1.0, cfl_every=2000,
                        record_every=10, kick=0.1, gamma=1.4, Pr=0.72, mu=5e-4, theta=0.0,
                        penalty_mode=0, C_pen=0.01, U_inf=[1.0, 0.1, 0.0, 1.8])
    run.settings.update(over)
    return run


def test_done_is_the_stepping_loops_condition():
    """done() is exactly the loop's `t < t_end / vel` test, also on a
    rounding edge where t * vel and t_end disagree."""
    run = _fake_run()
    t_end = 0.3
    run.t = t_end / run.vel
    assert run.done(t_end)
    run.t = np.nextafter(t_end / run.vel, 0.0)
    assert not run.done(t_end)
    # a clock where the product rounds up to t_end but the loop would go on
    for x in np.linspace(0.1, 10.0, 997):
        run.t = np.nextafter(x / run.vel, 0.0)
        assert run.done(x) == (not (run.t < x / run.vel))


def test_checkpoint_keeps_settings_and_wall_time(tmp_path):
    run = _fake_run()
    run.t, run.steps = 1.25, 4000
    run.t_rec, run.CD, run.CL = [np.array([0.1, 0.2])], [np.array([1.3, 1.31])], [np.array([0.0, 0.1])]
    run.dts = [1e-4, 1e-4]
    path = str(tmp_path / "ck.npz")
    run.save(path, wall_s=12.5)
    other = _fake_run()
    other.U.zero_()
    assert other.load(path) == 12.5
    assert other.steps == 4000 and other.t == 1.25 and float(other.U.sum()) == float(run.U.sum())
    for key, val in (("precision", 0), ("overint", True), ("mu", 1e-3), ("C_cfl", 8.0),
                     ("kick", 0.2), ("U_inf", [1.0, 0.2, 0.0, 1.8])):
        with pytest.raises(ValueError, match="other settings"):
            _fake_run(**{key: val}).load(path)
    with pytest.raises(ValueError, match="another order"):
        _fake_run(p=4).load(path)
