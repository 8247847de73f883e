"""GPU parity of the perturbation forms (dg_precision) against the FP64 oracle.

DG_FP64_PERT evaluates every flux as F(U_inf + U') - F(U_inf) in binary64;
in exact arithmetic that is the plain right-hand side, so it is held to the
plain form's bound (test_gpu_parity).

DG_FP32_PERT does the same in binary32 (RK registers stay binary64).  Its
error is measured against the size of the perturbation terms, not of the
full ones: T'_f = the largest magnitude, over the oracle's volume, surface
and theta parts of field f, of parts(U) - parts(U_inf) (the parts of the
uniform free stream carry the constant F(U_inf) that the perturbation form
never forms).  Each term is a chain of a few dozen binary32 operations
followed by a matrix-core sum over Np + 3 Nfp <= 49 products, so its
rounding is bounded by about 100 units of 2^-24 ~ 6e-6 of T'_f; the bound
below is 1e-5 T'_f, plus 1e-5 of the field's own max |R|.
"""
import numpy as np
import pytest

import meshgen as mg
from oracle.dg import LSERK_A, LSERK_B
from tests.oracle_helpers import build, uniform

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5
# bfloat16 operator products: both operands of every product rounded to
# 8 significant bits (u = 2^-9), FP32 accumulation; the operands of the
# divergence and lifts are themselves built from rounded gradients: about
# ten u of the perturbation-term scale
TOLBF = 2e-2


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(msg):
    print("[gpu-case] " + msg, flush=True)


def _solver(mesh, p, phys, precision):
    from paper_2508_17917_amd import Solver
    return Solver(p, mesh, gamma=phys.gamma, Pr=phys.Pr, mu=phys.mu, theta=phys.theta,
                  penalty_mode=phys.penalty_mode, C_pen=phys.C_pen, U_inf=phys.U_inf,
                  precision=precision)


def _to_dev(torch, U):
    return torch.from_numpy(np.ascontiguousarray(np.transpose(U, (2, 0, 1)))).cuda()


def _from_dev(T):
    return np.transpose(T.cpu().numpy(), (1, 2, 0))


PARTS = ("vol", "surf", "theta")


def term_scale(parts):
    return np.array([max(np.abs(parts[k][f]).max() for k in PARTS) for f in range(4)])


def pert_term_scale(dg, parts, vw):
    """Largest perturbation-sized term per field: parts(U) - parts(U_inf)."""
    _, p0 = dg.rhs(uniform(dg, dg.phys.U_inf), vw, return_parts=True)
    return np.array([max(np.abs(parts[k][f] - p0[k][f]).max() for k in PARTS)
                     for f in range(4)])


def _check(got, want, tol, terms, what):
    """Per field: err <= tol max|R| (relative), else <= tol T'_f (term scale);
    prints err/max|R| per field and which bound held."""
    worst = 0.0
    report = []
    for f in range(4):
        scale = np.abs(want[f]).max()
        err = np.abs(got[f] - want[f]).max()
        bound = max(tol * scale, terms[f] * tol)
        worst = max(worst, err / bound)
        report.append("f%d %.2e(%s)" % (f, err / scale if scale > 0 else 0.0,
                                        "rel" if err <= tol * scale else "terms"))
        assert err <= bound, "%s field %d: err %.3e bound %.3e (max|R| %.3e, T' %.3e)" % (
            what, f, err, bound, scale, terms[f])
    _say("%s: worst err/bound %.3f; err/max|R| %s" % (what, worst, " ".join(report)))


CASES = [
    # name, mesh builder, p, physics overrides, state recipe, v_w
    ("cylinder-p4", lambda: mg.ogrid(12, 5, 0.5, 6.0, 1.3), 4,
     dict(mu=2e-3, penalty_mode=0, C_pen=1.0), "noise", (0.0, 0.0)),
    ("cylinder-moving-p4", lambda: mg.ogrid(10, 4, 0.5, 5.0, 1.3), 4,
     dict(mu=2e-3, penalty_mode=0, C_pen=1.0), "noise", (0.013, -0.021)),
    ("vortex-periodic-p3", lambda: mg.periodic_square(5, 4, 10.0, 8.0), 3,
     dict(mu=3e-3, penalty_mode=1, C_pen=1.0, U_inf=mg.free_stream(0.3)), "vortex", (0.0, 0.0)),
    ("cylinder-p5-iipg", lambda: mg.ogrid(9, 4, 0.5, 5.0, 1.3), 5,
     dict(mu=2e-3, penalty_mode=0, C_pen=0.01, theta=0.0), "noise", (0.0, 0.0)),
    ("periodic-p6", lambda: mg.periodic_square(4, 4, 10.0, 10.0), 6,
     dict(mu=3e-3, penalty_mode=0, C_pen=1.0, U_inf=mg.free_stream(0.3)), "fourier", (0.0, 0.0)),
    ("periodic-p1-nipg", lambda: mg.periodic_square(7, 3, 2.0, 1.0), 1,
     dict(mu=1e-2, penalty_mode=1, C_pen=2.0, theta=-1.0), "fourier", (0.05, 0.0)),
    # 70 elements: a partly filled last tile at four elements per tile (p = 4)
    # and at three (p = 5)
    ("cylinder-ragged-p4", lambda: mg.ogrid(7, 5, 0.5, 5.0, 1.3), 4,
     dict(mu=2e-3, penalty_mode=0, C_pen=1.0), "noise", (0.011, 0.017)),
    ("cylinder-ragged-p5", lambda: mg.ogrid(7, 5, 0.5, 5.0, 1.3), 5,
     dict(mu=2e-3, penalty_mode=0, C_pen=1.0), "noise", (0.0, 0.0)),
]


def _state(dg, recipe, seed):
    m = dg.mesh
    rng = np.random.default_rng(seed)
    if recipe == "vortex":
        return mg.isentropic_vortex(m.x, m.y, M=0.3, xc=5.0, yc=4.0, Lper=None)
    if recipe == "noise":
        return mg.noisy_free_stream((4,) + m.x.shape, dg.phys.U_inf, rng)
    L = max(np.ptp(m.x), np.ptp(m.y))
    return mg.fourier_modes(m.x, m.y, rng, L=L, amp=0.05, q0=(1.0, 0.3, 0.0, 1.0 / 1.4))


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_rhs_perturbation_forms(case):
    from paper_2508_17917_amd import DG_FP32_PERT, DG_FP64_PERT
    torch = _torch()
    name, mk, p, over, recipe, vw = case
    mesh = mk()
    dg = build(mesh, p, **over)
    U = _state(dg, recipe, 7)
    want, parts = dg.rhs(U, vw, return_parts=True)
    Ud = _to_dev(torch, U)
    _say("rhs fp64-pert %s K=%d p=%d" % (name, dg.mesh.K, p))
    s = _solver(mesh, p, dg.phys, DG_FP64_PERT)
    R = s.rhs(Ud, v_w=vw)
    torch.cuda.synchronize()
    _check(_from_dev(R), want, TOL64, 0.1 * term_scale(parts), "fp64-pert " + name)
    s.close()
    _say("rhs fp32-pert %s K=%d p=%d" % (name, dg.mesh.K, p))
    s = _solver(mesh, p, dg.phys, DG_FP32_PERT)
    R = s.rhs(Ud, v_w=vw)
    torch.cuda.synchronize()
    _check(_from_dev(R), want, TOL32, pert_term_scale(dg, parts, vw), "fp32-pert " + name)
    R2 = s.rhs(Ud, v_w=vw)
    torch.cuda.synchronize()
    assert torch.equal(R, R2)
    if "ragged" in name:
        # every launch shape covers the partly filled last tile with the same bits
        for waves in (2, 4):
            for grid in (0, 1, 2, 3):
                s.set_tuning(waves, grid)
                assert torch.equal(s.rhs(Ud, v_w=vw), R), (waves, grid)
    s.close()
    from paper_2508_17917_amd import DG_FP32_PERT_BF16OPS
    _say("rhs bf16-ops %s K=%d p=%d" % (name, dg.mesh.K, p))
    s = _solver(mesh, p, dg.phys, DG_FP32_PERT_BF16OPS)
    R = s.rhs(Ud, v_w=vw)
    torch.cuda.synchronize()
    _check(_from_dev(R), want, TOLBF, pert_term_scale(dg, parts, vw), "bf16-ops " + name)
    s.close()


RK_CASES = CASES[:2] + CASES[-2:]


@pytest.mark.parametrize("case", RK_CASES, ids=[c[0] for c in RK_CASES])
def test_rk_step_fp32_pert(case):
    """Five stages in the FP32 perturbation form: the increment U_new - U against
    the oracle's LSERK step, to the FP32 bound scaled by dt; the stage entry
    point chained by hand gives the same bits."""
    from paper_2508_17917_amd import DG_FP32_PERT
    torch = _torch()
    name, mk, p, over, recipe, vw = case
    mesh = mk()
    dg = build(mesh, p, **over)
    U = _state(dg, recipe, 11)
    dt = 1e-4
    want, _ = dg.lserk_step(U, dt, vw)
    _, parts = dg.rhs(U, vw, return_parts=True)
    terms = dt * pert_term_scale(dg, parts, vw)
    _say("rk_step fp32-pert %s K=%d p=%d" % (name, dg.mesh.K, p))
    s = _solver(mesh, p, dg.phys, DG_FP32_PERT)
    Ud = _to_dev(torch, U)
    K1 = torch.zeros_like(Ud)
    s.rk_step(Ud, K1, dt, v_w=vw)
    torch.cuda.synchronize()
    _check(_from_dev(Ud) - U, want - U, TOL32, 10 * terms, "rk fp32-pert " + name)
    Ua = _to_dev(torch, U)
    Ub = torch.empty_like(Ua)
    K1b = torch.zeros_like(Ua)
    for i, (a, b) in enumerate(zip(LSERK_A, LSERK_B)):
        src, dst = (Ua, Ub) if i % 2 == 0 else (Ub, Ua)
        s.rk_stage(src, dst, K1b, a, b, dt, v_w=vw)
    torch.cuda.synchronize()
    assert torch.equal(Ub, Ud)
    s.close()


def test_free_stream_preserved_fp32_pert():
    """The uniform far-field state is an exact steady solution away from walls:
    on a periodic mesh the perturbation form returns exactly zero (every term
    is formed from U' = 0)."""
    from paper_2508_17917_amd import DG_FP32_PERT
    torch = _torch()
    mesh = mg.periodic_square(6, 5, 3.0, 2.0)
    dg = build(mesh, 4, mu=2e-3, penalty_mode=0, C_pen=1.0, U_inf=mg.free_stream(0.2))
    _say("free stream fp32-pert K=%d" % dg.mesh.K)
    s = _solver(mesh, 4, dg.phys, DG_FP32_PERT)
    R = s.rhs(_to_dev(torch, uniform(dg, dg.phys.U_inf)))
    torch.cuda.synchronize()
    assert float(R.abs().max()) == 0.0
    s.close()


def test_rhs_fp32_pert_cylinder20k_full_size():
    """The benchmark workload at full size (K = 20480, p = 4) in the FP32
    perturbation form."""
    from paper_2508_17917_amd import DG_FP32_PERT
    torch = _torch()
    w = mg.workload("cylinder20k")
    dg = build(w["mesh"], w["p"], gamma=w["gamma"], Pr=w["Pr"], mu=w["mu"], theta=w["theta"],
               penalty_mode=w["penalty_mode"], C_pen=w["C_pen"], U_inf=w["U_inf"])
    U = mg.noisy_free_stream((4,) + dg.mesh.x.shape, dg.phys.U_inf, mg.rng_for(1))
    want, parts = dg.rhs(U, return_parts=True)
    _say("rhs fp32-pert cylinder20k K=%d" % dg.mesh.K)
    s = _solver(w["mesh"], w["p"], dg.phys, DG_FP32_PERT)
    R = s.rhs(_to_dev(torch, U))
    torch.cuda.synchronize()
    _check(_from_dev(R), want, TOL32, pert_term_scale(dg, parts, (0.0, 0.0)),
           "fp32-pert cylinder20k")
    s.close()


@pytest.mark.timeout(900)
def test_rhs_periodic51k_full_size_all_forms():
    """The precision-stress workload at full size (160x160x2 periodic, p = 6,
    three Fourier modes of amplitude 1e-2): every form against the oracle."""
    from paper_2508_17917_amd import DG_FP32_PERT, DG_FP32_PERT_BF16OPS, DG_FP64, DG_FP64_PERT
    torch = _torch()
    w = mg.workload("periodic51k")
    dg = build(w["mesh"], w["p"], gamma=w["gamma"], Pr=w["Pr"], mu=w["mu"], theta=w["theta"],
               penalty_mode=w["penalty_mode"], C_pen=w["C_pen"], U_inf=w["U_inf"])
    m = dg.mesh
    U = mg.fourier_modes(m.x, m.y, mg.rng_for(3), L=10.0, amp=1e-2,
                         q0=(1.0, 0.3, 0.0, 1.0 / w["gamma"]), gamma=w["gamma"])
    _say("oracle rhs periodic51k K=%d p=%d" % (m.K, w["p"]))
    want, parts = dg.rhs(U, return_parts=True)
    pts = pert_term_scale(dg, parts, (0.0, 0.0))
    Ud = _to_dev(torch, U)
    for prec, tol, terms, name in ((DG_FP64, TOL64, 0.1 * term_scale(parts), "fp64"),
                                   (DG_FP64_PERT, TOL64, 0.1 * term_scale(parts), "fp64-pert"),
                                   (DG_FP32_PERT, TOL32, pts, "fp32-pert"),
                                   (DG_FP32_PERT_BF16OPS, TOLBF, pts, "bf16-ops")):
        _say("rhs periodic51k %s" % name)
        s = _solver(w["mesh"], w["p"], dg.phys, prec)
        R = s.rhs(Ud)
        torch.cuda.synchronize()
        _check(_from_dev(R), want, tol, terms, name + " periodic51k")
        s.close()
