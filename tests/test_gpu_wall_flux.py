"""GPU parity of the two wall viscous fluxes (needs an MI355X).

DG_WALL_ADIABATIC (the default) drops heat conduction from the wall's viscous
flux and theta term; DG_WALL_PRINTED keeps the printed G(U^b) grad U+ with the
interior's conduction (Sec. 2.2.4 and the boundary flux of the weak form).
Each is checked against the oracle with the matching Physics.wall_heat_flux,
in every evaluation form, with the bounds of the nodal, perturbation and
over-integrated parity tests.  The states are chosen so that the two modes
differ by far more than those bounds: a noisy free stream around a cylinder
(at rest and moving wall), and a closed annulus at rest with a radial
temperature profile, where the printed flux alone lets heat through.

At rest the energy right-hand side is a small remainder: the ghost state
U^b = [rho+, v_w, p+] is rebuilt from the trace, so the jump U+ - U^b is a
rounding residue that the penalty (large on the annulus's thin elements)
multiplies.  The oracle itself moves by about 1e-10 when its input is changed
by one unit in the last place; the FP64 bounds below therefore also admit
that spread, measured per field over two seeded one-ulp perturbations.
"""
import numpy as np
import pytest

import meshgen as mg
from oracle.overint import DGOracleOI
from tests.oracle_helpers import build
from tests.test_gpu_parity import _check, _from_dev, _say, _state, _to_dev, _torch, term_scale
from tests.test_gpu_precision import TOL32, TOL64, pert_term_scale
from tests.test_gpu_precision import _check as _check_pert

pytestmark = pytest.mark.gpu


def _annulus_mesh():
    m = mg.ogrid(16, 4, 0.5, 2.0, 1.2)
    ft = m["face_tag"].copy()
    ft[ft == mg.TAG_FAR] = mg.TAG_WALL
    m = dict(m)
    m["face_tag"] = ft
    return m


CASES = [
    # name, mesh builder, p, physics overrides, state recipe, v_w
    ("cylinder-p4", lambda: mg.ogrid(12, 5, 0.5, 6.0, 1.3), 4,
     dict(mu=2e-3, penalty_mode=0, C_pen=1.0), "noise", (0.0, 0.0)),
    ("cylinder-moving-p3", lambda: mg.ogrid(10, 4, 0.5, 5.0, 1.3), 3,
     dict(mu=5e-3, penalty_mode=0, C_pen=1.0), "noise", (0.013, -0.021)),
    ("cylinder-p5-iipg", lambda: mg.ogrid(9, 4, 0.5, 5.0, 1.3), 5,
     dict(mu=2e-3, penalty_mode=0, C_pen=0.01, theta=0.0), "noise", (0.0, 0.0)),
    ("annulus-rest-p3", _annulus_mesh, 3,
     dict(mu=5e-2, penalty_mode=0, C_pen=1.0), "rest", (0.0, 0.0)),
]


def _rest_state(dg, gamma=1.4):
    x, y = dg.mesh.x, dg.mesh.y
    r = np.hypot(x, y)
    T = 1.0 / gamma * (1.0 + 0.2 * np.sin(2.0 * r) + 0.05 * x)
    rho = (1.0 / gamma) / T
    zero = np.zeros_like(r)
    return np.stack([rho, zero, zero, (1.0 / gamma) / (gamma - 1.0) * np.ones_like(r)])


def _ulp_spread(oracle, U, vw):
    """Per field: the largest change of the oracle's right-hand side under
    two seeded relative perturbations of U by about one unit in the last
    place."""
    rng = np.random.default_rng(5)
    R = oracle.rhs(U, vw)
    out = np.zeros(4)
    for _ in range(2):
        Up = U * (1.0 + 2.0 ** -52 * rng.standard_normal(U.shape))
        out = np.maximum(out, np.abs(oracle.rhs(Up, vw) - R).max(axis=(1, 2)))
    return out


def _floor(terms, spread, tol):
    """Term scales raised so that the term bound (0.1 tol T_f) admits the
    one-ulp spread."""
    return np.maximum(terms, spread / (0.1 * tol))


def _solver(mesh, p, phys, wall_flux, **kw):
    from paper_2508_17917_amd import Solver
    return Solver(p, mesh, gamma=phys.gamma, Pr=phys.Pr, mu=phys.mu, theta=phys.theta,
                  penalty_mode=phys.penalty_mode, C_pen=phys.C_pen, U_inf=phys.U_inf,
                  wall_flux=wall_flux, **kw)


def _inputs(case, printed):
    name, mk, p, over, recipe, vw = case
    mesh = mk()
    dg = build(mesh, p, wall_heat_flux=printed, **over)
    U = _rest_state(dg) if recipe == "rest" else _state(dg, recipe, 7)
    return mesh, dg, U


@pytest.mark.parametrize("printed", [False, True], ids=["adiabatic", "printed"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_wall_flux_rhs_all_forms(case, printed):
    from paper_2508_17917_amd import (DG_FP32_PERT, DG_FP64, DG_FP64_PERT, DG_WALL_ADIABATIC,
                                      DG_WALL_PRINTED)
    torch = _torch()
    name, _, p, _, _, vw = case
    mode = DG_WALL_PRINTED if printed else DG_WALL_ADIABATIC
    tag = "%s %s" % (name, "printed" if printed else "adiabatic")
    mesh, dg, U = _inputs(case, printed)
    want, parts = dg.rhs(U, vw, return_parts=True)
    # the other mode's oracle differs from this one by far more than the bound
    other = build(mesh, p, wall_heat_flux=not printed, **case[3]).rhs(U, vw)
    gap = np.abs(other[3] - want[3]).max()
    assert gap > 1e-6 * np.abs(want[3]).max(), gap
    Ud = _to_dev(torch, U)
    spread = _ulp_spread(dg, U, vw)

    _say("wall-flux rhs fp64 %s K=%d p=%d" % (tag, dg.mesh.K, p))
    s = _solver(mesh, p, dg.phys, mode, precision=DG_FP64)
    R = s.rhs(Ud, v_w=vw)
    torch.cuda.synchronize()
    _check(_from_dev(R), want, what="fp64 " + tag, terms=_floor(term_scale(parts), spread, 1e-12))
    # switching the mode on the same context gives the other mode's bits
    s.set_wall_flux(DG_WALL_ADIABATIC if printed else DG_WALL_PRINTED)
    Ro = s.rhs(Ud, v_w=vw)
    s.set_wall_flux(mode)
    assert torch.equal(s.rhs(Ud, v_w=vw), R)
    torch.cuda.synchronize()
    dgo = build(mesh, p, wall_heat_flux=not printed, **case[3])
    _check(_from_dev(Ro), other, what="fp64 switched " + tag,
           terms=_floor(term_scale(dgo.rhs(U, vw, return_parts=True)[1]), _ulp_spread(dgo, U, vw),
                        1e-12))
    s.close()

    _say("wall-flux rhs fp64-pert %s" % tag)
    s = _solver(mesh, p, dg.phys, mode, precision=DG_FP64_PERT)
    R = s.rhs(Ud, v_w=vw)
    torch.cuda.synchronize()
    _check_pert(_from_dev(R), want, TOL64, _floor(0.1 * term_scale(parts), spread, 10 * TOL64),
                "fp64-pert " + tag)
    s.close()

    _say("wall-flux rhs fp32-pert %s" % tag)
    s = _solver(mesh, p, dg.phys, mode, precision=DG_FP32_PERT)
    R = s.rhs(Ud, v_w=vw)
    torch.cuda.synchronize()
    _check_pert(_from_dev(R), want, TOL32, pert_term_scale(dg, parts, vw), "fp32-pert " + tag)
    s.close()

    _say("wall-flux rhs overint %s" % tag)
    oi = DGOracleOI(dg.mesh, dg.phys)
    want_oi, parts_oi = oi.rhs(U, vw, return_parts=True)
    spread_oi = _ulp_spread(oi, U, vw)
    s = _solver(mesh, p, dg.phys, mode, overintegration=True)
    R = s.rhs(Ud, v_w=vw)
    torch.cuda.synchronize()
    _check(_from_dev(R), want_oi, what="overint " + tag,
           terms=_floor(term_scale(parts_oi), spread_oi, 1e-12))
    s.close()


def test_printed_wall_flux_rk_step():
    """One LSERK step of the annulus at rest with the printed wall flux."""
    from paper_2508_17917_amd import DG_WALL_PRINTED
    torch = _torch()
    case = CASES[3]
    mesh, dg, U = _inputs(case, True)
    dt = 1e-4
    want, _ = dg.lserk_step(U, dt)
    terms = dt * _floor(term_scale(dg.rhs(U, return_parts=True)[1]), _ulp_spread(dg, U, (0.0, 0.0)),
                        1e-12)
    _say("wall-flux rk_step printed %s K=%d" % (case[0], dg.mesh.K))
    s = _solver(mesh, case[2], dg.phys, DG_WALL_PRINTED)
    Ud = _to_dev(torch, U)
    K1 = torch.zeros_like(Ud)
    s.rk_step(Ud, K1, dt)
    torch.cuda.synchronize()
    _check(_from_dev(Ud) - U, want - U, tol=1e-11, what="rk_step printed", terms=10 * terms)
    s.close()
