"""GPU parity of the HIP path against the FP64 oracle (needs an MI355X).

Tolerance (FP64), per conserved field f:
    max |R_gpu - R_oracle| <= max(1e-12 max|R_oracle,f|, 1e-13 T_f)
with T_f the largest magnitude of the oracle's separate volume, surface and
theta contributions to field f.  The GPU evaluates the strong form and the
oracle the weak form; they agree in exact arithmetic, so the difference is
rounding of the individual terms.  Where a field's right-hand side is a small
remainder of large terms (near free stream, or the transverse momentum of a
flow along x) that rounding is set by T_f, not by R_f.  Inputs are seeded
synthetic states of the workloads' shapes (meshgen), identical on both sides.
"""
import numpy as np
import pytest

import meshgen as mg
from oracle import fsi
from oracle.dg import LSERK_A, LSERK_B
from tests.oracle_helpers import build

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(msg):
    print("[gpu-case] " + msg, flush=True)


def _solver(mesh, p, phys):
    from paper_2508_17917_amd import Solver
    return Solver(p, mesh, gamma=phys.gamma, Pr=phys.Pr, mu=phys.mu, theta=phys.theta,
                  penalty_mode=phys.penalty_mode, C_pen=phys.C_pen, U_inf=phys.U_inf)


def _to_dev(torch, U):
    return torch.from_numpy(np.ascontiguousarray(np.transpose(U, (2, 0, 1)))).cuda()


def _from_dev(T):
    return np.transpose(T.cpu().numpy(), (1, 2, 0))


def term_scale(parts):
    return np.array([max(np.abs(parts[k][f]).max() for k in ("vol", "surf", "theta"))
                     for f in range(4)])


def _check(got, want, tol=TOL, what="", terms=None):
    """Per field: err <= tol max|R| (the relative bound), else <= 0.1 tol T_f
    (the term-scale bound); prints err/max|R| and which bound held."""
    report = []
    for f in range(4):
        scale = np.abs(want[f]).max()
        err = np.abs(got[f] - want[f]).max()
        rel = err / scale if scale > 0 else (0.0 if err == 0 else np.inf)
        branch = "rel" if err <= tol * scale else "terms"
        bound = tol * scale
        if terms is not None:
            bound = max(bound, 0.1 * tol * terms[f])
        report.append("f%d %.2e(%s)" % (f, rel, branch))
        assert err <= bound, "%s field %d: err %.3e scale %.3e ratio %.3e" % (
            what, f, err, scale, err / scale)
    print("[parity] %s err/max|R|: %s" % (what, " ".join(report)), flush=True)


CASES = [
    # name, mesh builder, p, physics overrides, state recipe, v_w
    ("vortex-periodic-p3", lambda: mg.periodic_square(5, 4, 10.0, 8.0), 3,
     dict(mu=3e-3, penalty_mode=1, C_pen=1.0, U_inf=mg.free_stream(0.3)), "vortex", (0.0, 0.0)),
    ("cylinder-p4", lambda: mg.ogrid(12, 5, 0.5, 6.0, 1.3), 4,
     dict(mu=2e-3, penalty_mode=0, C_pen=1.0), "noise", (0.0, 0.0)),
    ("cylinder-moving-p4", lambda: mg.ogrid(10, 4, 0.5, 5.0, 1.3), 4,
     dict(mu=2e-3, penalty_mode=0, C_pen=1.0), "noise", (0.013, -0.021)),
    ("cylinder-p5-iipg", lambda: mg.ogrid(9, 4, 0.5, 5.0, 1.3), 5,
     dict(mu=2e-3, penalty_mode=0, C_pen=0.01, theta=0.0), "noise", (0.0, 0.0)),
    ("periodic-p6", lambda: mg.periodic_square(4, 4, 10.0, 10.0), 6,
     dict(mu=3e-3, penalty_mode=0, C_pen=1.0, U_inf=mg.free_stream(0.3)), "fourier", (0.0, 0.0)),
    ("two-elements-p2", lambda: mg.periodic_square(1, 1, 1.0, 1.0), 2,
     dict(mu=1e-2, penalty_mode=1, C_pen=1.0), "fourier", (0.0, 0.0)),
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
def test_rhs_parity(case):
    torch = _torch()
    name, mk, p, over, recipe, vw = case
    mesh = mk()
    dg = build(mesh, p, **over)
    U = _state(dg, recipe, 7)
    want, parts = dg.rhs(U, vw, return_parts=True)
    _say("rhs %s K=%d p=%d" % (name, dg.mesh.K, p))
    s = _solver(mesh, p, dg.phys)
    Ud = _to_dev(torch, U)
    R = s.rhs(Ud, v_w=vw)
    torch.cuda.synchronize()
    _check(_from_dev(R), want, what=name, terms=term_scale(parts))
    # bitwise reproducible
    R2 = s.rhs(Ud, v_w=vw)
    torch.cuda.synchronize()
    assert torch.equal(R, R2)
    if "ragged" in name:
        # every launch shape (waves per workgroup, persistent or 1-3 tiles per
        # wave) covers the partly filled last tile with the same bits
        for waves in (2, 4):
            for grid in (0, 1, 2, 3):
                s.set_tuning(waves, grid)
                assert torch.equal(s.rhs(Ud, v_w=vw), R), (waves, grid)
    s.close()


RK_CASES = CASES[:3] + CASES[-2:]


@pytest.mark.parametrize("case", RK_CASES, ids=[c[0] for c in RK_CASES])
def test_rk_step_parity(case):
    torch = _torch()
    name, mk, p, over, recipe, vw = case
    mesh = mk()
    dg = build(mesh, p, **over)
    U = _state(dg, recipe, 11)
    dt = 1e-4
    want, _ = dg.lserk_step(U, dt, vw)
    terms = dt * term_scale(dg.rhs(U, vw, return_parts=True)[1])
    _say("rk_step %s K=%d p=%d" % (name, dg.mesh.K, p))
    s = _solver(mesh, p, dg.phys)
    Ud = _to_dev(torch, U)
    K1 = torch.full_like(Ud, float("nan"))  # A_1 = 0: K1 is never read
    s.rk_step(Ud, K1, dt, v_w=vw)
    torch.cuda.synchronize()
    got = _from_dev(Ud)
    # compare increments (U changes by O(dt |R|))
    _check(got - U, want - U, tol=1e-11, what=name, terms=10 * terms)
    # the stage entry point chained by hand gives the same bits
    Ua = _to_dev(torch, U)
    Ub = torch.empty_like(Ua)
    K1b = torch.zeros_like(Ua)
    for i, (a, b) in enumerate(zip(LSERK_A, LSERK_B)):
        src, dst = (Ua, Ub) if i % 2 == 0 else (Ub, Ua)
        s.rk_stage(src, dst, K1b, a, b, dt, v_w=vw)
    torch.cuda.synchronize()
    assert torch.equal(Ub, Ud)
    s.close()


def test_force_parity():
    torch = _torch()
    mesh = mg.ogrid(16, 4, 0.5, 5.0, 1.3)
    for p, vw in [(3, (0.0, 0.0)), (4, (0.01, -0.02))]:
        dg = build(mesh, p, mu=5e-3, penalty_mode=0, C_pen=1.0)
        U = _state(dg, "noise", 5)
        want = fsi.wall_force(dg, U, vw)
        _say("force p=%d" % p)
        s = _solver(mesh, p, dg.phys)
        Ud = _to_dev(torch, U)
        got = s.force(Ud, v_w=vw)
        out = torch.zeros(3, dtype=torch.float64, device="cuda")
        s.force_device(Ud, out, v_w=vw)
        assert np.array_equal(out.cpu().numpy(), got)
        # the net force is a small remainder of the pressure integral around the
        # closed wall: compare against that integral's size, p_inf x perimeter
        scale = (1.0 / 1.4) * np.pi
        assert np.abs(got - want).max() <= 1e-12 * scale, (got, want)
        s.close()


def test_rhs_parity_cylinder20k_full_size():
    """The benchmark workload at full size (80 x 128 O-grid, K = 20480, p = 4)."""
    torch = _torch()
    w = mg.workload("cylinder20k")
    dg = build(w["mesh"], w["p"], gamma=w["gamma"], Pr=w["Pr"], mu=w["mu"], theta=w["theta"],
               penalty_mode=w["penalty_mode"], C_pen=1.0, U_inf=w["U_inf"])
    U = mg.noisy_free_stream((4,) + dg.mesh.x.shape, dg.phys.U_inf, mg.rng_for(1))
    want, parts = dg.rhs(U, return_parts=True)
    _say("rhs cylinder20k K=%d" % dg.mesh.K)
    s = _solver(w["mesh"], w["p"], dg.phys)
    R = s.rhs(_to_dev(torch, U))
    torch.cuda.synchronize()
    _check(_from_dev(R), want, what="cylinder20k", terms=term_scale(parts))
    s.close()


def test_rk_steps_equal_repeated_steps():
    """The multi-step call (state alternating between two buffers, force
    after every step) gives the bits of repeated single steps, for an even
    and an odd step count."""
    torch = _torch()
    mesh = mg.ogrid(12, 5, 0.5, 6.0, 1.3)
    dg = build(mesh, 4, mu=2e-3, penalty_mode=0, C_pen=1.0)
    U = _state(dg, "noise", 3)
    s = _solver(mesh, 4, dg.phys)
    vw = (0.0, 0.01)
    for n in (2, 3):
        _say("rk_steps n=%d" % n)
        Ua, Ka = _to_dev(torch, U), torch.zeros(s.K, 4, s.Np, dtype=torch.float64, device="cuda")
        Fa = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
        s.rk_steps(Ua, Ka, n, 1e-4, v_w=vw, force=Fa)
        Ub, Kb = _to_dev(torch, U), torch.zeros_like(Ka)
        Fb = torch.zeros_like(Fa)
        for i in range(n):
            s.rk_step(Ub, Kb, 1e-4, v_w=vw)
            s.force_device(Ub, Fb[i], v_w=vw)
        torch.cuda.synchronize()
        assert torch.equal(Ua, Ub) and torch.equal(Fa, Fb)
    s.close()


def test_rk_steps_with_forces_at_full_size():
    """cylinder20k (K = 20,480, p = 4, FP32 perturbation form): the
    multi-step call with a force after every step equals single steps with a
    force after each, bit for bit, over an odd number of steps."""
    torch = _torch()
    from paper_2508_17917_amd import Solver
    w = mg.workload("cylinder20k")
    s = Solver(4, w["mesh"], gamma=w["gamma"], Pr=w["Pr"], mu=w["mu"], theta=w["theta"],
               penalty_mode=w["penalty_mode"], C_pen=w["C_pen"], U_inf=w["U_inf"], precision=2)
    U0 = mg.noisy_free_stream((4, s.Np, s.K), w["U_inf"], mg.rng_for(1))
    U0 = torch.from_numpy(np.ascontiguousarray(np.transpose(U0, (2, 0, 1)))).cuda()
    n, dt, vw = 7, 1e-7, (0.0, 0.002)
    _say("rk_steps with forces cylinder20k n=%d" % n)
    Ua, Ka = U0.clone(), torch.zeros_like(U0)
    Fa = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
    s.rk_steps(Ua, Ka, n, dt, v_w=vw, force=Fa)
    Ub, Kb = U0.clone(), torch.zeros_like(U0)
    Fb = torch.zeros_like(Fa)
    for i in range(n):
        s.rk_step(Ub, Kb, dt, v_w=vw)
        s.force_device(Ub, Fb[i], v_w=vw)
    torch.cuda.synchronize()
    assert torch.equal(Ua, Ub) and torch.equal(Fa, Fb)
    s.close()


def test_conservation_and_free_stream_at_large_size():
    """Properties that hold at any size, on a 320x320x2 periodic mesh
    (K = 204,800, p = 4): the discrete integral sum_K J_K 1^T M R_K of every
    field vanishes to rounding (local conservation), and the free stream is
    a steady state, in plain FP64 and in the FP32 perturbation form."""
    torch = _torch()
    from paper_2508_17917_amd import Solver
    mesh = mg.periodic_square(320, 320, 10.0, 10.0)
    U_inf = mg.free_stream(0.3)
    for prec in (0, 2):
        s = Solver(4, mesh, gamma=1.4, Pr=0.72, mu=3e-3, theta=1.0, penalty_mode=0, C_pen=1.0,
                   U_inf=U_inf, precision=prec)
        _say("large periodic K=%d precision=%d" % (s.K, prec))
        x, y = s.nodes()
        U = mg.fourier_modes(x.T, y.T, np.random.default_rng(9), L=10.0, amp=1e-2,
                             q0=(1.0, 0.3, 0.0, 1.0 / 1.4))
        R = s.rhs(_to_dev(torch, U)).cpu().numpy()          # (K, 4, Np)
        M = s.table("M").reshape(s.Np, s.Np)
        geo = s.table("geo").reshape(s.K, 16)
        J = 1.0 / (geo[:, 0] * geo[:, 3] - geo[:, 1] * geo[:, 2])
        w = M.sum(axis=0)
        tot = np.einsum("kcn,n,k->c", R, w, J)
        mag = np.einsum("kcn,n,k->c", np.abs(R), w, J)
        # the identity is exact for the discrete operator; what remains is the
        # rounding of each R_K, ~1e-13 (FP64) / ~1e-7 (FP32) of its volume and
        # surface terms, which exceed |R_K| by one to two orders here
        _say("conservation precision=%d: %s of %s" % (prec, np.abs(tot), mag))
        assert np.all(np.abs(tot) <= (1e-11 if prec == 0 else 1e-6) * mag), (prec, tot, mag)
        Uf = np.broadcast_to(np.asarray(U_inf)[None, :, None], (s.K, 4, s.Np)).copy()
        Rf = s.rhs(torch.from_numpy(Uf).cuda()).abs().max().item()
        # FP64: rounding of O(1) fluxes over h = 1/32 (the oracle pin: 1e-12 p^2 at h = 2/3);
        # the perturbation form forms nothing from U_inf: exactly zero
        assert Rf <= (5e-10 if prec == 0 else 0.0), (prec, Rf)
        s.close()
