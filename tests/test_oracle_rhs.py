"""Pins of the oracle's right-hand side (CPU).

* free-stream preservation (periodic and all-far-field meshes, moving frame),
  and a uniform flow moving with the wall on a cylinder mesh;
* discrete conservation on periodic meshes (the paper's local conservation);
* the strong/weak integration-by-parts identity of the nodal operators;
* brute-force assembly of the weak form with independent cubature on a
  two-triangle mesh;
* the theta term is the adjoint of the viscous consistency term (SIPG
  symmetry, linearised at a constant state where G is frozen);
* the linearised operator at a constant state has no growing modes, which
  fixes the signs of the Roe upwinding, the penalty and the theta term.
"""
import numpy as np
import pytest
from scipy.special import roots_jacobi, roots_legendre

import meshgen as mg
from oracle import nodes
from tests.oracle_helpers import build, uniform


def ogrid_all_far(nt=10, nr=4):
    m = mg.ogrid(nt, nr, 0.5, 4.0, 1.3)
    ft = m["face_tag"].copy()
    ft[ft == 1] = 2
    return m, ft


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("vw", [(0.0, 0.0), (0.04, -0.13)])
def test_free_stream_preserved(p, vw):
    dg = build(mg.periodic_square(3, 3, 2.0, 2.0), p)
    U = uniform(dg, dg.phys.U_inf)
    assert np.abs(dg.rhs(U, vw)).max() < 1e-12 * p * p
    m, ft = ogrid_all_far()
    dg = build(m, p, face_tag=ft)
    U = uniform(dg, dg.phys.U_inf)
    assert np.abs(dg.rhs(U, vw)).max() < 1e-11 * p * p


@pytest.mark.parametrize("p", [2, 4])
def test_flow_moving_with_wall_is_steady(p):
    vw = (0.05, -0.03)
    Uinf = mg.free_stream(0.0)
    rho, E = Uinf[0], Uinf[3]
    Uw = np.array([rho, rho * vw[0], rho * vw[1], E + 0.5 * rho * (vw[0] ** 2 + vw[1] ** 2)])
    dg = build(mg.ogrid(10, 4, 0.5, 4.0, 1.3), p, U_inf=Uw)
    U = uniform(dg, Uw)
    assert np.abs(dg.rhs(U, vw)).max() < 1e-11 * p * p


@pytest.mark.parametrize("p", [1, 3, 5])
def test_conservation_periodic(p):
    dg = build(mg.periodic_square(4, 3, 3.0, 2.0), p, mu=0.05)
    x, y = dg.mesh.x, dg.mesh.y
    rng = np.random.default_rng(p)
    U = mg.fourier_modes(x, y, rng, L=1.0, amp=0.05) + 0.01 * rng.standard_normal((4,) + x.shape)
    R = dg.rhs(U, vw=(0.02, 0.01))
    tot = dg.integral(R)
    assert np.abs(tot).max() < 1e-12 * np.abs(R).max()


@pytest.mark.parametrize("p", [2, 4, 6])
def test_strong_equals_weak_volume(p):
    """Drw Fr + Dsw Fs = -(Dr Fr + Ds Fs) + LIFT(Fscale (F . n)|faces) for any nodal F."""
    m, ft = ogrid_all_far(8, 3)
    dg = build(m, p, face_tag=ft)
    ref, me = dg.ref, dg.mesh
    rng = np.random.default_rng(7)
    Fx = rng.standard_normal((4, ref.Np, me.K))
    Fy = rng.standard_normal((4, ref.Np, me.K))
    Fr = me.rx * Fx + me.ry * Fy
    Fs = me.sx * Fx + me.sy * Fy
    weak = np.einsum('ij,fjk->fik', ref.Drw, Fr) + np.einsum('ij,fjk->fik', ref.Dsw, Fs)
    fn = Fx[:, ref.Fmask, :] * me.nx[None, :, None, :] + Fy[:, ref.Fmask, :] * me.ny[None, :, None, :]
    lifted = np.einsum('ij,fjk->fik', ref.LIFT,
                       (me.Fscale[None, :, None, :] * fn).reshape(4, 3 * ref.Nfp, me.K))
    strong = -(np.einsum('ij,fjk->fik', ref.Dr, Fr) + np.einsum('ij,fjk->fik', ref.Ds, Fs)) + lifted
    assert np.abs(weak - strong).max() < 1e-11 * np.abs(weak).max()


def test_brute_force_weak_form_two_triangles():
    """Assemble M dU/dt = int F.grad(l) - int H_m l + int q.grad(l) with independent cubature."""
    p = 3
    dg = build(mg.periodic_square(1, 1, 1.3, 0.9), p, mu=0.03)
    ref, me = dg.ref, dg.mesh
    rng = np.random.default_rng(11)
    U = mg.fourier_modes(me.x, me.y, rng, L=1.0, amp=0.1) + 0.02 * rng.standard_normal((4, ref.Np, me.K))
    R, parts = dg.rhs(U, vw=(0.03, 0.0), return_parts=True)
    vinv = np.linalg.inv(ref.V)
    # volume cubature: collapsed Gauss-Jacobi, exact for degree <= 2(p+2)-1
    qa, wa = roots_jacobi(p + 2, 0, 0)
    qb, wb = roots_jacobi(p + 2, 1, 0)
    A, B = np.meshgrid(qa, qb, indexing="ij")
    W = (np.outer(wa, wb) * 0.5).ravel()
    rq = (0.5 * (1 + A) * (1 - B) - 1).ravel()
    sq = B.ravel()
    Lq = nodes.vandermonde_2d(p, rq, sq) @ vinv                 # l_j at cubature points
    Vr, Vs = nodes.grad_vandermonde_2d(p, rq, sq)
    Lr, Ls = Vr @ vinv, Vs @ vinv
    # face cubature: Gauss-Legendre in the face parameter xi
    gx, gw = roots_legendre(p + 2)
    for k in range(me.K):
        J = me.J[k]
        rhs_k = np.zeros((4, ref.Np))
        Fxq = Lq @ parts["Fx"][:, :, k].T                        # (nq, 4)
        Fyq = Lq @ parts["Fy"][:, :, k].T
        dlx = me.rx[k] * Lr + me.sx[k] * Ls                      # (nq, Np)
        dly = me.ry[k] * Lr + me.sy[k] * Ls
        rhs_k += J * ((dlx * W[:, None]).T @ Fxq + (dly * W[:, None]).T @ Fyq).T
        for f in range(3):
            if f == 0:
                rf, sf = gx, -np.ones_like(gx)
            elif f == 1:
                rf, sf = -gx, gx
            else:
                rf, sf = -np.ones_like(gx), -gx
            Lf = nodes.vandermonde_2d(p, rf, sf) @ vinv          # volume basis on the face
            # face values: 1D interpolation of the nodal H_m / q along the face
            xi_nodes = [ref.r, ref.s, -ref.s][f][ref.Fmask[f]]
            V1 = nodes.vandermonde_1d(p, xi_nodes)
            I1 = nodes.vandermonde_1d(p, gx) @ np.linalg.inv(V1)
            Hq = I1 @ parts["Hm"][:, f, :, k].T                  # (ng, 4)
            qxq = I1 @ parts["qx"][:, f, :, k].T
            qyq = I1 @ parts["qy"][:, f, :, k].T
            Vrf, Vsf = nodes.grad_vandermonde_2d(p, rf, sf)
            dlxf = me.rx[k] * (Vrf @ vinv) + me.sx[k] * (Vsf @ vinv)
            dlyf = me.ry[k] * (Vrf @ vinv) + me.sy[k] * (Vsf @ vinv)
            sJ = me.sJ[f, k]
            rhs_k -= sJ * ((Lf * gw[:, None]).T @ Hq).T
            rhs_k += sJ * ((dlxf * gw[:, None]).T @ qxq + (dlyf * gw[:, None]).T @ qyq).T
        dudt = np.linalg.solve(J * ref.M, rhs_k.T).T
        assert np.abs(dudt - R[:, :, k]).max() < 1e-11 * np.abs(R).max()


def _linearise(fun, U0, eps=1e-6):
    n = U0.size
    cols = []
    for i in range(n):
        d = np.zeros(n)
        d[i] = eps
        d = d.reshape(U0.shape)
        cols.append(((fun(U0 + d) - fun(U0 - d)) / (2 * eps)).ravel())
    return np.stack(cols, axis=1)


def test_theta_term_is_adjoint_of_consistency_term():
    p = 2
    dg = build(mg.periodic_square(2, 1, 1.0, 0.6), p, mu=0.05, theta=1.0)
    ref, me = dg.ref, dg.mesh
    U0 = uniform(dg, mg.free_stream(0.25))

    def theta_part(U):
        return dg.rhs(U, return_parts=True)[1]["theta"]

    def consistency_part(U):
        return dg.rhs(U, return_parts=True)[1]["surf_visc"]

    Lt = _linearise(theta_part, U0)
    Lc = _linearise(consistency_part, U0)
    # (M^K)-weighted operators: Mt[(f,i,k),(g,j,l)] = J_k M_ij Lt[...]
    MJ = np.einsum('ij,k->ijk', ref.M, me.J)
    W = np.zeros((4, ref.Np, me.K, 4, ref.Np, me.K))
    for f in range(4):
        for k in range(me.K):
            W[f, :, k, f, :, k] = MJ[:, :, k]
    W = W.reshape(Lt.shape)
    # the consistency part lifted here is -int {G grad U}.n l with H_m's sign, i.e. +c(U, l)
    a = W @ Lt
    b = (W @ Lc).T
    assert np.abs(a - b).max() < 1e-6 * np.abs(a).max()
    dg.phys.theta = 0.0
    assert np.abs(dg.rhs(U0 * 1.001, return_parts=True)[1]["theta"]).max() == 0.0


@pytest.mark.parametrize("theta", [1.0, 0.0])
def test_linearised_operator_has_no_growing_modes(theta):
    p = 2
    dg = build(mg.periodic_square(2, 2, 1.0, 1.0), p, mu=0.02, theta=theta, C_pen=1.0)
    U0 = uniform(dg, mg.free_stream(0.3))
    L = _linearise(lambda U: dg.rhs(U), U0)
    lam = np.linalg.eigvals(L)
    assert lam.real.max() < 1e-6 * np.abs(lam).max()
