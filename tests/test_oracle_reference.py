"""Pins of the oracle's reference-element operators (CPU).

Each check compares against something the oracle does not compute itself:
library Gauss-Jacobi rules, closed-form monomial integrals on the simplex,
the closed-form Legendre-Gauss-Lobatto weights, the triangle's symmetry
group and the summation-by-parts identity of exact nodal operators.
"""
import math

import numpy as np
import pytest
from scipy.special import eval_jacobi, roots_jacobi, eval_legendre

from oracle import nodes

ORDERS = [1, 2, 3, 4, 5, 6, 7, 8]


@pytest.mark.parametrize("ab", [(0, 0), (1, 1), (3, 0), (7, 0), (2, 5)])
def test_jacobi_orthonormal_against_library_quadrature(ab):
    a, b = ab
    x, w = roots_jacobi(20, a, b)
    P = np.stack([nodes.jacobi_p(x, a, b, n) for n in range(10)])
    assert np.abs((P * w) @ P.T - np.eye(10)).max() < 1e-13
    # proportional to the library's (unnormalised) Jacobi polynomials, positive factor
    xs = np.linspace(-0.9, 0.9, 7)
    for n in range(1, 8):
        mine, lib = nodes.jacobi_p(xs, a, b, n), eval_jacobi(n, a, b, xs)
        c = np.dot(mine, lib) / np.dot(lib, lib)
        assert c > 0 and np.abs(mine - c * lib).max() < 1e-12 * np.abs(mine).max()


@pytest.mark.parametrize("N", ORDERS)
def test_lgl_points_and_weights(N):
    x = nodes.gauss_lobatto(N)
    # closed-form LGL weights 2 / (N (N+1) P_N(x)^2) integrate degree 2N-1 exactly
    w = 2.0 / (N * (N + 1) * eval_legendre(N, x) ** 2)
    for d in range(2 * N):
        exact = (1.0 - (-1.0) ** (d + 1)) / (d + 1)
        assert abs(np.dot(w, x ** d) - exact) < 1e-13
    ref = nodes.RefElement(N)
    # the face nodes of the warp & blend set are the LGL points; the face
    # quadrature weights (column sums of the face mass) are the LGL weights
    for f in range(3):
        xi = [ref.r, ref.s, -ref.s][f][ref.Fmask[f]]
        assert np.abs(np.sort(xi) - x).max() < 1e-13
        assert np.abs(np.sort(ref.wface[f]) - np.sort(w)).max() < 1e-13


def _simplex_monomial_integral(a, b):
    """int_{K^} r^a s^b dr ds via r = 2 xi - 1, s = 2 eta - 1 and the Dirichlet integral."""
    tot = 0.0
    for i in range(a + 1):
        for j in range(b + 1):
            c = math.comb(a, i) * math.comb(b, j) * 2.0 ** (i + j) * (-1.0) ** (a - i + b - j)
            tot += c * math.factorial(i) * math.factorial(j) / math.factorial(i + j + 2)
    return 4.0 * tot


@pytest.mark.parametrize("N", ORDERS)
def test_nodes_symmetric_and_inside(N):
    x, y = nodes.nodes_equilateral(N)
    pts = np.stack([x, y], axis=1)
    assert len(x) == (N + 1) * (N + 2) // 2
    for k in range(3):
        ang = 2.0 * math.pi * k / 3.0
        R = np.array([[math.cos(ang), -math.sin(ang)], [math.sin(ang), math.cos(ang)]])
        for mirror in (False, True):
            q = pts.copy()
            if mirror:
                q[:, 0] = -q[:, 0]
            q = q @ R.T
            d = np.linalg.norm(q[:, None, :] - pts[None, :, :], axis=2).min(axis=1)
            assert d.max() < 1e-12
    r, s = nodes.nodes_rs(N)
    assert r.min() > -1 - 1e-13 and s.min() > -1 - 1e-13 and (r + s).max() < 1e-13


@pytest.mark.parametrize("N", ORDERS)
def test_pkd_orthonormal_with_collapsed_gauss_rule(N):
    # tensor Gauss-Jacobi rule in (a, b): weight (1 - b) from the collapse
    qa, wa = roots_jacobi(N + 2, 0, 0)
    qb, wb = roots_jacobi(N + 2, 1, 0)
    A, B = np.meshgrid(qa, qb, indexing="ij")
    W = np.outer(wa, wb) * 0.5
    r = 0.5 * (1.0 + A) * (1.0 - B) - 1.0
    s = B
    V = nodes.vandermonde_2d(N, r.ravel(), s.ravel())
    G = (V * W.ravel()[:, None]).T @ V
    assert np.abs(G - np.eye(G.shape[0])).max() < 1e-12


@pytest.mark.parametrize("N", ORDERS)
def test_dr_ds_exact_on_monomials(N):
    ref = nodes.RefElement(N)
    r, s = ref.r, ref.s
    for a in range(N + 1):
        for b in range(N + 1 - a):
            f = r ** a * s ** b
            fr = a * r ** (a - 1) * s ** b if a else 0 * f
            fs = b * r ** a * s ** (b - 1) if b else 0 * f
            assert np.abs(ref.Dr @ f - fr).max() < 5e-12 * N ** 2
            assert np.abs(ref.Ds @ f - fs).max() < 5e-12 * N ** 2


@pytest.mark.parametrize("N", ORDERS)
def test_mass_matrix_integrates_monomials(N):
    ref = nodes.RefElement(N)
    ones = np.ones(ref.Np)
    for a in range(N + 1):
        for b in range(N + 1 - a):
            got = ones @ ref.M @ (ref.r ** a * ref.s ** b)
            assert abs(got - _simplex_monomial_integral(a, b)) < 1e-12


@pytest.mark.parametrize("N", ORDERS)
def test_summation_by_parts(N):
    """M Dr + Dr^T M = E_1 - E_2 and M Ds + Ds^T M = E_1 - E_0 (reference normals x lengths)."""
    ref = nodes.RefElement(N)
    Nfp = ref.Nfp
    Ef = []
    for f in range(3):
        E = np.zeros((ref.Np, ref.Np))
        blk = ref.E[ref.Fmask[f], f * Nfp:(f + 1) * Nfp]
        E[np.ix_(ref.Fmask[f], ref.Fmask[f])] = blk
        Ef.append(E)
    # face 0: n=(0,-1), |e|/2 = 1; face 1: n=(1,1)/sqrt2, |e|/2 = sqrt2; face 2: n=(-1,0), 1
    lhs_r = ref.M @ ref.Dr + ref.Dr.T @ ref.M
    lhs_s = ref.M @ ref.Ds + ref.Ds.T @ ref.M
    assert np.abs(lhs_r - (Ef[1] - Ef[2])).max() < 1e-12 * N ** 2
    assert np.abs(lhs_s - (Ef[1] - Ef[0])).max() < 1e-12 * N ** 2


@pytest.mark.parametrize("N", [2, 4, 6])
def test_lift_reproduces_face_integrals(N):
    ref = nodes.RefElement(N)
    rng = np.random.default_rng(N)
    g = rng.standard_normal(3 * ref.Nfp)
    assert np.abs(ref.M @ ref.LIFT @ g - ref.E @ g).max() < 1e-12
    # theta lifts: M LIFTr = Dr^T E
    assert np.abs(ref.M @ ref.LIFTr - ref.Dr.T @ ref.E).max() < 1e-11 * N ** 2
