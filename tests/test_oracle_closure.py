"""Pins of the closure oracle: restriction / interpolation against polynomial
exactness and L2-orthogonality, the network's gradients against central
finite differences, GELU and Adam against closed forms, bfloat16 rounding
against the format's definition."""
import math

import numpy as np
import pytest
from scipy.special import erf

from oracle import closure as C
from oracle.nodes import RefElement


def _poly(r, s, a, b):
    return r ** a * s ** b


@pytest.mark.parametrize("hi,lo", [(4, 2), (3, 1), (6, 2)])
def test_restriction_and_interpolation_exact_on_low_degree(hi, lo):
    P, I = C.restriction(hi, lo), C.interpolation(lo, hi)
    H, L = RefElement(hi), RefElement(lo)
    for a in range(lo + 1):
        for b in range(lo + 1 - a):
            assert np.abs(P @ _poly(H.r, H.s, a, b) - _poly(L.r, L.s, a, b)).max() < 1e-12
            assert np.abs(I @ _poly(L.r, L.s, a, b) - _poly(H.r, H.s, a, b)).max() < 1e-12
    assert np.abs(P @ I - np.eye(L.Np)).max() < 1e-12


@pytest.mark.parametrize("hi,lo", [(4, 2), (5, 3)])
def test_restriction_is_the_l2_projection(hi, lo):
    """f - I P f is M-orthogonal to every polynomial of degree <= lo (the
    reference mass matrix M of order hi integrates degree <= 2 hi exactly)."""
    P, I = C.restriction(hi, lo), C.interpolation(lo, hi)
    H = RefElement(hi)
    rng = np.random.default_rng(3)
    f = rng.standard_normal(H.Np)          # a random degree-hi polynomial (nodal)
    res = f - I @ (P @ f)
    for a in range(lo + 1):
        for b in range(lo + 1 - a):
            q = _poly(H.r, H.s, a, b)
            assert abs(res @ H.M @ q) < 1e-12
    # and the projection of a degree-hi monomial with a degree > lo part is not
    # the identity (a dropped-mode mistake would pass the exactness test above)
    g = _poly(H.r, H.s, hi, 0)
    assert np.abs(g - I @ (P @ g)).max() > 1e-3


def test_gelu_closed_forms():
    z = np.linspace(-6.0, 6.0, 41)
    assert C.gelu(np.array(0.0)) == 0.0
    assert np.abs(C.gelu(z) - C.gelu(-z) - z).max() < 1e-14
    assert abs(C.gelu(np.array(1.0)) - 0.5 * (1.0 + math.erf(1.0 / math.sqrt(2.0)))) < 1e-15
    h = 1e-6
    fd = (C.gelu(z + h) - C.gelu(z - h)) / (2.0 * h)
    assert np.abs(fd - C.gelu_grad(z)).max() < 1e-8
    assert np.abs(C.gelu(z) - 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))).max() == 0.0


def _params(rng, n_in, h, n_out):
    return {"W1": rng.standard_normal((h, n_in)) / math.sqrt(n_in), "b1": 0.1 * rng.standard_normal(h),
            "W2": rng.standard_normal((h, h)) / math.sqrt(h), "b2": 0.1 * rng.standard_normal(h),
            "W3": rng.standard_normal((n_out, h)) / math.sqrt(h), "b3": 0.1 * rng.standard_normal(n_out)}


def test_gradients_match_central_differences():
    rng = np.random.default_rng(11)
    p = _params(rng, 5, 7, 3)
    X = rng.standard_normal((6, 5))
    T = rng.standard_normal((6, 3))
    _, g = C.loss_and_grads(p, X, T)
    h = 1e-6
    for k in p:
        flat = p[k].reshape(-1)
        for idx in range(flat.size):
            q = {kk: vv.copy() for kk, vv in p.items()}
            q[k].reshape(-1)[idx] += h
            lp, _ = C.loss_and_grads(q, X, T)
            q[k].reshape(-1)[idx] -= 2 * h
            lm, _ = C.loss_and_grads(q, X, T)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[k].reshape(-1)[idx]) <= 1e-7 * max(1.0, abs(fd)), (k, idx)


def test_adam_first_step_is_a_signed_step():
    """With m = v = 0, step 1: m^ = g and v^ = g^2, so p moves by -lr g/(|g| + eps)."""
    p = {"w": np.array([1.0, -2.0, 0.5])}
    g = {"w": np.array([0.3, -4.0, 1e-3])}
    z = {"w": np.zeros(3)}
    out, m, v = C.adam_step(p, g, z, z, 1, lr=0.01, eps=1e-12)
    assert np.abs(out["w"] - (p["w"] - 0.01 * np.sign(g["w"]))).max() < 1e-9
    assert np.allclose(m["w"], 0.1 * g["w"]) and np.allclose(v["w"], 0.001 * g["w"] ** 2)


def test_round_bf16_definition():
    one = np.float32(1.0)
    ulp = 2.0 ** -7                       # bfloat16 spacing at 1
    cases = [(1.0, 1.0), (1.0 + ulp, 1.0 + ulp),
             (1.0 + ulp / 2, 1.0),               # tie -> even (1.0)
             (1.0 + 3 * ulp / 2, 1.0 + 2 * ulp),  # tie -> even (1 + 2 ulp)
             (1.0 + ulp / 2 + 2.0 ** -20, 1.0 + ulp),
             (-3.0, -3.0), (0.0, 0.0)]
    for x, want in cases:
        assert C.round_bf16(np.float32(x)) == np.float32(want), x
    x = np.random.default_rng(0).standard_normal(1000).astype(np.float32)
    r = C.round_bf16(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8)
    assert np.all(r.view(np.uint32) & 0xFFFF == 0)
    del one


def test_features_targets_apply_roundtrip():
    """apply_closure(P U, I, targets(U)) = U for an order-hi state, and the
    features of the restricted state equal those computed through P."""
    rng = np.random.default_rng(5)
    P, I = C.restriction(4, 2), C.interpolation(2, 4)
    U = rng.standard_normal((4, 15, 9))
    geo = rng.standard_normal((9, 4))
    Uinf = np.array([1.0, 0.2, 0.0, 1.8])
    T = C.targets(U, P, I)
    Ulo = np.einsum("mn,cnk->cmk", P, U)
    assert np.abs(C.apply_closure(Ulo, I, T) - U).max() < 1e-12
    assert np.abs(C.features(U, geo, Uinf, P) - C.features(Ulo, geo, Uinf)).max() < 1e-13
    assert C.features(Ulo, geo, Uinf).shape == (9, 28)


def test_corrector_rows_round_trip_and_layout():
    """The corrector's target rows and its update are inverse to each other,
    and both use the samples' field-major layout (element k, field f, node n
    at column f Np + n)."""
    rng = np.random.default_rng(5)
    U = rng.standard_normal((4, 6, 7))
    U_ref = U + 1e-3 * rng.standard_normal(U.shape)
    T = C.drift_targets(U_ref, U)
    assert T.shape == (7, 24)
    for k, f, n in ((0, 0, 0), (3, 2, 5), (6, 3, 1)):
        assert T[k, f * 6 + n] == U_ref[f, n, k] - U[f, n, k]
    assert np.abs(C.apply_correction(U, T) - U_ref).max() <= 1e-15
    assert np.array_equal(C.drift_targets(U, U), np.zeros((7, 24)))
    # the layout of the samples' state columns is the same
    geo = rng.standard_normal((7, 4))
    X = C.features(U + 1.0, geo, np.ones(4))
    assert np.abs(X[:, :24] - C.drift_targets(U, np.zeros_like(U))).max() <= 1e-15


def test_free_stream_sample_is_the_sample_of_the_free_stream():
    """The free-stream sample equals the sample of a uniform U_inf state (order
    lo directly, and order hi through the restriction, which keeps constants)."""
    rng = np.random.default_rng(6)
    U_inf = np.array([1.0, 0.2, 0.0, 1.8])
    geo = rng.standard_normal((5, 4))
    X0 = C.free_features(geo, 6)
    lo_state = np.broadcast_to(U_inf[:, None, None], (4, 6, 5)).copy()
    hi_state = np.broadcast_to(U_inf[:, None, None], (4, 15, 5)).copy()
    assert np.abs(C.features(lo_state, geo, U_inf) - X0).max() == 0.0
    assert np.abs(C.features(hi_state, geo, U_inf, C.restriction(4, 2)) - X0).max() < 1e-13
