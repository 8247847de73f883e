"""Learned closure: restriction/interpolation between orders and a plain MLP
(oracle; test infrastructure -- only tests, smoke() and the benchmark's CPU
leg use it).

Closure protocol (a spec extension, not in the paper):

* restriction Pi_lo: the L2 projection of an order-p_hi nodal field onto
  polynomials of degree <= p_lo, evaluated at the order-p_lo nodes.  With the
  orthonormal PKD basis the projection is the truncation of the modal
  coefficients c = V_hi^-1 u to the modes of degree i + j <= p_lo;
* interpolation I: the order-p_lo nodal field evaluated at the order-p_hi
  nodes (exact, degree p_lo <= p_hi);
* sample of element k: input x = [Pi_lo(U - U_inf) (Np_lo nodes x 4 fields,
  field-major), rx, ry, sx, sy], target t = U_hi - I Pi_lo U_hi
  (Np_hi x 4, field-major);
* corrector of the order-lo solve: target t = Pi_lo U_hi(t + m dt) -
  Phi_lo^m(Pi_lo U_hi(t)) (the drift of m order-lo steps from the restricted
  state; Np_lo x 4, field-major), input the sample of the order-lo state
  after those m steps; applied as U_lo + y(x) - y(x0) every m steps, x0 the
  free stream's sample (state columns zero), and the reconstruction likewise
  as I U_lo + y(x) - y(x0);
* network: y = W3 g(W2 g(W1 x + b1) + b2) + b3 with the exact-erf GELU g,
  on normalised x and t (per-column mean and standard deviation), loss the
  mean of (y - t)^2 over samples and outputs, Adam with bias correction.

Each step is written out in FP64 in the plainest form; the gradients are
the chain rule by hand (pinned against central finite differences).
"""
import numpy as np
from scipy.special import erf

from .nodes import RefElement, mode_indices, rs_to_ab, pkd_mode


# ---------------------------------------------------------------- operators
def _low_mode_matrix(N_hi, N_lo, r, s):
    """Values at (r, s) of the order-N_hi PKD modes of degree <= N_lo, in the
    order-N_hi mode order (columns), restricted to those modes."""
    a, b = rs_to_ab(r, s)
    cols = [pkd_mode(a, b, i, j) for (i, j) in mode_indices(N_hi) if i + j <= N_lo]
    return np.stack(cols, axis=1)


def restriction(N_hi, N_lo):
    """(Np_lo x Np_hi) matrix of Pi_lo: nodal order N_hi -> nodal order N_lo."""
    hi, lo = RefElement(N_hi), RefElement(N_lo)
    keep = [m for m, (i, j) in enumerate(mode_indices(N_hi)) if i + j <= N_lo]
    vinv = np.linalg.inv(hi.V)
    return _low_mode_matrix(N_hi, N_lo, lo.r, lo.s) @ vinv[keep, :]


def interpolation(N_lo, N_hi):
    """(Np_hi x Np_lo) matrix of I: nodal order N_lo -> values at order-N_hi nodes."""
    hi, lo = RefElement(N_hi), RefElement(N_lo)
    return _low_mode_matrix(N_lo, N_lo, hi.r, hi.s) @ np.linalg.inv(lo.V)


def features(U, geo, U_inf, P=None):
    """Samples x (K x (4 Np_lo + 4)) of a state U (4, Np, K): with P (the
    restriction) for an order-p_hi state, else the order-p_lo state itself.
    geo: (K, 4) = rx, ry, sx, sy."""
    D = U - np.asarray(U_inf)[:, None, None]
    if P is not None:
        D = np.einsum("mn,cnk->cmk", P, D)
    K = U.shape[2]
    return np.concatenate([D.transpose(2, 0, 1).reshape(K, -1), np.asarray(geo)], axis=1)


def targets(U_hi, P, I):
    """t = U_hi - I P U_hi per element, (K, 4 Np_hi) field-major."""
    R = U_hi - np.einsum("mn,cnk->cmk", I @ P, U_hi)
    return R.transpose(2, 0, 1).reshape(U_hi.shape[2], -1)


def apply_closure(U_lo, I, Y):
    """Corrected order-p_hi state I U_lo + Y (Y: (K, 4 Np_hi) field-major)."""
    K = U_lo.shape[2]
    Np_hi = I.shape[0]
    return np.einsum("mn,cnk->cmk", I, U_lo) + Y.reshape(K, 4, Np_hi).transpose(1, 2, 0)


def drift_targets(U_ref, U):
    """Corrector targets (K, 4 Np) field-major: U_ref - U per element (both
    order-lo states (4, Np, K))."""
    D = U_ref - U
    return D.transpose(2, 0, 1).reshape(U.shape[2], -1)


def free_features(geo, Np_lo):
    """The free stream's samples (K x (4 Np_lo + 4)): no deviation, the
    element's metrics."""
    geo = np.asarray(geo)
    return np.concatenate([np.zeros((geo.shape[0], 4 * Np_lo)), geo], axis=1)


def apply_correction(U, Y):
    """The order-lo state U + Y (Y: (K, 4 Np) field-major)."""
    K, Np = U.shape[2], U.shape[1]
    return U + Y.reshape(K, 4, Np).transpose(1, 2, 0)


# ---------------------------------------------------------------- network
def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_grad(z):
    """d/dz of z Phi(z) = Phi(z) + z phi(z)."""
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def forward(params, X):
    """Y for samples X (B x n_in, already normalised); also the activations."""
    Z1 = X @ params["W1"].T + params["b1"]
    H1 = gelu(Z1)
    Z2 = H1 @ params["W2"].T + params["b2"]
    H2 = gelu(Z2)
    Y = H2 @ params["W3"].T + params["b3"]
    return Y, (X, Z1, H1, Z2, H2)


def loss_and_grads(params, X, T):
    """Mean squared error over all B x n_out entries and its gradients."""
    Y, (X, Z1, H1, Z2, H2) = forward(params, X)
    n = Y.size
    R = Y - T
    loss = float((R * R).sum() / n)
    dY = 2.0 * R / n
    g = {"W3": dY.T @ H2, "b3": dY.sum(axis=0)}
    dZ2 = (dY @ params["W3"]) * gelu_grad(Z2)
    g["W2"] = dZ2.T @ H1
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ params["W2"]) * gelu_grad(Z1)
    g["W1"] = dZ1.T @ X
    g["b1"] = dZ1.sum(axis=0)
    return loss, g


def adam_step(params, grads, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) with bias correction; step t >= 1."""
    out_p, out_m, out_v = {}, {}, {}
    for k in params:
        out_m[k] = beta1 * m[k] + (1.0 - beta1) * grads[k]
        out_v[k] = beta2 * v[k] + (1.0 - beta2) * grads[k] ** 2
        mh = out_m[k] / (1.0 - beta1 ** t)
        vh = out_v[k] / (1.0 - beta2 ** t)
        out_p[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
    return out_p, out_m, out_v


def round_bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float32:
    keep the upper 16 bits of the binary32 pattern after adding half an ulp of
    bfloat16 plus the parity of the kept part."""
    u = np.ascontiguousarray(np.asarray(x, dtype=np.float32)).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32)
