"""The allocation-free multi-step entry point against dg_rk_steps (needs an MI355X).

Collected last (its name), so that a failure here hides no other test.

dg_rk_steps_noalloc runs the same kernels as dg_rk_steps with its stage
ping-pong state and force partials in a static device array, so its states,
K1 registers and wall forces must equal dg_rk_steps's bitwise.  Two calls in
a row (the second on a smaller mesh, so the array holds the first call's
larger contents), odd and even step counts (the copy-back and no-copy
endings), the plain FP64 and FP32 perturbation forms, a mesh without walls,
and the size limit.
"""
import numpy as np
import pytest

import meshgen as mg

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(msg):
    print("[gpu-case] " + msg, flush=True)


def _solver(mesh, p, precision):
    from paper_2508_17917_amd import Solver
    w = mg.physics_params(Re=100.0, M=0.2)
    return Solver(p, mesh, precision=precision, penalty_mode=0, C_pen=1.0, theta=1.0, **w)


def _run_pair(torch, s, nsteps, dt, v_w, seed):
    from paper_2508_17917_amd import _lib as L
    U0 = np.transpose(mg.noisy_free_stream((4, s.Np, s.K), mg.free_stream(0.2),
                                           mg.rng_for(1, salt=seed), amp=1e-2), (2, 0, 1))
    Ua = torch.from_numpy(np.ascontiguousarray(U0)).cuda()
    Ub = Ua.clone()
    K1a = torch.zeros_like(Ua)
    K1b = torch.full_like(Ua, 7.0)        # K1 need not be initialised (A_1 = 0)
    Fa = torch.zeros(3 * nsteps, dtype=torch.float64, device="cuda")
    Fb = torch.full_like(Fa, -1.0)
    L.dg_rk_steps(s.h, Ua, K1a, nsteps, dt, v_w, Fa)
    L.dg_rk_steps_noalloc(s.h, Ub, K1b, nsteps, dt, v_w, Fb)
    torch.cuda.synchronize()
    assert torch.equal(Ua, Ub), "state differs"
    assert torch.equal(K1a, K1b), "K1 differs"
    assert torch.equal(Fa, Fb), "forces differ"
    assert bool(torch.isfinite(Ua).all())
    assert not torch.equal(Ua, torch.from_numpy(np.ascontiguousarray(U0)).cuda())


@pytest.mark.parametrize("precision", [0, 2])
def test_noalloc_equals_rk_steps_two_calls(precision):
    torch = _torch()
    big = _solver(mg.ogrid(24, 10, 0.5, 6.0, 1.2), 4, precision)
    small = _solver(mg.ogrid(10, 4, 0.5, 5.0, 1.3), 4, precision)
    try:
        _say("noalloc precision %d: K=%d then K=%d" % (precision, big.K, small.K))
        _run_pair(torch, big, 3, 2e-6, (0.0, 0.01), 1)
        _run_pair(torch, small, 2, 2e-6, (0.0, -0.02), 2)
        _run_pair(torch, small, 3, 2e-6, (0.0, 0.0), 3)
    finally:
        big.close()
        small.close()


def test_noalloc_without_walls_and_other_order():
    torch = _torch()
    s = _solver(mg.periodic_square(6, 5, 10.0, 8.0), 3, 0)
    try:
        _say("noalloc periodic p=3 K=%d" % s.K)
        _run_pair(torch, s, 3, 1e-3, (0.0, 0.0), 4)
    finally:
        s.close()


def test_noalloc_rejects_a_state_beyond_the_array():
    """K * 4 * Np * 8 bytes above 64 MiB is refused before any launch."""
    torch = _torch()
    from paper_2508_17917_amd import _lib as L
    s = _solver(mg.periodic_square(160, 160, 10.0, 10.0), 6, 0)   # 51,200 x 28 nodes: 45.9 MB fits
    try:
        assert s.K * 4 * s.Np * 8 < 64 << 20
    finally:
        s.close()
    s = _solver(mg.periodic_square(200, 200, 10.0, 10.0), 6, 0)   # 80,000 x 28 nodes: 71.7 MB
    try:
        _say("noalloc size limit K=%d" % s.K)
        U = torch.zeros((s.K, 4, s.Np), dtype=torch.float64, device="cuda")
        K1 = torch.zeros_like(U)
        with pytest.raises(L.DGError) as e:
            L.dg_rk_steps_noalloc(s.h, U, K1, 1, 1e-6)
        assert e.value.code == L.DG_EINVAL and "exceeds" in str(e.value)
    finally:
        s.close()
