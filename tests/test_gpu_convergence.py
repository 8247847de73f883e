"""Convergence of the GPU path to an exact solution, independent of the
oracle: the isentropic vortex (strength 5, radius 1) advected by the free
stream (M = 0.3) through a periodic [0, 10]^2 is an exact solution of the
inviscid equations (mu = 0, so the interior-penalty terms vanish and the
scheme is the Roe-flux DG of Sec. 2.2). After t = 1 (LSERK steps at
dt = 1 / Lambda, the CFL bound) the L2 error of every conserved field,
(sum_K J_K e^T M e)^(1/2), against the translated vortex falls under mesh
refinement at a rate above p on the finest pair of meshes — the order the
paper reports for its convergence study (Sec. 3.1: r_2(p) > p) — measured
2.4-2.7 at p = 2, 3.5-3.8 at p = 3, 4.2-4.6 at p = 4."""
import numpy as np
import pytest

import meshgen as mg

pytestmark = pytest.mark.gpu

M, L, T = 0.3, 10.0, 1.0


def _vortex_error(n, p):
    import torch
    from paper_2508_17917_amd import Solver
    U_inf = mg.free_stream(M)
    mesh = mg.periodic_square(n, n, L, L)
    s = Solver(p, mesh, gamma=1.4, Pr=0.72, mu=0.0, theta=1.0, penalty_mode=0, C_pen=1.0,
               U_inf=U_inf, precision=0)
    x, y = s.nodes()
    U0 = mg.isentropic_vortex(x, y, M=M, xc=5.0, yc=5.0, Lper=L)          # (4, K, Np)
    U = torch.from_numpy(np.ascontiguousarray(np.transpose(U0, (1, 0, 2)))).cuda()
    K1 = torch.zeros_like(U)
    _, dt = s.cfl_time_step(U, C_cfl=1.0)
    nsteps = int(np.ceil(T / dt))
    s.rk_steps(U, K1, nsteps, T / nsteps)
    Ue = mg.isentropic_vortex(x, y, M=M, xc=5.0 + M * T, yc=5.0, Lper=L)
    d = U.cpu().numpy() - np.transpose(Ue, (1, 0, 2))
    Mref = s.table("M").reshape(s.Np, s.Np)
    geo = s.table("geo").reshape(s.K, 16)
    J = 1.0 / (geo[:, 0] * geo[:, 3] - geo[:, 1] * geo[:, 2])
    s.close()
    return np.sqrt(np.einsum("kcn,nm,kcm,k->c", d, Mref, d, J))


@pytest.mark.parametrize("p,coarse", [(2, 32), (3, 16), (4, 16)])
def test_vortex_converges_at_order_above_p(p, coarse):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("[gpu-case] isentropic vortex p=%d n=%d,%d" % (p, coarse, 2 * coarse), flush=True)
    e1 = _vortex_error(coarse, p)
    e2 = _vortex_error(2 * coarse, p)
    rates = np.log2(e1 / e2)
    assert np.all(e2 < e1) and np.all(rates > p), (e1, e2, rates)
