"""Write the oracle's trajectory of the viscous isentropic vortex workload
(vortex512: periodic [0,10]^2, 16 x 16 quads split into 512 triangles, p = 3,
Re = 100, M = 0.3, vortex of strength 5 and radius 1 at (5, 5), literature
penalty with C = 1, theta = 1) to vortex512_p3_oracle.npz: 200 LSERK steps at
dt = 0.3 / Lambda (Lambda the CFL bound of the initial state, C_grad = 1),
states after 10, 100 and 200 steps.  Calls only the oracle and the input
generators.  Run: python tests/golden/make_vortex512.py  (about 2-3 minutes).
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import meshgen as mg  # noqa: E402
from oracle.cfl import CFLOracle  # noqa: E402
from oracle.dg import DGOracle, Physics  # noqa: E402
from oracle.mesh import Mesh  # noqa: E402
from oracle.nodes import RefElement  # noqa: E402

OUT = os.path.join(HERE, "vortex512_p3_oracle.npz")
STEPS = (10, 100, 200)
C_CFL = 0.3


def setup():
    w = mg.workload("vortex512")
    ref = RefElement(w["p"])
    mesh = w["mesh"]
    m = Mesh(ref, mesh["VX"], mesh["VY"], mesh["EToV"], mesh["face_tag"], mesh["period"])
    phys = Physics(gamma=w["gamma"], Pr=w["Pr"], mu=w["mu"], theta=w["theta"],
                   penalty_mode=w["penalty_mode"], C_pen=w["C_pen"], U_inf=w["U_inf"])
    dg = DGOracle(m, phys)
    U0 = mg.isentropic_vortex(m.x, m.y, M=0.3, Lper=10.0)
    lam, dt = CFLOracle(m, phys).time_step(U0, C_cfl=C_CFL)
    return w, dg, U0, lam, dt


def main():
    w, dg, U0, lam, dt = setup()
    U = U0.copy()
    snaps = {}
    for n in range(1, STEPS[-1] + 1):
        U, _ = dg.lserk_step(U, dt)
        if n in STEPS:
            snaps["U%d" % n] = U.copy()
            print("step %d" % n, flush=True)
    np.savez_compressed(OUT, U0=U0, dt=dt, Lambda=lam, steps=np.array(STEPS), **snaps)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
