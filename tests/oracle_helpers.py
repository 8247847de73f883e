"""Builders shared by the CPU tests: oracle instances from meshgen inputs."""
import numpy as np

import meshgen as mg
from oracle.dg import DGOracle, Physics
from oracle.mesh import Mesh
from oracle.nodes import RefElement

_REF = {}


def ref_element(p):
    if p not in _REF:
        _REF[p] = RefElement(p)
    return _REF[p]


def build(mesh, p, gamma=1.4, Pr=0.72, mu=2e-3, theta=1.0, penalty_mode=0, C_pen=0.01,
          U_inf=None, face_tag=None, wall_heat_flux=False):
    ref = ref_element(p)
    ft = mesh["face_tag"] if face_tag is None else face_tag
    m = Mesh(ref, mesh["VX"], mesh["VY"], mesh["EToV"], ft, mesh["period"])
    if U_inf is None:
        U_inf = mg.free_stream(0.2, gamma)
    phys = Physics(gamma=gamma, Pr=Pr, mu=mu, theta=theta, penalty_mode=penalty_mode,
                   C_pen=C_pen, U_inf=U_inf, wall_heat_flux=wall_heat_flux)
    return DGOracle(m, phys)


def build_workload(name, p=None, **over):
    w = mg.workload(name, p)
    kw = dict(gamma=w["gamma"], Pr=w["Pr"], mu=w["mu"], theta=w["theta"],
              penalty_mode=w["penalty_mode"], C_pen=w["C_pen"], U_inf=w["U_inf"])
    kw.update(over)
    return build(w["mesh"], w["p"], **kw), w


def uniform(dg, U):
    return np.broadcast_to(np.asarray(U)[:, None, None], (4, dg.ref.Np, dg.mesh.K)).copy()
