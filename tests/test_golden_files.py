"""Stored oracle outputs are the oracle's (CPU): re-running the start of each
recorded trajectory with the current oracle reproduces the file (to the
rounding of the host's floating-point libraries)."""
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def test_vortex512_golden_is_the_oracles():
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "make_vortex512", os.path.join(HERE, "golden", "make_vortex512.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    g = np.load(mk.OUT)
    _, dg, U0, lam, dt = mk.setup()
    assert np.array_equal(U0, g["U0"])
    assert float(dt) == float(g["dt"]) and float(lam) == float(g["Lambda"])
    U = U0.copy()
    for _ in range(10):
        U, _k = dg.lserk_step(U, dt)
    # the same arithmetic in the same order: equal up to the host's rounding
    assert np.abs(U - g["U10"]).max() <= 1e-13 * np.abs(g["U10"]).max()
