"""Shared test helpers: relative L2 and GPU runs through the C ABI."""
import numpy as np


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def gpu_run(case, nsteps=None, band_rows=None, k=None, steps_per_pass=1):
    """Run a case through the C ABI; returns (eta, u, v, folds of the last k steps). With
    steps_per_pass > 1, band_rows is the band height of the temporally blocked passes."""
    from paper_1711_04471_amd.sw2d import Sw2d, ring_capacity
    n = case.steps if nsteps is None else nsteps
    with Sw2d.from_case(case) as sim:
        if steps_per_pass > 1:
            sim.set_time_blocking(steps_per_pass, rows=band_rows or 32)
        elif band_rows is not None:
            sim.band_rows = band_rows
        sim.step(n)
        kk = min(n, ring_capacity()) if k is None else k
        red = sim.reduce(kk) if kk > 0 else None
        e, u, v = sim.state_numpy()
    return e, u, v, red
