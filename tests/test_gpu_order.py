"""Observed temporal order of the full IMEX step on the GPU (ARK pairs of Sec. 4.2.2,
Alg. imex_scheme_update): an isentropic vortex with an implicit HDG-IP strip, run to a
fixed time on one mesh with m, 2m and 4m steps.  The spatial error is the same for the
three runs, so the ratio of successive differences gives the temporal order: 2 for
ARS(2,2,2) and 3 for ARS(3,4,3) (self-convergence; the oracle's test of the same
property uses a reference run on the CPU)."""
import dataclasses
import math

import numpy as np
import pytest

from _common import gpu_engine
from paper_2607_16044_amd import workloads as W

pytestmark = pytest.mark.gpu


def _run(wl, T, m, precision):
    eng = gpu_engine(wl, precision=precision)
    U = eng.initial_state()
    H = eng.init_facets(U)
    for _ in range(m):
        eng.ark_step(T / m, U, H)
    out = U.cpu().numpy()
    eng.close()
    return out


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("tableau,order", [("ARS222", 2), ("ARS343", 3)])
def test_observed_temporal_order(tableau, order, precision):
    wl = dataclasses.replace(W.vortex(nx=8, ny=8, k=3, strip_rows=2, compression=4.0, name="vortex_order"),
                             tableau=tableau)
    m = 8
    T = m * wl.dt                       # the coarsest run takes the workload's stable step
    u = [_run(wl, T, m * 2 ** i, precision) for i in range(3)]
    d1 = np.abs(u[0] - u[1]).max()
    d2 = np.abs(u[1] - u[2]).max()
    observed = math.log2(d1 / d2)
    print(tableau, precision, "differences", d1, d2, "observed order", observed)
    assert d2 > 1e-11 * np.abs(u[2]).max()       # well above the solver tolerances
    assert abs(observed - order) < 0.3
