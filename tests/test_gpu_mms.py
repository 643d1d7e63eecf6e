"""Manufactured solution on the GPU (Sec. 5.1.1).

* The source's load vector against the oracle's (closed-form state and gradient, the
  flux divergence by the complex step there; by hand-coded derivatives in the kernel).
* Whole ARK steps with the source against the oracle's, on a periodic square whose middle
  element columns are implicit, for both tableaux, to the FP64 path's 1e-10.
* Temporal order: the error of the step against a solution with 16 times smaller steps
  falls as dt^2 for ARS(2,2,2) and dt^3 for ARS(3,4,3); the error against the exact
  solution U_e itself decreases to the spatial discretisation's level.
"""
import numpy as np
import pytest

from _common import MMS, gpu_engine, mms_workload, rel_err
from oracle import physics as ph
from oracle.ark import IMEXSolver
from oracle.basis import Basis
from oracle.mesh import Mesh
from oracle.mms import exact_state, source_load
from paper_2607_16044_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("k", [2, 4])
def test_mms_load_matches_oracle(k):
    wl = mms_workload(n=6, k=k, implicit_cols=(2, 3))
    eng = gpu_engine(wl)
    eng.set_mms_source(*MMS)
    mesh, basis = Mesh(wl), Basis(k)
    gas = ph.Gas(wl.gamma, wl.R, wl.mu, wl.Pr)
    for t in (0.0, 3.7e-4):
        b = eng.mms_load(t).cpu().numpy()
        ref = source_load(t, *MMS, mesh, basis, gas)
        e = rel_err(b, ref)
        print(k, t, e)
        assert e < 1e-12
    eng.close()


@pytest.mark.parametrize("tableau", ["ARS222", "ARS343"])
@pytest.mark.parametrize("variant", [W.HDG_MX, W.HDG_IP])
def test_mms_steps_match_oracle(tableau, variant):
    wl = mms_workload(n=4, k=2, implicit_cols=(1, 2), variant=variant, tableau=tableau, dt=2e-4)
    eng = gpu_engine(wl)
    eng.set_mms_source(*MMS, t0=0.0)
    U = eng.initial_state()
    H = eng.init_facets(U)
    ora = IMEXSolver(wl)
    ora.mms = MMS
    for _ in range(3):
        eng.ark_step(wl.dt, U, H)
        ora.step()
    e = rel_err(U.cpu().numpy(), ora.U)
    print(tableau, variant, e)
    assert e < 1e-10
    # without the source the same steps end elsewhere: the source is really applied
    eng2 = gpu_engine(wl)
    U2 = eng2.initial_state()
    H2 = eng2.init_facets(U2)
    for _ in range(3):
        eng2.ark_step(wl.dt, U2, H2)
    assert rel_err(U2.cpu().numpy(), ora.U) > 1e-4
    eng.close()
    eng2.close()


def _run(wl, dt, steps):
    eng = gpu_engine(wl)
    eng.set_mms_source(*MMS, t0=0.0)
    U = eng.initial_state()
    H = eng.init_facets(U)
    for _ in range(steps):
        eng.ark_step(dt, U, H)
    out = U.cpu().numpy()
    X, Y = eng.node_coords()
    eng.close()
    return out, X, Y


@pytest.mark.parametrize("tableau,order", [("ARS222", 2), ("ARS343", 3)])
def test_mms_temporal_order(tableau, order):
    T = 2e-3
    wl = mms_workload(n=8, k=4, implicit_cols=(2, 3, 4, 5), tableau=tableau)
    ref, X, Y = _run(wl, T / 160, 160)
    errs, exact_errs = [], []
    Ue = np.moveaxis(exact_state(X, Y, T, *MMS), 0, 1)
    for m in (5, 10, 20):
        u, _, _ = _run(wl, T / m, m)
        errs.append(np.sqrt(np.mean((u - ref) ** 2)))
        exact_errs.append(np.sqrt(np.mean((u - Ue) ** 2)))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    print(tableau, errs, rates, exact_errs)
    assert min(rates) > order - 0.25
    assert exact_errs[2] < exact_errs[0]
