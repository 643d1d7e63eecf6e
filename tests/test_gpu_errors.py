"""Failure paths of the C ABI on the device: every one returns a status, none faults.

* ENOCONV: Newton capped at one correction, and facet solves capped at one GMRES
  iteration (a capped solve certifies nothing, so Newton runs out of corrections).
* ENONFINITE: a NaN in the implicit stage's initial state, and in the interface data
  that the facet rows read.
* EINVAL / ENOTIMPL: tableaux whose fsal or stiffly_accurate flag disagrees with the
  coefficients, and an implicit tableau that is not stiffly accurate; rejected before
  any work, the state untouched.
* Re-setting the regions with graph replay on drops the captured graphs (their kernel
  arguments point into the old workspaces): the step equals a fresh context's.
The conditions are all set from the host; every kernel runs to its normal end.
"""
import math

import numpy as np
import pytest
import torch

from _common import gpu_engine, rel_err
from paper_2607_16044_amd import tableaux
from paper_2607_16044_amd import workloads as W
from paper_2607_16044_amd.binding import IMEXError, Tableau

pytestmark = pytest.mark.gpu

ENOCONV, ENONFINITE, EINVAL, ENOTIMPL = -4, -5, -1, -6


def _setup(wl, **kw):
    eng = gpu_engine(wl, **kw)
    U = eng.initial_state()
    H = eng.init_facets(U)
    return eng, U, H


@pytest.mark.parametrize("kw", [{"newton_maxit": 1}, {"gmres_maxit": 1, "newton_maxit": 4}])
def test_capped_newton_or_gmres_is_enoconv(kw):
    wl = W.get("boundary_layer_small")
    eng, U, H = _setup(wl, **kw)
    U0 = U.clone()
    with pytest.raises(IMEXError) as ei:
        eng.ark_step(wl.dt, U, H)
    assert ei.value.status == ENOCONV, ei.value
    assert torch.equal(U, U0)              # the step leaves U unchanged on failure
    eng.close()
    # the same context recovers with the default caps once they are lifted (a fresh one)
    eng, U, H = _setup(wl)
    eng.ark_step(wl.dt, U, H)
    assert torch.isfinite(U).all()
    eng.close()


@pytest.mark.parametrize("where", ["implicit", "interface"])
def test_nan_input_is_enonfinite(where):
    wl = W.get("boundary_layer_small")
    eng, U, H = _setup(wl)
    im = np.flatnonzero(wl.implicit_flags())
    ex = np.flatnonzero(~wl.implicit_flags().astype(bool))
    rhs = U.clone()
    if where == "implicit":
        U[int(im[0]), 3, 0] = math.nan
    else:
        # an explicit element next to the implicit strip: its trace is interface data
        row = wl.nx * int(np.max(np.flatnonzero(wl.implicit.any(axis=1))) + 1)
        assert row in ex
        U[row, 0, 0] = math.nan
    with pytest.raises(IMEXError) as ei:
        eng.implicit_stage_solve(0.4 * wl.dt, rhs * 1.0, U, H)
    assert ei.value.status == ENONFINITE, ei.value
    eng.close()


def _bad_tableaux():
    t = tableaux.get("ARS222")
    out = []
    flipped = t.to_ctypes(Tableau)
    flipped.fsal = 0                        # be equals the last row of Ae: fsal must be 1
    out.append(("fsal flag", flipped, EINVAL))
    flipped = t.to_ctypes(Tableau)
    flipped.stiffly_accurate = 0
    out.append(("stiffly accurate flag", flipped, EINVAL))
    nsa = t.to_ctypes(Tableau)              # bi != last row of Ai, flagged honestly
    nsa.bi[0] = 0.5
    nsa.bi[1] = 0.5
    nsa.stiffly_accurate = 0
    out.append(("not stiffly accurate", nsa, ENOTIMPL))
    upper = t.to_ctypes(Tableau)
    upper.Ae[1] = 0.1                       # Ae[0][1]: not strictly lower triangular
    out.append(("upper entry", upper, EINVAL))
    return out


@pytest.mark.parametrize("name,tab,status", _bad_tableaux(), ids=[b[0] for b in _bad_tableaux()])
def test_bad_tableau_rejected_before_work(name, tab, status):
    import ctypes
    from paper_2607_16044_amd.binding import Stats, _ptr
    wl = W.get("vortex_small")
    eng, U, H = _setup(wl)
    U0, H0 = U.clone(), H.clone()
    st = Stats()
    rc = eng.lib.imex_ark_step(eng.ctx, ctypes.byref(tab), wl.dt, _ptr(U), _ptr(H), ctypes.byref(st))
    assert rc == status, (name, rc, eng.lib.imex_last_error(eng.ctx))
    assert torch.equal(U, U0) and torch.equal(H, H0)
    eng.close()


def test_reset_regions_with_graphs_equals_fresh_context():
    wl = W.get("vortex_small")             # periodic: the all-explicit split below is valid
    eng, U, H = _setup(wl)
    eng.set_graphs(True)
    for _ in range(2):
        eng.ark_step(wl.dt, U, H)          # graphs captured against the first workspaces
    flags = wl.implicit_flags()
    eng.set_regions(np.zeros_like(flags))  # all explicit: workspaces freed ...
    eng.set_regions(flags)                 # ... and reallocated
    U2 = eng.initial_state()
    H2 = eng.init_facets(U2)
    for _ in range(2):
        eng.ark_step(wl.dt, U2, H2)
    eng.close()
    ref, Ur, Hr = _setup(wl)
    for _ in range(2):
        ref.ark_step(wl.dt, Ur, Hr)
    ref.close()
    assert rel_err(U2.cpu().numpy(), Ur.cpu().numpy()) < 1e-13
    assert rel_err(H2.cpu().numpy(), Hr.cpu().numpy()) < 1e-13


def test_wall_flag_on_explicit_element_leaves_context_usable():
    """A split with an explicit element on a wall is rejected before the context changes:
    the previous regions keep working."""
    wl = W.get("boundary_layer_small")
    eng, U, H = _setup(wl)
    bad = np.zeros_like(wl.implicit_flags())
    with pytest.raises(IMEXError) as ei:
        eng.set_regions(bad)
    assert ei.value.status == EINVAL
    eng.ark_step(wl.dt, U, H)
    assert torch.isfinite(U).all()
    eng.close()


def test_timer_mask_selects_the_timed_phases():
    """imex_set_timer_mask: masked phases record no events and their counters stay put;
    the step matches a context with every phase timed (to the parity gate: the solver's
    refresh decisions follow measured times); bits beyond the phases are EINVAL."""
    wl = W.get("boundary_layer_small")
    ref, U_ref, H_ref = _setup(wl)
    ref.ark_step(wl.dt, U_ref, H_ref)
    ref.close()
    eng, U, H = _setup(wl)
    eng.set_timer_mask(["eliminate"])
    eng.ark_step(wl.dt, U, H)
    t = eng.timers(reset=True)
    assert t["eliminate_launches"] > 0
    assert all(t[n + "_launches"] == 0 for n in eng.TIMER_NAMES if n != "eliminate")
    assert rel_err(U.cpu(), U_ref.cpu()) < 1e-10 and rel_err(H.cpu(), H_ref.cpu()) < 1e-10
    eng.set_timer_mask([])
    eng.ark_step(wl.dt, U, H)
    assert all(v == 0 for v in eng.timers(reset=True).values())
    eng.set_timer_mask(None)
    eng.ark_step(wl.dt, U, H)
    assert eng.timers()["assemble_launches"] > 0
    with pytest.raises(IMEXError) as e:
        eng._check(eng.lib.imex_set_timer_mask(eng.ctx, 1 << 11))
    assert e.value.status == EINVAL
    eng.close()
