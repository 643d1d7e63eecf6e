"""Degree-4 parity of the launch shapes the benchmark times, against the oracle.

The boundary-layer benchmark runs at k = 4, where the augmented element system is
180 x 180 (NU = 100, NF = 80) and the whole-matrix FP32 GEMM shapes split it into parts
(codes 2007 / 2008: 96 x 192 or 96 x 96 parts, 2009 / 2010 the same parts with FP32 products
emulated on the bf16 matrix cores; 2001..2006 hold it whole or fall back to
the 64 tile).  Each shape set through imex_set_launch_shapes must reach the oracle's
root: one implicit stage (eqs. dirk_stage_update_*, solved through
eqs. statically_condensed_system / SchurCompliment / local_solve_static_condensation)
and one full ARS(3,4,3) IMEX step (Alg. imex_scheme_update) on a 3 x 4 boundary-layer
mesh with two HDG-MX wall rows, compared per conservative field.  Bars: 1e-10 (FP64),
1e-9 (FP32 element linear algebra with FP64 refinement).
"""
import functools

import numpy as np
import pytest
import torch

from _common import gpu_engine, rel_err
from oracle.ark import IMEXSolver
from paper_2607_16044_amd import workloads as W

pytestmark = pytest.mark.gpu

BAR = {0: 1e-10, 1: 1e-9}
# default shapes, every single code, and the combinations the autotuner picks on the full mesh
SHAPES = [None] + [{"gemm_tile_eliminate": t, "gemm_tile_condense": t, "gemm_tile_schur": t}
                   for t in (64, 32, 1064, 1032, 2001, 2002, 2003, 2004, 2005, 2006, 2007, 2008, 2009, 2010, 2011)] + [
    {"gemm_tile_eliminate": 2008, "gemm_tile_condense": 2004, "gemm_tile_schur": 2008},
    {"gemm_tile_eliminate": 2009, "gemm_tile_condense": 2004, "gemm_tile_schur": 2009},
    {"gemm_tile_eliminate": 2010, "gemm_tile_condense": 2004, "gemm_tile_schur": 2009},
    {"gemm_tile_eliminate": 2009, "gemm_tile_condense": 2011, "gemm_tile_schur": 2009},
    {"gemm_tile_eliminate": 2001, "gemm_tile_condense": 2004, "gemm_tile_schur": 2008},
    {"gemm_tile_eliminate": 2007, "gemm_tile_condense": 2005, "gemm_tile_schur": 2007},
]
FP64_SHAPES = [None, {"gemm_tile_eliminate": 64, "gemm_tile_condense": 64, "gemm_tile_schur": 64},
               {"gemm_tile_eliminate": 32, "gemm_tile_condense": 32, "gemm_tile_schur": 32}]


def _wl():
    return W.boundary_layer(nx=3, ny=4, k=4, implicit_rows=2, Lx=3 * 2.0 / 256, height=None, steps=1,
                            name="bl_k4")


@functools.lru_cache(maxsize=None)
def _oracle():
    """The oracle's stage root and one IMEX step from the initial state (computed once)."""
    wl = _wl()
    ora = IMEXSolver(wl)
    U0, H0 = ora.U.copy(), ora.Uhat.copy()
    dt_a = 0.43586652150845895 * wl.dt                 # the ARS(3,4,3) diagonal
    rhs = ora.mass_apply(ora.U)
    im = ora.mesh.im_elems
    Us, Qs, Hs = ora.U.copy(), ora.Q.copy(), ora.Uhat.copy()
    ora.system.newton(Us, Qs, Hs, dt_a, rhs[im])
    ora.step()
    return U0, H0, dt_a, rhs, Us, Hs, ora.U.copy(), ora.Uhat.copy(), im


def _engine(precision, shapes):
    eng = gpu_engine(_wl(), precision=precision)
    if shapes is not None:
        eng.set_launch_shapes(shapes)
    return eng


def _name(s):
    return "default" if s is None else "-".join(str(s[k]) for k in
                                                ("gemm_tile_eliminate", "gemm_tile_condense", "gemm_tile_schur"))


@pytest.mark.parametrize("precision,shapes", [(0, s) for s in FP64_SHAPES] + [(1, s) for s in SHAPES],
                         ids=lambda v: _name(v) if isinstance(v, dict) or v is None else str(v))
def test_k4_stage_and_step_against_oracle(precision, shapes):
    U0, H0, dt_a, rhs, Us, Hs, U1, H1, im = _oracle()
    wl = _wl()
    eng = _engine(precision, shapes)
    U = torch.tensor(U0, device="cuda")
    H = torch.tensor(H0, device="cuda")
    eng.implicit_stage_solve(dt_a, torch.tensor(rhs, device="cuda"), U, H)
    eu = rel_err(U.cpu().numpy()[im], Us[im])
    eh = rel_err(H.cpu().numpy(), Hs)
    U = torch.tensor(U0, device="cuda")
    H = torch.tensor(H0, device="cuda")
    eng.ark_step(wl.dt, U, H)
    su = rel_err(U.cpu().numpy(), U1)
    sh = rel_err(H.cpu().numpy(), H1)
    eng.close()
    print(precision, _name(shapes), "stage", eu, eh, "step", su, sh)
    assert max(eu, eh, su, sh) < BAR[precision], (eu, eh, su, sh)
