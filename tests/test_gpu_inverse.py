"""The element inverse K^-1 by blocked Gauss-Jordan on the matrix cores (FP32,
imex_element_inverse method 1) against the oracle.

The condensation (eq. local_solve_static_condensation) needs K^-1 of every implicit
element; method 1 pivots in panels of 16 factorised by one wave and applies each
panel's rank-16 transformation with v_mfma_f32_16x16x4f32.  One implicit stage
(eqs. dirk_stage_update_*) and one ARS(3,4,3) IMEX step (Alg. imex_scheme_update) on a
3 x 4 boundary-layer mesh with two HDG-MX wall rows must reach the oracle's root at the
mixed-precision bar 1e-9 per conservative field, for k = 1..4 (at k = 4 also with the
GEMM shapes the benchmark picks).  The method is FP32 only: FP64 contexts reject it.
"""
import functools

import pytest
import torch

from _common import gpu_engine, rel_err
from oracle.ark import IMEXSolver
from paper_2607_16044_amd import workloads as W
from paper_2607_16044_amd.binding import IMEXError

pytestmark = pytest.mark.gpu

EINVAL = -1


def _wl(k):
    return W.boundary_layer(nx=3, ny=4, k=k, implicit_rows=2, Lx=3 * 2.0 / 256, height=None, steps=1,
                            name=f"bl_k{k}")


@functools.lru_cache(maxsize=None)
def _oracle(k):
    wl = _wl(k)
    ora = IMEXSolver(wl)
    U0, H0 = ora.U.copy(), ora.Uhat.copy()
    dt_a = 0.43586652150845895 * wl.dt                 # the ARS(3,4,3) diagonal
    rhs = ora.mass_apply(ora.U)
    im = ora.mesh.im_elems
    Us, Qs, Hs = ora.U.copy(), ora.Q.copy(), ora.Uhat.copy()
    ora.system.newton(Us, Qs, Hs, dt_a, rhs[im])
    ora.step()
    return U0, H0, dt_a, rhs, Us, Hs, ora.U.copy(), ora.Uhat.copy(), im


BENCH_SHAPES = {"gemm_tile_eliminate": 2008, "gemm_tile_condense": 2004, "gemm_tile_schur": 2008}


@pytest.mark.parametrize("k,shapes", [(1, None), (2, None), (3, None), (4, None), (4, BENCH_SHAPES)],
                         ids=["k1", "k2", "k3", "k4", "k4-bench-shapes"])
def test_matrix_core_inverse_against_oracle(k, shapes):
    U0, H0, dt_a, rhs, Us, Hs, U1, H1, im = _oracle(k)
    wl = _wl(k)
    eng = gpu_engine(wl, precision=1)
    if shapes is not None:
        eng.set_launch_shapes(shapes)
    assert eng.element_inverse(1) == 1
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
    assert eng.element_inverse() == 1
    eng.close()
    print(k, shapes, "stage", eu, eh, "step", su, sh)
    assert max(eu, eh, su, sh) < 1e-9, (eu, eh, su, sh)


def test_inverse_method_selection():
    wl = _wl(2)
    e64 = gpu_engine(wl, precision=0)
    assert e64.element_inverse() == 0
    with pytest.raises(IMEXError) as err:
        e64.element_inverse(1)
    assert err.value.status == EINVAL
    assert e64.element_inverse() == 0
    e64.close()
    e32 = gpu_engine(wl, precision=1)
    with pytest.raises(IMEXError) as err:
        e32.element_inverse(2)
    assert err.value.status == EINVAL
    assert e32.element_inverse(1) == 1 and e32.element_inverse(0) == 0
    e32.close()
