"""Mixed precision (FP32 linear algebra, FP64 residuals): GPU parity with the oracle.

In IMEX_FP32_REFINE mode the element Jacobians, the mixed elimination, K^-1,
the condensation, the Schur complement S and the Schwarz preconditioner are
FP32 (FP32 MFMA for the batched GEMMs); the Newton residual, the state, the
Krylov vectors and the conservation sums stay FP64.  Newton with the FP64
residual is the iterative refinement, so the converged states must match the
FP64 oracle to 1e-9 relative; the element blocks themselves only to FP32
rounding.
"""
import numpy as np
import pytest
import torch

from _common import gpu_engine, rel_err, smooth_square
from oracle.ark import IMEXSolver
from paper_2607_16044_amd import workloads as W

pytestmark = pytest.mark.gpu

FP32_REFINE = 1
BAR = 1e-9

CASES = {
    "vortex_small": lambda: W.get("vortex_small"),
    "square_ip": lambda: smooth_square(4, 2, viscous=True, variant=W.HDG_IP, implicit_rows=(1, 2)),
    "square_mx": lambda: smooth_square(4, 2, viscous=True, variant=W.HDG_MX, implicit_rows=(1, 2)),
    "bl_small": lambda: W.get("boundary_layer_small"),
    "bl_k4": lambda: W.boundary_layer(nx=3, ny=4, k=4, implicit_rows=2, Lx=3 * 2.0 / 256, height=None, steps=1,
                                      name="bl_k4"),
}


@pytest.mark.parametrize("case", ["square_mx", "bl_k4", "square_ip"])
def test_local_system_fp32_vs_fp64(case):
    """FP32 blocks equal the FP64 blocks to FP32 rounding (same kernels, other element type)."""
    wl = CASES[case]()
    ora = IMEXSolver(wl)
    U = torch.tensor(ora.U, device="cuda")
    Uhat = torch.tensor(ora.Uhat, device="cuda")
    rhs = torch.tensor(ora.mass_apply(ora.U) * 0.999, device="cuda")
    dt_a = 0.4 * wl.dt
    ref = [t.cpu().numpy() for t in gpu_engine(wl).local_system(dt_a, rhs, U, Uhat)]
    got = [t.cpu().numpy() for t in gpu_engine(wl, precision=FP32_REFINE).local_system(dt_a, rhs, U, Uhat)]
    for name, a, b in zip("fhKCDE", got, ref):
        e = rel_err(a, b)
        print(case, name, e)
        assert e < 2e-5, (case, name, e)


@pytest.mark.parametrize("case", ["vortex_small", "square_ip", "square_mx", "bl_small"])
def test_stage_solve_mixed_parity(case):
    wl = CASES[case]()
    eng = gpu_engine(wl, precision=FP32_REFINE)
    ora = IMEXSolver(wl)
    U = torch.tensor(ora.U, device="cuda")
    Uhat = torch.tensor(ora.Uhat, device="cuda")
    dt_a = 0.4 * wl.dt
    rhs = ora.mass_apply(ora.U)
    R, st = eng.implicit_stage_solve(dt_a, torch.tensor(rhs, device="cuda"), U, Uhat)
    ora.system.newton(ora.U, ora.Q, ora.Uhat, dt_a, rhs[ora.mesh.im_elems])
    im = ora.mesh.im_elems
    eu = rel_err(U.cpu().numpy()[im], ora.U[im])
    eh = rel_err(Uhat.cpu().numpy(), ora.Uhat)
    print(case, "newton", st["newton_its"], "U", eu, "Uhat", eh)
    assert eu < BAR and eh < BAR


@pytest.mark.parametrize("case,steps", [("vortex_small", 3), ("bl_small", 2), ("square_mx", 2)])
def test_ark_steps_mixed_parity(case, steps):
    wl = CASES[case]()
    eng = gpu_engine(wl, precision=FP32_REFINE)
    ora = IMEXSolver(wl)
    U = torch.tensor(ora.U, device="cuda")
    Uhat = torch.tensor(ora.Uhat, device="cuda")
    for _ in range(steps):
        eng.ark_step(wl.dt, U, Uhat)
        ora.step()
    e = rel_err(U.cpu().numpy(), ora.U)
    print(case, "U", e)
    assert e < BAR
    assert rel_err(Uhat.cpu().numpy(), ora.Uhat) < BAR


def test_vortex_full_run_mixed_parity():
    """The vortex workload, all 20 steps, in mixed precision."""
    wl = W.get("vortex")
    eng = gpu_engine(wl, precision=FP32_REFINE)
    ora = IMEXSolver(wl)
    U = torch.tensor(ora.U, device="cuda")
    Uhat = torch.tensor(ora.Uhat, device="cuda")
    for _ in range(wl.steps):
        eng.ark_step(wl.dt, U, Uhat)
        ora.step()
    e = rel_err(U.cpu().numpy(), ora.U)
    print("vortex mixed 20 steps rel err", e)
    assert e < BAR


def test_boundary_layer_mixed_vs_fp64_full_size():
    """Full-size boundary layer (256x128, k=4, 4096 HDG-MX elements): two ARS(3,4,3)
    steps in mixed precision against the FP64 path, whose stage solves are held
    to the oracle above; the bar is the mixed path's 1e-9."""
    wl = W.get("boundary_layer")
    res = []
    for prec in (0, FP32_REFINE):
        eng = gpu_engine(wl, precision=prec)
        U = eng.initial_state()
        Uhat = eng.init_facets(U)
        for _ in range(2):
            eng.ark_step(wl.dt, U, Uhat)
        res.append((U.cpu().numpy(), Uhat.cpu().numpy()))
        eng.close()
    e = rel_err(res[1][0], res[0][0])
    print("boundary layer mixed vs fp64", e, rel_err(res[1][1], res[0][1]))
    assert e < BAR and rel_err(res[1][1], res[0][1]) < BAR
