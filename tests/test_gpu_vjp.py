"""GPU vector-Jacobian products (reverse mode) against the oracle's directional derivatives.

The oracle has no adjoint code: its forward residual, evaluated on a complex
perturbation U + i h d (complex step, exact to rounding for the smooth fluxes)
or by central differences (Lax-Friedrichs: its wave-speed bound takes a modulus,
which the complex step does not differentiate), gives J d; the GPU's transposed
product must satisfy <Ubar, d> = <Rbar, J d>.

* DG residual: interior, far-field and interface faces, viscous and inviscid.
* One explicit ARK step: the oracle's explicit stage recursion on complex input.
* One IMEX step with an implicit HDG-IP region (transposed condensed solves):
  central differences of the GPU forward map and of the oracle's own step.
* Rollout with checkpointed recomputation (torch.autograd.Function): gradients with
  and without checkpointing agree, and match central finite differences of the GPU
  forward map (h = 1e-6), explicit-only and with an implicit region.
"""
import numpy as np
import pytest
import torch

from _common import gpu_engine, smooth_square
from oracle.ark import IMEXSolver, _sub
from oracle.dg import apply_minv, dg_residual
from paper_2607_16044_amd import workloads as W

pytestmark = pytest.mark.gpu

CASES = {
    "square_explicit": lambda: smooth_square(4, 2, viscous=True),
    "square_farfield": lambda: smooth_square(4, 2, viscous=True, bc=(W.BC_FARFIELD,) * 4),
    "square_interface_ip": lambda: smooth_square(4, 2, viscous=True, variant=W.HDG_IP, implicit_rows=(1,)),
    "square_k3_euler": lambda: smooth_square(3, 3, viscous=False),
    "vortex_small": lambda: W.get("vortex_small"),
}


def _oracle_jvp(f, U, d, lf):
    if lf:
        h = 1e-6
        return (f(U + h * d) - f(U - h * d)) / (2 * h)
    h = 1e-30
    return np.imag(f(U + 1j * h * d)) / h


@pytest.mark.parametrize("case", list(CASES))
def test_dg_residual_vjp(case):
    wl = CASES[case]()
    lf = wl.dg_flux == W.FLUX_LAX_FRIEDRICHS
    ora = IMEXSolver(wl)
    rng = np.random.default_rng(7)
    U = ora.U
    if lf:
        # the Lax-Friedrichs bound max(|u.n| + c) over both sides has kinks where the two
        # wave speeds tie, as in an exactly uniform free stream; evaluate at a generic point
        U = U * (1.0 + 1e-3 * rng.standard_normal(U.shape))
    d = rng.standard_normal(U.shape) * 1e-2 * np.abs(U).max()
    Rbar = rng.standard_normal(U.shape)
    Rbar[ora.mesh.im_elems] = 0.0

    def f(X):
        return dg_residual(X, None, wl, ora.mesh, ora.basis, ora.gas)
    jd = _oracle_jvp(f, U, d, lf)
    ref = float(np.sum(Rbar * jd))
    eng = gpu_engine(wl)
    Ub = eng.vjp_dg_residual(torch.tensor(U, device="cuda"), torch.tensor(Rbar, device="cuda")).cpu().numpy()
    got = float(np.sum(Ub * d))
    err = abs(got - ref) / max(abs(ref), 1e-300)
    print(case, got, ref, err)
    assert err < (1e-7 if lf else 1e-10)


def _oracle_explicit_step(ora, U):
    """The oracle's explicit ARK recursion (all elements explicit), any dtype."""
    tab, dt = ora.tab, ora.wl.dt
    ex = ora.mesh.ex_elems
    sub = _sub(ora.geo, ex)
    Y = U.copy()
    Rs = []
    for i in range(1, tab.s + 1):
        Rs.append(dg_residual(Y, None, ora.wl, ora.mesh, ora.basis, ora.gas))
        acc = sum(tab.Ae[i, j] * Rs[j] for j in range(i))
        Y = Y.copy()
        Y[ex] = U[ex] - dt * apply_minv(acc[ex], ora.basis, sub)
    if tab.fsal:
        return Y
    Rs.append(dg_residual(Y, None, ora.wl, ora.mesh, ora.basis, ora.gas))
    acc = sum(tab.be[j] * Rs[j] for j in range(tab.s + 1))
    out = U.copy()
    out[ex] = U[ex] - dt * apply_minv(acc[ex], ora.basis, sub)
    return out


@pytest.mark.parametrize("case,tableau", [("square_explicit", "ARS222"), ("square_explicit", "ARS343"),
                                          ("square_farfield", "ARS343")])
def test_ark_step_vjp(case, tableau):
    wl = CASES[case]()
    wl.tableau = tableau
    ora = IMEXSolver(wl)
    rng = np.random.default_rng(11)
    U = ora.U
    d = rng.standard_normal(U.shape) * 1e-2 * np.abs(U).max()
    Ub_next = rng.standard_normal(U.shape)
    jd = _oracle_jvp(lambda X: _oracle_explicit_step(ora, X), U, d, False)
    # the forward recursion itself matches the GPU step
    eng = gpu_engine(wl)
    Ut = torch.tensor(U, device="cuda")
    U1 = Ut.clone()
    eng.ark_step(wl.dt, U1, None)
    assert np.abs(U1.cpu().numpy() - _oracle_explicit_step(ora, U)).max() < 1e-11 * np.abs(U).max()
    ref = float(np.sum(Ub_next * jd))
    Ub = eng.vjp_ark_step(wl.dt, Ut, torch.tensor(Ub_next, device="cuda")).cpu().numpy()
    got = float(np.sum(Ub * d))
    err = abs(got - ref) / abs(ref)
    print(case, tableau, got, ref, err)
    assert err < 1e-10


def test_rollout_checkpointing_and_fd():
    from paper_2607_16044_amd.autograd import ark_rollout
    wl = smooth_square(4, 2, viscous=True)
    eng = gpu_engine(wl)
    U0 = eng.initial_state()
    nsteps, record = 7, [3, 5, 7]
    rng = np.random.default_rng(3)
    w = torch.tensor(rng.standard_normal((len(record),) + tuple(U0.shape)), device="cuda")

    def J(U, every):
        out = ark_rollout(eng, U, wl.dt, nsteps, record, checkpoint=every)
        return (out * w).sum() / len(record)

    grads = []
    for every in (2, 3, 100):
        U = U0.clone().requires_grad_(True)
        J(U, every).backward()
        grads.append(U.grad.detach().clone())
    for g in grads[1:]:
        assert torch.allclose(g, grads[0], rtol=0, atol=1e-13 * float(grads[0].abs().max()))
    d = torch.tensor(rng.standard_normal(tuple(U0.shape)), device="cuda") * 1e-2 * float(U0.abs().max())
    h = 1e-6
    with torch.no_grad():
        fd = (J(U0 + h * d, 100) - J(U0 - h * d, 100)) / (2 * h)
    got = float((grads[0] * d).sum())
    err = abs(got - float(fd)) / abs(float(fd))
    print("rollout", got, float(fd), err)
    assert err < 1e-6


IMEX_CASES = {
    "vortex_small": lambda: W.get("vortex_small"),
    "square_ip_viscous": lambda: smooth_square(4, 2, viscous=True, variant=W.HDG_IP, implicit_rows=(1, 2)),
    "bl_small_ip": lambda: W.boundary_layer(nx=4, ny=5, k=2, implicit_rows=2, Lx=4 * 2.0 / 256, height=None,
                                            steps=1, name="bl_ip", hdg_variant=W.HDG_IP),
}


@pytest.mark.parametrize("case", list(IMEX_CASES))
def test_imex_step_vjp(case):
    wl = IMEX_CASES[case]()
    eng = gpu_engine(wl, newton_rtol=1e-14, gmres_rtol=1e-13)
    rng = np.random.default_rng(5)
    # a generic point: the Lax-Friedrichs bound has kinks where the wave speeds of both
    # sides tie, as in an exactly uniform free stream
    U0 = eng.initial_state()
    U0 = U0 * (1.0 + 1e-3 * torch.tensor(rng.standard_normal(tuple(U0.shape)), device="cuda"))
    H0 = eng.init_facets(U0)
    c = torch.tensor(rng.standard_normal(tuple(U0.shape)), device="cuda")
    d = torch.tensor(rng.standard_normal(tuple(U0.shape)), device="cuda") * 1e-2 * float(U0.abs().max())
    Ub = eng.vjp_imex_step(wl.dt, U0, H0, c)
    got = float((Ub * d).sum())

    def J(U):
        U = U.clone()
        H = eng.init_facets(U)
        eng.ark_step(wl.dt, U, H)
        return float((c * U).sum())
    h = 1e-6
    fd = (J(U0 + h * d) - J(U0 - h * d)) / (2 * h)
    err = abs(got - fd) / abs(fd)
    # the oracle's step (its own Newton and sparse direct solves)
    cn, U0n, dn = c.cpu().numpy(), U0.cpu().numpy(), d.cpu().numpy()

    def Jo(U):
        ora = IMEXSolver(wl, U0=U)
        ora.step()
        return float(np.sum(cn * ora.U))
    fdo = (Jo(U0n + 1e-5 * dn) - Jo(U0n - 1e-5 * dn)) / 2e-5
    erro = abs(got - fdo) / abs(fdo)
    print(case, got, fd, err, fdo, erro, eng.last_adjoint_stats)
    assert err < 1e-6
    assert erro < 1e-4


def test_rollout_imex_checkpointing():
    from paper_2607_16044_amd.autograd import ark_rollout
    wl = W.get("vortex_small")
    eng = gpu_engine(wl, newton_rtol=1e-14, gmres_rtol=1e-13)
    rng = np.random.default_rng(9)
    U0 = eng.initial_state()
    U0 = U0 * (1.0 + 1e-3 * torch.tensor(rng.standard_normal(tuple(U0.shape)), device="cuda"))
    nsteps, record = 4, [2, 4]
    w = torch.tensor(rng.standard_normal((len(record),) + tuple(U0.shape)), device="cuda")

    def J(U, every):
        return (ark_rollout(eng, U, wl.dt, nsteps, record, checkpoint=every) * w).sum()

    grads = []
    for every in (1, 3, 10):
        U = U0.clone().requires_grad_(True)
        J(U, every).backward()
        grads.append(U.grad.detach().clone())
    for g in grads[1:]:
        assert torch.allclose(g, grads[0], rtol=0, atol=1e-12 * float(grads[0].abs().max()))
    d = torch.tensor(rng.standard_normal(tuple(U0.shape)), device="cuda") * 1e-2 * float(U0.abs().max())
    h = 1e-6
    with torch.no_grad():
        fd = (J(U0 + h * d, 10) - J(U0 - h * d, 10)) / (2 * h)
    got = float((grads[0] * d).sum())
    err = abs(got - float(fd)) / abs(float(fd))
    print("rollout imex", got, float(fd), err)
    assert err < 1e-6
