"""The 3D explicit DG residual on the GPU against the oracle (eq. bilinear_form_interior_sdg
in three dimensions, five variables).

* Small meshes, every degree 1..3: Euler with Lax-Friedrichs on a periodic box;
  Navier-Stokes with the Vijayasundaram flux on a periodic box, on a box with far-field
  sides and graded rows, and with Lax-Friedrichs and far-field sides; per-field relative
  error 1e-12.
* A uniform state has a zero residual on the GPU (free stream, far-field sides).
* The channel at full size (64 x 32 x 32 hexahedra, k = 3, 21 M unknowns, rows graded to a
  first-cell aspect ratio of 500): sampled elements against the oracle at 1e-10 (the
  element residual is a sum of face and volume terms each about 1e3 times larger than
  itself on the thinnest rows; the FP64 cancellation leaves about 1e-13 of those terms).
"""
import numpy as np
import pytest
import torch

from _common import ensure_built, rel_err
from oracle import dg3d as D
from paper_2607_16044_amd import workloads as W

pytestmark = pytest.mark.gpu


def _engine(wl):
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    ensure_built()
    from paper_2607_16044_amd.binding import Engine3D
    return Engine3D(wl)


def _oracle(wl, U, elems=None):
    b, m, g = D.Basis3(wl.degree), D.Mesh3(wl), D.Gas3(wl.gamma, wl.R, wl.mu, wl.Pr)
    return D.dg_residual3d(U, wl, m, b, g, elems=elems)


CASES = [
    ("euler_lf_periodic", dict(viscous=False, flux=W.FLUX_LAX_FRIEDRICHS)),
    ("ns_vij_periodic", dict(viscous=True, flux=W.FLUX_VIJAYASUNDARAM)),
    ("ns_vij_farfield_graded", dict(viscous=True, flux=W.FLUX_VIJAYASUNDARAM, bc=(W.BC_FARFIELD,) * 6, stretch=0.4)),
    ("ns_lf_farfield", dict(viscous=True, flux=W.FLUX_LAX_FRIEDRICHS,
                            bc=(W.BC_PERIODIC, W.BC_PERIODIC, W.BC_FARFIELD, W.BC_FARFIELD, W.BC_FARFIELD,
                                W.BC_FARFIELD))),
]


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("name,kw", CASES, ids=[c[0] for c in CASES])
def test_residual_matches_oracle(name, kw, k):
    wl = W.smooth_box3d(n=(3, 2, 4), k=k, **kw)
    eng = _engine(wl)
    U = eng.initial_state()
    R = eng.residual(U).cpu().numpy()
    ref = _oracle(wl, U.cpu().numpy())
    e = rel_err(R, ref)
    print(name, k, e)
    assert e < 1e-12
    eng.close()


def test_free_stream():
    wl = W.smooth_box3d(n=(2, 3, 2), k=3, viscous=True, bc=(W.BC_FARFIELD,) * 6)
    eng = _engine(wl)
    U = torch.tensor(np.broadcast_to(wl.u_inf.reshape(1, 5, 1), eng.state_shape()).copy(), device="cuda")
    R = eng.residual(U)
    assert float(R.abs().max()) < 1e-12
    eng.close()


def test_channel_full_size_samples():
    wl = W.channel3d()
    eng = _engine(wl)
    U = eng.initial_state()
    R = eng.residual(U)
    torch.cuda.synchronize()
    rng = np.random.default_rng(7)
    E = eng.n_elem
    nx, ny = wl.nx, wl.ny
    rows = [0, 1, 15, 30, 31]                                # wall-adjacent, core and top rows
    sample = np.unique(np.concatenate([rng.integers(0, E, 24),
                                       [rng.integers(0, nx) + nx * (r + ny * rng.integers(0, wl.nz)) for r in rows]]))
    ref = _oracle(wl, U.cpu().numpy(), elems=sample)
    e = rel_err(R.cpu().numpy()[sample], ref)
    print("channel samples", len(sample), e)
    assert e < 1e-10
    assert torch.isfinite(R).all()
    eng.close()
