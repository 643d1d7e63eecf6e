"""The speedup model of the split (Sec. 4.4, eqs. speedup, time_step_ratio, efficiency) on the GPU.

S = r_t eta with r_t the ratio of the stable time steps of the IMEX run and of the fully
explicit run and eta the ratio of their costs per step.  On isentropic vortices whose
centred strip is compressed by a factor r, the explicit step is set by the thinnest
elements and the IMEX step by the uncompressed explicit ones, so r_t grows linearly in
r; r_t >= 1 by construction and eta < 1 when implicit elements cost more.  The stable step is
found by bisection (a run to t_end stays finite with the density in (0, 2 max rho_0]).
"""
import math

import pytest

pytestmark = pytest.mark.gpu


def test_time_step_ratio_grows_linearly_with_the_compression():
    import bench
    res = bench.dt_study(compressions=(4.0, 16.0), n=16, k=2, strip_rows=2, t_end=0.1, bisections=6)
    rows = {r["compression"]: r for r in res["rows"]}
    for r in rows.values():
        print(r)
        assert r["r_t"] >= 1.0
        assert math.isclose(r["speedup"], r["r_t"] * r["eta"], rel_tol=1e-12)
        assert 0.0 < r["eta"] < 1.0                    # an implicit element costs more than an explicit one
    growth = rows[16.0]["r_t"] / rows[4.0]["r_t"]
    print("r_t(16) / r_t(4) =", growth)
    assert 2.5 < growth < 5.5                          # linear in the compression: 4, within the bisection

