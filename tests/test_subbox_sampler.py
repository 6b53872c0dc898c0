"""The sampled-parity machinery itself, on the CPU: an oracle run on the
domain-of-dependence sub-box around a cell reproduces the full-grid oracle
result at that cell (so full-size GPU runs can be checked cell by cell)."""
import numpy as np
import pytest

from paper_2210_17509_amd import inputs as I
from tests import gpu_helpers as H


@pytest.mark.parametrize("make,n", [(I.config1, 28), (I.config0, 24)])
def test_subbox_matches_full_grid(orc, make, n):
    prob = make(n=n)
    U, P = orc.prim2con(prob), prob.P.copy()
    orc.rk_step(prob, U, P)
    rng = np.random.default_rng(0)
    cells = [tuple(int(v) for v in rng.integers(0, n, 3)) for _ in range(6)] + [(0, 0, 0), (n - 1, n - 1, n - 1)]
    bx = prob.boxes[0]
    g = bx.ng
    Uv, Pv = prob.box_view(U, 0), prob.box_view(P, 0)
    for c in cells:
        sub, ci = H.sub_problem(prob, c, radius=9)
        Us, Ps = orc.prim2con(sub), sub.P.copy()
        orc.rk_step(sub, Us, Ps)
        sv_U, sv_P = sub.box_view(Us, 0), sub.box_view(Ps, 0)
        a = sv_U[:, ci[2] + g, ci[1] + g, ci[0] + g]
        b = Uv[:, c[2] + g, c[1] + g, c[0] + g]
        np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-15, err_msg=str(c))
        np.testing.assert_allclose(sv_P[:, ci[2] + g, ci[1] + g, ci[0] + g], Pv[:, c[2] + g, c[1] + g, c[0] + g],
                                   rtol=1e-13, atol=1e-15, err_msg=str(c))
