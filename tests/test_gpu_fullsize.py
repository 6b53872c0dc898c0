"""GPU parity at the workloads' full sizes, every interior cell against the oracle.

- the curved 256^3 WENO5 step (the benchmark workload), in the benchmark's
  launch configuration (steps from the current primitives, default tile and
  schedule), every one of its 16.8 M cells;
- a 112^3 grid whose tile walk needs several strips with a partial last one
  (28 tile rows of 16x4x3 tiles in strips of 9);
- the 400-box batch, every cell of every box, stepped as the benchmark steps it
  (autotuned tile shape and schedule, the step captured in a graph);
- mixed precision: 50 SSPRK3 steps of the 384^3 workload's recipe and spacing
  on the central 64^3 of its domain, with a stated per-field bound on the
  relative L-inf and L2 error against the FP64 oracle.

The oracle runs threaded over k-planes (bitwise equal to its serial build).
"""
import numpy as np
import pytest

from paper_2210_17509_amd import inputs as I
from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu
TOL = 1e-12
ORACLE_THREADS = 16  # the GPU machine's CPU share


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


@pytest.fixture
def orc16(orc):
    orc.set_threads(ORACLE_THREADS)
    yield orc
    orc.set_threads(8)


def _compare_all(prob, gpu_U, gpu_P, Uo, Po, tol, what):
    for name, a, b in (("U", gpu_U, Uo), ("P", gpu_P, Po)):
        r = H.rel_linf(H.interior_fields(prob, a), H.interior_fields(prob, b))
        print(f"{what} {name} rel L-inf per field: " + " ".join(f"{x:.2e}" for x in r), flush=True)
        assert np.all(r <= tol), f"{what} {name}: {r}"


def _step_current_prims(prob, steps=1):
    """Steps as the benchmark runs them: each from the primitives already in P."""
    g = H.G()
    d = H.Dev(prob)
    d.par.p_current = 1
    ws = None
    for _ in range(steps):
        ws = g.grmhd_rk_step(d.dom, d.par, d.met, d.U, d.P, prob.dt, g.GRMHD_SSPRK3, None, d.rate, d.nfail, ws)
    return d


def test_curved256_every_cell(orc16):
    prob = I.config1()
    d = _step_current_prims(prob)
    Ug, Pg = d.host(d.U), d.host(d.P)
    rate_g, nf_g = float(d.host(d.rate)[0]), int(d.host(d.nfail)[0])
    del d
    Uo, Po = orc16.prim2con(prob), prob.P.copy()
    rate_o, nf_o = orc16.rk_step(prob, Uo, Po)
    _compare_all(prob, Ug, Pg, Uo, Po, TOL, "curved 256^3")
    assert nf_g == nf_o == 0
    assert rate_g == pytest.approx(rate_o, rel=1e-12)


def test_partial_last_strip_every_cell(orc16):
    prob = I.config1(n=112, seed=I.SEED_BASE + 112)
    ntx, nty = -(-112 // 16), -(-112 // 4)
    sh = max(1, min(nty, 64 // ntx))
    assert nty > sh and nty % sh != 0  # several strips, the last one partial
    d = _step_current_prims(prob, steps=2)
    Uo, Po = orc16.prim2con(prob), prob.P.copy()
    rate_o, nf_o = orc16.rk_step(prob, Uo, Po, steps=2)
    _compare_all(prob, d.host(d.U), d.host(d.P), Uo, Po, TOL, "curved 112^3")
    assert int(d.host(d.nfail)[0]) == nf_o == 0
    assert float(d.host(d.rate)[0]) == pytest.approx(rate_o, rel=1e-12)


def test_batched400_every_box_every_cell(orc16):
    import torch
    from paper_2210_17509_amd.autotune import StepGraph, autotune
    g = H.G()
    prob = I.config2()
    d = H.Dev(prob)
    d.par.p_current = 1
    par, _ = autotune(d.dom, d.par, d.met, d.U, d.P, prob.dt, reps=1)
    graph = StepGraph(d.dom, par, d.met, d.U, d.P, prob.dt, max_rate=d.rate, n_fail=d.nfail)
    graph.replay()
    torch.cuda.synchronize()
    print(f"batched 400: tile {par.tile} schedule {par.schedule}", flush=True)
    Ug, Pg = d.host(d.U), d.host(d.P)
    nf_g = int(d.host(d.nfail)[0])
    del graph, d
    Uo, Po = orc16.prim2con(prob), prob.P.copy()
    rate_o, nf_o = orc16.rk_step(prob, Uo, Po)
    assert nf_g == nf_o == 0
    # per box, so a wrong box cannot hide behind the pooled maxima
    worst = 0.0
    for b, bx in enumerate(prob.boxes):
        c0, m = prob.cell_off[b], I.interior_mask(bx).ravel()
        for a, ref in ((Ug, Uo), (Pg, Po)):
            r = H.rel_linf(a[:, c0:c0 + bx.ncell][:, m], ref[:, c0:c0 + bx.ncell][:, m])
            worst = max(worst, float(r.max()))
            assert np.all(r <= TOL), f"box {b} {bx.n}: {r}"
    print(f"batched 400: worst per-box rel L-inf {worst:.2e}", flush=True)


# Mixed precision (FP32 reconstruction and HLLE) over 50 SSPRK3 steps against the
# FP64 oracle.  FP32's unit roundoff is 6e-8; the face states and fluxes carry a
# few of it, each stage adds dt/dx = 1/4 of a flux difference, and 150 stages of
# such perturbations (largely uncorrelated) leave the conserved fields within
# ~1e-6 of FP64.  The primitives amplify that through con2prim where pressure is
# small against the other energies.  Bounds per field (relative L-inf, relative L2):
MIXED50_BOUND_U = (5e-6, 1e-6)
MIXED50_BOUND_P = (2e-5, 2e-6)


def test_mixed_precision_50_steps_per_field(orc16):
    """The config-3 recipe (curved metric, WENO5, Gamma = 2) at its 384^3 spacing
    dx = 1/48 on the central 64^3 (no con2prim failure there over 50 steps)."""
    prob = I.config1(n=64, extent=64.0 / 96.0, seed=I.SEED_BASE + 3, steps=50, precision=I.PREC_MIXED)
    d = H.Dev(prob)
    d.step(50)
    Ug, Pg = d.host(d.U), d.host(d.P)
    assert int(d.host(d.nfail)[0]) == 0
    Uo, Po = orc16.prim2con(prob), prob.P.copy()
    _, nf = orc16.rk_step(prob, Uo, Po, steps=50)
    assert nf == 0
    for name, a, b, (linf, l2) in (("U", Ug, Uo, MIXED50_BOUND_U), ("P", Pg, Po, MIXED50_BOUND_P)):
        A, B = H.interior_fields(prob, a), H.interior_fields(prob, b)
        ri = H.rel_linf(A, B)
        r2 = np.linalg.norm(A - B, axis=1) / np.maximum(np.linalg.norm(B, axis=1), 1e-300)
        print(f"mixed 50 steps {name} rel L-inf: " + " ".join(f"{x:.2e}" for x in ri), flush=True)
        print(f"mixed 50 steps {name} rel L2:    " + " ".join(f"{x:.2e}" for x in r2), flush=True)
        assert ri.max() > 1e-10  # it ran in FP32
        assert np.all(ri <= linf), f"{name} rel L-inf {ri}"
        assert np.all(r2 <= l2), f"{name} rel L2 {r2}"
