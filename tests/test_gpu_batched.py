"""Batched uneven boxes, persistent queue scheduling and graph capture on the GPU.

- every box of a batch equals the same box run alone (bit for bit: the same
  per-tile arithmetic), and the batch matches the oracle box by box (1e-12);
- the persistent per-XCD queue schedule gives the same bits as one workgroup
  per tile, for every tile shape;
- a captured step replayed several times (with eager work in between) gives
  the bits of the eager step each time.
"""
import numpy as np
import pytest

from paper_2210_17509_amd import inputs as I
from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _small_batch(nbox=10, seed=99):
    return I.config2(nbox=nbox, seed=seed, edges=(6, 8, 12, 16, 20))


def _single(prob, b):
    """Box b of a pooled problem as a problem of its own (same data, same metric)."""
    bx = prob.boxes[b]
    c0, v0 = prob.cell_off[b], prob.vert_off[b]
    P = prob.P[:, c0:c0 + bx.ncell]
    a = prob.alpha[v0:v0 + bx.nvert]
    g = prob.gamma[:, v0:v0 + bx.nvert]
    be = None if prob.beta is None else prob.beta[:, v0:v0 + bx.nvert]
    nx, ny, nz = bx.cdims
    vx, vy, vz = bx.vdims
    return I._assemble("single", [bx], prob.params, [[P[q].reshape(nz, ny, nx) for q in range(8)]],
                       [(a.reshape(vz, vy, vx), None if be is None else be.reshape(3, vz, vy, vx),
                         g.reshape(6, vz, vy, vx))], prob.dt, 1, prob.seed)


def test_batch_equals_single_boxes_bitwise():
    prob = _small_batch()
    d = H.Dev(prob)
    d.step(1)
    Ub = d.host(d.U)
    Pb = d.host(d.P)
    for b in range(len(prob.boxes)):
        s = _single(prob, b)
        ds = H.Dev(s)
        ds.step(1)
        c0 = prob.cell_off[b]
        n = prob.boxes[b].ncell
        m = I.interior_mask(prob.boxes[b]).ravel()
        np.testing.assert_array_equal(ds.host(ds.U)[:, :n][:, m], Ub[:, c0:c0 + n][:, m])
        np.testing.assert_array_equal(ds.host(ds.P)[:, :n][:, m], Pb[:, c0:c0 + n][:, m])


@pytest.mark.parametrize("p_current,steps", [(0, 1), (1, 2)])
def test_batch_matches_oracle(orc, p_current, steps):
    prob = _small_batch(8, seed=5)
    d = H.Dev(prob)
    d.par.p_current = p_current
    d.step(steps)
    Uo, Po = orc.prim2con(prob), prob.P.copy()
    orc.rk_step(prob, Uo, Po, steps=steps)
    for a, b in ((d.host(d.U), Uo), (d.host(d.P), Po)):
        r = H.rel_linf(H.interior_fields(prob, a), H.interior_fields(prob, b))
        assert np.all(r <= 1e-12), r


@pytest.mark.parametrize("recon", [I.RECON_MINMOD, I.RECON_WENO5, I.RECON_WENOZ])
def test_thin_boxes_match_oracle(orc, recon):
    """Boxes of 1 to 5 cells a side, fewer than the reconstruction stencil
    reaches: the outflow ghost map sends several stencil cells of a face to the
    same interior cell, and most tiles are mostly empty."""
    prob = I.config2(nbox=12, seed=11, edges=(1, 2, 3, 5), recon=recon)
    assert min(min(b.n) for b in prob.boxes) == 1
    d = H.Dev(prob)
    d.step(2)
    Uo, Po = orc.prim2con(prob), prob.P.copy()
    _, nfail = orc.rk_step(prob, Uo, Po, steps=2)
    assert nfail == 0
    for a, b in ((d.host(d.U), Uo), (d.host(d.P), Po)):
        r = H.rel_linf(H.interior_fields(prob, a), H.interior_fields(prob, b))
        assert np.all(r <= 1e-12), r


@pytest.mark.parametrize("recon", [I.RECON_MINMOD, I.RECON_WENO5, I.RECON_WENOZ])
def test_every_tile_and_schedule_matches_oracle(orc, recon):
    """One SSPRK3 step of a small mixed flat/curved batch, for every tile shape
    and both schedules, against the oracle: each compiled stage-kernel instance
    of the reconstruction is checked on its own (1e-12)."""
    prob = I.config2(nbox=8, seed=61, edges=(6, 12, 20), recon=recon)
    Uo, Po = orc.prim2con(prob), prob.P.copy()
    rate_o, nf_o = orc.rk_step(prob, Uo, Po)
    G = H.G()
    for tile in range(G.GRMHD_NTILE):
        for sched in (G.GRMHD_SCHED_GRID, G.GRMHD_SCHED_QUEUE):
            d = H.Dev(prob, tile=tile)
            d.par.schedule = sched
            d.step(1)
            for name, a, b in (("U", d.host(d.U), Uo), ("P", d.host(d.P), Po)):
                r = H.rel_linf(H.interior_fields(prob, a), H.interior_fields(prob, b))
                assert np.all(r <= 1e-12), f"recon {recon} tile {tile} schedule {sched} {name}: {r}"
            assert int(d.host(d.nfail)[0]) == nf_o
            assert float(d.host(d.rate)[0]) == pytest.approx(rate_o, rel=1e-12)


def _instances_box(shift, precision, recon, wenoz_p=1):
    from tests import problems as T
    beta = ((lambda X, Y, Z: [0.1 * np.sin(2 * np.pi * Y), 0.05 + 0 * X, -0.08 * np.cos(2 * np.pi * X)])
            if shift else None)
    met = T.conformal_metric(lambda X, Y, Z: 1.0 + 0.05 * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Z),
                             alpha_fn=lambda X, Y, Z: 0.9 + 0.05 * np.cos(2 * np.pi * Y), beta_fn=beta)
    bc = (I.BC_OUTFLOW, I.BC_OUTFLOW, I.BC_PERIODIC, I.BC_PERIODIC, I.BC_OUTFLOW, I.BC_OUTFLOW)
    return T.build((37, 13, 11), T.smooth_fields(17, 2.0), met, bc=bc,
                   params=I.Params(recon=recon, eos_gamma=2.0, precision=precision, wenoz_p=wenoz_p))


@pytest.mark.parametrize("kind", ["shift-fp64-weno5", "noshift-mixed-weno5", "shift-mixed-wenoz", "noshift-fp64-wenoz2",
                                  "noshift-mixed-minmod", "shift-fp64-weno5-rk4", "noshift-mixed-weno5-rk4"])
def test_every_instance_agrees_bitwise(kind):
    """Every tile shape and schedule computes the same face numbers, so two steps
    (SSPRK3, or classic RK4 with its step accumulator) agree bit for bit with
    the default tile's grid launch: this checks each compiled stage-kernel
    instance (shifted metric, FP32 faces, WENO-Z with p = 2) against the one the
    parity tests compare with the oracle."""
    parts = kind.split("-")
    shift = parts[0] == "shift"
    precision = I.PREC_MIXED if parts[1] == "mixed" else I.PREC_FP64
    recon = {"weno5": I.RECON_WENO5, "wenoz": I.RECON_WENOZ, "wenoz2": I.RECON_WENOZ,
             "minmod": I.RECON_MINMOD}[parts[2]]
    scheme = 2 if kind.endswith("rk4") else 0
    prob = _instances_box(shift, precision, recon, 2 if parts[2] == "wenoz2" else 1)
    G = H.G()
    outs = {}
    for tile in range(G.GRMHD_NTILE):
        for sched in (G.GRMHD_SCHED_GRID, G.GRMHD_SCHED_QUEUE):
            d = H.Dev(prob, tile=tile)
            d.par.schedule = sched
            d.step(2, scheme=scheme)
            outs[(tile, sched)] = (H.interior_fields(prob, d.host(d.U)), H.interior_fields(prob, d.host(d.P)),
                                   float(d.host(d.rate)[0]))
    ref = outs[(3, G.GRMHD_SCHED_GRID)]
    for key, (U, P, rate) in outs.items():
        np.testing.assert_array_equal(U, ref[0], err_msg=f"{kind} tile/schedule {key} U")
        np.testing.assert_array_equal(P, ref[1], err_msg=f"{kind} tile/schedule {key} P")
        assert rate == ref[2], key


@pytest.mark.parametrize("p_current", [0, 1])
@pytest.mark.parametrize("tile", [0, 1, 2, 3])
def test_queue_schedule_bitwise(tile, p_current):
    """The persistent schedule reproduces the grid schedule bit for bit (with
    p_current = 1 the queue counters follow a third workspace set)."""
    import torch
    G = H.G()
    for prob in (_small_batch(12, seed=7), I.config1(n=40)):
        outs = []
        for sched in (G.GRMHD_SCHED_GRID, G.GRMHD_SCHED_QUEUE):
            d = H.Dev(prob, tile=tile)
            d.par.schedule = sched
            d.par.p_current = p_current
            rate = torch.zeros(1, dtype=torch.float64, device="cuda")
            for _ in range(2):
                G.grmhd_rk_step(d.dom, d.par, d.met, d.U, d.P, prob.dt, max_rate=rate)
            outs.append((d.host(d.U), d.host(d.P), float(d.host(rate)[0])))
        np.testing.assert_array_equal(H.interior_fields(prob, outs[0][0]), H.interior_fields(prob, outs[1][0]))
        np.testing.assert_array_equal(H.interior_fields(prob, outs[0][1]), H.interior_fields(prob, outs[1][1]))
        assert outs[0][2] == outs[1][2]


@pytest.mark.parametrize("sched,p_current", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_graph_replay_matches_eager(sched, p_current):
    """Replays of a captured step (eager work in between) reproduce the eager step each time."""
    import torch
    from paper_2210_17509_amd.autotune import StepGraph
    G = H.G()
    prob = _small_batch(6, seed=11)
    ge = H.Dev(prob)      # eager reference
    gg = H.Dev(prob)      # graph-driven copy
    ge.par.schedule = gg.par.schedule = sched
    ge.par.p_current = gg.par.p_current = p_current
    graph = StepGraph(gg.dom, gg.par, gg.met, gg.U, gg.P, prob.dt, max_rate=gg.rate, n_fail=gg.nfail)
    for rep in range(3):
        G.grmhd_rk_step(ge.dom, ge.par, ge.met, ge.U, ge.P, prob.dt, max_rate=ge.rate, n_fail=ge.nfail)
        graph.replay()
        torch.cuda.synchronize()
        # unrelated eager work between replays
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(H.interior_fields(prob, gg.host(gg.U)), H.interior_fields(prob, ge.host(ge.U)))
        np.testing.assert_array_equal(H.interior_fields(prob, gg.host(gg.P)), H.interior_fields(prob, ge.host(ge.P)))
        assert float(gg.host(gg.rate)[0]) == float(ge.host(ge.rate)[0])
        del junk


def test_autotune_returns_a_compiled_shape():
    from paper_2210_17509_amd.autotune import autotune
    prob = _small_batch(6, seed=13)
    d = H.Dev(prob)
    p, times = autotune(d.dom, d.par, d.met, d.U, d.P, prob.dt, reps=1)
    assert (p.tile, p.schedule) in times and len(times) == 2 * H.G().GRMHD_NTILE
    assert times[(p.tile, p.schedule)] == min(times.values())
