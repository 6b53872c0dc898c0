"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bar: per-field relative L-infinity (max |gpu - oracle| / max |oracle| over
interior cells) <= 1e-12 in FP64, integer outputs (con2prim status, failure
counts) bit-exact.  Small problems are compared everywhere; the workloads at
full size are compared on sampled cells, each computed by the oracle on its
domain of dependence.
"""
import os

import numpy as np
import pytest

from paper_2210_17509_amd import inputs as I
from tests import gpu_helpers as H
from tests import problems as T

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2210_17509_amd import grmhd  # noqa: F401  (fails loudly if the library is missing)


def _ragged(recon=I.RECON_WENO5):
    bc = (I.BC_OUTFLOW, I.BC_OUTFLOW, I.BC_PERIODIC, I.BC_PERIODIC, I.BC_OUTFLOW, I.BC_OUTFLOW)
    def f(X, Y, Z):
        return I.flat_fields(np.random.default_rng(77), X, Y, Z, 5.0 / 3.0, jump_at=0.4)
    return T.build((19, 13, 10), f, bc=bc, params=I.Params(recon=recon))


def _shifted():
    met = T.conformal_metric(lambda X, Y, Z: 1.0 + 0.05 * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Z),
                             alpha_fn=lambda X, Y, Z: 0.9 + 0.05 * np.cos(2 * np.pi * Y),
                             beta_fn=lambda X, Y, Z: [0.1 * np.sin(2 * np.pi * Y), 0.05 + 0 * X,
                                                      -0.08 * np.cos(2 * np.pi * X)])
    return T.build((12, 10, 9), T.smooth_fields(5, 2.0), met, params=I.Params(recon=I.RECON_WENO5, eos_gamma=2.0))


def _oned():
    bc = (I.BC_OUTFLOW, I.BC_OUTFLOW) + (I.BC_PERIODIC,) * 4
    def f(X, Y, Z):
        left = X < 0.5
        row = [np.where(left, 1.0, 0.125), 0 * X, 0 * X, 0 * X, np.where(left, 1.0, 0.8), 0.5 + 0 * X,
               np.where(left, 1.0, -1.0), 0 * X]
        return row
    return T.build((40, 1, 1), f, bc=bc, dx=(1 / 40, 1.0, 1.0), params=I.Params(recon=I.RECON_MINMOD, eos_gamma=2.0),
                   dt=0.25 / 40)


CASES = {
    "config0_minmod_jump": lambda: I.config0(n=16),
    "config1_weno5_curved": lambda: I.config1(n=24),
    "config4_wenoz": lambda: I.config4(n=16),
    "ragged_weno5": _ragged,
    "ragged_minmod_ng2": lambda: _ragged_ng2(),
    "shifted_metric": _shifted,
    "oned_periodic_yz": _oned,
}


def _ragged_ng2():
    bc = (I.BC_PERIODIC,) * 2 + (I.BC_OUTFLOW,) * 4
    def f(X, Y, Z):
        return I.flat_fields(np.random.default_rng(78), X, Y, Z, 5.0 / 3.0, jump_at=0.6)
    return T.build((11, 7, 17), f, bc=bc, ng=2, params=I.Params(recon=I.RECON_MINMOD))


def _assert_close(gpu, ref, tol=TOL, what=""):
    r = H.rel_linf(gpu, ref)
    assert np.all(r <= tol), f"{what} rel L-inf per field {r}"
    return r


@pytest.mark.parametrize("case", sorted(CASES))
def test_prim2con_parity(orc, case):
    prob = CASES[case]()
    d = H.Dev(prob)
    Ug = H.interior_fields(prob, d.host(d.U))
    Uo = H.interior_fields(prob, orc.prim2con(prob))
    _assert_close(Ug, Uo, 1e-14, case)


@pytest.mark.parametrize("case", ["config1_weno5_curved", "ragged_weno5", "shifted_metric"])
def test_con2prim_parity(orc, case):
    """Perturbed conserved state, previous primitives as the guess; P and the status codes."""
    import torch
    prob = CASES[case]()
    Uo = orc.prim2con(prob)
    rng = np.random.default_rng(1)
    Uo = Uo * (1.0 + 1e-3 * rng.standard_normal(Uo.shape))
    Po = prob.P.copy()
    st_o, nf_o = orc.con2prim(prob, Uo_c := Uo.copy(), Po)
    d = H.Dev(prob)
    d.U.copy_(torch.as_tensor(Uo))
    status = torch.zeros(prob.cell_stride, dtype=torch.int32, device="cuda")
    H.G().grmhd_con2prim(d.dom, d.par, d.met, d.U, d.P, status, d.nfail)
    _assert_close(H.interior_fields(prob, d.host(d.P)), H.interior_fields(prob, Po), TOL, case)
    _assert_close(H.interior_fields(prob, d.host(d.U)), H.interior_fields(prob, Uo_c), 1e-15, case)
    sg = d.host(status)
    mask = np.concatenate([I.interior_mask(b).ravel() for b in prob.boxes])
    np.testing.assert_array_equal(sg[:mask.size][mask], st_o[:mask.size][mask])
    assert int(d.host(d.nfail)[0]) == nf_o


def test_con2prim_failures_and_atmosphere(orc):
    """Unrecoverable and floor states: identical statuses, atmosphere values and U rewrite."""
    import torch
    prob = I.config1(n=12)
    U = orc.prim2con(prob)
    bx = prob.boxes[0]
    Uv = prob.box_view(U, 0)
    g = bx.ng
    Uv[1, g + 2, g + 3, g + 4] = 50.0 * (Uv[4, g + 2, g + 3, g + 4] + Uv[0, g + 2, g + 3, g + 4])  # superluminal
    Uv[0, g + 5, g + 5, g + 5] = 1e-14                                                              # below floor
    Uv[4, g + 1, g + 7, g + 2] = np.nan                                                             # non-finite
    Po = prob.P.copy()
    Uo = U.copy()
    st_o, nf_o = orc.con2prim(prob, Uo, Po)
    d = H.Dev(prob)
    d.U.copy_(torch.as_tensor(U))
    status = torch.zeros(prob.cell_stride, dtype=torch.int32, device="cuda")
    H.G().grmhd_con2prim(d.dom, d.par, d.met, d.U, d.P, status, d.nfail)
    m = I.interior_mask(bx).ravel()
    np.testing.assert_array_equal(d.host(status)[m], st_o[m])
    assert set(np.unique(st_o[m])) >= {0, 1, 4}
    assert int(d.host(d.nfail)[0]) == nf_o >= 2
    _assert_close(H.interior_fields(prob, d.host(d.P)), H.interior_fields(prob, Po), TOL)
    _assert_close(H.interior_fields(prob, d.host(d.U)), H.interior_fields(prob, Uo), TOL)


def test_con2prim_atmosphere_state_is_a_fixed_point(orc):
    """Cells already at the atmosphere in strong fields (B^2 up to ~1.4, so the
    thermal energy lies below the rounding of tau) keep status FLOOR and their
    U bit for bit, on the GPU as in the oracle; a density 1% above the floor is
    recovered (status 0)."""
    import torch
    prob = I.config0(n=12)
    par = prob.params
    eps_atm = par.atm_K * par.rho_atm ** par.atm_gamma / ((par.eos_gamma - 1.0) * par.rho_atm)
    U = orc.prim2con(prob)
    bx = prob.boxes[0]
    Uv, Pv = prob.box_view(U, 0), prob.box_view(prob.P, 0)
    g = bx.ng
    cells = [(g + 1, g + 2, g + 3), (g + 5, g + 4, g + 7), (g + 9, g + 9, g + 1)]
    fields = [[1.0, 0.5, -0.3], [0.2, -0.9, 0.7], [-0.6, 0.1, 0.4]]
    P0 = prob.P.copy()
    P0v = prob.box_view(P0, 0)
    for (k, j, i), B in zip(cells, fields):
        Pa = np.array([par.rho_atm, 0, 0, 0, eps_atm] + B)
        Uv[:, k, j, i] = orc.point_p2c(Pa, par.eos_gamma)
        P0v[:, k, j, i] = Pa
    k1, j1, i1 = g + 3, g + 8, g + 6  # 1% above the floor, weak field
    P1 = np.array([1.01 * par.rho_atm, 0.1, 0, 0, 1.0, 1e-6, 0, 0])
    Uv[:, k1, j1, i1] = orc.point_p2c(P1, par.eos_gamma)
    P0v[:, k1, j1, i1] = P1 * 0.99
    Uo, Po = U.copy(), P0.copy()
    st_o, nf_o = orc.con2prim(prob, Uo, Po)
    d = H.Dev(prob)
    d.U.copy_(torch.as_tensor(U))
    d.P.copy_(torch.as_tensor(P0))
    status = torch.zeros(prob.cell_stride, dtype=torch.int32, device="cuda")
    H.G().grmhd_con2prim(d.dom, d.par, d.met, d.U, d.P, status, d.nfail)
    sg = d.host(status)
    m = I.interior_mask(bx).ravel()
    np.testing.assert_array_equal(sg[m], st_o[m])
    nx, ny = bx.cdims[0], bx.cdims[1]
    flat = lambda k, j, i: (k * ny + j) * nx + i
    Ug = d.host(d.U)
    for (k, j, i) in cells:
        c = flat(k, j, i)
        assert sg[c] == 1 and st_o[c] == 1
        np.testing.assert_array_equal(Ug[:, c], U[:, c])
    assert sg[flat(k1, j1, i1)] == 0
    assert int(d.host(d.nfail)[0]) == nf_o
    _assert_close(H.interior_fields(prob, d.host(d.P)), H.interior_fields(prob, Po), TOL)


def test_con2prim_newman_hamlin_recovery(orc):
    """A strongly magnetised state behind a Balsara 2 shock (B^2 = 40, S^2 = 890)
    seeded with the pre-shock primitives: the 3D Newton diverges, the
    Newman-Hamlin fallback recovers it (status 5) with the oracle's primitives.
    Regression: a finiteness test written x - x == 0 was contracted into
    fma(a, b, -x) and rejected the fallback's first (finite) pressure."""
    import torch
    prob = T.build((4, 4, 4), T.uniform_fields([1.0, 0.0, 0.0, 0.0, 1.5, 5.0, 0.7, 0.7]),
                   params=I.Params(recon=I.RECON_MINMOD, eos_gamma=5.0 / 3.0))
    U = orc.prim2con(prob)
    Uv = prob.box_view(U, 0)
    g = prob.boxes[0].ng
    Uv[:, g + 1, g + 2, g + 1] = [1.0, 25.804, -10.6, -10.6, 45.09551569773622, 5.0, 2.753021556739678,
                                  2.753021556739678]
    Po, Uo = prob.P.copy(), U.copy()
    st_o, _ = orc.con2prim(prob, Uo, Po)
    d = H.Dev(prob)
    d.U.copy_(torch.as_tensor(U))
    status = torch.zeros(prob.cell_stride, dtype=torch.int32, device="cuda")
    H.G().grmhd_con2prim(d.dom, d.par, d.met, d.U, d.P, status, d.nfail)
    m = I.interior_mask(prob.boxes[0]).ravel()
    np.testing.assert_array_equal(d.host(status)[m], st_o[m])
    assert 5 in set(st_o[m].tolist())
    _assert_close(H.interior_fields(prob, d.host(d.P)), H.interior_fields(prob, Po), TOL)


@pytest.mark.parametrize("tile", [0, 1, 2, 3])
@pytest.mark.parametrize("case", sorted(CASES))
def test_rhs_parity(orc, case, tile):
    prob = CASES[case]()
    d = H.Dev(prob, tile=tile)
    dg = H.interior_fields(prob, d.host(d.rhs()))
    Uo = orc.prim2con(prob)
    do, rate_o, nf_o = orc.rhs(prob, Uo, prob.P.copy())
    _assert_close(dg, H.interior_fields(prob, do), TOL, case)
    assert float(d.host(d.rate)[0]) == pytest.approx(rate_o, rel=1e-12)
    assert int(d.host(d.nfail)[0]) == nf_o


@pytest.mark.parametrize("case", sorted(CASES))
def test_rk_step_parity(orc, case):
    prob = CASES[case]()
    steps = 2 if case in ("config0_minmod_jump", "oned_periodic_yz") else 1
    d = H.Dev(prob)
    d.step(steps)
    Uo, Po = orc.prim2con(prob), prob.P.copy()
    rate_o, nf_o = orc.rk_step(prob, Uo, Po, steps=steps)
    _assert_close(H.interior_fields(prob, d.host(d.U)), H.interior_fields(prob, Uo), TOL, case + " U")
    _assert_close(H.interior_fields(prob, d.host(d.P)), H.interior_fields(prob, Po), TOL, case + " P")
    assert float(d.host(d.rate)[0]) == pytest.approx(rate_o, rel=1e-12)
    assert int(d.host(d.nfail)[0]) == nf_o


@pytest.mark.parametrize("scheme", [0, 1, 2])
def test_rk_step_through_con2prim_failures(orc, scheme):
    """The flat jump recipe at 32^3 (magnetisation up to about 30) over 6 steps:
    from step 4 on, con2prim fails in a growing set of cells inside the fused
    stages (22 cells over the 6 SSPRK3 steps in the oracle) and those cells are
    reset to the atmosphere mid-step.  The failure count must be the oracle's
    exactly and the fields, atmosphere cells and their neighbours included, the
    oracle's to the FP64 bar."""
    prob = I.config0(n=32)
    steps = 6
    d = H.Dev(prob)
    d.step(steps, scheme=scheme)
    Uo, Po = orc.prim2con(prob), prob.P.copy()
    rate_o, nf_o = orc.rk_step(prob, Uo, Po, steps=steps, scheme=scheme)
    nf_g = int(d.host(d.nfail)[0])
    print(f"scheme {scheme}: n_fail gpu {nf_g} oracle {nf_o}", flush=True)
    assert nf_o > 0
    assert nf_g == nf_o
    _assert_close(H.interior_fields(prob, d.host(d.U)), H.interior_fields(prob, Uo), TOL, "U")
    _assert_close(H.interior_fields(prob, d.host(d.P)), H.interior_fields(prob, Po), TOL, "P")
    assert float(d.host(d.rate)[0]) == pytest.approx(rate_o, rel=1e-12)


def test_ssprk2_and_checkpoints(orc):
    import torch
    prob = I.config1(n=20)
    d = H.Dev(prob)
    ck = torch.zeros((2,) + tuple(d.U.shape), dtype=torch.float64, device="cuda")
    d.step(1, scheme=1, ckpt=ck)
    Uo, Po = orc.prim2con(prob), prob.P.copy()
    _, _, cko = orc.rk_step(prob, Uo, Po, scheme=1, ckpt=True)
    _assert_close(H.interior_fields(prob, d.host(d.U)), H.interior_fields(prob, Uo), TOL)
    # the checkpoints hold the primitives of U^n and of the stage state, recovered
    # from the oracle's conserved checkpoints with the same chain of guesses
    ckg = d.host(ck)
    Pg = prob.P.copy()
    for s in range(2):
        Us = cko[0][s].reshape(8, -1).copy()
        orc.con2prim(prob, Us, Pg)
        _assert_close(H.interior_fields(prob, ckg[s]), H.interior_fields(prob, Pg), TOL)


@pytest.mark.parametrize("scheme,schedule", [(0, 0), (0, 1), (1, 0)])
def test_rk_step_from_current_primitives(orc, scheme, schedule):
    """p_current = 1: the step starts from the caller's P (here the primitives U
    was built from, then those each step leaves) instead of recovering them from
    U^n; the result matches the oracle and the default path, and checkpoint 0 is
    the given P itself."""
    import torch
    g = H.G()
    prob = _ragged()
    steps = 3
    d0, d1 = H.Dev(prob), H.Dev(prob)
    d1.par.p_current = 1
    d1.par.schedule = schedule
    nst = 3 if scheme == 0 else 2
    ck = torch.zeros((nst,) + tuple(d1.U.shape), dtype=torch.float64, device="cuda")
    ws = None
    for k in range(steps):
        P_in = d1.P.clone()
        last = k == steps - 1
        ws = g.grmhd_rk_step(d1.dom, d1.par, d1.met, d1.U, d1.P, prob.dt, scheme, ck if last else None, d1.rate,
                             d1.nfail, ws)
    d0.step(steps, scheme=scheme)
    Uo, Po = orc.prim2con(prob), prob.P.copy()
    orc.rk_step(prob, Uo, Po, steps=steps, scheme=scheme)
    U1, P1 = H.interior_fields(prob, d1.host(d1.U)), H.interior_fields(prob, d1.host(d1.P))
    _assert_close(U1, H.interior_fields(prob, Uo), TOL, "U vs oracle")
    _assert_close(P1, H.interior_fields(prob, Po), TOL, "P vs oracle")
    _assert_close(U1, H.interior_fields(prob, d0.host(d0.U)), TOL, "U vs default path")
    _assert_close(P1, H.interior_fields(prob, d0.host(d0.P)), TOL, "P vs default path")
    assert int(d1.host(d1.nfail)[0]) == int(d0.host(d0.nfail)[0])
    np.testing.assert_array_equal(H.interior_fields(prob, d1.host(ck)[0]), H.interior_fields(prob, d1.host(P_in)))
    # SSPRK3 from the caller's P needs a third 8-field set of workspace
    need = g.grmhd_workspace_bytes(d1.dom, d1.par, scheme)
    field = 8 * 8 * d1.dom.cell_stride
    assert need == (3 if scheme == 0 else 2) * field + 256
    if scheme == 0:
        small = torch.empty((2 * field + 256) // 8, dtype=torch.float64, device="cuda")
        with pytest.raises(g.GrmhdError) as e:
            g.grmhd_rk_step(d1.dom, d1.par, d1.met, d1.U, d1.P, prob.dt, scheme, None, None, None, small)
        assert e.value.code == g.GRMHD_EWORKSPACE


@pytest.mark.parametrize("case,p_current,schedule", [("ragged_weno5", 0, 0), ("config0_minmod_jump", 1, 0),
                                                      ("shifted_metric", 1, 1)])
def test_rk4_parity(orc, case, p_current, schedule):
    """Classic RK4 (con2prim, L, combine per stage) against the oracle's RK4, two steps."""
    g = H.G()
    prob = CASES[case]()
    d = H.Dev(prob)
    d.par.p_current = p_current
    d.par.schedule = schedule
    d.step(2, scheme=g.GRMHD_RK4)
    Uo, Po = orc.prim2con(prob), prob.P.copy()
    rate_o, nf_o = orc.rk_step(prob, Uo, Po, steps=2, scheme=2)
    _assert_close(H.interior_fields(prob, d.host(d.U)), H.interior_fields(prob, Uo), TOL, case + " U")
    _assert_close(H.interior_fields(prob, d.host(d.P)), H.interior_fields(prob, Po), TOL, case + " P")
    assert float(d.host(d.rate)[0]) == pytest.approx(rate_o, rel=1e-12)
    assert int(d.host(d.nfail)[0]) == nf_o


def test_rk4_refuses_checkpoints():
    import torch
    g = H.G()
    prob = I.config1(n=8)
    d = H.Dev(prob)
    ck = torch.zeros((4,) + tuple(d.U.shape), dtype=torch.float64, device="cuda")
    with pytest.raises(g.GrmhdError) as e:
        g.grmhd_rk_step(d.dom, d.par, d.met, d.U, d.P, prob.dt, g.GRMHD_RK4, ck)
    assert e.value.code == g.GRMHD_EINVAL


def test_balsara1_rk4_cfl08_gpu():
    """Sec. IV A on the GPU with the paper's shock-tube settings: Balsara 1, 1600
    cells, minmod, HLLE, classic RK4 at dt/dx = 0.8; the peak Lorentz factor at
    t = 0.4 is the printed W ~ 1.458 (within 0.01) and no cell fails con2prim."""
    import json
    g = H.G()
    with open(os.path.join(os.path.dirname(__file__), "golden", "balsara_table1.json")) as f:
        tab = json.load(f)
    t = tab["tests"]["balsara1"]
    L, R = t["left"], t["right"]
    N = 1600

    def fields(X, Y, Z):
        left = X < 0
        rho, eps, vx, vy, vz, bx, by, bz = [np.where(left, l, r) for l, r in zip(L, R)]
        return [rho, vx, vy, vz, eps, bx, by, bz]

    bc = (I.BC_OUTFLOW, I.BC_OUTFLOW) + (I.BC_PERIODIC,) * 4
    prob = T.build((N, 1, 1), fields, bc=bc, x0=(-0.5, 0, 0), dx=(1.0 / N, 1.0, 1.0),
                   params=I.Params(recon=I.RECON_MINMOD, eos_gamma=t["gamma"]), dt=0.8 / N)
    d = H.Dev(prob)
    d.par.p_current = 1
    d.step(int(round(t["t_ref"] / prob.dt)), scheme=g.GRMHD_RK4)
    Pi = T.interior(prob, d.host(d.P))[:, 0, 0, :]
    W = 1.0 / np.sqrt(1.0 - (Pi[1] ** 2 + Pi[2] ** 2 + Pi[3] ** 2))
    assert int(d.host(d.nfail)[0]) == 0
    assert abs(W.max() - tab["printed_values"]["balsara1_max_W_at_t_ref"]["value"]) < 0.01, W.max()


@pytest.mark.parametrize("name", ["balsara1", "balsara2", "balsara3", "balsara4", "balsara5"])
def test_balsara_tubes_rk4_parity(orc, name):
    """The five Table I shock tubes (Sec. IV A) on 200 cells, minmod, HLLE, classic
    RK4 at dt/dx = 0.8 for 25 steps: the GPU against the oracle.  Strong shocks,
    p up to 1000 and the W = 22.4 streams of test 4; con2prim failure counts
    bit-exact, fields within 1e-12 (1e-10 for test 4: the inversion is
    conditioned like W^2)."""
    import json
    g = H.G()
    with open(os.path.join(os.path.dirname(__file__), "golden", "balsara_table1.json")) as f:
        tab = json.load(f)
    t = tab["tests"][name]
    L, R = t["left"], t["right"]
    N = 200

    def fields(X, Y, Z):
        left = X < 0
        rho, eps, vx, vy, vz, bx, by, bz = [np.where(left, l, r) for l, r in zip(L, R)]
        return [rho, vx, vy, vz, eps, bx, by, bz]

    bc = (I.BC_OUTFLOW, I.BC_OUTFLOW) + (I.BC_PERIODIC,) * 4
    prob = T.build((N, 1, 1), fields, bc=bc, x0=(-0.5, 0, 0), dx=(1.0 / N, 1.0, 1.0),
                   params=I.Params(recon=I.RECON_MINMOD, eos_gamma=t["gamma"]), dt=0.8 / N)
    d = H.Dev(prob)
    d.par.p_current = 1
    d.step(25, scheme=g.GRMHD_RK4)
    Uo, Po = orc.prim2con(prob), prob.P.copy()
    _, nf_o = orc.rk_step(prob, Uo, Po, steps=25, scheme=2)
    tol = 1e-10 if name == "balsara4" else TOL
    _assert_close(H.interior_fields(prob, d.host(d.U)), H.interior_fields(prob, Uo), tol, name + " U")
    _assert_close(H.interior_fields(prob, d.host(d.P)), H.interior_fields(prob, Po), tol, name + " P")
    assert int(d.host(d.nfail)[0]) == nf_o


def test_setupA_recipe_parity(orc):
    """The setupA stand-in (curved recipe, periodic faces, RK2 = SSPRK2) against the
    oracle: two steps from the current primitives."""
    prob = I.config1(n=20, bc=I.BC_PERIODIC)
    d = H.Dev(prob)
    d.par.p_current = 1
    d.step(2, scheme=1)
    Uo, Po = orc.prim2con(prob), prob.P.copy()
    orc.rk_step(prob, Uo, Po, steps=2, scheme=1)
    _assert_close(H.interior_fields(prob, d.host(d.U)), H.interior_fields(prob, Uo), TOL, "U")
    _assert_close(H.interior_fields(prob, d.host(d.P)), H.interior_fields(prob, Po), TOL, "P")


def test_rk_step_from_current_primitives_mixed():
    """Mixed precision (FP32 reconstruction + HLLE) from the caller's P matches the
    default mixed-precision path: the skipped con2prim polish moves P by an FP64
    ulp at most, which can flip the FP32 rounding of a face value (one FP32 ulp,
    6e-8, times dt / dx in U), hence 1e-7."""
    prob = I.config3(n=24, steps=1)
    d0, d1 = H.Dev(prob), H.Dev(prob)
    d1.par.p_current = 1
    d0.step(3)
    d1.step(3)
    _assert_close(H.interior_fields(prob, d1.host(d1.U)), H.interior_fields(prob, d0.host(d0.U)), 1e-7, "U")
    _assert_close(H.interior_fields(prob, d1.host(d1.P)), H.interior_fields(prob, d0.host(d0.P)), 1e-7, "P")


@pytest.mark.parametrize("recon", [I.RECON_MINMOD, I.RECON_WENO5, I.RECON_WENOZ])
def test_uniform_state_bitwise(recon):
    state = [0.7, 0.3, -0.2, 0.1, 1.2, 0.5, -0.4, 0.8]
    bc = (I.BC_OUTFLOW, I.BC_OUTFLOW, I.BC_PERIODIC, I.BC_PERIODIC, I.BC_OUTFLOW, I.BC_OUTFLOW)
    prob = T.build((21, 9, 6), T.uniform_fields(state), bc=bc, params=I.Params(recon=recon))
    d = H.Dev(prob)
    U0 = d.host(d.U).copy()
    d.step(2)
    np.testing.assert_array_equal(H.interior_fields(prob, d.host(d.U)), H.interior_fields(prob, U0))
    Pi = H.interior_fields(prob, d.host(d.P))
    assert np.all(Pi == Pi[:, :1])


def test_conservation_periodic():
    prob = T.build((24, 20, 16), T.smooth_fields(4, 5.0 / 3.0), params=I.Params(recon=I.RECON_WENO5))
    d = H.Dev(prob)
    dd = H.interior_fields(prob, d.host(d.rhs()))
    for q in range(8):
        assert abs(dd[q].sum()) <= 1e-13 * np.abs(dd[q]).sum()


@pytest.mark.parametrize("n", [(1, 2, 3), (2, 1, 5)])
@pytest.mark.parametrize("recon", [I.RECON_MINMOD, I.RECON_WENO5, I.RECON_WENOZ])
def test_periodic_box_narrower_than_ghosts(orc, n, recon):
    """Periodic box with 1 or 2 cells along an axis, fewer than its 3 ghost
    layers: the periodic ghost map wraps more than once."""
    met = T.conformal_metric(lambda X, Y, Z: 1.0 + 0.05 * np.sin(2 * np.pi * Z),
                             alpha_fn=lambda X, Y, Z: 0.95 + 0 * X)
    prob = T.build(n, T.smooth_fields(15, 5.0 / 3.0), met, dx=(0.2, 0.2, 0.2), params=I.Params(recon=recon))
    d = H.Dev(prob)
    d.step(2)
    Uo, Po = orc.prim2con(prob), prob.P.copy()
    _, nfail = orc.rk_step(prob, Uo, Po, steps=2)
    assert nfail == 0
    for a, b in ((d.host(d.U), Uo), (d.host(d.P), Po)):
        r = H.rel_linf(H.interior_fields(prob, a), H.interior_fields(prob, b))
        assert np.all(r <= 1e-12), r


def test_config0_full_size(orc):
    """64^3 minmod with the jump: every interior cell against the oracle."""
    prob = I.config0()
    d = H.Dev(prob)
    d.step(1)
    Uo, Po = orc.prim2con(prob), prob.P.copy()
    rate_o, nf_o = orc.rk_step(prob, Uo, Po)
    _assert_close(H.interior_fields(prob, d.host(d.U)), H.interior_fields(prob, Uo), TOL, "U")
    _assert_close(H.interior_fields(prob, d.host(d.P)), H.interior_fields(prob, Po), TOL, "P")
    assert float(d.host(d.rate)[0]) == pytest.approx(rate_o, rel=1e-12)
    assert int(d.host(d.nfail)[0]) == nf_o == 0


def _sampled(orc, prob, d, nsample, seed, tol):
    bx = prob.boxes[0]
    g = bx.ng
    n = bx.n
    rng = np.random.default_rng(seed)
    cells = [tuple(int(rng.integers(0, n[q])) for q in range(3)) for _ in range(nsample)]
    cells += [(0, 0, 0), (n[0] - 1, n[1] - 1, n[2] - 1), (n[0] // 2, n[1] // 2, n[2] // 2)]
    Ug = prob.box_view(d.host(d.U), 0)
    Pg = prob.box_view(d.host(d.P), 0)
    ref_U, ref_P, got_U, got_P = [], [], [], []
    for c in cells:
        sub, ci = H.sub_problem(prob, c, radius=9)
        Us, Ps = orc.prim2con(sub), sub.P.copy()
        orc.rk_step(sub, Us, Ps)
        ref_U.append(sub.box_view(Us, 0)[:, ci[2] + g, ci[1] + g, ci[0] + g])
        ref_P.append(sub.box_view(Ps, 0)[:, ci[2] + g, ci[1] + g, ci[0] + g])
        got_U.append(Ug[:, c[2] + g, c[1] + g, c[0] + g])
        got_P.append(Pg[:, c[2] + g, c[1] + g, c[0] + g])
    _assert_close(np.array(got_U).T, np.array(ref_U).T, tol, "sampled U")
    _assert_close(np.array(got_P).T, np.array(ref_P).T, tol, "sampled P")


def test_config1_full_size_sampled(orc):
    """256^3 curved WENO5 step in the benchmark's launch configuration, sampled cells."""
    prob = I.config1()
    d = H.Dev(prob)
    d.step(1)
    assert int(d.host(d.nfail)[0]) == 0
    _sampled(orc, prob, d, 24, 5, TOL)


def test_config1_384_sampled(orc):
    """Largest single-box size in the workloads: 384^3 curved WENO5 (FP64)."""
    prob = I.config1(n=384, seed=I.SEED_BASE + 3)
    d = H.Dev(prob)
    d.step(1)
    _sampled(orc, prob, d, 12, 6, TOL)


def test_mixed_precision_error_bound(orc):
    """FP32 reconstruction + HLLE, FP64 elsewhere: one step of the curved WENO5 workload
    stays within 2e-6 relative L-infinity of the FP64 oracle per field."""
    prob = I.config1(n=32, precision=I.PREC_MIXED)
    d = H.Dev(prob)
    d.step(1)
    Uo, Po = orc.prim2con(prob), prob.P.copy()
    orc.rk_step(prob, Uo, Po)
    r = _assert_close(H.interior_fields(prob, d.host(d.U)), H.interior_fields(prob, Uo), 2e-6, "mixed U")
    assert r.max() > 1e-12  # it really ran in FP32
    _assert_close(H.interior_fields(prob, d.host(d.P)), H.interior_fields(prob, Po), 2e-6, "mixed P")


def test_error_returns_on_device():
    import torch
    g = H.G()
    prob = I.config1(n=8)
    d = H.Dev(prob)
    small = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(g.GrmhdError) as e:
        g.grmhd_rk_step(d.dom, d.par, d.met, d.U, d.P, prob.dt, ws=small)
    assert e.value.code == g.GRMHD_EWORKSPACE
    with pytest.raises(g.GrmhdError) as e:
        g.grmhd_rk_step(d.dom, d.par, d.met, d.U, d.P, -1.0)
    assert e.value.code == g.GRMHD_EINVAL
    # the host box list changed after prepare: refused until prepared again
    d.dom._boxes[0].n[0] += 1
    with pytest.raises(g.GrmhdError) as e:
        g.grmhd_rhs(d.dom, d.par, d.met, d.U, d.P, torch.zeros_like(d.U))
    assert "changed" in str(e.value)
    d.dom._boxes[0].n[0] -= 1
    g.grmhd_rhs(d.dom, d.par, d.met, d.U, d.P, torch.zeros_like(d.U))
    # WENO needs 3 ghost layers
    prob2 = T.build((8, 8, 8), T.smooth_fields(1, 5.0 / 3.0), ng=2, params=I.Params(recon=I.RECON_WENO5))
    d2 = H.Dev(prob2)
    with pytest.raises(g.GrmhdError) as e:
        g.grmhd_rhs(d2.dom, d2.par, d2.met, d2.U, d2.P, torch.zeros_like(d2.U))
    assert "ghost" in str(e.value)
