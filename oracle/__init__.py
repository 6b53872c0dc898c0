"""ctypes wrapper of the serial FP64 GRMHD oracle (``oracle/grmhd_oracle.cpp``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the package smoke check and
the benchmark's CPU-baseline leg.  The product path never imports it.

All arrays are numpy float64 in the pooled layout of
``paper_2210_17509_amd.inputs``; the oracle works on one box at a time, so the
helpers here slice a problem into per-box arrays and back.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "grmhd_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force=True):
    """Compile the oracle with g++ (serial semantics, no FP contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wno-unused-function", _SRC, "-o", _LIB + ".tmp"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Box(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("ng", ctypes.c_int32), ("bc", ctypes.c_int32 * 6),
                ("x0", ctypes.c_double * 3), ("dx", ctypes.c_double * 3)]


class Par(ctypes.Structure):
    _fields_ = [("recon", ctypes.c_int32), ("wenoz_p", ctypes.c_int32), ("c2p_maxit", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("gam", ctypes.c_double), ("weno_eps", ctypes.c_double),
                ("wenoz_eps", ctypes.c_double), ("c2p_tol", ctypes.c_double), ("rho_atm", ctypes.c_double),
                ("atm_K", ctypes.c_double), ("atm_gamma", ctypes.c_double)]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int32)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        pb, pp = ctypes.POINTER(Box), ctypes.POINTER(Par)
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_max_threads.restype = ctypes.c_int
        L.orc_prim2con.argtypes = [pb, pp, _D, _D, _D, _D, _D]
        L.orc_con2prim.argtypes = [pb, pp, _D, _D, _D, _D, _D, _I]
        L.orc_con2prim.restype = ctypes.c_long
        L.orc_rhs.argtypes = [pb, pp, _D, _D, _D, _D, _D, _D, _D]
        L.orc_rhs.restype = ctypes.c_long
        L.orc_rk_step.argtypes = [pb, pp, _D, _D, _D, _D, _D, ctypes.c_double, ctypes.c_int, _D, _D]
        L.orc_rk_step.restype = ctypes.c_long
        L.orc_rk_step_jvp.argtypes = [pb, pp, _D, _D, _D, _D, _D, _D, ctypes.c_double, ctypes.c_int,
                                      ctypes.c_int]
        L.orc_rk_step_jvp.restype = ctypes.c_long
        L.orc_point_p2c.argtypes = [_D, ctypes.c_double, _D, _D, ctypes.c_double, _D]
        L.orc_point_p2c_tmunu.argtypes = [_D, ctypes.c_double, _D, _D, ctypes.c_double, _D]
        L.orc_point_flux.argtypes = [_D, ctypes.c_double, _D, _D, ctypes.c_double, ctypes.c_int, _D]
        L.orc_point_flux_tmunu.argtypes = [_D, ctypes.c_double, _D, _D, ctypes.c_double, ctypes.c_int, _D]
        L.orc_point_speeds.argtypes = [_D, ctypes.c_double, _D, _D, ctypes.c_double, ctypes.c_int, _D, _D]
        L.orc_point_lorentz.argtypes = [_D, ctypes.c_double, _D, _D, ctypes.c_double, _D, _D, _D]
        L.orc_point_c2p.argtypes = [_D, _D, _D, pp]
        L.orc_point_c2p.restype = ctypes.c_int
        L.orc_point_hlle.argtypes = [_D, _D, ctypes.c_double, _D, _D, ctypes.c_double, ctypes.c_int, _D, _D, _D]
        L.orc_recon_line.argtypes = [pp, ctypes.c_int, _D, _D, _D, ctypes.c_int]
        L.orc_point_sources.argtypes = [_D, ctypes.c_double, _D, _D, _D, _D, _D, ctypes.c_double, ctypes.c_int,
                                        _D]
        L.orc_count_ops.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_long)]
        L.orc_point_nh_map.argtypes = [_D, _D, pp, ctypes.c_double, _D]
        L.orc_point_nh_map.restype = ctypes.c_int
        L.orc_point_nh_solve.argtypes = [_D, _D, pp, ctypes.c_double, _D]
        L.orc_point_nh_solve.restype = ctypes.c_int
        L.orc_fill_ghosts.argtypes = [pb, _D]
        L.orc_ct_init.argtypes = [pb, _D, _D, _D, _D, _D, _D]
        L.orc_ct_face_field.argtypes = [pb, _D, _D]
        L.orc_ct_step.argtypes = [pb, pp, _D, _D, _D, _D, _D, _D, ctypes.c_double, ctypes.c_int, ctypes.c_int, _D]
        L.orc_ct_step.restype = ctypes.c_long
        L.orc_ct_edge_rhs.argtypes = [pb, pp, _D, _D, _D, _D, _D]
        _lib = L
    return _lib


def set_threads(n):
    lib().orc_set_threads(int(n))


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _arr(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if n is not None:
        assert a.size == n
    return a


def make_box(spec):
    b = Box()
    for d in range(3):
        b.n[d] = int(spec.n[d])
        b.x0[d] = float(spec.x0[d])
        b.dx[d] = float(spec.dx[d])
    b.ng = int(spec.ng)
    for q in range(6):
        b.bc[q] = int(spec.bc[q])
    return b


def make_par(params):
    p = Par()
    p.recon = int(params.recon)
    p.wenoz_p = int(params.wenoz_p)
    p.c2p_maxit = int(params.c2p_maxit)
    p.gam = float(params.eos_gamma)
    p.weno_eps = float(params.weno_eps)
    p.wenoz_eps = float(params.wenoz_eps)
    p.c2p_tol = float(params.c2p_tol)
    p.rho_atm = float(params.rho_atm)
    p.atm_K = float(params.atm_K)
    p.atm_gamma = float(params.atm_gamma)
    return p


# ---------------------------------------------------------------- point functions

def point_p2c(P, gam, alpha=1.0, beta=None, g=(1, 0, 0, 1, 0, 1), tmunu=False):
    P, g = _arr(P, 8), _arr(g, 6)
    b = None if beta is None else _arr(beta, 3)
    U = np.zeros(8)
    f = lib().orc_point_p2c_tmunu if tmunu else lib().orc_point_p2c
    f(_p(P), float(alpha), _p(b), _p(g), float(gam), _p(U))
    return U


def point_flux(P, gam, d, alpha=1.0, beta=None, g=(1, 0, 0, 1, 0, 1), tmunu=False):
    P, g = _arr(P, 8), _arr(g, 6)
    b = None if beta is None else _arr(beta, 3)
    F = np.zeros(8)
    f = lib().orc_point_flux_tmunu if tmunu else lib().orc_point_flux
    f(_p(P), float(alpha), _p(b), _p(g), float(gam), int(d), _p(F))
    return F


def point_speeds(P, gam, d, alpha=1.0, beta=None, g=(1, 0, 0, 1, 0, 1)):
    P, g = _arr(P, 8), _arr(g, 6)
    b = None if beta is None else _arr(beta, 3)
    lp, lm = ctypes.c_double(), ctypes.c_double()
    lib().orc_point_speeds(_p(P), float(alpha), _p(b), _p(g), float(gam), int(d), ctypes.byref(lp),
                           ctypes.byref(lm))
    return lp.value, lm.value


def point_lorentz(P, gam, alpha=1.0, beta=None, g=(1, 0, 0, 1, 0, 1)):
    P, g = _arr(P, 8), _arr(g, 6)
    b = None if beta is None else _arr(beta, 3)
    W, b2, p = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib().orc_point_lorentz(_p(P), float(alpha), _p(b), _p(g), float(gam), ctypes.byref(W), ctypes.byref(b2),
                            ctypes.byref(p))
    return W.value, b2.value, p.value


def point_c2p(U, guess, params, g=(1, 0, 0, 1, 0, 1)):
    U, P, g = _arr(U, 8).copy(), _arr(guess, 8).copy(), _arr(g, 6)
    st = lib().orc_point_c2p(_p(U), _p(P), _p(g), ctypes.byref(make_par(params)))
    return P, U, st


def point_nh_map(U, p, params, g=(1, 0, 0, 1, 0, 1)):
    """One Newman-Hamlin map p -> p' of the conserved state U: (ok, p', W, z)."""
    U, g = _arr(U, 8), _arr(g, 6)
    out = np.zeros(3)
    ok = lib().orc_point_nh_map(_p(U), _p(g), ctypes.byref(make_par(params)), float(p), _p(out))
    return bool(ok), out[0], out[1], out[2]


def point_nh_solve(U, p0, params, g=(1, 0, 0, 1, 0, 1)):
    """The Newman-Hamlin pressure iteration alone from p0: (ok, p, W, z, T)."""
    U, g = _arr(U, 8), _arr(g, 6)
    out = np.zeros(4)
    ok = lib().orc_point_nh_solve(_p(U), _p(g), ctypes.byref(make_par(params)), float(p0), _p(out))
    return bool(ok), out[0], out[1], out[2], out[3]


def fill_ghosts(spec, P):
    """Boundary fill of one box's (8, ncell) primitive array (returns a filled copy)."""
    Pb = np.ascontiguousarray(np.array(P, dtype=np.float64))
    lib().orc_fill_ghosts(ctypes.byref(make_box(spec)), _p(Pb))
    return Pb


def point_hlle(PL, PR, gam, d, alpha=1.0, beta=None, g=(1, 0, 0, 1, 0, 1)):
    PL, PR, g = _arr(PL, 8), _arr(PR, 8), _arr(g, 6)
    b = None if beta is None else _arr(beta, 3)
    F = np.zeros(8)
    xp, xm = ctypes.c_double(), ctypes.c_double()
    lib().orc_point_hlle(_p(PL), _p(PR), float(alpha), _p(b), _p(g), float(gam), int(d), _p(F),
                         ctypes.byref(xp), ctypes.byref(xm))
    return F, xp.value, xm.value


def recon_line(params, q, linear=False):
    q = _arr(q)
    nf = max(q.size - 5, 0)
    qL, qR = np.zeros(nf), np.zeros(nf)
    lib().orc_recon_line(ctypes.byref(make_par(params)), q.size, _p(q), _p(qL), _p(qR), int(linear))
    return qL, qR


def point_sources(P, gam, alpha, beta, g, dalpha, dbeta, dgamma, form=0):
    P, g, da, dg = _arr(P, 8), _arr(g, 6), _arr(dalpha, 3), _arr(dgamma, 18)
    b = None if beta is None else _arr(beta, 3)
    db = None if dbeta is None else _arr(dbeta, 9)
    S = np.zeros(8)
    lib().orc_point_sources(_p(P), float(alpha), _p(b), _p(g), _p(da), _p(db), _p(dg), float(gam), int(form),
                            _p(S))
    return S


# ---------------------------------------------------------------- box functions

def _box_metric(prob, b):
    """Contiguous per-box metric arrays (alpha, beta or None, gamma)."""
    bx = prob.boxes[b]
    v0, nv = prob.vert_off[b], bx.nvert
    a = np.ascontiguousarray(prob.alpha[v0:v0 + nv])
    be = None if prob.beta is None else np.ascontiguousarray(prob.beta[:, v0:v0 + nv])
    g = np.ascontiguousarray(prob.gamma[:, v0:v0 + nv])
    return a, be, g


def _box_cells(prob, arr, b):
    bx = prob.boxes[b]
    c0 = prob.cell_off[b]
    return np.ascontiguousarray(arr[:, c0:c0 + bx.ncell])


def prim2con(prob, P=None):
    """Conserved variables on interior cells of every box (ghost entries zero)."""
    P = prob.P if P is None else P
    U = np.zeros_like(P)
    L = lib()
    par = make_par(prob.params)
    for b, bx in enumerate(prob.boxes):
        a, be, g = _box_metric(prob, b)
        Pb = _box_cells(prob, P, b)
        Ub = np.zeros_like(Pb)
        L.orc_prim2con(ctypes.byref(make_box(bx)), ctypes.byref(par), _p(a), _p(be), _p(g), _p(Pb), _p(Ub))
        c0 = prob.cell_off[b]
        U[:, c0:c0 + bx.ncell] = Ub
    return U


def con2prim(prob, U, P):
    """In-place con2prim on interior cells of every box; returns (status, n_fail)."""
    L = lib()
    par = make_par(prob.params)
    status = np.zeros(U.shape[1], dtype=np.int32)
    nfail = 0
    for b, bx in enumerate(prob.boxes):
        a, be, g = _box_metric(prob, b)
        Ub, Pb = _box_cells(prob, U, b), _box_cells(prob, P, b)
        st = np.zeros(bx.ncell, dtype=np.int32)
        nfail += L.orc_con2prim(ctypes.byref(make_box(bx)), ctypes.byref(par), _p(a), _p(be), _p(g), _p(Ub),
                                _p(Pb), st.ctypes.data_as(_I))
        c0 = prob.cell_off[b]
        U[:, c0:c0 + bx.ncell] = Ub
        P[:, c0:c0 + bx.ncell] = Pb
        status[c0:c0 + bx.ncell] = st
    return status, nfail


def rhs(prob, U, P):
    """dU/dt on interior cells (U, P updated in place by con2prim); returns (dUdt, max_rate, n_fail)."""
    L = lib()
    par = make_par(prob.params)
    dU = np.zeros_like(U)
    rate = ctypes.c_double(0.0)
    nfail = 0
    for b, bx in enumerate(prob.boxes):
        a, be, g = _box_metric(prob, b)
        Ub, Pb = _box_cells(prob, U, b), _box_cells(prob, P, b)
        dUb = np.zeros_like(Ub)
        nfail += L.orc_rhs(ctypes.byref(make_box(bx)), ctypes.byref(par), _p(a), _p(be), _p(g), _p(Ub), _p(Pb),
                           _p(dUb), ctypes.byref(rate))
        c0 = prob.cell_off[b]
        U[:, c0:c0 + bx.ncell] = Ub
        P[:, c0:c0 + bx.ncell] = Pb
        dU[:, c0:c0 + bx.ncell] = dUb
    return dU, rate.value, nfail


def rk_step(prob, U, P, dt=None, scheme=0, steps=1, ckpt=False):
    """In-place RK steps (scheme 0 = SSPRK3, 1 = SSPRK2, 2 = classic RK4); returns
    (max_rate, n_fail[, ckpts]).  Checkpoints are written for the SSPRK schemes only."""
    if ckpt and scheme == 2:
        raise ValueError("checkpoints are written for the SSPRK schemes only")
    L = lib()
    par = make_par(prob.params)
    dt = prob.dt if dt is None else dt
    rate = ctypes.c_double(0.0)
    nfail = 0
    nst = 2 if scheme == 1 else 3
    cks = []
    for b, bx in enumerate(prob.boxes):
        a, be, g = _box_metric(prob, b)
        Ub, Pb = _box_cells(prob, U, b), _box_cells(prob, P, b)
        ck = np.zeros((nst,) + Ub.shape) if ckpt else None
        for _ in range(steps):
            nfail += L.orc_rk_step(ctypes.byref(make_box(bx)), ctypes.byref(par), _p(a), _p(be), _p(g), _p(Ub),
                                   _p(Pb), float(dt), int(scheme), _p(ck), ctypes.byref(rate))
        c0 = prob.cell_off[b]
        U[:, c0:c0 + bx.ncell] = Ub
        P[:, c0:c0 + bx.ncell] = Pb
        cks.append(ck)
    if ckpt:
        return rate.value, nfail, cks
    return rate.value, nfail


def rk_step_jvp(prob, U, dU, P, dt=None, scheme=0, steps=1):
    """Exact JVP of `steps` RK steps on box 0: returns (U_out, dU_out, P_out)."""
    assert len(prob.boxes) == 1
    L = lib()
    par = make_par(prob.params)
    dt = prob.dt if dt is None else dt
    a, be, g = _box_metric(prob, 0)
    Ub, dUb, Pb = (np.ascontiguousarray(x.copy()) for x in (U, dU, P))
    L.orc_rk_step_jvp(ctypes.byref(make_box(prob.boxes[0])), ctypes.byref(par), _p(a), _p(be), _p(g), _p(Ub),
                      _p(dUb), _p(Pb), float(dt), int(scheme), int(steps))
    return Ub, dUb, Pb


def count_ops(recon):
    """Arithmetic of the method per face and per cell: dict of (add, mul, div, sqrt)."""
    out = (ctypes.c_long * 8)()
    lib().orc_count_ops(int(recon), out)
    return {"face": tuple(out[0:4]), "cell": tuple(out[4:8])}


# ---------------------------------------------------------------- constrained transport (Sec. III B)
#
# A: (3, vert_stride) edge fields (A_x, A_y, A_z), each box's edges stored like its
# vertex metric; A_e of an edge along e sits at the vertex-shaped index with the
# cell index along e in place of that vertex index.

def _box_verts(prob, arr, b):
    bx = prob.boxes[b]
    v0 = prob.vert_off[b]
    return np.ascontiguousarray(arr[:, v0:v0 + bx.nvert])


def ct_init(prob, A, P):
    """Initial data with constrained transport: P's B from the cell-centred Bcal =
    curl A, then U from P.  P is updated in place; returns U."""
    L = lib()
    for b, bx in enumerate(prob.boxes):
        a, be, g = _box_metric(prob, b)
        Ab, Pb = _box_verts(prob, A, b), _box_cells(prob, P, b)
        Ub = np.zeros_like(Pb)
        L.orc_ct_init(ctypes.byref(make_box(bx)), _p(a), _p(be), _p(g), _p(Ab), _p(Ub), _p(Pb))
        c0 = prob.cell_off[b]
        P[:, c0:c0 + bx.ncell] = Pb
    return prim2con(prob, P)


def ct_face_field(prob, A, b=0):
    """Face field Bcal = curl A of box b: (3, ncell) cell-shaped arrays; the d-face at
    vertex index m along d sits at the cell index m (m = n in the first ghost cell)."""
    bx = prob.boxes[b]
    out = np.zeros((3, bx.ncell))
    lib().orc_ct_face_field(ctypes.byref(make_box(bx)), _p(_box_verts(prob, A, b)), _p(out))
    return out


def ct_edge_rhs(prob, P, b=0):
    """dA/dt of box b from primitives P (the magnetic face fluxes of their RHS)."""
    bx = prob.boxes[b]
    a, be, g = _box_metric(prob, b)
    Pb = _box_cells(prob, P, b)
    dA = np.zeros((3, bx.nvert))
    lib().orc_ct_edge_rhs(ctypes.byref(make_box(bx)), ctypes.byref(make_par(prob.params)), _p(a), _p(be), _p(g),
                          _p(Pb), _p(dA))
    return dA


def ct_rk_step(prob, U, P, A, dt=None, scheme=0, steps=1, p_current=0):
    """In-place RK steps with constrained transport (U, P, A); returns (max_rate, n_fail)."""
    L = lib()
    par = make_par(prob.params)
    dt = prob.dt if dt is None else dt
    rate = ctypes.c_double(0.0)
    nfail = 0
    for b, bx in enumerate(prob.boxes):
        a, be, g = _box_metric(prob, b)
        Ub, Pb, Ab = _box_cells(prob, U, b), _box_cells(prob, P, b), _box_verts(prob, A, b)
        for k in range(steps):
            nfail += L.orc_ct_step(ctypes.byref(make_box(bx)), ctypes.byref(par), _p(a), _p(be), _p(g), _p(Ub),
                                   _p(Pb), _p(Ab), float(dt), int(scheme), int(p_current),
                                   ctypes.byref(rate))
        c0, v0 = prob.cell_off[b], prob.vert_off[b]
        U[:, c0:c0 + bx.ncell] = Ub
        P[:, c0:c0 + bx.ncell] = Pb
        A[:, v0:v0 + bx.nvert] = Ab
    return rate.value, nfail
