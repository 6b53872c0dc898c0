"""Thin ctypes binding of libgrmhd.so (the C ABI in include/grmhd.h).

The functions carry the C names and only marshal arguments: torch tensors in
device memory become pointers, the current torch stream becomes the HIP
stream, negative return codes become ``GrmhdError``.  All arithmetic runs in
the library's HIP kernels; there is no fallback path.  Importing this module
fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgrmhd.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2210_17509_amd.build` "
                      "or __graft_entry__.build()")

_lib = ctypes.CDLL(LIB_PATH)

GRMHD_OK, GRMHD_EINVAL, GRMHD_EHIP, GRMHD_EWORKSPACE = 0, -1, -2, -3
GRMHD_SSPRK3, GRMHD_SSPRK2, GRMHD_RK4 = 0, 1, 2


class grmhd_box(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("ng", ctypes.c_int32), ("bc", ctypes.c_int32 * 6),
                ("x0", ctypes.c_double * 3), ("dx", ctypes.c_double * 3), ("cell_off", ctypes.c_int64),
                ("vert_off", ctypes.c_int64)]


class grmhd_domain(ctypes.Structure):
    _fields_ = [("box", ctypes.POINTER(grmhd_box)), ("nbox", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("cell_stride", ctypes.c_int64), ("vert_stride", ctypes.c_int64), ("table", ctypes.c_void_p)]


class grmhd_params(ctypes.Structure):
    _fields_ = [("recon", ctypes.c_int32), ("precision", ctypes.c_int32), ("wenoz_p", ctypes.c_int32),
                ("c2p_maxit", ctypes.c_int32), ("tile", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("p_current", ctypes.c_int32),
                ("eos_gamma", ctypes.c_double), ("weno_eps", ctypes.c_double),
                ("wenoz_eps", ctypes.c_double), ("c2p_tol", ctypes.c_double), ("rho_atm", ctypes.c_double),
                ("atm_K", ctypes.c_double), ("atm_gamma", ctypes.c_double)]


class grmhd_metric(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_void_p), ("beta", ctypes.c_void_p), ("gamma", ctypes.c_void_p)]


_P = ctypes.c_void_p
_pd, _pp, _pm = ctypes.POINTER(grmhd_domain), ctypes.POINTER(grmhd_params), ctypes.POINTER(grmhd_metric)
_lib.grmhd_domain_table_bytes.argtypes = [ctypes.c_int32]
_lib.grmhd_domain_table_bytes.restype = ctypes.c_size_t
_lib.grmhd_domain_prepare.argtypes = [_pd, _P]
_lib.grmhd_prim2con.argtypes = [_pd, _pp, _pm, _P, _P, _P]
_lib.grmhd_con2prim.argtypes = [_pd, _pp, _pm, _P, _P, _P, _P, _P]
_lib.grmhd_rhs.argtypes = [_pd, _pp, _pm, _P, _P, _P, _P, _P, _P]
_lib.grmhd_rk_step.argtypes = [_pd, _pp, _pm, _P, _P, ctypes.c_double, ctypes.c_int32, _P, _P, _P, _P,
                               ctypes.c_size_t, _P]
_lib.grmhd_rk_step_noalloc.argtypes = [_pd, _pp, _pm, _P, _P, ctypes.c_double, ctypes.c_int32, _P, _P, _P, _P]
_lib.grmhd_ct_init.argtypes = [_pd, _pp, _pm, _P, _P, _P, _P]
_lib.grmhd_ct_face_field.argtypes = [_pd, _P, _P, _P]
_lib.grmhd_rk_step_ct.argtypes = [_pd, _pp, _pm, _P, _P, _P, ctypes.c_double, ctypes.c_int32, _P, _P, _P,
                                  ctypes.c_size_t, _P]
_lib.grmhd_ct_workspace_bytes.argtypes = [_pd, _pp, ctypes.c_int32]
_lib.grmhd_ct_workspace_bytes.restype = ctypes.c_size_t
_lib.grmhd_workspace_bytes.argtypes = [_pd, _pp, ctypes.c_int32, ctypes.c_int32]
_lib.grmhd_workspace_bytes.restype = ctypes.c_size_t
_lib.grmhd_strerror.argtypes = [ctypes.c_int]
_lib.grmhd_strerror.restype = ctypes.c_char_p
_lib.grmhd_last_error.restype = ctypes.c_char_p
_lib.grmhd_con2prim_adjoint.argtypes = [_pd, _pp, _pm, _P, _P, _P, _P]
_lib.grmhd_rk_step_adjoint.argtypes = [_pd, _pp, _pm, _P, _P, ctypes.c_double, ctypes.c_int32, _P, _P, _P,
                                       ctypes.c_size_t, _P]
_lib.grmhd_timing_enable.argtypes = [ctypes.c_int32]
_lib.grmhd_timing_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]

EXPORTED = ["grmhd_domain_table_bytes", "grmhd_domain_prepare", "grmhd_prim2con", "grmhd_con2prim", "grmhd_rhs",
            "grmhd_rk_step", "grmhd_workspace_bytes", "grmhd_strerror", "grmhd_last_error", "grmhd_timing_enable",
            "grmhd_timing_read", "grmhd_con2prim_adjoint", "grmhd_rk_step_adjoint", "grmhd_rk_step_noalloc",
            "grmhd_ct_init", "grmhd_ct_face_field", "grmhd_rk_step_ct", "grmhd_ct_workspace_bytes"]

GRMHD_NOALLOC_SCRATCH_BYTES = 256 << 20  # the fixed scratch of grmhd_rk_step_noalloc


class GrmhdError(RuntimeError):
    def __init__(self, code):
        self.code = code
        super().__init__(f"{grmhd_strerror(code)}: {grmhd_last_error()}")


def _check(code):
    if code != GRMHD_OK:
        raise GrmhdError(code)


def _ptr(t, dtype=torch.float64):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a device tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"expected a contiguous {dtype} tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


# ------------------------------------------------------------------ domain / metric / params holders

class Domain:
    """Pooled box list plus its prepared device table (keeps everything alive)."""

    def __init__(self, boxes, cell_off, vert_off, cell_stride, vert_stride, device="cuda", stream=None):
        n = len(boxes)
        self._boxes = (grmhd_box * n)()
        for b, (bx, co, vo) in enumerate(zip(boxes, cell_off, vert_off)):
            x = self._boxes[b]
            for d in range(3):
                x.n[d] = int(bx.n[d])
                x.x0[d] = float(bx.x0[d])
                x.dx[d] = float(bx.dx[d])
            x.ng = int(bx.ng)
            for q in range(6):
                x.bc[q] = int(bx.bc[q])
            x.cell_off = int(co)
            x.vert_off = int(vo)
        nbytes = int(_lib.grmhd_domain_table_bytes(n))
        self.table = torch.zeros((nbytes + 7) // 8, dtype=torch.int64, device=device)
        self.c = grmhd_domain(ctypes.cast(self._boxes, ctypes.POINTER(grmhd_box)), n, 0, int(cell_stride),
                              int(vert_stride), ctypes.c_void_p(self.table.data_ptr()))
        self.cell_stride = int(cell_stride)
        self.vert_stride = int(vert_stride)
        self.nbox = n
        grmhd_domain_prepare(self, stream)

    @classmethod
    def from_problem(cls, prob, device="cuda", stream=None):
        return cls(prob.boxes, prob.cell_off, prob.vert_off, prob.cell_stride, prob.vert_stride, device, stream)


class Metric:
    """Device copies of the vertex metric (alpha, optional beta, gamma)."""

    def __init__(self, alpha, beta, gamma, device="cuda"):
        t = lambda a: None if a is None else torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64,
                                                             device=device).contiguous()
        self.alpha, self.beta, self.gamma = t(alpha), t(beta), t(gamma)
        self.c = grmhd_metric(_ptr(self.alpha), _ptr(self.beta) if self.beta is not None else None, _ptr(self.gamma))

    @classmethod
    def from_problem(cls, prob, device="cuda"):
        return cls(prob.alpha, prob.beta, prob.gamma, device)


GRMHD_SCHED_GRID, GRMHD_SCHED_QUEUE = 0, 1
GRMHD_NTILE = 4  # stage-kernel tile shapes: 16x4x4, 8x8x4, 64x2x2, 16x4x3


def make_params(p, tile=-1, schedule=GRMHD_SCHED_GRID, p_current=0):
    """grmhd_params from a paper_2210_17509_amd.inputs.Params."""
    return grmhd_params(int(p.recon), int(p.precision), int(p.wenoz_p), int(p.c2p_maxit), int(tile), int(schedule),
                        int(p_current), float(p.eos_gamma),
                        float(p.weno_eps), float(p.wenoz_eps), float(p.c2p_tol), float(p.rho_atm), float(p.atm_K),
                        float(p.atm_gamma))


def _par(p):
    return p if isinstance(p, grmhd_params) else make_params(p)


# ------------------------------------------------------------------ the C entry points

def grmhd_strerror(code):
    return _lib.grmhd_strerror(int(code)).decode()


def grmhd_last_error():
    return _lib.grmhd_last_error().decode()


def grmhd_domain_table_bytes(nbox):
    return int(_lib.grmhd_domain_table_bytes(int(nbox)))


def grmhd_domain_prepare(dom, stream=None):
    _check(_lib.grmhd_domain_prepare(ctypes.byref(dom.c), _stream(stream)))


def grmhd_prim2con(dom, params, met, P, U, stream=None):
    _check(_lib.grmhd_prim2con(ctypes.byref(dom.c), ctypes.byref(_par(params)), ctypes.byref(met.c), _ptr(P),
                               _ptr(U), _stream(stream)))


def grmhd_con2prim(dom, params, met, U, P, status=None, n_fail=None, stream=None):
    _check(_lib.grmhd_con2prim(ctypes.byref(dom.c), ctypes.byref(_par(params)), ctypes.byref(met.c), _ptr(U),
                               _ptr(P), _ptr(status, torch.int32), _ptr(n_fail, torch.int64), _stream(stream)))


def grmhd_rhs(dom, params, met, U, P, dUdt, max_rate=None, n_fail=None, stream=None):
    _check(_lib.grmhd_rhs(ctypes.byref(dom.c), ctypes.byref(_par(params)), ctypes.byref(met.c), _ptr(U), _ptr(P),
                          _ptr(dUdt), _ptr(max_rate), _ptr(n_fail, torch.int64), _stream(stream)))


def grmhd_workspace_bytes(dom, params, scheme=GRMHD_SSPRK3, for_adjoint=0):
    return int(_lib.grmhd_workspace_bytes(ctypes.byref(dom.c), ctypes.byref(_par(params)), int(scheme),
                                          int(for_adjoint)))


def grmhd_rk_step(dom, params, met, U, P, dt, scheme=GRMHD_SSPRK3, stage_ckpt=None, max_rate=None, n_fail=None,
                  ws=None, stream=None):
    pc = _par(params)
    need = grmhd_workspace_bytes(dom, pc, scheme, 0)
    if ws is None:
        ws = torch.empty((need + 7) // 8, dtype=torch.float64, device=U.device)
    _check(_lib.grmhd_rk_step(ctypes.byref(dom.c), ctypes.byref(pc), ctypes.byref(met.c), _ptr(U), _ptr(P),
                              float(dt), int(scheme), _ptr(stage_ckpt), _ptr(max_rate), _ptr(n_fail, torch.int64),
                              ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel() * ws.element_size()),
                              _stream(stream)))
    return ws


def grmhd_rk_step_noalloc(dom, params, met, U, P, dt, scheme=GRMHD_SSPRK3, stage_ckpt=None, max_rate=None,
                          n_fail=None, stream=None):
    _check(_lib.grmhd_rk_step_noalloc(ctypes.byref(dom.c), ctypes.byref(_par(params)), ctypes.byref(met.c), _ptr(U),
                                      _ptr(P), float(dt), int(scheme), _ptr(stage_ckpt), _ptr(max_rate),
                                      _ptr(n_fail, torch.int64), _stream(stream)))


def grmhd_timing_enable(on=True):
    _check(_lib.grmhd_timing_enable(1 if on else 0))


def grmhd_timing_read():
    """{'stage': (ms, launches), 'con2prim': (ms, launches)} since timing was enabled."""
    ms = (ctypes.c_double * 2)()
    n = (ctypes.c_int64 * 2)()
    _check(_lib.grmhd_timing_read(ms, n))
    return {"stage": (ms[0], n[0]), "con2prim": (ms[1], n[1])}


def grmhd_con2prim_adjoint(dom, params, met, P, gP, gU, stream=None):
    _check(_lib.grmhd_con2prim_adjoint(ctypes.byref(dom.c), ctypes.byref(_par(params)), ctypes.byref(met.c), _ptr(P),
                                       _ptr(gP), _ptr(gU), _stream(stream)))


def grmhd_rk_step_adjoint(dom, params, met, stage_ckpt, P, dt, gU_out, gU_in, scheme=GRMHD_SSPRK3, ws=None,
                          stream=None):
    pc = _par(params)
    need = grmhd_workspace_bytes(dom, pc, scheme, 1)
    if ws is None:
        ws = torch.empty((need + 7) // 8, dtype=torch.float64, device=gU_out.device)
    _check(_lib.grmhd_rk_step_adjoint(ctypes.byref(dom.c), ctypes.byref(pc), ctypes.byref(met.c), _ptr(stage_ckpt),
                                      _ptr(P), float(dt), int(scheme), _ptr(gU_out), _ptr(gU_in),
                                      ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel() * ws.element_size()),
                                      _stream(stream)))
    return ws


# ------------------------------------------------------------------ constrained transport

def grmhd_ct_init(dom, params, met, A, U, P, stream=None):
    _check(_lib.grmhd_ct_init(ctypes.byref(dom.c), ctypes.byref(_par(params)), ctypes.byref(met.c), _ptr(A), _ptr(U),
                              _ptr(P), _stream(stream)))


def grmhd_ct_face_field(dom, A, Bface, stream=None):
    _check(_lib.grmhd_ct_face_field(ctypes.byref(dom.c), _ptr(A), _ptr(Bface), _stream(stream)))


def grmhd_ct_workspace_bytes(dom, params, scheme=GRMHD_SSPRK3):
    return int(_lib.grmhd_ct_workspace_bytes(ctypes.byref(dom.c), ctypes.byref(_par(params)), int(scheme)))


def grmhd_rk_step_ct(dom, params, met, U, P, A, dt, scheme=GRMHD_SSPRK3, max_rate=None, n_fail=None, ws=None,
                     stream=None):
    pc = _par(params)
    need = grmhd_ct_workspace_bytes(dom, pc, scheme)
    if ws is None:
        ws = torch.empty((need + 7) // 8, dtype=torch.float64, device=U.device)
    _check(_lib.grmhd_rk_step_ct(ctypes.byref(dom.c), ctypes.byref(pc), ctypes.byref(met.c), _ptr(U), _ptr(P), _ptr(A),
                                 float(dt), int(scheme), _ptr(max_rate), _ptr(n_fail, torch.int64),
                                 ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel() * ws.element_size()),
                                 _stream(stream)))
    return ws

