"""The C-ABI library loads and exports what include/grmhd.h declares (no GPU).

Only host-side paths run here: argument validation returns before any HIP
call, so no device is touched.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "grmhd.h")
LIB = os.path.join(ROOT, "paper_2210_17509_amd", "libgrmhd.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(grmhd_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2210_17509_amd.build import build_hip
        build_hip()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("grmhd_rhs", "grmhd_con2prim", "grmhd_rk_step", "grmhd_prim2con", "grmhd_domain_prepare",
              "grmhd_workspace_bytes", "grmhd_strerror"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_names_match_header():
    from paper_2210_17509_amd import grmhd
    assert sorted(grmhd.EXPORTED) == _declared()
    for n in grmhd.EXPORTED:
        assert callable(getattr(grmhd, n))


def test_strerror_and_sizes(lib):
    from paper_2210_17509_amd import grmhd as G
    assert G.grmhd_strerror(0) == "success"
    assert G.grmhd_strerror(-1) == "invalid argument"
    assert G.grmhd_strerror(-3) == "workspace too small"
    assert G.grmhd_domain_table_bytes(0) == 0
    assert G.grmhd_domain_table_bytes(400) > G.grmhd_domain_table_bytes(1) > 0


def _domain(G, n=(8, 8, 8), ng=3, bc=(0,) * 6, cell_stride=None, vert_stride=None, dx=0.1):
    box = (G.grmhd_box * 1)()
    b = box[0]
    for d in range(3):
        b.n[d] = n[d]
        b.dx[d] = dx
    b.ng = ng
    for q in range(6):
        b.bc[q] = bc[q]
    nc = (n[0] + 2 * ng) * (n[1] + 2 * ng) * (n[2] + 2 * ng)
    nv = (n[0] + 2 * ng + 1) * (n[1] + 2 * ng + 1) * (n[2] + 2 * ng + 1)
    d = G.grmhd_domain(ctypes.cast(box, ctypes.POINTER(G.grmhd_box)), 1, 0, cell_stride or nc, vert_stride or nv,
                       ctypes.c_void_p(0x1000))
    return d, box


@pytest.mark.parametrize("kw,why", [
    (dict(n=(0, 8, 8)), "n < 1"),
    (dict(ng=1), "ghost"),
    (dict(bc=(0, 1, 0, 0, 0, 0)), "periodic boundary on only one side"),
    (dict(bc=(7, 7, 0, 0, 0, 0)), "unknown boundary"),
    (dict(cell_stride=10), "outside the cell stride"),
    (dict(dx=-1.0), "dx"),
    # 812^3 storage cells and 813^3 vertices: element indices past 2^29 would
    # wrap the stage kernel's 32-bit byte offsets
    (dict(n=(806, 806, 806)), "2^29"),
    (dict(n=(2000, 2000, 130)), "2^29"),
])
def test_prepare_rejects_bad_boxes_without_touching_the_gpu(lib, kw, why):
    from paper_2210_17509_amd import grmhd as G
    d, keep = _domain(G, **kw)
    rc = lib.grmhd_domain_prepare(ctypes.byref(d), None)
    assert rc == G.GRMHD_EINVAL
    assert why in G.grmhd_last_error()


def test_entry_points_reject_unprepared_domain(lib):
    from paper_2210_17509_amd import grmhd as G
    d, keep = _domain(G)
    par = G.grmhd_params(1, 0, 1, 100, -1, 0, 0, 5 / 3, 1e-6, 1e-40, 1e-12, 1e-10, 100.0, 2.0)
    met = G.grmhd_metric(ctypes.c_void_p(0x2000), None, ctypes.c_void_p(0x3000))
    fake = ctypes.c_void_p(0x4000)
    assert lib.grmhd_rhs(ctypes.byref(d), ctypes.byref(par), ctypes.byref(met), fake, fake, fake, None, None,
                         None) == G.GRMHD_EINVAL
    assert "not prepared" in G.grmhd_last_error()
    assert lib.grmhd_con2prim(None, ctypes.byref(par), ctypes.byref(met), fake, fake, None, None, None) == G.GRMHD_EINVAL
    assert lib.grmhd_rk_step(ctypes.byref(d), ctypes.byref(par), ctypes.byref(met), fake, fake, ctypes.c_double(0.1),
                             0, None, None, None, fake, ctypes.c_size_t(1 << 30), None) == G.GRMHD_EINVAL


def test_workspace_size(lib):
    from paper_2210_17509_amd import grmhd as G
    d, keep = _domain(G)
    par = G.grmhd_params(1, 0, 1, 100, -1, 0, 0, 5 / 3, 1e-6, 1e-40, 1e-12, 1e-10, 100.0, 2.0)
    assert G._lib.grmhd_workspace_bytes(ctypes.byref(d), ctypes.byref(par), 0, 0) == 2 * 8 * 8 * d.cell_stride + 256
    assert G._lib.grmhd_workspace_bytes(ctypes.byref(d), ctypes.byref(par), 0, 1) == 2 * 8 * 8 * d.cell_stride
    # starting from the caller's primitives, SSPRK3 needs a second primitive buffer
    # classic RK4 (stages fused): stage state, accumulated step and two primitive buffers
    assert G._lib.grmhd_workspace_bytes(ctypes.byref(d), ctypes.byref(par), 2, 0) == 4 * 8 * 8 * d.cell_stride + 256
    par.p_current = 1
    assert G._lib.grmhd_workspace_bytes(ctypes.byref(d), ctypes.byref(par), 0, 0) == 3 * 8 * 8 * d.cell_stride + 256
    assert G._lib.grmhd_workspace_bytes(ctypes.byref(d), ctypes.byref(par), 1, 0) == 2 * 8 * 8 * d.cell_stride + 256
    assert G._lib.grmhd_workspace_bytes(ctypes.byref(d), ctypes.byref(par), 0, 1) == 2 * 8 * 8 * d.cell_stride
