"""Seeded synthetic inputs for the GRMHD hot path.

This module only draws and lays out input data: primitive fields at cell
centres and an ADM metric (lapse, optional shift, spatial metric) sampled at
cell vertices.  It holds none of the method's arithmetic (no prim->cons map,
no reconstruction, no Riemann solver), so both the HIP path and the CPU oracle
can take their inputs from here without sharing any numerics.

Storage layout (shared by every consumer):
  * a problem is a list of boxes; a single grid is one box;
  * cell fields are pooled: field f of box b, storage cell (i, j, k) with
    ghost layers included, sits at f * cell_stride + cell_off[b]
    + (k * NYg + j) * NXg + i, NXg = nx + 2 ng (x fastest);
  * vertex fields use the same rule with (n + 2 ng + 1) points per axis, the
    vertex with storage index I lying at x0 + (I - ng) dx;
  * the primitive vector is [rho, v^x, v^y, v^z, eps, B^x, B^y, B^z]
    (Sec. II C of the paper), v^i the contravariant Valencia velocity.

Boundary codes: 0 = periodic, 1 = outflow (copy of the nearest interior cell).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

BC_PERIODIC = 0
BC_OUTFLOW = 1

RECON_MINMOD = 0
RECON_WENO5 = 1
RECON_WENOZ = 2

PREC_FP64 = 0
PREC_MIXED = 1

NPRIM = 8
SEED_BASE = 17509


@dataclass
class BoxSpec:
    n: Tuple[int, int, int]
    ng: int
    bc: Tuple[int, int, int, int, int, int]  # xlo xhi ylo yhi zlo zhi
    x0: Tuple[float, float, float]            # coordinate of the interior's lower corner
    dx: Tuple[float, float, float]

    @property
    def cdims(self):
        """Storage cell counts (x, y, z) including ghosts."""
        return tuple(int(v) + 2 * self.ng for v in self.n)

    @property
    def vdims(self):
        return tuple(int(v) + 2 * self.ng + 1 for v in self.n)

    @property
    def ncell(self):
        a, b, c = self.cdims
        return a * b * c

    @property
    def nvert(self):
        a, b, c = self.vdims
        return a * b * c

    @property
    def ninterior(self):
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])


@dataclass
class Params:
    recon: int = RECON_WENO5
    precision: int = PREC_FP64
    eos_gamma: float = 5.0 / 3.0
    weno_eps: float = 1e-6
    wenoz_eps: float = 1e-40
    wenoz_p: int = 1
    c2p_tol: float = 1e-12
    c2p_maxit: int = 100
    rho_atm: float = 1e-10
    atm_K: float = 100.0
    atm_gamma: float = 2.0


@dataclass
class Problem:
    name: str
    boxes: List[BoxSpec]
    params: Params
    P: np.ndarray                 # (8, cell_stride) float64
    alpha: np.ndarray             # (vert_stride,)
    beta: Optional[np.ndarray]    # (3, vert_stride) or None (zero shift)
    gamma: np.ndarray             # (6, vert_stride): xx xy xz yy yz zz
    cell_off: List[int] = field(default_factory=list)
    vert_off: List[int] = field(default_factory=list)
    dt: float = 0.0
    steps: int = 1
    seed: int = 0

    @property
    def cell_stride(self):
        return self.P.shape[1]

    @property
    def vert_stride(self):
        return self.alpha.shape[0]

    @property
    def ninterior(self):
        return sum(b.ninterior for b in self.boxes)

    def box_view(self, arr, b, vertex=False):
        """Reshape the pooled storage of box b to (..., NZ, NY, NX)."""
        bx = self.boxes[b]
        if vertex:
            nx, ny, nz = bx.vdims
            off = self.vert_off[b]
            cnt = bx.nvert
        else:
            nx, ny, nz = bx.cdims
            off = self.cell_off[b]
            cnt = bx.ncell
        lead = arr.shape[:-1]
        return arr[..., off:off + cnt].reshape(lead + (nz, ny, nx))


def _pool(boxes):
    cell_off, vert_off = [], []
    c = v = 0
    for b in boxes:
        cell_off.append(c)
        vert_off.append(v)
        c += b.ncell
        v += b.nvert
    return cell_off, vert_off, c, v


def cell_centres(box: BoxSpec):
    """Coordinates (X, Y, Z), each shaped (NZ, NY, NX), of all storage cells."""
    ax = []
    for d in range(3):
        i = np.arange(box.cdims[d], dtype=np.float64)
        ax.append(box.x0[d] + (i - box.ng + 0.5) * box.dx[d])
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return X, Y, Z


def vertex_coords(box: BoxSpec):
    ax = []
    for d in range(3):
        i = np.arange(box.vdims[d], dtype=np.float64)
        ax.append(box.x0[d] + (i - box.ng) * box.dx[d])
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return X, Y, Z


# --------------------------------------------------------------------------
# field recipes
# --------------------------------------------------------------------------

def _fourier_field(rng, X, Y, Z, nmodes=6, kmax=4):
    """Smooth random field in [-1, 1]: sum_m a_m sin(2 pi k_m.x + phi_m) / sum a_m."""
    ks = []
    while len(ks) < nmodes:
        k = rng.integers(-kmax, kmax + 1, size=3)
        if np.any(k != 0):
            ks.append(k)
    a = rng.uniform(0.0, 1.0, size=nmodes)
    phi = rng.uniform(0.0, 2.0 * np.pi, size=nmodes)
    g = np.zeros_like(X)
    for m in range(nmodes):
        kx, ky, kz = (float(v) for v in ks[m])
        g += a[m] * np.sin(2.0 * np.pi * (kx * X + ky * Y + kz * Z) + phi[m])
    return g / a.sum()


# ranges of the smooth flat-space recipe: rho, p, v^x, v^y, v^z, B^x, B^y, B^z
_FLAT_RANGES = [(0.1, 1.0), (0.1, 1.0), (-0.5, 0.5), (-0.5, 0.5), (-0.5, 0.5),
                (-1.0, 1.0), (-1.0, 1.0), (-1.0, 1.0)]


# milder ranges (moderate flow speeds and magnetisation, pressure-dominated) for
# the flat boxes of the batched workload, which must evolve for many steps
_FLAT_RANGES_MILD = [(0.5, 1.0), (0.5, 1.0), (-0.3, 0.3), (-0.3, 0.3), (-0.3, 0.3),
                     (-0.3, 0.3), (-0.3, 0.3), (-0.3, 0.3)]


def _smooth_draw(rng, X, Y, Z, ranges=_FLAT_RANGES):
    out = []
    for lo, hi in ranges:
        g = _fourier_field(rng, X, Y, Z)
        out.append(lo + (hi - lo) * 0.5 * (1.0 + g))
    return out


def flat_fields(rng, X, Y, Z, gam, jump_at=None, mild=False):
    """Smooth random primitives (optionally with a planar jump at x = jump_at;
    mild: the milder value ranges).

    Returns the 8 primitive arrays; eps = p / ((Gamma - 1) rho)."""
    ranges = _FLAT_RANGES_MILD if mild else _FLAT_RANGES
    q = _smooth_draw(rng, X, Y, Z, ranges)
    if jump_at is not None:
        q2 = _smooth_draw(rng, X, Y, Z, ranges)
        right = X >= jump_at
        q = [np.where(right, b, a) for a, b in zip(q, q2)]
    rho, p, vx, vy, vz, bx, by, bz = q
    eps = p / ((gam - 1.0) * rho)
    return [rho, vx, vy, vz, eps, bx, by, bz]


def curved_fields(rng, X, Y, Z, gam):
    """Polytrope-like ball: rho = max(1e-3, 1 - r^2/4) (1 + 0.01 u), p = 100 rho^2,
    v = 0, weak random B."""
    r2 = X * X + Y * Y + Z * Z
    u = rng.uniform(-1.0, 1.0, size=X.shape)
    rho = np.maximum(1e-3, 1.0 - 0.25 * r2) * (1.0 + 0.01 * u)
    p = 100.0 * rho * rho
    eps = p / ((gam - 1.0) * rho)
    z = np.zeros_like(X)
    b = rng.uniform(-0.01, 0.01, size=(3,) + X.shape)
    return [rho, z, z.copy(), z.copy(), eps, b[0], b[1], b[2]]


def flat_metric(box: BoxSpec):
    nx, ny, nz = box.vdims
    alpha = np.ones((nz, ny, nx))
    gamma = np.zeros((6, nz, ny, nx))
    gamma[0] = gamma[3] = gamma[5] = 1.0
    return alpha, None, gamma


def curved_metric(box: BoxSpec, mass=1.0, rmin=0.2):
    """Conformally flat static metric regularised inside r = rmin:
    psi = 1 + M / (2 max(r, rmin)), gamma_ij = psi^4 delta_ij, alpha = psi^-2, beta = 0."""
    X, Y, Z = vertex_coords(box)
    r = np.sqrt(X * X + Y * Y + Z * Z)
    psi = 1.0 + mass / (2.0 * np.maximum(r, rmin))
    alpha = psi ** -2
    gamma = np.zeros((6,) + X.shape)
    gamma[0] = gamma[3] = gamma[5] = psi ** 4
    return alpha, None, gamma


def _assemble(name, boxes, params, fields_per_box, metric_per_box, dt, steps, seed):
    cell_off, vert_off, nc, nv = _pool(boxes)
    P = np.zeros((NPRIM, nc))
    alpha = np.zeros(nv)
    gamma = np.zeros((6, nv))
    any_beta = any(m[1] is not None for m in metric_per_box)
    beta = np.zeros((3, nv)) if any_beta else None
    for b, bx in enumerate(boxes):
        c0, v0 = cell_off[b], vert_off[b]
        for f in range(NPRIM):
            P[f, c0:c0 + bx.ncell] = fields_per_box[b][f].ravel()
        a, be, g = metric_per_box[b]
        alpha[v0:v0 + bx.nvert] = a.ravel()
        gamma[:, v0:v0 + bx.nvert] = g.reshape(6, -1)
        if beta is not None and be is not None:
            beta[:, v0:v0 + bx.nvert] = be.reshape(3, -1)
    return Problem(name=name, boxes=boxes, params=params, P=P, alpha=alpha, beta=beta,
                   gamma=gamma, cell_off=cell_off, vert_off=vert_off, dt=dt, steps=steps,
                   seed=seed)


# --------------------------------------------------------------------------
# the five workloads (sizes are parameters so tests can shrink them)
# --------------------------------------------------------------------------

def config0(n=64, seed=SEED_BASE + 0, jump=True, recon=RECON_MINMOD, steps=1, ng=3):
    """Flat space, Gamma = 5/3, smooth random fields plus a planar jump at x = 0.5,
    outflow in x, periodic in y and z, minmod + HLLE, one SSPRK3 step, dt = dx/4."""
    rng = np.random.default_rng(seed)
    gam = 5.0 / 3.0
    dx = 1.0 / n
    box = BoxSpec((n, n, n), ng, (BC_OUTFLOW, BC_OUTFLOW, BC_PERIODIC, BC_PERIODIC,
                                  BC_PERIODIC, BC_PERIODIC), (0.0, 0.0, 0.0), (dx, dx, dx))
    X, Y, Z = cell_centres(box)
    f = flat_fields(rng, X, Y, Z, gam, jump_at=0.5 if jump else None)
    par = Params(recon=recon, eos_gamma=gam)
    return _assemble("config0", [box], par, [f], [flat_metric(box)], 0.25 * dx, steps, seed)


def config1(n=256, seed=SEED_BASE + 1, recon=RECON_WENO5, steps=1, extent=4.0, ng=3,
            precision=PREC_FP64, bc=BC_OUTFLOW):
    """Static curved metric on [-extent, extent]^3, Gamma = 2, polytrope-like ball,
    outflow everywhere (or bc on every face), WENO5 + HLLE, atmosphere 1e-10,
    dt = dx/4."""
    rng = np.random.default_rng(seed)
    gam = 2.0
    dx = 2.0 * extent / n
    box = BoxSpec((n, n, n), ng, (bc,) * 6, (-extent,) * 3, (dx, dx, dx))
    X, Y, Z = cell_centres(box)
    f = curved_fields(rng, X, Y, Z, gam)
    par = Params(recon=recon, eos_gamma=gam, precision=precision)
    return _assemble("config1", [box], par, [f], [curved_metric(box)], 0.25 * dx, steps, seed)


def config2(nbox=400, seed=SEED_BASE + 2, edges=(16, 24, 32, 48, 64), ng=3,
            recon=RECON_WENO5, steps=1):
    """Batch of uneven boxes (edges drawn per axis), outflow on every box face, each
    box flat (smooth recipe with the milder ranges, dx = 1/64, inside [0,1]^3) or
    curved (ball recipe, dx = 1/32, inside [-4,4]^3) by a coin flip; one Gamma = 2
    for the whole batch."""
    rng = np.random.default_rng(seed)
    gam = 2.0
    boxes, fields, metrics = [], [], []
    kinds = []
    for _ in range(nbox):
        n = tuple(int(v) for v in rng.choice(edges, size=3))
        curved = bool(rng.integers(0, 2))
        if curved:
            dx = 1.0 / 32.0
            lo, hi = -4.0, 4.0
        else:
            dx = 1.0 / 64.0
            lo, hi = 0.0, 1.0
        x0 = tuple(float(rng.uniform(lo, hi - n[d] * dx)) if hi - n[d] * dx > lo else lo
                   for d in range(3))
        bx = BoxSpec(n, ng, (BC_OUTFLOW,) * 6, x0, (dx, dx, dx))
        X, Y, Z = cell_centres(bx)
        if curved:
            fields.append(curved_fields(rng, X, Y, Z, gam))
            metrics.append(curved_metric(bx))
        else:
            fields.append(flat_fields(rng, X, Y, Z, gam, mild=True))
            metrics.append(flat_metric(bx))
        boxes.append(bx)
        kinds.append(curved)
    par = Params(recon=recon, eos_gamma=gam)
    prob = _assemble("config2", boxes, par, fields, metrics, 0.25 / 64.0, steps, seed)
    prob.kinds = kinds
    return prob


def config3(n=384, seed=SEED_BASE + 3, steps=50, precision=PREC_MIXED):
    """The curved recipe at 384^3 (dx = 1/48), run in mixed precision."""
    p = config1(n=n, seed=seed, steps=steps, precision=precision)
    p.name = "config3"
    return p


def config4(n=128, seed=SEED_BASE + 4, steps=10):
    """Flat smooth recipe without the jump, WENO5-Z, 10 steps (adjoint workload)."""
    p = config0(n=n, seed=seed, jump=False, recon=RECON_WENOZ, steps=steps)
    p.name = "config4"
    return p


def adjoint_weight(prob: Problem, seed, width=0.1):
    """Seeded Gaussian weight w(x) = exp(-|x - c|^2 / (2 width^2)) on interior cells of
    box 0, c ~ U[0.3, 0.7]^3; zero on ghost cells."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.3, 0.7, size=3)
    bx = prob.boxes[0]
    X, Y, Z = cell_centres(bx)
    w = np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) / (2.0 * width ** 2))
    g = bx.ng
    mask = np.zeros_like(w)
    mask[g:g + bx.n[2], g:g + bx.n[1], g:g + bx.n[0]] = 1.0
    return w * mask


def interior_mask(box: BoxSpec):
    nx, ny, nz = box.cdims
    m = np.zeros((nz, ny, nx), dtype=bool)
    g = box.ng
    m[g:g + box.n[2], g:g + box.n[1], g:g + box.n[0]] = True
    return m


# --------------------------------------------------------------------------
# constrained transport (Sec. III B): the vector potential on cell edges
# --------------------------------------------------------------------------
#
# A is (3, vert_stride): A_e of an edge along e is stored like a vertex field
# with the cell index along e in place of that vertex index; its position has
# the cell-centre coordinate along e and vertex coordinates along the others.

def edge_coords(box: BoxSpec, e):
    """Coordinates (X, Y, Z), each shaped like the box's vertex grid, of the edges along e."""
    ax = []
    for d in range(3):
        i = np.arange(box.vdims[d], dtype=np.float64)
        ax.append(box.x0[d] + (i - box.ng + (0.5 if d == e else 0.0)) * box.dx[d])
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return X, Y, Z


def uniform_potential(box: BoxSpec, B):
    """A = (B^y z, B^z x, B^x y) on the edges: curl A = (B^x, B^y, B^z) everywhere."""
    Xx, Yx, Zx = edge_coords(box, 0)
    Xy, Yy, Zy = edge_coords(box, 1)
    Xz, Yz, Zz = edge_coords(box, 2)
    return np.stack([B[1] * Zx, B[2] * Xy, B[0] * Yz])


def _pool_edges(prob, per_box):
    A = np.zeros((3, prob.vert_stride))
    for b, bx in enumerate(prob.boxes):
        v0 = prob.vert_off[b]
        A[:, v0:v0 + bx.nvert] = per_box[b].reshape(3, -1)
    return A


def ct_random(n=(12, 10, 8), seed=SEED_BASE + 31, recon=RECON_WENO5, bc=BC_PERIODIC, curved=False, amp=0.05):
    """Smooth random flat-space primitives (mild ranges, Gamma = 5/3) on the unit cube
    with a smooth random potential: A_e = amp / (2 pi) * (Fourier field, wavenumbers up
    to 4) plus the potential of a uniform field (0.3, -0.2, 0.25).  The primitives' B is replaced by
    curl A / sqrt(gamma) through the oracle's or the library's CT initialisation.
    curved: the conformally flat metric of the curved recipe around (0.5, 0.5, 0.5)."""
    rng = np.random.default_rng(seed)
    gam = 5.0 / 3.0
    dx = tuple(1.0 / v for v in n)
    box = BoxSpec(tuple(n), 3, (bc,) * 6, (0.0, 0.0, 0.0), dx)
    X, Y, Z = cell_centres(box)
    f = flat_fields(rng, X, Y, Z, gam, mild=True)
    if curved:
        shifted = BoxSpec(box.n, box.ng, box.bc, (-0.5 - 2.0, -0.5, -0.5), dx)
        met = curved_metric(shifted)
    else:
        met = flat_metric(box)
    par = Params(recon=recon, eos_gamma=gam)
    prob = _assemble("ct_random", [box], par, [f], [met], 0.25 * min(dx), 1, seed)
    A = uniform_potential(box, (0.3, -0.2, 0.25))
    for e in range(3):
        A[e] += amp / (2.0 * np.pi) * _fourier_field(rng, *edge_coords(box, e))
    prob.A = _pool_edges(prob, [A])
    return prob


def rotor(n=400, nz=1, seed=SEED_BASE + 40):
    """The relativistic magnetic rotor (Sec. IV C): [-0.5, 0.5]^2, a cylinder of radius
    0.1 with rho = 10 rotating at Omega = 9.95 (v_max = 0.995) in rho = 1, p = 1 everywhere,
    B = (1, 0, 0); Gamma = 5/3, minmod, HLLE, copy boundaries in x and y (periodic along
    the cylinder axis, n_z cells), flat metric, dt = dx / 4 (CFL 0.25)."""
    gam = 5.0 / 3.0
    dx = 1.0 / n
    box = BoxSpec((n, n, nz), 3, (BC_OUTFLOW,) * 4 + (BC_PERIODIC,) * 2, (-0.5, -0.5, -0.5 * nz * dx),
                  (dx, dx, dx))
    X, Y, Z = cell_centres(box)
    r = np.sqrt(X * X + Y * Y)
    inside = r < 0.1
    omega = 9.95
    rho = np.where(inside, 10.0, 1.0)
    p = np.ones_like(X)
    vx = np.where(inside, -omega * Y, 0.0)
    vy = np.where(inside, omega * X, 0.0)
    z = np.zeros_like(X)
    eps = p / ((gam - 1.0) * rho)
    f = [rho, vx, vy, z, eps, z.copy(), z.copy(), z.copy()]
    par = Params(recon=RECON_MINMOD, eos_gamma=gam)
    prob = _assemble("rotor", [box], par, [f], [flat_metric(box)], 0.25 * dx, 1, seed)
    prob.A = _pool_edges(prob, [uniform_potential(box, (1.0, 0.0, 0.0))])
    return prob


def cylindrical_explosion(n=200, nz=1, seed=SEED_BASE + 41):
    """The cylindrical explosion (Sec. IV B): [-6, 6]^2, rho and p equal to their inner
    values for r <= 0.8 and their outer values for r >= 1, with log-linear profiles in
    between (R29); rho 1e-2 / 1e-4, p 1 / 3e-5, v = 0, B = (0.1, 0, 0), Gamma = 4/3,
    minmod, HLLE, copy boundaries, flat metric, dt = dx / 4."""
    gam = 4.0 / 3.0
    dx = 12.0 / n
    box = BoxSpec((n, n, nz), 3, (BC_OUTFLOW,) * 4 + (BC_PERIODIC,) * 2, (-6.0, -6.0, -0.5 * nz * dx),
                  (dx, dx, dx))
    X, Y, Z = cell_centres(box)
    r = np.sqrt(X * X + Y * Y)
    r_in, r_out = 0.8, 1.0

    def profile(q_in, q_out):
        t = np.clip((r - r_in) / (r_out - r_in), 0.0, 1.0)
        return np.exp((1.0 - t) * np.log(q_in) + t * np.log(q_out))

    rho = profile(1e-2, 1e-4)
    p = profile(1.0, 3e-5)
    z = np.zeros_like(X)
    eps = p / ((gam - 1.0) * rho)
    f = [rho, z, z.copy(), z.copy(), eps, z.copy(), z.copy(), z.copy()]
    par = Params(recon=RECON_MINMOD, eos_gamma=gam)
    prob = _assemble("explosion", [box], par, [f], [flat_metric(box)], 0.25 * dx, 1, seed)
    prob.A = _pool_edges(prob, [uniform_potential(box, (0.1, 0.0, 0.0))])
    return prob


def field_loop(n=32, seed=SEED_BASE + 42, A0=1e-3, R=0.3, v=(0.5, 0.25)):
    """Field-loop advection on the periodic unit square (flat space, Gamma = 5/3, rho = 1,
    p = 1, uniform v, weak loop A_z = A0 (R - r) for r < R around (0.5, 0.5)): an exact
    solution that translates with v, minmod + HLLE, dt = dx / 4."""
    gam = 5.0 / 3.0
    dx = 1.0 / n
    box = BoxSpec((n, n, 1), 3, (BC_PERIODIC,) * 6, (0.0, 0.0, -0.5 * dx), (dx, dx, dx))
    X, Y, Z = cell_centres(box)
    one = np.ones_like(X)
    z = np.zeros_like(X)
    f = [one, v[0] * one, v[1] * one, z, one / (gam - 1.0), z.copy(), z.copy(), z.copy()]
    par = Params(recon=RECON_MINMOD, eos_gamma=gam)
    prob = _assemble("field_loop", [box], par, [f], [flat_metric(box)], 0.25 * dx, 1, seed)
    prob.A = _pool_edges(prob, [field_loop_potential(box, 0.0, A0, R, v)])
    return prob


def field_loop_potential(box: BoxSpec, t, A0=1e-3, R=0.3, v=(0.5, 0.25)):
    """The loop's potential translated by v t (periodic images on the unit square)."""
    A = np.zeros((3,) + tuple(reversed(box.vdims)))
    X, Y, _ = edge_coords(box, 2)
    dxp = (X - 0.5 - v[0] * t + 0.5) % 1.0 - 0.5
    dyp = (Y - 0.5 - v[1] * t + 0.5) % 1.0 - 0.5
    r = np.sqrt(dxp * dxp + dyp * dyp)
    A[2] = np.where(r < R, A0 * (R - r), 0.0)
    return A

