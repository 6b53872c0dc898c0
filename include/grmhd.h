/*
 * grmhd.h -- C ABI of the MI355X (gfx950) GRMHD hot path.
 *
 * The library evaluates the Valencia-formulation right-hand side of ideal
 * GRMHD on a static 3+1 metric (GRaM-X, arXiv:2210.17509, Sec. II B-C):
 * con2prim, reconstruction of the primitives P = [rho, v^i, eps, B^i] on cell
 * faces (TVD-minmod, WENO5, WENO5-Z), the HLLE flux, the flux divergence plus
 * the metric source terms, and SSPRK time steps of the method of lines.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Pointers are DEVICE pointers unless marked (host).  Every call validates its
 * arguments on the host, enqueues its kernels on `stream` (a hipStream_t,
 * NULL = the null stream) and returns without synchronizing.  The library
 * keeps no pointer after a call returns and allocates no device memory in
 * these calls; scratch memory comes from the caller's workspace `ws` (or, for
 * grmhd_rk_step_noalloc, from a fixed array the library holds per device).
 *
 * Grid.  A problem is a list of boxes (a single grid is one box).  Each box
 * has n[d] interior cells per axis and ng >= 3 ghost layers (ng >= 2 is
 * enough for minmod).  Cell fields are pooled:
 *   field f of box b, storage cell (i, j, k), i fastest, ghosts included, at
 *   f * cell_stride + cell_off[b] + (k * NYg + j) * NXg + i,  NXg = n[0] + 2 ng.
 * Vertex fields (the metric) use the same rule with n[d] + 2 ng + 1 points
 * per axis; vertex storage index I sits at x0[d] + (I - ng) dx[d].  Fluid data
 * are cell averages, the spacetime lives on vertices (Sec. III).
 *   P fields: rho, v^x, v^y, v^z (contravariant Valencia velocity, Eq. (vel)),
 *             eps, B^x, B^y, B^z.
 *   U fields: D, S_x, S_y, S_z, tau, Bcal^x, Bcal^y, Bcal^z (Eqs. (p2c1)-(p2c4)).
 * Only interior cells are read from U and written to U, P and dU/dt; ghost
 * primitives are never stored: boundary conditions (periodic wrap, or outflow
 * = copy of the nearest interior cell, Sec. IV A) are applied by index
 * mapping when faces read their stencils.
 *
 * Errors.  0 on success, or a negative code:
 *   GRMHD_EINVAL     bad argument (null pointer, size, ghost count, Gamma <= 1,
 *                    dt <= 0, non-finite parameter, domain not prepared or
 *                    changed since grmhd_domain_prepare); nothing enqueued.
 *   GRMHD_EHIP       a HIP launch or runtime call failed; grmhd_strerror(code)
 *                    and grmhd_last_error() describe it.
 *   GRMHD_EWORKSPACE ws_bytes smaller than grmhd_workspace_bytes().
 * A con2prim failure is not an error return: the cell is reset to the
 * atmosphere, its status code records why, and *n_fail is incremented.
 */
#ifndef GRMHD_H
#define GRMHD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GRMHD_OK 0
#define GRMHD_EINVAL (-1)
#define GRMHD_EHIP (-2)
#define GRMHD_EWORKSPACE (-3)

enum { GRMHD_BC_PERIODIC = 0, GRMHD_BC_OUTFLOW = 1 };
enum { GRMHD_RECON_MINMOD = 0, GRMHD_RECON_WENO5 = 1, GRMHD_RECON_WENOZ = 2 };
/* GRMHD_MIXED: reconstruction and HLLE in FP32; con2prim, sources, the flux
 * divergence accumulation, the time update and the atmosphere stay FP64. */
enum { GRMHD_FP64 = 0, GRMHD_MIXED = 1 };
/* SSPRK3 (Shu-Osher) and SSPRK2 (Heun, the method of lines' RK2), written
 * U_{s+1} = U^n + c_s ((U_s - U^n) + dt L(U_s)); classic RK4 with stage states
 * U^n + a_s dt L(U_s), a = (1/2, 1/2, 1), and U^{n+1} = U^n + dt (L_0 + 2 L_1 + 2 L_2
 * + L_3) / 6 (the paper's RK4; no stage checkpoints, no adjoint). */
enum { GRMHD_SSPRK3 = 0, GRMHD_SSPRK2 = 1, GRMHD_RK4 = 2 };
/* Stage-kernel tiles (cells per 256-thread workgroup): 0 = 16x4x4, 1 = 8x8x4, 2 = 64x2x2,
 * 3 = 16x4x3 (192 cells: the faces of each direction fit one pass of the workgroup). */
#define GRMHD_NTILE 4
/* Stage-kernel scheduling in grmhd_rk_step: one workgroup per tile, or persistent
 * workgroups popping tiles from per-XCD atomic queues kept in the workspace. */
enum { GRMHD_SCHED_GRID = 0, GRMHD_SCHED_QUEUE = 1 };
/* per-cell con2prim status */
enum {
  GRMHD_C2P_OK = 0,        /* 3D Newton-Raphson converged */
  GRMHD_C2P_FLOOR = 1,     /* density below rho_atm (1 + 1e-6): atmosphere applied */
  GRMHD_C2P_NOCONV = 2,    /* no method converged: atmosphere applied */
  GRMHD_C2P_UNPHYS = 3,    /* only unphysical roots found: atmosphere applied */
  GRMHD_C2P_NONFINITE = 4, /* non-finite conserved input: atmosphere applied */
  GRMHD_C2P_FALLBACK = 5   /* recovered by the Newman-Hamlin fallback */
};

/* (host) One box of the pooled grid. */
typedef struct {
  int32_t n[3];      /* interior cells per axis, >= 1; a box holds fewer than 2^29
                      * cells and vertices, ghosts included (at most 805^3 interior
                      * cells with ng = 3): larger grids are split into boxes */
  int32_t ng;        /* ghost layers */
  int32_t bc[6];     /* x-lo, x-hi, y-lo, y-hi, z-lo, z-hi: GRMHD_BC_* */
  double x0[3];      /* coordinates of the interior's lower corner (a vertex) */
  double dx[3];      /* cell spacing */
  int64_t cell_off;  /* element offset of this box in the pooled cell arrays */
  int64_t vert_off;  /* element offset in the pooled vertex arrays */
} grmhd_box;

/* A prepared domain: the host box list plus a device copy of the derived
 * per-box launch tables, written by grmhd_domain_prepare into caller-owned
 * device memory `table` of grmhd_domain_table_bytes(nbox) bytes. */
typedef struct {
  const grmhd_box* box;  /* (host) nbox boxes */
  int32_t nbox;
  int32_t pad;
  int64_t cell_stride;   /* elements between consecutive fields of P, U, dU/dt */
  int64_t vert_stride;   /* elements between consecutive metric fields */
  void* table;           /* device memory holding the launch tables */
} grmhd_domain;

/* (host) Physics and method parameters. */
typedef struct {
  int32_t recon;      /* GRMHD_RECON_* */
  int32_t precision;  /* GRMHD_FP64 | GRMHD_MIXED */
  int32_t wenoz_p;    /* WENO-Z exponent: 1 or 2 */
  int32_t c2p_maxit;  /* iteration cap of each con2prim method, e.g. 100 */
  int32_t tile;       /* stage-kernel tile shape: -1 = library choice (16x4x3), else 0 .. GRMHD_NTILE-1 */
  int32_t schedule;   /* GRMHD_SCHED_GRID | GRMHD_SCHED_QUEUE (grmhd_rk_step only) */
  int32_t p_current;  /* grmhd_rk_step only: 0 = start with con2prim(U^n); 1 = P already holds the
                       * primitives of U^n (as the previous grmhd_rk_step, grmhd_con2prim or the
                       * P given to grmhd_prim2con leave it), so that con2prim is skipped */
  double eos_gamma;   /* Gamma-law EOS p = (Gamma - 1) rho eps, Gamma > 1 */
  double weno_eps;    /* WENO5-JS epsilon, e.g. 1e-6 */
  double wenoz_eps;   /* WENO5-Z epsilon, e.g. 1e-40 */
  double c2p_tol;     /* relative Newton step tolerance, e.g. 1e-12 */
  double rho_atm;     /* atmosphere density, e.g. 1e-10 */
  double atm_K;       /* atmosphere polytrope p = K rho^atm_gamma, e.g. 100 */
  double atm_gamma;   /* e.g. 2 */
} grmhd_params;

/* Vertex-centred ADM metric of a static spacetime (Sec. II A): lapse alpha
 * (1 field), shift beta^i (3 fields, or NULL for zero shift), spatial metric
 * gamma_ij (6 fields: xx xy xz yy yz zz), each field vert_stride apart. */
typedef struct {
  const double* alpha;
  const double* beta;
  const double* gamma;
} grmhd_metric;

/* Bytes of device memory grmhd_domain_prepare needs for nbox boxes. */
size_t grmhd_domain_table_bytes(int32_t nbox);

/* Validate the boxes and write the derived launch tables to dom->table
 * (an asynchronous host-to-device copy on `stream`; the host boxes may be
 * reused once the call returns).  Every other entry point checks that the
 * host boxes still match what was prepared into dom->table. */
int grmhd_domain_prepare(const grmhd_domain* dom, void* stream);

/* Conserved from primitive variables on interior cells, Eqs. (p2c1)-(p2c4)
 * with Eq. (vel) and the Gamma-law EOS (Sec. II C, initialization step 2).
 * The spatial metric is averaged from the cell's 8 vertices. */
int grmhd_prim2con(const grmhd_domain* dom, const grmhd_params* par, const grmhd_metric* met,
                   const double* P, double* U, void* stream);

/* Primitive from conserved variables on interior cells (Sec. II C, RHS step 1):
 * a 3D Newton-Raphson in (W, z = rho h W^2, T = p / rho) seeded with the
 * primitives already in P, falling back to the Newman-Hamlin pressure
 * iteration (then a Newton polish) when it fails.  P is the guess on input
 * and the result on output.  Cells that cannot be recovered, or whose density
 * (D / sqrt(gamma) before, rho after a recovery) is below rho_atm (1 + 1e-6),
 * are reset to the atmosphere (rho_atm, v = 0, p = atm_K rho_atm^atm_gamma,
 * B kept) and U is rewritten there; a cell already at the atmosphere thus
 * stays there with status FLOOR.
 * status: per storage cell int32 GRMHD_C2P_* (interior cells written), or NULL.
 * n_fail: device int64 incremented by the count of statuses 2-4, or NULL. */
int grmhd_con2prim(const grmhd_domain* dom, const grmhd_params* par, const grmhd_metric* met,
                   double* U, double* P, int32_t* status, int64_t* n_fail, void* stream);

/* dU/dt on interior cells (Sec. II C, the four RHS steps; Eqs.
 * (definition-of-flux), (definition-of-source)): con2prim (U, P updated in
 * place as above), reconstruction with the metric interpolated linearly from
 * vertices to face centres, HLLE, and -sum_d (F_{+1/2} - F_{-1/2}) / dx_d + S.
 * max_rate: device double, raised (atomic max) to max over faces of
 * max(xi+, -xi-) / dx_d, or NULL.  The caller initialises it. */
int grmhd_rhs(const grmhd_domain* dom, const grmhd_params* par, const grmhd_metric* met,
              double* U, double* P, double* dUdt, double* max_rate, int64_t* n_fail, void* stream);

/* One SSPRK step of the method of lines (Sec. II C) with fixed dt:
 * con2prim(U^n) (skipped when par->p_current = 1: P then already holds the
 * primitives of U^n), then per stage s: U_{s+1} = U^n + c_s ((U_s - U^n) +
 * dt L(U_s)) with con2prim of each new stage state, ending with P consistent
 * with U^{n+1}; a sequence of steps thus recovers the primitives once per
 * stage.  U, P are updated in place.  stage_ckpt (SSPRK schemes; NULL for RK4): NULL, or device memory for
 * nstage * 8 * cell_stride doubles receiving the primitives of U^n and of the
 * stage states (as con2prim recovered them) for the adjoint.  max_rate /
 * n_fail as above, accumulated over all stages.  The con2prim of each stage
 * state runs inside the stage kernel; the primitives rotate between P and
 * copies in the workspace and end in P.  ws: grmhd_workspace_bytes() bytes
 * (two 8-field sets, three for SSPRK3 with p_current = 1, four for RK4: its
 * stage state, accumulator and two primitive buffers; then 256 bytes of
 * tile-queue counters).  RK4 stages are fused the same way: each stage
 * kernel accumulates the step, forms the next stage state and recovers its
 * primitives. */
int grmhd_rk_step(const grmhd_domain* dom, const grmhd_params* par, const grmhd_metric* met,
                  double* U, double* P, double dt, int32_t scheme, double* stage_ckpt,
                  double* max_rate, int64_t* n_fail, void* ws, size_t ws_bytes, void* stream);

/* grmhd_rk_step for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same step, bit for bit, with the workspace taken from a fixed array
 * that the library holds on every device it runs on, for the life of the
 * process, instead of the caller's ws.  The call itself allocates nothing.
 * Limit: grmhd_workspace_bytes(dom, par, scheme, 0) must not exceed
 * GRMHD_NOALLOC_SCRATCH_BYTES (256 MiB: about 2.09 M cells with ghosts for
 * SSPRK2/3 without p_current, 1.39 M for SSPRK3 with p_current = 1, 1.05 M
 * for RK4, e.g. a 121^3, 105^3 or 95^3 box with 3 ghost layers); larger
 * domains get GRMHD_EWORKSPACE and
 * nothing is enqueued.  All calls on one device share that device's array and
 * leave it dirty; the step writes every scratch value before reading it.
 * Calls that overlap on one device (concurrent streams or threads) race on the
 * array and must be serialized by the caller.  The current device must be the
 * one `stream` belongs to.  Other arguments and errors as grmhd_rk_step. */
#define GRMHD_NOALLOC_SCRATCH_BYTES (256u << 20)
int grmhd_rk_step_noalloc(const grmhd_domain* dom, const grmhd_params* par, const grmhd_metric* met, double* U,
                          double* P, double dt, int32_t scheme, double* stage_ckpt, double* max_rate,
                          int64_t* n_fail, void* stream);

/* Vector-Jacobian product of con2prim on interior cells: gU = (dP/dU)^T gP,
 * through the implicit-function theorem (con2prim inverts Eqs. (p2c1)-(p2c4),
 * so dP/dU = (dU/dP)^{-1}, evaluated at the primitives P).  FP64. */
int grmhd_con2prim_adjoint(const grmhd_domain* dom, const grmhd_params* par, const grmhd_metric* met,
                           const double* P, const double* gP, double* gU, void* stream);

/* Adjoint of one grmhd_rk_step: gU_in = (dU^{n+1}/dU^n)^T gU_out on interior
 * cells, from the stage checkpoints that grmhd_rk_step wrote (the primitives
 * of U^n and of the stage states).  Per stage, in reverse: the transposed flux
 * divergence, HLLE and reconstruction (scattered with FP64 atomics, so the
 * last bits can vary between runs), the source-term VJP, con2prim through the
 * implicit-function theorem and the transposed stage combine.  Branches
 * (minmod, max/min of the wave speeds, positivity fallback) follow the forward
 * choice; atmosphere resets are not differentiated.  P receives the primitives
 * of U^n.  FP64 whatever par->precision says.
 * ws: grmhd_workspace_bytes(..., for_adjoint = 1) bytes. */
int grmhd_rk_step_adjoint(const grmhd_domain* dom, const grmhd_params* par, const grmhd_metric* met,
                          const double* stage_ckpt, double* P, double dt, int32_t scheme, const double* gU_out,
                          double* gU_in, void* ws, size_t ws_bytes, void* stream);

/* ---- constrained transport (Sec. III B: the vector potential on cell edges) ----
 *
 * A: 3 fields (A_x, A_y, A_z), each vert_stride apart and laid out like the
 * vertex metric.  A_e of the edge along axis e at cell index c_e along e and
 * vertex indices along the two other axes sits at the vertex storage index
 * with c_e in place of that vertex index.  Edges of the interior (cell index
 * 0..n-1 along e, vertex index 0..n along the others) are read and written.
 * The face field is Bcal = curl A (Bcal^d = d_a A_b - d_b A_a, (d, a, b)
 * cyclic, one-sided differences across the face), whose discrete divergence
 * vanishes to round-off; the cell-centred Bcal of U is the mean of the two
 * face values.  The induction equation becomes d_t A_e = F^a(Bcal^b) =
 * -F^b(Bcal^a), each taken as the mean of the HLLE fluxes of the two faces
 * beside the edge (ghost columns have the fluxes of the columns they copy), the
 * edge value the mean of the two.  The gauge term of A, a gradient that curl
 * removes, is left out. */

/* Initial data: P's B = (cell-centred curl A) / sqrt(gamma) on interior cells
 * (P's other fields are kept), then U from P as grmhd_prim2con does. */
int grmhd_ct_init(const grmhd_domain* dom, const grmhd_params* par, const grmhd_metric* met, const double* A,
                  double* U, double* P, void* stream);

/* Face field curl A on every interior face: 3 fields laid out like cells; the
 * d-face at vertex index m along d sits at cell index m (m = n in the first
 * ghost layer).  Other entries are not written. */
int grmhd_ct_face_field(const grmhd_domain* dom, const double* A, double* Bface, void* stream);

/* One method-of-lines step (SSPRK3, SSPRK2 or classic RK4) with constrained
 * transport: U's Bcal is set from A^n, con2prim (skipped with p_current = 1),
 * then per stage the stage kernel (its magnetic face fluxes kept), the same
 * stage combine for A from the edge averages, and U_{s+1}'s Bcal from
 * A_{s+1} before its con2prim.  U, P, A are updated in place.  max_rate,
 * n_fail as grmhd_rk_step.  ws: grmhd_ct_workspace_bytes() bytes.  No stage
 * checkpoints or adjoint. */
int grmhd_rk_step_ct(const grmhd_domain* dom, const grmhd_params* par, const grmhd_metric* met, double* U, double* P,
                     double* A, double dt, int32_t scheme, double* max_rate, int64_t* n_fail, void* ws,
                     size_t ws_bytes, void* stream);

/* Workspace bytes for grmhd_rk_step_ct. */
size_t grmhd_ct_workspace_bytes(const grmhd_domain* dom, const grmhd_params* par, int32_t scheme);

/* Workspace bytes for grmhd_rk_step (for_adjoint = 0) or
 * grmhd_rk_step_adjoint (for_adjoint = 1). */
size_t grmhd_workspace_bytes(const grmhd_domain* dom, const grmhd_params* par, int32_t scheme,
                             int32_t for_adjoint);

/* Kernel timing for measurement: while enabled, every stage-kernel and
 * con2prim-kernel launch is bracketed by HIP events recorded on the launch
 * stream.  grmhd_timing_read synchronizes on those events and returns, per
 * kernel kind (0 = stage kernel, 1 = con2prim kernel), the summed duration in
 * milliseconds and the number of launches since grmhd_timing_enable(1).
 * Not thread-safe; meant for benchmarks. */
int grmhd_timing_enable(int32_t on);
int grmhd_timing_read(double* ms /* (host) [2] */, int64_t* launches /* (host) [2] */);

/* Message for an error code. */
const char* grmhd_strerror(int code);

/* Text of the last HIP error seen by the calling thread ("" if none). */
const char* grmhd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GRMHD_H */
