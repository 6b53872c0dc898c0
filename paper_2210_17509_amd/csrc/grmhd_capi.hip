// gfx950 kernels of the GRMHD hot path and the C ABI declared in grmhd.h.
//
// Kernels
//   k_prim2con  one thread per interior cell (Eqs. (p2c1)-(p2c4)).
//   k_con2prim  one thread per interior cell: 3D Newton, Newman-Hamlin fallback,
//               atmosphere (Sec. II C, RHS step 1).
//   k_adj_face, k_adj_cell  the adjoint of a stage (per face direction, per cell).
// The fused stage kernel is in grmhd_stage.h, compiled per reconstruction in
// stage_<recon>.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "grmhd.h"
#include "grmhd_adjoint.h"
#include "grmhd_device.h"
#include "grmhd_stage.h"

using namespace gk;

namespace {

constexpr uint64_t TABLE_MAGIC = 0x47524d4844544231ull;  // "GRMHDTB1"

struct CellArgs {
  Table tab;
  double* U;
  double* P;     // guess
  double* Pout;  // result (may be P)
  int32_t write_u;  // 0: U is read only (atmosphere resets are not written back)
  double* ckpt;  // nullable copy of the recovered primitives
  int32_t* status;
  unsigned long long* n_fail;
  const double* __restrict__ gamma;
  int64_t cs, vs;
  KPhys ph;
};

// ---------------------------------------------------------------- cell kernels

__device__ __forceinline__ bool cell_of(const Table& tab, int blk, int tid, int& b, int& c, int& vb) {
  b = find_box(tab.c2p_prefix, tab.nbox, blk);
  const KBox& bx = tab.box[b];
  const int lin = (blk - tab.c2p_prefix[b]) * C2P_BLOCK + tid;
  const int nxy = bx.n[0] * bx.n[1];
  if (lin >= nxy * bx.n[2]) return false;
  const int k = lin / nxy;
  const int r = lin - k * nxy;
  const int j = r / bx.n[0];
  const int i = r - j * bx.n[0];
  const int ng = bx.ng;
  c = ((k + ng) * (bx.NXY / bx.NX) + (j + ng)) * bx.NX + (i + ng);
  vb = ((k + ng) * (bx.VXY / bx.VX) + (j + ng)) * bx.VX + (i + ng);
  return true;
}

__global__ __launch_bounds__(C2P_BLOCK) void k_con2prim(CellArgs a) {
  int b, c, vb;
  unsigned long long fail = 0;
  if (cell_of(a.tab, blockIdx.x, threadIdx.x, b, c, vb)) {
    const KBox& bx = a.tab.box[b];
    CentreMetric cm;
    centre_metric<false, false>(GlobalVerts{nullptr, nullptr, a.gamma + bx.vert_off, a.vs}, vb, bx.VX, bx.VXY, cm);
    const int64_t cc = bx.cell_off + c;
    double U[8], P[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      U[q] = a.U[q * a.cs + cc];
      P[q] = a.P[q * a.cs + cc];
    }
    const int st = c2p_cell(cm.g, cm.gi, cm.sqrtg, a.ph, U, P);
#pragma unroll
    for (int q = 0; q < 8; ++q) a.Pout[q * a.cs + cc] = P[q];
    if (a.write_u && st != C2P_OK && st != C2P_FALLBACK) {
#pragma unroll
      for (int q = 0; q < 8; ++q) a.U[q * a.cs + cc] = U[q];
    }
    if (a.ckpt) {
#pragma unroll
      for (int q = 0; q < 8; ++q) a.ckpt[q * a.cs + cc] = P[q];
    }
    if (a.status) a.status[cc] = st;
    fail = (st >= C2P_NOCONV && st <= C2P_NONFINITE) ? 1ull : 0ull;
  }
  if (a.n_fail) {
    for (int o = 32; o > 0; o >>= 1) fail += __shfl_xor(fail, o, 64);
    if ((threadIdx.x & 63) == 0 && fail) atomicAdd(a.n_fail, fail);
  }
}

__global__ __launch_bounds__(C2P_BLOCK) void k_prim2con(Table tab, const double* __restrict__ P,
                                                        double* __restrict__ U, const double* __restrict__ gamma,
                                                        int64_t cs, int64_t vs, double gm1) {
  int b, c, vb;
  if (!cell_of(tab, blockIdx.x, threadIdx.x, b, c, vb)) return;
  const KBox& bx = tab.box[b];
  CentreMetric cm;
  centre_metric<false, false>(GlobalVerts{nullptr, nullptr, gamma + bx.vert_off, vs}, vb, bx.VX, bx.VXY, cm);
  const int64_t cc = bx.cell_off + c;
  double p[8], u[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) p[q] = P[q * cs + cc];
  p2c_cell(cm.g, cm.sqrtg, gm1, p, u);
#pragma unroll
  for (int q = 0; q < 8; ++q) U[q * cs + cc] = u[q];
}


// ---------------------------------------------------------------- adjoint kernels

struct AdjArgs {
  Table tab;
  const double* __restrict__ P;   // primitives of the stage state
  const double* __restrict__ V;   // vector the Jacobian transpose is applied to
  double* __restrict__ Pbar;      // accumulated adjoint of the primitives
  const double* __restrict__ alpha;
  const double* __restrict__ beta;
  const double* __restrict__ gamma;
  int64_t cs, vs;
  KPhys ph;
};

// Reverse of one face's two reconstructions for one field: d[0..5] = the
// adjoints (aL, aR of the left and right side values) carried back to the
// face's stencil cells s[0..5]; a side that fell back to first order passes its
// adjoint to its own cell.  Branch-free (a fallen-back side is differentiated
// with a zero adjoint), so callers can add d into register arrays at constant
// offsets.
template <int RECON>
__device__ __forceinline__ void recon_reverse(const double* s, double aL, double aR, bool fbL, bool fbR, double eps,
                                              double d[6]) {
  constexpr bool ZW = (RECON >= GRMHD_RECON_WENOZ);
  constexpr int ZP = (RECON == RECON_WENOZ2) ? 2 : 1;
  const double wL = fbL ? 0.0 : aL, wR = fbR ? 0.0 : aR;
  if (RECON == GRMHD_RECON_MINMOD) {
    double gl[3], gr[3];
    minmod_grad(s[1], s[2], s[3], gl);
    minmod_grad(s[4], s[3], s[2], gr);
    d[0] = 0.0;
    d[1] = wL * gl[0];
    d[2] = wL * gl[1] + wR * gr[2];
    d[3] = wL * gl[2] + wR * gr[1];
    d[4] = wR * gr[0];
    d[5] = 0.0;
  } else {
    double gl[5], gr[5];
    weno5_vjp<ZW, ZP>(s, eps, ZP, wL, gl);
    const double sr[5] = {s[5], s[4], s[3], s[2], s[1]};
    weno5_vjp<ZW, ZP>(sr, eps, ZP, wR, gr);
    d[0] = gl[0];
    d[1] = gl[1] + gr[4];
    d[2] = gl[2] + gr[3];
    d[3] = gl[3] + gr[2];
    d[4] = gl[4] + gr[1];
    d[5] = gr[0];
  }
  d[2] += fbL ? aL : 0.0;
  d[3] += fbR ? aR : 0.0;
}

// The face's forward pass (reconstruction of the two side states from the
// stencil cells idx[0..5], the metric at the face centre, the side states and
// HLLE) and its reverse from the flux adjoint Fb down to the adjoints qbL, qbR
// of the two reconstructed side states; fbL, fbR: the side fell back to
// first order (the positivity fallback).
template <int D, int RECON, bool SHIFT>
__device__ __forceinline__ void face_side_adjoints(const AdjArgs& a, const KBox& bx, const double* __restrict__ Pb,
                                                   const int idx[6], int i, int j, int k, const double Fb[8],
                                                   double qbL[8], double qbR[8], bool& fbL, bool& fbR) {
  // forward reconstruction values
  const int ng = bx.ng;
  double PL[8], PR[8];
  constexpr bool ZW = (RECON >= GRMHD_RECON_WENOZ);
  constexpr int ZP = (RECON == RECON_WENOZ2) ? 2 : 1;
  const double eps = ZW ? a.ph.wenoz_eps : a.ph.weno_eps;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const double* __restrict__ f = Pb + q * a.cs;
    double s[6];
#pragma unroll
    for (int o = 0; o < 6; ++o) s[o] = (RECON == GRMHD_RECON_MINMOD && (o == 0 || o == 5)) ? 0.0 : f[idx[o]];
    if (RECON == GRMHD_RECON_MINMOD) {
      PL[q] = s[2] + 0.5 * minmod(s[2] - s[1], s[3] - s[2]);
      PR[q] = s[3] - 0.5 * minmod(s[3] - s[2], s[4] - s[3]);
    } else {
      PL[q] = weno5<ZW, ZP>(s[0], s[1], s[2], s[3], s[4], eps, ZP);
      PR[q] = weno5<ZW, ZP>(s[5], s[4], s[3], s[2], s[1], eps, ZP);
    }
  }
  const int vb = ((k + ng) * (bx.VXY / bx.VX) + (j + ng)) * bx.VX + (i + ng);
  constexpr int A = (D + 1) % 3, B = (D + 2) % 3;
  const int sa = (A == 0) ? 1 : (A == 1 ? bx.VX : bx.VXY);
  const int sb = (B == 0) ? 1 : (B == 1 ? bx.VX : bx.VXY);
  FaceMetric<double> m;
  face_metric<D, SHIFT, double>(
      GlobalVerts{a.alpha + bx.vert_off, SHIFT ? a.beta + bx.vert_off : nullptr, a.gamma + bx.vert_off, a.vs}, vb, sa,
      sb, m);
  SideState<double> sL, sR;
  side_v2(m, PL, sL);
  side_v2(m, PR, sR);
  fbL = !side_ok(PL, sL.v2);
  fbR = !side_ok(PR, sR.v2);
  if (fbL) {
#pragma unroll
    for (int q = 0; q < 8; ++q) PL[q] = Pb[q * a.cs + idx[2]];
    side_v2(m, PL, sL);
  }
  if (fbR) {
#pragma unroll
    for (int q = 0; q < 8; ++q) PR[q] = Pb[q * a.cs + idx[3]];
    side_v2(m, PR, sR);
  }
  const double gam = a.ph.gam, gm1 = a.ph.gm1;
  side_rest(m, PL, gm1, sL);
  side_rest(m, PR, gm1, sR);
  double lpL, lmL, lpR, lmR;
  side_speeds<D>(m, PL, sL, gam, lpL, lmL);
  side_speeds<D>(m, PR, sR, gam, lpR, lmR);
  // forward branch choices of xi+ = max(0, max(lpL, lpR)), xi- = min(0, min(lmL, lmR))
  const double mp = (lpL < lpR) ? lpR : lpL;
  const int mpi = (lpL < lpR) ? 2 : 1;
  const double mn = (lmR < lmL) ? lmR : lmL;
  const int mni = (lmR < lmL) ? 2 : 1;
  const double xip = (0.0 < mp) ? mp : 0.0;
  const int ip = (0.0 < mp) ? mpi : 0;
  const double xim = (mn < 0.0) ? mn : 0.0;
  const int im = (mn < 0.0) ? mni : 0;
  const double den = xip - xim;
  double UL[8], FL[8], UR[8], FR[8];
  side_cons_flux<D>(m, PL, sL, UL, FL);
  side_cons_flux<D>(m, PR, sR, UR, FR);
  double gFL[8], gFR[8], gUL[8], gUR[8];
  double xbp = 0.0, xbm = 0.0;
  if (den > 0.0) {
    const double idn = rcp_r(den);
    const double xx = xip * xim;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double du = UR[q] - UL[q];
      const double Fs = (xip * FL[q] - xim * FR[q] + xx * du) * idn;
      gFL[q] = Fb[q] * xip * idn;
      gFR[q] = -Fb[q] * xim * idn;
      gUL[q] = -Fb[q] * xx * idn;
      gUR[q] = Fb[q] * xx * idn;
      xbp += Fb[q] * (FL[q] + xim * du - Fs) * idn;
      xbm += Fb[q] * (-FR[q] + xip * du + Fs) * idn;
    }
  } else {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      gFL[q] = gFR[q] = 0.5 * Fb[q];
      gUL[q] = gUR[q] = 0.0;
    }
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) qbL[q] = qbR[q] = 0.0;
  side_vjp<D>(m, PL, gam, gm1, gUL, gFL, ip == 1 ? xbp : 0.0, im == 1 ? xbm : 0.0, qbL);
  side_vjp<D>(m, PR, gam, gm1, gUR, gFR, ip == 2 ? xbp : 0.0, im == 2 ? xbm : 0.0, qbR);
}

// Face VJP: Fbar = (v_c - v_{c-1}) / dx_D, then the reverse of HLLE, of the two
// side states and of the reconstruction, scattered onto the stencil cells of
// the face (ghost cells map onto the interior cells they copy).
template <int D, int RECON, bool SHIFT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_adj_face(AdjArgs a) {
  const int nb = a.tab.nbox;
  const int32_t* pre = a.tab.face_prefix + D * (nb + 1);
  // y and z faces: each XCD takes a contiguous run of face blocks, so blocks
  // with overlapping stencils share its L2
  const int blk = (D != 0) ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
  const int b = find_box(pre, nb, blk);
  const KBox& bx = a.tab.box[b];
  const int nfx = bx.n[0] + (D == 0), nfy = bx.n[1] + (D == 1), nfz = bx.n[2] + (D == 2);
  int i, j, k;
  bool live;
  // x faces: a block is FACE_BLOCK consecutive faces in storage order.  Lanes
  // past the box's last face take part (with nothing to add) in the wave-level
  // exchange of the x faces below.
  // y and z faces: a block is a patch of ADJ_PX faces along x by ADJ_PD faces
  // along D (lane = x fastest) at one index po of the third axis; px, pd: the
  // patch's indices along x and D.
  const int local = blk - pre[b];
  int px = 0, pd = 0, po = 0;
  if constexpr (D == 0) {
    const int lin_raw = local * FACE_BLOCK + threadIdx.x;
    live = lin_raw < nfx * nfy * nfz;
    const int lin = live ? lin_raw : 0;
    i = lin % nfx;
    const int r = lin / nfx;
    j = r % nfy;
    k = r / nfy;
  } else {
    const int nfD = (D == 1) ? nfy : nfz;
    const int pbx = (bx.n[0] + ADJ_PX - 1) / ADJ_PX, pbd = (nfD + ADJ_PD - 1) / ADJ_PD;
    px = local % pbx;
    pd = (local / pbx) % pbd;
    po = local / (pbx * pbd);
    const int ix = px * ADJ_PX + (int)threadIdx.x % ADJ_PX, id = pd * ADJ_PD + (int)threadIdx.x / ADJ_PX;
    live = ix < bx.n[0] && id < nfD;
    i = live ? ix : 0;
    j = (D == 1) ? (live ? id : 0) : po;
    k = (D == 2) ? (live ? id : 0) : po;
  }
  const int ng = bx.ng;
  const int c = (D == 0) ? i : (D == 1 ? j : k);
  const int nD = bx.n[D];
  const int sD = (D == 0) ? 1 : (D == 1 ? bx.NX : bx.NXY);
  const int base = (D == 0)   ? ((k + ng) * (bx.NXY / bx.NX) + (j + ng)) * bx.NX + ng
                   : (D == 1) ? (k + ng) * bx.NXY + ng * bx.NX + (i + ng)
                              : ng * bx.NXY + (j + ng) * bx.NX + (i + ng);
  int idx[6];
#pragma unroll
  for (int o = 0; o < 6; ++o) {
    const int m = c + o - 3;
    const int mm = (m < 0) ? bx.mlo[D][(m + 3) < 0 ? 0 : m + 3] : (m >= nD ? bx.mhi[D][(m - nD) > 2 ? 2 : m - nD] : m);
    idx[o] = base + mm * sD;
  }
  const double* __restrict__ Pb = a.P + bx.cell_off;
  const double* __restrict__ Vb = a.V + bx.cell_off;
  double* __restrict__ Gb = a.Pbar + bx.cell_off;
  // adjoint of the face flux
  double Fb[8];
  bool any = false;
  const double id = bx.inv_dx[D];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const double vr = (c < nD) ? Vb[q * a.cs + idx[3]] : 0.0;
    const double vl = (c >= 1) ? Vb[q * a.cs + idx[2]] : 0.0;
    Fb[q] = live ? (vr - vl) * id : 0.0;
    any = any || (Fb[q] != 0.0);
  }
  // y and z faces add their stencil contributions into an LDS patch of the
  // ADJ_PD + 5 cell rows along D that the block's faces reach (all 8 fields),
  // and the patch is added to Pbar with one atomic per nonzero element at the
  // end (instead of an atomic per contribution).  Row r of the patch is the cell
  // pd * ADJ_PD - 3 + r along D.
  __shared__ double spatch[(D == 0) ? 1 : 8 * ADJ_ROWS * (ADJ_PX + 1)];
  if constexpr (D != 0) {
    for (int e = threadIdx.x; e < 8 * ADJ_ROWS * (ADJ_PX + 1); e += FACE_BLOCK) spatch[e] = 0.0;
    __syncthreads();
  }
  const bool skip = !__any(any);  // the whole wave has nothing to propagate
  if constexpr (D == 0) {
    if (skip) return;
  }
  double qbL[8], qbR[8];
  bool fbL = false, fbR = false;
  if (!skip) face_side_adjoints<D, RECON, SHIFT>(a, bx, Pb, idx, i, j, k, Fb, qbL, qbR, fbL, fbR);
  const double eps = (RECON >= GRMHD_RECON_WENOZ) ? a.ph.wenoz_eps : a.ph.weno_eps;
  // x faces: a wave holds consecutive faces of one grid line, so the lane of the
  // face just below cell m (the cell's "owner") gathers the contributions of its
  // neighbour lanes to m and adds them with one atomic.  give[o]: stencil cell o
  // is an interior cell whose owner is in this wave; take[o]: this lane's own
  // cell receives contribution o of lane + 3 - o.
  const int lane = threadIdx.x & 63;
  bool give[6], take[6];
#pragma unroll
  for (int o = 0; o < 6; ++o) {
    const int m = c + o - 3, owner = lane + o - 3, from = lane + 3 - o, fc = c + 3 - o;
    give[o] = (D == 0) && live && m >= 0 && m < nD && owner >= 0 && owner < 64;
    take[o] = (D == 0) && live && c < nD && from >= 0 && from < 64 && fc >= 0 && fc <= nD;
  }
  // reverse of the reconstruction, scattered onto the stencil cells, one field at
  // a time (only one stencil is live; prefetching the next field's stencil
  // costs more in registers than it hides).  The per-field adjoints are shifted
  // down one slot per iteration so every register index is static.
  constexpr int O0 = (RECON == GRMHD_RECON_MINMOD) ? 1 : 0, O1 = (RECON == GRMHD_RECON_MINMOD) ? 5 : 6;

#pragma clang loop unroll(disable)
  for (int q = 0; q < 8 && !skip; ++q) {
    double s[6] = {0, 0, 0, 0, 0, 0};
    const double* __restrict__ f = Pb + q * a.cs;
#pragma unroll
    for (int o = O0; o < O1; ++o) s[o] = f[idx[o]];
    const double aL = qbL[0], aR = qbR[0];
#pragma unroll
    for (int t = 0; t < 7; ++t) {
      qbL[t] = qbL[t + 1];
      qbR[t] = qbR[t + 1];
    }
    double sb[6];
    recon_reverse<RECON>(s, aL, aR, fbL, fbR, eps, sb);
    if (D == 0) {
      double own = 0.0;
#pragma unroll
      for (int o = 0; o < 6; ++o) {
        const double x = __shfl(sb[o], (lane + 3 - o) & 63);
        if (take[o]) own += x;
        if (!give[o] && sb[o] != 0.0) unsafeAtomicAdd(Gb + q * a.cs + idx[o], sb[o]);
      }
      if (own != 0.0) unsafeAtomicAdd(Gb + q * a.cs + idx[3], own);
    } else {
      const int lx = (int)threadIdx.x % ADJ_PX, ld = (int)threadIdx.x / ADJ_PX;
#pragma unroll
      for (int o = 0; o < 6; ++o)  // only faces that exist add (their rows stay within the ghost maps)
        if (live && sb[o] != 0.0) atomicAdd(&spatch[(q * ADJ_ROWS + ld + o) * (ADJ_PX + 1) + lx], sb[o]);
    }
  }
  if constexpr (D != 0) {
    __syncthreads();
    for (int e = threadIdx.x; e < 8 * ADJ_ROWS * ADJ_PX; e += FACE_BLOCK) {
      const int lx = e % ADJ_PX, rr = (e / ADJ_PX) % ADJ_ROWS, q = e / (ADJ_PX * ADJ_ROWS);
      const double v = spatch[(q * ADJ_ROWS + rr) * (ADJ_PX + 1) + lx];
      if (v == 0.0) continue;
      const int ix = px * ADJ_PX + lx;
      const int m = pd * ADJ_PD - 3 + rr;  // cell index along D (ghost rows map to the cells they copy)
      const int mm = (m < 0) ? bx.mlo[D][m + 3] : (m >= nD ? bx.mhi[D][m - nD] : m);
      const int cell = (D == 1) ? ((po + ng) * bx.NXY + (mm + ng) * bx.NX + (ix + ng))
                                : ((mm + ng) * bx.NXY + (po + ng) * bx.NX + (ix + ng));
      unsafeAtomicAdd(Gb + q * a.cs + cell, v);
    }
  }
}

// Solve A^T x = y for the 8x8 Jacobian A = dU/dP of Eqs. (p2c1)-(p2c4); A has
// the block form [[A11, A12], [0, sqrt(g) I3]] (U_B = sqrt(g) B).
// J[r][c] = dU_r/dP_c for the first five rows.
__device__ __forceinline__ void solve_dUdP_T(const double (*J)[8], double sqrtg, const double* y, double* x) {
  double M[5][6];  // A11^T | rhs
#pragma unroll
  for (int r = 0; r < 5; ++r) {
#pragma unroll
    for (int cc = 0; cc < 5; ++cc) M[r][cc] = J[cc][r];
    M[r][5] = y[r];
  }
  // Gaussian elimination with partial pivoting
#pragma unroll
  for (int col = 0; col < 5; ++col) {
    int piv = col;
    double best = fabs(M[col][col]);
#pragma unroll
    for (int r = col + 1; r < 5; ++r)
      if (fabs(M[r][col]) > best) { best = fabs(M[r][col]); piv = r; }
#pragma unroll
    for (int r = col + 1; r < 5; ++r) {  // row swap with static indices only
      const bool sw = (r == piv);
#pragma unroll
      for (int cc = 0; cc < 6; ++cc) {
        const double t = M[col][cc];
        M[col][cc] = sw ? M[r][cc] : t;
        M[r][cc] = sw ? t : M[r][cc];
      }
    }
    const double ip = 1.0 / M[col][col];
#pragma unroll
    for (int r = col + 1; r < 5; ++r) {
      const double f = M[r][col] * ip;
#pragma unroll
      for (int cc = col; cc < 6; ++cc) M[r][cc] -= f * M[col][cc];
    }
  }
#pragma unroll
  for (int r = 4; r >= 0; --r) {
    double t = M[r][5];
#pragma unroll
    for (int cc = r + 1; cc < 5; ++cc) t -= M[r][cc] * x[cc];
    x[r] = t / M[r][r];
  }
  // rows of A^T for the field components: sum_{q<5} A[q][5+k] x_q + sqrt(g) x_{5+k} = y_{5+k}
  const double is = 1.0 / sqrtg;
#pragma unroll
  for (int kk = 0; kk < 3; ++kk) {
    double t = y[5 + kk];
#pragma unroll
    for (int q = 0; q < 5; ++q) t -= J[q][5 + kk] * x[q];
    x[5 + kk] = t * is;
  }
}

struct AdjCellArgs {
  Table tab;
  const double* __restrict__ P;
  const double* Vin;              // v = adjoint of U_{s+1}
  double* V;                      // out (stage > 0): adjoint of U_s (may alias Vin)
  double* Gn;                     // accumulated adjoint of U^n
  double* Pbar;                   // read, then cleared for the next stage's faces
  const double* __restrict__ alpha;
  const double* __restrict__ beta;
  const double* __restrict__ gamma;
  int64_t cs, vs;
  KPhys ph;
  double cstage, dt;
  double* Pout;                   // stage 0 only (else null): receives the checkpointed primitives of U^n
  int32_t first_stage;            // stage 0: its adjoint adds to Gn, and P-bar is left as is
  int32_t gn_init;                // Gn is written, not accumulated (first stage processed)
  int32_t mode;  // 0: RK stage adjoint; 1: con2prim adjoint only (V = gP in, Gn = gU out)
};

// Cell part of the stage adjoint: source VJP, con2prim through the implicit-
// function theorem, and the transposed stage combine
// U_{s+1} = (1 - c) U^n + c U_s + c dt L(U_s).
// Waves per SIMD: three fit the zero-shift variant without spills (156 VGPRs),
// the shift variant needs the register budget of two.
template <bool SHIFT>
__global__ __launch_bounds__(C2P_BLOCK) __attribute__((amdgpu_waves_per_eu(SHIFT ? 2 : 3))) void k_adj_cell(
    AdjCellArgs a) {
  int b, c, vb;
  if (!cell_of(a.tab, blockIdx.x, threadIdx.x, b, c, vb)) return;
  const KBox& bx = a.tab.box[b];
  const int64_t cc = bx.cell_off + c;
  // centre metric (and for the stage adjoint its derivatives) first, one vertex
  // field at a time, before the cell's own fields are loaded
  const GlobalVerts gv{a.alpha + bx.vert_off, SHIFT ? a.beta + bx.vert_off : nullptr, a.gamma + bx.vert_off, a.vs};
  CentreMetric cm;
  MetricDeriv md;
  if (a.mode == 0) centre_metric_deriv<SHIFT>(gv, vb, bx.VX, bx.VXY, bx.inv_dx, cm, md);
  else centre_metric<false, false>(gv, vb, bx.VX, bx.VXY, cm);
  double P[8], v[8], pb[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    P[q] = a.P[q * a.cs + cc];
    v[q] = a.Vin[q * a.cs + cc];
    pb[q] = (a.mode == 0) ? a.Pbar[q * a.cs + cc] : v[q];
  }
  // stores only after every load (the pointers may alias as far as the
  // compiler knows, so a store would hold back the loads behind it)
  if (a.mode == 0 && !a.first_stage) {
#pragma unroll
    for (int q = 0; q < 8; ++q) a.Pbar[q * a.cs + cc] = 0.0;
  }
  if (a.Pout) {
#pragma unroll
    for (int q = 0; q < 8; ++q) a.Pout[q * a.cs + cc] = P[q];
  }
  // (dS/dP)^T v by reverse mode, then dU/dP written out, then the transposed
  // solve (implicit-function theorem for con2prim).
  if (a.mode == 0) sources_vjp<SHIFT>(cm, md, P, a.ph.gam, v, pb);
  double J[5][8];
  p2c_jacobian(cm.g, cm.sqrtg, a.ph.gm1, P, J);
  double w[8];
  solve_dUdP_T(J, cm.sqrtg, pb, w);
  if (a.mode == 1) {
#pragma unroll
    for (int q = 0; q < 8; ++q) a.Gn[q * a.cs + cc] = w[q];
    return;
  }
  const double cs = a.cstage;
  double gp[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) gp[q] = a.gn_init ? 0.0 : a.Gn[q * a.cs + cc];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const double gs = cs * (v[q] + a.dt * w[q]);
    double gn = gp[q] + (1.0 - cs) * v[q];
    if (a.first_stage) gn += gs;
    else a.V[q * a.cs + cc] = gs;
    a.Gn[q * a.cs + cc] = gn;
  }
}

// Classic RK4 after stage s: A = (first ? U^n : A) + b_s dt L; then either the
// next stage state Unext = U^n + a_s dt L or, after the last stage, U = A.
__global__ __launch_bounds__(C2P_BLOCK) void k_rk4_combine(Table tab, double* U, const double* __restrict__ L,
                                                            double* A, double* Unext, double adt, double bdt,
                                                            int32_t first, int32_t last, int64_t cs) {
  int b, c, vb;
  if (!cell_of(tab, blockIdx.x, threadIdx.x, b, c, vb)) return;
  const int64_t cc = tab.box[b].cell_off + c;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int64_t x = q * cs + cc;
    const double l = L[x];
    const double un = U[x];
    const double acc = (first ? un : A[x]) + bdt * l;
    if (last) {
      U[x] = acc;
    } else {
      A[x] = acc;
      Unext[x] = un + adt * l;
    }
  }
}

// Fill the interior cells of 8 pooled fields with a value.
__global__ __launch_bounds__(C2P_BLOCK) void k_fill(Table tab, double* X, int64_t cs, double val) {
  int b, c, vb;
  if (!cell_of(tab, blockIdx.x, threadIdx.x, b, c, vb)) return;
  const int64_t cc = tab.box[b].cell_off + c;
#pragma unroll
  for (int q = 0; q < 8; ++q) X[q * cs + cc] = val;
}

// ---------------------------------------------------------------- constrained transport (Sec. III B)
//
// The vector potential A (3 fields, stored like the vertex metric) lives on cell
// edges: A_e of the edge along e at cell index c_e and vertex indices along the
// two other axes sits at the vertex-shaped index with c_e in place of that vertex
// index.  The face field is Bcal = curl A, the cell's Bcal the mean of its two
// face values; d_t A_e = F^a(Bcal^b) = -F^b(Bcal^a) (a = e+1, b = e+2 cyclic),
// each the mean of the HLLE fluxes of the two faces beside the edge, and the
// edge value the mean of the two.  The gauge term of A is a gradient, which curl
// removes: it is left out.

// Interior vertex point (n + 1 per axis) of workgroup blk, thread tid.
__device__ __forceinline__ bool vert_point_of(const Table& tab, int blk, int tid, int& b, int p[3]) {
  b = find_box(tab.vert_prefix, tab.nbox, blk);
  const KBox& bx = tab.box[b];
  const int lin = (blk - tab.vert_prefix[b]) * C2P_BLOCK + tid;
  const int nx = bx.n[0] + 1, nxy = nx * (bx.n[1] + 1);
  if (lin >= nxy * (bx.n[2] + 1)) return false;
  p[2] = lin / nxy;
  const int r = lin - p[2] * nxy;
  p[1] = r / nx;
  p[0] = r - p[1] * nx;
  return true;
}

// box-local storage index of an interior-coordinate point on the vertex / cell grids
__device__ __forceinline__ int64_t vpos(const KBox& bx, const int p[3]) {
  return ((int64_t)(p[2] + bx.ng) * (bx.VXY / bx.VX) + (p[1] + bx.ng)) * bx.VX + (p[0] + bx.ng);
}
__device__ __forceinline__ int64_t cpos(const KBox& bx, const int p[3]) {
  return ((int64_t)(p[2] + bx.ng) * (bx.NXY / bx.NX) + (p[1] + bx.ng)) * bx.NX + (p[0] + bx.ng);
}
// cell coordinate c (-1 <= c <= n) along an axis mapped into the box: the fluxes
// of a ghost column are those of the column it copies
__device__ __forceinline__ int col_map(const KBox& bx, int axis, int c) {
  return c < 0 ? bx.mlo[axis][c + 3] : (c >= bx.n[axis] ? bx.mhi[axis][c - bx.n[axis]] : c);
}

// Face field Bcal^d of the d-face at vertex index p[d] along d (cells p[a], p[b]).
__device__ __forceinline__ double face_curl(const KBox& bx, const double* __restrict__ A, int64_t vs, int d,
                                            const int p[3]) {
  const int a = (d + 1) % 3, b = (d + 2) % 3;
  int pa[3] = {p[0], p[1], p[2]}, pb[3] = {p[0], p[1], p[2]};
  ++pa[a];
  ++pb[b];
  const double dAb = A[b * vs + vpos(bx, pa)] - A[b * vs + vpos(bx, p)];
  const double dAa = A[a * vs + vpos(bx, pb)] - A[a * vs + vpos(bx, p)];
  return dAb * bx.inv_dx[a] - dAa * bx.inv_dx[b];
}

struct CTEdgeArgs {
  Table tab;
  const double* __restrict__ bflux;  // the stage kernel's transverse magnetic face fluxes (6 fields)
  const double* An;                  // A^n
  const double* As;                  // the stage state's potential
  double* Aout;                      // SSPRK: A_{s+1}; RK4: the next stage state, or A^{n+1}
  double* Acc;                       // RK4 accumulator
  int64_t cs, vs;
  double c, dt;                      // SSPRK: A_{s+1} = A^n + c ((A_s - A^n) + dt dA/dt)
  double adt, bdt;                   // RK4: next = A^n + a dt dA/dt, Acc += b dt dA/dt
  int32_t rk4, first, last;
};

__global__ __launch_bounds__(C2P_BLOCK) void k_ct_edge(CTEdgeArgs a) {
  int b, p[3];
  if (!vert_point_of(a.tab, blockIdx.x, threadIdx.x, b, p)) return;
  const KBox& bx = a.tab.box[b];
  const double* bf = a.bflux + bx.cell_off;
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    if (p[e] >= bx.n[e]) continue;  // an edge along e has a cell index along e
    const int ea = (e + 1) % 3, eb = (e + 2) % 3;
    double fa = 0.0, fb = 0.0;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      int c1[3] = {p[0], p[1], p[2]}, c2[3] = {p[0], p[1], p[2]};
      c1[eb] = col_map(bx, eb, p[eb] - 1 + side);  // a-faces beside the edge: F^a(Bcal^b)
      c2[ea] = col_map(bx, ea, p[ea] - 1 + side);  // b-faces beside the edge: F^b(Bcal^a)
      fa += bf[(2 * ea) * a.cs + cpos(bx, c1)];
      fb += bf[(2 * eb + 1) * a.cs + cpos(bx, c2)];
    }
    const double E = 0.5 * (0.5 * fa - 0.5 * fb);
    const int64_t x = e * a.vs + bx.vert_off + vpos(bx, p);
    const double an = a.An[x];
    if (!a.rk4) {
      a.Aout[x] = an + a.c * ((a.As[x] - an) + a.dt * E);
    } else {
      const double acc = (a.first ? an : a.Acc[x]) + a.bdt * E;
      if (a.last) {
        a.Aout[x] = acc;
      } else {
        a.Acc[x] = acc;
        a.Aout[x] = an + a.adt * E;
      }
    }
  }
}

struct CTCellArgs {
  Table tab;
  const double* __restrict__ A;
  double* U;
  double* P;
  const double* __restrict__ gamma;
  int64_t cs, vs;
  KPhys ph;
  int32_t mode;  // 0: U's Bcal from A, then con2prim; 1: U's Bcal only; 2: P's B = Bcal / sqrt(gamma), U = P->U
  unsigned long long* n_fail;
};

__global__ __launch_bounds__(C2P_BLOCK) void k_ct_cell(CTCellArgs a) {
  int b, c, vb;
  unsigned long long fail = 0;
  if (cell_of(a.tab, blockIdx.x, threadIdx.x, b, c, vb)) {
    const KBox& bx = a.tab.box[b];
    const double* Ab = a.A + bx.vert_off;
    const int ng = bx.ng;
    const int k = c / bx.NXY - ng, j = (c / bx.NX) % (bx.NXY / bx.NX) - ng, i = c % bx.NX - ng;
    double Bc[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      int lo[3] = {i, j, k}, hi[3] = {i, j, k};
      ++hi[d];
      Bc[d] = 0.5 * (face_curl(bx, Ab, a.vs, d, lo) + face_curl(bx, Ab, a.vs, d, hi));
    }
    const int64_t cc = bx.cell_off + c;
    if (a.mode == 1) {
#pragma unroll
      for (int d = 0; d < 3; ++d) a.U[(5 + d) * a.cs + cc] = Bc[d];
    } else {
      CentreMetric cm;
      centre_metric<false, false>(GlobalVerts{nullptr, nullptr, a.gamma + bx.vert_off, a.vs}, vb, bx.VX, bx.VXY, cm);
      double U[8], P[8];
      if (a.mode == 2) {
#pragma unroll
        for (int q = 0; q < 8; ++q) P[q] = a.P[q * a.cs + cc];
        const double is = 1.0 / cm.sqrtg;
#pragma unroll
        for (int d = 0; d < 3; ++d) P[5 + d] = Bc[d] * is;
        p2c_cell(cm.g, cm.sqrtg, a.ph.gm1, P, U);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          a.P[q * a.cs + cc] = P[q];
          a.U[q * a.cs + cc] = U[q];
        }
      } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          U[q] = (q >= 5) ? Bc[q - 5] : a.U[q * a.cs + cc];
          P[q] = a.P[q * a.cs + cc];
        }
        const int st = c2p_cell(cm.g, cm.gi, cm.sqrtg, a.ph, U, P);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          a.P[q * a.cs + cc] = P[q];
          a.U[q * a.cs + cc] = U[q];
        }
        fail = (st >= C2P_NOCONV && st <= C2P_NONFINITE) ? 1ull : 0ull;
      }
    }
  }
  if (a.n_fail) {
    for (int o = 32; o > 0; o >>= 1) fail += __shfl_xor(fail, o, 64);
    if ((threadIdx.x & 63) == 0 && fail) atomicAdd(a.n_fail, fail);
  }
}

// Face field curl A on every interior face, 3 cell-shaped fields (the d-face at
// vertex index m along d at the cell index m).
__global__ __launch_bounds__(C2P_BLOCK) void k_ct_face(Table tab, const double* __restrict__ A, double* Bf, int64_t cs,
                                                       int64_t vs) {
  int b, p[3];
  if (!vert_point_of(tab, blockIdx.x, threadIdx.x, b, p)) return;
  const KBox& bx = tab.box[b];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int ea = (d + 1) % 3, eb = (d + 2) % 3;
    if (p[ea] >= bx.n[ea] || p[eb] >= bx.n[eb]) continue;
    Bf[d * cs + bx.cell_off + cpos(bx, p)] = face_curl(bx, A + bx.vert_off, vs, d, p);
  }
}

// ---------------------------------------------------------------- host side

thread_local std::string g_last_error;

// ---- optional per-launch timing (benchmarks) ----
struct TimedLaunch {
  hipEvent_t a, b;
  int kind;
};
bool g_timing = false;
std::vector<TimedLaunch> g_timed;      // pending pairs
std::vector<hipEvent_t> g_event_pool;  // reusable events
double g_time_ms[2] = {0, 0};
int64_t g_time_n[2] = {0, 0};

hipEvent_t pool_event() {
  if (!g_event_pool.empty()) {
    hipEvent_t e = g_event_pool.back();
    g_event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void drain_timing() {
  for (auto& t : g_timed) {
    float ms = 0.f;
    if (hipEventSynchronize(t.b) == hipSuccess && hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
      g_time_ms[t.kind] += ms;
      g_time_n[t.kind] += 1;
    }
    g_event_pool.push_back(t.a);
    g_event_pool.push_back(t.b);
  }
  g_timed.clear();
}

struct TimeScope {
  hipEvent_t a = nullptr, b = nullptr;
  hipStream_t s;
  int kind;
  TimeScope(int k, hipStream_t st) : s(st), kind(k) {
    if (!g_timing) return;
    if (g_timed.size() > 4096) drain_timing();
    a = pool_event();
    b = pool_event();
    if (!a || !b || hipEventRecord(a, s) != hipSuccess) release();  // this launch goes untimed
  }
  ~TimeScope() {
    if (!a || !b) return;
    if (hipEventRecord(b, s) != hipSuccess) {
      release();
      return;
    }
    g_timed.push_back({a, b, kind});
  }
  void release() {
    if (a) g_event_pool.push_back(a);
    if (b) g_event_pool.push_back(b);
    a = b = nullptr;
  }
};

struct Prepared {
  uint64_t hash;
  int32_t nbox;
  int64_t c2p_blocks;
  int64_t tiles[NTILE];
  int64_t face_blocks[3];
  int64_t vert_blocks;
};
std::mutex g_mu;
std::unordered_map<const void*, Prepared> g_prepared;

uint64_t fnv1a(const void* p, size_t n, uint64_t h = 1469598103934665603ull) {
  const unsigned char* c = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) {
    h ^= c[i];
    h *= 1099511628211ull;
  }
  return h;
}

uint64_t domain_hash(const grmhd_domain* dom) {
  uint64_t h = fnv1a(&dom->nbox, sizeof(dom->nbox));
  h = fnv1a(&dom->cell_stride, sizeof(dom->cell_stride), h);
  h = fnv1a(&dom->vert_stride, sizeof(dom->vert_stride), h);
  return fnv1a(dom->box, sizeof(grmhd_box) * (size_t)dom->nbox, h);
}

int fail_hip(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return GRMHD_EHIP;
}

int invalid(const char* why) {
  g_last_error = why;
  return GRMHD_EINVAL;
}

size_t table_bytes(int32_t nbox) {
  return sizeof(TableHeader) + sizeof(KBox) * (size_t)nbox + sizeof(int32_t) * (size_t)(nbox + 1) * (1 + NTILE + 3 + 1);
}

int periodic_map(int m, int n) { return ((m % n) + n) % n; }

int check_box(const grmhd_box& b, int64_t cs, int64_t vs) {
  for (int d = 0; d < 3; ++d) {
    if (b.n[d] < 1) return invalid("box with n < 1");
    if (!(b.dx[d] > 0.0) || !std::isfinite(b.dx[d])) return invalid("box with dx <= 0 or non-finite");
    if (!std::isfinite(b.x0[d])) return invalid("box with non-finite x0");
  }
  for (int q = 0; q < 6; ++q)
    if (b.bc[q] != GRMHD_BC_PERIODIC && b.bc[q] != GRMHD_BC_OUTFLOW) return invalid("unknown boundary code");
  for (int d = 0; d < 3; ++d)
    if ((b.bc[2 * d] == GRMHD_BC_PERIODIC) != (b.bc[2 * d + 1] == GRMHD_BC_PERIODIC))
      return invalid("periodic boundary on only one side of an axis");
  if (b.ng < 2 || b.ng > 16) return invalid("ghost layers must be in [2, 16]");
  const int64_t NX = b.n[0] + 2 * b.ng, NY = b.n[1] + 2 * b.ng, NZ = b.n[2] + 2 * b.ng;
  const int64_t nc = NX * NY * NZ, nv = (NX + 1) * (NY + 1) * (NZ + 1);
  // The stage kernel addresses a box's cells and vertices as base + 32-bit byte
  // offset (element index << 3), so every element index must stay below 2^29.
  if (nc >= (int64_t(1) << 29) || nv >= (int64_t(1) << 29))
    return invalid("box too large: cells or vertices with ghosts reach 2^29 (32-bit byte offsets)");
  if (b.cell_off < 0 || b.cell_off + nc > cs) return invalid("box cells outside the cell stride");
  if (b.vert_off < 0 || b.vert_off + nv > vs) return invalid("box vertices outside the vertex stride");
  return GRMHD_OK;
}

int check_domain_struct(const grmhd_domain* dom) {
  if (!dom || !dom->box || dom->nbox < 1 || !dom->table) return invalid("null domain, box list or table");
  if (dom->cell_stride < 1 || dom->vert_stride < 1) return invalid("bad field strides");
  for (int b = 0; b < dom->nbox; ++b) {
    int r = check_box(dom->box[b], dom->cell_stride, dom->vert_stride);
    if (r) return r;
  }
  // boxes must not overlap in the pooled arrays
  std::vector<std::pair<int64_t, int64_t>> iv;
  for (int b = 0; b < dom->nbox; ++b) {
    const grmhd_box& x = dom->box[b];
    const int64_t nc = int64_t(x.n[0] + 2 * x.ng) * (x.n[1] + 2 * x.ng) * (x.n[2] + 2 * x.ng);
    iv.push_back({x.cell_off, x.cell_off + nc});
  }
  std::sort(iv.begin(), iv.end());
  for (size_t q = 1; q < iv.size(); ++q)
    if (iv[q].first < iv[q - 1].second) return invalid("boxes overlap in the cell arrays");
  return GRMHD_OK;
}

// Validated, prepared domain: returns the launch totals.
int check_domain(const grmhd_domain* dom, Prepared& out) {
  if (!dom || !dom->box || !dom->table) return invalid("null domain, box list or table");
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_prepared.find(dom->table);
  if (it == g_prepared.end()) return invalid("domain table not prepared (call grmhd_domain_prepare)");
  if (it->second.nbox != dom->nbox || it->second.hash != domain_hash(dom))
    return invalid("domain changed since grmhd_domain_prepare");
  out = it->second;
  return GRMHD_OK;
}

int check_params(const grmhd_params* p, const grmhd_domain* dom, KPhys& ph) {
  if (!p) return invalid("null params");
  if (p->recon < GRMHD_RECON_MINMOD || p->recon > GRMHD_RECON_WENOZ) return invalid("unknown reconstruction");
  if (p->precision != GRMHD_FP64 && p->precision != GRMHD_MIXED) return invalid("unknown precision");
  if (!(p->eos_gamma > 1.0) || !std::isfinite(p->eos_gamma)) return invalid("eos_gamma must be > 1");
  if (!(p->weno_eps > 0.0) || !(p->wenoz_eps > 0.0) || !std::isfinite(p->weno_eps) || !std::isfinite(p->wenoz_eps))
    return invalid("WENO epsilons must be positive");
  if (p->wenoz_p != 1 && p->wenoz_p != 2) return invalid("wenoz_p must be 1 or 2");
  if (!(p->c2p_tol > 0.0) || p->c2p_maxit < 1 || p->c2p_maxit > 100000) return invalid("bad con2prim tolerance");
  if (p->tile < -1 || p->tile >= NTILE) return invalid("unknown tile shape");
  if (p->schedule != GRMHD_SCHED_GRID && p->schedule != GRMHD_SCHED_QUEUE) return invalid("unknown schedule");
  if (p->p_current != 0 && p->p_current != 1) return invalid("p_current must be 0 or 1");
  if (!(p->rho_atm > 0.0) || !(p->atm_K > 0.0) || !(p->atm_gamma > 0.0) || !std::isfinite(p->rho_atm) ||
      !std::isfinite(p->atm_K) || !std::isfinite(p->atm_gamma))
    return invalid("bad atmosphere parameters");
  const int need = (p->recon == GRMHD_RECON_MINMOD) ? 2 : 3;
  if (dom)
    for (int b = 0; b < dom->nbox; ++b)
      if (dom->box[b].ng < need) return invalid("not enough ghost layers for the reconstruction");
  ph.gam = p->eos_gamma;
  ph.gm1 = p->eos_gamma - 1.0;
  ph.gf = p->eos_gamma / (p->eos_gamma - 1.0);
  ph.weno_eps = p->weno_eps;
  ph.wenoz_eps = p->wenoz_eps;
  ph.wenoz_p = p->wenoz_p;
  ph.c2p_tol = p->c2p_tol;
  ph.c2p_maxit = p->c2p_maxit;
  ph.rho_atm = p->rho_atm;
  // A state whose density is within a relative 1e-6 of rho_atm is taken as the
  // atmosphere without a recovery: for the atmosphere state itself in a strong
  // field the thermal energy lies below the rounding of tau, so whether its
  // recovery succeeds would be decided by the last bit of tau.
  ph.rho_floor = p->rho_atm * (1.0 + 1e-6);
  ph.p_atm = p->atm_K * std::pow(p->rho_atm, p->atm_gamma);
  ph.eps_atm = ph.p_atm / ((p->eos_gamma - 1.0) * p->rho_atm);
  return GRMHD_OK;
}

Table make_table(const grmhd_domain* dom) {
  Table t;
  const char* base = static_cast<const char*>(dom->table);
  t.box = reinterpret_cast<const KBox*>(base + sizeof(TableHeader));
  t.c2p_prefix = reinterpret_cast<const int32_t*>(base + sizeof(TableHeader) + sizeof(KBox) * (size_t)dom->nbox);
  t.tile_prefix = t.c2p_prefix + (dom->nbox + 1);
  t.face_prefix = t.tile_prefix + NTILE * (dom->nbox + 1);
  t.vert_prefix = t.face_prefix + 3 * (dom->nbox + 1);
  t.nbox = dom->nbox;
  return t;
}

// Compute units of the current device (a persistent launch keeps as many
// 256-thread workgroups per CU resident as the kernel has waves per SIMD).
int persistent_blocks() {
  static int n = [] {
    int dev = 0, cus = 256;
    int n = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
      cus = n;
    return cus;
  }();
  return n;
}

int pick_tile(const grmhd_domain* dom, const grmhd_params* par) {
  if (par->tile >= 0) return par->tile;
  (void)dom;
  // 16x4x3: every direction's faces take one pass of the workgroup
  return 3;
}

hipError_t launch_stage(const StageArgs& a, int recon, int precision, int64_t blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  TimeScope ts(0, s);
  switch (recon) {
    case GRMHD_RECON_MINMOD: return launch_stage_recon<GRMHD_RECON_MINMOD>(a, precision, blocks, s);
    case GRMHD_RECON_WENO5: return launch_stage_recon<GRMHD_RECON_WENO5>(a, precision, blocks, s);
    default:
      return (a.ph.wenoz_p == 2) ? launch_stage_recon<RECON_WENOZ2>(a, precision, blocks, s)
                                 : launch_stage_recon<GRMHD_RECON_WENOZ>(a, precision, blocks, s);
  }
}

int check_metric(const grmhd_metric* m, bool need_alpha) {
  if (!m || !m->gamma || (need_alpha && !m->alpha)) return invalid("null metric field");
  return GRMHD_OK;
}

hipError_t launch_c2p(const grmhd_domain* dom, const Prepared& pr, const KPhys& ph, const grmhd_metric* met, double* U,
                      double* P, double* ckpt, int32_t* status, int64_t* n_fail, hipStream_t s,
                      double* Pout = nullptr) {
  CellArgs a;
  a.tab = make_table(dom);
  a.U = U;
  a.P = P;
  a.Pout = Pout ? Pout : P;
  a.write_u = 1;
  a.ckpt = ckpt;
  a.status = status;
  a.n_fail = reinterpret_cast<unsigned long long*>(n_fail);
  a.gamma = met->gamma;
  a.cs = dom->cell_stride;
  a.vs = dom->vert_stride;
  a.ph = ph;
  TimeScope ts(1, s);
  hipLaunchKernelGGL(k_con2prim, dim3((unsigned)pr.c2p_blocks), dim3(C2P_BLOCK), 0, s, a);
  return hipGetLastError();
}

StageArgs stage_args(const grmhd_domain* dom, const grmhd_params* par, const KPhys& ph, const grmhd_metric* met,
                     const double* P) {
  StageArgs a;
  a.tab = make_table(dom);
  a.tile = pick_tile(dom, par);
  a.P = P;
  a.Us = a.Un = nullptr;
  a.Uout = nullptr;
  a.alpha = met->alpha;
  a.beta = met->beta;
  a.gamma = met->gamma;
  a.cs = dom->cell_stride;
  a.vs = dom->vert_stride;
  a.cstage = 1.0;
  a.dt = 0.0;
  a.mode = 0;
  a.ph = ph;
  a.max_rate = nullptr;
  a.queue = nullptr;
  a.persist_blocks = 0;
  a.Pout = nullptr;
  a.ckpt = nullptr;
  a.ckpt_in = nullptr;
  a.n_fail = nullptr;
  a.bflux = nullptr;
  a.Acc = nullptr;
  a.adt = a.bdt = 0.0;
  a.rk_first = a.rk_last = 0;
  return a;
}


template <int RECON, bool SHIFT>
hipError_t launch_adj_faces(const AdjArgs& a, const Prepared& pr, hipStream_t s) {
  if (pr.face_blocks[0] > 0) hipLaunchKernelGGL((k_adj_face<0, RECON, SHIFT>), dim3((unsigned)pr.face_blocks[0]), dim3(FACE_BLOCK), 0, s, a);
  if (pr.face_blocks[1] > 0) hipLaunchKernelGGL((k_adj_face<1, RECON, SHIFT>), dim3((unsigned)pr.face_blocks[1]), dim3(FACE_BLOCK), 0, s, a);
  if (pr.face_blocks[2] > 0) hipLaunchKernelGGL((k_adj_face<2, RECON, SHIFT>), dim3((unsigned)pr.face_blocks[2]), dim3(FACE_BLOCK), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_adj_faces_r(const AdjArgs& a, int recon, const Prepared& pr, hipStream_t s) {
  const bool sh = a.beta != nullptr;
  switch (recon) {
    case GRMHD_RECON_MINMOD:
      return sh ? launch_adj_faces<GRMHD_RECON_MINMOD, true>(a, pr, s) : launch_adj_faces<GRMHD_RECON_MINMOD, false>(a, pr, s);
    case GRMHD_RECON_WENO5:
      return sh ? launch_adj_faces<GRMHD_RECON_WENO5, true>(a, pr, s) : launch_adj_faces<GRMHD_RECON_WENO5, false>(a, pr, s);
    default:
      if (a.ph.wenoz_p == 2)
        return sh ? launch_adj_faces<RECON_WENOZ2, true>(a, pr, s) : launch_adj_faces<RECON_WENOZ2, false>(a, pr, s);
      return sh ? launch_adj_faces<GRMHD_RECON_WENOZ, true>(a, pr, s) : launch_adj_faces<GRMHD_RECON_WENOZ, false>(a, pr, s);
  }
}

hipError_t launch_adj_cell(const AdjCellArgs& a, const Prepared& pr, hipStream_t s) {
  if (a.beta)
    hipLaunchKernelGGL((k_adj_cell<true>), dim3((unsigned)pr.c2p_blocks), dim3(C2P_BLOCK), 0, s, a);
  else
    hipLaunchKernelGGL((k_adj_cell<false>), dim3((unsigned)pr.c2p_blocks), dim3(C2P_BLOCK), 0, s, a);
  return hipGetLastError();
}

// ---- fixed scratch of grmhd_rk_step_noalloc ----
// The step's workspace for callers that cannot allocate: one array per device,
// held for the life of the process.  Host code never uses the array's name as
// a device address; it takes the address hipGetSymbolAddress returns for the
// current device, once per device.
__device__ __align__(256) unsigned char scratch[GRMHD_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
void* g_scratch_ptr[MAX_DEVICES] = {};
std::mutex g_scratch_mu;

int scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
  if (dev < 0 || dev >= MAX_DEVICES) return invalid("device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return fail_hip(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail_hip(hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch) returned null");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return GRMHD_OK;
}

}  // namespace

extern "C" {

size_t grmhd_domain_table_bytes(int32_t nbox) { return nbox < 1 ? 0 : table_bytes(nbox); }

int grmhd_domain_prepare(const grmhd_domain* dom, void* stream) {
  int r = check_domain_struct(dom);
  if (r) return r;
  const int nb = dom->nbox;
  std::vector<char> buf(table_bytes(nb), 0);
  TableHeader* h = reinterpret_cast<TableHeader*>(buf.data());
  KBox* kb = reinterpret_cast<KBox*>(buf.data() + sizeof(TableHeader));
  int32_t* c2p = reinterpret_cast<int32_t*>(buf.data() + sizeof(TableHeader) + sizeof(KBox) * nb);
  int32_t* tp = c2p + (nb + 1);
  int32_t* fp = tp + NTILE * (nb + 1);
  int32_t* vp = fp + 3 * (nb + 1);
  Prepared pr;
  int64_t acc_c2p = 0, acc_t[NTILE] = {}, acc_f[3] = {0, 0, 0}, acc_v = 0;
  for (int b = 0; b < nb; ++b) {
    const grmhd_box& x = dom->box[b];
    KBox& k = kb[b];
    std::memset(&k, 0, sizeof(k));
    for (int d = 0; d < 3; ++d) k.n[d] = x.n[d];
    k.ng = x.ng;
    k.NX = x.n[0] + 2 * x.ng;
    k.NXY = k.NX * (x.n[1] + 2 * x.ng);
    k.VX = k.NX + 1;
    k.VXY = k.VX * (x.n[1] + 2 * x.ng + 1);
    k.cell_off = x.cell_off;
    k.vert_off = x.vert_off;
    for (int d = 0; d < 3; ++d) {
      k.inv_dx[d] = 1.0 / x.dx[d];
      const bool per = x.bc[2 * d] == GRMHD_BC_PERIODIC;
      for (int o = 0; o < 3; ++o) {
        const int mlo = o - 3, mhi = x.n[d] + o;
        k.mlo[d][o] = per ? periodic_map(mlo, x.n[d]) : 0;
        k.mhi[d][o] = per ? periodic_map(mhi, x.n[d]) : x.n[d] - 1;
      }
    }
    c2p[b] = (int32_t)acc_c2p;
    const int64_t nint = int64_t(x.n[0]) * x.n[1] * x.n[2];
    acc_c2p += (nint + C2P_BLOCK - 1) / C2P_BLOCK;
    for (int t = 0; t < NTILE; ++t) {
      tp[t * (nb + 1) + b] = (int32_t)acc_t[t];
      acc_t[t] += int64_t((x.n[0] + TILE_X[t] - 1) / TILE_X[t]) * ((x.n[1] + TILE_Y[t] - 1) / TILE_Y[t]) *
                  ((x.n[2] + TILE_Z[t] - 1) / TILE_Z[t]);
    }
    for (int d = 0; d < 3; ++d) {
      fp[d * (nb + 1) + b] = (int32_t)acc_f[d];
      if (d == 0) {
        const int64_t nf = int64_t(x.n[0] + 1) * x.n[1] * x.n[2];
        acc_f[d] += (nf + FACE_BLOCK - 1) / FACE_BLOCK;
      } else {  // patches of ADJ_PX x ADJ_PD faces at each index of the third axis
        const int64_t nfd = x.n[d] + 1, nother = (d == 1) ? x.n[2] : x.n[1];
        acc_f[d] += int64_t((x.n[0] + ADJ_PX - 1) / ADJ_PX) * ((nfd + ADJ_PD - 1) / ADJ_PD) * nother;
      }
    }
    vp[b] = (int32_t)acc_v;
    const int64_t nvp = int64_t(x.n[0] + 1) * (x.n[1] + 1) * (x.n[2] + 1);
    acc_v += (nvp + C2P_BLOCK - 1) / C2P_BLOCK;
  }
  if (acc_v >= (int64_t(1) << 31)) return invalid("too many vertices");
  vp[nb] = (int32_t)acc_v;
  h->vert_blocks = acc_v;
  if (acc_c2p >= (int64_t(1) << 31)) return invalid("too many cells");
  c2p[nb] = (int32_t)acc_c2p;
  for (int t = 0; t < NTILE; ++t) {
    if (acc_t[t] >= (int64_t(1) << 31)) return invalid("too many tiles");
    tp[t * (nb + 1) + nb] = (int32_t)acc_t[t];
  }
  for (int d = 0; d < 3; ++d) {
    if (acc_f[d] >= (int64_t(1) << 31)) return invalid("too many faces");
    fp[d * (nb + 1) + nb] = (int32_t)acc_f[d];
    h->face_blocks[d] = acc_f[d];
  }
  h->magic = TABLE_MAGIC;
  h->hash = domain_hash(dom);
  h->nbox = nb;
  h->c2p_blocks = acc_c2p;
  for (int t = 0; t < NTILE; ++t) h->tiles[t] = acc_t[t];
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(dom->table, buf.data(), buf.size(), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return fail_hip(e, "hipMemcpyAsync(table)");
  e = hipStreamSynchronize(s);  // the host staging buffer dies with this call
  if (e != hipSuccess) return fail_hip(e, "hipStreamSynchronize");
  pr.hash = h->hash;
  pr.nbox = nb;
  pr.c2p_blocks = acc_c2p;
  for (int t = 0; t < NTILE; ++t) pr.tiles[t] = acc_t[t];
  for (int d = 0; d < 3; ++d) pr.face_blocks[d] = acc_f[d];
  pr.vert_blocks = acc_v;
  std::lock_guard<std::mutex> lk(g_mu);
  g_prepared[dom->table] = pr;
  return GRMHD_OK;
}

int grmhd_prim2con(const grmhd_domain* dom, const grmhd_params* par, const grmhd_metric* met, const double* P,
                   double* U, void* stream) {
  Prepared pr;
  KPhys ph;
  int r;
  if ((r = check_domain(dom, pr)) || (r = check_params(par, nullptr, ph)) || (r = check_metric(met, false))) return r;
  if (!P || !U) return invalid("null P or U");
  hipLaunchKernelGGL(k_prim2con, dim3((unsigned)pr.c2p_blocks), dim3(C2P_BLOCK), 0, static_cast<hipStream_t>(stream),
                     make_table(dom), P, U, met->gamma, dom->cell_stride, dom->vert_stride, ph.gm1);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? GRMHD_OK : fail_hip(e, "k_prim2con");
}

int grmhd_con2prim(const grmhd_domain* dom, const grmhd_params* par, const grmhd_metric* met, double* U, double* P,
                   int32_t* status, int64_t* n_fail, void* stream) {
  Prepared pr;
  KPhys ph;
  int r;
  if ((r = check_domain(dom, pr)) || (r = check_params(par, nullptr, ph)) || (r = check_metric(met, false))) return r;
  if (!P || !U) return invalid("null P or U");
  hipError_t e = launch_c2p(dom, pr, ph, met, U, P, nullptr, status, n_fail, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? GRMHD_OK : fail_hip(e, "k_con2prim");
}

int grmhd_rhs(const grmhd_domain* dom, const grmhd_params* par, const grmhd_metric* met, double* U, double* P,
              double* dUdt, double* max_rate, int64_t* n_fail, void* stream) {
  Prepared pr;
  KPhys ph;
  int r;
  if ((r = check_domain(dom, pr)) || (r = check_params(par, dom, ph)) || (r = check_metric(met, true))) return r;
  if (!P || !U || !dUdt) return invalid("null P, U or dUdt");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = launch_c2p(dom, pr, ph, met, U, P, nullptr, nullptr, n_fail, s);
  if (e != hipSuccess) return fail_hip(e, "k_con2prim");
  StageArgs a = stage_args(dom, par, ph, met, P);
  a.Uout = dUdt;
  a.mode = 0;
  a.max_rate = max_rate;
  e = launch_stage(a, par->recon, par->precision, pr.tiles[a.tile], s);
  return e == hipSuccess ? GRMHD_OK : fail_hip(e, "k_stage");
}

// 8-field sets of the step workspace: the stage state W1 and one primitive
// buffer, plus a second primitive buffer when the step starts from the caller's
// P with an odd number of stages (so the last stage can end in P).
static size_t step_sets(const grmhd_params* par, int32_t scheme) {
  if (scheme == GRMHD_RK4) return 4;  // stage state, accumulator, two primitive buffers
  return (par && par->p_current == 1 && scheme == GRMHD_SSPRK3) ? 3 : 2;
}

size_t grmhd_workspace_bytes(const grmhd_domain* dom, const grmhd_params* par, int32_t scheme, int32_t for_adjoint) {
  if (!dom || dom->cell_stride < 1) return 0;
  const size_t field = sizeof(double) * 8 * (size_t)dom->cell_stride;
  return for_adjoint ? 2 * field : step_sets(par, scheme) * field + QUEUE_BYTES;
}

// Classic RK4 (Sec. IV A, Sec. V setupB), fused like the SSPRK stages: con2prim
// of U^n (skipped with p_current), then per stage the stage kernel evaluates L,
// accumulates the step (Acc), forms the next stage state (or U^{n+1}) and
// recovers its primitives in registers.  The primitives rotate P -> Pw -> Pw2
// -> Pw -> P, so the step ends in the caller's P.
static int rk4_step(const grmhd_domain* dom, const Prepared& pr, const KPhys& ph, const grmhd_params* par,
                    const grmhd_metric* met, double* U, double* P, double dt, double* max_rate, int64_t* n_fail,
                    void* ws, hipStream_t s) {
  static const double a4[3] = {0.5, 0.5, 1.0};
  static const double b4[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
  const size_t fsz = 8 * (size_t)dom->cell_stride;
  double* W1 = static_cast<double*>(ws);  // stage state
  double* WA = W1 + fsz;                  // accumulated step
  double* Pw = WA + fsz;                  // primitive buffers
  double* Pw2 = Pw + fsz;
  hipError_t e = hipSuccess;
  if (par->p_current != 1) {
    e = launch_c2p(dom, pr, ph, met, U, P, nullptr, nullptr, n_fail, s);
    if (e != hipSuccess) return fail_hip(e, "k_con2prim");
  }
  StageArgs a = stage_args(dom, par, ph, met, P);
  a.mode = 2;
  a.max_rate = max_rate;
  a.n_fail = reinterpret_cast<unsigned long long*>(n_fail);
  a.Un = U;
  a.Acc = WA;
  if (par->schedule == GRMHD_SCHED_QUEUE) {
    a.queue = reinterpret_cast<unsigned int*>(static_cast<char*>(ws) + sizeof(double) * step_sets(par, GRMHD_RK4) * fsz);
    a.persist_blocks = persistent_blocks();
  }
  double* pin[4] = {P, Pw, Pw2, Pw};
  double* pout[4] = {Pw, Pw2, Pw, P};
  for (int st = 0; st < 4; ++st) {
    a.P = pin[st];
    a.Pout = pout[st];
    a.Uout = (st == 3) ? U : W1;
    a.adt = st < 3 ? a4[st] * dt : 0.0;
    a.bdt = b4[st] * dt;
    a.rk_first = (st == 0);
    a.rk_last = (st == 3);
    e = launch_stage(a, par->recon, par->precision, pr.tiles[a.tile], s);
    if (e != hipSuccess) return fail_hip(e, "k_stage");
  }
  return GRMHD_OK;
}

// One step of grmhd_rk_step with the workspace ws (ws_bytes bytes).
static int rk_step_impl(const grmhd_domain* dom, const grmhd_params* par, const grmhd_metric* met, double* U,
                        double* P, double dt, int32_t scheme, double* stage_ckpt, double* max_rate, int64_t* n_fail,
                        void* ws, size_t ws_bytes, void* stream) {
  Prepared pr;
  KPhys ph;
  int r;
  if ((r = check_domain(dom, pr)) || (r = check_params(par, dom, ph)) || (r = check_metric(met, true))) return r;
  if (!P || !U) return invalid("null P or U");
  if (!(dt > 0.0) || !std::isfinite(dt)) return invalid("dt must be positive and finite");
  if (scheme != GRMHD_SSPRK3 && scheme != GRMHD_SSPRK2 && scheme != GRMHD_RK4)
    return invalid("unknown time integrator");
  if (scheme == GRMHD_RK4 && stage_ckpt) return invalid("stage checkpoints are written for the SSPRK schemes only");
  if (!ws) return invalid("null workspace");
  if (ws_bytes < grmhd_workspace_bytes(dom, par, scheme, 0)) {
    g_last_error = "workspace too small";
    return GRMHD_EWORKSPACE;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (scheme == GRMHD_RK4) return rk4_step(dom, pr, ph, par, met, U, P, dt, max_rate, n_fail, ws, s);
  static const double c3[3] = {1.0, 0.25, 2.0 / 3.0};
  static const double c2[2] = {1.0, 0.5};
  const double* cst = scheme == GRMHD_SSPRK2 ? c2 : c3;
  const int nst = scheme == GRMHD_SSPRK2 ? 2 : 3;
  // Workspace: the intermediate stage state W1, primitive buffers Pw (and Pw2)
  // and the tile-queue counters.  Each stage kernel recovers the primitives of
  // the state it writes (con2prim fused into the stage) into a buffer other than
  // the one it reads.  Starting with con2prim(U^n), the primitives alternate
  // between P and Pw, the first recovery going to the buffer that makes the
  // last stage end in P.  Starting from the caller's P (p_current), stages
  // before the last write Pw, Pw2, ... and the last writes P.
  const size_t fsz = 8 * (size_t)dom->cell_stride;
  const bool pcur = par->p_current == 1;
  double* W1 = static_cast<double*>(ws);
  double* Pw = W1 + fsz;
  double* Pw2 = Pw + fsz;  // SSPRK3 with p_current only
  double* Pcur = P;
  hipError_t e = hipSuccess;
  if (!pcur) {
    Pcur = (nst % 2) ? Pw : P;
    e = launch_c2p(dom, pr, ph, met, U, P, stage_ckpt, nullptr, n_fail, s, Pcur);
    if (e != hipSuccess) return fail_hip(e, "k_con2prim");
  }
  StageArgs a = stage_args(dom, par, ph, met, Pcur);
  a.mode = 1;
  a.dt = dt;
  a.max_rate = max_rate;
  a.n_fail = reinterpret_cast<unsigned long long*>(n_fail);
  a.Un = U;
  if (par->schedule == GRMHD_SCHED_QUEUE) {
    a.queue = reinterpret_cast<unsigned int*>(static_cast<char*>(ws) + sizeof(double) * step_sets(par, scheme) * fsz);
    a.persist_blocks = persistent_blocks();
  }
  for (int st = 0; st < nst; ++st) {
    a.Us = (st == 0) ? U : W1;
    a.Uout = (st == nst - 1) ? U : W1;
    a.cstage = cst[st];
    a.P = Pcur;
    if (!pcur) a.Pout = (Pcur == P) ? Pw : P;
    else a.Pout = (st == nst - 1) ? P : ((st % 2 == 0) ? Pw : Pw2);
    a.ckpt = (stage_ckpt && st + 1 < nst) ? stage_ckpt + (st + 1) * fsz : nullptr;
    a.ckpt_in = (pcur && st == 0) ? stage_ckpt : nullptr;  // primitives of U^n, as given
    e = launch_stage(a, par->recon, par->precision, pr.tiles[a.tile], s);
    if (e != hipSuccess) return fail_hip(e, "k_stage");
    Pcur = a.Pout;
  }
  return GRMHD_OK;
}

int grmhd_rk_step(const grmhd_domain* dom, const grmhd_params* par, const grmhd_metric* met, double* U, double* P,
                  double dt, int32_t scheme, double* stage_ckpt, double* max_rate, int64_t* n_fail, void* ws,
                  size_t ws_bytes, void* stream) {
  return rk_step_impl(dom, par, met, U, P, dt, scheme, stage_ckpt, max_rate, n_fail, ws, ws_bytes, stream);
}

int grmhd_rk_step_noalloc(const grmhd_domain* dom, const grmhd_params* par, const grmhd_metric* met, double* U,
                          double* P, double dt, int32_t scheme, double* stage_ckpt, double* max_rate, int64_t* n_fail,
                          void* stream) {
  if (!dom || dom->cell_stride < 1) return invalid("null domain or bad cell stride");
  const size_t need = grmhd_workspace_bytes(dom, par, scheme, 0);
  if (need > (size_t)GRMHD_NOALLOC_SCRATCH_BYTES) {
    g_last_error = "grmhd_rk_step_noalloc: the step needs " + std::to_string(need) +
                   " bytes of scratch, more than the library's fixed " +
                   std::to_string((size_t)GRMHD_NOALLOC_SCRATCH_BYTES) +
                   " bytes (use grmhd_rk_step with a caller workspace)";
    return GRMHD_EWORKSPACE;
  }
  void* ws = nullptr;
  const int r = scratch_address(&ws);
  if (r) return r;
  return rk_step_impl(dom, par, met, U, P, dt, scheme, stage_ckpt, max_rate, n_fail, ws,
                      (size_t)GRMHD_NOALLOC_SCRATCH_BYTES, stream);
}


int grmhd_con2prim_adjoint(const grmhd_domain* dom, const grmhd_params* par, const grmhd_metric* met, const double* P,
                           const double* gP, double* gU, void* stream) {
  Prepared pr;
  KPhys ph;
  int r;
  if ((r = check_domain(dom, pr)) || (r = check_params(par, nullptr, ph)) || (r = check_metric(met, false))) return r;
  if (!P || !gP || !gU) return invalid("null P, gP or gU");
  AdjCellArgs a;
  a.tab = make_table(dom);
  a.P = P;
  a.Vin = gP;
  a.V = nullptr;  // not written in this mode
  a.Gn = gU;
  a.Pbar = nullptr;
  a.alpha = met->gamma;  // not read in this mode (only the spatial metric enters dU/dP)
  a.beta = nullptr;
  a.gamma = met->gamma;
  a.cs = dom->cell_stride;
  a.vs = dom->vert_stride;
  a.ph = ph;
  a.cstage = 1.0;
  a.dt = 0.0;
  a.Pout = nullptr;
  a.first_stage = 0;
  a.gn_init = 0;
  a.mode = 1;
  hipError_t e = launch_adj_cell(a, pr, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? GRMHD_OK : fail_hip(e, "k_adj_cell");
}

int grmhd_rk_step_adjoint(const grmhd_domain* dom, const grmhd_params* par, const grmhd_metric* met,
                          const double* stage_ckpt, double* P, double dt, int32_t scheme, const double* gU_out,
                          double* gU_in, void* ws, size_t ws_bytes, void* stream) {
  Prepared pr;
  KPhys ph;
  int r;
  if ((r = check_domain(dom, pr)) || (r = check_params(par, dom, ph)) || (r = check_metric(met, true))) return r;
  if (!stage_ckpt || !P || !gU_out || !gU_in) return invalid("null checkpoint, P or adjoint vector");
  if (gU_out == gU_in) return invalid("gU_out and gU_in must not alias");
  if (!(dt > 0.0) || !std::isfinite(dt)) return invalid("dt must be positive and finite");
  if (scheme != GRMHD_SSPRK3 && scheme != GRMHD_SSPRK2) return invalid("unknown time integrator");
  if (!ws) return invalid("null workspace");
  if (ws_bytes < grmhd_workspace_bytes(dom, par, scheme, 1)) {
    g_last_error = "workspace too small";
    return GRMHD_EWORKSPACE;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  static const double c3[3] = {1.0, 0.25, 2.0 / 3.0};
  static const double c2[2] = {1.0, 0.5};
  const double* cst = scheme == GRMHD_SSPRK2 ? c2 : c3;
  const int nst = scheme == GRMHD_SSPRK2 ? 2 : 3;
  const size_t fsz = 8 * (size_t)dom->cell_stride;
  double* V = static_cast<double*>(ws);
  double* Pbar = V + fsz;
  const Table tab = make_table(dom);
  const unsigned cb = (unsigned)pr.c2p_blocks;
  // P-bar starts at zero; the cell kernels of the later stages clear it again
  // after use.  gU_in is written by the first stage processed, then accumulated.
  hipLaunchKernelGGL(k_fill, dim3(cb), dim3(C2P_BLOCK), 0, s, tab, Pbar, dom->cell_stride, 0.0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail_hip(e, "adjoint setup");
  for (int st = nst - 1; st >= 0; --st) {
    // the primitives of the stage state, as the forward step recovered them
    const double* Ps = stage_ckpt + st * fsz;
    // the adjoint of U_{s+1}: gU_out for the last stage, then the workspace copy
    const double* Vin = (st == nst - 1) ? gU_out : V;
    AdjArgs fa;
    fa.tab = tab;
    fa.P = Ps;
    fa.V = Vin;
    fa.Pbar = Pbar;
    fa.alpha = met->alpha;
    fa.beta = met->beta;
    fa.gamma = met->gamma;
    fa.cs = dom->cell_stride;
    fa.vs = dom->vert_stride;
    fa.ph = ph;
    e = launch_adj_faces_r(fa, par->recon, pr, s);
    if (e != hipSuccess) return fail_hip(e, "k_adj_face");
    AdjCellArgs a;
    a.tab = tab;
    a.P = Ps;
    a.Vin = Vin;
    a.V = V;
    a.Gn = gU_in;
    a.Pbar = Pbar;
    a.alpha = met->alpha;
    a.beta = met->beta;
    a.gamma = met->gamma;
    a.cs = dom->cell_stride;
    a.vs = dom->vert_stride;
    a.ph = ph;
    a.cstage = cst[st];
    a.dt = dt;
    a.Pout = (st == 0) ? P : nullptr;
    a.first_stage = (st == 0);
    a.gn_init = (st == nst - 1);
    a.mode = 0;
    e = launch_adj_cell(a, pr, s);
    if (e != hipSuccess) return fail_hip(e, "k_adj_cell");
  }
  return GRMHD_OK;
}

// ---- constrained transport ----

// Workspace of grmhd_rk_step_ct: U-sets (SSPRK: the stage state; RK4: stage state,
// L, accumulator), 6 magnetic face-flux fields, A-sets (SSPRK: stage state; RK4:
// stage state, accumulator).
static void ct_layout(const grmhd_domain* dom, int32_t scheme, size_t& u_sets, size_t& a_sets, size_t& bytes) {
  u_sets = (scheme == GRMHD_RK4) ? 3 : 1;
  a_sets = (scheme == GRMHD_RK4) ? 2 : 1;
  bytes = sizeof(double) * ((8 * u_sets + 6) * (size_t)dom->cell_stride + 3 * a_sets * (size_t)dom->vert_stride);
}

size_t grmhd_ct_workspace_bytes(const grmhd_domain* dom, const grmhd_params* par, int32_t scheme) {
  (void)par;
  if (!dom || dom->cell_stride < 1 || dom->vert_stride < 1) return 0;
  size_t u, a, b;
  ct_layout(dom, scheme, u, a, b);
  return b;
}

static hipError_t launch_ct_cell(const grmhd_domain* dom, const Prepared& pr, const KPhys& ph, const grmhd_metric* met,
                                 const double* A, double* U, double* P, int mode, int64_t* n_fail, hipStream_t s) {
  CTCellArgs c;
  c.tab = make_table(dom);
  c.A = A;
  c.U = U;
  c.P = P;
  c.gamma = met->gamma;
  c.cs = dom->cell_stride;
  c.vs = dom->vert_stride;
  c.ph = ph;
  c.mode = mode;
  c.n_fail = reinterpret_cast<unsigned long long*>(n_fail);
  TimeScope ts(1, s);
  hipLaunchKernelGGL(k_ct_cell, dim3((unsigned)pr.c2p_blocks), dim3(C2P_BLOCK), 0, s, c);
  return hipGetLastError();
}

int grmhd_ct_init(const grmhd_domain* dom, const grmhd_params* par, const grmhd_metric* met, const double* A, double* U,
                  double* P, void* stream) {
  Prepared pr;
  KPhys ph;
  int r;
  if ((r = check_domain(dom, pr)) || (r = check_params(par, nullptr, ph)) || (r = check_metric(met, false))) return r;
  if (!A || !U || !P) return invalid("null A, U or P");
  hipError_t e = launch_ct_cell(dom, pr, ph, met, A, U, P, 2, nullptr, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? GRMHD_OK : fail_hip(e, "k_ct_cell");
}

int grmhd_ct_face_field(const grmhd_domain* dom, const double* A, double* Bface, void* stream) {
  Prepared pr;
  int r;
  if ((r = check_domain(dom, pr))) return r;
  if (!A || !Bface) return invalid("null A or Bface");
  hipLaunchKernelGGL(k_ct_face, dim3((unsigned)pr.vert_blocks), dim3(C2P_BLOCK), 0, static_cast<hipStream_t>(stream),
                     make_table(dom), A, Bface, dom->cell_stride, dom->vert_stride);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? GRMHD_OK : fail_hip(e, "k_ct_face");
}

int grmhd_rk_step_ct(const grmhd_domain* dom, const grmhd_params* par, const grmhd_metric* met, double* U, double* P,
                     double* A, double dt, int32_t scheme, double* max_rate, int64_t* n_fail, void* ws,
                     size_t ws_bytes, void* stream) {
  Prepared pr;
  KPhys ph;
  int r;
  if ((r = check_domain(dom, pr)) || (r = check_params(par, dom, ph)) || (r = check_metric(met, true))) return r;
  if (!P || !U || !A) return invalid("null P, U or A");
  if (!(dt > 0.0) || !std::isfinite(dt)) return invalid("dt must be positive and finite");
  if (scheme != GRMHD_SSPRK3 && scheme != GRMHD_SSPRK2 && scheme != GRMHD_RK4) return invalid("unknown time integrator");
  if (!ws) return invalid("null workspace");
  size_t u_sets, a_sets, need;
  ct_layout(dom, scheme, u_sets, a_sets, need);
  if (ws_bytes < need) {
    g_last_error = "workspace too small";
    return GRMHD_EWORKSPACE;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t fsz = 8 * (size_t)dom->cell_stride;
  double* W1 = static_cast<double*>(ws);             // stage state
  double* WL = W1 + fsz;                             // RK4: L of the stage state
  double* WA = WL + fsz;                             // RK4: accumulated step
  double* BF = W1 + u_sets * fsz;                    // magnetic face fluxes
  double* A1 = BF + 6 * (size_t)dom->cell_stride;    // the stage state's potential
  double* AA = A1 + 3 * (size_t)dom->vert_stride;    // RK4: accumulated potential
  const Table tab = make_table(dom);
  // U^n's Bcal from A^n, then its primitives (unless P already holds them)
  hipError_t e = launch_ct_cell(dom, pr, ph, met, A, U, P, par->p_current == 1 ? 1 : 0, n_fail, s);
  if (e != hipSuccess) return fail_hip(e, "k_ct_cell");
  CTEdgeArgs ea;
  ea.tab = tab;
  ea.bflux = BF;
  ea.An = A;
  ea.Acc = AA;
  ea.cs = dom->cell_stride;
  ea.vs = dom->vert_stride;
  ea.dt = dt;
  ea.rk4 = (scheme == GRMHD_RK4);
  StageArgs a = stage_args(dom, par, ph, met, P);
  a.max_rate = max_rate;
  a.bflux = BF;
  a.tile = CT_TILE;
  if (scheme == GRMHD_RK4) {
    static const double a4[3] = {0.5, 0.5, 1.0};
    static const double b4[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    a.mode = 0;
    a.Uout = WL;
    for (int st = 0; st < 4; ++st) {
      const bool last = (st == 3);
      e = launch_stage(a, par->recon, par->precision, pr.tiles[a.tile], s);
      if (e != hipSuccess) return fail_hip(e, "k_stage");
      hipLaunchKernelGGL(k_rk4_combine, dim3((unsigned)pr.c2p_blocks), dim3(C2P_BLOCK), 0, s, tab, U, WL, WA, W1,
                         st < 3 ? a4[st] * dt : 0.0, b4[st] * dt, (int32_t)(st == 0), (int32_t)last, dom->cell_stride);
      ea.As = nullptr;
      ea.Aout = last ? A : A1;
      ea.adt = st < 3 ? a4[st] * dt : 0.0;
      ea.bdt = b4[st] * dt;
      ea.first = (st == 0);
      ea.last = last;
      ea.c = 0.0;
      hipLaunchKernelGGL(k_ct_edge, dim3((unsigned)pr.vert_blocks), dim3(C2P_BLOCK), 0, s, ea);
      e = hipGetLastError();
      if (e != hipSuccess) return fail_hip(e, "k_ct_edge");
      e = launch_ct_cell(dom, pr, ph, met, last ? A : A1, last ? U : W1, P, 0, n_fail, s);
      if (e != hipSuccess) return fail_hip(e, "k_ct_cell");
    }
    return GRMHD_OK;
  }
  static const double c3[3] = {1.0, 0.25, 2.0 / 3.0};
  static const double c2[2] = {1.0, 0.5};
  const double* cst = scheme == GRMHD_SSPRK2 ? c2 : c3;
  const int nst = scheme == GRMHD_SSPRK2 ? 2 : 3;
  a.mode = 1;
  a.dt = dt;
  a.Un = U;
  for (int st = 0; st < nst; ++st) {
    const bool last = (st == nst - 1);
    a.Us = (st == 0) ? U : W1;
    a.Uout = last ? U : W1;
    a.cstage = cst[st];
    e = launch_stage(a, par->recon, par->precision, pr.tiles[a.tile], s);
    if (e != hipSuccess) return fail_hip(e, "k_stage");
    ea.As = (st == 0) ? A : A1;
    ea.Aout = last ? A : A1;
    ea.c = cst[st];
    ea.first = ea.last = 0;
    ea.adt = ea.bdt = 0.0;
    hipLaunchKernelGGL(k_ct_edge, dim3((unsigned)pr.vert_blocks), dim3(C2P_BLOCK), 0, s, ea);
    e = hipGetLastError();
    if (e != hipSuccess) return fail_hip(e, "k_ct_edge");
    e = launch_ct_cell(dom, pr, ph, met, last ? A : A1, last ? U : W1, P, 0, n_fail, s);
    if (e != hipSuccess) return fail_hip(e, "k_ct_cell");
  }
  return GRMHD_OK;
}

int grmhd_timing_enable(int32_t on) {
  drain_timing();
  g_timing = on != 0;
  g_time_ms[0] = g_time_ms[1] = 0.0;
  g_time_n[0] = g_time_n[1] = 0;
  return GRMHD_OK;
}

int grmhd_timing_read(double* ms, int64_t* launches) {
  if (!ms || !launches) return invalid("null output");
  drain_timing();
  for (int k = 0; k < 2; ++k) {
    ms[k] = g_time_ms[k];
    launches[k] = g_time_n[k];
  }
  return GRMHD_OK;
}

const char* grmhd_strerror(int code) {
  switch (code) {
    case GRMHD_OK: return "success";
    case GRMHD_EINVAL: return "invalid argument";
    case GRMHD_EHIP: return "HIP runtime error";
    case GRMHD_EWORKSPACE: return "workspace too small";
    default: return "unknown error";
  }
}

const char* grmhd_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
