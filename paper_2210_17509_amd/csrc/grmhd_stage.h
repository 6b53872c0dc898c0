// The fused stage kernel of the GRMHD hot path (Sec. II C, RHS steps 1-4): shared
// declarations, and with GRMHD_STAGE_KERNELS defined the kernels themselves and
// their launchers.  Each reconstruction's kernels are compiled in a translation
// unit of their own (stage_<recon>.hip), which instantiates launch_stage_recon.
//
//   k_stage        one workgroup per TX x TY x TZ tile: the tile's vertex metric
//                  is staged in LDS; for each direction every thread reads its
//                  face's stencil (coalesced SoA rows, served by L1/L2),
//                  reconstructs and solves the Riemann problem on its cell's
//                  low face (or one of the tile's high faces), fluxes are
//                  exchanged through LDS, and the divergence, the source terms,
//                  the SSPRK stage combine and con2prim of the new state are
//                  fused, so no face quantity ever reaches HBM.
//   k_stage_queue  the same tile work for persistent workgroups popping tiles
//                  from per-XCD queues.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>

#include "grmhd.h"
#include "grmhd_device.h"

namespace gk {

// Stage-kernel reconstruction codes: the public ones, plus WENO-Z with exponent 2
// (the exponent is a compile-time constant of each stage-kernel instance).
constexpr int RECON_WENOZ2 = GRMHD_RECON_WENOZ + 1;
constexpr size_t QUEUE_BYTES = 256;  // per-XCD tile-queue counters at the end of the step workspace

// tile shapes of the stage kernel (TX * TY * TZ = 256)
constexpr int TILE_X[NTILE] = {16, 8, 64, 16};
constexpr int TILE_Y[NTILE] = {4, 8, 2, 4};
constexpr int TILE_Z[NTILE] = {4, 4, 2, 3};
constexpr int CT_TILE = 3;  // the tile of stage launches that keep the magnetic face fluxes

struct StageArgs {
  Table tab;
  int tile;
  const double* __restrict__ P;
  // Us, Un and Uout alias (an in-place stage writes the state it reads), so
  // they carry no restrict
  const double* Us;
  const double* Un;
  double* Uout;
  const double* __restrict__ alpha;
  const double* __restrict__ beta;
  const double* __restrict__ gamma;
  int64_t cs, vs;
  double cstage, dt;
  int32_t mode;  // 0: Uout = dU/dt; 1: Uout = Un + c ((Us - Un) + dt dU/dt); 2: classic RK4 stage
  // mode 2: Acc = (rk_first ? Un : Acc) + bdt dU/dt; Uout = Un + adt dU/dt, or Acc after the last stage
  double* Acc;
  double adt, bdt;
  int32_t rk_first, rk_last;
  KPhys ph;
  double* max_rate;
  unsigned int* queue;  // non-null: persistent launch over per-XCD tile queues
  int32_t persist_blocks;  // compute units of the device (persistent launch)
  // mode 1 only, nullable: con2prim of each new cell state inside the stage
  // kernel, guessed from P; results to Pout (which must not alias P: other
  // tiles still read P) and to the checkpoint ckpt
  double* Pout;
  double* ckpt;
  double* ckpt_in;  // nullable: receives the stage's input primitives (P) of each cell
  unsigned long long* n_fail;
  // nullable (constrained transport): the two transverse magnetic fluxes of every
  // face, field 2 D + t (t = 0: Bcal^{(D+1)%3}, t = 1: Bcal^{(D+2)%3}) at the storage
  // index of the face's cell (its high neighbour along D); non-null selects the
  // CT_TILE grid launch (tile and schedule are ignored)
  double* bflux;
};

__device__ __forceinline__ void block_max_atomic(double v, double* target) {
  // v >= 0: the IEEE bit pattern orders like an unsigned integer
  __shared__ double red[4];
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    if (m > 0.0) atomicMax(reinterpret_cast<unsigned long long*>(target), (unsigned long long)__double_as_longlong(m));
  }
}

// Global tile index for workgroup blk of a grid of n: workgroup blk runs on XCD
// blk mod 8, which receives the contiguous tile range of its share.
__device__ __forceinline__ int xcd_tile(int blk, int n) {
  const int x = blk & 7, m = blk >> 3;
  const int q = n >> 3, r = n & 7;
  return x * q + (x < r ? x : r) + m;
}

// Sum of the per-thread failure counts of a wave, added by its first lane.
__device__ __forceinline__ void wave_count_atomic(unsigned long long v, unsigned long long* target) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd(target, v);
}

// Launch the stage kernel of reconstruction RECON (a public code or
// RECON_WENOZ2) for the given precision over `blocks` tiles (defined in
// stage_<recon>.hip).
template <int RECON>
hipError_t launch_stage_recon(const StageArgs& a, int precision, int64_t blocks, hipStream_t s);

}  // namespace gk

#ifdef GRMHD_STAGE_KERNELS
namespace gk {
namespace {

// Stencil prefetch distance of the face loop, in fields, for FP64 reconstruction.
// One field ahead is 5% faster than none on the curved 256^3 step (two or three
// ahead gain nothing more); with FP32 reconstruction the same prefetch is 5%
// slower, so there the loads stay where they are used.
constexpr int FACE_PF64 = 1;

// Flux through the low face (direction D) of cell (i, j, k); the face's 4
// vertices are read through vt at vb, vb + sa, vb + sb, vb + sa + sb.
template <int D, int RECON, typename R, bool SHIFT, typename V>
__device__ __forceinline__ void face_flux(const StageArgs& a, const KBox& bx, const double* __restrict__ Pb,
                                          const V& vt, uint32_t vb, uint32_t sa, uint32_t sb, int i, int j, int k,
                                          double F[8], double& rate) {
  const int ng = bx.ng;
  const int c = (D == 0) ? i : (D == 1 ? j : k);
  const int nD = bx.n[D];
  const int sD = (D == 0) ? 1 : (D == 1 ? bx.NX : bx.NXY);
  // storage index of the cell with coordinate 0 along D on this grid line
  const int base = (D == 0)   ? ((k + ng) * (bx.NXY / bx.NX) + (j + ng)) * bx.NX + ng
                   : (D == 1) ? (k + ng) * bx.NXY + ng * bx.NX + (i + ng)
                              : ng * bx.NXY + (j + ng) * bx.NX + (i + ng);
  constexpr int O0 = (RECON == GRMHD_RECON_MINMOD) ? 1 : 0;  // minmod reads cells c-2 .. c+1
  constexpr int O1 = (RECON == GRMHD_RECON_MINMOD) ? 5 : 6;
  uint32_t idx[6];
#pragma unroll
  for (int o = O0; o < O1; ++o) {
    const int m = c + o - 3;
    const int mm = (m < 0) ? bx.mlo[D][m + 3] : (m >= nD ? bx.mhi[D][m - nD] : m);
    idx[o] = (uint32_t)(base + mm * sD);
  }
  // The stencils of the next PF fields are loaded while a field is being
  // reconstructed, so that several fields' loads are in flight at once.
  constexpr int PF = sizeof(R) == 8 ? FACE_PF64 : 0;
  constexpr int NB = PF + 1;
  double ring[NB][6];
#pragma unroll
  for (int p = 0; p < PF; ++p)
#pragma unroll
    for (int o = O0; o < O1; ++o) ring[p][o] = ldg(Pb + p * a.cs, idx[o]);
  R PL[8], PR[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    if (q + PF < 8) {
#pragma unroll
      for (int o = O0; o < O1; ++o) ring[(q + PF) % NB][o] = ldg(Pb + (q + PF) * a.cs, idx[o]);
    }
    R s[6];
#pragma unroll
    for (int o = O0; o < O1; ++o) s[o] = (R)ring[q % NB][o];
    if (RECON == GRMHD_RECON_MINMOD) {
      PL[q] = s[2] + R(0.5) * minmod(s[2] - s[1], s[3] - s[2]);
      PR[q] = s[3] - R(0.5) * minmod(s[3] - s[2], s[4] - s[3]);
    } else {
      constexpr bool z = (RECON >= GRMHD_RECON_WENOZ);
      constexpr int zp = (RECON == RECON_WENOZ2) ? 2 : 1;
      const R eps = (R)(z ? a.ph.wenoz_eps : a.ph.weno_eps);
      if constexpr (sizeof(R) == 8 || !z) {
        // both sides at once (shared candidates and smoothness terms)
        weno5_lr<z, zp>(s, eps, zp, PL[q], PR[q]);
      } else {
        // FP32 WENO-Z keeps its per-weight ratios, side by side
        PL[q] = weno5<z, zp>(s[0], s[1], s[2], s[3], s[4], eps, zp);
        PR[q] = weno5<z, zp>(s[5], s[4], s[3], s[2], s[1], eps, zp);
      }
    }
  }
  FaceMetric<R> m;
  face_metric<D, SHIFT, R>(vt, vb, sa, sb, m);
  // positivity: fall back to the cell values on a side that is not physical
  SideState<R> sL, sR;
  side_v2(m, PL, sL);
  side_v2(m, PR, sR);
  if (!side_ok(PL, sL.v2)) {
#pragma unroll
    for (int q = 0; q < 8; ++q) PL[q] = (R)ldg(Pb + q * a.cs, idx[2]);
    side_v2(m, PL, sL);
  }
  if (!side_ok(PR, sR.v2)) {
#pragma unroll
    for (int q = 0; q < 8; ++q) PR[q] = (R)ldg(Pb + q * a.cs, idx[3]);
    side_v2(m, PR, sR);
  }
  const R gm1 = (R)a.ph.gm1, gam = (R)a.ph.gam;
  side_rest(m, PL, gm1, sL);
  side_rest(m, PR, gm1, sR);
  R Fs[8], xp, xm;
  hlle<D>(m, PL, sL, PR, sR, gam, Fs, xp, xm);
#pragma unroll
  for (int q = 0; q < 8; ++q) F[q] = (double)Fs[q];
  rate = fmax(rate, fmax((double)xp, -(double)xm) * bx.inv_dx[D]);
}

template <int TX, int TY, int TZ> struct TileGeo {
  static constexpr int SX[3] = {TX + 1, TX, TX};
  static constexpr int SY[3] = {TY, TY + 1, TY};
  static constexpr int SZ[3] = {TZ, TZ, TZ + 1};
  static constexpr int slots(int d) { return SX[d] * SY[d] * SZ[d]; }
  static constexpr int maxslots() {
    return std::max(slots(0), std::max(slots(1), slots(2)));
  }
  // the tile's vertex block: vertices org .. org + T along each axis
  static constexpr int VBX = TX + 1, VBY = TY + 1, VBZ = TZ + 1, NVB = VBX * VBY * VBZ;
  static constexpr int nvf(bool shift) { return shift ? 10 : 7; }
};

template <int D, int RECON, typename R, bool SHIFT, int TX, int TY, int TZ, bool BF>
__device__ __forceinline__ void direction_phase(const StageArgs& a, const KBox& bx, const double* __restrict__ Pb,
                                                const double* sV, const int org[3], const int l[3], bool valid,
                                                double (*sF)[TileGeo<TX, TY, TZ>::maxslots()], double acc[8],
                                                double& rate) {
  using G = TileGeo<TX, TY, TZ>;
  constexpr int SX = G::SX[D], SY = G::SY[D];
  constexpr int T_D = (D == 0) ? TX : (D == 1 ? TY : TZ);
  constexpr int TA = (D == 0) ? TY : TX;           // first other axis extent
  constexpr int NEXTRA = (D == 0) ? TY * TZ : (D == 1 ? TX * TZ : TX * TY);
  constexpr int AX = (D == 0) ? 1 : 0;             // first other axis
  constexpr int BX = (D == 2) ? 1 : 2;             // second other axis
  const int tid = threadIdx.x;
  const int lastD = min(T_D, bx.n[D] - org[D]);    // face index after the tile's last valid cell
  constexpr int NCELL = TX * TY * TZ;
  for (int job = tid; job < NCELL + NEXTRA; job += 256) {
    int fl[3];
    bool ok;
    if (job < NCELL) {
      fl[0] = l[0];
      fl[1] = l[1];
      fl[2] = l[2];
      ok = valid;
    } else {
      const int e = job - NCELL;
      fl[AX] = e % TA;
      fl[BX] = e / TA;
      fl[D] = lastD;
      ok = (org[AX] + fl[AX] < bx.n[AX]) && (org[BX] + fl[BX] < bx.n[BX]);
    }
    if (ok) {
      double F[8];
      constexpr uint32_t VS[3] = {1u, (uint32_t)G::VBX, (uint32_t)(G::VBX * G::VBY)};
      const uint32_t lv = fl[0] + G::VBX * (fl[1] + G::VBY * fl[2]);
      face_flux<D, RECON, R, SHIFT>(a, bx, Pb, LdsVerts<G::NVB>{sV}, lv, VS[(D + 1) % 3], VS[(D + 2) % 3],
                                    org[0] + fl[0], org[1] + fl[1], org[2] + fl[2], F, rate);
      const int slot = fl[0] + SX * (fl[1] + SY * fl[2]);
#pragma unroll
      for (int q = 0; q < 8; ++q) sF[q][slot] = F[q];
      if constexpr (BF) {
        const int ng = bx.ng;
        const uint32_t c = ((org[2] + fl[2] + ng) * (bx.NXY / bx.NX) + (org[1] + fl[1] + ng)) * bx.NX + (org[0] + fl[0] + ng);
        double* bf = a.bflux + bx.cell_off;
        stg(bf + (2 * D) * a.cs, c, F[5 + (D + 1) % 3]);
        stg(bf + (2 * D + 1) * a.cs, c, F[5 + (D + 2) % 3]);
      }
    }
  }
  __syncthreads();
  if (valid) {
    const int lo = l[0] + SX * (l[1] + SY * l[2]);
    const int hi = lo + ((D == 0) ? 1 : (D == 1 ? SX : SX * SY));
    const double idx = bx.inv_dx[D];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] += (sF[q][lo] - sF[q][hi]) * idx;
  }
  // The next direction rewrites sF.  After the last one nothing in this tile
  // does, and the next tile of a persistent workgroup starts behind barriers,
  // so FP64 instances go on to the cell update without waiting (0.5% faster);
  // the FP32 instances keep the barrier (dropping it there was 2% slower).
  if constexpr (D != 2 || sizeof(R) != 8) __syncthreads();
}

template <int RECON, typename R, bool SHIFT, int TI, bool BF = false>
__device__ __forceinline__ void stage_tile(const StageArgs& a, int tg,
                                           double (*sF)[TileGeo<TILE_X[TI], TILE_Y[TI], TILE_Z[TI]>::maxslots()],
                                           double* sV, double& rate, unsigned long long& fail) {
  constexpr int TX = TILE_X[TI], TY = TILE_Y[TI], TZ = TILE_Z[TI];
  using G = TileGeo<TX, TY, TZ>;
  const int b = find_box(a.tab.tile_prefix + TI * (a.tab.nbox + 1), a.tab.nbox, tg);
  const KBox& bx = a.tab.box[b];
  const int t = tg - a.tab.tile_prefix[TI * (a.tab.nbox + 1) + b];
  // Tile walk: x fastest, then y within a strip of SH tile rows (about 64
  // tiles), then z, then the next strip.  A contiguous run of tiles (one XCD's
  // share) thus marches up z through a strip narrower than the 96 tiles one XCD
  // holds at once, so the z-halo rows a tile layer loads are still in that
  // XCD's L2 when the next layer needs them as its own cells.
  const int ntx = (bx.n[0] + TX - 1) / TX, nty = (bx.n[1] + TY - 1) / TY, ntz = (bx.n[2] + TZ - 1) / TZ;
  const int SH = max(1, min(nty, 64 / ntx));
  const int r = t / ntx, st = r / (SH * ntz), h = min(SH, nty - st * SH), r3 = r - st * SH * ntz;
  const int org[3] = {(t % ntx) * TX, (st * SH + r3 % h) * TY, (r3 / h) * TZ};
  const int tid = threadIdx.x;
  const int l[3] = {tid % TX, (tid / TX) % TY, tid / (TX * TY)};
  const int i = org[0] + l[0], j = org[1] + l[1], k = org[2] + l[2];
  const bool valid = (tid < TX * TY * TZ) && (i < bx.n[0]) && (j < bx.n[1]) && (k < bx.n[2]);
  const double* __restrict__ Pb = a.P + bx.cell_off;
  // Stage the tile's vertex metric in LDS: every face and cell of the tile reads
  // its vertices from this block.  Vertices past the box's last interior vertex
  // plane are not loaded (no valid cell or face of the tile reads them).
  {
    const GlobalVerts gv{a.alpha + bx.vert_off, SHIFT ? a.beta + bx.vert_off : nullptr, a.gamma + bx.vert_off,
                         a.vs};
    const int ng = bx.ng, VY = bx.VXY / bx.VX;
    for (int e = tid; e < G::NVB; e += 256) {
      const int vx = e % G::VBX, vy = (e / G::VBX) % G::VBY, vz = e / (G::VBX * G::VBY);
      if (org[0] + vx <= bx.n[0] && org[1] + vy <= bx.n[1] && org[2] + vz <= bx.n[2]) {
        const uint32_t v = ((org[2] + vz + ng) * VY + (org[1] + vy + ng)) * bx.VX + (org[0] + vx + ng);
#pragma unroll
        for (int f = 0; f < G::nvf(SHIFT); ++f) sV[f * G::NVB + e] = gv(f, v);
      }
    }
  }
  __syncthreads();
  // The cell's source terms first (the centre metric, its derivatives and
  // T^{mu nu}(P)), so that their temporaries are dead before the face phases; the
  // flux differences are then added to them (the oracle's order of summation).
  const int ng = bx.ng;
  const int c = ((k + ng) * (bx.NXY / bx.NX) + (j + ng)) * bx.NX + (i + ng);
  const uint32_t lv = l[0] + G::VBX * (l[1] + G::VBY * l[2]);
  const LdsVerts<G::NVB> vt{sV};
  double acc[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) acc[q] = 0.0;
  if (valid) {
    CentreMetric cm;
    centre_metric<SHIFT, true>(vt, lv, G::VBX, G::VBX * G::VBY, cm);
    MetricDeriv md;
    metric_deriv<SHIFT>(vt, lv, G::VBX, G::VBX * G::VBY, bx.inv_dx, md);
    double P[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) P[q] = ldg(Pb + q * a.cs, (uint32_t)c);
    sources_T<SHIFT>(cm, md, P, a.ph.gam, acc);
  }
  direction_phase<0, RECON, R, SHIFT, TX, TY, TZ, BF>(a, bx, Pb, sV, org, l, valid, sF, acc, rate);
  direction_phase<1, RECON, R, SHIFT, TX, TY, TZ, BF>(a, bx, Pb, sV, org, l, valid, sF, acc, rate);
  direction_phase<2, RECON, R, SHIFT, TX, TY, TZ, BF>(a, bx, Pb, sV, org, l, valid, sF, acc, rate);
  if (valid) {
    // The centre metric for con2prim.  FP64 faces: con2prim reads it from the
    // tile's LDS block before and after its Newton iteration instead of holding
    // it in registers across it, which removes the kernel's register spill (1.4%
    // faster at 256^3).  FP32 faces: computed here once (fetching it twice was 2%
    // slower there).
    CentreMetric cm;
    if constexpr (sizeof(R) != 8) centre_metric<false, false>(vt, lv, G::VBX, G::VBX * G::VBY, cm);
    double P[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) P[q] = ldg(Pb + q * a.cs, (uint32_t)c);
    if (a.mode == 0) {
#pragma unroll
      for (int q = 0; q < 8; ++q) stg(a.Uout + q * a.cs + bx.cell_off, (uint32_t)c, acc[q]);
    } else {
      double u[8];
      if (a.mode == 1) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const double un = ldg(a.Un + q * a.cs + bx.cell_off, (uint32_t)c);
          const double us = ldg(a.Us + q * a.cs + bx.cell_off, (uint32_t)c);
          u[q] = un + a.cstage * ((us - un) + a.dt * acc[q]);
        }
      } else {
        // classic RK4: the step's accumulator and the next stage state (or the step's end)
        double ac[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const double un = ldg(a.Un + q * a.cs + bx.cell_off, (uint32_t)c);
          const double prev = a.rk_first ? un : ldg(a.Acc + q * a.cs + bx.cell_off, (uint32_t)c);
          const double L = acc[q];
          ac[q] = prev + a.bdt * L;
          u[q] = a.rk_last ? ac[q] : un + a.adt * L;
        }
        if (!a.rk_last) {
#pragma unroll
          for (int q = 0; q < 8; ++q) stg(a.Acc + q * a.cs + bx.cell_off, (uint32_t)c, ac[q]);
        }
      }
      if (a.ckpt_in) {  // after the loads above (a store ahead of them would hold them back)
#pragma unroll
        for (int q = 0; q < 8; ++q) stg(a.ckpt_in + q * a.cs + bx.cell_off, (uint32_t)c, P[q]);
      }
      if (a.Pout) {
        // con2prim of the new state while it is in registers (the same routine,
        // inputs and metric as the con2prim kernel); an atmosphere reset
        // rewrites u as well
        int st;
        if constexpr (sizeof(R) == 8) {
          CentreMetric m1, m2;
          centre_metric<false, false>(vt, lv, G::VBX, G::VBX * G::VBY, m1);
          const auto refetch = [&](const double*& g, const double*& gi, double& sg) {
            centre_metric<false, false>(vt, lv, G::VBX, G::VBX * G::VBY, m2);
            g = m2.g;
            gi = m2.gi;
            sg = m2.sqrtg;
          };
          st = c2p_cell<true>(m1.g, m1.gi, m1.sqrtg, a.ph, u, P, &refetch);
        } else {
          st = c2p_cell(cm.g, cm.gi, cm.sqrtg, a.ph, u, P);
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) stg(a.Pout + q * a.cs + bx.cell_off, (uint32_t)c, P[q]);
        if (a.ckpt) {
#pragma unroll
          for (int q = 0; q < 8; ++q) stg(a.ckpt + q * a.cs + bx.cell_off, (uint32_t)c, P[q]);
        }
        fail += (st >= C2P_NOCONV && st <= C2P_NONFINITE) ? 1ull : 0ull;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) stg(a.Uout + q * a.cs + bx.cell_off, (uint32_t)c, u[q]);
    }
  }
}

// Waves per SIMD each stage-kernel instance is compiled for: without shift three
// (168 VGPRs with a spill of under 80 bytes; FP64 faces use the two-sided WENO,
// which made that possible), except WENO-Z with p = 2 in FP64 (which would spill
// ~300 bytes); with shift two.
template <typename R, bool SHIFT, int RECON> struct StageWaves {
  static constexpr int value = (!SHIFT && (sizeof(R) == 4 || RECON != RECON_WENOZ2)) ? 3 : 2;
};

// One workgroup per tile.  Workgroups are dispatched round-robin over the 8
// XCDs; each XCD gets a contiguous run of tiles so tiles sharing halos share an L2.
// BF: also store the transverse magnetic face fluxes (a.bflux, constrained transport).
template <int RECON, typename R, bool SHIFT, int TI, bool BF = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(StageWaves<R, SHIFT, RECON>::value))) void k_stage(StageArgs a) {
  using G = TileGeo<TILE_X[TI], TILE_Y[TI], TILE_Z[TI]>;
  __shared__ double sF[8][G::maxslots()];
  __shared__ double sV[G::nvf(SHIFT) * G::NVB];
  double rate = 0.0;
  unsigned long long fail = 0;
  stage_tile<RECON, R, SHIFT, TI, BF>(a, xcd_tile(blockIdx.x, gridDim.x), sF, sV, rate, fail);
  if (a.max_rate) block_max_atomic(rate, a.max_rate);
  if (a.n_fail) wave_count_atomic(fail, a.n_fail);
}

// Persistent workgroups: each pops tiles from the queue of its XCD (a
// contiguous tile range per XCD) until the range is exhausted.  The queue
// counters live in the workspace and are zeroed by k_reset_queue before the
// launch; every workgroup leaves the loop once its counter passes the range.
template <int RECON, typename R, bool SHIFT, int TI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(StageWaves<R, SHIFT, RECON>::value))) void k_stage_queue(StageArgs a, unsigned int* queue,
                                                                                                    int ntile) {
  using G = TileGeo<TILE_X[TI], TILE_Y[TI], TILE_Z[TI]>;
  __shared__ double sF[8][G::maxslots()];
  __shared__ double sV[G::nvf(SHIFT) * G::NVB];
  __shared__ int s_tile;
  const int x = blockIdx.x & 7;
  const int q = ntile >> 3, r = ntile & 7;
  const int lo = x * q + (x < r ? x : r);
  const int cnt = q + (x < r ? 1 : 0);
  double rate = 0.0;
  unsigned long long fail = 0;
  for (;;) {
    if (threadIdx.x == 0) s_tile = (int)atomicAdd(queue + x, 1u);
    __syncthreads();
    const int k = s_tile;
    __syncthreads();
    if (k >= cnt) break;
    stage_tile<RECON, R, SHIFT, TI>(a, lo + k, sF, sV, rate, fail);
  }
  if (a.max_rate) block_max_atomic(rate, a.max_rate);
  if (a.n_fail) wave_count_atomic(fail, a.n_fail);
}

__global__ void k_reset_queue(unsigned int* queue) {
  if (threadIdx.x < 8) queue[threadIdx.x] = 0u;
}

template <int RECON, typename R, bool SHIFT, int TI>
hipError_t launch_stage_t(const StageArgs& a, int64_t blocks, hipStream_t s) {
  if (a.queue) {
    hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(64), 0, s, a.queue);
    // one workgroup of 4 waves per SIMD-wave slot: waves per SIMD workgroups per CU
    const int64_t nb = std::min<int64_t>(blocks, (int64_t)a.persist_blocks * StageWaves<R, SHIFT, RECON>::value);
    hipLaunchKernelGGL((k_stage_queue<RECON, R, SHIFT, TI>), dim3((unsigned)nb), dim3(256), 0, s, a, a.queue,
                       (int)blocks);
  } else {
    hipLaunchKernelGGL((k_stage<RECON, R, SHIFT, TI>), dim3((unsigned)blocks), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

template <int RECON, typename R, bool SHIFT>
hipError_t launch_stage_r(const StageArgs& a, int64_t blocks, hipStream_t s) {
  if (a.bflux) {  // constrained transport: the 16x4x3 tile, one workgroup per tile
    hipLaunchKernelGGL((k_stage<RECON, R, SHIFT, CT_TILE, true>), dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
  }
  switch (a.tile) {
    case 0: return launch_stage_t<RECON, R, SHIFT, 0>(a, blocks, s);
    case 1: return launch_stage_t<RECON, R, SHIFT, 1>(a, blocks, s);
    case 2: return launch_stage_t<RECON, R, SHIFT, 2>(a, blocks, s);
    default: return launch_stage_t<RECON, R, SHIFT, 3>(a, blocks, s);
  }
}


}  // namespace

template <int RECON>
hipError_t launch_stage_recon(const StageArgs& a, int precision, int64_t blocks, hipStream_t s) {
  const bool sh = a.beta != nullptr;
  if (precision == GRMHD_MIXED)
    return sh ? launch_stage_r<RECON, float, true>(a, blocks, s) : launch_stage_r<RECON, float, false>(a, blocks, s);
  return sh ? launch_stage_r<RECON, double, true>(a, blocks, s) : launch_stage_r<RECON, double, false>(a, blocks, s);
}

}  // namespace gk
#endif  // GRMHD_STAGE_KERNELS
