// Device-side building blocks of the gfx950 GRMHD hot path (GRaM-X,
// arXiv:2210.17509): pointwise prim->cons, fluxes and wave speeds,
// reconstruction, HLLE, static-metric source terms and con2prim.
//
// R is the arithmetic type of reconstruction and HLLE (double, or float in the
// mixed-precision mode); everything else is double.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "grmhd.h"

namespace gk {

// ---------------------------------------------------------------- launch tables

constexpr int NTILE = GRMHD_NTILE;  // compiled stage-kernel tile shapes
constexpr int C2P_BLOCK = 256;

// Per-box data the kernels read (derived on the host from grmhd_box).
struct KBox {
  int32_t n[3];
  int32_t ng;
  int32_t NX, NXY;  // storage cell strides (x, xy) including ghosts
  int32_t VX, VXY;  // vertex strides
  int64_t cell_off, vert_off;
  double inv_dx[3];
  int32_t mlo[3][3];  // interior index read for ghost coordinates -3, -2, -1
  int32_t mhi[3][3];  // interior index read for coordinates n, n+1, n+2
  int32_t pad[2];
};
static_assert(sizeof(KBox) % 8 == 0, "KBox alignment");

constexpr int FACE_BLOCK = 256;
// face-adjoint blocks of y and z faces: patches of ADJ_PX faces along x by ADJ_PD
// along the face direction (ADJ_PX * ADJ_PD = FACE_BLOCK); their stencils reach
// ADJ_ROWS cell rows along that direction
constexpr int ADJ_PX = 32, ADJ_PD = 8, ADJ_ROWS = ADJ_PD + 5;
static_assert(ADJ_PX * ADJ_PD == FACE_BLOCK, "one face per thread");

struct TableHeader {
  uint64_t magic;
  uint64_t hash;
  int32_t nbox;
  int32_t pad;
  int64_t c2p_blocks;
  int64_t tiles[NTILE];
  int64_t face_blocks[3];
  int64_t vert_blocks;
};

// Device table: header | KBox[nbox] | int32 c2p_prefix[nbox+1] | int32 tile_prefix[NTILE][nbox+1]
//               | int32 face_prefix[3][nbox+1] | int32 vert_prefix[nbox+1]
struct Table {
  const KBox* box;
  const int32_t* c2p_prefix;
  const int32_t* tile_prefix;  // [NTILE][nbox+1]
  const int32_t* face_prefix;  // [3][nbox+1], face-adjoint blocks per direction (x: FACE_BLOCK faces; y, z: patches)
  const int32_t* vert_prefix;  // blocks of C2P_BLOCK interior vertex points (n+1 per axis)
  int32_t nbox;
};

__device__ __forceinline__ int find_box(const int32_t* prefix, int nbox, int blk) {
  int lo = 0, hi = nbox;  // prefix[lo] <= blk < prefix[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (prefix[mid] <= blk) lo = mid; else hi = mid;
  }
  return lo;
}

// ---------------------------------------------------------------- physics constants

struct KPhys {
  double gam, gm1, gf;      // Gamma, Gamma - 1, Gamma / (Gamma - 1)
  double weno_eps, wenoz_eps;
  double c2p_tol;
  double rho_atm, p_atm, eps_atm;
  double rho_floor;  // densities below rho_atm (1 + 1e-6) are the atmosphere
  int32_t c2p_maxit, wenoz_p;
};

// ---------------------------------------------------------------- small helpers

template <typename R> __device__ __forceinline__ R rsq(R x) { return x * x; }

// Reciprocal: the hardware estimate refined by two Newton-Raphson steps
// r <- r (2 - x r) (FP64; one step for FP32), within an ulp or two of 1/x for
// the finite, non-zero, normal arguments the kernels divide by.
__device__ __forceinline__ double rcp_r(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float rcp_r(float x) {
  float r = __builtin_amdgcn_rcpf(x);
  float e = __builtin_fmaf(-x, r, 1.0f);
  return __builtin_fmaf(r, e, r);
}

// Loads and stores through a uniform base pointer and an unsigned 32-bit
// element index, so the address is base + 32-bit byte offset.
__device__ __forceinline__ double ldg(const double* __restrict__ base, uint32_t i) {
  return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(base) + (i << 3));
}
__device__ __forceinline__ void stg(double* __restrict__ base, uint32_t i, double v) {
  *reinterpret_cast<double*>(reinterpret_cast<char*>(base) + (i << 3)) = v;
}
// Square root of a finite x >= 0 (normal or zero): the hardware 1/sqrt estimate
// refined by Goldschmidt's iteration (g -> sqrt(x), h -> 1/(2 sqrt(x))) and a
// final Newton correction; within an ulp or two of sqrt(x).
__device__ __forceinline__ double sqrt_r(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  double r = __builtin_fma(-h, g, 0.5);
  g = __builtin_fma(g, r, g);
  h = __builtin_fma(h, r, h);
  r = __builtin_fma(-h, g, 0.5);
  g = __builtin_fma(g, r, g);
  h = __builtin_fma(h, r, h);
  const double d = __builtin_fma(-g, g, x);
  g = __builtin_fma(d, h, g);
  return x > 0.0 ? g : 0.0;
}
__device__ __forceinline__ float sqrt_r(float x) { return sqrtf(x); }
template <typename R> __device__ __forceinline__ R rmax(R a, R b) { return a < b ? b : a; }
template <typename R> __device__ __forceinline__ R rmin(R a, R b) { return b < a ? b : a; }
template <typename R> __device__ __forceinline__ R rabs(R a) { return a < R(0) ? -a : a; }

// symmetric 3x3 storage: xx xy xz yy yz zz
__device__ __forceinline__ constexpr int sidx(int i, int j) {
  return (i == 0) ? j : (i == 1 ? (j == 0 ? 1 : j + 2) : (j == 0 ? 2 : (j == 1 ? 4 : 5)));
}

// ---------------------------------------------------------------- vertex metric access

// Vertex fields: 0 = alpha, 1..6 = gamma_ij (xx xy xz yy yz zz), 7..9 = beta^i.
constexpr int VF_ALPHA = 0, VF_GAMMA = 1, VF_BETA = 7;

// The vertex metric of one box in HBM: field f of the vertex with box-local
// storage index v.
struct GlobalVerts {
  const double* __restrict__ alpha;
  const double* __restrict__ beta;
  const double* __restrict__ gamma;
  int64_t vs;
  __device__ __forceinline__ double operator()(int f, uint32_t v) const {
    if (f == VF_ALPHA) return ldg(alpha, v);
    if (f < VF_BETA) return ldg(gamma + (f - VF_GAMMA) * vs, v);
    return ldg(beta + (f - VF_BETA) * vs, v);
  }
};

// A block of vertices staged in LDS: field f of block-local vertex v at s[f * STRIDE + v].
template <int STRIDE> struct LdsVerts {
  const double* s;
  __device__ __forceinline__ double operator()(int f, uint32_t v) const { return s[f * STRIDE + v]; }
};

// ---------------------------------------------------------------- face metric

template <typename R> struct FaceMetric {
  R alpha, ialpha, beta[3], g[6], sqrtg, gdd;
};

// Mean of the four vertices of the low face (direction D) of the cell whose
// lower corner is vertex vb (sa, sb: vertex strides of the two other axes):
// the metric is interpolated linearly from the vertices to the face centre
// (Sec. II C).
template <int D, bool SHIFT, typename R, typename V>
__device__ __forceinline__ void face_metric(const V& vt, uint32_t vb, uint32_t sa, uint32_t sb, FaceMetric<R>& m) {
  const uint32_t v0 = vb, v1 = vb + sa, v2 = vb + sb, v3 = vb + sa + sb;
  auto avg = [&](int f) -> double { return 0.25 * ((vt(f, v0) + vt(f, v1)) + (vt(f, v2) + vt(f, v3))); };
  double g[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) g[q] = avg(VF_GAMMA + q);
  const double al = avg(VF_ALPHA);
  m.alpha = (R)al;
  m.ialpha = (R)rcp_r(al);
#pragma unroll
  for (int q = 0; q < 3; ++q) m.beta[q] = SHIFT ? (R)avg(VF_BETA + q) : R(0);
  // cofactors: det and the one inverse component gamma^{DD}
  const double cxx = g[3] * g[5] - g[4] * g[4];
  const double cxy = g[2] * g[4] - g[1] * g[5];
  const double cxz = g[1] * g[4] - g[2] * g[3];
  const double det = g[0] * cxx + g[1] * cxy + g[2] * cxz;
  double cdd;
  if (D == 0) cdd = cxx;
  else if (D == 1) cdd = g[0] * g[5] - g[2] * g[2];
  else cdd = g[0] * g[3] - g[1] * g[1];
#pragma unroll
  for (int q = 0; q < 6; ++q) m.g[q] = (R)g[q];
  m.sqrtg = (R)sqrt_r(det);
  m.gdd = (R)(cdd * rcp_r(det));
}

// ---------------------------------------------------------------- one side of a face

// Derived quantities of a primitive state at a face, Eqs. (p2c1)-(p2c4):
// W, v_i, B_i, alpha b^0 = W B.v, b^2 = (B^2 + (alpha b^0)^2) / W^2, Gamma law.
template <typename R> struct SideState {
  R vlow[3], Blow[3];
  R v2, iW, W, B2, ab0, b2, p, rhoh;
};

template <typename R, typename RM>
__device__ __forceinline__ void side_v2(const FaceMetric<RM>& m, const R* P, SideState<R>& s) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
    s.vlow[i] = m.g[sidx(i, 0)] * P[1] + m.g[sidx(i, 1)] * P[2] + m.g[sidx(i, 2)] * P[3];
  s.v2 = s.vlow[0] * P[1] + s.vlow[1] * P[2] + s.vlow[2] * P[3];
}

template <typename R> __device__ __forceinline__ bool side_ok(const R* P, R v2) {
  bool fin = true;
#pragma unroll
  // an exact class test: "x - x == 0" is not one under FMA contraction, which
  // can turn it into fma(a, b, -x) = the rounding error of a product x = a b
  for (int q = 0; q < 8; ++q) fin = fin && __builtin_isfinite(P[q]);
  return fin && (P[0] > R(0)) && (P[4] > R(0)) && (v2 < R(1));
}

template <typename R, typename RM>
__device__ __forceinline__ void side_rest(const FaceMetric<RM>& m, const R* P, RM gm1, SideState<R>& s) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
    s.Blow[i] = m.g[sidx(i, 0)] * P[5] + m.g[sidx(i, 1)] * P[6] + m.g[sidx(i, 2)] * P[7];
  s.iW = sqrt_r(R(1) - s.v2);
  s.W = rcp_r(s.iW);
  s.B2 = s.Blow[0] * P[5] + s.Blow[1] * P[6] + s.Blow[2] * P[7];
  const R Bv = s.Blow[0] * P[1] + s.Blow[1] * P[2] + s.Blow[2] * P[3];
  s.ab0 = s.W * Bv;
  s.b2 = (s.B2 + s.ab0 * s.ab0) * (s.iW * s.iW);
  s.p = gm1 * P[0] * P[4];
  s.rhoh = P[0] * (R(1) + P[4]) + s.p;
}

// Bounds of the characteristic speeds in direction D: the 3+1 hydrodynamic
// eigenvalues with the sound speed replaced by the fast magnetosonic bound
// c_f^2 = c_s^2 + c_a^2 - c_s^2 c_a^2.
template <int D, typename R, typename RM>
__device__ __forceinline__ void side_speeds(const FaceMetric<RM>& m, const R* P, const SideState<R>& s, RM gam, R& lp,
                                            R& lm) {
  const R rh = s.rhoh, rhb = s.rhoh + s.b2;
  const R ir = rcp_r(rh * rhb);  // one reciprocal for c_s^2 and c_a^2
  const R cs2 = gam * s.p * rhb * ir;
  const R ca2 = s.b2 * rh * ir;
  const R cf2 = cs2 + ca2 - cs2 * ca2;
  const R vd = P[1 + D];
  const R den = R(1) - s.v2 * cf2;
  const R disc = (R(1) - s.v2) * (m.gdd * den - vd * vd * (R(1) - cf2));
  const R root = sqrt_r(cf2 * rmax(disc, R(0)));
  const R base = vd * (R(1) - cf2);
  const R ad = R(m.alpha) * rcp_r(den);
  lp = ad * (base + root) - m.beta[D];
  lm = ad * (base - root) - m.beta[D];
}

// Conserved variables and the direction-D flux, Eqs. (p2c1)-(p2c4) and
// (definition-of-flux) with v~ = v - beta / alpha.
template <int D, typename R, typename RM>
__device__ __forceinline__ void side_cons_flux(const FaceMetric<RM>& m, const R* P, const SideState<R>& s, R U[8],
                                               R F[8]) {
  const RM sg = m.sqrtg;
  const R W2 = s.W * s.W;
  const R rhohs = s.rhoh + s.b2;
  const R Ps = s.p + R(0.5) * s.b2;
  R blow[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) blow[i] = s.Blow[i] * s.iW + s.ab0 * s.vlow[i];
  U[0] = sg * P[0] * s.W;
#pragma unroll
  for (int j = 0; j < 3; ++j) U[1 + j] = sg * (rhohs * W2 * s.vlow[j] - s.ab0 * blow[j]);
  U[4] = sg * (rhohs * W2 - Ps - s.ab0 * s.ab0) - U[0];
#pragma unroll
  for (int k = 0; k < 3; ++k) U[5 + k] = sg * P[5 + k];
  const RM a = m.alpha;
  const RM ia = m.ialpha;
  R vt[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) vt[i] = P[1 + i] - m.beta[i] * ia;
  const R BnW = U[5 + D] * s.iW;
  F[0] = a * (U[0] * vt[D]);
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    R t = U[1 + j] * vt[D] - blow[j] * BnW;
    if (j == D) t = t + sg * Ps;
    F[1 + j] = a * t;
  }
  F[4] = a * (U[4] * vt[D] + sg * Ps * P[1 + D] - s.ab0 * BnW);
#pragma unroll
  for (int k = 0; k < 3; ++k) F[5 + k] = (k == D) ? R(0) : a * (U[5 + k] * vt[D] - U[5 + D] * vt[k]);
}

// ---------------------------------------------------------------- reconstruction

// TVD minmod [Toro]: slope of the centre cell, 0 at extrema.
template <typename R> __device__ __forceinline__ R minmod(R a, R b) {
  return (a * b <= R(0)) ? R(0) : (rabs(a) < rabs(b) ? a : b);
}

// Un-normalised WENO5 weights from the smoothness indicators [Shu 98]:
// Jiang-Shu d_k / (eps + beta_k)^2 (ZW = false) or Borges WENO-Z
// d_k (1 + (|beta_0 - beta_2| / (beta_k + eps))^p) (ZW = true), each multiplied
// by a common positive factor (which the normalisation removes) so that no
// division is needed in FP64.
template <bool ZW, typename R>
__device__ __forceinline__ void weno5_weights(R b0, R b1, R b2, R eps, int zp, R& w0, R& w1, R& w2) {
  if (!ZW) {
    const R t0 = rsq(eps + b0), t1 = rsq(eps + b1), t2 = rsq(eps + b2);
    w0 = R(0.1) * (t1 * t2);
    w1 = R(0.6) * (t0 * t2);
    w2 = R(0.3) * (t0 * t1);
  } else {
    const R tau = rabs(b0 - b2);
    const R e0 = b0 + eps, e1 = b1 + eps, e2 = b2 + eps;
    if (sizeof(R) == 8) {
      if (zp == 2) {
        const R s0 = e0 * e0, s1 = e1 * e1, s2 = e2 * e2, t2 = tau * tau;
        w0 = R(0.1) * (s0 + t2) * (s1 * s2);
        w1 = R(0.6) * (s1 + t2) * (s0 * s2);
        w2 = R(0.3) * (s2 + t2) * (s0 * s1);
      } else {
        w0 = R(0.1) * (e0 + tau) * (e1 * e2);
        w1 = R(0.6) * (e1 + tau) * (e0 * e2);
        w2 = R(0.3) * (e2 + tau) * (e0 * e1);
      }
    } else {  // FP32: the products of tiny eps could underflow, divide per weight
      R r0 = tau / e0, r1 = tau / e1, r2 = tau / e2;
      if (zp == 2) { r0 *= r0; r1 *= r1; r2 *= r2; }
      w0 = R(0.1) * (R(1) + r0);
      w1 = R(0.6) * (R(1) + r1);
      w2 = R(0.3) * (R(1) + r2);
    }
  }
}

// WENO5 value at the right face of the centre cell c of (a, b, c, d, e).
// ZPC = 1 or 2 fixes the WENO-Z exponent at compile time; ZPC = 0 takes it from zp.
template <bool ZW, int ZPC = 0, typename R>
__device__ __forceinline__ R weno5(R a, R b, R c, R d, R e, R eps, int zp) {
  if (ZPC != 0) zp = ZPC;
  const R q0 = R(2) * a - R(7) * b + R(11) * c;  // x6
  const R q1 = -b + R(5) * c + R(2) * d;
  const R q2 = R(2) * c + R(5) * d - e;
  const R b0 = R(13.0 / 12.0) * rsq(a - R(2) * b + c) + R(0.25) * rsq(a - R(4) * b + R(3) * c);
  const R b1 = R(13.0 / 12.0) * rsq(b - R(2) * c + d) + R(0.25) * rsq(b - d);
  const R b2 = R(13.0 / 12.0) * rsq(c - R(2) * d + e) + R(0.25) * rsq(R(3) * c - R(4) * d + e);
  R w0, w1, w2;
  weno5_weights<ZW>(b0, b1, b2, eps, zp, w0, w1, w2);
  return (w0 * q0 + w1 * q1 + w2 * q2) * rcp_r(R(6) * (w0 + w1 + w2));
}

// Both WENO5 values at the face between cells s[2] and s[3] of the six-cell
// stencil s[0..5]: PL from (s0, .., s4), PR from the mirrored (s5, .., s1).
// The two sides share two of their three candidate values (q1 of one side is q2
// of the other) and two of their three second differences (those over cells
// 1..3 and 2..4).  In FP64 one reciprocal serves both normalisations while
// the product of the two denominators stays well inside the exponent range
// (not for WENO-Z with p = 2, whose denominators can reach 1e-240); FP32 takes
// one refined reciprocal per side.
template <bool ZW, int ZPC = 0, typename R>
__device__ __forceinline__ void weno5_lr(const R* s, R eps, int zp, R& PL, R& PR) {
  if (ZPC != 0) zp = ZPC;
  const R qa = R(2) * s[0] - R(7) * s[1] + R(11) * s[2];  // x6: q0 of L
  const R qb = -s[1] + R(5) * s[2] + R(2) * s[3];          // q1 of L, q2 of R
  const R qc = R(2) * s[2] + R(5) * s[3] - s[4];           // q2 of L, q1 of R
  const R qd = R(2) * s[5] - R(7) * s[4] + R(11) * s[3];  // q0 of R
  const R c13 = R(13.0 / 12.0);
  const R E1 = c13 * rsq(s[1] - R(2) * s[2] + s[3]);
  const R E2 = c13 * rsq(s[2] - R(2) * s[3] + s[4]);
  const R bL0 = c13 * rsq(s[0] - R(2) * s[1] + s[2]) + R(0.25) * rsq(s[0] - R(4) * s[1] + R(3) * s[2]);
  const R bL1 = E1 + R(0.25) * rsq(s[1] - s[3]);
  const R bL2 = E2 + R(0.25) * rsq(R(3) * s[2] - R(4) * s[3] + s[4]);
  const R bR0 = c13 * rsq(s[5] - R(2) * s[4] + s[3]) + R(0.25) * rsq(s[5] - R(4) * s[4] + R(3) * s[3]);
  const R bR1 = E2 + R(0.25) * rsq(s[4] - s[2]);
  const R bR2 = E1 + R(0.25) * rsq(R(3) * s[3] - R(4) * s[2] + s[1]);
  R l0, l1, l2, r0, r1, r2;
  weno5_weights<ZW>(bL0, bL1, bL2, eps, zp, l0, l1, l2);
  weno5_weights<ZW>(bR0, bR1, bR2, eps, zp, r0, r1, r2);
  const R nL = l0 * qa + l1 * qb + l2 * qc, dL = R(6) * (l0 + l1 + l2);
  const R nR = r0 * qd + r1 * qc + r2 * qb, dR = R(6) * (r0 + r1 + r2);
  if constexpr (sizeof(R) == 4) {
    // FP32: a refined reciprocal per side (the product of the two denominators
    // could leave the FP32 range)
    PL = nL * rcp_r(dL);
    PR = nR * rcp_r(dR);
  } else {
    const R prod = dL * dR;
    if (!(ZW && zp == 2) && prod > R(1e-300) && prod < R(1e300)) {
      const R inv = rcp_r(prod);
      PL = nL * (dR * inv);
      PR = nR * (dL * inv);
    } else {
      PL = nL / dL;
      PR = nR / dR;
    }
  }
}

// ---------------------------------------------------------------- HLLE

// F* = (xi+ F_L - xi- F_R + xi+ xi- (U_R - U_L)) / (xi+ - xi-), xi+ = max(0, lambda+),
// xi- = min(0, lambda-) over both sides [Harten-Lax-van Leer, Einfeldt].
template <int D, typename R>
__device__ __forceinline__ void hlle(const FaceMetric<R>& m, const R* PL, const SideState<R>& sL, const R* PR,
                                     const SideState<R>& sR, R gam, R Fs[8], R& xip, R& xim) {
  R lpL, lmL, lpR, lmR;
  side_speeds<D>(m, PL, sL, gam, lpL, lmL);
  side_speeds<D>(m, PR, sR, gam, lpR, lmR);
  xip = rmax(R(0), rmax(lpL, lpR));
  xim = rmin(R(0), rmin(lmL, lmR));
  const R den = xip - xim;
  R UL[8], FL[8], UR[8], FR[8];
  side_cons_flux<D>(m, PL, sL, UL, FL);
  side_cons_flux<D>(m, PR, sR, UR, FR);
  if (den > R(0)) {
    const R id = rcp_r(den);
    const R xx = xip * xim;
#pragma unroll
    for (int q = 0; q < 8; ++q) Fs[q] = (xip * FL[q] - xim * FR[q] + xx * (UR[q] - UL[q])) * id;
  } else {
#pragma unroll
    for (int q = 0; q < 8; ++q) Fs[q] = R(0.5) * (FL[q] + FR[q]);
  }
}

// ---------------------------------------------------------------- centre metric and sources

struct CentreMetric {
  double alpha, beta[3], g[6], gi[6], sqrtg;
};

// Inverse spatial metric and sqrt(gamma) from the centre gamma_ij.
__device__ __forceinline__ void centre_inverse(CentreMetric& m) {
  const double* g = m.g;
  const double cxx = g[3] * g[5] - g[4] * g[4];
  const double cxy = g[2] * g[4] - g[1] * g[5];
  const double cxz = g[1] * g[4] - g[2] * g[3];
  const double cyy = g[0] * g[5] - g[2] * g[2];
  const double cyz = g[1] * g[2] - g[0] * g[4];
  const double czz = g[0] * g[3] - g[1] * g[1];
  const double det = g[0] * cxx + g[1] * cxy + g[2] * cxz;
  const double id = rcp_r(det);
  m.gi[0] = cxx * id; m.gi[1] = cxy * id; m.gi[2] = cxz * id;
  m.gi[3] = cyy * id; m.gi[4] = cyz * id; m.gi[5] = czz * id;
  m.sqrtg = sqrt_r(det);
}

// Cell-centre metric: mean of the cell's 8 vertices; inverse and sqrt(gamma)
// from the averaged gamma_ij.
template <bool SHIFT, bool NEED_ALPHA, typename V>
__device__ __forceinline__ void centre_metric(const V& vt, uint32_t vb, uint32_t VX, uint32_t VXY, CentreMetric& m) {
  const uint32_t o[8] = {0u, 1u, VX, VX + 1u, VXY, VXY + 1u, VXY + VX, VXY + VX + 1u};
  const uint32_t v = vb;
  auto avg = [&](int f) -> double {
    return 0.125 * (((vt(f, v + o[0]) + vt(f, v + o[1])) + (vt(f, v + o[2]) + vt(f, v + o[3]))) +
                    ((vt(f, v + o[4]) + vt(f, v + o[5])) + (vt(f, v + o[6]) + vt(f, v + o[7]))));
  };
#pragma unroll
  for (int q = 0; q < 6; ++q) m.g[q] = avg(VF_GAMMA + q);
  m.alpha = NEED_ALPHA ? avg(VF_ALPHA) : 1.0;
#pragma unroll
  for (int q = 0; q < 3; ++q) m.beta[q] = SHIFT ? avg(VF_BETA + q) : 0.0;
  centre_inverse(m);
}

// d_e f at the cell centre: mean over the 4 edges along e of the vertex
// difference, times 1/dx_e (second order).
template <typename V>
__device__ __forceinline__ double edge_deriv(const V& vt, int f, uint32_t v, uint32_t e, uint32_t a, uint32_t b,
                                             double idx) {
  const double s0 = vt(f, v + e) - vt(f, v);
  const double s1 = vt(f, v + a + e) - vt(f, v + a);
  const double s2 = vt(f, v + b + e) - vt(f, v + b);
  const double s3 = vt(f, v + a + b + e) - vt(f, v + a + b);
  return 0.25 * ((s0 + s1) + (s2 + s3)) * idx;
}

// First derivatives of the vertex metric at a cell centre.
struct MetricDeriv {
  double da[3], dg[3][6], db[3][3];
};

template <bool SHIFT, typename V>
__device__ __forceinline__ void metric_deriv(const V& vt, uint32_t vb, uint32_t VX, uint32_t VXY,
                                             const double* inv_dx, MetricDeriv& md) {
  const uint32_t st[3] = {1u, VX, VXY};
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const uint32_t se = st[e], sa = st[(e + 1) % 3], sb = st[(e + 2) % 3];
    md.da[e] = edge_deriv(vt, VF_ALPHA, vb, se, sa, sb, inv_dx[e]);
#pragma unroll
    for (int q = 0; q < 6; ++q) md.dg[e][q] = edge_deriv(vt, VF_GAMMA + q, vb, se, sa, sb, inv_dx[e]);
#pragma unroll
    for (int q = 0; q < 3; ++q) md.db[e][q] = SHIFT ? edge_deriv(vt, VF_BETA + q, vb, se, sa, sb, inv_dx[e]) : 0.0;
  }
}

// The cell's 8 vertex values of one field, addressed like a vertex block with
// strides 1, 2, 4.
struct OneCorner {
  double c[8];
  __device__ __forceinline__ double operator()(int, uint32_t k) const { return c[k]; }
};

// Centre metric (as centre_metric) and its first derivatives (as metric_deriv)
// from global vertices, one field at a time, so only one field's 8 vertices are
// live at once.
template <bool SHIFT, typename V>
__device__ __forceinline__ void centre_metric_deriv(const V& vt, uint32_t vb, uint32_t VX, uint32_t VXY,
                                                    const double* inv_dx, CentreMetric& m, MetricDeriv& md) {
  const uint32_t o[8] = {0u, 1u, VX, VX + 1u, VXY, VXY + 1u, VXY + VX, VXY + VX + 1u};
  auto field = [&](int f, double& mean, double* d) {
    OneCorner w;
#pragma unroll
    for (int k = 0; k < 8; ++k) w.c[k] = vt(f, vb + o[k]);
    mean = 0.125 * (((w.c[0] + w.c[1]) + (w.c[2] + w.c[3])) + ((w.c[4] + w.c[5]) + (w.c[6] + w.c[7])));
#pragma unroll
    for (int e = 0; e < 3; ++e)
      d[e] = edge_deriv(w, 0, 0u, 1u << e, 1u << ((e + 1) % 3), 1u << ((e + 2) % 3), inv_dx[e]);
  };
  double d[3];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    field(VF_GAMMA + q, m.g[q], d);
#pragma unroll
    for (int e = 0; e < 3; ++e) md.dg[e][q] = d[e];
  }
  field(VF_ALPHA, m.alpha, md.da);
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    if (SHIFT) {
      field(VF_BETA + q, m.beta[q], d);
#pragma unroll
      for (int e = 0; e < 3; ++e) md.db[e][q] = d[e];
    } else {
      m.beta[q] = 0.0;
#pragma unroll
      for (int e = 0; e < 3; ++e) md.db[e][q] = 0.0;
    }
  }
  centre_inverse(m);
}

// T^{mu nu} of Eq. (mhd-stress-energy-tensor) at a cell centre from the
// 4-velocity and the magnetic 4-vector: T00, T^{0i} and T^{ij} (symmetric
// storage).  T = double, or a dual number.
template <typename T>
__device__ __forceinline__ void tmunu_T(const CentreMetric& m, const T* P, double gam, T& T00, T T0[3], T Tij[6]) {
  T vlow[3], Blow[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    vlow[i] = m.g[sidx(i, 0)] * P[1] + m.g[sidx(i, 1)] * P[2] + m.g[sidx(i, 2)] * P[3];
    Blow[i] = m.g[sidx(i, 0)] * P[5] + m.g[sidx(i, 1)] * P[6] + m.g[sidx(i, 2)] * P[7];
  }
  const T v2 = vlow[0] * P[1] + vlow[1] * P[2] + vlow[2] * P[3];
  const T iW = sqrt_r(T(1.0) - v2);
  const T W = T(1.0) / iW;
  const T B2 = Blow[0] * P[5] + Blow[1] * P[6] + Blow[2] * P[7];
  const T Bv = Blow[0] * P[1] + Blow[1] * P[2] + Blow[2] * P[3];
  const double ia = 1.0 / m.alpha;
  const T b0 = W * Bv * ia;
  const T b2 = B2 * (iW * iW) + Bv * Bv;
  const T p = (gam - 1.0) * P[0] * P[4];
  const T rhohs = P[0] * (T(1.0) + P[4]) + p + b2;
  const T Ps = p + T(0.5) * b2;
  const T u0 = W * ia;
  T u[3], b[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    u[i] = W * (P[1 + i] - m.beta[i] * ia);
    b[i] = (P[5 + i] + m.alpha * b0 * u[i]) * iW;
  }
  const double ia2 = ia * ia;
  T00 = rhohs * u0 * u0 - Ps * ia2 - b0 * b0;
#pragma unroll
  for (int i = 0; i < 3; ++i) T0[i] = rhohs * u0 * u[i] + Ps * (m.beta[i] * ia2) - b0 * b[i];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j)
      Tij[sidx(i, j)] = rhohs * u[i] * u[j] + Ps * (m.gi[sidx(i, j)] - m.beta[i] * m.beta[j] * ia2) - b[i] * b[j];
}

// Static-metric source terms of Eq. (definition-of-source) in 3+1 form:
//   S_Sj  = alpha sqrt(g) [T^00 (beta^i beta^k d_j g_ik / 2 - alpha d_j alpha)
//           + T^0i beta^k d_j g_ik + T^0_i d_j beta^i + T^ik d_j g_ik / 2]
//   S_tau = alpha sqrt(g) [T^00 (beta^i beta^j K_ij - beta^i d_i alpha)
//           + T^0i (2 beta^j K_ij - d_i alpha) + T^ij K_ij]
// with K_ij = (gamma_jk d_i beta^k + gamma_ik d_j beta^k + beta^k d_k gamma_ij) / (2 alpha)
// for a time-independent slice; S_D = S_B = 0.  The sources are linear in
// T^{mu nu} for a fixed metric.  T = double, or a dual number for the adjoint.
template <bool SHIFT, typename T>
__device__ __forceinline__ void sources_tail(const CentreMetric& m, const MetricDeriv& md, const T& T00, const T* T0,
                                             const T* Tij, T S[8]) {
  const double* da = md.da;
  const double ia = 1.0 / m.alpha;
  const double as = m.alpha * m.sqrtg;
  S[0] = T(0.0);
  S[5] = S[6] = S[7] = T(0.0);
  if (!SHIFT) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      T tdg = T(0.0);
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) tdg = tdg + Tij[sidx(i, k)] * md.dg[j][sidx(i, k)];
      S[1 + j] = as * (T(0.5) * tdg - m.alpha * T00 * da[j]);
    }
    S[4] = -as * (T0[0] * da[0] + T0[1] * da[1] + T0[2] * da[2]);
  } else {
    const double* be = m.beta;
    double blw[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) blw[i] = m.g[sidx(i, 0)] * be[0] + m.g[sidx(i, 1)] * be[1] + m.g[sidx(i, 2)] * be[2];
    T T0low[3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
      T0low[i] = T00 * blw[i] + T0[0] * m.g[sidx(0, i)] + T0[1] * m.g[sidx(1, i)] + T0[2] * m.g[sidx(2, i)];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double bbdg = 0.0;
      T tdg = T(0.0), t0bdg = T(0.0), t0db = T(0.0);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        t0db = t0db + T0low[i] * md.db[j][i];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const double dgik = md.dg[j][sidx(i, k)];
          bbdg += be[i] * be[k] * dgik;
          tdg = tdg + Tij[sidx(i, k)] * dgik;
          t0bdg = t0bdg + T0[i] * (be[k] * dgik);
        }
      }
      S[1 + j] = as * (T00 * (0.5 * bbdg - m.alpha * da[j]) + t0bdg + t0db + T(0.5) * tdg);
    }
    double K[6];
    const double i2a = 0.5 * ia;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k)
          t += m.g[sidx(j, k)] * md.db[i][k] + m.g[sidx(i, k)] * md.db[j][k] + be[k] * md.dg[k][sidx(i, j)];
        K[sidx(i, j)] = t * i2a;
      }
    double bbK = 0.0, bda = 0.0;
    T t0i = T(0.0), tK = T(0.0);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      bda += be[i] * da[i];
      double bK = 0.0;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        bbK += be[i] * be[j] * K[sidx(i, j)];
        bK += be[j] * K[sidx(i, j)];
        tK = tK + Tij[sidx(i, j)] * K[sidx(i, j)];
      }
      t0i = t0i + T0[i] * (2.0 * bK - da[i]);
    }
    S[4] = as * (T00 * (bbK - bda) + t0i + tK);
  }
}

template <bool SHIFT, typename T>
__device__ __forceinline__ void sources_T(const CentreMetric& m, const MetricDeriv& md, const T* P, double gam,
                                          T S[8]) {
  T T00, T0[3], Tij[6];
  tmunu_T(m, P, gam, T00, T0, Tij);
  sources_tail<SHIFT>(m, md, T00, T0, Tij, S);
}

// ---------------------------------------------------------------- prim -> cons at a cell

// Eqs. (p2c1)-(p2c4) at a cell centre; T = double, or a dual number for the
// Jacobian dU/dP used by the adjoint.
template <typename T>
__device__ __forceinline__ void p2c_cell(const double* g, double sqrtg, double gm1, const T* P, T U[8]) {
  T vlow[3], Blow[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    vlow[i] = g[sidx(i, 0)] * P[1] + g[sidx(i, 1)] * P[2] + g[sidx(i, 2)] * P[3];
    Blow[i] = g[sidx(i, 0)] * P[5] + g[sidx(i, 1)] * P[6] + g[sidx(i, 2)] * P[7];
  }
  const T v2 = vlow[0] * P[1] + vlow[1] * P[2] + vlow[2] * P[3];
  const T iW = sqrt_r(T(1.0) - v2);
  const T W = T(1.0) / iW;
  const T B2 = Blow[0] * P[5] + Blow[1] * P[6] + Blow[2] * P[7];
  const T Bv = Blow[0] * P[1] + Blow[1] * P[2] + Blow[2] * P[3];
  const T ab0 = W * Bv;
  const T b2 = (B2 + ab0 * ab0) * (iW * iW);
  const T p = gm1 * P[0] * P[4];
  const T rhohs = P[0] * (T(1.0) + P[4]) + p + b2;
  const T Ps = p + T(0.5) * b2;
  const T W2 = W * W;
  U[0] = sqrtg * P[0] * W;
#pragma unroll
  for (int j = 0; j < 3; ++j) U[1 + j] = sqrtg * (rhohs * W2 * vlow[j] - ab0 * (Blow[j] * iW + ab0 * vlow[j]));
  U[4] = sqrtg * (rhohs * W2 - Ps - ab0 * ab0) - U[0];
#pragma unroll
  for (int k = 0; k < 3; ++k) U[5 + k] = sqrtg * P[5 + k];
}

// ---------------------------------------------------------------- con2prim (FP64)

enum { C2P_OK = 0, C2P_FLOOR = 1, C2P_NOCONV = 2, C2P_UNPHYS = 3, C2P_NONFINITE = 4, C2P_FALLBACK = 5 };

struct C2PIn {
  double Dt, St[3], taut, B[3];
  double S2, B2, SB;
};

// Finite (not inf, not NaN), by the exponent class; contraction-proof (see side_ok).
__device__ __forceinline__ bool dfinite(double x) { return __builtin_isfinite(x); }

// 3D Newton-Raphson in (W, z = rho h W^2, T = p / rho) (Sec. II C).  With
// B.v = S.B / z and S_j = (z + B^2) v_j - (B.v) B_j the three equations are
//   f1 = S^2 - (z + B^2)^2 (1 - 1/W^2) + (S.B)^2 (2 z + B^2) / z^2
//   f2 = tau + D - z - B^2 + D T / W + B^2 / (2 W^2) + (S.B)^2 / (2 z^2)
//   f3 = z - D W (1 + Gamma T / (Gamma - 1)).
__device__ bool c2p_newton(const C2PIn& c, const KPhys& ph, double& W, double& z, double& T) {
  const double gf = ph.gf;
  const double SB2 = c.SB * c.SB;
  for (int it = 0; it < ph.c2p_maxit; ++it) {
    const double zB = z + c.B2;
    const double iW = rcp_r(W);
    const double iW2 = iW * iW;
    const double iz = rcp_r(z);
    const double iz2 = iz * iz;
    const double om = 1.0 - iW2;
    const double f1 = c.S2 - zB * zB * om + SB2 * (2.0 * z + c.B2) * iz2;
    const double f2 = c.taut + c.Dt - z - c.B2 + c.Dt * T * iW + 0.5 * c.B2 * iW2 + 0.5 * SB2 * iz2;
    const double hW = 1.0 + gf * T;
    const double f3 = z - c.Dt * W * hW;
    const double J11 = -2.0 * zB * zB * iW2 * iW;
    const double J12 = -2.0 * zB * om - 2.0 * SB2 * zB * iz2 * iz;
    const double J21 = -c.Dt * T * iW2 - c.B2 * iW2 * iW;
    const double J22 = -1.0 - SB2 * iz2 * iz;
    const double J23 = c.Dt * iW;
    const double J31 = -c.Dt * hW;
    const double J33 = -c.Dt * W * gf;
    // J13 = 0, J32 = 1: Cramer's rule on J dx = -f
    const double m1 = J22 * J33 - J23;        // minor of J11
    const double m2 = J21 * J33 - J23 * J31;  // minor of J12
    const double det = J11 * m1 - J12 * m2;
    if (!(det != 0.0) || !dfinite(det)) return false;
    const double id = rcp_r(det);
    const double r1 = -f1, r2 = -f2, r3 = -f3;
    const double d1 = (r1 * m1 - J12 * (r2 * J33 - J23 * r3)) * id;
    const double d2 = (J11 * (r2 * J33 - J23 * r3) - r1 * m2) * id;
    const double d3 = (J11 * (J22 * r3 - r2) - J12 * (J21 * r3 - r2 * J31) + r1 * (J21 - J22 * J31)) * id;
    W += d1;
    z += d2;
    T += d3;
    if (!(dfinite(W) && dfinite(z) && dfinite(T))) return false;
    // max_k |dx_k / x_k| < tol, without divisions
    const double tol = ph.c2p_tol;
    if (fabs(d1) < tol * fabs(W) && fabs(d2) < tol * fabs(z) && fabs(d3) < tol * fabs(T)) return true;
  }
  return false;
}

// Newman-Hamlin map p -> p' (Sec. II C): the largest root x = z + B^2 of
// x^3 - (E + p + B^2/2) x^2 + (B^2 S^2 - (S.B)^2)/2 = 0, E = tau + D, then
// 1/W^2 = 1 - (S^2 + (S.B)^2 (2z + B^2) / z^2) / x^2 and the Gamma-law
// p' = (Gamma - 1)/Gamma (z/W^2 - D/W).
__device__ bool nh_map(const C2PIn& c, const KPhys& ph, double p, double& pn, double& W, double& z) {
  const double E = c.taut + c.Dt;
  const double dd = fmax(0.0, 0.5 * (c.B2 * c.S2 - c.SB * c.SB));
  const double a = -(E + p + 0.5 * c.B2);
  double x = -a;  // f(-a) = dd >= 0 and f is convex there: Newton descends onto the root
  for (int it = 0; it < 100; ++it) {
    const double f = x * x * (x + a) + dd;
    const double fp = x * (3.0 * x + 2.0 * a);
    const double dx = f / fp;
    x -= dx;
    if (!(fabs(dx) > 1e-15 * fabs(x))) break;
  }
  z = x - c.B2;
  if (!(z > 0.0)) return false;
  const double iW2 = 1.0 - (c.S2 + c.SB * c.SB * (2.0 * z + c.B2) / (z * z)) / (x * x);
  if (!(iW2 > 0.0)) return false;
  const double iW = sqrt(iW2);
  W = 1.0 / iW;
  pn = (ph.gm1 / ph.gam) * (z * iW2 - c.Dt * iW);
  return dfinite(pn);
}

// Fixed-point iteration on the pressure with Aitken extrapolation on every
// third iterate; returns the (W, z, T) that seed a Newton polish.
__device__ bool c2p_newman(const C2PIn& c, const KPhys& ph, double p0, double& W, double& z, double& T) {
  double s1 = p0, s2 = p0;
  for (int k = 0; k < ph.c2p_maxit; ++k) {
    double pn;
    if (!nh_map(c, ph, s2, pn, W, z)) return false;
    if (!(pn > 0.0)) return false;
    if (fabs(pn - s2) <= ph.c2p_tol * fabs(pn)) {
      T = pn * W / c.Dt;
      return true;
    }
    if ((k + 1) % 3 == 0) {
      const double den = pn - 2.0 * s2 + s1;
      if (den != 0.0) {
        const double pa = pn - (pn - s2) * (pn - s2) / den;
        if (pa > 0.0 && dfinite(pa)) pn = pa;
      }
    }
    s1 = s2;
    s2 = pn;
  }
  return false;
}

__device__ int c2p_recover(const C2PIn& c, const double* g, const double* gi, double gm1, double W, double z, double T,
                           double* P) {
  const double izB = rcp_r(z + c.B2);
  const double sbz = c.SB * rcp_r(z);
  double vlow[3], v[3];
#pragma unroll
  for (int j = 0; j < 3; ++j)
    vlow[j] = (c.St[j] + sbz * (g[sidx(j, 0)] * c.B[0] + g[sidx(j, 1)] * c.B[1] + g[sidx(j, 2)] * c.B[2])) * izB;
#pragma unroll
  for (int i = 0; i < 3; ++i) v[i] = gi[sidx(i, 0)] * vlow[0] + gi[sidx(i, 1)] * vlow[1] + gi[sidx(i, 2)] * vlow[2];
  const double v2 = vlow[0] * v[0] + vlow[1] * v[1] + vlow[2] * v[2];
  const double rho = c.Dt * rcp_r(W);
  if (!(W >= 1.0) || !(z > 0.0) || !(T > 0.0) || !(rho > 0.0) || !(v2 < 1.0)) return C2P_UNPHYS;
  P[0] = rho;
  P[1] = v[0];
  P[2] = v[1];
  P[3] = v[2];
  P[4] = T / gm1;
  P[5] = c.B[0];
  P[6] = c.B[1];
  P[7] = c.B[2];
  return C2P_OK;
}

// Atmosphere (Sec. IV, TOV test): rho_atm, v = 0, polytropic p, B kept; U rewritten.
__device__ __forceinline__ void c2p_atmosphere(const double* g, double sqrtg, const KPhys& ph, double U[8], double P[8]) {
  const double is = 1.0 / sqrtg;
  P[0] = ph.rho_atm;
  P[1] = P[2] = P[3] = 0.0;
  P[4] = ph.eps_atm;
#pragma unroll
  for (int k = 0; k < 3; ++k) P[5 + k] = U[5 + k] * is;
  p2c_cell(g, sqrtg, ph.gm1, P, U);
}

// Full recovery of one cell: U (in/out: atmosphere rewrites it), P (guess in, result out).
// With REFETCH, (*mf)(g, gi, sqrtg) re-points the metric after the Newton
// iteration (which does not use it), so a caller that can recompute the metric
// cheaply need not hold it in registers across the iteration.
struct NoRefetch {
  __device__ void operator()(const double*&, const double*&, double&) const {}
};
template <bool REFETCH = false, typename MF = NoRefetch>
__device__ int c2p_cell(const double* g, const double* gi, double sqrtg, const KPhys& ph, double U[8], double P[8],
                        const MF* mf = nullptr) {
  bool fin = true;
#pragma unroll
  for (int q = 0; q < 8; ++q) fin = fin && dfinite(U[q]);
  if (!fin) {
#pragma unroll
    for (int k = 5; k < 8; ++k) U[k] = dfinite(U[k]) ? U[k] : 0.0;
    c2p_atmosphere(g, sqrtg, ph, U, P);
    return C2P_NONFINITE;
  }
  const double is = rcp_r(sqrtg);
  C2PIn c;
  c.Dt = U[0] * is;
  if (c.Dt < ph.rho_floor) {
    c2p_atmosphere(g, sqrtg, ph, U, P);
    return C2P_FLOOR;
  }
#pragma unroll
  for (int j = 0; j < 3; ++j) c.St[j] = U[1 + j] * is;
  c.taut = U[4] * is;
#pragma unroll
  for (int k = 0; k < 3; ++k) c.B[k] = U[5 + k] * is;
  double S2 = 0.0, B2 = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      S2 += gi[sidx(i, j)] * c.St[i] * c.St[j];
      B2 += g[sidx(i, j)] * c.B[i] * c.B[j];
    }
  c.S2 = S2;
  c.B2 = B2;
  c.SB = c.St[0] * c.B[0] + c.St[1] * c.B[1] + c.St[2] * c.B[2];
  // seed from the previous primitives
  double W, z, T, p0;
  {
    double v2 = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) v2 += g[sidx(i, j)] * P[1 + i] * P[1 + j];
    const bool ok = dfinite(v2) && v2 < 1.0 && P[0] > 0.0 && P[4] > 0.0 && dfinite(P[0]) && dfinite(P[4]);
    if (ok) {
      W = rcp_r(sqrt_r(1.0 - v2));
      p0 = ph.gm1 * P[0] * P[4];
      z = (P[0] + P[0] * P[4] + p0) * W * W;
      T = p0 / P[0];
    } else {
      W = 1.0;
      T = ph.gm1 * fmax(c.taut - 0.5 * B2, 1e-10 * c.Dt) / c.Dt;
      z = c.Dt * (1.0 + ph.gf * T);
      p0 = c.Dt * T;
    }
  }
  double Pn[8];
  int st = C2P_NOCONV;
  {
    double W1 = W, z1 = z, T1 = T;
    const bool conv = c2p_newton(c, ph, W1, z1, T1);
    if constexpr (REFETCH) (*mf)(g, gi, sqrtg);
    if (conv) st = c2p_recover(c, g, gi, ph.gm1, W1, z1, T1, Pn);
  }
  if (st != C2P_OK) {
    double W2, z2, T2;
    int st2 = C2P_NOCONV;
    if (c2p_newman(c, ph, p0, W2, z2, T2) && c2p_newton(c, ph, W2, z2, T2))
      st2 = c2p_recover(c, g, gi, ph.gm1, W2, z2, T2, Pn);
    if (st2 == C2P_OK) st = C2P_FALLBACK;
    else if (st == C2P_NOCONV) st = st2;
  }
  if (st != C2P_OK && st != C2P_FALLBACK) {
    c2p_atmosphere(g, sqrtg, ph, U, P);
    return st;
  }
  if (Pn[0] < ph.rho_floor) {
    c2p_atmosphere(g, sqrtg, ph, U, P);
    return C2P_FLOOR;
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) P[q] = Pn[q];
  return st;
}

}  // namespace gk
