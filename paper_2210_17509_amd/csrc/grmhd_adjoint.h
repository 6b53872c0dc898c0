// Adjoint (vector-Jacobian product) building blocks of the SSPRK step.
//
// For L(U) = sum_d (F_lo - F_hi) / dx_d + S(P), P = con2prim(U):
//   J^T v = (dU/dP)^{-T} [ sum_faces (dF*/dP_stencil)^T Fbar + (dS/dP)^T v ],
//   Fbar(face between cells c-1, c) = (v_c - v_{c-1}) / dx_d,
// where con2prim is differentiated through the implicit-function theorem
// (it inverts prim->cons, so dP/dU = (dU/dP)^{-1}).  The face part is reverse
// mode written by hand: the HLLE combine, then each side's flux, state and
// speeds (side_vjp), then the gradient of the reconstruction, scattered onto
// the stencil cells.  The cell part (sources) uses forward-mode dual numbers
// DN<8>, one tangent per primitive.  Max/min branches follow the forward choice.
#pragma once

#include "grmhd_device.h"

namespace gk {

// ---------------------------------------------------------------- dual numbers

template <int N> struct DN {
  double v;
  double d[N];
  __device__ __forceinline__ DN() {}
  __device__ __forceinline__ DN(double a) : v(a) {
#pragma unroll
    for (int k = 0; k < N; ++k) d[k] = 0.0;
  }
};

template <int N> __device__ __forceinline__ DN<N> operator+(const DN<N>& a, const DN<N>& b) {
  DN<N> r;
  r.v = a.v + b.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] + b.d[k];
  return r;
}
template <int N> __device__ __forceinline__ DN<N> operator-(const DN<N>& a, const DN<N>& b) {
  DN<N> r;
  r.v = a.v - b.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] - b.d[k];
  return r;
}
template <int N> __device__ __forceinline__ DN<N> operator-(const DN<N>& a) {
  DN<N> r;
  r.v = -a.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = -a.d[k];
  return r;
}
template <int N> __device__ __forceinline__ DN<N> operator*(const DN<N>& a, const DN<N>& b) {
  DN<N> r;
  r.v = a.v * b.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
template <int N> __device__ __forceinline__ DN<N> operator/(const DN<N>& a, const DN<N>& b) {
  DN<N> r;
  const double ib = 1.0 / b.v;
  r.v = a.v * ib;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) * ib;
  return r;
}
template <int N> __device__ __forceinline__ DN<N> operator+(const DN<N>& a, double b) {
  DN<N> r = a;
  r.v += b;
  return r;
}
template <int N> __device__ __forceinline__ DN<N> operator+(double a, const DN<N>& b) { return b + a; }
template <int N> __device__ __forceinline__ DN<N> operator-(const DN<N>& a, double b) {
  DN<N> r = a;
  r.v -= b;
  return r;
}
template <int N> __device__ __forceinline__ DN<N> operator-(double a, const DN<N>& b) {
  DN<N> r;
  r.v = a - b.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = -b.d[k];
  return r;
}
template <int N> __device__ __forceinline__ DN<N> operator*(const DN<N>& a, double b) {
  DN<N> r;
  r.v = a.v * b;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * b;
  return r;
}
template <int N> __device__ __forceinline__ DN<N> operator*(double a, const DN<N>& b) { return b * a; }
template <int N> __device__ __forceinline__ DN<N> operator/(const DN<N>& a, double b) { return a * (1.0 / b); }
template <int N> __device__ __forceinline__ DN<N> operator/(double a, const DN<N>& b) {
  DN<N> r;
  const double ib = 1.0 / b.v;
  r.v = a * ib;
  const double s = -r.v * ib;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = s * b.d[k];
  return r;
}
template <int N> __device__ __forceinline__ bool operator<(const DN<N>& a, const DN<N>& b) { return a.v < b.v; }
template <int N> __device__ __forceinline__ bool operator>(const DN<N>& a, const DN<N>& b) { return a.v > b.v; }
template <int N> __device__ __forceinline__ bool operator<=(const DN<N>& a, const DN<N>& b) { return a.v <= b.v; }
template <int N> __device__ __forceinline__ bool operator==(const DN<N>& a, const DN<N>& b) { return a.v == b.v; }
template <int N> __device__ __forceinline__ DN<N> sqrt_r(const DN<N>& a) {
  DN<N> r;
  r.v = sqrt(a.v);
  const double h = 0.5 / r.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * h;
  return r;
}

// ---------------------------------------------------------------- dU/dP

// Rows D, S_j, tau of dU/dP for Eqs. (p2c1)-(p2c4), written out: J[r][c] =
// dU_r/dP_c, P = (rho, v^1..3, eps, B^1..3).  For the Gamma law rho h = rho (1 +
// Gamma eps), and with H = rho h W^2 + B^2 the conserved variables reduce to
//   D = sqrt(g) rho W,  S_j = sqrt(g) (H v_j - (B.v) B_j),
//   tau = sqrt(g) (H - p - B^2 / (2 W^2) - (B.v)^2 / 2) - D,
// with dW/dv^k = W^3 v_k (the ℬ rows are sqrt(g) times the identity).
__device__ __forceinline__ void p2c_jacobian(const double* g, double sqrtg, double gm1, const double* P,
                                             double J[5][8]) {
  const double rho = P[0], eps = P[4], gam = gm1 + 1.0;
  double vl[3], Bl[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    vl[i] = g[sidx(i, 0)] * P[1] + g[sidx(i, 1)] * P[2] + g[sidx(i, 2)] * P[3];
    Bl[i] = g[sidx(i, 0)] * P[5] + g[sidx(i, 1)] * P[6] + g[sidx(i, 2)] * P[7];
  }
  const double v2 = vl[0] * P[1] + vl[1] * P[2] + vl[2] * P[3];
  const double W = 1.0 / sqrt_r(1.0 - v2), W2 = W * W, W3 = W2 * W, W4 = W2 * W2;
  const double B2 = Bl[0] * P[5] + Bl[1] * P[6] + Bl[2] * P[7];
  const double Bv = Bl[0] * P[1] + Bl[1] * P[2] + Bl[2] * P[3];
  const double dhr = 1.0 + gam * eps;  // d(rho h)/d rho
  const double rh = rho * dhr;
  const double H = rh * W2 + B2;
  const double s = sqrtg;
  J[0][0] = s * W;
  J[0][4] = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    J[0][1 + k] = s * rho * W3 * vl[k];
    J[0][5 + k] = 0.0;
  }
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    J[1 + j][0] = s * dhr * W2 * vl[j];
    J[1 + j][4] = s * gam * rho * W2 * vl[j];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      J[1 + j][1 + k] = s * (2.0 * rh * W4 * vl[k] * vl[j] + H * g[sidx(j, k)] - Bl[k] * Bl[j]);
      J[1 + j][5 + k] = s * (2.0 * Bl[k] * vl[j] - vl[k] * Bl[j] - Bv * g[sidx(j, k)]);
    }
  }
  J[4][0] = s * (dhr * W2 - gm1 * eps - W);
  J[4][4] = s * (gam * rho * W2 - gm1 * rho);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    J[4][1 + k] = s * (2.0 * rh * W4 * vl[k] + B2 * vl[k] - Bv * Bl[k] - rho * W3 * vl[k]);
    J[4][5 + k] = s * (2.0 * Bl[k] - Bl[k] / W2 - Bv * vl[k]);
  }
}

// ---------------------------------------------------------------- sources

// Reverse of tmunu_T: Pb += d/dP (Tb00 T00 + sum_i Tb0_i T^{0i} + sum_{i<=j} Tbij_ij T^{ij})
// (symmetric storage: each off-diagonal T^{ij} once).
__device__ __forceinline__ void tmunu_vjp(const CentreMetric& m, const double* P, double gam, double Tb00,
                                          const double* Tb0, const double* Tbij, double* Pb) {
  // forward values, as in tmunu_T
  double vlow[3], Blow[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    vlow[i] = m.g[sidx(i, 0)] * P[1] + m.g[sidx(i, 1)] * P[2] + m.g[sidx(i, 2)] * P[3];
    Blow[i] = m.g[sidx(i, 0)] * P[5] + m.g[sidx(i, 1)] * P[6] + m.g[sidx(i, 2)] * P[7];
  }
  const double v2 = vlow[0] * P[1] + vlow[1] * P[2] + vlow[2] * P[3];
  const double iW = sqrt_r(1.0 - v2);
  const double W = 1.0 / iW;
  const double B2 = Blow[0] * P[5] + Blow[1] * P[6] + Blow[2] * P[7];
  const double Bv = Blow[0] * P[1] + Blow[1] * P[2] + Blow[2] * P[3];
  const double ia = 1.0 / m.alpha, ia2 = ia * ia;
  const double b0 = W * Bv * ia;
  const double b2 = B2 * (iW * iW) + Bv * Bv;
  const double p = (gam - 1.0) * P[0] * P[4];
  const double rhohs = P[0] * (1.0 + P[4]) + p + b2;
  const double u0 = W * ia;
  double u[3], b[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    u[i] = W * (P[1 + i] - m.beta[i] * ia);
    b[i] = (P[5 + i] + m.alpha * b0 * u[i]) * iW;
  }
  // adjoints of rho h*, P*, u^0, u^i, b^0, b^i from T^{mu nu}; A is Tbij as a full
  // symmetric matrix with the diagonal doubled (d(x_i x_i) = 2 x_i)
  double A[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) A[i][j] = (i == j) ? 2.0 * Tbij[sidx(i, i)] : Tbij[sidx(i, j)];
  double rhb = Tb00 * u0 * u0, Psb = -Tb00 * ia2, u0b = 2.0 * Tb00 * rhohs * u0, b0b = -2.0 * Tb00 * b0;
  double ub[3], bb[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    rhb += Tb0[i] * u0 * u[i];
    Psb += Tb0[i] * m.beta[i] * ia2;
    u0b += Tb0[i] * rhohs * u[i];
    b0b -= Tb0[i] * b[i];
    ub[i] = Tb0[i] * rhohs * u0;
    bb[i] = -Tb0[i] * b0;
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int j = i; j < 3; ++j) {
      rhb += Tbij[sidx(i, j)] * u[i] * u[j];
      Psb += Tbij[sidx(i, j)] * (m.gi[sidx(i, j)] - m.beta[i] * m.beta[j] * ia2);
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      ub[i] += rhohs * A[i][j] * u[j];
      bb[i] -= A[i][j] * b[j];
    }
  }
  // b^i = (B^i + alpha b^0 u^i) / W
  double iWb = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    Pb[5 + i] += bb[i] * iW;
    b0b += bb[i] * m.alpha * u[i] * iW;
    ub[i] += bb[i] * m.alpha * b0 * iW;
    iWb += bb[i] * (P[5 + i] + m.alpha * b0 * u[i]);
  }
  // u^i = W (v^i - beta^i / alpha), u^0 = W / alpha
  double Wb = u0b * ia;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    Wb += ub[i] * (P[1 + i] - m.beta[i] * ia);
    Pb[1 + i] += ub[i] * W;
  }
  // P* = p + b^2 / 2, rho h* = rho (1 + eps) + p + b^2, p = (Gamma - 1) rho eps
  const double pb = Psb + rhb, b2b = 0.5 * Psb + rhb;
  Pb[0] += rhb * (1.0 + P[4]) + pb * (gam - 1.0) * P[4];
  Pb[4] += rhb * P[0] + pb * (gam - 1.0) * P[0];
  // alpha b^0 = W (B.v), b^2 = B^2 / W^2 + (B.v)^2
  Wb += b0b * Bv * ia;
  const double Bvb = b0b * W * ia + 2.0 * b2b * Bv;
  const double B2b = b2b * iW * iW;
  iWb += 2.0 * b2b * B2 * iW;
  // W = 1 / iW, iW = sqrt(1 - v^2)
  iWb -= Wb * W * W;
  const double v2b = -0.5 * iWb * W;
  // v^2 = v.g.v, B^2 = B.g.B, B.v = B.g.v
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    Pb[1 + k] += 2.0 * v2b * vlow[k] + Bvb * Blow[k];
    Pb[5 + k] += 2.0 * B2b * Blow[k] + Bvb * vlow[k];
  }
}

// Pb += (dS/dP)^T v for the source terms (v indexed like U; only the momenta and
// tau carry sources).  The map T^{mu nu} -> S is linear, so its transpose applied
// to v comes from one evaluation on dual numbers with a unit tangent per
// component of T^{mu nu}; the rest is the reverse of tmunu_T.
template <bool SHIFT>
__device__ __forceinline__ void sources_vjp(const CentreMetric& m, const MetricDeriv& md, const double* P, double gam,
                                            const double* v, double* Pb) {
  DN<10> T00(0.0), T0[3], Tij[6];
  T00.d[0] = 1.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    T0[i] = DN<10>(0.0);
    T0[i].d[1 + i] = 1.0;
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    Tij[q] = DN<10>(0.0);
    Tij[q].d[4 + q] = 1.0;
  }
  DN<10> S[8];
  sources_tail<SHIFT>(m, md, T00, T0, Tij, S);
  double Tb[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) Tb[k] = v[1] * S[1].d[k] + v[2] * S[2].d[k] + v[3] * S[3].d[k] + v[4] * S[4].d[k];
  tmunu_vjp(m, P, gam, Tb[0], Tb + 1, Tb + 4, Pb);
}

// ---------------------------------------------------------------- reconstruction gradients

// Adjoint of the WENO5 value at the right face of c in (a, b, c, d, e): g[o] =
// ab * d(value)/d(s_o).  Reverse mode through the normalisation and through
// the weights in their un-normalised product form (JS: d_k prod_{j != k}
// (eps + beta_j)^2; Z: d_k (e_k^p + tau^p) prod_{j != k} e_j^p, e = beta + eps,
// tau = |beta_0 - beta_2|), which normalises to the forward kernel's weights.
template <bool ZW, int ZPC = 0>
__device__ __forceinline__ void weno5_vjp(const double* s, double eps, int zp, double ab, double g[5]) {
  if (ZPC != 0) zp = ZPC;  // exponent fixed at compile time
  const double a = s[0], b = s[1], c = s[2], d = s[3], e = s[4];
  const double q[3] = {2 * a - 7 * b + 11 * c, -b + 5 * c + 2 * d, 2 * c + 5 * d - e};
  const double X0 = a - 2 * b + c, Y0 = a - 4 * b + 3 * c;
  const double X1 = b - 2 * c + d, Y1 = b - d;
  const double X2 = c - 2 * d + e, Y2 = 3 * c - 4 * d + e;
  const double be[3] = {13.0 / 12.0 * X0 * X0 + 0.25 * Y0 * Y0, 13.0 / 12.0 * X1 * X1 + 0.25 * Y1 * Y1,
                        13.0 / 12.0 * X2 * X2 + 0.25 * Y2 * Y2};
  const double dk[3] = {0.1, 0.6, 0.3};
  // forward: un-normalised weights and the pieces their adjoint needs
  double w[3], t[3], f[3], tpd = 0.0, sg = 0.0;
  if (!ZW) {
#pragma unroll
    for (int k = 0; k < 3; ++k) t[k] = (eps + be[k]) * (eps + be[k]);
    w[0] = dk[0] * t[1] * t[2];
    w[1] = dk[1] * t[0] * t[2];
    w[2] = dk[2] * t[0] * t[1];
  } else {
    const double tau = fabs(be[0] - be[2]);
    sg = (be[0] > be[2]) ? 1.0 : ((be[0] < be[2]) ? -1.0 : 0.0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double ek = be[k] + eps;
      t[k] = (zp == 2) ? ek * ek : ek;  // e_k^p
    }
    const double tp = (zp == 2) ? tau * tau : tau;
    tpd = (zp == 2) ? 2.0 * tau : 1.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      f[k] = t[k] + tp;
      w[k] = dk[k] * f[k] * t[(k + 1) % 3] * t[(k + 2) % 3];
    }
  }
  const double i6W = rcp_r(6.0 * (w[0] + w[1] + w[2]));
  const double qv = (w[0] * q[0] + w[1] * q[1] + w[2] * q[2]) * i6W;
  // reverse: value -> weights -> e_k^p (or (eps + beta_k)^2) -> beta_k
  double wb[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) wb[k] = ab * (q[k] - 6.0 * qv) * i6W * dk[k];  // adjoint of w_k / d_k
  double bb[3];
  if (!ZW) {
    const double tb0 = wb[1] * t[2] + wb[2] * t[1];
    const double tb1 = wb[0] * t[2] + wb[2] * t[0];
    const double tb2 = wb[0] * t[1] + wb[1] * t[0];
    bb[0] = 2.0 * (eps + be[0]) * tb0;
    bb[1] = 2.0 * (eps + be[1]) * tb1;
    bb[2] = 2.0 * (eps + be[2]) * tb2;
  } else {
    // w_k / d_k = f_k t_j t_l with f_k = t_k + tau^p
    double tb[3] = {0.0, 0.0, 0.0}, tpb = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int j = (k + 1) % 3, l = (k + 2) % 3;
      const double fb = wb[k] * t[j] * t[l];
      const double wf = wb[k] * f[k];
      tb[k] += fb;
      tpb += fb;
      tb[j] += wf * t[l];
      tb[l] += wf * t[j];
    }
    const double taub = tpb * tpd;
#pragma unroll
    for (int k = 0; k < 3; ++k) bb[k] = (zp == 2) ? 2.0 * (be[k] + eps) * tb[k] : tb[k];
    bb[0] += sg * taub;
    bb[2] -= sg * taub;
  }
  // beta_m = 13/12 X_m^2 + 1/4 Y_m^2, and the candidates q_k, are linear in the stencil
  const double xb0 = 13.0 / 6.0 * X0 * bb[0], yb0 = 0.5 * Y0 * bb[0];
  const double xb1 = 13.0 / 6.0 * X1 * bb[1], yb1 = 0.5 * Y1 * bb[1];
  const double xb2 = 13.0 / 6.0 * X2 * bb[2], yb2 = 0.5 * Y2 * bb[2];
  const double o0 = ab * w[0] * i6W, o1 = ab * w[1] * i6W, o2 = ab * w[2] * i6W;
  // candidates: q0 = (2, -7, 11, 0, 0), q1 = (0, -1, 5, 2, 0), q2 = (0, 0, 2, 5, -1)
  g[0] = 2 * o0 + xb0 + yb0;
  g[1] = -7 * o0 - o1 - 2 * xb0 - 4 * yb0 + xb1 + yb1;
  g[2] = 11 * o0 + 5 * o1 + 2 * o2 + xb0 + 3 * yb0 - 2 * xb1 + xb2 + 3 * yb2;
  g[3] = 2 * o1 + 5 * o2 + xb1 - yb1 - 2 * xb2 - 4 * yb2;
  g[4] = -o2 + xb2 + yb2;
}

// minmod left state s[2] + mm(s[2]-s[1], s[3]-s[2]) / 2 and its gradient w.r.t. s[1..3]
__device__ __forceinline__ double minmod_grad(double s1, double s2, double s3, double g[3]) {
  const double x = s2 - s1, y = s3 - s2;
  if (x * y <= 0.0) {
    g[0] = 0.0; g[1] = 1.0; g[2] = 0.0;
    return s2;
  }
  if (fabs(x) < fabs(y)) {
    g[0] = -0.5; g[1] = 1.5; g[2] = 0.0;
    return s2 + 0.5 * x;
  }
  g[0] = 0.0; g[1] = 0.5; g[2] = 0.5;
  return s2 + 0.5 * y;
}

}  // namespace gk

namespace gk {

// Reverse pass of one face side (FP64): given the adjoints of the side's
// conserved variables Ub, direction-D fluxes Fb and speed bounds lpb, lmb,
// accumulate the adjoint of its 8 primitives into Pb.  The forward
// intermediates are recomputed in the same order as side_v2 / side_rest /
// side_speeds / side_cons_flux, then every statement is reversed.
template <int D>
__device__ __forceinline__ void side_vjp(const FaceMetric<double>& m, const double* P, double gam, double gm1,
                                         const double* Ub, const double* Fb, double lpb, double lmb, double* Pb) {
  const double* g = m.g;
  const double rho = P[0], eps = P[4];
  const double v[3] = {P[1], P[2], P[3]};
  const double B[3] = {P[5], P[6], P[7]};
  double vl[3], Bl[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    vl[i] = g[sidx(i, 0)] * v[0] + g[sidx(i, 1)] * v[1] + g[sidx(i, 2)] * v[2];
    Bl[i] = g[sidx(i, 0)] * B[0] + g[sidx(i, 1)] * B[1] + g[sidx(i, 2)] * B[2];
  }
  const double v2 = vl[0] * v[0] + vl[1] * v[1] + vl[2] * v[2];
  const double om = 1.0 - v2;
  const double iW = sqrt_r(om);
  const double W = rcp_r(iW);
  const double B2 = Bl[0] * B[0] + Bl[1] * B[1] + Bl[2] * B[2];
  const double Bv = Bl[0] * v[0] + Bl[1] * v[1] + Bl[2] * v[2];
  const double ab0 = W * Bv;
  const double iW2 = iW * iW;
  const double b2 = (B2 + ab0 * ab0) * iW2;
  const double p = gm1 * rho * eps;
  const double rhoh = rho * (1.0 + eps) + p;
  // speeds (one reciprocal for c_s^2 and c_a^2, as in side_speeds)
  const double qq = rhoh + b2;
  const double ir = rcp_r(rhoh * qq);
  const double irhoh = qq * ir, iqq = rhoh * ir;
  const double cs2 = gam * p * qq * ir;
  const double ca2 = b2 * rhoh * ir;
  const double cf2 = cs2 + ca2 - cs2 * ca2;
  const double vd = v[D];
  const double den = 1.0 - v2 * cf2;
  const double X = m.gdd * den - vd * vd * (1.0 - cf2);
  const double disc = om * X;
  const double dc = disc < 0.0 ? 0.0 : disc;
  const double root = sqrt_r(cf2 * dc);
  const double base = vd * (1.0 - cf2);
  const double iden = rcp_r(den);
  const double ad = m.alpha * iden;
  // cons / flux
  const double W2 = W * W;
  const double rhohs = rhoh + b2;
  const double Ps = p + 0.5 * b2;
  const double sg = m.sqrtg, al = m.alpha;
  double bl[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) bl[i] = Bl[i] * iW + ab0 * vl[i];
  double U[8];
  U[0] = sg * rho * W;
#pragma unroll
  for (int j = 0; j < 3; ++j) U[1 + j] = sg * (rhohs * W2 * vl[j] - ab0 * bl[j]);
  U[4] = sg * (rhohs * W2 - Ps - ab0 * ab0) - U[0];
#pragma unroll
  for (int k = 0; k < 3; ++k) U[5 + k] = sg * B[k];
  const double ia = m.ialpha;
  double vt[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) vt[i] = v[i] - m.beta[i] * ia;
  const double BnW = U[5 + D] * iW;

  // ---- reverse ----
  double Ubar[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) Ubar[q] = Ub[q];
  double vtb[3] = {0.0, 0.0, 0.0}, vb_[3] = {0.0, 0.0, 0.0}, Bb_[3] = {0.0, 0.0, 0.0};
  double Psb = 0.0, ab0b = 0.0, BnWb = 0.0, blb[3] = {0.0, 0.0, 0.0};
  // F_{5+k}, k != D
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (k == D) continue;
    const double f = Fb[5 + k] * al;
    Ubar[5 + k] += f * vt[D];
    vtb[D] += f * U[5 + k];
    Ubar[5 + D] -= f * vt[k];
    vtb[k] -= f * U[5 + D];
  }
  {  // F4
    const double f = Fb[4] * al;
    Ubar[4] += f * vt[D];
    vtb[D] += f * U[4];
    Psb += f * sg * v[D];
    vb_[D] += f * sg * Ps;
    ab0b -= f * BnW;
    BnWb -= f * ab0;
  }
#pragma unroll
  for (int j = 0; j < 3; ++j) {  // F_{1+j}
    const double f = Fb[1 + j] * al;
    Ubar[1 + j] += f * vt[D];
    vtb[D] += f * U[1 + j];
    blb[j] -= f * BnW;
    BnWb -= f * bl[j];
    if (j == D) Psb += f * sg;
  }
  {  // F0
    const double f = Fb[0] * al;
    Ubar[0] += f * vt[D];
    vtb[D] += f * U[0];
  }
  double iWb = 0.0;
  Ubar[5 + D] += BnWb * iW;
  iWb += BnWb * U[5 + D];
#pragma unroll
  for (int i = 0; i < 3; ++i) vb_[i] += vtb[i];
#pragma unroll
  for (int k = 0; k < 3; ++k) Bb_[k] += Ubar[5 + k] * sg;
  double rhohsb = 0.0, W2b = 0.0, Wb = 0.0, rhob = 0.0, vlb[3] = {0.0, 0.0, 0.0};
  {  // U4
    const double f = Ubar[4] * sg;
    rhohsb += f * W2;
    W2b += f * rhohs;
    Psb -= f;
    ab0b -= f * 2.0 * ab0;
    Ubar[0] -= Ubar[4];
  }
#pragma unroll
  for (int j = 0; j < 3; ++j) {  // U_{1+j}
    const double f = Ubar[1 + j] * sg;
    rhohsb += f * W2 * vl[j];
    W2b += f * rhohs * vl[j];
    vlb[j] += f * rhohs * W2;
    ab0b -= f * bl[j];
    blb[j] -= f * ab0;
  }
  rhob += Ubar[0] * sg * W;
  Wb += Ubar[0] * sg * rho;
  double Blb[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {  // bl_i = Bl_i iW + ab0 vl_i
    Blb[i] = blb[i] * iW;
    iWb += blb[i] * Bl[i];
    ab0b += blb[i] * vl[i];
    vlb[i] += blb[i] * ab0;
  }
  double pb = Psb, b2b = 0.5 * Psb;
  double rhohb = rhohsb;
  b2b += rhohsb;
  Wb += 2.0 * W * W2b;
  // speeds
  const double lsum = lpb * (base + root) + lmb * (base - root);
  const double adb = lsum;
  const double baseb = (lpb + lmb) * ad;
  const double rootb = (lpb - lmb) * ad;
  double denb = -adb * ad * iden;
  double vdb = baseb * (1.0 - cf2);
  double cf2b = -baseb * vd;
  double dcb = 0.0;
  if (root > 0.0) {
    const double r2b = rootb * 0.5 * rcp_r(root);
    cf2b += r2b * dc;
    dcb = r2b * cf2;
  }
  const double discb = disc < 0.0 ? 0.0 : dcb;
  double omb = discb * X;
  const double Xb = discb * om;
  denb += Xb * m.gdd;
  vdb -= Xb * 2.0 * vd * (1.0 - cf2);
  cf2b += Xb * vd * vd;
  double v2b = -denb * cf2;
  cf2b -= denb * v2;
  vb_[D] += vdb;
  const double cs2b = cf2b * (1.0 - ca2);
  const double ca2b = cf2b * (1.0 - cs2);
  b2b += ca2b * (1.0 - ca2) * iqq;
  rhohb -= ca2b * ca2 * iqq;
  pb += cs2b * gam * irhoh;
  rhohb -= cs2b * cs2 * irhoh;
  // state
  rhob += rhohb * (1.0 + eps);
  double epsb = rhohb * rho;
  pb += rhohb;
  rhob += pb * gm1 * eps;
  epsb += pb * gm1 * rho;
  const double B2b = b2b * iW2;
  ab0b += b2b * iW2 * 2.0 * ab0;
  const double iW2b = b2b * (B2 + ab0 * ab0);
  iWb += 2.0 * iW * iW2b;
  Wb += ab0b * Bv;
  const double Bvb = ab0b * W;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    Blb[i] += Bvb * v[i] + B2b * B[i];
    vb_[i] += Bvb * Bl[i];
    Bb_[i] += B2b * Bl[i];
  }
  iWb += -Wb * W * W;
  omb += iWb * 0.5 * W;
  v2b -= omb;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    vlb[i] += v2b * v[i];
    vb_[i] += v2b * vl[i];
  }
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    Bb_[j] += g[sidx(0, j)] * Blb[0] + g[sidx(1, j)] * Blb[1] + g[sidx(2, j)] * Blb[2];
    vb_[j] += g[sidx(0, j)] * vlb[0] + g[sidx(1, j)] * vlb[1] + g[sidx(2, j)] * vlb[2];
  }
  Pb[0] += rhob;
  Pb[1] += vb_[0];
  Pb[2] += vb_[1];
  Pb[3] += vb_[2];
  Pb[4] += epsb;
  Pb[5] += Bb_[0];
  Pb[6] += Bb_[1];
  Pb[7] += Bb_[2];
}

}  // namespace gk
