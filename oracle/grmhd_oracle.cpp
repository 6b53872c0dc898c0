/*
 * GRMHD oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, serial FP64 CPU implementation of the static-metric Valencia
 * GRMHD hot path of GRaM-X (arXiv:2210.17509): prim->cons map, con2prim by a
 * 3D Newton-Raphson in (W, z, T), TVD-minmod / WENO5 / WENO5-Z reconstruction
 * of primitives, the HLLE flux, flux divergence plus the metric source terms,
 * and an SSPRK3 method-of-lines step.
 *
 * Only the test suite, the package smoke check and the benchmark's CPU baseline
 * may load this library.  It shares no code with the HIP path and is built
 * with -ffp-contract=off so every floating-point operation is the one written.
 *
 * Everything is templated on the scalar type: T = double is the reference,
 * T = Dual carries one tangent and gives exact Jacobian-vector products
 * (used to check the hand-written adjoint).
 *
 * Citations name the paper's section and equation labels:
 *   Sec. II B   Valencia formulation: T^{mu nu} (mhd-stress-energy-tensor),
 *               prim->cons (p2c1)-(p2c4), velocity (vel), fluxes
 *               (definition-of-flux), sources (definition-of-source).
 *   Sec. II C   Numerical methods: MoL RHS in four steps, TVD [Toro] and WENO5
 *               [Shu 98] reconstruction of P on faces with the metric
 *               interpolated linearly from vertices to face centres, HLLE
 *               [Harten-Lax-van Leer, Einfeldt], Gamma-law EOS, 3D-NR con2prim
 *               in (W, z = rho h W^2, T).
 *   Sec. III    cell-averaged fluid, vertex-centred spacetime.
 *   Sec. IV A   boundary "copy from the nearest interior point".
 * Readings of points the paper leaves open are listed in the design notes
 * (R-numbers in comments refer to that list).
 */
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

/* ------------------------------------------------------------------------ */
/* scalar types                                                             */
/* ------------------------------------------------------------------------ */

struct Dual {
  double v, d;
  Dual() : v(0), d(0) {}
  Dual(double a) : v(a), d(0) {}
  Dual(double a, double b) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
  double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
inline Dual operator+(Dual a, double b) { return Dual(a.v + b, a.d); }
inline Dual operator+(double a, Dual b) { return Dual(a + b.v, b.d); }
inline Dual operator-(Dual a, double b) { return Dual(a.v - b, a.d); }
inline Dual operator-(double a, Dual b) { return Dual(a - b.v, -b.d); }
inline Dual operator*(Dual a, double b) { return Dual(a.v * b, a.d * b); }
inline Dual operator*(double a, Dual b) { return Dual(a * b.v, a * b.d); }
inline Dual operator/(Dual a, double b) { return Dual(a.v / b, a.d / b); }
inline Dual operator/(double a, Dual b) {
  double q = a / b.v;
  return Dual(q, -q * b.d / b.v);
}
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
inline bool operator<(Dual a, Dual b) { return a.v < b.v; }
inline bool operator>(Dual a, Dual b) { return a.v > b.v; }
inline bool operator<=(Dual a, Dual b) { return a.v <= b.v; }
inline bool operator>=(Dual a, Dual b) { return a.v >= b.v; }
inline bool operator<(Dual a, double b) { return a.v < b; }
inline bool operator>(Dual a, double b) { return a.v > b; }
inline bool operator<=(Dual a, double b) { return a.v <= b; }
inline bool operator>=(Dual a, double b) { return a.v >= b; }
inline bool operator==(Dual a, double b) { return a.v == b; }
inline Dual sqrt(Dual a) {
  double s = std::sqrt(a.v);
  return Dual(s, a.d / (2.0 * s));
}
inline Dual fabs(Dual a) { return a.v < 0 ? -a : a; }

inline double val(double a) { return a; }
inline double val(const Dual& a) { return a.v; }
inline bool finite(double a) { return std::isfinite(a); }
inline bool finite(const Dual& a) { return std::isfinite(a.v) && std::isfinite(a.d); }
using std::fabs;
using std::sqrt;

// Op-counting scalar: every +, -, *, / and sqrt on it is tallied (comparisons
// and fabs are not floating-point work).  Used to count the method's
// arithmetic per face and per cell.
struct OpTally { long add, mul, div, sqrt; };
static OpTally g_tally = {0, 0, 0, 0};
struct Cnt {
  double v;
  Cnt() : v(0) {}
  Cnt(double a) : v(a) {}
};
inline Cnt operator+(Cnt a, Cnt b) { ++g_tally.add; return Cnt(a.v + b.v); }
inline Cnt operator-(Cnt a, Cnt b) { ++g_tally.add; return Cnt(a.v - b.v); }
inline Cnt operator-(Cnt a) { return Cnt(-a.v); }
inline Cnt operator*(Cnt a, Cnt b) { ++g_tally.mul; return Cnt(a.v * b.v); }
inline Cnt operator/(Cnt a, Cnt b) { ++g_tally.div; return Cnt(a.v / b.v); }
inline Cnt operator+(Cnt a, double b) { return a + Cnt(b); }
inline Cnt operator+(double a, Cnt b) { return Cnt(a) + b; }
inline Cnt operator-(Cnt a, double b) { return a - Cnt(b); }
inline Cnt operator-(double a, Cnt b) { return Cnt(a) - b; }
inline Cnt operator*(Cnt a, double b) { return a * Cnt(b); }
inline Cnt operator*(double a, Cnt b) { return Cnt(a) * b; }
inline Cnt operator/(Cnt a, double b) { return a / Cnt(b); }
inline Cnt operator/(double a, Cnt b) { return Cnt(a) / b; }
inline Cnt& operator+=(Cnt& a, Cnt b) { a = a + b; return a; }
inline Cnt& operator-=(Cnt& a, Cnt b) { a = a - b; return a; }
inline bool operator<(Cnt a, Cnt b) { return a.v < b.v; }
inline bool operator>(Cnt a, Cnt b) { return a.v > b.v; }
inline bool operator<=(Cnt a, Cnt b) { return a.v <= b.v; }
inline bool operator>=(Cnt a, Cnt b) { return a.v >= b.v; }
inline bool operator<(Cnt a, double b) { return a.v < b; }
inline bool operator>(Cnt a, double b) { return a.v > b; }
inline bool operator<=(Cnt a, double b) { return a.v <= b; }
inline bool operator>=(Cnt a, double b) { return a.v >= b; }
inline bool operator==(Cnt a, double b) { return a.v == b; }
inline Cnt sqrt(Cnt a) { ++g_tally.sqrt; return Cnt(std::sqrt(a.v)); }
inline Cnt fabs(Cnt a) { return Cnt(std::fabs(a.v)); }
inline double val(const Cnt& a) { return a.v; }
inline bool finite(const Cnt& a) { return std::isfinite(a.v); }

template <class T> inline T sq(T x) { return x * x; }
template <class T> inline T tmax(T a, T b) { return (a < b) ? b : a; }
template <class T> inline T tmin(T a, T b) { return (b < a) ? b : a; }

template <class T> struct extra_newton { static const int n = 0; };
template <> struct extra_newton<Dual> { static const int n = 2; };

/* ------------------------------------------------------------------------ */
/* grid description                                                         */
/* ------------------------------------------------------------------------ */

enum { BC_PERIODIC = 0, BC_OUTFLOW = 1 };
enum { REC_MINMOD = 0, REC_WENO5 = 1, REC_WENOZ = 2 };

struct Box {
  int32_t n[3];
  int32_t ng;
  int32_t bc[6];
  double x0[3];
  double dx[3];
};

struct Par {
  int32_t recon;
  int32_t wenoz_p;
  int32_t c2p_maxit;
  int32_t pad;
  double gam;
  double weno_eps;
  double wenoz_eps;
  double c2p_tol;
  double rho_atm;
  double atm_K;
  double atm_gamma;
};

struct Geo {
  int n[3], ng;
  long NX, NY, NZ;     // storage cells per axis
  long VX, VY, VZ;     // vertices per axis
  long ncell, nvert;
  Geo(const Box& b) {
    for (int d = 0; d < 3; ++d) n[d] = b.n[d];
    ng = b.ng;
    NX = n[0] + 2 * ng; NY = n[1] + 2 * ng; NZ = n[2] + 2 * ng;
    VX = NX + 1; VY = NY + 1; VZ = NZ + 1;
    ncell = NX * NY * NZ;
    nvert = VX * VY * VZ;
  }
  // storage index of interior cell (i, j, k); ghosts have negative / >= n coords
  long c(long i, long j, long k) const { return ((k + ng) * NY + (j + ng)) * NX + (i + ng); }
  // storage index of the vertex at the lower corner of interior cell (i, j, k)
  long v(long i, long j, long k) const { return ((k + ng) * VY + (j + ng)) * VX + (i + ng); }
};

// metric fields as stored on vertices
struct VMetric {
  const double* alpha;  // one field
  const double* beta;   // 3 fields or null (zero shift)
  const double* gamma;  // 6 fields: xx xy xz yy yz zz
  long stride;          // elements between fields
};

/* ------------------------------------------------------------------------ */
/* metric at a point (Sec. II C: vertex data interpolated linearly)         */
/* ------------------------------------------------------------------------ */

inline int sym(int i, int j) {
  static const int t[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
  return t[i][j];
}

template <class T> struct PMetric {
  T alpha;
  T beta[3];
  T g[6];     // gamma_ij
  T det;      // gamma
  T sqrtg;    // sqrt(gamma)
  T ginv[6];  // gamma^ij
};

template <class T> void metric_finish(PMetric<T>& m) {
  const T* g = m.g;
  T cxx = g[3] * g[5] - g[4] * g[4];
  T cxy = g[2] * g[4] - g[1] * g[5];
  T cxz = g[1] * g[4] - g[2] * g[3];
  T cyy = g[0] * g[5] - g[2] * g[2];
  T cyz = g[1] * g[2] - g[0] * g[4];
  T czz = g[0] * g[3] - g[1] * g[1];
  m.det = g[0] * cxx + g[1] * cxy + g[2] * cxz;
  m.sqrtg = sqrt(m.det);
  T inv = T(1.0) / m.det;
  m.ginv[0] = cxx * inv; m.ginv[1] = cxy * inv; m.ginv[2] = cxz * inv;
  m.ginv[3] = cyy * inv; m.ginv[4] = cyz * inv; m.ginv[5] = czz * inv;
}

// Mean of vertex values at a list of storage indices.
static double vmean(const double* f, const long* idx, int cnt) {
  if (cnt == 4) return 0.25 * ((f[idx[0]] + f[idx[1]]) + (f[idx[2]] + f[idx[3]]));
  return 0.125 * (((f[idx[0]] + f[idx[1]]) + (f[idx[2]] + f[idx[3]])) +
                  ((f[idx[4]] + f[idx[5]]) + (f[idx[6]] + f[idx[7]])));
}

template <class T> void metric_at(const VMetric& vm, const long* idx, int cnt, PMetric<T>& m) {
  m.alpha = T(vmean(vm.alpha, idx, cnt));
  for (int a = 0; a < 3; ++a) m.beta[a] = vm.beta ? T(vmean(vm.beta + a * vm.stride, idx, cnt)) : T(0.0);
  for (int a = 0; a < 6; ++a) m.g[a] = T(vmean(vm.gamma + a * vm.stride, idx, cnt));
  metric_finish(m);
}

// Face centre of the low face (direction d) of interior cell (i,j,k): 4-vertex mean (R4).
template <class T> void metric_face(const Geo& G, const VMetric& vm, int d, long i, long j, long k, PMetric<T>& m) {
  long idx[4];
  int a = (d + 1) % 3, b = (d + 2) % 3;
  long base[3] = {i, j, k};
  int q = 0;
  for (int cb = 0; cb < 2; ++cb)
    for (int ca = 0; ca < 2; ++ca) {
      long p[3] = {base[0], base[1], base[2]};
      p[a] += ca;
      p[b] += cb;
      idx[q++] = G.v(p[0], p[1], p[2]);
    }
  metric_at(vm, idx, 4, m);
}

// Cell centre: 8-vertex mean (R4).
template <class T> void metric_centre(const Geo& G, const VMetric& vm, long i, long j, long k, PMetric<T>& m) {
  long idx[8];
  int q = 0;
  for (int c = 0; c < 2; ++c)
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a) idx[q++] = G.v(i + a, j + b, k + c);
  metric_at(vm, idx, 8, m);
}

// d/dx^e of a vertex field at the centre of cell (i,j,k): mean over the four
// edges along e of the one-sided difference (second order, R4).
static double vderiv(const Geo& G, const double* f, int e, long i, long j, long k, double dx) {
  int a = (e + 1) % 3, b = (e + 2) % 3;
  double s[4];
  int q = 0;
  for (int cb = 0; cb < 2; ++cb)
    for (int ca = 0; ca < 2; ++ca) {
      long p[3] = {i, j, k};
      p[a] += ca;
      p[b] += cb;
      long lo = G.v(p[0], p[1], p[2]);
      p[e] += 1;
      long hi = G.v(p[0], p[1], p[2]);
      s[q++] = f[hi] - f[lo];
    }
  return 0.25 * ((s[0] + s[1]) + (s[2] + s[3])) / dx;
}

struct MetricDeriv {
  double dalpha[3];
  double dbeta[3][3];   // [e][a] = d_e beta^a
  double dgamma[3][6];  // [e][ij] = d_e gamma_ij
};

static void metric_deriv(const Geo& G, const VMetric& vm, const Box& bx, long i, long j, long k, MetricDeriv& D) {
  for (int e = 0; e < 3; ++e) {
    D.dalpha[e] = vderiv(G, vm.alpha, e, i, j, k, bx.dx[e]);
    for (int a = 0; a < 3; ++a) D.dbeta[e][a] = vm.beta ? vderiv(G, vm.beta + a * vm.stride, e, i, j, k, bx.dx[e]) : 0.0;
    for (int a = 0; a < 6; ++a) D.dgamma[e][a] = vderiv(G, vm.gamma + a * vm.stride, e, i, j, k, bx.dx[e]);
  }
}

/* ------------------------------------------------------------------------ */
/* prim -> cons, Eqs. (p2c1)-(p2c4) with Eq. (vel) and the Gamma-law EOS     */
/* ------------------------------------------------------------------------ */

template <class T> struct PState {
  T W;          // Lorentz factor
  T vlow[3];    // v_i
  T v2;
  T Blow[3];    // B_i
  T B2;
  T Bv;         // B^i v_i
  T ab0;        // alpha b^0
  T b2;         // b^mu b_mu
  T p;          // gas pressure
  T rhoh;       // rho h = rho (1 + eps) + p
  T rhohs;      // rho h* = rho h + b^2
  T Ps;         // P* = p + b^2 / 2
  T blow[3];    // b_j
};

template <class T> void prim_state(const PMetric<T>& m, const T* P, double gam, PState<T>& s) {
  const T rho = P[0], eps = P[4];
  const T v[3] = {P[1], P[2], P[3]};
  const T B[3] = {P[5], P[6], P[7]};
  for (int i = 0; i < 3; ++i) {
    s.vlow[i] = m.g[sym(i, 0)] * v[0] + m.g[sym(i, 1)] * v[1] + m.g[sym(i, 2)] * v[2];
    s.Blow[i] = m.g[sym(i, 0)] * B[0] + m.g[sym(i, 1)] * B[1] + m.g[sym(i, 2)] * B[2];
  }
  s.v2 = s.vlow[0] * v[0] + s.vlow[1] * v[1] + s.vlow[2] * v[2];
  s.W = T(1.0) / sqrt(T(1.0) - s.v2);
  s.B2 = s.Blow[0] * B[0] + s.Blow[1] * B[1] + s.Blow[2] * B[2];
  s.Bv = s.Blow[0] * v[0] + s.Blow[1] * v[1] + s.Blow[2] * v[2];
  s.ab0 = s.W * s.Bv;
  s.b2 = (s.B2 + s.ab0 * s.ab0) / (s.W * s.W);
  s.p = (gam - 1.0) * rho * eps;
  s.rhoh = rho * (T(1.0) + eps) + s.p;
  s.rhohs = s.rhoh + s.b2;
  s.Ps = s.p + 0.5 * s.b2;
  for (int i = 0; i < 3; ++i) s.blow[i] = s.Blow[i] / s.W + s.ab0 * s.vlow[i];
}

template <class T> void prim_to_cons(const PMetric<T>& m, const T* P, const PState<T>& s, T* U) {
  const T sg = m.sqrtg;
  const T W2 = s.W * s.W;
  U[0] = sg * P[0] * s.W;                                            // (p2c1)
  for (int j = 0; j < 3; ++j)
    U[1 + j] = sg * (s.rhohs * W2 * s.vlow[j] - s.ab0 * s.blow[j]);  // (p2c2)
  U[4] = sg * (s.rhohs * W2 - s.Ps - s.ab0 * s.ab0) - U[0];         // (p2c3)
  for (int k = 0; k < 3; ++k) U[5 + k] = sg * P[5 + k];             // (p2c4)
}

// Flux in direction d, Eq. (definition-of-flux), v~ = v - beta / alpha.
template <class T> void flux_dir(const PMetric<T>& m, const T* P, const PState<T>& s, const T* U, int d, T* F) {
  const T a = m.alpha;
  T vt[3];
  for (int i = 0; i < 3; ++i) vt[i] = P[1 + i] - m.beta[i] / a;
  F[0] = a * (U[0] * vt[d]);
  for (int j = 0; j < 3; ++j) {
    T t = U[1 + j] * vt[d] - s.blow[j] * U[5 + d] / s.W;
    if (j == d) t = t + m.sqrtg * s.Ps;
    F[1 + j] = a * t;
  }
  F[4] = a * (U[4] * vt[d] + m.sqrtg * s.Ps * P[1 + d] - s.ab0 * U[5 + d] / s.W);
  for (int k = 0; k < 3; ++k) F[5 + k] = a * (U[5 + k] * vt[d] - U[5 + d] * vt[k]);
}

// Characteristic speed bounds in direction d: 3+1 eigenvalues with the sound
// speed replaced by the fast magnetosonic bound c_f^2 = cs^2 + ca^2 - cs^2 ca^2 (R5).
template <class T> void speeds_dir(const PMetric<T>& m, const T* P, const PState<T>& s, double gam, int d, T& lp, T& lm) {
  const T cs2 = gam * s.p / s.rhoh;
  const T ca2 = s.b2 / (s.rhoh + s.b2);
  const T cf2 = cs2 + ca2 - cs2 * ca2;
  const T vd = P[1 + d];
  const T gdd = m.ginv[sym(d, d)];
  const T den = T(1.0) - s.v2 * cf2;
  const T disc = (T(1.0) - s.v2) * (gdd * den - vd * vd * (T(1.0) - cf2));
  const T root = sqrt(cf2) * sqrt(tmax(disc, T(0.0)));
  const T base = vd * (T(1.0) - cf2);
  lp = m.alpha * (base + root) / den - m.beta[d];
  lm = m.alpha * (base - root) / den - m.beta[d];
}

/* ------------------------------------------------------------------------ */
/* stress-energy tensor, Eq. (mhd-stress-energy-tensor), as a second path    */
/* ------------------------------------------------------------------------ */

template <class T> struct FourMetric {
  T g[4][4];     // g_{mu nu}
  T ginv[4][4];  // g^{mu nu}
};

template <class T> void four_metric(const PMetric<T>& m, FourMetric<T>& M) {
  T blow[3];
  for (int i = 0; i < 3; ++i)
    blow[i] = m.g[sym(i, 0)] * m.beta[0] + m.g[sym(i, 1)] * m.beta[1] + m.g[sym(i, 2)] * m.beta[2];
  T bb = blow[0] * m.beta[0] + blow[1] * m.beta[1] + blow[2] * m.beta[2];
  M.g[0][0] = -m.alpha * m.alpha + bb;
  for (int i = 0; i < 3; ++i) {
    M.g[0][1 + i] = blow[i];
    M.g[1 + i][0] = blow[i];
    for (int j = 0; j < 3; ++j) M.g[1 + i][1 + j] = m.g[sym(i, j)];
  }
  T ia2 = T(1.0) / (m.alpha * m.alpha);
  M.ginv[0][0] = -ia2;
  for (int i = 0; i < 3; ++i) {
    M.ginv[0][1 + i] = m.beta[i] * ia2;
    M.ginv[1 + i][0] = m.beta[i] * ia2;
    for (int j = 0; j < 3; ++j) M.ginv[1 + i][1 + j] = m.ginv[sym(i, j)] - m.beta[i] * m.beta[j] * ia2;
  }
}

// u^mu, b^mu and T^{mu nu}; b^2 is contracted with the 4-metric.
template <class T> void tmunu(const PMetric<T>& m, const FourMetric<T>& M, const T* P, double gam, T u[4], T b[4], T Tm[4][4]) {
  T W;
  {
    T v2 = T(0.0);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) v2 = v2 + m.g[sym(i, j)] * P[1 + i] * P[1 + j];
    W = T(1.0) / sqrt(T(1.0) - v2);
  }
  u[0] = W / m.alpha;
  for (int i = 0; i < 3; ++i) u[1 + i] = W * (P[1 + i] - m.beta[i] / m.alpha);  // Eq. (vel)
  T Bv = T(0.0);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Bv = Bv + m.g[sym(i, j)] * P[5 + i] * P[1 + j];
  b[0] = W * Bv / m.alpha;
  for (int i = 0; i < 3; ++i) b[1 + i] = (P[5 + i] + m.alpha * b[0] * u[1 + i]) / W;
  T b2 = T(0.0);
  for (int a = 0; a < 4; ++a)
    for (int c = 0; c < 4; ++c) b2 = b2 + M.g[a][c] * b[a] * b[c];
  T p = (gam - 1.0) * P[0] * P[4];
  T rhohs = P[0] + P[0] * P[4] + p + b2;
  T Ps = p + 0.5 * b2;
  for (int a = 0; a < 4; ++a)
    for (int c = 0; c < 4; ++c) Tm[a][c] = rhohs * u[a] * u[c] + Ps * M.ginv[a][c] - b[a] * b[c];
}

// Conserved variables from T^{mu nu}: D = alpha sqrt(gamma) rho u^0,
// S_j = alpha sqrt(gamma) T^0_j, tau = alpha^2 sqrt(gamma) T^00 - D.
template <class T> void cons_from_tmunu(const PMetric<T>& m, const T* P, double gam, T* U) {
  FourMetric<T> M;
  four_metric(m, M);
  T u[4], b[4], Tm[4][4];
  tmunu(m, M, P, gam, u, b, Tm);
  const T as = m.alpha * m.sqrtg;
  U[0] = as * P[0] * u[0];
  for (int j = 0; j < 3; ++j) {
    T t = T(0.0);
    for (int a = 0; a < 4; ++a) t = t + Tm[0][a] * M.g[a][1 + j];
    U[1 + j] = as * t;
  }
  U[4] = m.alpha * as * Tm[0][0] - U[0];
  for (int k = 0; k < 3; ++k) U[5 + k] = m.sqrtg * P[5 + k];
}

// Fluxes from the 4-vectors: F_D = alpha sqrt(g) rho u^d, F_Sj = alpha sqrt(g) T^d_j,
// F_tau = alpha sqrt(g) (alpha T^{0d} - rho u^d), F_B^k = alpha sqrt(g) (b^k u^d - b^d u^k).
template <class T> void flux_from_tmunu(const PMetric<T>& m, const T* P, double gam, int d, T* F) {
  FourMetric<T> M;
  four_metric(m, M);
  T u[4], b[4], Tm[4][4];
  tmunu(m, M, P, gam, u, b, Tm);
  const T as = m.alpha * m.sqrtg;
  F[0] = as * P[0] * u[1 + d];
  for (int j = 0; j < 3; ++j) {
    T t = T(0.0);
    for (int a = 0; a < 4; ++a) t = t + Tm[1 + d][a] * M.g[a][1 + j];
    F[1 + j] = as * t;
  }
  F[4] = as * (m.alpha * Tm[0][1 + d] - P[0] * u[1 + d]);
  for (int k = 0; k < 3; ++k) F[5 + k] = as * (b[1 + k] * u[1 + d] - b[1 + d] * u[1 + k]);
}

/* ------------------------------------------------------------------------ */
/* sources, Eq. (definition-of-source), static metric (d_t g = 0)           */
/* ------------------------------------------------------------------------ */

// d_e g_{mu nu} from the ADM derivatives by the chain rule.
template <class T> void four_metric_deriv(const PMetric<T>& m, const MetricDeriv& D, T dg[4][4][4]) {
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) dg[0][a][b] = T(0.0);  // static
  for (int e = 0; e < 3; ++e) {
    T blow[3], dblow[3];
    for (int i = 0; i < 3; ++i) {
      blow[i] = T(0.0);
      dblow[i] = T(0.0);
      for (int j = 0; j < 3; ++j) {
        blow[i] = blow[i] + m.g[sym(i, j)] * m.beta[j];
        dblow[i] = dblow[i] + D.dgamma[e][sym(i, j)] * m.beta[j] + m.g[sym(i, j)] * D.dbeta[e][j];
      }
    }
    T dbb = T(0.0);
    for (int i = 0; i < 3; ++i) dbb = dbb + dblow[i] * m.beta[i] + blow[i] * D.dbeta[e][i];
    T (*G)[4] = dg[1 + e];
    G[0][0] = -2.0 * m.alpha * D.dalpha[e] + dbb;
    for (int i = 0; i < 3; ++i) {
      G[0][1 + i] = dblow[i];
      G[1 + i][0] = dblow[i];
      for (int j = 0; j < 3; ++j) G[1 + i][1 + j] = T(D.dgamma[e][sym(i, j)]);
    }
  }
}

// Literal covariant form: Christoffels from g and dg, contracted with T^{mu nu}.
template <class T> void sources_covariant(const PMetric<T>& m, const MetricDeriv& D, const T* P, double gam, T* S) {
  FourMetric<T> M;
  four_metric(m, M);
  T u[4], b[4], Tm[4][4];
  tmunu(m, M, P, gam, u, b, Tm);
  T dg[4][4][4];  // dg[lam][mu][nu] = d_lam g_{mu nu}
  four_metric_deriv(m, D, dg);
  // Gamma^l_{mn} = 1/2 g^{ls} (d_m g_{sn} + d_n g_{sm} - d_s g_{mn})
  T Gam[4][4][4];
  for (int l = 0; l < 4; ++l)
    for (int a = 0; a < 4; ++a)
      for (int c = 0; c < 4; ++c) {
        T t = T(0.0);
        for (int s = 0; s < 4; ++s) t = t + M.ginv[l][s] * (dg[a][s][c] + dg[c][s][a] - dg[s][a][c]);
        Gam[l][a][c] = 0.5 * t;
      }
  const T as = m.alpha * m.sqrtg;
  S[0] = T(0.0);
  for (int j = 0; j < 3; ++j) {
    T t = T(0.0);
    for (int a = 0; a < 4; ++a)
      for (int c = 0; c < 4; ++c) {
        T gl = T(0.0);
        for (int l = 0; l < 4; ++l) gl = gl + Gam[l][a][c] * M.g[l][1 + j];
        t = t + Tm[a][c] * (dg[a][c][1 + j] - gl);
      }
    S[1 + j] = as * t;
  }
  T t1 = T(0.0);
  for (int a = 1; a < 4; ++a) t1 = t1 + Tm[a][0] * (D.dalpha[a - 1] / m.alpha);
  T t2 = T(0.0);
  for (int a = 0; a < 4; ++a)
    for (int c = 0; c < 4; ++c) t2 = t2 + Tm[a][c] * Gam[0][a][c];
  S[4] = as * m.alpha * (t1 - t2);
  S[5] = S[6] = S[7] = T(0.0);
}

// 3+1 form with the extrinsic curvature of a static slice,
// K_ij = (gamma_jk d_i beta^k + gamma_ik d_j beta^k + beta^k d_k gamma_ij) / (2 alpha).
template <class T> void sources_3p1(const PMetric<T>& m, const MetricDeriv& D, const T* P, double gam, T* S) {
  FourMetric<T> M;
  four_metric(m, M);
  T u[4], b[4], Tm[4][4];
  tmunu(m, M, P, gam, u, b, Tm);
  T K[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      T t = T(0.0);
      for (int k = 0; k < 3; ++k)
        t = t + m.g[sym(j, k)] * D.dbeta[i][k] + m.g[sym(i, k)] * D.dbeta[j][k] + m.beta[k] * D.dgamma[k][sym(i, j)];
      K[i][j] = t / (2.0 * m.alpha);
    }
  T blow[3];
  for (int i = 0; i < 3; ++i)
    blow[i] = m.g[sym(i, 0)] * m.beta[0] + m.g[sym(i, 1)] * m.beta[1] + m.g[sym(i, 2)] * m.beta[2];
  T T0low[3];  // T^0_i = T^00 beta_i + T^0k gamma_ki
  for (int i = 0; i < 3; ++i) {
    T t = Tm[0][0] * blow[i];
    for (int k = 0; k < 3; ++k) t = t + Tm[0][1 + k] * m.g[sym(k, i)];
    T0low[i] = t;
  }
  const T as = m.alpha * m.sqrtg;
  S[0] = T(0.0);
  for (int j = 0; j < 3; ++j) {
    T bbdg = T(0.0), tdg = T(0.0), t0bdg = T(0.0), t0db = T(0.0);
    for (int i = 0; i < 3; ++i) {
      t0db = t0db + T0low[i] * D.dbeta[j][i];
      for (int k = 0; k < 3; ++k) {
        bbdg = bbdg + m.beta[i] * m.beta[k] * D.dgamma[j][sym(i, k)];
        tdg = tdg + Tm[1 + i][1 + k] * D.dgamma[j][sym(i, k)];
        t0bdg = t0bdg + Tm[0][1 + i] * m.beta[k] * D.dgamma[j][sym(i, k)];
      }
    }
    S[1 + j] = as * (Tm[0][0] * (0.5 * bbdg - m.alpha * D.dalpha[j]) + t0bdg + t0db + 0.5 * tdg);
  }
  T bbK = T(0.0), bda = T(0.0), t0i = T(0.0), tK = T(0.0);
  for (int i = 0; i < 3; ++i) {
    bda = bda + m.beta[i] * D.dalpha[i];
    T bK = T(0.0);
    for (int j = 0; j < 3; ++j) {
      bbK = bbK + m.beta[i] * m.beta[j] * K[i][j];
      bK = bK + m.beta[j] * K[i][j];
      tK = tK + Tm[1 + i][1 + j] * K[i][j];
    }
    t0i = t0i + Tm[0][1 + i] * (2.0 * bK - D.dalpha[i]);
  }
  S[4] = as * (Tm[0][0] * (bbK - bda) + t0i + tK);
  S[5] = S[6] = S[7] = T(0.0);
}

/* ------------------------------------------------------------------------ */
/* con2prim: 3D Newton-Raphson in (W, z = rho h W^2, T = p / rho), Sec. II C */
/* ------------------------------------------------------------------------ */

enum { C2P_OK = 0, C2P_FLOOR = 1, C2P_NOCONV = 2, C2P_UNPHYS = 3, C2P_NONFINITE = 4, C2P_FALLBACK = 5 };

// rho, p: the atmosphere state; floor: densities below it are the atmosphere.
// The floor sits a relative 1e-6 above rho (a reading: the paper gives only the
// atmosphere's values).  The atmosphere state itself in a strong field has its
// thermal energy below the rounding of tau, so recovering it would succeed or
// fail on the last bit of tau; at the floor it is recognised before any recovery.
struct AtmData { double rho, p, floor; };

// Atmosphere state (Sec. IV, TOV test): rho = rho_atm, v = 0, p from the
// polytrope K rho^gamma_atm, eps = p / ((Gamma-1) rho), B kept; U rewritten.
template <class T> void atmosphere(const PMetric<T>& m, const Par& par, const AtmData& atm, T* U, T* P) {
  T Bup[3];
  for (int k = 0; k < 3; ++k) Bup[k] = U[5 + k] / m.sqrtg;
  P[0] = T(atm.rho);
  P[1] = P[2] = P[3] = T(0.0);
  P[4] = T(atm.p / ((par.gam - 1.0) * atm.rho));
  for (int k = 0; k < 3; ++k) P[5 + k] = Bup[k];
  PState<T> s;
  prim_state(m, P, par.gam, s);
  prim_to_cons(m, P, s, U);
}

// Undensitized conserved scalars entering the recovery.
template <class T> struct C2PIn {
  T Dt, St[3], taut, B[3];
  T S2, B2, SB;
};

// 3D Newton-Raphson on f(W, z, T) = 0 (Sec. II C).  The residuals follow from
// Eqs. (p2c1)-(p2c3) with S_j = (z + B^2) v_j - (B.v) B_j and B.v = S.B / z:
//   f1 = S^2 - (z+B^2)^2 (1 - W^-2) + (S.B)^2 (2z + B^2) / z^2
//   f2 = tau + D - z - B^2 + p + B^2 / (2 W^2) + (S.B)^2 / (2 z^2),  p = D T / W
//   f3 = z - D W (1 + Gamma T / (Gamma - 1))
// Stops when max_k |dx_k / x_k| < tol.  Returns true on convergence.
template <class T> bool newton3d(const C2PIn<T>& c, const Par& par, T& W, T& z, T& Tt) {
  const double gf = par.gam / (par.gam - 1.0);
  const T Dt = c.Dt, B2 = c.B2, SB2 = c.SB * c.SB, S2 = c.S2, taut = c.taut;
  bool conv = false;
  const int extra = extra_newton<T>::n;
  int post = 0;
  for (int it = 0; it < par.c2p_maxit + extra; ++it) {
    const T zB = z + B2;
    const T iW2 = T(1.0) / (W * W);
    const T iW3 = iW2 / W;
    const T iz2 = T(1.0) / (z * z);
    const T iz3 = iz2 / z;
    const T p = Dt * Tt / W;
    const T f1 = S2 - zB * zB * (T(1.0) - iW2) + SB2 * (2.0 * z + B2) * iz2;
    const T f2 = taut + Dt - z - B2 + p + 0.5 * B2 * iW2 + 0.5 * SB2 * iz2;
    const T f3 = z - Dt * W * (T(1.0) + gf * Tt);
    const T J11 = -2.0 * zB * zB * iW3;
    const T J12 = -2.0 * zB * (T(1.0) - iW2) - 2.0 * SB2 * zB * iz3;
    const T J13 = T(0.0);
    const T J21 = -Dt * Tt * iW2 - B2 * iW3;
    const T J22 = T(-1.0) - SB2 * iz3;
    const T J23 = Dt / W;
    const T J31 = -Dt * (T(1.0) + gf * Tt);
    const T J32 = T(1.0);
    const T J33 = -Dt * W * gf;
    // Cramer's rule for J dx = -f
    const T det = J11 * (J22 * J33 - J23 * J32) - J12 * (J21 * J33 - J23 * J31) + J13 * (J21 * J32 - J22 * J31);
    const T r1 = -f1, r2 = -f2, r3 = -f3;
    const T d1 = (r1 * (J22 * J33 - J23 * J32) - J12 * (r2 * J33 - J23 * r3) + J13 * (r2 * J32 - J22 * r3)) / det;
    const T d2 = (J11 * (r2 * J33 - J23 * r3) - r1 * (J21 * J33 - J23 * J31) + J13 * (J21 * r3 - r2 * J31)) / det;
    const T d3 = (J11 * (J22 * r3 - r2 * J32) - J12 * (J21 * r3 - r2 * J31) + r1 * (J21 * J32 - J22 * J31)) / det;
    W = W + d1;
    z = z + d2;
    Tt = Tt + d3;
    if (conv) {
      if (++post >= extra) break;
      continue;
    }
    if (!finite(W) || !finite(z) || !finite(Tt)) return false;
    const T err = tmax(fabs(d1 / W), tmax(fabs(d2 / z), fabs(d3 / Tt)));
    if (err < par.c2p_tol) {
      conv = true;
      if (extra == 0) break;
    }
  }
  return conv;
}

// Largest root of the Newman-Hamlin cubic x^3 + a x^2 + d = 0 (a < 0, d >= 0):
// Newton from x = -a, where f >= 0 and f is convex, so the iterates decrease
// monotonically onto the root.
template <class T> T nh_cubic_root(T a, T d) {
  T x = -a;
  for (int it = 0; it < 100; ++it) {
    const T f = x * x * (x + a) + d;
    const T fp = x * (3.0 * x + 2.0 * a);
    const T dx = f / fp;
    x = x - dx;
    if (!(fabs(dx) > 1e-15 * fabs(x))) break;
  }
  return x;
}

// One Newman-Hamlin map p -> p': with x = z + B^2 the energy and momentum
// equations combine into x^3 - (E + p + B^2/2) x^2 + (B^2 S^2 - (S.B)^2)/2 = 0,
// E = tau + D (the cubic of Sec. II C); its largest root gives z, then
// W^-2 = 1 - (S^2 + (S.B)^2 (2z + B^2) / z^2) / x^2, rho = D / W, rho h = z / W^2,
// and the Gamma-law EOS returns p' = (Gamma-1)/Gamma (rho h - rho).
template <class T> bool nh_map(const C2PIn<T>& c, double gam, T p, T& pn, T& W, T& z) {
  const T E = c.taut + c.Dt;
  const T dd = tmax(T(0.0), 0.5 * (c.B2 * c.S2 - c.SB * c.SB));
  const T a = -(E + p + 0.5 * c.B2);
  const T x = nh_cubic_root(a, dd);
  z = x - c.B2;
  if (!(z > 0.0)) return false;
  const T iW2 = T(1.0) - (c.S2 + c.SB * c.SB * (2.0 * z + c.B2) / (z * z)) / (x * x);
  if (!(iW2 > 0.0)) return false;
  W = T(1.0) / sqrt(iW2);
  const T rho = c.Dt / W;
  const T rhoh = z * iW2;
  pn = ((gam - 1.0) / gam) * (rhoh - rho);
  return finite(pn);
}

// Newman-Hamlin fallback (Sec. II C): fixed-point iteration on the pressure,
// with Aitken extrapolation on every third iterate.  On success returns the
// (W, z, T) that seed a final Newton polish.
template <class T> bool newman_hamlin(const C2PIn<T>& c, const Par& par, T p0, T& W, T& z, T& Tt) {
  T s0 = p0, s1 = p0, s2 = p0;  // s2 = current iterate, s1, s0 = the two before it
  for (int k = 0; k < par.c2p_maxit; ++k) {
    T pn;
    if (!nh_map(c, par.gam, s2, pn, W, z)) return false;
    if (!(pn > 0.0)) return false;
    if (fabs(pn - s2) <= par.c2p_tol * fabs(pn)) {
      Tt = pn * W / c.Dt;
      return true;
    }
    if ((k + 1) % 3 == 0) {
      const T den = pn - 2.0 * s2 + s1;
      if (!(den == 0.0)) {
        const T pa = pn - (pn - s2) * (pn - s2) / den;
        if (pa > 0.0 && finite(pa)) pn = pa;
      }
    }
    s0 = s1;
    s1 = s2;
    s2 = pn;
  }
  (void)s0;
  return false;
}

// Physicality of a recovered (W, z, T) and the primitives it gives.
template <class T> int recover(const PMetric<T>& m, const C2PIn<T>& c, const Par& par, T W, T z, T Tt, T* Pout) {
  const T zB = z + c.B2;
  const T rho = c.Dt / W;
  T vlow[3], v[3];
  for (int j = 0; j < 3; ++j)
    vlow[j] = (c.St[j] + (c.SB / z) * (m.g[sym(j, 0)] * c.B[0] + m.g[sym(j, 1)] * c.B[1] + m.g[sym(j, 2)] * c.B[2])) / zB;
  for (int i = 0; i < 3; ++i) v[i] = m.ginv[sym(i, 0)] * vlow[0] + m.ginv[sym(i, 1)] * vlow[1] + m.ginv[sym(i, 2)] * vlow[2];
  const T v2 = vlow[0] * v[0] + vlow[1] * v[1] + vlow[2] * v[2];
  if (!(W >= 1.0) || !(z > 0.0) || !(Tt > 0.0) || !(rho > 0.0) || !(v2 < 1.0)) return C2P_UNPHYS;
  Pout[0] = rho;
  Pout[1] = v[0];
  Pout[2] = v[1];
  Pout[3] = v[2];
  Pout[4] = Tt / (par.gam - 1.0);
  for (int k = 0; k < 3; ++k) Pout[5 + k] = c.B[k];
  return C2P_OK;
}

// Undensitize U (divide by sqrt(gamma)) and form S^2 = gamma^ij S_i S_j,
// B^2 = gamma_ij B^i B^j and S.B = S_i B^i.
template <class T> void c2p_inputs(const PMetric<T>& m, const T* U, C2PIn<T>& c) {
  c.Dt = U[0] / m.sqrtg;
  for (int j = 0; j < 3; ++j) c.St[j] = U[1 + j] / m.sqrtg;
  c.taut = U[4] / m.sqrtg;
  for (int k = 0; k < 3; ++k) c.B[k] = U[5 + k] / m.sqrtg;
  c.S2 = T(0.0);
  c.B2 = T(0.0);
  c.SB = T(0.0);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      c.S2 = c.S2 + m.ginv[sym(i, j)] * c.St[i] * c.St[j];
      c.B2 = c.B2 + m.g[sym(i, j)] * c.B[i] * c.B[j];
    }
  for (int i = 0; i < 3; ++i) c.SB = c.SB + c.St[i] * c.B[i];
}

template <class T> int con2prim_point(const PMetric<T>& m, const Par& par, const AtmData& atm, T* U, T* P) {
  for (int q = 0; q < 8; ++q)
    if (!finite(U[q])) {
      for (int k = 0; k < 3; ++k) U[5 + k] = finite(U[5 + k]) ? U[5 + k] : T(0.0);
      atmosphere(m, par, atm, U, P);
      return C2P_NONFINITE;
    }
  const double gam = par.gam;
  const double gf = gam / (gam - 1.0);
  C2PIn<T> c;
  c2p_inputs(m, U, c);
  if (c.Dt < atm.floor) {
    atmosphere(m, par, atm, U, P);
    return C2P_FLOOR;
  }

  // initial guess from the supplied primitives
  T W, z, Tt, p0;
  {
    T v2 = T(0.0);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) v2 = v2 + m.g[sym(i, j)] * P[1 + i] * P[1 + j];
    bool ok = finite(v2) && v2 < 1.0 && P[0] > 0.0 && P[4] > 0.0 && finite(P[0]) && finite(P[4]);
    if (ok) {
      W = T(1.0) / sqrt(T(1.0) - v2);
      p0 = (gam - 1.0) * P[0] * P[4];
      z = (P[0] + P[0] * P[4] + p0) * W * W;
      Tt = p0 / P[0];
    } else {  // no usable guess: fluid at rest with the available energy
      W = T(1.0);
      Tt = (gam - 1.0) * tmax(c.taut - 0.5 * c.B2, T(1e-10) * c.Dt) / c.Dt;
      z = c.Dt * (T(1.0) + gf * Tt);
      p0 = c.Dt * Tt;
    }
  }
  T Pn[8];
  int st = C2P_NOCONV;
  {
    T W1 = W, z1 = z, T1 = Tt;
    if (newton3d(c, par, W1, z1, T1)) st = recover(m, c, par, W1, z1, T1, Pn);
  }
  if (st != C2P_OK) {  // fallback chain: Newman-Hamlin, then a Newton polish from its solution
    T W2, z2, T2;
    int st2 = C2P_NOCONV;
    if (newman_hamlin(c, par, p0, W2, z2, T2) && newton3d(c, par, W2, z2, T2)) st2 = recover(m, c, par, W2, z2, T2, Pn);
    if (st2 == C2P_OK)
      st = C2P_FALLBACK;
    else if (st == C2P_NOCONV)
      st = st2;
  }
  if (st != C2P_OK && st != C2P_FALLBACK) {
    atmosphere(m, par, atm, U, P);
    return st;
  }
  if (Pn[0] < atm.floor) {
    atmosphere(m, par, atm, U, P);
    return C2P_FLOOR;
  }
  for (int q = 0; q < 8; ++q) P[q] = Pn[q];
  return st;
}

/* ------------------------------------------------------------------------ */
/* reconstruction, Sec. II C                                                */
/* ------------------------------------------------------------------------ */

// TVD with the minmod limiter [Toro].
template <class T> T minmod(T a, T b) {
  if (a * b <= 0.0) return T(0.0);
  return (fabs(a) < fabs(b)) ? a : b;
}

// WENO5 value at the right face of the centre cell c of (a, b, c, d, e):
// three third-order candidates blended with Jiang-Shu or Borges (Z) weights.
// mode: 0 = JS, 1 = Z, 2 = linear weights only.
template <class T> T weno5_face(T a, T b, T c, T d, T e, int mode, double eps, int zp) {
  const T q0 = (2.0 * a - 7.0 * b + 11.0 * c) / 6.0;
  const T q1 = (-b + 5.0 * c + 2.0 * d) / 6.0;
  const T q2 = (2.0 * c + 5.0 * d - e) / 6.0;
  const double d0 = 0.1, d1 = 0.6, d2 = 0.3;
  if (mode == 2) return d0 * q0 + d1 * q1 + d2 * q2;
  const T b0 = (13.0 / 12.0) * sq(a - 2.0 * b + c) + 0.25 * sq(a - 4.0 * b + 3.0 * c);
  const T b1 = (13.0 / 12.0) * sq(b - 2.0 * c + d) + 0.25 * sq(b - d);
  const T b2 = (13.0 / 12.0) * sq(c - 2.0 * d + e) + 0.25 * sq(3.0 * c - 4.0 * d + e);
  T w0, w1, w2;
  if (mode == 0) {
    w0 = d0 / sq(eps + b0);
    w1 = d1 / sq(eps + b1);
    w2 = d2 / sq(eps + b2);
  } else {
    const T tau = fabs(b0 - b2);
    T r0 = tau / (b0 + eps), r1 = tau / (b1 + eps), r2 = tau / (b2 + eps);
    if (zp == 2) {
      r0 = r0 * r0;
      r1 = r1 * r1;
      r2 = r2 * r2;
    }
    w0 = d0 * (1.0 + r0);
    w1 = d1 * (1.0 + r1);
    w2 = d2 * (1.0 + r2);
  }
  const T s = w0 + w1 + w2;
  return (w0 * q0 + w1 * q1 + w2 * q2) / s;
}

// Left and right states at the face between s[2] and s[3] of a six-cell
// stencil s[0..5] (cells c-3 .. c+2 around face c-1/2).
template <class T> void recon_face(const Par& par, const T* s, T& qL, T& qR, int linear = 0) {
  if (par.recon == REC_MINMOD) {
    T sl = minmod(s[2] - s[1], s[3] - s[2]);
    T sr = minmod(s[3] - s[2], s[4] - s[3]);
    qL = s[2] + 0.5 * sl;
    qR = s[3] - 0.5 * sr;
    return;
  }
  int mode = linear ? 2 : (par.recon == REC_WENOZ ? 1 : 0);
  double eps = (par.recon == REC_WENOZ) ? par.wenoz_eps : par.weno_eps;
  qL = weno5_face(s[0], s[1], s[2], s[3], s[4], mode, eps, par.wenoz_p);
  qR = weno5_face(s[5], s[4], s[3], s[2], s[1], mode, eps, par.wenoz_p);
}

/* ------------------------------------------------------------------------ */
/* HLLE flux [Harten-Lax-van Leer, Einfeldt], Sec. II C                     */
/* ------------------------------------------------------------------------ */

template <class T> void hlle(const PMetric<T>& m, const T* PL, const T* PR, double gam, int d, T* Fs, T& xip, T& xim) {
  PState<T> sL, sR;
  prim_state(m, PL, gam, sL);
  prim_state(m, PR, gam, sR);
  T UL[8], UR[8], FL[8], FR[8];
  prim_to_cons(m, PL, sL, UL);
  prim_to_cons(m, PR, sR, UR);
  flux_dir(m, PL, sL, UL, d, FL);
  flux_dir(m, PR, sR, UR, d, FR);
  T lpL, lmL, lpR, lmR;
  speeds_dir(m, PL, sL, gam, d, lpL, lmL);
  speeds_dir(m, PR, sR, gam, d, lpR, lmR);
  xip = tmax(T(0.0), tmax(lpL, lpR));
  xim = tmin(T(0.0), tmin(lmL, lmR));
  const T den = xip - xim;
  for (int q = 0; q < 8; ++q) {
    if (den > 0.0)
      Fs[q] = (xip * FL[q] - xim * FR[q] + xip * xim * (UR[q] - UL[q])) / den;
    else
      Fs[q] = 0.5 * (FL[q] + FR[q]);
  }
}

// Positivity check of a reconstructed state with the face metric (R8).
template <class T> bool state_ok(const PMetric<T>& m, const T* P) {
  T v2 = T(0.0);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) v2 = v2 + m.g[sym(i, j)] * P[1 + i] * P[1 + j];
  for (int q = 0; q < 8; ++q)
    if (!finite(P[q])) return false;
  return (P[0] > 0.0) && (P[4] > 0.0) && (v2 < 1.0);
}

/* ------------------------------------------------------------------------ */
/* box-level operations                                                     */
/* ------------------------------------------------------------------------ */

static int nthreads_req = 1;

static long bc_map(long i, int n, int lo, int hi) {
  if (i < 0) return lo == BC_PERIODIC ? ((i % n) + n) % n : 0;
  if (i >= n) return hi == BC_PERIODIC ? i % n : n - 1;
  return i;
}

// Boundary conditions on P (Sec. IV A, "copy" for outflow; periodic wrap).
template <class T> void fill_ghosts(const Box& bx, const Geo& G, T* P) {
  const int g = G.ng;
  for (int f = 0; f < 8; ++f) {
    T* q = P + f * G.ncell;
    for (long k = -g; k < G.n[2] + g; ++k)
      for (long j = -g; j < G.n[1] + g; ++j)
        for (long i = -g; i < G.n[0] + g; ++i) {
          bool inside = (i >= 0 && i < G.n[0] && j >= 0 && j < G.n[1] && k >= 0 && k < G.n[2]);
          if (inside) continue;
          long si = bc_map(i, G.n[0], bx.bc[0], bx.bc[1]);
          long sj = bc_map(j, G.n[1], bx.bc[2], bx.bc[3]);
          long sk = bc_map(k, G.n[2], bx.bc[4], bx.bc[5]);
          q[G.c(i, j, k)] = q[G.c(si, sj, sk)];
        }
  }
}

static AtmData atm_of(const Par& par) {
  AtmData a;
  a.rho = par.rho_atm;
  a.floor = par.rho_atm * (1.0 + 1e-6);
  a.p = par.atm_K * std::pow(par.rho_atm, par.atm_gamma);
  return a;
}

template <class T> long con2prim_box(const Box& bx, const Par& par, const VMetric& vm, T* U, T* P, int32_t* status) {
  Geo G(bx);
  AtmData atm = atm_of(par);
  long nfail = 0;
#pragma omp parallel for reduction(+ : nfail) schedule(static) num_threads(nthreads_req)
  for (long k = 0; k < G.n[2]; ++k)
    for (long j = 0; j < G.n[1]; ++j)
      for (long i = 0; i < G.n[0]; ++i) {
        PMetric<T> m;
        metric_centre(G, vm, i, j, k, m);
        long c = G.c(i, j, k);
        T u[8], p[8];
        for (int q = 0; q < 8; ++q) {
          u[q] = U[q * G.ncell + c];
          p[q] = P[q * G.ncell + c];
        }
        int st = con2prim_point(m, par, atm, u, p);
        for (int q = 0; q < 8; ++q) {
          U[q * G.ncell + c] = u[q];
          P[q * G.ncell + c] = p[q];
        }
        if (status) status[c] = st;
        if (st >= C2P_NOCONV && st <= C2P_NONFINITE) ++nfail;
      }
  return nfail;
}

template <class T> void prim2con_box(const Box& bx, const Par& par, const VMetric& vm, const T* P, T* U) {
  Geo G(bx);
#pragma omp parallel for schedule(static) num_threads(nthreads_req)
  for (long k = 0; k < G.n[2]; ++k)
    for (long j = 0; j < G.n[1]; ++j)
      for (long i = 0; i < G.n[0]; ++i) {
        PMetric<T> m;
        metric_centre(G, vm, i, j, k, m);
        long c = G.c(i, j, k);
        T p[8], u[8];
        for (int q = 0; q < 8; ++q) p[q] = P[q * G.ncell + c];
        PState<T> s;
        prim_state(m, p, par.gam, s);
        prim_to_cons(m, p, s, u);
        for (int q = 0; q < 8; ++q) U[q * G.ncell + c] = u[q];
      }
}

// RHS from given primitives (steps 2-4 of the paper's RHS evaluation):
// dUdt = -sum_d (F_{+1/2} - F_{-1/2}) / dx_d + S on interior cells.
// Face fluxes of the magnetic field components, kept for constrained transport:
// f[d][c * nface_d + fi] = the HLLE flux through d-faces of Bcal^c, fi = face
// index (k * nf_y + j) * nf_x + i over the face grid of direction d.
template <class T> struct MagFlux {
  std::vector<T> f[3];
  long nf[3][3];
};

template <class T> void rhs_from_prims(const Box& bx, const Par& par, const VMetric& vm, T* P, T* dUdt, double* max_rate,
                                       MagFlux<T>* mf = nullptr) {
  Geo G(bx);
  fill_ghosts(bx, G, P);
  for (int q = 0; q < 8; ++q)
    for (long c = 0; c < G.ncell; ++c) dUdt[q * G.ncell + c] = T(0.0);
  // sources
#pragma omp parallel for schedule(static) num_threads(nthreads_req)
  for (long k = 0; k < G.n[2]; ++k)
    for (long j = 0; j < G.n[1]; ++j)
      for (long i = 0; i < G.n[0]; ++i) {
        PMetric<T> m;
        metric_centre(G, vm, i, j, k, m);
        MetricDeriv D;
        metric_deriv(G, vm, bx, i, j, k, D);
        long c = G.c(i, j, k);
        T p[8], S[8];
        for (int q = 0; q < 8; ++q) p[q] = P[q * G.ncell + c];
        sources_covariant(m, D, p, par.gam, S);
        for (int q = 0; q < 8; ++q) dUdt[q * G.ncell + c] = S[q];
      }
  double rate = 0.0;
  for (int d = 0; d < 3; ++d) {
    long nf[3] = {G.n[0], G.n[1], G.n[2]};
    nf[d] += 1;
    const long nface = nf[0] * nf[1] * nf[2];
    std::vector<T> F(8 * nface);
    long st[3] = {1, G.NX, G.NX * G.NY};
    double drate = 0.0;
#pragma omp parallel for reduction(max : drate) schedule(static) num_threads(nthreads_req)
    for (long k = 0; k < nf[2]; ++k)
      for (long j = 0; j < nf[1]; ++j)
        for (long i = 0; i < nf[0]; ++i) {
          // face between cells (i,j,k) - e_d and (i,j,k)
          long c = G.c(i, j, k);
          T PL[8], PR[8], s[6];
          for (int q = 0; q < 8; ++q) {
            for (int o = 0; o < 6; ++o) s[o] = P[q * G.ncell + c + (o - 3) * st[d]];
            recon_face(par, s, PL[q], PR[q]);
          }
          PMetric<T> m;
          metric_face(G, vm, d, i, j, k, m);
          if (!state_ok(m, PL))
            for (int q = 0; q < 8; ++q) PL[q] = P[q * G.ncell + c - st[d]];
          if (!state_ok(m, PR))
            for (int q = 0; q < 8; ++q) PR[q] = P[q * G.ncell + c];
          T Fs[8], xp, xm;
          hlle(m, PL, PR, par.gam, d, Fs, xp, xm);
          long fi = (k * nf[1] + j) * nf[0] + i;
          for (int q = 0; q < 8; ++q) F[q * nface + fi] = Fs[q];
          double r = std::max(val(xp), -val(xm)) / bx.dx[d];
          drate = std::max(drate, r);
        }
    rate = std::max(rate, drate);
    if (mf) {
      for (int e = 0; e < 3; ++e) mf->nf[d][e] = nf[e];
      mf->f[d].assign(F.begin() + 5 * nface, F.begin() + 8 * nface);
    }
#pragma omp parallel for schedule(static) num_threads(nthreads_req)
    for (long k = 0; k < G.n[2]; ++k)
      for (long j = 0; j < G.n[1]; ++j)
        for (long i = 0; i < G.n[0]; ++i) {
          long lo = (k * nf[1] + j) * nf[0] + i;
          long e[3] = {i, j, k};
          e[d] += 1;
          long hi = (e[2] * nf[1] + e[1]) * nf[0] + e[0];
          long c = G.c(i, j, k);
          for (int q = 0; q < 8; ++q)
            dUdt[q * G.ncell + c] = dUdt[q * G.ncell + c] + (F[q * nface + lo] - F[q * nface + hi]) / bx.dx[d];
        }
  }
  if (max_rate) *max_rate = std::max(*max_rate, rate);
}

// SSPRK3 (Shu-Osher) in the form U_{s+1} = U^n + c_s ((U_s - U^n) + dt L(U_s)),
// c = (1, 1/4, 2/3), which equals the textbook convex combinations and keeps a
// state with L = 0 unchanged bit for bit.  scheme 1 = SSPRK2 (Heun), c = (1, 1/2).
// Classic fourth-order Runge-Kutta (scheme 2): stage states U_{s+1} = U^n + a_s dt
// L(U_s), a = (1/2, 1/2, 1), and U^{n+1} = U^n + dt (L_0 + 2 L_1 + 2 L_2 + L_3) / 6,
// accumulated stage by stage as A_s = A_{s-1} + b_s dt L_s from A_{-1} = U^n,
// b = (1/6, 1/3, 1/3, 1/6).  No checkpoints (the adjoint covers the SSPRK schemes).
template <class T> long rk4_step_box(const Box& bx, const Par& par, const VMetric& vm, T* U, T* P, double dt,
                                     double* max_rate) {
  Geo G(bx);
  const long N = 8 * G.ncell;
  static const double a[3] = {0.5, 0.5, 1.0};
  static const double b[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
  long nfail = con2prim_box(bx, par, vm, U, P, (int32_t*)nullptr);
  std::vector<T> Un(U, U + N), A(U, U + N), L(N);
  for (int s = 0; s < 4; ++s) {
    if (s > 0) nfail += con2prim_box(bx, par, vm, U, P, (int32_t*)nullptr);
    rhs_from_prims(bx, par, vm, P, L.data(), max_rate);
    for (int q = 0; q < 8; ++q)
      for (long k = 0; k < G.n[2]; ++k)
        for (long j = 0; j < G.n[1]; ++j)
          for (long i = 0; i < G.n[0]; ++i) {
            long x = q * G.ncell + G.c(i, j, k);
            A[x] = A[x] + (b[s] * dt) * L[x];
            U[x] = (s < 3) ? Un[x] + (a[s] * dt) * L[x] : A[x];
          }
  }
  nfail += con2prim_box(bx, par, vm, U, P, (int32_t*)nullptr);
  return nfail;
}

template <class T> long rk_step_box(const Box& bx, const Par& par, const VMetric& vm, T* U, T* P, double dt, int scheme,
                                    T* ckpt, double* max_rate) {
  if (scheme == 2) return rk4_step_box(bx, par, vm, U, P, dt, max_rate);
  Geo G(bx);
  const long N = 8 * G.ncell;
  static const double c3[3] = {1.0, 0.25, 2.0 / 3.0};
  static const double c2[2] = {1.0, 0.5};
  const double* cs = scheme == 1 ? c2 : c3;
  const int nst = scheme == 1 ? 2 : 3;
  long nfail = con2prim_box(bx, par, vm, U, P, (int32_t*)nullptr);
  std::vector<T> Un(U, U + N), L(N);
  for (int s = 0; s < nst; ++s) {
    if (s > 0) nfail += con2prim_box(bx, par, vm, U, P, (int32_t*)nullptr);
    if (ckpt) std::copy(U, U + N, ckpt + s * N);
    rhs_from_prims(bx, par, vm, P, L.data(), max_rate);
    for (int q = 0; q < 8; ++q)
      for (long k = 0; k < G.n[2]; ++k)
        for (long j = 0; j < G.n[1]; ++j)
          for (long i = 0; i < G.n[0]; ++i) {
            long x = q * G.ncell + G.c(i, j, k);
            U[x] = Un[x] + cs[s] * ((U[x] - Un[x]) + dt * L[x]);
          }
  }
  nfail += con2prim_box(bx, par, vm, U, P, (int32_t*)nullptr);
  return nfail;
}

/* ------------------------------------------------------------------------ */
/* constrained transport (Sec. III B: vector potential on cell edges)       */
/* ------------------------------------------------------------------------ */
//
// A_e lives on the edges along axis e: at cell index c_e along e and vertex
// indices along the two other axes, stored like a vertex field (index
// G.v(i, j, k) with the cell index along e in place of that vertex index).
// The face field is Bcal = curl A (Bcal^d = d_a A_b - d_b A_a, a = d+1, b = d+2
// cyclic), so its discrete divergence vanishes identically; the cell-centred
// Bcal entering U is the mean of a cell's two d-face values.  The induction
// equation d_t Bcal^d + d_j F^j(Bcal^d) = 0 follows from d_t A_e = F^a(Bcal^b)
// = -F^b(Bcal^a) (the flux is antisymmetric): at an edge each of the two is the
// mean of the HLLE fluxes on the two faces beside it, and the edge value is
// their mean (R28).  The gauge term of the potential is a gradient, which curl
// removes: it is left out.

// vertex-shaped storage index of grid point (x, y, z) (cell or vertex indices)
static long vidx(const Geo& G, long x, long y, long z) { return G.v(x, y, z); }

// face index of the d-face with (i, j, k) on the face grid nf[d]
template <class T> static long face_at(const MagFlux<T>& mf, int d, long i, long j, long k) {
  return (k * mf.nf[d][1] + j) * mf.nf[d][0] + i;
}

// interior cell index along an axis for a transverse neighbour just outside the
// box (the boundary map of the primitives: the fluxes of a ghost column are
// those of the column it copies)
static long col_map(const Box& bx, int axis, long c) { return bc_map(c, bx.n[axis], bx.bc[2 * axis], bx.bc[2 * axis + 1]); }

// dA/dt on every interior edge from the magnetic face fluxes.
template <class T> void ct_edge_rhs(const Box& bx, const MagFlux<T>& mf, T* dA) {
  Geo G(bx);
  for (int q = 0; q < 3; ++q)
    for (long x = 0; x < G.nvert; ++x) dA[q * G.nvert + x] = T(0.0);
  for (int e = 0; e < 3; ++e) {
    const int a = (e + 1) % 3, b = (e + 2) % 3;
    long hi[3];
    for (int d = 0; d < 3; ++d) hi[d] = (d == e) ? bx.n[d] : bx.n[d] + 1;
    for (long z = 0; z < hi[2]; ++z)
      for (long y = 0; y < hi[1]; ++y)
        for (long x = 0; x < hi[0]; ++x) {
          const long p[3] = {x, y, z};
          // F^a(Bcal^b) on the a-faces at vertex p[a] along a, cells p[b]-1 and p[b] along b
          T fa = T(0.0), fb = T(0.0);
          for (int side = 0; side < 2; ++side) {
            long c[3] = {p[0], p[1], p[2]};
            c[b] = col_map(bx, b, p[b] - 1 + side);
            fa = fa + mf.f[a][b * (mf.nf[a][0] * mf.nf[a][1] * mf.nf[a][2]) + face_at(mf, a, c[0], c[1], c[2])];
            long c2[3] = {p[0], p[1], p[2]};
            c2[a] = col_map(bx, a, p[a] - 1 + side);
            fb = fb + mf.f[b][a * (mf.nf[b][0] * mf.nf[b][1] * mf.nf[b][2]) + face_at(mf, b, c2[0], c2[1], c2[2])];
          }
          dA[e * G.nvert + vidx(G, x, y, z)] = 0.5 * (0.5 * fa - 0.5 * fb);
        }
  }
}

// Face field Bcal^d on every interior d-face: out[d * G.ncell + G.c(i, j, k)] for
// the d-face at vertex index (i, j, k)[d] along d (cell-shaped storage; the face
// at n along d sits in the first ghost cell).
template <class T> void ct_face_field(const Box& bx, const T* A, T* out) {
  Geo G(bx);
  for (int d = 0; d < 3; ++d) {
    const int a = (d + 1) % 3, b = (d + 2) % 3;
    long hi[3] = {bx.n[0], bx.n[1], bx.n[2]};
    hi[d] += 1;
    for (long k = 0; k < hi[2]; ++k)
      for (long j = 0; j < hi[1]; ++j)
        for (long i = 0; i < hi[0]; ++i) {
          const long p[3] = {i, j, k};
          long pa[3] = {i, j, k}, pb[3] = {i, j, k};
          pa[a] += 1;  // the b-edge one vertex up along a
          pb[b] += 1;  // the a-edge one vertex up along b
          const T dAb = A[b * G.nvert + vidx(G, pa[0], pa[1], pa[2])] - A[b * G.nvert + vidx(G, p[0], p[1], p[2])];
          const T dAa = A[a * G.nvert + vidx(G, pb[0], pb[1], pb[2])] - A[a * G.nvert + vidx(G, p[0], p[1], p[2])];
          out[d * G.ncell + G.c(i, j, k)] = dAb / bx.dx[a] - dAa / bx.dx[b];
        }
  }
}

// U's Bcal (fields 5..7) on interior cells from A: the mean of the two face values.
template <class T> void ct_cell_field(const Box& bx, const T* A, T* U) {
  Geo G(bx);
  std::vector<T> Bf(3 * G.ncell);
  ct_face_field(bx, A, Bf.data());
  for (int d = 0; d < 3; ++d) {
    long up[3] = {0, 0, 0};
    up[d] = 1;
    for (long k = 0; k < bx.n[2]; ++k)
      for (long j = 0; j < bx.n[1]; ++j)
        for (long i = 0; i < bx.n[0]; ++i)
          U[(5 + d) * G.ncell + G.c(i, j, k)] =
              0.5 * (Bf[d * G.ncell + G.c(i, j, k)] + Bf[d * G.ncell + G.c(i + up[0], j + up[1], k + up[2])]);
  }
}

// One method-of-lines step with constrained transport: U^n's Bcal from A^n,
// con2prim (unless p_current), then per stage the RHS of U (its Bcal components
// are replaced), dA/dt from the stage's magnetic face fluxes, the same stage
// combine for U and A, and U_{s+1}'s Bcal from A_{s+1} before its con2prim.
template <class T> long ct_step_box(const Box& bx, const Par& par, const VMetric& vm, T* U, T* P, T* A, double dt,
                                    int scheme, int p_current, double* max_rate) {
  Geo G(bx);
  const long N = 8 * G.ncell, NA = 3 * G.nvert;
  ct_cell_field(bx, A, U);
  long nfail = p_current ? 0 : con2prim_box(bx, par, vm, U, P, (int32_t*)nullptr);
  std::vector<T> Un(U, U + N), An(A, A + NA), L(N), LA(NA);
  if (scheme == 2) {  // classic RK4 (as rk4_step_box)
    static const double a4[3] = {0.5, 0.5, 1.0};
    static const double b4[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    std::vector<T> Acc(U, U + N), AccA(A, A + NA);
    for (int s = 0; s < 4; ++s) {
      if (s > 0) nfail += con2prim_box(bx, par, vm, U, P, (int32_t*)nullptr);
      MagFlux<T> mf;
      rhs_from_prims(bx, par, vm, P, L.data(), max_rate, &mf);
      ct_edge_rhs(bx, mf, LA.data());
      for (long x = 0; x < N; ++x) {
        Acc[x] = Acc[x] + (b4[s] * dt) * L[x];
        U[x] = (s < 3) ? Un[x] + (a4[s] * dt) * L[x] : Acc[x];
      }
      for (long x = 0; x < NA; ++x) {
        AccA[x] = AccA[x] + (b4[s] * dt) * LA[x];
        A[x] = (s < 3) ? An[x] + (a4[s] * dt) * LA[x] : AccA[x];
      }
      ct_cell_field(bx, A, U);
    }
  } else {
    static const double c3[3] = {1.0, 0.25, 2.0 / 3.0};
    static const double c2[2] = {1.0, 0.5};
    const double* cs = scheme == 1 ? c2 : c3;
    const int nst = scheme == 1 ? 2 : 3;
    for (int s = 0; s < nst; ++s) {
      if (s > 0) nfail += con2prim_box(bx, par, vm, U, P, (int32_t*)nullptr);
      MagFlux<T> mf;
      rhs_from_prims(bx, par, vm, P, L.data(), max_rate, &mf);
      ct_edge_rhs(bx, mf, LA.data());
      for (long x = 0; x < N; ++x) U[x] = Un[x] + cs[s] * ((U[x] - Un[x]) + dt * L[x]);
      for (long x = 0; x < NA; ++x) A[x] = An[x] + cs[s] * ((A[x] - An[x]) + dt * LA[x]);
      ct_cell_field(bx, A, U);
    }
  }
  nfail += con2prim_box(bx, par, vm, U, P, (int32_t*)nullptr);
  return nfail;
}

VMetric make_vm(const Box& bx, const double* alpha, const double* beta, const double* gamma) {
  Geo G(bx);
  VMetric vm;
  vm.alpha = alpha;
  vm.beta = beta;
  vm.gamma = gamma;
  vm.stride = G.nvert;
  return vm;
}

PMetric<double> point_metric(double alpha, const double* beta, const double* g) {
  PMetric<double> m;
  m.alpha = alpha;
  for (int i = 0; i < 3; ++i) m.beta[i] = beta ? beta[i] : 0.0;
  for (int i = 0; i < 6; ++i) m.g[i] = g[i];
  metric_finish(m);
  return m;
}

}  // namespace

/* ------------------------------------------------------------------------ */
/* C ABI (host pointers; one box per call; arrays sized for that box)       */
/* ------------------------------------------------------------------------ */

extern "C" {

void orc_set_threads(int n) { nthreads_req = n < 1 ? 1 : n; }

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_prim2con(const Box* bx, const Par* par, const double* alpha, const double* beta, const double* gamma,
                  const double* P, double* U) {
  prim2con_box(*bx, *par, make_vm(*bx, alpha, beta, gamma), P, U);
}

long orc_con2prim(const Box* bx, const Par* par, const double* alpha, const double* beta, const double* gamma,
                  double* U, double* P, int32_t* status) {
  return con2prim_box(*bx, *par, make_vm(*bx, alpha, beta, gamma), U, P, status);
}

// U -> dU/dt (con2prim, then steps 2-4), U and P updated by con2prim.
long orc_rhs(const Box* bx, const Par* par, const double* alpha, const double* beta, const double* gamma, double* U,
             double* P, double* dUdt, double* max_rate) {
  VMetric vm = make_vm(*bx, alpha, beta, gamma);
  long nfail = con2prim_box(*bx, *par, vm, U, P, (int32_t*)nullptr);
  rhs_from_prims(*bx, *par, vm, P, dUdt, max_rate);
  return nfail;
}

long orc_rk_step(const Box* bx, const Par* par, const double* alpha, const double* beta, const double* gamma,
                 double* U, double* P, double dt, int scheme, double* ckpt, double* max_rate) {
  return rk_step_box(*bx, *par, make_vm(*bx, alpha, beta, gamma), U, P, dt, scheme, ckpt, max_rate);
}

// Jacobian-vector product of nsteps RK steps: (U, dU) -> (U_out, dU_out), exact
// to round-off through dual numbers.  P is the guess in and the result out.
long orc_rk_step_jvp(const Box* bx, const Par* par, const double* alpha, const double* beta, const double* gamma,
                     double* U, double* dU, double* P, double dt, int scheme, int nsteps) {
  Geo G(*bx);
  const long N = 8 * G.ncell;
  std::vector<Dual> Ud(N), Pd(N);
  for (long x = 0; x < N; ++x) {
    Ud[x] = Dual(U[x], dU[x]);
    Pd[x] = Dual(P[x], 0.0);
  }
  VMetric vm = make_vm(*bx, alpha, beta, gamma);
  long nfail = 0;
  double rate = 0.0;
  for (int s = 0; s < nsteps; ++s) nfail += rk_step_box(*bx, *par, vm, Ud.data(), Pd.data(), dt, scheme, (Dual*)nullptr, &rate);
  for (long x = 0; x < N; ++x) {
    U[x] = Ud[x].v;
    dU[x] = Ud[x].d;
    P[x] = Pd[x].v;
  }
  return nfail;
}

// ----- point functions used to pin the oracle -----

void orc_point_p2c(const double* P, double alpha, const double* beta, const double* g, double gam, double* U) {
  PMetric<double> m = point_metric(alpha, beta, g);
  PState<double> s;
  prim_state(m, P, gam, s);
  prim_to_cons(m, P, s, U);
}

void orc_point_p2c_tmunu(const double* P, double alpha, const double* beta, const double* g, double gam, double* U) {
  PMetric<double> m = point_metric(alpha, beta, g);
  cons_from_tmunu(m, P, gam, U);
}

void orc_point_flux(const double* P, double alpha, const double* beta, const double* g, double gam, int d, double* F) {
  PMetric<double> m = point_metric(alpha, beta, g);
  PState<double> s;
  prim_state(m, P, gam, s);
  double U[8];
  prim_to_cons(m, P, s, U);
  flux_dir(m, P, s, U, d, F);
}

void orc_point_flux_tmunu(const double* P, double alpha, const double* beta, const double* g, double gam, int d,
                          double* F) {
  PMetric<double> m = point_metric(alpha, beta, g);
  flux_from_tmunu(m, P, gam, d, F);
}

void orc_point_speeds(const double* P, double alpha, const double* beta, const double* g, double gam, int d,
                      double* lp, double* lm) {
  PMetric<double> m = point_metric(alpha, beta, g);
  PState<double> s;
  prim_state(m, P, gam, s);
  speeds_dir(m, P, s, gam, d, *lp, *lm);
}

void orc_point_lorentz(const double* P, double alpha, const double* beta, const double* g, double gam, double* W,
                       double* b2, double* p) {
  PMetric<double> m = point_metric(alpha, beta, g);
  PState<double> s;
  prim_state(m, P, gam, s);
  *W = s.W;
  *b2 = s.b2;
  *p = s.p;
}

int orc_point_c2p(double* U, double* P, const double* g, const Par* par) {
  const double zero[3] = {0, 0, 0};
  PMetric<double> m = point_metric(1.0, zero, g);
  AtmData atm = atm_of(*par);
  return con2prim_point(m, *par, atm, U, P);
}

// One Newman-Hamlin map p -> p' for the conserved state U (spatial metric g):
// out = (p', W, z).  Returns 0 when the map has no physical image.
int orc_point_nh_map(const double* U, const double* g, const Par* par, double p, double* out) {
  const double zero[3] = {0, 0, 0};
  PMetric<double> m = point_metric(1.0, zero, g);
  C2PIn<double> c;
  c2p_inputs(m, U, c);
  double pn = 0, W = 0, z = 0;
  const bool ok = nh_map(c, par->gam, p, pn, W, z);
  out[0] = pn;
  out[1] = W;
  out[2] = z;
  return ok ? 1 : 0;
}

// The Newman-Hamlin pressure iteration alone (no Newton polish) from p0:
// out = (p, W, z, T).  Returns 1 on convergence.
int orc_point_nh_solve(const double* U, const double* g, const Par* par, double p0, double* out) {
  const double zero[3] = {0, 0, 0};
  PMetric<double> m = point_metric(1.0, zero, g);
  C2PIn<double> c;
  c2p_inputs(m, U, c);
  double W = 0, z = 0, Tt = 0;
  const bool ok = newman_hamlin(c, *par, p0, W, z, Tt);
  out[0] = ok ? c.Dt * Tt / W : 0.0;
  out[1] = W;
  out[2] = z;
  out[3] = Tt;
  return ok ? 1 : 0;
}

// Boundary fill of the 8 primitive fields of one box (ghost cells only).
// Constrained transport: U's Bcal from A, and P's B = Bcal / sqrt(gamma) at the
// cell centre (initial data).
void orc_ct_init(const Box* bx, const double* alpha, const double* beta, const double* gamma, const double* A, double* U,
                 double* P) {
  Geo G(*bx);
  VMetric vm = make_vm(*bx, alpha, beta, gamma);
  ct_cell_field(*bx, A, U);
  for (long k = 0; k < bx->n[2]; ++k)
    for (long j = 0; j < bx->n[1]; ++j)
      for (long i = 0; i < bx->n[0]; ++i) {
        PMetric<double> m;
        metric_centre(G, vm, i, j, k, m);
        for (int d = 0; d < 3; ++d) P[(5 + d) * G.ncell + G.c(i, j, k)] = U[(5 + d) * G.ncell + G.c(i, j, k)] / m.sqrtg;
      }
}

void orc_ct_face_field(const Box* bx, const double* A, double* Bf) { ct_face_field(*bx, A, Bf); }

long orc_ct_step(const Box* bx, const Par* par, const double* alpha, const double* beta, const double* gamma, double* U,
                 double* P, double* A, double dt, int scheme, int p_current, double* max_rate) {
  return ct_step_box(*bx, *par, make_vm(*bx, alpha, beta, gamma), U, P, A, dt, scheme, p_current, max_rate);
}

// dA/dt from given primitives (their RHS's magnetic face fluxes).
void orc_ct_edge_rhs(const Box* bx, const Par* par, const double* alpha, const double* beta, const double* gamma,
                     double* P, double* dA) {
  Geo G(*bx);
  std::vector<double> L(8 * G.ncell);
  MagFlux<double> mf;
  rhs_from_prims(*bx, *par, make_vm(*bx, alpha, beta, gamma), P, L.data(), nullptr, &mf);
  ct_edge_rhs(*bx, mf, dA);
}

void orc_fill_ghosts(const Box* bx, double* P) {
  Geo G(*bx);
  fill_ghosts(*bx, G, P);
}

void orc_point_hlle(const double* PL, const double* PR, double alpha, const double* beta, const double* g, double gam,
                    int d, double* F, double* xip, double* xim) {
  PMetric<double> m = point_metric(alpha, beta, g);
  hlle(m, PL, PR, gam, d, F, *xip, *xim);
}

// Reconstruct a 1D line q[0..n) at its n-5 interior faces; face f sits between
// q[f+2] and q[f+3].  linear = 1 forces the linear WENO weights.
void orc_recon_line(const Par* par, int n, const double* q, double* qL, double* qR, int linear) {
  for (int f = 0; f + 6 <= n; ++f) recon_face(*par, q + f, qL[f], qR[f], linear);
}

// Sources at a point from the centre metric and its first derivatives.
// dalpha[3], dbeta[3*3] ([e][a]), dgamma[3*6] ([e][ij]).
void orc_point_sources(const double* P, double alpha, const double* beta, const double* g, const double* dalpha,
                       const double* dbeta, const double* dgamma, double gam, int form, double* S) {
  PMetric<double> m = point_metric(alpha, beta, g);
  MetricDeriv D;
  for (int e = 0; e < 3; ++e) {
    D.dalpha[e] = dalpha[e];
    for (int a = 0; a < 3; ++a) D.dbeta[e][a] = dbeta ? dbeta[3 * e + a] : 0.0;
    for (int a = 0; a < 6; ++a) D.dgamma[e][a] = dgamma[6 * e + a];
  }
  if (form == 0)
    sources_covariant(m, D, P, gam, S);
  else
    sources_3p1(m, D, P, gam, S);
}


// Arithmetic of the method per unit, tallied with the counting scalar on a
// smooth physical state (zero shift, conformally flat metric):
//   out[0..3] one face in direction 0: 4-vertex metric averages of alpha and
//             gamma_ij, det / gamma^dd / sqrt(gamma), reconstruction of 8
//             fields on both sides, the two positivity checks and HLLE;
//   out[4..7] one cell: 8-vertex metric averages and inverse, edge-averaged
//             derivatives of alpha and gamma_ij, the zero-shift source terms,
//             the divergence of 3 face pairs and the SSPRK stage combine.
// Each group is (add/sub, mul, div, sqrt).
void orc_count_ops(int recon, long* out) {
  Par par;
  std::memset(&par, 0, sizeof(par));
  par.recon = recon;
  par.gam = 5.0 / 3.0;
  par.weno_eps = 1e-6;
  par.wenoz_eps = 1e-40;
  par.wenoz_p = 1;
  // ---- one face ----
  g_tally = {0, 0, 0, 0};
  Cnt stencil[8][6];
  for (int q = 0; q < 8; ++q)
    for (int o = 0; o < 6; ++o) stencil[q][o] = Cnt((q == 0 ? 1.0 : (q == 4 ? 1.5 : 0.1)) + 0.01 * o * (q + 1));
  Cnt v4[7][4];
  for (int f = 0; f < 7; ++f)
    for (int c = 0; c < 4; ++c) v4[f][c] = Cnt((f == 0 || f == 1 || f == 4 || f == 6) ? 1.0 + 0.001 * c : 0.0);
  PMetric<Cnt> m;
  {
    Cnt av[7];
    for (int f = 0; f < 7; ++f) av[f] = 0.25 * ((v4[f][0] + v4[f][1]) + (v4[f][2] + v4[f][3]));
    m.alpha = av[0];
    for (int a = 0; a < 3; ++a) m.beta[a] = Cnt(0.0);
    for (int a = 0; a < 6; ++a) m.g[a] = av[1 + a];
    // only det, sqrt(gamma) and gamma^dd are needed on a face
    const Cnt* g = m.g;
    Cnt cxx = g[3] * g[5] - g[4] * g[4];
    Cnt cxy = g[2] * g[4] - g[1] * g[5];
    Cnt cxz = g[1] * g[4] - g[2] * g[3];
    m.det = g[0] * cxx + g[1] * cxy + g[2] * cxz;
    m.sqrtg = sqrt(m.det);
    m.ginv[0] = cxx / m.det;
  }
  Cnt PL[8], PR[8];
  for (int q = 0; q < 8; ++q) recon_face(par, stencil[q], PL[q], PR[q]);
  (void)state_ok(m, PL);
  (void)state_ok(m, PR);
  Cnt Fs[8], xp, xm;
  hlle(m, PL, PR, par.gam, 0, Fs, xp, xm);
  out[0] = g_tally.add; out[1] = g_tally.mul; out[2] = g_tally.div; out[3] = g_tally.sqrt;
  // ---- one cell ----
  g_tally = {0, 0, 0, 0};
  Cnt v8[7][8];
  for (int f = 0; f < 7; ++f)
    for (int c = 0; c < 8; ++c) v8[f][c] = Cnt((f == 0 || f == 1 || f == 4 || f == 6) ? 1.0 + 0.001 * c : 0.0);
  PMetric<Cnt> mc;
  {
    Cnt av[7];
    for (int f = 0; f < 7; ++f)
      av[f] = 0.125 * (((v8[f][0] + v8[f][1]) + (v8[f][2] + v8[f][3])) + ((v8[f][4] + v8[f][5]) + (v8[f][6] + v8[f][7])));
    mc.alpha = av[0];
    for (int a = 0; a < 3; ++a) mc.beta[a] = Cnt(0.0);
    for (int a = 0; a < 6; ++a) mc.g[a] = av[1 + a];
    metric_finish(mc);
  }
  Cnt dal[3], dgm[3][6];
  const Cnt idx(64.0);
  for (int e = 0; e < 3; ++e) {
    Cnt d[7];
    for (int f = 0; f < 7; ++f) {
      Cnt s0 = v8[f][1] - v8[f][0], s1 = v8[f][3] - v8[f][2], s2 = v8[f][5] - v8[f][4], s3 = v8[f][7] - v8[f][6];
      d[f] = 0.25 * ((s0 + s1) + (s2 + s3)) * idx;
    }
    dal[e] = d[0];
    for (int a = 0; a < 6; ++a) dgm[e][a] = d[1 + a];
  }
  Cnt Pc[8];
  for (int q = 0; q < 8; ++q) Pc[q] = stencil[q][2];
  {
    // zero-shift static sources: S_Sj = alpha sqrt(g) (-alpha T^00 d_j alpha + T^ik d_j gamma_ik / 2),
    // S_tau = -alpha sqrt(g) T^0i d_i alpha, with T^{mu nu} from u^mu, b^mu (Eq. (mhd-stress-energy-tensor))
    PState<Cnt> s;
    prim_state(mc, Pc, par.gam, s);
    Cnt ia = Cnt(1.0) / mc.alpha;
    Cnt u0 = s.W * ia, b0 = s.ab0 * ia * ia;
    Cnt u[3], b[3];
    for (int i = 0; i < 3; ++i) {
      u[i] = s.W * Pc[1 + i];
      b[i] = (Pc[5 + i] + mc.alpha * b0 * u[i]) / s.W;
    }
    Cnt ia2 = ia * ia;
    Cnt T00 = s.rhohs * u0 * u0 - s.Ps * ia2 - b0 * b0;
    Cnt T0[3], Tij[6];
    for (int i = 0; i < 3; ++i) T0[i] = s.rhohs * u0 * u[i] - b0 * b[i];
    for (int i = 0; i < 3; ++i)
      for (int j = i; j < 3; ++j) Tij[sym(i, j)] = s.rhohs * u[i] * u[j] + s.Ps * mc.ginv[sym(i, j)] - b[i] * b[j];
    Cnt as = mc.alpha * mc.sqrtg;
    Cnt S[8];
    for (int j = 0; j < 3; ++j) {
      Cnt t = Cnt(0.0);
      for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) t = t + Tij[sym(i, k)] * dgm[j][sym(i, k)];
      S[1 + j] = as * (0.5 * t - mc.alpha * T00 * dal[j]);
    }
    S[4] = Cnt(0.0) - as * (T0[0] * dal[0] + T0[1] * dal[1] + T0[2] * dal[2]);
    // divergence of 3 face pairs and the stage combine U^n + c ((U_s - U^n) + dt L)
    Cnt acc[8], Fl(0.3), Fh(0.2), un(1.0), us(1.1), dt(0.01), cs(0.25);
    for (int q = 0; q < 8; ++q) {
      acc[q] = (q == 0 || q >= 5) ? Cnt(0.0) : S[q];
      for (int d = 0; d < 3; ++d) acc[q] = acc[q] + (Fl - Fh) * idx;
      Cnt o = un + cs * ((us - un) + dt * acc[q]);
      (void)o;
    }
  }
  out[4] = g_tally.add; out[5] = g_tally.mul; out[6] = g_tally.div; out[7] = g_tally.sqrt;
}

}  // extern "C"
