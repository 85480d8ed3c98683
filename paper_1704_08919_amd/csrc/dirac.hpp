// Per-mode arithmetic of the momentum-space Dirac evolution in 2x2 blocks (Sec. II A of
// arXiv:1704.08919), shared by the evolution kernels and the yield-gradient kernel: the series
// for the exact exponential of a frozen block Hamiltonian, the block states, the rotation
// applied per step, the initial negative-energy state and the projection on the outgoing
// positive-energy state.  Translation units that include it compile with contraction off and
// write every fused multiply-add out, so each mode's arithmetic is one fixed instruction
// sequence.
#pragma once

#include "common.hpp"
#include "tan_fit.hpp"

#pragma clang fp contract(off)

namespace po {
namespace {

constexpr int kChunk = kChunkSteps;   // steps staged per LDS buffer

constexpr double factorial(int n) { return n <= 1 ? 1.0 : double(n) * factorial(n - 1); }
// Maclaurin coefficients of cos(sqrt x) and sin(sqrt x)/sqrt x.
constexpr double cos_coef(int k) { return (k % 2 ? -1.0 : 1.0) / factorial(2 * k); }
constexpr double sinc_coef(int k) { return (k % 2 ? -1.0 : 1.0) / factorial(2 * k + 1); }

// Series variants: T(x) = tan(sqrt x)/sqrt x = 1 + x R(x) with R a polynomial fit of degree
// n - 1 (n = 4..11, tan_fit.hpp: Chebyshev interpolation on [0, X_n], |T_fit - T| <= 2^-57 there,
// about two degrees fewer than the Maclaurin series needs for the same range).  Beyond the last
// X_n, index kFineHalving: C and S of degree 7 (first omitted term x^8/16! < 2^-56 for
// x <= 0.3612; both series alternate with decreasing terms) after h angle halvings.
constexpr int kNumFine = kNumFit;
constexpr int kFineHalving = kNumFine;
constexpr double kCosSinXmax = 0.3612;
constexpr int kMaxHalvings = 60;  // x up to 0.3612 * 4^60 ~ 5e35; beyond (or non-finite) the choice stops here
constexpr double kSqrt3Over6 = 0.28867513459481288225;  // sqrt(3)/6, Gauss-Legendre nodes 1/2 -+ sqrt(3)/6

// Horner step k of the C and S series, coefficients forced to compile-time constants.
template <int K>
__device__ __forceinline__ void horner_cs(double x, double& C, double& S) {
  constexpr double cc = cos_coef(K), sc = sinc_coef(K);
  C = fma(C, x, cc);
  S = fma(S, x, sc);
  if constexpr (K > 0) horner_cs<K - 1>(x, C, S);
}

template <int D>
__device__ __forceinline__ void cos_sinc(double x, double& C, double& S) {
  constexpr double cd = cos_coef(D), sd = sinc_coef(D);
  C = cd;
  S = sd;
  horner_cs<D - 1>(x, C, S);
}

// Coefficients of the fit of variant V, put in scalar registers where the caller loads them: the
// empty asm statement per value keeps the compiler from materialising the constants of every
// variant of a kernel at its entry (which exhausts the scalar registers); the values are unchanged.
template <int V>
struct Fit {
  double c[kFitDegree[V]];
};

template <int V>
__device__ __forceinline__ Fit<V> load_fit() {
  Fit<V> f;
#pragma unroll
  for (int k = 0; k < kFitDegree[V]; ++k) {
    f.c[k] = kFitCoef[V][k];
    asm volatile("" : "+s"(f.c[k]));
  }
  return f;
}

// R(x) = (T(x) - 1)/x of variant V (degree kFitDegree[V] - 1), by Horner's rule.
template <int V>
__device__ __forceinline__ double fit_R(double x, const Fit<V>& f) {
  constexpr int n = kFitDegree[V];
  double R = f.c[n - 1];
#pragma unroll
  for (int k = n - 2; k >= 0; --k) R = fma(R, x, f.c[k]);
  return R;
}

// T(x) = tan(sqrt x)/sqrt x of variant V: kFitDegree[V] fused multiply-adds.
template <int V>
__device__ __forceinline__ double tan_ratio(double x, const Fit<V>& f) {
  return fma(fit_R<V>(x, f), x, 1.0);
}

// (a_r, a_i, b_r, b_i) of block s = +1 and (c_r, c_i, d_r, d_i) of block s = -1.
struct State {
  double ar, ai, br, bi, cr, ci, dr, di;
};

// psi <- (C - i S Q_s) psi for both blocks:
//   s = +1:  a' = (C - i sz) a + (-sy - i sx) b ;  b' = (sy - i sx) a + (C + i sz) b,  s_q = S q;
//   s = -1:  the same with sy -> -sy.
__device__ __forceinline__ void rotate(State& v, double C, double S, double qx, double qy, double qz) {
  const double sx = S * qx, sy = S * qy, sz = S * qz;
  const double ar = fma(sx, v.bi, fma(-sy, v.br, fma(sz, v.ai, C * v.ar)));
  const double ai = fma(-sx, v.br, fma(-sy, v.bi, fma(-sz, v.ar, C * v.ai)));
  const double br = fma(-sz, v.bi, fma(C, v.br, fma(sx, v.ai, sy * v.ar)));
  const double bi = fma(sz, v.br, fma(C, v.bi, fma(-sx, v.ar, sy * v.ai)));
  const double cr = fma(sx, v.di, fma(sy, v.dr, fma(sz, v.ci, C * v.cr)));
  const double ci = fma(-sx, v.dr, fma(sy, v.di, fma(-sz, v.cr, C * v.ci)));
  const double dr = fma(-sz, v.di, fma(C, v.dr, fma(sx, v.ci, -sy * v.cr)));
  const double di = fma(sz, v.dr, fma(C, v.di, fma(-sx, v.cr, -sy * v.ci)));
  v = State{ar, ai, br, bi, cr, ci, dr, di};
}

// psi <- (1 - i T Q_s) psi for both blocks: the rotation above with C -> 1 and S -> T.
__device__ __forceinline__ void rotate_tan(State& v, double T, double qx, double qy, double qz) {
  const double tx = T * qx, ty = T * qy, tz = T * qz;
  const double ar = fma(tx, v.bi, fma(-ty, v.br, fma(tz, v.ai, v.ar)));
  const double ai = fma(-tx, v.br, fma(-ty, v.bi, fma(-tz, v.ar, v.ai)));
  const double br = fma(-tz, v.bi, fma(tx, v.ai, fma(ty, v.ar, v.br)));
  const double bi = fma(tz, v.br, fma(-tx, v.ar, fma(ty, v.ai, v.bi)));
  const double cr = fma(tx, v.di, fma(ty, v.dr, fma(tz, v.ci, v.cr)));
  const double ci = fma(-tx, v.dr, fma(ty, v.di, fma(-tz, v.cr, v.ci)));
  const double dr = fma(-tz, v.di, fma(tx, v.ci, fma(-ty, v.cr, v.dr)));
  const double di = fma(tz, v.dr, fma(-tx, v.cr, fma(-ty, v.ci, v.di)));
  v = State{ar, ai, br, bi, cr, ci, dr, di};
}

template <int V>  // series variant
__device__ __forceinline__ void step_tan(State& v, double2 rec, double pxdt, double pydt, double qz, double qz2,
                                         const Fit<V>& f) {
  const double qx = pxdt + rec.x;  // rec = -A dt
  const double qy = pydt + rec.y;
  const double x = fma(qx, qx, fma(qy, qy, qz2));
  rotate_tan(v, tan_ratio<V>(x, f), qx, qy, qz);
}

// Large-step path: C, S at x / 4^h, then h double-angle steps; the step stays unitary.
__device__ __forceinline__ void step_halving(State& v, double2 rec, double pxdt, double pydt, double qz, double qz2,
                                             int h, double inv4h) {
  const double qx = pxdt + rec.x;
  const double qy = pydt + rec.y;
  const double x = fma(qx, qx, fma(qy, qy, qz2));
  double xs = x * inv4h;
  double C, S;
  cos_sinc<7>(xs, C, S);  // xs <= kCosSinXmax
  for (int i = 0; i < h; ++i) {
    const double c2 = fma(C, C, -(xs * S) * S);  // cos 2t = cos^2 t - t^2 (sin t / t)^2
    S = S * C;                                 // sin 2t / 2t = (sin t / t) cos t
    C = c2;
    xs *= 4.0;
  }
  rotate(v, C, S, qx, qy, qz);
}

// C = cos sqrt x, S = sin sqrt x / sqrt x from the degree-7 series at x / 4^h and h double-angle steps.
__device__ __forceinline__ void cos_sinc_halved(double x, int h, double inv4h, double& C, double& S) {
  double xs = x * inv4h;
  cos_sinc<7>(xs, C, S);
  for (int i = 0; i < h; ++i) {
    const double c2 = fma(C, C, -(xs * S) * S);
    S = S * C;
    C = c2;
    xs *= 4.0;
  }
}

// psi <- (1 - i t . tau) psi for one block (a, b).
__device__ __forceinline__ void rotate_block_tan(double& ar, double& ai, double& br, double& bi, double tx, double ty,
                                                 double tz) {
  const double nar = fma(tx, bi, fma(-ty, br, fma(tz, ai, ar)));
  const double nai = fma(-tx, br, fma(-ty, bi, fma(-tz, ar, ai)));
  const double nbr = fma(-tz, bi, fma(tx, ai, fma(ty, ar, br)));
  const double nbi = fma(tz, br, fma(-tx, ar, fma(ty, ai, bi)));
  ar = nar; ai = nai; br = nbr; bi = nbi;
}

// psi <- (C - i s . tau) psi for one block (a, b).
__device__ __forceinline__ void rotate_block(double& ar, double& ai, double& br, double& bi, double C, double sx,
                                             double sy, double sz) {
  const double nar = fma(sx, bi, fma(-sy, br, fma(sz, ai, C * ar)));
  const double nai = fma(-sx, br, fma(-sy, bi, fma(-sz, ar, C * ai)));
  const double nbr = fma(-sz, bi, fma(C, br, fma(sx, ai, sy * ar)));
  const double nbi = fma(sz, br, fma(C, bi, fma(-sx, ar, sy * ai)));
  ar = nar; ai = nai; br = nbr; bi = nbi;
}

// Rescales the state by an exact power of two (no rounding) so that |psi_{+1}|^2 is O(1).
__device__ __forceinline__ void renormalise(State& v) {
  const double n2 = fma(v.bi, v.bi, fma(v.br, v.br, fma(v.ai, v.ai, v.ar * v.ar)));
  const int e = -(ilogb(n2) >> 1);
  v.ar = ldexp(v.ar, e); v.ai = ldexp(v.ai, e); v.br = ldexp(v.br, e); v.bi = ldexp(v.bi, e);
  v.cr = ldexp(v.cr, e); v.ci = ldexp(v.ci, e); v.dr = ldexp(v.dr, e); v.di = ldexp(v.di, e);
}

// Negative-energy eigenvector of h_s(P): (-(P_x - i s P_y), w + e) / sqrt(2 w (w + e)).
__device__ __forceinline__ void init_state(State& v, double Px, double Py, double e) {
  const double w = sqrt(fma(Px, Px, fma(Py, Py, e * e)));
  const double n = 1.0 / sqrt((2.0 * w) * (w + e));
  v.ar = -Px * n; v.ai = Py * n;  v.br = (w + e) * n; v.bi = 0.0;   // s = +1
  v.cr = -Px * n; v.ci = -Py * n; v.dr = (w + e) * n; v.di = 0.0;   // s = -1
}

// f = sum_s |<+_s(P)|psi_s>|^2 / |psi_s|^2 with |+_s> = (w + e, P_x + i s P_y) / sqrt(2 w (w + e)).
__device__ __forceinline__ double project(const State& v, double Px, double Py, double e) {
  const double w = sqrt(fma(Px, Px, fma(Py, Py, e * e)));
  const double we = w + e;
  const double n2 = 1.0 / ((2.0 * w) * we);
  // s = +1: (w+e) a + (P_x - i P_y) b
  const double r1 = fma(Py, v.bi, fma(Px, v.br, we * v.ar));
  const double i1 = fma(-Py, v.br, fma(Px, v.bi, we * v.ai));
  // s = -1: (w+e) c + (P_x + i P_y) d
  const double r2 = fma(-Py, v.di, fma(Px, v.dr, we * v.cr));
  const double i2 = fma(Py, v.dr, fma(Px, v.di, we * v.ci));
  const double m1 = fma(v.bi, v.bi, fma(v.br, v.br, fma(v.ai, v.ai, v.ar * v.ar)));
  const double m2 = fma(v.di, v.di, fma(v.dr, v.dr, fma(v.ci, v.ci, v.cr * v.cr)));
  return (fma(i1, i1, r1 * r1) / m1 + fma(i2, i2, r2 * r2) / m2) * n2;
}
}  // namespace
}  // namespace po
