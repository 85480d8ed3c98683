// Gradient of the pair yield J = dV sum_p f(p) with respect to the vector-potential table: the
// exact derivative (discrete adjoint) of the exponential-midpoint Dirac scheme of Sec. II A.  It
// serves the local search of Sec. IV A, which needs the gradient of the objective with respect to
// the field parameters; the paper obtains it from the adjoint of the kinetic equation, here it is
// the adjoint of the Dirac steps that evaluate J.
//
// Per block s and mode, f_s = |alpha_s|^2 with alpha_s = <+_s(P_out)| U_{N-1} ... U_0 |-_s(P_in)>
// and U_n = exp(-i q_n . tau), q_n = dt (P_x, s P_y, e_perp), P = p - A_n.  With the forward
// states psi_n = U_{n-1} ... U_0 |-> and the backward states chi_n = U_n^+ ... U_{N-1}^+ |+>,
//     df_s / dA_n = 2 Re[ conj(alpha_s) <chi_{n+1}| dU_n/dA_n |psi_n> ],
// and, writing U = C - i S q.tau with C = cos|q|, S = sin|q|/|q|, D = (C - S)/|q|^2,
//     dU/dq_j = q_j (-S - i D q.tau) - i S tau_j,   dq_x/dA_x = -dt,  dq_y/dA_y = -s dt.
// The initial and final states depend on A(t_i) and A(t_f) through P_in and P_out (first-order
// perturbation of the block eigenvectors, energies -+ omega):
//     d|->  = -|+><+|dh|->/(2 omega),   d<+|psi> = <+|dh|-><-|psi>/(2 omega),   dP = -dA.
//
// Since f_s is the same with chi_s replaced by alpha_s chi_s, the backward sweep carries
// chi'_s = alpha_s chi_s and each term is 2 Re <chi'_{n+1}| dU/dq_j |psi_n>, of which only
// Re <chi'|psi> and Im <chi'|tau_k|psi> enter.
//
// One workgroup of 256 lanes per 256-mode item, one mode per lane.  Forward: the evolution's own
// step (tangent form or C, S with the pulse's angle halvings), states unit-normalised per block at
// t_f.  Backward: the table is staged through LDS chunk by chunk in reverse; each step applies U^+
// to psi and chi' (tangent form with the factors C carried in a per-lane scale, or the exact C, S
// form on the angle-halving path) and forms the two derivative terms.  Their sum over the item's
// modes is taken per step in a fixed order: each lane stores its terms for 8 steps in LDS, the wave
// reads them back transposed (lane (j, p) adds the lanes p, p + 8, ..., p + 56 of step j), pairs
// up the 8 lanes of a step (DPP), and the four waves are added in order; the results are written
// as item partials [item][n][2], and a second kernel sums the items of each pulse in order.  So
// the gradient, like J, does not depend on scheduling.
#include "dirac.hpp"
#include "reduce.hpp"

#pragma clang fp contract(off)

namespace po {
namespace {

// C = cos sqrt x and S = sin sqrt x / sqrt x by their degree-7 series (x <= 0.3612 keeps both
// remainders below 2^-56), and D = (C - S)/x = C1 - S1, where C = 1 + x C1 and S = 1 + x S1 are the
// last Horner steps (no cancellation: C1 ~ -1/2, S1 ~ -1/6; remainder of D below 2^-54).
template <int K>
__device__ __forceinline__ void horner_cs1(double x, double& C, double& S) {
  constexpr double cc = cos_coef(K), sc = sinc_coef(K);
  C = fma(C, x, cc);
  S = fma(S, x, sc);
  if constexpr (K > 1) horner_cs1<K - 1>(x, C, S);
}

__device__ __forceinline__ void csd_series(double x, double& C, double& S, double& D) {
  constexpr double c7 = cos_coef(7), s7 = sinc_coef(7);
  double C1 = c7, S1 = s7;
  horner_cs1<6>(x, C1, S1);
  D = C1 - S1;
  C = fma(C1, x, 1.0);
  S = fma(S1, x, 1.0);
}

// The same after h halvings of the angle (x / 4^h in the series range, h double-angle steps for C
// and S); D = (C - S)/x has no cancellation there (x > 0.36).
__device__ __forceinline__ void csd(double x, int h, double inv4h, double& C, double& S, double& D) {
  if (h == 0) {
    csd_series(x, C, S, D);
  } else {
    cos_sinc_halved(x, h, inv4h, C, S);
    D = (C - S) / x;
  }
}

struct Blk {
  double ar, ai, br, bi;
};

// Block s (0: s = +1, 1: s = -1) of a two-block state.
__device__ __forceinline__ Blk block_of(const State& v, int s) {
  return s == 0 ? Blk{v.ar, v.ai, v.br, v.bi} : Blk{v.cr, v.ci, v.dr, v.di};
}

// z b for a complex scalar z and a block vector b.
__device__ __forceinline__ Blk cscale(double zr, double zi, const Blk& b) {
  return Blk{fma(zr, b.ar, -(zi * b.ai)), fma(zr, b.ai, zi * b.ar), fma(zr, b.br, -(zi * b.bi)),
             fma(zr, b.bi, zi * b.br)};
}

// Unit eigenvectors of h_s(P) = P_x tau_x + s P_y tau_y + e tau_z: |+> = (w + e, P_x + i s P_y)/N,
// |-> = (-(P_x - i s P_y), w + e)/N, N = sqrt(2 w (w + e)).
__device__ __forceinline__ void eig_pm(double Px, double Py, double e, double s, Blk& up, Blk& dn, double& w) {
  w = sqrt(fma(Px, Px, fma(Py, Py, e * e)));
  const double n = 1.0 / sqrt((2.0 * w) * (w + e));
  up = Blk{(w + e) * n, 0.0, Px * n, s * Py * n};
  dn = Blk{-(Px * n), s * Py * n, (w + e) * n, 0.0};
}

// <a|b> for two block vectors.
__device__ __forceinline__ void inner(const Blk& a, const Blk& b, double& r, double& i) {
  r = fma(a.ar, b.ar, fma(a.ai, b.ai, fma(a.br, b.br, a.bi * b.bi)));
  i = fma(a.ar, b.ai, fma(-a.ai, b.ar, fma(a.br, b.bi, -(a.bi * b.br))));
}

// <x|tau_x|y> and <x|s tau_y|y>.
__device__ __forceinline__ void tau_xy(const Blk& x, const Blk& y, double s, double& xr, double& xi, double& yr,
                                       double& yi) {
  // conj(x1) y2 + conj(x2) y1
  const double a_r = fma(x.ar, y.br, x.ai * y.bi), a_i = fma(x.ar, y.bi, -(x.ai * y.br));  // conj(x1) y2
  const double b_r = fma(x.br, y.ar, x.bi * y.ai), b_i = fma(x.br, y.ai, -(x.bi * y.ar));  // conj(x2) y1
  xr = a_r + b_r;
  xi = a_i + b_i;
  // tau_y: -i conj(x1) y2 + i conj(x2) y1
  yr = s * (a_i - b_i);
  yi = s * (b_r - a_r);
}

// Re <chi| dU/dq_j |psi> for j = x, y of one block, chi = (c1, c2) already carrying the factor
// alpha, psi = (p1, p2), q = (qx, qy, qz) the block's vector.  Only four real numbers of the
// block products enter: a = Re <chi|psi> and the imaginary parts of t_k = <chi|tau_k|psi>;
//   Re[q_j (-S a - i D q.t) - i S t_j] = q_j (D q.Im t - S Re a) + S Im t_j.
__device__ __forceinline__ void block_grad(double c1r, double c1i, double c2r, double c2i, double p1r, double p1i,
                                           double p2r, double p2i, double S, double D, double qx, double qy,
                                           double qz, double& gx, double& gy) {
  const double a = fma(c2i, p2i, fma(c2r, p2r, fma(c1i, p1i, c1r * p1r)));
  const double tx = fma(-c2i, p1r, fma(c2r, p1i, fma(-c1i, p2r, c1r * p2i)));   // Im(c1* p2 + c2* p1)
  const double ty = fma(-c1i, p2i, fma(-c1r, p2r, fma(c2i, p1i, c2r * p1r)));   // Re(c2* p1 - c1* p2)
  const double tz = fma(c2i, p2r, fma(-c2r, p2i, fma(-c1i, p1r, c1r * p1i)));   // Im(c1* p1 - c2* p2)
  const double b = fma(qz, tz, fma(qy, ty, qx * tx));
  const double w = fma(D, b, -(S * a));
  gx = fma(qx, w, S * tx);
  gy = fma(qy, w, S * ty);
}

// One backward step n: psi <- U_n^+ psi (psi_{n+1} -> psi_n), the derivative terms with chi_{n+1},
// then chi <- U_n^+ chi.  Returns (sum_s Re<chi|dU/dq_x|psi>, sum_s s Re<chi|dU/dq_y|psi>).
// SERIES: the step angle is within the degree-7 range (no halving, D from its own series).
template <bool SERIES>
__device__ __forceinline__ double2 back_step(State& psi, State& chi, double2 r, double pxdt, double pydt, double qz,
                                             double qz2, int h, double inv4h) {
  const double qx = pxdt + r.x, qy = pydt + r.y;
  const double x = fma(qx, qx, fma(qy, qy, qz2));
  double C, S, D;
  if constexpr (SERIES) {
    csd_series(x, C, S, D);
  } else {
    csd(x, h, inv4h, C, S, D);
  }
  rotate(psi, C, -S, qx, qy, qz);
  double gx0, gy0, gx1, gy1;
  block_grad(chi.ar, chi.ai, chi.br, chi.bi, psi.ar, psi.ai, psi.br, psi.bi, S, D, qx, qy, qz, gx0, gy0);
  block_grad(chi.cr, chi.ci, chi.dr, chi.di, psi.cr, psi.ci, psi.dr, psi.di, S, D, qx, -qy, qz, gx1, gy1);
  rotate(chi, C, -S, qx, qy, qz);
  return make_double2(gx0 + gx1, gy0 - gy1);
}

// Tangent form of the backward step (steps within the T-series range).  With U = C (1 - i T Q)
// and S = C T, D = (C - S)/x = -C R where R = (T - 1)/x, the step applies (1 + i T Q) to psi and
// chi' and leaves out the factors C: psi_n = sigma_n psi~_n and chi'_{n+1} = sigma_{n+1} chi~_{n+1}
// with sigma_n = C_n sigma_{n+1}, so the term of step n is Sigma_n = sigma_n^2 = C_n^2 Sigma_{n+1}
// times the same expression in psi~, chi~ with (S, D) -> (T, -R).  C^2 = cos^2 sqrt x comes from its
// own series, R is the variant's fit (T = 1 + x R).
// cos^2 sqrt x = 1 + sum_{k >= 1} (-1)^k 2^(2k-1) x^k / (2k)!, alternating with decreasing terms;
// degree kFitCos2Degree[v] keeps the remainder below 2^-59 up to the variant's largest x.
constexpr double pow2i(int n) { return n == 0 ? 1.0 : 2.0 * pow2i(n - 1); }
constexpr double cos2_coef(int k) { return k == 0 ? 1.0 : (k % 2 ? -1.0 : 1.0) * pow2i(2 * k - 1) / factorial(2 * k); }

template <int K>
__device__ __forceinline__ void horner_cos2(double x, double& c) {
  constexpr double ck = cos2_coef(K);
  c = fma(c, x, ck);
  if constexpr (K > 0) horner_cos2<K - 1>(x, c);
}

template <int M>
__device__ __forceinline__ double cos2_series(double x) {
  constexpr double cm = cos2_coef(M);
  double c = cm;
  horner_cos2<M - 1>(x, c);
  return c;
}

template <int MODE>
__device__ __forceinline__ double2 back_step_tan(State& psi, State& chi, double2 r, double pxdt, double pydt,
                                                 double qz, double qz2, double& sig, const Fit<MODE>& f) {
  constexpr int M = kFitCos2Degree[MODE];
  const double qx = pxdt + r.x, qy = pydt + r.y;
  const double x = fma(qx, qx, fma(qy, qy, qz2));
  const double R = fit_R<MODE>(x, f);
  const double T = fma(R, x, 1.0);
  const double c2 = cos2_series<M>(x);
  rotate_tan(psi, -T, qx, qy, qz);
  double gx0, gy0, gx1, gy1;
  block_grad(chi.ar, chi.ai, chi.br, chi.bi, psi.ar, psi.ai, psi.br, psi.bi, T, -R, qx, qy, qz, gx0, gy0);
  block_grad(chi.cr, chi.ci, chi.dr, chi.di, psi.cr, psi.ci, psi.dr, psi.di, T, -R, qx, -qy, qz, gx1, gy1);
  rotate_tan(chi, -T, qx, qy, qz);
  sig *= c2;
  return make_double2(sig * (gx0 + gx1), sig * (gy0 - gy1));
}

// Folds Sigma back into the states (psi~, chi~ <- sqrt(Sigma) psi~, chi~ are then the true states) so
// Sigma restarts at 1; once per chunk, which keeps Sigma far from underflow.
__device__ __forceinline__ void fold_scale(State& psi, State& chi, double& sig) {
  const double s = sqrt(sig);
  psi.ar *= s; psi.ai *= s; psi.br *= s; psi.bi *= s; psi.cr *= s; psi.ci *= s; psi.dr *= s; psi.di *= s;
  chi.ar *= s; chi.ai *= s; chi.br *= s; chi.bi *= s; chi.cr *= s; chi.ci *= s; chi.dr *= s; chi.di *= s;
  sig = 1.0;
}

// Coefficients of the fit for the tangent-form variants (an empty record for the halving path).
template <int MODE, bool TAN = (MODE < kFineHalving)>
struct FitOf {
  using type = Fit<MODE>;
};
template <int MODE>
struct FitOf<MODE, false> {
  struct type {};
};

template <int MODE>
__device__ __forceinline__ typename FitOf<MODE>::type load_fit_of() {
  if constexpr (MODE < kFineHalving) return load_fit<MODE>();
  else return typename FitOf<MODE>::type{};
}

// One backward step in the form of the pulse's variant: tangent form (scale in sig) or exact C, S.
template <int MODE>
__device__ __forceinline__ double2 back_any(State& psi, State& chi, double2 r, double pxdt, double pydt, double qz,
                                            double qz2, int h, double inv4h, double& sig,
                                            const typename FitOf<MODE>::type& f) {
  if constexpr (MODE < kFineHalving) return back_step_tan<MODE>(psi, chi, r, pxdt, pydt, qz, qz2, sig, f);
  else return back_step<false>(psi, chi, r, pxdt, pydt, qz, qz2, h, inv4h);
}

// Forward step of the evolution in the form the pulse's series choice selects.
template <int MODE>
__device__ __forceinline__ void fwd_step(State& v, double2 rec, double pxdt, double pydt, double qz, double qz2, int h,
                                         double inv4h, const typename FitOf<MODE>::type& f) {
  if constexpr (MODE < kFineHalving) step_tan<MODE>(v, rec, pxdt, pydt, qz, qz2, f);
  else step_halving(v, rec, pxdt, pydt, qz, qz2, h, inv4h);
}

// Lane-to-lane moves inside rows of 16 (DPP): pairs (l, l^1), (l, l^2), l <-> 7 - l within 8 lanes and
// l <-> 15 - l within 16 lanes.
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;

template <int CTRL>
__device__ __forceinline__ double dpp_get(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// Sum over each aligned group of L lanes (L = 8 or 16); every lane of a group gets the same value.
template <int L>
__device__ __forceinline__ double group_sum(double v) {
  v += dpp_get<kDppXor1>(v);
  v += dpp_get<kDppXor2>(v);
  v += dpp_get<kDppHalfMirror>(v);
  if constexpr (L == 16) v += dpp_get<kDppMirror>(v);
  return v;
}

// Per-step sums over the 64 lanes of a wave for kGroup steps at once: each lane has written its
// (gx, gy) of step j to buf[j][lane]; lane (j, p) (j = lane / L, p = lane % L, L = 64 / kGroup)
// adds the lanes p, p + L, ... in order, then the L lanes of its step pair up.  Lane p = 0 of step
// j returns the wave's sum of step j.
constexpr int kGroup = 8;
constexpr int kLanesPerStep = 64 / kGroup;

__device__ __forceinline__ double2 group_reduce(const double2 (*buf)[64], int lane) {
  const int j = lane / kLanesPerStep, p = lane % kLanesPerStep;
  double2 v = buf[j][p];
#pragma unroll
  for (int i = 1; i < kGroup; ++i) {
    const double2 u = buf[j][i * kLanesPerStep + p];
    v.x += u.x;
    v.y += u.y;
  }
  return make_double2(group_sum<kLanesPerStep>(v.x), group_sum<kLanesPerStep>(v.y));
}

// Reduces a group of cnt steps (rows 0..cnt-1 of buf, steps top, top - 1, ...) and stores the
// wave's step sums in red[top - j].  The wave reads what its own lanes wrote: the fences complete
// the stores before the loads and the loads before the next group's stores (no other wave uses buf).
__device__ __forceinline__ void group_store(double2 (*buf)[64], double2* red, int lane, int top, int cnt) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  const double2 v = group_reduce(buf, lane);
  const int j = lane / kLanesPerStep;
  if (lane % kLanesPerStep == 0 && j < cnt) red[top - j] = v;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

struct GradArgs {
  const PulseDev* desc;
  int n_pulses;
  const double* A;
  const double* Aedge;
  const int2* sel;      // per selection block (the evolution's k_block_select)
  const int64_t* goff;  // per pulse: first double of its item partials
  double* part;         // [items of pulse][nt][2] per pulse
  double* epart;        // [total items][4]: dA(t_i) x, y, dA(t_f) x, y
  double* units;        // 64-mode sums of f
};

constexpr int kWaves = kItem / 64;

// LDS: tab[kChunk] (-A dt of the chunk), red[kWaves][kChunk] (per-wave step sums of the chunk),
// bufs[kWaves][kGroup][64] (lane values of kGroup steps, per wave); separate arrays, so the
// compiler sees that the table reads do not depend on the buf stores.
template <int MODE>
__device__ __forceinline__ void grad_item(const GradArgs& a, int item, int pi, double2* tab, double2 (*red)[kChunk],
                                          double2 (*bufs)[kGroup][64]) {
  const PulseDev& d = a.desc[pi];
  const int nt = d.nt;
  const double dt = d.dt;
  const int64_t nmodes = int64_t(d.n[0]) * d.n[1] * d.n[2];
  const int li = item - d.item_off;
  const int64_t m = int64_t(li) * kItem + threadIdx.x;
  const bool active = m < nmodes;
  const int h = a.sel[d.blk_off + li * kItem / kSelBlock].y;
  const double inv4h = ldexp(1.0, -2 * h);
  const auto fit = load_fit_of<MODE>();
  const double2* A = reinterpret_cast<const double2*>(a.A) + d.tab_off;
  const double2 ain = reinterpret_cast<const double2*>(a.Aedge)[2 * pi];
  const double2 aout = reinterpret_cast<const double2*>(a.Aedge)[2 * pi + 1];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;

  double px, py, pz;
  mode_momentum(d, active ? m : 0, px, py, pz);
  const double e = sqrt(fma(pz, pz, 1.0));
  const double pxdt = px * dt, pydt = py * dt, qz = e * dt, qz2 = qz * qz;

  // forward: psi_s from |-_s(P_in)>, in the evolution's own step form (the tangent form drops the
  // common factor C of every step; the blocks are normalised at t_f)
  State psi;
  init_state(psi, px - ain.x, py - ain.y, e);
  const int nchunks = (nt + kChunk - 1) / kChunk;
  for (int c = 0; c < nchunks; ++c) {
    const int n0 = c * kChunk, len = min(kChunk, nt - n0);
    __syncthreads();
    if (int(threadIdx.x) < len) {
      const double2 t = A[n0 + threadIdx.x];
      tab[threadIdx.x] = make_double2(-t.x * dt, -t.y * dt);
    }
    __syncthreads();
    if (len == kChunk) {
#pragma unroll 4
      for (int k = 0; k < kChunk; ++k) fwd_step<MODE>(psi, tab[k], pxdt, pydt, qz, qz2, h, inv4h, fit);
    } else {
      for (int k = 0; k < len; ++k) fwd_step<MODE>(psi, tab[k], pxdt, pydt, qz, qz2, h, inv4h, fit);
    }
    if constexpr (MODE < kFineHalving) renormalise(psi);
  }

  // t_f: normalise each block, alpha_s = <+_s(P_out)|psi_s>, final-state terms; chi_s = alpha_s |+_s>
  State chi;
  double g_out_x = 0.0, g_out_y = 0.0, f = 0.0;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const double sg = s == 0 ? 1.0 : -1.0;
    Blk up_out, dn_out;
    double w_out;
    eig_pm(px - aout.x, py - aout.y, e, sg, up_out, dn_out, w_out);
    Blk p = block_of(psi, s);
    double nr, ni;
    inner(p, p, nr, ni);
    const double inv = 1.0 / sqrt(nr);
    p = Blk{p.ar * inv, p.ai * inv, p.br * inv, p.bi * inv};
    double al_r, al_i;
    inner(up_out, p, al_r, al_i);
    if (!active) al_r = al_i = 0.0;
    f += fma(al_r, al_r, al_i * al_i);
    // d alpha = <+|dh|-><-|psi>/(2 w), dh = tau_x dP_x + s tau_y dP_y, dP = -dA(t_f)
    double xr, xi, yr, yi, mr, mi;
    tau_xy(up_out, dn_out, sg, xr, xi, yr, yi);
    inner(dn_out, p, mr, mi);
    const double k = -1.0 / (2.0 * w_out);
    // Re[conj(alpha) (t m)]
    const double tmx_r = fma(xr, mr, -(xi * mi)), tmx_i = fma(xr, mi, xi * mr);
    const double tmy_r = fma(yr, mr, -(yi * mi)), tmy_i = fma(yr, mi, yi * mr);
    g_out_x += 2.0 * k * fma(al_r, tmx_r, al_i * tmx_i);
    g_out_y += 2.0 * k * fma(al_r, tmy_r, al_i * tmy_i);
    const Blk cb = cscale(al_r, al_i, up_out);
    if (s == 0) {
      psi.ar = p.ar; psi.ai = p.ai; psi.br = p.br; psi.bi = p.bi;
      chi.ar = cb.ar; chi.ai = cb.ai; chi.br = cb.br; chi.bi = cb.bi;
    } else {
      psi.cr = p.ar; psi.ci = p.ai; psi.dr = p.br; psi.di = p.bi;
      chi.cr = cb.ar; chi.ci = cb.ai; chi.dr = cb.br; chi.di = cb.bi;
    }
  }

  // backward over the chunks in reverse, kGroup steps at a time (the last group of a chunk may be short)
  double sig = 1.0;  // Sigma of the tangent form (unused by the exact form)
  double* part = a.part + a.goff[pi] + int64_t(li) * nt * 2;
  double2 (*buf)[64] = bufs[wave];
  for (int c = nchunks - 1; c >= 0; --c) {
    const int n0 = c * kChunk, len = min(kChunk, nt - n0);
    __syncthreads();
    if (int(threadIdx.x) < len) {
      const double2 t = A[n0 + threadIdx.x];
      tab[threadIdx.x] = make_double2(-t.x * dt, -t.y * dt);
    }
    __syncthreads();
    if constexpr (MODE < kFineHalving) fold_scale(psi, chi, sig);
    // a short group first (len not a multiple of kGroup), then full groups
    int top = len - 1;
    const int r = len % kGroup;
    if (r != 0) {
#pragma unroll 1
      for (int j = 0; j < r; ++j)
        buf[j][lane] = back_any<MODE>(psi, chi, tab[top - j], pxdt, pydt, qz, qz2, h, inv4h, sig, fit);
      group_store(buf, red[wave], lane, top, r);
      top -= r;
    }
    for (; top >= 0; top -= kGroup) {
#pragma unroll
      for (int j = 0; j < kGroup; ++j)
        buf[j][lane] = back_any<MODE>(psi, chi, tab[top - j], pxdt, pydt, qz, qz2, h, inv4h, sig, fit);
      group_store(buf, red[wave], lane, top, kGroup);
    }
    __syncthreads();
    if (int(threadIdx.x) < len) {
      double2 v = red[0][threadIdx.x];
#pragma unroll
      for (int w = 1; w < kWaves; ++w) {
        v.x += red[w][threadIdx.x].x;
        v.y += red[w][threadIdx.x].y;
      }
      reinterpret_cast<double2*>(part)[n0 + threadIdx.x] = v;
    }
  }

  if constexpr (MODE < kFineHalving) fold_scale(psi, chi, sig);  // chi~ -> the true chi'_0

  // t_i: d|-> = -|+><+|dh|->/(2 w), dP = -dA(t_i); chi holds U^+ ... alpha |+_out> = alpha chi_0
  double g_in_x = 0.0, g_in_y = 0.0;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const double sg = s == 0 ? 1.0 : -1.0;
    Blk up_in, dn_in;
    double w_in;
    eig_pm(px - ain.x, py - ain.y, e, sg, up_in, dn_in, w_in);
    double xr, xi, yr, yi, cr, ci;
    tau_xy(up_in, dn_in, sg, xr, xi, yr, yi);
    inner(block_of(chi, s), up_in, cr, ci);
    const double k = 1.0 / (2.0 * w_in);  // (-1/(2w)) * (dP/dA = -1)
    g_in_x += 2.0 * k * fma(cr, xr, -(ci * xi));
    g_in_y += 2.0 * k * fma(cr, yr, -(ci * yi));
  }
  const double e4[4] = {g_in_x, g_in_y, g_out_x, g_out_y};
  __syncthreads();
  for (int j = 0; j < 4; ++j) {
    const double sj = wave_sum(e4[j]);
    if (lane == 0) red[wave][j] = make_double2(sj, 0.0);
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    double v = red[0][threadIdx.x].x;
#pragma unroll
    for (int w = 1; w < kWaves; ++w) v += red[w][threadIdx.x].x;
    a.epart[int64_t(item) * 4 + threadIdx.x] = v;
  }
  if (a.units) write_unit(d, a.units, m, nmodes, active ? f : 0.0);
}

__global__ void __launch_bounds__(kItem) __attribute__((amdgpu_waves_per_eu(3))) k_yield_grad(GradArgs a) {
  __shared__ double2 tab[kChunk];
  __shared__ double2 red[kWaves][kChunk];
  __shared__ double2 bufs[kWaves][kGroup][64];
  const int item = xcd_item(blockIdx.x, gridDim.x);
  const int pi = find_pulse_item(a.desc, a.n_pulses, item);
  // the item's variant is that of the evolution's selection block holding it
  const PulseDev& d = a.desc[pi];
  switch (a.sel[d.blk_off + (item - d.item_off) * kItem / kSelBlock].x) {
    case 0: grad_item<0>(a, item, pi, tab, red, bufs); break;
    case 1: grad_item<1>(a, item, pi, tab, red, bufs); break;
    case 2: grad_item<2>(a, item, pi, tab, red, bufs); break;
    case 3: grad_item<3>(a, item, pi, tab, red, bufs); break;
    case 4: grad_item<4>(a, item, pi, tab, red, bufs); break;
    case 5: grad_item<5>(a, item, pi, tab, red, bufs); break;
    case 6: grad_item<6>(a, item, pi, tab, red, bufs); break;
    case 7: grad_item<7>(a, item, pi, tab, red, bufs); break;
    default: grad_item<kFineHalving>(a, item, pi, tab, red, bufs); break;
  }
}

// dJ/dA[n] = -2 dt dV sum over the pulse's items (in order) of the partials (the edge partials carry
// their factors); one thread per (n, component).
__global__ void __launch_bounds__(256) k_grad_reduce(const PulseDev* __restrict__ desc, const int64_t* __restrict__ goff,
                                                     const double* __restrict__ part, const double* __restrict__ epart,
                                                     double* __restrict__ gA, double* __restrict__ gedge) {
  const PulseDev& d = desc[blockIdx.y];
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const int64_t per = 2 * int64_t(d.nt);
  if (e < per) {
    const double* p = part + goff[blockIdx.y];
    double v = 0.0;
    for (int i = 0; i < d.nitems; ++i) v += p[int64_t(i) * per + e];
    gA[2 * d.tab_off + e] = v * (-2.0 * d.dt) * d.dv;  // dq_x/dA_x = -dt; the factor 2 of 2 Re[...]
  }
  if (gedge && blockIdx.x == 0 && threadIdx.x < 4) {
    double v = 0.0;
    for (int i = 0; i < d.nitems; ++i) v += epart[int64_t(d.item_off + i) * 4 + threadIdx.x];
    gedge[4 * blockIdx.y + threadIdx.x] = v * d.dv;
  }
}

}  // namespace

po_status launch_yield_grad(const Batch& b, const PulseDev* d_desc, const double* d_A, const double* d_A_edge,
                            const int2* d_sel, const int64_t* d_goff, double* d_part, double* d_epart, double* d_units,
                            double* d_gA, double* d_gedge, hipStream_t s) {
  GradArgs a{d_desc, b.n_pulses, d_A, d_A_edge, d_sel, d_goff, d_part, d_epart, d_units};
  hipLaunchKernelGGL(k_yield_grad, dim3(b.total_items), dim3(kItem), 0, s, a);
  PO_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_grad_reduce, dim3(unsigned((2 * int64_t(b.max_nt) + 255) / 256), b.n_pulses), dim3(256), 0, s,
                     d_desc, d_goff, d_part, d_epart, d_gA, d_gedge);
  PO_HIP(hipGetLastError());
  return PO_OK;
}

}  // namespace po
