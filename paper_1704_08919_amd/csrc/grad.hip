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
// Since f_s is the same with chi_s replaced by alpha_s chi_s, each term is
// 2 Re <chi'_{n+1}| dU/dq_j |psi_n> with chi'_s = alpha_s chi_s, and it depends on the two states
// only through W_s = Im <chi'_s|tau|psi_s>, a real 3-vector that the backward steps rotate.
//
// One workgroup of 256 lanes per 256-mode item, one mode per lane.  Forward: the evolution's own
// step (tangent form or C, S with the pulse's angle halvings), states unit-normalised per block at
// t_f.  Backward: the table is staged through LDS chunk by chunk in reverse; each step forms the
// two derivative terms from W_{n+1} and rotates it to W_n (coefficients from the tangent form's
// fit and a cos^2 series, or from the exact C, S on the angle-halving path).  Their sum over the
// item's modes is taken per step in a fixed order: each lane stores its terms for 8 steps in LDS,
// the wave reads them back transposed (lane (j, p) adds the lanes p, p + 8, ..., p + 56 of step
// j), pairs up the 8 lanes of a step (DPP), and the four waves are added in order; the results are
// written as item partials [item][n][2], and a second kernel sums the items of each pulse in
// order.  So the gradient, like J, does not depend on scheduling.
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
// and S).  The halving count comes from the block's bound on x, so a single mode-step here can
// have any x >= (e_perp dt)^2; D = (C - S)/x then loses digits to cancellation (C - S ~ -x/3, so
// D carries a relative error of about 3 x 2^-53 / x: 3e-13 at the DE workload's smallest
// x = dt^2 = 2.4e-3), far inside the gradient's error bar.
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

// The backward sweep carries, per block, the real 3-vector W = Im <chi'|tau|psi> instead of the two
// states.  Moving both states back by one step changes V_k = <chi'|tau_k|psi> by the rotation that
// the step induces on the Pauli vector,
//     U tau_k U^+ = (C^2 - S^2 x) tau_k + 2 S^2 q_k (q.tau) - 2 C S (e_k x q).tau,
// which is real, so W_n = (C^2 - S^2 x) W + 2 S^2 (q.W) q - 2 C S (q x W) with W = W_{n+1}.  And
// since dU/dq_j U^+ = -i [q_j (S^2 + C D) q.tau + C S tau_j - S^2 (e_j x q).tau] has no identity part,
//     Re <chi'_{n+1}| dU/dq_j |psi_n> = Re <chi'_{n+1}| dU/dq_j U^+ |psi_{n+1}>
//                                    = q_j (S^2 + C D)(q.W) + C S W_j - S^2 (q x W)_j.
// Block s = -1 has q = (q_x, -q_y, q_z); its y term enters with the sign s (dq_y/dA_y = -s dt).
struct WPair {
  double ax, ay, az;  // block s = +1
  double bx, by, bz;  // block s = -1
};

// One backward step on W given the step's coefficients: k1 = C^2 - S^2 x, kq = 2 S^2, cb = S^2 + C D,
// cs = C S, and the cross products u x W with u = l q, where the rotation takes -(2 C S / l) (u x W)
// and the terms -(S^2 / l) (u x W).  Returns the two terms summed over the blocks.
__device__ __forceinline__ double2 back_w(WPair& w, double qx, double qy, double qz, double k1, double kq, double cb,
                                          double cs, double l, double rot_c, double term_c) {
  const double ux = l * qx, uy = l * qy, uz = l * qz;
  const double p0 = fma(qz, w.az, fma(qy, w.ay, qx * w.ax));
  const double p1 = fma(qz, w.bz, fma(-qy, w.by, qx * w.bx));
  const double c0x = fma(uy, w.az, -(uz * w.ay)), c0y = fma(uz, w.ax, -(ux * w.az)), c0z = fma(ux, w.ay, -(uy * w.ax));
  const double c1x = fma(-uy, w.bz, -(uz * w.by)), c1y = fma(uz, w.bx, -(ux * w.bz)), c1z = fma(ux, w.by, uy * w.bx);
  const double bp = cb * (p0 + p1);
  const double gx = fma(qx, bp, fma(-term_c, c0x + c1x, cs * (w.ax + w.bx)));
  const double gy = fma(qy, bp, fma(-term_c, c0y - c1y, cs * (w.ay - w.by)));
  const double kp0 = kq * p0, kp1 = kq * p1;
  w.ax = fma(k1, w.ax, fma(kp0, qx, -(rot_c * c0x)));
  w.ay = fma(k1, w.ay, fma(kp0, qy, -(rot_c * c0y)));
  w.az = fma(k1, w.az, fma(kp0, qz, -(rot_c * c0z)));
  w.bx = fma(k1, w.bx, fma(kp1, qx, -(rot_c * c1x)));
  w.by = fma(k1, w.by, fma(-kp1, qy, -(rot_c * c1y)));
  w.bz = fma(k1, w.bz, fma(kp1, qz, -(rot_c * c1z)));
  return make_double2(gx, gy);
}

// Exact C, S form (the angle-halving path): l = 1, the products with 2 C S and S^2 are explicit.
__device__ __forceinline__ double2 back_w_exact(WPair& w, double2 r, double pxdt, double pydt, double qz, double qz2,
                                                int h, double inv4h) {
  const double qx = pxdt + r.x, qy = pydt + r.y;
  const double x = fma(qx, qx, fma(qy, qy, qz2));
  double C, S, D;
  csd(x, h, inv4h, C, S, D);
  const double S2 = S * S, cs = C * S;
  return back_w(w, qx, qy, qz, fma(-S2, x, C * C), S2 + S2, fma(C, D, S2), cs, 1.0, cs + cs, S2);
}

// Tangent form (steps within the fit's range): with S = C T and C D = -C^2 R, R = (T - 1)/x, the
// coefficients are C^2 (1 - T^2 x), 2 C^2 T^2, C^2 (T^2 - R) and C^2 T; C^2 = cos^2 sqrt x comes
// from its own series, R is the variant's fit (T = 1 + x R).  The cross products carry l = 2 C^2 T,
// which the rotation takes as it is and the terms times S^2 / l = T / 2.
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
__device__ __forceinline__ double2 back_w_tan(WPair& w, double2 r, double pxdt, double pydt, double qz, double qz2,
                                              const Fit<MODE>& f) {
  constexpr int M = kFitCos2Degree[MODE];
  const double qx = pxdt + r.x, qy = pydt + r.y;
  const double x = fma(qx, qx, fma(qy, qy, qz2));
  const double R = fit_R<MODE>(x, f);
  const double T = fma(R, x, 1.0);
  const double c2 = cos2_series<M>(x);
  const double T2 = T * T;
  const double cs = c2 * T, s2 = cs * T;
  return back_w(w, qx, qy, qz, c2 * fma(-T2, x, 1.0), s2 + s2, c2 * (T2 - R), cs, cs + cs, 1.0, 0.5 * T);
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

// One backward step in the form of the pulse's variant.
template <int MODE>
__device__ __forceinline__ double2 back_any(WPair& w, double2 r, double pxdt, double pydt, double qz, double qz2, int h,
                                            double inv4h, const typename FitOf<MODE>::type& f) {
  if constexpr (MODE < kFineHalving) return back_w_tan<MODE>(w, r, pxdt, pydt, qz, qz2, f);
  else return back_w_exact(w, r, pxdt, pydt, qz, qz2, h, inv4h);
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

  // t_f: normalise each block, alpha_s = <+_s(P_out)|psi_s>, final-state terms, and
  // W_s = Im(conj(alpha_s) <+_s|tau|psi_s>), the start of the backward sweep (chi'_s = alpha_s |+_s>)
  WPair w;
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
    // <+|tau_x|psi>, <+|tau_y|psi> (tau_y itself: s = 1), <+|tau_z|psi> = conj(u1) p1 - conj(u2) p2
    double vxr, vxi, vyr, vyi;
    tau_xy(up_out, p, 1.0, vxr, vxi, vyr, vyi);
    const double vzr = fma(up_out.ar, p.ar, fma(up_out.ai, p.ai, -fma(up_out.br, p.br, up_out.bi * p.bi)));
    const double vzi = fma(up_out.ar, p.ai, fma(-up_out.ai, p.ar, -fma(up_out.br, p.bi, -(up_out.bi * p.br))));
    const double wx = fma(al_r, vxi, -(al_i * vxr)), wy = fma(al_r, vyi, -(al_i * vyr)),
                 wz = fma(al_r, vzi, -(al_i * vzr));
    if (s == 0) {
      w.ax = wx; w.ay = wy; w.az = wz;
    } else {
      w.bx = wx; w.by = wy; w.bz = wz;
    }
  }

  // backward over the chunks in reverse, kGroup steps at a time (the last group of a chunk may be short)
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
    // a short group first (len not a multiple of kGroup), then full groups
    int top = len - 1;
    const int r = len % kGroup;
    if (r != 0) {
#pragma unroll 1
      for (int j = 0; j < r; ++j) buf[j][lane] = back_any<MODE>(w, tab[top - j], pxdt, pydt, qz, qz2, h, inv4h, fit);
      group_store(buf, red[wave], lane, top, r);
      top -= r;
    }
    for (; top >= 0; top -= kGroup) {
#pragma unroll
      for (int j = 0; j < kGroup; ++j)
        buf[j][lane] = back_any<MODE>(w, tab[top - j], pxdt, pydt, qz, qz2, h, inv4h, fit);
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

  // t_i: d|-> = -|+><+|dh|->/(2 w), dP = -dA(t_i).  With chi'_0 = a |+> + b |->, the part of W_0
  // across n = (P_x, s P_y, e)/w gives conj(a) <+|tau_k|-> = (n x W_0)_k, so the term of block s is
  // (n x W_0)_x / w for x and s (n x W_0)_y / w for y.
  const double Px = px - ain.x, Py = py - ain.y;
  const double inv_w2 = 1.0 / fma(Px, Px, fma(Py, Py, e * e));
  const double g_in_x = (fma(Py, w.az - w.bz, -(e * (w.ay + w.by)))) * inv_w2;
  const double g_in_y = (fma(e, w.ax - w.bx, -(Px * (w.az - w.bz)))) * inv_w2;
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
