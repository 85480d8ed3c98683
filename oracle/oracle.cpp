// Plain CPU oracle for the pair-yield evaluation of Fillion-Gourdeau, Hebenstreit,
// Gagnon & MacLean, "Pulse shape optimization for electron-positron production in
// rotating fields" (arXiv:1704.08919).
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or calls this
// file; only the test-suite, the smoke check and the benchmark's CPU-baseline leg do.
// It shares no code, header, constant or table with the HIP path.
//
// Every routine is written from the paper's definitions, slowly and literally:
//   * B-splines: Cox-de Boor recursion on a clamped knot vector (Sec. III, the
//     B-spline recursion and knot-vector equations).
//   * Field: cosine sum of the sampled spectrum times the Hann window (Sec. III, Eq. field
//     and Eq. hann); vector potential A(t) = -int_{t_f}^t E (Sec. III, Eq. vector_potential
//     with A(t_f) = 0), written as a definite integral that stays regular at zero frequency.
//   * Dirac evolution: the literal 4x4 momentum-space Dirac Hamiltonian in the Dirac
//     representation (Sec. II A, Eq. dirac_eq_mom), one exact exponential of the frozen
//     Hamiltonian at each step midpoint (a second-order unitary scheme).
//   * Projection: spin-traced overlap of the evolved negative-energy spinors with the
//     outgoing positive-energy spinors (Sec. II A, Eq. pair_prod_homo, free-spinor
//     equations), J as the midpoint-rule momentum integral (Sec. IV A, Eq. opt_prob).
//   * Quantum kinetic equation: the 6-component ODE of Sec. II B (Eq. qke, Eq. matrix)
//     with classical fourth-order Runge-Kutta; a cross-check, not part of the hot path.
//   * Fourth-order Magnus step (two Gauss-Legendre nodes), the fourth-order Dirac scheme that
//     Sec. V C names as future work; an extension checked by its convergence order.
//   * Gradients of J and U for the local search (Sec. IV A) by central differences.
//   * Differential evolution DE/rand/1/bin (Sec. IV B) driven by Philox4x32-10
//     (Salmon, Moraes, Dror, Shaw, SC'11), implemented from that paper's definition.
//
// Units: c = hbar = m = 1 and the charge is absorbed into the fields (eE -> E, eA -> A),
// so the Schwinger field is 1 (Sec. II).  The field lies in the x-y plane; p_z is the
// out-of-plane momentum (the paper's e_1 direction).
//
// Every routine is templated on the real type; the _ld entry points compute in long
// double (the parity reference), the _d entry points in double (the timed baseline).

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>

#include <omp.h>
#include <quadmath.h>

namespace {

inline int nthreads_or_default(int n) { return n > 0 ? n : omp_get_max_threads(); }

template <class R> inline R pi_() { return R(3.141592653589793238462643383279502884L); }

// Square root for every real type used here, including __float128 (quadmath).
inline double sqrt_r(double x) { return std::sqrt(x); }
inline long double sqrt_r(long double x) { return std::sqrt(x); }
inline __float128 sqrt_r(__float128 x) { return sqrtq(x); }

// ---------------------------------------------------------------------------------------
// B-splines (Sec. III): order k means degree k-1; clamped knots with multiplicity k at
// omega_min and omega_max and n - 2 equidistant simple interior knots, N_s = n + k - 2.
// ---------------------------------------------------------------------------------------
template <class R>
std::vector<R> knots(int k, int ns, R wmin, R wmax) {
  const int n = ns - k + 2;  // breakpoints, including the two end points
  std::vector<R> t;
  for (int i = 0; i < k; ++i) t.push_back(wmin);
  for (int i = 1; i < n - 1; ++i) t.push_back(wmin + (wmax - wmin) * R(i) / R(n - 1));
  for (int i = 0; i < k; ++i) t.push_back(wmax);
  return t;  // 2k + n - 2 = ns + k knots
}

// b_i^{(k)}(w), 0-based i, by the recursion with 0/0 := 0.  b^{(1)} is the indicator of the
// half-open knot span, except that the last non-empty span is closed at omega_max so that
// the sampled frequency Omega_N = omega_max is covered.
template <class R>
R bspline(int i, int k, const std::vector<R>& t, R w) {
  if (k == 1) {
    if (t[i] <= w && w < t[i + 1]) return R(1);
    if (w == t.back() && t[i] < t[i + 1] && t[i + 1] == t.back()) return R(1);
    return R(0);
  }
  R left = 0, right = 0;
  const R d1 = t[i + k - 1] - t[i];
  if (d1 != 0) left = (w - t[i]) / d1 * bspline(i, k - 1, t, w);
  const R d2 = t[i + k] - t[i + 1];
  if (d2 != 0) right = (t[i + k] - w) / d2 * bspline(i + 1, k - 1, t, w);
  return left + right;
}

// ---------------------------------------------------------------------------------------
// Spectral sampling and field synthesis (Sec. III).
// coeff layout per pulse: [component l in {x,y}][kind in {amplitude, phase}][N_s];
// a phase coefficient c in [-1,1] maps to a^(phi) = pi (c + 1) in [0, 2 pi].
// ---------------------------------------------------------------------------------------
template <class R>
struct Pulse {
  int ns = 0, order = 0, nt = 0, norm = 0;
  R wmin = 0, wmax = 0, T = 0, norm_value = 0;
  R dw = 0;           // Delta omega = 2 pi / T
  long nmin = 0;      // N_min = omega_min / Delta omega
  int nmodes = 0;     // N + 1
  std::vector<R> Om;  // Omega_j
  std::vector<R> Ej[2], Phj[2];
  R scale = 1;
};

template <class R>
Pulse<R> make_pulse(int ns, int order, double wmin, double wmax, double T, int nt, int norm,
                    double norm_value, const double* coeff) {
  Pulse<R> P;
  P.ns = ns; P.order = order; P.nt = nt; P.norm = norm;
  P.wmin = R(wmin); P.wmax = R(wmax); P.T = R(T); P.norm_value = R(norm_value);
  P.dw = R(2) * pi_<R>() / P.T;
  P.nmin = std::lround((long double)(P.wmin / P.dw));
  const long N = (long)std::floor((long double)((P.wmax - P.wmin) / P.dw) + 1e-9L);
  P.nmodes = (int)N + 1;
  const std::vector<R> t = knots<R>(order, ns, P.wmin, P.wmax);
  P.Om.resize(P.nmodes);
  for (int l = 0; l < 2; ++l) { P.Ej[l].assign(P.nmodes, 0); P.Phj[l].assign(P.nmodes, 0); }
  for (int j = 0; j < P.nmodes; ++j) {
    P.Om[j] = R(P.nmin + j) * P.dw;
    // the lines sample the band [omega_min, omega_max] including both ends: the basis is
    // evaluated at Omega_j clamped into the band, so rounding of (N_min + j) Delta omega cannot
    // move an end line off its end knot
    const R wb = std::min(std::max(P.Om[j], P.wmin), P.wmax);
    for (int i = 0; i < ns; ++i) {
      const R b = bspline<R>(i, order, t, wb);
      for (int l = 0; l < 2; ++l) {
        const R aE = R(coeff[(l * 2 + 0) * ns + i]);
        const R aP = pi_<R>() * (R(coeff[(l * 2 + 1) * ns + i]) + R(1));
        P.Ej[l][j] += aE * b;
        P.Phj[l][j] += aP * b;
      }
    }
  }
  return P;
}

// Hann-windowed cosine sum, unscaled: E_l(t) = cos^2(pi t / T) sum_j E_lj cos(Om_j t - Phi_lj).
template <class R>
void field(const Pulse<R>& P, R t, R E[2]) {
  const R g = std::cos(pi_<R>() * t / P.T);
  for (int l = 0; l < 2; ++l) {
    R s = 0;
    for (int j = 0; j < P.nmodes; ++j) s += P.Ej[l][j] * std::cos(P.Om[j] * t - P.Phj[l][j]);
    E[l] = g * g * s;
  }
}

// Time derivative of the unscaled field (used by the kinetic-equation cross-check only).
template <class R>
void field_dot(const Pulse<R>& P, R t, R Ed[2]) {
  const R a = pi_<R>() * t / P.T;
  const R g = std::cos(a) * std::cos(a);
  const R gd = -R(2) * std::cos(a) * std::sin(a) * pi_<R>() / P.T;
  for (int l = 0; l < 2; ++l) {
    R s = 0, sd = 0;
    for (int j = 0; j < P.nmodes; ++j) {
      const R ph = P.Om[j] * t - P.Phj[l][j];
      s += P.Ej[l][j] * std::cos(ph);
      sd -= P.Ej[l][j] * P.Om[j] * std::sin(ph);
    }
    Ed[l] = gd * s + g * sd;
  }
}

// I(w, phi; t) = int_{t_f}^{t} cos(w s + phi) ds = (t - t_f) cos(w (t + t_f)/2 + phi) sinc(w (t - t_f)/2)
template <class R>
R cos_integral(R w, R phi, R t, R tf) {
  const R h = t - tf;
  const R z = w * h / R(2);
  const R sinc = (z == 0) ? R(1) : std::sin(z) / z;
  return h * std::cos(w * (t + tf) / R(2) + phi) * sinc;
}

// Unscaled A_l(t) = -int_{t_f}^t E_l.  With cos^2 = (1 + cos(2 Om_T s))/2 and 2 Om_T = Delta omega,
// each spectral line splits into frequencies Om_j and Delta omega +- Om_j.
template <class R>
void potential(const Pulse<R>& P, R t, R A[2]) {
  const R tf = P.T / R(2);
  for (int l = 0; l < 2; ++l) {
    R s = 0;
    for (int j = 0; j < P.nmodes; ++j) {
      const R w = P.Om[j], ph = P.Phj[l][j];
      const R I0 = cos_integral<R>(w, -ph, t, tf);
      const R Ip = cos_integral<R>(P.dw + w, -ph, t, tf);
      const R Im = cos_integral<R>(P.dw - w, ph, t, tf);
      s += P.Ej[l][j] * (I0 / R(2) + Ip / R(4) + Im / R(4));
    }
    A[l] = -s;
  }
}

// Normalisation: 0 = none, 1 = peak |E| over the Nt+1 step nodes, 2 = energy U = int E^2 dt
// (midpoint rule on the step midpoints), Sec. III Eq. energy and Sec. IV B (global renormalisation).
template <class R>
void set_scale(Pulse<R>& P) {
  const R dt = P.T / R(P.nt);
  const R ti = -P.T / R(2);
  if (P.norm == 1) {
    R peak = 0;
    for (int n = 0; n <= P.nt; ++n) {
      R E[2];
      field<R>(P, ti + R(n) * dt, E);
      peak = std::max(peak, std::sqrt(E[0] * E[0] + E[1] * E[1]));
    }
    P.scale = (peak > 0) ? P.norm_value / peak : R(0);
  } else if (P.norm == 2) {
    R U = 0;
    for (int n = 0; n < P.nt; ++n) {
      R E[2];
      field<R>(P, ti + (R(n) + R(0.5)) * dt, E);
      U += E[0] * E[0] + E[1] * E[1];
    }
    U *= dt;
    P.scale = (U > 0) ? std::sqrt(P.norm_value / U) : R(0);
  } else {
    P.scale = 1;
  }
}

// ---------------------------------------------------------------------------------------
// Dirac equation in momentum space (Sec. II A).  Dirac representation:
// alpha = sigma_x (x) sigma, beta = sigma_z (x) 1, so H(P) = [[m, sigma.P], [sigma.P, -m]].
// ---------------------------------------------------------------------------------------
template <class R> using C = std::complex<R>;

template <class R>
void sigma_dot(const R P[3], C<R> s[2][2]) {
  s[0][0] = C<R>(P[2], 0);     s[0][1] = C<R>(P[0], -P[1]);
  s[1][0] = C<R>(P[0], P[1]);  s[1][1] = C<R>(-P[2], 0);
}

template <class R>
void hamiltonian(const R P[3], C<R> H[4][4]) {
  C<R> s[2][2];
  sigma_dot<R>(P, s);
  for (int a = 0; a < 4; ++a) for (int b = 0; b < 4; ++b) H[a][b] = 0;
  for (int a = 0; a < 2; ++a) {
    H[a][a] = R(1);
    H[a + 2][a + 2] = R(-1);
    for (int b = 0; b < 2; ++b) { H[a][b + 2] = s[a][b]; H[a + 2][b] = s[a][b]; }
  }
}

// Free spinors at kinematic momentum P (Sec. II A): norm^2 = 2 omega.
// u_s = [(omega+m) xi_s, (sigma.P) xi_s] / sqrt(omega+m),
// v_s = [-(sigma.P) eta_s, (omega+m) eta_s] / sqrt(omega+m),
// xi_1 = eta_2 = (1,0), xi_2 = eta_1 = (0,1).
template <class R>
void free_spinors(const R P[3], C<R> u[2][4], C<R> v[2][4], R* omega) {
  const R w = std::sqrt(R(1) + P[0] * P[0] + P[1] * P[1] + P[2] * P[2]);
  const R nrm = R(1) / std::sqrt(w + R(1));
  C<R> s[2][2];
  sigma_dot<R>(P, s);
  const int xi_up[2] = {0, 1};   // xi_1 = (1,0) -> component 0; xi_2 = (0,1) -> component 1
  const int eta_up[2] = {1, 0};  // eta_1 = (0,1), eta_2 = (1,0)
  for (int sp = 0; sp < 2; ++sp) {
    const int a = xi_up[sp];
    u[sp][0] = (a == 0 ? C<R>(w + 1) : C<R>(0)) * nrm;
    u[sp][1] = (a == 1 ? C<R>(w + 1) : C<R>(0)) * nrm;
    u[sp][2] = s[0][a] * nrm;
    u[sp][3] = s[1][a] * nrm;
    const int b = eta_up[sp];
    v[sp][0] = -s[0][b] * nrm;
    v[sp][1] = -s[1][b] * nrm;
    v[sp][2] = (b == 0 ? C<R>(w + 1) : C<R>(0)) * nrm;
    v[sp][3] = (b == 1 ? C<R>(w + 1) : C<R>(0)) * nrm;
  }
  *omega = w;
}

// Evolves both negative-energy spinors of one momentum mode through the A table and returns
// the spin-traced pair density
//   f = sum_{s,s'} |u_{s'}^out^dagger psi_s(t_f)|^2 / (2 omega_out 2 omega_in).
// One step: exact exponential of the Hamiltonian frozen at the midpoint t_{n+1/2};
// since H^2 = omega^2, exp(-i H dt) = cos(omega dt) - i sin(omega dt)/omega H.
// Optionally returns the final state psi[s][4] (scaled by 1/sqrt(2 omega_in)).
template <class R>
R evolve_mode(int nt, R dt, const double* Amid, const double Ain[2], const double Aout[2],
              const double p[3], double* psi_out /* [2][4][2] or null */) {
  const R px = R(p[0]), py = R(p[1]), pz = R(p[2]);
  R Pin[3] = {px - R(Ain[0]), py - R(Ain[1]), pz};
  C<R> u[2][4], v[2][4];
  R w_in;
  free_spinors<R>(Pin, u, v, &w_in);
  C<R> psi[2][4];
  for (int s = 0; s < 2; ++s) for (int a = 0; a < 4; ++a) psi[s][a] = v[s][a];
  C<R> H[4][4], U[4][4];
  for (int n = 0; n < nt; ++n) {
    R P[3] = {px - R(Amid[2 * n]), py - R(Amid[2 * n + 1]), pz};
    const R w = std::sqrt(R(1) + P[0] * P[0] + P[1] * P[1] + P[2] * P[2]);
    const R c = std::cos(w * dt), sw = std::sin(w * dt) / w;
    hamiltonian<R>(P, H);
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b)
        U[a][b] = (a == b ? C<R>(c) : C<R>(0)) - C<R>(0, 1) * sw * H[a][b];
    for (int s = 0; s < 2; ++s) {
      C<R> nxt[4];
      for (int a = 0; a < 4; ++a) {
        nxt[a] = 0;
        for (int b = 0; b < 4; ++b) nxt[a] += U[a][b] * psi[s][b];
      }
      for (int a = 0; a < 4; ++a) psi[s][a] = nxt[a];
    }
  }
  R Pout[3] = {px - R(Aout[0]), py - R(Aout[1]), pz};
  C<R> uo[2][4], vo[2][4];
  R w_out;
  free_spinors<R>(Pout, uo, vo, &w_out);
  R f = 0;
  for (int s = 0; s < 2; ++s)
    for (int sp = 0; sp < 2; ++sp) {
      C<R> ov = 0;
      for (int a = 0; a < 4; ++a) ov += std::conj(uo[sp][a]) * psi[s][a];
      f += std::norm(ov);
    }
  f /= (R(2) * w_out) * (R(2) * w_in);
  if (psi_out) {
    const R nrm = R(1) / std::sqrt(R(2) * w_in);
    for (int s = 0; s < 2; ++s)
      for (int a = 0; a < 4; ++a) {
        psi_out[(s * 4 + a) * 2 + 0] = double(psi[s][a].real() * nrm);
        psi_out[(s * 4 + a) * 2 + 1] = double(psi[s][a].imag() * nrm);
      }
  }
  return f;
}

// ---------------------------------------------------------------------------------------
// Fourth-order step (an extension: the paper names a fourth-order Dirac scheme as future work,
// Sec. V C).  Fourth-order Magnus integrator with two Gauss-Legendre nodes (Blanes, Casas, Oteo
// & Ros, Phys. Rep. 470 (2009) 151, Sec. 5): for i dpsi/dt = H psi, with
//   H_1 = H(t_n + c_1 dt), H_2 = H(t_n + c_2 dt), c_{1,2} = 1/2 -+ sqrt(3)/6,
//   Omega = -i dt/2 (H_1 + H_2) - sqrt(3)/12 dt^2 [H_2, H_1],   psi_{n+1} = exp(Omega) psi_n.
// exp(Omega) psi is summed as its Taylor series until the terms drop below long-double
// resolution (|Omega| < 1 for the step sizes used).  Ag holds A at the two nodes of every step,
// [nt][2 nodes][2 components].
// ---------------------------------------------------------------------------------------
template <class R>
void apply_exp(const C<R> W[4][4], C<R> psi[4]) {
  C<R> term[4], sum[4];
  for (int a = 0; a < 4; ++a) term[a] = sum[a] = psi[a];
  for (int k = 1; k < 200; ++k) {
    C<R> nxt[4];
    R mag = 0;
    for (int a = 0; a < 4; ++a) {
      nxt[a] = 0;
      for (int b = 0; b < 4; ++b) nxt[a] += W[a][b] * term[b];
      nxt[a] /= R(k);
      mag = std::max(mag, std::abs(nxt[a]));
    }
    for (int a = 0; a < 4; ++a) { term[a] = nxt[a]; sum[a] += nxt[a]; }
    if (mag < R(1e-40)) break;
  }
  for (int a = 0; a < 4; ++a) psi[a] = sum[a];
}

template <class R>
R evolve4_mode(int nt, R dt, const double* Ag, const double Ain[2], const double Aout[2], const double p[3]) {
  const R px = R(p[0]), py = R(p[1]), pz = R(p[2]);
  const R kc = std::sqrt(R(3)) / R(12);
  R Pin[3] = {px - R(Ain[0]), py - R(Ain[1]), pz};
  C<R> u[2][4], v[2][4];
  R w_in;
  free_spinors<R>(Pin, u, v, &w_in);
  C<R> psi[2][4];
  for (int s = 0; s < 2; ++s) for (int a = 0; a < 4; ++a) psi[s][a] = v[s][a];
  C<R> H1[4][4], H2[4][4], W[4][4];
  for (int n = 0; n < nt; ++n) {
    R P1[3] = {px - R(Ag[4 * n + 0]), py - R(Ag[4 * n + 1]), pz};
    R P2[3] = {px - R(Ag[4 * n + 2]), py - R(Ag[4 * n + 3]), pz};
    hamiltonian<R>(P1, H1);
    hamiltonian<R>(P2, H2);
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        C<R> cm = 0;  // [H_2, H_1]_{ab}
        for (int c = 0; c < 4; ++c) cm += H2[a][c] * H1[c][b] - H1[a][c] * H2[c][b];
        W[a][b] = C<R>(0, -1) * (dt / R(2)) * (H1[a][b] + H2[a][b]) - kc * dt * dt * cm;
      }
    for (int s = 0; s < 2; ++s) apply_exp<R>(W, psi[s]);
  }
  R Pout[3] = {px - R(Aout[0]), py - R(Aout[1]), pz};
  C<R> uo[2][4], vo[2][4];
  R w_out;
  free_spinors<R>(Pout, uo, vo, &w_out);
  R f = 0;
  for (int s = 0; s < 2; ++s)
    for (int sp = 0; sp < 2; ++sp) {
      C<R> ov = 0;
      for (int a = 0; a < 4; ++a) ov += std::conj(uo[sp][a]) * psi[s][a];
      f += std::norm(ov);
    }
  return f / ((R(2) * w_out) * (R(2) * w_in));
}

// ---------------------------------------------------------------------------------------
// Split-operator steps (Sec. II A names a second-order split-operator scheme; Sec. V C names a
// fourth-order splitting as future work).  The frozen Hamiltonian splits into the part the field
// does not touch and the field-driven transverse part,
//   H_0 = alpha_z p_z + beta m,   H_perp(t) = alpha_x P_x(t) + alpha_y P_y(t),
// (at p_z = 0 this is the mass / kinetic split), and each factor is exponentiated exactly:
// H_0^2 = (m^2 + p_z^2) 1 and H_perp^2 = (P_x^2 + P_y^2) 1, so
//   exp(-i H h) = cos(|H| h) - i sin(|H| h) / |H| * H   for either part.
// One Strang step of size h with the transverse field frozen at the step midpoint:
//   psi <- exp(-i H_0 h/2) exp(-i H_perp(t + h/2) h) exp(-i H_0 h/2) psi.
// Fourth order: the triple-jump composition of that symmetric step (Yoshida, Phys. Lett. A 150
// (1990) 262), sizes w1 dt, w0 dt, w1 dt with w1 = 1 / (2 - 2^(1/3)), w0 = 1 - 2 w1; the field of
// substep i is taken at its own midpoint, i.e. at t_n + c_i dt with c = (w1/2, 1/2, 1 - w1/2).
// At[nt][nsub][2] holds A at those points (nsub = 1: the step midpoint).
// ---------------------------------------------------------------------------------------
template <class R>
void apply_matrix(const C<R> U[4][4], C<R> psi[4]) {
  C<R> nxt[4];
  for (int a = 0; a < 4; ++a) {
    nxt[a] = 0;
    for (int b = 0; b < 4; ++b) nxt[a] += U[a][b] * psi[b];
  }
  for (int a = 0; a < 4; ++a) psi[a] = nxt[a];
}

// exp(-i H h) for a Hermitian 4x4 H with H^2 = w^2 1 (w >= 0).
template <class R>
void exp_involutive(const C<R> H[4][4], R w, R h, C<R> U[4][4]) {
  const R c = std::cos(w * h), sw = (w > 0) ? std::sin(w * h) / w : h;
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) U[a][b] = (a == b ? C<R>(c) : C<R>(0)) - C<R>(0, 1) * sw * H[a][b];
}

template <class R>
R evolve_split_mode(int nt, R dt, int nsub, const double* At, const double Ain[2], const double Aout[2],
                    const double p[3]) {
  const R px = R(p[0]), py = R(p[1]), pz = R(p[2]);
  const R w1 = R(1) / (R(2) - std::cbrt(R(2)));
  const R w[3] = {nsub == 1 ? R(1) : w1, R(1) - R(2) * w1, w1};
  R Pin[3] = {px - R(Ain[0]), py - R(Ain[1]), pz};
  C<R> u[2][4], v[2][4];
  R w_in;
  free_spinors<R>(Pin, u, v, &w_in);
  C<R> psi[2][4];
  for (int s = 0; s < 2; ++s) for (int a = 0; a < 4; ++a) psi[s][a] = v[s][a];
  // H_0 = alpha_z p_z + beta m: the Hamiltonian at P = (0, 0, p_z) minus nothing else.
  const R Pz[3] = {R(0), R(0), pz};
  C<R> H0[4][4];
  hamiltonian<R>(Pz, H0);
  const R e = std::sqrt(R(1) + pz * pz);
  for (int n = 0; n < nt; ++n)
    for (int i = 0; i < nsub; ++i) {
      const R h = w[i] * dt;
      const R Px = px - R(At[2 * (nsub * n + i)]), Py = py - R(At[2 * (nsub * n + i) + 1]);
      // H_perp = alpha_x P_x + alpha_y P_y: the Hamiltonian at (P_x, P_y, 0) without beta m
      const R Pp[3] = {Px, Py, R(0)};
      C<R> Hp[4][4], Uh[4][4], Up[4][4];
      hamiltonian<R>(Pp, Hp);
      for (int a = 0; a < 4; ++a) Hp[a][a] -= (a < 2 ? R(1) : R(-1));
      exp_involutive<R>(H0, e, h / R(2), Uh);
      exp_involutive<R>(Hp, std::sqrt(Px * Px + Py * Py), h, Up);
      for (int s = 0; s < 2; ++s) {
        apply_matrix<R>(Uh, psi[s]);
        apply_matrix<R>(Up, psi[s]);
        apply_matrix<R>(Uh, psi[s]);
      }
    }
  R Pout[3] = {px - R(Aout[0]), py - R(Aout[1]), pz};
  C<R> uo[2][4], vo[2][4];
  R w_out;
  free_spinors<R>(Pout, uo, vo, &w_out);
  R f = 0;
  for (int s = 0; s < 2; ++s)
    for (int sp = 0; sp < 2; ++sp) {
      C<R> ov = 0;
      for (int a = 0; a < 4; ++a) ov += std::conj(uo[sp][a]) * psi[s][a];
      f += std::norm(ov);
    }
  return f / ((R(2) * w_out) * (R(2) * w_in));
}

// ---------------------------------------------------------------------------------------
// Quantum kinetic equation (Sec. II B), 6 components, classical RK4.  The paper's field
// plane (e_2, e_3) is the x-y plane here and e_1 is z (a cyclic relabelling, so
// (E x Edot).e_1 = Ex Edot_y - Ey Edot_x and p_1 = p_z).  f = 1 - chi_1.
// For a field along x only, the signed Q = E_x sqrt(1 + P_y^2 + p_z^2) / omega^2 is used:
// the unsigned root flips the e_2 basis vector whenever E crosses zero.
// ---------------------------------------------------------------------------------------
// Field samples needed by RK4 over [-T/2, T/2] with nt steps: E, dE/dt and A at the 2 nt + 1
// points t_i + h dt/2, h = 0..2nt (scaled), tabulated once per pulse and shared by all modes.
template <class R>
struct QkeTable {
  std::vector<R> E, Ed, A;  // [2nt+1][2]
};

template <class R>
QkeTable<R> qke_table(const Pulse<R>& Pu, int nt) {
  QkeTable<R> tb;
  const int nh = 2 * nt + 1;
  tb.E.resize(2 * nh); tb.Ed.resize(2 * nh); tb.A.resize(2 * nh);
  const R dt = Pu.T / R(nt), ti = -Pu.T / R(2);
  for (int h = 0; h < nh; ++h) {
    const R t = ti + R(h) * dt / R(2);
    R E[2], Ed[2], A[2];
    field<R>(Pu, t, E);
    field_dot<R>(Pu, t, Ed);
    potential<R>(Pu, t, A);
    for (int l = 0; l < 2; ++l) {
      tb.E[2 * h + l] = Pu.scale * E[l];
      tb.Ed[2 * h + l] = Pu.scale * Ed[l];
      tb.A[2 * h + l] = Pu.scale * A[l];
    }
  }
  return tb;
}

// Right-hand side N(t,P) chi at table point h.
template <class R>
void qke_rhs(const QkeTable<R>& tb, bool linear, int h, const R p[3], const R chi[6], R out[6]) {
  const R* E = &tb.E[2 * h];
  const R* Ed = &tb.Ed[2 * h];
  const R* A = &tb.A[2 * h];
  const R Px = p[0] - A[0], Py = p[1] - A[1], pz = p[2];
  const R w2 = R(1) + Px * Px + Py * Py + pz * pz;
  const R w = sqrt_r(w2);
  const R eperp = sqrt_r(R(1) + pz * pz);
  R Q, Rr;
  if (linear) {
    Q = E[0] * sqrt_r(R(1) + Py * Py + pz * pz) / w2;
    Rr = 0;
  } else {
    const R EE = E[0] * E[0] + E[1] * E[1];
    const R EP = E[0] * Px + E[1] * Py;
    const R X = w2 * EE - EP * EP;
    Q = (X > 0) ? sqrt_r(X) / w2 : R(0);
    Rr = (X > 0) ? eperp * w * (E[0] * Ed[1] - E[1] * Ed[0]) / X : R(0);
  }
  // N(t,P), skew-symmetric (Eq. matrix)
  out[0] = -Q * chi[1];
  out[1] = Q * chi[0] - R(2) * w * chi[2] + Rr * chi[3];
  out[2] = R(2) * w * chi[1] - Rr * chi[4];
  out[3] = -Rr * chi[1] + R(2) * w * chi[4];
  out[4] = Rr * chi[2] - R(2) * w * chi[3] + Q * chi[5];
  out[5] = -Q * chi[4];
}

template <class R>
R qke_mode(const QkeTable<R>& tb, bool linear, int nt, R dt, const double p[3], double* fmax = nullptr) {
  const R pr[3] = {R(p[0]), R(p[1]), R(p[2])};
  R chi[6] = {1, 0, 0, 0, 0, 0};
  R k1[6], k2[6], k3[6], k4[6], tmp[6];
  double peak = 0;
  for (int n = 0; n < nt; ++n) {
    qke_rhs<R>(tb, linear, 2 * n, pr, chi, k1);
    for (int i = 0; i < 6; ++i) tmp[i] = chi[i] + dt / R(2) * k1[i];
    qke_rhs<R>(tb, linear, 2 * n + 1, pr, tmp, k2);
    for (int i = 0; i < 6; ++i) tmp[i] = chi[i] + dt / R(2) * k2[i];
    qke_rhs<R>(tb, linear, 2 * n + 1, pr, tmp, k3);
    for (int i = 0; i < 6; ++i) tmp[i] = chi[i] + dt * k3[i];
    qke_rhs<R>(tb, linear, 2 * n + 2, pr, tmp, k4);
    for (int i = 0; i < 6; ++i) chi[i] += dt / R(6) * (k1[i] + R(2) * k2[i] + R(2) * k3[i] + k4[i]);
    if (fmax) peak = std::max(peak, std::fabs(double(R(1) - chi[0])));
  }
  if (fmax) *fmax = peak;
  return R(1) - chi[0];
}

// ---------------------------------------------------------------------------------------
// Momentum grid: cell-centred points p_d = lo_d + (i + 1/2) (hi_d - lo_d)/n_d; a dimension
// with n_d = 1 and lo_d = hi_d is a sheet (p_d = lo_d, no measure factor).  Mode order:
// x fastest, then y, then z.
// ---------------------------------------------------------------------------------------
inline void grid_point(const int n[3], const double lo[3], const double hi[3], long idx, double p[3]) {
  long ix = idx % n[0];
  long iy = (idx / n[0]) % n[1];
  long iz = idx / ((long)n[0] * n[1]);
  const long id[3] = {ix, iy, iz};
  for (int d = 0; d < 3; ++d) {
    if (n[d] == 1 && lo[d] == hi[d]) p[d] = lo[d];
    else p[d] = lo[d] + (double(id[d]) + 0.5) * (hi[d] - lo[d]) / double(n[d]);
  }
}

inline double cell_volume(const int n[3], const double lo[3], const double hi[3]) {
  double v = 1;
  for (int d = 0; d < 3; ++d)
    if (!(n[d] == 1 && lo[d] == hi[d])) v *= (hi[d] - lo[d]) / double(n[d]);
  return v;
}

// ---------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): 10 rounds of the 4x32 Philox S-box with
// multipliers 0xD2511F53, 0xCD9E8D57 and Weyl key increments 0x9E3779B9, 0xBB67AE85.
// ---------------------------------------------------------------------------------------
void philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint64_t m0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t m1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t hi0 = (uint32_t)(m0 >> 32), lo0 = (uint32_t)m0;
    const uint32_t hi1 = (uint32_t)(m1 >> 32), lo1 = (uint32_t)m1;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// Draw word w (0..3) of block b for individual i in generation g.
inline uint32_t de_word(uint64_t seed, int64_t g, int i, int b, int w) {
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  const uint32_t ctr[4] = {(uint32_t)i, (uint32_t)b, (uint32_t)(uint64_t)g, (uint32_t)((uint64_t)g >> 32)};
  uint32_t o[4];
  philox(ctr, key, o);
  return o[w];
}

inline uint32_t uniform_index(uint32_t u, uint32_t n) { return (uint32_t)(((uint64_t)u * n) >> 32); }
inline double uniform_open01(uint32_t u) { return (double(u) + 0.5) * (1.0 / 4294967296.0); }

// Neumaier-compensated sum of f in mode order, times the cell volume.
double yield_sum(const int n[3], const double lo[3], const double hi[3], const double* f) {
  const long nm = (long)n[0] * n[1] * n[2];
  double s = 0, c = 0;
  for (long m = 0; m < nm; ++m) {
    const double x = f[m];
    const double t = s + x;
    if (std::fabs(s) >= std::fabs(x)) c += (s - t) + x; else c += (x - t) + s;
    s = t;
  }
  return cell_volume(n, lo, hi) * (s + c);
}

template <class R>
void synth_impl(int ns, int order, double wmin, double wmax, double T, int nt, int norm,
                       double norm_value, const double* coeff, double* Amid, double* Emid,
                       double* Aedge, double* scale) {
  auto P = make_pulse<R>(ns, order, wmin, wmax, T, nt, norm, norm_value, coeff);
  set_scale<R>(P);
  const R dt = P.T / R(nt), ti = -P.T / R(2), tf = P.T / R(2);
  for (int n = 0; n < nt; ++n) {
    const R t = ti + (R(n) + R(0.5)) * dt;
    R a[2];
    potential<R>(P, t, a);
    Amid[2 * n] = double(P.scale * a[0]);
    Amid[2 * n + 1] = double(P.scale * a[1]);
    if (Emid) {
      R e[2];
      field<R>(P, t, e);
      Emid[2 * n] = double(P.scale * e[0]);
      Emid[2 * n + 1] = double(P.scale * e[1]);
    }
  }
  R a0[2], a1[2];
  potential<R>(P, ti, a0);
  potential<R>(P, tf, a1);
  Aedge[0] = double(P.scale * a0[0]); Aedge[1] = double(P.scale * a0[1]);
  Aedge[2] = double(P.scale * a1[0]); Aedge[3] = double(P.scale * a1[1]);
  *scale = double(P.scale);
}

template <class R>
void evolve_impl(int nt, double dt, const double* Amid, const double* Aedge, long nm,
                        const double* p, double* f, int nthreads) {
  const int nth = nthreads_or_default(nthreads);
#pragma omp parallel for schedule(dynamic, 16) num_threads(nth)
  for (long m = 0; m < nm; ++m)
    f[m] = double(evolve_mode<R>(nt, R(dt), Amid, Aedge, Aedge + 2, p + 3 * m, nullptr));
}

template <class R>
double evaluate_impl(int ns, int order, double wmin, double wmax, double T, int nt, int norm,
                            double norm_value, const double* coeff, const int* n, const double* lo,
                            const double* hi, double* f, int nthreads) {
  std::vector<double> Amid(2 * (size_t)nt), Aedge(4);
  double scale;
  synth_impl<R>(ns, order, wmin, wmax, T, nt, norm, norm_value, coeff, Amid.data(), nullptr, Aedge.data(), &scale);
  const long nm = (long)n[0] * n[1] * n[2];
  std::vector<double> p(3 * (size_t)nm), ff((size_t)nm);
  for (long m = 0; m < nm; ++m) grid_point(n, lo, hi, m, p.data() + 3 * m);
  evolve_impl<R>(nt, T / nt, Amid.data(), Aedge.data(), nm, p.data(), ff.data(), nthreads);
  if (f) std::memcpy(f, ff.data(), sizeof(double) * nm);
  return yield_sum(n, lo, hi, ff.data());
}

}  // namespace

// =======================================================================================
// C entry points (ctypes).  Sizes are plain ints; arrays are contiguous, row-major.
// =======================================================================================
extern "C" {

int orc_version(void) { return 1; }

// B-spline basis values b_i^{(k)}(w) for i = 0..ns-1.
void orc_bspline_ld(int order, int ns, double wmin, double wmax, double w, double* out) {
  using R = long double;
  const auto t = knots<R>(order, ns, wmin, wmax);
  for (int i = 0; i < ns; ++i) out[i] = double(bspline<R>(i, order, t, R(w)));
}

// Spectral samples: Omega[N+1], E[2][N+1], Phi[2][N+1]; returns N+1 (or the required size if
// cap is too small, without writing).
int orc_spectra_ld(int ns, int order, double wmin, double wmax, double T, const double* coeff,
                   int cap, double* Om, double* E, double* Ph) {
  auto P = make_pulse<long double>(ns, order, wmin, wmax, T, 2, 0, 0, coeff);
  if (P.nmodes > cap) return P.nmodes;
  for (int j = 0; j < P.nmodes; ++j) {
    Om[j] = double(P.Om[j]);
    for (int l = 0; l < 2; ++l) {
      E[l * P.nmodes + j] = double(P.Ej[l][j]);
      Ph[l * P.nmodes + j] = double(P.Phj[l][j]);
    }
  }
  return P.nmodes;
}

// Unscaled E(t) and A(t) at arbitrary times: E[n][2], A[n][2].
void orc_field_at_ld(int ns, int order, double wmin, double wmax, double T, const double* coeff,
                     int n, const double* t, double* E, double* A) {
  auto P = make_pulse<long double>(ns, order, wmin, wmax, T, 2, 0, 0, coeff);
  for (int i = 0; i < n; ++i) {
    long double e[2], a[2];
    field<long double>(P, (long double)t[i], e);
    potential<long double>(P, (long double)t[i], a);
    E[2 * i] = double(e[0]); E[2 * i + 1] = double(e[1]);
    A[2 * i] = double(a[0]); A[2 * i + 1] = double(a[1]);
  }
}

// Full synthesis of one pulse: scaled A and E at the nt step midpoints (A_mid[nt][2],
// E_mid[nt][2] or null), A_edge = [A(t_i), A(t_f)] (4 values), scale.
void orc_synth_ld(int ns, int order, double wmin, double wmax, double T, int nt, int norm,
                  double norm_value, const double* coeff, double* Amid, double* Emid,
                  double* Aedge, double* scale) {
  synth_impl<long double>(ns, order, wmin, wmax, T, nt, norm, norm_value, coeff, Amid, Emid, Aedge, scale);
}
void orc_synth_d(int ns, int order, double wmin, double wmax, double T, int nt, int norm,
                 double norm_value, const double* coeff, double* Amid, double* Emid,
                 double* Aedge, double* scale) {
  synth_impl<double>(ns, order, wmin, wmax, T, nt, norm, norm_value, coeff, Amid, Emid, Aedge, scale);
}

// Pair density f at explicit momenta p[nm][3] for an A table (any table, not only a synthesised
// one).  nthreads <= 0 uses the OpenMP default.
void orc_evolve_points_ld(int nt, double dt, const double* Amid, const double* Aedge, long nm,
                          const double* p, double* f, int nthreads) {
  evolve_impl<long double>(nt, dt, Amid, Aedge, nm, p, f, nthreads);
}
void orc_evolve_points_d(int nt, double dt, const double* Amid, const double* Aedge, long nm,
                         const double* p, double* f, int nthreads) {
  evolve_impl<double>(nt, dt, Amid, Aedge, nm, p, f, nthreads);
}

// Final state of one mode: psi[2 spins][4][re,im], unit-normalised initial spinors.
double orc_evolve_state_ld(int nt, double dt, const double* Amid, const double* Aedge,
                           const double* p, double* psi) {
  return double(evolve_mode<long double>(nt, (long double)dt, Amid, Aedge, Aedge + 2, p, psi));
}

// Unit-normalised free spinors at kinematic momentum P: u[2][4][2], v[2][4][2]; returns omega.
double orc_free_spinors_ld(const double* P, double* u, double* v) {
  using R = long double;
  R Pr[3] = {R(P[0]), R(P[1]), R(P[2])};
  C<R> uu[2][4], vv[2][4];
  R w;
  free_spinors<R>(Pr, uu, vv, &w);
  const R nrm = R(1) / std::sqrt(R(2) * w);
  for (int s = 0; s < 2; ++s)
    for (int a = 0; a < 4; ++a) {
      u[(s * 4 + a) * 2] = double(uu[s][a].real() * nrm); u[(s * 4 + a) * 2 + 1] = double(uu[s][a].imag() * nrm);
      v[(s * 4 + a) * 2] = double(vv[s][a].real() * nrm); v[(s * 4 + a) * 2 + 1] = double(vv[s][a].imag() * nrm);
    }
  return double(w);
}

// Grid points of a cell-centred grid: p[nx*ny*nz][3]; returns the cell volume.
double orc_grid_points(const int* n, const double* lo, const double* hi, double* p) {
  const long nm = (long)n[0] * n[1] * n[2];
  for (long m = 0; m < nm; ++m) grid_point(n, lo, hi, m, p + 3 * m);
  return cell_volume(n, lo, hi);
}

// J = Delta V * sum_p f(p), Neumaier-compensated, in mode order.
double orc_yield(const int* n, const double* lo, const double* hi, const double* f) {
  return yield_sum(n, lo, hi, f);
}

// Whole objective for one pulse: synthesis, evolution of every grid mode, yield.
// f (optional) receives the per-mode densities in mode order.
double orc_evaluate_ld(int ns, int order, double wmin, double wmax, double T, int nt, int norm,
                       double norm_value, const double* coeff, const int* n, const double* lo,
                       const double* hi, double* f, int nthreads) {
  return evaluate_impl<long double>(ns, order, wmin, wmax, T, nt, norm, norm_value, coeff, n, lo, hi, f, nthreads);
}
double orc_evaluate_d(int ns, int order, double wmin, double wmax, double T, int nt, int norm,
                      double norm_value, const double* coeff, const int* n, const double* lo,
                      const double* hi, double* f, int nthreads) {
  return evaluate_impl<double>(ns, order, wmin, wmax, T, nt, norm, norm_value, coeff, n, lo, hi, f, nthreads);
}

// Kinetic-equation cross-check: f = 1 - chi_1 at momenta p[nm][3] for a synthesised pulse,
// RK4 with nt steps over [-T/2, T/2].  linear != 0 selects the signed-Q linear form.
void orc_qke_points_ld(int ns, int order, double wmin, double wmax, double T, int norm, double norm_value,
                       const double* coeff, int linear, int nt, long nm, const double* p, double* f,
                       int nthreads) {
  using R = long double;
  auto P = make_pulse<R>(ns, order, wmin, wmax, T, nt, norm, norm_value, coeff);
  set_scale<R>(P);
  const auto tb = qke_table<R>(P, nt);
  const int nth = nthreads_or_default(nthreads);
#pragma omp parallel for schedule(dynamic, 1) num_threads(nth)
  for (long m = 0; m < nm; ++m) f[m] = double(qke_mode<R>(tb, linear != 0, nt, P.T / R(nt), p + 3 * m));
}

// Kinetic-equation cross-check on caller-supplied samples: E, dE/dt and A at the 2 nt + 1 RK4
// points t_i + h dt / 2 (arrays [2nt+1][2]); the same RK4 as above.
void orc_qke_tabulated_ld(int nt, double dt, const double* E, const double* Ed, const double* A, int linear,
                          long nm, const double* p, double* f, int nthreads) {
  using R = long double;
  QkeTable<R> tb;
  const int nh = 2 * nt + 1;
  tb.E.assign(E, E + 2 * nh); tb.Ed.assign(Ed, Ed + 2 * nh); tb.A.assign(A, A + 2 * nh);
  const int nth = nthreads_or_default(nthreads);
#pragma omp parallel for schedule(dynamic, 1) num_threads(nth)
  for (long m = 0; m < nm; ++m) f[m] = double(qke_mode<R>(tb, linear != 0, nt, R(dt), p + 3 * m));
}

// Same kinetic equation in quadruple precision (__float128): the parity reference.  f = 1 - chi_1
// cancels to far below the pair density reached during the pulse, so a long-double evaluation
// carries an absolute error ~ 2^-64 sqrt(nt); in quadruple precision that error is ~ 1e-30.
// fmax[nm] (optional) receives the largest |1 - chi_1(t)| over the steps, which sets the FP64
// rounding floor of f.
void orc_qke_tabulated_q(int nt, double dt, const double* E, const double* Ed, const double* A, int linear,
                         long nm, const double* p, double* f, double* fmax, int nthreads) {
  using R = __float128;
  QkeTable<R> tb;
  const int nh = 2 * nt + 1;
  tb.E.assign(E, E + 2 * nh); tb.Ed.assign(Ed, Ed + 2 * nh); tb.A.assign(A, A + 2 * nh);
  const int nth = nthreads_or_default(nthreads);
#pragma omp parallel for schedule(dynamic, 1) num_threads(nth)
  for (long m = 0; m < nm; ++m) f[m] = double(qke_mode<R>(tb, linear != 0, nt, R(dt), p + 3 * m, fmax ? fmax + m : nullptr));
}

// Same kinetic equation computed in double (used to size the rounding floor of the parity bar).
void orc_qke_tabulated_d(int nt, double dt, const double* E, const double* Ed, const double* A, int linear,
                         long nm, const double* p, double* f, int nthreads) {
  QkeTable<double> tb;
  const int nh = 2 * nt + 1;
  tb.E.assign(E, E + 2 * nh); tb.Ed.assign(Ed, Ed + 2 * nh); tb.A.assign(A, A + 2 * nh);
  const int nth = nthreads_or_default(nthreads);
#pragma omp parallel for schedule(dynamic, 1) num_threads(nth)
  for (long m = 0; m < nm; ++m) f[m] = qke_mode<double>(tb, linear != 0, nt, dt, p + 3 * m);
}

// Scaled field samples of a synthesised pulse at t_i + (n + c_r) dt, n = 0..nt-1, r = 0..n_sub-1
// (row n n_sub + r), plus t_f as the last row when with_end != 0.  E, Ed (dE/dt) and A are
// [rows][2]; any of them may be null.  The scale is that of the pulse's normalisation.
void orc_field_samples_ld(int ns, int order, double wmin, double wmax, double T, int nt, int norm,
                          double norm_value, const double* coeff, int n_sub, const double* offsets,
                          int with_end, double* E, double* Ed, double* A) {
  using R = long double;
  auto P = make_pulse<R>(ns, order, wmin, wmax, T, nt, norm, norm_value, coeff);
  set_scale<R>(P);
  const R dt = P.T / R(nt), ti = -P.T / R(2);
  const long rows = (long)nt * n_sub + (with_end ? 1 : 0);
  for (long k = 0; k < rows; ++k) {
    const R t = (k == (long)nt * n_sub) ? P.T / R(2) : ti + (R(k / n_sub) + R(offsets[k % n_sub])) * dt;
    R e[2], ed[2], a[2];
    field<R>(P, t, e);
    field_dot<R>(P, t, ed);
    potential<R>(P, t, a);
    for (int l = 0; l < 2; ++l) {
      if (E) E[2 * k + l] = double(P.scale * e[l]);
      if (Ed) Ed[2 * k + l] = double(P.scale * ed[l]);
      if (A) A[2 * k + l] = double(P.scale * a[l]);
    }
  }
}

// Fourth-order Magnus evolution (see evolve4_mode) of modes p[nm][3]; Ag[nt][2][2] holds A at the
// two Gauss-Legendre nodes of every step, Aedge[2][2] A(t_i) and A(t_f).
void orc_evolve4_points_ld(int nt, double dt, const double* Ag, const double* Aedge, long nm, const double* p,
                           double* f, int nthreads) {
  using R = long double;
  const int nth = nthreads_or_default(nthreads);
#pragma omp parallel for schedule(dynamic, 1) num_threads(nth)
  for (long m = 0; m < nm; ++m) f[m] = double(evolve4_mode<R>(nt, R(dt), Ag, Aedge, Aedge + 2, p + 3 * m));
}

// Split-operator evolution (see evolve_split_mode) of modes p[nm][3]: order 2 (Strang, At[nt][2]
// at the step midpoints) or 4 (triple jump, At[nt][3][2]); Aedge[2][2] A(t_i) and A(t_f).
void orc_evolve_split_points_ld(int order, int nt, double dt, const double* At, const double* Aedge, long nm,
                                const double* p, double* f, int nthreads) {
  using R = long double;
  const int nsub = order == 4 ? 3 : 1;
  const int nth = nthreads_or_default(nthreads);
#pragma omp parallel for schedule(dynamic, 1) num_threads(nth)
  for (long m = 0; m < nm; ++m)
    f[m] = double(evolve_split_mode<R>(nt, R(dt), nsub, At, Aedge, Aedge + 2, p + 3 * m));
}

// ---------------------------------------------------------------------------------------
// Gradients by central differences (the definition of the derivative, fourth-order stencil
// (8 [F(h) - F(-h)] - [F(2h) - F(-2h)]) / (12 h)), for the local search of Sec. IV A.
// J is accumulated in long double from long-double f, without rounding f to double.  The steps
// are powers of two, so x +- h and x +- 2h are exact in double for |x| < 2^33 h.
// ---------------------------------------------------------------------------------------
long double yield_table_ld(int nt, long double dt, const double* Amid, const double* Aedge, const int n[3],
                           const double lo[3], const double hi[3], int nthreads) {
  const long nm = (long)n[0] * n[1] * n[2];
  std::vector<long double> f((size_t)nm);
  const int nth = nthreads_or_default(nthreads);
#pragma omp parallel for schedule(dynamic, 1) num_threads(nth)
  for (long m = 0; m < nm; ++m) {
    double p[3];
    grid_point(n, lo, hi, m, p);
    f[m] = evolve_mode<long double>(nt, dt, Amid, Aedge, Aedge + 2, p, nullptr);
  }
  long double s = 0;
  for (long m = 0; m < nm; ++m) s += f[m];
  return s * (long double)cell_volume(n, lo, hi);
}

// dJ/dx for table entries: e < 2 nt is A_mid[e/2][e%2], e = 2 nt + r is A_edge[r/2][r%2].
void orc_grad_table_fd_ld(int nt, double dt, const double* Amid, const double* Aedge, const int* n, const double* lo,
                          const double* hi, double h, int nidx, const long* idx, double* out, int nthreads) {
  std::vector<double> A(Amid, Amid + 2 * (size_t)nt), E(Aedge, Aedge + 4);
  for (int q = 0; q < nidx; ++q) {
    const long e = idx[q];
    double* x = e < 2L * nt ? &A[e] : &E[e - 2L * nt];
    const double x0 = *x;
    long double F[4];
    const double st[4] = {h, -h, 2 * h, -2 * h};
    for (int k = 0; k < 4; ++k) {
      *x = x0 + st[k];
      F[k] = yield_table_ld(nt, (long double)dt, A.data(), E.data(), n, lo, hi, nthreads);
    }
    *x = x0;
    out[q] = double((8 * (F[0] - F[1]) - (F[2] - F[3])) / (12 * (long double)h));
  }
}

// J and U = int |E|^2 dt (midpoint rule) of a synthesised pulse and their derivatives with
// respect to every coefficient; tables from the long-double synthesis (rounded to double).
void orc_grad_coeff_fd_ld(int ns, int order, double wmin, double wmax, double T, int nt, int norm, double norm_value,
                          const double* coeff, const int* n, const double* lo, const double* hi, double h, double* gJ,
                          double* gU, double* J0, double* U0, int nthreads) {
  const int nc = 4 * ns;
  std::vector<double> c(coeff, coeff + nc), Amid(2 * (size_t)nt), Emid(2 * (size_t)nt), Aedge(4);
  auto eval = [&](long double* J, long double* U) {
    double scale;
    synth_impl<long double>(ns, order, wmin, wmax, T, nt, norm, norm_value, c.data(), Amid.data(), Emid.data(),
                            Aedge.data(), &scale);
    // energy of the field: recompute E in long double at the midpoints (the double table only
    // stores it rounded)
    auto P = make_pulse<long double>(ns, order, wmin, wmax, T, nt, norm, norm_value, c.data());
    set_scale<long double>(P);
    const long double dt = P.T / (long double)nt, ti = -P.T / 2;
    long double u = 0;
    for (int k = 0; k < nt; ++k) {
      long double e[2];
      field<long double>(P, ti + ((long double)k + 0.5L) * dt, e);
      u += P.scale * P.scale * (e[0] * e[0] + e[1] * e[1]);
    }
    *U = u * dt;
    *J = yield_table_ld(nt, (long double)T / nt, Amid.data(), Aedge.data(), n, lo, hi, nthreads);
  };
  long double J, U;
  eval(&J, &U);
  if (J0) *J0 = double(J);
  if (U0) *U0 = double(U);
  for (int i = 0; i < nc; ++i) {
    const double x0 = c[i];
    long double Fj[4], Fu[4];
    const double st[4] = {h, -h, 2 * h, -2 * h};
    for (int k = 0; k < 4; ++k) {
      c[i] = x0 + st[k];
      eval(&Fj[k], &Fu[k]);
    }
    c[i] = x0;
    if (gJ) gJ[i] = double((8 * (Fj[0] - Fj[1]) - (Fj[2] - Fj[3])) / (12 * (long double)h));
    if (gU) gU[i] = double((8 * (Fu[0] - Fu[1]) - (Fu[2] - Fu[3])) / (12 * (long double)h));
  }
}

// Philox4x32-10 block.
void orc_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out) { philox(ctr, key, out); }

// DE/rand/1/bin proposal (Sec. IV B), one trial per individual.
//   pop[N][D] -> trial[N][D]; idx[N][4] receives (a, b, c, R) when non-null.
// Random words: key = seed; counter = (i, block, generation lo, generation hi).  Block 0 gives
// (a, b, c, R); blocks 1.. the crossover uniforms (gene j -> block 1 + j/4, word j%4); the next
// ceil(D/4) blocks the redraw uniforms for genes that leave [lo, hi].
// Genes in odd blocks of n_s (the phase coefficients) wrap periodically into [lo, hi]; the
// others are redrawn uniformly in [lo, hi].  n_s = 0 makes every gene an amplitude gene.
// Mutation is u = a + F (b - c), each operation rounded separately: the file is compiled with
// floating-point contraction off, so no multiply-add is fused.
void orc_de_propose(int N, int D, int n_s, double F, double CR, double lo, double hi, uint64_t seed,
                    int64_t gen, const double* pop, double* trial, int32_t* idx) {
  const int nb = (D + 3) / 4;
  for (int i = 0; i < N; ++i) {
    const uint32_t w0 = de_word(seed, gen, i, 0, 0), w1 = de_word(seed, gen, i, 0, 1);
    const uint32_t w2 = de_word(seed, gen, i, 0, 2), w3 = de_word(seed, gen, i, 0, 3);
    // a, b, c: uniform over the individuals not yet excluded, ascending skip of exclusions.
    std::vector<int> excl = {i};
    int pick[3];
    const uint32_t words[3] = {w0, w1, w2};
    for (int r = 0; r < 3; ++r) {
      int x = (int)uniform_index(words[r], (uint32_t)(N - 1 - r));
      std::vector<int> e = excl;
      std::sort(e.begin(), e.end());
      for (int ex : e) if (x >= ex) ++x;
      pick[r] = x;
      excl.push_back(x);
    }
    const int Rj = (int)uniform_index(w3, (uint32_t)D);
    if (idx) { idx[4 * i] = pick[0]; idx[4 * i + 1] = pick[1]; idx[4 * i + 2] = pick[2]; idx[4 * i + 3] = Rj; }
    const double* a = pop + (size_t)pick[0] * D;
    const double* b = pop + (size_t)pick[1] * D;
    const double* c = pop + (size_t)pick[2] * D;
    const double* x = pop + (size_t)i * D;
    for (int j = 0; j < D; ++j) {
      const double r = uniform_open01(de_word(seed, gen, i, 1 + j / 4, j % 4));
      double y;
      if (r <= CR || j == Rj) {
        const double diff = b[j] - c[j];
        const double step = F * diff;
        y = a[j] + step;
      } else {
        y = x[j];
      }
      const bool phase = (n_s > 0) && ((j / n_s) % 2 == 1);
      if (y < lo || y > hi) {
        if (phase) {
          const double w = hi - lo;
          const double k = std::floor((y - lo) / w);
          y = y - w * k;
        } else {
          const double r2 = uniform_open01(de_word(seed, gen, i, 1 + nb + j / 4, j % 4));
          y = lo + (hi - lo) * r2;
        }
      }
      trial[(size_t)i * D + j] = y;
    }
  }
}

// Selection (maximisation): individual i takes the trial iff mask[i] != 0 (or mask is null)
// and trial_fit[i] >= fit[i].
void orc_de_select(int N, int D, double* pop, double* fit, const double* trial, const double* trial_fit,
                   const uint8_t* mask) {
  for (int i = 0; i < N; ++i) {
    if (mask && !mask[i]) continue;
    if (trial_fit[i] >= fit[i]) {
      for (int j = 0; j < D; ++j) pop[(size_t)i * D + j] = trial[(size_t)i * D + j];
      fit[i] = trial_fit[i];
    }
  }
}

// Self-adaptive DE, jDE (Brest, Greiner, Boskovic, Mernik & Zumer, IEEE Trans. Evol. Comput. 10
// (2006) 646; the self-adaptive variant named in Sec. IV B), on a population split into equal
// islands (the island model of Sec. IV B).  Every individual carries its own (F, CR) in
// fcr[N][2].  For individual i of island k (islands of S = N / islands consecutive members):
//   * a, b, c: distinct members of island k other than i, drawn as in orc_de_propose but over
//     the S - 1 other members (local indices, ascending skip of the exclusions);
//   * with probability tau1, F' = Flo + u (Fhi - Flo), else F' = F_i; with probability tau2,
//     CR' = u, else CR' = CR_i;
//   * the trial is DE/rand/1/bin with F', CR' and the bound handling of orc_de_propose.
// Random words as orc_de_propose; the extra block 1 + 2 ceil(D/4) gives (u_F?, u_F, u_CR?, u_CR).
void orc_jde_propose(int N, int D, int n_s, int islands, double tau1, double tau2, double Flo, double Fhi,
                     double lo, double hi, uint64_t seed, int64_t gen, const double* pop, const double* fcr,
                     double* trial, double* tfcr, int32_t* idx) {
  const int nb = (D + 3) / 4;
  const int S = N / islands;
  for (int i = 0; i < N; ++i) {
    const int base = (i / S) * S, li = i - base;
    const uint32_t w[4] = {de_word(seed, gen, i, 0, 0), de_word(seed, gen, i, 0, 1), de_word(seed, gen, i, 0, 2),
                           de_word(seed, gen, i, 0, 3)};
    std::vector<int> excl = {li};
    int pick[3];
    for (int r = 0; r < 3; ++r) {
      int x = (int)uniform_index(w[r], (uint32_t)(S - 1 - r));
      std::vector<int> e = excl;
      std::sort(e.begin(), e.end());
      for (int ex : e) if (x >= ex) ++x;
      excl.push_back(x);
      pick[r] = base + x;
    }
    const int Rj = (int)uniform_index(w[3], (uint32_t)D);
    if (idx) { idx[4 * i] = pick[0]; idx[4 * i + 1] = pick[1]; idx[4 * i + 2] = pick[2]; idx[4 * i + 3] = Rj; }
    const int pb = 1 + 2 * nb;
    double F = fcr[2 * i], CR = fcr[2 * i + 1];
    if (uniform_open01(de_word(seed, gen, i, pb, 0)) < tau1) {
      const double span = Fhi - Flo;
      const double step = uniform_open01(de_word(seed, gen, i, pb, 1)) * span;
      F = Flo + step;
    }
    if (uniform_open01(de_word(seed, gen, i, pb, 2)) < tau2) CR = uniform_open01(de_word(seed, gen, i, pb, 3));
    tfcr[2 * i] = F;
    tfcr[2 * i + 1] = CR;
    const double* a = pop + (size_t)pick[0] * D;
    const double* b = pop + (size_t)pick[1] * D;
    const double* c = pop + (size_t)pick[2] * D;
    const double* x = pop + (size_t)i * D;
    for (int j = 0; j < D; ++j) {
      const double r = uniform_open01(de_word(seed, gen, i, 1 + j / 4, j % 4));
      double y;
      if (r <= CR || j == Rj) {
        const double diff = b[j] - c[j];
        const double step = F * diff;
        y = a[j] + step;
      } else {
        y = x[j];
      }
      const bool phase = (n_s > 0) && ((j / n_s) % 2 == 1);
      if (y < lo || y > hi) {
        if (phase) {
          const double wd = hi - lo;
          const double k = std::floor((y - lo) / wd);
          y = y - wd * k;
        } else {
          const double r2 = uniform_open01(de_word(seed, gen, i, 1 + nb + j / 4, j % 4));
          y = lo + (hi - lo) * r2;
        }
      }
      trial[(size_t)i * D + j] = y;
    }
  }
}

// jDE selection (maximisation): individual i takes the trial and its (F, CR) iff mask[i] != 0
// (or mask is null) and trial_fit[i] >= fit[i].
void orc_jde_select(int N, int D, double* pop, double* fit, double* fcr, const double* trial, const double* trial_fit,
                    const double* tfcr, const uint8_t* mask) {
  for (int i = 0; i < N; ++i) {
    if (mask && !mask[i]) continue;
    if (trial_fit[i] >= fit[i]) {
      for (int j = 0; j < D; ++j) pop[(size_t)i * D + j] = trial[(size_t)i * D + j];
      fit[i] = trial_fit[i];
      fcr[2 * i] = tfcr[2 * i];
      fcr[2 * i + 1] = tfcr[2 * i + 1];
    }
  }
}

// Ring migration between islands (Sec. IV B): from the state before the call, the best member
// of island k (largest fit, lowest index on ties) replaces the worst member of island
// (k + 1) mod islands (smallest fit, lowest index on ties) when it is strictly better; genes, fit
// and (F, CR) move together.  All islands migrate at once.
void orc_island_migrate(int N, int D, int islands, double* pop, double* fit, double* fcr) {
  const int S = N / islands;
  std::vector<double> p0(pop, pop + (size_t)N * D), f0(fit, fit + N), c0(fcr, fcr + 2 * (size_t)N);
  for (int k = 0; k < islands; ++k) {
    int best = k * S;
    for (int i = k * S; i < (k + 1) * S; ++i) if (f0[i] > f0[best]) best = i;
    const int k2 = (k + 1) % islands;
    int worst = k2 * S;
    for (int i = k2 * S; i < (k2 + 1) * S; ++i) if (f0[i] < f0[worst]) worst = i;
    if (f0[best] > f0[worst]) {
      for (int j = 0; j < D; ++j) pop[(size_t)worst * D + j] = p0[(size_t)best * D + j];
      fit[worst] = f0[best];
      fcr[2 * worst] = c0[2 * best];
      fcr[2 * worst + 1] = c0[2 * best + 1];
    }
  }
}

}  // extern "C"
