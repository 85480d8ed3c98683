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
// One workgroup of 256 lanes per 256-mode item, one mode per lane.  Forward: the exact C, S form
// (degree-7 series with the pulse's angle halvings), states unit-normalised at t_f.  Backward:
// the table is staged through LDS chunk by chunk in reverse; each step applies U^+ to psi and chi
// and forms the two derivative terms; their sum over the item's modes is taken per step, a fixed
// butterfly per wave and then the four waves in order, and written as item partials
// [item][n][2]; a second kernel sums the items of each pulse in order.  So the gradient, like J,
// does not depend on scheduling.
#include "dirac.hpp"
#include "reduce.hpp"

#pragma clang fp contract(off)

namespace po {
namespace {

// Maclaurin coefficients of D(x) = (cos sqrt x - sin sqrt x / sqrt x) / x
//   = sum_k (-1)^(k+1) 2 (k+1) x^k / (2k+3)!   (-1/3 + x/30 - x^2/840 + ...).
constexpr double dser_coef(int k) { return (k % 2 ? 1.0 : -1.0) * 2.0 * double(k + 1) / factorial(2 * k + 3); }

template <int K>
__device__ __forceinline__ void horner_d(double x, double& D) {
  constexpr double c = dser_coef(K);
  D = fma(D, x, c);
  if constexpr (K > 0) horner_d<K - 1>(x, D);
}

// C, S and D at x = |q|^2: degree-7 series (x / 4^h <= 0.3612 keeps every remainder below
// 2^-56), h double-angle steps for C and S; D = (C - S)/x when halved (x > 0.36: no cancellation).
__device__ __forceinline__ void csd(double x, int h, double inv4h, double& C, double& S, double& D) {
  if (h == 0) {
    cos_sinc<7>(x, C, S);
    constexpr double d7 = dser_coef(7);
    D = d7;
    horner_d<6>(x, D);
  } else {
    cos_sinc_halved(x, h, inv4h, C, S);
    D = (C - S) / x;
  }
}

struct Blk {
  double ar, ai, br, bi;
};

// psi <- U^+ psi = (C + i S q.tau) psi for one block, q = (qx, qy, qz) the block's vector.
__device__ __forceinline__ void back_rotate(Blk& v, double C, double S, double qx, double qy, double qz) {
  rotate_block(v.ar, v.ai, v.br, v.bi, C, -(S * qx), -(S * qy), -(S * qz));
}

// 2 Re[conj(alpha) <chi| dU/dq_j |psi>] for j = x, y of one block.
__device__ __forceinline__ void block_terms(const Blk& c, const Blk& p, double ar_, double ai_, double C, double S,
                                            double D, double qx, double qy, double qz, double& gx, double& gy) {
  (void)C;
  // conj(c1) p1, conj(c2) p2, conj(c1) p2, conj(c2) p1
  const double u11r = fma(c.ar, p.ar, c.ai * p.ai), u11i = fma(c.ar, p.ai, -(c.ai * p.ar));
  const double u22r = fma(c.br, p.br, c.bi * p.bi), u22i = fma(c.br, p.bi, -(c.bi * p.br));
  const double u12r = fma(c.ar, p.br, c.ai * p.bi), u12i = fma(c.ar, p.bi, -(c.ai * p.br));
  const double u21r = fma(c.br, p.ar, c.bi * p.ai), u21i = fma(c.br, p.ai, -(c.bi * p.ar));
  const double a_r = u11r + u22r, a_i = u11i + u22i;              // <chi|psi>
  const double tz_r = u11r - u22r, tz_i = u11i - u22i;            // <chi|tau_z|psi>
  const double tx_r = u12r + u21r, tx_i = u12i + u21i;            // <chi|tau_x|psi>
  const double ty_r = -(u21i - u12i), ty_i = u21r - u12r;         // i (conj(c2) p1 - conj(c1) p2)
  const double b_r = fma(qx, tx_r, fma(qy, ty_r, qz * tz_r));     // <chi|q.tau|psi>
  const double b_i = fma(qx, tx_i, fma(qy, ty_i, qz * tz_i));
  const double w_r = fma(-S, a_r, D * b_i), w_i = fma(-S, a_i, -(D * b_r));  // -S a - i D b
  const double dx_r = fma(qx, w_r, S * tx_i), dx_i = fma(qx, w_i, -(S * tx_r));
  const double dy_r = fma(qy, w_r, S * ty_i), dy_i = fma(qy, w_i, -(S * ty_r));
  gx = 2.0 * fma(ar_, dx_r, ai_ * dx_i);
  gy = 2.0 * fma(ar_, dy_r, ai_ * dy_i);
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

struct GradArgs {
  const PulseDev* desc;
  int n_pulses;
  const double* A;
  const double* Aedge;
  const int2* sel;
  const int64_t* goff;  // per pulse: first double of its item partials
  double* part;         // [items of pulse][nt][2] per pulse
  double* epart;        // [total items][4]: dA(t_i) x, y, dA(t_f) x, y
  double* units;        // 64-mode sums of f
};

constexpr int kWaves = kItem / 64;

__global__ void __launch_bounds__(kItem) __attribute__((amdgpu_waves_per_eu(3))) k_yield_grad(GradArgs a) {
  __shared__ double2 tab[kChunk];
  __shared__ double2 red[kWaves][kChunk];
  const int item = xcd_item(blockIdx.x, gridDim.x);
  const int pi = find_pulse_item(a.desc, a.n_pulses, item);
  const PulseDev& d = a.desc[pi];
  const int nt = d.nt;
  const double dt = d.dt;
  const int64_t nmodes = int64_t(d.n[0]) * d.n[1] * d.n[2];
  const int li = item - d.item_off;
  const int64_t m = int64_t(li) * kItem + threadIdx.x;
  const bool active = m < nmodes;
  const int h = a.sel[pi].y;
  const double inv4h = ldexp(1.0, -2 * h);
  const double2* A = reinterpret_cast<const double2*>(a.A) + d.tab_off;
  const double2 ain = reinterpret_cast<const double2*>(a.Aedge)[2 * pi];
  const double2 aout = reinterpret_cast<const double2*>(a.Aedge)[2 * pi + 1];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;

  double px, py, pz;
  mode_momentum(d, active ? m : 0, px, py, pz);
  const double e = sqrt(fma(pz, pz, 1.0));
  const double pxdt = px * dt, pydt = py * dt, qz = e * dt, qz2 = qz * qz;

  // forward: psi_s from |-_s(P_in)>
  Blk psi[2];
  {
    Blk up, dn;
    double w;
    eig_pm(px - ain.x, py - ain.y, e, 1.0, up, dn, w);
    psi[0] = dn;
    eig_pm(px - ain.x, py - ain.y, e, -1.0, up, dn, w);
    psi[1] = dn;
  }
  const int nchunks = (nt + kChunk - 1) / kChunk;
  for (int c = 0; c < nchunks; ++c) {
    const int n0 = c * kChunk, len = min(kChunk, nt - n0);
    __syncthreads();
    if (int(threadIdx.x) < len) {
      const double2 t = A[n0 + threadIdx.x];
      tab[threadIdx.x] = make_double2(-t.x * dt, -t.y * dt);
    }
    __syncthreads();
#pragma unroll 1
    for (int k = 0; k < len; ++k) {
      const double2 r = tab[k];
      const double qx = pxdt + r.x, qy = pydt + r.y;
      const double x = fma(qx, qx, fma(qy, qy, qz2));
      double C, S;
      if (h == 0) cos_sinc<7>(x, C, S);
      else cos_sinc_halved(x, h, inv4h, C, S);
      rotate_block(psi[0].ar, psi[0].ai, psi[0].br, psi[0].bi, C, S * qx, S * qy, S * qz);
      rotate_block(psi[1].ar, psi[1].ai, psi[1].br, psi[1].bi, C, S * qx, -(S * qy), S * qz);
    }
  }

  // t_f: normalise, alpha_s = <+_s(P_out)|psi_s>, final-state terms
  Blk chi[2];
  double al_r[2], al_i[2];
  double g_out_x = 0.0, g_out_y = 0.0, f = 0.0;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const double sg = s == 0 ? 1.0 : -1.0;
    Blk up_out, dn_out;
    double w_out;
    eig_pm(px - aout.x, py - aout.y, e, sg, up_out, dn_out, w_out);
    double nr, ni;
    inner(psi[s], psi[s], nr, ni);
    const double inv = 1.0 / sqrt(nr);
    psi[s] = Blk{psi[s].ar * inv, psi[s].ai * inv, psi[s].br * inv, psi[s].bi * inv};
    inner(up_out, psi[s], al_r[s], al_i[s]);
    if (!active) al_r[s] = al_i[s] = 0.0;
    f += fma(al_r[s], al_r[s], al_i[s] * al_i[s]);
    // d alpha = <+|dh|-><-|psi>/(2 w), dh = tau_x dP_x + s tau_y dP_y, dP = -dA(t_f)
    double xr, xi, yr, yi, mr, mi;
    tau_xy(up_out, dn_out, sg, xr, xi, yr, yi);
    inner(dn_out, psi[s], mr, mi);
    const double k = -1.0 / (2.0 * w_out);
    // Re[conj(alpha) (t m)]
    const double tmx_r = fma(xr, mr, -(xi * mi)), tmx_i = fma(xr, mi, xi * mr);
    const double tmy_r = fma(yr, mr, -(yi * mi)), tmy_i = fma(yr, mi, yi * mr);
    g_out_x += 2.0 * k * fma(al_r[s], tmx_r, al_i[s] * tmx_i);
    g_out_y += 2.0 * k * fma(al_r[s], tmy_r, al_i[s] * tmy_i);
    chi[s] = up_out;
  }

  // backward over the chunks in reverse
  double* part = a.part + a.goff[pi] + int64_t(li) * nt * 2;
  for (int c = nchunks - 1; c >= 0; --c) {
    const int n0 = c * kChunk, len = min(kChunk, nt - n0);
    __syncthreads();
    if (int(threadIdx.x) < len) {
      const double2 t = A[n0 + threadIdx.x];
      tab[threadIdx.x] = make_double2(-t.x * dt, -t.y * dt);
    }
    __syncthreads();
#pragma unroll 1
    for (int k = len - 1; k >= 0; --k) {
      const double2 r = tab[k];
      const double qx = pxdt + r.x, qy = pydt + r.y;
      const double x = fma(qx, qx, fma(qy, qy, qz2));
      double C, S, D;
      csd(x, h, inv4h, C, S, D);
      double gx = 0.0, gy = 0.0;
    #pragma unroll
  for (int s = 0; s < 2; ++s) {
        const double qys = s == 0 ? qy : -qy;
        back_rotate(psi[s], C, S, qx, qys, qz);  // psi_n
        double bx, by;
        block_terms(chi[s], psi[s], al_r[s], al_i[s], C, S, D, qx, qys, qz, bx, by);
        gx += bx;
        gy += s == 0 ? by : -by;  // dq_y/dA_y = -s dt
        back_rotate(chi[s], C, S, qx, qys, qz);  // chi_n
      }
      gx = wave_sum(-dt * gx);
      gy = wave_sum(-dt * gy);
      if (lane == 0) red[wave][k] = make_double2(gx, gy);
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

  // t_i: d|-> = -|+><+|dh|->/(2 w), dP = -dA(t_i); chi holds U^+ ... |+_out> = chi_0
  double g_in_x = 0.0, g_in_y = 0.0;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const double sg = s == 0 ? 1.0 : -1.0;
    Blk up_in, dn_in;
    double w_in;
    eig_pm(px - ain.x, py - ain.y, e, sg, up_in, dn_in, w_in);
    double xr, xi, yr, yi, cr, ci;
    tau_xy(up_in, dn_in, sg, xr, xi, yr, yi);
    inner(chi[s], up_in, cr, ci);
    const double k = 1.0 / (2.0 * w_in);  // (-1/(2w)) * (dP/dA = -1)
    const double tmx_r = fma(cr, xr, -(ci * xi)), tmx_i = fma(cr, xi, ci * xr);
    const double tmy_r = fma(cr, yr, -(ci * yi)), tmy_i = fma(cr, yi, ci * yr);
    g_in_x += 2.0 * k * fma(al_r[s], tmx_r, al_i[s] * tmx_i);
    g_in_y += 2.0 * k * fma(al_r[s], tmy_r, al_i[s] * tmy_i);
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

// dJ/dA[n] = dV sum over the pulse's items (in order) of the partials; one thread per (n, component).
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
    gA[2 * d.tab_off + e] = v * d.dv;
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
