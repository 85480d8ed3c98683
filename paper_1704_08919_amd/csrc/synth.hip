// Pulse synthesis on gfx950: B-spline spectra -> field statistics -> scale -> A/E tables.
//
// Sec. III of arXiv:1704.08919: the spectral density and phase of each component are B-spline
// expansions; the field is a Hann-windowed cosine sum over the lines Omega_j = (N_min + j) dw,
// dw = 2 pi / T; A(t) is its antiderivative with A(t_f) = 0.  The global renormalisation of
// Sec. IV B scales E and A by one factor per pulse (peak |E| or energy U).
//
// Time is indexed by half-steps h: t = -T/2 + h dt / 2 (h even: step nodes, h odd: midpoints).
// Every line frequency is an integer multiple k of dw, so the phase Omega_k t equals
// pi k (h - nt) / nt exactly; it is reduced modulo 2 in integers and evaluated with sincospi,
// which keeps all trig arguments in [0, 2) whatever T is.
#include "common.hpp"

namespace po {
namespace {

// Fixed-order tree sum of one value per thread over a 256-thread workgroup (every thread gets it).
__device__ __forceinline__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Knot w_i of the clamped knot vector (multiplicity k at both ends, equidistant interior knots).
__device__ __forceinline__ double knot(int i, int k, int ns, double wmin, double wmax) {
  if (i < k) return wmin;
  if (i >= ns) return wmax;
  const int nb = ns - k + 2;  // breakpoints
  return wmin + (wmax - wmin) * double(i - k + 1) / double(nb - 1);
}

// All basis values b_i^{(k)}(w), i < ns, by raising the order of the indicator functions
// (Cox-de Boor recursion, 0/0 := 0); the last non-empty span is closed at omega_max.
__device__ void bspline_all(int k, int ns, double wmin, double wmax, double w, double* b /*[ns+k]*/) {
  const int nk = ns + k;
  for (int i = 0; i < nk - 1; ++i) {
    const double a = knot(i, k, ns, wmin, wmax), c = knot(i + 1, k, ns, wmin, wmax);
    b[i] = (a <= w && w < c) ? 1.0 : 0.0;
    if (w == wmax && a < c && c == wmax) b[i] = 1.0;
  }
  for (int r = 2; r <= k; ++r) {
    for (int i = 0; i < nk - r; ++i) {
      const double ti = knot(i, k, ns, wmin, wmax), tir1 = knot(i + r - 1, k, ns, wmin, wmax);
      const double ti1 = knot(i + 1, k, ns, wmin, wmax), tir = knot(i + r, k, ns, wmin, wmax);
      double v = 0.0;
      if (tir1 != ti) v += (w - ti) / (tir1 - ti) * b[i];
      if (tir != ti1) v += (tir - w) / (tir - ti1) * b[i + 1];
      b[i] = v;
    }
  }
}

// One block per pulse; each thread fills lines j.  Output per line: (E cos Phi, E sin Phi) for x
// and y, i.e. spec[off + 4 j + {0,1,2,3}] = (cEx, sEx, cEy, sEy).
__global__ void __launch_bounds__(128) k_spectra(const PulseDev* __restrict__ desc,
                                                 const double* __restrict__ coeff, double* __restrict__ spec) {
  const PulseDev d = desc[blockIdx.x];
  const double* a = coeff + d.coeff_off;
  double b[2 * kMaxNs + 2];
  for (int j = threadIdx.x; j < d.nlines; j += blockDim.x) {
    // basis at the line frequency clamped into the band: the end lines sample the end knots
    // whatever the rounding of (N_min + j) dw
    const double w = fmin(fmax(double(d.nmin + j) * d.dw, d.wmin), d.wmax);
    bspline_all(d.order, d.ns, d.wmin, d.wmax, w, b);
    double out[4];
    for (int l = 0; l < 2; ++l) {
      double E = 0.0, ph = 0.0;
      for (int i = 0; i < d.ns; ++i) {
        E += a[(l * 2 + 0) * d.ns + i] * b[i];
        ph += M_PI * (a[(l * 2 + 1) * d.ns + i] + 1.0) * b[i];
      }
      double sp, cp;
      sincos(ph, &sp, &cp);
      out[2 * l] = E * cp;
      out[2 * l + 1] = E * sp;
    }
    double4* dst = reinterpret_cast<double4*>(spec + d.spec_off) + j;
    *dst = make_double4(out[0], out[1], out[2], out[3]);
  }
}

// sincos(pi k (h - nt) / nt) with the argument reduced exactly in integers.
__device__ __forceinline__ void line_phase(int64_t k, int64_t hm, int64_t two_nt, double inv_nt, double* s, double* c) {
  int64_t r = (k * hm) % two_nt;
  if (r < 0) r += two_nt;
  sincospi(double(r) * inv_nt, s, c);
}

// Unscaled field (want_E) and potential (want_A) at half-step index h.
__device__ void field_at(const PulseDev& d, const double4* __restrict__ sp, int64_t h, bool want_E, bool want_A,
                         double E[2], double A[2]) {
  const int64_t nt = d.nt, two_nt = 2 * int64_t(d.nt);
  const int64_t hm = h - nt;
  const double inv_nt = 1.0 / double(d.nt);
  double ex = 0.0, ey = 0.0, ax = 0.0, ay = 0.0;
  double sd = 0.0, cd = 1.0;  // Delta omega t
  if (want_A) line_phase(1, hm, two_nt, inv_nt, &sd, &cd);
  const double tmf = double(h - two_nt) * (0.5 * d.dt);  // t - t_f
  for (int j = 0; j < d.nlines; ++j) {
    const int64_t k = int64_t(d.nmin) + j;
    double s, c;
    line_phase(k, hm, two_nt, inv_nt, &s, &c);
    const double4 q = sp[j];  // (cEx, sEx, cEy, sEy)
    if (want_E) {
      ex += q.x * c + q.y * s;
      ey += q.z * c + q.w * s;
    }
    if (want_A) {
      // E_j [I(Om, -Phi)/2 + I(dw + Om, -Phi)/4 + I(dw - Om, +Phi)/4], I(w, phi; t) = int_{t_f}^t cos(w s + phi) ds
      //   = [sin(w t + phi) - (-1)^k' sin(phi)] / w with w t_f = k' pi; (t - t_f) cos(phi) when w = 0.
      const double sgn = (k & 1) ? -1.0 : 1.0;
      const double cp = c * cd - s * sd, spp = s * cd + c * sd;  // (Om + dw) t
      const double cm = cd * c + sd * s, smm = sd * c - cd * s;  // (dw - Om) t
      const double om = double(k) * d.dw, wp = double(k + 1) * d.dw, wm = double(1 - k) * d.dw;
      double tx, ty;
      // main line
      if (k == 0) {
        tx = 0.5 * tmf * q.x;
        ty = 0.5 * tmf * q.z;
      } else {
        tx = 0.5 * (q.x * s - q.y * c + sgn * q.y) / om;
        ty = 0.5 * (q.z * s - q.w * c + sgn * q.w) / om;
      }
      // upper side line dw + Om (never zero)
      tx += 0.25 * (q.x * spp - q.y * cp - sgn * q.y) / wp;
      ty += 0.25 * (q.z * spp - q.w * cp - sgn * q.w) / wp;
      // lower side line dw - Om
      if (k == 1) {
        tx += 0.25 * tmf * q.x;
        ty += 0.25 * tmf * q.z;
      } else {
        tx += 0.25 * (q.x * smm + q.y * cm + sgn * q.y) / wm;
        ty += 0.25 * (q.z * smm + q.w * cm + sgn * q.w) / wm;
      }
      ax -= tx;
      ay -= ty;
    }
  }
  if (want_E) {
    const double g = cospi(double(hm) * (0.5 * inv_nt));  // cos(pi t / T)
    E[0] = g * g * ex;
    E[1] = g * g * ey;
  }
  if (want_A) {
    A[0] = ax;
    A[1] = ay;
  }
}

// Line data of up to 256 lines of a pulse, staged in LDS by a workgroup: the spectral record and
// the factors 1/(2 Om), 1/(4 (dw + Om)), 1/(4 (dw - Om)) of the three terms of A (0 where the
// frequency vanishes and the term takes its t - t_f form instead).
struct LineTile {
  double4 q[256];
  double f0[256], f1[256], f2[256];
};

// field_at for every lane of a workgroup at its own half-step index h (all lanes must call it:
// the lines are staged tile by tile with barriers).  The phase index r = k (h - nt) mod 2 nt
// advances by h - nt from one line to the next, so only the first line needs a division; the
// phase itself is evaluated exactly (sincospi of the reduced index) on every 16th line and carried
// to the next 15 by rotating with the step angle pi (h - nt) / nt (a few ulps per line).
__device__ void field_tiled(const PulseDev& d, const double4* __restrict__ sp, int64_t h, bool want_E, bool want_A,
                            LineTile& L, double E[2], double A[2]) {
  const int64_t nt = d.nt, two_nt = 2 * int64_t(d.nt);
  const int64_t hm = h - nt;
  const double inv_nt = 1.0 / double(d.nt);
  double ex = 0.0, ey = 0.0, ax = 0.0, ay = 0.0;
  double sd = 0.0, cd = 1.0;  // Delta omega t
  if (want_A) line_phase(1, hm, two_nt, inv_nt, &sd, &cd);
  const double tmf = double(h - two_nt) * (0.5 * d.dt);  // t - t_f
  int64_t r = (int64_t(d.nmin) * hm) % two_nt;
  if (r < 0) r += two_nt;
  double sr, cr;  // rotation by one line: pi (h - nt) / nt
  sincospi(double(hm < 0 ? hm + two_nt : hm) * inv_nt, &sr, &cr);
  double s = 0.0, c = 1.0;
  for (int j0 = 0; j0 < d.nlines; j0 += 256) {
    const int cnt = min(256, d.nlines - j0);
    __syncthreads();
    if (int(threadIdx.x) < cnt) {
      const int64_t k = int64_t(d.nmin) + j0 + threadIdx.x;
      L.q[threadIdx.x] = sp[j0 + threadIdx.x];
      L.f0[threadIdx.x] = k == 0 ? 0.0 : 0.5 / (double(k) * d.dw);
      L.f1[threadIdx.x] = 0.25 / (double(k + 1) * d.dw);
      L.f2[threadIdx.x] = k == 1 ? 0.0 : 0.25 / (double(1 - k) * d.dw);
    }
    __syncthreads();
    for (int t = 0; t < cnt; ++t) {
      const int64_t k = int64_t(d.nmin) + j0 + t;
      if (((j0 + t) & 15) == 0) {
        sincospi(double(r) * inv_nt, &s, &c);
      } else {
        const double cn = fma(c, cr, -(s * sr));
        s = fma(s, cr, c * sr);
        c = cn;
      }
      r += hm;
      if (r >= two_nt) r -= two_nt;
      if (r < 0) r += two_nt;
      const double4 q = L.q[t];  // (cEx, sEx, cEy, sEy)
      if (want_E) {
        ex += q.x * c + q.y * s;
        ey += q.z * c + q.w * s;
      }
      if (want_A) {
        const double sgn = (k & 1) ? -1.0 : 1.0;
        const double cp = c * cd - s * sd, spp = s * cd + c * sd;  // (Om + dw) t
        const double cm = cd * c + sd * s, smm = sd * c - cd * s;  // (dw - Om) t
        double tx, ty;
        if (k == 0) {
          tx = 0.5 * tmf * q.x;
          ty = 0.5 * tmf * q.z;
        } else {
          tx = L.f0[t] * (q.x * s - q.y * c + sgn * q.y);
          ty = L.f0[t] * (q.z * s - q.w * c + sgn * q.w);
        }
        tx += L.f1[t] * (q.x * spp - q.y * cp - sgn * q.y);
        ty += L.f1[t] * (q.z * spp - q.w * cp - sgn * q.w);
        if (k == 1) {
          tx += 0.25 * tmf * q.x;
          ty += 0.25 * tmf * q.z;
        } else {
          tx += L.f2[t] * (q.x * smm + q.y * cm + sgn * q.y);
          ty += L.f2[t] * (q.z * smm + q.w * cm + sgn * q.w);
        }
        ax -= tx;
        ay -= ty;
      }
    }
  }
  if (want_E) {
    const double g = cospi(double(hm) * (0.5 * inv_nt));  // cos(pi t / T)
    E[0] = g * g * ex;
    E[1] = g * g * ey;
  }
  if (want_A) {
    A[0] = ax;
    A[1] = ay;
  }
}

// Per block: max |E| over step nodes (PEAK) or sum |E|^2 over midpoints (ENERGY) -> part[pulse][block].
__global__ void __launch_bounds__(256) k_field_stats(const PulseDev* __restrict__ desc,
                                                     const double* __restrict__ spec, int stride,
                                                     double* __restrict__ part) {
  const PulseDev d = desc[blockIdx.y];
  if (d.norm == PO_NORM_NONE || int(blockIdx.x) >= d.stat_blocks) return;
  const double4* sp = reinterpret_cast<const double4*>(spec + d.spec_off);
  __shared__ double red[256];
  __shared__ LineTile L;
  const int64_t n = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const bool peak = d.norm == PO_NORM_PEAK;
  // nodes 0..nt (PEAK) or midpoints 0..nt-1 (ENERGY); every lane takes part in the line staging
  const bool active = peak ? n <= d.nt : n < d.nt;
  double E[2], A[2];
  field_tiled(d, sp, active ? (peak ? 2 * n : 2 * n + 1) : 0, true, false, L, E, A);
  double v = 0.0;
  if (active) v = peak ? sqrt(E[0] * E[0] + E[1] * E[1]) : E[0] * E[0] + E[1] * E[1];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) {
      const double o = red[threadIdx.x + w];
      red[threadIdx.x] = (d.norm == PO_NORM_PEAK) ? fmax(red[threadIdx.x], o) : red[threadIdx.x] + o;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) part[size_t(blockIdx.y) * stride + blockIdx.x] = red[0];
}

// One block per pulse: fixed-order reduction of the partials -> scale.
__global__ void __launch_bounds__(256) k_scale(const PulseDev* __restrict__ desc, const double* __restrict__ part,
                                               int stride, double* __restrict__ scale_ws,
                                               double* __restrict__ scale_out) {
  const PulseDev d = desc[blockIdx.x];
  __shared__ double red[256];
  const bool peak = d.norm == PO_NORM_PEAK;
  double v = 0.0;
  for (int i = threadIdx.x; i < d.stat_blocks; i += 256) {
    const double x = part[size_t(blockIdx.x) * stride + i];
    v = peak ? fmax(v, x) : v + x;
  }
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] = peak ? fmax(red[threadIdx.x], red[threadIdx.x + w])
                                                      : red[threadIdx.x] + red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double s = 1.0;
    if (d.norm == PO_NORM_PEAK) s = red[0] > 0.0 ? d.norm_value / red[0] : 0.0;
    else if (d.norm == PO_NORM_ENERGY) {
      const double U = red[0] * d.dt;
      s = U > 0.0 ? sqrt(d.norm_value / U) : 0.0;
    }
    scale_ws[blockIdx.x] = s;
    if (scale_out) scale_out[blockIdx.x] = s;
  }
}

// Scaled A (and E) at every step midpoint; block (0, pulse) also writes A(t_i), A(t_f).
__global__ void __launch_bounds__(256) k_tables(const PulseDev* __restrict__ desc, const double* __restrict__ spec,
                                                const double* __restrict__ scale, double* __restrict__ Aout,
                                                double* __restrict__ Eout, double* __restrict__ Aedge) {
  const PulseDev d = desc[blockIdx.y];
  if (int64_t(blockIdx.x) * 256 >= d.nt) return;  // whole workgroup: beyond this pulse's steps
  const int64_t n = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const double4* sp = reinterpret_cast<const double4*>(spec + d.spec_off);
  const double s = scale[blockIdx.y];
  __shared__ LineTile L;
  {
    double E[2], A[2];
    field_tiled(d, sp, n < d.nt ? 2 * n + 1 : 1, Eout != nullptr, true, L, E, A);
    if (n < d.nt) {
      reinterpret_cast<double2*>(Aout)[d.tab_off + n] = make_double2(s * A[0], s * A[1]);
      if (Eout) reinterpret_cast<double2*>(Eout)[d.tab_off + n] = make_double2(s * E[0], s * E[1]);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x < 2) {
    double E[2], A[2];
    field_at(d, sp, threadIdx.x == 0 ? 0 : 2 * int64_t(d.nt), false, true, E, A);
    reinterpret_cast<double2*>(Aedge)[2 * blockIdx.y + threadIdx.x] = make_double2(s * A[0], s * A[1]);
  }
}

// Unscaled E, dE/dt and A at t = t_i + (n + c) dt for any offset c (0 <= n <= nt).  The phase of
// line k is pi [k (2n - nt) mod 2nt] / nt + 2 pi k c / nt: the step part is reduced exactly in
// integers, the offset part (below 2 pi k / nt) is added in floating point.
__device__ void field_sample(const PulseDev& d, const double4* __restrict__ sp, int64_t n, double c, bool want_E,
                             bool want_Ed, bool want_A, double E[2], double Ed[2], double A[2]) {
  const int64_t nt = d.nt, two_nt = 2 * nt, hm = 2 * n - nt;
  const double inv_nt = 1.0 / double(nt), cfrac = 2.0 * c * inv_nt;
  auto phase = [&](int64_t k, double* s, double* co) {
    int64_t r = (k * hm) % two_nt;
    if (r < 0) r += two_nt;
    double u = fma(double(k), cfrac, double(r) * inv_nt);
    if (u >= 2.0) u -= 2.0;
    sincospi(u, s, co);
  };
  double ex = 0.0, ey = 0.0, dx = 0.0, dy = 0.0, ax = 0.0, ay = 0.0;
  double sd = 0.0, cd = 1.0;
  if (want_A) phase(1, &sd, &cd);
  const double tmf = (double(n - nt) + c) * d.dt;  // t - t_f
  for (int j = 0; j < d.nlines; ++j) {
    const int64_t k = int64_t(d.nmin) + j;
    double s, co;
    phase(k, &s, &co);
    const double4 q = sp[j];  // (cEx, sEx, cEy, sEy)
    if (want_E || want_Ed) {
      ex += q.x * co + q.y * s;
      ey += q.z * co + q.w * s;
    }
    if (want_Ed) {
      const double om = double(k) * d.dw;
      dx += om * (q.y * co - q.x * s);
      dy += om * (q.w * co - q.z * s);
    }
    if (want_A) {
      // the line terms of field_at, at this phase
      const double sgn = (k & 1) ? -1.0 : 1.0;
      const double cp = co * cd - s * sd, spp = s * cd + co * sd;
      const double cm = cd * co + sd * s, smm = sd * co - cd * s;
      const double om = double(k) * d.dw, wp = double(k + 1) * d.dw, wm = double(1 - k) * d.dw;
      double tx, ty;
      if (k == 0) {
        tx = 0.5 * tmf * q.x;
        ty = 0.5 * tmf * q.z;
      } else {
        tx = 0.5 * (q.x * s - q.y * co + sgn * q.y) / om;
        ty = 0.5 * (q.z * s - q.w * co + sgn * q.w) / om;
      }
      tx += 0.25 * (q.x * spp - q.y * cp - sgn * q.y) / wp;
      ty += 0.25 * (q.z * spp - q.w * cp - sgn * q.w) / wp;
      if (k == 1) {
        tx += 0.25 * tmf * q.x;
        ty += 0.25 * tmf * q.z;
      } else {
        tx += 0.25 * (q.x * smm + q.y * cm + sgn * q.y) / wm;
        ty += 0.25 * (q.z * smm + q.w * cm + sgn * q.w) / wm;
      }
      ax -= tx;
      ay -= ty;
    }
  }
  const double arg = (double(hm) + 2.0 * c) * inv_nt;  // 2 t / T
  const double g = cospi(0.5 * arg);                   // cos(pi t / T)
  if (want_E) {
    E[0] = g * g * ex;
    E[1] = g * g * ey;
  }
  if (want_Ed) {
    const double g2d = -(M_PI / d.T) * sinpi(arg);  // d cos^2(pi t/T) / dt
    Ed[0] = g2d * ex + g * g * dx;
    Ed[1] = g2d * ey + g * g * dy;
  }
  if (want_A) {
    A[0] = ax;
    A[1] = ay;
  }
}

struct Offsets {
  double c[kMaxSub];
};

// Scaled samples: row r of pulse i is t_i + (r / n_sub + c_{r % n_sub}) dt; with_end adds t_f.
__global__ void __launch_bounds__(256) k_samples(const PulseDev* __restrict__ desc, const double* __restrict__ spec,
                                                 const double* __restrict__ scale, int n_sub, Offsets off,
                                                 int with_end, double* __restrict__ Eout, double* __restrict__ Edout,
                                                 double* __restrict__ Aout, double* __restrict__ Aedge) {
  const PulseDev d = desc[blockIdx.y];
  const int64_t rows = int64_t(d.nt) * n_sub + (with_end ? 1 : 0);
  const int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const double4* sp = reinterpret_cast<const double4*>(spec + d.spec_off);
  const double s = scale[blockIdx.y];
  if (k < rows) {
    const bool end = k == int64_t(d.nt) * n_sub;
    const int64_t n = end ? d.nt : k / n_sub;
    const double c = end ? 0.0 : off.c[k % n_sub];
    double E[2], Ed[2], A[2];
    field_sample(d, sp, n, c, Eout != nullptr, Edout != nullptr, Aout != nullptr, E, Ed, A);
    const int64_t row = d.tab_off + k;
    if (Eout) reinterpret_cast<double2*>(Eout)[row] = make_double2(s * E[0], s * E[1]);
    if (Edout) reinterpret_cast<double2*>(Edout)[row] = make_double2(s * Ed[0], s * Ed[1]);
    if (Aout) reinterpret_cast<double2*>(Aout)[row] = make_double2(s * A[0], s * A[1]);
  }
  if (Aedge && blockIdx.x == 0 && threadIdx.x < 2) {
    double E[2], A[2];
    field_at(d, sp, threadIdx.x == 0 ? 0 : 2 * int64_t(d.nt), false, true, E, A);
    reinterpret_cast<double2*>(Aedge)[2 * blockIdx.y + threadIdx.x] = make_double2(s * A[0], s * A[1]);
  }
}

// ------------------------------------------------------------------------------------------
// Adjoint of the synthesis (gradient of J and of the energy U with respect to the coefficients).
// A_l(t) and E_l(t) are linear in the line values cE = E_j cos Phi_j, sE = E_j sin Phi_j of every
// line: A_l(t) = -sum_j [cE_lj alpha_j(t) + sE_lj beta_j(t)] with alpha_j, beta_j the line terms
// of field_at, E_l(t) = g(t)^2 sum_j [cE_lj cos(Om_j t) + sE_lj sin(Om_j t)].  Per line the kernel
// forms G = sum_t gA(t) dA(t)/d(cE, sE) over the step midpoints and both ends, and
// dU/d(cE, sE) = 2 dt sum_n E_l(t_n) g^2 (cos, sin)(Om_j t_n) over the midpoints.
// ------------------------------------------------------------------------------------------

// Unscaled line terms (alpha, beta) of line k at half-step index hh (as in field_at).
__device__ __forceinline__ void line_terms(const PulseDev& d, int64_t k, int64_t hh, double& al, double& be,
                                           double& co, double& si) {
  const int64_t nt = d.nt, two_nt = 2 * nt, hm = hh - nt;
  const double inv_nt = 1.0 / double(nt);
  double s, c, sd, cd;
  line_phase(k, hm, two_nt, inv_nt, &s, &c);
  line_phase(1, hm, two_nt, inv_nt, &sd, &cd);
  co = c;
  si = s;
  const double tmf = double(hh - two_nt) * (0.5 * d.dt);
  const double sgn = (k & 1) ? -1.0 : 1.0;
  const double cp = c * cd - s * sd, spp = s * cd + c * sd;
  const double cm = cd * c + sd * s, smm = sd * c - cd * s;
  const double om = double(k) * d.dw, wp = double(k + 1) * d.dw, wm = double(1 - k) * d.dw;
  if (k == 0) {
    al = 0.5 * tmf;
    be = 0.0;
  } else {
    al = 0.5 * s / om;
    be = 0.5 * (sgn - c) / om;
  }
  al += 0.25 * spp / wp;
  be += 0.25 * (-cp - sgn) / wp;
  if (k == 1) {
    al += 0.25 * tmf;
  } else {
    al += 0.25 * smm / wm;
    be += 0.25 * (cm + sgn) / wm;
  }
}

// One workgroup per (line, pulse).  The eight line sums G = sum_t gA(t) dA(t)/d(cE, sE) per component
// and dU/d(cE, sE) (unscaled field) are formed with fixed-order block sums; then thread c < 4 n_s
// chains them through cE = E cos Phi, sE = E sin Phi and the B-spline expansions of E and
// Phi = pi (c + 1) for coefficient c, writing out[line][c] (dJ) and out[line][4 n_s + c] (dU),
// line slots of `stride` = 8 max n_s doubles.
__global__ void __launch_bounds__(256) k_adjoint_lines(const PulseDev* __restrict__ desc, const double* __restrict__ coeff,
                                                       const double* __restrict__ gA, const double* __restrict__ gedge,
                                                       const double* __restrict__ E, const double* __restrict__ scale,
                                                       int stride, double* __restrict__ out) {
  const PulseDev d = desc[blockIdx.y];
  const int j = blockIdx.x;
  if (j >= d.nlines) return;
  const int64_t k = int64_t(d.nmin) + j;
  const double inv_s = scale[blockIdx.y] != 0.0 ? 1.0 / scale[blockIdx.y] : 0.0;
  const double2* g = reinterpret_cast<const double2*>(gA) + d.tab_off;
  const double2* Et = reinterpret_cast<const double2*>(E) + d.tab_off;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t n = threadIdx.x; n < int64_t(d.nt) + 2; n += blockDim.x) {
    double2 gv;
    int64_t hh;
    const bool mid = n < d.nt;
    if (mid) {
      gv = g[n];
      hh = 2 * n + 1;
    } else {
      gv = gedge ? reinterpret_cast<const double2*>(gedge)[2 * blockIdx.y + (n - d.nt)] : make_double2(0.0, 0.0);
      hh = (n == d.nt) ? 0 : 2 * int64_t(d.nt);
    }
    double al, be, co, si;
    line_terms(d, k, hh, al, be, co, si);
    acc[0] -= gv.x * al;
    acc[1] -= gv.x * be;
    acc[2] -= gv.y * al;
    acc[3] -= gv.y * be;
    if (mid) {
      const double gg = cospi(double(hh - d.nt) * (0.5 / double(d.nt)));
      const double w = 2.0 * d.dt * gg * gg * inv_s;
      const double2 ev = Et[n];
      acc[4] += w * ev.x * co;
      acc[5] += w * ev.x * si;
      acc[6] += w * ev.y * co;
      acc[7] += w * ev.y * si;
    }
  }
  __shared__ double red[256];
  double L[8];
  for (int q = 0; q < 8; ++q) L[q] = block_sum(acc[q], red);
  const int t = threadIdx.x;
  if (t >= 4 * d.ns) return;
  const int l = t / (2 * d.ns), kind = (t / d.ns) % 2, i = t % d.ns;
  const double* a = coeff + d.coeff_off;
  double b[2 * kMaxNs + 2];
  const double w = fmin(fmax(double(k) * d.dw, d.wmin), d.wmax);
  bspline_all(d.order, d.ns, d.wmin, d.wmax, w, b);
  double Ev = 0.0, ph = 0.0;
  for (int q = 0; q < d.ns; ++q) {
    Ev += a[(l * 2 + 0) * d.ns + q] * b[q];
    ph += M_PI * (a[(l * 2 + 1) * d.ns + q] + 1.0) * b[q];
  }
  double sp, cp;
  sincos(ph, &sp, &cp);
  const double Gc = L[2 * l], Gs = L[2 * l + 1], Uc = L[4 + 2 * l], Us = L[4 + 2 * l + 1];
  double dJ, dU;
  if (kind == 0) {  // amplitude: d(cE, sE)/dE = (cos Phi, sin Phi)
    dJ = Gc * cp + Gs * sp;
    dU = Uc * cp + Us * sp;
  } else {          // phase: d(cE, sE)/dPhi = (-E sin Phi, E cos Phi), dPhi/dc = pi b_i
    dJ = M_PI * Ev * (Gs * cp - Gc * sp);
    dU = M_PI * Ev * (Us * cp - Uc * sp);
  }
  double* o = out + (d.spec_off / 4 + j) * stride;
  o[t] = dJ * b[i];
  o[4 * d.ns + t] = dU * b[i];
}

// One workgroup per pulse.  Fixed-order sums of g.A over the table and of |E|^2 (the energy),
// then thread c < 4 n_s sums its line contributions in line order.
__global__ void __launch_bounds__(256) k_adjoint_coeff(const PulseDev* __restrict__ desc, const double* __restrict__ lines,
                                                       const double* __restrict__ gA, const double* __restrict__ gedge,
                                                       const double* __restrict__ A, const double* __restrict__ Aedge,
                                                       const double* __restrict__ E, const double* __restrict__ scale,
                                                       int stride, double* __restrict__ grad, double* __restrict__ Uout,
                                                       double* __restrict__ gU) {
  const PulseDev d = desc[blockIdx.x];
  __shared__ double red[256];
  const double2* g = reinterpret_cast<const double2*>(gA) + d.tab_off;
  const double2* At = reinterpret_cast<const double2*>(A) + d.tab_off;
  const double2* Et = reinterpret_cast<const double2*>(E) + d.tab_off;
  double ga = 0.0, uu = 0.0;
  for (int64_t n = threadIdx.x; n < d.nt; n += blockDim.x) {
    const double2 gv = g[n], av = At[n], ev = Et[n];
    ga += gv.x * av.x + gv.y * av.y;
    uu += ev.x * ev.x + ev.y * ev.y;
  }
  if (gedge && threadIdx.x < 2) {
    const double2 gv = reinterpret_cast<const double2*>(gedge)[2 * blockIdx.x + threadIdx.x];
    const double2 av = reinterpret_cast<const double2*>(Aedge)[2 * blockIdx.x + threadIdx.x];
    ga += gv.x * av.x + gv.y * av.y;
  }
  const double gdotA = block_sum(ga, red);
  const double U = block_sum(uu, red) * d.dt;  // energy of the scaled field (midpoint rule)
  const double s = scale[blockIdx.x];
  const bool energy = d.norm == PO_NORM_ENERGY;
  const double Uraw = s != 0.0 ? U / (s * s) : 0.0;
  if (threadIdx.x == 0 && Uout) Uout[blockIdx.x] = U;
  const int t = threadIdx.x;
  if (t >= 4 * d.ns) return;
  const double* ln = lines + (d.spec_off / 4) * stride;
  double gj = 0.0, gu = 0.0;
  for (int j = 0; j < d.nlines; ++j) {
    gj += ln[int64_t(j) * stride + t];
    gu += ln[int64_t(j) * stride + 4 * d.ns + t];
  }
  // A = s A_raw: NORM_NONE has s = 1; NORM_ENERGY has s = sqrt(U0 / U_raw), so
  // dJ/dc = s dJ_raw/dc - (g.A) / (2 U_raw) dU_raw/dc and the energy stays U0.
  double outv = s * gj;
  if (energy && Uraw > 0.0) outv -= gdotA / (2.0 * Uraw) * gu;
  grad[d.coeff_off + t] = outv;
  if (gU) gU[d.coeff_off + t] = energy ? 0.0 : gu;
}

}  // namespace

po_status launch_synth(const Batch& b, const PulseDev* d_desc, const double* d_coeff, double* d_spec,
                       double* d_part, double* d_scale_ws, double* d_A, double* d_E, double* d_A_edge,
                       double* d_scale_out, hipStream_t s) {
  const int P = b.n_pulses;
  hipLaunchKernelGGL(k_spectra, dim3(P), dim3(128), 0, s, d_desc, d_coeff, d_spec);
  PO_HIP(hipGetLastError());
  if (b.max_stat_blocks > 0) {
    hipLaunchKernelGGL(k_field_stats, dim3(b.max_stat_blocks, P), dim3(256), 0, s, d_desc, d_spec,
                       b.max_stat_blocks, d_part);
    PO_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_scale, dim3(P), dim3(256), 0, s, d_desc, d_part, b.max_stat_blocks, d_scale_ws,
                     d_scale_out);
  PO_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_tables, dim3((b.max_nt + 255) / 256, P), dim3(256), 0, s, d_desc, d_spec, d_scale_ws,
                     d_A, d_E, d_A_edge);
  PO_HIP(hipGetLastError());
  return PO_OK;
}

po_status launch_synth_adjoint(const Batch& b, const PulseDev* d_desc, const double* d_coeff, const double* d_gA,
                               const double* d_gedge, const double* d_A, const double* d_A_edge, const double* d_E,
                               const double* d_scale, double* d_lines, double* d_grad, double* d_U, double* d_gU,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_adjoint_lines, dim3(b.max_lines, b.n_pulses), dim3(256), 0, s, d_desc, d_coeff, d_gA, d_gedge,
                     d_E, d_scale, 8 * b.max_ns, d_lines);
  PO_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_adjoint_coeff, dim3(b.n_pulses), dim3(256), 0, s, d_desc, d_lines, d_gA, d_gedge, d_A, d_A_edge,
                     d_E, d_scale, 8 * b.max_ns, d_grad, d_U, d_gU);
  PO_HIP(hipGetLastError());
  return PO_OK;
}

po_status launch_samples(const Batch& b, const PulseDev* d_desc, const double* d_coeff, double* d_spec, double* d_part,
                         double* d_scale_ws, int n_sub, const double* offsets, int with_end, double* d_E,
                         double* d_Ed, double* d_A, double* d_A_edge, double* d_scale_out, hipStream_t s) {
  const int P = b.n_pulses;
  Offsets off{};
  for (int r = 0; r < n_sub; ++r) off.c[r] = offsets[r];
  hipLaunchKernelGGL(k_spectra, dim3(P), dim3(128), 0, s, d_desc, d_coeff, d_spec);
  PO_HIP(hipGetLastError());
  if (b.max_stat_blocks > 0) {
    hipLaunchKernelGGL(k_field_stats, dim3(b.max_stat_blocks, P), dim3(256), 0, s, d_desc, d_spec,
                       b.max_stat_blocks, d_part);
    PO_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_scale, dim3(P), dim3(256), 0, s, d_desc, d_part, b.max_stat_blocks, d_scale_ws,
                     d_scale_out);
  PO_HIP(hipGetLastError());
  const int64_t rows = int64_t(b.max_nt) * n_sub + (with_end ? 1 : 0);
  hipLaunchKernelGGL(k_samples, dim3(unsigned((rows + 255) / 256), P), dim3(256), 0, s, d_desc, d_spec, d_scale_ws,
                     n_sub, off, with_end, d_E, d_Ed, d_A, d_A_edge);
  PO_HIP(hipGetLastError());
  return PO_OK;
}

}  // namespace po
