// Quantum kinetic equation per momentum mode (gfx950, FP64): the second formulation of the pair
// density in Sec. II B of arXiv:1704.08919, integrated with classical fourth-order Runge-Kutta.
//
// For a field E(t) in the x-y plane the six-component vector chi obeys chi' = N(t, P) chi with
// the skew-symmetric N of Eq. matrix, chi(t_i) = (1, 0, 0, 0, 0, 0) and f = 1 - chi_1 at t_f.
// With P = p - A(t), omega^2 = 1 + P^2 + p_z^2 and e_perp^2 = 1 + p_z^2, the entries are
//     Q = sqrt(X) / omega^2,  R = e_perp omega (E x dE/dt)_z / X,  X = omega^2 |E|^2 - (E.P)^2
// (X = 0 only where E = 0, and R := 0 there); a field along x alone uses the signed
// Q = E_x sqrt(1 + P_y^2 + p_z^2) / omega^2 and R = 0, which keeps the basis continuous where E
// changes sign.
//
// The kernel integrates y = (f, chi_2, ..., chi_6) instead of chi: RK4 commutes with this affine
// change of variables, so the discrete solution is the same, but f is then carried with a
// relative rounding error instead of the absolute error of 1 - chi_1 (|chi| = 1 is conserved, so
// chi_2..chi_6 are O(sqrt f)).  In units of dt / 2, with q = Q dt/2, W = omega dt, r = R dt/2:
//     K(y) = (q y_2,  q (1 - f) - W y_3 + r y_4,  W y_2 - r y_5,  -r y_2 + W y_5,
//             r y_3 - W y_4 + q y_6,  -q y_5),
// and a step is K1 = K(y; t_n), K2 = K(y + K1; t_n + dt/2), K3 = K(y + K2; t_n + dt/2),
// K4 = K(y + 2 K3; t_n + dt), y += (K1 + 2 K2 + 2 K3 + K4) / 3.
//
// Tables: E, dE/dt and A at the 2 nt + 1 half-step points t_i + h dt/2 of each pulse.  A
// workgroup of 256 lanes owns 256 consecutive modes (one per lane); per chunk of 128 steps each
// lane stages one point -- (A_x, A_y), (E_x, E_y), (|E|^2, (E x dE/dt)_z) -- into LDS
// (double-buffered) and every lane reads the same record (broadcast).  The coefficients at
// t_n + dt are carried to the next step, so each step evaluates them at two new points.
#include "reduce.hpp"

#pragma clang fp contract(off)

namespace po {
namespace {

constexpr int kQChunk = 128;               // steps per LDS chunk
constexpr int kQPoints = 2 * kQChunk;      // half-step points per chunk (= threads)

struct QkeArgs {
  const PulseDev* desc;
  int n_pulses;
  const double* E;
  const double* Ed;
  const double* A;
  double* f;
  double* units;
};

struct Coef {
  double q, W, r;
};

struct Point {
  double2 a, e, s;  // (A_x, A_y), (E_x, E_y), (|E|^2, (E x dE/dt)_z)
};

template <bool LINEAR>
__device__ __forceinline__ Coef coef_at(const Point& pt, double px, double py, double e2, double ep, double dt,
                                        double hdt) {
  const double Px = px - pt.a.x, Py = py - pt.a.y;
  const double t2 = fma(Py, Py, e2);  // 1 + P_y^2 + p_z^2
  const double w2 = fma(Px, Px, t2);
  const double rw = rsqrt(w2);
  const double w = w2 * rw;
  Coef c;
  c.W = w * dt;
  if constexpr (LINEAR) {
    c.q = (pt.e.x * sqrt(t2)) * (rw * rw) * hdt;
    c.r = 0.0;
  } else {
    const double EP = fma(pt.e.x, Px, pt.e.y * Py);
    const double X = fma(w2, pt.s.x, -(EP * EP));
    if (X > 0.0) {
      const double rX = rsqrt(X);
      c.q = (X * rX) * (rw * rw) * hdt;
      c.r = ((ep * w) * pt.s.y) * (rX * rX) * hdt;
    } else {
      c.q = 0.0;
      c.r = 0.0;
    }
  }
  return c;
}

struct Y6 {
  double f, c2, c3, c4, c5, c6;
};

template <bool LINEAR>
__device__ __forceinline__ Y6 rhs(const Y6& y, const Coef& k) {
  Y6 o;
  o.f = k.q * y.c2;
  if constexpr (LINEAR) {
    o.c2 = fma(-k.W, y.c3, fma(-k.q, y.f, k.q));
    o.c3 = k.W * y.c2;
    o.c4 = o.c5 = o.c6 = 0.0;
  } else {
    o.c2 = fma(k.r, y.c4, fma(-k.W, y.c3, fma(-k.q, y.f, k.q)));
    o.c3 = fma(-k.r, y.c5, k.W * y.c2);
    o.c4 = fma(k.W, y.c5, -(k.r * y.c2));
    o.c5 = fma(k.q, y.c6, fma(-k.W, y.c4, k.r * y.c3));
    o.c6 = -(k.q * y.c5);
  }
  return o;
}

__device__ __forceinline__ Y6 axpy(const Y6& y, double s, const Y6& k) {
  return Y6{fma(s, k.f, y.f), fma(s, k.c2, y.c2), fma(s, k.c3, y.c3),
            fma(s, k.c4, y.c4), fma(s, k.c5, y.c5), fma(s, k.c6, y.c6)};
}

__device__ __forceinline__ Y6 add(const Y6& y, const Y6& k) {
  return Y6{y.f + k.f, y.c2 + k.c2, y.c3 + k.c3, y.c4 + k.c4, y.c5 + k.c5, y.c6 + k.c6};
}

template <bool LINEAR>
__device__ __forceinline__ void rk4_step(Y6& y, const Coef& k0, const Coef& k1, const Coef& k2) {
  const Y6 K1 = rhs<LINEAR>(y, k0);
  const Y6 K2 = rhs<LINEAR>(add(y, K1), k1);
  const Y6 K3 = rhs<LINEAR>(add(y, K2), k1);
  const Y6 K4 = rhs<LINEAR>(axpy(y, 2.0, K3), k2);
  const Y6 s = add(axpy(axpy(K1, 2.0, K2), 2.0, K3), K4);
  y = axpy(y, 1.0 / 3.0, s);
}

__device__ __forceinline__ Point load_point(const double2* __restrict__ E, const double2* __restrict__ Ed,
                                            const double2* __restrict__ A, int64_t h) {
  const double2 a = A[h], e = E[h], ed = Ed[h];
  return Point{a, e, make_double2(fma(e.x, e.x, e.y * e.y), fma(e.x, ed.y, -(e.y * ed.x)))};
}

template <bool LINEAR>
__global__ void __launch_bounds__(kQPoints) k_qke(QkeArgs a) {
  __shared__ Point lds[2][kQPoints];
  const int item = xcd_item(blockIdx.x, gridDim.x);
  const int pi = find_pulse_item(a.desc, a.n_pulses, item);
  const PulseDev& d = a.desc[pi];
  const int nt = d.nt;
  const int64_t npts = 2 * int64_t(nt) + 1;
  const double dt = d.dt, hdt = 0.5 * d.dt;
  const int64_t nmodes = int64_t(d.n[0]) * d.n[1] * d.n[2];
  const double2* E = reinterpret_cast<const double2*>(a.E) + d.tab_off;
  const double2* Ed = reinterpret_cast<const double2*>(a.Ed) + d.tab_off;
  const double2* A = reinterpret_cast<const double2*>(a.A) + d.tab_off;

  const int64_t m = int64_t(item - d.item_off) * kItem + threadIdx.x;
  double px, py, pz;
  mode_momentum(d, m < nmodes ? m : 0, px, py, pz);
  const double e2 = fma(pz, pz, 1.0), ep = sqrt(e2);

  // chunk c holds the points h = 2 c kQChunk + 1 + i, i < kQPoints
  const int nchunks = (nt + kQChunk - 1) / kQChunk;
  {
    const int64_t h = 1 + threadIdx.x;
    lds[0][threadIdx.x] = h < npts ? load_point(E, Ed, A, h) : Point{};
  }
  Coef k0 = coef_at<LINEAR>(load_point(E, Ed, A, 0), px, py, e2, ep, dt, hdt);
  __syncthreads();
  Y6 y{0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int c = 0; c < nchunks; ++c) {
    const int64_t h = int64_t(c + 1) * kQPoints + 1 + threadIdx.x;
    const Point pre = (c + 1 < nchunks && h < npts) ? load_point(E, Ed, A, h) : Point{};
    const Point* buf = lds[c & 1];
    const int len = min(kQChunk, nt - c * kQChunk);
    for (int k = 0; k < len; ++k) {
      const Coef k1 = coef_at<LINEAR>(buf[2 * k], px, py, e2, ep, dt, hdt);
      const Coef k2 = coef_at<LINEAR>(buf[2 * k + 1], px, py, e2, ep, dt, hdt);
      rk4_step<LINEAR>(y, k0, k1, k2);
      k0 = k2;
    }
    lds[(c + 1) & 1][threadIdx.x] = pre;
    __syncthreads();
  }

  double fv = 0.0;
  if (m < nmodes) {
    fv = y.f;
    if (a.f) a.f[d.mode_off + m] = fv;
  }
  if (a.units) write_unit(d, a.units, m, nmodes, fv);
}

}  // namespace

po_status launch_qke_grid(const Batch& b, const PulseDev* d_desc, const double* d_E, const double* d_Ed,
                          const double* d_A, int linear, double* d_f, double* d_units, hipStream_t s) {
  static_assert(kQPoints == kItem, "one mode per lane and one staged point per lane");
  QkeArgs a{d_desc, b.n_pulses, d_E, d_Ed, d_A, d_f, d_units};
  if (linear) hipLaunchKernelGGL(k_qke<true>, dim3(b.total_items), dim3(kItem), 0, s, a);
  else hipLaunchKernelGGL(k_qke<false>, dim3(b.total_items), dim3(kItem), 0, s, a);
  PO_HIP(hipGetLastError());
  return PO_OK;
}

}  // namespace po
