// Per-mode evolution of the momentum-space Dirac equation and projection (gfx950, FP64).
//
// Sec. II A of arXiv:1704.08919.  For a field in the x-y plane, p_z is conserved and the 4x4
// Hamiltonian alpha.(p - A) + beta m commutes with an operator K with K^2 = 1, so it splits into
// two 2x2 blocks
//     h_s(P) = P_x tau_x + s P_y tau_y + e_perp tau_z,   s = +1, -1,   e_perp = sqrt(1 + p_z^2),
// each holding one positive- and one negative-energy state of H.  The spin-summed density is
// the sum over the two blocks of |<+_s(P_out)| U_s |-_s(P_in)>|^2, which equals the trace over
// both spinors of the 4x4 form.
//
// One time step is the exact exponential of h frozen at the step midpoint (a second-order,
// unitary scheme): with q = (p - A_{n+1/2}) dt, q_z = e_perp dt and x = |q|^2 = (omega dt)^2,
//     U = C(x) 1 - i S(x) (q_x tau_x + s q_y tau_y + q_z tau_z),
//     C(x) = cos sqrt(x),  S(x) = sin sqrt(x) / sqrt(x),
// where C and S are evaluated as truncated Maclaurin series in x whose first omitted term is
// below 2^-56 on the launch's range of x (angle halving beyond it).  C and S are shared by both
// blocks, because omega does not depend on s.
//
// Work decomposition: a workgroup of 256 lanes (four 64-wide waves) owns one tile of 256
// consecutive modes of one pulse, one mode per lane.  The pulse's table of -A dt is staged
// through LDS in chunks of 256 steps (double-buffered, one barrier per chunk) and every lane
// reads the same record, an LDS broadcast.  The state (2 blocks x 2 complex amplitudes) stays
// in VGPRs for all nt steps.  Partial sums of f over each tile are formed in a fixed tree
// order, so J does not depend on scheduling.
#include "common.hpp"

namespace po {
namespace {

constexpr int kChunk = 256;   // steps staged per LDS buffer
constexpr int kThreads = 256; // lanes per workgroup = modes per tile

constexpr double factorial(int n) { return n <= 1 ? 1.0 : double(n) * factorial(n - 1); }
// Maclaurin coefficients of cos(sqrt x) and sin(sqrt x)/sqrt x.
constexpr double cos_coef(int k) { return (k % 2 ? -1.0 : 1.0) / factorial(2 * k); }
constexpr double sinc_coef(int k) { return (k % 2 ? -1.0 : 1.0) / factorial(2 * k + 1); }

// Largest x for which the first omitted term of the degree-D series, x^{D+1}/(2D+2)!, is below 2^-56.
constexpr double kXmax6 = 0.14;
constexpr double kXmax7 = 0.36;

// Horner step k of both series, with the coefficients forced to compile-time constants.
template <int K>
__device__ __forceinline__ void horner(double x, double& C, double& S) {
  constexpr double cc = cos_coef(K), sc = sinc_coef(K);
  C = fma(C, x, cc);
  S = fma(S, x, sc);
  if constexpr (K > 0) horner<K - 1>(x, C, S);
}

template <int D>
__device__ __forceinline__ void cos_sinc(double x, double& C, double& S) {
  constexpr double cd = cos_coef(D), sd = sinc_coef(D);
  C = cd;
  S = sd;
  horner<D - 1>(x, C, S);
}

// State layout: st[0..3] = (a_r, a_i, b_r, b_i) of block s = +1, st[4..7] the same for s = -1.
struct State {
  double ar, ai, br, bi, cr, ci, dr, di;
};

// Applies U_s for both blocks given C, S and q.
__device__ __forceinline__ void rotate(State& v, double C, double S, double qx, double qy, double qz) {
  const double sx = S * qx, sy = S * qy, sz = S * qz;
  // s = +1:  a' = (C - i sz) a + (-sy - i sx) b ;  b' = (sy - i sx) a + (C + i sz) b
  const double ar = C * v.ar + sz * v.ai - sy * v.br + sx * v.bi;
  const double ai = C * v.ai - sz * v.ar - sy * v.bi - sx * v.br;
  const double br = sy * v.ar + sx * v.ai + C * v.br - sz * v.bi;
  const double bi = sy * v.ai - sx * v.ar + C * v.bi + sz * v.br;
  // s = -1: same with sy -> -sy
  const double cr = C * v.cr + sz * v.ci + sy * v.dr + sx * v.di;
  const double ci = C * v.ci - sz * v.cr + sy * v.di - sx * v.dr;
  const double dr = -sy * v.cr + sx * v.ci + C * v.dr - sz * v.di;
  const double di = -sy * v.ci - sx * v.cr + C * v.di + sz * v.dr;
  v = State{ar, ai, br, bi, cr, ci, dr, di};
}

template <int D>
__device__ __forceinline__ void step(State& v, double2 rec, double pxdt, double pydt, double qz, double qz2) {
  const double qx = pxdt + rec.x;  // rec = -A dt
  const double qy = pydt + rec.y;
  const double x = fma(qx, qx, fma(qy, qy, qz2));
  double C, S;
  cos_sinc<D>(x, C, S);
  rotate(v, C, S, qx, qy, qz);
}

// Angle-halving variant for large steps: evaluate at x / 4^h, then double h times.
__device__ __forceinline__ void step_halving(State& v, double2 rec, double pxdt, double pydt, double qz, double qz2,
                                             int h, double inv4h) {
  const double qx = pxdt + rec.x;
  const double qy = pydt + rec.y;
  const double x = fma(qx, qx, fma(qy, qy, qz2));
  double xs = x * inv4h;
  double C, S;
  cos_sinc<7>(xs, C, S);
  for (int i = 0; i < h; ++i) {
    const double c2 = fma(C, C, -xs * S * S);  // cos 2t = cos^2 t - t^2 (sin t / t)^2
    S = S * C;                                 // sin 2t / 2t = (sin t / t) cos t
    C = c2;
    xs *= 4.0;
  }
  rotate(v, C, S, qx, qy, qz);
}

// Negative-energy eigenvector of h_s(P): (-(P_x - i s P_y), w + e) / sqrt(2 w (w + e)).
__device__ __forceinline__ void init_state(State& v, double Px, double Py, double e) {
  const double w = sqrt(fma(Px, Px, fma(Py, Py, e * e)));
  const double n = 1.0 / sqrt(2.0 * w * (w + e));
  v.ar = -Px * n; v.ai = Py * n;  v.br = (w + e) * n; v.bi = 0.0;   // s = +1
  v.cr = -Px * n; v.ci = -Py * n; v.dr = (w + e) * n; v.di = 0.0;   // s = -1
}

// f = sum_s |<+_s(P)|psi_s>|^2 with |+_s> = (w + e, P_x + i s P_y) / sqrt(2 w (w + e)).
__device__ __forceinline__ double project(const State& v, double Px, double Py, double e) {
  const double w = sqrt(fma(Px, Px, fma(Py, Py, e * e)));
  const double we = w + e;
  const double n2 = 1.0 / (2.0 * w * we);
  // s = +1: (w+e) a + (P_x - i P_y) b
  const double r1 = we * v.ar + Px * v.br + Py * v.bi;
  const double i1 = we * v.ai + Px * v.bi - Py * v.br;
  // s = -1: (w+e) c + (P_x + i P_y) d
  const double r2 = we * v.cr + Px * v.dr - Py * v.di;
  const double i2 = we * v.ci + Px * v.di + Py * v.dr;
  return (r1 * r1 + i1 * i1 + r2 * r2 + i2 * i2) * n2;
}

__device__ __forceinline__ int find_pulse(const PulseDev* __restrict__ desc, int n, int tile) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (desc[mid].tile_off <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Fixed-order tree sum of one value per lane over a 256-lane workgroup.
__device__ __forceinline__ double block_sum256(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  return red[0];
}

// Largest |A| of each pulse's table (bounds the step angle so the series degree can be chosen).
__global__ void __launch_bounds__(256) k_amax(const PulseDev* __restrict__ desc, const double* __restrict__ A,
                                              const double* __restrict__ Aedge, double* __restrict__ amax) {
  const PulseDev d = desc[blockIdx.x];
  const double2* tab = reinterpret_cast<const double2*>(A) + d.tab_off;
  double m = 0.0;
  for (int64_t n = threadIdx.x; n < d.nt; n += blockDim.x) {
    const double2 a = tab[n];
    m = fmax(m, sqrt(a.x * a.x + a.y * a.y));
  }
  if (threadIdx.x < 2) {
    const double2 a = reinterpret_cast<const double2*>(Aedge)[2 * blockIdx.x + threadIdx.x];
    m = fmax(m, sqrt(a.x * a.x + a.y * a.y));
  }
  __shared__ double red[256];
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) amax[blockIdx.x] = red[0];
}

template <int MODE>  // 0: degree 6, 1: degree 7, 2: degree 7 with angle halving
__device__ __forceinline__ void run_chunk(State& v, const double2* buf, int len, double pxdt, double pydt, double qz,
                                          double qz2, int h, double inv4h) {
  if (len == kChunk) {
#pragma unroll 4
    for (int k = 0; k < kChunk; ++k) {
      if (MODE == 0) step<6>(v, buf[k], pxdt, pydt, qz, qz2);
      else if (MODE == 1) step<7>(v, buf[k], pxdt, pydt, qz, qz2);
      else step_halving(v, buf[k], pxdt, pydt, qz, qz2, h, inv4h);
    }
  } else {
    for (int k = 0; k < len; ++k) {
      if (MODE == 0) step<6>(v, buf[k], pxdt, pydt, qz, qz2);
      else if (MODE == 1) step<7>(v, buf[k], pxdt, pydt, qz, qz2);
      else step_halving(v, buf[k], pxdt, pydt, qz, qz2, h, inv4h);
    }
  }
}

template <int MODE>
__device__ void evolve_tile(State& v, const double2* __restrict__ tab, int nt, double dt, double pxdt, double pydt,
                            double qz, double qz2, int h, double inv4h, double2 (*lds)[kChunk]) {
  const int nchunks = (nt + kChunk - 1) / kChunk;
  {
    const int n = threadIdx.x;
    double2 a = n < nt ? tab[n] : make_double2(0.0, 0.0);
    lds[0][threadIdx.x] = make_double2(-a.x * dt, -a.y * dt);
  }
  __syncthreads();
  for (int c = 0; c < nchunks; ++c) {
    const int nn = (c + 1) * kChunk + threadIdx.x;
    double2 a = (c + 1 < nchunks && nn < nt) ? tab[nn] : make_double2(0.0, 0.0);
    const int len = min(kChunk, nt - c * kChunk);
    run_chunk<MODE>(v, lds[c & 1], len, pxdt, pydt, qz, qz2, h, inv4h);
    lds[(c + 1) & 1][threadIdx.x] = make_double2(-a.x * dt, -a.y * dt);
    __syncthreads();
  }
}

// Bound on x = (omega dt)^2 over a whole pulse (grid corners and the largest |A|), which selects the
// series: 0 = degree 6, 1 = degree 7, 2 = degree 7 with h angle halvings.  Per pulse, so every
// mode of a pulse uses the same arithmetic whatever the tiling.
__device__ __forceinline__ int series_mode(const PulseDev& d, double amax, int* h, double* inv4h) {
  const double pxm = fmax(fabs(d.lo[0]), fabs(d.lo[0] + d.n[0] * d.dp[0]));
  const double pym = fmax(fabs(d.lo[1]), fabs(d.lo[1] + d.n[1] * d.dp[1]));
  const double pzm = fmax(fabs(d.lo[2]), fabs(d.lo[2] + d.n[2] * d.dp[2]));
  const double pr = sqrt(pxm * pxm + pym * pym) + amax;
  const double xb = (pr * pr + 1.0 + pzm * pzm) * d.dt * d.dt * (1.0 + 1e-6);
  *h = 0;
  *inv4h = 1.0;
  if (xb <= kXmax6) return 0;
  if (xb <= kXmax7) return 1;
  while (xb * *inv4h > kXmax7) {
    ++*h;
    *inv4h *= 0.25;
  }
  return 2;
}

// One launch per series variant; a workgroup whose pulse needs another variant exits at once.
template <int MODE>
__global__ void __launch_bounds__(kThreads) k_evolve(const PulseDev* __restrict__ desc, int n_pulses,
                                                     const double* __restrict__ A, const double* __restrict__ Aedge,
                                                     const double* __restrict__ amax, double* __restrict__ f,
                                                     double* __restrict__ tile_sums) {
  __shared__ double2 lds[2][kChunk];
  __shared__ double red[kThreads];
  const int tile = blockIdx.x;
  const int pi = find_pulse(desc, n_pulses, tile);
  const PulseDev& dref = desc[pi];
  int h;
  double inv4h;
  if (series_mode(dref, amax[pi], &h, &inv4h) != MODE) return;
  const int64_t mode_off = dref.mode_off, tab_off = dref.tab_off;
  const int nt = dref.nt;
  const double dt = dref.dt;
  const int nx = dref.n[0], ny = dref.n[1], nz = dref.n[2];
  const int64_t nmodes = int64_t(nx) * ny * nz;
  const int64_t m = int64_t(tile - dref.tile_off) * kThreads + threadIdx.x;
  const bool active = m < nmodes;
  const int64_t mm = active ? m : 0;
  const int ix = int(mm % nx), iy = int((mm / nx) % ny), iz = int(mm / (int64_t(nx) * ny));
  const double px = __dadd_rn(dref.lo[0], __dmul_rn(double(ix) + 0.5, dref.dp[0]));
  const double py = __dadd_rn(dref.lo[1], __dmul_rn(double(iy) + 0.5, dref.dp[1]));
  const double pz = __dadd_rn(dref.lo[2], __dmul_rn(double(iz) + 0.5, dref.dp[2]));
  const double e = sqrt(fma(pz, pz, 1.0));

  const double2* edge = reinterpret_cast<const double2*>(Aedge) + 2 * pi;
  const double2 ain = edge[0], aout = edge[1];
  State v;
  init_state(v, px - ain.x, py - ain.y, e);

  const double pxdt = px * dt, pydt = py * dt, qz = e * dt, qz2 = qz * qz;
  const double2* tab = reinterpret_cast<const double2*>(A) + tab_off;
  evolve_tile<MODE>(v, tab, nt, dt, pxdt, pydt, qz, qz2, h, inv4h, lds);

  const double fv = active ? project(v, px - aout.x, py - aout.y, e) : 0.0;
  if (f && active) f[mode_off + m] = fv;
  if (tile_sums) {
    const double s = block_sum256(fv, red);
    if (threadIdx.x == 0) tile_sums[tile] = s;
  }
}

// Tile sums from a stored f array, in the same tree order as the fused reduction.
__global__ void __launch_bounds__(kThreads) k_tile_sums(const PulseDev* __restrict__ desc, int n_pulses,
                                                        const double* __restrict__ f, double* __restrict__ tile_sums) {
  __shared__ double red[kThreads];
  const int tile = blockIdx.x;
  const int pi = find_pulse(desc, n_pulses, tile);
  const PulseDev& d = desc[pi];
  const int64_t nmodes = int64_t(d.n[0]) * d.n[1] * d.n[2];
  const int64_t m = int64_t(tile - d.tile_off) * kThreads + threadIdx.x;
  const double v = m < nmodes ? f[d.mode_off + m] : 0.0;
  const double s = block_sum256(v, red);
  if (threadIdx.x == 0) tile_sums[tile] = s;
}

// J per pulse: fixed-order tree over the pulse's tile sums, times the cell volume.
__global__ void __launch_bounds__(kThreads) k_yield(const PulseDev* __restrict__ desc,
                                                    const double* __restrict__ tile_sums, double* __restrict__ J) {
  __shared__ double red[kThreads];
  const PulseDev& d = desc[blockIdx.x];
  double v = 0.0;
  for (int t = threadIdx.x; t < d.ntiles; t += kThreads) v += tile_sums[d.tile_off + t];
  const double s = block_sum256(v, red);
  if (threadIdx.x == 0) J[blockIdx.x] = s * d.dv;
}

}  // namespace

po_status launch_evolve(const Batch& b, const PulseDev* d_desc, const double* d_A, const double* d_A_edge,
                        double* d_f, double* d_tile_sums, hipStream_t s) {
  Scratch am;
  PO_TRY(am.alloc(sizeof(double) * b.n_pulses, s));
  double* d_amax = static_cast<double*>(am.ptr);
  hipLaunchKernelGGL(k_amax, dim3(b.n_pulses), dim3(256), 0, s, d_desc, d_A, d_A_edge, d_amax);
  PO_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_evolve<0>, dim3(b.total_tiles), dim3(kThreads), 0, s, d_desc, b.n_pulses, d_A, d_A_edge,
                     d_amax, d_f, d_tile_sums);
  PO_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_evolve<1>, dim3(b.total_tiles), dim3(kThreads), 0, s, d_desc, b.n_pulses, d_A, d_A_edge,
                     d_amax, d_f, d_tile_sums);
  PO_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_evolve<2>, dim3(b.total_tiles), dim3(kThreads), 0, s, d_desc, b.n_pulses, d_A, d_A_edge,
                     d_amax, d_f, d_tile_sums);
  PO_HIP(hipGetLastError());
  return PO_OK;
}

po_status launch_tile_sums_from_f(const Batch& b, const PulseDev* d_desc, const double* d_f, double* d_tile_sums,
                                  hipStream_t s) {
  hipLaunchKernelGGL(k_tile_sums, dim3(b.total_tiles), dim3(kThreads), 0, s, d_desc, b.n_pulses, d_f, d_tile_sums);
  PO_HIP(hipGetLastError());
  return PO_OK;
}

po_status launch_yield_from_tiles(const Batch& b, const PulseDev* d_desc, const double* d_tile_sums, double* d_J,
                                  hipStream_t s) {
  hipLaunchKernelGGL(k_yield, dim3(b.n_pulses), dim3(kThreads), 0, s, d_desc, d_tile_sums, d_J);
  PO_HIP(hipGetLastError());
  return PO_OK;
}

}  // namespace po
