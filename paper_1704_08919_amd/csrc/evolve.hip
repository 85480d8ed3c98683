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
// unitary scheme): with q = (p - A_{n+1/2}) dt, q_z = e_perp dt, Q_s = q_x tau_x + s q_y tau_y +
// q_z tau_z and x = |q|^2 = (omega dt)^2 (so Q_s^2 = x),
//     U = C(x) 1 - i S(x) Q_s = C(x) [1 - i T(x) Q_s],
//     C(x) = cos sqrt(x),  S(x) = sin sqrt(x) / sqrt(x),  T(x) = tan sqrt(x) / sqrt(x).
// The scalar C is common to both blocks, and f is a ratio of squared norms, so the kernel
// applies only 1 - i T Q_s (three FMAs per real component) and divides by the norms at the
// end; the state is rescaled by an exact power of two once per LDS chunk to stay in range.
// For any value of T, 1 - i T Q_s is a scalar multiple of a unitary matrix (its square modulus
// is (1 + T^2 x) 1), so rounding in T perturbs only the rotation angle.  T is a polynomial in x
// (a fit of (T - 1)/x whose error is below 2^-57) of the lowest degree that covers the whole
// range of x of the 512-mode block the item belongs to in the 256-step chunk (a box of momenta
// against the range of the table in the chunk); beyond the fits' range the large-step path
// halves the angle and takes C and S from truncated Maclaurin series (remainder below 2^-56).
// Either is shared by both blocks, because omega does not depend on s.
//
// Work decomposition: a workgroup of THREADS lanes (64-wide waves) owns an item of
// THREADS x MPL consecutive modes of one pulse, MPL modes per lane.  The pulse's table of -A dt
// is staged through LDS in chunks of 256 steps (double-buffered, one barrier per chunk) and
// every lane reads the same record, an LDS broadcast.  The states (2 blocks x 2 complex
// amplitudes per mode) stay in VGPRs for all nt steps.  f is summed per 64-mode unit by one
// wave in a fixed butterfly order, and units per pulse in a fixed tree, so J does not depend on
// the launch shape or on scheduling.  Two launch forms share the item code: one workgroup per
// 256-mode item, or persistent workgroups that pull items (longest pulses first) from a device
// queue through an atomic counter.
#include <algorithm>

#include "dirac.hpp"
#include "reduce.hpp"

// Every fused multiply-add below is written out: automatic contraction is off, so each mode's
// arithmetic is the same instruction sequence in every launch shape (threads, modes per lane,
// persistent or not) and f is bitwise independent of the launch.
#pragma clang fp contract(off)

namespace po {
namespace {

// Box of cell-centred momenta of selection block b (kSelBlock consecutive modes) of a pulse:
// [pxl, pxh] x [pyl, pyh] and the largest p_z^2.
struct BlockBox {
  double pxl, pxh, pyl, pyh, pz2;
};

__device__ __forceinline__ BlockBox block_box(const PulseDev& d, int b) {
  const int nx = d.n[0], ny = d.n[1];
  const int64_t nmodes = int64_t(nx) * ny * d.n[2];
  const int64_t m0 = int64_t(b) * kSelBlock, m1 = min(m0 + kSelBlock, nmodes) - 1;
  const int64_t r0 = m0 / nx, r1 = m1 / nx;  // rows (iy, iz)
  const int64_t z0 = r0 / ny, z1 = r1 / ny;
  const int ix0 = r0 == r1 ? int(m0 % nx) : 0, ix1 = r0 == r1 ? int(m1 % nx) : nx - 1;
  const int iy0 = z0 == z1 ? int(r0 % ny) : 0, iy1 = z0 == z1 ? int(r1 % ny) : ny - 1;
  const double px0 = d.lo[0] + (ix0 + 0.5) * d.dp[0], px1 = d.lo[0] + (ix1 + 0.5) * d.dp[0];
  const double py0 = d.lo[1] + (iy0 + 0.5) * d.dp[1], py1 = d.lo[1] + (iy1 + 0.5) * d.dp[1];
  const double pz0 = d.lo[2] + (z0 + 0.5) * d.dp[2], pz1 = d.lo[2] + (z1 + 0.5) * d.dp[2];
  return BlockBox{fmin(px0, px1), fmax(px0, px1), fmin(py0, py1), fmax(py0, py1), fmax(pz0 * pz0, pz1 * pz1)};
}

// Series variant (x: index of the T fits or kFineHalving; y: angle halvings) for a bound xb on
// the step angle squared.  For a block box against a range [lx, hx] x [ly, hy] of table values,
// with the largest |p - A| per component,
//   x = (omega dt)^2 <= dt^2 [ max|p_x - A_x|^2 + max|p_y - A_y|^2 + 1 + max p_z^2 ].
__device__ __forceinline__ int2 variant_for_x(double xb) {
  int mode = kFineHalving, h = 0;
  for (int k = kNumFine - 1; k >= 0; --k)
    if (xb <= kFitXmax[k]) mode = k;
  if (mode == kFineHalving) {
    double x = xb;
    while (x > kCosSinXmax && h < kMaxHalvings) {
      x *= 0.25;
      ++h;
    }
  }
  return make_int2(mode, h);
}

// Bound on (omega dt)^2 for a block box against a range [lx, hx] x [ly, hy] of table values.
__device__ __forceinline__ double x_bound(const BlockBox& bb, double lx, double hx, double ly, double hy, double dt) {
  const double X = fmax(fmax(bb.pxh - lx, hx - bb.pxl), 0.0);
  const double Y = fmax(fmax(bb.pyh - ly, hy - bb.pyl), 0.0);
  return (X * X + Y * Y + 1.0 + bb.pz2) * dt * dt * (1.0 + 1e-6);
}

// NODES = 1: the second-order step's angle.  NODES = 2: the fourth-order step's, from theta^2 the
// bound above over both Gauss nodes, |w_s| <= theta + (sqrt3/6) theta^2.
template <int NODES>
__device__ __forceinline__ int2 choose_variant(const BlockBox& bb, double lx, double hx, double ly, double hy,
                                               double dt) {
  double xb = x_bound(bb, lx, hx, ly, hy, dt);
  if constexpr (NODES == 2) {
    const double th = sqrt(xb);
    xb = (th + kSqrt3Over6 * th * th) * (th + kSqrt3Over6 * th * th) * (1.0 + 1e-6);
  }
  return variant_for_x(xb);
}

// Variant of a block for the whole table (the union of its nchunks chunk ranges rg[c][4]).
template <int NODES = 1>
__device__ __forceinline__ int2 block_variant(const BlockBox& bb, const double* rg, int nchunks, double dt) {
  double lx = rg[0], hx = rg[1], ly = rg[2], hy = rg[3];
  for (int c = 1; c < nchunks; ++c) {
    lx = fmin(lx, rg[4 * c]); hx = fmax(hx, rg[4 * c + 1]);
    ly = fmin(ly, rg[4 * c + 2]); hy = fmax(hy, rg[4 * c + 3]);
  }
  return choose_variant<NODES>(bb, lx, hx, ly, hy, dt);
}

// Variant of chunk c given the block's (bmode).  A block within the T-series range: the lower of
// the block's variant and the one for the chunk's own range (both cover the chunk's steps).  A
// block on the angle-halving path: its chunks take that path with their own number of halvings,
// or, when their own range allows any T fit, the degree-11 one (two code paths only, so the
// loop keeps to its register budget).
template <int NODES = 1>
__device__ __forceinline__ int2 chunk_variant(const BlockBox& bb, const double* rg, int c, int bmode, double dt) {
  const int2 own = choose_variant<NODES>(bb, rg[4 * c], rg[4 * c + 1], rg[4 * c + 2], rg[4 * c + 3], dt);
  if (bmode == kFineHalving) return own.x == kFineHalving ? own : make_int2(kNumFine - 1, 0);
  return make_int2(min(own.x, bmode), 0);
}

// Range (min A_x, max A_x, min A_y, max A_y) of the table over chunk blockIdx.x of pulse blockIdx.y
// (NODES = 2: over both Gauss-node values of every step).
template <int NODES>
__global__ void __launch_bounds__(256) k_chunk_ranges(const PulseDev* __restrict__ desc, const double* __restrict__ A,
                                                      double* __restrict__ ranges) {
  const PulseDev d = desc[blockIdx.y];
  const int c = blockIdx.x;
  const int nchunks = (d.nt + kChunk - 1) / kChunk;
  if (c >= nchunks) return;
  const int n = c * kChunk + int(threadIdx.x);
  double lx = INFINITY, hx = -INFINITY, ly = INFINITY, hy = -INFINITY;
  if (n < d.nt) {
#pragma unroll
    for (int k = 0; k < NODES; ++k) {
      const double2 a = reinterpret_cast<const double2*>(A)[NODES * (d.tab_off + n) + k];
      lx = fmin(lx, a.x); hx = fmax(hx, a.x);
      ly = fmin(ly, a.y); hy = fmax(hy, a.y);
    }
  }
  __shared__ double red[4][256];
  red[0][threadIdx.x] = -lx; red[1][threadIdx.x] = hx; red[2][threadIdx.x] = -ly; red[3][threadIdx.x] = hy;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w)
      for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = fmax(red[k][threadIdx.x], red[k][threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x < 4) {
    const double v = red[threadIdx.x][0];
    ranges[4 * int64_t(d.chk_off + c) + threadIdx.x] = (threadIdx.x % 2 == 0) ? -v : v;
  }
}

// Per block of kSelBlock consecutive modes of a pulse, the variant for the range of the whole
// table (the yield gradient's choice).  Items of every launch shape lie inside one block.  One
// workgroup per pulse: the table's extremes, then one thread per block.
__global__ void __launch_bounds__(256) k_block_select(const PulseDev* __restrict__ desc, const double* __restrict__ A,
                                                      int2* __restrict__ bsel) {
  const PulseDev d = desc[blockIdx.x];
  const double2* tab = reinterpret_cast<const double2*>(A) + d.tab_off;
  double lx = INFINITY, hx = -INFINITY, ly = INFINITY, hy = -INFINITY;
  for (int64_t n = threadIdx.x; n < d.nt; n += blockDim.x) {
    const double2 a = tab[n];
    lx = fmin(lx, a.x); hx = fmax(hx, a.x);
    ly = fmin(ly, a.y); hy = fmax(hy, a.y);
  }
  __shared__ double red[4][256];
  red[0][threadIdx.x] = -lx; red[1][threadIdx.x] = hx; red[2][threadIdx.x] = -ly; red[3][threadIdx.x] = hy;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w)
      for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = fmax(red[k][threadIdx.x], red[k][threadIdx.x + w]);
    __syncthreads();
  }
  const double axl = -red[0][0], axh = red[1][0], ayl = -red[2][0], ayh = red[3][0];
  const int64_t nmodes = int64_t(d.n[0]) * d.n[1] * d.n[2];
  const int nblk = int((nmodes + kSelBlock - 1) / kSelBlock);
  for (int b = threadIdx.x; b < nblk; b += blockDim.x)
    bsel[d.blk_off + b] = choose_variant<1>(block_box(d, b), axl, axh, ayl, ayh, d.dt);
}

struct EvolveArgs {
  const PulseDev* desc;
  int n_pulses;
  const double* A;
  const double* Aedge;
  const double* ranges;  // [total_chunks][4] table range per chunk (k_chunk_ranges)
  double* f;
  double* units;
};

// Steps of one chunk (len records of buf) in series variant MODE for the MPL modes of a lane; the
// tangent form (the variant's fit coefficients loaded once per chunk) then rescales the states by
// exact powers of two.
template <int MODE, int MPL>
__device__ __forceinline__ void run_chunk(State (&v)[MPL], const double2* buf, int len, const double (&pxdt)[MPL],
                                          const double (&pydt)[MPL], const double (&qz)[MPL], const double (&qz2)[MPL],
                                          int h) {
  if constexpr (MODE < kFineHalving) {
    const Fit<MODE> f = load_fit<MODE>();
    if (len == kChunk) {
#pragma unroll(MPL == 1 ? 4 : 2)
      for (int k = 0; k < kChunk; ++k) {
        const double2 rec = buf[k];
#pragma unroll
        for (int j = 0; j < MPL; ++j) step_tan<MODE>(v[j], rec, pxdt[j], pydt[j], qz[j], qz2[j], f);
      }
    } else {
      for (int k = 0; k < len; ++k) {
        const double2 rec = buf[k];
#pragma unroll
        for (int j = 0; j < MPL; ++j) step_tan<MODE>(v[j], rec, pxdt[j], pydt[j], qz[j], qz2[j], f);
      }
    }
#pragma unroll
    for (int j = 0; j < MPL; ++j) renormalise(v[j]);
  } else {
    const double inv4h = ldexp(1.0, -2 * h);
    if (len == kChunk) {
#pragma unroll(MPL == 1 ? 4 : 2)
      for (int k = 0; k < kChunk; ++k) {
        const double2 rec = buf[k];
#pragma unroll
        for (int j = 0; j < MPL; ++j) step_halving(v[j], rec, pxdt[j], pydt[j], qz[j], qz2[j], h, inv4h);
      }
    } else {
      for (int k = 0; k < len; ++k) {
        const double2 rec = buf[k];
#pragma unroll
        for (int j = 0; j < MPL; ++j) step_halving(v[j], rec, pxdt[j], pydt[j], qz[j], qz2[j], h, inv4h);
      }
    }
  }
}

// The chunks of an item: table records staged through LDS (double-buffered, one barrier per
// chunk) and the steps of each chunk in its variant (chunk_variant); HALVING: the block's own
// variant is the angle-halving path.
template <bool HALVING, int THREADS, int MPL>
__device__ __forceinline__ void chunk_loop(State (&v)[MPL], const double2* tab, int nt, double dt, const double* rg,
                                           const BlockBox& bb, int bmode, const double (&pxdt)[MPL],
                                           const double (&pydt)[MPL], const double (&qz)[MPL],
                                           const double (&qz2)[MPL], double2 (*lds)[kChunk]) {
  constexpr int kPre = kChunk / THREADS;  // table records each lane stages per chunk
  const int nchunks = (nt + kChunk - 1) / kChunk;
#pragma unroll
  for (int r = 0; r < kPre; ++r) {
    const int n = r * THREADS + threadIdx.x;
    const double2 t = n < nt ? tab[n] : make_double2(0.0, 0.0);
    lds[0][n] = make_double2(-t.x * dt, -t.y * dt);
  }
  __syncthreads();
  for (int c = 0; c < nchunks; ++c) {
    double2 pre[kPre];
#pragma unroll
    for (int r = 0; r < kPre; ++r) {
      const int n = (c + 1) * kChunk + r * THREADS + threadIdx.x;
      pre[r] = (c + 1 < nchunks && n < nt) ? tab[n] : make_double2(0.0, 0.0);
    }
    const double2* buf = lds[c & 1];
    const int len = min(kChunk, nt - c * kChunk);
    const int2 cv = chunk_variant(bb, rg, c, bmode, dt);
    const int mode = __builtin_amdgcn_readfirstlane(cv.x);
    if constexpr (HALVING) {
      if (mode == kFineHalving)
        run_chunk<kFineHalving, MPL>(v, buf, len, pxdt, pydt, qz, qz2, __builtin_amdgcn_readfirstlane(cv.y));
      else
        run_chunk<kNumFine - 1, MPL>(v, buf, len, pxdt, pydt, qz, qz2, 0);
    } else {
      switch (mode) {
        case 0: run_chunk<0, MPL>(v, buf, len, pxdt, pydt, qz, qz2, 0); break;
        case 1: run_chunk<1, MPL>(v, buf, len, pxdt, pydt, qz, qz2, 0); break;
        case 2: run_chunk<2, MPL>(v, buf, len, pxdt, pydt, qz, qz2, 0); break;
        case 3: run_chunk<3, MPL>(v, buf, len, pxdt, pydt, qz, qz2, 0); break;
        case 4: run_chunk<4, MPL>(v, buf, len, pxdt, pydt, qz, qz2, 0); break;
        case 5: run_chunk<5, MPL>(v, buf, len, pxdt, pydt, qz, qz2, 0); break;
        case 6: run_chunk<6, MPL>(v, buf, len, pxdt, pydt, qz, qz2, 0); break;
        default: run_chunk<7, MPL>(v, buf, len, pxdt, pydt, qz, qz2, 0); break;
      }
    }
#pragma unroll
    for (int r = 0; r < kPre; ++r)
      lds[(c + 1) & 1][r * THREADS + threadIdx.x] = make_double2(-pre[r].x * dt, -pre[r].y * dt);
    __syncthreads();
  }
}

// Evolves the item of THREADS * MPL modes of pulse pi starting at mode `first`, writes f and the
// 64-mode unit sums.  Every lane of the workgroup must call it (it contains barriers).  The
// series variant is chosen from the item's selection block (items never straddle blocks) and the
// table ranges, so it depends only on the pulse, the block and the chunk, never on the launch.
template <int THREADS, int MPL>
__device__ __forceinline__ void process_item(const EvolveArgs& a, int pi, int first, double2 (*lds)[kChunk]) {
  const PulseDev& d = a.desc[pi];
  const int nt = d.nt;
  const double dt = d.dt;
  const int nx = d.n[0], ny = d.n[1];
  const int64_t nmodes = int64_t(nx) * ny * d.n[2];
  const double2* tab = reinterpret_cast<const double2*>(a.A) + d.tab_off;
  const double2* edge = reinterpret_cast<const double2*>(a.Aedge) + 2 * pi;
  const double2 ain = edge[0];
  const BlockBox bb = block_box(d, first / kSelBlock);
  const double* rg = a.ranges + 4 * int64_t(d.chk_off);

  State v[MPL];
  double pxdt[MPL], pydt[MPL], qz[MPL], qz2[MPL];
#pragma unroll
  for (int j = 0; j < MPL; ++j) {
    const int64_t m = int64_t(first) + j * THREADS + threadIdx.x;
    const int64_t mm = m < nmodes ? m : 0;
    const int ix = int(mm % nx), iy = int((mm / nx) % ny), iz = int(mm / (int64_t(nx) * ny));
    const double px = __dadd_rn(d.lo[0], __dmul_rn(double(ix) + 0.5, d.dp[0]));
    const double py = __dadd_rn(d.lo[1], __dmul_rn(double(iy) + 0.5, d.dp[1]));
    const double pz = __dadd_rn(d.lo[2], __dmul_rn(double(iz) + 0.5, d.dp[2]));
    const double e = sqrt(fma(pz, pz, 1.0));
    init_state(v[j], px - ain.x, py - ain.y, e);
    pxdt[j] = px * dt;
    pydt[j] = py * dt;
    qz[j] = e * dt;
    qz2[j] = qz[j] * qz[j];
  }

  // The block's variant for the whole table bounds its chunks' (chunk_variant).
  const int bmode = __builtin_amdgcn_readfirstlane(block_variant(bb, rg, (nt + kChunk - 1) / kChunk, dt).x);
  if (bmode == kFineHalving)
    chunk_loop<true, THREADS, MPL>(v, tab, nt, dt, rg, bb, bmode, pxdt, pydt, qz, qz2, lds);
  else
    chunk_loop<false, THREADS, MPL>(v, tab, nt, dt, rg, bb, bmode, pxdt, pydt, qz, qz2, lds);

  const double2 aout = edge[1];
#pragma unroll
  for (int j = 0; j < MPL; ++j) {
    const int64_t m = int64_t(first) + j * THREADS + threadIdx.x;
    const bool active = m < nmodes;
    double fv = 0.0;
    if (active) {
      const int64_t mm = m;
      const int ix = int(mm % nx), iy = int((mm / nx) % ny), iz = int(mm / (int64_t(nx) * ny));
      const double px = __dadd_rn(d.lo[0], __dmul_rn(double(ix) + 0.5, d.dp[0]));
      const double py = __dadd_rn(d.lo[1], __dmul_rn(double(iy) + 0.5, d.dp[1]));
      const double pz = __dadd_rn(d.lo[2], __dmul_rn(double(iz) + 0.5, d.dp[2]));
      fv = project(v[j], px - aout.x, py - aout.y, sqrt(fma(pz, pz, 1.0)));
      if (a.f) a.f[d.mode_off + m] = fv;
    }
    if (a.units) {
      const double s = wave_sum(fv);
      const int64_t base = int64_t(first) + j * THREADS + (threadIdx.x & ~63);
      if ((threadIdx.x & 63) == 0 && base < nmodes) a.units[d.unit_off + base / kUnit] = s;
    }
  }
}

// One workgroup per 256-mode item; four waves per SIMD (the register budget of the variant
// switch, met without spills).
__global__ void __launch_bounds__(kItem) __attribute__((amdgpu_waves_per_eu(4))) k_evolve(EvolveArgs a) {
  __shared__ double2 lds[2][kChunk];
  const int item = xcd_item(blockIdx.x, gridDim.x);
  const int pi = find_pulse_item(a.desc, a.n_pulses, item);
  process_item<kItem, 1>(a, pi, (item - a.desc[pi].item_off) * kItem, lds);
}

__global__ void k_reset_counter(int* counter) { *counter = 0; }

// Persistent workgroups: pull {pulse, first mode} items in queue order until the queue is empty.
// Every workgroup reaches the exit: the counter only grows, and each pull returns a new index.
// Register budget: four waves per SIMD with one mode per lane; two with two modes per lane, which
// keep the same number of modes in flight per SIMD without spilling.
template <int THREADS, int MPL>
__global__ void __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(MPL == 1 ? 4 : 2)))
k_evolve_persistent(EvolveArgs a, const int2* __restrict__ queue, int n_items, int* __restrict__ counter) {
  __shared__ double2 lds[2][kChunk];
  __shared__ int s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const int item = s_item;
    __syncthreads();
    if (item >= n_items) break;
    const int2 q = queue[item];
    process_item<THREADS, MPL>(a, q.x, q.y, lds);
  }
}

// Unit sums from a stored f array, in the same butterfly order as the fused reduction.
__global__ void __launch_bounds__(256) k_unit_sums(const PulseDev* __restrict__ desc, int n_pulses,
                                                   const double* __restrict__ f, double* __restrict__ units) {
  const int item = blockIdx.x;
  const int pi = find_pulse_item(desc, n_pulses, item);
  const PulseDev& d = desc[pi];
  const int64_t nmodes = int64_t(d.n[0]) * d.n[1] * d.n[2];
  const int64_t m = int64_t(item - d.item_off) * kItem + threadIdx.x;
  const double v = m < nmodes ? f[d.mode_off + m] : 0.0;
  const double s = wave_sum(v);
  const int64_t base = m - (threadIdx.x & 63);
  if ((threadIdx.x & 63) == 0 && base < nmodes) units[d.unit_off + base / kUnit] = s;
}

// J per pulse: each lane sums units t, t + 256, ... in order, then a fixed tree; times the cell volume.
__global__ void __launch_bounds__(256) k_yield(const PulseDev* __restrict__ desc, const double* __restrict__ units,
                                               double* __restrict__ J) {
  __shared__ double red[256];
  const PulseDev& d = desc[blockIdx.x];
  double v = 0.0;
  for (int t = threadIdx.x; t < d.nunits; t += 256) v += units[d.unit_off + t];
  const double s = block_sum256(v, red);
  if (threadIdx.x == 0) J[blockIdx.x] = s * d.dv;
}

// Diagnostics: adds modes x steps of every (selection block, chunk) of every pulse to the count
// of the variant the evolution chose for it (the same block_variant and chunk_variant).
// One workgroup per pulse, one thread per block.
__global__ void __launch_bounds__(256) k_count_mode_steps(const PulseDev* __restrict__ desc,
                                                          const double* __restrict__ ranges,
                                                          unsigned long long* __restrict__ counts) {
  const PulseDev& d = desc[blockIdx.x];
  const int64_t nmodes = int64_t(d.n[0]) * d.n[1] * d.n[2];
  const int nblk = int((nmodes + kSelBlock - 1) / kSelBlock);
  const int nch = (d.nt + kChunk - 1) / kChunk;
  const double* rg = ranges + 4 * int64_t(d.chk_off);
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
    const BlockBox bb = block_box(d, b);
    const unsigned long long mb = (unsigned long long)min(int64_t(kSelBlock), nmodes - int64_t(b) * kSelBlock);
    unsigned long long local[kSeriesVariants] = {};
    const int bmode = block_variant(bb, rg, nch, d.dt).x;
    for (int c = 0; c < nch; ++c) {
      const int mode = chunk_variant(bb, rg, c, bmode, d.dt).x;
      local[min(max(mode, 0), kSeriesVariants - 1)] += mb * (unsigned long long)min(kChunk, d.nt - c * kChunk);
    }
    for (int k = 0; k < kSeriesVariants; ++k)
      if (local[k]) atomicAdd(&counts[k], local[k]);
  }
}

template <int THREADS, int MPL>
void launch_persistent_t(EvolveArgs a, const int2* q, int n_items, int nwg, int* counter, hipStream_t s) {
  hipLaunchKernelGGL((k_evolve_persistent<THREADS, MPL>), dim3(nwg), dim3(THREADS), 0, s, a, q, n_items, counter);
}

// ---------------------------------------------------------------------------------------------
// Fourth-order Magnus step with two Gauss-Legendre nodes t_n + (1/2 -+ sqrt3/6) dt per step
// (Blanes, Casas, Oteo & Ros, Phys. Rep. 470 (2009) 151): the fourth-order Dirac scheme that
// Sec. V C of the paper leaves for future work.  For the blocks h_s(t) = v_s . tau with
// v_s = (P_x, s P_y, e_perp), [h_2, h_1] = 2i (v_2 x v_1) . tau, so the Magnus exponent of a step
// is -i w_s . tau with
//     w_s = dt (v_1 + v_2)/2 + (sqrt3/6) dt^2 (v_2 x v_1),
// and the step is again U = C [1 - i T(|w_s|^2) w_s . tau], now with one w_s (and one T) per
// block.  With a_k = (p_x - A_x(t_k)) dt, b_k likewise, e = e_perp dt, abar = (a_1 + a_2)/2 and
// g = (sqrt3/6) (a_1 - a_2, b_1 - b_2):
//     w_s = (abar - s e g_y,  s (bbar + s e g_x),  e + s (abar g_y - bbar g_x)).
// The record staged per step is (-(A_1 + A_2) dt/2, (sqrt3/6)(A_2 - A_1) dt): abar and g cost one
// add each.  The two blocks now rotate by different angles, so each is rescaled on its own.
// ---------------------------------------------------------------------------------------------

struct Magnus4 {
  double Xp, Yp, Zp, Xm, Ym, Zm;  // w_{+1} = (Xp, Yp, Zp); w_{-1} = (Xm, -Ym, Zm)
};

__device__ __forceinline__ Magnus4 magnus4(double4 rec, double pxdt, double pydt, double e) {
  const double ab = pxdt + rec.x, bb = pydt + rec.y;
  const double egx = e * rec.z, egy = e * rec.w;
  const double g = fma(ab, rec.w, -(bb * rec.z));
  return Magnus4{ab - egy, bb + egx, e + g, ab + egy, bb - egx, e - g};
}

template <int V>  // series variant
__device__ __forceinline__ void step4_tan(State& v, double4 rec, double pxdt, double pydt, double e, const Fit<V>& f) {
  const Magnus4 w = magnus4(rec, pxdt, pydt, e);
  const double xp = fma(w.Xp, w.Xp, fma(w.Yp, w.Yp, w.Zp * w.Zp));
  const double xm = fma(w.Xm, w.Xm, fma(w.Ym, w.Ym, w.Zm * w.Zm));
  const double Tp = tan_ratio<V>(xp, f), Tm = tan_ratio<V>(xm, f);
  rotate_block_tan(v.ar, v.ai, v.br, v.bi, Tp * w.Xp, Tp * w.Yp, Tp * w.Zp);
  rotate_block_tan(v.cr, v.ci, v.dr, v.di, Tm * w.Xm, -(Tm * w.Ym), Tm * w.Zm);
}

__device__ __forceinline__ void step4_halving(State& v, double4 rec, double pxdt, double pydt, double e, int h,
                                              double inv4h) {
  const Magnus4 w = magnus4(rec, pxdt, pydt, e);
  const double xp = fma(w.Xp, w.Xp, fma(w.Yp, w.Yp, w.Zp * w.Zp));
  const double xm = fma(w.Xm, w.Xm, fma(w.Ym, w.Ym, w.Zm * w.Zm));
  double Cp, Sp, Cm, Sm;
  cos_sinc_halved(xp, h, inv4h, Cp, Sp);
  cos_sinc_halved(xm, h, inv4h, Cm, Sm);
  rotate_block(v.ar, v.ai, v.br, v.bi, Cp, Sp * w.Xp, Sp * w.Yp, Sp * w.Zp);
  rotate_block(v.cr, v.ci, v.dr, v.di, Cm, Sm * w.Xm, -(Sm * w.Ym), Sm * w.Zm);
}

// Rescales each block by its own exact power of two.
__device__ __forceinline__ void renormalise_blocks(State& v) {
  const double n1 = fma(v.bi, v.bi, fma(v.br, v.br, fma(v.ai, v.ai, v.ar * v.ar)));
  const double n2 = fma(v.di, v.di, fma(v.dr, v.dr, fma(v.ci, v.ci, v.cr * v.cr)));
  const int e1 = -(ilogb(n1) >> 1), e2 = -(ilogb(n2) >> 1);
  v.ar = ldexp(v.ar, e1); v.ai = ldexp(v.ai, e1); v.br = ldexp(v.br, e1); v.bi = ldexp(v.bi, e1);
  v.cr = ldexp(v.cr, e2); v.ci = ldexp(v.ci, e2); v.dr = ldexp(v.dr, e2); v.di = ldexp(v.di, e2);
}

// Steps of one chunk in variant MODE; the tangent form then rescales each block.
template <int MODE>
__device__ __forceinline__ void run_chunk4(State& v, const double4* buf, int len, double pxdt, double pydt, double e,
                                           int h) {
  if constexpr (MODE < kFineHalving) {
    const Fit<MODE> f = load_fit<MODE>();
    if (len == kChunk) {
#pragma unroll 2
      for (int k = 0; k < kChunk; ++k) step4_tan<MODE>(v, buf[k], pxdt, pydt, e, f);
    } else {
      for (int k = 0; k < len; ++k) step4_tan<MODE>(v, buf[k], pxdt, pydt, e, f);
    }
    renormalise_blocks(v);
  } else {
    const double inv4h = ldexp(1.0, -2 * h);
    if (len == kChunk) {
#pragma unroll 2
      for (int k = 0; k < kChunk; ++k) step4_halving(v, buf[k], pxdt, pydt, e, h, inv4h);
    } else {
      for (int k = 0; k < len; ++k) step4_halving(v, buf[k], pxdt, pydt, e, h, inv4h);
    }
  }
}

struct Evolve4Args {
  const PulseDev* desc;
  int n_pulses;
  const double* Ag;  // [sum nt][2 nodes][2] A at the Gauss-Legendre nodes
  const double* Aedge;
  const double* ranges;  // [total_chunks][4] range of the node values per chunk (k_chunk_ranges<2>)
  double* f;
  double* units;
};

// The chunks of a fourth-order item, as chunk_loop: the record staged per step is
// (-(A_1 + A_2) dt/2, (sqrt3/6)(A_2 - A_1) dt); each chunk in its variant (chunk_variant<2>).
template <bool HALVING>
__device__ __forceinline__ void chunk_loop4(State& v, const double4* tab, int nt, double dt, const double* rg,
                                            const BlockBox& bb, int bmode, double pxdt, double pydt, double e,
                                            double4 (*lds)[kChunk]) {
  const double hdt = -0.5 * dt, kdt = kSqrt3Over6 * dt;
  const int nchunks = (nt + kChunk - 1) / kChunk;
  {
    const double4 t = int(threadIdx.x) < nt ? tab[threadIdx.x] : make_double4(0.0, 0.0, 0.0, 0.0);
    lds[0][threadIdx.x] = make_double4(hdt * (t.x + t.z), hdt * (t.y + t.w), kdt * (t.z - t.x), kdt * (t.w - t.y));
  }
  __syncthreads();
  for (int c = 0; c < nchunks; ++c) {
    const int n = (c + 1) * kChunk + threadIdx.x;
    const double4 pre = (c + 1 < nchunks && n < nt) ? tab[n] : make_double4(0.0, 0.0, 0.0, 0.0);
    const double4* buf = lds[c & 1];
    const int len = min(kChunk, nt - c * kChunk);
    const int2 cv = chunk_variant<2>(bb, rg, c, bmode, dt);
    const int mode = __builtin_amdgcn_readfirstlane(cv.x);
    if constexpr (HALVING) {
      if (mode == kFineHalving)
        run_chunk4<kFineHalving>(v, buf, len, pxdt, pydt, e, __builtin_amdgcn_readfirstlane(cv.y));
      else
        run_chunk4<kNumFine - 1>(v, buf, len, pxdt, pydt, e, 0);
    } else {
      switch (mode) {
        case 0: run_chunk4<0>(v, buf, len, pxdt, pydt, e, 0); break;
        case 1: run_chunk4<1>(v, buf, len, pxdt, pydt, e, 0); break;
        case 2: run_chunk4<2>(v, buf, len, pxdt, pydt, e, 0); break;
        case 3: run_chunk4<3>(v, buf, len, pxdt, pydt, e, 0); break;
        case 4: run_chunk4<4>(v, buf, len, pxdt, pydt, e, 0); break;
        case 5: run_chunk4<5>(v, buf, len, pxdt, pydt, e, 0); break;
        case 6: run_chunk4<6>(v, buf, len, pxdt, pydt, e, 0); break;
        default: run_chunk4<7>(v, buf, len, pxdt, pydt, e, 0); break;
      }
    }
    lds[(c + 1) & 1][threadIdx.x] =
        make_double4(hdt * (pre.x + pre.z), hdt * (pre.y + pre.w), kdt * (pre.z - pre.x), kdt * (pre.w - pre.y));
    __syncthreads();
  }
}

// One 256-mode item of pulse pi, one mode per lane; the structure of process_item, with the
// series variant per (selection block, chunk) from the range of both node values.
__device__ __forceinline__ void process_item4(const Evolve4Args& a, int pi, int first, double4 (*lds)[kChunk]) {
  const PulseDev& d = a.desc[pi];
  const int nt = d.nt;
  const double dt = d.dt;
  const int64_t nmodes = int64_t(d.n[0]) * d.n[1] * d.n[2];
  const double4* tab = reinterpret_cast<const double4*>(a.Ag) + d.tab_off;
  const double2* edge = reinterpret_cast<const double2*>(a.Aedge) + 2 * pi;
  const int64_t m = int64_t(first) + threadIdx.x;
  double px, py, pz;
  mode_momentum(d, m < nmodes ? m : 0, px, py, pz);
  const double ep = sqrt(fma(pz, pz, 1.0));
  State v;
  const double2 ain = edge[0];
  init_state(v, px - ain.x, py - ain.y, ep);
  const double pxdt = px * dt, pydt = py * dt, e = ep * dt;
  const BlockBox bb = block_box(d, first / kSelBlock);
  const double* rg = a.ranges + 4 * int64_t(d.chk_off);
  const int bmode = __builtin_amdgcn_readfirstlane(block_variant<2>(bb, rg, (nt + kChunk - 1) / kChunk, dt).x);
  if (bmode == kFineHalving)
    chunk_loop4<true>(v, tab, nt, dt, rg, bb, bmode, pxdt, pydt, e, lds);
  else
    chunk_loop4<false>(v, tab, nt, dt, rg, bb, bmode, pxdt, pydt, e, lds);

  const double2 aout = edge[1];
  double fv = 0.0;
  if (m < nmodes) {
    fv = project(v, px - aout.x, py - aout.y, ep);
    if (a.f) a.f[d.mode_off + m] = fv;
  }
  if (a.units) write_unit(d, a.units, m, nmodes, fv);
}

__global__ void __launch_bounds__(kItem) __attribute__((amdgpu_waves_per_eu(4))) k_evolve4(Evolve4Args a) {
  __shared__ double4 lds[2][kChunk];
  const int item = xcd_item(blockIdx.x, gridDim.x);
  const int pi = find_pulse_item(a.desc, a.n_pulses, item);
  process_item4(a, pi, (item - a.desc[pi].item_off) * kItem, lds);
}

// ---------------------------------------------------------------------------------------------
// Split-operator steps: the frozen Hamiltonian splits into the part the field does not touch,
// alpha_z p_z + beta m (in each 2x2 block e_perp tau_z), and the field-driven transverse part
// P_x tau_x + s P_y tau_y; Strang's symmetric step with the field at the step midpoint is second
// order (the split-operator scheme Sec. II A names), and the triple-jump composition of three such
// steps of sizes w1 dt, w0 dt, w1 dt (w1 = 1/(2 - 2^(1/3)), w0 = 1 - 2 w1; Yoshida, Phys. Lett. A
// 150 (1990) 262) is fourth order (the splitting Sec. V C leaves for future work).
//
// Per block the constant factor is R(theta) = exp(-i theta tau_z), theta a multiple of e_perp dt,
// and the transverse one K = exp(-i Q_s) with Q_s = q_x tau_x + s q_y tau_y, q = (p - A) w dt.
// Adjacent half steps of R merge, so the whole evolution is
//     R(-theta_0) [prod over steps, substeps i: R(theta_i) K_i] R(theta_0),
// theta_0 = e dt/2 (Strang) or w1 e dt/2, theta_i = e dt (Strang) or ((w1 + w0)/2, (w1 + w0)/2,
// w1) e dt.  In tangent form R(theta) = cos(theta) (1 - i a tau_z), a = tan(theta), and
// K = C (1 - i T Q_s) with T = tan|q| / |q| (the evolution's polynomial fits, x = |q|^2); since
// tau_z Q_s = i (q_x tau_y - s q_y tau_x), the product is 1 - i w_s . tau with
//     w_s = (u - s a v, s v + a u, a),   u = T q_x, v = T q_y,
// again a scalar multiple of a unitary matrix, of the same norm for both blocks: one rescaling per
// chunk, as in the midpoint step (34 + n VALU instructions per substep against 31 + n).  Beyond
// the fits' range the exact C, S (angle halving) and c = cos(theta), s = sin(theta) give
//     R K = c C - i (S (c q_x - s_b s q_y), S (s_b c q_y + s q_x), s C) . tau,   s_b = +-1.
// ---------------------------------------------------------------------------------------------
constexpr double kTripleW1 = 1.3512071919596576;   // 1 / (2 - 2^(1/3))
constexpr double kTripleW0 = -1.7024143839193153;  // 1 - 2 w1

template <int NSUB>
struct SplitMode {
  double pxw[NSUB == 1 ? 1 : 2], pyw[NSUB == 1 ? 1 : 2];  // p w dt for the distinct weights
  double a[NSUB == 1 ? 1 : 2], c[NSUB == 1 ? 1 : 2], s[NSUB == 1 ? 1 : 2];  // tan, cos, sin of theta_i
};

// Weight index (into pxw, pyw) and angle index (into a, c, s) of substep i.
__device__ __forceinline__ constexpr int split_w(int i) { return i == 1 ? 1 : 0; }
__device__ __forceinline__ constexpr int split_t(int i) { return i == 2 ? 1 : 0; }

// psi <- R(phi) psi for both blocks: a <- a e^{-i phi}, b <- b e^{i phi}.
__device__ __forceinline__ void phase_z(State& v, double cp, double sp) {
  double r, i;
  r = fma(v.ai, sp, v.ar * cp); i = fma(-v.ar, sp, v.ai * cp); v.ar = r; v.ai = i;
  r = fma(-v.bi, sp, v.br * cp); i = fma(v.br, sp, v.bi * cp); v.br = r; v.bi = i;
  r = fma(v.ci, sp, v.cr * cp); i = fma(-v.cr, sp, v.ci * cp); v.cr = r; v.ci = i;
  r = fma(-v.di, sp, v.dr * cp); i = fma(v.dr, sp, v.di * cp); v.dr = r; v.di = i;
}

template <int V>
__device__ __forceinline__ void substep_split_tan(State& v, double2 rec, double pxw, double pyw, double a,
                                                  const Fit<V>& f) {
  const double qx = pxw + rec.x, qy = pyw + rec.y;  // rec = -A w dt
  const double x = fma(qx, qx, qy * qy);
  const double T = tan_ratio<V>(x, f);
  const double u = T * qx, w = T * qy;
  rotate_block_tan(v.ar, v.ai, v.br, v.bi, fma(-a, w, u), fma(a, u, w), a);
  rotate_block_tan(v.cr, v.ci, v.dr, v.di, fma(a, w, u), fma(a, u, -w), a);
}

__device__ __forceinline__ void substep_split_halving(State& v, double2 rec, double pxw, double pyw, double c,
                                                      double s, int h, double inv4h) {
  const double qx = pxw + rec.x, qy = pyw + rec.y;
  const double x = fma(qx, qx, qy * qy);
  double C, S;
  cos_sinc_halved(x, h, inv4h, C, S);
  const double cC = c * C, sz = s * C;
  const double cx = c * qx, cy = c * qy, sx = s * qx, sy = s * qy;
  rotate_block(v.ar, v.ai, v.br, v.bi, cC, S * (cx - sy), S * (cy + sx), sz);
  rotate_block(v.cr, v.ci, v.dr, v.di, cC, S * (cx + sy), S * (sx - cy), sz);
}

template <int NSUB, int MODE>
__device__ __forceinline__ void run_chunk_split(State& v, const double2* buf, int len, const SplitMode<NSUB>& k,
                                                int h) {
  if constexpr (MODE < kFineHalving) {
    const Fit<MODE> f = load_fit<MODE>();
    if (len == kChunk) {
#pragma unroll(NSUB == 1 ? 4 : 1)
      for (int n = 0; n < kChunk; ++n)
#pragma unroll
        for (int i = 0; i < NSUB; ++i)
          substep_split_tan<MODE>(v, buf[n * NSUB + i], k.pxw[split_w(i)], k.pyw[split_w(i)], k.a[split_t(i)], f);
    } else {
      for (int n = 0; n < len; ++n)
#pragma unroll
        for (int i = 0; i < NSUB; ++i)
          substep_split_tan<MODE>(v, buf[n * NSUB + i], k.pxw[split_w(i)], k.pyw[split_w(i)], k.a[split_t(i)], f);
    }
    renormalise(v);
  } else {
    const double inv4h = ldexp(1.0, -2 * h);
    for (int n = 0; n < len; ++n)
#pragma unroll
      for (int i = 0; i < NSUB; ++i)
        substep_split_halving(v, buf[n * NSUB + i], k.pxw[split_w(i)], k.pyw[split_w(i)], k.c[split_t(i)],
                              k.s[split_t(i)], h, inv4h);
  }
}

struct SplitArgs {
  const PulseDev* desc;
  int n_pulses;
  const double* At;  // [sum nt][NSUB][2] A at the substep midpoints
  const double* Aedge;
  const double* ranges;  // [total_chunks][4] range of the table per chunk (k_chunk_ranges<NSUB>)
  double* f;
  double* units;
};

// The chunks of an item: NSUB records per step staged through LDS as -A w_i dt (double-buffered,
// one barrier per chunk), each chunk in its variant for steps of size w_max dt.
template <int NSUB, bool HALVING>
__device__ __forceinline__ void chunk_loop_split(State& v, const double2* tab, int nt, double dt, double dtw,
                                                 const double* rg, const BlockBox& bb, int bmode,
                                                 const SplitMode<NSUB>& k, double2 (*lds)[NSUB * kChunk]) {
  const double wdt[3] = {NSUB == 1 ? -dt : -kTripleW1 * dt, -kTripleW0 * dt, -kTripleW1 * dt};
  const int nchunks = (nt + kChunk - 1) / kChunk;
#pragma unroll
  for (int i = 0; i < NSUB; ++i) {
    const double2 t = int(threadIdx.x) < nt ? tab[NSUB * threadIdx.x + i] : make_double2(0.0, 0.0);
    lds[0][NSUB * threadIdx.x + i] = make_double2(t.x * wdt[i], t.y * wdt[i]);
  }
  __syncthreads();
  for (int c = 0; c < nchunks; ++c) {
    double2 pre[NSUB];
    const int n = (c + 1) * kChunk + threadIdx.x;
#pragma unroll
    for (int i = 0; i < NSUB; ++i) pre[i] = (c + 1 < nchunks && n < nt) ? tab[NSUB * n + i] : make_double2(0.0, 0.0);
    const double2* buf = lds[c & 1];
    const int len = min(kChunk, nt - c * kChunk);
    const int2 cv = chunk_variant<1>(bb, rg, c, bmode, dtw);
    const int mode = __builtin_amdgcn_readfirstlane(cv.x);
    if constexpr (HALVING) {
      if (mode == kFineHalving)
        run_chunk_split<NSUB, kFineHalving>(v, buf, len, k, __builtin_amdgcn_readfirstlane(cv.y));
      else
        run_chunk_split<NSUB, kNumFine - 1>(v, buf, len, k, 0);
    } else {
      switch (mode) {
        case 0: run_chunk_split<NSUB, 0>(v, buf, len, k, 0); break;
        case 1: run_chunk_split<NSUB, 1>(v, buf, len, k, 0); break;
        case 2: run_chunk_split<NSUB, 2>(v, buf, len, k, 0); break;
        case 3: run_chunk_split<NSUB, 3>(v, buf, len, k, 0); break;
        case 4: run_chunk_split<NSUB, 4>(v, buf, len, k, 0); break;
        case 5: run_chunk_split<NSUB, 5>(v, buf, len, k, 0); break;
        case 6: run_chunk_split<NSUB, 6>(v, buf, len, k, 0); break;
        default: run_chunk_split<NSUB, 7>(v, buf, len, k, 0); break;
      }
    }
#pragma unroll
    for (int i = 0; i < NSUB; ++i)
      lds[(c + 1) & 1][NSUB * threadIdx.x + i] = make_double2(pre[i].x * wdt[i], pre[i].y * wdt[i]);
    __syncthreads();
  }
}

// One 256-mode item of pulse pi, one mode per lane, the structure of process_item4.  The series
// variant per (selection block, chunk) bounds |q|^2 <= |p - A|^2 (w_max dt)^2 through the
// second-order bound at step w_max dt (which also counts (1 + p_z^2)(w_max dt)^2: conservative).
template <int NSUB>
__device__ __forceinline__ void process_item_split(const SplitArgs& a, int pi, int first,
                                                   double2 (*lds)[NSUB * kChunk]) {
  const PulseDev& d = a.desc[pi];
  const int nt = d.nt;
  const double dt = d.dt;
  const double dtw = NSUB == 1 ? dt : -kTripleW0 * dt;  // the largest substep
  const int64_t nmodes = int64_t(d.n[0]) * d.n[1] * d.n[2];
  const double2* tab = reinterpret_cast<const double2*>(a.At) + NSUB * d.tab_off;
  const double2* edge = reinterpret_cast<const double2*>(a.Aedge) + 2 * pi;
  const int64_t m = int64_t(first) + threadIdx.x;
  double px, py, pz;
  mode_momentum(d, m < nmodes ? m : 0, px, py, pz);
  const double ep = sqrt(fma(pz, pz, 1.0));
  SplitMode<NSUB> k;
  double th0;
  if constexpr (NSUB == 1) {
    k.pxw[0] = px * dt;
    k.pyw[0] = py * dt;
    sincos(ep * dt, &k.s[0], &k.c[0]);
    th0 = 0.5 * ep * dt;
  } else {
    k.pxw[0] = px * (kTripleW1 * dt); k.pyw[0] = py * (kTripleW1 * dt);
    k.pxw[1] = px * (kTripleW0 * dt); k.pyw[1] = py * (kTripleW0 * dt);
    sincos(0.5 * (kTripleW1 + kTripleW0) * ep * dt, &k.s[0], &k.c[0]);
    sincos(kTripleW1 * ep * dt, &k.s[1], &k.c[1]);
    th0 = 0.5 * kTripleW1 * ep * dt;
  }
#pragma unroll
  for (int j = 0; j < (NSUB == 1 ? 1 : 2); ++j) k.a[j] = k.s[j] / k.c[j];
  double s0, c0;
  sincos(th0, &s0, &c0);
  State v;
  const double2 ain = edge[0];
  init_state(v, px - ain.x, py - ain.y, ep);
  phase_z(v, c0, s0);
  const BlockBox bb = block_box(d, first / kSelBlock);
  const double* rg = a.ranges + 4 * int64_t(d.chk_off);
  const int bmode = __builtin_amdgcn_readfirstlane(block_variant<1>(bb, rg, (nt + kChunk - 1) / kChunk, dtw).x);
  if (bmode == kFineHalving)
    chunk_loop_split<NSUB, true>(v, tab, nt, dt, dtw, rg, bb, bmode, k, lds);
  else
    chunk_loop_split<NSUB, false>(v, tab, nt, dt, dtw, rg, bb, bmode, k, lds);
  phase_z(v, c0, -s0);

  const double2 aout = edge[1];
  double fv = 0.0;
  if (m < nmodes) {
    fv = project(v, px - aout.x, py - aout.y, ep);
    if (a.f) a.f[d.mode_off + m] = fv;
  }
  if (a.units) write_unit(d, a.units, m, nmodes, fv);
}

template <int NSUB>
__global__ void __launch_bounds__(kItem) k_evolve_split(SplitArgs a) {
  __shared__ double2 lds[2][NSUB * kChunk];
  const int item = xcd_item(blockIdx.x, gridDim.x);
  const int pi = find_pulse_item(a.desc, a.n_pulses, item);
  process_item_split<NSUB>(a, pi, (item - a.desc[pi].item_off) * kItem, lds);
}

}  // namespace

po_status launch_block_select(const Batch& b, const PulseDev* d_desc, const double* d_A, int2* d_bsel,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_block_select, dim3(b.n_pulses), dim3(256), 0, s, d_desc, d_A, d_bsel);
  PO_HIP(hipGetLastError());
  return PO_OK;
}

po_status launch_chunk_ranges(const Batch& b, const PulseDev* d_desc, const double* d_A, double* d_ranges,
                              hipStream_t s) {
  const int max_chunks = (b.max_nt + kChunk - 1) / kChunk;
  hipLaunchKernelGGL(k_chunk_ranges<1>, dim3(max_chunks, b.n_pulses), dim3(256), 0, s, d_desc, d_A, d_ranges);
  PO_HIP(hipGetLastError());
  return PO_OK;
}

po_status launch_evolve_grid(const Batch& b, const PulseDev* d_desc, const double* d_A, const double* d_A_edge,
                             const double* d_ranges, double* d_f, double* d_units, hipStream_t s) {
  EvolveArgs a{d_desc, b.n_pulses, d_A, d_A_edge, d_ranges, d_f, d_units};
  hipLaunchKernelGGL(k_evolve, dim3(b.total_items), dim3(kItem), 0, s, a);
  PO_HIP(hipGetLastError());
  return PO_OK;
}

template <int THREADS, int MPL>
int resident_persistent_t() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(&k_evolve_persistent<THREADS, MPL>),
                                                   THREADS, 0) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return n;
}

int evolve_workgroups_per_cu(const EvolveConfig& cfg) {
  // workgroups of the instantiated persistent kernel that fit on one CU at its register and LDS
  // use (the runtime's occupancy query); if the query fails, the waves-per-SIMD bound each
  // instantiation is compiled for (4 with one mode per lane, 2 with two), four SIMDs per CU
  int n = 0;
  switch (cfg.threads * 10 + cfg.mpl) {
    case 641: n = resident_persistent_t<64, 1>(); break;
    case 642: n = resident_persistent_t<64, 2>(); break;
    case 1281: n = resident_persistent_t<128, 1>(); break;
    case 1282: n = resident_persistent_t<128, 2>(); break;
    case 2561: n = resident_persistent_t<256, 1>(); break;
    case 2562: n = resident_persistent_t<256, 2>(); break;
    default: break;
  }
  if (n > 0) return n;
  const int waves_per_simd = cfg.mpl == 1 ? 4 : 2;
  return std::max(1, waves_per_simd * 4 / (cfg.threads / 64));
}

po_status launch_evolve_persistent(const EvolveConfig& cfg, int n_pulses, const PulseDev* d_desc, const double* d_A,
                                   const double* d_A_edge, const double* d_ranges, const int2* d_queue, int n_items,
                                   int n_workgroups, int* d_counter, double* d_f, double* d_units, hipStream_t s) {
  EvolveArgs a{d_desc, n_pulses, d_A, d_A_edge, d_ranges, d_f, d_units};
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, s, d_counter);
  PO_HIP(hipGetLastError());
  const int key = cfg.threads * 10 + cfg.mpl;
  switch (key) {
    case 641: launch_persistent_t<64, 1>(a, d_queue, n_items, n_workgroups, d_counter, s); break;
    case 642: launch_persistent_t<64, 2>(a, d_queue, n_items, n_workgroups, d_counter, s); break;
    case 1281: launch_persistent_t<128, 1>(a, d_queue, n_items, n_workgroups, d_counter, s); break;
    case 1282: launch_persistent_t<128, 2>(a, d_queue, n_items, n_workgroups, d_counter, s); break;
    case 2561: launch_persistent_t<256, 1>(a, d_queue, n_items, n_workgroups, d_counter, s); break;
    case 2562: launch_persistent_t<256, 2>(a, d_queue, n_items, n_workgroups, d_counter, s); break;
    default: return set_error(PO_ERR_INVALID, "unsupported evolution config threads=%d mpl=%d", cfg.threads, cfg.mpl);
  }
  PO_HIP(hipGetLastError());
  return PO_OK;
}

po_status launch_count_mode_steps(int n_pulses, const PulseDev* d_desc, const double* d_ranges,
                                  unsigned long long* d_counts, hipStream_t s) {
  hipLaunchKernelGGL(k_count_mode_steps, dim3(n_pulses), dim3(256), 0, s, d_desc, d_ranges, d_counts);
  PO_HIP(hipGetLastError());
  return PO_OK;
}

po_status launch_unit_sums_from_f(const Batch& b, const PulseDev* d_desc, const double* d_f, double* d_units,
                                  hipStream_t s) {
  hipLaunchKernelGGL(k_unit_sums, dim3(b.total_items), dim3(256), 0, s, d_desc, b.n_pulses, d_f, d_units);
  PO_HIP(hipGetLastError());
  return PO_OK;
}

po_status launch_yield_from_units(const Batch& b, const PulseDev* d_desc, const double* d_units, double* d_J,
                                  hipStream_t s) {
  hipLaunchKernelGGL(k_yield, dim3(b.n_pulses), dim3(256), 0, s, d_desc, d_units, d_J);
  PO_HIP(hipGetLastError());
  return PO_OK;
}

po_status launch_chunk_ranges4(const Batch& b, const PulseDev* d_desc, const double* d_Ag, double* d_ranges,
                               hipStream_t s) {
  const int max_chunks = (b.max_nt + kChunk - 1) / kChunk;
  hipLaunchKernelGGL(k_chunk_ranges<2>, dim3(max_chunks, b.n_pulses), dim3(256), 0, s, d_desc, d_Ag, d_ranges);
  PO_HIP(hipGetLastError());
  return PO_OK;
}

po_status launch_evolve4_grid(const Batch& b, const PulseDev* d_desc, const double* d_Ag, const double* d_A_edge,
                              const double* d_ranges, double* d_f, double* d_units, hipStream_t s) {
  Evolve4Args a{d_desc, b.n_pulses, d_Ag, d_A_edge, d_ranges, d_f, d_units};
  hipLaunchKernelGGL(k_evolve4, dim3(b.total_items), dim3(kItem), 0, s, a);
  PO_HIP(hipGetLastError());
  return PO_OK;
}

po_status launch_evolve_split_grid(const Batch& b, int order, const PulseDev* d_desc, const double* d_At,
                                   const double* d_A_edge, double* d_ranges, double* d_f, double* d_units,
                                   hipStream_t s) {
  const int max_chunks = (b.max_nt + kChunk - 1) / kChunk;
  SplitArgs a{d_desc, b.n_pulses, d_At, d_A_edge, d_ranges, d_f, d_units};
  if (order == 2) {
    hipLaunchKernelGGL(k_chunk_ranges<1>, dim3(max_chunks, b.n_pulses), dim3(256), 0, s, d_desc, d_At, d_ranges);
    PO_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_evolve_split<1>, dim3(b.total_items), dim3(kItem), 0, s, a);
  } else {
    hipLaunchKernelGGL(k_chunk_ranges<3>, dim3(max_chunks, b.n_pulses), dim3(256), 0, s, d_desc, d_At, d_ranges);
    PO_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_evolve_split<3>, dim3(b.total_items), dim3(kItem), 0, s, a);
  }
  PO_HIP(hipGetLastError());
  return PO_OK;
}

}  // namespace po
