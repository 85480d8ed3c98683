// Differential evolution DE/rand/1/bin (Sec. IV B of arXiv:1704.08919) on the GPU.
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of the 4x32
// Philox S-box with multipliers 0xD2511F53 / 0xCD9E8D57 and Weyl key increments 0x9E3779B9 /
// 0xBB67AE85.  Counter = (individual, block, generation lo, generation hi), key = seed.
// The arithmetic of a proposal rounds every operation separately (contraction is off in this
// file), so trials are identical bit for bit to any IEEE-754 evaluation of the same rules.
#include "common.hpp"

#pragma clang fp contract(off)

namespace po {
namespace {

constexpr int kMaxIslands = 64;      // islands per population (one migrating thread each)
constexpr int kMaxMigrateDim = 64;   // genes per individual staged by the migration kernel

struct U4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t m0 = uint64_t(0xD2511F53u) * c.x;
    const uint64_t m1 = uint64_t(0xCD9E8D57u) * c.z;
    c = U4{uint32_t(m1 >> 32) ^ c.y ^ k0, uint32_t(m1), uint32_t(m0 >> 32) ^ c.w ^ k1, uint32_t(m0)};
  }
  return c;
}

__device__ __forceinline__ uint32_t word(const U4& u, int w) {
  return w == 0 ? u.x : w == 1 ? u.y : w == 2 ? u.z : u.w;
}

__device__ __forceinline__ uint32_t index_below(uint32_t u, uint32_t n) {
  return uint32_t((uint64_t(u) * n) >> 32);
}

__device__ __forceinline__ double open01(uint32_t u) { return (double(u) + 0.5) * (1.0 / 4294967296.0); }

__global__ void __launch_bounds__(128) k_de_propose(po_de_params prm, int64_t gen, const double* __restrict__ pop,
                                                    double* __restrict__ trial, int32_t* __restrict__ idx) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int N = prm.pop, D = prm.dim;
  if (i >= N) return;
  const uint32_t k0 = uint32_t(prm.seed), k1 = uint32_t(prm.seed >> 32);
  const uint32_t g0 = uint32_t(uint64_t(gen)), g1 = uint32_t(uint64_t(gen) >> 32);
  const U4 r0 = philox4x32_10(U4{uint32_t(i), 0u, g0, g1}, k0, k1);
  // a, b, c: uniform over the individuals not yet excluded; exclusions skipped in ascending order.
  int ex[4] = {i, 0, 0, 0};
  int nex = 1;
  int pick[3];
  const uint32_t w3[3] = {r0.x, r0.y, r0.z};
  for (int r = 0; r < 3; ++r) {
    int x = int(index_below(w3[r], uint32_t(N - 1 - r)));
    int srt[4];
    for (int q = 0; q < nex; ++q) srt[q] = ex[q];
    for (int q = 1; q < nex; ++q)  // insertion sort of at most 3 values
      for (int z = q; z > 0 && srt[z - 1] > srt[z]; --z) {
        const int t = srt[z]; srt[z] = srt[z - 1]; srt[z - 1] = t;
      }
    for (int q = 0; q < nex; ++q)
      if (x >= srt[q]) ++x;
    pick[r] = x;
    ex[nex++] = x;
  }
  const int R = int(index_below(r0.w, uint32_t(D)));
  if (idx) {
    idx[4 * i + 0] = pick[0];
    idx[4 * i + 1] = pick[1];
    idx[4 * i + 2] = pick[2];
    idx[4 * i + 3] = R;
  }
  const double* a = pop + size_t(pick[0]) * D;
  const double* b = pop + size_t(pick[1]) * D;
  const double* c = pop + size_t(pick[2]) * D;
  const double* x = pop + size_t(i) * D;
  double* y = trial + size_t(i) * D;
  const int nb = (D + 3) / 4;
  U4 cr{}, rd{};
  for (int j = 0; j < D; ++j) {
    if ((j & 3) == 0) {
      cr = philox4x32_10(U4{uint32_t(i), uint32_t(1 + j / 4), g0, g1}, k0, k1);
      rd = philox4x32_10(U4{uint32_t(i), uint32_t(1 + nb + j / 4), g0, g1}, k0, k1);
    }
    const double r = open01(word(cr, j & 3));
    double v;
    if (r <= prm.CR || j == R) {
      const double diff = b[j] - c[j];
      const double st = prm.F * diff;
      v = a[j] + st;
    } else {
      v = x[j];
    }
    if (v < prm.lo || v > prm.hi) {
      const bool phase = prm.n_s > 0 && ((j / prm.n_s) & 1);
      const double w = prm.hi - prm.lo;
      if (phase) {
        const double k = floor((v - prm.lo) / w);
        v = v - w * k;
      } else {
        v = prm.lo + w * open01(word(rd, j & 3));
      }
    }
    y[j] = v;
  }
}

__global__ void __launch_bounds__(128) k_de_select(po_de_params prm, double* __restrict__ pop, double* __restrict__ fit,
                                                   const double* __restrict__ trial, const double* __restrict__ tfit,
                                                   const uint8_t* __restrict__ mask) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= prm.pop) return;
  if (mask && !mask[i]) return;
  if (tfit[i] >= fit[i]) {
    for (int j = 0; j < prm.dim; ++j) pop[size_t(i) * prm.dim + j] = trial[size_t(i) * prm.dim + j];
    fit[i] = tfit[i];
  }
}

// Indices of the set entries of a 0/1 mask, in increasing order (single workgroup, n <= 8192).
__global__ void __launch_bounds__(1024) k_mask_indices(const uint8_t* __restrict__ mask, int n, int32_t* __restrict__ idx,
                                                       int32_t* __restrict__ count) {
  __shared__ int32_t part[1024];
  const int per = (n + 1023) / 1024;
  const int lo = threadIdx.x * per, hi = min(n, lo + per);
  int c = 0;
  for (int i = lo; i < hi; ++i) c += mask[i] != 0;
  part[threadIdx.x] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int t = 0; t < 1024; ++t) {
      const int v = part[t];
      part[t] = run;
      run += v;
    }
    if (count) *count = run;
  }
  __syncthreads();
  int o = part[threadIdx.x];
  for (int i = lo; i < hi; ++i)
    if (mask[i]) idx[o++] = i;
}

// Rows whose index is out of [0, rows) read as NaN (no access outside the source).
__global__ void k_gather_rows(const double* __restrict__ src, int rows, int cols, const int32_t* __restrict__ idx,
                              int n_idx, double* __restrict__ dst) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= int64_t(n_idx) * cols) return;
  const int r = int(e / cols), c = int(e % cols);
  const int q = idx[r];
  dst[e] = (q >= 0 && q < rows) ? src[int64_t(q) * cols + c] : __longlong_as_double(0x7ff8000000000000LL);
}

// Self-adaptive DE (jDE: Brest, Greiner, Boskovic, Mernik & Zumer, IEEE Trans. Evol. Comput. 10
// (2006) 646, the variant named in Sec. IV B) on islands of S = pop / islands consecutive
// members.  Donors are drawn among the other members of the individual's island; (F, CR) are
// redrawn with probabilities tau1, tau2 from the extra Philox block 1 + 2 ceil(D/4).
__global__ void __launch_bounds__(128) k_jde_propose(po_jde_params prm, int64_t gen, const double* __restrict__ pop,
                                                     const double* __restrict__ fcr, double* __restrict__ trial,
                                                     double* __restrict__ tfcr, int32_t* __restrict__ idx) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int N = prm.pop, D = prm.dim;
  if (i >= N) return;
  const int S = N / prm.islands, base = (i / S) * S;
  const uint32_t k0 = uint32_t(prm.seed), k1 = uint32_t(prm.seed >> 32);
  const uint32_t g0 = uint32_t(uint64_t(gen)), g1 = uint32_t(uint64_t(gen) >> 32);
  const U4 r0 = philox4x32_10(U4{uint32_t(i), 0u, g0, g1}, k0, k1);
  int ex[4] = {i - base, 0, 0, 0};
  int nex = 1;
  int pick[3];
  const uint32_t w3[3] = {r0.x, r0.y, r0.z};
  for (int r = 0; r < 3; ++r) {
    int x = int(index_below(w3[r], uint32_t(S - 1 - r)));
    int srt[4];
    for (int q = 0; q < nex; ++q) srt[q] = ex[q];
    for (int q = 1; q < nex; ++q)
      for (int z = q; z > 0 && srt[z - 1] > srt[z]; --z) {
        const int t = srt[z]; srt[z] = srt[z - 1]; srt[z - 1] = t;
      }
    for (int q = 0; q < nex; ++q)
      if (x >= srt[q]) ++x;
    ex[nex++] = x;
    pick[r] = base + x;
  }
  const int R = int(index_below(r0.w, uint32_t(D)));
  if (idx) {
    idx[4 * i + 0] = pick[0];
    idx[4 * i + 1] = pick[1];
    idx[4 * i + 2] = pick[2];
    idx[4 * i + 3] = R;
  }
  const int nb = (D + 3) / 4;
  const U4 rp = philox4x32_10(U4{uint32_t(i), uint32_t(1 + 2 * nb), g0, g1}, k0, k1);
  double F = fcr[2 * i], CR = fcr[2 * i + 1];
  if (open01(rp.x) < prm.tau1) {
    const double span = prm.F_hi - prm.F_lo;
    const double step = open01(rp.y) * span;
    F = prm.F_lo + step;
  }
  if (open01(rp.z) < prm.tau2) CR = open01(rp.w);
  tfcr[2 * i] = F;
  tfcr[2 * i + 1] = CR;
  const double* a = pop + size_t(pick[0]) * D;
  const double* b = pop + size_t(pick[1]) * D;
  const double* c = pop + size_t(pick[2]) * D;
  const double* x = pop + size_t(i) * D;
  double* y = trial + size_t(i) * D;
  U4 cr{}, rd{};
  for (int j = 0; j < D; ++j) {
    if ((j & 3) == 0) {
      cr = philox4x32_10(U4{uint32_t(i), uint32_t(1 + j / 4), g0, g1}, k0, k1);
      rd = philox4x32_10(U4{uint32_t(i), uint32_t(1 + nb + j / 4), g0, g1}, k0, k1);
    }
    const double r = open01(word(cr, j & 3));
    double v;
    if (r <= CR || j == R) {
      const double diff = b[j] - c[j];
      const double st = F * diff;
      v = a[j] + st;
    } else {
      v = x[j];
    }
    if (v < prm.lo || v > prm.hi) {
      const bool phase = prm.n_s > 0 && ((j / prm.n_s) & 1);
      const double w = prm.hi - prm.lo;
      if (phase) {
        const double k = floor((v - prm.lo) / w);
        v = v - w * k;
      } else {
        v = prm.lo + w * open01(word(rd, j & 3));
      }
    }
    y[j] = v;
  }
}

__global__ void __launch_bounds__(128) k_jde_select(po_jde_params prm, double* __restrict__ pop, double* __restrict__ fit,
                                                    double* __restrict__ fcr, const double* __restrict__ trial,
                                                    const double* __restrict__ tfit, const double* __restrict__ tfcr,
                                                    const uint8_t* __restrict__ mask) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= prm.pop) return;
  if (mask && !mask[i]) return;
  if (tfit[i] >= fit[i]) {
    for (int j = 0; j < prm.dim; ++j) pop[size_t(i) * prm.dim + j] = trial[size_t(i) * prm.dim + j];
    fit[i] = tfit[i];
    fcr[2 * i] = tfcr[2 * i];
    fcr[2 * i + 1] = tfcr[2 * i + 1];
  }
}

// Ring migration in one workgroup: thread k finds the best member of island k and the worst of
// island k + 1 (lowest index on ties) in the state before the call, the moving rows are staged
// in LDS, then written.
__global__ void __launch_bounds__(kMaxIslands) k_island_migrate(po_jde_params prm, double* __restrict__ pop,
                                                               double* __restrict__ fit, double* __restrict__ fcr) {
  __shared__ double stage[kMaxIslands][kMaxMigrateDim + 3];
  __shared__ int dst[kMaxIslands];
  const int K = prm.islands, S = prm.pop / K, D = prm.dim;
  const int k = threadIdx.x;
  if (k < K) {
    int best = k * S;
    for (int i = k * S; i < (k + 1) * S; ++i)
      if (fit[i] > fit[best]) best = i;
    const int k2 = (k + 1) % K;
    int worst = k2 * S;
    for (int i = k2 * S; i < (k2 + 1) * S; ++i)
      if (fit[i] < fit[worst]) worst = i;
    dst[k] = fit[best] > fit[worst] ? worst : -1;
    for (int j = 0; j < D; ++j) stage[k][j] = pop[size_t(best) * D + j];
    stage[k][D] = fit[best];
    stage[k][D + 1] = fcr[2 * best];
    stage[k][D + 2] = fcr[2 * best + 1];
  }
  __syncthreads();
  if (k < K && dst[k] >= 0) {
    const int w = dst[k];
    for (int j = 0; j < D; ++j) pop[size_t(w) * D + j] = stage[k][j];
    fit[w] = stage[k][D];
    fcr[2 * w] = stage[k][D + 1];
    fcr[2 * w + 1] = stage[k][D + 2];
  }
}

}  // namespace

po_status launch_de_propose(const po_de_params& p, int64_t gen, const double* d_pop, double* d_trial, int32_t* d_idx,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_de_propose, dim3((p.pop + 127) / 128), dim3(128), 0, s, p, gen, d_pop, d_trial, d_idx);
  PO_HIP(hipGetLastError());
  return PO_OK;
}

po_status launch_de_select(const po_de_params& p, double* d_pop, double* d_fit, const double* d_trial,
                           const double* d_trial_fit, const uint8_t* d_mask, hipStream_t s) {
  hipLaunchKernelGGL(k_de_select, dim3((p.pop + 127) / 128), dim3(128), 0, s, p, d_pop, d_fit, d_trial, d_trial_fit,
                     d_mask);
  PO_HIP(hipGetLastError());
  return PO_OK;
}

po_status launch_jde_propose(const po_jde_params& p, int64_t gen, const double* d_pop, const double* d_fcr,
                             double* d_trial, double* d_tfcr, int32_t* d_idx, hipStream_t s) {
  hipLaunchKernelGGL(k_jde_propose, dim3((p.pop + 127) / 128), dim3(128), 0, s, p, gen, d_pop, d_fcr, d_trial, d_tfcr,
                     d_idx);
  PO_HIP(hipGetLastError());
  return PO_OK;
}

po_status launch_jde_select(const po_jde_params& p, double* d_pop, double* d_fit, double* d_fcr, const double* d_trial,
                            const double* d_tfit, const double* d_tfcr, const uint8_t* d_mask, hipStream_t s) {
  hipLaunchKernelGGL(k_jde_select, dim3((p.pop + 127) / 128), dim3(128), 0, s, p, d_pop, d_fit, d_fcr, d_trial, d_tfit,
                     d_tfcr, d_mask);
  PO_HIP(hipGetLastError());
  return PO_OK;
}

po_status launch_island_migrate(const po_jde_params& p, double* d_pop, double* d_fit, double* d_fcr, hipStream_t s) {
  hipLaunchKernelGGL(k_island_migrate, dim3(1), dim3(kMaxIslands), 0, s, p, d_pop, d_fit, d_fcr);
  PO_HIP(hipGetLastError());
  return PO_OK;
}

}  // namespace po

using namespace po;

namespace {
__global__ void k_fill(double* __restrict__ dst, int n, double v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = v;
}
// Indices out of [0, n_dst) are skipped (no access outside the destination).
__global__ void k_scatter(const double* __restrict__ vals, const int32_t* __restrict__ idx, int n_idx,
                          double* __restrict__ dst, int n_dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_idx && idx[i] >= 0 && idx[i] < n_dst) dst[idx[i]] = vals[i];
}
}  // namespace

extern "C" {

po_status po_mask_indices(const uint8_t* d_mask, int32_t n, int32_t* d_idx, int32_t* d_count, void* stream) {
  if (n < 1 || n > 8192) return set_error(PO_ERR_INVALID, "n must be in [1, 8192]");
  PO_TRY(check_device_range(d_mask, size_t(n), 1, "d_mask"));
  PO_TRY(check_device_range(d_idx, sizeof(int32_t) * n, 4, "d_idx"));
  if (d_count) PO_TRY(check_device_range(d_count, sizeof(int32_t), 4, "d_count"));
  hipLaunchKernelGGL(k_mask_indices, dim3(1), dim3(1024), 0, static_cast<hipStream_t>(stream), d_mask, n, d_idx,
                     d_count);
  PO_HIP(hipGetLastError());
  return PO_OK;
}

po_status po_gather_rows(const double* d_src, int32_t rows, int32_t cols, const int32_t* d_idx, int32_t n_idx,
                         double* d_dst, void* stream) {
  if (rows < 1 || cols < 1 || n_idx < 1) return set_error(PO_ERR_INVALID, "rows, cols and n_idx must be >= 1");
  PO_TRY(check_device_range(d_src, sizeof(double) * size_t(rows) * cols, 8, "d_src"));
  PO_TRY(check_device_range(d_idx, sizeof(int32_t) * n_idx, 4, "d_idx"));
  PO_TRY(check_device_range(d_dst, sizeof(double) * size_t(n_idx) * cols, 8, "d_dst"));
  const int64_t n = int64_t(n_idx) * cols;
  hipLaunchKernelGGL(k_gather_rows, dim3(int((n + 255) / 256)), dim3(256), 0, static_cast<hipStream_t>(stream), d_src,
                     rows, cols, d_idx, n_idx, d_dst);
  PO_HIP(hipGetLastError());
  return PO_OK;
}

po_status po_scatter_values(const double* d_vals, const int32_t* d_idx, int32_t n_idx, double fill, double* d_dst,
                            int32_t n_dst, void* stream) {
  if (n_idx < 0 || n_dst < 1) return set_error(PO_ERR_INVALID, "need n_idx >= 0 and n_dst >= 1");
  PO_TRY(check_device_range(d_dst, sizeof(double) * n_dst, 8, "d_dst"));
  if (n_idx > 0) {
    PO_TRY(check_device_range(d_vals, sizeof(double) * n_idx, 8, "d_vals"));
    PO_TRY(check_device_range(d_idx, sizeof(int32_t) * n_idx, 4, "d_idx"));
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_fill, dim3((n_dst + 255) / 256), dim3(256), 0, s, d_dst, n_dst, fill);
  PO_HIP(hipGetLastError());
  if (n_idx > 0) {
    hipLaunchKernelGGL(k_scatter, dim3((n_idx + 255) / 256), dim3(256), 0, s, d_vals, d_idx, n_idx, d_dst, n_dst);
    PO_HIP(hipGetLastError());
  }
  return PO_OK;
}

}  // extern "C"
