// Device helpers shared by the per-mode kernels: fixed-order reductions and the mapping of
// workgroups to work items.  Every sum here has an order that depends only on the sizes of the
// problem, so results do not depend on launch shape or scheduling.
#pragma once

#include "common.hpp"

namespace po {

// Fixed-order sum over the 64 lanes of a wave (butterfly); every lane gets the same value.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Fixed-order tree sum of one value per lane over a 256-lane workgroup.
__device__ __forceinline__ double block_sum256(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int w = 128; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  return red[0];
}

// Pulse owning default-launch item `item` (binary search over the item offsets).
__device__ __forceinline__ int find_pulse_item(const PulseDev* __restrict__ desc, int n, int item) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (desc[mid].item_off <= item) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Workgroup IDs are dispatched round-robin over the 8 XCDs (each with its own L2), so block b runs
// on XCD b % 8.  Give each XCD a contiguous range of items -- whole stretches of one pulse -- so a
// pulse's table is fetched from HBM by one L2 rather than by all eight.  A bijection on [0, n).
__device__ __forceinline__ int xcd_item(int b, int n) {
  constexpr int kXcd = 8;
  const int x = b % kXcd, q = n / kXcd, r = n % kXcd;
  return x * q + min(x, r) + b / kXcd;
}

// Cell-centred momentum of mode m (x fastest): p_d = lo_d + (i_d + 1/2) dp_d.
__device__ __forceinline__ void mode_momentum(const PulseDev& d, int64_t m, double& px, double& py, double& pz) {
  const int nx = d.n[0], ny = d.n[1];
  const int ix = int(m % nx), iy = int((m / nx) % ny), iz = int(m / (int64_t(nx) * ny));
  px = __dadd_rn(d.lo[0], __dmul_rn(double(ix) + 0.5, d.dp[0]));
  py = __dadd_rn(d.lo[1], __dmul_rn(double(iy) + 0.5, d.dp[1]));
  pz = __dadd_rn(d.lo[2], __dmul_rn(double(iz) + 0.5, d.dp[2]));
}

// Writes the 64-mode unit sum of fv (lanes beyond the pulse's modes pass 0).
__device__ __forceinline__ void write_unit(const PulseDev& d, double* __restrict__ units, int64_t lane_mode,
                                           int64_t nmodes, double fv) {
  const double s = wave_sum(fv);
  const int64_t base = lane_mode - (threadIdx.x & 63);
  if ((threadIdx.x & 63) == 0 && base < nmodes) units[d.unit_off + base / kUnit] = s;
}

}  // namespace po
