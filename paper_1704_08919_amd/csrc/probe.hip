// Diagnostics: the FP64 FMA issue rate the device sustains at a given number of waves per SIMD
// and a given number of independent dependency chains per lane -- the ceiling against which the
// evolution kernels' FP64 rates are read.  Not part of the method.
//
// Every lane runs `iters` rounds of CHAINS independent chains a_c <- fma(a_c, x, y) (x, y chosen
// so the values stay bounded), 2 FLOP each, and writes the sum of its chains so nothing is
// removed.  Exactly `waves_per_simd` waves run on every SIMD: the grid holds 256 x waves_per_simd
// workgroups of four waves (one per SIMD), and each workgroup reserves a share of the 160 KiB of
// LDS per CU so that no more than waves_per_simd of them fit on one CU.
#include "common.hpp"

namespace po {
namespace {

constexpr int kLdsPerCu = 160 * 1024;

template <int CHAINS>
__global__ void __launch_bounds__(256) k_fma_probe(int64_t iters, double x, double y, double* __restrict__ sink) {
  extern __shared__ double reserve[];
  double a[CHAINS];
#pragma unroll
  for (int c = 0; c < CHAINS; ++c) a[c] = 1.0 + 1e-3 * (threadIdx.x + c);
  for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int c = 0; c < CHAINS; ++c) a[c] = fma(a[c], x, y);
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < CHAINS; ++c) s += a[c];
  if (threadIdx.x == 0) reserve[0] = s;  // touches the reserved LDS; the value is not used
  sink[int64_t(blockIdx.x) * blockDim.x + threadIdx.x] = s;
}

template <int CHAINS>
po_status launch_probe(int waves_per_simd, int64_t iters, double* d_sink, int n_cu, hipStream_t s) {
  const size_t lds = size_t(kLdsPerCu / waves_per_simd) - 1024;
  hipLaunchKernelGGL(k_fma_probe<CHAINS>, dim3(n_cu * waves_per_simd), dim3(256), lds, s, iters, 0.999999, 1e-6,
                     d_sink);
  PO_HIP(hipGetLastError());
  return PO_OK;
}

}  // namespace
}  // namespace po

using namespace po;

extern "C" {

po_status po_probe_fp64_fma(int32_t waves_per_simd, int32_t chains, int64_t iters, double* d_sink, double* flop,
                            void* stream) {
  if (waves_per_simd < 3 || waves_per_simd > 8) return set_error(PO_ERR_INVALID, "waves_per_simd must be in [3, 8]");
  if (chains != 1 && chains != 2 && chains != 4 && chains != 8)
    return set_error(PO_ERR_INVALID, "chains must be 1, 2, 4 or 8");
  if (iters < 1) return set_error(PO_ERR_INVALID, "iters must be >= 1");
  int dev = -1, n_cu = 0;
  PO_HIP(hipGetDevice(&dev));
  PO_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  PO_TRY(check_device_range(d_sink, sizeof(double) * size_t(n_cu) * waves_per_simd * 256, 8, "d_sink"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  switch (chains) {
    case 1: PO_TRY(launch_probe<1>(waves_per_simd, iters, d_sink, n_cu, s)); break;
    case 2: PO_TRY(launch_probe<2>(waves_per_simd, iters, d_sink, n_cu, s)); break;
    case 4: PO_TRY(launch_probe<4>(waves_per_simd, iters, d_sink, n_cu, s)); break;
    default: PO_TRY(launch_probe<8>(waves_per_simd, iters, d_sink, n_cu, s)); break;
  }
  if (flop) *flop = 2.0 * 8.0 * double(chains) * double(iters) * double(n_cu) * waves_per_simd * 256.0;
  return PO_OK;
}

}  // extern "C"
