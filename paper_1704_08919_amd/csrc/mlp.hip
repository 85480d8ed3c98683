// Surrogate MLP on gfx950: BF16 operands on the matrix cores, FP32 accumulation, FP32 master
// weights, Adam.  n_in -> depth x (width, GELU) -> 1; the input is the pulse's coefficient
// vector, the output a standardised log10 pair yield.
//
// Hidden layers are GEMMs on v_mfma_f32_16x16x32_bf16: one wave owns a 16x16 tile of C, each
// lane feeding 8 consecutive-k bf16 values of one A row and one B column per instruction and
// receiving 4 rows of one C column.  Epilogues are fused: bias + GELU + bf16 rounding in the
// forward pass, GELU' in the backward pass.  The 1-wide output layer is a dot product per sample.
// All reductions (bias gradients, loss, output layer) run in a fixed order, so a training step is
// bitwise reproducible.
#include <cmath>
#include <new>
#include <vector>

#include "common.hpp"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

struct po_mlp {
  int n_in = 0, width = 0, depth = 0, max_batch = 0, device = 0;
  int64_t n_params = 0;
  int64_t t = 0;               // Adam steps taken
  float* p = nullptr;          // master parameters, fp32 (layout of the header)
  float* m = nullptr;          // Adam first moment
  float* v = nullptr;          // Adam second moment
  float* g = nullptr;          // last gradient
  __bf16* wb = nullptr;        // bf16 copies of the weight matrices (same offsets as p)
  __bf16* h = nullptr;         // activations [depth + 1][max_batch][max(width, n_in)] bf16
  float* z = nullptr;          // pre-activations [depth][max_batch][width]
  float* dz = nullptr;         // fp32 gradient of a pre-activation, two buffers [2][max_batch][width]
  __bf16* dzb = nullptr;       // their bf16 copies (matrix operands), [2][max_batch][width]
  float* y = nullptr;          // outputs [max_batch]
  float* dy = nullptr;         // dL/dy [max_batch]
  float* loss_parts = nullptr; // per-block partial squared errors
};

namespace po {
namespace {

constexpr int kLossBlocks = 64;

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// C[M][N] += A[M][K] B[K][N] with A(m, k) = A[m sam + k sak], B(k, n) = B[k sbk + n sbn].
// Requires M, N multiples of 16 and K a multiple of 32.  EPI selects the epilogue.
enum { EPI_FWD = 0, EPI_BWD = 1, EPI_WGRAD = 2 };

template <int EPI>
__global__ void __launch_bounds__(256) k_gemm(const __bf16* __restrict__ A, int sam, int sak,
                                              const __bf16* __restrict__ B, int sbk, int sbn, int M, int N, int K,
                                              const float* __restrict__ bias, const float* __restrict__ zin,
                                              float* __restrict__ Cf, __bf16* __restrict__ Cb) {
  const int lane = threadIdx.x & 63;
  const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int tiles_n = N / 16;
  if (tile >= (M / 16) * tiles_n) return;
  const int tm = tile / tiles_n, tn = tile % tiles_n;
  const int arow = tm * 16 + (lane & 15), bcol = tn * 16 + (lane & 15), kq = (lane >> 4) * 8;
  floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = 0; k0 < K; k0 += 32) {
    bf16x8 a, b;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      a[i] = A[size_t(arow) * sam + size_t(k0 + kq + i) * sak];
      b[i] = B[size_t(k0 + kq + i) * sbk + size_t(bcol) * sbn];
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
  }
  const int col = tn * 16 + (lane & 15);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int row = tm * 16 + (lane >> 4) * 4 + i;
    const size_t o = size_t(row) * N + col;
    if constexpr (EPI == EPI_FWD) {
      const float zz = acc[i] + bias[col];
      Cf[o] = zz;
      Cb[o] = __bf16(gelu(zz));
    } else if constexpr (EPI == EPI_BWD) {
      const float d = acc[i] * gelu_grad(zin[o]);
      Cf[o] = d;
      Cb[o] = __bf16(d);
    } else {
      Cf[o] = acc[i];
    }
  }
}

// Input coefficients (double) -> bf16 through float, round to nearest even.
__global__ void k_input(const double* __restrict__ x, int64_t n, __bf16* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = __bf16(float(x[i]));
}

// Master weights -> bf16 copies (weights only; biases are used in fp32).
__global__ void k_weights_to_bf16(const float* __restrict__ p, int64_t n, __bf16* __restrict__ wb) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) wb[i] = __bf16(p[i]);
}

// Output layer: y[b] = sum_j h[b][j] w[j] + b0, one wave per sample, fixed butterfly order.
__global__ void __launch_bounds__(256) k_out_fwd(const __bf16* __restrict__ h, const __bf16* __restrict__ w,
                                                 const float* __restrict__ b0, int width, int batch,
                                                 float* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int s = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (s >= batch) return;
  float acc = 0.0f;
  for (int j = lane; j < width; j += 64) acc = fmaf(float(h[size_t(s) * width + j]), float(w[j]), acc);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) y[s] = acc + b0[0];
}

// dL/dy = 2 (y - t) / B, per-block partial squared errors.
__global__ void __launch_bounds__(256) k_out_loss(const float* __restrict__ y, const float* __restrict__ t, int batch,
                                                  float* __restrict__ dy, float* __restrict__ parts) {
  __shared__ float red[256];
  float sq = 0.0f;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < batch; i += gridDim.x * 256) {
    const float d = y[i] - t[i];
    dy[i] = 2.0f * d / float(batch);
    sq = fmaf(d, d, sq);
  }
  red[threadIdx.x] = sq;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) parts[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_loss_final(const float* __restrict__ parts, int n, int batch,
                                                    float* __restrict__ loss) {
  if (threadIdx.x == 0) {
    float s = 0.0f;
    for (int i = 0; i < n; ++i) s += parts[i];
    *loss = s / float(batch);
  }
}

// Output-layer gradients: gw[j] = sum_b h[b][j] dy[b] (one thread per j, b in order), gb = sum dy;
// and dz[b][j] = dy[b] w[j] gelu'(z[b][j]) for the last hidden layer (fp32 and bf16).
__global__ void __launch_bounds__(256) k_out_bwd(const __bf16* __restrict__ h, const __bf16* __restrict__ w,
                                                 const float* __restrict__ dy, const float* __restrict__ z, int width,
                                                 int batch, float* __restrict__ gw, float* __restrict__ gb,
                                                 float* __restrict__ dz, __bf16* __restrict__ dzb) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j < width) {
    float acc = 0.0f;
    for (int b = 0; b < batch; ++b) acc = fmaf(float(h[size_t(b) * width + j]), dy[b], acc);
    gw[j] = acc;
    const float wj = float(w[j]);
    for (int b = 0; b < batch; ++b) {
      const size_t o = size_t(b) * width + j;
      const float d = dy[b] * wj * gelu_grad(z[o]);
      dz[o] = d;
      dzb[o] = __bf16(d);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    float s = 0.0f;
    for (int b = 0; b < batch; ++b) s += dy[b];
    gb[0] = s;
  }
}

// Bias gradient: column sums of dz over the batch, in batch order.
__global__ void __launch_bounds__(256) k_colsum(const float* __restrict__ dz, int width, int batch,
                                                float* __restrict__ gb) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= width) return;
  float s = 0.0f;
  for (int b = 0; b < batch; ++b) s += dz[size_t(b) * width + j];
  gb[j] = s;
}

__global__ void k_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, int64_t n, float lr, float bc1, float bc2) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + 1e-8f);
}

// Philox4x32-10 (Salmon et al., SC'11) for the initial weights.
__device__ __forceinline__ uint32_t philox_word(uint32_t c0, uint32_t c1, uint32_t k0, uint32_t k1) {
  uint32_t c2 = 0, c3 = 0;
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t m0 = uint64_t(0xD2511F53u) * c0, m1 = uint64_t(0xCD9E8D57u) * c2;
    const uint32_t n0 = uint32_t(m1 >> 32) ^ c1 ^ k0, n2 = uint32_t(m0 >> 32) ^ c3 ^ k1;
    c1 = uint32_t(m1);
    c3 = uint32_t(m0);
    c0 = n0;
    c2 = n2;
  }
  return c0;
}

// Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) for every parameter of a layer (weights and bias).
__global__ void k_init(float* __restrict__ p, int64_t off, int64_t n, float bound, uint64_t seed, uint32_t layer) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t u = philox_word(uint32_t(i), layer, uint32_t(seed), uint32_t(seed >> 32));
  const float r = (float(u) + 0.5f) * (1.0f / 4294967296.0f);
  p[off + i] = bound * (2.0f * r - 1.0f);
}

__global__ void __launch_bounds__(1024) k_topk(const float* __restrict__ s, int n, int k, uint8_t* __restrict__ mask) {
  // rank_i = #{j : s_j > s_i, or s_j == s_i and j < i}; NaN ranks below every number
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const float si = s[i];
    const bool nan_i = si != si;
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const float sj = s[j];
      const bool nan_j = sj != sj;
      bool before;
      if (nan_i) before = !nan_j || j < i;
      else if (nan_j) before = false;
      else before = sj > si || (sj == si && j < i);
      rank += before;
    }
    mask[i] = rank < k ? 1 : 0;
  }
}

__global__ void k_log10_standardize(const double* __restrict__ J, int n, double floor_, double mean, double inv_std,
                                    float* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = float((log10(fmax(J[i], floor_)) - mean) * inv_std);
}

// ------------------------------------------------------------------ layout helpers
int64_t layer_w_off(const po_mlp* a, int l) {
  int64_t o = 0, k = a->n_in;
  for (int i = 0; i < l; ++i) {
    o += k * a->width + a->width;
    k = a->width;
  }
  return o;
}
int64_t layer_k(const po_mlp* a, int l) { return l == 0 ? a->n_in : a->width; }

int blocks(int64_t n, int t = 256) { return int((n + t - 1) / t); }

po_status forward_impl(po_mlp* a, const double* d_x, int B, float* d_y, hipStream_t s) {
  const int W = a->width;
  const int hstride = std::max(a->width, a->n_in);
  hipLaunchKernelGGL(k_input, dim3(blocks(int64_t(B) * a->n_in)), dim3(256), 0, s, d_x, int64_t(B) * a->n_in, a->h);
  PO_HIP(hipGetLastError());
  for (int l = 0; l < a->depth; ++l) {
    const int K = int(layer_k(a, l));
    const int64_t wo = layer_w_off(a, l);
    const __bf16* hin = a->h + size_t(l) * a->max_batch * hstride;
    __bf16* hout = a->h + size_t(l + 1) * a->max_batch * hstride;
    float* z = a->z + size_t(l) * a->max_batch * W;
    const int tiles = (B / 16) * (W / 16);
    hipLaunchKernelGGL(k_gemm<EPI_FWD>, dim3(blocks(tiles, 4)), dim3(256), 0, s, hin, K, 1, a->wb + wo, W, 1, B, W, K,
                       a->p + wo + int64_t(K) * W, nullptr, z, hout);
    PO_HIP(hipGetLastError());
  }
  const int64_t wo = layer_w_off(a, a->depth);
  const __bf16* hl = a->h + size_t(a->depth) * a->max_batch * hstride;
  hipLaunchKernelGGL(k_out_fwd, dim3(blocks(B, 4)), dim3(256), 0, s, hl, a->wb + wo, a->p + wo + W, W, B,
                     d_y ? d_y : a->y);
  PO_HIP(hipGetLastError());
  return PO_OK;
}

po_status grad_impl(po_mlp* a, const double* d_x, const float* d_t, int B, float* d_loss, hipStream_t s) {
  const int W = a->width;
  const int hstride = std::max(a->width, a->n_in);
  PO_TRY(forward_impl(a, d_x, B, a->y, s));
  const int lb = std::min(kLossBlocks, blocks(B));
  hipLaunchKernelGGL(k_out_loss, dim3(lb), dim3(256), 0, s, a->y, d_t, B, a->dy, a->loss_parts);
  PO_HIP(hipGetLastError());
  if (d_loss) {
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, s, a->loss_parts, lb, B, d_loss);
    PO_HIP(hipGetLastError());
  }
  const int D = a->depth;
  const int64_t wo = layer_w_off(a, D);
  const __bf16* hl = a->h + size_t(D) * a->max_batch * hstride;
  const size_t slot = size_t(a->max_batch) * W;
  int cur = 0;
  hipLaunchKernelGGL(k_out_bwd, dim3(blocks(W)), dim3(256), 0, s, hl, a->wb + wo, a->dy,
                     a->z + size_t(D - 1) * a->max_batch * W, W, B, a->g + wo, a->g + wo + W, a->dz, a->dzb);
  PO_HIP(hipGetLastError());
  for (int l = D - 1; l >= 0; --l) {
    const int K = int(layer_k(a, l));
    const int64_t o = layer_w_off(a, l);
    const __bf16* hin = a->h + size_t(l) * a->max_batch * hstride;
    const float* dz = a->dz + cur * slot;
    const __bf16* dzb = a->dzb + cur * slot;
    // dW_l[k][n] = sum_b h_l[b][k] dz[b][n]: A = h_l^T (K x B), B = dz (B x W)
    const int tiles_w = (K / 16) * (W / 16);
    hipLaunchKernelGGL(k_gemm<EPI_WGRAD>, dim3(blocks(tiles_w, 4)), dim3(256), 0, s, hin, 1, K, dzb, W, 1, K, W, B,
                       nullptr, nullptr, a->g + o, nullptr);
    PO_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_colsum, dim3(blocks(W)), dim3(256), 0, s, dz, W, B, a->g + o + int64_t(K) * W);
    PO_HIP(hipGetLastError());
    if (l > 0) {
      // dh_l[b][k] = sum_n dz[b][n] W_l[k][n]: A = dz (B x W), B = W_l^T (W x K); times gelu'(z_{l-1}),
      // written to the other buffer of the pair
      const int tiles_h = (B / 16) * (K / 16);
      hipLaunchKernelGGL(k_gemm<EPI_BWD>, dim3(blocks(tiles_h, 4)), dim3(256), 0, s, dzb, W, 1, a->wb + o, 1, W, B, K, W,
                         nullptr, a->z + size_t(l - 1) * a->max_batch * W, a->dz + (1 - cur) * slot,
                         a->dzb + (1 - cur) * slot);
      PO_HIP(hipGetLastError());
      cur = 1 - cur;
    }
  }
  return PO_OK;
}

po_status adam_impl(po_mlp* a, const float* g, float lr, hipStream_t s) {
  a->t += 1;
  const float bc1 = float(1.0 - std::pow(0.9, double(a->t)));
  const float bc2 = float(1.0 - std::pow(0.999, double(a->t)));
  hipLaunchKernelGGL(k_adam, dim3(blocks(a->n_params)), dim3(256), 0, s, a->p, a->m, a->v, g, a->n_params, lr, bc1, bc2);
  PO_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_weights_to_bf16, dim3(blocks(a->n_params)), dim3(256), 0, s, a->p, a->n_params, a->wb);
  PO_HIP(hipGetLastError());
  return PO_OK;
}

po_status check_batch(const po_mlp* a, int B) {
  if (B < 32 || B > a->max_batch || B % 32) return set_error(PO_ERR_INVALID, "batch must be a multiple of 32 in [32, %d]",
                                                             a->max_batch);
  int dev = -1;
  PO_HIP(hipGetDevice(&dev));
  if (dev != a->device) return set_error(PO_ERR_INVALID, "network lives on device %d, current is %d", a->device, dev);
  return PO_OK;
}

void mlp_free(po_mlp* a) {
  void* bufs[] = {a->p, a->m, a->v, a->g, a->wb, a->h, a->z, a->dz, a->dzb, a->y, a->dy, a->loss_parts};
  for (void* q : bufs)
    if (q) (void)hipFree(q);
}

template <class T>
po_status dalloc(T** out, size_t count) {
  void* q = nullptr;
  PO_HIP(hipMalloc(&q, sizeof(T) * std::max<size_t>(count, 1)));
  *out = static_cast<T*>(q);
  return PO_OK;
}

po_status create_impl(po_mlp* a, uint64_t seed, hipStream_t s) {
  PO_HIP(hipGetDevice(&a->device));
  int64_t np = 0, k = a->n_in;
  for (int l = 0; l < a->depth; ++l) {
    np += k * a->width + a->width;
    k = a->width;
  }
  np += a->width + 1;
  a->n_params = np;
  const int hstride = std::max(a->width, a->n_in);
  PO_TRY(dalloc(&a->p, np));
  PO_TRY(dalloc(&a->m, np));
  PO_TRY(dalloc(&a->v, np));
  PO_TRY(dalloc(&a->g, np));
  PO_TRY(dalloc(&a->wb, np));
  PO_TRY(dalloc(&a->h, size_t(a->depth + 1) * a->max_batch * hstride));
  PO_TRY(dalloc(&a->z, size_t(a->depth) * a->max_batch * a->width));
  PO_TRY(dalloc(&a->dz, 2 * size_t(a->max_batch) * a->width));
  PO_TRY(dalloc(&a->dzb, 2 * size_t(a->max_batch) * a->width));
  PO_TRY(dalloc(&a->y, a->max_batch));
  PO_TRY(dalloc(&a->dy, a->max_batch));
  PO_TRY(dalloc(&a->loss_parts, kLossBlocks));
  PO_HIP(hipMemsetAsync(a->m, 0, sizeof(float) * np, s));
  PO_HIP(hipMemsetAsync(a->v, 0, sizeof(float) * np, s));
  k = a->n_in;
  for (int l = 0; l <= a->depth; ++l) {
    const int64_t kin = (l < a->depth) ? k : a->width;
    const int64_t n = (l < a->depth) ? kin * a->width + a->width : a->width + 1;
    const float bound = float(1.0 / std::sqrt(double(kin)));
    hipLaunchKernelGGL(k_init, dim3(blocks(n)), dim3(256), 0, s, a->p, layer_w_off(a, l), n, bound, seed, uint32_t(l));
    PO_HIP(hipGetLastError());
    k = a->width;
  }
  hipLaunchKernelGGL(k_weights_to_bf16, dim3(blocks(np)), dim3(256), 0, s, a->p, np, a->wb);
  PO_HIP(hipGetLastError());
  PO_HIP(hipStreamSynchronize(s));
  return PO_OK;
}

}  // namespace
}  // namespace po

using namespace po;

extern "C" {

po_status po_mlp_create(int32_t n_in, int32_t width, int32_t depth, int32_t max_batch, uint64_t seed, void* stream,
                        struct po_mlp** out) {
  if (!out) return set_error(PO_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (n_in < 32 || n_in % 32) return set_error(PO_ERR_INVALID, "n_in must be a positive multiple of 32");
  if (width < 32 || width % 32 || width > 4096) return set_error(PO_ERR_INVALID, "width must be a multiple of 32 in [32, 4096]");
  if (depth < 1 || depth > 16) return set_error(PO_ERR_INVALID, "depth must be in [1, 16]");
  if (max_batch < 32 || max_batch % 32 || max_batch > (1 << 20))
    return set_error(PO_ERR_INVALID, "max_batch must be a multiple of 32 in [32, 2^20]");
  po_mlp* a = new (std::nothrow) po_mlp();
  if (!a) return set_error(PO_ERR_NOMEM, "allocation failed");
  a->n_in = n_in;
  a->width = width;
  a->depth = depth;
  a->max_batch = max_batch;
  const po_status st = create_impl(a, seed, static_cast<hipStream_t>(stream));
  if (st != PO_OK) {
    mlp_free(a);
    delete a;
    return st;
  }
  *out = a;
  return PO_OK;
}

int64_t po_mlp_param_count(const struct po_mlp* a) { return a ? a->n_params : -1; }

po_status po_mlp_get_params(const struct po_mlp* a, float* d_params, void* stream) {
  if (!a) return set_error(PO_ERR_INVALID, "network is NULL");
  PO_TRY(check_device_range(d_params, sizeof(float) * a->n_params, 4, "d_params"));
  PO_HIP(hipMemcpyAsync(d_params, a->p, sizeof(float) * a->n_params, hipMemcpyDeviceToDevice,
                        static_cast<hipStream_t>(stream)));
  return PO_OK;
}

po_status po_mlp_set_params(struct po_mlp* a, const float* d_params, void* stream) {
  if (!a) return set_error(PO_ERR_INVALID, "network is NULL");
  PO_TRY(check_device_range(d_params, sizeof(float) * a->n_params, 4, "d_params"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  PO_HIP(hipMemcpyAsync(a->p, d_params, sizeof(float) * a->n_params, hipMemcpyDeviceToDevice, s));
  PO_HIP(hipMemsetAsync(a->m, 0, sizeof(float) * a->n_params, s));
  PO_HIP(hipMemsetAsync(a->v, 0, sizeof(float) * a->n_params, s));
  a->t = 0;
  hipLaunchKernelGGL(k_weights_to_bf16, dim3(blocks(a->n_params)), dim3(256), 0, s, a->p, a->n_params, a->wb);
  PO_HIP(hipGetLastError());
  return PO_OK;
}

po_status po_mlp_forward(struct po_mlp* a, const double* d_x, int32_t batch, float* d_y, void* stream) {
  if (!a) return set_error(PO_ERR_INVALID, "network is NULL");
  PO_TRY(check_batch(a, batch));
  PO_TRY(check_device_range(d_x, sizeof(double) * size_t(batch) * a->n_in, 8, "d_x"));
  PO_TRY(check_device_range(d_y, sizeof(float) * batch, 4, "d_y"));
  return forward_impl(a, d_x, batch, d_y, static_cast<hipStream_t>(stream));
}

po_status po_mlp_loss_grad(struct po_mlp* a, const double* d_x, const float* d_target, int32_t batch, float* d_loss,
                           float* d_grad, void* stream) {
  if (!a) return set_error(PO_ERR_INVALID, "network is NULL");
  PO_TRY(check_batch(a, batch));
  PO_TRY(check_device_range(d_x, sizeof(double) * size_t(batch) * a->n_in, 8, "d_x"));
  PO_TRY(check_device_range(d_target, sizeof(float) * batch, 4, "d_target"));
  if (d_loss) PO_TRY(check_device_range(d_loss, sizeof(float), 4, "d_loss"));
  if (d_grad) PO_TRY(check_device_range(d_grad, sizeof(float) * a->n_params, 4, "d_grad"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  PO_TRY(grad_impl(a, d_x, d_target, batch, d_loss, s));
  if (d_grad) PO_HIP(hipMemcpyAsync(d_grad, a->g, sizeof(float) * a->n_params, hipMemcpyDeviceToDevice, s));
  return PO_OK;
}

po_status po_mlp_adam_step(struct po_mlp* a, const float* d_grad, float lr, void* stream) {
  if (!a) return set_error(PO_ERR_INVALID, "network is NULL");
  if (!(lr >= 0.0f) || !std::isfinite(lr)) return set_error(PO_ERR_INVALID, "lr must be finite and >= 0");
  if (d_grad) PO_TRY(check_device_range(d_grad, sizeof(float) * a->n_params, 4, "d_grad"));
  return adam_impl(a, d_grad ? d_grad : a->g, lr, static_cast<hipStream_t>(stream));
}

po_status po_mlp_train_step(struct po_mlp* a, const double* d_x, const float* d_target, int32_t batch, float lr,
                            float* d_loss, void* stream) {
  PO_TRY(po_mlp_loss_grad(a, d_x, d_target, batch, d_loss, nullptr, stream));
  return po_mlp_adam_step(a, nullptr, lr, stream);
}

void po_mlp_destroy(struct po_mlp* a) {
  if (!a) return;
  (void)hipDeviceSynchronize();
  mlp_free(a);
  delete a;
}

po_status po_topk_mask(const float* d_score, int32_t n, int32_t k, uint8_t* d_mask, void* stream) {
  if (n < 1 || n > 8192) return set_error(PO_ERR_INVALID, "n must be in [1, 8192]");
  if (k < 0 || k > n) return set_error(PO_ERR_INVALID, "k must be in [0, n]");
  PO_TRY(check_device_range(d_score, sizeof(float) * n, 4, "d_score"));
  PO_TRY(check_device_range(d_mask, n, 1, "d_mask"));
  hipLaunchKernelGGL(k_topk, dim3(1), dim3(1024), 0, static_cast<hipStream_t>(stream), d_score, n, k, d_mask);
  PO_HIP(hipGetLastError());
  return PO_OK;
}

po_status po_log10_standardize(const double* d_J, int32_t n, double floor_value, double mean, double inv_std,
                               float* d_out, void* stream) {
  if (n < 1) return set_error(PO_ERR_INVALID, "n must be >= 1");
  if (!(floor_value > 0.0)) return set_error(PO_ERR_INVALID, "floor must be > 0");
  PO_TRY(check_device_range(d_J, sizeof(double) * n, 8, "d_J"));
  PO_TRY(check_device_range(d_out, sizeof(float) * n, 4, "d_out"));
  hipLaunchKernelGGL(k_log10_standardize, dim3(blocks(n)), dim3(256), 0, static_cast<hipStream_t>(stream), d_J, n,
                     floor_value, mean, inv_std, d_out);
  PO_HIP(hipGetLastError());
  return PO_OK;
}

}  // extern "C"
