// Surrogate MLP on gfx950: BF16 operands on the matrix cores, FP32 accumulation, FP32 master
// weights, Adam.  n_in -> depth x (width, GELU) -> 1; the input is the pulse's coefficient
// vector, the output a standardised log10 pair yield.
//
// Every matrix product is C[m][n] = sum_k A[m][k] Bt[n][k] with both operands contiguous in k, so
// each lane of a v_mfma_f32_16x16x32_bf16 fetches its 8 consecutive-k values of one A row and one
// B column with one 16-byte load, straight from L2 (every operand of a step, ~1 MB, stays there).
// One wave owns a 32x32 tile of C (2 x 2 MFMA tiles: each fragment feeds two instructions); four
// independent waves per workgroup.  The layouts that make k contiguous are produced by the
// epilogues that write the operands: the forward pass writes every hidden activation both
// row-major ([batch][width], the next layer's A) and transposed ([width][batch], the A of the
// weight gradient); the backward pass writes each pre-activation gradient row-major (A of the
// next input gradient) and transposed (Bt of the weight gradient); the optimiser keeps every
// weight matrix in bf16 both as W[k_in][width] (Bt of the input gradient) and as W^T (Bt of the
// forward product).  Weight gradients (k = batch) are split over k into fixed partial sums that
// the optimiser adds in order, bias gradients are column sums per 32-row tile fused into the
// epilogue that produces the pre-activation gradient, and the output layer (a dot product per
// sample), the loss, dL/dy and the last hidden layer's gradient are one kernel, and the weight
// gradient of a layer shares a launch with the input gradient of the layer below (the transposed
// gradients alternate between two buffers).  A training step is 9 launches, captured once into a
// HIP graph and replayed; every reduction has a fixed order, so a step is bitwise reproducible.
//
// Rounding points (the oracle emulates them): the input is rounded to bf16 through float, every
// weight matrix used as an operand, every hidden activation gelu(z) and every pre-activation
// gradient used as an operand are bf16; biases, pre-activations, GELU derivatives, weight and bias
// gradients and the optimiser state are fp32.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <type_traits>

#include "common.hpp"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

namespace po {
namespace {

constexpr int kTile = 32;      // C tile per wave (rows and columns)
constexpr int kMaxSplit = 4;   // k-splits of the weight-gradient products

// Device-side counters of a network: the Adam step, its bias corrections and the batch cursor of
// indexed training (which minibatch of the index array the next step reads).
struct Counters {
  long long t;
  float bc1, bc2;
  int cursor;
  int pad;
};

}  // namespace
}  // namespace po

struct po_mlp {
  int n_in = 0, width = 0, depth = 0, max_batch = 0, device = 0;
  int64_t n_params = 0;
  float* p = nullptr;          // master parameters, fp32 (layout of the header)
  float* m = nullptr;          // Adam first moment
  float* v = nullptr;          // Adam second moment
  float* g = nullptr;          // last assembled gradient
  __bf16* wb = nullptr;        // bf16 weights, W_l[k][n] at the parameter offsets
  __bf16* wt = nullptr;        // bf16 transposed weights, W_l^T[n][k] at the same offsets
  __bf16* h = nullptr;         // activations h_1..h_depth [depth][max_batch][width] bf16
  __bf16* hT = nullptr;        // transposed h_0 (the input)..h_{depth-1} [depth][hstride][max_batch]
  float* gp = nullptr;         // gelu'(z_l) [depth][max_batch][width] fp32
  __bf16* dz = nullptr;        // pre-activation gradients [2][max_batch][width] bf16 (ping-pong)
  __bf16* dzT = nullptr;       // transposed [2][width][max_batch] bf16 (ping-pong)
  float* y = nullptr;          // outputs [max_batch]
  float* wpart = nullptr;      // weight-gradient partials, per layer [kMaxSplit][k_in][width]
  float* bpart = nullptr;      // bias-gradient partials, per layer [max_batch / 32][width]
  float* opart = nullptr;      // output layer partials [max_batch / 32][width + 2] (w, b, loss)
  po::Counters* ctr = nullptr; // device counters
  hipStream_t cap = nullptr;   // capture stream
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // the captured step's arguments
  const void* key_x = nullptr;
  const void* key_t = nullptr;
  const void* key_J = nullptr;
  const void* key_idx = nullptr;
  const void* key_loss = nullptr;
  int key_batch = 0, key_rows = 0;
  float key_lr = 0.0f;
  double key_mean = 0.0, key_istd = 0.0;
};

namespace po {
namespace {

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

enum Epi { EPI_FWD = 0, EPI_FWD_TRAIN = 1, EPI_BWD = 2, EPI_PART = 3 };

// Row map of indexed training: row m of a minibatch is row idx[cursor * batch + m] of the data
// (rows outside [0, n_rows) read row 0).
struct RowMap {
  const int* idx;
  const Counters* ctr;
  int batch, n_rows;
  __device__ __forceinline__ int row(int m) const {
    if (!idx) return m;
    const int r = idx[int64_t(ctr->cursor) * batch + m];
    return (r >= 0 && r < n_rows) ? r : 0;
  }
};

struct MMArgs {
  const void* A;      // A[m][k] (bf16, or double rounded to bf16 through float), row stride lda
  int lda;
  RowMap rows;        // rows of A (double input only)
  const __bf16* Bt;   // Bt[n][k], row stride ldb
  int ldb;
  int M, N, K, splits;
  const float* bias;  // [N] (forward)
  const float* gp_in; // [M][N] gelu' of the layer below (backward)
  float* gp_out;      // [M][N] gelu'(z) (forward, training)
  __bf16* C;          // row-major bf16 output [M][N] or NULL
  __bf16* CT;         // transposed bf16 output [N][ldct] or NULL
  int ldct;
  float* part;        // EPI_PART: [splits][M][N]; EPI_BWD: column sums per 32-row tile [M / 32][N]
  __bf16* AT;         // double input: its bf16 transpose [K][ldat], written by the tiles of column 0
  int ldat;
};

__device__ __forceinline__ bf16x8 load8(const __bf16* p) { return *reinterpret_cast<const bf16x8*>(p); }

__device__ __forceinline__ bf16x8 load8(const double* p) {
  bf16x8 r;
  const double2* q = reinterpret_cast<const double2*>(p);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double2 d = q[i];
    r[2 * i] = __bf16(float(d.x));
    r[2 * i + 1] = __bf16(float(d.y));
  }
  return r;
}

// C = A Bt^T for one 32x32 tile per wave; EPI selects what the tile writes.  `block` is the
// workgroup's index within this product.
template <class TA, int EPI>
__device__ __forceinline__ void mm_body(const MMArgs& a, int block) {
  const int lane = threadIdx.x & 63;
  const int tm_n = a.M / kTile, tn_n = a.N / kTile;
  const int w = block * 4 + (threadIdx.x >> 6);
  if (w >= tm_n * tn_n * a.splits) return;
  const int split = w / (tm_n * tn_n);
  const int tt = w - split * tm_n * tn_n;
  const int tm = tt / tn_n, tn = tt - tm * tn_n;
  const int kc = a.K / a.splits;
  const int k_beg = split * kc, k_end = k_beg + kc;
  const int r16 = lane & 15, kq = (lane >> 4) * 8;
  const TA* A = static_cast<const TA*>(a.A);
  int arow[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int m = tm * kTile + i * 16 + r16;
    arow[i] = std::is_same<TA, double>::value ? a.rows.row(m) : m;
  }
  floatx4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
  // k-steps in groups of four: the group's operands are all loaded before its products, so the
  // loads of a group are in flight together (the products still run in k order)
  for (int kb = k_beg; kb < k_end; kb += 4 * 32) {
    bf16x8 af[4][2], bf[4][2];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k0 = kb + 32 * u;
      if (k0 < k_end) {
#pragma unroll
        for (int i = 0; i < 2; ++i) af[u][i] = load8(A + size_t(arow[i]) * a.lda + k0 + kq);
#pragma unroll
        for (int j = 0; j < 2; ++j) bf[u][j] = load8(a.Bt + size_t(tn * kTile + j * 16 + r16) * a.ldb + k0 + kq);
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k0 = kb + 32 * u;
      if (k0 < k_end) {
        if constexpr (std::is_same<TA, double>::value) {
          if (a.AT && tn == 0) {
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
              for (int e = 0; e < 8; ++e) a.AT[size_t(k0 + kq + e) * a.ldat + tm * kTile + i * 16 + r16] = af[u][i][e];
          }
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[u][i], bf[u][j], acc[i][j], 0, 0, 0);
      }
    }
  }
  // lane holds rows tm*32 + i*16 + (lane >> 4)*4 + r, r = 0..3, of column tn*32 + j*16 + (lane & 15)
  const int rq = (lane >> 4) * 4;
  // every value the epilogue reads is loaded before its first store (the stores could alias them)
  float pre[2][2][4];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int n = tn * kTile + j * 16 + r16;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if constexpr (EPI == EPI_FWD || EPI == EPI_FWD_TRAIN) {
          pre[j][i][r] = (i == 0 && r == 0) ? a.bias[n] : 0.0f;
        } else if constexpr (EPI == EPI_BWD) {
          pre[j][i][r] = a.gp_in[size_t(tm * kTile + i * 16 + rq + r) * a.N + n];
        } else {
          pre[j][i][r] = 0.0f;
        }
      }
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int n = tn * kTile + j * 16 + r16;
    float colsum = 0.0f;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int m0 = tm * kTile + i * 16 + rq;
      bf16x4 t4;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + r;
        const size_t o = size_t(m) * a.N + n;
        const float c = acc[i][j][r];
        if constexpr (EPI == EPI_FWD || EPI == EPI_FWD_TRAIN) {
          const float z = c + pre[j][0][0];
          const __bf16 hb = __bf16(gelu(z));
          a.C[o] = hb;
          if constexpr (EPI == EPI_FWD_TRAIN) {
            a.gp_out[o] = gelu_grad(z);
            t4[r] = hb;
          }
        } else if constexpr (EPI == EPI_BWD) {
          const float d = c * pre[j][i][r];
          const __bf16 db = __bf16(d);
          if (a.C) a.C[o] = db;
          t4[r] = db;
          colsum += d;
        } else {
          a.part[size_t(split) * a.M * a.N + o] = c;
        }
      }
      if constexpr (EPI == EPI_FWD_TRAIN || EPI == EPI_BWD) {
        if (a.CT) *reinterpret_cast<bf16x4*>(a.CT + size_t(n) * a.ldct + m0) = t4;
      }
    }
    if constexpr (EPI == EPI_BWD) {
      // column sum over the tile's 32 rows: lanes n, n + 16, n + 32, n + 48 hold 8 rows each
      colsum += __shfl_xor(colsum, 16, 64);
      colsum += __shfl_xor(colsum, 32, 64);
      if (lane < 16) a.part[size_t(tm) * a.N + n] = colsum;
    }
  }
}

template <class TA, int EPI>
__global__ void __launch_bounds__(256) k_mm(MMArgs a) {
  mm_body<TA, EPI>(a, blockIdx.x);
}

// Two independent products in one launch: workgroups [0, nb1) do the first, the rest the second.
template <class TA1, int EPI1, class TA2, int EPI2>
__global__ void __launch_bounds__(256) k_mm2(MMArgs a1, int nb1, MMArgs a2) {
  if (int(blockIdx.x) < nb1)
    mm_body<TA1, EPI1>(a1, blockIdx.x);
  else
    mm_body<TA2, EPI2>(a2, int(blockIdx.x) - nb1);
}

// Output layer and loss of a training step, one workgroup per 32 samples b0..b0+31:
// y = h w + b0, t the target (given, or the standardised log10 J of the sample's data row),
// dy = 2 (y - t) / B; dz = dy w gelu'(z) of the last hidden layer (bf16 row-major and transposed);
// per-workgroup partial sums (in sample order) of dL/dw = h dy, of the last layer's bias gradient
// sum dz, of dL/db = sum dy and of the squared error.
struct OutArgs {
  const __bf16* h;    // [B][W] last hidden activations
  const __bf16* w;    // [W] output weights (bf16)
  const float* b0;    // [1] output bias
  const float* gp;    // [B][W] gelu' of the last hidden layer
  const float* target;  // [B] or NULL
  const double* J;    // data yields (indexed training) or NULL
  RowMap rows;
  double mean, inv_std;
  int W, B;
  float* y;
  __bf16* dz;         // [B][W]
  __bf16* dzT;        // [W][ldt]
  int ldt;
  float* bpart;       // [B / 32][W] bias partials of the last hidden layer
  float* opart;       // [B / 32][W + 2]: dL/dw partials, then dL/db, squared error
};

// Output layer, loss, dL/dy and the last hidden layer's gradient for 32 samples per workgroup.
// y[b] = sum_j h[b][j] w[j] is summed in one fixed grouping: partial p_l over the columns
// l, l + 64, ... for l = 0..63, then pairwise p_l + p_(l^32), ^16, ^8, ^4, ^2, ^1.  A wave does its
// 8 samples at once with 8 lanes per sample: lane `part` of a sample holds the partials of
// l = 8 part + e (e = 0..7, one 16-byte load per 64 columns), combines l^32, ^16, ^8 across the
// sample's lanes and l^4, ^2, ^1 in its registers.
__global__ void __launch_bounds__(256) k_out_train(OutArgs a) {
  __shared__ float s_dy[32], s_sq[32];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int b0 = blockIdx.x * 32;
  {
    const int g = lane >> 3, part = lane & 7;
    const int b = b0 + wv * 8 + g;
    float p[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) p[e] = 0.0f;
    for (int j0 = 8 * part; j0 < a.W; j0 += 64) {
      const bf16x8 hv = load8(a.h + size_t(b) * a.W + j0);
      const bf16x8 wv8 = load8(a.w + j0);
#pragma unroll
      for (int e = 0; e < 8; ++e) p[e] = fmaf(float(hv[e]), float(wv8[e]), p[e]);
    }
#pragma unroll
    for (int off = 4; off > 0; off >>= 1)  // l ^ 32, l ^ 16, l ^ 8
#pragma unroll
      for (int e = 0; e < 8; ++e) p[e] += __shfl_xor(p[e], off, 64);
#pragma unroll
    for (int off = 4; off > 0; off >>= 1) {  // l ^ 4, l ^ 2, l ^ 1
      float q[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) q[e] = p[e] + p[e ^ off];
#pragma unroll
      for (int e = 0; e < 8; ++e) p[e] = q[e];
    }
    if (part == 0) {
      const float yb = p[0] + a.b0[0];
      a.y[b] = yb;
      float t;
      if (a.J) {
        const double Jv = a.J[a.rows.row(b)];
        t = float((log10(fmax(Jv, 1e-300)) - a.mean) * a.inv_std);
      } else {
        t = a.target[b];
      }
      const float d = yb - t;
      s_dy[wv * 8 + g] = 2.0f * d / float(a.B);
      s_sq[wv * 8 + g] = d * d;
    }
  }
  __syncthreads();
  // one column per thread: its 32 rows are read before anything is written
  for (int j = threadIdx.x; j < a.W; j += 256) {
    const float wj = float(a.w[j]);
    float gv[32], hv[32];
#pragma unroll
    for (int r = 0; r < 32; ++r) {
      const size_t o = size_t(b0 + r) * a.W + j;
      gv[r] = a.gp[o];
      hv[r] = float(a.h[o]);
    }
    float sb = 0.0f, sw = 0.0f;
#pragma unroll
    for (int r = 0; r < 32; r += 4) {
      bf16x4 t4;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const size_t o = size_t(b0 + r + e) * a.W + j;
        const float d = s_dy[r + e] * wj * gv[r + e];
        const __bf16 db = __bf16(d);
        a.dz[o] = db;
        t4[e] = db;
        sb += d;
        sw = fmaf(hv[r + e], s_dy[r + e], sw);
      }
      *reinterpret_cast<bf16x4*>(a.dzT + size_t(j) * a.ldt + b0 + r) = t4;
    }
    a.bpart[size_t(blockIdx.x) * a.W + j] = sb;
    a.opart[size_t(blockIdx.x) * (a.W + 2) + j] = sw;
  }
  if (threadIdx.x == 0) {
    float sd = 0.0f, sq = 0.0f;
    for (int r = 0; r < 32; ++r) {
      sd += s_dy[r];
      sq += s_sq[r];
    }
    a.opart[size_t(blockIdx.x) * (a.W + 2) + a.W] = sd;
    a.opart[size_t(blockIdx.x) * (a.W + 2) + a.W + 1] = sq;
  }
}

// Output layer for inference: y[b] = sum_j h[b][j] w[j] + b0, one wave per sample.
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

// Where parameter i lives: hidden layer l weight (k, n) or bias n, or the output layer.
struct ParamMap {
  int n_in, width, depth, splits, nblk, batch;
  int64_t n_params;
  const float* wpart;  // per layer [kMaxSplit][k_in][width]
  const float* bpart;  // per layer [max_batch / 32][width]
  const float* opart;  // [max_batch / 32][width + 2]
  int64_t bpart_stride;  // max_batch / 32 * width
};

__device__ __forceinline__ int64_t wpart_off(const ParamMap& q, int l) {
  return l == 0 ? 0 : int64_t(kMaxSplit) * q.n_in * q.width + int64_t(l - 1) * kMaxSplit * q.width * q.width;
}

// Gradient of parameter i: its partial sums added in a fixed order (the loops are unrolled so that
// their loads are in flight together; the additions stay in order).
__device__ __forceinline__ float assembled_grad(const ParamMap& q, int64_t i) {
  int64_t off = 0;
  int kin = q.n_in;
  for (int l = 0; l < q.depth; ++l) {
    const int64_t nw = int64_t(kin) * q.width;
    if (i < off + nw) {
      const int64_t e = i - off;
      const float* pp = q.wpart + wpart_off(q, l);
      float s = 0.0f;
#pragma unroll 4
      for (int sp = 0; sp < q.splits; ++sp) s += pp[sp * nw + e];
      return s;
    }
    if (i < off + nw + q.width) {
      const int n = int(i - off - nw);
      const float* bp = q.bpart + l * q.bpart_stride;
      float s = 0.0f;
#pragma unroll 8
      for (int t = 0; t < q.nblk; ++t) s += bp[int64_t(t) * q.width + n];
      return s;
    }
    off += nw + q.width;
    kin = q.width;
  }
  const int j = int(i - off);  // 0..width-1: output weights; width: output bias
  float s = 0.0f;
#pragma unroll 8
  for (int t = 0; t < q.nblk; ++t) s += q.opart[int64_t(t) * (q.width + 2) + j];
  return s;
}

// Transposed position of parameter i (weights of a hidden layer; others map to themselves).
__device__ __forceinline__ int64_t transposed_index(const ParamMap& q, int64_t i) {
  int64_t off = 0;
  int kin = q.n_in;
  for (int l = 0; l < q.depth; ++l) {
    const int64_t nw = int64_t(kin) * q.width;
    if (i < off + nw) {
      const int64_t e = i - off;
      const int64_t k = e / q.width, n = e - k * q.width;
      return off + n * kin + k;
    }
    if (i < off + nw + q.width) return i;  // the layer's bias
    off += nw + q.width;
    kin = q.width;
  }
  return i;
}

// Starts an optimiser step: t += 1 and its bias corrections; advances the indexed-training cursor.
__global__ void k_adam_begin(Counters* c) {
  const long long t = c->t + 1;
  c->t = t;
  c->bc1 = float(1.0 - pow(0.9, double(t)));
  c->bc2 = float(1.0 - pow(0.999, double(t)));
  c->cursor += 1;
}

// Assembles the gradient (from the partials, or takes g_in), then Adam and the bf16 copies.
// Thread 0 of block 0 also writes the loss of the step (sum of the squared-error partials / B).
__global__ void __launch_bounds__(256) k_adam(ParamMap q, const float* __restrict__ g_in, float* __restrict__ p,
                                              float* __restrict__ m, float* __restrict__ v, float* __restrict__ g_out,
                                              __bf16* __restrict__ wb, __bf16* __restrict__ wt, float lr,
                                              const Counters* __restrict__ c, float* __restrict__ loss,
                                              int loss_by_cursor) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i == 0 && loss) {
    float s = 0.0f;
#pragma unroll 8
    for (int t = 0; t < q.nblk; ++t) s += q.opart[int64_t(t) * (q.width + 2) + q.width + 1];
    loss[loss_by_cursor ? c->cursor - 1 : 0] = s / float(q.batch);
  }
  if (i >= q.n_params) return;
  const float gi = g_in ? g_in[i] : assembled_grad(q, i);
  if (g_out) g_out[i] = gi;
  if (lr < 0.0f) return;  // gradient only
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / c->bc1) / (sqrtf(vi / c->bc2) + 1e-8f);
  p[i] = pi;
  const __bf16 pb = __bf16(pi);
  wb[i] = pb;
  wt[transposed_index(q, i)] = pb;
}

// Master weights -> bf16 copies, row-major and transposed.
__global__ void k_weights_to_bf16(ParamMap q, const float* __restrict__ p, __bf16* __restrict__ wb,
                                  __bf16* __restrict__ wt) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= q.n_params) return;
  const __bf16 pb = __bf16(p[i]);
  wb[i] = pb;
  wt[transposed_index(q, i)] = pb;
}

__global__ void k_reset_counters(Counters* c, int reset_t) {
  if (reset_t) {
    c->t = 0;
    c->bc1 = c->bc2 = 1.0f;
  }
  c->cursor = 0;
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
int layer_k(const po_mlp* a, int l) { return l == 0 ? a->n_in : a->width; }
int hstride(const po_mlp* a) { return std::max(a->width, a->n_in); }
int blocks(int64_t n, int t = 256) { return int((n + t - 1) / t); }

int splits_for(int B) {
  const int kt = B / 32;
  return kt % 4 == 0 ? 4 : (kt % 2 == 0 ? 2 : 1);
}

ParamMap param_map(const po_mlp* a, int B) {
  ParamMap q;
  q.n_in = a->n_in;
  q.width = a->width;
  q.depth = a->depth;
  q.splits = splits_for(B);
  q.nblk = B / 32;
  q.batch = B;
  q.n_params = a->n_params;
  q.wpart = a->wpart;
  q.bpart = a->bpart;
  q.opart = a->opart;
  q.bpart_stride = int64_t(a->max_batch / 32) * a->width;
  return q;
}

int64_t wpart_offset(const po_mlp* a, int l) {
  return l == 0 ? 0 : int64_t(kMaxSplit) * a->n_in * a->width + int64_t(l - 1) * kMaxSplit * a->width * a->width;
}

template <class TA, int EPI>
po_status launch_mm(const MMArgs& m, hipStream_t s) {
  const int waves = (m.M / kTile) * (m.N / kTile) * m.splits;
  hipLaunchKernelGGL((k_mm<TA, EPI>), dim3(blocks(waves, 4)), dim3(256), 0, s, m);
  PO_HIP(hipGetLastError());
  return PO_OK;
}

int mm_blocks(const MMArgs& m) { return blocks(int64_t(m.M / kTile) * (m.N / kTile) * m.splits, 4); }

template <class TA1, int EPI1, class TA2, int EPI2>
po_status launch_mm2(const MMArgs& m1, const MMArgs& m2, hipStream_t s) {
  const int nb1 = mm_blocks(m1);
  hipLaunchKernelGGL((k_mm2<TA1, EPI1, TA2, EPI2>), dim3(nb1 + mm_blocks(m2)), dim3(256), 0, s, m1, nb1, m2);
  PO_HIP(hipGetLastError());
  return PO_OK;
}

MMArgs mm_base() {
  MMArgs m;
  std::memset(&m, 0, sizeof m);
  m.splits = 1;
  return m;
}

// Forward pass through the hidden layers.  train: also gelu' and the transposed activations.
po_status hidden_forward(po_mlp* a, const double* d_x, RowMap rows, int B, bool train, hipStream_t s) {
  const int W = a->width, hs = hstride(a);
  for (int l = 0; l < a->depth; ++l) {
    const int K = layer_k(a, l);
    const int64_t wo = layer_w_off(a, l);
    MMArgs m = mm_base();
    m.lda = K;
    m.Bt = a->wt + wo;
    m.ldb = K;
    m.M = B;
    m.N = W;
    m.K = K;
    m.bias = a->p + wo + int64_t(K) * W;
    m.C = a->h + size_t(l) * a->max_batch * W;
    if (train) {
      m.gp_out = a->gp + size_t(l) * a->max_batch * W;
      m.CT = l + 1 < a->depth ? a->hT + size_t(l + 1) * hs * a->max_batch : nullptr;
      m.ldct = a->max_batch;
    }
    if (l == 0) {
      m.A = d_x;
      m.rows = rows;
      if (train) {
        m.AT = a->hT;
        m.ldat = a->max_batch;
      }
      PO_TRY((train ? launch_mm<double, EPI_FWD_TRAIN>(m, s) : launch_mm<double, EPI_FWD>(m, s)));
    } else {
      m.A = a->h + size_t(l - 1) * a->max_batch * W;
      PO_TRY((train ? launch_mm<__bf16, EPI_FWD_TRAIN>(m, s) : launch_mm<__bf16, EPI_FWD>(m, s)));
    }
  }
  return PO_OK;
}

po_status forward_impl(po_mlp* a, const double* d_x, int B, float* d_y, hipStream_t s) {
  RowMap rows{nullptr, nullptr, B, B};
  PO_TRY(hidden_forward(a, d_x, rows, B, false, s));
  const int64_t wo = layer_w_off(a, a->depth);
  hipLaunchKernelGGL(k_out_fwd, dim3(blocks(B, 4)), dim3(256), 0, s, a->h + size_t(a->depth - 1) * a->max_batch * a->width,
                     a->wb + wo, a->p + wo + a->width, a->width, B, d_y);
  PO_HIP(hipGetLastError());
  return PO_OK;
}

// Forward and backward pass of one minibatch: fills the gradient partials and the loss partials.
// Targets: d_t[b], or (d_J != NULL) the standardised log10 of the yield of the sample's data row.
po_status grad_impl(po_mlp* a, const double* d_x, RowMap rows, const float* d_t, const double* d_J, double mean,
                    double inv_std, int B, hipStream_t s) {
  const int W = a->width, D = a->depth, hs = hstride(a);
  const int S = splits_for(B);
  PO_TRY(hidden_forward(a, d_x, rows, B, true, s));
  const size_t slot = size_t(a->max_batch) * W;
  OutArgs o;
  std::memset(&o, 0, sizeof o);
  const int64_t wo = layer_w_off(a, D);
  o.h = a->h + size_t(D - 1) * slot;
  o.w = a->wb + wo;
  o.b0 = a->p + wo + W;
  o.gp = a->gp + size_t(D - 1) * slot;
  o.target = d_t;
  o.J = d_J;
  o.rows = rows;
  o.mean = mean;
  o.inv_std = inv_std;
  o.W = W;
  o.B = B;
  o.y = a->y;
  o.dz = a->dz;
  o.dzT = a->dzT;
  o.ldt = a->max_batch;
  o.bpart = a->bpart + size_t(D - 1) * (a->max_batch / 32) * W;
  o.opart = a->opart;
  hipLaunchKernelGGL(k_out_train, dim3(B / 32), dim3(256), 0, s, o);
  PO_HIP(hipGetLastError());
  // dz_l row-major in dz[cur], transposed in dzT[cur]; the weight gradient of layer l and the
  // gradient of layer l - 1 only read them, so both products run in one launch and the latter
  // writes the other buffers.
  const size_t tslot = size_t(W) * a->max_batch;
  int cur = 0;
  for (int l = D - 1; l >= 0; --l) {
    const int K = layer_k(a, l);
    const int64_t off = layer_w_off(a, l);
    // dW_l[k][n] = sum_b h_l[b][k] dz_l[b][n]: A = h_l^T [K][B], Bt = dz_l^T [W][B], split over b
    MMArgs g = mm_base();
    g.A = a->hT + size_t(l) * hs * a->max_batch;
    g.lda = a->max_batch;
    g.Bt = a->dzT + cur * tslot;
    g.ldb = a->max_batch;
    g.M = K;
    g.N = W;
    g.K = B;
    g.splits = S;
    g.part = a->wpart + wpart_offset(a, l);
    if (l > 0) {
      // dh_{l}[b][k] = sum_n dz_l[b][n] W_l[k][n]: A = dz_l [B][W], Bt = W_l [K][W]; times gelu'(z_{l-1})
      MMArgs d = mm_base();
      d.A = a->dz + cur * slot;
      d.lda = W;
      d.Bt = a->wb + off;
      d.ldb = W;
      d.M = B;
      d.N = K;
      d.K = W;
      d.gp_in = a->gp + size_t(l - 1) * slot;
      d.C = l - 1 > 0 ? a->dz + (1 - cur) * slot : nullptr;
      d.CT = a->dzT + (1 - cur) * tslot;
      d.ldct = a->max_batch;
      d.part = a->bpart + size_t(l - 1) * (a->max_batch / 32) * W;
      PO_TRY((launch_mm2<__bf16, EPI_PART, __bf16, EPI_BWD>(g, d, s)));
      cur = 1 - cur;
    } else {
      PO_TRY((launch_mm<__bf16, EPI_PART>(g, s)));
    }
  }
  return PO_OK;
}

po_status adam_launch(po_mlp* a, int B, const float* g_in, float* g_out, float lr, float* loss, int loss_by_cursor,
                      hipStream_t s) {
  if (lr >= 0.0f) {
    hipLaunchKernelGGL(k_adam_begin, dim3(1), dim3(1), 0, s, a->ctr);
    PO_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_adam, dim3(blocks(a->n_params)), dim3(256), 0, s, param_map(a, B), g_in, a->p, a->m, a->v, g_out,
                     a->wb, a->wt, lr, a->ctr, loss, loss_by_cursor);
  PO_HIP(hipGetLastError());
  return PO_OK;
}

// Captures one training step (forward, backward, optimiser) with the given arguments unless the
// graph already holds them, then replays it `steps` times on stream s.
po_status train_replay(po_mlp* a, const double* d_x, const float* d_t, const double* d_J, const int* d_idx, int n_rows,
                       double mean, double inv_std, int B, float lr, float* d_loss, int steps, hipStream_t s) {
  const bool same = a->exec && a->key_x == d_x && a->key_t == d_t && a->key_J == d_J && a->key_idx == d_idx &&
                    a->key_loss == d_loss && a->key_batch == B && a->key_rows == n_rows && a->key_lr == lr &&
                    a->key_mean == mean && a->key_istd == inv_std;
  if (!same) {
    if (a->exec) (void)hipGraphExecDestroy(a->exec);
    if (a->graph) (void)hipGraphDestroy(a->graph);
    a->exec = nullptr;
    a->graph = nullptr;
    PO_HIP(hipStreamBeginCapture(a->cap, hipStreamCaptureModeThreadLocal));
    RowMap rows{d_idx, a->ctr, B, n_rows};
    po_status st = grad_impl(a, d_x, rows, d_t, d_J, mean, inv_std, B, a->cap);
    if (st == PO_OK) st = adam_launch(a, B, nullptr, a->g, lr, d_loss, d_idx ? 1 : 0, a->cap);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(a->cap, &g);
    if (st != PO_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return device_error(e, "hipStreamEndCapture");
    a->graph = g;
    PO_HIP(hipGraphInstantiate(&a->exec, a->graph, nullptr, nullptr, 0));
    a->key_x = d_x;
    a->key_t = d_t;
    a->key_J = d_J;
    a->key_idx = d_idx;
    a->key_loss = d_loss;
    a->key_batch = B;
    a->key_rows = n_rows;
    a->key_lr = lr;
    a->key_mean = mean;
    a->key_istd = inv_std;
  }
  for (int i = 0; i < steps; ++i) PO_HIP(hipGraphLaunch(a->exec, s));
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
  if (a->exec) (void)hipGraphExecDestroy(a->exec);
  if (a->graph) (void)hipGraphDestroy(a->graph);
  if (a->cap) (void)hipStreamDestroy(a->cap);
  void* bufs[] = {a->p,  a->m, a->v,     a->g,     a->wb,    a->wt,    a->h,  a->hT,
                  a->gp, a->dz, a->dzT,  a->y,     a->wpart, a->bpart, a->opart, a->ctr};
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
  const int W = a->width, hs = hstride(a), MB = a->max_batch;
  PO_TRY(dalloc(&a->p, np));
  PO_TRY(dalloc(&a->m, np));
  PO_TRY(dalloc(&a->v, np));
  PO_TRY(dalloc(&a->g, np));
  PO_TRY(dalloc(&a->wb, np));
  PO_TRY(dalloc(&a->wt, np));
  PO_TRY(dalloc(&a->h, size_t(a->depth) * MB * W));
  PO_TRY(dalloc(&a->hT, size_t(a->depth) * hs * MB));
  PO_TRY(dalloc(&a->gp, size_t(a->depth) * MB * W));
  PO_TRY(dalloc(&a->dz, 2 * size_t(MB) * W));
  PO_TRY(dalloc(&a->dzT, 2 * size_t(W) * MB));
  PO_TRY(dalloc(&a->y, MB));
  PO_TRY(dalloc(&a->wpart, size_t(kMaxSplit) * (size_t(a->n_in) * W + size_t(a->depth - 1) * W * W)));
  PO_TRY(dalloc(&a->bpart, size_t(a->depth) * (MB / 32) * W));
  PO_TRY(dalloc(&a->opart, size_t(MB / 32) * (W + 2)));
  PO_TRY(dalloc(&a->ctr, 1));
  PO_HIP(hipStreamCreateWithFlags(&a->cap, hipStreamNonBlocking));
  PO_HIP(hipMemsetAsync(a->m, 0, sizeof(float) * np, s));
  PO_HIP(hipMemsetAsync(a->v, 0, sizeof(float) * np, s));
  hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(1), 0, s, a->ctr, 1);
  PO_HIP(hipGetLastError());
  k = a->n_in;
  for (int l = 0; l <= a->depth; ++l) {
    const int64_t kin = (l < a->depth) ? k : a->width;
    const int64_t n = (l < a->depth) ? kin * a->width + a->width : a->width + 1;
    const float bound = float(1.0 / std::sqrt(double(kin)));
    hipLaunchKernelGGL(k_init, dim3(blocks(n)), dim3(256), 0, s, a->p, layer_w_off(a, l), n, bound, seed, uint32_t(l));
    PO_HIP(hipGetLastError());
    k = a->width;
  }
  hipLaunchKernelGGL(k_weights_to_bf16, dim3(blocks(np)), dim3(256), 0, s, param_map(a, 32), a->p, a->wb, a->wt);
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
  hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(1), 0, s, a->ctr, 1);
  PO_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_weights_to_bf16, dim3(blocks(a->n_params)), dim3(256), 0, s, param_map(a, 32), a->p, a->wb,
                     a->wt);
  PO_HIP(hipGetLastError());
  return PO_OK;
}

po_status po_mlp_forward(struct po_mlp* a, const double* d_x, int32_t batch, float* d_y, void* stream) {
  if (!a) return set_error(PO_ERR_INVALID, "network is NULL");
  PO_TRY(check_batch(a, batch));
  PO_TRY(check_device_range(d_x, sizeof(double) * size_t(batch) * a->n_in, 16, "d_x"));
  PO_TRY(check_device_range(d_y, sizeof(float) * batch, 4, "d_y"));
  return forward_impl(a, d_x, batch, d_y, static_cast<hipStream_t>(stream));
}

po_status po_mlp_loss_grad(struct po_mlp* a, const double* d_x, const float* d_target, int32_t batch, float* d_loss,
                           float* d_grad, void* stream) {
  if (!a) return set_error(PO_ERR_INVALID, "network is NULL");
  PO_TRY(check_batch(a, batch));
  PO_TRY(check_device_range(d_x, sizeof(double) * size_t(batch) * a->n_in, 16, "d_x"));
  PO_TRY(check_device_range(d_target, sizeof(float) * batch, 4, "d_target"));
  if (d_loss) PO_TRY(check_device_range(d_loss, sizeof(float), 4, "d_loss"));
  if (d_grad) PO_TRY(check_device_range(d_grad, sizeof(float) * a->n_params, 4, "d_grad"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  RowMap rows{nullptr, nullptr, batch, batch};
  PO_TRY(grad_impl(a, d_x, rows, d_target, nullptr, 0.0, 1.0, batch, s));
  PO_TRY(adam_launch(a, batch, nullptr, a->g, -1.0f, d_loss, 0, s));  // assemble only
  if (d_grad) PO_HIP(hipMemcpyAsync(d_grad, a->g, sizeof(float) * a->n_params, hipMemcpyDeviceToDevice, s));
  return PO_OK;
}

po_status po_mlp_adam_step(struct po_mlp* a, const float* d_grad, float lr, void* stream) {
  if (!a) return set_error(PO_ERR_INVALID, "network is NULL");
  if (!(lr >= 0.0f) || !std::isfinite(lr)) return set_error(PO_ERR_INVALID, "lr must be finite and >= 0");
  if (d_grad) PO_TRY(check_device_range(d_grad, sizeof(float) * a->n_params, 4, "d_grad"));
  return adam_launch(a, 32, d_grad ? d_grad : a->g, nullptr, lr, nullptr, 0, static_cast<hipStream_t>(stream));
}

po_status po_mlp_train_step(struct po_mlp* a, const double* d_x, const float* d_target, int32_t batch, float lr,
                            float* d_loss, void* stream) {
  if (!a) return set_error(PO_ERR_INVALID, "network is NULL");
  PO_TRY(check_batch(a, batch));
  if (!(lr >= 0.0f) || !std::isfinite(lr)) return set_error(PO_ERR_INVALID, "lr must be finite and >= 0");
  PO_TRY(check_device_range(d_x, sizeof(double) * size_t(batch) * a->n_in, 16, "d_x"));
  PO_TRY(check_device_range(d_target, sizeof(float) * batch, 4, "d_target"));
  if (d_loss) PO_TRY(check_device_range(d_loss, sizeof(float), 4, "d_loss"));
  return train_replay(a, d_x, d_target, nullptr, nullptr, batch, 0.0, 1.0, batch, lr, d_loss, 1,
                      static_cast<hipStream_t>(stream));
}

po_status po_mlp_train_indexed(struct po_mlp* a, const double* d_X, const double* d_J, int32_t n_rows,
                               const int32_t* d_idx, int32_t steps, int32_t batch, double mean, double inv_std,
                               float lr, float* d_losses, void* stream) {
  if (!a) return set_error(PO_ERR_INVALID, "network is NULL");
  PO_TRY(check_batch(a, batch));
  if (n_rows < 1) return set_error(PO_ERR_INVALID, "n_rows must be >= 1");
  if (steps < 0) return set_error(PO_ERR_INVALID, "steps must be >= 0");
  if (!(lr >= 0.0f) || !std::isfinite(lr)) return set_error(PO_ERR_INVALID, "lr must be finite and >= 0");
  if (!std::isfinite(mean) || !std::isfinite(inv_std)) return set_error(PO_ERR_INVALID, "mean and inv_std must be finite");
  PO_TRY(check_device_range(d_X, sizeof(double) * size_t(n_rows) * a->n_in, 16, "d_X"));
  PO_TRY(check_device_range(d_J, sizeof(double) * size_t(n_rows), 8, "d_J"));
  if (steps == 0) return PO_OK;
  PO_TRY(check_device_range(d_idx, sizeof(int32_t) * size_t(steps) * batch, 4, "d_idx"));
  if (d_losses) PO_TRY(check_device_range(d_losses, sizeof(float) * size_t(steps), 4, "d_losses"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(1), 0, s, a->ctr, 0);
  PO_HIP(hipGetLastError());
  return train_replay(a, d_X, nullptr, d_J, d_idx, n_rows, mean, inv_std, batch, lr, d_losses, steps, s);
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
