// C ABI of libpairopt.so: argument validation, per-pulse descriptors, scratch management and
// the sequencing of the synthesis, evolution, reduction and differential-evolution kernels.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <mutex>
#include <utility>
#include <cstdio>
#include <cstring>
#include <vector>

#include "common.hpp"

namespace po {

static thread_local std::string g_error;

po_status set_error(po_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
  return s;
}

po_status device_error(hipError_t e, const char* what) {
  (void)hipGetLastError();
  return set_error(e == hipErrorOutOfMemory ? PO_ERR_NOMEM : PO_ERR_DEVICE, "%s failed: %s", what,
                   hipGetErrorString(e));
}

po_status check_device_range(const void* p, size_t bytes, size_t align, const char* name) {
  if (!p) return set_error(PO_ERR_INVALID, "%s is NULL", name);
  if (reinterpret_cast<uintptr_t>(p) % align) return set_error(PO_ERR_INVALID, "%s is not %zu-byte aligned", name, align);
  hipPointerAttribute_t attr;
  std::memset(&attr, 0, sizeof attr);
  hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return set_error(PO_ERR_INVALID, "%s is not a device pointer (%s)", name, hipGetErrorString(e));
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
    return set_error(PO_ERR_INVALID, "%s is not device memory (type %d)", name, int(attr.type));
  int dev = -1;
  PO_HIP(hipGetDevice(&dev));
  if (attr.type == hipMemoryTypeDevice && attr.device != dev)
    return set_error(PO_ERR_INVALID, "%s lives on device %d, current device is %d", name, attr.device, dev);
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  e = hipMemGetAddressRange(&base, &size, const_cast<void*>(p));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return set_error(PO_ERR_INVALID, "%s: allocation range unknown (%s)", name, hipGetErrorString(e));
  }
  const uintptr_t lo = reinterpret_cast<uintptr_t>(base), q = reinterpret_cast<uintptr_t>(p);
  if (q < lo || q - lo > size || bytes > size - (q - lo))
    return set_error(PO_ERR_INVALID, "%s: %zu bytes needed, allocation holds %zu from this pointer", name, bytes,
                     size_t(lo + size - q));
  return PO_OK;
}

po_status Scratch::alloc(size_t bytes, hipStream_t s) {
  stream = s;
  if (bytes == 0) bytes = 8;
  hipError_t e = hipMallocAsync(&ptr, bytes, s);
  if (e != hipSuccess) {
    ptr = nullptr;
    return device_error(e, "hipMallocAsync");
  }
  return PO_OK;
}

po_status validate_spec(const po_pulse_spec& s, int i) {
  if (!(s.T > 0.0) || !std::isfinite(s.T)) return set_error(PO_ERR_INVALID, "spec %d: T must be finite and > 0", i);
  if (s.nt < 2 || s.nt > (1 << 24)) return set_error(PO_ERR_INVALID, "spec %d: nt must be in [2, 2^24]", i);
  if (s.order < 1 || s.n_s < s.order || s.n_s > kMaxNs)
    return set_error(PO_ERR_INVALID, "spec %d: need 1 <= order <= n_s <= %d", i, kMaxNs);
  if (!(s.omega_min >= 0.0) || !(s.omega_max > s.omega_min) || !std::isfinite(s.omega_max))
    return set_error(PO_ERR_INVALID, "spec %d: need 0 <= omega_min < omega_max", i);
  const double dw = 2.0 * M_PI / s.T;
  const double r = s.omega_min / dw;
  if (std::fabs(r - std::nearbyint(r)) > 1e-9) return set_error(PO_ERR_INVALID, "spec %d: omega_min / (2 pi / T) must be an integer", i);
  const double nl = std::floor((s.omega_max - s.omega_min) / dw + 1e-9) + 1.0;
  if (nl > kMaxLines) return set_error(PO_ERR_INVALID, "spec %d: %g spectral lines exceed %d", i, nl, kMaxLines);
  if (s.norm != PO_NORM_NONE && s.norm != PO_NORM_PEAK && s.norm != PO_NORM_ENERGY)
    return set_error(PO_ERR_INVALID, "spec %d: unknown norm %d", i, s.norm);
  if (s.norm != PO_NORM_NONE && !(s.norm_value > 0.0 && std::isfinite(s.norm_value)))
    return set_error(PO_ERR_INVALID, "spec %d: norm_value must be finite and > 0", i);
  return PO_OK;
}

po_status validate_grid(const po_grid& g, int i) {
  for (int d = 0; d < 3; ++d) {
    if (g.n[d] < 1) return set_error(PO_ERR_INVALID, "grid %d: n[%d] must be >= 1", i, d);
    if (!std::isfinite(g.lo[d]) || !std::isfinite(g.hi[d]) || g.lo[d] > g.hi[d])
      return set_error(PO_ERR_INVALID, "grid %d: need finite lo[%d] <= hi[%d]", i, d, d);
    if (g.n[d] > 1 && !(g.lo[d] < g.hi[d])) return set_error(PO_ERR_INVALID, "grid %d: n[%d] > 1 needs lo < hi", i, d);
  }
  const int64_t m = int64_t(g.n[0]) * g.n[1] * g.n[2];
  if (m > (int64_t(1) << 30)) return set_error(PO_ERR_INVALID, "grid %d: more than 2^30 modes", i);
  return PO_OK;
}

po_status build_batch(int32_t n, const po_pulse_spec* specs, const po_grid* grids, PulseDev* out, Batch* b) {
  *b = Batch{};
  b->n_pulses = n;
  int64_t tab = 0, modes = 0, coeff = 0, spec = 0;
  int64_t units = 0, items = 0, blocks = 0, chunks = 0;
  for (int i = 0; i < n; ++i) {
    PulseDev d;
    std::memset(&d, 0, sizeof d);
    d.tab_off = tab;
    d.mode_off = modes;
    d.coeff_off = coeff;
    d.spec_off = spec;
    d.unit_off = units;
    d.item_off = int32_t(items);
    d.blk_off = int32_t(blocks);
    d.chk_off = int32_t(chunks);
    if (specs) {
      const po_pulse_spec& s = specs[i];
      d.nt = s.nt;
      d.ns = s.n_s;
      d.order = s.order;
      d.T = s.T;
      d.dt = s.T / double(s.nt);
      d.dw = 2.0 * M_PI / s.T;
      d.wmin = s.omega_min;
      d.wmax = s.omega_max;
      d.nmin = int32_t(std::nearbyint(s.omega_min / d.dw));
      d.nlines = int32_t(std::floor((s.omega_max - s.omega_min) / d.dw + 1e-9)) + 1;
      d.norm = s.norm;
      d.norm_value = s.norm_value;
      d.stat_blocks = s.norm == PO_NORM_NONE ? 0 : (s.nt + 1 + 255) / 256;
      tab += s.nt;
      chunks += (s.nt + kChunkSteps - 1) / kChunkSteps;
      coeff += 4 * int64_t(s.n_s);
      spec += 4 * int64_t(d.nlines);
      b->max_nt = std::max(b->max_nt, s.nt);
      b->max_lines = std::max(b->max_lines, d.nlines);
      b->max_ns = std::max(b->max_ns, d.ns);
      b->max_stat_blocks = std::max(b->max_stat_blocks, d.stat_blocks);
      if (i > 0 && (s.nt != specs[0].nt || s.T != specs[0].T)) b->uniform = false;
    }
    if (grids) {
      const po_grid& g = grids[i];
      double dv = 1.0;
      for (int k = 0; k < 3; ++k) {
        d.n[k] = g.n[k];
        d.lo[k] = g.lo[k];
        const bool sheet = g.n[k] == 1 && g.lo[k] == g.hi[k];
        d.dp[k] = sheet ? 0.0 : (g.hi[k] - g.lo[k]) / double(g.n[k]);
        if (!sheet) dv *= d.dp[k];
      }
      d.dv = dv;
      const int64_t m = int64_t(g.n[0]) * g.n[1] * g.n[2];
      d.nunits = int32_t((m + kUnit - 1) / kUnit);
      d.nitems = int32_t((m + kItem - 1) / kItem);
      modes += m;
      units += d.nunits;
      items += d.nitems;
      blocks += (m + kSelBlock - 1) / kSelBlock;
      if (i > 0 && std::memcmp(&g, &grids[0], sizeof g) != 0) b->uniform = false;
    }
    out[i] = d;
  }
  if (items > (int64_t(1) << 31) - 1) return set_error(PO_ERR_INVALID, "batch has too many modes");
  b->total_rows = tab;
  b->total_modes = modes;
  b->total_coeff = coeff;
  b->total_spec = spec;
  b->total_units = units;
  b->total_items = int32_t(items);
  b->total_blocks = int32_t(blocks);
  b->total_chunks = int32_t(chunks);
  return PO_OK;
}

namespace {

po_status check_specs(int32_t n, const po_pulse_spec* specs) {
  if (!specs) return set_error(PO_ERR_INVALID, "specs is NULL");
  for (int i = 0; i < n; ++i) PO_TRY(validate_spec(specs[i], i));
  return PO_OK;
}

po_status check_grids(int32_t n, const po_grid* grids) {
  if (!grids) return set_error(PO_ERR_INVALID, "grids is NULL");
  for (int i = 0; i < n; ++i) PO_TRY(validate_grid(grids[i], i));
  return PO_OK;
}

// Uploads the descriptors into a stream-ordered buffer.
po_status upload(const std::vector<PulseDev>& h, Scratch& sc, hipStream_t s) {
  PO_TRY(sc.alloc(sizeof(PulseDev) * h.size(), s));
  PO_HIP(hipMemcpyAsync(sc.ptr, h.data(), sizeof(PulseDev) * h.size(), hipMemcpyHostToDevice, s));
  return PO_OK;
}

// Scratch of one evaluation (synthesis + evolution + yield), in elements.
struct EvalSizes {
  size_t spec, part, scl, units, ranges;
};

EvalSizes eval_sizes(int32_t n, const Batch& b) {
  return EvalSizes{size_t(b.total_spec), size_t(std::max(1, b.max_stat_blocks)) * n, size_t(n),
                   size_t(b.total_units), 4 * size_t(b.total_chunks)};
}

po_status synth_into(const po_pulse_spec* specs, const double* d_coeff, double* d_A, double* d_E, double* d_A_edge,
                     double* d_scale, hipStream_t s, const Batch& b, const PulseDev* d_desc, double* d_spec,
                     double* d_part, double* d_scl) {
  (void)specs;
  return launch_synth(b, d_desc, d_coeff, d_spec, d_part, d_scl, d_A, d_E, d_A_edge, d_scale, s);
}

po_status synth_impl(int32_t n, const po_pulse_spec* specs, const double* d_coeff, double* d_A, double* d_E,
                     double* d_A_edge, double* d_scale, hipStream_t s, const Batch& b, const PulseDev* d_desc) {
  const EvalSizes z = eval_sizes(n, b);
  Scratch spec, part, scl;
  PO_TRY(spec.alloc(sizeof(double) * z.spec, s));
  PO_TRY(part.alloc(sizeof(double) * z.part, s));
  PO_TRY(scl.alloc(sizeof(double) * z.scl, s));
  return synth_into(specs, d_coeff, d_A, d_E, d_A_edge, d_scale, s, b, d_desc, static_cast<double*>(spec.ptr),
                    static_cast<double*>(part.ptr), static_cast<double*>(scl.ptr));
}

// Event pairs bracketing evolution launches while timers are enabled.
std::mutex g_timer_mu;
bool g_timer_on = false;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_timer_events;
unsigned long long* g_counts = nullptr;  // device: mode-steps per series variant (diagnostics)

// Evolution and yield into caller-provided scratch: d_units [total_units] (used when d_J is
// non-NULL), d_ranges [4 total_chunks].  timed: bracket the evolution with the kernel timers.
po_status evolve_into(const Batch& b, const PulseDev* d_desc, const double* d_A, const double* d_A_edge, double* d_f,
                      double* d_J, hipStream_t s, double* d_units, double* d_ranges, bool timed_ok) {
  hipEvent_t e0 = nullptr;
  const bool timed = timed_ok && timer_start(s, &e0);
  PO_TRY(launch_chunk_ranges(b, d_desc, d_A, d_ranges, s));
  PO_TRY(launch_evolve_grid(b, d_desc, d_A, d_A_edge, d_ranges, d_f, d_J ? d_units : nullptr, s));
  if (timed) {
    timer_stop(s, e0);
    PO_TRY(timer_count(b.n_pulses, d_desc, d_ranges, s));
  }
  if (d_J) PO_TRY(launch_yield_from_units(b, d_desc, d_units, d_J, s));
  return PO_OK;
}

po_status evolve_impl(const Batch& b, const PulseDev* d_desc, const double* d_A, const double* d_A_edge, double* d_f,
                      double* d_J, hipStream_t s) {
  Scratch units, sel;
  double* d_units = nullptr;
  if (d_J) {
    PO_TRY(units.alloc(sizeof(double) * size_t(b.total_units), s));
    d_units = static_cast<double*>(units.ptr);
  }
  PO_TRY(sel.alloc(sizeof(double) * 4 * size_t(b.total_chunks), s));
  return evolve_into(b, d_desc, d_A, d_A_edge, d_f, d_J, s, d_units, static_cast<double*>(sel.ptr), true);
}

// Gradient of J with respect to the tables (forward + adjoint sweep per mode, fixed-order sums).
po_status yield_grad_impl(const Batch& b, const std::vector<PulseDev>& h, const PulseDev* d_desc, const double* d_A,
                          const double* d_A_edge, double* d_J, double* d_gA, double* d_gedge, hipStream_t s) {
  std::vector<int64_t> goff(b.n_pulses);
  int64_t tot = 0;
  for (int i = 0; i < b.n_pulses; ++i) {
    goff[i] = tot;
    tot += int64_t(h[i].nitems) * h[i].nt * 2;
  }
  Scratch sgoff, part, epart, units, sel, ged;
  PO_TRY(part.alloc(sizeof(double) * size_t(tot), s));  // the large one first: fail before enqueueing work
  PO_TRY(sgoff.alloc(sizeof(int64_t) * goff.size(), s));
  PO_HIP(hipMemcpyAsync(sgoff.ptr, goff.data(), sizeof(int64_t) * goff.size(), hipMemcpyHostToDevice, s));
  PO_TRY(epart.alloc(sizeof(double) * 4 * size_t(b.total_items), s));
  PO_TRY(units.alloc(sizeof(double) * size_t(b.total_units), s));
  PO_TRY(sel.alloc(sizeof(int2) * size_t(b.total_blocks), s));
  int2* d_sel = static_cast<int2*>(sel.ptr);
  double* d_units = static_cast<double*>(units.ptr);
  PO_TRY(launch_block_select(b, d_desc, d_A, d_sel, s));
  PO_TRY(launch_yield_grad(b, d_desc, d_A, d_A_edge, d_sel, static_cast<int64_t*>(sgoff.ptr),
                           static_cast<double*>(part.ptr), static_cast<double*>(epart.ptr), d_units, d_gA, d_gedge, s));
  if (d_J) PO_TRY(launch_yield_from_units(b, d_desc, d_units, d_J, s));
  return PO_OK;
}

po_status check_differentiable(int32_t n, const po_pulse_spec* specs) {
  for (int i = 0; i < n; ++i)
    if (specs[i].norm == PO_NORM_PEAK)
      return set_error(PO_ERR_UNSUPPORTED, "spec %d: the peak normalisation is not differentiable; use "
                                           "PO_NORM_NONE (with an energy penalty) or PO_NORM_ENERGY", i);
  return PO_OK;
}

std::atomic<int32_t> g_check_finite{0};

__global__ void k_zero_count(unsigned int* count) { *count = 0u; }

// Adds the number of non-finite entries of v[0, n) to *count (grid-stride; one atomic per block).
__global__ void __launch_bounds__(256) k_count_nonfinite(const double* __restrict__ v, int64_t n,
                                                         unsigned int* __restrict__ count) {
  __shared__ unsigned int part[256];
  unsigned int c = 0;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
    c += std::isfinite(v[i]) ? 0u : 1u;
  part[threadIdx.x] = c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0 && part[0] != 0u) atomicAdd(count, part[0]);
}

// With the check enabled: counts the non-finite entries of d_v[0, n) on the stream, waits for it,
// and returns PO_ERR_NUMERIC if there are any.
po_status check_finite(const double* d_v, int64_t n, const char* what, hipStream_t s) {
  if (!g_check_finite.load(std::memory_order_relaxed) || n <= 0) return PO_OK;
  Scratch cnt;
  PO_TRY(cnt.alloc(sizeof(unsigned int), s));
  unsigned int* d_c = static_cast<unsigned int*>(cnt.ptr);
  hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(1), 0, s, d_c);
  PO_HIP(hipGetLastError());
  const int64_t blocks = std::min<int64_t>(1024, (n + 255) / 256);
  hipLaunchKernelGGL(k_count_nonfinite, dim3(unsigned(blocks)), dim3(256), 0, s, d_v, n, d_c);
  PO_HIP(hipGetLastError());
  unsigned int h_c = 0;
  PO_HIP(hipMemcpyAsync(&h_c, d_c, sizeof(h_c), hipMemcpyDeviceToHost, s));
  PO_HIP(hipStreamSynchronize(s));
  if (h_c != 0u) return set_error(PO_ERR_NUMERIC, "%u non-finite values in %s", h_c, what);
  return PO_OK;
}

// The evolution's checked output: J, or f when J is not requested.
po_status check_outputs(const Batch& b, const double* d_f, const double* d_J, hipStream_t s) {
  return d_J ? check_finite(d_J, b.n_pulses, "d_J", s) : check_finite(d_f, b.total_modes, "d_f", s);
}

}  // namespace

bool timer_start(hipStream_t s, hipEvent_t* e0) {
  {
    std::lock_guard<std::mutex> lk(g_timer_mu);
    if (!g_timer_on) return false;
  }
  if (hipEventCreate(e0) != hipSuccess) return false;
  if (hipEventRecord(*e0, s) != hipSuccess) {
    (void)hipEventDestroy(*e0);
    return false;
  }
  return true;
}

po_status timer_count(int n_pulses, const PulseDev* d_desc, const double* d_ranges, hipStream_t s) {
  unsigned long long* c;
  {
    std::lock_guard<std::mutex> lk(g_timer_mu);
    if (!g_timer_on || !g_counts) return PO_OK;
    c = g_counts;
  }
  return launch_count_mode_steps(n_pulses, d_desc, d_ranges, c, s);
}

void timer_stop(hipStream_t s, hipEvent_t e0) {
  hipEvent_t e1 = nullptr;
  if (hipEventCreate(&e1) != hipSuccess || hipEventRecord(e1, s) != hipSuccess) {
    (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return;
  }
  std::lock_guard<std::mutex> lk(g_timer_mu);
  g_timer_events.emplace_back(e0, e1);
}

// ---------------------------------------------------------------------------------------------
// Allocation-free evaluation: every scratch buffer of po_evaluate_noalloc lives in this file-scope
// device array (each device holds its own copy until the process ends).  In host code `scratch`
// is only a stand-in for the symbol: its device address comes from hipGetSymbolAddress, taken once
// per device with that device current, and only that address is handed to kernels and copies.
// ---------------------------------------------------------------------------------------------
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr int kNoAllocMaxPulses = 4096;
constexpr int kNoAllocMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_noalloc_mu;                               // guards the two arrays below
void* g_scratch_dev[kNoAllocMaxDevices] = {};          // device address of `scratch`, per device
PulseDev g_noalloc_desc[kNoAllocMaxPulses];            // host staging of the pulse descriptors

// Device address of `scratch` on the current device (looked up on the first call there).
po_status noalloc_scratch(void** out) {
  int dev = -1;
  PO_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoAllocMaxDevices) return set_error(PO_ERR_UNSUPPORTED, "device %d out of range", dev);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return device_error(e == hipSuccess ? hipErrorInvalidSymbol : e, "hipGetSymbolAddress");
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return PO_OK;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace po

using namespace po;

extern "C" {

int po_abi_version(void) { return 1; }

int32_t po_set_check_finite(int32_t enable) { return g_check_finite.exchange(enable ? 1 : 0); }

const char* po_last_error(void) { return g_error.c_str(); }

po_status po_pulse_synth(int32_t n, const po_pulse_spec* specs, const double* d_coeff, double* d_A, double* d_E,
                         double* d_A_edge, double* d_scale, void* stream) {
  if (n < 1) return set_error(PO_ERR_INVALID, "n_pulses must be >= 1");
  PO_TRY(check_specs(n, specs));
  std::vector<PulseDev> h(n);
  Batch b;
  PO_TRY(build_batch(n, specs, nullptr, h.data(), &b));
  PO_TRY(check_device_range(d_coeff, sizeof(double) * b.total_coeff, 8, "d_coeff"));
  PO_TRY(check_device_range(d_A, sizeof(double) * 2 * b.total_rows, 8, "d_A"));
  if (d_E) PO_TRY(check_device_range(d_E, sizeof(double) * 2 * b.total_rows, 8, "d_E"));
  PO_TRY(check_device_range(d_A_edge, sizeof(double) * 4 * n, 8, "d_A_edge"));
  if (d_scale) PO_TRY(check_device_range(d_scale, sizeof(double) * n, 8, "d_scale"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  Scratch desc;
  PO_TRY(upload(h, desc, s));
  PO_TRY(synth_impl(n, specs, d_coeff, d_A, d_E, d_A_edge, d_scale, s, b, static_cast<PulseDev*>(desc.ptr)));
  return check_finite(d_A, 2 * b.total_rows, "d_A", s);
}

po_status po_evolve_modes(int32_t n, const po_pulse_spec* specs, const po_grid* grids, const double* d_A,
                          const double* d_A_edge, double* d_f, double* d_J, const struct po_plan* plan, void* stream) {
  if (n < 1) return set_error(PO_ERR_INVALID, "n_pulses must be >= 1");
  PO_TRY(check_specs(n, specs));
  PO_TRY(check_grids(n, grids));
  if (!d_f && !d_J) return set_error(PO_ERR_INVALID, "at least one of d_f, d_J must be non-NULL");
  std::vector<PulseDev> h(n);
  Batch b;
  PO_TRY(build_batch(n, specs, grids, h.data(), &b));
  PO_TRY(check_device_range(d_A, sizeof(double) * 2 * b.total_rows, 8, "d_A"));
  PO_TRY(check_device_range(d_A_edge, sizeof(double) * 4 * n, 8, "d_A_edge"));
  if (d_f) PO_TRY(check_device_range(d_f, sizeof(double) * b.total_modes, 8, "d_f"));
  if (d_J) PO_TRY(check_device_range(d_J, sizeof(double) * n, 8, "d_J"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (plan) {
    hipEvent_t e0 = nullptr;
    const bool timed = timer_start(s, &e0);
    PO_TRY(plan_evolve(plan, n, specs, grids, d_A, d_A_edge, d_f, d_J, s));
    if (timed) timer_stop(s, e0);
    return check_outputs(b, d_f, d_J, s);
  }
  Scratch desc;
  PO_TRY(upload(h, desc, s));
  PO_TRY(evolve_impl(b, static_cast<PulseDev*>(desc.ptr), d_A, d_A_edge, d_f, d_J, s));
  return check_outputs(b, d_f, d_J, s);
}

po_status po_field_samples(int32_t n, const po_pulse_spec* specs, const double* d_coeff, int32_t n_sub,
                           const double* offsets, int32_t with_end, double* d_E, double* d_Ed, double* d_A,
                           double* d_A_edge, double* d_scale, void* stream) {
  if (n < 1) return set_error(PO_ERR_INVALID, "n_pulses must be >= 1");
  PO_TRY(check_specs(n, specs));
  if (n_sub < 1 || n_sub > kMaxSub) return set_error(PO_ERR_INVALID, "n_sub must be in [1, %d]", kMaxSub);
  if (!offsets) return set_error(PO_ERR_INVALID, "offsets is NULL");
  for (int r = 0; r < n_sub; ++r)
    if (!(offsets[r] >= 0.0 && offsets[r] <= 1.0)) return set_error(PO_ERR_INVALID, "offsets[%d] not in [0, 1]", r);
  if (!d_E && !d_Ed && !d_A && !d_A_edge)
    return set_error(PO_ERR_INVALID, "at least one of d_E, d_Ed, d_A, d_A_edge must be non-NULL");
  std::vector<PulseDev> h(n);
  Batch b;
  PO_TRY(build_batch(n, specs, nullptr, h.data(), &b));
  int64_t rows = 0;
  for (int i = 0; i < n; ++i) {
    h[i].tab_off = rows;
    rows += int64_t(specs[i].nt) * n_sub + (with_end ? 1 : 0);
  }
  PO_TRY(check_device_range(d_coeff, sizeof(double) * b.total_coeff, 8, "d_coeff"));
  if (d_E) PO_TRY(check_device_range(d_E, sizeof(double) * 2 * rows, 8, "d_E"));
  if (d_Ed) PO_TRY(check_device_range(d_Ed, sizeof(double) * 2 * rows, 8, "d_Ed"));
  if (d_A) PO_TRY(check_device_range(d_A, sizeof(double) * 2 * rows, 8, "d_A"));
  if (d_A_edge) PO_TRY(check_device_range(d_A_edge, sizeof(double) * 4 * n, 8, "d_A_edge"));
  if (d_scale) PO_TRY(check_device_range(d_scale, sizeof(double) * n, 8, "d_scale"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  Scratch desc, spec, part, scl;
  PO_TRY(upload(h, desc, s));
  PO_TRY(spec.alloc(sizeof(double) * b.total_spec, s));
  PO_TRY(part.alloc(sizeof(double) * size_t(std::max(1, b.max_stat_blocks)) * n, s));
  PO_TRY(scl.alloc(sizeof(double) * n, s));
  return launch_samples(b, static_cast<PulseDev*>(desc.ptr), d_coeff, static_cast<double*>(spec.ptr),
                        static_cast<double*>(part.ptr), static_cast<double*>(scl.ptr), n_sub, offsets, with_end ? 1 : 0,
                        d_E, d_Ed, d_A, d_A_edge, d_scale, s);
}

po_status po_qke_modes(int32_t n, const po_pulse_spec* specs, const po_grid* grids, const double* d_E,
                       const double* d_Ed, const double* d_A, int32_t linear, double* d_f, double* d_J, void* stream) {
  if (n < 1) return set_error(PO_ERR_INVALID, "n_pulses must be >= 1");
  PO_TRY(check_specs(n, specs));
  PO_TRY(check_grids(n, grids));
  if (!d_f && !d_J) return set_error(PO_ERR_INVALID, "at least one of d_f, d_J must be non-NULL");
  std::vector<PulseDev> h(n);
  Batch b;
  PO_TRY(build_batch(n, specs, grids, h.data(), &b));
  int64_t rows = 0;
  for (int i = 0; i < n; ++i) {
    h[i].tab_off = rows;
    rows += 2 * int64_t(specs[i].nt) + 1;
  }
  PO_TRY(check_device_range(d_E, sizeof(double) * 2 * rows, 8, "d_E"));
  PO_TRY(check_device_range(d_Ed, sizeof(double) * 2 * rows, 8, "d_Ed"));
  PO_TRY(check_device_range(d_A, sizeof(double) * 2 * rows, 8, "d_A"));
  if (d_f) PO_TRY(check_device_range(d_f, sizeof(double) * b.total_modes, 8, "d_f"));
  if (d_J) PO_TRY(check_device_range(d_J, sizeof(double) * n, 8, "d_J"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  Scratch desc, units;
  PO_TRY(upload(h, desc, s));
  double* d_units = nullptr;
  if (d_J) {
    PO_TRY(units.alloc(sizeof(double) * size_t(b.total_units), s));
    d_units = static_cast<double*>(units.ptr);
  }
  const PulseDev* d_desc = static_cast<PulseDev*>(desc.ptr);
  PO_TRY(launch_qke_grid(b, d_desc, d_E, d_Ed, d_A, linear ? 1 : 0, d_f, d_units, s));
  if (d_J) PO_TRY(launch_yield_from_units(b, d_desc, d_units, d_J, s));
  return PO_OK;
}

po_status po_evolve_modes_m4(int32_t n, const po_pulse_spec* specs, const po_grid* grids, const double* d_Ag,
                             const double* d_A_edge, double* d_f, double* d_J, void* stream) {
  if (n < 1) return set_error(PO_ERR_INVALID, "n_pulses must be >= 1");
  PO_TRY(check_specs(n, specs));
  PO_TRY(check_grids(n, grids));
  if (!d_f && !d_J) return set_error(PO_ERR_INVALID, "at least one of d_f, d_J must be non-NULL");
  std::vector<PulseDev> h(n);
  Batch b;
  PO_TRY(build_batch(n, specs, grids, h.data(), &b));
  PO_TRY(check_device_range(d_Ag, sizeof(double) * 4 * b.total_rows, 16, "d_Ag"));
  PO_TRY(check_device_range(d_A_edge, sizeof(double) * 4 * n, 8, "d_A_edge"));
  if (d_f) PO_TRY(check_device_range(d_f, sizeof(double) * b.total_modes, 8, "d_f"));
  if (d_J) PO_TRY(check_device_range(d_J, sizeof(double) * n, 8, "d_J"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  Scratch desc, units, sel;
  PO_TRY(upload(h, desc, s));
  double* d_units = nullptr;
  if (d_J) {
    PO_TRY(units.alloc(sizeof(double) * size_t(b.total_units), s));
    d_units = static_cast<double*>(units.ptr);
  }
  PO_TRY(sel.alloc(sizeof(double) * 4 * size_t(b.total_chunks), s));
  const PulseDev* d_desc = static_cast<PulseDev*>(desc.ptr);
  double* d_ranges = static_cast<double*>(sel.ptr);
  PO_TRY(launch_chunk_ranges4(b, d_desc, d_Ag, d_ranges, s));
  PO_TRY(launch_evolve4_grid(b, d_desc, d_Ag, d_A_edge, d_ranges, d_f, d_units, s));
  if (d_J) PO_TRY(launch_yield_from_units(b, d_desc, d_units, d_J, s));
  return PO_OK;
}

po_status po_evolve_modes_split(int32_t n, const po_pulse_spec* specs, const po_grid* grids, int32_t order,
                                const double* d_At, const double* d_A_edge, double* d_f, double* d_J, void* stream) {
  if (n < 1) return set_error(PO_ERR_INVALID, "n_pulses must be >= 1");
  if (order != 2 && order != 4) return set_error(PO_ERR_INVALID, "order must be 2 or 4");
  PO_TRY(check_specs(n, specs));
  PO_TRY(check_grids(n, grids));
  if (!d_f && !d_J) return set_error(PO_ERR_INVALID, "at least one of d_f, d_J must be non-NULL");
  std::vector<PulseDev> h(n);
  Batch b;
  PO_TRY(build_batch(n, specs, grids, h.data(), &b));
  const int nsub = order == 2 ? 1 : 3;
  PO_TRY(check_device_range(d_At, sizeof(double) * 2 * nsub * b.total_rows, 16, "d_At"));
  PO_TRY(check_device_range(d_A_edge, sizeof(double) * 4 * n, 16, "d_A_edge"));
  if (d_f) PO_TRY(check_device_range(d_f, sizeof(double) * b.total_modes, 8, "d_f"));
  if (d_J) PO_TRY(check_device_range(d_J, sizeof(double) * n, 8, "d_J"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  Scratch desc, units, sel;
  PO_TRY(upload(h, desc, s));
  double* d_units = nullptr;
  if (d_J) {
    PO_TRY(units.alloc(sizeof(double) * size_t(b.total_units), s));
    d_units = static_cast<double*>(units.ptr);
  }
  PO_TRY(sel.alloc(sizeof(double) * 4 * size_t(b.total_chunks), s));
  const PulseDev* d_desc = static_cast<PulseDev*>(desc.ptr);
  PO_TRY(launch_evolve_split_grid(b, order, d_desc, d_At, d_A_edge, static_cast<double*>(sel.ptr), d_f, d_units, s));
  if (d_J) PO_TRY(launch_yield_from_units(b, d_desc, d_units, d_J, s));
  return PO_OK;
}

po_status po_yield_gradient(int32_t n, const po_pulse_spec* specs, const po_grid* grids, const double* d_A,
                            const double* d_A_edge, double* d_J, double* d_gA, double* d_gedge, void* stream) {
  if (n < 1) return set_error(PO_ERR_INVALID, "n_pulses must be >= 1");
  PO_TRY(check_specs(n, specs));
  PO_TRY(check_grids(n, grids));
  std::vector<PulseDev> h(n);
  Batch b;
  PO_TRY(build_batch(n, specs, grids, h.data(), &b));
  PO_TRY(check_device_range(d_A, sizeof(double) * 2 * b.total_rows, 8, "d_A"));
  PO_TRY(check_device_range(d_A_edge, sizeof(double) * 4 * n, 8, "d_A_edge"));
  PO_TRY(check_device_range(d_gA, sizeof(double) * 2 * b.total_rows, 8, "d_gA"));
  if (d_gedge) PO_TRY(check_device_range(d_gedge, sizeof(double) * 4 * n, 8, "d_gedge"));
  if (d_J) PO_TRY(check_device_range(d_J, sizeof(double) * n, 8, "d_J"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  Scratch desc;
  PO_TRY(upload(h, desc, s));
  return yield_grad_impl(b, h, static_cast<PulseDev*>(desc.ptr), d_A, d_A_edge, d_J, d_gA, d_gedge, s);
}

po_status po_synth_gradient(int32_t n, const po_pulse_spec* specs, const double* d_coeff, const double* d_gA,
                            const double* d_gedge, double* d_grad, double* d_U, double* d_gU, void* stream) {
  if (n < 1) return set_error(PO_ERR_INVALID, "n_pulses must be >= 1");
  PO_TRY(check_specs(n, specs));
  PO_TRY(check_differentiable(n, specs));
  std::vector<PulseDev> h(n);
  Batch b;
  PO_TRY(build_batch(n, specs, nullptr, h.data(), &b));
  PO_TRY(check_device_range(d_coeff, sizeof(double) * b.total_coeff, 8, "d_coeff"));
  PO_TRY(check_device_range(d_gA, sizeof(double) * 2 * b.total_rows, 8, "d_gA"));
  if (d_gedge) PO_TRY(check_device_range(d_gedge, sizeof(double) * 4 * n, 8, "d_gedge"));
  PO_TRY(check_device_range(d_grad, sizeof(double) * b.total_coeff, 8, "d_grad"));
  if (d_U) PO_TRY(check_device_range(d_U, sizeof(double) * n, 8, "d_U"));
  if (d_gU) PO_TRY(check_device_range(d_gU, sizeof(double) * b.total_coeff, 8, "d_gU"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  Scratch desc, A, E, edge, scl, lines;
  PO_TRY(upload(h, desc, s));
  const PulseDev* d_desc = static_cast<PulseDev*>(desc.ptr);
  PO_TRY(A.alloc(sizeof(double) * 2 * b.total_rows, s));
  PO_TRY(E.alloc(sizeof(double) * 2 * b.total_rows, s));
  PO_TRY(edge.alloc(sizeof(double) * 4 * n, s));
  PO_TRY(scl.alloc(sizeof(double) * n, s));
  PO_TRY(lines.alloc(sizeof(double) * size_t(b.total_spec / 4) * 8 * size_t(b.max_ns), s));
  double *dA = static_cast<double*>(A.ptr), *dE = static_cast<double*>(E.ptr), *de = static_cast<double*>(edge.ptr);
  double* dscale = static_cast<double*>(scl.ptr);
  PO_TRY(synth_impl(n, specs, d_coeff, dA, dE, de, dscale, s, b, d_desc));
  return launch_synth_adjoint(b, d_desc, d_coeff, d_gA, d_gedge, dA, de, dE, dscale, static_cast<double*>(lines.ptr),
                              d_grad, d_U, d_gU, s);
}

po_status po_evaluate_gradient(int32_t n, const po_pulse_spec* specs, const po_grid* grids, const double* d_coeff,
                               double* d_J, double* d_grad, double* d_U, double* d_gU, void* stream) {
  if (n < 1) return set_error(PO_ERR_INVALID, "n_pulses must be >= 1");
  PO_TRY(check_specs(n, specs));
  PO_TRY(check_grids(n, grids));
  PO_TRY(check_differentiable(n, specs));
  std::vector<PulseDev> h(n);
  Batch b;
  PO_TRY(build_batch(n, specs, grids, h.data(), &b));
  PO_TRY(check_device_range(d_coeff, sizeof(double) * b.total_coeff, 8, "d_coeff"));
  PO_TRY(check_device_range(d_J, sizeof(double) * n, 8, "d_J"));
  PO_TRY(check_device_range(d_grad, sizeof(double) * b.total_coeff, 8, "d_grad"));
  if (d_U) PO_TRY(check_device_range(d_U, sizeof(double) * n, 8, "d_U"));
  if (d_gU) PO_TRY(check_device_range(d_gU, sizeof(double) * b.total_coeff, 8, "d_gU"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  Scratch desc, A, E, edge, scl, gA, gedge, lines;
  PO_TRY(upload(h, desc, s));
  const PulseDev* d_desc = static_cast<PulseDev*>(desc.ptr);
  PO_TRY(A.alloc(sizeof(double) * 2 * b.total_rows, s));
  PO_TRY(E.alloc(sizeof(double) * 2 * b.total_rows, s));
  PO_TRY(edge.alloc(sizeof(double) * 4 * n, s));
  PO_TRY(scl.alloc(sizeof(double) * n, s));
  PO_TRY(gA.alloc(sizeof(double) * 2 * b.total_rows, s));
  PO_TRY(gedge.alloc(sizeof(double) * 4 * n, s));
  PO_TRY(lines.alloc(sizeof(double) * size_t(b.total_spec / 4) * 8 * size_t(b.max_ns), s));
  double *dA = static_cast<double*>(A.ptr), *dE = static_cast<double*>(E.ptr), *de = static_cast<double*>(edge.ptr);
  double *dscale = static_cast<double*>(scl.ptr), *dgA = static_cast<double*>(gA.ptr);
  double* dge = static_cast<double*>(gedge.ptr);
  PO_TRY(synth_impl(n, specs, d_coeff, dA, dE, de, dscale, s, b, d_desc));
  PO_TRY(yield_grad_impl(b, h, d_desc, dA, de, d_J, dgA, dge, s));
  return launch_synth_adjoint(b, d_desc, d_coeff, dgA, dge, dA, de, dE, dscale, static_cast<double*>(lines.ptr),
                              d_grad, d_U, d_gU, s);
}

po_status po_pair_yield(int32_t n, const po_grid* grids, const double* d_f, double* d_J, void* stream) {
  if (n < 1) return set_error(PO_ERR_INVALID, "n_pulses must be >= 1");
  PO_TRY(check_grids(n, grids));
  std::vector<PulseDev> h(n);
  Batch b;
  PO_TRY(build_batch(n, nullptr, grids, h.data(), &b));
  PO_TRY(check_device_range(d_f, sizeof(double) * b.total_modes, 8, "d_f"));
  PO_TRY(check_device_range(d_J, sizeof(double) * n, 8, "d_J"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  Scratch desc, units;
  PO_TRY(upload(h, desc, s));
  PO_TRY(units.alloc(sizeof(double) * size_t(b.total_units), s));
  const PulseDev* d_desc = static_cast<PulseDev*>(desc.ptr);
  PO_TRY(launch_unit_sums_from_f(b, d_desc, d_f, static_cast<double*>(units.ptr), s));
  PO_TRY(launch_yield_from_units(b, d_desc, static_cast<double*>(units.ptr), d_J, s));
  return check_finite(d_J, n, "d_J", s);
}

po_status po_evaluate(int32_t n, const po_pulse_spec* specs, const po_grid* grids, const double* d_coeff, double* d_A,
                      double* d_A_edge, double* d_scale, double* d_f, double* d_J, const struct po_plan* plan,
                      void* stream) {
  if (n < 1) return set_error(PO_ERR_INVALID, "n_pulses must be >= 1");
  PO_TRY(check_specs(n, specs));
  PO_TRY(check_grids(n, grids));
  if (!d_f && !d_J) return set_error(PO_ERR_INVALID, "at least one of d_f, d_J must be non-NULL");
  std::vector<PulseDev> h(n);
  Batch b;
  PO_TRY(build_batch(n, specs, grids, h.data(), &b));
  PO_TRY(check_device_range(d_coeff, sizeof(double) * b.total_coeff, 8, "d_coeff"));
  PO_TRY(check_device_range(d_A, sizeof(double) * 2 * b.total_rows, 8, "d_A"));
  PO_TRY(check_device_range(d_A_edge, sizeof(double) * 4 * n, 8, "d_A_edge"));
  if (d_scale) PO_TRY(check_device_range(d_scale, sizeof(double) * n, 8, "d_scale"));
  if (d_f) PO_TRY(check_device_range(d_f, sizeof(double) * b.total_modes, 8, "d_f"));
  if (d_J) PO_TRY(check_device_range(d_J, sizeof(double) * n, 8, "d_J"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  Scratch desc;
  PO_TRY(upload(h, desc, s));
  const PulseDev* d_desc = static_cast<PulseDev*>(desc.ptr);
  PO_TRY(synth_impl(n, specs, d_coeff, d_A, nullptr, d_A_edge, d_scale, s, b, d_desc));
  PO_TRY(check_finite(d_A, 2 * b.total_rows, "d_A", s));
  if (plan) {
    hipEvent_t e0 = nullptr;
    const bool timed = timer_start(s, &e0);
    PO_TRY(plan_evolve(plan, n, specs, grids, d_A, d_A_edge, d_f, d_J, s));
    if (timed) timer_stop(s, e0);
    return check_outputs(b, d_f, d_J, s);
  }
  PO_TRY(evolve_impl(b, d_desc, d_A, d_A_edge, d_f, d_J, s));
  return check_outputs(b, d_f, d_J, s);
}

po_status po_evaluate_noalloc(int32_t n, const po_pulse_spec* specs, const po_grid* grids, const double* d_coeff,
                              double* d_A, double* d_A_edge, double* d_scale, double* d_f, double* d_J, void* stream) {
  if (n < 1) return set_error(PO_ERR_INVALID, "n_pulses must be >= 1");
  if (n > kNoAllocMaxPulses) return set_error(PO_ERR_INVALID, "n_pulses must be <= %d", kNoAllocMaxPulses);
  PO_TRY(check_specs(n, specs));
  PO_TRY(check_grids(n, grids));
  if (!d_f && !d_J) return set_error(PO_ERR_INVALID, "at least one of d_f, d_J must be non-NULL");
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  Batch b;
  PO_TRY(build_batch(n, specs, grids, g_noalloc_desc, &b));
  const EvalSizes z = eval_sizes(n, b);
  const size_t o_desc = 0;
  const size_t o_spec = o_desc + align256(sizeof(PulseDev) * size_t(n));
  const size_t o_part = o_spec + align256(sizeof(double) * z.spec);
  const size_t o_scl = o_part + align256(sizeof(double) * z.part);
  const size_t o_units = o_scl + align256(sizeof(double) * z.scl);
  const size_t o_ranges = o_units + align256(sizeof(double) * z.units);
  const size_t need = o_ranges + align256(sizeof(double) * z.ranges);
  if (need > kNoAllocScratchBytes)
    return set_error(PO_ERR_INVALID, "batch needs %zu bytes of scratch, the allocation-free path holds %zu", need,
                     kNoAllocScratchBytes);
  PO_TRY(check_device_range(d_coeff, sizeof(double) * b.total_coeff, 8, "d_coeff"));
  PO_TRY(check_device_range(d_A, sizeof(double) * 2 * b.total_rows, 8, "d_A"));
  PO_TRY(check_device_range(d_A_edge, sizeof(double) * 4 * n, 8, "d_A_edge"));
  if (d_scale) PO_TRY(check_device_range(d_scale, sizeof(double) * n, 8, "d_scale"));
  if (d_f) PO_TRY(check_device_range(d_f, sizeof(double) * b.total_modes, 8, "d_f"));
  if (d_J) PO_TRY(check_device_range(d_J, sizeof(double) * n, 8, "d_J"));
  void* base = nullptr;
  PO_TRY(noalloc_scratch(&base));
  unsigned char* sc = static_cast<unsigned char*>(base);
  hipStream_t s = static_cast<hipStream_t>(stream);
  PulseDev* d_desc = reinterpret_cast<PulseDev*>(sc + o_desc);
  PO_HIP(hipMemcpyAsync(d_desc, g_noalloc_desc, sizeof(PulseDev) * size_t(n), hipMemcpyHostToDevice, s));
  PO_TRY(synth_into(specs, d_coeff, d_A, nullptr, d_A_edge, d_scale, s, b, d_desc,
                    reinterpret_cast<double*>(sc + o_spec), reinterpret_cast<double*>(sc + o_part),
                    reinterpret_cast<double*>(sc + o_scl)));
  return evolve_into(b, d_desc, d_A, d_A_edge, d_f, d_J, s, reinterpret_cast<double*>(sc + o_units),
                     reinterpret_cast<double*>(sc + o_ranges), false);
}

po_status po_timer_enable(int on) {
  std::lock_guard<std::mutex> lk(g_timer_mu);
  if (on && !g_counts) {
    void* p = nullptr;
    PO_HIP(hipMalloc(&p, sizeof(unsigned long long) * kSeriesVariants));
    PO_HIP(hipMemset(p, 0, sizeof(unsigned long long) * kSeriesVariants));
    g_counts = static_cast<unsigned long long*>(p);
  }
  g_timer_on = on != 0;
  return PO_OK;
}

po_status po_timer_mode_steps(uint64_t* counts, int32_t n) {
  if (!counts || n < 1) return set_error(PO_ERR_INVALID, "counts must hold at least one entry");
  unsigned long long h[kSeriesVariants] = {};
  {
    std::lock_guard<std::mutex> lk(g_timer_mu);
    if (g_counts) {
      PO_HIP(hipDeviceSynchronize());
      PO_HIP(hipMemcpy(h, g_counts, sizeof h, hipMemcpyDeviceToHost));
      PO_HIP(hipMemset(g_counts, 0, sizeof h));
    }
  }
  for (int i = 0; i < n; ++i) counts[i] = i < kSeriesVariants ? uint64_t(h[i]) : 0;
  return PO_OK;
}

po_status po_timer_read(double* ms_total, int64_t* calls) {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  {
    std::lock_guard<std::mutex> lk(g_timer_mu);
    ev.swap(g_timer_events);
  }
  double total = 0.0;
  po_status st = PO_OK;
  for (auto& p : ev) {
    float ms = 0.0f;
    hipError_t e = hipEventSynchronize(p.second);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.first, p.second);
    if (e != hipSuccess && st == PO_OK) st = device_error(e, "hipEventElapsedTime");
    total += ms;
    (void)hipEventDestroy(p.first);
    (void)hipEventDestroy(p.second);
  }
  if (ms_total) *ms_total = total;
  if (calls) *calls = int64_t(ev.size());
  return st;
}

static po_status check_de(const po_de_params* p) {
  if (!p) return set_error(PO_ERR_INVALID, "params is NULL");
  if (p->pop < 4) return set_error(PO_ERR_INVALID, "pop must be >= 4");
  if (p->dim < 1) return set_error(PO_ERR_INVALID, "dim must be >= 1");
  if (p->n_s < 0) return set_error(PO_ERR_INVALID, "n_s must be >= 0");
  if (!(p->F >= 0.0 && p->F <= 2.0)) return set_error(PO_ERR_INVALID, "F must be in [0, 2]");
  if (!(p->CR >= 0.0 && p->CR <= 1.0)) return set_error(PO_ERR_INVALID, "CR must be in [0, 1]");
  if (!(p->lo < p->hi) || !std::isfinite(p->lo) || !std::isfinite(p->hi))
    return set_error(PO_ERR_INVALID, "need finite lo < hi");
  return PO_OK;
}

po_status po_de_propose(const po_de_params* prm, int64_t generation, const double* d_pop, double* d_trial,
                        int32_t* d_idx, void* stream) {
  PO_TRY(check_de(prm));
  const size_t nd = size_t(prm->pop) * prm->dim;
  PO_TRY(check_device_range(d_pop, sizeof(double) * nd, 8, "d_pop"));
  PO_TRY(check_device_range(d_trial, sizeof(double) * nd, 8, "d_trial"));
  if (d_idx) PO_TRY(check_device_range(d_idx, sizeof(int32_t) * 4 * prm->pop, 4, "d_idx"));
  return launch_de_propose(*prm, generation, d_pop, d_trial, d_idx, static_cast<hipStream_t>(stream));
}

po_status po_de_select(const po_de_params* prm, double* d_pop, double* d_fit, const double* d_trial,
                       const double* d_trial_fit, const uint8_t* d_mask, void* stream) {
  PO_TRY(check_de(prm));
  const size_t nd = size_t(prm->pop) * prm->dim;
  PO_TRY(check_device_range(d_pop, sizeof(double) * nd, 8, "d_pop"));
  PO_TRY(check_device_range(d_fit, sizeof(double) * prm->pop, 8, "d_fit"));
  PO_TRY(check_device_range(d_trial, sizeof(double) * nd, 8, "d_trial"));
  PO_TRY(check_device_range(d_trial_fit, sizeof(double) * prm->pop, 8, "d_trial_fit"));
  if (d_mask) PO_TRY(check_device_range(d_mask, prm->pop, 1, "d_mask"));
  return launch_de_select(*prm, d_pop, d_fit, d_trial, d_trial_fit, d_mask, static_cast<hipStream_t>(stream));
}

po_status po_de_generation(const po_de_params* prm, int64_t generation, const po_pulse_spec* spec, const po_grid* grid,
                           double* d_pop, double* d_fit, double* d_trial, double* d_trial_fit, void* stream) {
  PO_TRY(check_de(prm));
  PO_TRY(check_specs(1, spec));
  PO_TRY(check_grids(1, grid));
  if (prm->dim != 4 * spec->n_s) return set_error(PO_ERR_INVALID, "dim must equal 4 n_s");
  const int32_t n = prm->pop;
  const size_t nd = size_t(n) * prm->dim;
  PO_TRY(check_device_range(d_pop, sizeof(double) * nd, 8, "d_pop"));
  PO_TRY(check_device_range(d_fit, sizeof(double) * n, 8, "d_fit"));
  PO_TRY(check_device_range(d_trial, sizeof(double) * nd, 8, "d_trial"));
  PO_TRY(check_device_range(d_trial_fit, sizeof(double) * n, 8, "d_trial_fit"));
  std::vector<po_pulse_spec> specs(n, *spec);
  std::vector<po_grid> grids(n, *grid);
  std::vector<PulseDev> h(n);
  Batch b;
  PO_TRY(build_batch(n, specs.data(), grids.data(), h.data(), &b));
  hipStream_t s = static_cast<hipStream_t>(stream);
  Scratch desc, tab, edge;
  PO_TRY(upload(h, desc, s));
  PO_TRY(tab.alloc(sizeof(double) * 2 * b.total_rows, s));
  PO_TRY(edge.alloc(sizeof(double) * 4 * n, s));
  const PulseDev* d_desc = static_cast<PulseDev*>(desc.ptr);
  double* d_A = static_cast<double*>(tab.ptr);
  double* d_edge = static_cast<double*>(edge.ptr);
  PO_TRY(launch_de_propose(*prm, generation, d_pop, d_trial, nullptr, s));
  PO_TRY(synth_impl(n, specs.data(), d_trial, d_A, nullptr, d_edge, nullptr, s, b, d_desc));
  PO_TRY(evolve_impl(b, d_desc, d_A, d_edge, nullptr, d_trial_fit, s));
  PO_TRY(launch_de_select(*prm, d_pop, d_fit, d_trial, d_trial_fit, nullptr, s));
  return check_finite(d_trial_fit, n, "d_trial_fit", s);
}

static po_status check_jde(const po_jde_params* p) {
  if (!p) return set_error(PO_ERR_INVALID, "params is NULL");
  if (p->islands < 1 || p->islands > 64) return set_error(PO_ERR_INVALID, "islands must be in [1, 64]");
  if (p->pop < 4 || p->pop % p->islands != 0 || p->pop / p->islands < 4)
    return set_error(PO_ERR_INVALID, "pop must be a multiple of islands with at least 4 members per island");
  if (p->dim < 1) return set_error(PO_ERR_INVALID, "dim must be >= 1");
  if (p->n_s < 0) return set_error(PO_ERR_INVALID, "n_s must be >= 0");
  if (!(p->tau1 >= 0.0 && p->tau1 <= 1.0) || !(p->tau2 >= 0.0 && p->tau2 <= 1.0))
    return set_error(PO_ERR_INVALID, "tau1 and tau2 must be in [0, 1]");
  if (!(p->F_lo >= 0.0 && p->F_lo <= p->F_hi && p->F_hi <= 2.0))
    return set_error(PO_ERR_INVALID, "need 0 <= F_lo <= F_hi <= 2");
  if (!(p->lo < p->hi) || !std::isfinite(p->lo) || !std::isfinite(p->hi))
    return set_error(PO_ERR_INVALID, "need finite lo < hi");
  return PO_OK;
}

static po_status check_jde_state(const po_jde_params* prm, const double* d_pop, const double* d_fit,
                                 const double* d_fcr) {
  const size_t nd = size_t(prm->pop) * prm->dim;
  PO_TRY(check_device_range(d_pop, sizeof(double) * nd, 8, "d_pop"));
  if (d_fit) PO_TRY(check_device_range(d_fit, sizeof(double) * prm->pop, 8, "d_fit"));
  PO_TRY(check_device_range(d_fcr, sizeof(double) * 2 * prm->pop, 8, "d_fcr"));
  return PO_OK;
}

po_status po_jde_propose(const po_jde_params* prm, int64_t generation, const double* d_pop, const double* d_fcr,
                         double* d_trial, double* d_trial_fcr, int32_t* d_idx, void* stream) {
  PO_TRY(check_jde(prm));
  PO_TRY(check_jde_state(prm, d_pop, nullptr, d_fcr));
  PO_TRY(check_jde_state(prm, d_trial, nullptr, d_trial_fcr));
  if (d_idx) PO_TRY(check_device_range(d_idx, sizeof(int32_t) * 4 * prm->pop, 4, "d_idx"));
  return launch_jde_propose(*prm, generation, d_pop, d_fcr, d_trial, d_trial_fcr, d_idx,
                            static_cast<hipStream_t>(stream));
}

po_status po_jde_select(const po_jde_params* prm, double* d_pop, double* d_fit, double* d_fcr, const double* d_trial,
                        const double* d_trial_fit, const double* d_trial_fcr, const uint8_t* d_mask, void* stream) {
  PO_TRY(check_jde(prm));
  PO_TRY(check_jde_state(prm, d_pop, d_fit, d_fcr));
  PO_TRY(check_jde_state(prm, d_trial, d_trial_fit, d_trial_fcr));
  if (d_mask) PO_TRY(check_device_range(d_mask, prm->pop, 1, "d_mask"));
  return launch_jde_select(*prm, d_pop, d_fit, d_fcr, d_trial, d_trial_fit, d_trial_fcr, d_mask,
                           static_cast<hipStream_t>(stream));
}

po_status po_island_migrate(const po_jde_params* prm, double* d_pop, double* d_fit, double* d_fcr, void* stream) {
  PO_TRY(check_jde(prm));
  if (prm->dim > 64) return set_error(PO_ERR_INVALID, "migration supports dim <= 64");
  PO_TRY(check_jde_state(prm, d_pop, d_fit, d_fcr));
  return launch_island_migrate(*prm, d_pop, d_fit, d_fcr, static_cast<hipStream_t>(stream));
}

po_status po_jde_generation(const po_jde_params* prm, int64_t generation, const po_pulse_spec* spec, const po_grid* grid,
                            double* d_pop, double* d_fit, double* d_fcr, double* d_trial, double* d_trial_fit,
                            double* d_trial_fcr, void* stream) {
  PO_TRY(check_jde(prm));
  PO_TRY(check_specs(1, spec));
  PO_TRY(check_grids(1, grid));
  if (prm->dim != 4 * spec->n_s) return set_error(PO_ERR_INVALID, "dim must equal 4 n_s");
  PO_TRY(check_jde_state(prm, d_pop, d_fit, d_fcr));
  PO_TRY(check_jde_state(prm, d_trial, d_trial_fit, d_trial_fcr));
  const int32_t n = prm->pop;
  std::vector<po_pulse_spec> specs(n, *spec);
  std::vector<po_grid> grids(n, *grid);
  std::vector<PulseDev> h(n);
  Batch b;
  PO_TRY(build_batch(n, specs.data(), grids.data(), h.data(), &b));
  hipStream_t s = static_cast<hipStream_t>(stream);
  Scratch desc, tab, edge;
  PO_TRY(upload(h, desc, s));
  PO_TRY(tab.alloc(sizeof(double) * 2 * b.total_rows, s));
  PO_TRY(edge.alloc(sizeof(double) * 4 * n, s));
  const PulseDev* d_desc = static_cast<PulseDev*>(desc.ptr);
  double* d_A = static_cast<double*>(tab.ptr);
  double* d_edge = static_cast<double*>(edge.ptr);
  PO_TRY(launch_jde_propose(*prm, generation, d_pop, d_fcr, d_trial, d_trial_fcr, nullptr, s));
  PO_TRY(synth_impl(n, specs.data(), d_trial, d_A, nullptr, d_edge, nullptr, s, b, d_desc));
  PO_TRY(evolve_impl(b, d_desc, d_A, d_edge, nullptr, d_trial_fit, s));
  return launch_jde_select(*prm, d_pop, d_fit, d_fcr, d_trial, d_trial_fit, d_trial_fcr, nullptr, s);
}

}  // extern "C"
