// Internal declarations shared by the translation units of libpairopt.so (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "pairopt.h"

namespace po {

// ------------------------------------------------------------------------------- errors
po_status set_error(po_status s, const char* fmt, ...);
po_status device_error(hipError_t e, const char* what);

#define PO_HIP(call)                                                  \
  do {                                                                \
    hipError_t e__ = (call);                                          \
    if (e__ != hipSuccess) return ::po::device_error(e__, #call);     \
  } while (0)

#define PO_TRY(expr)                          \
  do {                                        \
    po_status s__ = (expr);                   \
    if (s__ != PO_OK) return s__;             \
  } while (0)

// Host-side check that [p, p + bytes) lies in one device allocation of the current device.
po_status check_device_range(const void* p, size_t bytes, size_t align, const char* name);

// ---------------------------------------------------------------- per-pulse descriptors
// One record per pulse, uploaded to device memory for every multi-pulse launch.
constexpr int kUnit = 64;         // momentum modes per reduction unit, one wave (fixed: sets the sum order)
constexpr int kItem = 256;        // modes per workgroup in the default (non-plan) evolution launch
constexpr int kSelBlock = 512;    // modes per series-selection block: a multiple of every launch's item
constexpr int kChunkSteps = 256;  // time steps per LDS chunk of the per-mode kernels (and per table range)
constexpr int kMaxLines = 8192;   // spectral lines per pulse
constexpr int kMaxNs = 64;        // B-spline coefficients per spectral function
constexpr int kMaxSub = 8;        // sample points per step of po_field_samples

struct PulseDev {
  int64_t tab_off;    // first table row (rows of 2 doubles)
  int64_t mode_off;   // first mode in the packed f array
  int64_t coeff_off;  // first coefficient (doubles)
  int64_t spec_off;   // first spectral record in the scratch spectra (4 doubles per line)
  int32_t nt, ns, order, nlines;
  int32_t nmin, norm, stat_blocks;
  int32_t chk_off;    // first 256-step chunk of this pulse in the batch (table ranges per chunk)
  int32_t n[3];
  int64_t unit_off;   // first 64-mode reduction unit of this pulse in the batch
  int32_t nunits;
  int32_t item_off;   // first workgroup item of this pulse in the default evolution launch
  int32_t nitems;
  int32_t blk_off;    // first series-selection block (kSelBlock modes) of this pulse in the batch
  double T, dt, dw, wmin, wmax, norm_value, dv;
  double lo[3], dp[3];  // p_d = lo_d + (i + 1/2) dp_d; dp_d = 0 for a sheet (then p_d = lo_d)
};

struct Batch {
  int32_t n_pulses = 0;
  int64_t total_rows = 0, total_modes = 0, total_coeff = 0, total_spec = 0;
  int64_t total_units = 0;
  int32_t total_items = 0;     // workgroups of the default evolution launch
  int32_t total_blocks = 0;    // series-selection blocks (kSelBlock modes, per pulse)
  int32_t total_chunks = 0;    // kChunkSteps-step chunks of all pulses
  int32_t max_stat_blocks = 0; // largest per-pulse block count of the field statistics pass
  int32_t max_nt = 0;
  int32_t max_lines = 0;       // most spectral lines of any pulse
  int32_t max_ns = 0;          // most B-spline coefficients per spectral function of any pulse
  bool uniform = true;         // all pulses share nt/grid (lets kernels skip the binary search)
};

po_status validate_spec(const po_pulse_spec& s, int i);
po_status validate_grid(const po_grid& g, int i);
// Fills host descriptors; specs/grids may be NULL when a call does not need them.
po_status build_batch(int32_t n, const po_pulse_spec* specs, const po_grid* grids, PulseDev* out,
                      Batch* b);

// Stream-ordered scratch buffer released on destruction (hipFreeAsync on the same stream).
struct Scratch {
  void* ptr = nullptr;
  hipStream_t stream = nullptr;
  ~Scratch() {
    if (ptr) (void)hipFreeAsync(ptr, stream);
  }
  po_status alloc(size_t bytes, hipStream_t s);
};

// --------------------------------------------------------------------- kernel launchers
po_status launch_synth(const Batch& b, const PulseDev* d_desc, const double* d_coeff, double* d_spec,
                       double* d_part, double* d_scale_ws, double* d_A, double* d_E, double* d_A_edge,
                       double* d_scale_out, hipStream_t s);
// Scaled field samples at t_i + (n + offsets[r]) dt (rows per pulse nt n_sub + with_end, from
// desc.tab_off); any of d_E, d_Ed, d_A, d_A_edge may be NULL.
po_status launch_samples(const Batch& b, const PulseDev* d_desc, const double* d_coeff, double* d_spec, double* d_part,
                         double* d_scale_ws, int n_sub, const double* offsets, int with_end, double* d_E,
                         double* d_Ed, double* d_A, double* d_A_edge, double* d_scale_out, hipStream_t s);
// Adjoint of the synthesis: d_lines scratch [sum lines][8 max_ns]; d_A, d_A_edge, d_E the (scaled) tables of
// the pulses and d_scale their scale; d_gA [sum nt][2] and d_gedge [n][2][2] (or NULL) the gradient of
// J with respect to the tables.  Writes dJ/dc, the energy U and dU/dc (NULL to skip).
po_status launch_synth_adjoint(const Batch& b, const PulseDev* d_desc, const double* d_coeff, const double* d_gA,
                               const double* d_gedge, const double* d_A, const double* d_A_edge, const double* d_E,
                               const double* d_scale, double* d_lines, double* d_grad, double* d_U, double* d_gU,
                               hipStream_t s);
// Yield gradient (grad.hip): d_part [sum items_i nt_i][2] item partials at d_goff[i]; d_epart [items][4].
po_status launch_yield_grad(const Batch& b, const PulseDev* d_desc, const double* d_A, const double* d_A_edge,
                            const int2* d_sel, const int64_t* d_goff, double* d_part, double* d_epart, double* d_units,
                            double* d_gA, double* d_gedge, hipStream_t s);
// Launch shape of the evolution kernel.  threads: lanes per workgroup (64, 128, 256);
// mpl: modes per lane (1, 2); persistent: workgroups pull items from a device queue.
struct EvolveConfig {
  int threads = 256;
  int mpl = 1;
  int persistent = 0;
};
// Per-block series selection of the yield gradient: x = variant of kFitDegree (or kFineHalving),
// y = number of angle halvings, one int2 per kSelBlock modes of each pulse (total_blocks).
po_status launch_block_select(const Batch& b, const PulseDev* d_desc, const double* d_A, int2* d_bsel,
                              hipStream_t s);
// Range of the table per 256-step chunk of each pulse, d_ranges [total_chunks][4] = (min A_x,
// max A_x, min A_y, max A_y); the second-order evolution picks its series variant per chunk and
// selection block from it.  The evolution launches below take this array; d_units holds
// total_units doubles (one partial sum per 64 modes).
po_status launch_chunk_ranges(const Batch& b, const PulseDev* d_desc, const double* d_A, double* d_ranges,
                              hipStream_t s);
po_status launch_evolve_grid(const Batch& b, const PulseDev* d_desc, const double* d_A, const double* d_A_edge,
                             const double* d_ranges, double* d_f, double* d_units, hipStream_t s);
// Persistent launch: items are {pulse, first mode} pairs of cfg.threads * cfg.mpl modes each,
// taken in queue order through the counter (reset on the stream before the launch).
po_status launch_evolve_persistent(const EvolveConfig& cfg, int n_pulses, const PulseDev* d_desc, const double* d_A,
                                   const double* d_A_edge, const double* d_ranges, const int2* d_queue, int n_items,
                                   int n_workgroups, int* d_counter, double* d_f, double* d_units, hipStream_t s);
int evolve_workgroups_per_cu(const EvolveConfig& cfg);
// Fourth-order (Magnus) evolution: table ranges over both nodes of every step per chunk
// (d_ranges [total_chunks][4]) and one workgroup per 256 modes; d_Ag is [sum nt][2 nodes][2] with
// desc.tab_off counted in steps.
po_status launch_chunk_ranges4(const Batch& b, const PulseDev* d_desc, const double* d_Ag, double* d_ranges,
                               hipStream_t s);
po_status launch_evolve4_grid(const Batch& b, const PulseDev* d_desc, const double* d_Ag, const double* d_A_edge,
                              const double* d_ranges, double* d_f, double* d_units, hipStream_t s);
// Split-operator evolution (order 2: Strang, order 4: triple jump): table ranges into d_ranges
// [total_chunks][4], then one workgroup per 256 modes; d_At is [sum nt][1 or 3][2], desc.tab_off in steps.
po_status launch_evolve_split_grid(const Batch& b, int order, const PulseDev* d_desc, const double* d_At,
                                   const double* d_A_edge, double* d_ranges, double* d_f, double* d_units,
                                   hipStream_t s);
// Kinetic equation (qke.hip): tables at the 2 nt + 1 half-step points, desc.tab_off in points.
po_status launch_qke_grid(const Batch& b, const PulseDev* d_desc, const double* d_E, const double* d_Ed,
                          const double* d_A, int linear, double* d_f, double* d_units, hipStream_t s);
po_status launch_unit_sums_from_f(const Batch& b, const PulseDev* d_desc, const double* d_f, double* d_units,
                                  hipStream_t s);
po_status launch_yield_from_units(const Batch& b, const PulseDev* d_desc, const double* d_units, double* d_J,
                                  hipStream_t s);
// Plans (plan.hip): evolution of caller tables with a plan's launch shape.
po_status plan_evolve(const po_plan* plan, int32_t n, const po_pulse_spec* specs, const po_grid* grids,
                      const double* d_A, const double* d_edge, double* d_f, double* d_J, hipStream_t s);
// Kernel timers (api.hip): start returns true (and records *e0) when timers are enabled;
// timer_count enqueues the per-variant mode-step count of an evolution launch from its chunk
// ranges (no-op when disabled).
constexpr int kSeriesVariants = 9;  // T fits of degree 4..11 (tan_fit.hpp), then the angle-halving path
bool timer_start(hipStream_t s, hipEvent_t* e0);
void timer_stop(hipStream_t s, hipEvent_t e0);
po_status timer_count(int n_pulses, const PulseDev* d_desc, const double* d_ranges, hipStream_t s);
po_status launch_count_mode_steps(int n_pulses, const PulseDev* d_desc, const double* d_ranges,
                                  unsigned long long* d_counts, hipStream_t s);

po_status launch_de_propose(const po_de_params& p, int64_t gen, const double* d_pop, double* d_trial,
                            int32_t* d_idx, hipStream_t s);
po_status launch_de_select(const po_de_params& p, double* d_pop, double* d_fit, const double* d_trial,
                           const double* d_trial_fit, const uint8_t* d_mask, hipStream_t s);

po_status launch_jde_propose(const po_jde_params& p, int64_t gen, const double* d_pop, const double* d_fcr,
                             double* d_trial, double* d_tfcr, int32_t* d_idx, hipStream_t s);
po_status launch_jde_select(const po_jde_params& p, double* d_pop, double* d_fit, double* d_fcr, const double* d_trial,
                            const double* d_tfit, const double* d_tfcr, const uint8_t* d_mask, hipStream_t s);
po_status launch_island_migrate(const po_jde_params& p, double* d_pop, double* d_fit, double* d_fcr, hipStream_t s);

}  // namespace po
