/*
 * pairopt.h -- C ABI of libpairopt.so, the gfx950 (MI355X) implementation of the pair-yield
 * objective of Fillion-Gourdeau, Hebenstreit, Gagnon & MacLean, "Pulse shape optimization
 * for electron-positron production in rotating fields" (arXiv:1704.08919), and of the
 * differential-evolution loop that maximises it.
 *
 * Units: c = hbar = m = 1 with the charge absorbed into the fields (eE -> E, eA -> A), so the
 * Schwinger field is 1 (Sec. II).  The field E(t) = (E_x, E_y, 0) lies in the x-y plane; p_z is
 * the out-of-plane momentum (the paper's e_1 axis).
 *
 * Conventions shared by every call
 *  - Pointers named d_* are DEVICE pointers on the current HIP device (e.g. the data pointer
 *    of a contiguous torch tensor of the stated dtype).  They are owned by the caller; the
 *    library never frees them and keeps none of them after the call returns.  Each one is
 *    checked on the host before any work is enqueued: it must lie inside one device
 *    allocation that is large enough for the documented extent, and be 8-byte aligned
 *    (4-byte for int32/float, 2-byte for bf16, 1-byte for uint8).
 *  - Host arrays (specs, grids, params) are read during the call only.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  Every call is
 *    asynchronous on that stream; results are valid once the stream reaches them.
 *  - Work buffers that a call needs beyond its arguments are taken from the stream-ordered
 *    memory pool (hipMallocAsync / hipFreeAsync on `stream`), so calls on different streams
 *    never share scratch memory.
 *  - Errors: every argument is validated before anything is enqueued.  Invalid arguments
 *    return PO_ERR_INVALID, HIP failures PO_ERR_DEVICE; in both cases po_last_error() gives a
 *    message (thread-local).  No C++ exception crosses the ABI.  Nothing is enqueued when a
 *    call returns an error from validation.  With po_set_check_finite enabled, the calls it
 *    lists also return PO_ERR_NUMERIC for non-finite results (and are then synchronous).
 *  - Results are bitwise reproducible: reductions use a fixed order that depends only on the
 *    sizes of the problem, not on launch shapes or scheduling.
 *
 * Packed multi-pulse layout: pulse i owns nt_i table rows, starting at row sum_{j<i} nt_j,
 * and M_i = n_x n_y n_z momentum modes, starting at sum_{j<i} M_j.  Coefficients of pulse i
 * start at sum_{j<i} 4 n_s,j and are laid out [2 components (x, y)][2 kinds (amplitude,
 * phase)][n_s].
 */
#ifndef PAIROPT_H
#define PAIROPT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PO_OK = 0,
  PO_ERR_INVALID = -1,     /* bad argument; nothing was enqueued */
  PO_ERR_DEVICE = -2,      /* a HIP call failed */
  PO_ERR_NOMEM = -3,       /* the stream-ordered pool could not supply a work buffer */
  PO_ERR_NUMERIC = -4,     /* a non-finite value was found where a finite one is required */
  PO_ERR_UNSUPPORTED = -5  /* valid request the library does not implement */
} po_status;

enum { PO_NORM_NONE = 0, PO_NORM_PEAK = 1, PO_NORM_ENERGY = 2 };

/* Pulse description (Sec. III).
 *  n_s            B-spline coefficients per spectral function (amplitude and phase each).
 *  order          B-spline order k in the paper's convention (degree k - 1; 4 = cubic).
 *                 Knots: multiplicity k at omega_min and omega_max, n_s - k equidistant
 *                 interior knots (Sec. III, clamped knot vector).  Requires 1 <= k <= n_s <= 64.
 *  omega_min/max  band [omega_min, omega_max] of angular frequencies, in units of m.
 *                 omega_min / Delta omega must be an integer to 1e-9, Delta omega = 2 pi / T.
 *  T              pulse length; time runs over [-T/2, T/2]; sampled lines
 *                 Omega_j = (N_min + j) Delta omega, j = 0..N, N = floor((omega_max -
 *                 omega_min)/Delta omega + 1e-9) (Sec. III, Eq. field).  N + 1 <= 8192.
 *  nt             time steps, dt = T / nt, 2 <= nt <= 2^24.
 *  norm           PO_NORM_PEAK: scale so that max |E| over the nt + 1 step nodes equals
 *                 norm_value; PO_NORM_ENERGY: scale so that U = int |E|^2 dt (midpoint rule)
 *                 equals norm_value (Sec. III, Eq. energy); PO_NORM_NONE: no scaling.
 *                 The amplitude coefficients are relative weights (Sec. IV B). */
typedef struct {
  int32_t n_s;
  int32_t order;
  double omega_min;
  double omega_max;
  double T;
  int32_t nt;
  int32_t norm;
  double norm_value;
} po_pulse_spec;

/* Cell-centred momentum grid: p_d = lo_d + (i + 1/2)(hi_d - lo_d)/n_d, i = 0..n_d - 1; mode
 * index = (i_z n_y + i_y) n_x + i_x.  A dimension with n_d = 1 and lo_d = hi_d is a sheet
 * (p_d = lo_d, no measure factor), e.g. the p_z = 0 plane of the paper's 2-D problem (Sec. V B).
 * Requires n_d >= 1, lo_d <= hi_d, and lo_d < hi_d whenever n_d > 1. */
typedef struct {
  int32_t n[3];
  double lo[3];
  double hi[3];
} po_grid;

/* Library version of this ABI (bumped on any incompatible change). */
int po_abi_version(void);

/* Thread-local message describing the last non-OK status returned on this thread. */
const char* po_last_error(void);

/* ---------------------------------------------------------------------------------------
 * po_pulse_synth -- coefficients -> field tables (Sec. III: B-spline expansions Eq.
 * coeff_basis_E / coeff_basis_phi, sampled spectrum, Eq. field with the Hann window Eq. hann,
 * vector potential Eq. vector_potential with A(t_f) = 0, and the global renormalisation of
 * Sec. IV B).
 *  d_coeff   [sum 4 n_s] double: amplitude coefficients a^(E) are used as given; a phase
 *            coefficient c maps to a^(phi) = pi (c + 1).
 *  d_A       out [sum nt][2] double: scaled A(t) at the step midpoints t_i + (n + 1/2) dt.
 *  d_E       out [sum nt][2] double or NULL: scaled E(t) at the same midpoints.
 *  d_A_edge  out [n_pulses][2][2] double: scaled A(t_i) and A(t_f) (= 0).
 *  d_scale   out [n_pulses] double or NULL: the applied scale factor s (E = s E_raw).
 * Returns PO_ERR_INVALID for n_pulses < 1 or an invalid spec.
 * --------------------------------------------------------------------------------------- */
po_status po_pulse_synth(int32_t n_pulses, const po_pulse_spec* specs, const double* d_coeff,
                         double* d_A, double* d_E, double* d_A_edge, double* d_scale, void* stream);

/* ---------------------------------------------------------------------------------------
 * po_evolve_modes -- per-mode time evolution and projection (Sec. II A: momentum-space Dirac
 * equation Eq. dirac_eq_mom, initial negative-energy spinors and the pair density
 * Eq. pair_prod_homo summed over both spin labels) for ANY A table, not only a synthesised one.
 * Each step applies the exact exponential of the Hamiltonian frozen at the step midpoint
 * (second-order, unitary).  The Hamiltonian splits into two 2x2 blocks that are evolved
 * separately and f is their sum, f in [0, 2].
 *  specs     only nt and T are read (dt = T / nt).
 *  d_A       [sum nt][2] double: A at the step midpoints.  The tables are not checked on the
 *            host: a non-finite or absurdly large entry (|A dt| beyond ~2^60) gives non-finite or
 *            meaningless f and J, and the call still completes.
 *  d_A_edge  [n_pulses][2][2] double: A(t_i) (initial state) and A(t_f) (projection).
 *  d_f       out [sum M] double or NULL: f(t_f, p) per mode.
 *  d_J       out [n_pulses] double or NULL: J = Delta V sum_p f (Sec. IV A, Eq. opt_prob).
 *            At least one of d_f, d_J must be non-NULL.
 *  plan      NULL (one workgroup per 256 modes) or a plan created for the same specs and
 *            grids, whose launch shape and queue are then used.
 * --------------------------------------------------------------------------------------- */
struct po_plan;
po_status po_evolve_modes(int32_t n_pulses, const po_pulse_spec* specs, const po_grid* grids,
                          const double* d_A, const double* d_A_edge, double* d_f, double* d_J,
                          const struct po_plan* plan, void* stream);

/* ---------------------------------------------------------------------------------------
 * po_pair_yield -- J = Delta V sum_p f(p) per pulse (Sec. IV A, Eq. opt_prob, midpoint rule on
 * the cell-centred grid).  Same summation order as the fused reduction of po_evolve_modes,
 * so both give identical bits.
 *  d_f  [sum M] double;  d_J  out [n_pulses] double.
 * --------------------------------------------------------------------------------------- */
po_status po_pair_yield(int32_t n_pulses, const po_grid* grids, const double* d_f, double* d_J,
                        void* stream);

/* ---------------------------------------------------------------------------------------
 * po_evaluate -- fused po_pulse_synth -> po_evolve_modes -> J.  Arguments as above; d_E is
 * not produced; d_f may be NULL.
 * --------------------------------------------------------------------------------------- */
po_status po_evaluate(int32_t n_pulses, const po_pulse_spec* specs, const po_grid* grids,
                      const double* d_coeff, double* d_A, double* d_A_edge, double* d_scale,
                      double* d_f, double* d_J, const struct po_plan* plan, void* stream);

/* ---------------------------------------------------------------------------------------
 * po_evaluate_noalloc -- po_evaluate (plan NULL) for callers that cannot allocate: code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation.  Same kernels, same
 * results bit for bit; it calls no hipMalloc, hipFree or other allocating routine.  Its scratch
 * (pulse descriptors, spectra, normalisation partials, per-64-mode partial sums and per-chunk
 * table ranges) lives in one file-scope device array of 64 MiB that each device holds from
 * the library's first use there until the process ends; the caller passes inputs and outputs as
 * for po_evaluate.  Limits: at most 4096 pulses, and a batch whose scratch (about
 * 8 (sum 4 lines + pulses (statistic blocks + 1) + sum modes / 64 + 4 sum ceil(nt/256)) bytes
 * plus descriptors, each part rounded up to 256 bytes) exceeds 64 MiB is rejected with
 * PO_ERR_INVALID before anything is enqueued.  Every call on a device shares that device's
 * array: calls that overlap on one device (on different streams, or from several threads) race
 * and must not be made; calls on one stream are ordered.  Kernel timers do not bracket it.
 * --------------------------------------------------------------------------------------- */
po_status po_evaluate_noalloc(int32_t n_pulses, const po_pulse_spec* specs, const po_grid* grids,
                              const double* d_coeff, double* d_A, double* d_A_edge, double* d_scale,
                              double* d_f, double* d_J, void* stream);

/* ---------------------------------------------------------------------------------------
 * po_field_samples -- scaled E, dE/dt and A of synthesised pulses at chosen points inside
 * every step (Sec. III, Eq. field, Eq. hann and Eq. vector_potential, with the scale of the
 * spec's normalisation as in po_pulse_synth).  Row r of pulse i is the time
 * t_i + (r / n_sub + offsets[r % n_sub]) dt for r < nt n_sub, and t_f for the extra last row
 * when with_end != 0; pulse i owns nt_i n_sub + with_end rows, packed in pulse order.
 *  n_sub     points per step, 1..8;  offsets  host [n_sub], each in [0, 1] (in units of dt).
 *  d_E, d_Ed, d_A  out [rows][2] double or NULL (dE/dt is the exact derivative of the sum).
 *  d_A_edge  out [n_pulses][2][2] double or NULL: A(t_i), A(t_f).
 *  d_scale   out [n_pulses] double or NULL.  At least one of d_E, d_Ed, d_A, d_A_edge is needed.
 * Offsets {0, 1/2} with with_end = 1 give the 2 nt + 1 points of po_qke_modes; offsets
 * {1/2 - sqrt3/6, 1/2 + sqrt3/6} the Gauss-Legendre nodes of po_evolve_modes_m4.
 * --------------------------------------------------------------------------------------- */
po_status po_field_samples(int32_t n_pulses, const po_pulse_spec* specs, const double* d_coeff,
                           int32_t n_sub, const double* offsets, int32_t with_end, double* d_E,
                           double* d_Ed, double* d_A, double* d_A_edge, double* d_scale, void* stream);

/* ---------------------------------------------------------------------------------------
 * po_qke_modes -- pair density from the quantum kinetic equation of Sec. II B (the
 * six-component system Eq. qke with the matrix Eq. matrix, chi(t_i) = (1,0,0,0,0,0),
 * f = 1 - chi_1 at t_f), integrated by classical fourth-order Runge-Kutta with nt steps.
 *  specs     only nt and T are read.
 *  d_E, d_Ed, d_A  [sum (2 nt + 1)][2] double: E, dE/dt and A at t_i + h dt/2, h = 0..2 nt.
 *  linear    0: rotating field (Q = sqrt(X)/omega^2, R = e_perp omega (E x dE/dt)_z / X,
 *            X = omega^2 |E|^2 - (E.P)^2, and Q = R = 0 where X = 0); 1: field along x only,
 *            with the signed Q = E_x sqrt(1 + P_y^2 + p_z^2)/omega^2 and R = 0.
 *  d_f, d_J  as for po_evolve_modes (at least one non-NULL; J uses the same fixed-order sum).
 * f is the spin-summed density of po_evolve_modes in the limit dt -> 0.
 * --------------------------------------------------------------------------------------- */
po_status po_qke_modes(int32_t n_pulses, const po_pulse_spec* specs, const po_grid* grids,
                       const double* d_E, const double* d_Ed, const double* d_A, int32_t linear,
                       double* d_f, double* d_J, void* stream);

/* ---------------------------------------------------------------------------------------
 * po_evolve_modes_m4 -- po_evolve_modes with a fourth-order step: the fourth-order Magnus
 * integrator with two Gauss-Legendre nodes per step (Blanes, Casas, Oteo & Ros, Phys. Rep. 470
 * (2009) 151), the higher-order Dirac scheme that Sec. V C names as future work.  Same
 * initial state, projection, f and J as po_evolve_modes.
 *  d_Ag      [sum nt][2 nodes][2] double, 16-byte aligned: A at t_i + (n + 1/2 -+ sqrt3/6) dt.
 *  d_A_edge  [n_pulses][2][2] double: A(t_i), A(t_f).
 * --------------------------------------------------------------------------------------- */
po_status po_evolve_modes_m4(int32_t n_pulses, const po_pulse_spec* specs, const po_grid* grids,
                             const double* d_Ag, const double* d_A_edge, double* d_f, double* d_J,
                             void* stream);

/* ---------------------------------------------------------------------------------------
 * po_evolve_modes_split -- po_evolve_modes with a split-operator step: the frozen Hamiltonian
 * splits into the part the field does not touch, alpha_z p_z + beta m, and the field-driven
 * transverse part alpha_x P_x + alpha_y P_y, each factor exponentiated exactly (Sec. II A names a
 * second-order split-operator scheme; at p_z = 0 this is the mass / kinetic split).
 *  order     2: Strang's symmetric step, field at the step midpoint;
 *            4: the triple-jump composition of three Strang steps of sizes w1 dt, w0 dt, w1 dt,
 *            w1 = 1/(2 - 2^(1/3)), w0 = 1 - 2 w1 (Yoshida, Phys. Lett. A 150 (1990) 262): the
 *            fourth-order splitting Sec. V C leaves for future work.
 *  d_At      order 2: [sum nt][2] double, A at the step midpoints (the table of po_evolve_modes);
 *            order 4: [sum nt][3][2] double, A at t_i + (n + c_k) dt with c = (w1/2, 1/2,
 *            1 - w1/2), the midpoints of the three substeps (po_field_samples, n_sub = 3).
 *  d_A_edge  [n_pulses][2][2] double: A(t_i), A(t_f).
 *  d_f, d_J  as for po_evolve_modes (at least one non-NULL; same projection and fixed-order J).
 * Unlike the midpoint exponential, a term split is not exact for a constant field: without any
 * field it leaves a spurious density of order dt^4 (order 2) or dt^8 (order 4).
 * Errors: PO_ERR_INVALID for an order other than 2 or 4 and as po_evolve_modes.
 * --------------------------------------------------------------------------------------- */
po_status po_evolve_modes_split(int32_t n_pulses, const po_pulse_spec* specs, const po_grid* grids,
                                int32_t order, const double* d_At, const double* d_A_edge, double* d_f,
                                double* d_J, void* stream);

/* ---------------------------------------------------------------------------------------
 * Gradients for the local search of Sec. IV A (the gradient of the objective with respect to
 * the field parameters, which the BFGS iteration needs).  The paper obtains it from the adjoint
 * of the kinetic equation; here it is the exact derivative of the discrete Dirac evaluation of
 * J (the adjoint of its steps), so it is the gradient of exactly the J that po_evaluate returns
 * up to rounding.
 *
 * po_yield_gradient -- J and dJ/dA for any tables (as po_evolve_modes):
 *  d_J      out [n_pulses] or NULL.
 *  d_gA     out [sum nt][2]: dJ/dA at every step midpoint.
 *  d_gedge  out [n_pulses][2][2] or NULL: dJ/dA(t_i), dJ/dA(t_f) (initial state, projection).
 * Work buffers of ceil(modes / 256) x nt x 16 bytes per pulse (the per-step partial sums of each
 * 256-mode item, added in a fixed order by a second kernel) come from the stream-ordered pool: 64 MiB
 * for a 64x64x16 pulse at nt = 16384, 1 GiB for a 128x128x32 pulse at nt = 32768.  A batch whose
 * work buffers do not fit in device memory returns PO_ERR_NOMEM before the gradient kernels are
 * enqueued; split it into several calls.
 *
 * po_synth_gradient -- chain rule through the synthesis (Sec. III) of po_pulse_synth:
 *  d_gA, d_gedge  as produced above (d_gedge may be NULL: no end-point terms).
 *  d_grad   out [sum 4 n_s]: dJ/dc for the coefficient layout of po_pulse_synth.
 *  d_U      out [n_pulses] or NULL: the energy U = int |E|^2 dt of the synthesised field
 *           (midpoint rule, Sec. III Eq. energy).
 *  d_gU     out [sum 4 n_s] or NULL: dU/dc (zero under PO_NORM_ENERGY, which fixes U).
 * PO_NORM_NONE differentiates the raw field (the paper's local search, with U handled by a
 * penalty); PO_NORM_ENERGY includes the dependence of the scale on c.  PO_NORM_PEAK is not
 * differentiable and returns PO_ERR_UNSUPPORTED.
 *
 * po_evaluate_gradient -- fused synthesis -> J and dJ/dA -> dJ/dc (and U, dU/dc).
 * --------------------------------------------------------------------------------------- */
po_status po_yield_gradient(int32_t n_pulses, const po_pulse_spec* specs, const po_grid* grids,
                            const double* d_A, const double* d_A_edge, double* d_J, double* d_gA,
                            double* d_gedge, void* stream);
po_status po_synth_gradient(int32_t n_pulses, const po_pulse_spec* specs, const double* d_coeff,
                            const double* d_gA, const double* d_gedge, double* d_grad, double* d_U,
                            double* d_gU, void* stream);
po_status po_evaluate_gradient(int32_t n_pulses, const po_pulse_spec* specs, const po_grid* grids,
                               const double* d_coeff, double* d_J, double* d_grad, double* d_U,
                               double* d_gU, void* stream);

/* ---------------------------------------------------------------------------------------
 * Differential evolution, DE/rand/1/bin with greedy selection for maximisation (Sec. IV B).
 *  pop, dim  population size N >= 4 and genes per individual D >= 1.
 *  n_s       genes in odd blocks of n_s (phase coefficients) wrap periodically into [lo, hi];
 *            the others are redrawn uniformly in [lo, hi] when a mutant leaves it.  0 makes every
 *            gene an amplitude gene.
 *  F, CR     differential weight in [0, 2] and crossover probability in [0, 1].
 *  seed      key of the Philox4x32-10 counter-based generator (Salmon et al., SC'11).
 * Random words for individual i in generation g: Philox(counter = (i, block, g_lo, g_hi),
 * key = (seed_lo, seed_hi)).  Block 0: words -> a, b, c (distinct, != i) and the forced
 * crossover gene R; blocks 1..ceil(D/4): crossover uniforms (gene j -> block 1 + j/4, word
 * j%4); the next ceil(D/4) blocks: redraw uniforms.  Index in [0, n) = floor(u n / 2^32),
 * skipping the excluded indices in ascending order; uniform real = (u + 1/2) / 2^32.
 * The mutant a + F (b - c) rounds each operation separately (no fused multiply-add), so the
 * proposal is bitwise reproducible on any IEEE-754 machine.
 * --------------------------------------------------------------------------------------- */
typedef struct {
  int32_t pop;
  int32_t dim;
  int32_t n_s;
  double F;
  double CR;
  double lo;
  double hi;
  uint64_t seed;
} po_de_params;

/* d_pop [N][D] double -> d_trial out [N][D] double; d_idx out [N][4] int32 (a, b, c, R) or NULL. */
po_status po_de_propose(const po_de_params* prm, int64_t generation, const double* d_pop,
                        double* d_trial, int32_t* d_idx, void* stream);

/* In place: individual i takes trial i iff (d_mask == NULL or d_mask[i] != 0) and
 * d_trial_fit[i] >= d_fit[i] (ties move; NaN never moves).  d_mask [N] uint8 or NULL. */
po_status po_de_select(const po_de_params* prm, double* d_pop, double* d_fit, const double* d_trial,
                       const double* d_trial_fit, const uint8_t* d_mask, void* stream);

/* ---------------------------------------------------------------------------------------
 * Self-adaptive DE on islands: jDE (Brest, Greiner, Boskovic, Mernik & Zumer, IEEE Trans.
 * Evol. Comput. 10 (2006) 646), the self-adaptive variant named in Sec. IV B, with the
 * population split into `islands` equal islands of S = pop / islands consecutive members and
 * ring migration between them (the island model of Sec. IV B).
 *  pop, dim, n_s, lo, hi, seed   as po_de_params; pop must be a multiple of islands with
 *                                S >= 4; 1 <= islands <= 64.
 *  tau1, tau2    probabilities in [0, 1] of redrawing F and CR for a trial.
 *  F_lo, F_hi    range of a redrawn F, 0 <= F_lo <= F_hi <= 2 (jDE: 0.1, 1.0); a redrawn CR is
 *                uniform in (0, 1).
 * Each individual carries (F, CR) in d_fcr [N][2] double.  Random words as po_de_propose
 * (donors drawn among the S - 1 other members of the island), plus the block
 * 1 + 2 ceil(D/4): (u < tau1 ?, u for F, u < tau2 ?, u for CR).  With tau1 = tau2 = 0, one
 * island and equal (F, CR) the trials are those of po_de_propose, bit for bit.
 * --------------------------------------------------------------------------------------- */
typedef struct {
  int32_t pop;
  int32_t dim;
  int32_t n_s;
  int32_t islands;
  double tau1;
  double tau2;
  double F_lo;
  double F_hi;
  double lo;
  double hi;
  uint64_t seed;
} po_jde_params;

/* d_pop [N][D], d_fcr [N][2] -> d_trial [N][D], d_trial_fcr [N][2]; d_idx [N][4] or NULL. */
po_status po_jde_propose(const po_jde_params* prm, int64_t generation, const double* d_pop,
                         const double* d_fcr, double* d_trial, double* d_trial_fcr, int32_t* d_idx,
                         void* stream);
/* As po_de_select; a moving individual also takes the trial's (F, CR). */
po_status po_jde_select(const po_jde_params* prm, double* d_pop, double* d_fit, double* d_fcr,
                        const double* d_trial, const double* d_trial_fit, const double* d_trial_fcr,
                        const uint8_t* d_mask, void* stream);
/* Ring migration, all islands at once from the state before the call: the best member of island
 * k (largest fit, lowest index on ties) replaces the worst member of island (k + 1) mod islands
 * (smallest fit, lowest index on ties) when strictly better; genes, fit and (F, CR) move
 * together.  dim <= 64. */
po_status po_island_migrate(const po_jde_params* prm, double* d_pop, double* d_fit, double* d_fcr,
                            void* stream);
/* One jDE generation on the device: propose -> synthesis -> evolution -> J -> select, as
 * po_de_generation; the caller migrates every few generations with po_island_migrate. */
po_status po_jde_generation(const po_jde_params* prm, int64_t generation, const po_pulse_spec* spec,
                            const po_grid* grid, double* d_pop, double* d_fit, double* d_fcr,
                            double* d_trial, double* d_trial_fit, double* d_trial_fcr, void* stream);

/* Compaction helpers for screened generations (only some trials evaluated):
 * po_mask_indices: d_idx[0..count) = positions of the non-zero entries of d_mask [n] uint8, in
 *   increasing order; d_count [1] int32 or NULL.  1 <= n <= 8192.
 * po_gather_rows: d_dst[i][:] = d_src[d_idx[i]][:] for i < n_idx (double rows of `cols`); a row
 *   index outside [0, rows) yields a row of NaN.
 * po_scatter_values: d_dst[:] = fill, then d_dst[d_idx[i]] = d_vals[i] for i < n_idx; indices
 *   outside [0, n_dst) are skipped, repeated indices leave one of their values. */
po_status po_mask_indices(const uint8_t* d_mask, int32_t n, int32_t* d_idx, int32_t* d_count, void* stream);
po_status po_gather_rows(const double* d_src, int32_t rows, int32_t cols, const int32_t* d_idx, int32_t n_idx,
                         double* d_dst, void* stream);
po_status po_scatter_values(const double* d_vals, const int32_t* d_idx, int32_t n_idx, double fill, double* d_dst,
                            int32_t n_dst, void* stream);

/* One generation on a population of pulses that share one spec and one grid (dim must equal
 * 4 spec->n_s): propose -> evaluate every trial (synthesis, evolution, yield) -> select.
 *  d_pop [N][D], d_fit [N]     in/out population and fitness (J).
 *  d_trial [N][D], d_trial_fit [N]   out: this generation's trials and their J (kept for the
 *                              caller, e.g. as surrogate training data).
 * Scratch tables (N nt 16 bytes) come from the stream-ordered pool. */
po_status po_de_generation(const po_de_params* prm, int64_t generation, const po_pulse_spec* spec,
                           const po_grid* grid, double* d_pop, double* d_fit, double* d_trial,
                           double* d_trial_fit, void* stream);

/* ---------------------------------------------------------------------------------------
 * Plans: a fixed batch of (possibly uneven) pulses evaluated many times -- e.g. a DE population
 * whose pulses differ in duration nt and momentum grid.  A plan owns every work buffer, the
 * per-pulse descriptors and a device work queue of (pulse, block of modes) items ordered by
 * decreasing cost (nt), so persistent workgroups take the longest work first.  The launch
 * shape is given or chosen by timing the candidates on the plan's own batch (autotuning); the
 * choice can be cached in a text file.  The first po_plan_evaluate with a given set of
 * pointers captures synthesis -> series selection -> evolution -> yield into a HIP graph, later
 * calls with the same pointers replay it.  Results do not depend on the launch shape: J is
 * bitwise identical to po_evaluate's.  Calls on one plan must not overlap (they share its
 * buffers); different plans are independent.
 * --------------------------------------------------------------------------------------- */
typedef struct {
  int32_t threads;         /* lanes per workgroup: 64, 128 or 256; 0 = autotune */
  int32_t modes_per_lane;  /* 1 or 2; 0 = autotune */
  int32_t persistent;      /* 1 = persistent workgroups on the work queue, 0 = one workgroup per
                              256 modes (threads must be 256, modes_per_lane 1), -1 = autotune */
  int32_t workgroups;      /* persistent workgroups; 0 = what the device holds resident */
} po_plan_config;

/* cfg NULL = autotune everything.  cache_path NULL = no cache; otherwise a text file read before
 * and appended after autotuning, keyed by the device and the batch shape.  Allocates device
 * memory (sum nt x 32 bytes + modes / 8 bytes + small); runs and synchronises `stream` while
 * autotuning. */
po_status po_plan_create(int32_t n_pulses, const po_pulse_spec* specs, const po_grid* grids,
                         const po_plan_config* cfg, const char* cache_path, void* stream,
                         struct po_plan** out);
/* The launch shape the plan uses (after autotuning). */
po_status po_plan_get_config(const struct po_plan* plan, po_plan_config* out);
/* d_coeff [sum 4 n_s] double; d_J out [n_pulses] double; d_f out [sum M] double or NULL.
 * Tables are written to the plan's own buffers. */
po_status po_plan_evaluate(struct po_plan* plan, const double* d_coeff, double* d_J, double* d_f,
                           void* stream);
void po_plan_destroy(struct po_plan* plan);

/* ---------------------------------------------------------------------------------------
 * Surrogate network (an addition to the paper's method): an MLP n_in -> depth x (width, GELU)
 * -> 1 that maps a pulse's coefficient vector to the standardised log10 of its pair yield, used
 * to pre-screen differential-evolution trial vectors.  BF16 weights and activations feed the
 * matrix cores (16x16x32 bf16 MFMA) with FP32 accumulation; FP32 master weights; Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8); loss = mean squared error.  GELU is the erf form.
 * Parameter vector (float): per hidden layer W [k_in][width] (row-major) then b [width]; then
 * the output weights [width] and bias [1].  Requires n_in and width multiples of 32; every
 * batch a multiple of 32 up to max_batch.  Inputs are the coefficients as doubles, 16-byte
 * aligned (rounded to bf16 through float inside: the boundary takes the coefficient vectors the
 * optimiser holds, so no separate conversion pass or bf16 copy is needed).  A network's calls must not overlap; it is bound to the device current at
 * creation.  Initial weights: uniform(-1/sqrt(k_in), 1/sqrt(k_in)) from Philox4x32-10(seed).
 * --------------------------------------------------------------------------------------- */
struct po_mlp;
po_status po_mlp_create(int32_t n_in, int32_t width, int32_t depth, int32_t max_batch, uint64_t seed,
                        void* stream, struct po_mlp** out);
int64_t po_mlp_param_count(const struct po_mlp* net);
/* d_params [param_count] float (device). set also resets the Adam state. */
po_status po_mlp_get_params(const struct po_mlp* net, float* d_params, void* stream);
po_status po_mlp_set_params(struct po_mlp* net, const float* d_params, void* stream);
/* d_x [batch][n_in] double -> d_y [batch] float. */
po_status po_mlp_forward(struct po_mlp* net, const double* d_x, int32_t batch, float* d_y, void* stream);
/* Loss (d_loss [1] float or NULL) and gradient (d_grad [param_count] float or NULL; kept inside
 * the network either way) for targets d_target [batch] float. */
po_status po_mlp_loss_grad(struct po_mlp* net, const double* d_x, const float* d_target, int32_t batch,
                           float* d_loss, float* d_grad, void* stream);
/* One Adam step with d_grad (NULL = the network's last gradient). */
po_status po_mlp_adam_step(struct po_mlp* net, const float* d_grad, float lr, void* stream);
/* po_mlp_loss_grad followed by po_mlp_adam_step (bitwise the same result).  The step's launches
 * are captured into a HIP graph on the first call with a given set of pointers, batch and lr, and
 * the graph is replayed by later calls with the same arguments. */
po_status po_mlp_train_step(struct po_mlp* net, const double* d_x, const float* d_target, int32_t batch,
                            float lr, float* d_loss, void* stream);
/* `steps` training steps on minibatches drawn from a data set held on the device:
 *  d_X [n_rows][n_in] double (16-byte aligned) and d_J [n_rows] double (yields); step s uses the
 *  rows d_idx[s batch .. s batch + batch - 1] (int32; entries outside [0, n_rows) read row 0) with
 *  targets (log10(max(J, 1e-300)) - mean) * inv_std, the standardisation of po_log10_standardize;
 *  d_losses [steps] float or NULL receives each step's loss.  Each step is the graph of
 *  po_mlp_train_step (captured once per set of arguments), replayed without host work between
 *  steps. */
po_status po_mlp_train_indexed(struct po_mlp* net, const double* d_X, const double* d_J, int32_t n_rows,
                               const int32_t* d_idx, int32_t steps, int32_t batch, double mean,
                               double inv_std, float lr, float* d_losses, void* stream);
void po_mlp_destroy(struct po_mlp* net);
/* d_mask[i] = 1 for the k largest scores (ties: lower index first; NaN ranks last), else 0.
 * 1 <= n <= 8192. */
po_status po_topk_mask(const float* d_score, int32_t n, int32_t k, uint8_t* d_mask, void* stream);
/* d_out[i] = (log10(max(d_J[i], floor)) - mean) * inv_std, as float (surrogate targets). */
po_status po_log10_standardize(const double* d_J, int32_t n, double floor_value, double mean, double inv_std,
                               float* d_out, void* stream);

/* ---------------------------------------------------------------------------------------
 * po_set_check_finite -- optional check that results are finite (off by default).  While it is
 * enabled, these calls count the non-finite entries of what they wrote, after their kernels:
 *   po_pulse_synth    the A table (d_A);
 *   po_evolve_modes   d_J, or d_f when d_J is NULL;
 *   po_evaluate       the A table, then d_J (or d_f when d_J is NULL);
 *   po_pair_yield     d_J;
 *   po_de_generation  the trials' J (d_trial_fit; the selection has already run: a trial whose J
 *                     is not finite never replaces its target).
 * A nonzero count returns PO_ERR_NUMERIC, the count and the buffer named in po_last_error; the
 * outputs are left as computed.  The check waits for the stream, so the calls become synchronous
 * and must not be captured into a graph; it costs one pass over the checked values.  Other entry
 * points (po_evaluate_noalloc included) are not checked.  The setting is process-wide; the call
 * returns the previous one.
 * --------------------------------------------------------------------------------------- */
int32_t po_set_check_finite(int32_t enable);

/* ---------------------------------------------------------------------------------------
 * Kernel timers (diagnostics, not part of the method).  While enabled, every po_evolve_modes /
 * po_evaluate / po_de_generation call records a pair of HIP events on its stream around the
 * launches of the per-mode evolution kernel.  po_timer_read waits for the recorded events,
 * returns the summed elapsed milliseconds and the number of bracketed calls, and clears them.
 * Timers are process-wide; enable them from one thread at a time.
 * --------------------------------------------------------------------------------------- */
po_status po_timer_enable(int on);
po_status po_timer_read(double* ms_total, int64_t* calls);
/* FP64 issue-rate probe (diagnostics): one launch in which exactly waves_per_simd (3..8) waves run
 * on every SIMD, each lane running iters x 8 rounds of `chains` (1, 2, 4, 8) independent
 * dependency chains of v_fma_f64.  d_sink [CUs x waves_per_simd x 256] double receives one value
 * per lane; *flop (host, may be NULL) the FP64 operations launched (2 per FMA).  The caller times
 * the launch on `stream`. */
po_status po_probe_fp64_fma(int32_t waves_per_simd, int32_t chains, int64_t iters, double* d_sink, double* flop,
                            void* stream);
/* Mode-steps evolved since the last read while timers were enabled, per series variant of the
 * second-order evolution kernel (chosen per block of 512 modes and chunk of 256 steps):
 * counts[0..7] = tan(theta)/theta polynomial of degree 4, 5, ..., 11; counts[8] = cos/sin series of
 * degree 7 with angle halving.
 * Entries beyond 9 are set to 0.  Synchronises the device; clears the counts. */
po_status po_timer_mode_steps(uint64_t* counts, int32_t n);

#ifdef __cplusplus
}
#endif

#endif /* PAIROPT_H */
