/*
 * cube.h -- C ABI of libcube: the hot path of CUBE's information-optimised particle-mesh step
 * (Yu, Pen & Wang, "CUBE: An Information-optimized parallel Cosmological N-body Algorithm",
 * arXiv:1712.06121) on one AMD Instinct MI355X (gfx950).
 *
 * Particles are stored as in Sec. 2.1-2.2 of the paper: a 1- or 2-byte position code per
 * dimension relative to the coarse cell that holds the particle (Eqs. (chi), (x)), a 1- or
 * 2-byte velocity code per dimension relative to the coarse-cell mean velocity (Eqs. (nu), (v)),
 * per-cell counts and cell-ordered storage. One step decodes, deposits the mass by cloud-in-cell,
 * solves Poisson's equation by FFT, interpolates the force, kicks and drifts, re-encodes and
 * re-orders the particles by coarse cell (Sec. 2.3.3, Figs. code, update_xp, update_vp).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every call returns CUBE_OK (0) or a negative CUBE_E_* code and never throws. The text of
 *   the last error of a simulation is returned by cube_last_error().
 * - Device work is enqueued on the stream given at creation (a hipStream_t; NULL = the null
 *   stream). Calls that take host buffers synchronise that stream before returning.
 * - The simulation owns all device memory it allocates (through the allocator callback when
 *   one is given, hipMalloc otherwise). The caller owns every host buffer it passes.
 * - One simulation must not be used by two host threads at the same time.
 * - Mesh and coarse-cell arrays are x-fastest: cell id c = x + N (y + N z).
 * - Units: lengths in fine-mesh cells, H0 = 1, momentum p = a^2 dx/dt (fine cells x H0).
 *   Mesh-to-coarse ratio R = nm_side / nc_side must be 4 (the paper's usual choice, Sec. 2.3.1).
 */
#ifndef CUBE_H
#define CUBE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------------------------ */
#define CUBE_OK 0
#define CUBE_DONE 1            /* cube_step reached a_final (not an error)                     */
#define CUBE_E_INVALID -1      /* bad argument or parameter combination                        */
#define CUBE_E_NOMEM -2        /* device or host allocation failed                             */
#define CUBE_E_DEVICE -3       /* a HIP runtime call failed                                    */
#define CUBE_E_CAPACITY -4     /* a particle count exceeds the capacity fixed at creation      */
#define CUBE_E_CFL -5          /* a particle moved more than one coarse cell in one step       */
#define CUBE_E_NONFINITE -6    /* a non-finite position or velocity appeared                   */
#define CUBE_E_OVERFLOW -7     /* an integer accumulator would overflow                        */
#define CUBE_E_STATE -8        /* call out of order (e.g. step before any particles exist)     */

#define CUBE_SIGMA_GLOBAL 0    /* one dispersion for the whole box (Sec. 2.2, last paragraph)  */
#define CUBE_SIGMA_PER_CELL 1  /* per-coarse-cell dispersion, global value as fallback         */

typedef struct cube_sim cube_sim;

/* Simulation parameters. Cosmology follows Sec. 2.2 (a, H, D, f); the initial conditions
 * follow Sec. 2.3.2: BBKS transfer function with shape Omega_m h, spectral index n_s, amplitude
 * fixed by sigma_8, Zel'dovich displacement at a_init. The schedule has n_steps steps between
 * a_init and a_final, uniform in ln a (spacing 0) or in a (spacing 1), integrated as DKD
 * leapfrog with merged drifts -- the paper's (DKKD)^n with the last half drift at the end. */
typedef struct {
  int32_t np_side;      /* particles per side of the initial lattice (N_p = np_side^3); an FFT
                           size (below) and a multiple of nc_side                                */
  int32_t nm_side;      /* fine mesh cells per side, an FFT size: 2^k or 3*2^k in 32 .. 2048
                           (32, 48, 64, 96, 128, 192, 256, 384, 512, 1024, 2048)                 */
  int32_t nc_side;      /* coarse cells per side; nm_side / 4, a multiple of 8                  */
  int32_t x_bytes;      /* n_chi in {1, 2}: bytes per position code and dimension, Eq. (chi)    */
  int32_t v_bytes;      /* n_nu in {1, 2}: bytes per velocity code and dimension, Eq. (nu)      */
  int32_t sigma_mode;   /* CUBE_SIGMA_GLOBAL or CUBE_SIGMA_PER_CELL                             */
  int32_t n_steps;      /* number of leapfrog steps from a_init to a_final                      */
  int32_t spacing;      /* 0: uniform in ln a, 1: uniform in a                                   */
  double box;           /* box side L in Mpc/h                                                   */
  double omega_m, omega_l, h, sigma8, n_s;
  double a_init, a_final;
  uint64_t seed;        /* seed of the Philox4x32-10 white-noise stream                          */
  int64_t capacity;     /* maximum particle count; 0 means np_side^3                             */
} cube_params;

/* Optional device allocator (e.g. a framework's caching allocator). alloc returns a device
 * pointer of at least `bytes` bytes aligned to 256 bytes, or NULL; free releases it. */
typedef struct {
  void* (*alloc)(size_t bytes, void* user);
  void (*free)(void* ptr, void* user);
  void* user;
} cube_allocator;

/* Create a simulation on the current HIP device. `stream` is a hipStream_t or NULL; `alloc`
 * may be NULL. Builds the FFT plans, the codec tables and the time-step schedule (the
 * paper's `initialize`). On success *out owns every device buffer and must be destroyed with
 * cube_destroy. Errors: CUBE_E_INVALID (sizes), CUBE_E_NOMEM, CUBE_E_DEVICE. */
int cube_create(const cube_params* params, void* stream, const cube_allocator* alloc, cube_sim** out);

/* Release every resource of the simulation (the paper's `finalize`). NULL is a no-op. */
void cube_destroy(cube_sim* sim);

/* Text of the last error of `sim` ("" if none), owned by the simulation. With sim == NULL: the
 * text of the last failed cube_create on the calling thread. */
const char* cube_last_error(const cube_sim* sim);

/* Zel'dovich initial conditions at a_init (Sec. 2.3.2, Fig. ic): Philox white noise on the
 * np_side^3 lattice, FFT, BBKS amplitude, spectral displacement with Nyquist planes removed,
 * then the two particle passes (count, then encode in cell order). Resets the schedule. */
int cube_init_ic(cube_sim* sim);
/* Refined initial conditions, for the PM-error reference of Sec. 3 (the same initial conditions
 * with more particles and cells): with parent_np > 0 every later cube_init_ic and
 * cube_get_ic_displacement takes, for each mode with all |n_i| < parent_np/2, the transformed
 * white noise of the parent_np^3 lattice of the same seed, scaled by (np_side/parent_np)^{3/2},
 * so a run of this simulation and one of np_side = parent_np hold the same Gaussian field on
 * those scales; every other mode comes from this lattice's own noise, drawn with the seed XOR
 * 0x9E3779B97F4A7C15. parent_np must divide np_side, be smaller and be a supported FFT size;
 * 0 switches refinement off. Errors: CUBE_E_INVALID. */
int cube_set_ic_parent(cube_sim* sim, int32_t parent_np);

/* Replace the particles by n host particles: x (n,3) positions in fine cells, v (n,3) momenta,
 * both FP64 row-major. Positions are encoded with Eq. (chi) in FP64, velocities rounded to
 * FP32 and encoded with Eq. (nu) against the statistics of their cell; storage order is the
 * input order, stably sorted by cell. Resets the schedule. Errors: CUBE_E_CAPACITY. */
int cube_load_particles(cube_sim* sim, const double* x, const double* v, int64_t n);

/* Advance k leapfrog steps (Fig. code): before the first step the initial half drift; each step
 * deposits, solves, kicks and drifts; the last step ends with the final half drift at a_final.
 * Returns CUBE_DONE when a_final has been reached (remaining steps are not taken).
 * The k steps are enqueued without waiting; the device error flags are read once at the end. A
 * step whose move raises a flag is not applied, and neither is any later one: the call then
 * returns the error with the state, cube_steps_done and cube_scale_factor those before the
 * failing step (or before the initial half drift), and the error text names that step.
 * Errors: CUBE_E_CFL, CUBE_E_NONFINITE, CUBE_E_OVERFLOW (a velocity of 2^15 fine cells x H0 or
 * more, or a coarse cell whose n x 3-D velocity variance reaches 2^34), CUBE_E_STATE. */
int cube_step(cube_sim* sim, int32_t k);

/* Two-level force (Sec. 2.3.1, 2.3.3, Fig. update_vp): the paper splits the force into a fine-mesh
 * part whose kernel vanishes beyond the buffer region and a compensating part computed from the
 * coarse density on a mesh R = 4 times coarser by one global FFT. With r_s > 0 every later Poisson
 * solve (steps, cube_stage_solve) uses
 *   phi(n) = G(n) [(1 - S(n)) D_f(n) + S(n) R^3 D_c(n) / B(n)]  for the modes with every |n_i| < N_c/2,
 *   phi(n) = G(n) (1 - S(n)) D_f(n)                              for the others,
 * with G = -3/2 Omega_m / k^2, S = exp(-k^2 r_s^2) (k in rad per fine cell), D_f the fine density's
 * spectrum, D_c that of its restriction to the coarse mesh with tent weights (1,3,5,7,7,5,3,1)/32 over
 * fine offsets -2..5 along each axis, and B the restriction's transfer: the fine part (kernel
 * G (1 - S), short-ranged: erfc(r / 2 r_s) / r) is solved by the fine-mesh FFT and the coarse part
 * joins it in Fourier space. The force is then the single-level one's 4-point gradient and CIC
 * interpolation. r_s in fine cells, between 4 (S negligible at the coarse Nyquist frequency) and
 * nm_side / 4; 0 switches back to the single-level solve and frees the coarse buffers (one
 * coarse-mesh FFT field, not counted by cube_footprint). Needs nc_side to be 16 or a supported FFT
 * size. Errors: CUBE_E_INVALID, CUBE_E_NOMEM. */
int cube_set_two_level(cube_sim* sim, double r_s);

/* Failure injection for tests of the error path: raise the device error bits `flag` (1 CFL,
 * 2 non-finite, 4 overflow, 8 count) just before the move of step `step` of later cube_step or
 * cube_batch_step calls, as if that move had raised them; step -1 switches it off.
 * Errors: CUBE_E_INVALID. */
int cube_debug_inject_flag(cube_sim* sim, int32_t step, uint32_t flag);

/* For tests of the error path: the gradient-tile scatter ranks a tile's chunks in storage order,
 * each chunk waiting (polling an LDS word) until the previous one is ranked; after `polls` polls
 * (default 2^22, far beyond any legitimate wait) a chunk stops waiting and raises the count error
 * (8), so the step fails with CUBE_E_STATE and is not applied. A small value forces that path.
 * Errors: CUBE_E_INVALID (polls 0). */
int cube_debug_set_turn_limit(cube_sim* sim, uint32_t polls);

/* Adaptive time steps (Sec. 2.3.3: the step is bounded by the particles' largest velocity and
 * acceleration and by the expansion), chosen before the first step; eta_v = eta_a = eta_e = 0
 * returns to the fixed schedule. Each interval [a0, a1] of the kicks is the largest with
 * a1 <= a0 (1 + eta_e), a1 <= a_final, vmax Delta(a0, a1) <= eta_v and
 * gmax K(a0, a1) Delta(a0, a1) <= eta_a (fine cells; Delta and K the drift and kick factors,
 * vmax the largest speed and gmax the largest force per unit kick factor), found by bisection.
 * The maxima come from the step two intervals earlier (the first two intervals: the largest speed
 * of the state and no force), because a step's drift already ends at the middle of the next
 * interval. n_steps bounds the number of steps (CUBE_E_STATE beyond it); cube_step returns
 * CUBE_DONE once a_final is reached. Every step reads the maxima back (one synchronisation).
 * Not for batches. Errors: CUBE_E_INVALID, CUBE_E_STATE (after the first step), CUBE_E_CFL
 * (a step that would shrink to nothing). */
int cube_set_adaptive(cube_sim* sim, double eta_v, double eta_a, double eta_e);
/* The adaptive schedule so far: the interval ends a_int[0 .. *n_a - 1] (a_int[0] = a_init) and
 * the maxima vmax, gmax[0 .. *n_meas - 1] (index 0: the state before the first step; j + 1: step
 * j). At most max_entries of each are written. CUBE_E_STATE when adaptive steps are off. */
int cube_get_adaptive_log(cube_sim* sim, int32_t max_entries, double* a_int, double* vmax, double* gmax,
                          int32_t* n_a, int32_t* n_meas);
/* The largest speed and force per unit kick factor of the last step pass (also after
 * cube_stage_move), when adaptive steps are on; CUBE_E_STATE otherwise. */
int cube_get_last_maxima(cube_sim* sim, double* vmax, double* gmax);

/* Scale factor of the particle positions (a_init before the first step, a_final at the end). */
double cube_scale_factor(const cube_sim* sim);
/* Number of steps completed. */
int32_t cube_steps_done(const cube_sim* sim);
/* Current particle count. */
int64_t cube_num_particles(const cube_sim* sim);

/* CIC density contrast delta = rho/<rho> - 1 of the current state (Sec. 3), nm^3 FP32 values
 * x-fastest, into `dst` (host memory if dst_on_device == 0, else device memory). */
int cube_get_density(cube_sim* sim, float* dst, int dst_on_device);

/* Auto power spectrum of the current state, Eq. (cps): CIC density, FFT, shells |n| rounded to
 * the nearest integer for n = 1 .. nbins (nbins <= nm_side/2). Host outputs of length nbins:
 * mean |k| (h/Mpc), mean P ((Mpc/h)^3, FP64 shell sums) and the number of modes. */
int cube_get_power(cube_sim* sim, int32_t nbins, double* k, double* pk, double* nmodes);

/* Allocation-free variant of cube_get_power, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid allocation): the same CIC
 * deposit, forward FFT and shell sums, with the FP64 shell sums kept in a fixed array of the
 * library (3 x 1025 doubles per device, held until the process ends) instead of the simulation's
 * allocation, and the results written to DEVICE arrays k, pk, nmodes of nbins doubles each (mean |k|
 * in h/Mpc, mean P in (Mpc/h)^3, mode counts). Everything is enqueued on the simulation's stream
 * and nothing is waited for; the call allocates no device memory. Every call on one GPU shares
 * that array and clears it first: calls that overlap on one GPU (simulations on different
 * streams) race and must be ordered by the caller. Overwrites the mesh (scratch between steps).
 * Errors: CUBE_E_INVALID (nbins outside [1, nm/2]), CUBE_E_STATE (no particles), CUBE_E_DEVICE. */
int cube_get_power_noalloc(cube_sim* sim, int32_t nbins, double* k, double* pk, double* nmodes);

/* Cross power spectrum of the current states of two simulations over the same box (Sec. 3,
 * Eq. (cps) with two fields; the cross-correlation coefficient of Eq. (ccc) is
 * pab / sqrt(paa pbb)). Both densities are CIC-deposited on their own meshes and transformed;
 * shells as in cube_get_power, n = 1 .. nbins, nbins <= nm/2 of the smaller mesh. Meshes of one
 * size use every mode; meshes of different sizes use the modes whose every integer component
 * has |n_i| < nm/2 of the smaller mesh (its Nyquist planes are aliased). Host outputs of length
 * nbins: mean |k|, P_aa, P_bb, P_ab and the number of modes. `a` and `b` may be the same
 * simulation; two simulations must be on one device (their streams are ordered by an event) and
 * have equal box sizes. Errors are reported on `a`: CUBE_E_INVALID, CUBE_E_STATE, CUBE_E_DEVICE.
 * Overwrites both meshes (scratch between steps). */
int cube_get_cross_power(cube_sim* a, cube_sim* b, int32_t nbins, double* k, double* paa, double* pbb,
                         double* pab, double* nmodes);

/* Checkpoint, the paper's "disjoint state" {rho_c, v_c, chi, nu} (Sec. 2.3.1): host buffers
 * (cube_get_state also accepts device buffers of the simulation's GPU: the copy direction follows
 * the pointers).
 * cnt: nc^3 uint32; chi: 3 planes of n codes (uint8 chi+128 for x_bytes 1, uint16 chi+32768
 * for 2); nu: 3 planes of n codes (int8 or int16); vc: 3 planes of nc^3 FP32; vs: nc^3 FP32
 * decode scales sigma sqrt(2/pi) of Eq. (v). cube_get_state writes them (n = current count);
 * cube_set_state reads them and also sets the scale factor and completed-step count. */
typedef struct {
  uint32_t* cnt;
  void* chi;
  void* nu;
  float* vc;
  float* vs;
  int64_t n;
  double a;
  int32_t steps_done;
} cube_state_view;
int cube_get_state(cube_sim* sim, cube_state_view* out);
/* The particle count of every coarse cell (nc^3 uint32, x-fastest) into host memory: the part of
 * the state that is small at any size (rho_c of Sec. 2.3.1). */
int cube_get_counts(cube_sim* sim, uint32_t* cnt);
int cube_set_state(cube_sim* sim, const cube_state_view* in);

/* The coarse-cell counts in the 1-byte checkpoint form of Sec. 2.1: rho1[c] = min(count, 255)
 * for the nc^3 cells (host, x fastest); every cell marked 255 holds 255 or more particles and
 * its true count is written to `overflow` (host, 4-byte integers, in cell order). *n_overflow
 * receives the number of such cells; when it exceeds max_overflow nothing is written to
 * `overflow` and CUBE_E_CAPACITY is returned (call again with a larger list). */
int cube_get_counts_u8(cube_sim* sim, uint8_t* rho1, uint32_t* overflow, int64_t max_overflow,
                       int64_t* n_overflow);
/* Host-only inverse (no simulation, no GPU): the ncells counts from rho1 and the overflow list.
 * CUBE_E_INVALID when the list does not match the cells marked 255. */
int cube_counts_from_u8(const uint8_t* rho1, int64_t ncells, const uint32_t* overflow, int64_t n_overflow,
                        uint32_t* cnt);

/* Particle IDs, the optional I_P array of Sec. 2.1: one pid_bytes-byte unsigned integer per
 * particle (4 or 8; 0 frees them), stored in the same order as chi and nu and carried through
 * every step, half drift and re-sort. IDs are assigned as follows: cube_init_ic gives each particle
 * its lattice index x + np (y + np z) (so its Lagrangian position q follows from the ID);
 * cube_load_particles gives the index in the input arrays; cube_set_state, and
 * cube_enable_pids when particles already exist, give 0 .. n-1 in storage order.
 * pid_bytes 4 needs capacity <= 2^32. Adds 2 x pid_bytes x capacity bytes of device memory (both
 * state buffers), which cube_footprint does not count. Errors: CUBE_E_INVALID, CUBE_E_NOMEM. */
int cube_enable_pids(cube_sim* sim, int32_t pid_bytes);
/* The n IDs of the current state in storage order (host memory, pid_bytes each), the checkpoint's
 * I_P; cube_set_pids writes them back after cube_set_state. Errors: CUBE_E_STATE when IDs are
 * not enabled or no particles exist. */
int cube_get_pids(cube_sim* sim, void* host_dst);
int cube_set_pids(cube_sim* sim, const void* host_src);

/* ---- stages of one step, for parity checks and profiling -------------------------------- */

/* CIC deposit of the current state into the mesh: delta in FP32 (exact integer accumulation,
 * one rounding). */
int cube_stage_deposit(cube_sim* sim);
/* Poisson solve in place on the mesh: phi = IFFT( -3/2 Omega_m / |k|^2 FFT(delta) ). */
int cube_stage_solve(cube_sim* sim);
/* Kick + drift + re-encode + counting sort with the potential held in the mesh:
 * v += kfac * D (D the unnormalised 4-point gradient, so kfac = -K/12), x += dfac * v. */
int cube_stage_move(cube_sim* sim, float kfac, float dfac);
/* Copy the real-space mesh (nm^3 FP32, x fastest) to or from host memory (cube_get_mesh also
 * writes device memory of the simulation's GPU: the copy direction follows the pointer). */
int cube_get_mesh(cube_sim* sim, float* dst);
int cube_set_mesh(cube_sim* sim, const float* host_src);
/* Zel'dovich displacement (3 planes of np^3 FP32, fine cells, lattice order) of the last
 * cube_init_ic, computed again from the noise. */
int cube_get_ic_displacement(cube_sim* sim, float* host_dst);
/* FP32 decode table T[nu] = tan(pi nu / M) and FP32 edge table of Eq. (nu), host copies;
 * sizes M and M - 1 with M = 2^(8 v_bytes) - 1. */
int cube_get_tables(cube_sim* sim, float* decode, float* edges);

/* Per-step kick and drift factors of the schedule (host, FP64): drift0, then kick[j], drift[j]
 * for j = 0 .. n_steps-1. kick/drift must have n_steps entries. */
int cube_get_schedule(const cube_sim* sim, double* drift0, double* kick, double* drift);

/* Device memory held by the simulation, in bytes. */
int64_t cube_device_bytes(const cube_sim* sim);

/* Average time per step of each kernel of the last cube_step call, measured with HIP events on
 * the simulation's stream (milliseconds). ms9: 0 deposit, 1 FFT x pass, 2 FFT y pass,
 * 3 fused z pass with the Green's function, 4 inverse y pass, 5 inverse x pass, 6 move count
 * pass, 7 link + scan + statistics, 8 move scatter pass. Profiling must be enabled with
 * cube_set_profiling(sim, 1); it adds one host synchronisation per step. */
int cube_set_profiling(cube_sim* sim, int enable);
int cube_get_timings(const cube_sim* sim, double* ms9);

/* ---- kernel variants and the autotuner ------------------------------------------------------
 * Some stages have equivalent kernel variants that give bit-identical results: the layout of the
 * work, never the arithmetic, differs. */
typedef struct {
  int32_t move_variant;    /* which move passes use the gradient tile (the 4-point gradient of the
                              whole tile precomputed in LDS, one row of coarse cells per wavefront,
                              1024-thread workgroups) instead of the gradient per CIC corner
                              (512-thread workgroups): 0 (default) neither, 1 both, 2 the scatter
                              pass, 3 the count pass; -1: both when there are at least half as many
                              particles as fine cells, else neither */
  int32_t fft_col_width;   /* complex columns per workgroup in the y/z passes: 8 or 16 for
                              nm_side <= 512, 4 or 8 above */
  int32_t fft_z_order;     /* workgroup order of the z passes: 0 dispatch order, 1 contiguous ranges
                              per XCD */
  int32_t deposit_variant; /* bit 0: particles of a layer visited with a stride of 1/64 of the layer
                              (lanes of a wavefront in different cells); bit 1: 512-thread
                              workgroups instead of 256; default 3 */
  int32_t fft_z_layout;    /* 0 (default): z pass in place on the mesh; 1: the forward y pass writes
                              a z-contiguous copy, the z pass works there and the inverse y pass
                              writes back (one more mesh-sized device buffer, allocated when chosen
                              and freed when 0 is set again; not counted by cube_footprint) */
  int32_t fft_z_width;     /* column width of the z pass on the z-contiguous copy: a supported
                              width dividing fft_col_width (default: fft_col_width) */
} cube_variant;
/* Time the variants on the current state (deposits, solves, then moves whose result is
 * discarded) and keep the fastest of each stage. The particle state is unchanged; the mesh
 * afterwards holds the potential of the current state. Errors: CUBE_E_STATE (no particles). */
int cube_autotune(cube_sim* sim);
/* The times the last cube_autotune measured, one "stage variant t ms;" item per timed variant
 * (text owned by the simulation; "" before the first call). */
const char* cube_autotune_report(const cube_sim* sim);
int cube_get_variant(const cube_sim* sim, cube_variant* out);
/* Errors: CUBE_E_INVALID for a value outside the ranges above (nothing is changed then). */
int cube_set_variant(cube_sim* sim, const cube_variant* v);

/* ---- ensembles of independent boxes ----------------------------------------------------------
 * A batch holds nbox simulations (box i created from params[i]; sizes, codecs and cosmologies may
 * differ, n_steps must be equal), each on its own HIP stream created by the batch. One step of the
 * whole ensemble is captured once into a HIP graph and replayed for every step (the kick and drift
 * factors are read on the device from each box's schedule), so the host makes one launch per
 * step. Every box evolves exactly as it would alone: the results are bit-identical to stepping it
 * by itself with cube_step. */
typedef struct cube_batch cube_batch;

/* `stream`: hipStream_t on which the step graphs are launched (NULL: a stream the batch creates,
 * since a graph cannot be captured on the null stream); alloc as in
 * cube_create. Errors: CUBE_E_INVALID (a box's parameters, unequal n_steps), CUBE_E_NOMEM,
 * CUBE_E_DEVICE. The text of a failed create is cube_batch_last_error(NULL) on that thread. */
int cube_batch_create(const cube_params* params, int32_t nbox, void* stream, const cube_allocator* alloc,
                      cube_batch** out);
void cube_batch_destroy(cube_batch* b);
const char* cube_batch_last_error(const cube_batch* b);
int32_t cube_batch_size(const cube_batch* b);
/* Box i as a simulation handle owned by the batch (NULL if out of range). Single-box calls
 * (state, density, power, ...) apply to it; stepping a box alone makes the batch refuse to step
 * until the boxes are at the same step again (CUBE_E_STATE). */
cube_sim* cube_batch_box(cube_batch* b, int32_t i);
/* How cube_batch_step launches the boxes' kernels:
 *   0 (default) one captured graph per step with an independent branch of kernels per box;
 *   1 each box's kernels enqueued directly on its own stream, box after box (no graph);
 *   2 one captured graph per step in which every stage (deposit, each FFT pass, count, link,
 *     block scan, finalize, scatter, step end) is one launch over all boxes: the kernels find
 *     their box and tile in device tables of per-box arguments, built when the graph is captured
 *     (a few kB per box). Boxes that use different kernels for a stage (FFT size and variants,
 *     deposit workgroup size, move-pass kernel, codec) get one launch each for it. Needs
 *     single-level solves in every box.
 * All modes give the same results. Changing the mode drops the captured graphs (after waiting for
 * the batch's stream). Errors: CUBE_E_INVALID (unknown mode; mode 2 with a box whose two-level
 * force is on). */
int cube_batch_set_mode(cube_batch* b, int32_t mode);
/* Initial conditions of every box (cube_init_ic on each). */
int cube_batch_init_ic(cube_batch* b);
/* cube_autotune on the first box of each distinct shape (mesh, lattice, codec); the choice is
 * applied to every box of that shape. */
int cube_batch_autotune(cube_batch* b);
/* Advance every box k steps (one graph launch per step); the error flags of every box are
 * checked once at the end. A box whose step fails stays at the state before that step, as in
 * cube_step, while the other boxes keep their steps; the first failure is returned (its text
 * names the box and the step) and the batch then refuses to step until the boxes are at one step
 * again. Returns CUBE_DONE when the boxes have reached a_final. */
int cube_batch_step(cube_batch* b, int32_t k);

/* ---- serving: continuous batching of simulation jobs -----------------------------------------
 * A server runs independent jobs (one cube_params each) on one GPU. Jobs are queued in submission
 * order; each scheduling round (cube_server_poll) checks the active jobs without waiting, enqueues
 * the next slice of steps of those whose previous slice has finished, and admits queued jobs
 * (oldest first) while their footprint fits the memory budget and an execution slot is free.
 * Every active job has its own stream, so jobs that arrive while others run overlap with them on
 * the device. Each job evolves exactly as it would alone: its state and P(k) are bit-identical to
 * a cube_create / cube_init_ic / cube_step run of the same parameters. */
typedef struct cube_server cube_server;

/* Device bytes that cube_create followed by cube_init_ic allocates for these parameters at most
 * (allocator rounding not included); negative (CUBE_E_INVALID) for malformed parameters. */
int64_t cube_footprint(const cube_params* params);

/* mem_budget_bytes: admission limit on the sum of the footprints of admitted, not yet released
 * jobs; max_active: execution slots (jobs stepped concurrently); slice_steps: steps enqueued per
 * job per round. alloc as in cube_create (used for every job's memory). */
int cube_server_create(int64_t mem_budget_bytes, int32_t max_active, int32_t slice_steps,
                       const cube_allocator* alloc, cube_server** out);
/* Waits for every job's stream and frees everything. */
void cube_server_destroy(cube_server* srv);
const char* cube_server_last_error(const cube_server* srv);
/* Queue a job under a caller-chosen id (unique among unreleased jobs). Errors: CUBE_E_INVALID,
 * CUBE_E_CAPACITY (the footprint alone exceeds the budget). */
int cube_server_submit(cube_server* srv, const cube_params* params, int64_t job_id);
/* One scheduling round (never waits for the GPU). Writes up to max_finished ids of jobs that have
 * finished or failed since the last poll into `finished` and their number into *n_finished;
 * ids that do not fit are returned by later polls. */
int cube_server_poll(cube_server* srv, int64_t* finished, int32_t max_finished, int32_t* n_finished);
/* State of a job: 0 queued, 1 active, 2 finished, 3 failed (*rc = its error code; the text is
 * cube_server_job_error). */
int cube_server_status(const cube_server* srv, int64_t job_id, int32_t* state, int32_t* rc);
const char* cube_server_job_error(const cube_server* srv, int64_t job_id);
/* The simulation of a finished job (owned by the server, valid until released): read its state,
 * density or P(k) with the single-box calls. NULL unless the job is finished. */
cube_sim* cube_server_job(cube_server* srv, int64_t job_id);
/* Free a finished or failed job's memory and forget its id. Errors: CUBE_E_STATE if it is still
 * queued or active. */
int cube_server_release(cube_server* srv, int64_t job_id);
int cube_server_stats(const cube_server* srv, int32_t* queued, int32_t* active, int64_t* bytes_in_use);

#ifdef __cplusplus
}
#endif
#endif /* CUBE_H */
