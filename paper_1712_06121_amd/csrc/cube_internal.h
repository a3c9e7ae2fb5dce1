// Internal structures of libcube (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "../../include/cube.h"
#include "cosmo.h"

namespace cube {

// ---- error handling -------------------------------------------------------------------------
struct Error {
  int code;
  std::string msg;
};

#define CUBE_HIP(call)                                                                       \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      throw ::cube::Error{CUBE_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

// device-side error flags (bit set by kernels, checked on the host after a step)
enum : uint32_t {
  FLAG_CFL = 1u,        // |displacement| > one coarse cell
  FLAG_NONFINITE = 2u,  // NaN/Inf position or velocity
  FLAG_OVERFLOW = 4u,   // moment accumulator out of range
  FLAG_COUNT = 8u,      // total count after the move differs from N
};

// ---- XCD-aware workgroup order ----------------------------------------------------------------
// The dispatcher hands workgroups of a launch to the 8 XCDs in turn (workgroup b to XCD b % 8),
// and each XCD has its own L2. Mapping the b-th dispatched workgroup to logical block
// (b % 8) * n/8 + b / 8 (with the remainder spread over the first XCDs) gives every XCD one
// contiguous range of logical blocks, so neighbouring blocks -- which share cache lines, halos
// and DRAM pages -- run on the same XCD at about the same time. It is a bijection for any n.
__host__ __device__ inline unsigned xcd_block(unsigned b, unsigned n) {
  const unsigned per = n / 8, rem = n % 8, x = b % 8, i = b / 8;
  return x * per + (x < rem ? x : rem) + i;
}

// ---- ensemble launches: one launch of a stage over several boxes ----------------------------
// The launch's logical workgroups (XCD-contiguous order) are cut into consecutive ranges, box b
// owning [first[b], first[b + 1]); args[b] holds box b's kernel arguments. The box of a workgroup
// is found by bisection over first[] (wave-uniform scalar reads).
template <class A>
struct BoxTable {
  const A* args;
  const uint32_t* first;  // nbox + 1 entries, first[0] = 0, first[nbox] = workgroups of the launch
  int nbox;
};

__device__ __forceinline__ int box_of(const uint32_t* __restrict__ first, int nbox, unsigned l) {
  int lo = 0, hi = nbox;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (first[mid] <= l) lo = mid;
    else hi = mid;
  }
  return lo;
}

// ---- FFT plan: one cubic size N, half-complex padded layout --------------------------------
// Real-space field: N x N rows of `pitch_c * 2` floats (x fastest, N used). Fourier space:
// the same rows hold pitch_c complex values, x-frequencies 0..N/2 (Nyquist at index N/2);
// columns beyond N/2 are padding processed as don't-care values.
struct FFTPlan {
  int n = 0;
  int bx = 0;        // row padding (complex values): the widest column block of the y/z passes
  int colbx = 0;     // column block width used by the y/z passes (tunable)
  int zorder = 0;    // workgroup order of the z passes: 0 dispatch order, 1 XCD-contiguous (tunable)
  int zlayout = 0;   // Poisson solve: 1 = z pass on a z-contiguous scratch copy (tunable)
  int zbx = 0;       // column block width of the z pass on the scratch copy (divides colbx; tunable)
  float2* zscratch = nullptr;  // field_floats() floats when allocated (owned by the simulation)
  int pitch_c = 0;   // complex values per row, = n/2 + bx
  float2* tw = nullptr;    // exp(-2 pi i t / n), t = 0..n-1 (device)
  float* k2 = nullptr;     // (2 pi f(t) / n)^2 with f the signed frequency of index t (device)
  size_t field_floats() const { return (size_t)n * n * pitch_c * 2; }
  size_t row_floats() const { return (size_t)pitch_c * 2; }
};

// ---- two-level force: the coarse-mesh term of the Poisson solve -------------------------------
struct CoarseTerm {
  const float2* spec = nullptr;   // coarse density spectrum in the coarse plan's layout (null: none)
  int64_t pitch_c = 0;            // complex values per coarse row
  int half = 0;                   // N_c / 2
  float rs2 = 0.0f;               // r_s^2, fine cells^2
  float scale = 0.0f;             // R^3
  const float2* inv_b = nullptr;  // 1 / B(f) for the signed coarse frequencies f + N_c/2, |f| < N_c/2
};

// ---- simulation ------------------------------------------------------------------------------
struct Sim {
  cube_params p{};
  hipStream_t stream = nullptr;
  int device = 0;  // the HIP device the simulation was created on
  cube_allocator alloc{};
  bool has_alloc = false;
  std::string last_error;

  int nm = 0, nc = 0, np = 0, nchi = 1, nnu = 1;
  int64_t nc3 = 0, capacity = 0, n = 0;
  int64_t dev_bytes = 0;

  // particle state, double buffered: [cur] is current
  void* chi[2] = {nullptr, nullptr};   // 3 planes x capacity x nchi bytes
  void* nu[2] = {nullptr, nullptr};    // 3 planes x capacity x nnu bytes
  uint32_t* cnt[2] = {nullptr, nullptr};
  uint64_t* off[2] = {nullptr, nullptr};  // nc3 + 1 (exclusive prefix, last = N)
  float* vc[2] = {nullptr, nullptr};      // 3 x nc3
  float* vs[2] = {nullptr, nullptr};      // nc3 decode scale
  void* pid[2] = {nullptr, nullptr};      // capacity particle IDs of pid_bytes each (optional)
  int pid_bytes = 0;
  int cur = 0;
  int config_gen = 0;  // bumped whenever captured step graphs of this simulation become stale

  // adaptive time steps: step j's interval [a_int[j], a_int[j+1]] is chosen from the maxima
  // measured two steps earlier (meas_*[0]: the state before the first step, [j + 1]: step j)
  bool adaptive = false;
  double eta_v = 0.0, eta_a = 0.0, eta_e = 0.0;
  std::vector<double> meas_v, meas_g;
  uint32_t* amax = nullptr;  // device: largest |v|^2 and |t|^2 of the last step pass (FP32 bits)

  // move scratch
  float* vinv = nullptr;       // nc3 encode scale 1/(sigma sqrt(2/pi))
  uint32_t* mig = nullptr;     // 27 x nc3 counts per (source cell, displacement)
  uint32_t* slot = nullptr;    // 27 x nc3 prefix per (new cell, source offset)
  int64_t* mom = nullptr;      // 4 x nc3: S1x, S1y, S1z, S2
  double* dev = nullptr;       // nc3 3-D velocity variance per cell
  uint64_t* blk_n = nullptr;   // per link block: count
  int64_t* blk_q = nullptr;    // per link block: dispersion sum
  uint64_t* blk_off = nullptr; // per link block: exclusive prefix
  double* scal = nullptr;      // [0] sigma_g^2
  uint32_t* flags = nullptr;   // error flags
  int64_t nblk = 0;

  // mesh
  FFTPlan mesh_plan;
  float* mesh = nullptr;
  FFTPlan lat_plan;            // lattice FFT for initial conditions (size np)

  // codec tables (device)
  float* tdec = nullptr;   // M entries
  float* tedge = nullptr;  // M + 1 entries: -inf, the M - 1 edges of Eq. (nu), +inf
  int16_t* tbucket = nullptr;  // first guess of the velocity code per bucket of u / (1 + |u|)
  int nbucket = 0;
  std::vector<float> h_tdec, h_tedge;
  int vm = 255;
  int ic_parent_np = 0;  // initial conditions refined from an ic_parent_np^3 parent (0: none)

  // two-level force (cube_set_two_level): split radius r_s in fine cells (0: single-level solve),
  // coarse FFT plan (size nc), coarse density / spectrum buffer, inverse restriction transfer
  double two_level_rs = 0.0;
  FFTPlan coarse_plan;
  float* coarse = nullptr;
  float2* inv_b = nullptr;

  // power spectrum accumulators
  double* pk_acc = nullptr;  // 5 x (nm/2 + 1): auto (3 rows) or cross (5 rows) shell sums

  // schedule
  Cosmo cosmo{};
  std::vector<double> a_int, a_half, kicks, drifts;
  double drift0 = 0.0;
  float* sched_dev = nullptr;  // FP32 (-kick_j / 12, drift_j) per step (device)
  int* step_dev = nullptr;     // step index read by graph-replayed move kernels (device)
  int steps_done = 0;
  bool half_drift_done = false;
  int move_variant = 0;     // move passes: -1 by particle density, 0 per-corner gradient, 1 gradient tile
  int deposit_variant = 3;  // bit 0: interleaved particle order, bit 1: 512-thread workgroups
  std::string autotune_report;  // per-variant times of the last cube_autotune
  double a_now = 0.0;
  bool have_particles = false;

  // phases (the initial half drift, steps) enqueued since the flags were last checked, with the
  // bookkeeping to restore when one of them fails: the device records the code of the first failing
  // phase in flags[1] (1: the initial half drift, j + 2: step j), and no later phase is applied
  struct PhaseRec {
    uint32_t code;
    int cur_before;
    int steps_done_before;
    bool half_before;
  };
  std::vector<PhaseRec> phases;
  // failure injection for tests of the error path: raise inject_flag before the move of step
  // inject_step (-1: never)
  int inject_step = -1;
  uint32_t inject_flag = 0;
  // polls of the gradient-tile scatter's ordered section before a chunk gives up waiting and
  // raises the count error (tests of that path set it small)
  uint32_t turn_limit = 1u << 22;

  // profiling: per-kernel event pairs recorded on the simulation's stream
  bool profiling = false;
  hipEvent_t ev[16] = {};
  double timings[16] = {};
  int timing_calls = 0;

  size_t pbytes = 0;  // bytes of one particle-state buffer (chi and nu planes)

  void* dmalloc(size_t bytes);
  void dfree(void* p);
  std::vector<void*> owned;
  std::vector<size_t> sizes;
};

// ---- host helpers (api.cpp) ------------------------------------------------------------------
void check_flags(Sim& s);         // reads and clears the device error flags; throws on a set flag
float gconst(const Sim& s);       // Green's constant -3/2 Omega_m / N^3
void require_particles(const Sim& s);
int enqueue_steps(Sim& s, int k);  // k steps on s.stream, no wait, flags unchecked; CUBE_DONE at a_final
int64_t footprint_bytes(const cube_params& p);

// ---- launchers (implemented in the .hip files) ---------------------------------------------
bool fft_size_supported(int n);
std::vector<int> fft_col_widths(int n);  // column block widths the y/z passes support at size n
void fft_plan_create(Sim& s, FFTPlan& pl, int n);
void fft_plan_destroy(Sim& s, FFTPlan& pl);
void fft_forward_3d(const FFTPlan& pl, float* data, hipStream_t st);
// evs (optional): 6 events recorded before the first pass and after each of the five passes
void fft_solve_poisson(const FFTPlan& pl, float* data, float gconst, hipStream_t st, hipEvent_t* evs = nullptr,
                       const CoarseTerm* ct = nullptr);
// sizes the coarse mesh of the two-level force may have (the FFT sizes and 16)
bool fft_coarse_size_supported(int n);
// tent-weight restriction of the fine mesh (plan fp) to the coarse mesh (plan cp, real layout)
void launch_restrict(const FFTPlan& fp, const float* mesh, const FFTPlan& cp, float* out, hipStream_t st);
// the Poisson solve of a step on the mesh: single-level, or two-level when switched on (api.cpp)
void solve_potential(Sim& s, hipStream_t st, hipEvent_t* evs = nullptr);
void fft_power(const FFTPlan& pl, float* data, double* acc, hipStream_t st);
// the modes with every |n_i| < np/2 of the forward-transformed field src (plan ps, size np) into
// dst (plan pd, a larger size), scaled
void splice_modes(const FFTPlan& ps, const float* src, const FFTPlan& pd, float* dst, float scale, hipStream_t st);
// shell sums of two forward-transformed meshes over one box: 5 x (n/2 + 1) doubles, n the smaller size
void cross_shells(const FFTPlan& pa, const float* a, const FFTPlan& pb, const float* b, double* acc,
                  hipStream_t st);
// initial conditions: psi_d = IFFT( i n_d tab[|n|^2] W ) with W the transformed noise
void fft_ic_component(const FFTPlan& pl, const float* wk, float* out, const float* tab, int dim,
                      hipStream_t st);

void launch_noise(const FFTPlan& pl, float* out, uint64_t seed, hipStream_t st);
void launch_deposit(Sim& s, hipStream_t st);
// move: mode 0 = step (force from mesh), 1 = drift only (no force), 2 = initial conditions
// dev_sched: take the kick/drift factors of step *step_dev from sched_dev (for captured graphs)
void launch_move(Sim& s, int mode, float kfac, float dfac, float* const* psi, float vfac, hipStream_t st,
                 hipEvent_t* evs, bool dev_sched = false);
// End of a phase of the run: records `code` in flags[1] if the flags are set and no earlier phase
// failed; with dev_sched the code is that of the step counter (+2), which is then advanced.
void launch_step_end(Sim& s, hipStream_t st, uint32_t code, bool dev_sched);
// flags[0] |= f (the failure injection of tests); with dev_sched only when the device step
// counter equals `at`
void launch_raise_flag(Sim& s, hipStream_t st, uint32_t f, bool dev_sched = false, int at = 0);
void launch_load(Sim& s, const double* dx, const float* dv, int64_t n, hipStream_t st);
// 1-byte counts into rho1 (nc3 bytes, device) and the counts >= 255 in cell order into over
// (nc3 entries at most, device); returns the number of the latter
int64_t launch_counts_u8(Sim& s, uint8_t* rho1, uint32_t* over, hipStream_t st);
// stable sort of n (key, value) pairs by key (keys <= max_key), ping-ponging between the given
// buffer pairs; *key_sorted / *val_sorted receive the pair that holds the result (sort.hip)
void sort_pairs_by_key(Sim& s, uint32_t* key, uint32_t* val, uint32_t* key_alt, uint32_t* val_alt, int64_t n,
                       uint32_t max_key, hipStream_t st, uint32_t** key_sorted, uint32_t** val_sorted);
// the values >= 255 of cnt[0 .. n) in order into out; returns their number (sort.hip)
int64_t select_at_least_255(Sim& s, const uint32_t* cnt, int64_t n, uint32_t* out, hipStream_t st);
// largest |v|^2 of the current state (uses amax as scratch; synchronises)
float launch_state_speed2(Sim& s, hipStream_t st);
// particle IDs 0 .. n-1 in storage order (when IDs are enabled)
void launch_pid_iota(Sim& s, hipStream_t st);
void launch_power_finish(Sim& s, int nbins, double* k, double* pk, double* nmodes);
// device address of the allocation-free entry point's fixed shell-sum array on device `dev`
// (looked up once per device; noalloc.hip)
double* noalloc_scratch(int dev);

}  // namespace cube

namespace cube {

// ---- ensemble steps: one launch per stage over every box (batch.cpp) -------------------------
// The launches of one step of an ensemble, planned from the boxes' current state parity. Their
// argument tables are staged on the host while the launches are planned and uploaded to one device
// buffer before the first launch; a launch finds its tables at the buffer's base plus an offset.
struct EnsembleStep {
  std::vector<char> staged;                               // host copy of every table
  char* dbase = nullptr;                                  // device copy (owned)
  std::vector<std::function<void(hipStream_t)>> launches;  // the step's launches, in order
  size_t put(const void* p, size_t bytes);                // stages a table; returns its offset
  template <class T>
  size_t put(const std::vector<T>& v) {
    return put(v.data(), v.size() * sizeof(T));
  }
  template <class T>
  T* at(size_t off) const {
    return reinterpret_cast<T*>(dbase + off);
  }
  void upload();  // allocates the device buffer and copies the staged tables (synchronous)
  void enqueue(hipStream_t st) const {
    for (const auto& f : launches) f(st);
  }
  EnsembleStep() = default;
  EnsembleStep(const EnsembleStep&) = delete;
  EnsembleStep& operator=(const EnsembleStep&) = delete;
  ~EnsembleStep();
};
// the stages of one step (every box at the same parity, single-level solves, fixed schedules):
// deposits grouped by kernel variant (particles.hip); Poisson solves grouped by mesh size and FFT
// variants (fft.hip); count passes grouped by kernel, then link, block scan and finalize of every
// box, then scatter passes grouped by kernel (particles.hip); the step-counter bump and failure
// record of every box (particles.hip)
void ensemble_deposit(EnsembleStep& es, const std::vector<Sim*>& boxes);
void ensemble_solve(EnsembleStep& es, const std::vector<Sim*>& boxes);
void ensemble_move(EnsembleStep& es, const std::vector<Sim*>& boxes);
void ensemble_step_end(EnsembleStep& es, const std::vector<Sim*>& boxes);

}  // namespace cube

struct cube_sim {
  cube::Sim s;
};
