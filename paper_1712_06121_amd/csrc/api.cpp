// C ABI of libcube (declared in include/cube.h): simulation lifetime, schedule, and the calls of
// the paper's main program (Fig. code): initial conditions, steps, checkpoint I/O, analysis.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <new>

#include "cube_internal.h"

namespace {
thread_local std::string g_create_error;  // text of the last failed cube_create on this thread
}

namespace cube {

void* Sim::dmalloc(size_t bytes) {
  void* p = nullptr;
  if (bytes == 0) bytes = 256;
  if (has_alloc) {
    p = alloc.alloc(bytes, alloc.user);
    if (!p) throw Error{CUBE_E_NOMEM, "device allocator returned NULL for " + std::to_string(bytes) + " bytes"};
  } else {
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Error{CUBE_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
    }
  }
  dev_bytes += (int64_t)bytes;
  owned.push_back(p);
  sizes.push_back(bytes);
  return p;
}

void Sim::dfree(void* p) {
  if (!p) return;
  for (size_t i = 0; i < owned.size(); ++i) {
    if (owned[i] == p) {
      dev_bytes -= (int64_t)sizes[i];
      owned.erase(owned.begin() + i);
      sizes.erase(sizes.begin() + i);
      break;
    }
  }
  if (has_alloc) alloc.free(p, alloc.user);
  else (void)hipFree(p);
}

// helpers shared with batch.cpp (declared in cube_internal.h)



void build_tables(Sim& s) {
  const int m = (1 << (8 * s.nnu)) - 1;
  const int half = (m - 1) / 2;
  s.vm = m;
  s.h_tdec.resize(m);
  s.h_tedge.resize(m - 1);
  for (int nu = -half; nu <= half; ++nu) s.h_tdec[nu + half] = (float)std::tan(M_PI * (double)nu / (double)m);
  for (int j = -(half - 1); j <= half; ++j) {
    const double e = std::tan(M_PI * ((double)j - 0.5) / (double)m);
    float f = (float)e;
    if ((double)f < e) f = std::nextafterf(f, INFINITY);
    s.h_tedge[j + half - 1] = f;
  }
  // bucket table: t = u / (1 + |u|) in (-1, 1) split into 4 (M + 1) buckets; each holds the code of
  // the bucket's lower end. Only a starting guess: the kernels finish with exact edge comparisons.
  s.nbucket = 4 * (m + 1);
  std::vector<int16_t> lo(s.nbucket);
  for (int b = 0; b < s.nbucket; ++b) {
    const double t = -1.0 + 2.0 * b / s.nbucket;
    const double u = b == 0 ? -INFINITY : t / (1.0 - std::fabs(t));
    const int cnt = (int)(std::upper_bound(s.h_tedge.begin(), s.h_tedge.end(), u,
                                           [](double a, float e) { return a < (double)e; }) - s.h_tedge.begin());
    lo[b] = (int16_t)(cnt - half);
  }
  // the move kernels rely on at most one edge per bucket (two exact steps then finish the search):
  // consecutive lower-end codes differ by at most one
  for (int b = 1; b < s.nbucket; ++b)
    if (lo[b] - lo[b - 1] > 1) throw Error{CUBE_E_INVALID, "velocity bucket table holds two edges in one bucket"};
  s.tbucket = static_cast<int16_t*>(s.dmalloc(sizeof(int16_t) * s.nbucket));
  CUBE_HIP(hipMemcpy(s.tbucket, lo.data(), sizeof(int16_t) * s.nbucket, hipMemcpyHostToDevice));
  s.tdec = static_cast<float*>(s.dmalloc(sizeof(float) * m));
  // device edge table with sentinels: ext[0] = -inf, ext[i] = E[i - 1], ext[M] = +inf, so code nu
  // is the one with ext[nu + h] <= u < ext[nu + h + 1] for every u, end codes included
  std::vector<float> ext(m + 1);
  ext[0] = -INFINITY;
  for (int i = 1; i < m; ++i) ext[i] = s.h_tedge[i - 1];
  ext[m] = INFINITY;
  s.tedge = static_cast<float*>(s.dmalloc(sizeof(float) * (m + 1)));
  CUBE_HIP(hipMemcpy(s.tdec, s.h_tdec.data(), sizeof(float) * m, hipMemcpyHostToDevice));
  CUBE_HIP(hipMemcpy(s.tedge, ext.data(), sizeof(float) * (m + 1), hipMemcpyHostToDevice));
}

void build_schedule(Sim& s) {
  const int n = s.p.n_steps;
  s.a_int.resize(n + 1);
  for (int j = 0; j <= n; ++j) {
    if (s.p.spacing == 0)
      s.a_int[j] = s.p.a_init * std::pow(s.p.a_final / s.p.a_init, (double)j / n);
    else
      s.a_int[j] = s.p.a_init + (s.p.a_final - s.p.a_init) * (double)j / n;
  }
  s.a_int[0] = s.p.a_init;
  s.a_int[n] = s.p.a_final;
  s.a_half.resize(n);
  for (int j = 0; j < n; ++j) s.a_half[j] = std::sqrt(s.a_int[j] * s.a_int[j + 1]);
  s.drift0 = s.cosmo.drift(s.a_int[0], s.a_half[0]);
  s.kicks.resize(n);
  s.drifts.resize(n);
  for (int j = 0; j < n; ++j) s.kicks[j] = s.cosmo.kick(s.a_int[j], s.a_int[j + 1]);
  for (int j = 0; j + 1 < n; ++j) s.drifts[j] = s.cosmo.drift(s.a_half[j], s.a_half[j + 1]);
  s.drifts[n - 1] = s.cosmo.drift(s.a_half[n - 1], s.a_int[n]);
}

void reset_schedule(Sim& s) {
  s.steps_done = 0;
  s.half_drift_done = false;
  if (s.adaptive) {
    s.a_int.clear();
    s.a_half.clear();
    s.meas_v.clear();
    s.meas_g.clear();
    std::fill(s.kicks.begin(), s.kicks.end(), 0.0);
    std::fill(s.drifts.begin(), s.drifts.end(), 0.0);
    s.drift0 = 0.0;
  }
}

// The end of the next interval from a0 (Sec. 2.3.3: the step is bounded by the particles' largest
// speed and acceleration and by the expansion): the largest a1 <= min(a0 (1 + eta_e), a_final)
// with vmax Delta(a0, a1) <= eta_v (the largest drift, fine cells) and
// gmax K(a0, a1) Delta(a0, a1) <= eta_a (the drift of the largest velocity change), by bisection.
double adaptive_next(const Sim& s, double a0, double vmax, double gmax) {
  const double af = s.p.a_final;
  double hi = std::min(a0 * (1.0 + s.eta_e), af);
  auto ok = [&](double a1) {
    const double d = s.cosmo.drift(a0, a1);
    if (vmax * d > s.eta_v) return false;
    return gmax * s.cosmo.kick(a0, a1) * d <= s.eta_a;
  };
  if (ok(hi)) return hi;
  double lo = a0;
  for (int it = 0; it < 60; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (ok(mid)) lo = mid;
    else hi = mid;
  }
  if (!(lo > a0)) throw Error{CUBE_E_CFL, "the adaptive time step collapsed to zero"};
  return lo;
}

void read_maxima(Sim& s, double* vmax, double* gmax) {
  uint32_t bits[2] = {0u, 0u};
  CUBE_HIP(hipMemcpyAsync(bits, s.amax, sizeof(bits), hipMemcpyDeviceToHost, s.stream));
  CUBE_HIP(hipStreamSynchronize(s.stream));
  float f[2];
  std::memcpy(f, bits, sizeof(f));
  *vmax = std::sqrt((double)f[0]);
  *gmax = std::sqrt((double)f[1]) / 12.0;  // t is 12 times the force per unit kick factor
}

int enqueue_adaptive(Sim& s, int k) {
  const double af = s.p.a_final;
  for (int i = 0; i < k; ++i) {
    if (!s.half_drift_done) {
      const double v0 = std::sqrt((double)launch_state_speed2(s, s.stream));
      s.meas_v.assign(1, v0);
      s.meas_g.assign(1, 0.0);
      s.a_int.assign(1, s.p.a_init);
      s.a_int.push_back(adaptive_next(s, s.p.a_init, v0, 0.0));
      s.a_int.push_back(s.a_int[1] >= af ? af : adaptive_next(s, s.a_int[1], v0, 0.0));
      s.a_half.assign(1, std::sqrt(s.a_int[0] * s.a_int[1]));
      s.drift0 = s.cosmo.drift(s.a_int[0], s.a_half[0]);
      s.phases.push_back({1u, s.cur, s.steps_done, false});
      launch_move(s, 1, 0.0f, (float)s.drift0, nullptr, 0.0f, s.stream, nullptr);
      launch_step_end(s, s.stream, 1u, false);
      s.half_drift_done = true;
    }
    const int j = s.steps_done;
    if (j > 0 && s.a_int[j] >= af) return CUBE_DONE;
    if (j >= s.p.n_steps) throw Error{CUBE_E_STATE, "the adaptive schedule needs more than n_steps steps"};
    const double ah = s.a_int[j + 1] >= af ? af : std::sqrt(s.a_int[j + 1] * s.a_int[j + 2]);
    s.a_half.resize(j + 2);
    s.a_half[j + 1] = ah;
    s.kicks[j] = s.cosmo.kick(s.a_int[j], s.a_int[j + 1]);
    s.drifts[j] = s.cosmo.drift(s.a_half[j], ah);
    s.phases.push_back({(uint32_t)j + 2u, s.cur, j, true});
    launch_deposit(s, s.stream);
    solve_potential(s, s.stream);
    if (s.inject_step == j) launch_raise_flag(s, s.stream, s.inject_flag);
    launch_move(s, 0, (float)(-s.kicks[j] / 12.0), (float)s.drifts[j], nullptr, 0.0f, s.stream, nullptr);
    launch_step_end(s, s.stream, (uint32_t)j + 2u, false);
    double vm = 0.0, gm = 0.0;
    read_maxima(s, &vm, &gm);
    check_flags(s);  // the step has been waited for anyway: stop at a failed step, not after k
    s.meas_v.push_back(vm);
    s.meas_g.push_back(gm);
    const double an = s.a_int[j + 2];
    s.a_int.push_back(an >= af ? af : adaptive_next(s, an, vm, gm));
    s.steps_done++;
  }
  return CUBE_OK;
}

void check_flags(Sim& s) {
  uint32_t f[2] = {0u, 0u};
  CUBE_HIP(hipMemcpyAsync(f, s.flags, sizeof(f), hipMemcpyDeviceToHost, s.stream));
  CUBE_HIP(hipStreamSynchronize(s.stream));
  std::vector<Sim::PhaseRec> log;
  log.swap(s.phases);
  if (!f[0]) return;
  // a link pass that returned early has left the count pass's sums in the moment accumulators
  CUBE_HIP(hipMemsetAsync(s.flags, 0, 2 * sizeof(uint32_t), s.stream));
  CUBE_HIP(hipMemsetAsync(s.mom, 0, sizeof(int64_t) * 4 * s.nc3, s.stream));
  CUBE_HIP(hipStreamSynchronize(s.stream));
  // the failing phase and every later one were not applied: back to the state before it
  std::string where;
  for (const Sim::PhaseRec& r : log) {
    if (r.code != f[1]) continue;
    s.cur = r.cur_before;
    s.steps_done = r.steps_done_before;
    s.half_drift_done = r.half_before;
    where = r.code == 1u ? " (in the initial half drift; the state is the one before it)"
                         : " (in step " + std::to_string(r.code - 2u) + "; the state is the one before that step)";
    break;
  }
  if (f[0] & FLAG_NONFINITE) throw Error{CUBE_E_NONFINITE, "non-finite particle position or velocity" + where};
  if (f[0] & FLAG_CFL) throw Error{CUBE_E_CFL, "a particle moved more than one coarse cell in one step" + where};
  if (f[0] & FLAG_OVERFLOW)
    throw Error{CUBE_E_OVERFLOW, "velocity or dispersion outside the range of the fixed-point accumulators" + where};
  if (f[0] & FLAG_COUNT) throw Error{CUBE_E_STATE, "particle count changed during the move" + where};
  throw Error{CUBE_E_STATE, "unknown device error flag" + where};
}

void copy_mesh_out(Sim& s, float* dst, hipMemcpyKind kind) {
  const size_t pitch = s.mesh_plan.row_floats() * sizeof(float);
  CUBE_HIP(hipMemcpy2DAsync(dst, sizeof(float) * s.nm, s.mesh, pitch, sizeof(float) * s.nm, (size_t)s.nm * s.nm, kind,
                            s.stream));
  CUBE_HIP(hipStreamSynchronize(s.stream));
}

// The Poisson solve of a step on the mesh. Two-level force (Sec. 2.3.3): the fine density is
// restricted to the coarse mesh and transformed there, and the fused z pass of the fine solve
// combines the short-range fine part with the compensating coarse part.
void solve_potential(Sim& s, hipStream_t st, hipEvent_t* evs) {
  if (s.two_level_rs > 0.0) {
    launch_restrict(s.mesh_plan, s.mesh, s.coarse_plan, s.coarse, st);
    fft_forward_3d(s.coarse_plan, s.coarse, st);
    CoarseTerm ct;
    ct.spec = reinterpret_cast<const float2*>(s.coarse);
    ct.pitch_c = s.coarse_plan.pitch_c;
    ct.half = s.nc / 2;
    ct.rs2 = (float)(s.two_level_rs * s.two_level_rs);
    ct.scale = 64.0f;  // R^3
    ct.inv_b = s.inv_b;
    fft_solve_poisson(s.mesh_plan, s.mesh, gconst(s), st, evs, &ct);
  } else {
    fft_solve_poisson(s.mesh_plan, s.mesh, gconst(s), st, evs);
  }
}

float gconst(const Sim& s) {
  const double n3 = (double)s.nm * s.nm * s.nm;
  return (float)(-1.5 * s.p.omega_m / n3);
}

void require_particles(const Sim& s) {
  if (!s.have_particles) throw Error{CUBE_E_STATE, "no particles: call cube_init_ic, cube_load_particles or cube_set_state"};
}

// psi buffers for the initial conditions; returns the transformed noise buffer
void ic_fields(Sim& s, float** psi, float** wk_out, std::vector<void*>& temps, bool use_state_buffer) {
  const size_t fbytes = s.lat_plan.field_floats() * sizeof(float);
  float* wk = nullptr;
  if (s.lat_plan.n == s.mesh_plan.n) {
    wk = s.mesh;
  } else {
    wk = static_cast<float*>(s.dmalloc(fbytes));
    temps.push_back(wk);
  }
  for (int d = 0; d < 3; ++d) {
    if (d == 0 && use_state_buffer && s.pbytes >= fbytes) {
      psi[d] = static_cast<float*>(s.chi[s.cur]);  // the lattice pre-state reads no stored codes
      continue;
    }
    psi[d] = static_cast<float*>(s.dmalloc(fbytes));
    temps.push_back(psi[d]);
  }
  // refined from a parent lattice: own noise from a second stream, the parent's on its scales
  const uint64_t refine_key = 0x9E3779B97F4A7C15ull;
  launch_noise(s.lat_plan, wk, s.ic_parent_np ? (s.p.seed ^ refine_key) : s.p.seed, s.stream);
  fft_forward_3d(s.lat_plan, wk, s.stream);
  if (s.ic_parent_np) {
    FFTPlan pp;
    fft_plan_create(s, pp, s.ic_parent_np);
    float* pw = nullptr;
    try {
      pw = static_cast<float*>(s.dmalloc(pp.field_floats() * sizeof(float)));
      launch_noise(pp, pw, s.p.seed, s.stream);
      fft_forward_3d(pp, pw, s.stream);
      splice_modes(pp, pw, s.lat_plan, wk, (float)std::pow((double)s.np / (double)s.ic_parent_np, 1.5), s.stream);
      CUBE_HIP(hipStreamSynchronize(s.stream));
    } catch (...) {
      (void)hipStreamSynchronize(s.stream);
      if (pw) s.dfree(pw);
      fft_plan_destroy(s, pp);
      throw;
    }
    s.dfree(pw);
    fft_plan_destroy(s, pp);
  }
  // i n_d tab[|n|^2] gives the displacement in fine cells after the unnormalised inverse FFT
  const int h = s.np / 2;
  const int64_t ntab = 3LL * h * h + 1;
  std::vector<float> tab(ntab, 0.0f);
  const double box = s.p.box, np3 = (double)s.np * s.np * s.np;
  const double di = s.cosmo.D(s.p.a_init);
  for (int64_t n2 = 1; n2 < ntab; ++n2) {
    const double k = 2.0 * M_PI * std::sqrt((double)n2) / box;
    const double amp = std::sqrt(np3 * s.cosmo.pk_shape(k) * di * di / (box * box * box));
    tab[n2] = (float)(amp * (double)s.nm / (2.0 * M_PI * (double)n2 * np3));
  }
  float* dtab = static_cast<float*>(s.dmalloc(sizeof(float) * ntab));
  temps.push_back(dtab);
  CUBE_HIP(hipMemcpy(dtab, tab.data(), sizeof(float) * ntab, hipMemcpyHostToDevice));
  for (int d = 0; d < 3; ++d) fft_ic_component(s.lat_plan, wk, psi[d], dtab, d, s.stream);
  *wk_out = wk;
}

// Enqueue k steps on the simulation's stream (the initial half drift first if it is due) without
// waiting for them; the device error flags are left for the caller to check. Returns CUBE_DONE
// when a_final is reached before k steps.
int enqueue_steps(Sim& s, int k) {
  require_particles(s);
  if (s.adaptive) return enqueue_adaptive(s, k);
  int rc = CUBE_OK;
  if (s.profiling) {
    for (double& t : s.timings) t = 0.0;
    s.timing_calls = 0;
  }
  for (int i = 0; i < k; ++i) {
    if (s.steps_done >= s.p.n_steps) {
      rc = CUBE_DONE;
      break;
    }
    if (!s.half_drift_done) {
      s.phases.push_back({1u, s.cur, s.steps_done, false});
      launch_move(s, 1, 0.0f, (float)s.drift0, nullptr, 0.0f, s.stream, nullptr);
      launch_step_end(s, s.stream, 1u, false);
      s.half_drift_done = true;
    }
    const int j = s.steps_done;
    s.phases.push_back({(uint32_t)j + 2u, s.cur, j, true});
    // profiling events: [0,1] deposit, [2..7] five FFT passes, [8..11] count, link, scatter
    hipEvent_t* ev = s.profiling ? s.ev : nullptr;
    if (ev) CUBE_HIP(hipEventRecord(ev[0], s.stream));
    launch_deposit(s, s.stream);
    if (ev) CUBE_HIP(hipEventRecord(ev[1], s.stream));
    solve_potential(s, s.stream, ev ? ev + 2 : nullptr);
    if (s.inject_step == j) launch_raise_flag(s, s.stream, s.inject_flag);
    launch_move(s, 0, (float)(-s.kicks[j] / 12.0), (float)s.drifts[j], nullptr, 0.0f, s.stream,
                ev ? ev + 8 : nullptr);
    launch_step_end(s, s.stream, (uint32_t)j + 2u, false);
    if (ev) {
      CUBE_HIP(hipEventSynchronize(ev[11]));
      const int pairs[9][2] = {{0, 1}, {2, 3}, {3, 4}, {4, 5}, {5, 6}, {6, 7}, {8, 9}, {9, 10}, {10, 11}};
      for (int q = 0; q < 9; ++q) {
        float ms = 0.f;
        CUBE_HIP(hipEventElapsedTime(&ms, ev[pairs[q][0]], ev[pairs[q][1]]));
        s.timings[q] += ms;
      }
      s.timing_calls++;
    }
    s.steps_done++;
  }
  return rc;
}

// Device bytes cube_create allocates for these parameters, plus the temporaries of
// cube_init_ic (the transformed noise when the lattice and mesh sizes differ, the displacement
// fields that do not fit in a particle buffer, the amplitude table). Mirrors the allocations of
// cube_create, ic_fields and fft_plan_create.
int64_t footprint_bytes(const cube_params& p) {
  const int64_t nm = p.nm_side, nc = p.nc_side, np = p.np_side, nc3 = nc * nc * nc;
  const int64_t cap = p.capacity > 0 ? p.capacity : np * np * np;
  const int64_t pb = 3 * cap * (p.x_bytes + p.v_bytes);
  auto field = [](int64_t n) { return n * n * (n / 2 + (n >= 1024 ? 8 : 16)) * 2 * (int64_t)sizeof(float); };
  int64_t b = 2 * (pb + 4 * nc3 + 8 * (nc3 + 1) + 12 * nc3 + 4 * nc3);  // state, double buffered
  b += 4 * nc3 + 2 * 108 * nc3 + 32 * nc3 + 8 * nc3;                  // vinv, mig, slot, mom, dev
  b += 24 * ((nc3 + 255) / 256) + 64 + 16 + 40 * (nm / 2 + 1);       // link blocks, scalars, flags, P(k)
  b += 12 * nm + (np != nm ? 12 * np : 0) + field(nm);               // FFT plans and the mesh
  const int64_t m = ((int64_t)1 << (8 * p.v_bytes)) - 1;
  b += 4 * m + 4 * (m - 1) + 2 * 4 * (m + 1);                         // codec tables
  b += 8 * (int64_t)p.n_steps + 16;                                   // device schedule
  const int64_t fl = field(np);
  b += ((np != nm ? 1 : 0) + (pb >= fl ? 2 : 3)) * fl + 4 * (3 * (np / 2) * (np / 2) + 1);
  return b;
}

int fail(cube_sim* sim, const Error& e) {
  if (sim) sim->s.last_error = e.msg;
  return e.code;
}

#define CUBE_GUARD(sim, ...)                                                          \
  try {                                                                               \
    __VA_ARGS__;                                                                      \
  } catch (const ::cube::Error& e) {                                                  \
    return ::cube::fail(sim, e);                                                      \
  } catch (const std::bad_alloc&) {                                                   \
    return ::cube::fail(sim, ::cube::Error{CUBE_E_NOMEM, "host allocation failed"});  \
  } catch (const std::exception& e) {                                                 \
    return ::cube::fail(sim, ::cube::Error{CUBE_E_INVALID, e.what()});                \
  }

}  // namespace cube

using cube::Error;

extern "C" {

int cube_create(const cube_params* params, void* stream, const cube_allocator* alloc, cube_sim** out) {
  if (!params || !out) return CUBE_E_INVALID;
  *out = nullptr;
  cube_sim* sim = nullptr;
  try {
    sim = new cube_sim();
  } catch (...) {
    return CUBE_E_NOMEM;
  }
  cube::Sim& s = sim->s;
  try {
    s.p = *params;
    s.stream = static_cast<hipStream_t>(stream);
    CUBE_HIP(hipGetDevice(&s.device));
    (void)cube::noalloc_scratch(s.device);  // set-up of the allocation-free entry point, once per device
    if (alloc && alloc->alloc && alloc->free) {
      s.alloc = *alloc;
      s.has_alloc = true;
    }
    const cube_params& p = s.p;
    if (!cube::fft_size_supported(p.nm_side))
      throw Error{CUBE_E_INVALID, "nm_side must be 2^k or 3*2^k in [32, 2048] (32, 48, 64, 96, ..., 1024, 2048)"};
    if (p.nc_side * 4 != p.nm_side) throw Error{CUBE_E_INVALID, "nc_side must be nm_side / 4"};
    if (p.nc_side % 8 != 0) throw Error{CUBE_E_INVALID, "nc_side must be a multiple of 8"};
    if (!cube::fft_size_supported(p.np_side) || p.np_side % p.nc_side != 0)
      throw Error{CUBE_E_INVALID, "np_side must be 2^k or 3*2^k in [32, 2048] and a multiple of nc_side"};
    if (p.x_bytes < 1 || p.x_bytes > 2 || p.v_bytes < 1 || p.v_bytes > 2)
      throw Error{CUBE_E_INVALID, "x_bytes and v_bytes must be 1 or 2"};
    if (p.sigma_mode != CUBE_SIGMA_GLOBAL && p.sigma_mode != CUBE_SIGMA_PER_CELL)
      throw Error{CUBE_E_INVALID, "sigma_mode must be CUBE_SIGMA_GLOBAL or CUBE_SIGMA_PER_CELL"};
    if (p.n_steps < 1 || !(p.a_init > 0.0) || !(p.a_final > p.a_init) || !(p.box > 0.0) || !(p.omega_m > 0.0))
      throw Error{CUBE_E_INVALID, "need n_steps >= 1, 0 < a_init < a_final, box > 0, omega_m > 0"};
    s.nm = p.nm_side;
    s.nc = p.nc_side;
    s.np = p.np_side;
    s.nchi = p.x_bytes;
    s.nnu = p.v_bytes;
    s.nc3 = (int64_t)s.nc * s.nc * s.nc;
    s.capacity = p.capacity > 0 ? p.capacity : (int64_t)s.np * s.np * s.np;
    if (s.capacity >= (int64_t)1 << 40) throw Error{CUBE_E_INVALID, "capacity too large"};
    s.cosmo.om = p.omega_m;
    s.cosmo.ol = p.omega_l;
    s.cosmo.h = p.h;
    s.cosmo.sigma8 = p.sigma8;
    s.cosmo.ns = p.n_s;
    s.cosmo.init();
    cube::build_schedule(s);
    // particle state, double buffered
    for (int b = 0; b < 2; ++b) {
      const size_t pb = (size_t)3 * s.capacity * (s.nchi + s.nnu);
      char* buf = static_cast<char*>(s.dmalloc(pb));
      s.chi[b] = buf;
      s.nu[b] = buf + (size_t)3 * s.capacity * s.nchi;
      s.pbytes = pb;
      s.cnt[b] = static_cast<uint32_t*>(s.dmalloc(sizeof(uint32_t) * s.nc3));
      s.off[b] = static_cast<uint64_t*>(s.dmalloc(sizeof(uint64_t) * (s.nc3 + 1)));
      s.vc[b] = static_cast<float*>(s.dmalloc(sizeof(float) * 3 * s.nc3));
      s.vs[b] = static_cast<float*>(s.dmalloc(sizeof(float) * s.nc3));
    }
    s.vinv = static_cast<float*>(s.dmalloc(sizeof(float) * s.nc3));
    s.mig = static_cast<uint32_t*>(s.dmalloc(sizeof(uint32_t) * 27 * s.nc3));
    s.slot = static_cast<uint32_t*>(s.dmalloc(sizeof(uint32_t) * 27 * s.nc3));
    s.mom = static_cast<int64_t*>(s.dmalloc(sizeof(int64_t) * 4 * s.nc3));
    s.dev = static_cast<double*>(s.dmalloc(sizeof(double) * s.nc3));
    s.nblk = (s.nc3 + 255) / 256;
    s.blk_n = static_cast<uint64_t*>(s.dmalloc(sizeof(uint64_t) * s.nblk));
    s.blk_q = static_cast<int64_t*>(s.dmalloc(sizeof(int64_t) * s.nblk));
    s.blk_off = static_cast<uint64_t*>(s.dmalloc(sizeof(uint64_t) * s.nblk));
    s.scal = static_cast<double*>(s.dmalloc(sizeof(double) * 8));
    s.flags = static_cast<uint32_t*>(s.dmalloc(sizeof(uint32_t) * 4));
    s.pk_acc = static_cast<double*>(s.dmalloc(sizeof(double) * 5 * (s.nm / 2 + 1)));
    cube::fft_plan_create(s, s.mesh_plan, s.nm);
    if (s.np == s.nm) s.lat_plan = s.mesh_plan;
    else cube::fft_plan_create(s, s.lat_plan, s.np);
    s.mesh = static_cast<float*>(s.dmalloc(s.mesh_plan.field_floats() * sizeof(float)));
    cube::build_tables(s);
    {
      // the schedule's FP32 factors on the device, for replayed step graphs (same rounding as the
      // immediate factors cube_step passes)
      std::vector<float> kd(2 * (size_t)p.n_steps);
      for (int j = 0; j < p.n_steps; ++j) {
        kd[2 * j] = (float)(-s.kicks[j] / 12.0);
        kd[2 * j + 1] = (float)s.drifts[j];
      }
      s.sched_dev = static_cast<float*>(s.dmalloc(sizeof(float) * kd.size()));
      s.step_dev = static_cast<int*>(s.dmalloc(sizeof(int) * 4));
      CUBE_HIP(hipMemcpy(s.sched_dev, kd.data(), sizeof(float) * kd.size(), hipMemcpyHostToDevice));
      CUBE_HIP(hipMemsetAsync(s.step_dev, 0, sizeof(int) * 4, s.stream));
    }
    CUBE_HIP(hipMemsetAsync(s.mom, 0, sizeof(int64_t) * 4 * s.nc3, s.stream));
    CUBE_HIP(hipMemsetAsync(s.flags, 0, sizeof(uint32_t) * 4, s.stream));
    CUBE_HIP(hipMemsetAsync(s.mesh, 0, s.mesh_plan.field_floats() * sizeof(float), s.stream));
    CUBE_HIP(hipStreamSynchronize(s.stream));
    for (auto& e : s.ev) CUBE_HIP(hipEventCreate(&e));
    s.a_now = p.a_init;
  } catch (const Error& e) {
    g_create_error = e.msg;
    cube_destroy(sim);
    return e.code;
  } catch (const std::exception& e) {
    g_create_error = e.what();
    cube_destroy(sim);
    return CUBE_E_NOMEM;
  }
  *out = sim;
  return CUBE_OK;
}

void cube_destroy(cube_sim* sim) {
  if (!sim) return;
  cube::Sim& s = sim->s;
  if (s.stream) (void)hipStreamSynchronize(s.stream);
  else (void)hipDeviceSynchronize();
  for (auto& e : s.ev)
    if (e) (void)hipEventDestroy(e);
  std::vector<void*> all = s.owned;
  for (void* p : all) s.dfree(p);
  delete sim;
}

const char* cube_last_error(const cube_sim* sim) { return sim ? sim->s.last_error.c_str() : g_create_error.c_str(); }

int cube_init_ic(cube_sim* sim) {
  if (!sim) return CUBE_E_INVALID;
  cube::Sim& s = sim->s;
  CUBE_GUARD(sim, {
    std::vector<void*> temps;
    float* psi[3];
    float* wk = nullptr;
    cube::ic_fields(s, psi, &wk, temps, true);
    s.n = (int64_t)s.np * s.np * s.np;
    if (s.n > s.capacity) throw Error{CUBE_E_CAPACITY, "np_side^3 exceeds the capacity"};
    const double a = s.p.a_init;
    const float vfac = (float)(a * a * s.cosmo.E(a) * s.cosmo.f(a));
    cube::launch_move(s, 2, 0.0f, 0.0f, psi, vfac, s.stream, nullptr);
    CUBE_HIP(hipStreamSynchronize(s.stream));
    for (void* t : temps) s.dfree(t);
    s.have_particles = true;
    cube::reset_schedule(s);
    cube::check_flags(s);
  });
  return CUBE_OK;
}

int cube_set_ic_parent(cube_sim* sim, int32_t parent_np) {
  if (!sim) return CUBE_E_INVALID;
  cube::Sim& s = sim->s;
  if (parent_np != 0 && (parent_np < 2 || parent_np >= s.np || s.np % parent_np != 0 ||
                         !cube::fft_size_supported(parent_np)))
    return cube::fail(sim, Error{CUBE_E_INVALID,
                                 "parent_np must be 0 or a supported FFT size that divides np_side and is smaller"});
  s.ic_parent_np = parent_np;
  return CUBE_OK;
}

int cube_get_ic_displacement(cube_sim* sim, float* host_dst) {
  if (!sim || !host_dst) return CUBE_E_INVALID;
  cube::Sim& s = sim->s;
  CUBE_GUARD(sim, {
    std::vector<void*> temps;
    float* psi[3];
    float* wk = nullptr;
    cube::ic_fields(s, psi, &wk, temps, false);
    const size_t pitch = s.lat_plan.row_floats() * sizeof(float);
    const size_t np3 = (size_t)s.np * s.np * s.np;
    for (int d = 0; d < 3; ++d)
      CUBE_HIP(hipMemcpy2DAsync(host_dst + d * np3, sizeof(float) * s.np, psi[d], pitch, sizeof(float) * s.np,
                                (size_t)s.np * s.np, hipMemcpyDeviceToHost, s.stream));
    CUBE_HIP(hipStreamSynchronize(s.stream));
    for (void* t : temps) s.dfree(t);
  });
  return CUBE_OK;
}

int cube_load_particles(cube_sim* sim, const double* x, const double* v, int64_t n) {
  if (!sim || n < 0 || (n > 0 && (!x || !v))) return CUBE_E_INVALID;
  cube::Sim& s = sim->s;
  CUBE_GUARD(sim, {
    if (n > s.capacity) throw Error{CUBE_E_CAPACITY, "particle count exceeds the capacity"};
    if (n >= ((int64_t)1 << 32)) throw Error{CUBE_E_CAPACITY, "load path supports fewer than 2^32 particles"};
    double* d = static_cast<double*>(s.dmalloc(sizeof(double) * 6 * (size_t)(n > 0 ? n : 1)));
    if (n > 0) {
      CUBE_HIP(hipMemcpyAsync(d, x, sizeof(double) * 3 * n, hipMemcpyHostToDevice, s.stream));
      CUBE_HIP(hipMemcpyAsync(d + 3 * n, v, sizeof(double) * 3 * n, hipMemcpyHostToDevice, s.stream));
    }
    s.n = n;
    cube::launch_load(s, d, nullptr, n, s.stream);
    s.dfree(d);
    s.have_particles = true;
    cube::reset_schedule(s);
    cube::check_flags(s);
  });
  return CUBE_OK;
}

int64_t cube_footprint(const cube_params* params) {
  if (!params || params->np_side < 1 || params->nm_side < 1 || params->nc_side < 1 || params->x_bytes < 1 ||
      params->x_bytes > 2 || params->v_bytes < 1 || params->v_bytes > 2 || params->n_steps < 1)
    return CUBE_E_INVALID;
  return cube::footprint_bytes(*params);
}

int cube_step(cube_sim* sim, int32_t k) {
  if (!sim || k < 0) return CUBE_E_INVALID;
  cube::Sim& s = sim->s;
  int rc = CUBE_OK;
  CUBE_GUARD(sim, {
    rc = cube::enqueue_steps(s, k);
    cube::check_flags(s);
  });
  return rc;
}


int cube_set_two_level(cube_sim* sim, double r_s) {
  if (!sim) return CUBE_E_INVALID;
  cube::Sim& s = sim->s;
  if (!(r_s <= 0.0) && !(r_s >= 4.0 && r_s <= 0.25 * s.nm))
    return cube::fail(sim, Error{CUBE_E_INVALID, "r_s must be 0 (off) or between 4 fine cells and nm_side / 4"});
  if (r_s > 0.0 && !cube::fft_coarse_size_supported(s.nc))
    return cube::fail(sim, Error{CUBE_E_INVALID, "the coarse mesh size is not a supported FFT size"});
  CUBE_GUARD(sim, {
    CUBE_HIP(hipStreamSynchronize(s.stream));
    if (r_s <= 0.0) {
      if (s.coarse) {
        s.dfree(s.coarse);
        s.dfree(s.inv_b);
        cube::fft_plan_destroy(s, s.coarse_plan);
        s.coarse = nullptr;
        s.inv_b = nullptr;
      }
    } else if (!s.coarse) {
      cube::fft_plan_create(s, s.coarse_plan, s.nc);
      s.coarse = static_cast<float*>(s.dmalloc(s.coarse_plan.field_floats() * sizeof(float)));
      // 1 / B(f): the restriction's transfer sum_b w_b exp(2 pi i f b / nm) over the tent weights
      // (1, 3, 5, 7, 7, 5, 3, 1) / 32 at offsets b = -2 .. 5, for the signed coarse frequencies
      const int h = s.nc / 2;
      std::vector<float2> tab(s.nc, make_float2(0.0f, 0.0f));
      const double w[8] = {1, 3, 5, 7, 7, 5, 3, 1};
      for (int f = -h + 1; f < h; ++f) {
        double re = 0.0, im = 0.0;
        for (int b = -2; b <= 5; ++b) {
          const double ang = 2.0 * M_PI * f * b / s.nm;
          re += w[b + 2] / 32.0 * std::cos(ang);
          im += w[b + 2] / 32.0 * std::sin(ang);
        }
        const double d = re * re + im * im;
        tab[f + h] = make_float2((float)(re / d), (float)(-im / d));
      }
      s.inv_b = static_cast<float2*>(s.dmalloc(sizeof(float2) * s.nc));
      CUBE_HIP(hipMemcpy(s.inv_b, tab.data(), sizeof(float2) * s.nc, hipMemcpyHostToDevice));
    }
    s.two_level_rs = r_s > 0.0 ? r_s : 0.0;
    s.config_gen++;  // captured step graphs hold the previous solve
  });
  return CUBE_OK;
}

int cube_debug_inject_flag(cube_sim* sim, int32_t step, uint32_t flag) {
  if (!sim) return CUBE_E_INVALID;
  const uint32_t known = cube::FLAG_CFL | cube::FLAG_NONFINITE | cube::FLAG_OVERFLOW | cube::FLAG_COUNT;
  if (step < -1 || (flag & ~known) != 0u)
    return cube::fail(sim, Error{CUBE_E_INVALID, "step must be >= -1 and flag a combination of the error bits"});
  sim->s.inject_step = step;
  sim->s.inject_flag = flag;
  sim->s.config_gen++;  // captured step graphs hold the previous injection
  return CUBE_OK;
}

int cube_debug_set_turn_limit(cube_sim* sim, uint32_t polls) {
  if (!sim || polls == 0u) return CUBE_E_INVALID;
  sim->s.turn_limit = polls;
  sim->s.config_gen++;  // captured step graphs hold the previous limit
  return CUBE_OK;
}

double cube_scale_factor(const cube_sim* sim) {
  if (!sim) return 0.0;
  const cube::Sim& s = sim->s;
  if (s.adaptive) {
    if (s.steps_done == 0 || s.a_int.size() <= (size_t)s.steps_done) return s.p.a_init;
    if (s.a_int[s.steps_done] >= s.p.a_final) return s.p.a_final;
    return s.a_half[s.steps_done];
  }
  if (s.steps_done >= s.p.n_steps) return s.p.a_final;
  if (s.steps_done == 0) return s.p.a_init;
  return s.a_half[s.steps_done];
}

int32_t cube_steps_done(const cube_sim* sim) { return sim ? sim->s.steps_done : 0; }
int64_t cube_num_particles(const cube_sim* sim) { return sim ? sim->s.n : 0; }

int cube_stage_deposit(cube_sim* sim) {
  if (!sim) return CUBE_E_INVALID;
  CUBE_GUARD(sim, {
    cube::require_particles(sim->s);
    cube::launch_deposit(sim->s, sim->s.stream);
    CUBE_HIP(hipStreamSynchronize(sim->s.stream));
  });
  return CUBE_OK;
}

int cube_stage_solve(cube_sim* sim) {
  if (!sim) return CUBE_E_INVALID;
  CUBE_GUARD(sim, {
    cube::solve_potential(sim->s, sim->s.stream);
    CUBE_HIP(hipStreamSynchronize(sim->s.stream));
  });
  return CUBE_OK;
}

int cube_stage_move(cube_sim* sim, float kfac, float dfac) {
  if (!sim) return CUBE_E_INVALID;
  CUBE_GUARD(sim, {
    cube::require_particles(sim->s);
    const int cur0 = sim->s.cur;
    cube::launch_move(sim->s, 0, kfac, dfac, nullptr, 0.0f, sim->s.stream, nullptr);
    CUBE_HIP(hipStreamSynchronize(sim->s.stream));
    try {
      cube::check_flags(sim->s);
    } catch (const Error&) {
      sim->s.cur = cur0;  // the failed move was not applied
      throw;
    }
  });
  return CUBE_OK;
}

int cube_get_mesh(cube_sim* sim, float* dst) {
  if (!sim || !dst) return CUBE_E_INVALID;
  CUBE_GUARD(sim, { cube::copy_mesh_out(sim->s, dst, hipMemcpyDefault); });
  return CUBE_OK;
}

int cube_set_mesh(cube_sim* sim, const float* host_src) {
  if (!sim || !host_src) return CUBE_E_INVALID;
  cube::Sim& s = sim->s;
  CUBE_GUARD(sim, {
    const size_t pitch = s.mesh_plan.row_floats() * sizeof(float);
    CUBE_HIP(hipMemcpy2DAsync(s.mesh, pitch, host_src, sizeof(float) * s.nm, sizeof(float) * s.nm, (size_t)s.nm * s.nm,
                              hipMemcpyHostToDevice, s.stream));
    CUBE_HIP(hipStreamSynchronize(s.stream));
  });
  return CUBE_OK;
}

int cube_get_density(cube_sim* sim, float* dst, int dst_on_device) {
  if (!sim || !dst) return CUBE_E_INVALID;
  cube::Sim& s = sim->s;
  CUBE_GUARD(sim, {
    cube::require_particles(s);
    cube::launch_deposit(s, s.stream);
    cube::copy_mesh_out(s, dst, dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost);
  });
  return CUBE_OK;
}

int cube_get_power(cube_sim* sim, int32_t nbins, double* k, double* pk, double* nmodes) {
  if (!sim || !k || !pk || !nmodes) return CUBE_E_INVALID;
  cube::Sim& s = sim->s;
  if (nbins < 1 || nbins > s.nm / 2) return cube::fail(sim, Error{CUBE_E_INVALID, "nbins must be in [1, nm/2]"});
  CUBE_GUARD(sim, {
    cube::require_particles(s);
    const int nb = s.nm / 2 + 1;
    cube::launch_deposit(s, s.stream);
    CUBE_HIP(hipMemsetAsync(s.pk_acc, 0, sizeof(double) * 3 * nb, s.stream));
    cube::fft_power(s.mesh_plan, s.mesh, s.pk_acc, s.stream);
    std::vector<double> acc(3 * nb);
    CUBE_HIP(hipMemcpyAsync(acc.data(), s.pk_acc, sizeof(double) * 3 * nb, hipMemcpyDeviceToHost, s.stream));
    CUBE_HIP(hipStreamSynchronize(s.stream));
    const double L = s.p.box, kf = 2.0 * M_PI / L;
    const double nm6 = std::pow((double)s.nm, 6);
    for (int b = 1; b <= nbins; ++b) {
      const double w = acc[2 * nb + b];
      nmodes[b - 1] = w;
      k[b - 1] = w > 0 ? kf * acc[nb + b] / w : 0.0;
      pk[b - 1] = w > 0 ? (L * L * L / nm6) * acc[b] / w : 0.0;
    }
  });
  return CUBE_OK;
}

int cube_get_cross_power(cube_sim* sa, cube_sim* sb, int32_t nbins, double* k, double* paa, double* pbb,
                         double* pab, double* nmodes) {
  if (!sa || !sb || !k || !paa || !pbb || !pab || !nmodes) return CUBE_E_INVALID;
  cube::Sim& a = sa->s;
  cube::Sim& b = sb->s;
  const int n = std::min(a.nm, b.nm);
  if (a.p.box != b.p.box) return cube::fail(sa, Error{CUBE_E_INVALID, "the two simulations have different box sizes"});
  if (nbins < 1 || nbins > n / 2)
    return cube::fail(sa, Error{CUBE_E_INVALID, "nbins must be in [1, nm/2] of the smaller mesh"});
  CUBE_GUARD(sa, {
    cube::require_particles(a);
    cube::require_particles(b);
    if (sa != sb) {
      hipPointerAttribute_t pa{}, pb{};
      CUBE_HIP(hipPointerGetAttributes(&pa, a.mesh));
      CUBE_HIP(hipPointerGetAttributes(&pb, b.mesh));
      if (pa.device != pb.device) throw Error{CUBE_E_INVALID, "the two simulations live on different devices"};
    }
    const int nsh = n / 2 + 1;
    cube::launch_deposit(a, a.stream);
    cube::fft_forward_3d(a.mesh_plan, a.mesh, a.stream);
    if (sa != sb) {
      cube::launch_deposit(b, b.stream);
      cube::fft_forward_3d(b.mesh_plan, b.mesh, b.stream);
      if (b.stream != a.stream) {
        hipEvent_t done;
        CUBE_HIP(hipEventCreateWithFlags(&done, hipEventDisableTiming));
        hipError_t e = hipEventRecord(done, b.stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(a.stream, done, 0);
        hipEventDestroy(done);
        CUBE_HIP(e);
      }
    }
    CUBE_HIP(hipMemsetAsync(a.pk_acc, 0, sizeof(double) * 5 * nsh, a.stream));
    cube::cross_shells(a.mesh_plan, a.mesh, b.mesh_plan, b.mesh, a.pk_acc, a.stream);
    std::vector<double> acc(5 * nsh);
    CUBE_HIP(hipMemcpyAsync(acc.data(), a.pk_acc, sizeof(double) * 5 * nsh, hipMemcpyDeviceToHost, a.stream));
    CUBE_HIP(hipStreamSynchronize(a.stream));
    const double L = a.p.box, kf = 2.0 * M_PI / L, v = L * L * L;
    const double na3 = std::pow((double)a.nm, 3), nb3 = std::pow((double)b.nm, 3);
    for (int m = 1; m <= nbins; ++m) {
      const double w = acc[4 * nsh + m];
      nmodes[m - 1] = w;
      k[m - 1] = w > 0 ? kf * acc[3 * nsh + m] / w : 0.0;
      pab[m - 1] = w > 0 ? v / (na3 * nb3) * acc[m] / w : 0.0;
      paa[m - 1] = w > 0 ? v / (na3 * na3) * acc[nsh + m] / w : 0.0;
      pbb[m - 1] = w > 0 ? v / (nb3 * nb3) * acc[2 * nsh + m] / w : 0.0;
    }
  });
  return CUBE_OK;
}

int cube_set_adaptive(cube_sim* sim, double eta_v, double eta_a, double eta_e) {
  if (!sim) return CUBE_E_INVALID;
  cube::Sim& s = sim->s;
  const bool off = eta_v == 0.0 && eta_a == 0.0 && eta_e == 0.0;
  if (!off && !(eta_v > 0.0 && eta_a > 0.0 && eta_e > 0.0 && std::isfinite(eta_v) && std::isfinite(eta_a) &&
                std::isfinite(eta_e)))
    return cube::fail(sim, Error{CUBE_E_INVALID, "eta_v, eta_a and eta_e must be positive and finite (all 0: off)"});
  if (s.steps_done > 0 || s.half_drift_done)
    return cube::fail(sim, Error{CUBE_E_STATE, "adaptive time steps must be chosen before the first step"});
  CUBE_GUARD(sim, {
    if (!off && !s.amax) s.amax = static_cast<uint32_t*>(s.dmalloc(2 * sizeof(uint32_t)));
    if (off && s.amax) {
      CUBE_HIP(hipStreamSynchronize(s.stream));
      s.dfree(s.amax);
      s.amax = nullptr;
    }
    s.adaptive = !off;
    s.eta_v = eta_v;
    s.eta_a = eta_a;
    s.eta_e = eta_e;
    s.config_gen++;
    cube::build_schedule(s);
    cube::reset_schedule(s);
  });
  return CUBE_OK;
}

int cube_get_adaptive_log(cube_sim* sim, int32_t max_entries, double* a_int, double* vmax, double* gmax,
                          int32_t* n_a, int32_t* n_meas) {
  if (!sim || !n_a || !n_meas || max_entries < 0 || (max_entries > 0 && (!a_int || !vmax || !gmax)))
    return CUBE_E_INVALID;
  const cube::Sim& s = sim->s;
  if (!s.adaptive) return cube::fail(sim, Error{CUBE_E_STATE, "adaptive time steps are off"});
  *n_a = (int32_t)s.a_int.size();
  *n_meas = (int32_t)s.meas_v.size();
  for (int32_t i = 0; i < *n_a && i < max_entries; ++i) a_int[i] = s.a_int[i];
  for (int32_t i = 0; i < *n_meas && i < max_entries; ++i) {
    vmax[i] = s.meas_v[i];
    gmax[i] = s.meas_g[i];
  }
  return CUBE_OK;
}

int cube_get_last_maxima(cube_sim* sim, double* vmax, double* gmax) {
  if (!sim || !vmax || !gmax) return CUBE_E_INVALID;
  cube::Sim& s = sim->s;
  if (!s.amax) return cube::fail(sim, Error{CUBE_E_STATE, "adaptive time steps are off"});
  CUBE_GUARD(sim, { cube::read_maxima(s, vmax, gmax); });
  return CUBE_OK;
}

int cube_get_counts(cube_sim* sim, uint32_t* cnt) {
  if (!sim || !cnt) return CUBE_E_INVALID;
  cube::Sim& s = sim->s;
  CUBE_GUARD(sim, {
    CUBE_HIP(hipMemcpyAsync(cnt, s.cnt[s.cur], sizeof(uint32_t) * s.nc3, hipMemcpyDeviceToHost, s.stream));
    CUBE_HIP(hipStreamSynchronize(s.stream));
  });
  return CUBE_OK;
}

int cube_get_counts_u8(cube_sim* sim, uint8_t* rho1, uint32_t* overflow, int64_t max_overflow, int64_t* n_overflow) {
  if (!sim || !rho1 || !n_overflow || max_overflow < 0 || (max_overflow > 0 && !overflow)) return CUBE_E_INVALID;
  cube::Sim& s = sim->s;
  CUBE_GUARD(sim, {
    uint8_t* d1 = static_cast<uint8_t*>(s.dmalloc((size_t)s.nc3));
    uint32_t* dov = static_cast<uint32_t*>(s.dmalloc(sizeof(uint32_t) * (size_t)s.nc3));
    int64_t n = 0;
    try {
      n = cube::launch_counts_u8(s, d1, dov, s.stream);
      CUBE_HIP(hipMemcpyAsync(rho1, d1, (size_t)s.nc3, hipMemcpyDeviceToHost, s.stream));
      if (n <= max_overflow && n > 0)
        CUBE_HIP(hipMemcpyAsync(overflow, dov, sizeof(uint32_t) * (size_t)n, hipMemcpyDeviceToHost, s.stream));
      CUBE_HIP(hipStreamSynchronize(s.stream));
    } catch (...) {
      s.dfree(dov);
      s.dfree(d1);
      throw;
    }
    s.dfree(dov);
    s.dfree(d1);
    *n_overflow = n;
    if (n > max_overflow) throw Error{CUBE_E_CAPACITY, "more cells hold 255 or more particles than max_overflow"};
  });
  return CUBE_OK;
}

int cube_counts_from_u8(const uint8_t* rho1, int64_t ncells, const uint32_t* overflow, int64_t n_overflow,
                        uint32_t* cnt) {
  if (!rho1 || !cnt || ncells < 0 || n_overflow < 0 || (n_overflow > 0 && !overflow)) return CUBE_E_INVALID;
  int64_t j = 0;
  for (int64_t c = 0; c < ncells; ++c) {
    if (rho1[c] < 255) {
      cnt[c] = rho1[c];
    } else {
      if (j >= n_overflow) return CUBE_E_INVALID;
      if (overflow[j] < 255) return CUBE_E_INVALID;
      cnt[c] = overflow[j++];
    }
  }
  return j == n_overflow ? CUBE_OK : CUBE_E_INVALID;
}

int cube_get_state(cube_sim* sim, cube_state_view* out) {
  if (!sim || !out || !out->cnt || !out->chi || !out->nu || !out->vc || !out->vs) return CUBE_E_INVALID;
  cube::Sim& s = sim->s;
  CUBE_GUARD(sim, {
    cube::require_particles(s);
    const int c = s.cur;
    const hipStream_t st = s.stream;
    CUBE_HIP(hipMemcpyAsync(out->cnt, s.cnt[c], sizeof(uint32_t) * s.nc3, hipMemcpyDefault, st));
    for (int d = 0; d < 3; ++d) {
      CUBE_HIP(hipMemcpyAsync(static_cast<char*>(out->chi) + (size_t)d * s.n * s.nchi,
                              static_cast<char*>(s.chi[c]) + (size_t)d * s.capacity * s.nchi, (size_t)s.n * s.nchi,
                              hipMemcpyDefault, st));
      CUBE_HIP(hipMemcpyAsync(static_cast<char*>(out->nu) + (size_t)d * s.n * s.nnu,
                              static_cast<char*>(s.nu[c]) + (size_t)d * s.capacity * s.nnu, (size_t)s.n * s.nnu,
                              hipMemcpyDefault, st));
    }
    CUBE_HIP(hipMemcpyAsync(out->vc, s.vc[c], sizeof(float) * 3 * s.nc3, hipMemcpyDefault, st));
    CUBE_HIP(hipMemcpyAsync(out->vs, s.vs[c], sizeof(float) * s.nc3, hipMemcpyDefault, st));
    CUBE_HIP(hipStreamSynchronize(st));
    out->n = s.n;
    out->a = cube_scale_factor(sim);
    out->steps_done = s.steps_done;
  });
  return CUBE_OK;
}

int cube_set_state(cube_sim* sim, const cube_state_view* in) {
  if (!sim || !in || !in->cnt || !in->chi || !in->nu || !in->vc || !in->vs || in->n < 0) return CUBE_E_INVALID;
  cube::Sim& s = sim->s;
  CUBE_GUARD(sim, {
    if (in->n > s.capacity) throw Error{CUBE_E_CAPACITY, "particle count exceeds the capacity"};
    std::vector<uint64_t> off(s.nc3 + 1);
    uint64_t run = 0;
    for (int64_t c = 0; c < s.nc3; ++c) {
      off[c] = run;
      run += in->cnt[c];
    }
    off[s.nc3] = run;
    if ((int64_t)run != in->n) throw Error{CUBE_E_INVALID, "sum of cell counts differs from n"};
    if (s.adaptive && in->steps_done != 0)
      throw Error{CUBE_E_STATE, "an adaptive run restarts from step 0 (its schedule is not part of the checkpoint)"};
    const int c = s.cur;
    const hipStream_t st = s.stream;
    s.n = in->n;
    CUBE_HIP(hipMemcpyAsync(s.cnt[c], in->cnt, sizeof(uint32_t) * s.nc3, hipMemcpyHostToDevice, st));
    CUBE_HIP(hipMemcpyAsync(s.off[c], off.data(), sizeof(uint64_t) * (s.nc3 + 1), hipMemcpyHostToDevice, st));
    for (int d = 0; d < 3; ++d) {
      CUBE_HIP(hipMemcpyAsync(static_cast<char*>(s.chi[c]) + (size_t)d * s.capacity * s.nchi,
                              static_cast<const char*>(in->chi) + (size_t)d * s.n * s.nchi, (size_t)s.n * s.nchi,
                              hipMemcpyHostToDevice, st));
      CUBE_HIP(hipMemcpyAsync(static_cast<char*>(s.nu[c]) + (size_t)d * s.capacity * s.nnu,
                              static_cast<const char*>(in->nu) + (size_t)d * s.n * s.nnu, (size_t)s.n * s.nnu,
                              hipMemcpyHostToDevice, st));
    }
    CUBE_HIP(hipMemcpyAsync(s.vc[c], in->vc, sizeof(float) * 3 * s.nc3, hipMemcpyHostToDevice, st));
    CUBE_HIP(hipMemcpyAsync(s.vs[c], in->vs, sizeof(float) * s.nc3, hipMemcpyHostToDevice, st));
    CUBE_HIP(hipStreamSynchronize(st));
    s.have_particles = true;
    s.steps_done = in->steps_done < 0 ? 0 : (in->steps_done > s.p.n_steps ? s.p.n_steps : in->steps_done);
    s.half_drift_done = s.steps_done > 0;
    cube::launch_pid_iota(s, st);
    CUBE_HIP(hipStreamSynchronize(st));
  });
  return CUBE_OK;
}

int cube_enable_pids(cube_sim* sim, int32_t pid_bytes) {
  if (!sim) return CUBE_E_INVALID;
  cube::Sim& s = sim->s;
  if (pid_bytes != 0 && pid_bytes != 4 && pid_bytes != 8)
    return cube::fail(sim, Error{CUBE_E_INVALID, "pid_bytes must be 0, 4 or 8"});
  CUBE_GUARD(sim, {
    if (pid_bytes == 4 && s.capacity > ((int64_t)1 << 32))
      throw Error{CUBE_E_INVALID, "4-byte particle IDs need a capacity of at most 2^32"};
    if (pid_bytes != s.pid_bytes) {
      CUBE_HIP(hipStreamSynchronize(s.stream));
      for (int b = 0; b < 2; ++b) {
        if (s.pid[b]) s.dfree(s.pid[b]);
        s.pid[b] = nullptr;
      }
      s.pid_bytes = 0;
      s.config_gen++;
      if (pid_bytes) {
        for (int b = 0; b < 2; ++b) s.pid[b] = s.dmalloc((size_t)pid_bytes * (size_t)(s.capacity > 0 ? s.capacity : 1));
        s.pid_bytes = pid_bytes;
        if (s.have_particles) cube::launch_pid_iota(s, s.stream);
        CUBE_HIP(hipStreamSynchronize(s.stream));
      }
    }
  });
  return CUBE_OK;
}

int cube_get_pids(cube_sim* sim, void* host_dst) {
  if (!sim || !host_dst) return CUBE_E_INVALID;
  cube::Sim& s = sim->s;
  CUBE_GUARD(sim, {
    if (!s.pid_bytes) throw Error{CUBE_E_STATE, "particle IDs are not enabled (cube_enable_pids)"};
    cube::require_particles(s);
    CUBE_HIP(hipMemcpyAsync(host_dst, s.pid[s.cur], (size_t)s.pid_bytes * s.n, hipMemcpyDeviceToHost, s.stream));
    CUBE_HIP(hipStreamSynchronize(s.stream));
  });
  return CUBE_OK;
}

int cube_set_pids(cube_sim* sim, const void* host_src) {
  if (!sim || !host_src) return CUBE_E_INVALID;
  cube::Sim& s = sim->s;
  CUBE_GUARD(sim, {
    if (!s.pid_bytes) throw Error{CUBE_E_STATE, "particle IDs are not enabled (cube_enable_pids)"};
    cube::require_particles(s);
    CUBE_HIP(hipMemcpyAsync(s.pid[s.cur], host_src, (size_t)s.pid_bytes * s.n, hipMemcpyHostToDevice, s.stream));
    CUBE_HIP(hipStreamSynchronize(s.stream));
  });
  return CUBE_OK;
}

int cube_get_tables(cube_sim* sim, float* decode, float* edges) {
  if (!sim || !decode || !edges) return CUBE_E_INVALID;
  const cube::Sim& s = sim->s;
  std::memcpy(decode, s.h_tdec.data(), sizeof(float) * s.h_tdec.size());
  std::memcpy(edges, s.h_tedge.data(), sizeof(float) * s.h_tedge.size());
  return CUBE_OK;
}

int cube_get_schedule(const cube_sim* sim, double* drift0, double* kick, double* drift) {
  if (!sim || !drift0 || !kick || !drift) return CUBE_E_INVALID;
  const cube::Sim& s = sim->s;
  *drift0 = s.drift0;
  for (int j = 0; j < s.p.n_steps; ++j) {
    kick[j] = s.kicks[j];
    drift[j] = s.drifts[j];
  }
  return CUBE_OK;
}

int64_t cube_device_bytes(const cube_sim* sim) { return sim ? sim->s.dev_bytes : 0; }

int cube_set_profiling(cube_sim* sim, int enable) {
  if (!sim) return CUBE_E_INVALID;
  sim->s.profiling = enable != 0;
  return CUBE_OK;
}

int cube_get_timings(const cube_sim* sim, double* ms9) {
  if (!sim || !ms9) return CUBE_E_INVALID;
  for (int i = 0; i < 9; ++i) ms9[i] = sim->s.timing_calls ? sim->s.timings[i] / sim->s.timing_calls : 0.0;
  return CUBE_OK;
}

}  // extern "C"
