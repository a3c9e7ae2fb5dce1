// Ensembles of independent boxes stepped together, and the variant autotuner.
//
// A batch owns one simulation per box, each on its own HIP stream. One step of the whole ensemble
// (deposit, five-pass Poisson solve, count / link / scatter move passes and a step-counter bump
// per box) is captured once into a HIP graph and replayed for every step: the kick and drift
// factors of each step are read on the device from the box's schedule table, and two graphs are
// kept, one per parity of the double-buffered state. In the graph either every box is an
// independent branch of its own kernels (mode 0), or every stage is one launch over all boxes
// (mode 2: the kernels find their box and tile in a table of per-box arguments, so the tiles of
// small boxes fill the GPU beside those of large ones and a step is a few dozen launches).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <memory>
#include <tuple>

#include "cube_internal.h"

struct cube_batch {
  std::vector<cube_sim*> boxes;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> joins;
  hipEvent_t fork = nullptr;
  hipStream_t main = nullptr;
  bool own_main = false;  // graphs cannot be captured on the null stream: the batch then makes its own
  // 0: one captured graph per step, a branch per box; 1: kernels enqueued box by box on the box
  // streams; 2: one captured graph per step, one launch per stage over all boxes
  int mode = 0;
  std::unique_ptr<cube::EnsembleStep> table[2];  // mode 2: the launches and tables of each parity
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  std::vector<int> gens;  // each box's config_gen when the graphs were captured
  std::string last_error;
};

namespace cube {
namespace {

thread_local std::string g_batch_create_error;

int batch_fail(cube_batch* b, const Error& e) {
  if (b) b->last_error = e.msg;
  return e.code;
}

#define CUBE_BATCH_GUARD(b, ...)                                                      \
  try {                                                                               \
    __VA_ARGS__;                                                                      \
  } catch (const ::cube::Error& e) {                                                  \
    return ::cube::batch_fail(b, e);                                                  \
  } catch (const std::bad_alloc&) {                                                   \
    return ::cube::batch_fail(b, ::cube::Error{CUBE_E_NOMEM, "host allocation failed"}); \
  } catch (const std::exception& e) {                                                 \
    return ::cube::batch_fail(b, ::cube::Error{CUBE_E_INVALID, e.what()});            \
  }

// one step of a box on stream st with the factors taken from the device schedule
// (the step-end kernel records a failure under the device step counter's code and advances it)
void enqueue_graph_step(Sim& s, hipStream_t st) {
  launch_deposit(s, st);
  solve_potential(s, st);
  if (s.inject_step >= 0) launch_raise_flag(s, st, s.inject_flag, true, s.inject_step);
  launch_move(s, 0, 0.0f, 0.0f, nullptr, 0.0f, st, nullptr, true);
  launch_step_end(s, st, 0u, true);
}

void destroy_graphs(cube_batch& b) {
  for (int p = 0; p < 2; ++p) {
    if (b.exec[p]) (void)hipGraphExecDestroy(b.exec[p]);
    if (b.graph[p]) (void)hipGraphDestroy(b.graph[p]);
    b.exec[p] = nullptr;
    b.graph[p] = nullptr;
    b.table[p].reset();
  }
}

// mode 2: the stages of one ensemble step from parity `par`, each one launch (per kernel variant)
// over every box, in the order of enqueue_graph_step
std::unique_ptr<EnsembleStep> plan_table_step(cube_batch& b) {
  std::vector<Sim*> ss;
  for (cube_sim* x : b.boxes) ss.push_back(&x->s);
  auto es = std::make_unique<EnsembleStep>();
  ensemble_deposit(*es, ss);
  ensemble_solve(*es, ss);
  for (Sim* s : ss)
    if (s->inject_step >= 0) {
      const uint32_t f = s->inject_flag;
      const int at = s->inject_step;
      es->launches.push_back([s, f, at](hipStream_t st) { launch_raise_flag(*s, st, f, true, at); });
    }
  ensemble_move(*es, ss);
  ensemble_step_end(*es, ss);
  es->upload();
  return es;
}

// capture one ensemble step starting from state parity `par` (every box has cur == par)
void build_graph(cube_batch& b, int par) {
  if (b.mode == 2 && !b.table[par]) b.table[par] = plan_table_step(b);
  CUBE_HIP(hipStreamBeginCapture(b.main, hipStreamCaptureModeRelaxed));
  try {
    if (b.mode == 2) {
      b.table[par]->enqueue(b.main);
    } else {
      CUBE_HIP(hipEventRecord(b.fork, b.main));
      for (size_t i = 0; i < b.boxes.size(); ++i) {
        Sim& s = b.boxes[i]->s;
        CUBE_HIP(hipStreamWaitEvent(b.streams[i], b.fork, 0));
        enqueue_graph_step(s, b.streams[i]);
        s.cur = par;  // the capture flipped the host-side parity; replays flip it instead
        CUBE_HIP(hipEventRecord(b.joins[i], b.streams[i]));
        CUBE_HIP(hipStreamWaitEvent(b.main, b.joins[i], 0));
      }
    }
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(b.main, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  CUBE_HIP(hipStreamEndCapture(b.main, &b.graph[par]));
  CUBE_HIP(hipGraphInstantiate(&b.exec[par], b.graph[par], nullptr, nullptr, 0));
}

// drop captured graphs that a later change of a box (variants, particle IDs) has made stale
void check_graphs(cube_batch& b) {
  std::vector<int> now(b.boxes.size());
  for (size_t i = 0; i < b.boxes.size(); ++i) now[i] = b.boxes[i]->s.config_gen;
  if (now != b.gens) {
    destroy_graphs(b);
    b.gens = now;
  }
}

// z layout of the solve: 1 allocates the scratch copy (one mesh-sized buffer) if needed, 0 keeps
// any allocated scratch, -1 selects 0 and frees the scratch. The scratch also holds the move
// passes' per (cell, displacement) counts and slots (27 x 4 bytes each per coarse cell, less than
// the mesh's 64 x 4): the copy is live only inside a solve, the counts and slots only inside a
// move, so one buffer serves both and their own allocation is given back.
void set_z_layout(Sim& s, int layout) {
  FFTPlan& pl = s.mesh_plan;
  s.config_gen++;
  const size_t mig_bytes = sizeof(uint32_t) * 27 * (size_t)s.nc3;
  if (layout == 1 && !pl.zscratch) {
    const size_t zb = pl.field_floats() * sizeof(float);
    char* w = static_cast<char*>(s.dmalloc(std::max(zb, 2 * mig_bytes)));
    s.dfree(s.mig);
    s.dfree(s.slot);
    pl.zscratch = reinterpret_cast<float2*>(w);
    s.mig = reinterpret_cast<uint32_t*>(w);
    s.slot = reinterpret_cast<uint32_t*>(w + mig_bytes);
  }
  if (layout < 0 && pl.zscratch) {
    uint32_t* m = static_cast<uint32_t*>(s.dmalloc(mig_bytes));
    uint32_t* sl = static_cast<uint32_t*>(s.dmalloc(mig_bytes));
    s.dfree(pl.zscratch);
    pl.zscratch = nullptr;
    s.mig = m;
    s.slot = sl;
  }
  pl.zlayout = layout > 0 ? 1 : 0;
}

float elapsed_ms(hipEvent_t a, hipEvent_t z) {
  CUBE_HIP(hipEventSynchronize(z));
  float ms = 0.f;
  CUBE_HIP(hipEventElapsedTime(&ms, a, z));
  return ms;
}

// Time the equivalent variants of the deposit, of the FFT column passes and of the move passes on
// the current state and keep the fastest of each. The particle state is left unchanged (timed
// moves write only the next-state buffers and scratch, and the parity is restored); the mesh is
// left holding the potential of the current state.
void autotune_sim(Sim& s) {
  require_particles(s);
  hipEvent_t e0 = s.ev[14], e1 = s.ev[15];
  constexpr int reps = 2;
  auto timed = [&](auto&& fn) {
    float t = 0.f;
    for (int r = 0; r <= reps; ++r) {
      CUBE_HIP(hipEventRecord(e0, s.stream));
      fn();
      CUBE_HIP(hipEventRecord(e1, s.stream));
      const float ms = elapsed_ms(e0, e1);
      if (r > 0) t += ms;  // the first run warms up
    }
    return t;
  };
  // deposit: particle order and workgroup size
  std::string rep;
  auto note = [&](const std::string& what, float ms) {
    char b[96];
    std::snprintf(b, sizeof(b), "%s %.3f ms; ", what.c_str(), ms / reps);
    rep += b;
  };
  int best_d = s.deposit_variant;
  float best = 1e30f;
  for (int v : {0, 1, 2, 3}) {
    s.deposit_variant = v;
    const float t = timed([&] { launch_deposit(s, s.stream); });
    note("deposit " + std::to_string(v), t);
    if (t < best) {
      best = t;
      best_d = v;
    }
  }
  s.deposit_variant = best_d;
  // FFT column width, z-pass workgroup order and z layout (the scratch layout only if its buffer
  // can be allocated)
  int best_bx = s.mesh_plan.colbx, best_z = s.mesh_plan.zorder, best_l = s.mesh_plan.zlayout;
  best = 1e30f;
  const bool had_scratch = s.mesh_plan.zscratch != nullptr;
  try {
    set_z_layout(s, 1);
  } catch (const Error& e) {
    if (e.code != CUBE_E_NOMEM) throw;
  }
  int best_zbx = s.mesh_plan.zbx;
  const int max_layout = s.mesh_plan.zscratch ? 1 : 0;
  const std::vector<int> widths = fft_col_widths(s.nm);
  for (int l = 0; l <= max_layout; ++l) {
    for (int bx : widths) {
      // layout 0: z passes of the same width in either workgroup order; layout 1: z passes of any
      // width dividing the layout's
      for (int zb : widths) {
        if (l == 0 ? zb != bx : bx % zb != 0) continue;
        for (int z = 0; z <= (l == 0 ? 1 : 0); ++z) {
          s.mesh_plan.colbx = bx;
          s.mesh_plan.zbx = zb;
          s.mesh_plan.zorder = z;
          s.mesh_plan.zlayout = l;
          launch_deposit(s, s.stream);
          const float t = timed([&] { solve_potential(s, s.stream); });
          note("solve layout " + std::to_string(l) + " width " + std::to_string(bx) + "/" + std::to_string(zb) +
                   " order " + std::to_string(z), t);
          if (t < best) {
            best = t;
            best_bx = bx;
            best_zbx = zb;
            best_z = z;
            best_l = l;
          }
        }
      }
    }
  }
  s.mesh_plan.colbx = best_bx;
  s.mesh_plan.zbx = best_zbx;
  s.mesh_plan.zorder = best_z;
  if (best_l == 0 && !had_scratch) CUBE_HIP(hipStreamSynchronize(s.stream));
  set_z_layout(s, best_l == 0 && !had_scratch ? -1 : best_l);
  launch_deposit(s, s.stream);
  solve_potential(s, s.stream);
  // move passes: per-corner gradient vs precomputed gradient tile, each pass timed on its own
  // (events around the count and the scatter pass), with this step's factors
  const int j = std::min(s.steps_done, s.p.n_steps - 1);
  const float kf = (float)(-s.kicks[j] / 12.0), df = (float)s.drifts[j];
  float tc[2] = {0.f, 0.f}, ts[2] = {0.f, 0.f};
  hipEvent_t* me = s.ev + 8;  // four events: before count, after count, after link, after scatter
  for (int v = 0; v <= 1; ++v) {
    s.move_variant = v;
    for (int r = 0; r <= reps; ++r) {
      const int cur = s.cur;
      launch_move(s, 0, kf, df, nullptr, 0.0f, s.stream, me);
      s.cur = cur;  // discard the result
      const float c = elapsed_ms(me[0], me[1]), sc = elapsed_ms(me[2], me[3]);
      if (r > 0) {
        tc[v] += c;
        ts[v] += sc;
      }
    }
  }
  for (int v = 0; v <= 1; ++v) {
    note("count " + std::to_string(v), tc[v]);
    note("scatter " + std::to_string(v), ts[v]);
  }
  s.autotune_report = rep;
  const bool tcnt = tc[1] < tc[0], tsct = ts[1] < ts[0];
  s.move_variant = tcnt ? (tsct ? 1 : 3) : (tsct ? 2 : 0);
  // a timed move may have raised a flag that the real step will raise again; clear it here
  CUBE_HIP(hipMemsetAsync(s.flags, 0, sizeof(uint32_t), s.stream));
  CUBE_HIP(hipStreamSynchronize(s.stream));
}

}  // namespace
}  // namespace cube

using cube::Error;

extern "C" {

int cube_autotune(cube_sim* sim) {
  if (!sim) return CUBE_E_INVALID;
  try {
    cube::autotune_sim(sim->s);
  } catch (const Error& e) {
    sim->s.last_error = e.msg;
    return e.code;
  } catch (const std::exception& e) {
    sim->s.last_error = e.what();
    return CUBE_E_INVALID;
  }
  return CUBE_OK;
}

const char* cube_autotune_report(const cube_sim* sim) { return sim ? sim->s.autotune_report.c_str() : ""; }

int cube_get_variant(const cube_sim* sim, cube_variant* out) {
  if (!sim || !out) return CUBE_E_INVALID;
  const cube::Sim& s = sim->s;
  out->move_variant = s.move_variant;
  out->fft_col_width = s.mesh_plan.colbx;
  out->fft_z_order = s.mesh_plan.zorder;
  out->deposit_variant = s.deposit_variant;
  out->fft_z_layout = s.mesh_plan.zlayout;
  out->fft_z_width = s.mesh_plan.zbx;
  return CUBE_OK;
}

int cube_set_variant(cube_sim* sim, const cube_variant* v) {
  if (!sim || !v) return CUBE_E_INVALID;
  cube::Sim& s = sim->s;
  const std::vector<int> ok = cube::fft_col_widths(s.nm);
  std::string err;
  if (v->move_variant < -1 || v->move_variant > 3) err = "move_variant must be in -1..3";
  else if (std::find(ok.begin(), ok.end(), v->fft_col_width) == ok.end())
    err = "unsupported FFT column width for this mesh size";
  else if (v->fft_z_order < 0 || v->fft_z_order > 1) err = "fft_z_order must be 0 or 1";
  else if (v->deposit_variant < 0 || v->deposit_variant > 3) err = "deposit_variant must be in 0..3";
  else if (v->fft_z_layout < 0 || v->fft_z_layout > 1) err = "fft_z_layout must be 0 or 1";
  else if (std::find(ok.begin(), ok.end(), v->fft_z_width) == ok.end() || v->fft_col_width % v->fft_z_width != 0)
    err = "fft_z_width must be a supported width dividing fft_col_width";
  if (!err.empty()) {
    s.last_error = err;
    return CUBE_E_INVALID;
  }
  try {
    if (v->fft_z_layout != s.mesh_plan.zlayout) CUBE_HIP(hipStreamSynchronize(s.stream));
    cube::set_z_layout(s, v->fft_z_layout ? 1 : -1);
  } catch (const Error& e) {
    s.last_error = e.msg;
    return e.code;
  }
  s.config_gen++;  // captured step graphs hold the previous kernels and buffers
  s.move_variant = v->move_variant;
  s.mesh_plan.colbx = v->fft_col_width;
  s.mesh_plan.zorder = v->fft_z_order;
  s.mesh_plan.zbx = v->fft_z_width;
  s.deposit_variant = v->deposit_variant;
  return CUBE_OK;
}

int cube_batch_create(const cube_params* params, int32_t nbox, void* stream, const cube_allocator* alloc,
                      cube_batch** out) {
  if (!params || !out || nbox < 1) return CUBE_E_INVALID;
  *out = nullptr;
  cube_batch* b = nullptr;
  try {
    b = new cube_batch();
  } catch (...) {
    return CUBE_E_NOMEM;
  }
  try {
    b->main = static_cast<hipStream_t>(stream);
    if (!b->main) {
      CUBE_HIP(hipStreamCreateWithFlags(&b->main, hipStreamNonBlocking));
      b->own_main = true;
    }
    for (int i = 1; i < nbox; ++i)
      if (params[i].n_steps != params[0].n_steps) throw Error{CUBE_E_INVALID, "every box must have the same n_steps"};
    CUBE_HIP(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
    for (int i = 0; i < nbox; ++i) {
      hipStream_t st = nullptr;
      CUBE_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      b->streams.push_back(st);
      hipEvent_t ev = nullptr;
      CUBE_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      b->joins.push_back(ev);
      cube_sim* sim = nullptr;
      const int rc = cube_create(&params[i], st, alloc, &sim);
      if (rc != CUBE_OK) throw Error{rc, "box " + std::to_string(i) + ": " + cube_last_error(nullptr)};
      b->boxes.push_back(sim);
    }
  } catch (const Error& e) {
    cube::g_batch_create_error = e.msg;
    cube_batch_destroy(b);
    return e.code;
  } catch (const std::exception& e) {
    cube::g_batch_create_error = e.what();
    cube_batch_destroy(b);
    return CUBE_E_NOMEM;
  }
  *out = b;
  return CUBE_OK;
}

void cube_batch_destroy(cube_batch* b) {
  if (!b) return;
  if (b->main) (void)hipStreamSynchronize(b->main);
  cube::destroy_graphs(*b);
  for (cube_sim* s : b->boxes) cube_destroy(s);
  for (hipStream_t st : b->streams) (void)hipStreamDestroy(st);
  for (hipEvent_t ev : b->joins) (void)hipEventDestroy(ev);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->own_main) (void)hipStreamDestroy(b->main);
  delete b;
}

const char* cube_batch_last_error(const cube_batch* b) {
  return b ? b->last_error.c_str() : cube::g_batch_create_error.c_str();
}

int32_t cube_batch_size(const cube_batch* b) { return b ? (int32_t)b->boxes.size() : 0; }

cube_sim* cube_batch_box(cube_batch* b, int32_t i) {
  if (!b || i < 0 || i >= (int32_t)b->boxes.size()) return nullptr;
  return b->boxes[i];
}

int cube_batch_set_mode(cube_batch* b, int32_t mode) {
  if (!b) return CUBE_E_INVALID;
  if (mode < 0 || mode > 2) {
    b->last_error = "batch mode must be 0 (graph of per-box branches), 1 (streams) or 2 (graph of ensemble launches)";
    return CUBE_E_INVALID;
  }
  if (mode == 2)
    for (size_t i = 0; i < b->boxes.size(); ++i)
      if (b->boxes[i]->s.two_level_rs > 0.0) {
        b->last_error = "box " + std::to_string(i) + ": ensemble launches need single-level solves";
        return CUBE_E_INVALID;
      }
  if (mode != b->mode) {
    if (b->main) (void)hipStreamSynchronize(b->main);
    cube::destroy_graphs(*b);
  }
  b->mode = mode;
  return CUBE_OK;
}

int cube_batch_init_ic(cube_batch* b) {
  if (!b) return CUBE_E_INVALID;
  for (size_t i = 0; i < b->boxes.size(); ++i) {
    const int rc = cube_init_ic(b->boxes[i]);
    if (rc != CUBE_OK) {
      b->last_error = "box " + std::to_string(i) + ": " + cube_last_error(b->boxes[i]);
      return rc;
    }
  }
  cube::destroy_graphs(*b);
  return CUBE_OK;
}

int cube_batch_autotune(cube_batch* b) {
  if (!b) return CUBE_E_INVALID;
  // one measurement per distinct box shape, applied to every box of that shape
  std::map<std::tuple<int, int, int, int>, cube_variant> chosen;
  for (size_t i = 0; i < b->boxes.size(); ++i) {
    cube::Sim& s = b->boxes[i]->s;
    const auto key = std::make_tuple(s.nm, s.np, s.nchi, s.nnu);
    auto it = chosen.find(key);
    if (it == chosen.end()) {
      const int rc = cube_autotune(b->boxes[i]);
      if (rc != CUBE_OK) {
        b->last_error = "box " + std::to_string(i) + ": " + cube_last_error(b->boxes[i]);
        return rc;
      }
      cube_variant v;
      cube_get_variant(b->boxes[i], &v);
      chosen[key] = v;
    } else {
      cube_set_variant(b->boxes[i], &it->second);
    }
  }
  cube::destroy_graphs(*b);  // the captured kernels depend on the variants
  return CUBE_OK;
}

int cube_batch_step(cube_batch* b, int32_t k) {
  if (!b || k < 0) return CUBE_E_INVALID;
  int rc = CUBE_OK;
  CUBE_BATCH_GUARD(b, {
    std::vector<cube::Sim*> ss;
    for (cube_sim* x : b->boxes) ss.push_back(&x->s);
    for (size_t i = 0; i < ss.size(); ++i) {
      cube::require_particles(*ss[i]);
      if (ss[i]->adaptive) throw Error{CUBE_E_INVALID, "adaptive time steps are not supported in a batch"};
      if (b->mode == 2 && ss[i]->two_level_rs > 0.0)
        throw Error{CUBE_E_INVALID, "box " + std::to_string(i) + ": ensemble launches need single-level solves"};
    }
    const int done = ss[0]->steps_done;
    for (cube::Sim* s : ss)
      if (s->steps_done != done || s->cur != ss[0]->cur)
        throw Error{CUBE_E_STATE, "boxes of a batch must be at the same step (step them with cube_batch_step only)"};
    // the initial half drift (no force) of every box, each on its own stream
    for (size_t i = 0; i < ss.size(); ++i) {
      cube::Sim& s = *ss[i];
      if (!s.half_drift_done) {
        s.phases.push_back({1u, s.cur, s.steps_done, false});
        cube::launch_move(s, 1, 0.0f, (float)s.drift0, nullptr, 0.0f, s.stream, nullptr);
        cube::launch_step_end(s, s.stream, 1u, false);
        s.half_drift_done = true;
      }
    }
    for (size_t i = 0; i < ss.size(); ++i) {
      cube::Sim& s = *ss[i];
      CUBE_HIP(hipMemcpyAsync(s.step_dev, &s.steps_done, sizeof(int), hipMemcpyHostToDevice, s.stream));
      CUBE_HIP(hipEventRecord(b->joins[i], s.stream));
      CUBE_HIP(hipStreamWaitEvent(b->main, b->joins[i], 0));
    }
    // the upload above reads host memory asynchronously: keep it alive until it has landed
    CUBE_HIP(hipStreamSynchronize(b->main));
    for (int i = 0; i < k; ++i) {
      if (ss[0]->steps_done >= ss[0]->p.n_steps) {
        rc = CUBE_DONE;
        break;
      }
      for (cube::Sim* s : ss) s->phases.push_back({(uint32_t)s->steps_done + 2u, s->cur, s->steps_done, true});
      if (b->mode != 1) {
        cube::check_graphs(*b);
        const int par = ss[0]->cur;
        if (!b->exec[par]) cube::build_graph(*b, par);
        CUBE_HIP(hipGraphLaunch(b->exec[par], b->main));
        for (cube::Sim* s : ss) {
          s->cur ^= 1;
          s->steps_done++;
        }
      } else {
        // one step of every box on its own stream: the hardware queues run them side by side
        for (size_t bi = 0; bi < ss.size(); ++bi) cube::enqueue_graph_step(*ss[bi], b->streams[bi]);
        for (cube::Sim* s : ss) s->steps_done++;  // launch_move flipped the parity already
      }
    }
    if (b->mode == 1)
      for (size_t bi = 0; bi < ss.size(); ++bi) {
        CUBE_HIP(hipEventRecord(b->joins[bi], b->streams[bi]));
        CUBE_HIP(hipStreamWaitEvent(b->main, b->joins[bi], 0));
      }
    CUBE_HIP(hipStreamSynchronize(b->main));
    // every box's flags are checked (a failed box goes back to the state before its failing step,
    // the others keep their steps); the first failure is reported
    std::string first;
    int first_code = CUBE_OK;
    for (size_t i = 0; i < ss.size(); ++i) {
      try {
        cube::check_flags(*ss[i]);
      } catch (const Error& e) {
        if (first_code == CUBE_OK) {
          first_code = e.code;
          first = "box " + std::to_string(i) + ": " + e.msg;
        }
      }
    }
    if (first_code != CUBE_OK) throw Error{first_code, first};
  });
  return rc;
}

}  // extern "C"
