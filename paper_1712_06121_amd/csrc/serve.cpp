// Simulation server: continuous batching of independent PM jobs on one GPU.
//
// Jobs are queued in submission order. A scheduling round (cube_server_poll) first looks at every
// active job: if the steps last enqueued for it have finished (an event query, no wait), its error
// flags are checked and either it is parked as finished or its next slice of steps is enqueued.
// Then queued jobs are admitted, oldest first, while their device footprint fits the memory left
// and an execution slot is free: each gets its own stream, its initial conditions and its first
// slice. Jobs therefore join and leave while others are running, and the kernels of all active
// jobs overlap on the device. A finished job keeps its memory (its state, density and P(k) stay
// readable through cube_server_job) until cube_server_release.
#include <algorithm>
#include <deque>
#include <map>

#include "cube_internal.h"

namespace {

enum JobState { QUEUED = 0, ACTIVE = 1, FINISHED = 2, FAILED = 3 };

struct Job {
  int64_t id = 0;
  cube_params p{};
  int64_t footprint = 0;
  cube_sim* sim = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;  // recorded after the last enqueued slice
  int state = QUEUED;
  int rc = CUBE_OK;
  std::string error;
};

}  // namespace

struct cube_server {
  int64_t budget = 0;
  int64_t in_use = 0;
  int max_active = 1;
  int slice = 1;
  cube_allocator alloc{};
  bool has_alloc = false;
  std::deque<Job*> queue;
  std::vector<Job*> active;
  std::map<int64_t, Job*> jobs;  // every job not yet released
  std::vector<hipStream_t> free_streams;
  std::vector<hipEvent_t> free_events;
  std::deque<int64_t> unreported;  // finished or failed, not yet returned by a poll
  std::string last_error;
};

namespace {

using cube::Error;

int server_fail(cube_server* s, const Error& e) {
  if (s) s->last_error = e.msg;
  return e.code;
}

void enqueue_slice(cube_server& srv, Job& j) {
  cube::Sim& s = j.sim->s;
  (void)cube::enqueue_steps(s, srv.slice);
  CUBE_HIP(hipEventRecord(j.done, j.stream));
}

// a finished or failed job keeps its stream (its simulation still uses it) until released
void retire(cube_server& srv, Job& j, int state) {
  j.state = state;
  srv.free_events.push_back(j.done);
  j.done = nullptr;
}

void admit(cube_server& srv, Job& j) {
  if (!srv.free_streams.empty()) {
    j.stream = srv.free_streams.back();
    srv.free_streams.pop_back();
  } else {
    CUBE_HIP(hipStreamCreateWithFlags(&j.stream, hipStreamNonBlocking));
  }
  if (!srv.free_events.empty()) {
    j.done = srv.free_events.back();
    srv.free_events.pop_back();
  } else {
    CUBE_HIP(hipEventCreateWithFlags(&j.done, hipEventDisableTiming));
  }
  srv.in_use += j.footprint;
  j.state = ACTIVE;
  int rc = cube_create(&j.p, j.stream, srv.has_alloc ? &srv.alloc : nullptr, &j.sim);
  if (rc == CUBE_OK) rc = cube_init_ic(j.sim);
  if (rc != CUBE_OK) {
    j.rc = rc;
    j.error = j.sim ? cube_last_error(j.sim) : cube_last_error(nullptr);
    retire(srv, j, FAILED);
    return;
  }
  enqueue_slice(srv, j);
}

}  // namespace

extern "C" {

int cube_server_create(int64_t mem_budget_bytes, int32_t max_active, int32_t slice_steps,
                       const cube_allocator* alloc, cube_server** out) {
  if (!out || mem_budget_bytes <= 0 || max_active < 1 || slice_steps < 1) return CUBE_E_INVALID;
  *out = nullptr;
  cube_server* s = nullptr;
  try {
    s = new cube_server();
  } catch (...) {
    return CUBE_E_NOMEM;
  }
  s->budget = mem_budget_bytes;
  s->max_active = max_active;
  s->slice = slice_steps;
  if (alloc && alloc->alloc && alloc->free) {
    s->alloc = *alloc;
    s->has_alloc = true;
  }
  *out = s;
  return CUBE_OK;
}

void cube_server_destroy(cube_server* srv) {
  if (!srv) return;
  for (auto& kv : srv->jobs) {
    Job* j = kv.second;
    if (j->stream) (void)hipStreamSynchronize(j->stream);
    if (j->sim) cube_destroy(j->sim);
    if (j->stream) (void)hipStreamDestroy(j->stream);
    if (j->done) (void)hipEventDestroy(j->done);
    delete j;
  }
  for (hipStream_t st : srv->free_streams) (void)hipStreamDestroy(st);
  for (hipEvent_t ev : srv->free_events) (void)hipEventDestroy(ev);
  delete srv;
}

const char* cube_server_last_error(const cube_server* srv) { return srv ? srv->last_error.c_str() : ""; }

int cube_server_submit(cube_server* srv, const cube_params* params, int64_t job_id) {
  if (!srv || !params) return CUBE_E_INVALID;
  if (srv->jobs.count(job_id)) return server_fail(srv, Error{CUBE_E_INVALID, "job id already in use"});
  const int64_t fp = cube_footprint(params);
  if (fp < 0) return server_fail(srv, Error{CUBE_E_INVALID, "invalid job parameters"});
  if (fp > srv->budget)
    return server_fail(srv, Error{CUBE_E_CAPACITY, "job footprint exceeds the server's memory budget"});
  Job* j = nullptr;
  try {
    j = new Job();
  } catch (...) {
    return CUBE_E_NOMEM;
  }
  j->id = job_id;
  j->p = *params;
  j->footprint = fp;
  srv->jobs[job_id] = j;
  srv->queue.push_back(j);
  return CUBE_OK;
}

int cube_server_poll(cube_server* srv, int64_t* finished, int32_t max_finished, int32_t* n_finished) {
  if (!srv || !n_finished || max_finished < 0 || (max_finished > 0 && !finished)) return CUBE_E_INVALID;
  *n_finished = 0;
  try {
    // progress of the active jobs
    std::vector<Job*> still;
    for (Job* j : srv->active) {
      const hipError_t q = hipEventQuery(j->done);
      if (q == hipErrorNotReady) {
        still.push_back(j);
        continue;
      }
      CUBE_HIP(q);
      cube::Sim& s = j->sim->s;
      try {
        cube::check_flags(s);
      } catch (const Error& e) {
        j->rc = e.code;
        j->error = e.msg;
        retire(*srv, *j, FAILED);
        srv->unreported.push_back(j->id);
        continue;
      }
      if (s.steps_done >= s.p.n_steps) {
        retire(*srv, *j, FINISHED);
        srv->unreported.push_back(j->id);
        continue;
      }
      enqueue_slice(*srv, *j);
      still.push_back(j);
    }
    srv->active.swap(still);
    // admission, oldest first, while memory and a slot are free
    while (!srv->queue.empty() && (int)srv->active.size() < srv->max_active &&
           srv->in_use + srv->queue.front()->footprint <= srv->budget) {
      Job* j = srv->queue.front();
      srv->queue.pop_front();
      admit(*srv, *j);
      if (j->state == ACTIVE) srv->active.push_back(j);
      else srv->unreported.push_back(j->id);  // failed at creation
    }
    while (!srv->unreported.empty() && *n_finished < max_finished) {
      finished[(*n_finished)++] = srv->unreported.front();
      srv->unreported.pop_front();
    }
  } catch (const Error& e) {
    return server_fail(srv, e);
  } catch (const std::exception& e) {
    return server_fail(srv, Error{CUBE_E_INVALID, e.what()});
  }
  return CUBE_OK;
}

int cube_server_status(const cube_server* srv, int64_t job_id, int32_t* state, int32_t* rc) {
  if (!srv) return CUBE_E_INVALID;
  auto it = srv->jobs.find(job_id);
  if (it == srv->jobs.end()) return CUBE_E_INVALID;
  if (state) *state = it->second->state;
  if (rc) *rc = it->second->rc;
  return CUBE_OK;
}

const char* cube_server_job_error(const cube_server* srv, int64_t job_id) {
  if (!srv) return "";
  auto it = srv->jobs.find(job_id);
  return it == srv->jobs.end() ? "" : it->second->error.c_str();
}

cube_sim* cube_server_job(cube_server* srv, int64_t job_id) {
  if (!srv) return nullptr;
  auto it = srv->jobs.find(job_id);
  if (it == srv->jobs.end() || it->second->state != FINISHED) return nullptr;
  return it->second->sim;
}

int cube_server_release(cube_server* srv, int64_t job_id) {
  if (!srv) return CUBE_E_INVALID;
  auto it = srv->jobs.find(job_id);
  if (it == srv->jobs.end()) return server_fail(srv, Error{CUBE_E_INVALID, "unknown job id"});
  Job* j = it->second;
  if (j->state != FINISHED && j->state != FAILED)
    return server_fail(srv, Error{CUBE_E_STATE, "only finished or failed jobs can be released"});
  if (j->sim) cube_destroy(j->sim);  // waits for the job's stream
  if (j->stream) srv->free_streams.push_back(j->stream);
  srv->in_use -= j->footprint;
  srv->jobs.erase(it);
  delete j;
  return CUBE_OK;
}

int cube_server_stats(const cube_server* srv, int32_t* queued, int32_t* active, int64_t* bytes_in_use) {
  if (!srv) return CUBE_E_INVALID;
  if (queued) *queued = (int32_t)srv->queue.size();
  if (active) *active = (int32_t)srv->active.size();
  if (bytes_in_use) *bytes_in_use = srv->in_use;
  return CUBE_OK;
}

}  // extern "C"
