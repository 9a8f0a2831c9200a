// Request loop of the served ADMM solver: a FIFO of submitted requests in front of the
// continuous-batching engine (epi_batch_*). progress() admits queued requests in arrival
// order while the engine has a free slot and HBM budget (a request that does not fit waits,
// and so do the requests behind it), runs one engine step when anything is running, and
// moves every finished volume's report to the completed list, releasing its slot (whose
// workspace the engine keeps for the next admission). Latency is completion time minus
// the arrival time the caller gave, both on the server's monotonic clock.
//
// Host code only: every iteration runs in the engine's kernels.
#include <hip/hip_runtime.h>

#include <string.h>

#include <chrono>
#include <deque>
#include <map>
#include <vector>

#include "epi.h"
#include "epi_internal.hpp"

#define EPI_API extern "C" __attribute__((visibility("default")))

using namespace epi;

namespace {

double now_s() {
  using clk = std::chrono::steady_clock;
  return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

struct Request {
  int64_t id = 0;
  double arrival = 0.0, admitted = 0.0, completed = 0.0;
  epi_grid grid{};
  const float *Ip = nullptr, *Im = nullptr;
  float *b = nullptr, *z = nullptr, *u = nullptr;
  epi_admm_opts opts{};
  int32_t slot = -1;
  // report, copied from the engine when the volume finishes
  int32_t iters = 0, converged = 0, status = EPI_OK, max_active = 0;
  int64_t hard_lines = 0;
  std::vector<double> hist[5];
};

}  // namespace

struct epi_server {
  epi_batch* engine = nullptr;
  std::deque<Request> queue;              // submitted, not yet admitted (arrival order)
  std::map<int32_t, Request> running;     // by slot
  std::deque<Request> done;               // finished, not yet taken (completion order)
  int64_t completed_total = 0;
};

EPI_API double epi_server_clock(void) { return now_s(); }

EPI_API epi_status epi_server_create(int32_t max_slots, int64_t hbm_budget_bytes,
                                     int32_t precision, int32_t iters_per_step, void* stream,
                                     epi_server** out) {
  if (!out) return fail(EPI_EINVAL, "null argument");
  *out = nullptr;
  epi_batch* bt = nullptr;
  epi_status s = epi_batch_create(max_slots, hbm_budget_bytes, precision, iters_per_step, stream, &bt);
  if (s != EPI_OK) return s;
  epi_server* sv = new epi_server();
  sv->engine = bt;
  *out = sv;
  return EPI_OK;
}

EPI_API void epi_server_destroy(epi_server* sv) {
  if (!sv) return;
  epi_batch_destroy(sv->engine);
  delete sv;
}

EPI_API epi_status epi_server_submit(epi_server* sv, int64_t request_id, double arrival_s,
                                     const epi_grid* grid, const float* d_Iplus,
                                     const float* d_Iminus, float* d_b, float* d_z, float* d_u,
                                     const epi_admm_opts* opts) {
  if (!sv || !grid || !d_Iplus || !d_Iminus || !d_b || !d_z || !d_u || !opts)
    return fail(EPI_EINVAL, "null argument");
  if (opts->max_iter < 1) return fail(EPI_EINVAL, "max_iter must be >= 1");
  epi_status vs = validate_grid(grid);
  if (vs != EPI_OK) return vs;
  Request r;
  r.id = request_id;
  r.arrival = arrival_s;
  r.grid = *grid;
  r.Ip = d_Iplus;
  r.Im = d_Iminus;
  r.b = d_b;
  r.z = d_z;
  r.u = d_u;
  r.opts = *opts;
  sv->queue.push_back(r);
  return EPI_OK;
}

// Admit from the head of the queue until the engine is busy. A request the engine rejects
// for another reason (infeasible start, bad options) completes at once with that status.
static epi_status admit_queued(epi_server* sv) {
  while (!sv->queue.empty()) {
    Request& r = sv->queue.front();
    int32_t slot = -1;
    epi_status s = epi_batch_admit(sv->engine, &r.grid, r.Ip, r.Im, r.b, r.z, r.u, &r.opts, &slot);
    if (s == EPI_EBUSY) {
      if (sv->running.empty())   // nothing will free up: the request can never fit
        return fail(EPI_ENOMEM, "request %lld does not fit the engine's slots or HBM budget",
                    (long long)r.id);
      return EPI_OK;
    }
    if (s == EPI_EHIP || s == EPI_ENOMEM) return s;
    r.admitted = now_s();
    if (s != EPI_OK) {
      r.status = s;
      r.completed = r.admitted;
      sv->done.push_back(r);
      sv->completed_total += 1;
    } else {
      r.slot = slot;
      sv->running[slot] = r;
    }
    sv->queue.pop_front();
  }
  return EPI_OK;
}

EPI_API epi_status epi_server_progress(epi_server* sv, int32_t* queued, int32_t* running,
                                       int32_t* ready) {
  if (!sv) return fail(EPI_EINVAL, "null argument");
  epi_status s = admit_queued(sv);
  if (s != EPI_OK) return s;
  if (!sv->running.empty()) {
    int32_t n = 0;
    s = epi_batch_step(sv->engine, &n);
    if (s != EPI_OK) return s;
    const double t = now_s();
    for (auto it = sv->running.begin(); it != sv->running.end();) {
      Request& r = it->second;
      int32_t fin = 0;
      s = epi_batch_poll(sv->engine, r.slot, &fin, nullptr);
      if (s != EPI_OK) return s;
      if (!fin) {
        ++it;
        continue;
      }
      const int cap = r.opts.max_iter;
      for (auto& h : r.hist) h.assign(cap, 0.0);
      epi_admm_report rep{};
      rep.r_pri = r.hist[0].data();
      rep.r_dual = r.hist[1].data();
      rep.eps_pri = r.hist[2].data();
      rep.eps_dual = r.hist[3].data();
      rep.rho = r.hist[4].data();
      s = epi_batch_poll(sv->engine, r.slot, &fin, &rep);
      if (s != EPI_OK) return s;
      r.iters = rep.iters;
      r.converged = rep.converged;
      r.status = rep.status;
      r.max_active = rep.max_active;
      r.hard_lines = rep.hard_lines;
      r.completed = t;
      s = epi_batch_release(sv->engine, r.slot);
      if (s != EPI_OK) return s;
      sv->done.push_back(r);
      sv->completed_total += 1;
      it = sv->running.erase(it);
    }
    // slots freed this step take queued requests before the caller's next call
    s = admit_queued(sv);
    if (s != EPI_OK) return s;
  }
  if (queued) *queued = (int32_t)sv->queue.size();
  if (running) *running = (int32_t)sv->running.size();
  if (ready) *ready = (int32_t)sv->done.size();
  return EPI_OK;
}

EPI_API epi_status epi_server_take(epi_server* sv, int64_t* request_id, double* latency_s,
                                   epi_admm_report* rep) {
  if (!sv || !request_id) return fail(EPI_EINVAL, "null argument");
  if (sv->done.empty()) return fail(EPI_EBUSY, "no finished request");
  Request r = sv->done.front();
  sv->done.pop_front();
  *request_id = r.id;
  if (latency_s) *latency_s = r.completed - r.arrival;
  if (rep) {
    rep->iters = r.iters;
    rep->converged = r.converged;
    rep->status = r.status;
    rep->max_active = r.max_active;
    rep->hard_lines = r.hard_lines;
    double* outs[5] = {rep->r_pri, rep->r_dual, rep->eps_pri, rep->eps_dual, rep->rho};
    for (int k = 0; k < 5; ++k)
      if (outs[k] && r.iters > 0 && !r.hist[k].empty())
        memcpy(outs[k], r.hist[k].data(), (size_t)r.iters * sizeof(double));
  }
  return EPI_OK;
}
