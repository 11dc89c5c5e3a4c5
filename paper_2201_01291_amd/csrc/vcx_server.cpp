// Request scheduler of the serving API (declarations in include/vcx.h).
//
// Continuous batching of independent solves.  A scheduler thread admits
// queued requests in arrival order while the slot count and the
// device-memory budget allow, advances all running requests of one scheme
// together (one launch per kernel per RK stage over every member's tiles) in
// chunks of a few steps, and hands requests that ended back for retirement.
// An I/O thread does the host work around the device loop: solver set-up (or
// reuse of an idle solver on the same mesh and physics), state upload, and
// result download, so the scheduler's chunks are not held up by transfers.
// Uploaded requests join their batch at the next chunk boundary.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "vcx.h"
#include "vcx_batch.h"

namespace {

using clk = std::chrono::steady_clock;

vcx_status set_err(vcx_status s, const std::string& m) { return vcx::set_error(s, m.c_str()); }

enum { QUEUED = 0, RUNNING = 1, DONE = 2 };

struct Request {
  int64_t id = 0;
  vcx_mesh mesh = nullptr;
  vcx_physics ph{};
  std::vector<double> U0, E;  // host copies taken at submission
  int nsteps = 0;
  double t_end = 0.0;
  size_t bytes = 0;
  vcx_solver s = nullptr;
  int state = QUEUED;
  bool admitted = false;  // holds a slot and its bytes of the budget
  vcx_status status = VCX_OK;
  std::string err;
  std::vector<double> U;  // final state (caller node order)
  double t = 0.0, dt_last = 0.0;
  int64_t steps = 0;
  bool ended = false;
  clk::time_point t_submit, t_admit, t_done;
};

struct Idle {
  vcx_solver s;
  size_t bytes;
  clk::time_point since;
};

struct Group {
  vcx::BatchGroup* g = nullptr;
  std::vector<Request*> mem;
  bool dirty = true;
};

double pct(std::vector<double> v, double p) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double pos = p / 100.0 * (double)(v.size() - 1);
  const size_t lo = (size_t)pos;
  const size_t hi = std::min(lo + 1, v.size() - 1);
  return v[lo] + (pos - (double)lo) * (v[hi] - v[lo]);
}

double ms_between(clk::time_point a, clk::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

}  // namespace

struct vcx_server_s {
  size_t budget = 0;
  int max_slots = 1;
  int chunk = 16;
  bool graphs = true;
  int device = 0;
  hipStream_t stream = nullptr;
  std::mutex mu;
  std::condition_variable cv_work, cv_io, cv_done;
  std::deque<Request*> queue;      // submitted, waiting for admission
  std::deque<Request*> io_start;   // admitted: solver set-up and state upload (I/O thread)
  std::deque<Request*> io_finish;  // ended: state download and release (I/O thread)
  std::deque<Request*> ready;      // uploaded: join a batch at the next chunk
  std::unordered_map<int64_t, std::unique_ptr<Request>> reqs;
  size_t resident = 0;    // bytes of admitted and idle solvers
  size_t idle_bytes = 0;
  int running = 0;        // admitted and not finished
  std::vector<Idle> idle; // finished solvers kept for reuse
  int64_t next_id = 1;
  uint64_t events = 0;  // submissions, finished requests and shutdown, counted
  bool stop = false;
  std::thread worker, io;
  // statistics (under mu)
  int64_t submitted = 0, completed = 0, failed = 0, member_steps = 0, chunks = 0, member_chunks = 0;
  std::vector<double> lat_ms, step_ms;
  size_t peak_resident = 0;
  int peak_running = 0;
  vcx_status worker_status = VCX_OK;
  std::string worker_err;

  void run();
  void run_io();
  void admit(std::vector<vcx_solver>& evict);
  void start(Request* r);
  void retire(Request* r);
  void finish_locked(Request* r, vcx_status st, const std::string& msg, bool keep);
};

// Bookkeeping of a finished request (mu held).  keep: its solver goes to the
// idle pool (bytes stay resident), else it has been destroyed.
void vcx_server_s::finish_locked(Request* r, vcx_status st, const std::string& msg, bool keep) {
  r->status = st;
  r->err = msg;
  r->state = DONE;
  r->t_done = clk::now();
  if (r->admitted) {
    if (keep)
      idle_bytes += r->bytes;
    else
      resident -= r->bytes;
    running -= 1;
    r->admitted = false;
  }
  if (st == VCX_OK) {
    completed += 1;
    lat_ms.push_back(ms_between(r->t_submit, r->t_done));
  } else {
    failed += 1;
  }
  events += 1;
  cv_done.notify_all();
  cv_work.notify_all();
}

// Admission (mu held): requests leave the queue in arrival order while a
// slot is free and their footprint fits the budget, counting idle solvers
// that can be reused as free and evicting other idle solvers when needed.
void vcx_server_s::admit(std::vector<vcx_solver>& evict) {
  while (!queue.empty() && running < max_slots) {
    Request* r = queue.front();
    if (r->bytes > budget) {
      queue.pop_front();
      r->status = VCX_E_OOM;
      r->err = "request footprint exceeds the server's device-memory budget";
      r->state = DONE;
      failed += 1;
      cv_done.notify_all();
      continue;
    }
    size_t reuse = idle.size();
    for (size_t k = 0; k < idle.size(); ++k)
      if (vcx::solver_matches(idle[k].s, r->mesh, &r->ph)) {
        reuse = k;
        break;
      }
    if (reuse < idle.size()) {
      r->s = idle[reuse].s;
      r->bytes = idle[reuse].bytes;
      idle_bytes -= r->bytes;
      idle.erase(idle.begin() + (long)reuse);
    } else {
      // evict the least recently used idle solvers until the request fits
      while (resident + r->bytes > budget && !idle.empty()) {
        auto lru = std::min_element(idle.begin(), idle.end(),
                                    [](const Idle& x, const Idle& y) { return x.since < y.since; });
        evict.push_back(lru->s);
        resident -= lru->bytes;
        idle_bytes -= lru->bytes;
        idle.erase(lru);
      }
      if (resident + r->bytes > budget) break;  // first in, first admitted
      resident += r->bytes;
    }
    queue.pop_front();
    r->admitted = true;
    running += 1;
    peak_resident = std::max(peak_resident, resident);
    peak_running = std::max(peak_running, running);
    io_start.push_back(r);
  }
  if (!io_start.empty()) cv_io.notify_one();
}

// I/O thread: solver set-up (or reuse) and state upload of an admitted request.
void vcx_server_s::start(Request* r) {
  r->t_admit = clk::now();
  vcx_status st = VCX_OK;
  if (r->s) {
    if (r->ph.model == VCX_MODEL_DRIFT_DIFFUSION) st = vcx::solver_set_field(r->s, r->E.data());
  } else {
    st = vcx_solver_create(r->mesh, &r->ph, r->E.empty() ? nullptr : r->E.data(), &r->s);
  }
  if (st == VCX_OK) st = vcx_state_upload(r->s, r->U0.data(), 0);
  std::vector<double>().swap(r->U0);
  std::vector<double>().swap(r->E);
  if (st != VCX_OK) {
    const std::string msg = vcx_last_error();
    if (r->s) (void)vcx_solver_destroy(r->s);
    r->s = nullptr;
    std::lock_guard<std::mutex> lk(mu);
    finish_locked(r, st, msg, false);
    return;
  }
  if (r->nsteps == 0) {
    retire(r);
    return;
  }
  std::lock_guard<std::mutex> lk(mu);
  r->state = RUNNING;
  ready.push_back(r);
  cv_work.notify_all();
}

// I/O thread: result download of an ended request, then its solver goes idle.
void vcx_server_s::retire(Request* r) {
  const int nvar = vcx_solver_nvar(r->s);
  vcx_status st = VCX_OK;
  std::string msg;
  std::vector<double> U((size_t)std::max(nvar, 0) * (size_t)vcx::mesh_nnodes(r->mesh));
  if (vcx_state_download(r->s, U.data(), 0) != VCX_OK) {
    st = VCX_E_HIP;
    msg = vcx_last_error();
  }
  (void)vcx_state_time(r->s, &r->t, &r->dt_last);
  if (st == VCX_OK && vcx::solver_failed(r->s)) {
    st = VCX_E_UNSTABLE;
    msg = "the solve became unstable; the result holds its last good state";
  }
  r->U.swap(U);
  const bool keep = st == VCX_OK || st == VCX_E_UNSTABLE;
  if (!keep) {
    (void)vcx_solver_destroy(r->s);
  }
  std::lock_guard<std::mutex> lk(mu);
  if (keep) idle.push_back(Idle{r->s, r->bytes, clk::now()});
  r->s = nullptr;
  finish_locked(r, st, msg, keep);
}

void vcx_server_s::run_io() {
  (void)hipSetDevice(device);
  for (;;) {
    Request* r = nullptr;
    bool fin = false;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_io.wait(lk, [&] { return !io_finish.empty() || !io_start.empty() || (stop && running == 0); });
      if (!io_finish.empty()) {  // results first: they free memory and slots
        r = io_finish.front();
        io_finish.pop_front();
        fin = true;
      } else if (!io_start.empty()) {
        r = io_start.front();
        io_start.pop_front();
      } else {
        break;
      }
    }
    if (fin)
      retire(r);
    else
      start(r);
  }
}

void vcx_server_s::run() {
  (void)hipSetDevice(device);
  std::vector<Group> groups;
  std::vector<int> ended;
  std::vector<vcx_solver> evict;
  std::vector<Request*> joined;
  uint64_t seen = ~(uint64_t)0;
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(mu);
      if (groups.empty()) {
        // nothing runs: sleep until a request is ready to join or something
        // that can change the admission decision happened (a submission, a
        // finished request, shutdown)
        cv_work.wait(lk, [&] { return !ready.empty() || events != seen || (stop && running == 0); });
      }
      seen = events;
      if (stop) {
        // cancel what has not been admitted; admitted requests are finished
        for (Request* r : queue) {
          r->status = VCX_E_BUSY;
          r->err = "server shut down before the request started";
          r->state = DONE;
          failed += 1;
        }
        queue.clear();
        cv_done.notify_all();
        if (running == 0) break;
      } else {
        admit(evict);
      }
      joined.assign(ready.begin(), ready.end());
      ready.clear();
    }
    for (vcx_solver s : evict) (void)vcx_solver_destroy(s);
    evict.clear();
    for (Request* r : joined) {
      Group* home = nullptr;
      for (Group& g : groups)
        if (!g.mem.empty() && vcx::batch_compatible(g.mem[0]->s, r->s)) home = &g;
      if (!home) {
        Group g;
        if (vcx::batch_create(stream, graphs, &g.g) != VCX_OK) {
          // no batch for it: the request ends with its uploaded state
          std::lock_guard<std::mutex> lk(mu);
          r->ended = true;
          io_finish.push_back(r);
          cv_io.notify_one();
          continue;
        }
        groups.push_back(g);
        home = &groups.back();
      }
      home->mem.push_back(r);
      home->dirty = true;
    }
    if (groups.empty()) continue;
    const auto t0 = clk::now();
    // steps of this chunk: no member runs past its budget inside the chunk
    int c = chunk;
    for (Group& g : groups)
      for (Request* r : g.mem) c = (int)std::min<int64_t>(c, std::max<int64_t>(1, r->nsteps - r->steps));
    vcx_status st = VCX_OK;
    for (Group& g : groups) {
      if (!g.dirty) continue;
      std::vector<vcx_solver> ss;
      std::vector<int> left;
      std::vector<double> te;
      for (Request* r : g.mem) {
        ss.push_back(r->s);
        left.push_back((int)(r->nsteps - r->steps));
        te.push_back(r->t_end);
      }
      st = vcx::batch_set(g.g, ss.data(), (int)ss.size(), left.data(), te.data());
      if (st != VCX_OK) break;
      g.dirty = false;
    }
    int members = 0;
    for (Group& g : groups) {
      if (st != VCX_OK) break;
      st = vcx::batch_run(g.g, c);
      members += (int)g.mem.size();
    }
    int64_t done_steps = 0;
    for (Group& g : groups) {
      if (st != VCX_OK) break;
      st = vcx::batch_sync(g.g, &ended);
      if (st != VCX_OK) break;
      for (size_t i = 0; i < g.mem.size(); ++i) {
        const int64_t k = vcx_steps_done(g.mem[i]->s);
        g.mem[i]->steps += k;
        g.mem[i]->ended = ended[i] != 0;
        done_steps += k;
      }
    }
    if (st != VCX_OK) {
      // a device error ends every running request of the server
      const std::string msg = vcx_last_error();
      std::lock_guard<std::mutex> lk(mu);
      for (Group& g : groups) {
        for (Request* r : g.mem) {
          if (r->s) (void)vcx_solver_destroy(r->s);
          r->s = nullptr;
          finish_locked(r, st, msg, false);
        }
        g.mem.clear();
      }
      worker_status = st;
      worker_err = msg;
    }
    {
      // ended requests go to the I/O thread for their results
      std::lock_guard<std::mutex> lk(mu);
      for (Group& g : groups) {
        for (Request*& r : g.mem)
          if (r->ended) {
            io_finish.push_back(r);
            r = nullptr;
            g.dirty = true;
          }
        g.mem.erase(std::remove(g.mem.begin(), g.mem.end(), nullptr), g.mem.end());
      }
      if (!io_finish.empty()) cv_io.notify_one();
    }
    const auto t1 = clk::now();
    {
      std::lock_guard<std::mutex> lk(mu);
      chunks += 1;
      member_chunks += members;
      member_steps += done_steps;
      step_ms.push_back(ms_between(t0, t1) / c);
    }
    for (Group& g : groups)
      if (g.mem.empty()) {
        vcx::batch_destroy(g.g);
        g.g = nullptr;
      }
    groups.erase(std::remove_if(groups.begin(), groups.end(), [](const Group& g) { return g.g == nullptr; }),
                 groups.end());
  }
  for (Group& g : groups) vcx::batch_destroy(g.g);
  {
    std::lock_guard<std::mutex> lk(mu);
    cv_io.notify_all();
  }
}

extern "C" vcx_status vcx_server_create(size_t hbm_budget, int max_slots, int chunk_steps, int use_graphs,
                                        vcx_server* out) {
  if (!out || max_slots < 1 || chunk_steps < 1 || hbm_budget == 0)
    return set_err(VCX_E_ARG, "server needs out, max_slots >= 1, chunk_steps >= 1 and a budget > 0");
  *out = nullptr;
  auto* sv = new (std::nothrow) vcx_server_s();
  if (!sv) return set_err(VCX_E_OOM, "host allocation failed");
  sv->budget = hbm_budget;
  sv->max_slots = max_slots;
  sv->chunk = chunk_steps;
  sv->graphs = use_graphs != 0;
  // (the device count first: it initialises the runtime in a process whose
  // first HIP call this is)
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0 || hipGetDevice(&sv->device) != hipSuccess ||
      hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking) != hipSuccess) {
    delete sv;
    return set_err(VCX_E_HIP, "no device or stream");
  }
  try {
    sv->io = std::thread([sv] { sv->run_io(); });
    sv->worker = std::thread([sv] { sv->run(); });
  } catch (...) {
    if (sv->io.joinable()) {
      {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
      }
      sv->cv_io.notify_all();
      sv->io.join();
    }
    (void)hipStreamDestroy(sv->stream);
    delete sv;
    return set_err(VCX_E_OOM, "cannot start the scheduler thread");
  }
  *out = sv;
  return VCX_OK;
}

extern "C" vcx_status vcx_server_submit(vcx_server sv, vcx_mesh mesh, const vcx_physics* phys, const double* U0,
                                        const double* E, int nsteps, double t_end, int64_t* id) {
  if (!sv || !mesh || !phys || !U0 || !id) return set_err(VCX_E_ARG, "NULL argument");
  if (nsteps < 0) return set_err(VCX_E_ARG, "nsteps must be >= 0");
  if (phys->model == VCX_MODEL_DRIFT_DIFFUSION && !E)
    return set_err(VCX_E_ARG, "drift-diffusion needs the electric field E");
  if (vcx::mesh_axisymmetric(mesh)) return set_err(VCX_E_ARG, "axisymmetric meshes are not served (not batched)");
  if (!vcx::mesh_simplex(mesh)) return set_err(VCX_E_ARG, "quadrilateral meshes are not served (not batched)");
  if (phys->closure == 2 || phys->predictor ||
      (phys->model == VCX_MODEL_DRIFT_DIFFUSION && phys->flux == VCX_FLUX_SG))
    return set_err(VCX_E_ARG, "the interpolated closure, the predictor and the Scharfetter-Gummel flux are "
                              "not served (not batched)");
  size_t bytes = 0;
  if (vcx::solver_footprint(mesh, phys, &bytes) != VCX_OK) return set_err(VCX_E_ARG, vcx_last_error());
  auto r = std::make_unique<Request>();
  const int nd = vcx::mesh_ndim(mesh);
  const int64_t nn = vcx::mesh_nnodes(mesh);
  const int nvar = phys->model == VCX_MODEL_DRIFT_DIFFUSION ? phys->nspecies : 2 + nd + phys->nspecies;
  r->mesh = mesh;
  r->ph = *phys;
  r->U0.assign(U0, U0 + (size_t)nvar * (size_t)nn);
  if (phys->model == VCX_MODEL_DRIFT_DIFFUSION) r->E.assign(E, E + (size_t)nd * (size_t)nn);
  r->nsteps = nsteps;
  r->t_end = t_end;
  r->bytes = bytes;
  r->t_submit = clk::now();
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) return set_err(VCX_E_BUSY, "server is shutting down");
    r->id = sv->next_id++;
    *id = r->id;
    sv->queue.push_back(r.get());
    sv->reqs.emplace(r->id, std::move(r));
    sv->submitted += 1;
    sv->events += 1;
  }
  sv->cv_work.notify_one();
  return VCX_OK;
}

extern "C" vcx_status vcx_server_poll(vcx_server sv, int64_t id, int* done, vcx_status* result, double* U_out,
                                      double* t_out) {
  if (!sv || !done) return set_err(VCX_E_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(id);
  if (it == sv->reqs.end()) return set_err(VCX_E_ARG, "unknown request id (or result already taken)");
  Request* r = it->second.get();
  *done = r->state == DONE;
  if (!*done) return VCX_OK;
  if (result) *result = r->status;
  if (t_out) *t_out = r->t;
  if (r->status != VCX_OK && !r->err.empty()) set_err(r->status, r->err);
  if (U_out) {
    if (!r->U.empty()) std::memcpy(U_out, r->U.data(), sizeof(double) * r->U.size());
    sv->reqs.erase(it);  // the result is handed over once
  }
  return VCX_OK;
}

extern "C" vcx_status vcx_server_wait(vcx_server sv, int64_t id, double timeout_s, int* done) {
  if (!sv || !done) return set_err(VCX_E_ARG, "NULL argument");
  std::unique_lock<std::mutex> lk(sv->mu);
  auto ready = [&] {
    auto it = sv->reqs.find(id);
    return it == sv->reqs.end() || it->second->state == DONE;
  };
  if (sv->reqs.find(id) == sv->reqs.end()) return set_err(VCX_E_ARG, "unknown request id (or result already taken)");
  if (timeout_s < 0)
    sv->cv_done.wait(lk, ready);
  else
    sv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready);
  *done = ready() ? 1 : 0;
  return VCX_OK;
}

extern "C" vcx_status vcx_server_stats(vcx_server sv, double* out) {
  if (!sv || !out) return set_err(VCX_E_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(sv->mu);
  out[0] = (double)sv->submitted;
  out[1] = (double)sv->completed;
  out[2] = (double)sv->failed;
  out[3] = (double)sv->queue.size();
  out[4] = (double)sv->running;
  out[5] = (double)sv->member_steps;
  out[6] = (double)sv->chunks;
  out[7] = sv->chunks ? (double)sv->member_chunks / (double)sv->chunks : 0.0;
  out[8] = pct(sv->lat_ms, 50.0);
  out[9] = pct(sv->lat_ms, 99.0);
  out[10] = pct(sv->step_ms, 50.0);
  out[11] = pct(sv->step_ms, 99.0);
  out[12] = (double)(sv->resident - sv->idle_bytes);
  out[13] = (double)sv->peak_resident;
  out[14] = (double)sv->peak_running;
  out[15] = (double)sv->worker_status;
  out[16] = (double)sv->idle_bytes;
  return VCX_OK;
}

extern "C" vcx_status vcx_server_destroy(vcx_server sv) {
  if (!sv) return set_err(VCX_E_ARG, "NULL server");
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
    sv->events += 1;
  }
  sv->cv_work.notify_all();
  sv->cv_io.notify_all();
  if (sv->worker.joinable()) sv->worker.join();
  if (sv->io.joinable()) sv->io.join();
  for (Idle& x : sv->idle) (void)vcx_solver_destroy(x.s);
  sv->idle.clear();
  (void)hipStreamSynchronize(sv->stream);
  (void)hipStreamDestroy(sv->stream);
  delete sv;
  return VCX_OK;
}
