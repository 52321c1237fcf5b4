// Serving: many solve requests for several gauge fields (different lattice
// sizes, masses and precisions) on one GPU, with continuous batching.
//
// Each registered field is a hierarchy (the bootstrap setup of Sec. 3.4) plus
// a slot engine (engine.cpp) on a stream of its own.  A field becomes
// resident when a request for it arrives and its device footprint (hierarchy
// + slots) fits in the memory budget next to the resident fields; idle
// resident fields are evicted, least recently used first, when the memory is
// needed.  Right-hand sides of queued requests take free slots of their
// field's engine at the start of every round, so requests that arrive while
// others are in flight join the running batch.  A round issues the work of
// every busy engine before waiting on any of them, so the kernels of
// different fields overlap on the device while the host does the Givens
// algebra of another.  A right-hand side's arithmetic does not depend on the
// other slots (engine.cpp), so every result equals the one obtained alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "hierarchy.h"

using namespace bamg;

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

struct Request {
  int64_t id = 0;
  int field = 0;
  const zd* B = nullptr;
  zd* X = nullptr;
  int nrhs = 0;
  double tol = 0;
  int done = 0;       // right-hand sides finished
  int status = BAMG_OK;
  bool finished = false;
  std::vector<bamg_solve_info> infos;
  Clock::time_point t_submit, t_done;
};

struct Field {
  int id = 0;
  std::vector<zd> gauge_host;  // U[mu][y][x], kept for re-setup after eviction
  double m = 0;
  bamg_params p{};
  size_t bytes = 0;  // device footprint when resident
  hipStream_t s = nullptr;
  bamg_hierarchy* h = nullptr;
  SlotEngine* e = nullptr;
  std::deque<std::pair<int64_t, int>> queue;  // (request, right-hand side) waiting for a slot
  Clock::time_point last_used;
  bool resident() const { return h != nullptr; }
};

}  // namespace

struct bamg_server {
  bamg_server_params sp{};
  size_t budget = 0, used = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::vector<std::unique_ptr<Field>> fields;  // a Field never moves (the worker holds references)
  std::map<int64_t, Request> reqs;
  int64_t next_id = 1;
  bool stop = false;
  std::thread worker;
  // statistics
  int64_t submitted = 0, completed = 0, rhs_completed = 0, rounds = 0;
  int evictions = 0, setups = 0;
  std::vector<double> latencies;
  bool any_submit = false;
  Clock::time_point t_first_submit, t_last_done;
  std::string worker_error;

  bool has_work_locked() const {
    for (const auto& f : fields)
      if (!f->queue.empty() || (f->e && engine_busy(f->e) > 0)) return true;
    return false;
  }

  void evict(Field& f) {
    engine_destroy(f.e);
    bamg_free(f.h);
    f.e = nullptr;
    f.h = nullptr;
    used -= f.bytes;
    ++evictions;
  }

  // fail every queued right-hand side of field f with `status` (lock held)
  void fail_queue_locked(Field& f, int status) {
    while (!f.queue.empty()) {
      const auto q = f.queue.front();
      f.queue.pop_front();
      auto it = reqs.find(q.first);
      if (it == reqs.end()) continue;
      Request& r = it->second;
      r.status = status;
      complete_rhs_locked(r, q.second, nullptr, status);
    }
  }

  void complete_rhs_locked(Request& r, int k, const bamg_solve_info* info, int status) {
    if (info) r.infos[k] = *info;
    if (status == BAMG_EDEVICE || status == BAMG_EINVAL || status == BAMG_ENOMEM || status == BAMG_ESINGULAR)
      r.status = status;
    else if (status == BAMG_NOT_CONVERGED && r.status == BAMG_OK)
      r.status = status;
    if (++r.done == r.nrhs) {
      r.finished = true;
      r.t_done = Clock::now();
      ++completed;
      rhs_completed += r.nrhs;
      latencies.push_back(ms_between(r.t_submit, r.t_done));
      t_last_done = r.t_done;
      cv_done.notify_all();
    }
  }

  // make field f resident if its footprint fits (evicting idle fields); lock held
  // only for the bookkeeping, not during the setup
  bool admit_field(Field& f, std::unique_lock<std::mutex>& lk) {
    if (f.resident()) return true;
    if (f.bytes > budget) {
      fail_queue_locked(f, BAMG_ENOMEM);
      return false;
    }
    while (used + f.bytes > budget) {
      Field* lru = nullptr;
      for (auto& gp : fields) {
        Field& g = *gp;
        if (g.resident() && engine_busy(g.e) == 0 && g.queue.empty() && (!lru || g.last_used < lru->last_used))
          lru = &g;
      }
      if (!lru) return false;  // everything resident is busy: wait for a later round
      evict(*lru);
    }
    used += f.bytes;
    const std::vector<zd>& gh = f.gauge_host;
    bamg_params p = f.p;
    p.stream = f.s;
    lk.unlock();
    int st = BAMG_OK;
    bamg_hierarchy* h = nullptr;
    SlotEngine* e = nullptr;
    zd* gdev = nullptr;
    try {
      gdev = dalloc<zd>(gh.size());
      HIPCHK(hipMemcpyAsync(gdev, gh.data(), gh.size() * sizeof(zd), hipMemcpyHostToDevice, f.s));
      st = bamg_setup(gdev, f.m, &p, &h);
      if (st == BAMG_OK) e = engine_create(h, sp.slots_per_field);
    } catch (const HipFail&) {
      st = BAMG_ENOMEM;
    }
    dfree(gdev);
    lk.lock();
    if (st != BAMG_OK || !e) {
      if (h) bamg_free(h);
      used -= f.bytes;
      fail_queue_locked(f, st == BAMG_OK ? BAMG_ENOMEM : st);
      return false;
    }
    f.h = h;
    f.e = e;
    ++setups;
    return true;
  }

  // one scheduling round over all fields (worker thread or bamg_server_progress)
  void round() {
    std::unique_lock<std::mutex> lk(mu);
    // admission: queued right-hand sides into free slots (fields may be added
    // by other threads while the lock is released for a setup: index loop)
    for (size_t fi = 0; fi < fields.size(); ++fi) {
      Field& f = *fields[fi];
      if (f.queue.empty()) continue;
      if (!admit_field(f, lk)) continue;
      while (!f.queue.empty() && engine_free_slots(f.e) > 0) {
        const auto q = f.queue.front();
        f.queue.pop_front();
        auto it = reqs.find(q.first);
        if (it == reqs.end()) continue;
        Request& r = it->second;
        const size_t n2 = (size_t)2 * f.p.N * f.p.N;
        engine_admit(f.e, r.B + (size_t)q.second * n2, r.X + (size_t)q.second * n2, r.tol,
                     ((uint64_t)q.first << 16) | (uint64_t)q.second);
      }
      f.last_used = Clock::now();
    }
    std::vector<Field*> busy;
    for (auto& f : fields)
      if (f->e && engine_busy(f->e) > 0) busy.push_back(f.get());
    lk.unlock();
    if (busy.empty()) return;
    std::vector<std::vector<SlotDone>> done(busy.size());
    std::vector<int> failed(busy.size(), 0);
    std::vector<std::string> why(busy.size());
    // every phase is issued for all fields before any is waited on
    auto each = [&](auto&& fn) {
      for (size_t i = 0; i < busy.size(); ++i) {
        if (failed[i]) continue;
        try {
          fn(i);
        } catch (const HipFail& e) {
          failed[i] = 1;
          why[i] = e.msg;
        }
      }
    };
    each([&](size_t i) { engine_issue_pre(busy[i]->e); });
    each([&](size_t i) {
      engine_finish_pre(busy[i]->e);
      engine_issue_main(busy[i]->e);
    });
    each([&](size_t i) { engine_finish_main(busy[i]->e, done[i]); });
    lk.lock();
    ++rounds;
    for (size_t i = 0; i < busy.size(); ++i) {
      for (const SlotDone& d : done[i]) {
        auto it = reqs.find((int64_t)(d.tag >> 16));
        if (it != reqs.end()) complete_rhs_locked(it->second, (int)(d.tag & 0xffff), &d.info, d.status);
      }
      if (failed[i]) {
        // a device error on this field: drop its hierarchy and fail what it held
        worker_error = why[i];
        Field& f = *busy[i];
        for (auto& kv : reqs) {
          Request& r = kv.second;
          if (r.field == f.id && !r.finished) {
            r.status = BAMG_EDEVICE;
            while (!r.finished) complete_rhs_locked(r, r.done, nullptr, BAMG_EDEVICE);
          }
        }
        f.queue.clear();
        (void)hipStreamSynchronize(f.s);
        evict(f);
      }
    }
  }

  void run() {
    while (true) {
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait(lk, [&] { return stop || has_work_locked(); });
        if (stop) return;
      }
      round();
    }
  }
};

extern "C" {

int bamg_server_default_params(bamg_server_params* sp) {
  if (!sp) return api_fail(BAMG_EINVAL, "params is NULL");
  sp->hbm_budget = 0;
  sp->slots_per_field = 32;
  sp->threaded = 1;
  return BAMG_OK;
}

int bamg_server_create(const bamg_server_params* sp, bamg_server** out) {
  if (!sp || !out) return api_fail(BAMG_EINVAL, "bad arguments");
  *out = nullptr;
  if (sp->slots_per_field < 1 || sp->slots_per_field > 4096)
    return api_fail(BAMG_EINVAL, "slots_per_field must be in [1, 4096]");
  bamg_server* s = new bamg_server();
  s->sp = *sp;
  s->budget = sp->hbm_budget;
  if (s->budget == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      delete s;
      return api_fail(BAMG_EDEVICE, "hipMemGetInfo failed");
    }
    s->budget = fr / 10 * 8;
  }
  if (sp->threaded) s->worker = std::thread([s] { s->run(); });
  *out = s;
  return BAMG_OK;
}

int bamg_server_add_field(bamg_server* s, const void* gauge, double m, const bamg_params* p, int32_t* field_id) {
  if (!s || !gauge || !p || !field_id) return api_fail(BAMG_EINVAL, "bad arguments");
  const size_t fp = bamg_footprint_bytes(p);
  if (fp == 0) return api_fail(BAMG_EINVAL, "invalid hierarchy parameters");
  if (!std::isfinite(m) || m + 2.0 == 0.0) return api_fail(BAMG_EINVAL, "mass gives c = m + 2 = 0 or non-finite");
  auto fp_ = std::make_unique<Field>();
  Field& f = *fp_;
  f.m = m;
  f.p = *p;
  f.p.init_tv_host = nullptr;
  f.p.stream = nullptr;
  const size_t nl = (size_t)2 * p->N * p->N;
  f.gauge_host.resize(nl);
  if (hipMemcpy(f.gauge_host.data(), gauge, nl * sizeof(zd), hipMemcpyDeviceToHost) != hipSuccess)
    return api_fail(BAMG_EDEVICE, "gauge copy failed");
  f.bytes = fp + hierarchy_slot_extra_bytes(p, s->sp.slots_per_field) +
            engine_slot_bytes((size_t)p->N * p->N, p->restart, s->sp.slots_per_field);
  if (hipStreamCreate(&f.s) != hipSuccess) return api_fail(BAMG_EDEVICE, "hipStreamCreate failed");
  std::lock_guard<std::mutex> lk(s->mu);
  f.id = (int)s->fields.size();
  f.last_used = Clock::now();
  *field_id = f.id;
  s->fields.push_back(std::move(fp_));
  return BAMG_OK;
}

int bamg_server_field_bytes(bamg_server* s, int32_t field_id, size_t* bytes) {
  if (!s || !bytes) return api_fail(BAMG_EINVAL, "bad arguments");
  std::lock_guard<std::mutex> lk(s->mu);
  if (field_id < 0 || field_id >= (int)s->fields.size()) return api_fail(BAMG_EINVAL, "unknown field");
  *bytes = s->fields[field_id]->bytes;
  return BAMG_OK;
}

int bamg_server_submit(bamg_server* s, int32_t field_id, const void* B, void* X, int32_t nrhs, double tol,
                       int64_t* request_id) {
  if (!s || !B || !X || !request_id || nrhs < 1) return api_fail(BAMG_EINVAL, "bad arguments");
  if (nrhs > 4096) return api_fail(BAMG_EINVAL, "nrhs > 4096");
  if (!(tol > 0)) return api_fail(BAMG_EINVAL, "tol must be > 0");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (field_id < 0 || field_id >= (int)s->fields.size()) return api_fail(BAMG_EINVAL, "unknown field");
    Request r;
    r.id = s->next_id++;
    r.field = field_id;
    r.B = (const zd*)B;
    r.X = (zd*)X;
    r.nrhs = nrhs;
    r.tol = tol;
    r.infos.assign(nrhs, bamg_solve_info{});
    r.t_submit = Clock::now();
    if (!s->any_submit) {
      s->any_submit = true;
      s->t_first_submit = r.t_submit;
    }
    ++s->submitted;
    Field& f = *s->fields[field_id];
    for (int k = 0; k < nrhs; ++k) f.queue.push_back({r.id, k});
    *request_id = r.id;
    s->reqs.emplace(r.id, std::move(r));
  }
  s->cv_work.notify_one();
  return BAMG_OK;
}

int bamg_server_progress(bamg_server* s, int32_t* pending) {
  if (!s) return api_fail(BAMG_EINVAL, "server is NULL");
  if (s->sp.threaded) return api_fail(BAMG_EINVAL, "the server runs its own worker thread");
  s->round();
  if (pending) {
    std::lock_guard<std::mutex> lk(s->mu);
    int32_t c = 0;
    for (const auto& kv : s->reqs)
      if (!kv.second.finished) ++c;
    *pending = c;
  }
  return BAMG_OK;
}

int bamg_server_wait(bamg_server* s, int64_t request_id, double timeout_ms, bamg_solve_info* infos) {
  if (!s) return api_fail(BAMG_EINVAL, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(request_id);
  if (it == s->reqs.end()) return api_fail(BAMG_EINVAL, "unknown request");
  if (!it->second.finished) {
    if (!s->sp.threaded) return BAMG_PENDING;
    auto pred = [&] { return it->second.finished; };
    if (timeout_ms < 0) s->cv_done.wait(lk, pred);
    else if (!s->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), pred)) return BAMG_PENDING;
  }
  Request& r = it->second;
  if (infos) std::copy(r.infos.begin(), r.infos.end(), infos);
  const int st = r.status;
  s->reqs.erase(it);
  if (st < 0) return api_fail(st, "request failed");
  return st;
}

int bamg_server_get_stats(bamg_server* s, bamg_server_stats* out) {
  if (!s || !out) return api_fail(BAMG_EINVAL, "bad arguments");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = bamg_server_stats{};
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->rhs_completed = s->rhs_completed;
  std::vector<double> l = s->latencies;
  std::sort(l.begin(), l.end());
  if (!l.empty()) {
    auto pct = [&](double q) {  // nearest-rank percentile
      size_t k = (size_t)std::ceil(q * l.size());
      if (k < 1) k = 1;
      return l[k - 1];
    };
    out->p50_ms = pct(0.50);
    out->p99_ms = pct(0.99);
    double sum = 0;
    for (double v : l) sum += v;
    out->mean_ms = sum / l.size();
    out->max_ms = l.back();
  }
  if (s->completed > 0) {
    out->busy_s = ms_between(s->t_first_submit, s->t_last_done) * 1e-3;
    out->solves_per_s = out->busy_s > 0 ? s->rhs_completed / out->busy_s : 0.0;
  }
  int res = 0;
  for (const auto& f : s->fields) res += f->resident() ? 1 : 0;
  out->resident_fields = res;
  out->evictions = s->evictions;
  out->setups = s->setups;
  out->bytes_in_use = s->used;
  out->budget_bytes = s->budget;
  out->rounds = s->rounds;
  return BAMG_OK;
}

int bamg_server_reset_stats(bamg_server* s) {
  if (!s) return api_fail(BAMG_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  s->submitted = s->completed = s->rhs_completed = s->rounds = 0;
  s->evictions = s->setups = 0;
  s->latencies.clear();
  s->any_submit = false;
  for (const auto& kv : s->reqs)
    if (!kv.second.finished) ++s->submitted;  // still in flight: counted as submitted from now on
  return BAMG_OK;
}

void bamg_server_free(bamg_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (auto& fp : s->fields) {
    Field& f = *fp;
    if (f.s) (void)hipStreamSynchronize(f.s);
    if (f.e) engine_destroy(f.e);
    if (f.h) bamg_free(f.h);
    if (f.s) (void)hipStreamDestroy(f.s);
  }
  delete s;
}

}  // extern "C"
