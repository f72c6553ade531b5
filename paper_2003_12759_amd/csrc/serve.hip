// Continuous-batching server for shifted solves on resident systems.
//
// Requests (system, sigma, b) arrive at any time from any thread.  One
// scheduler thread owns the device work: between iteration segments it
// admits waiting requests into free column slots (by device-memory footprint),
// builds each new request's preconditioner, starts its recurrence, runs one
// segment of BiCG iterations on every system that has work (one stream per
// system, so systems overlap on the device), checks the true residuals of
// columns that stopped, and retires finished columns.
//
// Preconditioner of a request (Section III-B, Table 2 second approach, and
// Section III-C): every system keeps a chain of anchor factors built once,
// SPAI at the first anchor and the column-wise update between consecutive
// anchors (log-spaced shifts).  A request at sigma adds one update factor
// from its nearest anchor a_k: P_sigma = Q(a_k -> sigma) Q(a_{k-1} -> a_k) ...
// P(a_0), applied factor by factor and never formed.
#include <math.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <thread>
#include <unordered_map>
#include <vector>

#include "krylov.h"

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
  uint64_t ticket = 0;
  morx_system sys = nullptr;
  double sigma = 0.0;
  const double* b = nullptr;
  double* x = nullptr;
  double t_submit = 0.0, t_done = 0.0;
  int done = 0;
  morx_col_stats st{};
  int slot = -1;
  int anchor = 0;
  morx_factor q = nullptr;
  size_t q_bytes = 0;
  bool started = false;  // its recurrence has been launched
  std::vector<morx_factor_spec> chain;  // filled at admission (under the server lock)
};

struct SysServe {
  morx_system sys = nullptr;
  KrylovBatch kb;
  hipStream_t stream = nullptr;
  std::vector<morx_factor> anchors;  // P(a_0), Q(a_0 -> a_1), ...
  std::vector<double> anchor_sigma;
  std::vector<Request*> slot_req;
  size_t bytes = 0;
  uint64_t last_use = 0;  // admission counter at the system's last admitted request
};

size_t factor_bytes(morx_system sys, int prec) {
  return (size_t)(sys->sell.nnz_sell + sys->sellT.nnz_sell) * prec_bytes(prec);
}


}  // namespace

struct morx_server_s {
  morx_ctx ctx = nullptr;
  morx_opts opts{};
  morx_serve_config cfg{};
  std::atomic<size_t> used{0};
  std::thread th;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request*> incoming;
  std::deque<Request*> waiting;  // scheduler-owned
  std::unordered_map<uint64_t, Request*> table;
  std::vector<SysServe*> systems;
  uint64_t next_ticket = 1;
  uint64_t submitted = 0, completed = 0;
  std::atomic<int> running{0};
  bool stop = false;
  morx_status fatal = MORX_OK;
  morx_serve_counts counts{};  // under mu
};

namespace {

void finish(morx_server srv, Request* r, int status) {
  r->st.status = status;
  r->t_done = now_s();
  std::lock_guard<std::mutex> lk(srv->mu);
  r->done = 1;
  srv->completed += 1;
  srv->cv.notify_all();
}

SysServe* system_of(morx_server srv, morx_system sys) {
  for (SysServe* s : srv->systems)
    if (s->sys == sys) return s;
  return nullptr;
}

// anchors of a system: SPAI at the first, updates along the rest (one launch)
morx_status build_anchors(morx_server srv, SysServe* ss) {
  const int na = srv->cfg.anchors;
  const int prec = srv->opts.precond_prec;
  std::vector<FactorJob> jobs;
  for (int k = 0; k < na; ++k) {
    const double t = na == 1 ? 0.0 : (double)k / (na - 1);
    const double a = srv->cfg.anchor_min * pow(srv->cfg.anchor_max / srv->cfg.anchor_min, t);
    morx_factor f = nullptr;
    MORX_TRY(factor_alloc(ss->sys, prec, &f));
    ss->anchors.push_back(f);
    ss->anchor_sigma.push_back(a);
    FactorJob jb{a, k == 0 ? 0.0 : ss->anchor_sigma[k - 1], k == 0 ? 1 : 0, f->vals.p, f->valsT.p};
    f->is_spai = k == 0;
    f->sigma_prev = jb.sigma_prev;
    f->sigma_new = a;
    jobs.push_back(jb);
  }
  return factor_build_many(ss->sys, prec, jobs.data(), na, ss->stream);
}

size_t system_bytes(morx_server srv, morx_system sys) {
  return batch_bytes(sys, srv->cfg.slots_per_system, srv->opts.apply_prec) +
         (size_t)srv->cfg.anchors * factor_bytes(sys, srv->opts.precond_prec);
}

bool idle(const SysServe* ss) {
  for (const Request* r : ss->slot_req)
    if (r) return false;
  return true;
}

// release a resident system: its slot batch, anchors and stream
void evict(morx_server srv, SysServe* ss) {
  hipStreamSynchronize(ss->stream);
  for (morx_factor f : ss->anchors) factor_discard(f);
  // finished requests' factors wait in the system's pool for its next
  // requests: free them with the system
  std::vector<morx_factor>& pool = ss->sys->factor_pool;
  for (morx_factor f : pool) factor_discard(f);
  pool.clear();
  batch_free(ss->kb);
  hipStreamDestroy(ss->stream);
  srv->used -= ss->bytes;
  srv->systems.erase(std::find(srv->systems.begin(), srv->systems.end(), ss));
  delete ss;
  std::lock_guard<std::mutex> lk(srv->mu);
  srv->counts.systems_evicted += 1;
  srv->counts.resident = (int32_t)srv->systems.size();
}

// make room for `need` more bytes by releasing idle systems other than
// `keep`, least recently used first; whether the bytes fit afterwards
bool make_room(morx_server srv, size_t need, const SysServe* keep) {
  while (srv->used + need > srv->cfg.hbm_budget_bytes) {
    SysServe* lru = nullptr;
    for (SysServe* ss : srv->systems)
      if (ss != keep && idle(ss) && (!lru || ss->last_use < lru->last_use)) lru = ss;
    if (!lru) return false;
    evict(srv, lru);
  }
  return true;
}

morx_status make_system(morx_server srv, morx_system sys, SysServe** out) {
  *out = nullptr;
  const int slots = srv->cfg.slots_per_system;
  const size_t need = system_bytes(srv, sys);
  if (!make_room(srv, need, nullptr)) return MORX_E_ADMISSION;
  SysServe* ss = new SysServe();
  ss->sys = sys;
  if (hipStreamCreateWithFlags(&ss->stream, hipStreamNonBlocking) != hipSuccess) {
    delete ss;
    morx_set_error("serve: stream creation failed");
    return MORX_E_HIP;
  }
  morx_status s = batch_alloc(ss->kb, sys, slots, srv->cfg.anchors + 1, srv->opts.precond_prec,
                              srv->opts.apply_prec, ss->stream);
  if (s == MORX_OK) s = build_anchors(srv, ss);
  if (s != MORX_OK) {
    hipStreamSynchronize(ss->stream);
    for (morx_factor f : ss->anchors) factor_discard(f);
    batch_free(ss->kb);
    hipStreamDestroy(ss->stream);
    delete ss;
    return s;
  }
  ss->slot_req.assign(slots, nullptr);
  ss->bytes = need;
  srv->used += need;
  srv->systems.push_back(ss);
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->counts.systems_made += 1;
    srv->counts.resident = (int32_t)srv->systems.size();
  }
  *out = ss;
  return MORX_OK;
}

int nearest_anchor(const SysServe* ss, double sigma) {
  int best = 0;
  double bd = 1e300;
  for (size_t k = 0; k < ss->anchor_sigma.size(); ++k) {
    const double d = fabs(log(sigma) - log(ss->anchor_sigma[k]));
    if (d < bd) {
      bd = d;
      best = (int)k;
    }
  }
  return best;
}

// admit waiting requests that fit, build their factors, start their columns
morx_status admit(morx_server srv) {
  std::vector<std::pair<SysServe*, Request*>> fresh;
  for (auto it = srv->waiting.begin(); it != srv->waiting.end();) {
    Request* r = *it;
    SysServe* ss = system_of(srv, r->sys);
    if (!ss) {
      morx_status s = make_system(srv, r->sys, &ss);
      if (s == MORX_E_ADMISSION) {
        if (srv->running == 0 && fresh.empty()) {
          // nothing will free memory: this request can never run
          it = srv->waiting.erase(it);
          finish(srv, r, MORX_E_ADMISSION);
          continue;
        }
        ++it;
        continue;
      }
      MORX_TRY(s);
    }
    int slot = -1;
    for (int k = 0; k < (int)ss->slot_req.size(); ++k)
      if (!ss->slot_req[k]) {
        slot = k;
        break;
      }
    const size_t qb = factor_bytes(r->sys, srv->opts.precond_prec);
    if (slot < 0 || !make_room(srv, qb, ss)) {
      if (slot >= 0 && srv->running == 0 && fresh.empty()) {
        it = srv->waiting.erase(it);
        finish(srv, r, MORX_E_ADMISSION);
        continue;
      }
      ++it;
      continue;
    }
    // joins work already on the device when another slot of its system is
    // iterating
    bool joins = false;
    for (const Request* o : ss->slot_req) joins = joins || (o && o->started);
    ss->slot_req[slot] = r;
    r->slot = slot;
    r->q_bytes = qb;
    srv->used += qb;
    srv->running += 1;
    {
      std::lock_guard<std::mutex> lk(srv->mu);
      ss->last_use = ++srv->counts.admitted;
      if (joins) srv->counts.joined_running += 1;
      srv->counts.max_running = std::max<int32_t>(srv->counts.max_running, srv->running);
    }
    fresh.push_back({ss, r});
    it = srv->waiting.erase(it);
  }
  // factors of the admitted requests, one launch per system
  for (SysServe* ss : srv->systems) {
    std::vector<FactorJob> jobs;
    std::vector<Request*> reqs;
    for (auto& p : fresh)
      if (p.first == ss) {
        Request* r = p.second;
        MORX_TRY(factor_alloc(ss->sys, srv->opts.precond_prec, &r->q));
        r->anchor = nearest_anchor(ss, r->sigma);
        r->q->is_spai = false;
        r->q->sigma_prev = ss->anchor_sigma[r->anchor];
        r->q->sigma_new = r->sigma;
        jobs.push_back({r->sigma, ss->anchor_sigma[r->anchor], 0, r->q->vals.p, r->q->valsT.p});
        reqs.push_back(r);
        std::vector<morx_factor_spec> ch;
        for (int k = 0; k <= r->anchor; ++k) {
          const morx_factor f = ss->anchors[k];
          ch.push_back({f->is_spai ? 1 : 0, 0, f->is_spai ? 0.0 : f->sigma_prev, f->sigma_new});
        }
        ch.push_back({0, 0, r->q->sigma_prev, r->q->sigma_new});
        std::lock_guard<std::mutex> lk(srv->mu);
        r->chain = std::move(ch);
      }
    if (jobs.empty()) continue;
    MORX_TRY(factor_build_many(ss->sys, srv->opts.precond_prec, jobs.data(), (int)jobs.size(),
                               ss->stream));
    KrylovBatch& b = ss->kb;
    const int maxit = srv->opts.maxit > 0 ? srv->opts.maxit
                                          : (int)std::min<int64_t>(ss->sys->n, 20000);
    for (Request* r : reqs) {
      ColInfo ci = {};
      ci.sigma = r->sigma;
      ci.tol = srv->opts.tol;
      ci.bsrc = r->b;
      ci.csrc = r->b;  // primal only: the shadow right-hand side is b
      ci.xout = r->x;
      ci.yout = nullptr;
      ci.state = COL_INIT;
      ci.L = r->anchor + 2;
      ci.first = 1;
      ci.max_restarts = srv->opts.max_restarts;
      ci.maxit = maxit;
      ci.check_p = 1;
      ci.check_d = 0;
      ci.out_x = 1;
      ci.out_y = 0;
      ci.status = MORX_E_NOT_CONVERGED;
      b.hcols[r->slot] = ci;
      for (int s = 0; s < b.lcap; ++s) {
        morx_factor f = s <= r->anchor ? ss->anchors[s] : (s == r->anchor + 1 ? r->q : nullptr);
        b.hftab[(size_t)r->slot * b.lcap + s] = f ? f->vals.p : nullptr;
        b.hftab[((size_t)b.cap + r->slot) * b.lcap + s] = f ? f->valsT.p : nullptr;
      }
      MORX_TRY(batch_upload(b, r->slot, 1, ss->stream));
    }
    MORX_TRY(batch_launch_init(b, b.cap, ss->stream));
    for (Request* r : reqs) r->started = true;
  }
  return MORX_OK;
}

// one segment on every busy system, then true residuals and retirements
morx_status step(morx_server srv) {
  int seg = std::max(2, srv->cfg.segment_iters);
  seg += seg & 1;
  std::vector<SysServe*> busy;
  for (SysServe* ss : srv->systems) {
    int maxL = 0;
    for (Request* r : ss->slot_req)
      if (r) maxL = std::max(maxL, r->anchor + 2);
    if (maxL == 0) continue;
    busy.push_back(ss);
    {
      std::lock_guard<std::mutex> lk(srv->mu);
      srv->counts.segments += 1;
    }
    MORX_TRY(batch_launch_segment(ss->kb, ss->kb.cap, maxL, seg, srv->opts.use_graph != 0,
                                  ss->stream, nullptr));
  }
  for (SysServe* ss : busy) {
    KrylovBatch& b = ss->kb;
    MORX_TRY(batch_download(b, ss->stream));
    bool stopped = false;
    for (int c = 0; c < b.cap; ++c) {
      const int st = b.hcols[c].state;
      if (st == COL_CONVERGED || st == COL_BREAKDOWN || st == COL_MAXIT) stopped = true;
    }
    if (stopped) {
      MORX_TRY(batch_launch_true(b, b.cap, ss->stream));
      MORX_TRY(batch_download(b, ss->stream));
    }
    std::vector<int> fin;
    for (int c = 0; c < b.cap; ++c) {
      const int st = b.hcols[c].state;
      if (ss->slot_req[c] && (st == COL_DONE || st == COL_FAILED)) fin.push_back(c);
    }
    if (fin.empty()) continue;
    MORX_TRY(batch_launch_copy_out(b, fin.data(), (int)fin.size(), ss->stream));
    MORX_HIP(hipStreamSynchronize(ss->stream));
    for (int c : fin) {
      Request* r = ss->slot_req[c];
      const ColInfo& ci = b.hcols[c];
      r->st.iters = ci.iters;
      r->st.restarts = ci.restarts;
      r->st.relres_primal = ci.relp;
      r->st.relres_dual = 0.0;
      const int status = ci.state == COL_DONE ? MORX_OK : ci.status;
      b.hcols[c].state = COL_IDLE;
      MORX_TRY(batch_upload(b, c, 1, ss->stream));
      factor_release(r->q);
      r->q = nullptr;
      srv->used -= r->q_bytes;
      srv->running -= 1;
      ss->slot_req[c] = nullptr;
      finish(srv, r, status);
    }
  }
  return MORX_OK;
}

void scheduler(morx_server srv) {
  hipSetDevice(srv->ctx->device);
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(srv->mu);
      srv->cv.wait(lk, [&] {
        return srv->stop || !srv->incoming.empty() || srv->running > 0 || !srv->waiting.empty();
      });
      while (!srv->incoming.empty()) {
        srv->waiting.push_back(srv->incoming.front());
        srv->incoming.pop_front();
      }
      if (srv->stop && srv->waiting.empty() && srv->running == 0) break;
    }
    morx_status s;
    {
      std::lock_guard<std::mutex> glk(srv->ctx->mu);
      s = admit(srv);
      if (s == MORX_OK) s = step(srv);
    }
    if (s != MORX_OK) {
      // a device failure ends the server: fail everything still pending
      std::vector<Request*> pend(srv->waiting.begin(), srv->waiting.end());
      srv->waiting.clear();
      for (SysServe* ss : srv->systems)
        for (Request*& r : ss->slot_req)
          if (r) {
            pend.push_back(r);
            r = nullptr;
          }
      {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->fatal = s;
        srv->running = 0;
        for (Request* r : srv->incoming) pend.push_back(r);
        srv->incoming.clear();
      }
      for (Request* r : pend) finish(srv, r, s);
      std::unique_lock<std::mutex> lk(srv->mu);
      srv->cv.wait(lk, [&] { return srv->stop; });
      break;
    }
  }
}

}  // namespace

extern "C" void morx_serve_config_default(morx_serve_config* c) {
  if (!c) return;
  c->hbm_budget_bytes = (size_t)16 << 30;
  c->slots_per_system = 8;
  c->anchors = 8;
  c->anchor_min = 1.0;
  c->anchor_max = 1e3;
  c->segment_iters = 8;
  c->reserved = 0;
}

extern "C" morx_status morx_serve_start(morx_ctx ctx, const morx_serve_config* cfg,
                                        const morx_opts* opts, morx_server* out) {
  MORX_REQUIRE(ctx && out, MORX_E_INVALID, "morx_serve_start: null argument");
  morx_server srv = new morx_server_s();
  srv->ctx = ctx;
  if (cfg) srv->cfg = *cfg;
  else morx_serve_config_default(&srv->cfg);
  if (opts) srv->opts = *opts;
  else morx_opts_default(&srv->opts);
  srv->opts.want_dual = 0;
  const morx_serve_config& c = srv->cfg;
  if (!(c.slots_per_system >= 1 && c.slots_per_system <= 64 && c.anchors >= 1 && c.anchors <= 31 &&
        c.anchor_min > 0.0 && c.anchor_max >= c.anchor_min && std::isfinite(c.anchor_max) &&
        srv->opts.precond_prec >= MORX_F64 && srv->opts.precond_prec <= MORX_BF16 &&
        (srv->opts.apply_prec == MORX_F64 || srv->opts.apply_prec == MORX_F32))) {
    delete srv;
    morx_set_error("morx_serve_start: bad configuration");
    return MORX_E_INVALID;
  }
  srv->th = std::thread(scheduler, srv);
  *out = srv;
  return MORX_OK;
}

extern "C" morx_status morx_serve_submit(morx_server srv, morx_system sys, double sigma,
                                         const double* b, double* x, uint64_t* ticket) {
  MORX_REQUIRE(srv && sys && b && x && ticket, MORX_E_INVALID, "morx_serve_submit: null argument");
  MORX_REQUIRE(sys->ctx == srv->ctx, MORX_E_INVALID, "morx_serve_submit: system of another context");
  MORX_REQUIRE(std::isfinite(sigma) && sigma > 0.0, MORX_E_INVALID,
               "morx_serve_submit: the shift must be finite and positive");
  MORX_REQUIRE(sys->ls_supported, MORX_E_UNSUPPORTED, "morx_serve_submit: pattern not supported");
  Request* r = new Request();
  r->sys = sys;
  r->sigma = sigma;
  r->b = b;
  r->x = x;
  r->t_submit = now_s();
  std::lock_guard<std::mutex> lk(srv->mu);
  if (srv->stop || srv->fatal != MORX_OK) {
    delete r;
    morx_set_error("morx_serve_submit: server stopped");
    return srv->fatal != MORX_OK ? srv->fatal : MORX_E_INVALID;
  }
  r->ticket = srv->next_ticket++;
  srv->table[r->ticket] = r;
  srv->incoming.push_back(r);
  srv->submitted += 1;
  *ticket = r->ticket;
  srv->cv.notify_all();
  return MORX_OK;
}

static morx_status take(morx_server srv, uint64_t ticket, bool wait, morx_col_stats* st,
                        double* latency_s) {
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->table.find(ticket);
  MORX_REQUIRE(it != srv->table.end(), MORX_E_INVALID, "serve: unknown ticket %llu",
               (unsigned long long)ticket);
  Request* r = it->second;
  if (wait) srv->cv.wait(lk, [&] { return r->done != 0; });
  if (!r->done) return MORX_E_PENDING;
  if (st) *st = r->st;
  if (latency_s) *latency_s = r->t_done - r->t_submit;
  const int status = r->st.status;
  srv->table.erase(it);
  delete r;
  return (morx_status)status;
}

extern "C" morx_status morx_serve_poll(morx_server srv, uint64_t ticket, morx_col_stats* st,
                                       double* latency_s) {
  MORX_REQUIRE(srv, MORX_E_INVALID, "morx_serve_poll: null server");
  return take(srv, ticket, false, st, latency_s);
}

extern "C" morx_status morx_serve_wait(morx_server srv, uint64_t ticket, morx_col_stats* st,
                                       double* latency_s) {
  MORX_REQUIRE(srv, MORX_E_INVALID, "morx_serve_wait: null server");
  return take(srv, ticket, true, st, latency_s);
}

extern "C" morx_status morx_serve_info(morx_server srv, uint64_t* submitted, uint64_t* completed,
                                       int32_t* running, int32_t* queued, int64_t* bytes_in_use) {
  MORX_REQUIRE(srv, MORX_E_INVALID, "morx_serve_info: null server");
  std::lock_guard<std::mutex> lk(srv->mu);
  if (submitted) *submitted = srv->submitted;
  if (completed) *completed = srv->completed;
  if (running) *running = srv->running;
  if (queued) *queued = (int32_t)(srv->incoming.size() + srv->waiting.size());
  if (bytes_in_use) *bytes_in_use = (int64_t)srv->used.load();
  return MORX_OK;
}

extern "C" morx_status morx_serve_footprint(const morx_serve_config* cfg, const morx_opts* opts,
                                            morx_system sys, size_t* system_bytes,
                                            size_t* request_bytes) {
  MORX_REQUIRE(sys && system_bytes && request_bytes, MORX_E_INVALID,
               "morx_serve_footprint: null argument");
  morx_serve_config c;
  morx_opts o;
  if (cfg) c = *cfg;
  else morx_serve_config_default(&c);
  if (opts) o = *opts;
  else morx_opts_default(&o);
  MORX_REQUIRE(c.slots_per_system >= 1 && c.anchors >= 1 && o.precond_prec >= MORX_F64 &&
                   o.precond_prec <= MORX_BF16 && (o.apply_prec == MORX_F64 || o.apply_prec == MORX_F32),
               MORX_E_INVALID, "morx_serve_footprint: bad configuration");
  *system_bytes = batch_bytes(sys, c.slots_per_system, o.apply_prec) +
                  (size_t)c.anchors * factor_bytes(sys, o.precond_prec);
  *request_bytes = factor_bytes(sys, o.precond_prec);
  return MORX_OK;
}

extern "C" morx_status morx_serve_counts_get(morx_server srv, morx_serve_counts* out) {
  MORX_REQUIRE(srv && out, MORX_E_INVALID, "morx_serve_counts_get: null argument");
  std::lock_guard<std::mutex> lk(srv->mu);
  *out = srv->counts;
  return MORX_OK;
}

extern "C" morx_status morx_serve_chain(morx_server srv, uint64_t ticket, int32_t cap, int32_t* len,
                                        morx_factor_spec* specs) {
  MORX_REQUIRE(srv && len && cap >= 0 && (cap == 0 || specs), MORX_E_INVALID,
               "morx_serve_chain: bad argument");
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->table.find(ticket);
  MORX_REQUIRE(it != srv->table.end(), MORX_E_INVALID, "serve: unknown ticket %llu",
               (unsigned long long)ticket);
  const Request* r = it->second;
  if (r->chain.empty()) return MORX_E_PENDING;
  *len = (int32_t)r->chain.size();
  for (int k = 0; k < cap && k < (int)r->chain.size(); ++k) specs[k] = r->chain[k];
  return MORX_OK;
}

extern "C" morx_status morx_serve_stop(morx_server srv) {
  if (!srv) return MORX_OK;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
    srv->cv.notify_all();
  }
  if (srv->th.joinable()) srv->th.join();
  {
    std::lock_guard<std::mutex> glk(srv->ctx->mu);
    hipSetDevice(srv->ctx->device);
    for (SysServe* ss : srv->systems) {
      hipStreamSynchronize(ss->stream);
      for (morx_factor f : ss->anchors) factor_discard(f);
      batch_free(ss->kb);
      hipStreamDestroy(ss->stream);
      delete ss;
    }
  }
  for (auto& kv : srv->table) delete kv.second;
  const morx_status fatal = srv->fatal;
  delete srv;
  return fatal;
}
