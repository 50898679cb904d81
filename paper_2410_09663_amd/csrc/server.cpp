// Serving loop for many independent controllers (continuous admission).
//
// Each controller is a liboic handle with its own stream, device-resident ensemble
// buffers, captured solve graph and applied-control state U_prev.  Requests (one MPC
// solve each: X_k, the reference window and a seed) enter a FIFO queue.  A pool of
// worker threads takes the oldest request whose controller is idle; if the
// controller's buffers are not resident it is admitted only when its HBM footprint
// fits the budget, evicting least-recently-used idle controllers (their U_prev is
// kept on the host) when needed.  Solves of different controllers run concurrently
// on their own streams, so requests that arrive while others are on the GPU start as
// soon as a worker slot and memory are free, and their kernels overlap on the device.
// Solves of one controller run in submission order (U_prev carries over).  Every
// solve reads only its own controller's buffers, so its result is the same alone and
// in any mix.
#include <hip/hip_runtime.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "oic_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Controller {
  oic_config cfg{};
  int N = 0, H = 0;
  std::vector<float> B, Q, R;
  std::vector<std::vector<float>> W, bias;
  std::vector<float> u_prev;  // host copy while evicted
  oic_handle h = nullptr;     // non-null while resident
  size_t footprint = 0;
  bool busy = false;
  long long last_used = 0;
};

struct Request {
  long long ticket = 0;
  int controller = 0;
  std::vector<float> X0, ref;
  uint64_t seed = 0;
  Clock::time_point submitted;
  int bypassed = 0;  // later requests started while this one waited for memory
};

// A request that waits for memory while later requests start is passed over at most
// this many times; after that no later request starts ahead of it, so the solves in
// flight finish, their controllers become idle and evictable, and it is admitted.  This
// bounds the wait of a large controller behind a stream of small ones.
constexpr int kMaxBypass = 8;

struct Result {
  bool done = false;
  int rc = OIC_OK;
  std::string err;
  std::vector<float> U, X;
  double latency_ms = 0.0, queue_ms = 0.0;
};

}  // namespace

struct oic_server {
  size_t budget = 0, used = 0;
  std::vector<std::unique_ptr<Controller>> ctrls;
  std::deque<Request> queue;
  std::map<long long, Result> results;
  long long next_ticket = 1, tick = 0;
  long long completed = 0, evictions = 0, admissions = 0, recycled = 0;
  size_t peak_used = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  std::vector<std::thread> workers;
  std::string err;
};

namespace {

// Device bytes oic_create allocates for cfg (mirrors its buffer list, rounded up).
size_t footprint_bytes(const oic_config& c) { return oic::handle_bytes(c); }

// Whether c's buffers are resident or can be, after evicting idle resident controllers.
bool can_admit(const oic_server* s, const Controller& c) {
  if (c.h) return true;
  size_t reclaimable = 0;
  for (auto& o : s->ctrls)
    if (o->h && !o->busy && o.get() != &c) reclaimable += o->footprint;
  return s->used - reclaimable + c.footprint <= s->budget;
}

// Whether handles created from a and b have the same buffers and captured solve: same
// grid, control rows, layer widths, activation, precision and (N, H).
bool same_shape(const oic_config& a, const oic_config& b) {
  if (a.n != b.n || a.m != b.m || a.l != b.l || a.n_layers != b.n_layers || a.activation != b.activation ||
      a.precision != b.precision || a.max_N != b.max_N || a.max_H != b.max_H || a.mem_mode != b.mem_mode)
    return false;
  for (int k = 0; k <= a.n_layers; ++k)
    if (a.channels[k] != b.channels[k]) return false;
  return true;
}

// Loads c's surrogate and applied control into a handle (a new one, or one taken over
// from an evicted controller of the same shape).
int load_controller(oic_handle h, const Controller& c) {
  std::vector<const float*> wp, bp;
  for (auto& w : c.W) wp.push_back(w.data());
  for (auto& b : c.bias) bp.push_back(b.empty() ? nullptr : b.data());
  int rc = oic_set_weights(h, c.B.data(), wp.data(), bp.data());
  if (rc != OIC_OK) return rc;
  if (!c.u_prev.empty()) return oic_set_u_prev(h, c.u_prev.data());
  const std::vector<float> zero((size_t)c.cfg.l * c.cfg.m, 0.f);  // a first admission
  return oic_set_u_prev(h, zero.data());
}

// Called with the lock held, right after the scheduling decision (same lock hold, so
// the budget check and the reservation are atomic).  If c does not fit beside the
// resident controllers and an idle one has c's shape, c takes over its handle: the evicted controller's U_prev is saved, c's
// weights and U_prev are copied into the same buffers, and the handle's captured solve
// stays valid (no device allocation, no free, no new capture).  Otherwise chooses the LRU
// idle victims, takes them and c's footprint out of the budget at once, then releases
// the lock for the slow part (saving the victims' U_prev, freeing them, creating c's
// handle).
int make_resident(oic_server* s, Controller& c, std::unique_lock<std::mutex>& lk) {
  if (c.h) return OIC_OK;
  Controller* donor = nullptr;
  if (s->used + c.footprint > s->budget)  // someone has to go: prefer a controller of c's shape
    for (auto& o : s->ctrls)
      if (o->h && !o->busy && o.get() != &c && same_shape(o->cfg, c.cfg) &&
          (!donor || o->last_used < donor->last_used))
        donor = o.get();
  if (donor) {
    oic_handle h = donor->h;
    donor->h = nullptr;
    donor->busy = true;  // its requests wait until its state is saved
    s->evictions++;
    lk.unlock();
    donor->u_prev.resize((size_t)donor->cfg.l * donor->cfg.m);
    int rc = oic_get_u_prev(h, donor->u_prev.data());
    if (rc == OIC_OK) rc = load_controller(h, c);
    lk.lock();
    donor->busy = false;
    if (rc != OIC_OK) {
      lk.unlock();
      oic_destroy(h);
      lk.lock();
      s->used -= donor->footprint;
      return rc;
    }
    c.h = h;  // same footprint: the budget is unchanged
    s->admissions++;
    s->recycled++;
    return OIC_OK;
  }
  std::vector<std::pair<oic_handle, Controller*>> victims;
  while (s->used + c.footprint > s->budget) {
    Controller* victim = nullptr;
    for (auto& o : s->ctrls)
      if (o->h && !o->busy && o.get() != &c && (!victim || o->last_used < victim->last_used))
        victim = o.get();
    if (!victim) {
      for (auto& v : victims) {  // undo (cannot happen after a positive can_admit)
        v.second->h = v.first;
        v.second->busy = false;
        s->used += v.second->footprint;
        s->evictions--;
      }
      return OIC_ENOMEM;
    }
    victims.emplace_back(victim->h, victim);
    victim->h = nullptr;
    victim->busy = true;  // its requests wait until its state is saved
    s->used -= victim->footprint;
    s->evictions++;
  }
  s->used += c.footprint;
  if (s->used > s->peak_used) s->peak_used = s->used;
  lk.unlock();
  for (auto& v : victims) {
    Controller* vc = v.second;
    vc->u_prev.resize((size_t)vc->cfg.l * vc->cfg.m);
    oic_get_u_prev(v.first, vc->u_prev.data());
    oic_destroy(v.first);
  }
  oic_handle h = nullptr;
  int rc = oic_create(&c.cfg, &h);
  if (rc == OIC_OK) {
    rc = load_controller(h, c);
    if (rc != OIC_OK) {
      oic_destroy(h);
      h = nullptr;
    }
  }
  lk.lock();
  for (auto& v : victims) v.second->busy = false;
  if (rc != OIC_OK) {
    s->used -= c.footprint;
    return rc;
  }
  c.h = h;
  s->admissions++;
  return OIC_OK;
}

void worker(oic_server* s) {
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    // oldest request whose controller is idle
    auto it = s->queue.end();
    auto blocked = s->queue.end();  // oldest request held back by memory alone
    s->cv_work.wait(lk, [&] {
      if (s->stop) return true;
      // oldest request whose controller is idle and whose buffers fit (admission by
      // HBM footprint: otherwise it waits until memory frees up); nothing starts behind a
      // request that has waited for memory past kMaxBypass
      blocked = s->queue.end();
      for (auto q = s->queue.begin(); q != s->queue.end(); ++q) {
        const Controller& c = *s->ctrls[q->controller];
        if (c.busy) continue;
        if (can_admit(s, c)) {
          it = q;
          return true;
        }
        if (blocked == s->queue.end()) {
          blocked = q;
          if (q->bypassed >= kMaxBypass) return false;  // reserved: wait for memory to free up
        }
      }
      return false;
    });
    if (s->stop) return;
    if (blocked != s->queue.end() && blocked < it) blocked->bypassed++;
    Request req = std::move(*it);
    s->queue.erase(it);
    Controller& c = *s->ctrls[req.controller];
    c.busy = true;
    c.last_used = ++s->tick;
    Result res;
    int rc = make_resident(s, c, lk);
    const auto start = Clock::now();
    if (rc == OIC_OK) {
      lk.unlock();
      res.U.resize((size_t)(c.H + 1) * c.cfg.l * c.cfg.m);
      res.X.resize((size_t)(c.H + 1) * c.cfg.n * c.cfg.m);
      rc = oic_solve(c.h, req.X0.data(), req.ref.data(), c.Q.data(), c.R.data(), c.N, c.H, req.seed,
                     res.U.data(), res.X.data());
      if (rc != OIC_OK) res.err = oic_last_error(c.h);
      lk.lock();
    } else {
      res.err = "controller does not fit the HBM budget";
    }
    const auto end = Clock::now();
    res.rc = rc;
    res.done = true;
    res.latency_ms = std::chrono::duration<double, std::milli>(end - req.submitted).count();
    res.queue_ms = std::chrono::duration<double, std::milli>(start - req.submitted).count();
    c.busy = false;
    s->results[req.ticket] = std::move(res);
    s->completed++;
    s->cv_done.notify_all();
    s->cv_work.notify_all();
  }
}

}  // namespace

extern "C" {

size_t oic_footprint_bytes(const oic_config* cfg) { return cfg ? footprint_bytes(*cfg) : 0; }

int oic_server_create(size_t hbm_budget_bytes, int max_inflight, oic_server_handle* out) {
  if (!out || max_inflight < 1 || max_inflight > 64 || hbm_budget_bytes == 0) return OIC_EINVAL;
  *out = nullptr;
  oic_server* s = new (std::nothrow) oic_server();
  if (!s) return OIC_ENOMEM;
  s->budget = hbm_budget_bytes;
  for (int w = 0; w < max_inflight; ++w) s->workers.emplace_back(worker, s);
  *out = s;
  return OIC_OK;
}

void oic_server_destroy(oic_server_handle s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (auto& t : s->workers) t.join();
  for (auto& c : s->ctrls)
    if (c->h) oic_destroy(c->h);
  delete s;
}

int oic_server_add(oic_server_handle s, const oic_config* cfg, const float* B, const float* const* W,
                   const float* const* bias, int N, int horizon, const float* Q, const float* R,
                   int* controller_id) {
  if (!s || !cfg || !B || !W || !Q || !R || !controller_id) return OIC_EINVAL;
  if (cfg->mem_mode != OIC_MEM_HOST || cfg->n_layers < 1 || cfg->n_layers > OIC_MAX_LAYERS)
    return OIC_EINVAL;
  if (N < 2 || horizon < 1) return OIC_EINVAL;
  auto c = std::make_unique<Controller>();
  c->cfg = *cfg;
  c->cfg.max_N = N;
  c->cfg.max_H = horizon;
  c->cfg.stream = nullptr;  // each controller gets its own stream
  c->N = N;
  c->H = horizon;
  const size_t n = cfg->n, l = cfg->l;
  c->B.assign(B, B + n * l);
  c->Q.assign(Q, Q + l * l);
  c->R.assign(R, R + n * n);
  for (int k = 0; k < cfg->n_layers; ++k) {
    const size_t cnt = (size_t)cfg->channels[k + 1] * cfg->channels[k] * 9;
    if (!W[k]) return OIC_EINVAL;
    c->W.emplace_back(W[k], W[k] + cnt);
    if (bias && bias[k])
      c->bias.emplace_back(bias[k], bias[k] + cfg->channels[k + 1]);
    else
      c->bias.emplace_back();
  }
  c->footprint = footprint_bytes(c->cfg);
  std::lock_guard<std::mutex> g(s->mu);
  if (c->footprint > s->budget) return OIC_ENOMEM;
  *controller_id = (int)s->ctrls.size();
  s->ctrls.push_back(std::move(c));
  return OIC_OK;
}

int oic_server_submit(oic_server_handle s, int controller_id, const float* X0, const float* reference,
                      uint64_t seed, long long* ticket) {
  if (!s || !X0 || !reference || !ticket) return OIC_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  if (controller_id < 0 || controller_id >= (int)s->ctrls.size()) return OIC_EINVAL;
  const Controller& c = *s->ctrls[controller_id];
  Request r;
  r.ticket = s->next_ticket++;
  r.controller = controller_id;
  r.X0.assign(X0, X0 + (size_t)c.cfg.n * c.cfg.m);
  r.ref.assign(reference, reference + (size_t)(c.H + 1) * c.cfg.n * c.cfg.m);
  r.seed = seed;
  r.submitted = Clock::now();
  *ticket = r.ticket;
  s->results[r.ticket] = Result();
  s->queue.push_back(std::move(r));
  s->cv_work.notify_all();
  return OIC_OK;
}

int oic_server_wait(oic_server_handle s, long long ticket, float* U_out, float* X_out,
                    double* latency_ms, double* queue_ms) {
  if (!s) return OIC_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->results.find(ticket);
  if (it == s->results.end()) return OIC_EINVAL;
  s->cv_done.wait(lk, [&] { return it->second.done; });
  Result res = std::move(it->second);
  s->results.erase(it);
  lk.unlock();
  if (res.rc != OIC_OK) {
    std::lock_guard<std::mutex> g(s->mu);
    s->err = res.err;
    return res.rc;
  }
  if (U_out) memcpy(U_out, res.U.data(), res.U.size() * sizeof(float));
  if (X_out) memcpy(X_out, res.X.data(), res.X.size() * sizeof(float));
  if (latency_ms) *latency_ms = res.latency_ms;
  if (queue_ms) *queue_ms = res.queue_ms;
  return OIC_OK;
}

int oic_server_stats(oic_server_handle s, long long* completed, long long* admissions,
                     long long* evictions, long long* recycled, size_t* bytes_in_use, size_t* peak_bytes) {
  if (!s) return OIC_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  if (completed) *completed = s->completed;
  if (admissions) *admissions = s->admissions;
  if (evictions) *evictions = s->evictions;
  if (recycled) *recycled = s->recycled;
  if (bytes_in_use) *bytes_in_use = s->used;
  if (peak_bytes) *peak_bytes = s->peak_used;
  return OIC_OK;
}

const char* oic_server_last_error(oic_server_handle s) { return s ? s->err.c_str() : "NULL server"; }

}  // extern "C"
