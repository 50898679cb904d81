// Serving loop for many independent controllers (continuous admission and batching).
//
// Controllers of one shape (grid, control rows, layer widths, activation, precision, N,
// H) live in the slots of packs: a pack is a liboic group, whose slots share one launch
// per kernel of a solve (oic_group_solve).  Requests (one MPC solve each: X_k, the
// reference window and a seed) enter a FIFO queue.  A pool of worker threads takes the
// oldest request whose controller can run: resident in a pack that is not solving, or
// placeable in a free slot of such a pack of its shape (while a solving pack of its shape
// has a free slot it waits for that pack's next batch), else in a new pack whose HBM
// footprint fits the budget beside the resident packs, else in the slot of an idle
// controller of its shape, else in a new pack after evicting idle packs.
// The worker then adds the oldest queued requests of other controllers of that pack (or
// that fit its free slots) up to its slot count, and runs them as one grouped solve;
// requests that arrive meanwhile queue for the next batch.  Packs of different shapes
// solve concurrently on their own streams.  Solves of one controller run in submission
// order (U_prev carries over), and every slot computes exactly its own solve, so each
// result is the same alone and in any mix.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
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

struct Pack;

struct Controller {
  oic_config cfg{};
  int N = 0, H = 0;
  std::vector<float> B, Q, R;
  bool q_diag = true, r_diag = true;
  std::vector<std::vector<float>> W, bias;
  std::vector<float> u_prev;  // host copy while not resident
  Pack* pack = nullptr;       // resident: its pack and slot
  int slot = -1;
  bool busy = false;          // in a batch, or its state is being saved
  long long last_used = 0;
};

struct Pack {
  oic_config cfg{};
  int slots = 1;
  oic_group_handle g = nullptr;    // null until created
  std::vector<Controller*> holder;  // resident controller per slot (or null)
  size_t footprint = 0;
  bool running = false;  // a batch is being loaded or solved
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
// flight finish, their packs become idle and evictable, and it is admitted.  This
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
  int max_slots = 8;
  std::vector<std::unique_ptr<Controller>> ctrls;
  std::vector<std::unique_ptr<Pack>> packs;
  std::deque<Request> queue;
  std::map<long long, Result> results;
  long long next_ticket = 1, tick = 0;
  long long completed = 0, evictions = 0, admissions = 0, recycled = 0;
  long long batches = 0, grouped = 0, packs_created = 0;
  bool started = false;
  size_t peak_used = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  std::vector<std::thread> workers;
  std::string err;
};

namespace {

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

// Slots of a new pack for c's shape: several where one solve leaves the GPU idle (about
// 2^22 pixel-members per launch fill it; the grouped kernels exist for the BF16 rollout),
// no more than the controllers of that shape, and a pack that fits the budget.
int slots_for(const oic_server* s, const Controller& c) {
  if (s->max_slots <= 1 || c.cfg.precision != OIC_PREC_BF16 || !oic::bf16_rollout_possible(c.cfg)) return 1;
  const double work = (double)c.cfg.n * c.cfg.m * c.N;
  int g = (int)std::min<double>(s->max_slots, std::floor(4194304.0 / work));
  int same = 0;
  for (auto& o : s->ctrls) same += same_shape(o->cfg, c.cfg) ? 1 : 0;
  g = std::max(1, std::min(g, same));
  while (g > 1 && oic_group_footprint_bytes(&c.cfg, g) > s->budget) g /= 2;
  return g;
}

// A free slot of a pack of c's shape (-1: none), in a pack that is not solving unless
// `running` is set.  *pack receives the pack.
int free_slot(const oic_server* s, const Controller& c, bool running, Pack** pack) {
  for (auto& p : s->packs) {
    if ((!running && (p->running || !p->g)) || !same_shape(p->cfg, c.cfg)) continue;
    for (int k = 0; k < p->slots; ++k)
      if (!p->holder[k]) {
        *pack = p.get();
        return k;
      }
  }
  return -1;
}

// The slot of the least recently used idle controller of c's shape in a pack that is not
// solving (-1: none).  *pack receives the pack.
int idle_slot(const oic_server* s, const Controller& c, Pack** pack) {
  int best_slot = -1;
  long long best_used = 0;
  for (auto& p : s->packs) {
    if (p->running || !p->g || !same_shape(p->cfg, c.cfg)) continue;
    for (int k = 0; k < p->slots; ++k) {
      Controller* o = p->holder[k];
      if (o && !o->busy && (best_slot < 0 || o->last_used < best_used)) {
        *pack = p.get();
        best_slot = k;
        best_used = o->last_used;
      }
    }
  }
  return best_slot;
}

// Device bytes of idle packs (not solving, no busy holder) that could be evicted.
size_t reclaimable(const oic_server* s) {
  size_t r = 0;
  for (auto& p : s->packs)
    if (!p->running && p->g) r += p->footprint;
  return r;
}

// Whether c's request can start now: resident in a pack that is not solving, or
// placeable in a free slot of such a pack; it waits for its pack (or for a solving pack
// of its shape with a free slot, which takes it in its next batch), else it can start in
// an idle controller's slot or a new pack that fits after evicting idle packs, or it
// waits for memory.
enum Readiness { kRun, kWaitPack, kWaitMemory };
Readiness readiness(const oic_server* s, const Controller& c) {
  if (c.busy) return kWaitPack;
  if (c.pack) return c.pack->running ? kWaitPack : kRun;
  Pack* p = nullptr;
  if (free_slot(s, c, false, &p) >= 0) return kRun;
  if (free_slot(s, c, true, &p) >= 0) return kWaitPack;
  if (idle_slot(s, c, &p) >= 0) return kRun;
  const size_t fp = oic_group_footprint_bytes(&c.cfg, slots_for(s, c));
  return s->used - reclaimable(s) + fp <= s->budget ? kRun : kWaitMemory;
}

// Device work of one batch, decided under the lock and done outside it.
struct Plan {
  std::vector<std::unique_ptr<Pack>> evicted;  // packs to save and destroy
  std::vector<Controller*> evicted_holders;    // their residents (busy until saved)
  std::vector<std::pair<Controller*, oic_handle>> displaced;  // take-overs: save U_prev first
  std::vector<Controller*> load;               // controllers to load into their slots
  bool create = false;                         // the pack is new
};

// Puts c into slot k of p (the lock is held); a holder there is displaced.
void place(oic_server* s, Controller& c, Pack* p, int k, Plan& plan) {
  if (Controller* o = p->holder[k]) {
    plan.displaced.emplace_back(o, p->g ? oic_group_slot(p->g, k) : nullptr);
    o->pack = nullptr;
    o->slot = -1;
    o->busy = true;  // its requests wait until its U_prev is saved
    s->evictions++;
    s->recycled++;
  }
  p->holder[k] = &c;
  c.pack = p;
  c.slot = k;
  plan.load.push_back(&c);
  s->admissions++;
}

// Makes c resident for a batch, marking its pack as running (the lock is held).
int make_resident(oic_server* s, Controller& c, Plan& plan) {
  if (c.pack) {
    c.pack->running = true;
    return OIC_OK;
  }
  Pack* p = nullptr;
  const int G = slots_for(s, c);
  const size_t fp = oic_group_footprint_bytes(&c.cfg, G);
  // a free slot of a same-shape pack; else (every pack of the shape full) a new pack if it
  // fits as things stand; else an idle controller's slot; else a new pack after evicting
  // least recently used idle packs
  int k = free_slot(s, c, false, &p);
  if (k < 0 && s->used + fp > s->budget) k = idle_slot(s, c, &p);
  if (k < 0) {
    while (s->used + fp > s->budget) {
      Pack* victim = nullptr;
      for (auto& q : s->packs)
        if (!q->running && q->g && (!victim || q->last_used < victim->last_used)) victim = q.get();
      if (!victim) return OIC_ENOMEM;  // cannot happen after kRun
      for (Controller* o : victim->holder)
        if (o) {
          o->pack = nullptr;
          o->slot = -1;
          o->busy = true;
          plan.evicted_holders.push_back(o);
          s->evictions++;
        }
      s->used -= victim->footprint;
      auto it = std::find_if(s->packs.begin(), s->packs.end(), [&](auto& q) { return q.get() == victim; });
      plan.evicted.push_back(std::move(*it));
      s->packs.erase(it);
    }
    auto np = std::make_unique<Pack>();
    np->cfg = c.cfg;
    np->slots = G;
    np->holder.assign(G, nullptr);
    np->footprint = fp;
    s->used += fp;
    s->peak_used = std::max(s->peak_used, s->used);
    s->packs_created++;
    p = np.get();
    s->packs.push_back(std::move(np));
    plan.create = true;
    k = 0;
  }
  place(s, c, p, k, plan);
  p->running = true;
  return OIC_OK;
}

// Loads c's surrogate and applied control into its slot's handle.
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

void save_u_prev(Controller* o, oic_handle h) {
  o->u_prev.resize((size_t)o->cfg.l * o->cfg.m);
  if (h) oic_get_u_prev(h, o->u_prev.data());
}

void worker(oic_server* s) {
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    auto it = s->queue.end();
    auto blocked = s->queue.end();  // oldest request held back by memory alone
    s->cv_work.wait(lk, [&] {
      if (s->stop) return true;
      // oldest request whose controller is idle and can run (admission by HBM footprint:
      // otherwise it waits until memory frees up); nothing starts behind a request that
      // has waited for memory past kMaxBypass
      blocked = s->queue.end();
      for (auto q = s->queue.begin(); q != s->queue.end(); ++q) {
        const Readiness r = readiness(s, *s->ctrls[q->controller]);
        if (r == kWaitPack) continue;
        if (r == kRun) {
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
    std::vector<Request> batch;
    batch.push_back(std::move(*it));
    s->queue.erase(it);
    Controller& c0 = *s->ctrls[batch[0].controller];
    c0.busy = true;
    c0.last_used = ++s->tick;
    Plan plan;
    int rc = make_resident(s, c0, plan);
    Pack* pk = c0.pack;
    if (rc == OIC_OK) {
      // the oldest queued requests of other controllers that this pack can take: resident
      // in it, or placeable in a free slot or an idle holder's slot; one per controller,
      // same Q and R structure (one batch draws its noise factors alike)
      for (auto q = s->queue.begin(); q != s->queue.end() && (int)batch.size() < pk->slots;) {
        Controller& c = *s->ctrls[q->controller];
        bool take = false;
        if (!c.busy && c.q_diag == c0.q_diag && c.r_diag == c0.r_diag) {
          if (c.pack == pk) {
            take = true;
          } else if (!c.pack && same_shape(c.cfg, pk->cfg)) {
            int k = -1;
            for (int j = 0; j < pk->slots && k < 0; ++j)
              if (!pk->holder[j]) k = j;
            if (k < 0) {  // the least recently used holder that is not in the batch
              long long lu = 0;
              for (int j = 0; j < pk->slots; ++j) {
                Controller* o = pk->holder[j];
                if (o && !o->busy && (k < 0 || o->last_used < lu)) {
                  k = j;
                  lu = o->last_used;
                }
              }
            }
            if (k >= 0) {
              place(s, c, pk, k, plan);
              take = true;
            }
          }
        }
        if (take) {
          c.busy = true;
          c.last_used = ++s->tick;
          batch.push_back(std::move(*q));
          q = s->queue.erase(q);
        } else {
          ++q;
        }
      }
    }
    lk.unlock();
    const auto start = Clock::now();
    const int count = (int)batch.size();
    std::vector<int> rcs(count, rc);
    std::vector<Result> res(count);
    std::string err = rc == OIC_OK ? "" : "controller does not fit the HBM budget";
    // evicted packs: save their residents' U_prev, free them; controllers that lose their
    // slot to the batch: save their U_prev before the slot is loaded
    for (auto& ep : plan.evicted) {
      for (int k = 0; k < ep->slots; ++k)
        if (Controller* o = ep->holder[k]) save_u_prev(o, oic_group_slot(ep->g, k));
      oic_group_destroy(ep->g);
    }
    for (auto& d : plan.displaced) save_u_prev(d.first, d.second);
    if (rc == OIC_OK) {
      if (plan.create) {
        oic_group_handle g = nullptr;
        rc = oic_group_create(&pk->cfg, pk->slots, &g);
        if (rc == OIC_OK) {
          pk->g = g;
        } else {
          err = "group creation failed";
        }
      }
      std::vector<int> slot_of(count, -1);
      std::vector<oic_solve_args> args(count);
      std::vector<int> sl;
      std::vector<oic_solve_args> run;
      std::vector<int> idx;
      for (int i = 0; i < count; ++i) {
        Controller& c = *s->ctrls[batch[i].controller];
        if (rc != OIC_OK) {
          rcs[i] = rc;
          continue;
        }
        if (std::find(plan.load.begin(), plan.load.end(), &c) != plan.load.end()) {
          rcs[i] = load_controller(oic_group_slot(pk->g, c.slot), c);
          if (rcs[i] != OIC_OK) continue;
        }
        res[i].U.resize((size_t)(c.H + 1) * c.cfg.l * c.cfg.m);
        res[i].X.resize((size_t)(c.H + 1) * c.cfg.n * c.cfg.m);
        oic_solve_args a{};
        a.X0 = batch[i].X0.data();
        a.reference = batch[i].ref.data();
        a.Q = c.Q.data();
        a.R = c.R.data();
        a.N = c.N;
        a.horizon = c.H;
        a.seed = batch[i].seed;
        a.U_out = res[i].U.data();
        a.X_out = res[i].X.data();
        run.push_back(a);
        sl.push_back(c.slot);
        idx.push_back(i);
      }
      if (!run.empty()) {
        std::vector<int> out(run.size(), OIC_OK);
        const int grc = oic_group_solve(pk->g, (int)run.size(), sl.data(), run.data(), out.data());
        if (grc != OIC_OK) err = oic_group_last_error(pk->g);
        for (size_t j = 0; j < run.size(); ++j) rcs[idx[j]] = out[j];
        if (grc != OIC_OK && std::all_of(out.begin(), out.end(), [](int v) { return v == OIC_OK; }))
          for (size_t j = 0; j < run.size(); ++j) rcs[idx[j]] = grc;  // the batch as a whole failed
      }
    }
    const auto end = Clock::now();
    lk.lock();
    for (Controller* o : plan.evicted_holders) o->busy = false;
    for (auto& d : plan.displaced) d.first->busy = false;
    if (pk) {
      if (plan.create && !pk->g) {  // creation failed: give the reservation back
        for (Controller* o : pk->holder)
          if (o) {
            o->pack = nullptr;
            o->slot = -1;
          }
        s->used -= pk->footprint;
        auto pit = std::find_if(s->packs.begin(), s->packs.end(), [&](auto& q) { return q.get() == pk; });
        if (pit != s->packs.end()) s->packs.erase(pit);
        pk = nullptr;
      } else {
        pk->running = false;
        pk->last_used = ++s->tick;
      }
    }
    s->batches++;
    if (count > 1) s->grouped += count;
    for (int i = 0; i < count; ++i) {
      Controller& c = *s->ctrls[batch[i].controller];
      if (rcs[i] != OIC_OK && pk && c.pack == pk && std::find(plan.load.begin(), plan.load.end(), &c) !=
                                                        plan.load.end()) {
        // a slot that could not be loaded holds nothing usable
        pk->holder[c.slot] = nullptr;
        c.pack = nullptr;
        c.slot = -1;
      }
      c.busy = false;
      Result& r = res[i];
      r.rc = rcs[i];
      if (rcs[i] != OIC_OK) r.err = err.empty() ? "solve failed" : err;
      r.done = true;
      r.latency_ms = std::chrono::duration<double, std::milli>(end - batch[i].submitted).count();
      r.queue_ms = std::chrono::duration<double, std::milli>(start - batch[i].submitted).count();
      s->results[batch[i].ticket] = std::move(r);
      s->completed++;
    }
    // evicted packs are freed outside the lock above; their objects go here
    plan.evicted.clear();
    s->cv_done.notify_all();
    s->cv_work.notify_all();
  }
}

}  // namespace

extern "C" {

size_t oic_footprint_bytes(const oic_config* cfg) { return oic_group_footprint_bytes(cfg, 1); }

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

int oic_server_set_group_slots(oic_server_handle s, int max_slots) {
  if (!s || max_slots < 1 || max_slots > OIC_MAX_GROUP_SLOTS) return OIC_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  if (s->started) return OIC_EINVAL;
  s->max_slots = max_slots;
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
  for (auto& p : s->packs)
    if (p->g) oic_group_destroy(p->g);
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
  c->cfg.stream = nullptr;  // each slot's handle gets its own stream
  c->N = N;
  c->H = horizon;
  const size_t n = cfg->n, l = cfg->l;
  c->B.assign(B, B + n * l);
  c->Q.assign(Q, Q + l * l);
  c->R.assign(R, R + n * n);
  auto diagonal = [](const std::vector<float>& A, size_t k) {
    for (size_t i = 0; i < k; ++i)
      for (size_t j = 0; j < k; ++j)
        if (i != j && A[i * k + j] != 0.f) return false;
    return true;
  };
  c->q_diag = diagonal(c->Q, l);
  c->r_diag = diagonal(c->R, n);
  for (int k = 0; k < cfg->n_layers; ++k) {
    const size_t cnt = (size_t)cfg->channels[k + 1] * cfg->channels[k] * 9;
    if (!W[k]) return OIC_EINVAL;
    c->W.emplace_back(W[k], W[k] + cnt);
    if (bias && bias[k])
      c->bias.emplace_back(bias[k], bias[k] + cfg->channels[k + 1]);
    else
      c->bias.emplace_back();
  }
  std::lock_guard<std::mutex> g(s->mu);
  if (oic_group_footprint_bytes(&c->cfg, 1) > s->budget) return OIC_ENOMEM;
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
  s->started = true;
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

int oic_server_batch_stats(oic_server_handle s, long long* batches, long long* grouped_solves,
                           long long* packs_created) {
  if (!s) return OIC_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  if (batches) *batches = s->batches;
  if (grouped_solves) *grouped_solves = s->grouped;
  if (packs_created) *packs_created = s->packs_created;
  return OIC_OK;
}

const char* oic_server_last_error(oic_server_handle s) { return s ? s->err.c_str() : "NULL server"; }

}  // extern "C"
