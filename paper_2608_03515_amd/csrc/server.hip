// Continuous-batching solve server.  Requests (a gauge field held by the server, a bare mass,
// setup parameters, 1..slots right-hand sides) are admitted into solver instances: a batch
// workspace of fixed slot count on its own HIP stream, bound to one AM-AMG hierarchy.
// Admission happens at restart-cycle boundaries, while the instance's other slots keep
// iterating, and instances bound to different hierarchies run concurrently on their streams.
// Hierarchies are cached per (gauge, mass, setup parameters) and evicted least recently used
// when the device-memory budget would be exceeded.
//
// One worker thread owns every device object of the server; the C entry points only queue
// requests, read gauges in and hand back completed requests.  Because an instance's slot
// count is fixed, a right-hand side's arithmetic (reduction blocking included) does not
// depend on which other requests share the device: a request's result is bitwise the same
// alone and in any mix.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>

#include "runtime.hpp"

using namespace amamg;
using namespace amamg::rt;

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t id = 0;
  int gauge = 0;
  double m0 = 0;
  double ref = NAN;            // the gauge's reference mass at submission (NaN: none)
  amamg_setup_params sp{};
  int nrhs = 0;
  std::vector<double> psi;     // copied at submission: [nrhs][n] complex
  double* x = nullptr;         // caller's output
  double t_submit = 0, t_admit = 0, t_done = 0;
  int status = AMAMG_OK;
  int remaining = 0;           // right-hand sides still running
  int iterations = 0, converged = 1, built = 0, instance = -1;
  double residual = 0;
};

struct CachedH {
  amamg_hierarchy* h = nullptr;
  int gauge = 0;
  double m0 = 0;
  double ref = NAN;            // mass its interpolation was built at, when a reference mass
                               // applies (NaN: a setup at m0 for requests without one)
  amamg_setup_params sp{};
  uint64_t last_use = 0;
  int users = 0;               // instances bound to it
  bool fresh = true;           // built, not bound yet: not evicted before its requests run
  size_t bytes = 0;
  CachedH* base = nullptr;     // derived at another mass from this full setup (shares its data)
  int derived = 0;             // cached hierarchies derived from this one
  int pending = 0;             // derivations from this one in flight
};

// A hierarchy build handed to the builder thread, and its outcome.
struct BuildJob {
  uint64_t id = 0;
  int gauge = 0;
  double m0 = 0;
  double ref = NAN;
  amamg_setup_params sp{};
  CachedH* base = nullptr;     // non-null: derive from this hierarchy instead of a setup
  size_t need = 0;             // bytes reserved for it in the budget while it runs
  amamg_hierarchy* h = nullptr;
  amamg_status code = AMAMG_OK;
  std::string msg;
  double seconds = 0;
};

struct Instance {
  int id = 0;
  hipStream_t stream = nullptr;
  Workspace ws;
  Arena io;                    // right-hand sides B and iterates X, [slots][n]
  int64_t n_io = 0;
  double2 *B = nullptr, *X = nullptr;
  Batch bt;
  CachedH* ch = nullptr;
  enum Phase { IDLE, CHECKING, RUNNING } phase = IDLE;
  std::vector<Request*> slot_req;     // request in the slot (nullptr: free)
  std::vector<int> slot_rhs;          // its right-hand-side index
  std::vector<int> checking;          // slots under the input check
  std::vector<Request*> reserved;     // requests waiting for this instance's next boundary
  uint64_t stamp = 0;                 // order of the last enqueued stage
  int free_slots() const {
    int f = 0;
    for (Request* r : slot_req) f += r ? 0 : 1;
    for (Request* r : reserved) f -= r->nrhs;
    return f;
  }
  bool busy() const { return phase != IDLE || !reserved.empty(); }
};

bool same_ref(double a, double b) { return (std::isnan(a) && std::isnan(b)) || a == b; }

bool same_params(const amamg_setup_params& a, const amamg_setup_params& b) {
  return a.levels == b.levels && a.agg_size == b.agg_size && a.overlap == b.overlap &&
         a.n_test_vectors == b.n_test_vectors && a.test_vector_sweeps == b.test_vector_sweeps &&
         a.pre_sweeps == b.pre_sweeps && a.post_sweeps == b.post_sweeps && a.norm == b.norm &&
         a.seed == b.seed && a.coarsest_tol == b.coarsest_tol && a.block_smoother == b.block_smoother &&
         (a.coarsest_tol == 0 || a.coarsest_max_iters == b.coarsest_max_iters);
}

}  // namespace

struct amamg_server {
  amamg_context* ctx = nullptr;
  amamg_server_params prm{};
  Clock::time_point t0;
  // shared with the callers and the builder (mu)
  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_build;
  std::deque<Request*> incoming;
  std::deque<Request*> done;
  std::vector<amamg_gauge*> gauges;
  std::vector<double> refs;           // reference mass per gauge (NaN: none)
  uint64_t next_job = 1;
  std::deque<BuildJob> jobs, built;
  uint64_t next_id = 1;
  int64_t outstanding = 0;
  bool stop = false, stop_builder = false;
  std::string err;
  int64_t setups = 0, evictions = 0, derivations = 0;
  size_t resident = 0, peak_resident = 0, last_estimate = 0, hier_bytes = 0;
  double setup_seconds = 0, setup_seconds_max = 0, derive_seconds = 0, derive_seconds_max = 0;
  // worker only
  std::thread worker;
  std::deque<Request*> queue;
  std::vector<std::unique_ptr<CachedH>> cache;
  std::vector<std::unique_ptr<Instance>> inst;
  std::vector<BuildJob> building;     // builds in flight (keys and reserved bytes)
  uint64_t tick = 0;
  // builders: one thread, stream and setup-scratch pool (reused from build to build) each
  struct Builder {
    std::thread th;
    hipStream_t stream = nullptr;
    Pool scratch;
    size_t scratch_bytes = 0;   // (mu)
  };
  std::vector<std::unique_ptr<Builder>> builders;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

amamg_solve_params solve_params(const amamg_server* S) {
  amamg_solve_params p;
  amamg_default_solve_params(&p);
  p.restart = S->prm.restart;
  p.max_iters = S->prm.max_iters;
  p.rel_tol = S->prm.rel_tol;
  p.precision = S->prm.precision;
  p.graphs = S->prm.graphs;
  return p;
}

size_t resident_bytes(amamg_server* S) {
  size_t b = 0;
  for (const auto& c : S->cache) b += c->bytes;
  for (const auto& I : S->inst) b += I->ws.block_bytes + I->io.bytes;
  for (const BuildJob& j : S->building) b += j.need;
  std::lock_guard<std::mutex> lk(S->mu);
  for (const auto& B : S->builders) b += B->scratch_bytes;
  return b;
}

void account(amamg_server* S) {
  const size_t r = resident_bytes(S);
  size_t hb = 0;
  for (const auto& c : S->cache) hb += c->bytes;
  std::lock_guard<std::mutex> lk(S->mu);
  S->resident = r;
  S->hier_bytes = hb;
  S->peak_resident = std::max(S->peak_resident, r);
}

void finish(amamg_server* S, Request* R) {
  R->t_done = S->now();
  std::lock_guard<std::mutex> lk(S->mu);
  S->done.push_back(R);
  S->outstanding -= 1;
  S->cv_done.notify_all();
}

void drop(amamg_server* S, CachedH* victim) {
  if (victim->base) {
    victim->base->derived -= 1;
    victim->h->base->derived -= 1;
  }
  victim->h->gauge->nhier -= 1;
  delete victim->h;
  S->cache.erase(std::find_if(S->cache.begin(), S->cache.end(),
                              [&](const std::unique_ptr<CachedH>& c) { return c.get() == victim; }));
  std::lock_guard<std::mutex> lk(S->mu);
  S->evictions += 1;
}

// Make `need` more bytes fit the budget: drop least recently used hierarchies that nothing
// holds (no instance bound, no derived hierarchy or derivation depending on them), unbinding
// idle instances and finally releasing idle instances' workspaces when nothing else is left.
// `keep` (if any) is never released.
bool make_room(amamg_server* S, size_t need, const Instance* keep = nullptr) {
  for (;;) {
    if (resident_bytes(S) + need <= S->prm.hbm_budget) return true;
    CachedH* victim = nullptr;
    for (const auto& c : S->cache)
      if (c->users == 0 && !c->fresh && c->derived == 0 && c->pending == 0 &&
          (!victim || c->last_use < victim->last_use))
        victim = c.get();
    if (victim) {
      drop(S, victim);
      continue;
    }
    // release the hierarchy of the idle instance used least recently, then look again
    Instance* idle = nullptr;
    for (const auto& I : S->inst)
      if (I.get() != keep && !I->busy() && I->ch && (!idle || I->ch->last_use < idle->ch->last_use))
        idle = I.get();
    if (idle) {
      idle->ch->users -= 1;
      idle->ch = nullptr;
      continue;
    }
    // then the device memory of an unbound idle instance
    Instance* empty = nullptr;
    for (const auto& I : S->inst)
      if (I.get() != keep && !I->busy() && !I->ch && (I->ws.block_bytes > 0 || I->io.bytes > 0)) empty = I.get();
    if (!empty) return false;
    empty->ws.release();
    empty->io.release();
    empty->n_io = 0;
  }
}

// Estimated device bytes of an instance workspace bound to a lattice with n fine unknowns.
size_t instance_estimate(const amamg_server* S, int64_t n) {
  const int m = S->prm.restart;
  const size_t zs = S->prm.precision == AMAMG_FP64 ? 16 : 8;
  return size_t(S->prm.slots) * n * (16 * size_t(m + 1) + zs * (m + 3) + 16 * 3);
}

bool has_ref(const Request* R) { return !std::isnan(R->ref); }

// the hierarchy that solves R: built at R's mass (no reference mass), the base at the reference
// mass (R at that mass) or derived from it
bool same_key(const CachedH& c, const Request* R) {
  return c.gauge == R->gauge && c.m0 == R->m0 && same_ref(c.ref, R->ref) && same_params(c.sp, R->sp);
}

CachedH* cached(amamg_server* S, const Request* R) {
  for (const auto& c : S->cache)
    if (same_key(*c, R)) return c.get();
  return nullptr;
}

// The base hierarchy R's would be derived from: built at R's reference mass.
CachedH* base_for(amamg_server* S, const Request* R) {
  for (const auto& c : S->cache)
    if (!c->base && c->gauge == R->gauge && c->m0 == R->ref && same_ref(c->ref, R->ref) &&
        same_params(c->sp, R->sp))
      return c.get();
  return nullptr;
}

// A build in flight that makes R's hierarchy, or the base R's hierarchy is derived from.
bool waiting_on_build(const amamg_server* S, const Request* R) {
  return std::any_of(S->building.begin(), S->building.end(), [&](const BuildJob& j) {
    if (j.gauge != R->gauge || !same_ref(j.ref, R->ref) || !same_params(j.sp, R->sp)) return false;
    return j.m0 == R->m0 || (has_ref(R) && !j.base && j.m0 == R->ref);
  });
}

// Queued requests that job j was building for (its hierarchy, or its base)
bool waits_for(const BuildJob& j, const Request* R) {
  if (j.gauge != R->gauge || !same_ref(j.ref, R->ref) || !same_params(j.sp, R->sp)) return false;
  return j.m0 == R->m0 || (!j.base && has_ref(R));
}

void queue_job(amamg_server* S, BuildJob& j, Request* R) {
  j.id = S->next_job++;
  S->building.push_back(j);
  R->built = 1;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->jobs.push_back(j);
  }
  S->cv_build.notify_one();
}

// Hand a derivation of the request's hierarchy from `base` to a builder when the budget allows.
bool dispatch_derive(amamg_server* S, Request* R, CachedH* base) {
  const amamg_hierarchy* h = base->h;
  const size_t need = derive_bytes(h) + instance_estimate(S, h->lv[0].g.ndof());
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->last_estimate = need;
  }
  base->pending += 1;             // not evicted meanwhile
  if (!make_room(S, need)) {
    base->pending -= 1;
    return false;
  }
  BuildJob j;
  j.gauge = R->gauge;
  j.m0 = R->m0;
  j.ref = R->ref;
  j.sp = R->sp;
  j.base = base;
  j.need = need;
  queue_job(S, j, R);
  return true;
}

// Hand a setup at mass `at` (R's mass, or its reference mass) to a builder when the budget
// allows (false: not now).
bool dispatch_build(amamg_server* S, Request* R, double at) {
  amamg_gauge* g;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    g = S->gauges[R->gauge];
  }
  const size_t need = setup_bytes(g->nt, g->nx, R->sp) + instance_estimate(S, int64_t(2) * g->nt * g->nx);
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->last_estimate = need;
  }
  if (!make_room(S, need)) return false;
  BuildJob j;
  j.gauge = R->gauge;
  j.m0 = at;
  j.ref = R->ref;
  j.sp = R->sp;
  j.need = need;
  queue_job(S, j, R);
  return true;
}

// Finished builds: cache the hierarchies, or fail the requests that wait for a failed one.
bool collect_builds(amamg_server* S) {
  std::deque<BuildJob> got;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    got.swap(S->built);
  }
  for (BuildJob& j : got) {
    S->building.erase(std::find_if(S->building.begin(), S->building.end(),
                                   [&](const BuildJob& b) { return b.id == j.id; }));
    if (j.base) j.base->pending -= 1;
    if (j.h) {
      auto c = std::make_unique<CachedH>();
      c->h = j.h;
      c->gauge = j.gauge;
      c->m0 = j.m0;
      c->ref = j.ref;
      c->sp = j.sp;
      c->bytes = j.h->mem.bytes();
      c->last_use = ++S->tick;
      c->base = j.base;
      if (j.base) {
        j.base->derived += 1;
        j.h->base->derived += 1;
      }
      j.h->gauge->nhier += 1;
      S->cache.push_back(std::move(c));
      continue;
    }
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->err = j.msg;
    }
    for (auto it = S->queue.begin(); it != S->queue.end();) {
      Request* R = *it;
      if (waits_for(j, R)) {
        R->status = j.code;
        finish(S, R);
        it = S->queue.erase(it);
      } else {
        ++it;
      }
    }
  }
  return !got.empty();
}

void builder_main(amamg_server* S, amamg_server::Builder* B) {
  (void)hipSetDevice(S->ctx->device);
  for (;;) {
    BuildJob j;
    amamg_gauge* g;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_build.wait(lk, [&] { return !S->jobs.empty() || S->stop_builder; });
      if (S->jobs.empty()) break;
      j = S->jobs.front();
      S->jobs.pop_front();
      g = S->gauges[j.gauge];
    }
    const auto t0 = Clock::now();
    if (j.base) {
      // the base stays cached while this runs (pending) and is only read
      try {
        j.h = derive_mass(j.base->h, j.m0, B->stream);
      } catch (const Fail& f) {
        j.code = f.code;
        j.msg = f.msg;
      }
    } else {
      amamg_hierarchy* h = new amamg_hierarchy();
      h->gauge = g;
      h->m0 = j.m0;
      h->prm = j.sp;
      try {
        run_setup(h, B->stream, &B->scratch);
        if (!std::isnan(j.ref)) ensure_mass_terms(h, B->stream);   // a base: for derivations
        j.h = h;
      } catch (const Fail& f) {
        delete h;
        j.code = f.code;
        j.msg = f.msg;
      }
    }
    j.seconds = std::chrono::duration<double>(Clock::now() - t0).count();
    {
      std::lock_guard<std::mutex> lk(S->mu);
      if (j.h && j.base) {
        S->derivations += 1;
        S->derive_seconds += j.seconds;
        S->derive_seconds_max = std::max(S->derive_seconds_max, j.seconds);
      } else if (j.h) {
        S->setups += 1;
        S->setup_seconds += j.seconds;
        S->setup_seconds_max = std::max(S->setup_seconds_max, j.seconds);
      }
      B->scratch_bytes = B->scratch.bytes();
      S->built.push_back(j);
    }
    S->cv_work.notify_all();
  }
}

void bind(amamg_server* S, Instance* I, CachedH* c) {
  if (I->ch == c) return;
  if (I->ch) I->ch->users -= 1;
  I->ch = c;
  c->users += 1;
  c->fresh = false;
  amamg_hierarchy* h = c->h;
  const int64_t n = h->lv[0].g.ndof();
  const amamg_solve_params p = solve_params(S);
  ensure_workspace(I->ws, h, S->prm.slots, p.restart, p.precision == AMAMG_FP64 ? F64 : F32,
                   2 * p.max_iters + 2);
  if (I->n_io < n) {
    I->io.release();
    I->B = I->io.alloc<double2>(size_t(S->prm.slots) * n);
    I->X = I->io.alloc<double2>(size_t(S->prm.slots) * n);
    I->n_io = n;
  }
  I->bt.init(h, &I->ws, I->stream, p, I->B, I->X, I->id);
}

// Start the input check of the reserved requests (instance at a boundary or idle).
void begin_admission(amamg_server* S, Instance* I) {
  const int64_t n = I->ch->h->lv[0].g.ndof();
  std::vector<int> slots;
  for (Request* R : I->reserved) {
    R->t_admit = S->now();
    R->instance = I->id;
    int k = 0;
    for (int s = 0; s < S->prm.slots && k < R->nrhs; ++s) {
      if (I->slot_req[s]) continue;
      I->slot_req[s] = R;
      I->slot_rhs[s] = k;
      HIPCHECK(hipMemcpyAsync(I->B + int64_t(s) * n, R->psi.data() + size_t(k) * 2 * n, sizeof(double2) * n,
                              hipMemcpyHostToDevice, I->stream));
      slots.push_back(s);
      ++k;
    }
    REQUIRE(k == R->nrhs, AMAMG_ERR_INVALID_ARG, "internal: reserved slots are not free");
    R->remaining = R->nrhs;
  }
  I->reserved.clear();
  I->checking = slots;
  I->ch->last_use = ++S->tick;
  I->bt.admit_begin(slots);
  I->phase = Instance::CHECKING;
  I->stamp = ++S->tick;
}

void release_slot(Instance* I, int s) {
  I->slot_req[s] = nullptr;
  I->slot_rhs[s] = -1;
}

// Input check landed: refuse requests with a non-finite right-hand side, start the others and
// enqueue the next cycle.
void finish_admission(amamg_server* S, Instance* I) {
  const std::vector<int> bad = I->bt.admit_nonfinite();
  std::vector<Request*> failed;
  for (int s : bad)
    if (std::find(failed.begin(), failed.end(), I->slot_req[s]) == failed.end()) failed.push_back(I->slot_req[s]);
  std::vector<int> reject;
  for (int s : I->checking)
    if (std::find(failed.begin(), failed.end(), I->slot_req[s]) != failed.end()) reject.push_back(s);
  I->bt.admit_finish(reject, false);
  for (int s : reject) release_slot(I, s);
  for (Request* R : failed) {
    R->status = AMAMG_ERR_NONFINITE;
    finish(S, R);
  }
  I->checking.clear();
  I->bt.enqueue_state_read();
  I->phase = Instance::RUNNING;
  I->stamp = ++S->tick;
}

// A state read landed: hand back finished right-hand sides and requests, admit what waits for
// this instance, enqueue the next cycle.
void cycle_end(amamg_server* S, Instance* I) {
  const bool any = I->bt.cycle_boundary();
  const int64_t n = I->ch->h->lv[0].g.ndof();
  for (int s = 0; s < S->prm.slots; ++s) {
    Request* R = I->slot_req[s];
    if (!R) continue;
    const RhsState& st = I->bt.state(s);
    if (st.in_cycle) continue;
    // finished: converged, capped or non-finite
    R->iterations = std::max(R->iterations, st.iters);
    R->converged = R->converged && st.converged;
    R->residual = std::max(R->residual, st.true_res);
    if (st.nonfinite) R->status = AMAMG_ERR_NONFINITE;
    HIPCHECK(hipMemcpyAsync(R->x + size_t(I->slot_rhs[s]) * 2 * n, I->X + int64_t(s) * n,
                            sizeof(double2) * n, hipMemcpyDeviceToHost, I->stream));
    HIPCHECK(hipStreamSynchronize(I->stream));
    release_slot(I, s);
    if (--R->remaining == 0) {
      if (R->status == AMAMG_OK && !R->converged) R->status = AMAMG_NOT_CONVERGED;
      finish(S, R);
    }
  }
  if (!I->reserved.empty()) {
    begin_admission(S, I);
    return;
  }
  if (any) {
    I->bt.enqueue_cycle();
    I->bt.enqueue_state_read();
    I->stamp = ++S->tick;
  } else {
    I->phase = Instance::IDLE;
  }
}

// Device bytes that binding instance I (nullptr: a new one) to hierarchy c adds: its workspace
// and right-hand-side buffers grow to c's size and are never shrunk.
size_t bind_bytes(const amamg_server* S, const Instance* I, const CachedH* c) {
  const amamg_solve_params p = solve_params(S);
  const size_t ws = workspace_bytes(c->h, S->prm.slots, p.restart, p.precision == AMAMG_FP64 ? F64 : F32,
                                    2 * p.max_iters + 2);
  const size_t io = sizeof(double2) * 2 * size_t(S->prm.slots) * c->h->lv[0].g.ndof();
  const size_t have_ws = I ? I->ws.block_bytes : 0;
  const size_t have_io = I ? I->io.bytes : 0;
  return (ws > have_ws ? ws - have_ws : 0) + (io > have_io ? io - have_io : 0);
}

// Place queued requests: an instance bound to the request's hierarchy with room (joining at its
// next boundary), else an idle or new instance rebound to it.  A request whose hierarchy is not
// cached starts its build (if the budget allows) and waits for it.
bool place(amamg_server* S) {
  bool did = false;
  for (auto it = S->queue.begin(); it != S->queue.end();) {
    Request* R = *it;
    CachedH* c = cached(S, R);
    if (!c) {
      if (!waiting_on_build(S, R)) {
        // with a reference mass: the base at that mass first, then R's hierarchy derived from it
        CachedH* base = has_ref(R) && R->m0 != R->ref ? base_for(S, R) : nullptr;
        const bool started = base ? dispatch_derive(S, R, base)
                                  : dispatch_build(S, R, has_ref(R) ? R->ref : R->m0);
        if (started) {
          did = true;
        } else if (S->building.empty() &&
                   std::none_of(S->inst.begin(), S->inst.end(),
                                [](const std::unique_ptr<Instance>& I) { return I->busy(); })) {
          // nothing running or building will free memory: this request cannot be served
          R->status = AMAMG_ERR_OUT_OF_MEMORY;
          finish(S, R);
          it = S->queue.erase(it);
          did = true;
          continue;
        }
      }
      ++it;
      continue;
    }
    Instance* target = nullptr;
    for (const auto& I : S->inst)
      if (I->ch == c && I->free_slots() >= R->nrhs) {
        target = I.get();
        break;
      }
    if (!target) {
      // an idle instance already bound to it, else the idle one used least recently
      Instance* idle = nullptr;
      auto lru = [](const Instance* I) { return I->ch ? I->ch->last_use : uint64_t(0); };
      for (const auto& I : S->inst) {
        if (I->busy()) continue;
        if (I->ch == c) {
          idle = I.get();
          break;
        }
        if (!idle || lru(I.get()) < lru(idle)) idle = I.get();
      }
      // a new instance, or the rebound one, grows its workspace and buffers to the hierarchy's
      // size: that has to fit the budget first
      bool blocked = false;
      c->users += 1;              // make_room must not drop the hierarchy to bind
      if (!idle && int(S->inst.size()) < S->prm.max_instances) {
        if (make_room(S, bind_bytes(S, nullptr, c))) {
          auto I = std::make_unique<Instance>();
          I->id = int(S->inst.size());
          HIPCHECK(hipStreamCreateWithFlags(&I->stream, hipStreamNonBlocking));
          I->slot_req.assign(S->prm.slots, nullptr);
          I->slot_rhs.assign(S->prm.slots, -1);
          S->inst.push_back(std::move(I));
          idle = S->inst.back().get();
        } else {
          blocked = true;
        }
      } else if (idle && idle->ch != c && !make_room(S, bind_bytes(S, idle, c), idle)) {
        idle = nullptr;
        blocked = true;
      }
      c->users -= 1;
      if (idle) {
        bind(S, idle, c);
        target = idle;
      } else if (blocked && S->building.empty() &&
                 std::none_of(S->inst.begin(), S->inst.end(),
                              [](const std::unique_ptr<Instance>& I) { return I->busy(); })) {
        // nothing running or building will free memory: this request cannot be served
        R->status = AMAMG_ERR_OUT_OF_MEMORY;
        finish(S, R);
        it = S->queue.erase(it);
        did = true;
        continue;
      }
    }
    if (!target) {
      ++it;
      continue;
    }
    target->reserved.push_back(R);
    c->last_use = ++S->tick;
    if (target->phase == Instance::IDLE) begin_admission(S, target);
    it = S->queue.erase(it);
    did = true;
  }
  account(S);
  return did;
}

bool progress(amamg_server* S) {
  bool did = false;
  for (const auto& I : S->inst) {
    if (I->phase == Instance::IDLE || !I->bt.ready()) continue;
    did = true;
    if (I->phase == Instance::CHECKING) finish_admission(S, I.get());
    else cycle_end(S, I.get());
  }
  return did;
}

// Device failure: every request in flight or queued fails with the error; instances restart
// empty.
void fail_all(amamg_server* S, const Fail& f) {
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->err = f.msg;
  }
  std::vector<Request*> victims(S->queue.begin(), S->queue.end());
  S->queue.clear();
  for (const auto& I : S->inst) {
    (void)hipStreamSynchronize(I->stream);
    for (Request* R : I->reserved) victims.push_back(R);
    I->reserved.clear();
    for (int s = 0; s < int(I->slot_req.size()); ++s)
      if (I->slot_req[s]) {
        if (std::find(victims.begin(), victims.end(), I->slot_req[s]) == victims.end())
          victims.push_back(I->slot_req[s]);
        release_slot(I.get(), s);
      }
    I->checking.clear();
    I->phase = Instance::IDLE;
    if (I->ch) {
      I->ch->users -= 1;
      I->ch = nullptr;
    }
    I->ws.release();
  }
  for (Request* R : victims) {
    R->status = f.code;
    finish(S, R);
  }
}

void worker_main(amamg_server* S) {
  (void)hipSetDevice(S->ctx->device);
  for (;;) {
    bool stopping;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      while (!S->incoming.empty()) {
        S->queue.push_back(S->incoming.front());
        S->incoming.pop_front();
      }
      stopping = S->stop;
    }
    const bool busy = !S->building.empty() ||
                      std::any_of(S->inst.begin(), S->inst.end(),
                                  [](const std::unique_ptr<Instance>& I) { return I->busy(); });
    if (stopping && S->queue.empty() && !busy) break;
    bool did = false;
    try {
      did = collect_builds(S);
      did = progress(S) || did;
      did = place(S) || did;
    } catch (const Fail& f) {
      fail_all(S, f);
      did = true;
    }
    if (did) continue;
    std::unique_lock<std::mutex> lk(S->mu);
    if (!S->incoming.empty() || !S->built.empty() || (S->stop && S->queue.empty() && !busy)) continue;
    if (busy) S->cv_work.wait_for(lk, std::chrono::microseconds(100));
    else S->cv_work.wait(lk, [&] { return !S->incoming.empty() || !S->built.empty() || S->stop; });
  }
}

}  // namespace

// ---------------------------------------------------------------------------------- ABI

extern "C" {

void amamg_server_default_params(amamg_server_params* p) {
  if (!p) return;
  p->slots = 16;
  p->max_instances = 4;
  p->precision = AMAMG_MIXED_FP32;
  p->restart = 20;
  p->max_iters = 10000;
  p->builders = 2;
  p->graphs = 0;
  p->rel_tol = 1e-10;
  p->hbm_budget = 0;
}

amamg_status amamg_server_create(int32_t device, const amamg_server_params* params, amamg_server** out) {
  if (!out) return AMAMG_ERR_INVALID_ARG;
  *out = nullptr;
  amamg_server_params p;
  if (params) p = *params;
  else amamg_server_default_params(&p);
  if (p.slots < 1 || p.slots > 256 || p.max_instances < 1 || p.max_instances > 16 || p.restart < 1 ||
      p.restart > 31 || p.max_iters < 1 || !(p.rel_tol > 0) || !std::isfinite(p.rel_tol) ||
      p.precision < 0 || p.precision > 2 || p.builders < 1 || p.builders > 8)
    return AMAMG_ERR_INVALID_ARG;
  amamg_context* ctx = nullptr;
  const amamg_status st = amamg_context_create(device, nullptr, &ctx);
  if (st != AMAMG_OK) return st;
  if (p.hbm_budget == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      amamg_context_destroy(ctx);
      return AMAMG_ERR_DEVICE;
    }
    p.hbm_budget = fr / 4 * 3;
  }
  amamg_server* S = new amamg_server();
  S->ctx = ctx;
  S->prm = p;
  S->t0 = Clock::now();
  for (int k = 0; k < p.builders; ++k) {
    auto B = std::make_unique<amamg_server::Builder>();
    if (hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking) != hipSuccess) {
      for (auto& b : S->builders) (void)hipStreamDestroy(b->stream);
      amamg_context_destroy(ctx);
      delete S;
      return AMAMG_ERR_DEVICE;
    }
    S->builders.push_back(std::move(B));
  }
  for (auto& B : S->builders) B->th = std::thread(builder_main, S, B.get());
  S->worker = std::thread(worker_main, S);
  *out = S;
  return AMAMG_OK;
}

amamg_status amamg_server_add_gauge(amamg_server* S, int32_t nt, int32_t nx, const double* links,
                                    int32_t* gauge_id) {
  if (!S || !links || !gauge_id) return AMAMG_ERR_INVALID_ARG;
  // a gauge of the server's context; the device copy is made here, on the caller's thread,
  // with a synchronous copy that does not touch the worker's streams
  amamg_gauge* g = new amamg_gauge();
  try {
    REQUIRE(nt >= 4 && nx >= 4 && nt % 2 == 0 && nx % 2 == 0, AMAMG_ERR_UNSUPPORTED_SHAPE,
            "lattice sizes must be even and >= 4");
    REQUIRE(int64_t(nt) * nx <= (int64_t(1) << 28), AMAMG_ERR_UNSUPPORTED_SHAPE, "lattice too large");
    const size_t nval = size_t(2) * nt * nx * 2;
    REQUIRE(finite_all(links, nval), AMAMG_ERR_NONFINITE, "non-finite link");
    HIPCHECK(hipSetDevice(S->ctx->device));
    g->ctx = S->ctx;
    g->nt = nt;
    g->nx = nx;
    g->U = g->mem.alloc<double2>(size_t(2) * nt * nx);
    HIPCHECK(hipMemcpy(g->U, links, sizeof(double) * nval, hipMemcpyHostToDevice));
  } catch (const Fail& f) {
    delete g;
    std::lock_guard<std::mutex> lk(S->mu);
    S->err = f.msg;
    return f.code;
  }
  std::lock_guard<std::mutex> lk(S->mu);
  S->gauges.push_back(g);
  S->refs.push_back(NAN);
  *gauge_id = int32_t(S->gauges.size()) - 1;
  return AMAMG_OK;
}

amamg_status amamg_server_set_reference_mass(amamg_server* S, int32_t gauge_id, double m_ref) {
  if (!S) return AMAMG_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  if (gauge_id < 0 || gauge_id >= int(S->gauges.size()) || std::isinf(m_ref)) {
    S->err = "unknown gauge or infinite reference mass";
    return AMAMG_ERR_INVALID_ARG;
  }
  S->refs[gauge_id] = m_ref;
  return AMAMG_OK;
}

amamg_status amamg_server_submit(amamg_server* S, int32_t gauge_id, double m0,
                                 const amamg_setup_params* setup, int32_t nrhs, const double* psi,
                                 double* x, uint64_t* request_id) {
  if (!S || !psi || !x || !request_id) return AMAMG_ERR_INVALID_ARG;
  auto R = std::make_unique<Request>();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (gauge_id < 0 || gauge_id >= int(S->gauges.size()) || nrhs < 1 || nrhs > S->prm.slots ||
        !std::isfinite(m0) || S->stop) {
      S->err = "bad request: unknown gauge, nrhs outside [1, slots], non-finite mass or stopped server";
      return AMAMG_ERR_INVALID_ARG;
    }
    const amamg_gauge* g = S->gauges[gauge_id];
    R->psi.assign(psi, psi + size_t(nrhs) * g->nt * g->nx * 4);
    R->ref = S->refs[gauge_id];
  }
  R->gauge = gauge_id;
  R->m0 = m0;
  if (setup) R->sp = *setup;
  else amamg_default_setup_params(&R->sp);
  R->nrhs = nrhs;
  R->x = x;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    try {
      const amamg_gauge* g = S->gauges[gauge_id];
      (void)setup_bytes(g->nt, g->nx, R->sp);     // validates the setup parameters and shape
    } catch (const Fail& f) {
      S->err = f.msg;
      return f.code;
    }
    R->id = S->next_id++;
    R->t_submit = S->now();
    *request_id = R->id;
    S->outstanding += 1;
    S->incoming.push_back(R.release());
  }
  S->cv_work.notify_one();
  return AMAMG_OK;
}

amamg_status amamg_server_poll(amamg_server* S, amamg_request_info* out, int32_t capacity,
                               int32_t* n_written) {
  if (!S || (!out && capacity > 0) || !n_written) return AMAMG_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  int k = 0;
  while (k < capacity && !S->done.empty()) {
    Request* R = S->done.front();
    S->done.pop_front();
    amamg_request_info& o = out[k++];
    o.id = R->id;
    o.status = R->status;
    o.nrhs = R->nrhs;
    o.iterations = R->iterations;
    o.converged = R->converged;
    o.true_rel_residual = R->residual;
    o.t_submit = R->t_submit;
    o.t_admit = R->t_admit;
    o.t_done = R->t_done;
    o.instance = R->instance;
    o.hierarchy_built = R->built;
    delete R;
  }
  *n_written = k;
  return AMAMG_OK;
}

amamg_status amamg_server_wait(amamg_server* S, double timeout_s) {
  if (!S) return AMAMG_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(S->mu);
  const bool ok = S->cv_done.wait_for(lk, std::chrono::duration<double>(std::max(0.0, timeout_s)),
                                      [&] { return S->outstanding == 0; });
  return ok ? AMAMG_OK : AMAMG_PENDING;
}

amamg_status amamg_server_stats(amamg_server* S, amamg_server_counters* out) {
  if (!S || !out) return AMAMG_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  out->setups = S->setups;
  out->evictions = S->evictions;
  out->resident_bytes = S->resident;
  out->hierarchy_bytes = S->hier_bytes;
  out->peak_resident_bytes = S->peak_resident;
  out->budget_bytes = S->prm.hbm_budget;
  out->outstanding = S->outstanding;
  out->clock = S->now();
  out->last_estimate_bytes = S->last_estimate;
  out->setup_seconds = S->setup_seconds;
  out->setup_seconds_max = S->setup_seconds_max;
  out->derivations = S->derivations;
  out->derive_seconds = S->derive_seconds;
  out->derive_seconds_max = S->derive_seconds_max;
  return AMAMG_OK;
}

const char* amamg_server_last_error(amamg_server* S) {
  if (!S) return "null server";
  std::lock_guard<std::mutex> lk(S->mu);
  return S->err.c_str();
}

amamg_status amamg_server_destroy(amamg_server* S) {
  if (!S) return AMAMG_ERR_INVALID_ARG;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  S->worker.join();          // drains every submitted request first
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop_builder = true;
  }
  S->cv_build.notify_all();
  for (auto& B : S->builders) B->th.join();
  for (BuildJob& j : S->built)
    if (j.h) delete j.h;
  S->built.clear();
  for (auto& B : S->builders) (void)hipStreamDestroy(B->stream);
  S->builders.clear();         // frees the builders' scratch pools
  for (auto& I : S->inst) {
    (void)hipStreamSynchronize(I->stream);
    I->ws.release();
    I->io.release();
    (void)hipStreamDestroy(I->stream);
  }
  S->inst.clear();
  for (auto& c : S->cache) {     // derived hierarchies own nothing of their base
    c->h->gauge->nhier -= 1;
    delete c->h;
  }
  S->cache.clear();
  for (Request* R : S->done) delete R;
  for (amamg_gauge* g : S->gauges) delete g;
  amamg_context_destroy(S->ctx);
  delete S;
  return AMAMG_OK;
}

}  // extern "C"
