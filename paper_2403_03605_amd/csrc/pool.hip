// Serving pool: many independent fracture solves resident in HBM at once,
// admitted against a device-memory budget and advanced together.
//
// Every pool step is one macro step (Algorithm 1) of every active request:
//  phase A  FE free steps (per request, on side streams), the PD substeps of all requests as
//           one batched launch per substep index j (requests sorted by step
//           ratio m, so substep j covers a prefix of them), then each coupled
//           request saves its bond states and takes its rebuild flag;
//  host     the rebuild checks of the previous pool step are resolved (the
//           same one-step-behind pipeline as a single solver, so results are
//           identical to running the request alone);
//  phase B  multiplier solves and final updates (per request, spread over
//           four side streams forked from and joined into the pool stream).
// While the set of active requests is unchanged, phases A and B are replayed
// from HIP graphs, one per phase and parity of the pool step (every per-step
// alternation of a request -- displacement buffer, state snapshot slot -- has
// period two).  Requests join and leave between pool steps: a request created
// (on a caller's thread, on a separate stream) while others run is admitted at
// the next step, and a finished request leaves the set at once.  Several
// requests may be built at once, each on a stream of its own.
#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "internal.h"

namespace mts {
namespace {



struct Req {
  uint64_t id = 0;
  Solver *s = nullptr;
  int64_t n_macro = 0, done = 0;
  int state = MTS_REQ_ACTIVE;
  int64_t charged = 0;
  bool tracked = false;
  bool pending = false;
  int pending_slot = 0;
  hipEvent_t done_ev = nullptr;
  bool read_ready = false;
};

void destroy_solver(Solver *s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  for (hipEvent_t e : s->flag_event)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : s->ev_pool) (void)hipEventDestroy(e);
  if (s->nf_event) (void)hipEventDestroy(s->nf_event);
  coupling_free(*s);
  fe_implicit_free(*s);
  pd_implicit_free(*s);
  if (s->pinned_flag) (void)hipHostFree(s->pinned_flag);
  s->arena.free_all();
  delete s;
}

}  // namespace
}  // namespace mts

using namespace mts;

struct mts_pool {
  hipStream_t stream = nullptr;   // pool steps
  hipStream_t read_st = nullptr;  // reads of finished requests
  bool own_stream = false;
  int dim = 2, precision = MTS_MIXED, lanes = 4;
  bool graphs = true;
  int64_t budget = 0, used = 0;
  int max_slots = 1;
  int creating = 0;       // requests under construction on other threads
  bool capturing = false;  // a graph capture is open on `stream`
  int64_t n_running = 0;   // active + ready (guarded by mu)
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Req *> ready;
  std::vector<Req *> active;
  std::unordered_map<uint64_t, Req *> reqs;
  uint64_t next_id = 1;
  // batched substep tables, per parity: [j - 1][request]
  void *tab[2] = {nullptr, nullptr};
  int32_t *blk_req = nullptr;
  size_t tab_bytes = 0, blk_cap = 0;
  std::vector<int64_t> grid_j;  // blocks of the launch of substep j (index j - 1)
  int max_m = 0;
  bool dirty = true;
  int stable = 0;
  hipGraphExec_t gexec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // [phase][parity]
  // per-request work (FE steps, multiplier solves) spread over side streams
  static constexpr int kSide = 4;
  hipStream_t side[kSide] = {};
  hipEvent_t fork_ev[2] = {}, join_ev[2][kSide] = {};
  hipEvent_t ev_a[2] = {nullptr, nullptr};
  int64_t ticks = 0, captures = 0, replays = 0;
};

namespace {

void drop_graphs(mts_pool *P) {
  for (auto &ph : P->gexec)
    for (auto &g : ph)
      if (g) {
        (void)hipGraphExecDestroy(g);
        g = nullptr;
      }
}

// Rebuild the batch tables for the current active set (stream drained first).
void rebuild_tables(mts_pool *P) {
  MTS_HIP(hipStreamSynchronize(P->stream));
  drop_graphs(P);
  std::stable_sort(P->active.begin(), P->active.end(), [](const Req *a, const Req *b) { return a->s->m > b->s->m; });
  const size_t n = P->active.size();
  P->max_m = 0;
  std::vector<int32_t> first(n);
  std::vector<int32_t> blk;
  for (size_t r = 0; r < n; r++) {
    Solver &s = *P->active[r]->s;
    P->max_m = std::max(P->max_m, s.m);
    first[r] = (int32_t)blk.size();
    const int64_t b = substep_blocks(s);
    for (int64_t q = 0; q < b; q++) blk.push_back((int32_t)r);
  }
  P->grid_j.assign(P->max_m, 0);
  for (int j = 1; j <= P->max_m; j++) {
    int64_t g = 0;
    for (size_t r = 0; r < n; r++)
      if (P->active[r]->s->m >= j) g = first[r] + substep_blocks(*P->active[r]->s);
    P->grid_j[j - 1] = g;
  }
  const size_t esz = substep_entry_size();
  const size_t need = esz * (size_t)std::max(P->max_m, 1) * std::max<size_t>(n, 1);
  if (need > P->tab_bytes) {
    for (auto &t : P->tab)
      if (t) (void)hipFree(t);
    for (auto &t : P->tab) MTS_HIP(hipMalloc(&t, need));
    P->tab_bytes = need;
  }
  if (blk.size() > P->blk_cap) {
    if (P->blk_req) (void)hipFree(P->blk_req);
    MTS_HIP(hipMalloc((void **)&P->blk_req, sizeof(int32_t) * blk.size()));
    P->blk_cap = blk.size();
  }
  if (!blk.empty())
    MTS_HIP(hipMemcpyAsync(P->blk_req, blk.data(), sizeof(int32_t) * blk.size(), hipMemcpyHostToDevice, P->stream));
  std::vector<unsigned char> host(need);
  const int par = (int)(P->ticks & 1);
  for (int p = 0; p < 2; p++) {
    std::fill(host.begin(), host.end(), 0);
    for (size_t r = 0; r < n; r++) {
      Solver &s = *P->active[r]->s;
      // displacement buffer at the start of a pool step of parity p
      const int cur0 = (p == par) ? s.cur : (s.cur ^ (s.m & 1));
      int cur = cur0;
      for (int j = 1; j <= s.m; j++) {
        substep_entry_fill(s, j, cur, first[r], host.data() + esz * ((size_t)(j - 1) * n + r));
        cur ^= 1;
      }
    }
    MTS_HIP(hipMemcpyAsync(P->tab[p], host.data(), need, hipMemcpyHostToDevice, P->stream));
    MTS_HIP(hipStreamSynchronize(P->stream));  // host buffers are reused / freed
  }
  P->dirty = false;
  P->stable = 0;
}

// Run fn(solver) for every running request, request k on side stream k % kSide,
// between a fork from and a join into the pool stream (recorded in a capture
// too, where it becomes parallel graph branches).
template <class Fn>
void on_side_streams(mts_pool *P, int phase, Fn fn) {
  MTS_HIP(hipEventRecord(P->fork_ev[phase], P->stream));
  for (auto st : P->side) MTS_HIP(hipStreamWaitEvent(st, P->fork_ev[phase], 0));
  size_t k = 0;
  for (Req *r : P->active) {
    Solver &s = *r->s;
    s.stream = P->side[k++ % mts_pool::kSide];
    try {
      fn(s);
    } catch (...) {
      s.stream = P->stream;
      throw;
    }
    s.stream = P->stream;
  }
  for (int q = 0; q < mts_pool::kSide; q++) {
    MTS_HIP(hipEventRecord(P->join_ev[phase][q], P->side[q]));
    MTS_HIP(hipStreamWaitEvent(P->stream, P->join_ev[phase][q], 0));
  }
}

void enqueue_phase_a(mts_pool *P, int par) {
  const size_t n = P->active.size();
  on_side_streams(P, 0, [](Solver &s) {
    if (s.p.mode == MTS_COUPLED) fe_free_step(s);
  });
  const size_t esz = substep_entry_size();
  for (int j = 1; j <= P->max_m; j++) {
    const void *tab = static_cast<const unsigned char *>(P->tab[par]) + esz * (size_t)(j - 1) * n;
    substep_batch_launch(P->dim, P->precision == MTS_MIXED, P->lanes, tab, P->blk_req, P->grid_j[j - 1], P->stream);
  }
  for (Req *r : P->active) {
    if (!r->tracked) continue;
    Solver &s = *r->s;
    snapshot_states(s, (int)(s.macro_steps & 1));  // on s.stream == the pool stream
  }
}

void enqueue_phase_b(mts_pool *P) {
  on_side_streams(P, 1, [](Solver &s) {
    if (s.p.mode == MTS_COUPLED) coupling_solve_and_correct(s);
  });
}

// Capture one phase into a graph.  No request is constructed on another thread
// while a capture is open (construction allocates and frees device memory).
bool capture_phase(mts_pool *P, int phase, int par) {
  {
    std::lock_guard<std::mutex> lk(P->mu);
    if (P->creating > 0) return false;
    P->capturing = true;
  }
  struct Done {
    mts_pool *P;
    ~Done() {
      {
        std::lock_guard<std::mutex> lk(P->mu);
        P->capturing = false;
      }
      P->cv.notify_all();
    }
  } done{P};
  hipGraph_t g = nullptr;
  MTS_HIP(hipStreamBeginCapture(P->stream, hipStreamCaptureModeRelaxed));
  try {
    if (phase == 0) enqueue_phase_a(P, par);
    else enqueue_phase_b(P);
  } catch (...) {
    (void)hipStreamEndCapture(P->stream, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  MTS_HIP(hipStreamEndCapture(P->stream, &g));
  hipGraphExec_t ex = nullptr;
  const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  MTS_HIP(e);
  P->gexec[phase][par] = ex;
  P->captures++;
  return true;
}

void run_phase(mts_pool *P, int phase, int par) {
  bool use_graph = P->graphs && P->stable >= 2;
  if (use_graph && !P->gexec[phase][par]) use_graph = capture_phase(P, phase, par);
  if (use_graph) {
    MTS_HIP(hipGraphLaunch(P->gexec[phase][par], P->stream));
    P->replays++;
  } else if (phase == 0) {
    enqueue_phase_a(P, par);
  } else {
    enqueue_phase_b(P);
  }
}

void step_impl(mts_pool *P, uint64_t *done_ids, int32_t cap, int32_t *n_done) {
  int32_t nd = 0;
  {
    std::lock_guard<std::mutex> lk(P->mu);
    while (!P->ready.empty()) {
      Req *r = P->ready.front();
      P->ready.pop_front();
      r->s->stream = P->stream;
      P->active.push_back(r);
      P->dirty = true;
    }
  }
  if (P->active.empty()) {
    if (n_done) *n_done = 0;
    return;
  }
  if (P->dirty) rebuild_tables(P);
  const int par = (int)(P->ticks & 1);
  run_phase(P, 0, par);
  MTS_HIP(hipEventRecord(P->ev_a[par], P->stream));
  // rebuild checks of the previous pool step
  bool waited = false;
  for (Req *r : P->active) {
    if (!r->pending) continue;
    if (!waited) {
      MTS_HIP(hipEventSynchronize(P->ev_a[par ^ 1]));
      waited = true;
    }
    r->pending = false;
    Solver &s = *r->s;
    if (s.pinned_flag[r->pending_slot]) {
      s.pinned_flag[r->pending_slot] = 0;
      coupling_rebuild(s, s.mask_snap[r->pending_slot]);
      s.n_rebuilds++;
    }
  }
  // displacement buffers after this step's substeps (phase B reads them)
  for (Req *r : P->active) {
    Solver &s = *r->s;
    s.cur ^= (s.m & 1);
    s.pd_steps += s.m;
  }
  run_phase(P, 1, par);
  std::vector<Req *> keep;
  keep.reserve(P->active.size());
  for (Req *r : P->active) {
    Solver &s = *r->s;
    if (r->tracked) {
      r->pending = true;
      r->pending_slot = (int)(s.macro_steps & 1);
    }
    s.macro_steps++;
    r->done++;
    if (r->done >= r->n_macro) {
      MTS_HIP(hipEventRecord(r->done_ev, P->stream));
      r->pending = false;
      std::lock_guard<std::mutex> lk(P->mu);
      r->state = MTS_REQ_DONE;
      P->n_running--;
      if (done_ids && nd < cap) done_ids[nd] = r->id;
      nd++;
      P->dirty = true;
    } else {
      keep.push_back(r);
    }
  }
  P->active.swap(keep);
  P->ticks++;
  if (!P->dirty) P->stable++;
  if (n_done) *n_done = nd;
}

Req *find_req(mts_pool *P, uint64_t id) {
  std::lock_guard<std::mutex> lk(P->mu);
  auto it = P->reqs.find(id);
  return it == P->reqs.end() ? nullptr : it->second;
}

}  // namespace

extern "C" {

mts_status mts_pool_create(int64_t budget_bytes, int32_t max_slots, int32_t dim, int32_t precision,
                           int32_t use_graphs, void *hip_stream, mts_pool **out) {
  if (!out) return (set_error("null output pointer"), MTS_EINVAL);
  *out = nullptr;
  if (budget_bytes <= 0 || max_slots < 1 || (dim != 2 && dim != 3) ||
      (precision != MTS_FP64 && precision != MTS_MIXED))
    return (set_error("bad pool arguments"), MTS_EINVAL);
  mts_pool *P = nullptr;
  try {
    P = new mts_pool();
    P->budget = budget_bytes;
    P->max_slots = max_slots;
    P->dim = dim;
    P->precision = precision;
    P->graphs = use_graphs != 0;
    P->lanes = 4;
    P->stream = (hipStream_t)hip_stream;
    if (!P->stream) {  // graphs cannot be captured on the null stream: use a stream of the pool's own
      MTS_HIP(hipStreamCreateWithFlags(&P->stream, hipStreamNonBlocking));
      P->own_stream = true;
    }
    MTS_HIP(hipStreamCreateWithFlags(&P->read_st, hipStreamNonBlocking));
    for (auto &e : P->ev_a) MTS_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (auto &st : P->side) MTS_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    for (auto &e : P->fork_ev) MTS_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (auto &ph : P->join_ev)
      for (auto &e : ph) MTS_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    *out = P;
    return MTS_OK;
  } catch (...) {
    mts_status st = fail_from_exception();
    if (P) mts_pool_destroy(P);
    return st;
  }
}

mts_status mts_pool_submit(mts_pool *P, const mts_problem *p, int64_t n_macro, uint64_t *id) {
  if (!P || !p || !id) return (set_error("null argument"), MTS_EINVAL);
  if (n_macro < 1) return (set_error("n_macro must be >= 1"), MTS_EINVAL);
  if (p->dim != P->dim || p->precision != P->precision)
    return (set_error("request dim/precision differ from the pool's"), MTS_EINVAL);
  if (p->fe_beta != 0.0) return (set_error("the pool runs the explicit FE step only (fe_beta = 0)"), MTS_EINVAL);
  if (p->pd_beta != 0.0) return (set_error("the pool runs the explicit PD step only (pd_beta = 0)"), MTS_EINVAL);
  if (p->traction_x != 0.0 || p->clamp_x0)
    return (set_error("the pool serves y-face tractions and the x-velocity load only"), MTS_EINVAL);
  mts_plan_info plan{};
  const mts_status pst = mts_plan(p, &plan);
  if (pst != MTS_OK) return pst;
  const int64_t est = plan.device_bytes_estimate;
  {
    std::unique_lock<std::mutex> lk(P->mu);
    if (est > P->budget) {
      set_error("request needs about %lld bytes, budget is %lld", (long long)est, (long long)P->budget);
      return MTS_ETOOBIG;
    }
    P->cv.wait(lk, [P] { return !P->capturing; });
    const int64_t slots = P->n_running + P->creating;
    if (slots >= P->max_slots || P->used + est > P->budget) {
      set_error("pool full");
      return MTS_EAGAIN;
    }
    P->used += est;
    P->creating++;
  }
  Req *r = new Req();
  r->n_macro = n_macro;
  r->charged = est;
  hipStream_t st = nullptr;  // per call, so that concurrent submits build in parallel
  try {
    MTS_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    r->s = new Solver();
    r->s->force_lanes = P->lanes;
    r->s->halo = false;  // one batched kernel for every request: neighbour gathers from global memory
    r->s->tiled = 0;
    // one build stream per request (its colour batches in sequence): with
    // four per request, a 256-request stream built on four threads ended in a
    // host segmentation fault whose cause was not found
    r->s->build_streams = 1;
    create_impl(p, st, r->s);  // ends with a synchronisation of st
    r->s->stream = P->stream;
    MTS_HIP(hipStreamDestroy(st));
    st = nullptr;
    MTS_HIP(hipEventCreateWithFlags(&r->done_ev, hipEventDisableTiming));
    r->tracked = p->mode == MTS_COUPLED && p->m >= 2;
  } catch (...) {
    const mts_status err = fail_from_exception();
    if (st) {
      (void)hipStreamSynchronize(st);
      if (r->s) r->s->stream = P->stream;
      (void)hipStreamDestroy(st);
    }
    destroy_solver(r->s);
    delete r;
    std::lock_guard<std::mutex> lk(P->mu);
    P->used -= est;
    P->creating--;
    P->cv.notify_all();
    return err;
  }
  std::lock_guard<std::mutex> lk(P->mu);
  const int64_t actual = (int64_t)r->s->arena.live;
  P->used += actual - est;
  r->charged = actual;
  P->creating--;
  r->id = P->next_id++;
  P->reqs[r->id] = r;
  P->ready.push_back(r);
  P->n_running++;
  *id = r->id;
  return MTS_OK;
}

mts_status mts_pool_step(mts_pool *P, int32_t *n_active, uint64_t *host_done_ids, int32_t cap, int32_t *n_done) {
  if (!P) return (set_error("null pool"), MTS_EINVAL);
  try {
    step_impl(P, host_done_ids, cap, n_done);
    if (n_active) *n_active = (int32_t)P->active.size();
    return MTS_OK;
  } catch (...) {
    return fail_from_exception();
  }
}

mts_status mts_pool_poll(mts_pool *P, uint64_t id, int32_t *state, int64_t *macro_done, mts_info *info) {
  if (!P) return (set_error("null pool"), MTS_EINVAL);
  Req *r = find_req(P, id);
  if (!r) return (set_error("unknown request id"), MTS_EINVAL);
  std::lock_guard<std::mutex> lk(P->mu);
  if (state) *state = r->state;
  if (macro_done) *macro_done = r->done;
  if (info) query_impl(*r->s, info);
  return MTS_OK;
}

mts_status mts_pool_read(mts_pool *P, uint64_t id, int32_t what, double *host_out, int64_t cap, int64_t *n) {
  if (!P || !host_out) return (set_error("null argument"), MTS_EINVAL);
  Req *r = find_req(P, id);
  if (!r) return (set_error("unknown request id"), MTS_EINVAL);
  if (r->state != MTS_REQ_DONE) return (set_error("request not finished"), MTS_ESTATE);
  try {
    if (!r->read_ready) {
      MTS_HIP(hipStreamWaitEvent(P->read_st, r->done_ev, 0));
      r->s->stream = P->read_st;
      r->read_ready = true;
    }
    return read_impl(*r->s, what, host_out, cap, n);
  } catch (...) {
    return fail_from_exception();
  }
}

mts_status mts_pool_release(mts_pool *P, uint64_t id) {
  if (!P) return (set_error("null pool"), MTS_EINVAL);
  Req *r = find_req(P, id);
  if (!r) return (set_error("unknown request id"), MTS_EINVAL);
  if (r->state != MTS_REQ_DONE) return (set_error("request not finished"), MTS_ESTATE);
  try {
    MTS_HIP(hipEventSynchronize(r->done_ev));
    (void)hipEventDestroy(r->done_ev);
    destroy_solver(r->s);
    std::lock_guard<std::mutex> lk(P->mu);
    P->used -= r->charged;
    P->reqs.erase(id);
    delete r;
    return MTS_OK;
  } catch (...) {
    return fail_from_exception();
  }
}

mts_status mts_pool_query(mts_pool *P, mts_pool_info *o) {
  if (!P || !o) return (set_error("null argument"), MTS_EINVAL);
  std::lock_guard<std::mutex> lk(P->mu);
  std::memset(o, 0, sizeof *o);
  o->budget_bytes = P->budget;
  o->used_bytes = P->used;
  o->n_running = (int32_t)P->n_running;
  o->n_ready = (int32_t)P->ready.size();
  o->max_slots = P->max_slots;
  o->lanes = P->lanes;
  o->ticks = P->ticks;
  o->graph_captures = P->captures;
  o->graph_replays = P->replays;
  return MTS_OK;
}

void mts_pool_destroy(mts_pool *P) {
  if (!P) return;
  if (P->stream) (void)hipStreamSynchronize(P->stream);
  drop_graphs(P);
  for (auto &kv : P->reqs) {
    Req *r = kv.second;
    if (r->done_ev) (void)hipEventDestroy(r->done_ev);
    destroy_solver(r->s);
    delete r;
  }
  for (auto &t : P->tab)
    if (t) (void)hipFree(t);
  if (P->blk_req) (void)hipFree(P->blk_req);
  for (auto &e : P->ev_a)
    if (e) (void)hipEventDestroy(e);
  for (auto &st : P->side)
    if (st) {
      (void)hipStreamSynchronize(st);
      (void)hipStreamDestroy(st);
    }
  for (auto &e : P->fork_ev)
    if (e) (void)hipEventDestroy(e);
  for (auto &ph : P->join_ev)
    for (auto &e : ph)
      if (e) (void)hipEventDestroy(e);
  if (P->own_stream) (void)hipStreamDestroy(P->stream);
  if (P->read_st) (void)hipStreamDestroy(P->read_st);
  delete P;
}

}  // extern "C"
