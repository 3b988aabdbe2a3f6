// Serving core: continuous batching of distance queries on one context.
//
// A worker thread repeats one device step while queries are queued or in
// flight:
//   1. admission: queued queries take free slots while the shared traversal
//      storage has room (the live entries after the last step fill less than
//      half of the spill stack) and the adaptive concurrency limit allows;
//      each new slot gets its descriptor, the refit of its moving tree, its
//      error window, greedy dive and root pair (through the admission segment);
//   2. traversal: the persistent kernel runs at most rounds_per_step rounds of
//      every slot in flight (new slots join the running fronts);
//   3. a per-slot histogram of the live front and leaf-pair entries;
//   4. every in-flight slot with no live entries is complete: the device flags
//      it, re-evaluates its candidates in FP64 and takes it out of flight;
//   5. one copy of the step's report (outcome, live counts, completion flags,
//      results) to pinned host memory, then one host wait; completed results
//      are queued for polling and their slots freed.
// Steps 2-5 have a fixed shape: they are built once as a HIP graph (the
// traversal as a cooperative kernel node, the rest captured from the stream)
// and replayed every step; the round index that selects the buffer parity
// lives on the device, so the replayed launches need no new arguments.  The
// graph is rebuilt when the spill stack grows.
// A spill-stack overflow puts every query in flight back at the head of the
// queue (keeping its submit time), clears the traversal storage and halves the
// concurrency limit; when a query overflows alone the stack doubles (up to
// 2^31 entries) before it runs again.  A query whose candidate region fills
// up (or that overflows the largest stack alone) is re-run by itself through
// the batched query path, whose storage grows as far as device memory allows;
// the other queries are not affected.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "host.hpp"

using namespace gd;

namespace {

constexpr uint64_t kServerCapLimit = 1ull << 28;  // entries per front / leaf-pair buffer

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Pending {
  gdist_query_desc_t q;
  uint64_t tag;
  uint64_t t_submit;
};

}  // namespace

struct gdist_server {
  gdist_ctx* c = nullptr;
  gdist_server_config_t cfg{};
  uint32_t S = 0, nb = 0, seg_f = 0, seg_l = 0, cps = 0;
  uint64_t stack_cap = 0;
  size_t box_stride = 0;  // floats of refitted boxes per slot
  uint32_t max_leaves = 0;
  DevBuf desc, st, boxes, front[2], leaf[2], stack, counts, cand, cand64, ctl, list, tab;
  DevBuf desc_stage;          // the descriptors admitted by a step, in list order
  DevBuf rep;                 // step report: StepHead, live[S], finish[S], results[S]
  size_t live_off = 0, fin_off = 0, res_off = 0, rep_bytes = 0;
  void* rep_host = nullptr;   // pinned copy of the report
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipGraphExec_t gexec[2] = {nullptr, nullptr};   // short steps, long steps
  TravParams gp{};            // the step parameters the graph (or the direct mode) was set up for
  bool gp_set = false;
  uint32_t graph_mode = 0;
  // slot table (worker thread only)
  std::vector<uint8_t> active;
  uint32_t fallbacks = 0;
  std::vector<Pending> slot_req;
  std::vector<uint32_t> free_slots;
  uint32_t n_active = 0, concurrency = 0, clean_steps = 0;
  uint64_t live_total = 0;
  // shared with the API threads
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Pending> pending;
  std::vector<gdist_completion_t> done;
  gdist_server_stats_t stats{};
  std::atomic<bool> stopping{false};
  std::thread worker;
};

namespace {

TravParams params(gdist_server* sv) {
  TravParams p;
  std::memset(&p, 0, sizeof(p));
  gdist_ctx* c = sv->c;
  p.stats = c->stats;
  p.cand_buf = c->cand_buf;
  p.desc = (const SlotDesc*)sv->desc.p;
  p.st = (SlotState*)sv->st.p;
  p.res = (gdist_result_t*)((char*)sv->rep.p + sv->res_off);
  p.front[0] = (uint4*)sv->front[0].p;
  p.front[1] = (uint4*)sv->front[1].p;
  p.leaf[0] = (uint4*)sv->leaf[0].p;
  p.leaf[1] = (uint4*)sv->leaf[1].p;
  uint32_t* cnt = (uint32_t*)sv->counts.p;
  p.fcount[0] = cnt;
  p.fcount[1] = cnt + (sv->nb + 1);
  p.lcount[0] = cnt + 2 * (sv->nb + 1);
  p.lcount[1] = cnt + 3 * (sv->nb + 1);
  p.stack = (uint4*)sv->stack.p;
  p.stack_cap = (uint32_t)sv->stack_cap;
  p.round_cap = round_cap_for(sv->seg_f < sv->seg_l ? sv->seg_f : sv->seg_l, sv->nb);
  p.cand = (Cand*)sv->cand.p;
  p.cand_d64 = (double*)sv->cand64.p;
  p.ctl = (Ctl*)sv->ctl.p;
  p.slot_list = (const uint32_t*)sv->list.p;
  p.seg_front = sv->seg_f;
  p.seg_leaf = sv->seg_l;
  p.cand_per_slot = sv->cps;
  p.nblocks = sv->nb;
  p.n_slots = sv->S;
  p.expand_budget = c->expand_budget;
  p.k_cap = c->k_cap;
  p.spin_limit = 1u << 26;
  p.round0 = 0;   // the device keeps the round base across steps
  p.max_rounds = sv->cfg.rounds_per_step;
  p.cand_stop = 0;
  return p;
}

// Pinned staging: descriptors, then a slot list, then the refit job tables.
size_t tab_offset(const gdist_server* sv) {
  return (sizeof(SlotDesc) * sv->S + 4ull * sv->S + 255) & ~(size_t)255;
}

// Double the spill stack (all queries are out of flight).
gdist_status_t grow_storage(gdist_server* sv) {
  if (2 * sv->stack_cap > kStackLimit) return GDIST_E_CAPACITY;
  sv->stack_cap *= 2;
  return ensure(sv->c, sv->stack, 16ull * sv->stack_cap);
}

void complete(gdist_server* sv, uint64_t tag, uint64_t t_submit, const gdist_result_t& r) {
  gdist_completion_t cpl;
  std::memset(&cpl, 0, sizeof(cpl));
  cpl.tag = tag;
  cpl.t_submit_ns = t_submit;
  cpl.t_done_ns = now_ns();
  cpl.result = r;
  std::lock_guard<std::mutex> g(sv->mu);
  sv->done.push_back(cpl);
  sv->stats.completed++;
  if (r.status != GDIST_OK) sv->stats.failed++;
}

// Re-run one query alone through the batched path (the server's stream is
// idle: the worker calls this between steps).
void run_alone(gdist_server* sv, const Pending& rq) {
  gdist_result_t r;
  std::memset(&r, 0, sizeof(r));
  gdist_status_t s = run_queries(sv->c, 1, &rq.q, &r);
  if (s != GDIST_OK) {
    std::memset(&r, 0, sizeof(r));
    r.status = (uint32_t)s;
    r.distance = __builtin_nan("");
  }
  {
    std::lock_guard<std::mutex> g(sv->mu);
    sv->fallbacks++;
  }
  complete(sv, rq.tag, rq.t_submit, r);
}

gdist_result_t failed_result(gdist_status_t s) {
  gdist_result_t r;
  std::memset(&r, 0, sizeof(r));
  r.status = (uint32_t)s;
  r.distance = __builtin_nan("");
  return r;
}

// Reset the traversal storage (counts of the current round's buffers, control block).
gdist_status_t reset_storage(gdist_server* sv) {
  TravParams p = params(sv);
  HIPCHK(launch_reset(p, sv->c->stream));
  return GDIST_OK;
}

// Admit the queries of `reqs` into free slots (refit, dive, root pairs).
// Steps 3-5 of a device step on the context's stream.
hipError_t enqueue_tail(gdist_server* sv, const TravParams& p) {
  char* rep = (char*)sv->rep.p;
  hipStream_t s = sv->c->stream;
  hipError_t e = launch_step_tail(p, (StepHead*)rep, (uint32_t*)(rep + sv->live_off), (uint32_t*)(rep + sv->fin_off), s);
  if (e == hipSuccess) e = hipMemcpyAsync(sv->rep_host, rep, sv->rep_bytes, hipMemcpyDeviceToHost, s);
  return e;
}

// Steps 2-5 launched one by one.
hipError_t enqueue_step(gdist_server* sv, const TravParams& p) {
  gdist_ctx* c = sv->c;
  hipError_t e = launch_traverse(p, c->trav_blocks, c->trav_threads, c->stream);
  return e == hipSuccess ? enqueue_tail(sv, p) : e;
}

void drop_graph(gdist_server* sv) {
  for (hipGraphExec_t& g : sv->gexec) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
  sv->graph_mode = 0;
}

// A step runs at most rounds_per_step rounds while queries wait to be
// admitted; with nobody waiting it runs up to kLongRounds, so a lone query
// usually completes within one step (the launch still ends as soon as every
// traversal has drained).
constexpr uint32_t kLongRounds = 64;
TravParams step_params(const TravParams& p, bool lng) {
  TravParams q = p;
  if (lng && q.max_rounds < kLongRounds) q.max_rounds = kLongRounds;
  return q;
}

// Build the step graph for parameters p: a cooperative kernel node for the
// traversal, then the captured tail as a child graph (7 nodes: 6 kernels and
// the report copy).  If the runtime refuses any part, the server launches the
// step's kernels one by one instead (graph_mode 0).
void build_graph(gdist_server* sv, const TravParams& p) {
  gdist_ctx* c = sv->c;
  drop_graph(sv);
  sv->gp = p;
  sv->gp_set = true;
  if (sv->cfg.flags & GDIST_SERVER_DIRECT) return;
  hipError_t e = hipSuccess;
  for (int i = 0; i < 2 && e == hipSuccess; ++i) {
    const TravParams q = step_params(p, i == 1);
    hipGraph_t g = nullptr, tail = nullptr;
    hipGraphNode_t tn = nullptr, cn = nullptr;
    e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t e1 = enqueue_tail(sv, q);
      hipError_t e2 = hipStreamEndCapture(c->stream, &tail);
      e = e1 != hipSuccess ? e1 : e2;
    }
    size_t n_tail = 0;
    if (e == hipSuccess) e = hipGraphGetNodes(tail, nullptr, &n_tail);
    if (e == hipSuccess && n_tail != 7) e = hipErrorInvalidValue;
    if (e == hipSuccess) e = hipGraphCreate(&g, 0);
    if (e == hipSuccess) e = add_traverse_node(g, q, c->trav_blocks, c->trav_threads, &tn);
    if (e == hipSuccess) e = hipGraphAddChildGraphNode(&cn, g, &tn, 1, tail);
    if (e == hipSuccess) e = hipGraphInstantiate(&sv->gexec[i], g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (tail) (void)hipGraphDestroy(tail);
  }
  if (e == hipSuccess) {
    sv->graph_mode = 1;
  } else {
    (void)hipGetLastError();
    drop_graph(sv);
  }
}

gdist_status_t admit(gdist_server* sv, std::vector<Pending>& reqs) {
  gdist_ctx* c = sv->c;
  std::vector<uint32_t> slots;
  std::vector<RefitJob> jobs;
  char* stage = (char*)sv->pinned;
  const size_t desc_off = 0, list_off = sizeof(SlotDesc) * sv->S, tab_off = tab_offset(sv);
  for (Pending& rq : reqs) {
    SlotDesc d;
    Mesh* B = nullptr;
    gdist_status_t s = make_slot(c, rq.q, 0, &d, &B);
    if (s == GDIST_OK && B->L > sv->max_leaves) s = GDIST_E_CAPACITY;
    if (s != GDIST_OK) {
      complete(sv, rq.tag, rq.t_submit, failed_result(s));
      continue;
    }
    uint32_t slot = sv->free_slots.back();
    sv->free_slots.pop_back();
    d.boxB = (const float*)sv->boxes.p + sv->box_stride * slot;
    std::memcpy(stage + desc_off + sizeof(SlotDesc) * slots.size(), &d, sizeof(SlotDesc));
    RefitJob j;
    std::memset(&j, 0, sizeof(j));
    j.tris = B->tris;
    j.boxes = (float*)d.boxB;
    j.T = d.T;
    j.n = B->n_tris;
    j.L = B->L;
    jobs.push_back(j);
    sv->slot_req[slot] = rq;
    sv->active[slot] = 1;
    slots.push_back(slot);
  }
  if (slots.empty()) return GDIST_OK;
  // one copy of the new descriptors (list order) and of the slot list, then
  // a kernel puts each descriptor in its slot
  HIPCHK(hipMemcpyAsync(sv->desc_stage.p, stage + desc_off, sizeof(SlotDesc) * slots.size(), hipMemcpyHostToDevice,
                        c->stream));
  std::memcpy(stage + list_off, slots.data(), 4 * slots.size());
  HIPCHK(hipMemcpyAsync(sv->list.p, stage + list_off, 4 * slots.size(), hipMemcpyHostToDevice, c->stream));
  HIPCHK(launch_put_desc((const SlotDesc*)sv->desc_stage.p, (const uint32_t*)sv->list.p, (uint32_t)slots.size(),
                         (SlotDesc*)sv->desc.p, c->stream));
  RefitPlan plan;
  const size_t cap = sv->pinned_bytes - tab_off;
  const size_t bytes = plan_refit_batch(jobs.data(), (uint32_t)jobs.size(), stage + tab_off, cap, &plan);
  if (bytes == 0 || bytes > sv->tab.bytes) return fail(GDIST_E_DEVICE, "server refit plan does not fit");
  HIPCHK(hipMemcpyAsync(sv->tab.p, stage + tab_off, bytes, hipMemcpyHostToDevice, c->stream));
  HIPCHK(launch_refit_batch(plan, sv->tab.p, c->stream));
  TravParams p = params(sv);
  p.n_list = (uint32_t)slots.size();
  HIPCHK(launch_admit(p, c->stream));
  sv->n_active += (uint32_t)slots.size();
  std::lock_guard<std::mutex> g(sv->mu);
  sv->stats.admitted += slots.size();
  return GDIST_OK;
}

// One device step.  Returns a non-OK status only for device failures.
gdist_status_t step(gdist_server* sv) {
  gdist_ctx* c = sv->c;
  // 0. the step graph follows the storage (the spill stack may have grown)
  const TravParams p = params(sv);
  if (!sv->gp_set || std::memcmp(&p, &sv->gp, sizeof(p)) != 0) {
    HIPCHK(hipStreamSynchronize(c->stream));
    build_graph(sv, p);
  }
  // 1. admission
  std::vector<Pending> reqs;
  {
    std::lock_guard<std::mutex> g(sv->mu);
    const uint64_t room = sv->stack_cap / 2;
    while (!sv->pending.empty() && !sv->free_slots.empty() && sv->n_active + reqs.size() < sv->concurrency &&
           sv->live_total < room && reqs.size() < sv->free_slots.size()) {
      reqs.push_back(sv->pending.front());
      sv->pending.pop_front();
    }
  }
  if (!reqs.empty()) {
    gdist_status_t s = admit(sv, reqs);
    if (s != GDIST_OK) return s;
  }
  if (sv->n_active == 0) return GDIST_OK;
  // 2-5. traversal, live counts, completion, re-evaluation, report copy
  bool lng;
  {
    std::lock_guard<std::mutex> g(sv->mu);
    lng = sv->pending.empty();
  }
  HIPCHK(hipEventRecord(sv->ev[0], c->stream));
  if (sv->gexec[lng]) HIPCHK(hipGraphLaunch(sv->gexec[lng], c->stream));
  else HIPCHK(enqueue_step(sv, step_params(p, lng)));
  HIPCHK(hipEventRecord(sv->ev[1], c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, sv->ev[0], sv->ev[1]));
  const char* rep = (const char*)sv->rep_host;
  StepHead head;
  std::memcpy(&head, rep, sizeof(head));
  const uint32_t* live = (const uint32_t*)(rep + sv->live_off);
  const uint32_t* finish = (const uint32_t*)(rep + sv->fin_off);
  const gdist_result_t* res = (const gdist_result_t*)(rep + sv->res_off);
  {
    std::lock_guard<std::mutex> g(sv->mu);
    sv->stats.steps++;
    sv->stats.rounds += head.rounds_done;
    sv->stats.device_ms += ms;
    if (sv->gexec[lng]) sv->stats.graph_steps++;
  }
  if (head.abort) return fail(GDIST_E_DEVICE, "server step: grid barrier timed out");
  if (head.overflow) {
    // pending pairs were lost: every query in flight starts over later
    std::vector<uint32_t> act;
    for (uint32_t s = 0; s < sv->S; ++s)
      if (sv->active[s]) act.push_back(s);
    bool requeue = act.size() > 1;
    if (!requeue) {
      gdist_status_t g = grow_storage(sv);
      if (g == GDIST_OK) requeue = true;
      else if (g != GDIST_E_CAPACITY) return g;
    }
    if (!requeue) {
      run_alone(sv, sv->slot_req[act[0]]);
    } else {
      std::lock_guard<std::mutex> g(sv->mu);
      for (auto it = act.rbegin(); it != act.rend(); ++it) sv->pending.push_front(sv->slot_req[*it]);
      sv->stats.requeued += act.size();
    }
    for (uint32_t s : act) {
      sv->active[s] = 0;
      sv->free_slots.push_back(s);
    }
    sv->n_active = 0;
    sv->live_total = 0;
    sv->concurrency = sv->concurrency > 1 ? sv->concurrency / 2 : 1;
    sv->clean_steps = 0;
    return reset_storage(sv);
  }
  // completions: the device flagged exactly the in-flight slots that drained
  std::vector<uint32_t> fin, bad;
  uint64_t total = 0;
  for (uint32_t s = 0; s < sv->S; ++s) {
    const bool drained = sv->active[s] && live[s] == 0;
    if (finish[s] > 2u || (finish[s] != 0u) != drained)
      return fail(GDIST_E_DEVICE, "server step: completion flags disagree with the slot table (slot %u)", s);
    if (!sv->active[s]) continue;
    total += live[s];
    if (finish[s] == 1u) fin.push_back(s);
    else if (finish[s] == 2u) bad.push_back(s);
  }
  sv->live_total = total;
  if (++sv->clean_steps > 16 && sv->concurrency < sv->S) {
    sv->concurrency++;
    sv->clean_steps = 0;
  }
  for (uint32_t s : fin) {
    const Pending& rq = sv->slot_req[s];
    complete(sv, rq.tag, rq.t_submit, res[s]);
  }
  for (uint32_t s : bad) run_alone(sv, sv->slot_req[s]);
  for (uint32_t s : bad) fin.push_back(s);
  for (uint32_t s : fin) {
    sv->active[s] = 0;
    sv->free_slots.push_back(s);
    sv->n_active--;
  }
  return GDIST_OK;
}

void worker_main(gdist_server* sv) {
  (void)hipSetDevice(sv->c->device);
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      if (sv->stopping.load()) break;
      if (sv->pending.empty() && sv->n_active == 0) {
        sv->cv.wait_for(lk, std::chrono::milliseconds(2));
        continue;
      }
    }
    gdist_status_t s = step(sv);
    if (s != GDIST_OK) {
      // device failure: fail everything in flight and queued, then stop
      for (uint32_t i = 0; i < sv->S; ++i)
        if (sv->active[i]) complete(sv, sv->slot_req[i].tag, sv->slot_req[i].t_submit, failed_result(s));
      std::deque<Pending> q;
      {
        std::lock_guard<std::mutex> g(sv->mu);
        q.swap(sv->pending);
      }
      for (const Pending& rq : q) complete(sv, rq.tag, rq.t_submit, failed_result(s));
      sv->n_active = 0;
      break;
    }
  }
}

void free_server(gdist_server* sv) {
  gdist_ctx* c = sv->c;
  drop_graph(sv);
  DevBuf* bufs[] = {&sv->desc,  &sv->desc_stage, &sv->st, &sv->rep, &sv->boxes, &sv->front[0], &sv->front[1],
                    &sv->leaf[0], &sv->leaf[1], &sv->stack, &sv->counts, &sv->cand,    &sv->cand64,
                    &sv->ctl,   &sv->list,   &sv->tab};
  for (DevBuf* b : bufs) release_buf(c, *b);
  if (sv->pinned) (void)hipHostFree(sv->pinned);
  if (sv->rep_host) (void)hipHostFree(sv->rep_host);
  for (int i = 0; i < 2; ++i)
    if (sv->ev[i]) (void)hipEventDestroy(sv->ev[i]);
}

}  // namespace

extern "C" {

gdist_status_t gdist_server_start(gdist_ctx_t c, const gdist_server_config_t* config, gdist_server_t* out) {
  if (!c) return fail(GDIST_E_HANDLE, "NULL context");
  if (!out) return fail(GDIST_E_INVALID, "NULL output pointer");
  *out = nullptr;
  if (c->busy) return fail(GDIST_E_BUSY, "the context already runs a server");
  drain_async(c);
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(hipStreamSynchronize(c->stream));
  gdist_server* sv = new gdist_server();
  sv->c = c;
  if (config) sv->cfg = *config;
  gdist_server_config_t& cf = sv->cfg;
  if (cf.max_slots == 0) cf.max_slots = 64;
  if (cf.rounds_per_step == 0) cf.rounds_per_step = 4;
  if (cf.front_capacity == 0) cf.front_capacity = 1ull << 25;
  if (cf.stack_capacity == 0) cf.stack_capacity = 1ull << 26;
  if (cf.cand_per_slot == 0) cf.cand_per_slot = 1u << 18;
  if (cf.max_tris == 0)
    for (auto& kv : c->meshes) cf.max_tris = std::max(cf.max_tris, kv.second->n_tris);
  if (cf.max_slots > 512 || cf.max_tris == 0 || cf.front_capacity > kServerCapLimit ||
      cf.cand_per_slot > (1u << 26) || cf.stack_capacity > kStackLimit) {
    delete sv;
    return fail(GDIST_E_INVALID, "server config out of range (max_slots <= 512, a mesh or max_tris > 0, "
                                 "front_capacity <= 2^28, cand_per_slot <= 2^26, stack_capacity <= 2^31)");
  }
  sv->S = cf.max_slots;
  sv->nb = c->trav_blocks;
  sv->max_leaves = 1u << (31 - __builtin_clz(cf.max_tris));
  sv->box_stride = (12ull * sv->max_leaves + 63) & ~(size_t)63;
  sv->seg_f = (uint32_t)std::max<uint64_t>(cf.front_capacity / (sv->nb + 1), sv->S);
  sv->seg_f = std::max(sv->seg_f, min_segment(c->expand_budget, sv->nb));
  sv->seg_l = sv->seg_f;
  sv->stack_cap = cf.stack_capacity;
  sv->cps = cf.cand_per_slot;
  sv->concurrency = sv->S;
  const uint64_t fcap = (uint64_t)sv->seg_f * (sv->nb + 1);
  gdist_status_t s = GDIST_OK;
  auto A = [&](DevBuf& b, size_t bytes) {
    if (s == GDIST_OK) s = ensure(c, b, bytes);
  };
  sv->live_off = sizeof(StepHead);
  sv->fin_off = sv->live_off + 4ull * sv->S;
  sv->res_off = (sv->fin_off + 4ull * sv->S + 255) & ~(size_t)255;
  sv->rep_bytes = sv->res_off + sizeof(gdist_result_t) * sv->S;
  A(sv->desc, sizeof(SlotDesc) * sv->S);
  A(sv->desc_stage, sizeof(SlotDesc) * sv->S);
  A(sv->st, sizeof(SlotState) * sv->S);
  A(sv->rep, sv->rep_bytes);
  A(sv->boxes, sizeof(float) * sv->box_stride * sv->S);
  for (int b = 0; b < 2; ++b) {
    A(sv->front[b], 16ull * fcap);
    A(sv->leaf[b], 16ull * fcap);
  }
  A(sv->stack, 16ull * sv->stack_cap);
  A(sv->counts, 16ull * (sv->nb + 1));
  A(sv->cand, sizeof(Cand) * (size_t)sv->cps * sv->S);
  A(sv->cand64, sizeof(double) * (size_t)sv->cps * sv->S);
  A(sv->ctl, sizeof(Ctl));
  A(sv->list, 4ull * sv->S);
  A(sv->tab, sizeof(RefitJob) * sv->S + sizeof(ReduceJob) * sv->S * kMaxRefitPasses + 256);
  if (s == GDIST_OK) {
    sv->pinned_bytes = tab_offset(sv) + sv->tab.bytes;
    if (hipHostMalloc(&sv->pinned, sv->pinned_bytes, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&sv->rep_host, sv->rep_bytes, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      s = fail(GDIST_E_OOM, "hipHostMalloc for the server failed");
    }
  }
  if (s == GDIST_OK && (hipEventCreate(&sv->ev[0]) != hipSuccess || hipEventCreate(&sv->ev[1]) != hipSuccess))
    s = fail(GDIST_E_DEVICE, "hipEventCreate failed");
  if (s == GDIST_OK) s = reset_storage(sv);
  if (s == GDIST_OK && hipStreamSynchronize(c->stream) != hipSuccess) s = fail(GDIST_E_DEVICE, "server reset failed");
  if (s == GDIST_OK) build_graph(sv, params(sv));
  if (s != GDIST_OK) {
    std::string msg = gdist_last_error();
    free_server(sv);
    delete sv;
    fail(s, "%s", msg.c_str());
    return s;
  }
  sv->active.assign(sv->S, 0);
  sv->slot_req.resize(sv->S);
  for (uint32_t i = 0; i < sv->S; ++i) sv->free_slots.push_back(sv->S - 1 - i);
  c->busy = true;
  sv->worker = std::thread(worker_main, sv);
  *out = sv;
  return GDIST_OK;
}

gdist_status_t gdist_server_submit(gdist_server_t sv, const gdist_query_desc_t* q, uint64_t tag) {
  if (!sv) return fail(GDIST_E_HANDLE, "NULL server");
  if (!q) return fail(GDIST_E_INVALID, "NULL query");
  SlotDesc d;
  Mesh* B = nullptr;
  gdist_status_t s = make_slot(sv->c, *q, 0, &d, &B, false);
  if (s != GDIST_OK) return s;
  if (B->L > sv->max_leaves)
    return fail(GDIST_E_CAPACITY, "mesh of %u triangles exceeds the server's max_tris", B->n_tris);
  {
    std::lock_guard<std::mutex> g(sv->mu);
    sv->pending.push_back(Pending{*q, tag, now_ns()});
    sv->stats.submitted++;
  }
  sv->cv.notify_one();
  return GDIST_OK;
}

uint32_t gdist_server_poll(gdist_server_t sv, gdist_completion_t* out, uint32_t max) {
  if (!sv || !out || max == 0) return 0;
  std::lock_guard<std::mutex> g(sv->mu);
  uint32_t n = (uint32_t)std::min<size_t>(max, sv->done.size());
  for (uint32_t i = 0; i < n; ++i) out[i] = sv->done[i];
  sv->done.erase(sv->done.begin(), sv->done.begin() + n);
  return n;
}

gdist_status_t gdist_server_stats(gdist_server_t sv, gdist_server_stats_t* out) {
  if (!sv) return fail(GDIST_E_HANDLE, "NULL server");
  if (!out) return fail(GDIST_E_INVALID, "NULL output");
  std::lock_guard<std::mutex> g(sv->mu);
  *out = sv->stats;
  out->active = sv->n_active;
  out->pending = (uint32_t)sv->pending.size();
  out->concurrency = sv->concurrency;
  out->fallbacks = sv->fallbacks;
  out->graph_mode = sv->graph_mode;
  return GDIST_OK;
}

gdist_status_t gdist_server_stop(gdist_server_t sv) {
  if (!sv) return GDIST_OK;
  sv->stopping.store(true);
  sv->cv.notify_all();
  if (sv->worker.joinable()) sv->worker.join();
  (void)hipSetDevice(sv->c->device);
  (void)hipStreamSynchronize(sv->c->stream);
  free_server(sv);
  sv->c->busy = false;
  delete sv;
  return GDIST_OK;
}

}  // extern "C"
