// Host side of libgdist: contexts, mesh handles, per-query workspaces and the
// C ABI declared in include/gdist.h.  Every device step of a query runs in the
// kernels of this library; the host validates, prepares the per-query
// descriptors (FP64 relative pose rounded to FP32, tie tolerance), launches,
// and copies the results back.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "host.hpp"

using namespace gd;

namespace gd {

thread_local std::string t_err;

gdist_status_t fail(gdist_status_t s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  t_err = buf;
  return s;
}

gdist_status_t dalloc(gdist_ctx* c, size_t bytes, void** p) {
  if (bytes == 0) bytes = 256;
  if (c->memory_budget && c->bytes_held + bytes > c->memory_budget)
    return fail(GDIST_E_OOM, "device memory budget exceeded (%llu + %zu > %llu bytes)",
                (unsigned long long)c->bytes_held, bytes, (unsigned long long)c->memory_budget);
  if (c->alloc_fn) {
    *p = c->alloc_fn(bytes, c->alloc_user);
    if (!*p) return fail(GDIST_E_OOM, "the caller's allocator returned NULL for %zu bytes", bytes);
  } else {
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      *p = nullptr;
      return fail(GDIST_E_OOM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
  }
  c->bytes_held += bytes;
  return GDIST_OK;
}

void dfree(gdist_ctx* c, void* p, size_t bytes) {
  if (!p) return;
  if (c->free_fn) c->free_fn(p, c->alloc_user);
  else (void)hipFree(p);
  c->bytes_held -= bytes ? bytes : 256;
}

// Wait until every asynchronous batch of the context has finished (other
// calls on the context do this first, so they never race with the worker).
void drain_async(gdist_ctx* c) {
  std::unique_lock<std::mutex> lk(c->amu);
  c->acv.wait(lk, [&] { return c->apending == 0; });
}

void async_worker(gdist_ctx* c) {
  (void)hipSetDevice(c->device);
  for (;;) {
    gdist_ctx::AsyncBatch b;
    {
      std::unique_lock<std::mutex> lk(c->amu);
      c->acv.wait(lk, [&] { return c->astop || !c->aq.empty(); });
      if (c->aq.empty()) return;   // stopping, nothing left
      b = std::move(c->aq.front());
      c->aq.pop_front();
    }
    gdist_status_t s = GDIST_OK;
    if (b.after && hipStreamWaitEvent(c->stream, b.after, 0) != hipSuccess)
      s = fail(GDIST_E_DEVICE, "hipStreamWaitEvent on the caller's stream failed");
    if (s == GDIST_OK) s = run_queries(c, (uint32_t)b.q.size(), b.q.data(), b.out);
    if (b.after) (void)hipEventDestroy(b.after);

    std::lock_guard<std::mutex> g(c->amu);
    if (s != GDIST_OK && c->aerr_status == GDIST_OK) {
      c->aerr_status = s;
      c->aerr_msg = t_err;
    }
    c->apending--;
    c->acv.notify_all();
  }
}

void stop_async(gdist_ctx* c) {
  {
    std::lock_guard<std::mutex> g(c->amu);
    c->astop = true;
  }
  c->acv.notify_all();
  if (c->aworker.joinable()) c->aworker.join();
}

gdist_status_t ensure(gdist_ctx* c, DevBuf& b, size_t bytes) {
  if (b.bytes >= bytes && b.p) return GDIST_OK;
  if (b.p) {
    HIPCHK(hipStreamSynchronize(c->stream));
    dfree(c, b.p, b.bytes);
    b.p = nullptr;
    b.bytes = 0;
  }
  gdist_status_t s = dalloc(c, bytes, &b.p);
  if (s != GDIST_OK) return s;
  b.bytes = bytes;
  return GDIST_OK;
}

gdist_status_t ensure_pinned(gdist_ctx* c, size_t bytes) {
  if (c->pinned_bytes >= bytes && c->pinned) return GDIST_OK;
  HIPCHK(hipStreamSynchronize(c->stream));
  if (c->pinned) (void)hipHostFree(c->pinned);
  c->pinned = nullptr;
  c->pinned_bytes = 0;
  size_t want = bytes < (1u << 16) ? (1u << 16) : bytes;
  if (hipHostMalloc(&c->pinned, want, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    c->pinned = nullptr;
    return fail(GDIST_E_OOM, "hipHostMalloc(%zu) failed", want);
  }
  c->pinned_bytes = want;
  return GDIST_OK;
}

void release_buf(gdist_ctx* c, DevBuf& b) {
  dfree(c, b.p, b.bytes);
  b.p = nullptr;
  b.bytes = 0;
}

gdist_status_t check_pose(const gdist_pose_t* p, const char* which) {
  if (!p) return fail(GDIST_E_INVALID, "pose %s is NULL", which);
  for (int i = 0; i < 9; ++i)
    if (!std::isfinite(p->R[i])) return fail(GDIST_E_INVALID, "pose %s has a non-finite rotation entry", which);
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(p->t[i])) return fail(GDIST_E_INVALID, "pose %s has a non-finite translation", which);
  double err = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += p->R[3 * k + i] * p->R[3 * k + j];
      err = std::fmax(err, std::fabs(s - (i == j ? 1.0 : 0.0)));
    }
  const double* R = p->R;
  double det = R[0] * (R[4] * R[8] - R[5] * R[7]) - R[1] * (R[3] * R[8] - R[5] * R[6]) +
               R[2] * (R[3] * R[7] - R[4] * R[6]);
  if (err > 1e-6 || det < 0.0)
    return fail(GDIST_E_INVALID, "pose %s is not a proper rotation (|R^T R - I| = %.3g, det = %.6f)", which, err, det);
  return GDIST_OK;
}

// largest |world coordinate| over the 8 corners of a local box under a pose
double world_extent(const float* box, const gdist_pose_t& P) {
  double m = 0.0;
  for (int c = 0; c < 8; ++c) {
    double x = (c & 1) ? box[3] : box[0], y = (c & 2) ? box[4] : box[1], z = (c & 4) ? box[5] : box[2];
    for (int r = 0; r < 3; ++r) {
      double w = P.R[3 * r] * x + P.R[3 * r + 1] * y + P.R[3 * r + 2] * z + P.t[r];
      m = std::fmax(m, std::fabs(w));
    }
  }
  return m;
}

Mesh* find_mesh(gdist_ctx* c, gdist_mesh_t h) {
  auto it = c->meshes.find(h);
  return it == c->meshes.end() ? nullptr : it->second;
}

void free_mesh(gdist_ctx* c, Mesh* m) {
  dfree(c, m->tris, 36ull * m->n_tris);
  dfree(c, m->orig, 4ull * m->n_tris);
  dfree(c, m->boxes, 48ull * m->L);
  dfree(c, m->fl, 12ull * m->n_tris);
  delete m;
}

uint32_t floor_log2(uint32_t x) { return 31u - (uint32_t)__builtin_clz(x); }

gdist_status_t refresh_grid(gdist_ctx* c) {
  HIPCHK(traverse_grid(c->device, c->blocks_per_cu, &c->trav_blocks, &c->trav_threads));
  return GDIST_OK;
}

constexpr uint32_t kCapLimit = 1u << 28;      // entries per front / leaf buffer
constexpr uint32_t kCandLimit = 1u << 26;     // FP64 candidates

void print_trace(gdist_ctx* c, uint32_t g0, uint32_t gn, const Ctl& h);

// Traversal + FP64 re-evaluation of slots [g0, g0 + gn), whose descriptors are
// already on the device.  On storage overflow the capacities grow and the
// group is run again; when they cannot grow any more and gn > 1, returns
// E_CAPACITY with *split set.
gdist_status_t traverse_group(gdist_ctx* c, uint32_t g0, uint32_t gn, gdist_result_t* out, bool* first_launch,
                              bool* split) {
  gdist_status_t s;
  const uint32_t nb = c->trav_blocks;
  // per-workgroup segments; the root pairs all start in segment 0
  auto seg_of = [&](uint32_t cap) {
    uint32_t v = cap / (nb + 1);
    if (v < gn) v = gn;   // the admission segment takes every root pair
    return v < 1u ? 1u : v;
  };
  uint32_t sf = seg_of(c->front_cap), sl = seg_of(c->leaf_cap);
  const uint32_t smin = min_segment(c->expand_budget, nb);
  if (sf < smin) sf = smin;
  if (sl < smin) sl = smin;
  uint64_t scap = c->stack_cap;
  uint32_t cps = c->cand_cap / gn;
  if (cps < 1024u) cps = 1024u;
  Ctl hctl;
  if ((s = ensure(c, c->counts, 16ull * (nb + 1))) != GDIST_OK) return s;
  for (uint32_t attempt = 0;; ++attempt) {
    const uint64_t fcap = (uint64_t)sf * (nb + 1), lcap = (uint64_t)sl * (nb + 1);
    const uint64_t ccap = (uint64_t)cps * gn;
    for (int b = 0; b < 2; ++b) {
      if ((s = ensure(c, c->front[b], 16ull * fcap)) != GDIST_OK) return s;
      if ((s = ensure(c, c->leaf[b], 16ull * lcap)) != GDIST_OK) return s;
    }
    if ((s = ensure(c, c->stack, 16ull * scap)) != GDIST_OK) return s;
    if ((s = ensure(c, c->cand, sizeof(Cand) * (size_t)ccap)) != GDIST_OK) return s;
    if ((s = ensure(c, c->cand64, sizeof(double) * (size_t)ccap)) != GDIST_OK) return s;
    TravParams p;
    std::memset(&p, 0, sizeof(p));
    p.stats = c->stats;
    p.cand_buf = c->cand_buf;
    p.desc = (const SlotDesc*)c->desc.p + g0;
    p.st = (SlotState*)c->st.p + g0;
    p.res = (gdist_result_t*)c->res.p + g0;
    p.front[0] = (uint4*)c->front[0].p;
    p.front[1] = (uint4*)c->front[1].p;
    p.leaf[0] = (uint4*)c->leaf[0].p;
    p.leaf[1] = (uint4*)c->leaf[1].p;
    uint32_t* cnt = (uint32_t*)c->counts.p;
    p.fcount[0] = cnt;
    p.fcount[1] = cnt + (nb + 1);
    p.lcount[0] = cnt + 2 * (nb + 1);
    p.lcount[1] = cnt + 3 * (nb + 1);
    p.nblocks = nb;
    p.cand = (Cand*)c->cand.p;
    p.cand_d64 = (double*)c->cand64.p;
    p.ctl = (Ctl*)c->ctl.p;
    p.slot_list = nullptr;
    p.n_list = gn;
    p.cand_per_slot = cps;
    p.round0 = 0;
    p.max_rounds = 0xffffffffu;
    p.seg_front = sf;
    p.seg_leaf = sl;
    p.n_slots = gn;
    p.expand_budget = c->expand_budget;
    p.k_cap = c->k_cap;
    p.spin_limit = 1u << 26;
    p.cand_stop = 1u;
    p.stack = (uint4*)c->stack.p;
    p.stack_cap = (uint32_t)scap;
    p.round_cap = round_cap_for(sf < sl ? sf : sl, nb);
    HIPCHK(launch_reset(p, c->stream));
    HIPCHK(launch_admit(p, c->stream));
    if (*first_launch) HIPCHK(hipEventRecord(c->ev[2], c->stream));
    *first_launch = false;
    HIPCHK(hipEventRecord(c->ev[4], c->stream));
    HIPCHK(launch_traverse(p, c->trav_blocks, c->trav_threads, c->stream));
    HIPCHK(hipEventRecord(c->ev[5], c->stream));
    HIPCHK(launch_reeval(p, c->stream));
    HIPCHK(hipEventRecord(c->ev[3], c->stream));
    // copy-back through pinned staging, one stream synchronisation
    char* back = (char*)c->pinned + c->back_off;
    HIPCHK(hipMemcpyAsync(back, c->ctl.p, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(back + c->back_res, p.res, sizeof(gdist_result_t) * gn, hipMemcpyDeviceToHost,
                          c->stream));
    if (c->warm_start)   // the reported pairs, for the next queries of the same meshes
      HIPCHK(hipMemcpyAsync(back + c->back_st, p.st, sizeof(SlotState) * gn, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    std::memcpy(&hctl, back, sizeof(Ctl));
    std::memcpy(out, back + c->back_res, sizeof(gdist_result_t) * gn);
    if (c->warm_start) std::memcpy(c->warm_st.data() + g0, back + c->back_st, sizeof(SlotState) * gn);
    float kms = 0.f;
    HIPCHK(hipEventElapsedTime(&kms, c->ev[4], c->ev[5]));
    c->last.ms_traverse_kernel += kms;
    c->last.traverse_launches += 1;
    if (hctl.abort) return fail(GDIST_E_DEVICE, "traversal grid barrier timed out");
    if (!hctl.overflow) {
      // keep grown capacities for the next queries on this context
      if (fcap > c->front_cap) c->front_cap = (uint32_t)fcap;
      if (lcap > c->leaf_cap) c->leaf_cap = (uint32_t)lcap;
      if (scap > c->stack_cap) c->stack_cap = scap;
      if (ccap > c->cand_cap) c->cand_cap = (uint32_t)(ccap < kCandLimit ? ccap : kCandLimit);
      break;
    }
    const bool can_grow = ((hctl.overflow & 1u) == 0 || 2ull * fcap <= kCapLimit) &&
                          ((hctl.overflow & 2u) == 0 || 2ull * lcap <= kCapLimit) &&
                          ((hctl.overflow & 4u) == 0 || 2ull * ccap <= kCandLimit) &&
                          ((hctl.overflow & 8u) == 0 || 2ull * scap <= kStackLimit);
    if (!can_grow || attempt >= c->max_retries) {
      *split = gn > 1;
      return fail(GDIST_E_CAPACITY,
                  "traversal storage exhausted (front %llu, leaf %llu, stack %llu, candidates %llu entries, %u queries)",
                  (unsigned long long)fcap, (unsigned long long)lcap, (unsigned long long)scap,
                  (unsigned long long)ccap, gn);
    }
    c->last.retries++;
    if (hctl.overflow & 1u) sf *= 2u;
    if (hctl.overflow & 2u) sl *= 2u;
    if (hctl.overflow & 4u) cps *= 2u;
    if (hctl.overflow & 8u) scap *= 2u;
  }
  for (int i = 0; i < ST_N; ++i) {
    if (i == ST_PEAK) c->last_ctl_sum[i] = std::max(c->last_ctl_sum[i], hctl.stats[i]);
    else c->last_ctl_sum[i] += hctl.stats[i];
  }
  if (c->trace) print_trace(c, g0, gn, hctl);
  return GDIST_OK;
}

void print_trace(gdist_ctx* c, uint32_t g0, uint32_t gn, const Ctl& h) {
  uint32_t R = (uint32_t)h.stats[ST_ROUNDS];
  double khz = c->wall_khz > 0 ? (double)c->wall_khz : 1e5;
  fprintf(stderr, "[gdist] slots %u..%u, %u rounds\n", g0, g0 + gn - 1, R);
  for (uint32_t r = 0; r < R && r < kTraceRounds; ++r) {
    unsigned long long t1 = (r + 1 < R && r + 1 < kTraceRounds) ? h.trace_t[r + 1] : h.trace_end;
    fprintf(stderr, "[gdist]   round %2u  front %10u  leaf pairs %10u  %9.1f us\n", r, h.trace_n[r], h.trace_nl[r],
            (double)(t1 - h.trace_t[r]) * 1e3 / khz);
  }
}

gdist_status_t make_slot(gdist_ctx* c, const gdist_query_desc_t& q, uint32_t idx, SlotDesc* dp, Mesh** Bout,
                         bool hints) {
  Mesh* ma = find_mesh(c, q.a);
  Mesh* mb = find_mesh(c, q.b);
  if (!ma || !mb) return fail(GDIST_E_HANDLE, "query %u: unknown mesh handle", idx);
  if (q.mode > 1) return fail(GDIST_E_INVALID, "query %u: unknown mode %u", idx, q.mode);
  gdist_status_t s = check_pose(&q.pa, "a");
  if (s != GDIST_OK) return s;
  s = check_pose(&q.pb, "b");
  if (s != GDIST_OK) return s;
  // refit the smaller tree into the larger one's frame
  bool swapped = ma->n_tris < mb->n_tris;
  Mesh* A = swapped ? mb : ma;
  Mesh* B = swapped ? ma : mb;
  const gdist_pose_t& PA = swapped ? q.pb : q.pa;
  const gdist_pose_t& PB = swapped ? q.pa : q.pb;
  SlotDesc& d = *dp;
  std::memset(&d, 0, sizeof(d));
  d.boxA = A->boxes;
  d.trisA = A->tris;
  d.trisB = B->tris;
  d.origA = A->orig;
  d.origB = B->orig;
  d.nA = A->n_tris;
  d.nB = B->n_tris;
  d.LA = A->L;
  d.LB = B->L;
  d.depthA = A->depth;
  d.depthB = B->depth;
  d.mode = q.mode;
  d.enhanced = c->bounds == 0 ? 1u : 0u;
  d.swapped = swapped ? 1u : 0u;
  d.kappa_u = (float)(c->kappa * std::ldexp(1.0, -24));
  // B local -> A local: R = RA^T RB, t = RA^T (tB - tA)
  for (int r = 0; r < 3; ++r) {
    for (int col = 0; col < 3; ++col) {
      double s2 = 0.0;
      for (int k = 0; k < 3; ++k) s2 += PA.R[3 * k + r] * PB.R[3 * k + col];
      d.T.R[3 * r + col] = (float)s2;
    }
    double s3 = 0.0;
    for (int k = 0; k < 3; ++k) s3 += PA.R[3 * k + r] * (PB.t[k] - PA.t[k]);
    d.T.t[r] = (float)s3;
  }
  for (int k = 0; k < 9; ++k) {
    d.RA[k] = PA.R[k];
    d.RB[k] = PB.R[k];
  }
  for (int k = 0; k < 3; ++k) {
    d.tA[k] = PA.t[k];
    d.tB[k] = PB.t[k];
  }
  if (hints && c->warm_start) {
    auto it = c->warm.find(gdist_ctx::WarmKey{q.a, q.b, q.mode});
    if (it != c->warm.end()) {
      d.hint = 1u;
      d.hint_a = it->second.first;
      d.hint_b = it->second.second;
    }
  }
  // The FP32 transform of B's vertices into A's frame rounds R and t (each
  // entry to within 2^-24 relative) and three fused multiply-adds per
  // coordinate.  With unit rows of R, every term and partial sum is at most
  // |x_B| + |t| in magnitude, so a coordinate's error is a few units of 2^-24
  // times |x_B| + |t|: B's largest local vertex norm plus the translation,
  // which can far exceed the query frame's coordinates when they cancel.  M
  // for the error window is at least that.
  {
    double ma = 0.0, tt = 0.0;
    for (int k = 0; k < 6; ++k) ma = std::fmax(ma, std::fabs((double)A->root[k]));
    for (int k = 0; k < 3; ++k) tt += (double)d.T.t[k] * (double)d.T.t[k];
    d.m_floor = (float)(std::fmax(ma, (double)B->rmax + std::sqrt(tt)) * (1.0 + 0x1p-20));
  }
  double M = std::fmax(world_extent(A->root, PA), world_extent(B->root, PB));
  d.tau = 1e-12 * std::fmax(1.0, M);
  d.err_bound = 1e-13 * std::fmax(1.0, M);
  *Bout = B;
  return GDIST_OK;
}

// The query workspace is a cache that grows on demand.  When a query call
// runs out of device memory (the budget or the device), the whole cache is
// released, so the context holds only its meshes again and stays usable.
void release_workspace(gdist_ctx* c) {
  (void)hipStreamSynchronize(c->stream);
  DevBuf* bufs[] = {&c->refit_tab, &c->ws_boxes, &c->front[0], &c->front[1], &c->leaf[0], &c->leaf[1], &c->stack,
                    &c->counts, &c->cand, &c->cand64, &c->ctl, &c->desc, &c->st, &c->res};
  for (DevBuf* b : bufs) release_buf(c, *b);
  for (auto& kv : c->world)
    for (auto& w : kv.second) release_buf(c, w.boxes);
  c->world.clear();
}

// World-frame trees of the static side of one-to-many calls
// (gdist_query_one_to_many): per mesh, the boxes of its tree refitted under
// the poses it was last queried at (a few, most recent last).
constexpr size_t kWorldPosesPerMesh = 4;

void drop_world_trees(gdist_ctx* c, gdist_mesh_t h) {
  auto it = c->world.find(h);
  if (it == c->world.end()) return;
  (void)hipStreamSynchronize(c->stream);   // no work in flight still reads them
  for (auto& w : it->second) release_buf(c, w.boxes);
  c->world.erase(it);
}

// What one query call runs: the slot descriptors and the refits ahead of the traversal.
struct CallPlan {
  std::vector<SlotDesc> desc;
  std::vector<RefitJob> jobs;
};

// Pairwise plan: each query refits its smaller mesh into the larger one's
// local frame (a box region of its own in ws_boxes).
gdist_status_t plan_pairwise(gdist_ctx* c, uint32_t n, const gdist_query_desc_t* q, CallPlan& cp) {
  cp.desc.assign(n, SlotDesc{});
  std::vector<Mesh*> Bs(n);
  std::vector<size_t> off(n);
  size_t box_floats = 0;
  for (uint32_t i = 0; i < n; ++i) {
    gdist_status_t s = make_slot(c, q[i], i, &cp.desc[i], &Bs[i]);
    if (s != GDIST_OK) return s;
    off[i] = box_floats;
    box_floats += 6ull * 2ull * Bs[i]->L;
    box_floats = (box_floats + 63) & ~(size_t)63;
  }
  gdist_status_t s = ensure(c, c->ws_boxes, box_floats * sizeof(float));
  if (s != GDIST_OK) return s;
  cp.jobs.assign(n, RefitJob{});
  for (uint32_t i = 0; i < n; ++i) {
    cp.desc[i].boxB = (const float*)c->ws_boxes.p + off[i];
    RefitJob& j = cp.jobs[i];
    std::memset(&j, 0, sizeof(j));
    j.tris = Bs[i]->tris;
    j.boxes = (float*)c->ws_boxes.p + off[i];
    j.T = cp.desc[i].T;
    j.n = Bs[i]->n_tris;
    j.L = Bs[i]->L;
  }
  return GDIST_OK;
}

Xf32 pose_f32(const gdist_pose_t& P) {
  Xf32 T;
  for (int k = 0; k < 9; ++k) T.R[k] = (float)P.R[k];
  for (int k = 0; k < 3; ++k) T.t[k] = (float)P.t[k];
  return T;
}

// Shared plan (one mesh against many, Sec. 8 future work): the query frame is
// the world.  Mesh a is refitted into it once for the whole call; each mesh
// b[i] uses its world-frame tree under pose pb[i], kept by the context from
// an earlier call with the same pose, or refitted in this call.  In every
// slot b[i] is the static side ("A", its triangles transformed by its pose in
// the narrow phase) and a the refitted side ("B").
gdist_status_t plan_shared(gdist_ctx* c, gdist_mesh_t a, const gdist_pose_t& pa, uint32_t n, const gdist_mesh_t* b,
                           const gdist_pose_t* pb, uint32_t mode, CallPlan& cp) {
  Mesh* ma = find_mesh(c, a);
  if (!ma) return fail(GDIST_E_HANDLE, "unknown mesh handle %llu", (unsigned long long)a);
  if (mode > 1) return fail(GDIST_E_INVALID, "unknown mode %u", mode);
  gdist_status_t s = check_pose(&pa, "a");
  if (s != GDIST_OK) return s;
  std::vector<Mesh*> mb(n);
  for (uint32_t i = 0; i < n; ++i) {
    mb[i] = find_mesh(c, b[i]);
    if (!mb[i]) return fail(GDIST_E_HANDLE, "query %u: unknown mesh handle", i);
    if ((s = check_pose(&pb[i], "b")) != GDIST_OK) return s;
  }
  // a's world-frame tree for this call
  if ((s = ensure(c, c->ws_boxes, 48ull * ma->L)) != GDIST_OK) return s;
  cp.jobs.clear();
  const Xf32 Ta = pose_f32(pa);
  {
    RefitJob j;
    std::memset(&j, 0, sizeof(j));
    j.tris = ma->tris;
    j.boxes = (float*)c->ws_boxes.p;
    j.T = Ta;
    j.n = ma->n_tris;
    j.L = ma->L;
    cp.jobs.push_back(j);
  }
  // the static side's world-frame trees: kept, or refitted now
  std::vector<const float*> wb(n);
  for (uint32_t i = 0; i < n; ++i) {
    auto& lst = c->world[b[i]];
    gdist_ctx::WorldTree* hit = nullptr;
    for (auto& w : lst)
      if (std::memcmp(&w.pose, &pb[i], sizeof(gdist_pose_t)) == 0) hit = &w;
    if (!hit) {
      if (lst.size() >= kWorldPosesPerMesh) {
        HIPCHK(hipStreamSynchronize(c->stream));
        release_buf(c, lst.front().boxes);
        lst.erase(lst.begin());
      }
      gdist_ctx::WorldTree w;
      w.pose = pb[i];
      if ((s = ensure(c, w.boxes, 48ull * mb[i]->L)) != GDIST_OK) return s;
      lst.push_back(w);
      hit = &lst.back();
      RefitJob j;
      std::memset(&j, 0, sizeof(j));
      j.tris = mb[i]->tris;
      j.boxes = (float*)hit->boxes.p;
      j.T = pose_f32(pb[i]);
      j.n = mb[i]->n_tris;
      j.L = mb[i]->L;
      cp.jobs.push_back(j);
    }
    wb[i] = (const float*)hit->boxes.p;
  }
  double ta = 0.0;
  for (int k = 0; k < 3; ++k) ta += (double)Ta.t[k] * (double)Ta.t[k];
  cp.desc.assign(n, SlotDesc{});
  for (uint32_t i = 0; i < n; ++i) {
    const Mesh* A = mb[i];
    SlotDesc& d = cp.desc[i];
    std::memset(&d, 0, sizeof(d));
    d.boxA = wb[i];
    d.boxB = (const float*)c->ws_boxes.p;
    d.trisA = A->tris;
    d.trisB = ma->tris;
    d.origA = A->orig;
    d.origB = ma->orig;
    d.nA = A->n_tris;
    d.nB = ma->n_tris;
    d.LA = A->L;
    d.LB = ma->L;
    d.depthA = A->depth;
    d.depthB = ma->depth;
    d.mode = mode;
    d.enhanced = c->bounds == 0 ? 1u : 0u;
    d.swapped = 1u;   // the caller's mesh a is the refitted side
    d.kappa_u = (float)(c->kappa * std::ldexp(1.0, -24));
    d.T = Ta;
    d.TA = pose_f32(pb[i]);
    d.xfA = 1u;
    for (int k = 0; k < 9; ++k) {
      d.RA[k] = pb[i].R[k];
      d.RB[k] = pa.R[k];
    }
    for (int k = 0; k < 3; ++k) {
      d.tA[k] = pb[i].t[k];
      d.tB[k] = pa.t[k];
    }
    // both sides are transformed in FP32 (see make_slot): M is at least each
    // side's largest local vertex norm plus its translation
    double tb = 0.0;
    for (int k = 0; k < 3; ++k) tb += (double)d.TA.t[k] * (double)d.TA.t[k];
    d.m_floor = (float)(std::fmax((double)A->rmax + std::sqrt(tb), (double)ma->rmax + std::sqrt(ta)) * (1.0 + 0x1p-20));
    double M = std::fmax(world_extent(A->root, pb[i]), world_extent(ma->root, pa));
    d.tau = 1e-12 * std::fmax(1.0, M);
    d.err_bound = 1e-13 * std::fmax(1.0, M);
  }
  return GDIST_OK;
}

gdist_status_t execute_plan(gdist_ctx* c, uint32_t n, const gdist_query_desc_t* q, CallPlan& cp,
                            gdist_result_t* out);

gdist_status_t run_queries_impl(gdist_ctx* c, uint32_t n, const gdist_query_desc_t* q, gdist_result_t* out) {
  if (n == 0) return GDIST_OK;
  if (!q || !out) return fail(GDIST_E_INVALID, "NULL query or result array");
  CallPlan cp;
  gdist_status_t s = plan_pairwise(c, n, q, cp);
  if (s != GDIST_OK) return s;
  return execute_plan(c, n, q, cp, out);
}

gdist_status_t run_queries(gdist_ctx* c, uint32_t n, const gdist_query_desc_t* q, gdist_result_t* out) {
  gdist_status_t s = run_queries_impl(c, n, q, out);
  if (s == GDIST_E_OOM) {
    std::string msg = t_err;
    release_workspace(c);
    t_err = msg;
  }
  return s;
}

// Upload, refits, traversal in groups of slots, FP64 re-evaluation, stats.
// q (optional) names the caller's meshes of each slot for the warm start.
gdist_status_t execute_plan(gdist_ctx* c, uint32_t n, const gdist_query_desc_t* q, CallPlan& cp,
                            gdist_result_t* out) {
  gdist_status_t s;
  std::vector<SlotDesc>& desc = cp.desc;
  const uint32_t njobs = (uint32_t)cp.jobs.size();
  if ((s = ensure(c, c->desc, sizeof(SlotDesc) * n)) != GDIST_OK) return s;
  if ((s = ensure(c, c->st, sizeof(SlotState) * n)) != GDIST_OK) return s;
  if ((s = ensure(c, c->res, sizeof(gdist_result_t) * n)) != GDIST_OK) return s;
  if ((s = ensure(c, c->ctl, sizeof(Ctl))) != GDIST_OK) return s;
  // descriptors and refit job tables go through pinned staging (async H2D)
  const size_t desc_bytes = (sizeof(SlotDesc) * n + 255) & ~(size_t)255;
  const size_t tab_cap = sizeof(RefitJob) * njobs + sizeof(ReduceJob) * njobs * kMaxRefitPasses + 256;
  // copy-back area after the tables: control block, results, slot states
  const auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
  c->back_off = al(desc_bytes + tab_cap);
  c->back_res = al(sizeof(Ctl));
  c->back_st = c->back_res + al(sizeof(gdist_result_t) * n);
  if ((s = ensure_pinned(c, c->back_off + c->back_st + sizeof(SlotState) * n)) != GDIST_OK) return s;
  std::memcpy(c->pinned, desc.data(), sizeof(SlotDesc) * n);
  RefitPlan rplan;
  const size_t tab_bytes = plan_refit_batch(cp.jobs.data(), njobs, (char*)c->pinned + desc_bytes, tab_cap, &rplan);
  if (tab_bytes == 0) return fail(GDIST_E_INVALID, "refit plan does not fit (%u trees)", njobs);
  if ((s = ensure(c, c->refit_tab, tab_bytes)) != GDIST_OK) return s;
  HIPCHK(hipMemcpyAsync(c->desc.p, c->pinned, sizeof(SlotDesc) * n, hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->refit_tab.p, (char*)c->pinned + desc_bytes, tab_bytes, hipMemcpyHostToDevice, c->stream));

  std::memset(&c->last, 0, sizeof(c->last));
  HIPCHK(hipEventRecord(c->ev[0], c->stream));
  HIPCHK(launch_refit_batch(rplan, c->refit_tab.p, c->stream));
  for (const RefitJob& j : cp.jobs) c->last.bytes_refit += 36ull * j.n + 24ull * (2ull * j.L - 1ull);
  c->last.refit_trees = njobs;
  HIPCHK(hipEventRecord(c->ev[1], c->stream));

  // Traversal in groups of slots.  A group whose storage overflows first
  // grows its capacities (up to kCapLimit entries per buffer); a group that
  // still does not fit is split in half, and later calls on this context
  // start from the smaller group size.
  std::memset(&c->last_ctl_sum, 0, sizeof(c->last_ctl_sum));
  const bool warm = c->warm_start && q;
  if (warm) c->warm_st.assign(n, SlotState{});
  uint32_t group = (c->group_hint && c->group_hint < n) ? c->group_hint : n;
  if (c->group_size && c->group_size < group) group = c->group_size;
  bool first_launch = true;
  for (uint32_t g0 = 0; g0 < n;) {
    const uint32_t gn = group < n - g0 ? group : n - g0;
    bool split = false;
    s = traverse_group(c, g0, gn, out + g0, &first_launch, &split);
    if (s == GDIST_E_CAPACITY && split) {
      group = gn / 2 > 0 ? gn / 2 : 1;
      c->group_hint = group;
      continue;
    }
    if (s != GDIST_OK) {
      // the queries from this group on did not complete: their results carry the failure
      for (uint32_t i = g0; i < n; ++i) {
        std::memset(&out[i], 0, sizeof(gdist_result_t));
        out[i].status = (uint32_t)s;
        out[i].distance = __builtin_nan("");
      }
      return s;
    }
    g0 += gn;
  }
  if (warm) {
    // remember each query's reported pair (leaf positions) for the next query of its meshes
    for (uint32_t i = 0; i < n; ++i)
      if (out[i].status == GDIST_OK && c->warm_st[i].pair_a != ~0u)
        c->warm[gdist_ctx::WarmKey{q[i].a, q[i].b, q[i].mode}] = {c->warm_st[i].pair_a, c->warm_st[i].pair_b};
  }
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
  c->last.ms_refit = ms;
  HIPCHK(hipEventElapsedTime(&ms, c->ev[2], c->ev[3]));
  c->last.ms_traversal = ms;
  HIPCHK(hipEventElapsedTime(&ms, c->ev[0], c->ev[3]));
  c->last.ms_total = ms;
  const unsigned long long* st = c->last_ctl_sum;
  c->last.rounds = st[ST_ROUNDS];
  c->last.entries_popped = st[ST_POPPED];
  c->last.child_pairs = st[ST_CHILD];
  c->last.entries_pushed = st[ST_PUSHED];
  c->last.leaf_pairs = st[ST_LEAF];
  c->last.tri_pairs = st[ST_TRI];
  c->last.tri_full = st[ST_FULL];
  c->last.candidates = st[ST_CAND];
  c->last.front_peak = st[ST_PEAK];
  c->last.child_boxes = st[ST_BOXES];
  c->last.leaf_tris = st[ST_LTRI];
  // algorithmic bytes: entries popped, child boxes (siblings read once per
  // popped entry) and entries pushed; leaf-pair entries and their triangles;
  // FP64 re-evaluation of the candidates (two triangles, 72 B each read twice)
  c->last.bytes_traversal = 16ull * c->last.entries_popped + 24ull * c->last.child_boxes + 16ull * c->last.entries_pushed;
  c->last.bytes_narrow = 16ull * c->last.leaf_pairs + 36ull * c->last.leaf_tris;
  c->last.bytes_reeval = 144ull * c->last.candidates;
  gdist_status_t first = GDIST_OK;
  for (uint32_t i = 0; i < n; ++i)
    if (out[i].status != GDIST_OK && first == GDIST_OK) first = (gdist_status_t)out[i].status;
  if (first != GDIST_OK) return fail(first, "a query found no admissible candidate");
  return GDIST_OK;
}

}  // namespace gd

extern "C" {

const char* gdist_last_error(void) { return t_err.c_str(); }

gdist_status_t gdist_create(int device, gdist_ctx_t* out) {
  if (!out) return fail(GDIST_E_INVALID, "NULL output pointer");
  *out = nullptr;
  int count = 0;
  HIPCHK(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return fail(GDIST_E_INVALID, "device %d out of range (%d devices)", device, count);
  HIPCHK(hipSetDevice(device));
  gdist_ctx* c = new gdist_ctx();
  c->device = device;
  if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return fail(GDIST_E_DEVICE, "hipStreamCreate failed");
  }
  for (int i = 0; i < 6; ++i) HIPCHK(hipEventCreate(&c->ev[i]));
  (void)hipDeviceGetAttribute(&c->wall_khz, hipDeviceAttributeWallClockRate, device);
  const char* tr = getenv("GDIST_TRACE");
  c->trace = tr && tr[0] && tr[0] != '0';
  gdist_status_t s = refresh_grid(c);
  if (s == GDIST_OK) s = noalloc_init(device);
  if (s != GDIST_OK) {
    gdist_destroy(c);
    return s;
  }
  *out = c;
  return GDIST_OK;
}

gdist_status_t gdist_destroy(gdist_ctx_t c) {
  if (!c) return GDIST_OK;
  if (c->busy) return fail(GDIST_E_BUSY, "a server runs on this context");
  drain_async(c);
  stop_async(c);
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (auto& kv : c->meshes) free_mesh(c, kv.second);
  c->meshes.clear();
  if (c->pinned) (void)hipHostFree(c->pinned);
  release_workspace(c);
  for (int i = 0; i < 6; ++i)
    if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
  if (c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
  return GDIST_OK;
}

gdist_status_t gdist_set_option(gdist_ctx_t c, const char* key, double v) {
  if (!c) return fail(GDIST_E_HANDLE, "NULL context");
  if (c->busy) return fail(GDIST_E_BUSY, "a server runs on this context");
  drain_async(c);
  if (!key) return fail(GDIST_E_INVALID, "NULL key");
  auto u32opt = [&](uint32_t* dst, double lo, double hi) -> gdist_status_t {
    if (!(v >= lo && v <= hi) || v != std::floor(v))
      return fail(GDIST_E_INVALID, "option %s=%g out of range [%g, %g]", key, v, lo, hi);
    *dst = (uint32_t)v;
    return GDIST_OK;
  };
  std::string k(key);
  if (k == "front_capacity") return u32opt(&c->front_cap, 64, 1u << 30);
  if (k == "leaf_capacity") return u32opt(&c->leaf_cap, 64, 1u << 30);
  if (k == "stack_capacity") {
    if (!(v >= 64.0 && v <= (double)kStackLimit) || v != std::floor(v))
      return fail(GDIST_E_INVALID, "option stack_capacity=%g out of range [64, 2^31]", v);
    c->stack_cap = (uint64_t)v;
    return GDIST_OK;
  }
  if (k == "cand_capacity") return u32opt(&c->cand_cap, 64, 1u << 30);
  if (k == "max_retries") return u32opt(&c->max_retries, 0, 32);
  if (k == "group_size") return u32opt(&c->group_size, 0, 1u << 30);
  if (k == "expand_budget") return u32opt(&c->expand_budget, 4, 1u << 30);
  if (k == "k_cap") return u32opt(&c->k_cap, 1, 8);
  if (k == "bounds") return u32opt(&c->bounds, 0, 1);
  if (k == "one_to_many") return u32opt(&c->one_to_many, 0, 2);
  if (k == "stats") return u32opt(&c->stats, 0, 1);
  if (k == "cand_buffer") return u32opt(&c->cand_buf, 0, kCandBuf);
  if (k == "warm_start") {
    gdist_status_t st = u32opt(&c->warm_start, 0, 1);
    if (st == GDIST_OK && !c->warm_start) c->warm.clear();
    return st;
  }
  if (k == "blocks_per_cu") {
    gdist_status_t s = u32opt(&c->blocks_per_cu, 0, 64);
    if (s != GDIST_OK) return s;
    HIPCHK(hipSetDevice(c->device));
    return refresh_grid(c);
  }
  if (k == "kappa") {
    if (!(v >= 1.0 && v <= 1e6)) return fail(GDIST_E_INVALID, "option kappa=%g out of range [1, 1e6]", v);
    c->kappa = v;
    return GDIST_OK;
  }
  if (k == "memory_budget") {
    if (!(v >= 0.0)) return fail(GDIST_E_INVALID, "option memory_budget=%g must be >= 0", v);
    c->memory_budget = (uint64_t)v;
    return GDIST_OK;
  }
  return fail(GDIST_E_INVALID, "unknown option '%s'", key);
}

// One build at a time per device in this process.  The sort's look-back
// waits only for tiles of its own launch, which the dispatcher places in
// index order; two sort launches from different streams on one device could
// interleave their placement so that each waits on a tile the other keeps
// from being placed (the bounded wait would then fail the build).
static std::mutex& build_mutex(int device) {
  static std::mutex guard;
  static std::map<int, std::mutex> per_device;
  std::lock_guard<std::mutex> lk(guard);
  return per_device[device];
}

gdist_status_t gdist_build(gdist_ctx_t c, const float* verts, uint32_t nv, const uint32_t* tris, uint32_t nt,
                           uint32_t flags, gdist_mesh_t* out) {
  if (!c) return fail(GDIST_E_HANDLE, "NULL context");
  if (c->busy) return fail(GDIST_E_BUSY, "a server runs on this context");
  drain_async(c);
  if (!out) return fail(GDIST_E_INVALID, "NULL output handle pointer");
  *out = 0;
  if (!verts || !tris) return fail(GDIST_E_INVALID, "NULL vertex or triangle array");
  if (nt == 0 || nt >= (1u << 31)) return fail(GDIST_E_INVALID, "n_tris = %u out of range [1, 2^31)", nt);
  if (nv == 0) return fail(GDIST_E_INVALID, "n_verts = 0");
  if (flags & ~(GDIST_BUILD_DEVICE_PTR | GDIST_BUILD_DEFORMABLE))
    return fail(GDIST_E_INVALID, "unknown build flags 0x%x", flags);
  std::lock_guard<std::mutex> build_lock(build_mutex(c->device));
  HIPCHK(hipSetDevice(c->device));
  const bool dev = (flags & GDIST_BUILD_DEVICE_PTR) != 0;
  const bool deformable = (flags & GDIST_BUILD_DEFORMABLE) != 0;
  gdist_status_t s = GDIST_OK;
  // temporaries
  void *dv = nullptr, *df = nullptr, *keys = nullptr, *keys2 = nullptr, *sortws = nullptr, *misc = nullptr;
  const size_t vb = 12ull * nv, fb = 12ull * nt, wb = sort_workspace_bytes(nt);
  const size_t mb = 64 + vertex_pass_scratch_bytes();
  Mesh* m = new Mesh();
  m->n_tris = nt;
  m->n_verts = nv;
  m->L = 1u << floor_log2(nt);
  m->depth = floor_log2(m->L);
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(c->stream);
    if (!dev) {
      dfree(c, dv, vb);
      dfree(c, df, fb);
    }
    dfree(c, keys, 8ull * nt);
    dfree(c, keys2, 8ull * nt);
    dfree(c, sortws, wb);
    dfree(c, misc, mb);
  };
  auto abort_build = [&](gdist_status_t st) {
    std::string msg = t_err;
    cleanup();
    free_mesh(c, m);
    t_err = msg;
    return st;
  };
#define TRY(expr)                         \
  do {                                    \
    gdist_status_t _s = (expr);           \
    if (_s != GDIST_OK) return abort_build(_s); \
  } while (0)
#define TRYHIP(expr)                                                                        \
  do {                                                                                      \
    hipError_t _e = (expr);                                                                 \
    if (_e != hipSuccess)                                                                   \
      return abort_build(fail(GDIST_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(_e))); \
  } while (0)
  if (dev) {
    dv = (void*)verts;
    df = (void*)tris;
  } else {
    TRY(dalloc(c, vb, &dv));
    TRY(dalloc(c, fb, &df));
    TRYHIP(hipMemcpyAsync(dv, verts, vb, hipMemcpyHostToDevice, c->stream));
    TRYHIP(hipMemcpyAsync(df, tris, fb, hipMemcpyHostToDevice, c->stream));
  }
  TRY(dalloc(c, mb, &misc));
  TRY(dalloc(c, 8ull * nt, &keys));
  TRY(dalloc(c, 8ull * nt, &keys2));
  TRY(dalloc(c, wb, &sortws));
  TRY(dalloc(c, 36ull * nt, (void**)&m->tris));
  TRY(dalloc(c, 4ull * nt, (void**)&m->orig));
  TRY(dalloc(c, 48ull * m->L, (void**)&m->boxes));
  if (deformable) TRY(dalloc(c, 12ull * nt, (void**)&m->fl));
  int* vbox = (int*)misc;
  uint32_t* vflags = (uint32_t*)((char*)misc + 32);
  // One pass over the device without a host round trip: the vertex and index
  // checks raise flags that are read at the end (the gathers clamp vertex
  // indices, so a rejected mesh reads nothing out of bounds).
  TRYHIP(launch_vertex_pass((const float*)dv, nv, vbox, vflags, (int*)((char*)misc + 64), c->stream));
  TRYHIP(launch_keys((const float*)dv, nv, (const uint32_t*)df, nt, vbox, (uint64_t*)keys, vflags, c->stream));
  int in_tmp = 0;
  const KeyLayout kl = key_layout(nt);
  TRYHIP(launch_sort((uint64_t*)keys, (uint64_t*)keys2, nt, kl.index_bits, 3u * kl.axis_bits, sortws, c->stream,
                     &in_tmp));
  const uint64_t* sorted = (const uint64_t*)(in_tmp ? keys2 : keys);
  TRYHIP(launch_emit_tree((const float*)dv, nv, (const uint32_t*)df, nt, sorted, kl.index_bits, m->L, m->tris, m->orig,
                          m->fl, m->boxes, c->stream));
  int hv[9] = {0};   // vertex box, largest norm, pad, flags
  uint32_t sort_timeout = 0;
  TRYHIP(hipMemcpyAsync(hv, misc, 36, hipMemcpyDeviceToHost, c->stream));
  TRYHIP(hipMemcpyAsync(m->root, m->boxes + 6, 24, hipMemcpyDeviceToHost, c->stream));
  TRYHIP(hipMemcpyAsync(&sort_timeout, sort_timeout_flag(sortws), 4, hipMemcpyDeviceToHost, c->stream));
  TRYHIP(hipStreamSynchronize(c->stream));
  const uint32_t hflags = (uint32_t)hv[8];
  std::memcpy(&m->rmax, &hv[6], 4);   // a non-negative float: its ordered int is its bits
  if (hflags & 1u) return abort_build(fail(GDIST_E_INVALID, "a triangle index is >= n_verts (%u)", nv));
  if (hflags & 2u) return abort_build(fail(GDIST_E_INVALID, "a vertex coordinate is not finite"));
  if (sort_timeout) return abort_build(fail(GDIST_E_DEVICE, "the radix sort's look-back wait timed out"));
#undef TRY
#undef TRYHIP
  cleanup();
  m->bytes = 36ull * nt + 4ull * nt + 48ull * m->L + (deformable ? 12ull * nt : 0ull);
  uint64_t h = c->next_handle++;
  c->meshes[h] = m;
  *out = h;
  (void)s;
  return GDIST_OK;
}

gdist_status_t gdist_release(gdist_ctx_t c, gdist_mesh_t h) {
  if (!c) return fail(GDIST_E_HANDLE, "NULL context");
  if (c->busy) return fail(GDIST_E_BUSY, "a server runs on this context");
  drain_async(c);
  Mesh* m = find_mesh(c, h);
  if (!m) return fail(GDIST_E_HANDLE, "unknown mesh handle %llu", (unsigned long long)h);
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(hipStreamSynchronize(c->stream));
  free_mesh(c, m);
  c->meshes.erase(h);
  drop_world_trees(c, h);
  for (auto it = c->warm.begin(); it != c->warm.end();)
    it = (it->first.a == h || it->first.b == h) ? c->warm.erase(it) : std::next(it);
  return GDIST_OK;
}

gdist_status_t gdist_update(gdist_ctx_t c, gdist_mesh_t h, const float* verts, uint32_t nv, uint32_t flags) {
  if (!c) return fail(GDIST_E_HANDLE, "NULL context");
  if (c->busy) return fail(GDIST_E_BUSY, "a server runs on this context");
  drain_async(c);
  Mesh* m = find_mesh(c, h);
  if (!m) return fail(GDIST_E_HANDLE, "unknown mesh handle %llu", (unsigned long long)h);
  if (!m->fl) return fail(GDIST_E_INVALID, "mesh %llu was not built with GDIST_BUILD_DEFORMABLE", (unsigned long long)h);
  if (!verts) return fail(GDIST_E_INVALID, "NULL vertex array");
  if (nv != m->n_verts) return fail(GDIST_E_INVALID, "n_verts = %u, the mesh has %u", nv, m->n_verts);
  if (flags & ~GDIST_BUILD_DEVICE_PTR) return fail(GDIST_E_INVALID, "unknown update flags 0x%x", flags);
  HIPCHK(hipSetDevice(c->device));
  const size_t vb = 12ull * nv;
  void* dv = (void*)verts;
  void* misc = nullptr;
  gdist_status_t s = GDIST_OK;
  if (!(flags & GDIST_BUILD_DEVICE_PTR)) {
    if ((s = dalloc(c, vb, &dv)) != GDIST_OK) return s;
  }
  const size_t mb = 64 + vertex_pass_scratch_bytes();
  if ((s = dalloc(c, mb, &misc)) == GDIST_OK) {
    hipError_t e = hipSuccess;
    if (!(flags & GDIST_BUILD_DEVICE_PTR)) e = hipMemcpyAsync(dv, verts, vb, hipMemcpyHostToDevice, c->stream);
    // finiteness before anything of the mesh changes (the leaf-order indices
    // were checked when the mesh was built)
    uint32_t hflags = 0;
    uint32_t* vflags = (uint32_t*)((char*)misc + 32);
    if (e == hipSuccess)
      e = launch_vertex_pass((const float*)dv, nv, (int*)misc, vflags, (int*)((char*)misc + 64), c->stream);
    int hrmax = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&hflags, vflags, 4, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&hrmax, (int*)misc + 6, 4, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess && !(hflags & 3u)) std::memcpy(&m->rmax, &hrmax, 4);
    if (e != hipSuccess) {
      s = fail(GDIST_E_DEVICE, "mesh update failed: %s", hipGetErrorString(e));
    } else if (hflags & 3u) {
      s = fail(GDIST_E_INVALID, "%s", (hflags & 2u) ? "a vertex coordinate is not finite"
                                                    : "a triangle index is >= n_verts");
    } else {
      Xf32 I;
      std::memset(&I, 0, sizeof(I));
      I.R[0] = I.R[4] = I.R[8] = 1.f;
      e = launch_gather_tris((const float*)dv, m->fl, m->n_tris, m->tris, c->stream);
      if (e == hipSuccess) e = launch_refit(m->tris, m->n_tris, m->L, I, m->boxes, c->stream);
      if (e == hipSuccess) e = hipMemcpyAsync(m->root, m->boxes + 6, 24, hipMemcpyDeviceToHost, c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
      if (e != hipSuccess) s = fail(GDIST_E_DEVICE, "mesh update failed: %s", hipGetErrorString(e));
    }
  }
  (void)hipStreamSynchronize(c->stream);
  if (!(flags & GDIST_BUILD_DEVICE_PTR)) dfree(c, dv, vb);
  dfree(c, misc, mb);
  if (s == GDIST_OK) drop_world_trees(c, h);   // refitted from the old vertices
  return s;
}

gdist_status_t gdist_mesh_info(gdist_ctx_t c, gdist_mesh_t h, gdist_mesh_info_t* out) {
  if (!c) return fail(GDIST_E_HANDLE, "NULL context");
  if (!out) return fail(GDIST_E_INVALID, "NULL output");
  Mesh* m = find_mesh(c, h);
  if (!m) return fail(GDIST_E_HANDLE, "unknown mesh handle %llu", (unsigned long long)h);
  std::memset(out, 0, sizeof(*out));
  out->n_tris = m->n_tris;
  out->n_leaves = m->L;
  out->depth = m->depth;
  out->device_bytes = m->bytes;
  for (int i = 0; i < 6; ++i) out->root_box[i] = m->root[i];
  return GDIST_OK;
}

gdist_status_t gdist_mesh_export(gdist_ctx_t c, gdist_mesh_t h, float* boxes, float* tris, uint32_t* orig) {
  if (!c) return fail(GDIST_E_HANDLE, "NULL context");
  drain_async(c);
  Mesh* m = find_mesh(c, h);
  if (!m) return fail(GDIST_E_HANDLE, "unknown mesh handle %llu", (unsigned long long)h);
  HIPCHK(hipSetDevice(c->device));
  if (boxes) HIPCHK(hipMemcpy(boxes, m->boxes, 48ull * m->L, hipMemcpyDeviceToHost));
  if (tris) HIPCHK(hipMemcpy(tris, m->tris, 36ull * m->n_tris, hipMemcpyDeviceToHost));
  if (orig) HIPCHK(hipMemcpy(orig, m->orig, 4ull * m->n_tris, hipMemcpyDeviceToHost));
  return GDIST_OK;
}

gdist_status_t gdist_query(gdist_ctx_t c, gdist_mesh_t a, gdist_mesh_t b, const gdist_pose_t* pa,
                           const gdist_pose_t* pb, gdist_mode_t mode, gdist_result_t* out) {
  if (!c) return fail(GDIST_E_HANDLE, "NULL context");
  if (c->busy) return fail(GDIST_E_BUSY, "a server runs on this context");
  drain_async(c);
  if (!out) return fail(GDIST_E_INVALID, "NULL result pointer");
  if (!pa || !pb) return fail(GDIST_E_INVALID, "NULL pose");
  gdist_query_desc_t d;
  std::memset(&d, 0, sizeof(d));
  d.a = a;
  d.b = b;
  d.pa = *pa;
  d.pb = *pb;
  d.mode = (uint32_t)mode;
  HIPCHK(hipSetDevice(c->device));
  return run_queries(c, 1, &d, out);
}

gdist_status_t gdist_query_batch(gdist_ctx_t c, uint32_t n, const gdist_query_desc_t* q, gdist_result_t* out) {
  if (!c) return fail(GDIST_E_HANDLE, "NULL context");
  if (c->busy) return fail(GDIST_E_BUSY, "a server runs on this context");
  drain_async(c);
  HIPCHK(hipSetDevice(c->device));
  return run_queries(c, n, q, out);
}

gdist_status_t gdist_query_one_to_many(gdist_ctx_t c, gdist_mesh_t a, const gdist_pose_t* pa, uint32_t n,
                                       const gdist_mesh_t* b, const gdist_pose_t* pb, gdist_mode_t mode,
                                       gdist_result_t* out) {
  if (!c) return fail(GDIST_E_HANDLE, "NULL context");
  if (c->busy) return fail(GDIST_E_BUSY, "a server runs on this context");
  if (n == 0) return GDIST_OK;
  if (!pa || !b || !pb || !out) return fail(GDIST_E_INVALID, "NULL pose, handle or result array");
  std::vector<gdist_query_desc_t> q(n);
  for (uint32_t i = 0; i < n; ++i) {
    std::memset(&q[i], 0, sizeof(q[i]));
    q[i].a = a;
    q[i].b = b[i];
    q[i].pa = *pa;
    q[i].pb = pb[i];
    q[i].mode = (uint32_t)mode;
  }
  drain_async(c);
  HIPCHK(hipSetDevice(c->device));
  // Shared refit (a once, into the world frame; b[i] from kept world-frame
  // trees) when it refits fewer triangles per call than the pairwise plan,
  // whose query i refits the smaller of a and b[i]; pairwise otherwise.
  bool shared = c->one_to_many == 2u;
  if (c->one_to_many == 1u && n > 1) {
    Mesh* ma = find_mesh(c, a);
    uint64_t pairwise = 0;
    for (uint32_t i = 0; i < n && ma; ++i) {
      Mesh* mb = find_mesh(c, b[i]);
      if (mb) pairwise += std::min(ma->n_tris, mb->n_tris);
    }
    shared = ma && (uint64_t)ma->n_tris < pairwise;
  }
  if (!shared) return run_queries(c, n, q.data(), out);
  CallPlan cp;
  gdist_status_t s = plan_shared(c, a, *pa, n, b, pb, (uint32_t)mode, cp);
  if (s == GDIST_OK) s = execute_plan(c, n, nullptr, cp, out);
  if (s == GDIST_E_OOM) {
    std::string msg = t_err;
    release_workspace(c);
    t_err = msg;
  }
  return s;
}

gdist_status_t gdist_query_batch_async(gdist_ctx_t c, uint32_t n, const gdist_query_desc_t* q, gdist_result_t* out,
                                       void* hip_stream) {
  if (!c) return fail(GDIST_E_HANDLE, "NULL context");
  if (c->busy) return fail(GDIST_E_BUSY, "a server runs on this context");
  if (n == 0) return GDIST_OK;
  if (!q || !out) return fail(GDIST_E_INVALID, "NULL query or result array");
  for (uint32_t i = 0; i < n; ++i) {   // validate now: errors surface at submit
    SlotDesc d;
    Mesh* B = nullptr;
    gdist_status_t s = make_slot(c, q[i], i, &d, &B, false);
    if (s != GDIST_OK) return s;
  }
  HIPCHK(hipSetDevice(c->device));
  gdist_ctx::AsyncBatch b;
  b.q.assign(q, q + n);
  b.out = out;
  if (hip_stream) {
    HIPCHK(hipEventCreateWithFlags(&b.after, hipEventDisableTiming));
    hipError_t e = hipEventRecord(b.after, (hipStream_t)hip_stream);
    if (e != hipSuccess) {
      (void)hipEventDestroy(b.after);
      return fail(GDIST_E_DEVICE, "hipEventRecord on the caller's stream failed: %s", hipGetErrorString(e));
    }
  }
  {
    std::lock_guard<std::mutex> g(c->amu);
    if (!c->aworker.joinable()) {
      c->astop = false;
      c->aworker = std::thread(async_worker, c);
    }
    c->aq.push_back(std::move(b));
    c->apending++;
  }
  c->acv.notify_all();
  return GDIST_OK;
}

gdist_status_t gdist_sync(gdist_ctx_t c, void* hip_stream) {
  if (!c) return fail(GDIST_E_HANDLE, "NULL context");
  drain_async(c);
  gdist_status_t s;
  std::string msg;
  {
    std::lock_guard<std::mutex> g(c->amu);
    s = c->aerr_status;
    msg = c->aerr_msg;
    c->aerr_status = GDIST_OK;
    c->aerr_msg.clear();
  }
  if (hip_stream) {
    // later work on the caller's stream starts after everything queued so far
    hipEvent_t ev = nullptr;
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    hipError_t e = hipEventRecord(ev, c->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent((hipStream_t)hip_stream, ev, 0);
    (void)hipEventDestroy(ev);
    if (e != hipSuccess) return fail(GDIST_E_DEVICE, "ordering the caller's stream failed: %s", hipGetErrorString(e));
  }
  if (s != GDIST_OK) return fail(s, "%s", msg.c_str());
  return GDIST_OK;
}

gdist_status_t gdist_set_allocator(gdist_ctx_t c, void* (*alloc)(size_t, void*), void (*free_)(void*, void*),
                                   void* user) {
  if (!c) return fail(GDIST_E_HANDLE, "NULL context");
  if (c->busy) return fail(GDIST_E_BUSY, "a server runs on this context");
  drain_async(c);
  if ((alloc == nullptr) != (free_ == nullptr)) return fail(GDIST_E_INVALID, "give both allocator functions or neither");
  if (c->bytes_held != 0)
    return fail(GDIST_E_INVALID, "the context already holds %llu device bytes; set the allocator right after "
                "gdist_create", (unsigned long long)c->bytes_held);
  c->alloc_fn = alloc;
  c->free_fn = free_;
  c->alloc_user = user;
  return GDIST_OK;
}

gdist_status_t gdist_last_stats(gdist_ctx_t c, gdist_stats_t* out) {
  if (!c) return fail(GDIST_E_HANDLE, "NULL context");
  drain_async(c);
  if (!out) return fail(GDIST_E_INVALID, "NULL output");
  *out = c->last;
  return GDIST_OK;
}

gdist_status_t gdist_eval_box_bounds(gdist_ctx_t c, uint32_t n, const float* a, const float* b, float* out) {
  if (!c) return fail(GDIST_E_HANDLE, "NULL context");
  if (c->busy) return fail(GDIST_E_BUSY, "a server runs on this context");
  drain_async(c);
  if (n == 0) return GDIST_OK;
  if (!a || !b || !out) return fail(GDIST_E_INVALID, "NULL array");
  HIPCHK(hipSetDevice(c->device));
  void *da = nullptr, *db = nullptr, *dout = nullptr;
  gdist_status_t s;
  if ((s = dalloc(c, 24ull * n, &da)) != GDIST_OK) return s;
  if ((s = dalloc(c, 24ull * n, &db)) != GDIST_OK) { dfree(c, da, 24ull * n); return s; }
  if ((s = dalloc(c, 16ull * n, &dout)) != GDIST_OK) { dfree(c, da, 24ull * n); dfree(c, db, 24ull * n); return s; }
  hipError_t e = hipMemcpy(da, a, 24ull * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(db, b, 24ull * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = launch_eval_bounds(n, (const float*)da, (const float*)db, (float*)dout, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(out, dout, 16ull * n, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  dfree(c, da, 24ull * n);
  dfree(c, db, 24ull * n);
  dfree(c, dout, 16ull * n);
  if (e != hipSuccess) return fail(GDIST_E_DEVICE, "box-bound evaluation failed: %s", hipGetErrorString(e));
  return GDIST_OK;
}

gdist_status_t gdist_eval_tri_tri(gdist_ctx_t c, uint32_t n, const float* p, const float* q, uint32_t mode,
                                  float* out32, double* out64) {
  if (!c) return fail(GDIST_E_HANDLE, "NULL context");
  if (c->busy) return fail(GDIST_E_BUSY, "a server runs on this context");
  drain_async(c);
  if (n == 0) return GDIST_OK;
  if (!p || !q || !out32 || !out64) return fail(GDIST_E_INVALID, "NULL array");
  if (mode > 1) return fail(GDIST_E_INVALID, "unknown mode %u", mode);
  HIPCHK(hipSetDevice(c->device));
  void *dp = nullptr, *dq = nullptr, *d32 = nullptr, *d64 = nullptr;
  gdist_status_t s;
  if ((s = dalloc(c, 36ull * n, &dp)) != GDIST_OK) return s;
  if ((s = dalloc(c, 36ull * n, &dq)) != GDIST_OK) { dfree(c, dp, 36ull * n); return s; }
  if ((s = dalloc(c, 4ull * n, &d32)) != GDIST_OK) { dfree(c, dp, 36ull * n); dfree(c, dq, 36ull * n); return s; }
  if ((s = dalloc(c, 8ull * n, &d64)) != GDIST_OK) {
    dfree(c, dp, 36ull * n); dfree(c, dq, 36ull * n); dfree(c, d32, 4ull * n);
    return s;
  }
  hipError_t e = hipMemcpy(dp, p, 36ull * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dq, q, 36ull * n, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = launch_eval_tri_tri(n, (const float*)dp, (const float*)dq, mode, (float*)d32, (double*)d64, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(out32, d32, 4ull * n, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(out64, d64, 8ull * n, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  dfree(c, dp, 36ull * n);
  dfree(c, dq, 36ull * n);
  dfree(c, d32, 4ull * n);
  dfree(c, d64, 8ull * n);
  if (e != hipSuccess) return fail(GDIST_E_DEVICE, "triangle evaluation failed: %s", hipGetErrorString(e));
  return GDIST_OK;
}

}  // extern "C"
