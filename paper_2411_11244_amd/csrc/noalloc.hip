// gdist_query_noalloc: the single-query path of gdist_query with every
// device buffer taken from one fixed array that the library holds per GPU,
// for callers that cannot allocate device memory (serving loops with a fixed
// footprint, code that must not call hipMalloc).  It runs the same kernels
// (refit, admission, persistent traversal, FP64 re-evaluation) on the
// context's stream.
//
// Limits, all checked on the host before anything is launched:
//   * the refitted tree (the smaller mesh of the pair) has at most
//     kNaMaxLeaves leaves (2^19, i.e. fewer than 2^20 triangles);
//   * the traversal runs on at most kNaBlocks workgroups with an expansion
//     budget of kNaBudget child pairs per round and a spill stack of
//     kNaStack entries; a query that needs more storage fails with
//     GDIST_E_CAPACITY (gdist_query grows its storage instead).
// Every call on one GPU uses that GPU's array, which keeps the last call's
// contents: calls that overlap on one GPU (two threads, two contexts of the
// same device) race and must be serialised by the caller.
#include <cstring>
#include <mutex>

#include "host.hpp"

namespace gd {
constexpr size_t kNaBytes = 128ull << 20;   // the array, per GPU
}

// The array itself.  Host code never uses this name as an address: the
// device address of each GPU's copy comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[gd::kNaBytes];

namespace gd {

constexpr int kNaMaxDevices = 64;
constexpr uint32_t kNaMaxLeaves = 1u << 19;
constexpr uint32_t kNaBlocks = 64;
constexpr uint32_t kNaBudget = 1u << 18;
constexpr uint32_t kNaStack = 1u << 20;
constexpr uint32_t kNaCand = 1u << 16;

namespace {
std::mutex g_na_mu;
void* g_na_ptr[kNaMaxDevices] = {};

size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

// Byte layout of the array for one query on nb workgroups and a refitted
// tree of L leaves.
struct NaLayout {
  size_t ctl, counts, desc, st, res, tab, boxes, front[2], leaf[2], stack, cand, cand64, end;
  uint32_t seg;
};
NaLayout na_layout(uint32_t nb, uint32_t L) {
  NaLayout o;
  o.seg = min_segment(kNaBudget, nb);
  size_t at = 0;
  auto put = [&](size_t bytes) {
    const size_t a = at;
    at = al256(at + bytes);
    return a;
  };
  o.ctl = put(sizeof(Ctl));
  o.counts = put(16ull * (nb + 1));
  o.desc = put(sizeof(SlotDesc));
  o.st = put(sizeof(SlotState));
  o.res = put(sizeof(gdist_result_t));
  o.tab = put(sizeof(RefitJob) + sizeof(ReduceJob) * kMaxRefitPasses + 256);
  o.boxes = put(48ull * L);
  const size_t fb = 16ull * o.seg * (nb + 1);
  for (int b = 0; b < 2; ++b) {
    o.front[b] = put(fb);
    o.leaf[b] = put(fb);
  }
  o.stack = put(16ull * kNaStack);
  o.cand = put(sizeof(Cand) * (size_t)kNaCand);
  o.cand64 = put(sizeof(double) * (size_t)kNaCand);
  o.end = at;
  return o;
}
}  // namespace

// Once per device, with that device current (gdist_create): the device
// address of this GPU's copy of the array.
gdist_status_t noalloc_init(int device) {
  std::lock_guard<std::mutex> g(g_na_mu);
  if (device < 0 || device >= kNaMaxDevices) return fail(GDIST_E_INVALID, "device %d beyond %d", device, kNaMaxDevices);
  if (g_na_ptr[device]) return GDIST_OK;
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || ptr == nullptr)
    return fail(GDIST_E_DEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", device, hipGetErrorString(e));
  g_na_ptr[device] = ptr;
  return GDIST_OK;
}

static void* noalloc_ptr(int device) {
  std::lock_guard<std::mutex> g(g_na_mu);
  return (device >= 0 && device < kNaMaxDevices) ? g_na_ptr[device] : nullptr;
}

gdist_status_t run_query_noalloc(gdist_ctx* c, const gdist_query_desc_t& q, gdist_result_t* out) {
  char* base = (char*)noalloc_ptr(c->device);
  if (!base) return fail(GDIST_E_DEVICE, "the no-allocation array of device %d is not set up", c->device);
  SlotDesc d;
  Mesh* B = nullptr;
  gdist_status_t s = make_slot(c, q, 0, &d, &B);
  if (s != GDIST_OK) return s;
  if (B->L > kNaMaxLeaves)
    return fail(GDIST_E_INVALID, "the refitted mesh has %u leaves; the no-allocation path takes at most %u (meshes of "
                "fewer than %u triangles)", B->L, kNaMaxLeaves, 2u * kNaMaxLeaves);
  const uint32_t nb = c->trav_blocks < kNaBlocks ? c->trav_blocks : kNaBlocks;
  const NaLayout lay = na_layout(nb, kNaMaxLeaves);
  if (lay.end > kNaBytes) return fail(GDIST_E_INVALID, "no-allocation layout exceeds the array");
  d.boxB = (const float*)(base + lay.boxes);

  // refit job table and descriptor: host staging on the stack, copied in
  RefitJob job;
  std::memset(&job, 0, sizeof(job));
  job.tris = B->tris;
  job.boxes = (float*)(base + lay.boxes);
  job.T = d.T;
  job.n = B->n_tris;
  job.L = B->L;
  alignas(16) char tab[sizeof(RefitJob) + sizeof(ReduceJob) * kMaxRefitPasses + 256];
  RefitPlan rplan;
  const size_t tab_bytes = plan_refit_batch(&job, 1, tab, sizeof(tab), &rplan);
  if (tab_bytes == 0) return fail(GDIST_E_INVALID, "refit plan does not fit");
  HIPCHK(hipMemcpyAsync(base + lay.desc, &d, sizeof(SlotDesc), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(base + lay.tab, tab, tab_bytes, hipMemcpyHostToDevice, c->stream));

  TravParams p;
  std::memset(&p, 0, sizeof(p));
  p.stats = c->stats;
  p.cand_buf = c->cand_buf;
  p.desc = (const SlotDesc*)(base + lay.desc);
  p.st = (SlotState*)(base + lay.st);
  p.res = (gdist_result_t*)(base + lay.res);
  for (int b = 0; b < 2; ++b) {
    p.front[b] = (uint4*)(base + lay.front[b]);
    p.leaf[b] = (uint4*)(base + lay.leaf[b]);
  }
  uint32_t* cnt = (uint32_t*)(base + lay.counts);
  p.fcount[0] = cnt;
  p.fcount[1] = cnt + (nb + 1);
  p.lcount[0] = cnt + 2 * (nb + 1);
  p.lcount[1] = cnt + 3 * (nb + 1);
  p.nblocks = nb;
  p.cand = (Cand*)(base + lay.cand);
  p.cand_d64 = (double*)(base + lay.cand64);
  p.ctl = (Ctl*)(base + lay.ctl);
  p.slot_list = nullptr;
  p.n_list = 1;
  p.cand_per_slot = kNaCand;
  p.round0 = 0;
  p.max_rounds = 0xffffffffu;
  p.seg_front = lay.seg;
  p.seg_leaf = lay.seg;
  p.n_slots = 1;
  p.expand_budget = c->expand_budget < kNaBudget ? c->expand_budget : kNaBudget;
  p.k_cap = c->k_cap;
  p.spin_limit = 1u << 26;
  p.cand_stop = 1u;
  p.stack = (uint4*)(base + lay.stack);
  p.stack_cap = kNaStack;
  p.round_cap = round_cap_for(lay.seg, nb);

  std::memset(&c->last, 0, sizeof(c->last));
  HIPCHK(hipEventRecord(c->ev[0], c->stream));
  HIPCHK(launch_refit_batch(rplan, base + lay.tab, c->stream));
  HIPCHK(hipEventRecord(c->ev[1], c->stream));
  HIPCHK(launch_reset(p, c->stream));     // control block and counts cleared by a kernel
  HIPCHK(launch_admit(p, c->stream));
  HIPCHK(hipEventRecord(c->ev[4], c->stream));
  HIPCHK(launch_traverse(p, nb, c->trav_threads, c->stream));
  HIPCHK(hipEventRecord(c->ev[5], c->stream));
  HIPCHK(launch_reeval(p, c->stream));
  HIPCHK(hipEventRecord(c->ev[3], c->stream));
  Ctl hctl;
  HIPCHK(hipMemcpyAsync(&hctl, p.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(out, p.res, sizeof(gdist_result_t), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (hctl.abort) return fail(GDIST_E_DEVICE, "traversal grid barrier timed out");
  if (hctl.overflow) {
    std::memset(out, 0, sizeof(*out));
    out->status = GDIST_E_CAPACITY;
    out->distance = __builtin_nan("");
    return fail(GDIST_E_CAPACITY, "the query needs more traversal storage than the no-allocation path holds "
                "(overflow flags 0x%x)", hctl.overflow);
  }
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
  c->last.ms_refit = ms;
  HIPCHK(hipEventElapsedTime(&ms, c->ev[1], c->ev[3]));
  c->last.ms_traversal = ms;
  HIPCHK(hipEventElapsedTime(&ms, c->ev[0], c->ev[3]));
  c->last.ms_total = ms;
  HIPCHK(hipEventElapsedTime(&ms, c->ev[4], c->ev[5]));
  c->last.ms_traverse_kernel = ms;
  c->last.traverse_launches = 1;
  const unsigned long long* st = hctl.stats;
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
  c->last.bytes_refit = 36ull * B->n_tris + 24ull * (2ull * B->L - 1ull);
  c->last.bytes_traversal = 16ull * c->last.entries_popped + 24ull * c->last.child_boxes + 16ull * c->last.entries_pushed;
  c->last.bytes_narrow = 16ull * c->last.leaf_pairs + 36ull * c->last.leaf_tris;
  c->last.bytes_reeval = 144ull * c->last.candidates;
  if (out->status != GDIST_OK) return fail((gdist_status_t)out->status, "the query found no admissible candidate");
  return GDIST_OK;
}

}  // namespace gd

using namespace gd;

extern "C" gdist_status_t gdist_query_noalloc(gdist_ctx_t c, gdist_mesh_t a, gdist_mesh_t b, const gdist_pose_t* pa,
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
  return run_query_noalloc(c, d, out);
}
