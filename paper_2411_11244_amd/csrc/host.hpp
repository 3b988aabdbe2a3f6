// Host-side definitions shared by the C ABI (api.cpp) and the serving core
// (server.cpp): contexts, mesh handles, device buffers and helpers.
#pragma once
#include <condition_variable>
#include <cstdarg>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.hpp"

struct gdist_ctx;

namespace gd {

gdist_status_t fail(gdist_status_t s, const char* fmt, ...);

#define HIPCHK(expr)                                                                              \
  do {                                                                                            \
    hipError_t _e = (expr);                                                                       \
    if (_e != hipSuccess) return fail(GDIST_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(_e)); \
  } while (0)

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct Mesh {
  uint32_t n_tris = 0, L = 0, depth = 0;
  uint32_t n_verts = 0;
  float* tris = nullptr;
  uint32_t* orig = nullptr;
  float* boxes = nullptr;
  uint32_t* fl = nullptr;   // deformable meshes: vertex indices of each triangle, leaf order
  float root[6] = {0, 0, 0, 0, 0, 0};
  float rmax = 0.f;         // upper bound of the largest local vertex norm
  uint64_t bytes = 0;
};


gdist_status_t dalloc(gdist_ctx* c, size_t bytes, void** p);
// Free a mesh's device data and the Mesh itself.
void free_mesh(gdist_ctx* c, Mesh* m);
void dfree(gdist_ctx* c, void* p, size_t bytes);
gdist_status_t ensure(gdist_ctx* c, DevBuf& b, size_t bytes);
void release_buf(gdist_ctx* c, DevBuf& b);
gdist_status_t check_pose(const gdist_pose_t* p, const char* which);
Mesh* find_mesh(gdist_ctx* c, gdist_mesh_t h);
// Validate one query and fill its descriptor (all but boxB); *B receives
// the tree that the query refits.
// With hints = false (validation on an API thread while a worker may run
// queries) the warm-start pairs are not read.
gdist_status_t make_slot(gdist_ctx* c, const gdist_query_desc_t& q, uint32_t idx, SlotDesc* d, Mesh** B,
                         bool hints = true);
// The batched query path (refit, grouped traversal with growing storage,
// FP64 re-evaluation) on the context's stream and workspace.
gdist_status_t run_queries(gdist_ctx* c, uint32_t n, const gdist_query_desc_t* q, gdist_result_t* out);
void drain_async(gdist_ctx* c);
// Set up the no-allocation array of `device` (current); once per device.
gdist_status_t noalloc_init(int device);

}  // namespace gd

struct gdist_ctx {
  using Mesh = gd::Mesh;
  using DevBuf = gd::DevBuf;
  int device = 0;
  hipStream_t stream = nullptr;
  hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  std::unordered_map<uint64_t, Mesh*> meshes;
  uint64_t next_handle = 1;
  // tunables
  uint32_t front_cap = 1u << 26, leaf_cap = 1u << 26, cand_cap = 1u << 21;
  uint64_t stack_cap = 1ull << 27;
  uint32_t max_retries = 8, expand_budget = 1u << 22, k_cap = 8, blocks_per_cu = 0, bounds = 0;
  double kappa = 64.0;
  uint64_t memory_budget = 0, bytes_held = 0;
  // workspace
  DevBuf ws_boxes, front[2], leaf[2], stack, counts, cand, cand64, ctl, desc, st, res, refit_tab;
  void* pinned = nullptr;       // host staging: descriptors and job tables, then the copy-back area
  size_t pinned_bytes = 0;
  size_t back_off = 0, back_res = 0, back_st = 0;   // copy-back area: Ctl, results, slot states
  uint32_t trav_blocks = 0, trav_threads = 0;
  int wall_khz = 0;
  bool trace = false;
  uint32_t group_hint = 0;                 // largest group of queries that fit one launch
  uint32_t group_size = 0;                 // queries per traversal launch (0 = all)
  // warm start (option warm_start): the leaf positions of the pair reported by
  // the latest query of each (mesh a, mesh b, mode), evaluated first by the
  // next query of the same meshes to seed its bound
  uint32_t warm_start = 0;
  struct WarmKey {
    uint64_t a, b;
    uint32_t mode;
    bool operator==(const WarmKey& o) const { return a == o.a && b == o.b && mode == o.mode; }
  };
  struct WarmHash {
    size_t operator()(const WarmKey& k) const { return (size_t)(k.a * 0x9E3779B97F4A7C15ull ^ (k.b << 1) ^ k.mode); }
  };
  std::unordered_map<WarmKey, std::pair<uint32_t, uint32_t>, WarmHash> warm;
  std::vector<gd::SlotState> warm_st;      // slot states copied back by the latest batch
  // one-to-many calls: world-frame trees of the static meshes under the poses
  // they were queried at (dropped when the mesh is released or updated)
  struct WorldTree {
    gdist_pose_t pose;
    DevBuf boxes;
  };
  std::unordered_map<uint64_t, std::vector<WorldTree>> world;
  uint32_t stats = 1;                      // 1: traversals count their work statistics
  uint32_t cand_buf = gd::kCandBuf;        // per-wave candidate buffer capacity used (<= kCandBuf)
  uint32_t one_to_many = 1;                // 0: pairwise refits, 1: shared refit when it refits less, 2: shared
  unsigned long long last_ctl_sum[gd::ST_N] = {};
  gdist_stats_t last{};
  bool busy = false;                       // a server owns the stream and workspace
  // caller-supplied device allocator (gdist_set_allocator); hipMalloc when unset
  void* (*alloc_fn)(size_t, void*) = nullptr;
  void (*free_fn)(void*, void*) = nullptr;
  void* alloc_user = nullptr;
  // asynchronous batches (gdist_query_batch_async), run in order by a worker thread
  struct AsyncBatch {
    std::vector<gdist_query_desc_t> q;
    gdist_result_t* out = nullptr;
    hipEvent_t after = nullptr;            // the caller's stream position to wait for
  };
  std::mutex amu;
  std::condition_variable acv;
  std::deque<AsyncBatch> aq;
  std::thread aworker;
  bool astop = false;
  uint32_t apending = 0;                   // queued or running batches
  gdist_status_t aerr_status = GDIST_OK;   // first failure since the last gdist_sync
  std::string aerr_msg;
};

