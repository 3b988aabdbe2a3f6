// Internal declarations shared by the host library and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gdist.h"
#include "gdist_dev.hpp"

namespace gd {

// Per-query description, written by the host once per query.
// "A" is the tree kept static (its local frame is the query frame); "B" is
// the tree refitted into A's frame.  `swapped` says the caller's mesh a is B.
// One-to-many calls with a shared refit use the world as the query frame:
// then A's tree was refitted into it under TA too, and the narrow phase
// transforms A's triangles by TA (xfA = 1).
struct SlotDesc {
  const float* boxA;    // [2 LA][6], A local frame
  const float* boxB;    // [2 LB][6], refitted into A's frame
  const float* trisA;   // [nA][9] leaf order, A local frame
  const float* trisB;   // [nB][9] leaf order, B local frame
  const uint32_t* origA;
  const uint32_t* origB;
  uint32_t nA, nB, LA, LB;
  uint32_t depthA, depthB;
  uint32_t mode;        // 0 = min, 1 = max
  uint32_t enhanced;    // 1 = enhanced bounds (Sec. 4), 0 = conventional only
  uint32_t swapped;
  uint32_t hint;        // 1: evaluate the triangle pair (hint_a of A, hint_b of B) first
  uint32_t hint_a, hint_b;   // leaf positions (warm start from an earlier query)
  float kappa_u;        // delta = kappa_u * M
  float m_floor;        // least M: bounds the FP32 transform's rounding, which grows with
                        //   B's local coordinates and the translation, not with the query frame
  Xf32 T;               // B local -> query frame (A local), FP32
  Xf32 TA;              // A local -> query frame when xfA (else unused)
  uint32_t xfA;
  double RA[9], tA[3];  // world pose of A, FP64
  double RB[9], tB[3];  // world pose of B, FP64
  double tau;           // tie tolerance (FP64)
  double err_bound;
};

// Per-query mutable state on the device.
struct SlotState {
  uint32_t best;             // float bits: min mode = upper bound of D_min (+delta),
                             // max mode = lower bound of D_max (-delta)
  uint32_t best32;           // float bits of the FP32 narrow-phase optimum (the best candidate
                             // value, taken at re-evaluation)
  float delta;               // FP32 error window
  uint32_t n_ties;
  unsigned long long key_d;  // double bits of the FP64 optimum
  unsigned long long key_pair;  // (caller tri a << 32) | caller tri b of the reported pair
  uint32_t n_admitted;       // candidates that passed the final window
  uint32_t n_cand;           // candidates appended to this slot's region
  uint32_t cand_overflow;    // the region filled up
  uint32_t active;           // the slot's query is in flight (set at admission, cleared at completion)
  uint32_t pair_a, pair_b;   // leaf positions of the reported pair (A, B roles)
};

// Candidate triangle pair for FP64 re-evaluation (positions in leaf order).
struct Cand {
  float d32;
  uint32_t slot;
  uint32_t ia, ib;
};

// ST_BOXES: child boxes read by the expansion, 2^kA + 2^kB per popped entry;
// ST_LTRI: triangles read by the narrow phase, tA + tB per leaf pair.
enum StatIdx {
  ST_POPPED = 0, ST_CHILD = 1, ST_PUSHED = 2, ST_LEAF = 3, ST_TRI = 4, ST_CAND = 5, ST_PEAK = 6, ST_ROUNDS = 7,
  ST_FULL = 8, ST_BOXES = 9, ST_LTRI = 10, ST_N = 11
};

constexpr uint32_t kTraceRounds = 48;
// Entries of a traversal wave's LDS candidate buffer (the "cand_buffer"
// option sets how many of them are used).
constexpr uint32_t kCandBuf = 128;
// A traversal workgroup appends at most its even share of a round's work items
// plus kSegSlack (its waves' last, partial task group); segments are sized
// from this so that the front and leaf-pair buffers cannot overflow.
constexpr uint32_t kSegSlack = 16384;
constexpr uint64_t kStackLimit = 1ull << 31;   // spill-stack entries (32 GiB)
// Front entries expanded per round for segments of `seg` entries and nb
// workgroups (each entry has at most 4 children when the round is large).
// At most 2^29, so a round's work items (4 per entry) stay below 2^31.
inline uint32_t round_cap_for(uint32_t seg, uint32_t nb) {
  uint64_t v = seg > kSegSlack ? (uint64_t)(seg - kSegSlack) * nb / 4u : 0u;
  if (v > (1ull << 29)) v = 1ull << 29;
  return v < 1u ? 1u : (uint32_t)v;
}
// Smallest segment that holds a round of `budget` work items beyond the
// clamped minimum of one level per side.
inline uint32_t min_segment(uint32_t budget, uint32_t nb) { return kSegSlack + 64u + budget / (nb ? nb : 1u); }

constexpr uint32_t kBarGroups = 8;    // grid-barrier groups (the XCDs, when workgroups go round-robin)
constexpr uint32_t kBarStride = 32;   // words between two groups' barrier words (128 bytes)

// Control block of one persistent traversal launch.
struct Ctl {
  uint32_t overflow;       // bit 0 front, bit 1 leaf pairs, bit 2 candidates, bit 3 spill stack
  uint32_t abort;          // a grid barrier timed out
  uint32_t bar_count;
  uint32_t bar_gen;
  uint32_t rounds_done;    // rounds completed by the latest launch
  uint32_t stack_top[2];   // spill-stack height at the start of a round of parity i
  uint32_t round_base;     // rounds run by earlier stepped launches (serving); a launch's
                           //   first round is round0 + round_base
  unsigned long long stats[ST_N];
  // per-round device timestamps (constant-rate wall clock) and front sizes
  unsigned long long trace_t[kTraceRounds];
  unsigned long long trace_end;
  uint32_t trace_n[kTraceRounds];
  uint32_t trace_nl[kTraceRounds];
  // two-level grid barrier: workgroup b arrives at group b % kBarGroups, whose
  // counter and generation word each own a 128-byte line
  uint32_t bar_grp[kBarGroups * kBarStride];
  uint32_t bar_ggen[kBarGroups * kBarStride];
};

struct TravParams {
  const SlotDesc* desc;
  SlotState* st;
  gdist_result_t* res;
  uint4* front[2];         // segmented: workgroup b owns [b * seg_front, (b+1) * seg_front); segment
  uint4* leaf[2];          //   nblocks (the last) receives the root pairs of newly admitted queries
  uint32_t* fcount[2];     // entry count of every segment of front[i] (nblocks + 1 each)
  uint32_t* lcount[2];
  uint4* stack;            // spill stack: front entries beyond round_cap wait here (LIFO)
  uint32_t stack_cap;      // entries
  uint32_t round_cap;      // most front entries expanded in one round (bounds every segment's output)
  Cand* cand;              // per-slot regions of cand_per_slot entries
  double* cand_d64;
  Ctl* ctl;
  const uint32_t* slot_list;  // slots to admit / re-evaluate (nullptr: slots 0 .. n_list-1)
  uint32_t n_list;
  uint32_t seg_front, seg_leaf, cand_per_slot;
  uint32_t nblocks;        // workgroups of the traversal launch
  uint32_t n_slots;        // size of the slot table
  uint32_t expand_budget;
  uint32_t k_cap;
  uint32_t spin_limit;
  uint32_t round0;         // global index of the first round of this launch (buffer parity)
  uint32_t max_rounds;     // rounds this launch may run (the serving step)
  uint32_t cand_stop;      // 1: a candidate-region overflow also stops the launch (the caller retries
                           //    with larger regions); 0: it only marks the slot
  const uint32_t* finish;  // re-evaluation over slots 0 .. n_list-1 where finish[slot] == 1
                           //   (nullptr: every listed slot)
  uint32_t stats;          // 1: count the work statistics (ST_*; rounds and the peak always)
  uint32_t cand_buf;       // candidates a wave keeps in LDS before they go to memory (0..128)
};

// Head of the report of one serving step (device buffer, copied to pinned
// host memory at the step's end); per-slot arrays follow at offsets the host
// computes: live entries (u32), completion flags (u32), results.
struct StepHead {
  uint32_t overflow;       // the traversal's Ctl::overflow and Ctl::abort
  uint32_t abort;
  uint32_t rounds_done;
  uint32_t pad;
};

// build.hip
// Vertex pass: vb = 7 ints (vertex box as ordered floats, largest vertex norm);
// flags = 2 if a vertex is not finite, else 0.  part: vertex_pass_scratch_bytes()
// of device scratch.
size_t vertex_pass_scratch_bytes();
hipError_t launch_vertex_pass(const float* v, uint32_t nv, int* vb, uint32_t* flags, int* part, hipStream_t s);
// Sort key of a mesh of nt triangles: Morton code (axis_bits per axis) above
// index_bits bits of triangle index, 3 axis_bits + index_bits <= 64.
struct KeyLayout {
  uint32_t index_bits, axis_bits;
};
KeyLayout key_layout(uint32_t nt);
// Packed key of every triangle; flags bit 0 = a vertex index >= nv.  Needs vb
// from launch_vertex_pass.
hipError_t launch_keys(const float* v, uint32_t nv, const uint32_t* f, uint32_t nt, const int* vb, uint64_t* keys,
                       uint32_t* flags, hipStream_t s);
// One-sweep LSD sort of n distinct u64 keys by bits [lo_bit, lo_bit + nbits),
// 8 bits per pass, ping-pong between the two buffers (*result_in_tmp says which
// holds the result).  ws: sort_workspace_bytes(n) of device memory (cleared
// here); after the stream reaches the end of the sort, *sort_timeout_flag(ws)
// is nonzero if a look-back wait gave up (the order is then invalid).
size_t sort_workspace_bytes(uint32_t n);
const uint32_t* sort_timeout_flag(const void* ws);
hipError_t launch_sort(uint64_t* keys, uint64_t* keys_tmp, uint32_t n, uint32_t lo_bit, uint32_t nbits, void* ws,
                       hipStream_t s, int* result_in_tmp);
// The tree of a new mesh from its sorted keys: triangles in key order (index =
// the low index_bits bits of each key), their caller indices, their vertex
// index triples if fl is set, and every node box (L = 2^floor(log2 nt)
// leaves).  Vertex indices are clamped to nv - 1 for the reads (a mesh with a
// larger one is rejected by the key pass's flag).
hipError_t launch_emit_tree(const float* v, uint32_t nv, const uint32_t* f, uint32_t nt, const uint64_t* sorted,
                            uint32_t index_bits, uint32_t L, float* tris, uint32_t* orig, uint32_t* fl, float* boxes,
                            hipStream_t s);
// Deformable meshes: triangles (leaf order) gathered from new vertices through
// the leaf-order index triples fl that launch_emit wrote.
hipError_t launch_gather_tris(const float* v, const uint32_t* fl, uint32_t nt, float* tris, hipStream_t s);

// refit.hip
hipError_t launch_refit(const float* tris, uint32_t n, uint32_t L, const Xf32& T, float* boxes, hipStream_t s);
// Upper levels of a tree whose level of `count` nodes (ids count .. 2 count - 1)
// is already written.
hipError_t launch_reduce_upper(float* boxes, uint32_t count, hipStream_t s);

// One tree of a batched refit: its triangles (leaf order), its output boxes,
// the transform; S and first_block are filled by the planner.
struct RefitJob {
  const float* tris;
  float* boxes;
  Xf32 T;
  uint32_t n, L, S, first_block;
};
struct ReduceJob {
  float* boxes;
  uint32_t first, S, first_block, pad;
};
constexpr uint32_t kMaxRefitPasses = 8;
struct RefitPlan {
  size_t leaf_off;
  uint32_t leaf_blocks, njobs, npasses;
  size_t pass_off[kMaxRefitPasses];
  uint32_t pass_jobs[kMaxRefitPasses], pass_blocks[kMaxRefitPasses];
};
size_t plan_refit_batch(const RefitJob* in, uint32_t njobs, void* staging, size_t cap, RefitPlan* plan);
hipError_t launch_refit_batch(const RefitPlan& plan, const void* dev, hipStream_t s);

// traverse.hip
hipError_t traverse_grid(int device, uint32_t blocks_per_cu, uint32_t* blocks, uint32_t* threads);
hipError_t launch_traverse(const TravParams& p, uint32_t blocks, uint32_t threads, hipStream_t s);
hipError_t launch_reeval(const TravParams& p, hipStream_t s);
hipError_t launch_reset(const TravParams& p, hipStream_t s);
hipError_t launch_admit(const TravParams& p, hipStream_t s);
hipError_t launch_slot_hist(const TravParams& p, uint32_t* live, hipStream_t s);
static_assert(sizeof(SlotDesc) % 4 == 0, "descriptors are copied in 4-byte words");
hipError_t launch_put_desc(const SlotDesc* stage, const uint32_t* list, uint32_t n, SlotDesc* desc, hipStream_t s);
// The part of a serving step after its traversal launch: report head and
// round advance, per-slot live counts, completion flags, FP64 re-evaluation
// of the slots that completed (results in p.res).  Every launch has a fixed
// shape, so the sequence can be replayed from a graph.
hipError_t launch_step_tail(const TravParams& p, StepHead* head, uint32_t* live, uint32_t* finish, hipStream_t s);
// Adds a root kernel node for a traversal launch with the cooperative attribute.
hipError_t add_traverse_node(hipGraph_t g, const TravParams& p, uint32_t blocks, uint32_t threads,
                             hipGraphNode_t* node);

// selfcheck.hip
hipError_t launch_eval_bounds(uint32_t n, const float* a, const float* b, float* out, hipStream_t s);
hipError_t launch_eval_tri_tri(uint32_t n, const float* p, const float* q, uint32_t mode, float* o32, double* o64,
                               hipStream_t s);

}  // namespace gd
