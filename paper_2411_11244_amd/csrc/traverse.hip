// Persistent BVH-vs-BVH traversal (gDist Alg. 1 and Alg. 2, Sec. 5-6) for a
// set of queries ("slots"), followed by the FP64 re-evaluation of the
// surviving candidates.  One cooperative launch runs the whole loop: the
// front length that the paper reads back to the host every iteration is read
// on the device, so the host does not synchronise inside a query.
//
// Before the rounds, one wave per query descends greedily from the root pair
// (always into the child pair with the best bound) to one leaf pair and
// evaluates its triangles: the running best starts close to the optimum, so
// the breadth-first rounds cull with a tight bound from the first level on.
//
// Round r (all workgroups, grid-stride over 64-item waves):
//   * expansion of the front: with n entries, k = largest value with
//     4^k n < C, clamped to [1, k_cap] (Sec. 5); lane t of the round handles
//     entry t >> 2k and the descendant pair named by the low 2k bits of t
//     (Sec. 6.3).  The 2k levels are shared between the two trees so both
//     reach their leaves (a side at its leaf level gives its budget to the
//     other).  Children are culled against the running best with the
//     conventional lower bound; the enhanced upper bound improves the best
//     (Alg. 2, Sec. 6.1).  Leaf-leaf survivors go to the narrow phase.
//   * narrow phase on the leaf pairs emitted in round r-1, one lane per
//     triangle pair (leaves hold 1 or 2 triangles, so 4 lanes per leaf pair).
//     A cheap separating-axis lower bound (the two triangle planes and the
//     centroid axis) rejects most pairs; the survivors are packed into a
//     per-wave LDS queue and the exact triangle-triangle distance runs on
//     full waves of 64 queued pairs.
//   * survivors are appended with one atomic per wave (ballot + mbcnt
//     compaction); the best is kept as float bits with integer atomics after
//     a wave-level reduction (Sec. 6.4).
//   * grid barrier, swap the double buffers.
//
// FP32 policy (the paper computes in FP32 without an error analysis and
// forbids enlarging boxes, Sec. 4): boxes stay tight, and every FP32 value is
// widened by delta = kappa 2^-24 M (M = largest coordinate magnitude of the
// two root boxes) in the conservative direction: a pair is culled only when
// lower - delta > best, the best is improved only with upper + delta, and a
// triangle pair becomes a candidate when d32 - delta <= best.  Max mode is the
// mirror image (Sec. 3: the maximum is computed symmetrically).
#include <cstring>

#include "internal.hpp"

namespace gd {

constexpr int kTravThreads = 256;                 // helper kernels
constexpr int kWavesPerBlock = kTravThreads / kWave;
constexpr int kTravBlock = 1024;                  // k_traverse: one 16-wave workgroup per CU
constexpr int kTravWaves = kTravBlock / kWave;
constexpr uint32_t kQueue = 320;  // per-wave LDS queue of triangle pairs (63 + 4 x 64)
constexpr int kRows = 8;          // expansion rows per wave iteration (one lane per child pair)
constexpr int kEntRows = 1;       // k = 1 rounds: rows of input entries per wave iteration (4 children each)
static_assert(kTravWaves * kRows * 64 + 256 <= (int)kSegSlack, "segment slack below one task group per wave");
static_assert(kEntRows * 4 <= kRows, "a k = 1 task appends no more than a child-pair task");

__device__ __forceinline__ uint32_t ld_rlx(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rlx(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid-wide barrier for a cooperative launch, in two levels.  The workgroup
// barrier orders every wave's writes before thread 0's device-scope release;
// thread 0 then arrives at its group's counter (group = workgroup index mod
// 8, the XCD of a round-robin placement); the last of a group resets that
// counter and arrives at the top counter; the last group's leader publishes
// the next generation in every group's word.  Thread 0 waits on its group's
// word with a bounded spin (a timeout raises `abort` so every wave still
// reaches the end of the kernel) and acquires at device scope for the whole
// workgroup before the closing workgroup barrier.  One counter per group
// instead of one for the grid: device-scope atomics on one word serialise at
// tens of ns each, so 256 arrivals on one word cost several microseconds per
// round, and 32 on each of eight words plus 8 on the top word a fraction.
__device__ void grid_sync(Ctl* c, uint32_t spin_limit) {
  // every wave's stores have reached L2 (vmcnt counts stores on this target)
  // before the workgroup barrier, so thread 0's L2 writeback covers them
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __builtin_amdgcn_s_waitcnt(0);
    const uint32_t groups = gridDim.x < kBarGroups ? gridDim.x : kBarGroups;
    const uint32_t g = blockIdx.x % kBarGroups;
    const uint32_t members = (gridDim.x - g + kBarGroups - 1u) / kBarGroups;
    uint32_t* const gen_word = &c->bar_ggen[g * kBarStride];
    const uint32_t gen = ld_rlx(gen_word);
    // relaxed arrivals: the release fence above already orders this
    // workgroup's writes before them (each cache writeback and invalidate is
    // a round's fixed cost, so every workgroup does one of each)
    const uint32_t arrived = __hip_atomic_fetch_add(&c->bar_grp[g * kBarStride], 1u, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
    bool wait = true;
    if (arrived == members - 1u) {
      // the group's last arrival: every member has arrived (and no member can
      // arrive again before the generation changes), so the counter resets;
      // it acquires the members' releases and releases them upward
      st_rlx(&c->bar_grp[g * kBarStride], 0u);
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
      const uint32_t top = __hip_atomic_fetch_add(&c->bar_count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (top == groups - 1u) {
        // the last group: acquire every group's release, reset, publish
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        st_rlx(&c->bar_count, 0u);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        for (uint32_t h = 0; h < groups; ++h) st_rlx(&c->bar_ggen[h * kBarStride], gen + 1u);
        wait = false;
      }
    }
    if (wait) {
      // relaxed polling: an acquire load here would invalidate L2 on every
      // poll; the single acquire fence below orders the reads that follow
      uint32_t spins = 0;
      while (ld_rlx(gen_word) == gen) {
        __builtin_amdgcn_s_sleep(2);
        if (++spins > spin_limit) {
          st_rlx(&c->abort, 1u);
          break;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

__device__ __forceinline__ uint32_t first_lane(uint64_t m) { return (uint32_t)__builtin_ctzll(m); }

// Improve the running bound of a slot: min mode lowers it, max mode raises it.
// The active lanes are grouped by slot, up to four groups (the slots of the
// lowest remaining lanes): each group reduces over the wave and its first lane
// issues one atomic, only if that improves the bound; lanes of further slots
// issue one each.  (Waves of batched calls mix slots; one atomic per lane on
// the word of a busy slot serialises.)  lds_copy, if set, is this workgroup's
// LDS copy of the bounds, updated the same way and with the value read from
// memory.
__device__ __forceinline__ void improve_bound(uint32_t* target_base, size_t stride_words, bool act, uint32_t slot,
                                              uint32_t mode, float v, uint32_t lane, uint32_t* lds_copy = nullptr) {
  uint64_t am = __ballot(act);
  if (am == 0) return;
#pragma unroll
  for (int it = 0; it < 4; ++it) {
    if (am == 0ull) break;
    const uint32_t fl = first_lane(am);
    const uint32_t s0 = lane_value(slot, fl);
    const uint32_t m0 = lane_value(mode, fl);
    const uint64_t grp = __ballot(act && slot == s0) & am;
    const bool in = (grp >> lane) & 1ull;
    float r = in ? v : (m0 == 0 ? __builtin_huge_valf() : 0.f);
    r = m0 == 0 ? wave_min(r) : wave_max(r);
    if (lane == fl) {
      uint32_t* t = target_base + stride_words * s0;
      // the bound in memory, read to skip an atomic that cannot help, also
      // tightens the workgroup's copy (other workgroups' progress this round)
      const uint32_t g = ld_rlx(t);
      if (m0 == 0) {
        if (fbits(r) < g) atomicMin(t, fbits(r));
        if (lds_copy) atomicMin(&lds_copy[s0], fbits(r) < g ? fbits(r) : g);
      } else {
        if (fbits(r) > g) atomicMax(t, fbits(r));
        if (lds_copy) atomicMax(&lds_copy[s0], fbits(r) > g ? fbits(r) : g);
      }
    }
    am &= ~grp;
  }
  if ((am >> lane) & 1ull) {
    uint32_t* t = target_base + stride_words * slot;
    if (mode == 0) {
      atomicMin(t, fbits(v));
      if (lds_copy) atomicMin(&lds_copy[slot], fbits(v));
    } else {
      atomicMax(t, fbits(v));
      if (lds_copy) atomicMax(&lds_copy[slot], fbits(v));
    }
  }
}

// Append the lanes with `take` set to buf[counter..] with one atomic per wave.
template <typename E>
__device__ __forceinline__ void append(bool take, const E& e, E* buf, uint32_t* counter, uint32_t cap,
                                       uint32_t* overflow, uint32_t ovf_bit, uint32_t lane, uint64_t lt) {
  uint64_t m = __ballot(take);
  if (m == 0ull) return;
  uint32_t cnt = (uint32_t)__popcll(m);
  uint32_t base = 0;
  if (lane == 0) {
    base = atomicAdd(counter, cnt);
    if (base + cnt > cap) atomicOr(overflow, ovf_bit);
  }
  base = lane_value(base, 0);
  if (take) {
    uint32_t idx = base + (uint32_t)__popcll(m & lt);
    if (idx < cap) buf[idx] = e;
  }
}

// Per-wave counters (wave-uniform values), flushed to LDS once per kernel.
// The launch without statistics instantiates ON = false, where counting
// compiles to nothing.
template <bool ON>
struct WaveStats {
  uint32_t v[ST_N];
};
template <bool ON>
__device__ __forceinline__ void add_stat(WaveStats<ON>& ws, int idx, bool pred) {
  if constexpr (ON) ws.v[idx] += (uint32_t)__popcll(__ballot(pred));
}
// Per-lane byte-count operands (summed over the wave once per round): child
// boxes read per popped entry and triangles read per leaf pair.
template <bool ON>
struct LaneStats {
  uint32_t boxes, ltris;
};
template <bool ON>
__device__ __forceinline__ void add_boxes(LaneStats<ON>& ls, uint32_t v) {
  if constexpr (ON) ls.boxes += v;
}
template <bool ON>
__device__ __forceinline__ void add_ltris(LaneStats<ON>& ls, uint32_t v) {
  if constexpr (ON) ls.ltris += v;
}

__device__ __forceinline__ uint32_t level_of(uint32_t node) { return 31u - (uint32_t)__clz(node); }

// Share 2k expansion levels between the two sides (Sec. 6.3 thread mapping):
// each side takes at most k, a side that has fewer levels left gives the rest
// to the other.
__device__ __forceinline__ void split_levels(uint32_t remA, uint32_t remB, uint32_t kk, uint32_t& kA,
                                             uint32_t& kB) {
  uint32_t h = kk / 2;
  kA = remA < h ? remA : h;
  kB = remB < kk - kA ? remB : kk - kA;
  kA = remA < kk - kB ? remA : kk - kB;
}

// Triangle range of leaf node `node` of a tree with n triangles and 2^D leaves.
__device__ __forceinline__ void leaf_range(uint32_t node, uint32_t D, uint32_t n, uint32_t& s, uint32_t& e) {
  uint32_t j = node - (1u << D);
  s = (uint32_t)(((uint64_t)j * n) >> D);
  e = (uint32_t)(((uint64_t)(j + 1) * n) >> D);
}

// A's triangle `pos` in the query frame: A's local frame, or transformed by
// TA when A's tree was refitted too (one-to-many calls in the world frame).
__device__ __forceinline__ void load_tri_a(const float* trisA, bool xfA, const Xf32& TA, uint32_t pos, float* o) {
  if (xfA) load_tri_xf(trisA, pos, TA, o);
  else load_tri(trisA, pos, o);
}

__device__ __forceinline__ void load_pair(const SlotDesc* d, uint32_t pa, uint32_t pb, V3<float>* P, V3<float>* Q) {
  float a[9], b[9];
  load_tri_a(d->trisA, d->xfA != 0u, d->TA, pa, a);
  load_tri_xf(d->trisB, pb, d->T, b);
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    P[v] = mk<float>(a[3 * v], a[3 * v + 1], a[3 * v + 2]);
    Q[v] = mk<float>(b[3 * v], b[3 * v + 1], b[3 * v + 2]);
  }
}

// Lower bound of the distance between triangles P and Q from three candidate
// separating axes: the line through the two centroids, the normal of P and
// the normal of Q.  Both vertex sets are projected onto each axis and the gap
// between the two intervals is the bound: a projection never increases
// distances, whatever direction the axis has, so the FP32 rounding of an
// axis's direction (large for the normal of a sliver) cannot make the bound
// exceed the distance; only the rounding of the projections themselves
// remains, which is a few units of 2^-24 times the coordinates' magnitude,
// inside the error window.  An axis whose squared length is below 1e-30 is
// skipped.  Zero when no axis separates.
//
// The centroid axis alone rejects almost every pair the normals reject (on
// two interlocked tori of 7.5M triangles each, over 100 poses, 8.35e9
// triangle pairs leave 1.15e6 after it and 1.12e6 after all three), so the
// filter tests it first for all of a lane's pairs and computes the normals
// only when some lane of the wave still has a surviving pair.

// Centroid axis: sp and sq are the triangles' vertex sums (three times the centroids).
__device__ __forceinline__ float sep_centroid(const V3<float>* P, V3<float> sp, const V3<float>* Q, V3<float> sq) {
  const V3<float> u = sq - sp;
  const float uu = dot(u, u);
  const float iu = uu >= 1e-30f ? rsqrt32(uu) : 0.f;
  // both sets from P's first vertex
  const float s1 = dot(u, P[1] - P[0]), s2 = dot(u, P[2] - P[0]);
  const float t0 = dot(u, Q[0] - P[0]), t1 = dot(u, Q[1] - P[0]), t2 = dot(u, Q[2] - P[0]);
  const float pmin = fminf(0.f, fminf(s1, s2)), pmax = fmaxf(0.f, fmaxf(s1, s2));
  const float qmin = fminf(t0, fminf(t1, t2)), qmax = fmaxf(t0, fmaxf(t1, t2));
  return fmaxf(fmaxf(qmin - pmax, pmin - qmax) * iu, 0.f);
}

// What depends on one triangle only for the normal axes: its normal, the
// normal's inverse length (0 when degenerate) and the triangle's own interval
// on its normal, measured from its first vertex.
struct TriAxes {
  V3<float> n;
  float inv, lo, hi;
};
__device__ __forceinline__ TriAxes tri_axes(const V3<float>* T) {
  TriAxes t;
  const V3<float> e1 = T[1] - T[0], e2 = T[2] - T[0];
  t.n = cross(e1, e2);
  const float nn = dot(t.n, t.n);
  t.inv = nn >= 1e-30f ? rsqrt32(nn) : 0.f;
  const float p1 = dot(t.n, e1), p2 = dot(t.n, e2);
  t.lo = fminf(0.f, fminf(p1, p2));
  t.hi = fmaxf(0.f, fmaxf(p1, p2));
  return t;
}
// Normal axes of P and Q.
__device__ __forceinline__ float sep_normals(const V3<float>* P, const TriAxes& a, const V3<float>* Q,
                                             const TriAxes& b) {
  // Q's vertices and P's edges, both from P's first vertex
  const V3<float> d0 = Q[0] - P[0], d1 = Q[1] - P[0], d2 = Q[2] - P[0];
  const V3<float> e1 = P[1] - P[0], e2 = P[2] - P[0];
  // P's normal: Q against P's own interval
  const float q0 = dot(a.n, d0), q1 = dot(a.n, d1), q2 = dot(a.n, d2);
  float lb = fmaxf(fminf(q0, fminf(q1, q2)) - a.hi, a.lo - fmaxf(q0, fmaxf(q1, q2))) * a.inv;
  // Q's normal: P from Q's first vertex (P0 - Q0 = -d0, Pk - Q0 = ek - d0) against Q's own interval
  const float c = dot(b.n, d0);
  const float r0 = -c, r1 = dot(b.n, e1) - c, r2 = dot(b.n, e2) - c;
  lb = fmaxf(lb, fmaxf(fminf(r0, fminf(r1, r2)) - b.hi, b.lo - fmaxf(r0, fmaxf(r1, r2))) * b.inv);
  return fmaxf(lb, 0.f);
}

// Zero the control block and the segment counts of the first round's buffers;
// no slot is in flight afterwards.
__global__ void k_reset(TravParams p) {
  uint32_t* w = reinterpret_cast<uint32_t*>(p.ctl);
  for (uint32_t i = threadIdx.x; i < sizeof(Ctl) / 4; i += blockDim.x) w[i] = 0u;
  const uint32_t cur = p.round0 & 1u;
  for (uint32_t i = threadIdx.x; i <= p.nblocks; i += blockDim.x) {
    p.fcount[cur][i] = 0u;
    p.lcount[cur][i] = 0u;
  }
  for (uint32_t i = threadIdx.x; i < p.n_slots; i += blockDim.x) p.st[i].active = 0u;
}

// One wave per admitted query: error window, root bounds, greedy dive, and
// its root pair appended to the admission segment of the next round's input.
__global__ __launch_bounds__(kTravThreads) void k_admit(TravParams p) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t li = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (li >= p.n_list) return;
  const uint32_t s = p.slot_list ? p.slot_list[li] : li;
  const SlotDesc& d = p.desc[s];
  const uint32_t mode = d.mode;
  const bool enh = d.enhanced != 0;
  Box ra = load_box(d.boxA, 1), rb = load_box(d.boxB, 1);
  float M = 0.f;
#pragma unroll
  for (int k = 0; k < 3; ++k)
    M = fmaxf(M, fmaxf(fmaxf(fabsf(ra.lo[k]), fabsf(ra.hi[k])), fmaxf(fabsf(rb.lo[k]), fabsf(rb.hi[k]))));
  M = fmaxf(fmaxf(M, d.m_floor), 0x1p-40f);   // the FP32 square roots need M >= 2^-40
  const float delta = d.kappa_u * M;
  float key, best;
  if (mode == 0) {
    float lo, up;
    bounds_min(ra, rb, enh, lo, up);
    best = up + delta;
    key = lo;
  } else {
    float up, lo;
    bounds_max(ra, rb, enh, up, lo);
    best = fmaxf(lo - delta, 0.f);
    key = up;
  }
  // greedy descent: 64 child pairs (3 levels per side) per step
  uint32_t a = 1u, b = 1u;
  for (int step = 0; step < 64; ++step) {
    uint32_t remA = d.depthA - level_of(a), remB = d.depthB - level_of(b);
    if (remA == 0u && remB == 0u) break;
    uint32_t kA, kB;
    split_levels(remA, remB, 6u, kA, kB);
    const bool act = lane < (1u << (kA + kB));
    const uint32_t ca = (a << kA) | (lane & ((1u << kA) - 1u));
    const uint32_t cb = (b << kB) | ((lane >> kA) & ((1u << kB) - 1u));
    float sel = mode == 0 ? __builtin_huge_valf() : -__builtin_huge_valf();
    float imp = mode == 0 ? __builtin_huge_valf() : 0.f;
    if (act) {
      Box ba = load_box(d.boxA, ca), bb = load_box(d.boxB, cb);
      float x, y;
      if (mode == 0) {
        bounds_min(ba, bb, enh, x, y);
        sel = x;
        imp = y;
      } else {
        bounds_max(ba, bb, enh, x, y);
        sel = x;
        imp = y;
      }
    }
    if (mode == 0) {
      best = fminf(best, wave_min(imp) + delta);
      float ext = wave_min(sel);
      uint32_t L = first_lane(__ballot(act && sel == ext));
      a = lane_value(ca, L);
      b = lane_value(cb, L);
    } else {
      best = fmaxf(best, fmaxf(wave_max(imp) - delta, 0.f));
      float ext = wave_max(sel);
      uint32_t L = first_lane(__ballot(act && sel == ext));
      a = lane_value(ca, L);
      b = lane_value(cb, L);
    }
  }
  {
    uint32_t sa, ea, sb, eb;
    leaf_range(a, d.depthA, d.nA, sa, ea);
    leaf_range(b, d.depthB, d.nB, sb, eb);
    const uint32_t pa = sa + (lane & 1u), pb = sb + ((lane >> 1) & 1u);
    const bool act = lane < 4u && pa < ea && pb < eb;
    float dd = mode == 0 ? __builtin_huge_valf() : 0.f;
    if (act) {
      V3<float> P[3], Q[3];
      load_pair(&d, pa, pb, P, Q);
      dd = sqrt32(mode == 0 ? tri_tri_min_d2<float, false>(P, Q, nullptr, nullptr)
                           : tri_tri_max_d2<float, false>(P, Q, nullptr, nullptr));
    }
    if (mode == 0) best = fminf(best, wave_min(dd) + delta);
    else best = fmaxf(best, fmaxf(wave_max(dd) - delta, 0.f));
  }
  // warm start: the pair an earlier query of the same meshes reported
  if (d.hint && d.hint_a < d.nA && d.hint_b < d.nB) {
    float dd = mode == 0 ? __builtin_huge_valf() : 0.f;
    if (lane == 0) {
      V3<float> P[3], Q[3];
      load_pair(&d, d.hint_a, d.hint_b, P, Q);
      dd = sqrt32(mode == 0 ? tri_tri_min_d2<float, false>(P, Q, nullptr, nullptr)
                           : tri_tri_max_d2<float, false>(P, Q, nullptr, nullptr));
    }
    if (mode == 0) best = fminf(best, wave_min(dd) + delta);
    else best = fmaxf(best, fmaxf(wave_max(dd) - delta, 0.f));
  }
  if (lane == 0) {
    SlotState& st = p.st[s];
    st.delta = delta;
    st.n_ties = 0;
    st.n_admitted = 0;
    st.n_cand = 0;
    st.cand_overflow = 0;
    st.active = 1u;
    st.pair_a = ~0u;
    st.pair_b = ~0u;
    st.key_pair = ~0ull;
    st.best = fbits(best);
    st.best32 = mode == 0 ? fbits(__builtin_huge_valf()) : 0u;
    st.key_d = mode == 0 ? ~0ull : 0ull;
    gdist_result_t& r = p.res[s];
    r.status = GDIST_E_DEVICE;
    r.flags = 0;
    // root pairs enter the next round through the admission segment
    const uint32_t cur = (p.round0 + p.ctl->round_base) & 1u, nb = p.nblocks;
    uint4 e = make_uint4(1u, 1u, fbits(key), s);
    if (d.LA == 1 && d.LB == 1) {
      uint32_t i = atomicAdd(&p.lcount[cur][nb], 1u);
      if (i < p.seg_leaf) p.leaf[cur][(uint64_t)nb * p.seg_leaf + i] = e;
      else atomicOr(&p.ctl->overflow, 2u);
    } else {
      uint32_t i = atomicAdd(&p.fcount[cur][nb], 1u);
      if (i < p.seg_front) p.front[cur][(uint64_t)nb * p.seg_front + i] = e;
      else atomicOr(&p.ctl->overflow, 1u);
    }
  }
}

// Per-workgroup LDS state of the traversal.  Appends of a round go to the
// workgroup's own segment of the output buffers, counted in LDS, so the hot
// loop issues no global atomics; at the round's end each workgroup publishes
// its counts, and the next round maps a global entry index to (segment,
// offset) through an exclusive prefix sum over the workgroups' counts.
constexpr uint32_t kMaxBlocks = 1023;   // segments (+ admission) fit the 1024-point search
constexpr uint32_t kLdsSlots = 512;
constexpr uint32_t kLdsDesc = 256;      // launches of at most this many slots keep their fields in LDS

// The per-slot descriptor fields the expansion and the narrow phase read, kept
// in LDS for the whole launch (a wave whose lanes belong to several queries
// would otherwise gather them per lane from global memory, a dependent round
// trip before every box and triangle load).
struct SlotLds {
  const float* boxA;
  const float* boxB;
  const float* trisA;
  const float* trisB;
  uint32_t mode, depthA, depthB, LA, LB, nA, nB, enh, xfA, pad[3];
  Xf32 T;
};

struct BlockState {
  uint32_t fpre[kMaxBlocks + 2];   // prefix of the current front's segment counts
  uint32_t lpre[kMaxBlocks + 2];   // (workgroup segments + admission segment)
  uint32_t fo, lo;                 // this workgroup's appends in the current round
  uint32_t best[kLdsSlots];        // per-slot running bound (float bits), refreshed each round
  float delta[kLdsSlots];
  unsigned long long stats[ST_N];
  SlotLds sd[kLdsDesc];            // when n_slots <= kLdsDesc
};

struct Round {
  const uint4* fin;
  uint4* fout;
  const uint4* lin;
  uint4* lout;
  uint4* stk;
  uint32_t nb, seg_f, seg_l;
  uint32_t n_in;      // front entries expanded this round (the first n_in by global index)
  uint32_t n_spill;   // front entries [n_in, n_in + n_spill) moved to the stack
  uint32_t st;        // stack height at the round's start
  uint32_t pop_base;  // stack entries [pop_base, st) are expanded after the front's
  bool lds_slots;
};

__device__ __forceinline__ float get_best(const TravParams& p, const BlockState* bs, bool lds, uint32_t slot) {
  return bitsf(lds ? bs->best[slot] : ld_rlx(&p.st[slot].best));
}
__device__ __forceinline__ float get_delta(const TravParams& p, const BlockState* bs, bool lds, uint32_t slot) {
  return lds ? bs->delta[slot] : p.st[slot].delta;
}

// Improve a slot's running bound in memory and in this workgroup's LDS copy.
__device__ __forceinline__ void improve_best(const TravParams& p, BlockState* bs, bool lds, bool act,
                                             uint32_t slot, uint32_t mode, float v, uint32_t lane) {
  improve_bound(&p.st[0].best, sizeof(SlotState) / 4, act, slot, mode, v, lane, lds ? bs->best : nullptr);
}

__device__ __forceinline__ uint32_t wave_uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Largest segment s < nb with pre[s] <= e, for a wave-uniform e < pre[nb]
// (pre is non-decreasing, pre[0] = 0, nb <= 1024).  Two parallel LDS probes
// and ballots instead of a dependent binary search: 64 coarse points 16
// segments apart, then the 16 segments after the last coarse point <= e.
// Needs the whole wave active.
__device__ __forceinline__ uint32_t seg_find_wave(const uint32_t* pre, uint32_t nb, uint32_t e, uint32_t lane) {
  const uint32_t ci = lane << 4;
  const uint32_t c = (uint32_t)__popcll(__ballot(ci < nb && pre[ci] <= e)) - 1u;
  const uint32_t fi = (c << 4) + (lane & 15u);
  const uint32_t f = (uint32_t)__popcll(__ballot(lane < 16u && fi < nb && pre[fi] <= e)) - 1u;
  return (c << 4) + f;
}
// Address s*seg + e - pre[s] of entry e >= pre[s0], stepping forward from the
// segment s0 of the row's first entry (used when a row crosses a segment end).
__device__ __forceinline__ uint32_t seg_addr_from(const uint32_t* pre, uint32_t nb, uint32_t seg, uint32_t s0,
                                                  uint32_t e) {
  uint32_t s = s0;
  while (s + 1u < nb && pre[s + 1u] <= e) ++s;
  return s * seg + (e - pre[s]);
}
// Address of entry e of a row whose entries span [e_first, e_last] (both
// wave-uniform, e_last < pre[nb]); the row usually lies in one segment.
__device__ __forceinline__ uint32_t row_addr(const uint32_t* pre, uint32_t nb, uint32_t seg, uint32_t e_first,
                                            uint32_t e_last, uint32_t e, uint32_t lane) {
  const uint32_t s0 = seg_find_wave(pre, nb, e_first, lane);
  if (pre[s0 + 1u] > e_last) return s0 * seg + (e - pre[s0]);
  return seg_addr_from(pre, nb, seg, s0, e);
}

// Per-query values a lane needs, read once per row: from scalar loads when the
// row's active lanes all belong to one query (the common case: segments hold
// runs of one query's entries), else per lane.
struct SlotView {
  const float* boxA;
  const float* boxB;
  const float* trisA;
  const float* trisB;
  uint32_t mode, depthA, depthB, LA, LB, nA, nB, enh, xfA;
  float delta, best;
};
__device__ __forceinline__ void fill_view(const TravParams& p, const BlockState* bs, bool lds, uint32_t slot,
                                          SlotView& v) {
  if (p.n_slots <= kLdsDesc) {
    const SlotLds& d = bs->sd[slot];
    v.boxA = d.boxA;
    v.boxB = d.boxB;
    v.trisA = d.trisA;
    v.trisB = d.trisB;
    v.mode = d.mode;
    v.depthA = d.depthA;
    v.depthB = d.depthB;
    v.LA = d.LA;
    v.LB = d.LB;
    v.nA = d.nA;
    v.nB = d.nB;
    v.enh = d.enh;
    v.xfA = d.xfA;
    v.delta = get_delta(p, bs, lds, slot);
    v.best = get_best(p, bs, lds, slot);
    return;
  }
  const SlotDesc& d = p.desc[slot];
  v.boxA = d.boxA;
  v.boxB = d.boxB;
  v.trisA = d.trisA;
  v.trisB = d.trisB;
  v.mode = d.mode;
  v.depthA = d.depthA;
  v.depthB = d.depthB;
  v.LA = d.LA;
  v.LB = d.LB;
  v.nA = d.nA;
  v.nB = d.nB;
  v.enh = d.enhanced;
  v.xfA = d.xfA;
  v.delta = get_delta(p, bs, lds, slot);
  v.best = get_best(p, bs, lds, slot);
}
// `act` lanes' slots; lane 0 must be active whenever any lane is.
__device__ __forceinline__ SlotView slot_view(const TravParams& p, const BlockState* bs, bool lds, bool act,
                                              uint32_t slot) {
  SlotView v;
  const uint32_t s_u = wave_uniform(slot);
  if (__ballot(act && slot != s_u) == 0ull) fill_view(p, bs, lds, s_u, v);
  else fill_view(p, bs, lds, slot, v);
  return v;
}

// Exclusive prefix over nb <= 1024 counts, pre[nb] = total, computed by one
// wave (lane l owns counts [16 l, 16 l + 16)): no workgroup barriers.
__device__ __forceinline__ void wave_prefix(const uint32_t* __restrict__ cnt, uint32_t nb, uint32_t* pre,
                                            uint32_t lane) {
  uint32_t v[16], sum = 0;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const uint32_t idx = 16u * lane + i;
    v[i] = idx < nb ? cnt[idx] : 0u;
    sum += v[i];
  }
  uint32_t incl = sum;   // inclusive scan of the lane sums
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t up = __shfl_up(incl, o, 64);
    if (lane >= (uint32_t)o) incl += up;
  }
  uint32_t run = incl - sum;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const uint32_t idx = 16u * lane + i;
    if (idx < nb) pre[idx] = run;
    run += v[i];
  }
  if (lane == 63u) pre[nb] = incl;
}

// Append the lanes flagged in R rows to this workgroup's segment of `buf`
// with one LDS atomic: row r's lanes land after the survivors of rows 0..r-1.
template <int R>
__device__ __forceinline__ void append_rows(const bool* take, const uint4* e, uint4* buf, uint32_t seg,
                                            uint32_t* lds_count, uint32_t* overflow, uint32_t ovf_bit, uint32_t lane,
                                            uint64_t lt) {
  uint64_t m[R];
  uint32_t tot = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    m[r] = __ballot(take[r]);
    tot += (uint32_t)__popcll(m[r]);
  }
  if (tot == 0u) return;
  uint32_t base = 0;
  if (lane == 0) {
    base = atomicAdd(lds_count, tot);
    if (base + tot > seg) atomicOr(overflow, ovf_bit);
  }
  base = lane_value(base, 0);
  uint4* out = buf + (uint64_t)blockIdx.x * seg;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (take[r]) {
      uint32_t idx = base + (uint32_t)__popcll(m[r] & lt);
      if (idx < seg) out[idx] = e[r];
    }
    base += (uint32_t)__popcll(m[r]);
  }
}

// Append up to four entries per lane (those with take[j] set) to this
// workgroup's segment of `buf`, lane after lane, each lane's entries
// contiguous and in order, with one LDS atomic: the children of one parent
// stay adjacent, as in the one-lane-per-child-pair order, so the next round
// reads neighbouring boxes and triangles from neighbouring lanes.
__device__ __forceinline__ void append_runs4(const bool* take, const uint4* e, uint4* buf, uint32_t seg,
                                             uint32_t* lds_count, uint32_t* overflow, uint32_t ovf_bit, uint32_t lane,
                                             uint64_t lt) {
  const uint32_t cnt = (uint32_t)take[0] + (uint32_t)take[1] + (uint32_t)take[2] + (uint32_t)take[3];
  const uint64_t b0 = __ballot(cnt & 1u), b1 = __ballot(cnt & 2u), b2 = __ballot(cnt & 4u);
  const uint32_t tot = (uint32_t)__popcll(b0) + 2u * (uint32_t)__popcll(b1) + 4u * (uint32_t)__popcll(b2);
  if (tot == 0u) return;
  uint32_t base = 0;
  if (lane == 0) {
    base = atomicAdd(lds_count, tot);
    if (base + tot > seg) atomicOr(overflow, ovf_bit);
  }
  base = lane_value(base, 0);
  uint32_t idx = base + (uint32_t)__popcll(b0 & lt) + 2u * (uint32_t)__popcll(b1 & lt) + 4u * (uint32_t)__popcll(b2 & lt);
  uint4* out = buf + (uint64_t)blockIdx.x * seg;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (take[j]) {
      if (idx < seg) out[idx] = e[j];
      ++idx;
    }
  }
}

// Expansion of R consecutive waves' worth of items of the current round's
// input (items it0 + 64 r + lane; item t is child t & (4^k - 1) of input
// entry t >> 2k).  All entry loads of the R rows are issued before any result
// is needed, and the survivors of the R rows are appended together.  Row
// starts and bounds are wave-uniform.
template <int R, bool ON>
__device__ __forceinline__ void expand_rows(const TravParams& p, BlockState* bs, const Round& rd, uint32_t base0,
                                            uint32_t n_items, uint32_t kk, uint32_t lane, uint64_t lt,
                                            WaveStats<ON>& ws, LaneStats<ON>& ls) {
  Ctl* c = p.ctl;
  uint4 ent[R];
  bool act[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t rb = base0 + 64u * r;
    const uint32_t it = rb + lane;
    act[r] = it < n_items;
    ent[r] = make_uint4(1u, 1u, 0u, 0u);
    if (rb < n_items) {
      // input entry ei: the front's first n_in entries, then popped stack entries
      const uint32_t ei = it >> kk, e0 = rb >> kk;
      const uint32_t elast = ((n_items - 1u < rb + 63u ? n_items - 1u : rb + 63u) >> kk);
      if (e0 < rd.n_in) {
        const uint32_t fend = elast < rd.n_in ? elast : rd.n_in - 1u;
        const uint32_t addr = row_addr(bs->fpre, rd.nb, rd.seg_f, e0, fend, ei < rd.n_in ? ei : fend, lane);
        if (act[r]) ent[r] = ei < rd.n_in ? rd.fin[addr] : rd.stk[(uint64_t)rd.pop_base + (ei - rd.n_in)];
      } else if (act[r]) {
        ent[r] = rd.stk[(uint64_t)rd.pop_base + (ei - rd.n_in)];
      }
    }
  }
  bool to_leaf[R], to_front[R];
  uint4 ne[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t it = base0 + 64u * r + lane;
    const uint32_t sub = it & ((1u << kk) - 1u);
    const uint32_t slot = ent[r].w;
    const SlotView v = slot_view(p, bs, rd.lds_slots, act[r], slot);
    const uint32_t mode = v.mode;
    const float delta = v.delta, best = v.best;
    const float key = bitsf(ent[r].z);
    bool a = act[r] && (mode == 0 ? !(key - delta > best) : !(key + delta < best));
    uint32_t kA, kB;
    split_levels(v.depthA - level_of(ent[r].x), v.depthB - level_of(ent[r].y), kk, kA, kB);
    a = a && (sub >> (kA + kB)) == 0u;
    add_stat(ws, ST_POPPED, a && sub == 0u);
    add_stat(ws, ST_CHILD, a);
    add_boxes(ls, (a && sub == 0u) ? (1u << kA) + (1u << kB) : 0u);
    const uint32_t ca = (ent[r].x << kA) | (sub & ((1u << kA) - 1u));
    const uint32_t cb = (ent[r].y << kB) | (sub >> kA);
    bool keep = false;
    float improve = 0.f, nkey = 0.f;
    if (a) {
      const Box ba = load_box(v.boxA, ca), bb = load_box(v.boxB, cb);
      const bool enh = v.enh != 0;
      // (a culled pair's improving bound cannot help: not computed)
      if (mode == 0) {
        nkey = min_lower(ba, bb);
        keep = nkey - delta <= best;
        improve = keep ? min_upper(ba, bb, enh) + delta : __builtin_huge_valf();
      } else {
        nkey = max_upper(ba, bb);
        keep = nkey + delta >= best;
        improve = keep ? fmaxf(max_lower(ba, bb, enh) - delta, 0.f) : 0.f;
      }
    }
    const bool isleaf = (ca >= v.LA) && (cb >= v.LB);
    ne[r] = make_uint4(ca, cb, fbits(nkey), slot);
    to_leaf[r] = a && keep && isleaf;
    to_front[r] = a && keep && !isleaf;
    add_stat(ws, ST_PUSHED, a && keep);
    // only a value that beats the bound this lane already saw can help
    const bool helps = a && (mode == 0 ? improve < best : improve > best);
    improve_best(p, bs, rd.lds_slots, helps, slot, mode, improve, lane);
  }
  append_rows<R>(to_leaf, ne, rd.lout, rd.seg_l, &bs->lo, &c->overflow, 2u, lane, lt);
  append_rows<R>(to_front, ne, rd.fout, rd.seg_f, &bs->fo, &c->overflow, 1u, lane, lt);
}

// One child pair of an expanded entry: cull bound, improving bound, output
// entry.  Boxes ba (of A) and bb (of B); `valid` lanes only.
struct ChildOut {
  bool leaf, front;
  uint4 e;
};
__device__ __forceinline__ void eval_child(const SlotView& v, bool valid, const Box& ba, const Box& bb, uint32_t ca,
                                           uint32_t cb, uint32_t slot, ChildOut& o, float& imp) {
  bool keep = false;
  float nkey = 0.f;
  if (valid) {
    const bool enh = v.enh != 0;
    // the improving bound of a culled pair cannot beat the running bound
    // (it is at least as far from it as the culling bound): not computed
    if (v.mode == 0) {
      nkey = min_lower(ba, bb);
      keep = nkey - v.delta <= v.best;
      if (keep) imp = fminf(imp, min_upper(ba, bb, enh) + v.delta);
    } else {
      nkey = max_upper(ba, bb);
      keep = nkey + v.delta >= v.best;
      if (keep) imp = fmaxf(imp, fmaxf(max_lower(ba, bb, enh) - v.delta, 0.f));
    }
  }
  const bool isleaf = (ca >= v.LA) && (cb >= v.LB);
  o.e = make_uint4(ca, cb, fbits(nkey), slot);
  o.leaf = keep && isleaf;
  o.front = keep && !isleaf;
}

// Expansion in rounds with k = 1, one lane per input entry (items it0 + 64 r
// + lane are input entries here, not child pairs).  The lane reads its entry
// once and the boxes of its children from registers-sized sibling groups,
// then evaluates its (up to) four child pairs: a quarter of the entry loads
// and about half the box loads of one lane per child pair.
//
// The two levels of a round are shared as in the child-pair mapping: one per
// side, or both to one side when the other is at its leaf level.  Call G the
// side that descends further (kG = max(kA, kB), 1 or 2) and S the other
// (kS = 0 or 1): the lane loads G's 2^kG children (one or two sibling pairs,
// 48 bytes each, three 16-byte loads per pair) and S's sibling pair holding
// its 2^kS children (for kS = 0, the pair holding S's own node).  The bounds
// are symmetric in their two boxes (bit for bit: A's and B's per-axis terms
// swap places in commutative sums, minima and maxima), so every child pair is
// evaluated as (G box, S box) whichever side G is, with no branch on the
// split: lanes of one wave may split differently.
// Input entry rb + lane of a k = 1 round (the front's first n_in entries,
// then popped stack entries); a lane past n_ent gets a dummy entry.
__device__ __forceinline__ uint4 entry_row(const BlockState* bs, const Round& rd, uint32_t rb, uint32_t n_ent,
                                           uint32_t lane) {
  const uint32_t ei = rb + lane;
  uint4 e = make_uint4(1u, 1u, 0u, 0u);
  if (rb < n_ent) {
    const uint32_t elast = n_ent - 1u < rb + 63u ? n_ent - 1u : rb + 63u;
    const bool act = ei < n_ent;
    if (rb < rd.n_in) {
      const uint32_t fend = elast < rd.n_in ? elast : rd.n_in - 1u;
      const uint32_t addr = row_addr(bs->fpre, rd.nb, rd.seg_f, rb, fend, ei < rd.n_in ? ei : fend, lane);
      if (act) e = ei < rd.n_in ? rd.fin[addr] : rd.stk[(uint64_t)rd.pop_base + (ei - rd.n_in)];
    } else if (act) {
      e = rd.stk[(uint64_t)rd.pop_base + (ei - rd.n_in)];
    }
  }
  return e;
}

// pre: the first row's entries, already loaded (one task ahead), or nullptr.
template <int R, bool ON>
__device__ __forceinline__ void expand_entries(const TravParams& p, BlockState* bs, const Round& rd, uint32_t base0,
                                               uint32_t n_ent, uint32_t lane, uint64_t lt, WaveStats<ON>& ws,
                                               LaneStats<ON>& ls, const uint4* pre) {
  Ctl* c = p.ctl;
  uint4 ent[R];
  bool act[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t rb = base0 + 64u * r;
    act[r] = rb + lane < n_ent;
    ent[r] = (r == 0 && pre) ? *pre : entry_row(bs, rd, rb, n_ent, lane);
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t x = ent[r].x, y = ent[r].y, slot = ent[r].w;
    const SlotView v = slot_view(p, bs, rd.lds_slots, act[r], slot);
    const uint32_t mode = v.mode;
    const float key = bitsf(ent[r].z);
    const bool a = act[r] && (mode == 0 ? !(key - v.delta > v.best) : !(key + v.delta < v.best));
    uint32_t kA, kB;
    split_levels(v.depthA - level_of(x), v.depthB - level_of(y), 2u, kA, kB);
    const bool gA = kA >= kB;                 // G = A (else B)
    const uint32_t kG = gA ? kA : kB, kS = gA ? kB : kA;
    const bool quad = kG == 2u;
    const uint32_t g = gA ? x : y, sn = gA ? y : x;
    const float* gbox = gA ? v.boxA : v.boxB;
    const float* sbox = gA ? v.boxB : v.boxA;
    const uint32_t gfirst = (g << kG) & ~1u;                // G's first child (kG >= 1: even)
    const uint32_t spair = (sn << kS) & ~1u;                // S's sibling pair
    Box G[4], S2[2];
    if (a) {
      load_box_pair(gbox, gfirst, G);
      load_box_pair(sbox, spair, S2);
    }
    if (a && quad) load_box_pair(gbox, gfirst + 2u, G + 2);
    add_stat(ws, ST_POPPED, a);
    add_boxes(ls, a ? (1u << kA) + (1u << kB) : 0u);
    // S's own node when it stays at its level
    if (kS == 0u && (sn & 1u)) S2[0] = S2[1];
    bool tl[4], tf[4];
    uint4 ne[4];
    float imp = mode == 0 ? __builtin_huge_valf() : 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      // child j: G child gi, S child si (quad: G's four children against S)
      const uint32_t gi = quad ? (uint32_t)j : ((uint32_t)j & 1u);
      const uint32_t si = quad ? 0u : ((uint32_t)j >> 1);
      const bool valid = a && (quad || si <= kS);
      Box gb = G[j & 1], sb = S2[0];
      if (j >= 2) {
        if (quad) gb = G[j];
        else sb = S2[1];
      }
      const uint32_t gc = gfirst | gi, sc = (sn << kS) | si;
      const uint32_t ca = gA ? gc : sc, cb = gA ? sc : gc;
      ChildOut o;
      eval_child(v, valid, gb, sb, ca, cb, slot, o, imp);
      add_stat(ws, ST_CHILD, valid);
      add_stat(ws, ST_PUSHED, o.leaf || o.front);
      tl[j] = o.leaf;
      tf[j] = o.front;
      ne[j] = o.e;
    }
    const bool helps = a && (mode == 0 ? imp < v.best : imp > v.best);
    improve_best(p, bs, rd.lds_slots, helps, slot, mode, imp, lane);
    append_runs4(tl, ne, rd.lout, rd.seg_l, &bs->lo, &c->overflow, 2u, lane, lt);
    append_runs4(tf, ne, rd.fout, rd.seg_f, &bs->fo, &c->overflow, 1u, lane, lt);
  }
}

// Move front entries [n_in + base, n_in + base + 64) onto the spill stack
// (one lane per entry).
__device__ __forceinline__ void spill_wave(const BlockState* bs, const Round& rd, uint32_t base, uint32_t lane) {
  const uint32_t j = base + lane;
  const uint32_t jl = (rd.n_spill - 1u < base + 63u ? rd.n_spill - 1u : base + 63u);
  const uint32_t addr =
      row_addr(bs->fpre, rd.nb, rd.seg_f, rd.n_in + base, rd.n_in + jl, rd.n_in + (j < rd.n_spill ? j : jl), lane);
  if (j < rd.n_spill) rd.stk[(uint64_t)rd.st + j] = rd.fin[addr];
}

// Place candidate number idx of a slot (or flag the slot's region as full).
__device__ __forceinline__ void put_candidate(const TravParams& p, uint32_t slot, uint32_t idx, uint32_t pa,
                                              uint32_t pb, float dd) {
  if (idx < p.cand_per_slot) {
    Cand ce;
    ce.d32 = dd;
    ce.slot = slot;
    ce.ia = pa;
    ce.ib = pb;
    p.cand[(uint64_t)slot * p.cand_per_slot + idx] = ce;
  } else {
    atomicOr(&p.st[slot].cand_overflow, 1u);
    if (p.cand_stop) atomicOr(&p.ctl->overflow, 4u);
  }
}
// Append the flagged lanes' candidates (d32 within the window of their slot's
// bound) to their slots' regions.  The flagged lanes are grouped by slot, up
// to four groups (the slots of the lowest remaining lanes), each taking its
// places with one atomic; lanes of further slots take one each.  Needs the
// whole wave.
__device__ __forceinline__ void add_candidates(const TravParams& p, bool cand, uint32_t slot, uint32_t pa,
                                               uint32_t pb, float dd, uint32_t lane, uint64_t lt) {
  uint64_t m = __ballot(cand);
  if (m == 0ull) return;
#pragma unroll
  for (int it = 0; it < 4; ++it) {
    if (m == 0ull) break;
    const uint32_t fl = first_lane(m);
    const uint32_t s0 = lane_value(slot, fl);
    const uint64_t grp = __ballot(cand && slot == s0) & m;
    uint32_t base = 0u;
    if (lane == fl) base = atomicAdd(&p.st[s0].n_cand, (uint32_t)__popcll(grp));
    base = lane_value(base, fl);
    if ((grp >> lane) & 1ull) put_candidate(p, s0, base + (uint32_t)__popcll(grp & lt), pa, pb, dd);
    m &= ~grp;
  }
  if ((m >> lane) & 1ull) put_candidate(p, slot, atomicAdd(&p.st[slot].n_cand, 1u), pa, pb, dd);
}

// Candidates (pairs whose FP32 value lies inside the window of the slot's
// bound: from the exact stage in min mode, from the filter in max mode) wait
// in the wave's LDS buffer cb (cbn of at most p.cand_buf <= kCandBuf entries,
// wave-uniform) instead
// of taking their places in memory one group at a time: a query whose bound
// moves slowly produces many candidates that the final bound no longer
// admits, and every append is an atomic on the same counter, which
// serialises across the device.  A full
// buffer is first pruned against the slots' current bounds (a bound only
// tightens, so an entry it no longer admits can never be needed again), and
// only flushed if that frees too little; the launch flushes the rest at its
// end, so the FP64 stage (a later launch) sees every candidate the final
// window can hold.  The last prune reads the workgroup's copy of the bounds,
// refreshed at the start of the round that found no work (the final bounds,
// then) or of the launch's last round (a stepped launch), instead of a load
// per wave of one word in memory.
__device__ __forceinline__ void prune_cands(const TravParams& p, const BlockState* bs, bool lds, Cand* cb,
                                            uint32_t& cbn, uint32_t lane, uint64_t lt) {
  uint32_t kept = 0u;   // rows are compacted in order, so a write never lands on an unread entry
#pragma unroll 1
  for (uint32_t r0 = 0u; r0 < cbn; r0 += 64u) {
    const uint32_t i = r0 + lane;
    bool k = i < cbn;
    const Cand e = cb[k ? i : 0u];
    if (k) {
      const uint32_t s = e.slot;
      const uint32_t mode = p.n_slots <= kLdsDesc ? bs->sd[s].mode : p.desc[s].mode;
      const float best = get_best(p, bs, lds, s);
      const float delta = get_delta(p, bs, lds, s);
      k = mode == 0 ? e.d32 - delta <= best : e.d32 + delta >= best;
    }
    const uint64_t m = __ballot(k);
    __builtin_amdgcn_wave_barrier();
    if (k) cb[kept + (uint32_t)__popcll(m & lt)] = e;
    __builtin_amdgcn_wave_barrier();
    kept += (uint32_t)__popcll(m);
  }
  cbn = kept;
}
template <bool ON>
__device__ __forceinline__ void flush_cands(const TravParams& p, Cand* cb, uint32_t& cbn, uint32_t lane, uint64_t lt,
                                            WaveStats<ON>& ws) {
#pragma unroll 1
  for (uint32_t r0 = 0u; r0 < cbn; r0 += 64u) {
    const uint32_t i = r0 + lane;
    const bool a = i < cbn;
    const Cand e = cb[a ? i : 0u];
    add_candidates(p, a, e.slot, e.ia, e.ib, e.d32, lane, lt);
    add_stat(ws, ST_CAND, a);
  }
  __builtin_amdgcn_wave_barrier();
  cbn = 0u;
}
// Put the lanes' candidates (those with `cand` set) into the wave's buffer,
// making room first if they do not fit.
template <bool ON>
__device__ __forceinline__ void buffer_cands(const TravParams& p, const BlockState* bs, bool lds, bool cand,
                                             uint32_t slot, uint32_t pa, uint32_t pb, float dd, uint32_t lane,
                                             uint64_t lt, Cand* cb, uint32_t& cbn, WaveStats<ON>& ws) {
  const uint64_t cm = __ballot(cand);
  if (cm == 0ull) return;
  const uint32_t nc = (uint32_t)__popcll(cm);
  if (cbn + nc > p.cand_buf) {
    prune_cands(p, bs, lds, cb, cbn, lane, lt);
    if (cbn + nc > p.cand_buf) flush_cands(p, cb, cbn, lane, lt, ws);
    if (nc > p.cand_buf) {   // a buffer smaller than the wave's candidates
      add_candidates(p, cand, slot, pa, pb, dd, lane, lt);
      add_stat(ws, ST_CAND, cand);
      return;
    }
  }
  if (cand) {
    Cand ce;
    ce.d32 = dd;
    ce.slot = slot;
    ce.ia = pa;
    ce.ib = pb;
    cb[cbn + (uint32_t)__popcll(cm & lt)] = ce;
  }
  __builtin_amdgcn_wave_barrier();
  cbn += nc;
}

// Narrow phase, stage 1: one lane per leaf pair.  The lane loads the leaf
// pair's 1-2 triangles of each side once.  Min mode: each of the (up to 4)
// triangle pairs gets the cheap separating-axis test, and the survivors go
// onto the wave's LDS queue (at most 4 x 64 per call) for the exact test.
// Max mode: the exact value (the largest of the 9 vertex-pair distances) costs
// no more than a filter, so the lane takes it here, improves the slot's bound
// with its best value and appends its candidates; no max-mode pair is queued.
// (A queued pair costs an LDS round trip and, in a batch, per-lane loads of
// its slot's fields and per-lane atomics on the slot's bound; every max-mode
// pair would pay them.)
// The leaf-pair entries [base, base + 64) of the current round (lane order);
// lanes past n_items get an inactive placeholder.
__device__ __forceinline__ uint4 leaf_row(const BlockState* bs, const Round& rd, uint32_t base, uint32_t n_items,
                                          uint32_t lane) {
  const uint32_t it = base + lane;
  uint4 ent = make_uint4(1u, 1u, 0u, 0u);
  const uint32_t il = n_items - 1u < base + 63u ? n_items - 1u : base + 63u;
  const uint32_t addr = row_addr(bs->lpre, rd.nb, rd.seg_l, base, il, it < n_items ? it : il, lane);
  if (it < n_items) ent = rd.lin[addr];
  return ent;
}

template <bool ON>
__device__ __forceinline__ void narrow_filter_wave(const TravParams& p, BlockState* bs, const Round& rd, uint32_t base,
                                                   uint32_t n_items, uint4 ent, uint32_t lane, uint64_t lt, uint4* q,
                                                   uint32_t& qn, Cand* cb, uint32_t& cbn, WaveStats<ON>& ws,
                                                   LaneStats<ON>& ls) {
  bool act = base + lane < n_items;
  const uint32_t slot = ent.w;
  const SlotView v = slot_view(p, bs, rd.lds_slots, act, slot);
  const uint32_t mode = v.mode;
  const float delta = v.delta, best = v.best;
  const float key = bitsf(ent.z);
  if (act) act = mode == 0 ? !(key - delta > best) : !(key + delta < best);
  add_stat(ws, ST_LEAF, act);
  uint32_t sa = 0, ea = 0, sb = 0, eb = 0;
  if (act) {
    leaf_range(ent.x, v.depthA, v.nA, sa, ea);
    leaf_range(ent.y, v.depthB, v.nB, sb, eb);
    add_ltris(ls, (ea - sa) + (eb - sb));
  }
  V3<float> P[2][3], Q[2][3];
  if (act) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      float a[9], b[9];
      const uint32_t ia = sa + i < ea ? sa + i : sa;
      const uint32_t ib = sb + i < eb ? sb + i : sb;
      load_tri_a(v.trisA, v.xfA != 0u, p.desc[slot].TA, ia, a);
      if (p.n_slots <= kLdsDesc) load_tri_xf(v.trisB, ib, bs->sd[slot].T, b);
      else load_tri_xf(v.trisB, ib, p.desc[slot].T, b);
#pragma unroll
      for (int w = 0; w < 3; ++w) {
        P[i][w] = mk<float>(a[3 * w], a[3 * w + 1], a[3 * w + 2]);
        Q[i][w] = mk<float>(b[3 * w], b[3 * w + 1], b[3 * w + 2]);
      }
    }
  }
  const bool any_max = __ballot(act && mode != 0) != 0ull;   // wave-uniform
  const bool any_min = __ballot(act && mode == 0) != 0ull;
  float imp = 0.f;   // max mode: the lane's best improvement of the bound
  // centroid axis for every pair of the lane (pairs in the order (P0,Q0),
  // (P1,Q0), (P0,Q1), (P1,Q1)); the normal axes only if a pair survives it
  bool pass4[4];
  if (any_min) {
    V3<float> SP[2], SQ[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      SP[i] = (P[i][0] + P[i][1]) + P[i][2];
      SQ[i] = (Q[i][0] + Q[i][1]) + Q[i][2];
    }
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const bool valid = act && mode == 0 && sa + (s4 & 1) < ea && sb + (s4 >> 1) < eb;
      pass4[s4] = valid && sep_centroid(P[s4 & 1], SP[s4 & 1], Q[s4 >> 1], SQ[s4 >> 1]) - delta <= best;
    }
    if (__ballot(pass4[0] || pass4[1] || pass4[2] || pass4[3])) {
      const TriAxes AP0 = tri_axes(P[0]), AP1 = tri_axes(P[1]);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const TriAxes aq = tri_axes(Q[j]);
        if (pass4[2 * j]) pass4[2 * j] = sep_normals(P[0], AP0, Q[j], aq) - delta <= best;
        if (pass4[2 * j + 1]) pass4[2 * j + 1] = sep_normals(P[1], AP1, Q[j], aq) - delta <= best;
      }
    }
  } else {
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) pass4[s4] = false;
  }
#pragma unroll
  for (int s4 = 0; s4 < 4; ++s4) {
    const uint32_t pa = sa + (s4 & 1), pb = sb + (s4 >> 1);
    const bool valid = act && pa < ea && pb < eb;
    const bool pass = pass4[s4];
    add_stat(ws, ST_TRI, valid);
    if (any_max) {
      const bool full = valid && mode != 0;
      bool cand = false;
      float dd = 0.f;
      if (full) {
        dd = sqrt32(tri_tri_max_d2<float, false>(P[s4 & 1], Q[s4 >> 1], nullptr, nullptr));
        imp = fmaxf(imp, fmaxf(dd - delta, 0.f));
        cand = dd + delta >= best;
      }
      // into the wave's candidate buffer while it has room, else straight to
      // memory (no pruning here: that code stays out of the filter)
      const uint64_t cm = __ballot(cand);
      if (cm) {
        const uint32_t nc = (uint32_t)__popcll(cm);
        if (cbn + nc <= p.cand_buf) {
          if (cand) {
            Cand ce;
            ce.d32 = dd;
            ce.slot = slot;
            ce.ia = pa;
            ce.ib = pb;
            cb[cbn + (uint32_t)__popcll(cm & lt)] = ce;
          }
          __builtin_amdgcn_wave_barrier();
          cbn += nc;
        } else {
          add_candidates(p, cand, slot, pa, pb, dd, lane, lt);
          add_stat(ws, ST_CAND, cand);
        }
      }
      add_stat(ws, ST_FULL, full);
    }
    uint64_t m = __ballot(pass);
    if (pass) q[qn + (uint32_t)__popcll(m & lt)] = make_uint4(slot, pa, pb, 0u);
    qn += (uint32_t)__popcll(m);
  }
  __builtin_amdgcn_wave_barrier();
  if (any_max) improve_best(p, bs, rd.lds_slots, act && mode != 0 && imp > best, slot, mode, imp, lane);
}

// Narrow phase, stage 2: exact FP32 triangle-triangle distance on queued pairs
// (the filter queues min-mode pairs only).
template <bool ON>
__device__ __forceinline__ void narrow_full(const TravParams& p, BlockState* bs, bool lds, uint4 e, bool act,
                                            uint32_t lane, uint64_t lt, Cand* cb, uint32_t& cbn, WaveStats<ON>& ws) {
  const uint32_t slot = e.x, pa = e.y, pb = e.z;
  const SlotView v = slot_view(p, bs, lds, act, slot);
  const uint32_t mode = v.mode;
  const float delta = v.delta;
  float dd = 0.f, improve = 0.f;
  bool cand = false;
  if (act) {
    V3<float> P[3], Q[3];
    {
      float a[9], b[9];
      load_tri_a(v.trisA, v.xfA != 0u, p.desc[slot].TA, pa, a);
      if (p.n_slots <= kLdsDesc) load_tri_xf(v.trisB, pb, bs->sd[slot].T, b);
      else load_tri_xf(v.trisB, pb, p.desc[slot].T, b);
#pragma unroll
      for (int w = 0; w < 3; ++w) {
        P[w] = mk<float>(a[3 * w], a[3 * w + 1], a[3 * w + 2]);
        Q[w] = mk<float>(b[3 * w], b[3 * w + 1], b[3 * w + 2]);
      }
    }
    dd = sqrt32(mode == 0 ? tri_tri_min_d2<float, false>(P, Q, nullptr, nullptr)
                         : tri_tri_max_d2<float, false>(P, Q, nullptr, nullptr));
    const float best = v.best;
    if (mode == 0) {
      improve = dd + delta;
      cand = dd - delta <= best;
    } else {
      improve = fmaxf(dd - delta, 0.f);
      cand = dd + delta >= best;
    }
  }
  add_stat(ws, ST_FULL, act);
  buffer_cands(p, bs, lds, act && cand, slot, pa, pb, dd, lane, lt, cb, cbn, ws);
  // only a value that beats the bound this lane already saw can help (the
  // others would cost a device-scope load of a word every wave reads)
  const bool helps = act && (mode == 0 ? improve < v.best : improve > v.best);
  improve_best(p, bs, lds, helps, slot, mode, improve, lane);
  // (the FP32 optimum, best32, is taken by the FP64 stage as the extreme over
  // the candidates: the optimal pair is always one, so nothing is kept here)
}

__device__ __forceinline__ void world_tri(const float* tris, uint32_t pos, const double* R, const double* t,
                                          V3<double>* out) {
  const float* q = tris + 9ull * pos;
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    double x = q[3 * v], y = q[3 * v + 1], z = q[3 * v + 2];
    double w[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) w[r] = ((R[3 * r] * x + R[3 * r + 1] * y) + R[3 * r + 2] * z) + t[r];
    out[v] = mk<double>(w[0], w[1], w[2]);
  }
}

// LDS_SLOTS: the per-query running bound and window live in LDS (n_slots <=
// kLdsSlots); a compile-time choice, so no load has to pick between LDS and
// global memory at run time.
template <bool LDS_SLOTS, bool STATS>
__global__ __launch_bounds__(kTravBlock) void k_traverse(TravParams p) {
  __shared__ BlockState bs_;
  __shared__ uint4 sq[kTravWaves][kQueue];
  __shared__ Cand scb[kTravWaves][kCandBuf];
  BlockState* bs = &bs_;
  Ctl* c = p.ctl;
  const uint32_t tid = threadIdx.x;
  const uint32_t lane = tid & 63u;
  const uint64_t lt = (1ull << lane) - 1ull;
  const uint32_t wib = wave_uniform(tid >> 6);
  const uint32_t gw = blockIdx.x * kTravWaves + wib;
  const uint32_t nw = gridDim.x * kTravWaves;
  uint4* q = sq[wib];
  Cand* cb = scb[wib];
  uint32_t cbn = 0u;   // wave-uniform fill of cb
  constexpr bool lds_slots = LDS_SLOTS;
  WaveStats<STATS> ws;
#pragma unroll
  for (int i = 0; i < ST_N; ++i) ws.v[i] = 0u;
  LaneStats<STATS> ls;
  ls.boxes = 0u;
  ls.ltris = 0u;
  if (tid < ST_N) bs->stats[tid] = 0ull;
  if (tid == 0) {
    bs->fo = 0u;
    bs->lo = 0u;
  }
  if (lds_slots)
    for (uint32_t s = tid; s < p.n_slots; s += kTravBlock) bs->delta[s] = p.st[s].delta;
  if (p.n_slots <= kLdsDesc)
    for (uint32_t s = tid; s < p.n_slots; s += kTravBlock) {
      const SlotDesc& d = p.desc[s];
      SlotLds& o = bs->sd[s];
      o.boxA = d.boxA;
      o.boxB = d.boxB;
      o.trisA = d.trisA;
      o.trisB = d.trisB;
      o.mode = d.mode;
      o.depthA = d.depthA;
      o.depthB = d.depthB;
      o.LA = d.LA;
      o.LB = d.LB;
      o.nA = d.nA;
      o.nB = d.nB;
      o.enh = d.enhanced;
      o.xfA = d.xfA;
      o.T = d.T;
    }
  // nothing in this launch writes round_base (the next stepped launch's base
  // is advanced by a later kernel)
  const uint32_t round0 = p.round0 + c->round_base;

  for (uint32_t r = 0; r < p.max_rounds; ++r) {
    const uint32_t round = round0 + r;     // global round: selects the buffer parity
    // the round's control words, read together (one line of the control
    // block): stop flags and the spill stack's height
    const uint32_t c_abort = ld_rlx(&c->abort), c_ovf = ld_rlx(&c->overflow);
    const uint32_t c_st = ld_rlx(&c->stack_top[round & 1u]);
    if (c_abort || c_ovf) break;
    Round rd;
    rd.nb = gridDim.x + 1u;                // workgroup segments + the admission segment
    rd.seg_f = p.seg_front;
    rd.seg_l = p.seg_leaf;
    rd.lds_slots = lds_slots;
    rd.fin = p.front[round & 1u];
    rd.fout = p.front[(round + 1u) & 1u];
    rd.lin = p.leaf[round & 1u];
    rd.lout = p.leaf[(round + 1u) & 1u];
    rd.stk = p.stack;
    // the slots' running bounds by waves 2.., at the same time as the segment
    // prefixes of this round's inputs by wave 0 (the front) and wave 1 (the
    // leaf pairs)
    if (lds_slots && tid >= 128u)
      for (uint32_t s = tid - 128u; s < p.n_slots; s += kTravBlock - 128u) bs->best[s] = ld_rlx(&p.st[s].best);
    if (wib == 0u) wave_prefix(p.fcount[round & 1u], rd.nb, bs->fpre, lane);
    else if (wib == 1u) wave_prefix(p.lcount[round & 1u], rd.nb, bs->lpre, lane);
    __syncthreads();
    const uint32_t n = bs->fpre[rd.nb];
    const uint32_t nl = bs->lpre[rd.nb];
    // Bounded memory: at most round_cap front entries are expanded per round.
    // A longer front moves its surplus onto the spill stack; a shorter one is
    // topped up from the stack's top (the most recently spilled, i.e. deepest
    // entries), so pending pairs are worked off depth-first in chunks.  Every
    // workgroup derives the same decision from the same counts.
    rd.st = c_st;
    if (n == 0u && nl == 0u && rd.st == 0u) break;
    rd.n_in = n < p.round_cap ? n : p.round_cap;
    rd.n_spill = n - rd.n_in;
    const uint32_t pop = rd.n_spill ? 0u : (rd.st < p.round_cap - rd.n_in ? rd.st : p.round_cap - rd.n_in);
    rd.pop_base = rd.st - pop;
    if ((uint64_t)rd.st + rd.n_spill > (uint64_t)p.stack_cap) {
      if (blockIdx.x == 0 && tid == 0) atomicOr(&c->overflow, 8u);
      break;
    }
    const uint32_t n_exp = rd.n_in + pop;
    if (blockIdx.x == 0 && tid == 0) {
      bs->stats[ST_ROUNDS] += 1ull;
      const unsigned long long live = (unsigned long long)n + rd.st;
      if (live > bs->stats[ST_PEAK]) bs->stats[ST_PEAK] = live;
      if (r < kTraceRounds) {
        c->trace_t[r] = (unsigned long long)wall_clock64();
        c->trace_n[r] = n;
        c->trace_nl[r] = nl;
      }
    }
    // k: the largest value with 4^k n < C, clamped to [1, k_cap] (Sec. 5);
    // item counts stay below 2^32 (the host bounds round_cap and C)
    uint32_t k = p.k_cap;
    while (k > 1u && ((uint64_t)n_exp << (2u * k)) >= (uint64_t)p.expand_budget) --k;
    const uint32_t kk = 2u * k;
    const uint32_t leaf_waves = (nl + 63u) >> 6;   // one lane per leaf pair
    const uint32_t spill_end = leaf_waves + ((rd.n_spill + 63u) >> 6);
    // k = 1: one lane per input entry, else one lane per child pair
    const bool by_entry = kk == 2u;
    const uint32_t exp_items = by_entry ? n_exp : n_exp << kk;
    const uint32_t rows = by_entry ? (uint32_t)kEntRows : (uint32_t)kRows;
    // expansion work is handed out in groups of `rows` waves' worth of items
    const uint32_t total = spill_end + (uint32_t)(((uint64_t)exp_items + 64u * rows - 1u) / (64u * rows));
    uint32_t qn = 0;  // wave-uniform fill of this wave's LDS queue
    // a leaf task's entries, and a k = 1 expansion task's, are loaded one
    // task ahead, so their latency overlaps the previous task's work
    auto row_of = [&](uint32_t ww) -> uint4 {   // ww is wave-uniform
      if (ww < leaf_waves) return leaf_row(bs, rd, ww * 64u, nl, lane);
      if (by_entry && ww >= spill_end && ww < total)
        return entry_row(bs, rd, (ww - spill_end) * 64u * kEntRows, exp_items, lane);
      return make_uint4(1u, 1u, 0u, 0u);
    };
    uint4 pre = row_of(gw);
    for (uint32_t w = gw;;) {
      const bool more = w < total;
      if (more) {
        const uint4 cur = pre;
        if (w + nw < total) pre = row_of(w + nw);
        if (w < leaf_waves) narrow_filter_wave(p, bs, rd, w * 64u, nl, cur, lane, lt, q, qn, cb, cbn, ws, ls);
        else if (w < spill_end) spill_wave(bs, rd, (w - leaf_waves) * 64u, lane);
        else if (by_entry) expand_entries<kEntRows>(p, bs, rd, (w - spill_end) * 64u * kEntRows, exp_items, lane, lt, ws, ls, &cur);
        else expand_rows<kRows>(p, bs, rd, (w - spill_end) * 64u * kRows, exp_items, kk, lane, lt, ws, ls);
        w += nw;
      }
      while (qn >= 64u || (!more && qn > 0u)) {
        const uint32_t take = qn >= 64u ? 64u : qn;
        qn -= take;
        const bool a = lane < take;
        const uint4 e = q[qn + (a ? lane : 0u)];
        __builtin_amdgcn_wave_barrier();
        narrow_full(p, bs, lds_slots, e, a, lane, lt, cb, cbn, ws);
      }
      if (!more) break;
    }
    if constexpr (STATS) {
      // the round's byte-count operands, summed per wave (kept per round so
      // the per-lane 32-bit sums cannot wrap)
      const uint32_t sb = wave_sum(ls.boxes), stt = wave_sum(ls.ltris);
      if (lane == 0u) {
        if (sb) atomicAdd(&bs->stats[ST_BOXES], (unsigned long long)sb);
        if (stt) atomicAdd(&bs->stats[ST_LTRI], (unsigned long long)stt);
      }
      ls.boxes = 0u;
      ls.ltris = 0u;
    }
    // publish this workgroup's output counts for the next round
    __syncthreads();
    if (tid == 0) {
      p.fcount[(round + 1u) & 1u][blockIdx.x] = bs->fo < rd.seg_f ? bs->fo : rd.seg_f;
      p.lcount[(round + 1u) & 1u][blockIdx.x] = bs->lo < rd.seg_l ? bs->lo : rd.seg_l;
      if (blockIdx.x == 0) {
        p.fcount[(round + 1u) & 1u][gridDim.x] = 0u;   // admission segment consumed
        p.lcount[(round + 1u) & 1u][gridDim.x] = 0u;
        st_rlx(&c->stack_top[(round + 1u) & 1u], rd.st + rd.n_spill - pop);
      }
      bs->fo = 0u;
      bs->lo = 0u;
    }
    grid_sync(c, p.spin_limit);
  }
  if (cbn) {   // the buffered candidates the bounds in memory still admit
    prune_cands(p, bs, lds_slots, cb, cbn, lane, lt);
    if (cbn) flush_cands(p, cb, cbn, lane, lt, ws);
  }
  if (blockIdx.x == 0 && tid == 0) {
    c->trace_end = (unsigned long long)wall_clock64();
    c->rounds_done = (uint32_t)bs->stats[ST_ROUNDS];
  }
  if (STATS && lane == 0)
    for (int i = 0; i < ST_N; ++i)
      if (i != ST_ROUNDS && i != ST_PEAK && i != ST_BOXES && i != ST_LTRI && ws.v[i])
        atomicAdd(&bs->stats[i], (unsigned long long)ws.v[i]);

  __syncthreads();
  if (tid < ST_N && bs->stats[tid]) {
    if (tid == ST_PEAK) atomicMax(&c->stats[ST_PEAK], bs->stats[ST_PEAK]);
    else if (tid == ST_ROUNDS) atomicMax(&c->stats[ST_ROUNDS], bs->stats[ST_ROUNDS]);
    else atomicAdd(&c->stats[tid], bs->stats[tid]);
  }
}

// FP64 re-evaluation, in three grid-wide steps (separate launches), over the
// listed slots.  Workgroups [i * G, (i+1) * G) serve the i-th listed slot and
// walk its candidate region.
// A: admit the candidates inside the final window and evaluate them in FP64
//    in the world frame from the caller's FP32 vertices and FP64 poses.
struct ReevalRange {
  uint32_t slot, begin, stride, end;
  bool skip;   // the slot does not complete in this launch
};
__device__ __forceinline__ ReevalRange reeval_range(const TravParams& p, uint32_t G) {
  ReevalRange r;
  const uint32_t i = blockIdx.x / G, part = blockIdx.x % G;
  r.slot = p.slot_list ? p.slot_list[i] : i;
  r.skip = p.finish && p.finish[r.slot] != 1u;
  uint32_t n = p.st[r.slot].n_cand;
  r.end = n < p.cand_per_slot ? n : p.cand_per_slot;
  r.begin = part * kTravThreads + threadIdx.x;
  r.stride = G * kTravThreads;
  return r;
}

// Smallest (take_min) or largest 64-bit value over the wave (every lane active).
__device__ __forceinline__ unsigned long long wave_extreme_u64(unsigned long long v, bool take_min) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long w = __shfl_xor(v, o, kWave);
    v = take_min ? (w < v ? w : v) : (w > v ? w : v);
  }
  return v;
}

__global__ __launch_bounds__(kTravThreads) void k_reeval_values(TravParams p, uint32_t G) {
  Ctl* c = p.ctl;
  if (ld_rlx(&c->abort) || ld_rlx(&c->overflow)) return;
  const ReevalRange rr = reeval_range(p, G);
  if (rr.skip) return;
  const SlotDesc& d = p.desc[rr.slot];
  SlotState& st = p.st[rr.slot];
  const Cand* cands = p.cand + (uint64_t)rr.slot * p.cand_per_slot;
  double* d64 = p.cand_d64 + (uint64_t)rr.slot * p.cand_per_slot;
  const float best = bitsf(ld_rlx(&st.best));
  const bool mn = d.mode == 0;
  // per-thread extremes and counts, reduced over the wave into one atomic per
  // word (every thread of the workgroup serves the same slot; an atomic per
  // candidate on one slot's words serialises when a query has many)
  float b32 = mn ? __builtin_huge_valf() : 0.f;
  unsigned long long kd = mn ? ~0ull : 0ull;
  uint32_t seen = 0u, nadm = 0u;
  for (uint32_t i = rr.begin; i < rr.end; i += rr.stride) {
    Cand cd = cands[i];
    // the FP32 optimum over the tested triangle pairs is the best candidate
    // value (max mode tests its pairs in the filter, which keeps no optimum)
    b32 = mn ? fminf(b32, cd.d32) : fmaxf(b32, cd.d32);
    ++seen;
    const bool adm = mn ? (cd.d32 - st.delta <= best) : (cd.d32 + st.delta >= best);
    if (!adm) {
      d64[i] = -1.0;
      continue;
    }
    V3<double> P[3], Q[3];
    world_tri(d.trisA, cd.ia, d.RA, d.tA, P);
    world_tri(d.trisB, cd.ib, d.RB, d.tB, Q);
    double d2 = mn ? tri_tri_min_d2<double, false>(P, Q, nullptr, nullptr)
                   : tri_tri_max_d2<double, false>(P, Q, nullptr, nullptr);
    double dd = sqrt(d2);
    d64[i] = dd;
    const unsigned long long b = (unsigned long long)__double_as_longlong(dd);   // ordered: dd >= 0
    kd = mn ? (b < kd ? b : kd) : (b > kd ? b : kd);
    ++nadm;
  }
  const uint32_t wseen = wave_sum(seen), wadm = wave_sum(nadm);
  const float wb = mn ? wave_min(b32) : wave_max(b32);
  kd = wave_extreme_u64(kd, mn);
  if (threadIdx.x % kWave == 0u) {
    if (wseen) {
      if (mn) atomicMin(&st.best32, fbits(wb));
      else atomicMax(&st.best32, fbits(wb));
    }
    if (wadm) {
      if (mn) atomicMin(&st.key_d, kd);
      else atomicMax(&st.key_d, kd);
      atomicAdd(&st.n_admitted, wadm);
    }
  }
}

__device__ __forceinline__ unsigned long long caller_pair(const SlotDesc& d, const Cand& cd) {
  uint32_t ta = d.origA[cd.ia], tb = d.origB[cd.ib];
  return d.swapped ? (((unsigned long long)tb << 32) | ta) : (((unsigned long long)ta << 32) | tb);
}

// B: the tie set and its lexicographically smallest caller pair.
__global__ __launch_bounds__(kTravThreads) void k_reeval_ties(TravParams p, uint32_t G) {
  Ctl* c = p.ctl;
  if (ld_rlx(&c->abort) || ld_rlx(&c->overflow)) return;
  const ReevalRange rr = reeval_range(p, G);
  if (rr.skip) return;
  const SlotDesc& d = p.desc[rr.slot];
  SlotState& st = p.st[rr.slot];
  const Cand* cands = p.cand + (uint64_t)rr.slot * p.cand_per_slot;
  const double* d64 = p.cand_d64 + (uint64_t)rr.slot * p.cand_per_slot;
  const double D = __longlong_as_double((long long)st.key_d);
  unsigned long long kp = ~0ull;   // smallest tied caller pair and tie count of this thread
  uint32_t nt = 0u;
  for (uint32_t i = rr.begin; i < rr.end; i += rr.stride) {
    double dd = d64[i];
    if (dd < 0.0) continue;
    if (fabs(dd - D) <= d.tau) {
      const unsigned long long k = caller_pair(d, cands[i]);
      kp = k < kp ? k : kp;
      ++nt;
    }
  }
  const uint32_t wnt = wave_sum(nt);
  kp = wave_extreme_u64(kp, true);
  if (threadIdx.x % kWave == 0u && wnt) {
    atomicMin(&st.key_pair, kp);
    atomicAdd(&st.n_ties, wnt);
  }
}

// C: closest (farthest) points of the reported pair, and the per-query summary.
__global__ __launch_bounds__(kTravThreads) void k_reeval_report(TravParams p, uint32_t G) {
  Ctl* c = p.ctl;
  if (ld_rlx(&c->abort) || ld_rlx(&c->overflow)) return;
  const ReevalRange rr = reeval_range(p, G);
  if (rr.skip) return;
  const SlotDesc& d = p.desc[rr.slot];
  const SlotState& st = p.st[rr.slot];
  const Cand* cands = p.cand + (uint64_t)rr.slot * p.cand_per_slot;
  const double* d64 = p.cand_d64 + (uint64_t)rr.slot * p.cand_per_slot;
  gdist_result_t& res = p.res[rr.slot];
  const double D = __longlong_as_double((long long)st.key_d);
  for (uint32_t i = rr.begin; i < rr.end; i += rr.stride) {
    const double dd = d64[i];
    if (dd < 0.0 || !(fabs(dd - D) <= d.tau)) continue;   // only a tie can be the reported pair
    const Cand cd = cands[i];
    unsigned long long key = caller_pair(d, cd);
    if (key != st.key_pair) continue;
    V3<double> P[3], Q[3], x, y;
    world_tri(d.trisA, cd.ia, d.RA, d.tA, P);
    world_tri(d.trisB, cd.ib, d.RB, d.tB, Q);
    if (d.mode == 0) tri_tri_min_d2<double, true>(P, Q, &x, &y);
    else tri_tri_max_d2<double, true>(P, Q, &x, &y);
    V3<double> qa = d.swapped ? y : x, qb = d.swapped ? x : y;
    res.point_a[0] = qa.x; res.point_a[1] = qa.y; res.point_a[2] = qa.z;
    res.point_b[0] = qb.x; res.point_b[1] = qb.y; res.point_b[2] = qb.z;
    res.tri_a = (uint32_t)(key >> 32);
    res.tri_b = (uint32_t)(key & 0xffffffffull);
    SlotState& sw = p.st[rr.slot];
    sw.pair_a = cd.ia;
    sw.pair_b = cd.ib;
  }
  if (blockIdx.x % G == 0 && threadIdx.x == 0) {
    res.n_candidates = st.n_admitted;
    res.n_ties = st.n_ties;
    res.distance_fp32 = (double)bitsf(st.best32);
    res.err_bound = d.err_bound;
    res.flags = 0;
    if (st.n_admitted == 0u) {
      res.status = GDIST_E_DEVICE;
      res.distance = __longlong_as_double(0x7ff8000000000000ll);
    } else {
      res.distance = D;
      res.status = GDIST_OK;
      res.flags = (st.n_ties > 1u ? GDIST_F_TIED : 0u) | ((d.mode == 0 && D == 0.0) ? GDIST_F_ZERO : 0u);
    }
  }
}

// Live entries per slot in the current front and leaf buffers and on the
// spill stack (after a step, whose launch advanced round_base): workgroup b counts segment b of each (the last
// workgroup the admission segment) and its grid-stride share of the stack in
// LDS, and adds its non-zero counts to live[].
__global__ __launch_bounds__(kTravThreads) void k_slot_hist(TravParams p, uint32_t* __restrict__ live) {
  __shared__ uint32_t h[kLdsSlots];
  if (p.ctl->abort || p.ctl->overflow) return;   // the storage is reset instead
  for (uint32_t i = threadIdx.x; i < p.n_slots; i += kTravThreads) h[i] = 0u;
  __syncthreads();
  const uint32_t cur = (p.round0 + p.ctl->round_base) & 1u, b = blockIdx.x;
  const uint32_t nf = p.fcount[cur][b], nl = p.lcount[cur][b];
  const uint4* fs = p.front[cur] + (uint64_t)b * p.seg_front;
  const uint4* ls = p.leaf[cur] + (uint64_t)b * p.seg_leaf;
  for (uint32_t i = threadIdx.x; i < nf; i += kTravThreads) atomicAdd(&h[fs[i].w], 1u);
  for (uint32_t i = threadIdx.x; i < nl; i += kTravThreads) atomicAdd(&h[ls[i].w], 1u);
  const uint32_t ns = p.ctl->stack_top[cur];
  for (uint32_t i = b * kTravThreads + threadIdx.x; i < ns; i += gridDim.x * kTravThreads)
    atomicAdd(&h[p.stack[i].w], 1u);
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < p.n_slots; i += kTravThreads)
    if (h[i]) atomicAdd(&live[i], h[i]);
}

// Serving step, after its traversal launch: copy the launch's outcome into
// the step report, advance the round base past the rounds it ran, clear the
// per-slot live counts.
__global__ void k_step_advance(TravParams p, StepHead* __restrict__ head, uint32_t* __restrict__ live) {
  Ctl* c = p.ctl;
  if (threadIdx.x == 0) {
    const uint32_t ov = c->overflow, ab = c->abort, rd = c->rounds_done;
    head->overflow = ov;
    head->abort = ab;
    head->rounds_done = rd;
    if (!ov && !ab) c->round_base += rd;
  }
  for (uint32_t i = threadIdx.x; i < p.n_slots; i += blockDim.x) live[i] = 0u;
}

// Serving step completion: an in-flight slot without live entries has
// drained.  finish = 1: re-evaluate it now; 2: its candidate region filled
// up (the host re-runs the query alone); 0: still running or idle.  A
// drained slot leaves flight.  Nothing completes after an overflow or abort.
__global__ void k_step_select(TravParams p, const StepHead* __restrict__ head, const uint32_t* __restrict__ live,
                              uint32_t* __restrict__ finish) {
  const bool stop = head->overflow || head->abort;
  for (uint32_t s = threadIdx.x; s < p.n_slots; s += blockDim.x) {
    SlotState& st = p.st[s];
    uint32_t f = 0u;
    if (!stop && st.active && live[s] == 0u) {
      f = st.cand_overflow ? 2u : 1u;
      st.active = 0u;
    }
    finish[s] = f;
  }
}

// Workgroups per listed slot in the re-evaluation: about 4,096 workgroups in
// all (a slot may hold 10^5 candidates; slots with few exit at once), at most
// 64 per slot.
uint32_t reeval_groups(uint32_t n_list) {
  uint32_t g = 4096u / (n_list ? n_list : 1u);
  return g < 1u ? 1u : (g > 64u ? 64u : g);
}

// Serving admission: descriptor i of a staged block goes to slot list[i]
// (one workgroup per descriptor), so a step's new descriptors need one copy.
__global__ void k_put_desc(const SlotDesc* __restrict__ stage, const uint32_t* __restrict__ list, uint32_t n,
                           SlotDesc* __restrict__ desc) {
  const uint32_t i = blockIdx.x;
  if (i >= n) return;
  const uint32_t* src = reinterpret_cast<const uint32_t*>(stage + i);
  uint32_t* dst = reinterpret_cast<uint32_t*>(desc + list[i]);
  for (uint32_t w = threadIdx.x; w < sizeof(SlotDesc) / 4; w += blockDim.x) dst[w] = src[w];
}

hipError_t launch_put_desc(const SlotDesc* stage, const uint32_t* list, uint32_t n, SlotDesc* desc, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_put_desc<<<n, 64, 0, s>>>(stage, list, n, desc);
  return hipGetLastError();
}

hipError_t launch_reset(const TravParams& p, hipStream_t s) {
  k_reset<<<1, 256, 0, s>>>(p);
  return hipGetLastError();
}

hipError_t launch_admit(const TravParams& p, hipStream_t s) {
  if (p.n_list == 0) return hipSuccess;
  k_admit<<<(p.n_list + kWavesPerBlock - 1) / kWavesPerBlock, kTravThreads, 0, s>>>(p);
  return hipGetLastError();
}

hipError_t launch_slot_hist(const TravParams& p, uint32_t* live, hipStream_t s) {
  if (p.n_slots > kLdsSlots) return hipErrorInvalidValue;
  k_slot_hist<<<p.nblocks + 1, kTravThreads, 0, s>>>(p, live);
  return hipGetLastError();
}

static const void* traverse_fn(const TravParams& p) {
  const bool lds = p.n_slots <= kLdsSlots;
  if (p.stats) return lds ? (const void*)k_traverse<true, true> : (const void*)k_traverse<false, true>;
  return lds ? (const void*)k_traverse<true, false> : (const void*)k_traverse<false, false>;
}

hipError_t traverse_grid(int device, uint32_t blocks_per_cu, uint32_t* blocks, uint32_t* threads) {
  // the smallest occupancy of the four instantiations (slot table in LDS or
  // not, statistics or not): one grid size fits every launch
  const void* fns[4] = {(const void*)k_traverse<true, true>, (const void*)k_traverse<false, true>,
                        (const void*)k_traverse<true, false>, (const void*)k_traverse<false, false>};
  int per_cu = 1 << 20;
  hipError_t e = hipSuccess;
  for (const void* fn : fns) {
    int n = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, kTravBlock, 0);
    if (e != hipSuccess) return e;
    if (n < per_cu) per_cu = n;
  }
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) return e;
  uint32_t b = (uint32_t)per_cu;
  // Every workgroup must be resident at once (grid barrier).  The occupancy
  // count assumes a workgroup's waves spread evenly over a CU's four SIMDs;
  // a workgroup whose wave count is not a multiple of four puts one more wave
  // on some SIMDs, so two of them can need more registers on one SIMD than it
  // has although the count says they fit.  Only then is the grid held to one
  // workgroup per CU.
  if ((kTravBlock / kWave) % 4 != 0 && b > 1u) b = 1u;
  if (blocks_per_cu > 0 && blocks_per_cu < b) b = blocks_per_cu;
  if (b == 0) b = 1;
  uint32_t total = b * (uint32_t)prop.multiProcessorCount;
  if (total > kMaxBlocks) total = kMaxBlocks;   // the per-round prefix lives in LDS
  *blocks = total;
  *threads = kTravBlock;
  return hipSuccess;
}

hipError_t launch_traverse(const TravParams& p, uint32_t blocks, uint32_t threads, hipStream_t s) {
  TravParams pp = p;
  void* args[] = {&pp};
  return hipLaunchCooperativeKernel(traverse_fn(p), dim3(blocks), dim3(threads), args, 0, s);
}

// Graph node of a traversal launch, marked cooperative like launch_traverse.
hipError_t add_traverse_node(hipGraph_t g, const TravParams& p, uint32_t blocks, uint32_t threads,
                             hipGraphNode_t* node) {
  TravParams pp = p;
  void* args[] = {&pp};
  hipKernelNodeParams kp;
  std::memset(&kp, 0, sizeof(kp));
  kp.func = const_cast<void*>(traverse_fn(p));
  kp.gridDim = dim3(blocks);
  kp.blockDim = dim3(threads);
  kp.kernelParams = args;
  hipError_t e = hipGraphAddKernelNode(node, g, nullptr, 0, &kp);
  if (e != hipSuccess) return e;
  hipKernelNodeAttrValue v;
  std::memset(&v, 0, sizeof(v));
  v.cooperative = 1;
  return hipGraphKernelNodeSetAttribute(*node, hipKernelNodeAttributeCooperative, &v);
}

hipError_t launch_step_tail(const TravParams& p, StepHead* head, uint32_t* live, uint32_t* finish, hipStream_t s) {
  if (p.n_slots > kLdsSlots) return hipErrorInvalidValue;
  k_step_advance<<<1, 256, 0, s>>>(p, head, live);
  k_slot_hist<<<p.nblocks + 1, kTravThreads, 0, s>>>(p, live);
  k_step_select<<<1, 512, 0, s>>>(p, head, live, finish);
  TravParams q = p;
  q.slot_list = nullptr;
  q.n_list = p.n_slots;
  q.finish = finish;
  return launch_reeval(q, s);
}

hipError_t launch_reeval(const TravParams& p, hipStream_t s) {
  if (p.n_list == 0) return hipSuccess;
  const uint32_t G = reeval_groups(p.n_list);
  k_reeval_values<<<p.n_list * G, kTravThreads, 0, s>>>(p, G);
  k_reeval_ties<<<p.n_list * G, kTravThreads, 0, s>>>(p, G);
  k_reeval_report<<<p.n_list * G, kTravThreads, 0, s>>>(p, G);
  return hipGetLastError();
}

}  // namespace gd
