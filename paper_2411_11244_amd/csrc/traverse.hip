// Persistent BVH-vs-BVH traversal (gDist Alg. 1 and Alg. 2, Sec. 5-6) for a
// set of queries ("slots"), followed by the FP64 re-evaluation of the
// surviving candidates.  One cooperative launch runs the whole loop: the
// front length that the paper reads back to the host every iteration is read
// on the device, so the host does not synchronise inside a query.
//
// Round r (all workgroups, grid-stride over 64-item waves):
//   * narrow phase on the leaf pairs emitted in round r-1: one lane per
//     triangle pair (leaves hold 1 or 2 triangles, so 4 lanes per leaf pair);
//     exact FP32 distance, running best improved, candidates appended;
//   * expansion of the front: with n entries, k = largest value with
//     4^k n < C, clamped to [1, k_cap] (Sec. 5); lane t of the round handles
//     entry t >> 2k and the descendant pair named by the low 2k bits of t
//     (Sec. 6.3).  The 2k levels are shared between the two trees so both
//     reach their leaves (a side at its leaf level gives its budget to the
//     other).  Children are culled against the running best with the
//     conventional lower bound; the enhanced upper bound improves the best
//     (Alg. 2, Sec. 6.1).
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
#include "internal.hpp"

namespace gd {

constexpr int kTravThreads = 256;

__device__ __forceinline__ uint32_t ld_rlx(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rlx(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid-wide barrier for a cooperative launch.  Every thread releases its
// writes at device scope before the workgroup barrier; one thread per
// workgroup arrives and waits with a bounded spin (a timeout raises `abort`
// so every wave still reaches the end of the kernel).
__device__ void grid_sync(Ctl* c, uint32_t spin_limit) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t gen = ld_rlx(&c->bar_gen);
    uint32_t arrived = __hip_atomic_fetch_add(&c->bar_count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == gridDim.x - 1) {
      st_rlx(&c->bar_count, 0u);
      __hip_atomic_store(&c->bar_gen, gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      uint32_t spins = 0;
      while (__hip_atomic_load(&c->bar_gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        __builtin_amdgcn_s_sleep(2);
        if (++spins > spin_limit) {
          st_rlx(&c->abort, 1u);
          break;
        }
      }
    }
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

__device__ __forceinline__ uint32_t first_lane(uint64_t m) { return (uint32_t)__builtin_ctzll(m); }

// Improve the running bound of a slot: min mode lowers it, max mode raises it.
// A wave whose active lanes share one slot reduces first and issues one atomic.
__device__ __forceinline__ void improve_bound(uint32_t* target_base, size_t stride_words, bool act, uint32_t slot,
                                              uint32_t mode, float v, uint32_t lane) {
  uint64_t am = __ballot(act);
  if (am == 0) return;
  uint32_t fl = first_lane(am);
  uint32_t s0 = __shfl(slot, fl, 64);
  uint32_t m0 = __shfl(mode, fl, 64);
  if (__ballot(act && slot != s0) == 0ull) {
    float r = act ? v : (m0 == 0 ? __builtin_huge_valf() : 0.f);
    r = m0 == 0 ? wave_min(r) : wave_max(r);
    if (lane == fl) {
      uint32_t* t = target_base + stride_words * s0;
      if (m0 == 0) {
        if (fbits(r) < ld_rlx(t)) atomicMin(t, fbits(r));
      } else {
        if (fbits(r) > ld_rlx(t)) atomicMax(t, fbits(r));
      }
    }
  } else if (act) {
    uint32_t* t = target_base + stride_words * slot;
    if (mode == 0) atomicMin(t, fbits(v));
    else atomicMax(t, fbits(v));
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
  base = __shfl(base, 0, 64);
  if (take) {
    uint32_t idx = base + (uint32_t)__popcll(m & lt);
    if (idx < cap) buf[idx] = e;
  }
}

__device__ __forceinline__ void add_stat(unsigned long long* s, int idx, bool pred, uint32_t lane) {
  uint64_t m = __ballot(pred);
  if (lane == 0 && m) atomicAdd(&s[idx], (unsigned long long)__popcll(m));
}

__global__ void k_init(TravParams p) {
  Ctl* c = p.ctl;
  if (threadIdx.x == 0) {
    for (int i = 0; i < 3; ++i) {
      c->front_len[i] = 0;
      c->leaf_len[i] = 0;
    }
    c->cand_len = 0;
    c->overflow = 0;
    c->abort = 0;
    c->bar_count = 0;
    c->bar_gen = 0;
    for (int i = 0; i < ST_N; ++i) c->stats[i] = 0;
  }
  __syncthreads();
  for (uint32_t s = threadIdx.x; s < p.n_slots; s += blockDim.x) {
    const SlotDesc& d = p.desc[s];
    Box ra = load_box(d.boxA, 1), rb = load_box(d.boxB, 1);
    float M = 0.f;
#pragma unroll
    for (int k = 0; k < 3; ++k)
      M = fmaxf(M, fmaxf(fmaxf(fabsf(ra.lo[k]), fabsf(ra.hi[k])), fmaxf(fabsf(rb.lo[k]), fabsf(rb.hi[k]))));
    M = fmaxf(M, 1e-30f);
    float delta = d.kappa_u * M;
    SlotState& st = p.st[s];
    st.delta = delta;
    st.n_ties = 0;
    st.n_admitted = 0;
    st.key_pair = ~0ull;
    float key;
    if (d.mode == 0) {
      float lo, up;
      bounds_min(ra, rb, d.enhanced != 0, lo, up);
      st.best = fbits(up + delta);
      st.best32 = fbits(__builtin_huge_valf());
      st.key_d = ~0ull;
      key = lo;
    } else {
      float up, lo;
      bounds_max(ra, rb, d.enhanced != 0, up, lo);
      st.best = fbits(fmaxf(lo - delta, 0.f));
      st.best32 = 0u;
      st.key_d = 0ull;
      key = up;
    }
    gdist_result_t& r = p.res[s];
    r.status = GDIST_E_DEVICE;
    r.flags = 0;
    uint4 e = make_uint4(1u, 1u, fbits(key), s);
    if (d.LA == 1 && d.LB == 1) {
      uint32_t i = atomicAdd(&c->leaf_len[0], 1u);
      p.leaf[0][i] = e;
    } else {
      uint32_t i = atomicAdd(&c->front_len[0], 1u);
      p.front[0][i] = e;
    }
  }
}

// Expansion of one wave's worth of items of the current front.
__device__ __forceinline__ void expand_wave(const TravParams& p, const uint4* __restrict__ fin,
                                            uint4* __restrict__ fout, uint4* __restrict__ lout, uint32_t o3,
                                            uint64_t it, uint64_t n_items, uint32_t k, unsigned long long* sst,
                                            uint32_t lane, uint64_t lt) {
  Ctl* c = p.ctl;
  bool act = it < n_items;
  const uint32_t kk = 2 * k;
  uint4 ent = make_uint4(1u, 1u, 0u, 0u);
  if (act) ent = fin[it >> kk];
  const uint32_t sub = (uint32_t)(it & ((1ull << kk) - 1ull));
  const uint32_t slot = ent.w;
  const SlotDesc* d = p.desc + slot;
  const uint32_t mode = d->mode;
  const float delta = p.st[slot].delta;
  const float best = bitsf(ld_rlx(&p.st[slot].best));
  const float key = bitsf(ent.z);
  if (act) act = mode == 0 ? !(key - delta > best) : !(key + delta < best);
  const uint32_t remA = d->depthA - (31u - (uint32_t)__clz(ent.x));
  const uint32_t remB = d->depthB - (31u - (uint32_t)__clz(ent.y));
  uint32_t kA = remA < k ? remA : k;
  uint32_t kB = remB < kk - kA ? remB : kk - kA;
  kA = remA < kk - kB ? remA : kk - kB;
  if (act) act = (sub >> (kA + kB)) == 0u;
  add_stat(sst, ST_POPPED, act && sub == 0u, lane);
  add_stat(sst, ST_CHILD, act, lane);
  const uint32_t ca = (ent.x << kA) | (sub & ((1u << kA) - 1u));
  const uint32_t cb = (ent.y << kB) | (sub >> kA);
  bool keep = false;
  float improve = 0.f, nkey = 0.f;
  if (act) {
    Box ba = load_box(d->boxA, ca), bb = load_box(d->boxB, cb);
    const bool enh = d->enhanced != 0;
    if (mode == 0) {
      float lo, up;
      bounds_min(ba, bb, enh, lo, up);
      keep = lo - delta <= best;
      improve = up + delta;
      nkey = lo;
    } else {
      float up, lo;
      bounds_max(ba, bb, enh, up, lo);
      keep = up + delta >= best;
      improve = fmaxf(lo - delta, 0.f);
      nkey = up;
    }
  }
  const bool isleaf = (ca >= d->LA) && (cb >= d->LB);
  const uint4 ne = make_uint4(ca, cb, fbits(nkey), slot);
  append(act && keep && isleaf, ne, lout, &c->leaf_len[o3], p.leaf_cap, &c->overflow, 2u, lane, lt);
  append(act && keep && !isleaf, ne, fout, &c->front_len[o3], p.front_cap, &c->overflow, 1u, lane, lt);
  add_stat(sst, ST_PUSHED, act && keep, lane);
  improve_bound(&p.st[0].best, sizeof(SlotState) / 4, act, slot, mode, improve, lane);
}

// Narrow phase for one wave: 4 lanes per leaf pair, one triangle pair each.
__device__ __forceinline__ void narrow_wave(const TravParams& p, const uint4* __restrict__ lin, uint64_t it,
                                            uint64_t n_items, unsigned long long* sst, uint32_t lane, uint64_t lt) {
  Ctl* c = p.ctl;
  bool act = it < n_items;
  uint4 ent = make_uint4(1u, 1u, 0u, 0u);
  if (act) ent = lin[it >> 2];
  const uint32_t s4 = (uint32_t)(it & 3ull);
  const uint32_t slot = ent.w;
  const SlotDesc* d = p.desc + slot;
  const uint32_t mode = d->mode;
  const float delta = p.st[slot].delta;
  const float best = bitsf(ld_rlx(&p.st[slot].best));
  const float key = bitsf(ent.z);
  if (act) act = mode == 0 ? !(key - delta > best) : !(key + delta < best);
  add_stat(sst, ST_LEAF, act && s4 == 0u, lane);
  const uint32_t LA = d->LA, LB = d->LB, nA = d->nA, nB = d->nB;
  const uint32_t ja = ent.x - LA, jb = ent.y - LB;
  const uint32_t sa = (uint32_t)(((uint64_t)ja * nA) / LA), ea = (uint32_t)(((uint64_t)(ja + 1) * nA) / LA);
  const uint32_t sb = (uint32_t)(((uint64_t)jb * nB) / LB), eb = (uint32_t)(((uint64_t)(jb + 1) * nB) / LB);
  const uint32_t pa = sa + (s4 & 1u), pb = sb + (s4 >> 1);
  if (act) act = pa < ea && pb < eb;
  float dd = 0.f;
  bool cand = false;
  float improve = 0.f;
  if (act) {
    float P[9], Q[9];
    load_tri(d->trisA, pa, P);
    load_tri_xf(d->trisB, pb, d->T, Q);
    V3<float> Pv[3], Qv[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      Pv[v] = mk<float>(P[3 * v], P[3 * v + 1], P[3 * v + 2]);
      Qv[v] = mk<float>(Q[3 * v], Q[3 * v + 1], Q[3 * v + 2]);
    }
    float d2 = mode == 0 ? tri_tri_min_d2<float, false>(Pv, Qv, nullptr, nullptr)
                         : tri_tri_max_d2<float, false>(Pv, Qv, nullptr, nullptr);
    dd = sqrtf(d2);
    if (mode == 0) {
      improve = dd + delta;
      cand = dd - delta <= best;
    } else {
      improve = fmaxf(dd - delta, 0.f);
      cand = dd + delta >= best;
    }
  }
  add_stat(sst, ST_TRI, act, lane);
  Cand ce;
  ce.d32 = dd;
  ce.slot = slot;
  ce.ia = pa;
  ce.ib = pb;
  append(act && cand, ce, p.cand, &c->cand_len, p.cand_cap, &c->overflow, 4u, lane, lt);
  add_stat(sst, ST_CAND, act && cand, lane);
  improve_bound(&p.st[0].best, sizeof(SlotState) / 4, act, slot, mode, improve, lane);
  improve_bound(&p.st[0].best32, sizeof(SlotState) / 4, act, slot, mode, dd, lane);
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

__global__ __launch_bounds__(kTravThreads) void k_traverse(TravParams p) {
  __shared__ unsigned long long sst[ST_N];
  if (threadIdx.x < ST_N) sst[threadIdx.x] = 0ull;
  __syncthreads();
  Ctl* c = p.ctl;
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t lt = (1ull << lane) - 1ull;
  const uint64_t wpb = blockDim.x >> 6;
  const uint64_t gw = (uint64_t)blockIdx.x * wpb + (threadIdx.x >> 6);
  const uint64_t nw = (uint64_t)gridDim.x * wpb;

  for (uint32_t round = 0;; ++round) {
    const uint32_t r3 = round % 3u, o3 = (round + 1u) % 3u;
    if (ld_rlx(&c->abort) || ld_rlx(&c->overflow)) break;
    uint32_t n = ld_rlx(&c->front_len[r3]);
    uint32_t nl = ld_rlx(&c->leaf_len[r3]);
    if (n == 0u && nl == 0u) break;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st_rlx(&c->front_len[(round + 2u) % 3u], 0u);
      st_rlx(&c->leaf_len[(round + 2u) % 3u], 0u);
      sst[ST_ROUNDS] += 1ull;
      if (n > sst[ST_PEAK]) sst[ST_PEAK] = n;
    }
    uint32_t k = p.k_cap;
    while (k > 1u && ((uint64_t)n << (2u * k)) >= (uint64_t)p.expand_budget) --k;
    const uint64_t leaf_items = (uint64_t)nl * 4ull;
    const uint64_t leaf_waves = (leaf_items + 63ull) >> 6;
    const uint64_t exp_items = (uint64_t)n << (2u * k);
    const uint64_t total = leaf_waves + ((exp_items + 63ull) >> 6);
    const uint4* fin = p.front[round & 1u];
    uint4* fout = p.front[(round + 1u) & 1u];
    const uint4* lin = p.leaf[round & 1u];
    uint4* lout = p.leaf[(round + 1u) & 1u];
    for (uint64_t w = gw; w < total; w += nw) {
      if (w < leaf_waves) narrow_wave(p, lin, w * 64ull + lane, leaf_items, sst, lane, lt);
      else expand_wave(p, fin, fout, lout, o3, (w - leaf_waves) * 64ull + lane, exp_items, k, sst, lane, lt);
    }
    grid_sync(c, p.spin_limit);
  }

  __syncthreads();
  if (threadIdx.x < ST_N && sst[threadIdx.x]) {
    if (threadIdx.x == ST_PEAK) atomicMax(&c->stats[ST_PEAK], sst[ST_PEAK]);
    else if (threadIdx.x == ST_ROUNDS) atomicMax(&c->stats[ST_ROUNDS], sst[ST_ROUNDS]);
    else atomicAdd(&c->stats[threadIdx.x], sst[threadIdx.x]);
  }
}


// FP64 re-evaluation, in three grid-wide steps (separate launches).
// A: admit the candidates inside the final window and evaluate them in FP64
//    in the world frame from the caller's FP32 vertices and FP64 poses.
__global__ __launch_bounds__(kTravThreads) void k_reeval_values(TravParams p) {
  Ctl* c = p.ctl;
  if (ld_rlx(&c->abort) || ld_rlx(&c->overflow)) return;
  const uint64_t gt = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t nt = (uint64_t)gridDim.x * blockDim.x;
  uint32_t ncand = ld_rlx(&c->cand_len);
  if (ncand > p.cand_cap) ncand = p.cand_cap;
  for (uint64_t i = gt; i < ncand; i += nt) {
    Cand cd = p.cand[i];
    const SlotDesc& d = p.desc[cd.slot];
    SlotState& st = p.st[cd.slot];
    const float best = bitsf(ld_rlx(&st.best));
    const bool adm = d.mode == 0 ? (cd.d32 - st.delta <= best) : (cd.d32 + st.delta >= best);
    if (!adm) {
      p.cand_d64[i] = -1.0;
      continue;
    }
    V3<double> P[3], Q[3];
    world_tri(d.trisA, cd.ia, d.RA, d.tA, P);
    world_tri(d.trisB, cd.ib, d.RB, d.tB, Q);
    double d2 = d.mode == 0 ? tri_tri_min_d2<double, false>(P, Q, nullptr, nullptr)
                            : tri_tri_max_d2<double, false>(P, Q, nullptr, nullptr);
    double dd = sqrt(d2);
    p.cand_d64[i] = dd;
    unsigned long long b = (unsigned long long)__double_as_longlong(dd);
    if (d.mode == 0) atomicMin(&st.key_d, b);
    else atomicMax(&st.key_d, b);
    atomicAdd(&st.n_admitted, 1u);
  }
}

__device__ __forceinline__ unsigned long long caller_pair(const SlotDesc& d, const Cand& cd) {
  uint32_t ta = d.origA[cd.ia], tb = d.origB[cd.ib];
  return d.swapped ? (((unsigned long long)tb << 32) | ta) : (((unsigned long long)ta << 32) | tb);
}

// B: the tie set and its lexicographically smallest caller pair.
__global__ __launch_bounds__(kTravThreads) void k_reeval_ties(TravParams p) {
  Ctl* c = p.ctl;
  if (ld_rlx(&c->abort) || ld_rlx(&c->overflow)) return;
  const uint64_t gt = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t nt = (uint64_t)gridDim.x * blockDim.x;
  uint32_t ncand = ld_rlx(&c->cand_len);
  if (ncand > p.cand_cap) ncand = p.cand_cap;
  for (uint64_t i = gt; i < ncand; i += nt) {
    double dd = p.cand_d64[i];
    if (dd < 0.0) continue;
    Cand cd = p.cand[i];
    const SlotDesc& d = p.desc[cd.slot];
    SlotState& st = p.st[cd.slot];
    double D = __longlong_as_double((long long)st.key_d);
    if (fabs(dd - D) <= d.tau) {
      atomicMin(&st.key_pair, caller_pair(d, cd));
      atomicAdd(&st.n_ties, 1u);
    }
  }
}

// C: closest (farthest) points of the reported pair, and the per-query summary.
__global__ __launch_bounds__(kTravThreads) void k_reeval_report(TravParams p) {
  Ctl* c = p.ctl;
  if (ld_rlx(&c->abort) || ld_rlx(&c->overflow)) return;
  const uint64_t gt = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t nt = (uint64_t)gridDim.x * blockDim.x;
  uint32_t ncand = ld_rlx(&c->cand_len);
  if (ncand > p.cand_cap) ncand = p.cand_cap;
  for (uint64_t i = gt; i < ncand; i += nt) {
    double dd = p.cand_d64[i];
    if (dd < 0.0) continue;
    Cand cd = p.cand[i];
    const SlotDesc& d = p.desc[cd.slot];
    const SlotState& st = p.st[cd.slot];
    unsigned long long key = caller_pair(d, cd);
    if (key != st.key_pair) continue;
    V3<double> P[3], Q[3], x, y;
    world_tri(d.trisA, cd.ia, d.RA, d.tA, P);
    world_tri(d.trisB, cd.ib, d.RB, d.tB, Q);
    if (d.mode == 0) tri_tri_min_d2<double, true>(P, Q, &x, &y);
    else tri_tri_max_d2<double, true>(P, Q, &x, &y);
    gdist_result_t& r = p.res[cd.slot];
    V3<double> qa = d.swapped ? y : x, qb = d.swapped ? x : y;
    r.point_a[0] = qa.x; r.point_a[1] = qa.y; r.point_a[2] = qa.z;
    r.point_b[0] = qb.x; r.point_b[1] = qb.y; r.point_b[2] = qb.z;
    r.tri_a = (uint32_t)(key >> 32);
    r.tri_b = (uint32_t)(key & 0xffffffffull);
  }
  for (uint64_t s = gt; s < p.n_slots; s += nt) {
    const SlotDesc& d = p.desc[s];
    const SlotState& st = p.st[s];
    gdist_result_t& r = p.res[s];
    r.n_candidates = st.n_admitted;
    r.n_ties = st.n_ties;
    r.distance_fp32 = (double)bitsf(st.best32);
    r.err_bound = d.err_bound;
    if (st.n_admitted == 0u) {
      r.status = GDIST_E_DEVICE;
      r.distance = __longlong_as_double(0x7ff8000000000000ll);
      continue;
    }
    double D = __longlong_as_double((long long)st.key_d);
    r.distance = D;
    r.status = GDIST_OK;
    r.flags = (st.n_ties > 1u ? GDIST_F_TIED : 0u) | ((d.mode == 0 && D == 0.0) ? GDIST_F_ZERO : 0u);
  }
}

hipError_t launch_init(const TravParams& p, hipStream_t s) {
  k_init<<<1, 256, 0, s>>>(p);
  return hipGetLastError();
}

hipError_t traverse_grid(int device, uint32_t blocks_per_cu, uint32_t* blocks, uint32_t* threads) {
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_traverse, kTravThreads, 0);
  if (e != hipSuccess) return e;
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) return e;
  uint32_t b = (uint32_t)per_cu;
  if (blocks_per_cu > 0 && blocks_per_cu < b) b = blocks_per_cu;
  if (b == 0) b = 1;
  *blocks = b * (uint32_t)prop.multiProcessorCount;
  *threads = kTravThreads;
  return hipSuccess;
}

hipError_t launch_traverse(const TravParams& p, uint32_t blocks, uint32_t threads, hipStream_t s) {
  TravParams pp = p;
  void* args[] = {&pp};
  return hipLaunchCooperativeKernel((const void*)k_traverse, dim3(blocks), dim3(threads), args, 0, s);
}

hipError_t launch_reeval(const TravParams& p, uint32_t blocks, hipStream_t s) {
  k_reeval_values<<<blocks, kTravThreads, 0, s>>>(p);
  k_reeval_ties<<<blocks, kTravThreads, 0, s>>>(p);
  k_reeval_report<<<blocks, kTravThreads, 0, s>>>(p);
  return hipGetLastError();
}

}  // namespace gd
