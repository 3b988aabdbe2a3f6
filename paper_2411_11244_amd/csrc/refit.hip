// Refit of an f12 tree under a rigid transform (gDist Sec. 7 refits the BVH
// for moving models; Sec. 4 requires tight boxes, so boxes are recomputed from
// the transformed vertices, never enlarged).
//
// Leaf j of a tree with N triangles and L = 2^D leaves holds the leaf-order
// triangles [floor(jN/L), floor((j+1)N/L)) (1 or 2 of them).  One workgroup
// owns a subtree of S leaves: it computes the S leaf boxes from the
// transformed triangles and reduces them in LDS through log2(S) levels,
// writing every node of the subtree once.  The remaining upper levels are
// reduced by the same LDS scheme over the subtree roots.  Per triangle the
// kernel reads 36 B; per node it writes 24 B.
#include <vector>

#include "internal.hpp"

namespace gd {

constexpr int kRefitThreads = 512;
constexpr uint32_t kStageFloats = 18u * kRefitThreads;   // at most two triangles per leaf

// Box of leaf blk * S + threadIdx.x (threads >= S: an empty box) of a tree
// with n triangles and L = 2^D leaves under transform T.  The workgroup's S
// leaves hold one contiguous run of at most 2S triangles; it is read with
// 16-byte loads across the whole workgroup (each wave reads 1 KB of
// consecutive bytes per instruction) into LDS, and every thread then
// transforms its leaf's one or two triangles from there, with the same fused
// multiply-add order as the narrow phase.
__device__ __forceinline__ Box staged_leaf_box(const float* __restrict__ tris, uint32_t n, uint32_t L, const Xf32& T,
                                               uint32_t blk, uint32_t S, float* __restrict__ stage) {
  const uint32_t D = 31u - (uint32_t)__clz(L);
  const uint32_t t0 = (uint32_t)(((uint64_t)blk * S * n) >> D);
  const uint32_t t1 = (uint32_t)(((uint64_t)(blk * S + S) * n) >> D);
  const uint32_t nf = 9u * (t1 - t0);
  const __attribute__((address_space(1))) float* src = gptr(tris) + 9ull * t0;
  const uint32_t n4 = nf >> 2;
  for (uint32_t i = threadIdx.x; i < n4; i += blockDim.x)
    *reinterpret_cast<f4v*>(stage + 4u * i) = gload<f4u>(src + 4u * i);
  for (uint32_t i = 4u * n4 + threadIdx.x; i < nf; i += blockDim.x) stage[i] = src[i];
  __syncthreads();
  Box b;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    b.lo[k] = __builtin_huge_valf();
    b.hi[k] = -__builtin_huge_valf();
  }
  const uint32_t j = threadIdx.x;
  if (j < S) {
    const uint32_t leaf = blk * S + j;
    const uint32_t start = (uint32_t)(((uint64_t)leaf * n) >> D);
    const uint32_t end = (uint32_t)(((uint64_t)(leaf + 1) * n) >> D);
    for (uint32_t p = start; p < end; ++p) {
      const float* q = stage + 9u * (p - t0);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        float w[3];
        xform(T, q[3 * c], q[3 * c + 1], q[3 * c + 2], w);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          b.lo[k] = fminf(b.lo[k], w[k]);
          b.hi[k] = fmaxf(b.hi[k], w[k]);
        }
      }
    }
  }
  return b;
}

__global__ __launch_bounds__(kRefitThreads) void k_refit_leaves(const float* __restrict__ tris, uint32_t n,
                                                                 uint32_t L, Xf32 T, float* __restrict__ boxes,
                                                                 uint32_t S) {
  __shared__ Box lb[kRefitThreads];
  __shared__ __align__(16) float stage[kStageFloats];
  const uint32_t j = threadIdx.x;
  const Box b = staged_leaf_box(tris, n, L, T, blockIdx.x, S, stage);
  if (j < S) {
    store_box(boxes, L + blockIdx.x * S + j, b);
    lb[j] = b;
  }
  uint32_t base = L + blockIdx.x * S;
  for (uint32_t cnt = S; cnt > 1; cnt >>= 1) {
    __syncthreads();
    Box nb;
    bool act = j < cnt / 2;
    if (act) nb = box_union(lb[2 * j], lb[2 * j + 1]);
    __syncthreads();
    base >>= 1;
    if (act) {
      lb[j] = nb;
      store_box(boxes, base + j, nb);
    }
  }
}

// Reduce `count` nodes starting at node id `first` (a whole level) up through
// log2(S) levels, S nodes per workgroup.
__global__ __launch_bounds__(kRefitThreads) void k_reduce_levels(float* __restrict__ boxes, uint32_t first,
                                                                  uint32_t S) {
  __shared__ Box lb[kRefitThreads];
  const uint32_t j = threadIdx.x;
  if (j < S) lb[j] = load_box(boxes, first + blockIdx.x * S + j);
  uint32_t base = first + blockIdx.x * S;
  for (uint32_t cnt = S; cnt > 1; cnt >>= 1) {
    __syncthreads();
    Box nb;
    bool act = j < cnt / 2;
    if (act) nb = box_union(lb[2 * j], lb[2 * j + 1]);
    __syncthreads();
    base >>= 1;
    if (act) {
      lb[j] = nb;
      store_box(boxes, base + j, nb);
    }
  }
}

// ------------------------------------------------------------------ batched
// Many trees refitted by one launch per pass.  Workgroup b serves the job j
// with first_block[j] <= b < first_block[j+1] (binary search in thread 0).
template <typename J>
__device__ __forceinline__ const J* find_job(const J* jobs, uint32_t njobs) {
  __shared__ uint32_t s_job;
  if (threadIdx.x == 0) {
    uint32_t lo = 0, hi = njobs;
    while (hi - lo > 1u) {
      uint32_t mid = (lo + hi) >> 1;
      if (jobs[mid].first_block <= blockIdx.x) lo = mid;
      else hi = mid;
    }
    s_job = lo;
  }
  __syncthreads();
  return jobs + s_job;
}

__global__ __launch_bounds__(kRefitThreads) void k_refit_leaves_batch(const RefitJob* __restrict__ jobs,
                                                                       uint32_t njobs) {
  __shared__ Box lb[kRefitThreads];
  __shared__ __align__(16) float stage[kStageFloats];
  const RefitJob* jp = find_job(jobs, njobs);
  const RefitJob J = *jp;
  const uint32_t j = threadIdx.x;
  const uint32_t blk = blockIdx.x - J.first_block;
  const uint32_t S = J.S, L = J.L;
  const Box b = staged_leaf_box(J.tris, J.n, L, J.T, blk, S, stage);
  if (j < S) {
    store_box(J.boxes, L + blk * S + j, b);
    lb[j] = b;
  }
  uint32_t base = L + blk * S;
  for (uint32_t cnt = S; cnt > 1; cnt >>= 1) {
    __syncthreads();
    Box nb;
    bool act = j < cnt / 2;
    if (act) nb = box_union(lb[2 * j], lb[2 * j + 1]);
    __syncthreads();
    base >>= 1;
    if (act) {
      lb[j] = nb;
      store_box(J.boxes, base + j, nb);
    }
  }
}

__global__ __launch_bounds__(kRefitThreads) void k_reduce_batch(const ReduceJob* __restrict__ jobs, uint32_t njobs) {
  __shared__ Box lb[kRefitThreads];
  const ReduceJob J = *find_job(jobs, njobs);
  const uint32_t j = threadIdx.x;
  const uint32_t blk = blockIdx.x - J.first_block;
  if (j < J.S) lb[j] = load_box(J.boxes, J.first + blk * J.S + j);
  uint32_t base = J.first + blk * J.S;
  for (uint32_t cnt = J.S; cnt > 1; cnt >>= 1) {
    __syncthreads();
    Box nb;
    bool act = j < cnt / 2;
    if (act) nb = box_union(lb[2 * j], lb[2 * j + 1]);
    __syncthreads();
    base >>= 1;
    if (act) {
      lb[j] = nb;
      store_box(J.boxes, base + j, nb);
    }
  }
}

// Plan the passes of a batched refit.  Writes the job tables into `staging`
// (host, pinned), returns their byte size; the tables are then copied to
// `dev` and the passes launched by launch_refit_batch.
size_t plan_refit_batch(const RefitJob* in, uint32_t njobs, void* staging, size_t cap, RefitPlan* plan) {
  char* out = (char*)staging;
  size_t used = 0;
  auto need = [&](size_t b) { return used + b <= cap; };
  plan->npasses = 0;
  // leaves
  if (!need(sizeof(RefitJob) * njobs)) return 0;
  RefitJob* lj = (RefitJob*)(out + used);
  uint32_t blocks = 0;
  std::vector<uint32_t> count(njobs);
  for (uint32_t i = 0; i < njobs; ++i) {
    lj[i] = in[i];
    lj[i].S = in[i].L < (uint32_t)kRefitThreads ? in[i].L : (uint32_t)kRefitThreads;
    lj[i].first_block = blocks;
    blocks += in[i].L / lj[i].S;
    count[i] = in[i].L / lj[i].S;
  }
  plan->leaf_off = used;
  plan->leaf_blocks = blocks;
  plan->njobs = njobs;
  used += sizeof(RefitJob) * njobs;
  // upper levels: each pass reduces up to 8 more levels of every tree that
  // still has more than one node at its current level
  for (;;) {
    uint32_t act = 0;
    for (uint32_t i = 0; i < njobs; ++i) act += count[i] > 1 ? 1u : 0u;
    if (act == 0) break;
    if (plan->npasses >= kMaxRefitPasses || !need(sizeof(ReduceJob) * act)) return 0;
    ReduceJob* rj = (ReduceJob*)(out + used);
    uint32_t k = 0, rb = 0;
    for (uint32_t i = 0; i < njobs; ++i) {
      if (count[i] <= 1) continue;
      uint32_t S2 = count[i] < (uint32_t)kRefitThreads ? count[i] : (uint32_t)kRefitThreads;
      rj[k].boxes = in[i].boxes;
      rj[k].first = count[i];
      rj[k].S = S2;
      rj[k].first_block = rb;
      rb += count[i] / S2;
      count[i] /= S2;
      ++k;
    }
    plan->pass_off[plan->npasses] = used;
    plan->pass_jobs[plan->npasses] = k;
    plan->pass_blocks[plan->npasses] = rb;
    plan->npasses++;
    used += sizeof(ReduceJob) * k;
  }
  return used;
}

hipError_t launch_refit_batch(const RefitPlan& plan, const void* dev, hipStream_t s) {
  const char* d = (const char*)dev;
  k_refit_leaves_batch<<<plan.leaf_blocks, kRefitThreads, 0, s>>>((const RefitJob*)(d + plan.leaf_off),
                                                                   plan.njobs);
  for (uint32_t p = 0; p < plan.npasses; ++p)
    k_reduce_batch<<<plan.pass_blocks[p], kRefitThreads, 0, s>>>((const ReduceJob*)(d + plan.pass_off[p]),
                                                                 plan.pass_jobs[p]);
  return hipGetLastError();
}

hipError_t launch_reduce_upper(float* boxes, uint32_t count, hipStream_t s) {
  while (count > 1) {
    uint32_t S2 = count < (uint32_t)kRefitThreads ? count : (uint32_t)kRefitThreads;
    k_reduce_levels<<<count / S2, kRefitThreads, 0, s>>>(boxes, count, S2);
    count /= S2;
  }
  return hipGetLastError();
}

hipError_t launch_refit(const float* tris, uint32_t n, uint32_t L, const Xf32& T, float* boxes, hipStream_t s) {
  uint32_t S = L < (uint32_t)kRefitThreads ? L : (uint32_t)kRefitThreads;
  k_refit_leaves<<<L / S, kRefitThreads, 0, s>>>(tris, n, L, T, boxes, S);
  // the level holding the subtree roots has L / S nodes
  return launch_reduce_upper(boxes, L / S, s);
}

}  // namespace gd
