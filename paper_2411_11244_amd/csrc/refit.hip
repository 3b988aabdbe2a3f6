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
#include "internal.hpp"

namespace gd {

constexpr int kRefitThreads = 256;

__global__ __launch_bounds__(kRefitThreads) void k_refit_leaves(const float* __restrict__ tris, uint32_t n,
                                                                 uint32_t L, Xf32 T, float* __restrict__ boxes,
                                                                 uint32_t S) {
  __shared__ Box lb[kRefitThreads];
  const uint32_t j = threadIdx.x;
  Box b;
  if (j < S) {
    uint32_t leaf = blockIdx.x * S + j;
    const uint32_t D = 31u - (uint32_t)__clz(L);   // L = 2^D
    uint32_t start = (uint32_t)(((uint64_t)leaf * n) >> D);
    uint32_t end = (uint32_t)(((uint64_t)(leaf + 1) * n) >> D);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      b.lo[k] = __builtin_huge_valf();
      b.hi[k] = -__builtin_huge_valf();
    }
    for (uint32_t p = start; p < end; ++p) {
      float t[9];
      load_tri_xf(tris, p, T, t);
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          b.lo[k] = fminf(b.lo[k], t[3 * c + k]);
          b.hi[k] = fmaxf(b.hi[k], t[3 * c + k]);
        }
    }
    store_box(boxes, L + leaf, b);
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

hipError_t launch_refit(const float* tris, uint32_t n, uint32_t L, const Xf32& T, float* boxes, hipStream_t s) {
  uint32_t S = L < (uint32_t)kRefitThreads ? L : (uint32_t)kRefitThreads;
  k_refit_leaves<<<L / S, kRefitThreads, 0, s>>>(tris, n, L, T, boxes, S);
  uint32_t count = L / S;  // nodes of the level holding the subtree roots
  while (count > 1) {
    uint32_t S2 = count < (uint32_t)kRefitThreads ? count : (uint32_t)kRefitThreads;
    k_reduce_levels<<<count / S2, kRefitThreads, 0, s>>>(boxes, count, S2);
    count /= S2;
  }
  return hipGetLastError();
}

}  // namespace gd
