// GPU construction of the f12 tree (gDist Sec. 6.3): triangles are ordered by
// the Morton code of their centroid, then split evenly over 2^floor(log2 N)
// leaves (1 or 2 consecutive triangles each) of a perfect binary tree stored
// implicitly in heap order.  The node boxes are produced by the refit kernels
// with the identity transform.
//
// Kernels here: a vertex pass (finiteness, vertex box, largest vertex norm),
// a key pass (index check and the 63-bit Morton code of each centroid, 21
// bits per axis, in the vertex box), a stable LSD radix sort of (u64 key, u32
// value) pairs with 8-bit digits, and the scatter of triangles into leaf
// order.
#include "internal.hpp"

namespace gd {

// Order-preserving map of a float onto a signed int (for atomic min/max).
__device__ __forceinline__ int ordered(float f) {
  int i = __float_as_int(f);
  return i >= 0 ? i : (i ^ 0x7fffffff);
}
__host__ __device__ inline float unordered(int i) {
  int j = i >= 0 ? i : (i ^ 0x7fffffff);
  float f;
  __builtin_memcpy(&f, &j, 4);
  return f;
}

// Wave-wide reductions (every lane active).
__device__ __forceinline__ float wave_max_reduce(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ float wave_min_reduce(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
  return v;
}

// Vertex pass.  vb: 7 ints (ordered floats): vertex box min xyz, max xyz,
// and an upper bound of the largest vertex norm |x|.  flags: bit 1 = a
// non-finite vertex.  One reduction per workgroup, one atomic per value.
constexpr int kVpThreads = 256;
__global__ __launch_bounds__(kVpThreads) void k_vertex_pass(const float* __restrict__ v, uint32_t nv,
                                                            int* __restrict__ vb, uint32_t* __restrict__ flags) {
  float lo[3] = {__builtin_huge_valf(), __builtin_huge_valf(), __builtin_huge_valf()};
  float hi[3] = {-__builtin_huge_valf(), -__builtin_huge_valf(), -__builtin_huge_valf()};
  float rmax = 0.f;
  uint32_t bad = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += stride) {
    const float x = v[3 * i], y = v[3 * i + 1], z = v[3 * i + 2];
    if (!(isfinite(x) && isfinite(y) && isfinite(z))) {
      bad = 2u;
      continue;
    }
    lo[0] = fminf(lo[0], x); lo[1] = fminf(lo[1], y); lo[2] = fminf(lo[2], z);
    hi[0] = fmaxf(hi[0], x); hi[1] = fmaxf(hi[1], y); hi[2] = fmaxf(hi[2], z);
    rmax = fmaxf(rmax, sqrtf(x * x + y * y + z * z));
  }
  // a few roundings of relative size 2^-24 each: widen by 2^-20
  float r[7];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    r[k] = wave_min_reduce(lo[k]);
    r[3 + k] = wave_max_reduce(hi[k]);
  }
  r[6] = wave_max_reduce(rmax) * (1.0f + 0x1p-20f);
  __shared__ float sr[kVpThreads / 64][7];
  __shared__ uint32_t s_bad;
  if (threadIdx.x == 0) s_bad = 0u;
  __syncthreads();
  if (bad) atomicOr(&s_bad, bad);
  const uint32_t w = threadIdx.x >> 6;
  if ((threadIdx.x & 63u) == 0u)
#pragma unroll
    for (int k = 0; k < 7; ++k) sr[w][k] = r[k];
  __syncthreads();
  if (threadIdx.x < 7) {
    const int k = threadIdx.x;
    float a = sr[0][k];
    for (int q = 1; q < kVpThreads / 64; ++q) a = k < 3 ? fminf(a, sr[q][k]) : fmaxf(a, sr[q][k]);
    if (k < 3) atomicMin(&vb[k], ordered(a));
    else atomicMax(&vb[k], ordered(a));
  }
  if (threadIdx.x == 0 && s_bad) atomicOr(flags, s_bad);
}

__global__ void k_init_vb(int* vb, uint32_t* flags) {
  if (threadIdx.x < 3) {
    vb[threadIdx.x] = ordered(__builtin_huge_valf());
    vb[3 + threadIdx.x] = ordered(-__builtin_huge_valf());
  }
  if (threadIdx.x == 3) vb[6] = 0;
  if (threadIdx.x == 0) *flags = 0;
}

// Spread the low 21 bits of x so that bit i lands at bit 3i.
__device__ __forceinline__ uint64_t spread3(uint64_t x) {
  x &= 0x1fffffull;
  x = (x | (x << 32)) & 0x001f00000000ffffull;
  x = (x | (x << 16)) & 0x001f0000ff0000ffull;
  x = (x | (x << 8)) & 0x100f00f00f00f00full;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}

// Key pass, one thread per triangle: the index check (flags bit 0) and the
// 63-bit Morton code of the FP32 centroid, normalised to the vertex box.
__global__ void k_keys(const float* __restrict__ v, uint32_t nv, const uint32_t* __restrict__ f, uint32_t nt,
                       const int* __restrict__ vb, uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                       uint32_t* __restrict__ flags) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  const uint32_t i0 = f[3 * t], i1 = f[3 * t + 1], i2 = f[3 * t + 2];
  uint64_t code = 0;
  if (i0 >= nv || i1 >= nv || i2 >= nv) {
    atomicOr(flags, 1u);
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float lo = unordered(vb[k]), hi = unordered(vb[3 + k]);
      const float c = (v[3ull * i0 + k] + v[3ull * i1 + k] + v[3ull * i2 + k]) * (1.0f / 3.0f);
      const float ext = hi - lo;
      const float u = ext > 0.f ? (c - lo) / ext : 0.f;
      const float sc = u * 2097152.0f;  // 2^21 cells per axis
      const uint32_t q = sc <= 0.f ? 0u : (sc >= 2097151.0f ? 2097151u : (uint32_t)sc);
      code |= spread3(q) << (2 - k);   // x on the highest of each bit triple
    }
  }
  keys[t] = code;
  vals[t] = (uint32_t)t;
}

// ---------------------------------------------------------------- radix sort
constexpr int kRsThreads = 256;
constexpr int kRsRowsPerWave = 16;
constexpr int kRsTile = kRsThreads * kRsRowsPerWave;  // 4096 keys per block

// hist[d * nblocks + b] = number of keys of block b with digit d
__global__ __launch_bounds__(kRsThreads) void k_rs_hist(const uint64_t* __restrict__ keys, uint32_t n,
                                                         uint32_t shift, uint32_t* __restrict__ hist,
                                                         uint32_t nblocks) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  uint64_t base = (uint64_t)blockIdx.x * kRsTile;
  for (int r = 0; r < kRsRowsPerWave; ++r) {
    uint64_t i = base + (uint64_t)r * kRsThreads + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(uint64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of `len` counts in three launches: tile sums, a scan of the
// tile sums, and the in-place rescan of each tile with its offset.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr uint64_t kScanTile = (uint64_t)kScanThreads * kScanItems;  // 4096 counts per workgroup

// Exclusive scan of one value per thread across the workgroup; returns the
// workgroup total.
__device__ __forceinline__ uint32_t block_exclusive(uint32_t v, uint32_t* s, uint32_t* excl) {
  const uint32_t t = threadIdx.x;
  s[t] = v;
  __syncthreads();
  for (uint32_t off = 1; off < kScanThreads; off <<= 1) {
    uint32_t x = t >= off ? s[t - off] : 0u;
    __syncthreads();
    s[t] += x;
    __syncthreads();
  }
  *excl = s[t] - v;
  uint32_t total = s[kScanThreads - 1];
  __syncthreads();
  return total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(const uint32_t* __restrict__ a, uint64_t len,
                                                             uint32_t* __restrict__ tile_sum) {
  __shared__ uint32_t s[kScanThreads];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
  uint32_t v = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < len) v += a[base + i];
  uint32_t excl;
  uint32_t total = block_exclusive(v, s, &excl);
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

// One workgroup scans the tile sums in place (exclusive).
__global__ __launch_bounds__(kScanThreads) void k_scan_sums(uint32_t* __restrict__ tile_sum, uint32_t n) {
  __shared__ uint32_t s[kScanThreads];
  uint32_t carry = 0;
  for (uint32_t b = 0; b < n; b += kScanThreads) {
    const uint32_t i = b + threadIdx.x;
    uint32_t v = i < n ? tile_sum[i] : 0u, excl;
    uint32_t total = block_exclusive(v, s, &excl);
    if (i < n) tile_sum[i] = carry + excl;
    carry += total;
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(uint32_t* __restrict__ a, uint64_t len,
                                                             const uint32_t* __restrict__ tile_sum) {
  __shared__ uint32_t s[kScanThreads];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems], sum = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = base + i < len ? a[base + i] : 0u;
    sum += v[i];
  }
  uint32_t excl;
  block_exclusive(sum, s, &excl);
  uint32_t run = tile_sum[blockIdx.x] + excl;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < len) a[base + i] = run;
    run += v[i];
  }
}

// Stable scatter.  Wave w of the block ranks rows w*16 .. w*16+15 of the
// block's tile (a row = 64 consecutive keys) in order: lanes holding the same
// digit are found with eight ballots, their order inside the row comes from
// mbcnt, and a per-wave running count per digit carries the order across
// rows.  A per-digit prefix over the four waves and an exclusive scan over the
// 256 digits give each key its place in the tile sorted by digit; the tile is
// reordered in LDS, and thread t then writes tile positions t, t + 256, ...
// to the digit's global offset for this block plus the position inside the
// digit's run, so consecutive threads store consecutive addresses of one run.
__global__ __launch_bounds__(kRsThreads) void k_rs_scatter(const uint64_t* __restrict__ kin,
                                                            const uint32_t* __restrict__ vin,
                                                            uint64_t* __restrict__ kout,
                                                            uint32_t* __restrict__ vout, uint32_t n,
                                                            uint32_t shift, const uint32_t* __restrict__ offs,
                                                            uint32_t nblocks) {
  __shared__ uint32_t wc[kRsThreads / kWave][257];
  __shared__ uint32_t lstart[256];
  __shared__ uint32_t scan_s[kScanThreads];
  __shared__ uint64_t tk[kRsTile];
  __shared__ uint32_t tv[kRsTile];
  const uint32_t w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  for (uint32_t i = threadIdx.x; i < (kRsThreads / kWave) * 257; i += kRsThreads) (&wc[0][0])[i] = 0;
  __syncthreads();
  uint64_t key[kRsRowsPerWave];
  uint32_t val[kRsRowsPerWave], dig[kRsRowsPerWave], rk[kRsRowsPerWave];
  const uint64_t base = (uint64_t)blockIdx.x * kRsTile + (uint64_t)w * kRsRowsPerWave * kWave;
  const uint64_t lt = (1ull << lane) - 1ull;
#pragma unroll
  for (int r = 0; r < kRsRowsPerWave; ++r) {
    uint64_t i = base + (uint64_t)r * kWave + lane;
    bool ok = i < n;
    key[r] = ok ? kin[i] : 0ull;
    val[r] = ok ? vin[i] : 0u;
    uint32_t d = ok ? (uint32_t)((key[r] >> shift) & 255u) : 256u;
    dig[r] = d;
    uint64_t same = __ballot(ok);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      uint64_t m = __ballot((d >> bit) & 1u);
      same &= ((d >> bit) & 1u) ? m : ~m;
    }
    uint32_t prev = ok ? wc[w][d] : 0u;
    rk[r] = prev + (uint32_t)__popcll(same & lt);
    // lowest lane of each digit group advances that digit's running count
    if (ok && (same & lt) == 0ull) wc[w][d] = prev + (uint32_t)__popcll(same);
  }
  __syncthreads();
  {
    // per digit: the four waves' offsets inside the digit's run, and the
    // run's start in the digit-sorted tile
    const uint32_t d = threadIdx.x;  // 256 threads, one per digit
    uint32_t run = 0;
#pragma unroll
    for (int q = 0; q < kRsThreads / kWave; ++q) {
      uint32_t c = wc[q][d];
      wc[q][d] = run;
      run += c;
    }
    uint32_t excl;
    block_exclusive(run, scan_s, &excl);
    lstart[d] = excl;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRsRowsPerWave; ++r) {
    if (dig[r] < 256u) {
      const uint32_t lp = lstart[dig[r]] + wc[w][dig[r]] + rk[r];
      tk[lp] = key[r];
      tv[lp] = val[r];
    }
  }
  __syncthreads();
  const uint64_t tile0 = (uint64_t)blockIdx.x * kRsTile;
  const uint32_t valid = n - tile0 < (uint64_t)kRsTile ? (uint32_t)(n - tile0) : (uint32_t)kRsTile;
  for (uint32_t i = threadIdx.x; i < valid; i += kRsThreads) {
    const uint64_t k = tk[i];
    const uint32_t d = (uint32_t)((k >> shift) & 255u);
    const uint32_t pos = offs[(uint64_t)d * nblocks + blockIdx.x] + (i - lstart[d]);
    kout[pos] = k;
    vout[pos] = tv[i];
  }
}

// Triangles in sorted (= leaf) order, plus the caller index of each.
// The 256 triangles of a workgroup are gathered into LDS, then written out
// as one contiguous block (9,216 bytes at a 16-byte aligned offset) with
// 16-byte stores.
constexpr int kEmitThreads = 256;
__global__ __launch_bounds__(kEmitThreads) void k_emit(const float* __restrict__ v, const uint32_t* __restrict__ f,
                                                       uint32_t nt, const uint32_t* __restrict__ sorted,
                                                       float* __restrict__ tris, uint32_t* __restrict__ orig,
                                                       uint32_t* __restrict__ fl) {
  __shared__ __align__(16) float st[9 * kEmitThreads];
  const uint64_t s0 = (uint64_t)blockIdx.x * kEmitThreads;
  const uint64_t s = s0 + threadIdx.x;
  if (s < nt) {
    const uint32_t o = sorted[s];
    orig[s] = o;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const uint32_t vi = f[3ull * o + c];
      if (fl) fl[3ull * s + c] = vi;
#pragma unroll
      for (int k = 0; k < 3; ++k) st[9 * threadIdx.x + 3 * c + k] = v[3ull * vi + k];
    }
  }
  __syncthreads();
  const uint32_t cnt = nt - s0 < (uint64_t)kEmitThreads ? (uint32_t)(nt - s0) : (uint32_t)kEmitThreads;
  const uint32_t nf = 9u * cnt, n4 = nf >> 2;
  float* out = tris + 9ull * s0;     // 36 * 256 * blockIdx.x bytes: 16-byte aligned
  for (uint32_t i = threadIdx.x; i < n4; i += kEmitThreads)
    *reinterpret_cast<f4v*>(out + 4u * i) = *reinterpret_cast<const f4v*>(st + 4u * i);
  for (uint32_t i = 4u * n4 + threadIdx.x; i < nf; i += kEmitThreads) out[i] = st[i];
}

// Deformable meshes: the triangles, in the leaf order of the original build,
// gathered again from new vertex positions (fl holds each triangle's vertex
// indices in that order, validated at build time).
__global__ void k_gather_tris(const float* __restrict__ v, const uint32_t* __restrict__ fl, uint32_t nt,
                              float* __restrict__ tris) {
  uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nt) return;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    uint32_t vi = fl[3ull * s + c];
#pragma unroll
    for (int k = 0; k < 3; ++k) tris[9 * s + 3 * c + k] = v[3ull * vi + k];
  }
}

// ---------------------------------------------------------------- launchers
hipError_t launch_vertex_pass(const float* v, uint32_t nv, int* vb, uint32_t* flags, hipStream_t s) {
  k_init_vb<<<1, 64, 0, s>>>(vb, flags);
  uint32_t blocks = (uint32_t)(((uint64_t)nv + kVpThreads - 1) / kVpThreads);
  if (blocks > 2048) blocks = 2048;
  if (blocks == 0) blocks = 1;
  k_vertex_pass<<<blocks, kVpThreads, 0, s>>>(v, nv, vb, flags);
  return hipGetLastError();
}

hipError_t launch_keys(const float* v, uint32_t nv, const uint32_t* f, uint32_t nt, const int* vb, uint64_t* keys,
                       uint32_t* vals, uint32_t* flags, hipStream_t s) {
  k_keys<<<(nt + 255) / 256, 256, 0, s>>>(v, nv, f, nt, vb, keys, vals, flags);
  return hipGetLastError();
}

// histogram words plus the scan's tile sums
size_t radix_hist_words(uint32_t n) {
  uint64_t h = (uint64_t)256 * ((n + kRsTile - 1) / kRsTile);
  return (size_t)(h + (h + kScanTile - 1) / kScanTile);
}

hipError_t launch_radix_sort(uint64_t* keys, uint32_t* vals, uint64_t* keys_tmp, uint32_t* vals_tmp,
                             uint32_t n, uint32_t* hist, hipStream_t s, int* result_in_tmp) {
  uint32_t nblocks = (n + kRsTile - 1) / kRsTile;
  const uint64_t hlen = (uint64_t)256 * nblocks;
  const uint32_t tiles = (uint32_t)((hlen + kScanTile - 1) / kScanTile);
  uint32_t* tile_sum = hist + hlen;
  uint64_t *ki = keys, *ko = keys_tmp;
  uint32_t *vi = vals, *vo = vals_tmp;
  for (uint32_t shift = 0; shift < 64; shift += 8) {
    k_rs_hist<<<nblocks, kRsThreads, 0, s>>>(ki, n, shift, hist, nblocks);
    k_scan_tiles<<<tiles, kScanThreads, 0, s>>>(hist, hlen, tile_sum);
    k_scan_sums<<<1, kScanThreads, 0, s>>>(tile_sum, tiles);
    k_scan_apply<<<tiles, kScanThreads, 0, s>>>(hist, hlen, tile_sum);
    k_rs_scatter<<<nblocks, kRsThreads, 0, s>>>(ki, vi, ko, vo, n, shift, hist, nblocks);
    uint64_t* tk = ki; ki = ko; ko = tk;
    uint32_t* tv = vi; vi = vo; vo = tv;
  }
  *result_in_tmp = (ki == keys_tmp);
  return hipGetLastError();
}

hipError_t launch_emit(const float* v, const uint32_t* f, uint32_t nt, const uint32_t* sorted, float* tris,
                       uint32_t* orig, uint32_t* fl, hipStream_t s) {
  k_emit<<<(nt + kEmitThreads - 1) / kEmitThreads, kEmitThreads, 0, s>>>(v, f, nt, sorted, tris, orig, fl);
  return hipGetLastError();
}

hipError_t launch_gather_tris(const float* v, const uint32_t* fl, uint32_t nt, float* tris, hipStream_t s) {
  k_gather_tris<<<(nt + 255) / 256, 256, 0, s>>>(v, fl, nt, tris);
  return hipGetLastError();
}

}  // namespace gd
