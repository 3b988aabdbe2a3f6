// GPU construction of the f12 tree (gDist Sec. 6.3): triangles are ordered by
// the Morton code of their centroid, then split evenly over 2^floor(log2 N)
// leaves (1 or 2 consecutive triangles each) of a perfect binary tree stored
// implicitly in heap order.  The node boxes are produced by the refit kernels
// with the identity transform.
//
// Kernels here: a vertex pass (finiteness, vertex box, largest vertex norm),
// a key pass (index check and the Morton code of each centroid in the vertex
// box, packed above the triangle's index into one u64), a one-sweep LSD radix
// sort of those keys over the code bits, 8 bits per pass, and the scatter of
// triangles into leaf order.
//
// Bits per axis: 4 more than a third of floor(log2 N) (rounded up), at most
// 21 and at most what fits in 64 bits beside the index: about 2^4 cells per
// axis for each triangle's share of the mesh, so two triangles rarely share a
// cell (ties keep their input order, which is spatially coherent too) while
// the sort runs only ceil(3 b / 8) passes (5 for 7.5M triangles instead of 8
// for the full 63 bits).
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

// Vertex pass.  Each workgroup reduces its share of the vertices to 8 ints
// in part[8 * block]: vertex box min xyz, max xyz (ordered floats), an upper
// bound of the largest vertex norm |x| (a non-negative float's bits), and the
// non-finite flag (2).  A one-workgroup pass then reduces the partials into
// vb[0..6] and flags (no atomics on a few hot addresses).
constexpr int kVpThreads = 256;
__global__ __launch_bounds__(kVpThreads) void k_vertex_pass(const float* __restrict__ v, uint32_t nv,
                                                            int* __restrict__ part) {
  float lo[3] = {__builtin_huge_valf(), __builtin_huge_valf(), __builtin_huge_valf()};
  float hi[3] = {-__builtin_huge_valf(), -__builtin_huge_valf(), -__builtin_huge_valf()};
  float r2max = 0.f;   // largest squared norm
  uint32_t bad = 0;
  // (a mesh with a non-finite vertex is rejected, so its box and norm do not matter)
  auto take = [&](float x, float y, float z) {
    if (!(isfinite(x) && isfinite(y) && isfinite(z))) bad = 2u;
    lo[0] = fminf(lo[0], x); lo[1] = fminf(lo[1], y); lo[2] = fminf(lo[2], z);
    hi[0] = fmaxf(hi[0], x); hi[1] = fmaxf(hi[1], y); hi[2] = fmaxf(hi[2], z);
    r2max = fmaxf(r2max, x * x + y * y + z * z);
  };
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t t0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // four vertices (48 bytes) per thread and step, three 16-byte loads
  const uint64_t ng = nv / 4u;
  for (uint64_t g = t0; g < ng; g += stride) {
    const __attribute__((address_space(1))) float* p = gptr(v) + 12ull * g;
    const f4u a = gload<f4u>(p), b = gload<f4u>(p + 4), c = gload<f4u>(p + 8);
    take(a.x, a.y, a.z);
    take(a.w, b.x, b.y);
    take(b.z, b.w, c.x);
    take(c.y, c.z, c.w);
  }
  for (uint64_t i = 4u * ng + t0; i < nv; i += stride) take(v[3 * i], v[3 * i + 1], v[3 * i + 2]);
  float r[7];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    r[k] = wave_min_reduce(lo[k]);
    r[3 + k] = wave_max_reduce(hi[k]);
  }
  // a few roundings of relative size 2^-24 each: widen by 2^-20
  r[6] = sqrtf(wave_max_reduce(r2max)) * (1.0f + 0x1p-20f);
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
    part[8ull * blockIdx.x + k] = ordered(a);
  }
  if (threadIdx.x == 7) part[8ull * blockIdx.x + 7] = (int)s_bad;
}

__device__ __forceinline__ int wave_min_i(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// One workgroup: min of the partial minima, max of the maxima and norms, or
// of the flags (the order-preserving int map keeps min and max).
__global__ __launch_bounds__(kVpThreads) void k_vertex_final(const int* __restrict__ part, uint32_t nblocks,
                                                             int* __restrict__ vb, uint32_t* __restrict__ flags) {
  int a[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) a[k] = k < 3 ? INT_MAX : (k < 7 ? INT_MIN : 0);
  for (uint32_t b = threadIdx.x; b < nblocks; b += kVpThreads) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int x = part[8ull * b + k];
      a[k] = k < 3 ? min(a[k], x) : (k < 7 ? max(a[k], x) : (a[k] | x));
    }
  }
  __shared__ int sa[kVpThreads / 64][8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    if (k < 3) a[k] = wave_min_i(a[k]);
    else if (k < 7) a[k] = wave_max_i(a[k]);
    else for (int o = 32; o > 0; o >>= 1) a[k] |= __shfl_xor(a[k], o, 64);
  }
  const uint32_t w = threadIdx.x >> 6;
  if ((threadIdx.x & 63u) == 0u)
#pragma unroll
    for (int k = 0; k < 8; ++k) sa[w][k] = a[k];
  __syncthreads();
  if (threadIdx.x < 8) {
    const int k = threadIdx.x;
    int x = sa[0][k];
    for (int q = 1; q < kVpThreads / 64; ++q) x = k < 3 ? min(x, sa[q][k]) : (k < 7 ? max(x, sa[q][k]) : (x | sa[q][k]));
    if (k < 7) vb[k] = x;
    else *flags = (uint32_t)x;
  }
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
// packed sort key of triangle t: the Morton code of its FP32 centroid,
// normalised to the vertex box with `bits` bits per axis, shifted above the
// index_bits low bits that hold t.
__global__ void k_keys(const float* __restrict__ v, uint32_t nv, const uint32_t* __restrict__ f, uint32_t nt,
                       const int* __restrict__ vb, uint32_t bits, uint32_t index_bits, uint64_t* __restrict__ keys,
                       uint32_t* __restrict__ flags) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  const u3u fi = gload3<u3u>(f, t);
  uint64_t code = 0;
  if (fi.x >= nv || fi.y >= nv || fi.z >= nv) {
    atomicOr(flags, 1u);
  } else {
    const f3u p0 = gload3<f3u>(v, fi.x), p1 = gload3<f3u>(v, fi.y), p2 = gload3<f3u>(v, fi.z);
    const float cells = (float)(1u << bits);   // cells per axis
    const uint32_t qmax = (1u << bits) - 1u;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float lo = unordered(vb[k]), hi = unordered(vb[3 + k]);
      const float c = (p0[k] + p1[k] + p2[k]) * (1.0f / 3.0f);
      const float ext = hi - lo;
      const float u = ext > 0.f ? (c - lo) / ext : 0.f;
      const float sc = u * cells;
      const uint32_t q = sc <= 0.f ? 0u : (sc >= (float)qmax ? qmax : (uint32_t)sc);
      code |= spread3(q) << (2 - k);   // x on the highest of each bit triple
    }
  }
  keys[t] = (code << index_bits) | t;
}

// ---------------------------------------------------------------- radix sort
// One-sweep LSD radix sort of the packed keys (Morton code above the triangle
// index: every key is distinct, and sorting by the code bits alone, stably,
// gives the order of the codes with ties in index order).  One kernel counts
// the digits of every pass in a single read of the keys.  Each pass is then
// one kernel: workgroup t ranks tile t's keys by digit in LDS, learns how many
// keys with each digit the earlier tiles hold through a decoupled look-back
// over the counts those tiles publish, and writes each key to its place.
//
// A workgroup waits only for tiles of lower index.  Workgroups reach the
// compute units in index order within each XCD, so the unfinished tile of
// lowest index is always resident (every workgroup of its XCD that was placed
// before it has a lower index and has therefore finished) and never waits:
// the waits end.  Every wait is also bounded: a timeout sets a flag that the
// host reports as an error.  (No global ticket counter: one atomic per
// workgroup on a single word serialises at tens of ns each.)
constexpr int kRsThreads = 256;                         // histogram workgroups
constexpr int kRsTile = 4096;                           // keys per histogram unit of work
constexpr int kPassThreads = 512;              // pass workgroups
constexpr int kRsRowsPerWave = 16;
constexpr int kPassTile = kPassThreads * kRsRowsPerWave;  // keys per tile
constexpr uint32_t kRsMaxPasses = 8;
constexpr uint32_t kRsSpinLimit = 1u << 20;
constexpr uint32_t kLookback = 16;   // look-back words read per round trip

struct SortCtl {                                // zeroed before the sort
  uint32_t hist[kRsMaxPasses][256];             // keys per digit, per pass
  uint32_t timeout;                             // a look-back wait gave up
};
constexpr size_t kSortCtlBytes = (sizeof(SortCtl) + 255) & ~size_t(255);

// Look-back word of (pass, tile, digit), one array per pass, cleared before
// the sort: 0 = not yet published; else bit 31 = inclusive and the low bits =
// 1 + the tile's count of the digit (aggregate) or 1 + the count over tiles
// 0..tile (inclusive; below n < 2^31, so it fits).
__device__ __forceinline__ uint32_t lb_word(bool incl, uint32_t v) { return (incl ? 0x80000000u : 0u) | (v + 1u); }

// Lanes of the wave (among those with ok set) whose digit has the same low 8
// bits as d: per bit, the ballot of lanes with the bit set, xor-ed with this
// lane's bit spread over a word, marks the lanes that differ in it; the union
// over the bits is the complement (four VALU instructions per bit).
__device__ __forceinline__ uint64_t digit_peers(uint32_t d, bool ok) {
  uint32_t diff_lo = 0u, diff_hi = 0u;
#pragma unroll
  for (int bit = 0; bit < 8; ++bit) {
    const uint32_t x = (uint32_t)__builtin_amdgcn_sbfe((int32_t)d, bit, 1);   // all ones if the bit is set
    const uint64_t m = __ballot(x != 0u);
    // diff | (m ^ x) in one instruction (truth table over (diff, m, x))
    diff_lo = __builtin_amdgcn_bitop3_b32(diff_lo, (uint32_t)m, x, 0xF6);
    diff_hi = __builtin_amdgcn_bitop3_b32(diff_hi, (uint32_t)(m >> 32), x, 0xF6);
  }
  return ~(((uint64_t)diff_hi << 32) | diff_lo) & __ballot(ok);
}

// Exclusive scan of one value per thread across a workgroup of T threads
// (wave scans, then the wave totals); *total = the workgroup's sum.  s4: T / 64
// words of LDS.
template <int T>
__device__ __forceinline__ uint32_t block_exclusive(uint32_t v, uint32_t* s4, uint32_t* total) {
  const uint32_t lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  uint32_t x = v;
#pragma unroll
  for (uint32_t off = 1; off < kWave; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, kWave);
    if (lane >= off) x += y;
  }
  if (lane == kWave - 1) s4[w] = x;
  __syncthreads();
  uint32_t pre = 0, all = 0;
#pragma unroll
  for (uint32_t q = 0; q < T / kWave; ++q) {
    const uint32_t t = s4[q];
    pre += q < w ? t : 0u;
    all += t;
  }
  __syncthreads();
  *total = all;
  return pre + x - v;
}

// Digit counts of all passes: each wave takes 8 rows of 64 keys at a time
// (their loads issued together) and adds each key's digit of each pass to the
// workgroup's LDS histogram, which is then stored whole as the workgroup's row
// of `part` (passes x 256 counts).  A row whose keys share the digit adds
// once (the high digits of a spatially coherent input); otherwise every key
// adds one to copy (lane mod C) of the histogram, so that lanes with equal
// digits, which serialise on one LDS word, are spread over C words in
// different banks (copies 257 words apart).  k_sort_hist_sum adds the rows
// up: a few thousand global atomic adds to distinct words, instead of one per
// bin and workgroup.
constexpr uint32_t kHistRows = 8;
constexpr uint32_t kHistMaxBlocks = 1024;
constexpr uint32_t kHistSumRows = 32;    // partial rows per thread of the sum
constexpr uint32_t kHistCopies = 4;
__global__ __launch_bounds__(kRsThreads) void k_sort_hist(const uint64_t* __restrict__ keys, uint32_t n,
                                                           uint32_t lo_bit, uint32_t passes,
                                                           uint32_t* __restrict__ part) {
  extern __shared__ uint32_t h[];   // [passes][kHistCopies][257]
  const uint32_t words = passes * kHistCopies * 257u;
  for (uint32_t i = threadIdx.x; i < words; i += kRsThreads) h[i] = 0u;
  __syncthreads();
  const uint32_t lane = threadIdx.x % kWave;
  const uint32_t copy = (lane % kHistCopies) * 257u;
  const uint64_t rows = ((uint64_t)n + kWave - 1) / kWave;
  const uint64_t waves = (uint64_t)gridDim.x * (kRsThreads / kWave);
  for (uint64_t r0 = ((uint64_t)blockIdx.x * (kRsThreads / kWave) + threadIdx.x / kWave) * kHistRows; r0 < rows;
       r0 += waves * kHistRows) {
    uint64_t k[kHistRows];
#pragma unroll
    for (uint32_t j = 0; j < kHistRows; ++j) {
      const uint64_t i = (r0 + j) * kWave + lane;
      k[j] = i < n ? keys[i] : 0ull;
    }
#pragma unroll
    for (uint32_t j = 0; j < kHistRows; ++j) {
      if (r0 + j >= rows) break;   // uniform across the wave
      const bool ok = (r0 + j) * kWave + lane < n;
      const uint64_t live = __ballot(ok);
      for (uint32_t p = 0; p < passes; ++p) {
        const uint32_t d = (uint32_t)(k[j] >> (lo_bit + 8u * p)) & 255u;
        uint32_t* hp = h + p * (kHistCopies * 257u);
        const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
        if (__ballot(ok && d == d0) == live) {
          if (lane == 0) atomicAdd(hp + d0, (uint32_t)__popcll(live));
        } else if (ok) {
          atomicAdd(hp + copy + d, 1u);
        }
      }
    }
  }
  __syncthreads();
  uint32_t* row = part + (uint64_t)blockIdx.x * passes * 256u;
  for (uint32_t i = threadIdx.x; i < passes * 256u; i += kRsThreads) {
    const uint32_t* hp = h + (i >> 8) * (kHistCopies * 257u) + (i & 255u);
    uint32_t c = 0;
#pragma unroll
    for (uint32_t q = 0; q < kHistCopies; ++q) c += hp[q * 257u];
    row[i] = c;
  }
}

// Workgroup (p, c): thread d adds digit d of pass p over partial rows
// c*32 .. c*32+31, then one global add.
__global__ __launch_bounds__(kRsThreads) void k_sort_hist_sum(const uint32_t* __restrict__ part, uint32_t rows,
                                                               uint32_t passes, SortCtl* ctl) {
  const uint32_t p = blockIdx.x, d = threadIdx.x;
  const uint32_t r0 = blockIdx.y * kHistSumRows;
  uint32_t sum = 0;
#pragma unroll
  for (uint32_t r = 0; r < kHistSumRows; ++r)
    if (r0 + r < rows) sum += part[((uint64_t)(r0 + r) * passes + p) * 256u + d];
  if (sum) atomicAdd(&ctl->hist[p][d], sum);
}

// One pass over the digit at bit `shift`.  Wave w ranks rows w*16 .. w*16+15
// of the tile (a row = 64 consecutive keys) in order: lanes holding the same
// digit are found with eight ballots, their order inside the row comes from
// the lane mask below them, and a per-wave running count per digit carries
// the order across rows.  A per-digit prefix over the waves and an exclusive
// scan over the 256 digits give each key its place in the tile sorted by
// digit; the tile is reordered in LDS, and thread t then writes tile
// positions t, t + T, ... to the digit's global start, plus the keys with
// that digit in earlier tiles, plus the position inside the digit's run, so
// consecutive threads store consecutive addresses of one run.  Threads
// 0..255 also stand for the 256 digits (publication and look-back).
__global__ __launch_bounds__(kPassThreads) void k_sort_pass(const uint64_t* __restrict__ kin,
                                                             uint64_t* __restrict__ kout, uint32_t n,
                                                             uint32_t shift, uint32_t pass, SortCtl* ctl,
                                                             uint32_t* lb) {
  constexpr int kWaves = kPassThreads / kWave;
  __shared__ uint32_t wc[kWaves][257];
  __shared__ uint32_t lstart[256];
  __shared__ uint32_t gbase[256];
  __shared__ uint32_t scan_s[kWaves];
  __shared__ uint64_t tk[kPassTile];
  const uint32_t w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  for (uint32_t i = threadIdx.x; i < kWaves * 257; i += kPassThreads) (&wc[0][0])[i] = 0;
  __syncthreads();
  const uint32_t tile = blockIdx.x;
  uint64_t key[kRsRowsPerWave];
  uint32_t dig[kRsRowsPerWave], rk[kRsRowsPerWave];
  const uint64_t base = (uint64_t)tile * kPassTile + (uint64_t)w * kRsRowsPerWave * kWave;
  const uint64_t lt = (1ull << lane) - 1ull;
#pragma unroll
  for (int r = 0; r < kRsRowsPerWave; ++r) {
    const uint64_t i = base + (uint64_t)r * kWave + lane;
    key[r] = i < n ? kin[i] : 0ull;
  }
#pragma unroll
  for (int r = 0; r < kRsRowsPerWave; ++r) {
    const bool ok = base + (uint64_t)r * kWave + lane < n;
    const uint32_t d = ok ? (uint32_t)((key[r] >> shift) & 255u) : 256u;
    dig[r] = d;
    const uint64_t same = digit_peers(d, ok);
    const uint32_t prev = ok ? wc[w][d] : 0u;
    rk[r] = prev + (uint32_t)__popcll(same & lt);
    // lowest lane of each digit group advances that digit's running count
    if (ok && (same & lt) == 0ull) wc[w][d] = prev + (uint32_t)__popcll(same);
  }
  __syncthreads();
  const bool is_digit = threadIdx.x < 256u;
  const uint32_t d = threadIdx.x & 255u;   // the digit of threads 0..255
  uint32_t run = 0;
  if (is_digit) {
#pragma unroll
    for (int q = 0; q < kWaves; ++q) {
      const uint32_t c = wc[q][d];
      wc[q][d] = run;
      run += c;
    }
  }
  // publish this tile's count of digit d (tile 0: already the inclusive count)
  uint32_t* const lbp = lb + (uint64_t)pass * gridDim.x * 256u;
  uint32_t* const my = lbp + (uint64_t)tile * 256u + d;
  if (is_digit) __hip_atomic_store(my, lb_word(tile == 0u, run), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  uint32_t total;
  const uint32_t ls = block_exclusive<kPassThreads>(is_digit ? run : 0u, scan_s, &total);
  if (is_digit) lstart[d] = ls;
  const uint32_t gstart = block_exclusive<kPassThreads>(is_digit ? ctl->hist[pass][d] : 0u, scan_s, &total);
#pragma unroll
  for (int r = 0; r < kRsRowsPerWave; ++r) {
    if (dig[r] < 256u) tk[lstart[dig[r]] + wc[w][dig[r]] + rk[r]] = key[r];
  }
  // look back over the earlier tiles' counts of digit d, kLookback tiles per
  // round trip: add published counts from the nearest tile down, up to and
  // including the first inclusive one; an unpublished tile ends the window
  // and is read again.
  if (is_digit) {
    uint32_t before = 0;
    if (tile > 0u) {
      uint32_t j = tile, spins = 0;   // tiles below j are still to be added
      for (;;) {
        uint32_t wd[kLookback];
#pragma unroll
        for (uint32_t q = 0; q < kLookback; ++q)
          wd[q] = q < j ? __hip_atomic_load(lbp + (uint64_t)(j - 1u - q) * 256u + d, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT)
                        : 0u;
        bool done = false;
        uint32_t used = 0;
#pragma unroll
        for (uint32_t q = 0; q < kLookback; ++q) {
          if (done || used != q || q >= j || wd[q] == 0u) continue;   // a zero word ends the window
          before += (wd[q] & 0x7fffffffu) - 1u;
          used = q + 1u;
          done = (wd[q] >> 31) != 0u;
        }
        j -= used;
        if (done || j == 0u) break;
        if (used == 0u) {
          if (++spins > kRsSpinLimit) {
            __hip_atomic_store(&ctl->timeout, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
      __hip_atomic_store(my, lb_word(true, before + run), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    gbase[d] = gstart + before - lstart[d];
  }
  __syncthreads();
  const uint64_t tile0 = (uint64_t)tile * kPassTile;
  const uint32_t valid = n - tile0 < (uint64_t)kPassTile ? (uint32_t)(n - tile0) : (uint32_t)kPassTile;
  for (uint32_t i = threadIdx.x; i < valid; i += kPassThreads) {
    const uint64_t k = tk[i];
    const uint32_t pos = gbase[(uint32_t)(k >> shift) & 255u] + i;
    if (pos < n) kout[pos] = k;   // always, unless a look-back wait timed out
  }
}

// Tree of a new mesh (identity pose).  Workgroup blk owns leaves
// [blk S, blk S + S) of the L = 2^D leaves, S = min(L, 512): leaf j holds the
// key-order triangles [floor(j n / L), floor((j + 1) n / L)) (1 or 2), so the
// workgroup's leaves hold one run of at most 2S triangles.  It gathers them
// (sorted key -> caller index -> vertex indices -> vertices) into LDS, writes
// them out as one contiguous run with 16-byte stores, computes its leaf boxes
// from LDS and reduces its subtree there, writing every node once.  The
// upper levels follow in k_reduce_levels.
constexpr int kTreeThreads = 512;
__global__ __launch_bounds__(kTreeThreads) void k_emit_tree(const float* __restrict__ v, uint32_t nv,
                                                            const uint32_t* __restrict__ f, uint32_t nt,
                                                            const uint64_t* __restrict__ sorted, uint64_t index_mask,
                                                            uint32_t L, uint32_t S, float* __restrict__ tris,
                                                            uint32_t* __restrict__ orig, uint32_t* __restrict__ fl,
                                                            float* __restrict__ boxes) {
  __shared__ __align__(16) float st[18 * kTreeThreads];
  __shared__ Box lb[kTreeThreads];
  const uint32_t D = 31u - (uint32_t)__clz(L);
  const uint32_t blk = blockIdx.x;
  const uint32_t t0 = (uint32_t)(((uint64_t)blk * S * nt) >> D);
  const uint32_t t1 = (uint32_t)(((uint64_t)(blk * S + S) * nt) >> D);
  const uint32_t cnt = t1 - t0;   // <= 2 S
  for (uint32_t i = threadIdx.x; i < cnt; i += kTreeThreads) {
    const uint64_t sp = (uint64_t)t0 + i;
    uint32_t o = (uint32_t)(sorted[sp] & index_mask);
    if (o >= nt) o = nt - 1u;   // only after a sort timeout, which rejects the mesh
    orig[sp] = o;
    const u3u fi = gload3<u3u>(f, o);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const uint32_t vi = fi[c];
      if (fl) fl[3ull * sp + c] = vi;
      const f3u p = gload3<f3u>(v, vi < nv ? vi : nv - 1u);
#pragma unroll
      for (int k = 0; k < 3; ++k) st[9 * i + 3 * c + k] = p[k];
    }
  }
  __syncthreads();
  // the run starts at float 9 t0 of a 16-byte aligned array: a scalar head
  // up to the next 16-byte boundary, 16-byte stores, a scalar tail
  const uint32_t nf = 9u * cnt;
  float* out = tris + 9ull * t0;
  uint32_t head = (4u - (uint32_t)((9ull * t0) & 3ull)) & 3u;
  if (head > nf) head = nf;
  const uint32_t n4 = (nf - head) >> 2;
  if (threadIdx.x < head) out[threadIdx.x] = st[threadIdx.x];
  for (uint32_t i = threadIdx.x; i < n4; i += kTreeThreads) {
    const uint32_t q = head + 4u * i;
    f4v x;
    x.x = st[q];
    x.y = st[q + 1];
    x.z = st[q + 2];
    x.w = st[q + 3];
    *reinterpret_cast<f4v*>(out + q) = x;
  }
  for (uint32_t i = head + 4u * n4 + threadIdx.x; i < nf; i += kTreeThreads) out[i] = st[i];
  // leaf boxes (the identity pose: the vertices themselves)
  const uint32_t j = threadIdx.x;
  if (j < S) {
    Box b;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      b.lo[k] = __builtin_huge_valf();
      b.hi[k] = -__builtin_huge_valf();
    }
    const uint32_t leaf = blk * S + j;
    const uint32_t start = (uint32_t)(((uint64_t)leaf * nt) >> D);
    const uint32_t end = (uint32_t)(((uint64_t)(leaf + 1) * nt) >> D);
    for (uint32_t p = start; p < end; ++p) {
      const float* q = st + 9u * (p - t0);
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          b.lo[k] = fminf(b.lo[k], q[3 * c + k]);
          b.hi[k] = fmaxf(b.hi[k], q[3 * c + k]);
        }
    }
    store_box(boxes, L + leaf, b);
    lb[j] = b;
  }
  uint32_t base = L + blk * S;
  for (uint32_t c = S; c > 1; c >>= 1) {
    __syncthreads();
    Box nb;
    const bool act = j < c / 2;
    if (act) nb = box_union(lb[2 * j], lb[2 * j + 1]);
    __syncthreads();
    base >>= 1;
    if (act) {
      lb[j] = nb;
      store_box(boxes, base + j, nb);
    }
  }
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
constexpr uint32_t kVpMaxBlocks = 1024;

size_t vertex_pass_scratch_bytes() { return (size_t)kVpMaxBlocks * 8u * sizeof(int); }

hipError_t launch_vertex_pass(const float* v, uint32_t nv, int* vb, uint32_t* flags, int* part, hipStream_t s) {
  uint32_t blocks = (uint32_t)(((uint64_t)nv / 4u + kVpThreads - 1) / kVpThreads);
  if (blocks > kVpMaxBlocks) blocks = kVpMaxBlocks;
  if (blocks == 0) blocks = 1;
  k_vertex_pass<<<blocks, kVpThreads, 0, s>>>(v, nv, part);
  k_vertex_final<<<1, kVpThreads, 0, s>>>(part, blocks, vb, flags);
  return hipGetLastError();
}

KeyLayout key_layout(uint32_t nt) {
  uint32_t d = 0;
  while (d < 31u && (2u << d) <= nt) ++d;   // floor(log2 nt)
  uint32_t ib = 0;
  while (ib < 32u && (1ull << ib) < nt) ++ib;   // bits of the largest index nt - 1
  uint32_t b = (d + 2u) / 3u + 4u;
  if (b > 21u) b = 21u;
  if (3u * b + ib > 64u) b = (64u - ib) / 3u;
  return KeyLayout{ib, b};
}

hipError_t launch_keys(const float* v, uint32_t nv, const uint32_t* f, uint32_t nt, const int* vb, uint64_t* keys,
                       uint32_t* flags, hipStream_t s) {
  const KeyLayout kl = key_layout(nt);
  k_keys<<<(nt + 255) / 256, 256, 0, s>>>(v, nv, f, nt, vb, kl.axis_bits, kl.index_bits, keys, flags);
  return hipGetLastError();
}

static uint32_t hist_blocks(uint32_t n) {
  const uint32_t units = (uint32_t)(((uint64_t)n + kRsTile - 1) / kRsTile);
  return units < kHistMaxBlocks ? units : kHistMaxBlocks;
}

static uint64_t pass_tiles(uint32_t n) { return ((uint64_t)n + kPassTile - 1) / kPassTile; }

// SortCtl, the look-back words (one per pass, tile and digit), the histogram
// partials (one row of up to 8 x 256 counts per histogram workgroup)
size_t sort_workspace_bytes(uint32_t n) {
  return kSortCtlBytes + (size_t)kRsMaxPasses * pass_tiles(n) * 256u * sizeof(uint32_t) +
         (size_t)hist_blocks(n) * kRsMaxPasses * 256u * sizeof(uint32_t);
}

const uint32_t* sort_timeout_flag(const void* ws) { return &reinterpret_cast<const SortCtl*>(ws)->timeout; }

hipError_t launch_sort(uint64_t* keys, uint64_t* keys_tmp, uint32_t n, uint32_t lo_bit, uint32_t nbits, void* ws,
                       hipStream_t s, int* result_in_tmp) {
  const uint32_t passes = (nbits + 7u) / 8u;
  if (n == 0 || passes == 0 || passes > kRsMaxPasses || lo_bit + nbits > 64u) return hipErrorInvalidValue;
  const uint32_t tiles = (uint32_t)pass_tiles(n);
  SortCtl* ctl = reinterpret_cast<SortCtl*>(ws);
  uint32_t* lb = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(ws) + kSortCtlBytes);
  uint32_t* part = lb + (uint64_t)kRsMaxPasses * tiles * 256u;
  // the partial rows are written whole before they are read: clear the rest
  hipError_t e = hipMemsetAsync(ws, 0, kSortCtlBytes + (size_t)passes * tiles * 256u * sizeof(uint32_t), s);
  if (e != hipSuccess) return e;
  const uint32_t hb = hist_blocks(n);
  k_sort_hist<<<hb, kRsThreads, passes * kHistCopies * 257u * sizeof(uint32_t), s>>>(keys, n, lo_bit, passes, part);
  k_sort_hist_sum<<<dim3(passes, (hb + kHistSumRows - 1) / kHistSumRows), kRsThreads, 0, s>>>(part, hb, passes, ctl);
  uint64_t *ki = keys, *ko = keys_tmp;
  for (uint32_t p = 0; p < passes; ++p) {
    k_sort_pass<<<tiles, kPassThreads, 0, s>>>(ki, ko, n, lo_bit + 8u * p, p, ctl, lb);
    uint64_t* t = ki;
    ki = ko;
    ko = t;
  }
  *result_in_tmp = (ki == keys_tmp);
  return hipGetLastError();
}

hipError_t launch_emit_tree(const float* v, uint32_t nv, const uint32_t* f, uint32_t nt, const uint64_t* sorted,
                            uint32_t index_bits, uint32_t L, float* tris, uint32_t* orig, uint32_t* fl, float* boxes,
                            hipStream_t s) {
  const uint64_t mask = index_bits >= 64u ? ~0ull : (1ull << index_bits) - 1ull;
  const uint32_t S = L < (uint32_t)kTreeThreads ? L : (uint32_t)kTreeThreads;
  k_emit_tree<<<L / S, kTreeThreads, 0, s>>>(v, nv, f, nt, sorted, mask, L, S, tris, orig, fl, boxes);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_reduce_upper(boxes, L / S, s);
}

hipError_t launch_gather_tris(const float* v, const uint32_t* fl, uint32_t nt, float* tris, hipStream_t s) {
  k_gather_tris<<<(nt + 255) / 256, 256, 0, s>>>(v, fl, nt, tris);
  return hipGetLastError();
}

}  // namespace gd
