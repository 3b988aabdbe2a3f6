// Device-side building blocks of the mesh-distance path (gfx950).
//
// - Box loads/stores (node boxes are 6 floats, heap order, 1-based ids).
// - The FP32 rigid transform used by both the refit and the narrow phase, with
//   an explicit fused-multiply-add order so the two produce identical bits.
// - AABB distance bounds of gDist Sec. 4: conventional lower bound of the
//   minimum and upper bound of the maximum, plus the enhanced bounds (best
//   face-rectangle pair).  The 36 face pairs are factorised: a face pair only
//   changes the per-axis terms of the axis each face is flat in, so every one
//   of the 36 squared distances is a sum of three non-negative per-axis terms
//   (no subtraction, hence no cancellation in FP32), and the minimum (maximum)
//   over the 36 reduces to 9 candidate sums.
// - Exact triangle-triangle distance (min over the 6 vertex-triangle and 9
//   edge-edge feature pairs; zero if an edge crosses the other triangle) in a
//   precision-generic template, instantiated in FP32 for the narrow phase and
//   in FP64 for the re-evaluation.  Vertex-triangle uses the Voronoi-region
//   walk (Ericson, Real-Time Collision Detection, 2005, 5.1.5), edge-edge the
//   clamped two-parameter solve (same book, 5.1.9).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gd {

constexpr int kWave = 64;

struct Box {
  float lo[3], hi[3];
};

// Mesh data always lives in device global memory; pointers read from
// descriptors are generic to the compiler, so loads through them would be
// flat accesses (which also hold the LDS wait counter).  Casting to the global
// address space keeps them plain global loads.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gptr(const T* p) {
  return (const __attribute__((address_space(1))) T*)(p);
}

typedef float f2v __attribute__((ext_vector_type(2)));
// Multi-dword global loads need only 4-byte alignment on this target, so a
// 16-byte piece of a 24-byte box or a 36-byte triangle is one instruction.
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f3u __attribute__((ext_vector_type(3), aligned(4)));        // a vertex
typedef uint32_t u3u __attribute__((ext_vector_type(3), aligned(4)));     // a triangle's vertex indices
template <typename V, typename T>
__device__ __forceinline__ V gload3(const T* p, uint64_t i) {   // element i of an array of 3-vectors
  return *reinterpret_cast<const __attribute__((address_space(1))) V*>(gptr(p) + 3ull * i);
}
template <typename T>
__device__ __forceinline__ T gload(const __attribute__((address_space(1))) float* p) {
  return *reinterpret_cast<const __attribute__((address_space(1))) T*>(p);
}

__device__ __forceinline__ Box load_box(const float* __restrict__ boxes, uint32_t node) {
  const __attribute__((address_space(1))) float* p = gptr(boxes) + 6ull * node;
  const f4u u = gload<f4u>(p);
  const f2v w = gload<f2v>(p + 4);
  Box r;
  r.lo[0] = u.x; r.lo[1] = u.y; r.lo[2] = u.z;
  r.hi[0] = u.w; r.hi[1] = w.x; r.hi[2] = w.y;
  return r;
}
// The two sibling boxes of an even node id (48 bytes, 16-byte aligned).
__device__ __forceinline__ void load_box_pair(const float* __restrict__ boxes, uint32_t even_node, Box* b) {
  const __attribute__((address_space(1))) float* p = gptr(boxes) + 6ull * even_node;
  const f4v u = gload<f4v>(p), v = gload<f4v>(p + 4), w = gload<f4v>(p + 8);
  b[0].lo[0] = u.x; b[0].lo[1] = u.y; b[0].lo[2] = u.z;
  b[0].hi[0] = u.w; b[0].hi[1] = v.x; b[0].hi[2] = v.y;
  b[1].lo[0] = v.z; b[1].lo[1] = v.w; b[1].lo[2] = w.x;
  b[1].hi[0] = w.y; b[1].hi[1] = w.z; b[1].hi[2] = w.w;
}

__device__ __forceinline__ void store_box(float* __restrict__ boxes, uint32_t node, const Box& b) {
  float2* p = reinterpret_cast<float2*>(boxes + 6ull * node);
  p[0] = make_float2(b.lo[0], b.lo[1]);
  p[1] = make_float2(b.lo[2], b.hi[0]);
  p[2] = make_float2(b.hi[1], b.hi[2]);
}

__device__ __forceinline__ Box box_union(const Box& a, const Box& b) {
  Box r;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    r.lo[i] = fminf(a.lo[i], b.lo[i]);
    r.hi[i] = fmaxf(a.hi[i], b.hi[i]);
  }
  return r;
}

// FP32 rigid transform, row-major R (9) and t (3):
// x'_i = fma(R_i0, x, fma(R_i1, y, fma(R_i2, z, t_i))).
struct Xf32 {
  float R[9];
  float t[3];
};

__device__ __forceinline__ void xform(const Xf32& T, float x, float y, float z, float* o) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
    o[i] = __builtin_fmaf(T.R[3 * i + 0], x,
                          __builtin_fmaf(T.R[3 * i + 1], y, __builtin_fmaf(T.R[3 * i + 2], z, T.t[i])));
}

// Load triangle `pos` (9 floats, leaf order) and optionally transform it.
__device__ __forceinline__ void load_tri(const float* __restrict__ tris, uint32_t pos, float* o) {
  const __attribute__((address_space(1))) float* p = gptr(tris) + 9ull * pos;
  const f4u u = gload<f4u>(p), v = gload<f4u>(p + 4);
  o[0] = u.x; o[1] = u.y; o[2] = u.z; o[3] = u.w;
  o[4] = v.x; o[5] = v.y; o[6] = v.z; o[7] = v.w;
  o[8] = p[8];
}
__device__ __forceinline__ void load_tri_xf(const float* __restrict__ tris, uint32_t pos, const Xf32& T,
                                            float* o) {
  float v[9];
  load_tri(tris, pos, v);
#pragma unroll
  for (int k = 0; k < 3; ++k) xform(T, v[3 * k], v[3 * k + 1], v[3 * k + 2], o + 3 * k);
}

// Square root and reciprocal square root of the FP32 path: the hardware
// instructions, within 1 ulp for normal inputs (the IEEE-rounded library
// forms cost about fifteen and five instructions each).  A squared distance
// below the smallest normal float (distances below 2^-63) may lose its
// relative accuracy, an absolute error below 2^-63, which the error window
// covers because the traversal floors its coordinate scale M at 2^-40.  Every
// FP32 value of the path is widened by that window; final values are FP64.
__device__ __forceinline__ float sqrt32(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float rsqrt32(float x) { return __builtin_amdgcn_rsqf(x); }

// --------------------------------------------------------------------------
// AABB bounds (Sec. 4)
// --------------------------------------------------------------------------
__device__ __forceinline__ float sq(float x) { return x * x; }

// The bounds come in two parts: the cull bound (conventional d_min^L for the
// minimum, conventional d_max^U for the maximum), needed for every pair, and
// the improving bound (enhanced d_min^U, resp. enhanced d_max^L), which can
// only help when the cull bound already beats the running best.  Each part
// is a sum of non-negative per-axis squares, so no subtraction cancels.

// Conventional d_min^L: the gap between the boxes.
__device__ __forceinline__ float min_lower(const Box& a, const Box& b) {
  float sgap = 0.f;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    float gap = fmaxf(0.f, fmaxf(b.lo[i] - a.hi[i], a.lo[i] - b.hi[i]));
    sgap += gap * gap;
  }
  return sqrt32(sgap);
}

// Enhanced d_min^U (Sec. 4): the smallest, over the 36 pairs of a face of A
// and a face of B, of the largest distance between the two faces; or, if
// !enhanced, the conventional upper bound d_max^U (farthest corners).
__device__ __forceinline__ float min_upper(const Box& a, const Box& b, bool enhanced) {
  float F[3], G[3], H[3], E[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) F[i] = sq(fmaxf(b.hi[i] - a.lo[i], a.hi[i] - b.lo[i]));   // full intervals
  if (!enhanced) return sqrt32(F[0] + F[1] + F[2]);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    // A's face flat on axis i at a in {lo, hi} against B's full interval
    float ga = fminf(fmaxf(a.lo[i] - b.lo[i], b.hi[i] - a.lo[i]), fmaxf(a.hi[i] - b.lo[i], b.hi[i] - a.hi[i]));
    // B's face flat on axis i against A's full interval
    float hb = fminf(fmaxf(b.lo[i] - a.lo[i], a.hi[i] - b.lo[i]), fmaxf(b.hi[i] - a.lo[i], a.hi[i] - b.hi[i]));
    // both faces flat on axis i: nearest pair of the two face planes
    float e = fminf(fminf(fabsf(a.lo[i] - b.lo[i]), fabsf(a.lo[i] - b.hi[i])),
                    fminf(fabsf(a.hi[i] - b.lo[i]), fabsf(a.hi[i] - b.hi[i])));
    G[i] = ga * ga;
    H[i] = hb * hb;
    E[i] = e * e;
  }
  // p != q: the third axis keeps its full-interval term
  float m = F[2] + fminf(G[0] + H[1], G[1] + H[0]);
  m = fminf(m, F[1] + fminf(G[0] + H[2], G[2] + H[0]));
  m = fminf(m, F[0] + fminf(G[1] + H[2], G[2] + H[1]));
  // p == q
  m = fminf(m, E[0] + (F[1] + F[2]));
  m = fminf(m, E[1] + (F[0] + F[2]));
  m = fminf(m, E[2] + (F[0] + F[1]));
  return sqrt32(m);
}

// Min-distance bounds of two boxes: `lower` = conventional d_min^L,
// `upper` = enhanced d_min^U (or, if !enhanced, the conventional upper bound
// d_max^U, the distance between the farthest points of the boxes).
__device__ __forceinline__ void bounds_min(const Box& a, const Box& b, bool enhanced, float& lower,
                                           float& upper) {
  lower = min_lower(a, b);
  upper = min_upper(a, b, enhanced);
}

// Conventional d_max^U: the distance between the farthest corners.
__device__ __forceinline__ float max_upper(const Box& a, const Box& b) {
  float F = 0.f;
#pragma unroll
  for (int i = 0; i < 3; ++i) F += sq(fmaxf(b.hi[i] - a.lo[i], a.hi[i] - b.lo[i]));
  return sqrt32(F);
}

// Enhanced d_max^L (Sec. 4, the mirror image for the maximum): the largest,
// over the 36 face pairs, of the smallest distance between the two faces; or,
// if !enhanced, the conventional lower bound d_min^L.
__device__ __forceinline__ float max_lower(const Box& a, const Box& b, bool enhanced) {
  float Gp[3], A2[3], B2[3], E[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    float gap = fmaxf(0.f, fmaxf(b.lo[i] - a.hi[i], a.lo[i] - b.hi[i]));
    Gp[i] = gap * gap;
  }
  if (!enhanced) return sqrt32(Gp[0] + Gp[1] + Gp[2]);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    // point a (a face of A flat on axis i) against B's interval: its gap
    float ga = fmaxf(fmaxf(0.f, fmaxf(b.lo[i] - a.lo[i], a.lo[i] - b.hi[i])),
                     fmaxf(0.f, fmaxf(b.lo[i] - a.hi[i], a.hi[i] - b.hi[i])));
    float hb = fmaxf(fmaxf(0.f, fmaxf(a.lo[i] - b.lo[i], b.lo[i] - a.hi[i])),
                     fmaxf(0.f, fmaxf(a.lo[i] - b.hi[i], b.hi[i] - a.hi[i])));
    float e = fmaxf(fmaxf(fabsf(a.lo[i] - b.lo[i]), fabsf(a.lo[i] - b.hi[i])),
                    fmaxf(fabsf(a.hi[i] - b.lo[i]), fabsf(a.hi[i] - b.hi[i])));
    A2[i] = ga * ga;
    B2[i] = hb * hb;
    E[i] = e * e;
  }
  float m = Gp[2] + fmaxf(A2[0] + B2[1], A2[1] + B2[0]);
  m = fmaxf(m, Gp[1] + fmaxf(A2[0] + B2[2], A2[2] + B2[0]));
  m = fmaxf(m, Gp[0] + fmaxf(A2[1] + B2[2], A2[2] + B2[1]));
  m = fmaxf(m, E[0] + (Gp[1] + Gp[2]));
  m = fmaxf(m, E[1] + (Gp[0] + Gp[2]));
  m = fmaxf(m, E[2] + (Gp[0] + Gp[1]));
  return sqrt32(m);
}

// Max-distance bounds: `upper` = conventional d_max^U, `lower` = enhanced
// d_max^L (or, if !enhanced, the conventional d_min^L).
__device__ __forceinline__ void bounds_max(const Box& a, const Box& b, bool enhanced, float& upper,
                                           float& lower) {
  upper = max_upper(a, b);
  lower = max_lower(a, b, enhanced);
}

// --------------------------------------------------------------------------
// Triangle-triangle distance, precision-generic
// --------------------------------------------------------------------------
template <typename T>
struct V3 {
  T x, y, z;
};
template <typename T>
__device__ __forceinline__ V3<T> mk(T x, T y, T z) {
  V3<T> r;
  r.x = x; r.y = y; r.z = z;
  return r;
}
template <typename T>
__device__ __forceinline__ V3<T> operator-(V3<T> a, V3<T> b) { return mk<T>(a.x - b.x, a.y - b.y, a.z - b.z); }
template <typename T>
__device__ __forceinline__ V3<T> operator+(V3<T> a, V3<T> b) { return mk<T>(a.x + b.x, a.y + b.y, a.z + b.z); }
template <typename T>
__device__ __forceinline__ V3<T> operator*(V3<T> a, T s) { return mk<T>(a.x * s, a.y * s, a.z * s); }
template <typename T>
__device__ __forceinline__ T dot(V3<T> a, V3<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <typename T>
__device__ __forceinline__ V3<T> cross(V3<T> a, V3<T> b) {
  return mk<T>(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
template <typename T>
__device__ __forceinline__ T inf_of();
template <>
__device__ __forceinline__ float inf_of<float>() { return __builtin_huge_valf(); }
template <>
__device__ __forceinline__ double inf_of<double>() { return __builtin_huge_val(); }

template <typename T>
__device__ __forceinline__ T safe_ratio(T num, T den) { return den > T(0) ? num / den : T(0); }
template <typename T>
__device__ __forceinline__ T clamp01(T x) { return x < T(0) ? T(0) : (x > T(1) ? T(1) : x); }

// Squared distance from p to closed triangle (a,b,c); closest point in *q.
// Regions are visited vertex A, vertex B, edge AB, vertex C, edge AC, edge BC,
// then the face.  A face hit of a zero-area triangle returns +inf: the
// edge-edge pairs already cover a degenerate triangle.
template <typename T, bool PTS>
__device__ __forceinline__ T pt_tri_d2(V3<T> p, V3<T> a, V3<T> b, V3<T> c, V3<T>* q) {
  V3<T> ab = b - a, ac = c - a, ap = p - a;
  T d1 = dot(ab, ap), d2 = dot(ac, ap);
  V3<T> r;
  if (d1 <= T(0) && d2 <= T(0)) {
    r = a;
  } else {
    V3<T> bp = p - b;
    T d3 = dot(ab, bp), d4 = dot(ac, bp);
    T vc = d1 * d4 - d3 * d2;
    if (d3 >= T(0) && d4 <= d3) {
      r = b;
    } else if (vc <= T(0) && d1 >= T(0) && d3 <= T(0)) {
      r = a + ab * safe_ratio(d1, d1 - d3);
    } else {
      V3<T> cp = p - c;
      T d5 = dot(ab, cp), d6 = dot(ac, cp);
      T vb = d5 * d2 - d1 * d6;
      if (d6 >= T(0) && d5 <= d6) {
        r = c;
      } else if (vb <= T(0) && d2 >= T(0) && d6 <= T(0)) {
        r = a + ac * safe_ratio(d2, d2 - d6);
      } else {
        T va = d3 * d6 - d5 * d4;
        T e1 = d4 - d3, e2 = d5 - d6;
        if (va <= T(0) && e1 >= T(0) && e2 >= T(0)) {
          r = b + (c - b) * safe_ratio(e1, e1 + e2);
        } else {
          T den = va + vb + vc;
          if (!(den > T(0))) return inf_of<T>();
          T v = vb / den, w = vc / den;
          r = a + ab * v + ac * w;
        }
      }
    }
  }
  if (PTS) *q = r;
  V3<T> d = p - r;
  return dot(d, d);
}

// Squared distance between segments [p1,q1] and [p2,q2]; closest points.
template <typename T, bool PTS>
__device__ __forceinline__ T seg_seg_d2(V3<T> p1, V3<T> q1, V3<T> p2, V3<T> q2, V3<T>* c1, V3<T>* c2) {
  V3<T> d1 = q1 - p1, d2 = q2 - p2, r = p1 - p2;
  T a = dot(d1, d1), e = dot(d2, d2), f = dot(d2, r);
  T s, t;
  if (a <= T(0) && e <= T(0)) {
    s = T(0); t = T(0);
  } else if (a <= T(0)) {
    s = T(0);
    t = clamp01(f / e);
  } else {
    T c = dot(d1, r);
    if (e <= T(0)) {
      t = T(0);
      s = clamp01(-c / a);
    } else {
      T b = dot(d1, d2);
      T den = a * e - b * b;
      s = den > T(0) ? clamp01((b * f - c * e) / den) : T(0);
      t = (b * s + f) / e;
      if (t < T(0)) {
        t = T(0);
        s = clamp01(-c / a);
      } else if (t > T(1)) {
        t = T(1);
        s = clamp01((b - c) / a);
      }
    }
  }
  V3<T> x = p1 + d1 * s, y = p2 + d2 * t;
  if (PTS) { *c1 = x; *c2 = y; }
  V3<T> d = x - y;
  return dot(d, d);
}

// Does segment [p0,p1] cross the plane of triangle (a,b,c) (normal n) at a
// single point inside the closed triangle?  Endpoints on the plane are left
// to the feature tests.
template <typename T>
__device__ __forceinline__ bool seg_crosses(V3<T> p0, V3<T> p1, V3<T> a, V3<T> b, V3<T> c, V3<T> n, V3<T>* x) {
  T s0 = dot(p0 - a, n), s1 = dot(p1 - a, n);
  if (!((s0 > T(0) && s1 < T(0)) || (s0 < T(0) && s1 > T(0)))) return false;
  V3<T> X = p0 + (p1 - p0) * (s0 / (s0 - s1));
  if (dot(cross(b - a, X - a), n) < T(0)) return false;
  if (dot(cross(c - b, X - b), n) < T(0)) return false;
  if (dot(cross(a - c, X - c), n) < T(0)) return false;
  *x = X;
  return true;
}

// Squared min distance between closed triangles P, Q (3 vertices each).
template <typename T, bool PTS>
__device__ __forceinline__ T tri_tri_min_d2(const V3<T>* P, const V3<T>* Q, V3<T>* cp, V3<T>* cq) {
  T best = inf_of<T>();
  V3<T> bp = P[0], bq = Q[0], u, w;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    T d = pt_tri_d2<T, PTS>(P[i], Q[0], Q[1], Q[2], &w);
    if (d < best) { best = d; if (PTS) { bp = P[i]; bq = w; } }
  }
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    T d = pt_tri_d2<T, PTS>(Q[j], P[0], P[1], P[2], &u);
    if (d < best) { best = d; if (PTS) { bp = u; bq = Q[j]; } }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      T d = seg_seg_d2<T, PTS>(P[i], P[(i + 1) % 3], Q[j], Q[(j + 1) % 3], &u, &w);
      if (d < best) { best = d; if (PTS) { bp = u; bq = w; } }
    }
  if (best > T(0)) {
    V3<T> nq = cross(Q[1] - Q[0], Q[2] - Q[0]);
    V3<T> np = cross(P[1] - P[0], P[2] - P[0]);
    V3<T> x;
    bool hit = false;
    if (dot(nq, nq) > T(0)) {
#pragma unroll
      for (int i = 0; i < 3; ++i)
        if (!hit && seg_crosses<T>(P[i], P[(i + 1) % 3], Q[0], Q[1], Q[2], nq, &x)) hit = true;
    }
    if (!hit && dot(np, np) > T(0)) {
#pragma unroll
      for (int j = 0; j < 3; ++j)
        if (!hit && seg_crosses<T>(Q[j], Q[(j + 1) % 3], P[0], P[1], P[2], np, &x)) hit = true;
    }
    if (hit) { best = T(0); if (PTS) { bp = x; bq = x; } }
  }
  if (PTS) { *cp = bp; *cq = bq; }
  return best;
}

// Squared max distance: the largest of the 9 vertex-pair distances.
template <typename T, bool PTS>
__device__ __forceinline__ T tri_tri_max_d2(const V3<T>* P, const V3<T>* Q, V3<T>* cp, V3<T>* cq) {
  T best = T(-1);
  int bi = 0, bj = 0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      V3<T> d = P[i] - Q[j];
      T s = dot(d, d);
      if (s > best) { best = s; bi = i; bj = j; }
    }
  if (PTS) { *cp = P[bi]; *cq = Q[bj]; }
  return best;
}

// --------------------------------------------------------------------------
// Wave helpers
// --------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// number of set bits of `mask` below this lane
__device__ __forceinline__ uint32_t rank_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Wave-wide min / max (the whole wave active): DPP exchanges inside each row
// of 16 lanes (quad swaps, then half-row and row mirrors leave every lane with
// its row's extreme), then the four row results are read as scalars.  No LDS
// traffic, unlike shuffles through the LDS crossbar.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v, float id) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(id), __float_as_int(v), CTRL, 0xf, 0xf, false));
}
__device__ __forceinline__ float row_lanes(float v, int l) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l)); }
__device__ __forceinline__ float wave_min(float v) {
  const float id = __builtin_huge_valf();
  v = fminf(v, dpp_f<0xB1>(v, id));    // quad_perm [1,0,3,2]
  v = fminf(v, dpp_f<0x4E>(v, id));    // quad_perm [2,3,0,1]
  v = fminf(v, dpp_f<0x141>(v, id));   // row_half_mirror
  v = fminf(v, dpp_f<0x140>(v, id));   // row_mirror
  return fminf(fminf(row_lanes(v, 0), row_lanes(v, 16)), fminf(row_lanes(v, 32), row_lanes(v, 48)));
}
__device__ __forceinline__ float wave_max(float v) {
  const float id = -__builtin_huge_valf();
  v = fmaxf(v, dpp_f<0xB1>(v, id));
  v = fmaxf(v, dpp_f<0x4E>(v, id));
  v = fmaxf(v, dpp_f<0x141>(v, id));
  v = fmaxf(v, dpp_f<0x140>(v, id));
  return fmaxf(fmaxf(row_lanes(v, 0), row_lanes(v, 16)), fmaxf(row_lanes(v, 32), row_lanes(v, 48)));
}
// Wave-wide sum (the whole wave active), same exchange pattern: after the
// quad swaps each lane holds its quad's sum, after the half-row mirror its
// half-row's, after the row mirror its row's.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_add(uint32_t v) {
  return v + (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xf, 0xf, false);
}
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
  v = dpp_add<0xB1>(v);
  v = dpp_add<0x4E>(v);
  v = dpp_add<0x141>(v);
  v = dpp_add<0x140>(v);
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 0) + (uint32_t)__builtin_amdgcn_readlane((int)v, 16) +
         (uint32_t)__builtin_amdgcn_readlane((int)v, 32) + (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
}
// Value of lane l (wave-uniform l) as a scalar.
__device__ __forceinline__ uint32_t lane_value(uint32_t v, uint32_t l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)l);
}

// Non-negative floats order like their bit patterns: atomics on the bits.
__device__ __forceinline__ uint32_t fbits(float x) { return __float_as_uint(x); }
__device__ __forceinline__ float bitsf(uint32_t x) { return __uint_as_float(x); }

}  // namespace gd
