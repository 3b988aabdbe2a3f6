// Device self-check kernels: run the production bound and triangle-triangle
// routines on caller-supplied inputs so tests can compare them with the CPU
// oracle element by element.
#include "internal.hpp"

namespace gd {

__global__ void k_eval_bounds(uint32_t n, const float* __restrict__ a, const float* __restrict__ b,
                              float* __restrict__ out) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  Box ba = load_box(a, i), bb = load_box(b, i);
  float lo, up, upm, lom;
  bounds_min(ba, bb, true, lo, up);
  bounds_max(ba, bb, true, upm, lom);
  out[4 * i + 0] = lo;
  out[4 * i + 1] = up;
  out[4 * i + 2] = upm;
  out[4 * i + 3] = lom;
}

__global__ void k_eval_tri_tri(uint32_t n, const float* __restrict__ p, const float* __restrict__ q, uint32_t mode,
                               float* __restrict__ o32, double* __restrict__ o64) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  V3<float> P[3], Q[3];
  V3<double> Pd[3], Qd[3];
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    P[v] = mk<float>(p[9ull * i + 3 * v], p[9ull * i + 3 * v + 1], p[9ull * i + 3 * v + 2]);
    Q[v] = mk<float>(q[9ull * i + 3 * v], q[9ull * i + 3 * v + 1], q[9ull * i + 3 * v + 2]);
    Pd[v] = mk<double>(P[v].x, P[v].y, P[v].z);
    Qd[v] = mk<double>(Q[v].x, Q[v].y, Q[v].z);
  }
  if (mode == 0) {
    o32[i] = sqrt32(tri_tri_min_d2<float, false>(P, Q, nullptr, nullptr));
    o64[i] = sqrt(tri_tri_min_d2<double, false>(Pd, Qd, nullptr, nullptr));
  } else {
    o32[i] = sqrt32(tri_tri_max_d2<float, false>(P, Q, nullptr, nullptr));
    o64[i] = sqrt(tri_tri_max_d2<double, false>(Pd, Qd, nullptr, nullptr));
  }
}

hipError_t launch_eval_bounds(uint32_t n, const float* a, const float* b, float* out, hipStream_t s) {
  // boxes are addressed as nodes 0..n-1 of a 6-float array
  k_eval_bounds<<<(n + 255) / 256, 256, 0, s>>>(n, a, b, out);
  return hipGetLastError();
}

hipError_t launch_eval_tri_tri(uint32_t n, const float* p, const float* q, uint32_t mode, float* o32, double* o64,
                               hipStream_t s) {
  k_eval_tri_tri<<<(n + 255) / 256, 256, 0, s>>>(n, p, q, mode, o32, o64);
  return hipGetLastError();
}

}  // namespace gd
