// Device helpers shared by the particle kernels: order-2 shapes, gather,
// Boris rotation, Philox4x32-10.
#pragma once

#include <type_traits>

#include "sfpic_common.h"

namespace sfpic {

// Segment of a prefix table: the largest j in [0, n) with off[j] <= x, for
// 0 <= x < off[n].  Empty segments (off[j] == off[j + 1]) are never returned.
// Called with wave-uniform arguments, so the loads are scalar.
__device__ __forceinline__ int find_segment(const uint32_t *off, int n,
                                            uint32_t x) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= x)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// Particles: order-2 shapes
// ---------------------------------------------------------------------------

// Three quadratic B-spline weights for offset d in [-1/2, 1/2] from the
// nearest node (nodes -1, 0, +1).
template <typename R>
__device__ __forceinline__ void weights3(R d, R w[3]) {
  const R a = R(0.5) - d, b = R(0.5) + d;
  w[0] = R(0.5) * a * a;
  w[1] = R(0.75) - d * d;
  w[2] = R(0.5) * b * b;
}

// Quadratic B-spline at distance d (cell units).
template <typename R>
__device__ __forceinline__ R spline2(R d) {
  const R a = fabs(d);
  const R b = R(1.5) - a;
  return a <= R(0.5) ? R(0.75) - a * a : (a <= R(1.5) ? R(0.5) * b * b : R(0));
}

// Weighted 3-tap (1D) or 3x3-tap (2D) gather from one field plane; (bx, by)
// is the array index of the first tap.
template <typename R, int DIMS>
__device__ __forceinline__ R gather_plane(const R *__restrict__ a, int P,
                                          int bx, int by, const R wx[3],
                                          const R wy[3]) {
  if (DIMS == 1) return wx[0] * a[bx] + wx[1] * a[bx + 1] + wx[2] * a[bx + 2];
  R v = R(0);
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const R *row = a + (size_t)(by + b) * P + bx;
    v += wy[b] * (wx[0] * row[0] + wx[1] * row[1] + wx[2] * row[2]);
  }
  return v;
}

// gather_plane of two interleaved planes (pairs a[2n], a[2n + 1] at node n)
// that share their taps: s0 from the first member, s1 from the second.
template <typename R, int DIMS>
__device__ __forceinline__ void gather_pair(const R *__restrict__ a, int P,
                                            int bx, int by, const R wx[3],
                                            const R wy[3], R &s0, R &s1) {
  using V = typename std::conditional<sizeof(R) == 4, float2, double2>::type;
  const V *p = (const V *)a;
  if (DIMS == 1) {
    const V t0 = p[bx], t1 = p[bx + 1], t2 = p[bx + 2];
    s0 = wx[0] * t0.x + wx[1] * t1.x + wx[2] * t2.x;
    s1 = wx[0] * t0.y + wx[1] * t1.y + wx[2] * t2.y;
    return;
  }
  R v0 = R(0), v1 = R(0);
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const V *row = p + (size_t)(by + b) * P + bx;
    const V t0 = row[0], t1 = row[1], t2 = row[2];
    v0 += wy[b] * (wx[0] * t0.x + wx[1] * t1.x + wx[2] * t2.x);
    v1 += wy[b] * (wx[0] * t0.y + wx[1] * t1.y + wx[2] * t2.y);
  }
  s0 = v0;
  s1 = v1;
}

// Boris rotation (Boris 1970) of u = gamma v for charge-to-mass ratio qm.
template <typename R>
__device__ __forceinline__ void boris(R qm, R dt, R u[3], const R E[3],
                                      const R B[3]) {
  const R h = R(0.5) * qm * dt;
  const R um0 = u[0] + h * E[0], um1 = u[1] + h * E[1], um2 = u[2] + h * E[2];
  const R gi = rsqrt(R(1) + um0 * um0 + um1 * um1 + um2 * um2);
  const R t0 = h * B[0] * gi, t1 = h * B[1] * gi, t2 = h * B[2] * gi;
  const R f = R(2) * rcp(R(1) + t0 * t0 + t1 * t1 + t2 * t2);
  const R s0 = f * t0, s1 = f * t1, s2 = f * t2;
  const R up0 = um0 + (um1 * t2 - um2 * t1);
  const R up1 = um1 + (um2 * t0 - um0 * t2);
  const R up2 = um2 + (um0 * t1 - um1 * t0);
  u[0] = um0 + (up1 * s2 - up2 * s1) + h * E[0];
  u[1] = um1 + (up2 * s0 - up0 * s2) + h * E[1];
  u[2] = um2 + (up0 * s1 - up1 * s0) + h * E[2];
}

// Philox4x32-10 (Salmon et al., SC'11) keyed by (seed, species index),
// counter (id low, id high, stream, 0).
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0,
                                              uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t h0 = (uint32_t)(p0 >> 32), l0 = (uint32_t)p0;
    const uint32_t h1 = (uint32_t)(p1 >> 32), l1 = (uint32_t)p1;
    const uint32_t n0 = h1 ^ c[1] ^ k0, n2 = h0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = l1;
    c[2] = n2;
    c[3] = l0;
  }
}

__device__ __forceinline__ void u01_pair(const uint32_t r[4], double &a,
                                         double &b) {
  const double sc = 1.0 / 9007199254740992.0;
  a = ((double)(r[0] >> 5) * 67108864.0 + (double)(r[1] >> 6)) * sc;
  b = ((double)(r[2] >> 5) * 67108864.0 + (double)(r[3] >> 6)) * sc;
}


// Position of particle slot i in cell units (double); false if removed.
__device__ __forceinline__ bool pos_of(const Particles<double> &p, int64_t i,
                                       int dims, double &xi, double &yi) {
  xi = p.px[i];
  yi = dims == 2 ? p.py[i] : 0.0;
  return xi >= -1.0;
}
__device__ __forceinline__ bool pos_of(const Particles<float> &p, int64_t i,
                                       int dims, double &xi, double &yi) {
  const uint32_t c = p.cell[i];
  if (c == kDeadCell) return false;
  xi = (double)(c & 0xFFFFu) + (double)p.ox[i];
  yi = dims == 2 ? (double)(c >> 16) + (double)p.oy[i] : 0.0;
  return true;
}

// Store a placed particle given its cell-unit position (offsets kept < 1).
__device__ __forceinline__ void place(const Particles<double> &p, int64_t i,
                                      int dims, int64_t cx, double fx,
                                      int64_t cy, double fy, double ux,
                                      double uy, double uz) {
  p.px[i] = (double)cx + fx;
  if (dims == 2) p.py[i] = (double)cy + fy;
  p.ux[i] = ux;
  p.uy[i] = uy;
  p.uz[i] = uz;
}
__device__ __forceinline__ void place(const Particles<float> &p, int64_t i,
                                      int dims, int64_t cx, double fx,
                                      int64_t cy, double fy, double ux,
                                      double uy, double uz) {
  float ox = (float)fx, oy = (float)fy;
  if (!(ox < 1.0f)) ox = 0.99999994f;
  if (!(oy < 1.0f)) oy = 0.99999994f;
  p.cell[i] = (uint32_t)cx | ((uint32_t)(dims == 2 ? cy : 0) << 16);
  p.ox[i] = ox;
  if (dims == 2) p.oy[i] = oy;
  p.ux[i] = (float)ux;
  p.uy[i] = (float)uy;
  p.uz[i] = (float)uz;
}

}  // namespace sfpic
