// Internal structures shared by the host runtime and the gfx950 kernels of the
// scattered-field PIC library.  Not part of the public ABI (include/sfpic.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sfpic {

constexpr int kGuard = 3;
constexpr double kDeadPos = -1.0e30;     // FP64 position of a removed particle
constexpr uint32_t kDeadCell = 0xFFFFFFFFu;  // FP32 cell of a removed particle

// ---------------------------------------------------------------------------
// Incident-field parameters (prepared on the host, read by every particle).
// ---------------------------------------------------------------------------
struct IncParams {
  int kind;        // SFPIC_INC_*
  int s_int;       // April: integer Poisson-spectrum parameter s
  double a0;       // plane pulse amplitude
  double t0;       // plane pulse centre
  double env_k;    // plane pulse: -4 / fwhm^2 (exponent base 2)
  // April: complex-source parameter a (k = 1 units) and 1/a.  The Gaussian
  // beam keeps its waist w0 and Rayleigh range zR = w0^2/2 in the same two
  // slots, so the kernels' argument block keeps its size (one 16 bytes
  // larger cost the FP64 push 2.5%).
  union {
    double a;
    double w0;
  };
  union {
    double inv_a;
    double zr;
  };
  double inv_s;
  double a_over_s;
  double x_focus, y_focus, t_focus;
  // N e^{i phi0} Gamma(s+n+1)/Gamma(s+1) (i a / s)^n for n = 0, 1, 2, with N
  // the amplitude normalization (real, imaginary pairs).
  double cr[3], ci[3];
  double e_phase_r, e_phase_i;  // N e^{i phi0}
  // 1: the incident field is sampled on the Yee nodes (Fields::iex ...) and
  // gathered with the scattered field instead of evaluated per particle
  int on_nodes;
};

// ---------------------------------------------------------------------------
// Field planes of one simulation (device pointers, row pitch in elements).
// ---------------------------------------------------------------------------
template <typename R>
struct Fields {
  R *ex, *ey, *ez, *bx, *by, *bz;  // scattered E^n, B^{n-1/2}
  R *jx, *jy, *jz;                 // current J^{n+1/2}
  R *mx, *my, *mz;                 // centred Bbar^n
  // incident E_x, E_y, B_z at t^n on the nodes of E_x, E_y, B_z (sampled
  // mode; in the plane y_paper = 0 the models have no other components);
  // null when the incident field is evaluated at the particles
  R *iex, *iey, *ibz;
  int nx_alloc, ny_alloc;          // NX, NY including guards
  int pitch;                       // row pitch (elements)
};

// Particle storage of one species: structure of arrays.
//  FP64: positions as doubles in cell units (xi = x / dx).
//  FP32: packed cell (ix | iy << 16) plus float in-cell offsets in [0, 1).
template <typename R>
struct Particles;

template <>
struct Particles<double> {
  double *px, *py, *ux, *uy, *uz;
  uint32_t *id;
};

template <>
struct Particles<float> {
  uint32_t *cell;
  float *ox, *oy, *ux, *uy, *uz;
  uint32_t *id;
};

// Drift allowance (cells) of a single sim's tile window, per precision.
#ifndef SFPIC_SLACK_F64
#define SFPIC_SLACK_F64 3
#endif
constexpr int kSingleSlackF64 = SFPIC_SLACK_F64;
#ifndef SFPIC_SLACK_F32
#define SFPIC_SLACK_F32 1
#endif
constexpr int kSingleSlackF32 = SFPIC_SLACK_F32;

// Particle tiles: tx x ty cells (ty = 1 in 1D).  Cells are keyed tile-major:
// key = tile * cells_per_tile + (iy mod ty) * tx + (ix mod tx).
struct TileGeom {
  int tx, ty;
  int ntx, nty, ntiles;
  uint32_t cells_per_tile;
  uint32_t nkeys;  // ntiles * cells_per_tile
  // cells a particle may drift outside its tile (as of the last sort) and
  // still be pushed by the tile's workgroup; sets the LDS window size
  int slack;
};

// Scratch of the counting sort (shared by the species of one sim; each
// species keeps its own `start` array, the exclusive scan of the counts,
// which also gives its tile ranges until the next sort).
struct SortScratch {
  uint32_t *counts;      // nkeys + 1
  uint32_t *block_sums;  // ceil((nkeys + 1) / 1024)
  uint32_t *key, *rank;  // per particle slot
};

// Per-step scalars of one species push.
struct PushParams {
  double dt, dx, dy;
  double inv_dx, inv_dy;
  double qm;       // q / m
  double qw;       // q * weight
  double time;     // t^n
  int nx, ny;      // physical cells
};

// ---------------------------------------------------------------------------
// Batched execution: many independent simulations of one precision and
// dimensionality advanced by the same launches.  Every launch reads a table
// of per-member descriptors; a workgroup finds its member from a prefix table
// of block (or tile) offsets.  The step counter, the steps still to run and
// the current particle buffer live on the device, so a captured graph of a
// few steps can be replayed without host updates.
// ---------------------------------------------------------------------------
struct MemberState {
  int64_t step;        // n of the next step (t^n = n dt)
  int64_t steps_left;  // 0: finished; every kernel skips the member
  int32_t since_sort;  // steps since the last sort
  int32_t sort_due;    // the sort launches of this step sort the member
};

// A member is sorted every c_max of its own steps (members that join a
// running group count from their own start).
struct SortRule {
  int32_t c_max;
};

template <typename R>
struct FieldJob {
  Fields<R> f;
  R dt, cx, cy, kx, ky;  // dt, dt/dx, dt/dy, Mur coefficients
  int member;
  int job0, njobs;       // the member's push jobs
};

template <typename R>
struct PushJob {
  Fields<R> f;
  Particles<R> pa[2];  // pa[cur] is the current set, the other the sort target
  uint32_t *start, *n_valid, *strag;
  SortScratch ss;
  TileGeom tg;
  PushParams pp;       // pp.time is formed on the device from the step
  IncParams inc;
  uint32_t n_slots;
  int member;
  int cur;             // flipped on the device by every sort
  // work items of the push, (tile, first particle), rebuilt after each of
  // the job's sorts; at most kmax particles each
  uint32_t *items, *n_items;
  uint32_t kmax;
};

// Device view of one batch group.  Offset tables have n + 1 entries.
template <typename R>
struct BatchView {
  const FieldJob<R> *fjobs;
  PushJob<R> *pjobs;
  MemberState *ms;
  int nmembers, nf, np;
  const uint32_t *far_off, *amp_off;  // field jobs: Faraday / Ampere blocks
  const uint32_t *tile_off;           // push jobs: tiles
  // [0] tile queue, [1 + j] stragglers of push job j, [1 + np] number of
  // push jobs to sort this step (listed in due), [2 + np + x] queue of the
  // push's item band x (x = 0 .. 7)
  uint32_t *counters;
  uint32_t *due;
  // push items of every job, prefix over the jobs (np + 1 entries; the
  // jobs of finished members have none), formed at the start of each step
  uint32_t *item_off;
  uint32_t n_far, n_amp, n_tiles;
};

// ---------------------------------------------------------------------------
// Minimal complex arithmetic for device code.
// ---------------------------------------------------------------------------
template <typename T>
struct cx {
  T r, i;
};

template <typename T>
__host__ __device__ __forceinline__ cx<T> mk(T r, T i) {
  return cx<T>{r, i};
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) {
  return cx<T>{a.r + b.r, a.i + b.i};
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) {
  return cx<T>{a.r - b.r, a.i - b.i};
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return cx<T>{a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) {
  return cx<T>{s * a.r, s * a.i};
}
// Reciprocal and reciprocal square root for the particle path.  On the
// device: the hardware estimate (v_rcp / v_rsq) refined by Newton-Raphson
// steps, y <- y + y (1 - a y) and y <- y + (y/2)(1 - a y^2), each of which
// squares the relative error; two steps bring the FP64 estimate to within
// about an ulp of the rounded result, far cheaper than the IEEE division
// and square-root sequences.  FP32 uses the estimate alone (about 1 ulp).
// The host (parameter preparation) divides.
__host__ __device__ __forceinline__ double rcp(double a) {
#if defined(__HIP_DEVICE_COMPILE__)
  double y = __builtin_amdgcn_rcp(a);
  y = fma(y, fma(-a, y, 1.0), y);
  return fma(y, fma(-a, y, 1.0), y);
#else
  return 1.0 / a;
#endif
}
__host__ __device__ __forceinline__ float rcp(float a) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(a);
#else
  return 1.0f / a;
#endif
}
__host__ __device__ __forceinline__ double rsqrt(double a) {
#if defined(__HIP_DEVICE_COMPILE__)
  double y = __builtin_amdgcn_rsq(a);
  y = fma(0.5 * y, fma(-a * y, y, 1.0), y);
  return fma(0.5 * y, fma(-a * y, y, 1.0), y);
#else
  return 1.0 / sqrt(a);
#endif
}
__host__ __device__ __forceinline__ float rsqrt(float a) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rsqf(a);
#else
  return 1.0f / sqrtf(a);
#endif
}

template <typename T>
__host__ __device__ __forceinline__ cx<T> cinv(cx<T> a) {
  T d = rcp(a.r * a.r + a.i * a.i);
  return cx<T>{a.r * d, -a.i * d};
}

// Integer power by binary exponentiation (n >= 1).
template <typename T>
__host__ __device__ __forceinline__ cx<T> cpowi(cx<T> b, int n) {
  cx<T> r = b;
  n -= 1;
  cx<T> p = b;
  while (n > 0) {
    if (n & 1) r = r * p;
    n >>= 1;
    if (n) p = p * p;
  }
  return r;
}

// b1^n and b2^n (n >= 1) in one binary exponentiation: n is the same in
// every lane, and with both powers in one loop each uniform branch guards
// eight products, which the compiler keeps as a branch instead of computing
// both sides in every iteration and selecting.
template <typename T>
__host__ __device__ __forceinline__ void cpowi2(cx<T> b1, cx<T> b2, int n,
                                                cx<T> &r1, cx<T> &r2) {
  r1 = b1;
  r2 = b2;
  for (n -= 1; n > 0; n >>= 1) {
    if (n & 1) {
      r1 = r1 * b1;
      r2 = r2 * b2;
    }
    if (n > 1) {
      b1 = b1 * b1;
      b2 = b2 * b2;
    }
  }
}

// Square root with a branch that is continuous away from the negative real
// axis; the April fields are even in this root, so any branch is valid.
// With h = (|z| + |Re z|)/2 > 0 the root's larger part is sqrt(h) = h /
// sqrt(h) and the other part Im z / (2 sqrt(h)); z = 0 is excluded by the
// callers (the ring neighbourhood uses the series).
template <typename T>
__host__ __device__ __forceinline__ cx<T> csqrt_any(cx<T> z) {
  const T q = z.r * z.r + z.i * z.i;
  const T m = q * rsqrt(q);
  const T h = T(0.5) * (m + fabs(z.r));
  const T g = rsqrt(h);
  const T big = h * g, small = T(0.5) * z.i * g;
  if (z.r >= T(0)) return cx<T>{big, small};
  return cx<T>{(z.i < T(0)) ? -small : small, (z.i < T(0)) ? -big : big};
}

// ---------------------------------------------------------------------------
// April isodiffracting pulse (Sec. 4.1).  All lengths are scaled by a:
// X = x/a etc.; u^2 = X^2 + Y^2 + (Z + i)^2.  The phasor Psi = [f(t+) -
// f(t-)]/Rtilde has field components that are second derivatives of Psi; with
// d/dX = (X/u) d/du they reduce to four blocks of u and T:
//   Phi_TT = G-2/u,
//   D1     = G+1/u^2 - G-0/u^3,
//   D1_T   = G+2/u^2 - G-1/u^3,
//   D2     = (3 G-0/u^3 - 3 G+1/u^2 + G-2/u) / u^2,
// where G+-n = g^(n)(tau+) +- g^(n)(tau-), tau+- = tau + a(+-u + i) and
// g^(n)(tau) = C_n (1 - i tau/s)^{-(s+n+1)}.
// On the ring u -> 0 (r = a in the focal plane) the blocks are 0/0 but
// analytic in u^2; there a Taylor series in u^2 about u = 0 is used with
// coefficients c_m = g^(m)(tau + i a).
// ---------------------------------------------------------------------------
constexpr double kRingU2 = 0.0625;  // series when |u^2| < 0.25^2
constexpr int kRingTerms = 16;

struct AprilBlocks {
  cx<double> phitt, d1, d1t, d2;
};

// Closed-form blocks from the root u and w+- = 1 - i tau+-/s, evaluated in
// precision T (the caller forms u and w+- in FP64: tau +- a u_r is where the
// phase is decided and cancellation happens).
template <typename T>
struct Blocks {
  cx<T> phitt, d1, d1t, d2;
};

template <typename T>
__host__ __device__ inline Blocks<T> april_blocks_rest(const IncParams &P,
                                                       cx<T> u, cx<T> wp,
                                                       cx<T> wm) {
  cx<T> rp = cinv(wp), rm = cinv(wm);
  cx<T> pp0, pm0;
  cpowi2(rp, rm, P.s_int + 1, pp0, pm0);
  cx<T> pp1 = pp0 * rp, pm1 = pm0 * rm;
  cx<T> pp2 = pp1 * rp, pm2 = pm1 * rm;
  cx<T> c0 = mk((T)P.cr[0], (T)P.ci[0]), c1 = mk((T)P.cr[1], (T)P.ci[1]),
        c2 = mk((T)P.cr[2], (T)P.ci[2]);
  cx<T> Gm0 = c0 * (pp0 - pm0);
  cx<T> Gp1 = c1 * (pp1 + pm1), Gm1 = c1 * (pp1 - pm1);
  cx<T> Gp2 = c2 * (pp2 + pm2), Gm2 = c2 * (pp2 - pm2);
  cx<T> iu = cinv(u);
  cx<T> iu2 = iu * iu, iu3 = iu2 * iu;
  Blocks<T> b;
  b.phitt = Gm2 * iu;
  b.d1 = Gp1 * iu2 - Gm0 * iu3;
  b.d1t = Gp2 * iu2 - Gm1 * iu3;
  b.d2 = (T(3) * (Gm0 * iu3) - T(3) * (Gp1 * iu2) + Gm2 * iu) * iu2;
  return b;
}

// FP64 phase part: root u of u^2 and w+- = (1 + a/s +- a u_i/s) - i (tau +-
// a u_r)/s.
__host__ __device__ inline void april_phase(const IncParams &P, cx<double> u2,
                                            double tau, cx<double> &u,
                                            cx<double> &wp, cx<double> &wm) {
  u = csqrt_any(u2);
  const double as = P.a_over_s;
  wp = mk(1.0 + as + as * u.i, -(tau + P.a * u.r) * P.inv_s);
  wm = mk(1.0 + as - as * u.i, -(tau - P.a * u.r) * P.inv_s);
}

__host__ __device__ inline AprilBlocks april_blocks_closed(const IncParams &P,
                                                            cx<double> u2,
                                                            double tau) {
  cx<double> u, wp, wm;
  april_phase(P, u2, tau, u, wp, wm);
  Blocks<double> b = april_blocks_rest<double>(P, u, wp, wm);
  AprilBlocks r;
  r.phitt = b.phitt;
  r.d1 = b.d1;
  r.d1t = b.d1t;
  r.d2 = b.d2;
  return r;
}

// Rare branch (particles near the ring): kept out of line so its registers do
// not add to those of the common closed-form path.  It takes the few
// parameters it reads by value: a reference to IncParams across a real call
// would make the kernels keep the whole block in per-lane scratch memory and
// read every incident parameter from there.
static __host__ __device__ __attribute__((noinline)) AprilBlocks
april_blocks_series(double a_over_s, double inv_s, int s_int,
                    cx<double> e_phase, cx<double> u2, double tau) {
  // c_m = N e^{i phi0} [prod_{k<=m} (s+k)] (i a/s)^m (1 + a/s - i tau/s)^{-(s+m+1)}
  // generated in order: c_{m} = (s + m) (i a/s) base c_{m-1}.
  cx<double> base = cinv(mk(1.0 + a_over_s, -tau * inv_s));
  const double s = (double)s_int;
  const cx<double> step_b = mk(0.0, a_over_s) * base;
  cx<double> c = e_phase * cpowi(base, s_int + 1);
  c = (s + 1.0) * (c * step_b);  // c_1
  cx<double> phitt = mk(0.0, 0.0), d1 = phitt, d1t = phitt, d2 = phitt;
  cx<double> pw = mk(1.0, 0.0), pw1 = mk(0.0, 0.0), pw2 = mk(0.0, 0.0);
  double inv_fact = 1.0;  // 1/(2j+1)!
#pragma unroll 1
  for (int j = 0; j < kRingTerms; ++j) {
    if (j > 0) inv_fact /= (2.0 * j) * (2.0 * j + 1.0);
    const cx<double> c1 = c;                                      // c_{2j+1}
    const cx<double> c2 = (s + 2.0 * j + 2.0) * (c1 * step_b);    // c_{2j+2}
    const cx<double> c3 = (s + 2.0 * j + 3.0) * (c2 * step_b);    // c_{2j+3}
    // pw = u^{2j}, pw1 = u^{2j-2}, pw2 = u^{2j-4}
    phitt = phitt + (2.0 * inv_fact) * (pw * c3);
    if (j >= 1) {
      d1 = d1 + (4.0 * j * inv_fact) * (pw1 * c1);
      d1t = d1t + (4.0 * j * inv_fact) * (pw1 * c2);
    }
    if (j >= 2) d2 = d2 + (4.0 * j * (2.0 * j - 2.0) * inv_fact) * (pw2 * c1);
    pw2 = pw1;
    pw1 = pw;
    pw = pw * u2;
    c = c3;
  }
  AprilBlocks b;
  b.phitt = phitt;
  b.d1 = d1;
  b.d1t = d1t;
  b.d2 = d2;
  return b;
}

// Complex fields in the paper's axes at dimensionless (X, Y, Z) and tau, with
// the normalization N folded in.  e[0..2] = E_x, E_y, E_z; b[0..2] = cB.
// KIND: 2 (LP) or 3 (RP) fixed at compile time, 0 read from P.kind.
template <int KIND = 0>
__host__ __device__ inline void april_complex_fields(const IncParams &P,
                                                     double X, double Y,
                                                     double Z, double tau,
                                                     cx<double> e[3],
                                                     cx<double> b[3]) {
  cx<double> u2 = mk(X * X + Y * Y + Z * Z - 1.0, 2.0 * Z);
  double m2 = u2.r * u2.r + u2.i * u2.i;
  AprilBlocks k = (m2 < kRingU2 * kRingU2)
                      ? april_blocks_series(P.a_over_s, P.inv_s, P.s_int,
                                            mk(P.e_phase_r, P.e_phase_i), u2,
                                            tau)
                      : april_blocks_closed(P, u2, tau);
  cx<double> zp = mk(Z, 1.0);
  if ((KIND ? KIND : P.kind) == 2) {  // LP
    cx<double> common = k.d1 - k.phitt + zp * k.d1t;
    e[0] = (X * X) * k.d2 + common;
    e[1] = (X * Y) * k.d2;
    e[2] = X * (zp * k.d2) - X * k.d1t;
    b[0] = e[1];
    b[1] = (Y * Y) * k.d2 + common;
    b[2] = Y * (zp * k.d2) - Y * k.d1t;
  } else {  // RP: Hertz vector along the propagation axis
    cx<double> zd2 = zp * k.d2;
    e[0] = X * zd2;
    e[1] = Y * zd2;
    e[2] = k.d1 + zp * zd2 - k.phitt;
    b[0] = Y * k.d1t;
    b[1] = -X * k.d1t;
    b[2] = mk(0.0, 0.0);
  }
}

// Sec. 3.2 paraxial Gaussian beam, focus at (x_focus, y_focus): with z along
// the axis and r across it, w = w0 sqrt(1 + (z/zR)^2), 1/R = z / (z^2 +
// zR^2), eta = atan(z/zR) / 2, psi = z - t + r^2/(2R) - eta,
// E_y = B_z = E0 sqrt(w0/w) e^{-r^2/w^2} cos(psi) env and the first-order
// longitudinal E_x = 2 (r / w^2) E0 sqrt(w0/w) e^{-r^2/w^2} sin(psi) env.
struct Gauss2 {
  double ex, ey;
};
__host__ __device__ __forceinline__ Gauss2
gauss2d_field(const IncParams &P, int dims, double x, double y, double t) {
  const double z = x - P.x_focus;
  const double r = dims == 2 ? y - P.y_focus : 0.0;
  const double zz = z / P.zr;
  const double w = P.w0 * sqrt(1.0 + zz * zz);
  const double inv_r = z / (z * z + P.zr * P.zr);
  const double psi = z - t + 0.5 * r * r * inv_r - 0.5 * atan(zz);
  const double ph = t - P.t0 - z;
  const double amp = P.a0 * sqrt(P.w0 / w) * exp(-r * r / (w * w)) *
                     exp2(P.env_k * ph * ph);
  Gauss2 g;
  g.ey = amp * cos(psi);
  g.ex = 2.0 * r / (w * w) * amp * sin(psi);
  return g;
}

// Real incident field in build axes (propagation +x, LP polarization y) at
// (x, y, z = 0) and time t.  kGauss = false compiles the plane pulse and the
// April beams only: the push kernels of those models are built without the
// Gaussian beam's code, which would otherwise cost them registers.
//
// KIND fixes the model at compile time (1 plane pulse, 2 April LP, 3 April
// RP; 0: the model P.kind names): a push compiled for one model carries
// neither the other models' code nor their parameters.
template <bool kGauss, int KIND = 0>
__host__ __device__ inline void incident_field_t(const IncParams &P, int dims,
                                                 double x, double y, double t,
                                                 double E[3], double B[3]) {
  E[0] = E[1] = E[2] = 0.0;
  B[0] = B[1] = B[2] = 0.0;
  const int kind = KIND ? KIND : P.kind;
  if (kind == 1) {
    double ph = t - P.t0 - x;
    double v = P.a0 * sin(ph) * exp2(P.env_k * ph * ph);
    E[1] = v;
    B[2] = v;
  } else if (kGauss && kind == 4) {
    const Gauss2 g = gauss2d_field(P, dims, x, y, t);
    E[0] = g.ex;
    E[1] = g.ey;
    B[2] = g.ey;
  } else if (kind == 2 || kind == 3) {
    double X = (dims == 2 ? (y - P.y_focus) : 0.0) * P.inv_a;  // paper x
    double Z = (x - P.x_focus) * P.inv_a;                       // paper z
    cx<double> e[3], b[3];
    april_complex_fields<KIND>(P, X, 0.0, Z, t - P.t_focus, e, b);
    E[0] = e[2].r;  // build x = paper z
    E[1] = e[0].r;  // build y = paper x
    E[2] = e[1].r;  // build z = paper y
    B[0] = b[2].r;
    B[1] = b[0].r;
    B[2] = b[1].r;
  }
}

// Every model.
__host__ __device__ inline void incident_field(const IncParams &P, int dims,
                                               double x, double y, double t,
                                               double E[3], double B[3]) {
  incident_field_t<true>(P, dims, x, y, t, E, B);
}

// Incident field for the FP32 form: the phase (positions, time, u, tau +-
// a u_r, the plane pulse's carrier phase after range reduction) and the ring
// neighbourhood in FP64, the powers, blocks and fields in FP32.
template <bool kGauss, int KIND = 0>
__device__ inline void incident_field_fp32(const IncParams &P, int dims,
                                           double x, double y, double t,
                                           float E[3], float B[3]) {
  E[0] = E[1] = E[2] = 0.0f;
  B[0] = B[1] = B[2] = 0.0f;
  const int kind = KIND ? KIND : P.kind;
  if (kind == 1) {
    const double ph = t - P.t0 - x;
    const double two_pi = 6.283185307179586;
    const double r = ph - two_pi * rint(ph * (1.0 / two_pi));  // |r| <= pi
    const float v = (float)P.a0 * sinf((float)r) *
                    exp2f((float)(P.env_k * ph * ph));
    E[1] = v;
    B[2] = v;
    return;
  }
  if (kGauss && kind == 4) {  // the FP64 closed form, rounded
    const Gauss2 g = gauss2d_field(P, dims, x, y, t);
    E[0] = (float)g.ex;
    E[1] = (float)g.ey;
    B[2] = (float)g.ey;
    return;
  }
  if (kind != 2 && kind != 3) return;
  const double X = (dims == 2 ? (y - P.y_focus) : 0.0) * P.inv_a;
  const double Z = (x - P.x_focus) * P.inv_a;
  const double tau = t - P.t_focus;
  const cx<double> u2 = mk(X * X + Z * Z - 1.0, 2.0 * Z);
  if (u2.r * u2.r + u2.i * u2.i < kRingU2 * kRingU2) {
    double Ed[3], Bd[3];
    incident_field_t<false, KIND>(P, dims, x, y, t, Ed, Bd);
    for (int c = 0; c < 3; ++c) {
      E[c] = (float)Ed[c];
      B[c] = (float)Bd[c];
    }
    return;
  }
  cx<double> u, wp, wm;
  april_phase(P, u2, tau, u, wp, wm);
  const Blocks<float> k = april_blocks_rest<float>(
      P, mk((float)u.r, (float)u.i), mk((float)wp.r, (float)wp.i),
      mk((float)wm.r, (float)wm.i));
  const float Xf = (float)X;
  const cx<float> zp = mk((float)Z, 1.0f);
  if (kind == 2) {  // LP, paper y = 0: E_x, E_z, cB_y
    const cx<float> common = k.d1 - k.phitt + zp * k.d1t;
    const cx<float> ex = (Xf * Xf) * k.d2 + common;
    const cx<float> ez = Xf * (zp * k.d2) - Xf * k.d1t;
    E[0] = ez.r;      // build x = paper z
    E[1] = ex.r;      // build y = paper x
    B[2] = common.r;  // build z = paper y (cB_y = common when Y = 0)
  } else {  // RP, paper y = 0: E_x, E_z, cB_y
    const cx<float> zd2 = zp * k.d2;
    const cx<float> ex = Xf * zd2;
    const cx<float> ez = k.d1 + zp * zd2 - k.phitt;
    const cx<float> by = -Xf * k.d1t;
    E[0] = ez.r;
    E[1] = ex.r;
    B[2] = by.r;
  }
}

// ---------------------------------------------------------------------------
// Kernel launchers (sfpic_kernels.hip)
// ---------------------------------------------------------------------------
template <typename R>
hipError_t launch_faraday(const Fields<R> &f, int dims, double dt, double dx,
                          double dy, hipStream_t st);
template <typename R>
hipError_t launch_ampere(const Fields<R> &f, int dims, double dt, double dx,
                         double dy, hipStream_t st);
// LDS of the push workgroup: all of it (static and dynamic), and the dynamic
// part passed at launch; batch: the batched push's; field_window: whether
// the push stages its field window (the FP32 form's single push with the
// incident field at the particles gathers from global memory instead).
template <typename R>
size_t push_lds_bytes(const TileGeom &tg, int dims, bool batch = false);
template <typename R>
size_t push_dyn_lds_bytes(const TileGeom &tg, int dims, bool batch = false,
                          bool field_window = true);
// Work items of the tiled push (tile, first particle), at most kmax
// particles each, rebuilt from the sort's start offsets after every sort;
// items holds push_items_words() words.
hipError_t launch_build_items(const uint32_t *start, const TileGeom &tg,
                              uint32_t kmax, uint32_t *items,
                              uint32_t *n_items, hipStream_t st);
size_t push_items_words(const TileGeom &tg, int64_t n_slots, uint32_t kmax);
// Tiled push over the work items; particles that drifted out of their tile
// window are appended to strag (count in *n_strag, reset by the launcher)
// for the straggler push.
template <typename R>
hipError_t launch_push_tiled(const Fields<R> &f, const Particles<R> &p,
                             const uint32_t *start, const uint32_t *items,
                             const uint32_t *n_items, uint32_t kmax,
                             int64_t n_slots, const TileGeom &tg, int dims,
                             const PushParams &pp, const IncParams &inc,
                             uint32_t *strag, uint32_t *n_strag,
                             hipStream_t st);
template <typename R>
hipError_t launch_push_stragglers(const Fields<R> &f, const Particles<R> &p,
                                  int dims, const PushParams &pp,
                                  const IncParams &inc, const uint32_t *strag,
                                  const uint32_t *n_strag, hipStream_t st);
// Sort src into dst by cell key; n_valid (device) holds the number of used
// slots of src on entry and of dst on exit.
template <typename R>
hipError_t launch_sort(const Particles<R> &src, const Particles<R> &dst,
                       uint32_t n_slots, uint32_t *n_valid, uint32_t *start,
                       const TileGeom &tg, int nx, int ny, int dims,
                       const SortScratch &s, hipStream_t st);
template <typename R>
hipError_t launch_init_particles(const Particles<R> &p, int64_t n, int dims,
                                 int64_t x0, int64_t ncx, int64_t y0,
                                 int ppc, double sigma, uint64_t seed,
                                 uint32_t key1, double dx, double dy,
                                 hipStream_t st);
template <typename R>
hipError_t launch_load_particles(const Particles<R> &p, int64_t n, int dims,
                                 const double *x, const double *y,
                                 const double *ux, const double *uy,
                                 const double *uz, double inv_dx,
                                 double inv_dy, int nx, int ny,
                                 hipStream_t st);
// Used slots as FP64: out holds 5 arrays of n (x, y, ux, uy, uz; removed
// particles have x = -1), ids the particle ids.
template <typename R>
hipError_t launch_export_particles(const Particles<R> &p, int64_t n, int dims,
                                   double dx, double dy, double *out,
                                   uint32_t *ids, hipStream_t st);

// FP64 diagnostics: particle sums {w_kin, charge, n_alive, nonfinite}.
template <typename R>
hipError_t launch_particle_sums(const Particles<R> &p, int64_t n,
                                const uint32_t *n_valid, int dims, double m,
                                double q, double wdv, double *acc,
                                hipStream_t st);
template <typename R>
hipError_t launch_field_sums(const Fields<R> &f, double *acc, hipStream_t st);
// Incident field sampled on the Yee nodes at time t into f.iex, f.iey, f.ibz.
template <typename R>
hipError_t launch_incident_nodes(const Fields<R> &f, int dims, double dx,
                                 double dy, double t, const IncParams &inc,
                                 hipStream_t st);
// acc[7] += 1/2 sum over physical nodes of |F_scatt + F_inc|^2 (E at tE, B
// at tB), each component at its Yee node.
template <typename R>
hipError_t launch_em_total(const Fields<R> &f, int dims, int nx, int ny,
                           double dx, double dy, double tE, double tB,
                           const IncParams &inc, double *acc, hipStream_t st);
template <typename R>
hipError_t launch_deposit_rho(const Particles<R> &p, int64_t n,
                              const uint32_t *n_valid, int dims, double qw,
                              double *rho, int pitch, hipStream_t st);
template <typename R>
hipError_t launch_gauss(const Fields<R> &f, int dims, int nx, int ny,
                        double dx, double dy, const double *rho,
                        const double *rho0, int rpitch, double *gprev,
                        int have_prev, double *acc, hipStream_t st);
template <typename R>
hipError_t launch_histogram(const Particles<R> &p, int64_t n,
                            const uint32_t *n_valid, int dims, double m,
                            double wdv, int n_e, double emax, int n_t,
                            double ek_min, int plane, double *hist,
                            double *mom, hipStream_t st);

// Batched launches (one per phase for the whole group).  `grid` of the push
// is the number of persistent workgroups pulling tiles from the queue.
template <typename R>
hipError_t launch_batch_faraday(const BatchView<R> &v, int dims,
                                hipStream_t st);
template <typename R>
hipError_t launch_batch_ampere(const BatchView<R> &v, int dims,
                               hipStream_t st);
// The incident field sampled on the nodes of the members that take it from
// there, at each member's own time.
template <typename R>
hipError_t launch_batch_incident_nodes(const BatchView<R> &v, int dims,
                                       hipStream_t st);
// april: every push job has an April beam at the particles (see
// batch_push_kernel)
template <typename R>
hipError_t launch_batch_push(const BatchView<R> &v, int dims, bool april,
                             size_t lds, int grid, hipStream_t st);
template <typename R>
hipError_t launch_batch_stragglers(const BatchView<R> &v, int dims,
                                   hipStream_t st);
template <typename R>
hipError_t launch_batch_sort(const BatchView<R> &v, int dims, hipStream_t st);
// The push items of every job of the step (item_off), from the jobs' item
// counts and their members' steps left.
template <typename R>
hipError_t launch_batch_item_offsets(const BatchView<R> &v, hipStream_t st);
template <typename R>
hipError_t launch_batch_advance(const BatchView<R> &v, SortRule rule,
                                hipStream_t st);
// Resident workgroups of the batched push per CU (0 on error).
int batch_push_blocks_per_cu(bool fp64, int dims, bool april, size_t lds);
hipError_t launch_fill_u32(uint32_t *a, uint32_t v, size_t n, hipStream_t st);

}  // namespace sfpic
