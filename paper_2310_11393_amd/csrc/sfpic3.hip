// 3D3V scattered-field PIC step (the method of Sec. 2 in three dimensions,
// as the runs of Sec. 4 use it): Yee update of the scattered E and B with all
// six components, order-2 gather of E^n and the centred B at the particle,
// the full six-component April LP / RP field (Sec. 4.1) or the plane pulse
// (Sec. 3.1) added at the particle, Boris, the 3D Esirkepov current, removal
// at the box faces and first-order Mur on tangential E.
//
// Layout: one FP64 array per component, [k][j][i] with i fastest, row pitch
// P (a multiple of 64 elements) >= NX = nx + 2G, NY = ny + 2G rows per
// slab, NZ = nz + 2G slabs; index I holds the primal node (I - G) h or the
// dual node (I - G + 1/2) h.  Staggering Ex(i+1/2,j,k) Ey(i,j+1/2,k)
// Ez(i,j,k+1/2) Bx(i,j+1/2,k+1/2) By(i+1/2,j,k+1/2) Bz(i+1/2,j+1/2,k), J with
// E.  Particles: positions in cell units (x / dx ...), FP64 momenta, a
// removed particle has x < -1.
//
// Every step sorts the particles by 8 x 4 x 4-cell tile (SFPIC3_TILE; a
// counting sort with creation ids carried along) and pushes each tile with
// one workgroup: the tile's E and centred B halo (T + 3 nodes per axis) is
// staged in LDS for the 27-tap gathers, and the tile's current accumulates
// in an FP64 LDS window (T + 5 nodes per axis) that is added to the global J
// once, with one atomic per window node.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/sfpic.h"
#include "sfpic_common.h"
#include "sfpic_device.h"

namespace sfpic {
int fail(int code, const std::string &msg);
// the calling entry point's handle, for sfpic_last_error(handle)
struct ErrScope {
  explicit ErrScope(const void *handle);
  ~ErrScope();
  ErrScope(const ErrScope &) = delete;
  ErrScope &operator=(const ErrScope &) = delete;
};
void forget_handle(const void *handle);
int prepare_incident_ext(const sfpic_incident *in, IncParams &P);
int profile_offsets(int32_t profile, double center, double fwhm, double order,
                    double xmin, int64_t x0, int64_t x1, double dx, int ppc,
                    std::vector<uint32_t> &off);
}  // namespace sfpic

namespace sfpic3 {
using sfpic::IncParams;

constexpr int G = SFPIC_GUARD;
// slots per species: ids, ranks and tile offsets are 32-bit
constexpr int64_t kMaxParticles = ((int64_t)1 << 31) - 1;
constexpr double kDead = -2.0;  // position marker of a removed particle

struct Geo {
  int NX, NY, NZ, P;  // array extents and row pitch
  int nx, ny, nz;     // physical cells
  __host__ __device__ size_t at(int i, int j, int k) const {
    return ((size_t)k * NY + j) * P + i;
  }
};

// Fields and momenta are stored as R (double, or float in the FP32 storage
// form); positions are always FP64 cell units and all arithmetic is FP64.
template <typename R>
struct F3 {
  R *e[3], *b[3], *j[3], *bb[3];  // E^n, B^{n-1/2}, J, centred B
};

template <typename R>
struct Parts3 {
  double *x[3];
  R *u[3];
};

template <typename R>
__device__ __forceinline__ double ld(const R *a, size_t i) {
  return (double)a[i];
}

// ---------------------------------------------------------------------------
// Yee solver
// ---------------------------------------------------------------------------

// B^{n+1/2} = B^{n-1/2} - dt curl_h E^n (forward differences), the centred
// B = (B^{n-1/2} + B^{n+1/2}) / 2, and J = 0 ahead of the deposit.  A
// component whose stencil would leave the array keeps its value.
template <typename R>
__global__ void __launch_bounds__(256)
faraday3(F3<R> f, Geo g, double cx, double cy, double cz) {
  const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y * 4 + threadIdx.y,
            k = blockIdx.z;
  if (i >= g.NX || j >= g.NY) return;
  const size_t n = g.at(i, j, k), sj = g.P, sk = (size_t)g.P * g.NY;
  const bool ix = i + 1 < g.NX, jy = j + 1 < g.NY, kz = k + 1 < g.NZ;
  double o = ld(f.b[0], n), v = o;
  if (jy && kz)
    v = o - (cy * (ld(f.e[2], n + sj) - ld(f.e[2], n)) -
             cz * (ld(f.e[1], n + sk) - ld(f.e[1], n)));
  f.b[0][n] = (R)v;
  f.bb[0][n] = (R)(0.5 * (o + v));
  o = ld(f.b[1], n);
  v = o;
  if (ix && kz)
    v = o - (cz * (ld(f.e[0], n + sk) - ld(f.e[0], n)) -
             cx * (ld(f.e[2], n + 1) - ld(f.e[2], n)));
  f.b[1][n] = (R)v;
  f.bb[1][n] = (R)(0.5 * (o + v));
  o = ld(f.b[2], n);
  v = o;
  if (ix && jy)
    v = o - (cx * (ld(f.e[1], n + 1) - ld(f.e[1], n)) -
             cy * (ld(f.e[0], n + sj) - ld(f.e[0], n)));
  f.b[2][n] = (R)v;
  f.bb[2][n] = (R)(0.5 * (o + v));
  f.j[0][n] = (R)0;
  f.j[1][n] = (R)0;
  f.j[2][n] = (R)0;
}

// E^{n+1} = E^n + dt (curl_h B^{n+1/2} - J^{n+1/2}) (backward differences) on
// the nodes that have both neighbours; the outer faces are left to Mur.
template <typename R>
__global__ void __launch_bounds__(256)
ampere3(F3<R> f, Geo g, double dt, double cx, double cy, double cz) {
  const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y * 4 + threadIdx.y,
            k = blockIdx.z;
  if (i >= g.NX || j >= g.NY) return;
  const size_t n = g.at(i, j, k), sj = g.P, sk = (size_t)g.P * g.NY;
  const bool xin = i >= 1 && i + 1 < g.NX, yin = j >= 1 && j + 1 < g.NY,
             zin = k >= 1 && k + 1 < g.NZ;
  const bool xlo = i + 1 < g.NX, ylo = j + 1 < g.NY, zlo = k + 1 < g.NZ;
  if (xlo && yin && zin)
    f.e[0][n] = (R)(ld(f.e[0], n) + cy * (ld(f.b[2], n) - ld(f.b[2], n - sj)) -
                    cz * (ld(f.b[1], n) - ld(f.b[1], n - sk)) -
                    dt * ld(f.j[0], n));
  if (xin && ylo && zin)
    f.e[1][n] = (R)(ld(f.e[1], n) + cz * (ld(f.b[0], n) - ld(f.b[0], n - sk)) -
                    cx * (ld(f.b[2], n) - ld(f.b[2], n - 1)) -
                    dt * ld(f.j[1], n));
  if (xin && yin && zlo)
    f.e[2][n] = (R)(ld(f.e[2], n) + cx * (ld(f.b[1], n) - ld(f.b[1], n - 1)) -
                    cy * (ld(f.b[0], n) - ld(f.b[0], n - sj)) -
                    dt * ld(f.j[2], n));
}

// Faces normal to axis A hold the tangential components T0 = (A+1)%3 and
// T1 = (A+2)%3.  The face buffer keeps E^n on the layers 0, 1, N-2, N-1
// along A for both: [layer][comp][f][e] over the full cross-section.
__host__ __device__ inline void face_axes(int A, int &e, int &fa) {
  e = (A + 1) % 3;
  fa = (A + 2) % 3;
}
__host__ __device__ inline int ext(const Geo &g, int a) {
  return a == 0 ? g.NX : (a == 1 ? g.NY : g.NZ);
}

template <int A, typename R>
__global__ void __launch_bounds__(256) save_faces3(F3<R> f, Geo g, double *buf) {
  int e, fa;
  face_axes(A, e, fa);
  const int ne = ext(g, e), nf = ext(g, fa), na = ext(g, A);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)ne * nf) return;
  const int ie = (int)(t % ne), jf = (int)(t / ne);
  const int layers[4] = {0, 1, na - 2, na - 1};
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    int idx[3];
    idx[A] = layers[l];
    idx[e] = ie;
    idx[fa] = jf;
    const size_t n = g.at(idx[0], idx[1], idx[2]);
    buf[((size_t)(l * 2 + 0) * nf + jf) * ne + ie] = ld(f.e[e], n);
    buf[((size_t)(l * 2 + 1) * nf + jf) * ne + ie] = ld(f.e[fa], n);
  }
}

// First-order Mur on the two faces normal to A: E_b^{n+1} = E_in^n +
// k (E_in^{n+1} - E_b^n), over every index a component occupies (the last
// index along an axis where it is dual is outside the grid).
template <int A, typename R>
__global__ void __launch_bounds__(256)
mur3(F3<R> f, Geo g, const double *buf, double kf) {
  int e, fa;
  face_axes(A, e, fa);
  const int ne = ext(g, e), nf = ext(g, fa), na = ext(g, A);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)ne * nf) return;
  const int ie = (int)(t % ne), jf = (int)(t / ne);
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int comp = c == 0 ? e : fa;  // E component index
    // component comp is dual along its own axis only
    const int dual_e = (comp == e), dual_f = (comp == fa);
    if (ie >= ne - dual_e || jf >= nf - dual_f) continue;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      int ib[3], ii[3];
      ib[A] = side ? na - 1 : 0;
      ii[A] = side ? na - 2 : 1;
      ib[e] = ii[e] = ie;
      ib[fa] = ii[fa] = jf;
      const int lb = side ? 3 : 0, li = side ? 2 : 1;
      const double in_old = buf[((size_t)(li * 2 + c) * nf + jf) * ne + ie];
      const double b_old = buf[((size_t)(lb * 2 + c) * nf + jf) * ne + ie];
      const double in_new = ld(f.e[comp], g.at(ii[0], ii[1], ii[2]));
      f.e[comp][g.at(ib[0], ib[1], ib[2])] = (R)(in_old + kf * (in_new - b_old));
    }
  }
}

// ---------------------------------------------------------------------------
// Particles
// ---------------------------------------------------------------------------

// Incident field at (x, y, z), time t, build axes (the paper's (z, x, y)).
// KIND = 0 takes the model IncParams::kind names at run time; the push also
// instantiates one model fixed at compile time (KIND = the model's constant),
// which leaves the others' code and registers out of the kernel.
template <int KIND = 0>
__device__ __forceinline__ void incident3(const IncParams &P, double z_focus,
                                          double x, double y, double z,
                                          double t, double E[3], double B[3]) {
  const int kind = KIND ? KIND : P.kind;
#pragma unroll
  for (int c = 0; c < 3; ++c) E[c] = B[c] = 0.0;
  if (kind == SFPIC_INC_PLANE_PULSE_1D) {
    const double ph = t - P.t0 - x;
    const double v = P.a0 * sin(ph) * exp2(P.env_k * ph * ph);
    E[1] = v;
    B[2] = v;
  } else if (kind == SFPIC_INC_APRIL_LP || kind == SFPIC_INC_APRIL_RP) {
    const double X = (y - P.y_focus) * P.inv_a;  // paper x
    const double Y = (z - z_focus) * P.inv_a;    // paper y
    const double Z = (x - P.x_focus) * P.inv_a;  // paper z
    sfpic::cx<double> e[3], b[3];
    sfpic::april_complex_fields<KIND>(P, X, Y, Z, t - P.t_focus, e, b);
    E[0] = e[2].r;
    E[1] = e[0].r;
    E[2] = e[1].r;
    B[0] = b[2].r;
    B[1] = b[0].r;
    B[2] = b[1].r;
  }
}

// Three order-2 weights of the node nearest to xi (primal nodes at integers,
// dual at half-integers) and the array index of the first tap.
__device__ __forceinline__ int taps3(double xi, int dual, double w[3]) {
  const double s = dual ? xi - 0.5 : xi;
  const double c = floor(s + 0.5);
  sfpic::weights3(s - c, w);
  return (int)c - 1 + G;
}

struct PushArgs {
  double dt, qm, qw;
  double inv_h[3], h_over_dt[3];  // 1/h, h/dt
  double h[3];
  double time, z_focus;
};

// Particle tiles: TX x TY x TZ cells (x, the contiguous axis, longest).
// Every step starts with the particles sorted by tile (removed ones last),
// so a particle's old nearest node is in
// [tile start, tile end] along each axis and, since it moves less than one
// cell per step (the CFL limit), every node its current touches lies in the
// tile's window of T + 5 nodes per axis (old nearest node -2 .. +2).
#ifndef SFPIC3_TILE
#define SFPIC3_TILE 8, 4, 4
#endif
#ifndef SFPIC3_PUSH_THREADS
#define SFPIC3_PUSH_THREADS 256  // threads per push workgroup
#endif
#ifndef SFPIC3_PUSH_WGS
#define SFPIC3_PUSH_WGS 3  // workgroups per CU the push is compiled for
#endif
constexpr int kTile[3] = {SFPIC3_TILE};
constexpr int TX = kTile[0], TY = kTile[1], TZ = kTile[2];
constexpr int WX = TX + 5, WY = TY + 5, WZ = TZ + 5, WN = WX * WY * WZ;
// Field window: every gather tap of a particle in the tile lies in nodes
// t0 - 1 .. t0 + T + 1 along each axis, for primal and dual components.
constexpr int FX = TX + 3, FY = TY + 3, FZ = TZ + 3, FN = FX * FY * FZ;

struct Tiles {
  int ntx, nty, ntz;
  uint32_t ntiles;  // the removed particles' key is ntiles
};

__device__ __forceinline__ uint32_t tile_key(const Tiles &t, double x,
                                             double y, double z) {
  if (x < -1.0) return t.ntiles;
  const int cx = min((int)x, t.ntx * TX - 1), cy = min((int)y, t.nty * TY - 1),
            cz = min((int)z, t.ntz * TZ - 1);
  return ((uint32_t)(cz / TZ) * t.nty + (uint32_t)(cy / TY)) * t.ntx +
         (uint32_t)(cx / TX);
}

// Counting pass: rank of each particle within its key.  The lanes of a wave
// that share a key take one atomic between them (one round per distinct key
// in the wave: the particles arrive sorted, so there are few).
template <typename R>
__global__ void __launch_bounds__(256)
tile_count3(Parts3<R> p, int64_t n, Tiles t, uint32_t *count, uint32_t *rank) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = s < n;
  const uint32_t key =
      active ? tile_key(t, p.x[0][s], p.x[1][s], p.x[2][s]) : 0u;
  const int lane = threadIdx.x & 63;
  uint64_t todo = __ballot(active);
  uint32_t r = 0;
  while (todo) {
    const int leader = __ffsll((unsigned long long)todo) - 1;
    const uint32_t lk = __shfl(key, leader, 64);
    const uint64_t same = __ballot(active && key == lk);
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(count + lk, (uint32_t)__popcll(same));
    base = __shfl(base, leader, 64);
    if ((same >> lane) & 1ull)
      r = base + (uint32_t)__popcll(same & ((1ull << lane) - 1ull));
    todo &= ~same;
  }
  if (active) rank[s] = r;
}

// Exclusive scan of m counters in three passes: per 1024-block scan with the
// block totals, a scan of the totals, and the add-back.
__device__ __forceinline__ uint32_t block_scan_excl(uint32_t v,
                                                    uint32_t *sh,
                                                    uint32_t &total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t incl = v;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t u = __shfl_up(incl, o, 64);
    if (lane >= o) incl += u;
  }
  if (lane == 63) sh[w] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
      const uint32_t c = sh[k];
      sh[k] = acc;
      acc += c;
    }
    sh[16] = acc;
  }
  __syncthreads();
  const uint32_t out = sh[w] + incl - v;
  total = sh[16];
  __syncthreads();
  return out;
}

__global__ void __launch_bounds__(1024)
scan3_blocks(const uint32_t *in, uint32_t *out, uint32_t *sums, uint32_t m) {
  __shared__ uint32_t sh[17];
  const uint32_t i = blockIdx.x * 1024u + threadIdx.x;
  uint32_t tot;
  const uint32_t e = block_scan_excl(i < m ? in[i] : 0u, sh, tot);
  if (i < m) out[i] = e;
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(1024) scan3_sums(uint32_t *sums, uint32_t nb) {
  __shared__ uint32_t sh[17];
  uint32_t carry = 0;
  for (uint32_t b0 = 0; b0 < nb; b0 += 1024u) {
    const uint32_t i = b0 + threadIdx.x;
    uint32_t tot;
    const uint32_t e = block_scan_excl(i < nb ? sums[i] : 0u, sh, tot);
    if (i < nb) sums[i] = e + carry;
    carry += tot;
  }
}

__global__ void __launch_bounds__(1024)
scan3_add(uint32_t *out, const uint32_t *sums, uint32_t m) {
  const uint32_t i = blockIdx.x * 1024u + threadIdx.x;
  if (i < m) out[i] += sums[blockIdx.x];
}

// Scatter every slot to start[key] + rank in the other buffer, id with it.
template <typename R>
__global__ void __launch_bounds__(256)
tile_scatter3(Parts3<R> src, Parts3<R> dst, const uint32_t *sid, uint32_t *did,
              int64_t n, Tiles t, const uint32_t *start, const uint32_t *rank) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const double x = src.x[0][s], y = src.x[1][s], z = src.x[2][s];
  const uint32_t d = start[tile_key(t, x, y, z)] + rank[s];
  dst.x[0][d] = x;
  dst.x[1][d] = y;
  dst.x[2][d] = z;
#pragma unroll
  for (int c = 0; c < 3; ++c) dst.u[c][d] = src.u[c][s];
  did[d] = sid[s];
}

// One workgroup per tile (XCD-aware: workgroup b takes tile (b mod 8) S +
// b / 8, S = ceil(tiles / 8), so each XCD walks a contiguous band of tiles
// whose field halos share its L2).  The current of the tile's particles is
// accumulated in an FP64 LDS window and added to the global J once.
template <typename R, int KIND>
__global__ void __launch_bounds__(SFPIC3_PUSH_THREADS, SFPIC3_PUSH_WGS)
push3_tiled(F3<R> f, Geo g, Parts3<R> p, const uint32_t *__restrict__ start, Tiles t,
            PushArgs a, IncParams inc) {
  __shared__ double sj[3 * WN];
  __shared__ double sf[6 * FN];
  const uint32_t S = (t.ntiles + 7) >> 3, b = blockIdx.x;
  const uint32_t tile = (b & 7) * S + (b >> 3);
  if ((b >> 3) >= S || tile >= t.ntiles) return;
  const uint32_t pbeg = start[tile], pend = start[tile + 1];
  if (pbeg == pend) return;
  const int tx = (int)(tile % (uint32_t)t.ntx),
            ty = (int)((tile / (uint32_t)t.ntx) % (uint32_t)t.nty),
            tz = (int)(tile / ((uint32_t)t.ntx * (uint32_t)t.nty));
  // window node (0, 0, 0) is cell-node t0 - 2 along each axis
  const int w0[3] = {tx * TX - 2, ty * TY - 2, tz * TZ - 2};
  constexpr int NT = SFPIC3_PUSH_THREADS;
  const int tid = (int)threadIdx.x;
#pragma unroll
  for (int it = 0; it < (3 * WN + NT - 1) / NT; ++it) {
    const int k = tid + it * NT;
    if (k < 3 * WN) sj[k] = 0.0;
  }
  // Stage E^n and the centred B on the field window (array index of window
  // node (0, 0, 0): w0 + 1 + G; nodes past the array read as zero and are
  // never tapped).  All of a thread's window loads are issued first; the
  // thread's first particle is loaded and its incident field (which needs
  // no window) computed while they are in flight.
  const int fo[3] = {w0[0] + 1 + G, w0[1] + 1 + G, w0[2] + 1 + G};
  constexpr int kStage = (FN + NT - 1) / NT;
  double stage[kStage][6];
#pragma unroll
  for (int it = 0; it < kStage; ++it) {
    const int k = tid + it * NT;
    const int gi = fo[0] + k % FX, gj = fo[1] + (k / FX) % FY,
              gk = fo[2] + k / (FX * FY);
    const bool in = k < FN && gi < g.NX && gj < g.NY && gk < g.NZ;
    const size_t n = in ? g.at(gi, gj, gk) : 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      stage[it][c] = in ? ld(f.e[c], n) : 0.0;
      stage[it][3 + c] = in ? ld(f.bb[c], n) : 0.0;
    }
  }
  uint32_t s = pbeg + (uint32_t)tid;
  double xi[3], u[3], E[3], B[3];
  // position, momentum and incident field of particle s
  auto load_particle = [&]() {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      xi[d] = p.x[d][s];
      u[d] = ld(p.u[d], s);
    }
    if (KIND || inc.kind != SFPIC_INC_NONE) {
      incident3<KIND>(inc, a.z_focus, xi[0] * a.h[0], xi[1] * a.h[1],
                      xi[2] * a.h[2], a.time, E, B);
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) E[c] = B[c] = 0.0;
    }
  };
  if (s < pend) load_particle();
#pragma unroll
  for (int it = 0; it < kStage; ++it) {
    const int k = tid + it * NT;
    if (k < FN) {
#pragma unroll
      for (int c = 0; c < 6; ++c) sf[c * FN + k] = stage[it][c];
    }
  }
  __syncthreads();
  for (; s < pend;) {
    // gather E^n and the centred B at x^n from the field window, added to
    // the incident field: one component per iteration (fully unrolled, the
    // 162 taps need more registers than three workgroups per CU leave);
    // staggering bits per component (Ex Ey Ez Bx By Bz): dual along x for
    // Ex By Bz, along y for Ey Bx Bz, along z for Ez Bx By
    {
      double wp[3][3], wd[3][3];
      int bp[3], bd[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        bp[d] = taps3(xi[d], 0, wp[d]);
        bd[d] = taps3(xi[d], 1, wd[d]);
      }
      constexpr int kDualX = 0x31, kDualY = 0x2A, kDualZ = 0x1C;
#pragma unroll 1
      for (int c = 0; c < 6; ++c) {
        const bool sx = (kDualX >> c) & 1, sy = (kDualY >> c) & 1,
                   sz = (kDualZ >> c) & 1;
        const double *plane = sf + c * FN;
        double wx[3], wy[3], wz[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          wx[q] = sx ? wd[0][q] : wp[0][q];
          wy[q] = sy ? wd[1][q] : wp[1][q];
          wz[q] = sz ? wd[2][q] : wp[2][q];
        }
        const int b[3] = {sx ? bd[0] : bp[0], sy ? bd[1] : bp[1],
                          sz ? bd[2] : bp[2]};
        double v = 0.0;
        {
          const int lx = b[0] - fo[0], ly = b[1] - fo[1], lz = b[2] - fo[2];
#pragma unroll
          for (int cz = 0; cz < 3; ++cz)
#pragma unroll
            for (int by = 0; by < 3; ++by) {
              const double *row = plane + ((lz + cz) * FY + (ly + by)) * FX + lx;
              const double wyz = wy[by] * wz[cz];
              v += wx[0] * wyz * row[0] + wx[1] * wyz * row[1] +
                   wx[2] * wyz * row[2];
            }
        }
        if (c == 0) E[0] = v + E[0];
        else if (c == 1) E[1] = v + E[1];
        else if (c == 2) E[2] = v + E[2];
        else if (c == 3) B[0] = v + B[0];
        else if (c == 4) B[1] = v + B[1];
        else B[2] = v + B[2];
      }
    }
    sfpic::boris<double>(a.qm, a.dt, u, E, B);
    const double gi =
        sfpic::rsqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    // Esirkepov on the 4 nodes per axis that the old and the new shape can
    // cover: around the old nearest node c, c - 1 .. c + 2 for a move up the
    // axis and c - 2 .. c + 1 otherwise (a move below one cell keeps the new
    // nearest node within one node of c).  S0 and S1 are the shapes before
    // and after the move, D = S1 - S0; the transverse weight of component d,
    //   S0_e S0_f + D_e S0_f / 2 + S0_e D_f / 2 + D_e D_f / 3,
    // equals M_e M_f + D_e D_f / 12 with M = S0 + D / 2, and the current
    // along d is the running sum of D_d over the first three nodes (the sum
    // over all four is zero).  When the nearest node does not change, the
    // shapes cover three nodes and only two entries of the running sum are
    // non-zero (the other is zero, or a rounding residue of a zero sum, and
    // is not added): entries kd_lo .. kd_hi.  Each shape is the three
    // order-2 weights about its nearest node (S1 about the new one, c1,
    // exactly as the next step's gather and S0 will find them), placed in
    // the frame: S0 from frame node 1 - up, S1 from frame node 0 when
    // c1 - c = up - 1 and from node 1 otherwise.
    double M[3][4], D[3][4], x1[3];
    int lo[3], kd_lo[3], kd_hi[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      x1[d] = xi[d] + a.dt * a.inv_h[d] * (u[d] * gi);
      const double c = floor(xi[d] + 0.5), c1 = floor(x1[d] + 0.5);
      const int up = x1[d] >= xi[d];
      const bool same = c1 == c;
      lo[d] = (int)c - 2 + up - w0[d];  // window index of the first node
      kd_lo[d] = (!up && same) ? 1 : 0;
      kd_hi[d] = (up && same) ? 1 : 2;
      double w[3], w1[3];
      sfpic::weights3(xi[d] - c, w);
      sfpic::weights3(x1[d] - c1, w1);
      const bool lead = c1 - c == (double)(up - 1);
      const double S0[4] = {up ? w[0] : 0.0, up ? w[1] : w[0],
                            up ? w[2] : w[1], up ? 0.0 : w[2]};
      const double S1[4] = {lead ? w1[0] : 0.0, lead ? w1[1] : w1[0],
                            lead ? w1[2] : w1[1], lead ? 0.0 : w1[2]};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        D[d][k] = S1[k] - S0[k];
        M[d][k] = S0[k] + 0.5 * D[d][k];
      }
    }
    constexpr double twelfth = 1.0 / 12.0;
    constexpr int kStride[3] = {1, WX, WX * WY};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int e = (d + 1) % 3, fa = (d + 2) % 3;
      const double scale = -a.qw * a.h_over_dt[d];
      double Mf[4], Df[4];  // rotated so that index 0 is the current kf
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        Mf[k] = M[fa][k];
        Df[k] = D[fa][k] * twelfth;
      }
      double sd[3];  // scale * D_d
#pragma unroll
      for (int k = 0; k < 3; ++k) sd[k] = scale * D[d][k];
      int addr = d * WN + lo[0] + lo[1] * WX + lo[2] * WX * WY;
#pragma unroll 1
      for (int kf = 0; kf < 4; ++kf) {
        const double mf = Mf[0], df = Df[0];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          Mf[k] = Mf[k + 1];
          Df[k] = Df[k + 1];
        }
#pragma unroll
        for (int ke = 0; ke < 4; ++ke) {
          const double tw = M[e][ke] * mf + D[e][ke] * df;
          if (tw == 0.0) continue;  // a node outside both shapes
          double acc = 0.0;
#pragma unroll
          for (int kd = 0; kd < 3; ++kd) {
            acc += sd[kd] * tw;
            if (kd >= kd_lo[d] && kd <= kd_hi[d])
              atomicAdd(&sj[addr + kd * kStride[d] + ke * kStride[e]], acc);
          }
        }
        addr += kStride[fa];
      }
    }
    // written as "inside" so that a non-finite position is removed too (it
    // would otherwise index the field arrays on the next step)
    const bool out = !(x1[0] >= 0.0 && x1[0] < (double)g.nx && x1[1] >= 0.0 &&
                       x1[1] < (double)g.ny && x1[2] >= 0.0 &&
                       x1[2] < (double)g.nz);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      p.x[d][s] = (d == 0 && out) ? kDead : x1[d];
      p.u[d][s] = (R)u[d];
    }
    s += NT;
    if (s < pend) load_particle();
  }
  __syncthreads();
  // add the window to the global current (windows of neighbouring tiles
  // overlap by 5 nodes per axis)
  for (int k = tid; k < WN; k += NT) {
    const int ix = k % WX, iy = (k / WX) % WY, iz = k / (WX * WY);
    const int gi = w0[0] + ix + G, gj = w0[1] + iy + G, gk = w0[2] + iz + G;
    if (gi >= g.NX || gj >= g.NY || gk >= g.NZ) continue;
    const size_t n = g.at(gi, gj, gk);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double v = sj[c * WN + k];
      if (v != 0.0) atomicAdd(f.j[c] + n, (R)v);
    }
  }
}

// The push for the incident model of the run: one model fixed at compile
// time when there is one at the particles, else the run-time choice.
template <typename R>
void launch_push3(uint32_t grid, hipStream_t st, F3<R> f, Geo g, Parts3<R> p,
                  const uint32_t *start, Tiles t, PushArgs a,
                  const IncParams &inc) {
  switch (inc.kind) {
    case SFPIC_INC_PLANE_PULSE_1D:
      push3_tiled<R, SFPIC_INC_PLANE_PULSE_1D><<<grid, SFPIC3_PUSH_THREADS, 0, st>>>(
          f, g, p, start, t, a, inc);
      break;
    case SFPIC_INC_APRIL_LP:
      push3_tiled<R, SFPIC_INC_APRIL_LP><<<grid, SFPIC3_PUSH_THREADS, 0, st>>>(f, g, p, start,
                                                               t, a, inc);
      break;
    case SFPIC_INC_APRIL_RP:
      push3_tiled<R, SFPIC_INC_APRIL_RP><<<grid, SFPIC3_PUSH_THREADS, 0, st>>>(f, g, p, start,
                                                               t, a, inc);
      break;
    default:
      push3_tiled<R, 0><<<grid, SFPIC3_PUSH_THREADS, 0, st>>>(f, g, p, start, t, a, inc);
  }
}

// Explicit particles: physical positions to cell units.
template <typename R>
__global__ void load3(Parts3<R> p, int64_t n, const double *x, const double *y,
                      const double *z, const double *ux, const double *uy,
                      const double *uz, double ihx, double ihy, double ihz) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  p.x[0][i] = x[i] * ihx;
  p.x[1][i] = y[i] * ihy;
  p.x[2][i] = z[i] * ihz;
  p.u[0][i] = (R)ux[i];
  p.u[1][i] = (R)uy[i];
  p.u[2][i] = (R)uz[i];
}

// Generated particles: ppc per cell of the region, uniform in the cell, the
// Philox4x32-10 stream keyed by (seed, species index) with counter (id, word
// 2 = 0 / 1 / 2 / 3); momenta Maxwellian of width sigma (Box-Muller).
// With a density profile (off != nullptr) particle i sits in region row
// i / per_row (y fastest, then z) and in the column whose offsets bracket
// i % per_row.
template <typename R>
__global__ void init3(Parts3<R> p, int64_t n, int64_t x0, int64_t y0, int64_t z0,
                      int64_t ncx, int64_t ncy, int ppc, double sigma,
                      uint32_t k0, uint32_t k1, const uint32_t *off,
                      uint32_t per_row) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t cx, cy, cz;
  if (off) {
    const int64_t row = i / per_row;
    cx = x0 + sfpic::find_segment(off, (int)ncx,
                                  (uint32_t)(i - row * per_row));
    cy = y0 + row % ncy;
    cz = z0 + row / ncy;
  } else {
    const int64_t cell = i / ppc;
    cx = x0 + cell % ncx;
    cy = y0 + (cell / ncx) % ncy;
    cz = z0 + cell / (ncx * ncy);
  }
  const uint32_t lo = (uint32_t)i, hi = (uint32_t)((uint64_t)i >> 32);
  uint32_t c[4] = {lo, hi, 0u, 0u}, c3[4] = {lo, hi, 3u, 0u};
  sfpic::philox4x32_10(c, k0, k1);
  sfpic::philox4x32_10(c3, k0, k1);
  double a, b, cc, unused;
  sfpic::u01_pair(c, a, b);
  sfpic::u01_pair(c3, cc, unused);
  double ux = 0.0, uy = 0.0, uz = 0.0;
  if (sigma > 0.0) {
    uint32_t c1[4] = {lo, hi, 1u, 0u}, c2[4] = {lo, hi, 2u, 0u};
    sfpic::philox4x32_10(c1, k0, k1);
    sfpic::philox4x32_10(c2, k0, k1);
    double a1, b1, a2, b2;
    sfpic::u01_pair(c1, a1, b1);
    sfpic::u01_pair(c2, a2, b2);
    const double r1 = sqrt(-2.0 * log1p(-a1)), r2 = sqrt(-2.0 * log1p(-a2));
    const double tp = 6.283185307179586;
    ux = sigma * r1 * cos(tp * b1);
    uy = sigma * r1 * sin(tp * b1);
    uz = sigma * r2 * cos(tp * b2);
  }
  p.x[0][i] = (double)cx + a;
  p.x[1][i] = (double)cy + b;
  p.x[2][i] = (double)cz + cc;
  p.u[0][i] = (R)ux;
  p.u[1][i] = (R)uy;
  p.u[2][i] = (R)uz;
}

// ---------------------------------------------------------------------------
// Diagnostics
// ---------------------------------------------------------------------------

__device__ __forceinline__ double block_sum(double v, double *sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += sh[k];
  __syncthreads();
  return t;
}

// acc[0] += sum (gamma - 1), acc[1] += live count; flag |= 1 on non-finite
template <typename R>
__global__ void __launch_bounds__(256)
psums3(Parts3<R> p, int64_t n, double *acc, int *flag) {
  __shared__ double sh[4];
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double g1 = 0.0, cnt = 0.0;
  if (s < n && p.x[0][s] >= -1.0) {
    const double u0 = ld(p.u[0], s), u1 = ld(p.u[1], s), u2 = ld(p.u[2], s);
    const double q = u0 * u0 + u1 * u1 + u2 * u2;
    if (!isfinite(q)) atomicOr(flag, 1);
    g1 = q / (sqrt(1.0 + q) + 1.0);  // gamma - 1 without cancellation
    cnt = 1.0;
  }
  g1 = block_sum(g1, sh);
  cnt = block_sum(cnt, sh);
  if (threadIdx.x == 0) {
    atomicAdd(acc, g1);
    atomicAdd(acc + 1, cnt);
  }
}

// acc[0] += 1/2 sum over every array element of E^2 + B^2
template <typename R>
__global__ void __launch_bounds__(256)
fsums3(F3<R> f, size_t n, double *acc, int *flag) {
  __shared__ double sh[4];
  const size_t s = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (s < n) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double e = ld(f.e[c], s), b = ld(f.b[c], s);
      v += e * e + b * b;
    }
    if (!isfinite(v)) atomicOr(flag, 1);
  }
  v = block_sum(0.5 * v, sh);
  if (threadIdx.x == 0) atomicAdd(acc, v);
}

// rho += q w S(x) on the primal nodes (order-2, 27 nodes per particle)
template <typename R>
__global__ void __launch_bounds__(256)
rho3(Parts3<R> p, int64_t n, Geo g, double qw, double *rho) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  double xi[3], w[3][3];
  int b[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) xi[d] = p.x[d][s];
  if (xi[0] < -1.0) return;
#pragma unroll
  for (int d = 0; d < 3; ++d) b[d] = taps3(xi[d], 0, w[d]);
  for (int c = 0; c < 3; ++c)
    for (int bb = 0; bb < 3; ++bb)
      for (int aa = 0; aa < 3; ++aa)
        atomicAdd(rho + g.at(b[0] + aa, b[1] + bb, b[2] + c),
                  qw * w[0][aa] * w[1][bb] * w[2][c]);
}

constexpr int kGaussPlanes = 8;

// max |div_h E - (rho - rho0)|, max |rho - rho0|, max |g - gprev| and max
// |rho| over nodes at least 4 cells inside the physical box, with g = div_h
// E - (rho - rho0) the per-node Gauss defect, stored into gprev for the next
// call (have_prev: gprev holds the previous call's defect, whose difference
// with g is the discrete continuity residual between the calls).  Maxima of
// non-negative doubles order as integers; a NaN counts as +inf.  The block
// reduces first and issues one atomic per maximum: an atomic per node on
// two addresses serializes the whole grid.
__device__ __forceinline__ double inf_if_nan3(double v) {
  return isnan(v) ? __builtin_huge_val() : v;
}

template <typename R>
__global__ void __launch_bounds__(256)
gauss3(F3<R> f, Geo g, const double *rho, const double *rho0, double ihx,
       double ihy, double ihz, double *gprev, int have_prev,
       unsigned long long *mx, unsigned long long *mx2) {
  __shared__ double sh[4][4];
  const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y * 4 + threadIdx.y;
  const int lo = G + 4;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  // each block covers kGaussPlanes consecutive z-planes
  for (int kk = 0; kk < kGaussPlanes; ++kk) {
    const int k = blockIdx.z * kGaussPlanes + kk;
    if (i < lo || j < lo || k < lo || i > G + g.nx - 4 || j > G + g.ny - 4 ||
        k > G + g.nz - 4)
      continue;
    const size_t n = g.at(i, j, k), sj = g.P, sk = (size_t)g.P * g.NY;
    const double div = (ld(f.e[0], n) - ld(f.e[0], n - 1)) * ihx +
                       (ld(f.e[1], n) - ld(f.e[1], n - sj)) * ihy +
                       (ld(f.e[2], n) - ld(f.e[2], n - sk)) * ihz;
    const double dr = rho[n] - rho0[n];
    const double gd = div - dr;
    v[0] = fmax(v[0], inf_if_nan3(fabs(gd)));
    v[1] = fmax(v[1], inf_if_nan3(fabs(dr)));
    if (have_prev) v[2] = fmax(v[2], inf_if_nan3(fabs(gd - gprev[n])));
    v[3] = fmax(v[3], inf_if_nan3(fabs(rho[n])));
    gprev[n] = gd;
  }
  for (int o = 32; o > 0; o >>= 1)
    for (int q = 0; q < 4; ++q) v[q] = fmax(v[q], __shfl_down(v[q], o, 64));
  // blockDim (64, 4): wave w is row threadIdx.y
  if (threadIdx.x == 0)
    for (int q = 0; q < 4; ++q) sh[q][threadIdx.y] = v[q];
  __syncthreads();
  if (threadIdx.x == 0 && threadIdx.y == 0) {
    for (int w = 1; w < 4; ++w)
      for (int q = 0; q < 4; ++q) v[q] = fmax(v[q], sh[q][w]);
    atomicMax(mx, (unsigned long long)__double_as_longlong(v[0]));
    atomicMax(mx + 1, (unsigned long long)__double_as_longlong(v[1]));
    atomicMax(mx2, (unsigned long long)__double_as_longlong(v[2]));
    atomicMax(mx2 + 1, (unsigned long long)__double_as_longlong(v[3]));
  }
}

// Half-cell offsets (0 or 1/2) of Ex Ey Ez Bx By Bz along x, y, z, the field
// pointer of component c and the matching incident component, as select
// chains (a run-time index would put the arrays in private memory).
__device__ __forceinline__ void stag3(int c, double &hx, double &hy,
                                      double &hz) {
  hx = (c == 0 || c == 4 || c == 5) ? 0.5 : 0.0;
  hy = (c == 1 || c == 3 || c == 5) ? 0.5 : 0.0;
  hz = (c == 2 || c == 3 || c == 4) ? 0.5 : 0.0;
}

template <typename R>
__device__ __forceinline__ const R *comp3(const F3<R> &f, int c) {
  return c == 0   ? f.e[0]
         : c == 1 ? f.e[1]
         : c == 2 ? f.e[2]
         : c == 3 ? f.b[0]
         : c == 4 ? f.b[1]
                  : f.b[2];
}

__device__ __forceinline__ double pick3(int c, const double E[3],
                                        const double B[3]) {
  return c == 0   ? E[0]
         : c == 1 ? E[1]
         : c == 2 ? E[2]
         : c == 3 ? B[0]
         : c == 4 ? B[1]
                  : B[2];
}

// acc[4] += 1/2 sum over the physical nodes (i, j, k < nx, ny, nz) of
// |F_scatt + F_inc|^2 over the six components, each at its own Yee node, E at
// tE = t^n and B at tB = t^{n-1/2}, the incident field in FP64 (the energy of
// the total field, Sec. 2).  Grid (ceil(nx / 256), ny, nz).
template <typename R>
__global__ void __launch_bounds__(256)
em_total3(F3<R> f, Geo g, IncParams inc, double z_focus, double dx, double dy,
          double dz, double tE, double tB, double *acc) {
  __shared__ double sh[4];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y, k = blockIdx.z;
  double e = 0.0;
  if (i < g.nx) {
    const size_t n = g.at(i + G, j + G, k + G);
#pragma unroll 1
    for (int c = 0; c < 6; ++c) {
      double hx, hy, hz, E[3], B[3];
      stag3(c, hx, hy, hz);
      incident3(inc, z_focus, (i + hx) * dx, (j + hy) * dy, (k + hz) * dz,
                c < 3 ? tE : tB, E, B);
      const double v = ld(comp3(f, c), n) + pick3(c, E, B);
      e += 0.5 * v * v;
    }
  }
  e = block_sum(e, sh);
  if (threadIdx.x == 0) atomicAdd(acc + 4, e);
}

// dst = F_scatt + F_inc of component c (0..5) at every array element, its
// node at ((i - G) + hx) dx, ((j - G) + hy) dy, ((k - G) + hz) dz, time t; FP64.
// Grid (ceil(NX / 256), NY, NZ).
template <typename R>
__global__ void __launch_bounds__(256)
total_field3(F3<R> f, Geo g, IncParams inc, double z_focus, int c, double dx,
             double dy, double dz, double t, double *dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y, k = blockIdx.z;
  if (i >= g.NX) return;
  const size_t n = g.at(i, j, k);
  double hx, hy, hz, E[3], B[3];
  stag3(c, hx, hy, hz);
  incident3(inc, z_focus, (i - G + hx) * dx, (j - G + hy) * dy,
            (k - G + hz) * dz, t, E, B);
  dst[n] = ld(comp3(f, c), n) + pick3(c, E, B);
}

// Energy-angle histogram of live particles (weights w dV): linear kinetic
// energy bins over [0, emax), angle from +x in [0, 180] degrees; moments
// {sum w, w E_k, w E_k^2, w theta, w theta^2} over E_k > ek_min.
template <typename R>
__global__ void __launch_bounds__(256)
hist3(Parts3<R> p, int64_t n, double m, double wdv, int n_e, double emax,
      int n_t, double ek_min, int plane, double *hist, double *mom) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n || p.x[0][s] < -1.0) return;
  const double ux = ld(p.u[0], s), uy = ld(p.u[1], s), uz = ld(p.u[2], s);
  const double ek = m * (sqrt(1.0 + ux * ux + uy * uy + uz * uz) - 1.0);
  // polar angle from +x, or of the momentum projected on the x-z (plane 1)
  // or x-y (plane 2) plane
  const double perp = plane == 1   ? fabs(uz)
                      : plane == 2 ? fabs(uy)
                                   : sqrt(uy * uy + uz * uz);
  const double th = atan2(perp, ux) * (180.0 / 3.14159265358979323846);
  if (!isfinite(ek) || !isfinite(th)) return;
  const double ie = floor(ek / emax * n_e);
  const double tt = fmin(floor(th / 180.0 * n_t), (double)(n_t - 1));
  if (ie >= 0.0 && ie < (double)n_e && tt >= 0.0)
    atomicAdd(&hist[(size_t)ie * n_t + (size_t)tt], wdv);
  if (ek > ek_min) {
    atomicAdd(&mom[0], wdv);
    atomicAdd(&mom[1], wdv * ek);
    atomicAdd(&mom[2], wdv * ek * ek);
    atomicAdd(&mom[3], wdv * th);
    atomicAdd(&mom[4], wdv * th * th);
  }
}

}  // namespace sfpic3

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
using namespace sfpic3;

// The host keeps one pointer set per object; the momentum (and field)
// pointers hold values of the storage type and are cast for the float
// kernels (parts_as, fields_as).
struct Species3 {
  double q = -1.0, m = 1.0, w = 0.0;
  int64_t n = 0;
  Parts3<double> p{}, alt{};               // particles, sort target
  uint32_t *id = nullptr, *id_alt = nullptr;  // creation index per slot
};

// iota: slot i holds particle i
__global__ void iota3(uint32_t *id, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) id[i] = (uint32_t)i;
}

struct sfpic3_sim {
  sfpic3_grid grid{};
  sfpic_runtime rt{};
  hipStream_t st = nullptr;
  Geo g{};
  size_t plane = 0;  // elements per field array
  IncParams inc{};
  double z_focus = 0.0;
  int64_t step = 0;
  bool fp32 = false;  // fields and momenta stored as float
  F3<double> f{};
  double *face[3] = {};
  Tiles tiles{};
  uint32_t *count = nullptr, *start = nullptr, *sums = nullptr;
  uint32_t *rank = nullptr;  // per slot, sized for the largest species
  std::vector<Species3> sp;
  double *rho0 = nullptr, *rho = nullptr, *acc = nullptr;
  // per-node Gauss defect of the last diagnostics call (allocated by the
  // first call) and its step (-1: none, or the state has changed since)
  double *gprev = nullptr;
  int64_t gprev_step = -1;
  std::vector<std::pair<void *, size_t>> allocs;

  void *dalloc(size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    void *p = nullptr;
    if (rt.alloc)
      p = rt.alloc(bytes, rt.alloc_ctx);
    else if (hipMalloc(&p, bytes) != hipSuccess)
      p = nullptr;
    if (p) allocs.emplace_back(p, bytes);
    return p;
  }
  void dfree(void *p) {
    for (size_t k = 0; k < allocs.size(); ++k)
      if (allocs[k].first == p) {
        if (rt.free)
          rt.free(p, allocs[k].second, rt.alloc_ctx);
        else
          (void)hipFree(p);
        allocs.erase(allocs.begin() + (long)k);
        return;
      }
  }
  void release() {
    for (auto &a : allocs) {
      if (rt.free)
        rt.free(a.first, a.second, rt.alloc_ctx);
      else
        (void)hipFree(a.first);
    }
    allocs.clear();
  }
};

namespace {

#define HIP3(expr)                                                        \
  do {                                                                    \
    hipError_t e_ = (expr);                                               \
    if (e_ != hipSuccess)                                                 \
      return sfpic::fail(SFPIC_E_DEVICE,                                  \
                         std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

dim3 node_grid(const Geo &g) {
  return dim3((unsigned)((g.NX + 63) / 64), (unsigned)((g.NY + 3) / 4),
              (unsigned)g.NZ);
}

// node_grid with kGaussPlanes z-planes per block
dim3 gauss_grid(const Geo &g) {
  const dim3 d = node_grid(g);
  return dim3(d.x, d.y, (unsigned)((g.NZ + kGaussPlanes - 1) / kGaussPlanes));
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

template <typename R>
F3<R> fields_as(const F3<double> &f) {
  F3<R> r;
  for (int c = 0; c < 3; ++c) {
    r.e[c] = (R *)f.e[c];
    r.b[c] = (R *)f.b[c];
    r.j[c] = (R *)f.j[c];
    r.bb[c] = (R *)f.bb[c];
  }
  return r;
}

template <typename R>
Parts3<R> parts_as(const Parts3<double> &p) {
  Parts3<R> r;
  for (int d = 0; d < 3; ++d) {
    r.x[d] = p.x[d];
    r.u[d] = (R *)p.u[d];
  }
  return r;
}

template <int A, typename R>
int face_pass(sfpic3_sim *S, bool save, double kf) {
  int e, fa;
  face_axes(A, e, fa);
  const int64_t area = (int64_t)ext(S->g, e) * ext(S->g, fa);
  const F3<R> f = fields_as<R>(S->f);
  if (save)
    save_faces3<A, R><<<blocks_for(area), 256, 0, S->st>>>(f, S->g, S->face[A]);
  else
    mur3<A, R><<<blocks_for(area), 256, 0, S->st>>>(f, S->g, S->face[A], kf);
  HIP3(hipGetLastError());
  return SFPIC_OK;
}

template <typename R>
int one_step_t(sfpic3_sim *S) {
  const sfpic3_grid &gr = S->grid;
  const double dt = gr.dt;
  const double cx = dt / gr.dx, cy = dt / gr.dy, cz = dt / gr.dz;
  const F3<R> f = fields_as<R>(S->f);
  faraday3<R><<<node_grid(S->g), dim3(64, 4), 0, S->st>>>(f, S->g, cx, cy, cz);
  HIP3(hipGetLastError());
  PushArgs a{};
  a.dt = dt;
  a.h[0] = gr.dx;
  a.h[1] = gr.dy;
  a.h[2] = gr.dz;
  for (int d = 0; d < 3; ++d) {
    a.inv_h[d] = 1.0 / a.h[d];
    a.h_over_dt[d] = a.h[d] / dt;
  }
  a.time = (double)S->step * dt;
  a.z_focus = S->z_focus;
  const Tiles &t = S->tiles;
  const uint32_t m = t.ntiles + 1, nb = (m + 1023) / 1024;
  const uint32_t grid8 = (t.ntiles + 7) / 8 * 8;
  for (auto &sp : S->sp) {
    if (sp.n == 0) continue;
    // sort by tile (removed particles last), ids along
    HIP3(hipMemsetAsync(S->count, 0, (size_t)m * 4, S->st));
    tile_count3<R><<<blocks_for(sp.n), 256, 0, S->st>>>(
        parts_as<R>(sp.p), sp.n, t, S->count, S->rank);
    scan3_blocks<<<nb, 1024, 0, S->st>>>(S->count, S->start, S->sums, m);
    scan3_sums<<<1, 1024, 0, S->st>>>(S->sums, nb);
    scan3_add<<<nb, 1024, 0, S->st>>>(S->start, S->sums, m);
    tile_scatter3<R><<<blocks_for(sp.n), 256, 0, S->st>>>(
        parts_as<R>(sp.p), parts_as<R>(sp.alt), sp.id, sp.id_alt, sp.n, t,
        S->start, S->rank);
    HIP3(hipGetLastError());
    std::swap(sp.p, sp.alt);
    std::swap(sp.id, sp.id_alt);
    a.qm = sp.q / sp.m;
    a.qw = sp.q * sp.w;
    launch_push3<R>(grid8, S->st, f, S->g, parts_as<R>(sp.p), S->start, t,
                    a, S->inc);
    HIP3(hipGetLastError());
  }
  if (int r = face_pass<0, R>(S, true, 0.0)) return r;
  if (int r = face_pass<1, R>(S, true, 0.0)) return r;
  if (int r = face_pass<2, R>(S, true, 0.0)) return r;
  ampere3<R><<<node_grid(S->g), dim3(64, 4), 0, S->st>>>(f, S->g, dt, cx, cy,
                                                         cz);
  HIP3(hipGetLastError());
  const double kx = (dt - gr.dx) / (dt + gr.dx), ky = (dt - gr.dy) / (dt + gr.dy),
               kz = (dt - gr.dz) / (dt + gr.dz);
  if (int r = face_pass<2, R>(S, false, kz)) return r;  // z faces first
  if (int r = face_pass<1, R>(S, false, ky)) return r;
  if (int r = face_pass<0, R>(S, false, kx)) return r;
  S->step++;
  return SFPIC_OK;
}

int one_step(sfpic3_sim *S) {
  return S->fp32 ? one_step_t<float>(S) : one_step_t<double>(S);
}

int deposit_rho(sfpic3_sim *S, double *rho) {
  HIP3(hipMemsetAsync(rho, 0, S->plane * 8, S->st));
  for (auto &sp : S->sp) {
    if (sp.n == 0) continue;
    if (S->fp32)
      rho3<float><<<blocks_for(sp.n), 256, 0, S->st>>>(
          parts_as<float>(sp.p), sp.n, S->g, sp.q * sp.w, rho);
    else
      rho3<double><<<blocks_for(sp.n), 256, 0, S->st>>>(sp.p, sp.n, S->g,
                                                        sp.q * sp.w, rho);
    HIP3(hipGetLastError());
  }
  return SFPIC_OK;
}

}  // namespace

extern "C" {

int sfpic3_create(const sfpic3_grid *grid, const sfpic3_species *species,
                  int nspecies, const sfpic_incident *incident,
                  sfpic_precision precision, const sfpic_runtime *runtime,
                  sfpic3_sim **out) {
  if (!out) return sfpic::fail(SFPIC_E_INVAL, "out is NULL");
  if (precision != SFPIC_FP64 && precision != SFPIC_FP32)
    return sfpic::fail(SFPIC_E_INVAL, "precision must be SFPIC_FP64 or SFPIC_FP32");
  *out = nullptr;
  if (!grid) return sfpic::fail(SFPIC_E_INVAL, "grid is NULL");
  const sfpic3_grid &g = *grid;
  if (g.nx < 1 || g.ny < 1 || g.nz < 1 || g.nx > 32768 || g.ny > 32768 ||
      g.nz > 32768)
    return sfpic::fail(SFPIC_E_INVAL, "3D grid needs 1 <= nx, ny, nz <= 32768");
  if (!(g.dx > 0.0) || !(g.dy > 0.0) || !(g.dz > 0.0) || !(g.dt > 0.0))
    return sfpic::fail(SFPIC_E_INVAL, "3D grid needs dx, dy, dz, dt > 0");
  const double cfl =
      g.dt * std::sqrt(1.0 / (g.dx * g.dx) + 1.0 / (g.dy * g.dy) +
                       1.0 / (g.dz * g.dz));
  if (!(cfl < 1.0)) return sfpic::fail(SFPIC_E_INVAL, "dt violates the 3D Yee CFL limit");
  if (nspecies < 0 || (nspecies > 0 && !species))
    return sfpic::fail(SFPIC_E_INVAL, "bad species list");
  IncParams P{};
  if (int r = sfpic::prepare_incident_ext(incident, P)) return r;
  if (P.kind == SFPIC_INC_GAUSS_2D)
    return sfpic::fail(SFPIC_E_INVAL, "the paraxial Gaussian beam is 2D only");
  if (P.on_nodes)
    return sfpic::fail(SFPIC_E_INVAL, "3D runs evaluate the incident field at the particles (on_nodes = 0)");
  // particles: validate on the host before anything is allocated
  for (int s = 0; s < nspecies; ++s) {
    const sfpic3_species &d = species[s];
    if (!(d.m > 0.0) || !std::isfinite(d.q))
      return sfpic::fail(SFPIC_E_INVAL, "species needs m > 0 and finite q");
    if (d.n_explicit > kMaxParticles)
      return sfpic::fail(SFPIC_E_SIZE, "too many explicit particles");
    if (d.n_explicit > 0) {
      if (!d.x || !d.y || !d.z || !d.ux || !d.uy || !d.uz)
        return sfpic::fail(SFPIC_E_INVAL, "explicit species needs all six arrays");
      if (!std::isfinite(d.weight))
        return sfpic::fail(SFPIC_E_INVAL, "explicit species needs a finite weight");
      const double hi[3] = {g.nx * g.dx, g.ny * g.dy, g.nz * g.dz};
      const double *xs[3] = {d.x, d.y, d.z};
      for (int64_t i = 0; i < d.n_explicit; ++i) {
        for (int a = 0; a < 3; ++a)
          if (!(xs[a][i] >= 0.0 && xs[a][i] < hi[a]))
            return sfpic::fail(SFPIC_E_INVAL, "explicit particle outside the box");
        if (!std::isfinite(d.ux[i]) || !std::isfinite(d.uy[i]) ||
            !std::isfinite(d.uz[i]))
          return sfpic::fail(SFPIC_E_INVAL, "non-finite explicit momentum");
      }
    } else if (d.n_explicit == 0 && d.ppc > 0) {
      const int64_t *r = d.region;
      if (!(r[0] >= 0 && r[0] < r[1] && r[1] <= g.nx && r[2] >= 0 &&
            r[2] < r[3] && r[3] <= g.ny && r[4] >= 0 && r[4] < r[5] &&
            r[5] <= g.nz))
        return sfpic::fail(SFPIC_E_INVAL, "species region outside the grid");
      if (d.temperature_ev < 0.0 || !std::isfinite(d.density))
        return sfpic::fail(SFPIC_E_INVAL, "bad density or temperature");
      // a profiled species is counted (and checked) once its column
      // offsets are known, below
      const int64_t np = (r[1] - r[0]) * (r[3] - r[2]) * (r[5] - r[4]) * d.ppc;
      if (d.profile == SFPIC_PROFILE_UNIFORM && np > kMaxParticles)
        return sfpic::fail(SFPIC_E_SIZE, "too many generated particles");
    } else if (d.n_explicit < 0 || d.ppc < 0) {
      return sfpic::fail(SFPIC_E_INVAL, "negative particle count");
    }
  }
  HIP3(hipSetDevice(runtime ? runtime->device : 0));
  sfpic3_sim *S = new sfpic3_sim();
  S->grid = g;
  S->fp32 = precision == SFPIC_FP32;
  const size_t esz = S->fp32 ? 4 : 8;  // bytes per field value and momentum
  if (runtime) S->rt = *runtime;
  S->st = (hipStream_t)S->rt.stream;
  S->inc = P;
  S->z_focus = incident ? incident->z_focus : 0.0;
  S->g.nx = (int)g.nx;
  S->g.ny = (int)g.ny;
  S->g.nz = (int)g.nz;
  S->g.NX = (int)g.nx + 2 * G;
  S->g.NY = (int)g.ny + 2 * G;
  S->g.NZ = (int)g.nz + 2 * G;
  S->g.P = (S->g.NX + 63) / 64 * 64;
  S->plane = (size_t)S->g.P * S->g.NY * S->g.NZ;
  auto fail_free = [&](int code, const char *msg) {
    S->release();
    delete S;
    return sfpic::fail(code, msg);
  };
  double *planes[12];
  for (int c = 0; c < 12; ++c) {
    planes[c] = (double *)S->dalloc(S->plane * esz);
    if (!planes[c]) return fail_free(SFPIC_E_NOMEM, "field allocation failed");
    if (hipMemsetAsync(planes[c], 0, S->plane * esz, S->st) != hipSuccess)
      return fail_free(SFPIC_E_DEVICE, "field clear failed");
  }
  for (int c = 0; c < 3; ++c) {
    S->f.e[c] = planes[c];
    S->f.b[c] = planes[3 + c];
    S->f.j[c] = planes[6 + c];
    S->f.bb[c] = planes[9 + c];
  }
  for (int A = 0; A < 3; ++A) {
    int e, fa;
    face_axes(A, e, fa);
    S->face[A] = (double *)S->dalloc((size_t)8 * 8 * ext(S->g, e) * ext(S->g, fa));
    if (!S->face[A]) return fail_free(SFPIC_E_NOMEM, "face buffer allocation failed");
  }
  S->tiles.ntx = (int)((g.nx + TX - 1) / TX);
  S->tiles.nty = (int)((g.ny + TY - 1) / TY);
  S->tiles.ntz = (int)((g.nz + TZ - 1) / TZ);
  S->tiles.ntiles =
      (uint32_t)S->tiles.ntx * (uint32_t)S->tiles.nty * (uint32_t)S->tiles.ntz;
  {
    // start holds ntiles + 2 offsets: the tiles, the removed bucket, the end
    const size_t m = (size_t)S->tiles.ntiles + 2;
    S->count = (uint32_t *)S->dalloc(m * 4);
    S->start = (uint32_t *)S->dalloc(m * 4);
    S->sums = (uint32_t *)S->dalloc(((m + 1023) / 1024 + 1) * 4);
    if (!S->count || !S->start || !S->sums)
      return fail_free(SFPIC_E_NOMEM, "sort scratch allocation failed");
  }
  S->rho0 = (double *)S->dalloc(S->plane * 8);
  S->rho = (double *)S->dalloc(S->plane * 8);
  S->acc = (double *)S->dalloc(128);
  if (!S->rho0 || !S->rho || !S->acc)
    return fail_free(SFPIC_E_NOMEM, "diagnostic allocation failed");
  std::vector<uint32_t> off;  // column offsets of a density profile
  for (int s = 0; s < nspecies; ++s) {
    const sfpic3_species &d = species[s];
    Species3 sp;
    sp.q = d.q;
    sp.m = d.m;
    if (d.n_explicit > 0) {
      sp.n = d.n_explicit;
      sp.w = d.weight;
    } else if (d.ppc > 0) {
      const int64_t *r = d.region;
      sp.n = (r[1] - r[0]) * (r[3] - r[2]) * (r[5] - r[4]) * d.ppc;
      sp.w = d.density / d.ppc;
      if (d.profile != SFPIC_PROFILE_UNIFORM) {
        if (int rc = sfpic::profile_offsets(d.profile, d.profile_center,
                                            d.profile_fwhm, d.profile_order,
                                            d.profile_xmin, r[0], r[1], g.dx,
                                            d.ppc, off)) {
          S->release();
          delete S;
          return rc;
        }
        sp.n = (int64_t)off.back() * (r[3] - r[2]) * (r[5] - r[4]);
        if (sp.n > kMaxParticles)
          return fail_free(SFPIC_E_SIZE, "too many generated particles");
      }
    }
    if (sp.n > 0) {
      for (int a = 0; a < 3; ++a) {
        sp.p.x[a] = (double *)S->dalloc((size_t)sp.n * 8);
        sp.p.u[a] = (double *)S->dalloc((size_t)sp.n * esz);
        sp.alt.x[a] = (double *)S->dalloc((size_t)sp.n * 8);
        sp.alt.u[a] = (double *)S->dalloc((size_t)sp.n * esz);
        if (!sp.p.x[a] || !sp.p.u[a] || !sp.alt.x[a] || !sp.alt.u[a])
          return fail_free(SFPIC_E_NOMEM, "particle allocation failed");
      }
      sp.id = (uint32_t *)S->dalloc((size_t)sp.n * 4);
      sp.id_alt = (uint32_t *)S->dalloc((size_t)sp.n * 4);
      if (!sp.id || !sp.id_alt)
        return fail_free(SFPIC_E_NOMEM, "particle id allocation failed");
      iota3<<<blocks_for(sp.n), 256, 0, S->st>>>(sp.id, sp.n);
      if (d.n_explicit > 0) {
        const size_t b = (size_t)sp.n * 8;
        double *tmp = (double *)S->dalloc(6 * b);
        if (!tmp) return fail_free(SFPIC_E_NOMEM, "staging allocation failed");
        const double *src[6] = {d.x, d.y, d.z, d.ux, d.uy, d.uz};
        for (int c = 0; c < 6; ++c)
          if (hipMemcpyAsync((char *)tmp + c * b, src[c], b,
                             hipMemcpyHostToDevice, S->st) != hipSuccess)
            return fail_free(SFPIC_E_DEVICE, "particle upload failed");
        if (S->fp32)
          load3<float><<<blocks_for(sp.n), 256, 0, S->st>>>(
              parts_as<float>(sp.p), sp.n, tmp, tmp + sp.n, tmp + 2 * sp.n,
              tmp + 3 * sp.n, tmp + 4 * sp.n, tmp + 5 * sp.n, 1.0 / g.dx,
              1.0 / g.dy, 1.0 / g.dz);
        else
          load3<double><<<blocks_for(sp.n), 256, 0, S->st>>>(
              sp.p, sp.n, tmp, tmp + sp.n, tmp + 2 * sp.n, tmp + 3 * sp.n,
              tmp + 4 * sp.n, tmp + 5 * sp.n, 1.0 / g.dx, 1.0 / g.dy,
              1.0 / g.dz);
        if (hipStreamSynchronize(S->st) != hipSuccess)
          return fail_free(SFPIC_E_DEVICE, "particle upload failed");
        S->dfree(tmp);
      } else {
        const int64_t *r = d.region;
        const double sigma =
            d.temperature_ev > 0.0 ? std::sqrt(d.temperature_ev / (510998.95 * d.m)) : 0.0;
        uint32_t *doff = nullptr;
        if (d.profile != SFPIC_PROFILE_UNIFORM) {
          doff = (uint32_t *)S->dalloc(off.size() * 4);
          if (!doff) return fail_free(SFPIC_E_NOMEM, "profile table allocation failed");
          if (hipMemcpyAsync(doff, off.data(), off.size() * 4,
                             hipMemcpyHostToDevice, S->st) != hipSuccess)
            return fail_free(SFPIC_E_DEVICE, "profile table upload failed");
        }
        if (S->fp32)
          init3<float><<<blocks_for(sp.n), 256, 0, S->st>>>(
              parts_as<float>(sp.p), sp.n, r[0], r[2], r[4], r[1] - r[0],
              r[3] - r[2], d.ppc, sigma, (uint32_t)d.seed,
              (uint32_t)d.species_index, doff, doff ? off.back() : 0u);
        else
          init3<double><<<blocks_for(sp.n), 256, 0, S->st>>>(
              sp.p, sp.n, r[0], r[2], r[4], r[1] - r[0], r[3] - r[2], d.ppc,
              sigma, (uint32_t)d.seed, (uint32_t)d.species_index, doff,
              doff ? off.back() : 0u);
        if (hipGetLastError() != hipSuccess)
          return fail_free(SFPIC_E_DEVICE, "particle generation failed");
      }
    }
    S->sp.push_back(sp);
  }
  int64_t nmax = 1;
  for (auto &sp : S->sp) nmax = std::max(nmax, sp.n);
  S->rank = (uint32_t *)S->dalloc((size_t)nmax * 4);
  if (!S->rank) return fail_free(SFPIC_E_NOMEM, "sort scratch allocation failed");
  if (deposit_rho(S, S->rho0) != SFPIC_OK ||
      hipStreamSynchronize(S->st) != hipSuccess)
    return fail_free(SFPIC_E_DEVICE, "initial charge density failed");
  *out = S;
  return SFPIC_OK;
}

int sfpic3_step(sfpic3_sim *sim, int64_t nsteps) {
  sfpic::ErrScope es_(sim);
  if (!sim || nsteps < 0) return sfpic::fail(SFPIC_E_INVAL, "bad step call");
  for (int64_t k = 0; k < nsteps; ++k)
    if (int r = one_step(sim)) return r;
  return SFPIC_OK;
}

int sfpic3_sync(sfpic3_sim *sim) {
  sfpic::ErrScope es_(sim);
  if (!sim) return sfpic::fail(SFPIC_E_INVAL, "sim is NULL");
  HIP3(hipStreamSynchronize(sim->st));
  return SFPIC_OK;
}

int sfpic3_dims(const sfpic3_sim *sim, int64_t out[3]) {
  sfpic::ErrScope es_(sim);
  if (!sim || !out) return sfpic::fail(SFPIC_E_INVAL, "NULL argument");
  out[0] = sim->g.NX;
  out[1] = sim->g.NY;
  out[2] = sim->g.NZ;
  return SFPIC_OK;
}

static double *comp_ptr(sfpic3_sim *S, int comp) {
  if (comp < 0 || comp >= SFPIC_NCOMP) return nullptr;
  if (comp < 3) return S->f.e[comp];
  if (comp < 6) return S->f.b[comp - 3];
  return S->f.j[comp - 6];
}

int sfpic3_read_field(sfpic3_sim *sim, int comp, double *out, size_t n) {
  sfpic::ErrScope es_(sim);
  if (!sim || !out) return sfpic::fail(SFPIC_E_INVAL, "NULL argument");
  double *src = comp_ptr(sim, comp);
  if (!src) return sfpic::fail(SFPIC_E_INVAL, "bad field component");
  const Geo &g = sim->g;
  if (n != (size_t)g.NX * g.NY * g.NZ)
    return sfpic::fail(SFPIC_E_SIZE, "field buffer must hold NX*NY*NZ values");
  if (!sim->fp32) {
    HIP3(hipMemcpy2DAsync(out, (size_t)g.NX * 8, src, (size_t)g.P * 8,
                          (size_t)g.NX * 8, (size_t)g.NY * g.NZ,
                          hipMemcpyDeviceToHost, sim->st));
    HIP3(hipStreamSynchronize(sim->st));
    return SFPIC_OK;
  }
  std::vector<float> tmp(n);
  HIP3(hipMemcpy2DAsync(tmp.data(), (size_t)g.NX * 4, src, (size_t)g.P * 4,
                        (size_t)g.NX * 4, (size_t)g.NY * g.NZ,
                        hipMemcpyDeviceToHost, sim->st));
  HIP3(hipStreamSynchronize(sim->st));
  for (size_t i = 0; i < n; ++i) out[i] = (double)tmp[i];
  return SFPIC_OK;
}

int sfpic3_write_field(sfpic3_sim *sim, int comp, const double *in, size_t n) {
  sfpic::ErrScope es_(sim);
  if (!sim || !in) return sfpic::fail(SFPIC_E_INVAL, "NULL argument");
  if (comp < 0 || comp >= 6)
    return sfpic::fail(SFPIC_E_INVAL, "only E and B can be written");
  double *dst = comp_ptr(sim, comp);
  const Geo &g = sim->g;
  if (n != (size_t)g.NX * g.NY * g.NZ)
    return sfpic::fail(SFPIC_E_SIZE, "field buffer must hold NX*NY*NZ values");
  if (!sim->fp32) {
    HIP3(hipMemcpy2DAsync(dst, (size_t)g.P * 8, in, (size_t)g.NX * 8,
                          (size_t)g.NX * 8, (size_t)g.NY * g.NZ,
                          hipMemcpyHostToDevice, sim->st));
    HIP3(hipStreamSynchronize(sim->st));
    return SFPIC_OK;
  }
  std::vector<float> tmp(in, in + n);  // rounded to the storage type
  HIP3(hipMemcpy2DAsync(dst, (size_t)g.P * 4, tmp.data(), (size_t)g.NX * 4,
                        (size_t)g.NX * 4, (size_t)g.NY * g.NZ,
                        hipMemcpyHostToDevice, sim->st));
  HIP3(hipStreamSynchronize(sim->st));
  return SFPIC_OK;
}

int sfpic3_particle_count(sfpic3_sim *sim, int species, int64_t *n) {
  sfpic::ErrScope es_(sim);
  if (!sim || !n) return sfpic::fail(SFPIC_E_INVAL, "NULL argument");
  if (species < 0 || species >= (int)sim->sp.size())
    return sfpic::fail(SFPIC_E_INVAL, "bad species index");
  *n = sim->sp[species].n;
  return SFPIC_OK;
}

int sfpic3_read_particles(sfpic3_sim *sim, int species, double *x, double *y,
                          double *z, double *ux, double *uy, double *uz,
                          uint8_t *alive, size_t n) {
  sfpic::ErrScope es_(sim);
  if (!sim || !x || !y || !z || !ux || !uy || !uz || !alive)
    return sfpic::fail(SFPIC_E_INVAL, "NULL argument");
  if (species < 0 || species >= (int)sim->sp.size())
    return sfpic::fail(SFPIC_E_INVAL, "bad species index");
  const Species3 &sp = sim->sp[species];
  if (n != (size_t)sp.n)
    return sfpic::fail(SFPIC_E_SIZE, "particle buffers must hold the slot count");
  if (n == 0) return SFPIC_OK;
  // slots are in tile order on the device: stage them, then place each by
  // its creation index
  double *dst[6] = {x, y, z, ux, uy, uz};
  std::vector<double> stage(6 * n);
  std::vector<float> ustage(sim->fp32 ? 3 * n : 0);
  std::vector<uint32_t> id(n);
  for (int a = 0; a < 3; ++a) {
    HIP3(hipMemcpyAsync(stage.data() + a * n, sp.p.x[a], n * 8,
                        hipMemcpyDeviceToHost, sim->st));
    if (sim->fp32)
      HIP3(hipMemcpyAsync(ustage.data() + a * n, sp.p.u[a], n * 4,
                          hipMemcpyDeviceToHost, sim->st));
    else
      HIP3(hipMemcpyAsync(stage.data() + (3 + a) * n, sp.p.u[a], n * 8,
                          hipMemcpyDeviceToHost, sim->st));
  }
  HIP3(hipMemcpyAsync(id.data(), sp.id, n * 4, hipMemcpyDeviceToHost, sim->st));
  HIP3(hipStreamSynchronize(sim->st));
  if (sim->fp32)
    for (size_t k = 0; k < 3 * n; ++k) stage[3 * n + k] = (double)ustage[k];
  const double h[3] = {sim->grid.dx, sim->grid.dy, sim->grid.dz};
  for (size_t s = 0; s < n; ++s) {
    const size_t i = id[s];
    if (i >= n) return sfpic::fail(SFPIC_E_STATE, "particle ids corrupted");
    alive[i] = stage[s] >= -1.0;
    for (int a = 0; a < 3; ++a) {
      dst[a][i] = stage[a * n + s] * h[a];
      dst[3 + a][i] = stage[(3 + a) * n + s];
    }
  }
  return SFPIC_OK;
}

int sfpic3_diagnostics(sfpic3_sim *sim, sfpic_diag *out) {
  sfpic::ErrScope es_(sim);
  if (!sim || !out) return sfpic::fail(SFPIC_E_INVAL, "NULL argument");
  sfpic3_sim *S = sim;
  const sfpic3_grid &g = S->grid;
  const double dV = g.dx * g.dy * g.dz;
  memset(out, 0, sizeof(*out));
  out->step = S->step;
  out->time = (double)S->step * g.dt;
  int *flag = (int *)(S->acc + 7);
  std::vector<double> host(8);
  for (auto &sp : S->sp) {
    HIP3(hipMemsetAsync(S->acc, 0, 64, S->st));
    if (sp.n > 0) {
      if (S->fp32)
        psums3<float><<<blocks_for(sp.n), 256, 0, S->st>>>(
            parts_as<float>(sp.p), sp.n, S->acc, flag);
      else
        psums3<double><<<blocks_for(sp.n), 256, 0, S->st>>>(sp.p, sp.n,
                                                            S->acc, flag);
      HIP3(hipGetLastError());
    }
    HIP3(hipMemcpyAsync(host.data(), S->acc, 64, hipMemcpyDeviceToHost, S->st));
    HIP3(hipStreamSynchronize(S->st));
    int fl = 0;
    memcpy(&fl, &host[7], sizeof(int));
    out->w_kin += sp.w * sp.m * host[0] * dV;
    out->charge += sp.q * sp.w * host[1] * dV;
    out->n_alive += (int64_t)host[1];
    out->nonfinite |= fl;
  }
  HIP3(hipMemsetAsync(S->acc, 0, 64, S->st));
  if (S->fp32)
    fsums3<float><<<blocks_for((int64_t)S->plane), 256, 0, S->st>>>(
        fields_as<float>(S->f), S->plane, S->acc, flag);
  else
    fsums3<double><<<blocks_for((int64_t)S->plane), 256, 0, S->st>>>(
        S->f, S->plane, S->acc, flag);
  HIP3(hipGetLastError());
  if (int r = deposit_rho(S, S->rho)) return r;
  if (!S->gprev) {
    S->gprev = (double *)S->dalloc(S->plane * 8);
    if (!S->gprev)
      return sfpic::fail(SFPIC_E_NOMEM, "diagnostic allocation failed");
    S->gprev_step = -1;
  }
  HIP3(hipMemsetAsync(S->acc + 8, 0, 16, S->st));
  unsigned long long *mx = (unsigned long long *)(S->acc + 2);
  unsigned long long *mx2 = (unsigned long long *)(S->acc + 8);
  const int have_prev = S->gprev_step >= 0;
  if (S->fp32)
    gauss3<float><<<gauss_grid(S->g), dim3(64, 4), 0, S->st>>>(
        fields_as<float>(S->f), S->g, S->rho, S->rho0, 1.0 / g.dx,
        1.0 / g.dy, 1.0 / g.dz, S->gprev, have_prev, mx, mx2);
  else
    gauss3<double><<<gauss_grid(S->g), dim3(64, 4), 0, S->st>>>(
        S->f, S->g, S->rho, S->rho0, 1.0 / g.dx, 1.0 / g.dy, 1.0 / g.dz,
        S->gprev, have_prev, mx, mx2);
  HIP3(hipGetLastError());
  host.resize(16);
  HIP3(hipMemcpyAsync(host.data(), S->acc, 128, hipMemcpyDeviceToHost, S->st));
  HIP3(hipStreamSynchronize(S->st));
  out->continuity_residual = have_prev ? host[8] : 0.0;
  out->continuity_steps = have_prev ? S->step - S->gprev_step : 0;
  out->rho_abs_max = host[9];
  S->gprev_step = S->step;
  out->w_em = host[0] * dV;
  unsigned long long r0 = 0, r1 = 0;
  memcpy(&r0, &host[2], 8);
  memcpy(&r1, &host[3], 8);
  double gr = 0.0, rm = 0.0;
  memcpy(&gr, &r0, 8);
  memcpy(&rm, &r1, 8);
  out->gauss_residual = gr;
  out->rho_max = rm;
  int fl = 0;
  memcpy(&fl, &host[7], sizeof(int));
  out->nonfinite |= fl;
  // energy of the total field (scattered + incident) on the physical nodes
  HIP3(hipMemsetAsync(S->acc + 4, 0, 8, S->st));
  {
    const double tE = (double)S->step * g.dt, tB = tE - 0.5 * g.dt;
    const dim3 grid3((g.nx + 255) / 256, g.ny, g.nz);
    if (S->fp32)
      em_total3<float><<<grid3, 256, 0, S->st>>>(
          fields_as<float>(S->f), S->g, S->inc, S->z_focus, g.dx, g.dy, g.dz,
          tE, tB, S->acc);
    else
      em_total3<double><<<grid3, 256, 0, S->st>>>(
          S->f, S->g, S->inc, S->z_focus, g.dx, g.dy, g.dz, tE, tB, S->acc);
    HIP3(hipGetLastError());
  }
  HIP3(hipMemcpyAsync(host.data(), S->acc, 64, hipMemcpyDeviceToHost, S->st));
  HIP3(hipStreamSynchronize(S->st));
  out->w_em_total = host[4] * dV;
  return SFPIC_OK;
}

int sfpic3_read_total_field(sfpic3_sim *sim, int comp, double *out,
                            size_t n) {
  sfpic::ErrScope es_(sim);
  if (!sim || !out) return sfpic::fail(SFPIC_E_INVAL, "NULL argument");
  if (comp < 0 || comp >= 6)
    return sfpic::fail(SFPIC_E_INVAL, "component must be E or B");
  sfpic3_sim *S = sim;
  const Geo &g = S->g;
  if (n != (size_t)g.NX * g.NY * g.NZ)
    return sfpic::fail(SFPIC_E_SIZE, "field buffer must hold NX*NY*NZ values");
  const sfpic3_grid &gr = S->grid;
  const double tE = (double)S->step * gr.dt;
  const double t = comp < 3 ? tE : tE - 0.5 * gr.dt;
  const dim3 grid3((g.NX + 255) / 256, g.NY, g.NZ);
  // S->rho is FP64 scratch of one field array; the charge diagnostics clear
  // and refill it before every use
  if (S->fp32)
    total_field3<float><<<grid3, 256, 0, S->st>>>(
        fields_as<float>(S->f), g, S->inc, S->z_focus, comp, gr.dx, gr.dy,
        gr.dz, t, S->rho);
  else
    total_field3<double><<<grid3, 256, 0, S->st>>>(
        S->f, g, S->inc, S->z_focus, comp, gr.dx, gr.dy, gr.dz, t, S->rho);
  HIP3(hipGetLastError());
  HIP3(hipMemcpy2DAsync(out, (size_t)g.NX * 8, S->rho, (size_t)g.P * 8,
                        (size_t)g.NX * 8, (size_t)g.NY * g.NZ,
                        hipMemcpyDeviceToHost, S->st));
  HIP3(hipStreamSynchronize(S->st));
  return SFPIC_OK;
}

int sfpic3_histogram(sfpic3_sim *sim, const sfpic_hist_spec *spec,
                     double *out, size_t n, double *moments) {
  sfpic::ErrScope es_(sim);
  if (!sim || !spec || !out) return sfpic::fail(SFPIC_E_INVAL, "NULL argument");
  if (spec->species < 0 || spec->species >= (int)sim->sp.size() ||
      spec->n_energy <= 0 || spec->n_theta <= 0 || !(spec->e_max > 0.0) ||
      spec->plane < SFPIC_ANGLE_POLAR || spec->plane > SFPIC_ANGLE_XY)
    return sfpic::fail(SFPIC_E_INVAL, "bad histogram spec");
  const size_t nb = (size_t)spec->n_energy * spec->n_theta;
  if (n != nb) return sfpic::fail(SFPIC_E_SIZE, "n must be n_energy * n_theta");
  double *d = (double *)sim->dalloc((nb + 8) * 8);
  if (!d) return sfpic::fail(SFPIC_E_NOMEM, "histogram allocation failed");
  const Species3 &sp = sim->sp[spec->species];
  const double wdv = sp.w * sim->grid.dx * sim->grid.dy * sim->grid.dz;
  double mom[8] = {0};
  int rc = SFPIC_OK;
  if (hipMemsetAsync(d, 0, (nb + 8) * 8, sim->st) != hipSuccess) rc = -1;
  if (!rc && sp.n > 0) {
    if (sim->fp32)
      hist3<float><<<blocks_for(sp.n), 256, 0, sim->st>>>(
          parts_as<float>(sp.p), sp.n, sp.m, wdv, spec->n_energy,
          spec->e_max, spec->n_theta, spec->ek_min, spec->plane, d + 8, d);
    else
      hist3<double><<<blocks_for(sp.n), 256, 0, sim->st>>>(
          sp.p, sp.n, sp.m, wdv, spec->n_energy, spec->e_max, spec->n_theta,
          spec->ek_min, spec->plane, d + 8, d);
    if (hipGetLastError() != hipSuccess) rc = -1;
  }
  if (!rc && (hipMemcpyAsync(out, d + 8, nb * 8, hipMemcpyDeviceToHost,
                             sim->st) != hipSuccess ||
              hipMemcpyAsync(mom, d, 8 * 8, hipMemcpyDeviceToHost, sim->st) !=
                  hipSuccess ||
              hipStreamSynchronize(sim->st) != hipSuccess))
    rc = -1;
  (void)hipStreamSynchronize(sim->st);
  sim->dfree(d);
  if (rc) return sfpic::fail(SFPIC_E_DEVICE, "histogram failed");
  if (moments) {
    moments[0] = mom[0];
    for (int k = 1; k < 5; ++k) moments[k] = mom[0] > 0.0 ? mom[k] / mom[0] : 0.0;
  }
  return SFPIC_OK;
}

// Checkpoint layout: header {magic, nx, ny, nz, storage bytes, nspecies,
// step, 0} as int64, then E and B (6 arrays [NZ][NY][NX] of the storage
// type), then per species its slot count and, in device order, x y z
// (double), ux uy uz (storage type) and the creation ids.  J and the centred
// B are recomputed by every step and are not saved.
static constexpr int64_t kState3Magic = 0x3353465049433344ll;

static size_t state3_bytes(const sfpic3_sim *S) {
  const size_t es = S->fp32 ? 4 : 8;
  size_t b = 8 * 8 + 6 * (size_t)S->g.NX * S->g.NY * S->g.NZ * es;
  for (const auto &sp : S->sp) b += 8 + (size_t)sp.n * (3 * 8 + 3 * es + 4);
  return b;
}

int sfpic3_get_state(sfpic3_sim *sim, void *buf, size_t *n) {
  sfpic::ErrScope es_(sim);
  if (!sim || !n) return sfpic::fail(SFPIC_E_INVAL, "NULL argument");
  const size_t need = state3_bytes(sim);
  if (!buf) {
    *n = need;
    return SFPIC_OK;
  }
  if (*n != need) return sfpic::fail(SFPIC_E_SIZE, "state buffer size mismatch");
  const Geo &g = sim->g;
  const size_t es = sim->fp32 ? 4 : 8;
  char *w = (char *)buf;
  const int64_t hdr[8] = {kState3Magic, g.nx, g.ny, g.nz, (int64_t)es,
                          (int64_t)sim->sp.size(), sim->step, 0};
  memcpy(w, hdr, sizeof(hdr));
  w += sizeof(hdr);
  for (int c = 0; c < 6; ++c) {
    const double *src = c < 3 ? sim->f.e[c] : sim->f.b[c - 3];
    HIP3(hipMemcpy2DAsync(w, (size_t)g.NX * es, src, (size_t)g.P * es,
                          (size_t)g.NX * es, (size_t)g.NY * g.NZ,
                          hipMemcpyDeviceToHost, sim->st));
    w += (size_t)g.NX * g.NY * g.NZ * es;
  }
  for (const auto &sp : sim->sp) {
    const int64_t cnt = sp.n;
    memcpy(w, &cnt, 8);
    w += 8;
    for (int a = 0; a < 3; ++a) {
      HIP3(hipMemcpyAsync(w, sp.p.x[a], (size_t)sp.n * 8,
                          hipMemcpyDeviceToHost, sim->st));
      w += (size_t)sp.n * 8;
    }
    for (int a = 0; a < 3; ++a) {
      HIP3(hipMemcpyAsync(w, sp.p.u[a], (size_t)sp.n * es,
                          hipMemcpyDeviceToHost, sim->st));
      w += (size_t)sp.n * es;
    }
    HIP3(hipMemcpyAsync(w, sp.id, (size_t)sp.n * 4, hipMemcpyDeviceToHost,
                        sim->st));
    w += (size_t)sp.n * 4;
  }
  HIP3(hipStreamSynchronize(sim->st));
  return SFPIC_OK;
}

int sfpic3_set_state(sfpic3_sim *sim, const void *buf, size_t n) {
  sfpic::ErrScope es_(sim);
  if (!sim || !buf) return sfpic::fail(SFPIC_E_INVAL, "NULL argument");
  if (n != state3_bytes(sim))
    return sfpic::fail(SFPIC_E_SIZE, "state does not fit this simulation");
  const Geo &g = sim->g;
  const size_t es = sim->fp32 ? 4 : 8;
  const char *r = (const char *)buf;
  int64_t hdr[8];
  memcpy(hdr, r, sizeof(hdr));
  r += sizeof(hdr);
  if (hdr[0] != kState3Magic || hdr[1] != g.nx || hdr[2] != g.ny ||
      hdr[3] != g.nz || hdr[4] != (int64_t)es ||
      hdr[5] != (int64_t)sim->sp.size() || hdr[6] < 0)
    return sfpic::fail(SFPIC_E_STATE, "state is from another configuration");
  for (int c = 0; c < 6; ++c) {
    double *dst = c < 3 ? sim->f.e[c] : sim->f.b[c - 3];
    HIP3(hipMemcpy2DAsync(dst, (size_t)g.P * es, r, (size_t)g.NX * es,
                          (size_t)g.NX * es, (size_t)g.NY * g.NZ,
                          hipMemcpyHostToDevice, sim->st));
    r += (size_t)g.NX * g.NY * g.NZ * es;
  }
  for (auto &sp : sim->sp) {
    int64_t cnt = 0;
    memcpy(&cnt, r, 8);
    r += 8;
    if (cnt != sp.n)
      return sfpic::fail(SFPIC_E_STATE, "state species sizes differ");
    for (int a = 0; a < 3; ++a) {
      HIP3(hipMemcpyAsync(sp.p.x[a], r, (size_t)sp.n * 8,
                          hipMemcpyHostToDevice, sim->st));
      r += (size_t)sp.n * 8;
    }
    for (int a = 0; a < 3; ++a) {
      HIP3(hipMemcpyAsync(sp.p.u[a], r, (size_t)sp.n * es,
                          hipMemcpyHostToDevice, sim->st));
      r += (size_t)sp.n * es;
    }
    HIP3(hipMemcpyAsync(sp.id, r, (size_t)sp.n * 4, hipMemcpyHostToDevice,
                        sim->st));
    r += (size_t)sp.n * 4;
  }
  HIP3(hipStreamSynchronize(sim->st));
  sim->step = hdr[6];
  sim->gprev_step = -1;
  return SFPIC_OK;
}

void sfpic3_destroy(sfpic3_sim *sim) {
  sfpic::ErrScope es_(sim);
  sfpic::forget_handle(sim);
  if (!sim) return;
  (void)hipStreamSynchronize(sim->st);
  sim->release();
  delete sim;
}

}  // extern "C"
