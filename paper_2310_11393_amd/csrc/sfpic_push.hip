// Particle side of the step on gfx950: counting sort of particles by cell
// (tile-major key) and the tiled push kernel (order-2 gather, incident field
// at the particle, Boris, Esirkepov deposition; Lytova et al., Sec. 2).
//
// Tiled push: after each sort the non-empty tiles of tx x ty cells are cut
// into work items of at most item_particles particles, one workgroup each.
// The workgroup accumulates the current in an FP64 LDS window of its tile's
// nodes (the tile plus slack + 2 nodes on every side) with LDS atomics and
// adds that window to the global current once; it gathers the scattered E
// and centred B from a window of the same shape staged in LDS, or, in the
// single simulation's FP32 push, straight from global memory (L1/L2, the
// LDS being that push's busiest unit).  The lanes of a wave push
// particles of different cells, which keeps their LDS atomics off common
// addresses: in FP64 the sort lays out each tile's particles with cell order
// running down the 64 columns of each block of 1024 slots and a wave reads
// and writes a row of 64 consecutive slots straight from HBM; in the FP32
// form chunks of the cell-sorted range are staged through LDS and taken in
// transposed order there.  A particle that has drifted more than `slack`
// cells out of its tile since the last sort is listed and pushed afterwards
// by the straggler kernel from global memory.
//
// Two precisions of the same kernels: FP64 (positions as doubles in cell
// units) and the FP32 form (packed integer cell plus float offsets, float
// fields and momenta, FP64 incident-field phase, FP64 current accumulation).
#include <type_traits>

#include "sfpic_common.h"
#include "sfpic_device.h"

namespace sfpic {

// Minimum resident workgroups per CU requested from the compiler for the
// push kernels (bounds their register use).
#ifndef SFPIC_PUSH_MIN_BLOCKS
#define SFPIC_PUSH_MIN_BLOCKS 2
#endif
// The LDS field window of a tile with drift allowance `slack` (TileGeom):
// a particle is pushed by its tile's workgroup while its cell is at most
// slack cells outside the tile, and its order-2 gather and deposit reach 2
// more nodes, so the window spans physical nodes c0 - slack - 2 .. c0 + T +
// slack + 2.  Window index of physical node c0 + k is k + slack + 2; array
// index of window index w is c0 + w - slack + 1 (3 guard cells).
__host__ __device__ __forceinline__ int win_extra(int slack) {
  return 2 * slack + 5;
}
// The single-simulation push has the default 2D tile (16 x 16 cells, the
// precision's default slack) compiled in; the FP32 form then pads each
// window row by one node (24 instead of 23: fewer LDS bank conflicts, 4096^2
// RP push 3.89 -> 3.81 ms); FP64 keeps 27, a 28th would cost its third
// workgroup per CU.
template <typename R>
__host__ __device__ constexpr int fixed_slack() {
  return sizeof(R) == 8 ? kSingleSlackF64 : kSingleSlackF32;
}
template <typename R>
__host__ __device__ constexpr int fixed_row_pad() {
  return sizeof(R) == 8 ? 0 : 1;
}
template <typename R>
__host__ __device__ inline bool fixed_geometry(const TileGeom &tg, int dims) {
  return dims == 2 && tg.tx == 16 && tg.ty == 16 &&
         tg.slack == fixed_slack<R>();
}

// LDS chunk of the staged particle path (the FP32 form, see PT): 256 PER
// particles per chunk, PER per thread; lane l of wave w takes chunk slots
// m(l)*4PER + w*PER + j with m(l) = 4 (l mod 16) + l / 16, so the lanes of a
// wave sit in different cells of the cell-sorted chunk, and so do (as far as
// the chunk allows) the 16 lanes whose LDS accesses the hardware serves
// together: their slots are 16 PER apart, and lanes that share a cell at a
// high particle density fall in different sixteens (against m(l) = l: single
// 4096^2 RP push 3.82 -> 3.76 ms, 64-member sweep 18.97 -> 20.42 G pushes/s;
// m(l) = 2 (l mod 32) + l / 32 and 8 (l mod 8) + l / 8 were slower).  One
// pad word every 4 PER spreads the lanes over the banks.  Both the single
// and the batched push take 2 per thread: the batch's smaller chunk lets
// four of its workgroups share a CU (16.3 -> 17.1 G pushes/s on a 64-member
// FP32 sweep), and with the lane map above the single push is faster with it
// too (3.76 -> 3.65 ms; with m(l) = l it was 7% slower).
constexpr int kChunkPer = 2, kBatchChunkPer = 2;
template <int PER>
struct Chunk {
  static constexpr int per = PER;
  static constexpr int size = 256 * per;
  static constexpr int stride = 4 * per;
  static constexpr int pad = size + size / stride;  // padded length
};
template <int PER>
__device__ __forceinline__ int chunk_slot(int k) {
  return k + k / Chunk<PER>::stride;
}
// Position m(l) of lane l among the 64 lane columns of a chunk.
__device__ __forceinline__ int chunk_lane_pos(int lane) {
  return (lane & 15) * 4 + (lane >> 4);
}

__global__ void fill_u32(uint32_t *a, uint32_t v, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// Largest value below 1 in precision R (offsets live in [0, 1)).
template <typename R>
__device__ __forceinline__ R one_below();
template <>
__device__ __forceinline__ double one_below<double>() {
  return 0.99999999999999989;  // 1 - 2^-53
}
template <>
__device__ __forceinline__ float one_below<float>() {
  return 0.99999994f;  // 1 - 2^-24
}

// ---------------------------------------------------------------------------
// Particle storage per precision: load and store of one slot as (cell,
// offset) per axis and u.  kStaged selects the particle path of the push:
//   FP64 (kStaged false): the sort transposes each block of 1024 slots (see
//     block_slot) and the push reads and writes its rows straight from HBM;
//   FP32 form (kStaged true): the sort keeps plain cell order and the push
//     stages chunks through LDS and transposes there (its particles are
//     small, so staging is cheap, and a transposing sort of 28-byte records
//     costs more than it saves).
// ---------------------------------------------------------------------------
template <typename R>
struct PT;

template <>
struct PT<double> {
  static constexpr bool kStaged = false;
  // Raw words of one slot, loaded ahead of their use, and their decoding
  // (false if the particle was removed).
  struct Raw {
    double x, y, ux, uy, uz;
  };
  __device__ static Raw fetch(const Particles<double> &p, uint32_t g,
                              int dims) {
    return Raw{p.px[g], dims == 2 ? p.py[g] : 0.0, p.ux[g], p.uy[g], p.uz[g]};
  }
  __device__ static bool decode(const Raw &r, int dims, int &ix, int &iy,
                                double &fx, double &fy, double u[3]) {
    if (r.x < -1.0) return false;
    ix = (int)floor(r.x);
    fx = r.x - ix;
    iy = 0;
    fy = 0.0;
    if (dims == 2) {
      iy = (int)floor(r.y);
      fy = r.y - iy;
    }
    u[0] = r.ux;
    u[1] = r.uy;
    u[2] = r.uz;
    return true;
  }
  __device__ static bool load_global(const Particles<double> &p, uint32_t g,
                                     int dims, int &ix, int &iy, double &fx,
                                     double &fy, double u[3]) {
    const double xi = p.px[g];
    if (xi < -1.0) return false;
    ix = (int)floor(xi);
    fx = xi - ix;
    iy = 0;
    fy = 0.0;
    if (dims == 2) {
      const double yi = p.py[g];
      iy = (int)floor(yi);
      fy = yi - iy;
    }
    u[0] = p.ux[g];
    u[1] = p.uy[g];
    u[2] = p.uz[g];
    return true;
  }
  __device__ static void store_global(const Particles<double> &p, uint32_t g,
                                      int dims, bool alive, int ix, int iy,
                                      double fx, double fy,
                                      const double u[3]) {
    p.px[g] = alive ? (double)ix + fx : kDeadPos;
    if (dims == 2) p.py[g] = (double)iy + fy;
    p.ux[g] = u[0];
    p.uy[g] = u[1];
    p.uz[g] = u[2];
  }
};

template <>
struct PT<float> {
  static constexpr bool kStaged = true;
  using Word = uint32_t;
  static constexpr int kWords = 6;  // cell ox oy ux uy uz
  // global slot g <-> LDS slot s; arrays st words apart in LDS
  __device__ static void g2l(const Particles<float> &p, uint32_t g, Word *sp,
                             int s, int st, int dims) {
    sp[s] = p.cell[g];
    sp[st + s] = __float_as_uint(p.ox[g]);
    if (dims == 2) sp[2 * st + s] = __float_as_uint(p.oy[g]);
    sp[3 * st + s] = __float_as_uint(p.ux[g]);
    sp[4 * st + s] = __float_as_uint(p.uy[g]);
    sp[5 * st + s] = __float_as_uint(p.uz[g]);
  }
  __device__ static void l2g(const Particles<float> &p, uint32_t g,
                             const Word *sp, int s, int st, int dims) {
    p.cell[g] = sp[s];
    p.ox[g] = __uint_as_float(sp[st + s]);
    if (dims == 2) p.oy[g] = __uint_as_float(sp[2 * st + s]);
    p.ux[g] = __uint_as_float(sp[3 * st + s]);
    p.uy[g] = __uint_as_float(sp[4 * st + s]);
    p.uz[g] = __uint_as_float(sp[5 * st + s]);
  }
  // g2l in two halves: the slot's words into registers, then into LDS
  __device__ static void fetch_words(const Particles<float> &p, uint32_t g,
                                     int dims, Word w[kWords]) {
    w[0] = p.cell[g];
    w[1] = __float_as_uint(p.ox[g]);
    w[2] = dims == 2 ? __float_as_uint(p.oy[g]) : 0u;
    w[3] = __float_as_uint(p.ux[g]);
    w[4] = __float_as_uint(p.uy[g]);
    w[5] = __float_as_uint(p.uz[g]);
  }
  __device__ static void put_words(Word *sp, int s, int st, const Word w[kWords],
                                   int dims) {
    sp[s] = w[0];
    sp[st + s] = w[1];
    if (dims == 2) sp[2 * st + s] = w[2];
    sp[3 * st + s] = w[3];
    sp[4 * st + s] = w[4];
    sp[5 * st + s] = w[5];
  }
  // Unpack LDS slot s (stride st between arrays); false if removed.
  __device__ static bool unpack(const Word *sp, int s, int st, int dims,
                                int &ix, int &iy, float &fx, float &fy,
                                float u[3]) {
    const uint32_t c = sp[s];
    if (c == kDeadCell) return false;
    ix = (int)(c & 0xFFFFu);
    iy = (int)(c >> 16);
    fx = __uint_as_float(sp[st + s]);
    fy = dims == 2 ? __uint_as_float(sp[2 * st + s]) : 0.0f;
    u[0] = __uint_as_float(sp[3 * st + s]);
    u[1] = __uint_as_float(sp[4 * st + s]);
    u[2] = __uint_as_float(sp[5 * st + s]);
    return true;
  }
  __device__ static void pack(Word *sp, int s, int st, int dims, bool alive,
                              int ix, int iy, float fx, float fy,
                              const float u[3]) {
    sp[s] = alive ? ((uint32_t)ix | ((uint32_t)iy << 16)) : kDeadCell;
    sp[st + s] = __float_as_uint(fx);
    if (dims == 2) sp[2 * st + s] = __float_as_uint(fy);
    sp[3 * st + s] = __float_as_uint(u[0]);
    sp[4 * st + s] = __float_as_uint(u[1]);
    sp[5 * st + s] = __float_as_uint(u[2]);
  }
  __device__ static bool load_global(const Particles<float> &p, uint32_t g,
                                     int dims, int &ix, int &iy, float &fx,
                                     float &fy, float u[3]) {
    const uint32_t c = p.cell[g];
    if (c == kDeadCell) return false;
    ix = (int)(c & 0xFFFFu);
    iy = (int)(c >> 16);
    fx = p.ox[g];
    fy = dims == 2 ? p.oy[g] : 0.0f;
    u[0] = p.ux[g];
    u[1] = p.uy[g];
    u[2] = p.uz[g];
    return true;
  }
  __device__ static void store_global(const Particles<float> &p, uint32_t g,
                                      int dims, bool alive, int ix, int iy,
                                      float fx, float fy, const float u[3]) {
    p.cell[g] = alive ? ((uint32_t)ix | ((uint32_t)iy << 16)) : kDeadCell;
    p.ox[g] = fx;
    if (dims == 2) p.oy[g] = fy;
    p.ux[g] = u[0];
    p.uy[g] = u[1];
    p.uz[g] = u[2];
  }
};

// Model a push instantiated with incident source INC is compiled for (0:
// the one IncParams::kind names at run time).
constexpr int inc_kind(int src) {
  return src == 5 ? 1 : (src == 6 ? 2 : (src == 7 ? 3 : 0));
}

// Incident field at a particle for the push instantiated with source INC
// (see IncSource): the Gaussian beam alone, every model, the plane pulse
// and the April beams, or one of those three.
template <int INC>
__device__ __forceinline__ void incident_r(const IncParams &inc, int dims,
                                           double x, double y, double t,
                                           double E[3], double B[3]) {
  if constexpr (INC == 3) {
    E[0] = E[1] = E[2] = B[0] = B[1] = B[2] = 0.0;
    const Gauss2 g = gauss2d_field(inc, dims, x, y, t);
    E[0] = g.ex;
    E[1] = g.ey;
    B[2] = g.ey;
  } else {
    incident_field_t<INC == 4, inc_kind(INC)>(inc, dims, x, y, t, E, B);
  }
}
template <int INC>
__device__ __forceinline__ void incident_r(const IncParams &inc, int dims,
                                           double x, double y, double t,
                                           float E[3], float B[3]) {
  if constexpr (INC == 3) {
    E[0] = E[1] = E[2] = B[0] = B[1] = B[2] = 0.0f;
    const Gauss2 g = gauss2d_field(inc, dims, x, y, t);
    E[0] = (float)g.ex;
    E[1] = (float)g.ey;
    B[2] = (float)g.ey;
  } else {
    incident_field_fp32<INC == 4, inc_kind(INC)>(inc, dims, x, y, t, E, B);
  }
}

// ---------------------------------------------------------------------------
// Esirkepov deposition of one particle on a 4-node frame per axis: S0 and S1
// are the order-2 shapes at x^n and x^{n+1} on the nodes ipx - 2 + ox ..
// ipx + 1 + ox (ipy - 2 + oy .. ipy + 1 + oy), which hold every node either
// shape touches (ox = 1 for a move up the axis, see shapes4); add(c, a, b,
// v) accumulates v into component c at frame node (a, b), i.e. node ipx - 2
// + ox + a (ipy - 2 + oy + b): the caller binds `add` to the frame's first
// node, so each entry's place is that base plus a constant.  Only nodes lo
// .. hi (frame indices), where S0 or S1 is non-zero, are touched, and along
// x (y) only the entries of the running sum that can be non-zero.
// ---------------------------------------------------------------------------
template <typename R, int DIMS, typename Add>
__device__ __forceinline__ void esirkepov(const R S0x[4], const R S1x[4],
                                          const R S0y[4], const R S1y[4],
                                          int lox, int hix, int loy, int hiy,
                                          R cxq, R cyq,
                                          R qvy, R qvz, Add add) {
  // All loops run over the full frame with compile-time indices (the shape
  // arrays stay in registers); nodes outside [lo, hi] are skipped per lane.
  if (DIMS == 1) {
    R acc = R(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      acc += cxq * (S1x[a] - S0x[a]);
      if (a >= lox && a < hix) add(0, a, 0, acc);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      if (a < lox || a > hix) continue;
      const R wv = R(0.5) * (S0x[a] + S1x[a]);
      add(1, a, 0, qvy * wv);
      add(2, a, 0, qvz * wv);
    }
    return;
  }
  // W_x = DSx (S0y + DSy/2), W_y = DSy (S0x + DSx/2),
  // W_z = S0x S0y + DSx S0y/2 + S0x DSy/2 + DSx DSy/3
  //     = S0x (S0y + DSy/2) + DSx (S0y/2 + DSy/3),
  // with the charge factors folded into the per-row / per-column terms.
  R DSx[4], DSy[4], cAy[4], qAy[4], qBy[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    DSx[k] = S1x[k] - S0x[k];
    DSy[k] = S1y[k] - S0y[k];
    const R ay = S0y[k] + R(0.5) * DSy[k];
    cAy[k] = cxq * ay;
    qAy[k] = qvz * ay;
    qBy[k] = qvz * (R(0.5) * S0y[k] + R(1.0 / 3.0) * DSy[k]);
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    if (b < loy || b > hiy) continue;
    R acc = R(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      acc += DSx[a] * cAy[b];
      if (a >= lox && a < hix) add(0, a, b, acc);
    }
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    if (a < lox || a > hix) continue;
    const R cAx = cyq * (S0x[a] + R(0.5) * DSx[a]);
    R acc = R(0);
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      acc += DSy[b] * cAx;
      if (b >= loy && b < hiy) add(1, a, b, acc);
    }
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    if (b < loy || b > hiy) continue;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      if (a < lox || a > hix) continue;
      add(2, a, b, S0x[a] * qAy[b] + DSx[a] * qBy[b]);
    }
  }
}

// Shapes on the 4-node frame of one axis, from the old nearest node ipx,
// the old offset d0 and the new one d1 = xi^{n+1} - ipx.  A move below one
// cell keeps the new nearest node within one of ipx, so the frame ipx - 1
// .. ipx + 2 (o = 1, d1 >= d0) or ipx - 2 .. ipx + 1 (o = 0) holds both
// shapes, each the three order-2 weights about its nearest node (w0 for
// S0); [lo, hi]: the frame nodes either touches.  (Frame node k is node
// ipx - 2 + o + k.)
template <typename R>
__device__ __forceinline__ void shapes4(const R w0[3], R d0, R d1, R S0[4],
                                        R S1[4], int &o, int &lo, int &hi) {
  o = d1 >= d0;
  S0[0] = o ? w0[0] : R(0);
  S0[1] = o ? w0[1] : w0[0];
  S0[2] = o ? w0[2] : w0[1];
  S0[3] = o ? R(0) : w0[2];
  // S1: the three weights about the new nearest node c1 (relative to ipx),
  // found as the next step will find it from the stored cell and offset,
  // so that S1 is that step's S0; its first node c1 - 1 is frame node 0
  // when o - c1 = 1 and frame node 1 when o = c1.
  const R cf = floor(d1), f1 = d1 - cf;
  const R h1 = f1 >= R(0.5) ? R(1) : R(0);
  R w1[3];
  weights3(f1 - h1, w1);
  const bool lead = R(o) - (cf + h1) == R(1);
  S1[0] = lead ? w1[0] : R(0);
  S1[1] = lead ? w1[1] : w1[0];
  S1[2] = lead ? w1[2] : w1[1];
  S1[3] = lead ? R(0) : w1[2];
  lo = (d1 < R(-0.5) ? 0 : 1) - o;
  hi = (d1 > R(0.5) ? 4 : 3) - o;
}

// Order-2 weights of a particle at (cell ix, offset fx): primal weights
// around the nearest node ipx = ix + (fx >= 1/2) and dual weights around the
// dual node of cell ix; returns ipx and sets d0 = offset from ipx.
template <typename R>
__device__ __forceinline__ int node_weights(int ix, R fx, R wp[3], R wd[3],
                                            R &d0) {
  const int h = fx >= R(0.5);
  d0 = fx - R(h);
  weights3(d0, wp);
  weights3(fx - R(0.5), wd);
  return ix + h;
}

// Where the push takes the incident field from: the closed form at each
// particle, the sampled Yee nodes (already in the gathered field), or either
// as IncParams::on_nodes says.  The runtime choice costs the closed form its
// overlap with the gather's loads but frees registers: the FP64 push uses it
// and runs three workgroups per CU (measured faster than two without it);
// the FP32 form and the batches instantiate the fixed choices.
// Where the push takes the incident field from and which models it is built
// for: kIncAtParticle, kIncRuntime -- the plane pulse and the April beams;
// kIncGauss -- the Gaussian beam at the particle; kIncAny -- every model,
// either source (the straggler path); kIncPulse, kIncLP, kIncRP -- one model
// at the particle, fixed at compile time.
enum IncSource {
  kIncAtParticle = 0,
  kIncOnNodes = 1,
  kIncRuntime = 2,
  kIncGauss = 3,
  kIncAny = 4,
  kIncPulse = 5,
  kIncLP = 6,
  kIncRP = 7
};

__device__ __forceinline__ bool inc_at_particle(int src, const IncParams &inc) {
  return src == kIncAtParticle || src == kIncGauss || src >= kIncPulse ||
         ((src == kIncRuntime || src == kIncAny) && !inc.on_nodes);
}

// One particle: gather (via `gather`), incident field, Boris, advance,
// deposit (through frame(ox, oy), which returns the add of esirkepov bound
// to the frame's first node ipx - 2 + ox, ipy - 2 + oy), removal test.
// Position is (cell, offset) per axis.
template <typename R, int DIMS, int INC, typename Gather, typename Frame>
__device__ __forceinline__ bool push_particle(int &ix, int &iy, R &fx, R &fy,
                                              R u[3], const PushParams &pp,
                                              const IncParams &inc,
                                              Gather gather, Frame frame) {
  // The incident field is evaluated before the weights and the gather, so
  // its temporaries are dead by the time those are live (fewer registers at
  // the peak); the sum is the same, scattered plus incident.
  R Ei[3] = {R(0), R(0), R(0)}, Bi[3] = {R(0), R(0), R(0)};
  const bool at_particle = inc_at_particle(INC, inc);
  if (at_particle)  // else the gathered field holds it
    incident_r<INC>(inc, DIMS, ((double)ix + (double)fx) * pp.dx,
               ((double)iy + (double)fy) * pp.dy, pp.time, Ei, Bi);
  R wxp[3], wxd[3], wyp[3] = {R(1), R(0), R(0)}, wyd[3] = {R(1), R(0), R(0)};
  R dx0, dy0 = R(0);
  const int ipx = node_weights(ix, fx, wxp, wxd, dx0);
  const int ipy = (DIMS == 2) ? node_weights(iy, fy, wyp, wyd, dy0) : 0;
  R E[3], B[3];
  gather(ix, iy, ipx, ipy, wxp, wxd, wyp, wyd, E, B);
  if (at_particle) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      E[c] += Ei[c];
      B[c] += Bi[c];
    }
  }
  boris<R>((R)pp.qm, (R)pp.dt, u, E, B);
  const R gi = rsqrt(R(1) + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  // new positions as offsets from the old nearest nodes
  const R d1x = dx0 + (R)(pp.dt * pp.inv_dx) * (u[0] * gi);
  const R d1y = (DIMS == 2) ? dy0 + (R)(pp.dt * pp.inv_dy) * (u[1] * gi) : R(0);
  R S0x[4], S1x[4], S0y[4] = {R(0), R(1), R(0), R(0)},
                    S1y[4] = {R(0), R(1), R(0), R(0)};
  int ox, lox, hix, oy = 0, loy = 1, hiy = 1;
  shapes4(wxp, dx0, d1x, S0x, S1x, ox, lox, hix);
  if (DIMS == 2) shapes4(wyp, dy0, d1y, S0y, S1y, oy, loy, hiy);
  const R qvy = (R)pp.qw * u[1] * gi, qvz = (R)pp.qw * u[2] * gi;
  esirkepov<R, DIMS>(S0x, S1x, S0y, S1y, lox, hix, loy, hiy,
                     (R)(-pp.qw * pp.dx / pp.dt), (R)(-pp.qw * pp.dy / pp.dt),
                     qvy, qvz, frame(ox, oy));
  // A move below one cell keeps |d1| < 2; a non-finite momentum (a
  // simulation gone numerically bad) makes d1 NaN, and such a particle is
  // removed here instead of being given a cell from a NaN.
  const bool finite_move =
      fabs(d1x) < R(4) && (DIMS == 1 || fabs(d1y) < R(4));
  // new cell and offset in [0, 1)
  const R cx1 = finite_move ? floor(d1x) : R(0);
  ix = ipx + (int)cx1;
  fx = finite_move ? d1x - cx1 : R(0);
  if (!(fx < R(1))) fx = one_below<R>();
  if (DIMS == 2) {
    const R cy1 = finite_move ? floor(d1y) : R(0);
    iy = ipy + (int)cy1;
    fy = finite_move ? d1y - cy1 : R(0);
    if (!(fy < R(1))) fy = one_below<R>();
  }
  return finite_move && ix >= 0 && ix < pp.nx &&
         (DIMS == 1 || (iy >= 0 && iy < pp.ny));
}

// ---------------------------------------------------------------------------
// Tiled push
// ---------------------------------------------------------------------------
// One workgroup pushes the particles pbeg .. pend - 1 of one tile (all of
// them, or one work item of a dense tile); smem holds the current window, the
// field window unless the push gathers from global memory, and, on the
// staged path, the particle chunk (push_dyn_lds_bytes).
// GX > 0 fixes the tile at GX x GY cells with slack GS at compile time (it
// must equal tg): the window strides are then constants, and the offsets of
// a particle's gather and deposit taps fold into the LDS instructions.
// SINGLE marks the single-simulation push: it loads the next particle chunk
// while pushing the current one, and in the FP32 form with the incident
// field at the particles it gathers E and Bbar from global memory instead of
// an LDS window (below).
template <typename R, int DIMS, int INC, int PER = kChunkPer, int GX = 0,
          int GY = 0, int GS = 0, bool SINGLE = false>
__device__ __forceinline__ void push_tile(const Fields<R> &f,
                                          const Particles<R> &p,
                                          const TileGeom &tg,
                                          const PushParams &pp,
                                          const IncParams &inc,
                                          uint32_t *strag, uint32_t *n_strag,
                                          int tile, uint32_t pbeg,
                                          uint32_t pend, double *smem) {
  const int TX = GX > 0 ? GX : tg.tx, TY = GX > 0 ? GY : tg.ty;
  const int kSlack = GX > 0 ? GS : tg.slack, kWinExtra = win_extra(kSlack);
  const int kWinLo = kSlack + 2;
  if (pbeg >= pend) return;
  const int cx0 = (tile % tg.ntx) * TX;
  const int cy0 = (DIMS == 2) ? (tile / tg.ntx) * TY : 0;
  const int WX = TX + kWinExtra + (GX > 0 ? fixed_row_pad<R>() : 0);
  const int WY = (DIMS == 2) ? TY + kWinExtra : 1;
  const int WN = WX * WY;
  // jx jy jz windows accumulate in FP64 in both precisions: on gfx950 an
  // FP64 LDS atomic add is several times faster than an FP32 one (the FP32
  // form's push with FP32 windows: 4.7 -> 17.0 ms on the 4096^2 RP run)
  using Acc = double;
  Acc *sj = smem;
  R *sf = (R *)(sj + 3 * WN);  // ex ey ez mx my mz windows
  const int P = f.pitch;

  // Staged path: the words of the first chunk are loaded before the field
  // window, so that their HBM latency overlaps the window loads; a single
  // simulation's push also loads the next chunk while the current one is
  // pushed (SINGLE; the batched push keeps those registers for its fourth
  // workgroup per CU and loads later chunks when it gets there).
  // Thread t holds slots t + 256 j of the chunk (blockDim.x = 256).
  constexpr bool kAhead = PT<R>::kStaged;
  constexpr bool kAheadNext = kAhead && SINGLE;
  constexpr int kAheadWords = 6;  // PT<float>::kWords
  using CK = Chunk<PER>;
  // (the FP32 form interleaves field pairs; the single FP32 push with the
  // incident field at the particles has no field window, see below)
  constexpr bool kPairs = sizeof(R) == 4;
  constexpr bool kFieldGlobal = kPairs && SINGLE && INC != kIncOnNodes;
  // particle chunk after the windows
  uint32_t *sp = (uint32_t *)(sf + (kFieldGlobal ? 0 : 6 * WN));
  uint32_t ahead[kAhead ? PER : 1][kAheadWords];
  auto fetch_chunk = [&](uint32_t c0) {
    if constexpr (kAhead) {
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        const uint32_t g = c0 + threadIdx.x + 256u * (uint32_t)j;
        if (g < pend) PT<R>::fetch_words(p, g, DIMS, ahead[j]);
      }
    }
  };
  auto put_chunk = [&](int cn) {
    if constexpr (kAhead) {
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        const int k = (int)threadIdx.x + 256 * j;
        if (k < cn)
          PT<R>::put_words(sp, chunk_slot<PER>(k), CK::pad, ahead[j], DIMS);
      }
    }
  };
  fetch_chunk(pbeg);

  // stage E^n and Bbar^n on the node window; array index = cx0 + local.
  // The FP32 form interleaves the components that share their taps, Ex
  // with Bbar_y and Ey with Bbar_x, so that one 8-byte LDS read serves both
  // (planes: (Ex, By) pairs, (Ey, Bx) pairs, Ez, Bz); FP64 keeps six planes.
  // The single simulation's FP32 push with the incident field at the
  // particles (kFieldGlobal) stages no field at all: it is bound by its LDS
  // traffic (the current atomics above all) while its vector memory path
  // has room, and the window's few KB per plane stay in the CU's L1 and the
  // XCD's L2, so its gathers read global memory (4096^2 RP push 3.57 ->
  // 3.37 ms; gathering Ez and Bz alone that way 3.45, four components 3.38;
  // the batched push, held to 128 VGPRs, lost 9% with it).
  for (int k = threadIdx.x; k < WN; k += blockDim.x) {
    if constexpr (!kFieldGlobal) {
      const int I = cx0 + k % WX - kSlack + 1;
      const int J = (DIMS == 2) ? cy0 + k / WX - kSlack + 1 : 0;
      const bool in = I >= 0 && I < f.nx_alloc && J >= 0 && J < f.ny_alloc;
      const size_t g = (size_t)J * P + I;
      R ex = in ? f.ex[g] : R(0), ey = in ? f.ey[g] : R(0);
      R mz = in ? f.mz[g] : R(0);
      if (!inc_at_particle(INC, inc) && in) {  // sampled incident field joins
        ex = f.ex[g] + f.iex[g];
        ey = f.ey[g] + f.iey[g];
        mz = f.mz[g] + f.ibz[g];
      }
      const R ez = in ? f.ez[g] : R(0), mx = in ? f.mx[g] : R(0),
              my = in ? f.my[g] : R(0);
      if constexpr (kPairs) {
        sf[2 * k] = ex;
        sf[2 * k + 1] = my;
        sf[2 * WN + 2 * k] = ey;
        sf[2 * WN + 2 * k + 1] = mx;
      } else {
        sf[k] = ex;
        sf[WN + k] = ey;
        sf[3 * WN + k] = mx;
        sf[4 * WN + k] = my;
      }
      sf[(kPairs ? 4 : 2) * WN + k] = ez;
      sf[5 * WN + k] = mz;
    }
    sj[k] = Acc(0);
    sj[WN + k] = Acc(0);
    sj[2 * WN + k] = Acc(0);
  }
  put_chunk((int)min((uint32_t)CK::size, pend - pbeg));
  __syncthreads();

  // gather from the LDS window (window index of node p: p - c0 + kWinLo)
  auto gather = [&](int ix, int iy, int ipx, int ipy, const R wxp[3],
                    const R wxd[3], const R wyp[3], const R wyd[3], R E[3],
                    R B[3]) {
    // first tap (node - 1) at window index node - c0 - 1 + kWinLo
    const int bxp = ipx - cx0 + kWinLo - 1, bxd = ix - cx0 + kWinLo - 1;
    const int byp = (DIMS == 2) ? ipy - cy0 + kWinLo - 1 : 0;
    const int byd = (DIMS == 2) ? iy - cy0 + kWinLo - 1 : 0;
    if constexpr (kFieldGlobal) {
      // array index of window index w: c0 + w - kSlack + 1 (as staged)
      const ptrdiff_t o0 =
          (DIMS == 2 ? (ptrdiff_t)(cy0 - kSlack + 1) * P : 0) +
          (cx0 - kSlack + 1);
      E[0] = gather_plane<R, DIMS>(f.ex + o0, P, bxd, byp, wxd, wyp);
      E[1] = gather_plane<R, DIMS>(f.ey + o0, P, bxp, byd, wxp, wyd);
      E[2] = gather_plane<R, DIMS>(f.ez + o0, P, bxp, byp, wxp, wyp);
      B[0] = (DIMS == 2) ? gather_plane<R, DIMS>(f.mx + o0, P, bxp, byd, wxp,
                                                 wyd)
                         : R(0);
      B[1] = gather_plane<R, DIMS>(f.my + o0, P, bxd, byp, wxd, wyp);
      B[2] = gather_plane<R, DIMS>(f.mz + o0, P, bxd, byd, wxd, wyd);
      return;
    }
    if constexpr (kPairs) {
      gather_pair<R, DIMS>(sf, WX, bxd, byp, wxd, wyp, E[0], B[1]);
      gather_pair<R, DIMS>(sf + 2 * WN, WX, bxp, byd, wxp, wyd, E[1], B[0]);
      if (DIMS == 1) B[0] = R(0);
      E[2] = gather_plane<R, DIMS>(sf + 4 * WN, WX, bxp, byp, wxp, wyp);
    } else {
      E[0] = gather_plane<R, DIMS>(sf, WX, bxd, byp, wxd, wyp);
      E[1] = gather_plane<R, DIMS>(sf + WN, WX, bxp, byd, wxp, wyd);
      E[2] = gather_plane<R, DIMS>(sf + 2 * WN, WX, bxp, byp, wxp, wyp);
      B[0] = (DIMS == 2)
                 ? gather_plane<R, DIMS>(sf + 3 * WN, WX, bxp, byd, wxp, wyd)
                 : R(0);
      B[1] = gather_plane<R, DIMS>(sf + 4 * WN, WX, bxd, byp, wxd, wyp);
    }
    B[2] = gather_plane<R, DIMS>(sf + 5 * WN, WX, bxd, byd, wxd, wyd);
  };

  // One particle at global slot g: a particle more than kSlack cells
  // outside the tile goes to the straggler list (pushed from global memory
  // after this kernel) and returns false with its state untouched;
  // otherwise it is pushed and `alive` tells whether it stays in the box.
  auto push_one = [&](int &ix, int &iy, R &fx, R &fy, R u[3], uint32_t g,
                      bool &alive) -> bool {
    if (!(ix >= cx0 - kSlack && ix < cx0 + TX + kSlack &&
          (DIMS == 1 ||
           (iy >= cy0 - kSlack && iy < cy0 + TY + kSlack)))) {
      strag[atomicAdd(n_strag, 1u)] = g;
      return false;
    }
    const int ipx0 = ix + (fx >= R(0.5));
    const int ipy0 = (DIMS == 2) ? iy + (fy >= R(0.5)) : 0;
    // window index of node ipx - 2, the first deposit node
    const int bx = ipx0 - cx0 + kWinLo - 2;
    const int by = (DIMS == 2) ? ipy0 - cy0 + kWinLo - 2 : 0;
    alive = push_particle<R, DIMS, INC>(
        ix, iy, fx, fy, u, pp, inc, gather, [&](int ox, int oy) {
          Acc *b0 = sj + (by + oy) * WX + bx + ox;
          return [=](int c, int a, int b, R v) {
            atomicAdd(&b0[c * WN + b * WX + a], (Acc)v);
          };
        });
    return true;
  };
  if constexpr (!PT<R>::kStaged) {
    // Straight from HBM: thread t pushes slots pbeg + t, pbeg + t + 256, ...;
    // a wave's 64 lanes read and write 64 consecutive slots, which the sort
    // laid out so that they belong to different cells.  The next slot's
    // words are loaded before the current particle is pushed, so their HBM
    // latency hides behind its arithmetic.
    using Raw = typename PT<R>::Raw;
    uint32_t g = pbeg + threadIdx.x;
    Raw next{};
    if (g < pend) next = PT<R>::fetch(p, g, DIMS);
#pragma unroll 1
    while (g < pend) {
      const Raw cur = next;
      const uint32_t gn = g + blockDim.x;
      if (gn < pend) next = PT<R>::fetch(p, gn, DIMS);
      int ix, iy;
      R fx, fy, u[3];
      bool alive;
      if (PT<R>::decode(cur, DIMS, ix, iy, fx, fy, u) &&
          push_one(ix, iy, fx, fy, u, g, alive))
        PT<R>::store_global(p, g, DIMS, alive, ix, iy, fx, fy, u);
      g = gn;
    }
    __syncthreads();
  } else {
    // Staged: chunks of the cell-sorted range through LDS, pushed in the
    // transposed order of Chunk.
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (uint32_t c0 = pbeg; c0 < pend; c0 += CK::size) {
      const int cn = (int)min((uint32_t)CK::size, pend - c0);
      const bool more = c0 + CK::size < pend;
      if constexpr (kAheadNext) {
        if (more) fetch_chunk(c0 + CK::size);
      } else if (c0 != pbeg) {  // the first chunk is in LDS already
        for (int k = threadIdx.x; k < cn; k += blockDim.x)
          PT<R>::g2l(p, c0 + k, sp, chunk_slot<PER>(k), CK::pad, DIMS);
        __syncthreads();
      }
#pragma unroll 1
      for (int j = 0; j < CK::per; ++j) {
        const int idx = chunk_lane_pos(lane) * CK::stride + wv * CK::per + j;
        if (idx >= cn) continue;
        const int sl = chunk_slot<PER>(idx);
        int ix, iy;
        R fx, fy, u[3];
        bool alive;
        if (!PT<R>::unpack(sp, sl, CK::pad, DIMS, ix, iy, fx, fy, u))
          continue;
        if (push_one(ix, iy, fx, fy, u, c0 + idx, alive))
          PT<R>::pack(sp, sl, CK::pad, DIMS, alive, ix, iy, fx, fy, u);
      }
      __syncthreads();
      // each thread writes back the slots it then refills with the next
      // chunk (its own slots: no barrier between the two)
      for (int k = threadIdx.x; k < cn; k += blockDim.x)
        PT<R>::l2g(p, c0 + k, sp, chunk_slot<PER>(k), CK::pad, DIMS);
      if constexpr (kAheadNext) {
        if (more) put_chunk((int)min((uint32_t)CK::size, pend - c0 - CK::size));
      }
      __syncthreads();
    }
  }
  // add the tile's current window to the grid
  for (int k = threadIdx.x; k < WN; k += blockDim.x) {
    const int I = cx0 + k % WX - kSlack + 1;
    const int J = (DIMS == 2) ? cy0 + k / WX - kSlack + 1 : 0;
    if (I < 0 || I >= f.nx_alloc || J < 0 || J >= f.ny_alloc) continue;
    const size_t g = (size_t)J * P + I;
    const Acc vx = sj[k], vy = sj[WN + k], vz = sj[2 * WN + k];
    if (vx != Acc(0)) unsafeAtomicAdd(&f.jx[g], (R)vx);
    if (vy != Acc(0)) unsafeAtomicAdd(&f.jy[g], (R)vy);
    if (vz != Acc(0)) unsafeAtomicAdd(&f.jz[g], (R)vz);
  }
}

// Work items of the tiled push.  After each sort every non-empty tile is cut
// into items of at most kmax particles, stored as (tile, first particle) in
// tile order: a dense tile (particles bunched by the beam) is shared by
// several workgroups instead of leaving one of them running long after the
// rest, and empty tiles cost nothing.  One workgroup of 1024 threads; each
// thread takes 8 consecutive tiles per pass.
__device__ __forceinline__ void build_items_at(const uint32_t *__restrict__ start,
                                               uint32_t cpt, int ntiles,
                                               uint32_t kmax, uint32_t *items,
                                               uint32_t *n_items,
                                               uint32_t *sh) {
  uint32_t carry = 0;
  for (int t0 = 0; t0 < ntiles; t0 += 8192) {
    const int tb = t0 + (int)threadIdx.x * 8;
    uint32_t tot = 0;
    for (int k = 0; k < 8 && tb + k < ntiles; ++k) {
      const size_t t = (size_t)(tb + k);
      const uint32_t c = start[(t + 1) * cpt] - start[t * cpt];
      tot += (c + kmax - 1) / kmax;
    }
    sh[threadIdx.x] = tot;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const uint32_t add =
          threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0u;
      __syncthreads();
      sh[threadIdx.x] += add;
      __syncthreads();
    }
    uint32_t run = carry + sh[threadIdx.x] - tot;
    for (int k = 0; k < 8 && tb + k < ntiles; ++k) {
      const size_t t = (size_t)(tb + k);
      const uint32_t e = start[(t + 1) * cpt];
      for (uint32_t q = start[t * cpt]; q < e; q += kmax, ++run) {
        items[2 * (size_t)run] = (uint32_t)t;
        items[2 * (size_t)run + 1] = q;
      }
    }
    carry += sh[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) *n_items = carry;
}

__global__ void __launch_bounds__(1024)
build_items(const uint32_t *__restrict__ start, uint32_t cpt, int ntiles,
            uint32_t kmax, uint32_t *items, uint32_t *n_items) {
  __shared__ uint32_t sh[1024];
  build_items_at(start, cpt, ntiles, kmax, items, n_items, sh);
}

// Upper bound of the item count: every tile once plus one per kmax particles.
__host__ __device__ __forceinline__ size_t push_item_capacity(
    const TileGeom &tg, int64_t n_slots, uint32_t kmax) {
  return (size_t)tg.ntiles + (size_t)(n_slots / kmax) + 1;
}

// Resident workgroups per CU asked of the compiler for the single-sim push:
// three for FP64 (its window alone, 52.5 KB for a 16 x 16 tile with slack 3,
// fits three times in the LDS; with the runtime incident choice the kernel
// then spills 20 VGPRs and is still 6% faster than at two), two for the
// FP32 form (its registers allow three anyway; its LDS allows three).
template <typename R>
constexpr int push_min_blocks() {
  return sizeof(R) == 8 ? 3 : SFPIC_PUSH_MIN_BLOCKS;
}

template <typename R, int DIMS, int INC, int GX = 0, int GY = 0, int GS = 0>
__global__ void __launch_bounds__(256, push_min_blocks<R>())
push_tiled(Fields<R> f, Particles<R> p, const uint32_t *__restrict__ start,
           const uint32_t *__restrict__ items,
           const uint32_t *__restrict__ n_items, uint32_t kmax, TileGeom tg,
           PushParams pp, IncParams inc, uint32_t *strag, uint32_t *n_strag) {
  extern __shared__ double smem[];
  // The hardware deals workgroups round-robin to the 8 XCDs; XCD x takes
  // items x*S .. x*S + S - 1 (S = ceil(n / 8)) in order, so neighbouring
  // tiles share halo rows in that XCD's L2.  The grid is sized for the most
  // items a sort can produce; the rest exit at once.
  const uint32_t n = *n_items, S = (n + 7) >> 3, b = blockIdx.x;
  if ((b >> 3) >= S) return;
  const uint32_t it = (b & 7) * S + (b >> 3);
  if (it >= n) return;
  const int tile = (int)items[2 * (size_t)it];
  const uint32_t pbeg = items[2 * (size_t)it + 1];
  const uint32_t tend = start[(size_t)(tile + 1) * tg.cells_per_tile];
  push_tile<R, DIMS, INC, kChunkPer, GX, GY, GS, true>(
      f, p, tg, pp, inc, strag, n_strag, tile, pbeg,
      tend - pbeg > kmax ? pbeg + kmax : tend, smem);
}

// Push of one particle listed by the tiled kernel (drifted more than slack
// cells out of its tile): global gather and global atomics.
template <typename R, int DIMS>
__device__ __forceinline__ void push_straggler(const Fields<R> &f,
                                               const Particles<R> &p,
                                               const PushParams &pp,
                                               const IncParams &inc,
                                               uint32_t ip) {
  const int P = f.pitch;
  auto gather = [&](int ix, int iy, int ipx, int ipy, const R wxp[3],
                    const R wxd[3], const R wyp[3], const R wyd[3], R E[3],
                    R B[3]) {
    const int bxp = ipx - 1 + kGuard, bxd = ix - 1 + kGuard;
    const int byp = (DIMS == 2) ? ipy - 1 + kGuard : 0;
    const int byd = (DIMS == 2) ? iy - 1 + kGuard : 0;
    E[0] = gather_plane<R, DIMS>(f.ex, P, bxd, byp, wxd, wyp);
    E[1] = gather_plane<R, DIMS>(f.ey, P, bxp, byd, wxp, wyd);
    E[2] = gather_plane<R, DIMS>(f.ez, P, bxp, byp, wxp, wyp);
    B[0] = (DIMS == 2) ? gather_plane<R, DIMS>(f.mx, P, bxp, byd, wxp, wyd)
                       : R(0);
    B[1] = gather_plane<R, DIMS>(f.my, P, bxd, byp, wxd, wyp);
    B[2] = gather_plane<R, DIMS>(f.mz, P, bxd, byd, wxd, wyd);
    if (inc.on_nodes) {  // the sampled incident field, same taps
      E[0] += gather_plane<R, DIMS>(f.iex, P, bxd, byp, wxd, wyp);
      E[1] += gather_plane<R, DIMS>(f.iey, P, bxp, byd, wxp, wyd);
      B[2] += gather_plane<R, DIMS>(f.ibz, P, bxd, byd, wxd, wyd);
    }
  };
  int ix, iy;
  R fx, fy, u[3];
  if (!PT<R>::load_global(p, ip, DIMS, ix, iy, fx, fy, u)) return;
  const int ipx0 = ix + (fx >= R(0.5));
  const int ipy0 = (DIMS == 2) ? iy + (fy >= R(0.5)) : 0;
  const int bx = ipx0 - 2 + kGuard;
  const int by = (DIMS == 2) ? ipy0 - 2 + kGuard : 0;
  const bool alive = push_particle<R, DIMS, kIncAny>(
      ix, iy, fx, fy, u, pp, inc, gather, [&](int ox, int oy) {
        const size_t b0 = (size_t)(by + oy) * P + bx + ox;
        return [=, &f](int c, int a, int b, R v) {
          R *jp = c == 0 ? f.jx : (c == 1 ? f.jy : f.jz);
          unsafeAtomicAdd(&jp[b0 + (size_t)b * P + a], v);
        };
      });
  PT<R>::store_global(p, ip, DIMS, alive, ix, iy, fx, fy, u);
}

template <typename R, int DIMS>
__global__ void __launch_bounds__(256)
push_stragglers(Fields<R> f, Particles<R> p, PushParams pp, IncParams inc,
                const uint32_t *strag, const uint32_t *n_strag) {
  const uint32_t n = *n_strag;
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += gridDim.x * blockDim.x)
    push_straggler<R, DIMS>(f, p, pp, inc, strag[k]);
}

template <typename R>
size_t push_dyn_lds_bytes(const TileGeom &tg, int dims, bool batch,
                          bool field_window) {
  const int WX = tg.tx + win_extra(tg.slack) +
                 (!batch && fixed_geometry<R>(tg, dims) ? fixed_row_pad<R>() : 0);
  const int WY = (dims == 2) ? tg.ty + win_extra(tg.slack) : 1;
  size_t b = (size_t)3 * WX * WY * sizeof(double) +
             (field_window ? (size_t)6 * WX * WY * sizeof(R) : 0);
  const int pad = batch ? Chunk<kBatchChunkPer>::pad : Chunk<kChunkPer>::pad;
  if constexpr (PT<R>::kStaged)
    b += (size_t)PT<R>::kWords * pad * sizeof(typename PT<R>::Word);
  return b;
}

// All LDS of the push workgroup (it has no static LDS, so this equals the
// dynamic size; the batched kernel adds a few bytes of its own).
template <typename R>
size_t push_lds_bytes(const TileGeom &tg, int dims, bool batch) {
  return push_dyn_lds_bytes<R>(tg, dims, batch);
}

hipError_t launch_build_items(const uint32_t *start, const TileGeom &tg,
                              uint32_t kmax, uint32_t *items,
                              uint32_t *n_items, hipStream_t st) {
  build_items<<<1, 1024, 0, st>>>(start, tg.cells_per_tile, tg.ntiles, kmax,
                                  items, n_items);
  return hipGetLastError();
}

size_t push_items_words(const TileGeom &tg, int64_t n_slots, uint32_t kmax) {
  return 2 * push_item_capacity(tg, n_slots, kmax);
}

template <typename R>
hipError_t launch_push_tiled(const Fields<R> &f, const Particles<R> &p,
                             const uint32_t *start, const uint32_t *items,
                             const uint32_t *n_items, uint32_t kmax,
                             int64_t n_slots, const TileGeom &tg, int dims,
                             const PushParams &pp, const IncParams &inc,
                             uint32_t *strag, uint32_t *n_strag,
                             hipStream_t st) {
  const size_t cap = push_item_capacity(tg, n_slots, kmax);
  const unsigned nb = (unsigned)((cap + 7) & ~(size_t)7);
  // the FP32 form's push gathers from global memory unless the incident
  // field is sampled on the nodes (push_tile)
  const size_t lds =
      push_dyn_lds_bytes<R>(tg, dims, false, sizeof(R) == 8 || inc.on_nodes);
  fill_u32<<<1, 64, 0, st>>>(n_strag, 0u, 1);
  // the default tile of a 2D run has its geometry compiled in for the
  // April beams (fixed_geometry; the LDS size above includes its row pad)
  constexpr int kFixSlack = fixed_slack<R>();
  const bool fixed = fixed_geometry<R>(tg, dims);
  auto go = [&](auto dims_c, auto inc_c) {
    constexpr int D = decltype(dims_c)::value, I = decltype(inc_c)::value;
    if constexpr (D == 2 && (I == kIncLP || I == kIncRP)) {
      if (fixed) {
        push_tiled<R, D, I, 16, 16, kFixSlack><<<nb, 256, lds, st>>>(
            f, p, start, items, n_items, kmax, tg, pp, inc, strag, n_strag);
        return;
      }
    }
    push_tiled<R, D, I><<<nb, 256, lds, st>>>(f, p, start, items, n_items,
                                              kmax, tg, pp, inc, strag,
                                              n_strag);
  };
  using D1 = std::integral_constant<int, 1>;
  using D2 = std::integral_constant<int, 2>;
  // a push compiled for the one model it evaluates at the particles keeps
  // fewer values live (the scalar registers no longer spill into vector
  // lanes): 4% (FP32 form) and 5% (FP64) faster on the 4096^2 RP run
  const bool one_model = !inc.on_nodes && inc.kind >= 1 && inc.kind <= 3;
  if (inc.kind == 4 && !inc.on_nodes) {  // the Gaussian beam
    using I = std::integral_constant<int, kIncGauss>;
    dims == 1 ? go(D1{}, I{}) : go(D2{}, I{});
  } else if (one_model && inc.kind == 1) {
    using I = std::integral_constant<int, kIncPulse>;
    dims == 1 ? go(D1{}, I{}) : go(D2{}, I{});
  } else if (one_model && inc.kind == 2) {
    using I = std::integral_constant<int, kIncLP>;
    dims == 1 ? go(D1{}, I{}) : go(D2{}, I{});
  } else if (one_model && inc.kind == 3) {
    using I = std::integral_constant<int, kIncRP>;
    dims == 1 ? go(D1{}, I{}) : go(D2{}, I{});
  } else if constexpr (sizeof(R) == 8) {
    using I = std::integral_constant<int, kIncRuntime>;
    dims == 1 ? go(D1{}, I{}) : go(D2{}, I{});
  } else if (inc.on_nodes) {
    using I = std::integral_constant<int, kIncOnNodes>;
    dims == 1 ? go(D1{}, I{}) : go(D2{}, I{});
  } else {
    using I = std::integral_constant<int, kIncAtParticle>;
    dims == 1 ? go(D1{}, I{}) : go(D2{}, I{});
  }
  return hipGetLastError();
}

template <typename R>
hipError_t launch_push_stragglers(const Fields<R> &f, const Particles<R> &p,
                                  int dims, const PushParams &pp,
                                  const IncParams &inc, const uint32_t *strag,
                                  const uint32_t *n_strag, hipStream_t st) {
  if (dims == 1)
    push_stragglers<R, 1><<<512, 256, 0, st>>>(f, p, pp, inc, strag, n_strag);
  else
    push_stragglers<R, 2><<<512, 256, 0, st>>>(f, p, pp, inc, strag, n_strag);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Counting sort by cell.  key = tile * cells_per_tile + cell within tile;
// removed particles and unused slots get key = nkeys and are dropped.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t cell_key(int ix, int iy,
                                             const TileGeom &tg) {
  const int tx = ix / tg.tx, ty = iy / tg.ty;
  return (uint32_t)(ty * tg.ntx + tx) * tg.cells_per_tile +
         (uint32_t)((iy - ty * tg.ty) * tg.tx + (ix - tx * tg.tx));
}

// Ranks within a cell come from atomics on the cell counters.  A wave whose
// lanes share keys (particles in cell order, as placed at creation) elects
// one leader lane per distinct key, which adds the group size and hands out
// consecutive ranks; after a few such rounds the lanes still waiting hold
// mostly distinct keys (the sorted layout puts a wave's lanes in different
// cells) and take their ranks with one atomic each.
__device__ __forceinline__ uint32_t wave_aggregated_rank(bool active,
                                                         uint32_t k,
                                                         uint32_t *counts) {
  const int lane = __lane_id();
  uint64_t pending = __ballot(active);
  uint32_t r = 0;
  for (int round = 0; round < 4 && pending; ++round) {
    const int leader = __ffsll((unsigned long long)pending) - 1;
    const uint32_t kl = __shfl(k, leader, 64);
    const bool mine = active && k == kl;
    const uint64_t same = __ballot(mine);
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(&counts[kl], (uint32_t)__popcll(same));
    base = __shfl(base, leader, 64);
    if (mine) r = base + (uint32_t)__popcll(same & ((1ull << lane) - 1ull));
    pending &= ~same;
  }
  if ((pending >> lane) & 1ull) r = atomicAdd(&counts[k], 1u);
  return r;
}

template <typename R>
__device__ __forceinline__ void sort_count_at(const Particles<R> &p,
                                              uint32_t i, uint32_t n_slots,
                                              uint32_t n_valid,
                                              const TileGeom &tg, int nx,
                                              int ny, int dims,
                                              uint32_t *counts, uint32_t *key,
                                              uint32_t *rank) {
  uint32_t k = tg.nkeys;
  if (i < n_slots && i < n_valid) {
    int ix, iy;
    R fx, fy, u[3];
    if (PT<R>::load_global(p, i, dims, ix, iy, fx, fy, u)) {
      ix = min(max(ix, 0), nx - 1);
      iy = dims == 2 ? min(max(iy, 0), ny - 1) : 0;
      k = cell_key(ix, iy, tg);
    }
  }
  const uint32_t r =
      wave_aggregated_rank(i < n_slots && k < tg.nkeys, k, counts);
  if (i < n_slots) {
    key[i] = k;
    rank[i] = r;
  }
}

template <typename R>
__global__ void sort_count(Particles<R> p, uint32_t n_slots,
                           const uint32_t *n_valid, TileGeom tg, int nx,
                           int ny, int dims, uint32_t *counts, uint32_t *key,
                           uint32_t *rank) {
  sort_count_at<R>(p, blockIdx.x * blockDim.x + threadIdx.x, n_slots,
                   *n_valid, tg, nx, ny, dims, counts, key, rank);
}

__device__ __forceinline__ void move_particle(const Particles<double> &src,
                                              const Particles<double> &dst,
                                              uint32_t i, uint32_t d,
                                              int dims) {
  dst.px[d] = src.px[i];
  if (dims == 2) dst.py[d] = src.py[i];
  dst.ux[d] = src.ux[i];
  dst.uy[d] = src.uy[i];
  dst.uz[d] = src.uz[i];
  dst.id[d] = src.id[i];
}
__device__ __forceinline__ void move_particle(const Particles<float> &src,
                                              const Particles<float> &dst,
                                              uint32_t i, uint32_t d,
                                              int dims) {
  dst.cell[d] = src.cell[i];
  dst.ox[d] = src.ox[i];
  if (dims == 2) dst.oy[d] = src.oy[i];
  dst.ux[d] = src.ux[i];
  dst.uy[d] = src.uy[i];
  dst.uz[d] = src.uz[i];
  dst.id[d] = src.id[i];
}

// Slot of the particle of rank rb within a block of m <= 1024 slots: the
// block is a row-major array of 64 columns (one per lane of the push's
// waves) whose ranks run down the columns, column c holding q + 1 ranks if
// c < r and q otherwise (m = 64 q + r).  In the full rows (row < q) the
// run of ranks c sits in column c / 4 + 16 (c mod 4), so that lane l of the
// wave that pushes the row takes run 4 (l mod 16) + l / 16, as the staged
// path's lanes do (chunk_lane_pos); the last, partial row keeps column c.
// The lanes of a wave are then in different cells and the 16 lanes served
// together 4 runs apart, so their LDS current atomics rarely meet, while
// the wave's loads and stores of its row stay contiguous (against plain
// column order: 4096^2 RP FP64 push 4.57 -> 4.38 ms, sort 1.01 -> 0.75 ms
// per step).
__device__ __forceinline__ uint32_t block_slot(uint32_t rb, uint32_t m) {
  const uint32_t q = m >> 6, r = m & 63u;
  uint32_t c, row;
  if (rb < r * (q + 1)) {
    c = rb / (q + 1);
    row = rb - c * (q + 1);
  } else {
    const uint32_t x = rb - r * (q + 1);
    c = r + x / q;
    row = x - (c - r) * q;
  }
  return row * 64 + (row < q ? (c >> 2) + 16 * (c & 3) : c);
}

// Scatter of slot i to its sorted place: tile-major, cell order within the
// tile; for the unstaged (FP64) path transposed within each block of 1024
// slots from the tile start.
template <typename R>
__device__ __forceinline__ void scatter_at(const Particles<R> &src,
                                           const Particles<R> &dst,
                                           uint32_t i, uint32_t n_slots,
                                           int dims,
                                           const uint32_t *__restrict__ key,
                                           const uint32_t *__restrict__ rank,
                                           const uint32_t *__restrict__ start,
                                           uint32_t nkeys, uint32_t cpt) {
  if (i >= n_slots) return;
  const uint32_t k = key[i];
  if (k >= nkeys) return;
  if constexpr (PT<R>::kStaged) {
    move_particle(src, dst, i, start[k] + rank[i], dims);
  } else {
    const size_t tk = (size_t)(k / cpt) * cpt;
    const uint32_t t0 = start[tk], tn = start[tk + cpt] - t0;
    const uint32_t rt = start[k] + rank[i] - t0;  // rank within the tile
    const uint32_t b0 = rt & ~1023u;
    const uint32_t m = tn - b0 < 1024u ? tn - b0 : 1024u;
    move_particle(src, dst, i, t0 + b0 + block_slot(rt - b0, m), dims);
  }
}

template <typename R>
__global__ void sort_scatter(Particles<R> src, Particles<R> dst,
                             uint32_t n_slots, int dims,
                             const uint32_t *__restrict__ key,
                             const uint32_t *__restrict__ rank,
                             const uint32_t *__restrict__ start,
                             uint32_t nkeys, uint32_t cpt) {
  // The hardware deals workgroups round-robin to the 8 XCDs.  XCD x takes a
  // contiguous band of source blocks, so the particles of one tile, which
  // land in the same destination lines, are written through one L2 and
  // merged there rather than leaving 8 partial copies of each line (the
  // grid is a multiple of 8 blocks).
  const uint32_t b = blockIdx.x, band = gridDim.x >> 3;
  const uint32_t lb = (b & 7) * band + (b >> 3);
  scatter_at<R>(src, dst, lb * blockDim.x + threadIdx.x, n_slots, dims, key,
                rank, start, nkeys, cpt);
}

// Exclusive scan of block lb of a 1024-element segment (256 threads x 4);
// sh is a 256-word LDS array.
__device__ __forceinline__ void scan_block_at(const uint32_t *in,
                                              uint32_t *out, uint32_t *sums,
                                              uint32_t n, uint32_t lb,
                                              uint32_t *sh) {
  const uint32_t base = lb * 1024 + threadIdx.x * 4;
  uint32_t v[4], tot = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0u;
    tot += v[k];
  }
  sh[threadIdx.x] = tot;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    const uint32_t add = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0u;
    __syncthreads();
    sh[threadIdx.x] += add;
    __syncthreads();
  }
  uint32_t run = sh[threadIdx.x] - tot;  // exclusive prefix of this thread
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == 255) sums[lb] = sh[255];
}

__global__ void __launch_bounds__(256)
scan_blocks(const uint32_t *in, uint32_t *out, uint32_t *sums, uint32_t n) {
  __shared__ uint32_t sh[256];
  scan_block_at(in, out, sums, n, blockIdx.x, sh);
}

// In-place exclusive scan of nb block sums by one workgroup of 1024 threads;
// sh is a 1024-word LDS array.
__device__ __forceinline__ void scan_sums_at(uint32_t *sums, uint32_t nb,
                                             uint32_t *sh) {
  uint32_t carry = 0;
  for (uint32_t b0 = 0; b0 < nb; b0 += 1024) {
    const uint32_t i = b0 + threadIdx.x;
    const uint32_t v = i < nb ? sums[i] : 0u;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const uint32_t add =
          threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0u;
      __syncthreads();
      sh[threadIdx.x] += add;
      __syncthreads();
    }
    if (i < nb) sums[i] = carry + sh[threadIdx.x] - v;
    const uint32_t total = sh[1023];
    __syncthreads();
    carry += total;
  }
}

__global__ void __launch_bounds__(1024) scan_sums(uint32_t *sums, uint32_t nb) {
  __shared__ uint32_t sh[1024];
  scan_sums_at(sums, nb, sh);
}

__device__ __forceinline__ void scan_add_at(uint32_t *out,
                                            const uint32_t *sums, uint32_t n,
                                            uint32_t lb) {
  const uint32_t i = lb * 1024 + threadIdx.x;
  const uint32_t add = sums[lb];
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (i + 256 * k < n) out[i + 256 * k] += add;
}

__global__ void scan_add(uint32_t *out, const uint32_t *sums, uint32_t n) {
  scan_add_at(out, sums, n, blockIdx.x);
}

__global__ void set_valid(uint32_t *n_valid, const uint32_t *start,
                          uint32_t nkeys) {
  *n_valid = start[nkeys];
}

template <typename R>
hipError_t launch_sort(const Particles<R> &src, const Particles<R> &dst,
                       uint32_t n_slots, uint32_t *n_valid, uint32_t *start,
                       const TileGeom &tg, int nx, int ny, int dims,
                       const SortScratch &s, hipStream_t st) {
  const uint32_t nk1 = tg.nkeys + 1;
  fill_u32<<<(nk1 + 255) / 256, 256, 0, st>>>(s.counts, 0u, nk1);
  if (n_slots > 0)
    sort_count<R><<<(n_slots + 255) / 256, 256, 0, st>>>(
        src, n_slots, n_valid, tg, nx, ny, dims, s.counts, s.key, s.rank);
  const uint32_t nb = (nk1 + 1023) / 1024;
  scan_blocks<<<nb, 256, 0, st>>>(s.counts, start, s.block_sums, nk1);
  scan_sums<<<1, 1024, 0, st>>>(s.block_sums, nb);
  scan_add<<<nb, 256, 0, st>>>(start, s.block_sums, nk1);
  if (n_slots > 0)
    sort_scatter<R><<<((n_slots + 255) / 256 + 7) & ~7u, 256, 0, st>>>(
        src, dst, n_slots, dims, s.key, s.rank, start, tg.nkeys,
        tg.cells_per_tile);
  set_valid<<<1, 1, 0, st>>>(n_valid, start, tg.nkeys);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *a, uint32_t v, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  fill_u32<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(a, v, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched particle phases.  The push is persistent: `grid` workgroups take
// tiles of all members from one atomic queue (counters[0], cleared by the
// first launch of the step) until the queue is exhausted, so large and small
// members share the chip without a tail per member.  A member whose
// steps_left is 0 is skipped by every phase.
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ PushParams member_params(const BatchView<R> &v,
                                                    const PushJob<R> &J) {
  PushParams pp = J.pp;
  pp.time = (double)v.ms[J.member].step * pp.dt;
  return pp;
}

// APRIL: every push job of the group has an April beam at the particles;
// each tile then runs the push compiled for its member's beam (LP or RP),
// whose registers leave room for more waves than the push built for every
// model and either source (the incident field at the particles or sampled
// on the nodes), which the other groups run.
template <typename R, bool APRIL>
constexpr int batch_push_min_blocks() {
  return (APRIL && sizeof(R) == 4) ? 4 : SFPIC_PUSH_MIN_BLOCKS;
}

template <typename R, int DIMS, bool APRIL>
__global__ void __launch_bounds__(256, (batch_push_min_blocks<R, APRIL>()))
batch_push_kernel(BatchView<R> v) {
  extern __shared__ double smem[];
  __shared__ uint32_t s_item;
  // Items in 8 bands of S = ceil(n / 8), one queue each (counters[2 + np +
  // x]); the hardware deals workgroups to the 8 XCDs round-robin, so
  // workgroup b starts on band b mod 8 -- neighbouring tiles, whose halos
  // overlap, are then pushed by one XCD and meet in its L2 -- and moves on
  // to the next band when its own is exhausted.  The items are the jobs'
  // work items (non-empty tiles, dense ones cut into pieces of at most kmax
  // particles) of the running members, in job order (item_off).
  const uint32_t n = v.item_off[v.np], S = (n + 7) >> 3;
  for (int band = 0; band < 8;) {
    const uint32_t x = (blockIdx.x + (uint32_t)band) & 7u;
    if (threadIdx.x == 0) s_item = atomicAdd(&v.counters[2 + v.np + x], 1u);
    __syncthreads();
    const uint32_t k = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();  // s_item is rewritten only after every thread read it
    const uint32_t item = x * S + k;
    if (k >= S || item >= n) {
      ++band;
      continue;
    }
    const int jb = find_segment(v.item_off, v.np, item);
    const PushJob<R> &J = v.pjobs[jb];
    const PushParams pp = member_params(v, J);
    const uint32_t q = item - v.item_off[jb];
    const int tile = (int)J.items[2 * (size_t)q];
    const uint32_t pb = J.items[2 * (size_t)q + 1];
    const uint32_t tend = J.start[(size_t)(tile + 1) * J.tg.cells_per_tile];
    const uint32_t pe = tend - pb > J.kmax ? pb + J.kmax : tend;
    if constexpr (APRIL) {
      if (J.inc.kind == 3)
        push_tile<R, DIMS, kIncRP, kBatchChunkPer>(
            J.f, J.pa[J.cur], J.tg, pp, J.inc, J.strag, &v.counters[1 + jb],
            tile, pb, pe, smem);
      else
        push_tile<R, DIMS, kIncLP, kBatchChunkPer>(
            J.f, J.pa[J.cur], J.tg, pp, J.inc, J.strag, &v.counters[1 + jb],
            tile, pb, pe, smem);
    } else {
      push_tile<R, DIMS, kIncAny, kBatchChunkPer>(
          J.f, J.pa[J.cur], J.tg, pp, J.inc, J.strag, &v.counters[1 + jb],
          tile, pb, pe, smem);
    }
  }
}

// Prefix of the jobs' item counts (one workgroup of 1024 threads): the jobs
// of members with no steps left contribute none.
template <typename R>
__global__ void __launch_bounds__(1024)
batch_item_offsets(BatchView<R> v) {
  __shared__ uint32_t sh[1024];
  uint32_t carry = 0;
  for (int base = 0; base < v.np; base += 1024) {
    const int j = base + (int)threadIdx.x;
    uint32_t c = 0;
    if (j < v.np) {
      const PushJob<R> &J = v.pjobs[j];
      if (v.ms[J.member].steps_left > 0) c = *J.n_items;
    }
    sh[threadIdx.x] = c;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const uint32_t add =
          threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0u;
      __syncthreads();
      sh[threadIdx.x] += add;
      __syncthreads();
    }
    if (j < v.np) v.item_off[j] = carry + sh[threadIdx.x] - c;
    carry += sh[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) v.item_off[v.np] = carry;
}

// Work items of the jobs sorted this step (one workgroup per job).
template <typename R>
__global__ void __launch_bounds__(1024) batch_build_items(BatchView<R> v) {
  __shared__ uint32_t sh[1024];
  const uint32_t nd = v.counters[1 + v.np];
  for (uint32_t d = blockIdx.x; d < nd; d += gridDim.x) {
    const PushJob<R> &J = v.pjobs[v.due[d]];
    build_items_at(J.start, J.tg.cells_per_tile, J.tg.ntiles, J.kmax, J.items,
                   J.n_items, sh);
  }
}

template <typename R>
hipError_t launch_batch_item_offsets(const BatchView<R> &v, hipStream_t st) {
  if (v.np == 0) return hipSuccess;
  batch_item_offsets<R><<<1, 1024, 0, st>>>(v);
  return hipGetLastError();
}

// Stragglers: a persistent grid; every workgroup takes its share of every
// push job's list, so a member with many stragglers is spread over the
// whole chip.
template <typename R, int DIMS>
__global__ void __launch_bounds__(256) batch_stragglers_kernel(BatchView<R> v) {
  const uint32_t stride = gridDim.x * blockDim.x;
  const uint32_t first = blockIdx.x * blockDim.x + threadIdx.x;
  for (int jb = 0; jb < v.np; ++jb) {
    const PushJob<R> &J = v.pjobs[jb];
    const uint32_t n = v.counters[1 + jb];
    if (n <= blockIdx.x * blockDim.x) continue;
    if (v.ms[J.member].steps_left <= 0) continue;
    const PushParams pp = member_params(v, J);
    const Particles<R> p = J.pa[J.cur];
    for (uint32_t k = first; k < n; k += stride)
      push_straggler<R, DIMS>(J.f, p, pp, J.inc, J.strag[k]);
  }
}

template <typename R>
hipError_t launch_batch_push(const BatchView<R> &v, int dims, bool april,
                             size_t lds, int grid, hipStream_t st) {
  if (v.np == 0) return hipSuccess;
  if (dims == 1)
    batch_push_kernel<R, 1, false><<<grid, 256, lds, st>>>(v);
  else if (april)
    batch_push_kernel<R, 2, true><<<grid, 256, lds, st>>>(v);
  else
    batch_push_kernel<R, 2, false><<<grid, 256, lds, st>>>(v);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_batch_stragglers(const BatchView<R> &v, int dims,
                                   hipStream_t st) {
  if (v.np == 0) return hipSuccess;
  const unsigned g = 2048;
  if (dims == 1)
    batch_stragglers_kernel<R, 1><<<g, 256, 0, st>>>(v);
  else
    batch_stragglers_kernel<R, 2><<<g, 256, 0, st>>>(v);
  return hipGetLastError();
}

template <typename R>
static int push_blocks_per_cu(int dims, bool april, size_t lds) {
  int nb = 0;
  const hipError_t e =
      dims == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                      &nb, batch_push_kernel<R, 1, false>, 256, lds)
      : april   ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                      &nb, batch_push_kernel<R, 2, true>, 256, lds)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                      &nb, batch_push_kernel<R, 2, false>, 256, lds);
  return e == hipSuccess ? nb : 0;
}

int batch_push_blocks_per_cu(bool fp64, int dims, bool april, size_t lds) {
  return fp64 ? push_blocks_per_cu<double>(dims, april, lds)
              : push_blocks_per_cu<float>(dims, april, lds);
}

// Batched counting sort: the same five passes as launch_sort, each one
// persistent launch that walks the push jobs the step's advance kernel
// listed as due (usually none or a few), sharing each job's blocks among
// its workgroups.  A step without sorts costs a handful of empty launches.
#define SFPIC_FOR_DUE(v, J, nblk, lb)                                  \
  for (uint32_t d_ = 0, nd_ = v.counters[1 + v.np]; d_ < nd_; ++d_)    \
    for (const PushJob<R> *J = &v.pjobs[v.due[d_]]; J; J = nullptr)    \
      for (uint32_t lb = blockIdx.x, nb_ = (nblk); lb < nb_;           \
           lb += gridDim.x)

template <typename R>
__global__ void __launch_bounds__(256) batch_sort_clear(BatchView<R> v) {
  SFPIC_FOR_DUE(v, J, (J->tg.nkeys + 1 + 255) / 256, lb) {
    const uint32_t i = lb * 256 + threadIdx.x;
    if (i <= J->tg.nkeys) J->ss.counts[i] = 0u;
  }
}

template <typename R>
__global__ void __launch_bounds__(256) batch_sort_count(BatchView<R> v,
                                                        int dims) {
  SFPIC_FOR_DUE(v, J, (J->n_slots + 255) / 256, lb) {
    sort_count_at<R>(J->pa[J->cur], lb * 256 + threadIdx.x, J->n_slots,
                     *J->n_valid, J->tg, J->pp.nx, J->pp.ny, dims,
                     J->ss.counts, J->ss.key, J->ss.rank);
  }
}

template <typename R>
__global__ void __launch_bounds__(256) batch_scan_blocks(BatchView<R> v) {
  __shared__ uint32_t sh[256];
  SFPIC_FOR_DUE(v, J, (J->tg.nkeys + 1 + 1023) / 1024, lb) {
    scan_block_at(J->ss.counts, J->start, J->ss.block_sums, J->tg.nkeys + 1,
                  lb, sh);
    __syncthreads();  // sh is reused by the next block of the loop
  }
}

template <typename R>
__global__ void __launch_bounds__(1024) batch_scan_sums(BatchView<R> v) {
  __shared__ uint32_t sh[1024];
  const uint32_t nd = v.counters[1 + v.np];
  for (uint32_t d = blockIdx.x; d < nd; d += gridDim.x) {
    const PushJob<R> &J = v.pjobs[v.due[d]];
    scan_sums_at(J.ss.block_sums, (J.tg.nkeys + 1 + 1023) / 1024, sh);
    __syncthreads();
  }
}

template <typename R>
__global__ void __launch_bounds__(256) batch_scan_add(BatchView<R> v) {
  SFPIC_FOR_DUE(v, J, (J->tg.nkeys + 1 + 1023) / 1024, lb) {
    scan_add_at(J->start, J->ss.block_sums, J->tg.nkeys + 1, lb);
  }
}

template <typename R>
__global__ void __launch_bounds__(256) batch_sort_scatter(BatchView<R> v,
                                                          int dims) {
  SFPIC_FOR_DUE(v, J, (J->n_slots + 255) / 256, lb) {
    scatter_at<R>(J->pa[J->cur], J->pa[J->cur ^ 1], lb * 256 + threadIdx.x,
                  J->n_slots, dims, J->ss.key, J->ss.rank, J->start,
                  J->tg.nkeys, J->tg.cells_per_tile);
  }
}

// Slots in use after the sort, and the sorted set becomes current.
template <typename R>
__global__ void batch_sort_finish(BatchView<R> v) {
  const uint32_t d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= v.counters[1 + v.np]) return;
  PushJob<R> &J = v.pjobs[v.due[d]];
  *J.n_valid = J.start[J.tg.nkeys];
  J.cur ^= 1;
}

#undef SFPIC_FOR_DUE

template <typename R>
hipError_t launch_batch_sort(const BatchView<R> &v, int dims, hipStream_t st) {
  if (v.np == 0) return hipSuccess;
  const unsigned g = 2048;
  batch_sort_clear<R><<<g, 256, 0, st>>>(v);
  batch_sort_count<R><<<g, 256, 0, st>>>(v, dims);
  batch_scan_blocks<R><<<g, 256, 0, st>>>(v);
  batch_scan_sums<R><<<(unsigned)(v.np < 256 ? v.np : 256), 1024, 0, st>>>(v);
  batch_scan_add<R><<<g, 256, 0, st>>>(v);
  batch_sort_scatter<R><<<g, 256, 0, st>>>(v, dims);
  batch_sort_finish<R><<<(v.np + 255) / 256, 256, 0, st>>>(v);
  batch_build_items<R><<<(unsigned)(v.np < 256 ? v.np : 256), 1024, 0, st>>>(
      v);
  return hipGetLastError();
}

#define SFPIC_INSTANTIATE(R)                                                 \
  template size_t push_lds_bytes<R>(const TileGeom &, int, bool);            \
  template size_t push_dyn_lds_bytes<R>(const TileGeom &, int, bool, bool);  \
  template hipError_t launch_push_tiled<R>(                                  \
      const Fields<R> &, const Particles<R> &, const uint32_t *,             \
      const uint32_t *, const uint32_t *, uint32_t, int64_t,                 \
      const TileGeom &, int, const PushParams &, const IncParams &,          \
      uint32_t *, uint32_t *, hipStream_t);                                  \
  template hipError_t launch_push_stragglers<R>(                             \
      const Fields<R> &, const Particles<R> &, int, const PushParams &,      \
      const IncParams &, const uint32_t *, const uint32_t *, hipStream_t);   \
  template hipError_t launch_sort<R>(                                        \
      const Particles<R> &, const Particles<R> &, uint32_t, uint32_t *,      \
      uint32_t *, const TileGeom &, int, int, int, const SortScratch &,      \
      hipStream_t);                                                          \
  template hipError_t launch_batch_push<R>(const BatchView<R> &, int, bool,  \
                                           size_t, int, hipStream_t);        \
  template hipError_t launch_batch_stragglers<R>(const BatchView<R> &, int,  \
                                                 hipStream_t);               \
  template hipError_t launch_batch_sort<R>(const BatchView<R> &, int,        \
                                           hipStream_t);                     \
  template hipError_t launch_batch_item_offsets<R>(const BatchView<R> &,     \
                                                   hipStream_t);

SFPIC_INSTANTIATE(double)
SFPIC_INSTANTIATE(float)

}  // namespace sfpic
