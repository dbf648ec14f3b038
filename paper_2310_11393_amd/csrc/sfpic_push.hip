// Particle side of the step on gfx950: counting sort of particles by cell
// (tile-major key) and the tiled push kernel (order-2 gather, incident field
// at the particle, Boris, Esirkepov deposition; Lytova et al., Sec. 2).
//
// Tiled push: one workgroup per tile of tx x ty cells.  The workgroup stages
// the scattered E and centred B on the tile's node window (tile plus 3 nodes
// below and 4 above in each direction) in LDS, accumulates the tile's current
// in an LDS window of the same shape with LDS atomics, and adds that window to
// the global current once.  Particles are staged through LDS in chunks of
// 1024 and processed in transposed order (lane l takes every 16th particle of
// the cell-sorted chunk), so the 64 lanes of a wave sit in different cells
// and their LDS atomics rarely hit the same address.  A particle that has
// drifted more than one cell out of its tile since the last sort takes the
// global-memory path (global gather, global atomics).
#include "sfpic_common.h"
#include "sfpic_device.h"

namespace sfpic {

constexpr int kChunk = 1024;
constexpr int kChunkPad = kChunk + kChunk / 16;  // one pad word per 16
constexpr int kWinExtra = 7;  // window: nodes c0-3 .. c0+T+3

__global__ void fill_u32(uint32_t *a, uint32_t v, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

__device__ __forceinline__ int chunk_slot(int k) { return k + (k >> 4); }

// Workgroup -> tile: the hardware deals workgroups round-robin to the 8 XCDs;
// giving each XCD a contiguous band of tiles keeps the halo rows that
// neighbouring tiles share in that XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  return (b & 7) * (nb >> 3) + (b >> 3);
}

// ---------------------------------------------------------------------------
// Esirkepov deposition of one particle into planes (jx, jy, jz) with row
// stride `st`; (bx, by) is the index of node (ipx - 2, ipy - 2).  S0 and S1
// are the order-2 shapes at x^n and x^{n+1} on the 5 nodes ipx-2 .. ipx+2.
// Only the nodes where S0 or S1 is non-zero are touched.
// ---------------------------------------------------------------------------
template <typename R, int DIMS, typename Add>
__device__ __forceinline__ void esirkepov(const R S0x[5], const R S1x[5],
                                          const R S0y[5], const R S1y[5],
                                          int lox, int hix, int loy, int hiy,
                                          R cxq, R cyq, R qvy, R qvz, Add add) {
  // All loops run over the full 5-node support with compile-time indices
  // (the shape arrays stay in registers); nodes outside [lo, hi] are skipped.
  if (DIMS == 1) {
    R acc = R(0);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      acc += cxq * (S1x[a] - S0x[a]);
      if (a >= lox && a < hix) add(0, a, 0, acc);
    }
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      if (a < lox || a > hix) continue;
      const R wv = R(0.5) * (S0x[a] + S1x[a]);
      add(1, a, 0, qvy * wv);
      add(2, a, 0, qvz * wv);
    }
    return;
  }
  R DSx[5], DSy[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    DSx[k] = S1x[k] - S0x[k];
    DSy[k] = S1y[k] - S0y[k];
  }
#pragma unroll
  for (int b = 0; b < 5; ++b) {
    if (b < loy || b > hiy) continue;
    const R wyb = S0y[b] + R(0.5) * DSy[b];
    R acc = R(0);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      acc += cxq * (DSx[a] * wyb);
      if (a >= lox && a < hix) add(0, a, b, acc);
    }
  }
#pragma unroll
  for (int a = 0; a < 5; ++a) {
    if (a < lox || a > hix) continue;
    const R wxa = S0x[a] + R(0.5) * DSx[a];
    R acc = R(0);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      acc += cyq * (DSy[b] * wxa);
      if (b >= loy && b < hiy) add(1, a, b, acc);
    }
  }
#pragma unroll
  for (int b = 0; b < 5; ++b) {
    if (b < loy || b > hiy) continue;
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      if (a < lox || a > hix) continue;
      const R wz = S0x[a] * S0y[b] + R(0.5) * DSx[a] * S0y[b] +
                   R(0.5) * S0x[a] * DSy[b] + DSx[a] * DSy[b] * R(1.0 / 3.0);
      add(2, a, b, qvz * wz);
    }
  }
}

// Shapes on the 5-node support: S0 from the three order-2 weights at x^n,
// S1 from the new offset d1 = xi^{n+1} - ipx; the support of S1 is
// [lo, hi] within 0..4.
template <typename R>
__device__ __forceinline__ void shapes5(const R w0[3], R d1, R S0[5], R S1[5],
                                        int &lo, int &hi) {
  S0[0] = R(0);
  S0[1] = w0[0];
  S0[2] = w0[1];
  S0[3] = w0[2];
  S0[4] = R(0);
#pragma unroll
  for (int k = 0; k < 5; ++k) S1[k] = spline2(d1 - R(k - 2));
  lo = d1 < R(-0.5) ? 0 : 1;
  hi = d1 > R(0.5) ? 4 : 3;
}

// ---------------------------------------------------------------------------
// Tiled push, FP64
// ---------------------------------------------------------------------------
template <int DIMS>
__global__ void __launch_bounds__(256, 2)
push_tiled_f64(Fields<double> f, Particles<double> p,
               const uint32_t *__restrict__ start, TileGeom tg, PushParams pp,
               IncParams inc, uint32_t *strag, uint32_t *n_strag) {
  extern __shared__ double smem[];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile >= tg.ntiles) return;
  const uint32_t cpt = tg.cells_per_tile;
  const uint32_t pbeg = start[(size_t)tile * cpt];
  const uint32_t pend = start[(size_t)(tile + 1) * cpt];
  if (pbeg >= pend) return;
  const int cx0 = (tile % tg.ntx) * tg.tx;
  const int cy0 = (DIMS == 2) ? (tile / tg.ntx) * tg.ty : 0;
  const int WX = tg.tx + kWinExtra;
  const int WY = (DIMS == 2) ? tg.ty + kWinExtra : 1;
  const int WN = WX * WY;
  double *sf = smem;          // ex ey ez mx my mz windows
  double *sj = smem + 6 * WN; // jx jy jz windows
  double *sp = sj + 3 * WN;   // particle chunk: px py ux uy uz
  const int P = f.pitch;

  // stage E^n and Bbar^n on the node window; array index = cx0 + local
  for (int k = threadIdx.x; k < WN; k += blockDim.x) {
    const int I = cx0 + k % WX, J = cy0 + k / WX;
    const bool in = I < f.nx_alloc && J < f.ny_alloc;
    const size_t g = (size_t)J * P + I;
    sf[k] = in ? f.ex[g] : 0.0;
    sf[WN + k] = in ? f.ey[g] : 0.0;
    sf[2 * WN + k] = in ? f.ez[g] : 0.0;
    sf[3 * WN + k] = in ? f.mx[g] : 0.0;
    sf[4 * WN + k] = in ? f.my[g] : 0.0;
    sf[5 * WN + k] = in ? f.mz[g] : 0.0;
    sj[k] = 0.0;
    sj[WN + k] = 0.0;
    sj[2 * WN + k] = 0.0;
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const double cxq = -pp.qw * pp.dx / pp.dt;
  const double cyq = -pp.qw * pp.dy / pp.dt;
  for (uint32_t c0 = pbeg; c0 < pend; c0 += kChunk) {
    const int cn = (int)min((uint32_t)kChunk, pend - c0);
    for (int k = threadIdx.x; k < cn; k += blockDim.x) {
      const int s = chunk_slot(k);
      sp[s] = p.px[c0 + k];
      if (DIMS == 2) sp[kChunkPad + s] = p.py[c0 + k];
      sp[2 * kChunkPad + s] = p.ux[c0 + k];
      sp[3 * kChunkPad + s] = p.uy[c0 + k];
      sp[4 * kChunkPad + s] = p.uz[c0 + k];
    }
    __syncthreads();
#pragma unroll 1
    for (int j = 0; j < 4; ++j) {
      const int idx = lane * 16 + wv * 4 + j;
      if (idx >= cn) continue;
      const int s = chunk_slot(idx);
      const double xi = sp[s];
      if (xi < -1.0) continue;  // removed
      const double yi = (DIMS == 2) ? sp[kChunkPad + s] : 0.0;
      const int ix = (int)floor(xi);
      const double fx = xi - ix;
      const int hx = fx >= 0.5;
      const int ipx = ix + hx;
      double wxp[3], wxd[3], wyp[3] = {1, 0, 0}, wyd[3] = {1, 0, 0};
      weights3(fx - hx, wxp);
      weights3(fx - 0.5, wxd);
      int iy = 0, ipy = 0;
      if (DIMS == 2) {
        iy = (int)floor(yi);
        const double fy = yi - iy;
        const int hy = fy >= 0.5;
        ipy = iy + hy;
        weights3(fy - hy, wyp);
        weights3(fy - 0.5, wyd);
      }
      // particles more than one cell outside the tile are pushed later by
      // the straggler kernel, from global memory
      if (!(ix >= cx0 - 1 && ix <= cx0 + tg.tx &&
            (DIMS == 1 || (iy >= cy0 - 1 && iy <= cy0 + tg.ty)))) {
        strag[atomicAdd(n_strag, 1u)] = c0 + idx;
        continue;
      }
      double E[3], B[3];
      {
        // window-local index of the first tap: node - (c0 - 3) - 1
        const int bxp = ipx - cx0 + 2, bxd = ix - cx0 + 2;
        const int byp = (DIMS == 2) ? ipy - cy0 + 2 : 0;
        const int byd = (DIMS == 2) ? iy - cy0 + 2 : 0;
        E[0] = gather_plane<double, DIMS>(sf, WX, bxd, byp, wxd, wyp);
        E[1] = gather_plane<double, DIMS>(sf + WN, WX, bxp, byd, wxp, wyd);
        E[2] = gather_plane<double, DIMS>(sf + 2 * WN, WX, bxp, byp, wxp, wyp);
        B[0] = (DIMS == 2)
                   ? gather_plane<double, DIMS>(sf + 3 * WN, WX, bxp, byd, wxp, wyd)
                   : 0.0;
        B[1] = gather_plane<double, DIMS>(sf + 4 * WN, WX, bxd, byp, wxd, wyp);
        B[2] = gather_plane<double, DIMS>(sf + 5 * WN, WX, bxd, byd, wxd, wyd);
      }
      double Ei[3], Bi[3];
      incident_field(inc, DIMS, xi * pp.dx, yi * pp.dy, pp.time, Ei, Bi);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        E[c] += Ei[c];
        B[c] += Bi[c];
      }
      double u[3] = {sp[2 * kChunkPad + s], sp[3 * kChunkPad + s],
                     sp[4 * kChunkPad + s]};
      boris(pp.qm, pp.dt, u, E, B);
      const double gi =
          1.0 / sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
      const double xi1 = xi + pp.dt * pp.inv_dx * (u[0] * gi);
      const double yi1 =
          (DIMS == 2) ? yi + pp.dt * pp.inv_dy * (u[1] * gi) : 0.0;

      double S0x[5], S1x[5], S0y[5] = {0, 1, 0, 0, 0}, S1y[5] = {0, 1, 0, 0, 0};
      int lox, hix, loy = 1, hiy = 1;
      shapes5(wxp, xi1 - ipx, S0x, S1x, lox, hix);
      if (DIMS == 2) shapes5(wyp, yi1 - ipy, S0y, S1y, loy, hiy);
      const double qvy = pp.qw * u[1] * gi, qvz = pp.qw * u[2] * gi;
      {
        // window-local index of node ipx - 2 is ipx - cx0 + 1
        const int bx = ipx - cx0 + 1, by = (DIMS == 2) ? ipy - cy0 + 1 : 0;
        esirkepov<double, DIMS>(
            S0x, S1x, S0y, S1y, lox, hix, loy, hiy, cxq, cyq, qvy, qvz,
            [&](int c, int a, int b, double v) {
              atomicAdd(&sj[c * WN + (by + b) * WX + bx + a], v);
            });
      }
      const bool inside = (xi1 >= 0.0 && xi1 < (double)pp.nx) &&
                          (DIMS == 1 || (yi1 >= 0.0 && yi1 < (double)pp.ny));
      sp[s] = inside ? xi1 : kDeadPos;
      if (DIMS == 2) sp[kChunkPad + s] = yi1;
      sp[2 * kChunkPad + s] = u[0];
      sp[3 * kChunkPad + s] = u[1];
      sp[4 * kChunkPad + s] = u[2];
    }
    __syncthreads();
    for (int k = threadIdx.x; k < cn; k += blockDim.x) {
      const int s = chunk_slot(k);
      p.px[c0 + k] = sp[s];
      if (DIMS == 2) p.py[c0 + k] = sp[kChunkPad + s];
      p.ux[c0 + k] = sp[2 * kChunkPad + s];
      p.uy[c0 + k] = sp[3 * kChunkPad + s];
      p.uz[c0 + k] = sp[4 * kChunkPad + s];
    }
    __syncthreads();
  }
  // add the tile's current window to the grid
  for (int k = threadIdx.x; k < WN; k += blockDim.x) {
    const int I = cx0 + k % WX, J = cy0 + k / WX;
    if (I >= f.nx_alloc || J >= f.ny_alloc) continue;
    const size_t g = (size_t)J * P + I;
    const double vx = sj[k], vy = sj[WN + k], vz = sj[2 * WN + k];
    if (vx != 0.0) unsafeAtomicAdd(&f.jx[g], vx);
    if (vy != 0.0) unsafeAtomicAdd(&f.jy[g], vy);
    if (vz != 0.0) unsafeAtomicAdd(&f.jz[g], vz);
  }
}

// Push of the particles listed by the tiled kernel (drifted more than one
// cell out of their tile): global gather and global atomics.
template <int DIMS>
__global__ void __launch_bounds__(256)
push_stragglers_f64(Fields<double> f, Particles<double> p, PushParams pp,
                    IncParams inc, const uint32_t *strag,
                    const uint32_t *n_strag) {
  const uint32_t n = *n_strag;
  const int P = f.pitch;
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += gridDim.x * blockDim.x) {
    const uint32_t ip = strag[k];
    const double xi = p.px[ip];
    const double yi = (DIMS == 2) ? p.py[ip] : 0.0;
    const int ix = (int)floor(xi);
    const double fx = xi - ix;
    const int hx = fx >= 0.5;
    const int ipx = ix + hx;
    double wxp[3], wxd[3], wyp[3] = {1, 0, 0}, wyd[3] = {1, 0, 0};
    weights3(fx - hx, wxp);
    weights3(fx - 0.5, wxd);
    int iy = 0, ipy = 0;
    if (DIMS == 2) {
      iy = (int)floor(yi);
      const double fy = yi - iy;
      const int hy = fy >= 0.5;
      ipy = iy + hy;
      weights3(fy - hy, wyp);
      weights3(fy - 0.5, wyd);
    }
    const int bxp = ipx - 1 + kGuard, bxd = ix - 1 + kGuard;
    const int byp = (DIMS == 2) ? ipy - 1 + kGuard : 0;
    const int byd = (DIMS == 2) ? iy - 1 + kGuard : 0;
    double E[3], B[3];
    E[0] = gather_plane<double, DIMS>(f.ex, P, bxd, byp, wxd, wyp);
    E[1] = gather_plane<double, DIMS>(f.ey, P, bxp, byd, wxp, wyd);
    E[2] = gather_plane<double, DIMS>(f.ez, P, bxp, byp, wxp, wyp);
    B[0] = (DIMS == 2) ? gather_plane<double, DIMS>(f.mx, P, bxp, byd, wxp, wyd)
                       : 0.0;
    B[1] = gather_plane<double, DIMS>(f.my, P, bxd, byp, wxd, wyp);
    B[2] = gather_plane<double, DIMS>(f.mz, P, bxd, byd, wxd, wyd);
    double Ei[3], Bi[3];
    incident_field(inc, DIMS, xi * pp.dx, yi * pp.dy, pp.time, Ei, Bi);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      E[c] += Ei[c];
      B[c] += Bi[c];
    }
    double u[3] = {p.ux[ip], p.uy[ip], p.uz[ip]};
    boris(pp.qm, pp.dt, u, E, B);
    const double gi = 1.0 / sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    const double xi1 = xi + pp.dt * pp.inv_dx * (u[0] * gi);
    const double yi1 = (DIMS == 2) ? yi + pp.dt * pp.inv_dy * (u[1] * gi) : 0.0;
    double S0x[5], S1x[5], S0y[5] = {0, 1, 0, 0, 0}, S1y[5] = {0, 1, 0, 0, 0};
    int lox, hix, loy = 1, hiy = 1;
    shapes5(wxp, xi1 - ipx, S0x, S1x, lox, hix);
    if (DIMS == 2) shapes5(wyp, yi1 - ipy, S0y, S1y, loy, hiy);
    const double qvy = pp.qw * u[1] * gi, qvz = pp.qw * u[2] * gi;
    const double cxq = -pp.qw * pp.dx / pp.dt, cyq = -pp.qw * pp.dy / pp.dt;
    const int bx = ipx - 2 + kGuard, by = (DIMS == 2) ? ipy - 2 + kGuard : 0;
    esirkepov<double, DIMS>(
        S0x, S1x, S0y, S1y, lox, hix, loy, hiy, cxq, cyq, qvy, qvz,
        [&](int c, int a, int b, double v) {
          double *jp = c == 0 ? f.jx : (c == 1 ? f.jy : f.jz);
          unsafeAtomicAdd(&jp[(size_t)(by + b) * P + bx + a], v);
        });
    const bool inside = (xi1 >= 0.0 && xi1 < (double)pp.nx) &&
                        (DIMS == 1 || (yi1 >= 0.0 && yi1 < (double)pp.ny));
    p.px[ip] = inside ? xi1 : kDeadPos;
    if (DIMS == 2) p.py[ip] = yi1;
    p.ux[ip] = u[0];
    p.uy[ip] = u[1];
    p.uz[ip] = u[2];
  }
}

template <>
size_t push_lds_bytes<double>(const TileGeom &tg, int dims) {
  const int WX = tg.tx + kWinExtra, WY = (dims == 2) ? tg.ty + kWinExtra : 1;
  return (size_t)(9 * WX * WY + 5 * kChunkPad) * sizeof(double);
}

template <>
hipError_t launch_push_tiled<double>(const Fields<double> &f,
                                     const Particles<double> &p,
                                     const uint32_t *start, const TileGeom &tg,
                                     int dims, const PushParams &pp,
                                     const IncParams &inc, uint32_t *strag,
                                     uint32_t *n_strag, hipStream_t st) {
  const unsigned nb = (unsigned)((tg.ntiles + 7) & ~7);
  const size_t lds = push_lds_bytes<double>(tg, dims);
  fill_u32<<<1, 64, 0, st>>>(n_strag, 0u, 1);
  if (dims == 1)
    push_tiled_f64<1><<<nb, 256, lds, st>>>(f, p, start, tg, pp, inc, strag,
                                            n_strag);
  else
    push_tiled_f64<2><<<nb, 256, lds, st>>>(f, p, start, tg, pp, inc, strag,
                                            n_strag);
  return hipGetLastError();
}

template <>
hipError_t launch_push_stragglers<double>(const Fields<double> &f,
                                          const Particles<double> &p,
                                          int dims, const PushParams &pp,
                                          const IncParams &inc,
                                          const uint32_t *strag,
                                          const uint32_t *n_strag,
                                          hipStream_t st) {
  if (dims == 1)
    push_stragglers_f64<1><<<512, 256, 0, st>>>(f, p, pp, inc, strag, n_strag);
  else
    push_stragglers_f64<2><<<512, 256, 0, st>>>(f, p, pp, inc, strag, n_strag);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Counting sort by cell.  key = tile * cells_per_tile + cell within tile;
// removed particles and unused slots get key = nkeys and are dropped.
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t cell_key(int ix, int iy, const TileGeom &tg) {
  const int tx = ix / tg.tx, ty = iy / tg.ty;
  return (uint32_t)(ty * tg.ntx + tx) * tg.cells_per_tile +
         (uint32_t)((iy - ty * tg.ty) * tg.tx + (ix - tx * tg.tx));
}

__global__ void sort_count_f64(Particles<double> p, uint32_t n_slots,
                               const uint32_t *n_valid, TileGeom tg, int nx,
                               int ny, int dims, uint32_t *counts,
                               uint32_t *key, uint32_t *rank) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_slots) return;
  uint32_t k = tg.nkeys;
  if (i < *n_valid) {
    const double xi = p.px[i];
    if (xi >= -1.0) {
      const int ix = min(max((int)floor(xi), 0), nx - 1);
      const int iy = dims == 2 ? min(max((int)floor(p.py[i]), 0), ny - 1) : 0;
      k = cell_key(ix, iy, tg);
    }
  }
  key[i] = k;
  rank[i] = (k < tg.nkeys) ? atomicAdd(&counts[k], 1u) : 0u;
}

__global__ void sort_scatter_f64(Particles<double> src, Particles<double> dst,
                                 uint32_t n_slots, int dims,
                                 const uint32_t *__restrict__ key,
                                 const uint32_t *__restrict__ rank,
                                 const uint32_t *__restrict__ start,
                                 uint32_t nkeys) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_slots) return;
  const uint32_t k = key[i];
  if (k >= nkeys) return;
  const uint32_t d = start[k] + rank[i];
  dst.px[d] = src.px[i];
  if (dims == 2) dst.py[d] = src.py[i];
  dst.ux[d] = src.ux[i];
  dst.uy[d] = src.uy[i];
  dst.uz[d] = src.uz[i];
  dst.id[d] = src.id[i];
}

// Exclusive scan, 1024 elements per block (256 threads x 4).
__global__ void __launch_bounds__(256)
scan_blocks(const uint32_t *in, uint32_t *out, uint32_t *sums, uint32_t n) {
  __shared__ uint32_t sh[256];
  const uint32_t base = blockIdx.x * 1024 + threadIdx.x * 4;
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
  if (threadIdx.x == 255) sums[blockIdx.x] = sh[255];
}

// In-place exclusive scan of the block sums by one workgroup.
__global__ void __launch_bounds__(1024) scan_sums(uint32_t *sums, uint32_t nb) {
  __shared__ uint32_t sh[1024];
  uint32_t carry = 0;
  for (uint32_t b0 = 0; b0 < nb; b0 += 1024) {
    const uint32_t i = b0 + threadIdx.x;
    const uint32_t v = i < nb ? sums[i] : 0u;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const uint32_t add = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0u;
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

__global__ void scan_add(uint32_t *out, const uint32_t *sums, uint32_t n) {
  const uint32_t i = blockIdx.x * 1024 + threadIdx.x;
  const uint32_t add = sums[blockIdx.x];
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (i + 256 * k < n) out[i + 256 * k] += add;
}

__global__ void set_valid(uint32_t *n_valid, const uint32_t *start,
                          uint32_t nkeys) {
  *n_valid = start[nkeys];
}

template <>
hipError_t launch_sort<double>(const Particles<double> &src,
                               const Particles<double> &dst, uint32_t n_slots,
                               uint32_t *n_valid, uint32_t *start,
                               const TileGeom &tg, int nx, int ny, int dims,
                               const SortScratch &s, hipStream_t st) {
  const uint32_t nk1 = tg.nkeys + 1;
  fill_u32<<<(nk1 + 255) / 256, 256, 0, st>>>(s.counts, 0u, nk1);
  if (n_slots > 0)
    sort_count_f64<<<(n_slots + 255) / 256, 256, 0, st>>>(
        src, n_slots, n_valid, tg, nx, ny, dims, s.counts, s.key, s.rank);
  const uint32_t nb = (nk1 + 1023) / 1024;
  scan_blocks<<<nb, 256, 0, st>>>(s.counts, start, s.block_sums, nk1);
  scan_sums<<<1, 1024, 0, st>>>(s.block_sums, nb);
  scan_add<<<nb, 256, 0, st>>>(start, s.block_sums, nk1);
  if (n_slots > 0)
    sort_scatter_f64<<<(n_slots + 255) / 256, 256, 0, st>>>(
        src, dst, n_slots, dims, s.key, s.rank, start, tg.nkeys);
  set_valid<<<1, 1, 0, st>>>(n_valid, start, tg.nkeys);
  return hipGetLastError();
}

}  // namespace sfpic
