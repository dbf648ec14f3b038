// gfx950 kernels of the scattered-field PIC step (Lytova et al., Sec. 2):
// Yee update of the scattered field, order-2 gather, closed-form incident
// field at the particle, Boris push, Esirkepov deposition; plus particle
// placement and FP64 diagnostics.
#include "sfpic_common.h"
#include "sfpic_device.h"

#include <math.h>

namespace sfpic {

// ---------------------------------------------------------------------------
// Yee solver for the scattered field (no incident-field terms: F_inc is a
// vacuum solution and never touches the grid).
// ---------------------------------------------------------------------------

// Faraday: B^{n+1/2} = B^{n-1/2} - dt curl E^n, Bbar^n = average, J = 0.
template <typename R, int DIMS>
__device__ __forceinline__ void faraday_at(const Fields<R> &f, int i, int j,
                                           R cx_, R cy_) {
  const int NX = f.nx_alloc, NY = f.ny_alloc, P = f.pitch;
  if (i >= NX || j >= NY) return;
  const size_t k = (size_t)j * P + i;
  const R bx = f.bx[k], by = f.by[k], bz = f.bz[k];
  R nbx = bx, nby = by, nbz = bz;
  if (DIMS == 1) {
    if (i + 1 < NX) {
      nby = by + cx_ * (f.ez[k + 1] - f.ez[k]);
      nbz = bz - cx_ * (f.ey[k + 1] - f.ey[k]);
    }
  } else {
    if (j + 1 < NY) nbx = bx - cy_ * (f.ez[k + P] - f.ez[k]);
    if (i + 1 < NX) nby = by + cx_ * (f.ez[k + 1] - f.ez[k]);
    if (i + 1 < NX && j + 1 < NY)
      nbz = bz - (cx_ * (f.ey[k + 1] - f.ey[k]) - cy_ * (f.ex[k + P] - f.ex[k]));
  }
  f.bx[k] = nbx;
  f.by[k] = nby;
  f.bz[k] = nbz;
  f.mx[k] = R(0.5) * (bx + nbx);
  f.my[k] = R(0.5) * (by + nby);
  f.mz[k] = R(0.5) * (bz + nbz);
  // the current of this step is accumulated from zero
  f.jx[k] = R(0);
  f.jy[k] = R(0);
  f.jz[k] = R(0);
}

template <typename R, int DIMS>
__global__ void __launch_bounds__(256)
faraday_kernel(Fields<R> f, R cx_, R cy_) {
  faraday_at<R, DIMS>(f, blockIdx.x * blockDim.x + threadIdx.x,
                      blockIdx.y * blockDim.y + threadIdx.y, cx_, cy_);
}

// First-order Mur: face node b, inward neighbour n.
template <typename R>
__device__ __forceinline__ R mur(R n_old, R n_new, R b_old, R k) {
  return n_old + k * (n_new - b_old);
}

// Ampere: E^{n+1} = E^n + dt (curl B^{n+1/2} - J^{n+1/2}).  Each thread owns interior node (i, j), i in [1, NX-2],
// j in [1, NY-2], and also the outer-ring nodes next to it, so the Mur update
// of a face node reads old and new values of its neighbour without a race.
template <typename R, int DIMS>
__device__ __forceinline__ void ampere_at(const Fields<R> &f, int i, int j,
                                          R dt, R cx_, R cy_, R kx, R ky) {
  const int NX = f.nx_alloc, NY = f.ny_alloc, P = f.pitch;
  if (i > NX - 2) return;
  if (DIMS == 2 && j > NY - 2) return;
  if (DIMS == 1) {
    const size_t k = i;
    const R ey_o = f.ey[k], ez_o = f.ez[k];
    f.ex[k] = f.ex[k] - dt * f.jx[k];
    const R ey_n = ey_o + (-cx_ * (f.bz[k] - f.bz[k - 1]) - dt * f.jy[k]);
    const R ez_n = ez_o + (cx_ * (f.by[k] - f.by[k - 1]) - dt * f.jz[k]);
    f.ey[k] = ey_n;
    f.ez[k] = ez_n;
    if (i == 1) {
      f.ex[0] = f.ex[0] - dt * f.jx[0];
      f.ey[0] = mur(ey_o, ey_n, f.ey[0], kx);
      f.ez[0] = mur(ez_o, ez_n, f.ez[0], kx);
    }
    if (i == NX - 2) {
      f.ey[NX - 1] = mur(ey_o, ey_n, f.ey[NX - 1], kx);
      f.ez[NX - 1] = mur(ez_o, ez_n, f.ez[NX - 1], kx);
    }
    return;
  }
  const size_t k = (size_t)j * P + i;
  const R ex_o = f.ex[k], ey_o = f.ey[k], ez_o = f.ez[k];
  const R ex_n = ex_o + (cy_ * (f.bz[k] - f.bz[k - P]) - dt * f.jx[k]);
  const R ey_n = ey_o + (-cx_ * (f.bz[k] - f.bz[k - 1]) - dt * f.jy[k]);
  const R ez_n = ez_o + (cx_ * (f.by[k] - f.by[k - 1]) -
                         cy_ * (f.bx[k] - f.bx[k - P]) - dt * f.jz[k]);
  f.ex[k] = ex_n;
  f.ey[k] = ey_n;
  f.ez[k] = ez_n;

  // Column 0 (x face) belongs to i == 1, column NX-1 to i == NX-2.
  R exl_o = R(0), exl_n = R(0);  // Ex(0, j): ordinary dual-x node
  if (i == 1) {
    const size_t kb = (size_t)j * P;
    exl_o = f.ex[kb];
    exl_n = exl_o + (cy_ * (f.bz[kb] - f.bz[kb - P]) - dt * f.jx[kb]);
    f.ex[kb] = exl_n;
    f.ey[kb] = mur(ey_o, ey_n, f.ey[kb], kx);
    f.ez[kb] = mur(ez_o, ez_n, f.ez[kb], kx);
  }
  if (i == NX - 2) {
    const size_t kb = (size_t)j * P + (NX - 1);
    f.ey[kb] = mur(ey_o, ey_n, f.ey[kb], kx);
    f.ez[kb] = mur(ez_o, ez_n, f.ez[kb], kx);
  }
  // Row 0 (y face) belongs to j == 1, row NY-1 to j == NY-2, together with
  // the corner nodes of that row.
  if (j == 1 || j == NY - 2) {
    const int jb = (j == 1) ? 0 : NY - 1;
    const size_t kb = (size_t)jb * P + i;
    const R eyb_o = f.ey[kb];
    R eyb_n = eyb_o;
    if (jb == 0) {  // Ey(i, 0) is an ordinary dual-y node
      eyb_n = eyb_o + (-cx_ * (f.bz[kb] - f.bz[kb - 1]) - dt * f.jy[kb]);
      f.ey[kb] = eyb_n;
    }
    const R ezb_o = f.ez[kb];
    const R ezb_n = mur(ez_o, ez_n, ezb_o, ky);
    f.ex[kb] = mur(ex_o, ex_n, f.ex[kb], ky);
    f.ez[kb] = ezb_n;
    if (i == 1) {
      const size_t kc = (size_t)jb * P;
      f.ex[kc] = mur(exl_o, exl_n, f.ex[kc], ky);
      if (jb == 0) f.ey[kc] = mur(eyb_o, eyb_n, f.ey[kc], kx);
      f.ez[kc] = mur(ezb_o, ezb_n, f.ez[kc], kx);
    }
    if (i == NX - 2) {
      const size_t kc = (size_t)jb * P + (NX - 1);
      if (jb == 0) f.ey[kc] = mur(eyb_o, eyb_n, f.ey[kc], kx);
      f.ez[kc] = mur(ezb_o, ezb_n, f.ez[kc], kx);
    }
  }
}

template <typename R, int DIMS>
__global__ void __launch_bounds__(256)
ampere_kernel(Fields<R> f, R dt, R cx_, R cy_, R kx, R ky) {
  ampere_at<R, DIMS>(f, blockIdx.x * blockDim.x + threadIdx.x + 1,
                     blockIdx.y * blockDim.y + threadIdx.y + (DIMS == 2 ? 1 : 0),
                     dt, cx_, cy_, kx, ky);
}

template <typename R>
hipError_t launch_faraday(const Fields<R> &f, int dims, double dt, double dx,
                          double dy, hipStream_t st) {
  if (dims == 1) {
    dim3 b(256, 1), g((f.nx_alloc + 255) / 256, 1);
    faraday_kernel<R, 1><<<g, b, 0, st>>>(f, R(dt / dx), R(0));
  } else {
    dim3 b(64, 4), g((f.nx_alloc + 63) / 64, (f.ny_alloc + 3) / 4);
    faraday_kernel<R, 2><<<g, b, 0, st>>>(f, R(dt / dx), R(dt / dy));
  }
  return hipGetLastError();
}

template <typename R>
hipError_t launch_ampere(const Fields<R> &f, int dims, double dt, double dx,
                         double dy, hipStream_t st) {
  const R kx = R((dt - dx) / (dt + dx)), ky = R((dt - dy) / (dt + dy));
  if (dims == 1) {
    dim3 b(256, 1), g((f.nx_alloc - 2 + 255) / 256, 1);
    ampere_kernel<R, 1><<<g, b, 0, st>>>(f, R(dt), R(dt / dx), R(0), kx, ky);
  } else {
    dim3 b(64, 4), g((f.nx_alloc - 2 + 63) / 64, (f.ny_alloc - 2 + 3) / 4);
    ampere_kernel<R, 2><<<g, b, 0, st>>>(f, R(dt), R(dt / dx), R(dt / dy), kx,
                                          ky);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched Yee sweeps: one launch for all members of a group.  Workgroups of
// 256 threads cover 64 x 4 nodes (2D) or 256 nodes (1D); block b belongs to
// the member whose segment of the block-offset table holds b.
// ---------------------------------------------------------------------------
template <typename R, int DIMS, bool FARADAY>
__global__ void __launch_bounds__(256)
batch_yee_kernel(BatchView<R> v) {
  const uint32_t *off = FARADAY ? v.far_off : v.amp_off;
  const uint32_t b = blockIdx.x;
  const int jb = find_segment(off, v.nf, b);
  const FieldJob<R> &J = v.fjobs[jb];
  if (v.ms[J.member].steps_left <= 0) return;
  const uint32_t lb = b - off[jb];
  const int t = threadIdx.x;
  // interior sweep of Ampere starts at node 1 in each direction
  const int o = FARADAY ? 0 : 1;
  int i, j;
  if (DIMS == 2) {
    const int nbx = (J.f.nx_alloc - 2 * o + 63) / 64;
    i = (int)(lb % nbx) * 64 + (t & 63) + o;
    j = (int)(lb / nbx) * 4 + (t >> 6) + o;
  } else {
    i = (int)lb * 256 + t + o;
    j = 0;
  }
  if (FARADAY) {
    faraday_at<R, DIMS>(J.f, i, j, J.cx, J.cy);
  } else {
    if (i > J.f.nx_alloc - 2 || (DIMS == 2 && j > J.f.ny_alloc - 2)) return;
    ampere_at<R, DIMS>(J.f, i, j, J.dt, J.cx, J.cy, J.kx, J.ky);
  }
}

template <typename R>
hipError_t launch_batch_faraday(const BatchView<R> &v, int dims,
                                hipStream_t st) {
  if (v.n_far == 0) return hipSuccess;
  if (dims == 1)
    batch_yee_kernel<R, 1, true><<<v.n_far, 256, 0, st>>>(v);
  else
    batch_yee_kernel<R, 2, true><<<v.n_far, 256, 0, st>>>(v);
  return hipGetLastError();
}

// The incident field sampled on the Yee nodes at t^n for the members that
// take it from there (IncParams::on_nodes), over the Faraday pass's blocks;
// as incident_nodes_kernel, with the member's time from its device step.
template <typename R, int DIMS>
__global__ void __launch_bounds__(256)
batch_incident_nodes_kernel(BatchView<R> v) {
  const uint32_t b = blockIdx.x;
  const int jb = find_segment(v.far_off, v.nf, b);
  const FieldJob<R> &J = v.fjobs[jb];
  const MemberState &m = v.ms[J.member];
  if (m.steps_left <= 0 || J.njobs == 0) return;
  const PushJob<R> &P = v.pjobs[J.job0];
  if (!P.inc.on_nodes) return;
  const uint32_t lb = b - v.far_off[jb];
  const int t = threadIdx.x;
  int i, j;
  if (DIMS == 2) {
    const int nbx = (J.f.nx_alloc + 63) / 64;
    i = (int)(lb % nbx) * 64 + (t & 63);
    j = (int)(lb / nbx) * 4 + (t >> 6);
  } else {
    i = (int)lb * 256 + t;
    j = 0;
  }
  if (i >= J.f.nx_alloc || j >= J.f.ny_alloc) return;
  const double dx = P.pp.dx, dy = P.pp.dy, time = (double)m.step * P.pp.dt;
  const size_t k = (size_t)j * J.f.pitch + i;
  const double xp = (double)(i - kGuard) * dx;
  const double xd = ((double)(i - kGuard) + 0.5) * dx;
  const double yp = DIMS == 2 ? (double)(j - kGuard) * dy : 0.0;
  const double yd = DIMS == 2 ? ((double)(j - kGuard) + 0.5) * dy : 0.0;
  double E[3], B[3];
  incident_field(P.inc, DIMS, xd, yp, time, E, B);
  J.f.iex[k] = (R)E[0];
  incident_field(P.inc, DIMS, xp, yd, time, E, B);
  J.f.iey[k] = (R)E[1];
  incident_field(P.inc, DIMS, xd, yd, time, E, B);
  J.f.ibz[k] = (R)B[2];
}

template <typename R>
hipError_t launch_batch_incident_nodes(const BatchView<R> &v, int dims,
                                       hipStream_t st) {
  if (v.n_far == 0) return hipSuccess;
  if (dims == 1)
    batch_incident_nodes_kernel<R, 1><<<v.n_far, 256, 0, st>>>(v);
  else
    batch_incident_nodes_kernel<R, 2><<<v.n_far, 256, 0, st>>>(v);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_batch_ampere(const BatchView<R> &v, int dims,
                               hipStream_t st) {
  if (v.n_amp == 0) return hipSuccess;
  if (dims == 1)
    batch_yee_kernel<R, 1, false><<<v.n_amp, 256, 0, st>>>(v);
  else
    batch_yee_kernel<R, 2, false><<<v.n_amp, 256, 0, st>>>(v);
  return hipGetLastError();
}

// End of a batched step: advance the step counter of every running member
// and decide whether the sort launches that follow sort it.
template <typename R>
__global__ void batch_advance_kernel(BatchView<R> v, SortRule rule) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= v.nmembers) return;
  MemberState &s = v.ms[m];
  s.sort_due = 0;
  if (s.steps_left <= 0) return;
  s.steps_left -= 1;
  s.step += 1;
  s.since_sort += 1;
  const FieldJob<R> &F = v.fjobs[m];
  if (s.steps_left > 0 && s.since_sort >= rule.c_max) {
    s.sort_due = 1;
    s.since_sort = 0;
    for (int j = F.job0; j < F.job0 + F.njobs; ++j)
      v.due[atomicAdd(&v.counters[1 + v.np], 1u)] = (uint32_t)j;
  }
}

template <typename R>
hipError_t launch_batch_advance(const BatchView<R> &v, SortRule rule,
                                hipStream_t st) {
  if (v.nmembers <= 0) return hipSuccess;
  batch_advance_kernel<R><<<(v.nmembers + 255) / 256, 256, 0, st>>>(v, rule);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Particle placement (Philox4x32-10 counter-based draws, see sfpic_device.h)
// ---------------------------------------------------------------------------
template <typename R>
__global__ void init_particles(Particles<R> p, int64_t n, int dims, int64_t x0,
                               int64_t ncx, int64_t y0, int ppc, double sigma,
                               uint32_t k0, uint32_t k1) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t cell = i / ppc;
  const int64_t cx = x0 + cell % ncx, cy = y0 + cell / ncx;
  uint32_t c[4] = {(uint32_t)i, (uint32_t)((uint64_t)i >> 32), 0u, 0u};
  philox4x32_10(c, k0, k1);
  double a, b;
  u01_pair(c, a, b);
  double ux = 0.0, uy = 0.0, uz = 0.0;
  if (sigma > 0.0) {
    uint32_t c1[4] = {(uint32_t)i, (uint32_t)((uint64_t)i >> 32), 1u, 0u};
    uint32_t c2[4] = {(uint32_t)i, (uint32_t)((uint64_t)i >> 32), 2u, 0u};
    philox4x32_10(c1, k0, k1);
    philox4x32_10(c2, k0, k1);
    double a1, b1, a2, b2;
    u01_pair(c1, a1, b1);
    u01_pair(c2, a2, b2);
    const double r1 = sqrt(-2.0 * log1p(-a1)), r2 = sqrt(-2.0 * log1p(-a2));
    const double tp = 6.283185307179586;
    ux = sigma * r1 * cos(tp * b1);
    uy = sigma * r1 * sin(tp * b1);
    uz = sigma * r2 * cos(tp * b2);
  }
  place(p, i, dims, cx, a, cy, b, ux, uy, uz);
  p.id[i] = (uint32_t)i;
}

template <typename R>
hipError_t launch_init_particles(const Particles<R> &p, int64_t n, int dims,
                                 int64_t x0, int64_t ncx, int64_t y0, int ppc,
                                 double sigma, uint64_t seed, uint32_t key1,
                                 double, double, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  init_particles<R><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(
      p, n, dims, x0, ncx, y0, ppc, sigma, (uint32_t)seed, key1);
  return hipGetLastError();
}

// Placement with a density profile along x: row i / per_row of the region,
// the column whose offsets bracket i % per_row; the draws are those of
// init_particles for the same id.
template <typename R>
__global__ void init_particles_profile(Particles<R> p, int64_t n, int dims,
                                       int64_t x0, int ncx, int64_t y0,
                                       const uint32_t *off, uint32_t per_row,
                                       double sigma, uint32_t k0, uint32_t k1) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t row = i / per_row;
  const uint32_t r = (uint32_t)(i - row * per_row);
  const int64_t cx = x0 + find_segment(off, ncx, r), cy = y0 + row;
  uint32_t c[4] = {(uint32_t)i, (uint32_t)((uint64_t)i >> 32), 0u, 0u};
  philox4x32_10(c, k0, k1);
  double a, b;
  u01_pair(c, a, b);
  double ux = 0.0, uy = 0.0, uz = 0.0;
  if (sigma > 0.0) {
    uint32_t c1[4] = {(uint32_t)i, (uint32_t)((uint64_t)i >> 32), 1u, 0u};
    uint32_t c2[4] = {(uint32_t)i, (uint32_t)((uint64_t)i >> 32), 2u, 0u};
    philox4x32_10(c1, k0, k1);
    philox4x32_10(c2, k0, k1);
    double a1, b1, a2, b2;
    u01_pair(c1, a1, b1);
    u01_pair(c2, a2, b2);
    const double r1 = sqrt(-2.0 * log1p(-a1)), r2 = sqrt(-2.0 * log1p(-a2));
    const double tp = 6.283185307179586;
    ux = sigma * r1 * cos(tp * b1);
    uy = sigma * r1 * sin(tp * b1);
    uz = sigma * r2 * cos(tp * b2);
  }
  place(p, i, dims, cx, a, cy, b, ux, uy, uz);
  p.id[i] = (uint32_t)i;
}

template <typename R>
hipError_t launch_init_particles_profile(const Particles<R> &p, int64_t n,
                                         int dims, int64_t x0, int ncx,
                                         int64_t y0, const uint32_t *off,
                                         uint32_t per_row, double sigma,
                                         uint64_t seed, uint32_t key1,
                                         hipStream_t st) {
  if (n <= 0) return hipSuccess;
  init_particles_profile<R><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(
      p, n, dims, x0, ncx, y0, off, per_row, sigma, (uint32_t)seed, key1);
  return hipGetLastError();
}

// Explicit particles: physical positions to (cell, offset), clamped into
// the physical box [0, nx) x [0, ny) against rounding.
template <typename R>
__global__ void load_particles(Particles<R> p, int64_t n, int dims,
                               const double *x, const double *y,
                               const double *ux, const double *uy,
                               const double *uz, double inv_dx, double inv_dy,
                               int nx, int ny) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double xi = x[i] * inv_dx;
  int64_t cx = (int64_t)floor(xi);
  double fx = xi - (double)cx;
  if (cx >= nx) {
    cx = nx - 1;
    fx = 0.99999999999999989;
  }
  int64_t cy = 0;
  double fy = 0.0;
  if (dims == 2) {
    const double yi = y[i] * inv_dy;
    cy = (int64_t)floor(yi);
    fy = yi - (double)cy;
    if (cy >= ny) {
      cy = ny - 1;
      fy = 0.99999999999999989;
    }
  }
  place(p, i, dims, cx, fx, cy, fy, ux[i], uy[i], uz[i]);
  p.id[i] = (uint32_t)i;
}

template <typename R>
hipError_t launch_load_particles(const Particles<R> &p, int64_t n, int dims,
                                 const double *x, const double *y,
                                 const double *ux, const double *uy,
                                 const double *uz, double inv_dx,
                                 double inv_dy, int nx, int ny,
                                 hipStream_t st) {
  if (n <= 0) return hipSuccess;
  load_particles<R><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(
      p, n, dims, x, y, ux, uy, uz, inv_dx, inv_dy, nx, ny);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64 diagnostics (off the hot path, at the caller's cadence)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double v, double *sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) r += sh[k];
  __syncthreads();
  return r;
}

__device__ __forceinline__ void atomic_max_pos(double *addr, double v) {
  // non-negative doubles order like their bit patterns
  atomicMax((unsigned long long *)addr,
            (unsigned long long)__double_as_longlong(v));
}

template <typename R>
__global__ void particle_sums(Particles<R> p, int64_t n,
                              const uint32_t *n_valid, int dims, double m,
                              double q, double wdv, double *acc) {
  __shared__ double sh[4][8];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double wk = 0.0, ch = 0.0, na = 0.0, bad = 0.0;
  double xi, yi;
  if (i < n && i < (int64_t)*n_valid && pos_of(p, i, dims, xi, yi)) {
    const double ux = p.ux[i], uy = p.uy[i], uz = p.uz[i];
    const double g = sqrt(1.0 + ux * ux + uy * uy + uz * uz);
    if (!isfinite(g)) bad = 1.0;
    wk = wdv * m * (g - 1.0);
    ch = q * wdv;
    na = 1.0;
  }
  wk = block_sum(wk, sh[0]);
  ch = block_sum(ch, sh[1]);
  na = block_sum(na, sh[2]);
  bad = block_sum(bad, sh[3]);
  if (threadIdx.x == 0) {
    unsafeAtomicAdd(&acc[0], wk);
    unsafeAtomicAdd(&acc[1], ch);
    unsafeAtomicAdd(&acc[2], na);
    if (bad > 0.0) unsafeAtomicAdd(&acc[3], bad);
  }
}

template <typename R>
hipError_t launch_particle_sums(const Particles<R> &p, int64_t n,
                                const uint32_t *n_valid, int dims, double m,
                                double q, double wdv, double *acc,
                                hipStream_t st) {
  if (n <= 0) return hipSuccess;
  particle_sums<R><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(
      p, n, n_valid, dims, m, q, wdv, acc);
  return hipGetLastError();
}

template <typename R>
__global__ void field_sums_kernel(Fields<R> f, double *acc) {
  __shared__ double sh[2][8];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  double e = 0.0, bad = 0.0;
  if (i < f.nx_alloc) {
    const size_t k = (size_t)j * f.pitch + i;
    const double v[6] = {(double)f.ex[k], (double)f.ey[k], (double)f.ez[k],
                         (double)f.bx[k], (double)f.by[k], (double)f.bz[k]};
    for (int c = 0; c < 6; ++c) {
      e += 0.5 * v[c] * v[c];
      if (!isfinite(v[c])) bad = 1.0;
    }
  }
  e = block_sum(e, sh[0]);
  bad = block_sum(bad, sh[1]);
  if (threadIdx.x == 0) {
    unsafeAtomicAdd(&acc[4], e);
    if (bad > 0.0) unsafeAtomicAdd(&acc[3], bad);
  }
}

template <typename R>
hipError_t launch_field_sums(const Fields<R> &f, double *acc, hipStream_t st) {
  dim3 g((f.nx_alloc + 255) / 256, f.ny_alloc);
  field_sums_kernel<R><<<g, 256, 0, st>>>(f, acc);
  return hipGetLastError();
}

// Component c (0..5: Ex Ey Ez Bx By Bz) of an (E, B) pair, as a select chain:
// a run-time index into E or B would put both in private memory.
__device__ inline double pick6(int c, const double E[3], const double B[3]) {
  return c == 0   ? E[0]
         : c == 1 ? E[1]
         : c == 2 ? E[2]
         : c == 3 ? B[0]
         : c == 4 ? B[1]
                  : B[2];
}

// Energy of the total field F_inc + F_scatt (Sec. 2) on the physical nodes:
// 1/2 sum |E_s^n + E_inc(t^n)|^2 + |B_s^{n-1/2} + B_inc(t^{n-1/2})|^2 over the
// six components, each taken at the node where the Yee grid stores it, with
// the incident field in FP64.  One thread per node; sum into acc[7].
template <typename R>
__global__ __launch_bounds__(256) void em_total_kernel(Fields<R> f, int dims, int nx, double dx,
                                double dy, double tE, double tB, IncParams inc,
                                double *acc) {
  __shared__ double sh[8];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  double e = 0.0;
  if (i < nx) {
    const size_t k = (size_t)(dims == 2 ? j + kGuard : 0) * f.pitch + i +
                     kGuard;
#pragma unroll 1
    for (int c = 0; c < 6; ++c) {
      // half-cell offsets of Ex Ey Ez Bx By Bz along x and y
      const int hx = c == 0 || c == 4 || c == 5;
      const int hy = c == 1 || c == 3 || c == 5;
      const R *src = c == 0   ? f.ex
                     : c == 1 ? f.ey
                     : c == 2 ? f.ez
                     : c == 3 ? f.bx
                     : c == 4 ? f.by
                              : f.bz;
      const double x = ((double)i + 0.5 * hx) * dx;
      const double y = dims == 2 ? ((double)j + 0.5 * hy) * dy : 0.0;
      double E[3], B[3];
      incident_field(inc, dims, x, y, c < 3 ? tE : tB, E, B);
      const double v = (double)src[k] + pick6(c, E, B);
      e += 0.5 * v * v;
    }
  }
  e = block_sum(e, sh);
  if (threadIdx.x == 0) unsafeAtomicAdd(&acc[7], e);
}

template <typename R>
hipError_t launch_em_total(const Fields<R> &f, int dims, int nx, int ny,
                           double dx, double dy, double tE, double tB,
                           const IncParams &inc, double *acc, hipStream_t st) {
  dim3 g((nx + 255) / 256, dims == 2 ? ny : 1);
  em_total_kernel<R><<<g, 256, 0, st>>>(f, dims, nx, dx, dy, tE, tB, inc, acc);
  return hipGetLastError();
}

// Incident field sampled on the Yee nodes at time t (the field superimposed
// on the grid fields, Sec. 2): E_x on its node (dual in x), E_y on its node
// (dual in y) and B_z on its node (dual in both) for every array element,
// guards included (the push windows reach them); the closed form in FP64.
// In the plane y_paper = 0 the incident models have no other components.
template <typename R>
__global__ void incident_nodes_kernel(Fields<R> f, int dims, double dx,
                                      double dy, double t, IncParams inc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= f.nx_alloc) return;
  const size_t k = (size_t)j * f.pitch + i;
  const double xp = (double)(i - kGuard) * dx;
  const double xd = ((double)(i - kGuard) + 0.5) * dx;
  const double yp = dims == 2 ? (double)(j - kGuard) * dy : 0.0;
  const double yd = dims == 2 ? ((double)(j - kGuard) + 0.5) * dy : 0.0;
  double E[3], B[3];
  incident_field(inc, dims, xd, yp, t, E, B);
  f.iex[k] = (R)E[0];
  incident_field(inc, dims, xp, yd, t, E, B);
  f.iey[k] = (R)E[1];
  incident_field(inc, dims, xd, yd, t, E, B);
  f.ibz[k] = (R)B[2];
}

template <typename R>
hipError_t launch_incident_nodes(const Fields<R> &f, int dims, double dx,
                                 double dy, double t, const IncParams &inc,
                                 hipStream_t st) {
  dim3 g((f.nx_alloc + 255) / 256, f.ny_alloc);
  incident_nodes_kernel<R><<<g, 256, 0, st>>>(f, dims, dx, dy, t, inc);
  return hipGetLastError();
}

// Total field F_scatt + F_inc (Sec. 2) of one stored component, in FP64, at
// every array element (guards included) of a plane of pitch `pitch`: the
// element (i, j) sits at ((i - G) + hx / 2) dx, ((j - G) + hy / 2) dy, where
// hx, hy are 1 for a component staggered by half a cell along that axis; the
// incident field is the FP64 closed form at time t.
template <typename R>
__global__ __launch_bounds__(256) void total_field_kernel(const R *src, int pitch, int NX, int comp,
                                   int hx, int hy, int dims, double dx,
                                   double dy, double t, IncParams inc,
                                   double *dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= NX) return;
  const size_t k = (size_t)j * pitch + i;
  const double x = ((double)(i - kGuard) + 0.5 * hx) * dx;
  const double y =
      dims == 2 ? ((double)(j - kGuard) + 0.5 * hy) * dy : 0.0;
  double E[3], B[3];
  incident_field(inc, dims, x, y, t, E, B);
  dst[k] = (double)src[k] + pick6(comp, E, B);
}

template <typename R>
hipError_t launch_total_field(const R *src, int pitch, int NX, int NY,
                              int comp, int hx, int hy, int dims, double dx,
                              double dy, double t, const IncParams &inc,
                              double *dst, hipStream_t st) {
  dim3 g((NX + 255) / 256, NY);
  total_field_kernel<R><<<g, 256, 0, st>>>(src, pitch, NX, comp, hx, hy, dims,
                                           dx, dy, t, inc, dst);
  return hipGetLastError();
}

template <typename R>
__global__ void deposit_rho(Particles<R> p, int64_t n, const uint32_t *n_valid,
                            int dims, double qw, double *rho, int pitch) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double xi, yi;
  if (i >= n || i >= (int64_t)*n_valid || !pos_of(p, i, dims, xi, yi)) return;
  const int ix = (int)floor(xi);
  const double fx = xi - ix;
  const int hx = fx >= 0.5;
  double wx[3], wy[3] = {1, 0, 0};
  weights3(fx - hx, wx);
  int by = 0;
  if (dims == 2) {
    const int iy = (int)floor(yi);
    const double fy = yi - iy;
    const int hy = fy >= 0.5;
    weights3(fy - hy, wy);
    by = iy + hy - 1 + kGuard;
  }
  const int bx = ix + hx - 1 + kGuard;
  for (int b = 0; b < (dims == 2 ? 3 : 1); ++b)
    for (int a = 0; a < 3; ++a)
      unsafeAtomicAdd(&rho[(size_t)(by + b) * pitch + bx + a],
                      qw * wx[a] * wy[b]);
}

template <typename R>
hipError_t launch_deposit_rho(const Particles<R> &p, int64_t n,
                              const uint32_t *n_valid, int dims, double qw,
                              double *rho, int pitch, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  deposit_rho<R><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(
      p, n, n_valid, dims, qw, rho, pitch);
  return hipGetLastError();
}

// Gauss-law residual |div_h E - (rho - rho0)| at primal nodes at least 4
// cells inside the physical box; acc[5] = max residual, acc[6] = max |rho -
// rho0| there.  The per-node defect g = div_h E - (rho - rho0) is kept in
// gprev; with have_prev the previous call's defect is read first and acc[8]
// = max |g - gprev| is the discrete continuity residual between the two
// calls.  acc[9] = max |rho|.  A non-finite value counts as +inf (fmax would
// drop a NaN).
__device__ __forceinline__ double inf_if_nan(double v) {
  return isnan(v) ? __builtin_huge_val() : v;
}

template <typename R>
__global__ void gauss_kernel(Fields<R> f, int dims, int nx, int ny,
                             double idx, double idy, const double *rho,
                             const double *rho0, int rp, double *gprev,
                             int have_prev, double *acc) {
  // 256 threads: the block takes the maxima first and issues one atomic for
  // each (an atomic per node on two addresses serializes the grid)
  __shared__ double sh[4][4];
  const int i = blockIdx.x * blockDim.x + threadIdx.x + 4;
  const int j = (dims == 2) ? blockIdx.y + 4 : 0;
  double v[4] = {0.0, 0.0, 0.0, 0.0};  // |g|, |rho - rho0|, |dg|, |rho|
  if (i <= nx - 4) {
    const int I = i + kGuard, J = (dims == 2) ? j + kGuard : 0;
    const size_t k = (size_t)J * f.pitch + I;
    double div = ((double)f.ex[k] - (double)f.ex[k - 1]) * idx;
    if (dims == 2) div += ((double)f.ey[k] - (double)f.ey[k - f.pitch]) * idy;
    const size_t kr = (size_t)J * rp + I;
    const double dr = rho[kr] - rho0[kr];
    const double g = div - dr;
    v[0] = inf_if_nan(fabs(g));
    v[1] = inf_if_nan(fabs(dr));
    if (have_prev) v[2] = inf_if_nan(fabs(g - gprev[kr]));
    v[3] = inf_if_nan(fabs(rho[kr]));
    gprev[kr] = g;
  }
  for (int o = 32; o > 0; o >>= 1)
    for (int q = 0; q < 4; ++q) v[q] = fmax(v[q], __shfl_down(v[q], o, 64));
  if ((threadIdx.x & 63) == 0)
    for (int q = 0; q < 4; ++q) sh[q][threadIdx.x >> 6] = v[q];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w)
      for (int q = 0; q < 4; ++q) v[q] = fmax(v[q], sh[q][w]);
    atomic_max_pos(&acc[5], v[0]);
    atomic_max_pos(&acc[6], v[1]);
    atomic_max_pos(&acc[8], v[2]);
    atomic_max_pos(&acc[9], v[3]);
  }
}

template <typename R>
hipError_t launch_gauss(const Fields<R> &f, int dims, int nx, int ny,
                        double dx, double dy, const double *rho,
                        const double *rho0, int rpitch, double *gprev,
                        int have_prev, double *acc, hipStream_t st) {
  if (nx < 9 || (dims == 2 && ny < 9)) return hipSuccess;
  dim3 g((nx - 7 + 255) / 256, dims == 2 ? ny - 7 : 1);
  gauss_kernel<R><<<g, 256, 0, st>>>(f, dims, nx, ny, 1.0 / dx, 1.0 / dy, rho,
                                     rho0, rpitch, gprev, have_prev, acc);
  return hipGetLastError();
}

// The angle from +x that a histogram bins (degrees): polar (plane 0), or
// of the momentum projected on the x-z (1) or x-y (2) plane.
__device__ __forceinline__ double hist_angle(int plane, double ux, double uy,
                                             double uz) {
  const double perp = plane == 1   ? fabs(uz)
                      : plane == 2 ? fabs(uy)
                                   : sqrt(uy * uy + uz * uz);
  return atan2(perp, ux) * (180.0 / 3.14159265358979323846);
}

template <typename R>
__global__ void histogram(Particles<R> p, int64_t n, const uint32_t *n_valid,
                          int dims, double m, double wdv, int n_e, double emax,
                          int n_t, double ek_min, int plane, double *hist,
                          double *mom) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double xi, yi;
  if (i >= n || i >= (int64_t)*n_valid || !pos_of(p, i, dims, xi, yi)) return;
  const double ux = p.ux[i], uy = p.uy[i], uz = p.uz[i];
  const double ek = m * (sqrt(1.0 + ux * ux + uy * uy + uz * uz) - 1.0);
  const double th = hist_angle(plane, ux, uy, uz);
  if (!isfinite(ek) || !isfinite(th)) return;
  const double ie = floor(ek / emax * n_e);
  const double tt = fmin(floor(th / 180.0 * n_t), (double)(n_t - 1));
  if (ie >= 0.0 && ie < (double)n_e && tt >= 0.0)
    unsafeAtomicAdd(&hist[(size_t)ie * n_t + (size_t)tt], wdv);
  if (ek > ek_min) {
    unsafeAtomicAdd(&mom[0], wdv);
    unsafeAtomicAdd(&mom[1], wdv * ek);
    unsafeAtomicAdd(&mom[2], wdv * ek * ek);
    unsafeAtomicAdd(&mom[3], wdv * th);
    unsafeAtomicAdd(&mom[4], wdv * th * th);
  }
}

template <typename R>
hipError_t launch_histogram(const Particles<R> &p, int64_t n,
                            const uint32_t *n_valid, int dims, double m,
                            double wdv, int n_e, double emax, int n_t,
                            double ek_min, int plane, double *hist,
                            double *mom, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  histogram<R><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(
      p, n, n_valid, dims, m, wdv, n_e, emax, n_t, ek_min, plane, hist, mom);
  return hipGetLastError();
}

// Copy the used slots of a particle set out as FP64 physical positions and
// momenta plus ids (removed particles get x = -1).
template <typename R>
__global__ void export_particles(Particles<R> p, int64_t n, int dims,
                                 double dx, double dy, double *out,
                                 uint32_t *ids) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double xi, yi;
  const bool live = pos_of(p, i, dims, xi, yi);
  out[i] = live ? xi * dx : -1.0;
  out[n + i] = live ? yi * dy : 0.0;
  out[2 * n + i] = (double)p.ux[i];
  out[3 * n + i] = (double)p.uy[i];
  out[4 * n + i] = (double)p.uz[i];
  ids[i] = p.id[i];
}

template <typename R>
hipError_t launch_export_particles(const Particles<R> &p, int64_t n, int dims,
                                   double dx, double dy, double *out,
                                   uint32_t *ids, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  export_particles<R><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(
      p, n, dims, dx, dy, out, ids);
  return hipGetLastError();
}

#define SFPIC_INSTANTIATE_K(R)                                                \
  template hipError_t launch_faraday<R>(const Fields<R> &, int, double,       \
                                        double, double, hipStream_t);         \
  template hipError_t launch_ampere<R>(const Fields<R> &, int, double,        \
                                       double, double, hipStream_t);          \
  template hipError_t launch_field_sums<R>(const Fields<R> &, double *,       \
                                           hipStream_t);                      \
  template hipError_t launch_incident_nodes<R>(const Fields<R> &, int, double, \
                                               double, double,                \
                                               const IncParams &,             \
                                               hipStream_t);                  \
  template hipError_t launch_em_total<R>(const Fields<R> &, int, int, int,    \
                                         double, double, double, double,      \
                                         const IncParams &, double *,         \
                                         hipStream_t);                        \
  template hipError_t launch_total_field<R>(const R *, int, int, int, int,  \
                                            int, int, int, double, double,    \
                                            double, const IncParams &,        \
                                            double *, hipStream_t);           \
  template hipError_t launch_gauss<R>(const Fields<R> &, int, int, int,       \
                                      double, double, const double *,         \
                                      const double *, int, double *, int,     \
                                      double *, hipStream_t);                           \
  template hipError_t launch_init_particles<R>(                              \
      const Particles<R> &, int64_t, int, int64_t, int64_t, int64_t, int,     \
      double, uint64_t, uint32_t, double, double, hipStream_t);               \
  template hipError_t launch_init_particles_profile<R>(                      \
      const Particles<R> &, int64_t, int, int64_t, int, int64_t,              \
      const uint32_t *, uint32_t, double, uint64_t, uint32_t, hipStream_t);   \
  template hipError_t launch_load_particles<R>(                              \
      const Particles<R> &, int64_t, int, const double *, const double *,     \
      const double *, const double *, const double *, double, double, int,    \
      int, hipStream_t);                                                      \
  template hipError_t launch_particle_sums<R>(const Particles<R> &, int64_t,  \
                                              const uint32_t *, int, double,  \
                                              double, double, double *,       \
                                              hipStream_t);                   \
  template hipError_t launch_deposit_rho<R>(const Particles<R> &, int64_t,    \
                                            const uint32_t *, int, double,    \
                                            double *, int, hipStream_t);      \
  template hipError_t launch_histogram<R>(                                   \
      const Particles<R> &, int64_t, const uint32_t *, int, double, double,   \
      int, double, int, double, int, double *, double *, hipStream_t);      \
  template hipError_t launch_export_particles<R>(                            \
      const Particles<R> &, int64_t, int, double, double, double *,           \
      uint32_t *, hipStream_t);                                               \
  template hipError_t launch_batch_faraday<R>(const BatchView<R> &, int,      \
                                              hipStream_t);                   \
  template hipError_t launch_batch_ampere<R>(const BatchView<R> &, int,       \
                                             hipStream_t);                    \
  template hipError_t launch_batch_incident_nodes<R>(const BatchView<R> &,    \
                                                     int, hipStream_t);       \
  template hipError_t launch_batch_advance<R>(const BatchView<R> &, SortRule, \
                                              hipStream_t);

SFPIC_INSTANTIATE_K(double)
SFPIC_INSTANTIATE_K(float)

}  // namespace sfpic
