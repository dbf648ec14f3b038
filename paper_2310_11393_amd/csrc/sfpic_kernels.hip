// gfx950 kernels of the scattered-field PIC step (Lytova et al., Sec. 2):
// Yee update of the scattered field, order-2 gather, closed-form incident
// field at the particle, Boris push, Esirkepov deposition; plus particle
// placement and FP64 diagnostics.
#include "sfpic_common.h"

#include <math.h>

namespace sfpic {

// ---------------------------------------------------------------------------
// Yee solver for the scattered field (no incident-field terms: F_inc is a
// vacuum solution and never touches the grid).
// ---------------------------------------------------------------------------

// Faraday: B^{n+1/2} = B^{n-1/2} - dt curl E^n, Bbar^n = average, J = 0.
template <typename R, int DIMS>
__global__ void __launch_bounds__(256)
faraday_kernel(Fields<R> f, R cx_, R cy_) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
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

// First-order Mur: face node b, inward neighbour n.
template <typename R>
__device__ __forceinline__ R mur(R n_old, R n_new, R b_old, R k) {
  return n_old + k * (n_new - b_old);
}

// Ampere: E^{n+1} = E^n + dt (curl B^{n+1/2} - J^{n+1/2}).  Each thread owns interior node (i, j), i in [1, NX-2],
// j in [1, NY-2], and also the outer-ring nodes next to it, so the Mur update
// of a face node reads old and new values of its neighbour without a race.
template <typename R, int DIMS>
__global__ void __launch_bounds__(256)
ampere_kernel(Fields<R> f, R dt, R cx_, R cy_, R kx, R ky) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x + 1;
  const int j = blockIdx.y * blockDim.y + threadIdx.y + (DIMS == 2 ? 1 : 0);
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

// Boris rotation (Boris 1970) of u = gamma v for charge-to-mass ratio qm.
template <typename R>
__device__ __forceinline__ void boris(R qm, R dt, R u[3], const R E[3],
                                      const R B[3]) {
  const R h = R(0.5) * qm * dt;
  const R um0 = u[0] + h * E[0], um1 = u[1] + h * E[1], um2 = u[2] + h * E[2];
  const R gi = R(1) / sqrt(R(1) + um0 * um0 + um1 * um1 + um2 * um2);
  const R t0 = h * B[0] * gi, t1 = h * B[1] * gi, t2 = h * B[2] * gi;
  const R f = R(2) / (R(1) + t0 * t0 + t1 * t1 + t2 * t2);
  const R s0 = f * t0, s1 = f * t1, s2 = f * t2;
  const R up0 = um0 + (um1 * t2 - um2 * t1);
  const R up1 = um1 + (um2 * t0 - um0 * t2);
  const R up2 = um2 + (um0 * t1 - um1 * t0);
  u[0] = um0 + (up1 * s2 - up2 * s1) + h * E[0];
  u[1] = um1 + (up2 * s0 - up0 * s2) + h * E[1];
  u[2] = um2 + (up0 * s1 - up1 * s0) + h * E[2];
}

// ---------------------------------------------------------------------------
// Push: gather + incident field + Boris + advance + Esirkepov deposit.
// One thread per particle; the current goes to the grid by global atomics.
// ---------------------------------------------------------------------------
template <int DIMS>
__global__ void __launch_bounds__(256)
push_kernel_f64(Fields<double> f, Particles<double> p, int64_t n,
                PushParams pp, IncParams inc) {
  const int64_t ip = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ip >= n) return;
  const double xi = p.px[ip];
  if (xi < -1.0) return;  // removed
  const double yi = (DIMS == 2) ? p.py[ip] : 0.0;
  const int P = f.pitch;

  // nearest primal / dual nodes and offsets
  const int ix = (int)floor(xi);
  const double fx = xi - ix;
  const int hx = fx >= 0.5;
  const int ipx = ix + hx;
  const double dpx = fx - hx;
  double wxp[3], wxd[3], wyp[3] = {1, 0, 0}, wyd[3] = {1, 0, 0};
  weights3(dpx, wxp);
  weights3(fx - 0.5, wxd);
  int iy = 0, ipy = 0;
  double dpy = 0.0;
  if (DIMS == 2) {
    iy = (int)floor(yi);
    const double fy = yi - iy;
    const int hy = fy >= 0.5;
    ipy = iy + hy;
    dpy = fy - hy;
    weights3(dpy, wyp);
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

  // incident field at (x^n, t^n), superposed on the scattered field
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

  // Esirkepov: shapes at x^n and x^{n+1} on the 5 nodes around ipx
  double S0x[5], S1x[5];
  S0x[0] = 0.0;
  S0x[1] = wxp[0];
  S0x[2] = wxp[1];
  S0x[3] = wxp[2];
  S0x[4] = 0.0;
  const double d1x = xi1 - ipx;
#pragma unroll
  for (int k = 0; k < 5; ++k) S1x[k] = spline2(d1x - (k - 2));
  double* jx = f.jx;
  double* jy = f.jy;
  double* jz = f.jz;
  if (DIMS == 1) {
    const double cxq = -pp.qw * pp.dx / pp.dt;
    double acc = 0.0;
    const int b0 = ipx - 2 + kGuard;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      acc += cxq * (S1x[k] - S0x[k]);
      if (acc != 0.0) unsafeAtomicAdd(&jx[b0 + k], acc);
    }
    const double qvy = pp.qw * u[1] * gi, qvz = pp.qw * u[2] * gi;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const double wv = 0.5 * (S0x[k] + S1x[k]);
      if (wv != 0.0) {
        unsafeAtomicAdd(&jy[b0 + k], qvy * wv);
        unsafeAtomicAdd(&jz[b0 + k], qvz * wv);
      }
    }
  } else {
    double S0y[5], S1y[5];
    S0y[0] = 0.0;
    S0y[1] = wyp[0];
    S0y[2] = wyp[1];
    S0y[3] = wyp[2];
    S0y[4] = 0.0;
    const double d1y = yi1 - ipy;
#pragma unroll
    for (int k = 0; k < 5; ++k) S1y[k] = spline2(d1y - (k - 2));
    double DSx[5], DSy[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      DSx[k] = S1x[k] - S0x[k];
      DSy[k] = S1y[k] - S0y[k];
    }
    const double cxq = -pp.qw * pp.dx / pp.dt;
    const double cyq = -pp.qw * pp.dy / pp.dt;
    const double qvz = pp.qw * u[2] * gi;
    const int bx0 = ipx - 2 + kGuard, by0 = ipy - 2 + kGuard;
#pragma unroll
    for (int b = 0; b < 5; ++b) {
      const double wyb = S0y[b] + 0.5 * DSy[b];
      double acc = 0.0;
      double *row = jx + (size_t)(by0 + b) * P + bx0;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        acc += cxq * (DSx[a] * wyb);
        if (acc != 0.0) unsafeAtomicAdd(&row[a], acc);
      }
    }
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      const double wxa = S0x[a] + 0.5 * DSx[a];
      double acc = 0.0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        acc += cyq * (DSy[b] * wxa);
        if (acc != 0.0)
          unsafeAtomicAdd(&jy[(size_t)(by0 + b) * P + bx0 + a], acc);
      }
    }
#pragma unroll
    for (int b = 0; b < 5; ++b) {
      double *row = jz + (size_t)(by0 + b) * P + bx0;
#pragma unroll
      for (int a = 0; a < 5; ++a) {
        const double wz = S0x[a] * S0y[b] + 0.5 * DSx[a] * S0y[b] +
                          0.5 * S0x[a] * DSy[b] +
                          DSx[a] * DSy[b] * (1.0 / 3.0);
        if (wz != 0.0) unsafeAtomicAdd(&row[a], qvz * wz);
      }
    }
  }

  p.ux[ip] = u[0];
  p.uy[ip] = u[1];
  p.uz[ip] = u[2];
  const bool inside = (xi1 >= 0.0 && xi1 < (double)pp.nx) &&
                      (DIMS == 1 || (yi1 >= 0.0 && yi1 < (double)pp.ny));
  p.px[ip] = inside ? xi1 : kDeadPos;
  if (DIMS == 2) p.py[ip] = yi1;
}

template <>
hipError_t launch_push<double>(const Fields<double> &f,
                               const Particles<double> &p, int64_t n,
                               int dims, const PushParams &pp,
                               const IncParams &inc, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int bs = 256;
  const unsigned g = (unsigned)((n + bs - 1) / bs);
  if (dims == 1)
    push_kernel_f64<1><<<g, bs, 0, st>>>(f, p, n, pp, inc);
  else
    push_kernel_f64<2><<<g, bs, 0, st>>>(f, p, n, pp, inc);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Particle placement: Philox4x32-10 (Salmon et al., SC'11) keyed by
// (seed, species index), counter (id low, id high, stream, 0).
// ---------------------------------------------------------------------------
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

__global__ void init_particles_f64(Particles<double> p, int64_t n, int dims,
                                   int64_t x0, int64_t ncx, int64_t y0,
                                   int ppc, double sigma, uint32_t k0,
                                   uint32_t k1) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t cell = i / ppc;
  const int64_t cx = x0 + cell % ncx, cy = y0 + cell / ncx;
  uint32_t c[4] = {(uint32_t)i, (uint32_t)((uint64_t)i >> 32), 0u, 0u};
  philox4x32_10(c, k0, k1);
  double a, b;
  u01_pair(c, a, b);
  p.px[i] = (double)cx + a;
  if (dims == 2) p.py[i] = (double)cy + b;
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
  p.ux[i] = ux;
  p.uy[i] = uy;
  p.uz[i] = uz;
  p.id[i] = (uint32_t)i;
}

template <>
hipError_t launch_init_particles<double>(const Particles<double> &p,
                                         int64_t n, int dims, int64_t x0,
                                         int64_t ncx, int64_t y0, int ppc,
                                         double sigma, uint64_t seed,
                                         uint32_t key1, double, double,
                                         hipStream_t st) {
  if (n <= 0) return hipSuccess;
  init_particles_f64<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(
      p, n, dims, x0, ncx, y0, ppc, sigma, (uint32_t)seed, key1);
  return hipGetLastError();
}

__global__ void load_particles_f64(Particles<double> p, int64_t n, int dims,
                                   const double *x, const double *y,
                                   const double *ux, const double *uy,
                                   const double *uz, double inv_dx,
                                   double inv_dy) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  p.px[i] = x[i] * inv_dx;
  if (dims == 2) p.py[i] = y[i] * inv_dy;
  p.ux[i] = ux[i];
  p.uy[i] = uy[i];
  p.uz[i] = uz[i];
  p.id[i] = (uint32_t)i;
}

template <>
hipError_t launch_load_particles<double>(const Particles<double> &p,
                                         int64_t n, int dims, const double *x,
                                         const double *y, const double *ux,
                                         const double *uy, const double *uz,
                                         double inv_dx, double inv_dy,
                                         hipStream_t st) {
  if (n <= 0) return hipSuccess;
  load_particles_f64<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(
      p, n, dims, x, y, ux, uy, uz, inv_dx, inv_dy);
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
  atomicMax((unsigned long long *)addr, (unsigned long long)__double_as_longlong(v));
}

__global__ void particle_sums_f64(Particles<double> p, int64_t n, double m,
                                  double q, double wdv, double *acc) {
  __shared__ double sh[4][8];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double wk = 0.0, ch = 0.0, na = 0.0, bad = 0.0;
  if (i < n && p.px[i] >= -1.0) {
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

template <>
hipError_t launch_particle_sums<double>(const Particles<double> &p, int64_t n,
                                        double m, double q, double wdv,
                                        double *acc, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  particle_sums_f64<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(p, n, m, q,
                                                                 wdv, acc);
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

__global__ void deposit_rho_f64(Particles<double> p, int64_t n, int dims,
                                double qw, double *rho, int pitch) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double xi = p.px[i];
  if (xi < -1.0) return;
  const int ix = (int)floor(xi);
  const double fx = xi - ix;
  const int hx = fx >= 0.5;
  double wx[3], wy[3] = {1, 0, 0};
  weights3(fx - hx, wx);
  int by = 0;
  if (dims == 2) {
    const double yi = p.py[i];
    const int iy = (int)floor(yi);
    const double fy = yi - iy;
    const int hy = fy >= 0.5;
    weights3(fy - hy, wy);
    by = iy + hy - 1 + kGuard;
  }
  const int bx = ix + hx - 1 + kGuard;
  for (int b = 0; b < (dims == 2 ? 3 : 1); ++b)
    for (int a = 0; a < 3; ++a)
      unsafeAtomicAdd(&rho[(size_t)(by + b) * pitch + bx + a], qw * wx[a] * wy[b]);
}

template <>
hipError_t launch_deposit_rho<double>(const Particles<double> &p, int64_t n,
                                      int dims, double qw, double *rho,
                                      int pitch, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  deposit_rho_f64<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(p, n, dims, qw,
                                                               rho, pitch);
  return hipGetLastError();
}

// Gauss-law residual |div_h E - (rho - rho0)| at primal nodes at least 4
// cells inside the physical box; acc[5] = max residual, acc[6] = max |rho -
// rho0| there.
template <typename R>
__global__ void gauss_kernel(Fields<R> f, int dims, int nx, int ny,
                             double idx, double idy, const double *rho,
                             const double *rho0, int rp, double *acc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x + 4;
  const int j = (dims == 2) ? blockIdx.y + 4 : 0;
  if (i > nx - 4) return;
  const int I = i + kGuard, J = (dims == 2) ? j + kGuard : 0;
  const size_t k = (size_t)J * f.pitch + I;
  double div = ((double)f.ex[k] - (double)f.ex[k - 1]) * idx;
  if (dims == 2) div += ((double)f.ey[k] - (double)f.ey[k - f.pitch]) * idy;
  const size_t kr = (size_t)J * rp + I;
  const double dr = rho[kr] - rho0[kr];
  atomic_max_pos(&acc[5], fabs(div - dr));
  atomic_max_pos(&acc[6], fabs(dr));
}

template <typename R>
hipError_t launch_gauss(const Fields<R> &f, int dims, int nx, int ny,
                        double dx, double dy, const double *rho,
                        const double *rho0, int rpitch, double *acc,
                        hipStream_t st) {
  if (nx < 9 || (dims == 2 && ny < 9)) return hipSuccess;
  dim3 g((nx - 7 + 255) / 256, dims == 2 ? ny - 7 : 1);
  gauss_kernel<R><<<g, 256, 0, st>>>(f, dims, nx, ny, 1.0 / dx, 1.0 / dy, rho,
                                     rho0, rpitch, acc);
  return hipGetLastError();
}

__global__ void histogram_f64(Particles<double> p, int64_t n, double m,
                              double wdv, int n_e, double emax, int n_t,
                              double ek_min, double *hist, double *mom) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || p.px[i] < -1.0) return;
  const double ux = p.ux[i], uy = p.uy[i], uz = p.uz[i];
  const double ek = m * (sqrt(1.0 + ux * ux + uy * uy + uz * uz) - 1.0);
  const double th = atan2(sqrt(uy * uy + uz * uz), ux) * (180.0 / 3.14159265358979323846);
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

template <>
hipError_t launch_histogram<double>(const Particles<double> &p, int64_t n,
                                    double m, double wdv, int n_e,
                                    double emax, int n_t, double ek_min,
                                    double *hist, double *mom,
                                    hipStream_t st) {
  if (n <= 0) return hipSuccess;
  histogram_f64<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(
      p, n, m, wdv, n_e, emax, n_t, ek_min, hist, mom);
  return hipGetLastError();
}

template hipError_t launch_faraday<double>(const Fields<double> &, int, double,
                                           double, double, hipStream_t);
template hipError_t launch_ampere<double>(const Fields<double> &, int, double,
                                          double, double, hipStream_t);
template hipError_t launch_field_sums<double>(const Fields<double> &, double *,
                                              hipStream_t);
template hipError_t launch_gauss<double>(const Fields<double> &, int, int, int,
                                         double, double, const double *,
                                         const double *, int, double *,
                                         hipStream_t);

}  // namespace sfpic
