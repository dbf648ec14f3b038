// Host runtime behind the C ABI of include/sfpic.h: validation, device memory,
// particle placement, step scheduling on the caller's HIP stream, reads,
// diagnostics and checkpoints.  The FP64 and FP32 forms share this code; the
// precision picks the kernel instantiation.
#include "sfpic_sim.h"

#include <math.h>
#include <string.h>

#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

using namespace sfpic;

namespace sfpic {

// Last failure of the calling thread, and of every handle: a call records
// its message for each handle whose entry point is active on this thread
// (the handle of the ABI call and of the inner calls it makes).
thread_local std::string g_last_error;
thread_local std::vector<const void *> g_scopes;
std::mutex g_err_mu;
std::unordered_map<const void *, std::string> g_err_by_handle;

int fail(int code, const std::string &msg) {
  g_last_error = msg;
  if (!g_scopes.empty()) {
    std::lock_guard<std::mutex> lk(g_err_mu);
    for (const void *h : g_scopes)
      if (h) g_err_by_handle[h] = msg;
  }
  return code;
}

ErrScope::ErrScope(const void *handle) { g_scopes.push_back(handle); }
ErrScope::~ErrScope() { g_scopes.pop_back(); }

void forget_handle(const void *handle) {
  if (!handle) return;
  std::lock_guard<std::mutex> lk(g_err_mu);
  g_err_by_handle.erase(handle);
}

}  // namespace sfpic

namespace {

constexpr uint64_t kStateMagic = 0x53465049435354ull;  // "SFPICST"

}  // namespace

namespace {

// Incident-field preparation: waist relation and amplitude normalization
// (a0 = modulus of the complex on-axis component at the focus and focal time).
int prepare_incident(const sfpic_incident *in, IncParams &P) {
  memset(&P, 0, sizeof(P));
  P.kind = in ? in->kind : SFPIC_INC_NONE;
  if (P.kind == SFPIC_INC_NONE) return SFPIC_OK;
  if (in->on_nodes != 0 && in->on_nodes != 1)
    return fail(SFPIC_E_INVAL, "incident on_nodes must be 0 or 1");
  P.on_nodes = in->on_nodes;
  if (P.kind == SFPIC_INC_PLANE_PULSE_1D) {
    if (!(in->fwhm_t > 0.0) || !isfinite(in->a0) || !isfinite(in->t0))
      return fail(SFPIC_E_INVAL, "plane pulse needs fwhm_t > 0, finite a0/t0");
    P.a0 = in->a0;
    P.t0 = in->t0;
    P.env_k = -4.0 / (in->fwhm_t * in->fwhm_t);
    return SFPIC_OK;
  }
  if (P.kind == SFPIC_INC_GAUSS_2D) {
    if (!(in->fwhm_t > 0.0) || !(in->w0 > 0.0) || !isfinite(in->a0) ||
        !isfinite(in->t0) || !isfinite(in->x_focus) || !isfinite(in->y_focus))
      return fail(SFPIC_E_INVAL,
                  "Gaussian beam needs w0 > 0, fwhm_t > 0 and finite a0, t0, "
                  "focus");
    P.a0 = in->a0;
    P.t0 = in->t0;
    P.env_k = -4.0 / (in->fwhm_t * in->fwhm_t);
    P.w0 = in->w0;
    P.zr = 0.5 * in->w0 * in->w0;
    P.x_focus = in->x_focus;
    P.y_focus = in->y_focus;
    return SFPIC_OK;
  }
  if (P.kind != SFPIC_INC_APRIL_LP && P.kind != SFPIC_INC_APRIL_RP)
    return fail(SFPIC_E_INVAL, "unknown incident kind");
  const double s = in->s;
  if (!(in->w0 > 0.0) || !(s >= 1.0) || s > 1000.0 || s != floor(s))
    return fail(SFPIC_E_INVAL, "April beam needs w0 > 0 and integer s >= 1");
  if (!isfinite(in->a0) || !isfinite(in->x_focus) || !isfinite(in->y_focus) ||
      !isfinite(in->t_focus) || !isfinite(in->phi0))
    return fail(SFPIC_E_INVAL, "April beam parameters must be finite");
  // k^2 w0^2 = 2 (sqrt(1 + (ka)^2) - 1)  =>  ka = sqrt((1 + w0^2/2)^2 - 1)
  const double h = 1.0 + 0.5 * in->w0 * in->w0;
  P.a = sqrt(h * h - 1.0);
  P.inv_a = 1.0 / P.a;
  P.s_int = (int)s;
  P.inv_s = 1.0 / s;
  P.a_over_s = P.a / s;
  P.x_focus = in->x_focus;
  P.y_focus = in->y_focus;
  P.t_focus = in->t_focus;
  auto set_coeffs = [&](double norm) {
    const double pr = norm * cos(in->phi0), pi = norm * sin(in->phi0);
    P.e_phase_r = pr;
    P.e_phase_i = pi;
    cx<double> c = mk(pr, pi);
    cx<double> ias = mk(0.0, P.a_over_s);
    for (int n = 0; n < 3; ++n) {
      P.cr[n] = c.r;
      P.ci[n] = c.i;
      c = (s + n + 1.0) * (c * ias);
    }
  };
  set_coeffs(1.0);
  cx<double> e[3], b[3];
  april_complex_fields(P, 0.0, 0.0, 0.0, 0.0, e, b);
  const cx<double> d = (P.kind == SFPIC_INC_APRIL_LP) ? e[0] : e[2];
  const double m = sqrt(d.r * d.r + d.i * d.i);
  if (!(m > 0.0) || !isfinite(m))
    return fail(SFPIC_E_INVAL, "April beam normalization failed");
  set_coeffs(in->a0 / m);
  return SFPIC_OK;
}

int check_grid(const sfpic_grid *g) {
  if (!g) return fail(SFPIC_E_INVAL, "grid is NULL");
  if (g->dims != 1 && g->dims != 2)
    return fail(SFPIC_E_INVAL, "dims must be 1 or 2");
  const int64_t lim = 65535 - 2 * kGuard;
  if (g->nx < 8 || g->nx > lim)
    return fail(SFPIC_E_INVAL, "nx out of range [8, 65529]");
  if (g->dims == 2 && (g->ny < 8 || g->ny > lim))
    return fail(SFPIC_E_INVAL, "ny out of range [8, 65529]");
  if (!(g->dx > 0.0) || (g->dims == 2 && !(g->dy > 0.0)) || !(g->dt > 0.0))
    return fail(SFPIC_E_INVAL, "dx, dy, dt must be positive");
  const double lim_dt =
      (g->dims == 2) ? 1.0 / sqrt(1.0 / (g->dx * g->dx) + 1.0 / (g->dy * g->dy))
                     : g->dx;
  if (!(g->dt < lim_dt)) return fail(SFPIC_E_INVAL, "dt violates the CFL limit");
  return SFPIC_OK;
}

template <typename R>
void set_field_ptrs(Fields<R> &f, void *const planes[12],
                    void *const inc_planes[3], int NX, int NY, int pitch) {
  R **dst[12] = {&f.ex, &f.ey, &f.ez, &f.bx, &f.by, &f.bz,
                 &f.jx, &f.jy, &f.jz, &f.mx, &f.my, &f.mz};
  for (int c = 0; c < 12; ++c) *dst[c] = (R *)planes[c];
  f.iex = (R *)inc_planes[0];
  f.iey = (R *)inc_planes[1];
  f.ibz = (R *)inc_planes[2];
  f.nx_alloc = NX;
  f.ny_alloc = NY;
  f.pitch = pitch;
}

// Device arrays of one particle set.
bool alloc_set(sfpic_sim *s, Particles<double> &q, size_t cnt) {
  double **arr[5] = {&q.px, &q.py, &q.ux, &q.uy, &q.uz};
  for (auto a : arr)
    if (!(*a = (double *)s->dalloc(cnt * 8))) return false;
  return (q.id = (uint32_t *)s->dalloc(cnt * 4)) != nullptr;
}
bool alloc_set(sfpic_sim *s, Particles<float> &q, size_t cnt) {
  if (!(q.cell = (uint32_t *)s->dalloc(cnt * 4))) return false;
  float **arr[5] = {&q.ox, &q.oy, &q.ux, &q.uy, &q.uz};
  for (auto a : arr)
    if (!(*a = (float *)s->dalloc(cnt * 4))) return false;
  return (q.id = (uint32_t *)s->dalloc(cnt * 4)) != nullptr;
}

// Raw arrays of a particle set (for checkpoints): pointers and element sizes.
int raw_arrays(Particles<double> &q, void *ptr[7], size_t sz[7]) {
  void *p[6] = {q.px, q.py, q.ux, q.uy, q.uz, q.id};
  size_t z[6] = {8, 8, 8, 8, 8, 4};
  for (int k = 0; k < 6; ++k) {
    ptr[k] = p[k];
    sz[k] = z[k];
  }
  return 6;
}
int raw_arrays(Particles<float> &q, void *ptr[7], size_t sz[7]) {
  void *p[7] = {q.cell, q.ox, q.oy, q.ux, q.uy, q.uz, q.id};
  for (int k = 0; k < 7; ++k) {
    ptr[k] = p[k];
    sz[k] = 4;
  }
  return 7;
}
size_t bytes_per_particle(int precision) {
  return precision == SFPIC_FP64 ? 5 * 8 + 4 : 7 * 4;
}

int alloc_species(sfpic_sim *s, SpeciesState &st, int64_t n) {
  st.n = n;
  const size_t cnt = (size_t)(n > 0 ? n : 1);
  st.n_valid = (uint32_t *)s->dalloc(4);
  if (!st.n_valid) return fail(SFPIC_E_NOMEM, "particle allocation failed");
  const bool ok =
      s->precision == SFPIC_FP64
          ? alloc_set(s, st.p64, cnt) && alloc_set(s, st.p64_alt, cnt)
          : alloc_set(s, st.p32, cnt) && alloc_set(s, st.p32_alt, cnt);
  if (!ok) return fail(SFPIC_E_NOMEM, "particle allocation failed");
  const uint32_t nv = (uint32_t)n;
  HIP_TRY(hipMemcpy(st.n_valid, &nv, 4, hipMemcpyHostToDevice));
  return SFPIC_OK;
}

int place_species(sfpic_sim *s, SpeciesState &st, const sfpic_species &in) {
  const sfpic_grid &g = s->grid;
  if (!(in.m > 0.0) || !isfinite(in.q))
    return fail(SFPIC_E_INVAL, "species needs m > 0 and finite q");
  st.q = in.q;
  st.m = in.m;
  if (in.n_explicit > 0) {
    const int64_t n = in.n_explicit;
    if (n > 0xFFFFFFFFll) return fail(SFPIC_E_INVAL, "too many particles");
    if (!in.x || !in.ux || !in.uy || !in.uz || (g.dims == 2 && !in.y))
      return fail(SFPIC_E_INVAL, "explicit particle arrays are NULL");
    if (!isfinite(in.weight)) return fail(SFPIC_E_NUMERIC, "weight not finite");
    const double X = g.nx * g.dx, Y = g.ny * g.dy;
    for (int64_t i = 0; i < n; ++i) {
      if (!isfinite(in.ux[i]) || !isfinite(in.uy[i]) || !isfinite(in.uz[i]))
        return fail(SFPIC_E_NUMERIC, "non-finite particle momentum");
      if (!(in.x[i] >= 0.0 && in.x[i] < X) ||
          (g.dims == 2 && !(in.y[i] >= 0.0 && in.y[i] < Y)))
        return fail(SFPIC_E_INVAL, "particle outside the physical box");
    }
    st.weight = in.weight;
    SF_TRY(alloc_species(s, st, n));
    // stage the host arrays through one device buffer
    double *tmp = (double *)s->dalloc((size_t)n * 5 * 8);
    if (!tmp) return fail(SFPIC_E_NOMEM, "staging allocation failed");
    const double *src[5] = {in.x, g.dims == 2 ? in.y : in.x, in.ux, in.uy,
                            in.uz};
    for (int k = 0; k < 5; ++k)
      HIP_TRY(hipMemcpyAsync(tmp + (size_t)k * n, src[k], (size_t)n * 8,
                             hipMemcpyHostToDevice, s->stream));
    const int r = s->dispatch([&](auto z) -> int {
      using R = decltype(z);
      HIP_TRY(launch_load_particles<R>(parts<R>(st), n, g.dims, tmp, tmp + n,
                                       tmp + 2 * n, tmp + 3 * n, tmp + 4 * n,
                                       1.0 / g.dx, 1.0 / g.dy, (int)g.nx,
                                       (int)g.ny, s->stream));
      return SFPIC_OK;
    });
    if (r) return r;
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->dfree(tmp);
    return SFPIC_OK;
  }
  // generated placement
  const int64_t x0 = in.region[0], x1 = in.region[1];
  int64_t y0 = in.region[2], y1 = in.region[3];
  if (g.dims == 1) {
    y0 = 0;
    y1 = 1;
  }
  if (in.ppc < 0 || x0 < 0 || x1 > g.nx || x0 > x1 || y0 < 0 ||
      (g.dims == 2 && y1 > g.ny) || y0 > y1)
    return fail(SFPIC_E_INVAL, "species region outside the grid");
  if (in.ppc > 0 && !(in.density >= 0.0))
    return fail(SFPIC_E_INVAL, "density < 0");
  if (!(in.temperature_ev >= 0.0))
    return fail(SFPIC_E_INVAL, "temperature < 0");
  const double sigma = sqrt(in.temperature_ev / (510998.95 * in.m));
  st.weight = in.ppc > 0 ? in.density / in.ppc : 0.0;
  if (in.profile != SFPIC_PROFILE_UNIFORM && in.ppc > 0 && x1 > x0) {
    std::vector<uint32_t> off;
    SF_TRY(profile_offsets(in.profile, in.profile_center, in.profile_fwhm,
                           in.profile_order, in.profile_xmin, x0, x1, g.dx,
                           in.ppc, off));
    const uint32_t per_row = off.back();
    const int64_t n = (int64_t)per_row * (y1 - y0);
    if (n > 0xFFFFFFFFll) return fail(SFPIC_E_INVAL, "too many particles");
    SF_TRY(alloc_species(s, st, n));
    if (n == 0) return SFPIC_OK;
    uint32_t *doff = (uint32_t *)s->dalloc(off.size() * 4);
    if (!doff) return fail(SFPIC_E_NOMEM, "profile table allocation failed");
    HIP_TRY(hipMemcpyAsync(doff, off.data(), off.size() * 4,
                           hipMemcpyHostToDevice, s->stream));
    const int r = s->dispatch([&](auto z) -> int {
      using R = decltype(z);
      HIP_TRY(launch_init_particles_profile<R>(
          parts<R>(st), n, g.dims, x0, (int)(x1 - x0), y0, doff, per_row,
          sigma, in.seed, (uint32_t)in.species_index, s->stream));
      return SFPIC_OK;
    });
    if (r) return r;
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->dfree(doff);
    return SFPIC_OK;
  }
  const int64_t n = (x1 - x0) * (y1 - y0) * (int64_t)in.ppc;
  if (n > 0xFFFFFFFFll) return fail(SFPIC_E_INVAL, "too many particles");
  SF_TRY(alloc_species(s, st, n));
  return s->dispatch([&](auto z) -> int {
    using R = decltype(z);
    HIP_TRY(launch_init_particles<R>(parts<R>(st), n, g.dims, x0, x1 - x0, y0,
                                     in.ppc > 0 ? in.ppc : 1, sigma, in.seed,
                                     (uint32_t)in.species_index, g.dx, g.dy,
                                     s->stream));
    return SFPIC_OK;
  });
}

int deposit_rho(sfpic_sim *s, double *rho) {
  const size_t bytes = (size_t)s->NY * s->pitch * 8;
  HIP_TRY(hipMemsetAsync(rho, 0, bytes, s->stream));
  return s->dispatch([&](auto z) -> int {
    using R = decltype(z);
    for (auto &st : s->sp)
      HIP_TRY(launch_deposit_rho<R>(parts<R>(st), st.n, st.n_valid,
                                    s->grid.dims, st.q * st.weight, rho,
                                    s->pitch, s->stream));
    return SFPIC_OK;
  });
}

int setup_tiles(sfpic_sim *s) {
  const sfpic_grid &g = s->grid;
  TileGeom &t = s->tg;
  int max_lds = 64 * 1024;
  (void)hipDeviceGetAttribute(&max_lds,
                              hipDeviceAttributeMaxSharedMemoryPerBlock,
                              s->rt.device);
  auto lds_of = [&](const TileGeom &tt) {
    return s->precision == SFPIC_FP64 ? push_lds_bytes<double>(tt, g.dims)
                                      : push_lds_bytes<float>(tt, g.dims);
  };
  // drift allowance of the tile window: 1 cell keeps two 16 x 16 FP64
  // workgroups (81.6 KB each) and three FP32 ones per CU (160 KiB LDS)
  // drift allowance: FP64 reads its particles straight from HBM, so its
  // LDS holds only the windows and a wide one is affordable; the FP32 form
  // stages particles in LDS and keeps the narrow one (three workgroups/CU)
  t.slack = s->precision == SFPIC_FP64 ? kSingleSlackF64 : kSingleSlackF32;
  if (g.dims == 1) {
    t.tx = s->rt.tile_x > 0 ? s->rt.tile_x : 256;
    t.ty = 1;
  } else {
    // 16 x 16 by default (measured fastest in both precisions on gfx950);
    // smaller tiles where the workgroup LDS limit is lower
    t.tx = s->rt.tile_x > 0 ? s->rt.tile_x : 16;
    t.ty = s->rt.tile_y > 0 ? s->rt.tile_y : 16;
    if (s->rt.tile_x <= 0 && s->rt.tile_y <= 0 && lds_of(t) > (size_t)max_lds)
      t.ty = 8;
    if (s->rt.tile_x <= 0 && s->rt.tile_y <= 0 && lds_of(t) > (size_t)max_lds)
      t.tx = 8;
  }
  if (t.tx < 1 || t.ty < 1 || t.tx > 1024 || t.ty > 256)
    return fail(SFPIC_E_INVAL, "tile size out of range");
  t.ntx = (int)((g.nx + t.tx - 1) / t.tx);
  t.nty = (g.dims == 2) ? (int)((g.ny + t.ty - 1) / t.ty) : 1;
  t.ntiles = t.ntx * t.nty;
  t.cells_per_tile = (uint32_t)(t.tx * t.ty);
  const uint64_t nk = (uint64_t)t.ntiles * t.cells_per_tile;
  if (nk >= 0xFFFFFFF0ull) return fail(SFPIC_E_INVAL, "too many cells");
  t.nkeys = (uint32_t)nk;
  if (lds_of(t) > (size_t)max_lds)
    return fail(SFPIC_E_INVAL, "tile too large for LDS");
  // sort cadence: FP64 single sims every 8 steps (their three cells of
  // drift allowance keep stragglers few between sorts); the FP32 form, with
  // one cell of allowance, every 4: once the beam heats the plasma, sorting
  // every 8 leaves a fifth of the step to the straggler push (measured on
  // the 4096^2 RP run at step 1500: 8.85 ms per step every 8, 7.59 every 4)
  s->sort_every = s->precision == SFPIC_FP32 ? 4 : 8;
  s->sort_adaptive = s->rt.sort_every <= 0;
  if (s->rt.sort_every > 0) s->sort_every = s->rt.sort_every;
  s->item_max = default_item_particles(s->precision);
  if (s->rt.item_particles != 0) {
    if (s->rt.item_particles < 64)
      return fail(SFPIC_E_INVAL, "item_particles must be >= 64");
    s->item_max = (uint32_t)s->rt.item_particles;
  }
  const size_t nk1 = (size_t)t.nkeys + 1;
  s->ss.counts = (uint32_t *)s->dalloc(nk1 * 4);
  for (auto &st : s->sp) {
    st.start = (uint32_t *)s->dalloc(nk1 * 4);
    if (!st.start) return fail(SFPIC_E_NOMEM, "sort allocation failed");
  }
  s->ss.block_sums = (uint32_t *)s->dalloc(((nk1 + 1023) / 1024 + 1) * 4);
  int64_t nmax = 1;
  for (auto &st : s->sp) nmax = st.n > nmax ? st.n : nmax;
  s->ss.key = (uint32_t *)s->dalloc((size_t)nmax * 4);
  s->ss.rank = (uint32_t *)s->dalloc((size_t)nmax * 4);
  s->strag = (uint32_t *)s->dalloc((size_t)nmax * 4);
  s->n_strag = (uint32_t *)s->dalloc(4);
  if (!s->ss.counts || !s->ss.block_sums || !s->ss.key || !s->ss.rank ||
      !s->strag || !s->n_strag)
    return fail(SFPIC_E_NOMEM, "sort scratch allocation failed");
  return SFPIC_OK;
}

}  // namespace

namespace sfpic {
int profile_offsets(int32_t profile, double center, double fwhm, double order,
                    double xmin, int64_t x0, int64_t x1, double dx, int ppc,
                    std::vector<uint32_t> &off) {
  if (profile != SFPIC_PROFILE_SUPERGAUSS)
    return fail(SFPIC_E_INVAL, "unknown density profile");
  if (!(fwhm > 0.0) || !(order > 0.0) || !isfinite(center) ||
      !isfinite(fwhm) || !isfinite(order) || isnan(xmin))
    return fail(SFPIC_E_INVAL, "profile needs fwhm > 0, order > 0, finite centre");
  off.assign((size_t)(x1 - x0) + 1, 0u);
  uint64_t acc = 0;
  for (int64_t c = x0; c < x1; ++c) {
    const double xc = ((double)c + 0.5) * dx;
    const double f =
        xc > xmin ? pow(2.0, -pow(fabs(2.0 * (xc - center) / fwhm), order))
                  : 0.0;
    acc += (uint64_t)floor((double)ppc * f + 0.5);
    if (acc > 0xFFFFFFFFull) return fail(SFPIC_E_INVAL, "too many particles");
    off[(size_t)(c - x0) + 1] = (uint32_t)acc;
  }
  return SFPIC_OK;
}

// The incident-field preparation for the 3D entry points (sfpic3.hip).
int prepare_incident_ext(const sfpic_incident *in, IncParams &P) {
  return prepare_incident(in, P);
}
}  // namespace sfpic

namespace sfpic {

// Counting sort of every species by cell (compacts removed particles).
int sort_all(sfpic_sim *s) {
  const int r = s->dispatch([&](auto z) -> int {
    using R = decltype(z);
    for (auto &st : s->sp) {
      HIP_TRY(launch_sort<R>(parts<R>(st), parts_alt<R>(st), (uint32_t)st.n,
                             st.n_valid, st.start, s->tg, (int)s->grid.nx,
                             (int)s->grid.ny, s->grid.dims, s->ss, s->stream));
      std::swap(parts<R>(st), parts_alt<R>(st));
      // (after a retile to more tiles the arrays may be too small: the next
      // step's refresh_items reallocates and builds them)
      if (st.items &&
          st.items_words >= push_items_words(s->tg, st.n, s->item_max))
        HIP_TRY(launch_build_items(st.start, s->tg, s->item_max, st.items,
                                   st.n_items, s->stream));
    }
    return SFPIC_OK;
  });
  s->since_sort = 0;
  return r;
}

int sim_retile(sfpic_sim *s, int tx, int ty, int slack) {
  if (!s) return fail(SFPIC_E_INVAL, "sim is NULL");
  const sfpic_grid &g = s->grid;
  TileGeom t{};
  t.slack = slack > 0 ? slack : s->tg.slack;
  if (t.slack < 1 || t.slack > 4)
    return fail(SFPIC_E_INVAL, "tile slack out of range");
  t.tx = tx;
  t.ty = g.dims == 2 ? ty : 1;
  if (t.tx < 1 || t.ty < 1 || t.tx > 1024 || t.ty > 256)
    return fail(SFPIC_E_INVAL, "tile size out of range");
  t.ntx = (int)((g.nx + t.tx - 1) / t.tx);
  t.nty = (g.dims == 2) ? (int)((g.ny + t.ty - 1) / t.ty) : 1;
  t.ntiles = t.ntx * t.nty;
  t.cells_per_tile = (uint32_t)(t.tx * t.ty);
  const uint64_t nk = (uint64_t)t.ntiles * t.cells_per_tile;
  if (nk >= 0xFFFFFFF0ull) return fail(SFPIC_E_INVAL, "too many cells");
  t.nkeys = (uint32_t)nk;
  int max_lds = 64 * 1024;
  (void)hipDeviceGetAttribute(&max_lds,
                              hipDeviceAttributeMaxSharedMemoryPerBlock,
                              s->rt.device);
  const size_t lds = s->precision == SFPIC_FP64
                         ? push_lds_bytes<double>(t, g.dims)
                         : push_lds_bytes<float>(t, g.dims);
  if (lds > (size_t)max_lds) return fail(SFPIC_E_INVAL, "tile too large for LDS");
  if (t.nkeys > s->tg.nkeys) {
    // the old arrays may still be in use by queued work
    HIP_TRY(hipStreamSynchronize(s->stream));
    const size_t nk1 = (size_t)t.nkeys + 1;
    uint32_t *counts = (uint32_t *)s->dalloc(nk1 * 4);
    uint32_t *sums = (uint32_t *)s->dalloc(((nk1 + 1023) / 1024 + 1) * 4);
    if (!counts || !sums) return fail(SFPIC_E_NOMEM, "sort allocation failed");
    std::vector<uint32_t *> starts;
    for (size_t k = 0; k < s->sp.size(); ++k) {
      uint32_t *st = (uint32_t *)s->dalloc(nk1 * 4);
      if (!st) return fail(SFPIC_E_NOMEM, "sort allocation failed");
      starts.push_back(st);
    }
    s->dfree(s->ss.counts);
    s->dfree(s->ss.block_sums);
    s->ss.counts = counts;
    s->ss.block_sums = sums;
    for (size_t k = 0; k < s->sp.size(); ++k) {
      s->dfree(s->sp[k].start);
      s->sp[k].start = starts[k];
    }
  }
  s->tg = t;
  return sort_all(s);
}

size_t sim_device_bytes(const sfpic_sim *s) {
  size_t b = 0;
  for (auto &a : s->allocs) b += a.second;
  return b;
}

int sim_footprint(const sfpic_grid *grid, const sfpic_species *species,
                  int nspecies, sfpic_precision precision,
                  const sfpic_runtime *rt, size_t *bytes) {
  SF_TRY(check_grid(grid));
  if (!bytes) return fail(SFPIC_E_INVAL, "bytes is NULL");
  if (nspecies < 0 || nspecies > 8 || (nspecies > 0 && !species))
    return fail(SFPIC_E_INVAL, "nspecies must be in [0, 8]");
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const int dims = grid->dims;
  const size_t es = precision == SFPIC_FP64 ? 8 : 4;
  const size_t NX = (size_t)grid->nx + 2 * kGuard;
  const size_t NY = dims == 2 ? (size_t)grid->ny + 2 * kGuard : 1;
  const size_t pitch = (NX + 63) & ~(size_t)63;
  size_t b = 12 * al(NY * pitch * es) + 3 * al(NY * pitch * 8) + al(64 * 8);
  int tx = rt && rt->tile_x > 0 ? rt->tile_x : (dims == 2 ? 16 : 256);
  int ty = dims == 2 ? (rt && rt->tile_y > 0 ? rt->tile_y : 16) : 1;
  const size_t ntx = ((size_t)grid->nx + tx - 1) / tx;
  const size_t nty = dims == 2 ? ((size_t)grid->ny + ty - 1) / ty : 1;
  const size_t nk1 = ntx * nty * (size_t)tx * ty + 1;
  b += al(nk1 * 4) + al(((nk1 + 1023) / 1024 + 1) * 4) + al(4);
  size_t nmax = 1, staging = 0;
  for (int k = 0; k < nspecies; ++k) {
    const sfpic_species &in = species[k];
    int64_t n = in.n_explicit;
    if (n <= 0) {
      const int64_t y0 = dims == 2 ? in.region[2] : 0;
      const int64_t y1 = dims == 2 ? in.region[3] : 1;
      n = (in.region[1] - in.region[0]) * (y1 - y0) * (int64_t)in.ppc;
      if (n < 0) return fail(SFPIC_E_INVAL, "species region is empty");
    } else if ((size_t)n * 40 > staging) {
      staging = (size_t)n * 40;
    }
    const size_t cnt = n > 0 ? (size_t)n : 1;
    nmax = cnt > nmax ? cnt : nmax;
    const size_t set = precision == SFPIC_FP64 ? 5 * al(cnt * 8) + al(cnt * 4)
                                               : 7 * al(cnt * 4);
    const size_t kmax = rt && rt->item_particles >= 64
                            ? (size_t)rt->item_particles
                            : (size_t)default_item_particles(precision);
    const size_t items = 2 * (ntx * nty + cnt / kmax + 1);
    b += al(4) + 2 * set + al(nk1 * 4) + al(items * 4) + al(4);
  }
  b += 3 * al(nmax * 4) + al(staging);
  *bytes = b;
  return SFPIC_OK;
}

// Work items of every species for the current sort (the start offsets may
// also have been rewritten by a batch's sorts); the arrays are (re)allocated
// here when the tiling needs more than they hold.
int refresh_items(sfpic_sim *s) {
  for (auto &st : s->sp) {
    const size_t words = push_items_words(s->tg, st.n, s->item_max);
    if (words > st.items_words) {
      HIP_TRY(hipStreamSynchronize(s->stream));  // old arrays may be queued
      s->dfree(st.items);
      if (!st.n_items) st.n_items = (uint32_t *)s->dalloc(4);
      st.items = (uint32_t *)s->dalloc(words * 4);
      if (!st.items || !st.n_items) {
        st.items_words = 0;
        return fail(SFPIC_E_NOMEM, "work-item allocation failed");
      }
      st.items_words = words;
    }
    HIP_TRY(launch_build_items(st.start, s->tg, s->item_max, st.items,
                               st.n_items, s->stream));
  }
  return SFPIC_OK;
}

}  // namespace sfpic

namespace {

// Field planes between device (rows of `pitch` elements) and host (rows of
// NX elements, [NY][NX]): one contiguous copy of the whole pitched plane
// and the row repacking on the host.  (2D copies are avoided: under the
// rocprofv3 profiler of ROCm 7.2 hipMemcpy2D from device planes of this
// size returned zeros while 1D copies were correct.)
int plane_to_host(const sfpic_sim *s, int comp, void *dst) {
  const size_t es = s->esize(), row = (size_t)s->NX * es;
  std::vector<uint8_t> tmp;
  try {
    tmp.resize((size_t)s->NY * s->pitch * es);
  } catch (...) {
    return fail(SFPIC_E_NOMEM, "host allocation failed");
  }
  HIP_TRY(hipMemcpy(tmp.data(), s->planes[comp], tmp.size(),
                    hipMemcpyDeviceToHost));
  for (int j = 0; j < s->NY; ++j)
    memcpy((uint8_t *)dst + j * row, tmp.data() + (size_t)j * s->pitch * es,
           row);
  return SFPIC_OK;
}

int plane_from_host(sfpic_sim *s, int comp, const void *src) {
  const size_t es = s->esize(), row = (size_t)s->NX * es;
  std::vector<uint8_t> tmp;
  try {
    tmp.assign((size_t)s->NY * s->pitch * es, 0);
  } catch (...) {
    return fail(SFPIC_E_NOMEM, "host allocation failed");
  }
  for (int j = 0; j < s->NY; ++j)
    memcpy(tmp.data() + (size_t)j * s->pitch * es,
           (const uint8_t *)src + j * row, row);
  HIP_TRY(hipMemcpy(s->planes[comp], tmp.data(), tmp.size(),
                    hipMemcpyHostToDevice));
  return SFPIC_OK;
}

int guarded(sfpic_sim *s) {
  if (!s) return fail(SFPIC_E_INVAL, "sim is NULL");
  HIP_TRY(hipSetDevice(s->rt.device));
  return SFPIC_OK;
}

// Launch helper: bracket a kernel launch with events when profiling.
template <typename F>
hipError_t timed(sfpic_sim *s, int cls, F &&launch) {
  if (!s->profiling) return launch();
  auto e = s->take_events();
  hipError_t r = hipEventRecord(e.first, s->stream);
  if (r == hipSuccess) r = launch();
  if (r == hipSuccess) r = hipEventRecord(e.second, s->stream);
  s->ev_used[cls].push_back(e);
  return r;
}

// Straggler fraction above which the adaptive cadence sorts (2^-10).  On
// the 4096^2 RP run, against the fixed cadence (FP32 form every 4 steps,
// FP64 every 8): first 200 steps 26.8 -> 28.0 and 22.1 -> 23.1 G pushes/s,
// the run to step 3000 20.5 -> 20.5 and 18.6 -> 18.8; 2^-13 sorted almost
// as often as the fixed cadence, 2^-8 and 2^-6 lost on the long run.
constexpr double kStragSortFrac = 1.0 / 1024.0;

// Whether a sort is due under the adaptive cadence (since_sort is at least
// sort_every and below sort_max): the push of two steps ago (its counts
// copied back to the pinned ring) listed more than kStragSortFrac of some
// species' slots as stragglers, or its record is missing.  Waiting on that
// step's event leaves the stream two steps of queued work.
int adaptive_sort_due(sfpic_sim *s, bool &due) {
  const int64_t want = s->step - 2;
  const int slot = (int)(want & (sfpic_sim::kStragRing - 1));
  due = true;
  if (want < 0 || s->strag_step[slot] != want) return SFPIC_OK;
  HIP_TRY(hipEventSynchronize(s->strag_ev[slot]));
  const size_t ns = s->sp.size();
  due = false;
  for (size_t i = 0; i < ns; ++i)
    if ((double)s->strag_host[(size_t)slot * ns + i] >
        kStragSortFrac * (double)s->sp[i].n)
      due = true;
  return SFPIC_OK;
}

int adaptive_sort_init(sfpic_sim *s) {
  if (s->strag_host) return SFPIC_OK;
  const size_t bytes = sfpic_sim::kStragRing * s->sp.size() * 4;
  HIP_TRY(hipHostMalloc((void **)&s->strag_host, bytes > 0 ? bytes : 4,
                        hipHostMallocDefault));
  for (auto &e : s->strag_ev)
    HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  for (auto &t : s->strag_step) t = -1;
  return SFPIC_OK;
}

template <typename R>
int step_impl(sfpic_sim *s, int64_t nsteps) {
  const sfpic_grid &g = s->grid;
  Fields<R> &f = s->fields<R>();
  if (nsteps > 0) SF_TRY(refresh_items(s));
  if (nsteps > 0 && s->sort_adaptive) SF_TRY(adaptive_sort_init(s));
  for (int64_t k = 0; k < nsteps; ++k) {
    bool sort_now = s->since_sort >= s->sort_every;
    if (sort_now && s->sort_adaptive && s->since_sort < s->sort_max)
      SF_TRY(adaptive_sort_due(s, sort_now));
    if (sort_now) {
      HIP_TRY(timed(s, 3, [&] {
        return sort_all(s) == SFPIC_OK ? hipSuccess : hipErrorUnknown;
      }));
    }
    // this step's straggler counts are read two steps later when that
    // step's decision is adaptive
    const bool record =
        s->sort_adaptive && s->since_sort + 2 >= s->sort_every;
    const int slot = (int)(s->step & (sfpic_sim::kStragRing - 1));
    HIP_TRY(timed(s, 0, [&] {
      return launch_faraday<R>(f, g.dims, g.dt, g.dx, g.dy, s->stream);
    }));
    if (s->inc.on_nodes)
      HIP_TRY(timed(s, 1, [&] {
        return launch_incident_nodes<R>(f, g.dims, g.dx, g.dy,
                                        (double)s->step * g.dt, s->inc,
                                        s->stream);
      }));
    for (auto &st : s->sp) {
      PushParams pp;
      pp.dt = g.dt;
      pp.dx = g.dx;
      pp.dy = g.dy;
      pp.inv_dx = 1.0 / g.dx;
      pp.inv_dy = 1.0 / g.dy;
      pp.qm = st.q / st.m;
      pp.qw = st.q * st.weight;
      pp.time = (double)s->step * g.dt;
      pp.nx = (int)g.nx;
      pp.ny = (int)g.ny;
      HIP_TRY(timed(s, 1, [&] {
        return launch_push_tiled<R>(f, parts<R>(st), st.start, st.items,
                                    st.n_items, s->item_max, st.n, s->tg,
                                    g.dims, pp, s->inc, s->strag, s->n_strag,
                                    s->stream);
      }));
      HIP_TRY(timed(s, 4, [&] {
        return launch_push_stragglers<R>(f, parts<R>(st), g.dims, pp, s->inc,
                                         s->strag, s->n_strag, s->stream);
      }));
      if (record)
        HIP_TRY(hipMemcpyAsync(
            s->strag_host + (size_t)slot * s->sp.size() + (&st - &s->sp[0]),
            s->n_strag, 4, hipMemcpyDeviceToHost, s->stream));
    }
    if (record) {
      HIP_TRY(hipEventRecord(s->strag_ev[slot], s->stream));
      s->strag_step[slot] = s->step;
    }
    HIP_TRY(timed(s, 2, [&] {
      return launch_ampere<R>(f, g.dims, g.dt, g.dx, g.dy, s->stream);
    }));
    s->step++;
    s->since_sort++;
  }
  return SFPIC_OK;
}

// Used slots of a species copied to host as FP64 (x, y, ux, uy, uz, id).
int fetch_particles(sfpic_sim *s, SpeciesState &st, std::vector<double> &h,
                    std::vector<uint32_t> &ids, size_t &n) {
  HIP_TRY(hipStreamSynchronize(s->stream));
  uint32_t nv = 0;
  HIP_TRY(hipMemcpy(&nv, st.n_valid, 4, hipMemcpyDeviceToHost));
  n = nv;
  h.assign(5 * n, 0.0);
  ids.assign(n, 0u);
  if (n == 0) return SFPIC_OK;
  double *d = (double *)s->dalloc(n * 5 * 8);
  uint32_t *di = (uint32_t *)s->dalloc(n * 4);
  if (!d || !di) {
    if (d) s->dfree(d);
    if (di) s->dfree(di);
    return fail(SFPIC_E_NOMEM, "export allocation failed");
  }
  int r = s->dispatch([&](auto z) -> int {
    using R = decltype(z);
    HIP_TRY(launch_export_particles<R>(parts<R>(st), (int64_t)n, s->grid.dims,
                                       s->grid.dx, s->grid.dy, d, di,
                                       s->stream));
    HIP_TRY(hipMemcpyAsync(h.data(), d, n * 5 * 8, hipMemcpyDeviceToHost,
                           s->stream));
    HIP_TRY(hipMemcpyAsync(ids.data(), di, n * 4, hipMemcpyDeviceToHost,
                           s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return SFPIC_OK;
  });
  s->dfree(d);
  s->dfree(di);
  return r;
}

}  // namespace

extern "C" {

const char *sfpic_last_error(const void *handle) {
  if (!handle) return g_last_error.c_str();
  std::lock_guard<std::mutex> lk(g_err_mu);
  auto it = g_err_by_handle.find(handle);
  return it == g_err_by_handle.end() ? "" : it->second.c_str();
}

const char *sfpic_version(void) { return "sfpic 0.2 (gfx950)"; }

int sfpic_create(const sfpic_grid *grid, const sfpic_species *species,
                 int nspecies, const sfpic_incident *incident,
                 sfpic_precision precision, const sfpic_runtime *runtime,
                 sfpic_sim **out) {
  try {
    if (!out) return fail(SFPIC_E_INVAL, "out is NULL");
    *out = nullptr;
    SF_TRY(check_grid(grid));
    if (nspecies < 0 || nspecies > 8 || (nspecies > 0 && !species))
      return fail(SFPIC_E_INVAL, "nspecies must be in [0, 8]");
    if (precision != SFPIC_FP64 && precision != SFPIC_FP32)
      return fail(SFPIC_E_INVAL, "unknown precision");
    IncParams inc;
    SF_TRY(prepare_incident(incident, inc));
    sfpic_sim *s = new (std::nothrow) sfpic_sim();
    if (!s) return fail(SFPIC_E_NOMEM, "host allocation failed");
    s->grid = *grid;
    if (grid->dims == 1) {
      s->grid.ny = 1;
      s->grid.dy = grid->dx;
    }
    s->precision = precision;
    if (runtime) s->rt = *runtime;
    s->stream = (hipStream_t)s->rt.stream;
    s->inc = inc;
    auto bail = [&](int code) {
      s->release();
      delete s;
      return code;
    };
    if (hipSetDevice(s->rt.device) != hipSuccess)
      return bail(fail(SFPIC_E_DEVICE, "hipSetDevice failed"));
    s->NX = (int)(s->grid.nx + 2 * kGuard);
    s->NY = (grid->dims == 2) ? (int)(s->grid.ny + 2 * kGuard) : 1;
    s->pitch = (s->NX + 63) & ~63;
    const size_t plane = (size_t)s->NY * s->pitch * s->esize();
    for (int c = 0; c < 12; ++c) {
      s->planes[c] = s->dalloc(plane);
      if (!s->planes[c])
        return bail(fail(SFPIC_E_NOMEM, "field allocation failed"));
      if (hipMemsetAsync(s->planes[c], 0, plane, s->stream) != hipSuccess)
        return bail(fail(SFPIC_E_DEVICE, "hipMemsetAsync failed"));
    }
    if (s->inc.on_nodes)
      for (int c = 0; c < 3; ++c)
        if (!(s->inc_planes[c] = s->dalloc(plane)))
          return bail(fail(SFPIC_E_NOMEM, "field allocation failed"));
    set_field_ptrs(s->f64, s->planes, s->inc_planes, s->NX, s->NY, s->pitch);
    set_field_ptrs(s->f32, s->planes, s->inc_planes, s->NX, s->NY, s->pitch);
    s->sp.resize(nspecies);
    for (int k = 0; k < nspecies; ++k) {
      const int r = place_species(s, s->sp[k], species[k]);
      if (r) return bail(r);
    }
    int r = setup_tiles(s);
    if (r) return bail(r);
    const size_t rbytes = (size_t)s->NY * s->pitch * 8;
    s->rho0 = (double *)s->dalloc(rbytes);
    s->rho = (double *)s->dalloc(rbytes);
    s->gprev = (double *)s->dalloc(rbytes);
    s->acc = (double *)s->dalloc(64 * 8);
    if (!s->rho0 || !s->rho || !s->gprev || !s->acc)
      return bail(fail(SFPIC_E_NOMEM, "diagnostic allocation failed"));
    r = deposit_rho(s, s->rho0);
    if (r) return bail(r);
    r = sort_all(s);
    if (r) return bail(r);
    if (hipStreamSynchronize(s->stream) != hipSuccess)
      return bail(fail(SFPIC_E_DEVICE, "initialization failed"));
    *out = s;
    return SFPIC_OK;
  } catch (...) {
    return fail(SFPIC_E_NOMEM, "exception during create");
  }
}

int sfpic_step(sfpic_sim *s, int64_t nsteps) {
  sfpic::ErrScope es_(s);
  SF_TRY(guarded(s));
  if (nsteps < 0) return fail(SFPIC_E_INVAL, "nsteps < 0");
  return s->dispatch(
      [&](auto z) -> int { return step_impl<decltype(z)>(s, nsteps); });
}

int sfpic_sync(sfpic_sim *s) {
  sfpic::ErrScope es_(s);
  SF_TRY(guarded(s));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return SFPIC_OK;
}

int sfpic_read_field(sfpic_sim *s, int comp, double *out, size_t n) {
  sfpic::ErrScope es_(s);
  SF_TRY(guarded(s));
  if (comp < 0 || comp >= SFPIC_NCOMP || !out)
    return fail(SFPIC_E_INVAL, "bad component or NULL output");
  if (n != (size_t)s->NX * s->NY) return fail(SFPIC_E_SIZE, "n must be NX*NY");
  HIP_TRY(hipStreamSynchronize(s->stream));
  try {
    if (s->precision == SFPIC_FP64) return plane_to_host(s, comp, out);
    std::vector<float> h(n);
    SF_TRY(plane_to_host(s, comp, h.data()));
    for (size_t k = 0; k < n; ++k) out[k] = h[k];
  } catch (...) {
    return fail(SFPIC_E_NOMEM, "host allocation failed");
  }
  return SFPIC_OK;
}

int sfpic_write_field(sfpic_sim *s, int comp, const double *in, size_t n) {
  sfpic::ErrScope es_(s);
  SF_TRY(guarded(s));
  if (comp < 0 || comp >= SFPIC_NCOMP || !in)
    return fail(SFPIC_E_INVAL, "bad component or NULL input");
  if (n != (size_t)s->NX * s->NY) return fail(SFPIC_E_SIZE, "n must be NX*NY");
  HIP_TRY(hipStreamSynchronize(s->stream));
  try {
    if (s->precision == SFPIC_FP64) return plane_from_host(s, comp, in);
    std::vector<float> h(in, in + n);
    SF_TRY(plane_from_host(s, comp, h.data()));
  } catch (...) {
    return fail(SFPIC_E_NOMEM, "host allocation failed");
  }
  return SFPIC_OK;
}

int sfpic_read_total_field(sfpic_sim *s, int comp, double *out, size_t n) {
  sfpic::ErrScope es_(s);
  SF_TRY(guarded(s));
  if (comp < SFPIC_EX || comp > SFPIC_BZ || !out)
    return fail(SFPIC_E_INVAL, "component must be E or B, output non-NULL");
  if (n != (size_t)s->NX * s->NY) return fail(SFPIC_E_SIZE, "n must be NX*NY");
  // half-cell offsets of Ex Ey Ez Bx By Bz along x and y on the Yee grid
  static const int hx[6] = {1, 0, 0, 0, 1, 1}, hy[6] = {0, 1, 0, 1, 0, 1};
  const double tE = (double)s->step * s->grid.dt;
  const double t = comp < 3 ? tE : tE - 0.5 * s->grid.dt;
  // s->rho is diagnostic scratch of NY x pitch doubles; the charge
  // diagnostics clear and refill it before every use
  SF_TRY(s->dispatch([&](auto z) -> int {
    using R = decltype(z);
    HIP_TRY(launch_total_field<R>((const R *)s->planes[comp], s->pitch, s->NX,
                                  s->NY, comp, hx[comp], hy[comp],
                                  s->grid.dims, s->grid.dx, s->grid.dy, t,
                                  s->inc, s->rho, s->stream));
    return SFPIC_OK;
  }));
  HIP_TRY(hipMemcpy2DAsync(out, (size_t)s->NX * 8, s->rho,
                           (size_t)s->pitch * 8, (size_t)s->NX * 8, s->NY,
                           hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return SFPIC_OK;
}

int sfpic_set_step_index(sfpic_sim *s, int64_t step) {
  sfpic::ErrScope es_(s);
  SF_TRY(guarded(s));
  if (step < 0) return fail(SFPIC_E_INVAL, "step < 0");
  s->step = step;
  for (auto &t : s->strag_step) t = -1;  // straggler records of the old count
  s->gprev_step = -1;
  return SFPIC_OK;
}

int sfpic_particle_count(sfpic_sim *s, int species, int64_t *n) {
  sfpic::ErrScope es_(s);
  SF_TRY(guarded(s));
  if (species < 0 || species >= (int)s->sp.size() || !n)
    return fail(SFPIC_E_INVAL, "bad species");
  SpeciesState &st = s->sp[species];
  HIP_TRY(hipMemsetAsync(s->acc, 0, 8 * 8, s->stream));
  SF_TRY(s->dispatch([&](auto z) -> int {
    using R = decltype(z);
    HIP_TRY(launch_particle_sums<R>(parts<R>(st), st.n, st.n_valid,
                                    s->grid.dims, st.m, st.q, 0.0, s->acc,
                                    s->stream));
    return SFPIC_OK;
  }));
  double h[8];
  HIP_TRY(hipMemcpyAsync(h, s->acc, 8 * 8, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  *n = (int64_t)llround(h[2]);
  return SFPIC_OK;
}

int sfpic_read_particles(sfpic_sim *s, int species, double *x, double *y,
                         double *ux, double *uy, double *uz, uint32_t *id,
                         size_t capacity, size_t *n_out) {
  sfpic::ErrScope es_(s);
  SF_TRY(guarded(s));
  if (species < 0 || species >= (int)s->sp.size())
    return fail(SFPIC_E_INVAL, "bad species");
  if (!x || !ux || !uy || !uz || (s->grid.dims == 2 && !y))
    return fail(SFPIC_E_INVAL, "NULL output array");
  try {
    std::vector<double> h;
    std::vector<uint32_t> hid;
    size_t n = 0;
    SF_TRY(fetch_particles(s, s->sp[species], h, hid, n));
    size_t live = 0;
    for (size_t i = 0; i < n; ++i) live += h[i] >= 0.0;
    if (n_out) *n_out = live;
    if (live > capacity) return fail(SFPIC_E_SIZE, "capacity too small");
    size_t o = 0;
    for (size_t i = 0; i < n; ++i) {
      if (h[i] < 0.0) continue;
      x[o] = h[i];
      if (y) y[o] = h[n + i];
      ux[o] = h[2 * n + i];
      uy[o] = h[3 * n + i];
      uz[o] = h[4 * n + i];
      if (id) id[o] = hid[i];
      ++o;
    }
    return SFPIC_OK;
  } catch (...) {
    return fail(SFPIC_E_NOMEM, "host allocation failed");
  }
}

int sfpic_diagnostics(sfpic_sim *s, sfpic_diag *out) {
  sfpic::ErrScope es_(s);
  SF_TRY(guarded(s));
  if (!out) return fail(SFPIC_E_INVAL, "out is NULL");
  const double dv = s->cell_volume();
  HIP_TRY(hipMemsetAsync(s->acc, 0, 16 * 8, s->stream));
  SF_TRY(s->dispatch([&](auto z) -> int {
    using R = decltype(z);
    for (auto &st : s->sp)
      HIP_TRY(launch_particle_sums<R>(parts<R>(st), st.n, st.n_valid,
                                      s->grid.dims, st.m, st.q,
                                      st.weight * dv, s->acc, s->stream));
    HIP_TRY(launch_field_sums<R>(s->fields<R>(), s->acc, s->stream));
    const double tE = (double)s->step * s->grid.dt;
    HIP_TRY(launch_em_total<R>(s->fields<R>(), s->grid.dims, (int)s->grid.nx,
                               (int)s->grid.ny, s->grid.dx, s->grid.dy, tE,
                               tE - 0.5 * s->grid.dt, s->inc, s->acc,
                               s->stream));
    return SFPIC_OK;
  }));
  SF_TRY(deposit_rho(s, s->rho));
  SF_TRY(s->dispatch([&](auto z) -> int {
    using R = decltype(z);
    HIP_TRY(launch_gauss<R>(s->fields<R>(), s->grid.dims, (int)s->grid.nx,
                            (int)s->grid.ny, s->grid.dx, s->grid.dy, s->rho,
                            s->rho0, s->pitch, s->gprev, s->gprev_step >= 0,
                            s->acc, s->stream));
    return SFPIC_OK;
  }));
  double h[16];
  HIP_TRY(hipMemcpyAsync(h, s->acc, 16 * 8, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  out->continuity_residual = s->gprev_step >= 0 ? h[8] : 0.0;
  out->continuity_steps = s->gprev_step >= 0 ? s->step - s->gprev_step : 0;
  out->rho_abs_max = h[9];
  s->gprev_step = s->step;
  out->step = s->step;
  out->time = (double)s->step * s->grid.dt;
  out->w_kin = h[0];
  out->charge = h[1];
  out->n_alive = (int64_t)llround(h[2]);
  out->nonfinite = h[3] > 0.0 ? 1 : 0;
  out->w_em = h[4] * dv;
  out->gauss_residual = h[5];
  out->rho_max = h[6];
  out->w_em_total = h[7] * dv;
  return SFPIC_OK;
}

}  // extern "C"

// Device scratch of sfpic_histogram_noalloc: the moment accumulators and
// the bins of one histogram.  Each GPU holds its own copy for the life of
// the process; host code reaches it only through the address that
// hipGetSymbolAddress returns on that device (the array's name is not a
// device address in host code).
static __device__ __align__(256) double
    scratch[8 + SFPIC_HIST_NOALLOC_MAX_BINS];

namespace {

int check_hist_spec(const sfpic_sim *s, const sfpic_hist_spec *spec,
                    const double *out, size_t n) {
  if (!spec || !out) return fail(SFPIC_E_INVAL, "NULL argument");
  if (spec->species < 0 || spec->species >= (int)s->sp.size() ||
      spec->n_energy <= 0 || spec->n_theta <= 0 || !(spec->e_max > 0.0) ||
      spec->plane < SFPIC_ANGLE_POLAR || spec->plane > SFPIC_ANGLE_XY)
    return fail(SFPIC_E_INVAL, "bad histogram spec");
  if (n != (size_t)spec->n_energy * spec->n_theta)
    return fail(SFPIC_E_SIZE, "n must be n_energy * n_theta");
  return SFPIC_OK;
}

// Histogram of a species into the device buffer d (8 moment accumulators,
// then the bins), already zeroed on the sim's stream; copies the result to
// the caller's arrays and waits for the stream.
int histogram_into(sfpic_sim *s, const sfpic_hist_spec *spec, double *d,
                   double *out, double *moments) {
  const size_t nb = (size_t)spec->n_energy * spec->n_theta;
  SpeciesState &st = s->sp[spec->species];
  double mom[8] = {0};
  SF_TRY(s->dispatch([&](auto z) -> int {
    using R = decltype(z);
    HIP_TRY(launch_histogram<R>(parts<R>(st), st.n, st.n_valid, s->grid.dims,
                                st.m, st.weight * s->cell_volume(),
                                spec->n_energy, spec->e_max, spec->n_theta,
                                spec->ek_min, spec->plane, d + 8, d,
                                s->stream));
    HIP_TRY(hipMemcpyAsync(out, d + 8, nb * 8, hipMemcpyDeviceToHost,
                           s->stream));
    HIP_TRY(hipMemcpyAsync(mom, d, 8 * 8, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return SFPIC_OK;
  }));
  if (moments) {
    moments[0] = mom[0];
    for (int k = 1; k < 5; ++k)
      moments[k] = mom[0] > 0.0 ? mom[k] / mom[0] : 0.0;
  }
  return SFPIC_OK;
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// The scratch address on device `dev`, looked up once per device with that
// device current (the caller has set it).
int scratch_on_device(int dev, double **ptr) {
  if (dev < 0 || dev >= kMaxDevices)
    return fail(SFPIC_E_INVAL, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(SFPIC_E_DEVICE,
                  std::string("hipGetSymbolAddress(scratch): ") +
                      hipGetErrorString(e));
    g_scratch_ptr[dev] = (double *)p;
  }
  *ptr = g_scratch_ptr[dev];
  return SFPIC_OK;
}

__global__ void zero_f64(double *p, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

}  // namespace

extern "C" {

int sfpic_histogram(sfpic_sim *s, const sfpic_hist_spec *spec, double *out,
                    size_t n, double *moments) {
  sfpic::ErrScope es_(s);
  SF_TRY(guarded(s));
  SF_TRY(check_hist_spec(s, spec, out, n));
  const size_t nb = (size_t)spec->n_energy * spec->n_theta;
  double *d = (double *)s->dalloc((nb + 8) * 8);
  if (!d) return fail(SFPIC_E_NOMEM, "histogram allocation failed");
  int rc = SFPIC_OK;
  if (hipMemsetAsync(d, 0, (nb + 8) * 8, s->stream) != hipSuccess)
    rc = fail(SFPIC_E_DEVICE, "hipMemsetAsync failed");
  if (rc == SFPIC_OK) rc = histogram_into(s, spec, d, out, moments);
  s->dfree(d);
  return rc;
}

int sfpic_histogram_noalloc(sfpic_sim *s, const sfpic_hist_spec *spec,
                            double *out, size_t n, double *moments) {
  sfpic::ErrScope es_(s);
  SF_TRY(guarded(s));
  SF_TRY(check_hist_spec(s, spec, out, n));
  const size_t nb = (size_t)spec->n_energy * spec->n_theta;
  if (nb > SFPIC_HIST_NOALLOC_MAX_BINS)
    return fail(SFPIC_E_SIZE,
                "n_energy * n_theta exceeds SFPIC_HIST_NOALLOC_MAX_BINS (" +
                    std::to_string(SFPIC_HIST_NOALLOC_MAX_BINS) + ")");
  double *d = nullptr;
  SF_TRY(scratch_on_device(s->rt.device, &d));
  // the previous call's bins are still there: clear what this one uses
  const size_t nz = nb + 8;
  zero_f64<<<(unsigned)((nz + 255) / 256), 256, 0, s->stream>>>(d, nz);
  HIP_TRY(hipGetLastError());
  return histogram_into(s, spec, d, out, moments);
}

// State layout: header (magic, dims, nx, ny, precision, nspecies, step,
// element size), 9 field planes [NY][NX] in the working precision, then per
// species: the used slot count and the raw particle arrays of those slots.
int sfpic_get_state(sfpic_sim *s, void *buf, size_t *n) {
  sfpic::ErrScope es_(s);
  SF_TRY(guarded(s));
  if (!n) return fail(SFPIC_E_INVAL, "n is NULL");
  const size_t es = s->esize(), bpp = bytes_per_particle(s->precision);
  HIP_TRY(hipStreamSynchronize(s->stream));
  std::vector<uint32_t> nv(s->sp.size());
  for (size_t k = 0; k < s->sp.size(); ++k)
    HIP_TRY(hipMemcpy(&nv[k], s->sp[k].n_valid, 4, hipMemcpyDeviceToHost));
  size_t need = 8 * 8 + 9 * (size_t)s->NX * s->NY * es;
  for (size_t k = 0; k < s->sp.size(); ++k) need += 8 + (size_t)nv[k] * bpp;
  if (!buf) {
    *n = need;
    return SFPIC_OK;
  }
  if (*n < need) return fail(SFPIC_E_SIZE, "state buffer too small");
  uint8_t *p = (uint8_t *)buf;
  int64_t hdr[8] = {(int64_t)kStateMagic, s->grid.dims, s->grid.nx,
                    s->grid.ny, s->precision, (int64_t)s->sp.size(), s->step,
                    (int64_t)es};
  memcpy(p, hdr, sizeof(hdr));
  p += sizeof(hdr);
  for (int c = 0; c < 9; ++c) {
    SF_TRY(plane_to_host(s, c, p));
    p += (size_t)s->NX * s->NY * es;
  }
  for (size_t k = 0; k < s->sp.size(); ++k) {
    SpeciesState &st = s->sp[k];
    const int64_t cnt = nv[k];
    memcpy(p, &cnt, 8);
    p += 8;
    void *ptr[7];
    size_t sz[7];
    const int na = s->precision == SFPIC_FP64 ? raw_arrays(st.p64, ptr, sz)
                                              : raw_arrays(st.p32, ptr, sz);
    for (int a = 0; a < na; ++a) {
      if (cnt)
        HIP_TRY(hipMemcpy(p, ptr[a], (size_t)cnt * sz[a],
                          hipMemcpyDeviceToHost));
      p += (size_t)cnt * sz[a];
    }
  }
  *n = need;
  return SFPIC_OK;
}

int sfpic_set_state(sfpic_sim *s, const void *buf, size_t n) {
  sfpic::ErrScope es_(s);
  SF_TRY(guarded(s));
  if (!buf) return fail(SFPIC_E_INVAL, "buf is NULL");
  const size_t es = s->esize(), bpp = bytes_per_particle(s->precision);
  if (n < 64) return fail(SFPIC_E_SIZE, "state too short");
  const uint8_t *p = (const uint8_t *)buf;
  const uint8_t *end = p + n;
  int64_t hdr[8];
  memcpy(hdr, p, sizeof(hdr));
  if (hdr[0] != (int64_t)kStateMagic || hdr[1] != s->grid.dims ||
      hdr[2] != s->grid.nx || hdr[3] != s->grid.ny ||
      hdr[4] != s->precision || hdr[5] != (int64_t)s->sp.size() ||
      hdr[7] != (int64_t)es || hdr[6] < 0)
    return fail(SFPIC_E_INVAL, "state does not match this sim");
  p += 64;
  const size_t plane = (size_t)s->NX * s->NY * es;
  if ((size_t)(end - p) < 9 * plane)
    return fail(SFPIC_E_SIZE, "state truncated");
  // validate the particle blocks before touching device state
  const uint8_t *q = p + 9 * plane;
  for (auto &st : s->sp) {
    if (end - q < 8) return fail(SFPIC_E_SIZE, "state truncated");
    int64_t cnt;
    memcpy(&cnt, q, 8);
    if (cnt < 0 || cnt > st.n)
      return fail(SFPIC_E_INVAL, "particle count exceeds this sim's capacity");
    q += 8;
    if ((size_t)(end - q) < (size_t)cnt * bpp)
      return fail(SFPIC_E_SIZE, "state truncated");
    q += (size_t)cnt * bpp;
  }
  if (q != end)
    return fail(SFPIC_E_SIZE, "state size does not match this sim");
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->gprev_step = -1;
  for (int c = 0; c < 9; ++c) {
    SF_TRY(plane_from_host(s, c, p));
    p += plane;
  }
  for (auto &st : s->sp) {
    int64_t cnt;
    memcpy(&cnt, p, 8);
    p += 8;
    void *ptr[7];
    size_t sz[7];
    const int na = s->precision == SFPIC_FP64 ? raw_arrays(st.p64, ptr, sz)
                                              : raw_arrays(st.p32, ptr, sz);
    for (int a = 0; a < na; ++a) {
      if (cnt)
        HIP_TRY(hipMemcpy(ptr[a], p, (size_t)cnt * sz[a],
                          hipMemcpyHostToDevice));
      p += (size_t)cnt * sz[a];
    }
    const uint32_t nv = (uint32_t)cnt;
    HIP_TRY(hipMemcpy(st.n_valid, &nv, 4, hipMemcpyHostToDevice));
  }
  s->step = hdr[6];
  for (auto &t : s->strag_step) t = -1;  // straggler records of the old run
  SF_TRY(sort_all(s));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return SFPIC_OK;
}

int sfpic_profile(sfpic_sim *s, int enable) {
  sfpic::ErrScope es_(s);
  SF_TRY(guarded(s));
  HIP_TRY(hipStreamSynchronize(s->stream));
  if (enable) s->recycle_events();
  s->profiling = enable != 0;
  return SFPIC_OK;
}

int sfpic_profile_read(sfpic_sim *s, sfpic_kernel_stats *out) {
  sfpic::ErrScope es_(s);
  SF_TRY(guarded(s));
  if (!out) return fail(SFPIC_E_INVAL, "out is NULL");
  HIP_TRY(hipStreamSynchronize(s->stream));
  for (int c = 0; c < SFPIC_KCLASSES; ++c) {
    out->launches[c] = (int64_t)s->ev_used[c].size();
    double tot = 0.0;
    for (auto &e : s->ev_used[c]) {
      float ms = 0.0f;
      HIP_TRY(hipEventElapsedTime(&ms, e.first, e.second));
      tot += ms;
    }
    out->total_ms[c] = tot;
  }
  return SFPIC_OK;
}

int sfpic_april_field(const sfpic_incident *inc, double x, double y, double z,
                      double t, double *out) {
  if (!inc || !out) return fail(SFPIC_E_INVAL, "NULL argument");
  if (inc->kind != SFPIC_INC_APRIL_LP && inc->kind != SFPIC_INC_APRIL_RP)
    return fail(SFPIC_E_INVAL, "not an April beam");
  IncParams P;
  SF_TRY(prepare_incident(inc, P));
  cx<double> e[3], b[3];
  april_complex_fields(P, x * P.inv_a, y * P.inv_a, z * P.inv_a, t, e, b);
  for (int c = 0; c < 3; ++c) {
    out[2 * c] = e[c].r;
    out[2 * c + 1] = e[c].i;
    out[6 + 2 * c] = b[c].r;
    out[6 + 2 * c + 1] = b[c].i;
  }
  return SFPIC_OK;
}

int sfpic_april_power(const sfpic_incident *inc, double *power) {
  if (!inc || !power) return fail(SFPIC_E_INVAL, "NULL argument");
  if (inc->kind != SFPIC_INC_APRIL_LP && inc->kind != SFPIC_INC_APRIL_RP)
    return fail(SFPIC_E_INVAL, "not an April beam");
  IncParams P;
  SF_TRY(prepare_incident(inc, P));
  const double w0 = inc->w0, h = w0 / 24.0;
  const int n = 8 * 24;  // nodes -n .. n per axis
  double sum = 0.0;
  for (int j = -n; j <= n; ++j)
    for (int i = -n; i <= n; ++i) {
      cx<double> e[3], b[3];
      april_complex_fields(P, i * h * P.inv_a, j * h * P.inv_a, 0.0, 0.0, e,
                           b);
      // Re{E_x cB_y*} - Re{E_y cB_x*}
      const double f = (e[0].r * b[1].r + e[0].i * b[1].i) -
                       (e[1].r * b[0].r + e[1].i * b[0].i);
      const double wi = (i == -n || i == n) ? 0.5 : 1.0;
      const double wj = (j == -n || j == n) ? 0.5 : 1.0;
      sum += wi * wj * f;
    }
  *power = 0.5 * sum * h * h;
  return SFPIC_OK;
}

int sfpic_device_bytes(sfpic_sim *s, size_t *bytes) {
  sfpic::ErrScope es_(s);
  SF_TRY(guarded(s));
  if (!bytes) return fail(SFPIC_E_INVAL, "bytes is NULL");
  *bytes = sim_device_bytes(s);
  return SFPIC_OK;
}

void sfpic_destroy(sfpic_sim *s) {
  sfpic::ErrScope es_(s);
  sfpic::forget_handle(s);
  if (!s) return;
  (void)hipSetDevice(s->rt.device);
  (void)hipStreamSynchronize(s->stream);
  s->destroy_events();
  s->release();
  delete s;
}

}  // extern "C"
