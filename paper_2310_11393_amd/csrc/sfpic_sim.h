// Host-side state of one simulation, shared by the single-simulation calls
// and the batch / server runtime.  Internal: not part of the public ABI.
#pragma once

#include "../../include/sfpic.h"
#include "sfpic_common.h"

#include <string>
#include <utility>
#include <vector>

namespace sfpic {

// Record msg as the calling thread's last error, and as the last error of
// every handle whose entry point is active on this thread, and return code.
int fail(int code, const std::string &msg);

// Marks an ABI entry point's handle active on this thread for its lifetime.
struct ErrScope {
  explicit ErrScope(const void *handle);
  ~ErrScope();
  ErrScope(const ErrScope &) = delete;
  ErrScope &operator=(const ErrScope &) = delete;
};

// Drop the recorded message of a handle that is being destroyed.
void forget_handle(const void *handle);

// Column offsets of a density profile along x over region columns
// [x0, x1): off[c + 1] - off[c] particles per cell of column c
// (SFPIC_PROFILE_*); fails on bad profile parameters.
int profile_offsets(int32_t profile, double center, double fwhm, double order,
                    double xmin, int64_t x0, int64_t x1, double dx, int ppc,
                    std::vector<uint32_t> &off);

// Placement with a profile: particle i sits in row i / per_row of the region
// (y0 + row) and in the column whose offsets bracket i % per_row.
template <typename R>
hipError_t launch_init_particles_profile(const Particles<R> &p, int64_t n,
                                         int dims, int64_t x0, int ncx,
                                         int64_t y0, const uint32_t *off,
                                         uint32_t per_row, double sigma,
                                         uint64_t seed, uint32_t key1,
                                         hipStream_t st);

// dst[j pitch + i] = F_scatt + F_inc of stored component comp (0..5) at its
// Yee node (hx, hy: half-cell offsets along x and y), every element of an
// NX x NY plane, FP64, incident field at time t.
template <typename R>
hipError_t launch_total_field(const R *src, int pitch, int NX, int NY,
                              int comp, int hx, int hy, int dims, double dx,
                              double dy, double t, const IncParams &inc,
                              double *dst, hipStream_t st);

#define HIP_TRY(expr)                                                   \
  do {                                                                  \
    hipError_t e_ = (expr);                                             \
    if (e_ != hipSuccess)                                               \
      return ::sfpic::fail(SFPIC_E_DEVICE, std::string(#expr) + ": " +  \
                                               hipGetErrorString(e_));  \
  } while (0)

#define SF_TRY(expr)               \
  do {                             \
    int r_ = (expr);               \
    if (r_ != SFPIC_OK) return r_; \
  } while (0)

struct SpeciesState {
  double q = -1.0, m = 1.0, weight = 0.0;
  int64_t n = 0;               // slots (capacity)
  uint32_t *n_valid = nullptr; // device: slots in use (live or removed)
  uint32_t *start = nullptr;   // device: cell start offsets (nkeys + 1)
  // device: work items of the single-sim push (allocated by its first step)
  uint32_t *items = nullptr, *n_items = nullptr;
  size_t items_words = 0;
  Particles<double> p64{}, p64_alt{};
  Particles<float> p32{}, p32_alt{};
  // Sort scratch and straggler list of a species other than the first when
  // its sim is advanced in a batch (all species of a member are pushed and
  // sorted by the same launches there); bss_nk1 is the key capacity.
  SortScratch bss{};
  uint32_t *bstrag = nullptr;
  size_t bss_nk1 = 0;
};

template <typename R>
Particles<R> &parts(SpeciesState &st);
template <>
inline Particles<double> &parts<double>(SpeciesState &st) { return st.p64; }
template <>
inline Particles<float> &parts<float>(SpeciesState &st) { return st.p32; }
template <typename R>
Particles<R> &parts_alt(SpeciesState &st);
template <>
inline Particles<double> &parts_alt<double>(SpeciesState &st) {
  return st.p64_alt;
}
template <>
inline Particles<float> &parts_alt<float>(SpeciesState &st) {
  return st.p32_alt;
}

}  // namespace sfpic

// Particles per work item of the push: a tile holding more is split over
// several workgroups.  The FP64 push stages its tile's field window again for
// every item, so its items stay large; the FP32 push only clears and flushes
// its current window per item, and the finer split balances dense tiles
// (4096^2 RP run: 29.6 -> 30.4 G pushes/s over 200 steps against 8192).
#ifndef SFPIC_ITEM_PARTICLES_F64
#define SFPIC_ITEM_PARTICLES_F64 8192
#endif
#ifndef SFPIC_ITEM_PARTICLES_F32
#define SFPIC_ITEM_PARTICLES_F32 4096
#endif
constexpr uint32_t kItemParticlesF64 = SFPIC_ITEM_PARTICLES_F64;
constexpr uint32_t kItemParticlesF32 = SFPIC_ITEM_PARTICLES_F32;
inline uint32_t default_item_particles(int precision) {
  return precision == SFPIC_FP64 ? kItemParticlesF64 : kItemParticlesF32;
}

struct sfpic_sim {
  using SpeciesState = sfpic::SpeciesState;
  using IncParams = sfpic::IncParams;
  using TileGeom = sfpic::TileGeom;
  using SortScratch = sfpic::SortScratch;
  template <typename R>
  using Fields = sfpic::Fields<R>;
  sfpic_grid grid{};
  int precision = SFPIC_FP64;
  sfpic_runtime rt{};
  hipStream_t stream = nullptr;
  int NX = 0, NY = 0, pitch = 0;
  int64_t step = 0;
  IncParams inc{};
  Fields<double> f64{};
  Fields<float> f32{};
  void *planes[12] = {};
  void *inc_planes[3] = {};  // sampled incident E_x, E_y, B_z (on_nodes)
  std::vector<SpeciesState> sp;
  TileGeom tg{};
  SortScratch ss{};
  int sort_every = 8;
  int64_t since_sort = 0;
  // Adaptive cadence (the default runtime): from sort_every steps after a
  // sort up to sort_max, the next sort waits while the push two steps
  // earlier listed no more than a fraction kStragSortFrac of any species'
  // slots as stragglers.  The counts come back through pinned host memory,
  // one ring slot per step, with an event each.
  bool sort_adaptive = false;
  int sort_max = 16;
  static constexpr int kStragRing = 4;
  uint32_t *strag_host = nullptr;  // kStragRing x species counts (pinned)
  hipEvent_t strag_ev[kStragRing] = {};
  int64_t strag_step[kStragRing] = {-1, -1, -1, -1};
  uint32_t item_max = kItemParticlesF64;  // particles per push work item
  uint32_t *strag = nullptr, *n_strag = nullptr;  // straggler list
  double *rho0 = nullptr, *rho = nullptr, *acc = nullptr;
  // per-node Gauss defect of the last diagnostics call and its step (-1:
  // none, or the state has been changed since)
  double *gprev = nullptr;
  int64_t gprev_step = -1;
  std::vector<std::pair<void *, size_t>> allocs;
  // profiling: event pairs per kernel class, recorded in launch order
  bool profiling = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_used[SFPIC_KCLASSES];
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_free;

  template <typename R>
  Fields<R> &fields();

  std::pair<hipEvent_t, hipEvent_t> take_events() {
    if (!ev_free.empty()) {
      auto e = ev_free.back();
      ev_free.pop_back();
      return e;
    }
    std::pair<hipEvent_t, hipEvent_t> e{nullptr, nullptr};
    (void)hipEventCreate(&e.first);
    (void)hipEventCreate(&e.second);
    return e;
  }
  void recycle_events() {
    for (auto &v : ev_used) {
      for (auto &e : v) ev_free.push_back(e);
      v.clear();
    }
  }
  void destroy_events() {
    for (auto &e : strag_ev)
      if (e) (void)hipEventDestroy(e);
    if (strag_host) (void)hipHostFree(strag_host);
    strag_host = nullptr;
    recycle_events();
    for (auto &e : ev_free) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
    ev_free.clear();
  }
  void *dalloc(size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    void *p = nullptr;
    if (rt.alloc) {
      p = rt.alloc(bytes, rt.alloc_ctx);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
      p = nullptr;
    }
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
        allocs.erase(allocs.begin() + k);
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
  size_t esize() const { return precision == SFPIC_FP64 ? 8 : 4; }
  double cell_volume() const {
    return grid.dims == 2 ? grid.dx * grid.dy : grid.dx;
  }
  // Run f with a value of the working precision's type.
  template <typename F>
  int dispatch(F &&f) {
    return precision == SFPIC_FP64 ? f(0.0) : f(0.0f);
  }
};

template <>
inline sfpic::Fields<double> &sfpic_sim::fields<double>() {
  return f64;
}
template <>
inline sfpic::Fields<float> &sfpic_sim::fields<float>() {
  return f32;
}

namespace sfpic {

// Internal operations used by the batch and server runtime.
int sort_all(sfpic_sim *s);
// (Re)allocate every species' push work items for the tiling and particle
// count and build them from the current sort.
int refresh_items(sfpic_sim *s);
// Set the particle tile to tx x ty cells with drift allowance slack (0:
// keep the current one), reallocating the sort arrays when the key count
// grows, and re-sort every species.
int sim_retile(sfpic_sim *s, int tx, int ty, int slack);
// Device bytes held by the sim.
size_t sim_device_bytes(const sfpic_sim *s);
// Device bytes a sim created from these arguments would hold (without
// creating it), with the runtime's tile.
int sim_footprint(const sfpic_grid *grid, const sfpic_species *species,
                  int nspecies, sfpic_precision precision,
                  const sfpic_runtime *rt, size_t *bytes);

}  // namespace sfpic
