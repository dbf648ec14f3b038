// Host runtime of sweeps: batches (sfpic_batch_*) and the request server
// (sfpic_server_*).  Both hold ordinary simulations (sfpic_sim) and advance
// all members of one precision and dimensionality with the batched launches:
// one launch per phase for the whole group, a persistent push kernel fed by
// a tile queue, a tile sort after every step that sorts only the members
// it is due for (each every sort_every of its own steps), and a HIP graph of a few steps that is captured once per
// membership and replayed.
#include "sfpic_sim.h"

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

using namespace sfpic;

namespace {

using Clock = std::chrono::steady_clock;

// Steps between the autotuner's re-timings of the sort cadence in a batch.
constexpr int64_t kRetuneSteps = 256;

double seconds_since(Clock::time_point t0) {
  return std::chrono::duration<double>(Clock::now() - t0).count();
}

// One simulation of a sweep and its bookkeeping.
struct Member {
  sfpic_sim *sim = nullptr;
  int64_t nsteps = 0;  // steps to run
  int64_t done = 0;    // steps run
  sfpic_hist_spec hist{};
  sfpic_result res{};
  std::vector<double> histogram;
  double n0 = 0.0;     // particles at creation
  bool finished = false;
};

// Particles a descriptor places (all alive at creation).
double desc_particles(const sfpic_sim_desc &d) {
  double n = 0.0;
  for (int k = 0; k < d.nspecies; ++k) {
    const sfpic_species &s = d.species[k];
    if (s.n_explicit > 0) {
      n += (double)s.n_explicit;
    } else {
      const int64_t y0 = d.grid.dims == 2 ? s.region[2] : 0;
      const int64_t y1 = d.grid.dims == 2 ? s.region[3] : 1;
      n += (double)(s.region[1] - s.region[0]) * (double)(y1 - y0) * s.ppc;
    }
  }
  return n;
}

int check_desc(const sfpic_sim_desc *d) {
  if (!d) return fail(SFPIC_E_INVAL, "descriptor is NULL");
  if (d->nsteps < 0) return fail(SFPIC_E_INVAL, "nsteps < 0");
  if (d->nspecies < 0 || d->nspecies > 8 || (d->nspecies > 0 && !d->species))
    return fail(SFPIC_E_INVAL, "nspecies must be in [0, 8]");
  if (d->hist.n_energy > 0 &&
      (d->hist.species < 0 || d->hist.species >= d->nspecies ||
       d->hist.n_theta <= 0 || !(d->hist.e_max > 0.0) ||
       d->hist.plane < SFPIC_ANGLE_POLAR || d->hist.plane > SFPIC_ANGLE_XY))
    return fail(SFPIC_E_INVAL, "bad histogram spec");
  return SFPIC_OK;
}

// Members of one (precision, dims) class and their device tables.
struct Group {
  int precision = SFPIC_FP64, dims = 2;
  std::vector<Member *> members;
  int tx = 0, ty = 0;
  // sort cadence: the default 4 (measured on the laser-focus sweep: every
  // 4 steps beats 8 once the beam has heated the plasma); the autotuner
  // times 2, 4 and 8 on the run's own steps and re-times them as the run
  // goes on, unless the runtime fixed it
  SortRule rule{4};
  bool cadence_fixed = false;
  int graph_steps = 8;  // steps per captured graph (a tick of the server)
  bool tuned = false;
  struct Trial {
    int tx, ty, c;
    double ns;
  };
  std::vector<Trial> trials;
  // device tables (one allocation) and their host image
  void *dbuf = nullptr;
  size_t dbytes = 0;
  std::vector<uint8_t> image;
  size_t off_ms = 0, off_pj = 0;
  int np = 0;
  BatchView<double> v64{};
  BatchView<float> v32{};
  size_t lds = 0;
  int grid = 0;
  // every member's beam is an April beam at the particles: the push runs
  // the kernel compiled for the LP and RP beams alone
  bool april = false;
  // some member takes the incident field sampled on the nodes
  bool on_nodes = false;
  hipGraphExec_t exec = nullptr;
  bool stale = true;  // tables (and graph) must be rebuilt before launching
  bool ran = false;   // work was launched since the host view was refreshed
  // members in the order of the device tables (as of the last build);
  // members added since are not on the device yet
  std::vector<Member *> built;
};

// Shared engine of batches and servers: one device, one stream.
struct Engine {
  sfpic_runtime rt{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int cus = 256;
  size_t max_lds = 64 * 1024;
  std::vector<Group> groups;
  int64_t graph_launches = 0;

  ~Engine() { release(); }

  int init(const sfpic_runtime *r, bool force_own_stream) {
    if (r) rt = *r;
    HIP_TRY(hipSetDevice(rt.device));
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount,
                              rt.device) == hipSuccess && v > 0)
      cus = v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock,
                              rt.device) == hipSuccess && v > 0)
      max_lds = (size_t)v;
    if (rt.stream && !force_own_stream) {
      stream = (hipStream_t)rt.stream;
    } else {
      HIP_TRY(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
      own_stream = true;
    }
    rt.stream = stream;
    return SFPIC_OK;
  }

  void release() {
    for (auto &g : groups) drop_tables(g);
    groups.clear();
    if (own_stream && stream) (void)hipStreamDestroy(stream);
    stream = nullptr;
    own_stream = false;
  }

  void drop_tables(Group &g) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g.exec = nullptr;
    if (g.dbuf) (void)hipFree(g.dbuf);
    g.dbuf = nullptr;
    g.dbytes = 0;
    g.stale = true;
  }

  Group &group_for(int precision, int dims) {
    for (auto &g : groups)
      if (g.precision == precision && g.dims == dims) return g;
    groups.emplace_back();
    Group &g = groups.back();
    g.precision = precision;
    g.dims = dims;
    if (rt.sort_every > 0) {
      g.rule = SortRule{rt.sort_every};
      g.cadence_fixed = true;
    }
    return g;
  }

  // Sort scratch and straggler list for the species past the first of a
  // member, sized for its current tile geometry.
  static int ensure_species_scratch(sfpic_sim *s) {
    const size_t nk1 = (size_t)s->tg.nkeys + 1;
    for (size_t k = 1; k < s->sp.size(); ++k) {
      SpeciesState &st = s->sp[k];
      const size_t cnt = (size_t)(st.n > 0 ? st.n : 1);
      if (!st.bstrag) {
        st.bstrag = (uint32_t *)s->dalloc(cnt * 4);
        st.bss.key = (uint32_t *)s->dalloc(cnt * 4);
        st.bss.rank = (uint32_t *)s->dalloc(cnt * 4);
        if (!st.bstrag || !st.bss.key || !st.bss.rank)
          return fail(SFPIC_E_NOMEM, "batch scratch allocation failed");
      }
      if (st.bss_nk1 < nk1) {
        if (st.bss.counts) s->dfree(st.bss.counts);
        if (st.bss.block_sums) s->dfree(st.bss.block_sums);
        st.bss.counts = (uint32_t *)s->dalloc(nk1 * 4);
        st.bss.block_sums =
            (uint32_t *)s->dalloc(((nk1 + 1023) / 1024 + 1) * 4);
        if (!st.bss.counts || !st.bss.block_sums)
          return fail(SFPIC_E_NOMEM, "batch scratch allocation failed");
        st.bss_nk1 = nk1;
      }
    }
    return SFPIC_OK;
  }

  // Build the device tables of a group from the host view of its members.
  template <typename R>
  int build_t(Group &g, BatchView<R> &v) {
    const int nm = (int)g.members.size();
    int np = 0;
    for (Member *m : g.members) {
      SF_TRY(ensure_species_scratch(m->sim));
      np += (int)m->sim->sp.size();
    }
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    size_t off = 0;
    const size_t o_ms = off;
    off = al(off + (size_t)nm * sizeof(MemberState));
    const size_t o_fj = off;
    off = al(off + (size_t)nm * sizeof(FieldJob<R>));
    const size_t o_pj = off;
    off = al(off + (size_t)np * sizeof(PushJob<R>));
    size_t o_tab[3];
    const size_t nent[3] = {(size_t)nm + 1, (size_t)nm + 1, (size_t)np + 1};
    for (int t = 0; t < 3; ++t) {
      o_tab[t] = off;
      off = al(off + nent[t] * 4);
    }
    const size_t o_cnt = off;
    off = al(off + (size_t)(2 + np + 8) * 4);
    const size_t o_due = off;
    off = al(off + (size_t)(np > 0 ? np : 1) * 4);
    const size_t o_item = off;
    off = al(off + (size_t)(np + 1) * 4);
    if (off > g.dbytes) {
      HIP_TRY(hipStreamSynchronize(stream));
      if (g.dbuf) (void)hipFree(g.dbuf);
      g.dbuf = nullptr;
      g.dbytes = 0;
      HIP_TRY(hipMalloc(&g.dbuf, off));
      g.dbytes = off;
    }
    g.image.assign(off, 0);
    uint8_t *h = g.image.data();
    uint8_t *d = (uint8_t *)g.dbuf;
    MemberState *ms = (MemberState *)(h + o_ms);
    FieldJob<R> *fj = (FieldJob<R> *)(h + o_fj);
    PushJob<R> *pj = (PushJob<R> *)(h + o_pj);
    uint32_t *tab[3];
    for (int t = 0; t < 3; ++t) tab[t] = (uint32_t *)(h + o_tab[t]);
    for (int t = 0; t < 3; ++t) tab[t][0] = 0;
    int j = 0;
    size_t lds = 0, dyn = 0;
    bool april = true, on_nodes = false;
    for (int mi = 0; mi < nm; ++mi) {
      Member *m = g.members[mi];
      sfpic_sim *s = m->sim;
      const sfpic_grid &gr = s->grid;
      // the push items of the member's current sort (the batch rebuilds
      // them after each of its sorts)
      SF_TRY(refresh_items(s));
      ms[mi].step = s->step;
      ms[mi].steps_left = m->nsteps - m->done;
      ms[mi].since_sort = 0;
      ms[mi].sort_due = 0;
      FieldJob<R> &F = fj[mi];
      F.f = s->fields<R>();
      F.dt = R(gr.dt);
      F.cx = R(gr.dt / gr.dx);
      F.cy = g.dims == 2 ? R(gr.dt / gr.dy) : R(0);
      F.kx = R((gr.dt - gr.dx) / (gr.dt + gr.dx));
      F.ky = R((gr.dt - gr.dy) / (gr.dt + gr.dy));
      F.member = mi;
      F.job0 = j;
      F.njobs = (int)s->sp.size();
      const uint32_t NX = (uint32_t)s->NX, NY = (uint32_t)s->NY;
      const uint32_t nfar = g.dims == 2 ? ((NX + 63) / 64) * ((NY + 3) / 4)
                                        : (NX + 255) / 256;
      const uint32_t namp = g.dims == 2
                                ? ((NX - 2 + 63) / 64) * ((NY - 2 + 3) / 4)
                                : (NX - 2 + 255) / 256;
      tab[0][mi + 1] = tab[0][mi] + nfar;
      tab[1][mi + 1] = tab[1][mi] + namp;
      const size_t l = g.precision == SFPIC_FP64
                           ? push_lds_bytes<double>(s->tg, g.dims, true)
                           : push_lds_bytes<float>(s->tg, g.dims, true);
      const size_t ld = g.precision == SFPIC_FP64
                            ? push_dyn_lds_bytes<double>(s->tg, g.dims, true)
                            : push_dyn_lds_bytes<float>(s->tg, g.dims, true);
      lds = l > lds ? l : lds;
      dyn = ld > dyn ? ld : dyn;
      april = april && !s->inc.on_nodes &&
              (s->inc.kind == SFPIC_INC_APRIL_LP ||
               s->inc.kind == SFPIC_INC_APRIL_RP);
      on_nodes = on_nodes || (s->inc.on_nodes && !s->sp.empty());
      for (size_t k = 0; k < s->sp.size(); ++k, ++j) {
        SpeciesState &st = s->sp[k];
        PushJob<R> &P = pj[j];
        P.f = s->fields<R>();
        P.pa[0] = parts<R>(st);
        P.pa[1] = parts_alt<R>(st);
        P.start = st.start;
        P.n_valid = st.n_valid;
        P.strag = k == 0 ? s->strag : st.bstrag;
        P.ss = k == 0 ? s->ss : st.bss;
        if (k == 0) {
          P.ss.key = s->ss.key;
          P.ss.rank = s->ss.rank;
        }
        P.tg = s->tg;
        P.pp.dt = gr.dt;
        P.pp.dx = gr.dx;
        P.pp.dy = gr.dy;
        P.pp.inv_dx = 1.0 / gr.dx;
        P.pp.inv_dy = 1.0 / gr.dy;
        P.pp.qm = st.q / st.m;
        P.pp.qw = st.q * st.weight;
        P.pp.time = 0.0;
        P.pp.nx = (int)gr.nx;
        P.pp.ny = (int)gr.ny;
        P.inc = s->inc;
        P.n_slots = (uint32_t)st.n;
        P.member = mi;
        P.cur = 0;
        P.items = st.items;
        P.n_items = st.n_items;
        P.kmax = s->item_max;
        tab[2][j + 1] = tab[2][j] + (uint32_t)s->tg.ntiles;
      }
    }
    if (lds > max_lds) return fail(SFPIC_E_INVAL, "tile too large for LDS");
    // queued work of this group may still read the old tables
    HIP_TRY(hipStreamSynchronize(stream));
    HIP_TRY(hipMemcpy(g.dbuf, h, off, hipMemcpyHostToDevice));
    v.fjobs = (const FieldJob<R> *)(d + o_fj);
    v.pjobs = (PushJob<R> *)(d + o_pj);
    v.ms = (MemberState *)(d + o_ms);
    v.nmembers = nm;
    v.nf = nm;
    v.np = np;
    v.far_off = (const uint32_t *)(d + o_tab[0]);
    v.amp_off = (const uint32_t *)(d + o_tab[1]);
    v.tile_off = (const uint32_t *)(d + o_tab[2]);
    v.counters = (uint32_t *)(d + o_cnt);
    v.due = (uint32_t *)(d + o_due);
    v.item_off = (uint32_t *)(d + o_item);
    v.n_far = tab[0][nm];
    v.n_amp = tab[1][nm];
    v.n_tiles = tab[2][np];
    g.off_ms = o_ms;
    g.off_pj = o_pj;
    g.np = np;
    g.built = g.members;
    g.lds = dyn;  // passed at launch; static chunk buffers come on top
    g.april = april && g.dims == 2;
    g.on_nodes = on_nodes;
    const int per_cu = batch_push_blocks_per_cu(g.precision == SFPIC_FP64,
                                                g.dims, g.april, dyn);
    int grid = cus * (per_cu > 0 ? per_cu : 1);
    if ((uint32_t)grid > v.n_tiles) grid = (int)(v.n_tiles > 0 ? v.n_tiles : 1);
    g.grid = grid;
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g.exec = nullptr;
    g.stale = false;
    return SFPIC_OK;
  }

  int build(Group &g) {
    SF_TRY(pull(g));
    if (g.members.empty()) {
      g.built.clear();
      g.stale = false;
      return SFPIC_OK;
    }
    return g.precision == SFPIC_FP64 ? build_t<double>(g, g.v64)
                                     : build_t<float>(g, g.v32);
  }

  // One step of every running member of the group.
  template <typename R>
  int enqueue_step_t(Group &g, const BatchView<R> &v) {
    HIP_TRY(launch_fill_u32(v.counters, 0u, (size_t)(2 + v.np + 8), stream));
    HIP_TRY(launch_batch_faraday<R>(v, g.dims, stream));
    if (g.on_nodes) HIP_TRY(launch_batch_incident_nodes<R>(v, g.dims, stream));
    HIP_TRY(launch_batch_item_offsets<R>(v, stream));
    HIP_TRY(launch_batch_push<R>(v, g.dims, g.april, g.lds, g.grid, stream));
    HIP_TRY(launch_batch_stragglers<R>(v, g.dims, stream));
    HIP_TRY(launch_batch_ampere<R>(v, g.dims, stream));
    HIP_TRY(launch_batch_advance<R>(v, g.rule, stream));
    HIP_TRY(launch_batch_sort<R>(v, g.dims, stream));
    return SFPIC_OK;
  }

  // `c` steps, each followed by the sort of the members it is due for.
  int enqueue_superstep(Group &g, int c) {
    for (int k = 0; k < c; ++k) {
      if (g.precision == SFPIC_FP64)
        SF_TRY(enqueue_step_t<double>(g, g.v64));
      else
        SF_TRY(enqueue_step_t<float>(g, g.v32));
    }
    return SFPIC_OK;
  }

  // Launch one super-step of graph_steps steps, replaying the captured
  // graph unless graphs are off.
  int launch_superstep(Group &g) {
    if (g.stale) SF_TRY(build(g));
    if (g.members.empty()) return SFPIC_OK;
    g.ran = true;
    if (rt.flags & SFPIC_RT_NO_GRAPH) return enqueue_superstep(g, g.graph_steps);
    if (!g.exec) {
      hipGraph_t graph = nullptr;
      HIP_TRY(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
      const int r = enqueue_superstep(g, g.graph_steps);
      const hipError_t e = hipStreamEndCapture(stream, &graph);
      if (r != SFPIC_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return r;
      }
      HIP_TRY(e);
      const hipError_t ei = hipGraphInstantiate(&g.exec, graph, nullptr,
                                                nullptr, 0);
      (void)hipGraphDestroy(graph);
      HIP_TRY(ei);
    }
    HIP_TRY(hipGraphLaunch(g.exec, stream));
    ++graph_launches;
    return SFPIC_OK;
  }

  // Step counters and steps run of the members, read back from the device
  // (waits for the stream).  The device tables stay valid.
  int counts(Group &g) {
    HIP_TRY(hipStreamSynchronize(stream));
    const int nm = (int)g.built.size();
    if (!g.ran || nm == 0) return SFPIC_OK;
    std::vector<MemberState> ms(nm);
    HIP_TRY(hipMemcpy(ms.data(), (uint8_t *)g.dbuf + g.off_ms,
                      nm * sizeof(MemberState), hipMemcpyDeviceToHost));
    for (int mi = 0; mi < nm; ++mi) {
      Member *m = g.built[mi];
      m->sim->step = ms[mi].step;
      m->done = m->nsteps - ms[mi].steps_left;
    }
    return SFPIC_OK;
  }

  // Bring the host view of the members fully up to date with the device:
  // counters and which particle buffer is current after the device-side
  // sorts.  Afterwards the device tables disagree with the host view, so
  // they are rebuilt before the next launch.  Waits for the stream.
  template <typename R>
  int pull_t(Group &g) {
    SF_TRY(counts(g));
    std::vector<PushJob<R>> pj(g.np);
    HIP_TRY(hipMemcpy(pj.data(), (uint8_t *)g.dbuf + g.off_pj,
                      g.np * sizeof(PushJob<R>), hipMemcpyDeviceToHost));
    int j = 0;
    for (Member *m : g.built) {
      sfpic_sim *s = m->sim;
      s->since_sort = s->sort_every;
      for (size_t k = 0; k < s->sp.size(); ++k, ++j)
        if (pj[j].cur) std::swap(parts<R>(s->sp[k]), parts_alt<R>(s->sp[k]));
    }
    g.ran = false;
    g.stale = true;
    return SFPIC_OK;
  }

  int pull(Group &g) {
    if (!g.ran || g.built.empty()) {
      g.ran = false;
      return SFPIC_OK;
    }
    return g.precision == SFPIC_FP64 ? pull_t<double>(g) : pull_t<float>(g);
  }

  static bool running(const Member *m) { return m->done < m->nsteps; }

  // Particle pushes of the next super-step of the group (approximate: the
  // particle count at creation).
  static double superstep_pushes(const Group &g) {
    double p = 0.0;
    for (const Member *m : g.members) {
      const int64_t left = m->nsteps - m->done;
      const int64_t k = left < g.graph_steps ? left : g.graph_steps;
      if (k > 0) p += m->n0 * (double)k;
    }
    return p;
  }

  // One autotuner trial: the next super-step of the run (graph_steps real
  // steps, eager launches) with tile tx x ty (members re-tiled if it
  // changes) and the group's current sort cadence, timed with events;
  // ns = nanoseconds per particle push (-1 when no member has steps left).
  int trial(Group &g, int tx, int ty, hipEvent_t e0, hipEvent_t e1,
            double &ns) {
    SF_TRY(pull(g));
    if (tx != g.tx || ty != g.ty) {
      for (Member *m : g.members) SF_TRY(sim_retile(m->sim, tx, ty, 0));
      g.tx = tx;
      g.ty = ty;
    }
    g.stale = true;
    SF_TRY(build(g));
    const double pushes = superstep_pushes(g);
    if (pushes <= 0.0) {
      ns = -1.0;
      return SFPIC_OK;
    }
    HIP_TRY(hipEventRecord(e0, stream));
    g.ran = true;
    SF_TRY(enqueue_superstep(g, g.graph_steps));
    HIP_TRY(hipEventRecord(e1, stream));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    ns = ms * 1e6 / pushes;
    g.trials.push_back({tx, ty, g.rule.c_max, ns});
    return SFPIC_OK;
  }

  // Time each candidate in `rounds` passes of alternating order (the slow
  // drift of the particle distribution during the run then favours none)
  // and return the index with the lowest mean time per push (-1: none ran).
  // set(k) makes candidate k current before its trial.
  template <typename Set>
  int best_of(Group &g, size_t n, int rounds, Set set, int &r) {
    hipEvent_t e0, e1;
    r = SFPIC_OK;
    if (hipEventCreate(&e0) != hipSuccess) {
      r = fail(SFPIC_E_DEVICE, "hipEventCreate failed");
      return -1;
    }
    if (hipEventCreate(&e1) != hipSuccess) {
      (void)hipEventDestroy(e0);
      r = fail(SFPIC_E_DEVICE, "hipEventCreate failed");
      return -1;
    }
    std::vector<double> sum(n, 0.0);
    std::vector<int> cnt(n, 0);
    for (int round = 0; round < rounds && r == SFPIC_OK; ++round)
      for (size_t q = 0; q < n && r == SFPIC_OK; ++q) {
        const size_t k = round % 2 == 0 ? q : n - 1 - q;
        int tx = g.tx, ty = g.ty;
        set(k, tx, ty);
        double ns = 0.0;
        r = trial(g, tx, ty, e0, e1, ns);
        if (ns > 0.0) {
          sum[k] += ns;
          cnt[k] += 1;
        }
      }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    int bt = -1;
    double best = 1e300;
    for (size_t k = 0; k < n; ++k)
      if (cnt[k] > 0 && sum[k] / cnt[k] < best) {
        best = sum[k] / cnt[k];
        bt = (int)k;
      }
    return bt;
  }

  // Autotuner: the particle tile, then the sort cadence, each candidate
  // timed on real super-steps of the run (graph_steps steps).
  int tune(Group &g, int rounds) {
    std::vector<std::pair<int, int>> tiles;
    if (g.dims == 2)
      tiles = {{16, 16}, {16, 8}, {32, 8}, {8, 8}};
    else
      tiles = {{256, 1}, {128, 1}, {512, 1}};
    std::vector<std::pair<int, int>> ok;
    for (auto t : tiles) {
      TileGeom tt{};
      tt.tx = t.first;
      tt.ty = t.second;
      tt.slack = g.members.empty() ? 1 : g.members[0]->sim->tg.slack;
      const size_t l = g.precision == SFPIC_FP64
                           ? push_lds_bytes<double>(tt, g.dims, true)
                           : push_lds_bytes<float>(tt, g.dims, true);
      if (l <= max_lds) ok.push_back(t);
    }
    if (ok.empty()) return SFPIC_OK;
    int r = SFPIC_OK;
    const int bt = best_of(g, ok.size(), rounds,
                           [&](size_t k, int &tx, int &ty) {
                             tx = ok[k].first;
                             ty = ok[k].second;
                           },
                           r);
    if (r != SFPIC_OK) return r;
    SF_TRY(pull(g));
    if (bt >= 0 && (ok[bt].first != g.tx || ok[bt].second != g.ty)) {
      for (Member *m : g.members)
        SF_TRY(sim_retile(m->sim, ok[bt].first, ok[bt].second, 0));
      g.tx = ok[bt].first;
      g.ty = ok[bt].second;
    }
    g.tuned = true;
    g.stale = true;
    if (!g.cadence_fixed) SF_TRY(tune_cadence(g, rounds));
    return SFPIC_OK;
  }

  // The sort cadence among 2, 4 and 8 steps, timed on the run's next
  // super-steps with the group's tile (each trial a super-step of 8 steps,
  // so every candidate sorts at least once in it).
  int tune_cadence(Group &g, int rounds) {
    static const int kCadences[3] = {2, 4, 8};
    int r = SFPIC_OK;
    const int bc = best_of(g, 3, rounds,
                           [&](size_t k, int &, int &) {
                             g.rule = SortRule{kCadences[k]};
                           },
                           r);
    if (r != SFPIC_OK) return r;
    if (bc >= 0) g.rule = SortRule{kCadences[bc]};
    g.stale = true;
    return SFPIC_OK;
  }

  // Result of a finished member (diagnostics and histogram on the stream).
  // A member whose fields or momenta are no longer finite fails alone with
  // SFPIC_E_NUMERIC (its result keeps the diagnostics that show it).
  static int finish_member(Member *m) {
    sfpic_result &res = m->res;
    res.steps = m->done;
    SF_TRY(sfpic_diagnostics(m->sim, &res.diag));
    res.pushes = (double)m->done * 0.5 * (m->n0 + (double)res.diag.n_alive);
    res.device_bytes = sim_device_bytes(m->sim);
    if (res.diag.nonfinite) {
      res.status = SFPIC_E_NUMERIC;
      snprintf(res.error, sizeof(res.error),
               "non-finite fields or momenta after %lld steps",
               (long long)m->done);
      return fail(SFPIC_E_NUMERIC, res.error);
    }
    if (m->hist.n_energy > 0) {
      const size_t nb = (size_t)m->hist.n_energy * m->hist.n_theta;
      m->histogram.assign(nb, 0.0);
      SF_TRY(sfpic_histogram(m->sim, &m->hist, m->histogram.data(), nb,
                             res.moments));
    }
    res.status = SFPIC_OK;
    return SFPIC_OK;
  }
};

// Create one member simulation on the engine's stream.
int create_member(Engine &eng, const sfpic_sim_desc &d, Member &m) {
  SF_TRY(check_desc(&d));
  sfpic_runtime rt = eng.rt;
  rt.stream = eng.stream;
  sfpic_sim *s = nullptr;
  SF_TRY(sfpic_create(&d.grid, d.species, d.nspecies, &d.incident,
                      d.precision, &rt, &s));
  m.sim = s;
  // the batched FP32 members take 2 cells of drift (the single sims' FP32
  // form takes 1): on the sweep, whose beams heat the plasma within a few
  // steps, the wider window keeps enough particles off the slower straggler
  // path to outweigh its larger LDS footprint (17.5 against 15.6 G pushes/s
  // with 1 on the 64-member, 200-step sweep at cadence 4)
  if (d.precision == SFPIC_FP32 && d.grid.dims == 2 && s->tg.slack < 2) {
    const int r = sim_retile(s, s->tg.tx, s->tg.ty, 2);
    if (r != SFPIC_OK) {
      sfpic_destroy(s);
      m.sim = nullptr;
      return r;
    }
  }
  m.nsteps = d.nsteps;
  m.done = 0;
  m.hist = d.hist;
  // particles placed (a density profile places fewer than region x ppc)
  m.n0 = 0.0;
  for (const auto &st : s->sp) m.n0 += (double)st.n;
  return SFPIC_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------
struct sfpic_batch {
  Engine eng;
  std::vector<std::unique_ptr<Member>> members;
  bool ran = false;
  double run_ms = 0.0, step_ms = 0.0, pushes = 0.0;
};

namespace {

int batch_run_impl(sfpic_batch *b) {
  Engine &eng = b->eng;
  const auto t0 = Clock::now();
  const bool autotune = !(eng.rt.flags & SFPIC_RT_NO_AUTOTUNE) &&
                        eng.rt.tile_x <= 0 && eng.rt.tile_y <= 0;
  hipEvent_t es, ee;
  HIP_TRY(hipEventCreate(&es));
  HIP_TRY(hipEventCreate(&ee));
  HIP_TRY(hipEventRecord(es, eng.stream));
  for (auto &g : eng.groups) {
    if (g.members.empty()) continue;
    g.tx = g.members[0]->sim->tg.tx;
    g.ty = g.members[0]->sim->tg.ty;
    // the trials are real steps of the run; keep them to a quarter of it
    int64_t longest = 0;
    for (Member *m : g.members)
      longest = std::max<int64_t>(longest, m->nsteps - m->done);
    const int rounds = longest >= 256 ? 2 : (longest >= 128 ? 1 : 0);
    if (autotune && rounds > 0) SF_TRY(eng.tune(g, rounds));
    // the particles heat and spread as the run goes on, which moves the
    // best cadence: re-time the cadences every kRetuneSteps steps
    const bool retune = autotune && rounds > 0 && !g.cadence_fixed;
    const int64_t chunk = kRetuneSteps / g.graph_steps;
    for (;;) {
      SF_TRY(eng.pull(g));
      bool any = false;
      for (Member *m : g.members) any = any || Engine::running(m);
      if (!any) break;
      int64_t left = 0;
      for (Member *m : g.members) {
        const int64_t l = m->nsteps - m->done;
        left = l > left ? l : left;
      }
      int64_t reps = (left + g.graph_steps - 1) / g.graph_steps;
      // enough steps after this chunk for a cadence pass and a chunk more
      const bool again = retune && reps > chunk + 3 + chunk / 2;
      if (again) reps = chunk;
      // these super-steps back to back, then one pull
      for (int64_t k = 0; k < reps; ++k) {
        SF_TRY(eng.launch_superstep(g));
      }
      SF_TRY(eng.pull(g));
      if (again) SF_TRY(eng.tune_cadence(g, 1));
    }
  }
  HIP_TRY(hipEventRecord(ee, eng.stream));
  HIP_TRY(hipEventSynchronize(ee));
  float ms = 0.0f;
  HIP_TRY(hipEventElapsedTime(&ms, es, ee));
  (void)hipEventDestroy(es);
  (void)hipEventDestroy(ee);
  b->step_ms = ms;
  const double t_step = seconds_since(t0);
  b->pushes = 0.0;
  for (auto &mp : b->members) {
    Member *m = mp.get();
    const int r = Engine::finish_member(m);
    if (r != SFPIC_OK && r != SFPIC_E_NUMERIC) return r;  // a device error
    m->res.t_submit = 0.0;
    m->res.t_start = 0.0;
    m->res.t_done = t_step;
    m->finished = true;
    b->pushes += m->res.pushes;
  }
  b->run_ms = seconds_since(t0) * 1e3;
  b->ran = true;
  return SFPIC_OK;
}

}  // namespace

extern "C" {

int sfpic_desc_footprint(const sfpic_sim_desc *desc, const sfpic_runtime *rt,
                         size_t *bytes) {
  try {
    SF_TRY(check_desc(desc));
    return sim_footprint(&desc->grid, desc->species, desc->nspecies,
                         desc->precision, rt, bytes);
  } catch (...) {
    return fail(SFPIC_E_NOMEM, "exception in footprint");
  }
}

int sfpic_batch_create(int n, const sfpic_sim_desc *descs,
                       const sfpic_runtime *rt, sfpic_batch **out) {
  try {
    if (!out) return fail(SFPIC_E_INVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || !descs) return fail(SFPIC_E_INVAL, "need n >= 1 members");
    for (int i = 0; i < n; ++i) SF_TRY(check_desc(&descs[i]));
    std::unique_ptr<sfpic_batch> b(new (std::nothrow) sfpic_batch());
    if (!b) return fail(SFPIC_E_NOMEM, "host allocation failed");
    SF_TRY(b->eng.init(rt, false));
    // members sorted by decreasing particle count, so the persistent push
    // starts on the largest members and the tail of the queue is small work
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
      return desc_particles(descs[a]) > desc_particles(descs[c]);
    });
    b->members.resize(n);
    for (int i = 0; i < n; ++i) b->members[i].reset(new Member());
    for (int k = 0; k < n; ++k) {
      const int i = order[k];
      const int r = create_member(b->eng, descs[i], *b->members[i]);
      if (r != SFPIC_OK) {
        const std::string msg = std::string("member ") + std::to_string(i) +
                                ": " + sfpic_last_error(nullptr);
        for (auto &m : b->members)
          if (m->sim) sfpic_destroy(m->sim);
        return fail(r, msg);
      }
      Group &g = b->eng.group_for(descs[i].precision, descs[i].grid.dims);
      g.members.push_back(b->members[i].get());
    }
    *out = b.release();
    return SFPIC_OK;
  } catch (...) {
    return fail(SFPIC_E_NOMEM, "exception during batch create");
  }
}

int sfpic_batch_run(sfpic_batch *b) {
  sfpic::ErrScope es_(b);
  if (!b) return fail(SFPIC_E_INVAL, "batch is NULL");
  if (b->ran) return fail(SFPIC_E_STATE, "batch already ran");
  try {
    HIP_TRY(hipSetDevice(b->eng.rt.device));
    return batch_run_impl(b);
  } catch (...) {
    return fail(SFPIC_E_NOMEM, "exception during batch run");
  }
}

int sfpic_batch_result(sfpic_batch *b, int i, sfpic_result *out) {
  sfpic::ErrScope es_(b);
  if (!b || !out) return fail(SFPIC_E_INVAL, "NULL argument");
  if (i < 0 || i >= (int)b->members.size())
    return fail(SFPIC_E_INVAL, "member index out of range");
  if (!b->ran) return fail(SFPIC_E_STATE, "batch has not run");
  *out = b->members[i]->res;
  return SFPIC_OK;
}

int sfpic_batch_member(sfpic_batch *b, int i, sfpic_sim **sim) {
  sfpic::ErrScope es_(b);
  if (!b || !sim) return fail(SFPIC_E_INVAL, "NULL argument");
  if (i < 0 || i >= (int)b->members.size())
    return fail(SFPIC_E_INVAL, "member index out of range");
  *sim = b->members[i]->sim;
  return SFPIC_OK;
}

int sfpic_batch_stats(sfpic_batch *b, sfpic_batch_info *out) {
  sfpic::ErrScope es_(b);
  if (!b || !out) return fail(SFPIC_E_INVAL, "NULL argument");
  memset(out, 0, sizeof(*out));
  int gi = 0;
  for (auto &g : b->eng.groups) {
    if (gi >= SFPIC_MAX_GROUPS) break;
    out->precision[gi] = g.precision;
    out->dims[gi] = g.dims;
    out->members[gi] = (int32_t)g.members.size();
    out->tile_x[gi] = g.tx;
    out->tile_y[gi] = g.ty;
    out->sort_every[gi] = g.rule.c_max;
    out->tuned[gi] = g.tuned ? 1 : 0;
    out->push_workgroups[gi] = g.grid;
    const int nt = (int)std::min<size_t>(g.trials.size(), SFPIC_MAX_CANDIDATES);
    out->n_candidates[gi] = nt;
    for (int k = 0; k < nt; ++k) {
      out->cand_tile_x[gi][k] = g.trials[k].tx;
      out->cand_tile_y[gi][k] = g.trials[k].ty;
      out->cand_sort_every[gi][k] = g.trials[k].c;
      out->cand_ns_per_push[gi][k] = g.trials[k].ns;
    }
    ++gi;
  }
  out->ngroups = gi;
  out->run_ms = b->run_ms;
  out->step_ms = b->step_ms;
  out->pushes = b->pushes;
  out->graph_launches = b->eng.graph_launches;
  return SFPIC_OK;
}

void sfpic_batch_destroy(sfpic_batch *b) {
  sfpic::ErrScope es_(b);
  sfpic::forget_handle(b);
  if (!b) return;
  (void)hipSetDevice(b->eng.rt.device);
  if (b->eng.stream) (void)hipStreamSynchronize(b->eng.stream);
  for (auto &m : b->members)
    if (m->sim) sfpic_destroy(m->sim);
  b->members.clear();
  b->eng.release();
  delete b;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Server
// ---------------------------------------------------------------------------
namespace {

struct Request {
  uint64_t ticket = 0;
  sfpic_sim_desc desc{};
  std::vector<sfpic_species> species;
  std::vector<std::vector<double>> arrays;  // copies of explicit particles
  size_t footprint = 0;
  int state = SFPIC_REQ_QUEUED;
  Member m;
  int group = -1;
};

}  // namespace

struct sfpic_server {
  Engine eng;
  size_t budget = 0, in_use = 0, peak = 0;
  int max_slots = 1;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request *> queue;
  std::map<uint64_t, std::unique_ptr<Request>> all;
  std::vector<Request *> running;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread worker;
  Clock::time_point t0 = Clock::now();
  std::vector<double> latencies;
  int64_t submitted = 0, admitted = 0, completed = 0, failed = 0, ticks = 0;
  int32_t max_running = 0;
  double pushes = 0.0, busy_s = 0.0;
  int init_status = SFPIC_OK;
  std::string init_error;
  bool ready = false;
};

namespace {

void server_fail_request(sfpic_server *S, Request *q, int code,
                         const std::string &msg) {
  q->m.res.status = code;
  snprintf(q->m.res.error, sizeof(q->m.res.error), "%s", msg.c_str());
  q->m.res.t_done = seconds_since(S->t0);
  q->state = SFPIC_REQ_FAILED;
  S->failed += 1;
}

// Remove finished members from their groups (the group tables are rebuilt
// at the next tick).
void drop_from_group(Engine &eng, Request *q) {
  if (q->group < 0) return;
  Group &g = eng.groups[q->group];
  q->group = -1;
  g.members.erase(std::remove(g.members.begin(), g.members.end(), &q->m),
                  g.members.end());
  g.stale = true;
  if (g.exec) {
    (void)hipGraphExecDestroy(g.exec);
    g.exec = nullptr;
  }
}

void server_loop(sfpic_server *S) {
  Engine &eng = S->eng;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->init_status = eng.init(&eng.rt, true);
    if (S->init_status != SFPIC_OK) S->init_error = sfpic_last_error(nullptr);
    S->ready = true;
  }
  S->cv_done.notify_all();
  if (S->init_status != SFPIC_OK) return;
  for (;;) {
    std::vector<Request *> admit;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      if (S->stop) break;
      // FIFO admission by slots and device footprint
      while (!S->queue.empty() &&
             (int)(S->running.size() + admit.size()) < S->max_slots &&
             S->in_use + S->queue.front()->footprint <= S->budget) {
        Request *q = S->queue.front();
        S->queue.pop_front();
        S->in_use += q->footprint;
        S->peak = S->in_use > S->peak ? S->in_use : S->peak;
        q->m.res.t_start = seconds_since(S->t0);
        admit.push_back(q);
      }
      if (admit.empty() && S->running.empty()) {
        S->cv_work.wait(lk, [&] { return S->stop || !S->queue.empty(); });
        continue;
      }
    }
    // create admitted members (their particles are placed on the stream)
    for (Request *q : admit) {
      int r = create_member(eng, q->desc, q->m);
      std::lock_guard<std::mutex> lk(S->mu);
      if (r != SFPIC_OK) {
        S->in_use -= q->footprint;
        server_fail_request(S, q, r, sfpic_last_error(nullptr));
        continue;
      }
      q->state = SFPIC_REQ_RUNNING;
      S->admitted += 1;
      Group &g = eng.group_for(q->desc.precision, q->desc.grid.dims);
      q->group = (int)(&g - eng.groups.data());
      g.members.push_back(&q->m);
      g.stale = true;
      if (g.exec) {
        (void)hipGraphExecDestroy(g.exec);
        g.exec = nullptr;
      }
      S->running.push_back(q);
      S->max_running = std::max<int32_t>(S->max_running,
                                         (int32_t)S->running.size());
    }
    S->cv_done.notify_all();
    if (S->running.empty()) continue;
    // one tick: a super-step of every group
    const auto tt = Clock::now();
    double tick_pushes = 0.0;
    int rc = SFPIC_OK;
    for (auto &g : eng.groups) {
      if (g.members.empty()) continue;
      if (g.tx == 0) {
        g.tx = g.members[0]->sim->tg.tx;
        g.ty = g.members[0]->sim->tg.ty;
      }
      tick_pushes += Engine::superstep_pushes(g);
      rc = eng.launch_superstep(g);
      if (rc != SFPIC_OK) break;
    }
    for (auto &g : eng.groups) {
      if (rc != SFPIC_OK) break;
      rc = eng.counts(g);
    }
    // harvest finished members (or fail every running one on an error); the
    // groups that lose members refresh their host view first
    std::vector<Request *> finished;
    for (Request *q : S->running)
      if (rc != SFPIC_OK || !Engine::running(&q->m)) finished.push_back(q);
    for (Request *q : finished) {
      if (rc != SFPIC_OK || q->group < 0) break;
      rc = eng.pull(eng.groups[q->group]);
    }
    const std::string err = rc != SFPIC_OK ? sfpic_last_error(nullptr) : "";
    if (rc != SFPIC_OK) {
      finished.clear();
      for (Request *q : S->running) finished.push_back(q);
    }
    for (Request *q : finished) {
      int r = rc;
      if (r == SFPIC_OK) r = Engine::finish_member(&q->m);
      const std::string msg = r != SFPIC_OK ? sfpic_last_error(nullptr) : "";
      drop_from_group(eng, q);
      sfpic_destroy(q->m.sim);
      q->m.sim = nullptr;
      std::lock_guard<std::mutex> lk(S->mu);
      S->in_use -= q->footprint;
      S->running.erase(std::find(S->running.begin(), S->running.end(), q));
      if (r != SFPIC_OK) {
        server_fail_request(S, q, r, rc != SFPIC_OK ? err : msg);
      } else {
        q->m.res.t_done = seconds_since(S->t0);
        q->state = SFPIC_REQ_DONE;
        S->completed += 1;
        S->latencies.push_back(q->m.res.t_done - q->m.res.t_submit);
      }
    }
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->ticks += 1;
      S->pushes += tick_pushes;
      S->busy_s += seconds_since(tt);
    }
    S->cv_done.notify_all();
  }
  // shut down: release resident members
  for (Request *q : S->running) {
    if (q->m.sim) sfpic_destroy(q->m.sim);
    q->m.sim = nullptr;
  }
  S->running.clear();
  eng.release();
}

double percentile(std::vector<double> v, double p) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  // nearest rank
  size_t k = (size_t)ceil(p * (double)v.size());
  if (k < 1) k = 1;
  if (k > v.size()) k = v.size();
  return v[k - 1];
}

}  // namespace

extern "C" {

int sfpic_server_create(size_t hbm_budget, int max_slots,
                        const sfpic_runtime *rt, sfpic_server **out) {
  try {
    if (!out) return fail(SFPIC_E_INVAL, "out is NULL");
    *out = nullptr;
    if (max_slots < 1) return fail(SFPIC_E_INVAL, "max_slots must be >= 1");
    std::unique_ptr<sfpic_server> S(new (std::nothrow) sfpic_server());
    if (!S) return fail(SFPIC_E_NOMEM, "host allocation failed");
    if (rt) S->eng.rt = *rt;
    S->eng.rt.stream = nullptr;
    S->eng.rt.alloc = nullptr;
    S->eng.rt.free = nullptr;
    S->eng.rt.alloc_ctx = nullptr;
    HIP_TRY(hipSetDevice(S->eng.rt.device));
    if (hbm_budget == 0) {
      size_t fr = 0, tot = 0;
      HIP_TRY(hipMemGetInfo(&fr, &tot));
      hbm_budget = (size_t)(0.9 * (double)fr);
    }
    S->budget = hbm_budget;
    S->max_slots = max_slots;
    S->t0 = Clock::now();
    sfpic_server *p = S.get();
    S->worker = std::thread(server_loop, p);
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_done.wait(lk, [&] { return S->ready; });
    }
    if (S->init_status != SFPIC_OK) {
      S->worker.join();
      return fail(S->init_status, S->init_error);
    }
    *out = S.release();
    return SFPIC_OK;
  } catch (...) {
    return fail(SFPIC_E_NOMEM, "exception during server create");
  }
}

int sfpic_server_submit(sfpic_server *S, const sfpic_sim_desc *desc,
                        uint64_t *ticket) {
  sfpic::ErrScope es_(S);
  try {
    if (!S || !ticket) return fail(SFPIC_E_INVAL, "NULL argument");
    SF_TRY(check_desc(desc));
    std::unique_ptr<Request> q(new Request());
    q->desc = *desc;
    q->species.assign(desc->species, desc->species + desc->nspecies);
    for (auto &sp : q->species) {
      if (sp.n_explicit <= 0) continue;
      const size_t n = (size_t)sp.n_explicit;
      const double *src[5] = {sp.x, sp.y, sp.ux, sp.uy, sp.uz};
      const double **dst[5] = {&sp.x, &sp.y, &sp.ux, &sp.uy, &sp.uz};
      for (int a = 0; a < 5; ++a) {
        if (!src[a]) continue;
        q->arrays.emplace_back(src[a], src[a] + n);
        *dst[a] = q->arrays.back().data();
      }
    }
    q->desc.species = q->species.data();
    SF_TRY(sim_footprint(&q->desc.grid, q->desc.species, q->desc.nspecies,
                         q->desc.precision, &S->eng.rt, &q->footprint));
    if (q->footprint > S->budget)
      return fail(SFPIC_E_INVAL, "request exceeds the server's HBM budget");
    std::lock_guard<std::mutex> lk(S->mu);
    q->ticket = S->next_ticket++;
    q->m.res.t_submit = seconds_since(S->t0);
    *ticket = q->ticket;
    S->queue.push_back(q.get());
    S->all[q->ticket] = std::move(q);
    S->submitted += 1;
    S->cv_work.notify_all();
    return SFPIC_OK;
  } catch (...) {
    return fail(SFPIC_E_NOMEM, "exception during submit");
  }
}

int sfpic_server_poll(sfpic_server *S, uint64_t ticket, int *state) {
  sfpic::ErrScope es_(S);
  if (!S || !state) return fail(SFPIC_E_INVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end()) return fail(SFPIC_E_INVAL, "unknown ticket");
  *state = it->second->state;
  return SFPIC_OK;
}

int sfpic_server_wait(sfpic_server *S, uint64_t ticket, double timeout_s) {
  sfpic::ErrScope es_(S);
  if (!S) return fail(SFPIC_E_INVAL, "server is NULL");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end()) return fail(SFPIC_E_INVAL, "unknown ticket");
  Request *q = it->second.get();
  const bool ok = S->cv_done.wait_for(
      lk, std::chrono::duration<double>(timeout_s > 0.0 ? timeout_s : 0.0),
      [&] {
        return q->state == SFPIC_REQ_DONE || q->state == SFPIC_REQ_FAILED;
      });
  return ok ? SFPIC_OK : fail(SFPIC_E_BUSY, "request not finished in time");
}

int sfpic_server_result(sfpic_server *S, uint64_t ticket, sfpic_result *out) {
  sfpic::ErrScope es_(S);
  if (!S || !out) return fail(SFPIC_E_INVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end()) return fail(SFPIC_E_INVAL, "unknown ticket");
  Request *q = it->second.get();
  if (q->state != SFPIC_REQ_DONE && q->state != SFPIC_REQ_FAILED)
    return fail(SFPIC_E_STATE, "request not finished");
  *out = q->m.res;
  return SFPIC_OK;
}

int sfpic_server_histogram(sfpic_server *S, uint64_t ticket, double *out,
                           size_t n) {
  sfpic::ErrScope es_(S);
  if (!S || !out) return fail(SFPIC_E_INVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end()) return fail(SFPIC_E_INVAL, "unknown ticket");
  Request *q = it->second.get();
  if (q->state != SFPIC_REQ_DONE)
    return fail(SFPIC_E_STATE, "request not done");
  if (n != q->m.histogram.size())
    return fail(SFPIC_E_SIZE, "n must be n_energy * n_theta");
  std::copy(q->m.histogram.begin(), q->m.histogram.end(), out);
  return SFPIC_OK;
}

int sfpic_server_stats(sfpic_server *S, sfpic_server_info *out) {
  sfpic::ErrScope es_(S);
  if (!S || !out) return fail(SFPIC_E_INVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  memset(out, 0, sizeof(*out));
  out->submitted = S->submitted;
  out->admitted = S->admitted;
  out->completed = S->completed;
  out->failed = S->failed;
  out->queued = (int64_t)S->queue.size();
  out->running = (int64_t)S->running.size();
  out->p50_s = percentile(S->latencies, 0.50);
  out->p99_s = percentile(S->latencies, 0.99);
  double sum = 0.0, mx = 0.0;
  for (double v : S->latencies) {
    sum += v;
    mx = v > mx ? v : mx;
  }
  out->mean_s = S->latencies.empty() ? 0.0 : sum / S->latencies.size();
  out->max_s = mx;
  out->pushes = S->pushes;
  out->busy_s = S->busy_s;
  out->pushes_per_s = S->busy_s > 0.0 ? S->pushes / S->busy_s : 0.0;
  out->bytes_in_use = S->in_use;
  out->bytes_peak = S->peak;
  out->budget = S->budget;
  out->ticks = S->ticks;
  out->max_running = S->max_running;
  return SFPIC_OK;
}

void sfpic_server_destroy(sfpic_server *S) {
  sfpic::ErrScope es_(S);
  sfpic::forget_handle(S);
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  if (S->worker.joinable()) S->worker.join();
  delete S;
}

}  // extern "C"
