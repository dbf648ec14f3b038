/*
 * sfpic.h -- C ABI of the scattered-field particle-in-cell library for AMD
 * MI355X (gfx950).
 *
 * The method (Lytova et al., arXiv 2310.11393, Sec. 2): the total field is
 * split as F = F_inc + F_scatt.  F_inc is a known vacuum solution evaluated in
 * closed form wherever it is needed; only F_scatt lives on a staggered Yee grid
 * and is advanced by Maxwell's equations with the plasma current as its only
 * source.  Macro-particles are pushed in F_inc + F_scatt taken at their own
 * position and time, and their charge-conserving current feeds F_scatt.
 *
 * One step n -> n+1 (state E^n, B^{n-1/2}, x^n, u^{n-1/2}; t^n = n dt):
 *   Faraday B^{n+1/2} = B^{n-1/2} - dt curl E^n; Bbar^n = (B^{n-1/2} +
 *   B^{n+1/2})/2; order-2 gather of E^n, Bbar^n at x^n; add F_inc(x^n, t^n);
 *   Boris push; x^{n+1} = x^n + dt u^{n+1/2}/gamma; Esirkepov current
 *   J^{n+1/2}; particles leaving the physical box are removed after they
 *   deposit; Ampere E^{n+1} = E^n + dt (curl B^{n+1/2} - J^{n+1/2}) with a
 *   first-order Mur absorbing condition on tangential E at the outer faces.
 *
 * Units (Table 1 of the paper): c = eps0 = 1; lengths in lambda/(2 pi), time
 * in 1/omega, E in m_e c omega / e, B in m_e omega / e, density in n_c,
 * current in e n_c c, charge in e, mass in m_e.  Momenta are u = gamma v.
 *
 * Axes: propagation +x, linear polarization along y, z ignorable.  The
 * paper's (x, y, z) map to (y, z, x) here (a cyclic permutation).
 *
 * Grid layout: dims = 1 or 2, nx (x ny) physical cells of size dx (x dy) and
 * SFPIC_GUARD guard cells on every side.  Array index I of a field holds the
 * primal node x = (I - GUARD) dx or the dual node x = (I - GUARD + 1/2) dx;
 * staggering Ex(I+1/2,J) Ey(I,J+1/2) Ez(I,J) Bx(I,J+1/2) By(I+1/2,J)
 * Bz(I+1/2,J+1/2), J co-located with E.  Host-side field arrays are row-major
 * [J][I] with I fastest, NX = nx + 2 GUARD, NY = ny + 2 GUARD (1 in 1D).
 * Physical particle box: [0, nx dx) x [0, ny dy).
 *
 * Conventions shared by every call:
 *   - Every call returns SFPIC_OK (0) or a negative status; no C++ exception
 *     crosses the ABI.  sfpic_last_error(handle) describes the last failure
 *     on a handle, sfpic_last_error(NULL) that of the calling thread.
 *   - Host buffers belong to the caller; inputs are read only during the call
 *     and outputs are written into caller-sized buffers (SFPIC_E_SIZE when
 *     the size does not match).
 *   - Device memory and handles belong to the library; *_destroy releases
 *     them.  A handle is used by one host thread at a time.
 *   - Work is enqueued on the runtime's HIP stream; sfpic_sync waits for it.
 *     Read calls synchronize the stream themselves.
 *   - Precision is fixed at create: SFPIC_FP64 stores everything in double;
 *     SFPIC_FP32 stores fields and momenta in float and positions as an
 *     integer cell plus a float offset, keeping double for the incident-field
 *     phase and for all diagnostics.
 */
#ifndef SFPIC_H
#define SFPIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SFPIC_OK 0
#define SFPIC_E_INVAL (-1)   /* invalid argument                          */
#define SFPIC_E_SIZE (-2)    /* caller buffer size mismatch               */
#define SFPIC_E_NOMEM (-3)   /* device or host allocation failed          */
#define SFPIC_E_DEVICE (-4)  /* HIP runtime error                         */
#define SFPIC_E_NUMERIC (-5) /* non-finite values found                   */
#define SFPIC_E_BUSY (-6)    /* resource limit reached (try again later)  */
#define SFPIC_E_STATE (-7)   /* call not valid in the current state       */

#define SFPIC_GUARD 3

enum {
  SFPIC_EX = 0, SFPIC_EY, SFPIC_EZ, SFPIC_BX, SFPIC_BY, SFPIC_BZ,
  SFPIC_JX, SFPIC_JY, SFPIC_JZ, SFPIC_NCOMP
};

typedef enum { SFPIC_FP64 = 0, SFPIC_FP32 = 1 } sfpic_precision;

/* Incident-field models (the paper's closed forms). */
enum {
  SFPIC_INC_NONE = 0,
  /* Sec. 3.1 exact plane-wave pulse along +x: E_y = B_z =
   * a0 sin(t - t0 - x) 2^{-4 (t - t0 - x)^2 / fwhm_t^2}. */
  SFPIC_INC_PLANE_PULSE_1D = 1,
  /* Sec. 4.1 April isodiffracting pulse, linear polarization (along y). */
  SFPIC_INC_APRIL_LP = 2,
  /* April pulse, radial polarization (TM01, electric Hertz vector along the
   * propagation axis; cited in Sec. 4, derived here from the same phasor). */
  SFPIC_INC_APRIL_RP = 3,
  /* Sec. 3.2 paraxial 2D Gaussian beam along +x, polarized along y, with a
   * Gaussian time envelope and the first-order longitudinal field: a0 (E0),
   * w0 (waist), fwhm_t and t0 (envelope 2^{-4 (t - t0 - z)^2 / fwhm_t^2}),
   * focus (x_focus, y_focus); z is the distance from the focus along x.
   * Single simulations only: batches and servers reject it. */
  SFPIC_INC_GAUSS_2D = 4
};

typedef struct {
  int32_t dims;      /* 1 or 2                                            */
  int64_t nx, ny;    /* physical cells (ny ignored in 1D)                 */
  double dx, dy;     /* cell sizes                                        */
  double dt;         /* time step; must satisfy the Yee CFL limit         */
} sfpic_grid;

/* One mobile particle species.  Either generated on the device (n_explicit
 * == 0: exactly ppc particles per cell of region, uniform in the cell,
 * Philox4x32-10 keyed by (seed, species_index), counter = particle id;
 * Maxwellian momenta of temperature_ev or cold) or given explicitly
 * (n_explicit > 0: arrays of length n_explicit in physical units, each
 * particle carrying density `weight`).  An immobile neutralizing background
 * equal to minus the initial charge density is implied. */
typedef struct {
  double q, m;              /* charge (e), mass (m_e)                      */
  double density;           /* generated: n_c units, weight = density/ppc */
  int64_t region[4];        /* generated: cells [x0,x1) x [y0,y1)         */
  int32_t ppc;              /* generated: particles per cell              */
  double temperature_ev;    /* generated: 0 = cold                        */
  uint64_t seed;            /* generated: Philox key word 0               */
  int32_t species_index;    /* generated: Philox key word 1               */
  int64_t n_explicit;       /* > 0: explicit arrays below                 */
  double weight;            /* explicit: density per macro-particle      */
  const double *x, *y, *ux, *uy, *uz; /* explicit (y ignored in 1D)      */
  /* generated, optional density profile along x (the propagation axis),
   * see SFPIC_PROFILE_* (Sec. 3.1) */
  int32_t profile;
  double profile_center, profile_fwhm, profile_order, profile_xmin;
} sfpic_species;

/* sfpic_species.profile: SFPIC_PROFILE_UNIFORM places ppc particles in every
 * cell of the region.  SFPIC_PROFILE_SUPERGAUSS follows the plasma profile of
 * Sec. 3.1 along x: n(x) = density 2^{-|2 (x - profile_center) /
 * profile_fwhm|^profile_order} for x > profile_xmin and 0 otherwise; cell
 * column c of the region (centre x_c) holds floor(ppc n(x_c) / density +
 * 1/2) particles per cell, each of weight density / ppc.  Particle ids run
 * over region rows (y; y then z in 3D) outermost, then columns, a column's
 * particles consecutive; positions and momenta use the same Philox streams
 * as the uniform placement, by id. */
#define SFPIC_PROFILE_UNIFORM 0
#define SFPIC_PROFILE_SUPERGAUSS 1

/* Incident field parameters.  April models: w0 is the waist (the complex
 * source parameter a follows from k^2 w0^2 = 2 (sqrt(1 + (ka)^2) - 1),
 * Sec. 4.1), s the Poisson-spectrum parameter (a positive integer here),
 * phi0 the constant phase, (x_focus, y_focus) the focus in the plane,
 * t_focus the focal time.  a0 is the modulus of the complex on-axis field
 * component at the focus at the focal time (E along y for LP, E along x for
 * RP).  Plane pulse: a0, fwhm_t (FWHM of the field envelope) and t0.
 * on_nodes: 0 (default) evaluates the closed form at each particle (Sec. 2:
 * the scattered field is interpolated and added to the incident field at the
 * macro-particle); 1 samples the incident field where the Yee grid stores
 * each component, at t^n, and the particles gather it with the scattered
 * field (the field superimposed on the grid fields, as the paper's
 * implementation does; O(dx^2) interpolation error, fewer closed-form
 * evaluations).  Single simulations only: batches and servers reject 1. */
typedef struct {
  int32_t kind;
  double a0;
  double fwhm_t, t0;
  double w0, s, phi0;
  double x_focus, y_focus, t_focus;
  int32_t on_nodes;
  double z_focus;  /* 3D runs (sfpic3_*): focus coordinate along z        */
} sfpic_incident;

/* Device allocator callback (e.g. a framework's caching allocator).  Must
 * return device memory of at least `bytes`, aligned to 256 bytes, or NULL. */
typedef void *(*sfpic_alloc_fn)(size_t bytes, void *ctx);
typedef void (*sfpic_free_fn)(void *ptr, size_t bytes, void *ctx);

typedef struct {
  void *stream;          /* hipStream_t; NULL = the null stream            */
  sfpic_alloc_fn alloc;  /* NULL = hipMalloc                               */
  sfpic_free_fn free;    /* NULL = hipFree                                 */
  void *alloc_ctx;
  int32_t tile_x, tile_y; /* particle tile in cells; 0 = library default   */
  int32_t sort_every;     /* steps between tile sorts; 0 = default: single
                             sims adaptive, sorting 4 (FP32 form) or 8
                             (FP64) to 16 steps after the last sort, as
                             soon as the push two steps earlier listed
                             more than 2^-10 of a species' particles as
                             stragglers; batches and servers autotuned or
                             4                                            */
  int32_t device;         /* HIP device ordinal                            */
  int32_t flags;          /* SFPIC_RT_* (batches and servers)              */
  int32_t item_particles; /* a tile holding more particles is pushed by
                             several workgroups, this many each (single
                             sims, batch and server members); 0 = default
                             (8192 in FP64, 4096 in the FP32 form);
                             must be >= 64                               */
} sfpic_runtime;

/* runtime.flags: launch a batch's steps one by one instead of replaying a
 * captured HIP graph of 8 steps. */
#define SFPIC_RT_NO_GRAPH 1
/* runtime.flags: never run the batch autotuner (the tile then comes from
 * tile_x, tile_y or the library default). */
#define SFPIC_RT_NO_AUTOTUNE 2

typedef struct {
  int64_t step;          /* steps taken                                    */
  double time;           /* step * dt                                      */
  int64_t n_alive;       /* live macro-particles, all species              */
  double w_kin;          /* sum w m (gamma - 1) dV                         */
  double w_em;           /* 1/2 sum (E^n . E^n + B^{n-1/2} . B^{n-1/2}) dV,
                            scattered field only                           */
  double charge;         /* sum q w dV of live particles                   */
  double gauss_residual; /* max |div_h E - (rho - rho_0)| over nodes at
                            least 4 cells inside the physical box          */
  double rho_max;        /* max |rho - rho_0| over the same nodes          */
  int32_t nonfinite;     /* 1 if a non-finite field or momentum was seen   */
  double w_em_total;     /* 1/2 sum |E_s^n + E_inc(t^n)|^2 + |B_s^{n-1/2} +
                            B_inc(t^{n-1/2})|^2 dV over the physical nodes,
                            each component at its Yee node: energy of the
                            total field F_inc + F_scatt (Sec. 2)            */
  /* Discrete continuity since the previous sfpic_diagnostics call on this
   * sim (Sec. 2 and the charge-conserving deposition it names): with the
   * per-node Gauss defect g^n = div_h E^n - (rho^n - rho_0), the maximum of
   * |g^n - g^m| = |[div_h E^n - div_h E^m] - [rho^n - rho^m]| over the
   * nodes of gauss_residual, m the step of that previous call; a field
   * written in between (sfpic_write_field) enters it like any other change
   * of E.  Zero, with continuity_steps = 0, on the first call and after
   * sfpic_set_state or sfpic_set_step_index.  A non-finite value makes
   * this and gauss_residual +inf.  3D: sfpic3_diagnostics, the same with
   * the 3D divergence (the first call allocates one FP64 field array).    */
  double continuity_residual;
  double rho_abs_max;        /* max |rho^n| over the same nodes            */
  int64_t continuity_steps;  /* n - m                                      */
} sfpic_diag;

typedef struct {
  int32_t species;
  int32_t n_energy;  /* linear kinetic-energy bins over [0, e_max) (m_e c^2) */
  double e_max;
  int32_t n_theta;   /* angle bins over [0, 180] degrees                   */
  double ek_min;     /* moments use particles with E_k > ek_min            */
  int32_t plane;     /* SFPIC_ANGLE_*: which angle the histogram bins      */
} sfpic_hist_spec;

/* sfpic_hist_spec.plane.  SFPIC_ANGLE_POLAR: the angle between the momentum
 * and the propagation axis +x, atan2(sqrt(u_y^2 + u_z^2), u_x).
 * SFPIC_ANGLE_XZ: the angle from +x of the momentum projected on the plane
 * of x and z, atan2(|u_z|, u_x): the plane through the propagation axis
 * across the linear polarization (the paper's (y, z) plane, in which
 * Secs. 4.2 and 4.3 bin their electron spectra, 20 degrees forward and
 * backward read as 20 and 160 degrees here).  SFPIC_ANGLE_XY: projected on
 * the plane of x and y (the polarization plane), atan2(|u_y|, u_x). */
#define SFPIC_ANGLE_POLAR 0
#define SFPIC_ANGLE_XZ 1
#define SFPIC_ANGLE_XY 2

typedef struct sfpic_sim sfpic_sim;

/* Create a simulation: allocate and zero the scattered field (Sec. 2: the
 * fields of the unperturbed plasma are zero at the initial time), place the
 * particles, set u^{-1/2} = u^0.  nspecies in [1, 8] (0 allowed: vacuum).
 * Returns SFPIC_E_INVAL for bad sizes or parameters, SFPIC_E_NOMEM when
 * device memory is short, SFPIC_E_DEVICE on HIP errors. */
int sfpic_create(const sfpic_grid *grid, const sfpic_species *species,
                 int nspecies, const sfpic_incident *incident,
                 sfpic_precision precision, const sfpic_runtime *runtime,
                 sfpic_sim **out);

/* Enqueue nsteps >= 0 steps on the runtime stream (asynchronous).  Each is
 * the scattered-field step of Sec. 2 (operations and order at the top of
 * this header: Yee update of F_scatt only, particles pushed in F_inc +
 * F_scatt at their position, charge-conserving current into F_scatt).
 * SFPIC_E_INVAL for nsteps < 0, SFPIC_E_DEVICE on a launch error. */
int sfpic_step(sfpic_sim *sim, int64_t nsteps);

/* Wait for all work queued on the sim's stream (runtime plumbing; no
 * passage of the paper defines it).  SFPIC_E_DEVICE if the work failed. */
int sfpic_sync(sfpic_sim *sim);

/* Copy one scattered-field component (SFPIC_EX .. SFPIC_JZ) to out, as
 * double, row-major [NY][NX] including guards; n must be NX * NY.  J holds
 * J^{n-1/2}, the current deposited by the last step.  This is F_scatt, the
 * only field the grid holds (Sec. 2); sfpic_read_total_field adds F_inc. */
int sfpic_read_field(sfpic_sim *sim, int comp, double *out, size_t n);

/* Overwrite one field component from a host array laid out as for
 * sfpic_read_field (for example to seed a run from an external state, such
 * as the pulse written on the grid at t = 0 by the full-field comparison
 * model of Sec. 3.1; Sec. 2 starts from a zero scattered field). */
int sfpic_write_field(sfpic_sim *sim, int comp, const double *in, size_t n);

/* Copy the total field F_scatt + F_inc (Sec. 2: the physical field, the
 * scattered field stored on the grid plus the incident field in closed
 * form) of one component (SFPIC_EX .. SFPIC_BZ) to out, laid out as for
 * sfpic_read_field, guards included.  Each element is taken at the node
 * where the Yee grid stores that component, E at t^n = n dt and B at
 * t^{n-1/2}, with the incident field evaluated on the device in FP64; for
 * on_nodes incidents this is the closed form, not its sampled copy.  A sim
 * without an incident field returns its stored field.  This is the field
 * the Sec. 3.1 norms compare between resolutions and between models; read
 * at step 0 it is the incident field on the grid, the initial condition of
 * a run that carries the whole pulse on the grid.  Returns SFPIC_E_INVAL
 * for J or a NULL out, SFPIC_E_SIZE unless n = NX NY. */
int sfpic_read_total_field(sfpic_sim *sim, int comp, double *out, size_t n);

/* Set the step counter n (the next step starts at t^n = n dt, the time at
 * which the Sec. 2 step evaluates F_inc at the particles). */
int sfpic_set_step_index(sfpic_sim *sim, int64_t step);

/* Number of live macro-particles of a species (the particles of the
 * Vlasov discretization, Sec. 2).  SFPIC_E_INVAL for a bad species. */
int sfpic_particle_count(sfpic_sim *sim, int species, int64_t *n);

/* Copy the live particles of a species (device order) as double, physical
 * units (Table 1); id (nullable) receives each particle's creation index.
 * capacity is the length of the caller's arrays; *n_out receives the count
 * written (SFPIC_E_SIZE if capacity is too small).  y may be NULL in 1D. */
int sfpic_read_particles(sfpic_sim *sim, int species, double *x, double *y,
                         double *ux, double *uy, double *uz, uint32_t *id,
                         size_t capacity, size_t *n_out);

/* FP64 global diagnostics: the kinetic, scattered-EM and total-EM energies
 * whose evolution Secs. 3.1 and 3.2 compare between resolutions and models,
 * the charge, and the Gauss-law and discrete-continuity residuals of the
 * charge-conserving deposition that Sec. 2 names (units of Table 1).  See
 * sfpic_diag for each quantity.  SFPIC_E_INVAL for a NULL out. */
int sfpic_diagnostics(sfpic_sim *sim, sfpic_diag *out);

/* Energy-angle histogram of a species (weights w dV), out has
 * n_energy * n_theta doubles [energy][theta]; moments (nullable) receives
 * {sum of weights, <E_k>, <E_k^2>, <theta>, <theta^2>} (theta in degrees,
 * the angle spec->plane selects) over particles with E_k > ek_min.  These
 * are the electron energy spectra against the angle from the propagation
 * axis of Secs. 4.2 and 4.3.  SFPIC_E_INVAL for a bad spec, SFPIC_E_SIZE
 * unless n = n_energy n_theta, SFPIC_E_NOMEM if its device buffer cannot
 * be allocated. */
int sfpic_histogram(sfpic_sim *sim, const sfpic_hist_spec *spec,
                    double *out, size_t n, double *moments);

/* sfpic_histogram for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same histogram and moments, with the bins accumulated in
 * a fixed device array of the library instead of a buffer allocated per
 * call.  It calls no hipMalloc, hipFree or allocating library routine; it
 * still copies the result to the caller's host arrays and waits for the
 * sim's stream.  n_energy * n_theta must not exceed
 * SFPIC_HIST_NOALLOC_MAX_BINS (SFPIC_E_SIZE otherwise); other errors as
 * sfpic_histogram.  The array (8 + SFPIC_HIST_NOALLOC_MAX_BINS doubles,
 * 512 KiB) exists once per GPU for the life of the process and every call
 * on that GPU uses it: calls that overlap on one GPU (several host threads,
 * or sims on different streams) race and must be serialized by the caller. */
#define SFPIC_HIST_NOALLOC_MAX_BINS 65536
int sfpic_histogram_noalloc(sfpic_sim *sim, const sfpic_hist_spec *spec,
                            double *out, size_t n, double *moments);

/* Checkpoint: serialize the full state (fields, particles, step) into buf.
 * With buf == NULL, *n receives the size needed.  Otherwise *n is the
 * buffer size on input and the size written on output (SFPIC_E_SIZE when
 * it is too small).  Runtime plumbing: no passage of the paper defines it. */
int sfpic_get_state(sfpic_sim *sim, void *buf, size_t *n);

/* Restore a state produced by sfpic_get_state of a sim with the same grid,
 * precision and species count (SFPIC_E_INVAL otherwise, SFPIC_E_SIZE for a
 * truncated buffer).  Runtime plumbing, as sfpic_get_state. */
int sfpic_set_state(sfpic_sim *sim, const void *buf, size_t n);

/* Per-kernel timing.  While profiling is on, every kernel launch of the
 * sim's steps is bracketed by HIP events on the sim's stream.  Kernel
 * classes: 0 Faraday (+ centred B, J clear), 1 tiled particle push (gather,
 * incident field, Boris, deposit), 2 Ampere + Mur, 3 cell sort, 4 push of
 * the particles that left their tile window since the last sort. */
#define SFPIC_KCLASSES 5
typedef struct {
  int64_t launches[SFPIC_KCLASSES];
  double total_ms[SFPIC_KCLASSES];
} sfpic_kernel_stats;

/* Start (enable != 0) or stop profiling; starting clears the counters
 * (measurement plumbing; no passage of the paper defines it). */
int sfpic_profile(sfpic_sim *sim, int enable);

/* Wait for the stream and return the accumulated per-class launch counts
 * and summed kernel durations since profiling was last started. */
int sfpic_profile_read(sfpic_sim *sim, sfpic_kernel_stats *out);

/* Release the sim and its device memory (waits for queued work; NULL is
 * ignored).  Runtime plumbing. */
void sfpic_destroy(sfpic_sim *sim);

/* Device memory held by the sim, in bytes (runtime plumbing). */
int sfpic_device_bytes(sfpic_sim *sim, size_t *bytes);

/* ---------------------------------------------------------------------------
 * Beam set-up on the host (no GPU).  Normalized units as everywhere here
 * (k = omega = c = 1, fields in m_e c omega / e); the caller converts from
 * SI with its wavelength.
 * ------------------------------------------------------------------------- */

/* Complex April field (Sec. 4.1) of an APRIL_LP or APRIL_RP incident at the
 * point (x, y, z) relative to the focus and time t relative to the focal
 * time, in the paper's own axes (z = propagation, x = LP polarization):
 * out = {Re, Im} of E_x, E_y, E_z, cB_x, cB_y, cB_z (12 doubles), scaled to
 * the incident's a0.  The physical field is the real part.  Returns
 * SFPIC_E_INVAL for other kinds or a NULL out. */
int sfpic_april_field(const sfpic_incident *inc, double x, double y, double z,
                      double t, double *out);

/* Peak power of an April beam (Sec. 4.1): the cycle-averaged Poynting flux
 * (1/2) Re{E_x cB_y* - E_y cB_x*} integrated over the focal plane at the
 * focal time, for the incident's a0, in units of eps0 c (m_e c omega/e)^2
 * / k^2.  The paper fixes the beam amplitude from the peak power this way;
 * with a0 = 1, a0 for a power P follows as sqrt(P / *power).  Trapezoid
 * rule on a square of half-side 8 w0 with spacing w0 / 24. */
int sfpic_april_power(const sfpic_incident *inc, double *power);

/* ---------------------------------------------------------------------------
 * Sweeps.  The paper studies the same set-up over ranges of beam and plasma
 * parameters (focusing, polarization, density: Secs. 3 and 4); a sweep runs
 * many independent simulations of uneven size on one GPU.  Members of one
 * precision and dimensionality advance together: each phase of a step is a
 * single launch over all of them (the particle push is a persistent kernel
 * that takes tiles of every member from one queue), and 8 steps are
 * captured once as a HIP graph and replayed.  After every step the tile
 * sort runs for the members it is due for: every sort_every of a member's
 * own steps (default 4).
 * ------------------------------------------------------------------------- */

/* One sweep member: the arguments of sfpic_create, the number of steps to
 * run and the energy-angle histogram reported with its result
 * (hist.n_energy == 0: none). */
typedef struct {
  sfpic_grid grid;
  const sfpic_species *species;
  int32_t nspecies;
  sfpic_incident incident;
  sfpic_precision precision;
  int64_t nsteps;
  sfpic_hist_spec hist;
} sfpic_sim_desc;

typedef struct {
  int32_t status;      /* SFPIC_OK, or the error that ended the member      */
  char error[128];     /* message when status != SFPIC_OK                   */
  sfpic_diag diag;     /* FP64 diagnostics at the end of the run            */
  double moments[5];   /* of hist, as sfpic_histogram; zeros if none        */
  int64_t steps;       /* steps run                                         */
  double pushes;       /* particle pushes (live particles x steps, approx.) */
  double t_submit;     /* seconds on the owner's clock: batch run start or  */
  double t_start;      /*   server creation; submit, admission and result   */
  double t_done;       /*   times                                           */
  size_t device_bytes; /* device memory the member held                     */
} sfpic_result;

/* Device bytes a simulation created from desc with runtime rt would hold. */
int sfpic_desc_footprint(const sfpic_sim_desc *desc, const sfpic_runtime *rt,
                         size_t *bytes);

typedef struct sfpic_batch sfpic_batch;

/* The sweep of Secs. 3 and 4 (focusing, polarization and density varied
 * over one set-up), each member the Sec. 2 step.
 * Create the n members (placing their particles).  rt->stream NULL: the
 * batch creates its own stream.  Tile: rt->tile_x, tile_y if given,
 * otherwise chosen by the autotuner in the first steps of sfpic_batch_run
 * (runs of 128 steps or more, unless SFPIC_RT_NO_AUTOTUNE).  Sort cadence:
 * rt->sort_every if given; else, when the tile is autotuned, the fastest
 * of every 2, 4 or 8 steps on the run's own steps after the tile, timed
 * again every 256 steps of a longer run; else 4.  The trials are real
 * steps of the run (sfpic_batch_stats lists them). */
int sfpic_batch_create(int n, const sfpic_sim_desc *descs,
                       const sfpic_runtime *rt, sfpic_batch **out);

/* Run every member to its nsteps and compute the results (blocking).  A
 * member whose fields or momenta stop being finite ends with status
 * SFPIC_E_NUMERIC in its result and does not affect the others; the call
 * itself then still returns SFPIC_OK (device errors return SFPIC_E_DEVICE). */
int sfpic_batch_run(sfpic_batch *batch);

/* Result of member i after sfpic_batch_run (FP64 diagnostics and the
 * energy-angle moments of Secs. 4.2 and 4.3).  SFPIC_E_STATE before the
 * run, SFPIC_E_INVAL for a bad index. */
int sfpic_batch_result(sfpic_batch *batch, int i, sfpic_result *out);

/* Borrowed handle of member i (fields, particles, histograms through the
 * single-simulation calls; not to be stepped or destroyed by the caller). */
int sfpic_batch_member(sfpic_batch *batch, int i, sfpic_sim **sim);

#define SFPIC_MAX_GROUPS 4
#define SFPIC_MAX_CANDIDATES 32
typedef struct {
  int32_t ngroups;     /* (precision, dims) classes                         */
  int32_t precision[SFPIC_MAX_GROUPS], dims[SFPIC_MAX_GROUPS];
  int32_t members[SFPIC_MAX_GROUPS];
  int32_t tile_x[SFPIC_MAX_GROUPS], tile_y[SFPIC_MAX_GROUPS];
  int32_t sort_every[SFPIC_MAX_GROUPS];
  int32_t tuned[SFPIC_MAX_GROUPS];  /* 1: tile chosen by the autotuner       */
  int32_t push_workgroups[SFPIC_MAX_GROUPS];  /* persistent push grid       */
  /* autotuner trials of each group in the order run (the first
   * SFPIC_MAX_CANDIDATES): tile, cadence, ns per particle push             */
  int32_t n_candidates[SFPIC_MAX_GROUPS];
  int32_t cand_tile_x[SFPIC_MAX_GROUPS][SFPIC_MAX_CANDIDATES];
  int32_t cand_tile_y[SFPIC_MAX_GROUPS][SFPIC_MAX_CANDIDATES];
  int32_t cand_sort_every[SFPIC_MAX_GROUPS][SFPIC_MAX_CANDIDATES];
  double cand_ns_per_push[SFPIC_MAX_GROUPS][SFPIC_MAX_CANDIDATES];
  double run_ms;       /* sfpic_batch_run, first launch to last result      */
  double step_ms;      /* of which stepping (stream time)                   */
  double pushes;       /* particle pushes of all members                    */
  int64_t graph_launches;
} sfpic_batch_info;

/* Group, tile, cadence and autotuner record of the batch (measurement
 * plumbing; no passage of the paper defines it). */
int sfpic_batch_stats(sfpic_batch *batch, sfpic_batch_info *out);
/* Release every member and the batch (NULL is ignored). */
void sfpic_batch_destroy(sfpic_batch *batch);

/* ---------------------------------------------------------------------------
 * Serving: a request loop on a library thread.  Submitted members wait in a
 * FIFO queue and are admitted when a slot is free and their device
 * footprint fits the HBM budget; admitted members stay resident and advance
 * together, 8 steps per tick, with members admitted later joining
 * at the next tick (continuous batching).  A finished member's result is
 * kept on the host and its device memory released.
 * ------------------------------------------------------------------------- */
typedef struct sfpic_server sfpic_server;

enum {
  SFPIC_REQ_QUEUED = 1,
  SFPIC_REQ_RUNNING = 2,
  SFPIC_REQ_DONE = 3,
  SFPIC_REQ_FAILED = 4
};

typedef struct {
  int64_t submitted, admitted, completed, failed, queued, running;
  double p50_s, p99_s, mean_s, max_s; /* submit-to-result of completed ones */
  double pushes;         /* particle pushes done (all requests)             */
  double busy_s;         /* wall time with at least one request running     */
  double pushes_per_s;   /* pushes / busy_s                                 */
  size_t bytes_in_use, bytes_peak, budget;
  int64_t ticks;
  int32_t max_running;   /* most requests resident at once                  */
} sfpic_server_info;

/* hbm_budget: device bytes the resident members may hold (0: 90% of the
 * free device memory at create); max_slots: most members resident at once.
 * The server allocates with hipMalloc on its own stream (rt->alloc and
 * rt->stream are not used); tile and cadence come from rt or the defaults. */
int sfpic_server_create(size_t hbm_budget, int max_slots,
                        const sfpic_runtime *rt, sfpic_server **out);

/* Queue a request (desc and its arrays are copied): one member of the
 * Secs. 3 and 4 sweep, the Sec. 2 step run for desc->nsteps.  SFPIC_E_INVAL
 * if it is invalid or could never fit the budget.  A request that goes
 * non-finite while it runs ends SFPIC_REQ_FAILED with status
 * SFPIC_E_NUMERIC; the others are unaffected. */
int sfpic_server_submit(sfpic_server *srv, const sfpic_sim_desc *desc,
                        uint64_t *ticket);

/* State of a request (SFPIC_REQ_*; SFPIC_E_INVAL for an unknown ticket). */
int sfpic_server_poll(sfpic_server *srv, uint64_t ticket, int *state);

/* Block until the request is done or failed, or timeout_s passes
 * (SFPIC_E_BUSY). */
int sfpic_server_wait(sfpic_server *srv, uint64_t ticket, double timeout_s);

/* Result of a finished request (SFPIC_E_STATE while it is not finished). */
int sfpic_server_result(sfpic_server *srv, uint64_t ticket,
                        sfpic_result *out);

/* The request's energy-angle histogram (Secs. 4.2 and 4.3; n =
 * hist.n_energy * hist.n_theta, SFPIC_E_SIZE otherwise). */
int sfpic_server_histogram(sfpic_server *srv, uint64_t ticket, double *out,
                           size_t n);

/* Counts, latency percentiles and throughput of the server (measurement
 * plumbing; no passage of the paper defines it). */
int sfpic_server_stats(sfpic_server *srv, sfpic_server_info *out);

/* Stop the loop (running requests are abandoned) and release everything. */
void sfpic_server_destroy(sfpic_server *srv);

/* ------------------------------------------------------------------------ */
/* 3D3V simulations (Sec. 4 runs the method in three dimensions with the    */
/* tightly focused April LP and RP pulses).                                 */
/* ------------------------------------------------------------------------ */
/* The step is the one described at the top of this header with every
 * operator in three dimensions: all six scattered components on the Yee
 * staggering Ex(i+1/2,j,k) Ey(i,j+1/2,k) Ez(i,j,k+1/2) Bx(i,j+1/2,k+1/2)
 * By(i+1/2,j,k+1/2) Bz(i+1/2,j+1/2,k), J co-located with E; 3 x 3 x 3
 * order-2 gathers; the incident field at each particle (plane pulse along x,
 * or the full six-component April LP / RP beam focused at (x_focus, y_focus,
 * z_focus) at t_focus; the paper's (x, y, z) are (y, z, x) here); the 3D
 * Esirkepov (2001) current; removal of particles that leave the physical
 * box [0, nx dx) x [0, ny dy) x [0, nz dz) after they deposit; first-order
 * Mur on tangential E at the outer faces (z faces, then y, then x; an edge
 * node takes the last face's value).  FP64, or FP32 storage of fields and
 * momenta (see sfpic3_create); single simulations only (no batches or
 * servers).  Host field arrays are [k][j][i] with i
 * fastest, NX = nx + 2 SFPIC_GUARD, NY = ny + 2 SFPIC_GUARD, NZ = nz + 2
 * SFPIC_GUARD. */
typedef struct {
  int64_t nx, ny, nz;  /* physical cells, each in [1, 32768]              */
  double dx, dy, dz;   /* cell sizes                                      */
  double dt;           /* dt sqrt(1/dx^2 + 1/dy^2 + 1/dz^2) < 1           */
} sfpic3_grid;

/* One mobile species, generated (n_explicit == 0, ppc > 0: ppc particles
 * per cell of region [x0,x1) x [y0,y1) x [z0,z1), uniform in the cell,
 * Philox4x32-10 keyed by (seed, species_index) with counter (particle id,
 * word 2 = 0 for x and y, 3 for z, 1 and 2 for Box-Muller momenta of
 * temperature_ev), weight density / ppc) or explicit (n_explicit > 0 arrays
 * in physical units, every position inside the box, each particle carrying
 * density `weight`).  As in 2D an immobile neutralizing background is
 * implied. */
typedef struct {
  double q, m;
  double density;
  int64_t region[6];
  int32_t ppc;
  double temperature_ev;
  uint64_t seed;
  int32_t species_index;
  int64_t n_explicit;
  double weight;
  const double *x, *y, *z, *ux, *uy, *uz;
  int32_t profile;  /* SFPIC_PROFILE_*, as in sfpic_species              */
  double profile_center, profile_fwhm, profile_order, profile_xmin;
} sfpic3_species;

typedef struct sfpic3_sim sfpic3_sim;

/* Create a 3D simulation (scattered field zero, u^{-1/2} = u^0).  Incident
 * kinds: none, plane pulse, April LP / RP with on_nodes = 0; the Gaussian
 * beam is 2D only.  precision: SFPIC_FP64, or SFPIC_FP32, the 3D storage
 * form: fields and momenta stored as float (half the field memory, 12 of 24
 * momentum bytes per particle), positions FP64 in cell units, every
 * operation and the current accumulation in FP64 (unlike the 2D FP32 form,
 * whose arithmetic is FP32).  SFPIC_E_INVAL for bad sizes, parameters or
 * explicit particles outside the box, SFPIC_E_NOMEM, SFPIC_E_DEVICE. */
int sfpic3_create(const sfpic3_grid *grid, const sfpic3_species *species,
                  int nspecies, const sfpic_incident *incident,
                  sfpic_precision precision, const sfpic_runtime *runtime,
                  sfpic3_sim **out);
/* Enqueue nsteps >= 0 steps on the runtime stream (asynchronous): the
 * Sec. 2 step in three dimensions, as Sec. 4 runs it.  SFPIC_E_INVAL for
 * nsteps < 0 or a NULL sim. */
int sfpic3_step(sfpic3_sim *sim, int64_t nsteps);
/* Wait for the queued work (runtime plumbing). */
int sfpic3_sync(sfpic3_sim *sim);
/* out = {NX, NY, NZ}, the extents of host field arrays (plumbing). */
int sfpic3_dims(const sfpic3_sim *sim, int64_t out[3]);
/* Copy one component (SFPIC_EX .. SFPIC_JZ) of the scattered field (the
 * only field on the grid, Sec. 2) as [k][j][i]; n = NX NY NZ. */
int sfpic3_read_field(sfpic3_sim *sim, int comp, double *out, size_t n);
/* Overwrite E or B (SFPIC_EX .. SFPIC_BZ) from a host array as above (an
 * initial condition other than the zero field of Sec. 2). */
int sfpic3_write_field(sfpic3_sim *sim, int comp, const double *in, size_t n);
/* Number of particle slots of a species (live and removed; Sec. 2). */
int sfpic3_particle_count(sfpic3_sim *sim, int species, int64_t *n);
/* Copy every slot of a species in creation order (physical units, Table 1);
 * alive[i] is 0 for a removed particle, whose other values are
 * meaningless.  n must equal the slot count (SFPIC_E_SIZE otherwise). */
int sfpic3_read_particles(sfpic3_sim *sim, int species, double *x, double *y,
                          double *z, double *ux, double *uy, double *uz,
                          uint8_t *alive, size_t n);
/* Total field F_scatt + F_inc of one component (SFPIC_EX .. SFPIC_BZ) at
 * its Yee node of every array element, as sfpic_read_total_field does in
 * 1D and 2D: E at t^n, B at t^{n-1/2}, the full six-component incident
 * field evaluated on the device in FP64; layout as sfpic3_read_field.
 * SFPIC_E_INVAL for J or a NULL out, SFPIC_E_SIZE unless n = NX NY NZ. */
int sfpic3_read_total_field(sfpic3_sim *sim, int comp, double *out, size_t n);
/* FP64 diagnostics as sfpic_diag (dV = dx dy dz; w_em over every array
 * node; gauss_residual and rho_max over nodes at least 4 cells inside the
 * box; w_em_total, the energy of the total field F_scatt + F_inc, over the
 * physical nodes i < nx, j < ny, k < nz with each component at its own Yee
 * node, as in 2D: six incident evaluations per node, so it costs about as
 * much as a push of six particles per node). */
int sfpic3_diagnostics(sfpic3_sim *sim, sfpic_diag *out);
/* Energy-angle histogram of a species, as sfpic_histogram (weights w dV,
 * dV = dx dy dz; angle from +x, the propagation axis; the spectra of
 * Sec. 4.2). */
int sfpic3_histogram(sfpic3_sim *sim, const sfpic_hist_spec *spec,
                     double *out, size_t n, double *moments);
/* Checkpoint / resume: with buf == NULL *n receives the state size;
 * otherwise the state (step, E, B, every particle slot with its id) is
 * written into the caller's buffer of *n bytes.  sfpic3_set_state restores
 * a state taken from a simulation created with the same grid, precision and
 * species sizes (SFPIC_E_STATE otherwise). */
int sfpic3_get_state(sfpic3_sim *sim, void *buf, size_t *n);
int sfpic3_set_state(sfpic3_sim *sim, const void *buf, size_t n);
/* Release the 3D simulation (NULL is ignored; runtime plumbing). */
void sfpic3_destroy(sfpic3_sim *sim);

/* Message of the last failure on this handle (a sim, 3D sim, batch or
 * server handle; "" if none), valid until the next call on the handle; a
 * failure inside a call on a handle (for example of a batch member's
 * diagnostics during sfpic_batch_run) is recorded for that handle too.
 * handle NULL: the last failure of the calling thread in any call, which
 * is how the failure of a create call is read. */
const char *sfpic_last_error(const void *handle);

/* Library version string (plumbing). */
const char *sfpic_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SFPIC_H */
