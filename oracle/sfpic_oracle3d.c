/*
 * sfpic_oracle3d.c -- plain FP64 CPU oracle of the 3D3V scattered-field PIC
 * step (Sec. 4 runs the method in 3D with the April LP and RP pulses).
 *
 * TEST INFRASTRUCTURE ONLY (see sfpic_oracle.h).  Single thread, fixed loop
 * order, no blocking or fusion.  The step is the 2D oracle's (Sec. 2: Yee
 * update of the scattered field, gather, incident field added at the
 * particle, Boris, Esirkepov current, removal, Ampere with first-order Mur)
 * with every operator written out in three dimensions:
 *
 *   staggering  Ex(i+1/2, j, k)  Ey(i, j+1/2, k)  Ez(i, j, k+1/2)
 *               Bx(i, j+1/2, k+1/2)  By(i+1/2, j, k+1/2)  Bz(i+1/2, j+1/2, k)
 *               J co-located with E;
 *   Faraday     B -= dt curl_h E   (forward differences onto B's nodes);
 *   Ampere      E += dt (curl_h B - J)  (backward differences onto E's nodes);
 *   gather      order-2 B-spline weights, 3 x 3 x 3 taps per component, each
 *               axis primal or dual as the component is stored;
 *   Esirkepov   (2001) 3D decomposition: with S0, S1 the old and new order-2
 *               shapes on the 5 nodes around the old nearest node and
 *               D = S1 - S0,
 *                 W_x = D_x (S0_y S0_z + D_y S0_z / 2 + S0_y D_z / 2
 *                            + D_y D_z / 3),  and cyclically,
 *               J_x(i+1/2) - J_x(i-1/2) = -q w (dx/dt) W_x(i), likewise J_y,
 *               J_z along their own axes, summed from the low edge.
 *
 * Mur order at the outer faces: tangential E on the z faces, then the y
 * faces, then the x faces; an edge node takes the value of the last face
 * that owns it.  The paper gives no boundary for the scattered field; the
 * kernels use the same order.
 *
 * Host array layout: [k][j][i], i fastest, NX = nx + 2G, NY = ny + 2G,
 * NZ = nz + 2G; index I holds the primal node (I - G) dx or the dual node
 * (I - G + 1/2) dx.
 */
#include "sfpic_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define G ORC_GUARD

typedef struct {
  double q, m, w;
  long n;
  double *x[3], *u[3];
  int *alive;
} orc3_species;

struct orc3_sim {
  orc3_grid g;
  orc_incident inc;
  long N[3]; /* NX, NY, NZ */
  long step;
  double *f[ORC_NCOMP];
  double *bold[3], *bbar[3], *eold[3];
  int nsp;
  orc3_species sp[8];
};

#define A3(S, a, i, j, k) \
  (a)[((long)(k) * (S)->N[1] + (long)(j)) * (S)->N[0] + (long)(i)]

/* staggering: 1 = dual along that axis, for Ex Ey Ez Bx By Bz */
static const int STAG3[6][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1},
                                {0, 1, 1}, {1, 0, 1}, {1, 1, 0}};

/* Incident field in build axes at (x, y, z), time t.  Build (x, y, z) are the
 * paper's (z, x, y): propagation along build x, LP polarization along build
 * y.  The plane pulse depends on x only; the April fields are the full
 * six-component closed form of Sec. 4.1 (LP) and the RP form. */
void orc3_incident_eval(const orc_incident *inc, double x, double y, double z,
                        double t, double E[3], double B[3]) {
  for (int c = 0; c < 3; ++c) E[c] = B[c] = 0.0;
  if (inc->kind == ORC_INC_PLANE_PULSE_1D) {
    orc_incident_eval(inc, 1, x, 0.0, t, E, B);
  } else if (inc->kind == ORC_INC_APRIL_LP || inc->kind == ORC_INC_APRIL_RP) {
    double a = inc->ka;
    double px = (y - inc->y_focus) / a; /* paper x */
    double py = (z - inc->z_focus) / a; /* paper y */
    double pz = (x - inc->x_focus) / a; /* paper z */
    double T = (t - inc->t_focus) / a;
    double f[12];
    orc_april_complex(inc->kind, px, py, pz, T, a, inc->s, inc->phi0, -1, f);
    E[0] = inc->norm * f[4];  /* build Ex = paper Ez */
    E[1] = inc->norm * f[0];  /* build Ey = paper Ex */
    E[2] = inc->norm * f[2];  /* build Ez = paper Ey */
    B[0] = inc->norm * f[10]; /* build Bx = paper Bz */
    B[1] = inc->norm * f[6];  /* build By = paper Bx */
    B[2] = inc->norm * f[8];  /* build Bz = paper By */
  }
}

orc3_sim *orc3_create(const orc3_grid *g, const orc_incident *inc) {
  if (g->nx < 1 || g->ny < 1 || g->nz < 1) return NULL;
  if (inc->kind == ORC_INC_GAUSS_2D || inc->on_nodes) return NULL;
  orc3_sim *S = (orc3_sim *)calloc(1, sizeof(orc3_sim));
  S->g = *g;
  S->inc = *inc;
  if (orc_incident_setup(&S->inc) != 0) {
    free(S);
    return NULL;
  }
  S->N[0] = g->nx + 2 * G;
  S->N[1] = g->ny + 2 * G;
  S->N[2] = g->nz + 2 * G;
  long n = S->N[0] * S->N[1] * S->N[2];
  for (int c = 0; c < ORC_NCOMP; ++c) S->f[c] = (double *)calloc(n, 8);
  for (int c = 0; c < 3; ++c) {
    S->bold[c] = (double *)calloc(n, 8);
    S->bbar[c] = (double *)calloc(n, 8);
    S->eold[c] = (double *)calloc(n, 8);
  }
  return S;
}

void orc3_destroy(orc3_sim *S) {
  if (!S) return;
  for (int c = 0; c < ORC_NCOMP; ++c) free(S->f[c]);
  for (int c = 0; c < 3; ++c) {
    free(S->bold[c]);
    free(S->bbar[c]);
    free(S->eold[c]);
  }
  for (int s = 0; s < S->nsp; ++s) {
    for (int d = 0; d < 3; ++d) {
      free(S->sp[s].x[d]);
      free(S->sp[s].u[d]);
    }
    free(S->sp[s].alive);
  }
  free(S);
}

int orc3_add_species(orc3_sim *S, double q, double m, double w, long n,
                     const double *x, const double *y, const double *z,
                     const double *ux, const double *uy, const double *uz) {
  if (S->nsp >= 8) return -1;
  orc3_species *p = &S->sp[S->nsp];
  p->q = q; p->m = m; p->w = w; p->n = n;
  size_t b = (size_t)(n > 0 ? n : 1) * 8;
  const double *src[6] = {x, y, z, ux, uy, uz};
  for (int d = 0; d < 3; ++d) {
    p->x[d] = (double *)malloc(b);
    p->u[d] = (double *)malloc(b);
    memcpy(p->x[d], src[d], (size_t)n * 8);
    memcpy(p->u[d], src[3 + d], (size_t)n * 8);
  }
  p->alive = (int *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int));
  for (long i = 0; i < n; ++i) p->alive[i] = 1;
  return S->nsp++;
}

long orc3_n_alloc(const orc3_sim *S, int axis) { return S->N[axis]; }
long orc3_step_index(const orc3_sim *S) { return S->step; }
double *orc3_field(orc3_sim *S, int comp) { return S->f[comp]; }
long orc3_count(const orc3_sim *S, int sp) { return S->sp[sp].n; }

void orc3_get_particles(const orc3_sim *S, int sp, double *x, double *y,
                        double *z, double *ux, double *uy, double *uz,
                        int *alive) {
  const orc3_species *p = &S->sp[sp];
  double *dst[6] = {x, y, z, ux, uy, uz};
  for (int d = 0; d < 3; ++d) {
    memcpy(dst[d], p->x[d], (size_t)p->n * 8);
    memcpy(dst[3 + d], p->u[d], (size_t)p->n * 8);
  }
  memcpy(alive, p->alive, (size_t)p->n * sizeof(int));
}

/* three order-2 weights around the nearest node (primal at integers, dual at
 * half-integers, cell units); returns the physical index of the first one */
static long w3(double xi, int dual, double w[3]) {
  double off = dual ? 0.5 : 0.0;
  long i0 = (long)floor(xi - off + 0.5);
  for (int k = -1; k <= 1; ++k) w[k + 1] = orc_shape2(xi - (i0 + k + off));
  return i0 - 1;
}

static double gather3(const orc3_sim *S, const double *arr, int comp,
                      const double xi[3]) {
  double w[3][3];
  long i0[3];
  for (int d = 0; d < 3; ++d) i0[d] = w3(xi[d], STAG3[comp][d], w[d]);
  double v = 0.0;
  for (int c = 0; c < 3; ++c)
    for (int b = 0; b < 3; ++b)
      for (int a = 0; a < 3; ++a)
        v += w[0][a] * w[1][b] * w[2][c] *
             A3(S, arr, i0[0] + a + G, i0[1] + b + G, i0[2] + c + G);
  return v;
}

void orc3_gather(const orc3_sim *S, double x, double y, double z, double E[3],
                 double B[3]) {
  const double xi[3] = {x / S->g.dx, y / S->g.dy, z / S->g.dz};
  for (int c = 0; c < 3; ++c) E[c] = gather3(S, S->f[ORC_EX + c], c, xi);
  for (int c = 0; c < 3; ++c) B[c] = gather3(S, S->f[ORC_BX + c], 3 + c, xi);
}

static void shape5(double xi, long i0, double S5[5]) {
  for (int k = -2; k <= 2; ++k) S5[k + 2] = orc_shape2(xi - (double)(i0 + k));
}

/* Esirkepov (2001) current of one particle moving x0 -> x1 in one step. */
static void deposit3(orc3_sim *S, double qw, const double x0[3],
                     const double x1[3]) {
  const double h[3] = {S->g.dx, S->g.dy, S->g.dz}, dt = S->g.dt;
  double S0[3][5], D[3][5];
  long c0[3];
  for (int d = 0; d < 3; ++d) {
    double a = x0[d] / h[d], b = x1[d] / h[d];
    double S1[5];
    c0[d] = (long)floor(a + 0.5);
    shape5(a, c0[d], S0[d]);
    shape5(b, c0[d], S1);
    for (int k = 0; k < 5; ++k) D[d][k] = S1[k] - S0[d][k];
  }
  double *J[3] = {S->f[ORC_JX], S->f[ORC_JY], S->f[ORC_JZ]};
  /* component d accumulates along axis d over the two other axes e, f */
  for (int d = 0; d < 3; ++d) {
    const int e = (d + 1) % 3, f = (d + 2) % 3;
    const double scale = -qw * h[d] / dt;
    for (int kf = 0; kf < 5; ++kf)
      for (int ke = 0; ke < 5; ++ke) {
        double acc = 0.0;
        for (int kd = 0; kd < 4; ++kd) {
          double wgt = D[d][kd] * (S0[e][ke] * S0[f][kf] +
                                   0.5 * D[e][ke] * S0[f][kf] +
                                   0.5 * S0[e][ke] * D[f][kf] +
                                   D[e][ke] * D[f][kf] / 3.0);
          acc += scale * wgt;
          long idx[3];
          idx[d] = c0[d] - 2 + kd + G;
          idx[e] = c0[e] - 2 + ke + G;
          idx[f] = c0[f] - 2 + kf + G;
          A3(S, J[d], idx[0], idx[1], idx[2]) += acc;
        }
      }
  }
}

static void faraday3(orc3_sim *S) {
  const long NX = S->N[0], NY = S->N[1], NZ = S->N[2], n = NX * NY * NZ;
  const double cx = S->g.dt / S->g.dx, cy = S->g.dt / S->g.dy,
               cz = S->g.dt / S->g.dz;
  double *Ex = S->f[ORC_EX], *Ey = S->f[ORC_EY], *Ez = S->f[ORC_EZ];
  double *Bx = S->f[ORC_BX], *By = S->f[ORC_BY], *Bz = S->f[ORC_BZ];
  for (int c = 0; c < 3; ++c) memcpy(S->bold[c], S->f[ORC_BX + c], (size_t)n * 8);
  /* Bx(i, j+1/2, k+1/2) -= dt (dEz/dy - dEy/dz) */
  for (long k = 0; k + 1 < NZ; ++k)
    for (long j = 0; j + 1 < NY; ++j)
      for (long i = 0; i < NX; ++i)
        A3(S, Bx, i, j, k) -= cy * (A3(S, Ez, i, j + 1, k) - A3(S, Ez, i, j, k)) -
                              cz * (A3(S, Ey, i, j, k + 1) - A3(S, Ey, i, j, k));
  /* By(i+1/2, j, k+1/2) -= dt (dEx/dz - dEz/dx) */
  for (long k = 0; k + 1 < NZ; ++k)
    for (long j = 0; j < NY; ++j)
      for (long i = 0; i + 1 < NX; ++i)
        A3(S, By, i, j, k) -= cz * (A3(S, Ex, i, j, k + 1) - A3(S, Ex, i, j, k)) -
                              cx * (A3(S, Ez, i + 1, j, k) - A3(S, Ez, i, j, k));
  /* Bz(i+1/2, j+1/2, k) -= dt (dEy/dx - dEx/dy) */
  for (long k = 0; k < NZ; ++k)
    for (long j = 0; j + 1 < NY; ++j)
      for (long i = 0; i + 1 < NX; ++i)
        A3(S, Bz, i, j, k) -= cx * (A3(S, Ey, i + 1, j, k) - A3(S, Ey, i, j, k)) -
                              cy * (A3(S, Ex, i, j + 1, k) - A3(S, Ex, i, j, k));
  for (int c = 0; c < 3; ++c)
    for (long q = 0; q < n; ++q)
      S->bbar[c][q] = 0.5 * (S->bold[c][q] + S->f[ORC_BX + c][q]);
}

/* first-order Mur: E_b^{n+1} = E_in^n + k (E_in^{n+1} - E_b^n) */
static double mur3(double in_old, double in_new, double b_old, double k) {
  return in_old + k * (in_new - b_old);
}

/* Mur on the two faces normal to `axis` for component `comp` (a tangential
 * one), over every index the component occupies along the other axes (the
 * last index along a dual axis is outside the grid and left alone). */
static void mur_faces(orc3_sim *S, int comp, int axis, double kf) {
  double *E = S->f[ORC_EX + comp], *O = S->eold[comp];
  const long N[3] = {S->N[0], S->N[1], S->N[2]};
  const int e = (axis + 1) % 3, f = (axis + 2) % 3;
  const long ne = N[e] - STAG3[comp][e], nf = N[f] - STAG3[comp][f];
  for (int side = 0; side < 2; ++side) {
    const long b = side ? N[axis] - 1 : 0, in = side ? N[axis] - 2 : 1;
    for (long jf = 0; jf < nf; ++jf)
      for (long je = 0; je < ne; ++je) {
        long ib[3], ii[3];
        ib[axis] = b;  ib[e] = je;  ib[f] = jf;
        ii[axis] = in; ii[e] = je;  ii[f] = jf;
        A3(S, E, ib[0], ib[1], ib[2]) =
            mur3(A3(S, O, ii[0], ii[1], ii[2]), A3(S, E, ii[0], ii[1], ii[2]),
                 A3(S, O, ib[0], ib[1], ib[2]), kf);
      }
  }
}

static void ampere3(orc3_sim *S) {
  const long NX = S->N[0], NY = S->N[1], NZ = S->N[2], n = NX * NY * NZ;
  const double dt = S->g.dt;
  const double cx = dt / S->g.dx, cy = dt / S->g.dy, cz = dt / S->g.dz;
  double *Ex = S->f[ORC_EX], *Ey = S->f[ORC_EY], *Ez = S->f[ORC_EZ];
  double *Bx = S->f[ORC_BX], *By = S->f[ORC_BY], *Bz = S->f[ORC_BZ];
  double *Jx = S->f[ORC_JX], *Jy = S->f[ORC_JY], *Jz = S->f[ORC_JZ];
  for (int c = 0; c < 3; ++c) memcpy(S->eold[c], S->f[ORC_EX + c], (size_t)n * 8);
  /* Ex(i+1/2, j, k) += dt (dBz/dy - dBy/dz - Jx) */
  for (long k = 1; k + 1 < NZ; ++k)
    for (long j = 1; j + 1 < NY; ++j)
      for (long i = 0; i + 1 < NX; ++i)
        A3(S, Ex, i, j, k) += cy * (A3(S, Bz, i, j, k) - A3(S, Bz, i, j - 1, k)) -
                              cz * (A3(S, By, i, j, k) - A3(S, By, i, j, k - 1)) -
                              dt * A3(S, Jx, i, j, k);
  /* Ey(i, j+1/2, k) += dt (dBx/dz - dBz/dx - Jy) */
  for (long k = 1; k + 1 < NZ; ++k)
    for (long j = 0; j + 1 < NY; ++j)
      for (long i = 1; i + 1 < NX; ++i)
        A3(S, Ey, i, j, k) += cz * (A3(S, Bx, i, j, k) - A3(S, Bx, i, j, k - 1)) -
                              cx * (A3(S, Bz, i, j, k) - A3(S, Bz, i - 1, j, k)) -
                              dt * A3(S, Jy, i, j, k);
  /* Ez(i, j, k+1/2) += dt (dBy/dx - dBx/dy - Jz) */
  for (long k = 0; k + 1 < NZ; ++k)
    for (long j = 1; j + 1 < NY; ++j)
      for (long i = 1; i + 1 < NX; ++i)
        A3(S, Ez, i, j, k) += cx * (A3(S, By, i, j, k) - A3(S, By, i - 1, j, k)) -
                              cy * (A3(S, Bx, i, j, k) - A3(S, Bx, i, j - 1, k)) -
                              dt * A3(S, Jz, i, j, k);
  const double kx = (dt - S->g.dx) / (dt + S->g.dx);
  const double ky = (dt - S->g.dy) / (dt + S->g.dy);
  const double kz = (dt - S->g.dz) / (dt + S->g.dz);
  mur_faces(S, 0, 2, kz); /* z faces: Ex, Ey */
  mur_faces(S, 1, 2, kz);
  mur_faces(S, 0, 1, ky); /* y faces: Ex, Ez */
  mur_faces(S, 2, 1, ky);
  mur_faces(S, 1, 0, kx); /* x faces: Ey, Ez */
  mur_faces(S, 2, 0, kx);
}

void orc3_step(orc3_sim *S, long nsteps) {
  const double dt = S->g.dt;
  const double hi[3] = {S->g.nx * S->g.dx, S->g.ny * S->g.dy,
                        S->g.nz * S->g.dz};
  const long n = S->N[0] * S->N[1] * S->N[2];
  for (long st = 0; st < nsteps; ++st) {
    const double t = (double)S->step * dt;
    faraday3(S);
    for (int c = 0; c < 3; ++c) memset(S->f[ORC_JX + c], 0, (size_t)n * 8);
    for (int s = 0; s < S->nsp; ++s) {
      orc3_species *p = &S->sp[s];
      const double qm = p->q / p->m;
      for (long i = 0; i < p->n; ++i) {
        if (!p->alive[i]) continue;
        const double x0[3] = {p->x[0][i], p->x[1][i], p->x[2][i]};
        const double xi[3] = {x0[0] / S->g.dx, x0[1] / S->g.dy, x0[2] / S->g.dz};
        double E[3], B[3], Ei[3], Bi[3];
        for (int c = 0; c < 3; ++c) {
          E[c] = gather3(S, S->f[ORC_EX + c], c, xi);
          B[c] = gather3(S, S->bbar[c], 3 + c, xi);
        }
        orc3_incident_eval(&S->inc, x0[0], x0[1], x0[2], t, Ei, Bi);
        for (int c = 0; c < 3; ++c) {
          E[c] += Ei[c];
          B[c] += Bi[c];
        }
        double u[3] = {p->u[0][i], p->u[1][i], p->u[2][i]};
        orc_boris(qm, dt, u, E, B);
        double gam = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        double x1[3];
        for (int d = 0; d < 3; ++d) x1[d] = x0[d] + dt * u[d] / gam;
        deposit3(S, p->q * p->w, x0, x1);
        int out = 0;
        for (int d = 0; d < 3; ++d) {
          p->x[d][i] = x1[d];
          p->u[d][i] = u[d];
          if (x1[d] < 0.0 || x1[d] >= hi[d]) out = 1;
        }
        if (out) p->alive[i] = 0;
      }
    }
    ampere3(S);
    S->step++;
  }
}

/* charge density of the live particles on the primal nodes */
void orc3_deposit_rho(const orc3_sim *S, double *rho) {
  memset(rho, 0, (size_t)(S->N[0] * S->N[1] * S->N[2]) * 8);
  const double h[3] = {S->g.dx, S->g.dy, S->g.dz};
  for (int s = 0; s < S->nsp; ++s) {
    const orc3_species *p = &S->sp[s];
    for (long i = 0; i < p->n; ++i) {
      if (!p->alive[i]) continue;
      double w[3][3];
      long i0[3];
      for (int d = 0; d < 3; ++d) i0[d] = w3(p->x[d][i] / h[d], 0, w[d]);
      for (int c = 0; c < 3; ++c)
        for (int b = 0; b < 3; ++b)
          for (int a = 0; a < 3; ++a)
            A3(S, rho, i0[0] + a + G, i0[1] + b + G, i0[2] + c + G) +=
                p->q * p->w * w[0][a] * w[1][b] * w[2][c];
    }
  }
}

/* out = {W_kin, W_em (scattered, every array node), charge, live count} */
void orc3_diagnostics(const orc3_sim *S, double out[4]) {
  const double dV = S->g.dx * S->g.dy * S->g.dz;
  const long n = S->N[0] * S->N[1] * S->N[2];
  double wk = 0.0, q = 0.0, na = 0.0, wem = 0.0;
  for (int s = 0; s < S->nsp; ++s) {
    const orc3_species *p = &S->sp[s];
    for (long i = 0; i < p->n; ++i) {
      if (!p->alive[i]) continue;
      double u2 = 0.0;
      for (int d = 0; d < 3; ++d) u2 += p->u[d][i] * p->u[d][i];
      wk += p->w * p->m * (sqrt(1.0 + u2) - 1.0) * dV;
      q += p->q * p->w * dV;
      na += 1.0;
    }
  }
  for (int c = 0; c < 6; ++c)
    for (long k = 0; k < n; ++k) wem += 0.5 * S->f[c][k] * S->f[c][k];
  out[0] = wk;
  out[1] = wem * dV;
  out[2] = q;
  out[3] = na;
}

/* Energy of the total field (Sec. 2: the physical field is the incident plus
 * the scattered one): 1/2 sum over the physical nodes i < nx, j < ny, k < nz
 * of (F_s + F_inc)^2 for the six components, each at its own staggered node,
 * E at t^n and B at t^{n-1/2}, times dV. */
double orc3_em_energy_total(const orc3_sim *S) {
  const double tE = (double)S->step * S->g.dt, tB = tE - 0.5 * S->g.dt;
  double w = 0.0;
  for (long k = 0; k < S->g.nz; ++k)
    for (long j = 0; j < S->g.ny; ++j)
      for (long i = 0; i < S->g.nx; ++i)
        for (int c = 0; c < 6; ++c) {
          double E[3], B[3];
          orc3_incident_eval(&S->inc, ((double)i + 0.5 * STAG3[c][0]) * S->g.dx,
                             ((double)j + 0.5 * STAG3[c][1]) * S->g.dy,
                             ((double)k + 0.5 * STAG3[c][2]) * S->g.dz,
                             c < 3 ? tE : tB, E, B);
          const double v = A3(S, S->f[c], i + G, j + G, k + G) +
                           (c < 3 ? E[c] : B[c - 3]);
          w += 0.5 * v * v;
        }
  return w * S->g.dx * S->g.dy * S->g.dz;
}

/* Energy-angle histogram of species sp (weights w dV), energy bins over
 * [0, emax) linear, angle from +x over [0, 180] degrees; mom = {sum w, <Ek>,
 * <Ek^2>, <theta>, <theta^2>} over particles with Ek > ek_min. */
void orc3_energy_angle(const orc3_sim *S, int sp, int n_e, double emax,
                       int n_theta, double ek_min, int plane, double *hist,
                       double mom[5]) {
  const orc3_species *p = &S->sp[sp];
  const double dV = S->g.dx * S->g.dy * S->g.dz;
  memset(hist, 0, (size_t)n_e * (size_t)n_theta * 8);
  for (int k = 0; k < 5; ++k) mom[k] = 0.0;
  for (long i = 0; i < p->n; ++i) {
    if (!p->alive[i]) continue;
    double ux = p->u[0][i], uy = p->u[1][i], uz = p->u[2][i];
    double ek = p->m * (sqrt(1.0 + ux * ux + uy * uy + uz * uz) - 1.0);
    /* the angle from +x of the momentum, or of its projection on the x-z
     * plane (plane 1: the plane of the propagation axis across the LP
     * polarization, the paper's (y, z) plane of the Sec. 4.2 spectra) or on
     * the x-y plane (plane 2) */
    double perp = plane == 1   ? fabs(uz)
                  : plane == 2 ? fabs(uy)
                               : sqrt(uy * uy + uz * uz);
    double th = atan2(perp, ux) * (180.0 / 3.14159265358979323846);
    double wt = p->w * dV;
    long ie = (long)floor(ek / emax * n_e);
    long it = (long)floor(th / 180.0 * n_theta);
    if (it >= n_theta) it = n_theta - 1;
    if (ie >= 0 && ie < n_e && it >= 0) hist[ie * n_theta + it] += wt;
    if (ek > ek_min) {
      mom[0] += wt;
      mom[1] += wt * ek;
      mom[2] += wt * ek * ek;
      mom[3] += wt * th;
      mom[4] += wt * th * th;
    }
  }
  if (mom[0] > 0.0)
    for (int k = 1; k < 5; ++k) mom[k] /= mom[0];
}
