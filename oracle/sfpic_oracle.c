/*
 * sfpic_oracle.c -- plain FP64 CPU oracle of the scattered-field PIC step.
 *
 * TEST INFRASTRUCTURE ONLY (see sfpic_oracle.h).  Written for clarity, not
 * speed: single thread, fixed loop order, no blocking or fusion.
 *
 * One step n -> n+1 (state E^n, B^{n-1/2}, particles x^n, u^{n-1/2}):
 *   1. Faraday  B^{n+1/2} = B^{n-1/2} - dt curl_h E^n          (Sec. 2, Yee)
 *   2. centred  Bbar^n = (B^{n-1/2} + B^{n+1/2}) / 2
 *   3. gather   E^n, Bbar^n at x^n with order-2 B-spline weights
 *   4. add the incident field F_inc(x^n, t^n) (Sec. 2: scattered field
 *      interpolated and added to the incident field at the macro-particle);
 *      with inc.on_nodes instead F_inc sampled on the Yee nodes at t^n is
 *      added to the arrays gathered in step 3 (the field superimposed on the
 *      grid fields, as the paper's implementation does, Sec. 2)
 *   5. Boris rotation u^{n-1/2} -> u^{n+1/2}                   (Sec. 2 pusher)
 *   6. x^{n+1} = x^n + dt u^{n+1/2} / gamma  (in-plane components)
 *   7. Esirkepov charge-conserving current J^{n+1/2}           (Sec. 2)
 *   8. particles whose x^{n+1} left the physical box are removed
 *   9. Ampere   E^{n+1} = E^n + dt (curl_h B^{n+1/2} - J^{n+1/2}), first-order
 *      Mur absorbing condition on tangential E at the outer faces.
 * The paper states the ingredients but not their staggering, boundaries or
 * step order; this order is the standard leapfrog and is used by both sides.
 */
#include "sfpic_oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define G ORC_GUARD
#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Incident fields                                                          */
/* ------------------------------------------------------------------------ */

/* Sec. 4.1: k^2 w0^2 = 2 (sqrt(1 + (ka)^2) - 1), solved for ka (k = 1). */
double orc_april_ka_from_w0(double w0) {
  double h = 1.0 + 0.5 * w0 * w0;
  return sqrt(h * h - 1.0);
}

/* Sec. 4.1, derivative of the Poisson-spectrum pulse:
 * g^(n)(tau) = e^{i phi0} Gamma(s+n+1)/Gamma(s+1) (i ka / s)^n
 *              (1 - i tau / s)^{-(s+n+1)}. */
static double complex april_g(int n, double complex tau, double ka, double s,
                              double phi0) {
  double gr = 1.0;
  for (int k = 1; k <= n; ++k) gr *= (s + k); /* Gamma(s+n+1)/Gamma(s+1) */
  double complex c = cexp(I * phi0) * gr * cpow(I * ka / s, n);
  return c * cpow(1.0 - I * tau / s, -(s + n + 1.0));
}

/* Building blocks of the April field in dimensionless variables.  With
 * u = Rtilde/a = sqrt(X^2 + Y^2 + (Z+i)^2) and G_{+-}^(n) = g^(n)(tau_+) +-
 * g^(n)(tau_-), tau_{+-} = tau + ka (+-u + i):
 *   Phi_TT = G_-^(2)/u
 *   D1     = (1/u) d/du (G_-^(0)/u)      = G_+^(1)/u^2 - G_-^(0)/u^3
 *   D1_T   = d/dT D1                     = G_+^(2)/u^2 - G_-^(1)/u^3
 *   D2     = (1/u) d/du D1  = (3 G_-^(0)/u^3 - 3 G_+^(1)/u^2 + G_-^(2)/u)/u^2
 * The printed Sec. 4.1 components are these blocks with
 * (x/r) sin(theta~) / Rtilde = X / u^2 etc. substituted, so no 1/r appears.
 * Near the ring u = 0 (r = a, z = 0) the blocks are 0/0; they are even in u
 * and analytic in u^2, so a Taylor series about u = 0 is used there:
 * with c_m = g^(m)(tau + i ka),
 *   Phi_TT = 2 sum_{j>=0} u^{2j} c_{2j+3}/(2j+1)!
 *   D1     = 2 sum_{j>=1} 2j u^{2j-2} c_{2j+1}/(2j+1)!
 *   D1_T   = 2 sum_{j>=1} 2j u^{2j-2} c_{2j+2}/(2j+1)!
 *   D2     = 2 sum_{j>=2} 2j (2j-2) u^{2j-4} c_{2j+1}/(2j+1)!          */
#define ORC_RING_U2 0.0625 /* series when |u|^2 < 0.25^2 */
#define ORC_RING_TERMS 16

static void april_blocks(double X, double Y, double Z, double T, double ka,
                         double s, double phi0, int use_series,
                         double complex blk[4] /* PhiTT, D1, D1T, D2 */) {
  double complex Zp = Z + I;
  double complex u2 = X * X + Y * Y + Zp * Zp;
  double tau = ka * T;
  int series = use_series;
  if (series < 0) series = cabs(u2) < ORC_RING_U2;
  if (!series) {
    double complex u = csqrt(u2);
    double complex tp = tau + ka * (u + I);
    double complex tm = tau + ka * (-u + I);
    double complex Gp[3], Gm[3];
    for (int n = 0; n < 3; ++n) {
      double complex a = april_g(n, tp, ka, s, phi0);
      double complex b = april_g(n, tm, ka, s, phi0);
      Gp[n] = a + b;
      Gm[n] = a - b;
    }
    double complex u_2 = u * u, u_3 = u_2 * u;
    blk[0] = Gm[2] / u;
    blk[1] = Gp[1] / u_2 - Gm[0] / u_3;
    blk[2] = Gp[2] / u_2 - Gm[1] / u_3;
    blk[3] = (3.0 * Gm[0] / u_3 - 3.0 * Gp[1] / u_2 + Gm[2] / u) / u_2;
  } else {
    double complex c[2 * ORC_RING_TERMS + 4];
    for (int m = 0; m < 2 * ORC_RING_TERMS + 4; ++m)
      c[m] = april_g(m, tau + I * ka, ka, s, phi0);
    double complex pw[ORC_RING_TERMS]; /* pw[j] = u^{2j} */
    pw[0] = 1.0;
    for (int j = 1; j < ORC_RING_TERMS; ++j) pw[j] = pw[j - 1] * u2;
    double complex phitt = 0, d1 = 0, d1t = 0, d2 = 0;
    double fact = 1.0; /* (2j+1)! */
    for (int j = 0; j < ORC_RING_TERMS; ++j) {
      if (j > 0) fact *= (2.0 * j) * (2.0 * j + 1.0);
      phitt += 2.0 * pw[j] * c[2 * j + 3] / fact;
      if (j >= 1) {
        d1 += 2.0 * (2.0 * j) * pw[j - 1] * c[2 * j + 1] / fact;
        d1t += 2.0 * (2.0 * j) * pw[j - 1] * c[2 * j + 2] / fact;
      }
      if (j >= 2)
        d2 += 2.0 * (2.0 * j) * (2.0 * j - 2.0) * pw[j - 2] * c[2 * j + 1] /
              fact;
    }
    blk[0] = phitt;
    blk[1] = d1;
    blk[2] = d1t;
    blk[3] = d2;
  }
}

/* Sec. 4.1 field components (LP: E_x = Psi_xx - Psi_tt + Psi_tz, E_y = Psi_xy,
 * E_z = Psi_zx - Psi_tx, cB_x = Psi_xy, cB_y = Psi_yy - Psi_tt + Psi_tz,
 * cB_z = Psi_zy - Psi_ty).  RP (TM01, electric Hertz vector z*Psi, cited in
 * Sec. 4 but not printed): E = grad(Psi_z) - z Psi_tt, cB = d/dt curl(z Psi).
 * With d/dX = X/u d/du etc. these become combinations of the blocks. */
void orc_april_complex(int kind, double X, double Y, double Z, double T,
                       double ka, double s, double phi0, int use_series,
                       double out[12]) {
  double complex b[4];
  april_blocks(X, Y, Z, T, ka, s, phi0, use_series, b);
  double complex phitt = b[0], d1 = b[1], d1t = b[2], d2 = b[3];
  double complex Zp = Z + I;
  double complex f[6];
  if (kind == ORC_INC_APRIL_LP) {
    f[0] = X * X * d2 + d1 - phitt + Zp * d1t; /* E_x  */
    f[1] = X * Y * d2;                         /* E_y  */
    f[2] = X * Zp * d2 - X * d1t;              /* E_z  */
    f[3] = X * Y * d2;                         /* cB_x */
    f[4] = Y * Y * d2 + d1 - phitt + Zp * d1t; /* cB_y */
    f[5] = Y * Zp * d2 - Y * d1t;              /* cB_z */
  } else {
    f[0] = X * Zp * d2;                 /* E_x = Psi_xz            */
    f[1] = Y * Zp * d2;                 /* E_y = Psi_yz            */
    f[2] = d1 + Zp * Zp * d2 - phitt;   /* E_z = Psi_zz - Psi_tt   */
    f[3] = Y * d1t;                     /* cB_x = Psi_ty           */
    f[4] = -X * d1t;                    /* cB_y = -Psi_tx          */
    f[5] = 0.0;                         /* cB_z = 0                */
  }
  for (int k = 0; k < 6; ++k) {
    out[2 * k] = creal(f[k]);
    out[2 * k + 1] = cimag(f[k]);
  }
}

/* Amplitude reading: a0 is the modulus of the complex on-axis field component
 * (E_x for LP, E_z for RP, paper axes) at the focus at the focal time. */
int orc_incident_setup(orc_incident *inc) {
  if (inc->kind == ORC_INC_APRIL_LP || inc->kind == ORC_INC_APRIL_RP) {
    double f[12];
    orc_april_complex(inc->kind, 0.0, 0.0, 0.0, 0.0, inc->ka, inc->s,
                      inc->phi0, 0, f);
    int c = (inc->kind == ORC_INC_APRIL_LP) ? 0 : 2;
    double m = hypot(f[2 * c], f[2 * c + 1]);
    if (!(m > 0.0)) return -1;
    inc->norm = inc->a0 / m;
  } else {
    inc->norm = 1.0;
  }
  return 0;
}

/* Incident field in build axes at (x, y, z = 0), time t.
 * Paper axes (x, y, z) map to build (y, z, x): paper z (propagation) is build
 * x, paper x (LP polarization) is build y, paper y is build z. */
void orc_incident_eval(const orc_incident *inc, int dims, double x, double y,
                       double t, double E[3], double B[3]) {
  for (int k = 0; k < 3; ++k) E[k] = B[k] = 0.0;
  if (inc->kind == ORC_INC_PLANE_PULSE_1D) {
    /* Sec. 3.1: E = B = E0 sin(t - t0 - z) 2^{-4 (t - t0 - z)^2 / FWHM^2}. */
    double ph = t - inc->t0 - x;
    double v = inc->a0 * sin(ph) *
               pow(2.0, -4.0 * ph * ph / (inc->fwhm_t * inc->fwhm_t));
    E[1] = v;
    B[2] = v;
  } else if (inc->kind == ORC_INC_GAUSS_2D) {
    /* Sec. 3.2, paraxial 2D Gaussian beam focused at the origin, paper axes
     * (z propagation, x transverse):
     *   E_x = E0 sqrt(w0/w) e^{-x^2/w^2} cos(psi) env,  B_y = E_x,
     *   E_z = 2 E0 (x / w^2) sqrt(w0/w) e^{-x^2/w^2} sin(psi) env,
     *   psi = z - t + x^2 / (2 R) - eta,  env = 2^{-4 (t - t0 - z)^2 / FWHM^2},
     *   w = w0 sqrt(1 + (z/zR)^2), R = z (1 + (zR/z)^2), eta = atan(z/zR)/2,
     *   zR = w0^2 / 2.  The longitudinal factor is x / w^2 (the leading order
     * of div E = 0; the printed x / w is not first order in 1/(k w0)), and
     * 1/R = z / (z^2 + zR^2) is used so that the focal plane needs no limit. */
    double z = x - inc->x_focus;
    double xp = (dims == 2) ? y - inc->y_focus : 0.0;
    double zr = 0.5 * inc->w0 * inc->w0;
    double w = inc->w0 * sqrt(1.0 + (z / zr) * (z / zr));
    double inv_r = z / (z * z + zr * zr);
    double eta = 0.5 * atan(z / zr);
    double psi = z - t + 0.5 * xp * xp * inv_r - eta;
    double ph = t - inc->t0 - z;
    double env = pow(2.0, -4.0 * ph * ph / (inc->fwhm_t * inc->fwhm_t));
    double amp = inc->a0 * sqrt(inc->w0 / w) * exp(-xp * xp / (w * w)) * env;
    E[1] = amp * cos(psi);                     /* build y = paper x */
    E[0] = 2.0 * xp / (w * w) * amp * sin(psi); /* build x = paper z */
    B[2] = E[1];                               /* build z = paper y */
  } else if (inc->kind == ORC_INC_APRIL_LP || inc->kind == ORC_INC_APRIL_RP) {
    double a = inc->ka;
    double px = (dims == 2 ? y - inc->y_focus : 0.0) / a; /* paper x */
    double py = 0.0;                                      /* paper y */
    double pz = (x - inc->x_focus) / a;                   /* paper z */
    double T = (t - inc->t_focus) / a;
    double f[12];
    orc_april_complex(inc->kind, px, py, pz, T, a, inc->s, inc->phi0, -1, f);
    /* real parts, paper (Ex,Ey,Ez,Bx,By,Bz) -> build */
    E[0] = inc->norm * f[4];  /* build Ex = paper Ez */
    E[1] = inc->norm * f[0];  /* build Ey = paper Ex */
    E[2] = inc->norm * f[2];  /* build Ez = paper Ey */
    B[0] = inc->norm * f[10]; /* build Bx = paper Bz */
    B[1] = inc->norm * f[6];  /* build By = paper Bx */
    B[2] = inc->norm * f[8];  /* build Bz = paper By */
  }
}

/* ------------------------------------------------------------------------ */
/* Particle building blocks                                                 */
/* ------------------------------------------------------------------------ */

/* Quadratic B-spline (interpolation order 2, Sec. 3.1) at distance d from a
 * node, in cell units. */
double orc_shape2(double d) {
  double a = fabs(d);
  if (a <= 0.5) return 0.75 - a * a;
  if (a <= 1.5) return 0.5 * (1.5 - a) * (1.5 - a);
  return 0.0;
}

/* Boris (1970) rotation for u = gamma v with charge-to-mass ratio qm. */
void orc_boris(double qm, double dt, double u[3], const double E[3],
               const double B[3]) {
  double h = 0.5 * qm * dt;
  double um[3] = {u[0] + h * E[0], u[1] + h * E[1], u[2] + h * E[2]};
  double gm = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
  double tv[3] = {h * B[0] / gm, h * B[1] / gm, h * B[2] / gm};
  double t2 = tv[0] * tv[0] + tv[1] * tv[1] + tv[2] * tv[2];
  double sv[3] = {2.0 * tv[0] / (1.0 + t2), 2.0 * tv[1] / (1.0 + t2),
                  2.0 * tv[2] / (1.0 + t2)};
  double up[3] = {um[0] + (um[1] * tv[2] - um[2] * tv[1]),
                  um[1] + (um[2] * tv[0] - um[0] * tv[2]),
                  um[2] + (um[0] * tv[1] - um[1] * tv[0])};
  double upl[3] = {um[0] + (up[1] * sv[2] - up[2] * sv[1]),
                   um[1] + (up[2] * sv[0] - up[0] * sv[2]),
                   um[2] + (up[0] * sv[1] - up[1] * sv[0])};
  u[0] = upl[0] + h * E[0];
  u[1] = upl[1] + h * E[1];
  u[2] = upl[2] + h * E[2];
}

/* ------------------------------------------------------------------------ */
/* Simulation state                                                         */
/* ------------------------------------------------------------------------ */

typedef struct {
  double q, m, w;
  long n;
  double *x, *y, *ux, *uy, *uz;
  int *alive;
} orc_species;

struct orc_sim {
  orc_grid g;
  orc_incident inc;
  long NX, NY;
  long step;
  double *f[ORC_NCOMP];
  double *bold[3], *bbar[3], *eold[3];
  int nsp;
  orc_species sp[8];
};

#define AT(a, i, j) (a)[(long)(j) * S->NX + (long)(i)]

orc_sim *orc_create(const orc_grid *g, const orc_incident *inc) {
  if (g->dims != 1 && g->dims != 2) return NULL;
  orc_sim *S = (orc_sim *)calloc(1, sizeof(orc_sim));
  S->g = *g;
  S->inc = *inc;
  if (orc_incident_setup(&S->inc) != 0) {
    free(S);
    return NULL;
  }
  S->NX = g->nx + 2 * G;
  S->NY = (g->dims == 2) ? g->ny + 2 * G : 1;
  long n = S->NX * S->NY;
  for (int c = 0; c < ORC_NCOMP; ++c) S->f[c] = (double *)calloc(n, 8);
  for (int c = 0; c < 3; ++c) {
    S->bold[c] = (double *)calloc(n, 8);
    S->bbar[c] = (double *)calloc(n, 8);
    S->eold[c] = (double *)calloc(n, 8);
  }
  return S;
}

void orc_destroy(orc_sim *S) {
  if (!S) return;
  for (int c = 0; c < ORC_NCOMP; ++c) free(S->f[c]);
  for (int c = 0; c < 3; ++c) {
    free(S->bold[c]);
    free(S->bbar[c]);
    free(S->eold[c]);
  }
  for (int s = 0; s < S->nsp; ++s) {
    orc_species *p = &S->sp[s];
    free(p->x); free(p->y); free(p->ux); free(p->uy); free(p->uz);
    free(p->alive);
  }
  free(S);
}

int orc_add_species(orc_sim *S, double q, double m, double w, long n,
                    const double *x, const double *y, const double *ux,
                    const double *uy, const double *uz) {
  if (S->nsp >= 8) return -1;
  orc_species *p = &S->sp[S->nsp];
  p->q = q; p->m = m; p->w = w; p->n = n;
  size_t b = (size_t)(n > 0 ? n : 1) * 8;
  p->x = (double *)malloc(b); p->y = (double *)malloc(b);
  p->ux = (double *)malloc(b); p->uy = (double *)malloc(b);
  p->uz = (double *)malloc(b);
  p->alive = (int *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int));
  for (long i = 0; i < n; ++i) {
    p->x[i] = x[i];
    p->y[i] = (S->g.dims == 2 && y) ? y[i] : 0.0;
    p->ux[i] = ux[i]; p->uy[i] = uy[i]; p->uz[i] = uz[i];
    p->alive[i] = 1;
  }
  return S->nsp++;
}

long orc_nx_alloc(const orc_sim *S) { return S->NX; }
long orc_ny_alloc(const orc_sim *S) { return S->NY; }
long orc_step_index(const orc_sim *S) { return S->step; }
void orc_set_step_index(orc_sim *S, long n) { S->step = n; }
double *orc_field(orc_sim *S, int comp) { return S->f[comp]; }
long orc_count(const orc_sim *S, int sp) { return S->sp[sp].n; }

long orc_alive(const orc_sim *S, int sp) {
  long c = 0;
  for (long i = 0; i < S->sp[sp].n; ++i) c += S->sp[sp].alive[i];
  return c;
}

void orc_get_particles(const orc_sim *S, int sp, double *x, double *y,
                       double *ux, double *uy, double *uz, int *alive) {
  const orc_species *p = &S->sp[sp];
  for (long i = 0; i < p->n; ++i) {
    x[i] = p->x[i]; y[i] = p->y[i];
    ux[i] = p->ux[i]; uy[i] = p->uy[i]; uz[i] = p->uz[i];
    alive[i] = p->alive[i];
  }
}

void orc_set_particles(orc_sim *S, int sp, const double *x, const double *y,
                       const double *ux, const double *uy, const double *uz,
                       const int *alive) {
  orc_species *p = &S->sp[sp];
  for (long i = 0; i < p->n; ++i) {
    p->x[i] = x[i]; p->y[i] = y[i];
    p->ux[i] = ux[i]; p->uy[i] = uy[i]; p->uz[i] = uz[i];
    p->alive[i] = alive[i];
  }
}

/* ------------------------------------------------------------------------ */
/* Interpolation                                                            */
/* ------------------------------------------------------------------------ */

/* Three order-2 weights around the node nearest to xi (cell units).  For a
 * primal component nodes sit at integers; for a dual one at half-integers.
 * Returns the node index (physical, without guard) of the first weight. */
static long weights3(double xi, int dual, double w[3]) {
  long i0;
  double off = dual ? 0.5 : 0.0;
  i0 = (long)floor(xi - off + 0.5);
  for (int k = -1; k <= 1; ++k) w[k + 1] = orc_shape2(xi - (i0 + k + off));
  return i0 - 1;
}

/* staggering flags (dual in x, dual in y) of Ex, Ey, Ez, Bx, By, Bz */
static const int STAG_X[6] = {1, 0, 0, 0, 1, 1};
static const int STAG_Y[6] = {0, 1, 0, 1, 0, 1};

static double gather_one(const orc_sim *S, const double *arr, int comp,
                         double xi, double yi) {
  double wx[3], wy[3] = {1.0, 0.0, 0.0};
  long i0 = weights3(xi, STAG_X[comp], wx);
  long j0 = 0;
  int ny = 1;
  if (S->g.dims == 2) {
    j0 = weights3(yi, STAG_Y[comp], wy);
    ny = 3;
  }
  double v = 0.0;
  for (int b = 0; b < ny; ++b)
    for (int a = 0; a < 3; ++a) {
      long ia = i0 + a + G;
      long ja = (S->g.dims == 2) ? j0 + b + G : 0;
      v += wx[a] * wy[b] * AT(arr, ia, ja);
    }
  return v;
}

static void gather6(const orc_sim *S, double *const src[6], double x, double y,
                    double E[3], double B[3]) {
  double xi = x / S->g.dx;
  double yi = (S->g.dims == 2) ? y / S->g.dy : 0.0;
  for (int c = 0; c < 3; ++c) E[c] = gather_one(S, src[c], c, xi, yi);
  for (int c = 0; c < 3; ++c) B[c] = gather_one(S, src[3 + c], 3 + c, xi, yi);
  if (S->g.dims == 1) B[0] = 0.0; /* 1D: Bx is constant (zero) */
}

void orc_gather_arrays(const orc_sim *S, double x, double y, double E[3],
                       double B[3]) {
  double *src[6] = {S->f[ORC_EX], S->f[ORC_EY], S->f[ORC_EZ],
                    S->f[ORC_BX], S->f[ORC_BY], S->f[ORC_BZ]};
  gather6(S, src, x, y, E, B);
}

/* ------------------------------------------------------------------------ */
/* Esirkepov (2001) charge-conserving deposition                            */
/* ------------------------------------------------------------------------ */

/* order-2 shape of a particle at xi on the 5 nodes i0-2 .. i0+2 */
static void shape5(double xi, long i0, double S5[5]) {
  for (int k = -2; k <= 2; ++k) S5[k + 2] = orc_shape2(xi - (double)(i0 + k));
}

static void deposit(orc_sim *S, double qw, double x0, double y0, double x1,
                    double y1, double vy, double vz) {
  const double dx = S->g.dx, dt = S->g.dt;
  double xi0 = x0 / dx, xi1 = x1 / dx;
  long ix = (long)floor(xi0 + 0.5);
  double S0x[5], S1x[5], DSx[5];
  shape5(xi0, ix, S0x);
  shape5(xi1, ix, S1x);
  for (int k = 0; k < 5; ++k) DSx[k] = S1x[k] - S0x[k];
  double *Jx = S->f[ORC_JX], *Jy = S->f[ORC_JY], *Jz = S->f[ORC_JZ];

  if (S->g.dims == 1) {
    /* longitudinal: J_x(i+1/2) - J_x(i-1/2) = -q w (dx/dt) (S1 - S0)(i) */
    double acc = 0.0;
    for (int k = 0; k < 4; ++k) {
      acc += -qw * (dx / dt) * DSx[k];
      AT(Jx, ix - 2 + k + G, 0) += acc;
    }
    /* transverse: q w v (S0 + S1)/2 */
    for (int k = 0; k < 5; ++k) {
      double wv = 0.5 * (S0x[k] + S1x[k]);
      AT(Jy, ix - 2 + k + G, 0) += qw * vy * wv;
      AT(Jz, ix - 2 + k + G, 0) += qw * vz * wv;
    }
    return;
  }

  const double dy = S->g.dy;
  double yi0 = y0 / dy, yi1 = y1 / dy;
  long iy = (long)floor(yi0 + 0.5);
  double S0y[5], S1y[5], DSy[5];
  shape5(yi0, iy, S0y);
  shape5(yi1, iy, S1y);
  for (int k = 0; k < 5; ++k) DSy[k] = S1y[k] - S0y[k];

  double Wx[5][5], Wy[5][5], Wz[5][5]; /* [kx][ky] */
  for (int a = 0; a < 5; ++a)
    for (int b = 0; b < 5; ++b) {
      Wx[a][b] = DSx[a] * (S0y[b] + 0.5 * DSy[b]);
      Wy[a][b] = DSy[b] * (S0x[a] + 0.5 * DSx[a]);
      Wz[a][b] = S0x[a] * S0y[b] + 0.5 * DSx[a] * S0y[b] +
                 0.5 * S0x[a] * DSy[b] + DSx[a] * DSy[b] / 3.0;
    }
  for (int b = 0; b < 5; ++b) {
    double acc = 0.0;
    for (int a = 0; a < 4; ++a) {
      acc += -qw * (dx / dt) * Wx[a][b];
      AT(Jx, ix - 2 + a + G, iy - 2 + b + G) += acc;
    }
  }
  for (int a = 0; a < 5; ++a) {
    double acc = 0.0;
    for (int b = 0; b < 4; ++b) {
      acc += -qw * (dy / dt) * Wy[a][b];
      AT(Jy, ix - 2 + a + G, iy - 2 + b + G) += acc;
    }
  }
  for (int a = 0; a < 5; ++a)
    for (int b = 0; b < 5; ++b)
      AT(Jz, ix - 2 + a + G, iy - 2 + b + G) += qw * vz * Wz[a][b];
}

/* ------------------------------------------------------------------------ */
/* Yee solver for the scattered field                                       */
/* ------------------------------------------------------------------------ */

static void faraday(orc_sim *S) {
  const long NX = S->NX, NY = S->NY;
  const double cx = S->g.dt / S->g.dx;
  double *Ex = S->f[ORC_EX], *Ey = S->f[ORC_EY], *Ez = S->f[ORC_EZ];
  double *Bx = S->f[ORC_BX], *By = S->f[ORC_BY], *Bz = S->f[ORC_BZ];
  for (int c = 0; c < 3; ++c)
    memcpy(S->bold[c], S->f[ORC_BX + c], (size_t)(NX * NY) * 8);
  if (S->g.dims == 1) {
    for (long i = 0; i + 1 < NX; ++i) {
      AT(By, i, 0) += cx * (AT(Ez, i + 1, 0) - AT(Ez, i, 0));
      AT(Bz, i, 0) -= cx * (AT(Ey, i + 1, 0) - AT(Ey, i, 0));
    }
  } else {
    const double cy = S->g.dt / S->g.dy;
    for (long j = 0; j + 1 < NY; ++j)
      for (long i = 0; i < NX; ++i)
        AT(Bx, i, j) -= cy * (AT(Ez, i, j + 1) - AT(Ez, i, j));
    for (long j = 0; j < NY; ++j)
      for (long i = 0; i + 1 < NX; ++i)
        AT(By, i, j) += cx * (AT(Ez, i + 1, j) - AT(Ez, i, j));
    for (long j = 0; j + 1 < NY; ++j)
      for (long i = 0; i + 1 < NX; ++i)
        AT(Bz, i, j) -= cx * (AT(Ey, i + 1, j) - AT(Ey, i, j)) -
                        cy * (AT(Ex, i, j + 1) - AT(Ex, i, j));
  }
  for (int c = 0; c < 3; ++c)
    for (long k = 0; k < NX * NY; ++k)
      S->bbar[c][k] = 0.5 * (S->bold[c][k] + S->f[ORC_BX + c][k]);
}

/* First-order Mur (1981): at a face node b with inward neighbour n,
 * E_b^{n+1} = E_n^n + (dt - h)/(dt + h) (E_n^{n+1} - E_b^n). */
static double mur(double en_old, double en_new, double eb_old, double k) {
  return en_old + k * (en_new - eb_old);
}

static void ampere(orc_sim *S) {
  const long NX = S->NX, NY = S->NY;
  const double dt = S->g.dt, cx = dt / S->g.dx;
  const double kx = (dt - S->g.dx) / (dt + S->g.dx);
  double *Ex = S->f[ORC_EX], *Ey = S->f[ORC_EY], *Ez = S->f[ORC_EZ];
  double *Bx = S->f[ORC_BX], *By = S->f[ORC_BY], *Bz = S->f[ORC_BZ];
  double *Jx = S->f[ORC_JX], *Jy = S->f[ORC_JY], *Jz = S->f[ORC_JZ];
  for (int c = 0; c < 3; ++c)
    memcpy(S->eold[c], S->f[ORC_EX + c], (size_t)(NX * NY) * 8);
  double *Ox = S->eold[0], *Oy = S->eold[1], *Oz = S->eold[2];

  if (S->g.dims == 1) {
    for (long i = 0; i + 1 < NX; ++i) AT(Ex, i, 0) -= dt * AT(Jx, i, 0);
    for (long i = 1; i + 1 < NX; ++i) {
      AT(Ey, i, 0) += -cx * (AT(Bz, i, 0) - AT(Bz, i - 1, 0)) - dt * AT(Jy, i, 0);
      AT(Ez, i, 0) += cx * (AT(By, i, 0) - AT(By, i - 1, 0)) - dt * AT(Jz, i, 0);
    }
    double *E2[2] = {Ey, Ez}, *O2[2] = {Oy, Oz};
    for (int c = 0; c < 2; ++c) {
      AT(E2[c], 0, 0) = mur(AT(O2[c], 1, 0), AT(E2[c], 1, 0), AT(O2[c], 0, 0), kx);
      AT(E2[c], NX - 1, 0) = mur(AT(O2[c], NX - 2, 0), AT(E2[c], NX - 2, 0),
                                 AT(O2[c], NX - 1, 0), kx);
    }
    return;
  }

  const double cy = dt / S->g.dy;
  const double ky = (dt - S->g.dy) / (dt + S->g.dy);
  for (long j = 1; j + 1 < NY; ++j)
    for (long i = 0; i + 1 < NX; ++i)
      AT(Ex, i, j) += cy * (AT(Bz, i, j) - AT(Bz, i, j - 1)) - dt * AT(Jx, i, j);
  for (long j = 0; j + 1 < NY; ++j)
    for (long i = 1; i + 1 < NX; ++i)
      AT(Ey, i, j) += -cx * (AT(Bz, i, j) - AT(Bz, i - 1, j)) - dt * AT(Jy, i, j);
  for (long j = 1; j + 1 < NY; ++j)
    for (long i = 1; i + 1 < NX; ++i)
      AT(Ez, i, j) += cx * (AT(By, i, j) - AT(By, i - 1, j)) -
                      cy * (AT(Bx, i, j) - AT(Bx, i, j - 1)) - dt * AT(Jz, i, j);
  /* tangential E on the y faces: Ex (all dual I), Ez (interior I) */
  for (long i = 0; i + 1 < NX; ++i) {
    AT(Ex, i, 0) = mur(AT(Ox, i, 1), AT(Ex, i, 1), AT(Ox, i, 0), ky);
    AT(Ex, i, NY - 1) = mur(AT(Ox, i, NY - 2), AT(Ex, i, NY - 2),
                            AT(Ox, i, NY - 1), ky);
  }
  for (long i = 1; i + 1 < NX; ++i) {
    AT(Ez, i, 0) = mur(AT(Oz, i, 1), AT(Ez, i, 1), AT(Oz, i, 0), ky);
    AT(Ez, i, NY - 1) = mur(AT(Oz, i, NY - 2), AT(Ez, i, NY - 2),
                            AT(Oz, i, NY - 1), ky);
  }
  /* tangential E on the x faces: Ey (all dual J), Ez (interior J) */
  for (long j = 0; j + 1 < NY; ++j) {
    AT(Ey, 0, j) = mur(AT(Oy, 1, j), AT(Ey, 1, j), AT(Oy, 0, j), kx);
    AT(Ey, NX - 1, j) = mur(AT(Oy, NX - 2, j), AT(Ey, NX - 2, j),
                            AT(Oy, NX - 1, j), kx);
  }
  for (long j = 1; j + 1 < NY; ++j) {
    AT(Ez, 0, j) = mur(AT(Oz, 1, j), AT(Ez, 1, j), AT(Oz, 0, j), kx);
    AT(Ez, NX - 1, j) = mur(AT(Oz, NX - 2, j), AT(Ez, NX - 2, j),
                            AT(Oz, NX - 1, j), kx);
  }
  /* Ez corners: x-face rule with the (already updated) y-face neighbour */
  long jc[2] = {0, NY - 1};
  for (int c = 0; c < 2; ++c) {
    long j = jc[c];
    AT(Ez, 0, j) = mur(AT(Oz, 1, j), AT(Ez, 1, j), AT(Oz, 0, j), kx);
    AT(Ez, NX - 1, j) = mur(AT(Oz, NX - 2, j), AT(Ez, NX - 2, j),
                            AT(Oz, NX - 1, j), kx);
  }
}

/* ------------------------------------------------------------------------ */
/* Step                                                                     */
/* ------------------------------------------------------------------------ */

/* Incident field sampled where the Yee grid stores each component, at time t
 * (the prescribed-field reading of Sec. 2): tot[c] = src[c] + F_inc,c at the
 * node of every array element, guard nodes included. */
static void add_incident_on_nodes(const orc_sim *S, double *const src[6],
                                  double t, double *tot[6]) {
  const int dims = S->g.dims;
  for (int c = 0; c < 6; ++c)
    for (long ja = 0; ja < S->NY; ++ja)
      for (long ia = 0; ia < S->NX; ++ia) {
        double x = ((double)(ia - G) + 0.5 * STAG_X[c]) * S->g.dx;
        double y = (dims == 2) ? ((double)(ja - G) + 0.5 * STAG_Y[c]) * S->g.dy
                               : 0.0;
        double E[3], B[3];
        orc_incident_eval(&S->inc, dims, x, y, t, E, B);
        AT(tot[c], ia, ja) = AT(src[c], ia, ja) + (c < 3 ? E[c] : B[c - 3]);
      }
}

void orc_step(orc_sim *S, long nsteps) {
  const double dt = S->g.dt;
  const int dims = S->g.dims;
  const double xmax = S->g.nx * S->g.dx;
  const double ymax = (dims == 2) ? S->g.ny * S->g.dy : 0.0;
  const long ncell = S->NX * S->NY;
  double *tot[6] = {0};
  if (S->inc.on_nodes)
    for (int c = 0; c < 6; ++c) tot[c] = (double *)malloc((size_t)ncell * 8);
  for (long k = 0; k < nsteps; ++k) {
    const double t = (double)S->step * dt;
    faraday(S);
    for (int c = 0; c < 3; ++c) memset(S->f[ORC_JX + c], 0, (size_t)ncell * 8);
    double *src[6] = {S->f[ORC_EX], S->f[ORC_EY], S->f[ORC_EZ],
                      S->bbar[0], S->bbar[1], S->bbar[2]};
    if (S->inc.on_nodes) {
      add_incident_on_nodes(S, src, t, tot);
      for (int c = 0; c < 6; ++c) src[c] = tot[c];
    }
    for (int s = 0; s < S->nsp; ++s) {
      orc_species *p = &S->sp[s];
      const double qm = p->q / p->m;
      for (long i = 0; i < p->n; ++i) {
        if (!p->alive[i]) continue;
        double x0 = p->x[i], y0 = p->y[i];
        double E[3], B[3], Ei[3], Bi[3];
        gather6(S, src, x0, y0, E, B);
        if (!S->inc.on_nodes) {
          orc_incident_eval(&S->inc, dims, x0, y0, t, Ei, Bi);
          for (int c = 0; c < 3; ++c) {
            E[c] += Ei[c];
            B[c] += Bi[c];
          }
        }
        double u[3] = {p->ux[i], p->uy[i], p->uz[i]};
        orc_boris(qm, dt, u, E, B);
        double gam = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        double x1 = x0 + dt * u[0] / gam;
        double y1 = (dims == 2) ? y0 + dt * u[1] / gam : 0.0;
        deposit(S, p->q * p->w, x0, y0, x1, y1, u[1] / gam, u[2] / gam);
        p->x[i] = x1;
        p->y[i] = y1;
        p->ux[i] = u[0];
        p->uy[i] = u[1];
        p->uz[i] = u[2];
        if (x1 < 0.0 || x1 >= xmax || (dims == 2 && (y1 < 0.0 || y1 >= ymax)))
          p->alive[i] = 0;
      }
    }
    ampere(S);
    S->step++;
  }
  for (int c = 0; c < 6; ++c) free(tot[c]);
}

/* ------------------------------------------------------------------------ */
/* Diagnostics                                                              */
/* ------------------------------------------------------------------------ */

void orc_deposit_rho(const orc_sim *S, double *rho) {
  memset(rho, 0, (size_t)(S->NX * S->NY) * 8);
  for (int s = 0; s < S->nsp; ++s) {
    const orc_species *p = &S->sp[s];
    for (long i = 0; i < p->n; ++i) {
      if (!p->alive[i]) continue;
      double wx[3], wy[3] = {1.0, 0.0, 0.0};
      long i0 = weights3(p->x[i] / S->g.dx, 0, wx), j0 = 0;
      int nb = 1;
      if (S->g.dims == 2) {
        j0 = weights3(p->y[i] / S->g.dy, 0, wy);
        nb = 3;
      }
      for (int b = 0; b < nb; ++b)
        for (int a = 0; a < 3; ++a) {
          long ja = (S->g.dims == 2) ? j0 + b + G : 0;
          AT(rho, i0 + a + G, ja) += p->q * p->w * wx[a] * wy[b];
        }
    }
  }
}

static double cell_volume(const orc_sim *S) {
  return (S->g.dims == 2) ? S->g.dx * S->g.dy : S->g.dx;
}

void orc_diagnostics(const orc_sim *S, double out[4]) {
  double dV = cell_volume(S);
  double wk = 0.0, q = 0.0, na = 0.0, wem = 0.0;
  for (int s = 0; s < S->nsp; ++s) {
    const orc_species *p = &S->sp[s];
    for (long i = 0; i < p->n; ++i) {
      if (!p->alive[i]) continue;
      double u2 = p->ux[i] * p->ux[i] + p->uy[i] * p->uy[i] + p->uz[i] * p->uz[i];
      wk += p->w * p->m * (sqrt(1.0 + u2) - 1.0) * dV;
      q += p->q * p->w * dV;
      na += 1.0;
    }
  }
  for (int c = 0; c < 6; ++c)
    for (long k = 0; k < S->NX * S->NY; ++k) wem += 0.5 * S->f[c][k] * S->f[c][k];
  out[0] = wk;
  out[1] = wem * dV;
  out[2] = q;
  out[3] = na;
}

/* Energy of the total field F_inc + F_scatt (Sec. 2) on the physical nodes:
 * (1/2) sum |E_s^n + E_inc(t^n)|^2 + |B_s^{n-1/2} + B_inc(t^{n-1/2})|^2 dV.
 * Each component is taken where the Yee grid stores it (the staggering in the
 * header) and at the time level of the stored scattered field. */
double orc_em_energy_total(const orc_sim *S) {
  const int dims = S->g.dims;
  const long ny = (dims == 2) ? S->g.ny : 1;
  const double tE = (double)S->step * S->g.dt;
  const double tB = tE - 0.5 * S->g.dt;
  double w = 0.0;
  for (long j = 0; j < ny; ++j)
    for (long i = 0; i < S->g.nx; ++i)
      for (int c = 0; c < 6; ++c) {
        double x = ((double)i + 0.5 * STAG_X[c]) * S->g.dx;
        double y = (dims == 2) ? ((double)j + 0.5 * STAG_Y[c]) * S->g.dy : 0.0;
        double E[3], B[3];
        orc_incident_eval(&S->inc, dims, x, y, c < 3 ? tE : tB, E, B);
        double fi = (c < 3) ? E[c] : B[c - 3];
        double fs = AT(S->f[c], i + G, (dims == 2) ? j + G : 0);
        w += 0.5 * (fs + fi) * (fs + fi);
      }
  return w * cell_volume(S);
}

void orc_energy_angle(const orc_sim *S, int sp, int n_e, double emax,
                      int n_theta, double ek_min, int plane, double *hist,
                      double mom[5]) {
  const orc_species *p = &S->sp[sp];
  double dV = cell_volume(S);
  memset(hist, 0, (size_t)n_e * (size_t)n_theta * 8);
  for (int k = 0; k < 5; ++k) mom[k] = 0.0;
  for (long i = 0; i < p->n; ++i) {
    if (!p->alive[i]) continue;
    double ux = p->ux[i], uy = p->uy[i], uz = p->uz[i];
    double ek = p->m * (sqrt(1.0 + ux * ux + uy * uy + uz * uz) - 1.0);
    /* angle from +x of u (plane 0) or of its projection on the x-z (1) or
     * x-y (2) plane */
    double perp = plane == 1   ? fabs(uz)
                  : plane == 2 ? fabs(uy)
                               : sqrt(uy * uy + uz * uz);
    double th = atan2(perp, ux) * (180.0 / ORC_PI);
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
