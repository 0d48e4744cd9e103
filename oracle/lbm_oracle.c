/*
 * lbm_oracle.c -- plain FP64 CPU reference of the plane-strain LBM of
 * arXiv 2301.00228 (Schlueter et al.).
 *
 * TEST INFRASTRUCTURE ONLY: used by the test-suite, the smoke entry point and
 * the benchmark's CPU-baseline leg to check and time the GPU library.  It is
 * deliberately slow and literal: every time step performs the sub-steps of
 * the paper's algorithm summary (Fig. 4) in the paper's order, with the
 * general BGK collision (explicit equilibrium and flux), separate arrays for
 * t and t+dt, and no fusion.  Build with -O2 -ffp-contract=off.
 *
 * Readings of points the paper leaves open (each one is applied identically
 * by the GPU library, which is written separately):
 *  - velocity set D2Q5 (Sec. 3, D2Q5 scheme);
 *  - shear speed c_s = sqrt(mu/rho): the derivation of eq. wave-navier needs
 *    mu, the printed lambda is a typo;
 *  - dt/tau = 2 both in eq. LBE and in eq. LBE_mod (tau = dt/2, Sec. 3);
 *  - J = sum over all alpha of c^alpha f^alpha (c^0 = 0), eq. feq;
 *  - initial flux J = 0: f(x,0) = f_eq(field, J = 0);
 *  - interior derivatives of phi and psi: central differences;
 *  - finite differences of u (Sec. 3.1, eq. consistency): per axis central
 *    if both neighbours are in the body, else one-sided 3-point second
 *    order, else 2-point first order, else 0;
 *  - Neumann cell (Sec. 3.1, eq. acc_neumann), mask rule: the cell spans half
 *    a spacing towards every in-body neighbour and ends at the node towards a
 *    missing one; internal side towards neighbour r has the cell's extent
 *    across it as length and +-e_x / +-e_y as normal; a caller-given table
 *    (V, l_E, l_N, l_W, l_S) may replace it.  Nodes lacking both neighbours
 *    along one axis are rejected (zero cell volume).  The sum of eq.
 *    acc_neumann runs over the neighbours in the body only: a length given
 *    towards a missing neighbour is not used;
 *  - Dirichlet acceleration uses u*(t+dt) (so that u(t+dt) = u*);
 *  - correction-f (eq. correction-f) uses the flux of the populations stored
 *    at the boundary node at time t (reading R1; orc_set_readings switches
 *    to R2: the flux of the post-collision populations that stream into the
 *    boundary node from its body neighbours, a missing neighbour adding 0);
 *  - eq. LBE_mod: equilibrium of the averaged populations' own moments
 *    (reading M1; orc_set_readings switches to M2: the equilibrium of the
 *    boundary node's populations at t);
 *  - velocity update of eq. integration uses only the acceleration at t
 *    (orc_set_integrator(p, 1) switches to the central difference, Newmark
 *    gamma = 1/2, for the variant study);
 *  - synchronization (Sec. 3.2) at the end of step m when m % l == 0, at
 *    every node, keeping the current flux;
 *  - Neumann load amplitude at t = n dt, Dirichlet at (n+1) dt, with t
 *    computed as n*dt;
 *  - fields are 0 outside the body.
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NQ 5
/* D2Q5 lattice directions in units of c (Sec. 3, lattice velocities). */
static const int CX[NQ] = {0, 1, 0, -1, 0};
static const int CY[NQ] = {0, 0, 1, 0, -1};

enum { CLS_OUT = 0, CLS_INT = 1, CLS_BND = 2 };
enum { BC_NEUMANN = 0, BC_DIRICHLET = 1 };

typedef struct {
  int n;
  double *t, *g;
} orc_load;

struct orc_plate {
  int nx, ny, px, py;
  double lam, mu, rho_m, dh, dt;
  double c, cd, cs;
  double a[2], a0[2];
  int sync_every;
  int integrator; /* 0: eq. integration as printed; 1: central difference */
  int flux_reading; /* eq. correction-f: 0 = R1, 1 = R2 (see file header) */
  int eq_reading;   /* eq. LBE_mod: 0 = M1, 1 = M2 (see file header) */
  int64_t n; /* completed steps */
  int started;
  uint8_t *in;  /* 1 = in body */
  uint8_t *cls; /* CLS_* */
  double *f[2][NQ];
  double *fn[2][NQ];
  double *ux, *uy, *vx, *vy, *ax, *ay;
  double *rho[2], *jx[2], *jy[2]; /* moments of f at time t */
  /* boundary data, per node */
  uint8_t *kind;
  double *bvx, *bvy;
  int *grp;
  uint8_t *has_cell;
  double *cell; /* 5 per node */
  int nload;
  orc_load *load;
};

/* ---------------------------------------------------------------- helpers */

/* Index of the node (i+di, j+dj) if it exists and lies in the body, else -1.
 * Periodic axes wrap. */
static long nbr(const orc_plate *p, int i, int j, int di, int dj) {
  int ii = i + di, jj = j + dj;
  if (ii < 0 || ii >= p->nx) {
    if (!p->px) return -1;
    ii = (ii % p->nx + p->nx) % p->nx;
  }
  if (jj < 0 || jj >= p->ny) {
    if (!p->py) return -1;
    jj = (jj % p->ny + p->ny) % p->ny;
  }
  long k = (long)jj * p->nx + ii;
  return p->in[k] ? k : -1;
}

/* Finite-difference derivative of q along axis ax (0 = x, 1 = y) at (i, j),
 * following the per-axis stencil rule listed in the file header. */
static double fd(const orc_plate *p, const double *q, int i, int j, int ax) {
  int di = ax == 0, dj = ax == 1;
  long k0 = (long)j * p->nx + i;
  long kp = nbr(p, i, j, di, dj);
  long km = nbr(p, i, j, -di, -dj);
  double h = p->dh;
  if (kp >= 0 && km >= 0) return (q[kp] - q[km]) / (2.0 * h);
  if (kp >= 0) {
    long kpp = nbr(p, i, j, 2 * di, 2 * dj);
    if (kpp >= 0) return ((-3.0 * q[k0] + 4.0 * q[kp]) - q[kpp]) / (2.0 * h);
    return (q[kp] - q[k0]) / h;
  }
  if (km >= 0) {
    long kmm = nbr(p, i, j, -2 * di, -2 * dj);
    if (kmm >= 0) return ((3.0 * q[k0] - 4.0 * q[km]) + q[kmm]) / (2.0 * h);
    return (q[k0] - q[km]) / h;
  }
  return 0.0;
}

/* div u and (curl u).e_z by finite differences (Sec. 2, eq. phi-psi). */
static void div_curl(const orc_plate *p, const double *ux, const double *uy, int i, int j,
                     double *dv, double *cu) {
  double dxux = fd(p, ux, i, j, 0), dyuy = fd(p, uy, i, j, 1);
  double dxuy = fd(p, uy, i, j, 0), dyux = fd(p, ux, i, j, 1);
  *dv = dxux + dyuy;
  *cu = dxuy - dyux;
}

/* Cauchy stress from Hooke's law (Sec. 2, eqs. strain and hooke) with the
 * strain from finite differences of u. */
static void stress(const orc_plate *p, const double *ux, const double *uy, int i, int j,
                   double *sxx, double *syy, double *sxy) {
  double exx = fd(p, ux, i, j, 0);
  double eyy = fd(p, uy, i, j, 1);
  double exy = 0.5 * (fd(p, ux, i, j, 1) + fd(p, uy, i, j, 0));
  double tr = exx + eyy;
  *sxx = p->lam * tr + 2.0 * p->mu * exx;
  *syy = p->lam * tr + 2.0 * p->mu * eyy;
  *sxy = 2.0 * p->mu * exy;
}

/* Equilibrium distribution of eq. feq (b = 1). */
static double feq(const orc_plate *p, int fld, int al, double rho, double jx, double jy) {
  if (al == 0) return p->a0[fld] * rho;
  double cax = p->c * CX[al], cay = p->c * CY[al];
  double b = 1.0;
  return p->a[fld] * rho + b * (cax * jx + cay * jy) / (2.0 * p->c * p->c);
}

/* Zeroth and first moments (eqs. interpretation and feq). */
static void moments(const orc_plate *p, const double *fa, double *rho, double *jx, double *jy) {
  *rho = fa[0] + ((fa[1] + fa[3]) + (fa[2] + fa[4]));
  double sx = 0.0, sy = 0.0;
  for (int al = 0; al < NQ; al++) {
    sx += (p->c * CX[al]) * fa[al];
    sy += (p->c * CY[al]) * fa[al];
  }
  *jx = sx;
  *jy = sy;
}

static double load_amp(const orc_plate *p, int g, double t) {
  if (g < 0) return 1.0;
  const orc_load *L = &p->load[g];
  if (L->n <= 0) return 1.0;
  if (t <= L->t[0]) return L->g[0];
  if (t >= L->t[L->n - 1]) return L->g[L->n - 1];
  for (int m = 0; m + 1 < L->n; m++) {
    if (t <= L->t[m + 1]) {
      double w = (t - L->t[m]) / (L->t[m + 1] - L->t[m]);
      return L->g[m] + w * (L->g[m + 1] - L->g[m]);
    }
  }
  return L->g[L->n - 1];
}

/* ------------------------------------------------------------- lifecycle */

static void *zalloc(size_t n) { return calloc(n ? n : 1, 1); }

void orc_destroy(orc_plate *p) {
  if (!p) return;
  free(p->in);
  free(p->cls);
  for (int fl = 0; fl < 2; fl++) {
    for (int al = 0; al < NQ; al++) {
      free(p->f[fl][al]);
      free(p->fn[fl][al]);
    }
    free(p->rho[fl]);
    free(p->jx[fl]);
    free(p->jy[fl]);
  }
  free(p->ux); free(p->uy); free(p->vx); free(p->vy); free(p->ax); free(p->ay);
  free(p->kind); free(p->bvx); free(p->bvy); free(p->grp); free(p->has_cell); free(p->cell);
  for (int g = 0; g < p->nload; g++) {
    free(p->load[g].t);
    free(p->load[g].g);
  }
  free(p->load);
  free(p);
}

orc_plate *orc_create(int nx, int ny, const uint8_t *mask, int periodic_x, int periodic_y,
                      double lambda, double mu, double rho_m, double dh, double dt,
                      int sync_every, const double *u0, const double *v0,
                      const double *e0, const double *w0, int *err) {
  int e = ORC_OK;
  if (err) *err = ORC_OK;
  if (nx < 3 || ny < 3 || !(dh > 0) || !(dt > 0) || !(rho_m > 0) || !(mu > 0) ||
      !(lambda + 2.0 * mu > 0) || sync_every < 0) {
    if (err) *err = ORC_E_INVAL;
    return NULL;
  }
  orc_plate *p = (orc_plate *)zalloc(sizeof(orc_plate));
  if (!p) { if (err) *err = ORC_E_NOMEM; return NULL; }
  size_t N = (size_t)nx * ny;
  p->nx = nx; p->ny = ny; p->px = periodic_x != 0; p->py = periodic_y != 0;
  p->lam = lambda; p->mu = mu; p->rho_m = rho_m; p->dh = dh; p->dt = dt;
  p->sync_every = sync_every;

  /* Parameters: Sec. 2 wave speeds, Sec. 3 eqs. feq_req,
   * parameters_to_wavespeed_relation and conditions-parameters. */
  p->cd = sqrt((lambda + 2.0 * mu) / rho_m);
  p->cs = sqrt(mu / rho_m);
  p->c = dh / dt;
  double rd = p->cd * dt / dh, rs = p->cs * dt / dh;
  p->a[0] = 0.5 * rd * rd;
  p->a[1] = 0.5 * rs * rs;
  p->a0[0] = 1.0 - 4.0 * p->a[0];
  p->a0[1] = 1.0 - 4.0 * p->a[1];
  if (p->a0[0] < -1e-12) { orc_destroy(p); if (err) *err = ORC_E_UNSTABLE_DT; return NULL; }

  p->in = (uint8_t *)zalloc(N);
  p->cls = (uint8_t *)zalloc(N);
  for (int fl = 0; fl < 2; fl++) {
    for (int al = 0; al < NQ; al++) {
      p->f[fl][al] = (double *)zalloc(N * sizeof(double));
      p->fn[fl][al] = (double *)zalloc(N * sizeof(double));
    }
    p->rho[fl] = (double *)zalloc(N * sizeof(double));
    p->jx[fl] = (double *)zalloc(N * sizeof(double));
    p->jy[fl] = (double *)zalloc(N * sizeof(double));
  }
  p->ux = (double *)zalloc(N * sizeof(double));
  p->uy = (double *)zalloc(N * sizeof(double));
  p->vx = (double *)zalloc(N * sizeof(double));
  p->vy = (double *)zalloc(N * sizeof(double));
  p->ax = (double *)zalloc(N * sizeof(double));
  p->ay = (double *)zalloc(N * sizeof(double));
  p->kind = (uint8_t *)zalloc(N);
  p->bvx = (double *)zalloc(N * sizeof(double));
  p->bvy = (double *)zalloc(N * sizeof(double));
  p->grp = (int *)zalloc(N * sizeof(int));
  p->has_cell = (uint8_t *)zalloc(N);
  p->cell = (double *)zalloc(5 * N * sizeof(double));
  if (!p->cell || !p->ay) { orc_destroy(p); if (err) *err = ORC_E_NOMEM; return NULL; }

  for (size_t k = 0; k < N; k++) {
    p->in[k] = mask ? (mask[k] != 0) : 1;
    p->grp[k] = -1;
  }
  /* Classification (Fig. 2 / Fig. 5): boundary = in-body node with at least
   * one missing D2Q5 neighbour. */
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      long k = (long)j * nx + i;
      if (!p->in[k]) { p->cls[k] = CLS_OUT; continue; }
      int hasE = nbr(p, i, j, 1, 0) >= 0, hasW = nbr(p, i, j, -1, 0) >= 0;
      int hasN = nbr(p, i, j, 0, 1) >= 0, hasS = nbr(p, i, j, 0, -1) >= 0;
      if ((!hasE && !hasW) || (!hasN && !hasS)) e = ORC_E_INVAL;
      p->cls[k] = (hasE && hasW && hasN && hasS) ? CLS_INT : CLS_BND;
    }
  if (e != ORC_OK) { orc_destroy(p); if (err) *err = e; return NULL; }

  for (size_t k = 0; k < N; k++) {
    if (!p->in[k]) continue;
    if (u0) { p->ux[k] = u0[k]; p->uy[k] = u0[N + k]; }
    if (v0) { p->vx[k] = v0[k]; p->vy[k] = v0[N + k]; }
  }
  /* Initialization (Fig. 4): phi, psi from finite differences of u0 unless
   * given; f = f_eq(field, J = 0). */
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      long k = (long)j * nx + i;
      if (!p->in[k]) continue;
      double dv, cu;
      div_curl(p, p->ux, p->uy, i, j, &dv, &cu);
      double fld0[2] = {e0 ? e0[k] : dv, w0 ? w0[k] : cu};
      for (int fl = 0; fl < 2; fl++)
        for (int al = 0; al < NQ; al++) p->f[fl][al][k] = feq(p, fl, al, fld0[fl], 0.0, 0.0);
    }
  return p;
}

int orc_set_integrator(orc_plate *p, int integrator) {
  if (!p || p->started || (integrator != 0 && integrator != 1)) return ORC_E_INVAL;
  p->integrator = integrator;
  return ORC_OK;
}

int orc_set_readings(orc_plate *p, int flux_reading, int eq_reading) {
  if (!p || p->started || (flux_reading != 0 && flux_reading != 1) ||
      (eq_reading != 0 && eq_reading != 1))
    return ORC_E_INVAL;
  p->flux_reading = flux_reading;
  p->eq_reading = eq_reading;
  return ORC_OK;
}

int orc_set_bc(orc_plate *p, int n, const int32_t *xy, const uint8_t *kind, const double *val,
               const double *cell, int n_knots, const double *knots) {
  if (!p || n < 0 || (n > 0 && (!xy || !kind || !val)) || n_knots < 0 || (n_knots > 0 && !knots))
    return ORC_E_INVAL;
  if (p->started) return ORC_E_STATE;
  for (int m = 0; m < n; m++) {
    int i = xy[2 * m], j = xy[2 * m + 1];
    if (i < 0 || i >= p->nx || j < 0 || j >= p->ny) return ORC_E_INVAL;
    if (p->cls[(long)j * p->nx + i] != CLS_BND) return ORC_E_INVAL;
    if (kind[m] > 1) return ORC_E_INVAL;
    if (cell && !(cell[5 * m] > 0)) return ORC_E_INVAL;
  }
  for (int m = 1; m < n_knots; m++)
    if (!(knots[2 * m] > knots[2 * m - 2])) return ORC_E_INVAL;
  int g = -1;
  if (n_knots > 0) {
    orc_load *L = (orc_load *)realloc(p->load, (size_t)(p->nload + 1) * sizeof(orc_load));
    if (!L) return ORC_E_NOMEM;
    p->load = L;
    g = p->nload++;
    L[g].n = n_knots;
    L[g].t = (double *)zalloc((size_t)n_knots * sizeof(double));
    L[g].g = (double *)zalloc((size_t)n_knots * sizeof(double));
    for (int m = 0; m < n_knots; m++) {
      L[g].t[m] = knots[2 * m];
      L[g].g[m] = knots[2 * m + 1];
    }
  }
  for (int m = 0; m < n; m++) {
    long k = (long)xy[2 * m + 1] * p->nx + xy[2 * m];
    p->kind[k] = kind[m];
    p->bvx[k] = val[2 * m];
    p->bvy[k] = val[2 * m + 1];
    p->grp[k] = g;
    if (cell) {
      p->has_cell[k] = 1;
      for (int q = 0; q < 5; q++) p->cell[5 * k + q] = cell[5 * m + q];
    }
  }
  return ORC_OK;
}

/* ------------------------------------------------------------ time step */

/* Neumann acceleration of eq. acc_neumann at boundary node (i, j). */
static void accel_neumann(const orc_plate *p, int i, int j, double g, double *ax, double *ay) {
  long k = (long)j * p->nx + i;
  long kE = nbr(p, i, j, 1, 0), kN = nbr(p, i, j, 0, 1);
  long kW = nbr(p, i, j, -1, 0), kS = nbr(p, i, j, 0, -1);
  double V, lE, lN, lW, lS;
  if (p->has_cell[k]) {
    const double *c = &p->cell[5 * k];
    V = c[0]; lE = c[1]; lN = c[2]; lW = c[3]; lS = c[4];
  } else {
    /* Mask rule: half a spacing towards each in-body neighbour. */
    double wx = 0.5 * p->dh * ((kW >= 0) + (kE >= 0));
    double wy = 0.5 * p->dh * ((kS >= 0) + (kN >= 0));
    V = wx * wy;
    lE = (kE >= 0) ? wy : 0.0;
    lW = (kW >= 0) ? wy : 0.0;
    lN = (kN >= 0) ? wx : 0.0;
    lS = (kS >= 0) ? wx : 0.0;
  }
  double sxx, syy, sxy;
  stress(p, p->ux, p->uy, i, j, &sxx, &syy, &sxy);
  /* sigma_kr n_kr l_kr with sigma_kr the mean of the two nodal stresses. */
  double tEx = 0, tEy = 0, tWx = 0, tWy = 0, tNx = 0, tNy = 0, tSx = 0, tSy = 0;
  double rxx, ryy, rxy;
  if (kE >= 0) {
    stress(p, p->ux, p->uy, (int)(kE % p->nx), (int)(kE / p->nx), &rxx, &ryy, &rxy);
    tEx = 0.5 * (sxx + rxx) * lE;
    tEy = 0.5 * (sxy + rxy) * lE;
  }
  if (kW >= 0) {
    stress(p, p->ux, p->uy, (int)(kW % p->nx), (int)(kW / p->nx), &rxx, &ryy, &rxy);
    tWx = -(0.5 * (sxx + rxx)) * lW;
    tWy = -(0.5 * (sxy + rxy)) * lW;
  }
  if (kN >= 0) {
    stress(p, p->ux, p->uy, (int)(kN % p->nx), (int)(kN / p->nx), &rxx, &ryy, &rxy);
    tNx = 0.5 * (sxy + rxy) * lN;
    tNy = 0.5 * (syy + ryy) * lN;
  }
  if (kS >= 0) {
    stress(p, p->ux, p->uy, (int)(kS % p->nx), (int)(kS / p->nx), &rxx, &ryy, &rxy);
    tSx = -(0.5 * (sxy + rxy)) * lS;
    tSy = -(0.5 * (syy + ryy)) * lS;
  }
  double Fx = g * p->bvx[k], Fy = g * p->bvy[k];
  *ax = (((tEx + tWx) + (tNx + tSx)) + Fx) / (p->rho_m * V);
  *ay = (((tEy + tWy) + (tNy + tSy)) + Fy) / (p->rho_m * V);
}

static void one_step(orc_plate *p) {
  const int nx = p->nx, ny = p->ny;
  const double dt = p->dt;
  const double t_now = (double)p->n * dt, t_next = (double)(p->n + 1) * dt;

  /* 1. Moments of f(t) at every in-body node. */
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      long k = (long)j * nx + i;
      if (!p->in[k]) continue;
      for (int fl = 0; fl < 2; fl++) {
        double fa[NQ];
        for (int al = 0; al < NQ; al++) fa[al] = p->f[fl][al][k];
        moments(p, fa, &p->rho[fl][k], &p->jx[fl][k], &p->jy[fl][k]);
      }
    }

  /* 2. Accelerations: interior by eq. navier (c_d^2 grad phi - c_s^2 curl
   *    psi), boundary by eqs. acc_neumann / acc_dirichlet. */
  const double cd2 = p->cd * p->cd, cs2 = p->cs * p->cs;
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      long k = (long)j * nx + i;
      if (p->cls[k] == CLS_INT) {
        long kE = nbr(p, i, j, 1, 0), kW = nbr(p, i, j, -1, 0);
        long kN = nbr(p, i, j, 0, 1), kS = nbr(p, i, j, 0, -1);
        double h2 = 2.0 * p->dh;
        double dphix = (p->rho[0][kE] - p->rho[0][kW]) / h2;
        double dphiy = (p->rho[0][kN] - p->rho[0][kS]) / h2;
        double dpsix = (p->rho[1][kE] - p->rho[1][kW]) / h2;
        double dpsiy = (p->rho[1][kN] - p->rho[1][kS]) / h2;
        /* curl of psi e_z = (d_y psi, -d_x psi) */
        p->ax[k] = cd2 * dphix - cs2 * dpsiy;
        p->ay[k] = cd2 * dphiy - cs2 * (-dpsix);
      } else if (p->cls[k] == CLS_BND) {
        if (p->kind[k] == BC_DIRICHLET) {
          double g = load_amp(p, p->grp[k], t_next);
          double usx = g * p->bvx[k], usy = g * p->bvy[k];
          if (p->integrator == 1 && p->n > 0) {
            /* central difference: u(t+dt) = u + dt (v + dt a) with v at t - dt/2 */
            p->ax[k] = (usx - p->ux[k]) / (dt * dt) - p->vx[k] / dt;
            p->ay[k] = (usy - p->uy[k]) / (dt * dt) - p->vy[k] / dt;
          } else {
            p->ax[k] = 2.0 / (dt * dt) * (usx - p->ux[k]) - 2.0 / dt * p->vx[k];
            p->ay[k] = 2.0 / (dt * dt) * (usy - p->uy[k]) - 2.0 / dt * p->vy[k];
          }
        } else {
          double g = load_amp(p, p->grp[k], t_now);
          accel_neumann(p, i, j, g, &p->ax[k], &p->ay[k]);
        }
      } else {
        p->ax[k] = 0.0;
        p->ay[k] = 0.0;
      }
    }

  /* 3. Explicit Newmark step of eq. integration at every in-body node. */
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      long k = (long)j * nx + i;
      if (!p->in[k]) continue;
      double ux = p->ux[k], uy = p->uy[k], vx = p->vx[k], vy = p->vy[k];
      if (p->integrator == 1) {
        /* central difference (Newmark gamma = 1/2, beta = 0) with the
         * velocity at half steps: v(t+dt/2) = v(t-dt/2) + dt a(t), u(t+dt) =
         * u(t) + dt v(t+dt/2); the first step starts from v(0):
         * v(dt/2) = v(0) + dt/2 a(0) */
        double h = p->n == 0 ? 0.5 * dt : dt;
        p->vx[k] = vx + h * p->ax[k];
        p->vy[k] = vy + h * p->ay[k];
        p->ux[k] = ux + dt * p->vx[k];
        p->uy[k] = uy + dt * p->vy[k];
      } else {
        p->ux[k] = ux + dt * vx + dt * dt / 2.0 * p->ax[k];
        p->uy[k] = uy + dt * vy + dt * dt / 2.0 * p->ay[k];
        p->vx[k] = vx + dt * p->ax[k];
        p->vy[k] = vy + dt * p->ay[k];
      }
    }

  /* 4. Boundary nodes: phi, psi from finite differences of u(t+dt)
   *    (eq. psi_phi_at_bound), populations by eq. correction-f with the
   *    flux J(x_k, t): R1, that of the populations stored there at time t;
   *    R2, that of the populations the LBE streams in from the body
   *    neighbours x_k - c^alpha dt (their post-collision populations at t,
   *    eq. LBE with dt/tau = 2), a missing neighbour contributing 0. */
  const double omega = dt / (0.5 * dt);
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      long k = (long)j * nx + i;
      if (p->cls[k] != CLS_BND) continue;
      double dv, cu;
      div_curl(p, p->ux, p->uy, i, j, &dv, &cu);
      double fld[2] = {dv, cu};
      for (int fl = 0; fl < 2; fl++) {
        double jx = p->jx[fl][k], jy = p->jy[fl][k];
        if (p->flux_reading == 1) {
          jx = 0.0;
          jy = 0.0;
          for (int al = 1; al < NQ; al++) {
            long ky = nbr(p, i, j, -CX[al], -CY[al]);
            if (ky < 0) continue;
            double fy = p->f[fl][al][ky];
            double fe = feq(p, fl, al, p->rho[fl][ky], p->jx[fl][ky], p->jy[fl][ky]);
            double fs = fy - omega * (fy - fe);
            jx += (p->c * CX[al]) * fs;
            jy += (p->c * CY[al]) * fs;
          }
        }
        for (int al = 0; al < NQ; al++) p->fn[fl][al][k] = feq(p, fl, al, fld[fl], jx, jy);
      }
    }

  /* 5. Interior nodes: LBE (eq. LBE, dt/tau = 2) pulled from the upwind
   *    neighbour; a population that leaves a boundary node is transported by
   *    eq. LBE_mod with the time-averaged boundary populations, collided
   *    towards the equilibrium of their own moments (M1) or of the boundary
   *    node's populations at t (M2). */
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      long k = (long)j * nx + i;
      if (p->cls[k] != CLS_INT) continue;
      for (int al = 0; al < NQ; al++) {
        long ks = nbr(p, i, j, -CX[al], -CY[al]); /* upwind node x - c^alpha dt */
        for (int fl = 0; fl < 2; fl++) {
          double fhat[NQ], rho, jx, jy;
          if (p->cls[ks] == CLS_BND) {
            for (int q = 0; q < NQ; q++) fhat[q] = 0.5 * (p->fn[fl][q][ks] + p->f[fl][q][ks]);
            if (p->eq_reading == 1) {
              rho = p->rho[fl][ks]; jx = p->jx[fl][ks]; jy = p->jy[fl][ks];
            } else {
              moments(p, fhat, &rho, &jx, &jy);
            }
          } else {
            for (int q = 0; q < NQ; q++) fhat[q] = p->f[fl][q][ks];
            rho = p->rho[fl][ks]; jx = p->jx[fl][ks]; jy = p->jy[fl][ks];
          }
          double fe = feq(p, fl, al, rho, jx, jy);
          p->fn[fl][al][k] = fhat[al] - omega * (fhat[al] - fe);
        }
      }
    }

  /* Swap t <-> t+dt populations. */
  for (int fl = 0; fl < 2; fl++)
    for (int al = 0; al < NQ; al++) {
      double *tmp = p->f[fl][al];
      p->f[fl][al] = p->fn[fl][al];
      p->fn[fl][al] = tmp;
    }
  p->n += 1;

  /* 6. Periodic synchronization (Sec. 3.2). */
  if (p->sync_every > 0 && p->n % p->sync_every == 0) {
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; j++)
      for (int i = 0; i < nx; i++) {
        long k = (long)j * nx + i;
        if (!p->in[k]) continue;
        double dv, cu;
        div_curl(p, p->ux, p->uy, i, j, &dv, &cu);
        double fld[2] = {dv, cu};
        for (int fl = 0; fl < 2; fl++) {
          double fa[NQ], rho, jx, jy;
          for (int al = 0; al < NQ; al++) fa[al] = p->f[fl][al][k];
          moments(p, fa, &rho, &jx, &jy);
          for (int al = 0; al < NQ; al++) p->f[fl][al][k] = feq(p, fl, al, fld[fl], jx, jy);
        }
      }
  }
}

int orc_step(orc_plate *p, int64_t n) {
  if (!p || n < 0) return ORC_E_INVAL;
  p->started = 1;
  for (int64_t s = 0; s < n; s++) one_step(p);
  return ORC_OK;
}

/* ------------------------------------------------------------- outputs */

void orc_fields(const orc_plate *p, double *e, double *w, double *u, double *v) {
  size_t N = (size_t)p->nx * p->ny;
  for (size_t k = 0; k < N; k++) {
    int inb = p->in[k];
    double s[2] = {0.0, 0.0};
    if (inb)
      for (int fl = 0; fl < 2; fl++)
        s[fl] = p->f[fl][0][k] + ((p->f[fl][1][k] + p->f[fl][3][k]) + (p->f[fl][2][k] + p->f[fl][4][k]));
    if (e) e[k] = s[0];
    if (w) w[k] = s[1];
    if (u) { u[k] = inb ? p->ux[k] : 0.0; u[N + k] = inb ? p->uy[k] : 0.0; }
    if (v) { v[k] = inb ? p->vx[k] : 0.0; v[N + k] = inb ? p->vy[k] : 0.0; }
  }
}

void orc_pops(const orc_plate *p, double *f) {
  size_t N = (size_t)p->nx * p->ny;
  for (int fl = 0; fl < 2; fl++)
    for (int al = 0; al < NQ; al++) memcpy(f + (size_t)(fl * NQ + al) * N, p->f[fl][al], N * sizeof(double));
}

void orc_set_pops(orc_plate *p, const double *f) {
  size_t N = (size_t)p->nx * p->ny;
  for (int fl = 0; fl < 2; fl++)
    for (int al = 0; al < NQ; al++) memcpy(p->f[fl][al], f + (size_t)(fl * NQ + al) * N, N * sizeof(double));
}

void orc_last_accel(const orc_plate *p, double *a) {
  size_t N = (size_t)p->nx * p->ny;
  memcpy(a, p->ax, N * sizeof(double));
  memcpy(a + N, p->ay, N * sizeof(double));
}

void orc_cons_err(const orc_plate *p, double *err) {
  for (int j = 0; j < p->ny; j++)
    for (int i = 0; i < p->nx; i++) {
      long k = (long)j * p->nx + i;
      if (!p->in[k]) { err[k] = 0.0; continue; }
      double dv, cu;
      div_curl(p, p->ux, p->uy, i, j, &dv, &cu);
      double s[2];
      for (int fl = 0; fl < 2; fl++)
        s[fl] = p->f[fl][0][k] + ((p->f[fl][1][k] + p->f[fl][3][k]) + (p->f[fl][2][k] + p->f[fl][4][k]));
      double d1 = s[1] - cu, d0 = s[0] - dv;
      err[k] = sqrt(d1 * d1 + d0 * d0);
    }
}

void orc_classes(const orc_plate *p, uint8_t *cls) { memcpy(cls, p->cls, (size_t)p->nx * p->ny); }

void orc_params(const orc_plate *p, double *o) {
  o[0] = p->a[0]; o[1] = p->a0[0]; o[2] = p->a[1]; o[3] = p->a0[1];
  o[4] = p->cd; o[5] = p->cs; o[6] = p->c;
}

int64_t orc_step_count(const orc_plate *p) { return p->n; }

int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
