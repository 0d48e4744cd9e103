/*
 * lbm_oracle.h -- plain FP64 CPU reference of the plane-strain lattice
 * Boltzmann method (Schlueter, Yan, Faust, Mueller, Mueller, arXiv 2301.00228).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against the paper.  Only the test-suite, the smoke entry point and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header,
 * table or helper with the GPU library, and the GPU library never calls it.
 *
 * Everything is FP64.  The algorithm follows the paper's Fig. 4 step order
 * literally (general BGK form with an explicit equilibrium and flux), with
 * separate population arrays for t and t+dt and plain loops over rows.
 *
 * Field index 0 is the dilatation phi = div u, field index 1 is the rotation
 * psi = (curl u).e_z (Sec. 2, eq. phi-psi).
 *
 * Arrays are row-major with x fastest: node (i, j) is at j*nx + i.  Vector
 * fields are planar: [2][ny][nx] (x component first).
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_plate orc_plate;

/* Error codes returned by the oracle. */
enum {
  ORC_OK = 0,
  ORC_E_INVAL = -1,        /* bad argument or unsupported mask            */
  ORC_E_UNSTABLE_DT = -2,  /* a_{0,phi} < 0 (Sec. 3, eq. feq_req)          */
  ORC_E_NOMEM = -3,
  ORC_E_STATE = -6         /* set_bc after the first step                  */
};

/* Create one plate.  mask: nx*ny bytes, 1 = node belongs to the body (NULL =
 * all nodes).  u0, v0: initial displacement and velocity, planar (NULL = 0).
 * e0, w0: optional direct initial dilatation / rotation (NULL = finite
 * differences of u0).  sync_every: l of Sec. 3.2 (0 = never).  On failure
 * returns NULL and writes the error code to *err (if err is non-NULL). */
orc_plate *orc_create(int nx, int ny, const uint8_t *mask, int periodic_x, int periodic_y,
                      double lambda, double mu, double rho_m, double dh, double dt,
                      int sync_every, const double *u0, const double *v0,
                      const double *e0, const double *w0, int *err);

/* Displacement update: 0 = eq. integration as printed (default), 1 = central
 * difference with the velocity kept at half steps.  Before the first step. */
int orc_set_integrator(orc_plate *p, int integrator);
/* Readings of two points the paper leaves open (Sec. 3.1), before the first
 * step.  flux_reading, the flux J(x_k, t) of eq. correction-f: 0 = R1, that
 * of the populations stored at the boundary node at t (default); 1 = R2,
 * that of the post-collision populations streaming into it from its body
 * neighbours (a missing neighbour contributes 0).  eq_reading, the
 * equilibrium of eq. LBE_mod: 0 = M1, that of the time-averaged populations'
 * own moments (default); 1 = M2, that of the boundary node's populations at
 * t. */
int orc_set_readings(orc_plate *p, int flux_reading, int eq_reading);
/* Boundary data for n boundary nodes.  xy: 2n ints (i, j).  kind: n bytes,
 * 0 = Neumann, 1 = Dirichlet.  val: 2n doubles, Dirichlet u* or Neumann
 * integrated external force over the cell's external boundary (per unit
 * thickness).  cell: NULL or 5n doubles (V, l_E, l_N, l_W, l_S) replacing
 * the mask-derived cell.  knots: n_knots (t, g) pairs giving a piecewise
 * linear amplitude g(t) (clamped outside the knot range) that multiplies val;
 * NULL means g = 1.  Listing a node that is not a boundary node is an error. */
int orc_set_bc(orc_plate *p, int n, const int32_t *xy, const uint8_t *kind, const double *val,
               const double *cell, int n_knots, const double *knots);

/* Advance n time steps. */
int orc_step(orc_plate *p, int64_t n);

/* e = sum f_phi, w = sum f_psi, u and v planar.  Any pointer may be NULL.
 * Nodes outside the body read 0. */
void orc_fields(const orc_plate *p, double *e, double *w, double *u, double *v);

/* Populations: 10*nx*ny doubles, [field][alpha][node]. */
void orc_pops(const orc_plate *p, double *f);
/* Overwrite the populations (same layout), e.g. to plant a perturbation. */
void orc_set_pops(orc_plate *p, const double *f);

/* Accelerations used in the most recent step (planar 2*nx*ny). */
void orc_last_accel(const orc_plate *p, double *a);

/* Consistency error of Sec. 4.1 at every node (nx*ny, 0 outside). */
void orc_cons_err(const orc_plate *p, double *err);

/* Node classes: 0 outside, 1 interior, 2 boundary (nx*ny bytes). */
void orc_classes(const orc_plate *p, uint8_t *cls);

/* Derived parameters: a_phi, a0_phi, a_psi, a0_psi, c_d, c_s, c. */
void orc_params(const orc_plate *p, double *out7);

int64_t orc_step_count(const orc_plate *p);

/* Number of OpenMP threads the oracle's loops use. */
int orc_threads(void);
void orc_destroy(orc_plate *p);

/* Set the number of OpenMP threads of the oracle's loops (n > 0). */
void orc_set_threads(int n);

#ifdef __cplusplus
}
#endif

#endif
