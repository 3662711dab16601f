/*
 * lb_oracle.h -- plain FP64 CPU oracle for the symmetric free-energy
 * multicomponent lattice Boltzmann method of Li & Wagner,
 * "A Symmetric Free Energy Based Multi-Component Lattice Boltzmann Method"
 * (arXiv:0704.3444).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against the paper.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load it.  It shares no source, header, table
 * or helper with the GPU library, and neither includes the other.
 *
 * Conventions (lattice units, dt = dx = 1, c_s^2 = 1/3):
 *   site index  s = x + nx*(y + ny*z)
 *   populations f[sigma][i][s]  (component-major structure of arrays)
 *   the state holds the post-streaming populations f_i(r, t).
 */
#ifndef LB_ORACLE_H
#define LB_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_COMP 8

enum { ORC_D1Q3 = 1, ORC_D2Q9 = 2, ORC_D3Q19 = 3 };
enum { ORC_FORCE_EXPANDED = 0, ORC_FORCE_LOG = 1 };

typedef struct {
  int32_t lattice;     /* ORC_D1Q3, ORC_D2Q9 or ORC_D3Q19                     */
  int32_t n_comp;      /* 1 .. ORC_MAX_COMP                                    */
  int32_t force_form;  /* ORC_FORCE_EXPANDED (default) or ORC_FORCE_LOG        */
  int32_t walls;       /* bit a set: axis a (0 x, 1 y, 2 z) is closed by walls
                          half a site beyond its first and last layers (not in
                          the paper; see orc_step); 0: periodic               */
  int64_t nx, ny, nz;  /* box; unused axes are 1                               */
  double tau;          /* BGK relaxation time, common to all components        */
  double theta;        /* temperature of the Flory-Huggins free energy         */
  double kappa;        /* square-gradient coefficient                          */
  double m[ORC_MAX_COMP];                  /* polymerisation m^sigma           */
  double chi[ORC_MAX_COMP * ORC_MAX_COMP]; /* chi^{sigma sigma'}, row-major,
                                              leading dimension ORC_MAX_COMP  */
} orc_params;

typedef struct orc_state orc_state;

/* Lattice tables: Q, D, velocities v[Q][3] (int), weights w[Q]. */
int orc_lattice(int32_t lattice, int32_t* Q, int32_t* D, int32_t* v, double* w);

/* Single-site pieces, exposed so that tests can check them one by one. */
void orc_feq(int32_t lattice, double rho, const double u[3], double* out);
void orc_forcing(int32_t lattice, const double A[3], const double usig[3], double* out);
/* Per-mer chemical potentials mu^sigma at one site from the component
 * densities rho[N] and the Laplacians lap[N] of rho^sigma. */
void orc_mu_site(const orc_params* p, const double* rho, const double* lap, double* mu);
/* Bulk Flory-Huggins free-energy density psi at one site. */
double orc_psi_site(const orc_params* p, const double* rho);

/* Whole-lattice state. */
orc_state* orc_create(const orc_params* p, const double* rho0 /* [N][S] */);
void orc_destroy(orc_state* st);
/* nsteps time steps.  With walls (the paper's boxes are periodic; walls are
 * this library's own addition): a population that would stream across a
 * wall returns to its site with the opposite velocity (half-way
 * bounce-back: no slip, every component's mass kept), and the gradient and
 * Laplacian stencils take the layer next to a wall as its own mirror image
 * beyond it (zero normal gradient: a wall that favours no component). */
void orc_step(orc_state* st, int64_t nsteps);
int64_t orc_time(const orc_state* st);
void orc_get_f(const orc_state* st, double* f /* [N][Q][S] */);
void orc_set_f(orc_state* st, const double* f /* [N][Q][S] */);
/* Observables at the current time.  Every pointer may be NULL.
 *   rho[N][S], U[D][S] (macroscopic velocity u + A/(2 rho)), mu[N][S],
 *   P[D*(D+1)/2][S] (pressure tensor: xx, xy, (xz), yy, (yz), (zz)),
 *   A[N][D][S] (force density rho^sigma a^sigma), mass[N], mom[D] (sum of
 *   the raw first moments over sites and components). */
void orc_observe(orc_state* st, double* rho, double* U, double* mu, double* P,
                 double* A, double* mass, double* mom);

#ifdef __cplusplus
}
#endif
#endif
