/*
 * lb_oracle.c -- plain FP64 CPU oracle for the symmetric free-energy
 * multicomponent lattice Boltzmann method (Li & Wagner, arXiv:0704.3444).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the GPU library.  It is written
 * for a reader holding the paper: each function names the section and
 * equation it follows, and the loops go site by site in the order the
 * method states, with no blocking or fusion.  Compiled with
 * -ffp-contract=off so that every operation rounds as written.
 *
 * One time step (Sec. III), for every site r and component sigma:
 *   1. rho^sigma = sum_i f_i^sigma                      (moments, Sec. III)
 *   2. mu^sigma from the Flory-Huggins free energy, Eq. (lgf), taken per mer
 *      and with a square-gradient term -kappa lap rho^sigma      (Sec. IV)
 *   3. j^sigma = sum_i f_i^sigma v_i, rho = sum rho^sigma,
 *      u = sum j^sigma / rho, u^sigma = j^sigma / rho^sigma     (Sec. III)
 *   4. force rho^sigma a^sigma from Eq. (definef)
 *   5. f^{sigma e}_i with the equilibrium moments of Sec. III, and F^sigma_i
 *      with the forcing moments Eqs. (ff1)-(ff3)
 *   6. BGK collision and streaming, Eq. (ssLB)
 *
 * Readings of points the paper leaves open (gradient stencils, the third
 * moments whose indices are garbled in the text, the kappa term, per-mer
 * chemical potentials) are the ones listed in the design notes; each is
 * repeated below where it is used.
 */
#include "lb_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------- */
/* Lattices.  D1Q3 is the paper's (Sec. IV); D2Q9 and D3Q19 are the usual  */
/* second-order sets with sum w v v = delta / 3.                           */
/* ---------------------------------------------------------------------- */

static const int D1Q3_V[3][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}};
static const double D1Q3_W[3] = {2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0};

static const int D2Q9_V[9][3] = {{0, 0, 0},  {1, 0, 0},  {0, 1, 0},
                                 {-1, 0, 0}, {0, -1, 0}, {1, 1, 0},
                                 {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
static const double D2Q9_W[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                                  1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                                  1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

static const int D3Q19_V[19][3] = {
    {0, 0, 0},   {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},  {0, -1, 0},
    {0, 0, 1},   {0, 0, -1},  {1, 1, 0},   {-1, -1, 0}, {1, -1, 0},
    {-1, 1, 0},  {1, 0, 1},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},   {0, -1, -1}, {0, 1, -1},  {0, -1, 1}};
static const double D3Q19_W[19] = {
    1.0 / 3.0,  1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
    1.0 / 18.0, 1.0 / 18.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

typedef struct {
  int Q, D;
  const int (*v)[3];
  const double* w;
} lattice_t;

static int get_lattice(int32_t lattice, lattice_t* L) {
  switch (lattice) {
    case ORC_D1Q3: L->Q = 3; L->D = 1; L->v = D1Q3_V; L->w = D1Q3_W; return 0;
    case ORC_D2Q9: L->Q = 9; L->D = 2; L->v = D2Q9_V; L->w = D2Q9_W; return 0;
    case ORC_D3Q19: L->Q = 19; L->D = 3; L->v = D3Q19_V; L->w = D3Q19_W; return 0;
    default: return -1;
  }
}

int orc_lattice(int32_t lattice, int32_t* Q, int32_t* D, int32_t* v, double* w) {
  lattice_t L;
  if (get_lattice(lattice, &L)) return -1;
  if (Q) *Q = L.Q;
  if (D) *D = L.D;
  for (int i = 0; i < L.Q; ++i) {
    if (v) for (int a = 0; a < 3; ++a) v[3 * i + a] = L.v[i][a];
    if (w) w[i] = L.w[i];
  }
  return 0;
}

/* ---------------------------------------------------------------------- */
/* Equilibrium and forcing populations at one site.                        */
/* ---------------------------------------------------------------------- */

/* f^e_i = w_i rho [1 + 3 v.u + (9/2)(v.u)^2 - (3/2) u.u].  Its moments are
 * the equilibrium moments of Sec. III: rho, rho u, rho/3 delta + rho u u,
 * and the symmetric third moment (rho/3)(u_a d_bc + u_b d_ac + u_c d_ab). */
void orc_feq(int32_t lattice, double rho, const double u[3], double* out) {
  lattice_t L;
  if (get_lattice(lattice, &L)) return;
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < L.Q; ++i) {
    double vu = L.v[i][0] * u[0] + L.v[i][1] * u[1] + L.v[i][2] * u[2];
    out[i] = L.w[i] * rho * (1.0 + 3.0 * vu + 4.5 * vu * vu - 1.5 * uu);
  }
}

/* F_i = w_i [3 v.A + 9 (v.A)(v.u^s) - 3 A.u^s] with A = rho^s a^s.  Its
 * moments are those of Eqs. (ff1)-(ff3): 0, A, A u^s + u^s A, and the
 * symmetric third moment (1/3)(A_a d_bc + A_b d_ac + A_c d_ab). */
void orc_forcing(int32_t lattice, const double A[3], const double us[3], double* out) {
  lattice_t L;
  if (get_lattice(lattice, &L)) return;
  double Au = A[0] * us[0] + A[1] * us[1] + A[2] * us[2];
  for (int i = 0; i < L.Q; ++i) {
    double vA = L.v[i][0] * A[0] + L.v[i][1] * A[1] + L.v[i][2] * A[2];
    double vu = L.v[i][0] * us[0] + L.v[i][1] * us[1] + L.v[i][2] * us[2];
    out[i] = L.w[i] * (3.0 * vA + 9.0 * vA * vu - 3.0 * Au);
  }
}

/* ---------------------------------------------------------------------- */
/* Thermodynamics, Sec. IV, Eq. (lgf).                                    */
/* ---------------------------------------------------------------------- */

/* Free-energy density of Eq. (lgf) in terms of mer densities rho^s = m^s n^s
 * and volume fractions phi^s = rho^s / rho:
 *   psi = theta sum_s n^s (ln phi^s - m^s)
 *       + (theta/2) sum_{s,t} chi^{st} rho^s phi^t. */
double orc_psi_site(const orc_params* p, const double* rho) {
  const int N = p->n_comp;
  double rt = 0.0;
  for (int s = 0; s < N; ++s) rt += rho[s];
  double psi = 0.0;
  for (int s = 0; s < N; ++s) {
    double n = rho[s] / p->m[s];
    double phi = rho[s] / rt;
    psi += p->theta * n * (log(phi) - p->m[s]);
  }
  for (int s = 0; s < N; ++s)
    for (int t = 0; t < N; ++t)
      psi += 0.5 * p->theta * p->chi[s * ORC_MAX_COMP + t] * rho[s] * (rho[t] / rt);
  return psi;
}

/* Chemical potential per mer, mu^s = (1/m^s) d psi / d n^s (Eq.
 * (chemicalpotential) divided by the polymerisation, so that rho^s grad mu^s
 * equals n^s grad of the per-molecule potential), with chi symmetric:
 *   mu^s = theta [ -1 + (1 + ln phi^s)/m^s - sum_t phi^t/m^t
 *                 + sum_t chi^{st} phi^t - (1/2) sum_{t,t'} chi^{tt'} phi^t phi^t' ]
 *          - kappa lap rho^s
 * The last term is the functional derivative of a square-gradient term
 * sum_s (kappa/2)|grad rho^s|^2, the reading used for the paper's kappa. */
void orc_mu_site(const orc_params* p, const double* rho, const double* lap, double* mu) {
  const int N = p->n_comp;
  double phi[ORC_MAX_COMP];
  double rt = 0.0;
  for (int s = 0; s < N; ++s) rt += rho[s];
  for (int s = 0; s < N; ++s) phi[s] = rho[s] / rt;
  double sum_phi_m = 0.0;
  for (int t = 0; t < N; ++t) sum_phi_m += phi[t] / p->m[t];
  double quad = 0.0;
  for (int t = 0; t < N; ++t)
    for (int t2 = 0; t2 < N; ++t2)
      quad += p->chi[t * ORC_MAX_COMP + t2] * phi[t] * phi[t2];
  for (int s = 0; s < N; ++s) {
    double lin = 0.0;
    for (int t = 0; t < N; ++t) lin += p->chi[s * ORC_MAX_COMP + t] * phi[t];
    double bulk = -1.0 + (1.0 + log(phi[s])) / p->m[s] - sum_phi_m + lin - 0.5 * quad;
    mu[s] = p->theta * bulk - p->kappa * (lap ? lap[s] : 0.0);
  }
}

/* ---------------------------------------------------------------------- */
/* Whole lattice.                                                          */
/* ---------------------------------------------------------------------- */

struct orc_state {
  orc_params p;
  lattice_t L;
  int64_t S;
  int64_t t;
  double* f;     /* [N][Q][S] post-streaming populations        */
  double* fnew;  /* [N][Q][S] streaming target                  */
  double* rho;   /* [N][S]                                      */
  double* lap;   /* [N][S] Laplacian of rho^sigma               */
  double* mu;    /* [N][S]                                      */
};

/* Coordinate c + d (|d| <= 1) along an axis of n layers: periodic, or, on
 * an axis closed by walls, the mirror image of the layer next to the wall
 * when c + d lies beyond it (a zero normal gradient of the field at the
 * wall). */
static int64_t axis_step(int64_t c, int d, int64_t n, int wall) {
  int64_t y = c + d;
  if (wall) return y < 0 ? -1 - y : (y >= n ? 2 * n - 1 - y : y);
  return (y % n + n) % n;
}

/* Site r + sign * v for the gradient and Laplacian stencils. */
static int64_t neighbour(const orc_state* st, int64_t s, const int v[3], int sign) {
  const int64_t nx = st->p.nx, ny = st->p.ny, nz = st->p.nz;
  const int w = st->p.walls;
  int64_t x = s % nx, y = (s / nx) % ny, z = s / (nx * ny);
  x = axis_step(x, sign * v[0], nx, w & 1);
  y = axis_step(y, sign * v[1], ny, w & 2);
  z = axis_step(z, sign * v[2], nz, w & 4);
  return x + nx * (y + ny * z);
}

/* Site that a population leaving s with velocity v reaches in one step, or
 * -1 if it meets a wall on the way (half-way bounce-back: it then returns to
 * s with velocity -v). */
static int64_t stream_target(const orc_state* st, int64_t s, const int v[3]) {
  const int64_t n[3] = {st->p.nx, st->p.ny, st->p.nz};
  int64_t c[3] = {s % n[0], (s / n[0]) % n[1], s / (n[0] * n[1])};
  for (int a = 0; a < 3; ++a) {
    int64_t y = c[a] + v[a];
    if ((st->p.walls >> a) & 1) {
      if (y < 0 || y >= n[a]) return -1;
    } else {
      y = (y % n[a] + n[a]) % n[a];
    }
    c[a] = y;
  }
  return c[0] + n[0] * (c[1] + n[1] * c[2]);
}

/* Index of the velocity -v_i. */
static int opposite(const lattice_t* L, int i) {
  for (int j = 0; j < L->Q; ++j)
    if (L->v[j][0] == -L->v[i][0] && L->v[j][1] == -L->v[i][1] && L->v[j][2] == -L->v[i][2]) return j;
  return -1;
}

#define F(arr, sg, i, s) (arr)[(((int64_t)(sg) * st->L.Q + (i)) * st->S) + (s)]
#define FLD(arr, sg, s) (arr)[((int64_t)(sg) * st->S) + (s)]

orc_state* orc_create(const orc_params* p, const double* rho0) {
  orc_state* st = (orc_state*)calloc(1, sizeof(orc_state));
  if (!st) return NULL;
  st->p = *p;
  if (get_lattice(p->lattice, &st->L) || p->n_comp < 1 || p->n_comp > ORC_MAX_COMP) {
    free(st);
    return NULL;
  }
  st->S = p->nx * p->ny * p->nz;
  const int N = p->n_comp, Q = st->L.Q;
  size_t nf = (size_t)N * Q * st->S, nr = (size_t)N * st->S;
  st->f = (double*)malloc(nf * sizeof(double));
  st->fnew = (double*)malloc(nf * sizeof(double));
  st->rho = (double*)malloc(nr * sizeof(double));
  st->lap = (double*)malloc(nr * sizeof(double));
  st->mu = (double*)malloc(nr * sizeof(double));
  if (!st->f || !st->fnew || !st->rho || !st->lap || !st->mu) {
    orc_destroy(st);
    return NULL;
  }
  /* Initial state: rest equilibrium f_i = w_i rho0 (the paper starts from
   * prescribed volume fractions at rest). */
  for (int sg = 0; sg < N; ++sg)
    for (int i = 0; i < Q; ++i)
      for (int64_t s = 0; s < st->S; ++s)
        F(st->f, sg, i, s) = st->L.w[i] * rho0[(int64_t)sg * st->S + s];
  return st;
}

void orc_destroy(orc_state* st) {
  if (!st) return;
  free(st->f);
  free(st->fnew);
  free(st->rho);
  free(st->lap);
  free(st->mu);
  free(st);
}

int64_t orc_time(const orc_state* st) { return st->t; }

void orc_get_f(const orc_state* st, double* f) {
  memcpy(f, st->f, sizeof(double) * (size_t)st->p.n_comp * st->L.Q * st->S);
}

void orc_set_f(orc_state* st, const double* f) {
  memcpy(st->f, f, sizeof(double) * (size_t)st->p.n_comp * st->L.Q * st->S);
}

/* Step 1: component densities rho^sigma = sum_i f_i^sigma. */
static void pass_density(orc_state* st) {
  const int N = st->p.n_comp, Q = st->L.Q;
#pragma omp parallel for schedule(static) if (st->S >= 16384)
  for (int64_t s = 0; s < st->S; ++s)
    for (int sg = 0; sg < N; ++sg) {
      double r = 0.0;
      for (int i = 0; i < Q; ++i) r += F(st->f, sg, i, s);
      FLD(st->rho, sg, s) = r;
    }
}

/* Isotropic lattice Laplacian: lap g(r) = 6 sum_i w_i [g(r + v_i) - g(r)]. */
static double lattice_laplacian(const orc_state* st, const double* g, int64_t s) {
  double acc = 0.0;
  for (int i = 0; i < st->L.Q; ++i)
    acc += st->L.w[i] * (g[neighbour(st, s, st->L.v[i], +1)] - g[s]);
  return 6.0 * acc;
}

/* Isotropic lattice gradient: grad g(r) = 3 sum_i w_i v_i g(r + v_i). */
static void lattice_gradient(const orc_state* st, const double* g, int64_t s, double out[3]) {
  out[0] = out[1] = out[2] = 0.0;
  for (int i = 0; i < st->L.Q; ++i) {
    double gi = g[neighbour(st, s, st->L.v[i], +1)];
    for (int a = 0; a < 3; ++a) out[a] += st->L.w[i] * st->L.v[i][a] * gi;
  }
  for (int a = 0; a < 3; ++a) out[a] *= 3.0;
}

/* Step 2: chemical potentials from the densities. */
static void pass_mu(orc_state* st) {
  const int N = st->p.n_comp;
#pragma omp parallel for schedule(static) if (st->S >= 16384)
  for (int64_t s = 0; s < st->S; ++s)
    for (int sg = 0; sg < N; ++sg)
      FLD(st->lap, sg, s) = lattice_laplacian(st, &FLD(st->rho, sg, 0), s);
#pragma omp parallel for schedule(static) if (st->S >= 16384)
  for (int64_t s = 0; s < st->S; ++s) {
    double rho[ORC_MAX_COMP], lap[ORC_MAX_COMP], mu[ORC_MAX_COMP];
    for (int sg = 0; sg < N; ++sg) {
      rho[sg] = FLD(st->rho, sg, s);
      lap[sg] = FLD(st->lap, sg, s);
    }
    orc_mu_site(&st->p, rho, lap, mu);
    for (int sg = 0; sg < N; ++sg) FLD(st->mu, sg, s) = mu[sg];
  }
}

/* Force density rho^s a^s of Eq. (definef), with c = w/tau = 1 - 1/(2 tau):
 *   expanded form (second line):  A = -c [rho^s grad mu^s - (1/3) grad rho^s]
 *   log form (first line):        A = -c rho^s grad (mu^s - (1/3) ln rho^s)  */
static void site_force(const orc_state* st, int sg, int64_t s, double A[3]) {
  const double c = 1.0 - 0.5 / st->p.tau;
  const double* rho = &FLD(st->rho, sg, 0);
  const double* mu = &FLD(st->mu, sg, 0);
  if (st->p.force_form == ORC_FORCE_LOG) {
    double g[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < st->L.Q; ++i) {
      int64_t n = neighbour(st, s, st->L.v[i], +1);
      double h = mu[n] - log(rho[n]) / 3.0;
      for (int a = 0; a < 3; ++a) g[a] += st->L.w[i] * st->L.v[i][a] * h;
    }
    for (int a = 0; a < 3; ++a) A[a] = -c * rho[s] * (3.0 * g[a]);
  } else {
    double gmu[3], grho[3];
    lattice_gradient(st, mu, s, gmu);
    lattice_gradient(st, rho, s, grho);
    for (int a = 0; a < 3; ++a) A[a] = -c * (rho[s] * gmu[a] - grho[a] / 3.0);
  }
}

/* First moments at a site: j^sigma and the barycentric velocity u. */
static void site_velocities(const orc_state* st, int64_t s, double j[][3], double u[3]) {
  const int N = st->p.n_comp;
  double rt = 0.0;
  u[0] = u[1] = u[2] = 0.0;
  for (int sg = 0; sg < N; ++sg) {
    j[sg][0] = j[sg][1] = j[sg][2] = 0.0;
    for (int i = 0; i < st->L.Q; ++i)
      for (int a = 0; a < 3; ++a) j[sg][a] += F(st->f, sg, i, s) * st->L.v[i][a];
    rt += FLD(st->rho, sg, s);
  }
  for (int a = 0; a < 3; ++a) {
    double acc = 0.0;
    for (int sg = 0; sg < N; ++sg) acc += j[sg][a];
    u[a] = acc / rt;
  }
}

/* Steps 3-6: collision and streaming, Eq. (ssLB). */
static void pass_collide_stream(orc_state* st) {
  const int N = st->p.n_comp, Q = st->L.Q;
  const double inv_tau = 1.0 / st->p.tau;
#pragma omp parallel for schedule(static) if (st->S >= 16384)
  for (int64_t s = 0; s < st->S; ++s) {
    double j[ORC_MAX_COMP][3], u[3];
    site_velocities(st, s, j, u);
    for (int sg = 0; sg < N; ++sg) {
      double rs = FLD(st->rho, sg, s);
      double us[3] = {j[sg][0] / rs, j[sg][1] / rs, j[sg][2] / rs};
      double A[3], feq[19], Fi[19];
      site_force(st, sg, s, A);
      orc_feq(st->p.lattice, rs, u, feq);
      orc_forcing(st->p.lattice, A, us, Fi);
      for (int i = 0; i < Q; ++i) {
        double fs = F(st->f, sg, i, s);
        double post = fs + inv_tau * (feq[i] - fs) + Fi[i];
        const int64_t d = stream_target(st, s, st->L.v[i]);
        if (d >= 0)
          F(st->fnew, sg, i, d) = post;
        else
          F(st->fnew, sg, opposite(&st->L, i), s) = post;  /* bounced at a wall */
      }
    }
  }
  double* tmp = st->f;
  st->f = st->fnew;
  st->fnew = tmp;
}

void orc_step(orc_state* st, int64_t nsteps) {
  for (int64_t n = 0; n < nsteps; ++n) {
    pass_density(st);
    pass_mu(st);
    pass_collide_stream(st);
    st->t += 1;
  }
}

/* Observables.  U = u + (1/2) sum_sigma A^sigma / rho is the macroscopic
 * velocity of Sec. III (U = u + a dt/2).  The pressure tensor is the one of
 * the free energy with the square-gradient term:
 *   P_ab = [p0 - kappa sum_s (rho^s lap rho^s + |grad rho^s|^2 / 2)] d_ab
 *        + kappa sum_s d_a rho^s d_b rho^s,
 * with the bulk pressure p0 = sum_s rho^s mu0^s - psi of Eq. (ppp) (mu0 the
 * per-mer potential without the gradient term).  It is a diagnostic; the
 * update never uses it. */
void orc_observe(orc_state* st, double* rho_out, double* U, double* mu_out, double* P,
                 double* A_out, double* mass, double* mom) {
  const int N = st->p.n_comp, D = st->L.D;
  const int64_t S = st->S;
  pass_density(st);
  pass_mu(st);
  if (rho_out) memcpy(rho_out, st->rho, sizeof(double) * N * S);
  if (mu_out) memcpy(mu_out, st->mu, sizeof(double) * N * S);
  if (U || A_out) {
    for (int64_t s = 0; s < S; ++s) {
      double j[ORC_MAX_COMP][3], u[3], rt = 0.0, asum[3] = {0.0, 0.0, 0.0};
      site_velocities(st, s, j, u);
      for (int sg = 0; sg < N; ++sg) {
        double A[3];
        site_force(st, sg, s, A);
        rt += FLD(st->rho, sg, s);
        for (int a = 0; a < 3; ++a) asum[a] += A[a];
        if (A_out)
          for (int a = 0; a < D; ++a) A_out[((int64_t)sg * D + a) * S + s] = A[a];
      }
      if (U)
        for (int a = 0; a < D; ++a) U[(int64_t)a * S + s] = u[a] + 0.5 * asum[a] / rt;
    }
  }
  if (P) {
    orc_params p0 = st->p;
    p0.kappa = 0.0;
    for (int64_t s = 0; s < S; ++s) {
      double rho[ORC_MAX_COMP], mu0[ORC_MAX_COMP], g[ORC_MAX_COMP][3];
      for (int sg = 0; sg < N; ++sg) rho[sg] = FLD(st->rho, sg, s);
      orc_mu_site(&p0, rho, NULL, mu0);
      double pb = -orc_psi_site(&p0, rho);
      double iso = 0.0;
      for (int sg = 0; sg < N; ++sg) {
        pb += rho[sg] * mu0[sg];
        lattice_gradient(st, &FLD(st->rho, sg, 0), s, g[sg]);
        double g2 = g[sg][0] * g[sg][0] + g[sg][1] * g[sg][1] + g[sg][2] * g[sg][2];
        iso += rho[sg] * FLD(st->lap, sg, s) + 0.5 * g2;
      }
      int k = 0;
      for (int a = 0; a < D; ++a)
        for (int b = a; b < D; ++b) {
          double grad = 0.0;
          for (int sg = 0; sg < N; ++sg) grad += g[sg][a] * g[sg][b];
          double val = st->p.kappa * grad;
          if (a == b) val += pb - st->p.kappa * iso;
          P[(int64_t)k * S + s] = val;
          ++k;
        }
    }
  }
  if (mass)
    for (int sg = 0; sg < N; ++sg) {
      double acc = 0.0;
      for (int64_t s = 0; s < S; ++s) acc += FLD(st->rho, sg, s);
      mass[sg] = acc;
    }
  if (mom) {
    for (int a = 0; a < D; ++a) mom[a] = 0.0;
    for (int64_t s = 0; s < S; ++s) {
      double j[ORC_MAX_COMP][3], u[3];
      site_velocities(st, s, j, u);
      for (int sg = 0; sg < N; ++sg)
        for (int a = 0; a < D; ++a) mom[a] += j[sg][a];
    }
  }
}
