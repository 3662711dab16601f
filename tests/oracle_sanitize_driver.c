/*
 * Driver of the sanitizer check of the FP64 CPU oracle (test infrastructure
 * only): exercises every lattice, both force forms, periodic boxes and every
 * wall combination, the single-site functions and the observables, on boxes
 * whose sides are 1, 2 or 3 layers as well as larger ones, so that every
 * wrap, mirror and bounce-back index of the oracle is taken.  Built with
 * AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_oracle_sanitizers.py; any out-of-bounds access, leak, signed
 * overflow or misaligned access aborts it.  Prints one line per case.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lb_oracle.h"

static int run_case(int lattice, int n, int form, int walls, int64_t nx, int64_t ny, int64_t nz, int steps) {
  orc_params p;
  memset(&p, 0, sizeof(p));
  p.lattice = lattice;
  p.n_comp = n;
  p.force_form = form;
  p.walls = walls;
  p.nx = nx;
  p.ny = ny;
  p.nz = nz;
  p.tau = 0.9;
  p.theta = 0.25;
  p.kappa = 0.02;
  for (int s = 0; s < n; ++s) {
    p.m[s] = (s % 2) ? 1.0 : 2.0;
    for (int t = 0; t < n; ++t) p.chi[s * ORC_MAX_COMP + t] = (s == t) ? 0.0 : 0.8 + 0.1 * (s + t);
  }
  const int64_t S = nx * ny * nz;
  int32_t Q = 0, D = 0;
  if (orc_lattice(lattice, &Q, &D, NULL, NULL)) return 1;
  double* rho0 = (double*)malloc(sizeof(double) * (size_t)(n * S));
  for (int64_t k = 0; k < n * S; ++k) rho0[k] = 0.4 + 0.05 * sin(0.7 * (double)k + 0.3);
  orc_state* st = orc_create(&p, rho0);
  if (!st) return 2;
  orc_step(st, steps);
  const int nP = D * (D + 1) / 2;
  double* rho = (double*)malloc(sizeof(double) * (size_t)(n * S));
  double* U = (double*)malloc(sizeof(double) * (size_t)(D * S));
  double* mu = (double*)malloc(sizeof(double) * (size_t)(n * S));
  double* P = (double*)malloc(sizeof(double) * (size_t)(nP * S));
  double* A = (double*)malloc(sizeof(double) * (size_t)(n * D * S));
  double* f = (double*)malloc(sizeof(double) * (size_t)(n * Q * S));
  double mass[ORC_MAX_COMP], mom[3];
  orc_observe(st, rho, U, mu, P, A, mass, mom);
  orc_get_f(st, f);
  orc_set_f(st, f);
  orc_step(st, 1);
  orc_observe(st, NULL, NULL, NULL, NULL, NULL, mass, mom);
  double m0 = 0.0, m1 = 0.0;
  for (int64_t k = 0; k < n * S; ++k) m0 += rho0[k];
  for (int s = 0; s < n; ++s) m1 += mass[s];
  printf("lattice %d N=%d form %d walls %d box %lldx%lldx%lld: t=%lld mass %.17g -> %.17g\n", lattice, n, form,
         walls, (long long)nx, (long long)ny, (long long)nz, (long long)orc_time(st), m0, m1);
  const int bad = !(fabs(m1 / m0 - 1.0) < 1e-12);
  orc_destroy(st);
  free(rho0); free(rho); free(U); free(mu); free(P); free(A); free(f);
  return bad ? 3 : 0;
}

int main(void) {
  /* single-site pieces */
  double u[3] = {0.01, -0.02, 0.005}, A[3] = {1e-3, 2e-3, -1e-3}, out[19];
  for (int lat = ORC_D1Q3; lat <= ORC_D3Q19; ++lat) {
    orc_feq(lat, 0.7, u, out);
    orc_forcing(lat, A, u, out);
  }
  int rc = 0;
  for (int form = 0; form < 2; ++form) {
    rc |= run_case(ORC_D1Q3, 3, form, 0, 7, 1, 1, 5);
    rc |= run_case(ORC_D1Q3, 2, form, 1, 2, 1, 1, 5);
    rc |= run_case(ORC_D1Q3, 1, form, 0, 1, 1, 1, 3);
    for (int walls = 0; walls < 4; ++walls) {
      rc |= run_case(ORC_D2Q9, 3, form, walls, 5, 4, 1, 4);
      rc |= run_case(ORC_D2Q9, 2, form, walls, 2, 3, 1, 3);
    }
    rc |= run_case(ORC_D2Q9, 8, form, 0, 3, 2, 1, 2);
    for (int walls = 0; walls < 8; ++walls) rc |= run_case(ORC_D3Q19, 2, form, walls, 3, 4, 2, 3);
    rc |= run_case(ORC_D3Q19, 3, form, 0, 1, 1, 1, 2);
  }
  printf("rc %d\n", rc);
  return rc;
}
