/* CPU check of the FP64 oracle under AddressSanitizer and
 * UndefinedBehaviorSanitizer: the oracle source is compiled into this file
 * (serially, without OpenMP) and every entry point runs on small cases that
 * reach its boundary paths: periodic and walled axes, moving walls, the
 * points' supports across periodic seams, every forcing option (residual
 * stop, unweighted inner sweep, warm start from a network and from a
 * previous correction), neighbour lists with empty and full sets, the MLP
 * loss, gradient and Adam step.  Prints OK on success; a sanitizer report
 * makes it fail. */
#include "../../oracle/lbm_ibm_oracle.c"

#include <stdio.h>

static double frand(uint64_t* s) { /* xorshift64*, in [-1, 1) */
  *s ^= *s >> 12;
  *s ^= *s << 25;
  *s ^= *s >> 27;
  return (double)((*s * 2685821657736338717ULL) >> 11) / (double)(1ULL << 52) - 1.0;
}

static int run_case(int nx, int ny, int nz, const int bc[3], int forcing, int flags, int n_iter,
                    int steps, uint64_t seed) {
  orc_params p;
  memset(&p, 0, sizeof(p));
  p.nx = nx; p.ny = ny; p.nz = nz;
  for (int a = 0; a < 3; ++a) p.bc[a] = bc[a];
  p.forcing = forcing;
  p.tau = 0.7;
  p.rho_wall = 1.0;
  p.wall_u[1][1][0] = 0.01;
  p.g_ext[0] = 1e-5;
  const int64_t n = (int64_t)nx * ny * nz;
  double* f = (double*)malloc(sizeof(double) * Q * n);
  const double u0[3] = {0.01, -0.02, 0.005};
  orc_init_equilibrium(&p, 1.0, u0, f);
  /* two small rotating bodies, one empty body between them */
  enum { NP = 40 };
  double rest[NP * 3], area[NP];
  for (int k = 0; k < NP; ++k) {
    rest[3 * k] = 1.5 * frand(&seed);
    rest[3 * k + 1] = 1.5 * frand(&seed);
    rest[3 * k + 2] = 1.5 * frand(&seed);
    area[k] = 0.5 + 0.4 * frand(&seed);
  }
  int64_t body_off[4] = {0, 25, 25, NP};
  orc_body bodies[3];
  for (int b = 0; b < 3; ++b) {
    /* the first body sits on the periodic seams of the axes that have them */
    bodies[b].center[0] = b == 0 && bc[0] == ORC_BC_PERIODIC ? 0.3 : nx / 2.0 + 0.1 * b;
    bodies[b].center[1] = b == 0 && bc[1] == ORC_BC_PERIODIC ? ny - 0.4 : ny / 2.0;
    bodies[b].center[2] = nz / 2.0 - 0.2;
    bodies[b].axis[0] = 0.2 + b;
    bodies[b].axis[1] = -0.3;
    bodies[b].axis[2] = 1.0;
    bodies[b].theta0 = 0.4 * b;
    bodies[b].omega = 0.03 - 0.01 * b;
  }
  double theta[MLP_NPARAM];
  for (int i = 0; i < MLP_NPARAM; ++i) theta[i] = 0.05 * frand(&seed);
  orc_points pts;
  memset(&pts, 0, sizeof(pts));
  pts.npts = NP;
  pts.rest = rest;
  pts.area = area;
  pts.body_off = body_off;
  pts.nbodies = 3;
  pts.n_iter = n_iter;
  pts.flags = flags;
  pts.bodies = bodies;
  pts.eps = 0.2;
  pts.theta = theta;
  double hist[4 * 8];
  int32_t sweeps[8];
  int err = orc_run(&p, f, &pts, 0, steps, hist, sweeps);
  /* one more step with every output */
  double sums[4], *G = (double*)malloc(sizeof(double) * 3 * n);
  double x[NP * 3], ub[NP * 3], g[NP * 3], du[NP * 3], resid[16], feat[NP * 12];
  int32_t ns = 0;
  orc_step_out o = {sums, G, x, ub, g, du, resid, feat, &ns};
  if (err == ORC_OK) err = orc_step(&p, f, &pts, steps, &o);
  for (int i = 0; err == ORC_OK && i < 4; ++i)
    if (!isfinite(sums[i])) err = -100;
  free(G);
  free(f);
  return err;
}

int main(void) {
  const int periodic[3] = {0, 0, 0}, walls_yz[3] = {0, 1, 1}, walls[3] = {1, 1, 1};
  const int flag_sets[5] = {0, ORC_IBM_INNER_UNWEIGHTED, ORC_IBM_STOP_RESIDUAL,
                            ORC_IBM_STOP_RESIDUAL | ORC_IBM_WARM_START,
                            ORC_IBM_STOP_RESIDUAL | ORC_IBM_WARM_PREV};
  int fails = 0;
  for (int fs = 0; fs < 5; ++fs) {
    fails += run_case(9, 8, 10, periodic, ORC_FORCE_GUO, flag_sets[fs], 4, 3, 11 + fs) != ORC_OK;
    fails += run_case(12, 11, 10, walls_yz, ORC_FORCE_SHIFT, flag_sets[fs], 3, 2, 21 + fs) != ORC_OK;
  }
  /* a support crossing a wall is reported, not read out of bounds */
  fails += run_case(4, 4, 4, walls, ORC_FORCE_GUO, 0, 2, 1, 31) != ORC_ERR_DOMAIN;
  /* delta kernel on and around its support ends */
  double acc = 0.0;
  for (int i = -300; i <= 300; ++i) acc += orc_delta(i / 100.0);
  if (!(fabs(acc / 100.0 - 1.0) < 1e-3)) ++fails;
  /* MLP loss, gradient and Adam on a small batch */
  enum { B = 5 };
  uint64_t seed = 99;
  double th[MLP_NPARAM], gr[MLP_NPARAM], m[MLP_NPARAM], v[MLP_NPARAM], xb[B * 12], tb[B * 3], yb[B * 3];
  for (int i = 0; i < MLP_NPARAM; ++i) {
    th[i] = 0.1 * frand(&seed);
    m[i] = v[i] = 0.0;
  }
  for (int i = 0; i < B * 12; ++i) xb[i] = frand(&seed);
  for (int i = 0; i < B * 3; ++i) tb[i] = frand(&seed);
  orc_mlp_forward(th, B, xb, yb);
  const double loss = orc_mlp_loss_grad(th, B, xb, tb, gr);
  orc_adam_step(th, gr, m, v, 1, 1e-3, 0.9, 0.999, 1e-8);
  if (!isfinite(loss)) ++fails;
  if (fails) {
    printf("FAILED %d\n", fails);
    return 1;
  }
  printf("OK\n");
  return 0;
}
