/*
 * FP64 CPU oracle for the LBM-IBM method of Beny & Latt, "Efficient LBM on
 * GPUs for dense moving objects using immersed boundary condition"
 * (arXiv 1904.02108).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code, header or table with the HIP
 * library: every constant below is written out here on its own.
 *
 * Plain, slow, obviously correct: double precision everywhere, one loop per
 * definition, no blocking or fusion beyond what the paper's step list states.
 *
 * Readings of the paper taken here (each is listed with its reason in the
 * design notes of the repository):
 *   - eq. (3) printed without a density factor; the step list evaluates the
 *     equilibrium with rho, so Eq_i = rho t_i [ ... ] (mass must be conserved).
 *   - Peskin's 4-point kernel, §3: the square root of the outer branch reads
 *     sqrt(-7 + 12|r| - 4 r^2) (the only reading continuous at |r| = 1, 2).
 *   - Delta-u accumulates s(k) g(k) from the first iteration on, as the text
 *     of §3 states (Algorithm 1's reset at the first iteration is read as the
 *     per-time-step reset of the accumulator).
 *   - The final spread of §3 / Algorithm 2 accumulates into G.
 *   - Inner spread: s(k) g(k) by default ("consistent" weighting); the
 *     paper-literal unweighted g(k) is selected with ORC_IBM_INNER_UNWEIGHTED.
 *   - Point velocity by finite difference of positions (Algorithm 1):
 *     u_b(n) = x(n) - x(n-1), theta_n = theta0 + omega n.
 *   - Forcing: the paper's velocity shift U^G = U + tau G (§2, step 3), or
 *     Guo's scheme with F = rho G.
 *   - Walls: halfway bounce-back (walls half a cell outside the first and last
 *     cell); a moving wall adds 6 t_i rho_w (e_i . u_w) to the reflected
 *     population (Ladd).  Where a link leaves the box through several walls at
 *     once, the wall of the lowest axis index (x, then y, then z) supplies u_w.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Number of OpenMP threads of the oracle's parallel loops (timing only: the
 * results do not depend on it beyond the order of FP64 atomic additions in
 * the spread).  Returns the number in effect. */
int orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

#define Q 19

/* ---------------------------------------------------------------------------
 * D3Q19 velocity set (§2: 19 populations per cell, vectors e_i linking a cell
 * to its neighbours).  Order: rest; the 6 axis links as (+,-) pairs along
 * x, y, z; the 12 diagonal links as (+,-) pairs in the xy, xz, yz planes.
 * ------------------------------------------------------------------------- */
static const int C[Q][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

/* Lattice weights t_i (§2; the paper refers to the standard D3Q19 values). */
static double weight(int i) {
  if (i == 0) return 1.0 / 3.0;
  if (i <= 6) return 1.0 / 18.0;
  return 1.0 / 36.0;
}

/* Index of the direction opposite to i, found by search (no table). */
static int opposite(int i) {
  for (int j = 0; j < Q; ++j)
    if (C[j][0] == -C[i][0] && C[j][1] == -C[i][1] && C[j][2] == -C[i][2])
      return j;
  return -1;
}

enum { ORC_BC_PERIODIC = 0, ORC_BC_BOUNCEBACK = 1 };
enum { ORC_FORCE_GUO = 0, ORC_FORCE_SHIFT = 1 };
enum {
  ORC_IBM_INNER_UNWEIGHTED = 1,
  ORC_IBM_STOP_RESIDUAL = 2, /* stop once sum s|g|^2 <= eps^2 sum s|u_b|^2 */
  ORC_IBM_WARM_START = 4,    /* learned warm start after the first sweep  */
  ORC_IBM_WARM_PREV = 32     /* warm start from the previous step's du    */
};
enum { ORC_OK = 0, ORC_ERR_DOMAIN = -5 };

typedef struct {
  int32_t nx, ny, nz;
  int32_t bc[3];          /* per axis: periodic or bounce-back on both faces */
  int32_t forcing;        /* ORC_FORCE_GUO or ORC_FORCE_SHIFT */
  int32_t pad_;
  double tau;             /* BGK relaxation time */
  double rho_wall;        /* density used in the moving-wall correction */
  double wall_u[3][2][3]; /* [axis][low face, high face][component] */
  double g_ext[3];        /* uniform acceleration added to G in every cell */
} orc_params;

typedef struct {
  double center[3];
  double axis[3];
  double theta0;
  double omega;
} orc_body;

static int64_t ncells(const orc_params* p) {
  return (int64_t)p->nx * p->ny * p->nz;
}

static int64_t cell_index(const orc_params* p, int x, int y, int z) {
  return (int64_t)x + (int64_t)p->nx * ((int64_t)y + (int64_t)p->ny * z);
}

/* Tables for the pin tests. */
void orc_d3q19(int32_t* e, double* w, int32_t* opp) {
  for (int i = 0; i < Q; ++i) {
    for (int a = 0; a < 3; ++a) e[3 * i + a] = C[i][a];
    w[i] = weight(i);
    opp[i] = opposite(i);
  }
}

/* ---------------------------------------------------------------------------
 * Equilibrium, eq. (3), with the density factor (see header):
 *   Eq_i = rho t_i [1 + 3 e_i.u + 9/2 (e_i.u)^2 - 3/2 u.u]
 * ------------------------------------------------------------------------- */
void orc_equilibrium(double rho, const double u[3], double eq[Q]) {
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < Q; ++i) {
    double eu = C[i][0] * u[0] + C[i][1] * u[1] + C[i][2] * u[2];
    eq[i] = rho * weight(i) * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
  }
}

/* Moments of one cell, eq. (1): rho = sum f_i, U = (1/rho) sum e_i f_i. */
static void cell_moments(const double* f, int64_t n, int64_t c, double* rho,
                         double U[3]) {
  double r = 0.0, m[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < Q; ++i) {
    double fi = f[(int64_t)i * n + c];
    r += fi;
    for (int a = 0; a < 3; ++a) m[a] += C[i][a] * fi;
  }
  *rho = r;
  for (int a = 0; a < 3; ++a) U[a] = m[a] / r;
}

/* Density and velocity on every cell (§2, step 1).
 * f: [19][ncell], rho: [ncell], U: [3][ncell]. */
void orc_moments(const orc_params* p, const double* f, double* rho, double* U) {
  int64_t n = ncells(p);
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < n; ++c) {
    double r, u[3];
    cell_moments(f, n, c, &r, u);
    rho[c] = r;
    for (int a = 0; a < 3; ++a) U[(int64_t)a * n + c] = u[a];
  }
}

/* Uniform equilibrium state Eq(rho0, u0) in every cell. */
void orc_init_equilibrium(const orc_params* p, double rho0, const double u0[3],
                          double* f) {
  int64_t n = ncells(p);
  double eq[Q];
  orc_equilibrium(rho0, u0, eq);
  for (int i = 0; i < Q; ++i)
    for (int64_t c = 0; c < n; ++c) f[(int64_t)i * n + c] = eq[i];
}

/* ---------------------------------------------------------------------------
 * Collision with forcing (§2, steps 3-5; eq. (2)) followed by streaming
 * (§2, step 6; eq. (4)), written as a push: the post-collision population
 * f*_i at X travels to X + e_i.  On a bounce-back axis a population whose
 * destination lies outside the box returns to X in the opposite direction.
 *
 * f: post-stream populations at time t, [19][ncell].
 * G: force field [3][ncell] (acceleration; NULL = zero); g_ext is added.
 * f_out: post-stream populations at time t+1.
 * ------------------------------------------------------------------------- */
void orc_collide_stream(const orc_params* p, const double* f, const double* G,
                        double* f_out) {
  const int64_t n = ncells(p);
  const int nx = p->nx, ny = p->ny, nz = p->nz;
  const int dims[3] = {nx, ny, nz};
  const double tau = p->tau;
#pragma omp parallel for collapse(2) schedule(static)
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const int64_t c = cell_index(p, x, y, z);
        double rho, U[3];
        cell_moments(f, n, c, &rho, U);
        double g[3];
        for (int a = 0; a < 3; ++a)
          g[a] = (G ? G[(int64_t)a * n + c] : 0.0) + p->g_ext[a];

        double ueq[3], eq[Q], post[Q];
        if (p->forcing == ORC_FORCE_SHIFT) {
          /* step 3: U^G = U + tau G, used in the equilibrium only */
          for (int a = 0; a < 3; ++a) ueq[a] = U[a] + tau * g[a];
          orc_equilibrium(rho, ueq, eq);
          for (int i = 0; i < Q; ++i) {
            double fi = f[(int64_t)i * n + c];
            post[i] = fi + (eq[i] - fi) / tau;
          }
        } else {
          /* Guo forcing: F = rho G, u = U + G/2,
           * S_i = (1 - 1/(2 tau)) t_i [3 (e_i - u) + 9 (e_i.u) e_i] . F */
          double F[3];
          for (int a = 0; a < 3; ++a) {
            F[a] = rho * g[a];
            ueq[a] = U[a] + 0.5 * g[a];
          }
          orc_equilibrium(rho, ueq, eq);
          for (int i = 0; i < Q; ++i) {
            double eu = C[i][0] * ueq[0] + C[i][1] * ueq[1] + C[i][2] * ueq[2];
            double s = 0.0;
            for (int a = 0; a < 3; ++a)
              s += (3.0 * (C[i][a] - ueq[a]) + 9.0 * eu * C[i][a]) * F[a];
            double fi = f[(int64_t)i * n + c];
            post[i] = fi + (eq[i] - fi) / tau +
                      (1.0 - 0.5 / tau) * weight(i) * s;
          }
        }

        /* streaming, eq. (4) */
        const int pos[3] = {x, y, z};
        for (int i = 0; i < Q; ++i) {
          int dst[3];
          int wall_axis = -1, wall_face = 0;
          for (int a = 0; a < 3; ++a) {
            int d = pos[a] + C[i][a];
            if (d < 0 || d >= dims[a]) {
              if (p->bc[a] == ORC_BC_PERIODIC) {
                d = (d + dims[a]) % dims[a];
              } else if (wall_axis < 0) {
                wall_axis = a;
                wall_face = d < 0 ? 0 : 1;
              }
            }
            dst[a] = d;
          }
          if (wall_axis < 0) {
            f_out[(int64_t)i * n + cell_index(p, dst[0], dst[1], dst[2])] =
                post[i];
          } else {
            int o = opposite(i);
            const double* uw = p->wall_u[wall_axis][wall_face];
            double eu = C[o][0] * uw[0] + C[o][1] * uw[1] + C[o][2] * uw[2];
            f_out[(int64_t)o * n + c] =
                post[i] + 6.0 * weight(o) * p->rho_wall * eu;
          }
        }
      }
}

/* Sums of mass and momentum over the box: out = {sum rho, sum rho U}. */
void orc_sums(const orc_params* p, const double* f, double out[4]) {
  const int64_t n = ncells(p);
  double s[4] = {0, 0, 0, 0};
  for (int64_t c = 0; c < n; ++c)
    for (int i = 0; i < Q; ++i) {
      double fi = f[(int64_t)i * n + c];
      s[0] += fi;
      for (int a = 0; a < 3; ++a) s[1 + a] += C[i][a] * fi;
    }
  for (int k = 0; k < 4; ++k) out[k] = s[k];
}

/* ---------------------------------------------------------------------------
 * Peskin's 4-point discrete delta (§3), with the outer-branch reading
 * sqrt(-7 + 12|r| - 4 r^2); zero for |r| >= 2.
 * ------------------------------------------------------------------------- */
double orc_delta(double r) {
  double a = fabs(r);
  if (a <= 1.0) return (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a)) / 8.0;
  if (a <= 2.0) {
    double q = -7.0 + 12.0 * a - 4.0 * a * a;
    if (q < 0.0) q = 0.0; /* rounding at a = 2 */
    return (5.0 - 2.0 * a - sqrt(q)) / 8.0;
  }
  return 0.0;
}

/* Cell coordinate on an axis: wraps on periodic axes; on bounce-back axes a
 * coordinate outside the box is reported with -1. */
static int axis_cell(const orc_params* p, int a, long v) {
  const int dims[3] = {p->nx, p->ny, p->nz};
  long d = dims[a];
  if (v >= 0 && v < d) return (int)v;
  if (p->bc[a] == ORC_BC_PERIODIC) return (int)(((v % d) + d) % d);
  return -1;
}

/*
 * Window of one Lagrangian point: the 5x5x5 cells centred on the nearest
 * cell (Algorithm 2); cells at distance >= 2 on some axis get weight 0.
 * Calls fn(cell, weight) for every cell with a nonzero weight.  Returns
 * ORC_ERR_DOMAIN if a nonzero weight would fall outside a walled box.
 */
typedef struct {
  int64_t cell[125];
  double w[125];
  int count;
} orc_window;

static int point_window(const orc_params* p, const double x[3], orc_window* out) {
  long base[3];
  double wa[3][5];
  int ca[3][5];
  for (int a = 0; a < 3; ++a) {
    base[a] = lround(x[a]);
    for (int j = 0; j < 5; ++j) {
      long X = base[a] - 2 + j;
      wa[a][j] = orc_delta(x[a] - (double)X);
      ca[a][j] = axis_cell(p, a, X);
      if (wa[a][j] != 0.0 && ca[a][j] < 0) return ORC_ERR_DOMAIN;
    }
  }
  out->count = 0;
  for (int k = 0; k < 5; ++k)
    for (int j = 0; j < 5; ++j)
      for (int i = 0; i < 5; ++i) {
        double w = wa[0][i] * wa[1][j] * wa[2][k];
        if (w == 0.0) continue;
        out->cell[out->count] = cell_index(p, ca[0][i], ca[1][j], ca[2][k]);
        out->w[out->count] = w;
        out->count++;
      }
  return ORC_OK;
}

/* Interpolation (§3): u(k) = sum_X U(X) w(x-X) w(y-Y) w(z-Z).
 * x: [n][3] point positions; U: [3][ncell]; u_out: [n][3]. */
int orc_interpolate(const orc_params* p, int64_t npts, const double* x,
                    const double* U, double* u_out) {
  const int64_t n = ncells(p);
  int err = ORC_OK;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < npts; ++k) {
    orc_window win;
    if (point_window(p, x + 3 * k, &win) != ORC_OK) {
#pragma omp atomic write
      err = ORC_ERR_DOMAIN;
      continue;
    }
    double u[3] = {0, 0, 0};
    for (int t = 0; t < win.count; ++t)
      for (int a = 0; a < 3; ++a) u[a] += U[(int64_t)a * n + win.cell[t]] * win.w[t];
    for (int a = 0; a < 3; ++a) u_out[3 * k + a] = u[a];
  }
  return err;
}

/* Spreading (§3): acc(X) += sum_k v(k) w(x-X) w(y-Y) w(z-Z).
 * v: [n][3]; acc: [3][ncell], accumulated in place.  Points run in parallel;
 * concurrent additions to one cell are atomic (FP64, so the order only
 * changes the last bits). */
int orc_spread(const orc_params* p, int64_t npts, const double* x,
               const double* v, double* acc) {
  const int64_t n = ncells(p);
  int err = ORC_OK;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < npts; ++k) {
    orc_window win;
    if (point_window(p, x + 3 * k, &win) != ORC_OK) {
#pragma omp atomic write
      err = ORC_ERR_DOMAIN;
      continue;
    }
    for (int t = 0; t < win.count; ++t)
      for (int a = 0; a < 3; ++a) {
#pragma omp atomic
        acc[(int64_t)a * n + win.cell[t]] += v[3 * k + a] * win.w[t];
      }
  }
  return err;
}

/* ---------------------------------------------------------------------------
 * Rigid motion (§4.2, Algorithm 1): rotation by theta_n = theta0 + omega n
 * about the body axis through its centre; point velocity by the finite
 * difference of positions between steps n and n-1.
 * rest: [n][3] relative to the body centre; body_off: [nb+1] point ranges.
 * ------------------------------------------------------------------------- */
static void rotate(const double axis_in[3], double theta, const double r[3],
                   double out[3]) {
  double len = sqrt(axis_in[0] * axis_in[0] + axis_in[1] * axis_in[1] +
                    axis_in[2] * axis_in[2]);
  double a[3] = {axis_in[0] / len, axis_in[1] / len, axis_in[2] / len};
  double c = cos(theta), s = sin(theta);
  double adr = a[0] * r[0] + a[1] * r[1] + a[2] * r[2];
  double axr[3] = {a[1] * r[2] - a[2] * r[1], a[2] * r[0] - a[0] * r[2],
                   a[0] * r[1] - a[1] * r[0]};
  for (int i = 0; i < 3; ++i)
    out[i] = r[i] * c + axr[i] * s + a[i] * adr * (1.0 - c); /* Rodrigues */
}

void orc_kinematics(int64_t npts, const double* rest, const int64_t* body_off,
                    int32_t nbodies, const orc_body* bodies, int64_t step,
                    double* x_out, double* ub_out) {
  for (int b = 0; b < nbodies; ++b) {
    const orc_body* B = &bodies[b];
    double th_now = B->theta0 + B->omega * (double)step;
    double th_prev = B->theta0 + B->omega * (double)(step - 1);
    for (int64_t k = body_off[b]; k < body_off[b + 1] && k < npts; ++k) {
      double now[3], prev[3];
      rotate(B->axis, th_now, rest + 3 * k, now);
      rotate(B->axis, th_prev, rest + 3 * k, prev);
      for (int a = 0; a < 3; ++a) {
        x_out[3 * k + a] = B->center[a] + now[a];
        ub_out[3 * k + a] = now[a] - prev[a];
      }
    }
  }
}

/* ---------------------------------------------------------------------------
 * Learned warm start, inputs (not part of the paper).
 *
 * orc_neighbours: N(k) for every point k (idx == NULL) or for the listed
 * points: up to 16 other points of k's body, nearest first, with squared
 * rest-frame distance ((dx^2 + dy^2) + dz^2) < 4, ties by index; -1 pads.
 * Brute force over the body.  nbr: [n][16] (rows of unlisted points are left
 * untouched).
 * ------------------------------------------------------------------------- */
#define NNBR 16
void orc_neighbours(int64_t npts, const double* rest, const int64_t* body_off,
                    int32_t nbodies, const int64_t* idx, int64_t n_idx, int32_t* nbr) {
  int32_t* body = (int32_t*)malloc(sizeof(int32_t) * (npts > 0 ? npts : 1));
  for (int32_t b = 0; b < nbodies; ++b)
    for (int64_t k = body_off[b]; k < body_off[b + 1]; ++k) body[k] = b;
  const int64_t m = idx ? n_idx : npts;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t j = 0; j < m; ++j) {
    const int64_t k = idx ? idx[j] : j;
    double bd[NNBR];
    int64_t bi[NNBR];
    int cnt = 0;
    const int32_t b = body[k];
    for (int64_t q = body_off[b]; q < body_off[b + 1]; ++q) {
      if (q == k) continue;
      const double dx = rest[3 * q] - rest[3 * k];
      const double dy = rest[3 * q + 1] - rest[3 * k + 1];
      const double dz = rest[3 * q + 2] - rest[3 * k + 2];
      const double d2 = (dx * dx + dy * dy) + dz * dz;
      if (!(d2 < 4.0)) continue;
      /* keep the 16 smallest (d2, q): insert q in order if it beats the last */
      int pos = cnt;
      while (pos > 0 && (d2 < bd[pos - 1] || (d2 == bd[pos - 1] && q < bi[pos - 1]))) --pos;
      if (pos >= NNBR) continue;
      const int last = cnt < NNBR ? cnt : NNBR - 1;
      for (int i = last; i > pos; --i) {
        bd[i] = bd[i - 1];
        bi[i] = bi[i - 1];
      }
      bd[pos] = d2;
      bi[pos] = q;
      if (cnt < NNBR) ++cnt;
    }
    for (int i = 0; i < NNBR; ++i) nbr[NNBR * k + i] = i < cnt ? (int32_t)bi[i] : -1;
  }
  free(body);
}

/* Reference speed of each body: |omega| max_k |r_k| over its rest points,
 * or 1 when that is zero (a body at rest). */
void orc_vref(const double* rest, const int64_t* body_off, int32_t nbodies,
              const orc_body* bodies, double* vref) {
  for (int32_t b = 0; b < nbodies; ++b) {
    double rmax = 0.0;
    for (int64_t k = body_off[b]; k < body_off[b + 1]; ++k) {
      const double* r = rest + 3 * k;
      const double len = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
      if (len > rmax) rmax = len;
    }
    const double v = fabs(bodies[b].omega) * rmax;
    vref[b] = v > 0.0 ? v : 1.0;
  }
}

/* Features of every point: g0 (3), u_b (3), the mean and the component-wise
 * maximum of g0 over N(k) (3 + 3; zeros when N(k) is empty), each divided
 * by v_pt[k], the reference speed of k's body.  feat: [n][12]. */
void orc_features(int64_t npts, const double* g0, const double* ub, const int32_t* nbr,
                  const double* v_pt, double* feat) {
  for (int64_t k = 0; k < npts; ++k) {
    double* x = feat + 12 * k;
    const double v = v_pt[k];
    double mean[3] = {0, 0, 0}, mx[3] = {0, 0, 0};
    int cnt = 0;
    for (int i = 0; i < NNBR; ++i) {
      const int32_t q = nbr[NNBR * k + i];
      if (q < 0) break;
      for (int a = 0; a < 3; ++a) {
        const double gq = g0[3 * q + a];
        mean[a] += gq;
        mx[a] = cnt == 0 ? gq : (gq > mx[a] ? gq : mx[a]);
      }
      ++cnt;
    }
    for (int a = 0; a < 3; ++a) {
      x[a] = g0[3 * k + a] / v;
      x[3 + a] = ub[3 * k + a] / v;
      x[6 + a] = cnt ? mean[a] / cnt / v : 0.0;
      x[9 + a] = cnt ? mx[a] / v : 0.0;
    }
  }
}

void orc_mlp_forward(const double* theta, int64_t n, const double* x, double* y);

/* ---------------------------------------------------------------------------
 * Multi-direct forcing (§3; Algorithms 1 and 2), up to n_iter sweeps:
 *   U_0 = U;  du = 0
 *   for it in 0 .. n_iter-1:
 *     u_it(k) = interpolation of U_it at x(k)
 *     g_it(k) = u_b(k) - u_it(k)
 *     du(k)  += s(k) g_it(k)
 *     stop after this sweep if it = n_iter-1, or, with ORC_IBM_STOP_RESIDUAL,
 *       if sum_k s|g_it|^2 <= eps^2 sum_k s|u_b|^2 (§3 remarks that the
 *       sweeps may continue until the deficit is small)
 *     otherwise U_{it+1} = U_it + spread of s(k) g_it(k)
 *                        (or of g_it(k) with ORC_IBM_INNER_UNWEIGHTED)
 *   G = spread of du(k)
 * With ORC_IBM_WARM_START (an extension, not in the paper) the first sweep
 * that does not stop replaces its correction: du(k) = s(k) v(k) y(k), with
 * y = MLP(theta; features of k) and v(k) the reference speed of k's body,
 * and U_1 = U_0 + spread of du.  ORC_IBM_WARM_PREV does the same with the
 * previous step's final du(k) of the same point (when there is one).
 * U0 is not modified.  resid[it] = sum_k s(k) |g_it(k)|^2.
 * G_out: [3][ncell] overwritten.  du_out, g_out: [n][3] (nullable);
 * feat_out [n][12] (nullable, needs nbr and v_pt); n_sweeps (nullable).
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t n_iter;
  int32_t flags;       /* ORC_IBM_* */
  double eps;          /* residual threshold of ORC_IBM_STOP_RESIDUAL */
  const double* theta; /* MLP parameters (ORC_IBM_WARM_START) */
  const int32_t* nbr;  /* [n][16] neighbour lists (features) */
  const double* v_pt;  /* [n] reference speed of each point's body */
  const double* du_prev; /* [n][3] previous step's du (ORC_IBM_WARM_PREV; NULL: none) */
} orc_ibm_opts;

static int ibm_core(const orc_params* p, int64_t npts, const double* x,
                    const double* ub, const double* s, double* U, const orc_ibm_opts* o,
                    double* G_out, double* du_out, double* g_out, double* resid,
                    double* feat_out, int32_t* n_sweeps) {
  const int64_t n = ncells(p);
  const int64_t m = npts > 0 ? npts : 1;
  const int warm = (o->flags & ORC_IBM_WARM_START) != 0;
  const int warm_prev = (o->flags & ORC_IBM_WARM_PREV) && o->du_prev;
  const int want_feat = warm || feat_out;
  double* u = (double*)malloc(sizeof(double) * 3 * m);
  double* g = (double*)malloc(sizeof(double) * 3 * m);
  double* v = (double*)malloc(sizeof(double) * 3 * m);
  double* du = (double*)calloc(3 * m, sizeof(double));
  double* feat = want_feat ? (double*)malloc(sizeof(double) * 12 * m) : NULL;
  double* y = warm ? (double*)malloc(sizeof(double) * 3 * m) : NULL;
  double thr = 0.0;
  for (int64_t k = 0; k < npts; ++k)
    thr += s[k] * (ub[3 * k] * ub[3 * k] + ub[3 * k + 1] * ub[3 * k + 1] +
                   ub[3 * k + 2] * ub[3 * k + 2]);
  thr *= o->eps * o->eps;
  int err = ORC_OK;
  int it = 0;
  for (it = 0; it < o->n_iter; ++it) {
    err = orc_interpolate(p, npts, x, U, u);
    if (err != ORC_OK) break;
    double r = 0.0;
    for (int64_t k = 0; k < npts; ++k) {
      double sq = 0.0;
      for (int a = 0; a < 3; ++a) {
        g[3 * k + a] = ub[3 * k + a] - u[3 * k + a];
        du[3 * k + a] += s[k] * g[3 * k + a];
        sq += g[3 * k + a] * g[3 * k + a];
      }
      r += s[k] * sq;
    }
    if (resid) resid[it] = r;
    if (it == 0 && want_feat) orc_features(npts, g, ub, o->nbr, o->v_pt, feat);
    const int stop = it == o->n_iter - 1 || ((o->flags & ORC_IBM_STOP_RESIDUAL) && r <= thr);
    if (stop) break;
    if (it == 0 && warm) {
      orc_mlp_forward(o->theta, npts, feat, y);
      for (int64_t k = 0; k < npts; ++k)
        for (int a = 0; a < 3; ++a) du[3 * k + a] = s[k] * o->v_pt[k] * y[3 * k + a];
      err = orc_spread(p, npts, x, du, U);
    } else if (it == 0 && warm_prev) {
      memcpy(du, o->du_prev, sizeof(double) * 3 * npts);
      err = orc_spread(p, npts, x, du, U);
    } else {
      for (int64_t k = 0; k < npts; ++k)
        for (int a = 0; a < 3; ++a)
          v[3 * k + a] = (o->flags & ORC_IBM_INNER_UNWEIGHTED)
                             ? g[3 * k + a]
                             : s[k] * g[3 * k + a];
      err = orc_spread(p, npts, x, v, U);
    }
    if (err != ORC_OK) break;
  }
  if (err == ORC_OK) {
    memset(G_out, 0, sizeof(double) * 3 * n);
    err = orc_spread(p, npts, x, du, G_out);
  }
  if (err == ORC_OK) {
    if (du_out) memcpy(du_out, du, sizeof(double) * 3 * npts);
    if (g_out) memcpy(g_out, g, sizeof(double) * 3 * npts);
    if (feat_out) memcpy(feat_out, feat, sizeof(double) * 12 * npts);
    if (n_sweeps) *n_sweeps = it < o->n_iter ? it + 1 : o->n_iter;
  }
  free(u);
  free(g);
  free(v);
  free(du);
  free(feat);
  free(y);
  return err;
}

int orc_ibm(const orc_params* p, int64_t npts, const double* x,
            const double* ub, const double* s, const double* U0,
            const orc_ibm_opts* o, double* G_out, double* du_out,
            double* g_out, double* resid, double* feat_out, int32_t* n_sweeps) {
  const int64_t n = ncells(p);
  double* U = (double*)malloc(sizeof(double) * 3 * n);
  memcpy(U, U0, sizeof(double) * 3 * n);
  int err = ibm_core(p, npts, x, ub, s, U, o, G_out, du_out, g_out, resid,
                     feat_out, n_sweeps);
  free(U);
  return err;
}

/* ---------------------------------------------------------------------------
 * One full time step (§2 step list, with §3 for step 2):
 *   1. rho, U from f                       (eq. 1)
 *   2. G = immersedBoundary(object, U)     (§3; skipped when npts == 0)
 *   3-5. forcing, equilibrium, collision   (eqs. 2-3)
 *   6. streaming                           (eq. 4)
 * f (post-stream state at time `step`) is replaced by the state at step+1.
 * Optional outputs (NULL to skip): sums of f before the step; G; point
 * positions, velocities, last deficit and accumulated correction; residuals.
 * ------------------------------------------------------------------------- */
typedef struct {
  int64_t npts;
  const double* rest;      /* [n][3] */
  const double* area;      /* [n]    */
  const int64_t* body_off; /* [nb+1] */
  int32_t nbodies;
  int32_t n_iter;
  int32_t flags;
  int32_t pad_;
  const orc_body* bodies;
  double eps;           /* ORC_IBM_STOP_RESIDUAL threshold */
  const double* theta;  /* ORC_IBM_WARM_START parameters */
  const double* du_prev; /* ORC_IBM_WARM_PREV: du of the step before the first (nullable) */
} orc_points;

typedef struct {
  double* sums;  /* [4] */
  double* G;     /* [3][ncell] */
  double* x;     /* [n][3] */
  double* ub;    /* [n][3] */
  double* g;     /* [n][3] */
  double* du;    /* [n][3] */
  double* resid; /* [n_iter] */
  double* feat;  /* [n][12] features of the first sweep */
  int32_t* n_sweeps;
} orc_step_out;

/* Buffers reused across the steps of one run. */
typedef struct {
  double *fn, *rho, *U, *G, *x, *ub;
  int32_t* nbr;  /* neighbour lists, found once per run when needed */
  double* v_pt;
  double* du_prev;  /* the last step's du within a run (ORC_IBM_WARM_PREV) */
  int have_prev;
} orc_ws;

static void ws_alloc(orc_ws* w, int64_t n, int64_t m) {
  if (m < 1) m = 1;
  w->fn = (double*)malloc(sizeof(double) * Q * n);
  w->rho = (double*)malloc(sizeof(double) * n);
  w->U = (double*)malloc(sizeof(double) * 3 * n);
  w->G = (double*)malloc(sizeof(double) * 3 * n);
  w->x = (double*)malloc(sizeof(double) * 3 * m);
  w->ub = (double*)malloc(sizeof(double) * 3 * m);
  w->nbr = NULL;
  w->v_pt = NULL;
  w->du_prev = (double*)malloc(sizeof(double) * 3 * m);
  w->have_prev = 0;
}

static void ws_free(orc_ws* w) {
  free(w->fn);
  free(w->rho);
  free(w->U);
  free(w->G);
  free(w->x);
  free(w->ub);
  free(w->nbr);
  free(w->v_pt);
  free(w->du_prev);
}

/* Neighbour lists and per-point reference speeds of the warm start. */
static void ws_learned(orc_ws* w, const orc_points* pts) {
  if (w->nbr) return;
  const int64_t m = pts->npts > 0 ? pts->npts : 1;
  w->nbr = (int32_t*)malloc(sizeof(int32_t) * NNBR * m);
  w->v_pt = (double*)malloc(sizeof(double) * m);
  double* vb = (double*)malloc(sizeof(double) * (pts->nbodies > 0 ? pts->nbodies : 1));
  orc_neighbours(pts->npts, pts->rest, pts->body_off, pts->nbodies, NULL, 0, w->nbr);
  orc_vref(pts->rest, pts->body_off, pts->nbodies, pts->bodies, vb);
  for (int32_t b = 0; b < pts->nbodies; ++b)
    for (int64_t k = pts->body_off[b]; k < pts->body_off[b + 1]; ++k) w->v_pt[k] = vb[b];
  free(vb);
}

/* One step from f into w->fn (f is left unchanged). */
static int step_into(const orc_params* p, const double* f, const orc_points* pts,
                     int64_t step, const orc_step_out* out, orc_ws* w) {
  const int64_t n = ncells(p);
  const double* G = NULL;
  int err = ORC_OK;
  if (out && out->sums) orc_sums(p, f, out->sums);
  if (pts && pts->npts > 0) {
    int64_t m = pts->npts;
    orc_moments(p, f, w->rho, w->U);
    orc_kinematics(m, pts->rest, pts->body_off, pts->nbodies, pts->bodies,
                   step, w->x, w->ub);
    const int learned = (pts->flags & ORC_IBM_WARM_START) || (out && out->feat);
    if (learned) ws_learned(w, pts);
    orc_ibm_opts o;
    o.n_iter = pts->n_iter;
    o.flags = pts->flags;
    o.eps = pts->eps;
    o.theta = pts->theta;
    o.nbr = w->nbr;
    o.v_pt = w->v_pt;
    o.du_prev = w->have_prev ? w->du_prev : pts->du_prev;
    double* du_new = (double*)malloc(sizeof(double) * 3 * m);
    err = ibm_core(p, m, w->x, w->ub, pts->area, w->U, &o, w->G, du_new,
                   out ? out->g : NULL, out ? out->resid : NULL,
                   out ? out->feat : NULL, out ? out->n_sweeps : NULL);
    if (err == ORC_OK) {
      if (out && out->du) memcpy(out->du, du_new, sizeof(double) * 3 * m);
      memcpy(w->du_prev, du_new, sizeof(double) * 3 * m);
      w->have_prev = 1;
    }
    free(du_new);
    if (out && out->x) memcpy(out->x, w->x, sizeof(double) * 3 * m);
    if (out && out->ub) memcpy(out->ub, w->ub, sizeof(double) * 3 * m);
    G = w->G;
  }
  if (err != ORC_OK) return err;
  if (out && out->G) {
    if (G)
      memcpy(out->G, G, sizeof(double) * 3 * n);
    else
      memset(out->G, 0, sizeof(double) * 3 * n);
  }
  orc_collide_stream(p, f, G, w->fn);
  return ORC_OK;
}

int orc_step(const orc_params* p, double* f, const orc_points* pts,
             int64_t step, const orc_step_out* out) {
  orc_ws w;
  ws_alloc(&w, ncells(p), pts ? pts->npts : 0);
  int err = step_into(p, f, pts, step, out, &w);
  if (err == ORC_OK) memcpy(f, w.fn, sizeof(double) * Q * ncells(p));
  ws_free(&w);
  return err;
}

/* n_steps full steps starting at time `step0`; sums_hist (nullable) gets
 * the sums before each step, [n_steps][4]; sweeps_hist (nullable) the
 * sweeps of each step's forcing, [n_steps]. */
int orc_run(const orc_params* p, double* f, const orc_points* pts,
            int64_t step0, int64_t n_steps, double* sums_hist, int32_t* sweeps_hist) {
  const int64_t n = ncells(p);
  orc_ws w;
  ws_alloc(&w, n, pts ? pts->npts : 0);
  double* cur = f;
  int err = ORC_OK;
  for (int64_t s = 0; s < n_steps && err == ORC_OK; ++s) {
    orc_step_out o;
    memset(&o, 0, sizeof(o));
    o.sums = sums_hist ? sums_hist + 4 * s : NULL;
    o.n_sweeps = sweeps_hist ? sweeps_hist + s : NULL;
    err = step_into(p, cur, pts, step0 + s, &o, &w);
    if (err == ORC_OK) { /* swap the state and the work lattice */
      double* t = w.fn;
      w.fn = cur;
      cur = t;
    }
  }
  if (cur != f) { /* final state lives in the work buffer */
    memcpy(f, cur, sizeof(double) * Q * n);
    w.fn = cur;
  }
  ws_free(&w);
  return err;
}

/* ---------------------------------------------------------------------------
 * Learned warm start: a per-point MLP 12 -> 64 -> 64 -> 64 -> 3 with SiLU
 * after each hidden layer (not part of the paper; its inputs are the point's
 * first deficit, its velocity and the mean and component-wise maximum of
 * the first deficit over its neighbours, all divided by a reference speed;
 * its output is the predicted correction du divided by that speed).
 *
 * Flat parameter layout (9347 values, row-major matrices, out x in):
 *   W1[64][12] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[3][64] b4[3]
 * Loss: L = (1 / (3 n)) sum_k sum_c (y_kc - t_kc)^2.
 * ------------------------------------------------------------------------- */
#define MLP_IN 12
#define MLP_H 64
#define MLP_OUT 3
#define MLP_NPARAM (MLP_H * MLP_IN + MLP_H + 2 * (MLP_H * MLP_H + MLP_H) + MLP_OUT * MLP_H + MLP_OUT)

static double sigmoid(double z) { return 1.0 / (1.0 + exp(-z)); }

int32_t orc_mlp_nparam(void) { return MLP_NPARAM; }

typedef struct {
  const double *W1, *b1, *W2, *b2, *W3, *b3, *W4, *b4;
} mlp_view;

static mlp_view mlp_split(const double* th) {
  mlp_view v;
  v.W1 = th;
  v.b1 = v.W1 + MLP_H * MLP_IN;
  v.W2 = v.b1 + MLP_H;
  v.b2 = v.W2 + MLP_H * MLP_H;
  v.W3 = v.b2 + MLP_H;
  v.b3 = v.W3 + MLP_H * MLP_H;
  v.W4 = v.b3 + MLP_H;
  v.b4 = v.W4 + MLP_OUT * MLP_H;
  return v;
}

/* One dense layer z = W a + b, optionally followed by SiLU into h. */
static void dense(const double* W, const double* b, const double* a, int nin, int nout,
                  double* z, double* h) {
  for (int o = 0; o < nout; ++o) {
    double s = b[o];
    for (int i = 0; i < nin; ++i) s += W[o * nin + i] * a[i];
    z[o] = s;
    if (h) h[o] = s * sigmoid(s);
  }
}

void orc_mlp_forward(const double* theta, int64_t n, const double* x, double* y) {
  mlp_view P = mlp_split(theta);
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; ++k) {
    double z1[MLP_H], h1[MLP_H], z2[MLP_H], h2[MLP_H], z3[MLP_H], h3[MLP_H];
    dense(P.W1, P.b1, x + MLP_IN * k, MLP_IN, MLP_H, z1, h1);
    dense(P.W2, P.b2, h1, MLP_H, MLP_H, z2, h2);
    dense(P.W3, P.b3, h2, MLP_H, MLP_H, z3, h3);
    dense(P.W4, P.b4, h3, MLP_H, MLP_OUT, y + MLP_OUT * k, NULL);
  }
}

/* d SiLU / dz */
static double silu_grad(double z) {
  double s = sigmoid(z);
  return s * (1.0 + z * (1.0 - s));
}

/* Loss and its gradient (back-propagation written out layer by layer);
 * samples are processed one after the other. */
double orc_mlp_loss_grad(const double* theta, int64_t n, const double* x, const double* t,
                         double* grad) {
  mlp_view P = mlp_split(theta);
  memset(grad, 0, sizeof(double) * MLP_NPARAM);
  double* gW1 = grad;
  double* gb1 = gW1 + MLP_H * MLP_IN;
  double* gW2 = gb1 + MLP_H;
  double* gb2 = gW2 + MLP_H * MLP_H;
  double* gW3 = gb2 + MLP_H;
  double* gb3 = gW3 + MLP_H * MLP_H;
  double* gW4 = gb3 + MLP_H;
  double* gb4 = gW4 + MLP_OUT * MLP_H;
  double loss = 0.0;
  const double scale = 1.0 / (3.0 * (double)n);
  for (int64_t k = 0; k < n; ++k) {
    const double* a0 = x + MLP_IN * k;
    double z1[MLP_H], h1[MLP_H], z2[MLP_H], h2[MLP_H], z3[MLP_H], h3[MLP_H], y[MLP_OUT];
    dense(P.W1, P.b1, a0, MLP_IN, MLP_H, z1, h1);
    dense(P.W2, P.b2, h1, MLP_H, MLP_H, z2, h2);
    dense(P.W3, P.b3, h2, MLP_H, MLP_H, z3, h3);
    dense(P.W4, P.b4, h3, MLP_H, MLP_OUT, y, NULL);
    double dy[MLP_OUT], d3[MLP_H], d2[MLP_H], d1[MLP_H];
    for (int c = 0; c < MLP_OUT; ++c) {
      double r = y[c] - t[MLP_OUT * k + c];
      loss += r * r * scale;
      dy[c] = 2.0 * r * scale; /* dL/dy */
    }
    /* output layer */
    for (int c = 0; c < MLP_OUT; ++c) {
      gb4[c] += dy[c];
      for (int i = 0; i < MLP_H; ++i) gW4[c * MLP_H + i] += dy[c] * h3[i];
    }
    for (int i = 0; i < MLP_H; ++i) {
      double s = 0.0;
      for (int c = 0; c < MLP_OUT; ++c) s += P.W4[c * MLP_H + i] * dy[c];
      d3[i] = s * silu_grad(z3[i]); /* dL/dz3 */
    }
    /* third layer */
    for (int o = 0; o < MLP_H; ++o) {
      gb3[o] += d3[o];
      for (int i = 0; i < MLP_H; ++i) gW3[o * MLP_H + i] += d3[o] * h2[i];
    }
    for (int i = 0; i < MLP_H; ++i) {
      double s = 0.0;
      for (int o = 0; o < MLP_H; ++o) s += P.W3[o * MLP_H + i] * d3[o];
      d2[i] = s * silu_grad(z2[i]);
    }
    /* second layer */
    for (int o = 0; o < MLP_H; ++o) {
      gb2[o] += d2[o];
      for (int i = 0; i < MLP_H; ++i) gW2[o * MLP_H + i] += d2[o] * h1[i];
    }
    for (int i = 0; i < MLP_H; ++i) {
      double s = 0.0;
      for (int o = 0; o < MLP_H; ++o) s += P.W2[o * MLP_H + i] * d2[o];
      d1[i] = s * silu_grad(z1[i]);
    }
    /* first layer */
    for (int o = 0; o < MLP_H; ++o) {
      gb1[o] += d1[o];
      for (int i = 0; i < MLP_IN; ++i) gW1[o * MLP_IN + i] += d1[o] * a0[i];
    }
  }
  return loss;
}

/* Adam (Kingma & Ba) with bias correction; step_t counts from 1. */
void orc_adam_step(double* theta, const double* grad, double* m, double* v, int64_t step_t,
                   double lr, double beta1, double beta2, double eps) {
  const double c1 = 1.0 - pow(beta1, (double)step_t);
  const double c2 = 1.0 - pow(beta2, (double)step_t);
  for (int p = 0; p < MLP_NPARAM; ++p) {
    m[p] = beta1 * m[p] + (1.0 - beta1) * grad[p];
    v[p] = beta2 * v[p] + (1.0 - beta2) * grad[p] * grad[p];
    theta[p] -= lr * (m[p] / c1) / (sqrt(v[p] / c2) + eps);
  }
}
