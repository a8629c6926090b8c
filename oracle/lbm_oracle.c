/*
 * FP64 CPU oracle of the site-based suspension lattice Boltzmann method
 * (dos Santos & Philippi).  TEST INFRASTRUCTURE ONLY: loaded by the tests,
 * the smoke check and the CPU-baseline leg of the benchmark, never by the
 * product path.  Plain loops, plain f, FP64, no blocking or fusion.  Each
 * function names the passage of the paper it follows; the readings taken where
 * the paper is silent are listed with the function.
 *
 * Threads: the per-site loops (collision, propagation, read-outs) may run on
 * several OpenMP threads.  Each of their iterations writes only its own sites
 * and no iteration reads what another writes, so the result is the same bit
 * for bit as with one thread; every sum over sites or particles (the BS
 * substep, the walls' momentum, the IS leak) stays a plain loop in a fixed
 * order on one thread.
 *
 * One time step, in the paper's order (section 2.2: the particle substeps sit
 * between collision and propagation):
 *   collide every site (eq. 1-3)
 *   BS substep on the current map: impose u_B' and sum dp, dl (eq. 5-9)
 *   particle acceleration (eq. 10-11), hard-core collisions (eq. 16-19)
 *   translation of particle and site sets (eq. 13-15)
 *   IS substep on the new map (eq. 12 and the fourth substep)
 *   propagate every site (eq. 3, left-hand side)
 * Optional walls close the box along chosen axes (section 3's closed boxes;
 * the paper does not say how its walls are imposed, see wall_substep).
 */
#include "lbm_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------
 * Velocity sets.  The paper draws D2Q9 (figure 1) without printing weights,
 * and never names its 3D lattice; D3Q19 with the standard weights is the
 * reading taken.  c_s^2 = 1/3 for both, consistent with tau = 0.6 giving
 * nu = 1/30 through eq. 4 (section 3.2).
 * ---------------------------------------------------------------------- */
static const int C9[9][3] = {{0, 0, 0},  {1, 0, 0},  {0, 1, 0},
                             {-1, 0, 0}, {0, -1, 0}, {1, 1, 0},
                             {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
static const double W9[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                             1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int C19[19][3] = {
    {0, 0, 0},   {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
    {0, 0, 1},   {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
    {-1, 1, 0},  {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},   {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static const double W19[19] = {
    1.0 / 3.0,  1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
    1.0 / 18.0, 1.0 / 18.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

int ora_lattice(int q, int32_t *c, double *w) {
  if (q != 9 && q != 19) return -1;
  for (int i = 0; i < q; i++) {
    for (int a = 0; a < 3; a++) c[3 * i + a] = q == 9 ? C9[i][a] : C19[i][a];
    w[i] = q == 9 ? W9[i] : W19[i];
  }
  return 0;
}

/* Equilibrium: the paper only says "a polynomial approximation of the
 * Maxwell-Boltzmann equilibrium" (section 2.1).  Reading: the usual
 * second-order form w_i rho [1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u]. */
void ora_feq(int q, double rho, const double u[3], double *feq) {
  const int(*c)[3] = q == 9 ? C9 : C19;
  const double *w = q == 9 ? W9 : W19;
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < q; i++) {
    double cu = c[i][0] * u[0] + c[i][1] * u[1] + c[i][2] * u[2];
    feq[i] = w[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
  }
}

/* ------------------------------------------------------------------------
 * State
 * ---------------------------------------------------------------------- */
typedef struct {
  double x[3], x0[3], u[3], om[3]; /* x unwrapped; x0 = x at creation */
  double r, m, I, V;
  double fext[3];      /* buoyancy-corrected weight (m - rho0 V) g */
  double F[3], T[3];   /* last step's -dP, -dL */
  int b0[3], k[3];     /* b0 = [x0]; k = [x - x0] (nearest integer) */
  double phi[3];       /* x0 - b0: sub-lattice offset of the centre */
  int nbs, nis;        /* template sizes */
  int *off;            /* [nbs+nis][3], BS entries first */
} particle;

struct ora_sim {
  int q, dim, nx, ny, nz;
  long N;
  double tau, rho0, g[3], fb_user[3], fb[3];
  int znf;
  const int (*c)[3];
  const double *w;
  double *f, *fs; /* [q][N]: post-propagation and post-collision */
  int *own_p, *own_e;
  int np, cap;
  particle *P;
  double leak[3];
  long conflicts;
  long step;
  int walls;              /* bit a: axis a closed by wall layers */
  double wall_u[3][2][3]; /* [axis][low, high][component] */
  double wall_dp[3];      /* momentum the walls gave the fluid, last step */
  int closure;            /* near-contact closure network on */
  double clo_p[4866];     /* its parameters (FP32 values) */
  double clo_h;           /* gap below which it acts */
  double (*Fc)[3];        /* closure force of the last step, per particle */
};

static long site_index(const ora_sim *s, long x, long y, long z) {
  return x + s->nx * (y + s->ny * z);
}

static long wrapi(long a, long n) {
  long r = a % n;
  return r < 0 ? r + n : r;
}

/* Wall layers.  Reading (the paper closes its boxes but does not describe
 * the walls): a wall is an immobile solid slab treated by the same site
 * rule as a particle.  A closed axis of n sites keeps layers 2 .. n-3 as
 * fluid; layers 1 and n-2 are the wall's BS sites (linked to the fluid),
 * layers 0 and n-1 its IS sites (linked to the BS layers; across the
 * periodic seam the two walls form one slab of four layers).  The wall
 * velocity U is tangential and applies to the layers of its side.  At a site
 * in the layers of several axes the lowest axis decides the velocity.
 * Returns 1 and the velocity for a wall site, 0 otherwise. */
static int wall_site(const ora_sim *s, long x, long y, long z, double U[3]) {
  long c[3] = {x, y, z};
  int L[3] = {s->nx, s->ny, s->nz};
  for (int a = 0; a < s->dim; a++) {
    if (!(s->walls & (1 << a))) continue;
    if (c[a] < 2 || c[a] >= L[a] - 2) {
      int side = c[a] >= L[a] - 2;
      if (U)
        for (int b = 0; b < 3; b++) U[b] = s->wall_u[a][side][b];
      return 1;
    }
  }
  return 0;
}

ora_sim *ora_create(int q, int nx, int ny, int nz, double tau, double rho0,
                    const double gravity[3], const double body_force[3],
                    int zero_net_force) {
  if ((q != 9 && q != 19) || nx < 1 || ny < 1 || nz < 1 || !(tau > 0.5))
    return NULL;
  if (q == 9 && nz != 1) return NULL;
  ora_sim *s = (ora_sim *)calloc(1, sizeof(ora_sim));
  s->q = q;
  s->dim = q == 9 ? 2 : 3;
  s->nx = nx;
  s->ny = ny;
  s->nz = nz;
  s->N = (long)nx * ny * nz;
  s->tau = tau;
  s->rho0 = rho0;
  for (int a = 0; a < 3; a++) {
    s->g[a] = gravity ? gravity[a] : 0.0;
    s->fb_user[a] = body_force ? body_force[a] : 0.0;
    s->fb[a] = s->fb_user[a];
  }
  s->znf = zero_net_force;
  s->c = q == 9 ? C9 : C19;
  s->w = q == 9 ? W9 : W19;
  s->f = (double *)malloc(sizeof(double) * q * s->N);
  s->fs = (double *)malloc(sizeof(double) * q * s->N);
  s->own_p = (int *)malloc(sizeof(int) * s->N);
  s->own_e = (int *)malloc(sizeof(int) * s->N);
  if (!s->f || !s->fs || !s->own_p || !s->own_e) {
    ora_destroy(s);
    return NULL;
  }
  /* Initial state: fluid at rest with density rho0 (the paper is silent). */
  for (int i = 0; i < q; i++) {
#pragma omp parallel for schedule(static)
    for (long n = 0; n < s->N; n++) s->f[i * s->N + n] = s->w[i] * rho0;
  }
#pragma omp parallel for schedule(static)
  for (long n = 0; n < s->N; n++) s->own_p[n] = s->own_e[n] = -1;
  return s;
}

void ora_destroy(ora_sim *s) {
  if (!s) return;
  for (int p = 0; p < s->np; p++) free(s->P[p].off);
  free(s->P);
  free(s->Fc);
  free(s->f);
  free(s->fs);
  free(s->own_p);
  free(s->own_e);
  free(s);
}

int ora_num_particles(const ora_sim *s) { return s->np; }

/* ------------------------------------------------------------------------
 * Particle template (section 2.2, figure 2).  Readings:
 *  - the particle's sites P are the lattice sites o (relative to b0 = [x0])
 *    with |o - phi| <= r, phi = x0 - b0;
 *  - BS: sites of P with a lattice link (any non-zero c_i of the lattice in
 *    use) to a site outside P ("particle sites in contact with fluid");
 *  - IS: sites of P that are not BS and have a link to a BS site ("particle
 *    sites in contact with the boundary sites");
 *  - deeper sites are ordinary sites (every site collides and propagates).
 * The set is later translated rigidly by the integer shift k (eq. 14-15 with
 * no rotation), so it is built once per particle.
 * ---------------------------------------------------------------------- */
static int build_template(const ora_sim *s, particle *P) {
  int R = (int)ceil(P->r) + 1;
  int ext = 2 * R + 3; /* one spare ring so o + c_i stays inside the grid */
  int h = R + 1;
  int ez = s->dim == 3 ? ext : 1, hz = s->dim == 3 ? h : 0;
  int nall = ext * ext * ez;
  char *in = (char *)calloc(nall, 1);
  char *bs = (char *)calloc(nall, 1);
#define GI(ox, oy, oz) (((oz) + hz) * ext * ext + ((oy) + h) * ext + ((ox) + h))
  int Rz = s->dim == 3 ? R : 0;
  for (int oz = -Rz; oz <= Rz; oz++)
    for (int oy = -R; oy <= R; oy++)
      for (int ox = -R; ox <= R; ox++) {
        double dx = ox - P->phi[0], dy = oy - P->phi[1], dz = oz - P->phi[2];
        if (dx * dx + dy * dy + dz * dz <= P->r * P->r) in[GI(ox, oy, oz)] = 1;
      }
  int nbs = 0, nis = 0;
  for (int oz = -Rz; oz <= Rz; oz++)
    for (int oy = -R; oy <= R; oy++)
      for (int ox = -R; ox <= R; ox++) {
        if (!in[GI(ox, oy, oz)]) continue;
        for (int i = 1; i < s->q; i++)
          if (!in[GI(ox + s->c[i][0], oy + s->c[i][1], oz + s->c[i][2])]) {
            bs[GI(ox, oy, oz)] = 1;
            break;
          }
        nbs += bs[GI(ox, oy, oz)];
      }
  char *is = (char *)calloc(nall, 1);
  for (int oz = -Rz; oz <= Rz; oz++)
    for (int oy = -R; oy <= R; oy++)
      for (int ox = -R; ox <= R; ox++) {
        if (!in[GI(ox, oy, oz)] || bs[GI(ox, oy, oz)]) continue;
        for (int i = 1; i < s->q; i++)
          if (bs[GI(ox + s->c[i][0], oy + s->c[i][1], oz + s->c[i][2])]) {
            is[GI(ox, oy, oz)] = 1;
            break;
          }
        nis += is[GI(ox, oy, oz)];
      }
  P->nbs = nbs;
  P->nis = nis;
  P->off = (int *)malloc(sizeof(int) * 3 * (nbs + nis > 0 ? nbs + nis : 1));
  int e = 0;
  for (int pass = 0; pass < 2; pass++)
    for (int oz = -Rz; oz <= Rz; oz++)
      for (int oy = -R; oy <= R; oy++)
        for (int ox = -R; ox <= R; ox++) {
          char want = pass == 0 ? bs[GI(ox, oy, oz)] : is[GI(ox, oy, oz)];
          if (!want) continue;
          P->off[3 * e] = ox;
          P->off[3 * e + 1] = oy;
          P->off[3 * e + 2] = oz;
          e++;
        }
#undef GI
  free(in);
  free(bs);
  free(is);
  return 0;
}

/* Site of template entry e of particle P at its current shift. */
static long entry_site(const ora_sim *s, const particle *P, int e) {
  long x = wrapi((long)P->b0[0] + P->k[0] + P->off[3 * e], s->nx);
  long y = wrapi((long)P->b0[1] + P->k[1] + P->off[3 * e + 1], s->ny);
  long z = wrapi((long)P->b0[2] + P->k[2] + P->off[3 * e + 2], s->nz);
  return site_index(s, x, y, z);
}

/* Lever arm x_B - x_p of entry e: constant o - phi, because the site set and
 * the centre move together (eq. 13-15).  The continuous arm is the reading
 * taken for eq. 5, 7 and 12. */
static void lever_arm(const particle *P, int e, double r[3]) {
  for (int a = 0; a < 3; a++) r[a] = (double)P->off[3 * e + a] - P->phi[a];
}

static void cross(const double a[3], const double b[3], double out[3]) {
  out[0] = a[1] * b[2] - a[2] * b[1];
  out[1] = a[2] * b[0] - a[0] * b[2];
  out[2] = a[0] * b[1] - a[1] * b[0];
}

static double min_image(double d, int n) { return d - n * floor(d / n + 0.5); }

/* Rasterise every particle at b0 + k (section 2.2, integer counterpart [x]).
 * A site claimed by two particles belongs to the lower id (the paper is
 * silent on overlapping site sets). */
static void raster(ora_sim *s) {
#pragma omp parallel for schedule(static)
  for (long n = 0; n < s->N; n++) s->own_p[n] = s->own_e[n] = -1;
  s->conflicts = 0;
  for (int p = 0; p < s->np; p++) {
    particle *P = &s->P[p];
    for (int e = 0; e < P->nbs + P->nis; e++) {
      long n = entry_site(s, P, e);
      /* wall sites belong to the wall (it acts as the lowest id) */
      if (wall_site(s, n % s->nx, (n / s->nx) % s->ny, n / ((long)s->nx * s->ny), NULL))
        continue;
      if (s->own_p[n] < 0) {
        s->own_p[n] = p;
        s->own_e[n] = e;
      } else {
        s->conflicts++;
      }
    }
  }
}

static double analytic_volume(int dim, double r) {
  return dim == 2 ? M_PI * r * r : 4.0 / 3.0 * M_PI * r * r * r;
}

/* Uniform fluid body force.  Periodic boxes with gravity on the particles
 * need a frame in which the whole suspension carries no net external force;
 * reading: the fluid carries -sum_p F_ext,p / N on every site. */
static void update_body_force(ora_sim *s) {
  double tot[3] = {0, 0, 0};
  for (int p = 0; p < s->np; p++)
    for (int a = 0; a < 3; a++) tot[a] += s->P[p].fext[a];
  for (int a = 0; a < 3; a++)
    s->fb[a] = s->fb_user[a] - (s->znf ? tot[a] / (double)s->N : 0.0);
}

int ora_add_particles(ora_sim *s, int n, const double *x, const double *u,
                      const double *omega, const double *radius,
                      const double *mass, const double *inertia) {
  if (n < 0) return -1;
  int first = s->np;
  if (s->np + n > s->cap) {
    int nc = s->cap ? s->cap : 16;
    while (nc < s->np + n) nc *= 2;
    particle *np = (particle *)realloc(s->P, sizeof(particle) * nc);
    if (!np) return -1;
    s->P = np;
    double(*fc)[3] = (double(*)[3])realloc(s->Fc, sizeof(double[3]) * nc);
    if (!fc) return -1;
    s->Fc = fc;
    s->cap = nc;
  }
  for (int j = 0; j < n; j++) {
    particle *P = &s->P[s->np];
    memset(P, 0, sizeof(*P));
    for (int a = 0; a < 3; a++) {
      P->x[a] = x[3 * j + a];
      P->x0[a] = P->x[a];
      P->u[a] = u ? u[3 * j + a] : 0.0;
      P->om[a] = omega ? omega[3 * j + a] : 0.0;
    }
    if (s->dim == 2) {
      P->x[2] = P->x0[2] = 0.0;
      P->u[2] = 0.0;
      P->om[0] = P->om[1] = 0.0;
    }
    P->r = radius[j];
    P->m = mass[j];
    P->I = inertia[j];
    P->V = analytic_volume(s->dim, P->r);
    for (int a = 0; a < 3; a++) {
      /* nearest integer, ties upward: [x] = floor(x + 1/2) */
      P->b0[a] = (int)floor(P->x0[a] + 0.5);
      P->phi[a] = P->x0[a] - (double)P->b0[a];
      P->k[a] = 0;
      /* gravity on particles, buoyancy-corrected; absent for kinematic
       * particles (infinite mass) */
      P->fext[a] = isinf(P->m) ? 0.0 : (P->m - s->rho0 * P->V) * s->g[a];
    }
    build_template(s, P);
    s->np++;
  }
  update_body_force(s);
  raster(s);
  return first;
}

/* ------------------------------------------------------------------------
 * Step pieces
 * ---------------------------------------------------------------------- */

/* Eq. 1-3: moments and BGK relaxation at every site, plus the body-force
 * term 3 w_i c_i.f_b (first-order forcing; adds exactly f_b momentum and no
 * mass). */
static void collide(ora_sim *s) {
  const int q = s->q;
  const long N = s->N;
#pragma omp parallel for schedule(static)
  for (long n = 0; n < N; n++) {
    double fi[19], feq[19], u[3];
    double rho = 0, j[3] = {0, 0, 0};
    for (int i = 0; i < q; i++) {
      fi[i] = s->f[i * N + n];
      rho += fi[i];
      for (int a = 0; a < 3; a++) j[a] += fi[i] * s->c[i][a];
    }
    for (int a = 0; a < 3; a++) u[a] = j[a] / rho;
    ora_feq(q, rho, u, feq);
    for (int i = 0; i < q; i++) {
      double cf = s->c[i][0] * s->fb[0] + s->c[i][1] * s->fb[1] +
                  s->c[i][2] * s->fb[2];
      s->fs[i * N + n] = fi[i] - (fi[i] - feq[i]) / s->tau + 3.0 * s->w[i] * cf;
    }
  }
}

/* Density and momentum of the post-collision distributions at site n. */
static void site_moments(const ora_sim *s, const double *f, long n,
                         double *rho, double u[3]) {
  double r = 0, j[3] = {0, 0, 0};
  for (int i = 0; i < s->q; i++) {
    double v = f[i * s->N + n];
    r += v;
    for (int a = 0; a < 3; a++) j[a] += v * s->c[i][a];
  }
  *rho = r;
  for (int a = 0; a < 3; a++) u[a] = j[a] / r;
}

static void impose_equilibrium(ora_sim *s, long n, double rho,
                               const double u[3]) {
  double feq[19];
  ora_feq(s->q, rho, u, feq);
  for (int i = 0; i < s->q; i++) s->fs[i * s->N + n] = feq[i];
}

/* First substep (eq. 5-9) on the map of the positions before translation:
 * every BS site takes f^eq(rho_B, u_B') with u_B' the rigid-body velocity of
 * the particle there; the momentum and angular momentum this gives the fluid
 * are summed per particle.  Readings:
 *  - u_B' = u_p + omega_p x r (the printed r x omega spins a particle up,
 *    see the spin-down test);
 *  - rho_B, u_B are the site's post-collision moments, and rho_B is kept in
 *    the imposed equilibrium (the imposition conserves mass per site). */
static void boundary_substep(ora_sim *s, double (*dP)[3], double (*dL)[3]) {
  for (int p = 0; p < s->np; p++) {
    particle *P = &s->P[p];
    for (int a = 0; a < 3; a++) dP[p][a] = dL[p][a] = 0.0;
    for (int e = 0; e < P->nbs; e++) {
      long n = entry_site(s, P, e);
      if (s->own_p[n] != p || s->own_e[n] != e) continue;
      double rho, uB[3], r[3], wr[3], uBp[3], dp[3], dl[3];
      site_moments(s, s->fs, n, &rho, uB);
      lever_arm(P, e, r);
      cross(P->om, r, wr);
      for (int a = 0; a < 3; a++) uBp[a] = P->u[a] + wr[a];
      for (int a = 0; a < 3; a++) dp[a] = rho * (uBp[a] - uB[a]);
      cross(r, dp, dl);
      impose_equilibrium(s, n, rho, uBp);
      for (int a = 0; a < 3; a++) {
        dP[p][a] += dp[a];
        dL[p][a] += dl[a];
      }
    }
  }
}

/* The wall's share of the substeps.  Every wall site takes f^eq(rho, U)
 * with its own post-collision density and the wall velocity, as BS and IS
 * sites of a particle do (eq. 5, 12).  The wall does not move, so its BS
 * sites (first substep) and IS sites (fourth substep) take the same values
 * whichever substep imposes them, and no particle owns a wall site; doing
 * all of them here gives the same state.  The momentum given to the fluid is
 * kept as a diagnostic. */
static void wall_substep(ora_sim *s) {
  for (int a = 0; a < 3; a++) s->wall_dp[a] = 0.0;
  if (!s->walls) return;
  for (long z = 0; z < s->nz; z++)
    for (long y = 0; y < s->ny; y++)
      for (long x = 0; x < s->nx; x++) {
        double U[3];
        if (!wall_site(s, x, y, z, U)) continue;
        long n = site_index(s, x, y, z);
        double rho, u[3];
        site_moments(s, s->fs, n, &rho, u);
        for (int a = 0; a < 3; a++) s->wall_dp[a] += rho * (U[a] - u[a]);
        impose_equilibrium(s, n, rho, U);
      }
}

/* ------------------------------------------------------------------------
 * Near-contact closure (not in the paper: it leaves lubrication untreated,
 * section 2.3).  A perceptron 8 -> 64 -> 64 -> 2 with tanh hidden units maps
 * the geometry of a close pair to the force the coarse lattice misses, in
 * units of mu U (2D Stokes forces per unit depth are mu U times a function of
 * the geometry).  Readings of the closure (the library's kernels take the
 * same ones, written separately):
 *  - every pair i < j whose surface gap h = |d| - r_i - r_j is below clo_h
 *    at the start of the step (minimum image); kinematic particles report
 *    the force but keep their velocity, as for the hydrodynamic force;
 *  - inputs: h, (r_i - 9)/3, (r_j - 9)/3, the unit vector n from i to j, the
 *    offset of the gap midpoint x_i + n (r_i + h/2) from its nearest site,
 *    and (tau - 0.7)/0.1; computed in FP64, rounded to FP32 and then FP16;
 *  - outputs (a_n, a_t): force on i = mu U (a_n n + a_t t), t = (-n_y, n_x),
 *    mu = rho0 nu, U = (u_i - u_j).n (approach speed); j takes the opposite;
 *  - the network rounds its inputs, weights and hidden activations to FP16
 *    (nearest even) and sums exactly;
 *  - the closure force joins the hydrodynamic force in the acceleration
 *    substep and in the reported F, before the hard-core collisions.
 * 2D only.
 * ---------------------------------------------------------------------- */

/* Round to the nearest IEEE binary16 value, ties to even (11 significant
 * bits, quantum 2^-24 below the smallest normal, overflow to infinity). */
static double to_half(double x) {
  if (x == 0.0 || x != x) return x;
  double a = fabs(x);
  if (a >= 65520.0) return copysign(INFINITY, x);
  int e;
  frexp(a, &e);
  double q = e >= -13 ? ldexp(1.0, e - 11) : ldexp(1.0, -24);
  return copysign(nearbyint(a / q) * q, x);
}

static double fp32_then_half(double x) { return to_half((double)(float)x); }

static void closure_inputs(const ora_sim *s, const particle *A, const particle *B,
                           const double d[3], double dist, double in[8]) {
  double n[2] = {d[0] / dist, d[1] / dist};
  double h = dist - A->r - B->r;
  double mx = A->x[0] + n[0] * (A->r + 0.5 * h), my = A->x[1] + n[1] * (A->r + 0.5 * h);
  in[0] = h;
  in[1] = (A->r - 9.0) / 3.0;
  in[2] = (B->r - 9.0) / 3.0;
  in[3] = n[0];
  in[4] = n[1];
  in[5] = mx - floor(mx + 0.5);
  in[6] = my - floor(my + 0.5);
  in[7] = (s->tau - 0.7) / 0.1;
}

/* y = tanh(tanh(x W1 + b1) W2 + b2) W3 + b3 at the FP16 rounding points. */
static void closure_net(const double *p, const double in[8], double y[2]) {
  const double *W1 = p, *b1 = p + 512, *W2 = p + 576, *b2 = p + 4672, *W3 = p + 4736, *b3 = p + 4864;
  double x[8], h1[64], h2[64];
  for (int k = 0; k < 8; k++) x[k] = fp32_then_half(in[k]);
  for (int m = 0; m < 64; m++) {
    double z = b1[m];
    for (int k = 0; k < 8; k++) z += x[k] * to_half(W1[k * 64 + m]);
    h1[m] = to_half(tanh(z));
  }
  for (int m = 0; m < 64; m++) {
    double z = b2[m];
    for (int k = 0; k < 64; k++) z += h1[k] * to_half(W2[k * 64 + m]);
    h2[m] = to_half(tanh(z));
  }
  for (int o = 0; o < 2; o++) {
    double z = b3[o];
    for (int k = 0; k < 64; k++) z += h2[k] * to_half(W3[k * 2 + o]);
    y[o] = z;
  }
}

static void closure_forces(ora_sim *s) {
  for (int p = 0; p < s->np; p++)
    for (int a = 0; a < 3; a++) s->Fc[p][a] = 0.0;
  if (!s->closure) return;
  int L[3] = {s->nx, s->ny, s->nz};
  double mu = s->rho0 * (s->tau - 0.5) / 3.0;
  for (int i = 0; i < s->np; i++)
    for (int j = i + 1; j < s->np; j++) {
      particle *A = &s->P[i], *B = &s->P[j];
      double d[3] = {0, 0, 0}, dd = 0;
      for (int a = 0; a < 2; a++) {
        d[a] = min_image(B->x[a] - A->x[a], L[a]);
        dd += d[a] * d[a];
      }
      double dist = sqrt(dd);
      if (!(dist - A->r - B->r < s->clo_h) || dist == 0.0) continue;
      double in[8], y[2];
      closure_inputs(s, A, B, d, dist, in);
      closure_net(s->clo_p, in, y);
      double n[2] = {d[0] / dist, d[1] / dist}, t[2] = {-n[1], n[0]};
      double U = (A->u[0] - B->u[0]) * n[0] + (A->u[1] - B->u[1]) * n[1];
      for (int a = 0; a < 2; a++) {
        double f = mu * U * (y[0] * n[a] + y[1] * t[a]);
        s->Fc[i][a] += f;
        s->Fc[j][a] -= f;
      }
    }
}

/* Second substep (eq. 10-11): the particle takes the opposite change.  The
 * buoyancy-corrected weight is added (the settling runs of section 3 need it
 * though eq. 10 omits it).  Kinematic particles keep their velocities. */
static void accelerate(ora_sim *s, double (*dP)[3], double (*dL)[3]) {
  for (int p = 0; p < s->np; p++) {
    particle *P = &s->P[p];
    for (int a = 0; a < 3; a++) {
      P->F[a] = -dP[p][a] + s->Fc[p][a];
      P->T[a] = -dL[p][a];
    }
    if (!isinf(P->m))
      for (int a = 0; a < 3; a++) P->u[a] = P->u[a] + (P->fext[a] - dP[p][a] + s->Fc[p][a]) / P->m;
    if (!isinf(P->I))
      for (int a = 0; a < 3; a++) P->om[a] = P->om[a] - dL[p][a] / P->I;
  }
}


/* Hard-core collisions (eq. 16-19): in the pair's centre-of-mass frame the
 * normal velocities reverse and the tangential ones are kept; applied as
 * part of the acceleration substep, before translation.  Readings: a pair
 * collides when the predicted centres overlap and approach; pairs are
 * visited once each in lexicographic order; a kinematic particle acts as an
 * infinite mass (the frame is its own); angular velocities are untouched. */
static void collisions(ora_sim *s) {
  int L[3] = {s->nx, s->ny, s->nz};
  for (int i = 0; i < s->np; i++)
    for (int j = i + 1; j < s->np; j++) {
      particle *A = &s->P[i], *B = &s->P[j];
      int infA = isinf(A->m), infB = isinf(B->m);
      if (infA && infB) continue;
      double d[3], dd = 0;
      for (int a = 0; a < 3; a++) {
        d[a] = (B->x[a] + B->u[a]) - (A->x[a] + A->u[a]);
        if (a < s->dim) d[a] = min_image(d[a], L[a]);
        dd += d[a] * d[a];
      }
      double dist = sqrt(dd);
      if (dist > A->r + B->r || dist == 0.0) continue;
      double nrm[3], vn = 0;
      for (int a = 0; a < 3; a++) {
        nrm[a] = d[a] / dist;
        vn += (B->u[a] - A->u[a]) * nrm[a];
      }
      if (!(vn < 0.0)) continue;
      double V[3];
      for (int a = 0; a < 3; a++) {
        if (infA) V[a] = A->u[a];
        else if (infB) V[a] = B->u[a];
        else V[a] = (A->m * A->u[a] + B->m * B->u[a]) / (A->m + B->m);
      }
      particle *pr[2] = {A, B};
      for (int t = 0; t < 2; t++) {
        double wv[3], wn = 0;
        for (int a = 0; a < 3; a++) {
          wv[a] = pr[t]->u[a] - V[a];
          wn += wv[a] * nrm[a];
        }
        for (int a = 0; a < 3; a++)
          pr[t]->u[a] = V[a] + (wv[a] - 2.0 * wn * nrm[a]);
      }
    }
}

/* Hard-core contact with a wall, after the pairs: the wall is an infinite
 * mass moving tangentially, so the particle's normal velocity reverses when
 * its predicted surface reaches the wall's BS layer (1 or n-2) while it
 * approaches.  Kinematic particles keep their velocity.  Particles in id
 * order, axes in order. */
static void wall_collisions(ora_sim *s) {
  if (!s->walls) return;
  int L[3] = {s->nx, s->ny, s->nz};
  for (int p = 0; p < s->np; p++) {
    particle *P = &s->P[p];
    if (isinf(P->m)) continue;
    for (int a = 0; a < s->dim; a++) {
      if (!(s->walls & (1 << a))) continue;
      double xp = P->x[a] + P->u[a];
      if ((xp - P->r <= 1.0 && P->u[a] < 0.0) ||
          (xp + P->r >= (double)(L[a] - 2) && P->u[a] > 0.0))
        P->u[a] = -P->u[a];
    }
  }
}

/* Third substep (eq. 13-15): x_p' = x_p + u_p'; the site sets move with the
 * particle without rotating, so the new map is the template at the nearest
 * integer shift k = [x_p - x_p0]. */
static void translate(ora_sim *s) {
  for (int p = 0; p < s->np; p++) {
    particle *P = &s->P[p];
    for (int a = 0; a < s->dim; a++) {
      P->x[a] = P->x[a] + P->u[a];
      P->k[a] = (int)floor(P->x[a] - P->x0[a] + 0.5);
    }
  }
  raster(s);
}

/* Fourth substep: f^eq(rho_I, u_I') at the internal sites of the new map,
 * u_I' = u_p' + omega_p' x r (eq. 12, same sign reading as eq. 5). */
static void internal_substep(ora_sim *s) {
  for (int a = 0; a < 3; a++) s->leak[a] = 0.0;
  for (int p = 0; p < s->np; p++) {
    particle *P = &s->P[p];
    for (int e = P->nbs; e < P->nbs + P->nis; e++) {
      long n = entry_site(s, P, e);
      if (s->own_p[n] != p || s->own_e[n] != e) continue;
      double rho, uI[3], r[3], wr[3], uIp[3];
      site_moments(s, s->fs, n, &rho, uI);
      lever_arm(P, e, r);
      cross(P->om, r, wr);
      for (int a = 0; a < 3; a++) uIp[a] = P->u[a] + wr[a];
      for (int a = 0; a < 3; a++) s->leak[a] += rho * (uIp[a] - uI[a]);
      impose_equilibrium(s, n, rho, uIp);
    }
  }
}

/* Propagation (left-hand side of eq. 3): f_i(x + c_i) <- f*_i(x). */
static void propagate(ora_sim *s) {
#pragma omp parallel for collapse(2) schedule(static)
  for (int i = 0; i < s->q; i++)
    for (long z = 0; z < s->nz; z++)
      for (long y = 0; y < s->ny; y++)
        for (long x = 0; x < s->nx; x++) {
          long to = site_index(s, wrapi(x + s->c[i][0], s->nx),
                               wrapi(y + s->c[i][1], s->ny),
                               wrapi(z + s->c[i][2], s->nz));
          s->f[i * s->N + to] = s->fs[i * s->N + site_index(s, x, y, z)];
        }
}

void ora_step(ora_sim *s, int nsteps) {
  double(*dP)[3] = (double(*)[3])calloc(s->np > 0 ? s->np : 1, sizeof(double[3]));
  double(*dL)[3] = (double(*)[3])calloc(s->np > 0 ? s->np : 1, sizeof(double[3]));
  for (int t = 0; t < nsteps; t++) {
    collide(s);
    boundary_substep(s, dP, dL);
    wall_substep(s);
    closure_forces(s);
    accelerate(s, dP, dL);
    collisions(s);
    wall_collisions(s);
    translate(s);
    internal_substep(s);
    propagate(s);
    s->step++;
  }
  free(dP);
  free(dL);
}

/* ------------------------------------------------------------------------
 * Read-out
 * ---------------------------------------------------------------------- */
void ora_forces(const ora_sim *s, double *F, double *T, double *x, double *u,
                double *omega) {
  for (int p = 0; p < s->np; p++)
    for (int a = 0; a < 3; a++) {
      if (F) F[3 * p + a] = s->P[p].F[a];
      if (T) T[3 * p + a] = s->P[p].T[a];
      if (x) x[3 * p + a] = s->P[p].x[a];
      if (u) u[3 * p + a] = s->P[p].u[a];
      if (omega) omega[3 * p + a] = s->P[p].om[a];
    }
}

void ora_fields(const ora_sim *s, double *rho, double *u, int32_t *owner) {
#pragma omp parallel for schedule(static)
  for (long n = 0; n < s->N; n++) {
    double r, v[3];
    site_moments(s, s->f, n, &r, v);
    if (rho) rho[n] = r;
    if (u)
      for (int a = 0; a < 3; a++) u[3 * n + a] = v[a];
    if (owner) owner[n] = s->own_p[n];
  }
}

void ora_site_kind(const ora_sim *s, int8_t *kind) {
  for (long n = 0; n < s->N; n++) {
    int p = s->own_p[n];
    kind[n] = p < 0 ? 0 : (s->own_e[n] < s->P[p].nbs ? 1 : 2);
  }
}

void ora_shifts(const ora_sim *s, int32_t *k) {
  for (int p = 0; p < s->np; p++)
    for (int a = 0; a < 3; a++) k[3 * p + a] = s->P[p].k[a];
}

void ora_get_f(const ora_sim *s, double *f) {
  memcpy(f, s->f, sizeof(double) * s->q * s->N);
}

void ora_set_f(ora_sim *s, const double *f) {
  memcpy(s->f, f, sizeof(double) * s->q * s->N);
}

void ora_get_fs(const ora_sim *s, double *fs) {
  memcpy(fs, s->fs, sizeof(double) * s->q * s->N);
}

int ora_template(const ora_sim *s, int p, int32_t *nbs, int32_t *nis,
                 int32_t *off, int8_t *kind) {
  if (p < 0 || p >= s->np) return -1;
  const particle *P = &s->P[p];
  if (nbs) *nbs = P->nbs;
  if (nis) *nis = P->nis;
  for (int e = 0; e < P->nbs + P->nis; e++) {
    if (off)
      for (int a = 0; a < 3; a++) off[3 * e + a] = P->off[3 * e + a];
    if (kind) kind[e] = e < P->nbs ? 1 : 2;
  }
  return 0;
}

void ora_diagnostics(const ora_sim *s, double *d) {
  double mass = 0, J[3] = {0, 0, 0};
  for (int i = 0; i < s->q; i++)
    for (long n = 0; n < s->N; n++) {
      double v = s->f[i * s->N + n];
      mass += v;
      for (int a = 0; a < 3; a++) J[a] += v * s->c[i][a];
    }
  d[0] = mass;
  for (int a = 0; a < 3; a++) d[1 + a] = J[a];
  for (int a = 0; a < 3; a++) d[4 + a] = s->leak[a];
  d[7] = (double)s->conflicts;
  double frag = INFINITY, gap = INFINITY;
  int L[3] = {s->nx, s->ny, s->nz};
  for (int p = 0; p < s->np; p++) {
    for (int a = 0; a < s->dim; a++) {
      double disp = s->P[p].x[a] - s->P[p].x0[a];
      double t = disp - floor(disp);
      double dist = fabs(t - 0.5);
      if (dist < frag) frag = dist;
    }
    for (int j = p + 1; j < s->np; j++) {
      double dd = 0;
      for (int a = 0; a < s->dim; a++) {
        double v = min_image(s->P[j].x[a] - s->P[p].x[a], L[a]);
        dd += v * v;
      }
      double g = sqrt(dd) - s->P[p].r - s->P[j].r;
      if (g < gap) gap = g;
    }
  }
  d[8] = frag;
  d[9] = gap;
  d[10] = (double)s->step;
  for (int a = 0; a < 3; a++) d[11 + a] = s->fb[a];
  for (int a = 0; a < 3; a++) d[14 + a] = s->wall_dp[a];
}

int ora_set_closure(ora_sim *s, const double *params, double h_max) {
  if (s->dim != 2 || !(h_max >= 0.0)) return -1;
  s->closure = params != NULL && h_max > 0.0;
  if (params)
    for (int k = 0; k < 4866; k++) s->clo_p[k] = (double)(float)params[k];
  s->clo_h = h_max;
  return 0;
}

double ora_half(double x) { return to_half(x); }

int ora_closure_inputs(const ora_sim *s, int i, int j, double *in) {
  if (i < 0 || j < 0 || i >= s->np || j >= s->np || i == j) return -1;
  int L[3] = {s->nx, s->ny, s->nz};
  double d[3] = {0, 0, 0}, dd = 0;
  for (int a = 0; a < 2; a++) {
    d[a] = min_image(s->P[j].x[a] - s->P[i].x[a], L[a]);
    dd += d[a] * d[a];
  }
  closure_inputs(s, &s->P[i], &s->P[j], d, sqrt(dd), in);
  return 0;
}

int ora_closure_net(const double *params, const double *in, double *y) {
  double p[4866];
  for (int k = 0; k < 4866; k++) p[k] = (double)(float)params[k];
  closure_net(p, in, y);
  return 0;
}

int ora_set_walls(ora_sim *s, int walls, const double *wall_u) {
  int L[3] = {s->nx, s->ny, s->nz};
  if (walls < 0 || walls >= (1 << s->dim) || s->np > 0) return -1;
  for (int a = 0; a < 3; a++)
    for (int side = 0; side < 2; side++)
      for (int b = 0; b < 3; b++) {
        double v = wall_u ? wall_u[6 * a + 3 * side + b] : 0.0;
        if (!(walls & (1 << a))) v = 0.0;
        if (b == a && v != 0.0) return -1; /* walls move tangentially only */
        s->wall_u[a][side][b] = v;
      }
  for (int a = 0; a < s->dim; a++)
    if ((walls & (1 << a)) && L[a] < 5) return -1;
  s->walls = walls;
  return 0;
}

/* ------------------------------------------------------------------------
 * Threads of the per-site loops (results do not depend on the count).
 * ---------------------------------------------------------------------- */
void ora_set_threads(int n) { omp_set_num_threads(n > 0 ? n : omp_get_num_procs()); }

int ora_threads(void) { return omp_get_max_threads(); }
