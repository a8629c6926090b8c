/*
 * FP64 CPU oracle of the site-based suspension lattice Boltzmann method
 * (dos Santos & Philippi, "An alternative method for simulating particle
 * suspensions using lattice Boltzmann").
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously-correct
 * reference that the GPU path is checked against.  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the GPU library.
 *
 * Lattice units: dx = dt = 1, c_s^2 = 1/3.  Distributions are stored as plain
 * f (not deviations), layout [q][nz][ny][nx], x fastest.  Velocity ordering:
 *   D2Q9 : 0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1) 5:(1,1) 6:(-1,1)
 *          7:(-1,-1) 8:(1,-1)
 *   D3Q19: 0:(0,0,0) 1:(1,0,0) 2:(-1,0,0) 3:(0,1,0) 4:(0,-1,0) 5:(0,0,1)
 *          6:(0,0,-1) 7:(1,1,0) 8:(-1,-1,0) 9:(1,-1,0) 10:(-1,1,0)
 *          11:(1,0,1) 12:(-1,0,-1) 13:(1,0,-1) 14:(-1,0,1) 15:(0,1,1)
 *          16:(0,-1,-1) 17:(0,1,-1) 18:(0,-1,1)
 * Particle vectors are [n][3] FP64; in 2D z components are 0 and the angular
 * velocity / torque live in component 2.
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ora_sim ora_sim;

/* Velocity set and weights of a lattice (q = 9 or 19).  c is [q][3]. */
int ora_lattice(int q, int32_t *c, double *w);

/* Equilibrium distribution (second-order Hermite form) at one site. */
void ora_feq(int q, double rho, const double u[3], double *feq);

/* Create a periodic box.  Initial state f_i = w_i rho0 (fluid at rest). */
ora_sim *ora_create(int q, int nx, int ny, int nz, double tau, double rho0,
                    const double gravity[3], const double body_force[3],
                    int zero_net_force);
void ora_destroy(ora_sim *s);

/* Append n particles (ids continue from the current count).  mass and
 * inertia may be +INFINITY for a kinematic particle with imposed velocity.
 * Returns the first id, or -1 on invalid input. */
int ora_add_particles(ora_sim *s, int n, const double *x, const double *u,
                      const double *omega, const double *radius,
                      const double *mass, const double *inertia);

/* Advance nsteps full time steps. */
void ora_step(ora_sim *s, int nsteps);

/* Last step's hydrodynamic force F = -dP and torque T = -dL, and the
 * current particle state.  Any pointer may be NULL. */
void ora_forces(const ora_sim *s, double *F, double *T, double *x, double *u,
                double *omega);

/* Density, velocity [N][3] of the current post-propagation state and the
 * owner id of every BS/IS site (-1 elsewhere).  Any pointer may be NULL. */
void ora_fields(const ora_sim *s, double *rho, double *u, int32_t *owner);

/* Site kind in the current map: 0 none, 1 BS, 2 IS. */
void ora_site_kind(const ora_sim *s, int8_t *kind);

/* Integer shift k of every particle, [n][3]. */
void ora_shifts(const ora_sim *s, int32_t *k);

/* Raw distributions [q][N] (post-propagation state). */
void ora_get_f(const ora_sim *s, double *f);
void ora_set_f(ora_sim *s, const double *f);

/* Post-collision, post-substep distributions of the last step [q][N]: the
 * array propagation read from. */
void ora_get_fs(const ora_sim *s, double *fs);

/* Template of particle p: number of BS and IS entries; offsets [n][3] and
 * kinds (1 BS, 2 IS) in template order if the pointers are non-NULL. */
int ora_template(const ora_sim *s, int p, int32_t *nbs, int32_t *nis,
                 int32_t *off, int8_t *kind);

/* Diagnostics (not part of the result):
 *  d[0] total mass, d[1..3] total fluid momentum,
 *  d[4..6] IS momentum leak of the last step,
 *  d[7] raster conflicts in the current map,
 *  d[8] smallest distance of any displacement component to a half integer,
 *  d[9] smallest surface gap between two particles,
 *  d[10] step counter,
 *  d[11..13] fluid body force density applied each step,
 *  d[14..16] momentum the walls gave the fluid in the last step. */
void ora_diagnostics(const ora_sim *s, double *d);

/* Close the box along the axes in the bit mask `walls` (bit 0 x, 1 y, 2 z)
 * with immobile site-based wall layers: on a closed axis of n sites, layers
 * 0, 1, n-2, n-1 are wall sites and 2 .. n-3 fluid.  wall_u is
 * [axis][low, high][3] (NULL = at rest); the component along the axis must
 * be 0.  Call before adding particles.  Returns 0, or -1 on invalid input. */
int ora_set_walls(ora_sim *s, int walls, const double *wall_u);

/* Near-contact closure network (2D): params are the 4866 network parameters
 * (W1 [8][64], b1, W2 [64][64], b2, W3 [64][2], b3; taken as FP32 values),
 * h_max the gap below which it acts (0 or params NULL: off).  Returns 0, or
 * -1 for a 3D box or a negative h_max. */
int ora_set_closure(ora_sim *s, const double *params, double h_max);

/* The closure's 8 inputs for particles i, j at the current positions, and
 * the network alone on given inputs (its FP16 rounding points included). */
int ora_closure_inputs(const ora_sim *s, int i, int j, double *in);
int ora_closure_net(const double *params, const double *in, double *y);

/* Nearest IEEE binary16 value (ties to even). */
double ora_half(double x);

int ora_num_particles(const ora_sim *s);

/* Threads the per-site loops use (n <= 0: one per processor), and the
 * current count.  Results are identical for every count. */
void ora_set_threads(int n);
int ora_threads(void);

#ifdef __cplusplus
}
#endif
#endif
