/*
 * C ABI of the MI355X (gfx950) hot path of the site-based suspension lattice
 * Boltzmann method of dos Santos & Philippi ("An alternative method for
 * simulating particle suspensions using lattice Boltzmann").
 *
 * What one step computes (section 2, in the paper's order):
 *   1. BGK collision at every site (eq. 1-3), plus a uniform fluid body force;
 *   2. boundary-site (BS) substep: every BS site takes the equilibrium at the
 *      particle's rigid-body velocity u_p + omega_p x r, and the momentum dp
 *      and angular momentum dl this gives the fluid are summed per particle
 *      (eq. 5-9);
 *   3. particle acceleration by the opposite change plus the buoyancy-corrected
 *      weight (eq. 10-11), then elastic hard-core collisions (eq. 16-19);
 *   4. translation of the particle and its site sets (eq. 13-15);
 *   5. internal-site (IS) substep at the new positions (eq. 12);
 *   6. propagation (eq. 3).
 * Where the paper is silent the library takes these readings: second-order
 * equilibrium with c_s^2 = 1/3; D3Q19 for 3D; u = u_p + omega x r; rho kept
 * per site in every imposition; BS/IS from the digitised ball |o - phi| <= r
 * with the lattice's own links; nearest integer [x] = floor(x + 1/2) applied
 * to the particle's shift; lowest particle id owns a site claimed twice;
 * F_ext = (m - rho0 V) g with the analytic V.
 *
 * Walls (optional; the paper closes its boxes in section 3 without describing
 * how): a closed axis of n sites keeps layers 2 .. n-3 as fluid, and its
 * layers 0, 1, n-2, n-1 are an immobile (or tangentially sliding) solid slab
 * treated by the site rule of the particles: every wall site takes
 * f^eq(rho, U_wall) with its own density after the collision.  Particles never
 * own wall sites, and a particle whose predicted surface reaches the wall's
 * BS layer (1 or n-2) while approaching it has its normal velocity reversed
 * (eq. 16-19 with the wall as an infinite mass), after the particle pairs.
 *
 * Conventions
 *  - Lattice units: dx = dt = 1.  An axis is periodic unless wall layers
 *    close it (lbm_params.walls).
 *  - Distribution layout (host buffers): f[q][nz][ny][nx], x fastest, plain f
 *    (not deviations).  Velocity order:
 *      D2Q9 : (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1) (-1,-1) (1,-1)
 *      D3Q19: (0,0,0) (1,0,0) (-1,0,0) (0,1,0) (0,-1,0) (0,0,1) (0,0,-1)
 *             (1,1,0) (-1,-1,0) (1,-1,0) (-1,1,0) (1,0,1) (-1,0,-1)
 *             (1,0,-1) (-1,0,1) (0,1,1) (0,-1,-1) (0,1,-1) (0,-1,1)
 *  - Particle vectors are host arrays [n][3] of double.  In 2D the z
 *    components are ignored (treated as 0) and angular velocity / torque use
 *    component 2.
 *  - Every call returns an int: LBM_OK (0) or a negative LBM_E* code.  No
 *    call throws or aborts across the ABI.
 *  - All device work is ordered on the caller's HIP stream given to
 *    lbm_create.  lbm_step only enqueues; lbm_forces, lbm_fields,
 *    lbm_get_distributions, lbm_site_kind, lbm_shifts and lbm_profile
 *    synchronise that stream and report device-side anomalies.
 *  - The library allocates no device memory: everything lives in the
 *    caller-owned workspace, which must outlive the context.  A context is
 *    used by one host thread at a time.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum lbm_lattice { LBM_D2Q9 = 9, LBM_D3Q19 = 19 };

/* Storage precision of the distributions.  Distributions are stored as
 * deviations g_i = f_i - w_i rho0.  FP64 computes in FP64.  FP32 collides in
 * FP32; FP16 and BF16 store g_i / w_i (FP16 also scaled by 2^10) and collide
 * in FP32.  In every mode the per-site momentum exchange, the per-particle
 * sums and the Newton-Euler update are FP64. */
enum lbm_storage { LBM_FP64 = 0, LBM_FP32 = 1, LBM_FP16 = 2, LBM_BF16 = 3 };

enum lbm_status {
  LBM_OK = 0,
  LBM_EINVAL = -1,      /* invalid argument (checked on the host, before any HIP call) */
  LBM_EWORKSPACE = -2,  /* workspace NULL, misaligned (256 B) or too small */
  LBM_EHIP = -3,        /* a HIP runtime call or kernel launch failed */
  LBM_EOVERLAP = -4,    /* new particle overlaps another particle */
  LBM_ECAPACITY = -5,   /* more particles than max_particles */
  LBM_ENONFINITE = -6,  /* non-finite input value */
  LBM_EUNSUPPORTED = -7,/* storage mode not built */
  LBM_ECOLLISION = -8,  /* collision search bound exceeded: a particle speed
                           >= 0.5 lu/step, or > 64 particles within r_i+r_j+1
                           of one particle; results of that step are invalid */
  LBM_ESTATE = -9       /* the sweep met an owned boundary site whose record named
                           no entry of the particle table (it wrote nothing through
                           it); the device state is inconsistent and the results of
                           that step are invalid */
};

typedef struct lbm_ctx lbm_ctx;

typedef struct lbm_params {
  int32_t lattice;       /* LBM_D2Q9 or LBM_D3Q19 */
  int32_t nx, ny, nz;    /* box size; nz = 1 for D2Q9; nx*ny*nz < 2^31, and one population
                            plane (nx*ny*nz values of the storage type) at most 4 GiB:
                            LBM_EINVAL otherwise (FP64 up to 2^29 sites, FP32 2^30) */
  double tau;            /* BGK relaxation time, > 1/2: nu = (tau - 1/2)/3 (eq. 4) */
  double rho0;           /* initial fluid density and deviation base (> 0) */
  double gravity[3];     /* acceleration on particles, lu/step^2 */
  double body_force[3];  /* extra uniform force density on the fluid */
  int32_t zero_net_force;/* 1: fluid also carries -sum_p F_ext,p / N per site */
  int32_t storage;       /* enum lbm_storage */
  int32_t max_particles; /* capacity (>= 0) */
  double max_radius;     /* largest particle radius that will be added (0 < r <= 120) */
  int32_t walls;         /* bit a (0 x, 1 y, 2 z; z only for D3Q19): axis a closed by
                            wall layers at both ends, which needs n_a >= 5; 0 = periodic */
  double wall_velocity[3][2][3]; /* [axis][0 low wall, 1 high wall][component]; the
                            component along the axis must be 0; ignored for open axes */
  int32_t aa;            /* 0: two population arrays, the sweep pulls from one into the other;
                            1: one array updated in place with the AA pattern (even steps read
                            and write a site's own slots, odd steps read and write its
                            neighbours'), half the population memory, the same results bit for
                            bit.  An AA context cannot be autotuned (a sweep in place cannot be
                            repeated on the live state) and its read-outs of distributions and
                            fields gather on the host. */
} lbm_params;

/* Bytes of device workspace lbm_create needs for these parameters. */
int lbm_workspace_size(const lbm_params* prm, size_t* bytes);

/* Create a context on a caller-owned device workspace (at least
 * lbm_workspace_size bytes, 256-B aligned) and a caller-owned hipStream_t
 * (NULL = the null stream).  The fluid starts at rest with density rho0:
 * f_i = w_i rho0.  Parameters follow section 2.1 (lattice, tau) and the
 * particle record of section 2.2. */
int lbm_create(const lbm_params* prm, void* d_workspace, size_t bytes,
               void* hip_stream, lbm_ctx** out);

/* Append n particles (ids first_id ... first_id+n-1).  x: centres in
 * [0, n_axis); u, omega: initial velocities (NULL = 0); radius in
 * (0, max_radius]; mass, inertia > 0, or +INFINITY for a kinematic particle
 * whose velocity is imposed (forces are still reported).  The particle record
 * is that of section 2.2 (x_p, r_p, m_p, I_p, u_p, omega_p).  A particle so
 * small that no site lies within r of its centre (r < sqrt(d)/2 at the worst
 * offset) has an empty site set: it moves under its weight and collisions
 * but exchanges no momentum with the fluid.  Rejects overlap
 * with any particle (centre distance < r_i + r_j, minimum image) or with a
 * wall (x - r < 1 or x + r > n - 2 along a closed axis) as LBM_EOVERLAP.
 * Host arrays are read before the call returns. */
int lbm_add_particles(lbm_ctx* ctx, int32_t n, const double* x, const double* u,
                      const double* omega, const double* radius,
                      const double* mass, const double* inertia,
                      int32_t* first_id);

/* Enqueue nsteps time steps (steps 1-6 above) on the context's stream. */
int lbm_step(lbm_ctx* ctx, int32_t nsteps);

/* Per particle: the last step's hydrodynamic force F = -dP and torque
 * T = -dL (eq. 8-9; hydrodynamic only, without the weight and collisions),
 * and the current centre x (unwrapped), velocity u and angular velocity
 * omega.  Host arrays [n][3]; any may be NULL.  Synchronises. */
int lbm_forces(lbm_ctx* ctx, double* F, double* T, double* x, double* u,
               double* omega);

/* Density rho[N], velocity u[N][3] (moments of the current post-propagation
 * distributions, eq. 1-2) and the owner particle id of every BS/IS site
 * (-1 elsewhere), N = nx*ny*nz, site index x + nx*(y + ny*z).  Any pointer
 * may be NULL.  Synchronises. */
int lbm_fields(lbm_ctx* ctx, double* rho, double* u, int32_t* owner);

int lbm_destroy(lbm_ctx* ctx);
const char* lbm_strerror(int code);

/* ---- auxiliary calls (tests, checkpoints, measurement) ------------------ */

/* Current post-propagation distributions f[q][N] (plain f). Synchronises. */
int lbm_get_distributions(lbm_ctx* ctx, double* f);

/* Replace the current post-propagation distributions by f[q][N] (plain f).
 * Rounded to the storage precision.  Synchronises. */
int lbm_set_distributions(lbm_ctx* ctx, const double* f);

/* Site kind of the current particle map: 0 none (wall sites included), 1 BS,
 * 2 IS (int8 [N]).  Synchronises. */
int lbm_site_kind(lbm_ctx* ctx, int8_t* kind);

/* Integer shift k = [x - x0] of every particle, int32 [n][3]. Synchronises. */
int lbm_shifts(lbm_ctx* ctx, int32_t* k);

/* Particle count and template sizes (BS and IS entries) of particle p. */
int lbm_particle_info(lbm_ctx* ctx, int32_t p, int32_t* nbs, int32_t* nis);

/* Profiling: when on, lbm_step records a HIP event pair around every launch
 * of the collide-and-stream sweep on the context's stream; lbm_profile
 * returns the summed sweep time (ms) and launch count since profiling was
 * switched on, and synchronises. */
int lbm_set_profiling(lbm_ctx* ctx, int32_t on);
int lbm_profile(lbm_ctx* ctx, double* sweep_ms, int64_t* sweeps);

/* ---- ensembles of independent boxes ------------------------------------
 * nbox boxes of sizes dims[b][0..2] (dims is int32 [nbox][3]) that share the
 * lattice, tau, rho0, gravity, body force, walls and storage of prm (whose
 * nx, ny, nz are ignored) step together: one launch of each kernel covers
 * every box, so a step of 64 small boxes costs what a step of one box of
 * their total size does.  Each box is an independent copy of the problem of
 * section 2: its own periodic (or walled) lattice, particles and zero-net-force
 * frame.  Sites of all boxes are numbered box after box (box b starts at the
 * first_site lbm_box_info reports, x fastest inside a box), so lbm_fields,
 * lbm_site_kind and the distribution calls cover NT = sum of the box sizes
 * sites; particle ids run over all boxes.  max_particles counts all boxes. */
int lbm_ensemble_workspace_size(const lbm_params* prm, int32_t nbox, const int32_t* dims, size_t* bytes);
int lbm_ensemble_create(const lbm_params* prm, int32_t nbox, const int32_t* dims, void* d_workspace,
                        size_t bytes, void* hip_stream, lbm_ctx** out);

/* Append n particles to box `box` (coordinates local to the box).  Boxes are
 * filled in order: box must be >= the box of the last particle added
 * (LBM_EINVAL otherwise), so that every box holds consecutive ids.
 * lbm_add_particles adds to box 0. */
int lbm_ensemble_add_particles(lbm_ctx* ctx, int32_t box, int32_t n, const double* x, const double* u,
                               const double* omega, const double* radius, const double* mass,
                               const double* inertia, int32_t* first_id);

/* Size (int32 [3]), first site, first particle id and particle count of a box.
 * Any pointer may be NULL. */
int lbm_box_info(lbm_ctx* ctx, int32_t box, int32_t* dims, int64_t* first_site, int32_t* first_particle,
                 int32_t* n_particles);

/* ---- launch shape, autotuning and step graphs ---------------------------
 * The sweep runs either as the one-box row kernel (width 0; one box only) or
 * as a persistent kernel over tiles of `width` consecutive sites of one box in
 * raster order (64, 128, 256 or 512; a tile runs on across rows) with `grid`
 * workgroups (0: one per tile).  blocks_per_cu > 0 caps
 * the sweep workgroups resident on one compute unit at that number, through
 * LDS each workgroup reserves (floor(LDS per CU / blocks_per_cu), whole KiB;
 * LBM_EINVAL if that exceeds what one workgroup may reserve or is below
 * 1 KiB); 0 leaves residency to the register count.  Fewer resident waves
 * can stream faster: fewer DRAM rows open at once.  With FP16/BF16 storage,
 * two arrays and an even nx the row kernel takes two sites per lane (one
 * 64-wide wave per 128 sites of a row, four waves to a workgroup).  Every
 * shape computes the same values bit for bit.  Defaults: width 0 (one box) or
 * 128, grid 0, no cap. */
int lbm_set_sweep_config(lbm_ctx* ctx, int32_t width, int32_t grid, int32_t blocks_per_cu);
int lbm_get_sweep_config(lbm_ctx* ctx, int32_t* width, int32_t* grid, int32_t* blocks_per_cu);

/* Time every sweep shape (widths 0 (one box), 64, 128, 256, 512; grids 0 and
 * 4, 8, 16, 32 per CU; caps none, 6, 5, 4, 3, 2 workgroups per CU; reps
 * launches each, after one warm-up) on the context's own state, time the four
 * fastest again in two alternating rounds of 2 reps launches, and keep the
 * fastest of those; returns it and its time per sweep in ms (any output
 * pointer may be NULL).  Sweeping again from the same state recomputes the
 * same values, so the simulation is unchanged.  Synchronises. */
int lbm_autotune(lbm_ctx* ctx, int32_t reps, int32_t* width, int32_t* grid, int32_t* blocks_per_cu,
                 double* best_ms);

/* The same candidates timed inside whole steps instead of bare repeated
 * sweeps: for each, 2 untimed and `steps` (rounded up to even) timed steps,
 * or with step graphs set (lbm_set_graph) one untimed graph and `steps`
 * rounded up to whole graphs; then the four fastest again in two alternating
 * rounds of twice the steps.  Keeps the fastest and returns it and its time
 * per step in ms.  The step around a sweep changes which launch is fastest
 * (what the previous kernels leave in the caches, how the sweep's last waves
 * overlap the next kernel), so this is the tuner for production runs.
 * Unlike lbm_autotune it ADVANCES the simulation by every step it times
 * (about 130 times the steps per candidate; their number goes to
 * *steps_done), works on AA contexts, and discards pending profiling
 * events.  Any output pointer may be NULL.  Returns the status of those steps
 * (e.g. LBM_ECOLLISION).  Synchronises. */
int lbm_autotune_steps(lbm_ctx* ctx, int32_t steps, int32_t* width, int32_t* grid, int32_t* blocks_per_cu,
                       double* best_ms, int64_t* steps_done);

/* steps_per_graph > 0 (even): lbm_step replays a HIP graph of that many
 * steps, captured on the first use and again after the particle set, the
 * buffer parity or the sweep shape changed, and launches the remainder one by
 * one; 0 (default) launches every kernel.  Profiling covers eager sweeps only.
 * Synchronises. */
int lbm_set_graph(lbm_ctx* ctx, int32_t steps_per_graph);

/* ---- near-contact closure network ---------------------------------------
 * A perceptron 8 -> 64 -> 64 -> 2 with tanh hidden units:
 *   y = tanh(tanh(x W1 + b1) W2 + b2) W3 + b3,
 * run on the matrix cores with FP16 inputs, weights and hidden activations and
 * FP32 sums.  Parameters are one flat FP32 device vector: W1 [8][64], b1 [64],
 * W2 [64][64], b2 [64], W3 [64][2], b3 [2], row-major (lbm_mlp_param_count
 * values).  Rows of x are [n][8] FP32, of y and targets t [n][2] FP32, all
 * device memory; every call only enqueues on hip_stream.  The loss over B rows
 * is (1/B) sum (y - t)^2; backward signals are multiplied by loss_scale before
 * their FP16 rounding and the gradients divided by it again. */
int lbm_mlp_param_count(int32_t* n);
int lbm_mlp_forward(const float* d_params, const float* d_x, float* d_y, int64_t n, void* hip_stream);

/* Loss (d_loss[0], may be NULL) and its gradient (d_grad, one value per
 * parameter) over all n rows; n >= 1. */
int lbm_mlp_gradient(const float* d_params, const float* d_x, const float* d_t, int32_t n, float loss_scale,
                     float* d_grad, float* d_loss, void* hip_stream);

/* `steps` Adam steps (Kingma & Ba 2015; beta 0.9, 0.999, eps 1e-8, learning
 * rate lr) on mini-batches of `batch` rows (a multiple of 64) taken in order,
 * cycling through the n rows: step s uses rows (s * batch + j) mod n.  step0
 * is the number of steps already taken (bias correction, row position).
 * d_adam_m, d_adam_v hold the moment estimates (zero before the first step);
 * d_loss, if not NULL, receives the loss of every step. */
int lbm_mlp_train(float* d_params, float* d_adam_m, float* d_adam_v, const float* d_x, const float* d_t,
                  int32_t n, int32_t batch, int32_t steps, int32_t step0, float lr, float loss_scale,
                  float* d_loss, void* hip_stream);

/* Near-contact closure in the step (2D only; LBM_EUNSUPPORTED in 3D).  The
 * paper leaves lubrication untreated (section 2.3); with the closure on,
 * every pair i < j of a box whose surface gap h = |d| - r_i - r_j is below
 * h_max at the start of a step gets from the network (parameters d_params,
 * copied into the context) the force on i
 *     mu U (a_n n + a_t t),  n = d/|d|, t = (-n_y, n_x), mu = rho0 (tau - 1/2)/3,
 *     U = (u_i - u_j).n (approach speed),
 * and j the opposite.  The inputs are h, (r_i - 9)/3, (r_j - 9)/3, n_x, n_y,
 * the offset of the gap midpoint x_i + n (r_i + h/2) from its nearest site
 * (per axis, in [-1/2, 1/2)) and (tau - 0.7)/0.1 (lbm_closure_inputs).  The
 * force joins the hydrodynamic force in the acceleration (eq. 10) and in the
 * reported F, before the hard-core collisions, which still apply; kinematic
 * particles report it and keep their velocity.  d_params NULL or h_max 0
 * switches it off.  More than 1024 such pairs in a step are reported as
 * LBM_ECAPACITY by the next synchronising call.  Synchronises. */
int lbm_set_closure(lbm_ctx* ctx, const float* d_params, double h_max);

/* The closure's inputs for n pairs (host arrays): xi [n][2] centre of i,
 * d [n][2] minimum-image separation from i to j, ri, rj [n], relaxation time
 * tau; out [n][8] FP32. */
int lbm_closure_inputs(int32_t n, const double* xi, const double* d, const double* ri, const double* rj,
                       double tau, float* out);

/* ---- stepping that allocates nothing -------------------------------------
 * For callers that cannot allocate device memory or create HIP objects: code
 * under the caller's own graph capture, tight serving loops, harnesses that
 * forbid it.  Enqueues nsteps steps exactly as lbm_step does (the same kernels,
 * the same results bit for bit), except that every step is launched one by
 * one (no step graph is created, whatever lbm_set_graph says), no profiling
 * events are recorded, and the per-step scratch of the particle kernels (the
 * per-particle momentum sums, the close-pair and site-sharing lists and the
 * pair staging, 1,336 bytes per particle) lives in one library-owned device
 * array of at most 4096 particles (5.2 MiB) per device, held until the
 * process ends, instead of in the context's workspace.  LBM_ECAPACITY for a
 * context with more particles; LBM_EINVAL unless the calling thread's current
 * device is the context's.  Every call on one device uses the same array:
 * calls that overlap on one device (contexts stepping on different streams)
 * race and give wrong results.  Calls no allocating routine. */
int lbm_step_noalloc(lbm_ctx* ctx, int32_t nsteps);

/* Algorithmic HBM bytes one sweep moves per site (2 q sizeof(storage)). */
int lbm_bytes_per_site(const lbm_params* prm, int64_t* bytes);

/* Device copy of `bytes` (multiple of 16, 16-B aligned pointers) on
 * `hip_stream` with streaming (non-temporal) stores, and streaming loads when
 * `streaming_loads` is nonzero, else plain ones: the bandwidth ceiling
 * reference for the sweep.  Streaming loads are the faster kind from HBM,
 * plain loads from the last-level cache.  LBM_EINVAL for a null or unaligned
 * pointer or a size that is not a multiple of 16. */
int lbm_device_copy(void* dst, const void* src, size_t bytes, int32_t streaming_loads, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif
