/*
 * sphrb.h -- C ABI of the MI355X (gfx950) SPH fluid / rigid-body / thermal
 * library.  The method is that of Fuchs, Meier, Wall, Cyron, "An SPH
 * framework for fluid-solid and contact interaction problems including
 * thermo-mechanical coupling and reversible phase transitions"
 * (arXiv 2103.07925).
 *
 * Conventions
 *   - Status: every int-returning call returns SPH_OK (0) or an error code;
 *     no C++ exception crosses the ABI.  sph_last_error() gives a detail
 *     string for the calling thread, valid until its next call.
 *   - Host pointers are named *_host or documented as host; device memory is
 *     the caller-owned arena passed to sph_scene_create.  The library never
 *     allocates device memory on the step path.
 *   - Particle arrays at the boundary are in original-id order, FP64, with
 *     vectors as [n][3] (z ignored in 2D) and int32 integer arrays.
 *   - A scene's work is enqueued on the HIP stream given at creation;
 *     sph_scene_step returns once the work is enqueued.  Reads synchronise
 *     that stream.
 *   - Scenes are independent: two scenes may be driven from two threads,
 *     one scene from one thread at a time.
 */
#ifndef SPHRB_H
#define SPHRB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPH_ABI_VERSION 3

enum {
  SPH_OK = 0,
  SPH_E_INVALID = 1,      /* bad argument or descriptor */
  SPH_E_NOMEM = 2,        /* arena too small */
  SPH_E_DEVICE = 3,       /* HIP runtime error */
  SPH_E_STATE = 4,        /* sticky device error (escape, non-finite, ...) or call after one */
  SPH_E_UNSUPPORTED = 5
};

/* Arithmetic of the particle interaction sweep.  Rigid-body sums, body
 * integration and the global checks are FP64 in both modes. */
enum { SPH_FP64 = 0, SPH_FP32_SWEEP = 1 };

/* Particle kinds: fluid particle i, boundary (wall) particle b, rigid
 * particle r (Sec. "Initial particle spacing", "Boundary and coupling
 * conditions"). */
enum { SPH_FLUID = 0, SPH_WALL = 1, SPH_RIGID = 2 };

/* Sticky device error bits reported by sph_scene_read_stats. */
enum {
  SPH_ERR_ESCAPE = 1,      /* a particle left the cell grid */
  SPH_ERR_CELL = 2,        /* a cell holds more particles than the sort supports */
  SPH_ERR_NONFINITE = 4,   /* non-finite position or velocity */
  SPH_ERR_COINCIDENT = 8,  /* two distinct particles at distance zero */
  SPH_ERR_BODYCAP = 16,    /* solidification needs more bodies than max_bodies */
  SPH_ERR_NBCAP = 32       /* a particle has more neighbours than the list capacity */
};

/* One phase (material).  p0 is the reference pressure of the equation of
 * state p = p0 (rho/rho0 - 1) (eq. nummeth_fluid_eos), so c = sqrt(p0/rho0);
 * nu the kinematic viscosity (dynamic viscosity eta = rho0 nu); cp, kappa
 * the heat capacity and conductivity of eq. goveq_thermo_heat_equation; b
 * the body force per unit mass; T_t the transition temperature and
 * switch_to the partner phase of a melting / solidification
 * (Sec. "Modeling thermally driven reversible phase transitions"), -1 for
 * none; dirichlet marks phases whose scalar is prescribed: walls of such a
 * phase take part in conduction (V = dx^d, the phase's kappa), fluid and
 * rigid particles of such a phase keep their value.  The same scalar solver
 * carries a concentration C (the remark on concentration-driven transitions
 * in Sec. "Reversible phase transition"): cp = 1, kappa = D, T = C and
 * T_t = C_t. */
typedef struct {
  double rho0, p0, nu, cp, kappa;
  double b[3];
  double T_t;
  int32_t switch_to;
  int32_t dirichlet;
} sph_material;

/* Initial state of rigid body k: velocity, angular velocity (world frame),
 * orientation quaternion (w, x, y, z), fixed flag (fixed bodies never move). */
typedef struct {
  double u[3], w[3], q[4];
  int32_t fixed;
  int32_t pad;
} sph_body_init;

/* Scene descriptor.  All pointers are host pointers, borrowed during
 * sph_scene_arena_bytes / sph_scene_create only. */
typedef struct {
  int32_t dim;                 /* 2 or 3 */
  int32_t precision;           /* SPH_FP64 or SPH_FP32_SWEEP */
  double dx;                   /* initial spacing = smoothing length h; r_c = 3h */
  double lo[3], hi[3];         /* the cell grid covers [lo, hi) */
  double cell_edge;            /* cell edge L >= r_c; 0: L = r_c */
  double dt;                   /* 0: eq. nummeth_timint_timestepcond at t = 0 */
  int64_t n;                   /* particles */
  const double *x, *u, *T;     /* [n][3], [n][3], [n] (T may be NULL) */
  const int32_t *kind;         /* SPH_FLUID / SPH_WALL / SPH_RIGID */
  const int32_t *phase;        /* material index, < n_mat */
  const int32_t *body;         /* body index of rigid particles, else ignored */
  const int32_t *moving;       /* walls following the wall motion (may be NULL) */
  int32_t n_mat, n_body;       /* 1..256 materials; fluid phases, switch targets and every
                                  phase of a thermal scene among the first 16 */
  const sph_material *mat;
  const sph_body_init *bodies;
  int32_t max_bodies;          /* capacity for bodies created by solidification */
  int32_t thermal, contact, phase_switch;
  double k_c, d_c;             /* contact stiffness / damping; < 0: defaults */
  double wall_A, wall_Omega, wall_dir[3];   /* moving walls: A (cos(Omega t) - 1) dir */
  int32_t heat_src;            /* Gaussian moving surface heat source */
  int32_t pad1;
  double src_Q, src_sigma, src_s0[2], src_v[2], src_ztop, src_depth;
  /* Transport-velocity formulation (Sec. "Momentum equation" applies a
   * constant background pressure p_b to all particles and takes the terms
   * from Adami, Hu, Adams 2013): fluid particles drift with
   * u~ = u + (dt/2) a_b, a_b = -(p_b/m_i) sum_j (V_i^2 + V_j^2) dW/dr e_ij
   * over all neighbours, and fluid pairs add the divergence of
   * A = rho u (u~ - u) to the momentum equation.  0: off (the printed
   * momentum equation only); the paper's examples use p_b = p0. */
  double p_b;
  /* Periodic axes (y and z only; x is the axis of the wave rows): the
   * extent hi - lo of a periodic axis is its period and must be a whole
   * number (>= 3) of cells; neighbours across the boundary are taken at
   * their image, positions are kept inside the box, a rigid body may
   * straddle the boundary (give its particles contiguous positions: its
   * centre of mass and frame come from them) and its centre of mass is not
   * wrapped.  Not combined with phase switching. */
  int32_t periodic[3];
  int32_t pad2;
} sph_scene_desc;

typedef struct sph_scene sph_scene;

/* Per-scene statistics (sph_scene_read_stats). */
typedef struct {
  int64_t step;                /* steps taken */
  double t, dt, k_c, d_c;
  int64_t n, n_fluid, n_wall, n_rigid;
  int32_t n_bodies, grid[3];
  int64_t pairs_last;          /* ordered pairs with a fluid member, last evaluation */
  int64_t pairs_total;         /* summed over all steps taken */
  int64_t pairs_fluid;         /* last evaluation: neighbours of fluid particles */
  int64_t pairs_rigid;         /* last evaluation: fluid neighbours of rigid particles */
  int64_t pairs_wall;          /* last evaluation: fluid neighbours of wall particles */
  uint32_t device_error;       /* SPH_ERR_* bits */
  uint32_t pad;
  double mass, momentum[3], kinetic;   /* FP64 global checks: fluid particles + active bodies
                                          (bodies: translation and rotation) */
  double potential;            /* energy of the body force, -sum m b.x (fluid + bodies) */
  int64_t n_melted;            /* phase switches since creation: rigid -> fluid */
  int64_t n_solidified;        /* and fluid -> rigid */
} sph_stats;

int sph_abi_version(void);
const char *sph_status_string(int status);
const char *sph_last_error(void);

/* Exact device-arena size in bytes for this descriptor (the HBM footprint
 * used for admission).  *status (may be NULL) receives the status; 0 is
 * returned on error. */
size_t sph_scene_arena_bytes(const sph_scene_desc *d, int *status);

/* Create a scene in the caller's device arena (at least
 * sph_scene_arena_bytes, 256-byte aligned) on the caller's HIP stream
 * (hipStream_t, may be NULL for the null stream), uploads the descriptor,
 * computes masses, body mass quantities (eqs. procwise_centerofmass,
 * procwise_inertia), the time step, and one evaluation that gives the
 * initial accelerations.  Arena and stream must outlive the scene.  On
 * error nothing is left allocated and *out is NULL. */
int sph_scene_create(const sph_scene_desc *d, void *dev_arena, size_t arena_bytes,
                     void *hip_stream, sph_scene **out);

/* Enqueue nsteps time steps (Sec. "Time integration following a
 * velocity-Verlet scheme" plus the phase switch).  Asynchronous. */
int sph_scene_step(sph_scene *s, int64_t nsteps);

/* Batches: several resident scenes advanced together.  Per step, every
 * scene's per-particle and per-body stages are enqueued on the batch stream
 * and the three interaction sweeps (density, extrapolation, forces) run as
 * one launch each over the concatenated waves of all scenes of the same
 * precision, dimension and thermal flag (a table of per-scene slots in the
 * caller's device workspace).  Every scene runs exactly the arithmetic of
 * sph_scene_step, so its results are bit for bit those it gets alone.
 *   sph_batch_bytes: device workspace for a batch of n scenes (256-byte
 *     aligned, caller-owned, must outlive the batch).
 *   sph_batch_create: n >= 1 distinct scenes (SPH_E_INVALID otherwise);
 *     hip_stream is the batch stream.  The scenes stay owned by the caller
 *     and must outlive the batch; a scene may be in several batches but
 *     only one may step it at a time.
 *   sph_batch_step: enqueues nsteps steps of every scene; asynchronous.
 *     Work already enqueued on a scene's own stream is waited for, and the
 *     scene's stream waits for the batch's work, through events.  Once the
 *     batch has taken a step in a given state of the scenes' buffer
 *     parities (there are two, alternating), the next step in that state is
 *     captured as a HIP graph and later ones replay it (not on the null
 *     stream; environment variable SPHRB_BATCH_GRAPHS=0 at
 *     sph_batch_create turns this off).
 *     Per-step timers of the scenes do not record batch steps.
 *   sph_batch_destroy: waits for the batch stream and frees the host side. */
typedef struct sph_batch sph_batch;
size_t sph_batch_bytes(int32_t n);
int sph_batch_create(sph_scene *const *scenes, int32_t n, void *dev_ws, size_t ws_bytes, void *hip_stream,
                     sph_batch **out);
int sph_batch_step(sph_batch *b, int64_t nsteps);
void sph_batch_destroy(sph_batch *b);

/* Wait for the scene's stream; returns SPH_E_STATE if a device error is set. */
int sph_scene_sync(sph_scene *s);

/* Particle fields for sph_scene_read_particles, packed in bit order, each
 * n (scalars) or 3n (vectors) doubles, original-id order. */
enum {
  SPH_F_X = 1u << 0, SPH_F_U = 1u << 1, SPH_F_A = 1u << 2, SPH_F_RHO = 1u << 3,
  SPH_F_P = 1u << 4, SPH_F_T = 1u << 5, SPH_F_PW = 1u << 6, SPH_F_UW = 1u << 7,
  SPH_F_FR = 1u << 8, SPH_F_M = 1u << 9, SPH_F_DTDT = 1u << 10,
  SPH_F_AB = 1u << 11,   /* background-pressure acceleration a_b (fluid; 0 elsewhere or when off) */
  SPH_F_UD = 1u << 12    /* u~ - u of the last drift (fluid; 0 elsewhere or when off) */
};
int sph_scene_read_particles(sph_scene *s, uint32_t field_mask, double *out_host);

/* Body records, SPH_BODY_REC doubles per body: m, r[3], q[4], u[3], w[3],
 * a[3], alpha[3], f[3], torque[3], world inertia (xx, yy, zz, xy, xz, yz;
 * 2D: zz only), active, fixed, 2 reserved.  *n_bodies receives the count;
 * at most cap records are written. */
#define SPH_BODY_REC 36
int sph_scene_read_bodies(sph_scene *s, double *out_host, int32_t cap, int32_t *n_bodies);

/* Neighbour lists (pairs a != b with |x_a - x_b| < r_c) as a CSR over
 * original ids with ascending ids per row.  Diagnostic; allocates device
 * scratch of its own.  Returns the number of pairs (fills ids only when it
 * fits in cap; offsets has n+1 entries), or -1 on error. */
int64_t sph_scene_read_neighbors(sph_scene *s, int64_t *offsets_host, int32_t *ids_host, int64_t cap);

/* Current order of the sorted particle arrays (ids by (cell, id)) and the
 * cell of every id (x-fastest linear index). */
int sph_scene_read_cell_order(sph_scene *s, int32_t *sorted_ids_host, int32_t *cell_of_id_host);

/* kind, phase, body of every id (any pointer may be NULL). */
int sph_scene_read_flags(sph_scene *s, int32_t *kind_host, int32_t *phase_host, int32_t *body_host);

int sph_scene_read_stats(sph_scene *s, sph_stats *out_host);

/* Kernel timing.  When enabled, every step records HIP events on the
 * scene's stream between its stages, without host synchronisation, for up
 * to SPH_TIMER_STEPS steps.  sph_scene_read_timers waits for the stream and
 * returns, summed over the recorded steps, the milliseconds of each stage:
 * [0] kick/drift and rigid/wall poses, [1] neighbour search (binning and
 * sort by (cell, id)), [2] density + EOS, [3] wall/rigid extrapolation,
 * [4] forces + heat, [5] per-body reduction + body integration, [6] rigid
 * particle velocities.  *steps receives the number of recorded steps and
 * step_ms (may be NULL) the duration of each recorded step (at most cap).
 * Enabling again restarts the record. */
#define SPH_TIMER_STEPS 4096
#define SPH_TIMER_STAGES 7
int sph_scene_enable_timers(sph_scene *s, int32_t enable);
int sph_scene_read_timers(sph_scene *s, double *stage_ms, int64_t *steps, double *step_ms, int64_t cap);

/* Checkpoint / resume.  A state image is a header (parameters, step
 * count, buffer parities) followed by the scene's device arena verbatim, so
 * a scene re-created from it continues bit for bit as the original would
 * have (timers are not part of the state).
 *   sph_scene_state_bytes: size of the image (0 for a NULL scene).
 *   sph_scene_read_state: waits for the scene's stream and writes the image
 *     into host_blob (at least sph_scene_state_bytes bytes, else
 *     SPH_E_INVALID).
 *   sph_state_arena_bytes: device arena size a scene re-created from the
 *     image needs; 0 and *status = SPH_E_INVALID for an image that is not
 *     one, was written by another ABI version or is truncated.
 *   sph_scene_create_from_state: re-creates the scene in the caller's
 *     256-byte aligned arena on the caller's stream (as sph_scene_create;
 *     the image is read during the call only).  On error nothing is left
 *     allocated and *out is NULL. */
size_t sph_scene_state_bytes(sph_scene *s);
int sph_scene_read_state(sph_scene *s, void *host_blob, size_t bytes);
size_t sph_state_arena_bytes(const void *host_blob, size_t bytes, int *status);
int sph_scene_create_from_state(const void *host_blob, size_t bytes, void *dev_arena, size_t arena_bytes,
                                void *hip_stream, sph_scene **out);

/* Release the scene's host-side handle.  Frees nothing the caller owns. */
void sph_scene_destroy(sph_scene *s);

#ifdef __cplusplus
}
#endif
#endif
