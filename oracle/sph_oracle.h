/*
 * sph_oracle.h -- plain FP64 CPU oracle of the SPH fluid / rigid-body /
 * thermal time step of Fuchs, Meier, Wall, Cyron (arXiv 2103.07925).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code
 * with the HIP library: its own types, its own kernel, its own neighbour
 * search, its own reductions.
 *
 * Every floating-point value is IEEE double; build with -O2
 * -ffp-contract=off and no fast-math, so that each expression rounds as
 * written.
 *
 * Layout conventions: particle arrays are indexed by original id; vectors
 * are stored as [n][3] (z ignored in 2D); integer arrays are int32.
 * Status codes: 0 ok, 1 invalid input, 2 out of memory, 4 state error
 * (particle left the cell grid, coincident particles, body capacity).
 */
#ifndef SPH_ORACLE_H
#define SPH_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_FLUID = 0, ORC_WALL = 1, ORC_RIGID = 2 };
enum { ORC_OK = 0, ORC_E_INVALID = 1, ORC_E_NOMEM = 2, ORC_E_STATE = 4 };

/* One phase (Sec. "Governing equations", multiple phases; material values of
 * the numerical examples). p0 is the reference pressure of the equation of
 * state, c = sqrt(p0/rho0). */
typedef struct {
  double rho0, p0, nu, cp, kappa;
  double b[3];          /* body force per unit mass */
  double T_t;           /* transition temperature */
  int32_t switch_to;    /* phase after a transition, -1: never switches */
  int32_t dirichlet;    /* wall phases: temperature prescribed (takes part in conduction) */
} orc_material;

typedef struct {
  double u[3], w[3], q[4];   /* q = (w, x, y, z) */
  int32_t fixed;
  int32_t pad;
} orc_body_init;

typedef struct {
  int32_t dim;
  int32_t pad0;
  double dx;                 /* initial spacing = smoothing length h */
  double lo[3], hi[3];       /* cell grid covers [lo, lo + ncell*L) */
  double cell_edge;          /* L >= r_c = 3 h */
  double dt;                 /* 0: stability bounds at t = 0 */
  int64_t n;
  const double *x, *u, *T;
  const int32_t *kind, *phase, *body, *moving;
  int32_t n_mat, n_body;
  const orc_material *mat;
  const orc_body_init *bodies;
  int32_t max_bodies;
  int32_t thermal, contact, phase_switch;
  double k_c, d_c;           /* < 0: defaults */
  double wall_A, wall_Omega, wall_dir[3];
  int32_t heat_src;
  int32_t pad1;
  double src_Q, src_sigma, src_s0[2], src_v[2], src_ztop, src_depth;
  double p_b;                /* background pressure of the transport-velocity formulation; 0: off */
  int32_t periodic[3];       /* periodic axes (y and z only); the extent must be a whole number of cells */
  int32_t pad2;
} orc_desc;

typedef struct orc_scene orc_scene;

/* Body record returned by orc_get_bodies, ORC_BODY_REC doubles per body:
 * [0] m, [1..3] r, [4..7] q, [8..10] u, [11..13] w, [14..16] a,
 * [17..19] alpha, [20..22] f, [23..25] torque, [26..31] world inertia
 * (xx, yy, zz, xy, xz, yz; 2D: zz only), [32] active, [33] fixed. */
#define ORC_BODY_REC 36

/* Particle fields for orc_get / orc_set. */
enum {
  ORC_F_X = 0, ORC_F_U = 1, ORC_F_A = 2, ORC_F_RHO = 3, ORC_F_P = 4, ORC_F_T = 5,
  ORC_F_PW = 6, ORC_F_UW = 7, ORC_F_FR = 8, ORC_F_M = 9, ORC_F_DTDT = 10,
  ORC_F_AB = 11,   /* background-pressure acceleration of fluid particles, last evaluation */
  ORC_F_UD = 12    /* transport minus momentum velocity u~ - u of fluid particles, last drift */
};
enum { ORC_I_KIND = 0, ORC_I_PHASE = 1, ORC_I_BODY = 2, ORC_I_CELL = 3 };

/* Stages of one evaluation, in the order of Sec. "Time integration". */
enum {
  ORC_S_NEIGHBORS = 4, ORC_S_DENSITY = 5, ORC_S_EXTRAP = 6, ORC_S_HEAT = 7,
  ORC_S_FORCES = 8, ORC_S_BODYSUMS = 9, ORC_S_BODYACC = 10
};

int orc_create(const orc_desc *d, orc_scene **out);
void orc_destroy(orc_scene *s);
int orc_step(orc_scene *s, int64_t nsteps);
double orc_get_dt(const orc_scene *s);
double orc_get_time(const orc_scene *s);
double orc_get_kc(const orc_scene *s);
double orc_get_dc(const orc_scene *s);
int32_t orc_n_bodies(const orc_scene *s);
int64_t orc_pair_count(const orc_scene *s);   /* ordered pairs with a fluid member, last evaluation */
int orc_get(const orc_scene *s, int32_t field, double *out);
int orc_set(orc_scene *s, int32_t field, const double *in);
int orc_get_int(const orc_scene *s, int32_t field, int32_t *out);
int orc_get_bodies(const orc_scene *s, double *out);
int orc_stage(orc_scene *s, int32_t stage);
/* neighbour CSR by id (pairs a != b, r < r_c), ids ascending per row;
 * returns the total, fills at most cap entries. */
int64_t orc_neighbors(orc_scene *s, int64_t *offsets, int32_t *ids, int64_t cap);
/* sorted order by (cell, id) and the cell of every id */
int orc_cell_order(orc_scene *s, int32_t *sorted_ids, int32_t *cell_of_id);
int orc_grid(const orc_scene *s, int32_t *ncell3);

/* Free functions, for pinning. */
double orc_kernel_W(int32_t dim, double h, double r);
double orc_kernel_dW(int32_t dim, double h, double r);
double orc_fsum(const double *v, int64_t n);
double orc_timestep(const orc_desc *d);
int orc_mass_props(int32_t dim, double dx, int64_t n, const double *x, const double *m,
                   double *out_m, double *out_r, double *out_I);
int orc_mass_props_partitioned(int32_t dim, double dx, int64_t n, const double *x,
                               const double *m, const int32_t *part, int32_t nparts,
                               double *out_m, double *out_r, double *out_I);

#ifdef __cplusplus
}
#endif
#endif
