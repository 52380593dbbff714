/*
 * sph_oracle.c -- plain FP64 CPU oracle of one SPH fluid / rigid-body /
 * thermal time step (Fuchs, Meier, Wall, Cyron, arXiv 2103.07925).
 *
 * TEST INFRASTRUCTURE ONLY: only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It is written for a reader who
 * checks it against the paper: plain loops over particles in original-id
 * order, one function per step of Sec. "Time integration following a
 * velocity-Verlet scheme", no blocking, no fusion, no parallelism.
 *
 * Readings of points the paper leaves open are listed in the design doc of the
 * repository and restated at the function that takes them.  The one
 * ordering choice that is not the paper's (it is needed so that an
 * independent implementation can reproduce sums bit for bit) is the
 * canonical gather order: neighbour cells in stencil order (dz outer, dy,
 * dx inner, each -1..1) and, inside a cell, ascending original id.
 */
#include "sph_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846

typedef struct {
  int32_t j;
  double d[3];   /* x_i - x_j */
  double r2;
} nb_t;

struct orc_scene {
  int dim;
  double dx, h, rc, rc2, L;
  double lo[3];
  int nc[3];
  int64_t ncells;
  double wnorm, dnorm, vol0, Ir_fac;
  double dt, t;
  int64_t step;
  int64_t n;
  /* particle state, original-id order */
  double *x, *u, *a, *rho, *p, *T, *dTdt, *m, *pw, *uw, *f, *rb, *rk, *aw, *x0;
  double *ab, *ud;   /* transport-velocity formulation: a_b and u~ - u */
  int32_t *kind, *phase, *body, *moving, *cell;
  /* cell lists: ids of cell c are cids[cstart[c] .. cstart[c+1]) ascending */
  int64_t *cstart;
  int32_t *cids;
  int64_t maxcell;
  /* materials */
  int n_mat;
  orc_material *mat;
  /* bodies */
  int nb, maxb;
  double *bm, *br, *bq, *bu, *bw, *ba, *bal, *bf, *bt, *bIb, *bb;
  int32_t *bfixed, *bactive;
  int64_t *bstart;
  int32_t *bids;
  /* options */
  int thermal, contact, pswitch;
  double kc, dc;
  double wall_A, wall_Om, wall_dir[3];
  int heat_src;
  double sQ, ssig, ss0[2], sv[2], sztop, sdepth;
  int tvf;
  double pb;
  int per[3];        /* periodic axes */
  double period[3];
  int64_t pairs;
  /* scratch */
  nb_t *nbuf;
  int64_t nbuf_cap;
  double *tmp;
  int64_t tmp_cap;
};

/* ------------------------------------------------------------------------ */
/* exact summation                                                          */
/* ------------------------------------------------------------------------ */

/* Exact sum of doubles rounded once to nearest (Shewchuk's non-overlapping
 * expansions, grown by error-free two-sums, then summed from the top with a
 * half-way correction).  Used wherever the text defines a plain sum over a
 * rigid body's particles (Sec. "Parallel evaluation of mass-related
 * quantities", "... of resultant force and torque"), so that the oracle's
 * value is the correctly rounded sum. */
double orc_fsum(const double *v, int64_t n) {
  double part[256];
  int np = 0;
  for (int64_t k = 0; k < n; ++k) {
    double x = v[k];
    int i = 0;
    for (int jj = 0; jj < np; ++jj) {
      double y = part[jj];
      if (fabs(x) < fabs(y)) { double t = x; x = y; y = t; }
      double hi = x + y;
      double lo = y - (hi - x);
      if (lo != 0.0) part[i++] = lo;
      x = hi;
    }
    np = i;
    part[np++] = x;
    if (np >= 250) return NAN;   /* impossible for finite doubles */
  }
  if (np == 0) return 0.0;
  int k = np - 1;
  double hi = part[k], lo = 0.0;
  while (k > 0) {
    double x = hi, y = part[--k];
    hi = x + y;
    double yr = hi - x;
    lo = y - yr;
    if (lo != 0.0) break;
  }
  if (k > 0 && ((lo < 0.0 && part[k - 1] < 0.0) || (lo > 0.0 && part[k - 1] > 0.0))) {
    double y = lo * 2.0;
    double x = hi + y;
    double yr = x - hi;
    if (y == yr) hi = x;
  }
  return hi;
}

/* ------------------------------------------------------------------------ */
/* smoothing kernel                                                          */
/* ------------------------------------------------------------------------ */

/* Quintic spline of Morris (1997) with support r_c = 3h (Remark "applied
 * kernel"): W = sigma_d / h^d [(3-q)^5 - 6(2-q)^5 + 15(1-q)^5], each bracket
 * taken only where positive, q = r/h.  sigma_d normalises the integral of W
 * to one (Remark "kernel properties"): sigma_1 = 1/120, sigma_2 = 7/(478 pi),
 * sigma_3 = 1/(120 pi). */
static double sigma_d(int dim) {
  if (dim == 1) return 1.0 / 120.0;
  if (dim == 2) return 7.0 / (478.0 * ORC_PI);
  return 1.0 / (120.0 * ORC_PI);
}
static double pow_d(double h, int d) {
  double r = h;
  for (int k = 1; k < d; ++k) r = r * h;
  return r;
}
static double p5(double s) { double t = s * s; t = t * t; return t * s; }
static double p4(double s) { double t = s * s; return t * t; }

static double quintic_w(double r, double h, double wnorm) {
  double q = r / h;
  if (!(q < 3.0)) return 0.0;
  double w = p5(3.0 - q);
  if (q < 2.0) w = w - 6.0 * p5(2.0 - q);
  if (q < 1.0) w = w + 15.0 * p5(1.0 - q);
  return w * wnorm;
}
static double quintic_dw(double r, double h, double dnorm) {
  double q = r / h;
  if (!(q < 3.0)) return 0.0;
  double g = p4(3.0 - q);
  if (q < 2.0) g = g - 6.0 * p4(2.0 - q);
  if (q < 1.0) g = g + 15.0 * p4(1.0 - q);
  return g * dnorm;
}
double orc_kernel_W(int32_t dim, double h, double r) {
  return quintic_w(r, h, sigma_d(dim) / pow_d(h, dim));
}
double orc_kernel_dW(int32_t dim, double h, double r) {
  return quintic_dw(r, h, -5.0 * sigma_d(dim) / pow_d(h, dim + 1));
}
static double kW(const orc_scene *s, double r) { return quintic_w(r, s->h, s->wnorm); }
static double kdW(const orc_scene *s, double r) { return quintic_dw(r, s->h, s->dnorm); }

/* ------------------------------------------------------------------------ */
/* small vector / quaternion helpers                                         */
/* ------------------------------------------------------------------------ */

static void cross3(const double *a, const double *b, double *c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Rotation matrix of the unit quaternion q = (w, x, y, z). */
static void quat_to_rot(const double *q, double R[9]) {
  double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1.0 - 2.0 * (y * y + z * z);
  R[1] = 2.0 * (x * y - w * z);
  R[2] = 2.0 * (x * z + w * y);
  R[3] = 2.0 * (x * y + w * z);
  R[4] = 1.0 - 2.0 * (x * x + z * z);
  R[5] = 2.0 * (y * z - w * x);
  R[6] = 2.0 * (x * z - w * y);
  R[7] = 2.0 * (y * z + w * x);
  R[8] = 1.0 - 2.0 * (x * x + y * y);
}
static void mat_vec(const double R[9], const double *v, double *o) {
  o[0] = R[0] * v[0] + R[1] * v[1] + R[2] * v[2];
  o[1] = R[3] * v[0] + R[4] * v[1] + R[5] * v[2];
  o[2] = R[6] * v[0] + R[7] * v[1] + R[8] * v[2];
}
static void matT_vec(const double R[9], const double *v, double *o) {
  o[0] = R[0] * v[0] + R[3] * v[1] + R[6] * v[2];
  o[1] = R[1] * v[0] + R[4] * v[1] + R[7] * v[2];
  o[2] = R[2] * v[0] + R[5] * v[1] + R[8] * v[2];
}
/* Hamilton product p o q. */
static void quat_mul(const double *p, const double *q, double *o) {
  o[0] = p[0] * q[0] - p[1] * q[1] - p[2] * q[2] - p[3] * q[3];
  o[1] = p[0] * q[1] + p[1] * q[0] + p[2] * q[3] - p[3] * q[2];
  o[2] = p[0] * q[2] - p[1] * q[3] + p[2] * q[0] + p[3] * q[1];
  o[3] = p[0] * q[3] + p[1] * q[2] - p[2] * q[1] + p[3] * q[0];
}
/* A B C^T style products: out = R M R^T (Rt = 0) or R^T M R (Rt = 1). */
static void rot_sandwich(const double R[9], const double M[9], int transpose_first, double out[9]) {
  double A[9], T[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      A[3 * i + j] = transpose_first ? R[3 * j + i] : R[3 * i + j];
    }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s = s + A[3 * i + k] * M[3 * k + j];
      T[3 * i + j] = s;
    }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s = s + T[3 * i + k] * A[3 * j + k];
      out[3 * i + j] = s;
    }
}

/* ------------------------------------------------------------------------ */
/* mass-related quantities of a rigid body                                   */
/* ------------------------------------------------------------------------ */

/* Inertia of one rigid particle about its own centre (Remark "rigid particle
 * inertia"): a disc (2D) or ball (3D) of the particle's effective volume.
 * The printed 0.5 m r_eff is read with r_eff squared (the units demand it,
 * and the disc example's plotted inertia range confirms it). */
static double particle_inertia_factor(int dim, double dx) {
  if (dim == 2) {
    double reff2 = dx * dx / ORC_PI;
    return 0.5 * reff2;
  }
  double reff = cbrt(0.75 / ORC_PI) * dx;
  return 0.4 * (reff * reff);
}

/* Mass, centre of mass and inertia of one set of particles about its own
 * centre of mass: eqs. procwise_centerofmass and procwise_inertia (which,
 * with one partition, are the body quantities; Remark "serial mass
 * quantities").  Sums are exact.  I is 3x3 row-major; in 2D only the polar
 * moment I[8] is set. */
static void mass_props_set(int dim, double Ir_fac, int64_t n, const int64_t *idx,
                           const double *x, const double *m, double *tmp,
                           double *om, double *orr, double *oI) {
  for (int64_t k = 0; k < n; ++k) tmp[k] = m[idx[k]];
  double M = orc_fsum(tmp, n);
  double r[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < dim; ++a) {
    for (int64_t k = 0; k < n; ++k) tmp[k] = m[idx[k]] * x[3 * idx[k] + a];
    r[a] = orc_fsum(tmp, n) / M;
  }
  for (int q = 0; q < 9; ++q) oI[q] = 0.0;
  if (dim == 2) {
    for (int64_t k = 0; k < n; ++k) {
      int64_t i = idx[k];
      double d0 = r[0] - x[3 * i + 0], d1 = r[1] - x[3 * i + 1];
      double dsq = d0 * d0 + d1 * d1;
      tmp[k] = Ir_fac * m[i] + dsq * m[i];
    }
    oI[8] = orc_fsum(tmp, n);
  } else {
    for (int ii = 0; ii < 3; ++ii)
      for (int jj = ii; jj < 3; ++jj) {
        for (int64_t k = 0; k < n; ++k) {
          int64_t i = idx[k];
          double d[3] = {r[0] - x[3 * i + 0], r[1] - x[3 * i + 1], r[2] - x[3 * i + 2]};
          double dsq = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
          if (ii == jj)
            tmp[k] = Ir_fac * m[i] + (dsq - d[ii] * d[jj]) * m[i];
          else
            tmp[k] = (-(d[ii] * d[jj])) * m[i];
        }
        double v = orc_fsum(tmp, n);
        oI[3 * ii + jj] = v;
        oI[3 * jj + ii] = v;
      }
  }
  *om = M;
  orr[0] = r[0]; orr[1] = r[1]; orr[2] = r[2];
}

int orc_mass_props(int32_t dim, double dx, int64_t n, const double *x, const double *m,
                   double *out_m, double *out_r, double *out_I) {
  if ((dim != 2 && dim != 3) || n <= 0) return ORC_E_INVALID;
  int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * n);
  double *tmp = (double *)malloc(sizeof(double) * n);
  if (!idx || !tmp) { free(idx); free(tmp); return ORC_E_NOMEM; }
  for (int64_t k = 0; k < n; ++k) idx[k] = k;
  mass_props_set(dim, particle_inertia_factor(dim, dx), n, idx, x, m, tmp, out_m, out_r, out_I);
  free(idx); free(tmp);
  return ORC_OK;
}

/* Processor-wise quantities of every partition, then combined on the
 * "owner": eqs. global_centerofmass and global_inertia (Huygens-Steiner). */
int orc_mass_props_partitioned(int32_t dim, double dx, int64_t n, const double *x,
                               const double *m, const int32_t *part, int32_t nparts,
                               double *out_m, double *out_r, double *out_I) {
  if ((dim != 2 && dim != 3) || n <= 0 || nparts <= 0) return ORC_E_INVALID;
  int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * n);
  double *tmp = (double *)malloc(sizeof(double) * (n > nparts ? n : nparts));
  double *pm = (double *)calloc(nparts, sizeof(double));
  double *pr = (double *)calloc(3 * (size_t)nparts, sizeof(double));
  double *pI = (double *)calloc(9 * (size_t)nparts, sizeof(double));
  if (!idx || !tmp || !pm || !pr || !pI) { free(idx); free(tmp); free(pm); free(pr); free(pI); return ORC_E_NOMEM; }
  double Ir = particle_inertia_factor(dim, dx);
  for (int32_t p = 0; p < nparts; ++p) {
    int64_t c = 0;
    for (int64_t k = 0; k < n; ++k) if (part[k] == p) idx[c++] = k;
    if (c == 0) continue;
    mass_props_set(dim, Ir, c, idx, x, m, tmp, &pm[p], &pr[3 * p], &pI[9 * p]);
  }
  double M = orc_fsum(pm, nparts);
  double r[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < dim; ++a) {
    for (int32_t p = 0; p < nparts; ++p) tmp[p] = pm[p] * pr[3 * p + a];
    r[a] = orc_fsum(tmp, nparts) / M;
  }
  for (int q = 0; q < 9; ++q) out_I[q] = 0.0;
  if (dim == 2) {
    for (int32_t p = 0; p < nparts; ++p) {
      double d0 = r[0] - pr[3 * p], d1 = r[1] - pr[3 * p + 1];
      tmp[p] = pI[9 * p + 8] + (d0 * d0 + d1 * d1) * pm[p];
    }
    out_I[8] = orc_fsum(tmp, nparts);
  } else {
    for (int ii = 0; ii < 3; ++ii)
      for (int jj = ii; jj < 3; ++jj) {
        for (int32_t p = 0; p < nparts; ++p) {
          double d[3] = {r[0] - pr[3 * p], r[1] - pr[3 * p + 1], r[2] - pr[3 * p + 2]};
          double dsq = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
          double st = (ii == jj) ? (dsq - d[ii] * d[jj]) : (-(d[ii] * d[jj]));
          tmp[p] = pI[9 * p + 3 * ii + jj] + st * pm[p];
        }
        double v = orc_fsum(tmp, nparts);
        out_I[3 * ii + jj] = v;
        out_I[3 * jj + ii] = v;
      }
  }
  *out_m = M;
  out_r[0] = r[0]; out_r[1] = r[1]; out_r[2] = r[2];
  free(idx); free(tmp); free(pm); free(pr); free(pI);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* time step size                                                            */
/* ------------------------------------------------------------------------ */

/* Eq. timestepcond evaluated once at t = 0 (CFL with the largest speed of
 * sound of the fluid phases present and the largest initial fluid speed;
 * viscous; body force; conduction when thermal).  The contact bound is
 * applied only for a user-given stiffness: the default stiffness is chosen
 * so that this bound equals twice the step and never binds. */
static int phase_used(const orc_desc *d, int kind, int ph) {
  for (int64_t i = 0; i < d->n; ++i)
    if (d->kind[i] == kind && d->phase[i] == ph) return 1;
  return 0;
}
static double timestep_without_contact(const orc_desc *d, double *m_min_out) {
  double h = d->dx;
  double cmax = 0.0, numax = 0.0, bmax = 0.0, heat = INFINITY, umax = 0.0, mmin = INFINITY;
  double vol0 = pow_d(d->dx, d->dim);
  for (int ph = 0; ph < d->n_mat; ++ph) {
    const orc_material *M = &d->mat[ph];
    int fl = phase_used(d, ORC_FLUID, ph), rg = phase_used(d, ORC_RIGID, ph);
    if (fl) {
      double c = sqrt(M->p0 / M->rho0);
      if (c > cmax) cmax = c;
      if (M->nu > numax) numax = M->nu;
    }
    if (fl || rg) {
      double bn = sqrt(M->b[0] * M->b[0] + M->b[1] * M->b[1] + M->b[2] * M->b[2]);
      if (bn > bmax) bmax = bn;
      if (d->thermal && M->kappa > 0.0) {
        double v = 0.1 * M->rho0 * M->cp * h * h / M->kappa;
        if (v < heat) heat = v;
      }
    }
    if (rg) {
      double mr = M->rho0 * vol0;
      if (mr < mmin) mmin = mr;
    }
  }
  for (int64_t i = 0; i < d->n; ++i)
    if (d->kind[i] == ORC_FLUID) {
      double v = sqrt(d->u[3 * i] * d->u[3 * i] + d->u[3 * i + 1] * d->u[3 * i + 1] +
                      d->u[3 * i + 2] * d->u[3 * i + 2]);
      if (v > umax) umax = v;
    }
  double dt = INFINITY;
  if (cmax > 0.0) { double v = 0.25 * h / (cmax + umax); if (v < dt) dt = v; }
  if (numax > 0.0) { double v = 0.125 * h * h / numax; if (v < dt) dt = v; }
  if (bmax > 0.0) { double v = 0.25 * sqrt(h / bmax); if (v < dt) dt = v; }
  if (heat < dt) dt = heat;
  *m_min_out = mmin;
  return dt;
}
double orc_timestep(const orc_desc *d) {
  double mmin;
  double dt = timestep_without_contact(d, &mmin);
  if (d->contact && d->k_c > 0.0 && isfinite(mmin)) {
    double v = 0.22 * sqrt(mmin / d->k_c);
    if (v < dt) dt = v;
  }
  return dt;
}

/* ------------------------------------------------------------------------ */
/* neighbour search (Sec. "Parallelization via spatial decomposition")      */
/* ------------------------------------------------------------------------ */

/* Every particle goes to the cubic cell floor((x - lo)/L) of a uniform
 * lattice whose edge L is at least r_c, so that all neighbours lie in the
 * same or an adjacent cell.  Cell lists hold ids in ascending order. */
static int build_cells(orc_scene *s) {
  int64_t C = s->ncells;
  for (int64_t c = 0; c <= C; ++c) s->cstart[c] = 0;
  for (int64_t i = 0; i < s->n; ++i) {
    int c3[3] = {0, 0, 0};
    for (int a = 0; a < s->dim; ++a) {
      double v = floor((s->x[3 * i + a] - s->lo[a]) / s->L);
      /* a wrapped coordinate a rounding below lo + period stays in the last cell */
      if (s->per[a] && v == (double)s->nc[a]) v = (double)(s->nc[a] - 1);
      if (!(v >= 0.0) || v >= (double)s->nc[a]) return ORC_E_STATE;
      c3[a] = (int)v;
    }
    int64_t lin = (int64_t)c3[0] + (int64_t)s->nc[0] * ((int64_t)c3[1] + (int64_t)s->nc[1] * c3[2]);
    s->cell[i] = (int32_t)lin;
    s->cstart[lin + 1] += 1;
  }
  int64_t mx = 0;
  for (int64_t c = 0; c < C; ++c) {
    if (s->cstart[c + 1] > mx) mx = s->cstart[c + 1];
    s->cstart[c + 1] += s->cstart[c];
  }
  s->maxcell = mx;
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (C > 0 ? C : 1));
  if (!fill) return ORC_E_NOMEM;
  for (int64_t c = 0; c < C; ++c) fill[c] = s->cstart[c];
  for (int64_t i = 0; i < s->n; ++i) s->cids[fill[s->cell[i]]++] = (int32_t)i;
  free(fill);
  int64_t need = (s->dim == 3 ? 27 : 9) * (mx > 0 ? mx : 1);
  if (need > s->nbuf_cap) {
    free(s->nbuf);
    s->nbuf = (nb_t *)malloc(sizeof(nb_t) * need);
    if (!s->nbuf) { s->nbuf_cap = 0; return ORC_E_NOMEM; }
    s->nbuf_cap = need;
  }
  return ORC_OK;
}

/* Neighbours j of particle i with |x_i - x_j|^2 < r_c^2, in canonical
 * gather order; i itself is included only when with_self is set.  Along a
 * periodic axis the stencil wraps and a neighbour across the boundary is
 * taken at its image x_j +- period (the nearest one: the grid has at least
 * three cells along the axis). */
static int64_t gather(const orc_scene *s, int64_t i, int with_self) {
  int64_t lin = s->cell[i];
  int ci[3];
  ci[0] = (int)(lin % s->nc[0]);
  ci[1] = (int)((lin / s->nc[0]) % s->nc[1]);
  ci[2] = (int)(lin / ((int64_t)s->nc[0] * s->nc[1]));
  int zr = (s->dim == 3) ? 1 : 0;
  int64_t cnt = 0;
  const double *xi = &s->x[3 * i];
  for (int dz = -zr; dz <= zr; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dxx = -1; dxx <= 1; ++dxx) {
        int cx = ci[0] + dxx, cy = ci[1] + dy, cz = ci[2] + dz;
        double sh1 = 0.0, sh2 = 0.0;
        if (s->per[1] && cy < 0) { cy += s->nc[1]; sh1 = -s->period[1]; }
        if (s->per[1] && cy >= s->nc[1]) { cy -= s->nc[1]; sh1 = s->period[1]; }
        if (s->per[2] && cz < 0) { cz += s->nc[2]; sh2 = -s->period[2]; }
        if (s->per[2] && cz >= s->nc[2]) { cz -= s->nc[2]; sh2 = s->period[2]; }
        if (cx < 0 || cy < 0 || cz < 0 || cx >= s->nc[0] || cy >= s->nc[1] || cz >= s->nc[2]) continue;
        int64_t c = (int64_t)cx + (int64_t)s->nc[0] * ((int64_t)cy + (int64_t)s->nc[1] * cz);
        for (int64_t k = s->cstart[c]; k < s->cstart[c + 1]; ++k) {
          int32_t j = s->cids[k];
          if (j == i && !with_self) continue;
          const double *xj = &s->x[3 * j];
          double d0 = xi[0] - xj[0], d1 = xi[1] - (xj[1] + sh1), d2 = 0.0;
          double r2 = d0 * d0 + d1 * d1;
          if (s->dim == 3) { d2 = xi[2] - (xj[2] + sh2); r2 = r2 + d2 * d2; }
          if (r2 < s->rc2) {
            nb_t *e = &s->nbuf[cnt++];
            e->j = j; e->d[0] = d0; e->d[1] = d1; e->d[2] = d2; e->r2 = r2;
          }
        }
      }
  return cnt;
}

/* ------------------------------------------------------------------------ */
/* interaction stages                                                        */
/* ------------------------------------------------------------------------ */

/* Eq. nummeth_fluid_densum (the particle itself included, W(0)) and the
 * equation of state eq. nummeth_fluid_eos, p = p0 (rho/rho0 - 1).  Rigid
 * particles keep their material density.  Also counts fluid-centred pairs. */
static void stage_density(orc_scene *s) {
  int64_t P = 0;
  for (int64_t i = 0; i < s->n; ++i) {
    const orc_material *M = &s->mat[s->phase[i]];
    if (s->kind[i] == ORC_RIGID) { s->rho[i] = M->rho0; continue; }
    if (s->kind[i] != ORC_FLUID) continue;
    int64_t cnt = gather(s, i, 1);
    double sum = 0.0;
    for (int64_t k = 0; k < cnt; ++k) sum = sum + kW(s, sqrt(s->nbuf[k].r2));
    P += cnt - 1;
    s->rho[i] = s->m[i] * sum;
    s->p[i] = M->p0 * (s->rho[i] / M->rho0 - 1.0);
  }
  s->pairs = P;
}

/* Acceleration of a rigid particle as a material point of its body:
 * a_k + alpha_k x r_rk + omega_k x (omega_k x r_rk). */
static void rigid_point_acc(const orc_scene *s, int64_t r, double *out) {
  int k = s->body[r];
  const double *rk = &s->rk[3 * r];
  double t1[3], t2[3], t3[3];
  cross3(&s->bal[3 * k], rk, t1);
  cross3(&s->bw[3 * k], rk, t2);
  cross3(&s->bw[3 * k], t2, t3);
  for (int a = 0; a < 3; ++a) out[a] = s->ba[3 * k + a] + t1[a] + t3[a];
}

/* Wall and rigid particle pressure and velocity extrapolated from the fluid
 * (Sec. "Boundary and coupling conditions", the local force balance of
 * Adami, Hu, Adams 2012): p_w = [sum p_f W + sum rho_f (b_f - a_w).(x_w - x_f) W]
 * / sum W, u~_w = 2 u_w - sum u_f W / sum W; no fluid neighbour: p_w = 0,
 * u~_w = u_w. */
static void stage_extrapolate(orc_scene *s) {
  int64_t P = 0;
  for (int64_t w = 0; w < s->n; ++w) {
    if (s->kind[w] == ORC_FLUID) continue;
    double aw[3] = {0.0, 0.0, 0.0};
    if (s->kind[w] == ORC_RIGID) rigid_point_acc(s, w, aw);
    else if (s->moving[w]) { aw[0] = s->aw[3 * w]; aw[1] = s->aw[3 * w + 1]; aw[2] = s->aw[3 * w + 2]; }
    int64_t cnt = gather(s, w, 0);
    double sW = 0.0, sp = 0.0, su[3] = {0.0, 0.0, 0.0};
    for (int64_t k = 0; k < cnt; ++k) {
      const nb_t *e = &s->nbuf[k];
      int32_t j = e->j;
      if (s->kind[j] != ORC_FLUID) continue;
      P += 1;
      const orc_material *Mj = &s->mat[s->phase[j]];
      double W = kW(s, sqrt(e->r2));
      double dot = (Mj->b[0] - aw[0]) * e->d[0] + (Mj->b[1] - aw[1]) * e->d[1];
      if (s->dim == 3) dot = dot + (Mj->b[2] - aw[2]) * e->d[2];
      sW = sW + W;
      sp = sp + (s->p[j] + s->rho[j] * dot) * W;
      for (int a = 0; a < s->dim; ++a) su[a] = su[a] + s->u[3 * j + a] * W;
    }
    if (sW > 0.0) {
      s->pw[w] = sp / sW;
      for (int a = 0; a < s->dim; ++a) s->uw[3 * w + a] = 2.0 * s->u[3 * w + a] - su[a] / sW;
    } else {
      s->pw[w] = 0.0;
      for (int a = 0; a < s->dim; ++a) s->uw[3 * w + a] = s->u[3 * w + a];
    }
    if (s->kind[w] == ORC_RIGID) s->p[w] = s->pw[w];
  }
  s->pairs += P;
}

/* Gaussian moving surface heat source (heat power per unit mass) of the
 * two-phase thermal configuration; zero unless enabled. */
static double heat_source(const orc_scene *s, int64_t a, double t) {
  if (!s->heat_src) return 0.0;
  int up = s->dim - 1;
  if (s->x[3 * a + up] < s->sztop - s->sdepth) return 0.0;
  double c0 = s->ss0[0] + s->sv[0] * t;
  double d0 = s->x[3 * a] - c0;
  double ss2 = s->ssig * s->ssig;
  if (s->dim == 3) {
    double c1 = s->ss0[1] + s->sv[1] * t;
    double d1 = s->x[3 * a + 1] - c1;
    double dd = d0 * d0 + d1 * d1;
    return s->sQ / (2.0 * ORC_PI * ss2) * exp(-dd / (2.0 * ss2));
  }
  double dd = d0 * d0;
  return s->sQ / (sqrt(2.0 * ORC_PI) * s->ssig) * exp(-dd / (2.0 * ss2));
}

/* Eq. nummeth_thermo_heat_equation (Cleary and Monaghan): for fluid and rigid
 * particles a, c_p,a dT_a/dt = 1/rho_a sum_b V_b 4 k_a k_b/(k_a + k_b)
 * T_ab / r_ab dW/dr, all rates from T^n; then T^{n+1} = T^n + dt dT/dt.
 * Walls take part as neighbours only where their temperature is
 * prescribed, with V_b = dx^d and their phase's conductivity.  With
 * c_p = 1 and k = D the same operator is the diffusion equation of a
 * concentration (the remark on concentration-driven transitions in Sec.
 * "Reversible phase transition"): C in place of T, transitions at C_t. */
static int stage_heat(orc_scene *s, int update) {
  double t = s->t;
  for (int64_t a = 0; a < s->n; ++a) {
    if (s->kind[a] == ORC_WALL) { s->dTdt[a] = 0.0; continue; }
    const orc_material *Ma = &s->mat[s->phase[a]];
    double rho_a = (s->kind[a] == ORC_FLUID) ? s->rho[a] : Ma->rho0;
    double ka = Ma->kappa;
    int64_t cnt = gather(s, a, 0);
    double sum = 0.0;
    for (int64_t k = 0; k < cnt; ++k) {
      const nb_t *e = &s->nbuf[k];
      int32_t j = e->j;
      const orc_material *Mb = &s->mat[s->phase[j]];
      double Vb;
      if (s->kind[j] == ORC_FLUID) Vb = s->m[j] / s->rho[j];
      else if (s->kind[j] == ORC_RIGID) Vb = s->m[j] / Mb->rho0;
      else if (Mb->dirichlet) Vb = s->vol0;
      else continue;
      double kb = Mb->kappa;
      if (!(ka + kb > 0.0)) continue;
      if (e->r2 == 0.0) return ORC_E_STATE;
      double kk = (4.0 * ka * kb) / (ka + kb);
      double r = sqrt(e->r2);
      sum = sum + (Vb * kk) * ((s->T[a] - s->T[j]) / r) * kdW(s, r);
    }
    double rate = sum / (rho_a * Ma->cp);
    if (s->heat_src) rate = rate + heat_source(s, a, t) / Ma->cp;
    s->dTdt[a] = rate;
  }
  /* a fluid or rigid phase with a prescribed value keeps it (the gastric
   * juice of Sec. "Gastric disintegration of food boluses" holds its
   * concentration at all times) */
  if (update)
    for (int64_t a = 0; a < s->n; ++a)
      if (s->kind[a] != ORC_WALL && !s->mat[s->phase[a]].dirichlet) s->T[a] = s->T[a] + s->dt * s->dTdt[a];
  return ORC_OK;
}

/* Pair force F_ij = m_i a_ij of eq. nummeth_fluid_momentum for fluid i and
 * neighbour j, d = x_i - x_j:
 *   F_ij = (V_i^2 + V_j^2) dW/dr [ -p~_ij e_ij + eta~_ij u_ij / r_ij ],
 *   p~ = (rho_j p_i + rho_i p_j)/(rho_i + rho_j), eta~ = 2 eta_i eta_j/(eta_i + eta_j),
 * eta = rho0 nu of the phase.  A wall or rigid neighbour enters with its
 * extrapolated p_w and u~_w, the density rho0_i (p_w/p0_i + 1) of i's phase,
 * the mass m_i and eta_i.  Written so that F_ji = -F_ij bit for bit.
 *
 * With the transport-velocity formulation (Sec. "Momentum equation" names
 * it and leaves its terms to Adami, Hu, Adams 2013) a fluid neighbour adds
 * the divergence of the tensor A = rho u (u~ - u) in the same pair form,
 *   (V_i^2 + V_j^2) dW/dr (1/2) (A_i + A_j) e_ij,
 * where A e = rho u ((u~ - u).e); wall and rigid neighbours carry no A.
 * *c_out receives (V_i^2 + V_j^2) dW/dr / r, the factor of the
 * background-pressure sum. */
static void pair_force(const orc_scene *s, int64_t i, int64_t j, const double *d, double r2, double *F,
                       double *c_out) {
  const orc_material *Mi = &s->mat[s->phase[i]];
  double rho_i = s->rho[i], p_i = s->p[i], m_i = s->m[i];
  double eta_i = Mi->rho0 * Mi->nu;
  double rho_j, p_j, m_j, eta_j;
  const double *u_j;
  if (s->kind[j] == ORC_FLUID) {
    const orc_material *Mj = &s->mat[s->phase[j]];
    rho_j = s->rho[j]; p_j = s->p[j]; m_j = s->m[j]; eta_j = Mj->rho0 * Mj->nu;
    u_j = &s->u[3 * j];
  } else {
    p_j = s->pw[j];
    rho_j = Mi->rho0 * (p_j / Mi->p0 + 1.0);
    m_j = m_i;
    eta_j = eta_i;
    u_j = &s->uw[3 * j];
  }
  double Vi = m_i / rho_i, Vj = m_j / rho_j;
  double vv = Vi * Vi + Vj * Vj;
  double pt = (rho_j * p_i + rho_i * p_j) / (rho_i + rho_j);
  double et = (eta_i + eta_j > 0.0) ? (2.0 * eta_i * eta_j) / (eta_i + eta_j) : 0.0;
  double r = sqrt(r2);
  double c = vv * kdW(s, r) / r;
  for (int a = 0; a < s->dim; ++a) F[a] = c * (et * (s->u[3 * i + a] - u_j[a]) - pt * d[a]);
  if (s->tvf && s->kind[j] == ORC_FLUID) {
    /* (1/2)(A_i + A_j) d with A d = rho u ((u~ - u).d) */
    double si = 0.0, sj = 0.0;
    for (int a = 0; a < s->dim; ++a) {
      si = si + s->ud[3 * i + a] * d[a];
      sj = sj + s->ud[3 * j + a] * d[a];
    }
    double hi = 0.5 * rho_i * si, hj = 0.5 * rho_j * sj;
    for (int a = 0; a < s->dim; ++a) F[a] = F[a] + c * (hi * s->u[3 * i + a] + hj * u_j[a]);
  }
  *c_out = c;
}

/* Eq. nummeth_fluid_momentum for fluid particles, a_i = (1/m_i) sum_j F_ij
 * + b_i; eq. nummeth_rigid_rigidparticle_force for rigid particles,
 * f_r = sum_i f_ri + contact, with the coupling force f_ri = -m_i a_ir
 * (eq. nummeth_fluid_couplingforce) and the spring-dashpot contact of
 * eq. nummeth_rigid_contactforce against rigid particles of other bodies
 * and wall particles, f = -min(0, k_c (r - dx) + d_c e.v) e for r < dx. */
static int stage_forces(orc_scene *s) {
  double dx2 = s->dx * s->dx;
  for (int64_t i = 0; i < s->n; ++i) {
    for (int a = 0; a < 3; ++a) s->ab[3 * i + a] = 0.0;
    if (s->kind[i] == ORC_WALL) continue;
    int64_t cnt = gather(s, i, 0);
    double acc[3] = {0.0, 0.0, 0.0};
    if (s->kind[i] == ORC_FLUID) {
      /* background-pressure acceleration of the transport velocity,
       * a_b = -(p_b/m_i) sum_j (V_i^2 + V_j^2) dW/dr e_ij over all neighbours */
      double bs[3] = {0.0, 0.0, 0.0};
      for (int64_t k = 0; k < cnt; ++k) {
        const nb_t *e = &s->nbuf[k];
        if (e->r2 == 0.0) return ORC_E_STATE;
        double F[3], c;
        pair_force(s, i, e->j, e->d, e->r2, F, &c);
        for (int a = 0; a < s->dim; ++a) {
          acc[a] = acc[a] + F[a];
          bs[a] = bs[a] + c * e->d[a];
        }
      }
      const orc_material *M = &s->mat[s->phase[i]];
      for (int a = 0; a < s->dim; ++a) s->a[3 * i + a] = acc[a] / s->m[i] + M->b[a];
      if (s->tvf)
        for (int a = 0; a < s->dim; ++a) s->ab[3 * i + a] = -(s->pb * bs[a]) / s->m[i];
    } else {
      for (int64_t k = 0; k < cnt; ++k) {
        const nb_t *e = &s->nbuf[k];
        int32_t j = e->j;
        if (e->r2 == 0.0) return ORC_E_STATE;
        if (s->kind[j] == ORC_FLUID) {
          double dj[3] = {-e->d[0], -e->d[1], -e->d[2]};
          double F[3], c;
          pair_force(s, j, i, dj, e->r2, F, &c);
          for (int a = 0; a < s->dim; ++a) acc[a] = acc[a] - F[a];
        } else if (s->contact && e->r2 < dx2 &&
                   (s->kind[j] == ORC_WALL || s->body[j] != s->body[i])) {
          double r = sqrt(e->r2);
          double ev[3] = {0.0, 0.0, 0.0};
          double en = 0.0;
          for (int a = 0; a < s->dim; ++a) {
            ev[a] = e->d[a] / r;
            en = en + ev[a] * (s->u[3 * i + a] - s->u[3 * j + a]);
          }
          double fn = s->kc * (r - s->dx) + s->dc * en;
          if (fn < 0.0)
            for (int a = 0; a < s->dim; ++a) acc[a] = acc[a] - fn * ev[a];
        }
      }
      for (int a = 0; a < 3; ++a) s->f[3 * i + a] = (a < s->dim) ? acc[a] : 0.0;
    }
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* rigid bodies                                                              */
/* ------------------------------------------------------------------------ */

static int build_body_lists(orc_scene *s) {
  for (int k = 0; k <= s->maxb; ++k) s->bstart[k] = 0;
  for (int64_t i = 0; i < s->n; ++i)
    if (s->kind[i] == ORC_RIGID) {
      if (s->body[i] < 0 || s->body[i] >= s->nb) return ORC_E_STATE;
      s->bstart[s->body[i] + 1] += 1;
    }
  for (int k = 0; k < s->maxb; ++k) s->bstart[k + 1] += s->bstart[k];
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (s->maxb > 0 ? s->maxb : 1));
  if (!fill) return ORC_E_NOMEM;
  for (int k = 0; k < s->maxb; ++k) fill[k] = s->bstart[k];
  for (int64_t i = 0; i < s->n; ++i)
    if (s->kind[i] == ORC_RIGID) s->bids[fill[s->body[i]]++] = (int32_t)i;
  free(fill);
  return ORC_OK;
}

static int ensure_tmp(orc_scene *s, int64_t need) {
  if (need <= s->tmp_cap) return ORC_OK;
  free(s->tmp);
  s->tmp = (double *)malloc(sizeof(double) * need);
  if (!s->tmp) { s->tmp_cap = 0; return ORC_E_NOMEM; }
  s->tmp_cap = need;
  return ORC_OK;
}

/* Recompute m_k, r_k and I_k of body k from its current particles (single
 * partition), the body-frame inertia I^b = R^T I R and the body-frame
 * offsets r_rk^b = R^T (x_r - r_k) (Remark "relative position"). */
static int body_recompute(orc_scene *s, int k) {
  int64_t b0 = s->bstart[k], b1 = s->bstart[k + 1], c = b1 - b0;
  if (c == 0) { s->bactive[k] = 0; return ORC_OK; }
  if (ensure_tmp(s, c) != ORC_OK) return ORC_E_NOMEM;
  int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * c);
  if (!idx) return ORC_E_NOMEM;
  for (int64_t q = 0; q < c; ++q) idx[q] = s->bids[b0 + q];
  double M, r[3], Iw[9], R[9];
  mass_props_set(s->dim, s->Ir_fac, c, idx, s->x, s->m, s->tmp, &M, r, Iw);
  s->bm[k] = M;
  for (int a = 0; a < 3; ++a) s->br[3 * k + a] = r[a];
  quat_to_rot(&s->bq[4 * k], R);
  if (s->dim == 3) rot_sandwich(R, Iw, 1, &s->bIb[9 * k]);
  else { for (int q = 0; q < 9; ++q) s->bIb[9 * k + q] = 0.0; s->bIb[9 * k + 8] = Iw[8]; }
  for (int64_t q = 0; q < c; ++q) {
    int64_t i = idx[q];
    double dd[3];
    for (int a = 0; a < 3; ++a) dd[a] = (a < s->dim) ? s->x[3 * i + a] - r[a] : 0.0;
    for (int a = 0; a < 3; ++a) s->rk[3 * i + a] = dd[a];
    matT_vec(R, dd, &s->rb[3 * i]);
    if (s->dim == 2) s->rb[3 * i + 2] = 0.0;
  }
  free(idx);
  s->bactive[k] = 1;
  return ORC_OK;
}

/* Rigid particle positions and velocities from their body (the drift step
 * of Sec. "Time integration"): r_rk = R(q_k) r_rk^b, x_r = r_k + r_rk,
 * u_r = u_k + omega_k x r_rk. */
/* a position along the periodic axes back into [lo, lo + period) */
static void wrap_pos(const orc_scene *s, double *x) {
  for (int a = 1; a < s->dim; ++a) {
    if (!s->per[a]) continue;
    if (x[a] >= s->lo[a] + s->period[a]) x[a] = x[a] - s->period[a];
    else if (x[a] < s->lo[a]) x[a] = x[a] + s->period[a];
  }
}

static void rigid_pose(orc_scene *s) {
  for (int k = 0; k < s->nb; ++k) {
    if (!s->bactive[k]) continue;
    double R[9];
    quat_to_rot(&s->bq[4 * k], R);
    for (int64_t q = s->bstart[k]; q < s->bstart[k + 1]; ++q) {
      int64_t i = s->bids[q];
      double rk[3], wr[3];
      mat_vec(R, &s->rb[3 * i], rk);
      if (s->dim == 2) rk[2] = 0.0;
      cross3(&s->bw[3 * k], rk, wr);
      for (int a = 0; a < 3; ++a) {
        s->rk[3 * i + a] = rk[a];
        s->x[3 * i + a] = (a < s->dim) ? s->br[3 * k + a] + rk[a] : 0.0;
      }
      wrap_pos(s, &s->x[3 * i]);
      for (int a = 0; a < 3; ++a) s->u[3 * i + a] = (a < s->dim) ? s->bu[3 * k + a] + wr[a] : 0.0;
    }
  }
}

static void rigid_velocities(orc_scene *s) {
  for (int k = 0; k < s->nb; ++k) {
    if (!s->bactive[k]) continue;
    for (int64_t q = s->bstart[k]; q < s->bstart[k + 1]; ++q) {
      int64_t i = s->bids[q];
      double wr[3];
      cross3(&s->bw[3 * k], &s->rk[3 * i], wr);
      for (int a = 0; a < 3; ++a) s->u[3 * i + a] = (a < s->dim) ? s->bu[3 * k + a] + wr[a] : 0.0;
    }
  }
}

/* Eqs. procwise_force / global_force with one partition: f_k = sum_r f_r,
 * m_k = sum_r r_rk x f_r, both as exact sums rounded once. */
static int stage_body_sums(orc_scene *s) {
  for (int k = 0; k < s->nb; ++k) {
    for (int a = 0; a < 3; ++a) { s->bf[3 * k + a] = 0.0; s->bt[3 * k + a] = 0.0; }
    if (!s->bactive[k]) continue;
    int64_t b0 = s->bstart[k], c = s->bstart[k + 1] - b0;
    if (ensure_tmp(s, c) != ORC_OK) return ORC_E_NOMEM;
    for (int a = 0; a < s->dim; ++a) {
      for (int64_t q = 0; q < c; ++q) s->tmp[q] = s->f[3 * s->bids[b0 + q] + a];
      s->bf[3 * k + a] = orc_fsum(s->tmp, c);
    }
    for (int a = (s->dim == 3 ? 0 : 2); a < 3; ++a) {
      for (int64_t q = 0; q < c; ++q) {
        int64_t i = s->bids[b0 + q];
        double tq[3];
        cross3(&s->rk[3 * i], &s->f[3 * i], tq);
        s->tmp[q] = tq[a];
      }
      s->bt[3 * k + a] = orc_fsum(s->tmp, c);
    }
  }
  return ORC_OK;
}

/* Balance of linear and angular momentum (eqs. goveq_solid_linearmomentum
 * and _angularmomentum): a_k = f_k/m_k + b_k, alpha_k = I^{-1} m_k with the
 * world-frame inertia R I^b R^T, no gyroscopic term (as printed). */
static void stage_body_acc(orc_scene *s) {
  for (int k = 0; k < s->nb; ++k) {
    double *ak = &s->ba[3 * k], *al = &s->bal[3 * k];
    if (!s->bactive[k] || s->bfixed[k]) {
      for (int a = 0; a < 3; ++a) { ak[a] = 0.0; al[a] = 0.0; }
      continue;
    }
    for (int a = 0; a < 3; ++a) ak[a] = (a < s->dim) ? s->bf[3 * k + a] / s->bm[k] + s->bb[3 * k + a] : 0.0;
    const double *tq = &s->bt[3 * k];
    if (s->dim == 2) {
      al[0] = 0.0; al[1] = 0.0;
      al[2] = tq[2] / s->bIb[9 * k + 8];
    } else {
      double R[9], I[9];
      quat_to_rot(&s->bq[4 * k], R);
      rot_sandwich(R, &s->bIb[9 * k], 0, I);
      double c00 = I[4] * I[8] - I[5] * I[7];
      double c01 = I[5] * I[6] - I[3] * I[8];
      double c02 = I[3] * I[7] - I[4] * I[6];
      double det = I[0] * c00 + I[1] * c01 + I[2] * c02;
      double inv[9];
      inv[0] = c00 / det;
      inv[1] = (I[2] * I[7] - I[1] * I[8]) / det;
      inv[2] = (I[1] * I[5] - I[2] * I[4]) / det;
      inv[3] = c01 / det;
      inv[4] = (I[0] * I[8] - I[2] * I[6]) / det;
      inv[5] = (I[2] * I[3] - I[0] * I[5]) / det;
      inv[6] = c02 / det;
      inv[7] = (I[1] * I[6] - I[0] * I[7]) / det;
      inv[8] = (I[0] * I[4] - I[1] * I[3]) / det;
      mat_vec(inv, tq, al);
    }
  }
}

/* ------------------------------------------------------------------------ */
/* reversible phase transition (Sec. "Modeling thermally driven reversible  */
/* phase transitions")                                                       */
/* ------------------------------------------------------------------------ */

static int32_t uf_find(int32_t *lab, int32_t i) {
  while (lab[i] != i) { lab[i] = lab[lab[i]]; i = lab[i]; }
  return i;
}

/* A rigid particle above T_t of its phase melts into the partner fluid
 * phase; a fluid particle below T_t of its phase solidifies into the
 * partner solid phase (strict comparisons; phases without a partner never
 * switch).  A solidifying particle joins the body of its nearest rigid
 * neighbour within r_c (ties: lower body id, then lower particle id);
 * solidifying particles without one form new bodies, one per connected
 * component under r < r_c, numbered in ascending order of the component's
 * smallest id.  Bodies that changed get new mass quantities and offsets;
 * their velocity follows rigid body motion with unchanged omega,
 * u_k = u'_k + omega_k x (r_k - r'_k). */
static int stage_phase_switch(orc_scene *s) {
  int64_t n = s->n;
  int8_t *flag = (int8_t *)calloc(n, 1);
  int32_t *target = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
  int32_t *lab = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
  int8_t *dirty = (int8_t *)calloc(s->maxb > 0 ? s->maxb : 1, 1);
  double *rold = (double *)malloc(sizeof(double) * 3 * (s->maxb > 0 ? s->maxb : 1));
  int st = ORC_OK;
  if (!flag || !target || !lab || !dirty || !rold) { st = ORC_E_NOMEM; goto done; }
  int64_t nflag = 0;
  for (int64_t i = 0; i < n; ++i) {
    const orc_material *M = &s->mat[s->phase[i]];
    if (M->switch_to < 0) continue;
    if (s->kind[i] == ORC_RIGID && s->T[i] > M->T_t) { flag[i] = 1; nflag++; }
    else if (s->kind[i] == ORC_FLUID && s->T[i] < M->T_t) { flag[i] = 2; nflag++; }
  }
  if (nflag == 0) goto done;
  for (int k = 0; k < s->maxb; ++k) { rold[3 * k] = s->br[3 * k]; rold[3 * k + 1] = s->br[3 * k + 1]; rold[3 * k + 2] = s->br[3 * k + 2]; }
  /* melting */
  for (int64_t i = 0; i < n; ++i) {
    if (flag[i] != 1) continue;
    int k = s->body[i];
    double acc[3];
    rigid_point_acc(s, i, acc);
    for (int a = 0; a < 3; ++a) s->a[3 * i + a] = (a < s->dim) ? acc[a] : 0.0;
    s->kind[i] = ORC_FLUID;
    s->phase[i] = s->mat[s->phase[i]].switch_to;
    s->body[i] = -1;
    dirty[k] = 1;
  }
  /* solidification: nearest rigid neighbour */
  for (int64_t i = 0; i < n; ++i) {
    target[i] = -1;
    lab[i] = (int32_t)i;
    if (flag[i] != 2) continue;
    int64_t cnt = gather(s, i, 0);
    int64_t best = -1;
    double br2 = 0.0;
    for (int64_t k = 0; k < cnt; ++k) {
      const nb_t *e = &s->nbuf[k];
      int32_t j = e->j;
      if (s->kind[j] != ORC_RIGID) continue;
      if (best < 0 || e->r2 < br2 ||
          (e->r2 == br2 && (s->body[j] < s->body[best] || (s->body[j] == s->body[best] && j < best)))) {
        best = j; br2 = e->r2;
      }
    }
    if (best >= 0) target[i] = s->body[best];
  }
  /* components of the solidifying particles left without a body */
  for (int64_t i = 0; i < n; ++i) {
    if (flag[i] != 2 || target[i] >= 0) continue;
    int64_t cnt = gather(s, i, 0);
    for (int64_t k = 0; k < cnt; ++k) {
      int32_t j = s->nbuf[k].j;
      if (flag[j] != 2 || target[j] >= 0) continue;
      int32_t ra = uf_find(lab, (int32_t)i), rb = uf_find(lab, j);
      if (ra < rb) lab[rb] = ra; else if (rb < ra) lab[ra] = rb;
    }
  }
  /* roots are the smallest ids of their components; new body ids follow
   * ascending root order */
  int kfirst_new = s->nb;
  for (int64_t i = 0; i < n; ++i) {
    if (flag[i] != 2 || target[i] >= 0) continue;
    int32_t r = uf_find(lab, (int32_t)i);
    if (r == i) {
      if (s->nb >= s->maxb) { st = ORC_E_STATE; goto done; }
      int k = s->nb++;
      const orc_material *M = &s->mat[s->phase[i]];
      const orc_material *Ms = &s->mat[M->switch_to];
      s->bq[4 * k] = 1.0; s->bq[4 * k + 1] = 0.0; s->bq[4 * k + 2] = 0.0; s->bq[4 * k + 3] = 0.0;
      for (int a = 0; a < 3; ++a) {
        s->bw[3 * k + a] = 0.0; s->bal[3 * k + a] = 0.0;
        s->bb[3 * k + a] = (a < s->dim) ? Ms->b[a] : 0.0;
      }
      s->bfixed[k] = 0;
      s->bactive[k] = 1;
      target[i] = k;
    }
  }
  for (int64_t i = 0; i < n; ++i) {
    if (flag[i] != 2 || target[i] >= 0) continue;
    int32_t r = uf_find(lab, (int32_t)i);
    target[i] = target[r];
    if (target[i] < 0) { st = ORC_E_STATE; goto done; }
  }
  for (int64_t i = 0; i < n; ++i) {
    if (flag[i] != 2) continue;
    s->kind[i] = ORC_RIGID;
    s->phase[i] = s->mat[s->phase[i]].switch_to;
    s->body[i] = target[i];
    dirty[target[i]] = 1;
  }
  if ((st = build_body_lists(s)) != ORC_OK) goto done;
  for (int k = kfirst_new; k < s->nb; ++k) {
    int64_t b0 = s->bstart[k], c = s->bstart[k + 1] - b0;
    if (c == 0) continue;
    if (ensure_tmp(s, c) != ORC_OK) { st = ORC_E_NOMEM; goto done; }
    for (int64_t q = 0; q < c; ++q) s->tmp[q] = s->m[s->bids[b0 + q]];
    double M = orc_fsum(s->tmp, c);
    for (int a = 0; a < 3; ++a) {
      if (a >= s->dim) { s->bu[3 * k + a] = 0.0; s->ba[3 * k + a] = 0.0; continue; }
      for (int64_t q = 0; q < c; ++q) { int64_t i = s->bids[b0 + q]; s->tmp[q] = s->m[i] * s->u[3 * i + a]; }
      s->bu[3 * k + a] = orc_fsum(s->tmp, c) / M;
      for (int64_t q = 0; q < c; ++q) { int64_t i = s->bids[b0 + q]; s->tmp[q] = s->m[i] * s->a[3 * i + a]; }
      s->ba[3 * k + a] = orc_fsum(s->tmp, c) / M;
    }
  }
  for (int k = 0; k < s->nb; ++k) {
    if (!dirty[k]) continue;
    int was_new = (k >= kfirst_new);
    if ((st = body_recompute(s, k)) != ORC_OK) goto done;
    if (!s->bactive[k]) continue;
    if (!was_new) {
      double dr[3], wr[3];
      for (int a = 0; a < 3; ++a) dr[a] = s->br[3 * k + a] - rold[3 * k + a];
      cross3(&s->bw[3 * k], dr, wr);
      for (int a = 0; a < s->dim; ++a) s->bu[3 * k + a] = s->bu[3 * k + a] + wr[a];
    }
  }
  rigid_velocities(s);
done:
  free(flag); free(target); free(lab); free(dirty); free(rold);
  return st;
}

/* ------------------------------------------------------------------------ */
/* create / step                                                             */
/* ------------------------------------------------------------------------ */

void orc_destroy(orc_scene *s) {
  if (!s) return;
  double *dp[] = {s->x, s->u, s->a, s->rho, s->p, s->T, s->dTdt, s->m, s->pw, s->uw, s->f, s->rb,
                  s->rk, s->aw, s->x0, s->bm, s->br, s->bq, s->bu, s->bw, s->ba, s->bal, s->bf,
                  s->bt, s->bIb, s->bb, s->tmp, s->ab, s->ud};
  for (size_t k = 0; k < sizeof(dp) / sizeof(dp[0]); ++k) free(dp[k]);
  free(s->kind); free(s->phase); free(s->body); free(s->moving); free(s->cell);
  free(s->cstart); free(s->cids); free(s->mat); free(s->bfixed); free(s->bactive);
  free(s->bstart); free(s->bids); free(s->nbuf);
  free(s);
}

static int evaluate(orc_scene *s, int with_heat) {
  int st;
  if ((st = build_cells(s)) != ORC_OK) return st;
  stage_density(s);
  stage_extrapolate(s);
  if (s->thermal && with_heat && (st = stage_heat(s, 1)) != ORC_OK) return st;
  if ((st = stage_forces(s)) != ORC_OK) return st;
  if ((st = stage_body_sums(s)) != ORC_OK) return st;
  stage_body_acc(s);
  return ORC_OK;
}

int orc_create(const orc_desc *d, orc_scene **out) {
  if (!d || !out) return ORC_E_INVALID;
  *out = NULL;
  if ((d->dim != 2 && d->dim != 3) || !(d->dx > 0.0) || d->n < 0 || d->n_mat <= 0 || d->n_body < 0)
    return ORC_E_INVALID;
  int64_t n = d->n;
  for (int64_t i = 0; i < n; ++i) {
    if (d->kind[i] < 0 || d->kind[i] > 2 || d->phase[i] < 0 || d->phase[i] >= d->n_mat) return ORC_E_INVALID;
    if (d->kind[i] == ORC_RIGID && (d->body[i] < 0 || d->body[i] >= d->n_body)) return ORC_E_INVALID;
    for (int a = 0; a < 3; ++a) if (!isfinite(d->x[3 * i + a]) || !isfinite(d->u[3 * i + a])) return ORC_E_INVALID;
  }
  orc_scene *s = (orc_scene *)calloc(1, sizeof(orc_scene));
  if (!s) return ORC_E_NOMEM;
  s->dim = d->dim;
  s->dx = d->dx; s->h = d->dx; s->rc = 3.0 * s->h; s->rc2 = s->rc * s->rc;
  s->L = d->cell_edge > 0.0 ? d->cell_edge : s->rc;
  if (s->L < s->rc) { free(s); return ORC_E_INVALID; }
  s->ncells = 1;
  for (int a = 0; a < 3; ++a) {
    s->lo[a] = d->lo[a];
    if (a < s->dim) {
      double ext = d->hi[a] - d->lo[a];
      if (!(ext > 0.0)) { free(s); return ORC_E_INVALID; }
      int nc = (int)ceil(ext / s->L * (1.0 - 1e-12));
      s->nc[a] = nc < 1 ? 1 : nc;
    } else {
      s->nc[a] = 1;
    }
    s->ncells *= s->nc[a];
  }
  double sg = sigma_d(s->dim);
  s->wnorm = sg / pow_d(s->h, s->dim);
  s->dnorm = -5.0 * sg / pow_d(s->h, s->dim + 1);
  s->vol0 = pow_d(s->dx, s->dim);
  s->Ir_fac = particle_inertia_factor(s->dim, s->dx);
  s->n = n;
  size_t v3 = sizeof(double) * 3 * (size_t)(n > 0 ? n : 1), v1 = sizeof(double) * (size_t)(n > 0 ? n : 1);
  size_t i1 = sizeof(int32_t) * (size_t)(n > 0 ? n : 1);
  s->x = (double *)malloc(v3); s->u = (double *)malloc(v3); s->a = (double *)calloc(1, v3);
  s->uw = (double *)calloc(1, v3); s->f = (double *)calloc(1, v3); s->rb = (double *)calloc(1, v3);
  s->rk = (double *)calloc(1, v3); s->aw = (double *)calloc(1, v3); s->x0 = (double *)malloc(v3);
  s->ab = (double *)calloc(1, v3); s->ud = (double *)calloc(1, v3);
  s->rho = (double *)calloc(1, v1); s->p = (double *)calloc(1, v1); s->T = (double *)malloc(v1);
  s->dTdt = (double *)calloc(1, v1); s->m = (double *)malloc(v1); s->pw = (double *)calloc(1, v1);
  s->kind = (int32_t *)malloc(i1); s->phase = (int32_t *)malloc(i1); s->body = (int32_t *)malloc(i1);
  s->moving = (int32_t *)malloc(i1); s->cell = (int32_t *)malloc(i1);
  s->cstart = (int64_t *)malloc(sizeof(int64_t) * (size_t)(s->ncells + 1));
  s->cids = (int32_t *)malloc(i1);
  s->n_mat = d->n_mat;
  s->mat = (orc_material *)malloc(sizeof(orc_material) * d->n_mat);
  s->nb = d->n_body;
  s->maxb = d->max_bodies > d->n_body ? d->max_bodies : d->n_body;
  int mb = s->maxb > 0 ? s->maxb : 1;
  s->bm = (double *)calloc(mb, sizeof(double)); s->br = (double *)calloc(3 * mb, sizeof(double));
  s->bq = (double *)calloc(4 * mb, sizeof(double)); s->bu = (double *)calloc(3 * mb, sizeof(double));
  s->bw = (double *)calloc(3 * mb, sizeof(double)); s->ba = (double *)calloc(3 * mb, sizeof(double));
  s->bal = (double *)calloc(3 * mb, sizeof(double)); s->bf = (double *)calloc(3 * mb, sizeof(double));
  s->bt = (double *)calloc(3 * mb, sizeof(double)); s->bIb = (double *)calloc(9 * mb, sizeof(double));
  s->bb = (double *)calloc(3 * mb, sizeof(double));
  s->bfixed = (int32_t *)calloc(mb, sizeof(int32_t)); s->bactive = (int32_t *)calloc(mb, sizeof(int32_t));
  s->bstart = (int64_t *)calloc(mb + 1, sizeof(int64_t)); s->bids = (int32_t *)malloc(i1);
  if (!s->x || !s->u || !s->a || !s->ab || !s->ud || !s->uw || !s->f || !s->rb || !s->rk || !s->aw || !s->x0 || !s->rho ||
      !s->p || !s->T || !s->dTdt || !s->m || !s->pw || !s->kind || !s->phase || !s->body || !s->moving ||
      !s->cell || !s->cstart || !s->cids || !s->mat || !s->bm || !s->br || !s->bq || !s->bu || !s->bw ||
      !s->ba || !s->bal || !s->bf || !s->bt || !s->bIb || !s->bb || !s->bfixed || !s->bactive ||
      !s->bstart || !s->bids) {
    orc_destroy(s);
    return ORC_E_NOMEM;
  }
  memcpy(s->mat, d->mat, sizeof(orc_material) * d->n_mat);
  for (int64_t i = 0; i < n; ++i) {
    for (int a = 0; a < 3; ++a) {
      s->x[3 * i + a] = (a < s->dim) ? d->x[3 * i + a] : 0.0;
      s->u[3 * i + a] = (a < s->dim) ? d->u[3 * i + a] : 0.0;
    }
    s->T[i] = d->T ? d->T[i] : 0.0;
    s->kind[i] = d->kind[i];
    s->phase[i] = d->phase[i];
    s->body[i] = d->kind[i] == ORC_RIGID ? d->body[i] : -1;
    s->moving[i] = (d->kind[i] == ORC_WALL && d->moving) ? d->moving[i] : 0;
    /* Sec. "Initial particle spacing": m = rho0 of the phase times dx^d */
    s->m[i] = s->mat[s->phase[i]].rho0 * s->vol0;
  }
  memcpy(s->x0, s->x, v3);
  s->thermal = d->thermal; s->contact = d->contact; s->pswitch = d->phase_switch;
  s->wall_A = d->wall_A; s->wall_Om = d->wall_Omega;
  for (int a = 0; a < 3; ++a) s->wall_dir[a] = d->wall_dir[a];
  s->heat_src = d->heat_src; s->sQ = d->src_Q; s->ssig = d->src_sigma;
  s->ss0[0] = d->src_s0[0]; s->ss0[1] = d->src_s0[1]; s->sv[0] = d->src_v[0]; s->sv[1] = d->src_v[1];
  s->sztop = d->src_ztop; s->sdepth = d->src_depth;
  s->tvf = d->p_b > 0.0;
  s->pb = s->tvf ? d->p_b : 0.0;
  /* periodic axes: y and z only, a whole number (>= 3) of cells per period,
   * no phase switching (the body quantities of a switch are not taken
   * across the boundary) */
  for (int a = 0; a < 3; ++a) {
    s->per[a] = (a < s->dim) ? (d->periodic[a] != 0) : 0;
    s->period[a] = s->per[a] ? d->hi[a] - d->lo[a] : 0.0;
    if (!s->per[a]) continue;
    double whole = (double)s->nc[a] * s->L;
    if (a == 0 || s->nc[a] < 3 || fabs(whole - s->period[a]) > 1e-9 * s->period[a] || d->phase_switch) {
      orc_destroy(s);
      return ORC_E_INVALID;
    }
  }
  /* time step and contact constants */
  double mmin;
  double dt0 = timestep_without_contact(d, &mmin);
  s->dt = d->dt > 0.0 ? d->dt : orc_timestep(d);
  if (d->k_c >= 0.0) s->kc = d->k_c;
  else if (isfinite(mmin)) { double b = 0.22 / (2.0 * (d->dt > 0.0 ? d->dt : dt0)); s->kc = mmin * (b * b); }
  else s->kc = 0.0;
  if (d->d_c >= 0.0) s->dc = d->d_c;
  else s->dc = isfinite(mmin) ? 0.2 * sqrt(s->kc * mmin / 2.0) : 0.0;
  if (!(s->dt > 0.0) || !isfinite(s->dt)) { orc_destroy(s); return ORC_E_INVALID; }
  /* bodies */
  int st = build_body_lists(s);
  if (st != ORC_OK) { orc_destroy(s); return st; }
  for (int k = 0; k < s->nb; ++k) {
    const orc_body_init *B = &d->bodies[k];
    double qn = sqrt(B->q[0] * B->q[0] + B->q[1] * B->q[1] + B->q[2] * B->q[2] + B->q[3] * B->q[3]);
    for (int a = 0; a < 4; ++a) s->bq[4 * k + a] = B->q[a] / qn;
    for (int a = 0; a < 3; ++a) {
      s->bu[3 * k + a] = (a < s->dim) ? B->u[a] : 0.0;
      s->bw[3 * k + a] = (s->dim == 3 || a == 2) ? B->w[a] : 0.0;
    }
    s->bfixed[k] = B->fixed;
    if (s->bstart[k + 1] > s->bstart[k]) {
      const orc_material *M = &s->mat[s->phase[s->bids[s->bstart[k]]]];
      for (int a = 0; a < 3; ++a) s->bb[3 * k + a] = (a < s->dim) ? M->b[a] : 0.0;
    }
    if ((st = body_recompute(s, k)) != ORC_OK) { orc_destroy(s); return st; }
  }
  rigid_velocities(s);
  for (int64_t i = 0; i < n; ++i)
    if (s->moving[i]) for (int a = 0; a < 3; ++a) s->u[3 * i + a] = 0.0;
  /* body quantities came from the positions as given (a body may extend
   * across a periodic boundary); every position now into the periodic box */
  for (int64_t i = 0; i < n; ++i) wrap_pos(s, &s->x[3 * i]);
  /* one evaluation without time update gives a^0 and the body accelerations */
  st = evaluate(s, 0);
  if (st != ORC_OK) { orc_destroy(s); return st; }
  *out = s;
  return ORC_OK;
}

/* Moving boundary particles: displacement A (cos(Omega t) - 1) along a unit
 * direction, with its velocity and acceleration. */
static void wall_motion(orc_scene *s, double t) {
  double sA = s->wall_A * (cos(s->wall_Om * t) - 1.0);
  double vA = -s->wall_A * s->wall_Om * sin(s->wall_Om * t);
  double aA = -s->wall_A * s->wall_Om * s->wall_Om * cos(s->wall_Om * t);
  for (int64_t i = 0; i < s->n; ++i) {
    if (!s->moving[i]) continue;
    for (int a = 0; a < s->dim; ++a) {
      s->x[3 * i + a] = s->x0[3 * i + a] + sA * s->wall_dir[a];
      s->u[3 * i + a] = vA * s->wall_dir[a];
      s->aw[3 * i + a] = aA * s->wall_dir[a];
    }
    wrap_pos(s, &s->x[3 * i]);
  }
}

/* One time step, Sec. "Time integration following a velocity-Verlet
 * scheme" (kick, drift, interaction, kick) followed by the phase switch. */
static int one_step(orc_scene *s) {
  double hdt = 0.5 * s->dt;
  int st;
  /* kick */
  for (int64_t i = 0; i < s->n; ++i)
    if (s->kind[i] == ORC_FLUID)
      for (int a = 0; a < s->dim; ++a) s->u[3 * i + a] = s->u[3 * i + a] + hdt * s->a[3 * i + a];
  for (int k = 0; k < s->nb; ++k) {
    if (!s->bactive[k] || s->bfixed[k]) continue;
    for (int a = 0; a < 3; ++a) {
      s->bu[3 * k + a] = s->bu[3 * k + a] + hdt * s->ba[3 * k + a];
      s->bw[3 * k + a] = s->bw[3 * k + a] + hdt * s->bal[3 * k + a];
    }
  }
  /* drift; with the transport-velocity formulation fluid particles move
   * with u~^{n+1/2} = u^{n+1/2} + (dt/2) a_b^n */
  for (int64_t i = 0; i < s->n; ++i)
    if (s->kind[i] == ORC_FLUID) {
      for (int a = 0; a < s->dim; ++a) {
        double v = s->u[3 * i + a];
        if (s->tvf) {
          s->ud[3 * i + a] = hdt * s->ab[3 * i + a];
          v = v + s->ud[3 * i + a];
        }
        s->x[3 * i + a] = s->x[3 * i + a] + s->dt * v;
      }
      wrap_pos(s, &s->x[3 * i]);
    }
  for (int k = 0; k < s->nb; ++k) {
    if (!s->bactive[k] || s->bfixed[k]) continue;
    for (int a = 0; a < 3; ++a) s->br[3 * k + a] = s->br[3 * k + a] + s->dt * s->bu[3 * k + a];
    /* transition quaternion of the increment phi = dt omega^{n+1/2} and
     * q^{n+1} = q^{n,n+1} o q^n, renormalised */
    double phi[3] = {s->dt * s->bw[3 * k], s->dt * s->bw[3 * k + 1], s->dt * s->bw[3 * k + 2]};
    double ang = sqrt(phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2]);
    if (ang > 0.0) {
      double sh = sin(0.5 * ang) / ang;
      double qi[4] = {cos(0.5 * ang), sh * phi[0], sh * phi[1], sh * phi[2]};
      double qn[4];
      quat_mul(qi, &s->bq[4 * k], qn);
      double nq = sqrt(qn[0] * qn[0] + qn[1] * qn[1] + qn[2] * qn[2] + qn[3] * qn[3]);
      for (int a = 0; a < 4; ++a) s->bq[4 * k + a] = qn[a] / nq;
    }
  }
  s->step += 1;
  s->t = (double)s->step * s->dt;
  wall_motion(s, s->t);
  rigid_pose(s);
  /* densities, extrapolation, temperatures, forces, body sums */
  if ((st = evaluate(s, 1)) != ORC_OK) return st;
  /* kick */
  for (int64_t i = 0; i < s->n; ++i)
    if (s->kind[i] == ORC_FLUID)
      for (int a = 0; a < s->dim; ++a) s->u[3 * i + a] = s->u[3 * i + a] + hdt * s->a[3 * i + a];
  for (int k = 0; k < s->nb; ++k) {
    if (!s->bactive[k] || s->bfixed[k]) continue;
    for (int a = 0; a < 3; ++a) {
      s->bu[3 * k + a] = s->bu[3 * k + a] + hdt * s->ba[3 * k + a];
      s->bw[3 * k + a] = s->bw[3 * k + a] + hdt * s->bal[3 * k + a];
    }
  }
  rigid_velocities(s);
  if (s->pswitch && (st = stage_phase_switch(s)) != ORC_OK) return st;
  for (int64_t i = 0; i < s->n; ++i)
    for (int a = 0; a < s->dim; ++a)
      if (!isfinite(s->x[3 * i + a]) || !isfinite(s->u[3 * i + a])) return ORC_E_STATE;
  return ORC_OK;
}

int orc_step(orc_scene *s, int64_t nsteps) {
  if (!s || nsteps < 0) return ORC_E_INVALID;
  for (int64_t k = 0; k < nsteps; ++k) {
    int st = one_step(s);
    if (st != ORC_OK) return st;
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* accessors                                                                 */
/* ------------------------------------------------------------------------ */

double orc_get_dt(const orc_scene *s) { return s->dt; }
double orc_get_time(const orc_scene *s) { return s->t; }
double orc_get_kc(const orc_scene *s) { return s->kc; }
double orc_get_dc(const orc_scene *s) { return s->dc; }
int32_t orc_n_bodies(const orc_scene *s) { return s->nb; }
int64_t orc_pair_count(const orc_scene *s) { return s->pairs; }
int orc_grid(const orc_scene *s, int32_t *nc) { nc[0] = s->nc[0]; nc[1] = s->nc[1]; nc[2] = s->nc[2]; return ORC_OK; }

static double *field_ptr(const orc_scene *s, int32_t f, int *width) {
  *width = 1;
  switch (f) {
    case ORC_F_X: *width = 3; return s->x;
    case ORC_F_U: *width = 3; return s->u;
    case ORC_F_A: *width = 3; return s->a;
    case ORC_F_RHO: return s->rho;
    case ORC_F_P: return s->p;
    case ORC_F_T: return s->T;
    case ORC_F_PW: return s->pw;
    case ORC_F_UW: *width = 3; return s->uw;
    case ORC_F_FR: *width = 3; return s->f;
    case ORC_F_M: return s->m;
    case ORC_F_DTDT: return s->dTdt;
    case ORC_F_AB: *width = 3; return s->ab;
    case ORC_F_UD: *width = 3; return s->ud;
    default: return NULL;
  }
}
int orc_get(const orc_scene *s, int32_t f, double *out) {
  int w;
  double *p = field_ptr(s, f, &w);
  if (!p) return ORC_E_INVALID;
  memcpy(out, p, sizeof(double) * w * (size_t)s->n);
  return ORC_OK;
}
int orc_set(orc_scene *s, int32_t f, const double *in) {
  int w;
  double *p = field_ptr(s, f, &w);
  if (!p) return ORC_E_INVALID;
  memcpy(p, in, sizeof(double) * w * (size_t)s->n);
  return ORC_OK;
}
int orc_get_int(const orc_scene *s, int32_t f, int32_t *out) {
  const int32_t *p = NULL;
  if (f == ORC_I_KIND) p = s->kind;
  else if (f == ORC_I_PHASE) p = s->phase;
  else if (f == ORC_I_BODY) p = s->body;
  else if (f == ORC_I_CELL) p = s->cell;
  if (!p) return ORC_E_INVALID;
  memcpy(out, p, sizeof(int32_t) * (size_t)s->n);
  return ORC_OK;
}
int orc_get_bodies(const orc_scene *s, double *out) {
  for (int k = 0; k < s->nb; ++k) {
    double *o = &out[ORC_BODY_REC * k];
    for (int q = 0; q < ORC_BODY_REC; ++q) o[q] = 0.0;
    o[0] = s->bm[k];
    for (int a = 0; a < 3; ++a) {
      o[1 + a] = s->br[3 * k + a]; o[8 + a] = s->bu[3 * k + a]; o[11 + a] = s->bw[3 * k + a];
      o[14 + a] = s->ba[3 * k + a]; o[17 + a] = s->bal[3 * k + a]; o[20 + a] = s->bf[3 * k + a];
      o[23 + a] = s->bt[3 * k + a];
    }
    for (int a = 0; a < 4; ++a) o[4 + a] = s->bq[4 * k + a];
    if (s->dim == 3) {
      double R[9], I[9];
      quat_to_rot(&s->bq[4 * k], R);
      rot_sandwich(R, &s->bIb[9 * k], 0, I);
      o[26] = I[0]; o[27] = I[4]; o[28] = I[8]; o[29] = I[1]; o[30] = I[2]; o[31] = I[5];
    } else {
      o[28] = s->bIb[9 * k + 8];
    }
    o[32] = s->bactive[k];
    o[33] = s->bfixed[k];
  }
  return ORC_OK;
}

int orc_stage(orc_scene *s, int32_t stage) {
  switch (stage) {
    case ORC_S_NEIGHBORS: return build_cells(s);
    case ORC_S_DENSITY: stage_density(s); return ORC_OK;
    case ORC_S_EXTRAP: stage_extrapolate(s); return ORC_OK;
    case ORC_S_HEAT: return stage_heat(s, 0);
    case ORC_S_FORCES: return stage_forces(s);
    case ORC_S_BODYSUMS: return stage_body_sums(s);
    case ORC_S_BODYACC: stage_body_acc(s); return ORC_OK;
    default: return ORC_E_INVALID;
  }
}

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

int64_t orc_neighbors(orc_scene *s, int64_t *offsets, int32_t *ids, int64_t cap) {
  if (build_cells(s) != ORC_OK) return -1;
  int64_t tot = 0;
  for (int64_t i = 0; i < s->n; ++i) {
    if (offsets) offsets[i] = tot;
    int64_t cnt = gather(s, i, 0);
    if (ids && tot + cnt <= cap) {
      for (int64_t k = 0; k < cnt; ++k) ids[tot + k] = s->nbuf[k].j;
      qsort(&ids[tot], (size_t)cnt, sizeof(int32_t), cmp_i32);
    }
    tot += cnt;
  }
  if (offsets) offsets[s->n] = tot;
  return tot;
}

int orc_cell_order(orc_scene *s, int32_t *sorted_ids, int32_t *cell_of_id) {
  int st = build_cells(s);
  if (st != ORC_OK) return st;
  if (sorted_ids) memcpy(sorted_ids, s->cids, sizeof(int32_t) * (size_t)s->n);
  if (cell_of_id) memcpy(cell_of_id, s->cell, sizeof(int32_t) * (size_t)s->n);
  return ORC_OK;
}
