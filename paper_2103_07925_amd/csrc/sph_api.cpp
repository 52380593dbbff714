// sph_api.cpp -- host implementation of the C ABI declared in include/sphrb.h.
//
// Owns no device memory: every device array of a scene is carved out of the
// caller's arena.  Set-up bookkeeping (validation, layout, slot order,
// material constants, time step) runs on the host; every step of the
// method runs in the kernels of sph_kernels.hip, enqueued on the scene's
// stream without host round trips.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/sphrb.h"
#include "sph_internal.h"

using namespace sphrb;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

#define HIP_TRY(expr)                                                                 \
  do {                                                                                \
    hipError_t _e = (expr);                                                           \
    if (_e != hipSuccess) return fail(SPH_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

constexpr double kPi = 3.14159265358979323846;
constexpr int kGlobalBlocks = 256;

size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

// Arena carving: the same sequence of requests sizes the arena and places
// the arrays in it.
struct Carver {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = align_up(off);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += sizeof(T) * (count > 0 ? count : 1);
    return p;
  }
};

double sigma_d(int dim) {
  if (dim == 2) return 7.0 / (478.0 * kPi);
  return 1.0 / (120.0 * kPi);
}
double powi(double h, int d) {
  double r = h;
  for (int k = 1; k < d; ++k) r = r * h;
  return r;
}

}  // namespace

struct sph_scene {
  Params P;
  int precision;
  hipStream_t stream;
  char* arena;
  size_t arena_bytes;
  int64_t step;
  int64_t n_fluid, n_wall;
  // buffers (typed as void* / raw; cast by precision)
  void* pos[2];
  uint32_t* cell[2];
  void* u[2];
  void* a[2];
  void* T[2];
  void* m[2];
  uint32_t* id[2];
  uint32_t* info[2];
  int32_t* aux[2];
  int ip, iu, iT;
  void* ud[2];       // transport-velocity formulation: u~ - u (permuted with pos)
  void *rho, *p, *pw, *uw, *dTdt, *pv, *ab;
  SortBufs sb;
  uint32_t* cstart;
  V4<double> *s_rb, *s_rk, *s_f, *s_aw, *s_x;
  double* s_m;
  int32_t *s_sorted, *s_body;
  uint32_t* s_id;
  V4<double> *w_x0, *w_aw;
  int32_t* w_sorted;
  Body* bodies;
  void* mat;
  uint32_t* err;
  unsigned long long* pairs;
  Lists nb;
  uint32_t *wcount, *woff, *wbsum;
  uint32_t* dyn;     // device: [0] rigid particles, [1] bodies
  unsigned long long* dstep;   // device: steps begun
  double* matb;      // device: body force of every material (FP64)
  PhaseBufs ps;
  double* gpart;
  double* gout;
  // timers: SPH_TIMER_STAGES + 1 events per recorded step
  int timers;
  std::vector<hipEvent_t>* ev;
  int64_t rec;
};

// A batch: scenes grouped by (precision, dim, mode); each group's sweeps
// run as one launch over a table of slots in the caller's workspace.  The
// slot table of a step depends on the scenes' buffer parities, which repeat
// every two steps, so two tables per group are kept and re-uploaded only
// when a scene was stepped outside the batch.
int scene_mode(const sph_scene* s) { return (s->P.thermal ? 1 : 0) | (s->P.tvf ? 2 : 0); }

struct sph_batch {
  struct Group {
    int precision, dim, mode;        // mode: bit 0 thermal, bit 1 transport-velocity formulation
    std::vector<int> members;
    uint32_t blocks;
    size_t off[2];                   // table offsets in the workspace
    std::vector<char> host[2];       // table images (kept for the async upload)
    std::vector<int> key[2];         // buffer parities the tables were made for
  };
  std::vector<sph_scene*> scenes;
  std::vector<Group> groups;
  hipStream_t stream;
  char* ws;
  size_t ws_bytes;
  std::vector<hipEvent_t> ev;        // one per scene, plus one for the batch stream
  // One step of all scenes captured as a HIP graph, for each of the (at
  // most two) buffer-parity states the scenes go through; a later step in
  // the same state replays it.  Every launch argument of a step is fixed
  // by the parities (times come from the scenes' device step counters).
  struct Graph {
    std::vector<int> key;
    hipGraphExec_t exec;
  };
  std::vector<Graph> graphs;
  int use_graphs;
};

namespace {

int validate(const sph_scene_desc* d) {
  if (!d) return fail(SPH_E_INVALID, "null descriptor");
  if (d->dim != 2 && d->dim != 3) return fail(SPH_E_INVALID, "dim must be 2 or 3");
  if (d->precision != SPH_FP64 && d->precision != SPH_FP32_SWEEP) return fail(SPH_E_INVALID, "bad precision");
  if (!(d->dx > 0.0) || !std::isfinite(d->dx)) return fail(SPH_E_INVALID, "dx must be positive");
  if (d->n < 0 || d->n > 0x7fffffffLL) return fail(SPH_E_INVALID, "particle count out of range");
  if (d->n > 0 && (!d->x || !d->u || !d->kind || !d->phase)) return fail(SPH_E_INVALID, "missing particle arrays");
  if (d->n_mat <= 0 || d->n_mat > 256 || !d->mat) return fail(SPH_E_INVALID, "1..256 materials required");
  if (d->phase_switch && !d->thermal)
    return fail(SPH_E_INVALID, "phase switching needs the scalar (thermal) solver");
  if (d->thermal && d->n_mat > kLdsPhases)
    return fail(SPH_E_UNSUPPORTED, "a thermal scene has at most " + std::to_string(kLdsPhases) + " materials");
  for (int k = 0; k < d->n_mat; ++k)
    if (d->mat[k].switch_to >= kLdsPhases && d->phase_switch)
      return fail(SPH_E_UNSUPPORTED, "switch targets must be among the first " + std::to_string(kLdsPhases) +
                                         " materials");
  if (d->n_body < 0 || (d->n_body > 0 && !d->bodies)) return fail(SPH_E_INVALID, "bad bodies");
  if (std::max(d->max_bodies, d->n_body) > 65534) return fail(SPH_E_INVALID, "too many bodies");
  double rc = 3.0 * d->dx;
  double L = d->cell_edge > 0.0 ? d->cell_edge : rc;
  if (L < rc) return fail(SPH_E_INVALID, "cell edge must be at least r_c = 3 dx");
  for (int a = 0; a < d->dim; ++a)
    if (!(d->hi[a] > d->lo[a])) return fail(SPH_E_INVALID, "empty domain");
  for (int k = 0; k < d->n_mat; ++k) {
    const sph_material& M = d->mat[k];
    if (!(M.rho0 > 0.0)) return fail(SPH_E_INVALID, "material density must be positive");
    if (M.switch_to >= d->n_mat) return fail(SPH_E_INVALID, "switch_to out of range");
  }
  for (int64_t i = 0; i < d->n; ++i) {
    int k = d->kind[i];
    if (k < 0 || k > 2) return fail(SPH_E_INVALID, "bad kind at " + std::to_string(i));
    if (d->phase[i] < 0 || d->phase[i] >= d->n_mat) return fail(SPH_E_INVALID, "bad phase at " + std::to_string(i));
    if (d->kind[i] == SPH_FLUID && d->phase[i] >= kLdsPhases)
      return fail(SPH_E_UNSUPPORTED, "fluid phases must be among the first " + std::to_string(kLdsPhases) +
                                         " materials (particle " + std::to_string(i) + ")");
    if (k == SPH_RIGID && (!d->body || d->body[i] < 0 || d->body[i] >= d->n_body))
      return fail(SPH_E_INVALID, "bad body at " + std::to_string(i));
    if (k == SPH_FLUID && d->mat[d->phase[i]].p0 <= 0.0)
      return fail(SPH_E_INVALID, "fluid phase needs p0 > 0");
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(d->x[3 * i + a]) || !std::isfinite(d->u[3 * i + a]))
        return fail(SPH_E_INVALID, "non-finite input at " + std::to_string(i));
  }
  return SPH_OK;
}

// Eq. nummeth_timint_timestepcond evaluated at t = 0: CFL with the fastest
// speed of sound among fluid phases present and the largest initial fluid
// speed, viscous and body-force bounds, conduction when thermal.  The
// contact bound is used only for a given stiffness.
double time_step(const sph_scene_desc* d, double* m_min) {
  const double h = d->dx;
  const double vol0 = powi(d->dx, d->dim);
  std::vector<char> fl(d->n_mat, 0), rg(d->n_mat, 0);
  double umax = 0.0;
  for (int64_t i = 0; i < d->n; ++i) {
    if (d->kind[i] == SPH_FLUID) {
      fl[d->phase[i]] = 1;
      const double* u = &d->u[3 * i];
      double s = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
      if (s > umax) umax = s;
    } else if (d->kind[i] == SPH_RIGID) {
      rg[d->phase[i]] = 1;
    }
  }
  double cmax = 0.0, numax = 0.0, bmax = 0.0, heat = INFINITY, mmin = INFINITY;
  for (int k = 0; k < d->n_mat; ++k) {
    const sph_material& M = d->mat[k];
    if (fl[k]) {
      cmax = std::max(cmax, std::sqrt(M.p0 / M.rho0));
      numax = std::max(numax, M.nu);
    }
    if (fl[k] || rg[k]) {
      bmax = std::max(bmax, std::sqrt(M.b[0] * M.b[0] + M.b[1] * M.b[1] + M.b[2] * M.b[2]));
      if (d->thermal && M.kappa > 0.0) heat = std::min(heat, 0.1 * M.rho0 * M.cp * h * h / M.kappa);
    }
    if (rg[k]) mmin = std::min(mmin, M.rho0 * vol0);
  }
  double dt = INFINITY;
  if (cmax > 0.0) dt = std::min(dt, 0.25 * h / (cmax + umax));
  if (numax > 0.0) dt = std::min(dt, 0.125 * h * h / numax);
  if (bmax > 0.0) dt = std::min(dt, 0.25 * std::sqrt(h / bmax));
  dt = std::min(dt, heat);
  *m_min = mmin;
  return dt;
}

struct Counts {
  int64_t n_rigid = 0, n_moving = 0, n_fluid = 0, n_wall = 0;
};

Counts count(const sph_scene_desc* d) {
  Counts c;
  for (int64_t i = 0; i < d->n; ++i) {
    if (d->kind[i] == SPH_RIGID) c.n_rigid++;
    else if (d->kind[i] == SPH_FLUID) c.n_fluid++;
    else {
      c.n_wall++;
      if (d->moving && d->moving[i]) c.n_moving++;
    }
  }
  return c;
}

template <typename R>
void carve(Carver& cv, sph_scene* s, const Params& P, int64_t nmat) {
  const size_t n = (size_t)P.n;
  for (int b = 0; b < 2; ++b) {
    s->pos[b] = cv.take<V4<R>>(n);
    s->cell[b] = cv.take<uint32_t>(n);
    s->u[b] = cv.take<V4<R>>(n);
    s->a[b] = cv.take<V4<R>>(n);
    s->T[b] = cv.take<R>(n);
    s->m[b] = cv.take<R>(n);
    s->id[b] = cv.take<uint32_t>(n);
    s->info[b] = cv.take<uint32_t>(n);
    s->aux[b] = cv.take<int32_t>(n);
    s->ud[b] = P.tvf ? cv.take<V4<R>>(n) : nullptr;
  }
  s->ab = P.tvf ? cv.take<V4<R>>(n) : nullptr;
  s->rho = cv.take<R>(n);
  s->p = cv.take<R>(n);
  s->pw = cv.take<R>(n);
  s->uw = cv.take<V4<R>>(n);
  s->dTdt = cv.take<R>(n);
  s->pv = cv.take<V4<R>>((size_t)rec_stride(std::is_same<R, double>::value, P.thermal != 0, P.tvf != 0) * n);
  s->sb.key = cv.take<uint32_t>(n);
  s->sb.rank = cv.take<uint32_t>(n);
  s->sb.tid = cv.take<uint32_t>(n);
  s->sb.tsrc = cv.take<uint32_t>(n);
  s->sb.perm = cv.take<uint32_t>(n);
  s->sb.ccount = cv.take<uint32_t>((size_t)P.ncells);
  s->sb.nbsum = (P.ncells + 1023) / 1024;
  s->sb.bsum = cv.take<uint32_t>((size_t)s->sb.nbsum + 1);
  s->cstart = cv.take<uint32_t>((size_t)P.ncells + 1);
  const size_t nr = (size_t)P.slot_cap, nw = (size_t)P.n_moving;
  s->s_rb = cv.take<V4<double>>(nr);
  s->s_rk = cv.take<V4<double>>(nr);
  s->s_f = cv.take<V4<double>>(nr);
  s->s_aw = cv.take<V4<double>>(nr);
  s->s_x = cv.take<V4<double>>(nr);
  s->s_m = cv.take<double>(nr);
  s->s_sorted = cv.take<int32_t>(nr);
  s->s_body = cv.take<int32_t>(nr);
  s->s_id = cv.take<uint32_t>(nr);
  s->w_x0 = cv.take<V4<double>>(nw);
  s->w_aw = cv.take<V4<double>>(nw);
  s->w_sorted = cv.take<int32_t>(nw);
  s->bodies = cv.take<Body>((size_t)std::max(P.maxb, 1));
  s->mat = cv.take<MatT<R>>((size_t)nmat);
  s->err = cv.take<uint32_t>(4);
  s->pairs = cv.take<unsigned long long>((size_t)kPairWords);
  // compact neighbour lists: one slot per possible wave
  const int cap = 192, nsr = P.dim == 3 ? 9 : 3;
  s->nb.table = cv.take<WaveInfo>((size_t)P.max_waves);
  s->nb.ent = cv.take<uint16_t>((size_t)P.max_waves * cap * 64);
  s->nb.cnt = cv.take<uint8_t>((size_t)P.max_waves * 64);
  s->nb.split = cv.take<uint8_t>((size_t)P.max_waves * 64);
  s->nb.ext = cv.take<uint32_t>((size_t)P.ext_cap);
  s->nb.ext_n = cv.take<uint32_t>(4);
  s->nb.jlo = cv.take<uint32_t>((size_t)P.max_waves * nsr);
  s->wcount = cv.take<uint32_t>((size_t)P.nrows);
  s->woff = cv.take<uint32_t>((size_t)P.nrows + 1);
  s->wbsum = cv.take<uint32_t>((size_t)(P.nrows + 1023) / 1024 + 1);
  s->nb.nwaves = s->woff + P.nrows;
  s->gpart = cv.take<double>(6 * kGlobalBlocks);
  s->gout = cv.take<double>(8);
  s->dyn = cv.take<uint32_t>(4);
  s->dstep = cv.take<unsigned long long>(1);
  s->matb = cv.take<double>(3 * (size_t)nmat);
  // phase switch work space (only with switching enabled)
  const size_t np = P.pswitch ? n : 0, nbp = P.pswitch ? (size_t)std::max(P.maxb, 1) : 0;
  PhaseBufs& ps = s->ps;
  ps.flag = cv.take<uint8_t>(np);
  ps.target = cv.take<int32_t>(np);
  ps.label = cv.take<uint32_t>(np);
  ps.body_of_id = cv.take<uint32_t>(np);
  ps.list = cv.take<uint32_t>(np);
  ps.roots = cv.take<uint32_t>(np);
  ps.ctr = cv.take<uint32_t>(8);
  ps.dirty = cv.take<uint32_t>(nbp);
  ps.rold = cv.take<V4<double>>(nbp);
  ps.alive = cv.take<uint32_t>(P.pswitch ? nr : 0);
  ps.alive_sc = cv.take<uint32_t>(P.pswitch ? nr + 1 : 0);
  ps.bsum = cv.take<uint32_t>(P.pswitch ? (nr + 1023) / 1024 + 1 : 0);
  for (int b = 0; b < 2; ++b) {
    ps.jkey[b] = cv.take<unsigned long long>(np);
    ps.jidx[b] = cv.take<uint32_t>(np);
  }
  const size_t ns = P.pswitch ? nr : 0;
  ps.snew = cv.take<uint32_t>(ns);
  ps.sbody = cv.take<int32_t>(ns);
  ps.sid = cv.take<uint32_t>(ns);
  ps.srb = cv.take<V4<double>>(ns);
  ps.srk = cv.take<V4<double>>(ns);
  ps.srf = cv.take<V4<double>>(ns);
}

int make_params(const sph_scene_desc* d, Params& P, double* m_min) {
  std::memset(&P, 0, sizeof(P));
  P.dim = d->dim;
  P.n = d->n;
  P.dx = d->dx;
  P.h = d->dx;
  P.rc = 3.0 * P.h;
  P.rc2 = P.rc * P.rc;
  P.L = d->cell_edge > 0.0 ? d->cell_edge : P.rc;
  P.ncells = 1;
  for (int a = 0; a < 3; ++a) {
    P.lo[a] = d->lo[a];
    if (a < d->dim) {
      double ext = d->hi[a] - d->lo[a];
      int nc = (int)std::ceil(ext / P.L * (1.0 - 1e-12));
      P.nc[a] = nc < 1 ? 1 : nc;
    } else {
      P.nc[a] = 1;
      P.lo[a] = 0.0;
    }
    P.ncells *= P.nc[a];
  }
  if (P.ncells > 0x7fffffffLL) return fail(SPH_E_INVALID, "cell grid too large");
  if (P.nc[0] > 65535) return fail(SPH_E_INVALID, "more than 65535 cells along x");
  const double sg = sigma_d(d->dim);
  P.wnorm = sg / powi(P.h, d->dim);
  P.dnorm = -5.0 * sg / powi(P.h, d->dim + 1);
  P.vol0 = powi(d->dx, d->dim);
  if (d->dim == 2) {
    double reff2 = d->dx * d->dx / kPi;
    P.Ir_fac = 0.5 * reff2;
  } else {
    double reff = std::cbrt(0.75 / kPi) * d->dx;
    P.Ir_fac = 0.4 * (reff * reff);
  }
  double mmin;
  double dt0 = time_step(d, &mmin);
  double dt = dt0;
  if (d->contact && d->k_c > 0.0 && std::isfinite(mmin)) dt = std::min(dt, 0.22 * std::sqrt(mmin / d->k_c));
  P.dt = d->dt > 0.0 ? d->dt : dt;
  if (!(P.dt > 0.0) || !std::isfinite(P.dt)) return fail(SPH_E_INVALID, "no finite time step");
  P.hdt = 0.5 * P.dt;
  if (d->k_c >= 0.0) P.kc = d->k_c;
  else if (std::isfinite(mmin)) {
    double b = 0.22 / (2.0 * (d->dt > 0.0 ? d->dt : dt0));
    P.kc = mmin * (b * b);
  } else P.kc = 0.0;
  if (d->d_c >= 0.0) P.dc = d->d_c;
  else P.dc = std::isfinite(mmin) ? 0.2 * std::sqrt(P.kc * mmin / 2.0) : 0.0;
  P.thermal = d->thermal;
  P.contact = d->contact;
  P.pswitch = d->phase_switch;
  P.wall_A = d->wall_A;
  P.wall_Om = d->wall_Omega;
  for (int a = 0; a < 3; ++a) P.wall_dir[a] = d->wall_dir[a];
  P.heat_src = d->heat_src;
  P.sQ = d->src_Q;
  P.ssig = d->src_sigma;
  for (int a = 0; a < 2; ++a) { P.ss0[a] = d->src_s0[a]; P.sv[a] = d->src_v[a]; }
  P.sztop = d->src_ztop;
  P.sdepth = d->src_depth;
  if (!(d->p_b >= 0.0) || !std::isfinite(d->p_b)) return fail(SPH_E_INVALID, "background pressure p_b must be >= 0");
  P.tvf = d->p_b > 0.0 ? 1 : 0;
  P.pb = P.tvf ? d->p_b : 0.0;
  // periodic axes: y and z only (waves run along x rows), a whole number of
  // at least 3 cells per period, no phase switching
  for (int a = 0; a < 3; ++a) {
    P.per[a] = (a < d->dim && d->periodic[a]) ? 1 : 0;
    P.period[a] = P.per[a] ? d->hi[a] - d->lo[a] : 0.0;
  }
  if (P.per[0]) return fail(SPH_E_UNSUPPORTED, "the x axis cannot be periodic (make a periodic direction y or z)");
  for (int a = 1; a < 3; ++a) {
    if (!P.per[a]) continue;
    if (P.nc[a] < 3) return fail(SPH_E_INVALID, "a periodic axis needs at least 3 cells");
    if (std::fabs((double)P.nc[a] * P.L - P.period[a]) > 1e-9 * P.period[a])
      return fail(SPH_E_INVALID, "a periodic extent must be a whole number of cells");
    if (d->phase_switch) return fail(SPH_E_UNSUPPORTED, "phase switching with periodic axes");
  }
  P.n_mat = d->n_mat;
  P.nb = d->n_body;
  P.maxb = std::max(d->max_bodies, d->n_body);
  Counts c = count(d);
  P.n_rigid = c.n_rigid;
  P.n_moving = c.n_moving;
  P.nrows = (int64_t)P.nc[1] * P.nc[2];
  P.max_waves = (P.n + 63) / 64 + P.nrows + 1;
  // with phase switching every particle may become rigid and every body
  // slot up to max_bodies may be in use
  P.slot_cap = P.pswitch ? P.n : P.n_rigid;
  P.ext_cap = std::min<int64_t>(P.n, c.n_wall + P.slot_cap);
  P.body_launch = P.pswitch ? P.maxb : P.nb;
  *m_min = mmin;
  return SPH_OK;
}

template <typename R>
KC<R> make_kc(const Params& P) {
  KC<R> k;
  k.h = (R)P.h;
  k.inv_h = (R)(1.0 / P.h);
  k.wnorm = (R)P.wnorm;
  k.dnorm = (R)P.dnorm;
  k.rc2 = (R)P.rc2;
  k.L = (R)P.L;
  k.dx = (R)P.dx;
  k.dx2 = (R)(P.dx * P.dx);
  k.vol0 = (R)P.vol0;
  k.kc = (R)P.kc;
  k.dc = (R)P.dc;
  k.dt = (R)P.dt;
  k.hdt = (R)P.hdt;
  k.pb = (R)P.pb;
  k.per_y = (R)P.period[1];
  k.per_z = (R)P.period[2];
  for (int a = 0; a < 3; ++a) k.lo[a] = (R)P.lo[a];
  return k;
}

template <typename R>
View<R> make_view(sph_scene* s, int ip, int iu, int iT) {
  View<R> v;
  v.pos = (V4<R>*)s->pos[ip];
  v.cell = s->cell[ip];
  v.u = (V4<R>*)s->u[iu];
  v.a = (V4<R>*)s->a[ip];
  v.T = (R*)s->T[iT];
  v.m = (R*)s->m[ip];
  v.id = s->id[ip];
  v.info = s->info[ip];
  v.aux = s->aux[ip];
  v.ud = (V4<R>*)s->ud[ip];
  v.ab = (V4<R>*)s->ab;
  v.u_out = (V4<R>*)s->u[1 - iu];
  v.T_out = (R*)s->T[1 - iT];
  v.rho = (R*)s->rho;
  v.p = (R*)s->p;
  v.pw = (R*)s->pw;
  v.uw = (V4<R>*)s->uw;
  v.dTdt = (R*)s->dTdt;
  v.pv = (V4<R>*)s->pv;
  v.pvs = rec_stride(std::is_same<R, double>::value, s->P.thermal != 0, s->P.tvf != 0);
  v.cstart = s->cstart;
  v.s_rb = s->s_rb;
  v.s_rk = s->s_rk;
  v.s_f = s->s_f;
  v.s_aw = s->s_aw;
  v.s_x = s->s_x;
  v.s_m = s->s_m;
  v.s_sorted = s->s_sorted;
  v.s_body = s->s_body;
  v.s_id = s->s_id;
  v.w_x0 = s->w_x0;
  v.w_aw = s->w_aw;
  v.w_sorted = s->w_sorted;
  v.mat = (const MatT<R>*)s->mat;
  v.bodies = s->bodies;
  v.err = s->err;
  v.pairs = s->pairs;
  v.nb = s->nb;
  v.dyn = s->dyn;
  v.dstep = s->dstep;
  v.ps = s->ps;
  return v;
}

template <typename R>
View<R> cur(sph_scene* s) {
  return make_view<R>(s, s->ip, s->iu, s->iT);
}

// clear the per-evaluation pair counters (and the running total)
void zero_pairs(sph_scene* s, bool total) { launch_zero_pairs(s->pairs, true, total, s->stream); }

// the pair counters: every counter summed over its parts
int read_pairs(sph_scene* s, unsigned long long out[kPairSlots]) {
  std::vector<unsigned long long> w((size_t)kPairWords);
  HIP_TRY(hipMemcpy(w.data(), s->pairs, sizeof(unsigned long long) * w.size(), hipMemcpyDeviceToHost));
  for (int slot = 0; slot < kPairSlots; ++slot) {
    out[slot] = 0ull;
    for (int p = 0; p < kPairParts; ++p) out[slot] += w[(size_t)pair_at(slot, p)];
  }
  return SPH_OK;
}

// counting sort by (cell, id) of the current buffers into the other set
template <typename R>
void sort_and_permute(sph_scene* s) {
  View<R> src = cur<R>(s);
  launch_sort_keys(s->P, s->sb, s->cstart, src.id, s->stream);
  View<R> dst = make_view<R>(s, 1 - s->ip, 1 - s->iu, 1 - s->iT);
  Launch<R>::gather(src, dst, s->P, s->sb, s->stream);
  launch_wave_table(s->P, s->cstart, s->wcount, s->woff, s->wbsum, s->nb.table, s->stream);
  s->ip = 1 - s->ip;
  s->iu = 1 - s->iu;
  s->iT = 1 - s->iT;
}

// The step's stages.  pre_step: counters, first kick and drift, bodies,
// rigid and wall poses, sort; sweeps: density, extrapolation, forces (+ heat,
// second fluid kick); post_step: body sums and second body kick, rigid
// velocities, phase switch.  A batch runs the sweeps of all its scenes as
// one launch per sweep between the scenes' pre and post stages.
template <typename R>
void pre_step(sph_scene* s, hipEvent_t* ev) {
  const Params& P = s->P;
  const KC<R> k = make_kc<R>(P);
  const double t_new = (double)(s->step + 1) * P.dt;
  if (ev) (void)hipEventRecord(ev[0], s->stream);
  View<R> v = cur<R>(s);   // kick_drift also starts the step (counters)
  Launch<R>::kick_drift(v, P, k, s->sb, s->stream);
  launch_body_kick_drift(s->bodies, P, P.pswitch ? s->dyn + 1 : nullptr, s->stream);
  Launch<R>::rigid_pose(v, P, k, s->sb, t_new, s->stream);
  Launch<R>::wall_motion(v, P, k, s->sb, t_new, s->stream);
  if (ev) (void)hipEventRecord(ev[1], s->stream);
  sort_and_permute<R>(s);
  if (ev) (void)hipEventRecord(ev[2], s->stream);
}

template <typename R>
void sweeps(sph_scene* s, int kick, int heat, hipEvent_t* ev) {
  const KC<R> k = make_kc<R>(s->P);
  View<R> v = cur<R>(s);
  Launch<R>::density(v, s->P, k, s->stream);
  if (ev) (void)hipEventRecord(ev[3], s->stream);
  Launch<R>::extrapolate(v, s->P, k, s->stream);
  if (ev) (void)hipEventRecord(ev[4], s->stream);
  Launch<R>::forces(v, s->P, k, kick, heat, s->stream);
  if (ev) (void)hipEventRecord(ev[5], s->stream);
}

// the sweeps wrote u (and T) into the other buffer; body sums
template <typename R>
void after_sweeps(sph_scene* s, int kick, hipEvent_t* ev) {
  s->iu = 1 - s->iu;
  if (s->P.thermal) s->iT = 1 - s->iT;
  launch_body_reduce(s->bodies, s->s_f, s->s_rk, s->P, kick, s->P.pswitch ? s->dyn + 1 : nullptr, s->stream);
  if (ev) (void)hipEventRecord(ev[6], s->stream);
}

template <typename R>
void post_step(sph_scene* s, hipEvent_t* ev) {
  const Params& P = s->P;
  after_sweeps<R>(s, 1, ev);
  View<R> v = cur<R>(s);
  Launch<R>::rigid_velocity(v, P, s->stream);
  if (P.pswitch) Launch<R>::phase_switch(v, P, make_kc<R>(P), s->matb, s->stream);
  if (ev) {
    (void)hipEventRecord(ev[7], s->stream);
    s->rec += 1;
  }
  s->step += 1;
}

size_t slot_bytes(int precision) { return precision == SPH_FP64 ? sizeof(Slot<double>) : sizeof(Slot<float>); }
constexpr size_t kSlotMax = sizeof(Slot<double>) > sizeof(Slot<float>) ? sizeof(Slot<double>) : sizeof(Slot<float>);

template <typename R>
void fill_slot(sph_scene* s, uint32_t b0, uint32_t nb, const char* gbase, char* dst) {
  Slot<R> sl;
  std::memset(&sl, 0, sizeof(sl));
  sl.v = cur<R>(s);
  // pointers as offsets from the batch's global base (see for_each_ptr)
  for_each_ptr(sl.v, [&](auto*& p) {
    using T = std::remove_reference_t<decltype(*p)>;
    p = reinterpret_cast<T*>(reinterpret_cast<intptr_t>(p) - reinterpret_cast<intptr_t>(gbase));
  });
  sl.P = s->P;
  sl.k = make_kc<R>(s->P);
  sl.b0 = b0;
  sl.nb = nb;
  std::memcpy(dst, &sl, sizeof(sl));
}

// the group's slot table for the scenes' current buffer parities: one of the
// two kept tables, or a new one written over the table not used last
int group_table(sph_batch* b, sph_batch::Group& g, int* which_out) {
  std::vector<int> key;
  for (int m : g.members) {
    sph_scene* s = b->scenes[m];
    key.push_back(s->ip * 4 + s->iu * 2 + s->iT);
  }
  for (int w = 0; w < 2; ++w)
    if (key == g.key[w]) {
      *which_out = w;
      return SPH_OK;
    }
  const int which = g.key[0].empty() ? 0 : 1;
  *which_out = which;
  // a table in flight is replaced: wait for the batch stream first; graphs
  // captured with the old table are dropped
  if (!g.key[which].empty()) {
    HIP_TRY(hipStreamSynchronize(b->stream));
    for (auto& gr : b->graphs) (void)hipGraphExecDestroy(gr.exec);
    b->graphs.clear();
  }
  const size_t sb = slot_bytes(g.precision);
  g.host[which].assign(g.members.size() * sb, 0);
  uint32_t b0 = 0;
  for (size_t q = 0; q < g.members.size(); ++q) {
    sph_scene* s = b->scenes[g.members[q]];
    const uint32_t nb = (uint32_t)((s->P.max_waves + 7) / 8 * 8);
    if (g.precision == SPH_FP64) fill_slot<double>(s, b0, nb, b->ws, &g.host[which][q * sb]);
    else fill_slot<float>(s, b0, nb, b->ws, &g.host[which][q * sb]);
    b0 += nb;
  }
  g.blocks = b0;
  HIP_TRY(hipMemcpyAsync(b->ws + g.off[which], g.host[which].data(), g.host[which].size(), hipMemcpyHostToDevice,
                         b->stream));
  g.key[which] = key;
  return SPH_OK;
}

template <typename R>
void group_sweep(sph_batch* b, sph_batch::Group& g, int which, int stage) {
  Launch<R>::batch_sweep(stage, reinterpret_cast<const Slot<R>*>(b->ws + g.off[which]), b->ws,
                         (int)g.members.size(), g.dim, g.mode, g.blocks, 1, 1, b->stream);
}

// the host-side bookkeeping of one step, without its launches (a replayed
// graph did the device work): the buffer parities and the step count change
// exactly as pre_step / after_sweeps / post_step change them
void advance_host_state(sph_scene* s) {
  s->ip = 1 - s->ip;
  s->iT = 1 - s->iT;
  if (s->P.thermal) s->iT = 1 - s->iT;
  s->step += 1;
}

std::vector<int> parity_key(const sph_batch* b) {
  std::vector<int> key;
  for (const sph_scene* s : b->scenes) key.push_back(s->ip * 4 + s->iu * 2 + s->iT);
  return key;
}

// enqueue one step of every scene of the batch (no graph)
int batch_enqueue_step(sph_batch* b) {
  for (sph_scene* s : b->scenes) {
    if (s->precision == SPH_FP64) pre_step<double>(s, nullptr);
    else pre_step<float>(s, nullptr);
  }
  std::vector<int> which(b->groups.size());
  for (size_t g = 0; g < b->groups.size(); ++g)
    if (int st = group_table(b, b->groups[g], &which[g])) return st;
  for (int stage = 0; stage < 3; ++stage)
    for (size_t g = 0; g < b->groups.size(); ++g) {
      sph_batch::Group& G = b->groups[g];
      if (G.precision == SPH_FP64) group_sweep<double>(b, G, which[g], stage);
      else group_sweep<float>(b, G, which[g], stage);
    }
  for (sph_scene* s : b->scenes) {
    if (s->precision == SPH_FP64) post_step<double>(s, nullptr);
    else post_step<float>(s, nullptr);
  }
  return SPH_OK;
}

// the slot tables of the state after the sort of the coming step exist
bool tables_ready(sph_batch* b) {
  for (auto& g : b->groups) {
    std::vector<int> key;
    for (int m : g.members) {
      const sph_scene* s = b->scenes[m];
      // the sweeps see the parities after the sort: ip, iu and iT flipped
      key.push_back((1 - s->ip) * 4 + (1 - s->iu) * 2 + (1 - s->iT));
    }
    if (key != g.key[0] && key != g.key[1]) return false;
  }
  return true;
}

int batch_one_step(sph_batch* b) {
  if (!b->use_graphs) return batch_enqueue_step(b);
  const std::vector<int> key = parity_key(b);
  for (auto& g : b->graphs)
    if (g.key == key) {
      HIP_TRY(hipGraphLaunch(g.exec, b->stream));
      for (sph_scene* s : b->scenes) advance_host_state(s);
      return SPH_OK;
    }
  // not captured yet: a plain step while a slot table is still missing,
  // else capture this step (the capture advances the host state) and run it
  if (b->graphs.size() >= 2 || !tables_ready(b)) return batch_enqueue_step(b);
  HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed));
  const int st = batch_enqueue_step(b);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(b->stream, &graph);
  if (st != SPH_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return fail(SPH_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  hipGraphExec_t exec = nullptr;
  const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e2 != hipSuccess) return fail(SPH_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
  b->graphs.push_back({key, exec});
  HIP_TRY(hipGraphLaunch(exec, b->stream));
  return SPH_OK;
}

template <typename R>
void one_step(sph_scene* s) {
  hipEvent_t* ev = nullptr;
  if (s->timers && s->rec < SPH_TIMER_STEPS) ev = &(*s->ev)[(size_t)s->rec * (SPH_TIMER_STAGES + 1)];
  pre_step<R>(s, ev);
  sweeps<R>(s, 1, 1, ev);
  post_step<R>(s, ev);
}

template <typename R>
int create_impl(const sph_scene_desc* d, sph_scene* s) {
  const Params& P = s->P;
  const int64_t n = P.n;
  hipStream_t st = s->stream;
  // host-side initial arrays in original-id order
  std::vector<V4<R>> pos(n), u(n), a(n);
  std::vector<uint32_t> cell(n), id(n), info(n);
  std::vector<int32_t> aux(n, -1);
  std::vector<R> T(n), m(n);
  // rigid slots ordered by (body, id); moving-wall slots by id
  std::vector<int64_t> bcount(std::max(P.maxb, 1) + 1, 0);
  for (int64_t i = 0; i < n; ++i)
    if (d->kind[i] == SPH_RIGID) bcount[d->body[i] + 1]++;
  for (int kb = 0; kb < P.maxb; ++kb) bcount[kb + 1] += bcount[kb];
  std::vector<int64_t> bfill(bcount.begin(), bcount.end() - 1);
  std::vector<uint32_t> s_id(std::max<int64_t>(P.n_rigid, 1));
  std::vector<int32_t> s_body(std::max<int64_t>(P.n_rigid, 1)), s_sorted(std::max<int64_t>(P.n_rigid, 1));
  std::vector<V4<double>> s_x(std::max<int64_t>(P.n_rigid, 1));
  std::vector<double> s_m(std::max<int64_t>(P.n_rigid, 1));
  std::vector<V4<double>> w_x0(std::max<int64_t>(P.n_moving, 1)), w_zero(std::max<int64_t>(P.n_moving, 1));
  std::vector<int32_t> w_sorted(std::max<int64_t>(P.n_moving, 1));
  int64_t nw = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int kind = d->kind[i];
    const int ph = d->phase[i];
    const int moving = (kind == SPH_WALL && d->moving && d->moving[i]) ? 1 : 0;
    const int body = kind == SPH_RIGID ? d->body[i] : -1;
    double x[3] = {d->x[3 * i], d->x[3 * i + 1], d->dim == 3 ? d->x[3 * i + 2] : 0.0};
    // the position binned: along periodic axes wrapped into the box (body
    // quantities and moving-wall references keep the position as given)
    double xw[3] = {x[0], x[1], x[2]};
    for (int ax = 1; ax < P.dim; ++ax) {
      if (!P.per[ax]) continue;
      if (xw[ax] >= P.lo[ax] + P.period[ax]) xw[ax] = xw[ax] - P.period[ax];
      else if (xw[ax] < P.lo[ax]) xw[ax] = xw[ax] + P.period[ax];
    }
    // cell of the initial position
    int c3[3] = {0, 0, 0};
    for (int ax = 0; ax < P.dim; ++ax) {
      double vv = std::floor((xw[ax] - P.lo[ax]) / P.L);
      if (P.per[ax] && vv == (double)P.nc[ax]) vv = (double)(P.nc[ax] - 1);
      if (!(vv >= 0.0) || vv >= (double)P.nc[ax])
        return fail(SPH_E_INVALID, "particle " + std::to_string(i) + " outside the cell grid");
      c3[ax] = (int)vv;
    }
    const uint32_t lin = (uint32_t)((int64_t)c3[0] + (int64_t)P.nc[0] * ((int64_t)c3[1] + (int64_t)P.nc[1] * c3[2]));
    cell[i] = lin;
    V4<R> o;
    if (sizeof(R) == 8) {
      o.x = (R)xw[0]; o.y = (R)xw[1]; o.z = (R)xw[2]; o.w = 0;
    } else {
      R off[3] = {0, 0, 0};
      for (int ax = 0; ax < P.dim; ++ax) {
        double rel = (xw[ax] - P.lo[ax]) - (double)c3[ax] * P.L;
        float f = (float)rel;
        off[ax] = f < 0.f ? 0.f : (f > (float)P.L ? (float)P.L : f);
      }
      o.x = off[0]; o.y = off[1]; o.z = off[2]; o.w = (R)c3[0];
    }
    pos[i] = o;
    V4<R> uu;
    uu.x = (R)d->u[3 * i];
    uu.y = (R)d->u[3 * i + 1];
    uu.z = d->dim == 3 ? (R)d->u[3 * i + 2] : (R)0;
    uu.w = 0;
    if (moving) uu.x = uu.y = uu.z = 0;
    u[i] = uu;
    V4<R> z;
    z.x = z.y = z.z = z.w = 0;
    a[i] = z;
    T[i] = d->T ? (R)d->T[i] : (R)0;
    // Sec. "Initial particle spacing": mass = reference density x dx^d
    const double mass = d->mat[ph].rho0 * P.vol0;
    m[i] = (R)mass;
    id[i] = (uint32_t)i;
    info[i] = mkinfo((uint32_t)kind, (uint32_t)ph, (uint32_t)moving, body);
    if (kind == SPH_RIGID) {
      const int64_t sl = bfill[body]++;
      aux[i] = (int32_t)sl;
      s_id[sl] = (uint32_t)i;
      s_body[sl] = body;
      s_sorted[sl] = (int32_t)i;
      V4<double> xs;
      xs.x = x[0]; xs.y = x[1]; xs.z = x[2]; xs.w = 0.0;
      s_x[sl] = xs;
      s_m[sl] = mass;
    } else if (moving) {
      aux[i] = (int32_t)nw;
      V4<double> xs;
      xs.x = x[0]; xs.y = x[1]; xs.z = x[2]; xs.w = 0.0;
      w_x0[nw] = xs;
      V4<double> zz;
      zz.x = zz.y = zz.z = zz.w = 0.0;
      w_zero[nw] = zz;
      w_sorted[nw] = (int32_t)i;
      nw++;
    }
  }
  // materials in the sweep precision
  std::vector<MatT<R>> mats(d->n_mat);
  for (int k = 0; k < d->n_mat; ++k) {
    const sph_material& M = d->mat[k];
    MatT<R>& o = mats[k];
    o.rho0 = (R)M.rho0;
    o.p0 = (R)M.p0;
    o.nu = (R)M.nu;
    o.cp = (R)M.cp;
    o.kappa = (R)M.kappa;
    o.eta = (R)(M.rho0 * M.nu);
    o.T_t = (R)M.T_t;
    o.inv_rho0 = (R)(1.0 / M.rho0);
    o.inv_p0 = (R)(M.p0 != 0.0 ? 1.0 / M.p0 : 0.0);
    o.inv_cp = (R)(M.cp != 0.0 ? 1.0 / M.cp : 0.0);
    for (int ax = 0; ax < 3; ++ax) o.b[ax] = (R)(ax < d->dim ? M.b[ax] : 0.0);
    o.switch_to = M.switch_to;
    o.mass = (R)(M.rho0 * P.vol0);
    o.dirichlet = M.dirichlet;
  }
  // bodies
  std::vector<Body> bodies(std::max(P.maxb, 1));
  std::memset(bodies.data(), 0, sizeof(Body) * bodies.size());
  for (int kb = 0; kb < P.nb; ++kb) {
    Body& B = bodies[kb];
    const sph_body_init& I = d->bodies[kb];
    const double qn = std::sqrt(I.q[0] * I.q[0] + I.q[1] * I.q[1] + I.q[2] * I.q[2] + I.q[3] * I.q[3]);
    for (int ax = 0; ax < 4; ++ax) B.q[ax] = I.q[ax] / qn;
    for (int ax = 0; ax < 3; ++ax) {
      B.u[ax] = ax < d->dim ? I.u[ax] : 0.0;
      B.w[ax] = (d->dim == 3 || ax == 2) ? I.w[ax] : 0.0;
    }
    B.fixed = I.fixed;
    B.slot0 = (int32_t)bcount[kb];
    B.nslot = (int32_t)(bcount[kb + 1] - bcount[kb]);
    B.active = B.nslot > 0;
    if (B.nslot > 0) {
      const sph_material& M = d->mat[d->phase[s_id[B.slot0]]];
      for (int ax = 0; ax < 3; ++ax) B.b[ax] = ax < d->dim ? M.b[ax] : 0.0;
    }
  }
  for (int kb = P.nb; kb < P.maxb; ++kb) {
    bodies[kb].q[0] = 1.0;
    bodies[kb].slot0 = (int32_t)P.n_rigid;
  }
  std::vector<double> matb(3 * (size_t)d->n_mat);
  for (int k = 0; k < d->n_mat; ++k)
    for (int ax = 0; ax < 3; ++ax) matb[3 * k + ax] = ax < d->dim ? d->mat[k].b[ax] : 0.0;
  const uint32_t dyn[4] = {(uint32_t)P.n_rigid, (uint32_t)P.nb, 0u, 0u};
  // upload into buffer set 0
  if (n > 0) {
    HIP_TRY(hipMemcpyAsync(s->pos[0], pos.data(), sizeof(V4<R>) * n, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(s->cell[0], cell.data(), 4 * n, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(s->sb.key, cell.data(), 4 * n, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(s->u[0], u.data(), sizeof(V4<R>) * n, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(s->a[0], a.data(), sizeof(V4<R>) * n, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(s->T[0], T.data(), sizeof(R) * n, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(s->T[1], T.data(), sizeof(R) * n, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(s->m[0], m.data(), sizeof(R) * n, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(s->id[0], id.data(), 4 * n, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(s->info[0], info.data(), 4 * n, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(s->aux[0], aux.data(), 4 * n, hipMemcpyHostToDevice, st));
  }
  if (P.n_rigid > 0) {
    const size_t nr = (size_t)P.n_rigid;
    HIP_TRY(hipMemcpyAsync(s->s_id, s_id.data(), 4 * nr, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(s->s_body, s_body.data(), 4 * nr, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(s->s_sorted, s_sorted.data(), 4 * nr, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(s->s_x, s_x.data(), sizeof(V4<double>) * nr, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(s->s_m, s_m.data(), 8 * nr, hipMemcpyHostToDevice, st));
  }
  if (P.n_moving > 0) {
    const size_t nm = (size_t)P.n_moving;
    HIP_TRY(hipMemcpyAsync(s->w_x0, w_x0.data(), sizeof(V4<double>) * nm, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(s->w_aw, w_zero.data(), sizeof(V4<double>) * nm, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(s->w_sorted, w_sorted.data(), 4 * nm, hipMemcpyHostToDevice, st));
  }
  HIP_TRY(hipMemcpyAsync(s->bodies, bodies.data(), sizeof(Body) * bodies.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(s->mat, mats.data(), sizeof(MatT<R>) * mats.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(s->matb, matb.data(), sizeof(double) * matb.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(s->dyn, dyn, sizeof(dyn), hipMemcpyHostToDevice, st));
  launch_fill_u32(s->err, 0u, 4, st);
  launch_fill_u32(s->ps.ctr, 0u, 8, st);
  if (P.pswitch) launch_fill_u32(s->ps.dirty, 0u, std::max(P.maxb, 1), st);
  zero_pairs(s, true);
  launch_fill_u32(reinterpret_cast<uint32_t*>(s->dstep), 0u, 2, st);
  launch_fill_u32(s->sb.ccount, 0u, P.ncells, st);
  if (P.tvf) {
    // u~ - u and a_b start at zero (the first evaluation sets a_b)
    const int64_t w = (int64_t)(sizeof(V4<R>) / 4) * P.n;
    launch_fill_u32(reinterpret_cast<uint32_t*>(s->ud[0]), 0u, w, st);
    launch_fill_u32(reinterpret_cast<uint32_t*>(s->ud[1]), 0u, w, st);
    launch_fill_u32(reinterpret_cast<uint32_t*>(s->ab), 0u, w, st);
  }
  launch_fill_u32(s->nb.ext_n, 0u, 1, st);
  s->ip = 0;
  s->iu = 0;
  s->iT = 0;
  // body mass quantities, body-frame offsets, rigid particle velocities
  if (P.nb > 0) {
    launch_mass_props_impl(s->bodies, s->s_x, s->s_m, s->s_rb, s->s_rk, P, nullptr, nullptr, st);
    Launch<R>::rigid_velocity(cur<R>(s), P, st);
    launch_rigid_aw(s->bodies, P, s->s_body, s->s_rk, s->s_aw, st);
  }
  // first sort, then one evaluation without time update
  sort_and_permute<R>(s);
  sweeps<R>(s, 0, 0, nullptr);
  after_sweeps<R>(s, 0, nullptr);
  HIP_TRY(hipStreamSynchronize(st));
  uint32_t err = 0;
  HIP_TRY(hipMemcpy(&err, s->err, 4, hipMemcpyDeviceToHost));
  if (err) return fail(SPH_E_STATE, "device error during set-up: " + std::to_string(err));
  // the running pair total counts steps only
  launch_zero_pairs(s->pairs, false, true, st);
  HIP_TRY(hipStreamSynchronize(st));
  return SPH_OK;
}

// rigid particles and bodies now (they change with phase switches)
int dyn_counts(sph_scene* s, int64_t* n_rigid, int* n_bodies) {
  if (!s->P.pswitch) {
    *n_rigid = s->P.n_rigid;
    *n_bodies = s->P.nb;
    return SPH_OK;
  }
  uint32_t d[2];
  HIP_TRY(hipStreamSynchronize(s->stream));
  HIP_TRY(hipMemcpy(d, s->dyn, sizeof(d), hipMemcpyDeviceToHost));
  *n_rigid = d[0];
  *n_bodies = (int)d[1];
  return SPH_OK;
}

size_t arena_for_params(int precision, const Params& P) {
  sph_scene tmp;
  std::memset(&tmp, 0, sizeof(tmp));
  Carver cv{nullptr, 0};
  if (precision == SPH_FP64) carve<double>(cv, &tmp, P, P.n_mat);
  else carve<float>(cv, &tmp, P, P.n_mat);
  return align_up(cv.off);
}

size_t arena_for(const sph_scene_desc* d, const Params& P) { return arena_for_params(d->precision, P); }

// State image: this header, then the scene's arena verbatim (the carve is a
// function of the parameters only, so the image maps onto a new arena).
struct StateHeader {
  char magic[8];
  int32_t abi, precision;
  uint64_t arena_used;
  int64_t step, n_fluid, n_wall;
  int32_t ip, iu, iT, pad;
  Params P;
};
constexpr char kStateMagic[8] = {'S', 'P', 'H', 'R', 'B', 'S', 'T', '1'};

int parse_state(const void* blob, size_t bytes, StateHeader* h) {
  if (!blob || bytes < sizeof(StateHeader)) return fail(SPH_E_INVALID, "state image too small");
  std::memcpy(h, blob, sizeof(StateHeader));
  if (std::memcmp(h->magic, kStateMagic, 8) != 0) return fail(SPH_E_INVALID, "not a scene state image");
  if (h->abi != SPH_ABI_VERSION) return fail(SPH_E_INVALID, "state image of another ABI version");
  if (h->precision != SPH_FP64 && h->precision != SPH_FP32_SWEEP) return fail(SPH_E_INVALID, "bad precision");
  if (h->arena_used != arena_for_params(h->precision, h->P)) return fail(SPH_E_INVALID, "inconsistent state image");
  if (bytes < sizeof(StateHeader) + h->arena_used) return fail(SPH_E_INVALID, "truncated state image");
  return SPH_OK;
}

int check_state(sph_scene* s) {
  if (!s) return fail(SPH_E_INVALID, "null scene");
  return SPH_OK;
}

template <typename R>
int read_particles_impl(sph_scene* s, uint32_t mask, double* out) {
  const int64_t n = s->P.n;
  const Params& P = s->P;
  hipStream_t st = s->stream;
  HIP_TRY(hipStreamSynchronize(st));
  std::vector<uint32_t> id(n), cell(n), info(n);
  std::vector<int32_t> aux(n);
  std::vector<V4<R>> pos(n), u(n), a(n), uw(n), ab, ud;
  std::vector<R> rho(n), p(n), T(n), pw(n), m(n), dT(n);
  int64_t nrig = 0;
  int nbod = 0;
  if (int e = dyn_counts(s, &nrig, &nbod)) return e;
  std::vector<V4<double>> sf(std::max<int64_t>(nrig, 1));
  if (n > 0) {
    HIP_TRY(hipMemcpy(id.data(), s->id[s->ip], 4 * n, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(cell.data(), s->cell[s->ip], 4 * n, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(info.data(), s->info[s->ip], 4 * n, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(aux.data(), s->aux[s->ip], 4 * n, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(pos.data(), s->pos[s->ip], sizeof(V4<R>) * n, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(u.data(), s->u[s->iu], sizeof(V4<R>) * n, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(a.data(), s->a[s->ip], sizeof(V4<R>) * n, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(uw.data(), s->uw, sizeof(V4<R>) * n, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(rho.data(), s->rho, sizeof(R) * n, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(p.data(), s->p, sizeof(R) * n, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(T.data(), s->T[s->iT], sizeof(R) * n, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(pw.data(), s->pw, sizeof(R) * n, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(m.data(), s->m[s->ip], sizeof(R) * n, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(dT.data(), s->dTdt, sizeof(R) * n, hipMemcpyDeviceToHost));
    if (P.tvf) {
      ab.resize(n);
      ud.resize(n);
      HIP_TRY(hipMemcpy(ab.data(), s->ab, sizeof(V4<R>) * n, hipMemcpyDeviceToHost));
      HIP_TRY(hipMemcpy(ud.data(), s->ud[s->ip], sizeof(V4<R>) * n, hipMemcpyDeviceToHost));
    }
  }
  if (nrig > 0) HIP_TRY(hipMemcpy(sf.data(), s->s_f, sizeof(V4<double>) * nrig, hipMemcpyDeviceToHost));
  double* o = out;
  auto vec = [&](auto getter) {
    for (int64_t i = 0; i < n; ++i) {
      double v3[3];
      getter(i, v3);
      double* dst = &o[3 * (int64_t)id[i]];
      dst[0] = v3[0];
      dst[1] = v3[1];
      dst[2] = P.dim == 3 ? v3[2] : 0.0;
    }
    o += 3 * n;
  };
  auto sca = [&](auto getter) {
    for (int64_t i = 0; i < n; ++i) o[id[i]] = getter(i);
    o += n;
  };
  const bool exact = sizeof(R) == 8;
  if (mask & SPH_F_X) vec([&](int64_t i, double* v3) {
    const V4<R>& q = pos[i];
    if (exact) { v3[0] = q.x; v3[1] = q.y; v3[2] = q.z; return; }
    uint32_t c = cell[i];
    int cx = (int)(c % (uint32_t)P.nc[0]);
    int cy = (int)((c / (uint32_t)P.nc[0]) % (uint32_t)P.nc[1]);
    int cz = (int)(c / ((uint32_t)P.nc[0] * (uint32_t)P.nc[1]));
    v3[0] = (P.lo[0] + (double)cx * P.L) + (double)q.x;
    v3[1] = (P.lo[1] + (double)cy * P.L) + (double)q.y;
    v3[2] = (P.lo[2] + (double)cz * P.L) + (double)q.z;
  });
  if (mask & SPH_F_U) vec([&](int64_t i, double* v3) { v3[0] = u[i].x; v3[1] = u[i].y; v3[2] = u[i].z; });
  if (mask & SPH_F_A) vec([&](int64_t i, double* v3) {
    bool f = ikind(info[i]) == KF;
    v3[0] = f ? (double)a[i].x : 0.0; v3[1] = f ? (double)a[i].y : 0.0; v3[2] = f ? (double)a[i].z : 0.0;
  });
  if (mask & SPH_F_RHO) sca([&](int64_t i) { return ikind(info[i]) == KW ? 0.0 : (double)rho[i]; });
  if (mask & SPH_F_P) sca([&](int64_t i) { return ikind(info[i]) == KW ? 0.0 : (double)p[i]; });
  if (mask & SPH_F_T) sca([&](int64_t i) { return (double)T[i]; });
  if (mask & SPH_F_PW) sca([&](int64_t i) { return ikind(info[i]) == KF ? 0.0 : (double)pw[i]; });
  if (mask & SPH_F_UW) vec([&](int64_t i, double* v3) {
    bool f = ikind(info[i]) == KF;
    v3[0] = f ? 0.0 : (double)uw[i].x; v3[1] = f ? 0.0 : (double)uw[i].y; v3[2] = f ? 0.0 : (double)uw[i].z;
  });
  if (mask & SPH_F_FR) vec([&](int64_t i, double* v3) {
    if (ikind(info[i]) == KR) { const V4<double>& f = sf[aux[i]]; v3[0] = f.x; v3[1] = f.y; v3[2] = f.z; }
    else { v3[0] = v3[1] = v3[2] = 0.0; }
  });
  if (mask & SPH_F_M) sca([&](int64_t i) { return (double)m[i]; });
  if (mask & SPH_F_DTDT) sca([&](int64_t i) { return (P.thermal && ikind(info[i]) != KW) ? (double)dT[i] : 0.0; });
  // transport-velocity formulation, fluid particles (zero elsewhere and when off)
  auto tv = [&](const std::vector<V4<R>>& f) {
    vec([&](int64_t i, double* v3) {
      const bool on = P.tvf && ikind(info[i]) == KF;
      v3[0] = on ? (double)f[i].x : 0.0; v3[1] = on ? (double)f[i].y : 0.0; v3[2] = on ? (double)f[i].z : 0.0;
    });
  };
  if (mask & SPH_F_AB) tv(ab);
  if (mask & SPH_F_UD) tv(ud);
  return SPH_OK;
}

template <typename R>
int64_t read_neighbors_impl(sph_scene* s, int64_t* offsets, int32_t* ids, int64_t cap) {
  const Params& P = s->P;
  const int64_t n = P.n;
  hipStream_t st = s->stream;
  const KC<R> k = make_kc<R>(P);
  uint32_t* dcnt = nullptr;
  if (hipMalloc(&dcnt, 4 * std::max<int64_t>(n, 1)) != hipSuccess) { fail(SPH_E_DEVICE, "hipMalloc"); return -1; }
  Launch<R>::nb_count(cur<R>(s), P, k, dcnt, st);
  std::vector<uint32_t> cnt(n);
  if (hipStreamSynchronize(st) != hipSuccess ||
      (n > 0 && hipMemcpy(cnt.data(), dcnt, 4 * n, hipMemcpyDeviceToHost) != hipSuccess)) {
    (void)hipFree(dcnt);
    fail(SPH_E_DEVICE, "neighbour count");
    return -1;
  }
  (void)hipFree(dcnt);
  std::vector<uint64_t> off(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) off[i + 1] = off[i] + cnt[i];
  const int64_t tot = (int64_t)off[n];
  if (offsets)
    for (int64_t i = 0; i <= n; ++i) offsets[i] = (int64_t)off[i];
  if (!ids || tot > cap) return tot;
  uint64_t* doff = nullptr;
  uint32_t* dids = nullptr;
  if (hipMalloc(&doff, 8 * (n + 1)) != hipSuccess || hipMalloc(&dids, 4 * std::max<int64_t>(tot, 1)) != hipSuccess) {
    (void)hipFree(doff);
    fail(SPH_E_DEVICE, "hipMalloc");
    return -1;
  }
  (void)hipMemcpy(doff, off.data(), 8 * (n + 1), hipMemcpyHostToDevice);
  Launch<R>::nb_fill(cur<R>(s), P, k, doff, dids, st);
  (void)hipStreamSynchronize(st);
  std::vector<uint32_t> hids(std::max<int64_t>(tot, 1));
  if (tot > 0) (void)hipMemcpy(hids.data(), dids, 4 * tot, hipMemcpyDeviceToHost);
  (void)hipFree(doff);
  (void)hipFree(dids);
  for (int64_t i = 0; i < n; ++i) {
    std::sort(hids.begin() + off[i], hids.begin() + off[i + 1]);
    for (uint64_t q = off[i]; q < off[i + 1]; ++q) ids[q] = (int32_t)hids[q];
  }
  return tot;
}

void quat_rot(const double* q, double* R) {
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

}  // namespace

extern "C" {

int sph_abi_version(void) { return SPH_ABI_VERSION; }

const char* sph_status_string(int status) {
  switch (status) {
    case SPH_OK: return "ok";
    case SPH_E_INVALID: return "invalid argument";
    case SPH_E_NOMEM: return "arena too small";
    case SPH_E_DEVICE: return "HIP runtime error";
    case SPH_E_STATE: return "device error state";
    case SPH_E_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

const char* sph_last_error(void) { return g_last_error.c_str(); }

size_t sph_scene_arena_bytes(const sph_scene_desc* d, int* status) {
  int st = validate(d);
  Params P;
  double mmin;
  if (st == SPH_OK) st = make_params(d, P, &mmin);
  if (status) *status = st;
  if (st != SPH_OK) return 0;
  return arena_for(d, P);
}

int sph_scene_create(const sph_scene_desc* d, void* dev_arena, size_t arena_bytes, void* hip_stream,
                     sph_scene** out) {
  if (!out) return fail(SPH_E_INVALID, "null out");
  *out = nullptr;
  int st = validate(d);
  if (st != SPH_OK) return st;
  sph_scene* s = new (std::nothrow) sph_scene;
  if (!s) return fail(SPH_E_NOMEM, "host allocation");
  std::memset(s, 0, sizeof(*s));
  double mmin;
  st = make_params(d, s->P, &mmin);
  if (st != SPH_OK) { delete s; return st; }
  const size_t need = arena_for(d, s->P);
  if (!dev_arena || arena_bytes < need) {
    delete s;
    return fail(SPH_E_NOMEM, "arena needs " + std::to_string(need) + " bytes");
  }
  if ((reinterpret_cast<uintptr_t>(dev_arena) & 255u) != 0) {
    delete s;
    return fail(SPH_E_INVALID, "arena must be 256-byte aligned");
  }
  s->precision = d->precision;
  s->stream = (hipStream_t)hip_stream;
  s->arena = (char*)dev_arena;
  s->arena_bytes = arena_bytes;
  Carver cv{s->arena, 0};
  if (d->precision == SPH_FP64) carve<double>(cv, s, s->P, d->n_mat);
  else carve<float>(cv, s, s->P, d->n_mat);
  Counts c = count(d);
  s->n_fluid = c.n_fluid;
  s->n_wall = c.n_wall;
  st = d->precision == SPH_FP64 ? create_impl<double>(d, s) : create_impl<float>(d, s);
  if (st != SPH_OK) {
    (void)hipStreamSynchronize(s->stream);
    delete s;
    return st;
  }
  *out = s;
  return SPH_OK;
}

int sph_scene_step(sph_scene* s, int64_t nsteps) {
  if (check_state(s)) return SPH_E_INVALID;
  if (nsteps < 0) return fail(SPH_E_INVALID, "negative step count");
  for (int64_t k = 0; k < nsteps; ++k) {
    if (s->precision == SPH_FP64) one_step<double>(s);
    else one_step<float>(s);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(SPH_E_DEVICE, std::string("launch: ") + hipGetErrorString(e));
  return SPH_OK;
}

size_t sph_batch_bytes(int32_t n) {
  if (n <= 0) return 0;
  // two tables per group, at most 16 groups (precision x dim x thermal x
  // transport-velocity formulation)
  return 2 * ((size_t)n * kSlotMax + 16 * 256) + 256;
}

int sph_batch_create(sph_scene* const* scenes, int32_t n, void* dev_ws, size_t ws_bytes, void* hip_stream,
                     sph_batch** out) {
  if (!out) return fail(SPH_E_INVALID, "null out");
  *out = nullptr;
  if (!scenes || n <= 0) return fail(SPH_E_INVALID, "a batch needs at least one scene");
  for (int32_t q = 0; q < n; ++q) {
    if (!scenes[q]) return fail(SPH_E_INVALID, "null scene in batch");
    for (int32_t r = 0; r < q; ++r)
      if (scenes[r] == scenes[q]) return fail(SPH_E_INVALID, "scene listed twice in batch");
  }
  if (!dev_ws || ws_bytes < sph_batch_bytes(n)) return fail(SPH_E_NOMEM, "batch workspace too small");
  if ((reinterpret_cast<uintptr_t>(dev_ws) & 255u) != 0) return fail(SPH_E_INVALID, "workspace must be 256-byte aligned");
  sph_batch* b = new (std::nothrow) sph_batch;
  if (!b) return fail(SPH_E_NOMEM, "host allocation");
  b->scenes.assign(scenes, scenes + n);
  b->stream = (hipStream_t)hip_stream;
  {
    const char* gv = std::getenv("SPHRB_BATCH_GRAPHS");
    b->use_graphs = gv ? (std::atoi(gv) != 0) : 1;
    // the null stream cannot be captured
    if (!b->stream) b->use_graphs = 0;
  }
  b->ws = (char*)dev_ws;
  b->ws_bytes = ws_bytes;
  size_t off = 0;
  for (int32_t q = 0; q < n; ++q) {
    sph_scene* s = scenes[q];
    sph_batch::Group* g = nullptr;
    for (auto& gg : b->groups)
      if (gg.precision == s->precision && gg.dim == s->P.dim && gg.mode == scene_mode(s)) g = &gg;
    if (!g) {
      b->groups.emplace_back();
      g = &b->groups.back();
      g->precision = s->precision;
      g->dim = s->P.dim;
      g->mode = scene_mode(s);
      g->blocks = 0;
    }
    g->members.push_back(q);
  }
  for (auto& g : b->groups)
    for (int w = 0; w < 2; ++w) {
      g.off[w] = off;
      off = align_up(off + g.members.size() * slot_bytes(g.precision));
    }
  b->ev.assign((size_t)n + 1, nullptr);
  for (auto& e : b->ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      for (auto& e2 : b->ev)
        if (e2) (void)hipEventDestroy(e2);
      delete b;
      return fail(SPH_E_DEVICE, "hipEventCreate");
    }
  *out = b;
  return SPH_OK;
}

int sph_batch_step(sph_batch* b, int64_t nsteps) {
  if (!b) return fail(SPH_E_INVALID, "null batch");
  if (nsteps < 0) return fail(SPH_E_INVALID, "negative step count");
  if (nsteps == 0) return SPH_OK;
  const size_t n = b->scenes.size();
  std::vector<hipStream_t> own(n);
  bool other = false;
  for (size_t q = 0; q < n; ++q) {
    sph_scene* s = b->scenes[q];
    own[q] = s->stream;
    if (s->stream != b->stream) {
      HIP_TRY(hipEventRecord(b->ev[q], s->stream));
      HIP_TRY(hipStreamWaitEvent(b->stream, b->ev[q], 0));
      other = true;
    }
    s->stream = b->stream;
  }
  int st = SPH_OK;
  for (int64_t k = 0; k < nsteps && st == SPH_OK; ++k) st = batch_one_step(b);
  for (size_t q = 0; q < n; ++q) b->scenes[q]->stream = own[q];
  if (other) {
    HIP_TRY(hipEventRecord(b->ev[n], b->stream));
    for (size_t q = 0; q < n; ++q)
      if (own[q] != b->stream) HIP_TRY(hipStreamWaitEvent(own[q], b->ev[n], 0));
  }
  if (st != SPH_OK) return st;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(SPH_E_DEVICE, std::string("launch: ") + hipGetErrorString(e));
  return SPH_OK;
}

void sph_batch_destroy(sph_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  for (auto& g : b->graphs) (void)hipGraphExecDestroy(g.exec);
  for (auto& e : b->ev)
    if (e) (void)hipEventDestroy(e);
  delete b;
}

int sph_scene_sync(sph_scene* s) {
  if (check_state(s)) return SPH_E_INVALID;
  HIP_TRY(hipStreamSynchronize(s->stream));
  uint32_t err = 0;
  HIP_TRY(hipMemcpy(&err, s->err, 4, hipMemcpyDeviceToHost));
  if (err) return fail(SPH_E_STATE, "device error bits " + std::to_string(err));
  return SPH_OK;
}

int sph_scene_read_particles(sph_scene* s, uint32_t field_mask, double* out_host) {
  if (check_state(s)) return SPH_E_INVALID;
  if (!out_host) return fail(SPH_E_INVALID, "null output");
  return s->precision == SPH_FP64 ? read_particles_impl<double>(s, field_mask, out_host)
                                  : read_particles_impl<float>(s, field_mask, out_host);
}

int sph_scene_read_bodies(sph_scene* s, double* out_host, int32_t cap, int32_t* n_bodies) {
  if (check_state(s)) return SPH_E_INVALID;
  HIP_TRY(hipStreamSynchronize(s->stream));
  int64_t nrig = 0;
  int nb = 0;
  if (int e = dyn_counts(s, &nrig, &nb)) return e;
  if (n_bodies) *n_bodies = nb;
  if (!out_host || nb == 0) return SPH_OK;
  std::vector<Body> b(nb);
  HIP_TRY(hipMemcpy(b.data(), s->bodies, sizeof(Body) * nb, hipMemcpyDeviceToHost));
  for (int k = 0; k < std::min(nb, cap); ++k) {
    double* o = &out_host[SPH_BODY_REC * k];
    std::memset(o, 0, sizeof(double) * SPH_BODY_REC);
    const Body& B = b[k];
    o[0] = B.m;
    for (int a = 0; a < 3; ++a) {
      o[1 + a] = B.r[a];
      o[8 + a] = B.u[a];
      o[11 + a] = B.w[a];
      o[14 + a] = B.a[a];
      o[17 + a] = B.al[a];
      o[20 + a] = B.f[a];
      o[23 + a] = B.t[a];
    }
    for (int a = 0; a < 4; ++a) o[4 + a] = B.q[a];
    if (s->P.dim == 3) {
      double R[9], T[9], I[9];
      quat_rot(B.q, R);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          double acc = 0.0;
          for (int q = 0; q < 3; ++q) acc += R[3 * i + q] * B.Ib[3 * q + j];
          T[3 * i + j] = acc;
        }
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          double acc = 0.0;
          for (int q = 0; q < 3; ++q) acc += T[3 * i + q] * R[3 * j + q];
          I[3 * i + j] = acc;
        }
      o[26] = I[0]; o[27] = I[4]; o[28] = I[8]; o[29] = I[1]; o[30] = I[2]; o[31] = I[5];
    } else {
      o[28] = B.Ib[8];
    }
    o[32] = B.active;
    o[33] = B.fixed;
  }
  return SPH_OK;
}

int64_t sph_scene_read_neighbors(sph_scene* s, int64_t* offsets_host, int32_t* ids_host, int64_t cap) {
  if (check_state(s)) return -1;
  if (hipStreamSynchronize(s->stream) != hipSuccess) return -1;
  return s->precision == SPH_FP64 ? read_neighbors_impl<double>(s, offsets_host, ids_host, cap)
                                  : read_neighbors_impl<float>(s, offsets_host, ids_host, cap);
}

int sph_scene_read_cell_order(sph_scene* s, int32_t* sorted_ids_host, int32_t* cell_of_id_host) {
  if (check_state(s)) return SPH_E_INVALID;
  HIP_TRY(hipStreamSynchronize(s->stream));
  const int64_t n = s->P.n;
  std::vector<uint32_t> id(n), cell(n);
  if (n > 0) {
    HIP_TRY(hipMemcpy(id.data(), s->id[s->ip], 4 * n, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(cell.data(), s->cell[s->ip], 4 * n, hipMemcpyDeviceToHost));
  }
  for (int64_t i = 0; i < n; ++i) {
    if (sorted_ids_host) sorted_ids_host[i] = (int32_t)id[i];
    if (cell_of_id_host) cell_of_id_host[id[i]] = (int32_t)cell[i];
  }
  return SPH_OK;
}

int sph_scene_read_flags(sph_scene* s, int32_t* kind_host, int32_t* phase_host, int32_t* body_host) {
  if (check_state(s)) return SPH_E_INVALID;
  HIP_TRY(hipStreamSynchronize(s->stream));
  const int64_t n = s->P.n;
  std::vector<uint32_t> id(n), info(n);
  if (n > 0) {
    HIP_TRY(hipMemcpy(id.data(), s->id[s->ip], 4 * n, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(info.data(), s->info[s->ip], 4 * n, hipMemcpyDeviceToHost));
  }
  for (int64_t i = 0; i < n; ++i) {
    if (kind_host) kind_host[id[i]] = (int32_t)ikind(info[i]);
    if (phase_host) phase_host[id[i]] = (int32_t)iphase(info[i]);
    if (body_host) body_host[id[i]] = ikind(info[i]) == KR ? ibody(info[i]) : -1;
  }
  return SPH_OK;
}

int sph_scene_read_stats(sph_scene* s, sph_stats* o) {
  if (check_state(s)) return SPH_E_INVALID;
  if (!o) return fail(SPH_E_INVALID, "null output");
  std::memset(o, 0, sizeof(*o));
  const Params& P = s->P;
  if (s->precision == SPH_FP64) Launch<double>::global_sums(cur<double>(s), P, s->gpart, kGlobalBlocks, s->gout, s->stream);
  else Launch<float>::global_sums(cur<float>(s), P, s->gpart, kGlobalBlocks, s->gout, s->stream);
  HIP_TRY(hipStreamSynchronize(s->stream));
  unsigned long long pr[kPairSlots];
  uint32_t err = 0;
  double g[6];
  uint32_t dyn[4];
  if (int e = read_pairs(s, pr)) return e;
  HIP_TRY(hipMemcpy(&err, s->err, 4, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(g, s->gout, sizeof(g), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(dyn, s->dyn, sizeof(dyn), hipMemcpyDeviceToHost));
  int64_t nrig = 0;
  int nbod = 0;
  if (int e = dyn_counts(s, &nrig, &nbod)) return e;
  o->step = s->step;
  o->t = (double)s->step * P.dt;
  o->dt = P.dt;
  o->k_c = P.kc;
  o->d_c = P.dc;
  o->n = P.n;
  o->n_fluid = P.n - s->n_wall - nrig;
  o->n_wall = s->n_wall;
  o->n_rigid = nrig;
  o->n_bodies = nbod;
  for (int a = 0; a < 3; ++a) o->grid[a] = P.nc[a];
  o->pairs_last = (int64_t)pr[0];
  o->pairs_total = (int64_t)pr[1];
  o->pairs_fluid = (int64_t)pr[2];
  o->pairs_rigid = (int64_t)pr[3];
  o->pairs_wall = (int64_t)pr[4];
  o->device_error = err;
  // fluid part from the device reduction, bodies added here
  double mass = g[0], mom[3] = {g[1], g[2], g[3]}, ke = g[4], pe = g[5];
  if (nbod > 0) {
    std::vector<Body> b(nbod);
    HIP_TRY(hipMemcpy(b.data(), s->bodies, sizeof(Body) * nbod, hipMemcpyDeviceToHost));
    for (const Body& B : b) {
      if (!B.active) continue;
      mass += B.m;
      for (int a = 0; a < 3; ++a) mom[a] += B.m * B.u[a];
      ke += 0.5 * B.m * (B.u[0] * B.u[0] + B.u[1] * B.u[1] + B.u[2] * B.u[2]);
      // rotational part, w . (R I^b R^T) w / 2
      if (P.dim == 3) {
        double R[9], wb[3], Iwb[3];
        quat_rot(B.q, R);
        for (int a = 0; a < 3; ++a) wb[a] = R[a] * B.w[0] + R[3 + a] * B.w[1] + R[6 + a] * B.w[2];
        for (int a = 0; a < 3; ++a) Iwb[a] = B.Ib[3 * a] * wb[0] + B.Ib[3 * a + 1] * wb[1] + B.Ib[3 * a + 2] * wb[2];
        ke += 0.5 * (wb[0] * Iwb[0] + wb[1] * Iwb[1] + wb[2] * Iwb[2]);
      } else {
        ke += 0.5 * B.Ib[8] * B.w[2] * B.w[2];
      }
      pe -= B.m * (B.b[0] * B.r[0] + B.b[1] * B.r[1] + B.b[2] * B.r[2]);
    }
  }
  o->mass = mass;
  for (int a = 0; a < 3; ++a) o->momentum[a] = mom[a];
  o->kinetic = ke;
  o->potential = pe;
  o->n_melted = P.pswitch ? (int64_t)dyn[2] : 0;
  o->n_solidified = P.pswitch ? (int64_t)dyn[3] : 0;
  return SPH_OK;
}

int sph_scene_enable_timers(sph_scene* s, int32_t enable) {
  if (check_state(s)) return SPH_E_INVALID;
  if (enable && !s->ev) {
    s->ev = new (std::nothrow) std::vector<hipEvent_t>((size_t)SPH_TIMER_STEPS * (SPH_TIMER_STAGES + 1), nullptr);
    if (!s->ev) return fail(SPH_E_NOMEM, "host allocation");
    for (hipEvent_t& e : *s->ev) HIP_TRY(hipEventCreate(&e));
  }
  s->timers = enable ? 1 : 0;
  s->rec = 0;
  return SPH_OK;
}

int sph_scene_read_timers(sph_scene* s, double* stage_ms, int64_t* steps, double* step_ms, int64_t cap) {
  if (check_state(s)) return SPH_E_INVALID;
  HIP_TRY(hipStreamSynchronize(s->stream));
  double sum[SPH_TIMER_STAGES] = {0.0};
  const int64_t nrec = s->ev ? s->rec : 0;
  for (int64_t q = 0; q < nrec; ++q) {
    hipEvent_t* e = &(*s->ev)[(size_t)q * (SPH_TIMER_STAGES + 1)];
    static const int from[SPH_TIMER_STAGES] = {0, 1, 2, 3, 4, 5, 6};
    for (int g = 0; g < SPH_TIMER_STAGES; ++g) {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, e[from[g]], e[from[g] + 1]));
      sum[g] += ms;
    }
    if (step_ms && q < cap) {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, e[0], e[SPH_TIMER_STAGES]));
      step_ms[q] = ms;
    }
  }
  if (stage_ms)
    for (int g = 0; g < SPH_TIMER_STAGES; ++g) stage_ms[g] = sum[g];
  if (steps) *steps = nrec;
  return SPH_OK;
}

size_t sph_scene_state_bytes(sph_scene* s) {
  if (!s) return 0;
  return sizeof(StateHeader) + arena_for_params(s->precision, s->P);
}

int sph_scene_read_state(sph_scene* s, void* host_blob, size_t bytes) {
  if (check_state(s)) return SPH_E_INVALID;
  const size_t used = arena_for_params(s->precision, s->P);
  if (!host_blob || bytes < sizeof(StateHeader) + used) return fail(SPH_E_INVALID, "state buffer too small");
  HIP_TRY(hipStreamSynchronize(s->stream));
  StateHeader h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, kStateMagic, 8);
  h.abi = SPH_ABI_VERSION;
  h.precision = s->precision;
  h.arena_used = used;
  h.step = s->step;
  h.n_fluid = s->n_fluid;
  h.n_wall = s->n_wall;
  h.ip = s->ip;
  h.iu = s->iu;
  h.iT = s->iT;
  h.P = s->P;
  std::memcpy(host_blob, &h, sizeof(h));
  HIP_TRY(hipMemcpy(static_cast<char*>(host_blob) + sizeof(h), s->arena, used, hipMemcpyDeviceToHost));
  return SPH_OK;
}

size_t sph_state_arena_bytes(const void* host_blob, size_t bytes, int* status) {
  StateHeader h;
  const int st = parse_state(host_blob, bytes, &h);
  if (status) *status = st;
  return st == SPH_OK ? (size_t)h.arena_used : 0;
}

int sph_scene_create_from_state(const void* host_blob, size_t bytes, void* dev_arena, size_t arena_bytes,
                                void* hip_stream, sph_scene** out) {
  if (!out) return fail(SPH_E_INVALID, "null out");
  *out = nullptr;
  StateHeader h;
  int st = parse_state(host_blob, bytes, &h);
  if (st != SPH_OK) return st;
  if (!dev_arena || arena_bytes < h.arena_used)
    return fail(SPH_E_NOMEM, "arena needs " + std::to_string(h.arena_used) + " bytes");
  if ((reinterpret_cast<uintptr_t>(dev_arena) & 255u) != 0) return fail(SPH_E_INVALID, "arena must be 256-byte aligned");
  sph_scene* s = new (std::nothrow) sph_scene;
  if (!s) return fail(SPH_E_NOMEM, "host allocation");
  std::memset(s, 0, sizeof(*s));
  s->P = h.P;
  s->precision = h.precision;
  s->stream = (hipStream_t)hip_stream;
  s->arena = (char*)dev_arena;
  s->arena_bytes = arena_bytes;
  Carver cv{s->arena, 0};
  if (h.precision == SPH_FP64) carve<double>(cv, s, s->P, s->P.n_mat);
  else carve<float>(cv, s, s->P, s->P.n_mat);
  s->step = h.step;
  s->n_fluid = h.n_fluid;
  s->n_wall = h.n_wall;
  s->ip = h.ip;
  s->iu = h.iu;
  s->iT = h.iT;
  hipError_t e = hipMemcpyAsync(s->arena, static_cast<const char*>(host_blob) + sizeof(StateHeader), h.arena_used,
                                hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) {
    delete s;
    return fail(SPH_E_DEVICE, std::string("state upload: ") + hipGetErrorString(e));
  }
  *out = s;
  return SPH_OK;
}

void sph_scene_destroy(sph_scene* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  if (s->ev) {
    for (hipEvent_t e : *s->ev)
      if (e) (void)hipEventDestroy(e);
    delete s->ev;
  }
  delete s;
}

}  // extern "C"
