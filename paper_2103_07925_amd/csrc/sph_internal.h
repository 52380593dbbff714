// sph_internal.h -- device data layout and launch interface of the HIP
// library behind include/sphrb.h (gfx950 only).
//
// Particle state lives in device memory sorted by (cell, original id); the
// fields that a sort permutes are double-buffered.  FP64 mode stores
// absolute positions; FP32 mode stores the linear cell index plus an FP32
// offset from the cell's origin, so that every position keeps the same
// absolute resolution wherever it is in the domain.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace sphrb {

// The sweeps keep the constants of the first kLdsPhases phases in LDS.
// Fluid phases (and the fluid phases a switch can produce) must be among
// them, and every phase of a thermal scene; rigid and wall particles of
// later phases carry their density and mass in their neighbour record.
constexpr int kLdsPhases = 16;

// Pair counters: kPairSlots counters ([0] last evaluation, [1] running
// total, [2] fluid targets, [3] fluid neighbours of rigid targets, [4] fluid
// neighbours of walls), each spread over kPairParts partial sums kPairStride
// words apart (one cache line each), so that the waves of a sweep do not
// all update one address; a counter's value is the sum of its parts.
constexpr int kPairSlots = 5, kPairParts = 32, kPairStride = 16;
constexpr int kPairWords = kPairSlots * kPairParts * kPairStride;
__host__ __device__ inline int pair_at(int slot, int part) { return (slot * kPairParts + part) * kPairStride; }

template <typename R>
struct alignas(16) V4 {
  R x, y, z, w;
};

enum : uint32_t { KF = 0, KW = 1, KR = 2 };

// info word: bits 0-1 kind, bit 2 moving wall, bits 8-15 phase, bits 16-31
// body + 1 (0: none)
__host__ __device__ inline uint32_t ikind(uint32_t v) { return v & 3u; }
__host__ __device__ inline bool imoving(uint32_t v) { return ((v >> 2) & 1u) != 0u; }
__host__ __device__ inline uint32_t iphase(uint32_t v) { return (v >> 8) & 0xffu; }
__host__ __device__ inline int ibody(uint32_t v) { return (int)(v >> 16) - 1; }
__host__ __device__ inline uint32_t mkinfo(uint32_t kind, uint32_t phase, uint32_t moving, int body) {
  return kind | (moving << 2) | (phase << 8) | ((uint32_t)(body + 1) << 16);
}

enum : uint32_t { ERR_ESCAPE = 1, ERR_CELL = 2, ERR_NONFINITE = 4, ERR_COINCIDENT = 8, ERR_BODYCAP = 16, ERR_NBCAP = 32 };

// per-phase constants in the sweep precision
template <typename R>
struct MatT {
  R rho0, p0, nu, cp, kappa, eta, T_t, inv_rho0, inv_p0, inv_cp;
  R mass;   // particle mass of the phase, rho0 dx^d (as set at creation)
  R b[3];
  int32_t switch_to, dirichlet;
};

// rigid body record (FP64)
struct Body {
  double m, r[3], q[4], u[3], w[3], a[3], al[3], f[3], t[3], Ib[9], b[3];
  int32_t fixed, active, slot0, nslot;
};

// scalar parameters of one scene
struct Params {
  int dim;
  int nc[3];
  int64_t ncells;
  int64_t n;
  double dx, h, rc, rc2, L, lo[3];
  double wnorm, dnorm, vol0, Ir_fac;
  double dt, hdt;
  double kc, dc;
  int thermal, contact, pswitch;
  double wall_A, wall_Om, wall_dir[3];
  int heat_src;
  double sQ, ssig, ss0[2], sv[2], sztop, sdepth;
  int n_mat, nb, maxb;
  int64_t n_rigid, n_moving;
  int64_t nrows, max_waves;
  int64_t slot_cap;     // rigid slot capacity (all particles when phases switch)
  int body_launch;      // bodies covered by body kernels (capacity when phases switch)
  int64_t ext_cap;      // wall and rigid particles at most (extrapolation targets)
  int tvf;              // transport-velocity formulation on
  double pb;            // its background pressure
  int per[3];           // periodic axes (y and z only)
  double period[3];     // their periods (a whole number of cells)
};

// one wavefront of the sweeps: up to 64 consecutive sorted particles of one
// x-row of cells
struct WaveInfo {
  uint32_t p0, cnt, row, pad;
};

// compact neighbour lists, [wave][entry][lane], 16-bit entries: stencil row
// (bits 12-15) and offset from that row's first candidate jlo[wave][row];
// every lane's entries in the canonical order
struct Lists {
  WaveInfo* table;
  uint32_t* nwaves;
  uint16_t* ent;
  uint8_t* cnt;        // entries of every lane (self included), [wave][lane]
  uint8_t* split;      // entries in canonical order from the front; wall and rigid
                       // lanes: their fluid neighbours (the rest from the end)
  uint32_t* ext;       // wall and rigid particles as (wave << 6 | lane), any order
  uint32_t* ext_n;     // their number
  uint32_t* jlo;
};

// constants in the sweep precision
template <typename R>
struct KC {
  R h, inv_h, wnorm, dnorm, rc2, L, dx, dx2, vol0, kc, dc, dt, hdt, pb;
  R per_y, per_z;   // periods of the periodic axes (0 otherwise)
  R lo[3];
};

// device buffers of the phase switch
struct PhaseBufs {
  uint8_t* flag;                // per particle: 1 melts, 2 solidifies
  int32_t* target;              // per particle: body a solidifying particle joins
  uint32_t* label;              // per particle: component label (an original id)
  uint32_t* body_of_id;         // per original id: new body of a component root
  uint32_t* list;               // solidifying particles without a rigid neighbour
  uint32_t* roots;              // component roots
  uint32_t* ctr;                // [0] flagged, [1] queued, [2] joiners, [3] old slots, [6] sorted buffer
  uint32_t* dirty;              // per body: 1 changed, 2 new
  V4<double>* rold;             // per body: centre of mass before the switch
  uint32_t* alive;              // per old slot: still rigid
  uint32_t* alive_sc;           // exclusive scan of alive (slot capacity + 1)
  uint32_t* bsum;               // scan scratch
  unsigned long long* jkey[2];  // joiners: (body << 32 | original id), ping-pong
  uint32_t* jidx[2];            // joiners: sorted particle index, ping-pong
  uint32_t* snew;               // new slots: particle
  int32_t* sbody;               // new slots: body
  uint32_t* sid;                // new slots: original id
  V4<double>* srb;              // new slots: body-frame offset (kept for survivors)
  V4<double>* srk;              // new slots: world-frame offset (kept for survivors)
  V4<double>* srf;              // new slots: particle force of the last evaluation (survivors)
};

// device pointers of one scene
// Neighbour records per particle, written every step by the list build:
// FP32 [pa, vp] (pa: cell offsets x, y, z and packed cell x | kind << 16 |
// phase << 18), then rm with heat; FP64 [rm, vp]; then a copy of u~ - u
// with the transport-velocity option.  vp = (u, p) of fluid, (u~_w, p_w)
// of wall and rigid particles; rm = (rho, m, info bits, T).
__host__ __device__ constexpr int rec_stride(bool fp64, bool thermal, bool tvf) {
  return 2 + ((!fp64 && thermal) ? 1 : 0) + (tvf ? 1 : 0);
}
__host__ __device__ constexpr int rec_rm_slot(bool fp64) { return fp64 ? 0 : 2; }

template <typename R>
struct View {
  // sorted, permuted state (current buffers)
  V4<R>* pos;
  uint32_t* cell;
  V4<R>* u;
  V4<R>* a;
  R* T;
  R* m;
  uint32_t* id;
  uint32_t* info;
  int32_t* aux;
  V4<R>* ud;   // transport-velocity formulation: u~ - u of the last drift (permuted)
  // outputs that are swapped in after a sweep
  V4<R>* u_out;
  R* T_out;
  // per-step fields, sorted order
  R* rho;
  R* p;
  R* pw;
  V4<R>* uw;
  R* dTdt;
  V4<R>* ab;   // transport-velocity formulation: background-pressure acceleration
  V4<R>* pv;   // neighbour records, pvs per particle side by side so that
               // one neighbour's records share cache lines (rec_stride)
  int32_t pvs;
  // cells
  uint32_t* cstart;   // C + 1
  // rigid slots (body-sorted)
  V4<double>* s_rb;   // body-frame offsets
  V4<double>* s_rk;   // world-frame offsets R r^b
  V4<double>* s_f;    // particle forces
  V4<double>* s_aw;   // particle accelerations as material points
  V4<double>* s_x;    // FP64 positions (set-up and phase switch)
  double* s_m;
  int32_t* s_sorted;
  int32_t* s_body;
  uint32_t* s_id;
  // moving walls
  V4<double>* w_x0;
  V4<double>* w_aw;
  int32_t* w_sorted;
  // tables
  const MatT<R>* mat;
  Body* bodies;
  // counters
  uint32_t* err;
  unsigned long long* pairs;   // kPairWords: spread pair counters (pair_at)
  Lists nb;
  uint32_t* dyn;               // [0] rigid particles, [1] bodies (change with phase switches)
  unsigned long long* dstep;   // steps begun (the step being taken, from 1)
  PhaseBufs ps;
};

// one scene of a batched sweep
template <typename R>
struct Slot {
  View<R> v;
  Params P;
  KC<R> k;
  uint32_t b0, nb;   // first block in the batched grid and block count (multiples of 8)
};

// Every buffer pointer of a view, for rebasing the views of a batched slot
// table: the host stores each pointer as an offset from one global base
// address (the batch workspace), the batched kernels add the base back, so
// the compiler sees pointers derived from a global kernel argument (global
// loads) instead of pointers read from memory (flat loads).
template <typename R, typename F>
__host__ __device__ inline void for_each_ptr(View<R>& v, F&& f) {
  f(v.pos); f(v.cell); f(v.u); f(v.a); f(v.T); f(v.m); f(v.id); f(v.info); f(v.aux); f(v.ud);
  f(v.u_out); f(v.T_out); f(v.rho); f(v.p); f(v.pw); f(v.uw); f(v.dTdt); f(v.ab); f(v.pv);
  f(v.cstart); f(v.s_rb); f(v.s_rk); f(v.s_f); f(v.s_aw); f(v.s_x); f(v.s_m); f(v.s_sorted); f(v.s_body);
  f(v.s_id); f(v.w_x0); f(v.w_aw); f(v.w_sorted); f(v.mat); f(v.bodies); f(v.err); f(v.pairs);
  f(v.nb.table); f(v.nb.nwaves); f(v.nb.ent); f(v.nb.cnt); f(v.nb.split); f(v.nb.ext); f(v.nb.ext_n);
  f(v.nb.jlo); f(v.dyn); f(v.dstep);
  f(v.ps.flag); f(v.ps.target); f(v.ps.label); f(v.ps.body_of_id); f(v.ps.list); f(v.ps.roots); f(v.ps.ctr);
  f(v.ps.dirty); f(v.ps.rold); f(v.ps.alive); f(v.ps.alive_sc); f(v.ps.bsum); f(v.ps.jkey[0]); f(v.ps.jkey[1]);
  f(v.ps.jidx[0]); f(v.ps.jidx[1]); f(v.ps.snew); f(v.ps.sbody); f(v.ps.sid); f(v.ps.srb); f(v.ps.srk);
  f(v.ps.srf);
}

struct SortBufs {
  uint32_t* key;
  uint32_t* rank;
  uint32_t* tid;
  uint32_t* tsrc;
  uint32_t* perm;
  uint32_t* ccount;
  uint32_t* bsum;
  int64_t nbsum;
};

// host launchers (one set per precision)
template <typename R>
struct Launch {
  static void kick_drift(const View<R>& v, const Params& P, const KC<R>& k, SortBufs sb, hipStream_t st);
  static void rigid_pose(const View<R>& v, const Params& P, const KC<R>& k, SortBufs sb, double t, hipStream_t st);
  static void wall_motion(const View<R>& v, const Params& P, const KC<R>& k, SortBufs sb, double t, hipStream_t st);
  static void gather(const View<R>& src, const View<R>& dst, const Params& P, SortBufs sb, hipStream_t st);
  static void density(const View<R>& v, const Params& P, const KC<R>& k, hipStream_t st);
  static void extrapolate(const View<R>& v, const Params& P, const KC<R>& k, hipStream_t st);
  static void forces(const View<R>& v, const Params& P, const KC<R>& k, int kick, int heat, hipStream_t st);
  // stage 0 density, 1 extrapolation, 2 forces, over all slots of the table
  // tab: slot table whose view pointers are offsets from gbase
  static void batch_sweep(int stage, const Slot<R>* tab, const char* gbase, int ns, int dim, int mode,
                          uint32_t blocks, int kick, int heat, hipStream_t st);
  static void rigid_velocity(const View<R>& v, const Params& P, hipStream_t st);
  static void global_sums(const View<R>& v, const Params& P, double* partials, int nblocks, double* out, hipStream_t st);
  static void nb_count(const View<R>& v, const Params& P, const KC<R>& k, uint32_t* cnt, hipStream_t st);
  static void nb_fill(const View<R>& v, const Params& P, const KC<R>& k, const uint64_t* off, uint32_t* ids, hipStream_t st);
  static void slot_positions(const View<R>& v, const Params& P, hipStream_t st);
  static void phase_switch(const View<R>& v, const Params& P, const KC<R>& k, const double* matb, hipStream_t st);
};

// precision-independent launchers
void launch_fill_u32(uint32_t* p, uint32_t val, int64_t n, hipStream_t st);
void launch_step_begin(unsigned long long* pairs, unsigned long long* dstep, hipStream_t st);
void launch_zero_pairs(unsigned long long* pairs, bool eval, bool total, hipStream_t st);
// gate (may be NULL): the scan is skipped when gate[0] == 0
void launch_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* bsum, hipStream_t st,
                     const uint32_t* gate = nullptr);
void launch_wave_table(const Params& P, const uint32_t* cstart, uint32_t* wcount, uint32_t* woff, uint32_t* bsum,
                       WaveInfo* table, hipStream_t st);
void launch_sort_keys(const Params& P, SortBufs sb, uint32_t* cstart, const uint32_t* id, hipStream_t st);
// nbd (may be NULL): device-side body count, else P.body_launch bodies
void launch_body_kick_drift(Body* b, const Params& P, const uint32_t* nbd, hipStream_t st);
void launch_mass_props_impl(Body* b, const V4<double>* s_x, const double* s_m, V4<double>* s_rb, V4<double>* s_rk,
                            const Params& P, const uint32_t* only, const uint32_t* nbd, hipStream_t st);
void launch_body_reduce(Body* b, const V4<double>* s_f, const V4<double>* s_rk, const Params& P, int kick,
                        const uint32_t* nbd, hipStream_t st);
void launch_rigid_aw(Body* b, const Params& P, const int32_t* s_body, const V4<double>* s_rk, V4<double>* s_aw, hipStream_t st);

}  // namespace sphrb
