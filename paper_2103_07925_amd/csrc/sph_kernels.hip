// sph_kernels.hip -- HIP kernels of one SPH time step for gfx950.
//
// Every kernel is written for 64-wide wavefronts.  FP64 mode evaluates each
// expression in the same order as the plain definition written out in the
// paper's equations (and gathers neighbours in the canonical order: cells
// dz, dy, dx = -1..1, ascending id inside a cell), so that its sums are
// reproducible by an independent implementation; it is compiled without
// floating-point contraction.  FP32 mode uses hardware reciprocal / square
// root and explicit fused multiply-adds.
#include "sph_internal.h"

namespace sphrb {

// ---------------------------------------------------------------------------
// arithmetic helpers
// ---------------------------------------------------------------------------

template <typename R> struct IsExact { static constexpr bool v = false; };
template <> struct IsExact<double> { static constexpr bool v = true; };

__device__ __forceinline__ double ksqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float ksqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double kdiv(double a, double b) { return a / b; }
__device__ __forceinline__ float kdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double kfma(double a, double b, double c) { return a * b + c; }
__device__ __forceinline__ float kfma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <typename R> __device__ __forceinline__ R p5(R s) { R t = s * s; t = t * t; return t * s; }
template <typename R> __device__ __forceinline__ R p4(R s) { R t = s * s; return t * t; }

// quintic spline (Morris 1997), support 3h, normalised in d dimensions
template <typename R>
__device__ __forceinline__ R kern_w(R r, const KC<R>& k) {
  if constexpr (IsExact<R>::v) {
    R q = r / k.h;
    if (!(q < R(3))) return R(0);
    R w = p5(R(3) - q);
    if (q < R(2)) w = w - R(6) * p5(R(2) - q);
    if (q < R(1)) w = w + R(15) * p5(R(1) - q);
    return w * k.wnorm;
  } else {
    R q = r * k.inv_h;
    R s3 = fmaxf(R(3) - q, R(0)), s2 = fmaxf(R(2) - q, R(0)), s1 = fmaxf(R(1) - q, R(0));
    R w = kfma(R(15), p5(s1), kfma(R(-6), p5(s2), p5(s3)));
    return w * k.wnorm;
  }
}
// W with the normalisation passed in (in FP64 the same arithmetic as kern_w
// when norm is k.wnorm; in FP32 the distances to the spline knots are fused)
template <typename R>
__device__ __forceinline__ R kern_w_norm(R r, const KC<R>& k, R norm) {
  if constexpr (IsExact<R>::v) {
    R q = r / k.h;
    if (!(q < R(3))) return R(0);
    R w = p5(R(3) - q);
    if (q < R(2)) w = w - R(6) * p5(R(2) - q);
    if (q < R(1)) w = w + R(15) * p5(R(1) - q);
    return w * norm;
  } else {
    // n - r / h in one rounding each
    const R mr = -r;
    R s3 = fmaxf(kfma(mr, k.inv_h, R(3)), R(0)), s2 = fmaxf(kfma(mr, k.inv_h, R(2)), R(0));
    R s1 = fmaxf(kfma(mr, k.inv_h, R(1)), R(0));
    R w = kfma(R(15), p5(s1), kfma(R(-6), p5(s2), p5(s3)));
    return w * norm;
  }
}
template <typename R>
__device__ __forceinline__ R kern_dw(R r, const KC<R>& k) {
  if constexpr (IsExact<R>::v) {
    R q = r / k.h;
    if (!(q < R(3))) return R(0);
    R g = p4(R(3) - q);
    if (q < R(2)) g = g - R(6) * p4(R(2) - q);
    if (q < R(1)) g = g + R(15) * p4(R(1) - q);
    return g * k.dnorm;
  } else {
    R q = r * k.inv_h;
    R s3 = fmaxf(R(3) - q, R(0)), s2 = fmaxf(R(2) - q, R(0)), s1 = fmaxf(R(1) - q, R(0));
    R g = kfma(R(15), p4(s1), kfma(R(-6), p4(s2), p4(s3)));
    return g * k.dnorm;
  }
}

__device__ __forceinline__ void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ __forceinline__ void quat_to_rot(const double* q, double* R) {
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
__device__ __forceinline__ void mat_vec(const double* R, const double* v, double* o) {
  o[0] = R[0] * v[0] + R[1] * v[1] + R[2] * v[2];
  o[1] = R[3] * v[0] + R[4] * v[1] + R[5] * v[2];
  o[2] = R[6] * v[0] + R[7] * v[1] + R[8] * v[2];
}
__device__ __forceinline__ void matT_vec(const double* R, const double* v, double* o) {
  o[0] = R[0] * v[0] + R[3] * v[1] + R[6] * v[2];
  o[1] = R[1] * v[0] + R[4] * v[1] + R[7] * v[2];
  o[2] = R[2] * v[0] + R[5] * v[1] + R[8] * v[2];
}
// out = A M A^T with A = R (transpose_first = 0) or R^T (1)
__device__ __forceinline__ void rot_sandwich(const double* R, const double* M, int tf, double* out) {
  double A[9], T[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) A[3 * i + j] = tf ? R[3 * j + i] : R[3 * i + j];
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

// error-free two-sum based (double-double) accumulation
struct DD {
  double hi, lo;
};
__device__ __forceinline__ void dd_add(DD& a, double x) {
  double s = a.hi + x;
  double bb = s - a.hi;
  double e = (a.hi - (s - bb)) + (x - bb);
  a.hi = s;
  a.lo = a.lo + e;
}
__device__ __forceinline__ DD dd_merge(DD a, DD b) {
  double s = a.hi + b.hi;
  double bb = s - a.hi;
  double e = (a.hi - (s - bb)) + (b.hi - bb);
  DD r;
  r.hi = s;
  r.lo = (a.lo + b.lo) + e;
  return r;
}

__device__ __forceinline__ void set_err(uint32_t* err, uint32_t bit) { atomicOr(err, bit); }

// linear cell index of an FP64 position, or -1 outside the grid
// a position along the periodic axes back into [lo, lo + period)
__device__ __forceinline__ void wrap_pos(const Params& P, double* x) {
  for (int a = 1; a < P.dim; ++a) {
    if (!P.per[a]) continue;
    if (x[a] >= P.lo[a] + P.period[a]) x[a] = x[a] - P.period[a];
    else if (x[a] < P.lo[a]) x[a] = x[a] + P.period[a];
  }
}

__device__ __forceinline__ long long cell_of(const Params& P, const double* x, int* c3) {
  long long lin = 0;
  c3[0] = c3[1] = c3[2] = 0;
  for (int a = 0; a < P.dim; ++a) {
    double v = floor((x[a] - P.lo[a]) / P.L);
    // a wrapped coordinate a rounding below lo + period stays in the last cell
    if (P.per[a] && v == (double)P.nc[a]) v = (double)(P.nc[a] - 1);
    if (!(v >= 0.0) || v >= (double)P.nc[a]) return -1;
    c3[a] = (int)v;
  }
  lin = (long long)c3[0] + (long long)P.nc[0] * ((long long)c3[1] + (long long)P.nc[1] * c3[2]);
  return lin;
}

// store an FP64 position into the sweep representation
template <typename R>
__device__ __forceinline__ void put_pos(const Params& P, const double* xin, V4<R>* pos, uint32_t* cell,
                                        uint32_t* key, int64_t i, uint32_t* err) {
  double x[3] = {xin[0], xin[1], xin[2]};
  wrap_pos(P, x);
  int c3[3];
  long long lin = cell_of(P, x, c3);
  if (lin < 0) {
    set_err(err, ERR_ESCAPE);
    lin = 0;
    for (int a = 0; a < P.dim; ++a) {
      double v = floor((x[a] - P.lo[a]) / P.L);
      c3[a] = v < 0.0 ? 0 : (v >= P.nc[a] ? P.nc[a] - 1 : (int)v);
    }
    lin = (long long)c3[0] + (long long)P.nc[0] * ((long long)c3[1] + (long long)P.nc[1] * c3[2]);
  }
  V4<R> o;
  if constexpr (IsExact<R>::v) {
    o.x = x[0]; o.y = x[1]; o.z = P.dim == 3 ? x[2] : 0.0; o.w = 0.0;
  } else {
    float Lf = (float)P.L;
    float off[3] = {0.f, 0.f, 0.f};
    for (int a = 0; a < P.dim; ++a) {
      double rel = (x[a] - P.lo[a]) - (double)c3[a] * P.L;
      float f = (float)rel;
      off[a] = f < 0.f ? 0.f : (f > Lf ? Lf : f);
    }
    o.x = off[0]; o.y = off[1]; o.z = off[2]; o.w = (float)c3[0];
  }
  pos[i] = o;
  if (cell) cell[i] = (uint32_t)lin;
  if (key) key[i] = (uint32_t)lin;
}

// FP64 position of sorted particle i
template <typename R>
__device__ __forceinline__ void get_pos(const Params& P, const View<R>& v, int64_t i, double* x) {
  V4<R> o = v.pos[i];
  if constexpr (IsExact<R>::v) {
    x[0] = o.x; x[1] = o.y; x[2] = o.z;
  } else {
    uint32_t c = v.cell[i];
    int cx = (int)(c % (uint32_t)P.nc[0]);
    int cy = (int)((c / (uint32_t)P.nc[0]) % (uint32_t)P.nc[1]);
    int cz = (int)(c / ((uint32_t)P.nc[0] * (uint32_t)P.nc[1]));
    x[0] = (P.lo[0] + (double)cx * P.L) + (double)o.x;
    x[1] = (P.lo[1] + (double)cy * P.L) + (double)o.y;
    x[2] = P.dim == 3 ? (P.lo[2] + (double)cz * P.L) + (double)o.z : 0.0;
  }
}

// a wave's pair count into the last-evaluation, running-total and per-kind
// counters, in the partial sums of part `part` (the caller's wave or block
// index, so that concurrent waves mostly update different parts)
__device__ __forceinline__ void block_add_pairs(unsigned long long* pairs, unsigned long long cnt, int slot,
                                                int part) {
  for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
  if ((threadIdx.x & 63) == 0 && cnt) {
    const int pt = part & (kPairParts - 1);
    atomicAdd(&pairs[pair_at(0, pt)], cnt);
    atomicAdd(&pairs[pair_at(1, pt)], cnt);
    atomicAdd(&pairs[pair_at(slot, pt)], cnt);
  }
}
// per-evaluation counters (all but the running total) to zero; thread t of
// nt threads clears every nt-th part
__device__ __forceinline__ void clear_eval_pairs(unsigned long long* pairs, int t, int nt) {
  for (int q = t; q < 4 * kPairParts; q += nt) {
    const int slot = q / kPairParts;
    pairs[pair_at(slot == 0 ? 0 : slot + 1, q % kPairParts)] = 0ull;
  }
}

// ---------------------------------------------------------------------------
// neighbour data
//
// The sweeps read each neighbour through records written once per step and
// kept side by side per particle (rec_stride): vp = (u, p) of fluid
// particles and (u~_w, p_w) of wall and rigid particles; rm = (rho, m, info
// bits, T); in FP32 pa, the position record.
// ---------------------------------------------------------------------------

template <typename R>
struct Nbr {
  uint32_t j;
  V4<R> vp;
  V4<R> rm;
  V4<R> ud;   // u~ - u (transport-velocity walks only)
};

__device__ __forceinline__ float info_to_r(uint32_t v, float) { return __uint_as_float(v); }
__device__ __forceinline__ double info_to_r(uint32_t v, double) { return (double)v; }
__device__ __forceinline__ uint32_t r_to_info(float v) { return __float_as_uint(v); }
__device__ __forceinline__ uint32_t r_to_info(double v) { return (uint32_t)v; }

// Per-phase constants the sweeps need for every neighbour, kept in LDS for
// the first kLdsPhases phases.  Set-up guarantees that the sweeps only ask
// for those (fluid phases, every phase of a thermal scene; a rigid or wall
// neighbour of a later phase brings its density and mass in its record), so
// a lookup is one LDS read: a fallback to the global table would become a
// flat load, which waits for every outstanding global load of the wave and
// defeats the pipelined list walks.
constexpr int kMatLds = kLdsPhases;
template <typename R>
struct MatL {
  R eta, kappa, rho0, p0, inv_p0, b0, b1, b2, dir, mass;
};
template <typename R>
__device__ __forceinline__ MatL<R> mat_from(const MatT<R>& M) {
  MatL<R> o;
  o.eta = M.eta; o.kappa = M.kappa; o.rho0 = M.rho0; o.p0 = M.p0; o.inv_p0 = M.inv_p0;
  o.b0 = M.b[0]; o.b1 = M.b[1]; o.b2 = M.b[2]; o.dir = M.dirichlet ? R(1) : R(0);
  o.mass = M.mass;
  return o;
}
// fills the table; every thread of the workgroup calls it (it synchronises)
template <typename R>
__device__ __forceinline__ void stage_mats(MatL<R>* sm, const View<R>& v, const Params& P) {
  const int nm = P.n_mat < kMatLds ? P.n_mat : kMatLds;
  for (int q = threadIdx.x; q < nm; q += blockDim.x) sm[q] = mat_from<R>(v.mat[q]);
  __syncthreads();
}
template <typename R>
__device__ __forceinline__ MatL<R> mat_of(const MatL<R>* sm, const View<R>&, uint32_t ph) {
  return sm[ph < (uint32_t)kMatLds ? ph : 0u];   // clamped: a later phase's result is never used
}

// wall / rigid extrapolation (local force balance of Adami et al. 2012):
// p_w = [sum p_f W + sum rho_f (b_f - a_w).(x_w - x_f) W] / sum W,
// u~_w = 2 u_w - sum u_f W / sum W; returns the number of fluid neighbours
// SUB lanes share a target (each takes every SUB-th neighbour); their
// partial sums are combined in a fixed order and the first lane writes
template <typename R, int DIM, int SUB, typename It>
__device__ __forceinline__ uint32_t extrap_one(const View<R>& v, const KC<R>& k, const MatL<R>* sm, uint32_t i,
                                               bool act, bool writer, It&& it) {
  const uint32_t inf = v.info[i];
  const uint32_t kind = ikind(inf);
  R aw[3] = {R(0), R(0), R(0)};
  if (act && kind == KR) {
    const V4<double> a = v.s_aw[v.aux[i]];
    aw[0] = (R)a.x; aw[1] = (R)a.y; aw[2] = (R)a.z;
  } else if (act && imoving(inf)) {
    const V4<double> a = v.w_aw[v.aux[i]];
    aw[0] = (R)a.x; aw[1] = (R)a.y; aw[2] = (R)a.z;
  }
  R sW = R(0), sp = R(0), su0 = R(0), su1 = R(0), su2 = R(0);
  uint32_t c = 0;
  it(false, [&](const Nbr<R>& nb, R d0, R d1, R d2, R r2) {
    const uint32_t ij = r_to_info(nb.rm.z);
    if (ikind(ij) != KF) return;
    ++c;
    const MatL<R> Mj = mat_of<R>(sm, v, iphase(ij));
    const R W = kern_w<R>(ksqrt(r2), k);
    R dot;
    if constexpr (IsExact<R>::v) {
      dot = (Mj.b0 - aw[0]) * d0 + (Mj.b1 - aw[1]) * d1;
      if (DIM == 3) dot = dot + (Mj.b2 - aw[2]) * d2;
    } else {
      dot = kfma(Mj.b1 - aw[1], d1, (Mj.b0 - aw[0]) * d0);
      if (DIM == 3) dot = kfma(Mj.b2 - aw[2], d2, dot);
    }
    sW = sW + W;
    if constexpr (IsExact<R>::v) {
      sp = sp + (nb.vp.w + nb.rm.x * dot) * W;
      su0 = su0 + nb.vp.x * W;
      su1 = su1 + nb.vp.y * W;
      if (DIM == 3) su2 = su2 + nb.vp.z * W;
    } else {
      sp = kfma(kfma(nb.rm.x, dot, nb.vp.w), W, sp);
      su0 = kfma(nb.vp.x, W, su0);
      su1 = kfma(nb.vp.y, W, su1);
      if (DIM == 3) su2 = kfma(nb.vp.z, W, su2);
    }
  });
  for (int off = 1; off < SUB; off <<= 1) {
    sW = sW + __shfl_xor(sW, off, 64);
    sp = sp + __shfl_xor(sp, off, 64);
    su0 = su0 + __shfl_xor(su0, off, 64);
    su1 = su1 + __shfl_xor(su1, off, 64);
    su2 = su2 + __shfl_xor(su2, off, 64);
    c = c + __shfl_xor(c, off, 64);
  }
  if (!act || !writer) return 0;
  const V4<R> ui = v.u[i];
  V4<R> o;
  R pw;
  if (sW > R(0)) {
    if constexpr (IsExact<R>::v) {
      pw = sp / sW;
      o.x = R(2) * ui.x - su0 / sW;
      o.y = R(2) * ui.y - su1 / sW;
      o.z = DIM == 3 ? R(2) * ui.z - su2 / sW : R(0);
    } else {
      const R inv = R(1) / sW;
      pw = sp * inv;
      o.x = kfma(R(2), ui.x, -su0 * inv);
      o.y = kfma(R(2), ui.y, -su1 * inv);
      o.z = DIM == 3 ? kfma(R(2), ui.z, -su2 * inv) : R(0);
    }
  } else {
    pw = R(0);
    o.x = ui.x; o.y = ui.y; o.z = DIM == 3 ? ui.z : R(0);
  }
  o.w = pw;
  v.pw[i] = pw;
  v.uw[i] = o;
  v.pv[(size_t)v.pvs * i + 1] = o;
  if (kind == KR) v.p[i] = pw;
  return c;
}

template <typename R>
__device__ __forceinline__ R heat_source(const Params& P, double t, const double* x) {
  if (!P.heat_src) return R(0);
  const int up = P.dim - 1;
  if (x[up] < P.sztop - P.sdepth) return R(0);
  const double c0 = P.ss0[0] + P.sv[0] * t;
  const double d0 = x[0] - c0;
  const double ss2 = P.ssig * P.ssig;
  if (P.dim == 3) {
    const double c1 = P.ss0[1] + P.sv[1] * t;
    const double d1 = x[1] - c1;
    const double dd = d0 * d0 + d1 * d1;
    return (R)(P.sQ / (2.0 * 3.14159265358979323846 * ss2) * exp(-dd / (2.0 * ss2)));
  }
  const double dd = d0 * d0;
  return (R)(P.sQ / (sqrt(2.0 * 3.14159265358979323846) * P.ssig) * exp(-dd / (2.0 * ss2)));
}

// Pair force F_ij = m_i a_ij of eq. nummeth_fluid_momentum for fluid "a"
// against neighbour "b" (d = x_a - x_b)
// (d = x_a - x_b); c_out receives (V_a^2 + V_b^2) dW/dr / r
template <typename R, int DIM>
__device__ __forceinline__ void pair_force(R rho_a, R p_a, R m_a, R eta_a, R uax, R uay, R uaz, R rho_b, R p_b,
                                           R m_b, R eta_b, R ubx, R uby, R ubz, R d0, R d1, R d2, R r, R dW,
                                           R* F, R& c_out) {
  if constexpr (IsExact<R>::v) {
    const R Va = m_a / rho_a, Vb = m_b / rho_b;
    const R vv = Va * Va + Vb * Vb;
    const R pt = (rho_b * p_a + rho_a * p_b) / (rho_a + rho_b);
    const R et = (eta_a + eta_b > R(0)) ? (R(2) * eta_a * eta_b) / (eta_a + eta_b) : R(0);
    const R c = vv * dW / r;
    F[0] = c * (et * (uax - ubx) - pt * d0);
    F[1] = c * (et * (uay - uby) - pt * d1);
    F[2] = DIM == 3 ? c * (et * (uaz - ubz) - pt * d2) : R(0);
    c_out = c;
  } else {
    const R Va = m_a * __builtin_amdgcn_rcpf(rho_a), Vb = m_b * __builtin_amdgcn_rcpf(rho_b);
    const R vv = kfma(Va, Va, Vb * Vb);
    const R pt = kfma(rho_b, p_a, rho_a * p_b) * __builtin_amdgcn_rcpf(rho_a + rho_b);
    const R es = eta_a + eta_b;
    const R et = es > R(0) ? (R(2) * eta_a * eta_b) * __builtin_amdgcn_rcpf(es) : R(0);
    const R c = vv * dW * __builtin_amdgcn_rcpf(r);
    F[0] = c * kfma(et, uax - ubx, -pt * d0);
    F[1] = c * kfma(et, uay - uby, -pt * d1);
    F[2] = DIM == 3 ? c * kfma(et, uaz - ubz, -pt * d2) : R(0);
    c_out = c;
  }
}

// Transport-velocity formulation (Sec. "Momentum equation" names it and
// leaves its terms to Adami, Hu, Adams 2013): between two fluid particles
// the divergence of A = rho u (u~ - u) in the pair form of the momentum
// equation, F += c (1/2) (rho_a u_a ((u~ - u)_a . d) + rho_b u_b ((u~ - u)_b . d))
// with the c of pair_force; antisymmetric in (a, b) like the pressure term.
template <typename R, int DIM>
__device__ __forceinline__ void pair_stress(R c, R rho_a, const V4<R>& ua, const V4<R>& da, R rho_b, R ubx,
                                            R uby, R ubz, const V4<R>& db, R d0, R d1, R d2, R* F) {
  if constexpr (IsExact<R>::v) {
    R sa = da.x * d0, sb = db.x * d0;
    sa = sa + da.y * d1;
    sb = sb + db.y * d1;
    if (DIM == 3) {
      sa = sa + da.z * d2;
      sb = sb + db.z * d2;
    }
    const R ha = R(0.5) * rho_a * sa, hb = R(0.5) * rho_b * sb;
    F[0] = F[0] + c * (ha * ua.x + hb * ubx);
    F[1] = F[1] + c * (ha * ua.y + hb * uby);
    if (DIM == 3) F[2] = F[2] + c * (ha * ua.z + hb * ubz);
  } else {
    R sa = da.x * d0, sb = db.x * d0;
    sa = kfma(da.y, d1, sa);
    sb = kfma(db.y, d1, sb);
    if (DIM == 3) {
      sa = kfma(da.z, d2, sa);
      sb = kfma(db.z, d2, sb);
    }
    const R ha = R(0.5) * rho_a * sa, hb = R(0.5) * rho_b * sb;
    F[0] = kfma(c, kfma(ha, ua.x, hb * ubx), F[0]);
    F[1] = kfma(c, kfma(ha, ua.y, hb * uby), F[1]);
    if (DIM == 3) F[2] = kfma(c, kfma(ha, ua.z, hb * ubz), F[2]);
  }
}

// conduction term of eq. nummeth_thermo_heat_equation for one neighbour
// (fluid neighbours: V = m/rho; rigid: m/rho0 of the phase; walls only
// with a prescribed temperature, V = dx^d)
template <typename R>
__device__ __forceinline__ void heat_pair(const KC<R>& k, uint32_t kj, const MatL<R>& Mj, const Nbr<R>& nb, R ka,
                                          R Ti, R r, R dW, R& hs) {
  const bool wall = kj == KW;
  const R Vm = kdiv(nb.rm.y, kj == KF ? nb.rm.x : Mj.rho0);
  const R Vb = wall ? k.vol0 : Vm;
  const R kb = Mj.kappa;
  const bool on = (!wall || Mj.dir != R(0)) && (ka + kb > R(0));
  if constexpr (IsExact<R>::v) {
    const R kk = (R(4) * ka * kb) / (ka + kb);
    const R add = (Vb * kk) * ((Ti - nb.rm.w) / r) * dW;
    if (on) hs = hs + add;
  } else {
    const R kk = (R(4) * ka * kb) * __builtin_amdgcn_rcpf(ka + kb);
    const R nh = kfma((Vb * kk) * ((Ti - nb.rm.w) * __builtin_amdgcn_rcpf(r)), dW, hs);
    hs = on ? nh : hs;
  }
}

// inverse equation of state of a phase: rho = rho0 (p / p0 + 1)
template <typename R>
__device__ __forceinline__ R inv_eos(const MatL<R>& M, R p) {
  if constexpr (IsExact<R>::v) return M.rho0 * (p / M.p0 + R(1));
  else return M.rho0 * kfma(p, M.inv_p0, R(1));
}

// Momentum (eq. nummeth_fluid_momentum) of fluid particles with the second
// kick, coupling force f_ri = -m_i a_ir (eq. nummeth_fluid_couplingforce)
// and spring-dashpot contact (eq. nummeth_rigid_contactforce) of rigid
// particles, and conduction (eq. nummeth_thermo_heat_equation), in one pass
// over the target's neighbours.  Every lane of the wave calls it (the
// iterator synchronises); only lanes with act set have a target.
// With TVF the transport-velocity formulation adds the stress term between
// fluid pairs and the background-pressure acceleration
// a_b = -(p_b / m_i) sum_j (V_i^2 + V_j^2) dW/dr e_ij over all neighbours of
// fluid targets.
template <typename R, int DIM, int THERMAL, int TVF, typename It>
__device__ __forceinline__ void forces_one(const View<R>& v, const Params& P, const KC<R>& k, const MatL<R>* sm,
                                           uint32_t i, bool act, int kick, int heat, double t, It&& it) {
  const uint32_t inf = v.info[i];
  const uint32_t kind = ikind(inf);
  const bool fluid = kind == KF;
  const V4<R> ui = v.u[i];
  const R Ti = THERMAL ? v.T[i] : R(0);
  const MatT<R>& Mi = v.mat[iphase(inf)];
  const MatL<R> Li = mat_of<R>(sm, v, iphase(inf));
  const R m_i = v.m[i];
  const R rho_i = v.rho[i];
  const R p_i = v.p[i];
  const R eta_i = Mi.eta;
  const R ka = Mi.kappa;
  const V4<R> vpr = v.pv[(size_t)rec_stride(IsExact<R>::v, THERMAL, TVF) * i + 1];
  const R pw_r = vpr.w;
  const int body_i = ibody(inf);
  V4<R> udi;
  if constexpr (TVF) udi = v.ud[i];
  R acc0 = R(0), acc1 = R(0), acc2 = R(0), hs = R(0);
  R bs0 = R(0), bs1 = R(0), bs2 = R(0);
  bool coincident = false;
  it(false, [&](const Nbr<R>& nb, R d0, R d1, R d2, R r2) {
    if (r2 == R(0)) { coincident = true; return; }
    const uint32_t ij = r_to_info(nb.rm.z);
    const uint32_t kj = ikind(ij);
    const bool fj = kj == KF;
    const MatL<R> Mj = mat_of<R>(sm, v, iphase(ij));
    const R r = ksqrt(r2);
    const R dW = kern_dw<R>(r, k);
    if (fluid || fj) {
      // one pair formula for both couplings: a fluid target against any
      // neighbour (a wall or rigid neighbour enters with p_w, u~_w, the
      // density of p_w under the target's phase, the target's mass and
      // viscosity), and a rigid target against a fluid neighbour (the
      // rigid side enters the same way under the neighbour's phase);
      // F(a, b, x_a - x_b) = -F(b, a, x_b - x_a) exactly, so the rigid
      // target's sum equals that of f_ri = -m_i a_ir
      const R rB = fj ? nb.rm.x : inv_eos<R>(Li, nb.vp.w);
      const R rA = fluid ? rho_i : inv_eos<R>(Mj, pw_r);
      const R pA = fluid ? p_i : pw_r;
      const R mA = fluid ? m_i : nb.rm.y;
      const R eA = fluid ? eta_i : Mj.eta;
      const R mB = fj ? nb.rm.y : m_i;
      const R eB = fj ? Mj.eta : eta_i;
      const R uA0 = fluid ? ui.x : vpr.x, uA1 = fluid ? ui.y : vpr.y, uA2 = fluid ? ui.z : vpr.z;
      R F[3], c;
      pair_force<R, DIM>(rA, pA, mA, eA, uA0, uA1, uA2, rB, nb.vp.w, mB, eB, nb.vp.x, nb.vp.y, nb.vp.z, d0, d1, d2,
                         r, dW, F, c);
      if constexpr (TVF) {
        if (fluid && fj) pair_stress<R, DIM>(c, rho_i, ui, udi, nb.rm.x, nb.vp.x, nb.vp.y, nb.vp.z, nb.ud, d0, d1,
                                             d2, F);
        if constexpr (IsExact<R>::v) {
          bs0 = bs0 + c * d0;
          bs1 = bs1 + c * d1;
          if (DIM == 3) bs2 = bs2 + c * d2;
        } else {
          bs0 = kfma(c, d0, bs0);
          bs1 = kfma(c, d1, bs1);
          if (DIM == 3) bs2 = kfma(c, d2, bs2);
        }
      }
      acc0 = acc0 + F[0];
      acc1 = acc1 + F[1];
      if (DIM == 3) acc2 = acc2 + F[2];
    } else if (P.contact && r2 < k.dx2 && (kj == KW || ibody(v.info[nb.j]) != body_i)) {
      const V4<R> uj = v.u[nb.j];
      R e0, e1, e2 = R(0), en;
      if constexpr (IsExact<R>::v) {
        e0 = d0 / r;
        e1 = d1 / r;
        en = e0 * (ui.x - uj.x);
        en = en + e1 * (ui.y - uj.y);
        if (DIM == 3) { e2 = d2 / r; en = en + e2 * (ui.z - uj.z); }
      } else {
        const R ir = __builtin_amdgcn_rcpf(r);
        e0 = d0 * ir;
        e1 = d1 * ir;
        en = kfma(e1, ui.y - uj.y, e0 * (ui.x - uj.x));
        if (DIM == 3) { e2 = d2 * ir; en = kfma(e2, ui.z - uj.z, en); }
      }
      const R fn = k.kc * (r - k.dx) + k.dc * en;
      if (fn < R(0)) {
        acc0 = acc0 - fn * e0;
        acc1 = acc1 - fn * e1;
        if (DIM == 3) acc2 = acc2 - fn * e2;
      }
    }
    if (THERMAL) heat_pair<R>(k, kj, Mj, nb, ka, Ti, r, dW, hs);
  });
  if (!act) return;
  if (fluid) {
    R a0, a1, a2;
    if constexpr (IsExact<R>::v) {
      a0 = acc0 / m_i + Mi.b[0];
      a1 = acc1 / m_i + Mi.b[1];
      a2 = DIM == 3 ? acc2 / m_i + Mi.b[2] : R(0);
    } else {
      const R im = R(1) / m_i;
      a0 = kfma(acc0, im, Mi.b[0]);
      a1 = kfma(acc1, im, Mi.b[1]);
      a2 = DIM == 3 ? kfma(acc2, im, Mi.b[2]) : R(0);
    }
    V4<R> av;
    av.x = a0; av.y = a1; av.z = a2; av.w = R(0);
    v.a[i] = av;
    if constexpr (TVF) {
      V4<R> b;
      if constexpr (IsExact<R>::v) {
        b.x = -(k.pb * bs0) / m_i;
        b.y = -(k.pb * bs1) / m_i;
        b.z = DIM == 3 ? -(k.pb * bs2) / m_i : R(0);
      } else {
        const R f = -k.pb / m_i;
        b.x = f * bs0;
        b.y = f * bs1;
        b.z = DIM == 3 ? f * bs2 : R(0);
      }
      b.w = R(0);
      v.ab[i] = b;
    }
    V4<R> un = ui;
    if (kick) {
      un.x = ui.x + k.hdt * a0;
      un.y = ui.y + k.hdt * a1;
      if (DIM == 3) un.z = ui.z + k.hdt * a2;
    }
    v.u_out[i] = un;
  } else {
    V4<double> f;
    f.x = (double)acc0; f.y = (double)acc1; f.z = DIM == 3 ? (double)acc2 : 0.0; f.w = 0.0;
    v.s_f[v.aux[i]] = f;
    v.u_out[i] = ui;
    if constexpr (TVF) {
      // a rigid particle that melts starts without a background acceleration
      V4<R> z;
      z.x = z.y = z.z = z.w = R(0);
      v.ab[i] = z;
    }
  }
  if (coincident) set_err(v.err, ERR_COINCIDENT);
  if (THERMAL) {
    const R rho_a = fluid ? rho_i : Mi.rho0;
    R rate;
    if constexpr (IsExact<R>::v) rate = hs / (rho_a * Mi.cp);
    else rate = hs * __builtin_amdgcn_rcpf(rho_a * Mi.cp);
    if (P.heat_src) {
      double x[3];
      get_pos<R>(P, v, i, x);
      if constexpr (IsExact<R>::v) rate = rate + heat_source<R>(P, t, x) / Mi.cp;
      else rate = kfma(heat_source<R>(P, t, x), Mi.inv_cp, rate);
    }
    v.dTdt[i] = rate;
    // a phase with a prescribed value (e.g. a fixed concentration) keeps it
    v.T_out[i] = (heat && Li.dir == R(0)) ? Ti + k.dt * rate : Ti;
  }
}

// ---------------------------------------------------------------------------
// compact neighbour lists
//
// Waves are aligned to x-rows of cells: wave w holds at most 64 consecutive
// sorted particles of one row, so its lanes share the 3 x 3 (3D) or 3 (2D)
// stencil rows, and in each stencil row the union of the lanes' windows is
// one contiguous range of the sorted arrays.  Every lane keeps its
// neighbours as 16-bit entries (row << 12 | offset from the row's first
// candidate) in the order the candidates are visited: stencil rows dz, dy
// (outer to inner), then memory order inside a row, i.e. cells dx = -1, 0, 1
// and ascending id -- the canonical gather order.  Waves are dispatched so
// that each XCD works on one contiguous share of them (a spatial slab that
// stays in its L2).
// ---------------------------------------------------------------------------

template <int DIM> struct Nb {
  static constexpr int cap = 192;   // entries per lane, self included (counts are bytes)
  static constexpr int rows = DIM == 3 ? 9 : 3;
};
template <typename R> struct Win { static constexpr int v = 256; };
template <> struct Win<double> { static constexpr int v = 128; };

// workgroup b of G -> wave index, so that XCD (b mod 8) gets a contiguous range
__device__ __forceinline__ int xcd_wave(int b, int G) {
  const int x = b & 7, q = G >> 3, r = G & 7;
  return x * q + (x < r ? x : r) + (b >> 3);
}

// geometry of one wave's stencil rows
struct WaveGeo {
  int cy, cz, cx_first, cx_last, clo, chi;
};

template <typename R>
__device__ __forceinline__ WaveGeo wave_geo(const View<R>& v, const Params& P, const WaveInfo& wi) {
  WaveGeo g;
  const int nx = P.nc[0], ny = P.nc[1];
  g.cy = (int)(wi.row % (uint32_t)ny);
  g.cz = (int)(wi.row / (uint32_t)ny);
  const uint32_t rowbase = wi.row * (uint32_t)nx;
  g.cx_first = (int)(v.cell[wi.p0] - rowbase);
  g.cx_last = (int)(v.cell[wi.p0 + wi.cnt - 1] - rowbase);
  g.clo = g.cx_first - 1 < 0 ? 0 : g.cx_first - 1;
  g.chi = g.cx_last + 1 > nx - 1 ? nx - 1 : g.cx_last + 1;
  return g;
}

// periodic image of every stencil row of a wave in cell row (cy, cz): 4 bits
// per row (y, z: 0 image below, 1 none, 2 image above); used by the FP64 walks
template <int DIM>
__device__ __forceinline__ uint64_t wrap_codes(const Params& P, int cy, int cz) {
  uint64_t wc = 0;
  for (int rr = 0; rr < (DIM == 3 ? 9 : 3); ++rr) {
    const int dy = rr % 3 - 1, dz = DIM == 3 ? rr / 3 - 1 : 0;
    const int yy = cy + dy, zz = cz + dz;
    const uint64_t ky = (P.per[1] && yy < 0) ? 0u : ((P.per[1] && yy >= P.nc[1]) ? 2u : 1u);
    const uint64_t kz = (DIM == 3 && P.per[2] && zz < 0) ? 0u : ((DIM == 3 && P.per[2] && zz >= P.nc[2]) ? 2u : 1u);
    wc |= (ky | (kz << 2)) << (4 * rr);
  }
  return wc;
}

// position in the wave's frame: FP64 absolute; FP32 relative to the origin
// of cell (cx_first, cy, cz), from the cell-relative offset
template <typename R>
__device__ __forceinline__ V4<R> to_frame(const V4<R>& p, const KC<R>& k, int cx_first, int dy, int dz) {
  if constexpr (IsExact<R>::v) {
    return p;
  } else {
    V4<R> s;
    s.x = kfma(p.w - (R)cx_first, k.L, p.x);
    s.y = kfma((R)dy, k.L, p.y);
    s.z = kfma((R)dz, k.L, p.z);
    s.w = R(0);
    return s;
  }
}

template <typename R, int DIM>
__device__ __forceinline__ R dist2(const V4<R>& T, const V4<R>& s, R& d0, R& d1, R& d2) {
  d0 = T.x - s.x;
  d1 = T.y - s.y;
  d2 = R(0);
  R r2;
  if constexpr (IsExact<R>::v) {
    r2 = d0 * d0 + d1 * d1;
    if (DIM == 3) { d2 = T.z - s.z; r2 = r2 + d2 * d2; }
  } else {
    r2 = kfma(d1, d1, d0 * d0);
    if (DIM == 3) { d2 = T.z - s.z; r2 = kfma(d2, d2, r2); }
  }
  return r2;
}

// 2 m + (r2 < rc2): in FP32 one compare into VCC and one add with carry
// (the compiler otherwise spends a select, a shift and an or per bit)
__device__ __forceinline__ uint32_t push_hit(uint32_t m, float r2, float rc2) {
  uint32_t out;
  asm("v_cmp_gt_f32 vcc, %2, %1\n\tv_addc_co_u32 %0, vcc, %3, %3, vcc"
      : "=v"(out) : "v"(r2), "s"(rc2), "v"(m) : "vcc");
  return out;
}
__device__ __forceinline__ uint32_t push_hit(uint32_t m, double r2, double rc2) {
  return m + m + (r2 < rc2 ? 1u : 0u);
}

// maximum over the wave, returned as a wave-uniform (scalar) value so that
// loops bounded by it are controlled by scalar instructions
__device__ __forceinline__ int wave_max_i(int x) {
  for (int off = 32; off > 0; off >>= 1) {
    int y = __shfl_xor(x, off, 64);
    x = y > x ? y : x;
  }
  return __builtin_amdgcn_readfirstlane(x);
}

// Walk one lane's list: entry q of lane l sits at [wave][q][l] (entries
// from split on at [wave][CAP - 1 - (q - split)][l]: the non-fluid
// neighbours of wall and rigid lanes, stored from the end), so the
// wave reads one 128-byte line per step; the entry gives the stencil row
// (bits 12-15) and the offset from that row's first candidate, whose index
// jl[] holds (LDS).  The neighbour's position and records are read straight
// from the sorted arrays (they stay in the L1/L2 caches across the lanes and
// the neighbouring waves).  Lanes go through their own count, so lanes of a
// wave finish together whatever part of their neighbourhood lies in which
// stencil row.
// FP32 sweeps without heat read two 16-byte records per neighbour, one
// 32-byte pair: pa (cell offsets, packed cell x / kind / phase) and vp; a
// fluid neighbour's density is recovered from its pressure by the inverse
// equation of state and its mass is that of its phase.  FP32 sweeps with
// heat add the neighbour's rm record (density, mass, temperature); FP64
// sweeps read the position and the pair (rm, vp); transport-velocity force
// sweeps add the neighbour's u~ - u.  A particle's records sit side by side
// (S per particle, rec_stride), so they share cache lines.
// The walk is software-pipelined: while neighbour q is evaluated, the
// records of q + 1 and the list entry of q + 2 are in flight.
template <typename R>
struct NbRec {
  V4<R> a, vp, rm, ud;
};

// gl: the lane's column of its wave's list block; jl: the stencil-row bases
// of the lane's wave; cx_first: the first cell of the lane's wave (frame)
// (entries q0, q0 + dq, ... of the first n_lane)
// frame offsets (dy L, dz L) of the stencil rows of the list walks, into LDS
// (rows in the order dz outer, dy inner; 2D: dz = 0); the caller synchronises
template <typename R, int DIM>
__device__ __forceinline__ void stage_rows(R* ro, const KC<R>& k) {
  constexpr int NR = Nb<DIM>::rows;
  const int t = (int)threadIdx.x;
  if (t < NR) {
    ro[2 * t] = (R)(t % 3 - 1) * k.L;
    ro[2 * t + 1] = DIM == 3 ? (R)(t / 3 - 1) * k.L : R(0);
  }
}

template <typename R, int DIM, bool PACKED, bool UD, typename F>
__device__ __forceinline__ void for_list(const View<R>& v, const KC<R>& k, const MatL<R>* sm, const R* ro,
                                         int cx_first, uint64_t wc, const uint32_t* jl, const uint16_t* gl,
                                         int S, int n_all, int split, uint32_t i, const V4<R>& T,
                                         bool with_self, F&& visit, int q0 = 0, int dq = 1) {
  constexpr int CAP = Nb<DIM>::cap;
  constexpr bool PK = PACKED && !IsExact<R>::v;
  const int n_lane = n_all > q0 ? (n_all - q0 + dq - 1) / dq : 0;   // this lane's entries
  const int nmax = wave_max_i(n_lane);
  // streamed once: kept out of the L1, which holds the gathered records
  auto entry = [&](int t) -> uint32_t {
    const int q = q0 + t * dq;
    const int at = q < split ? q : CAP - 1 - (q - split);
    return __builtin_nontemporal_load(gl + (size_t)at * 64);
  };
  auto index = [&](uint32_t e) -> uint32_t { return jl[e >> 12] + (e & 0xfffu); };
  auto fetch = [&](uint32_t e, NbRec<R>& r) {
    const uint32_t j = index(e);
    const V4<R>* rec = v.pv + (uint32_t)S * j;   // below 2^32 records: the arena is smaller
    if constexpr (PK) {
      r.a = rec[0];
      r.vp = rec[1];
    } else if constexpr (IsExact<R>::v) {
      r.a = v.pos[j];
      r.rm = rec[rec_rm_slot(true)];
      r.vp = rec[1];
    } else {
      r.a = rec[0];
      r.vp = rec[1];
      r.rm = rec[rec_rm_slot(false)];
    }
    if constexpr (UD) r.ud = rec[S - 1];
  };
  uint32_t e0 = 0u, e1 = 0u;
  NbRec<R> r0;
  if (n_lane > 0) {
    e0 = entry(0);
    fetch(e0, r0);
  }
  if (n_lane > 1) e1 = entry(1);
  for (int q = 0; q < nmax; ++q) {
    NbRec<R> r1;
    uint32_t e2 = 0u;
    if (q + 1 < n_lane) fetch(e1, r1);
    if (q + 2 < n_lane) e2 = entry(q + 2);
    if (q < n_lane) {
      const uint32_t rr = e0 >> 12;
      const uint32_t j = index(e0);
      if (j != i || with_self) {
        Nbr<R> nb;
        nb.j = j;
        nb.vp = r0.vp;
        if constexpr (UD) nb.ud = r0.ud;
        V4<R> pj;
        if constexpr (PK) {
          const uint32_t pk = __float_as_uint(r0.a.w);
          pj.x = r0.a.x;
          pj.y = r0.a.y;
          pj.z = r0.a.z;
          pj.w = (R)(pk & 0xffffu);
          // density and mass from the phase: a fluid neighbour has its
          // phase's mass (only melting, which needs the scalar solver and so
          // the unpacked walk, makes a fluid particle with another mass); a
          // wall or rigid neighbour's density and mass are not used by the
          // walks that take packed records
          const uint32_t kj = (pk >> 16) & 3u, ph = (pk >> 18) & 0xffu;
          const MatL<R> M = mat_of<R>(sm, v, ph);
          nb.rm.x = kj == KF ? inv_eos<R>(M, nb.vp.w) : M.rho0;
          nb.rm.y = M.mass;
          nb.rm.z = info_to_r(mkinfo(kj, ph, 0u, -1), R(0));
          nb.rm.w = R(0);
        } else if constexpr (IsExact<R>::v) {
          pj = r0.a;
          nb.rm = r0.rm;
        } else {
          const uint32_t pk = __float_as_uint(r0.a.w);
          pj.x = r0.a.x;
          pj.y = r0.a.y;
          pj.z = r0.a.z;
          pj.w = (R)(pk & 0xffffu);
          nb.rm = r0.rm;
        }
        V4<R> sj;
        if constexpr (IsExact<R>::v) {
          // periodic image of the row (a zero shift leaves the position as is)
          const uint32_t cw = (uint32_t)(wc >> (4u * rr)) & 15u;
          sj = pj;
          sj.y = pj.y + (R)((int)(cw & 3u) - 1) * k.per_y;
          sj.z = pj.z + (R)((int)(cw >> 2) - 1) * k.per_z;
        } else {
          // the wave's frame (cf. to_frame): dy L and dz L are exact, so the
          // sums round like the fused forms
          sj.x = kfma(pj.w - (R)cx_first, k.L, pj.x);
          sj.y = pj.y + ro[2 * rr];
          sj.z = pj.z + ro[2 * rr + 1];
          sj.w = R(0);
        }
        R d0, d1, d2;
        const R r2 = dist2<R, DIM>(T, sj, d0, d1, d2);
        visit(nb, d0, d1, d2, r2);
      }
    }
    e0 = e1;
    e1 = e2;
    r0 = r1;
  }
}

// the wave's stencil-row bases into LDS (every lane of the wave calls it)
template <int DIM>
__device__ __forceinline__ void stage_jlo(uint32_t* jl, const Lists& nb, int w) {
  constexpr int NR = Nb<DIM>::rows;
  if ((int)threadIdx.x < NR) jl[threadIdx.x] = nb.jlo[(size_t)w * NR + threadIdx.x];
  __syncthreads();
}

__global__ void __launch_bounds__(256) k_row_waves(const uint32_t* cstart, int nx, int64_t nrows, uint32_t* wcount) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  const uint32_t n = cstart[(r + 1) * nx] - cstart[r * nx];
  wcount[r] = (n + 63u) >> 6;
}

__global__ void __launch_bounds__(256) k_row_waves_fill(const uint32_t* cstart, int nx, int64_t nrows,
                                                        const uint32_t* woff, WaveInfo* table) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  const uint32_t s = cstart[r * nx];
  const uint32_t n = cstart[(r + 1) * nx] - s;
  const uint32_t w0 = woff[r];
  for (uint32_t q = 0; q * 64u < n; ++q) {
    WaveInfo wi;
    wi.p0 = s + 64u * q;
    wi.cnt = n - 64u * q < 64u ? n - 64u * q : 64u;
    wi.row = (uint32_t)r;
    wi.pad = 0u;
    table[w0 + q] = wi;
  }
}

// Candidate test and density.  Per stencil row the wave stages the row's
// candidate window in LDS (positions in the wave frame; the sign of the
// fourth component marks a non-fluid candidate).  Every lane tests a run of
// 32-candidate words that covers its own cells cx - 1 .. cx + 1 (a common
// word count from a clamped start, so that loop bounds stay wave-uniform)
// and keeps the hit masks in LDS; then it walks its hits in candidate order
// across the words: W summed for the density (eq. nummeth_fluid_densum, the
// particle itself included) and the entry (stencil row << 12 | offset from
// the row's first candidate) appended to its list in HBM for the
// extrapolation and force sweeps.  The equation of state (eq.
// nummeth_fluid_eos) closes the density; the particle's neighbour records
// in pv are written here.

template <typename R, int DIM>
__device__ __forceinline__ void build_density_wave(const View<R>& v, const Params& P, const KC<R>& k, int w) {
  constexpr int CAP = Nb<DIM>::cap, NR = Nb<DIM>::rows, WIN = Win<R>::v, NWD = WIN / 32;
  __shared__ V4<R> stg[WIN + 32];
  __shared__ uint32_t msk[NWD * 64];
  if (w >= (int)*v.nb.nwaves) return;
  const WaveInfo wi = v.nb.table[w];
  const int lane = threadIdx.x;
  const bool active = lane < (int)wi.cnt;
  const uint32_t i = wi.p0 + (active ? (uint32_t)lane : 0u);
  const WaveGeo g = wave_geo<R>(v, P, wi);
  const int nx = P.nc[0], ny = P.nc[1], nz = P.nc[2];
  const V4<R> T = to_frame<R>(v.pos[i], k, g.cx_first, 0, 0);
  const uint32_t inf = v.info[i];
  const uint32_t kind = ikind(inf);
  const bool dens = active && kind == KF;
  // inactive lanes test against an unreachable point and never hit
  const R far = R(1e30);
  const R T0 = active ? T.x : far, T1 = active ? T.y : far, T2 = active ? T.z : far;
  // wall and rigid lanes keep their fluid neighbours first (in canonical
  // order), the others from the end of their block backwards
  const bool part = active && kind != KF;
  // the lane's own cells of every stencil row: cx - 1 .. cx + 1
  const int cxl = active ? (int)(v.cell[i] - wi.row * (uint32_t)nx) : g.cx_first;
  const int ca = cxl - 1 < 0 ? 0 : cxl - 1, cb = cxl + 1 > nx - 1 ? nx - 1 : cxl + 1;
  char* glw = (char*)(v.nb.ent + (size_t)w * CAP * 64);
  // the lane's next front and back slots in its wave's list block (byte
  // offsets: entry q of lane l at 2 (q * 64 + l)); a list with more hits
  // than slots (an error) has its slots overwritten, every one with a
  // valid entry, and is cut to its capacity below
  const int lo2 = 2 * lane, hi2 = 2 * ((CAP - 1) * 64 + lane);
  int fo = lo2, bo = hi2;
  bool overflow = false;
  // W's normalisation for the lanes that sum a density, zero for the others
  const R wsig = dens ? k.wnorm : R(0);
  R sum = R(0);
  for (int rr = 0; rr < NR; ++rr) {
    const int dz = DIM == 3 ? rr / 3 - 1 : 0, dy = rr % 3 - 1;
    int yy = g.cy + dy, zz = g.cz + dz;
    // periodic axes: the stencil row wraps; in FP64 the row's particles are
    // taken at their image (FP32 frames are cell-relative already)
    R shy = R(0), shz = R(0);
    if (P.per[1] && yy < 0) { yy += ny; shy = -(R)P.period[1]; }
    else if (P.per[1] && yy >= ny) { yy -= ny; shy = (R)P.period[1]; }
    if (DIM == 3 && P.per[2] && zz < 0) { zz += nz; shz = -(R)P.period[2]; }
    else if (DIM == 3 && P.per[2] && zz >= nz) { zz -= nz; shz = (R)P.period[2]; }
    uint32_t jlo = 0u, jhi = 0u, llo = 0u, lhi = 0u;
    if (yy >= 0 && yy < ny && zz >= 0 && zz < nz) {
      const uint32_t rb2 = (uint32_t)((zz * ny + yy) * nx);
      jlo = v.cstart[rb2 + g.clo];
      jhi = v.cstart[rb2 + g.chi + 1];
      llo = v.cstart[rb2 + ca] - jlo;
      lhi = v.cstart[rb2 + cb + 1] - jlo;
    }
    if (!active) lhi = llo;
    if (lane == rr) v.nb.jlo[(size_t)w * NR + rr] = jlo;
    for (uint32_t seg = jlo; seg < jhi; seg += (uint32_t)WIN) {
      const int ns = (int)(jhi - seg < (uint32_t)WIN ? jhi - seg : (uint32_t)WIN);
      for (int q = lane; q < ns + 32; q += 64) {
        V4<R> sq;
        if (q < ns) {
          sq = to_frame<R>(v.pos[seg + q], k, g.cx_first, dy, dz);
          if constexpr (IsExact<R>::v) {
            sq.y = sq.y + shy;
            sq.z = sq.z + shz;
          }
          sq.w = ikind(v.info[seg + q]) == KF ? R(0) : R(-1);   // non-fluid: < 0
        } else {
          sq.x = sq.y = sq.z = -far;    // padding: never a neighbour
          sq.w = R(0);
        }
        stg[q] = sq;
      }
      __syncthreads();
      const uint32_t so = seg - jlo;
      const uint32_t tag = ((uint32_t)rr << 12) | so;
      // this lane's candidates inside the segment: [qa, qb); every lane
      // runs over the same number of candidates from qs <= qa, so that it
      // stays inside the segment -- the extra ones lie in cells out of the
      // lane's reach (at least one cell edge >= r_c away in x) and never hit
      const int qa = (int)((llo > so ? llo : so) - so);
      int qb = (int)((lhi < so + (uint32_t)ns ? lhi : so + (uint32_t)ns) - so);
      if (qb < qa) qb = qa;
      if (jhi - jlo > 4096u) {            // entries hold 12-bit offsets: an error
        qb = qa;
        overflow = overflow || active;
      }
      const int mlen = wave_max_i(qb - qa);
      const int qs = qa < ns - mlen ? qa : ns - mlen;
      const int nwd = (mlen + 31) >> 5, wlast = nwd - 1;
      // candidate tests: bit 31 - u of word wd is candidate qs + 32 wd + u
      for (int wd = 0; wd < nwd; ++wd) {
        const V4<R>* sp = stg + qs + 32 * wd;
        uint32_t m = 0u;
#pragma unroll 8
        for (int u = 0; u < 32; ++u) {
          R e0, e1, e2;
          const R a0 = dist2<R, DIM>(V4<R>{T0, T1, T2, R(0)}, sp[u], e0, e1, e2);
          m = push_hit(m, a0, k.rc2);
        }
        msk[wd * 64 + lane] = m;
      }
      // the hits in candidate order: density, and into the lane's list.
      // Every lane walks its own hits across all words of the segment, so
      // the wave loops max-over-lanes of the segment's hits (not the sum
      // over words of each word's maximum)
      // the current word: its mask, its first candidate, that candidate's entry
      int wd = 0;
      uint32_t m = nwd > 0 ? msk[lane] : 0u;
      while (m == 0u && wd < wlast) m = msk[++wd * 64 + lane];
      const V4<R>* sw = stg + qs + 32 * wd;
      uint32_t tw = tag + (uint32_t)(qs + 32 * wd);
      while (m != 0u) {
        const int bit = __builtin_clz(m);
        m &= ~(0x80000000u >> bit);
        const V4<R> sj = sw[bit];
        R d0, d1, d2;
        const R r2 = dist2<R, DIM>(T, sj, d0, d1, d2);
        sum = sum + kern_w_norm<R>(ksqrt(r2), k, wsig);
        const bool front = !part || !(sj.w < R(0));
        const int at = min(max(front ? fo : bo, lo2), hi2);
        *(uint16_t*)(glw + (uint32_t)at) = (uint16_t)(tw + (uint32_t)bit);
        fo += front ? 128 : 0;
        bo -= front ? 0 : 128;
        while (m == 0u && wd < wlast) {
          m = msk[++wd * 64 + lane];
          sw += 32;
          tw += 32u;
        }
      }
      __syncthreads();
    }
  }
  const int nhf = (fo - lo2) >> 7, nhb = (hi2 - bo) >> 7;   // hits, front and back
  overflow = overflow || nhf + nhb > CAP;
  if (overflow && active) set_err(v.err, ERR_NBCAP);
  const int nf = nhf < CAP ? nhf : CAP;
  const int cnt = active ? (nhf + nhb < CAP ? nhf + nhb : CAP) : 0;
  v.nb.cnt[(size_t)w * 64 + lane] = (uint8_t)cnt;
  // wall and rigid lanes join the compact extrapolation list
  const unsigned long long pm = __ballot(part);
  if (pm) {
    uint32_t base = 0u;
    if (lane == 0) base = atomicAdd(v.nb.ext_n, (uint32_t)__popcll(pm));
    base = __shfl(base, 0, 64);
    if (part) {
      const uint32_t below = (uint32_t)__popcll(pm & ((1ull << lane) - 1ull));
      v.nb.ext[base + below] = ((uint32_t)w << 6) | (uint32_t)lane;
    }
  }
  v.nb.split[(size_t)w * 64 + lane] = (uint8_t)(active ? nf : 0);
  unsigned long long pairs = 0;
  if (active) {
    const MatT<R>& M = v.mat[iphase(inf)];
    R rho;
    if (kind == KF) {
      rho = v.m[i] * sum;
      R p;
      if constexpr (IsExact<R>::v) p = M.p0 * (rho / M.rho0 - R(1));
      else p = M.p0 * kfma(rho, M.inv_rho0, R(-1));
      v.p[i] = p;
      V4<R> vp = v.u[i];
      vp.w = p;
      v.pv[(size_t)v.pvs * i + 1] = vp;
      pairs = (unsigned long long)(cnt - 1);
    } else {
      rho = kind == KR ? M.rho0 : R(0);
      if (kind == KW) v.p[i] = R(0);
    }
    v.rho[i] = rho;
    if constexpr (!IsExact<R>::v) {
      const V4<R> po = v.pos[i];
      const uint32_t pk = (uint32_t)po.w | (kind << 16) | (iphase(inf) << 18);
      V4<R> pa;
      pa.x = po.x;
      pa.y = po.y;
      pa.z = po.z;
      pa.w = __uint_as_float(pk);
      v.pv[(size_t)v.pvs * i] = pa;
    }
    V4<R> rm;
    rm.x = rho;
    rm.y = v.m[i];
    rm.z = info_to_r(inf, R(0));
    rm.w = P.thermal ? v.T[i] : R(0);
    // FP32 walks without heat derive density and mass from the phase
    if (IsExact<R>::v || P.thermal) v.pv[(size_t)v.pvs * i + rec_rm_slot(IsExact<R>::v)] = rm;
    // the transport-velocity walks read a neighbour's u~ - u beside its records
    if (P.tvf) v.pv[(size_t)v.pvs * i + v.pvs - 1] = v.ud[i];
  }
  block_add_pairs(v.pairs, pairs, 2, w);
}

template <typename R, int DIM>
__global__ void __launch_bounds__(64) k_build_density(View<R> v, Params P, KC<R> k) {
  build_density_wave<R, DIM>(v, P, k, xcd_wave(blockIdx.x, gridDim.x));
}

// Extrapolation runs over the compact list of wall and rigid particles the
// list build appends (wave << 6 | lane), 64 targets per workgroup, one lane
// each, whatever share of a target's wave was fluid; workgroups stride over
// the list.  (Splitting a target over several lanes makes each list-entry
// load touch several rows of the [entry][lane] layout: slower.)
template <typename R> struct ExtSub { static constexpr int v = 1; };

template <typename R, int DIM>
__device__ __forceinline__ void extrapolate_wave(const View<R>& v, const Params& P, const KC<R>& k, int blk,
                                                 int nblk) {
  constexpr int NR = Nb<DIM>::rows, CAP = Nb<DIM>::cap;
  constexpr int kExtSub = ExtSub<R>::v, kExtPerBlock = 64 / kExtSub;
  __shared__ uint32_t jls[64 * NR];
  const uint32_t total = *v.nb.ext_n;
  if ((uint32_t)blk * kExtPerBlock >= total) return;
  __shared__ MatL<R> smat[kMatLds];
  __shared__ R ro[2 * NR];
  stage_rows<R, DIM>(ro, k);
  stage_mats<R>(smat, v, P);
  const int lane = threadIdx.x, sub = lane & (kExtSub - 1);
  for (uint32_t b = (uint32_t)blk; b * kExtPerBlock < total; b += (uint32_t)nblk) {
    const uint32_t slot = b * kExtPerBlock + (uint32_t)(lane / kExtSub);
    const bool need = slot < total;
    const uint32_t e = v.nb.ext[need ? slot : b * kExtPerBlock];
    const int w = (int)(e >> 6), l = (int)(e & 63u);
    const WaveInfo wi = v.nb.table[w];
    const uint32_t i = wi.p0 + (uint32_t)l;
    const uint32_t kind = ikind(v.info[i]);
    for (int rr = 0; rr < NR; ++rr) jls[lane * NR + rr] = v.nb.jlo[(size_t)w * NR + rr];
    const WaveGeo g = wave_geo<R>(v, P, wi);
    const V4<R> T = to_frame<R>(v.pos[i], k, g.cx_first, 0, 0);
    // fluid neighbours only: the first split entries of a wall / rigid lane
    const int n_f = need ? (int)v.nb.split[(size_t)w * 64 + l] : 0;
    unsigned long long cr = 0, cw = 0;
    const uint32_t c = extrap_one<R, DIM, kExtSub>(v, k, smat, i, need, sub == 0, [&](bool ws, auto&& f) {
      for_list<R, DIM, true, false>(v, k, smat, ro, g.cx_first, wrap_codes<DIM>(P, g.cy, g.cz), jls + lane * NR,
                                    v.nb.ent + (size_t)w * CAP * 64 + l, v.pvs, n_f,
                                    n_f, i, T, ws, f, sub, kExtSub);
    });
    if (need && sub == 0 && kind == KR) cr = c;
    else if (need && sub == 0) cw = c;
    block_add_pairs(v.pairs, cr, 3, (int)b);
    block_add_pairs(v.pairs, cw, 4, (int)b);
  }
}

template <typename R, int DIM>
__global__ void __launch_bounds__(64) k_extrapolate_list(View<R> v, Params P, KC<R> k) {
  extrapolate_wave<R, DIM>(v, P, k, (int)blockIdx.x, (int)gridDim.x);
}

// one wave's force sweep (wave w, lane lane); the material table, the row
// offsets and the wave's stencil-row bases are staged by the caller.
// t = (steps begun) x dt, from the scene's device step counter
template <typename R, int DIM, int THERMAL, int TVF>
__device__ __forceinline__ void forces_wave_body(const View<R>& v, const Params& P, const KC<R>& k, int w,
                                                 int lane, const MatL<R>* smat, const R* ro, const uint32_t* jl,
                                                 int kick, int heat) {
  const WaveInfo wi = v.nb.table[w];
  const bool active = lane < (int)wi.cnt;
  const uint32_t i = wi.p0 + (active ? (uint32_t)lane : 0u);
  const uint32_t kind = ikind(v.info[i]);
  const WaveGeo g = wave_geo<R>(v, P, wi);
  if (active && kind == KW) {
    v.u_out[i] = v.u[i];
    if (THERMAL) v.T_out[i] = v.T[i];
  }
  const bool need = active && kind != KW;
  if (!__any(need)) return;
  const V4<R> T = to_frame<R>(v.pos[i], k, g.cx_first, 0, 0);
  const int n_lane = need ? (int)v.nb.cnt[(size_t)w * 64 + lane] : 0;
  const int split = v.nb.split[(size_t)w * 64 + lane];
  const double t = (double)(*v.dstep) * P.dt;
  forces_one<R, DIM, THERMAL, TVF>(v, P, k, smat, i, need, kick, heat, t, [&](bool ws, auto&& f) {
    for_list<R, DIM, THERMAL == 0, TVF != 0>(v, k, smat, ro, g.cx_first, wrap_codes<DIM>(P, g.cy, g.cz), jl,
                                             v.nb.ent + (size_t)w * Nb<DIM>::cap * 64 + lane,
                                             rec_stride(IsExact<R>::v, THERMAL, TVF), n_lane, split, i, T, ws, f);
  });
}

// kFwpb consecutive waves per workgroup: they run on one CU and share its
// L1, where their neighbour records overlap (0.641 -> 0.628 ms on the 3D
// column against one wave per workgroup; 8 waves: 0.651 ms); group g of
// the scene's groups, every barrier before any wave leaves
constexpr int kFwpb = 4;
template <typename R, int DIM, int THERMAL, int TVF>
__device__ __forceinline__ void forces_group(const View<R>& v, const Params& P, const KC<R>& k, int g, int kick,
                                             int heat) {
  constexpr int NR = Nb<DIM>::rows;
  __shared__ uint32_t jl[kFwpb][NR];
  __shared__ MatL<R> smat[kMatLds];
  __shared__ R ro[2 * NR];
  const int wv = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63u);
  const int w = g * kFwpb + wv;
  const int nwaves = (int)*v.nb.nwaves;
  if (threadIdx.x < (unsigned)NR) {
    const int t = (int)threadIdx.x;
    ro[2 * t] = (R)(t % 3 - 1) * k.L;
    ro[2 * t + 1] = DIM == 3 ? (R)(t / 3 - 1) * k.L : R(0);
  }
  const int nm = P.n_mat < kMatLds ? P.n_mat : kMatLds;
  for (int q = (int)threadIdx.x; q < nm; q += (int)blockDim.x) smat[q] = mat_from<R>(v.mat[q]);
  if (lane < NR && w < nwaves) jl[wv][lane] = v.nb.jlo[(size_t)w * NR + lane];
  __syncthreads();
  if (w < nwaves) forces_wave_body<R, DIM, THERMAL, TVF>(v, P, k, w, lane, smat, ro, jl[wv], kick, heat);
}

template <typename R, int DIM, int THERMAL, int TVF>
__global__ void __launch_bounds__(64 * kFwpb) k_forces_list(View<R> v, Params P, KC<R> k, int kick, int heat) {
  forces_group<R, DIM, THERMAL, TVF>(v, P, k, xcd_wave(blockIdx.x, gridDim.x), kick, heat);
}

// ---------------------------------------------------------------------------
// batched sweeps: one launch over the concatenated waves of several scenes
// of the same kind.  Scene s owns blocks [b0, b0 + nb) of the grid (b0 and
// nb multiples of 8, so a scene's blocks keep their XCD assignment) and runs
// exactly the code of the single-scene kernels.
// ---------------------------------------------------------------------------

// a slot's view with its offsets turned back into pointers from gbase
template <typename R>
__device__ __forceinline__ View<R> slot_view(const Slot<R>& S, const char* gbase) {
  View<R> v = S.v;
  for_each_ptr(v, [&](auto*& p) {
    using T = std::remove_reference_t<decltype(*p)>;
    p = reinterpret_cast<T*>(const_cast<char*>(gbase) + reinterpret_cast<intptr_t>(p));
  });
  return v;
}

template <typename R>
__device__ __forceinline__ int find_slot(const Slot<R>* tab, int ns, uint32_t b) {
  int lo = 0, hi = ns;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (tab[mid].b0 <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <typename R, int DIM>
__global__ void __launch_bounds__(64) k_build_density_batch(const Slot<R>* tab, const char* gbase, int ns) {
  const Slot<R>& S = tab[find_slot<R>(tab, ns, blockIdx.x)];
  const View<R> v = slot_view<R>(S, gbase);
  const Params P = S.P;
  const KC<R> k = S.k;
  build_density_wave<R, DIM>(v, P, k, xcd_wave((int)(blockIdx.x - S.b0), (int)S.nb));
}

template <typename R, int DIM>
__global__ void __launch_bounds__(64) k_extrapolate_batch(const Slot<R>* tab, const char* gbase, int ns) {
  const Slot<R>& S = tab[find_slot<R>(tab, ns, blockIdx.x)];
  const View<R> v = slot_view<R>(S, gbase);
  const Params P = S.P;
  const KC<R> k = S.k;
  extrapolate_wave<R, DIM>(v, P, k, (int)(blockIdx.x - S.b0), (int)S.nb);
}

// workgroup q covers the scene blocks kFwpb q .. kFwpb q + kFwpb - 1, all of
// one scene (b0 and nb are multiples of 8)
template <typename R, int DIM, int THERMAL, int TVF>
__global__ void __launch_bounds__(64 * kFwpb) k_forces_batch(const Slot<R>* tab, const char* gbase, int ns, int kick,
                                                             int heat) {
  const uint32_t b = blockIdx.x * (uint32_t)kFwpb;
  const Slot<R>& S = tab[find_slot<R>(tab, ns, b)];
  const View<R> v = slot_view<R>(S, gbase);
  const Params P = S.P;
  const KC<R> k = S.k;
  forces_group<R, DIM, THERMAL, TVF>(v, P, k, xcd_wave((int)((b - S.b0) / kFwpb), (int)(S.nb / kFwpb)), kick,
                                     heat);
}

// start of a step: per-evaluation pair counters cleared, step counter advanced
__global__ void __launch_bounds__(64) k_step_begin(unsigned long long* pairs, unsigned long long* dstep) {
  clear_eval_pairs(pairs, (int)threadIdx.x, 64);
  if (threadIdx.x == 0) dstep[0] = dstep[0] + 1ull;
}
// pair counters to zero: the per-evaluation ones and / or the running total
__global__ void __launch_bounds__(256) k_zero_pairs(unsigned long long* pairs, int eval, int total) {
  if (eval) clear_eval_pairs(pairs, (int)threadIdx.x, 256);
  if (total && (int)threadIdx.x < kPairParts) pairs[pair_at(1, (int)threadIdx.x)] = 0ull;
}

// neighbour export from the lists (diagnostic): counts, then ids
template <typename R, int DIM>
__global__ void __launch_bounds__(64) k_list_count(View<R> v, Params P, uint32_t* out) {
  constexpr int NR = Nb<DIM>::rows;
  const int w = blockIdx.x;
  if (w >= (int)*v.nb.nwaves) return;
  const WaveInfo wi = v.nb.table[w];
  const int lane = threadIdx.x;
  if (lane >= (int)wi.cnt) return;
  const uint32_t i = wi.p0 + (uint32_t)lane;
  const uint32_t c = v.nb.cnt[(size_t)w * 64 + lane];
  out[v.id[i]] = c > 0 ? c - 1 : 0u;
}

template <typename R, int DIM>
__global__ void __launch_bounds__(64) k_list_fill(View<R> v, Params P, const uint64_t* off, uint32_t* ids) {
  constexpr int CAP = Nb<DIM>::cap, NR = Nb<DIM>::rows;
  const int w = blockIdx.x;
  if (w >= (int)*v.nb.nwaves) return;
  const WaveInfo wi = v.nb.table[w];
  const int lane = threadIdx.x;
  if (lane >= (int)wi.cnt) return;
  const uint32_t i = wi.p0 + (uint32_t)lane;
  const uint16_t* gl = v.nb.ent + (size_t)w * CAP * 64 + lane;
  const uint32_t* jlo = v.nb.jlo + (size_t)w * NR;
  uint64_t o = off[v.id[i]];
  const int c = v.nb.cnt[(size_t)w * 64 + lane], split = v.nb.split[(size_t)w * 64 + lane];
  for (int q = 0; q < c; ++q) {
    const uint32_t e = gl[(size_t)(q < split ? q : CAP - 1 - (q - split)) * 64];
    const uint32_t j = jlo[e >> 12] + (e & 0xfffu);
    if (j != i) ids[o++] = v.id[j];
  }
}

// ---------------------------------------------------------------------------
// time integration of particles
// ---------------------------------------------------------------------------

// first kick and drift of fluid particles, new cell keys of every particle
// (the first workgroup also starts the step: pair counters, step counter)
template <typename R>
__global__ void __launch_bounds__(256) k_kick_drift(View<R> v, Params P, KC<R> k, uint32_t* key) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.x == 0) clear_eval_pairs(v.pairs, (int)threadIdx.x, 256);
  if (i == 0) {
    v.dstep[0] = v.dstep[0] + 1ull;
    *v.nb.ext_n = 0u;
  }
  if (i >= P.n) return;
  const uint32_t inf = v.info[i];
  uint32_t c = v.cell[i];
  if (ikind(inf) == KF) {
    V4<R> u = v.u[i];
    const V4<R> a = v.a[i];
    V4<R> x = v.pos[i];
    u.x = u.x + k.hdt * a.x;
    u.y = u.y + k.hdt * a.y;
    if (P.dim == 3) u.z = u.z + k.hdt * a.z;
    v.u[i] = u;
    if (!isfinite((double)u.x) || !isfinite((double)u.y) || !isfinite((double)u.z)) set_err(v.err, ERR_NONFINITE);
    // the drift velocity: u^{n+1/2}, or with the transport-velocity
    // formulation u~^{n+1/2} = u^{n+1/2} + (dt/2) a_b^n
    V4<R> w = u;
    if (P.tvf) {
      const V4<R> b = v.ab[i];
      V4<R> d;
      d.x = k.hdt * b.x;
      d.y = k.hdt * b.y;
      d.z = P.dim == 3 ? k.hdt * b.z : R(0);
      d.w = R(0);
      v.ud[i] = d;
      w.x = u.x + d.x;
      w.y = u.y + d.y;
      if (P.dim == 3) w.z = u.z + d.z;
    }
    if constexpr (IsExact<R>::v) {
      x.x = x.x + k.dt * w.x;
      x.y = x.y + k.dt * w.y;
      if (P.dim == 3) x.z = x.z + k.dt * w.z;
      double xx[3] = {x.x, x.y, x.z};
      wrap_pos(P, xx);
      x.y = xx[1];
      if (P.dim == 3) x.z = xx[2];
      int c3[3];
      long long lin = cell_of(P, xx, c3);
      if (lin < 0) { set_err(v.err, ERR_ESCAPE); lin = c; }
      c = (uint32_t)lin;
    } else {
      int c3[3];
      c3[0] = (int)(c % (uint32_t)P.nc[0]);
      c3[1] = (int)((c / (uint32_t)P.nc[0]) % (uint32_t)P.nc[1]);
      c3[2] = (int)(c / ((uint32_t)P.nc[0] * (uint32_t)P.nc[1]));
      R o[3] = {x.x, x.y, x.z};
      const R uu[3] = {w.x, w.y, w.z};
      bool esc = false;
      for (int a = 0; a < P.dim; ++a) {
        o[a] = kfma(k.dt, uu[a], o[a]);
        if (o[a] >= k.L || o[a] < R(0)) {
          // re-home by as many cells as the particle moved (one at most
          // under the time-step bounds; more only after a blow-up)
          const R sh = floorf(o[a] / k.L);
          if (!(fabsf(sh) < R(1 << 24))) {
            esc = true;
          } else {
            const int ish = (int)sh;
            o[a] = o[a] - sh * k.L;
            if (P.per[a]) c3[a] = ((c3[a] + ish) % P.nc[a] + P.nc[a]) % P.nc[a];   // through the periodic boundary
            else if (ish < -c3[a] || ish > P.nc[a] - 1 - c3[a]) esc = true;
            else c3[a] += ish;
          }
        }
        if (o[a] < R(0)) o[a] = R(0);
        if (o[a] > k.L) o[a] = k.L;
      }
      if (esc || !isfinite(o[0]) || !isfinite(o[1]) || !isfinite(o[2])) set_err(v.err, esc ? ERR_ESCAPE : ERR_NONFINITE);
      x.x = o[0]; x.y = o[1]; x.z = o[2]; x.w = (R)c3[0];
      c = (uint32_t)((long long)c3[0] + (long long)P.nc[0] * ((long long)c3[1] + (long long)P.nc[1] * c3[2]));
      v.cell[i] = c;
    }
    v.pos[i] = x;
  }
  key[i] = c;
}

// rigid particle pose from its body: r_rk = R r^b, x_r = r_k + r_rk,
// u_r = u_k + w x r_rk, and its acceleration as a material point
template <typename R>
__global__ void __launch_bounds__(256) k_rigid_pose(View<R> v, Params P, uint32_t* key) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= (P.pswitch ? (int64_t)v.dyn[0] : P.n_rigid)) return;
  const int kb = v.s_body[s];
  const Body& B = v.bodies[kb];
  const int64_t i = v.s_sorted[s];
  double Rm[9];
  quat_to_rot(B.q, Rm);
  const V4<double> rb = v.s_rb[s];
  const double rbv[3] = {rb.x, rb.y, rb.z};
  double rk[3], wr[3], t1[3], t3[3];
  mat_vec(Rm, rbv, rk);
  if (P.dim == 2) rk[2] = 0.0;
  cross3(B.w, rk, wr);
  double x[3];
  for (int a = 0; a < 3; ++a) x[a] = a < P.dim ? B.r[a] + rk[a] : 0.0;
  V4<double> rko;
  rko.x = rk[0]; rko.y = rk[1]; rko.z = rk[2]; rko.w = 0.0;
  v.s_rk[s] = rko;
  put_pos<R>(P, x, v.pos, v.cell, key, i, v.err);
  V4<R> u;
  u.x = (R)(B.u[0] + wr[0]);
  u.y = (R)(B.u[1] + wr[1]);
  u.z = P.dim == 3 ? (R)(B.u[2] + wr[2]) : R(0);
  u.w = R(0);
  v.u[i] = u;
  cross3(B.al, rk, t1);
  cross3(B.w, wr, t3);
  V4<double> aw;
  aw.x = B.a[0] + t1[0] + t3[0];
  aw.y = B.a[1] + t1[1] + t3[1];
  aw.z = B.a[2] + t1[2] + t3[2];
  aw.w = 0.0;
  v.s_aw[s] = aw;
}

// moving boundary particles: displacement A (cos(Omega t) - 1) along dir, at
// t = (steps begun) x dt from the scene's device step counter
template <typename R>
__global__ void __launch_bounds__(256) k_wall_motion(View<R> v, Params P, uint32_t* key) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= P.n_moving) return;
  const double t = (double)(*v.dstep) * P.dt;
  const int64_t i = v.w_sorted[s];
  const double sA = P.wall_A * (cos(P.wall_Om * t) - 1.0);
  const double vA = -P.wall_A * P.wall_Om * sin(P.wall_Om * t);
  const double aA = -P.wall_A * P.wall_Om * P.wall_Om * cos(P.wall_Om * t);
  const V4<double> x0 = v.w_x0[s];
  const double xb[3] = {x0.x, x0.y, x0.z};
  double x[3] = {0.0, 0.0, 0.0};
  V4<double> aw;
  aw.x = aw.y = aw.z = aw.w = 0.0;
  V4<R> u;
  u.x = u.y = u.z = u.w = R(0);
  double uu[3] = {0.0, 0.0, 0.0}, aa[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < P.dim; ++a) {
    x[a] = xb[a] + sA * P.wall_dir[a];
    uu[a] = vA * P.wall_dir[a];
    aa[a] = aA * P.wall_dir[a];
  }
  u.x = (R)uu[0]; u.y = (R)uu[1]; u.z = (R)uu[2];
  aw.x = aa[0]; aw.y = aa[1]; aw.z = aa[2];
  put_pos<R>(P, x, v.pos, v.cell, key, i, v.err);
  v.u[i] = u;
  v.w_aw[s] = aw;
}

// u_r = u_k + w_k x r_rk (second kick of rigid particles)
template <typename R>
__global__ void __launch_bounds__(256) k_rigid_velocity(View<R> v, Params P, const uint32_t* gate) {
  if (gate && gate[0] == 0u) return;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= (P.pswitch ? (int64_t)v.dyn[0] : P.n_rigid)) return;
  const Body& B = v.bodies[v.s_body[s]];
  const V4<double> rk = v.s_rk[s];
  const double r[3] = {rk.x, rk.y, rk.z};
  double wr[3];
  cross3(B.w, r, wr);
  V4<R> u;
  u.x = (R)(B.u[0] + wr[0]);
  u.y = (R)(B.u[1] + wr[1]);
  u.z = P.dim == 3 ? (R)(B.u[2] + wr[2]) : R(0);
  u.w = R(0);
  v.u[v.s_sorted[s]] = u;
}

// FP64 positions of rigid slots (for the mass quantities)
template <typename R>
__global__ void __launch_bounds__(256) k_slot_positions(View<R> v, Params P, const uint32_t* gate) {
  if (gate && gate[0] == 0u) return;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= (P.pswitch ? (int64_t)v.dyn[0] : P.n_rigid)) return;
  const int64_t i = v.s_sorted[s];
  double x[3];
  get_pos<R>(P, v, i, x);
  V4<double> o;
  o.x = x[0]; o.y = x[1]; o.z = x[2]; o.w = 0.0;
  v.s_x[s] = o;
  v.s_m[s] = (double)v.m[i];
}

// ---------------------------------------------------------------------------
// counting sort by (cell, id)
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) k_fill_u32(uint32_t* p, uint32_t val, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = val;
}

// Cell counts and a unique rank of every particle inside its cell (the
// order is fixed later by original id).  The keys arrive nearly sorted (the
// previous step's order), so each wave adds whole runs of equal keys with
// one atomic per run.
__global__ void __launch_bounds__(256) k_count(const uint32_t* key, uint32_t* count, uint32_t* rank, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const bool valid = i < n;
  const uint32_t k = valid ? key[i] : 0xffffffffu;
  const uint32_t prev = __shfl_up(k, 1, 64);
  const bool start = lane == 0 || k != prev;
  const unsigned long long starts = __ballot(start);
  const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
  const int leader = 63 - __clzll(starts & upto);
  const unsigned long long after = starts & ~upto;
  const int next = after ? __ffsll((long long)after) - 1 : 64;
  uint32_t base = 0u;
  if (start && valid) base = atomicAdd(&count[k], (uint32_t)(next - lane));
  base = __shfl(base, leader, 64);
  if (valid) rank[i] = base + (uint32_t)(lane - leader);
}

// exclusive scan, 1024 elements per block (256 threads x 4)
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t x, uint32_t* total) {
  __shared__ uint32_t wsum[4];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t inc = x;
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t y = __shfl_up(inc, off, 64);
    if (lane >= off) inc += y;
  }
  if (lane == 63) wsum[wid] = inc;
  __syncthreads();
  uint32_t base = 0, tot = 0;
  for (int w = 0; w < 4; ++w) {
    if (w < wid) base += wsum[w];
    tot += wsum[w];
  }
  __syncthreads();
  *total = tot;
  return base + inc - x;
}

__global__ void __launch_bounds__(256) k_scan_blocks(const uint32_t* in, uint32_t* out, uint32_t* bsum, int64_t n,
                                                     const uint32_t* gate) {
  if (gate && gate[0] == 0u) return;
  const int64_t base = (int64_t)blockIdx.x * 1024 + threadIdx.x * 4;
  uint32_t v[4], s = 0;
  for (int q = 0; q < 4; ++q) {
    v[q] = (base + q < n) ? in[base + q] : 0u;
    s += v[q];
  }
  uint32_t tot;
  uint32_t ex = block_exclusive_scan(s, &tot);
  for (int q = 0; q < 4; ++q) {
    if (base + q < n) out[base + q] = ex;
    ex += v[q];
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(256) k_scan_bsum(uint32_t* bsum, int64_t nb, uint32_t* out_total,
                                                   const uint32_t* gate) {
  if (gate && gate[0] == 0u) return;
  __shared__ uint32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < nb; base += 256) {
    const int64_t i = base + threadIdx.x;
    const uint32_t x = i < nb ? bsum[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(x, &tot);
    const uint32_t c = carry;
    if (i < nb) bsum[i] = ex + c;
    __syncthreads();
    if (threadIdx.x == 0) carry = c + tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) *out_total = carry;
}

__global__ void __launch_bounds__(256) k_scan_add(uint32_t* out, const uint32_t* bsum, int64_t n,
                                                  const uint32_t* gate) {
  if (gate && gate[0] == 0u) return;
  const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x * 4;
  const uint32_t add = bsum[blockIdx.x];
  for (int q = 0; q < 4; ++q)
    if (i + q < n) out[i + q] += add;
}

__global__ void __launch_bounds__(256) k_scatter(const uint32_t* key, const uint32_t* rank, const uint32_t* cstart,
                                                 const uint32_t* id, uint32_t* tid, uint32_t* tsrc, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t d = cstart[key[i]] + rank[i];
  tid[d] = id[i];
  tsrc[d] = (uint32_t)i;
}

// rank inside the cell by original id -> destination of every source
constexpr uint32_t kMaxCellSort = 8192;
__global__ void __launch_bounds__(256) k_rank(const uint32_t* key, const uint32_t* cstart, const uint32_t* tid,
                                              const uint32_t* tsrc, uint32_t* perm, uint32_t* err, int64_t n) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const uint32_t src = tsrc[p];
  const uint32_t c = key[src];
  const uint32_t s0 = cstart[c], s1 = cstart[c + 1];
  if (s1 - s0 > kMaxCellSort) {
    set_err(err, ERR_CELL);
    perm[p] = src;
    return;
  }
  const uint32_t my = tid[p];
  uint32_t r = 0;
  uint32_t q = s0;
  // eight loads in flight per round (one at a time waits out each load)
  for (; q + 8u <= s1; q += 8u) {
    uint32_t t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) t[u] = tid[q + (uint32_t)u];
#pragma unroll
    for (int u = 0; u < 8; ++u) r += (t[u] < my) ? 1u : 0u;
  }
  for (; q < s1; ++q) r += (tid[q] < my) ? 1u : 0u;
  perm[s0 + r] = src;
}

template <typename R>
__global__ void __launch_bounds__(256) k_gather(View<R> a, View<R> b, Params P, const uint32_t* perm,
                                                const uint32_t* key) {
  const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= P.n) return;
  const uint32_t s = perm[d];
  b.pos[d] = a.pos[s];
  b.cell[d] = key[s];
  b.u[d] = a.u[s];
  b.a[d] = a.a[s];
  if (P.tvf) b.ud[d] = a.ud[s];
  b.T[d] = a.T[s];
  b.m[d] = a.m[s];
  b.id[d] = a.id[s];
  const uint32_t inf = a.info[s];
  b.info[d] = inf;
  const int32_t ax = a.aux[s];
  b.aux[d] = ax;
  if (ikind(inf) == KR) a.s_sorted[ax] = (int32_t)d;
  else if (ikind(inf) == KW && imoving(inf)) a.w_sorted[ax] = (int32_t)d;
}

// ---------------------------------------------------------------------------
// rigid bodies
// ---------------------------------------------------------------------------

__device__ __forceinline__ DD wave_reduce_dd(DD a) {
  for (int off = 32; off > 0; off >>= 1) {
    DD b;
    b.hi = __shfl_xor(a.hi, off, 64);
    b.lo = __shfl_xor(a.lo, off, 64);
    a = dd_merge(a, b);
  }
  return a;
}

// block (256 threads) reduction of NV double-double accumulators
template <int NV>
__device__ __forceinline__ void block_reduce_dd(DD* acc, double* out) {
  __shared__ double sh[4][NV][2];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int q = 0; q < NV; ++q) {
    DD r = wave_reduce_dd(acc[q]);
    if (lane == 0) { sh[wid][q][0] = r.hi; sh[wid][q][1] = r.lo; }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 0; q < NV; ++q) {
      DD t;
      t.hi = sh[0][q][0];
      t.lo = sh[0][q][1];
      for (int w = 1; w < 4; ++w) {
        DD b;
        b.hi = sh[w][q][0];
        b.lo = sh[w][q][1];
        t = dd_merge(t, b);
      }
      out[q] = t.hi + t.lo;
    }
  }
  __syncthreads();
}

// body accelerations: a = f/m + b, alpha = (R I^b R^T)^{-1} torque
__device__ void body_accel(Body& B, int dim) {
  if (!B.active || B.fixed) {
    for (int a = 0; a < 3; ++a) { B.a[a] = 0.0; B.al[a] = 0.0; }
    return;
  }
  for (int a = 0; a < 3; ++a) B.a[a] = a < dim ? B.f[a] / B.m + B.b[a] : 0.0;
  if (dim == 2) {
    B.al[0] = 0.0;
    B.al[1] = 0.0;
    B.al[2] = B.t[2] / B.Ib[8];
  } else {
    double Rm[9], I[9];
    quat_to_rot(B.q, Rm);
    rot_sandwich(Rm, B.Ib, 0, I);
    const double c00 = I[4] * I[8] - I[5] * I[7];
    const double c01 = I[5] * I[6] - I[3] * I[8];
    const double c02 = I[3] * I[7] - I[4] * I[6];
    const double det = I[0] * c00 + I[1] * c01 + I[2] * c02;
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
    mat_vec(inv, B.t, B.al);
  }
}

// Per-body force and torque (eqs. procwise_force, global_force): one
// workgroup per body; each lane accumulates a strided share of the body's
// particles in double-double, the wavefront and then the workgroup combine
// the partial sums; lane 0 forms the accelerations and the second kick.
__global__ void __launch_bounds__(256) k_body_reduce(Body* bodies, const V4<double>* s_f, const V4<double>* s_rk,
                                                     int dim, double hdt, int kick, int nbh, const uint32_t* nbd) {
  const int nb = nbd ? (int)*nbd : nbh;
  for (int kb = blockIdx.x; kb < nb; kb += gridDim.x) {
  Body& B = bodies[kb];
  DD acc[6];
  for (int q = 0; q < 6; ++q) { acc[q].hi = 0.0; acc[q].lo = 0.0; }
  const int s0 = B.slot0, ns = B.active ? B.nslot : 0;
  for (int q = threadIdx.x; q < ns; q += blockDim.x) {
    const V4<double> f = s_f[s0 + q];
    const V4<double> r = s_rk[s0 + q];
    const double fv[3] = {f.x, f.y, f.z}, rv[3] = {r.x, r.y, r.z};
    double t[3];
    cross3(rv, fv, t);
    dd_add(acc[0], fv[0]);
    dd_add(acc[1], fv[1]);
    dd_add(acc[2], fv[2]);
    dd_add(acc[3], t[0]);
    dd_add(acc[4], t[1]);
    dd_add(acc[5], t[2]);
  }
  double out[6];
  block_reduce_dd<6>(acc, out);
  if (threadIdx.x == 0) {
    for (int a = 0; a < 3; ++a) {
      B.f[a] = a < dim ? out[a] : 0.0;
      B.t[a] = (dim == 3 || a == 2) ? out[3 + a] : 0.0;
    }
    body_accel(B, dim);
    if (kick && B.active && !B.fixed) {
      for (int a = 0; a < 3; ++a) {
        B.u[a] = B.u[a] + hdt * B.a[a];
        B.w[a] = B.w[a] + hdt * B.al[a];
      }
    }
  }
  }
}

// first kick, drift and orientation update of every body
__global__ void __launch_bounds__(64) k_body_kick_drift(Body* bodies, int nbh, const uint32_t* nbd, double dt,
                                                        double hdt) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (nbd ? (int)*nbd : nbh)) return;
  Body& B = bodies[k];
  if (!B.active || B.fixed) return;
  for (int a = 0; a < 3; ++a) {
    B.u[a] = B.u[a] + hdt * B.a[a];
    B.w[a] = B.w[a] + hdt * B.al[a];
  }
  for (int a = 0; a < 3; ++a) B.r[a] = B.r[a] + dt * B.u[a];
  const double phi[3] = {dt * B.w[0], dt * B.w[1], dt * B.w[2]};
  const double ang = sqrt(phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2]);
  if (ang > 0.0) {
    const double sh = sin(0.5 * ang) / ang;
    const double qi[4] = {cos(0.5 * ang), sh * phi[0], sh * phi[1], sh * phi[2]};
    const double* q = B.q;
    double qn[4];
    qn[0] = qi[0] * q[0] - qi[1] * q[1] - qi[2] * q[2] - qi[3] * q[3];
    qn[1] = qi[0] * q[1] + qi[1] * q[0] + qi[2] * q[3] - qi[3] * q[2];
    qn[2] = qi[0] * q[2] - qi[1] * q[3] + qi[2] * q[0] + qi[3] * q[1];
    qn[3] = qi[0] * q[3] + qi[1] * q[2] - qi[2] * q[1] + qi[3] * q[0];
    const double nq = sqrt(qn[0] * qn[0] + qn[1] * qn[1] + qn[2] * qn[2] + qn[3] * qn[3]);
    for (int a = 0; a < 4; ++a) B.q[a] = qn[a] / nq;
  }
}

// Mass quantities of every body (eqs. procwise_centerofmass and
// procwise_inertia): each wavefront of the workgroup forms the partial mass,
// centre of mass and inertia of its share of particles (a "processor-wise"
// partial), and the partials are combined with Huygens-Steiner (eqs.
// global_centerofmass, global_inertia).  Then I^b = R^T I R and the
// body-frame offsets r^b = R^T (x_r - r_k).
__global__ void __launch_bounds__(256) k_mass_props(Body* bodies, const V4<double>* s_x, const double* s_m,
                                                    V4<double>* s_rb, V4<double>* s_rk, int dim, double Ir_fac,
                                                    const uint32_t* only, int nbh, const uint32_t* nbd,
                                                    const uint32_t* gate) {
  if (gate && gate[0] == 0u) return;
  __shared__ double shm[4], shr[4][3], shI[4][6];
  __shared__ double gr[3];
  const int nb = nbd ? (int)*nbd : nbh;
  for (int kb = blockIdx.x; kb < nb; kb += gridDim.x) {
  __syncthreads();
  if (only && only[kb] == 0u) continue;
  Body& B = bodies[kb];
  const int s0 = B.slot0, ns = B.nslot;
  if (ns == 0) {
    // a body without particles keeps its last state and goes inactive
    if (threadIdx.x == 0) B.active = 0;
    continue;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  // partition: wavefront w takes slots w, w+4, ... in chunks of 64 lanes
  DD am, ax[3];
  am.hi = am.lo = 0.0;
  for (int a = 0; a < 3; ++a) ax[a].hi = ax[a].lo = 0.0;
  for (int q = threadIdx.x; q < ns; q += blockDim.x) {
    const V4<double> x = s_x[s0 + q];
    const double m = s_m[s0 + q];
    dd_add(am, m);
    dd_add(ax[0], m * x.x);
    dd_add(ax[1], m * x.y);
    dd_add(ax[2], m * x.z);
  }
  DD rm = wave_reduce_dd(am);
  DD rx[3] = {wave_reduce_dd(ax[0]), wave_reduce_dd(ax[1]), wave_reduce_dd(ax[2])};
  const double pm = rm.hi + rm.lo;
  double pr[3];
  for (int a = 0; a < 3; ++a) pr[a] = pm > 0.0 ? (rx[a].hi + rx[a].lo) / pm : 0.0;
  // partial inertia about the partial centre of mass
  DD aI[6];
  for (int q = 0; q < 6; ++q) aI[q].hi = aI[q].lo = 0.0;
  for (int q = threadIdx.x; q < ns; q += blockDim.x) {
    const V4<double> x = s_x[s0 + q];
    const double m = s_m[s0 + q];
    const double d[3] = {pr[0] - x.x, pr[1] - x.y, dim == 3 ? pr[2] - x.z : 0.0};
    const double dsq = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (dim == 2) {
      dd_add(aI[2], Ir_fac * m + dsq * m);
    } else {
      dd_add(aI[0], Ir_fac * m + (dsq - d[0] * d[0]) * m);
      dd_add(aI[1], Ir_fac * m + (dsq - d[1] * d[1]) * m);
      dd_add(aI[2], Ir_fac * m + (dsq - d[2] * d[2]) * m);
      dd_add(aI[3], (-(d[0] * d[1])) * m);
      dd_add(aI[4], (-(d[0] * d[2])) * m);
      dd_add(aI[5], (-(d[1] * d[2])) * m);
    }
  }
  double pI[6];
  for (int q = 0; q < 6; ++q) {
    DD r = wave_reduce_dd(aI[q]);
    pI[q] = r.hi + r.lo;
  }
  if (lane == 0) {
    shm[wid] = pm;
    for (int a = 0; a < 3; ++a) shr[wid][a] = pr[a];
    for (int q = 0; q < 6; ++q) shI[wid][q] = pI[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    DD M;
    M.hi = M.lo = 0.0;
    for (int w = 0; w < 4; ++w) dd_add(M, shm[w]);
    const double m = M.hi + M.lo;
    double r[3];
    for (int a = 0; a < 3; ++a) {
      DD s;
      s.hi = s.lo = 0.0;
      for (int w = 0; w < 4; ++w) dd_add(s, shm[w] * shr[w][a]);
      r[a] = (a < dim && m > 0.0) ? (s.hi + s.lo) / m : 0.0;
    }
    double I6[6];
    for (int q = 0; q < 6; ++q) {
      DD s;
      s.hi = s.lo = 0.0;
      for (int w = 0; w < 4; ++w) {
        const double d[3] = {r[0] - shr[w][0], r[1] - shr[w][1], dim == 3 ? r[2] - shr[w][2] : 0.0};
        const double dsq = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        double st;
        if (q < 3) st = dsq - d[q] * d[q];
        else if (q == 3) st = -(d[0] * d[1]);
        else if (q == 4) st = -(d[0] * d[2]);
        else st = -(d[1] * d[2]);
        if (dim == 2 && q != 2) continue;
        dd_add(s, shI[w][q] + st * shm[w]);
      }
      I6[q] = s.hi + s.lo;
    }
    B.m = m;
    for (int a = 0; a < 3; ++a) B.r[a] = r[a];
    double Iw[9] = {I6[0], I6[3], I6[4], I6[3], I6[1], I6[5], I6[4], I6[5], I6[2]};
    if (dim == 2) {
      for (int q = 0; q < 9; ++q) B.Ib[q] = 0.0;
      B.Ib[8] = I6[2];
    } else {
      double Rm[9];
      quat_to_rot(B.q, Rm);
      rot_sandwich(Rm, Iw, 1, B.Ib);
    }
    B.active = ns > 0 ? 1 : 0;
    for (int a = 0; a < 3; ++a) gr[a] = r[a];
  }
  __syncthreads();
  double Rm[9];
  quat_to_rot(B.q, Rm);
  for (int q = threadIdx.x; q < ns; q += blockDim.x) {
    const V4<double> x = s_x[s0 + q];
    double d[3] = {x.x - gr[0], x.y - gr[1], dim == 3 ? x.z - gr[2] : 0.0};
    double rb[3];
    matT_vec(Rm, d, rb);
    if (dim == 2) rb[2] = 0.0;
    V4<double> o;
    o.x = d[0]; o.y = d[1]; o.z = d[2]; o.w = 0.0;
    s_rk[s0 + q] = o;
    o.x = rb[0]; o.y = rb[1]; o.z = rb[2];
    s_rb[s0 + q] = o;
  }
  }
}

// acceleration of rigid particles as material points (used at set-up)
__global__ void __launch_bounds__(256) k_rigid_aw(const Body* bodies, const int32_t* s_body, const V4<double>* s_rk,
                                                  V4<double>* s_aw, int64_t nr) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nr) return;
  const Body& B = bodies[s_body[s]];
  const V4<double> r = s_rk[s];
  const double rk[3] = {r.x, r.y, r.z};
  double t1[3], t2[3], t3[3];
  cross3(B.al, rk, t1);
  cross3(B.w, rk, t2);
  cross3(B.w, t2, t3);
  V4<double> o;
  o.x = B.a[0] + t1[0] + t3[0];
  o.y = B.a[1] + t1[1] + t3[1];
  o.z = B.a[2] + t1[2] + t3[2];
  o.w = 0.0;
  s_aw[s] = o;
}

// ---------------------------------------------------------------------------
// global FP64 checks: mass, momentum, kinetic energy of fluid particles
// ---------------------------------------------------------------------------

// fluid mass, momentum, kinetic energy and potential energy of the body
// force, -m b.x
template <typename R>
__global__ void __launch_bounds__(256) k_global_partials(View<R> v, Params P, double* part) {
  DD acc[6];
  for (int q = 0; q < 6; ++q) acc[q].hi = acc[q].lo = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P.n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t inf = v.info[i];
    if (ikind(inf) != KF) continue;
    const double m = (double)v.m[i];
    const V4<R> u = v.u[i];
    const double ux = u.x, uy = u.y, uz = u.z;
    double x[3];
    get_pos<R>(P, v, i, x);
    const MatT<R>& M = v.mat[iphase(inf)];
    const double bx = (double)M.b[0] * x[0] + (double)M.b[1] * x[1] + (P.dim == 3 ? (double)M.b[2] * x[2] : 0.0);
    dd_add(acc[0], m);
    dd_add(acc[1], m * ux);
    dd_add(acc[2], m * uy);
    dd_add(acc[3], m * uz);
    dd_add(acc[4], 0.5 * m * (ux * ux + uy * uy + uz * uz));
    dd_add(acc[5], -(m * bx));
  }
  double out[6];
  block_reduce_dd<6>(acc, out);
  if (threadIdx.x == 0)
    for (int q = 0; q < 6; ++q) part[6 * blockIdx.x + q] = out[q];
}

__global__ void __launch_bounds__(256) k_global_final(const double* part, int nb, double* out) {
  DD acc[6];
  for (int q = 0; q < 6; ++q) acc[q].hi = acc[q].lo = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x)
    for (int q = 0; q < 6; ++q) dd_add(acc[q], part[6 * b + q]);
  double o[6];
  block_reduce_dd<6>(acc, o);
  if (threadIdx.x == 0)
    for (int q = 0; q < 6; ++q) out[q] = o[q];
}

// ---------------------------------------------------------------------------
// single-workgroup forms of the scan and the wave table for small arrays:
// one launch instead of three
// ---------------------------------------------------------------------------

constexpr int64_t kSmallScan = 16384;     // scans: one workgroup up to here
constexpr int64_t kSmallRows = 65536;     // wave table: one workgroup up to here

// exclusive scan over the 1024 threads of the workgroup
__device__ __forceinline__ uint32_t block1024_exclusive_scan(uint32_t x, uint32_t* total) {
  __shared__ uint32_t wsum[16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t inc = x;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(inc, off, 64);
    if (lane >= off) inc += y;
  }
  if (lane == 63) wsum[wid] = inc;
  __syncthreads();
  uint32_t base = 0u, tot = 0u;
  for (int w = 0; w < 16; ++w) {
    const uint32_t v = wsum[w];
    if (w < wid) base += v;
    tot += v;
  }
  __syncthreads();
  *total = tot;
  return base + inc - x;
}

// out[i] = sum of in[0..i), out[n] = total; in is cleared when asked (the
// cell counts, ready for the next step).  Tiles of 4096 entries, each
// thread four consecutive ones, a running carry between tiles.
__global__ void __launch_bounds__(1024) k_scan_small(uint32_t* in, uint32_t* out, int64_t n, int clear,
                                                     const uint32_t* gate) {
  if (gate && gate[0] == 0u) return;
  uint32_t carry = 0u;
  for (int64_t base = 0; base < n; base += 4096) {
    const int64_t a = base + 4 * (int64_t)threadIdx.x;
    uint32_t v[4], sum = 0u;
    for (int q = 0; q < 4; ++q) {
      v[q] = a + q < n ? in[a + q] : 0u;
      sum += v[q];
    }
    uint32_t tot;
    uint32_t run = carry + block1024_exclusive_scan(sum, &tot);
    for (int q = 0; q < 4; ++q)
      if (a + q < n) {
        out[a + q] = run;
        run += v[q];
        if (clear) in[a + q] = 0u;
      }
    carry += tot;
  }
  if (threadIdx.x == 0) out[n] = carry;
}

// waves of every x-row of cells (64 particles at most, one row each) and
// the wave table; woff[nrows] receives the wave count.  Every workgroup
// scans the rows' wave counts (one workgroup's work), then writes the
// table entries of its share of the rows, so that the scattered table
// stores are spread over kWaveTableBlocks CUs
constexpr int kWaveTableBlocks = 16;
__global__ void __launch_bounds__(1024) k_wave_table_small(const uint32_t* cstart, int nx, int64_t nrows,
                                                           uint32_t* woff, WaveInfo* table) {
  const int64_t chunk = (nrows + 1023) / 1024;
  const int64_t a = (int64_t)threadIdx.x * chunk;
  const int64_t b = a + chunk < nrows ? a + chunk : nrows;
  uint32_t sum = 0u;
  for (int64_t r = a; r < b; ++r) sum += (cstart[(r + 1) * nx] - cstart[r * nx] + 63u) >> 6;
  uint32_t tot;
  uint32_t w0 = block1024_exclusive_scan(sum, &tot);
  // this workgroup's threads: [t0, t1)
  const int t0 = (int)(blockIdx.x * 1024u / gridDim.x), t1 = (int)((blockIdx.x + 1u) * 1024u / gridDim.x);
  if ((int)threadIdx.x < t0 || (int)threadIdx.x >= t1) return;
  for (int64_t r = a; r < b; ++r) {
    const uint32_t s0 = cstart[r * nx];
    const uint32_t n = cstart[(r + 1) * nx] - s0;
    woff[r] = w0;
    for (uint32_t q = 0; q * 64u < n; ++q) {
      WaveInfo wi;
      wi.p0 = s0 + 64u * q;
      wi.cnt = n - 64u * q < 64u ? n - 64u * q : 64u;
      wi.row = (uint32_t)r;
      wi.pad = 0u;
      table[w0 + q] = wi;
    }
    w0 += (n + 63u) >> 6;
  }
  if (threadIdx.x == 0) woff[nrows] = tot;   // only in workgroup 0 (t0 = 0)
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------

static inline unsigned nblk(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

void launch_fill_u32(uint32_t* p, uint32_t val, int64_t n, hipStream_t st) {
  if (n > 0) k_fill_u32<<<nblk(n), 256, 0, st>>>(p, val, n);
}

void launch_step_begin(unsigned long long* pairs, unsigned long long* dstep, hipStream_t st) {
  k_step_begin<<<1, 64, 0, st>>>(pairs, dstep);
}
void launch_zero_pairs(unsigned long long* pairs, bool eval, bool total, hipStream_t st) {
  k_zero_pairs<<<1, 256, 0, st>>>(pairs, eval ? 1 : 0, total ? 1 : 0);
}

void launch_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* bsum, hipStream_t st,
                     const uint32_t* gate) {
  if (n <= kSmallScan) {
    k_scan_small<<<1, 1024, 0, st>>>(const_cast<uint32_t*>(in), out, n, 0, gate);
    return;
  }
  const int64_t nb = (n + 1023) / 1024;
  if (nb > 0) k_scan_blocks<<<(unsigned)nb, 256, 0, st>>>(in, out, bsum, n, gate);
  k_scan_bsum<<<1, 256, 0, st>>>(bsum, nb, out + n, gate);
  if (nb > 0) k_scan_add<<<(unsigned)nb, 256, 0, st>>>(out, bsum, n, gate);
}

void launch_wave_table(const Params& P, const uint32_t* cstart, uint32_t* wcount, uint32_t* woff, uint32_t* bsum,
                       WaveInfo* table, hipStream_t st) {
  if (P.nrows <= kSmallRows) {
    k_wave_table_small<<<kWaveTableBlocks, 1024, 0, st>>>(cstart, P.nc[0], P.nrows, woff, table);
    return;
  }
  k_row_waves<<<nblk(P.nrows), 256, 0, st>>>(cstart, P.nc[0], P.nrows, wcount);
  launch_scan_u32(wcount, woff, P.nrows, bsum, st);
  k_row_waves_fill<<<nblk(P.nrows), 256, 0, st>>>(cstart, P.nc[0], P.nrows, woff, table);
}

// the cell counts are zero on entry: cleared at creation and by the
// single-workgroup scan after use (the multi-workgroup path clears them here)
void launch_sort_keys(const Params& P, SortBufs sb, uint32_t* cstart, const uint32_t* id, hipStream_t st) {
  const int64_t C = P.ncells, n = P.n;
  const bool small = C <= kSmallScan;
  if (!small) launch_fill_u32(sb.ccount, 0u, C, st);
  if (n > 0) k_count<<<nblk(n), 256, 0, st>>>(sb.key, sb.ccount, sb.rank, n);
  if (small) k_scan_small<<<1, 1024, 0, st>>>(sb.ccount, cstart, C, 1, nullptr);
  else launch_scan_u32(sb.ccount, cstart, C, sb.bsum, st);
  if (n > 0) {
    k_scatter<<<nblk(n), 256, 0, st>>>(sb.key, sb.rank, cstart, id, sb.tid, sb.tsrc, n);
  }
}

// body kernels loop over the bodies: up to 1024 workgroups
static inline unsigned body_grid(const Params& P) { return (unsigned)std::min(P.body_launch, 1024); }

void launch_body_kick_drift(Body* b, const Params& P, const uint32_t* nbd, hipStream_t st) {
  if (P.body_launch > 0)
    k_body_kick_drift<<<nblk(P.body_launch, 64), 64, 0, st>>>(b, P.body_launch, nbd, P.dt, P.hdt);
}

void launch_body_reduce(Body* b, const V4<double>* s_f, const V4<double>* s_rk, const Params& P, int kick,
                        const uint32_t* nbd, hipStream_t st) {
  if (P.body_launch > 0)
    k_body_reduce<<<body_grid(P), 256, 0, st>>>(b, s_f, s_rk, P.dim, P.hdt, kick, P.body_launch, nbd);
}

void launch_mass_props_impl(Body* b, const V4<double>* s_x, const double* s_m, V4<double>* s_rb, V4<double>* s_rk,
                            const Params& P, const uint32_t* only, const uint32_t* nbd, hipStream_t st) {
  if (P.body_launch > 0)
    k_mass_props<<<body_grid(P), 256, 0, st>>>(b, s_x, s_m, s_rb, s_rk, P.dim, P.Ir_fac, only, P.body_launch, nbd,
                                              nullptr);
}

void launch_rigid_aw(Body* b, const Params& P, const int32_t* s_body, const V4<double>* s_rk, V4<double>* s_aw,
                     hipStream_t st) {
  if (P.n_rigid > 0) k_rigid_aw<<<nblk(P.n_rigid), 256, 0, st>>>(b, s_body, s_rk, s_aw, P.n_rigid);
}

template <typename R>
void Launch<R>::kick_drift(const View<R>& v, const Params& P, const KC<R>& k, SortBufs sb, hipStream_t st) {
  if (P.n > 0) k_kick_drift<R><<<nblk(P.n), 256, 0, st>>>(v, P, k, sb.key);
  else launch_step_begin(v.pairs, v.dstep, st);
}
template <typename R>
void Launch<R>::rigid_pose(const View<R>& v, const Params& P, const KC<R>&, SortBufs sb, double, hipStream_t st) {
  if (P.slot_cap > 0) k_rigid_pose<R><<<nblk(P.slot_cap), 256, 0, st>>>(v, P, sb.key);
}
template <typename R>
void Launch<R>::wall_motion(const View<R>& v, const Params& P, const KC<R>&, SortBufs sb, double, hipStream_t st) {
  if (P.n_moving > 0) k_wall_motion<R><<<nblk(P.n_moving), 256, 0, st>>>(v, P, sb.key);
}
template <typename R>
void Launch<R>::gather(const View<R>& src, const View<R>& dst, const Params& P, SortBufs sb, hipStream_t st) {
  if (P.n <= 0) return;
  k_rank<<<nblk(P.n), 256, 0, st>>>(sb.key, src.cstart, sb.tid, sb.tsrc, sb.perm, src.err, P.n);
  k_gather<R><<<nblk(P.n), 256, 0, st>>>(src, dst, P, sb.perm, sb.key);
}
template <typename R>
void Launch<R>::density(const View<R>& v, const Params& P, const KC<R>& k, hipStream_t st) {
  if (P.n <= 0) return;
  const unsigned g = (unsigned)P.max_waves;
  if (P.dim == 2) k_build_density<R, 2><<<g, 64, 0, st>>>(v, P, k);
  else k_build_density<R, 3><<<g, 64, 0, st>>>(v, P, k);
}
template <typename R>
void Launch<R>::extrapolate(const View<R>& v, const Params& P, const KC<R>& k, hipStream_t st) {
  if (P.n <= 0) return;
  const unsigned g = nblk(P.ext_cap, 64 / ExtSub<R>::v);
  if (g == 0) return;
  if (P.dim == 2) k_extrapolate_list<R, 2><<<g, 64, 0, st>>>(v, P, k);
  else k_extrapolate_list<R, 3><<<g, 64, 0, st>>>(v, P, k);
}
// unused dynamic LDS that holds the FP32 force sweep's workgroups of kFwpb
// waves at 4 per CU (16 waves, 4 per SIMD): the gathers share the L1, and
// more waves only evict each other's lines (per SIMD, one wave per
// workgroup: 0.653 ms at 8, 0.641 at 3.5, 0.682 at 2.25; four per workgroup:
// 0.631 at 5, 0.628 at 4); FP64 is held at 4 by its registers
template <typename R>
constexpr size_t forces_multi_lds() { return IsExact<R>::v ? 0 : 39000; }

template <typename R>
void Launch<R>::forces(const View<R>& v, const Params& P, const KC<R>& k, int kick, int heat, hipStream_t st) {
  if (P.n <= 0) return;
  const unsigned g = (unsigned)((P.max_waves + kFwpb - 1) / kFwpb);
  const int mode = (P.thermal ? 1 : 0) | (P.tvf ? 2 : 0);
  switch (mode | (P.dim == 3 ? 4 : 0)) {
    case 0: k_forces_list<R, 2, 0, 0><<<g, 64 * kFwpb, forces_multi_lds<R>(), st>>>(v, P, k, kick, heat); break;
    case 1: k_forces_list<R, 2, 1, 0><<<g, 64 * kFwpb, forces_multi_lds<R>(), st>>>(v, P, k, kick, heat); break;
    case 2: k_forces_list<R, 2, 0, 1><<<g, 64 * kFwpb, forces_multi_lds<R>(), st>>>(v, P, k, kick, heat); break;
    case 3: k_forces_list<R, 2, 1, 1><<<g, 64 * kFwpb, forces_multi_lds<R>(), st>>>(v, P, k, kick, heat); break;
    case 4: k_forces_list<R, 3, 0, 0><<<g, 64 * kFwpb, forces_multi_lds<R>(), st>>>(v, P, k, kick, heat); break;
    case 5: k_forces_list<R, 3, 1, 0><<<g, 64 * kFwpb, forces_multi_lds<R>(), st>>>(v, P, k, kick, heat); break;
    case 6: k_forces_list<R, 3, 0, 1><<<g, 64 * kFwpb, forces_multi_lds<R>(), st>>>(v, P, k, kick, heat); break;
    default: k_forces_list<R, 3, 1, 1><<<g, 64 * kFwpb, forces_multi_lds<R>(), st>>>(v, P, k, kick, heat); break;
  }
}
template <typename R>
void Launch<R>::batch_sweep(int stage, const Slot<R>* tab, const char* gbase, int ns, int dim, int mode,
                            uint32_t blocks, int kick, int heat, hipStream_t st) {
  if (ns <= 0 || blocks == 0) return;
  if (stage == 0) {
    if (dim == 2) k_build_density_batch<R, 2><<<blocks, 64, 0, st>>>(tab, gbase, ns);
    else k_build_density_batch<R, 3><<<blocks, 64, 0, st>>>(tab, gbase, ns);
  } else if (stage == 1) {
    if (dim == 2) k_extrapolate_batch<R, 2><<<blocks, 64, 0, st>>>(tab, gbase, ns);
    else k_extrapolate_batch<R, 3><<<blocks, 64, 0, st>>>(tab, gbase, ns);
  } else {
    // mode: bit 0 thermal, bit 1 transport-velocity formulation
    switch ((mode & 3) | (dim == 3 ? 4 : 0)) {
      case 0: k_forces_batch<R, 2, 0, 0><<<blocks / kFwpb, 64 * kFwpb, forces_multi_lds<R>(), st>>>(tab, gbase, ns, kick, heat); break;
      case 1: k_forces_batch<R, 2, 1, 0><<<blocks / kFwpb, 64 * kFwpb, forces_multi_lds<R>(), st>>>(tab, gbase, ns, kick, heat); break;
      case 2: k_forces_batch<R, 2, 0, 1><<<blocks / kFwpb, 64 * kFwpb, forces_multi_lds<R>(), st>>>(tab, gbase, ns, kick, heat); break;
      case 3: k_forces_batch<R, 2, 1, 1><<<blocks / kFwpb, 64 * kFwpb, forces_multi_lds<R>(), st>>>(tab, gbase, ns, kick, heat); break;
      case 4: k_forces_batch<R, 3, 0, 0><<<blocks / kFwpb, 64 * kFwpb, forces_multi_lds<R>(), st>>>(tab, gbase, ns, kick, heat); break;
      case 5: k_forces_batch<R, 3, 1, 0><<<blocks / kFwpb, 64 * kFwpb, forces_multi_lds<R>(), st>>>(tab, gbase, ns, kick, heat); break;
      case 6: k_forces_batch<R, 3, 0, 1><<<blocks / kFwpb, 64 * kFwpb, forces_multi_lds<R>(), st>>>(tab, gbase, ns, kick, heat); break;
      default: k_forces_batch<R, 3, 1, 1><<<blocks / kFwpb, 64 * kFwpb, forces_multi_lds<R>(), st>>>(tab, gbase, ns, kick, heat); break;
    }
  }
}
template <typename R>
void Launch<R>::rigid_velocity(const View<R>& v, const Params& P, hipStream_t st) {
  if (P.slot_cap > 0) k_rigid_velocity<R><<<nblk(P.slot_cap), 256, 0, st>>>(v, P, nullptr);
}
template <typename R>
void Launch<R>::global_sums(const View<R>& v, const Params& P, double* partials, int nblocks, double* out,
                            hipStream_t st) {
  k_global_partials<R><<<(unsigned)nblocks, 256, 0, st>>>(v, P, partials);
  k_global_final<<<1, 256, 0, st>>>(partials, nblocks, out);
}
template <typename R>
void Launch<R>::nb_count(const View<R>& v, const Params& P, const KC<R>&, uint32_t* cnt, hipStream_t st) {
  if (P.n <= 0) return;
  if (P.dim == 2) k_list_count<R, 2><<<(unsigned)P.max_waves, 64, 0, st>>>(v, P, cnt);
  else k_list_count<R, 3><<<(unsigned)P.max_waves, 64, 0, st>>>(v, P, cnt);
}
template <typename R>
void Launch<R>::nb_fill(const View<R>& v, const Params& P, const KC<R>&, const uint64_t* off, uint32_t* ids,
                        hipStream_t st) {
  if (P.n <= 0) return;
  if (P.dim == 2) k_list_fill<R, 2><<<(unsigned)P.max_waves, 64, 0, st>>>(v, P, off, ids);
  else k_list_fill<R, 3><<<(unsigned)P.max_waves, 64, 0, st>>>(v, P, off, ids);
}
template <typename R>
void Launch<R>::slot_positions(const View<R>& v, const Params& P, hipStream_t st) {
  if (P.slot_cap > 0) k_slot_positions<R><<<nblk(P.slot_cap), 256, 0, st>>>(v, P, nullptr);
}

// ---------------------------------------------------------------------------
// reversible phase transition (Sec. "Modeling thermally driven reversible
// phase transitions")
//
// Enqueued after every step when enabled.  Apart from the flag pass, every
// kernel returns at once unless some particle crossed its transition
// temperature, so a step without a switch costs one pass over the
// particles.  Readings: strict comparisons, phases without a partner never
// switch; melting first, then every solidifying particle joins the body of
// its nearest rigid neighbour within r_c (ties: lower body id, then lower
// original id); the remaining solidifying particles form one new body per
// connected component (pairs closer than r_c), numbered in ascending order
// of the component's smallest original id; bodies that changed get new mass
// quantities and offsets, and their velocity follows rigid body motion with
// unchanged angular velocity.  Rigid slots stay ordered by (body, original
// id): the surviving slots keep that order, the joining particles are
// sorted by the same key and the two sequences are merged.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void wave_count(uint32_t* ctr, bool pred) {
  const unsigned long long m = __ballot(pred);
  if ((threadIdx.x & 63) == 0 && m) atomicAdd(ctr, (uint32_t)__popcll(m));
}

__device__ __forceinline__ unsigned long long slot_key(int body, uint32_t id) {
  return ((unsigned long long)(uint32_t)body << 32) | (unsigned long long)id;
}

// first index in [0, n) whose key is not below x
__device__ __forceinline__ uint32_t lower_bound_u64(const unsigned long long* a, uint32_t n, unsigned long long x) {
  uint32_t lo = 0u, hi = n;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1u;
    else hi = mid;
  }
  return lo;
}

// the wave holding sorted particle i (waves are in ascending p0 order)
template <typename R>
__device__ __forceinline__ uint32_t wave_of(const View<R>& v, uint32_t i) {
  uint32_t lo = 0u, hi = *v.nb.nwaves;
  while (hi - lo > 1u) {
    const uint32_t mid = (lo + hi) >> 1;
    if (v.nb.table[mid].p0 <= i) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <typename R>
__global__ void __launch_bounds__(64) k_ps_begin(View<R> v) {
  if (threadIdx.x < 8) v.ps.ctr[threadIdx.x] = threadIdx.x == 3 ? v.dyn[0] : 0u;
}

template <typename R>
__global__ void __launch_bounds__(256) k_ps_flags(View<R> v, Params P) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool any = false;
  if (i < P.n) {
    const uint32_t inf = v.info[i];
    const uint32_t kind = ikind(inf);
    const MatT<R>& M = v.mat[iphase(inf)];
    uint8_t f = 0;
    if (M.switch_to >= 0) {
      const R T = v.T[i];
      if (kind == KR && T > M.T_t) f = 1;
      else if (kind == KF && T < M.T_t) f = 2;
    }
    v.ps.flag[i] = f;
    any = f != 0;
  }
  wave_count(&v.ps.ctr[0], any);
  const uint8_t fl = i < P.n ? v.ps.flag[i] : (uint8_t)0;
  wave_count(&v.dyn[2], fl == 1);     // melted, cumulative
  wave_count(&v.dyn[3], fl == 2);     // solidifying, cumulative
}

// melting: the particle keeps the velocity and the acceleration of its
// material point, a_k + alpha_k x r_rk + omega_k x (omega_k x r_rk)
template <typename R>
__global__ void __launch_bounds__(256) k_ps_melt(View<R> v, Params P) {
  if (v.ps.ctr[0] == 0u) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P.n || v.ps.flag[i] != 1) return;
  const uint32_t inf = v.info[i];
  const int32_t s = v.aux[i];
  const int kb = v.s_body[s];
  const Body& B = v.bodies[kb];
  const V4<double> r4 = v.s_rk[s];
  const double rk[3] = {r4.x, r4.y, r4.z};
  double t1[3], t2[3], t3[3];
  cross3(B.al, rk, t1);
  cross3(B.w, rk, t2);
  cross3(B.w, t2, t3);
  V4<R> a;
  a.x = (R)(B.a[0] + t1[0] + t3[0]);
  a.y = (R)(B.a[1] + t1[1] + t3[1]);
  a.z = P.dim == 3 ? (R)(B.a[2] + t1[2] + t3[2]) : R(0);
  a.w = R(0);
  v.a[i] = a;
  v.info[i] = mkinfo(KF, (uint32_t)v.mat[iphase(inf)].switch_to, 0u, -1);
  v.aux[i] = -1;
  v.ps.dirty[kb] = 1u;
}

// nearest rigid neighbour of every solidifying particle, from its list;
// particles without one are queued for the component search
template <typename R, int DIM>
__global__ void __launch_bounds__(64) k_ps_nearest(View<R> v, Params P, KC<R> k) {
  constexpr int CAP = Nb<DIM>::cap, NR = Nb<DIM>::rows;
  if (v.ps.ctr[0] == 0u) return;
  const int w = blockIdx.x;
  if (w >= (int)*v.nb.nwaves) return;
  const WaveInfo wi = v.nb.table[w];
  const int lane = threadIdx.x;
  if (lane >= (int)wi.cnt) return;
  const uint32_t i = wi.p0 + (uint32_t)lane;
  if (v.ps.flag[i] != 2) return;
  const WaveGeo g = wave_geo<R>(v, P, wi);
  const V4<R> T = to_frame<R>(v.pos[i], k, g.cx_first, 0, 0);
  const uint16_t* gl = v.nb.ent + (size_t)w * CAP * 64 + lane;
  bool found = false;
  R br2 = R(0);
  int bb = 0;
  uint32_t bid = 0u;
  const int c = v.nb.cnt[(size_t)w * 64 + lane];   // a fluid lane: not split
  for (int t = 0; t < c; ++t) {
    const uint32_t e = gl[(size_t)t * 64];
    const int rr = (int)(e >> 12);
    const int dz = DIM == 3 ? rr / 3 - 1 : 0, dy = rr % 3 - 1;
    const uint32_t j = v.nb.jlo[(size_t)w * NR + rr] + (e & 0xfffu);
    if (j == i) continue;
    const uint32_t ij = v.info[j];
    if (ikind(ij) != KR) continue;
    R d0, d1, d2;
    const R r2 = dist2<R, DIM>(T, to_frame<R>(v.pos[j], k, g.cx_first, dy, dz), d0, d1, d2);
    const int bj = ibody(ij);
    const uint32_t idj = v.id[j];
    if (!found || r2 < br2 || (r2 == br2 && (bj < bb || (bj == bb && idj < bid)))) {
      found = true;
      br2 = r2;
      bb = bj;
      bid = idj;
    }
  }
  if (found) {
    v.ps.target[i] = bb;
  } else {
    v.ps.target[i] = -1;
    v.ps.label[i] = v.id[i];
    v.ps.list[atomicAdd(&v.ps.ctr[1], 1u)] = i;
  }
}

// Connected components of the queued particles and their new bodies, in one
// workgroup: every particle's label (an original id) drops to the smallest
// label among its queued neighbours until no label changes, which leaves
// the smallest original id of the component.
template <typename R, int DIM>
__global__ void __launch_bounds__(256) k_ps_components(View<R> v, Params P, const double* matb) {
  constexpr int CAP = Nb<DIM>::cap, NR = Nb<DIM>::rows;
  const uint32_t nu = v.ps.ctr[1];
  if (nu == 0u) return;
  __shared__ uint32_t nroot, changed;
  if (threadIdx.x == 0) nroot = 0u;
  for (;;) {
    if (threadIdx.x == 0) changed = 0u;
    __syncthreads();
    for (uint32_t q = threadIdx.x; q < nu; q += blockDim.x) {
      const uint32_t i = v.ps.list[q];
      const uint32_t w = wave_of<R>(v, i);
      const int lane = (int)(i - v.nb.table[w].p0);
      const uint16_t* gl = v.nb.ent + (size_t)w * CAP * 64 + lane;
      uint32_t m = v.ps.label[i];
      const int c = v.nb.cnt[(size_t)w * 64 + lane];   // a fluid lane: not split
      for (int t = 0; t < c; ++t) {
        const uint32_t e = gl[(size_t)t * 64];
        const uint32_t j = v.nb.jlo[(size_t)w * NR + (e >> 12)] + (e & 0xfffu);
        if (j == i || v.ps.flag[j] != 2 || v.ps.target[j] >= 0) continue;
        const uint32_t lj = v.ps.label[j];
        if (lj < m) m = lj;
      }
      if (m < v.ps.label[i]) {
        v.ps.label[i] = m;
        changed = 1u;
      }
    }
    __syncthreads();
    const uint32_t c = changed;
    __syncthreads();
    if (c == 0u) break;
  }
  // roots, numbered by ascending original id after the existing bodies
  for (uint32_t q = threadIdx.x; q < nu; q += blockDim.x) {
    const uint32_t i = v.ps.list[q];
    if (v.ps.label[i] == v.id[i]) v.ps.roots[atomicAdd(&nroot, 1u)] = i;
  }
  __syncthreads();
  const uint32_t nr = nroot;
  const uint32_t nb0 = v.dyn[1];
  for (uint32_t q = threadIdx.x; q < nr; q += blockDim.x) {
    const uint32_t i = v.ps.roots[q];
    const uint32_t my = v.id[i];
    uint32_t rank = 0u;
    for (uint32_t o = 0; o < nr; ++o) rank += v.id[v.ps.roots[o]] < my ? 1u : 0u;
    const uint32_t kb = nb0 + rank;
    if (kb >= (uint32_t)P.maxb) {
      set_err(v.err, ERR_BODYCAP);
      v.ps.body_of_id[my] = 0xffffffffu;
      continue;
    }
    v.ps.body_of_id[my] = kb;
    Body& B = v.bodies[kb];
    B.q[0] = 1.0; B.q[1] = 0.0; B.q[2] = 0.0; B.q[3] = 0.0;
    const int ps = v.mat[iphase(v.info[i])].switch_to;
    for (int a = 0; a < 3; ++a) {
      B.w[a] = 0.0;
      B.al[a] = 0.0;
      B.f[a] = 0.0;
      B.t[a] = 0.0;
      B.b[a] = a < P.dim ? matb[3 * ps + a] : 0.0;
    }
    B.fixed = 0;
    B.active = 1;
    v.ps.dirty[kb] = 2u;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t nbn = nb0 + nr;
    v.dyn[1] = nbn < (uint32_t)P.maxb ? nbn : (uint32_t)P.maxb;
  }
  for (uint32_t q = threadIdx.x; q < nu; q += blockDim.x) {
    const uint32_t i = v.ps.list[q];
    const uint32_t kb = v.ps.body_of_id[v.ps.label[i]];
    v.ps.target[i] = kb == 0xffffffffu ? -1 : (int32_t)kb;
  }
}

// solidification: kind, phase and body; the joining particles are queued
// with their slot key
template <typename R>
__global__ void __launch_bounds__(256) k_ps_apply(View<R> v, Params P) {
  if (v.ps.ctr[0] == 0u) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P.n || v.ps.flag[i] != 2) return;
  const int32_t t = v.ps.target[i];
  if (t < 0) return;
  const uint32_t inf = v.info[i];
  v.info[i] = mkinfo(KR, (uint32_t)v.mat[iphase(inf)].switch_to, 0u, t);
  if (v.ps.dirty[t] == 0u) v.ps.dirty[t] = 1u;
  const uint32_t q = atomicAdd(&v.ps.ctr[2], 1u);
  v.ps.jkey[0][q] = slot_key(t, v.id[i]);
  v.ps.jidx[0][q] = (uint32_t)i;
}

// old slots that stay rigid
template <typename R>
__global__ void __launch_bounds__(256) k_ps_alive(View<R> v, Params P) {
  if (v.ps.ctr[0] == 0u) return;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= P.slot_cap) return;
  const uint32_t nold = v.ps.ctr[3];
  v.ps.alive[s] = (s < (int64_t)nold && ikind(v.info[v.s_sorted[s]]) == KR) ? 1u : 0u;
}

// bottom-up merge sort of the joiner keys in one workgroup (keys are
// unique); the result ends in buffer ctr[6]
__global__ void __launch_bounds__(256) k_ps_sort_joiners(PhaseBufs ps) {
  const uint32_t nj = ps.ctr[2];
  if (ps.ctr[0] == 0u || nj == 0u) return;
  int cur = 0;
  for (uint32_t w = 1u; w < nj; w <<= 1) {
    const unsigned long long* ka = ps.jkey[cur];
    const uint32_t* ia = ps.jidx[cur];
    unsigned long long* kb = ps.jkey[1 - cur];
    uint32_t* ib = ps.jidx[1 - cur];
    for (uint32_t e = threadIdx.x; e < nj; e += blockDim.x) {
      const uint32_t start = e / (2u * w) * (2u * w);
      const uint32_t mid = start + w < nj ? start + w : nj;
      const uint32_t end = start + 2u * w < nj ? start + 2u * w : nj;
      const unsigned long long key = ka[e];
      uint32_t pos;
      if (e < mid) pos = (e - start) + lower_bound_u64(ka + mid, end - mid, key);
      else pos = (e - mid) + lower_bound_u64(ka + start, mid - start, key);
      kb[start + pos] = key;
      ib[start + pos] = ia[e];
    }
    __syncthreads();
    cur = 1 - cur;
  }
  if (threadIdx.x == 0) ps.ctr[6] = (uint32_t)cur;
}

// merge of the surviving slots (already in key order) with the sorted
// joiners into the new slot order
template <typename R>
__global__ void __launch_bounds__(256) k_ps_place(View<R> v, Params P) {
  if (v.ps.ctr[0] == 0u) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t nold = v.ps.ctr[3], nj = v.ps.ctr[2];
  const unsigned long long* jk = v.ps.jkey[v.ps.ctr[6]];
  const uint32_t* ji = v.ps.jidx[v.ps.ctr[6]];
  if (t < (int64_t)nold && v.ps.alive[t]) {
    const unsigned long long key = slot_key(v.s_body[t], v.s_id[t]);
    const uint32_t pos = v.ps.alive_sc[t] + lower_bound_u64(jk, nj, key);
    v.ps.snew[pos] = (uint32_t)v.s_sorted[t];
    v.ps.sbody[pos] = v.s_body[t];
    v.ps.sid[pos] = v.s_id[t];
    v.ps.srb[pos] = v.s_rb[t];
    v.ps.srk[pos] = v.s_rk[t];
    v.ps.srf[pos] = v.s_f[t];
  }
  if (t < (int64_t)nj) {
    const unsigned long long key = jk[t];
    // old slots below the key (dead ones included), then the live ones among them
    uint32_t lo = 0u, hi = nold;
    while (lo < hi) {
      const uint32_t mid = (lo + hi) >> 1;
      if (slot_key(v.s_body[mid], v.s_id[mid]) < key) lo = mid + 1u;
      else hi = mid;
    }
    const uint32_t pos = (uint32_t)t + v.ps.alive_sc[lo];
    V4<double> z;
    z.x = z.y = z.z = z.w = 0.0;
    v.ps.snew[pos] = ji[t];
    v.ps.sbody[pos] = (int32_t)(key >> 32);
    v.ps.sid[pos] = (uint32_t)(key & 0xffffffffull);
    v.ps.srb[pos] = z;
    v.ps.srk[pos] = z;
    v.ps.srf[pos] = z;
  }
}

// every body's old centre of mass; slot ranges cleared
template <typename R>
__global__ void __launch_bounds__(256) k_ps_bodies(View<R> v, Params P) {
  if (v.ps.ctr[0] == 0u) return;
  const uint32_t nb = v.dyn[1];
  for (uint32_t kb = blockIdx.x * blockDim.x + threadIdx.x; kb < nb; kb += gridDim.x * blockDim.x) {
    Body& B = v.bodies[kb];
    V4<double> r;
    r.x = B.r[0]; r.y = B.r[1]; r.z = B.r[2]; r.w = 0.0;
    v.ps.rold[kb] = r;
    B.nslot = 0;
  }
}

// new slot arrays, body slot ranges (first slot), rigid count
template <typename R>
__global__ void __launch_bounds__(256) k_ps_slots(View<R> v, Params P) {
  if (v.ps.ctr[0] == 0u) return;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t total = v.ps.alive_sc[v.ps.ctr[3]] + v.ps.ctr[2];
  if (s == 0) v.dyn[0] = total;
  if (s >= (int64_t)total) return;
  const uint32_t i = v.ps.snew[s];
  const int kb = v.ps.sbody[s];
  v.s_sorted[s] = (int32_t)i;
  v.s_body[s] = kb;
  v.s_id[s] = v.ps.sid[s];
  v.s_rb[s] = v.ps.srb[s];
  v.s_rk[s] = v.ps.srk[s];
  v.s_f[s] = v.ps.srf[s];
  v.aux[i] = (int32_t)s;
  if (s == 0 || v.ps.sbody[s - 1] != kb) v.bodies[kb].slot0 = (int32_t)s;
}

// body slot ranges (count), after the first slots are known
template <typename R>
__global__ void __launch_bounds__(256) k_ps_slot_ends(View<R> v, Params P) {
  if (v.ps.ctr[0] == 0u) return;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t total = v.dyn[0];
  if (s >= (int64_t)total) return;
  const int kb = v.ps.sbody[s];
  if (s + 1 == (int64_t)total || v.ps.sbody[s + 1] != kb) v.bodies[kb].nslot = (int32_t)(s + 1) - v.bodies[kb].slot0;
}

// after the new mass quantities: velocity of changed bodies follows rigid
// motion, u_k += omega_k x (r_k - r_k,old); new bodies take the
// mass-weighted velocity and acceleration of their particles
template <typename R>
__global__ void __launch_bounds__(256) k_ps_fix(View<R> v, Params P) {
  if (v.ps.ctr[0] == 0u) return;
  const uint32_t nb = v.dyn[1];
  for (uint32_t kb = blockIdx.x; kb < nb; kb += gridDim.x) {
    const uint32_t d = v.ps.dirty[kb];
    Body& B = v.bodies[kb];
    const int act = B.active;
    __syncthreads();
    if (d == 0u) continue;
    if (threadIdx.x == 0) v.ps.dirty[kb] = 0u;
    if (!act) continue;
    if (d == 1u) {
      if (threadIdx.x == 0) {
        const V4<double> ro = v.ps.rold[kb];
        const double dr[3] = {B.r[0] - ro.x, B.r[1] - ro.y, B.r[2] - ro.z};
        double wr[3];
        cross3(B.w, dr, wr);
        for (int a = 0; a < P.dim; ++a) B.u[a] = B.u[a] + wr[a];
      }
      continue;
    }
    DD acc[7];
    for (int q = 0; q < 7; ++q) acc[q].hi = acc[q].lo = 0.0;
    for (int q = threadIdx.x; q < B.nslot; q += blockDim.x) {
      const int64_t i = v.s_sorted[B.slot0 + q];
      const double m = (double)v.m[i];
      const V4<R> u = v.u[i];
      const V4<R> a = v.a[i];
      dd_add(acc[0], m);
      dd_add(acc[1], m * (double)u.x);
      dd_add(acc[2], m * (double)u.y);
      dd_add(acc[3], m * (double)u.z);
      dd_add(acc[4], m * (double)a.x);
      dd_add(acc[5], m * (double)a.y);
      dd_add(acc[6], m * (double)a.z);
    }
    double o[7];
    block_reduce_dd<7>(acc, o);
    if (threadIdx.x == 0) {
      for (int a = 0; a < 3; ++a) {
        B.u[a] = a < P.dim ? o[1 + a] / o[0] : 0.0;
        B.a[a] = a < P.dim ? o[4 + a] / o[0] : 0.0;
      }
    }
  }
}

template <typename R>
void Launch<R>::phase_switch(const View<R>& v, const Params& P, const KC<R>& k, const double* matb, hipStream_t st) {
  if (P.n <= 0 || !P.pswitch) return;
  const unsigned gn = nblk(P.n), gs = nblk(P.slot_cap);
  const unsigned gb = (unsigned)std::min(std::max(P.maxb, 1), 1024);
  k_ps_begin<R><<<1, 64, 0, st>>>(v);
  k_ps_flags<R><<<gn, 256, 0, st>>>(v, P);
  k_ps_melt<R><<<gn, 256, 0, st>>>(v, P);
  if (P.dim == 2) {
    k_ps_nearest<R, 2><<<(unsigned)P.max_waves, 64, 0, st>>>(v, P, k);
    k_ps_components<R, 2><<<1, 256, 0, st>>>(v, P, matb);
  } else {
    k_ps_nearest<R, 3><<<(unsigned)P.max_waves, 64, 0, st>>>(v, P, k);
    k_ps_components<R, 3><<<1, 256, 0, st>>>(v, P, matb);
  }
  k_ps_apply<R><<<gn, 256, 0, st>>>(v, P);
  k_ps_alive<R><<<gs, 256, 0, st>>>(v, P);
  launch_scan_u32(v.ps.alive, v.ps.alive_sc, P.slot_cap, v.ps.bsum, st, v.ps.ctr);
  k_ps_sort_joiners<<<1, 256, 0, st>>>(v.ps);
  k_ps_place<R><<<gs, 256, 0, st>>>(v, P);
  k_ps_bodies<R><<<nblk(P.maxb), 256, 0, st>>>(v, P);
  k_ps_slots<R><<<gs, 256, 0, st>>>(v, P);
  k_ps_slot_ends<R><<<gs, 256, 0, st>>>(v, P);
  k_slot_positions<R><<<gs, 256, 0, st>>>(v, P, v.ps.ctr);
  k_mass_props<<<gb, 256, 0, st>>>(v.bodies, v.s_x, v.s_m, v.s_rb, v.s_rk, P.dim, P.Ir_fac, v.ps.dirty, P.maxb,
                                   v.dyn + 1, v.ps.ctr);
  k_ps_fix<R><<<gb, 256, 0, st>>>(v, P);
  k_rigid_velocity<R><<<gs, 256, 0, st>>>(v, P, v.ps.ctr);
}

template struct Launch<float>;
template struct Launch<double>;

}  // namespace sphrb
