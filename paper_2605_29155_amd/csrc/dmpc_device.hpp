// dmpc_device.hpp -- device routines of the batched differentiable MPC layer
// for gfx950 (CDNA4, wave64).
//
// Mapping: one problem instance per 16-lane DPP row; a wave64 carries four
// instances.  Within a row, lane l owns column col(l) of F_t = [A_t | B_t]
// (col(0) = 16, i.e. B's last column; col(l) = l otherwise) and row l of the
// value matrix V (l < 13).  Column 0 of A_t (the p_x direction) is the unit
// vector e_0 for this model (nothing depends on position), so it is handled
// implicitly and 17 columns fit in 16 lanes.  Matrix operands move between
// lanes with DPP row broadcasts (row_newbcast), reductions with DPP quad and
// mirror permutes; there is no LDS traffic in the stage algebra.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dmpc_dev {

constexpr int NX = 13, NU = 4, NZ = 17, NPK = 153;
constexpr int ZS = 20;      // floats per stage in a trajectory slot: x at 0..12, u at 16..19
constexpr int NSLOT = 5;    // nominal + four line-search candidates
constexpr int GS = 68;      // gains per stage: K row-major [4][16] (13 used per row), then k[4] at 64
constexpr int FS = 17 * 16; // linearisation per stage: 17 columns of 13 floats, stride 16
constexpr int TS = FS + 52 + 32; // tail per stage: F, K [13][4], M (4x4 masked inverse, FP64)
constexpr int SW = 8;       // per-instance state words

// per-instance state words
constexpr int S_NOM = 0, S_ITERS = 1, S_STATUS = 2, S_DONE = 3, S_T = 4;
constexpr int S_FB = 5;  // time-parallel Riccati: a stage's clamp pattern differed from the assumed one

constexpr uint32_t ST_CONVERGED = 0x1u, ST_MAXITER = 0x2u, ST_NONFINITE = 0x4u, ST_FP64 = 0x8u,
                   ST_QPMAXITER = 0x10u, ST_REGULARIZED = 0x20u, ST_REDONE = 0x40u;

// model constants in the precision R of the dynamics (float, or double in the
// FP64 form)
template <class R>
struct DynT {
  R h, h2, h6, g, inv_m, arm_a, kappa, iJx, iJy, iJz, cx, cy, cz, hover;
};
using Dyn = DynT<float>;
using Dyn64 = DynT<double>;

// ---------------------------------------------------------------------------
// lane helpers (16-lane DPP rows)
// ---------------------------------------------------------------------------

// broadcast lane L of this 16-lane row to the whole row (L must fold to a
// constant after unrolling)
__device__ __forceinline__ float rb(float v, int L) {
  const int x = __float_as_int(v);
  int r;
  switch (L) {
    case 0: r = __builtin_amdgcn_mov_dpp(x, 0x150, 0xF, 0xF, false); break;
    case 1: r = __builtin_amdgcn_mov_dpp(x, 0x151, 0xF, 0xF, false); break;
    case 2: r = __builtin_amdgcn_mov_dpp(x, 0x152, 0xF, 0xF, false); break;
    case 3: r = __builtin_amdgcn_mov_dpp(x, 0x153, 0xF, 0xF, false); break;
    case 4: r = __builtin_amdgcn_mov_dpp(x, 0x154, 0xF, 0xF, false); break;
    case 5: r = __builtin_amdgcn_mov_dpp(x, 0x155, 0xF, 0xF, false); break;
    case 6: r = __builtin_amdgcn_mov_dpp(x, 0x156, 0xF, 0xF, false); break;
    case 7: r = __builtin_amdgcn_mov_dpp(x, 0x157, 0xF, 0xF, false); break;
    case 8: r = __builtin_amdgcn_mov_dpp(x, 0x158, 0xF, 0xF, false); break;
    case 9: r = __builtin_amdgcn_mov_dpp(x, 0x159, 0xF, 0xF, false); break;
    case 10: r = __builtin_amdgcn_mov_dpp(x, 0x15A, 0xF, 0xF, false); break;
    case 11: r = __builtin_amdgcn_mov_dpp(x, 0x15B, 0xF, 0xF, false); break;
    case 12: r = __builtin_amdgcn_mov_dpp(x, 0x15C, 0xF, 0xF, false); break;
    case 13: r = __builtin_amdgcn_mov_dpp(x, 0x15D, 0xF, 0xF, false); break;
    case 14: r = __builtin_amdgcn_mov_dpp(x, 0x15E, 0xF, 0xF, false); break;
    default: r = __builtin_amdgcn_mov_dpp(x, 0x15F, 0xF, 0xF, false); break;
  }
  return __int_as_float(r);
}

// 64-bit row broadcast as two 32-bit DPP moves
__device__ __forceinline__ double rb64(double v, int L) {
  const long long x = __double_as_longlong(v);
  const float lo = __int_as_float((int)(x & 0xffffffffLL));
  const float hi = __int_as_float((int)(x >> 32));
  const unsigned long long r =
      ((unsigned long long)(unsigned)__float_as_int(rb(hi, L)) << 32) | (unsigned)__float_as_int(rb(lo, L));
  return __longlong_as_double((long long)r);
}

// broadcast lane Q of each 4-lane quad to the quad (Q constant after unrolling)
__device__ __forceinline__ float qb(float v, int Q) {
  const int x = __float_as_int(v);
  int r;
  switch (Q) {
    case 0: r = __builtin_amdgcn_mov_dpp(x, 0x00, 0xF, 0xF, false); break;
    case 1: r = __builtin_amdgcn_mov_dpp(x, 0x55, 0xF, 0xF, false); break;
    case 2: r = __builtin_amdgcn_mov_dpp(x, 0xAA, 0xF, 0xF, false); break;
    default: r = __builtin_amdgcn_mov_dpp(x, 0xFF, 0xF, 0xF, false); break;
  }
  return __int_as_float(r);
}
// sum / max over a 4-lane quad, identical in all four lanes
__device__ __forceinline__ float quad_sum(float v) {
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, false));
  return v;
}
__device__ __forceinline__ float quad_max(float v) {
  v = fmaxf(v, __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false)));
  v = fmaxf(v, __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, false)));
  return v;
}

// 64-bit versions (two 32-bit DPP moves each)
__device__ __forceinline__ double qb(double v, int Q) {
  const long long x = __double_as_longlong(v);
  const int lo = __float_as_int(qb(__int_as_float((int)x), Q));
  const int hi = __float_as_int(qb(__int_as_float((int)(x >> 32)), Q));
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ double dpp_b1(double v) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(x >> 32), 0xB1, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ double dpp_4e(double v) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)x, 0x4E, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(x >> 32), 0x4E, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ double quad_max(double v) {
  v = fmax(v, dpp_b1(v));
  v = fmax(v, dpp_4e(v));
  return v;
}

// lane holding column j of F (j >= 1)
__host__ __device__ constexpr int lane_of(int j) { return j == 16 ? 0 : j; }

// ---------------------------------------------------------------------------
// quadrotor dynamics, its tangent, RK4
// ---------------------------------------------------------------------------

template <class R>
__device__ __forceinline__ void forces(const DynT<R>& P, const R* u, R& s, R& tx, R& ty, R& tz) {
  s = (u[0] + u[1] + u[2] + u[3]) * P.inv_m;
  tx = P.arm_a * (u[0] + u[1] - u[2] - u[3]) * P.iJx;
  ty = P.arm_a * (-u[0] + u[1] + u[2] - u[3]) * P.iJy;
  tz = P.kappa * (u[0] - u[1] + u[2] - u[3]) * P.iJz;
}

// xdot = F(x, u) with the input entering through (s, tx, ty, tz)
template <class R>
__device__ __forceinline__ void rhs(const DynT<R>& P, const R* x, R s, R tx, R ty, R tz, R* o) {
  const R qw = x[3], qx = x[4], qy = x[5], qz = x[6], wx = x[10], wy = x[11], wz = x[12];
  o[0] = x[7];
  o[1] = x[8];
  o[2] = x[9];
  o[3] = R(0.5) * (-qx * wx - qy * wy - qz * wz);
  o[4] = R(0.5) * (qw * wx + qy * wz - qz * wy);
  o[5] = R(0.5) * (qw * wy - qx * wz + qz * wx);
  o[6] = R(0.5) * (qw * wz + qx * wy - qy * wx);
  o[7] = s * (R(2) * (qx * qz + qw * qy));
  o[8] = s * (R(2) * (qy * qz - qw * qx));
  o[9] = s * (R(1) - R(2) * (qx * qx + qy * qy)) - P.g;
  o[10] = tx - P.cx * wy * wz;
  o[11] = ty - P.cy * wz * wx;
  o[12] = tz - P.cz * wx * wy;
}

// directional derivative of F at (x, u) along (d, du), du entering as (ds, dtx, dty, dtz)
template <class R>
__device__ __forceinline__ void rhs_tan(const DynT<R>& P, const R* x, const R* d, R s, R ds, R dtx, R dty, R dtz,
                                        R* o) {
  const R qw = x[3], qx = x[4], qy = x[5], qz = x[6], wx = x[10], wy = x[11], wz = x[12];
  const R dqw = d[3], dqx = d[4], dqy = d[5], dqz = d[6], dwx = d[10], dwy = d[11], dwz = d[12];
  o[0] = d[7];
  o[1] = d[8];
  o[2] = d[9];
  o[3] = R(0.5) * (-(dqx * wx + qx * dwx) - (dqy * wy + qy * dwy) - (dqz * wz + qz * dwz));
  o[4] = R(0.5) * ((dqw * wx + qw * dwx) + (dqy * wz + qy * dwz) - (dqz * wy + qz * dwy));
  o[5] = R(0.5) * ((dqw * wy + qw * dwy) - (dqx * wz + qx * dwz) + (dqz * wx + qz * dwx));
  o[6] = R(0.5) * ((dqw * wz + qw * dwz) + (dqx * wy + qx * dwy) - (dqy * wx + qy * dwx));
  const R b0 = R(2) * (qx * qz + qw * qy), b1 = R(2) * (qy * qz - qw * qx), b2 = R(1) - R(2) * (qx * qx + qy * qy);
  const R db0 = R(2) * (dqx * qz + qx * dqz + dqw * qy + qw * dqy);
  const R db1 = R(2) * (dqy * qz + qy * dqz - dqw * qx - qw * dqx);
  const R db2 = R(-4) * (qx * dqx + qy * dqy);
  o[7] = ds * b0 + s * db0;
  o[8] = ds * b1 + s * db1;
  o[9] = ds * b2 + s * db2;
  o[10] = dtx - P.cx * (dwy * wz + wy * dwz);
  o[11] = dty - P.cy * (dwz * wx + wz * dwx);
  o[12] = dtz - P.cz * (dwx * wy + wx * dwy);
}

// one RK4 step x -> xn with the thrust held over the step
template <class R>
__device__ __forceinline__ void rk4(const DynT<R>& P, const R* x, const R* u, R* xn) {
  R s, tx, ty, tz, k[NX], acc[NX], xs[NX];
  forces(P, u, s, tx, ty, tz);
  rhs(P, x, s, tx, ty, tz, k);
#pragma unroll
  for (int i = 0; i < NX; ++i) {
    acc[i] = k[i];
    xs[i] = x[i] + P.h2 * k[i];
  }
  rhs(P, xs, s, tx, ty, tz, k);
#pragma unroll
  for (int i = 0; i < NX; ++i) {
    acc[i] += R(2) * k[i];
    xs[i] = x[i] + P.h2 * k[i];
  }
  rhs(P, xs, s, tx, ty, tz, k);
#pragma unroll
  for (int i = 0; i < NX; ++i) {
    acc[i] += R(2) * k[i];
    xs[i] = x[i] + P.h * k[i];
  }
  rhs(P, xs, s, tx, ty, tz, k);
#pragma unroll
  for (int i = 0; i < NX; ++i) xn[i] = x[i] + P.h6 * (acc[i] + k[i]);
}

// tangent direction owned by a lane: e_col for state columns, e_{col-13} for inputs
template <class R>
struct LaneDir {
  R dx[NX];
  R ds, dtx, dty, dtz;
};

template <class R>
__device__ __forceinline__ LaneDir<R> make_dir(const DynT<R>& P, int col) {
  LaneDir<R> d;
#pragma unroll
  for (int i = 0; i < NX; ++i) d.dx[i] = (i == col) ? R(1) : R(0);
  const int a = col - NX;
  const bool isu = col >= NX;
  const R mx = (a == 0 || a == 1) ? R(1) : -R(1);
  const R my = (a == 1 || a == 2) ? R(1) : -R(1);
  const R mz = (a == 0 || a == 2) ? R(1) : -R(1);
  d.ds = isu ? P.inv_m : R(0);
  d.dtx = isu ? P.arm_a * mx * P.iJx : R(0);
  d.dty = isu ? P.arm_a * my * P.iJy : R(0);
  d.dtz = isu ? P.kappa * mz * P.iJz : R(0);
  return d;
}

// column of [A | B] = d f(x, u) / d(direction), by forward-mode differentiation
// of the RK4 step (exact derivative of the discrete map)
template <class R>
__device__ __forceinline__ void rk4_column(const DynT<R>& P, const R* x, const R* u, const LaneDir<R>& D, R* col) {
  R s, tx, ty, tz, k[NX], dk[NX], acc[NX], dacc[NX], xs[NX], dxs[NX];
  forces(P, u, s, tx, ty, tz);
  rhs(P, x, s, tx, ty, tz, k);
  rhs_tan(P, x, D.dx, s, D.ds, D.dtx, D.dty, D.dtz, dk);
#pragma unroll
  for (int i = 0; i < NX; ++i) {
    acc[i] = k[i];
    dacc[i] = dk[i];
    xs[i] = x[i] + P.h2 * k[i];
    dxs[i] = D.dx[i] + P.h2 * dk[i];
  }
  rhs(P, xs, s, tx, ty, tz, k);
  rhs_tan(P, xs, dxs, s, D.ds, D.dtx, D.dty, D.dtz, dk);
#pragma unroll
  for (int i = 0; i < NX; ++i) {
    acc[i] += R(2) * k[i];
    dacc[i] += R(2) * dk[i];
    xs[i] = x[i] + P.h2 * k[i];
    dxs[i] = D.dx[i] + P.h2 * dk[i];
  }
  rhs(P, xs, s, tx, ty, tz, k);
  rhs_tan(P, xs, dxs, s, D.ds, D.dtx, D.dty, D.dtz, dk);
#pragma unroll
  for (int i = 0; i < NX; ++i) {
    acc[i] += R(2) * k[i];
    dacc[i] += R(2) * dk[i];
    xs[i] = x[i] + P.h * k[i];
    dxs[i] = D.dx[i] + P.h * dk[i];
  }
  rhs_tan(P, xs, dxs, s, D.ds, D.dtx, D.dty, D.dtz, dk);
#pragma unroll
  for (int i = 0; i < NX; ++i) col[i] = D.dx[i] + P.h6 * (dacc[i] + dk[i]);
  (void)acc;
}

// ---------------------------------------------------------------------------
// 4x4 control block: LDL^T factorisation of the free block (clamped rows/cols
// replaced by identity) and the stagewise box-QP, in FP64.  The control block of the stage
// Hessian is ill-conditioned for these costs (collective thrust has curvature
// ~R = 1e-2 next to torque curvature ~1e3 in rotor coordinates), so it is
// accumulated and solved in double precision.
// ---------------------------------------------------------------------------

// H~ = L D L^T with L unit lower triangular
struct Fact4 {
  double L[10];  // D0 L10 D1 L20 L21 D2 L30 L31 L32 D3 (packed lower triangle, the pivots on the diagonal)
  double iD[4];  // 1 / D_i
};

// 1/d from the hardware estimate (relative error ~5e-8 on gfx950) plus one
// Newton step (each step doubles the correct bits: ~4e-15 after one), instead
// of the IEEE divide sequence
__device__ __forceinline__ double rcp_nr(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  return r;
}

__device__ __forceinline__ bool ldl4_core(const double* h, double* L, double* iD, double& dmin) {
  // LDL^T: u_ij = L_ij D_j are formed first, so each pivot's reciprocal is
  // the only long-latency step on the chain
  const double d0 = h[0];
  const double i0 = rcp_nr(d0 > 0.0 ? d0 : 1e-300);
  const double l10 = h[4] * i0, l20 = h[8] * i0, l30 = h[12] * i0;
  const double d1 = h[5] - l10 * h[4];
  const double i1 = rcp_nr(d1 > 0.0 ? d1 : 1e-300);
  const double u21 = h[9] - l20 * h[4], u31 = h[13] - l30 * h[4];
  const double l21 = u21 * i1, l31 = u31 * i1;
  const double d2 = h[10] - l20 * h[8] - l21 * u21;
  const double i2 = rcp_nr(d2 > 0.0 ? d2 : 1e-300);
  const double u32 = h[14] - l30 * h[8] - l31 * u21;
  const double l32 = u32 * i2;
  const double d3 = h[15] - l30 * h[12] - l31 * u31 - l32 * u32;
  const double i3 = rcp_nr(d3 > 0.0 ? d3 : 1e-300);
  L[0] = d0; L[1] = l10; L[2] = d1; L[3] = l20; L[4] = l21;
  L[5] = d2; L[6] = l30; L[7] = l31; L[8] = l32; L[9] = d3;
  iD[0] = i0; iD[1] = i1; iD[2] = i2; iD[3] = i3;
  const double m01 = d0 < d1 ? d0 : d1, m23 = d2 < d3 ? d2 : d3;
  dmin = m01 < m23 ? m01 : m23;
  return dmin > 0.0;
}

// H full symmetric 4x4 (row-major); fr[a] = 1 free, 0 clamped.  A pivot below
// piv marks the stage ill-conditioned (ST_FP64); a pivot that is not positive
// gets a diagonal shift of 1e-6 max(1, max diag) (x10 until it factors) and
// ST_REGULARIZED.
__device__ __forceinline__ void ldl4(const double* H, const double* fr, float piv, Fact4& C, uint32_t& st) {
  double h[16];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
      h[a * 4 + b] = (a == b) ? (fr[a] != 0.0 ? H[a * 4 + a] : 1.0) : fr[a] * fr[b] * H[a * 4 + b];
  double dmin;
  bool ok = ldl4_core(h, C.L, C.iD, dmin);
  if (piv > 0.f && !(dmin >= (double)piv)) st |= ST_FP64;
  if (!ok) {
    double mx = 1.0;
#pragma unroll
    for (int a = 0; a < 4; ++a) mx = h[a * 5] > mx ? h[a * 5] : mx;
    double shift = 1e-6 * mx;
    for (int tries = 0; tries < 8 && !ok; ++tries) {
      double hs[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) hs[i] = h[i];
#pragma unroll
      for (int a = 0; a < 4; ++a) hs[a * 5] += shift;
      ok = ldl4_core(hs, C.L, C.iD, dmin);
      shift *= 10.0;
    }
    st |= ST_REGULARIZED;
  }
}

// r <- Htilde^{-1} r
__device__ __forceinline__ void solve4(const Fact4& C, double* r) {
  const double* L = C.L;
  const double* iD = C.iD;
  const double w0 = r[0];
  const double w1 = r[1] - L[1] * w0;
  const double w2 = r[2] - L[3] * w0 - L[4] * w1;
  const double w3 = r[3] - L[6] * w0 - L[7] * w1 - L[8] * w2;
  const double y3 = w3 * iD[3];
  const double y2 = w2 * iD[2] - L[8] * y3;
  const double y1 = w1 * iD[1] - L[4] * y2 - L[7] * y3;
  const double y0 = w0 * iD[0] - L[1] * y1 - L[3] * y2 - L[6] * y3;
  r[0] = y0; r[1] = y1; r[2] = y2; r[3] = y3;
}

__device__ __forceinline__ float clampf(float v, float lo, float hi) { return v < lo ? lo : (v > hi ? hi : v); }
__device__ __forceinline__ double clampd(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

__device__ __forceinline__ double qp_val(const double* H, const double* q, const double* x) {
  double f = 0.0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    double s = 0.0;
#pragma unroll
    for (int b = 0; b < 4; ++b) s = fma(H[a * 4 + b], x[b], s);
    f = fma(x[a], fma(0.5, s, q[a]), f);
  }
  return f;
}

__device__ __forceinline__ void qp_grad(const double* H, const double* q, const double* x, double* g) {
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    double s = q[a];
#pragma unroll
    for (int b = 0; b < 4; ++b) s = fma(H[a * 4 + b], x[b], s);
    g[a] = s;
  }
}

__device__ __forceinline__ bool qp_clamped(double x, double g, double lo, double hi) {
  return (x <= lo && g > 0.0) || (x >= hi && g < 0.0);
}

// Stagewise box-QP min 1/2 d^T H d + q^T d, lo <= d <= hi (the bounded
// control update of Tassa, Mansard & Todorov 2014), solved by a primal
// active-set method on the 4-D box: from the warm start, a working set of
// coordinates held on a bound; each iteration takes the Newton step on the free
// face, either stops at the first bound it crosses (that coordinate joins the
// working set) or reaches the face minimiser, where the bound with the most
// wrongly signed multiplier is released; it stops when every multiplier has the
// right sign.  Finite for H > 0.
// On return x is the step, fr the free mask (1/0) and C the factor of the free
// block for that mask.
__device__ __forceinline__ void boxqp(const double* H, const double* q, const double* lo, const double* hi,
                                      const double* xw, float piv, double* x, double* fr, Fact4& C, uint32_t& st) {
  double g[4];
  bool W[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) x[a] = clampd(xw[a], lo[a], hi[a]);
  qp_grad(H, q, x, g);
#pragma unroll
  for (int a = 0; a < 4; ++a) W[a] = (lo[a] >= hi[a]) || qp_clamped(x[a], g[a], lo[a], hi[a]);
  bool done = false;
  for (int it = 0; it < 16 && !done; ++it) {
#pragma unroll
    for (int a = 0; a < 4; ++a) fr[a] = W[a] ? 0.0 : 1.0;
    ldl4(H, fr, piv, C, st);
    double d[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) d[a] = -fr[a] * g[a];
    solve4(C, d);
    // first bound crossed along the step, if any
    double tau = 1.0;
    int blk = -1;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      if (W[a]) continue;
      const double v = x[a] + d[a];
      if (d[a] < 0.0 && v < lo[a]) {
        const double t = (lo[a] - x[a]) * rcp_nr(d[a]);
        if (t < tau) { tau = t; blk = a; }
      } else if (d[a] > 0.0 && v > hi[a]) {
        const double t = (hi[a] - x[a]) * rcp_nr(d[a]);
        if (t < tau) { tau = t; blk = a; }
      }
    }
    if (blk >= 0) {
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        double v = x[a] + tau * d[a];
        if (a == blk) {
          v = d[a] < 0.0 ? lo[a] : hi[a];
          W[a] = true;
        }
        x[a] = clampd(v, lo[a], hi[a]);
      }
      qp_grad(H, q, x, g);
      continue;
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) x[a] += d[a];
    qp_grad(H, q, x, g);
    // face minimiser: release the bound whose multiplier has the most wrong sign
    int worst = -1;
    double wv = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      if (!W[a] || !(lo[a] < hi[a])) continue;
      const double v = (x[a] <= lo[a]) ? -g[a] : g[a];
      if (v > wv) { wv = v; worst = a; }
    }
    if (worst < 0) {
      done = true;
    } else {
#pragma unroll
      for (int a = 0; a < 4; ++a)
        if (a == worst) W[a] = false;
    }
  }
  if (!done) {
#pragma unroll
    for (int a = 0; a < 4; ++a) fr[a] = W[a] ? 0.0 : 1.0;
    ldl4(H, fr, piv, C, st);
#pragma unroll
    for (int a = 0; a < 4; ++a) x[a] = clampd(x[a], lo[a], hi[a]);
    st |= ST_QPMAXITER;
  }
}


// value of v in the lane whose byte address (4 x lane) is addr
__device__ __forceinline__ double lane_read(int addr, double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_ds_bpermute(addr, (int)(unsigned)b);
  const unsigned hi = (unsigned)__builtin_amdgcn_ds_bpermute(addr, (int)(unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// The same stagewise box-QP, solved by the 16 lanes of an instance's row at
// once (every lane holds H, q and the bounds).  Lane j takes the coordinates
// of the set bits of j as free and the others on a bound, solves the face
// problem for the free ones and checks the optimality conditions (free
// coordinates inside the box, clamped ones with correctly signed
// multipliers); the 16 lanes cover every free/clamped split for one choice of
// bound per coordinate.  For H > 0 the minimiser is unique, so the valid
// lanes agree, and the row takes the lowest one's step, free mask, factor and
// flags.  The bound of a coordinate is guessed twice:
//  1. the one the clamped warm start sits on, else the one its gradient there
//     points to (descent lowers it: lower bound, else upper);
//  2. (rows with no valid lane) the one the unconstrained minimiser (lane 15's
//     solution, all free) lies beyond, else the first guess.
// Rows with no valid lane after both run the active-set method (boxqp).  On
// the workloads the first guess covers 95-99% of the stage QPs and the second
// all but 0-0.5%; the active-set iterations it replaces take two or more
// passes in about a third of the stages, and their count differs between the
// four instances of a wave.  row0: the row's first lane in the wave; j: the
// lane's index within the row.  All 16 lanes of the row must be active.
__device__ __forceinline__ void boxqp_row(const double* H, const double* q, const double* lo, const double* hi,
                                          const double* xw, float piv, int row0, int j, double* x, double* fr,
                                          Fact4& C, uint32_t& st) {
  double x0[4], g0[4];
  bool fixed[4], onlo[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) x0[a] = clampd(xw[a], lo[a], hi[a]);
  qp_grad(H, q, x0, g0);
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    fixed[a] = !(lo[a] < hi[a]);
    onlo[a] = x0[a] <= lo[a] ? true : (x0[a] >= hi[a] ? false : g0[a] > 0.0);
  }
  double xl[4];
  Fact4 Cl;
  uint32_t stl;
  // one pass for the bounds onlo: this lane's face solution and its validity
  auto pass = [&]() -> unsigned {
    double xc[4], frl[4], r[4], g[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      frl[a] = (!fixed[a] && ((j >> a) & 1)) ? 1.0 : 0.0;
      xc[a] = fixed[a] ? x0[a] : (onlo[a] ? lo[a] : hi[a]);
    }
    // right-hand side of the free block: -(q_F + H_FC x_C)
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      double s = q[a];
#pragma unroll
      for (int b = 0; b < 4; ++b) s = fma(H[a * 4 + b], (1.0 - frl[b]) * xc[b], s);
      r[a] = -frl[a] * s;
    }
    stl = 0;
    ldl4(H, frl, piv, Cl, stl);
    solve4(Cl, r);
#pragma unroll
    for (int a = 0; a < 4; ++a) xl[a] = frl[a] != 0.0 ? r[a] : xc[a];
    qp_grad(H, q, xl, g);
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      if (fixed[a]) ok = ok && !((j >> a) & 1);  // a fixed coordinate is never free
      else if (frl[a] != 0.0) ok = ok && xl[a] >= lo[a] && xl[a] <= hi[a];
      else ok = ok && (onlo[a] ? g[a] >= 0.0 : g[a] <= 0.0);
    }
    return (unsigned)(__ballot(ok) >> row0) & 0xffffu;
  };
  unsigned rm = pass();
  if (rm == 0u) {
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const double xu = lane_read((row0 + 15) * 4, xl[a]);
      onlo[a] = xu < lo[a] ? true : (xu > hi[a] ? false : onlo[a]);
    }
    rm = pass();
  }
  const int src = rm ? __builtin_ctz(rm) : 0;
  const int addr = (row0 + src) * 4;
#pragma unroll
  for (int a = 0; a < 4; ++a) x[a] = lane_read(addr, xl[a]);
#pragma unroll
  for (int i = 0; i < 10; ++i) C.L[i] = lane_read(addr, Cl.L[i]);
#pragma unroll
  for (int i = 0; i < 4; ++i) C.iD[i] = lane_read(addr, Cl.iD[i]);
  st |= (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)stl);
#pragma unroll
  for (int a = 0; a < 4; ++a) fr[a] = ((src >> a) & 1) ? 1.0 : 0.0;
  if (rm == 0u) boxqp(H, q, lo, hi, xw, piv, x, fr, C, st);
}

}  // namespace dmpc_dev
