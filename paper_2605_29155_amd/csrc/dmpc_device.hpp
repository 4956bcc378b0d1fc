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
constexpr int GS = 56;      // gains per stage: K column-major [13][4], then k[4]
constexpr int FS = 17 * 16; // linearisation per stage: 17 columns of 13 floats, stride 16
constexpr int TS = FS + 52 + 16; // tail per stage: F, K [13][4], M (4x4 masked inverse)
constexpr int SW = 8;       // per-instance state words

// per-instance state words
constexpr int S_NOM = 0, S_ITERS = 1, S_STATUS = 2, S_DONE = 3, S_T = 4;

constexpr uint32_t ST_CONVERGED = 0x1u, ST_MAXITER = 0x2u, ST_NONFINITE = 0x4u, ST_FP64 = 0x8u,
                   ST_QPMAXITER = 0x10u, ST_REGULARIZED = 0x20u;

struct Dyn {
  float h, h2, h6, g, inv_m, arm_a, kappa, iJx, iJy, iJz, cx, cy, cz, hover;
};

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

// lane holding column j of F (j >= 1)
__host__ __device__ constexpr int lane_of(int j) { return j == 16 ? 0 : j; }

// ---------------------------------------------------------------------------
// quadrotor dynamics, its tangent, RK4
// ---------------------------------------------------------------------------

__device__ __forceinline__ void forces(const Dyn& P, const float* u, float& s, float& tx, float& ty, float& tz) {
  s = (u[0] + u[1] + u[2] + u[3]) * P.inv_m;
  tx = P.arm_a * (u[0] + u[1] - u[2] - u[3]) * P.iJx;
  ty = P.arm_a * (-u[0] + u[1] + u[2] - u[3]) * P.iJy;
  tz = P.kappa * (u[0] - u[1] + u[2] - u[3]) * P.iJz;
}

// xdot = F(x, u) with the input entering through (s, tx, ty, tz)
__device__ __forceinline__ void rhs(const Dyn& P, const float* x, float s, float tx, float ty, float tz, float* o) {
  const float qw = x[3], qx = x[4], qy = x[5], qz = x[6], wx = x[10], wy = x[11], wz = x[12];
  o[0] = x[7];
  o[1] = x[8];
  o[2] = x[9];
  o[3] = 0.5f * (-qx * wx - qy * wy - qz * wz);
  o[4] = 0.5f * (qw * wx + qy * wz - qz * wy);
  o[5] = 0.5f * (qw * wy - qx * wz + qz * wx);
  o[6] = 0.5f * (qw * wz + qx * wy - qy * wx);
  o[7] = s * (2.f * (qx * qz + qw * qy));
  o[8] = s * (2.f * (qy * qz - qw * qx));
  o[9] = s * (1.f - 2.f * (qx * qx + qy * qy)) - P.g;
  o[10] = tx - P.cx * wy * wz;
  o[11] = ty - P.cy * wz * wx;
  o[12] = tz - P.cz * wx * wy;
}

// directional derivative of F at (x, u) along (d, du), du entering as (ds, dtx, dty, dtz)
__device__ __forceinline__ void rhs_tan(const Dyn& P, const float* x, const float* d, float s, float ds, float dtx,
                                        float dty, float dtz, float* o) {
  const float qw = x[3], qx = x[4], qy = x[5], qz = x[6], wx = x[10], wy = x[11], wz = x[12];
  const float dqw = d[3], dqx = d[4], dqy = d[5], dqz = d[6], dwx = d[10], dwy = d[11], dwz = d[12];
  o[0] = d[7];
  o[1] = d[8];
  o[2] = d[9];
  o[3] = 0.5f * (-(dqx * wx + qx * dwx) - (dqy * wy + qy * dwy) - (dqz * wz + qz * dwz));
  o[4] = 0.5f * ((dqw * wx + qw * dwx) + (dqy * wz + qy * dwz) - (dqz * wy + qz * dwy));
  o[5] = 0.5f * ((dqw * wy + qw * dwy) - (dqx * wz + qx * dwz) + (dqz * wx + qz * dwx));
  o[6] = 0.5f * ((dqw * wz + qw * dwz) + (dqx * wy + qx * dwy) - (dqy * wx + qy * dwx));
  const float b0 = 2.f * (qx * qz + qw * qy), b1 = 2.f * (qy * qz - qw * qx), b2 = 1.f - 2.f * (qx * qx + qy * qy);
  const float db0 = 2.f * (dqx * qz + qx * dqz + dqw * qy + qw * dqy);
  const float db1 = 2.f * (dqy * qz + qy * dqz - dqw * qx - qw * dqx);
  const float db2 = -4.f * (qx * dqx + qy * dqy);
  o[7] = ds * b0 + s * db0;
  o[8] = ds * b1 + s * db1;
  o[9] = ds * b2 + s * db2;
  o[10] = dtx - P.cx * (dwy * wz + wy * dwz);
  o[11] = dty - P.cy * (dwz * wx + wz * dwx);
  o[12] = dtz - P.cz * (dwx * wy + wx * dwy);
}

// one RK4 step x -> xn with the thrust held over the step
__device__ __forceinline__ void rk4(const Dyn& P, const float* x, const float* u, float* xn) {
  float s, tx, ty, tz, k[NX], acc[NX], xs[NX];
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
    acc[i] += 2.f * k[i];
    xs[i] = x[i] + P.h2 * k[i];
  }
  rhs(P, xs, s, tx, ty, tz, k);
#pragma unroll
  for (int i = 0; i < NX; ++i) {
    acc[i] += 2.f * k[i];
    xs[i] = x[i] + P.h * k[i];
  }
  rhs(P, xs, s, tx, ty, tz, k);
#pragma unroll
  for (int i = 0; i < NX; ++i) xn[i] = x[i] + P.h6 * (acc[i] + k[i]);
}

// tangent direction owned by a lane: e_col for state columns, e_{col-13} for inputs
struct LaneDir {
  float dx[NX];
  float ds, dtx, dty, dtz;
};

__device__ __forceinline__ LaneDir make_dir(const Dyn& P, int col) {
  LaneDir d;
#pragma unroll
  for (int i = 0; i < NX; ++i) d.dx[i] = (i == col) ? 1.f : 0.f;
  const int a = col - NX;
  const bool isu = col >= NX;
  const float mx = (a == 0 || a == 1) ? 1.f : -1.f;
  const float my = (a == 1 || a == 2) ? 1.f : -1.f;
  const float mz = (a == 0 || a == 2) ? 1.f : -1.f;
  d.ds = isu ? P.inv_m : 0.f;
  d.dtx = isu ? P.arm_a * mx * P.iJx : 0.f;
  d.dty = isu ? P.arm_a * my * P.iJy : 0.f;
  d.dtz = isu ? P.kappa * mz * P.iJz : 0.f;
  return d;
}

// column of [A | B] = d f(x, u) / d(direction), by forward-mode differentiation
// of the RK4 step (exact derivative of the discrete map)
__device__ __forceinline__ void rk4_column(const Dyn& P, const float* x, const float* u, const LaneDir& D,
                                           float* col) {
  float s, tx, ty, tz, k[NX], dk[NX], acc[NX], dacc[NX], xs[NX], dxs[NX];
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
    acc[i] += 2.f * k[i];
    dacc[i] += 2.f * dk[i];
    xs[i] = x[i] + P.h2 * k[i];
    dxs[i] = D.dx[i] + P.h2 * dk[i];
  }
  rhs(P, xs, s, tx, ty, tz, k);
  rhs_tan(P, xs, dxs, s, D.ds, D.dtx, D.dty, D.dtz, dk);
#pragma unroll
  for (int i = 0; i < NX; ++i) {
    acc[i] += 2.f * k[i];
    dacc[i] += 2.f * dk[i];
    xs[i] = x[i] + P.h * k[i];
    dxs[i] = D.dx[i] + P.h * dk[i];
  }
  rhs_tan(P, xs, dxs, s, D.ds, D.dtx, D.dty, D.dtz, dk);
#pragma unroll
  for (int i = 0; i < NX; ++i) col[i] = D.dx[i] + P.h6 * (dacc[i] + dk[i]);
  (void)acc;
}

// ---------------------------------------------------------------------------
// 4x4 Cholesky of the free block (clamped rows/cols replaced by identity),
// FP32 with an FP64 redo when a pivot falls below the threshold
// ---------------------------------------------------------------------------

struct Chol4 {
  float L[10];   // L00 L10 L11 L20 L21 L22 L30 L31 L32 L33
  float iD[4];   // 1 / L_ii
  double Ld[10];
  double iDd[4];
  bool f64;
};

template <typename R>
__device__ __forceinline__ bool chol4_core(const R* h, R* L, R* iD, R& dmin) {
  R d0 = h[0];
  R l00 = sqrt(d0 > R(0) ? d0 : R(0));
  R i0 = R(1) / l00;
  R l10 = h[4] * i0, l20 = h[8] * i0, l30 = h[12] * i0;
  R d1 = h[5] - l10 * l10;
  R l11 = sqrt(d1 > R(0) ? d1 : R(0));
  R i1 = R(1) / l11;
  R l21 = (h[9] - l20 * l10) * i1, l31 = (h[13] - l30 * l10) * i1;
  R d2 = h[10] - l20 * l20 - l21 * l21;
  R l22 = sqrt(d2 > R(0) ? d2 : R(0));
  R i2 = R(1) / l22;
  R l32 = (h[14] - l30 * l20 - l31 * l21) * i2;
  R d3 = h[15] - l30 * l30 - l31 * l31 - l32 * l32;
  R l33 = sqrt(d3 > R(0) ? d3 : R(0));
  R i3 = R(1) / l33;
  L[0] = l00; L[1] = l10; L[2] = l11; L[3] = l20; L[4] = l21;
  L[5] = l22; L[6] = l30; L[7] = l31; L[8] = l32; L[9] = l33;
  iD[0] = i0; iD[1] = i1; iD[2] = i2; iD[3] = i3;
  R m01 = d0 < d1 ? d0 : d1, m23 = d2 < d3 ? d2 : d3;
  dmin = m01 < m23 ? m01 : m23;
  return dmin > R(0);
}

// H is the full symmetric 4x4 (row-major); fr[a] = 1 free, 0 clamped
__device__ __forceinline__ void chol4(const float* H, const float* fr, float piv, Chol4& C, uint32_t& st) {
  float h[16];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
      h[a * 4 + b] = (a == b) ? (fr[a] != 0.f ? H[a * 4 + a] : 1.f) : fr[a] * fr[b] * H[a * 4 + b];
  float dmin;
  const bool ok = chol4_core<float>(h, C.L, C.iD, dmin);
  C.f64 = false;
  if (piv > 0.f ? !(dmin >= piv) : !ok) {
    // pivot below threshold (or non-positive with the fallback disabled):
    // refactor in FP64; a pivot that is still not positive gets a shift
    double hd[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) hd[i] = (double)h[i];
    double dm;
    bool ok2 = chol4_core<double>(hd, C.Ld, C.iDd, dm);
    if (piv > 0.f) st |= ST_FP64;
    if (!ok2) {
      double mx = 1.0;
#pragma unroll
      for (int a = 0; a < 4; ++a) mx = hd[a * 5] > mx ? hd[a * 5] : mx;
      double shift = 1e-6 * mx;
      for (int tries = 0; tries < 8 && !ok2; ++tries) {
#pragma unroll
        for (int a = 0; a < 4; ++a) hd[a * 5] = (double)h[a * 5] + shift;
        ok2 = chol4_core<double>(hd, C.Ld, C.iDd, dm);
        shift *= 10.0;
      }
      st |= ST_REGULARIZED;
    }
    C.f64 = true;
  }
}

template <typename R>
__device__ __forceinline__ void solve4_core(const R* L, const R* iD, R* r) {
  R z0 = r[0] * iD[0];
  R z1 = (r[1] - L[1] * z0) * iD[1];
  R z2 = (r[2] - L[3] * z0 - L[4] * z1) * iD[2];
  R z3 = (r[3] - L[6] * z0 - L[7] * z1 - L[8] * z2) * iD[3];
  R y3 = z3 * iD[3];
  R y2 = (z2 - L[8] * y3) * iD[2];
  R y1 = (z1 - L[4] * y2 - L[7] * y3) * iD[1];
  R y0 = (z0 - L[1] * y1 - L[3] * y2 - L[6] * y3) * iD[0];
  r[0] = y0; r[1] = y1; r[2] = y2; r[3] = y3;
}

// r <- Htilde^{-1} r
__device__ __forceinline__ void solve4(const Chol4& C, float* r) {
  if (C.f64) {
    double rd[4] = {(double)r[0], (double)r[1], (double)r[2], (double)r[3]};
    solve4_core<double>(C.Ld, C.iDd, rd);
#pragma unroll
    for (int a = 0; a < 4; ++a) r[a] = (float)rd[a];
  } else {
    solve4_core<float>(C.L, C.iD, r);
  }
}

__device__ __forceinline__ float clampf(float v, float lo, float hi) { return v < lo ? lo : (v > hi ? hi : v); }

__device__ __forceinline__ float qp_val(const float* H, const float* q, const float* x) {
  float f = 0.f;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    float s = 0.f;
#pragma unroll
    for (int b = 0; b < 4; ++b) s += H[a * 4 + b] * x[b];
    f += x[a] * (0.5f * s + q[a]);
  }
  return f;
}

// Stagewise box-QP min 1/2 d^T H d + q^T d, lo <= d <= hi, by projected Newton
// (Tassa, Mansard & Todorov 2014): clamped set = coordinates on a bound whose
// gradient points outward (strict), Newton step on the free block, projected
// Armijo search.  On return x is the step, fr the free mask (1/0) and C the
// factor of the free block for that mask.
__device__ __forceinline__ void boxqp(const float* H, const float* q, const float* lo, const float* hi,
                                      const float* xw, float piv, float* x, float* fr, Chol4& C, uint32_t& st) {
  float qn = 0.f;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    x[a] = clampf(xw[a], lo[a], hi[a]);
    qn = fmaxf(qn, fabsf(q[a]));
  }
  const float tolg = 1e-6f * (1.f + qn);
  bool current = false;
  bool converged = false;
  for (int it = 0; it < 16; ++it) {
    float g[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      float s = q[a];
#pragma unroll
      for (int b = 0; b < 4; ++b) s += H[a * 4 + b] * x[b];
      g[a] = s;
    }
    float gn = 0.f;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const bool cl = (x[a] <= lo[a] && g[a] > 0.f) || (x[a] >= hi[a] && g[a] < 0.f);
      fr[a] = cl ? 0.f : 1.f;
      gn = fmaxf(gn, fr[a] * fabsf(g[a]));
    }
    chol4(H, fr, piv, C, st);
    current = true;
    if (gn <= tolg) {
      converged = true;
      break;
    }
    float d[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) d[a] = -fr[a] * g[a];
    solve4(C, d);
    const float fx = qp_val(H, q, x);
    float step = 1.f, xn[4];
    bool acc = false;
    for (int ls = 0; ls < 12; ++ls) {
      float dec = 0.f;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        xn[a] = clampf(x[a] + step * d[a], lo[a], hi[a]);
        dec += g[a] * (xn[a] - x[a]);
      }
      const float fn = qp_val(H, q, xn);
      if (fn - fx <= 0.1f * dec) {
        acc = true;
        break;
      }
      step *= 0.5f;
    }
    if (!acc) break;
    bool moved = false;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      moved |= (xn[a] != x[a]);
      x[a] = xn[a];
    }
    current = false;
    if (!moved) break;
  }
  if (!converged) {
    // final clamped set and factor at the returned point
    float g[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      float s = q[a];
#pragma unroll
      for (int b = 0; b < 4; ++b) s += H[a * 4 + b] * x[b];
      g[a] = s;
    }
    float gn = 0.f;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const bool cl = (x[a] <= lo[a] && g[a] > 0.f) || (x[a] >= hi[a] && g[a] < 0.f);
      fr[a] = cl ? 0.f : 1.f;
      gn = fmaxf(gn, fr[a] * fabsf(g[a]));
    }
    if (!current) chol4(H, fr, piv, C, st);
    if (!(gn <= 1e-4f * (1.f + qn))) st |= ST_QPMAXITER;
  }
}

}  // namespace dmpc_dev
