// Gradient with respect to the model constants theta = (mass, Jxx, Jyy, Jzz,
// arm, kappa, dt, g), carried along the backward's forward sweep.
//
// The backward differentiates the LQ problem of the model linearised at the
// solution (after Amos et al.): with F_t = df/dz(z*_t) and offset
// f_t = f(z*_t) - F_t z*_t, the gradients with respect to F_t and f_t chained
// to theta give
//   dL/dtheta = sum_t  lt_{t+1}^T df/dtheta(z*_t) + ls_{t+1}^T d(F_t zt_t)/dtheta,
// with zt the adjoint solution (= dL/dc) and lt / ls the costates of the
// adjoint solution and of the solution, both of the form
//   l_t = h_t + A_t^T l_{t+1},  l_T = 0,
//   ht_t = (C_t zt_t + dL/dz*_t)_x,  hs_t = (C_t z*_t + c_t)_x.
// Swapping the order of summation turns each costate sum into a forward
// recursion of a state sensitivity: with xi_{t+1} = A_t xi_t + df/dtheta and
// eta_{t+1} = A_t eta_t + d(F_t zt_t)/dtheta (xi_0 = eta_0 = 0),
//   dL/dtheta = sum_t ht_t^T xi_t + hs_t^T eta_t,
// which needs no backward pass and no storage.  Lane j < 8 of an instance
// owns constant j: it evaluates one RK4 step in a five-part number
//   v + e eps + d del + ed eps del + s sig
// with the state seeded (x*, xt, 0, eta_j, xi_j), the controls (u*, ut, 0, 0,
// 0) and constant j seeded with del = sig = 1.  The sig part of the result is
// xi_{t+1} (first order in sig: A xi + df/dtheta_j) and the eps-del part is
// eta_{t+1} (A eta + d(F zt)/dtheta_j; the state carries no del part, so no
// second derivative in the state enters).  Products of sig with eps or del
// are not tracked.
#pragma once

namespace dmpc_theta {

using dmpc_dev::NU;
using dmpc_dev::NX;

struct N5 {
  float v, e, d, ed, s;
};

__device__ __forceinline__ N5 cst(float v) { return {v, 0.f, 0.f, 0.f, 0.f}; }
__device__ __forceinline__ N5 operator+(const N5& a, const N5& b) {
  return {a.v + b.v, a.e + b.e, a.d + b.d, a.ed + b.ed, a.s + b.s};
}
__device__ __forceinline__ N5 operator-(const N5& a, const N5& b) {
  return {a.v - b.v, a.e - b.e, a.d - b.d, a.ed - b.ed, a.s - b.s};
}
__device__ __forceinline__ N5 operator-(const N5& a) { return {-a.v, -a.e, -a.d, -a.ed, -a.s}; }
__device__ __forceinline__ N5 operator*(float c, const N5& a) { return {c * a.v, c * a.e, c * a.d, c * a.ed, c * a.s}; }
__device__ __forceinline__ N5 operator*(const N5& a, const N5& b) {
  return {a.v * b.v, fmaf(a.v, b.e, a.e * b.v), fmaf(a.v, b.d, a.d * b.v),
          fmaf(a.v, b.ed, fmaf(a.e, b.d, fmaf(a.d, b.e, a.ed * b.v))), fmaf(a.v, b.s, a.s * b.v)};
}
// 1 / a: r - r^2 (e eps + d del + s sig) + (2 r^3 e d - r^2 ed) eps del
__device__ __forceinline__ N5 inv(const N5& a) {
  const float r = 1.f / a.v, r2 = r * r;
  return {r, -a.e * r2, -a.d * r2, r2 * (2.f * r * a.e * a.d - a.ed), -a.s * r2};
}

// model constants as five-part numbers, constant j seeded
struct PN {
  N5 im, a, kappa, iJx, iJy, iJz, cx, cy, cz, h, g;
};

__device__ __forceinline__ PN make_pn(const dmpc_quad_params& q, int j) {
  const float raw[8] = {q.mass, q.Jxx, q.Jyy, q.Jzz, q.arm, q.kappa, q.dt, q.g};
  N5 th[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) th[i] = {raw[i], 0.f, (i == j) ? 1.f : 0.f, 0.f, (i == j) ? 1.f : 0.f};
  PN P;
  P.im = inv(th[0]);
  P.a = 0.70710678118654752f * th[4];
  P.kappa = th[5];
  P.iJx = inv(th[1]);
  P.iJy = inv(th[2]);
  P.iJz = inv(th[3]);
  P.cx = (th[3] - th[2]) * P.iJx;  // (Jzz - Jyy) / Jxx
  P.cy = (th[1] - th[3]) * P.iJy;  // (Jxx - Jzz) / Jyy
  P.cz = (th[2] - th[1]) * P.iJz;  // (Jyy - Jxx) / Jzz
  P.h = th[6];
  P.g = th[7];
  return P;
}

// right-hand side of eq. (1) for the X-configuration quadrotor (rotor i at
// pi/4 + i pi/2, spin signs +,-,+,-; scalar-first quaternion, body rates)
__device__ __forceinline__ void rhs5(const PN& P, const N5* x, const N5& s, const N5& tx, const N5& ty, const N5& tz,
                                     N5* o) {
  const N5 qw = x[3], qx = x[4], qy = x[5], qz = x[6], wx = x[10], wy = x[11], wz = x[12];
  o[0] = x[7];
  o[1] = x[8];
  o[2] = x[9];
  o[3] = 0.5f * (-(qx * wx) - qy * wy - qz * wz);
  o[4] = 0.5f * (qw * wx + qy * wz - qz * wy);
  o[5] = 0.5f * (qw * wy - qx * wz + qz * wx);
  o[6] = 0.5f * (qw * wz + qx * wy - qy * wx);
  o[7] = s * (2.f * (qx * qz + qw * qy));
  o[8] = s * (2.f * (qy * qz - qw * qx));
  o[9] = s * (cst(1.f) - 2.f * (qx * qx + qy * qy)) - P.g;
  o[10] = tx - P.cx * wy * wz;
  o[11] = ty - P.cy * wz * wx;
  o[12] = tz - P.cz * wx * wy;
}

// one RK4 step with the thrust held; x and the result are 13 five-part numbers
__device__ __forceinline__ void rk4_5(const PN& P, const N5* x, const N5* u, N5* xn) {
  const N5 s = (u[0] + u[1] + u[2] + u[3]) * P.im;
  const N5 tx = P.a * (u[0] + u[1] - u[2] - u[3]) * P.iJx;
  const N5 ty = P.a * (u[1] + u[2] - u[0] - u[3]) * P.iJy;
  const N5 tz = P.kappa * (u[0] - u[1] + u[2] - u[3]) * P.iJz;
  const N5 h2 = 0.5f * P.h, h6 = (1.f / 6.f) * P.h;
  N5 k[NX], acc[NX], xs[NX];
  rhs5(P, x, s, tx, ty, tz, k);
#pragma unroll
  for (int i = 0; i < NX; ++i) {
    acc[i] = k[i];
    xs[i] = x[i] + h2 * k[i];
  }
  rhs5(P, xs, s, tx, ty, tz, k);
#pragma unroll
  for (int i = 0; i < NX; ++i) {
    acc[i] = acc[i] + 2.f * k[i];
    xs[i] = x[i] + h2 * k[i];
  }
  rhs5(P, xs, s, tx, ty, tz, k);
#pragma unroll
  for (int i = 0; i < NX; ++i) {
    acc[i] = acc[i] + 2.f * k[i];
    xs[i] = x[i] + P.h * k[i];
  }
  rhs5(P, xs, s, tx, ty, tz, k);
#pragma unroll
  for (int i = 0; i < NX; ++i) xn[i] = x[i] + h6 * (acc[i] + k[i]);
}

// one stage of the recursions on lane j < 8: xi, eta <- their values at t + 1
__device__ __forceinline__ void propagate(const PN& P, const float* xs, const float* us, const float* xt,
                                          const float* ut, float* xi, float* eta) {
  N5 x[NX], u[NU], y[NX];
#pragma unroll
  for (int i = 0; i < NX; ++i) x[i] = {xs[i], xt[i], 0.f, eta[i], xi[i]};
#pragma unroll
  for (int a = 0; a < NU; ++a) u[a] = {us[a], ut[a], 0.f, 0.f, 0.f};
  rk4_5(P, x, u, y);
#pragma unroll
  for (int i = 0; i < NX; ++i) {
    xi[i] = y[i].s;
    eta[i] = y[i].ed;
  }
}

}  // namespace dmpc_theta
