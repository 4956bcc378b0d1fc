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
// which needs no backward pass and no storage.  Constant j is owned by two
// lanes of the instance's row, each taking one RK4 step per stage in its own
// number type:
//  * lane j carries xi_j in dual numbers v + s sig, state seeded (x*, xi_j),
//    constant j seeded with sig: the sig part of the step is A xi_j +
//    df/dtheta_j = xi_{t+1};
//  * lane 8 + j carries eta_j in numbers v + e eps + d del + ed eps del,
//    state seeded (x*, xt, 0, eta_j), controls (u*, ut, 0, 0), constant j
//    seeded with del: the eps-del part is A eta_j + d(F zt)/dtheta_j =
//    eta_{t+1} (the state carries no del part, so no second derivative in
//    the state enters).
// The constants themselves are pairs (value, derivative along constant j).
#pragma once

namespace dmpc_theta {

using dmpc_dev::NU;
using dmpc_dev::NX;

// a model constant (or a function of them) and its derivative along constant j
struct P2 {
  float v, d;
};
__device__ __forceinline__ P2 operator+(const P2& a, const P2& b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ P2 operator-(const P2& a, const P2& b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ P2 operator*(float c, const P2& a) { return {c * a.v, c * a.d}; }
__device__ __forceinline__ P2 operator*(const P2& a, const P2& b) { return {a.v * b.v, fmaf(a.v, b.d, a.d * b.v)}; }
__device__ __forceinline__ P2 inv(const P2& a) {
  const float r = 1.f / a.v;
  return {r, -a.d * r * r};
}

// dual number for xi: value and derivative along constant j
struct D2 {
  float v, s;
};
__device__ __forceinline__ D2 lift(const P2& p, D2*) { return {p.v, p.d}; }
__device__ __forceinline__ D2 operator+(const D2& a, const D2& b) { return {a.v + b.v, a.s + b.s}; }
__device__ __forceinline__ D2 operator-(const D2& a, const D2& b) { return {a.v - b.v, a.s - b.s}; }
__device__ __forceinline__ D2 operator-(const D2& a) { return {-a.v, -a.s}; }
__device__ __forceinline__ D2 operator*(float c, const D2& a) { return {c * a.v, c * a.s}; }
__device__ __forceinline__ D2 operator*(const D2& a, const D2& b) { return {a.v * b.v, fmaf(a.v, b.s, a.s * b.v)}; }
__device__ __forceinline__ D2 operator*(const D2& a, const P2& b) { return {a.v * b.v, fmaf(a.v, b.d, a.s * b.v)}; }

// hyper-dual number for eta: value, tangent along the adjoint solution,
// derivative along constant j, mixed part
struct H4 {
  float v, e, d, ed;
};
__device__ __forceinline__ H4 lift(const P2& p, H4*) { return {p.v, 0.f, p.d, 0.f}; }
__device__ __forceinline__ H4 operator+(const H4& a, const H4& b) { return {a.v + b.v, a.e + b.e, a.d + b.d, a.ed + b.ed}; }
__device__ __forceinline__ H4 operator-(const H4& a, const H4& b) { return {a.v - b.v, a.e - b.e, a.d - b.d, a.ed - b.ed}; }
__device__ __forceinline__ H4 operator-(const H4& a) { return {-a.v, -a.e, -a.d, -a.ed}; }
__device__ __forceinline__ H4 operator*(float c, const H4& a) { return {c * a.v, c * a.e, c * a.d, c * a.ed}; }
__device__ __forceinline__ H4 operator*(const H4& a, const H4& b) {
  return {a.v * b.v, fmaf(a.v, b.e, a.e * b.v), fmaf(a.v, b.d, a.d * b.v),
          fmaf(a.v, b.ed, fmaf(a.e, b.d, fmaf(a.d, b.e, a.ed * b.v)))};
}
__device__ __forceinline__ H4 operator*(const H4& a, const P2& b) {
  return {a.v * b.v, a.e * b.v, fmaf(a.v, b.d, a.d * b.v), fmaf(a.e, b.d, a.ed * b.v)};
}

// model constants as pairs, constant j seeded
struct PN {
  P2 im, a, kappa, iJx, iJy, iJz, cx, cy, cz, h, h2, h6, g;
};

__device__ __forceinline__ PN make_pn(const dmpc_quad_params& q, int j) {
  const float raw[8] = {q.mass, q.Jxx, q.Jyy, q.Jzz, q.arm, q.kappa, q.dt, q.g};
  P2 th[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) th[i] = {raw[i], (i == j) ? 1.f : 0.f};
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
  P.h2 = 0.5f * th[6];
  P.h6 = (1.f / 6.f) * th[6];
  P.g = th[7];
  return P;
}

// derivatives of the rotational and velocity states (eq. (1), X-configuration
// quadrotor, scalar-first quaternion, body rates); the position derivative is
// the velocity itself and is taken by the caller.  x holds q (3..6), v (7..9)
// and w (10..12) at their usual indices.
template <class N>
__device__ __forceinline__ void rhs_qvw(const PN& P, const N* x, const N& s, const N& tx, const N& ty, const N& tz,
                                        N* o) {
  const N qw = x[3], qx = x[4], qy = x[5], qz = x[6], wx = x[10], wy = x[11], wz = x[12];
  o[3] = 0.5f * (-(qx * wx) - qy * wy - qz * wz);
  o[4] = 0.5f * (qw * wx + qy * wz - qz * wy);
  o[5] = 0.5f * (qw * wy - qx * wz + qz * wx);
  o[6] = 0.5f * (qw * wz + qx * wy - qy * wx);
  o[7] = s * (2.f * (qx * qz + qw * qy));
  o[8] = s * (2.f * (qy * qz - qw * qx));
  N one{};
  one.v = 1.f;
  o[9] = s * (one - 2.f * (qx * qx + qy * qy)) - lift(P.g, (N*)nullptr);
  o[10] = tx - (wy * wz) * P.cx;
  o[11] = ty - (wz * wx) * P.cy;
  o[12] = tz - (wx * wy) * P.cz;
}

// one RK4 step with the thrust held.  Position enters no derivative, so the
// stage points keep only q, v, w, and the position's stage derivative (the
// stage point's velocity) is accumulated directly.
template <class N>
__device__ __forceinline__ void rk4_n(const PN& P, const N* x, const N* u, N* xn) {
  const N s = (u[0] + u[1] + u[2] + u[3]) * P.im;
  const N tx = ((u[0] + u[1] - u[2] - u[3]) * P.a) * P.iJx;
  const N ty = ((u[1] + u[2] - u[0] - u[3]) * P.a) * P.iJy;
  const N tz = ((u[0] - u[1] + u[2] - u[3]) * P.kappa) * P.iJz;
  N acc[NX], xs[NX], k[NX];
#pragma unroll
  for (int i = 0; i < NX; ++i) xs[i] = x[i];
  // stage 1
  rhs_qvw(P, xs, s, tx, ty, tz, k);
#pragma unroll
  for (int i = 0; i < 3; ++i) acc[i] = xs[7 + i];
#pragma unroll
  for (int i = 3; i < NX; ++i) acc[i] = k[i];
#pragma unroll
  for (int i = 3; i < NX; ++i) xs[i] = x[i] + k[i] * P.h2;
  // stages 2 and 3 (weight 2)
#pragma unroll
  for (int st = 0; st < 2; ++st) {
    rhs_qvw(P, xs, s, tx, ty, tz, k);
#pragma unroll
    for (int i = 0; i < 3; ++i) acc[i] = acc[i] + 2.f * xs[7 + i];
#pragma unroll
    for (int i = 3; i < NX; ++i) acc[i] = acc[i] + 2.f * k[i];
    const P2 c = (st == 0) ? P.h2 : P.h;
#pragma unroll
    for (int i = 3; i < NX; ++i) xs[i] = x[i] + k[i] * c;
  }
  // stage 4
  rhs_qvw(P, xs, s, tx, ty, tz, k);
#pragma unroll
  for (int i = 0; i < 3; ++i) xn[i] = x[i] + (acc[i] + xs[7 + i]) * P.h6;
#pragma unroll
  for (int i = 3; i < NX; ++i) xn[i] = x[i] + (acc[i] + k[i]) * P.h6;
}

// lane j < 8: xi_j <- xi_j at t + 1
__device__ __forceinline__ void propagate_xi(const PN& P, const float* xs, const float* us, float* xi) {
  D2 x[NX], u[NU], y[NX];
#pragma unroll
  for (int i = 0; i < NX; ++i) x[i] = {xs[i], xi[i]};
#pragma unroll
  for (int a = 0; a < NU; ++a) u[a] = {us[a], 0.f};
  rk4_n(P, x, u, y);
#pragma unroll
  for (int i = 0; i < NX; ++i) xi[i] = y[i].s;
}

// lane 8 + j: eta_j <- eta_j at t + 1
__device__ __forceinline__ void propagate_eta(const PN& P, const float* xs, const float* us, const float* xt,
                                              const float* ut, float* eta) {
  H4 x[NX], u[NU], y[NX];
#pragma unroll
  for (int i = 0; i < NX; ++i) x[i] = {xs[i], xt[i], 0.f, eta[i]};
#pragma unroll
  for (int a = 0; a < NU; ++a) u[a] = {us[a], ut[a], 0.f, 0.f};
  rk4_n(P, x, u, y);
#pragma unroll
  for (int i = 0; i < NX; ++i) eta[i] = y[i].ed;
}

}  // namespace dmpc_theta
