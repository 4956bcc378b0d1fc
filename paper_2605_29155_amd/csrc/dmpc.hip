// dmpc.hip -- kernels and C ABI of the batched differentiable MPC layer
// (CA-AC-MPC, Sec. IV: control-limited iLQR forward with rollout and
// linearisation, Riccati backward pass with input bounds, line-search forward
// pass; implicit-KKT backward).  Target: gfx950 only.
//
// Two launch forms share the same device routines:
//  * persistent form: one launch runs the whole forward for every instance
//    (waves pop four-instance units from an atomic queue; per-instance early
//    exit; optional longest-horizon-first order), one launch runs the backward;
//  * per-launch form (DMPC_PLAIN): init, then linearise / Riccati / line search
//    as three launches per iteration, then the tail and the outputs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <mutex>
#include <vector>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <utility>

#include "dmpc.h"
#include "dmpc_device.hpp"
#include "dmpc_theta.hpp"

using namespace dmpc_dev;

namespace {

struct Ws {
  int* state;   // [B][SW]
  int* queue;   // work counter of the persistent launch
  int* order;   // [B] instance order (longest horizon first)
  float* traj;  // [B][NSLOT][Tm][ZS] in the dynamics precision (float, or double in the FP64 form)
  float* gains; // [B][Tm][GS] in the dynamics precision
  float* lin;   // [B][Tm][FS]  (per-launch form)
  float* tail;  // [B][tstride][TS]  stage factors for the backward: every stage,
                //   or (checkpointing) one segment, recomputed by the backward
  float* ktil;  // [B][Tm][4]   (backward scratch)
  double* ck;   // [B][nck][CK_W] checkpoints of (V, v) at stages j * ckpt
  double* elem;  // [2][B][Tm][EL_W] time-parallel Riccati elements (ping-pong), or null
  uint8_t* pat;  // [B][Tm] clamp pattern of the last backward pass (time-parallel guess), or null
};

struct KArgs {
  Dyn P;
  int B, Tm, K, need_grad, use_order, nquads;
  int ckpt, nck, tstride;  // checkpoint interval (0 = off), checkpoints per instance, tail stages per instance
  int has_lin;             // the workspace holds the per-launch form's linearisation buffer
  int tpar;                // per-launch form with the time-parallel Riccati: serial sweep only as fallback
  float tol, piv;
  const float *x0, *Q, *p, *lo, *hi;
  const float* uinit;  // [B][Tm][4] initial controls (warm start) or null (hover thrust)
  const int* T;
  float *u_out, *x_out;
  uint32_t* status;
  uint8_t* dlog;
  Ws ws;
  const float *gu, *gx;
  float *gQ, *gp, *gx0;
  float* gdyn;           // [B][8] dL/d(model constants) or null
  dmpc_quad_params raw;  // model constants as given (for gdyn)
  Dyn64 P64;             // the constants of P in double (the FP64 form's dynamics)
  // FP64 redo of flagged instances: their number (device), or null for a
  // launch over the whole batch; the float trajectory region the redo copies
  // its final nominal into (read by the backward)
  const int* redo_count;
  float* traj_f;
  // with DMPC_F64_REDO: the redo's own trajectories [B][NSLOT][Tm][ZS] and
  // gains [B][Tm][GS], doubles (else null)
  float* traj64;
  float* gains64;
};

struct Grp {
  int b, T, l, col;
  bool valid;
  float lo[4], hi[4];
};

__device__ __forceinline__ void mem_fence_wg() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// the dynamics constants in precision R
template <class R>
__device__ __forceinline__ const DynT<R>& dyn_of(const KArgs& A);
template <>
__device__ __forceinline__ const DynT<float>& dyn_of<float>(const KArgs& A) { return A.P; }
template <>
__device__ __forceinline__ const DynT<double>& dyn_of<double>(const KArgs& A) { return A.P64; }

template <class R = float>
__device__ __forceinline__ R* traj_at(const KArgs& A, int b, int s, int t) {
  return (R*)A.ws.traj + (((size_t)b * NSLOT + s) * A.Tm + t) * ZS;
}
template <class R = float>
__device__ __forceinline__ R* gains_at(const KArgs& A, int b, int t) {
  return (R*)A.ws.gains + ((size_t)b * A.Tm + t) * GS;
}
__device__ __forceinline__ float* lin_at(const KArgs& A, int b, int t) { return A.ws.lin + ((size_t)b * A.Tm + t) * FS; }
// tl: stage index within the stored range (t itself, or t - segment start)
__device__ __forceinline__ float* tail_at(const KArgs& A, int b, int tl) {
  return A.ws.tail + ((size_t)b * A.tstride + tl) * TS;
}

// four values of precision R: one 16-byte access for float, two for double
template <class R>
struct V4 {
  R x, y, z, w;
};
__device__ __forceinline__ const float4& ld4(const float* p) { return *(const float4*)p; }
template <class R>
__device__ __forceinline__ auto zero4() {
  if constexpr (sizeof(R) == sizeof(float)) return make_float4(0.f, 0.f, 0.f, 0.f);
  else return V4<double>{0.0, 0.0, 0.0, 0.0};
}
__device__ __forceinline__ V4<double> ld4(const double* p) {
  const double2 a = *(const double2*)p, c = *(const double2*)(p + 2);
  return {a.x, a.y, c.x, c.y};
}
__device__ __forceinline__ void st4(float* p, float a, float b, float c, float d) {
  *(float4*)p = make_float4(a, b, c, d);
}
__device__ __forceinline__ void st4(double* p, double a, double b, double c, double d) {
  *(double2*)p = make_double2(a, b);
  *(double2*)(p + 2) = make_double2(c, d);
}

__device__ __forceinline__ int pidx(int i, int j) { return 17 * i - (i * (i - 1)) / 2 + (j - i); }

__device__ __forceinline__ void load_z(const double* zp, double* z) {
#pragma unroll
  for (int i = 0; i < 12; i += 2) {
    const double2 w = *(const double2*)(zp + i);
    z[i] = w.x;
    z[i + 1] = w.y;
  }
  z[12] = zp[12];
#pragma unroll
  for (int i = 0; i < 4; i += 2) {
    const double2 w = *(const double2*)(zp + 16 + i);
    z[13 + i] = w.x;
    z[14 + i] = w.y;
  }
}

__device__ __forceinline__ void store_z(double* zp, const double* x, const double* u) {
#pragma unroll
  for (int i = 0; i < 12; i += 2) *(double2*)(zp + i) = make_double2(x[i], x[i + 1]);
  *(double2*)(zp + 12) = make_double2(x[12], 0.0);
  *(double2*)(zp + 14) = make_double2(0.0, 0.0);
  *(double2*)(zp + 16) = make_double2(u[0], u[1]);
  *(double2*)(zp + 18) = make_double2(u[2], u[3]);
}

__device__ __forceinline__ void load_z(const float* zp, float* z) {
  const float4 a = *(const float4*)(zp);
  const float4 b = *(const float4*)(zp + 4);
  const float4 c = *(const float4*)(zp + 8);
  const float4 u = *(const float4*)(zp + 16);
  z[0] = a.x; z[1] = a.y; z[2] = a.z; z[3] = a.w;
  z[4] = b.x; z[5] = b.y; z[6] = b.z; z[7] = b.w;
  z[8] = c.x; z[9] = c.y; z[10] = c.z; z[11] = c.w;
  z[12] = zp[12];
  z[13] = u.x; z[14] = u.y; z[15] = u.z; z[16] = u.w;
}

__device__ __forceinline__ void store_z(float* zp, const float* x, const float* u) {
  *(float4*)(zp) = make_float4(x[0], x[1], x[2], x[3]);
  *(float4*)(zp + 4) = make_float4(x[4], x[5], x[6], x[7]);
  *(float4*)(zp + 8) = make_float4(x[8], x[9], x[10], x[11]);
  *(float4*)(zp + 12) = make_float4(x[12], 0.f, 0.f, 0.f);
  *(float4*)(zp + 16) = make_float4(u[0], u[1], u[2], u[3]);
}

__device__ __forceinline__ Grp make_grp(const KArgs& A, int slot, int l, int nb = -1) {
  Grp G;
  G.l = l;
  G.col = (l == 0) ? 16 : l;
  G.valid = slot < (nb < 0 ? A.B : nb);
  G.b = G.valid ? (A.use_order ? A.ws.order[slot] : slot) : 0;
  int T = A.Tm;
  if (G.valid && A.T) T = A.T[G.b];
  T = T < 0 ? 0 : (T > A.Tm ? A.Tm : T);
  G.T = G.valid ? T : 0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    G.lo[a] = G.valid ? A.lo[(size_t)G.b * 4 + a] : 0.f;
    G.hi[a] = G.valid ? A.hi[(size_t)G.b * 4 + a] : 0.f;
  }
  return G;
}

// initial nominal (Alg. 2, Rollout): U^0 = clamp(warm start, or m g / 4 without
// one), X^0 by RK4
template <class R = float>
__device__ void grp_init(const KArgs& A, const Grp& G) {
  R x[NX], xn[NX], u[NU];
#pragma unroll
  for (int i = 0; i < NX; ++i) x[i] = (R)A.x0[(size_t)G.b * NX + i];
  for (int t = 0; t < G.T; ++t) {
    const float* ui = A.uinit ? A.uinit + ((size_t)G.b * A.Tm + t) * NU : nullptr;
#pragma unroll
    for (int a = 0; a < NU; ++a) {
      if constexpr (sizeof(R) == sizeof(float))
        u[a] = clampf(ui ? ui[a] : A.P.hover, G.lo[a], G.hi[a]);
      else
        u[a] = clampd(ui ? (double)ui[a] : A.P64.hover, (double)G.lo[a], (double)G.hi[a]);
    }
    if (G.l == 0) store_z(traj_at<R>(A, G.b, 0, t), x, u);
    if (t + 1 < G.T) {
      rk4(dyn_of<R>(A), x, u, xn);
#pragma unroll
      for (int i = 0; i < NX; ++i) x[i] = xn[i];
    }
  }
}

// LDS region of one instance (doubles): the symmetric V being assembled (13
// rows, stride 14), each lane's Q_xx column parked while the control block is
// solved (stride 14), and one dummy slot per lane for the writes the V update
// masks out.  Everything else a stage needs from other lanes comes through DPP
// row broadcasts.
constexpr int L_V = 0, L_QX = 198, L_DUM = 438, L_REG = 516;
// checkpoint record (doubles): V rows at stride 14, v at CK_VV
constexpr int CK_VV = 182, CK_W = 198;

// orders the row's LDS traffic only (outstanding global loads stay in flight)
__device__ __forceinline__ void lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  __builtin_amdgcn_wave_barrier();
}

template <int N>
__device__ __forceinline__ void lds_read(const double* p, double* v) {
#pragma unroll
  for (int i = 0; i + 1 < N; i += 2) {
    const double2 w = *(const double2*)(p + i);
    v[i] = w.x;
    v[i + 1] = w.y;
  }
  if (N & 1) v[N - 1] = p[N - 1];
}

template <int N>
__device__ __forceinline__ void lds_write(double* p, const double* v) {
#pragma unroll
  for (int i = 0; i + 1 < N; i += 2) *(double2*)(p + i) = make_double2(v[i], v[i + 1]);
  if (N & 1) p[N - 1] = v[N - 1];
}

// One backward sweep t = t_hi-1 .. t_lo of the Riccati recursion (Sec. IV
// "Backward pass with input bounds"), starting from V = v = 0 or from a
// checkpoint (vinit: a record of V and v at stage t_hi).  MODE 0: stagewise
// box-QP, writes K_t, k_t to the gains and the pattern to the decision log.
// MODE 1 (tail): the active set is fixed to the controls that sit on a bound,
// writes F_t, K_t and the masked inverse of the free block for the backward at
// tail index t - tbase.  MODE 2 (tail with checkpointing): as MODE 1 but stores
// only V and v at the stages j * ckpt, from which the backward recomputes the
// factors segment by segment.  LIN_INLINE: A_t, B_t computed here (persistent
// form) or read from the linearisation buffer (per-launch).
//
// The stage algebra accumulates in FP64: without it the Schur-complement
// update of V loses several digits on these costs.  Lane l forms column col(l)
// of Q = C + F^T V F and keeps row l of V in registers; the operands a lane
// needs from the others (rows of V, columns of F, row 0 of Q, the control
// block, gain columns) arrive by 64-bit DPP row broadcasts, fused into the
// FMAs that consume them (y_block, q_block_*, v_block, fv_chain), so the
// contractions do not go through LDS.  Known columns of F are used exactly: F[:,0..2] = e_0..e_2
// (nothing depends on position), F[:,7..9] = dt e_0..2 + e_7..9 (velocity only
// drives position), and rows 10..12 of F[:,3..6] are zero (body rates do not
// depend on the attitude).
// Fused row-broadcast FMAs.  gfx950 has v_fmac_f64 with a DPP row_newbcast
// source (the broadcast operand read from one lane of the 16-lane row, then
// multiplied and accumulated in FP64), but the compiler only emits 64-bit DPP
// as two 32-bit DPP moves followed by the FMA.  These helpers issue the fused
// form from inline asm, one block per group of independent updates.  DPP reads
// need wait states after a VALU write of the source (and after an EXEC
// write), which the compiler does not insert around inline asm; each block
// therefore starts with s_nop 4 (five wait states), and inside a block no
// instruction writes a DPP source (outputs are read-write operands, so they
// cannot share a register with an input).  Accumulation order per output is
// the order of the calls, as in the plain fma() form.
// Y[i] += (V[i] of lane K) * f, i < 13
template <int K>
__device__ __forceinline__ void y_block(double (&Y)[NX], const double (&V)[NX], double f) {
  asm("s_nop 4\n\tv_fmac_f64_dpp %0, %13, %26 row_newbcast:%27 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %1, %14, %26 row_newbcast:%27 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %2, %15, %26 row_newbcast:%27 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %3, %16, %26 row_newbcast:%27 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %4, %17, %26 row_newbcast:%27 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %5, %18, %26 row_newbcast:%27 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %6, %19, %26 row_newbcast:%27 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %7, %20, %26 row_newbcast:%27 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %8, %21, %26 row_newbcast:%27 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %9, %22, %26 row_newbcast:%27 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %10, %23, %26 row_newbcast:%27 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %11, %24, %26 row_newbcast:%27 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %12, %25, %26 row_newbcast:%27 row_mask:0xf bank_mask:0xf"
      : "+v"(Y[0]), "+v"(Y[1]), "+v"(Y[2]), "+v"(Y[3]), "+v"(Y[4]), "+v"(Y[5]), "+v"(Y[6]), "+v"(Y[7]), "+v"(Y[8]), "+v"(Y[9]), "+v"(Y[10]), "+v"(Y[11]), "+v"(Y[12])
      : "v"(V[0]), "v"(V[1]), "v"(V[2]), "v"(V[3]), "v"(V[4]), "v"(V[5]), "v"(V[6]), "v"(V[7]), "v"(V[8]), "v"(V[9]), "v"(V[10]), "v"(V[11]), "v"(V[12]), "v"(f), "n"(K));
}

// Q[i] += (f of lane lane_of(i)) * y for i in 3..6, 10..16 (one stage k < 10 of F^T Y)
__device__ __forceinline__ void q_block_a(double (&Q)[NZ], double f, double y) {
  asm("s_nop 4\n\tv_fmac_f64_dpp %0, %11, %12 row_newbcast:3 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %1, %11, %12 row_newbcast:4 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %2, %11, %12 row_newbcast:5 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %3, %11, %12 row_newbcast:6 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %4, %11, %12 row_newbcast:10 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %5, %11, %12 row_newbcast:11 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %6, %11, %12 row_newbcast:12 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %7, %11, %12 row_newbcast:13 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %8, %11, %12 row_newbcast:14 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %9, %11, %12 row_newbcast:15 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %10, %11, %12 row_newbcast:0 row_mask:0xf bank_mask:0xf"
      : "+v"(Q[3]), "+v"(Q[4]), "+v"(Q[5]), "+v"(Q[6]), "+v"(Q[10]), "+v"(Q[11]), "+v"(Q[12]), "+v"(Q[13]), "+v"(Q[14]), "+v"(Q[15]), "+v"(Q[16])
      : "v"(f), "v"(y));
}

// Q[i] += (f of lane lane_of(i)) * y for i in 10..16 (stages k >= 10 of F^T Y)
__device__ __forceinline__ void q_block_b(double (&Q)[NZ], double f, double y) {
  asm("s_nop 4\n\tv_fmac_f64_dpp %0, %7, %8 row_newbcast:10 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %1, %7, %8 row_newbcast:11 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %2, %7, %8 row_newbcast:12 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %3, %7, %8 row_newbcast:13 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %4, %7, %8 row_newbcast:14 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %5, %7, %8 row_newbcast:15 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %6, %7, %8 row_newbcast:0 row_mask:0xf bank_mask:0xf"
      : "+v"(Q[10]), "+v"(Q[11]), "+v"(Q[12]), "+v"(Q[13]), "+v"(Q[14]), "+v"(Q[15]), "+v"(Q[16])
      : "v"(f), "v"(y));
}

// S[j] += (k of lane j) * q for j < 13 (one control's term of the V update)
__device__ __forceinline__ void v_block(double (&S)[NX], double k, double q) {
  asm("s_nop 4\n\tv_fmac_f64_dpp %0, %13, %14 row_newbcast:0 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %1, %13, %14 row_newbcast:1 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %2, %13, %14 row_newbcast:2 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %3, %13, %14 row_newbcast:3 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %4, %13, %14 row_newbcast:4 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %5, %13, %14 row_newbcast:5 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %6, %13, %14 row_newbcast:6 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %7, %13, %14 row_newbcast:7 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %8, %13, %14 row_newbcast:8 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %9, %13, %14 row_newbcast:9 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %10, %13, %14 row_newbcast:10 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %11, %13, %14 row_newbcast:11 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %12, %13, %14 row_newbcast:12 row_mask:0xf bank_mask:0xf"
      : "+v"(S[0]), "+v"(S[1]), "+v"(S[2]), "+v"(S[3]), "+v"(S[4]), "+v"(S[5]), "+v"(S[6]), "+v"(S[7]), "+v"(S[8]), "+v"(S[9]), "+v"(S[10]), "+v"(S[11]), "+v"(S[12])
      : "v"(k), "v"(q));
}

// acc += sum_k (v of lane k) * F[k], k = 0..12 in order
__device__ __forceinline__ void fv_chain(double& acc, double v, const double (&F)[NX]) {
  asm("s_nop 4\n\tv_fmac_f64_dpp %0, %1, %2 row_newbcast:0 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %0, %1, %3 row_newbcast:1 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %0, %1, %4 row_newbcast:2 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %0, %1, %5 row_newbcast:3 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %0, %1, %6 row_newbcast:4 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %0, %1, %7 row_newbcast:5 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %0, %1, %8 row_newbcast:6 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %0, %1, %9 row_newbcast:7 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %0, %1, %10 row_newbcast:8 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %0, %1, %11 row_newbcast:9 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %0, %1, %12 row_newbcast:10 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %0, %1, %13 row_newbcast:11 row_mask:0xf bank_mask:0xf\n\tv_fmac_f64_dpp %0, %1, %14 row_newbcast:12 row_mask:0xf bank_mask:0xf"
      : "+v"(acc)
      : "v"(v), "v"(F[0]), "v"(F[1]), "v"(F[2]), "v"(F[3]), "v"(F[4]), "v"(F[5]), "v"(F[6]), "v"(F[7]), "v"(F[8]), "v"(F[9]), "v"(F[10]), "v"(F[11]), "v"(F[12]));
}

// B[j] = v of lane j, j < 16
__device__ __forceinline__ void bcast16(double (&Bv)[16], double v) {
  asm("s_nop 4\n\tv_mov_b64_dpp %0, %16 row_newbcast:0 row_mask:0xf bank_mask:0xf\n\tv_mov_b64_dpp %1, %16 row_newbcast:1 row_mask:0xf bank_mask:0xf\n\tv_mov_b64_dpp %2, %16 row_newbcast:2 row_mask:0xf bank_mask:0xf\n\tv_mov_b64_dpp %3, %16 row_newbcast:3 row_mask:0xf bank_mask:0xf\n\tv_mov_b64_dpp %4, %16 row_newbcast:4 row_mask:0xf bank_mask:0xf\n\tv_mov_b64_dpp %5, %16 row_newbcast:5 row_mask:0xf bank_mask:0xf\n\tv_mov_b64_dpp %6, %16 row_newbcast:6 row_mask:0xf bank_mask:0xf\n\tv_mov_b64_dpp %7, %16 row_newbcast:7 row_mask:0xf bank_mask:0xf\n\tv_mov_b64_dpp %8, %16 row_newbcast:8 row_mask:0xf bank_mask:0xf\n\tv_mov_b64_dpp %9, %16 row_newbcast:9 row_mask:0xf bank_mask:0xf\n\tv_mov_b64_dpp %10, %16 row_newbcast:10 row_mask:0xf bank_mask:0xf\n\tv_mov_b64_dpp %11, %16 row_newbcast:11 row_mask:0xf bank_mask:0xf\n\tv_mov_b64_dpp %12, %16 row_newbcast:12 row_mask:0xf bank_mask:0xf\n\tv_mov_b64_dpp %13, %16 row_newbcast:13 row_mask:0xf bank_mask:0xf\n\tv_mov_b64_dpp %14, %16 row_newbcast:14 row_mask:0xf bank_mask:0xf\n\tv_mov_b64_dpp %15, %16 row_newbcast:15 row_mask:0xf bank_mask:0xf"
      : "=&v"(Bv[0]), "=&v"(Bv[1]), "=&v"(Bv[2]), "=&v"(Bv[3]), "=&v"(Bv[4]), "=&v"(Bv[5]), "=&v"(Bv[6]), "=&v"(Bv[7]), "=&v"(Bv[8]), "=&v"(Bv[9]), "=&v"(Bv[10]), "=&v"(Bv[11]), "=&v"(Bv[12]), "=&v"(Bv[13]), "=&v"(Bv[14]), "=&v"(Bv[15])
      : "v"(v));
}

// the 4x4 control block Q[13+a][13+b] (upper triangle, column b from lane
// lane_of(13+b): h[] in the order (0,0) (0,1) (1,1) (0,2) (1,2) (2,2) (0,3) ..)
// and q_u[b] from the same lanes
__device__ __forceinline__ void hq_block(double (&h)[10], double (&qu)[4], const double (&Qc)[NZ], double qc) {
  asm("s_nop 4\n\tv_mov_b64_dpp %0, %14 row_newbcast:13 row_mask:0xf bank_mask:0xf\n\tv_mov_b64_dpp %1, %14 row_newbcast:14 row_mask:0xf bank_mask:0xf\n\tv_mov_b64_dpp %2, %15 row_newbcast:14 row_mask:0xf bank_mask:0xf\n\tv_mov_b64_dpp %3, %14 row_newbcast:15 row_mask:0xf bank_mask:0xf\n\tv_mov_b64_dpp %4, %15 row_newbcast:15 row_mask:0xf bank_mask:0xf\n\tv_mov_b64_dpp %5, %16 row_newbcast:15 row_mask:0xf bank_mask:0xf\n\tv_mov_b64_dpp %6, %14 row_newbcast:0 row_mask:0xf bank_mask:0xf\n\tv_mov_b64_dpp %7, %15 row_newbcast:0 row_mask:0xf bank_mask:0xf\n\tv_mov_b64_dpp %8, %16 row_newbcast:0 row_mask:0xf bank_mask:0xf\n\tv_mov_b64_dpp %9, %17 row_newbcast:0 row_mask:0xf bank_mask:0xf\n\tv_mov_b64_dpp %10, %18 row_newbcast:13 row_mask:0xf bank_mask:0xf\n\tv_mov_b64_dpp %11, %18 row_newbcast:14 row_mask:0xf bank_mask:0xf\n\tv_mov_b64_dpp %12, %18 row_newbcast:15 row_mask:0xf bank_mask:0xf\n\tv_mov_b64_dpp %13, %18 row_newbcast:0 row_mask:0xf bank_mask:0xf"
      : "=&v"(h[0]), "=&v"(h[1]), "=&v"(h[2]), "=&v"(h[3]), "=&v"(h[4]), "=&v"(h[5]), "=&v"(h[6]), "=&v"(h[7]), "=&v"(h[8]), "=&v"(h[9]), "=&v"(qu[0]), "=&v"(qu[1]), "=&v"(qu[2]), "=&v"(qu[3])
      : "v"(Qc[13]), "v"(Qc[14]), "v"(Qc[15]), "v"(Qc[16]), "v"(qc));
}

// value of v in lane L of this lane's 16-lane row (L a compile-time constant)
template <int L>
__device__ __forceinline__ double bc(double v) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)x, 0x150 + L, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(x >> 32), 0x150 + L, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
// f(integral_constant<0>) .. f(integral_constant<N-1>): a loop whose index
// is a compile-time constant in the body (DPP lane selects must be)
template <int... I, class F>
__device__ __forceinline__ void sfor_impl(std::integer_sequence<int, I...>, F&& f) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void sfor(F&& f) {
  sfor_impl(std::make_integer_sequence<int, N>{}, f);
}
// LOWREG: for a kernel capped at 256 registers (two waves per SIMD): the
// symmetric V is written with masked stores from two bases, and the lane and
// column indices are made opaque at each stage so that the compiler recomputes
// the addresses and masks derived from them instead of holding them (or
// spilling them) across the stages.  Same operations, same results.
template <bool DENSE, int MODE, bool LIN_INLINE, class R = float, bool LOWREG = false>
__device__ void grp_sweep(const KArgs& A, const Grp& G, int n, int kit, double* L, uint32_t& st, int t_hi,
                          int t_lo = 0, const double* vinit = nullptr, int tbase = 0) {
  const int l = G.l, col = G.col, b = G.b, T = G.T;
  const double hdt = (double)A.P.h;
  double Vr[NX], vl = 0.0;  // lane l < 13: row l of V and v_l at the stage being entered
#pragma unroll
  for (int j = 0; j < NX; ++j) Vr[j] = (vinit && l < NX) ? vinit[l * 14 + j] : 0.0;
  if (vinit && l < NX) vl = vinit[CK_VV + l];
  R zn[NZ];
  if (t_hi > t_lo) load_z(traj_at<R>(A, b, n, t_hi - 1), zn);
  __builtin_amdgcn_s_waitcnt(0);  // no load pending on loop entry (see grp_ls)
  for (int t = t_hi - 1; t >= t_lo; --t) {
    // LOWREG: this stage's copies of the lane and column indices, opaque to the
    // compiler, so that what it derives from them is recomputed per stage
    int l_s = l, col_s = col;
    if (LOWREG) asm volatile("" : "+v"(l_s), "+v"(col_s));
    if (MODE == 2 && t + 1 < T && (t + 1) % A.ckpt == 0) {
      // V, v of stage t + 1 (complete since the last row sync): exact FP64 image
      double* ck = A.ws.ck + ((size_t)b * A.nck + ((t + 1) / A.ckpt - 1)) * CK_W;
      if (l_s < NX) {
#pragma unroll
        for (int j = 0; j < NX; ++j) ck[l_s * 14 + j] = Vr[j];
        ck[CK_VV + l_s] = vl;
      }
    }
    const R* zp = traj_at<R>(A, b, n, t);
    // this stage's own scalars are loaded before the next stage's nominal: the
    // vector-memory counter is in order, so they can then be waited for
    // without also waiting for the prefetch
    const size_t srow0 = (size_t)b * A.Tm + t;
    const R s_zc = zp[col_s < NX ? col_s : col_s + 3];
    const float s_qc = DENSE ? 0.f : A.Q[srow0 * NZ + col_s];
    const float s_q0 = DENSE ? 0.f : A.Q[srow0 * NZ];
    const float s_pc = A.p[srow0 * NZ + col_s];
    const float s_p0 = A.p[srow0 * NZ];
    // No branch around these loads (nor around the stores at the end of the
    // stage): the wait-count insertion assumes the fewest operations in flight
    // over the paths into a wait, so a skippable load or store makes a later
    // wait also cover the loads issued after it.  The previous iteration's k
    // (the box-QP's warm start) is read at every iteration and ignored at the
    // first; at the last stage the "next" nominal is this stage's again.
    auto s_kw = zero4<R>();
    if (MODE == 0) {
      if constexpr (sizeof(R) == sizeof(float)) {
        const float4 w = *(const float4*)(gains_at(A, b, t) + 64);
        if (kit > 0) s_kw = w;
      } else {
        const auto w = ld4(gains_at<R>(A, b, t) + 64);
        if (kit > 0) s_kw = w;
      }
    }
    R zb[NZ];
#pragma unroll
    for (int i = 0; i < NZ; ++i) zb[i] = zn[i];
    load_z(traj_at<R>(A, b, n, t > t_lo ? t - 1 : t), zn);
    const bool has_dyn = (t + 1 < T);
    R Fc[NX];
    if (has_dyn) {
      if (LIN_INLINE) {
        const LaneDir<R> D = make_dir(dyn_of<R>(A), col_s);
        rk4_column(dyn_of<R>(A), zb, zb + NX, D, Fc);
      } else {
        const float* fp = lin_at(A, b, t) + col_s * 16;
#pragma unroll
        for (int k = 0; k < NX; ++k) Fc[k] = fp[k];
      }
    } else {
#pragma unroll
      for (int k = 0; k < NX; ++k) Fc[k] = R(0);
    }
    if (MODE == 1) {
      float* tp = tail_at(A, b, t - tbase);
      float* fc = tp + col_s * 16;
      *(float4*)(fc) = make_float4((float)Fc[0], (float)Fc[1], (float)Fc[2], (float)Fc[3]);
      *(float4*)(fc + 4) = make_float4((float)Fc[4], (float)Fc[5], (float)Fc[6], (float)Fc[7]);
      *(float4*)(fc + 8) = make_float4((float)Fc[8], (float)Fc[9], (float)Fc[10], (float)Fc[11]);
      fc[12] = (float)Fc[12];
      if (l_s == NX) {  // column 0 = e_0 (zero at the last stage)
        const float e = has_dyn ? 1.f : 0.f;
        *(float4*)(tp) = make_float4(e, 0.f, 0.f, 0.f);
        *(float4*)(tp + 4) = make_float4(0.f, 0.f, 0.f, 0.f);
        *(float4*)(tp + 8) = make_float4(0.f, 0.f, 0.f, 0.f);
        tp[12] = 0.f;
      }
    }
    double Fd[NX];
#pragma unroll
    for (int k = 0; k < NX; ++k) Fd[k] = (double)Fc[k];

    // Y[:, col] = V F[:, col]: lane k holds row k of V (= column k)
    double Yc[NX];
#pragma unroll
    for (int i = 0; i < NX; ++i) Yc[i] = 0.0;
    sfor<NX>([&](auto K) { y_block<K>(Yc, Vr, Fd[K]); });
    // Q[:, col] = (F^T V F)[:, col]; column i of F comes from lane lane_of(i)
    double Qc[NZ];
    Qc[0] = Yc[0];
    Qc[1] = Yc[1];
    Qc[2] = Yc[2];
#pragma unroll
    for (int m = 0; m < 3; ++m) Qc[7 + m] = fma(hdt, Yc[m], Yc[7 + m]);
#pragma unroll
    for (int i = 3; i < 7; ++i) Qc[i] = 0.0;
#pragma unroll
    for (int i = 10; i < NZ; ++i) Qc[i] = 0.0;
#pragma unroll
    for (int k = 0; k < 10; ++k) q_block_a(Qc, Fd[k], Yc[k]);
#pragma unroll
    for (int k = 10; k < NX; ++k) q_block_b(Qc, Fd[k], Yc[k]);

    // stage cost: Q += C_t, q = g + F^T v with g = C_t z + c_t
    const size_t srow = (size_t)b * A.Tm + t;
    const float* prow = A.p + srow * NZ;
    double qc, g0, c00, qdiag = 0.0;
    {
      const double zb_c = (double)s_zc;
      if (!DENSE) {
        const double qd_c = (double)s_qc;
        c00 = (double)s_q0;
        qc = fma(qd_c, zb_c, (double)s_pc);
        g0 = fma(c00, (double)zb[0], (double)s_p0);
        qdiag = qd_c;
      } else {
        const float* crow = A.Q + srow * NPK;
        double gc = (double)prow[col_s], gz = (double)prow[0];
#pragma unroll
        for (int i = 0; i < NZ; ++i) {
          const double cc = (double)crow[i <= col_s ? pidx(i, col_s) : pidx(col_s, i)];
          Qc[i] += cc;
          gc = fma(cc, (double)zb[i], gc);
          gz = fma((double)crow[i], (double)zb[i], gz);
        }
        c00 = (double)crow[0];
        qc = gc;
        g0 = gz;
      }
    }
    fv_chain(qc, vl, Fd);
    const double q0 = g0 + bc<0>(vl);
    const double v00 = bc<0>(Vr[0]);
    // control block and q_u from the lanes owning columns 13..16
    double H[16], qu[4];
    {
      double h[10];
      hq_block(h, qu, Qc, qc);
      // a diagonal cost adds to the diagonal only: its four control entries
      // here, the state entry of the parked column below (rather than a
      // 16-way select over this lane's column)
      if (!DENSE) {
        h[0] += bc<13>(qdiag);
        h[2] += bc<14>(qdiag);
        h[5] += bc<15>(qdiag);
        h[9] += bc<0>(qdiag);
      }
      int m = 0;
#pragma unroll
      for (int bb = 0; bb < 4; ++bb)
#pragma unroll
        for (int a = 0; a <= bb; ++a, ++m) {
          H[a * 4 + bb] = h[m];
          H[bb * 4 + a] = h[m];
        }
    }
    lds_write<NX>(L + L_QX + l_s * 14, Qc);
    // this lane's diagonal entry of the block, read now and completed with the
    // diagonal cost after the box-QP (the read's latency then hides behind it)
    const double qdd = DENSE ? 0.0 : L[L_QX + l_s * 15];
    // Y[0, :] by lane (row 0 of Q without the cost), broadcast only after the
    // box-QP so that its 32 registers are free during the QP
    double y0b[16];
    // row 0 of Q (lane 0's x-row; its own column is 16)
    auto R0 = [&](int j) -> double {
      double r = (j == 0) ? v00 + c00 : y0b[lane_of(j)];
      if (DENSE && j > 0) r += (double)A.Q[srow * NPK + j];
      return r;
    };
    double dl[4], dh[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      dl[a] = (double)G.lo[a] - (double)zb[NX + a];
      dh[a] = (double)G.hi[a] - (double)zb[NX + a];
    }

    double kv[4] = {0.0, 0.0, 0.0, 0.0}, fr[4];
    Fact4 C;
    R* gp = gains_at<R>(A, b, t);
    if (MODE == 0) {
      double kw[4] = {0.0, 0.0, 0.0, 0.0};
      kw[0] = s_kw.x; kw[1] = s_kw.y; kw[2] = s_kw.z; kw[3] = s_kw.w;
      // the dense FP64 kernel is at its register limit: the row solver's extra
      // registers spill inside the stage loop there (13.0 against 9.1 ms
      // forward at B=16384, T=50), so it keeps the active-set loop
      if constexpr (DENSE && sizeof(R) == sizeof(double))
        boxqp(H, qu, dl, dh, kw, A.piv, kv, fr, C, st);
      else
        boxqp_row(H, qu, dl, dh, kw, A.piv, (int)(__lane_id() & 48u), l_s, kv, fr, C, st);
    } else {
#pragma unroll
      for (int a = 0; a < 4; ++a) fr[a] = (zb[NX + a] == G.lo[a] || zb[NX + a] == G.hi[a]) ? 0.0 : 1.0;
      ldl4(H, fr, A.piv, C, st);
    }
    // every lane writes its diagonal entry back (row 0 and rows 13..15 are not
    // read below); then the rows of Q are read ahead of their use
    if (!DENSE) L[L_QX + l_s * 15] = qdd + qdiag;
    double Sq[NX];
#pragma unroll
    for (int j = 0; j < NX; ++j) Sq[j] = L[L_QX + l_s * 14 + j];

    bcast16(y0b, Yc[0]);
    // gain column: K[:, l] = -Qff^{-1} Q_ux[:, l] on the free rows, 0 on clamped rows
    double Qux[4], Kd[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      Qux[a] = (l_s == 0) ? R0(NX + a) : Qc[NX + a];
      Kd[a] = fr[a] * Qux[a];
    }
    solve4(C, Kd);
#pragma unroll
    for (int a = 0; a < 4; ++a) Kd[a] = -Kd[a];
    const R Kc[4] = {(R)Kd[0], (R)Kd[1], (R)Kd[2], (R)Kd[3]};
    // V row l = Q_xx[l, :] + Q_ux[:, l]^T K ;  v_l = Q_x[l] + Q_ux[:, l]^T k
    // (gain column j broadcast from lane j).  V is kept exactly symmetric:
    // lane l forms the entries j >= l of its row and writes each to (l, j) and
    // (j, l) (the others go to its dummy slot, which keeps the loop free of
    // branches), then every lane reads its row back.  Row k of V is used as
    // column k in the next stage, and an antisymmetric rounding residue would
    // otherwise be carried and amplified from stage to stage over long
    // horizons (the control-limited DDP of Tassa et al. 2014, cited for the
    // Riccati pass in Sec. IV, likewise keeps V symmetric).
    double R0r[NX];
#pragma unroll
    for (int j = 0; j < NX; ++j) R0r[j] = (j == 0) ? v00 + c00 : R0(j);
    if (l_s < NX) {
      double vi = (l_s == 0) ? q0 : qc;
#pragma unroll
      for (int a = 0; a < 4; ++a) vi = fma(Qux[a], kv[a], vi);
      double S[NX];
#pragma unroll
      for (int j = 0; j < NX; ++j) S[j] = (l_s == 0) ? R0r[j] : Sq[j];
#pragma unroll
      for (int a = 0; a < 4; ++a) v_block(S, Kd[a], Qux[a]);
      if (LOWREG) {
        // masked stores from two bases (row l, column l) with constant
        // offsets: no per-entry address is held across the stages
        double* row = L + L_V + l_s * 14;
        double* colm = L + L_V + l_s;
        sfor<NX>([&](auto J) {
          constexpr int j = J;
          if (j >= l_s) row[j] = S[j];
          if (j > l_s) colm[j * 14] = S[j];
        });
      } else {
        sfor<NX>([&](auto J) {
          constexpr int j = J;
          const double s = S[j];
          const int a1 = (j >= l_s) ? (L_V + l_s * 14 + j) : (L_DUM + l_s);
          const int a2 = (j > l_s) ? (L_V + j * 14 + l_s) : (L_DUM + l_s);
          L[a1] = s;
          L[a2] = s;
        });
      }
      vl = vi;
    }
    lds_sync();
    if (l_s < NX) lds_read<NX>(L + L_V + l_s * 14, Vr);

    if (MODE == 0) {
      // no branch around the stores (see the loads at the top of the stage):
      // lanes 13..15 fill the unused padding of the gain rows, and every lane
      // writes the same k
#pragma unroll
      for (int a = 0; a < 4; ++a) gp[a * 16 + l_s] = Kc[a];
      st4(gp + 64, (R)kv[0], (R)kv[1], (R)kv[2], (R)kv[3]);
      if ((A.dlog || A.ws.pat) && l_s == 0) {
        unsigned code = 0;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const unsigned c = (fr[a] != 0.0) ? 0u : (kv[a] <= dl[a] ? 1u : 2u);
          code |= c << (2 * a);
        }
        if (A.dlog) A.dlog[((size_t)b * A.K + kit) * (1 + A.Tm) + 1 + t] = (uint8_t)code;
        if (A.ws.pat) A.ws.pat[(size_t)b * A.Tm + t] = (uint8_t)code;
      }
    } else if (MODE == 1) {
      float* tp = tail_at(A, b, t - tbase);
      if (l_s < NX) *(float4*)(tp + FS + l_s * 4) = make_float4((float)Kc[0], (float)Kc[1], (float)Kc[2], (float)Kc[3]);
      // M = masked inverse of the free block (zero rows/columns on clamped controls), FP64
      if (l_s == NX + 1) {
        double M[16];
#pragma unroll
        for (int bb = 0; bb < 4; ++bb) {
          double e[4];
#pragma unroll
          for (int a = 0; a < 4; ++a) e[a] = (a == bb) ? fr[bb] : 0.0;
          solve4(C, e);
#pragma unroll
          for (int a = 0; a < 4; ++a) M[a * 4 + bb] = fr[a] * e[a];
        }
        double* mp = (double*)(tp + FS + 52);
#pragma unroll
        for (int i = 0; i < 16; i += 2) *(double2*)(mp + i) = make_double2(M[i], M[i + 1]);
      }
    }
  }
}

// Forward pass with line search (Sec. IV): the 16 lanes of an instance form
// four quads, one per candidate alpha; lane r of a quad forms control r,
//   u_r = clamp(u_bar_r + alpha k_r + K[r, :] (x - x_bar), lo_r, hi_r),
// the quad shares the four controls, rolls the state out and sums the cost.
// The next stage's nominal, gain row and cost are loaded while the current
// stage is computed.
template <bool DENSE, class R = float>
struct LsStage {
  R xb[NX];
  R ub, kr;
  R Kr[NX];
  float q[DENSE ? 1 : NZ];
  float p[NZ];
};

__device__ __forceinline__ float fmaR(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fmaR(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float clampR(float v, float lo, float hi) { return clampf(v, lo, hi); }
__device__ __forceinline__ double clampR(double v, float lo, float hi) { return clampd(v, (double)lo, (double)hi); }
__device__ __forceinline__ float absR(float v) { return fabsf(v); }
__device__ __forceinline__ double absR(double v) { return fabs(v); }
__device__ __forceinline__ float maxR(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ double maxR(double a, double b) { return fmax(a, b); }

template <bool DENSE, class R>
__device__ __forceinline__ void ls_load(const KArgs& A, int b, int n, int t, int r, LsStage<DENSE, R>& S) {
  const R* zp = traj_at<R>(A, b, n, t);
  const auto a0 = ld4(zp), a1 = ld4(zp + 4), a2 = ld4(zp + 8);
  S.xb[0] = a0.x; S.xb[1] = a0.y; S.xb[2] = a0.z; S.xb[3] = a0.w;
  S.xb[4] = a1.x; S.xb[5] = a1.y; S.xb[6] = a1.z; S.xb[7] = a1.w;
  S.xb[8] = a2.x; S.xb[9] = a2.y; S.xb[10] = a2.z; S.xb[11] = a2.w;
  S.xb[12] = zp[12];
  S.ub = zp[16 + r];
  const R* gp = gains_at<R>(A, b, t);
  S.kr = gp[64 + r];
  const R* kp = gp + r * 16;
  const auto k0 = ld4(kp), k1 = ld4(kp + 4), k2 = ld4(kp + 8);
  S.Kr[0] = k0.x; S.Kr[1] = k0.y; S.Kr[2] = k0.z; S.Kr[3] = k0.w;
  S.Kr[4] = k1.x; S.Kr[5] = k1.y; S.Kr[6] = k1.z; S.Kr[7] = k1.w;
  S.Kr[8] = k2.x; S.Kr[9] = k2.y; S.Kr[10] = k2.z; S.Kr[11] = k2.w;
  S.Kr[12] = kp[12];
  const size_t srow = (size_t)b * A.Tm + t;
  const float* prow = A.p + srow * NZ;
#pragma unroll
  for (int i = 0; i < NZ; ++i) S.p[i] = prow[i];
  if (!DENSE) {
    const float* qrow = A.Q + srow * NZ;
#pragma unroll
    for (int i = 0; i < NZ; ++i) S.q[i] = qrow[i];
  }
}

// one stage of the line search: control, cost and stage record from cur and
// the state x, prefetch of the next stage into nxt, the next state into xn
template <bool DENSE, class R>
__device__ __forceinline__ void ls_stage(const KArgs& A, int b, int n, int t, int T, int r, int sc, R alpha,
                                         float lo_r, float hi_r, const LsStage<DENSE, R>& cur,
                                         LsStage<DENSE, R>& nxt, const R* x, R* xn, R& J, R& dm) {
  // the next stage's record (at the last stage this one's again: no branch
  // around the loads, which keeps the wait counts exact)
  ls_load<DENSE, R>(A, b, n, t + 1 < T ? t + 1 : t, r, nxt);
  R ur = cur.ub + alpha * cur.kr;
#pragma unroll
  for (int j = 0; j < NX; ++j) ur = fmaR(cur.Kr[j], x[j] - cur.xb[j], ur);
  ur = clampR(ur, lo_r, hi_r);
  dm = maxR(dm, absR(ur - cur.ub));
  R z[NZ];
#pragma unroll
  for (int i = 0; i < NX; ++i) z[i] = x[i];
#pragma unroll
  for (int c = 0; c < NU; ++c) z[NX + c] = qb(ur, c);
  const size_t srow = (size_t)b * A.Tm + t;
  if (!DENSE) {
#pragma unroll
    for (int i = 0; i < NZ; ++i) J = fmaR(fmaR(R(0.5) * (R)cur.q[i], z[i], (R)cur.p[i]), z[i], J);
  } else {
    const float* crow = A.Q + srow * NPK;
    int m = 0;
#pragma unroll
    for (int i = 0; i < NZ; ++i) {
      R s = R(0.5) * (R)crow[m++] * z[i];
#pragma unroll
      for (int j = i + 1; j < NZ; ++j) s = fmaR((R)crow[m++], z[j], s);
      J = fmaR(s + (R)cur.p[i], z[i], J);
    }
  }
  {
    // lane r of the quad writes entries 4r..4r+3 of the stage record
    R* zo = traj_at<R>(A, b, sc, t);
    if constexpr (sizeof(R) == sizeof(float)) {
      const float4 w = r == 0 ? make_float4(x[0], x[1], x[2], x[3])
                     : (r == 1 ? make_float4(x[4], x[5], x[6], x[7])
                     : (r == 2 ? make_float4(x[8], x[9], x[10], x[11]) : make_float4(x[12], 0.f, 0.f, 0.f)));
      *(float4*)(zo + 4 * r) = w;
    } else {
      const R w0 = r == 0 ? x[0] : (r == 1 ? x[4] : (r == 2 ? x[8] : x[12]));
      const R w1 = r == 0 ? x[1] : (r == 1 ? x[5] : (r == 2 ? x[9] : R(0)));
      const R w2 = r == 0 ? x[2] : (r == 1 ? x[6] : (r == 2 ? x[10] : R(0)));
      const R w3 = r == 0 ? x[3] : (r == 1 ? x[7] : (r == 2 ? x[11] : R(0)));
      st4(zo + 4 * r, w0, w1, w2, w3);
    }
    // all four lanes write the same controls: no branch around the store
    st4(zo + 16, z[13], z[14], z[15], z[16]);
  }
  if (t + 1 < T) rk4(dyn_of<R>(A), x, z + NX, xn);
}

template <bool DENSE, class R = float>
__device__ void grp_ls(const KArgs& A, const Grp& G, int n, R& Jout, R& dmax) {
  const int a = G.l >> 2, r = G.l & 3, b = G.b, T = G.T;
  const R alpha = a == 0 ? R(1) : (a == 1 ? R(0.5) : (a == 2 ? R(0.25) : R(0.1)));
  const int sc = (n + 1 + a) % NSLOT;
  const float lo_r = A.lo[(size_t)b * NU + r], hi_r = A.hi[(size_t)b * NU + r];
  R x[NX], xn[NX];
#pragma unroll
  for (int i = 0; i < NX; ++i) x[i] = (R)A.x0[(size_t)b * NX + i];
  R J = R(0), dm = R(0);
  LsStage<DENSE, R> sa, sb;
  if (T > 0) ls_load<DENSE, R>(A, b, n, 0, r, sa);
  // Let the first stage's loads land before the loop: with loads still
  // pending on entry, the wait counters inside the loop have to assume that
  // any register could be one of them, and (the vector-memory counter being
  // in order) the loop would wait on the next stage's prefetch at every stage.
  __builtin_amdgcn_s_waitcnt(0);
  // two stages per trip with the stage records and the state swapping roles,
  // so that nothing is copied from one stage to the next
  for (int t = 0; t < T; t += 2) {
    ls_stage<DENSE, R>(A, b, n, t, T, r, sc, alpha, lo_r, hi_r, sa, sb, x, xn, J, dm);
    if (t + 1 >= T) break;
    ls_stage<DENSE, R>(A, b, n, t + 1, T, r, sc, alpha, lo_r, hi_r, sb, sa, xn, x, J, dm);
  }
  Jout = J;  // all four lanes of a quad hold the same cost
  dmax = quad_max(dm);
}

__device__ __forceinline__ float finite_or_inf(float v) {
  return (v == v && fabsf(v) <= 3.402823466e38f) ? v : INFINITY;
}
__device__ __forceinline__ double finite_or_inf(double v) {
  return (v == v && fabs(v) <= 1.7976931348623157e308) ? v : (double)INFINITY;
}
__device__ __forceinline__ float rbR(float v, int L) { return rb(v, L); }
__device__ __forceinline__ double rbR(double v, int L) { return rb64(v, L); }

// pick the first minimiser of the four candidate costs; returns -1 if none is finite
template <class R>
__device__ __forceinline__ int ls_select(R J, R dm, R& dsel) {
  const R c0 = finite_or_inf(rbR(J, 0)), c1 = finite_or_inf(rbR(J, 4)), c2 = finite_or_inf(rbR(J, 8)),
          c3 = finite_or_inf(rbR(J, 12));
  const R d0 = rbR(dm, 0), d1 = rbR(dm, 4), d2 = rbR(dm, 8), d3 = rbR(dm, 12);
  int best = -1;
  R bj = (R)INFINITY;
  dsel = R(0);
  if (c0 < bj) { best = 0; bj = c0; dsel = d0; }
  if (c1 < bj) { best = 1; bj = c1; dsel = d1; }
  if (c2 < bj) { best = 2; bj = c2; dsel = d2; }
  if (c3 < bj) { best = 3; bj = c3; dsel = d3; }
  return best;
}

// writes u_out / x_out (zeros past T_b) from the nominal slot
// (the 16 lanes take the stage entries in turn, eight loads in flight before
// their stores: the outputs may alias nothing, but the compiler cannot know)
template <class R = float>
__device__ void grp_outputs(const KArgs& A, const Grp& G, int n) {
  const int b = G.b, total = A.Tm * NZ;
  for (int i0 = G.l; i0 < total; i0 += 16 * 8) {
    float v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int i = i0 + 16 * j, t = i / NZ, e = i % NZ;
      v[j] = (i < total && t < G.T) ? (float)traj_at<R>(A, b, n, t)[e < NX ? e : e + 3] : 0.f;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int i = i0 + 16 * j, t = i / NZ, e = i % NZ;
      if (i >= total) break;
      if (e < NX) {
        if (A.x_out) A.x_out[((size_t)b * A.Tm + t) * NX + e] = v[j];
      } else {
        A.u_out[((size_t)b * A.Tm + t) * NU + (e - NX)] = v[j];
      }
    }
  }
}

__device__ __forceinline__ void grp_write_state(const KArgs& A, const Grp& G, int n, int iters, uint32_t st, int done) {
  if (G.l == 0) {
    int* s = A.ws.state + (size_t)G.b * SW;
    s[S_NOM] = n;
    s[S_ITERS] = iters;
    s[S_STATUS] = (int)st;
    s[S_DONE] = done;
    s[S_T] = G.T;
  }
}

// ---------------------------------------------------------------------------
// persistent forward
// ---------------------------------------------------------------------------

// OCC: waves per SIMD the register allocation is capped for (1: no cap beyond
// the 512-register file; 2: at most 256 registers, two waves share a SIMD and
// hide each other's latency when there are more waves than SIMDs).
// R: precision of the dynamics, the linearisation, the line search and the
// stored trajectories and gains (float; double in the FP64 form).
// IPW: instances per wave (4: one per 16-lane row; 2 or 1: the other rows
// idle), so that a small batch spreads over more SIMDs and an instance does
// not wait for the slowest of four in the box-QP's iterations.
template <bool DENSE, int OCC, class R = float, int IPW = 4>
__global__ __launch_bounds__(64, OCC) void k_fwd_persistent(KArgs A) {
  __shared__ double lds[4 * L_REG];
  const int lane = threadIdx.x, grp = lane >> 4, l = lane & 15;
  double* L = lds + grp * L_REG;
  // an FP64 redo takes the flagged instances listed in ws.order
  int nb = A.B, nq = (IPW == 4) ? A.nquads : (A.B + IPW - 1) / IPW;
  if constexpr (sizeof(R) == sizeof(double)) {
    if (A.redo_count) {
      nb = __builtin_amdgcn_readfirstlane(*A.redo_count);
      nq = (nb + IPW - 1) / IPW;
    }
  }
  for (;;) {
    int q = 0;
    if (lane == 0) q = atomicAdd(A.ws.queue, 1);
    q = __builtin_amdgcn_readfirstlane(q);
    if (q >= nq) break;
    const Grp G = make_grp(A, (IPW == 4 || grp < IPW) ? q * IPW + grp : nb, l, nb);
    if (!G.valid) continue;
    uint32_t st = 0;
    int n = 0, iters = 0;
    if (G.T > 0) {
      grp_init<R>(A, G);
      mem_fence_wg();
      bool done = false;
      for (int k = 0; k < A.K; ++k) {
        if (done) continue;
        grp_sweep<DENSE, 0, true, R, OCC == 2>(A, G, n, k, L, st, G.T);
        mem_fence_wg();
        R J, dm, dsel;
        grp_ls<DENSE, R>(A, G, n, J, dm);
        mem_fence_wg();
        const int best = ls_select(J, dm, dsel);
        if (A.dlog && l == 0) A.dlog[((size_t)G.b * A.K + k) * (1 + A.Tm)] = best < 0 ? 255 : (uint8_t)best;
        iters = k + 1;
        if (best < 0) {
          st |= ST_NONFINITE;
        } else {
          n = (n + 1 + best) % NSLOT;
          if (A.tol > 0.f && dsel < (R)A.tol) {
            st |= ST_CONVERGED;
            done = true;
          }
        }
      }
      if (A.tol > 0.f && !(st & ST_CONVERGED)) st |= ST_MAXITER;
      if (A.need_grad) {
        if (A.ckpt > 0) grp_sweep<DENSE, 2, true, R, OCC == 2>(A, G, n, 0, L, st, G.T);
        else grp_sweep<DENSE, 1, true, R, OCC == 2>(A, G, n, 0, L, st, G.T);
      }
    }
    grp_outputs<R>(A, G, n);
    if constexpr (sizeof(R) == sizeof(double)) {
      if (A.traj_f) {
        // FP64 redo: the final nominal, rounded, into the float region the
        // backward reads
        const R* src = traj_at<R>(A, G.b, n, 0);
        float* dst = A.traj_f + ((size_t)G.b * NSLOT + n) * A.Tm * ZS;
        for (int i = l; i < G.T * ZS; i += 16) dst[i] = (float)src[i];
        st |= ST_REDONE;
      }
    }
    grp_write_state(A, G, n, iters, st, 1);
    if (l == 0) A.status[G.b] = st | ((uint32_t)iters << DMPC_ST_ITERS_SHIFT);
  }
}

// FP64 redo: resets the redo list's count and queue counter
__global__ void k_reset_redo(int* count, int* queue) {
  if (threadIdx.x == 0) {
    *count = 0;
    *queue = 0;
  }
}

// FP64 redo: the instances whose control block had a pivot below the
// threshold, in any order (each instance's result does not depend on the
// wave that solves it)
__global__ __launch_bounds__(256) void k_redo_list(const uint32_t* status, int B, int* list, int* count) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b < B && (status[b] & ST_FP64)) list[atomicAdd(count, 1)] = b;
}

__global__ void k_reset_queue(int* queue) {
  if (threadIdx.x == 0) *queue = 0;
}

// counting sort of the instances by decreasing horizon (one workgroup)
__global__ __launch_bounds__(1024) void k_sort_by_T(const int* T, int B, int Tm, int* order, int* queue) {
  __shared__ int cnt[DMPC_T_LIMIT + 2];
  for (int i = threadIdx.x; i <= Tm + 1; i += blockDim.x) cnt[i] = 0;
  __syncthreads();
  for (int b = threadIdx.x; b < B; b += blockDim.x) {
    int t = T[b];
    t = t < 0 ? 0 : (t > Tm ? Tm : t);
    atomicAdd(&cnt[t], 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int t = Tm; t >= 0; --t) {
      const int c = cnt[t];
      cnt[t] = run;
      run += c;
    }
    *queue = 0;
  }
  __syncthreads();
  for (int b = threadIdx.x; b < B; b += blockDim.x) {
    int t = T[b];
    t = t < 0 ? 0 : (t > Tm ? Tm : t);
    order[atomicAdd(&cnt[t], 1)] = b;
  }
}

// ---------------------------------------------------------------------------
// per-launch form
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(64) void k_plain_init(KArgs A) {
  const int lane = threadIdx.x, l = lane & 15;
  const Grp G = make_grp(A, blockIdx.x * 4 + (lane >> 4), l);
  if (!G.valid) return;
  if (G.T > 0) grp_init(A, G);
  grp_write_state(A, G, 0, 0, 0u, G.T > 0 ? 0 : 1);
  if (A.tpar) {
    // first pattern guess: a control of U^0 equal to a bound is clamped there
    // (a shifted warm start keeps the clamps of the solution it came from)
    mem_fence_wg();
    if (l == 0) A.ws.state[(size_t)G.b * SW + S_FB] = 0;
    for (int t = l; t < A.Tm; t += 16) {
      unsigned code = 0;
      if (t < G.T) {
        const float* zp = traj_at(A, G.b, 0, t);
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const float u = zp[16 + a];
          code |= (u == G.lo[a] ? 1u : (u == G.hi[a] ? 2u : 0u)) << (2 * a);
        }
      }
      A.ws.pat[(size_t)G.b * A.Tm + t] = (uint8_t)code;
    }
  }
}

// linearisation of every stage along the nominal: one 16-lane row per (b, t)
__global__ __launch_bounds__(64) void k_plain_lin(KArgs A, int tail) {
  const int lane = threadIdx.x, l = lane & 15, col = (l == 0) ? 16 : l;
  const long long unit = (long long)blockIdx.x * 4 + (lane >> 4);
  if (unit >= (long long)A.B * A.Tm) return;
  const int b = (int)(unit / A.Tm), t = (int)(unit % A.Tm);
  const int* s = A.ws.state + (size_t)b * SW;
  const int T = s[S_T];
  if (t + 1 >= T) return;
  if (!tail && s[S_DONE]) return;
  const int n = s[S_NOM];
  float zb[NZ], Fc[NX];
  load_z(traj_at(A, b, n, t), zb);
  const LaneDir D = make_dir(A.P, col);
  rk4_column(A.P, zb, zb + NX, D, Fc);
  float* fp = lin_at(A, b, t) + col * 16;
#pragma unroll
  for (int k = 0; k < NX; ++k) fp[k] = Fc[k];
}

template <bool DENSE, int MODE>
__global__ __launch_bounds__(64) void k_plain_riccati(KArgs A) {
  __shared__ double lds[4 * L_REG];
  const int lane = threadIdx.x, l = lane & 15;
  double* L = lds + (lane >> 4) * L_REG;
  const Grp G = make_grp(A, blockIdx.x * 4 + (lane >> 4), l);
  if (!G.valid || G.T == 0) return;
  int* s = A.ws.state + (size_t)G.b * SW;
  if (MODE == 0 && s[S_DONE]) return;
  // with the time-parallel Riccati this sweep runs only where its pattern check failed
  if (MODE == 0 && A.tpar && !s[S_FB]) return;
  uint32_t st = 0;
  grp_sweep<DENSE, MODE, false>(A, G, s[S_NOM], s[S_ITERS], L, st, G.T);
  mem_fence_wg();
  if (l == 0 && st) atomicOr((unsigned*)&s[S_STATUS], st);
  if (MODE == 0 && A.tpar && l == 0) s[S_FB] = 0;
}

template <bool DENSE>
__global__ __launch_bounds__(64) void k_plain_ls(KArgs A) {
  const int lane = threadIdx.x, l = lane & 15;
  const Grp G = make_grp(A, blockIdx.x * 4 + (lane >> 4), l);
  if (!G.valid || G.T == 0) return;
  int* s = A.ws.state + (size_t)G.b * SW;
  if (s[S_DONE]) return;
  const int n = s[S_NOM], k = s[S_ITERS];
  float J, dm, dsel;
  grp_ls<DENSE>(A, G, n, J, dm);
  mem_fence_wg();
  const int best = ls_select(J, dm, dsel);
  if (l == 0) {
    if (A.dlog) A.dlog[((size_t)G.b * A.K + k) * (1 + A.Tm)] = best < 0 ? 255 : (uint8_t)best;
    uint32_t st = (uint32_t)s[S_STATUS];
    int done = 0, nn = n;
    if (best < 0) {
      st |= ST_NONFINITE;
    } else {
      nn = (n + 1 + best) % NSLOT;
      if (A.tol > 0.f && dsel < A.tol) {
        st |= ST_CONVERGED;
        done = 1;
      }
    }
    s[S_NOM] = nn;
    s[S_ITERS] = k + 1;
    s[S_STATUS] = (int)st;
    s[S_DONE] = done;
  }
}

__global__ __launch_bounds__(64) void k_plain_finalize(KArgs A) {
  const int lane = threadIdx.x, l = lane & 15;
  const Grp G = make_grp(A, blockIdx.x * 4 + (lane >> 4), l);
  if (!G.valid) return;
  int* s = A.ws.state + (size_t)G.b * SW;
  const int n = s[S_NOM], iters = s[S_ITERS];
  uint32_t st = (uint32_t)s[S_STATUS];
  if (A.tol > 0.f && G.T > 0 && !(st & ST_CONVERGED)) st |= ST_MAXITER;
  grp_outputs(A, G, n);
  mem_fence_wg();
  if (l == 0) {
    s[S_STATUS] = (int)st;
    s[S_DONE] = 1;
    A.status[G.b] = st | ((uint32_t)iters << DMPC_ST_ITERS_SHIFT);
  }
}

// ---------------------------------------------------------------------------
// time-parallel Riccati (per-launch form with DMPC_TPAR)
//
// The backward pass of one iteration solves, for a given clamp pattern, the
// LQ problem in deviations from the nominal: dx' = A dx + B du, stage cost
// 1/2 dz^T C dz + g^T dz (g = C z_bar + c), clamped controls held at their
// bound.  Its value functions V_t(dx) = 1/2 dx^T V_t dx + v_t^T dx are suffix
// products of one element per stage under an associative combination (the
// conditional value functions of Saerkkae and Garcia-Fernandez's temporal
// parallelisation of dynamic programming, the associative-scan route the
// paper cites as the alternative to the serial recursion in time):
//   element t:  (A, b, C, eta, J) with V_{t->t+1}(x, y) = 1/2 x^T J x - eta^T x
//               + 1/2 w^T C^+ w for y = A x + b + w, w in range(C)
//   (i then j): A = A_j M^-1 A_i,  b = A_j M^-1 (b_i + C_i eta_j) + b_j,
//               C = A_j M^-1 C_i A_j^T + C_j,
//               eta = A_i^T M^-T (eta_j - J_j b_i) + eta_i,
//               J = A_i^T M^-T J_j A_i + J_i,      M = I + C_i J_j,
// and the last stage's element is terminal (A = 0, b = 0, C = 0), so the
// suffix product from t holds V_t = J and v_t = -eta.  The element of stage
// t < T-1 removes the cross term and the clamped controls from the stage:
// with R = C_ff (free controls f, clamped c held at k_c),
//   r = C_fc k_c + g_f,  J = C_xx - C_xf R^-1 C_fx,
//   eta = -(g_x + C_xc k_c - C_xf R^-1 r),  A = A_t - B_f R^-1 C_fx,
//   b = B_c k_c - B_f R^-1 r,  C = B_f R^-1 B_f^T.
// The clamp pattern is not known before V_{t+1} is: each iteration takes the
// previous iteration's pattern (free at the first), and the gains kernel
// re-solves every stage's box-QP with the scanned V_{t+1}.  If every stage
// reproduces the assumed pattern, then by induction from the last stage the
// serial recursion would have taken the same decisions and computed the same
// V (up to rounding); otherwise the instance is flagged and its serial sweep
// runs instead.  One wavefront per (instance, stage); FP64 throughout.
// ---------------------------------------------------------------------------

constexpr int SCAN_NT = 256;  // threads per combination
constexpr int EL_A = 0, EL_B = 169, EL_C = 182, EL_E = 351, EL_J = 364, EL_W = 536;  // doubles per element

__device__ __forceinline__ double* elem_at(const KArgs& A, int buf, int b, int t) {
  return A.ws.elem + (((size_t)buf * A.B + b) * A.Tm + t) * EL_W;
}

// value of v in lane `lane` (a wave-uniform index) of the wavefront
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)bits, lane);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// out = op(X) op(Y) for 13 x 13 row-major matrices in LDS (tX / tY
// transpose), outputs spread over the NT threads of the block
template <int NT>
__device__ __forceinline__ void lds_mm(double* out, const double* X, const double* Y, bool tX, bool tY) {
  for (int idx = threadIdx.x; idx < 169; idx += NT) {
    const int r = idx / 13, c = idx % 13;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 13; ++k) s = fma(tX ? X[k * 13 + r] : X[r * 13 + k], tY ? Y[c * 13 + k] : Y[k * 13 + c], s);
    out[idx] = s;
  }
  __syncthreads();
}

// out = op(X) y for a 13 x 13 matrix and a 13-vector
__device__ __forceinline__ void lds_mv(double* out, const double* X, const double* y, bool tX) {
  if (threadIdx.x < 13) {
    const int r = threadIdx.x;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 13; ++k) s = fma(tX ? X[k * 13 + r] : X[r * 13 + k], y[k], s);
    out[r] = s;
  }
  __syncthreads();
}

// masked inverse of the free block of a symmetric positive definite 4 x 4
// matrix (zero rows and columns on clamped controls), by Gauss-Jordan on the
// free block with the clamped rows replaced by identity (no pivoting is needed
// for a positive definite block); every thread computes it
__device__ __forceinline__ void masked_inv4(const double* H, const bool* fr, double* M) {
  double a[4][8];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) a[i][j] = (j < 4) ? ((fr[i] && fr[j]) ? H[i * 4 + j] : (i == j ? 1.0 : 0.0))
                                                  : ((j - 4) == i ? 1.0 : 0.0);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double ip = 1.0 / a[k][k];
#pragma unroll
    for (int j = 0; j < 8; ++j) a[k][j] *= ip;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (r == k) continue;
      const double f = a[r][k];
#pragma unroll
      for (int j = 0; j < 8; ++j) a[r][j] = fma(-f, a[k][j], a[r][j]);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) M[i * 4 + j] = (fr[i] && fr[j]) ? a[i][4 + j] : 0.0;
}

// stage cost matrix C_t (17 x 17, LDS) and g_t = C_t z_bar + c_t
template <bool DENSE>
__device__ __forceinline__ void stage_cost_lds(const KArgs& A, size_t srow, const float* zb, double* C, double* g) {
  for (int idx = threadIdx.x; idx < NZ * NZ; idx += 64) {
    const int i = idx / NZ, j = idx % NZ;
    double v;
    if (DENSE) v = (double)A.Q[srow * NPK + (i <= j ? pidx(i, j) : pidx(j, i))];
    else v = (i == j) ? (double)A.Q[srow * NZ + i] : 0.0;
    C[idx] = v;
  }
  __syncthreads();
  if (threadIdx.x < NZ) {
    const int i = threadIdx.x;
    double s = (double)A.p[srow * NZ + i];
#pragma unroll
    for (int j = 0; j < NZ; ++j) s = fma(C[i * NZ + j], (double)zb[j], s);
    g[i] = s;
  }
  __syncthreads();
}

// F = [A | B] of stage t (13 x 17, LDS, row-major) from the linearisation
// buffer; column 0 (position x) is e_0 exactly and is not stored there
__device__ __forceinline__ void load_F(const KArgs& A, int b, int t, double* F) {
  const float* fp = lin_at(A, b, t);
  for (int idx = threadIdx.x; idx < NX * NZ; idx += 64) {
    const int r = idx / NZ, c = idx % NZ;
    F[idx] = (c == 0) ? (r == 0 ? 1.0 : 0.0) : (double)fp[c * 16 + r];
  }
  __syncthreads();
}

// tail != 0: the fixed-mask problem at the solution (controls equal to a bound
// held there), for every instance whether it has converged or not
template <bool DENSE>
__global__ __launch_bounds__(64) void k_tpar_elem(KArgs A, int tail) {
  __shared__ double C[NZ * NZ], F[NX * NZ], g[NZ], T1[NX * 4], W[NX * 4];
  const int unit = blockIdx.x, b = unit / A.Tm, t = unit % A.Tm;
  const int* s = A.ws.state + (size_t)b * SW;
  const int T = s[S_T];
  if (t >= T || (!tail && s[S_DONE])) return;
  const size_t srow = (size_t)b * A.Tm + t;
  const int n = s[S_NOM];
  float zb[NZ];
  load_z(traj_at(A, b, n, t), zb);
  const bool term = (t + 1 == T);
  stage_cost_lds<DENSE>(A, srow, zb, C, g);
  if (!term) load_F(A, b, t, F);
  // assumed pattern: free, or clamped at the lower / upper bound
  unsigned code = 0;
  if (tail) {
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const float u = zb[NX + a];
      code |= (u == A.lo[(size_t)b * 4 + a] ? 1u : (u == A.hi[(size_t)b * 4 + a] ? 2u : 0u)) << (2 * a);
    }
  } else {
    code = A.ws.pat[srow];
  }
  bool fr[4];
  double kc[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const unsigned c = (code >> (2 * a)) & 3u;
    fr[a] = (c == 0);
    const double lo = (double)A.lo[(size_t)b * 4 + a] - (double)zb[NX + a];
    const double hi = (double)A.hi[(size_t)b * 4 + a] - (double)zb[NX + a];
    kc[a] = (c == 0) ? 0.0 : (c == 1 ? lo : hi);
  }
  double Ruu[16], iR[16];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) Ruu[i * 4 + j] = C[(NX + i) * NZ + NX + j];
  masked_inv4(Ruu, fr, iR);
  // r = C_fc k_c + g_f on the free controls (0 on clamped ones)
  double r[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    double v = g[NX + a];
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) v = fma(fr[bb] ? 0.0 : Ruu[a * 4 + bb], kc[bb], v);
    r[a] = fr[a] ? v : 0.0;
  }
  // T1 = C_xu R^-1 (13 x 4) and W = B R^-1 (13 x 4), free columns only
  if (threadIdx.x < NX) {
    const int i = threadIdx.x;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      double s1 = 0.0, s2 = 0.0;
#pragma unroll
      for (int bb = 0; bb < 4; ++bb) {
        s1 = fma(C[i * NZ + NX + bb], iR[bb * 4 + a], s1);
        if (!term) s2 = fma(F[i * NZ + NX + bb], iR[bb * 4 + a], s2);
      }
      T1[i * 4 + a] = s1;
      W[i * 4 + a] = s2;
    }
  }
  __syncthreads();
  double* E = elem_at(A, 0, b, t);
  for (int idx = threadIdx.x; idx < 169; idx += 64) {
    const int i = idx / 13, j = idx % 13;
    // J = C_xx - C_xu R^-1 C_ux, symmetrised
    double Jv = C[i * NZ + j], Jw = C[j * NZ + i], Av = 0.0, Cv = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      Jv = fma(-T1[i * 4 + a], C[(NX + a) * NZ + j], Jv);
      Jw = fma(-T1[j * 4 + a], C[(NX + a) * NZ + i], Jw);
    }
    Jv = 0.5 * (Jv + Jw);
    if (!term) {
      Av = F[i * NZ + j];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        Av = fma(-W[i * 4 + a], C[(NX + a) * NZ + j], Av);
        Cv = fma(W[i * 4 + a], F[j * NZ + NX + a], Cv);
      }
    }
    E[EL_J + idx] = Jv;
    E[EL_A + idx] = Av;
    E[EL_C + idx] = Cv;
  }
  if (threadIdx.x < NX) {
    const int i = threadIdx.x;
    // eta = -(g_x + C_xc k_c - C_xu R^-1 r),  b = B_c k_c - B R^-1 r
    double q = g[i], bv = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      q = fma(fr[a] ? 0.0 : C[i * NZ + NX + a], kc[a], q);
      q = fma(-T1[i * 4 + a], r[a], q);
      if (!term) {
        bv = fma(fr[a] ? 0.0 : F[i * NZ + NX + a], kc[a], bv);
        bv = fma(-W[i * 4 + a], r[a], bv);
      }
    }
    E[EL_E + i] = -q;
    E[EL_B + i] = bv;
  }
}

// one level of the suffix scan: out[t] = in[t] (x) in[t + step] (or in[t]);
// one NT-thread block per (instance, stage)
template <int NT>
__global__ __launch_bounds__(NT) void k_tpar_scan(KArgs A, int step, int src, int tail) {
  __shared__ double Ai[169], Ci[169], Ji[169], Aj[169], Cj[169], Jj[169], bi[13], ei[13], bj[13], ej[13];
  __shared__ double X1[169], X2[169], X3[169], v1[13], v2[13];
  const int tid = threadIdx.x;
  const int unit = blockIdx.x, b = unit / A.Tm, t = unit % A.Tm;
  const int* s = A.ws.state + (size_t)b * SW;
  const int T = s[S_T];
  if (t >= T || (!tail && s[S_DONE])) return;
  const double* ein = elem_at(A, src, b, t);
  double* eout = elem_at(A, 1 - src, b, t);
  if (t + step >= T) {
    for (int k = tid; k < EL_W; k += NT) eout[k] = ein[k];
    return;
  }
  const double* ejn = elem_at(A, src, b, t + step);
  for (int k = tid; k < 169 + 13; k += NT) {
    if (k < 169) {
      Ai[k] = ein[EL_A + k];
      Ci[k] = ein[EL_C + k];
      Ji[k] = ein[EL_J + k];
      Aj[k] = ejn[EL_A + k];
      Cj[k] = ejn[EL_C + k];
      Jj[k] = ejn[EL_J + k];
    } else {
      const int m = k - 169;
      bi[m] = ein[EL_B + m];
      ei[m] = ein[EL_E + m];
      bj[m] = ejn[EL_B + m];
      ej[m] = ejn[EL_E + m];
    }
  }
  __syncthreads();
  // M = I + C_i J_j (X1 holds C_i J_j)
  lds_mm<NT>(X1, Ci, Jj, false, false);
  // X2 = M^-1 by Gauss-Jordan on [M | I] in the registers of the first wave,
  // one row per lane (lanes 0..12), with implicit partial pivoting: the pivot
  // row of step k stays in its lane and reaches the others by readlane, and
  // no rows move; at the end the lane that was pivot at step k holds row k of
  // M^-1.  No barrier inside the elimination.
  if (tid < 64) {
    const int r = tid;
    double a[26];
#pragma unroll
    for (int c = 0; c < 26; ++c) {
      double v = 0.0;
      if (r < 13) v = (c < 13) ? X1[r * 13 + c] + (r == c ? 1.0 : 0.0) : ((c - 13) == r ? 1.0 : 0.0);
      a[c] = v;
    }
    bool used = (r >= 13);
    int mystep = 0;
#pragma unroll
    for (int k = 0; k < 13; ++k) {
      const double cand = used ? -1.0 : fabs(a[k]);
      int p = 0;
      double best = -2.0;
#pragma unroll
      for (int q = 0; q < 13; ++q) {
        const double vq = readlane_f64(cand, q);
        const bool take = vq > best;
        best = take ? vq : best;
        p = take ? q : p;
      }
      p = __builtin_amdgcn_readfirstlane(p);
      double pr[26];
#pragma unroll
      for (int c = 0; c < 26; ++c) pr[c] = readlane_f64(a[c], p);
      const double ip = rcp_nr(pr[k]);
      const double f = a[k] * ip;
      const bool piv = (r == p);
#pragma unroll
      for (int c = 0; c < 26; ++c) a[c] = piv ? pr[c] * ip : fma(-f, pr[c], a[c]);
      mystep = piv ? k : mystep;
      used = used || piv;
    }
    if (r < 13) {
#pragma unroll
      for (int c = 0; c < 13; ++c) X2[mystep * 13 + c] = a[13 + c];
    }
  }
  __syncthreads();
  // b = A_j M^-1 (b_i + C_i eta_j) + b_j
  lds_mv(v1, Ci, ej, false);
  if (tid < 13) v1[tid] += bi[tid];
  __syncthreads();
  lds_mv(v2, X2, v1, false);
  lds_mv(v1, Aj, v2, false);
  if (tid < 13) eout[EL_B + tid] = v1[tid] + bj[tid];
  // eta = A_i^T M^-T (eta_j - J_j b_i) + eta_i
  lds_mv(v1, Jj, bi, false);
  if (tid < 13) v1[tid] = ej[tid] - v1[tid];
  __syncthreads();
  lds_mv(v2, X2, v1, true);
  lds_mv(v1, Ai, v2, true);
  if (tid < 13) eout[EL_E + tid] = v1[tid] + ei[tid];
  // A = A_j M^-1 A_i
  lds_mm<NT>(X1, X2, Ai, false, false);
  lds_mm<NT>(X3, Aj, X1, false, false);
  for (int k = tid; k < 169; k += NT) eout[EL_A + k] = X3[k];
  // C = A_j M^-1 C_i A_j^T + C_j (symmetrised)
  lds_mm<NT>(X1, X2, Ci, false, false);
  lds_mm<NT>(X3, Aj, X1, false, false);
  lds_mm<NT>(X1, X3, Aj, false, true);
  for (int k = tid; k < 169; k += NT) {
    const int r = k / 13, c = k % 13;
    eout[EL_C + k] = 0.5 * (X1[k] + X1[c * 13 + r]) + Cj[k];
  }
  // J = A_i^T M^-T J_j A_i + J_i (symmetrised)
  lds_mm<NT>(X3, Jj, Ai, false, false);  // J_j A_i
  lds_mm<NT>(X1, X2, X3, true, false);   // M^-T J_j A_i
  lds_mm<NT>(X3, Ai, X1, true, false);   // A_i^T M^-T J_j A_i
  for (int k = tid; k < 169; k += NT) {
    const int r = k / 13, c = k % 13;
    eout[EL_J + k] = 0.5 * (X3[k] + X3[c * 13 + r]) + Ji[k];
  }
}

// gains of every stage from the scanned V_{t+1}: Q = C + F^T V F,
// q = g + F^T v, the stage's box-QP, K = -Q_ff^-1 Q_fx; the pattern is
// checked against the one the elements assumed
template <bool DENSE>
__global__ __launch_bounds__(64) void k_tpar_gains(KArgs A, int src) {
  __shared__ double C[NZ * NZ], F[NX * NZ], g[NZ], V[169], v[13], Y[NX * NZ], Q[NZ * NZ], q[NZ];
  const int unit = blockIdx.x, b = unit / A.Tm, t = unit % A.Tm;
  int* s = A.ws.state + (size_t)b * SW;
  const int T = s[S_T];
  if (t >= T || s[S_DONE]) return;
  const int kit = s[S_ITERS], n = s[S_NOM];
  const size_t srow = (size_t)b * A.Tm + t;
  float zb[NZ];
  load_z(traj_at(A, b, n, t), zb);
  stage_cost_lds<DENSE>(A, srow, zb, C, g);
  const bool has_dyn = (t + 1 < T);
  if (has_dyn) {
    load_F(A, b, t, F);
    const double* E = elem_at(A, src, b, t + 1);
    for (int k = threadIdx.x; k < 169; k += 64) V[k] = E[EL_J + k];
    if (threadIdx.x < 13) v[threadIdx.x] = -E[EL_E + threadIdx.x];
    __syncthreads();
    // Y = V F (13 x 17)
    for (int idx = threadIdx.x; idx < NX * NZ; idx += 64) {
      const int r = idx / NZ, c = idx % NZ;
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < NX; ++k) acc = fma(V[r * 13 + k], F[k * NZ + c], acc);
      Y[idx] = acc;
    }
    __syncthreads();
  }
  // Q = C + F^T Y, q = g + F^T v
  for (int idx = threadIdx.x; idx < NZ * NZ; idx += 64) {
    const int r = idx / NZ, c = idx % NZ;
    double acc = C[idx];
    if (has_dyn) {
#pragma unroll
      for (int k = 0; k < NX; ++k) acc = fma(F[k * NZ + r], Y[k * NZ + c], acc);
    }
    Q[idx] = acc;
  }
  if (threadIdx.x < NZ) {
    const int r = threadIdx.x;
    double acc = g[r];
    if (has_dyn) {
#pragma unroll
      for (int k = 0; k < NX; ++k) acc = fma(F[k * NZ + r], v[k], acc);
    }
    q[r] = acc;
  }
  __syncthreads();
  double H[16], qu[4], dl[4], dh[4], kw[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int a = 0; a < 4; ++a) {
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) H[a * 4 + bb] = 0.5 * (Q[(NX + a) * NZ + NX + bb] + Q[(NX + bb) * NZ + NX + a]);
    qu[a] = q[NX + a];
    dl[a] = (double)A.lo[(size_t)b * 4 + a] - (double)zb[NX + a];
    dh[a] = (double)A.hi[(size_t)b * 4 + a] - (double)zb[NX + a];
  }
  float* gp = gains_at(A, b, t);
  if (kit > 0) {
    const float4 w = *(const float4*)(gp + 64);
    kw[0] = w.x; kw[1] = w.y; kw[2] = w.z; kw[3] = w.w;
  }
  __syncthreads();  // every thread has read the previous feedforward before it is overwritten
  double kv[4], fr[4];
  Fact4 Ch;
  uint32_t st = 0;
  boxqp(H, qu, dl, dh, kw, A.piv, kv, fr, Ch, st);
  unsigned code = 0;
#pragma unroll
  for (int a = 0; a < 4; ++a) code |= ((fr[a] != 0.0) ? 0u : (kv[a] <= dl[a] ? 1u : 2u)) << (2 * a);
  if (threadIdx.x < NX) {
    const int c = threadIdx.x;
    double Kd[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) Kd[a] = fr[a] * 0.5 * (Q[(NX + a) * NZ + c] + Q[c * NZ + NX + a]);
    solve4(Ch, Kd);
#pragma unroll
    for (int a = 0; a < 4; ++a) gp[a * 16 + c] = (float)(-Kd[a]);
  }
  if (threadIdx.x == 0) {
    *(float4*)(gp + 64) = make_float4((float)kv[0], (float)kv[1], (float)kv[2], (float)kv[3]);
    if (A.dlog) A.dlog[((size_t)b * A.K + kit) * (1 + A.Tm) + 1 + t] = (uint8_t)code;
    if (code != A.ws.pat[srow]) atomicOr(&s[S_FB], 1);
    A.ws.pat[srow] = (uint8_t)code;
    if (st) atomicOr(&s[S_STATUS], (int)st);
  }
}

// forward tail from the scanned value functions: the stage factors the
// backward reads (F, K, masked inverse of the free control block), with the
// controls that equal a bound held fixed, as the serial tail sweep stores them
template <bool DENSE>
__global__ __launch_bounds__(64) void k_tpar_tail(KArgs A, int src) {
  __shared__ double C[NZ * NZ], F[NX * NZ], g[NZ], V[169], Y[NX * NZ], Q[NZ * NZ];
  const int unit = blockIdx.x, b = unit / A.Tm, t = unit % A.Tm;
  int* s = A.ws.state + (size_t)b * SW;
  const int T = s[S_T];
  if (t >= T) return;
  const int n = s[S_NOM];
  const size_t srow = (size_t)b * A.Tm + t;
  float zb[NZ];
  load_z(traj_at(A, b, n, t), zb);
  stage_cost_lds<DENSE>(A, srow, zb, C, g);
  const bool has_dyn = (t + 1 < T);
  if (has_dyn) {
    load_F(A, b, t, F);
    const double* E = elem_at(A, src, b, t + 1);
    for (int k = threadIdx.x; k < 169; k += 64) V[k] = E[EL_J + k];
    __syncthreads();
    for (int idx = threadIdx.x; idx < NX * NZ; idx += 64) {
      const int r = idx / NZ, c = idx % NZ;
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < NX; ++k) acc = fma(V[r * 13 + k], F[k * NZ + c], acc);
      Y[idx] = acc;
    }
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < NZ * NZ; idx += 64) {
    const int r = idx / NZ, c = idx % NZ;
    double acc = C[idx];
    if (has_dyn) {
#pragma unroll
      for (int k = 0; k < NX; ++k) acc = fma(F[k * NZ + r], Y[k * NZ + c], acc);
    }
    Q[idx] = acc;
  }
  __syncthreads();
  double H[16], fr[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) H[a * 4 + bb] = 0.5 * (Q[(NX + a) * NZ + NX + bb] + Q[(NX + bb) * NZ + NX + a]);
    const float u = zb[NX + a];
    fr[a] = (u == A.lo[(size_t)b * 4 + a] || u == A.hi[(size_t)b * 4 + a]) ? 0.0 : 1.0;
  }
  Fact4 Ch;
  uint32_t st = 0;
  ldl4(H, fr, A.piv, Ch, st);
  float* tp = tail_at(A, b, t);
  for (int idx = threadIdx.x; idx < NZ * NX; idx += 64) {
    const int c = idx / NX, r = idx % NX;
    tp[c * 16 + r] = has_dyn ? (float)F[r * NZ + c] : 0.f;
  }
  if (threadIdx.x < NX) {
    const int c = threadIdx.x;
    double Kd[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) Kd[a] = fr[a] * 0.5 * (Q[(NX + a) * NZ + c] + Q[c * NZ + NX + a]);
    solve4(Ch, Kd);
    *(float4*)(tp + FS + c * 4) = make_float4((float)(-Kd[0]), (float)(-Kd[1]), (float)(-Kd[2]), (float)(-Kd[3]));
  }
  if (threadIdx.x == NX) {
    double M[16];
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) {
      double e[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) e[a] = (a == bb) ? fr[bb] : 0.0;
      solve4(Ch, e);
#pragma unroll
      for (int a = 0; a < 4; ++a) M[a * 4 + bb] = fr[a] * e[a];
    }
    double* mp = (double*)(tp + FS + 52);
#pragma unroll
    for (int i = 0; i < 16; i += 2) *(double2*)(mp + i) = make_double2(M[i], M[i + 1]);
  }
  if (threadIdx.x == 0 && st) atomicOr(&s[S_STATUS], (int)st);
}

// ---------------------------------------------------------------------------
// backward: Riccati adjoint at (x*, u*) with the forward's active set
// ---------------------------------------------------------------------------

// (i, j) of packed-upper entry m, row by row.  Initialised in the code
// object itself, so every device the library runs on holds its own copy from
// load time on, with nothing to upload.
struct PackTable {
  uint8_t i[NPK], j[NPK];
};
constexpr PackTable make_pack_table() {
  PackTable t{};
  int m = 0;
  for (int i = 0; i < NZ; ++i)
    for (int j = i; j < NZ; ++j) {
      t.i[m] = (uint8_t)i;
      t.j[m] = (uint8_t)j;
      ++m;
    }
  return t;
}
__constant__ PackTable c_pk = make_pack_table();

// The stage factors (F_t, K_t, masked inverse) come from the forward's tail.
// With checkpointing (CKPT) only V, v at the stages j * ckpt were kept: the
// horizon is cut into segments of ckpt stages and each segment's factors are
// recomputed from its end checkpoint by the tail sweep, last segment first for
// the backward vector sweep and first segment first for the forward sweep.
// The checkpoint is the exact FP64 state of the forward's sweep, so the
// recomputed factors are the ones the forward would have stored.
template <bool DENSE, bool CKPT, bool THETA, class R = float>
__global__ __launch_bounds__(64) void k_bwd(KArgs A) {
  __shared__ float zz[4][2][20];
  __shared__ double lds[CKPT ? 4 * L_REG : 2];
  const int lane = threadIdx.x, grp = lane >> 4, l = lane & 15, col = (l == 0) ? 16 : l;
  const int b = blockIdx.x * 4 + grp;
  if (b >= A.B) return;
  const int* s = A.ws.state + (size_t)b * SW;
  const int T = s[S_T], n = s[S_NOM], Tm = A.Tm;
  const int W = DENSE ? NPK : NZ;
  const int seg = CKPT ? A.ckpt : (T > 0 ? T : 1);
  const int nseg = (T + seg - 1) / seg;
  Grp G;
  double* L = lds + (CKPT ? grp * L_REG : 0);
  if (CKPT) {
    G.b = b;
    G.T = T;
    G.l = l;
    G.col = col;
    G.valid = true;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      G.lo[a] = A.lo[(size_t)b * 4 + a];
      G.hi[a] = A.hi[(size_t)b * 4 + a];
    }
  }
  // factors of stages [a, e) into the tail at index t - a
  auto recompute = [&](int a, int e) {
    uint32_t st = 0;
    const double* vinit = (e < T) ? A.ws.ck + ((size_t)b * A.nck + (e / seg - 1)) * CK_W : nullptr;
    grp_sweep<DENSE, 1, true, R>(A, G, n, 0, L, st, e, a, vinit, a);
    mem_fence_wg();
  };
  // backward vector sweep: q~ = d + F^T v, k~ = -M q~_u, v = q~_x + K^T q~_u.
  // Each stage's factors are loaded one stage ahead (they do not depend on
  // the recursion); lane l < 13 carries v_l.
  struct VStage {
    float fc[NX];
    float dc, d0;
    double M[16];
    float4 kc;
  };
  auto vload = [&](int t, int a0, VStage& S) {
    const float* tp = tail_at(A, b, CKPT ? t - a0 : t);
    const size_t srow = (size_t)b * Tm + t;
    // one load per value from a selected address (dL/du* stands in for an
    // absent dL/dx*), so that no branch surrounds the loads
    const float* gur = A.gu + srow * NU;
    const float* gxr = A.gx ? A.gx + srow * NX : gur;
    const float vdc = *((col < NX) ? gxr + (A.gx ? col : 0) : gur + (col - NX));
    const float vd0 = *gxr;
    S.dc = (col < NX && !A.gx) ? 0.f : vdc;
    S.d0 = A.gx ? vd0 : 0.f;
    const float* fc = tp + col * 16;
    const float4 f0 = *(const float4*)(fc), f1 = *(const float4*)(fc + 4), f2 = *(const float4*)(fc + 8);
    S.fc[0] = f0.x; S.fc[1] = f0.y; S.fc[2] = f0.z; S.fc[3] = f0.w;
    S.fc[4] = f1.x; S.fc[5] = f1.y; S.fc[6] = f1.z; S.fc[7] = f1.w;
    S.fc[8] = f2.x; S.fc[9] = f2.y; S.fc[10] = f2.z; S.fc[11] = f2.w;
    S.fc[12] = fc[12];
    const double2* mp = (const double2*)(tp + FS + 52);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const double2 w = mp[i];
      S.M[2 * i] = w.x;
      S.M[2 * i + 1] = w.y;
    }
    S.kc = *(const float4*)(tp + FS + (l < NX ? l : 0) * 4);
  };
  double vi = 0.0;
  // one stage of the sweep from cs, the next stage's factors loaded into ns
  auto vstep = [&](int t, int a, const VStage& cs, VStage& ns) {
    vload(t > a ? t - 1 : t, a, ns);  // at the segment's first stage, this one's again
    const size_t srow = (size_t)b * Tm + t;
    double Fd[NX];
#pragma unroll
    for (int k = 0; k < NX; ++k) Fd[k] = (double)cs.fc[k];
    double qc = (double)cs.dc;
    fv_chain(qc, vi, Fd);
    const double q0 = (double)cs.d0 + bc<0>(vi);
    double qu[4];
#pragma unroll
    for (int a4 = 0; a4 < 4; ++a4) qu[a4] = rb64(qc, lane_of(NX + a4));
    double kt[4];
#pragma unroll
    for (int a4 = 0; a4 < 4; ++a4) {
      double acc = 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) acc = fma(cs.M[a4 * 4 + c], qu[c], acc);
      kt[a4] = -acc;
    }
    // every lane of the instance writes the same k~ (no branch around the store)
    *(float4*)(A.ws.ktil + srow * 4) = make_float4((float)kt[0], (float)kt[1], (float)kt[2], (float)kt[3]);
    double vn = (l == 0) ? q0 : qc;
    vn = fma((double)cs.kc.x, qu[0], vn);
    vn = fma((double)cs.kc.y, qu[1], vn);
    vn = fma((double)cs.kc.z, qu[2], vn);
    vn = fma((double)cs.kc.w, qu[3], vn);
    vi = (l < NX) ? vn : 0.0;
  };
  VStage s0, s1;
  for (int sg = nseg - 1; sg >= 0; --sg) {
    const int a = sg * seg, e = (a + seg < T) ? a + seg : T;
    if (CKPT) recompute(a, e);
    vload(e - 1, a, s0);
    __builtin_amdgcn_s_waitcnt(0);  // no load pending on loop entry (see grp_ls)
    // two stages per trip with the stage records swapping roles, so that
    // nothing is copied from one stage to the next
    for (int t = e - 1; t >= a; t -= 2) {
      vstep(t, a, s0, s1);
      if (t - 1 < a) break;
      vstep(t - 1, a, s1, s0);
    }
  }
  if (l < NX) A.gx0[(size_t)b * NX + l] = (T > 0) ? (float)vi : 0.f;
  mem_fence_wg();  // k~ written by lane 0 above is read by every lane below
  // forward sweep: u~ = K x~ + k~, x~' = A x~ + B u~;  dL/dc = z~, dL/dC from z~ and z*
  struct FStage {
    float4 kk;
    float4 K[NX];
    float zs[NZ];
    float fr[NZ];
    float crow[DENSE ? NZ : 1];  // row l of C_t (THETA)
    float cl, gl;                // c_t and dL/dx*_t at row l (THETA)
  };
  auto fload = [&](int t, int a0, FStage& S) {
    const float* tp = tail_at(A, b, CKPT ? t - a0 : t);
    const size_t srow = (size_t)b * Tm + t;
    S.kk = *(const float4*)(A.ws.ktil + srow * 4);
#pragma unroll
    for (int j = 0; j < NX; ++j) S.K[j] = *(const float4*)(tp + FS + j * 4);
    if constexpr (sizeof(R) == sizeof(float)) {
      load_z(traj_at<float>(A, b, n, t), S.zs);
    } else {
      R zd[NZ];
      load_z(traj_at<R>(A, b, n, t), zd);
#pragma unroll
      for (int i = 0; i < NZ; ++i) S.zs[i] = (float)zd[i];
    }
    // row l of F = [A | B]: column c stored at c * 16
#pragma unroll
    for (int c = 0; c < NZ; ++c) S.fr[c] = tp[c * 16 + (l < NX ? l : 0)];
    if constexpr (THETA) {
      const int r = l < NX ? l : 0;
      if constexpr (DENSE) {
        const float* q = A.Q + srow * NPK;
#pragma unroll
        for (int c = 0; c < NZ; ++c) {
          const int i = r < c ? r : c, j = r < c ? c : r;  // packed upper triangle, row-major
          S.crow[c] = q[i * NZ - i * (i - 1) / 2 + (j - i)];
        }
      } else {
        S.crow[0] = A.Q[srow * NZ + r];
      }
      S.cl = A.p[srow * NZ + r];
      const float g = *(A.gx ? A.gx + srow * NX + r : A.p + srow * NZ + r);
      S.gl = A.gx ? g : 0.f;
    }
  };
  float xt[NX];
#pragma unroll
  for (int i = 0; i < NX; ++i) xt[i] = 0.f;
  // gradient w.r.t. the model constants (forward form of the two costate
  // sums): lane j < 8 carries xi_j, lane 8 + j carries eta_j of constant j
  float sv[THETA ? NX : 1];
  double gth = 0.0;
  dmpc_theta::PN PN;
  if constexpr (THETA) {
#pragma unroll
    for (int i = 0; i < NX; ++i) sv[i] = 0.f;
    PN = dmpc_theta::make_pn(A.raw, l & 7);
  }
  // one stage of the sweep from cf, the next stage's factors loaded into nf
  auto fstep = [&](int t, int a, int e, const FStage& cf, FStage& nf) {
    fload(t + 1 < e ? t + 1 : t, a, nf);  // at the segment's last stage, this one's again
    const size_t srow = (size_t)b * Tm + t;
    float ut[4] = {cf.kk.x, cf.kk.y, cf.kk.z, cf.kk.w};
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      ut[0] = fmaf(cf.K[j].x, xt[j], ut[0]);
      ut[1] = fmaf(cf.K[j].y, xt[j], ut[1]);
      ut[2] = fmaf(cf.K[j].z, xt[j], ut[2]);
      ut[3] = fmaf(cf.K[j].w, xt[j], ut[3]);
    }
    if (l == 0) {
      float* zt = zz[grp][0];
      float* zr = zz[grp][1];
      for (int i = 0; i < NX; ++i) zt[i] = xt[i];
      for (int a4 = 0; a4 < NU; ++a4) zt[NX + a4] = ut[a4];
      for (int i = 0; i < NZ; ++i) zr[i] = cf.zs[i];
    }
    lds_sync();
    const float* zt = zz[grp][0];
    const float* zr = zz[grp][1];
    // entry l from lane l, entry 16 from every lane (the same value): no
    // branch around the stores
    A.gp[srow * NZ + l] = zt[l];
    A.gp[srow * NZ + 16] = zt[16];
    if (!DENSE) {
      A.gQ[srow * NZ + l] = zt[l] * zr[l];
      A.gQ[srow * NZ + 16] = zt[16] * zr[16];
    } else {
      for (int m = l; m < NPK; m += 16) {
        const int i = c_pk.i[m], j = c_pk.j[m];
        A.gQ[srow * NPK + m] = (i == j) ? zt[i] * zr[i] : zt[i] * zr[j] + zt[j] * zr[i];
      }
    }
    lds_sync();
    if constexpr (THETA) {
      // row l of (C z~ + dL/dz*)_x and of (C z* + c)_x, then
      // gth += ht^T xi_j + hs^T eta_j and one RK4 step of the sensitivities
      float ht, hs;
      if constexpr (DENSE) {
        ht = cf.gl;
        hs = cf.cl;
#pragma unroll
        for (int c = 0; c < NX; ++c) {
          ht = fmaf(cf.crow[c], xt[c], ht);
          hs = fmaf(cf.crow[c], cf.zs[c], hs);
        }
#pragma unroll
        for (int a4 = 0; a4 < NU; ++a4) {
          ht = fmaf(cf.crow[NX + a4], ut[a4], ht);
          hs = fmaf(cf.crow[NX + a4], cf.zs[NX + a4], hs);
        }
      } else {
        float xl = xt[0], zl = cf.zs[0];
#pragma unroll
        for (int c = 1; c < NX; ++c) {
          xl = (l == c) ? xt[c] : xl;
          zl = (l == c) ? cf.zs[c] : zl;
        }
        ht = fmaf(cf.crow[0], xl, cf.gl);
        hs = fmaf(cf.crow[0], zl, cf.cl);
      }
      float dot = 0.f;
#pragma unroll
      for (int k = 0; k < NX; ++k) {
        // both broadcasts on every lane (a broadcast inside a lane-dependent
        // branch would read lanes that the branch has switched off)
        const float bt = rb(ht, k), bs = rb(hs, k);
        dot = fmaf((l < 8) ? bt : bs, sv[k], dot);
      }
      gth += (double)dot;
      if (t + 1 < T) {
        if (l < 8) dmpc_theta::propagate_xi(PN, cf.zs, cf.zs + NX, sv);
        else dmpc_theta::propagate_eta(PN, cf.zs, cf.zs + NX, xt, ut, sv);
      }
    }
    if (t + 1 < T) {
      float xi = 0.f;
      if (l < NX) {
#pragma unroll
        for (int c = 0; c < NX; ++c) xi = fmaf(cf.fr[c], xt[c], xi);
#pragma unroll
        for (int a4 = 0; a4 < NU; ++a4) xi = fmaf(cf.fr[NX + a4], ut[a4], xi);
      }
#pragma unroll
      for (int j = 0; j < NX; ++j) xt[j] = rb(xi, j);
    }
  };
  FStage f0, f1;
  for (int sg = 0; sg < nseg; ++sg) {
    const int a = sg * seg, e = (a + seg < T) ? a + seg : T;
    // the adjoint sweep above ended on the first segment, whose factors are
    // still in the buffer
    if (CKPT && sg > 0) recompute(a, e);
    fload(a, a, f0);
    __builtin_amdgcn_s_waitcnt(0);  // no load pending on loop entry
    for (int t = a; t < e; t += 2) {
      fstep(t, a, e, f0, f1);
      if (t + 1 >= e) break;
      fstep(t + 1, a, e, f1, f0);
    }
  }
  for (int t = T; t < Tm; ++t) {
    const size_t srow = (size_t)b * Tm + t;
    for (int ee = l; ee < NZ; ee += 16) A.gp[srow * NZ + ee] = 0.f;
    for (int m = l; m < W; m += 16) A.gQ[srow * W + m] = 0.f;
  }
  if constexpr (THETA) {
    const double both = gth + __shfl_xor(gth, 8, 16);  // xi part (lane j) + eta part (lane 8 + j)
    if (l < 8) A.gdyn[(size_t)b * 8 + l] = (float)both;
  }
}

// ---------------------------------------------------------------------------
// receding horizon (Alg. 1 outer loop): apply u*_0 to the state with one RK4
// step of the model, and shift the solution by one stage for the next solve's
// warm start (the last stage repeats).  One 64-thread block per instance: the
// instance's controls are staged in LDS before any is written, so u_warm may
// be the same buffer as u_star.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(64) void k_mpc_step(Dyn P, int B, int Tm, const int* Tarr, float* xs, const float* us,
                                                 float* uw, float* ua) {
  __shared__ float ur[DMPC_T_LIMIT * NU];
  const int b = blockIdx.x, tid = threadIdx.x;
  int T = Tarr ? Tarr[b] : Tm;
  T = T < 0 ? 0 : (T > Tm ? Tm : T);
  const float* row = us + (size_t)b * Tm * NU;
  for (int i = tid; i < T * NU; i += 64) ur[i] = row[i];
  __syncthreads();
  if (tid == 0 && T > 0) {
    float x[NX], xn[NX], u0[NU];
#pragma unroll
    for (int a = 0; a < NU; ++a) u0[a] = ur[a];
#pragma unroll
    for (int i = 0; i < NX; ++i) x[i] = xs[(size_t)b * NX + i];
    rk4(P, x, u0, xn);
#pragma unroll
    for (int i = 0; i < NX; ++i) xs[(size_t)b * NX + i] = xn[i];
  }
  if (ua && tid < NU) ua[(size_t)b * NU + tid] = (T > 0) ? ur[tid] : 0.f;
  if (uw) {
    for (int i = tid; i < Tm * NU; i += 64) {
      const int t = i / NU, a = i % NU;
      const int src = (t + 1 < T) ? t + 1 : T - 1;
      uw[(size_t)b * Tm * NU + i] = (t < T) ? ur[src * NU + a] : 0.f;
    }
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

struct Layout {
  size_t state, queue, order, traj, gains, lin, tail, ktil, ck, elem, pat, traj64, gains64, total;
  int tstride, nck;
  bool has_lin, has_tpar, has_redo;
};

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

int check_cfg(const dmpc_config* c) {
  if (!c) return DMPC_EINVAL;
  if (c->B < 0 || c->T_max < 1 || c->max_iter < 0) return DMPC_EINVAL;
  if (c->T_max > DMPC_T_LIMIT || c->max_iter > DMPC_K_LIMIT) return DMPC_EUNSUPPORTED;
  if (c->cost_kind != DMPC_COST_DIAG && c->cost_kind != DMPC_COST_DENSE) return DMPC_EUNSUPPORTED;
  if (c->ckpt_every < 0) return DMPC_EINVAL;
  if (!(c->tol_du == c->tol_du) || !(c->fp64_pivot == c->fp64_pivot)) return DMPC_EINVAL;
  if (c->flags & ~(DMPC_NEED_GRAD | DMPC_PLAIN | DMPC_LPT | DMPC_TUNED | DMPC_TPAR | DMPC_F64 | DMPC_F64_REDO))
    return DMPC_EINVAL;
  if ((c->flags & (DMPC_F64 | DMPC_F64_REDO)) && (c->flags & (DMPC_PLAIN | DMPC_TPAR))) return DMPC_EUNSUPPORTED;
  if ((c->flags & DMPC_F64) && (c->flags & DMPC_F64_REDO)) return DMPC_EINVAL;
  return DMPC_OK;
}

Layout make_layout(const dmpc_config* c) {
  Layout L;
  const size_t B = (size_t)c->B, Tm = (size_t)c->T_max;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  L.state = take(B * SW * sizeof(int));
  L.queue = take(256);
  L.order = take(B * sizeof(int));
  // trajectories and gains in the dynamics precision
  const size_t rs = (c->flags & DMPC_F64) ? sizeof(double) : sizeof(float);
  L.traj = take(B * NSLOT * Tm * ZS * rs);
  L.gains = take(B * Tm * GS * rs);
  // the per-launch form's linearisation buffer: present when that form may run
  // (requested, or possibly chosen by a tuned launch)
  L.has_lin = (c->flags & (DMPC_PLAIN | DMPC_TUNED | DMPC_TPAR)) != 0;
  L.lin = L.has_lin ? take(B * Tm * FS * sizeof(float)) : take(0);
  // the time-parallel Riccati's two element buffers and pattern guesses
  L.has_tpar = (c->flags & DMPC_TPAR) != 0;
  L.elem = take(L.has_tpar ? 2 * B * Tm * EL_W * sizeof(double) : 0);
  L.pat = take(L.has_tpar ? B * Tm : 0);
  const bool g = (c->flags & DMPC_NEED_GRAD) != 0;
  const int ck = c->ckpt_every;
  // checkpointing keeps one segment of factors per instance (the backward's
  // recompute buffer) and (V, v) at the stages j * ck < T_max
  L.tstride = (ck > 0) ? std::min(ck, c->T_max) : c->T_max;
  L.nck = (ck > 0) ? (c->T_max - 1) / ck : 0;
  L.tail = take(g ? B * (size_t)L.tstride * TS * sizeof(float) : 0);
  L.ktil = take(g ? B * Tm * 4 * sizeof(float) : 0);
  L.ck = take(g ? B * (size_t)L.nck * CK_W * sizeof(double) : 0);
  // the FP64 redo's own trajectories and gains
  L.has_redo = (c->flags & DMPC_F64_REDO) != 0;
  L.traj64 = take(L.has_redo ? B * NSLOT * Tm * ZS * sizeof(double) : 0);
  L.gains64 = take(L.has_redo ? B * Tm * GS * sizeof(double) : 0);
  L.total = off;
  return L;
}

// the same constants formed in double from the float inputs
Dyn64 make_dyn64(const dmpc_quad_params& q) {
  Dyn64 P;
  const double mass = q.mass, Jxx = q.Jxx, Jyy = q.Jyy, Jzz = q.Jzz, dt = q.dt;
  P.h = dt;
  P.h2 = 0.5 * dt;
  P.h6 = dt / 6.0;
  P.g = q.g;
  P.inv_m = 1.0 / mass;
  P.arm_a = (double)q.arm / std::sqrt(2.0);
  P.kappa = q.kappa;
  P.iJx = 1.0 / Jxx;
  P.iJy = 1.0 / Jyy;
  P.iJz = 1.0 / Jzz;
  P.cx = (Jzz - Jyy) / Jxx;
  P.cy = (Jxx - Jzz) / Jyy;
  P.cz = (Jyy - Jxx) / Jzz;
  P.hover = mass * (double)q.g / 4.0;
  return P;
}

Dyn make_dyn(const dmpc_quad_params& q) {
  Dyn P;
  P.h = q.dt;
  P.h2 = 0.5f * q.dt;
  P.h6 = q.dt / 6.f;
  P.g = q.g;
  P.inv_m = 1.f / q.mass;
  P.arm_a = q.arm / sqrtf(2.f);
  P.kappa = q.kappa;
  P.iJx = 1.f / q.Jxx;
  P.iJy = 1.f / q.Jyy;
  P.iJz = 1.f / q.Jzz;
  P.cx = (q.Jzz - q.Jyy) / q.Jxx;
  P.cy = (q.Jxx - q.Jzz) / q.Jyy;
  P.cz = (q.Jyy - q.Jxx) / q.Jzz;
  P.hover = q.mass * q.g / 4.f;
  return P;
}

thread_local std::string g_err;

}  // namespace

struct dmpc_handle_s {
  int device = 0;
  int cu = 0;
  std::string arch;  // the device's architecture name (gcnArchName), keys saved launch choices
  int occ[2][2] = {{1, 1}, {1, 1}};  // resident workgroups per CU: [dense][waves-per-SIMD variant]
  int last_launches = 0;
  void* scratch = nullptr;  // device address of this device's `scratch` array
  dmpc_launch_choice last_choice{};
  // launch choices found by dmpc_autotune (or set), per problem shape
  std::map<std::array<int, 6>, dmpc_launch_choice> tuned;
  std::string err;
};

// Workspace of dmpc_forward_noalloc: file-scope device memory, one copy on
// every device the library is loaded on, held until the process ends.  Host
// code never passes this name to a kernel or a copy (on the host it is only a
// stand-in); it uses the device address hipGetSymbolAddress returns, looked
// up once per device with that device current (scratch_address below).
static __device__ __align__(256) unsigned char scratch[DMPC_NOALLOC_WORKSPACE_BYTES];

namespace {

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;  // device -> address of that device's `scratch`

int fail(dmpc_handle h, int code, const std::string& msg) {
  if (h) h->err = msg;
  g_err = msg;
  return code;
}

int hip_check(dmpc_handle h, hipError_t e, const char* what) {
  if (e == hipSuccess) return DMPC_OK;
  return fail(h, DMPC_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Address of `scratch` on `device`, which must be current.
int scratch_address(dmpc_handle h, int device, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  if (it == g_scratch_ptr.end()) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(h, DMPC_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    it = g_scratch_ptr.emplace(device, ptr).first;
  }
  *out = it->second;
  return DMPC_OK;
}

// Makes a handle's device current for the life of the object and gives the
// calling thread its previous device back afterwards.
class DeviceScope {
 public:
  explicit DeviceScope(int device) {
    err_ = hipGetDevice(&prev_);
    if (err_ == hipSuccess && prev_ != device) {
      err_ = hipSetDevice(device);
      switched_ = err_ == hipSuccess;
    }
  }
  ~DeviceScope() {
    if (switched_) (void)hipSetDevice(prev_);
  }
  DeviceScope(const DeviceScope&) = delete;
  DeviceScope& operator=(const DeviceScope&) = delete;
  hipError_t status() const { return err_; }

 private:
  int prev_ = 0;
  bool switched_ = false;
  hipError_t err_ = hipSuccess;
};

KArgs base_args(const dmpc_config* c, void* workspace) {
  KArgs A;
  std::memset(&A, 0, sizeof A);
  const Layout L = make_layout(c);
  char* w = (char*)workspace;
  A.B = c->B;
  A.Tm = c->T_max;
  A.K = c->max_iter;
  A.tol = c->tol_du;
  A.piv = c->fp64_pivot;
  A.need_grad = (c->flags & DMPC_NEED_GRAD) ? 1 : 0;
  A.nquads = (c->B + 3) / 4;
  A.ws.state = (int*)(w + L.state);
  A.ws.queue = (int*)(w + L.queue);
  A.ws.order = (int*)(w + L.order);
  A.ws.traj = (float*)(w + L.traj);
  A.ws.gains = (float*)(w + L.gains);
  A.ws.lin = (float*)(w + L.lin);
  A.ws.tail = (float*)(w + L.tail);
  A.ws.ktil = (float*)(w + L.ktil);
  A.ws.ck = (double*)(w + L.ck);
  A.ws.elem = L.has_tpar ? (double*)(w + L.elem) : nullptr;
  A.ws.pat = L.has_tpar ? (uint8_t*)(w + L.pat) : nullptr;
  A.traj64 = L.has_redo ? (float*)(w + L.traj64) : nullptr;
  A.gains64 = L.has_redo ? (float*)(w + L.gains64) : nullptr;
  A.ckpt = c->ckpt_every;
  A.nck = L.nck;
  A.tstride = L.tstride;
  A.has_lin = L.has_lin ? 1 : 0;
  return A;
}

// problem shape a tuned launch choice applies to
// (the flags field holds DMPC_NEED_GRAD, DMPC_F64 and DMPC_F64_REDO)
std::array<int, 6> shape_key(const dmpc_config* c, bool has_T) {
  return {c->B, c->T_max, c->cost_kind, (int)(c->flags & (DMPC_NEED_GRAD | DMPC_F64 | DMPC_F64_REDO)),
          c->ckpt_every > 0 ? 1 : 0, has_T ? 1 : 0};
}

dmpc_launch_choice default_choice(const dmpc_config* c) {
  dmpc_launch_choice d{};
  d.plain = (c->flags & DMPC_TPAR) ? 2 : ((c->flags & DMPC_PLAIN) ? 1 : 0);
  d.lpt = (c->flags & DMPC_LPT) ? 1 : 0;
  d.waves_per_simd = 1;
  d.grid_mode = 0;
  d.inst_per_wave = 4;
  d.ms = 0.f;
  return d;
}

int forward_args(dmpc_handle h, const dmpc_config* cfg, dmpc_quad_params dyn, const float* x0, const float* Q,
                 const float* p, const float* u_lo, const float* u_hi, const int32_t* T, const float* u_init,
                 float* u_out,
                 float* x_out, uint32_t* status, void* workspace, size_t workspace_bytes, uint8_t* decision_log,
                 KArgs& A) {
  if (!h) return fail(nullptr, DMPC_EINVAL, "NULL handle");
  int rc = check_cfg(cfg);
  if (rc) return fail(h, rc, "invalid configuration");
  h->last_launches = 0;
  if (cfg->B == 0) return DMPC_OK;
  if (!x0 || !Q || !p || !u_lo || !u_hi || !u_out || !status)
    return fail(h, DMPC_EINVAL, "NULL required pointer");
  if (!(dyn.mass > 0.f) || !(dyn.Jxx > 0.f) || !(dyn.Jyy > 0.f) || !(dyn.Jzz > 0.f) || !(dyn.dt > 0.f))
    return fail(h, DMPC_EINVAL, "non-positive mass, inertia or step");
  const Layout L = make_layout(cfg);
  if (!workspace || workspace_bytes < L.total || ((uintptr_t)workspace & 255))
    return fail(h, DMPC_EWORKSPACE, "workspace missing, misaligned or smaller than dmpc_workspace_bytes()");
  A = base_args(cfg, workspace);
  A.P = make_dyn(dyn);
  A.P64 = make_dyn64(dyn);
  A.x0 = x0;
  A.Q = Q;
  A.p = p;
  A.lo = u_lo;
  A.hi = u_hi;
  A.T = T;
  A.uinit = u_init;
  A.u_out = u_out;
  A.x_out = x_out;
  A.status = status;
  A.dlog = decision_log;
  return DMPC_OK;
}

template <class R>
void launch_bwd(bool dense, bool ckpt, bool theta, int g, hipStream_t s, const KArgs& A) {
  if (ckpt) {
    if (theta) {
      if (dense) k_bwd<true, true, true, R><<<g, 64, 0, s>>>(A);
      else k_bwd<false, true, true, R><<<g, 64, 0, s>>>(A);
    } else {
      if (dense) k_bwd<true, true, false, R><<<g, 64, 0, s>>>(A);
      else k_bwd<false, true, false, R><<<g, 64, 0, s>>>(A);
    }
  } else {
    if (theta) {
      if (dense) k_bwd<true, false, true, R><<<g, 64, 0, s>>>(A);
      else k_bwd<false, false, true, R><<<g, 64, 0, s>>>(A);
    } else {
      if (dense) k_bwd<true, false, false, R><<<g, 64, 0, s>>>(A);
      else k_bwd<false, false, false, R><<<g, 64, 0, s>>>(A);
    }
  }
}

template <bool DENSE, class R>
void launch_persistent(int occ, int ipw, int grid, hipStream_t s, const KArgs& A) {
  if (ipw == 1) k_fwd_persistent<DENSE, 1, R, 1><<<grid, 64, 0, s>>>(A);
  else if (ipw == 2) k_fwd_persistent<DENSE, 1, R, 2><<<grid, 64, 0, s>>>(A);
  else if (occ == 2) k_fwd_persistent<DENSE, 2, R><<<grid, 64, 0, s>>>(A);
  else k_fwd_persistent<DENSE, 1, R><<<grid, 64, 0, s>>>(A);
}

int launch_forward(dmpc_handle h, const dmpc_config* cfg, KArgs A, const int32_t* T, const dmpc_launch_choice& c,
                   hipStream_t s) {
  const bool dense = cfg->cost_kind == DMPC_COST_DENSE;
  const int nq = A.nquads;
  int launches = 0;
  const bool f64 = (cfg->flags & DMPC_F64) != 0, redo = (cfg->flags & DMPC_F64_REDO) != 0;
  if (c.plain && (f64 || redo))
    return fail(h, DMPC_EUNSUPPORTED, "the FP64 form (DMPC_F64, DMPC_F64_REDO) runs as the persistent launch only");
  if (c.plain && !A.has_lin)
    return fail(h, DMPC_EWORKSPACE, "the per-launch form needs a workspace sized with DMPC_PLAIN or DMPC_TUNED");
  if (c.plain == 2 && !A.ws.elem)
    return fail(h, DMPC_EWORKSPACE, "the time-parallel Riccati needs a workspace sized with DMPC_TPAR");
  if (c.plain) {
    const long long units = (long long)cfg->B * cfg->T_max;
    const int lin_grid = (int)((units + 3) / 4);
    A.tpar = (c.plain == 2) ? 1 : 0;
    int levels = 0;
    while ((1 << levels) < cfg->T_max) ++levels;
    k_plain_init<<<nq, 64, 0, s>>>(A);
    ++launches;
    for (int k = 0; k < cfg->max_iter; ++k) {
      k_plain_lin<<<lin_grid, 64, 0, s>>>(A, 0);
      ++launches;
      if (A.tpar) {
        const unsigned ug = (unsigned)units;
        if (dense) k_tpar_elem<true><<<ug, 64, 0, s>>>(A, 0);
        else k_tpar_elem<false><<<ug, 64, 0, s>>>(A, 0);
        int src = 0;
        for (int lv = 0; lv < levels; ++lv, src = 1 - src) k_tpar_scan<SCAN_NT><<<ug, SCAN_NT, 0, s>>>(A, 1 << lv, src, 0);
        if (dense) k_tpar_gains<true><<<ug, 64, 0, s>>>(A, src);
        else k_tpar_gains<false><<<ug, 64, 0, s>>>(A, src);
        launches += levels + 2;
      }
      if (dense) k_plain_riccati<true, 0><<<nq, 64, 0, s>>>(A);
      else k_plain_riccati<false, 0><<<nq, 64, 0, s>>>(A);
      if (dense) k_plain_ls<true><<<nq, 64, 0, s>>>(A);
      else k_plain_ls<false><<<nq, 64, 0, s>>>(A);
      launches += 2;
    }
    A.tpar = 0;
    if (A.need_grad && c.plain == 2 && A.ckpt == 0) {
      // the tail's fixed-mask problem through the same scan
      const unsigned ug = (unsigned)units;
      k_plain_lin<<<lin_grid, 64, 0, s>>>(A, 1);
      if (dense) k_tpar_elem<true><<<ug, 64, 0, s>>>(A, 1);
      else k_tpar_elem<false><<<ug, 64, 0, s>>>(A, 1);
      int src = 0;
      for (int lv = 0; lv < levels; ++lv, src = 1 - src) k_tpar_scan<SCAN_NT><<<ug, SCAN_NT, 0, s>>>(A, 1 << lv, src, 1);
      if (dense) k_tpar_tail<true><<<ug, 64, 0, s>>>(A, src);
      else k_tpar_tail<false><<<ug, 64, 0, s>>>(A, src);
      launches += levels + 3;
    } else if (A.need_grad) {
      k_plain_lin<<<lin_grid, 64, 0, s>>>(A, 1);
      if (A.ckpt > 0) {
        if (dense) k_plain_riccati<true, 2><<<nq, 64, 0, s>>>(A);
        else k_plain_riccati<false, 2><<<nq, 64, 0, s>>>(A);
      } else {
        if (dense) k_plain_riccati<true, 1><<<nq, 64, 0, s>>>(A);
        else k_plain_riccati<false, 1><<<nq, 64, 0, s>>>(A);
      }
      launches += 2;
    }
    k_plain_finalize<<<nq, 64, 0, s>>>(A);
    ++launches;
  } else {
    const bool lpt = c.lpt && T;
    A.use_order = lpt ? 1 : 0;
    if (lpt) k_sort_by_T<<<1, 1024, 0, s>>>(T, cfg->B, cfg->T_max, A.ws.order, A.ws.queue);
    else k_reset_queue<<<1, 64, 0, s>>>(A.ws.queue);
    // instances per wave: 4, or 2 / 1 with one wave per SIMD (registers uncapped)
    const int ipw = (c.inst_per_wave == 1 || c.inst_per_wave == 2) ? c.inst_per_wave : 4;
    const int occ = (ipw == 4 && c.waves_per_simd == 2) ? 2 : 1;
    const int cap = std::max(1, h->cu * h->occ[dense ? 1 : 0][occ - 1]);
    const int units = (cfg->B + ipw - 1) / ipw;
    const int grid = c.grid_mode == 1 ? units : std::min(units, cap);
    if (f64) {
      if (dense) launch_persistent<true, double>(occ, ipw, grid, s, A);
      else launch_persistent<false, double>(occ, ipw, grid, s, A);
    } else {
      if (dense) launch_persistent<true, float>(occ, ipw, grid, s, A);
      else launch_persistent<false, float>(occ, ipw, grid, s, A);
    }
    launches += 2;
    if (redo) {
      // the instances whose control block had a pivot below fp64_pivot are
      // solved again, from the start, in the FP64 form, in their own
      // trajectory and gain regions; the instance list reuses ws.order (the
      // FP32 launch no longer reads it) and the redo's counters sit in the
      // queue block, apart from the FP32 launch's counter
      KArgs Rd = A;
      Rd.ws.traj = A.traj64;
      Rd.ws.gains = A.gains64;
      Rd.ws.queue = A.ws.queue + 32;
      Rd.redo_count = A.ws.queue + 16;
      Rd.traj_f = A.ws.traj;
      Rd.use_order = 1;
      k_reset_redo<<<1, 64, 0, s>>>(A.ws.queue + 16, A.ws.queue + 32);
      k_redo_list<<<(cfg->B + 255) / 256, 256, 0, s>>>(A.status, cfg->B, A.ws.order, A.ws.queue + 16);
      if (dense) launch_persistent<true, double>(occ, ipw, grid, s, Rd);
      else launch_persistent<false, double>(occ, ipw, grid, s, Rd);
      launches += 3;
    }
  }
  h->last_launches = launches;
  h->last_choice = c;
  return hip_check(h, hipGetLastError(), "kernel launch");
}

}  // namespace

extern "C" {

int dmpc_validate(const dmpc_config* cfg) {
  const int rc = check_cfg(cfg);
  if (rc) g_err = "invalid configuration";
  return rc;
}

size_t dmpc_workspace_bytes(const dmpc_config* cfg) {
  if (check_cfg(cfg)) return 0;
  return make_layout(cfg).total;
}

int dmpc_create(dmpc_handle* out, int device) {
  if (!out) return fail(nullptr, DMPC_EINVAL, "NULL handle pointer");
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n)
    return fail(nullptr, DMPC_EHIP, "no such HIP device");
  dmpc_handle h = new dmpc_handle_s();
  h->device = device;
  hipDeviceProp_t prop;
  int rc = hip_check(h, hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
  if (rc) {
    delete h;
    return rc;
  }
  h->cu = prop.multiProcessorCount;
  h->arch = prop.gcnArchName;
  DeviceScope scope(device);
  rc = hip_check(h, scope.status(), "hipSetDevice");
  if (!rc) rc = scratch_address(h, device, &h->scratch);
  if (rc) {
    delete h;
    return rc;
  }
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_fwd_persistent<false, 1>, 64, 0) == hipSuccess && occ > 0)
    h->occ[0][0] = occ;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_fwd_persistent<true, 1>, 64, 0) == hipSuccess && occ > 0)
    h->occ[1][0] = occ;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_fwd_persistent<false, 2>, 64, 0) == hipSuccess && occ > 0)
    h->occ[0][1] = occ;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_fwd_persistent<true, 2>, 64, 0) == hipSuccess && occ > 0)
    h->occ[1][1] = occ;
  *out = h;
  return DMPC_OK;
}

int dmpc_destroy(dmpc_handle h) {
  delete h;
  return DMPC_OK;
}

const char* dmpc_last_error(dmpc_handle h) { return h ? h->err.c_str() : g_err.c_str(); }

int dmpc_last_launch_count(dmpc_handle h) { return h ? h->last_launches : -1; }

int dmpc_forward(dmpc_handle h, const dmpc_config* cfg, dmpc_quad_params dyn, const float* x0, const float* Q,
                 const float* p, const float* u_lo, const float* u_hi, const int32_t* T, const float* u_init,
                 float* u_out, float* x_out, uint32_t* status, void* workspace, size_t workspace_bytes,
                 uint8_t* decision_log, void* stream) {
  KArgs A;
  int rc = forward_args(h, cfg, dyn, x0, Q, p, u_lo, u_hi, T, u_init, u_out, x_out, status, workspace,
                        workspace_bytes, decision_log, A);
  if (rc || cfg->B == 0) return rc;
  DeviceScope scope(h->device);
  rc = hip_check(h, scope.status(), "hipSetDevice");
  if (rc) return rc;
  dmpc_launch_choice c = default_choice(cfg);
  if (cfg->flags & DMPC_TUNED) {
    auto it = h->tuned.find(shape_key(cfg, T != nullptr));
    if (it != h->tuned.end()) c = it->second;
  }
  return launch_forward(h, cfg, A, T, c, (hipStream_t)stream);
}

int dmpc_forward_noalloc(dmpc_handle h, const dmpc_config* cfg, dmpc_quad_params dyn, const float* x0,
                         const float* Q, const float* p, const float* u_lo, const float* u_hi, const int32_t* T,
                         const float* u_init, float* u_out, float* x_out, uint32_t* status, uint8_t* decision_log,
                         void* stream) {
  if (!h) return fail(nullptr, DMPC_EINVAL, "NULL handle");
  h->last_launches = 0;
  int rc = check_cfg(cfg);
  if (rc) return fail(h, rc, "invalid configuration");
  if (cfg->flags & DMPC_NEED_GRAD)
    return fail(h, DMPC_EINVAL,
                "dmpc_forward_noalloc keeps no workspace for a backward: DMPC_NEED_GRAD needs dmpc_forward");
  const size_t need = make_layout(cfg).total;
  if (need > (size_t)DMPC_NOALLOC_WORKSPACE_BYTES)
    return fail(h, DMPC_EUNSUPPORTED,
                "dmpc_forward_noalloc: this problem needs " + std::to_string(need) +
                    " bytes of workspace, more than the library's static " +
                    std::to_string((size_t)DMPC_NOALLOC_WORKSPACE_BYTES) + " bytes; use dmpc_forward");
  KArgs A;
  rc = forward_args(h, cfg, dyn, x0, Q, p, u_lo, u_hi, T, u_init, u_out, x_out, status, h->scratch,
                    (size_t)DMPC_NOALLOC_WORKSPACE_BYTES, decision_log, A);
  if (rc || cfg->B == 0) return rc;
  DeviceScope scope(h->device);
  rc = hip_check(h, scope.status(), "hipSetDevice");
  if (rc) return rc;
  dmpc_launch_choice c = default_choice(cfg);
  if (cfg->flags & DMPC_TUNED) {
    auto it = h->tuned.find(shape_key(cfg, T != nullptr));
    if (it != h->tuned.end()) c = it->second;
  }
  return launch_forward(h, cfg, A, T, c, (hipStream_t)stream);
}

int dmpc_autotune(dmpc_handle h, const dmpc_config* cfg, dmpc_quad_params dyn, const float* x0, const float* Q,
                  const float* p, const float* u_lo, const float* u_hi, const int32_t* T, const float* u_init,
                  float* u_out, float* x_out, uint32_t* status, void* workspace, size_t workspace_bytes,
                  void* stream, dmpc_launch_choice* chosen) {
  KArgs A;
  int rc = forward_args(h, cfg, dyn, x0, Q, p, u_lo, u_hi, T, u_init, u_out, x_out, status, workspace,
                        workspace_bytes, nullptr, A);
  if (rc) return rc;
  DeviceScope scope(h->device);
  rc = hip_check(h, scope.status(), "hipSetDevice");
  if (rc) return rc;
  dmpc_launch_choice best = default_choice(cfg);
  best.ms = 0.f;
  if (cfg->B > 0) {
    // candidates: per-launch form (and its time-parallel variant when the
    // workspace has room for it); persistent form x occupancy target x grid x order
    std::vector<dmpc_launch_choice> cand;
    const bool f64 = (cfg->flags & (DMPC_F64 | DMPC_F64_REDO)) != 0;
    if (A.has_lin && !f64) cand.push_back(dmpc_launch_choice{1, 0, 1, 0, 0.f, 4});
    if (A.ws.elem && !f64) cand.push_back(dmpc_launch_choice{2, 0, 1, 0, 0.f, 4});
    for (int occ = 1; occ <= 2; ++occ)
      for (int grid = 0; grid <= 1; ++grid)
        for (int lpt = 0; lpt <= (T ? 1 : 0); ++lpt) cand.push_back(dmpc_launch_choice{0, lpt, occ, grid, 0.f, 4});
    // fewer instances per wave: worth trying only while the batch leaves SIMDs idle
    if (cfg->B < 4 * h->cu * 4)
      for (int ipw = 2; ipw >= 1; ipw /= 2)
        for (int lpt = 0; lpt <= (T ? 1 : 0); ++lpt) cand.push_back(dmpc_launch_choice{0, lpt, 1, 1, 0.f, ipw});
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    rc = hip_check(h, hipEventCreate(&e0), "hipEventCreate");
    if (rc) return rc;
    rc = hip_check(h, hipEventCreate(&e1), "hipEventCreate");
    if (rc) {
      (void)hipEventDestroy(e0);
      return rc;
    }
    float best_ms = 0.f;
    for (size_t i = 0; i < cand.size() && !rc; ++i) {
      rc = launch_forward(h, cfg, A, T, cand[i], s);  // warm-up
      float ms = 0.f;
      for (int r = 0; r < 3 && !rc; ++r) {
        rc = hip_check(h, hipEventRecord(e0, s), "hipEventRecord");
        if (!rc) rc = launch_forward(h, cfg, A, T, cand[i], s);
        if (!rc) rc = hip_check(h, hipEventRecord(e1, s), "hipEventRecord");
        if (!rc) rc = hip_check(h, hipEventSynchronize(e1), "hipEventSynchronize");
        float m = 0.f;
        if (!rc) rc = hip_check(h, hipEventElapsedTime(&m, e0, e1), "hipEventElapsedTime");
        if (!rc && (r == 0 || m < ms)) ms = m;
      }
      if (!rc && (i == 0 || ms < best_ms)) {
        best_ms = ms;
        best = cand[i];
        best.ms = ms;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    // leave the outputs and the workspace of the chosen configuration
    rc = launch_forward(h, cfg, A, T, best, s);
    if (rc) return rc;
  }
  h->tuned[shape_key(cfg, T != nullptr)] = best;
  if (chosen) *chosen = best;
  return DMPC_OK;
}

int dmpc_set_tuned(dmpc_handle h, const dmpc_config* cfg, int has_T, const dmpc_launch_choice* choice) {
  if (!h || !choice) return fail(h, DMPC_EINVAL, "NULL argument");
  int rc = check_cfg(cfg);
  if (rc) return fail(h, rc, "invalid configuration");
  if (choice->plain < 0 || choice->plain > 2 || choice->lpt < 0 || choice->lpt > 1 || choice->waves_per_simd < 1 ||
      choice->waves_per_simd > 2 || choice->grid_mode < 0 || choice->grid_mode > 1 ||
      !(choice->inst_per_wave == 1 || choice->inst_per_wave == 2 || choice->inst_per_wave == 4))
    return fail(h, DMPC_EINVAL, "launch choice out of range");
  h->tuned[shape_key(cfg, has_T != 0)] = *choice;
  return DMPC_OK;
}

int dmpc_get_tuned(dmpc_handle h, const dmpc_config* cfg, int has_T, dmpc_launch_choice* choice) {
  if (!h || !choice) return fail(h, DMPC_EINVAL, "NULL argument");
  int rc = check_cfg(cfg);
  if (rc) return fail(h, rc, "invalid configuration");
  auto it = h->tuned.find(shape_key(cfg, has_T != 0));
  if (it == h->tuned.end()) return fail(h, DMPC_EINVAL, "no tuned launch choice for this shape");
  *choice = it->second;
  return DMPC_OK;
}

// One line per tuned shape:
//   dmpc-tuned-v1 <arch> <cu> <B> <T_max> <cost_kind> <need_grad> <ckpt> <has_T> <plain> <lpt> <waves> <grid> <ms>
int dmpc_tuned_save(dmpc_handle h, const char* path) {
  if (!h || !path) return fail(h, DMPC_EINVAL, "NULL argument");
  std::ostringstream o;
  for (const auto& kv : h->tuned) {
    const auto& k = kv.first;
    const auto& c = kv.second;
    o << "dmpc-tuned-v1 " << h->arch << ' ' << h->cu;
    for (int v : k) o << ' ' << v;
    o << ' ' << c.plain << ' ' << c.lpt << ' ' << c.waves_per_simd << ' ' << c.grid_mode << ' ' << c.ms << ' '
      << c.inst_per_wave << '\n';
  }
  std::ofstream f(path, std::ios::trunc);
  if (!f) return fail(h, DMPC_EINVAL, std::string("cannot write ") + path);
  f << o.str();
  f.close();
  if (!f) return fail(h, DMPC_EINVAL, std::string("cannot write ") + path);
  return (int)h->tuned.size();
}

int dmpc_tuned_load(dmpc_handle h, const char* path) {
  if (!h || !path) return fail(h, DMPC_EINVAL, "NULL argument");
  std::ifstream f(path);
  if (!f) return fail(h, DMPC_EINVAL, std::string("cannot read ") + path);
  std::string line;
  int n = 0;
  while (std::getline(f, line)) {
    std::istringstream in(line);
    std::string tag, arch;
    int cu = 0;
    std::array<int, 6> k{};
    dmpc_launch_choice c{};
    if (!(in >> tag >> arch >> cu) || tag != "dmpc-tuned-v1") continue;
    bool ok = true;
    for (int& v : k) ok = ok && (bool)(in >> v);
    ok = ok && (bool)(in >> c.plain >> c.lpt >> c.waves_per_simd >> c.grid_mode >> c.ms);
    if (!(in >> c.inst_per_wave)) c.inst_per_wave = 4;  // lines written before this field existed
    if (!ok || arch != h->arch || cu != h->cu) continue;
    if (c.plain < 0 || c.plain > 2 || c.lpt < 0 || c.lpt > 1 || c.waves_per_simd < 1 || c.waves_per_simd > 2 ||
        c.grid_mode < 0 || c.grid_mode > 1 || !(c.inst_per_wave == 1 || c.inst_per_wave == 2 || c.inst_per_wave == 4))
      continue;
    h->tuned[k] = c;
    ++n;
  }
  return n;
}

int dmpc_last_launch_choice(dmpc_handle h, dmpc_launch_choice* choice) {
  if (!h || !choice) return fail(h, DMPC_EINVAL, "NULL argument");
  *choice = h->last_choice;
  return DMPC_OK;
}

int dmpc_backward(dmpc_handle h, const dmpc_config* cfg, dmpc_quad_params dyn, const float* Q, const float* p,
                  const float* u_lo, const float* u_hi, const void* workspace, size_t workspace_bytes,
                  const float* grad_u, const float* grad_x, float* grad_Q, float* grad_p, float* grad_x0,
                  float* grad_dyn, void* stream) {
  if (!h) return fail(nullptr, DMPC_EINVAL, "NULL handle");
  int rc = check_cfg(cfg);
  if (rc) return fail(h, rc, "invalid configuration");
  h->last_launches = 0;
  if (!(cfg->flags & DMPC_NEED_GRAD)) return fail(h, DMPC_EINVAL, "backward needs a forward run with DMPC_NEED_GRAD");
  if (cfg->B == 0) return DMPC_OK;
  if (!grad_u || !grad_Q || !grad_p || !grad_x0) return fail(h, DMPC_EINVAL, "NULL required pointer");
  const bool ckpt = cfg->ckpt_every > 0;
  if (ckpt && (!Q || !p || !u_lo || !u_hi))
    return fail(h, DMPC_EINVAL, "checkpointed backward needs the forward's Q, p, u_lo, u_hi");
  const bool theta = grad_dyn != nullptr;
  if (theta && (!Q || !p)) return fail(h, DMPC_EINVAL, "grad_dyn needs the forward's Q and p");
  if ((ckpt || theta) &&
      (!(dyn.mass > 0.f) || !(dyn.Jxx > 0.f) || !(dyn.Jyy > 0.f) || !(dyn.Jzz > 0.f) || !(dyn.dt > 0.f)))
    return fail(h, DMPC_EINVAL, "non-positive mass, inertia or step");
  const Layout L = make_layout(cfg);
  if (!workspace || workspace_bytes < L.total || ((uintptr_t)workspace & 255))
    return fail(h, DMPC_EWORKSPACE, "workspace missing, misaligned or smaller than dmpc_workspace_bytes()");
  DeviceScope scope(h->device);
  rc = hip_check(h, scope.status(), "hipSetDevice");
  if (rc) return rc;
  KArgs A = base_args(cfg, (void*)workspace);
  A.gu = grad_u;
  A.gx = grad_x;
  A.gQ = grad_Q;
  A.gp = grad_p;
  A.gx0 = grad_x0;
  A.gdyn = grad_dyn;
  A.raw = dyn;
  hipStream_t s = (hipStream_t)stream;
  const bool dense = cfg->cost_kind == DMPC_COST_DENSE;
  if (ckpt || theta) {
    A.P = make_dyn(dyn);
    A.P64 = make_dyn64(dyn);
    A.Q = Q;
    A.p = p;
    A.lo = u_lo;
    A.hi = u_hi;
  }
  const int g = A.nquads;
  if (cfg->flags & DMPC_F64)
    launch_bwd<double>(dense, ckpt, theta, g, s, A);
  else
    launch_bwd<float>(dense, ckpt, theta, g, s, A);
  h->last_launches = 1;
  return hip_check(h, hipGetLastError(), "kernel launch");
}

int dmpc_mpc_step(dmpc_handle h, const dmpc_config* cfg, dmpc_quad_params dyn, const int32_t* T, float* x_state,
                  const float* u_star, float* u_warm, float* u_applied, void* stream) {
  if (!h) return fail(nullptr, DMPC_EINVAL, "NULL handle");
  int rc = check_cfg(cfg);
  if (rc) return fail(h, rc, "invalid configuration");
  h->last_launches = 0;
  if (cfg->B == 0) return DMPC_OK;
  if (!x_state || !u_star) return fail(h, DMPC_EINVAL, "NULL required pointer");
  if (!(dyn.mass > 0.f) || !(dyn.Jxx > 0.f) || !(dyn.Jyy > 0.f) || !(dyn.Jzz > 0.f) || !(dyn.dt > 0.f))
    return fail(h, DMPC_EINVAL, "non-positive mass, inertia or step");
  DeviceScope scope(h->device);
  rc = hip_check(h, scope.status(), "hipSetDevice");
  if (rc) return rc;
  k_mpc_step<<<cfg->B, 64, 0, (hipStream_t)stream>>>(make_dyn(dyn), cfg->B, cfg->T_max, T, x_state, u_star, u_warm,
                                                       u_applied);
  h->last_launches = 1;
  return hip_check(h, hipGetLastError(), "kernel launch");
}

int dmpc_capture_begin(dmpc_handle h, void* stream) {
  if (!h) return fail(nullptr, DMPC_EINVAL, "NULL handle");
  return hip_check(h, hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal), "begin capture");
}

int dmpc_capture_end(dmpc_handle h, void* stream, void** graph_exec) {
  if (!h || !graph_exec) return fail(h, DMPC_EINVAL, "NULL argument");
  hipGraph_t g = nullptr;
  int rc = hip_check(h, hipStreamEndCapture((hipStream_t)stream, &g), "end capture");
  if (rc) return rc;
  hipGraphExec_t e = nullptr;
  rc = hip_check(h, hipGraphInstantiate(&e, g, nullptr, nullptr, 0), "graph instantiate");
  (void)hipGraphDestroy(g);
  if (rc) return rc;
  *graph_exec = (void*)e;
  return DMPC_OK;
}

int dmpc_graph_launch(dmpc_handle h, void* graph_exec, void* stream) {
  if (!h || !graph_exec) return fail(h, DMPC_EINVAL, "NULL argument");
  return hip_check(h, hipGraphLaunch((hipGraphExec_t)graph_exec, (hipStream_t)stream), "graph launch");
}

int dmpc_graph_destroy(dmpc_handle h, void* graph_exec) {
  if (!graph_exec) return DMPC_OK;
  return hip_check(h, hipGraphExecDestroy((hipGraphExec_t)graph_exec), "graph destroy");
}

}  // extern "C"
