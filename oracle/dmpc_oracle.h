/*
 * dmpc_oracle.h -- FP64 CPU oracle for the batched differentiable MPC layer.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this code: only the test suite, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code, header or constant with the HIP
 * library under paper_2605_29155_amd/.
 *
 * What it computes (CA-AC-MPC, Sec. IV, eq. (3) and Alg. 2):
 *   min_{x,u} sum_{t=0}^{T-1} 1/2 z_t^T C_t z_t + c_t^T z_t,   z_t = (x_t, u_t)
 *   s.t. x_{t+1} = f(x_t, u_t), x_0 = x_init, lo <= u_t <= hi,
 * solved by control-limited iLQR (the paper's Sec. IV, "three-stage loop",
 * after Tassa et al. 2014), and the gradient of an external loss w.r.t.
 * (C_t, c_t, x_init) by implicit differentiation of the KKT conditions at the
 * returned solution (Sec. IV, after eq. (3); Amos et al. 2018).
 *
 * Conventions (the paper never states its quadrotor model; these are this
 * project's readings):
 *   state x = (p[3], q[4] = (qw,qx,qy,qz), v[3], w[3]),  n_x = 13
 *   input u = four rotor thrusts [N],                      n_u = 4
 *   one RK4 step of the rigid-body ODE with zero-order-hold thrust, no
 *   quaternion renormalisation; T states x_0..x_{T-1} and T controls; no
 *   terminal cost (eq. (3) has none), so x_T never enters the cost.
 *
 * Layout of every batched array: instance-major, row-major,
 *   x0 [B][13], Q [B][T_max][17 | 153 | 289], p [B][T_max][17],
 *   lo/hi [B][4], T [B], u [B][T_max][4], x [B][T_max][13].
 * All floating point is double.
 */
#ifndef DMPC_ORACLE_H
#define DMPC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_NX 13
#define ORC_NU 4
#define ORC_NZ 17
#define ORC_NPACK 153 /* 17*18/2 packed upper triangle */
#define ORC_NALPHA 4  /* line-search candidates, Sec. IV "Forward pass with line-search" */

/* cost_kind */
#define ORC_COST_DIAG 0   /* Q[t] holds the 17 diagonal entries of C_t       */
#define ORC_COST_PACKED 1 /* Q[t] holds the 153-entry packed upper triangle  */
#define ORC_COST_FULL 2   /* Q[t] holds the full 17x17 row-major matrix      */

/* dyn_kind */
#define ORC_DYN_QUAD 0   /* quadrotor RK4 map                                 */
#define ORC_DYN_AFFINE 1 /* given x_{t+1} = A_t x_t + B_t u_t + r_t            */

/* status bits (oracle's own; same meaning as the library's) */
#define ORC_ST_CONVERGED 0x1u
#define ORC_ST_MAXITER 0x2u
#define ORC_ST_NONFINITE 0x4u
#define ORC_ST_QPFAIL 0x10u
#define ORC_ST_REGULARIZED 0x20u

/* box-QP pattern codes, one per control coordinate */
#define ORC_FREE 0
#define ORC_LOWER 1
#define ORC_UPPER 2

#define ORC_ALPHA_NONE 255 /* line search found no finite candidate */
#define ORC_NTHETA 8       /* model constants: the fields of orc_params, in order */

typedef struct {
  double mass, Jxx, Jyy, Jzz, arm, kappa, dt, g;
} orc_params;

typedef struct {
  int32_t B, T_max;
  int32_t cost_kind; /* ORC_COST_* */
  int32_t dyn_kind;  /* ORC_DYN_* */
  int32_t max_iter;  /* K */
  double tol;        /* >0: stop when ||U^k - U^{k-1}||_inf < tol */
  int32_t nthreads;  /* worker threads over instances (>=1) */
} orc_config;

/* ---- single-instance building blocks (pinned directly by tests) ---- */

/* The line-search step lengths the forward tries, in the order it tries them
 * (Sec. IV "Forward pass with line-search"): writes ORC_NALPHA values to out
 * (when not NULL) and returns ORC_NALPHA. */
int orc_alphas(double* out);

/* continuous-time right-hand side xdot = F(x, u) */
void orc_dyn(const orc_params* P, const double* x, const double* u, double* xdot);
/* one RK4 step x_next = f(x, u) */
void orc_rk4(const orc_params* P, const double* x, const double* u, double* xn);
/* directional derivative of f along dir = (dx[13], du[4]) by the complex step
 * Im f(x + i h dx, u + i h du) / h; used only to pin orc_rk4_jac */
void orc_rk4_complex_step(const orc_params* P, const double* x, const double* u, const double* dir,
                          double h, double* out);
/* analytic partials of F: Fx [13][13], Fu [13][4] */
void orc_dyn_jac(const orc_params* P, const double* x, const double* u, double* Fx, double* Fu);
/* exact Jacobian of the RK4 map by the chain rule: A [13][13], B [13][4] */
void orc_rk4_jac(const orc_params* P, const double* x, const double* u, double* A, double* B);

/* Stagewise box-QP: min 1/2 d^T H d + q^T d s.t. a <= d <= b, H 4x4 SPD,
 * solved exactly by enumerating all 3^4 patterns.  pattern[i] gets
 * ORC_FREE/ORC_LOWER/ORC_UPPER.  Returns 0, or ORC_ST_QPFAIL /
 * ORC_ST_NONFINITE when no pattern passes. */
uint32_t orc_boxqp(const double* H, const double* q, const double* a, const double* b, double* d,
                   int32_t* pattern);

/* Dense LU solve with partial pivoting of the n x n system M x = r (M is
 * overwritten).  Returns 0 on success, -1 on a zero pivot. */
int orc_lu_solve(int n, double* M, double* r);

/* ---- batched forward: control-limited iLQR (Alg. 2 inner loop) ----
 * Aff/Bff/rff: affine dynamics [B][T_max][169|52|13] when dyn_kind is
 *   ORC_DYN_AFFINE, else NULL.
 * u_init: [B][T_max][4] initial controls or NULL (NULL: hover thrust
 *   m g / 4 per rotor for the quadrotor, 0 for affine, then clamped).
 * replay_*: NULL for a free run.  Otherwise the decisions to take instead of
 *   the oracle's own: replay_iters [B] iterations to run, replay_alpha
 *   [B][K] candidate index per iteration, replay_pattern [B][K][T_max] box-QP
 *   pattern per stage (2 bits per control, control i at bits 2i..2i+1).
 * Outputs (any may be NULL): u_out, x_out, J_out [B], iters_out [B],
 *   status_out [B], alpha_log [B][K], pattern_log [B][K][T_max],
 *   cand_cost [B][K][4] line-search costs J(alpha), replay_viol [B][K][T_max]
 *   (replay only, else zero): how far each replayed stage pattern is from
 *   the optimality conditions of the oracle's own stagewise box-QP (free
 *   coordinates inside the box, multipliers of clamped ones correctly
 *   signed), as the smallest relative tolerance at which they hold (0 for a
 *   valid pattern), taken before the replayed step is clamped into the box.
 */
int orc_forward(const orc_config* cfg, const orc_params* P, const double* x0, const double* Q,
                const double* p, const double* lo, const double* hi, const int32_t* T,
                const double* Aff, const double* Bff, const double* rff, const double* u_init,
                const int32_t* replay_iters, const uint8_t* replay_alpha, const uint8_t* replay_pattern,
                double* u_out, double* x_out, double* J_out, int32_t* iters_out, uint32_t* status_out,
                uint8_t* alpha_log, uint8_t* pattern_log, double* cand_cost, double* replay_viol);

/* ---- batched backward: implicit differentiation at (x*, u*) ----
 * method 0: Riccati adjoint (an LQR solve with the active controls fixed);
 * method 1: dense KKT system solved by LU.  The two must agree.
 * mask: [B][T_max] bit i set = control i active; NULL = derive from u* by
 *   exact equality with lo/hi.
 * grad_u [B][T_max][4] = dL/du*, grad_x [B][T_max][13] = dL/dx* or NULL.
 * Outputs: dQ [B][T_max][17|153|289] (layout of Q), dp [B][T_max][17],
 *   dx0 [B][13]; dtheta [B][8] or NULL: dL/d(mass, Jxx, Jyy, Jzz, arm, kappa,
 *   dt, g) through the linearised dynamics (quadrotor only; -1 with affine).
 */
int orc_backward(const orc_config* cfg, const orc_params* P, const double* x0, const double* Q,
                 const double* p, const double* lo, const double* hi, const int32_t* T,
                 const double* Aff, const double* Bff, const double* rff, const double* u_star,
                 const double* x_star, const uint8_t* mask, const double* grad_u, const double* grad_x,
                 int32_t method, double* dQ, double* dp, double* dx0, double* dtheta);

#ifdef __cplusplus
}
#endif
#endif
