/*
 * dmpc_oracle.c -- plain FP64 CPU oracle for the batched differentiable MPC
 * layer of CA-AC-MPC.  TEST INFRASTRUCTURE ONLY: used by the test suite, the
 * smoke check and the benchmark's CPU-baseline leg, never by the product path.
 *
 * Written for obviousness, not speed: full 17x17 matrices, no blocking, no
 * fusion, one instance at a time (threads only split the batch).
 *
 * Paper passages followed (CA-AC-MPC, Buo et al.):
 *  - eq. (2), (3): quadratic stage cost 1/2 z^T C z + c^T z, dynamics,
 *    x_0 = x_init, input box.
 *  - Sec. IV "Rollout and linearization": rollout plus the Jacobians
 *    A_t = df/dx, B_t = df/du (here the exact derivative of the RK4 map).
 *  - Sec. IV "Backward pass with input bounds": Riccati recursion giving
 *    K_t, k_t, with a stagewise box-constrained QP (Tassa et al. 2014).
 *  - Sec. IV "Forward pass with line-search": candidates
 *    alpha in {1, 0.5, 0.25, 0.1}, affine feedback update, rollout, cost;
 *    the best candidate becomes the new nominal.
 *  - Alg. 2 (CA-AC-MPC deployment), inner loop: Rollout, then K times
 *    LQ -> FBP -> FFP, with an optional convergence break.
 *  - Sec. IV after eq. (3): gradients w.r.t. (C_t, c_t, x_init) by implicit
 *    differentiation of the KKT conditions at the solution (Amos et al. 2018).
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *  - no terminal cost: V_T = 0 and x_T is not formed;
 *  - U^0 = clamp(m g / 4) per rotor;
 *  - the stagewise box-QP is solved exactly by enumerating the 3^4 patterns;
 *    among valid patterns the one with the fewest clamped controls wins
 *    (weakly active controls are free);
 *  - the new control is projected onto the box after the affine update;
 *  - the line search always moves to the best candidate (ties go to the
 *    earlier, larger alpha; non-finite cost counts as +inf);
 *  - convergence: ||U^k - U^{k-1}||_inf < tol, only when tol > 0;
 *  - the backward linearises at the returned (x*, u*) and fixes as active every
 *    control that equals a bound exactly.
 */
#include "dmpc_oracle.h"

#include <complex.h>
#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define NX ORC_NX
#define NU ORC_NU
#define NZ ORC_NZ

/* model constants as complex numbers: the complex step in one of them gives
 * the derivative with respect to it (dynamics-parameter gradients) */
typedef struct {
  double _Complex mass, Jxx, Jyy, Jzz, arm, kappa, dt, g;
} orc_params_cx;

/* real instantiation of the dynamics */
#define SC double
#define PT orc_params
#define PSC double
#define FN(n) n##_r
#include "dyn_impl.inc"
#undef SC
#undef PT
#undef PSC
#undef FN
/* complex states, real constants: the complex step in (x, u) */
#define SC double _Complex
#define PT orc_params
#define PSC double
#define FN(n) n##_c
#include "dyn_impl.inc"
#undef SC
#undef PT
#undef PSC
#undef FN
/* complex states and constants: the complex step in a model constant */
#define SC double _Complex
#define PT orc_params_cx
#define PSC double _Complex
#define FN(n) n##_p
#include "dyn_impl.inc"
#undef SC
#undef PT
#undef PSC
#undef FN

static const double kAlphas[ORC_NALPHA] = {1.0, 0.5, 0.25, 0.1};

int orc_alphas(double* out) {
  int i;
  if (out)
    for (i = 0; i < ORC_NALPHA; ++i) out[i] = kAlphas[i];
  return ORC_NALPHA;
}

/* ------------------------------------------------------------------------ */
/* dynamics and its derivatives                                             */
/* ------------------------------------------------------------------------ */

void orc_dyn(const orc_params* P, const double* x, const double* u, double* xdot) { dyn_r(P, x, u, xdot); }

void orc_rk4(const orc_params* P, const double* x, const double* u, double* xn) { rk4_r(P, x, u, xn); }

void orc_rk4_complex_step(const orc_params* P, const double* x, const double* u, const double* dir,
                          double h, double* out) {
  double _Complex xc[NX], uc[NU], yc[NX];
  int i;
  for (i = 0; i < NX; ++i) xc[i] = x[i] + h * dir[i] * _Complex_I;
  for (i = 0; i < NU; ++i) uc[i] = u[i] + h * dir[NX + i] * _Complex_I;
  rk4_c(P, xc, uc, yc);
  for (i = 0; i < NX; ++i) out[i] = cimag(yc[i]) / h;
}

void orc_dyn_jac(const orc_params* P, const double* x, const double* u, double* Fx, double* Fu) {
  dyn_jac_r(P, x, u, Fx, Fu);
}

void orc_rk4_jac(const orc_params* P, const double* x, const double* u, double* A, double* B) {
  rk4_jac_r(P, x, u, A, B);
}

/* ------------------------------------------------------------------------ */
/* small dense linear algebra                                               */
/* ------------------------------------------------------------------------ */

/* Cholesky of the n x n SPD block of H (leading dim ld) selected by idx into
 * L (n x n, row-major lower).  Pivot d_j = H_jj - sum_k L_jk^2 is taken before
 * the square root; if a pivot is not positive the matrix is shifted by
 * 1e-6 max(1, max diag) (repeatedly, x10) and *flags gets ORC_ST_REGULARIZED. */
static void chol_sub(const double* H, int ld, const int* idx, int n, double* L, uint32_t* flags) {
  double shift = 0.0, maxdiag = 1.0;
  int i, j, k, tries;
  for (i = 0; i < n; ++i)
    if (H[idx[i] * ld + idx[i]] > maxdiag) maxdiag = H[idx[i] * ld + idx[i]];
  for (tries = 0; tries < 8; ++tries) {
    int ok = 1;
    for (j = 0; j < n && ok; ++j) {
      double d = H[idx[j] * ld + idx[j]] + shift;
      for (k = 0; k < j; ++k) d -= L[j * n + k] * L[j * n + k];
      if (!(d > 0.0)) {
        ok = 0;
        break;
      }
      L[j * n + j] = sqrt(d);
      for (i = j + 1; i < n; ++i) {
        double e = H[idx[i] * ld + idx[j]];
        for (k = 0; k < j; ++k) e -= L[i * n + k] * L[j * n + k];
        L[i * n + j] = e / L[j * n + j];
      }
      for (i = 0; i < j; ++i) L[i * n + j] = 0.0;
    }
    if (ok) return;
    shift = (shift == 0.0) ? 1e-6 * maxdiag : shift * 10.0;
    if (flags) *flags |= ORC_ST_REGULARIZED;
  }
}

/* solve L L^T y = r in place (n x n lower L) */
static void chol_solve(const double* L, int n, double* r) {
  int i, k;
  for (i = 0; i < n; ++i) {
    double s = r[i];
    for (k = 0; k < i; ++k) s -= L[i * n + k] * r[k];
    r[i] = s / L[i * n + i];
  }
  for (i = n - 1; i >= 0; --i) {
    double s = r[i];
    for (k = i + 1; k < n; ++k) s -= L[k * n + i] * r[k];
    r[i] = s / L[i * n + i];
  }
}

int orc_lu_solve(int n, double* M, double* r) {
  int i, j, k;
  for (k = 0; k < n; ++k) {
    int piv = k;
    double best = fabs(M[(size_t)k * n + k]);
    for (i = k + 1; i < n; ++i) {
      double v = fabs(M[(size_t)i * n + k]);
      if (v > best) {
        best = v;
        piv = i;
      }
    }
    if (best == 0.0) return -1;
    if (piv != k) {
      for (j = 0; j < n; ++j) {
        double t = M[(size_t)k * n + j];
        M[(size_t)k * n + j] = M[(size_t)piv * n + j];
        M[(size_t)piv * n + j] = t;
      }
      {
        double t = r[k];
        r[k] = r[piv];
        r[piv] = t;
      }
    }
    for (i = k + 1; i < n; ++i) {
      double f = M[(size_t)i * n + k] / M[(size_t)k * n + k];
      if (f == 0.0) continue;
      M[(size_t)i * n + k] = 0.0;
      for (j = k + 1; j < n; ++j) M[(size_t)i * n + j] -= f * M[(size_t)k * n + j];
      r[i] -= f * r[k];
    }
  }
  for (i = n - 1; i >= 0; --i) {
    double s = r[i];
    for (j = i + 1; j < n; ++j) s -= M[(size_t)i * n + j] * r[j];
    r[i] = s / M[(size_t)i * n + i];
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* stagewise box-QP (Tassa et al. 2014 problem; solved here by enumeration) */
/* ------------------------------------------------------------------------ */

/* Solve the equality-constrained QP of one pattern: clamped coordinates sit on
 * their bound, the free block solves H_ff d_f = -(q_f + H_fc d_c). */
static void qp_pattern_solve(const double* H, const double* q, const double* a, const double* b,
                             const int32_t* pat, double* d, uint32_t* flags) {
  int idx[NU], nf = 0, i, j;
  double rhs[NU], L[NU * NU];
  for (i = 0; i < NU; ++i) d[i] = (pat[i] == ORC_LOWER) ? a[i] : (pat[i] == ORC_UPPER ? b[i] : 0.0);
  for (i = 0; i < NU; ++i)
    if (pat[i] == ORC_FREE) idx[nf++] = i;
  if (nf == 0) return;
  for (i = 0; i < nf; ++i) {
    double s = q[idx[i]];
    for (j = 0; j < NU; ++j)
      if (pat[j] != ORC_FREE) s += H[idx[i] * NU + j] * d[j];
    rhs[i] = -s;
  }
  chol_sub(H, NU, idx, nf, L, flags);
  chol_solve(L, nf, rhs);
  for (i = 0; i < nf; ++i) d[idx[i]] = rhs[i];
}

/* How far a pattern's solution d (from qp_pattern_solve) is from the
 * optimality conditions of the stagewise box-QP that orc_boxqp enforces: a
 * free coordinate inside [a, b], a coordinate on its lower (upper) bound with
 * a non-negative (non-positive) multiplier g = H d + q.  Returned as the
 * smallest relative tolerance at which every condition holds, in orc_boxqp's
 * scaling (free: violation / (1 + |d_i|); clamped: wrong-signed g_i over the
 * magnitude |q_i| + sum_j |H_ij d_j| of its terms); 0 for a valid pattern.  A
 * coordinate with a_i = b_i is fixed whichever bound the pattern names. */
static double pattern_violation(const double* H, const double* q, const double* a, const double* b,
                                const int32_t* pat, const double* d) {
  double worst = 0.0;
  int i, j;
  for (i = 0; i < NU; ++i) {
    double g = q[i], mag = fabs(q[i]), v = 0.0;
    for (j = 0; j < NU; ++j) {
      g += H[i * NU + j] * d[j];
      mag += fabs(H[i * NU + j] * d[j]);
    }
    if (pat[i] == ORC_FREE) {
      const double out = d[i] < a[i] ? a[i] - d[i] : (d[i] > b[i] ? d[i] - b[i] : 0.0);
      v = out / (1.0 + fabs(d[i]));
    } else if (a[i] < b[i]) {
      const double wrong = (pat[i] == ORC_LOWER) ? -g : g;
      v = wrong > 0.0 ? wrong / (mag > 0.0 ? mag : 1e-300) : 0.0;
    }
    if (!(v <= worst)) worst = v; /* a NaN propagates */
  }
  return worst;
}

uint32_t orc_boxqp(const double* H, const double* q, const double* a, const double* b, double* d,
                   int32_t* pattern) {
  int s, i, j, tier;
  uint32_t flags = 0;
  for (i = 0; i < NU; ++i) {
    int bad = !isfinite(q[i]) || isnan(a[i]) || isnan(b[i]);
    for (j = 0; j < NU; ++j) bad |= !isfinite(H[i * NU + j]);
    if (bad) {
      for (j = 0; j < NU; ++j) {
        d[j] = 0.0;
        pattern[j] = ORC_FREE;
      }
      return ORC_ST_NONFINITE;
    }
  }
  for (tier = 0; tier < 3; ++tier) {
    const double rel = 1e-11 * pow(100.0, tier);
    int best = -1, bestnc = NU + 1;
    double bestd[NU];
    for (s = 0; s < 81; ++s) {
      int32_t pat[NU];
      double dd[NU], g[NU];
      int nc = 0, ok = 1, code = s;
      uint32_t f2 = 0;
      for (i = 0; i < NU; ++i) {
        pat[i] = code % 3;
        code /= 3;
        nc += (pat[i] != ORC_FREE);
      }
      if (nc >= bestnc) continue;
      qp_pattern_solve(H, q, a, b, pat, dd, &f2);
      for (i = 0; i < NU; ++i) {
        double mag = q[i] < 0 ? -q[i] : q[i];
        g[i] = q[i];
        for (j = 0; j < NU; ++j) {
          g[i] += H[i * NU + j] * dd[j];
          mag += fabs(H[i * NU + j] * dd[j]);
        }
        if (pat[i] == ORC_FREE) {
          const double tp = rel * (1.0 + fabs(dd[i]));
          if (!(dd[i] >= a[i] - tp && dd[i] <= b[i] + tp)) ok = 0;
        } else if (pat[i] == ORC_LOWER) {
          if (!(g[i] >= -rel * mag)) ok = 0;
        } else {
          if (!(g[i] <= rel * mag)) ok = 0;
        }
      }
      if (ok) {
        best = s;
        bestnc = nc;
        memcpy(bestd, dd, sizeof dd);
        flags |= f2;
      }
    }
    if (best >= 0) {
      int code = best;
      for (i = 0; i < NU; ++i) {
        pattern[i] = code % 3;
        code /= 3;
        /* free coordinates may sit a rounding error outside the box */
        d[i] = bestd[i] < a[i] ? a[i] : (bestd[i] > b[i] ? b[i] : bestd[i]);
      }
      return flags;
    }
  }
  for (j = 0; j < NU; ++j) {
    d[j] = 0.0 < a[j] ? a[j] : (0.0 > b[j] ? b[j] : 0.0);
    pattern[j] = ORC_FREE;
  }
  return ORC_ST_QPFAIL;
}

/* ------------------------------------------------------------------------ */
/* one problem instance                                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
  int T;
  const orc_params* P;
  int dyn_kind;
  const double* x0; /* 13 */
  const double* lo; /* 4 */
  const double* hi; /* 4 */
  const double* c;  /* T*17 */
  double* C;        /* T*17*17 full, expanded from the input layout */
  const double* Aff;
  const double* Bff;
  const double* rff;
} inst_t;

static int cost_width(int kind) { return kind == ORC_COST_DIAG ? NZ : (kind == ORC_COST_PACKED ? ORC_NPACK : NZ * NZ); }

static void expand_cost(int kind, const double* q, double* C) {
  int i, j, n = 0;
  memset(C, 0, sizeof(double) * NZ * NZ);
  if (kind == ORC_COST_DIAG) {
    for (i = 0; i < NZ; ++i) C[i * NZ + i] = q[i];
  } else if (kind == ORC_COST_PACKED) {
    for (i = 0; i < NZ; ++i)
      for (j = i; j < NZ; ++j) {
        C[i * NZ + j] = q[n];
        C[j * NZ + i] = q[n];
        ++n;
      }
  } else {
    memcpy(C, q, sizeof(double) * NZ * NZ);
  }
}

static void step_dyn(const inst_t* in, int t, const double* x, const double* u, double* xn) {
  if (in->dyn_kind == ORC_DYN_QUAD) {
    rk4_r(in->P, x, u, xn);
  } else {
    const double* A = in->Aff + (size_t)t * NX * NX;
    const double* B = in->Bff + (size_t)t * NX * NU;
    const double* r = in->rff + (size_t)t * NX;
    int i, j;
    for (i = 0; i < NX; ++i) {
      double s = r[i];
      for (j = 0; j < NX; ++j) s += A[i * NX + j] * x[j];
      for (j = 0; j < NU; ++j) s += B[i * NU + j] * u[j];
      xn[i] = s;
    }
  }
}

static void lin_dyn(const inst_t* in, int t, const double* x, const double* u, double* A, double* B) {
  if (in->dyn_kind == ORC_DYN_QUAD) {
    orc_rk4_jac(in->P, x, u, A, B);
  } else {
    memcpy(A, in->Aff + (size_t)t * NX * NX, sizeof(double) * NX * NX);
    memcpy(B, in->Bff + (size_t)t * NX * NU, sizeof(double) * NX * NU);
  }
}

/* 1/2 z^T C z + c^T z */
static double stage_cost(const double* C, const double* c, const double* x, const double* u) {
  double z[NZ], J = 0.0;
  int i, j;
  for (i = 0; i < NX; ++i) z[i] = x[i];
  for (i = 0; i < NU; ++i) z[NX + i] = u[i];
  for (i = 0; i < NZ; ++i) {
    double s = 0.0;
    for (j = 0; j < NZ; ++j) s += C[i * NZ + j] * z[j];
    J += 0.5 * z[i] * s + c[i] * z[i];
  }
  return J;
}

static double clampd(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* X from x0 and U by the dynamics (Alg. 2, Rollout) */
static void rollout(const inst_t* in, const double* U, double* X) {
  int t;
  memcpy(X, in->x0, sizeof(double) * NX);
  for (t = 0; t + 1 < in->T; ++t) step_dyn(in, t, X + t * NX, U + t * NU, X + (t + 1) * NX);
}

static double traj_cost(const inst_t* in, const double* X, const double* U) {
  double J = 0.0;
  int t;
  for (t = 0; t < in->T; ++t) J += stage_cost(in->C + (size_t)t * NZ * NZ, in->c + t * NZ, X + t * NX, U + t * NU);
  return J;
}

/* Q = C + F^T V F and q = g + F^T v for F = [A | B]; with_dyn = 0 at the
 * last stage (V_{t+1} = 0, no dynamics out of it). */
static void stage_q(const double* C, const double* g, const double* A, const double* B, const double* V,
                    const double* v, int with_dyn, double* Q, double* q) {
  int i, j, k, l;
  memcpy(Q, C, sizeof(double) * NZ * NZ);
  memcpy(q, g, sizeof(double) * NZ);
  if (!with_dyn) return;
  {
    double F[NX * NZ], VF[NX * NZ];
    for (i = 0; i < NX; ++i) {
      for (j = 0; j < NX; ++j) F[i * NZ + j] = A[i * NX + j];
      for (j = 0; j < NU; ++j) F[i * NZ + NX + j] = B[i * NU + j];
    }
    for (i = 0; i < NX; ++i)
      for (j = 0; j < NZ; ++j) {
        double s = 0.0;
        for (k = 0; k < NX; ++k) s += V[i * NX + k] * F[k * NZ + j];
        VF[i * NZ + j] = s;
      }
    for (i = 0; i < NZ; ++i)
      for (j = 0; j < NZ; ++j) {
        double s = 0.0;
        for (l = 0; l < NX; ++l) s += F[l * NZ + i] * VF[l * NZ + j];
        Q[i * NZ + j] += s;
      }
    for (i = 0; i < NZ; ++i) {
      double s = 0.0;
      for (l = 0; l < NX; ++l) s += F[l * NZ + i] * v[l];
      q[i] += s;
    }
  }
}

/* Given the stage Q, q, a free set and the control step k, form the gain K
 * (zero rows on clamped controls) and update the value function:
 *   K_f = -Q_uu,ff^{-1} Q_ux,f
 *   V = Q_xx + K^T Q_uu K + K^T Q_ux + Q_ux^T K,  then V <- (V + V^T)/2
 *   v = Q_x + K^T Q_uu k + K^T Q_u + Q_ux^T k
 * (Tassa et al. 2014, control-limited value update). */
static void gain_and_value(const double* Q, const double* q, const int* isfree, const double* k, double* K,
                           double* V, double* v, uint32_t* flags) {
  double Quu[NU * NU], Qux[NU * NX], L[NU * NU];
  int idx[NU], nf = 0, i, j, a, b2;
  for (a = 0; a < NU; ++a) {
    for (b2 = 0; b2 < NU; ++b2) Quu[a * NU + b2] = Q[(NX + a) * NZ + NX + b2];
    for (j = 0; j < NX; ++j) Qux[a * NX + j] = Q[(NX + a) * NZ + j];
  }
  for (a = 0; a < NU; ++a)
    if (isfree[a]) idx[nf++] = a;
  memset(K, 0, sizeof(double) * NU * NX);
  if (nf > 0) {
    chol_sub(Quu, NU, idx, nf, L, flags);
    for (j = 0; j < NX; ++j) {
      double col[NU];
      for (i = 0; i < nf; ++i) col[i] = Qux[idx[i] * NX + j];
      chol_solve(L, nf, col);
      for (i = 0; i < nf; ++i) K[idx[i] * NX + j] = -col[i];
    }
  }
  {
    double QuuK[NU * NX], Vn[NX * NX], Quuk[NU];
    for (a = 0; a < NU; ++a) {
      for (j = 0; j < NX; ++j) {
        double s = 0.0;
        for (b2 = 0; b2 < NU; ++b2) s += Quu[a * NU + b2] * K[b2 * NX + j];
        QuuK[a * NX + j] = s;
      }
      {
        double s = 0.0;
        for (b2 = 0; b2 < NU; ++b2) s += Quu[a * NU + b2] * k[b2];
        Quuk[a] = s;
      }
    }
    for (i = 0; i < NX; ++i)
      for (j = 0; j < NX; ++j) {
        double s = Q[i * NZ + j];
        for (a = 0; a < NU; ++a)
          s += K[a * NX + i] * QuuK[a * NX + j] + K[a * NX + i] * Qux[a * NX + j] + Qux[a * NX + i] * K[a * NX + j];
        Vn[i * NX + j] = s;
      }
    for (i = 0; i < NX; ++i)
      for (j = 0; j < NX; ++j) V[i * NX + j] = 0.5 * (Vn[i * NX + j] + Vn[j * NX + i]);
    for (i = 0; i < NX; ++i) {
      double s = q[i];
      for (a = 0; a < NU; ++a) s += K[a * NX + i] * Quuk[a] + K[a * NX + i] * q[NX + a] + Qux[a * NX + i] * k[a];
      v[i] = s;
    }
  }
}

typedef struct {
  int K;
  double tol;
  const double* u_init; /* T*4 or NULL */
  int replay;           /* 0 free run */
  int replay_iters;
  const uint8_t* replay_alpha;   /* K */
  const uint8_t* replay_pattern; /* K*Tmax */
  int Tmax;
  /* outputs */
  double* U; /* T*4 */
  double* X; /* T*13 */
  double J;
  int iters;
  uint32_t status;
  uint8_t* alpha_log;   /* K or NULL */
  uint8_t* pattern_log; /* K*Tmax or NULL */
  double* cand_cost;    /* K*4 or NULL */
  double* replay_viol;  /* K*Tmax or NULL: pattern_violation of each replayed stage pattern */
} ilqr_io;

static void ilqr_one(const inst_t* in, ilqr_io* io) {
  const int T = in->T;
  double *Xn, *Un, *Kg, *kf, *Ac, *Bc, *Xc, *Uc;
  int k, t, i, j;
  io->status = 0;
  io->iters = 0;
  io->J = 0.0;
  if (T <= 0) return;
  Xn = io->X;
  Un = io->U;
  Kg = (double*)calloc((size_t)T * NU * NX, sizeof(double));
  kf = (double*)calloc((size_t)T * NU, sizeof(double));
  Ac = (double*)calloc((size_t)T * NX * NX, sizeof(double));
  Bc = (double*)calloc((size_t)T * NX * NU, sizeof(double));
  Xc = (double*)calloc((size_t)ORC_NALPHA * T * NX, sizeof(double));
  Uc = (double*)calloc((size_t)ORC_NALPHA * T * NU, sizeof(double));

  /* initial nominal: U^0 then X^0 by rollout */
  for (t = 0; t < T; ++t)
    for (i = 0; i < NU; ++i) {
      double u0 = io->u_init ? io->u_init[t * NU + i]
                             : (in->dyn_kind == ORC_DYN_QUAD ? in->P->mass * in->P->g / 4.0 : 0.0);
      Un[t * NU + i] = clampd(u0, in->lo[i], in->hi[i]);
    }
  rollout(in, Un, Xn);
  io->J = traj_cost(in, Xn, Un);

  {
    const int K = io->replay ? io->replay_iters : io->K;
    int converged = 0;
    for (k = 0; k < K; ++k) {
      double V[NX * NX], v[NX];
      /* (a) LQ: linearise the dynamics along the nominal */
      for (t = 0; t + 1 < T; ++t) lin_dyn(in, t, Xn + t * NX, Un + t * NU, Ac + t * NX * NX, Bc + t * NX * NU);
      /* (b) backward pass with input bounds */
      memset(V, 0, sizeof V);
      memset(v, 0, sizeof v);
      for (t = T - 1; t >= 0; --t) {
        const double* C = in->C + (size_t)t * NZ * NZ;
        double g[NZ], Q[NZ * NZ], q[NZ], z[NZ], H[NU * NU], qu[NU], a[NU], b[NU], d[NU];
        int32_t pat[NU];
        int isfree[NU];
        for (i = 0; i < NX; ++i) z[i] = Xn[t * NX + i];
        for (i = 0; i < NU; ++i) z[NX + i] = Un[t * NU + i];
        for (i = 0; i < NZ; ++i) {
          double s = in->c[t * NZ + i];
          for (j = 0; j < NZ; ++j) s += C[i * NZ + j] * z[j];
          g[i] = s;
        }
        stage_q(C, g, Ac + t * NX * NX, Bc + t * NX * NU, V, v, t + 1 < T, Q, q);
        for (i = 0; i < NU; ++i) {
          for (j = 0; j < NU; ++j) H[i * NU + j] = Q[(NX + i) * NZ + NX + j];
          qu[i] = q[NX + i];
          a[i] = in->lo[i] - Un[t * NU + i];
          b[i] = in->hi[i] - Un[t * NU + i];
        }
        if (io->replay) {
          uint8_t code = io->replay_pattern[(size_t)k * io->Tmax + t];
          for (i = 0; i < NU; ++i) pat[i] = (code >> (2 * i)) & 3;
          qp_pattern_solve(H, qu, a, b, pat, d, &io->status);
          /* score the replayed pattern against this stage's own QP before the
           * step is clamped into the box (the clamp would hide a wrong one) */
          if (io->replay_viol) io->replay_viol[(size_t)k * io->Tmax + t] = pattern_violation(H, qu, a, b, pat, d);
          for (i = 0; i < NU; ++i) d[i] = clampd(d[i], a[i], b[i]);
        } else {
          io->status |= orc_boxqp(H, qu, a, b, d, pat);
        }
        for (i = 0; i < NU; ++i) isfree[i] = (pat[i] == ORC_FREE);
        if (io->pattern_log) {
          uint8_t code = 0;
          for (i = 0; i < NU; ++i) code |= (uint8_t)(pat[i] << (2 * i));
          io->pattern_log[(size_t)k * io->Tmax + t] = code;
        }
        memcpy(kf + t * NU, d, sizeof d);
        gain_and_value(Q, q, isfree, d, Kg + (size_t)t * NU * NX, V, v, &io->status);
      }
      /* (c) forward pass with line search over the four candidates */
      {
        double Jc[ORC_NALPHA];
        int ai, best = -1;
        for (ai = 0; ai < ORC_NALPHA; ++ai) {
          double* X = Xc + (size_t)ai * T * NX;
          double* U = Uc + (size_t)ai * T * NU;
          memcpy(X, in->x0, sizeof(double) * NX);
          for (t = 0; t < T; ++t) {
            for (i = 0; i < NU; ++i) {
              double s = Un[t * NU + i] + kAlphas[ai] * kf[t * NU + i];
              for (j = 0; j < NX; ++j) s += Kg[(size_t)t * NU * NX + i * NX + j] * (X[t * NX + j] - Xn[t * NX + j]);
              U[t * NU + i] = clampd(s, in->lo[i], in->hi[i]);
            }
            if (t + 1 < T) step_dyn(in, t, X + t * NX, U + t * NU, X + (t + 1) * NX);
          }
          Jc[ai] = traj_cost(in, X, U);
          if (!isfinite(Jc[ai])) Jc[ai] = INFINITY;
          if (io->cand_cost) io->cand_cost[k * ORC_NALPHA + ai] = Jc[ai];
        }
        if (io->replay) {
          best = io->replay_alpha[k] == ORC_ALPHA_NONE ? -1 : (int)io->replay_alpha[k];
        } else {
          for (ai = 0; ai < ORC_NALPHA; ++ai)
            if (Jc[ai] < INFINITY && (best < 0 || Jc[ai] < Jc[best])) best = ai;
        }
        if (io->alpha_log) io->alpha_log[k] = best < 0 ? ORC_ALPHA_NONE : (uint8_t)best;
        io->iters = k + 1;
        if (best < 0) {
          io->status |= ORC_ST_NONFINITE;
        } else {
          double du = 0.0;
          const double* U = Uc + (size_t)best * T * NU;
          for (i = 0; i < T * NU; ++i) {
            double e = fabs(U[i] - Un[i]);
            if (e > du) du = e;
          }
          memcpy(Un, U, sizeof(double) * T * NU);
          memcpy(Xn, Xc + (size_t)best * T * NX, sizeof(double) * T * NX);
          io->J = Jc[best];
          /* (d) convergence test */
          if (!io->replay && io->tol > 0.0 && du < io->tol) {
            converged = 1;
            break;
          }
        }
      }
    }
    if (converged) io->status |= ORC_ST_CONVERGED;
    else if (io->tol > 0.0 && !io->replay) io->status |= ORC_ST_MAXITER;
  }
  free(Kg);
  free(kf);
  free(Ac);
  free(Bc);
  free(Xc);
  free(Uc);
}

/* ------------------------------------------------------------------------ */
/* backward: implicit differentiation at the solution                       */
/* ------------------------------------------------------------------------ */

/* Riccati adjoint: solve the LQR with costs C_t, linear term d_t = dL/dz*_t,
 * homogeneous linearised dynamics, x~_0 = 0 and the active controls fixed at
 * zero.  Its solution z~ is dL/dc; its value gradient v_0 is dL/dx_init. */
static void bwd_riccati_one(const inst_t* in, const double* Xs, const double* Us, const int* act, const double* d,
                            double* zt, double* dx0) {
  const int T = in->T;
  double* A = (double*)calloc((size_t)T * NX * NX, sizeof(double));
  double* B = (double*)calloc((size_t)T * NX * NU, sizeof(double));
  double* Kg = (double*)calloc((size_t)T * NU * NX, sizeof(double));
  double* kf = (double*)calloc((size_t)T * NU, sizeof(double));
  double V[NX * NX], v[NX], xt[NX];
  int t, i, j;
  uint32_t dummy = 0;
  for (t = 0; t + 1 < T; ++t) lin_dyn(in, t, Xs + t * NX, Us + t * NU, A + t * NX * NX, B + t * NX * NU);
  memset(V, 0, sizeof V);
  memset(v, 0, sizeof v);
  for (t = T - 1; t >= 0; --t) {
    double Q[NZ * NZ], q[NZ], k[NU];
    int isfree[NU], idx[NU], nf = 0;
    stage_q(in->C + (size_t)t * NZ * NZ, d + t * NZ, A + t * NX * NX, B + t * NX * NU, V, v, t + 1 < T, Q, q);
    for (i = 0; i < NU; ++i) {
      isfree[i] = !act[t * NU + i];
      k[i] = 0.0;
      if (isfree[i]) idx[nf++] = i;
    }
    if (nf > 0) {
      double Quu[NU * NU], L[NU * NU], rhs[NU];
      for (i = 0; i < NU; ++i)
        for (j = 0; j < NU; ++j) Quu[i * NU + j] = Q[(NX + i) * NZ + NX + j];
      chol_sub(Quu, NU, idx, nf, L, &dummy);
      for (i = 0; i < nf; ++i) rhs[i] = -q[NX + idx[i]];
      chol_solve(L, nf, rhs);
      for (i = 0; i < nf; ++i) k[idx[i]] = rhs[i];
    }
    memcpy(kf + t * NU, k, sizeof k);
    gain_and_value(Q, q, isfree, k, Kg + (size_t)t * NU * NX, V, v, &dummy);
  }
  memcpy(dx0, v, sizeof v);
  memset(xt, 0, sizeof xt);
  for (t = 0; t < T; ++t) {
    double ut[NU], xn[NX];
    for (i = 0; i < NU; ++i) {
      double s = kf[t * NU + i];
      for (j = 0; j < NX; ++j) s += Kg[(size_t)t * NU * NX + i * NX + j] * xt[j];
      ut[i] = s;
    }
    for (i = 0; i < NX; ++i) zt[t * NZ + i] = xt[i];
    for (i = 0; i < NU; ++i) zt[t * NZ + NX + i] = ut[i];
    if (t + 1 < T) {
      for (i = 0; i < NX; ++i) {
        double s = 0.0;
        for (j = 0; j < NX; ++j) s += A[t * NX * NX + i * NX + j] * xt[j];
        for (j = 0; j < NU; ++j) s += B[t * NX * NU + i * NU + j] * ut[j];
        xn[i] = s;
      }
      memcpy(xt, xn, sizeof xn);
    }
  }
  free(A);
  free(B);
  free(Kg);
  free(kf);
}

/* Dense KKT: unknowns (z_0..z_{T-1}; nu).  Constraint rows: x_0 = x_init;
 * x_{t+1} - A_t x_t - B_t u_t = r_t; u_{t,i} = bound for each active (t,i).
 * Solve [H G^T; G 0][d_z; d_nu] = [-dL/dz; 0] with H = blockdiag(C_t).
 * Then dL/dc = d_z and dL/dx_init = -d_nu(x_0 rows). */
static int bwd_kkt_one(const inst_t* in, const double* Xs, const double* Us, const int* act, const double* d,
                       double* zt, double* dx0) {
  const int T = in->T;
  int nact = 0, t, i, j, a, rc;
  for (t = 0; t < T; ++t)
    for (a = 0; a < NU; ++a) nact += act[t * NU + a] ? 1 : 0;
  {
    const int nz = NZ * T, nc = NX * T + nact, n = nz + nc;
    double* M = (double*)calloc((size_t)n * n, sizeof(double));
    double* r = (double*)calloc((size_t)n, sizeof(double));
    double A[NX * NX], B[NX * NU];
    int row = nz;
    for (t = 0; t < T; ++t)
      for (i = 0; i < NZ; ++i) {
        for (j = 0; j < NZ; ++j) M[(size_t)(t * NZ + i) * n + t * NZ + j] = in->C[(size_t)t * NZ * NZ + i * NZ + j];
        r[t * NZ + i] = -d[t * NZ + i];
      }
    /* G and G^T entries are written symmetrically */
#define GSET(rw, col, val)                  \
  do {                                      \
    M[(size_t)(rw) * n + (col)] = (val);    \
    M[(size_t)(col) * n + (rw)] = (val);    \
  } while (0)
    for (i = 0; i < NX; ++i) GSET(row + i, i, 1.0);
    row += NX;
    for (t = 0; t + 1 < T; ++t) {
      lin_dyn(in, t, Xs + t * NX, Us + t * NU, A, B);
      for (i = 0; i < NX; ++i) {
        GSET(row + i, (t + 1) * NZ + i, 1.0);
        for (j = 0; j < NX; ++j) GSET(row + i, t * NZ + j, -A[i * NX + j]);
        for (j = 0; j < NU; ++j) GSET(row + i, t * NZ + NX + j, -B[i * NU + j]);
      }
      row += NX;
    }
    for (t = 0; t < T; ++t)
      for (a = 0; a < NU; ++a)
        if (act[t * NU + a]) {
          GSET(row, t * NZ + NX + a, 1.0);
          ++row;
        }
#undef GSET
    rc = orc_lu_solve(n, M, r);
    for (i = 0; i < nz; ++i) zt[i] = r[i];
    for (i = 0; i < NX; ++i) dx0[i] = -r[nz + i];
    free(M);
    free(r);
  }
  return rc;
}

/* The model constants with the imaginary step ih added to the j-th one
 * (order of orc_params: mass, Jxx, Jyy, Jzz, arm, kappa, dt, g). */
static void params_step(const orc_params* P, int j, double h, orc_params_cx* Pc) {
  const double _Complex ih = h * _Complex_I;
  Pc->mass = P->mass + (j == 0 ? ih : 0.0);
  Pc->Jxx = P->Jxx + (j == 1 ? ih : 0.0);
  Pc->Jyy = P->Jyy + (j == 2 ? ih : 0.0);
  Pc->Jzz = P->Jzz + (j == 3 ? ih : 0.0);
  Pc->arm = P->arm + (j == 4 ? ih : 0.0);
  Pc->kappa = P->kappa + (j == 5 ? ih : 0.0);
  Pc->dt = P->dt + (j == 6 ? ih : 0.0);
  Pc->g = P->g + (j == 7 ? ih : 0.0);
}

/* Gradient with respect to the model constants theta.  The backward
 * differentiates the LQ problem of the model linearised at the solution,
 * x_{t+1} = F_t z_t + f_t with F_t = df/dz(z*_t; theta) and
 * f_t = f(z*_t; theta) - F_t z*_t.  Amos et al.'s gradients with respect to
 * F_t and f_t, carried to theta by the chain rule, give
 *   dL/dtheta = sum_{t < T-1}  lt_{t+1}^T df/dtheta(z*_t) + ls_{t+1}^T d(F_t zt_t)/dtheta,
 * where zt = dL/dc is the adjoint LQ solution and lt, ls are the costates of
 * the adjoint solution and of the solution itself:
 *   lt_t = (C_t zt_t + d_t)_x + A_t^T lt_{t+1},   ls_t = (C_t z*_t + c_t)_x + A_t^T ls_{t+1},
 * with l_T = 0 (d = dL/dz*).  df/dtheta and d(F zt)/dtheta come from the
 * complex step in each constant, through the RK4 map and its exact Jacobian. */
static void theta_grad_one(const inst_t* in, const double* Xs, const double* Us, const double* zt, const double* d,
                           double* dth) {
  const int T = in->T;
  const double h = 1e-30;
  double lt[NX], ls[NX], nt[NX], ns[NX], A[NX * NX], B[NX * NU];
  int t, i, j, k;
  for (j = 0; j < ORC_NTHETA; ++j) dth[j] = 0.0;
  memset(lt, 0, sizeof lt);
  memset(ls, 0, sizeof ls);
  for (t = T - 1; t >= 0; --t) {
    const double* C = in->C + (size_t)t * NZ * NZ;
    double zs[NZ];
    for (i = 0; i < NX; ++i) zs[i] = Xs[t * NX + i];
    for (i = 0; i < NU; ++i) zs[NX + i] = Us[t * NU + i];
    if (t + 1 < T) {
      /* lt, ls hold l_{t+1} here */
      double _Complex xc[NX], uc[NU], yc[NX], Ac[NX * NX], Bc[NX * NU];
      for (i = 0; i < NX; ++i) xc[i] = zs[i];
      for (i = 0; i < NU; ++i) uc[i] = zs[NX + i];
      for (j = 0; j < ORC_NTHETA; ++j) {
        orc_params_cx Pc;
        double acc = 0.0;
        params_step(in->P, j, h, &Pc);
        rk4_p(&Pc, xc, uc, yc);
        rk4_jac_p(&Pc, xc, uc, Ac, Bc);
        for (i = 0; i < NX; ++i) {
          double _Complex fz = 0.0;
          for (k = 0; k < NX; ++k) fz += Ac[i * NX + k] * zt[t * NZ + k];
          for (k = 0; k < NU; ++k) fz += Bc[i * NU + k] * zt[t * NZ + NX + k];
          acc += lt[i] * (cimag(yc[i]) / h) + ls[i] * (cimag(fz) / h);
        }
        dth[j] += acc;
      }
      orc_rk4_jac(in->P, zs, zs + NX, A, B);
    }
    /* costates of stage t */
    for (i = 0; i < NX; ++i) {
      double gt = d[t * NZ + i], gs = in->c[t * NZ + i];
      for (k = 0; k < NZ; ++k) {
        gt += C[i * NZ + k] * zt[t * NZ + k];
        gs += C[i * NZ + k] * zs[k];
      }
      if (t + 1 < T)
        for (k = 0; k < NX; ++k) {
          gt += A[k * NX + i] * lt[k];
          gs += A[k * NX + i] * ls[k];
        }
      nt[i] = gt;
      ns[i] = gs;
    }
    memcpy(lt, nt, sizeof lt);
    memcpy(ls, ns, sizeof ls);
  }
}

/* ------------------------------------------------------------------------ */
/* batched drivers                                                          */
/* ------------------------------------------------------------------------ */

typedef struct {
  const orc_config* cfg;
  const orc_params* P;
  const double *x0, *Q, *p, *lo, *hi, *Aff, *Bff, *rff, *u_init;
  const int32_t* T;
  /* forward */
  const int32_t* replay_iters;
  const uint8_t *replay_alpha, *replay_pattern;
  double *u_out, *x_out, *J_out, *cand_cost, *replay_viol;
  int32_t* iters_out;
  uint32_t* status_out;
  uint8_t *alpha_log, *pattern_log;
  /* backward */
  const double *u_star, *x_star, *grad_u, *grad_x;
  const uint8_t* mask;
  int32_t method;
  double *dQ, *dp, *dx0, *dtheta;
  int rc;
  /* partition */
  int b0, b1;
} job_t;

static void make_inst(const job_t* jb, int b, inst_t* in) {
  const orc_config* cfg = jb->cfg;
  const int Tm = cfg->T_max, w = cost_width(cfg->cost_kind);
  int t;
  in->T = jb->T ? jb->T[b] : Tm;
  if (in->T > Tm) in->T = Tm;
  if (in->T < 0) in->T = 0;
  in->P = jb->P;
  in->dyn_kind = cfg->dyn_kind;
  in->x0 = jb->x0 + (size_t)b * NX;
  in->lo = jb->lo + (size_t)b * NU;
  in->hi = jb->hi + (size_t)b * NU;
  in->c = jb->p + (size_t)b * Tm * NZ;
  in->C = (double*)calloc((size_t)(Tm > 0 ? Tm : 1) * NZ * NZ, sizeof(double));
  for (t = 0; t < in->T; ++t) expand_cost(cfg->cost_kind, jb->Q + ((size_t)b * Tm + t) * w, in->C + (size_t)t * NZ * NZ);
  in->Aff = jb->Aff ? jb->Aff + (size_t)b * Tm * NX * NX : NULL;
  in->Bff = jb->Bff ? jb->Bff + (size_t)b * Tm * NX * NU : NULL;
  in->rff = jb->rff ? jb->rff + (size_t)b * Tm * NX : NULL;
}

static void* fwd_worker(void* arg) {
  job_t* jb = (job_t*)arg;
  const orc_config* cfg = jb->cfg;
  const int Tm = cfg->T_max, K = cfg->max_iter;
  int b;
  for (b = jb->b0; b < jb->b1; ++b) {
    inst_t in;
    ilqr_io io;
    double* U = (double*)calloc((size_t)(Tm > 0 ? Tm : 1) * NU, sizeof(double));
    double* X = (double*)calloc((size_t)(Tm > 0 ? Tm : 1) * NX, sizeof(double));
    make_inst(jb, b, &in);
    memset(&io, 0, sizeof io);
    io.K = K;
    io.tol = cfg->tol;
    io.Tmax = Tm;
    io.u_init = jb->u_init ? jb->u_init + (size_t)b * Tm * NU : NULL;
    if (jb->replay_iters) {
      io.replay = 1;
      io.replay_iters = jb->replay_iters[b];
      if (io.replay_iters > K) io.replay_iters = K;
      io.replay_alpha = jb->replay_alpha + (size_t)b * K;
      io.replay_pattern = jb->replay_pattern + (size_t)b * K * Tm;
    }
    io.U = U;
    io.X = X;
    io.alpha_log = jb->alpha_log ? jb->alpha_log + (size_t)b * K : NULL;
    io.pattern_log = jb->pattern_log ? jb->pattern_log + (size_t)b * K * Tm : NULL;
    io.cand_cost = jb->cand_cost ? jb->cand_cost + (size_t)b * K * ORC_NALPHA : NULL;
    io.replay_viol = (jb->replay_viol && io.replay) ? jb->replay_viol + (size_t)b * K * Tm : NULL;
    if (jb->replay_viol) {
      int i;
      for (i = 0; i < K * Tm; ++i) jb->replay_viol[(size_t)b * K * Tm + i] = 0.0;
    }
    if (io.alpha_log) memset(io.alpha_log, ORC_ALPHA_NONE, (size_t)K);
    if (io.pattern_log) memset(io.pattern_log, 0, (size_t)K * Tm);
    if (io.cand_cost) {
      int i;
      for (i = 0; i < K * ORC_NALPHA; ++i) io.cand_cost[i] = NAN;
    }
    ilqr_one(&in, &io);
    if (jb->u_out) memcpy(jb->u_out + (size_t)b * Tm * NU, U, sizeof(double) * Tm * NU);
    if (jb->x_out) memcpy(jb->x_out + (size_t)b * Tm * NX, X, sizeof(double) * Tm * NX);
    if (jb->J_out) jb->J_out[b] = io.J;
    if (jb->iters_out) jb->iters_out[b] = io.iters;
    if (jb->status_out) jb->status_out[b] = io.status;
    free(in.C);
    free(U);
    free(X);
  }
  return NULL;
}

static void* bwd_worker(void* arg) {
  job_t* jb = (job_t*)arg;
  const orc_config* cfg = jb->cfg;
  const int Tm = cfg->T_max, w = cost_width(cfg->cost_kind);
  int b, t, i, j;
  for (b = jb->b0; b < jb->b1; ++b) {
    inst_t in;
    const size_t one = (size_t)(Tm > 0 ? Tm : 1);
    int* act = (int*)calloc(one * NU, sizeof(int));
    double* d = (double*)calloc(one * NZ, sizeof(double));
    double* zt = (double*)calloc(one * NZ, sizeof(double));
    double g0[NX];
    const double* Us = jb->u_star + (size_t)b * Tm * NU;
    const double* Xs = jb->x_star + (size_t)b * Tm * NX;
    double* dQb = jb->dQ ? jb->dQ + (size_t)b * Tm * w : NULL;
    double* dpb = jb->dp ? jb->dp + (size_t)b * Tm * NZ : NULL;
    make_inst(jb, b, &in);
    for (t = 0; t < in.T; ++t)
      for (i = 0; i < NU; ++i) {
        if (jb->mask)
          act[t * NU + i] = (jb->mask[(size_t)b * Tm + t] >> i) & 1;
        else
          act[t * NU + i] = (Us[t * NU + i] == in.lo[i]) || (Us[t * NU + i] == in.hi[i]);
      }
    for (t = 0; t < in.T; ++t) {
      for (i = 0; i < NX; ++i) d[t * NZ + i] = jb->grad_x ? jb->grad_x[((size_t)b * Tm + t) * NX + i] : 0.0;
      for (i = 0; i < NU; ++i) d[t * NZ + NX + i] = jb->grad_u[((size_t)b * Tm + t) * NU + i];
    }
    memset(g0, 0, sizeof g0);
    if (in.T > 0) {
      if (jb->method == 1) {
        if (bwd_kkt_one(&in, Xs, Us, act, d, zt, g0) != 0) jb->rc = -1;
      } else {
        bwd_riccati_one(&in, Xs, Us, act, d, zt, g0);
      }
    }
    if (jb->dx0) memcpy(jb->dx0 + (size_t)b * NX, g0, sizeof g0);
    if (jb->dtheta) {
      double* o = jb->dtheta + (size_t)b * ORC_NTHETA;
      if (in.T > 0)
        theta_grad_one(&in, Xs, Us, zt, d, o);
      else
        for (i = 0; i < ORC_NTHETA; ++i) o[i] = 0.0;
    }
    if (dpb) {
      memset(dpb, 0, sizeof(double) * Tm * NZ);
      memcpy(dpb, zt, sizeof(double) * in.T * NZ);
    }
    if (dQb) {
      memset(dQb, 0, sizeof(double) * Tm * w);
      for (t = 0; t < in.T; ++t) {
        double zs[NZ];
        const double* zz = zt + t * NZ;
        double* o = dQb + (size_t)t * w;
        for (i = 0; i < NX; ++i) zs[i] = Xs[t * NX + i];
        for (i = 0; i < NU; ++i) zs[NX + i] = Us[t * NU + i];
        if (cfg->cost_kind == ORC_COST_DIAG) {
          for (i = 0; i < NZ; ++i) o[i] = zz[i] * zs[i];
        } else if (cfg->cost_kind == ORC_COST_PACKED) {
          int n = 0;
          for (i = 0; i < NZ; ++i)
            for (j = i; j < NZ; ++j) o[n++] = (i == j) ? zz[i] * zs[i] : zz[i] * zs[j] + zz[j] * zs[i];
        } else {
          for (i = 0; i < NZ; ++i)
            for (j = 0; j < NZ; ++j) o[i * NZ + j] = 0.5 * (zz[i] * zs[j] + zz[j] * zs[i]);
        }
      }
    }
    free(in.C);
    free(act);
    free(d);
    free(zt);
  }
  return NULL;
}

static int run_jobs(job_t* proto, void* (*fn)(void*)) {
  int nt = proto->cfg->nthreads < 1 ? 1 : proto->cfg->nthreads;
  const int B = proto->cfg->B;
  int i, rc = 0;
  job_t* jobs;
  pthread_t* th;
  if (B <= 0) return 0;
  if (nt > B) nt = B;
  jobs = (job_t*)calloc((size_t)nt, sizeof(job_t));
  th = (pthread_t*)calloc((size_t)nt, sizeof(pthread_t));
  for (i = 0; i < nt; ++i) {
    jobs[i] = *proto;
    jobs[i].rc = 0;
    jobs[i].b0 = (int)((long long)B * i / nt);
    jobs[i].b1 = (int)((long long)B * (i + 1) / nt);
  }
  if (nt == 1) {
    fn(&jobs[0]);
  } else {
    for (i = 0; i < nt; ++i) pthread_create(&th[i], NULL, fn, &jobs[i]);
    for (i = 0; i < nt; ++i) pthread_join(th[i], NULL);
  }
  for (i = 0; i < nt; ++i)
    if (jobs[i].rc) rc = jobs[i].rc;
  free(jobs);
  free(th);
  return rc;
}

static int check_cfg(const orc_config* cfg) {
  if (!cfg || cfg->B < 0 || cfg->T_max < 0 || cfg->max_iter < 0) return -1;
  if (cfg->cost_kind < 0 || cfg->cost_kind > 2 || cfg->dyn_kind < 0 || cfg->dyn_kind > 1) return -1;
  return 0;
}

int orc_forward(const orc_config* cfg, const orc_params* P, const double* x0, const double* Q,
                const double* p, const double* lo, const double* hi, const int32_t* T,
                const double* Aff, const double* Bff, const double* rff, const double* u_init,
                const int32_t* replay_iters, const uint8_t* replay_alpha, const uint8_t* replay_pattern,
                double* u_out, double* x_out, double* J_out, int32_t* iters_out, uint32_t* status_out,
                uint8_t* alpha_log, uint8_t* pattern_log, double* cand_cost, double* replay_viol) {
  job_t jb;
  if (check_cfg(cfg)) return -1;
  if (cfg->dyn_kind == ORC_DYN_AFFINE && (!Aff || !Bff || !rff)) return -1;
  if (replay_iters && (!replay_alpha || !replay_pattern)) return -1;
  memset(&jb, 0, sizeof jb);
  jb.cfg = cfg;
  jb.P = P;
  jb.x0 = x0;
  jb.Q = Q;
  jb.p = p;
  jb.lo = lo;
  jb.hi = hi;
  jb.T = T;
  jb.Aff = Aff;
  jb.Bff = Bff;
  jb.rff = rff;
  jb.u_init = u_init;
  jb.replay_iters = replay_iters;
  jb.replay_alpha = replay_alpha;
  jb.replay_pattern = replay_pattern;
  jb.u_out = u_out;
  jb.x_out = x_out;
  jb.J_out = J_out;
  jb.iters_out = iters_out;
  jb.status_out = status_out;
  jb.alpha_log = alpha_log;
  jb.pattern_log = pattern_log;
  jb.cand_cost = cand_cost;
  jb.replay_viol = replay_viol;
  return run_jobs(&jb, fwd_worker);
}

int orc_backward(const orc_config* cfg, const orc_params* P, const double* x0, const double* Q,
                 const double* p, const double* lo, const double* hi, const int32_t* T,
                 const double* Aff, const double* Bff, const double* rff, const double* u_star,
                 const double* x_star, const uint8_t* mask, const double* grad_u, const double* grad_x,
                 int32_t method, double* dQ, double* dp, double* dx0, double* dtheta) {
  job_t jb;
  if (check_cfg(cfg) || !u_star || !x_star || !grad_u) return -1;
  if (cfg->dyn_kind == ORC_DYN_AFFINE && (!Aff || !Bff || !rff)) return -1;
  if (cfg->dyn_kind == ORC_DYN_AFFINE && dtheta) return -1; /* no model constants */
  memset(&jb, 0, sizeof jb);
  jb.cfg = cfg;
  jb.P = P;
  jb.x0 = x0;
  jb.Q = Q;
  jb.p = p;
  jb.lo = lo;
  jb.hi = hi;
  jb.T = T;
  jb.Aff = Aff;
  jb.Bff = Bff;
  jb.rff = rff;
  jb.u_star = u_star;
  jb.x_star = x_star;
  jb.mask = mask;
  jb.grad_u = grad_u;
  jb.grad_x = grad_x;
  jb.method = method;
  jb.dQ = dQ;
  jb.dp = dp;
  jb.dx0 = dx0;
  jb.dtheta = dtheta;
  return run_jobs(&jb, bwd_worker);
}
