/*
 * dmpc.h -- C ABI of the batched differentiable MPC layer on MI355X (gfx950).
 *
 * The layer solves, for every instance b of a batch, the box-constrained
 * optimal control problem of CA-AC-MPC eq. (3):
 *
 *     min_{x,u}  sum_{t=0}^{T_b-1} 1/2 z_t^T C_t z_t + c_t^T z_t,   z_t = (x_t, u_t)
 *     s.t.       x_{t+1} = f(x_t, u_t),  x_0 = x_init,  u_lo <= u_t <= u_hi
 *
 * by control-limited iLQR (Sec. IV: rollout and linearisation, Riccati backward
 * pass with input bounds, forward pass with a four-point line search; Alg. 2,
 * inner loop), and returns the gradient of an external loss w.r.t. (C_t, c_t,
 * x_init) by implicit differentiation of the KKT conditions at the returned
 * solution (Sec. IV, after eq. (3)).
 *
 * Dynamics f: one RK4 step of a 13-state quadrotor (p[3], q[4] scalar-first,
 * v[3], w[3]) driven by four rotor thrusts in an X configuration (rotor i at
 * angle pi/4 + i pi/2, spin signs +,-,+,-); A_t, B_t are the exact derivatives
 * of that discrete map.  There is no terminal cost, so x_T is not formed.
 *
 * Conventions for every entry point:
 *  - All array arguments are DEVICE pointers owned by the caller; the library
 *    never allocates or frees device memory on these paths.  Scratch space is
 *    the caller's workspace (see dmpc_workspace_bytes).
 *  - Layout is instance-major, row-major, float32 unless stated:
 *      x0        [B][13]
 *      Q         [B][T_max][17]   cost_kind DMPC_COST_DIAG: diagonal of C_t
 *                [B][T_max][153]  cost_kind DMPC_COST_DENSE: upper triangle of
 *                                 C_t, packed row by row: (0,0),(0,1)..(0,16),(1,1)..
 *      p         [B][T_max][17]   c_t
 *      u_lo/u_hi [B][4]
 *      T         [B] int32 horizons in [0, T_max], or NULL (every T_b = T_max)
 *      u_out     [B][T_max][4],  x_out [B][T_max][13]; stages t >= T_b are zero
 *  - Calls are asynchronous on `stream` (a hipStream_t passed as void*), never
 *    synchronise the host and never allocate, so a caller may capture them in a
 *    HIP graph.  A handle is bound to one device and is not thread-safe.
 *    An entry point that launches work makes the handle's device current for
 *    the call and gives the calling thread its previous device back before it
 *    returns; handles on several devices may live in one process.
 *  - Return value: DMPC_OK or a negative DMPC_E* code; dmpc_last_error() gives
 *    the message.  Numerical trouble is never an error return: it is reported
 *    per instance in `status`.
 */
#ifndef DMPC_H
#define DMPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DMPC_NX 13
#define DMPC_NU 4
#define DMPC_NZ 17
#define DMPC_NPACK 153
#define DMPC_T_LIMIT 1024 /* largest supported T_max */
#define DMPC_K_LIMIT 255  /* largest supported max_iter (fits the 8-bit count) */

/* return codes */
#define DMPC_OK 0
#define DMPC_EINVAL (-1)      /* bad sizes, NULL required pointer, lo > hi on the host side */
#define DMPC_EUNSUPPORTED (-2) /* T_max > DMPC_T_LIMIT, max_iter > DMPC_K_LIMIT, unknown cost kind */
#define DMPC_EHIP (-3)        /* HIP runtime or launch error */
#define DMPC_EWORKSPACE (-4)  /* workspace NULL or smaller than dmpc_workspace_bytes() */

/* cost kinds */
#define DMPC_COST_DIAG 0
#define DMPC_COST_DENSE 1

/* config flags */
#define DMPC_NEED_GRAD 0x1u /* forward also factors the stages at (x*, u*) for dmpc_backward */
#define DMPC_PLAIN 0x2u     /* per-launch form: init, three launches per iteration, tail, outputs */
#define DMPC_LPT 0x4u       /* persistent form: process instances by decreasing T_b */
#define DMPC_TUNED 0x8u     /* use the launch choice dmpc_autotune (or dmpc_set_tuned) stored on the
                               handle for this problem shape, instead of DMPC_PLAIN / DMPC_LPT; without
                               a stored choice the flags decide */
#define DMPC_TPAR 0x10u     /* per-launch form whose backward pass is a time-parallel Riccati: an
                               associative scan over the stages (ceil(log2 T_max) launches per
                               iteration) under the previous iteration's clamp pattern, checked stage
                               by stage; instances whose check fails take the serial sweep.  Same
                               results as the serial form up to rounding; meant for small B and long
                               T, where the serial recursion in time sets the latency.  Sizes the
                               workspace for it (about 8.4 KiB more per instance-stage) */
#define DMPC_F64 0x20u      /* FP64 form of the persistent forward: the dynamics, the linearisation,
                               the line search and the stored trajectories and gains in double
                               precision (the stage algebra and the control block are FP64 in both
                               forms).  For long unconverged runs whose iterate is sensitive to
                               FP32 rounding.  Inputs and outputs stay float32; the workspace's
                               trajectory and gain regions double in size.  Not with DMPC_PLAIN or
                               DMPC_TPAR (DMPC_EUNSUPPORTED) */
#define DMPC_F64_REDO 0x40u /* FP64 path for ill-conditioned costs: after the FP32 form's forward,
                               every instance with DMPC_ST_FP64 (a pivot of its control-block
                               factorisation below fp64_pivot) is solved again from the start in the
                               FP64 form and gets DMPC_ST_F64_REDONE; its outputs, decision log and
                               backward factors are the FP64 form's.  Three more launches; the
                               workspace grows by the FP64 form's trajectory and gain regions.  Not
                               with DMPC_PLAIN or DMPC_TPAR (DMPC_EUNSUPPORTED) nor DMPC_F64
                               (DMPC_EINVAL) */

/* per-instance status word */
#define DMPC_ST_CONVERGED 0x1u   /* tol_du > 0 and ||U^k - U^{k-1}||_inf < tol_du was reached */
#define DMPC_ST_MAXITER 0x2u     /* tol_du > 0 and the iteration cap was hit first */
#define DMPC_ST_NONFINITE 0x4u   /* a non-finite value appeared (all line-search costs non-finite) */
#define DMPC_ST_FP64 0x8u        /* a pivot of a stage's control-block factorisation fell below fp64_pivot
                                    (ill-conditioned stage; the block is always factored in FP64, as
                                    L D L^T, whose pivots D_i are the squares of Cholesky's) */
#define DMPC_ST_QPMAXITER 0x10u  /* a stagewise box-QP hit its iteration cap */
#define DMPC_ST_REGULARIZED 0x20u /* a non-positive pivot remained; the block was shifted */
#define DMPC_ST_F64_REDONE 0x40u /* DMPC_F64_REDO: the instance was solved again in the FP64 form */
#define DMPC_ST_ITERS_SHIFT 8    /* bits 8..15: iLQR iterations performed */

/* decision log (optional forward output): [B][max_iter][1 + T_max] bytes.
 * Byte 0 of iteration k: index of the chosen line-search candidate
 * (0..3 for alpha = 1, 0.5, 0.25, 0.1; 255 when every candidate was
 * non-finite).  Byte 1 + t: box-QP pattern of stage t, control i in bits
 * 2i..2i+1 (0 free, 1 at the lower bound, 2 at the upper bound).  Iterations
 * not performed are left as written by the caller. */
#define DMPC_ALPHA_NONE 255

typedef struct {
  float mass;  /* kg */
  float Jxx, Jyy, Jzz; /* principal inertia, kg m^2 */
  float arm;   /* rotor distance from the centre, m */
  float kappa; /* yaw torque per unit thrust, m */
  float dt;    /* RK4 step, s */
  float g;     /* gravity, m/s^2 */
} dmpc_quad_params;

typedef struct {
  int32_t B;          /* batch size (>= 0) */
  int32_t T_max;      /* stage dimension of every [B][T_max][...] array (>= 1) */
  int32_t cost_kind;  /* DMPC_COST_DIAG or DMPC_COST_DENSE */
  int32_t max_iter;   /* iLQR iterations K (0..DMPC_K_LIMIT) */
  float tol_du;       /* <= 0: always K iterations; > 0: per-instance stop at ||dU||_inf < tol_du */
  int32_t ckpt_every; /* 0: the forward stores every stage's factors for the backward (F_t, K_t and the
                         masked inverse of the free control block, 1424 bytes per stage).  c > 0: it
                         stores only V_t, v_t at t = c, 2c, ... (1584 bytes each) and dmpc_backward
                         recomputes the factors segment by segment from those checkpoints;
                         the gradients are the same.  Checkpointing for long horizons. */
  float fp64_pivot;   /* pivot threshold below which a stage sets DMPC_ST_FP64; <= 0 disables */
  uint32_t flags;     /* DMPC_NEED_GRAD | DMPC_PLAIN | DMPC_LPT | DMPC_TUNED | DMPC_TPAR | DMPC_F64 |
                         DMPC_F64_REDO */
} dmpc_config;

/* How a forward is launched.  None of these changes the arithmetic of the
 * persistent form (its results are bitwise the same for every choice); the
 * per-launch form agrees with it to rounding (it forms A_t, B_t in a separate
 * launch). */
typedef struct {
  int32_t plain;          /* 1: per-launch form (3 launches per iteration); 2: per-launch form with the
                             time-parallel Riccati (DMPC_TPAR workspace); 0: one persistent launch */
  int32_t lpt;            /* persistent: take instances by decreasing T_b (needs the T array) */
  int32_t waves_per_simd; /* persistent: 1 = registers uncapped; 2 = capped at 256 so that two waves
                             share a SIMD (helps when there are more instances than 4 per SIMD) */
  int32_t grid_mode;      /* persistent: 0 = as many waves as fit at once, popping four-instance units
                             from a queue; 1 = one wave per four-instance unit */
  float ms;               /* dmpc_autotune: measured forward time of this choice (ms); else 0 */
  int32_t inst_per_wave;  /* persistent: instances per wave, 4 (one per 16-lane row), or 2 / 1 with the
                             other rows idle (one wave per SIMD), so that a small batch spreads over more
                             SIMDs; the results are the same bits */
} dmpc_launch_choice;

typedef struct dmpc_handle_s* dmpc_handle;

/* Create a handle on HIP device `device` (queries its compute-unit count).
 * Returns DMPC_EHIP when no such device is present. */
int dmpc_create(dmpc_handle* h, int device);
int dmpc_destroy(dmpc_handle h);

/* Host-only check of a configuration; needs no GPU.  DMPC_OK, DMPC_EINVAL or
 * DMPC_EUNSUPPORTED. */
int dmpc_validate(const dmpc_config* cfg);

/* Bytes of device workspace a forward/backward pair needs for cfg (0 if cfg
 * is invalid).  Host-only. */
size_t dmpc_workspace_bytes(const dmpc_config* cfg);

/* Forward solve (Alg. 2 inner loop).  Reads x0, Q, p, u_lo, u_hi, T and
 * u_init; writes u_out, x_out (may be NULL), status [B] (bits above,
 * iterations in bits 8..15) and, when decision_log is not NULL, the decisions
 * taken.  u_init [B][T_max][4] is the initial control sequence U^0 of the
 * first rollout (a warm start; each entry clamped into [u_lo, u_hi]); NULL
 * starts from hover thrust m g / 4 per rotor, clamped.  u_init may alias
 * u_out only if the caller does not need u_init afterwards.  The
 * workspace (>= dmpc_workspace_bytes(cfg) bytes, 256-byte aligned) keeps the
 * solution and, with DMPC_NEED_GRAD, the stage factors read by dmpc_backward;
 * it must not be reused before that backward has run. */
int dmpc_forward(dmpc_handle h, const dmpc_config* cfg, dmpc_quad_params dyn, const float* x0, const float* Q,
                 const float* p, const float* u_lo, const float* u_hi, const int32_t* T, const float* u_init,
                 float* u_out, float* x_out, uint32_t* status, void* workspace, size_t workspace_bytes,
                 uint8_t* decision_log, void* stream);

/* Size of the library's static workspace used by dmpc_forward_noalloc: one
 * array of this many bytes in device memory on every device the library runs
 * on, held until the process ends (64 MiB: a forward without DMPC_NEED_GRAD
 * at B = 4096, T_max = 20 needs 55.2 MB, at B = 256, T_max = 50 8.6 MB). */
#define DMPC_NOALLOC_WORKSPACE_BYTES (64u << 20)

/* dmpc_forward without a caller workspace, for callers that cannot allocate
 * device memory at the point of the call (code under HIP graph capture,
 * control loops that forbid allocation).  Arguments and results as
 * dmpc_forward, whose kernels it launches; the workspace is the library's
 * static device array of DMPC_NOALLOC_WORKSPACE_BYTES on the handle's device.
 * It allocates and frees nothing, and never synchronises.
 * - cfg->flags must not hold DMPC_NEED_GRAD (DMPC_EINVAL): a backward would
 *   read the workspace, which the next call overwrites.
 * - A problem whose dmpc_workspace_bytes(cfg) exceeds
 *   DMPC_NOALLOC_WORKSPACE_BYTES is DMPC_EUNSUPPORTED, with nothing launched.
 * - Every call on one device shares that device's array: calls whose work
 *   overlaps in time on one device (other streams, other handles, other host
 *   threads) race and give undefined results.  Order them on one stream.
 *   Nothing in the array is assumed to start at zero; the forward initialises
 *   what it reads. */
int dmpc_forward_noalloc(dmpc_handle h, const dmpc_config* cfg, dmpc_quad_params dyn, const float* x0,
                         const float* Q, const float* p, const float* u_lo, const float* u_hi, const int32_t* T,
                         const float* u_init, float* u_out, float* x_out, uint32_t* status, uint8_t* decision_log,
                         void* stream);

/* Backward (Sec. IV after eq. (3)): given dL/du* [B][T_max][4] and
 * optionally dL/dx* [B][T_max][13] (NULL = zero), writes
 * grad_Q [B][T_max][17|153] (layout of Q; for the packed dense cost the
 * derivative w.r.t. each packed entry, i.e. G_ij + G_ji off the diagonal),
 * grad_p [B][T_max][17] and grad_x0 [B][13].  Uses the workspace of the
 * preceding dmpc_forward, which must have had DMPC_NEED_GRAD and the same cfg.
 * The active set is the one of the forward solution (controls equal to a
 * bound are held fixed).
 * grad_dyn [B][8] (may be NULL) receives, per instance, dL/d of the model
 * constants in the field order of dmpc_quad_params (mass, Jxx, Jyy, Jzz, arm,
 * kappa, dt, g): the gradients with respect to the linearised dynamics F_t
 * and its offset f_t (after Amos et al.) carried to the constants through
 * F_t = df/dz and f_t = f - F_t z* at the solution.  A caller with one set of
 * constants for the whole batch sums over instances.
 * dyn, Q, p, u_lo, u_hi: the forward's inputs, unchanged since that call.
 * They are read only when cfg->ckpt_every > 0 (the stage factors are then
 * recomputed from the checkpoints) or, dyn, Q and p, when grad_dyn is not
 * NULL, and may be NULL otherwise; a NULL one that is needed is DMPC_EINVAL. */
int dmpc_backward(dmpc_handle h, const dmpc_config* cfg, dmpc_quad_params dyn, const float* Q, const float* p,
                  const float* u_lo, const float* u_hi, const void* workspace, size_t workspace_bytes,
                  const float* grad_u, const float* grad_x, float* grad_Q, float* grad_p, float* grad_x0,
                  float* grad_dyn, void* stream);

/* Number of kernel launches the last dmpc_forward / dmpc_backward issued on
 * this handle (host-side count; for tests of the launch structure). */
int dmpc_last_launch_count(dmpc_handle h);

/* Autotuner (the persistent-batching row of the scope: launch structure
 * picked per problem shape).  Runs the forward once per candidate launch
 * choice (the per-launch form; the persistent form for each waves-per-SIMD
 * cap, grid mode and, when T is given, instance order), times each with HIP
 * events on `stream` (best of three after a warm-up), and stores the fastest
 * on the handle under the shape (B, T_max, cost_kind, DMPC_NEED_GRAD,
 * ckpt_every > 0, T given).  Arguments as dmpc_forward; on return the outputs
 * and the workspace hold a forward with the chosen launch.  Unlike every other
 * entry point it synchronises `stream` (it measures), so it cannot be
 * captured in a graph; call it once before capturing.  `chosen` may be NULL. */
int dmpc_autotune(dmpc_handle h, const dmpc_config* cfg, dmpc_quad_params dyn, const float* x0, const float* Q,
                  const float* p, const float* u_lo, const float* u_hi, const int32_t* T, const float* u_init,
                  float* u_out, float* x_out, uint32_t* status, void* workspace, size_t workspace_bytes,
                  void* stream, dmpc_launch_choice* chosen);

/* One receding-horizon step (Alg. 1, outer loop: the first control of each
 * solve is applied, then the horizon moves on by one stage).  For every
 * instance b with horizon T_b = T[b] (T_max when T is NULL):
 *   u_applied[b] = u_star[b][0]                                 ([B][4], may be NULL)
 *   x_state[b]  <- RK4 step of the model (eq. (1), step dyn.dt) from x_state[b]
 *                  under u_star[b][0]                            ([B][13], in place)
 *   u_warm[b][t] = u_star[b][min(t + 1, T_b - 1)] for t < T_b, 0 beyond
 *                                                                ([B][T_max][4], may be NULL)
 * u_warm is meant as the u_init of the next dmpc_forward and may be the same
 * buffer as u_star.  An instance with T_b = 0 keeps its state and gets zero
 * controls.  All pointers are device pointers; one kernel launch, no
 * workspace, no synchronisation.  DMPC_EINVAL for a NULL handle, cfg, x_state
 * or u_star (with B > 0) or non-positive mass, inertia or step. */
int dmpc_mpc_step(dmpc_handle h, const dmpc_config* cfg, dmpc_quad_params dyn, const int32_t* T, float* x_state,
                  const float* u_star, float* u_warm, float* u_applied, void* stream);

/* Store (set) or read (get) the launch choice for the shape of cfg, with
 * has_T != 0 for calls that pass a T array.  get returns DMPC_EINVAL when no
 * choice is stored; set rejects out-of-range fields with DMPC_EINVAL. */
int dmpc_set_tuned(dmpc_handle h, const dmpc_config* cfg, int has_T, const dmpc_launch_choice* choice);
int dmpc_get_tuned(dmpc_handle h, const dmpc_config* cfg, int has_T, dmpc_launch_choice* choice);

/* The launch choice the last dmpc_forward / dmpc_autotune on this handle used. */
int dmpc_last_launch_choice(dmpc_handle h, dmpc_launch_choice* choice);

/* Persisted launch choices, so that a shape is tuned once per machine rather
 * than once per process.  dmpc_tuned_save writes every choice stored on the
 * handle to the text file `path` (replacing it), one line per shape, keyed by
 * the device's architecture name and compute-unit count; it returns the
 * number of lines written.  dmpc_tuned_load adds the choices of such a file
 * to the handle, skipping lines saved for another architecture or CU count
 * and malformed ones, and returns the number taken.  DMPC_EINVAL for a NULL
 * argument or a file that cannot be opened.  Host-only; no GPU work. */
int dmpc_tuned_save(dmpc_handle h, const char* path);
int dmpc_tuned_load(dmpc_handle h, const char* path);

/* Graph helpers: begin capturing `stream`; enqueue dmpc_forward/dmpc_backward
 * calls; end the capture into an executable graph.  The captured work uses
 * kernels only (no memset or copy nodes). */
int dmpc_capture_begin(dmpc_handle h, void* stream);
int dmpc_capture_end(dmpc_handle h, void* stream, void** graph_exec);
int dmpc_graph_launch(dmpc_handle h, void* graph_exec, void* stream);
int dmpc_graph_destroy(dmpc_handle h, void* graph_exec);

/* Message for the last error on this handle (or of the last failed call
 * without a handle when h is NULL). */
const char* dmpc_last_error(dmpc_handle h);

#ifdef __cplusplus
}
#endif
#endif
