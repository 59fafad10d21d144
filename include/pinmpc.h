/* pinmpc.h -- C ABI of the MI355X batched parallel-in-horizon MPC solver.
 *
 * Solves, for every problem b of a batch independently, the standard-form
 * linear time-varying MPC quadratic program of the paper's Sec. III
 * ("pi^n MPC", with C = I):
 *
 *   min  sum_{k=0}^{N-1} 1/2 (x_{k+1} - x_ref[k])^T Q (x_{k+1} - x_ref[k])
 *                        + 1/2 (u_k - u_ref[k])^T R (u_k - u_ref[k])
 *   s.t. x_{k+1} = A_k x_k + B_k u_k + e_k,   x_0 = x0,
 *        stance contact i at stage k:  |f_x|, |f_y| <= mu f_z,  f_z <= fz_max,
 *                                      |tau_j| <= tau_max          (Sec. II-B)
 *        swing contact:                f = 0, tau = 0
 *
 * with n = 13 states, m = 12 inputs = 2 contacts x (force 3, moment 3), in
 * the order (f0x, f0y, f0z, t0x, t0y, t0z, f1x, ..., t1z).  For
 * loco-manipulation (Sec. II-A: the contact set may hold hand contacts beside
 * the feet) a batch may instead carry 4 contacts per stage, m = 24 inputs
 * (pinmpc_batch.contacts): every contact's force and moment are expressed in
 * that contact's own frame (its B_k columns carry the frame), so the same
 * wrench rows, with the pyramid about the contact normal, hold for each.
 *
 * The solve runs the paper's ADMM (velocity-form lifting, the z/v variable
 * splitting, three stage-parallel closed-form block updates with cached
 * J_k, H_k, Nesterov-type acceleration with restart) in FP32 on the GPU, then
 * an FP64 refinement on the GPU (active-set passes from the ADMM faces, an
 * interior-point fallback, an exact equality-constrained Riccati polish) that
 * certifies every result by its KKT residuals.
 *
 * Conventions
 *  - Every array pointer in pinmpc_batch / pinmpc_out is a DEVICE pointer
 *    (for example a torch tensor's data_ptr()).  The caller owns every buffer
 *    it passes; the library never frees caller memory.  The library owns only
 *    its workspace, allocated lazily inside pinmpc_solve and bounded by the
 *    context's hbm_budget_bytes.
 *  - All calls are ordered on the given hipStream_t (NULL = default stream).
 *    pinmpc_solve returns after enqueuing; results are ready when the stream
 *    reaches that point.  A context must not be used from two host threads at
 *    once and must not run two solves concurrently (workspace is shared).
 *  - Layout is row-major C order, problem index slowest.  Horizons shorter
 *    than n_max are padded at the end; padded stages are ignored.
 *  - Return codes: < 0 is an API error (the context stays usable); a problem
 *    that does not certify is not an error, it gets a per-problem status.
 */
#ifndef PINMPC_H
#define PINMPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PINMPC_NX 13
#define PINMPC_NU 12
#define PINMPC_NCONTACT 2
#define PINMPC_NCONTACT_MAX 4   /* feet and hands (pinmpc_batch.contacts) */
#define PINMPC_NU_MAX 24
#define PINMPC_NRES 5      /* r_dyn, r_ineq, r_stat, r_comp, r_sign */
#define PINMPC_NMAX 64     /* largest horizon of the serving loop and of the
                              one-workgroup-per-problem kernels */
#define PINMPC_NMAX_LONG 512  /* largest horizon pinmpc_solve accepts: beyond
                              PINMPC_NMAX the ADMM splits each horizon across
                              workgroups and the refinement keeps its stage
                              buffers in the workspace */

enum {
  PINMPC_OK = 0,
  PINMPC_EINVAL = -1,   /* bad argument: null pointer, size or setting */
  PINMPC_ENOMEM = -2,   /* device allocation failed */
  PINMPC_EBUDGET = -3,  /* workspace would exceed hbm_budget_bytes */
  PINMPC_EDEVICE = -4,  /* HIP runtime or launch error */
  PINMPC_EBUSY = -5,   /* server: no free slot / request still running */
  PINMPC_ETOOBIG = -6   /* batch needs more workspace than the static scratch
                           of pinmpc_solve_noalloc holds */
};

/* Per-problem status written to pinmpc_out.status. */
enum {
  PINMPC_ST_OK = 0,          /* certified: every KKT residual <= kkt_tol */
  PINMPC_ST_MAXITER = 1,     /* refinement disabled; ADMM iterate returned */
  PINMPC_ST_UNPOLISHED = 2,  /* refinement ran out of passes; best iterate */
  PINMPC_ST_NONFINITE = 3,   /* NaN/Inf in this problem's data (stage arrays,
                                x0, u_prev, u_ref, weights or bounds) */
  PINMPC_ST_BADINPUT = 4     /* malformed bounds or horizon (mu <= 0,
                                fz_max < 0, tau_max < 0, weight <= 0,
                                Q or R not positive, N outside 1..n_max) */
};

/* Solver settings.  pinmpc_default_settings fills the defaults. */
typedef struct {
  float rho;               /* ADMM penalty (Sec. III rho); default 10 */
  int32_t iters;           /* ADMM sweeps K (fixed count); default 100 */
  int32_t accel;           /* 1: fast ADMM with restart; default 1 */
  float restart_eta;       /* restart test c_m < eta c_{m-1}; default 0.999 */
  int32_t scaling;         /* 1: block-constant input scaling; default 1 */
  int32_t refine;          /* 1: FP64 refinement and certificate; default 1 */
  int32_t refine_passes;   /* active-set passes from the ADMM faces; 8 */
  int32_t ipm_iters;       /* interior-point fallback iterations cap; 40 */
  int32_t polish_passes;   /* active-set passes after the fallback; 6
                              (each of the three in 0..1000; with refine = 1,
                              refine_passes and ipm_iters not both 0) */
  double kkt_tol;          /* certification threshold; default 1e-9 */
  int32_t precision;       /* 0: FP32 operators; 1: BF16 operators */
  int32_t form;            /* 0: plain (one launch per sweep);
                              1: fused (all sweeps in one launch: operators in
                                 registers up to 40 stages, streamed beyond);
                              -1: pack problems by horizon class;
                              2: horizon split across workgroups (a chain of
                                 stage-parallel launches per sweep).
                              Horizons beyond PINMPC_NMAX always split.  Every
                              form computes bitwise the same iterates. */
  int32_t graph;           /* 1: capture the whole solve as a hipGraph on first
                              use and replay it while the batch shape, buffers
                              and settings are unchanged; default 1 */
  int32_t first_passes;    /* active-set passes run for every problem in the
                              first refinement launch; a problem they do not
                              certify continues (remaining passes, then the
                              interior point) in a second launch with the
                              other uncertified problems.  0: all passes in
                              the first launch; default 4 */
  int32_t group;           /* problems per workgroup of the fused sweep kernel
                              (1, 2 or 4; fewer when the horizon leaves no
                              room: each problem takes round_up(25 N, 64)
                              threads of at most 1024); default 1 */
  int32_t scan;            /* the refinement's backward recursion (the LQ
                              solve of every active-set pass and the factored
                              Newton step of every interior-point iteration):
                              0: sequential over the horizon, one wave per
                              problem; 2, 4 or 8: an associative scan over
                              that many chunks of the horizon (one wave per
                              chunk; depth about 3 N / W + W stage steps
                              instead of N; results equal the sequential
                              recursion's to rounding).  Horizons shorter than
                              8 stages stay sequential.  Default 0 */
} pinmpc_settings;

typedef struct pinmpc_ctx_s* pinmpc_ctx;

/* One batch of problems (device pointers). */
typedef struct {
  int32_t batch;           /* number of problems B (0 allowed) */
  int32_t n_max;           /* padded horizon, 1..PINMPC_NMAX_LONG (the
                              serving loop: 1..PINMPC_NMAX) */
  const int32_t* N;        /* [B] horizon per problem in 1..n_max; NULL: all n_max */
  const float* A;          /* [B][n_max][13][13] */
  const float* Bu;         /* [B][n_max][13][12] (m = 6 contacts inputs) */
  const float* e;          /* [B][n_max][13]; NULL: 0 */
  const float* x0;         /* [B][13] */
  const float* u_prev;     /* [B][12] input before stage 0 (velocity form); NULL: 0 */
  const float* x_ref;      /* [B][n_max][13] reference of x_{k+1} */
  const float* u_ref;      /* [B][n_max][12]; NULL: 0 */
  const float* Q;          /* [B][13] diagonal state weight, > 0 */
  const float* R;          /* [B][12] diagonal input weight, > 0 */
  const uint8_t* contact;  /* [B][n_max][2] 1 = stance, 0 = swing */
  const float* mu;         /* [B] friction coefficient */
  const float* fz_max;     /* [B] normal-force upper bound */
  const float* tau_max;    /* [B] moment bound per axis */
  const float* weight;     /* [B] force scale m g (input scaling and residual
                              normalisation); NULL: fz_max / 2 */
  int32_t contacts;        /* contacts per stage C: 2 (the feet; 0 means 2)
                              or 4 (feet and hands, loco-manipulation).  The
                              input arrays above and the output u hold m =
                              6 C inputs per stage: Bu [B][n_max][13][m],
                              u_prev [B][m], u_ref [B][n_max][m], R [B][m],
                              contact [B][n_max][C], u [B][n_max][m].  With 4
                              contacts: n_max <= PINMPC_NMAX, the ADMM sweeps
                              run in the streamed form (settings.form 0: one
                              launch per sweep, else all sweeps in one launch)
                              and the FP64 refinement is the interior point
                              alone (settings.ipm_iters iterations, at least
                              1; refine_passes, first_passes, polish_passes
                              and scan do not apply); the serving loop takes
                              2 contacts only */
} pinmpc_batch;

/* Outputs (device pointers, caller-allocated). */
typedef struct {
  float* u;                /* [B][n_max][12] optimal inputs (0 on padding;
                              [B][n_max][24] with 4 contacts) */
  float* x;                /* [B][n_max+1][13] rollout of u (x_0 = x0) */
  float* res;              /* [B][PINMPC_NRES] FP64-evaluated KKT residuals of
                              the returned (u, x), each normalised by the
                              largest term it compares (r_dyn, r_stat), by
                              m g (r_ineq), or by 1 + |mu| m g (r_comp);
                              r_sign is the most negative inequality
                              multiplier so normalised; may be NULL */
  int32_t* iters;          /* [B] ADMM sweeps + refinement passes; may be NULL */
  int32_t* status;         /* [B] PINMPC_ST_*; may be NULL */
  int32_t* detail;         /* [B][4] work of the FP64 refinement, may be NULL:
                              equality-constrained passes (active-set,
                              crossover and polish), interior-point
                              iterations, stages whose backward recursion the
                              equality passes factored (a pass restarted at
                              stage k factors k stages; with four contacts:
                              the stages of the interior point's factoring
                              recursions, every predictor and the correctors
                              near the optimum, the other correctors running
                              the recursion's vector part only), and the
                              refinement launch (1 or 2) that finished the
                              problem; 0 0 0 0 for a problem with bad input */
} pinmpc_out;

/* Fill *s with the defaults listed above (host memory, caller-owned; a null
 * s is ignored).  rho is the penalty of the augmented Lagrangian of Sec. III;
 * the iteration count K replaces a residual stop by design (a short FP32 ADMM
 * run only supplies the starting faces of the FP64 refinement). */
void pinmpc_default_settings(pinmpc_settings* s);

/* Create a context on HIP device `device` (host call; *out receives the
 * handle, which the caller releases with pinmpc_destroy).  hbm_budget_bytes
 * bounds the library's workspace (0 = 64 GiB).  Settings are copied and
 * validated: PINMPC_EINVAL for a bad setting or null out, PINMPC_EDEVICE for
 * a missing device, PINMPC_ENOMEM if the context cannot be made. */
int pinmpc_create(pinmpc_ctx* out, int device, size_t hbm_budget_bytes,
                  const pinmpc_settings* s);

/* Replace the context's settings (validated; PINMPC_EINVAL leaves the old
 * ones in place). */
int pinmpc_set_settings(pinmpc_ctx c, const pinmpc_settings* s);

/* Bytes of workspace a solve of this shape needs with 2 contacts per stage
 * (host call, no GPU work; PINMPC_EINVAL for a shape outside 0 <= batch,
 * 1 <= n_max <= PINMPC_NMAX_LONG).  A batch with 4 contacts needs the bytes
 * of pinmpc_workspace_bytes_contacts. */
int pinmpc_workspace_bytes(const pinmpc_settings* s, int32_t batch, int32_t n_max,
                           size_t* bytes);
/* The same for `contacts` (2 or 4) contacts per stage; PINMPC_EINVAL also
 * for another contact count, or 4 contacts with n_max > PINMPC_NMAX. */
int pinmpc_workspace_bytes_contacts(const pinmpc_settings* s, int32_t batch, int32_t n_max,
                                    int32_t contacts, size_t* bytes);

/* Solve every problem of `in`, the standard-form LTV MPC of Sec. III with the
 * wrench sets of Sec. II-B, by the ADMM of Sec. III (velocity-form lifting,
 * z/v splitting, the three stage-parallel closed-form block updates)
 * followed by the FP64 refinement and certificate; results into `out`
 * (device buffers of the documented shapes, caller-owned, fully written for
 * every problem including padding).  Stream-ordered and asynchronous: the
 * call returns after enqueuing on hip_stream.  The first solve of a larger
 * shape (re)allocates the context's workspace (PINMPC_EBUDGET beyond the
 * budget, PINMPC_ENOMEM if the allocation fails); PINMPC_EINVAL for a null or
 * malformed argument, PINMPC_EDEVICE for a launch failure.  Bad data in one
 * problem only sets that problem's status. */
int pinmpc_solve(pinmpc_ctx c, const pinmpc_batch* in, pinmpc_out* out,
                 void* hip_stream);

/* pinmpc_solve for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and the same results as pinmpc_solve with the context's
 * settings, launched eagerly on `hip_stream` (never captured or replayed as a
 * graph by the library), with the workspace taken from a file-scope device
 * array of PINMPC_NOALLOC_SCRATCH_BYTES per GPU instead of the context's
 * allocation.  The call allocates nothing (no hipMalloc, hipFree or
 * allocating library routine); its first call on a device resolves that
 * device's copy of the array once.  Each GPU that runs it holds the array
 * until the process ends.  A batch whose workspace (pinmpc_workspace_bytes)
 * exceeds the array returns PINMPC_ETOOBIG before any GPU work: at 12.3 KB
 * per stage that is about 21 800 stages, e.g. 1091 problems at N = 20 or 364
 * at N = 60.  Every call on one GPU shares that GPU's array and leaves its
 * contents behind (the kernels initialise everything they read): calls that
 * overlap on one GPU (two streams, two host threads, two contexts) race and
 * must be serialised by the caller. */
#define PINMPC_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int pinmpc_solve_noalloc(pinmpc_ctx c, const pinmpc_batch* in, pinmpc_out* out,
                         void* hip_stream);

/* The ADMM of Sec. III only (setup and `iters` sweeps, no refinement), for
 * iterate-level checks.  z_out: caller-owned device buffer [B][n_max][25] of
 * the final z iterates (lifted (x_{k+1}, u_k), inputs unscaled; [B][n_max][37]
 * with 4 contacts).
 * Stream-ordered; errors as pinmpc_solve. */
int pinmpc_admm(pinmpc_ctx c, const pinmpc_batch* in, int32_t iters,
                float* z_out, void* hip_stream);

/* Measurement of the solve (not a step of the method).
 * Time of the last solve's phases in ms (host pointers; any may be NULL),
 * measured with HIP events on the solve's stream.  Blocks until the last
 * solve finished.  setup + admm + refine = total.  A solve replayed from a
 * captured graph reports only its total (setup, admm, refine = -1).
 * PINMPC_EINVAL if the context has made no solve. */
int pinmpc_stats(pinmpc_ctx c, double* total_ms, double* setup_ms,
                 double* admm_ms, double* refine_ms);

/* The same for an earlier solve: back = 0 is the last solve, 1 the one
 * before, up to PINMPC_STATS_RING - 1 (a context keeps the events of its last
 * PINMPC_STATS_RING solves, so back-to-back solves can be timed without a
 * synchronisation between them).  PINMPC_EINVAL if back is out of that range
 * or fewer than back + 1 solves were made. */
#define PINMPC_STATS_RING 64
int pinmpc_stats_back(pinmpc_ctx c, int32_t back, double* total_ms, double* setup_ms,
                      double* admm_ms, double* refine_ms);

/* Algorithmic HBM bytes of the last solve and their rate over its measured
 * time (host pointers; either may be NULL).  The byte model counts, per
 * stage, PINMPC_SETUP_BYTES once (operators read, H_k, M_k, qbar_k and the
 * scaled B written), PINMPC_SWEEP_BYTES per ADMM sweep (FP32 operators and
 * both iterate sets streamed), and PINMPC_REFINE_BYTES per stage of every
 * equality-constrained pass and interior-point iteration of the FP64
 * refinement (counted on the device).  Blocks until the last solve finished;
 * only valid while no later solve on this context has been enqueued.
 * PINMPC_EINVAL if the context has made no solve. */
#define PINMPC_SETUP_BYTES 3200
#define PINMPC_SWEEP_BYTES 5070
#define PINMPC_REFINE_BYTES 4500
int pinmpc_stats_traffic(pinmpc_ctx c, double* bytes, double* gbytes_per_s);

/* Release the context and its workspace (waits for the device first). */
int pinmpc_destroy(pinmpc_ctx c);

/* Static text of a return code. */
const char* pinmpc_strerror(int code);

/* ------------------------------------------------------- stage matrices
 * The step before the solve: A_k and B_k of the centroidal model from compact
 * physics, on the device.  The paper's discrete centroidal dynamics (Sec.
 * II-A: CoM, linear and angular momentum driven by the contact forces through
 * the lever arms p_{i,k} - c_k and by the contact moments) in the 13-state
 * single-rigid-body form with gravity as a state, forward Euler, the lever arm
 * taken at the reference CoM:
 *   A_k = I + dt A_c(psi_k), A_c: angle rates R_z(psi_k)^T omega, CoM rate v,
 *         v_z rate + gravity state;
 *   B_k = dt B_c: omega rows I_w^{-1} [p_{i,k} - c_ref,k]_x (forces) and I_w^{-1}
 *         (moments) with I_w = R_z(psi_k) diag(I_body) R_z(psi_k)^T; v rows I/m.
 * Model 1 is the paper's own 9-state form (CoM c, linear momentum l_G,
 * angular momentum k_G about the CoM) in slots 0..8 of the same layout:
 *   c' = c + dt l / m,  l' = l + dt (m g + sum f_i),
 *   k' = k + dt sum ((p_{i,k} - c_ref,k) x f_i + tau_i),
 * gravity in the affine term e_k = (0, dt m g, 0); slots 9..12 are inert
 * (A = I, B = 0, e = 0): with zero initial value and reference they leave the
 * optimum of the 9-state problem unchanged.
 * Matrices are built for every stage whatever the contact state (a swing
 * contact's inputs are fixed to zero by the solve); padding stages
 * (k >= N[b]) get A = I, B = 0, e = 0.  FP32 arithmetic. */
typedef struct {
  int32_t batch;           /* B (0 allowed) */
  int32_t n_max;           /* padded horizon, 1..PINMPC_NMAX_LONG */
  int32_t model;           /* 0: 13-state single rigid body; 1: 9-state momentum */
  const int32_t* N;        /* [B] horizon per problem; NULL: all n_max */
  const float* yaw;        /* [B][n_max] yaw psi_k of the linearisation */
  const float* c_ref;      /* [B][n_max][3] reference CoM at stage k */
  const float* feet;       /* [B][n_max][2][3] contact positions at stage k */
  const float* mass;       /* [B] total mass m */
  const float* inertia;    /* [B][3] principal moments of the body (yaw frame;
                              unused by model 1) */
  const float* dt;         /* [B] time step */
} pinmpc_physics;

/* A: [B][n_max][13][13], Bu: [B][n_max][13][12], e: [B][n_max][13]
 * caller-owned device buffers (the layouts pinmpc_batch takes); e may be NULL
 * for model 0 (whose e is zero), not for model 1.  Device pointers in `in`.
 * Stream-ordered; PINMPC_EINVAL for null pointers, a bad shape or model,
 * PINMPC_EDEVICE for a launch failure; no workspace, no allocation. */
int pinmpc_build_dynamics(const pinmpc_physics* in, float* A, float* Bu, float* e,
                          void* hip_stream);

/* ------------------------------------------------------ landmark reward
 * The step after the solve: the MPC landmark guidance reward of Sec. II-C.
 * Each solve made at tick T stores, per environment, the predicted CoM
 * (entries 3..5 of x_n) at the landmark offsets n_l = 1 + floor(s_l (N - 1)),
 * s_l = l / (n_landmarks - 1) (s_0 = 0: the next MPC step; the last: the end
 * of the horizon), for the ticks T + n_l ticks_per_step.  When the rollout
 * reaches tick t, the reward is
 *   r_t = exp(-sum_l alpha_l |c_t - c_hat_l(t)|_Qc^2 / sigma^2)  in (0, 1],
 * over the landmarks predicted for t only (none early in an episode).
 * The store is caller-owned device memory: com [envs][ring][n_landmarks][3]
 * FP32 and tag [envs][ring][n_landmarks] int32 (the tick a landmark is for;
 * -1 = empty), slot = target tick mod ring; ring must exceed
 * n_max * ticks_per_step so a landmark survives until its tick.  Ticks are
 * nonnegative.  All calls are stream-ordered, allocate nothing, and return
 * PINMPC_EINVAL for null pointers or out-of-range sizes, PINMPC_EDEVICE for a
 * launch failure. */
typedef struct {
  int32_t envs;            /* E (0 allowed) */
  int32_t n_landmarks;     /* N_L, 1..31 */
  int32_t ring;            /* slots per environment */
  int32_t ticks_per_step;  /* reward-loop ticks per MPC step dt, >= 1 */
  float* com;              /* [E][ring][N_L][3] */
  int32_t* tag;            /* [E][ring][N_L] */
} pinmpc_landmarks;

/* Mark every landmark of the environments with env_mask[e] != 0 empty (a new
 * episode); env_mask NULL clears the whole store. */
int pinmpc_landmarks_clear(const pinmpc_landmarks* st, const uint8_t* env_mask,
                           void* hip_stream);

/* Store the landmarks of the solves made at `tick`: x [E][n_max+1][13] (the
 * x output of pinmpc_solve), N [E] horizons (NULL: all n_max; an environment
 * with a horizon outside 1..n_max stores nothing). */
int pinmpc_landmarks_push(const pinmpc_landmarks* st, int32_t n_max, const int32_t* N,
                          const float* x, int32_t tick, void* hip_stream);

/* r_t for every environment at `tick` from its realised CoM com [E][3]:
 * alpha [N_L] confidence weights, qc [3] diagonal of Q_c (device memory),
 * sigma > 0.  reward [E]; used [E] (may be NULL) receives the bit set of the
 * landmarks that entered the reward. */
int pinmpc_landmark_reward(const pinmpc_landmarks* st, const float* com, int32_t tick,
                           const float* alpha, const float* qc, float sigma, float* reward,
                           int32_t* used, void* hip_stream);

/* ------------------------------------------------------------------ serving
 * The solve inside a training loop (Sec. III: one problem per environment,
 * solved every control tick).  Continuous-batching front end: requests (batches of problems in caller
 * device memory, typically one environment group's problems of one control
 * tick) are queued and packed into whichever of n_lanes concurrent lanes
 * (each with its own HIP stream and workspace) frees up first; a lane takes
 * every waiting request that fits its capacity.  Caller buffers of a request
 * must stay valid and untouched until the request is done.  Each problem is
 * solved exactly as pinmpc_solve would solve it alone (bitwise), whatever
 * else shares its launch.  Warm start: problem i of a request submitted with
 * warm_base >= 0 starts from the iterates kept in device slot warm_base + i
 * (shifted by one stage) and leaves its final iterates there; slots persist
 * for the server's lifetime. */
typedef struct pinmpc_server_s* pinmpc_server;

/* hbm_budget_bytes bounds lanes x (workspace + staging) + warm slots
 * (0 = 64 GiB); exceeding it returns PINMPC_EBUDGET.  lane_capacity is the
 * most problems one launch holds; a request larger than it is rejected.
 * Every lane's memory is allocated here (PINMPC_ENOMEM on failure), none by
 * later calls; *out is released by pinmpc_server_destroy. */
int pinmpc_server_create(pinmpc_server* out, int device, const pinmpc_settings* s,
                         int n_lanes, int32_t lane_capacity, int32_t warm_slots,
                         size_t hbm_budget_bytes);

/* Queue one request (host struct pointing at device data that must stay
 * valid until the request is done); *ticket identifies it.  Thread-safe.
 * PINMPC_EINVAL for a malformed request or one larger than the lane
 * capacity.  PINMPC_EBUSY if
 * the request's warm-slot range [warm_base, warm_base + batch) overlaps the
 * range of a request that is not done yet (a slot is read and rewritten by
 * its solve, so it serves one request at a time). */
int pinmpc_submit(pinmpc_server s, const pinmpc_batch* req, const pinmpc_out* out,
                  int32_t warm_base, int64_t* ticket);

/* *done = 1 once the request's outputs are in its buffers; latency_ms is
 * submit-to-ready.  A finished ticket is released by the call that reports it
 * (PINMPC_EINVAL for an unknown or released ticket; the request's own launch
 * error, if any, is returned with done = 1). */
int pinmpc_poll(pinmpc_server s, int64_t ticket, int* done, double* latency_ms);

/* Block until the request is done (then as pinmpc_poll). */
int pinmpc_wait(pinmpc_server s, int64_t ticket, double* latency_ms);

/* Launches made and problems solved so far; returns the first launch error. */
int pinmpc_server_stats(pinmpc_server s, int64_t* launches, int64_t* problems);

/* Checkpoint and resume of the warm-start state: copy the device iterates of
 * warm slots [slot_base, slot_base + count) to caller-owned host memory, or
 * back from it.  The image is a 16-byte header (the bytes "PMWS", version 1,
 * count, PINMPC_NMAX as int32) followed by count slots of
 * PINMPC_WARM_SLOT_BYTES (FP32 iterates z, v, theta, beta, lambda of the ADMM
 * of Sec. III per stage, [PINMPC_NMAX][5][25], inputs scaled); bytes must be
 * at least PINMPC_WARM_IMAGE_BYTES(count).  Synchronous (returns when the
 * copy is done).  PINMPC_EINVAL for a range outside the server's slots, a
 * short buffer or (import) a header that does not match; PINMPC_EBUSY while
 * a request using one of those slots is in flight. */
#define PINMPC_WARM_SLOT_BYTES ((size_t)PINMPC_NMAX * 5 * 25 * 4)
#define PINMPC_WARM_IMAGE_BYTES(count) (16 + (size_t)(count) * PINMPC_WARM_SLOT_BYTES)
int pinmpc_server_export_state(pinmpc_server s, int32_t slot_base, int32_t count,
                               void* host_buf, size_t bytes);
int pinmpc_server_import_state(pinmpc_server s, int32_t slot_base, int32_t count,
                               const void* host_buf, size_t bytes);

/* Finish every queued request, then free the server. */
int pinmpc_server_destroy(pinmpc_server s);

#ifdef __cplusplus
}
#endif
#endif /* PINMPC_H */
