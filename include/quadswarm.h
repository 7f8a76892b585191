/*
 * quadswarm.h -- C ABI of the MI355X batched quadrotor-swarm stepper.
 *
 * The library advances E independent environments, each holding a swarm of
 * 1..64 Crazyflie-class quadrotors (Q quads in total), with the dynamics of
 * Huang et al., "QuadSwarm" (arXiv 2306.09537), §III-A (rigid body, motor lag
 * and noise) and §III-B (walls, ceiling, floor, quad-quad collisions), and
 * produces the §III-C observation with the K nearest swarm-mates.
 *
 * Conventions shared by every entry point:
 *  - Every function returns QS_OK (0) or a negative QS_ERR_* code and never
 *    throws.  qs_error_string() turns a code into a static string.
 *  - Pointers named h_* are host memory, read only during the call.
 *    Pointers named d_* are device memory owned by the caller, borrowed for
 *    the duration of the (stream-ordered) work the call enqueues.
 *  - `stream` is a hipStream_t passed as void*; NULL is the null stream.
 *    All device work of a call is enqueued on that stream and the call
 *    returns without waiting, except where noted.  A handle is not
 *    thread-safe; calls on one handle must be ordered by the caller.
 *  - Argument errors are detected on the host before anything is enqueued.
 *    Device-side errors (a non-finite value produced in the state, a
 *    non-finite action, or a rejected qs_set_params row) are sticky in the
 *    handle and are returned by the next qs_sync().
 *  - All device arithmetic is IEEE float32.
 *  - Device pointers: d_actions 16-byte aligned, d_obs and d_mask 8-byte
 *    aligned, others 4-byte aligned (QS_ERR_ALIGN otherwise).
 *  - The device buffers a call writes must not overlap the buffers it
 *    reads or each other (QS_ERR_INVALID), except where a call names one
 *    buffer as both input and output (d_gstate of qs_rollout_backward) or
 *    allows it (qs_step_backward: d_gstate_in may be d_gstate_out).
 *  - Environment overrides of launch choices (the library picks each by
 *    itself; results are bit-identical whichever form runs):
 *      QS_BLOCK_SIZE=64|128  workgroup size, read by qs_create (default 64;
 *                            128 for >= 262,144 single-quad swarms);
 *      QS_BUCKETED=0         uneven swarm sizes run one workgroup per packed
 *                            block instead of the persistent bucketed
 *                            launch, read by qs_create;
 *      QS_STEP_PIPE, QS_ROLLOUT_PIPE, QS_RECOMPUTE_PIPE,
 *      QS_REVERSE_PIPE = 0|1
 *                            force the multi-wavefront forms off or on:
 *                            multi-substep step calls on two wavefronts
 *                            per workgroup (uniform 8-quad swarms),
 *                            qs_rollout on two (three with the penalty in
 *                            8-quad swarms), the recompute of
 *                            qs_rollout_backward on two and its reverse
 *                            sweep on four (swarms of 1 or 8); default on
 *                            up to 1024 workgroups; read on every call;
 *      QS_STAGE_ROWS=n       observation rows per LDS staging pass (a power
 *                            of two up to the workgroup size; 0: each lane
 *                            stores its own row), read once;
 *      QS_TAPE_BYTES         tape budget of qs_rollout_backward (below).
 *
 * Canonical layouts (row-major, float32):
 *  state  [Q][27] = x(3) v(3) R(9, row-major, body->world) omega(3, body)
 *                   u_f(4, filtered rotor speed) eps(4, motor noise, N)
 *                   resting-on-floor flag(1: 0 or 1)
 *  params [Q][6]  = mass (kg), ixx, iyy, izz (kg m^2), thrust_to_weight,
 *                   motor time constant tau_m (s)          (qs_quad_params)
 *  action [Q][4]  = per-rotor normalised thrust command a (§III-A.1),
 *                   rotors front-right, back-right, back-left, front-left
 *  goal   [Q][3]  = goal position (m)
 *  obs    [Q][18+6K] = x - goal, v, R (row-major), omega, then K slots of
 *                   (x_j - x_i, v_j - v_i) for the K nearest swarm-mates in
 *                   order of (distance, index); zero slots when n_e - 1 < K.
 * Quads of one environment are contiguous: env e owns quads
 * [env_offsets[e], env_offsets[e+1]).
 */
#ifndef QUADSWARM_H
#define QUADSWARM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---- */
#define QS_OK 0
#define QS_ERR_NULL (-1)          /* a required pointer is NULL */
#define QS_ERR_INVALID (-2)       /* a count, size or constant is out of range */
#define QS_ERR_ENV_SIZE (-3)      /* env_offsets not CSR, or a swarm of 0 or >64 */
#define QS_ERR_HIP (-4)           /* a HIP runtime call failed */
#define QS_ERR_NONFINITE (-5)     /* sticky: non-finite action or state on device */
#define QS_ERR_NOMEM (-6)         /* device or host allocation failed */
#define QS_ERR_ALIGN (-7)         /* a device pointer is misaligned (see above) */
#define QS_ERR_UNSUPPORTED (-8)   /* valid request this build does not handle */
#define QS_ERR_TOO_LARGE (-9)     /* exceeds the fixed scratch of qs_step_backward_noalloc */

/* ---- physics switches (qs_desc.flags) ---- */
#define QS_ROOM 1u            /* §III-B.2 walls and ceiling bounce the quad */
#define QS_FLOOR 2u           /* §III-B.3 floor hit, resting, friction, take-off */
#define QS_COLLIDE 4u         /* §III-B.1 in-env pair detection and response */
#define QS_MOTOR_NOISE 8u     /* §III-A.2 AR(1) motor noise */
#define QS_APPROACH_ONLY 16u  /* pair response only while the pair approaches */
#define QS_ACT_UNIT 32u       /* f_hat = clip(a,0,1) instead of (clip(a,-1,1)+1)/2 */
#define QS_DOWNWASH 64u       /* §III-B.4 downwash of upper swarm-mates on lower ones */
#define QS_SENSOR_NOISE 128u  /* §III-C noise on the own-state part of observations */

#define QS_STATE_DIM 27
#define QS_PARAM_DIM 6
#define QS_MAX_SWARM 64
#define QS_MAX_QUADS (1 << 26) /* quads per handle (67,108,864: 7.2 GB of state) */
#define QS_NOALLOC_SCRATCH_BYTES (64 << 20) /* fixed scratch per device, 64 MiB */

typedef struct qs_handle qs_handle;

/*
 * Global constants of one handle.  env_offsets is a host array of n_envs+1
 * non-decreasing int32 (CSR), env_offsets[0] == 0, every swarm 1..64 quads,
 * at most QS_MAX_QUADS quads in all (QS_ERR_INVALID beyond).
 *  dt               substep length (s), > 0 (200 Hz simulation: 0.005)
 *  gravity          g (m/s^2), acts along -z
 *  arm_length       rotor distance from the centre (m); X layout
 *  k_tau            propeller reaction torque per newton of thrust (m)
 *  drag_coef        linear world-frame drag c_d (N s/m), >= 0
 *  floor_mu         floor friction coefficient, >= 0
 *  motor_noise_decay alpha_nd in [0,1); motor_noise_std sigma >= 0 in units
 *                   of f_max (stationary std of the noise is sigma f_max)
 *  room_min/max     room box (m); room_min[2] is the floor height
 *  wall_restitution e in [0,1] (1: the normal velocity is mirrored)
 *  col_dist         centre distance below which two quads are in contact (m)
 *  col_decay        velocity decay alpha after a collision (1: none)
 *  col_noise_v/w    std of the velocity / body-rate noise added on a
 *                   collision (m/s, rad/s), >= 0
 *  k_neighbors      K >= 0, at most 63
 *  flags            OR of QS_* switches above
 *  seed             key of the counter-based noise (Philox4x32-10)
 *  dw_*             downwash (QS_DOWNWASH): an airborne quad with a
 *                   swarm-mate above it, horizontal offset < dw_radius (m) and
 *                   height difference dz in (0, dw_height) (m), gets the
 *                   acceleration -dw_k1 (dw_k2 dz + dw_b1) e_z (summed over
 *                   such swarm-mates) plus N(0, dw_noise_a^2) per axis
 *                   (m/s^2), and N(0, dw_noise_w^2) angular acceleration
 *                   (rad/s^2), as a kick of dt times them after the pair
 *                   response.  Not differentiated.
 *  sn_x, sn_v, sn_w sensor noise (QS_SENSOR_NOISE), all >= 0: each
 *                   observation row gets U(-sn_x, sn_x) added to every
 *                   component of x - goal (m), U(-sn_v, sn_v) to v (m/s) and
 *                   N(0, sn_w^2) to omega (rad/s), drawn at the substep index
 *                   of the observed state; R and the neighbour slots are
 *                   exact.
 */
typedef struct {
  int32_t n_envs;
  const int32_t* env_offsets;
  float dt, gravity, arm_length, k_tau, drag_coef, floor_mu;
  float motor_noise_decay, motor_noise_std;
  float room_min[3], room_max[3], wall_restitution;
  float col_dist, col_decay, col_noise_v, col_noise_w;
  int32_t k_neighbors;
  uint32_t flags;
  uint64_t seed;
  float dw_k1, dw_k2, dw_b1, dw_radius, dw_height, dw_noise_a, dw_noise_w;
  float sn_x, sn_v, sn_w;
} qs_desc;

/* Per-quad domain-randomised physical parameters (§I, §III-A). */
typedef struct {
  float mass, ixx, iyy, izz, thrust_to_weight, motor_tau;
} qs_quad_params;

/*
 * Create a handle on the current HIP device: validates desc, h_params [Q]
 * and h_state0 [Q][27] (all finite; mass, inertia, thrust-to-weight and
 * tau_m > 0), derives f_max = m g t2w / 4 and alpha_lag = 1 - exp(-dt/tau_m)
 * per quad, allocates the private device state and uploads it (synchronous).
 * The substep counter starts at 0.  On error *out is left NULL.
 */
int qs_create(const qs_desc* desc, const qs_quad_params* h_params,
              const float* h_state0, qs_handle** out);

/* Free the handle and its device memory (synchronises the device). NULL is OK.
 * Infrastructure: no passage of the paper; it releases what qs_create took. */
int qs_destroy(qs_handle* h);

/* Sizes of a handle: number of quads, of environments, and the §III-C
 * observation row length 18 + 6K.  Infrastructure. */
int qs_sizes(const qs_handle* h, int32_t* n_quads, int32_t* n_envs, int32_t* obs_dim);

/* Substep counter: number of substeps enqueued so far (keys the noise).
 * Infrastructure. */
int qs_substep_index(const qs_handle* h, uint64_t* substep_index);

/*
 * Advance every quad by n_substeps substeps of dt, holding d_actions [Q][4]
 * for all of them (§III-A.1: the policy acts once per control step; the
 * simulator takes several physics substeps per action).  Each substep runs
 * motor command, lag and noise, thrust and torque mix, gravity and drag,
 * semi-implicit Euler with Gram-Schmidt re-orthonormalisation, walls,
 * ceiling and floor, then the in-env pair pass.  n_substeps >= 0.
 */
int qs_step(qs_handle* h, const float* d_actions, int32_t n_substeps, void* stream);

/* §III-C observation of the current state into d_obs [Q][18+6K]. */
int qs_observe(qs_handle* h, const float* d_goals, float* d_obs, void* stream);

/*
 * qs_step followed by qs_observe, in one launch: the state stays in
 * registers across the substeps and the observation is written from them.
 * Results are identical to the two calls made one after the other.
 */
int qs_step_observe(qs_handle* h, const float* d_actions, int32_t n_substeps,
                    const float* d_goals, float* d_obs, void* stream);

/*
 * §III-E reward weights of the handle, h_w[15] (host): alpha_pos, alpha_vel,
 * alpha_ori, alpha_spin, alpha_act, alpha_dact, alpha_rot, alpha_yaw,
 * alpha_floor_hit, alpha_on_floor, alpha_wall, alpha_ceiling, alpha_quad,
 * alpha_prox, d_prox.  All finite, d_prox > 0 (QS_ERR_INVALID otherwise).
 * Synchronises the device (work already enqueued keeps the old weights),
 * then applies to calls enqueued after it.  A new handle has all weights 0
 * and d_prox = 1.  Not to be called during stream capture.
 */
int qs_set_reward_weights(qs_handle* h, const float* h_w);

/*
 * qs_step_observe that also writes each quad's reward of the call into
 * d_reward [Q] (n_substeps >= 1):
 *   r = a_pos |x - goal| + a_vel |v| + a_ori R22 + a_spin |omega|
 *     + a_act |f| + a_dact |f - f_prev| + a_rot (tr R - 1)/2 + a_yaw R00
 *     + a_floor_hit [hit the floor] + a_on_floor [resting at the end]
 *     + a_wall [bounced off a wall] + a_ceiling [bounced off the ceiling]
 *     + a_quad [received a collision response]
 *     + a_prox sum over the K neighbour slots of max(1 - |x_j - x_i| / d_prox, 0)
 * with x, v, R, omega the state after the call, f = f_max u_f^2 + eps the
 * rotor thrusts after (f) and before (f_prev) the call, and each [event]
 * 1 if it happened at any substep of the call.  The reward reads the exact
 * (noise-free) observation; QS_SENSOR_NOISE noise goes into d_obs only.
 */
int qs_step_observe_reward(qs_handle* h, const float* d_actions, int32_t n_substeps,
                           const float* d_goals, float* d_obs, float* d_reward, void* stream);

/*
 * Copy the state into d_state [Q][27] (canonical layout) and return the
 * substep counter (number of substeps enqueued so far; host value).
 * substep_index may be NULL.  The state is §III-A's rigid body (x, v, R,
 * omega) with the rotor state of §III-A.1/§III-A.2 (u_f, eps) and the
 * resting flag of §III-B.3; the layout is the library's own.
 */
int qs_get_state(qs_handle* h, float* d_state, uint64_t* substep_index, void* stream);

/*
 * Load d_state [Q][27] for the environments whose d_env_mask[e] != 0
 * (d_env_mask NULL: all) and set the substep counter, which keys the noise.
 * Values are taken as given (not validated on the device).  Same state as
 * qs_get_state (§III-A, §III-A.1/2, §III-B.3); resetting environments
 * between episodes is what the training loop of §III-D asks of it.
 */
int qs_set_state(qs_handle* h, const float* d_state, uint64_t substep_index,
                 const uint8_t* d_env_mask, void* stream);

/*
 * Replace the per-quad parameters (§I domain randomisation of the §III-A
 * mass and inertia, §III-A.2 thrust-to-weight, §III-A.1 motor time
 * constant) of the environments whose d_env_mask[e] != 0 (NULL: all) with
 * d_params [Q][6] (device memory, qs_quad_params rows, 4-byte aligned), and
 * re-derive f_max = m g t2w / 4 and alpha_lag = 1 - exp(-dt / tau_m) on the
 * device, as qs_create does.  Stream-ordered: calls enqueued after it use
 * the new values.  Every entry of a selected row must be finite and > 0; a
 * row that is not keeps its old values and makes the next qs_sync return
 * QS_ERR_INVALID.  Allocates nothing (can be captured in a graph).
 */
int qs_set_params(qs_handle* h, const float* d_params, const uint8_t* d_env_mask, void* stream);

/*
 * Enable (enable != 0) or disable recording of the §III-B.1 contact sets
 * (centre distance below col_dist within an environment).  While
 * enabled, every qs_step / qs_step_observe writes, for each quad, the mask
 * of swarm-mates it was in contact with (|x_i - x_j| < col_dist) at its last
 * substep; qs_debug_contacts copies it to d_mask [Q] (bit j = the
 * environment's j-th quad).  Recording costs 8 bytes per quad per call.
 */
int qs_record_contacts(qs_handle* h, int32_t enable);
int qs_debug_contacts(qs_handle* h, uint64_t* d_mask, void* stream);

/*
 * Wait for the handle's work on `stream` and return the sticky device error
 * raised since the last qs_sync: QS_ERR_NONFINITE for a non-finite action
 * or state, else QS_ERR_INVALID for a rejected qs_set_params row; QS_OK if
 * none.  Synchronous.  The error is cleared by the call that reports it.
 * Infrastructure (no passage of the paper).
 */
int qs_sync(qs_handle* h, void* stream);

/* ---- differentiation (reverse mode) ----------------------------------------
 * Loss model: L = l(final state) + sum_q gpen[q] * pen[q], where pen[q] is
 * quad q's half-share of the smoothed collision penalty
 *     sum over substeps, env-mates j of softplus(beta (col_dist - d_qj)) / beta
 * (d_qj: centre distance after the substep's motion; a smooth version of
 * the hinge proximity term of §III-E).  Derivatives are exact for the branch
 * each event took (walls, floor, contacts, friction regime); the resting
 * flag carries none.  Handles with QS_DOWNWASH return QS_ERR_UNSUPPORTED
 * from the two backward calls.  Checkpoint k of a rollout is the state at the start of
 * call k * ckpt_every, stored field-major [27][Q] (state row layout, one
 * field after another).
 */

/*
 * Run n_calls calls of n_substeps substeps from the handle's state, the
 * action of call k being d_actions + k*Q*4 ([n_calls][Q][4], 16-byte
 * aligned).  d_ckpt (optional): ceil(n_calls/ckpt_every) checkpoints
 * [..][27][Q].  d_penalty (optional, [Q]): pen[q] is ADDED (beta > 0).
 * The handle's state and substep counter advance as n_calls qs_step calls
 * would (bitwise identical states).
 */
int qs_rollout(qs_handle* h, const float* d_actions, int32_t n_calls, int32_t n_substeps,
               int32_t ckpt_every, float* d_ckpt, float* d_penalty, float beta, void* stream);

/*
 * Reverse pass of a qs_rollout that started at substep substep_index0 with
 * the same d_actions, n_calls, n_substeps, ckpt_every and its d_ckpt.
 * d_gstate [Q][27]: dL/d(final state) on entry, dL/d(initial state) on
 * return.  d_gpenalty (optional, [Q]): dL/d pen.  Writes d_gactions
 * [n_calls][Q][4] and ADDS dL/d(mass, ixx, iyy, izz, thrust_to_weight,
 * motor_tau) into d_gparams [Q][6].  Each segment of ckpt_every calls is
 * recomputed from its checkpoint into a tape of ckpt_every*n_substeps
 * states and motor-noise draws (31 floats per quad and substep; device
 * scratch owned by the handle, grown on first use, at most the tape budget:
 * environment QS_TAPE_BYTES, default 8 GiB, and one segment).  Does not
 * change the handle's state.
 */
int qs_rollout_backward(qs_handle* h, const float* d_actions, int32_t n_calls,
                        int32_t n_substeps, int32_t ckpt_every, const float* d_ckpt,
                        uint64_t substep_index0, float* d_gstate, const float* d_gpenalty,
                        float beta, float* d_gactions, float* d_gparams, void* stream);

/*
 * Vector-Jacobian product of one qs_step call: from d_state_in [Q][27] (the
 * state before the call), d_actions [Q][4], n_substeps and the call's first
 * substep index, map d_gstate_out [Q][27] = dL/d(state after) to
 * d_gstate_in [Q][27] = dL/d(state before) and d_gactions [Q][4], and ADD
 * dL/d(params) into d_gparams [Q][6].  No penalty term.  d_gstate_in may
 * be the same buffer as d_gstate_out (both are staged through the handle's
 * scratch).
 */
int qs_step_backward(qs_handle* h, const float* d_state_in, const float* d_actions,
                     int32_t n_substeps, uint64_t substep_index, const float* d_gstate_out,
                     float* d_gstate_in, float* d_gactions, float* d_gparams, void* stream);

/*
 * qs_step_backward for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, checks and results (bit-identical) as
 * qs_step_backward, same kernels; it calls no hipMalloc, hipFree or other
 * allocating routine.  Its scratch -- the state before the call and the
 * state adjoint ([27][Q] each), the parameter gradient ([6][Q]) and the
 * tape of the call's substeps ([n_substeps][31][Q]), each part rounded up
 * to 64 floats -- lives in a fixed device array of QS_NOALLOC_SCRATCH_BYTES
 * that the library holds on every device it runs on until the process
 * ends.  A request that does not fit returns QS_ERR_TOO_LARGE before
 * anything is enqueued: (60 + 31 n_substeps) Q floats must stay within
 * 16,777,216 (e.g. at most 184,000 quads for one substep, 45,000 for ten).
 * Every call on a device shares that device's array and the array keeps
 * the last call's contents (each call overwrites what it reads): calls
 * that overlap in time on one device (several streams, threads or
 * handles) race, and the caller must order them.
 */
int qs_step_backward_noalloc(qs_handle* h, const float* d_state_in, const float* d_actions,
                             int32_t n_substeps, uint64_t substep_index,
                             const float* d_gstate_out, float* d_gstate_in, float* d_gactions,
                             float* d_gparams, void* stream);

/* ---- batching and scheduling ------------------------------------------------
 * Swarms of uneven sizes run in one persistent launch: every swarm gets a
 * slot of the next power of two >= its size, slots of one size are grouped
 * into work items, and each workgroup strides over the items running code
 * specialised for the item's slot size (environment QS_BUCKETED=0 at
 * qs_create falls back to one workgroup per greedy block of swarms).
 */

/*
 * Graph mode (enable != 0): every step launch reads the base substep index
 * from device memory and the last workgroup of the launch advances it, so a
 * captured hipGraph of qs_step / qs_step_observe calls draws fresh noise on
 * every replay.  While on, qs_substep_index synchronises the device and
 * reads the device counter.  qs_rollout/qs_rollout_backward keep using the
 * host counter.  Synchronises `stream`.
 */
int qs_set_graph_mode(qs_handle* h, int32_t enable, void* stream);

/*
 * Set the launch configuration explicitly: workgroup size 64 or 128 and, for
 * uneven swarm sizes, the persistent grid size (0: one workgroup per work
 * item).  Synchronises the device.
 */
int qs_set_launch(qs_handle* h, int32_t block, int32_t grid);

/*
 * The project's autotuner: time candidate launch configurations of
 * qs_step_observe (d_goals and d_obs non-NULL) or qs_step (both NULL) with
 * n_substeps substeps on the handle's own swarms (each candidate from the
 * same saved state), keep the fastest, and restore the state, the substep
 * counter and the sticky error word.  Uniform swarm sizes: workgroup size
 * 64 or 128.  Uneven sizes (the bucketed form): (1) workgroup sizes 64 and
 * 128 and persistent grids, every slot size with the in-swarm loops taking
 * one partner at a time; (2) per slot size of 16 and 32, its work items
 * alone with that body and with the body that takes the partners in chunks
 * of four; (3) the call with each slot size on its faster body, over the
 * grids; the faster of (1) and (3) is kept.  choice (optional, int32[3])
 * receives (workgroup size, grid size or 0 for one workgroup per item,
 * bucketed ? 1 : 0); qs_launch_plan gives the per-slot table.  Not
 * available in graph mode.  Synchronous.  This is the batching workload's
 * schedule search; the paper has no counterpart.
 */
int qs_autotune(qs_handle* h, const float* d_actions, int32_t n_substeps, const float* d_goals,
                float* d_obs, int32_t* choice, void* stream);

/*
 * Bucketed form: the slot sizes whose work items take the in-swarm
 * partners in chunks of four (their loads in flight together) instead of
 * one at a time: bit k of slot_mask for slots of 2^k quads, k = 4 or 5
 * (slots of 16 and 32; QS_ERR_INVALID for other bits).  Results are
 * bit-identical either way.  Synchronises the device.  (qs_autotune sets it
 * from its measurements.)
 */
int qs_set_partner_chunks(qs_handle* h, uint32_t slot_mask);

/*
 * The per-slot-size plan of the bucketed form, into plan [7][5] (host), one
 * row per slot size present, largest first: slot size, swarms, 1 if its
 * items take the chunked body else 0, and the times (ns per launch) the
 * last qs_autotune measured for the slot's items alone with the
 * one-partner and with the chunked body (0 where not measured).  *n_rows
 * receives the number of rows (0 for handles of uniform sizes).
 */
int qs_launch_plan(const qs_handle* h, int32_t* plan, int32_t* n_rows);

/* ---- diagnostics -------------------------------------------------------------
 * The noise of §III-A.2 (motor), §III-B (wall, pair and downwash kicks) and
 * §III-C (sensor) comes from one counter-based generator, Philox4x32-10
 * (Salmon et al., SC'11; the paper names no generator): key = seed, counter
 * = (quad, substep low word, substep high word, noise_stream << 8 | draw),
 * streams 0 motor, 1 wall, 2 pair, 3 downwash, 4 sensor.
 *
 * qs_debug_philox writes, for quads quad0 .. quad0 + n - 1 at substep_index,
 * the generator's four 32-bit words into d_words [n][4] and, if d_normals
 * is not NULL, the four N(0,1) draws the library builds from them (uniforms
 * (2 (r >> 9) + 1) 2^-24, Box-Muller on (w0, w1) and (w2, w3)) into
 * d_normals [n][4].  Device buffers, 4-byte aligned, not overlapping;
 * noise_stream < 2^24, draw < 256, quad0 + n <= 2^32 (QS_ERR_INVALID
 * otherwise).  No handle: it runs on the current device and `stream`.
 * For tests of the generator against an independent implementation.
 */
int qs_debug_philox(uint64_t seed, uint32_t noise_stream, uint32_t draw, uint64_t substep_index,
                    uint32_t quad0, int32_t n, uint32_t* d_words, float* d_normals,
                    void* stream);

/* Static description of a return code. */
const char* qs_error_string(int code);

#ifdef __cplusplus
}
#endif

#endif /* QUADSWARM_H */
