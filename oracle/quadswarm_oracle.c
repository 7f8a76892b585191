/*
 * FP64 reference stepper for the batched quadrotor-swarm simulator of
 * "QuadSwarm: A Modular Multi-Quadrotor Simulator for Deep Reinforcement
 * Learning with Direct Thrust Control" (Huang et al., arXiv 2306.09537).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * constant generator with the GPU library: every convention it needs is
 * written out again here from the paper and from the readings listed below.
 *
 * It is deliberately plain: one quad at a time, one substep at a time, every
 * step in the order the paper's equations give it, in double precision.
 * OpenMP runs independent environments in parallel; inside an environment
 * everything is serial.
 *
 * Readings of points the paper leaves open (each one is also a test pin):
 *  - Action map (§III-A.1): fhat = (clip(a,-1,1)+1)/2, uhat = sqrt(fhat);
 *    with ACT_UNIT the action is fhat itself, clipped to [0,1].
 *  - Motor lag (§III-A.1): u <- u + alpha_lag (uhat - u), with
 *    alpha_lag = 1 - exp(-dt/tau_m) (exact discretisation of a first-order
 *    lag of time constant tau_m; its 2 % settling time is 3.9 tau_m).
 *  - Motor noise (§III-A.2): eps <- a_nd eps + a_ns N(0,1), in newtons, with
 *    a_ns = sigma f_max sqrt(1 - a_nd^2) so that the stationary std is
 *    sigma f_max.  N(0,1) comes from Philox4x32-10 (Salmon et al., SC'11)
 *    keyed by the seed, counter (quad, t_lo, t_hi, stream), mapped to
 *    uniforms (2 (r >> 9) + 1) 2^-24 and paired by Box-Muller (1958).
 *  - Thrust (§III-A.2): f = f_max u^2 + eps, f_max = m g t2w / 4, no clamp.
 *  - Mix (§III-A): X configuration, body frame forward-left-up, rotors at
 *    d(+1,-1), d(-1,-1), d(-1,+1), d(+1,+1), d = arm/sqrt(2); thrust torque
 *    sum r_i x f_i e_z; propeller reaction k_tau s_i f_i e_z, s = (+,-,+,-).
 *  - Frames (§III-A): R maps body to world; omega is a body rate, so the
 *    attitude rate is R [omega]x (the paper's "omega_x R" read as the body
 *    form, which is the one consistent with a constant inertia matrix).
 *  - Integrator: semi-implicit Euler: accelerations from the start-of-substep
 *    state, v then x, omega then R; then Gram-Schmidt on the columns of R.
 *  - Drag: -c_d v in the world frame (c_d = 0 gives the paper's equations).
 *  - Walls and ceiling (§III-B.2): the wall acts as the quad's mirror image,
 *    so the pair rule gives v_n <- -e v_n; position clamped onto the wall;
 *    decay and noise applied once per substep in which any wall bounced.
 *  - Floor (§III-B.3): z < floor height is a hit: z on the floor, v = w = 0,
 *    R upright with the yaw kept, resting flag set.  While resting and the
 *    world-z thrust does not exceed m g: a_z = v_z = 0, omega = 0, R held,
 *    static friction if v_xy = 0 else kinetic friction opposite v_xy, and a
 *    zero-crossing guard.  The floor does not bounce.
 *  - Pairs (§III-B.1): contact iff |x_i - x_j|^2 < d_col^2 within an env;
 *    response only while approaching ((v_j - v_i).n > 0) when APPROACH_ONLY;
 *    simultaneous contacts summed from pre-response velocities (Jacobi);
 *    decay and noise applied once per responding quad; n = +e_z for the lower
 *    index when the two positions coincide (|dx|^2 < 1e-12).
 *  - Observation (§III-C): [x - goal, v, R row-major, omega, K slots of
 *    (x_j - x_i, v_j - v_i)] for the K nearest by (d^2, index), zero padding.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_ROOM 1u
#define OR_FLOOR 2u
#define OR_COLLIDE 4u
#define OR_MOTOR_NOISE 8u
#define OR_APPROACH_ONLY 16u
#define OR_ACT_UNIT 32u

/* canonical state row: x3 v3 R9 (row-major) w3 u4 eps4 floor1 */
enum { IX = 0, IV = 3, IR = 6, IW = 15, IU = 18, IE = 22, IF = 26, NS = 27 };
/* parameter row: mass, ixx, iyy, izz, thrust_to_weight, motor_tau */
enum { PM = 0, PJX = 1, PJY = 2, PJZ = 3, PT2W = 4, PTAU = 5, NP = 6 };

/* noise streams (fourth counter word = stream << 8 | draw) */
enum { STREAM_MOTOR = 0, STREAM_WALL = 1, STREAM_PAIR = 2 };

/* per-quad event bits reported by or_step (OR over the call's substeps) */
enum {
  EV_WALL = 1, EV_FLOOR_HIT = 2, EV_FRICTION = 4, EV_TAKEOFF = 8,
  EV_PAIR_RESPONSE = 16, EV_CONTACT = 32
};

typedef struct {
  int32_t n_envs;
  const int32_t* env_offsets; /* [E+1] CSR, 1 <= n_e <= 64 */
  double dt, gravity, arm_length, k_tau, drag_coef, floor_mu;
  double motor_noise_decay, motor_noise_std;
  double room_min[3], room_max[3], wall_restitution;
  double col_dist, col_decay, col_noise_v, col_noise_w;
  int32_t k_neighbors;
  uint32_t flags;
  uint64_t seed;
  uint32_t quad_id_offset; /* global index of quad 0 (noise counter) */
} or_desc;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as  */
/* easy as 1, 2, 3", SC'11).  A round multiplies counter words 0 and 2 by   */
/* two fixed odd constants into 64-bit products; the new counter is         */
/* (hi(w2*M1) ^ w1 ^ k0, lo(w2*M1), hi(w0*M0) ^ w3 ^ k1, lo(w0*M0)); the     */
/* key is bumped by the two Weyl constants between rounds.                  */
/* ------------------------------------------------------------------------ */
void or_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                      uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
    uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += W0; k1 += W1;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform in (0,1) from the top 23 bits: (2k+1) 2^-24, never 0 or 1. */
double or_uniform_from_u32(uint32_t r) {
  return (double)(2u * (r >> 9) + 1u) * (1.0 / 16777216.0);
}

/* Four standard normals for (quad, substep t, stream, draw). */
void or_normal4(uint64_t seed, uint32_t quad, uint64_t t, uint32_t stream,
                uint32_t draw, double z[4]) {
  uint32_t ctr[4] = {quad, (uint32_t)t, (uint32_t)(t >> 32), (stream << 8) | draw};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t r[4];
  or_philox4x32_10(ctr, key, r);
  const double two_pi = 6.283185307179586476925286766559;
  for (int p = 0; p < 2; ++p) {
    double u1 = or_uniform_from_u32(r[2 * p]);
    double u2 = or_uniform_from_u32(r[2 * p + 1]);
    double rad = sqrt(-2.0 * log(u1));
    z[2 * p] = rad * cos(two_pi * u2);
    z[2 * p + 1] = rad * sin(two_pi * u2);
  }
}

/* ------------------------------------------------------------------------ */
/* Per-quad part of one substep (everything before the in-env pair pass).   */
/* ------------------------------------------------------------------------ */
static double clampd(double a, double lo, double hi) {
  return a < lo ? lo : (a > hi ? hi : a);
}

static void upd_margin(double* mg, double v) {
  v = fabs(v);
  if (v < *mg) *mg = v;
}

/* mg: smallest distance of any threshold decision of this substep from its
 * threshold (diagnostic only; it does not change the arithmetic). */
static void quad_substep(const or_desc* d, const double* p, double* s,
                         const double* act, uint32_t q, uint64_t t,
                         uint32_t* ev, double* mg) {
  const double dt = d->dt, g = d->gravity;
  const double m = p[PM], jx = p[PJX], jy = p[PJY], jz = p[PJZ];
  const double f_max = 0.25 * m * g * p[PT2W];              /* §III-A.2 */
  const double alpha_lag = 1.0 - exp(-dt / p[PTAU]);          /* §III-A.1 */
  const double a_nd = d->motor_noise_decay;
  const double a_ns = d->motor_noise_std * f_max * sqrt(1.0 - a_nd * a_nd);
  const double arm_d = d->arm_length / sqrt(2.0);

  /* §III-A.1: normalised thrust command, then rotor speed command */
  double uhat[4];
  for (int i = 0; i < 4; ++i) {
    double fhat = (d->flags & OR_ACT_UNIT) ? clampd(act[i], 0.0, 1.0)
                                           : 0.5 * (clampd(act[i], -1.0, 1.0) + 1.0);
    uhat[i] = sqrt(fhat);
  }
  /* §III-A.1: first-order low-pass motor lag */
  for (int i = 0; i < 4; ++i) s[IU + i] = alpha_lag * (uhat[i] - s[IU + i]) + s[IU + i];
  /* §III-A.2: AR(1) motor noise */
  if (d->flags & OR_MOTOR_NOISE) {
    double z[4];
    or_normal4(d->seed, q, t, STREAM_MOTOR, 0, z);
    for (int i = 0; i < 4; ++i) s[IE + i] = a_nd * s[IE + i] + a_ns * z[i];
  }
  /* §III-A.2: per-motor thrust */
  double f[4];
  for (int i = 0; i < 4; ++i) f[i] = f_max * s[IU + i] * s[IU + i] + s[IE + i];

  /* §III-A: total thrust and torque = thrust moments + propeller reaction */
  double T = (f[0] + f[1]) + (f[2] + f[3]);
  double tau[3];
  tau[0] = arm_d * ((f[2] + f[3]) - (f[0] + f[1]));
  tau[1] = arm_d * ((f[1] + f[2]) - (f[0] + f[3]));
  tau[2] = d->k_tau * ((f[0] + f[2]) - (f[1] + f[3]));

  double* x = s + IX;
  double* v = s + IV;
  double* R = s + IR; /* row-major: R[3*r + c] */
  double* w = s + IW;

  /* §III-A: world-frame thrust force R (0,0,T) */
  double F[3] = {T * R[2], T * R[5], T * R[8]};

  int friction = (d->flags & OR_FLOOR) && s[IF] != 0.0 && F[2] <= m * g;
  if ((d->flags & OR_FLOOR) && s[IF] != 0.0) upd_margin(mg, (F[2] - m * g) / (m * g));
  if (!friction) {
    if (s[IF] != 0.0) *ev |= EV_TAKEOFF;
    s[IF] = 0.0;
    /* linear acceleration: gravity + thrust/m - drag */
    double acc[3];
    for (int k = 0; k < 3; ++k) acc[k] = F[k] / m - d->drag_coef / m * v[k];
    acc[2] -= g;
    /* Euler's equation from the start-of-substep omega */
    double Jw[3] = {jx * w[0], jy * w[1], jz * w[2]};
    double wxJw[3] = {w[1] * Jw[2] - w[2] * Jw[1], w[2] * Jw[0] - w[0] * Jw[2],
                      w[0] * Jw[1] - w[1] * Jw[0]};
    double wdot[3] = {(tau[0] - wxJw[0]) / jx, (tau[1] - wxJw[1]) / jy,
                      (tau[2] - wxJw[2]) / jz};
    /* semi-implicit Euler */
    for (int k = 0; k < 3; ++k) v[k] += dt * acc[k];
    for (int k = 0; k < 3; ++k) x[k] += dt * v[k];
    for (int k = 0; k < 3; ++k) w[k] += dt * wdot[k];
    /* attitude: R <- R + dt R [w]x, with the new omega */
    double W[9] = {0.0, -w[2], w[1], w[2], 0.0, -w[0], -w[1], w[0], 0.0};
    double Rn[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        double acc_rc = 0.0;
        for (int k = 0; k < 3; ++k) acc_rc += R[3 * r + k] * W[3 * k + c];
        Rn[3 * r + c] = R[3 * r + c] + dt * acc_rc;
      }
    /* Gram-Schmidt on the columns: c0, c1 orthonormalised, c2 = c0 x c1 */
    double c0[3] = {Rn[0], Rn[3], Rn[6]}, c1[3] = {Rn[1], Rn[4], Rn[7]};
    double n0 = sqrt(c0[0] * c0[0] + c0[1] * c0[1] + c0[2] * c0[2]);
    for (int k = 0; k < 3; ++k) c0[k] /= n0;
    double dp = c0[0] * c1[0] + c0[1] * c1[1] + c0[2] * c1[2];
    for (int k = 0; k < 3; ++k) c1[k] -= dp * c0[k];
    double n1 = sqrt(c1[0] * c1[0] + c1[1] * c1[1] + c1[2] * c1[2]);
    for (int k = 0; k < 3; ++k) c1[k] /= n1;
    double c2[3] = {c0[1] * c1[2] - c0[2] * c1[1], c0[2] * c1[0] - c0[0] * c1[2],
                    c0[0] * c1[1] - c0[1] * c1[0]};
    for (int r = 0; r < 3; ++r) {
      R[3 * r + 0] = c0[r];
      R[3 * r + 1] = c1[r];
      R[3 * r + 2] = c2[r];
    }
  } else {
    /* §III-B.3: resting on the floor with thrust too small to take off */
    *ev |= EV_FRICTION;
    double N = m * g - F[2];
    double mu_n = d->floor_mu * N;
    double fb[2];
    double vxy0[2] = {v[0], v[1]};
    if (v[0] == 0.0 && v[1] == 0.0) {
      double nf = sqrt(F[0] * F[0] + F[1] * F[1]);
      double mag = nf - mu_n > 0.0 ? nf - mu_n : 0.0;
      fb[0] = nf > 0.0 ? mag * F[0] / nf : 0.0;
      fb[1] = nf > 0.0 ? mag * F[1] / nf : 0.0;
    } else {
      double nv = sqrt(v[0] * v[0] + v[1] * v[1]);
      fb[0] = F[0] - mu_n * v[0] / nv;
      fb[1] = F[1] - mu_n * v[1] / nv;
    }
    double acc[2] = {(fb[0] - d->drag_coef * v[0]) / m, (fb[1] - d->drag_coef * v[1]) / m};
    v[0] += dt * acc[0];
    v[1] += dt * acc[1];
    v[2] = 0.0;
    double dot = v[0] * vxy0[0] + v[1] * vxy0[1];
    if (vxy0[0] != 0.0 || vxy0[1] != 0.0)
      upd_margin(mg, dot / (vxy0[0] * vxy0[0] + vxy0[1] * vxy0[1]));
    if (dot < 0.0) { v[0] = 0.0; v[1] = 0.0; }
    for (int k = 0; k < 3; ++k) x[k] += dt * v[k];
    w[0] = w[1] = w[2] = 0.0;
  }

  /* §III-B.2: walls (x, y) and ceiling (z max) */
  if (d->flags & OR_ROOM) {
    int bounced = 0;
    const double e = d->wall_restitution;
    for (int k = 0; k < 3; ++k) {
      if (k < 2) upd_margin(mg, x[k] - d->room_min[k]);
      upd_margin(mg, x[k] - d->room_max[k]);
      if (k < 2 && x[k] < d->room_min[k]) {
        x[k] = d->room_min[k];
        if (v[k] < 0.0) { v[k] = -e * v[k]; bounced = 1; }
      }
      if (x[k] > d->room_max[k]) {
        x[k] = d->room_max[k];
        if (v[k] > 0.0) { v[k] = -e * v[k]; bounced = 1; }
      }
    }
    if (bounced) {
      *ev |= EV_WALL;
      double zv[4] = {0, 0, 0, 0}, zw[4] = {0, 0, 0, 0};
      if (d->col_noise_v > 0.0 || d->col_noise_w > 0.0) {
        or_normal4(d->seed, q, t, STREAM_WALL, 0, zv);
        or_normal4(d->seed, q, t, STREAM_WALL, 1, zw);
      }
      for (int k = 0; k < 3; ++k) {
        v[k] = d->col_decay * (v[k] + d->col_noise_v * zv[k]);
        w[k] = w[k] + d->col_noise_w * zw[k];
      }
    }
  }

  /* §III-B.3: floor hit */
  if ((d->flags & OR_FLOOR) && s[IF] == 0.0) upd_margin(mg, x[2] - d->room_min[2]);
  if ((d->flags & OR_FLOOR) && x[2] < d->room_min[2]) {
    *ev |= EV_FLOOR_HIT;
    x[2] = d->room_min[2];
    v[0] = v[1] = v[2] = 0.0;
    w[0] = w[1] = w[2] = 0.0;
    s[IF] = 1.0;
    double hx = R[0], hy = R[3];
    double nh = sqrt(hx * hx + hy * hy);
    double c0[3], c1[3];
    if (nh >= 1e-6) {
      c0[0] = hx / nh; c0[1] = hy / nh; c0[2] = 0.0;
      c1[0] = -c0[1]; c1[1] = c0[0]; c1[2] = 0.0;       /* e_z x c0 */
    } else {
      double kx = R[1], ky = R[4];
      double nk = sqrt(kx * kx + ky * ky);
      if (nk > 0.0) { c1[0] = kx / nk; c1[1] = ky / nk; }
      else { c1[0] = 0.0; c1[1] = 1.0; }
      c1[2] = 0.0;
      c0[0] = c1[1]; c0[1] = -c1[0]; c0[2] = 0.0;       /* c1 x e_z */
    }
    for (int r = 0; r < 3; ++r) {
      R[3 * r + 0] = c0[r];
      R[3 * r + 1] = c1[r];
      R[3 * r + 2] = r == 2 ? 1.0 : 0.0;
    }
  }
}

/* §III-B.1: pair pass of one environment after every quad moved. */
static void env_pairs(const or_desc* d, double* S, int q0, int n, uint64_t t,
                      uint64_t* contacts, uint32_t* events, double* mg) {
  double dv[64][3];
  int marked[64];
  memset(dv, 0, sizeof(dv));
  memset(marked, 0, sizeof(marked));
  const double dc2 = d->col_dist * d->col_dist;
  for (int i = 0; i < n; ++i) {
    const double* si = S + (size_t)(q0 + i) * NS;
    for (int j = i + 1; j < n; ++j) {
      const double* sj = S + (size_t)(q0 + j) * NS;
      double dx[3] = {si[IX] - sj[IX], si[IX + 1] - sj[IX + 1], si[IX + 2] - sj[IX + 2]};
      double d2 = dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2];
      double dm = sqrt(d2) - d->col_dist;
      upd_margin(&mg[q0 + i], dm);
      upd_margin(&mg[q0 + j], dm);
      if (!(d2 < dc2)) continue;
      if (contacts) {
        contacts[q0 + i] |= 1ull << j;
        contacts[q0 + j] |= 1ull << i;
      }
      events[q0 + i] |= EV_CONTACT;
      events[q0 + j] |= EV_CONTACT;
      double nrm[3];
      if (d2 < 1e-12) {
        nrm[0] = 0.0; nrm[1] = 0.0; nrm[2] = 1.0;
      } else {
        double dd = sqrt(d2);
        for (int k = 0; k < 3; ++k) nrm[k] = dx[k] / dd;
      }
      double sp = 0.0;
      for (int k = 0; k < 3; ++k) sp += (sj[IV + k] - si[IV + k]) * nrm[k];
      if (d->flags & OR_APPROACH_ONLY) {
        upd_margin(&mg[q0 + i], sp);
        upd_margin(&mg[q0 + j], sp);
      }
      if ((d->flags & OR_APPROACH_ONLY) && !(sp > 0.0)) continue;
      for (int k = 0; k < 3; ++k) {
        dv[i][k] += sp * nrm[k];
        dv[j][k] -= sp * nrm[k];
      }
      marked[i] = marked[j] = 1;
    }
  }
  for (int i = 0; i < n; ++i) {
    if (!marked[i]) continue;
    double* si = S + (size_t)(q0 + i) * NS;
    events[q0 + i] |= EV_PAIR_RESPONSE;
    double zv[4] = {0, 0, 0, 0}, zw[4] = {0, 0, 0, 0};
    if (d->col_noise_v > 0.0 || d->col_noise_w > 0.0) {
      or_normal4(d->seed, d->quad_id_offset + (uint32_t)(q0 + i), t, STREAM_PAIR, 0, zv);
      or_normal4(d->seed, d->quad_id_offset + (uint32_t)(q0 + i), t, STREAM_PAIR, 1, zw);
    }
    for (int k = 0; k < 3; ++k) {
      si[IV + k] = d->col_decay * (si[IV + k] + dv[i][k] + d->col_noise_v * zv[k]);
      si[IW + k] = si[IW + k] + d->col_noise_w * zw[k];
    }
  }
}

/* Argument checks shared by the entry points; 0 when valid. */
static int check_desc(const or_desc* d) {
  if (!d || !d->env_offsets || d->n_envs < 1 || d->k_neighbors < 0) return -1;
  if (d->env_offsets[0] != 0) return -1;
  for (int e = 0; e < d->n_envs; ++e) {
    int n = d->env_offsets[e + 1] - d->env_offsets[e];
    if (n < 1 || n > 64) return -1;
  }
  return 0;
}

/*
 * Advance every quad by n_sub substeps, holding the actions.  state[Q][27]
 * is updated in place; substep t0 + s draws the noise of step s.  contacts
 * (optional) receives, per quad, the contact bitmask of the last substep
 * (bit j = in contact with the env's quad j).  events (optional) receives
 * the OR of the EV_* bits over the call.  margin (optional) receives, per
 * quad, the smallest distance of any threshold decision taken for it during
 * the call from its threshold (metres for walls, floor and contact
 * distance; m/s for the approach test; relative for the take-off test and
 * the friction zero-crossing) -- a diagnostic for comparisons at a
 * different precision.  Returns 0, or -1 on bad arguments.
 */
int or_step(const or_desc* d, const double* params, double* state,
            const double* actions, int n_sub, uint64_t t0, uint64_t* contacts,
            uint32_t* events, double* margin) {
  if (check_desc(d) || !params || !state || !actions || n_sub < 0) return -1;
  const int E = d->n_envs;
  const int Q = d->env_offsets[E];
  uint32_t* ev = events ? events : (uint32_t*)calloc((size_t)Q + 1, sizeof(uint32_t));
  double* mg = margin ? margin : (double*)malloc(((size_t)Q + 1) * sizeof(double));
  if (!ev || !mg) {
    if (!events) free(ev);
    if (!margin) free(mg);
    return -1;
  }
  if (events) memset(events, 0, (size_t)Q * sizeof(uint32_t));
  for (int q = 0; q < Q; ++q) mg[q] = INFINITY;
  for (int sub = 0; sub < n_sub; ++sub) {
    const uint64_t t = t0 + (uint64_t)sub;
    if (contacts) memset(contacts, 0, (size_t)Q * sizeof(uint64_t));
#pragma omp parallel for schedule(static)
    for (int e = 0; e < E; ++e) {
      const int q0 = d->env_offsets[e], n = d->env_offsets[e + 1] - q0;
      for (int i = 0; i < n; ++i) {
        const int q = q0 + i;
        quad_substep(d, params + (size_t)q * NP, state + (size_t)q * NS,
                     actions + (size_t)q * 4, d->quad_id_offset + (uint32_t)q, t,
                     &ev[q], &mg[q]);
      }
      if ((d->flags & OR_COLLIDE) && n > 1) env_pairs(d, state, q0, n, t, contacts, ev, mg);
    }
  }
  if (!events) free(ev);
  if (!margin) free(mg);
  return 0;
}

/*
 * §III-C observation of every quad, obs[Q][18 + 6K]:
 * [x - goal, v, R row-major, omega, K x (x_j - x_i, v_j - v_i)] with the
 * K nearest env-mates ordered by (squared distance, index); slots beyond
 * n_e - 1 are zero.  nbr (optional, [Q][K]) receives the neighbour's local
 * index, -1 for a padded slot.
 */
int or_observe(const or_desc* d, const double* state, const double* goals,
               double* obs, int32_t* nbr) {
  if (check_desc(d) || !state || !goals || !obs) return -1;
  const int E = d->n_envs, K = d->k_neighbors, OD = 18 + 6 * K;
#pragma omp parallel for schedule(static)
  for (int e = 0; e < E; ++e) {
    const int q0 = d->env_offsets[e], n = d->env_offsets[e + 1] - q0;
    for (int i = 0; i < n; ++i) {
      const double* si = state + (size_t)(q0 + i) * NS;
      double* o = obs + (size_t)(q0 + i) * OD;
      for (int k = 0; k < 3; ++k) o[k] = si[IX + k] - goals[(size_t)(q0 + i) * 3 + k];
      for (int k = 0; k < 3; ++k) o[3 + k] = si[IV + k];
      for (int k = 0; k < 9; ++k) o[6 + k] = si[IR + k];
      for (int k = 0; k < 3; ++k) o[15 + k] = si[IW + k];
      /* selection sort of the env-mates by (d^2, index), first K kept */
      double dist[64];
      int used[64];
      for (int j = 0; j < n; ++j) {
        const double* sj = state + (size_t)(q0 + j) * NS;
        double a = sj[IX] - si[IX], b = sj[IX + 1] - si[IX + 1], c = sj[IX + 2] - si[IX + 2];
        dist[j] = a * a + b * b + c * c;
        used[j] = (j == i);
      }
      for (int slot = 0; slot < K; ++slot) {
        int best = -1;
        for (int j = 0; j < n; ++j)
          if (!used[j] && (best < 0 || dist[j] < dist[best])) best = j;
        double* os = o + 18 + 6 * slot;
        if (best < 0) {
          for (int k = 0; k < 6; ++k) os[k] = 0.0;
          if (nbr) nbr[(size_t)(q0 + i) * K + slot] = -1;
          continue;
        }
        used[best] = 1;
        const double* sj = state + (size_t)(q0 + best) * NS;
        for (int k = 0; k < 3; ++k) os[k] = sj[IX + k] - si[IX + k];
        for (int k = 0; k < 3; ++k) os[3 + k] = sj[IV + k] - si[IV + k];
        if (nbr) nbr[(size_t)(q0 + i) * K + slot] = best;
      }
    }
  }
  return 0;
}

int or_flag_values(uint32_t out[6]) {
  out[0] = OR_ROOM; out[1] = OR_FLOOR; out[2] = OR_COLLIDE;
  out[3] = OR_MOTOR_NOISE; out[4] = OR_APPROACH_ONLY; out[5] = OR_ACT_UNIT;
  return 0;
}
