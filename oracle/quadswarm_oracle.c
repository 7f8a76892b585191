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
 *  - Downwash (§III-B.4): an airborne quad i below quad j with
 *    |(x_j - x_i)_xy| < r and 0 < z_j - z_i < h gets the acceleration
 *    -k1 (k2 (z_j - z_i) + b1) e_z, summed over such j, plus N(0, s_a^2)
 *    acceleration noise and N(0, s_w^2) angular-acceleration noise, applied
 *    as a velocity / body-rate kick of dt times them after the pair response
 *    (evaluated on the post-motion positions).
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
#define OR_DOWNWASH 64u
#define OR_SENSOR_NOISE 128u

/* canonical state row: x3 v3 R9 (row-major) w3 u4 eps4 floor1 */
enum { IX = 0, IV = 3, IR = 6, IW = 15, IU = 18, IE = 22, IF = 26, NS = 27 };
/* parameter row: mass, ixx, iyy, izz, thrust_to_weight, motor_tau */
enum { PM = 0, PJX = 1, PJY = 2, PJZ = 3, PT2W = 4, PTAU = 5, NP = 6 };

/* noise streams (fourth counter word = stream << 8 | draw) */
enum { STREAM_MOTOR = 0, STREAM_WALL = 1, STREAM_PAIR = 2, STREAM_DOWNWASH = 3, STREAM_SENSOR = 4 };

/* per-quad event bits reported by or_step (OR over the call's substeps) */
enum {
  EV_WALL = 1, EV_FLOOR_HIT = 2, EV_FRICTION = 4, EV_TAKEOFF = 8,
  EV_PAIR_RESPONSE = 16, EV_CONTACT = 32, EV_DOWNWASH = 64, EV_CEILING = 128
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
  /* downwash (§III-B.4): a = -k1 (k2 dz + b1) e_z on the lower quad of a pair
   * overlapping in xy (|dxy| < dw_radius) with 0 < dz < dw_height */
  double dw_k1, dw_k2, dw_b1, dw_radius, dw_height, dw_noise_a, dw_noise_w;
  /* observation sensor noise (§III-C): half-widths of the uniform noise on
   * x - goal and v, standard deviation of the Gaussian noise on omega */
  double sn_x, sn_v, sn_w;
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

/* Markers for the op-counting build (oracle/opcount.cpp), which defines them
 * to leave what they wrap out of its count; here they are plain.
 * OR_MARGIN: a threshold-margin update (diagnostic output, not the method).
 * OR_CONST: a constant derived from a quad's parameters or the global
 * constants (f_max, alpha_lag, ...), which this plain oracle recomputes on
 * every substep although it is fixed for the quad. */
#ifndef OR_MARGIN
#define OR_MARGIN(mg, v) upd_margin(mg, v)
#endif
#ifndef OR_CONST
#define OR_CONST(x) (x)
#endif

/* Intermediates of one substep of one quad, kept for the reverse sweep. */
typedef struct {
  double uhat[4], u0[4], e0[4], z[4], u1[4], f[4];
  double f_max, alpha_lag, T, F[3], P[9], w0[3], v0[3];
  int noise, rest;
  /* free flight */
  double Jw[3], wxJw[3], wdot[3], w1[3], A0[3], A1[3], n0, c0[3], dp, n1, c1[3];
  /* resting on the floor */
  int statik, guard;
  double mu_n, fb[2], nv, nf, mag;
  /* walls and floor */
  int clamp[3], flip[3], bounced, hit, fallback;
  double hx, hy, nh, kx, ky, nk;
} or_rec;

/* mg: smallest distance of any threshold decision of this substep from its
 * threshold (diagnostic only; it does not change the arithmetic).
 * rec (optional) receives the substep's intermediates. */
static void quad_substep(const or_desc* d, const double* p, double* s,
                         const double* act, uint32_t q, uint64_t t,
                         uint32_t* ev, double* mg, or_rec* rec) {
  or_rec scratch_rec;
  or_rec* r = rec ? rec : &scratch_rec;
  memset(r, 0, sizeof(*r));
  const double dt = d->dt, g = d->gravity;
  const double m = p[PM], jx = p[PJX], jy = p[PJY], jz = p[PJZ];
  const double f_max = OR_CONST(0.25 * m * g * p[PT2W]);     /* §III-A.2 */
  const double alpha_lag = OR_CONST(1.0 - exp(-dt / p[PTAU])); /* §III-A.1 */
  const double a_nd = d->motor_noise_decay;
  const double a_ns = OR_CONST(d->motor_noise_std * f_max * sqrt(1.0 - a_nd * a_nd));
  const double arm_d = OR_CONST(d->arm_length / sqrt(2.0));

  /* §III-A.1: normalised thrust command, then rotor speed command */
  double uhat[4];
  for (int i = 0; i < 4; ++i) {
    double fhat = (d->flags & OR_ACT_UNIT) ? clampd(act[i], 0.0, 1.0)
                                           : 0.5 * (clampd(act[i], -1.0, 1.0) + 1.0);
    uhat[i] = sqrt(fhat);
  }
  r->f_max = f_max;
  r->alpha_lag = alpha_lag;
  for (int i = 0; i < 4; ++i) {
    r->uhat[i] = uhat[i];
    r->u0[i] = s[IU + i];
    r->e0[i] = s[IE + i];
  }
  for (int k = 0; k < 9; ++k) r->P[k] = s[IR + k];
  for (int k = 0; k < 3; ++k) {
    r->w0[k] = s[IW + k];
    r->v0[k] = s[IV + k];
  }
  /* §III-A.1: first-order low-pass motor lag */
  for (int i = 0; i < 4; ++i) s[IU + i] = alpha_lag * (uhat[i] - s[IU + i]) + s[IU + i];
  /* §III-A.2: AR(1) motor noise */
  if (d->flags & OR_MOTOR_NOISE) {
    double z[4];
    or_normal4(d->seed, q, t, STREAM_MOTOR, 0, z);
    for (int i = 0; i < 4; ++i) s[IE + i] = a_nd * s[IE + i] + a_ns * z[i];
    r->noise = 1;
    for (int i = 0; i < 4; ++i) r->z[i] = z[i];
  }
  /* §III-A.2: per-motor thrust */
  double f[4];
  for (int i = 0; i < 4; ++i) f[i] = f_max * s[IU + i] * s[IU + i] + s[IE + i];
  for (int i = 0; i < 4; ++i) {
    r->u1[i] = s[IU + i];
    r->f[i] = f[i];
  }

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
  r->T = T;
  for (int k = 0; k < 3; ++k) r->F[k] = F[k];

  int friction = (d->flags & OR_FLOOR) && s[IF] != 0.0 && F[2] <= m * g;
  r->rest = friction;
  if ((d->flags & OR_FLOOR) && s[IF] != 0.0) OR_MARGIN(mg, (F[2] - m * g) / (m * g));
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
    for (int k = 0; k < 3; ++k) {
      r->Jw[k] = Jw[k];
      r->wxJw[k] = wxJw[k];
      r->wdot[k] = wdot[k];
      r->w1[k] = w[k];
    }
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
    for (int k = 0; k < 3; ++k) {
      r->A0[k] = c0[k];
      r->A1[k] = c1[k];
    }
    double n0 = sqrt(c0[0] * c0[0] + c0[1] * c0[1] + c0[2] * c0[2]);
    for (int k = 0; k < 3; ++k) c0[k] /= n0;
    double dp = c0[0] * c1[0] + c0[1] * c1[1] + c0[2] * c1[2];
    for (int k = 0; k < 3; ++k) c1[k] -= dp * c0[k];
    double n1 = sqrt(c1[0] * c1[0] + c1[1] * c1[1] + c1[2] * c1[2]);
    for (int k = 0; k < 3; ++k) c1[k] /= n1;
    r->n0 = n0;
    r->dp = dp;
    r->n1 = n1;
    for (int k = 0; k < 3; ++k) {
      r->c0[k] = c0[k];
      r->c1[k] = c1[k];
    }
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
      r->statik = 1;
      r->nf = nf;
      r->mag = nf > 0.0 ? mag : 0.0;
    } else {
      double nv = sqrt(v[0] * v[0] + v[1] * v[1]);
      fb[0] = F[0] - mu_n * v[0] / nv;
      fb[1] = F[1] - mu_n * v[1] / nv;
      r->nv = nv;
    }
    r->mu_n = mu_n;
    r->fb[0] = fb[0];
    r->fb[1] = fb[1];
    double acc[2] = {(fb[0] - d->drag_coef * v[0]) / m, (fb[1] - d->drag_coef * v[1]) / m};
    v[0] += dt * acc[0];
    v[1] += dt * acc[1];
    v[2] = 0.0;
    double dot = v[0] * vxy0[0] + v[1] * vxy0[1];
    if (vxy0[0] != 0.0 || vxy0[1] != 0.0)
      OR_MARGIN(mg, dot / (vxy0[0] * vxy0[0] + vxy0[1] * vxy0[1]));
    if (dot < 0.0) { v[0] = 0.0; v[1] = 0.0; r->guard = 1; }
    for (int k = 0; k < 3; ++k) x[k] += dt * v[k];
    w[0] = w[1] = w[2] = 0.0;
  }

  /* §III-B.2: walls (x, y) and ceiling (z max) */
  if (d->flags & OR_ROOM) {
    int bounced = 0;
    const double e = d->wall_restitution;
    for (int k = 0; k < 3; ++k) {
      if (k < 2) OR_MARGIN(mg, x[k] - d->room_min[k]);
      OR_MARGIN(mg, x[k] - d->room_max[k]);
      if (k < 2 && x[k] < d->room_min[k]) {
        x[k] = d->room_min[k];
        r->clamp[k] = 1;
        if (v[k] < 0.0) { v[k] = -e * v[k]; bounced = 1; r->flip[k] = 1; }
      }
      if (x[k] > d->room_max[k]) {
        x[k] = d->room_max[k];
        r->clamp[k] = 1;
        if (v[k] > 0.0) { v[k] = -e * v[k]; bounced = 1; r->flip[k] = 1; }
      }
    }
    r->bounced = bounced;
    if (bounced) {
      if (r->flip[0] || r->flip[1]) *ev |= EV_WALL;
      if (r->flip[2]) *ev |= EV_CEILING;
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
  if ((d->flags & OR_FLOOR) && s[IF] == 0.0) OR_MARGIN(mg, x[2] - d->room_min[2]);
  if ((d->flags & OR_FLOOR) && x[2] < d->room_min[2]) {
    *ev |= EV_FLOOR_HIT;
    x[2] = d->room_min[2];
    v[0] = v[1] = v[2] = 0.0;
    w[0] = w[1] = w[2] = 0.0;
    s[IF] = 1.0;
    double hx = R[0], hy = R[3];
    double nh = sqrt(hx * hx + hy * hy);
    double c0[3], c1[3];
    r->hit = 1;
    r->hx = hx;
    r->hy = hy;
    r->nh = nh;
    r->fallback = !(nh >= 1e-6);
    r->kx = R[1];
    r->ky = R[4];
    r->nk = sqrt(R[1] * R[1] + R[4] * R[4]);
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
static double softplus(double x) { return x > 30.0 ? x : log1p(exp(x)); }
static double sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }

/* pen (optional): each quad's half of the smoothed collision penalty
 * softplus(beta (d_col - d_ij)) / beta over every pair of its env, added. */
static void env_pairs(const or_desc* d, double* S, int q0, int n, uint64_t t,
                      uint64_t* contacts, uint32_t* events, double* mg,
                      double* pen, double beta) {
  double dv[64][3];
  int marked[64];
  memset(dv, 0, sizeof(dv));
  memset(marked, 0, sizeof(marked));
  const double dc2 = OR_CONST(d->col_dist * d->col_dist);
  for (int i = 0; i < n; ++i) {
    const double* si = S + (size_t)(q0 + i) * NS;
    for (int j = i + 1; j < n; ++j) {
      const double* sj = S + (size_t)(q0 + j) * NS;
      double dx[3] = {si[IX] - sj[IX], si[IX + 1] - sj[IX + 1], si[IX + 2] - sj[IX + 2]};
      double d2 = dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2];
      OR_MARGIN(&mg[q0 + i], sqrt(d2) - d->col_dist);
      OR_MARGIN(&mg[q0 + j], sqrt(d2) - d->col_dist);
      if (pen) {
        double h = 0.5 * softplus(beta * (d->col_dist - sqrt(d2))) / beta;
        pen[q0 + i] += h;
        pen[q0 + j] += h;
      }
      if (!(d->flags & OR_COLLIDE) || !(d2 < dc2)) continue;
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
        OR_MARGIN(&mg[q0 + i], sp);
        OR_MARGIN(&mg[q0 + j], sp);
      }
      if ((d->flags & OR_APPROACH_ONLY) && !(sp > 0.0)) continue;
      for (int k = 0; k < 3; ++k) {
        dv[i][k] += sp * nrm[k];
        dv[j][k] -= sp * nrm[k];
      }
      marked[i] = marked[j] = 1;
    }
  }
  /* §III-B.4 downwash: the upper quads' airflow on a lower quad, from the
   * post-motion positions, applied as a velocity kick after the response */
  double adw[64];
  int dwhit[64];
  memset(adw, 0, sizeof(adw));
  memset(dwhit, 0, sizeof(dwhit));
  if (d->flags & OR_DOWNWASH) {
    const double dw_r2 = OR_CONST(d->dw_radius * d->dw_radius);
    for (int i = 0; i < n; ++i) {
      const double* si = S + (size_t)(q0 + i) * NS;
      if (si[IF] != 0.0) continue; /* resting on the floor */
      for (int j = 0; j < n; ++j) {
        if (j == i) continue;
        const double* sj = S + (size_t)(q0 + j) * NS;
        double hx = sj[IX] - si[IX], hy = sj[IX + 1] - si[IX + 1], dz = sj[IX + 2] - si[IX + 2];
        OR_MARGIN(&mg[q0 + i], sqrt(hx * hx + hy * hy) - d->dw_radius);
        OR_MARGIN(&mg[q0 + i], dz);
        OR_MARGIN(&mg[q0 + i], dz - d->dw_height);
        if (hx * hx + hy * hy < dw_r2 && dz > 0.0 && dz < d->dw_height) {
          adw[i] += -d->dw_k1 * (d->dw_k2 * dz + d->dw_b1);
          dwhit[i] = 1;
        }
      }
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
  for (int i = 0; i < n; ++i) {
    if (!dwhit[i]) continue;
    double* si = S + (size_t)(q0 + i) * NS;
    events[q0 + i] |= EV_DOWNWASH;
    double za[4] = {0, 0, 0, 0}, zw[4] = {0, 0, 0, 0};
    if (d->dw_noise_a > 0.0 || d->dw_noise_w > 0.0) {
      or_normal4(d->seed, d->quad_id_offset + (uint32_t)(q0 + i), t, STREAM_DOWNWASH, 0, za);
      or_normal4(d->seed, d->quad_id_offset + (uint32_t)(q0 + i), t, STREAM_DOWNWASH, 1, zw);
    }
    for (int k = 0; k < 3; ++k) {
      double a = (k == 2 ? adw[i] : 0.0) + d->dw_noise_a * za[k];
      si[IV + k] += d->dt * a;
      si[IW + k] += d->dt * d->dw_noise_w * zw[k];
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
                     &ev[q], &mg[q], NULL);
      }
      if ((d->flags & (OR_COLLIDE | OR_DOWNWASH)) && n > 1)
        env_pairs(d, state, q0, n, t, contacts, ev, mg, NULL, 0.0);
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


/* ======================================================================== */
/* Differentiation (reverse mode, double precision).                         */
/*                                                                          */
/* The loss is any function of the state after the rollout plus a weighted  */
/* sum of each quad's smoothed collision penalty                             */
/*   pen_i = sum over substeps, env-mates j of 1/2 softplus(beta(d_col -    */
/*           d_ij))/beta, with d_ij the centre distance after the motion of */
/*   the substep (before the pair response).                                */
/* Events (walls, floor, contacts, friction regime) take the derivative of  */
/* the branch that was taken; the resting flag carries no derivative.       */
/* ======================================================================== */

static void cross3(const double a[3], const double b[3], double o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* Reverse of one quad's substep up to the pair pass.  lam[27] holds dL/d
 * (state after the floor step) on entry and dL/d(state at the start of the
 * substep) on exit; guhat[4] accumulates dL/d(rotor-speed command) and
 * gp[6] dL/d(mass, ixx, iyy, izz, thrust_to_weight, motor_tau). */
static void quad_vjp(const or_desc* d, const double* p, const or_rec* r, double* lam,
                     double* guhat, double* gp) {
  const double dt = d->dt, g = d->gravity, m = p[PM];
  const double J[3] = {p[PJX], p[PJY], p[PJZ]};
  const double arm_d = OR_CONST(d->arm_length / sqrt(2.0));
  double lx[3], lv[3], lR[9], lw[3], lu[4], le[4];
  for (int k = 0; k < 3; ++k) {
    lx[k] = lam[IX + k];
    lv[k] = lam[IV + k];
    lw[k] = lam[IW + k];
  }
  for (int k = 0; k < 9; ++k) lR[k] = lam[IR + k];
  for (int k = 0; k < 4; ++k) {
    lu[k] = lam[IU + k];
    le[k] = lam[IE + k];
  }

  /* floor hit: z, v, omega set to constants; R levelled from its heading */
  if (r->hit) {
    lx[2] = 0.0;
    for (int k = 0; k < 3; ++k) lv[k] = lw[k] = 0.0;
    double gr[2] = {0.0, 0.0};
    if (!r->fallback) {
      /* column 0 = h = (hx, hy)/nh, column 1 = (-h_y, h_x) */
      double h[2] = {r->hx / r->nh, r->hy / r->nh};
      double gh[2] = {lR[0] + lR[4], lR[3] - lR[1]};
      double dd = gh[0] * h[0] + gh[1] * h[1];
      gr[0] = (gh[0] - dd * h[0]) / r->nh;
      gr[1] = (gh[1] - dd * h[1]) / r->nh;
      for (int k = 0; k < 9; ++k) lR[k] = 0.0;
      lR[0] = gr[0];
      lR[3] = gr[1];
    } else {
      /* column 1 = k = (kx, ky)/nk, column 0 = (k_y, -k_x) */
      double gk[2] = {0.0, 0.0};
      if (r->nk > 0.0) {
        double k[2] = {r->kx / r->nk, r->ky / r->nk};
        double gkk[2] = {lR[1] - lR[3], lR[4] + lR[0]};
        double dd = gkk[0] * k[0] + gkk[1] * k[1];
        gk[0] = (gkk[0] - dd * k[0]) / r->nk;
        gk[1] = (gkk[1] - dd * k[1]) / r->nk;
      }
      for (int k = 0; k < 9; ++k) lR[k] = 0.0;
      lR[1] = gk[0];
      lR[4] = gk[1];
    }
  }
  /* walls: decay once, then per-axis mirror and clamp */
  if (r->bounced)
    for (int k = 0; k < 3; ++k) lv[k] *= d->col_decay;
  for (int k = 0; k < 3; ++k) {
    if (r->flip[k]) lv[k] *= -d->wall_restitution;
    if (r->clamp[k]) lx[k] = 0.0;
  }

  double lT = 0.0, lF[3] = {0.0, 0.0, 0.0}, ltau[3] = {0.0, 0.0, 0.0};
  double lm = 0.0, lJ[3] = {0.0, 0.0, 0.0};
  double lP[9], lx0[3], lv0[3], lw0[3];
  const double* P = r->P;
  for (int k = 0; k < 3; ++k) lx0[k] = lx[k];
  if (!r->rest) {
    /* R = Gram-Schmidt(A): c2 = c0 x c1, c1 = b/|b|, b = A1 - (c0.A1) c0, c0 = A0/|A0| */
    double lc0[3] = {lR[0], lR[3], lR[6]}, lc1[3] = {lR[1], lR[4], lR[7]};
    double lc2[3] = {lR[2], lR[5], lR[8]}, tmp[3];
    cross3(r->c1, lc2, tmp);
    for (int k = 0; k < 3; ++k) lc0[k] += tmp[k];
    cross3(lc2, r->c0, tmp);
    for (int k = 0; k < 3; ++k) lc1[k] += tmp[k];
    double lb[3], dd = dot3(lc1, r->c1);
    for (int k = 0; k < 3; ++k) lb[k] = (lc1[k] - dd * r->c1[k]) / r->n1;
    double lA1[3], ldp = -dot3(lb, r->c0);
    for (int k = 0; k < 3; ++k) {
      lA1[k] = lb[k] + ldp * r->c0[k];
      lc0[k] += -r->dp * lb[k] + ldp * r->A1[k];
    }
    double lA0[3];
    dd = dot3(lc0, r->c0);
    for (int k = 0; k < 3; ++k) lA0[k] = (lc0[k] - dd * r->c0[k]) / r->n0;
    /* A0 = P0 + dt (P1 w1z - P2 w1y), A1 = P1 + dt (P2 w1x - P0 w1z) (columns) */
    const double* w1 = r->w1;
    double P0[3] = {P[0], P[3], P[6]}, P1[3] = {P[1], P[4], P[7]}, P2[3] = {P[2], P[5], P[8]};
    double lw1[3] = {lw[0] + dt * dot3(P2, lA1), lw[1] - dt * dot3(P2, lA0),
                     lw[2] + dt * (dot3(P1, lA0) - dot3(P0, lA1))};
    for (int rr = 0; rr < 3; ++rr) {
      lP[3 * rr + 0] = lA0[rr] - dt * w1[2] * lA1[rr];
      lP[3 * rr + 1] = lA1[rr] + dt * w1[2] * lA0[rr];
      lP[3 * rr + 2] = -dt * w1[1] * lA0[rr] + dt * w1[0] * lA1[rr];
    }
    /* w1 = w0 + dt wdot, wdot_k = (tau_k - (w0 x J w0)_k) / J_k */
    double lwd[3], lc[3], lJw[3];
    for (int k = 0; k < 3; ++k) {
      lw0[k] = lw1[k];
      lwd[k] = dt * lw1[k];
      ltau[k] = lwd[k] / J[k];
      lc[k] = -lwd[k] / J[k];
      lJ[k] += -lwd[k] * r->wdot[k] / J[k];
    }
    cross3(r->Jw, lc, tmp);
    for (int k = 0; k < 3; ++k) lw0[k] += tmp[k];
    cross3(lc, r->w0, lJw);
    for (int k = 0; k < 3; ++k) {
      lw0[k] += J[k] * lJw[k];
      lJ[k] += r->w0[k] * lJw[k];
    }
    /* x1 = x0 + dt v1, v1 = v0 + dt acc, acc = F/m - c_d v0/m - g e_z */
    double lacc[3];
    for (int k = 0; k < 3; ++k) {
      double lv1 = lv[k] + dt * lx[k];
      lacc[k] = dt * lv1;
      lv0[k] = lv1 - d->drag_coef / m * lacc[k];
      lF[k] = lacc[k] / m;
      lm += -(r->F[k] - d->drag_coef * r->v0[k]) * lacc[k] / (m * m);
    }
  } else {
    /* resting: R held, omega zeroed, v_z zeroed, x_z unchanged */
    for (int k = 0; k < 9; ++k) lP[k] = lR[k];
    for (int k = 0; k < 3; ++k) lw0[k] = 0.0;
    lv0[0] = lv0[1] = lv0[2] = 0.0;
    if (!r->guard) {
      double lv1[2] = {lv[0] + dt * lx[0], lv[1] + dt * lx[1]};
      double lfb[2] = {dt * lv1[0] / m, dt * lv1[1] / m};
      for (int k = 0; k < 2; ++k) {
        lv0[k] = lv1[k] * (1.0 - dt * d->drag_coef / m);
        lm += -dt * (r->fb[k] - d->drag_coef * r->v0[k]) * lv1[k] / (m * m);
      }
      double lmu = 0.0;
      if (r->statik) {
        if (r->mag > 0.0) {
          double Fh[2] = {r->F[0] / r->nf, r->F[1] / r->nf};
          double dd = lfb[0] * Fh[0] + lfb[1] * Fh[1];
          for (int k = 0; k < 2; ++k) lF[k] += lfb[k] - r->mu_n * (lfb[k] - dd * Fh[k]) / r->nf;
          lmu = -dd;
        }
      } else {
        double vh[2] = {r->v0[0] / r->nv, r->v0[1] / r->nv};
        for (int k = 0; k < 2; ++k) lF[k] += lfb[k];
        lmu = -(lfb[0] * vh[0] + lfb[1] * vh[1]);
        double lvh[2] = {-r->mu_n * lfb[0], -r->mu_n * lfb[1]};
        double dd = lvh[0] * vh[0] + lvh[1] * vh[1];
        for (int k = 0; k < 2; ++k) lv0[k] += (lvh[k] - dd * vh[k]) / r->nv;
      }
      /* mu_n = mu (m g - F_z) */
      lm += d->floor_mu * g * lmu;
      lF[2] += -d->floor_mu * lmu;
    }
  }
  /* F = T * (third column of R) */
  lT += lF[0] * P[2] + lF[1] * P[5] + lF[2] * P[8];
  lP[2] += r->T * lF[0];
  lP[5] += r->T * lF[1];
  lP[8] += r->T * lF[2];
  /* total thrust and torques from the rotor thrusts */
  static const double sx[4] = {-1, -1, 1, 1}, sy[4] = {-1, 1, 1, -1}, sz[4] = {1, -1, 1, -1};
  double lf[4], lfmax = 0.0;
  for (int i = 0; i < 4; ++i) {
    lf[i] = lT + arm_d * (sx[i] * ltau[0] + sy[i] * ltau[1]) + d->k_tau * sz[i] * ltau[2];
    lu[i] += 2.0 * r->f_max * r->u1[i] * lf[i];
    le[i] += lf[i];
    lfmax += r->u1[i] * r->u1[i] * lf[i];
  }
  /* motor noise and lag */
  double le0[4], lu0[4], lalag = 0.0;
  for (int i = 0; i < 4; ++i) {
    if (r->noise) {
      le0[i] = d->motor_noise_decay * le[i];
      lfmax += d->motor_noise_std * sqrt(1.0 - d->motor_noise_decay * d->motor_noise_decay) *
               r->z[i] * le[i];
    } else {
      le0[i] = le[i];
    }
    lu0[i] = (1.0 - r->alpha_lag) * lu[i];
    guhat[i] += r->alpha_lag * lu[i];
    lalag += (r->uhat[i] - r->u0[i]) * lu[i];
  }
  /* f_max = m g t2w / 4, alpha_lag = 1 - exp(-dt/tau) */
  lm += OR_CONST(0.25 * g * p[PT2W]) * lfmax;
  gp[PT2W] += OR_CONST(0.25 * m * g) * lfmax;
  gp[PTAU] += lalag * OR_CONST(-exp(-dt / p[PTAU]) * dt / (p[PTAU] * p[PTAU]));
  gp[PM] += lm;
  for (int k = 0; k < 3; ++k) gp[PJX + k] += lJ[k];

  for (int k = 0; k < 3; ++k) {
    lam[IX + k] = lx0[k];
    lam[IV + k] = lv0[k];
    lam[IW + k] = lw0[k];
  }
  for (int k = 0; k < 9; ++k) lam[IR + k] = lP[k];
  for (int k = 0; k < 4; ++k) {
    lam[IU + k] = lu0[k];
    lam[IE + k] = le0[k];
  }
  lam[IF] = 0.0;
}

/* Reverse of the pair response and of the penalty of one environment.
 * S1 holds the env's states after the floor step (before the response);
 * lam (state adjoints of the env's quads) enters as dL/d(state after the
 * response) and leaves as dL/d(state before the response). */
static void env_pairs_vjp(const or_desc* d, const double* S1, double* lam, int q0, int n,
                          const double* gpen, double beta) {
  double ldv[64][3];
  int marked[64];
  memset(marked, 0, sizeof(marked));
  const double dc2 = OR_CONST(d->col_dist * d->col_dist);
  const int collide = (d->flags & OR_COLLIDE) != 0;
  /* which quads responded (recomputed exactly as in the forward pass) */
  if (collide) {
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) {
        const double* si = S1 + (size_t)(q0 + i) * NS;
        const double* sj = S1 + (size_t)(q0 + j) * NS;
        double dx[3] = {si[IX] - sj[IX], si[IX + 1] - sj[IX + 1], si[IX + 2] - sj[IX + 2]};
        double d2 = dot3(dx, dx);
        if (!(d2 < dc2)) continue;
        double nrm[3];
        if (d2 < 1e-12) { nrm[0] = nrm[1] = 0.0; nrm[2] = 1.0; }
        else for (int k = 0; k < 3; ++k) nrm[k] = dx[k] / sqrt(d2);
        double sp = 0.0;
        for (int k = 0; k < 3; ++k) sp += (sj[IV + k] - si[IV + k]) * nrm[k];
        if ((d->flags & OR_APPROACH_ONLY) && !(sp > 0.0)) continue;
        marked[i] = marked[j] = 1;
      }
  }
  /* v2 = decay (v1 + dv + noise) for responding quads */
  for (int i = 0; i < n; ++i) {
    double* li = lam + (size_t)(q0 + i) * NS;
    for (int k = 0; k < 3; ++k) {
      ldv[i][k] = marked[i] ? d->col_decay * li[IV + k] : 0.0;
      if (marked[i]) li[IV + k] *= d->col_decay;
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      const double* si = S1 + (size_t)(q0 + i) * NS;
      const double* sj = S1 + (size_t)(q0 + j) * NS;
      double* li = lam + (size_t)(q0 + i) * NS;
      double* lj = lam + (size_t)(q0 + j) * NS;
      double dx[3] = {si[IX] - sj[IX], si[IX + 1] - sj[IX + 1], si[IX + 2] - sj[IX + 2]};
      double d2 = dot3(dx, dx), dd = sqrt(d2);
      /* penalty: d/dx_i of w_ij softplus(beta (dc - d))/beta = -w_ij sigmoid(.) n */
      if (gpen && dd > 0.0) {
        double coef = -0.5 * (gpen[q0 + i] + gpen[q0 + j]) * sigmoid(beta * (d->col_dist - dd));
        for (int k = 0; k < 3; ++k) {
          li[IX + k] += coef * dx[k] / dd;
          lj[IX + k] -= coef * dx[k] / dd;
        }
      }
      if (!collide || !(d2 < dc2)) continue;
      double nrm[3];
      int coincident = d2 < 1e-12;
      if (coincident) { nrm[0] = nrm[1] = 0.0; nrm[2] = 1.0; }
      else for (int k = 0; k < 3; ++k) nrm[k] = dx[k] / dd;
      double wv[3];
      for (int k = 0; k < 3; ++k) wv[k] = sj[IV + k] - si[IV + k];
      double sp = dot3(wv, nrm);
      if ((d->flags & OR_APPROACH_ONLY) && !(sp > 0.0)) continue;
      /* dv_i = sp n, dv_j = -sp n, sp = (v_j - v_i).n, n = (x_i - x_j)/d */
      double mu[3];
      for (int k = 0; k < 3; ++k) mu[k] = ldv[i][k] - ldv[j][k];
      double mn = dot3(mu, nrm);
      for (int k = 0; k < 3; ++k) {
        li[IV + k] += -mn * nrm[k];
        lj[IV + k] += mn * nrm[k];
      }
      if (!coincident) {
        double gn[3];
        for (int k = 0; k < 3; ++k) gn[k] = sp * mu[k] + mn * wv[k];
        double gnn = dot3(gn, nrm);
        for (int k = 0; k < 3; ++k) {
          double gx = (gn[k] - gnn * nrm[k]) / dd;
          li[IX + k] += gx;
          lj[IX + k] -= gx;
        }
      }
    }
}

static double dfhat_da(const or_desc* d, double a) {
  if (d->flags & OR_ACT_UNIT) return (a > 0.0 && a < 1.0) ? 1.0 : 0.0;
  return (a > -1.0 && a < 1.0) ? 0.5 : 0.0;
}

/*
 * Rollout of n_calls calls of n_sub substeps each from state[Q][27] (updated
 * in place), actions [n_calls][Q][4], first substep index t0.  pen
 * (optional, [Q]) accumulates each quad's penalty share (see above).
 */
int or_rollout(const or_desc* d, const double* params, double* state, const double* actions,
               int n_calls, int n_sub, uint64_t t0, double* pen, double beta) {
  if (check_desc(d) || !params || !state || !actions || n_calls < 0 || n_sub < 0) return -1;
  const int E = d->n_envs, Q = d->env_offsets[E];
  uint32_t* ev = (uint32_t*)calloc((size_t)Q + 1, sizeof(uint32_t));
  double* mg = (double*)malloc(((size_t)Q + 1) * sizeof(double));
  if (!ev || !mg) { free(ev); free(mg); return -1; }
  for (int c = 0; c < n_calls; ++c)
    for (int sub = 0; sub < n_sub; ++sub) {
      const uint64_t t = t0 + (uint64_t)c * n_sub + sub;
#pragma omp parallel for schedule(static)
      for (int e = 0; e < E; ++e) {
        const int q0 = d->env_offsets[e], n = d->env_offsets[e + 1] - q0;
        for (int i = 0; i < n; ++i) {
          const int q = q0 + i;
          quad_substep(d, params + (size_t)q * NP, state + (size_t)q * NS,
                       actions + ((size_t)c * Q + q) * 4, d->quad_id_offset + (uint32_t)q, t,
                       &ev[q], &mg[q], NULL);
        }
        if (n > 1 && ((d->flags & (OR_COLLIDE | OR_DOWNWASH)) || pen))
          env_pairs(d, state, q0, n, t, NULL, ev, mg, pen, beta);
      }
    }
  free(ev);
  free(mg);
  return 0;
}

/*
 * Reverse pass of or_rollout (same arguments; state0 is the state the
 * rollout started from and is not modified).  gstate [Q][27] enters as
 * dL/d(final state) and leaves as dL/d(initial state); gpen (optional, [Q])
 * is dL/d(pen); gact [n_calls][Q][4] receives dL/d(actions); gparams [Q][6]
 * receives dL/d(mass, ixx, iyy, izz, thrust_to_weight, motor_tau).  The
 * whole trajectory is kept in memory (no checkpointing).
 */
int or_rollout_vjp(const or_desc* d, const double* params, const double* state0,
                   const double* actions, int n_calls, int n_sub, uint64_t t0,
                   double* gstate, const double* gpen, double beta, double* gact,
                   double* gparams) {
  if (check_desc(d) || !params || !state0 || !actions || !gstate || !gact || !gparams ||
      n_calls < 0 || n_sub < 0 || (d->flags & OR_DOWNWASH))
    return -1;
  const int E = d->n_envs, Q = d->env_offsets[E];
  const size_t S = (size_t)n_calls * n_sub;
  const size_t QS = (size_t)Q * NS;
  double* traj = (double*)malloc((S + 1) * QS * sizeof(double));
  double* S1 = (double*)malloc(QS * sizeof(double));
  or_rec* rec = (or_rec*)malloc(((size_t)Q + 1) * sizeof(or_rec));
  double* gu = (double*)calloc((size_t)Q * 4 + 1, sizeof(double));
  uint32_t* ev = (uint32_t*)calloc((size_t)Q + 1, sizeof(uint32_t));
  double* mg = (double*)malloc(((size_t)Q + 1) * sizeof(double));
  if (!traj || !S1 || !rec || !gu || !ev || !mg) {
    free(traj); free(S1); free(rec); free(gu); free(ev); free(mg);
    return -1;
  }
  /* forward, keeping the state at the start of every substep */
  memcpy(traj, state0, QS * sizeof(double));
  for (size_t k = 0; k < S; ++k) {
    memcpy(traj + (k + 1) * QS, traj + k * QS, QS * sizeof(double));
    const int c = (int)(k / (size_t)n_sub);
#pragma omp parallel for schedule(static)
    for (int e = 0; e < E; ++e) {
      const int q0 = d->env_offsets[e], n = d->env_offsets[e + 1] - q0;
      double* st = traj + (k + 1) * QS;
      for (int i = 0; i < n; ++i) {
        const int q = q0 + i;
        quad_substep(d, params + (size_t)q * NP, st + (size_t)q * NS,
                     actions + ((size_t)c * Q + q) * 4, d->quad_id_offset + (uint32_t)q,
                     t0 + k, &ev[q], &mg[q], NULL);
      }
      if ((d->flags & (OR_COLLIDE | OR_DOWNWASH)) && n > 1)
        env_pairs(d, st, q0, n, t0 + k, NULL, ev, mg, NULL, 0.0);
    }
  }
  memset(gparams, 0, (size_t)Q * NP * sizeof(double));
  /* reverse sweep */
  for (size_t kk = S; kk-- > 0;) {
    const int c = (int)(kk / (size_t)n_sub);
    memcpy(S1, traj + kk * QS, QS * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int e = 0; e < E; ++e) {
      const int q0 = d->env_offsets[e], n = d->env_offsets[e + 1] - q0;
      for (int i = 0; i < n; ++i) {
        const int q = q0 + i;
        quad_substep(d, params + (size_t)q * NP, S1 + (size_t)q * NS,
                     actions + ((size_t)c * Q + q) * 4, d->quad_id_offset + (uint32_t)q,
                     t0 + kk, &ev[q], &mg[q], &rec[q]);
      }
      if (n > 1) env_pairs_vjp(d, S1, gstate, q0, n, gpen, beta);
      for (int i = 0; i < n; ++i) {
        const int q = q0 + i;
        quad_vjp(d, params + (size_t)q * NP, &rec[q], gstate + (size_t)q * NS,
                 gu + (size_t)q * 4, gparams + (size_t)q * NP);
      }
    }
    if (kk % (size_t)n_sub == 0) {
      /* first substep of call c: the held command's gradient becomes the action's */
      for (int q = 0; q < Q; ++q)
        for (int i = 0; i < 4; ++i) {
          const double a = actions[((size_t)c * Q + q) * 4 + i];
          const double uh = rec[q].uhat[i];
          gact[((size_t)c * Q + q) * 4 + i] =
              uh > 0.0 ? gu[(size_t)q * 4 + i] * 0.5 / uh * dfhat_da(d, a) : 0.0;
          gu[(size_t)q * 4 + i] = 0.0;
        }
    }
  }
  free(traj); free(S1); free(rec); free(gu); free(ev); free(mg);
  return 0;
}


/*
 * §III-C sensor noise, added in place to obs[Q][18+6K] as produced by
 * or_observe: uniform U(-sn_x, sn_x) on each component of x - goal,
 * U(-sn_v, sn_v) on v, N(0, sn_w^2) on omega, from Philox stream SENSOR at
 * substep index t (draw 0: position, 1: velocity, 2: body rate); the
 * uniforms come from the same (2k+1) 2^-24 map as the Gaussian draws.
 */
int or_observe_noise(const or_desc* d, double* obs, uint64_t t) {
  if (check_desc(d) || !obs) return -1;
  const int Q = d->env_offsets[d->n_envs], OD = 18 + 6 * d->k_neighbors;
  const uint32_t key[2] = {(uint32_t)d->seed, (uint32_t)(d->seed >> 32)};
  for (int q = 0; q < Q; ++q) {
    double* o = obs + (size_t)q * OD;
    const uint32_t gq = d->quad_id_offset + (uint32_t)q;
    for (int draw = 0; draw < 2; ++draw) {
      uint32_t ctr[4] = {gq, (uint32_t)t, (uint32_t)(t >> 32), (STREAM_SENSOR << 8) | draw};
      uint32_t r[4];
      or_philox4x32_10(ctr, key, r);
      const double a = draw == 0 ? d->sn_x : d->sn_v;
      for (int k = 0; k < 3; ++k) o[3 * draw + k] += a * (2.0 * or_uniform_from_u32(r[k]) - 1.0);
    }
    double z[4];
    or_normal4(d->seed, gq, t, STREAM_SENSOR, 2, z);
    for (int k = 0; k < 3; ++k) o[15 + k] += d->sn_w * z[k];
  }
  return 0;
}

/*
 * §III-E reward of one control call per quad.  w[15]: alpha_pos, _vel, _ori,
 * _spin, _act, _dact, _rot, _yaw, _floor_hit, _on_floor, _wall, _ceiling,
 * _quad, _prox, d_prox.  s0/s1: state before/after the call; ev: the call's
 * event bits (or_step); obs: the noise-free observation after the call
 * (its neighbour slots give the proximity term).
 *   r = a_pos |x - goal| + a_vel |v| + a_ori R22 + a_spin |w| + a_act |f|
 *     + a_dact |f - f_prev| + a_rot (tr R - 1)/2 + a_yaw R00
 *     + a_floor_hit [hit floor] + a_on_floor [resting] + a_wall [wall bounce]
 *     + a_ceiling [ceiling bounce] + a_quad [collision response]
 *     + a_prox sum_k max(1 - |x~_k| / d_prox, 0) over the min(K, n_e - 1) real
 *       neighbour slots (padded slots add nothing)
 * with f = f_max u_f^2 + eps the rotor thrusts after (f) and before (f_prev)
 * the call.
 */
int or_reward(const or_desc* d, const double* params, const double* s0, const double* s1,
              const uint32_t* ev, const double* goals, const double* obs, const double* w,
              double* reward) {
  if (check_desc(d) || !params || !s0 || !s1 || !ev || !goals || !obs || !w || !reward) return -1;
  const int K = d->k_neighbors, OD = 18 + 6 * K;
  for (int e = 0; e < d->n_envs; ++e) {
    const int q0 = d->env_offsets[e], n = d->env_offsets[e + 1] - q0;
    /* the real neighbour slots are the first min(K, n_e - 1); the rest are
       padding and add nothing, whatever their values */
    const int kr = n - 1 < K ? n - 1 : K;
    for (int q = q0; q < q0 + n; ++q) {
      const double* a = s0 + (size_t)q * NS;
      const double* b = s1 + (size_t)q * NS;
      const double f_max =
          0.25 * params[(size_t)q * NP + PM] * d->gravity * params[(size_t)q * NP + PT2W];
      double dx2 = 0, v2 = 0, w2 = 0, f2 = 0, df2 = 0;
      for (int k = 0; k < 3; ++k) {
        const double g = b[IX + k] - goals[(size_t)q * 3 + k];
        dx2 += g * g;
        v2 += b[IV + k] * b[IV + k];
        w2 += b[IW + k] * b[IW + k];
      }
      for (int i = 0; i < 4; ++i) {
        const double f1 = f_max * b[IU + i] * b[IU + i] + b[IE + i];
        const double f0 = f_max * a[IU + i] * a[IU + i] + a[IE + i];
        f2 += f1 * f1;
        df2 += (f1 - f0) * (f1 - f0);
      }
      double r = w[0] * sqrt(dx2) + w[1] * sqrt(v2) + w[2] * b[IR + 8] + w[3] * sqrt(w2) +
                 w[4] * sqrt(f2) + w[5] * sqrt(df2) +
                 w[6] * (b[IR + 0] + b[IR + 4] + b[IR + 8] - 1.0) / 2.0 + w[7] * b[IR + 0];
      r += w[8] * ((ev[q] & EV_FLOOR_HIT) ? 1.0 : 0.0) + w[9] * (b[IF] != 0.0 ? 1.0 : 0.0) +
           w[10] * ((ev[q] & EV_WALL) ? 1.0 : 0.0) + w[11] * ((ev[q] & EV_CEILING) ? 1.0 : 0.0) +
           w[12] * ((ev[q] & EV_PAIR_RESPONSE) ? 1.0 : 0.0);
      const double* o = obs + (size_t)q * OD;
      for (int k = 0; k < kr; ++k) {
        const double* x = o + 18 + 6 * k;
        const double dd = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
        const double h = 1.0 - dd / w[14];
        r += w[13] * (h > 0.0 ? h : 0.0);
      }
      reward[q] = r;
    }
  }
  return 0;
}

/*
 * The generator over a range of quads, for comparisons with another
 * implementation: words[n][4] = Philox4x32-10 of the counter (quad0 + i,
 * t_lo, t_hi, stream << 8 | draw) under key seed, and normals[n][4] (may be
 * NULL) the Box-Muller draws or_normal4 builds from them.
 */
int or_noise_batch(uint64_t seed, uint32_t stream, uint32_t draw, uint64_t t, uint32_t quad0,
                   int n, uint32_t* words, double* normals) {
  if (n < 0 || !words) return -1;
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (int i = 0; i < n; ++i) {
    const uint32_t q = quad0 + (uint32_t)i;
    const uint32_t ctr[4] = {q, (uint32_t)t, (uint32_t)(t >> 32), (stream << 8) | draw};
    or_philox4x32_10(ctr, key, words + 4 * (size_t)i);
    if (normals) or_normal4(seed, q, t, stream, draw, normals + 4 * (size_t)i);
  }
  return 0;
}

int or_flag_values(uint32_t out[8]) {
  out[0] = OR_ROOM; out[1] = OR_FLOOR; out[2] = OR_COLLIDE;
  out[3] = OR_MOTOR_NOISE; out[4] = OR_APPROACH_ONLY; out[5] = OR_ACT_UNIT;
  out[6] = OR_DOWNWASH; out[7] = OR_SENSOR_NOISE;
  return 0;
}
