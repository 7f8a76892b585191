/*
 * The FP64 oracle (test infrastructure) built with AddressSanitizer and
 * UndefinedBehaviorSanitizer and run on the CPU over every entry point:
 * swarms of 1, 2, 5, 8, 32 and 64 quads, K from 0 to 63 (more slots than
 * swarm-mates), every physics flag, packed and coincident quads, quads on
 * the floor and against the walls, with every buffer allocated at its exact
 * size.  Exit status 0 and no sanitizer report on success.
 */
#include "../../oracle/quadswarm_oracle.c"

#include <stdio.h>

static double rnd(uint64_t* s) {
  *s = *s * 6364136223846793005ull + 1442695040888963407ull;
  return (double)(*s >> 11) * (1.0 / 9007199254740992.0);
}

static int run_case(int k, uint32_t flags, uint64_t seed) {
  static const int sizes[] = {1, 2, 5, 8, 32, 64, 3};
  const int E = (int)(sizeof sizes / sizeof sizes[0]);
  int32_t* offs = (int32_t*)malloc((E + 1) * sizeof(int32_t));
  offs[0] = 0;
  for (int e = 0; e < E; ++e) offs[e + 1] = offs[e] + sizes[e];
  const int Q = offs[E], OD = 18 + 6 * k, T = 3;
  or_desc d;
  memset(&d, 0, sizeof d);
  d.n_envs = E;
  d.env_offsets = offs;
  d.dt = 0.005; d.gravity = 9.81; d.arm_length = 0.046; d.k_tau = 0.006;
  d.drag_coef = 0.02; d.floor_mu = 0.6; d.motor_noise_decay = 0.9; d.motor_noise_std = 0.05;
  d.room_min[0] = d.room_min[1] = -5.0; d.room_min[2] = 0.0;
  d.room_max[0] = d.room_max[1] = 5.0; d.room_max[2] = 10.0;
  d.wall_restitution = 0.8; d.col_dist = 0.1; d.col_decay = 0.9;
  d.col_noise_v = 0.01; d.col_noise_w = 0.02; d.k_neighbors = k; d.flags = flags;
  d.seed = seed; d.quad_id_offset = 17;
  d.dw_k1 = 2.0; d.dw_k2 = -2.0; d.dw_b1 = 1.0; d.dw_radius = 0.1; d.dw_height = 0.5;
  d.sn_x = 5e-3; d.sn_v = 1e-2; d.sn_w = 1.75e-4;
  double* par = (double*)malloc((size_t)Q * 6 * sizeof(double));
  double* s = (double*)malloc((size_t)Q * 27 * sizeof(double));
  double* s0 = (double*)malloc((size_t)Q * 27 * sizeof(double));
  double* act = (double*)malloc((size_t)T * Q * 4 * sizeof(double));
  double* goal = (double*)malloc((size_t)Q * 3 * sizeof(double));
  uint64_t r = seed;
  for (int q = 0; q < Q; ++q) {
    const double p[6] = {0.028, 1.66e-5, 1.66e-5, 2.93e-5, 2.0, 0.015};
    for (int i = 0; i < 6; ++i) par[q * 6 + i] = p[i] * (0.8 + 0.4 * rnd(&r));
    double* x = s + (size_t)q * 27;
    memset(x, 0, 27 * sizeof(double));
    for (int i = 0; i < 3; ++i) x[i] = (i == 2 ? 2.0 : 0.0) + 0.15 * rnd(&r);  /* packed */
    if (q % 7 == 0) { x[2] = 0.0; x[26] = 1.0; }                            /* on the floor */
    if (q % 11 == 0) { x[0] = 4.999; x[3] = 2.0; }                          /* at a wall */
    if (q % 13 == 1 && q > 0) memcpy(x, s + (size_t)(q - 1) * 27, 3 * sizeof(double));
    for (int i = 3; i < 6; ++i) x[i] = rnd(&r) - 0.5;
    x[6] = x[10] = x[14] = 1.0;
    for (int i = 15; i < 18; ++i) x[i] = rnd(&r) - 0.5;
    for (int i = 18; i < 22; ++i) x[i] = 0.7;
    for (int i = 0; i < 3; ++i) goal[q * 3 + i] = rnd(&r);
  }
  for (size_t i = 0; i < (size_t)T * Q * 4; ++i) act[i] = 2.0 * rnd(&r) - 1.0;
  memcpy(s0, s, (size_t)Q * 27 * sizeof(double));
  uint64_t* con = (uint64_t*)malloc((size_t)Q * sizeof(uint64_t));
  uint32_t* ev = (uint32_t*)malloc((size_t)Q * sizeof(uint32_t));
  double* mg = (double*)malloc((size_t)Q * sizeof(double));
  int bad = 0;
  bad |= or_step(&d, par, s, act, 3, 5, con, ev, mg);
  double* obs = (double*)malloc((size_t)Q * OD * sizeof(double));
  int32_t* nbr = (int32_t*)malloc((size_t)Q * (k > 0 ? k : 1) * sizeof(int32_t));
  bad |= or_observe(&d, s, goal, obs, k > 0 ? nbr : NULL);
  double* rew = (double*)malloc((size_t)Q * sizeof(double));
  const double w[15] = {-1, -0.1, 0.2, -0.05, -0.05, -0.1, 0.1, 0.1, -5, -1, -2, -2, -5, -1, 0.5};
  bad |= or_reward(&d, par, s0, s, ev, goal, obs, w, rew);
  bad |= or_observe_noise(&d, obs, 8);
  double* pen = (double*)calloc((size_t)Q, sizeof(double));
  memcpy(s, s0, (size_t)Q * 27 * sizeof(double));
  bad |= or_rollout(&d, par, s, act, T, 2, 0, pen, 100.0);
  if (!(flags & OR_DOWNWASH)) {
    double* g = (double*)malloc((size_t)Q * 27 * sizeof(double));
    for (size_t i = 0; i < (size_t)Q * 27; ++i) g[i] = rnd(&r) - 0.5;
    double* ga = (double*)malloc((size_t)T * Q * 4 * sizeof(double));
    double* gp = (double*)calloc((size_t)Q * 6, sizeof(double));
    bad |= or_rollout_vjp(&d, par, s0, act, T, 2, 0, g, pen, 100.0, ga, gp);
    free(g); free(ga); free(gp);
  }
  uint32_t* words = (uint32_t*)malloc((size_t)Q * 4 * sizeof(uint32_t));
  double* normals = (double*)malloc((size_t)Q * 4 * sizeof(double));
  bad |= or_noise_batch(seed, 2, 1, 1ull << 33, 0xffffff00u, Q, words, normals);
  free(words); free(normals); free(pen); free(rew); free(nbr); free(obs);
  free(con); free(ev); free(mg); free(act); free(goal); free(s0); free(s); free(par); free(offs);
  return bad;
}

int main(void) {
  const uint32_t all = OR_ROOM | OR_FLOOR | OR_COLLIDE | OR_MOTOR_NOISE | OR_APPROACH_ONLY;
  int bad = 0;
  bad |= run_case(0, all, 1);
  bad |= run_case(6, all, 2);
  bad |= run_case(63, all | OR_SENSOR_NOISE, 3);
  bad |= run_case(3, all | OR_DOWNWASH | OR_ACT_UNIT, 4);
  bad |= run_case(6, 0, 5);
  printf("%s\n", bad ? "FAILED: an entry point refused valid arguments" : "ok");
  return bad ? 1 : 0;
}
