/*
 * A C99 caller of the library with no Python and no PyTorch: device memory
 * from the HIP runtime's C API, one handle of 4 swarms of 8 quads packed
 * closely enough to collide, one qs_step_observe call of two substeps, the
 * state read back, qs_sync, qs_destroy.  It writes its constants, inputs and
 * outputs to the file named by argv[1] for the test to check against the
 * oracle:
 *   int32  magic 0x51534331, Q, E, K, n_substeps, obs_dim
 *   uint32 flags;  uint64 seed;  uint64 substep index after the call
 *   float  dt, gravity, arm_length, k_tau, drag_coef, floor_mu,
 *          motor_noise_decay, motor_noise_std, room_min[3], room_max[3],
 *          wall_restitution, col_dist, col_decay, col_noise_v, col_noise_w
 *   int32  env_offsets[E + 1]
 *   float  params[Q][6], state0[Q][27], actions[Q][4], goals[Q][3],
 *          state[Q][27], obs[Q][obs_dim]
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "quadswarm.h"

#define E 4
#define N 8
#define Q (E * N)
#define K 6
#define OD (18 + 6 * K)
#define NSUB 2

static int qs_fail(const char* what, int rc) {
  fprintf(stderr, "%s: %d (%s)\n", what, rc, qs_error_string(rc));
  return 1;
}

static int hip_fail(const char* what, hipError_t e) {
  fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
  return 1;
}

static int put(FILE* f, const void* p, size_t bytes) {
  return fwrite(p, 1, bytes, f) == bytes ? 0 : 1;
}

int main(int argc, char** argv) {
  if (argc != 2) {
    fprintf(stderr, "usage: abi_smoke OUTPUT\n");
    return 2;
  }
  int32_t offs[E + 1];
  for (int e = 0; e <= E; ++e) offs[e] = e * N;

  qs_desc d;
  memset(&d, 0, sizeof d);
  d.n_envs = E;
  d.env_offsets = offs;
  d.dt = 0.005f;
  d.gravity = 9.81f;
  d.arm_length = 0.046f;
  d.k_tau = 0.006f;
  d.drag_coef = 0.0f;
  d.floor_mu = 0.6f;
  d.motor_noise_decay = 0.9f;
  d.motor_noise_std = 0.05f;
  d.room_min[0] = -5.0f; d.room_min[1] = -5.0f; d.room_min[2] = 0.0f;
  d.room_max[0] = 5.0f; d.room_max[1] = 5.0f; d.room_max[2] = 10.0f;
  d.wall_restitution = 1.0f;
  d.col_dist = 0.1f;
  d.col_decay = 1.0f;
  d.k_neighbors = K;
  d.flags = QS_ROOM | QS_FLOOR | QS_COLLIDE | QS_MOTOR_NOISE | QS_APPROACH_ONLY;
  d.seed = 7u;
  d.dw_k1 = 2.0f; d.dw_k2 = -2.0f; d.dw_b1 = 1.0f; d.dw_radius = 0.1f; d.dw_height = 0.5f;

  static qs_quad_params par[Q];
  static float s0[Q * 27], act[Q * 4], goal[Q * 3], st[Q * 27], obs[Q * OD];
  memset(s0, 0, sizeof s0);
  for (int q = 0; q < Q; ++q) {
    const int e = q / N, i = q % N;
    par[q].mass = 0.028f * (1.0f + 0.02f * (float)(q % 5));
    par[q].ixx = 1.66e-5f;
    par[q].iyy = 1.7e-5f;
    par[q].izz = 2.93e-5f;
    par[q].thrust_to_weight = 2.0f;
    par[q].motor_tau = 0.015f;
    float* s = s0 + 27 * q;
    s[0] = (float)e - 1.5f + 0.07f * (float)(i % 4);   /* swarm-mates 7 cm apart */
    s[1] = 0.07f * (float)(i / 4);
    s[2] = 2.0f + 0.01f * (float)i;
    s[3] = 0.3f * sinf((float)q);
    s[4] = 0.2f * cosf((float)q);
    s[5] = 0.1f;
    s[6] = 1.0f; s[10] = 1.0f; s[14] = 1.0f;             /* R = I */
    s[15] = 0.1f * (float)(q % 3);
    s[16] = -0.05f * (float)(q % 3);
    s[17] = 0.02f;
    for (int k = 0; k < 4; ++k) s[18 + k] = sqrtf(0.5f);  /* hover rotor speed */
    for (int k = 0; k < 4; ++k) act[4 * q + k] = 0.3f * sinf((float)(q + k));
    goal[3 * q + 0] = 0.0f;
    goal[3 * q + 1] = 0.0f;
    goal[3 * q + 2] = 2.0f;
  }

  float *d_act = NULL, *d_goal = NULL, *d_obs = NULL, *d_st = NULL;
  hipError_t he;
  if ((he = hipMalloc((void**)&d_act, sizeof act)) != hipSuccess) return hip_fail("hipMalloc", he);
  if ((he = hipMalloc((void**)&d_goal, sizeof goal)) != hipSuccess) return hip_fail("hipMalloc", he);
  if ((he = hipMalloc((void**)&d_obs, sizeof obs)) != hipSuccess) return hip_fail("hipMalloc", he);
  if ((he = hipMalloc((void**)&d_st, sizeof st)) != hipSuccess) return hip_fail("hipMalloc", he);
  if ((he = hipMemcpy(d_act, act, sizeof act, hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail("hipMemcpy", he);
  if ((he = hipMemcpy(d_goal, goal, sizeof goal, hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail("hipMemcpy", he);

  qs_handle* h = NULL;
  int rc = qs_create(&d, par, s0, &h);
  if (rc != QS_OK) return qs_fail("qs_create", rc);
  int32_t nq = 0, ne = 0, od = 0;
  if ((rc = qs_sizes(h, &nq, &ne, &od)) != QS_OK) return qs_fail("qs_sizes", rc);
  if (nq != Q || ne != E || od != OD) {
    fprintf(stderr, "qs_sizes: %d %d %d\n", nq, ne, od);
    return 1;
  }
  if ((rc = qs_step_observe(h, d_act, NSUB, d_goal, d_obs, NULL)) != QS_OK)
    return qs_fail("qs_step_observe", rc);
  uint64_t t = 0;
  if ((rc = qs_get_state(h, d_st, &t, NULL)) != QS_OK) return qs_fail("qs_get_state", rc);
  if ((rc = qs_sync(h, NULL)) != QS_OK) return qs_fail("qs_sync", rc);
  if ((he = hipMemcpy(st, d_st, sizeof st, hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail("hipMemcpy", he);
  if ((he = hipMemcpy(obs, d_obs, sizeof obs, hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail("hipMemcpy", he);
  if ((rc = qs_destroy(h)) != QS_OK) return qs_fail("qs_destroy", rc);
  hipFree(d_act);
  hipFree(d_goal);
  hipFree(d_obs);
  hipFree(d_st);

  FILE* f = fopen(argv[1], "wb");
  if (!f) {
    perror(argv[1]);
    return 1;
  }
  const int32_t head[6] = {0x51534331, Q, E, K, NSUB, OD};
  const float cf[19] = {d.dt, d.gravity, d.arm_length, d.k_tau, d.drag_coef, d.floor_mu,
                        d.motor_noise_decay, d.motor_noise_std,
                        d.room_min[0], d.room_min[1], d.room_min[2],
                        d.room_max[0], d.room_max[1], d.room_max[2],
                        d.wall_restitution, d.col_dist, d.col_decay, d.col_noise_v, d.col_noise_w};
  float pf[Q * 6];
  for (int q = 0; q < Q; ++q) {
    pf[6 * q + 0] = par[q].mass;
    pf[6 * q + 1] = par[q].ixx;
    pf[6 * q + 2] = par[q].iyy;
    pf[6 * q + 3] = par[q].izz;
    pf[6 * q + 4] = par[q].thrust_to_weight;
    pf[6 * q + 5] = par[q].motor_tau;
  }
  const uint64_t seed = d.seed;
  int bad = put(f, head, sizeof head) | put(f, &d.flags, sizeof d.flags) | put(f, &seed, sizeof seed) |
            put(f, &t, sizeof t) | put(f, cf, sizeof cf) | put(f, offs, sizeof offs) |
            put(f, pf, sizeof pf) | put(f, s0, sizeof s0) | put(f, act, sizeof act) |
            put(f, goal, sizeof goal) | put(f, st, sizeof st) | put(f, obs, sizeof obs);
  if (fclose(f) != 0 || bad) {
    fprintf(stderr, "writing %s failed\n", argv[1]);
    return 1;
  }
  printf("abi_smoke ok: %d quads, substep index %llu\n", Q, (unsigned long long)t);
  return 0;
}
