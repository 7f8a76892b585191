// The C ABI's host-side argument checks (paper_2306_09537_amd/csrc/qs_checks.h),
// built with AddressSanitizer and UndefinedBehaviorSanitizer and run on the
// CPU: descriptions with every kind of defect, per-quad inputs bad in their
// last element, alignment and overlap rules.  Exit status 0 and no
// sanitizer report on success.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "qs_checks.h"

static int failures = 0;

static void expect(int got, int want, const char* what) {
  if (got != want) {
    std::printf("FAIL %s: got %d, want %d\n", what, got, want);
    ++failures;
  }
}

static qs_desc base_desc(int32_t n_envs, const int32_t* offs) {
  qs_desc d;
  std::memset(&d, 0, sizeof d);
  d.n_envs = n_envs;
  d.env_offsets = offs;
  d.dt = 0.005f;
  d.gravity = 9.81f;
  d.arm_length = 0.046f;
  d.k_tau = 0.006f;
  d.floor_mu = 0.6f;
  d.motor_noise_decay = 0.9f;
  d.motor_noise_std = 0.05f;
  d.room_min[0] = d.room_min[1] = -5.f;
  d.room_max[0] = d.room_max[1] = 5.f;
  d.room_max[2] = 10.f;
  d.wall_restitution = 1.f;
  d.col_dist = 0.1f;
  d.col_decay = 1.f;
  d.k_neighbors = 6;
  d.flags = 31u;
  d.seed = 7u;
  return d;
}

int main() {
  using namespace qs_host;
  const int E = 4096, N = 8, Q = E * N;
  // exact-size heap arrays, so that a read past an end is reported
  std::vector<int32_t> offs(E + 1);
  for (int e = 0; e <= E; ++e) offs[e] = e * N;
  std::vector<qs_quad_params> par(Q, qs_quad_params{0.028f, 1.66e-5f, 1.66e-5f, 2.93e-5f, 2.f,
                                                    0.015f});
  std::vector<float> st((size_t)Q * QS_STATE_DIM, 0.f);
  qs_desc d = base_desc(E, offs.data());
  expect(check_desc(&d), QS_OK, "valid description");
  expect(check_quads(Q, par.data(), st.data()), QS_OK, "valid quads");
  expect(check_desc(nullptr), QS_ERR_NULL, "null description");
  qs_desc bad = d;
  bad.env_offsets = nullptr;
  expect(check_desc(&bad), QS_ERR_NULL, "null offsets");
  bad = d;
  bad.n_envs = 0;
  expect(check_desc(&bad), QS_ERR_INVALID, "no environments");
  offs[7] = offs[6];
  expect(check_desc(&d), QS_ERR_ENV_SIZE, "empty swarm");
  offs[7] = offs[6] + 65;
  expect(check_desc(&d), QS_ERR_ENV_SIZE, "swarm of 65");
  offs[7] = 7 * N;
  offs[E] = offs[E - 1];
  expect(check_desc(&d), QS_ERR_ENV_SIZE, "empty last swarm");
  offs[E] = E * N;
  offs[0] = 1;
  expect(check_desc(&d), QS_ERR_ENV_SIZE, "offsets not from 0");
  offs[0] = 0;
  {
    // more quads than a handle takes
    const int64_t n_max = (int64_t)QS_MAX_QUADS;
    const int32_t big_e = (int32_t)(n_max / 64 + 2);
    std::vector<int32_t> big(big_e + 1);
    for (int32_t e = 0; e <= big_e; ++e) big[e] = e * 64;
    qs_desc dd = base_desc(big_e, big.data());
    expect(check_desc(&dd), QS_ERR_INVALID, "too many quads");
  }
  struct FloatField {
    float qs_desc::*m;
    float v;
    const char* what;
  };
  const FloatField fields[] = {
      {&qs_desc::dt, NAN, "dt nan"},
      {&qs_desc::dt, 0.f, "dt 0"},
      {&qs_desc::drag_coef, -1.f, "negative drag"},
      {&qs_desc::motor_noise_decay, 1.f, "decay 1"},
      {&qs_desc::wall_restitution, 1.5f, "restitution 1.5"},
      {&qs_desc::col_dist, -0.1f, "negative contact distance"},
      {&qs_desc::dw_radius, -1.f, "negative downwash radius"},
      {&qs_desc::sn_w, INFINITY, "sensor noise inf"},
  };
  for (const FloatField& f : fields) {
    bad = d;
    bad.*(f.m) = f.v;
    expect(check_desc(&bad), QS_ERR_INVALID, f.what);
  }
  bad = d;
  bad.room_min[0] = 5.f;
  expect(check_desc(&bad), QS_ERR_INVALID, "empty room");
  bad = d;
  bad.k_neighbors = 64;
  expect(check_desc(&bad), QS_ERR_INVALID, "K 64");
  bad = d;
  bad.flags = 256u;
  expect(check_desc(&bad), QS_ERR_INVALID, "unknown flag");
  // per-quad inputs, bad in the very last element
  par[Q - 1].motor_tau = 0.f;
  expect(check_quads(Q, par.data(), st.data()), QS_ERR_INVALID, "last tau 0");
  par[Q - 1].motor_tau = NAN;
  expect(check_quads(Q, par.data(), st.data()), QS_ERR_INVALID, "last tau nan");
  par[Q - 1].motor_tau = 0.015f;
  st.back() = INFINITY;
  expect(check_quads(Q, par.data(), st.data()), QS_ERR_INVALID, "last state inf");
  st.back() = 0.f;
  expect(check_quads(0, par.data(), st.data()), QS_OK, "no quads");
  // alignment and overlaps
  alignas(16) float buf[64];
  expect(aligned(buf, 16), 1, "aligned");
  expect(aligned(buf + 1, 16), 0, "misaligned");
  expect(overlap({buf, 16}, {buf + 4, 16}), 0, "adjacent ranges");
  expect(overlap({buf, 17}, {buf + 4, 16}), 1, "one shared byte");
  expect(overlap({nullptr, 16}, {buf, 16}), 0, "null range");
  expect(overlap({buf, 0}, {buf, 16}), 0, "empty range");
  expect(outputs_overlap({{buf, 64}, {buf + 16, 64}}, {{buf + 40, 16}}), 0, "disjoint outputs");
  expect(outputs_overlap({{buf, 64}, {buf + 8, 64}}, {}), 1, "outputs overlap");
  expect(outputs_overlap({{buf, 64}}, {{buf + 15, 8}}), 1, "output over an input");
  std::printf("%s (%d failures)\n", failures ? "FAILED" : "ok", failures);
  return failures ? 1 : 0;
}
