// Host-side argument checks of the C ABI (no device code): the handle
// description, per-quad inputs, pointer alignment and buffer overlaps.
// Kept apart from the kernels so that they can be built and exercised on
// their own (the sanitizer test of the host checks builds this header with
// AddressSanitizer and UndefinedBehaviorSanitizer).
#pragma once
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <initializer_list>

#include "quadswarm.h"

namespace qs_host {

inline bool finite(float v) { return std::isfinite(v); }

inline bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

// Byte range [p, p + n) of a caller buffer; a null pointer takes no part.
struct Span {
  const void* p;
  size_t n;
};

inline bool overlap(const Span& a, const Span& b) {
  if (!a.p || !b.p || !a.n || !b.n) return false;
  const uintptr_t x = (uintptr_t)a.p, y = (uintptr_t)b.p;
  return x < y + b.n && y < x + a.n;
}

// Does an output buffer share a byte with another output or with an input?
inline bool outputs_overlap(std::initializer_list<Span> outs, std::initializer_list<Span> ins) {
  for (auto o = outs.begin(); o != outs.end(); ++o) {
    for (auto o2 = o + 1; o2 != outs.end(); ++o2)
      if (overlap(*o, *o2)) return true;
    for (const Span& i : ins)
      if (overlap(*o, i)) return true;
  }
  return false;
}

inline int check_desc(const qs_desc* d) {
  if (!d || !d->env_offsets) return QS_ERR_NULL;
  if (d->n_envs < 1) return QS_ERR_INVALID;
  if (d->env_offsets[0] != 0) return QS_ERR_ENV_SIZE;
  for (int e = 0; e < d->n_envs; ++e) {
    const long long n = (long long)d->env_offsets[e + 1] - d->env_offsets[e];
    if (n < 1 || n > QS_MAX_SWARM) return QS_ERR_ENV_SIZE;
  }
  // field offsets (field * Qp + q) stay within int32 and byte offsets of a
  // quad within a field within 32 bits
  if (d->env_offsets[d->n_envs] > QS_MAX_QUADS) return QS_ERR_INVALID;
  const float vals[] = {d->dt, d->gravity, d->arm_length, d->k_tau, d->drag_coef, d->floor_mu,
                        d->motor_noise_decay, d->motor_noise_std, d->room_min[0], d->room_min[1],
                        d->room_min[2], d->room_max[0], d->room_max[1], d->room_max[2],
                        d->wall_restitution, d->col_dist, d->col_decay, d->col_noise_v,
                        d->col_noise_w};
  for (float v : vals)
    if (!finite(v)) return QS_ERR_INVALID;
  if (!(d->dt > 0.f) || d->arm_length < 0.f || d->drag_coef < 0.f || d->floor_mu < 0.f)
    return QS_ERR_INVALID;
  if (d->motor_noise_decay < 0.f || d->motor_noise_decay >= 1.f || d->motor_noise_std < 0.f)
    return QS_ERR_INVALID;
  for (int k = 0; k < 3; ++k)
    if (!(d->room_min[k] < d->room_max[k])) return QS_ERR_INVALID;
  if (d->wall_restitution < 0.f || d->wall_restitution > 1.f || d->col_dist < 0.f ||
      d->col_noise_v < 0.f || d->col_noise_w < 0.f)
    return QS_ERR_INVALID;
  if (d->k_neighbors < 0 || d->k_neighbors >= QS_MAX_SWARM) return QS_ERR_INVALID;
  if (d->flags & ~255u) return QS_ERR_INVALID;
  const float dwv[] = {d->dw_k1, d->dw_k2, d->dw_b1, d->dw_radius, d->dw_height, d->dw_noise_a,
                       d->dw_noise_w};
  for (float v : dwv)
    if (!finite(v)) return QS_ERR_INVALID;
  if (d->dw_radius < 0.f || d->dw_height < 0.f || d->dw_noise_a < 0.f || d->dw_noise_w < 0.f)
    return QS_ERR_INVALID;
  if (!(d->sn_x >= 0.f && d->sn_v >= 0.f && d->sn_w >= 0.f && finite(d->sn_x) &&
        finite(d->sn_v) && finite(d->sn_w)))
    return QS_ERR_INVALID;
  return QS_OK;
}

// Per-quad inputs of qs_create: every parameter finite and > 0, every state
// value finite.
inline int check_quads(int Q, const qs_quad_params* h_params, const float* h_state0) {
  for (int q = 0; q < Q; ++q) {
    const qs_quad_params& p = h_params[q];
    const float v[] = {p.mass, p.ixx, p.iyy, p.izz, p.thrust_to_weight, p.motor_tau};
    for (float x : v)
      if (!finite(x) || !(x > 0.f)) return QS_ERR_INVALID;
  }
  for (size_t i = 0; i < (size_t)Q * QS_STATE_DIM; ++i)
    if (!finite(h_state0[i])) return QS_ERR_INVALID;
  return QS_OK;
}

}  // namespace qs_host
