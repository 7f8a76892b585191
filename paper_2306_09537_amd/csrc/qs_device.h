// Device-side building blocks of the quadrotor-swarm step (gfx950, wave64).
//
// One lane owns one quad.  Its state lives in VGPRs for the whole call; a
// workgroup owns whole environments (never split), so the in-env pair pass
// and the nearest-neighbour search read swarm-mates' positions and
// velocities from LDS after a workgroup barrier (swarms of at most 8 take
// the neighbour candidates' positions from their lanes instead, and larger
// swarms take the neighbour keys from the last pair pass's screen).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace qs {

enum : uint32_t {
  F_ROOM = 1u, F_FLOOR = 2u, F_COLLIDE = 4u, F_NOISE = 8u, F_APPROACH = 16u, F_ACT_UNIT = 32u,
  F_DOWNWASH = 64u, F_SENSOR = 128u
};
enum : int { NSTATE = 27, NPARAM = 8 };
// clang vector types, for the non-temporal store builtin
typedef float v2f __attribute__((ext_vector_type(2)));
typedef float v4f __attribute__((ext_vector_type(4)));
// SoA field index of the private state: x3 v3 R9 (row-major) w3 u4 eps4 floor
enum : int { S_X = 0, S_V = 3, S_R = 6, S_W = 15, S_U = 18, S_E = 22, S_F = 26 };
// SoA field index of the per-quad parameters (the forward reads the first six)
enum : int { P_M = 0, P_JX = 1, P_JY = 2, P_JZ = 3, P_FMAX = 4, P_ALAG = 5, P_T2W = 6, P_TAU = 7 };
// noise streams: fourth Philox counter word = stream << 8 | draw
enum : uint32_t {
  STREAM_MOTOR = 0, STREAM_WALL = 1, STREAM_PAIR = 2, STREAM_DOWNWASH = 3, STREAM_SENSOR = 4
};
// events of a call, for the reward's interaction terms
enum : uint32_t { EVF_FLOOR_HIT = 1u, EVF_WALL = 2u, EVF_CEILING = 4u, EVF_QUAD = 8u };
enum : int { ERRBIT_STATE = 1, ERRBIT_ACTION = 2, ERRBIT_PARAM = 4 };

struct Consts {
  float dt, g, arm_d, k_tau, drag, mu;
  float a_nd, ns_scale;  // motor noise: eps <- a_nd eps + ns_scale f_max z
  float rmin0, rmin1, rmin2, rmax0, rmax1, rmax2, e_wall;
  float dcol2, dcol, col_decay, col_nv, col_nw;
  uint32_t flags;
  uint32_t key0, key1;
  int32_t K;
  int32_t obs_dim;
  // downwash: -k1 (k2 dz + b1) e_z within |dxy|^2 < dw_r2, 0 < dz < dw_h
  float dw_k1, dw_k2, dw_b1, dw_r2, dw_h, dw_na, dw_nw;
  // observation sensor noise: uniform half-widths (x - goal, v), Gaussian std (omega)
  float sn_x, sn_v, sn_w;
  // reward weights: pos, vel, ori, spin, act, dact, rot, yaw, floor_hit,
  // on_floor, wall, ceiling, quad, prox, and the proximity distance
  float rw[15];
};

struct Ptrs {
  float* st;                    // [27][Qp] private SoA state
  const float* par;             // [8][Qp] m, jx, jy, jz, f_max, alpha_lag, t2w, tau
  const uint32_t* sw;           // [Qp] (env start within the block << 8) | n_e
  const int2* blk;              // [nblk] (first quad, quad count)
  unsigned long long* contacts; // [Qp] or nullptr
  int* err;                     // sticky error bits
  int Qp;                       // padded quad count (SoA field stride)
  int Q;                        // quad count
  const int4* items;            // uneven sizes: (slot size, first env entry, swarms, -)
  const int2* item_envs;        // uneven sizes: (first quad, size) per swarm of an item
};

// Philox4x32-10, Salmon et al. SC'11: ten rounds of two 32x32->64 products
// with a Weyl-sequence key schedule.
__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2,
                                              uint32_t& c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t pa = (uint64_t)0xD2511F53u * c0;
    const uint64_t pb = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)pb;
    c3 = (uint32_t)pa;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// Uniform (2 (r >> 9) + 1) 2^-24 in (0,1): exact in float32.
__device__ __forceinline__ float u01(uint32_t r) {
  return (float)(((r >> 9) << 1) | 1u) * 5.9604644775390625e-8f;
}

// Four N(0,1) draws by Box-Muller for (quad, substep, stream, draw):
// radius sqrt(-2 ln u0) = sqrt(-2 ln2 log2 u0), angle 2 pi u1.  The hardware
// log2, sqrt and the sine/cosine of an angle given in revolutions are used
// directly: on every u = (2m + 1) 2^-24 their errors are about one ulp
// (sin/cos 1.3e-7 absolute, log2 1.2e-7 relative, near u = 1 included),
// giving draws within 6e-7 of the exact ones, at a fraction of the library
// functions' instruction count.
__device__ __forceinline__ void normal4(const Consts& c, uint32_t q, uint64_t t,
                                        uint32_t stream, uint32_t draw, float z[4]) {
  uint32_t r0 = q, r1 = (uint32_t)t, r2 = (uint32_t)(t >> 32), r3 = (stream << 8) | draw;
  philox4x32_10(r0, r1, r2, r3, c.key0, c.key1);
  constexpr float m2ln2 = -1.3862943611198906f;  // -2 ln 2
  float rad = __builtin_amdgcn_sqrtf(m2ln2 * __builtin_amdgcn_logf(u01(r0)));
  float a = u01(r1);
  z[0] = rad * __builtin_amdgcn_cosf(a);
  z[1] = rad * __builtin_amdgcn_sinf(a);
  rad = __builtin_amdgcn_sqrtf(m2ln2 * __builtin_amdgcn_logf(u01(r2)));
  a = u01(r3);
  z[2] = rad * __builtin_amdgcn_cosf(a);
  z[3] = rad * __builtin_amdgcn_sinf(a);
}

// Per-quad registers.  xo/inc are the substep's start position and
// displacement: the pair pass measures separations as
// (xo_i - xo_j) + (inc_i - inc_j), which keeps ~1e-9 m accuracy for
// centimetre gaps between quads several metres from the origin, where the
// difference of the rounded end positions would be off by ~1e-6 m.
struct Quad {
  float x[3], v[3], R[9], w[3], u[4], e[4];
  float fl;
  float xo[3], inc[3];
  uint32_t ev;  // EVF_* bits of the current call
};

struct QuadPar {
  float m, inv_m, jx, jy, jz, ijx, ijy, ijz, f_max, a_lag, a_ns;
};

// Median of three unsigned words (one v_med3_u32).
__device__ __forceinline__ uint32_t umed3(uint32_t a, uint32_t b, uint32_t c) {
  return max(min(a, b), min(max(a, b), c));
}

__device__ __forceinline__ float clampf(float a, float lo, float hi) {
  return fminf(fmaxf(a, lo), hi);
}

// §III-A.1: rotor-speed command from the normalised thrust action.
__device__ __forceinline__ float rotor_cmd(float a, bool unit) {
  // both maps, then a select: a branch on the flag would end the scheduling
  // region (and wait for the action load) once per rotor
  const float fu = clampf(a, 0.0f, 1.0f);
  const float fs = 0.5f * (clampf(a, -1.0f, 1.0f) + 1.0f);
  return sqrtf(unit ? fu : fs);
}

// Intermediates of one substep kept for the reverse sweep (adjoint).
struct Rec {
  float z[4], u0[4], u1[4], P[9], w0[3], v0[3], T, F[3];
  float wdot[3], w1[3], A1[3], i0, c0[3], dp, i1, c1[3];  // i0, i1: inverse column norms
  float mu_n, fb[2], nv, nf, mag;
  float hx, hy, nh, kx, ky, nk;
  bool rest, statik, guard, bounced, hit, fallback;
  bool clamp[3], flip[3];
};

// Where the motor-noise draws of a substep come from: generated (Z_DRAW),
// generated and also written to zio[4] (Z_EXPORT), or read from zio[4]
// (Z_IMPORT: the draws an earlier Z_EXPORT run saved for this quad and
// substep).
enum ZMode { Z_DRAW, Z_EXPORT, Z_IMPORT };

// Thrust and body torques of one substep: the output of the motor part.
struct Drive {
  float T, tx, ty, tz;
};

// §III-A.1 motor lag, §III-A.2 motor noise (AR(1)) and per-rotor thrust,
// §III-A X mix: updates the rotor state (u, eps) and returns the thrust and
// torques.  Depends on the rotor state, the command and the substep's draws
// only (not on position, velocity or attitude).  z: the draws (zeros
// without motor noise).
template <ZMode ZM = Z_DRAW>
__device__ __forceinline__ Drive motor_step(const Consts& c, const QuadPar& p, float u[4],
                                            float e[4], const float uhat[4], uint32_t q,
                                            uint64_t t, float z[4], float* zio = nullptr) {
#pragma unroll
  for (int i = 0; i < 4; ++i) u[i] = fmaf(p.a_lag, uhat[i] - u[i], u[i]);
  if (c.flags & F_NOISE) {
    if constexpr (ZM == Z_IMPORT) {
#pragma unroll
      for (int i = 0; i < 4; ++i) z[i] = zio[i];
    } else {
      normal4(c, q, t, STREAM_MOTOR, 0, z);
    }
    if constexpr (ZM == Z_EXPORT) {
#pragma unroll
      for (int i = 0; i < 4; ++i) zio[i] = z[i];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) e[i] = fmaf(c.a_nd, e[i], p.a_ns * z[i]);
  }
  // X layout FR, BR, BL, FL
  float f[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) f[i] = fmaf(p.f_max * u[i], u[i], e[i]);
  Drive d;
  d.T = (f[0] + f[1]) + (f[2] + f[3]);
  d.tx = c.arm_d * ((f[2] + f[3]) - (f[0] + f[1]));
  d.ty = c.arm_d * ((f[1] + f[2]) - (f[0] + f[3]));
  d.tz = c.k_tau * ((f[0] + f[2]) - (f[1] + f[3]));
  return d;
}

// The rest of a substep from its thrust and torques: floor-rest or
// free-flight dynamics with semi-implicit Euler and Gram-Schmidt, walls and
// floor (not the rotor state).  REC: also record the intermediates the
// adjoint needs into *r (the rotor fields are the caller's).
template <bool REC = false>
__device__ __forceinline__ void body_step(const Consts& c, const QuadPar& p, Quad& s,
                                          const Drive& d, uint32_t q, uint64_t t,
                                          Rec* r = nullptr) {
  if constexpr (REC) {
#pragma unroll
    for (int k = 0; k < 9; ++k) r->P[k] = s.R[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      r->w0[k] = s.w[k];
      r->v0[k] = s.v[k];
      r->clamp[k] = false;
      r->flip[k] = false;
    }
    r->statik = r->guard = r->bounced = r->hit = r->fallback = false;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) s.xo[k] = s.x[k];
  const float T = d.T, tx = d.tx, ty = d.ty, tz = d.tz;
  // world-frame thrust = T * third column of R
  const float Fx = T * s.R[2], Fy = T * s.R[5], Fz = T * s.R[8];

  const bool rest = (c.flags & F_FLOOR) && s.fl != 0.0f && Fz <= p.m * c.g;
  if constexpr (REC) {
    r->T = T;
    r->F[0] = Fx;
    r->F[1] = Fy;
    r->F[2] = Fz;
    r->rest = rest;
  }
  // Free flight is computed for every lane (one scheduling region); the
  // rare resting lane then redoes the substep from the saved start values.
  const float v0r[2] = {s.v[0], s.v[1]};
  float R0r[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) R0r[k] = s.R[k];
  const float fl0 = s.fl;
  {
    s.fl = 0.0f;
    const float dm = c.drag * p.inv_m;
    const float ax = fmaf(Fx, p.inv_m, -dm * s.v[0]);
    const float ay = fmaf(Fy, p.inv_m, -dm * s.v[1]);
    const float az = fmaf(Fz, p.inv_m, -dm * s.v[2]) - c.g;
    // Euler's equation with the start-of-substep body rate
    const float Lx = p.jx * s.w[0], Ly = p.jy * s.w[1], Lz = p.jz * s.w[2];
    const float cx = s.w[1] * Lz - s.w[2] * Ly;
    const float cy = s.w[2] * Lx - s.w[0] * Lz;
    const float cz = s.w[0] * Ly - s.w[1] * Lx;
    const float wdx = (tx - cx) * p.ijx, wdy = (ty - cy) * p.ijy, wdz = (tz - cz) * p.ijz;
    // semi-implicit Euler
    s.v[0] = fmaf(c.dt, ax, s.v[0]);
    s.v[1] = fmaf(c.dt, ay, s.v[1]);
    s.v[2] = fmaf(c.dt, az, s.v[2]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      s.inc[k] = c.dt * s.v[k];
      s.x[k] = fmaf(c.dt, s.v[k], s.x[k]);
    }
    s.w[0] = fmaf(c.dt, wdx, s.w[0]);
    s.w[1] = fmaf(c.dt, wdy, s.w[1]);
    s.w[2] = fmaf(c.dt, wdz, s.w[2]);
    if constexpr (REC) {
      r->wdot[0] = wdx;
      r->wdot[1] = wdy;
      r->wdot[2] = wdz;
#pragma unroll
      for (int k = 0; k < 3; ++k) r->w1[k] = s.w[k];
    }
    // R <- R + dt R [w]x (body rate), then Gram-Schmidt on the columns
    const float hx = c.dt * s.w[0], hy = c.dt * s.w[1], hz = c.dt * s.w[2];
    float c0[3], c1[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float r0 = s.R[3 * k], r1 = s.R[3 * k + 1], r2 = s.R[3 * k + 2];
      c0[k] = r0 + (r1 * hz - r2 * hy);
      c1[k] = r1 + (r2 * hx - r0 * hz);
    }
    if constexpr (REC) {
#pragma unroll
      for (int k = 0; k < 3; ++k) r->A1[k] = c1[k];
    }
    const float i0 = rsqrtf(c0[0] * c0[0] + c0[1] * c0[1] + c0[2] * c0[2]);
#pragma unroll
    for (int k = 0; k < 3; ++k) c0[k] *= i0;
    const float dp = c0[0] * c1[0] + c0[1] * c1[1] + c0[2] * c1[2];
#pragma unroll
    for (int k = 0; k < 3; ++k) c1[k] = fmaf(-dp, c0[k], c1[k]);
    const float i1 = rsqrtf(c1[0] * c1[0] + c1[1] * c1[1] + c1[2] * c1[2]);
#pragma unroll
    for (int k = 0; k < 3; ++k) c1[k] *= i1;
    if constexpr (REC) {
      r->i0 = i0;
      r->i1 = i1;
      r->dp = dp;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        r->c0[k] = c0[k];
        r->c1[k] = c1[k];
      }
    }
    s.R[0] = c0[0]; s.R[3] = c0[1]; s.R[6] = c0[2];
    s.R[1] = c1[0]; s.R[4] = c1[1]; s.R[7] = c1[2];
    s.R[2] = c0[1] * c1[2] - c0[2] * c1[1];
    s.R[5] = c0[2] * c1[0] - c0[0] * c1[2];
    s.R[8] = c0[0] * c1[1] - c0[1] * c1[0];
  }
  if (rest) {
    // §III-B.3 resting on the floor: friction in xy, no vertical motion,
    // no rotation; static friction when still, kinetic when sliding.
    s.fl = fl0;
#pragma unroll
    for (int k = 0; k < 9; ++k) s.R[k] = R0r[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) s.x[k] = s.xo[k];  // the substep's start position
    const float mu_n = c.mu * (p.m * c.g - Fz);
    float fbx, fby;
    // the record's fields are written once after the branch: stores to
    // different fields on the two sides get merged into one store through a
    // selected address, which keeps the record out of registers
    float rnf = 0.0f, rmag = 0.0f, rnv = 0.0f;
    const float vx0 = v0r[0], vy0 = v0r[1];
    const bool still = vx0 == 0.0f && vy0 == 0.0f;
    if (still) {
      const float nf = sqrtf(Fx * Fx + Fy * Fy);
      const float mag = fmaxf(nf - mu_n, 0.0f);
      const float sc = nf > 0.0f ? mag / nf : 0.0f;
      fbx = sc * Fx;
      fby = sc * Fy;
      rnf = nf;
      rmag = nf > 0.0f ? mag : 0.0f;
    } else {
      const float nv = sqrtf(vx0 * vx0 + vy0 * vy0);
      const float iv = mu_n / nv;
      fbx = Fx - iv * vx0;
      fby = Fy - iv * vy0;
      rnv = nv;
    }
    if constexpr (REC) {
      r->statik = still;
      r->nf = rnf;
      r->mag = rmag;
      r->nv = rnv;
      r->mu_n = mu_n;
      r->fb[0] = fbx;
      r->fb[1] = fby;
    }
    s.v[0] = fmaf(c.dt, (fbx - c.drag * vx0) * p.inv_m, vx0);
    s.v[1] = fmaf(c.dt, (fby - c.drag * vy0) * p.inv_m, vy0);
    s.v[2] = 0.0f;
    if (s.v[0] * vx0 + s.v[1] * vy0 < 0.0f) {
      s.v[0] = 0.0f;
      s.v[1] = 0.0f;
      if constexpr (REC) r->guard = true;
    }
    s.inc[0] = c.dt * s.v[0];
    s.inc[1] = c.dt * s.v[1];
    s.inc[2] = 0.0f;
    s.x[0] = fmaf(c.dt, s.v[0], s.x[0]);
    s.x[1] = fmaf(c.dt, s.v[1], s.x[1]);
    s.w[0] = s.w[1] = s.w[2] = 0.0f;
  }

  // §III-B.2 walls and ceiling: the quad meets its mirror image
  if (c.flags & F_ROOM) {
    bool b = false;
    const float lo[2] = {c.rmin0, c.rmin1};
    const float hi[3] = {c.rmax0, c.rmax1, c.rmax2};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      // selects, not branches: hits are rare and the rest of the substep
      // stays one scheduling region
      if (k < 2) {
        const bool out = s.x[k] < lo[k];
        const bool flip = out && s.v[k] < 0.0f;
        s.x[k] = out ? lo[k] : s.x[k];
        s.inc[k] = out ? s.x[k] - s.xo[k] : s.inc[k];
        s.v[k] = flip ? -c.e_wall * s.v[k] : s.v[k];
        b = b | flip;
        s.ev |= flip ? (uint32_t)EVF_WALL : 0u;
        if constexpr (REC) {
          r->clamp[k] = r->clamp[k] | out;
          r->flip[k] = r->flip[k] | flip;
        }
      }
      const bool out = s.x[k] > hi[k];
      const bool flip = out && s.v[k] > 0.0f;
      s.x[k] = out ? hi[k] : s.x[k];
      s.inc[k] = out ? s.x[k] - s.xo[k] : s.inc[k];
      s.v[k] = flip ? -c.e_wall * s.v[k] : s.v[k];
      b = b | flip;
      s.ev |= flip ? (uint32_t)(k == 2 ? EVF_CEILING : EVF_WALL) : 0u;
      if constexpr (REC) {
        r->clamp[k] = r->clamp[k] | out;
        r->flip[k] = r->flip[k] | flip;
      }
    }
    if constexpr (REC) r->bounced = b;
    if (b) {
      float zv[4] = {0.f, 0.f, 0.f, 0.f}, zw[4] = {0.f, 0.f, 0.f, 0.f};
      if (c.col_nv > 0.0f || c.col_nw > 0.0f) {
        normal4(c, q, t, STREAM_WALL, 0, zv);
        normal4(c, q, t, STREAM_WALL, 1, zw);
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        s.v[k] = c.col_decay * fmaf(c.col_nv, zv[k], s.v[k]);
        s.w[k] = fmaf(c.col_nw, zw[k], s.w[k]);
      }
    }
  }

  // §III-B.3 floor hit: stop, level the body keeping its heading, rest
  if ((c.flags & F_FLOOR) && s.x[2] < c.rmin2) {
    s.ev |= EVF_FLOOR_HIT;
    s.x[2] = c.rmin2;
    s.inc[2] = s.x[2] - s.xo[2];
    s.v[0] = s.v[1] = s.v[2] = 0.0f;
    s.w[0] = s.w[1] = s.w[2] = 0.0f;
    s.fl = 1.0f;
    const float hx = s.R[0], hy = s.R[3];
    const float nh = sqrtf(hx * hx + hy * hy);
    if constexpr (REC) {
      r->hit = true;
      r->hx = hx;
      r->hy = hy;
      r->nh = nh;
      r->fallback = !(nh >= 1e-6f);
      r->kx = s.R[1];
      r->ky = s.R[4];
      r->nk = sqrtf(s.R[1] * s.R[1] + s.R[4] * s.R[4]);
    }
    float ax, ay;  // unit heading of body x in the floor plane
    if (nh >= 1e-6f) {
      ax = hx / nh;
      ay = hy / nh;
    } else {
      const float kx = s.R[1], ky = s.R[4];
      const float nk = sqrtf(kx * kx + ky * ky);
      const float bx = nk > 0.0f ? kx / nk : 0.0f, by = nk > 0.0f ? ky / nk : 1.0f;
      ax = by;   // body x = body y x e_z
      ay = -bx;
    }
    s.R[0] = ax;  s.R[1] = -ay; s.R[2] = 0.0f;
    s.R[3] = ay;  s.R[4] = ax;  s.R[5] = 0.0f;
    s.R[6] = 0.0f; s.R[7] = 0.0f; s.R[8] = 1.0f;
  }
}

// One substep of one quad up to (not including) the in-env pair pass: the
// motor part, then the body part.  REC: also record the intermediates the
// adjoint needs into *r.
template <bool REC = false, ZMode ZM = Z_DRAW>
__device__ __forceinline__ void quad_substep(const Consts& c, const QuadPar& p, Quad& s,
                                             const float uhat[4], uint32_t q, uint64_t t,
                                             Rec* r = nullptr, float* zio = nullptr) {
  if constexpr (REC) {
#pragma unroll
    for (int i = 0; i < 4; ++i) r->u0[i] = s.u[i];
  }
  float z[4] = {0.f, 0.f, 0.f, 0.f};
  const Drive d = motor_step<ZM>(c, p, s.u, s.e, uhat, q, t, z, zio);
  if constexpr (REC) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      r->z[i] = z[i];
      r->u1[i] = s.u[i];
    }
  }
  body_step<REC>(c, p, s, d, q, t, r);
}

// Geometry of the pair (i, j) for the in-env pass, from partner j's start
// position pj[0..2] and displacement pj[3..5] (rows 0-5 of the tile; rows
// 6-8 hold the velocities).  Returns true when the pair is in contact; then
// pair_normal gives the unit normal from j to i and sp = (v_j - v_i).n.
// Shared by the forward pass and the adjoint's recomputation so both take
// identical decisions.
// Separation from partner pj after the substep's motion and the contact
// test d^2 < d_col^2.  For the quad itself d = 0 exactly and the test is
// true: callers clear their own bit once after the partner loop instead of
// testing every partner's index.
__device__ __forceinline__ bool pair_geom_v(const Consts& c, const float pj[6], const Quad& s,
                                            float& dx, float& dy, float& dz, float& d2) {
  dx = (s.xo[0] - pj[0]) + (s.inc[0] - pj[3]);
  dy = (s.xo[1] - pj[1]) + (s.inc[1] - pj[4]);
  dz = (s.xo[2] - pj[2]) + (s.inc[2] - pj[5]);
  d2 = dx * dx + dy * dy + dz * dz;
  return d2 < c.dcol2;
}

template <int BS>
__device__ __forceinline__ void pair_normal(const float (*tile)[BS], const Quad& s, int j, int jj,
                                            int me, float dx, float dy, float dz, float d2,
                                            float n[3], float& sp) {
  if (d2 < 1e-12f) {
    n[0] = 0.f;
    n[1] = 0.f;
    n[2] = me < jj ? 1.f : -1.f;
  } else {
    const float id = rsqrtf(d2);
    n[0] = dx * id;
    n[1] = dy * id;
    n[2] = dz * id;
  }
  sp = (tile[6][j] - s.v[0]) * n[0] + (tile[7][j] - s.v[1]) * n[1] + (tile[8][j] - s.v[2]) * n[2];
}

// Smoothed collision penalty: softplus(x) = max(x, 0) + ln(1 + e^-|x|) and
// its derivative, the logistic sigmoid, from the hardware base-2 exponential,
// logarithm and reciprocal (about 1 ulp each); ln(1 + e) for e < 1e-4 from
// its series, where 1 + e would round away most of e.
__device__ __forceinline__ float softplus_hw(float x) {
  const float e = __builtin_amdgcn_exp2f(-fabsf(x) * 1.4426950408889634f);
  const float l = e < 1e-4f ? e * fmaf(-0.5f, e, 1.0f)
                            : 0.6931471805599453f * __builtin_amdgcn_logf(1.0f + e);
  return fmaxf(x, 0.f) + l;
}
__device__ __forceinline__ float sigmoid_hw(float x) {
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-x * 1.4426950408889634f));
}

// Workgroup barrier with the LDS fences around it, for kernels whose
// wavefronts run different code (each reaching it the same number of times).
__device__ __forceinline__ void wg_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// LDS written by some lanes of a wavefront, then read by others of the same
// wavefront.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The value of lane (lane xor D) for 1 <= D <= 7: a swarm of at most 8
// quads in an aligned group of 8 lanes takes a swarm-mate's register by a
// data-parallel-primitive move, with no LDS.  quad_perm covers D = 1, 2, 3
// within groups of 4 lanes; row_half_mirror (lane i of each group of 8 from
// lane 7 - i, i.e. xor 7) composed with one of them covers D = 4 .. 7.
// Every source lane lies inside the destination's own group of 8.  Callers
// run it with every lane of the wavefront active (uniform control flow);
// `none` is only the value a move would leave where no source lane were
// available.
template <int D>
__device__ __forceinline__ float lane_xor8(float v, float none) {
  static_assert(D >= 1 && D <= 7, "partners within a group of 8 lanes");
  constexpr int QP[4] = {0xE4, 0xB1, 0x4E, 0x1B};  // quad_perm: identity, xor 1, xor 2, xor 3
  constexpr int HALF_MIRROR = 0x141;
  const int o = __float_as_int(none);
  int x = __float_as_int(v);
  if constexpr (D >= 4) x = __builtin_amdgcn_update_dpp(o, x, HALF_MIRROR, 0xF, 0xF, false);
  constexpr int r = D >= 4 ? (D ^ 7) : D;
  if constexpr (r != 0) x = __builtin_amdgcn_update_dpp(o, x, QP[r], 0xF, 0xF, false);
  return __int_as_float(x);
}

// compile-time booleans for generic lambdas
struct TrueT { static constexpr bool value = true; };
struct FalseT { static constexpr bool value = false; };

// Contact mask of a swarm slot of N quads: 32 bits suffice up to 32 (one
// select and one OR per partner instead of two of each).
template <int N>
using PairMask = typename std::conditional<(N > 0 && N <= 32), uint32_t,
                                           unsigned long long>::type;

// Calls f(jj, pj) for every swarm-mate jj of the lane's swarm (itself
// included), in increasing jj, pj[0..5] being its start position and
// displacement from rows 0-5 of the tile and pj[6] row XR (XR < 0: none).
// For a compile-time swarm size the reads go out a chunk of eight partners
// at a time, ahead of the per-pair branches, so they overlap instead of
// waiting one by one.
template <int BS, int N, int XR = -1, typename T, typename F>
__device__ __forceinline__ void for_partners(T tile, int ls, int n, F&& f) {
  if constexpr (N > 0) {
    // chunks of eight partners, four in swarms of 16 and more (32-quad
    // swarms: 168 -> 120 VGPRs in the step, four wavefronts per SIMD
    // instead of three)
    constexpr int CH = N < 8 ? N : (N >= 16 ? 4 : 8);
    auto chunk = [&](int j0) {
      float pj[CH][7];
#pragma unroll
      for (int u = 0; u < CH; ++u) {
#pragma unroll
        for (int r = 0; r < 6; ++r) pj[u][r] = tile[r][ls + j0 + u];
        pj[u][6] = XR >= 0 ? tile[XR < 0 ? 0 : XR][ls + j0 + u] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < CH; ++u) f(j0 + u, pj[u]);
    };
    if constexpr (N >= 16) {
      // large swarms: a run-time loop over the chunks keeps the registers
      // of an eight-partner body
#pragma unroll 1
      for (int j0 = 0; j0 < N; j0 += CH) chunk(j0);
    } else {
#pragma unroll
      for (int j0 = 0; j0 < N; j0 += CH) chunk(j0);
    }
  } else {
    for (int jj = 0; jj < n; ++jj) {
      const int j = ls + jj;
      const float pj[7] = {tile[0][j], tile[1][j], tile[2][j], tile[3][j], tile[4][j],
                           tile[5][j], XR >= 0 ? tile[XR < 0 ? 0 : XR][j] : 0.f};
      f(jj, pj);
    }
  }
}

// Rows of the exchange tile that hold each quad's post-motion position
// (x after walls and floor) and its squared norm, written beside rows 0-8 by
// kernels whose in-swarm pass screens partners on it (pair_pass with CO).
constexpr int XROW = 9;
constexpr int XSQ = XROW + 3;
constexpr int TILE_ROWS_CO = XROW + 4;
// Positions (every coordinate, metres) within which the screen of swarms of
// 16 and 32 uses the expanded squared distance; the room of the workloads
// spans [-5, 5] x [-5, 5] x [0, 10].
constexpr float SCREEN_BOX = 10.0f;

// Swarm slots whose screen reads the squared norms (row XSQ).
template <int N>
constexpr bool kScreenSq = N >= 16 && N <= 32;

// The screen rows of one lane: x and, SQ, |x|^2 (one expression, so every
// kernel writes the same value), or, for a padding lane, a far-away
// sentinel.
template <bool SQ, typename T>
__device__ __forceinline__ void put_screen_rows(T tile, int tid, const float x[3]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) tile[XROW + k][tid] = x[k];
  if constexpr (SQ) tile[XSQ][tid] = fmaf(x[2], x[2], fmaf(x[1], x[1], x[0] * x[0]));
}
template <bool SQ, typename T>
__device__ __forceinline__ void put_screen_pad(T tile, int tid) {
#pragma unroll
  for (int k = 0; k < 3; ++k) tile[XROW + k][tid] = 1e30f;
  if constexpr (SQ) tile[XSQ][tid] = INFINITY;
}

// Calls f(jj, pj) for every swarm-mate jj (itself included), in increasing
// jj, with pj[0..2] its post-motion position from rows XROW..XROW+2 (and,
// NR = 4, pj[3] its squared norm from row XSQ), read a chunk of partners
// ahead of their arithmetic (chunk sizes as for_partners).
template <int BS, int N, int NR = 3, typename T, typename F>
__device__ __forceinline__ void for_partner_pos(T tile, int ls, int n, F&& f) {
  if constexpr (N > 0) {
    constexpr int CH = N < 8 ? N : (N >= 16 ? 4 : 8);
    auto chunk = [&](int j0) {
      float pj[CH][NR];
#pragma unroll
      for (int u = 0; u < CH; ++u) {
#pragma unroll
        for (int r = 0; r < NR; ++r) pj[u][r] = tile[XROW + r][ls + j0 + u];
      }
#pragma unroll
      for (int u = 0; u < CH; ++u) f(j0 + u, pj[u]);
    };
    if constexpr (N >= 16) {
#pragma unroll 1
      for (int j0 = 0; j0 < N; j0 += CH) chunk(j0);
    } else {
#pragma unroll
      for (int j0 = 0; j0 < N; j0 += CH) chunk(j0);
    }
  } else {
    for (int jj = 0; jj < n; ++jj) {
      const int j = ls + jj;
      float pj[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) pj[r] = tile[XROW + r][j];
      f(jj, pj);
    }
  }
}

// Neighbour keys (§III-C, the K nearest by (d^2, index)).  A candidate at
// squared distance d2 becomes one 32-bit key: the bits of d2 (non-negative,
// so they order as the values) with the low six replaced by the partner's
// index jj within the swarm (swarms hold at most 64).  key[0..L-1] is a
// sorted list of the L smallest keys so far; a candidate enters with one min
// and L - 1 medians, all independent of each other:
// new[0] = min(old[0], x), new[k] = med3(old[k-1], x, old[k]).  The quad
// itself and non-finite distances never enter.  The list does not depend on
// the order in which candidates arrive.
constexpr uint32_t KEY_EMPTY = 0xffffffffu;
template <int L>
__device__ __forceinline__ void knn_insert(uint32_t key[L], int jj, int me, float d2) {
  const uint32_t kx = (jj != me && d2 < INFINITY)
                          ? ((__float_as_uint(d2) & ~63u) | (uint32_t)jj) : KEY_EMPTY;
  uint32_t nk[L];
  nk[0] = min(key[0], kx);
#pragma unroll
  for (int k = 1; k < L; ++k) nk[k] = umed3(key[k - 1], kx, key[k]);
#pragma unroll
  for (int k = 0; k < L; ++k) key[k] = nk[k];
}

// Squared distance from the lane's position to partner position pj[0..2]
// (one expression for the partner screen and the neighbour search, so both
// round identically).
__device__ __forceinline__ float sq_dist(const float pj[3], const float x[3]) {
  const float dx = pj[0] - x[0], dy = pj[1] - x[1], dz = pj[2] - x[2];
  return dx * dx + dy * dy + dz * dz;
}

// In-swarm pass of one live lane after the tile (start positions,
// displacements, velocities) is written and the workgroup synchronised:
// §III-B.1 contact detection and Jacobi velocity exchange (every response
// from the pre-response velocities), the smoothed collision penalty (PEN),
// and §III-B.4 downwash from the swarm-mates above, applied as a velocity
// kick after the response.  N > 0 unrolls over the swarm slot; padding
// partners hold far-away sentinels.  Returns the contact mask.
// CO (no penalty, tile rows XROW.. written): without downwash, partners are
// first screened on the post-motion positions with a contact distance
// widened by 1 mm, and the exact test runs for the survivors only.  The
// screen never drops a pair the exact test would mark: for positions within
// 1000 m of the origin, x differs from (start + displacement) by at most an
// ulp of 1000 (6.1e-5 m) per quad and axis, well inside the 1 mm; a lane
// further out tests every partner exactly.  So the contact set, and every
// result, is the same as without the screen.  L > 0 (swarms other than 8,
// with the screen): the screen's squared distances also enter the
// neighbour key list key[0..L-1] (knn_insert); the pass changes only
// velocities and body rates, so they are the distances of the post-pass
// positions.
template <int BS, int N, bool PEN, bool CO = false, int L = 0>
__device__ __forceinline__ unsigned long long pair_pass(const Consts& c, const float (*tile)[BS],
                                                        Quad& s, int ls, int n, int me,
                                                        uint32_t q, unsigned long long t,
                                                        float& pacc, float beta,
                                                        uint32_t* key = nullptr) {
  static_assert(L == 0 || (CO && !PEN && N != 8), "keys from the plain screen only");
  const bool collide = (c.flags & F_COLLIDE) != 0;
  const bool dw = (c.flags & F_DOWNWASH) != 0 && s.fl == 0.0f;
  using M = PairMask<N>;
  M cm = 0;
  float dv[3] = {0.f, 0.f, 0.f};
  float adw = 0.f;
  bool hit = false, dwhit = false;
  const float hb = PEN ? 0.5f / beta : 0.f;  // each quad of a pair carries half
  // Every partner's geometry, branch-free (contacts are rare; a branch per
  // partner would end the scheduling region and serialise the partners'
  // arithmetic): the contact set, the penalty and, when it is on (a uniform
  // choice between two loops), downwash.
  const float dw_r2 = c.dw_r2, dw_h = c.dw_h, dw_k1 = c.dw_k1, dw_k2 = c.dw_k2, dw_b1 = c.dw_b1;
  // In passes over every partner in index order (in_order), swarms of 16
  // and 32 shift the contact bits in (the sign bit of d^2 - d_col^2, for
  // finite d^2 exactly the comparison's outcome, by one funnel shift) and
  // bit-reverse them once after the pass.
  constexpr bool ACC = N >= 16 && N <= 32;
  uint32_t acc = 0u;
  auto pair = [&](int jj, const float* pj, auto with_dw, auto in_order) {
    float dx, dy, dz, d2;
    const bool con = pair_geom_v(c, pj, s, dx, dy, dz, d2);
    if constexpr (PEN) {
      const float sp = hb * softplus_hw(beta * (c.dcol - __builtin_amdgcn_sqrtf(d2)));
      pacc = jj != me ? pacc + sp : pacc;
    }
    if constexpr (ACC && decltype(in_order)::value)
      acc = __builtin_amdgcn_alignbit(acc, __float_as_uint(d2 - c.dcol2), 31u);
    else
      cm |= con ? (M)1 << jj : (M)0;
    if constexpr (decltype(with_dw)::value) {
      // swarm-mate j above (z_j - z_i = -dz) and overlapping in xy (never
      // the quad itself: dz = 0 there)
      const bool dwc = dw & (dx * dx + dy * dy < dw_r2) & (-dz > 0.f) & (-dz < dw_h);
      adw = dwc ? adw - dw_k1 * (dw_k2 * -dz + dw_b1) : adw;
      dwhit = dwhit | dwc;
    }
  };
  if (c.flags & F_DOWNWASH) {
    for_partners<BS, N>(tile, ls, n,
                        [&](int jj, const float* pj) { pair(jj, pj, TrueT{}, TrueT{}); });
    if constexpr (ACC) cm = (M)(__builtin_bitreverse32(acc) >> (32 - N));
  } else if constexpr (CO && !PEN) {
    const float dw = c.dcol + 1e-3f, thr = dw * dw;
    M cand = 0;
    bool in_box = true;  // the expanded screen's domain (swarms of 16 and 32)
    if constexpr (N == 8) {
      // Each unordered pair screened once: the lane screens partner
      // me + o (mod N) for o = 1 .. N/2 and takes from lane me - o its
      // screen of the same pair (the squared distance is symmetric bit for
      // bit); for o = N/2 both lanes of the pair screen it.  Bit b of rot
      // stands for partner me + b (mod N).  A swarm never straddles a
      // wavefront.  Half the screens for a lane permute per pair: in swarms
      // of 8 the forward rollout at 1024 x 8 went from 0.242 to 0.225 ms;
      // in swarms of 32 the per-lane tile reads and permutes cost more than
      // the broadcast reads of the plain screen (ten substeps at
      // 32768 x 32: 49.1 -> 47.4 G quad-steps/s), so larger swarms keep it.
      const int base = ((ls + me) & 63) - me;  // the swarm's first lane
      uint32_t rot = 0u;
      // offsets four at a time (their reads ahead of their arithmetic); a
      // run-time loop over the groups keeps the registers of one group
#pragma unroll 1
      for (int o0 = 1; o0 <= N / 2; o0 += 4) {
        float pj[4][3];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int j = ls + ((me + o0 + u) & (N - 1));
#pragma unroll
          for (int r = 0; r < 3; ++r) pj[u][r] = tile[XROW + r][j];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int o = o0 + u;
          const float dx = pj[u][0] - s.x[0], dy = pj[u][1] - s.x[1], dz = pj[u][2] - s.x[2];
          // the sign of d^2 - thr as one FMA chain (as in larger swarms);
          // dx -> -dx leaves it unchanged, so both lanes of a pair agree
          const uint32_t h = __float_as_uint(fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, -thr)))) >> 31;
          rot |= h << o;
          if (o < N / 2) {
            const int src = base + ((me - o) & (N - 1));
            const uint32_t g = (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)h) & 1u;
            rot |= g << (N - o);
          }
        }
      }
      constexpr uint32_t full = (1u << N) - 1u;
      rot &= full;
      cand = (M)(me == 0 ? rot : ((rot << me) | (rot >> (N - me))) & full);
    } else {
      if constexpr (N >= 16 && N <= 32) {
        // Partners arrive in index order, so the mask is accumulated as
        // acc = 2 acc + bit and bit-reversed once: partner jj's bit lands at
        // position N - 1 - jj, then at jj.
        uint32_t acc = 0u;
        if constexpr (L > 0) {
          for_partner_pos<BS, N>(tile, ls, n, [&](int jj, const float* pj) {
            const float d2 = sq_dist(pj, s.x);
            acc = acc + acc + (d2 < thr ? 1u : 0u);
            knn_insert<L>(key, jj, me, d2);
          });
        } else {
          // Without keys the bit is the sign of
          //   e = |b|^2 + (|a|^2 - thr_x) - 2 a.b  (= |a - b|^2 - thr_x),
          // three FMAs and an add per partner (|b|^2 from row XSQ, the rest
          // once per lane), shifted in by one funnel shift
          // ((acc << 1) | (e >> 31), v_alignbit).  Rounding: |e - (|a - b|^2
          // - thr_x)| <= 7 u ((|a| + |b|)^2 + thr_x), u = 2^-24.  For a lane
          // with every |a_k| <= SCREEN_BOX and a partner in contact,
          // |a| + |b| <= reach = 2 sqrt(3) SCREEN_BOX + d_col + 1 mm, so the
          // widening thr_x - d_col^2 = 3 err, err = 7 u (reach^2 + d_col^2)
          // (+1 %), exceeds the rounding three times over and no contact is
          // dropped; a lane outside the box tests every partner exactly.
          // An extra survivor only meets the exact test.
          const float reach = 2.0f * 1.7320508f * SCREEN_BOX + c.dcol + 1e-3f;
          const float err = 1.01f * 7.0f * 5.9604645e-8f * (reach * reach + c.dcol2);
          const float thr_x = c.dcol2 + 3.0f * err;
          const float na = fmaf(s.x[2], s.x[2], fmaf(s.x[1], s.x[1], fmaf(s.x[0], s.x[0], -thr_x)));
          const float a0 = -2.0f * s.x[0], a1 = -2.0f * s.x[1], a2 = -2.0f * s.x[2];
          for_partner_pos<BS, N, 4>(tile, ls, n, [&](int, const float* pj) {
            const float e = fmaf(a2, pj[2], fmaf(a1, pj[1], fmaf(a0, pj[0], pj[3] + na)));
            acc = __builtin_amdgcn_alignbit(acc, __float_as_uint(e), 31u);
          });
          in_box = fmaxf(fabsf(s.x[0]), fmaxf(fabsf(s.x[1]), fabsf(s.x[2]))) <= SCREEN_BOX;
        }
        cand = (M)(__builtin_bitreverse32(acc) >> (32 - N));
      } else {
        for_partner_pos<BS, N>(tile, ls, n, [&](int jj, const float* pj) {
          const float d2 = sq_dist(pj, s.x);
          cand |= d2 < thr ? (M)1 << jj : (M)0;
          if constexpr (L > 0) knn_insert<L>(key, jj, me, d2);
        });
      }
    }
    const bool near_origin =
        fmaxf(fabsf(s.x[0]), fmaxf(fabsf(s.x[1]), fabsf(s.x[2]))) <= 1000.0f;
    if (!(near_origin && in_box)) cand = (M)(n >= 64 ? ~0ull : (1ull << n) - 1ull);
    // the quad itself (distance 0) leaves the contact mask below anyway
    cand &= ~((M)1 << me);
    for (unsigned long long m = cand; m != 0ull; m &= m - 1ull) {
      const int jj = __builtin_ctzll(m);
      const int j = ls + jj;
      const float pj[6] = {tile[0][j], tile[1][j], tile[2][j], tile[3][j], tile[4][j], tile[5][j]};
      pair(jj, pj, FalseT{}, FalseT{});
    }
  } else {
    for_partners<BS, N>(tile, ls, n,
                        [&](int jj, const float* pj) { pair(jj, pj, FalseT{}, TrueT{}); });
    if constexpr (ACC) cm = (M)(__builtin_bitreverse32(acc) >> (32 - N));
  }
  const unsigned long long cmask = collide ? (unsigned long long)(cm & ~((M)1 << me)) : 0ull;
  // The responses, for the partners in contact only, in partner order.
  for (unsigned long long m = cmask; m != 0ull; m &= m - 1ull) {
    const int jj = __builtin_ctzll(m);
    const int j = ls + jj;
    const float pj[6] = {tile[0][j], tile[1][j], tile[2][j], tile[3][j], tile[4][j], tile[5][j]};
    float dx, dy, dz, d2, nn[3], sp;
    pair_geom_v(c, pj, s, dx, dy, dz, d2);
    pair_normal<BS>(tile, s, j, jj, me, dx, dy, dz, d2, nn, sp);
    if (!(c.flags & F_APPROACH) || sp > 0.f) {
#pragma unroll
      for (int k = 0; k < 3; ++k) dv[k] = fmaf(sp, nn[k], dv[k]);
      hit = true;
    }
  }
  if (hit) {
    s.ev |= EVF_QUAD;
    float zv[4] = {0.f, 0.f, 0.f, 0.f}, zw[4] = {0.f, 0.f, 0.f, 0.f};
    if (c.col_nv > 0.0f || c.col_nw > 0.0f) {
      normal4(c, q, t, STREAM_PAIR, 0, zv);
      normal4(c, q, t, STREAM_PAIR, 1, zw);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      s.v[k] = c.col_decay * (s.v[k] + dv[k] + c.col_nv * zv[k]);
      s.w[k] = fmaf(c.col_nw, zw[k], s.w[k]);
    }
  }
  if (dwhit) {
    float za[4] = {0.f, 0.f, 0.f, 0.f}, zw[4] = {0.f, 0.f, 0.f, 0.f};
    if (c.dw_na > 0.0f || c.dw_nw > 0.0f) {
      normal4(c, q, t, STREAM_DOWNWASH, 0, za);
      normal4(c, q, t, STREAM_DOWNWASH, 1, zw);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float a = (k == 2 ? adw : 0.f) + c.dw_na * za[k];
      s.v[k] = fmaf(c.dt, a, s.v[k]);
      s.w[k] = fmaf(c.dt, c.dw_nw * zw[k], s.w[k]);
    }
  }
  return cmask;
}

// The smoothed collision penalty of one live lane alone: the PEN term of
// pair_pass (same partners, same order, same arithmetic), for a wavefront
// that sums it apart from the motion.
template <int BS, int N>
__device__ __forceinline__ void penalty_pass(const Consts& c, const float (*tile)[BS],
                                             const Quad& s, int ls, int n, int me, float& pacc,
                                             float beta) {
  const float hb = 0.5f / beta;  // each quad of a pair carries half
  for_partners<BS, N>(tile, ls, n, [&](int jj, const float* pj) {
    float dx, dy, dz, d2;
    pair_geom_v(c, pj, s, dx, dy, dz, d2);
    const float sp = hb * softplus_hw(beta * (c.dcol - __builtin_amdgcn_sqrtf(d2)));
    pacc = jj != me ? pacc + sp : pacc;
  });
}

// §III-C sensor noise on the own-state part of an observation row:
// U(-sn_x, sn_x) on x - goal, U(-sn_v, sn_v) on v, N(0, sn_w^2) on omega,
// from stream SENSOR at the observation's substep index.
__device__ __forceinline__ void sensor_noise(const Consts& c, uint32_t q, unsigned long long t,
                                             float o_x[3], float o_v[3], float o_w[3]) {
#pragma unroll
  for (int draw = 0; draw < 2; ++draw) {
    uint32_t r0 = q, r1 = (uint32_t)t, r2 = (uint32_t)(t >> 32), r3 = (STREAM_SENSOR << 8) | draw;
    philox4x32_10(r0, r1, r2, r3, c.key0, c.key1);
    const float a = draw == 0 ? c.sn_x : c.sn_v;
    float* o = draw == 0 ? o_x : o_v;
    o[0] = fmaf(a, 2.0f * u01(r0) - 1.0f, o[0]);
    o[1] = fmaf(a, 2.0f * u01(r1) - 1.0f, o[1]);
    o[2] = fmaf(a, 2.0f * u01(r2) - 1.0f, o[2]);
  }
  float z[4];
  normal4(c, q, t, STREAM_SENSOR, 2, z);
#pragma unroll
  for (int k = 0; k < 3; ++k) o_w[k] = fmaf(c.sn_w, z[k], o_w[k]);
}

// §III-E reward of a call from the post-call state, the goal offset dx, the
// rotor thrusts before the call (f0) and the call's events; the proximity
// term is added by the caller per neighbour slot (reward_prox).
__device__ __forceinline__ float reward_state(const Consts& c, const Quad& s, float f_max,
                                              const float dx[3], const float f0[4]) {
  float f2 = 0.f, df2 = 0.f;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float f1 = fmaf(f_max * s.u[i], s.u[i], s.e[i]);
    f2 = fmaf(f1, f1, f2);
    df2 = fmaf(f1 - f0[i], f1 - f0[i], df2);
  }
  const float* w = c.rw;
  float r = w[0] * sqrtf(dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2]);
  r += w[1] * sqrtf(s.v[0] * s.v[0] + s.v[1] * s.v[1] + s.v[2] * s.v[2]);
  r += w[2] * s.R[8];
  r += w[3] * sqrtf(s.w[0] * s.w[0] + s.w[1] * s.w[1] + s.w[2] * s.w[2]);
  r += w[4] * sqrtf(f2) + w[5] * sqrtf(df2);
  r += w[6] * (s.R[0] + s.R[4] + s.R[8] - 1.0f) * 0.5f + w[7] * s.R[0];
  r += (s.ev & EVF_FLOOR_HIT) ? w[8] : 0.f;
  r += s.fl != 0.f ? w[9] : 0.f;
  r += (s.ev & EVF_WALL) ? w[10] : 0.f;
  r += (s.ev & EVF_CEILING) ? w[11] : 0.f;
  r += (s.ev & EVF_QUAD) ? w[12] : 0.f;
  return r;
}

__device__ __forceinline__ float reward_prox(const Consts& c, float rx, float ry, float rz) {
  return c.rw[13] * fmaxf(1.0f - sqrtf(rx * rx + ry * ry + rz * rz) / c.rw[14], 0.f);
}

}  // namespace qs
