// Differentiable rollouts: a multi-call forward kernel (a fresh action per
// call, checkpoints of the state, the smoothed collision penalty) and the
// backward pass: a kernel that recomputes checkpoint segments in parallel,
// taping the per-substep states and motor-noise draws, and a kernel that
// sweeps the tape in reverse.
//
// Layouts: checkpoints and adjoint scratch are field-major [27][Q], tape
// rows [31][Q] (state and draws; coalesced per field); actions and their
// gradients are [call][Q][4].
#pragma once
#include "qs_adjoint.h"

namespace qs {

// Partner count the forward rollout's in-swarm loop is specialised for.
// With the penalty, swarms of 16 and more take their partners in chunks of
// four in a run-time loop (for_partners; 118 VGPRs at 32768 x 32, four
// wavefronts per SIMD), which measured faster than one partner at a time
// (forward 3.76 -> 3.43 ms; a fully unrolled loop had taken 6.4 ms against
// 4.2 for one at a time).  Without the penalty the chunked loop would
// cross 128 VGPRs, so those rollouts loop one partner at a time.
template <int N, bool PEN>
constexpr int kUnroll = (PEN || N < 16) ? N : 0;

// Workgroup -> quads mapping shared by the kernels (see step_kernel).
template <int BS, int N>
__device__ __forceinline__ void block_map(const Ptrs& p, int tid, int& qb, int& cnt, int& ls,
                                          int& n) {
  if constexpr (N > 0) {
    qb = blockIdx.x * BS;
    cnt = min(BS, p.Q - qb);
    ls = (tid / N) * N;
    n = N;
  } else {
    const int2 bq = p.blk[blockIdx.x];
    qb = bq.x;
    cnt = bq.y;
    const uint32_t swd = tid < cnt ? p.sw[qb + tid] : 0u;
    ls = (int)(swd >> 8);
    n = (int)(swd & 0xffu);
  }
}

__device__ __forceinline__ void load_state(const float* __restrict__ S, long long ld, int q,
                                           Quad& s) {
#pragma unroll
  for (int k = 0; k < 3; ++k) s.x[k] = S[(S_X + k) * ld + q];
#pragma unroll
  for (int k = 0; k < 3; ++k) s.v[k] = S[(S_V + k) * ld + q];
#pragma unroll
  for (int k = 0; k < 9; ++k) s.R[k] = S[(S_R + k) * ld + q];
#pragma unroll
  for (int k = 0; k < 3; ++k) s.w[k] = S[(S_W + k) * ld + q];
#pragma unroll
  for (int k = 0; k < 4; ++k) s.u[k] = S[(S_U + k) * ld + q];
#pragma unroll
  for (int k = 0; k < 4; ++k) s.e[k] = S[(S_E + k) * ld + q];
  s.fl = S[S_F * ld + q];
  s.ev = 0u;
}

__device__ __forceinline__ void store_state(float* __restrict__ S, long long ld, int q,
                                            const Quad& s) {
#pragma unroll
  for (int k = 0; k < 3; ++k) S[(S_X + k) * ld + q] = s.x[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) S[(S_V + k) * ld + q] = s.v[k];
#pragma unroll
  for (int k = 0; k < 9; ++k) S[(S_R + k) * ld + q] = s.R[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) S[(S_W + k) * ld + q] = s.w[k];
#pragma unroll
  for (int k = 0; k < 4; ++k) S[(S_U + k) * ld + q] = s.u[k];
#pragma unroll
  for (int k = 0; k < 4; ++k) S[(S_E + k) * ld + q] = s.e[k];
  S[S_F * ld + q] = s.fl;
}

// A tape row: the state at the start of a substep (27 fields) and the
// motor-noise draws of that substep (4 fields), field-major over Q quads.
constexpr int NTAPE = NSTATE + 4;

__device__ __forceinline__ void load_draws(const Consts& c, const float* __restrict__ row,
                                           long long ld, int q, float z[4]) {
  if (c.flags & F_NOISE) {
#pragma unroll
    for (int i = 0; i < 4; ++i) z[i] = row[(NSTATE + i) * ld + q];
  }
}

__device__ __forceinline__ void load_params(const Ptrs& p, const Consts& c, int q, QuadPar& pp,
                                            ParAdj& pa) {
  const int Qp = p.Qp;
  pp.m = p.par[P_M * Qp + q];
  pp.jx = p.par[P_JX * Qp + q];
  pp.jy = p.par[P_JY * Qp + q];
  pp.jz = p.par[P_JZ * Qp + q];
  pp.f_max = p.par[P_FMAX * Qp + q];
  pp.a_lag = p.par[P_ALAG * Qp + q];
  pp.inv_m = 1.0f / pp.m;
  pp.ijx = 1.0f / pp.jx;
  pp.ijy = 1.0f / pp.jy;
  pp.ijz = 1.0f / pp.jz;
  pp.a_ns = c.ns_scale * pp.f_max;
  pa.m = pp.m;
  pa.jx = pp.jx;
  pa.jy = pp.jy;
  pa.jz = pp.jz;
  pa.t2w = p.par[P_T2W * Qp + q];
  const float tau = p.par[P_TAU * Qp + q];
  pa.dlag_dtau = -(1.0f - pp.a_lag) * c.dt / (tau * tau);
}

// The action row of quad q for one call.  The multi-call kernels load it a
// call ahead, so the load's latency overlaps the previous call's substeps
// instead of stalling every call.
__device__ __forceinline__ float4 load_act(const float* act, int q) {
  return reinterpret_cast<const float4*>(act)[q];
}

// Rotor commands of an action row; a non-finite action sets the sticky
// error bit.
__device__ __forceinline__ void act_uhat(const Consts& c, const Ptrs& p, const float4& a4,
                                         float uhat[4]) {
  const bool unit = (c.flags & F_ACT_UNIT) != 0;
  uhat[0] = rotor_cmd(a4.x, unit);
  uhat[1] = rotor_cmd(a4.y, unit);
  uhat[2] = rotor_cmd(a4.z, unit);
  uhat[3] = rotor_cmd(a4.w, unit);
  if (!(isfinite(a4.x) && isfinite(a4.y) && isfinite(a4.z) && isfinite(a4.w)))
    __hip_atomic_fetch_or(p.err, ERRBIT_ACTION, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// d uhat / d a for one action component (0 where the clip is active or the
// command is zero).
__device__ __forceinline__ float duhat_da(const Consts& c, float a, float uhat) {
  if (!(uhat > 0.f)) return 0.f;
  if (c.flags & F_ACT_UNIT) return (a > 0.f && a < 1.f) ? 0.5f / uhat : 0.f;
  return (a > -1.f && a < 1.f) ? 0.25f / uhat : 0.f;
}

// ---------------------------------------------------------------------------
// Forward rollout: ncalls calls of nsub substeps from the handle's state,
// action of call k at act + k Q 4.  ckpt (optional): the state at the start
// of every ckpt_every-th call, checkpoint k at ckpt + k 27 Q.  pen
// (optional, PEN): each quad's share of the smoothed collision penalty,
// sum over substeps and env-mates of softplus(beta (d_col - d))/(2 beta).
// ---------------------------------------------------------------------------
template <int BS, int N, bool PEN>
__global__ __launch_bounds__(BS) void rollout_kernel(const Consts* __restrict__ cp, Ptrs p,
                                                     const float* __restrict__ act, int ncalls,
                                                     int nsub, unsigned long long t0,
                                                     float* __restrict__ ckpt, int ckpt_every,
                                                     float* __restrict__ pen, float beta) {
  __shared__ float sxv[2][9][BS];
  const Consts& c = *cp;
  const int tid = threadIdx.x;
  int qb, cnt, ls, n;
  block_map<BS, N>(p, tid, qb, cnt, ls, n);
  const bool live = tid < cnt;
  const int q = qb + (live ? tid : 0);
  const int me = tid - ls;
  const long long Q = p.Q;

  Quad s;
  QuadPar pp;
  ParAdj pa;
  if (live) {
    load_state(p.st, p.Qp, q, s);
    load_params(p, c, q, pp, pa);
  }
  const bool pairs = N != 1 && ((c.flags & (F_COLLIDE | F_DOWNWASH)) != 0 || PEN);
  float pacc = 0.f;
  int sidx = 0;
  float4 a_nx = make_float4(0.f, 0.f, 0.f, 0.f);
  if (live && ncalls > 0) a_nx = load_act(act, q);
  for (int call = 0; call < ncalls; ++call) {
    const float4 a4 = a_nx;
    if (live && call + 1 < ncalls) a_nx = load_act(act + (long long)(call + 1) * Q * 4, q);
    if (ckpt && call % ckpt_every == 0 && live)
      store_state(ckpt + (long long)(call / ckpt_every) * NSTATE * Q, Q, q, s);
    float uhat[4] = {0.f, 0.f, 0.f, 0.f};
    if (live) act_uhat(c, p, a4, uhat);
    for (int sub = 0; sub < nsub; ++sub, ++sidx) {
      const unsigned long long t = t0 + (unsigned long long)sidx;
      if (live) quad_substep(c, pp, s, uhat, (uint32_t)q, t);
      if (pairs) {
        float(*tile)[BS] = sxv[sidx & 1];
        if (live) {
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            tile[k][tid] = s.xo[k];
            tile[3 + k][tid] = s.inc[k];
            tile[6 + k][tid] = s.v[k];
          }
        }
        __syncthreads();
        if (live) pair_pass<BS, kUnroll<N, PEN>, PEN>(c, tile, s, ls, n, me, (uint32_t)q, t, pacc, beta);
      }
    }
  }
  if (live) {
    store_state(p.st, p.Qp, q, s);
    float chk = 0.f;
#pragma unroll
    for (int k = 0; k < 3; ++k) chk += s.x[k] + s.v[k] + s.w[k];
#pragma unroll
    for (int k = 0; k < 9; ++k) chk += s.R[k];
    if (!isfinite(chk))
      __hip_atomic_fetch_or(p.err, ERRBIT_STATE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if constexpr (PEN) pen[q] += pacc;
  }
}

// ---------------------------------------------------------------------------
// Backward pass of a rollout, two launches per chunk of checkpoint segments
// (a segment: ce calls from one checkpoint).
//
// recompute_kernel, grid (workgroups, segments of the chunk): workgroup
// (b, g) re-runs segment g of the chunk from its checkpoint ckpt + g 27 Q
// and tapes, for the chunk's k-th substep, the state at its start and its
// motor-noise draws, tape[k][31][Q] (the reverse sweep then re-runs the
// substep without regenerating the draws).  Given the checkpoints the
// segments are independent, so a chunk is recomputed in one parallel launch.
//  act: the chunk's first call; ncalls: calls in the chunk; t0: substep
//  index of the chunk's first substep.
// ---------------------------------------------------------------------------
template <int BS, int N>
__global__ __launch_bounds__(BS) void recompute_kernel(const Consts* __restrict__ cp, Ptrs p,
                                                       const float* __restrict__ ckpt,
                                                       const float* __restrict__ act, int ncalls,
                                                       int ce, int nsub, unsigned long long t0,
                                                       float* __restrict__ tape) {
  __shared__ float sxv[2][TILE_ROWS_CO][BS];
  const Consts& c = *cp;
  const int tid = threadIdx.x;
  int qb, cnt, ls, n;
  block_map<BS, N>(p, tid, qb, cnt, ls, n);
  const bool live = tid < cnt;
  const int q = qb + (live ? tid : 0);
  const int me = tid - ls;
  const long long Q = p.Q;
  const int c0 = blockIdx.y * ce;
  const int nc = min(ce, ncalls - c0);
  const bool pairs = N != 1 && (c.flags & (F_COLLIDE | F_DOWNWASH)) != 0;

  Quad s;
  QuadPar pp;
  ParAdj pa;
  if (live) {
    load_state(ckpt + (long long)blockIdx.y * NSTATE * Q, Q, q, s);
    load_params(p, c, q, pp, pa);
  }
  int sidx = c0 * nsub;
  float4 a_nx = make_float4(0.f, 0.f, 0.f, 0.f);
  if (live && nc > 0) a_nx = load_act(act + (long long)c0 * Q * 4, q);
  for (int call = c0; call < c0 + nc; ++call) {
    const float4 a4 = a_nx;
    if (live && call + 1 < c0 + nc) a_nx = load_act(act + (long long)(call + 1) * Q * 4, q);
    float uhat[4] = {0.f, 0.f, 0.f, 0.f};
    if (live) act_uhat(c, p, a4, uhat);
    for (int sub = 0; sub < nsub; ++sub, ++sidx) {
      const unsigned long long t = t0 + (unsigned long long)sidx;
      if (live) {
        float* row = tape + (long long)sidx * NTAPE * Q;
        store_state(row, Q, q, s);
        float z[4];
        quad_substep<false, Z_EXPORT>(c, pp, s, uhat, (uint32_t)q, t, nullptr, z);
        if (c.flags & F_NOISE) {
#pragma unroll
          for (int i = 0; i < 4; ++i) row[(NSTATE + i) * Q + q] = z[i];
        }
      }
      if (pairs) {
        float(*tile)[BS] = sxv[sidx & 1];
        if (live) {
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            tile[k][tid] = s.xo[k];
            tile[3 + k][tid] = s.inc[k];
            tile[6 + k][tid] = s.v[k];
          }
          put_screen_rows<kScreenSq<N>>(tile, tid, s.x);
        }
        __syncthreads();
        float unused = 0.f;
        if (live) pair_pass<BS, N, false, true>(c, tile, s, ls, n, me, (uint32_t)q, t, unused, 0.f);
      }
    }
  }
}

// Position, velocity, attitude, body rates and the floor flag of one tape
// or checkpoint row (field-major, leading dimension ld).
__device__ __forceinline__ void load_body(const float* __restrict__ row, long long ld, int q,
                                          Quad& s) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    s.x[k] = row[(S_X + k) * ld + q];
    s.v[k] = row[(S_V + k) * ld + q];
    s.w[k] = row[(S_W + k) * ld + q];
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) s.R[k] = row[(S_R + k) * ld + q];
  s.fl = row[S_F * ld + q];
  s.ev = 0u;
}

// recompute_pipe_kernel: recompute_kernel for small batches (swarms of 1
// or 8, up to 1024 workgroups of 64 quads), over two wavefronts per
// workgroup as in rollout_pipe_kernel: wavefront 0 runs the motor part of
// each substep one substep ahead (taping the rotor state and the draws) and
// hands thrust and torques through a two-slot LDS ring; wavefront 1 tapes the
// pose, velocity, rates and floor flag, runs the body part and the in-swarm
// pass.  Same arithmetic in the same order as recompute_kernel, so the tape
// is identical.
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(128) void recompute_pipe_kernel(const Consts* __restrict__ cp,
                                                             Ptrs p,
                                                             const float* __restrict__ ckpt,
                                                             const float* __restrict__ act,
                                                             int ncalls, int ce, int nsub,
                                                             unsigned long long t0,
                                                             float* __restrict__ tape) {
  constexpr int BS = 64;
  static_assert(N == 1 || N == 8, "pipelined recompute for swarms of 1 or 8");
  __shared__ float sxv[2][TILE_ROWS_CO][BS];
  __shared__ float ring[2][4][BS];
  const Consts& c = *cp;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int tid = threadIdx.x & 63;
  int qb, cnt, ls, n;
  block_map<BS, N>(p, tid, qb, cnt, ls, n);
  const bool live = tid < cnt;
  const int q = qb + (live ? tid : 0);
  const int me = tid - ls;
  const long long Q = p.Q;
  const int c0 = blockIdx.y * ce;
  const int nc = min(ce, ncalls - c0);
  const int n_steps = nc * nsub;  // substeps of the segment
  const int s0 = c0 * nsub;       // its first substep within the chunk
  const float* ck = ckpt + (long long)blockIdx.y * NSTATE * Q;
  QuadPar pp;
  ParAdj pa;
  if (live) load_params(p, c, q, pp, pa);

  if (wave == 0) {
    // ---- motor part of substep i at step i
    float u[4], e[4];
    if (live) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        u[k] = ck[(S_U + k) * Q + q];
        e[k] = ck[(S_E + k) * Q + q];
      }
    }
    float uhat[4] = {0.f, 0.f, 0.f, 0.f};
    float4 a_nx = make_float4(0.f, 0.f, 0.f, 0.f);
    if (live && nc > 0) a_nx = load_act(act + (long long)c0 * Q * 4, q);
    for (int i = 0; i <= n_steps; ++i) {
      if (i < n_steps) {
        const int cl = i / nsub, sub = i - cl * nsub;
        const int call = c0 + cl;
        if (sub == 0) {
          const float4 a4 = a_nx;
          if (live && call + 1 < c0 + nc) a_nx = load_act(act + (long long)(call + 1) * Q * 4, q);
          if (live) act_uhat(c, p, a4, uhat);
        }
        if (live) {
          float* row = tape + (long long)(s0 + i) * NTAPE * Q;
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            row[(S_U + k) * Q + q] = u[k];
            row[(S_E + k) * Q + q] = e[k];
          }
          float z[4] = {0.f, 0.f, 0.f, 0.f}, zio[4];
          const Drive d = motor_step<Z_EXPORT>(c, pp, u, e, uhat, (uint32_t)q,
                                               t0 + (unsigned long long)(s0 + i), z, zio);
          if (c.flags & F_NOISE) {
#pragma unroll
            for (int k = 0; k < 4; ++k) row[(NSTATE + k) * Q + q] = zio[k];
          }
          float(*slot)[BS] = ring[i & 1];
          slot[0][tid] = d.T;
          slot[1][tid] = d.tx;
          slot[2][tid] = d.ty;
          slot[3][tid] = d.tz;
        }
      }
      wg_sync();
    }
  } else {
    // ---- body part and in-swarm pass of substep i - 1 at step i
    Quad s;
    if (live) load_body(ck, Q, q, s);
    const bool pairs = N != 1 && (c.flags & (F_COLLIDE | F_DOWNWASH)) != 0;
    wg_sync();  // step 0: no thrust yet
    for (int i = 1; i <= n_steps; ++i) {
      const int sidx = i - 1;
      const unsigned long long t = t0 + (unsigned long long)(s0 + sidx);
      if (live) {
        float* row = tape + (long long)(s0 + sidx) * NTAPE * Q;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          row[(S_X + k) * Q + q] = s.x[k];
          row[(S_V + k) * Q + q] = s.v[k];
          row[(S_W + k) * Q + q] = s.w[k];
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) row[(S_R + k) * Q + q] = s.R[k];
        row[S_F * Q + q] = s.fl;
        const float(*slot)[BS] = ring[sidx & 1];
        Drive d;
        d.T = slot[0][tid];
        d.tx = slot[1][tid];
        d.ty = slot[2][tid];
        d.tz = slot[3][tid];
        body_step(c, pp, s, d, (uint32_t)q, t);
      }
      if (pairs) {
        float(*tile)[BS] = sxv[sidx & 1];
        if (live) {
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            tile[k][tid] = s.xo[k];
            tile[3 + k][tid] = s.inc[k];
            tile[6 + k][tid] = s.v[k];
          }
          put_screen_rows<kScreenSq<N>>(tile, tid, s.x);
        }
        wave_sync();
        float unused = 0.f;
        if (live) pair_pass<BS, N, false, true>(c, tile, s, ls, n, me, (uint32_t)q, t, unused, 0.f);
      }
      wg_sync();
    }
  }
}

// One branch-free pass over the partners of a substep in the reverse sweep:
// the contact set (the quad itself excluded) and, with the penalty, its
// adjoint w.r.t. the quad's position,
//   d pen / d x_i = -(g_i + g_j)/2 sigmoid(beta (d_col - d)) (x_i - x_j) / d,
// summed over the partners in partner order into pen3 (added to lambda_x by
// the caller).  h_me = -g_me/2, and row 12 of the tile holds -g_j/2 for the
// partners (halving is exact, so h_me + h_j rounds as -(g_me + g_j)/2).
template <int BS, int N, bool PEN, typename T>
__device__ __forceinline__ unsigned long long mark_contacts(const Consts& c, T tile, const Quad& s,
                                                            int ls, int n, int me, float beta,
                                                            float h_me, float pen3[3]) {
  const bool collide = (c.flags & F_COLLIDE) != 0;
  PairMask<N> cm32 = 0;
  // Swarms of 16 and 32: partners arrive in index order, so the contact
  // bits are shifted in ((acc << 1) | sign bit of d^2 - d_col^2, one funnel
  // shift; for finite d^2 the sign of the difference is exactly the outcome
  // of the comparison)
  // and bit-reversed once, as in the forward screen.
  constexpr bool ACC = N >= 16 && N <= 32;
  uint32_t acc = 0u;
  auto mark = [&](int jj, const float* pj) {
    float dx, dy, dz, d2;
    const bool con = pair_geom_v(c, pj, s, dx, dy, dz, d2);
    if constexpr (ACC)
      acc = __builtin_amdgcn_alignbit(acc, __float_as_uint(d2 - c.dcol2), 31u);
    else
      cm32 |= (collide & con) ? (PairMask<N>)1 << jj : (PairMask<N>)0;
    if constexpr (PEN) {
      // the quad itself has d^2 = 0 exactly, so d^2 > 0 also leaves it out
      const float rd = __builtin_amdgcn_rsqf(d2);
      const float coef = d2 > 0.f
                             ? (h_me + pj[6]) * sigmoid_hw(beta * (c.dcol - d2 * rd)) * rd
                             : 0.f;
      pen3[0] = fmaf(coef, dx, pen3[0]);
      pen3[1] = fmaf(coef, dy, pen3[1]);
      pen3[2] = fmaf(coef, dz, pen3[2]);
    }
  };
  for_partners<BS, N, PEN ? 12 : -1>(tile, ls, n, mark);
  if constexpr (ACC) cm32 = collide ? (PairMask<N>)(__builtin_bitreverse32(acc) >> (32 - N)) : 0;
  return (unsigned long long)(cm32 & ~((PairMask<N>)1 << me));  // not the quad itself
}

// Approach test of the contact set: does the quad receive a response?
template <int BS>
__device__ __forceinline__ bool any_response(const Consts& c, const float (*tile)[BS],
                                             const Quad& s, int ls, int me,
                                             unsigned long long cm) {
  bool hit = false;
  for (unsigned long long m = cm; m != 0ull; m &= m - 1ull) {
    const int jj = __builtin_ctzll(m);
    const int j = ls + jj;
    const float pj[6] = {tile[0][j], tile[1][j], tile[2][j], tile[3][j], tile[4][j], tile[5][j]};
    float dx, dy, dz, d2, nn[3], sp;
    pair_geom_v(c, pj, s, dx, dy, dz, d2);
    pair_normal<BS>(tile, s, j, jj, me, dx, dy, dz, d2, nn, sp);
    if (!(c.flags & F_APPROACH) || sp > 0.f) hit = true;
  }
  return hit;
}

// Adjoint of the collision responses of one quad (the partners in contact):
// ldv (rows 9-11 for the partners): adjoint of each quad's velocity change.
template <int BS>
__device__ __forceinline__ void response_vjp(const Consts& c, const float (*tile)[BS],
                                             const float (*ldvt)[BS], const Quad& s, int ls,
                                             int me, unsigned long long cm, const float ldv[3],
                                             Adj& l) {
  for (unsigned long long m = cm; m != 0ull; m &= m - 1ull) {
    const int jj = __builtin_ctzll(m);
    const int j = ls + jj;
    const float pj[6] = {tile[0][j], tile[1][j], tile[2][j], tile[3][j], tile[4][j], tile[5][j]};
    float dx, dy, dz, d2, nn[3], sp;
    pair_geom_v(c, pj, s, dx, dy, dz, d2);
    pair_normal<BS>(tile, s, j, jj, me, dx, dy, dz, d2, nn, sp);
    if (!(c.flags & F_APPROACH) || sp > 0.f) {
      const float mu[3] = {ldv[0] - ldvt[0][j], ldv[1] - ldvt[1][j], ldv[2] - ldvt[2][j]};
      const float mn = dot3f(mu, nn);
#pragma unroll
      for (int k = 0; k < 3; ++k) l.v[k] = fmaf(-mn, nn[k], l.v[k]);
      if (!(d2 < 1e-12f)) {
        const float wv[3] = {tile[6][j] - s.v[0], tile[7][j] - s.v[1], tile[8][j] - s.v[2]};
        float gn[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) gn[k] = fmaf(sp, mu[k], mn * wv[k]);
        const float gnn = dot3f(gn, nn);
        const float id = rsqrtf(d2);
#pragma unroll
        for (int k = 0; k < 3; ++k) l.x[k] = fmaf(gn[k] - gnn * nn[k], id, l.x[k]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// reverse_kernel: the reverse sweep over the chunk's ncalls nsub substeps,
// last to first, from the tape; the adjoint of the state stays in
// registers for the whole chunk and the tape row of the next substep to
// process is loaded while the current one is differentiated.
//  lam: [27][Q] dL/d(chunk end) in, dL/d(chunk start) out; gpen: dL/d pen
//  (PEN); act/gact: the chunk's first call; gpar: [6][Q]
//  dL/d(m, ixx, iyy, izz, t2w, tau), accumulated.
// ---------------------------------------------------------------------------
template <int BS, int N, bool PEN>
__global__ __launch_bounds__(BS) void reverse_kernel(const Consts* __restrict__ cp, Ptrs p,
                                                     const float* __restrict__ act, int ncalls,
                                                     int nsub, unsigned long long t0,
                                                     const float* __restrict__ tape,
                                                     float* __restrict__ lam,
                                                     const float* __restrict__ gpen, float beta,
                                                     float* __restrict__ gact,
                                                     float* __restrict__ gpar) {
  // rows 0-8 as in the forward tile; 9-11: adjoint of the collision
  // velocity change; 12: penalty weight dL/d pen
  __shared__ float tl[13][BS];
  const Consts& c = *cp;
  const int tid = threadIdx.x;
  int qb, cnt, ls, n;
  block_map<BS, N>(p, tid, qb, cnt, ls, n);
  const bool live = tid < cnt;
  const int q = qb + (live ? tid : 0);
  const int me = tid - ls;
  const long long Q = p.Q;
  const bool collide = (c.flags & F_COLLIDE) != 0;
  const bool pairs = N != 1 && (collide || PEN);
  float(*tile)[BS] = tl;

  Quad s, sn;
  float z[4], zn[4] = {0.f, 0.f, 0.f, 0.f};  // motor-noise draws of s and sn
  QuadPar pp;
  ParAdj pa;
  const int n_steps = ncalls * nsub;
  if (live) {
    load_params(p, c, q, pp, pa);
    load_state(tape + (long long)(n_steps - 1) * NTAPE * Q, Q, q, sn);
    load_draws(c, tape + (long long)(n_steps - 1) * NTAPE * Q, Q, q, zn);
  }
  if constexpr (PEN) {
    tl[12][tid] = live ? -0.5f * gpen[q] : 0.f;  // -g/2 (mark_contacts)
  }

  // ---- reverse sweep
  Adj l;
  float gp[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (live) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      l.x[k] = lam[(S_X + k) * Q + q];
      l.v[k] = lam[(S_V + k) * Q + q];
      l.w[k] = lam[(S_W + k) * Q + q];
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) l.R[k] = lam[(S_R + k) * Q + q];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      l.u[k] = lam[(S_U + k) * Q + q];
      l.e[k] = lam[(S_E + k) * Q + q];
    }
  }
  float4 a_nx = make_float4(0.f, 0.f, 0.f, 0.f);
  if (live && ncalls > 0) a_nx = load_act(act + (long long)(ncalls - 1) * Q * 4, q);
  for (int call = ncalls - 1; call >= 0; --call) {
    float uhat[4] = {0.f, 0.f, 0.f, 0.f}, gu[4] = {0.f, 0.f, 0.f, 0.f};
    const float4 a4 = a_nx;
    if (live && call > 0) a_nx = load_act(act + (long long)(call - 1) * Q * 4, q);
    if (live) act_uhat(c, p, a4, uhat);
    for (int sub = nsub - 1; sub >= 0; --sub) {
      const int k_s = call * nsub + sub;
      const unsigned long long t = t0 + (unsigned long long)k_s;
      Rec r;
      if (live) {
        s = sn;
#pragma unroll
        for (int i = 0; i < 4; ++i) z[i] = zn[i];
        if (k_s > 0) {
          const float* row = tape + (long long)(k_s - 1) * NTAPE * Q;
          load_state(row, Q, q, sn);
          load_draws(c, row, Q, q, zn);
        }
        quad_substep<true, Z_IMPORT>(c, pp, s, uhat, (uint32_t)q, t, &r, z);
      }
      if (pairs) {
        __syncthreads();  // previous readers of the tile are done
        if (live) {
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            tile[k][tid] = s.xo[k];
            tile[3 + k][tid] = s.inc[k];
            tile[6 + k][tid] = s.v[k];
          }
        }
        __syncthreads();
        // which quads responded, and the adjoint of their velocity change:
        // one branch-free pass over the partners gives the contact set and
        // the penalty's adjoint (penalty weights in row 12, written before the
        // sweep); the approach test runs for the (rare) contacts only
        bool hit = false;
        unsigned long long cm = 0ull;  // contact set of this substep
        if (live) {
          float pen3[3] = {0.f, 0.f, 0.f};
          cm = mark_contacts<BS, N, PEN>(c, tile, s, ls, n, me, beta, tile[12][tid], pen3);
          if constexpr (PEN) {
#pragma unroll
            for (int k = 0; k < 3; ++k) l.x[k] += pen3[k];
          }
          hit = any_response<BS>(c, tile, s, ls, me, cm);
        }
        float ldv[3] = {0.f, 0.f, 0.f};
        if (live && hit) {
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            ldv[k] = c.col_decay * l.v[k];
            l.v[k] = ldv[k];
          }
        }
        if (live) {
#pragma unroll
          for (int k = 0; k < 3; ++k) tile[9 + k][tid] = ldv[k];
        }
        __syncthreads();
        if (live) response_vjp<BS>(c, tile, tile + 9, s, ls, me, cm, ldv, l);
      }
      if (live) quad_vjp(c, pp, pa, r, uhat, l, gu, gp);
    }
    if (live) {
      float4 g;
      g.x = gu[0] * duhat_da(c, a4.x, uhat[0]);
      g.y = gu[1] * duhat_da(c, a4.y, uhat[1]);
      g.z = gu[2] * duhat_da(c, a4.z, uhat[2]);
      g.w = gu[3] * duhat_da(c, a4.w, uhat[3]);
      reinterpret_cast<float4*>(gact + (long long)call * Q * 4)[q] = g;
    }
  }
  if (live) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      lam[(S_X + k) * Q + q] = l.x[k];
      lam[(S_V + k) * Q + q] = l.v[k];
      lam[(S_W + k) * Q + q] = l.w[k];
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) lam[(S_R + k) * Q + q] = l.R[k];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      lam[(S_U + k) * Q + q] = l.u[k];
      lam[(S_E + k) * Q + q] = l.e[k];
    }
    lam[S_F * Q + q] = 0.f;
#pragma unroll
    for (int k = 0; k < 6; ++k) gpar[k * Q + q] += gp[k];
  }
}

// ---------------------------------------------------------------------------
// reverse_pipe_kernel: the reverse sweep of reverse_kernel for small batches
// (one wavefront per SIMD or fewer), as a four-stage pipeline over the
// substeps (last to first) on four wavefronts per workgroup of 64 quads, one
// per SIMD of the compute unit.  Substep k passes through
//  - wavefront 0 at step i: the motor part re-run (lag, noise, thrust, mix)
//    from the taped rotor state and draws; the thrust, the torques, the
//    rotor fields of the record and the call's rotor commands with their
//    derivatives w.r.t. the action go on through a four-slot LDS ring;
//  - wavefront 1 at step i + 1: the body part re-run (body_step with its
//    record) from the taped pose and rates; the post-motion exchange tile and
//    the body fields of the record (in 16-byte groups) go on through
//    three-slot rings;
//  - wavefront 2 at step i + 2: the contact set, the approach test and the
//    penalty's adjoint from the exchange tile, through a two-slot ring;
//  - wavefront 3 at step i + 3: the derivative (response adjoint, quad_vjp);
//    it holds the adjoint state.
// A substep's re-run starts from its taped state, so no stage waits for the
// substep after it; one workgroup barrier per step hands the slots over.
// Same arithmetic in the same order as reverse_kernel, so the results are
// identical.
// ---------------------------------------------------------------------------
constexpr int REC_BODY = 49;  // the float fields of Rec that body_step sets
// ring of the body stage: the body fields and Rec's flags, in 16-byte
// groups (one LDS vector access per group)
constexpr int RING_WORDS = REC_BODY + 1;
constexpr int RING_VEC = (RING_WORDS + 3) / 4;
// motor ring, 16-byte groups: draws, rotor speeds before and after, thrust
// and torques, the rotor commands and their derivatives w.r.t. the action
constexpr int MOTOR_VEC = 6;
// contact ring words: response flag, contact set, penalty adjoint
constexpr int CON_WORDS = 5;

template <typename R, typename F>
__device__ __forceinline__ void rec_body_floats(R& r, F&& f) {
  int w = 0;
  auto g = [&](auto& v) { f(w++, v); };
#pragma unroll
  for (int k = 0; k < 9; ++k) g(r.P[k]);
#pragma unroll
  for (int k = 0; k < 3; ++k) { g(r.w0[k]); g(r.v0[k]); g(r.F[k]); g(r.wdot[k]); g(r.w1[k]); }
#pragma unroll
  for (int k = 0; k < 3; ++k) { g(r.A1[k]); g(r.c0[k]); g(r.c1[k]); }
  g(r.T); g(r.i0); g(r.dp); g(r.i1);
  g(r.mu_n); g(r.fb[0]); g(r.fb[1]); g(r.nv); g(r.nf); g(r.mag);
  g(r.hx); g(r.hy); g(r.nh); g(r.kx); g(r.ky); g(r.nk);
}

__device__ __forceinline__ uint32_t rec_flags(const Rec& r) {
  uint32_t b = (uint32_t)r.rest | (uint32_t)r.statik << 1 | (uint32_t)r.guard << 2 |
               (uint32_t)r.bounced << 3 | (uint32_t)r.hit << 4 | (uint32_t)r.fallback << 5;
#pragma unroll
  for (int k = 0; k < 3; ++k) b |= (uint32_t)r.clamp[k] << (6 + k) | (uint32_t)r.flip[k] << (9 + k);
  return b;
}

__device__ __forceinline__ void rec_unflag(Rec& r, uint32_t b) {
  r.rest = b & 1u;
  r.statik = (b >> 1) & 1u;
  r.guard = (b >> 2) & 1u;
  r.bounced = (b >> 3) & 1u;
  r.hit = (b >> 4) & 1u;
  r.fallback = (b >> 5) & 1u;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    r.clamp[k] = (b >> (6 + k)) & 1u;
    r.flip[k] = (b >> (9 + k)) & 1u;
  }
}

// The rotor state and the draws of one tape row.
__device__ __forceinline__ void load_rotor(const Consts& c, const float* __restrict__ row,
                                           long long ld, int q, float u[4], float e[4],
                                           float z[4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    u[k] = row[(S_U + k) * ld + q];
    e[k] = row[(S_E + k) * ld + q];
  }
  load_draws(c, row, ld, q, z);
}

template <int N, bool PEN>
__global__ __launch_bounds__(256) void reverse_pipe_kernel(const Consts* __restrict__ cp, Ptrs p,
                                                           const float* __restrict__ act,
                                                           int ncalls, int nsub,
                                                           unsigned long long t0,
                                                           const float* __restrict__ tape,
                                                           float* __restrict__ lam,
                                                           const float* __restrict__ gpen,
                                                           float beta, float* __restrict__ gact,
                                                           float* __restrict__ gpar) {
  constexpr int BS = 64;
  static_assert(N == 1 || N == 8, "pipelined reverse sweep for swarms of 1 or 8");
  // Slots are indexed by the substep k.  Tile rows 0-8 post-motion start
  // position, displacement, velocity (wavefront 1); 9-11 adjoint of the
  // collision velocity change (wavefront 3); 12 penalty weights.
  __shared__ float tl[3][13][BS];
  __shared__ float4 ring[3][RING_VEC][BS];
  __shared__ float4 mring[4][MOTOR_VEC][BS];
  __shared__ float cring[2][CON_WORDS][BS];
  const Consts& c = *cp;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int tid = threadIdx.x & 63;
  int qb, cnt, ls, n;
  block_map<BS, N>(p, tid, qb, cnt, ls, n);
  const bool live = tid < cnt;
  const int q = qb + (live ? tid : 0);
  const int me = tid - ls;
  const long long Q = p.Q;
  const bool collide = (c.flags & F_COLLIDE) != 0;
  const bool pairs = N != 1 && (collide || PEN);
  const int n_steps = ncalls * nsub;
  const int n_pipe = n_steps + 3;  // steps of the pipeline

  QuadPar pp;
  ParAdj pa;
  if (live) load_params(p, c, q, pp, pa);
  if (PEN && wave == 2) {
    const float g = live ? -0.5f * gpen[q] : 0.f;  // -g/2 (mark_contacts)
#pragma unroll
    for (int m = 0; m < 3; ++m) tl[m][12][tid] = g;
  }

  if (wave == 0) {
    // ---- motor part of substep k = n_steps - 1 - i at step i
    float un[4], en[4], zn[4] = {0.f, 0.f, 0.f, 0.f};
    float uhat[4] = {0.f, 0.f, 0.f, 0.f}, dua[4] = {0.f, 0.f, 0.f, 0.f};
    float4 a_nx = make_float4(0.f, 0.f, 0.f, 0.f);
    if (live && n_steps > 0) {
      load_rotor(c, tape + (long long)(n_steps - 1) * NTAPE * Q, Q, q, un, en, zn);
      a_nx = load_act(act + (long long)(ncalls - 1) * Q * 4, q);
    }
    for (int i = 0; i < n_pipe; ++i) {
      if (i < n_steps) {
        const int k = n_steps - 1 - i;
        const int call = k / nsub, sub = k - call * nsub;
        if (sub == nsub - 1) {  // the call's last substep comes first
          const float4 a4 = a_nx;
          if (live && call > 0) a_nx = load_act(act + (long long)(call - 1) * Q * 4, q);
          if (live) {
            act_uhat(c, p, a4, uhat);
            dua[0] = duhat_da(c, a4.x, uhat[0]);
            dua[1] = duhat_da(c, a4.y, uhat[1]);
            dua[2] = duhat_da(c, a4.z, uhat[2]);
            dua[3] = duhat_da(c, a4.w, uhat[3]);
          }
        }
        if (live) {
          float u[4], e[4], zi[4], z[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            u[m] = un[m];
            e[m] = en[m];
            zi[m] = zn[m];
          }
          if (k > 0) load_rotor(c, tape + (long long)(k - 1) * NTAPE * Q, Q, q, un, en, zn);
          float4(*ms)[BS] = mring[k & 3];
          ms[1][tid] = make_float4(u[0], u[1], u[2], u[3]);
          const Drive d = motor_step<Z_IMPORT>(c, pp, u, e, uhat, (uint32_t)q,
                                               t0 + (unsigned long long)k, z, zi);
          ms[0][tid] = make_float4(z[0], z[1], z[2], z[3]);
          ms[2][tid] = make_float4(u[0], u[1], u[2], u[3]);
          ms[3][tid] = make_float4(d.T, d.tx, d.ty, d.tz);
          ms[4][tid] = make_float4(uhat[0], uhat[1], uhat[2], uhat[3]);
          ms[5][tid] = make_float4(dua[0], dua[1], dua[2], dua[3]);
        }
      }
      wg_sync();
    }
  } else if (wave == 1) {
    // ---- body part of substep k = n_steps - i at step i >= 1
    Quad sn;
    if (live && n_steps > 0) load_body(tape + (long long)(n_steps - 1) * NTAPE * Q, Q, q, sn);
    wg_sync();  // step 0: no thrust yet
    for (int i = 1; i < n_pipe; ++i) {
      if (i <= n_steps && live) {
        const int k = n_steps - i;
        Quad s = sn;
        if (k > 0) load_body(tape + (long long)(k - 1) * NTAPE * Q, Q, q, sn);
        const float4 dv = mring[k & 3][3][tid];
        Drive d;
        d.T = dv.x;
        d.tx = dv.y;
        d.ty = dv.z;
        d.tz = dv.w;
        Rec r;
        body_step<true>(c, pp, s, d, (uint32_t)q, t0 + (unsigned long long)k, &r);
        if (pairs) {
          float(*tile)[BS] = tl[k % 3];
#pragma unroll
          for (int m = 0; m < 3; ++m) {
            tile[m][tid] = s.xo[m];
            tile[3 + m][tid] = s.inc[m];
            tile[6 + m][tid] = s.v[m];
          }
        }
        float w4[4 * RING_VEC];
        rec_body_floats(r, [&](int w, const float& v) { w4[w] = v; });
        w4[REC_BODY] = __uint_as_float(rec_flags(r));
#pragma unroll
        for (int w = RING_WORDS; w < 4 * RING_VEC; ++w) w4[w] = 0.f;
        float4(*slot)[BS] = ring[k % 3];
#pragma unroll
        for (int g = 0; g < RING_VEC; ++g)
          slot[g][tid] = make_float4(w4[4 * g], w4[4 * g + 1], w4[4 * g + 2], w4[4 * g + 3]);
      }
      wg_sync();
    }
  } else if (wave == 2) {
    // ---- contacts of substep k = n_steps + 1 - i at step i >= 2
    wg_sync();  // steps 0 and 1: no exchange tile yet
    wg_sync();
    for (int i = 2; i < n_pipe; ++i) {
      if (pairs && i <= n_steps + 1 && live) {
        const int k = n_steps + 1 - i;
        const float(*tile)[BS] = tl[k % 3];
        Quad so;  // the quad's post-motion position and velocity
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          so.xo[m] = tile[m][tid];
          so.inc[m] = tile[3 + m][tid];
          so.v[m] = tile[6 + m][tid];
        }
        float pen3[3] = {0.f, 0.f, 0.f};
        const unsigned long long cm =
            mark_contacts<BS, N, PEN>(c, tile, so, ls, n, me, beta, tile[12][tid], pen3);
        const bool hit = any_response<BS>(c, tile, so, ls, me, cm);
        float(*cs)[BS] = cring[k & 1];
        cs[0][tid] = hit ? 1.f : 0.f;
        cs[1][tid] = __uint_as_float((uint32_t)cm);
#pragma unroll
        for (int m = 0; m < 3; ++m) cs[2 + m][tid] = pen3[m];
      }
      wg_sync();
    }
  } else {
    // ---- differentiate substep k = n_steps + 2 - i at step i >= 3
    Adj l;
    float gp[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (live) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        l.x[k] = lam[(S_X + k) * Q + q];
        l.v[k] = lam[(S_V + k) * Q + q];
        l.w[k] = lam[(S_W + k) * Q + q];
      }
#pragma unroll
      for (int k = 0; k < 9; ++k) l.R[k] = lam[(S_R + k) * Q + q];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        l.u[k] = lam[(S_U + k) * Q + q];
        l.e[k] = lam[(S_E + k) * Q + q];
      }
    }
    // the rotor commands and their derivatives come from the motor stage
    float gu[4] = {0.f, 0.f, 0.f, 0.f};
    wg_sync();  // steps 0 to 2: no record complete yet
    wg_sync();
    wg_sync();
    for (int i = 3; i < n_pipe; ++i) {
      const int k = n_steps + 2 - i;
      const int call = k / nsub, sub = k - call * nsub;
      if (sub == nsub - 1) {
#pragma unroll
        for (int m = 0; m < 4; ++m) gu[m] = 0.f;
      }
      if (live) {
        const float4(*slot)[BS] = ring[k % 3];
        const float4(*ms)[BS] = mring[k & 3];
        Rec r;
        const float4 z4 = ms[0][tid], u04 = ms[1][tid], u14 = ms[2][tid], uh4 = ms[4][tid];
        r.z[0] = z4.x; r.z[1] = z4.y; r.z[2] = z4.z; r.z[3] = z4.w;
        r.u0[0] = u04.x; r.u0[1] = u04.y; r.u0[2] = u04.z; r.u0[3] = u04.w;
        r.u1[0] = u14.x; r.u1[1] = u14.y; r.u1[2] = u14.z; r.u1[3] = u14.w;
        const float uhat[4] = {uh4.x, uh4.y, uh4.z, uh4.w};
        float w4[4 * RING_VEC];
#pragma unroll
        for (int g = 0; g < RING_VEC; ++g) {
          const float4 v4 = slot[g][tid];
          w4[4 * g] = v4.x;
          w4[4 * g + 1] = v4.y;
          w4[4 * g + 2] = v4.z;
          w4[4 * g + 3] = v4.w;
        }
        rec_body_floats(r, [&](int w, float& v) { v = w4[w]; });
        rec_unflag(r, __float_as_uint(w4[REC_BODY]));
        if (pairs) {
          const float(*cs)[BS] = cring[k & 1];
          const bool hit = cs[0][tid] != 0.f;
          const unsigned long long cm = __float_as_uint(cs[1][tid]);
          if constexpr (PEN) {
#pragma unroll
            for (int m = 0; m < 3; ++m) l.x[m] += cs[2 + m][tid];
          }
          float(*tile)[BS] = tl[k % 3];
          float ldv[3] = {0.f, 0.f, 0.f};
          if (hit) {
#pragma unroll
            for (int m = 0; m < 3; ++m) {
              ldv[m] = c.col_decay * l.v[m];
              l.v[m] = ldv[m];
            }
          }
#pragma unroll
          for (int m = 0; m < 3; ++m) tile[9 + m][tid] = ldv[m];
          wave_sync();
          if (cm != 0ull) {
            Quad so;  // the quad's post-motion position and velocity
#pragma unroll
            for (int m = 0; m < 3; ++m) {
              so.xo[m] = tile[m][tid];
              so.inc[m] = tile[3 + m][tid];
              so.v[m] = tile[6 + m][tid];
            }
            response_vjp<BS>(c, tile, tile + 9, so, ls, me, cm, ldv, l);
          }
        }
        quad_vjp(c, pp, pa, r, uhat, l, gu, gp);
        if (sub == 0) {
          const float4 da = ms[5][tid];
          float4 g;
          g.x = gu[0] * da.x;
          g.y = gu[1] * da.y;
          g.z = gu[2] * da.z;
          g.w = gu[3] * da.w;
          reinterpret_cast<float4*>(gact + (long long)call * Q * 4)[q] = g;
        }
      } else if (pairs) {
        wave_sync();
      }
      wg_sync();
    }
    if (live) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        lam[(S_X + k) * Q + q] = l.x[k];
        lam[(S_V + k) * Q + q] = l.v[k];
        lam[(S_W + k) * Q + q] = l.w[k];
      }
#pragma unroll
      for (int k = 0; k < 9; ++k) lam[(S_R + k) * Q + q] = l.R[k];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        lam[(S_U + k) * Q + q] = l.u[k];
        lam[(S_E + k) * Q + q] = l.e[k];
      }
      lam[S_F * Q + q] = 0.f;
#pragma unroll
      for (int k = 0; k < 6; ++k) gpar[k * Q + q] += gp[k];
    }
  }
}

// ---------------------------------------------------------------------------
// rollout_pipe_kernel: rollout_kernel for small batches, over two or three
// wavefronts per workgroup of 64 quads.  The motor part of a substep (lag,
// noise, thrust, mix) depends on the rotor state, the action and the
// substep's draws only, so wavefront 0 runs it one substep ahead and hands
// the thrust and torques (4 words per quad) to wavefront 1 through a
// two-slot LDS ring; wavefront 1 runs the body part and the in-swarm pass.
// The smoothed collision penalty never feeds back into the motion, so in
// swarms with a penalty wavefront 2 sums it one substep behind, from the
// post-motion exchange tile.  One workgroup barrier per substep; each
// wavefront stores its own fields of the checkpoints and of the final state.
// Same arithmetic in the same order as rollout_kernel, so the results are
// identical.
// ---------------------------------------------------------------------------
template <int N, bool PEN>
constexpr int kRollWaves = (PEN && N != 1) ? 3 : 2;

template <int N, bool PEN>
__global__ __launch_bounds__(192) void rollout_pipe_kernel(const Consts* __restrict__ cp, Ptrs p,
                                                           const float* __restrict__ act,
                                                           int ncalls, int nsub,
                                                           unsigned long long t0,
                                                           float* __restrict__ ckpt,
                                                           int ckpt_every,
                                                           float* __restrict__ pen, float beta) {
  constexpr int BS = 64;
  constexpr bool PW = kRollWaves<N, PEN> == 3;  // penalty on its own wavefront
  static_assert(N == 1 || N == 8, "pipelined rollout for swarms of 1 or 8");
  __shared__ float sxv[2][TILE_ROWS_CO][BS];
  __shared__ float ring[2][4][BS];
  const Consts& c = *cp;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int tid = threadIdx.x & 63;
  int qb, cnt, ls, n;
  block_map<BS, N>(p, tid, qb, cnt, ls, n);
  const bool live = tid < cnt;
  const int q = qb + (live ? tid : 0);
  const int me = tid - ls;
  const long long Q = p.Q;
  const int n_steps = ncalls * nsub;
  const int n_pipe = n_steps + (PW ? 2 : 1);  // steps of the pipeline
  QuadPar pp;
  ParAdj pa;
  if (live) load_params(p, c, q, pp, pa);

  if (wave == 0) {
    // ---- motor part of substep i at step i
    float u[4], e[4];
    if (live) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        u[k] = p.st[(S_U + k) * p.Qp + q];
        e[k] = p.st[(S_E + k) * p.Qp + q];
      }
    }
    float uhat[4] = {0.f, 0.f, 0.f, 0.f};
    float4 a_nx = make_float4(0.f, 0.f, 0.f, 0.f);
    if (live && ncalls > 0) a_nx = load_act(act, q);
    for (int i = 0; i < n_pipe; ++i) {
      if (i < n_steps) {
        const int call = i / nsub, sub = i - call * nsub;
        if (sub == 0) {
          const float4 a4 = a_nx;
          if (live && call + 1 < ncalls) a_nx = load_act(act + (long long)(call + 1) * Q * 4, q);
          if (ckpt && call % ckpt_every == 0 && live) {
            float* ck = ckpt + (long long)(call / ckpt_every) * NSTATE * Q;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              ck[(S_U + k) * Q + q] = u[k];
              ck[(S_E + k) * Q + q] = e[k];
            }
          }
          if (live) act_uhat(c, p, a4, uhat);
        }
        if (live) {
          float z[4] = {0.f, 0.f, 0.f, 0.f};
          const Drive d = motor_step(c, pp, u, e, uhat, (uint32_t)q, t0 + (unsigned long long)i, z);
          float(*slot)[BS] = ring[i & 1];
          slot[0][tid] = d.T;
          slot[1][tid] = d.tx;
          slot[2][tid] = d.ty;
          slot[3][tid] = d.tz;
        }
      }
      wg_sync();
    }
    if (live) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        p.st[(S_U + k) * p.Qp + q] = u[k];
        p.st[(S_E + k) * p.Qp + q] = e[k];
      }
    }
  } else if (wave == 1) {
    // ---- body part and in-swarm pass of substep i - 1 at step i
    Quad s;
    if (live) load_state(p.st, p.Qp, q, s);
    const bool pairs = N != 1 && ((c.flags & (F_COLLIDE | F_DOWNWASH)) != 0 || PEN);
    float pacc = 0.f;
    wg_sync();  // step 0: no thrust yet
    for (int i = 1; i < n_pipe; ++i) {
      if (i <= n_steps) {
        const int sidx = i - 1;
        const int call = sidx / nsub, sub = sidx - call * nsub;
        if (sub == 0 && ckpt && call % ckpt_every == 0 && live) {
          float* ck = ckpt + (long long)(call / ckpt_every) * NSTATE * Q;
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            ck[(S_X + k) * Q + q] = s.x[k];
            ck[(S_V + k) * Q + q] = s.v[k];
            ck[(S_W + k) * Q + q] = s.w[k];
          }
#pragma unroll
          for (int k = 0; k < 9; ++k) ck[(S_R + k) * Q + q] = s.R[k];
          ck[S_F * Q + q] = s.fl;
        }
        const unsigned long long t = t0 + (unsigned long long)sidx;
        if (live) {
          const float(*slot)[BS] = ring[sidx & 1];
          Drive d;
          d.T = slot[0][tid];
          d.tx = slot[1][tid];
          d.ty = slot[2][tid];
          d.tz = slot[3][tid];
          body_step(c, pp, s, d, (uint32_t)q, t);
        }
        if (pairs) {
          float(*tile)[BS] = sxv[sidx & 1];
          if (live) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
              tile[k][tid] = s.xo[k];
              tile[3 + k][tid] = s.inc[k];
              tile[6 + k][tid] = s.v[k];
            }
            put_screen_rows<kScreenSq<kUnroll<N, PEN>>>(tile, tid, s.x);
          }
          wave_sync();
          if (live)
            pair_pass<BS, kUnroll<N, PEN>, PEN && !PW, !(PEN && !PW)>(c, tile, s, ls, n, me,
                                                                (uint32_t)q, t, pacc, beta);
        }
      }
      wg_sync();
    }
    if (live) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        p.st[(S_X + k) * p.Qp + q] = s.x[k];
        p.st[(S_V + k) * p.Qp + q] = s.v[k];
        p.st[(S_W + k) * p.Qp + q] = s.w[k];
      }
#pragma unroll
      for (int k = 0; k < 9; ++k) p.st[(S_R + k) * p.Qp + q] = s.R[k];
      p.st[S_F * p.Qp + q] = s.fl;
      float chk = 0.f;
#pragma unroll
      for (int k = 0; k < 3; ++k) chk += s.x[k] + s.v[k] + s.w[k];
#pragma unroll
      for (int k = 0; k < 9; ++k) chk += s.R[k];
      if (!isfinite(chk))
        __hip_atomic_fetch_or(p.err, ERRBIT_STATE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if constexpr (PEN && !PW) pen[q] += pacc;
    }
  } else if constexpr (PW) {
    // ---- penalty of substep i - 2 at step i, from the exchange tile
    float pacc = 0.f;
    wg_sync();  // steps 0 and 1: no tile yet
    wg_sync();
    for (int i = 2; i < n_pipe; ++i) {
      if (live) {
        const float(*tile)[BS] = sxv[(i - 2) & 1];
        Quad so;  // the quad's start position and displacement
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          so.xo[k] = tile[k][tid];
          so.inc[k] = tile[3 + k][tid];
        }
        penalty_pass<BS, kUnroll<N, PEN>>(c, tile, so, ls, n, me, pacc, beta);
      }
      wg_sync();
    }
    if (live) pen[q] += pacc;
  }
}

// ---------------------------------------------------------------------------
// [rows][Q] field-major <-> [Q][rows] row-major conversions (optionally
// adding into the destination).
__global__ void fm_to_rm_kernel(const float* __restrict__ src, float* __restrict__ dst, int Q,
                                int rows, int accumulate) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)Q * rows) return;
  const int q = (int)(i / rows), f = (int)(i - (long long)q * rows);
  const float v = src[(long long)f * Q + q];
  dst[i] = accumulate ? dst[i] + v : v;
}

__global__ void rm_to_fm_kernel(const float* __restrict__ src, float* __restrict__ dst, int Q,
                                int rows) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)Q * rows) return;
  const int q = (int)(i / rows), f = (int)(i - (long long)q * rows);
  dst[(long long)f * Q + q] = src[i];
}

__global__ void fill_kernel(float* __restrict__ dst, long long n, float v) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = v;
}

}  // namespace qs
