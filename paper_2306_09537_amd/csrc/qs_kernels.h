// Kernels of the batched quadrotor-swarm step.
//
// Grid: one workgroup per "block" of whole environments (host-built
// partition, at most BS quads); one lane per quad.  The state is loaded
// from the SoA arrays once (coalesced), kept in VGPRs for all substeps of
// the call, and stored once.  Per substep, lanes exchange positions and
// velocities through a double-buffered LDS tile for the in-env pair pass
// (one barrier per substep).  The observation epilogue ranks swarm-mates
// from the same tile, stages the output rows in LDS and writes them with
// contiguous stores.
#pragma once
#include "qs_device.h"

namespace qs {

// Mapping of a workgroup's lanes to quads.
//  MAP_DENSE:  every swarm holds N quads; workgroup b owns quads [b BS, (b+1) BS).
//  MAP_TABLE:  any sizes; the host-built table gives each workgroup's first quad
//              and count, and each quad's swarm start (within the workgroup)
//              and size.
//  MAP_ITEM:   one work item of the uneven-size bucketing: up to BS/N swarms of
//              at most N quads each, lane t serving quad t % N of swarm t / N;
//              lanes past a swarm's size are padding.
enum : int { MAP_DENSE = 0, MAP_TABLE = 1, MAP_ITEM = 2 };

// Graph-safe substep counter: every workgroup reads the base substep index
// from device memory, after the loads of its first quads are in flight (the
// read goes to the coherence point; issued first, it would hold back every
// later load of the workgroup); the last workgroup to finish advances it by
// nsub.  No ordering beyond atomicity is needed: the last workgroup
// finishes after every other one has read the counter (each counts itself
// done after its reads), and the next launch reads the new value after the
// kernel boundary.  (A release here would write back the XCD's L2 from
// every workgroup.)
//
// The completion count is two-level: workgroup b counts itself in
// sub-counter b mod 64 (each on a 128-byte line of its own), and the last
// workgroup of each sub-counter counts in the top one.  Returning atomics on
// one address are performed one after another at the coherence point; with
// one counter, 2,700 workgroups took ~70 us to count themselves out
// (16384 uneven environments, ten substeps per call: 53 -> 71 us per call),
// with 65 lines at most ~42 + 64 of them queue on any one.
enum : int { DONE_SUBS = 64, DONE_STRIDE = 32, DONE_WORDS = (DONE_SUBS + 1) * DONE_STRIDE };

__device__ __forceinline__ unsigned long long read_counter(const unsigned long long* tdev) {
  return __hip_atomic_load(tdev, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// total: the workgroups of the launch; the last of them to finish advances
// the counter.  done: DONE_WORDS words, zero between launches.
__device__ __forceinline__ void advance_counter(unsigned long long* tdev, unsigned int* done,
                                                int nsub, unsigned int total) {
  __syncthreads();  // every thread of the workgroup has read the counter
  if (threadIdx.x == 0) {
    const unsigned int j = blockIdx.x % DONE_SUBS;
    const unsigned int in_sub = (total - j + DONE_SUBS - 1) / DONE_SUBS;
    unsigned int* sub = done + DONE_STRIDE * j;
    const unsigned int prev = __hip_atomic_fetch_add(sub, 1u, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
    if (prev == in_sub - 1) {
      __hip_atomic_store(sub, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      unsigned int* top = done + DONE_STRIDE * DONE_SUBS;
      const unsigned int n_subs = total < DONE_SUBS ? total : DONE_SUBS;
      const unsigned int p2 = __hip_atomic_fetch_add(top, 1u, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
      if (p2 == n_subs - 1) {
        __hip_atomic_fetch_add(tdev, (unsigned long long)nsub, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

// Body of one step (+ observation) over one workgroup's quads.
// KT: -2 step only; -1 observation with runtime K (selection); >= 0 observation
// with compile-time K (register insertion network).
// N: swarm (slot) size known at compile time (MAP_DENSE, MAP_ITEM), or 0.
// NU: partner count the in-swarm loops are unrolled for (N, or 0 for loops
// over the swarm's runtime size: fewer registers for large slots).
// sxv: LDS tile [2][TILE_ROWS_CO][BS]; st_obs: LDS staging of observation rows.
// ROLE: -1 one wavefront does everything; in a workgroup of two wavefronts
// over the same 64 quads (step_pipe_kernel), 0 runs the motor part of every
// substep one substep ahead and hands thrust and torques through ring, 1
// runs the rest (body part, in-swarm pass, observation); rx hands the rotor
// state over for the reward.
template <int BS, int KT, int N, int MAP, int NU = N, int ROLE = -1>
__device__ __forceinline__ void step_body(const Consts& c, const Ptrs& p,
                                          const float* __restrict__ act, int nsub,
                                          unsigned long long t0,
                                          const float* __restrict__ goals,
                                          float* __restrict__ obs, int stage_obs,
                                          float (*sxv)[TILE_ROWS_CO][BS], float* st_obs, int item,
                                          float* __restrict__ reward,
                                          const unsigned long long* tdev = nullptr,
                                          float (*ring)[4][BS] = nullptr,
                                          float (*rx)[BS] = nullptr) {
  static_assert(ROLE < 0 || (MAP == MAP_DENSE && BS == 64), "two roles: dense 64-quad groups");
  static_assert(N == 0 || BS % N == 0, "workgroups hold whole swarms");
  static_assert(MAP != MAP_TABLE || N == 0, "the table mapping has runtime sizes");
  constexpr bool OBS = KT != -2;
  const float4* st_obs4 = reinterpret_cast<const float4*>(st_obs);

  const int tid = ROLE < 0 ? (int)threadIdx.x : (int)(threadIdx.x & 63);
  // the in-swarm exchanges: every wavefront of the workgroup, or (two roles)
  // the one that runs them
  auto quad_sync = [&]() {
    if constexpr (ROLE < 0) __syncthreads();
    else wave_sync();
  };
  int qb = 0, cnt = 0, ls = 0, n = 0;
  bool live = false;
  int q = 0;
  if constexpr (MAP == MAP_DENSE) {
    qb = blockIdx.x * BS;
    cnt = min(BS, p.Q - qb);
    ls = (tid / N) * N;
    n = N;
    live = tid < cnt;
    q = qb + (live ? tid : 0);
  } else if constexpr (MAP == MAP_TABLE) {
    const int2 bq = p.blk[blockIdx.x];
    qb = bq.x;
    cnt = bq.y;
    live = tid < cnt;
    q = qb + (live ? tid : 0);
    const uint32_t swd = live ? p.sw[q] : 0u;
    ls = (int)(swd >> 8);
    n = (int)(swd & 0xffu);
  } else {
    const int4 it = p.items[item];  // (slot size, first env entry, swarms, -)
    const int k = tid / N, r = tid - (tid / N) * N;
    ls = k * N;
    if (k < it.z) {
      const int2 e = p.item_envs[it.y + k];  // (first quad, size)
      n = e.y;
      if (r < n) {
        live = true;
        q = e.x + r;
      }
    }
  }
  const int me = tid - ls;  // index within the swarm
  const int Qp = p.Qp;
  const float* __restrict__ S = p.st;
  // field f of quad q: a uniform field base plus the quad's 32-bit byte
  // offset (one address add per access instead of an index multiply,
  // sign extension and shift)
  const uint32_t qo = 4u * (uint32_t)q;
  auto at = [&](const float* base, int f) -> const float& {
    return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base + (size_t)f * Qp) + qo);
  };

  Quad s;
  s.ev = 0u;
  QuadPar pp;
  float uhat[4] = {0.f, 0.f, 0.f, 0.f};
  float f0[4] = {0.f, 0.f, 0.f, 0.f};  // rotor thrusts before the call (reward)
  float4 a4 = make_float4(0.f, 0.f, 0.f, 0.f);  // the call's action
  // the goal is loaded with the state: a load issued after the state stores
  // would wait for their completion (one in-order counter for both)
  float g0 = 0.f, g1 = 0.f, g2 = 0.f;
  if (OBS && ROLE != 0 && live) {
    g0 = goals[3 * q];
    g1 = goals[3 * q + 1];
    g2 = goals[3 * q + 2];
  }
  if (live) {
    if constexpr (ROLE != 0) {
#pragma unroll
      for (int k = 0; k < 3; ++k) s.x[k] = at(S, S_X + k);
#pragma unroll
      for (int k = 0; k < 3; ++k) s.v[k] = at(S, S_V + k);
#pragma unroll
      for (int k = 0; k < 9; ++k) s.R[k] = at(S, S_R + k);
#pragma unroll
      for (int k = 0; k < 3; ++k) s.w[k] = at(S, S_W + k);
    }
    if (nsub > 0) {
      if constexpr (ROLE != 1) {
#pragma unroll
        for (int k = 0; k < 4; ++k) s.u[k] = at(S, S_U + k);
#pragma unroll
        for (int k = 0; k < 4; ++k) s.e[k] = at(S, S_E + k);
      }
      if constexpr (ROLE != 0) s.fl = at(S, S_F);
      pp.m = at(p.par, P_M);
      pp.jx = at(p.par, P_JX);
      pp.jy = at(p.par, P_JY);
      pp.jz = at(p.par, P_JZ);
      pp.f_max = at(p.par, P_FMAX);
      pp.a_lag = at(p.par, P_ALAG);
    }
  }
  // the call's action, loaded by every lane without a branch (an idle lane's
  // q is still a valid quad: its workgroup's first, or quad 0 in the bucketed
  // launch; a call without substeps reads a row of the state instead), so no
  // merge of its value has to wait for it
  if constexpr (ROLE != 1)
    a4 = reinterpret_cast<const float4*>(nsub > 0 ? act : p.st)[q];
  // §III-A.2 motor noise: the draws depend on the quad, the substep index and
  // the seed only.  With the index known at launch, the first substep's are
  // drawn here, between issuing the loads above and using what they return.
  const bool noise = (c.flags & F_NOISE) != 0;
  const bool early_z = ROLE != 1 && tdev == nullptr && nsub > 0 && noise;
  float z0[4] = {0.f, 0.f, 0.f, 0.f};
  if (early_z && live) normal4(c, (uint32_t)q, t0, STREAM_MOTOR, 0, z0);
  if (live && nsub > 0) {
    pp.inv_m = 1.0f / pp.m;
    pp.ijx = 1.0f / pp.jx;
    pp.ijy = 1.0f / pp.jy;
    pp.ijz = 1.0f / pp.jz;
    pp.a_ns = c.ns_scale * pp.f_max;
    if constexpr (ROLE != 1) {
      if (reward) {
#pragma unroll
        for (int i = 0; i < 4; ++i) f0[i] = fmaf(pp.f_max * s.u[i], s.u[i], s.e[i]);
      }
      const bool unit = (c.flags & F_ACT_UNIT) != 0;
      uhat[0] = rotor_cmd(a4.x, unit);
      uhat[1] = rotor_cmd(a4.y, unit);
      uhat[2] = rotor_cmd(a4.z, unit);
      uhat[3] = rotor_cmd(a4.w, unit);
      if (!(isfinite(a4.x) && isfinite(a4.y) && isfinite(a4.z) && isfinite(a4.w)))
        __hip_atomic_fetch_or(p.err, ERRBIT_ACTION, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  // graph mode: the substep index comes from the device counter (read after
  // the state loads are in flight)
  if (tdev) t0 = read_counter(tdev);

  const bool collide = N != 1 && (c.flags & (F_COLLIDE | F_DOWNWASH)) != 0;
  unsigned long long cmask = 0ull;
  // Swarms of 16 and more (dense mapping): the last substep's partner screen
  // also builds the neighbour key list, from the same squared distances
  // (the pair pass moves no position), so the observation need not go over
  // the swarm again.  Without the screen (no pair pass, or downwash on) the
  // observation builds the list itself.
  constexpr bool SCREEN_KEYS = OBS && KT > 0 && MAP == MAP_DENSE && NU >= 16 && ROLE < 0;
  static_assert(!SCREEN_KEYS || N > 8, "swarms of up to 8 use cross-lane candidates");
  constexpr int NKEY = KT > 0 ? KT + 1 : 1;
  uint32_t skey[NKEY];
#pragma unroll
  for (int k = 0; k < NKEY; ++k) skey[k] = KEY_EMPTY;
  for (int sub = 0; sub < nsub; ++sub) {
    const unsigned long long t = t0 + (unsigned long long)sub;
    // this substep's motor-noise draws
    float zs[4] = {z0[0], z0[1], z0[2], z0[3]};
    if constexpr (ROLE != 1) {
      if (noise && live && !(sub == 0 && early_z)) normal4(c, (uint32_t)q, t, STREAM_MOTOR, 0, zs);
    }
    if constexpr (ROLE == 0) {
      if (live) {
        float z[4] = {0.f, 0.f, 0.f, 0.f};
        const Drive d = motor_step<Z_IMPORT>(c, pp, s.u, s.e, uhat, (uint32_t)q, t, z, zs);
        ring[sub & 1][0][tid] = d.T;
        ring[sub & 1][1][tid] = d.tx;
        ring[sub & 1][2][tid] = d.ty;
        ring[sub & 1][3][tid] = d.tz;
      }
      wg_sync();
      continue;
    }
    if constexpr (ROLE == 1) {
      wg_sync();
      if (live) {
        Drive d;
        d.T = ring[sub & 1][0][tid];
        d.tx = ring[sub & 1][1][tid];
        d.ty = ring[sub & 1][2][tid];
        d.tz = ring[sub & 1][3][tid];
        body_step(c, pp, s, d, (uint32_t)q, t);
      }
    } else {
      if (live) quad_substep<false, Z_IMPORT>(c, pp, s, uhat, (uint32_t)q, t, nullptr, zs);
    }
    if (collide) {
      // §III-B.1 in-env pair pass (Jacobi: every response from the
      // pre-response velocities of this substep)
      float(*tile)[BS] = sxv[sub & 1];
      if (live) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          tile[k][tid] = s.xo[k];
          tile[3 + k][tid] = s.inc[k];
          tile[6 + k][tid] = s.v[k];
        }
        put_screen_rows<kScreenSq<NU>>(tile, tid, s.x);
      } else if constexpr (MAP == MAP_ITEM) {
        // padding lane: far away, so it is never in contact
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          tile[k][tid] = 1e30f;
          tile[3 + k][tid] = 0.f;
          tile[6 + k][tid] = 0.f;
        }
        put_screen_pad<kScreenSq<NU>>(tile, tid);
      }
      quad_sync();
      cmask = 0ull;
      if (live) {
        float unused = 0.f;
        if constexpr (SCREEN_KEYS) {
          if (sub == nsub - 1)
            cmask = pair_pass<BS, NU, false, true, KT + 1>(c, tile, s, ls, n, me, (uint32_t)q, t,
                                                            unused, 0.f, skey);
          else
            cmask = pair_pass<BS, NU, false, true>(c, tile, s, ls, n, me, (uint32_t)q, t, unused,
                                                   0.f);
        } else {
          cmask = pair_pass<BS, NU, false, true>(c, tile, s, ls, n, me, (uint32_t)q, t, unused,
                                                 0.f);
        }
      }
    }
  }

  // Every load of the call has been consumed once a substep has run; the
  // explicit wait says so to the compiler, whose conservative merge with the
  // no-substep path would otherwise make the observation wait for the state
  // stores (loads and stores share one in-order counter).
  __builtin_amdgcn_s_waitcnt(0);
  if (live && nsub > 0) {
    float* St = p.st;
    auto to = [&](int f) -> float& {
      return *reinterpret_cast<float*>(reinterpret_cast<char*>(St + (size_t)f * Qp) + qo);
    };
    float chk = 0.f;
    if constexpr (ROLE != 0) {
#pragma unroll
      for (int k = 0; k < 3; ++k) { to(S_X + k) = s.x[k]; chk += s.x[k]; }
#pragma unroll
      for (int k = 0; k < 3; ++k) { to(S_V + k) = s.v[k]; chk += s.v[k]; }
#pragma unroll
      for (int k = 0; k < 9; ++k) { to(S_R + k) = s.R[k]; chk += s.R[k]; }
#pragma unroll
      for (int k = 0; k < 3; ++k) { to(S_W + k) = s.w[k]; chk += s.w[k]; }
    }
    if constexpr (ROLE != 1) {
#pragma unroll
      for (int k = 0; k < 4; ++k) { to(S_U + k) = s.u[k]; chk += s.u[k]; }
#pragma unroll
      for (int k = 0; k < 4; ++k) { to(S_E + k) = s.e[k]; chk += s.e[k]; }
    }
    if constexpr (ROLE != 0) to(S_F) = s.fl;
    if (!isfinite(chk))
      __hip_atomic_fetch_or(p.err, ERRBIT_STATE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (ROLE != 0 && p.contacts) p.contacts[q] = cmask;
  }
  // two roles: the motor wavefront hands the rotor state (start and end of
  // the call) over for the reward, and is done
  if constexpr (ROLE == 0) {
    if (OBS && reward) {
      if (live) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          rx[i][tid] = f0[i];
          rx[4 + i][tid] = s.u[i];
          rx[8 + i][tid] = s.e[i];
        }
      }
      wg_sync();
    }
    return;
  }
  if constexpr (ROLE == 1) {
    if (OBS && reward) {
      wg_sync();
      if (live) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          f0[i] = rx[i][tid];
          s.u[i] = rx[4 + i][tid];
          s.e[i] = rx[8 + i][tid];
        }
      }
    }
  }

  if constexpr (OBS) {
    // §III-C observation from the post-collision state
    float(*tile)[BS] = sxv[nsub & 1];
    // swarms of 2 to 8 (aligned lane groups of the wavefront) take the
    // candidates' positions from their lanes by cross-lane moves; the tile
    // then serves the selected slots' rows only
    constexpr bool LANE_KNN = KT > 0 && N > 1 && N <= 8;
    if constexpr (KT != 0) {  // the neighbour slots come from the tile
      if (live) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          tile[k][tid] = s.x[k];
          tile[6 + k][tid] = s.v[k];
        }
      } else if constexpr (MAP == MAP_ITEM) {
        // padding lane: never among the nearest
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          tile[k][tid] = 1e30f;
          tile[6 + k][tid] = 0.f;
        }
      }
      if constexpr (!LANE_KNN) quad_sync();
    }
    if constexpr (KT >= 0) {
      constexpr int OD = 18 + 6 * KT;
      float ov[OD];
      ov[0] = s.x[0] - g0;
      ov[1] = s.x[1] - g1;
      ov[2] = s.x[2] - g2;
#pragma unroll
      for (int k = 0; k < 3; ++k) ov[3 + k] = s.v[k];
#pragma unroll
      for (int k = 0; k < 9; ++k) ov[6 + k] = s.R[k];
#pragma unroll
      for (int k = 0; k < 3; ++k) ov[15 + k] = s.w[k];
      if constexpr (KT > 0) {
        // The KT nearest by (d^2, index): a sorted list of KT + 1 keys
        // (knn_insert).  Keys order as (d^2 truncated to 2^-17 relative,
        // index): the list is the exact (d^2, index) order unless two
        // neighbouring entries share a truncated distance (an exact or near
        // tie); such a lane selects again with exact comparisons below.
        constexpr uint32_t EMPTY = KEY_EMPTY;
        uint32_t key[KT + 1];
        bool screened = false;  // the list came with the last pair pass
        if constexpr (SCREEN_KEYS) screened = collide && nsub > 0 && !(c.flags & F_DOWNWASH);
#pragma unroll
        for (int k = 0; k <= KT; ++k) key[k] = SCREEN_KEYS ? skey[k] : EMPTY;
        auto cand = [&](int jj, float xj, float yj, float zj) {
          const float pj[3] = {xj, yj, zj};
          knn_insert<KT + 1>(key, jj, me, sq_dist(pj, s.x));
        };
        if (!screened) {
          if constexpr (LANE_KNN) {
            const float mx = live ? s.x[0] : 1e30f, my = live ? s.x[1] : 1e30f,
                        mz = live ? s.x[2] : 1e30f;
            auto mate = [&](auto dc) {
              constexpr int D = decltype(dc)::value;
              if constexpr (D < N)
                cand(me ^ D, lane_xor8<D>(mx, 1e30f), lane_xor8<D>(my, 1e30f),
                     lane_xor8<D>(mz, 1e30f));
            };
            mate(std::integral_constant<int, 1>{});
            mate(std::integral_constant<int, 2>{});
            mate(std::integral_constant<int, 3>{});
            mate(std::integral_constant<int, 4>{});
            mate(std::integral_constant<int, 5>{});
            mate(std::integral_constant<int, 6>{});
            mate(std::integral_constant<int, 7>{});
            quad_sync();  // the tile rows, for the selected slots below
          } else if constexpr (NU > 1) {
            constexpr int CH = NU < 8 ? NU : 8;
            auto chunk = [&](int j0) {
              float px[CH][3];
#pragma unroll
              for (int u = 0; u < CH; ++u)
#pragma unroll
                for (int r = 0; r < 3; ++r) px[u][r] = tile[r][ls + j0 + u];
#pragma unroll
              for (int u = 0; u < CH; ++u) cand(j0 + u, px[u][0], px[u][1], px[u][2]);
            };
            if constexpr (NU >= 16) {
#pragma unroll 1
              for (int j0 = 0; j0 < NU; j0 += CH) chunk(j0);
            } else {
#pragma unroll
              for (int j0 = 0; j0 < NU; j0 += CH) chunk(j0);
            }
          } else if constexpr (NU == 0) {
            if (live)
              for (int jj = 0; jj < n; ++jj)
                cand(jj, tile[0][ls + jj], tile[1][ls + jj], tile[2][ls + jj]);
          }
        }
        bool tie = false;
#pragma unroll
        for (int k = 0; k < KT; ++k) tie |= key[k + 1] != EMPTY && (key[k] >> 6) == (key[k + 1] >> 6);
        if (tie && live) {
          // exact (d^2, index) insertion over the swarm (rare)
          float bd[KT];
          int bj[KT];
#pragma unroll
          for (int k = 0; k < KT; ++k) { bd[k] = INFINITY; bj[k] = -1; }
          for (int jj = 0; jj < n; ++jj) {
            const float rx = tile[0][ls + jj] - s.x[0], ry = tile[1][ls + jj] - s.x[1],
                        rz = tile[2][ls + jj] - s.x[2];
            const float d2 = jj == me ? INFINITY : rx * rx + ry * ry + rz * rz;
#pragma unroll
            for (int k = KT - 1; k > 0; --k) {
              const bool shift = bd[k - 1] > d2;
              const bool here = bd[k] > d2;
              bd[k] = shift ? bd[k - 1] : (here ? d2 : bd[k]);
              bj[k] = shift ? bj[k - 1] : (here ? jj : bj[k]);
            }
            if (bd[0] > d2) { bd[0] = d2; bj[0] = jj; }
          }
#pragma unroll
          for (int k = 0; k < KT; ++k) key[k] = bj[k] >= 0 ? (uint32_t)bj[k] : EMPTY;
        }
        int bj[KT];
#pragma unroll
        for (int k = 0; k < KT; ++k) bj[k] = key[k] != EMPTY ? (int)(key[k] & 63u) : -1;
        // the slots' rows are read unconditionally (j is always a valid
        // column) and selected afterwards, so all reads are in flight at
        // once instead of one guarded read and wait per value
        float nb[KT][6];
#pragma unroll
        for (int k = 0; k < KT; ++k) {
          const int j = ls + (bj[k] >= 0 ? bj[k] : 0);
          nb[k][0] = tile[0][j];
          nb[k][1] = tile[1][j];
          nb[k][2] = tile[2][j];
          nb[k][3] = tile[6][j];
          nb[k][4] = tile[7][j];
          nb[k][5] = tile[8][j];
        }
#pragma unroll
        for (int k = 0; k < KT; ++k) {
          const bool have = bj[k] >= 0;
          ov[18 + 6 * k + 0] = have ? nb[k][0] - s.x[0] : 0.f;
          ov[18 + 6 * k + 1] = have ? nb[k][1] - s.x[1] : 0.f;
          ov[18 + 6 * k + 2] = have ? nb[k][2] - s.x[2] : 0.f;
          ov[18 + 6 * k + 3] = have ? nb[k][3] - s.v[0] : 0.f;
          ov[18 + 6 * k + 4] = have ? nb[k][4] - s.v[1] : 0.f;
          ov[18 + 6 * k + 5] = have ? nb[k][5] - s.v[2] : 0.f;
        }
        if (reward && live) {
          float rp = 0.f;
#pragma unroll
          for (int k = 0; k < KT; ++k)
            if (bj[k] >= 0) rp += reward_prox(c, ov[18 + 6 * k], ov[19 + 6 * k], ov[20 + 6 * k]);
          reward[q] = reward_state(c, s, pp.f_max, ov, f0) + rp;
        }
      } else {
        if (reward && live) reward[q] = reward_state(c, s, pp.f_max, ov, f0);
      }
      if (c.flags & F_SENSOR) sensor_noise(c, (uint32_t)q, t0 + nsub, &ov[0], &ov[3], &ov[15]);
      if (stage_obs) {
        // the workgroup's rows leave through LDS in passes of stage_obs
        // rows, each copied out with contiguous stores: 16-byte stores when
        // the destination allows, else 8-byte stores; non-temporal, since
        // the rows go to their consumer and this kernel never reads them
        // back (fewer dirty L2 lines left to write back when the kernel
        // ends).  A small staging area (a few KiB) keeps LDS from limiting
        // how many workgroups share a CU.
        const int R = stage_obs;
        if constexpr (MAP == MAP_ITEM) {
          // an item's swarms are separate runs of rows: a pass (whole
          // swarms, R being a multiple of the slot size) leaves swarm by
          // swarm, each run with contiguous 8-byte stores
          const int4 itm = p.items[item];
          for (int p0 = 0; p0 < itm.z * N; p0 += R) {
            if (live && tid >= p0 && tid < p0 + R) {
              float2* r2 = reinterpret_cast<float2*>(st_obs + (tid - p0) * OD);
#pragma unroll
              for (int k = 0; k < OD / 2; ++k) r2[k] = make_float2(ov[2 * k], ov[2 * k + 1]);
            }
            quad_sync();
            const int k1 = min((p0 + R) / N, itm.z);
            for (int k = p0 / N; k < k1; ++k) {
              const int2 e = p.item_envs[itm.y + k];
              const int n2 = e.y * OD / 2;
              v2f* d2p = reinterpret_cast<v2f*>(obs + (size_t)e.x * OD);
              const v2f* s2p = reinterpret_cast<const v2f*>(st_obs + (k * N - p0) * OD);
              for (int i = tid; i < n2; i += BS) __builtin_nontemporal_store(s2p[i], d2p + i);
            }
            if (p0 + R < itm.z * N) quad_sync();
          }
        } else
        for (int p0 = 0; p0 < cnt; p0 += R) {
          if (live && tid >= p0 && tid < p0 + R) {
            float2* r2 = reinterpret_cast<float2*>(st_obs + (tid - p0) * OD);
#pragma unroll
            for (int k = 0; k < OD / 2; ++k) r2[k] = make_float2(ov[2 * k], ov[2 * k + 1]);
          }
          quad_sync();
          const int total = min(R, cnt - p0) * OD;
          float* dst = obs + (size_t)(qb + p0) * OD;
          if ((reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
            const int n4 = total >> 2;
            v4f* d4 = reinterpret_cast<v4f*>(dst);
            const v4f* s4 = reinterpret_cast<const v4f*>(st_obs4);
#pragma unroll 4
            for (int i = tid; i < n4; i += BS) __builtin_nontemporal_store(s4[i], d4 + i);
            if ((total & 3) && tid == 0)
              __builtin_nontemporal_store(reinterpret_cast<const v2f*>(st_obs)[2 * n4],
                                          reinterpret_cast<v2f*>(dst) + 2 * n4);
          } else {
            const int n2 = total >> 1;
            v2f* d2p = reinterpret_cast<v2f*>(dst);
            const v2f* s2p = reinterpret_cast<const v2f*>(st_obs);
#pragma unroll 4
            for (int i = tid; i < n2; i += BS) __builtin_nontemporal_store(s2p[i], d2p + i);
          }
          // the copy has read this pass's rows before the next pass writes
          if (p0 + R < cnt) quad_sync();
        }
      } else if (live) {
        float2* r2 = reinterpret_cast<float2*>(obs + (size_t)q * OD);
#pragma unroll
        for (int k = 0; k < OD / 2; ++k) r2[k] = make_float2(ov[2 * k], ov[2 * k + 1]);
      }
    } else {
      // runtime K (rare sizes): K passes of selection of the next
      // (d^2, index) pair; each lane writes its own row
      const int K = c.K, OD = c.obs_dim;
      if (live) {
        float* row = obs + (size_t)q * OD;
        float ox[3] = {s.x[0] - g0, s.x[1] - g1, s.x[2] - g2};
        float ovl[3] = {s.v[0], s.v[1], s.v[2]}, ow[3] = {s.w[0], s.w[1], s.w[2]};
        float rwd = reward ? reward_state(c, s, pp.f_max, ox, f0) : 0.f;
        if (c.flags & F_SENSOR) sensor_noise(c, (uint32_t)q, t0 + nsub, ox, ovl, ow);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          row[k] = ox[k];
          row[3 + k] = ovl[k];
          row[15 + k] = ow[k];
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) row[6 + k] = s.R[k];
        float pd = -1.0f;
        int pj = -1;
        for (int k = 0; k < K; ++k) {
          float bd = INFINITY;
          int bj = -1;
          for (int jj = 0; jj < n; ++jj) {
            if (jj == me) continue;
            const int j = ls + jj;
            const float rx = tile[0][j] - s.x[0], ry = tile[1][j] - s.x[1], rz = tile[2][j] - s.x[2];
            const float d2 = rx * rx + ry * ry + rz * rz;
            const bool after = d2 > pd || (d2 == pd && jj > pj);
            const bool better = d2 < bd || (d2 == bd && jj < bj);
            if (after && better) { bd = d2; bj = jj; }
          }
          float* o = row + 18 + 6 * k;
          if (bj >= 0) {
            const int j = ls + bj;
            o[0] = tile[0][j] - s.x[0];
            o[1] = tile[1][j] - s.x[1];
            o[2] = tile[2][j] - s.x[2];
            o[3] = tile[6][j] - s.v[0];
            o[4] = tile[7][j] - s.v[1];
            o[5] = tile[8][j] - s.v[2];
            if (reward) rwd += reward_prox(c, o[0], o[1], o[2]);
            pd = bd;
            pj = bj;
          } else {
            for (int m = 0; m < 6; ++m) o[m] = 0.f;
            pd = INFINITY;
            pj = 1 << 30;
          }
        }
        if (reward) reward[q] = rwd;
      }
    }
  }
}

// Kernel arguments: the leading ones (state, parameters, actions, goals,
// constants, sizes) are what the dense mapping needs before its first load
// and fit the fourteen SGPRs the hardware can preload where the firmware
// supports it; the constants live in device memory written at creation.

// One workgroup per block of quads (dense or table mapping).  Held to 128
// VGPRs (four wavefronts per SIMD): the neighbour keys that swarms of 16 and
// more carry through the last pair pass would otherwise take the allocation
// to 134 and the occupancy to three.
template <int BS, int KT, int N>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(4))) void step_kernel(
    float* __restrict__ st, const float* __restrict__ par, const float* __restrict__ act,
    const float* __restrict__ goals, const Consts* __restrict__ cp, int Qp, int Q, int nsub,
    unsigned long long t0, Ptrs p, float* __restrict__ obs, int stage_obs,
    unsigned long long* tdev, unsigned int* done, float* __restrict__ reward) {
  __shared__ float sxv[2][TILE_ROWS_CO][BS];
  extern __shared__ float4 st_obs4[];
  p.st = st;
  p.par = par;
  p.Qp = Qp;
  p.Q = Q;
  const Consts& c = *cp;
  constexpr int MAP = (N > 0) ? MAP_DENSE : MAP_TABLE;
  step_body<BS, KT, N, MAP>(c, p, act, nsub, t0, goals, obs, stage_obs, sxv,
                            reinterpret_cast<float*>(st_obs4), 0, reward, tdev);
  if (tdev) advance_counter(tdev, done, nsub, gridDim.x);
}

// Several substeps per call for small batches of swarms of 8: two
// wavefronts per workgroup of 64 quads, the motor part of each substep one
// substep ahead of the rest (step_body ROLE 0 and 1).  Same arithmetic in
// the same order as step_kernel, so identical results.
template <int KT, int N>
__global__ __launch_bounds__(128) void step_pipe_kernel(float* __restrict__ st,
                                                        const float* __restrict__ par,
                                                        const float* __restrict__ act,
                                                        const float* __restrict__ goals,
                                                        const Consts* __restrict__ cp, int Qp,
                                                        int Q, int nsub, unsigned long long t0,
                                                        Ptrs p, float* __restrict__ obs,
                                                        int stage_obs, unsigned long long* tdev,
                                                        unsigned int* done,
                                                        float* __restrict__ reward) {
  constexpr int BS = 64;
  __shared__ float sxv[2][TILE_ROWS_CO][BS];
  __shared__ float ring[2][4][BS];
  __shared__ float rx[12][BS];
  extern __shared__ float4 st_obs4[];
  p.st = st;
  p.par = par;
  p.Qp = Qp;
  p.Q = Q;
  const Consts& c = *cp;
  const int role = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  if (role == 0)
    step_body<BS, KT, N, MAP_DENSE, N, 0>(c, p, act, nsub, t0, goals, obs, stage_obs, sxv,
                                          reinterpret_cast<float*>(st_obs4), 0, reward, tdev,
                                          ring, rx);
  else
    step_body<BS, KT, N, MAP_DENSE, N, 1>(c, p, act, nsub, t0, goals, obs, stage_obs, sxv,
                                          reinterpret_cast<float*>(st_obs4), 0, reward, tdev,
                                          ring, rx);
  if (tdev) advance_counter(tdev, done, nsub, gridDim.x);
}

// Observation rows per staging pass of the bucketed kernel (slots of 4 to
// 32 quads, whose swarms are runs of several rows: per-lane row stores
// measured 7 % slower on the one-substep uneven launch, 5.09 -> 5.48 G
// quad-steps/s staged; slots of 1 and 2 would copy one short run per swarm
// and keep per-lane stores).
constexpr int BUCKET_STAGE_ROWS = 32;

// Persistent launch over the work items [item0, item0 + n_items) of uneven
// swarm sizes; workgroups stride over them and run the body specialised for
// each item's slot size N.  Slots of 4 and more loop over the swarm at run
// time, one partner at a time, in the pair pass (and slots of 16 and 32 in
// the neighbour search as well): unrolled, their bodies would set the whole
// kernel's register count, and with it the occupancy (135 VGPRs instead of
// 381: 3 wavefronts per SIMD instead of 1).  Slots of 16 and 32 also have a
// body that takes the partners in chunks of four (their loads in flight
// together), chosen per item (items[it].w, set per slot size by the
// autotuner); with both bodies the kernel stays at 3 wavefronts per SIMD.
template <int BS, int KT>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(3))) void bucket_kernel(
                                                    float* __restrict__ st,
                                                    const float* __restrict__ par,
                                                    const float* __restrict__ act,
                                                    const float* __restrict__ goals,
                                                    const Consts* __restrict__ cp, int Qp, int Q,
                                                    int nsub, unsigned long long t0, Ptrs p,
                                                    float* __restrict__ obs, int item0,
                                                    int n_items, unsigned long long* tdev,
                                                    unsigned int* done,
                                                    float* __restrict__ reward) {
  __shared__ float sxv[2][TILE_ROWS_CO][BS];
  extern __shared__ float4 st_obs4[];
  float* so = reinterpret_cast<float*>(st_obs4);
  // slots of 4 to 32 stage their observation rows, 32 rows a pass
  constexpr int SR = KT >= 0 ? BUCKET_STAGE_ROWS : 0;
  p.st = st;
  p.par = par;
  p.Qp = Qp;
  p.Q = Q;
  const Consts& c = *cp;
  for (int it = item0 + blockIdx.x; it < item0 + n_items; it += gridDim.x) {
    __syncthreads();  // the previous item's readers of the tile are done
    const int4 item = p.items[it];
    const bool chunked = item.w != 0;
    switch (item.x) {
      case 1: step_body<BS, KT, 1, MAP_ITEM>(c, p, act, nsub, t0, goals, obs, 0, sxv, nullptr, it, reward, tdev); break;
      case 2: step_body<BS, KT, 2, MAP_ITEM>(c, p, act, nsub, t0, goals, obs, 0, sxv, nullptr, it, reward, tdev); break;
      case 4: step_body<BS, KT, 4, MAP_ITEM, 0>(c, p, act, nsub, t0, goals, obs, SR, sxv, so, it, reward, tdev); break;
      case 8: step_body<BS, KT, 8, MAP_ITEM, 0>(c, p, act, nsub, t0, goals, obs, SR, sxv, so, it, reward, tdev); break;
      case 16:
        if (chunked) step_body<BS, KT, 16, MAP_ITEM>(c, p, act, nsub, t0, goals, obs, SR, sxv, so, it, reward, tdev);
        else step_body<BS, KT, 16, MAP_ITEM, 0>(c, p, act, nsub, t0, goals, obs, SR, sxv, so, it, reward, tdev);
        break;
      case 32:
        if (chunked) step_body<BS, KT, 32, MAP_ITEM>(c, p, act, nsub, t0, goals, obs, SR, sxv, so, it, reward, tdev);
        else step_body<BS, KT, 32, MAP_ITEM, 0>(c, p, act, nsub, t0, goals, obs, SR, sxv, so, it, reward, tdev);
        break;
      default: step_body<BS, KT, 64, MAP_ITEM, 0>(c, p, act, nsub, t0, goals, obs, 0, sxv, nullptr, it, reward, tdev); break;
    }
  }
  if (tdev) advance_counter(tdev, done, nsub, gridDim.x);
}

// Set the graph-mode counter and clear the completion counts (one
// workgroup of 64 threads).
__global__ void set_counter_kernel(unsigned long long* tdev, unsigned int* done,
                                   unsigned long long v) {
  if (blockIdx.x != 0) return;
  if (threadIdx.x == 0) __hip_atomic_exchange(tdev, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (int i = threadIdx.x; i <= DONE_SUBS; i += blockDim.x)
    __hip_atomic_exchange(done + DONE_STRIDE * i, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Per-quad parameters [Q][6] (mass, ixx, iyy, izz, thrust-to-weight, tau_m)
// -> private SoA, for environments selected by env_mask, with f_max and
// alpha_lag derived in double and rounded once (as at creation).  A row
// with a non-finite or non-positive entry is left as it was and raises the
// sticky parameter error bit.
__global__ void set_params_kernel(float* __restrict__ par, int Qp, int Q,
                                  const float* __restrict__ src,
                                  const int32_t* __restrict__ qenv,
                                  const uint8_t* __restrict__ env_mask, float dt, float g,
                                  int* err) {
  const int q = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (q >= Q) return;
  if (env_mask && env_mask[qenv[q]] == 0) return;
  float v[6];
  bool ok = true;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    v[k] = src[(size_t)q * 6 + k];
    ok = ok && isfinite(v[k]) && v[k] > 0.0f;
  }
  if (!ok) {
    __hip_atomic_fetch_or(err, ERRBIT_PARAM, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  par[(size_t)P_M * Qp + q] = v[0];
  par[(size_t)P_JX * Qp + q] = v[1];
  par[(size_t)P_JY * Qp + q] = v[2];
  par[(size_t)P_JZ * Qp + q] = v[3];
  par[(size_t)P_FMAX * Qp + q] = (float)(0.25 * (double)v[0] * (double)g * (double)v[4]);
  par[(size_t)P_ALAG * Qp + q] = (float)(1.0 - exp(-(double)dt / (double)v[5]));
  par[(size_t)P_T2W * Qp + q] = v[4];
  par[(size_t)P_TAU * Qp + q] = v[5];
}

// The library's counter-based generator, exported for tests: for quads
// quad0 .. quad0 + n - 1 at substep t, the four Philox4x32-10 words of
// (stream, draw) into words[n][4] and, when normals is not null, the four
// N(0,1) draws built from them into normals[n][4].
__global__ void philox_debug_kernel(uint32_t key0, uint32_t key1, uint32_t stream,
                                    uint32_t draw, unsigned long long t, uint32_t quad0, int n,
                                    uint32_t* __restrict__ words, float* __restrict__ normals) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= n) return;
  const uint32_t q = quad0 + (uint32_t)i;
  uint32_t r0 = q, r1 = (uint32_t)t, r2 = (uint32_t)(t >> 32), r3 = (stream << 8) | draw;
  philox4x32_10(r0, r1, r2, r3, key0, key1);
  words[4 * (size_t)i + 0] = r0;
  words[4 * (size_t)i + 1] = r1;
  words[4 * (size_t)i + 2] = r2;
  words[4 * (size_t)i + 3] = r3;
  if (normals) {
    Consts c{};
    c.key0 = key0;
    c.key1 = key1;
    float z[4];
    normal4(c, q, t, stream, draw, z);
#pragma unroll
    for (int k = 0; k < 4; ++k) normals[4 * (size_t)i + k] = z[k];
  }
}

// Canonical [Q][27] -> private SoA, for environments selected by env_mask.
__global__ void set_state_kernel(float* __restrict__ st, int Qp, int Q,
                                 const float* __restrict__ src,
                                 const int32_t* __restrict__ qenv,
                                 const uint8_t* __restrict__ env_mask) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)Q * NSTATE) return;
  const int q = (int)(i / NSTATE), f = (int)(i - (long long)q * NSTATE);
  if (env_mask && env_mask[qenv[q]] == 0) return;
  st[(size_t)f * Qp + q] = src[i];
}

// Private SoA -> canonical [Q][27].
__global__ void get_state_kernel(const float* __restrict__ st, int Qp, int Q,
                                 float* __restrict__ dst) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)Q * NSTATE) return;
  const int q = (int)(i / NSTATE), f = (int)(i - (long long)q * NSTATE);
  dst[i] = st[(size_t)f * Qp + q];
}

}  // namespace qs
